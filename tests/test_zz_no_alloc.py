"""The no-allocation inference entry point (adc_mlp_forward_noalloc) against
the allocating one (adc_mlp_forward) and the FP64 oracle forward, on two
calls in a row (the second with fewer rows, so stale rows of the shared
static array must not leak into it), FP32 and BF16 hidden layer, plus its
size checks.  Tolerances as for the forward parity test: FP32 1e-4 and BF16
2e-2 of the output scale against the oracle; the two entry points run the
same kernels and may differ only by the tile choice of the hidden product
(sums in another order), 1e-5 (FP32) and 1e-2 (BF16) of the scale."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_noalloc_forward_matches_context_forward_and_oracle():
    import paper_2012_06714_amd as adc
    from oracle import mlp
    from synthetic import small_system
    eps, B = small_system(3, 7, 24, 2)
    ctx = adc.Context(torch.tensor(eps, device="cuda"), torch.tensor(B, device="cuda"), 3, 2, "ea")
    rng = np.random.default_rng(21)
    p = mlp.init_params(22)
    v = mlp.unpack(p)
    v["w3"][...] = rng.standard_normal(mlp.WIDTH) * 0.3
    v["b1"][...] = rng.standard_normal(mlp.WIDTH) * 0.1
    v["b2"][...] = rng.standard_normal(mlp.WIDTH) * 0.1
    p32 = p.astype(np.float32)
    pd = torch.tensor(p32, device="cuda")
    for n in (adc.MLP_NOALLOC_ROWS, 1234):
        _say(f"case no-alloc forward n={n}")
        F = rng.standard_normal((n, mlp.NF)).astype(np.float32)
        Fd = torch.tensor(F, device="cuda")
        y_ref, _ = mlp.forward(p32.astype(np.float64), F.astype(np.float64))
        scale = np.abs(y_ref).max()
        for bf16, tol_o, tol_c in ((False, 1e-4, 1e-5), (True, 2e-2, 1e-2)):
            y = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
            adc.mlp_forward_noalloc(pd, Fd, y, bf16=bf16)
            torch.cuda.synchronize()
            y_ctx = ctx.mlp_forward(pd, Fd, bf16=bf16).cpu().numpy()
            yn = y.cpu().numpy()
            assert np.isfinite(yn).all()
            assert np.abs(yn - y_ref).max() <= tol_o * scale
            assert np.abs(yn - y_ctx).max() <= tol_c * scale
    ctx.close()
    # sizes beyond the static array, and empty input, are refused before any launch
    y = torch.zeros(4, dtype=torch.float32, device="cuda")
    F = torch.zeros((4, mlp.NF), dtype=torch.float32, device="cuda")
    lib = adc.lib
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for bad in (0, adc.MLP_NOALLOC_ROWS + 1):
        rc = lib.adc_mlp_forward_noalloc(ctypes.c_void_p(pd.data_ptr()),
                                         ctypes.c_void_p(F.data_ptr()), bad, 0,
                                         ctypes.c_void_p(y.data_ptr()), st)
        assert rc == adc.ADC_E_ARG and "8192" in adc.last_error()
    assert lib.adc_mlp_forward_noalloc(None, ctypes.c_void_p(F.data_ptr()), 4, 0,
                                       ctypes.c_void_p(y.data_ptr()), st) == adc.ADC_E_ARG
