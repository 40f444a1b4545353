"""Every compiled matrix-core tile configuration, forced, against references
computed on the CPU.

* adc_gemm (the product under every contraction) for each storage/compute
  type and each of its configurations, on ragged shapes (M, N, K not
  multiples of any tile), all four transpose combinations, beta zero and not,
  row-major and permuted output maps: element by element against the FP64
  product of the same operands (BF16: the operands rounded to BF16 to nearest
  even first), within the accumulation bound (K + 2) u (|alpha| |A||B| +
  |beta| |C0|) of the type's sum precision u.
* sigma of EA-ADC(3) and IP-ADC(3) with each configuration forced on every
  product of the context, at each precision level, element by element against
  the oracle's sigma, scaled by the oracle's magnitude of the same sums
  (|coefficients| x |tensors| x |X|).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U_SUM = {0: 2.0 ** -53, 1: 2.0 ** -24, 2: 2.0 ** -24, 3: 2.0 ** -24}
NAMES = {0: "fp64", 1: "fp32", 2: "bf16(fp32 in)", 3: "bf16"}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _bf16_round(x):
    """float32 -> nearest-even BF16 values (as float32), in numpy."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _operand(rng, rows, cols, dtype):
    a = rng.standard_normal((rows, cols))
    if dtype == 0:
        return a, a
    a32 = a.astype(np.float32)
    if dtype == 1:
        return a32, a32.astype(np.float64)
    return a32, _bf16_round(a32).astype(np.float64)


def _dev(a, dtype):
    t = torch.tensor(a)
    if dtype == 3:
        return t.to(torch.bfloat16).cuda()   # torch rounds FP32 to BF16 to nearest even
    return t.cuda()


# K = 1000 and 40: rows of 16-byte aligned BF16 (K a multiple of 8), where the
# NT form of configuration 8 loads its operands straight into LDS; 1000 ends in
# a ragged k-tile, 40 has no full one
SHAPES = [(517, 389, 301), (300, 700, 1029), (64, 65, 7), (517, 389, 1000), (300, 260, 40)]


@pytest.mark.parametrize("dtype", [0, 1, 2, 3])
def test_gemm_every_config_ragged(dtype):
    import paper_2012_06714_amd as adc
    cfgs = adc.gemm_configs(dtype)
    assert 0 in cfgs and len(cfgs) >= 3
    rng = np.random.default_rng(100 + dtype)
    worst = 0.0
    for (M, N, K) in SHAPES:
        for ta in (0, 1):
            for tb in (0, 1):
                a_st, a_ref = _operand(rng, K if ta else M, M if ta else K, dtype)
                b_st, b_ref = _operand(rng, N if tb else K, K if tb else N, dtype)
                if dtype == 3:
                    # BF16 storage: the device rounds once when converting; the
                    # reference uses the same nearest-even rounding
                    a_ref = _bf16_round(a_st.astype(np.float32)).astype(np.float64)
                    b_ref = _bf16_round(b_st.astype(np.float32)).astype(np.float64)
                opA = a_ref.T if ta else a_ref
                opB = b_ref.T if tb else b_ref
                prod = opA @ opB
                mag = np.abs(opA) @ np.abs(opB)
                lda, ldb = a_st.shape[1], b_st.shape[1]
                for beta in (0.0, -0.75):
                    for mapped in (False, True):
                        cdt = np.float64 if dtype == 0 else np.float32
                        if mapped:
                            # rows m = (m1, m2) with m2 < 7, columns n = (n1, n2) with n2 < 5,
                            # stored as [n1][m2][m1][n2] (a permutation of a dense array)
                            rs, cs = 7, 5
                            nm1, nn1 = -(-M // rs), -(-N // cs)
                            omap = (rs, cs, nm1 * cs, cs, rs * nm1 * cs, 1)
                            size = nn1 * rs * nm1 * cs
                            m = np.arange(M)[:, None]
                            n = np.arange(N)[None, :]
                            off = (m // rs) * cs + (m % rs) * nm1 * cs + (n // cs) * rs * nm1 * cs + n % cs
                            assert off.max() < size and np.unique(off).size == M * N
                        else:
                            omap, size = None, M * N
                            off = np.arange(M)[:, None] * N + np.arange(N)[None, :]
                        c0 = rng.standard_normal(size).astype(cdt)
                        A = _dev(a_st, dtype)
                        B = _dev(b_st, dtype)
                        C = torch.tensor(c0).cuda()
                        for cfg in cfgs:
                            C.copy_(torch.tensor(c0))
                            adc.gemm(dtype, ta, tb, M, N, K, 1.25, A, lda, B, ldb, beta, C, N,
                                     omap=omap, config=cfg)
                            out = C.cpu().numpy().astype(np.float64)
                            got = out[off]
                            ref = 1.25 * prod + beta * c0.astype(np.float64)[off]
                            bound = (K + 2) * U_SUM[dtype] * (1.25 * mag + abs(beta) *
                                                             np.abs(c0.astype(np.float64)[off]))
                            err = np.abs(got - ref)
                            ratio = float((err / (bound + 1e-300)).max())
                            worst = max(worst, ratio)
                            # untouched entries of a mapped output keep their value
                            if mapped:
                                mask = np.ones(size, bool)
                                mask[off.ravel()] = False
                                assert np.array_equal(out[mask], c0.astype(np.float64)[mask])
                            assert ratio <= 1.0, (f"{NAMES[dtype]} cfg {cfg} {M}x{N}x{K} "
                                                  f"t{ta}{tb} beta {beta} map {mapped}: {ratio}")
    _say(f"gemm {NAMES[dtype]} configs {cfgs}: worst error / bound {worst:.3e}")


def _ctx(eps, B, O, order, kind):
    import paper_2012_06714_amd as adc
    return adc.Context(torch.tensor(eps, device="cuda"), torch.tensor(B, device="cuda"), O,
                       order, kind)


# per precision level: the bound on |sigma_gpu - sigma_oracle| / magnitude
# (measured: FP64 ~2e-17, BF16 products ~4e-5, FP32 products ~9e-9; a term
# lost at a tile edge would be of the order of its share of the magnitude)
LEVEL_TOL = {0: 1e-14, 1: 2e-3, 2: 1e-6}
LEVEL_TYPE = {0: 0, 1: 2, 2: 1}


@pytest.mark.parametrize("kind,O,V,Q", [("ea", 8, 96, 200), ("ip", 12, 40, 120)])
def test_sigma_every_config_vs_oracle(kind, O, V, Q):
    import paper_2012_06714_amd as adc
    from oracle.radc import RADC
    from synthetic import random_vectors, small_system
    eps, B = small_system(O, V, Q, 77)
    _say(f"case sigma tiles {kind} O={O} V={V} Q={Q}: oracle")
    ref = RADC(eps, B, O, 3, kind)
    X = random_vectors(ref.dim, 4, 78)
    s_ref = ref.sigma(X)
    mag = ref.sigma_magnitude(X)
    ctx = _ctx(eps, B, O, 3, kind)
    Xd = torch.tensor(X, device="cuda")
    for level in (0, 1, 2):
        ctx.set_option("precision", level)
        for cfg in adc.gemm_configs(LEVEL_TYPE[level]):
            ctx.set_option("gemm_config", cfg)
            s = ctx.sigma(Xd).cpu().numpy()
            ratio = float((np.abs(s - s_ref) / (mag + 1e-300)).max())
            _say(f"  {kind} level {level} config {cfg}: max |err| / magnitude {ratio:.3e}")
            assert np.isfinite(s).all()
            assert ratio <= LEVEL_TOL[level], (level, cfg, ratio)
    ctx.close()
