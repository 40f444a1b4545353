"""Python binding of the MI355X EA/IP-ADC(n) library (libadc.so).

Argument marshalling only: every step runs in the HIP library.  Device
arrays are torch CUDA (HIP) tensors; PyTorch provides memory and streams.
Importing this module loads the shared library and raises if it is missing:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libadc.so")

ADC_IP, ADC_EA = 0, 1
ADC_OK, ADC_E_ARG, ADC_E_OOM, ADC_E_HIP, ADC_E_STATE, ADC_E_NUMERIC, ADC_E_NOCONV = (
    0, -1, -2, -3, -4, -5, 1)

# every symbol declared in include/adc.h
ABI_SYMBOLS = ("adc_setup", "adc_set_option", "adc_set_stream", "adc_dim", "adc_diag",
               "adc_sigma", "adc_davidson", "adc_spec_factors", "adc_set_guess",
               "adc_last_error", "adc_destroy", "adc_last_stats", "adc_workspace", "adc_sigma_flops",
               "adc_sigma_timed", "adc_history", "adc_mlp_nparams", "adc_precond_mlp",
               "adc_mlp_status", "adc_mlp_pairs", "adc_mlp_forward", "adc_mlp_loss_grad",
               "adc_mlp_adam", "adc_record_count", "adc_record_get", "adc_graph_launches",
               "adc_batch_davidson", "adc_setup_batch", "adc_batch_set_option",
               "adc_davidson_batch", "adc_batch_context", "adc_batch_destroy", "adc_gemm",
               "adc_gemm_configs", "adc_mlp_forward_noalloc", "adc_set_setup_option",
               "adc_spectral_function", "adc_propagator_diag", "adc_setup_u")


class ADCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    sig = {
        "adc_setup": (i, [vp, vp, i, i, i, i, i, ctypes.POINTER(vp)]),
        "adc_setup_u": (i, [vp, vp, vp, vp, i, i, i, i, i, i, ctypes.POINTER(vp)]),
        "adc_set_option": (i, [vp, ctypes.c_char_p, d]),
        "adc_set_stream": (i, [vp, vp]),
        "adc_dim": (ll, [vp]),
        "adc_diag": (i, [vp, vp]),
        "adc_sigma": (i, [vp, vp, vp, i]),
        "adc_davidson": (i, [vp, i, vp, vp, vp, vp]),
        "adc_spec_factors": (i, [vp, vp, i, vp, vp]),
        "adc_set_guess": (i, [vp, vp, i]),
        "adc_last_error": (ctypes.c_char_p, [vp]),
        "adc_destroy": (None, [vp]),
        "adc_last_stats": (i, [vp, vp, vp, vp, vp]),
        "adc_workspace": (i, [vp, vp, vp]),
        "adc_sigma_flops": (i, [vp, i, vp, vp]),
        "adc_sigma_timed": (i, [vp, vp, vp, i, vp, vp]),
        "adc_history": (i, [vp, i, vp, vp, vp, vp]),
        "adc_mlp_nparams": (ll, []),
        "adc_precond_mlp": (i, [vp, vp, ll]),
        "adc_mlp_status": (i, [vp, vp, vp]),
        "adc_mlp_pairs": (i, [vp, vp, vp, d, vp, vp, ll, vp, vp, vp]),
        "adc_mlp_forward": (i, [vp, vp, vp, ll, i, vp]),
        "adc_mlp_loss_grad": (i, [vp, vp, vp, vp, vp, ll, vp, vp]),
        "adc_mlp_adam": (i, [vp, vp, vp, vp, vp, i, d]),
        "adc_record_count": (i, [vp]),
        "adc_record_get": (i, [vp, i, vp, vp, vp, vp]),
        "adc_graph_launches": (ll, [vp]),
        "adc_batch_davidson": (i, [vp, i, i, i, vp, vp, vp, vp, vp]),
        "adc_setup_batch": (i, [i, vp, ctypes.POINTER(vp)]),
        "adc_batch_set_option": (i, [vp, ctypes.c_char_p, d]),
        "adc_davidson_batch": (i, [vp, i, i, vp, vp, vp, vp, vp]),
        "adc_batch_context": (vp, [vp, i]),
        "adc_batch_destroy": (None, [vp]),
        "adc_gemm": (i, [i, i, i, ll, ll, ll, d, vp, ll, vp, ll, d, vp, ll, vp, i, vp]),
        "adc_gemm_configs": (i, [i, vp]),
        "adc_mlp_forward_noalloc": (i, [vp, vp, ll, i, vp, vp]),
        "adc_set_setup_option": (i, [ctypes.c_char_p, d]),
        "adc_spectral_function": (i, [vp, i, vp, vp, i, d, vp, vp]),
        "adc_propagator_diag": (i, [vp, i, vp, vp, i, i, d, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def last_error(ctx=None) -> str:
    return lib.adc_last_error(ctx).decode()


def _check(rc, ctx=None, allow_noconv=False):
    if rc == ADC_OK or (allow_noconv and rc == ADC_E_NOCONV):
        return rc
    raise ADCError(rc, last_error(ctx))


def _dev(x, torch, dtype=None):
    dtype = dtype or torch.float64
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == dtype and x.is_contiguous()):
        raise TypeError("expected a contiguous CUDA tensor of dtype %s" % dtype)
    return ctypes.c_void_p(x.data_ptr())


def _dev_or_host(x, torch):
    """A float64 input adc_setup accepts in device or host memory: a contiguous
    CUDA tensor, a contiguous CPU tensor or a C-contiguous numpy array."""
    import numpy as np
    if isinstance(x, np.ndarray):
        if x.dtype != np.float64 or not x.flags["C_CONTIGUOUS"]:
            raise TypeError("expected a C-contiguous float64 array")
        return ctypes.c_void_p(x.ctypes.data)
    if isinstance(x, torch.Tensor) and not x.is_cuda:
        if x.dtype != torch.float64 or not x.is_contiguous():
            raise TypeError("expected a contiguous float64 tensor")
        return ctypes.c_void_p(x.data_ptr())
    return _dev(x, torch)


def batch_davidson(contexts, nroots, use_graph=True, concurrent=False, threads=0):
    """Solve several systems together (adc_batch_davidson): in lockstep, or
    concurrently on host threads (concurrent=True; `threads` of them, 0: 8).  Returns
    (energies [nsys][nroots], P [nsys][nroots], iterations [nsys],
    statuses [nsys], stats {iterations, graph_launches, captures})."""
    import numpy as np
    n = len(contexts)
    arr = (ctypes.c_void_p * n)(*[c._h.value if isinstance(c._h, ctypes.c_void_p) else c._h
                                  for c in contexts])
    e = np.zeros((n, nroots))
    P = np.zeros((n, nroots))
    it = np.zeros(n, dtype=np.int32)
    st = np.zeros(n, dtype=np.int32)
    stats = np.zeros(5, dtype=np.int64)
    flags = int(bool(use_graph)) | (2 if concurrent else 0) | 4 | (int(threads) << 8)
    rc = lib.adc_batch_davidson(arr, n, int(nroots), flags,
                                e.ctypes.data_as(ctypes.c_void_p), P.ctypes.data_as(ctypes.c_void_p),
                                it.ctypes.data_as(ctypes.c_void_p), st.ctypes.data_as(ctypes.c_void_p),
                                stats.ctypes.data_as(ctypes.c_void_p))
    if rc not in (ADC_OK, ADC_E_NOCONV):
        raise ADCError(rc, last_error(None))
    return e, P, it, st, {"iterations": int(stats[0]), "graph_launches": int(stats[1]),
                          "captures": int(stats[2]), "launches": int(stats[3]),
                          "instantiations": int(stats[4])}


def gemm_configs(dtype):
    """Tile configuration ids compiled for a product type (adc_gemm_configs)."""
    ids = (ctypes.c_int * 8)()
    n = lib.adc_gemm_configs(int(dtype), ids)
    if n < 0:
        raise ADCError(n, last_error(None))
    return list(ids[:n])


def gemm(dtype, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, omap=None, config=-1):
    """adc_gemm on torch device tensors (A, B, C: contiguous CUDA tensors of
    the storage type of `dtype`; BF16 operands as torch.bfloat16)."""
    import torch
    st = {0: (torch.float64, torch.float64), 1: (torch.float32, torch.float32),
          2: (torch.float32, torch.float32), 3: (torch.bfloat16, torch.float32)}[int(dtype)]
    m = None
    if omap is not None:
        m = (ctypes.c_longlong * 6)(*[int(x) for x in omap])
    _check(lib.adc_gemm(int(dtype), int(ta), int(tb), int(M), int(N), int(K), float(alpha),
                        _dev(A, torch, st[0]), int(lda), _dev(B, torch, st[0]), int(ldb),
                        float(beta), _dev(C, torch, st[1]), int(ldc), m, int(config),
                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))


MLP_NOALLOC_ROWS = 8192


def spectral_function(omega, energies, P, eta):
    """adc_spectral_function on float64 CUDA tensors: A(omega) [nomega]."""
    import torch
    A = torch.empty_like(omega)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _check(lib.adc_spectral_function(_dev(omega, torch), omega.numel(), _dev(energies, torch),
                                     _dev(P, torch), energies.numel(), float(eta), _dev(A, torch),
                                     st))
    return A


def propagator_diag(omega, energies, X, eta):
    """adc_propagator_diag: complex [nomega, norb] tensor G_pp(omega + i eta)."""
    import torch
    nr, norb = X.shape
    G = torch.empty((omega.numel(), norb, 2), dtype=torch.float64, device=omega.device)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _check(lib.adc_propagator_diag(_dev(omega, torch), omega.numel(), _dev(energies, torch),
                                   _dev(X.contiguous(), torch), nr, norb, float(eta),
                                   _dev(G, torch), st))
    return torch.complex(G[..., 0], G[..., 1])


def set_setup_option(key, value):
    """adc_set_setup_option: an option for later adc_setup calls of this thread."""
    _check(lib.adc_set_setup_option(key.encode(), float(value)))


def mlp_forward_noalloc(params, F, y, bf16=False, stream=None):
    """adc_mlp_forward_noalloc: y[n] (float32 device, written) for features
    F [n, 7] (float32 device), no allocation anywhere; enqueued on `stream`
    (default: torch's current stream) without synchronising."""
    import torch
    f32 = torch.float32
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib.adc_mlp_forward_noalloc(_dev(params, torch, f32), _dev(F, torch, f32),
                                       int(F.shape[0]), int(bool(bf16)), _dev(y, torch, f32),
                                       ctypes.c_void_p(st.cuda_stream)))


class _SystemDesc(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_void_p), ("B", ctypes.c_void_p), ("nocc", ctypes.c_int),
                ("nvir", ctypes.c_int), ("naux", ctypes.c_int), ("order", ctypes.c_int),
                ("kind", ctypes.c_int)]


class Batch:
    """Several systems owned by one batch object (adc_setup_batch).

    systems: list of (eps [N] CUDA float64, B [Naux, N, N] CUDA float64, nocc,
    order, kind)."""

    def __init__(self, systems):
        import torch
        self._torch = torch
        n = len(systems)
        descs = (_SystemDesc * n)()
        self.dims = []
        for k, (eps, B, nocc, order, kind) in enumerate(systems):
            kk = ADC_EA if kind == "ea" else ADC_IP if kind == "ip" else -9
            descs[k] = _SystemDesc(_dev(eps, torch).value, _dev(B, torch).value, int(nocc),
                                   int(eps.shape[0]) - int(nocc), int(B.shape[0]), int(order), kk)
        h = ctypes.c_void_p()
        _check(lib.adc_setup_batch(n, descs, ctypes.byref(h)))
        self._h = h
        self.n = n
        self.dims = [int(lib.adc_dim(lib.adc_batch_context(h, k))) for k in range(n)]

    def set_option(self, key, value):
        _check(lib.adc_batch_set_option(self._h, key.encode(), float(value)))

    def davidson(self, nroots, use_graph=True, concurrent=False, threads=0):
        """adc_davidson_batch: (energies [n][nroots], P, iterations, statuses, stats)."""
        import numpy as np
        n = self.n
        e = np.zeros((n, nroots))
        P = np.zeros((n, nroots))
        it = np.zeros(n, dtype=np.int32)
        st = np.zeros(n, dtype=np.int32)
        stats = np.zeros(3, dtype=np.int64)
        flags = int(bool(use_graph)) | (2 if concurrent else 0) | (int(threads) << 8)
        rc = lib.adc_davidson_batch(self._h, int(nroots), flags,
                                    e.ctypes.data_as(ctypes.c_void_p),
                                    P.ctypes.data_as(ctypes.c_void_p),
                                    it.ctypes.data_as(ctypes.c_void_p),
                                    st.ctypes.data_as(ctypes.c_void_p),
                                    stats.ctypes.data_as(ctypes.c_void_p))
        if rc not in (ADC_OK, ADC_E_NOCONV):
            raise ADCError(rc, last_error(None))
        return e, P, it, st, {"iterations": int(stats[0]), "graph_launches": int(stats[1]),
                              "captures": int(stats[2])}

    def close(self):
        if getattr(self, "_h", None):
            lib.adc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """One ADC(n) problem resident on the current GPU.

    eps: [N], B: [Naux, N, N], float64: CUDA tensors, or host memory (CPU
    tensors or numpy arrays; B is then staged in blocks).
    kind: "ea" or "ip"; order: 2 or 3.
    """

    def __init__(self, eps, B, nocc, order=2, kind="ea", stream=None):
        import torch
        self._torch = torch
        self.nocc = int(nocc)
        self.nvir = int(eps.shape[0]) - self.nocc
        self.naux = int(B.shape[0])
        self.order, self.kind = int(order), kind
        h = ctypes.c_void_p()
        k = ADC_EA if kind == "ea" else ADC_IP if kind == "ip" else -9
        rc = lib.adc_setup(_dev_or_host(eps, torch), _dev_or_host(B, torch), self.nocc,
                           self.nvir, self.naux, self.order, k, ctypes.byref(h))
        _check(rc)
        self._h = h
        self.dim = int(lib.adc_dim(h))
        self.nmo = self.nocc + self.nvir
        if stream is not None:
            self.set_stream(stream)

    # ------------------------------------------------------------------
    def set_option(self, key, value):
        _check(lib.adc_set_option(self._h, key.encode(), float(value)), self._h)

    def set_stream(self, stream):
        ptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        _check(lib.adc_set_stream(self._h, ctypes.c_void_p(ptr)), self._h)

    def diag(self):
        torch = self._torch
        d = torch.empty(self.dim, dtype=torch.float64, device="cuda")
        _check(lib.adc_diag(self._h, _dev(d, torch)), self._h)
        return d

    def sigma(self, X, out=None):
        torch = self._torch
        X = X.reshape(-1, self.dim)
        if out is None:
            out = torch.empty_like(X)
        _check(lib.adc_sigma(self._h, _dev(X, torch), _dev(out, torch), X.shape[0]), self._h)
        return out

    def davidson(self, nroots, want_vectors=True):
        """Returns (energies [nroots], P [nroots], vectors or None, iterations, converged)."""
        torch = self._torch
        e = (ctypes.c_double * nroots)()
        P = (ctypes.c_double * nroots)()
        it = ctypes.c_int()
        vecs = torch.empty((nroots, self.dim), dtype=torch.float64, device="cuda") \
            if want_vectors else None
        rc = lib.adc_davidson(self._h, int(nroots), e, P,
                              _dev(vecs, torch) if want_vectors else None, ctypes.byref(it))
        _check(rc, self._h, allow_noconv=True)
        return list(e), list(P), vecs, it.value, rc == ADC_OK

    def spec_factors(self, vecs):
        torch = self._torch
        vecs = vecs.reshape(-1, self.dim)
        n = vecs.shape[0]
        P = (ctypes.c_double * n)()
        X = torch.empty((n, self.nmo), dtype=torch.float64, device="cuda")
        _check(lib.adc_spec_factors(self._h, _dev(vecs, torch), n, P, _dev(X, torch)), self._h)
        return list(P), X

    def set_guess(self, V0):
        torch = self._torch
        V0 = V0.reshape(-1, self.dim)
        _check(lib.adc_set_guess(self._h, _dev(V0, torch), V0.shape[0]), self._h)

    def sigma_flops(self, nvec):
        t, p = ctypes.c_double(), ctypes.c_double()
        _check(lib.adc_sigma_flops(self._h, int(nvec), ctypes.byref(t), ctypes.byref(p)), self._h)
        return t.value, p.value

    def sigma_timed(self, X, out=None):
        """sigma with HIP-event timing: returns (Y, ms_pp, ms_total)."""
        torch = self._torch
        X = X.reshape(-1, self.dim)
        if out is None:
            out = torch.empty_like(X)
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(lib.adc_sigma_timed(self._h, _dev(X, torch), _dev(out, torch), X.shape[0],
                                   ctypes.byref(a), ctypes.byref(b)), self._h)
        return out, a.value, b.value

    def history(self, nroots, max_entries=100000):
        """(seconds [n], theta [n, nroots], rnorm [n, nroots], mixed [n]) of the last solve."""
        import numpy as np
        n = lib.adc_history(self._h, 0, None, None, None, None)
        if n < 0:
            _check(n, self._h)
        n = min(n, max_entries)
        t = np.zeros(n)
        th = np.zeros((n, nroots))
        r = np.zeros((n, nroots))
        mx = np.zeros(n, dtype=np.int32)
        lib.adc_history(self._h, n, t.ctypes.data_as(ctypes.c_void_p),
                        th.ctypes.data_as(ctypes.c_void_p), r.ctypes.data_as(ctypes.c_void_p),
                        mx.ctypes.data_as(ctypes.c_void_p))
        return t, th, r, mx

    def stats(self):
        it, sv, mi, sec = ctypes.c_int(), ctypes.c_longlong(), ctypes.c_int(), ctypes.c_double()
        _check(lib.adc_last_stats(self._h, ctypes.byref(it), ctypes.byref(sv), ctypes.byref(mi),
                                  ctypes.byref(sec)), self._h)
        return {"iters": it.value, "sigma_vectors": sv.value, "mixed_iters": mi.value,
                "seconds": sec.value}

    def workspace(self):
        """Device bytes the context holds now and at most so far."""
        used, peak = ctypes.c_longlong(), ctypes.c_longlong()
        _check(lib.adc_workspace(self._h, ctypes.byref(used), ctypes.byref(peak)), self._h)
        return {"used": used.value, "peak": peak.value}

    def graph_launches(self):
        return int(lib.adc_graph_launches(self._h))

    # ---- learned preconditioner ------------------------------------------
    def precond_mlp(self, params):
        """Install FP32 device parameters (or None for the diagonal one)."""
        torch = self._torch
        if params is None:
            _check(lib.adc_precond_mlp(self._h, None, 0), self._h)
        else:
            _check(lib.adc_precond_mlp(self._h, _dev(params, torch, torch.float32),
                                       params.numel()), self._h)

    def mlp_status(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(lib.adc_mlp_status(self._h, ctypes.byref(a), ctypes.byref(b)), self._h)
        return bool(a.value), b.value

    def mlp_pairs(self, x, r, theta, xstar, idx):
        """Features F [n, 7], a [n], t [n] (float32 device) for sampled elements."""
        torch = self._torch
        n = idx.numel()
        F = torch.empty((n, 7), dtype=torch.float32, device="cuda")
        a = torch.empty(n, dtype=torch.float32, device="cuda")
        t = torch.empty(n, dtype=torch.float32, device="cuda")
        _check(lib.adc_mlp_pairs(self._h, _dev(x, torch), _dev(r, torch), float(theta),
                                 _dev(xstar, torch), _dev(idx, torch, torch.int64), n,
                                 _dev(F, torch, torch.float32), _dev(a, torch, torch.float32),
                                 _dev(t, torch, torch.float32)), self._h)
        return F, a, t

    def mlp_forward(self, params, F, bf16=False):
        torch = self._torch
        y = torch.empty(F.shape[0], dtype=torch.float32, device="cuda")
        _check(lib.adc_mlp_forward(self._h, _dev(params, torch, torch.float32),
                                   _dev(F, torch, torch.float32), F.shape[0], int(bf16),
                                   _dev(y, torch, torch.float32)), self._h)
        return y

    def mlp_loss_grad(self, params, F, a, t, grad=None):
        torch = self._torch
        if grad is None:
            grad = torch.empty_like(params)
        loss = ctypes.c_double()
        f32 = torch.float32
        _check(lib.adc_mlp_loss_grad(self._h, _dev(params, torch, f32), _dev(F, torch, f32),
                                     _dev(a, torch, f32), _dev(t, torch, f32), F.shape[0],
                                     _dev(grad, torch, f32), ctypes.byref(loss)), self._h)
        return loss.value, grad

    def mlp_adam(self, params, grad, m, v, step, lr):
        torch = self._torch
        f32 = torch.float32
        _check(lib.adc_mlp_adam(self._h, _dev(params, torch, f32), _dev(grad, torch, f32),
                                _dev(m, torch, f32), _dev(v, torch, f32), int(step), float(lr)),
               self._h)

    def records(self):
        """Recorded iterates of the last solve: list of (x, r, theta, root)."""
        torch = self._torch
        n = lib.adc_record_count(self._h)
        out = []
        for i in range(n):
            x = torch.empty(self.dim, dtype=torch.float64, device="cuda")
            r = torch.empty_like(x)
            th, rt = ctypes.c_double(), ctypes.c_int()
            _check(lib.adc_record_get(self._h, i, _dev(x, torch), _dev(r, torch),
                                      ctypes.byref(th), ctypes.byref(rt)), self._h)
            out.append((x, r, th.value, rt.value))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib.adc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class ContextU(Context):
    """An unrestricted (open-shell) EA/IP-ADC(2) problem (adc_setup_u).

    eps_a, eps_b: [N]; B_a, B_b: [Naux, N, N], float64, on the GPU or in host
    memory; nocc_a / nocc_b alpha / beta electrons.  Vectors hold both spin
    sectors (layout in include/adc.h); spectroscopic amplitudes have 2N rows
    (alpha orbitals, then beta) and the factors are sum |X|^2 over them."""

    def __init__(self, eps_a, eps_b, B_a, B_b, nocc_a, nocc_b, order=2, kind="ea", stream=None):
        import torch
        self._torch = torch
        self.nocc, self.nocc_b = int(nocc_a), int(nocc_b)
        n = int(eps_a.shape[0])
        self.nvir = n - self.nocc
        self.naux = int(B_a.shape[0])
        self.order, self.kind = int(order), kind
        h = ctypes.c_void_p()
        k = ADC_EA if kind == "ea" else ADC_IP if kind == "ip" else -9
        rc = lib.adc_setup_u(_dev_or_host(eps_a, torch), _dev_or_host(eps_b, torch),
                             _dev_or_host(B_a, torch), _dev_or_host(B_b, torch), self.nocc,
                             self.nocc_b, n, self.naux, self.order, k, ctypes.byref(h))
        _check(rc)
        self._h = h
        self.dim = int(lib.adc_dim(h))
        self.nmo = 2 * n          # rows of the spectroscopic amplitudes
        if stream is not None:
            self.set_stream(stream)
