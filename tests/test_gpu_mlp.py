"""GPU parity of the learned-preconditioner kernels against the oracle
(oracle/mlp.py), and its behaviour inside the Davidson solver.

Tolerances: FP32 kernels against the FP64 oracle, relative 1e-4 on outputs
and 1e-3 on gradients (sums of n * 256 FP32 products); the BF16 inference
layer to 2e-2 of the output scale (8-bit mantissas on 256-term sums)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ctx(eps, B, O, order, kind):
    import paper_2012_06714_amd as adc
    dev = torch.device("cuda:0")
    return adc.Context(torch.tensor(eps, device=dev), torch.tensor(B, device=dev), O, order, kind)


def _params(seed, scale_out=0.3):
    from oracle import mlp
    p = mlp.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    v = mlp.unpack(p)
    v["w3"][...] = rng.standard_normal(mlp.WIDTH) * scale_out
    v["b1"][...] = rng.standard_normal(mlp.WIDTH) * 0.1
    v["b2"][...] = rng.standard_normal(mlp.WIDTH) * 0.1
    v["b3"][0] = 0.05
    return p


def _small_ctx():
    from synthetic import small_system
    eps, B = small_system(3, 7, 24, 2)
    return _ctx(eps, B, 3, 2, "ea"), eps


def test_forward_matches_oracle():
    from oracle import mlp
    ctx, _ = _small_ctx()
    p = _params(11).astype(np.float32)
    rng = np.random.default_rng(12)
    n = 3000
    F = rng.standard_normal((n, mlp.NF)).astype(np.float32)
    y_ref, _ = mlp.forward(p.astype(np.float64), F.astype(np.float64))
    pd, Fd = torch.tensor(p, device="cuda"), torch.tensor(F, device="cuda")
    y32 = ctx.mlp_forward(pd, Fd, bf16=False).cpu().numpy()
    y16 = ctx.mlp_forward(pd, Fd, bf16=True).cpu().numpy()
    ctx.close()
    scale = np.abs(y_ref).max()
    assert np.abs(y32 - y_ref).max() <= 1e-4 * scale
    assert np.abs(y16 - y_ref).max() <= 2e-2 * scale
    assert np.abs(y16 - y_ref).max() > 1e-7 * scale      # really BF16


@pytest.mark.parametrize("n", [777, 20000])
def test_loss_and_gradient_match_oracle(n):
    """n = 20000 takes the split-K path of the weight-gradient products."""
    from oracle import mlp
    ctx, _ = _small_ctx()
    p = _params(13).astype(np.float32)
    rng = np.random.default_rng(14)
    F = rng.standard_normal((n, mlp.NF)).astype(np.float32)
    a = rng.standard_normal(n).astype(np.float32)
    t = rng.standard_normal(n).astype(np.float32)
    loss_ref, g_ref = mlp.loss_and_grad(p.astype(np.float64), F.astype(np.float64),
                                        a.astype(np.float64), np.ones(n), t.astype(np.float64))
    loss, g = ctx.mlp_loss_grad(torch.tensor(p, device="cuda"), torch.tensor(F, device="cuda"),
                                torch.tensor(a, device="cuda"), torch.tensor(t, device="cuda"))
    ctx.close()
    g = g.cpu().numpy()
    assert abs(loss - loss_ref) <= 1e-4 * abs(loss_ref)
    for name, gv in mlp.unpack(g).items():
        rv = mlp.unpack(g_ref)[name]
        assert np.abs(gv - rv).max() <= 1e-3 * max(np.abs(rv).max(), 1e-12), name


def test_adam_step_matches_oracle():
    from oracle import mlp
    ctx, _ = _small_ctx()
    rng = np.random.default_rng(15)
    npar = mlp.NPARAM
    p = rng.standard_normal(npar).astype(np.float32)
    g = rng.standard_normal(npar).astype(np.float32)
    m = rng.standard_normal(npar).astype(np.float32) * 0.1
    v = np.abs(rng.standard_normal(npar)).astype(np.float32) * 0.1
    pr, mr, vr = mlp.adam_step(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                               v.astype(np.float64), 3, 1e-3)
    pd, md, vd = (torch.tensor(x, device="cuda") for x in (p, m, v))
    ctx.mlp_adam(pd, torch.tensor(g, device="cuda"), md, vd, 3, 1e-3)
    ctx.close()
    assert np.abs(pd.cpu().numpy() - pr).max() <= 1e-5 * np.abs(pr).max()
    assert np.abs(md.cpu().numpy() - mr).max() <= 1e-5 * np.abs(mr).max()
    assert np.abs(vd.cpu().numpy() - vr).max() <= 1e-5 * np.abs(vr).max()


@pytest.mark.parametrize("kind", ["ea", "ip"])
def test_training_pairs_match_oracle(kind):
    """Recorded Davidson iterates -> features, diagonal factor, target (all
    elements sampled) against the oracle's definitions."""
    from oracle import mlp
    from synthetic import small_system
    O, V, Q = 3, 9, 30
    eps, B = small_system(O, V, Q, 21)
    _say(f"case pairs {kind}")
    ctx = _ctx(eps, B, O, 2, kind)
    ctx.set_option("record", 6)
    e, P, vecs, it, conv = ctx.davidson(2, want_vectors=True)
    recs = ctx.records()
    assert len(recs) == 6
    D = ctx.diag().cpu().numpy()
    idx = torch.arange(ctx.dim, device="cuda", dtype=torch.int64)
    for x, r, theta, root in recs[2:4]:
        F, a, t = ctx.mlp_pairs(x, r, theta, vecs[root].contiguous(), idx)
        xh, rh, xs = x.cpu().numpy(), r.cpu().numpy(), vecs[root].cpu().numpy()
        F_ref = mlp.features(kind, O, eps, D, theta, rh)
        q = mlp.diag_factor(theta, D)
        t_ref = mlp.target(xh, xs, F_ref[:, 1], q)
        assert np.allclose(F.cpu().numpy(), F_ref, rtol=1e-6, atol=1e-6)
        assert np.allclose(a.cpu().numpy(), F_ref[:, 1] * q, rtol=1e-6, atol=1e-7)
        assert np.allclose(t.cpu().numpy(), t_ref, rtol=1e-5, atol=1e-6 * np.abs(t_ref).max())
    ctx.close()


def test_untrained_network_reproduces_diagonal_solve():
    """Zero output layer: the learned correction is the diagonal one, so the
    solve follows the same path (same iterations and energies)."""
    from paper_2012_06714_amd import mlp_train
    from synthetic import small_system
    eps, B = small_system(4, 11, 33, 3)
    ctx = _ctx(eps, B, 4, 2, "ea")
    ctx.set_option("tol_e", 1e-9)
    ctx.set_option("tol_r", 1e-6)
    e0, _, _, it0, c0 = ctx.davidson(3, want_vectors=False)
    ctx.precond_mlp(mlp_train.init_params(5, torch))
    e1, _, _, it1, c1 = ctx.davidson(3, want_vectors=False)
    ctx.close()
    assert c0 and c1
    assert abs(it1 - it0) <= 1
    assert np.abs(np.array(e1) - np.array(e0)).max() < 1e-8


def test_nonfinite_network_falls_back_to_diagonal():
    """NaN weights: the solve switches to the diagonal preconditioner and
    still converges to the same roots."""
    from paper_2012_06714_amd import mlp_train
    from synthetic import small_system
    eps, B = small_system(4, 11, 33, 3)
    ctx = _ctx(eps, B, 4, 2, "ea")
    ctx.set_option("tol_e", 1e-9)
    ctx.set_option("tol_r", 1e-6)
    e0, _, _, _, _ = ctx.davidson(3, want_vectors=False)
    p = mlp_train.init_params(5, torch)
    p[-1] = float("nan")
    ctx.precond_mlp(p)
    e1, _, _, _, c1 = ctx.davidson(3, want_vectors=False)
    installed, fallbacks = ctx.mlp_status()
    ctx.close()
    assert c1 and installed and fallbacks == 1
    assert np.abs(np.array(e1) - np.array(e0)).max() < 1e-8


def test_trained_network_gain_is_measured():
    """Train on the iterates of two systems of the batched EA-ADC(2) family
    (nocc capped at 10), then solve two held-out systems with and without the
    network.  Both reach the same roots; the iteration counts are printed
    (the measured gain may be negative: the diagonal fallback bounds the
    loss).  The bound asserted, at most twice the diagonal solve's iterations
    plus 8, is loose: on the 64 held-out systems of the full batched family
    the learned solves took at most 30 % more iterations than the diagonal
    ones (18 of them fewer)."""
    import paper_2012_06714_amd as adc
    from paper_2012_06714_amd import mlp_train
    from synthetic import make_batch_system
    dev = torch.device("cuda:0")

    def ctx_for(s):
        eps, B, (O, V, Q) = make_batch_system(s, 10)
        return adc.Context(torch.tensor(eps, device=dev), torch.tensor(B, device=dev), O, 2, "ea")

    Fs, As, Ts = [], [], []
    for s in (100, 101):
        c = ctx_for(s)
        c.set_option("tol_e", 1e-8)
        c.set_option("tol_r", 1e-6)
        F, a, t, _ = mlp_train.collect_pairs(c, 2, 2048, s, torch, max_records=40, block=4)
        Fs.append(F)
        As.append(a)
        Ts.append(t)
        c.close()
    F, a, t = torch.cat(Fs), torch.cat(As), torch.cat(Ts)
    c = ctx_for(0)
    params, hist = mlp_train.train(c, F, a, t, 300, 1e-3, 8192, 3, torch)
    c.close()
    assert np.mean(hist[-30:]) < hist[0]          # training lowers the loss
    for s in (0, 1):
        c = ctx_for(s)
        c.set_option("tol_e", 1e-8)
        c.set_option("tol_r", 1e-6)
        c.set_option("block", 4)
        e0, _, _, it0, ok0 = c.davidson(2, want_vectors=False)
        c.precond_mlp(params)
        e1, _, _, it1, ok1 = c.davidson(2, want_vectors=False)
        _, fb = c.mlp_status()
        c.close()
        _say(f"system {s}: diagonal {it0} iterations, learned {it1} (fallbacks {fb})")
        assert ok0 and ok1
        assert np.abs(np.array(e0) - np.array(e1)).max() < 1e-7
        assert it1 <= 2 * it0 + 8, (it0, it1)
