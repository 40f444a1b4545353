"""Training of the learned Davidson preconditioner (orchestration only: every
arithmetic step runs in the library's kernels through the C ABI).

Training pairs come from the method's own iterates: a Davidson solve with
the diagonal preconditioner records its Ritz vectors and residuals
(option "record"); against the converged eigenvectors each record yields
features, the diagonal correction and the target for a random sample of
elements (adc_mlp_pairs).  The network is then fitted with FP32
forward/backward kernels (adc_mlp_loss_grad) and Adam (adc_mlp_adam).
"""
from __future__ import annotations

import numpy as np

NF = 7
WIDTH = 256


def init_params(seed, torch):
    """Layers 1-2 Gaussian with std 1/sqrt(fan_in); the output layer starts at
    zero, so the untrained network is the diagonal preconditioner."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal((WIDTH, NF)) / np.sqrt(NF)
    w2 = rng.standard_normal((WIDTH, WIDTH)) / np.sqrt(WIDTH)
    p = np.concatenate([w1.ravel(), np.zeros(WIDTH), w2.ravel(), np.zeros(WIDTH),
                        np.zeros(WIDTH), np.zeros(1)]).astype(np.float32)
    return torch.tensor(p, device="cuda")


def collect_pairs(ctx, nroots, per_record, seed, torch, max_records=200, block=None):
    """Solve with the diagonal preconditioner, record the iterates and turn
    them into (F, a, t) pairs for `per_record` random elements each."""
    if ctx.mlp_status()[0]:
        ctx.set_option("precond", 0)
    ctx.set_option("record", max_records)
    if block:
        ctx.set_option("block", block)
    e, P, vecs, it, conv = ctx.davidson(nroots, want_vectors=True)
    recs = ctx.records()
    ctx.set_option("record", 0)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(seed))
    Fs, As, Ts = [], [], []
    for x, r, theta, root in recs:
        if float(r.norm()) == 0.0:
            continue
        n = min(per_record, ctx.dim)
        idx = torch.randint(0, ctx.dim, (n,), device="cuda", generator=gen, dtype=torch.int64)
        F, a, t = ctx.mlp_pairs(x, r, theta, vecs[root].contiguous(), idx)
        Fs.append(F)
        As.append(a)
        Ts.append(t)
    return torch.cat(Fs), torch.cat(As), torch.cat(Ts), it


def train(ctx, F, a, t, steps, lr, batch, seed, torch, params=None, log=None):
    """Adam on minibatches of the pairs; returns (params, loss history)."""
    if params is None:
        params = init_params(seed, torch)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.empty_like(params)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(seed) + 1)
    n = F.shape[0]
    hist = []
    for step in range(1, steps + 1):
        sel = torch.randint(0, n, (min(batch, n),), device="cuda", generator=gen)
        Fb, ab, tb = F[sel].contiguous(), a[sel].contiguous(), t[sel].contiguous()
        loss, _ = ctx.mlp_loss_grad(params, Fb, ab, tb, grad)
        ctx.mlp_adam(params, grad, m, v, step, lr)
        hist.append(loss)
        if log and (step % max(1, steps // 10) == 0 or step == 1):
            log(f"mlp train step {step}: loss {loss:.4e}")
    return params, hist
