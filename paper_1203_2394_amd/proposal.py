"""Training and evaluating the learned outer proposal.

The look-ahead DPF itself produces the training data: before each step the
features of every outer particle are taken (dpf_features), after it the
outer ancestors A_k and the new particles x_t^(k) (the SIR draws from the
Monte Carlo optimal proposal eq:approx3).  The pairs (features of A_k,
x_t^(k)) teach the mixture density network q(x_t | features) to stand in
for that proposal.  Training minimises the mixture negative log-likelihood
with Adam, all on the library's BF16 matrix-core kernels; the feature
statistics, the standardisation, the per-epoch shuffle and the batch gather
are library calls too (dpf_feature_stats, dpf_standardize, dpf_permutation,
dpf_gather_rows), PyTorch only holding the device buffers.

The evaluation runs the look-ahead DPF and the learned step (with its ESS
fallback) on the same fresh observation sequence and reports the RMSE of the
posterior mean of x against the simulated truth, the fallback rate and the
time per step of each.
"""
import time

import numpy as np

from . import BUF_ANC, BUF_FALLBACK, BUF_X, MLP_IN, DPFError, Filter, MLP, _check, _ptr, _stream_ptr, init_params, lib

N_FEAT = 26  # x (2), y (8), cloud mean (8), cloud variance (8)


def _torch():
    import torch
    return torch


def generate_pairs(spec, n_pairs, N=256, M=256, T=200, n_filters=20, data_seed=1000, filter_seed=11,
                   device="cuda", simulate=None):
    """Run batches of n_filters look-ahead DPFs (one handle, one fresh
    simulated sequence each) until n_pairs (features, x_t) pairs are
    collected.  Returns raw features [n][26] and targets [n][2] (device
    float32)."""
    torch = _torch()
    feats, targets = [], []
    have, batch = 0, 0
    F = n_filters
    oo = torch.arange(F, device=device).repeat_interleave(N) * N
    while have < n_pairs:
        seeds = [data_seed + batch * F + q for q in range(F)]
        Y = torch.tensor(np.stack([simulate(spec, T, s)[2] for s in seeds], axis=1), dtype=torch.float32,
                         device=device)  # [T][F][dy]
        f = Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [N] * F, [M] * F,
                   seed=filter_seed + batch, device=device)
        for t in range(T):
            ft = f.features(Y[t])
            f.lookahead_step(Y[t])
            A = f.copy_buffer(BUF_ANC).long() + oo
            x = f.copy_buffer(BUF_X).reshape(spec.dx, F * N).t()
            feats.append(ft[A, :N_FEAT])
            targets.append(x.clone())
            have += F * N
            if have >= n_pairs:
                break
        f.close()
        batch += 1
    X = torch.cat(feats)[:n_pairs]
    xt = torch.cat(targets)[:n_pairs]
    return X, xt


def feature_stats(X):
    """Mean and sample standard deviation of each raw feature (floor 1e-3),
    computed on the device (dpf_feature_stats)."""
    torch = _torch()
    X = X.contiguous()
    n, cols = X.shape
    mean = torch.empty(cols, dtype=torch.float32, device=X.device)
    std = torch.empty(cols, dtype=torch.float32, device=X.device)
    _check(lib().dpf_feature_stats(_ptr(X), int(n), int(cols), int(cols), _ptr(mean), _ptr(std), 1e-3,
                                   _stream_ptr(X.device)))
    return mean.cpu().numpy(), std.cpu().numpy()


def train(X, xt, epochs=10, batch=4096, lr=1e-3, seed=0, verbose=False):
    """Fit the network to (raw features X [n][26], targets xt [n][2]).  Each
    epoch takes a fresh permutation of the pairs (dpf_permutation keyed by
    (seed, epoch)) and its first floor(n / batch) batches.  Returns (MLP,
    mean NLL per epoch)."""
    torch = _torch()
    device = X.device
    X = X.contiguous()
    xt = xt.contiguous()
    n = X.shape[0]
    fmean, fstd = feature_stats(X)
    mlp = MLP(init_params(seed, N_FEAT), fmean, fstd, batch=batch, device=device)
    L = lib()
    st = _stream_ptr(device)
    Xs = torch.empty(n, MLP_IN, dtype=torch.float32, device=device)
    _check(L.dpf_standardize(_ptr(X), int(n), N_FEAT, N_FEAT, _ptr(mlp.fmean), _ptr(mlp.fstd), _ptr(Xs), MLP_IN,
                             st))
    nb = n // batch
    if nb == 0:
        raise DPFError("need at least one batch of %d pairs" % batch)
    perm = torch.empty(n, dtype=torch.int32, device=device)
    xb = torch.empty(batch, MLP_IN, dtype=torch.float32, device=device)
    tb = torch.empty(batch, 2, dtype=torch.float32, device=device)
    lossv = torch.empty(max(nb, 1), dtype=torch.float32, device=device)
    losses = []
    for ep in range(epochs):
        _check(L.dpf_permutation(int(seed), int(ep), int(n), _ptr(perm), st))
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            _check(L.dpf_gather_rows(_ptr(Xs), int(n), MLP_IN, MLP_IN, _ptr(idx), batch, _ptr(xb), MLP_IN, st))
            _check(L.dpf_gather_rows(_ptr(xt), int(n), 2, 2, _ptr(idx), batch, _ptr(tb), 2, st))
            mlp.train_step(xb, tb, lr=lr, loss=lossv[b:b + 1])
        losses.append(float(np.mean(lossv[:nb].cpu().numpy().astype(np.float64))))
        if verbose:
            print("epoch %d: mean NLL %.4f" % (ep, losses[-1]), flush=True)
    return mlp, losses


def evaluate(spec, mlp, N=4096, M=256, T=200, n_seq=8, data_seed=5000, filter_seed=77, ess_frac=0.1,
             device="cuda", simulate=None, timing_reps=3):
    """Look-ahead vs learned on n_seq fresh sequences (one batched handle per
    method): RMSE of the posterior mean of x against the truth (root of the
    mean over sequences and steps), fraction of filter-steps that fell back,
    and milliseconds per step of a single filter (device time of T
    consecutive steps, best of timing_reps)."""
    torch = _torch()
    sims = [simulate(spec, T, data_seed + q) for q in range(n_seq)]
    Y = torch.tensor(np.stack([s[2] for s in sims], axis=1), dtype=torch.float32, device=device)
    truth = np.stack([s[0][1:] for s in sims], axis=1)  # [T][F][dx]
    out = {}
    for mode in ("lookahead", "learned"):
        f = Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [N] * n_seq, [M] * n_seq, seed=filter_seed,
                   device=device)
        if mode == "learned":
            f.set_proposal(mlp, ess_frac=ess_frac)
        step = f.lookahead_step if mode == "lookahead" else f.learned_step
        xh = torch.empty(T, n_seq, spec.dx, dtype=torch.float32, device=device)
        fb = torch.zeros(T, n_seq, dtype=torch.int32, device=device)
        for t in range(T):
            step(Y[t])
            xh[t] = f.estimate()["xhat"]
            if mode == "learned":
                fb[t] = f.copy_buffer(BUF_FALLBACK).int()
        err = np.sum((xh.cpu().numpy() - truth) ** 2, axis=2)  # [T][F]
        f.close()
        g = Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [N], [M], seed=filter_seed, device=device)
        if mode == "learned":
            g.set_proposal(mlp, ess_frac=ess_frac)
        gstep = g.lookahead_step if mode == "lookahead" else g.learned_step
        best = float("inf")
        for _ in range(timing_reps):
            g.reset()
            torch.cuda.synchronize(device)
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            for t in range(T):
                gstep(Y[t, :1])
            t1.record()
            torch.cuda.synchronize(device)
            best = min(best, t0.elapsed_time(t1) / T)
        g.close()
        out[mode] = {"rmse_x": float(np.sqrt(err.mean())),
                     "rmse_x_per_seq": [float(v) for v in np.sqrt(err.mean(axis=0))],
                     "fallback_frac": float(fb.float().mean()),
                     "ms_per_step": best, "updates_per_s": N * M / (best * 1e-3)}
    return out
