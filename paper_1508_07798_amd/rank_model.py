"""Rank-predictor MLP: training data from factorizations, training on the GPU.

The library sizes each separator's randomized sampling from a predicted ID rank
k^ as l = 32 ceil((m k^ + p_os) / 32), m = 3 by default (hss_opts_t.rank_model,
model_margin): samples well
above the rank keep the a-posteriori error estimate reliable, so few boxes need
a second round, and give better skeletons, so fewer GMRES iterations. The paper chooses an
anticipated rank from observed rank laws (Section 4); here a small network
8 -> 64 -> 64 -> 1 (tanh, tanh, linear) learns log2(1 + k) from the ranks the
adaptive ID itself produced on other problems. The judge and the rank-growth
fallback stay in place, so a poor prediction costs time, never accuracy.

Training runs on the device through the library's own forward / backward /
Adam kernels (hss_mlp_train).
"""
from __future__ import annotations

import time

import numpy as np

from . import hss

SIZES = (8, 64, 64, 1)


def init_weights(seed: int = 0) -> np.ndarray:
    """Flat parameter vector in the library's layout (W1, b1, W2, b2, W3, b3,
    row-major [out][in]); weights N(0, 1/fan_in), biases 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(3):
        fan_in, fan_out = SIZES[i], SIZES[i + 1]
        parts.append((rng.standard_normal((fan_out, fan_in)) / np.sqrt(fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == hss.MLP_NPARAMS
    return w


def samples(handle) -> tuple[np.ndarray, np.ndarray]:
    """(features [nbox, 8], largest ID rank per box) of a factorization; boxes
    whose complement was not compressed (rank 0) are left out."""
    f = np.asarray(handle.query("features"), dtype=np.float32).reshape(-1, 8)
    k = np.asarray(handle.query("ranks"), dtype=np.float64)
    keep = k > 0
    return f[keep], k[keep]


def collect(problems, prec="fp32", device="cuda:0"):
    """Factor every problem with the plain adaptive ID and gather (features, ranks)."""
    import torch
    X, K = [], []
    for P in problems:
        vals = torch.from_numpy(P.op.vals).to(device)
        kh = P.kappa / P.op.n if P.kappa else 0.0
        h = hss.factor(P.op, P.tree, P.tol, prec=prec, seed=P.seed, vals_dev=vals, kappa_h=kh)
        x, k = samples(h)
        h.close()
        X.append(x)
        K.append(k)
    return np.concatenate(X), np.concatenate(K)


def train(X: np.ndarray, ranks: np.ndarray, steps: int = 1500, lr: float = 3e-3, seed: int = 0,
          device="cuda:0"):
    """Full-batch Adam on the device; returns (weights as a host float32 array, loss history)."""
    import torch
    w = torch.from_numpy(init_weights(seed)).to(device)
    x = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(device)
    t = torch.from_numpy(np.log2(1.0 + ranks).astype(np.float32)).to(device)
    hist = hss.mlp_train(w, x, t, steps, lr=lr)
    return w.cpu().numpy(), hist.cpu().numpy()


def predict_rank(w: np.ndarray, X: np.ndarray, device="cuda:0") -> np.ndarray:
    import torch
    wd = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).to(device)
    x = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(device)
    y = hss.mlp_forward(wd, x).cpu().numpy().astype(np.float64)
    return np.exp2(y) - 1.0


def training_problems(family="helmholtz_p2_64", seed_offsets=(1, 2), grids=(16, 24, 32, 40, 48)):
    """Smaller seeded problems of the measured workload's family (same PDE, degree
    and tolerance) with other seeds than the measured workload."""
    from workloads import configs
    out = []
    for so in seed_offsets:
        for n in grids:
            out.append(configs.make(family, n=n, seed_offset=so))
    return out


def configs123_problems():
    """The Poisson (16 x 16, p = 1), Helmholtz (p = 2) and variable-coefficient Poisson
    (p = 3) workloads at their full sizes and on smaller grids of the same families,
    each factorized in its own precision: the runs the p = 4 Helmholtz configuration's
    rank model learns from."""
    from workloads import configs
    out = [(configs.make("poisson_p1_16"), "fp64")]
    for n in (16, 24, 32, 48, 64):
        out.append((configs.make("helmholtz_p2_64", n=n), "fp32"))
    for n in (16, 32, 64, 128):
        out.append((configs.make("varpoisson_p3_128", n=n), "bf16"))
    return out


def collect_mixed(problems, device="cuda:0"):
    """collect() over (problem, precision) pairs."""
    X, K = [], []
    for P, prec in problems:
        x, k = collect([P], prec=prec, device=device)
        X.append(x)
        K.append(k)
    return np.concatenate(X), np.concatenate(K)


def fit_default(device="cuda:0", steps=1500, family="helmholtz_p2_64", prec="fp32"):
    """Collect ranks on the training problems and train; returns (weights, info).
    family "configs123" trains on the Poisson, Helmholtz p = 2 and variable-coefficient
    Poisson runs (configs123_problems)."""
    t0 = time.perf_counter()
    if family == "configs123":
        X, K = collect_mixed(configs123_problems(), device=device)
    else:
        X, K = collect(training_problems(family), prec=prec, device=device)
    t1 = time.perf_counter()
    w, hist = train(X, K, steps=steps, device=device)
    t2 = time.perf_counter()
    pred = predict_rank(w, X, device=device)
    info = {"samples": int(X.shape[0]), "collect_s": round(t1 - t0, 3), "train_s": round(t2 - t1, 3),
            "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
            "train_under_predicted": float(np.mean(pred < K))}
    return w, info
