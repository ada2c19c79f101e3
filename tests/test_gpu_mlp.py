"""The rank-predictor MLP on the GPU (through the C ABI) against the FP64 oracle.

  * forward pass and gradient of the mean squared error equal the oracle's
    (oracle/mlp.py, itself pinned by central differences) to FP32 accuracy;
  * Adam training on the device follows the oracle's Adam trajectory;
  * the gain: a model trained on ranks from smaller problems sizes the sampling
    of a larger problem so that fewer compression attempts are needed than with
    the plain adaptive ID, at the same accuracy (GMRES within +-1 iteration of
    the oracle's count, true residual at the target).
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import mlp as omlp  # noqa: E402
from paper_1508_07798_amd import hss, rank_model  # noqa: E402
from workloads import configs  # noqa: E402

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_runs.json")))
DEV = "cuda"


def _params(w):
    """Flat library layout -> oracle parameter list (row-major [out, in])."""
    w = np.asarray(w, dtype=np.float64)
    out, off = [], 0
    for i in range(3):
        fi, fo = omlp.SIZES[i], omlp.SIZES[i + 1]
        out.append(w[off:off + fo * fi].reshape(fo, fi))
        off += fo * fi
        out.append(w[off:off + fo])
        off += fo
    assert off == hss.MLP_NPARAMS
    return out


def _flat(params):
    return np.concatenate([p.ravel() for p in params])


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, size=(n, 8)).astype(np.float32)
    t = (np.sin(X[:, 0] * 2.0) + X[:, 1] * X[:, 2] + 0.5 * X[:, 3]).astype(np.float32)
    return X, t


@pytest.mark.parametrize("n", [1, 37, 300])
def test_forward_and_gradient_match_oracle(n):
    print(f"mlp forward/grad n={n}", flush=True)
    w = rank_model.init_weights(seed=3)
    X, t = _data(n, seed=n)
    wd = torch.from_numpy(w).to(DEV)
    xd = torch.from_numpy(X).to(DEV)
    td = torch.from_numpy(t).to(DEV)
    y = hss.mlp_forward(wd, xd).cpu().numpy()
    params = _params(w)
    yo, _ = omlp.forward(params, X.astype(np.float64))
    assert np.max(np.abs(y - yo)) <= 1e-5 * max(1.0, np.max(np.abs(yo)))
    g, loss = hss.mlp_grad(wd, xd, td)
    lo, go = omlp.loss_and_grad(params, X.astype(np.float64), t.astype(np.float64))
    go = _flat(go)
    assert abs(loss - lo) <= 1e-5 * max(1.0, lo)
    assert np.max(np.abs(g.cpu().numpy() - go)) <= 1e-4 * np.max(np.abs(go))


def test_adam_training_follows_oracle():
    print("mlp adam trajectory", flush=True)
    steps, lr = 60, 1e-2
    w0 = rank_model.init_weights(seed=5)
    X, t = _data(200, seed=11)
    wd = torch.from_numpy(w0.copy()).to(DEV)
    hist = hss.mlp_train(wd, torch.from_numpy(X).to(DEV), torch.from_numpy(t).to(DEV), steps, lr=lr)
    hist = hist.cpu().numpy()
    params = _params(w0)
    state: dict = {}
    losses = []
    for _ in range(steps):
        lo, g = omlp.loss_and_grad(params, X.astype(np.float64), t.astype(np.float64))
        losses.append(lo)
        params = omlp.adam_step(params, g, state, lr=lr)
    losses = np.array(losses)
    assert losses[-1] < 0.5 * losses[0]
    assert np.max(np.abs(hist - losses) / losses) <= 2e-3
    assert np.max(np.abs(wd.cpu().numpy() - _flat(params))) <= 2e-3


def test_trained_model_reduces_compression_attempts():
    # the p = 4 family: its ranks (up to ~40 at 32 x 32 elements) exceed what the
    # plain method's first sample of 32 can certify, so the plain method grows
    # its samples where the model sizes them in advance
    print("rank model gain: train on p=4 n=16,24, apply to n=32", flush=True)
    train = [configs.make("helmholtz_p4_256", n=n, seed_offset=so) for so in (1, 2) for n in (16, 24)]
    X, K = rank_model.collect(train)
    w, hist = rank_model.train(X, K, steps=1500)
    assert hist[-1] < 0.1 * hist[0]
    P = configs.make("helmholtz_p4_256", n=32)
    vals = torch.from_numpy(P.op.vals).to(DEV)
    b = torch.from_numpy(np.ascontiguousarray(P.rhs[:, 0])).to(DEV)
    kh = P.kappa / P.op.n
    res = {}
    for name, model in (("plain", None), ("model", w)):
        h = hss.factor(P.op, P.tree, P.tol, prec="fp32", seed=P.seed, vals_dev=vals, kappa_h=kh,
                       rank_model=model)
        att = np.asarray(h.query("attempts"))
        err = np.asarray(h.query("err"))
        x, info = h.gmres(b, tol=P.gmres_tol, restart=P.restart)
        res[name] = (int(att.sum()), info[0]["iters"], info[0]["true_relres"], float(err.max()))
        h.close()
    print(res, flush=True)
    gold = GOLD["helmholtz_p4_256@32"]["iters"]
    for name in res:
        assert abs(res[name][1] - gold) <= 1
        assert res[name][2] <= P.gmres_tol
        assert res[name][3] <= P.tol
    assert res["model"][0] < res["plain"][0]
