"""The C ABI's boundary options on the GPU.

  * host buffers (on_device = 0) give the same apply and GMRES results as device
    buffers (to the last bits: split apply tiles add their partial sums with
    atomics, so the order of those additions varies between calls);
  * non-finite device values are refused with HSS_EINVAL and non-symmetric values
    with HSS_EUNSUPPORTED, before any factorization work;
  * the HSS leaf size option: FP64 factorizations with leaf sizes 2 and 7 match the
    oracle built with the same leaf size (ranks, apply element by element);
  * hss_rank_model_train writes a weights file that hss_factor reads through
    rank_model_path, with the same result as passing the weights directly.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.factor import OracleFactor  # noqa: E402
from paper_1508_07798_amd import hss, rank_model  # noqa: E402
from workloads import configs  # noqa: E402

DEV = "cuda"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def test_host_buffers_match_device_buffers():
    P = configs.make("helmholtz_p2_64", n=16)
    print("host buffers", flush=True)
    h = hss.factor(P.op, P.tree, P.tol, prec="fp32", seed=P.seed)
    b = np.ascontiguousarray(P.rhs[:, :2])
    yd = h.apply(_t(b)).cpu().numpy()
    yh = h.apply(b)
    assert np.linalg.norm(yd - yh) <= 1e-12 * np.linalg.norm(yd)
    xd, infd = h.gmres(_t(b), tol=P.gmres_tol)
    xh, infh = h.gmres(b, tol=P.gmres_tol)
    assert abs(infd[0]["iters"] - infh[0]["iters"]) <= 1
    A = P.op.to_scipy()
    for x in (xd.cpu().numpy(), xh):
        assert np.linalg.norm(b - A @ x) <= P.gmres_tol * 1.01 * np.linalg.norm(b)
    h.close()


def test_nonfinite_device_values_are_refused():
    P = configs.make("poisson_p1_16")
    print("nan on device", flush=True)
    v = P.op.vals.copy()
    v.reshape(-1)[123] = np.nan
    with pytest.raises(hss.HssError) as e:
        hss.factor(P.op, P.tree, P.tol, prec="fp64", seed=P.seed, vals_dev=_t(v))
    assert e.value.status == hss.HSS_EINVAL
    v.reshape(-1)[123] = np.inf
    with pytest.raises(hss.HssError) as e:
        hss.factor(P.op, P.tree, P.tol, prec="fp64", seed=P.seed, vals_dev=_t(v))
    assert e.value.status == hss.HSS_EINVAL


@pytest.mark.parametrize("on_device", [True, False])
def test_nonsymmetric_values_are_refused(on_device):
    P = configs.make("helmholtz_p2_64", n=16)
    print(f"nonsymmetric on_device={on_device}", flush=True)
    op = P.op
    # first off-diagonal block of element 0: A(0, f) for f != 0
    k = next(k for k in range(op.row_ptr[0], op.row_ptr[1]) if op.col_idx[k] != 0)
    v = op.vals.copy()
    v[k, 0, 1] += 1e-6 * np.abs(v).max()
    op2 = dataclasses.replace(op, vals=v)
    with pytest.raises(hss.HssError) as e:
        if on_device:
            hss.factor(op, P.tree, P.tol, prec="fp32", seed=P.seed, vals_dev=_t(v))
        else:
            hss.factor(op2, P.tree, P.tol, prec="fp32", seed=P.seed)
    assert e.value.status == hss.HSS_EUNSUPPORTED


@pytest.mark.parametrize("leaf", [2, 7])
def test_hss_leaf_size_matches_oracle(leaf):
    P = configs.make("poisson_p1_16")
    print(f"leaf size {leaf}", flush=True)
    h = hss.factor(P.op, P.tree, P.tol, prec="fp64", seed=P.seed, hss_leaf_elems=leaf)
    F = OracleFactor(P.op, P.tree, P.tol, seed=P.seed, hss_leaf_elems=leaf)
    heap = h.query("node_heap").astype(int)
    assert dict(zip(heap, h.query("ranks").astype(int))) == F.ranks()
    assert h.query("err").max() <= P.tol
    b = P.rhs[:, 0]
    y = h.apply(_t(b)).cpu().numpy()
    yr = F.apply(b)
    assert np.linalg.norm(y - yr) <= 1e-10 * np.linalg.norm(yr)
    h.close()


def test_rank_model_file_round_trip(tmp_path):
    P = configs.make("helmholtz_p2_64", n=24)
    print("rank model file", flush=True)
    X, K = rank_model.collect([P], prec="fp32")
    path = str(tmp_path / "rank.hssmlp")
    hss.rank_model_train(X, K, path, seed=3)
    raw = open(path, "rb").read()
    assert raw[:8] == b"HSSMLP01"
    assert int(np.frombuffer(raw[8:12], dtype=np.int32)[0]) == hss.MLP_NPARAMS
    w = np.frombuffer(raw[12:], dtype=np.float32)
    assert w.size == hss.MLP_NPARAMS and np.all(np.isfinite(w))
    Q = configs.make("helmholtz_p2_64", n=32)
    kh = Q.kappa / Q.op.n
    h1 = hss.factor(Q.op, Q.tree, Q.tol, prec="fp32", seed=Q.seed, kappa_h=kh, rank_model_path=path)
    h2 = hss.factor(Q.op, Q.tree, Q.tol, prec="fp32", seed=Q.seed, kappa_h=kh, rank_model=w.copy())
    assert np.array_equal(h1.query("l_init"), h2.query("l_init"))
    assert np.array_equal(h1.query("ranks"), h2.query("ranks"))
    assert h1.query("max_err")[0] <= Q.tol
    rng = np.random.default_rng(5)
    x = rng.standard_normal(Q.op.ndof) + 1j * rng.standard_normal(Q.op.ndof)
    y1, y2 = h1.apply(x), h2.apply(x)
    assert np.linalg.norm(y1 - y2) <= 1e-12 * np.linalg.norm(y1)
    h1.close()
    h2.close()
    with pytest.raises(hss.HssError) as e:
        hss.factor(Q.op, Q.tree, Q.tol, prec="fp32", seed=Q.seed, rank_model_path=str(tmp_path / "missing"))
    assert e.value.status == hss.HSS_EINVAL


@pytest.mark.parametrize("name,prec,box,tol_s", [("poisson_p1_16", "fp64", "leaf", 1e-12),
                                                 ("poisson_p1_16", "fp64", 2, 1e-10),
                                                 ("helmholtz_p2_64", "fp32", "leaf", 2e-5)])
def test_kept_schur_complement_matches_oracle(name, prec, box, tol_s):
    """One box's Schur complement S (symmetrized, before compression) and its
    compressed S~, kept by the handle (keep_box): S equals the oracle's S of the same
    box element by element (a leaf takes identical inputs; in FP64 a merge box too,
    since its children's S~ then agree), and ||S - S~||_F / ||S||_F recomputed on the
    host meets tol and equals the judge's figure for the box."""
    P = configs.make(name, n=16)
    heap = int(P.tree.leaf_node[0]) if box == "leaf" else box
    print(f"kept S {name} {prec} box {heap}", flush=True)
    kh = P.kappa / P.op.n if P.kappa else 0.0
    h = hss.factor(P.op, P.tree, P.tol, prec=prec, seed=P.seed, kappa_h=kh, keep_box=heap)
    S, St = h.kept_schur()
    F = OracleFactor(P.op, P.tree, P.tol, seed=P.seed)
    nf = F.nodes[heap]
    assert S.shape == nf.S.shape and S.shape[0] > 0
    assert np.linalg.norm(S - nf.S) <= tol_s * np.linalg.norm(nf.S)
    e = np.linalg.norm(S - St) / np.linalg.norm(S)
    assert e <= P.tol
    heaps = h.query("node_heap").astype(int)
    e_dev = float(h.query("err")[heaps == heap][0])
    assert abs(e - e_dev) <= 1e-3 * e_dev + 1e-12
    if prec == "fp64":
        assert np.linalg.norm(St - nf.S_tilde) <= 1e-8 * np.linalg.norm(nf.S_tilde)
    h.close()
    with pytest.raises(hss.HssError) as ex:
        hss.factor(P.op, P.tree, P.tol, prec=prec, seed=P.seed, keep_box=1 << 20)
    assert ex.value.status == hss.HSS_EINVAL
    with pytest.raises(hss.HssError) as ex:
        hss.factor(P.op, P.tree, P.tol, prec=prec, seed=P.seed, ldu=3)
    assert ex.value.status == hss.HSS_EINVAL
    with pytest.raises(hss.HssError) as ex:
        hss.factor(P.op, P.tree, P.tol, prec=prec, seed=P.seed, model_margin=0.5)
    assert ex.value.status == hss.HSS_EINVAL
