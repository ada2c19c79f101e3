"""Host-side checks of the C-ABI library (no GPU needed).

  * libhss.so loads and exports every function the headers declare;
  * the host planner's interior / boundary sets, orderings and HSS trees equal
    the oracle's, independently computed, on several workloads;
  * argument validation returns the documented status codes.
"""
import os
import re

import numpy as np
import pytest

from oracle.sets import TreeSets, hss_postorder
from paper_1508_07798_amd import hss
from workloads import configs, partition, sipg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in ("hss.h", "hss_debug.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        names += re.findall(r"^\s*(?:hss_status_t|void|const char\s*\*)\s*\*?\s*(\w+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_exports_every_declared_symbol():
    L = hss.lib()
    names = _declared()
    assert len(names) >= 16
    for n in names:
        assert hasattr(L, n), n


def _check_plan(op, tree, leaf=4):
    pl = hss.Plan(op, tree, hss_leaf_elems=leaf)
    T = TreeSets(op.row_ptr, op.col_idx, op.q, tree, hss_leaf_elems=leaf)
    for s in T.nodes:
        ns = T.sets[s]
        assert np.array_equal(pl.query("idof", s), ns.idof), s
        assert np.array_equal(pl.query("bdof", s), ns.bdof), s
        assert int(pl.query("height", s)[0]) == T.height[s]
        q4 = pl.query("hss", s).reshape(-1, 4)
        ref = hss_postorder(ns.hss)
        assert q4.shape[0] == len(ref)
        for row, t in zip(q4, ref):
            assert (row[0], row[1]) == (t.lo, t.hi)
            assert (row[2] < 0) == t.is_leaf
    assert np.array_equal(pl.query("root"), T.root_idof)
    pl.close()


@pytest.mark.parametrize("n,p,pde,scheme", [(16, 1, "poisson", "boxes"), (32, 2, "helmholtz", "boxes"),
                                             (21, 1, "poisson", "boxes"), (16, 1, "poisson", "hslabs"),
                                             (12, 3, "poisson", "vslabs")])
def test_planner_matches_oracle(n, p, pde, scheme):
    op = sipg.assemble(n, p, pde, kappa=10.0)
    tree = partition.build_tree(n, n, 16, scheme=scheme)
    _check_plan(op, tree)


@pytest.mark.parametrize("leaf", [1, 2, 7])
def test_planner_hss_leaf_size_matches_oracle(leaf):
    op = sipg.assemble(24, 2, "helmholtz", kappa=10.0)
    tree = partition.build_tree(24, 24, 16)
    _check_plan(op, tree, leaf)


def test_planner_full_helmholtz_workload():
    P = configs.make("helmholtz_p2_64")
    _check_plan(P.op, P.tree)


def test_bad_inputs_are_rejected():
    P = configs.make("poisson_p1_16", n=8)
    # an element in no leaf
    t = partition.build_tree(8, 8, 16)
    t.leaf_ptr = t.leaf_ptr.copy()
    t.leaf_ptr[-1] -= 1
    with pytest.raises(hss.HssError) as e:
        hss.Plan(P.op, t)
    assert e.value.status == hss.HSS_EINVAL
    # a structurally nonsymmetric operator
    op = sipg.assemble(8, 1)
    rp, ci = op.row_ptr.copy(), op.col_idx.copy()
    keep = [c for c in range(rp[0], rp[1]) if ci[c] != 0]   # drop a coupling of row 0
    drop = next(c for c in range(rp[0], rp[1]) if ci[c] != 0)
    mask = np.ones(ci.size, bool)
    mask[drop] = False
    op2 = sipg.BlockOperator(op.n, op.p, op.q, np.concatenate([[0], np.cumsum([
        rp[e + 1] - rp[e] - (1 if e == 0 else 0) for e in range(op.n_el)])]).astype(np.int32),
        ci[mask], op.vals[mask], op.h)
    with pytest.raises(hss.HssError) as e:
        hss.Plan(op2, P.tree)
    assert e.value.status == hss.HSS_EUNSUPPORTED
    del keep


def test_factor_without_gpu_or_with_nan_fails_cleanly():
    P = configs.make("poisson_p1_16", n=8)
    op = sipg.assemble(8, 1)
    op.vals = op.vals.copy()
    op.vals[3, 1, 1] = np.nan
    with pytest.raises(hss.HssError) as e:
        hss.factor(op, P.tree, 1e-6, stream=0)
    assert e.value.status == hss.HSS_EINVAL
    with pytest.raises(hss.HssError) as e:
        hss.factor(P.op, P.tree, -1.0, stream=0)
    assert e.value.status == hss.HSS_EINVAL


def test_tuning_table_io(tmp_path):
    """The tuning table: compiled shapes per class, the JSON reader, and the checks."""
    import json
    c = hss.tuning_candidates("complex64", 1024)
    assert (16, 4, 256) in c and all(r * t >= 1024 for _, r, t in c)
    assert (8, 4, 256) in hss.tuning_candidates("complex128", 1000)
    assert hss.tuning_candidates("complex64", 3000) == []
    assert (16, 8, 512) in hss.tuning_candidates("float32", 4096)
    good = tmp_path / "t.json"
    good.write_text(json.dumps({"arch": "gfx950", "entries": [
        {"scalar": "complex64", "rows": 1024, "nb": 16, "rpt": 4, "nt": 256, "block": 128, "ms": 1.5,
         "tried": [{"nb": 16, "ms": 2.0}]},
        {"scalar": "float64", "rows": 128, "nb": 0, "rpt": 0, "nt": 0, "block": -1}]}))
    hss.tuning_load(str(good))
    for text in ('{"entries": [{"scalar": "complex64", "rows": 1000}]}',   # not a size class
                 '{"entries": [{"scalar": "int8", "rows": 128}]}',         # not a scalar type
                 '{"entries": [{"scalar": "float32", "rows": 128}'):        # truncated
        bad = tmp_path / "b.json"
        bad.write_text(text)
        with pytest.raises(hss.HssError) as e:
            hss.tuning_load(str(bad))
        assert e.value.status == hss.HSS_EINVAL
    with pytest.raises(hss.HssError):
        hss.tuning_set("float32", 100, 16, 1, 128, 0)
    with pytest.raises(hss.HssError):
        hss.tuning_load(str(tmp_path / "missing.json"))
    hss.tuning_clear()
