"""The allocation-free MLP gradient (hss_mlp_grad_noalloc) against hss_mlp_grad:
two calls in a row, the second on fewer samples, through the C ABI; sizes above
the fixed array's limit are rejected."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1508_07798_amd import hss, rank_model  # noqa: E402


def test_noalloc_gradient_matches_allocating_entry_point():
    rng = np.random.default_rng(41)
    w = torch.from_numpy(rank_model.init_weights(4)).cuda()
    for n in (3000, 257):
        print(f"noalloc grad n={n}", flush=True)
        x = torch.from_numpy(rng.standard_normal((n, 8)).astype(np.float32)).cuda()
        t = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda()
        g_ref, l_ref = hss.mlp_grad(w, x, t)
        g = torch.full((hss.MLP_NPARAMS,), float("nan"), dtype=torch.float32, device="cuda")
        loss = hss.mlp_grad_noalloc(w, x, t, g)
        torch.cuda.synchronize()
        # the same kernels on the same inputs: identical results
        assert torch.equal(g, g_ref), n
        assert loss == l_ref, n


def test_noalloc_gradient_rejects_too_many_samples():
    n = hss.MLP_NOALLOC_MAX_N + 1
    w = torch.from_numpy(rank_model.init_weights(4)).cuda()
    x = torch.zeros((n, 8), dtype=torch.float32, device="cuda")
    t = torch.zeros(n, dtype=torch.float32, device="cuda")
    g = torch.zeros(hss.MLP_NPARAMS, dtype=torch.float32, device="cuda")
    with pytest.raises(hss.HssError) as e:
        hss.mlp_grad_noalloc(w, x, t, g)
    assert e.value.status == hss.HSS_EINVAL
