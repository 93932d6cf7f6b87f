"""The GPU reverse mode against central finite differences of the GPU
forward pass itself (no oracle involved): the differentiable refinement
through a two-level hierarchy, every level with learnable log-weights,
loss = <G, Z_0>.  Directional derivatives: along a random direction v of the
coarse embedding (the refinement is linear in it, so a unit step has no
truncation error) and along a random direction u of each level's
log-weights (step 1e-2, second-order accurate).  Measured agreement: about
1e-7 relative along v and 1e-4 along u; the bounds are 1e-5 and 1e-3, and
each directional derivative must be well away from zero."""
import numpy as np
import pytest

from tests.cases import random_hypergraph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_09660_amd as H
    return H


@pytest.mark.parametrize("order", ["jacobi", "edge_first"])
def test_directional_finite_differences(H, order):
    import torch
    hg = random_hypergraph(77, 2000, 1200, 1, 10, weighted=False)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 1)
    L = hier.n_levels - 1
    assert L == 1
    d, K, omega = 16, 3, 0.5
    plan = H.Plan(hier, d, "f32", options={"order": order})
    rng = np.random.default_rng(77)
    zc0 = torch.as_tensor(rng.standard_normal((hier.levels[L].rows, d)).astype(np.float32)).cuda()
    th0 = [torch.as_tensor(rng.uniform(-0.5, 0.5, lv.n_edges).astype(np.float32)).cuda() for lv in hier.levels]
    G = torch.as_tensor(rng.standard_normal((hier.levels[0].rows, d))).cuda()

    def loss(zc, ths):
        z = H.refine_hierarchy(zc, ths, plan, [K] * (L + 1), omega, ckpt_every=2)
        return (z.double() * G).sum()

    zc = zc0.clone().requires_grad_(True)
    ths = [t.clone().requires_grad_(True) for t in th0]
    loss(zc, ths).backward()
    gz = zc.grad.double()
    gth = [t.grad.double() for t in ths]

    with torch.no_grad():
        v = torch.as_tensor(rng.standard_normal(zc0.shape).astype(np.float32)).cuda()
        fd = (loss(zc0 + v, th0) - loss(zc0 - v, th0)).item() / 2.0
        an = float((gz * v.double()).sum())
        print("dL/dZc along v:", fd, an, flush=True)
        assert abs(an) > 1.0 and abs(fd - an) <= 1e-5 * abs(an), ("dL/dZc", fd, an)
        h = 1e-2
        for l in range(L + 1):
            u = torch.as_tensor(rng.standard_normal(th0[l].shape).astype(np.float32)).cuda()
            tp = [t.clone() for t in th0]
            tm = [t.clone() for t in th0]
            tp[l] += h * u
            tm[l] -= h * u
            # the steps as stored in float32 (the weights' storage type)
            step_p, step_m = (tp[l] - th0[l]).double(), (th0[l] - tm[l]).double()
            fd = (loss(zc0, tp) - loss(zc0, tm)).item()
            an = float((gth[l] * (step_p + step_m)).sum())
            print(f"dL/dtheta level {l} along u:", fd, an, flush=True)
            assert abs(an) > 1e-2 and abs(fd - an) <= 1e-3 * abs(an), (f"dL/dtheta level {l}", fd, an)
