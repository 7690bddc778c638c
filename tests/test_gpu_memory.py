"""The workspace model (Eq. (10)-(12) adapted to the library's buffers)
against what a context actually holds on the GPU.

* The model's prediction (kmeans_workspace_bytes, leaf and group counts
  estimated with cells half full) is within 4% of the bytes the context
  allocated (the paper reports its estimate within 3% of the measured
  memory).  The drop in free device memory that hipMemGetInfo shows across
  kmeans_init is at least those bytes and at most one runtime page (2 MiB)
  more per allocation; at 1e7 points it is within 5% of them.
* With the actual leaf and group counts the model is exact.
* A budget picks the smallest leaf size whose modelled workspace fits, and
  the context then stays within the budget.
"""

import sys

import numpy as np
import pytest

from synth import batched_clouds, make_config

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ekm():
    import torch
    import paper_2412_02244_amd as m
    m.load_library()
    assert torch.cuda.is_available()
    return m


def _free():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


PAGE = 2 << 20  # the runtime's device allocation granularity


@pytest.fixture(scope="module", autouse=True)
def warm(ekm):
    """A first context loads the code objects and the runtime's own pools."""
    import torch
    x = torch.rand(100_000, 2, device="cuda")
    ekm.kmeans_init(x, 100).close()
    torch.cuda.synchronize()


def _check(ekm, name, make_ctx, predicted, rel_used=None):
    import torch
    torch.cuda.empty_cache()
    before = _free()
    ctx = make_ctx()
    after = _free()
    info = ekm.kmeans_context_info(ctx)
    used = before - after
    ctx.close()
    _say(f"{name}: model {predicted / 2**20:.2f} MiB, context {info['device_bytes'] / 2**20:.2f} MiB, "
         f"hipMemGetInfo {used / 2**20:.2f} MiB, leaves {info['leaves']} groups {info['groups']} f {info['leaf_size']}")
    assert info["model_bytes"] == predicted
    assert info["model_bytes_actual_counts"] == info["device_bytes"]
    # two arenas (index build; the rest) and the statistics rows, plus the
    # group buffers with cell leaves, the brute path's statistics rows
    assert info["allocations"] <= 7
    assert abs(predicted - info["device_bytes"]) <= 0.04 * info["device_bytes"]
    assert info["device_bytes"] - PAGE <= used <= info["device_bytes"] + PAGE * info["allocations"]
    if rel_used is not None:
        assert abs(used - info["device_bytes"]) <= rel_used * info["device_bytes"]
    return info


@pytest.mark.parametrize("leaf_size", [64, 32, 16])
def test_model_matches_geo2d_1e6(ekm, leaf_size):
    import torch
    x, c0, _ = make_config(1)
    xt = torch.from_numpy(x).cuda()
    pred = ekm.kmeans_workspace_bytes(x.shape[0], c0.shape[0], 2, leaf_size=leaf_size)
    _check(ekm, f"geo2d 1e6 k=1000 f={leaf_size}", lambda: ekm.kmeans_init(xt, c0.shape[0], leaf_size=leaf_size),
           pred)


def test_model_matches_surfaces3d_1e7(ekm):
    import torch
    x, _, _ = make_config(2)
    xt = torch.from_numpy(x).cuda()
    for k in (10_000, 100_000):
        pred = ekm.kmeans_workspace_bytes(x.shape[0], k, 3)
        _check(ekm, f"surfaces3d 1e7 k={k}", lambda: ekm.kmeans_init(xt, k), pred, rel_used=0.05)


def test_model_matches_brute_and_batched(ekm):
    import torch
    x, c0, _ = make_config(1)
    xt = torch.from_numpy(x).cuda()
    pred = ekm.kmeans_workspace_bytes(x.shape[0], c0.shape[0], 2, algo=ekm.KM_BRUTE)
    _check(ekm, "geo2d brute", lambda: ekm.kmeans_init(xt, c0.shape[0], algo=ekm.KM_BRUTE), pred)
    xb, po, cb, co = batched_clouds(n_clouds=256, seed=1203, init_seed=2203)
    xbt = torch.from_numpy(xb).cuda()
    ctx = ekm.kmeans_init_batched(xbt, po, co)
    info = ekm.kmeans_context_info(ctx)
    ctx.close()
    _say(f"batched 256: model {info['model_bytes'] / 2**20:.2f} MiB, context {info['device_bytes'] / 2**20:.2f} MiB")
    assert info["model_bytes_actual_counts"] == info["device_bytes"]
    assert abs(info["model_bytes"] - info["device_bytes"]) <= 0.04 * info["device_bytes"]


def test_budget_chooses_leaf_size(ekm):
    import torch
    x, c0, _ = make_config(1)
    n, k = x.shape[0], c0.shape[0]
    xt = torch.from_numpy(x).cuda()
    m = {f: ekm.kmeans_workspace_bytes(n, k, 2, leaf_size=f) for f in (8, 16, 32, 64)}
    for f, limit in ((32, m[32] + (m[16] - m[32]) // 2), (64, m[64] + (m[32] - m[64]) // 2)):
        ctx = ekm.kmeans_init(xt, k, workspace_limit_bytes=limit)
        info = ekm.kmeans_context_info(ctx)
        # the run is still exact: a few steps against the oracle
        c = torch.from_numpy(c0).cuda()
        ekm.kmeans_run(ctx, c, 3)
        ctx.close()
        _say(f"budget {limit / 2**20:.2f} MiB: f {info['leaf_size']}, context {info['device_bytes'] / 2**20:.2f} MiB")
        assert info["leaf_size"] == f
        assert info["device_bytes"] <= limit
        import oracle
        ref = oracle.lloyd(x, c0, max_iter=3, history=False)
        np.testing.assert_array_equal(c.cpu().numpy(), ref["c"])
    with pytest.raises(ekm.EKMError):
        ekm.kmeans_init(xt, k, workspace_limit_bytes=m[64] // 2)
