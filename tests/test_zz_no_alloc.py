"""perch_eval_successors_noalloc (the allocation-free entry point) against
perch_eval_successors through the C ABI: the same kernels on the same inputs, so
status, cost and components must agree bit for bit.  Two calls in a row share the
library's fixed per-GPU array; the second is smaller (a 160 x 120 scene after a
640 x 480 one, and fewer successors), so stale contents of the first call would
show.  Also: sizes beyond the limit and call-order errors are refused before any
work."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1510_05613_amd import perch  # noqa: E402
from tests import helpers as H  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    perch.load()


def _cands(mesh, pose):
    c = np.stack([np.asarray(mesh, np.int32), np.asarray(pose, np.int32)], 1)
    return torch.as_tensor(np.ascontiguousarray(c)).cuda()


def _run(ctx, fn, parent, cands):
    n = cands.shape[0]
    cost = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    status = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    comps = torch.full((n, 5), -7, dtype=torch.int32, device="cuda")
    fn(parent, cands, cost, status, comps)
    torch.cuda.synchronize()
    return status.cpu().numpy(), cost.cpu().numpy(), comps.cpu().numpy()


def _goal_case(sc, n, seed):
    """Goal-level successors (the set U is used) under the true prefix."""
    rng = np.random.default_rng(seed)
    order = list(sc.gt_order)
    parent = [(int(sc.obj_mesh[o]), int(sc.gt_pose[o])) for o in order[:-1]]
    m = int(sc.obj_mesh[order[-1]])
    ps = rng.choice(sc.grid.P, size=n, replace=False)
    ps[0] = int(sc.gt_pose[order[-1]])
    return parent, _cands(np.full(n, m), ps)


def test_noalloc_matches_eval_successors_twice_second_smaller():
    big = H.c2_scene(0)
    small = H.c1_scene(1)
    ctx_big = perch.context_from_scene(big)
    ctx_small = perch.context_from_scene(small)
    cases = [(ctx_big, *_goal_case(big, 3000, 1)), (ctx_small, *_goal_case(small, 400, 2))]
    # the reference entry point first on both contexts (this also uploads the meshes)
    ref = [_run(c, c.eval_successors, par, cd) for c, par, cd in cases]
    for (c, par, cd), r in zip(cases, ref):
        got = _run(c, c.eval_successors_noalloc, par, cd)
        for a, b, name in zip(got, r, ("status", "cost", "comps")):
            assert np.array_equal(a, b), name
        assert (r[0] == 1).sum() > 0
    # the first case again after the smaller one: nothing stale in the shared array
    c, par, cd = cases[0]
    got = _run(c, c.eval_successors_noalloc, par, cd)
    for a, b in zip(got, ref[0]):
        assert np.array_equal(a, b)
    # at the root (no parent) and below the goal level (no U; K = 3 at 640 x 480)
    first = big.gt_order[0]
    ps = np.arange(0, big.grid.P, 97)
    for parent in ([], [(int(big.obj_mesh[first]), int(big.gt_pose[first]))]):
        cd = _cands(np.full(len(ps), int(big.obj_mesh[big.gt_order[1]])), ps)
        a = _run(ctx_big, ctx_big.eval_successors_noalloc, parent, cd)
        b = _run(ctx_big, ctx_big.eval_successors, parent, cd)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_noalloc_refuses_before_any_work():
    sc = H.c1_scene(0)
    ctx = perch.context_from_scene(sc)
    cd = _cands([0], [0])
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    # the mesh library was never uploaded by an allocating call
    with pytest.raises(perch.PerchError, match="not uploaded"):
        ctx.eval_successors_noalloc([], cd, out, out)
    ctx.render([(0, 0)])  # uploads the library
    with pytest.raises(perch.PerchError, match="bad parent"):
        ctx.eval_successors_noalloc([(0, 0)] * 5, cd, out, out)
    # an image beyond the fixed array's 1,048,576 pixels
    big = H.down_camera(W=2048, H=1024, cx=1023.5, cy=511.5)
    ctx2 = perch.Context(big)
    with pytest.raises(perch.PerchError, match="allocation-free limit"):
        ctx2.eval_successors_noalloc([], cd, out, out)
