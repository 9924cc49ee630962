"""Searches with rotationally symmetric objects (tried once per (x, y), Sec. IV-E)
and with replicated instances (one mesh id several times in the multiset),
GPU-evaluated through the C ABI, against the oracle's searches under the same
rules: same optimum, same goal, same evaluation counts."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Oracle, render_fn  # noqa: E402
from paper_1510_05613_amd import perch, scenes  # noqa: E402
from tests import helpers as H  # noqa: E402

NTH = max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    perch.load()


def _canon(mesh, pose):
    return sorted((int(m), int(p)) for m, p in zip(mesh, pose))


def _compare(sc, o, ctx, sub):
    ex_o = o.search_exhaustive(sub)
    ex_g = ctx.search(perch.SEARCH_EXHAUSTIVE, pose_subset=sub)
    assert ex_g["found"] and ex_g["cost"] == ex_o["cost"]
    assert ex_g["canonical"] == _canon(ex_o["mesh"], ex_o["pose"])
    assert ex_g["n_evaluated"] == ex_o["n_eval"]
    uc_o = o.search_ucs(sub)
    uc_g = ctx.search(perch.SEARCH_UCS, pose_subset=sub)
    assert uc_g["cost"] == uc_o["cost"] == ex_o["cost"]
    assert uc_g["canonical"] == _canon(uc_o["mesh"], uc_o["pose"])
    assert uc_g["n_expanded"] == uc_o["n_expanded"]
    return ex_g, uc_g


@pytest.mark.parametrize("k", [0, 1])
def test_symmetric_mesh_matches_oracle(k):
    sc = H.c1_scene(k)
    sub = scenes.pose_subset_around(sc, 2, yaw_stride=1)
    o = Oracle.from_scene(sc, nthreads=NTH)
    ctx = perch.context_from_scene(sc)
    plain = ctx.search(perch.SEARCH_EXHAUSTIVE, pose_subset=sub)
    for m in sc.obj_mesh:
        o.set_symmetric(int(m))
        ctx.set_symmetric(int(m))
    ex_g, _ = _compare(sc, o, ctx, sub)
    # one pose per (x, y) for every mesh: n_yaw times fewer level-1 children
    assert ex_g["n_evaluated"] < plain["n_evaluated"]
    focal = ctx.search(perch.SEARCH_FOCAL, w=2.0, pose_subset=sub)
    assert focal["cost"] <= 2.0 * ex_g["cost"]
    with pytest.raises(perch.PerchError):
        ctx.search(perch.SEARCH_LEARNED, w=2.0, pose_subset=sub)


@pytest.mark.parametrize("idx", [0, 1])
def test_replicated_instances_match_oracle(idx):
    lib = H.c1_library()
    one = scenes.Library([lib.meshes[2]])
    sc = scenes.make_scene(1, 200 + idx, render_fn, one, overrides=dict(K=(2, 2)))
    assert sc.obj_mesh[0] == sc.obj_mesh[1]
    sub = scenes.pose_subset_around(sc, 1, yaw_stride=2)
    o = Oracle.from_scene(sc, nthreads=NTH)
    ctx = perch.context_from_scene(sc)
    ex_g, uc_g = _compare(sc, o, ctx, sub)
    assert uc_g["n_evaluated"] <= ex_g["n_evaluated"]


@pytest.fixture(scope="module")
def board():
    return scenes.chessboard_scene(render_fn, 0)


def test_twelve_object_parent_matches_oracle(board):
    """Successors under an 11-object parent (more objects than a state held before
    the limit was raised): every pose of the last piece's mesh, against the oracle."""
    from tests.test_gpu_parity import compare

    sc = board
    order = [int(k) for k in sc.gt_order]
    parent = [(int(sc.obj_mesh[k]), int(sc.gt_pose[k])) for k in order[:-1]]
    last = order[-1]
    m = int(sc.obj_mesh[last])
    cands = np.stack([np.full(sc.grid.P, m, np.int32), np.arange(sc.grid.P, dtype=np.int32)], 1)
    ctx = perch.context_from_scene(sc)
    st, cost, comps = ctx.evaluate(parent, torch.as_tensor(cands).cuda())
    torch.cuda.synchronize()
    o = Oracle.from_scene(sc, nthreads=NTH)
    ref = o.eval([p[0] for p in parent], [p[1] for p in parent], cands[:, 0], cands[:, 1])
    r = compare((st.cpu().numpy(), cost.cpu().numpy(), comps.cpu().numpy()), ref, "12 objects")
    assert r["valid"] > 0
    # the true pose completes the scene at its one-shot cost
    k = int(np.nonzero(cands[:, 1] == sc.gt_pose[last])[0][0])
    assert int(st[k]) == 1


def test_chessboard_search_within_w(board):
    """The twelve-piece stand-in with the paper's w = 15: Focal-MHA* returns a goal
    within w of the lower bound it proves, with symmetric pawns and kings placed at
    yaw 0 only and the replicated pieces searched as sets."""
    sc = board
    ctx = perch.context_from_scene(sc)
    ctx.set_symmetric(0)
    ctx.set_symmetric(2)
    r = ctx.search(perch.SEARCH_MHA, w=15.0, budget_s=60.0)
    assert r["found"] and not r["budget_exhausted"]
    assert r["cost"] <= 15.0 * r["lower_bound"] + 1e-9 or r["cost"] == 0
    assert sum(r["edge_cost"]) == r["cost"] and len(r["objs"]) == 12
    assert sorted(m for m, _ in r["objs"]) == sorted(int(v) for v in sc.obj_mesh)
    for m, p in r["objs"]:
        if m in (0, 2):
            assert sc.grid.unindex(p)[2] == 0
