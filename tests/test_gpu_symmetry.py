"""Searches with rotationally symmetric objects (tried once per (x, y), Sec. V-A)
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
