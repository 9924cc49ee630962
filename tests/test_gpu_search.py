"""Tree search (Alg. 1) on GPU-evaluated successors against the oracle's searches:
same optimum and same chosen goal for the plain modes (exhaustive, uniform-cost),
the w-suboptimality bound for the focal mode (Theorem 2), budgets."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Oracle  # noqa: E402
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


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_plain_searches_match_oracle_on_pose_subsets(k):
    sc = H.c1_scene(k)
    sub = scenes.pose_subset_around(sc, 2, yaw_stride=2)
    o = Oracle.from_scene(sc, nthreads=NTH)
    ctx = perch.context_from_scene(sc)
    ex_o = o.search_exhaustive(sub)
    ex_g = ctx.search(perch.SEARCH_EXHAUSTIVE, pose_subset=sub)
    assert ex_g["found"] and ex_g["cost"] == ex_o["cost"]
    assert ex_g["canonical"] == _canon(ex_o["mesh"], ex_o["pose"])
    assert ex_g["n_evaluated"] == ex_o["n_eval"]
    assert sum(ex_g["edge_cost"]) == ex_g["cost"]
    uc_o = o.search_ucs(sub)
    uc_g = ctx.search(perch.SEARCH_UCS, pose_subset=sub)
    assert uc_g["cost"] == uc_o["cost"] == ex_o["cost"]
    assert uc_g["canonical"] == _canon(uc_o["mesh"], uc_o["pose"])
    assert uc_g["n_expanded"] == uc_o["n_expanded"]


def test_exhaustive_full_grid_160x120():
    """The whole config-1 tree (2 x 1,152 + 2 x 1,152 x 1,152 evaluations)."""
    sc = H.c1_scene(0)
    ctx = perch.context_from_scene(sc)
    ex = ctx.search(perch.SEARCH_EXHAUSTIVE)
    P = sc.grid.P
    assert ex["found"]
    # the root has no occluder, so all 2P level-1 children are valid and expanded
    assert ex["n_expanded"] == 1 + 2 * P
    assert ex["n_evaluated"] == 2 * P + 2 * P * P
    uc = ctx.search(perch.SEARCH_UCS)
    assert uc["cost"] == ex["cost"]
    o = Oracle.from_scene(sc, nthreads=NTH)
    uc_o = o.search_ucs()
    assert uc_o["cost"] == ex["cost"]
    assert uc["canonical"] == _canon(uc_o["mesh"], uc_o["pose"])
    # the optimum found is the ground truth up to the object symmetries: its
    # one-shot cost is the optimum
    r = o.jtree([m for m, _ in ex["canonical"]], [p for _, p in ex["canonical"]])
    assert r["J_tree"] == ex["cost"]


@pytest.mark.parametrize("w", [1.0, 1.5, 3.0])
def test_focal_cost_within_w_of_optimum(w):
    sc = H.c1_scene(4)
    ctx = perch.context_from_scene(sc)
    opt = ctx.search(perch.SEARCH_UCS)["cost"]
    f = ctx.search(perch.SEARCH_FOCAL, w=w)
    assert f["found"] and f["cost"] <= w * opt + 1e-9
    a = ctx.search(perch.SEARCH_FOCAL, w=w, anytime=True)
    assert a["cost"] == opt and a["t_best_s"] <= a["t_total_s"]


def test_budget_returns_incumbent_status():
    sc = H.c1_scene(5)
    ctx = perch.context_from_scene(sc)
    r = ctx.search(perch.SEARCH_UCS, budget_expansions=1)
    assert r["budget_exhausted"] and r["n_expanded"] == 1


@pytest.mark.parametrize("w", [1.0, 1.5, 3.0])
def test_multi_heuristic_cost_within_w_of_optimum(w):
    """Focal-MHA* with the paper's two inadmissible heuristics (h_depth, h_overlap):
    the first goal costs at most w * OPT (Theorem 2); run anytime it returns OPT."""
    sc = H.c1_scene(6)
    ctx = perch.context_from_scene(sc)
    opt = ctx.search(perch.SEARCH_UCS)["cost"]
    f = ctx.search(perch.SEARCH_MHA, w=w)
    assert f["found"] and f["cost"] <= w * opt + 1e-9
    a = ctx.search(perch.SEARCH_MHA, w=w, anytime=True)
    assert a["cost"] == opt and a["lower_bound"] >= opt


def test_multi_heuristic_on_pose_subsets_matches_oracle_optimum():
    sc = H.c2_scene(0)
    sub = scenes.pose_subset_around(sc, 2, yaw_stride=4)
    o = Oracle.from_scene(sc, nthreads=NTH)
    ctx = perch.context_from_scene(sc)
    opt = o.search_ucs(sub)["cost"]
    a = ctx.search(perch.SEARCH_MHA, w=3.0, anytime=True, pose_subset=sub)
    assert a["found"] and a["cost"] == opt
    f = ctx.search(perch.SEARCH_MHA, w=3.0, pose_subset=sub)
    assert f["cost"] <= 3.0 * opt


@pytest.mark.parametrize("w", [1.0, 2.0])
def test_pose_prior_queue_keeps_the_w_bound(w):
    """A third inadmissible queue on the pose-prior heuristic (Sec. IV-C), with
    estimates that are right (the true poses) or wrong (shifted across the
    table): Theorem 2's bound holds whatever the estimates say."""
    sc = H.c1_scene(2)
    sub = scenes.pose_subset_around(sc, 2, yaw_stride=2)
    opt = Oracle.from_scene(sc, nthreads=NTH).search_exhaustive(sub)["cost"]
    ctx = perch.context_from_scene(sc)
    true = [(int(m), float(sc.poses[p, 0]), float(sc.poses[p, 1]),
             float(np.arctan2(sc.poses[p, 3], sc.poses[p, 2])))
            for m, p in zip(sc.obj_mesh, sc.gt_pose)]
    wrong = [(m, -x, -y, th + 1.0) for (m, x, y, th) in true]
    for pri in (true, wrong):
        r = ctx.search(perch.SEARCH_MHA, w=w, pose_subset=sub, priors=pri)
        assert r["found"] and r["cost"] <= w * opt + 1e-9
        assert sum(r["edge_cost"]) == r["cost"]
        a = ctx.search(perch.SEARCH_MHA, w=w, anytime=True, pose_subset=sub, priors=pri)
        assert a["cost"] == opt and a["lower_bound"] >= a["cost"]
    with pytest.raises(perch.PerchError):  # a queue of the multi-heuristic search only
        ctx.search(perch.SEARCH_FOCAL, w=w, pose_subset=sub, priors=true)


def test_search_log_records_each_search(tmp_path, monkeypatch):
    """PERCH_SEARCH_LOG: one JSON line per search with its options and outcome."""
    import json

    path = tmp_path / "searches.jsonl"
    monkeypatch.setenv("PERCH_SEARCH_LOG", str(path))
    sc = H.c1_scene(0)
    ctx = perch.context_from_scene(sc)
    sub = scenes.pose_subset_around(sc, 2, yaw_stride=2)
    r1 = ctx.search(perch.SEARCH_UCS, pose_subset=sub)
    r2 = ctx.search(perch.SEARCH_FOCAL, w=3.0, anytime=True, pose_subset=sub)
    monkeypatch.delenv("PERCH_SEARCH_LOG")
    ctx.search(perch.SEARCH_UCS, pose_subset=sub)  # not logged
    rows = [json.loads(line) for line in path.read_text().splitlines()]
    assert len(rows) == 2
    for row, r, mode in zip(rows, (r1, r2), (perch.SEARCH_UCS, perch.SEARCH_FOCAL)):
        assert row["mode"] == mode and row["found"] == int(r["found"])
        assert row["cost"] == r["cost"] and row["n_evaluated"] == r["n_evaluated"]
        assert row["n_expanded"] == r["n_expanded"] and row["lower_bound"] == r["lower_bound"]
        assert [tuple(o[:2]) for o in row["objs"]] == [tuple(o) for o in r["objs"]]
        assert sum(o[2] for o in row["objs"]) == r["cost"]
        assert len(row["trace"]) == len(r["trace"])
    assert rows[1]["w"] == 3.0 and rows[1]["anytime"] == 1
