"""Host-side logic of the learned heuristic's data pipeline (no GPU): which
parents and pose cells are labelled."""
import numpy as np

from paper_1510_05613_amd import learn, scenes
from oracle import render_fn


def _scene():
    return scenes.make_scene(2, 1, render_fn, scenes.make_library("c2"))


def test_prefixes_follow_a_valid_order():
    sc = _scene()
    pre = learn.gt_prefixes(sc)
    assert pre[0] == [] and len(pre) == sc.K
    for j, p in enumerate(pre):
        assert p == [(int(sc.obj_mesh[k]), int(sc.gt_pose[k])) for k in sc.gt_order[:j]]
        left = learn.remaining_meshes(sc, p)
        assert sorted(left) == sorted(set(int(sc.obj_mesh[k]) for k in sc.gt_order[j:]))


def test_sampled_cells_hold_the_true_poses():
    sc = _scene()
    g = sc.grid
    rng = np.random.default_rng(0)
    for p in learn.gt_prefixes(sc):
        cells = learn.sample_cells(sc, p, 256, rng)
        assert cells is not None and len(cells) == 256
        assert np.all(np.diff(cells) > 0) and cells.min() >= 0 and cells.max() < g.nx * g.ny
        placed = {q for _, q in p}
        for k in range(sc.K):
            if int(sc.gt_pose[k]) not in placed:
                assert int(sc.gt_pose[k]) // g.n_yaw in set(cells.tolist())
    # a grid that fits takes every cell
    assert learn.sample_cells(sc, [], g.nx * g.ny, rng) is None


def test_cell_centres_are_the_pose_table_positions():
    g = scenes.make_grid(scenes.CONFIGS[4])
    xy = learn.cell_centres(g)
    t = g.table()
    assert xy.shape == (g.nx * g.ny, 2)
    assert np.array_equal(xy[np.arange(g.P) // g.n_yaw], t[:, :2])
