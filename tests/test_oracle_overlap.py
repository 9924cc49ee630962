"""The oracle's overlap heuristic (Sec. IV-C: points of I outside the volumes of the
objects placed so far) against independent counts."""
import numpy as np

from oracle import Oracle
from tests import helpers as H


def _world_points(sc):
    """Observed cloud in the world frame, from the depth image (numpy, FP64)."""
    s = sc.sensor
    v, u = np.nonzero(sc.depth_obs > 0)
    z = sc.depth_obs[v, u].astype(np.float64)
    cam = np.stack([(u - s.cx) / s.fx * z, (v - s.cy) / s.fy * z, z], 1)
    M = s.cam_from_world.astype(np.float64)
    return (cam - M[:, 3]) @ np.linalg.inv(M[:, :3]).T


def test_root_counts_every_observed_point():
    sc = H.c1_scene(0)
    o = Oracle.from_scene(sc)
    h, hc, fl = o.overlap([], [], [], [])
    assert h == int((sc.depth_obs > 0).sum()) == o.n_points


def test_box_volume_recount_and_monotone():
    """Mesh 0 of the library is a box: 'inside' is |x| <= a, |y| <= b, 0 <= z <= c in
    the object frame, whatever the mesh's plane list says."""
    sc = H.c1_scene(0)
    box = sc.library.meshes[0]
    lo, hi = box.verts.min(0).astype(np.float64), box.verts.max(0).astype(np.float64)
    o = Oracle.from_scene(sc)
    P = _world_points(sc)
    rng = np.random.default_rng(1)
    poses = rng.choice(sc.grid.P, 60, replace=False)
    # include the true pose of the first object, whatever its mesh
    parent = ([int(sc.obj_mesh[1])], [int(sc.gt_pose[1])])
    for pm, pp in (([], []), parent):
        h0, hc, fl = o.overlap(pm, pp, np.zeros(len(poses), np.int32), poses)
        assert np.all(hc <= h0)
        # points already inside the parent volumes (oracle's own decision, parent only)
        _, hc_par, _ = o.overlap([], [], pm, pp) if pm else (None, np.array([h0]), None)
        assert h0 == int(hc_par[0])
        for k, p in enumerate(poses):
            x, y, c, s = sc.poses[p].astype(np.float64)
            d = P[:, :2] - [x, y]
            ox, oy = c * d[:, 0] + s * d[:, 1], -s * d[:, 0] + c * d[:, 1]
            inside_box = ((ox >= lo[0]) & (ox <= hi[0]) & (oy >= lo[1]) & (oy <= hi[1]) &
                          (P[:, 2] >= lo[2]) & (P[:, 2] <= hi[2]))
            if not pm:
                assert abs((h0 - hc[k]) - int(inside_box.sum())) <= fl[k], (p, h0 - hc[k],
                                                                            inside_box.sum())


def test_ground_truth_scene_leaves_only_noise():
    """Observing the unquantised ground-truth render, every observed point lies on a
    placed object's surface: the full ground-truth assignment leaves no point
    outside, up to points within the flag band of a boundary."""
    from oracle import render_fn

    sc = H.c1_scene(2)
    D = render_fn(sc.sensor, sc.library, sc.obj_mesh, sc.gt_pose, sc.poses)
    gt = np.min(D, axis=0)
    d = np.where(np.isfinite(gt), gt, 0.0).astype(np.float32)
    o = Oracle.from_scene(sc, depth_obs=d)
    order = sc.gt_order
    pm = [int(sc.obj_mesh[k]) for k in order[:-1]]
    pp = [int(sc.gt_pose[k]) for k in order[:-1]]
    last = order[-1]
    h0, hc, fl = o.overlap(pm, pp, [int(sc.obj_mesh[last])], [int(sc.gt_pose[last])])
    assert 0 <= hc[0] <= fl[0]
    assert h0 > hc[0]
