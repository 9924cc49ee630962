"""Pins of the oracle's local ICP (Sec. IV-E, compensating for a coarse pose
discretization) against what the geometry fixes: a first-order step recovers a
known small motion of exact planar correspondences, a translation exactly; an
object already at its observed pose stays there; an object observed off the
grid is pulled onto its observed pose; an occluding candidate is not aligned.
The association (projective, kept within the 2 cm radius of Sec. V-B) and the
point-to-plane step are readings of the paper, which names ICP without the
variant; the scenes are 640 x 480, the resolution the readings are stated for."""
import numpy as np
import pytest

from oracle import Oracle, icp_step
from tests import helpers as H


def _planar_pairs(rng, n_per=40):
    """Points on three vertical and one horizontal plane (world frame) with
    their unit normals."""
    normals = np.array([[1, 0, 0], [0, 1, 0], [np.sqrt(0.5), -np.sqrt(0.5), 0], [0, 0, 1.0]])
    pts, nrm = [], []
    for n in normals:
        base = rng.uniform(-0.1, 0.1, size=(n_per, 3)) + np.array([0.3, -0.2, 0.05])
        base -= np.outer((base - np.array([0.3, -0.2, 0.05])) @ n, n)  # onto the plane
        pts.append(base)
        nrm.append(np.repeat(n[None], n_per, 0))
    return np.concatenate(pts), np.concatenate(nrm)


def _move(a, phi, t, c):
    """Rotation phi about the vertical axis through c (x, y), then translation t."""
    R = np.array([[np.cos(phi), -np.sin(phi)], [np.sin(phi), np.cos(phi)]])
    out = a.copy()
    out[:, :2] = (a[:, :2] - c) @ R.T + c + t
    return out


def test_step_recovers_a_pure_translation_exactly():
    """Point-to-plane residuals are linear in a translation: one step is exact up
    to the 1e-6 relative damping of the normal matrix."""
    rng = np.random.default_rng(1)
    a, nrm = _planar_pairs(rng)
    t0 = np.array([1.5e-3, -2.5e-3])
    p = a.copy()
    p[:, :2] += t0
    # the normals sit at p: translating a plane keeps its normal
    phi, tx, ty = icp_step(a, p, nrm)
    assert abs(phi) < 1e-8
    assert abs(tx - t0[0]) < 1e-8 and abs(ty - t0[1]) < 1e-8


@pytest.mark.parametrize("phi0", [2e-4, -5e-4])
def test_step_recovers_a_small_rotation_to_first_order(phi0):
    """p = R(phi0) a about the centroid, plus t0; normals rotate with the planes.
    The linearised step returns the same motion up to O(phi0^2) (sign and pivot
    conventions: a wrong sign doubles the error, a wrong pivot adds |c| phi0)."""
    rng = np.random.default_rng(2)
    a, nrm = _planar_pairs(rng)
    c = a[:, :2].mean(0)
    t0 = np.array([4e-4, 3e-4])
    p = _move(a, phi0, t0, c)
    R = np.array([[np.cos(phi0), -np.sin(phi0)], [np.sin(phi0), np.cos(phi0)]])
    nr = nrm.copy()
    nr[:, :2] = nrm[:, :2] @ R.T
    phi, tx, ty = icp_step(a, p, nr)
    # the same motion about the world origin: t' = c + t0 - R c
    tw = c + t0 - R @ c
    assert abs(phi - phi0) < 10 * phi0 ** 2
    assert abs(tx - tw[0]) < 1e-6 and abs(ty - tw[1]) < 1e-6


def _single_object_scene(sc, mesh, pose_row):
    """A scene whose observation is the noise-free render of one object at the
    pose pose_row (appended to the scene's pose table as the last entry)."""
    poses = np.concatenate([sc.poses, np.asarray(pose_row, np.float32)[None]]).astype(np.float32)
    D = Oracle(sc.sensor, sc.library, poses, [mesh]).render_objects([mesh], [len(poses) - 1])[0]
    obs = np.where(np.isfinite(D), D, 0).astype(np.float32)
    return Oracle(sc.sensor, sc.library, poses, [mesh, mesh], obs), poses


def _offset(g, dx, dy, dth):
    th = np.arctan2(g[3], g[2]) + dth
    return np.array([g[0] + dx, g[1] + dy, np.cos(th), np.sin(th)])


@pytest.mark.parametrize("k", [0, 1, 2])
def test_object_at_its_observed_pose_stays(k):
    sc = H.c2_scene(0)
    m, gp = int(sc.obj_mesh[k]), int(sc.gt_pose[k])
    o, poses = _single_object_scene(sc, m, sc.poses[gp])
    P, nm, st, fl = o.icp([], [], [m], [gp], iters=10, radius=0.02)
    assert st[0] == 1 and nm[0] > 100
    g = poses[gp].astype(np.float64)
    assert np.hypot(P[0, 0] - g[0], P[0, 1] - g[1]) < 1e-6
    assert abs(np.arctan2(P[0, 3], P[0, 2]) - np.arctan2(g[3], g[2])) < 1e-6


def _asymmetric_objects(sc):
    """Objects of the scene whose mesh is not a cylinder (yaw is observable)."""
    out = []
    for k, m in enumerate(sc.obj_mesh):
        if len(sc.library.meshes[int(m)].planes) != 64:  # the library's cylinders
            out.append(k)
    return out


@pytest.mark.parametrize("off", [(0.006, -0.004, 3.0), (-0.015, 0.010, -10.0)])
def test_object_observed_off_grid_is_pulled_onto_its_pose(off):
    """ICP from the grid pose converges onto the observed off-grid pose (within
    0.2 mm and 0.05 degrees) for objects whose yaw the surface fixes; a
    cylinder's translation converges too (its yaw is free)."""
    sc = H.c2_scene(0)
    dx, dy, dth = off[0], off[1], np.radians(off[2])
    for k in range(sc.K):
        m, gp = int(sc.obj_mesh[k]), int(sc.gt_pose[k])
        g = sc.poses[gp].astype(np.float64)
        tgt = _offset(g, dx, dy, dth)
        o, poses = _single_object_scene(sc, m, tgt)
        P, nm, st, fl = o.icp([], [], [m], [gp], iters=10, radius=0.02)
        assert st[0] == 1
        e_t = np.hypot(P[0, 0] - poses[-1, 0], P[0, 1] - poses[-1, 1])
        e0 = np.hypot(dx, dy)
        assert e_t < 2e-4, (k, e_t, e0)
        if k in _asymmetric_objects(sc):
            e_a = np.arctan2(P[0, 3], P[0, 2]) - np.arctan2(poses[-1, 3], poses[-1, 2])
            assert abs(np.degrees(e_a)) < 0.05, (k, np.degrees(e_a))
        # the adjusted pose keeps a unit (cos, sin) pair
        assert abs(P[0, 2] ** 2 + P[0, 3] ** 2 - 1) < 1e-6


def test_zero_iterations_return_the_grid_pose():
    sc = H.c2_scene(0)
    m, gp = int(sc.obj_mesh[0]), int(sc.gt_pose[0])
    o = Oracle.from_scene(sc)
    P, nm, st, fl = o.icp([], [], [m], [gp], iters=0, radius=0.02)
    assert st[0] == 1 and nm[0] == 0
    assert np.allclose(P[0], sc.poses[gp], atol=0)


def test_occluding_candidate_is_not_aligned():
    """A candidate in front of the parent's object (Eq. 3 fails) keeps its grid
    pose with status 0 and no matches.  The 640 x 480 scenes hold a pair of
    objects one of which occludes the other by about 20 %."""
    sc = H.c2_scene(0)
    o = Oracle.from_scene(sc)
    found = 0
    for a in range(sc.K):
        for b in range(sc.K):
            if a == b:
                continue
            pm, pp = [int(sc.obj_mesh[a])], [int(sc.gt_pose[a])]
            cm, cp = [int(sc.obj_mesh[b])], [int(sc.gt_pose[b])]
            st_eval, *_ = o.eval(pm, pp, cm, cp)
            P, nm, st, fl = o.icp(pm, pp, cm, cp)
            assert st[0] == st_eval[0]
            if st[0] == 0:
                found += 1
                assert np.array_equal(P[0], sc.poses[cp[0]].astype(np.float64)) and nm[0] == 0
    assert found >= 1
