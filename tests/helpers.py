"""Shared helpers for the tests: hand-built cameras, meshes and scenes, and
independent (numpy / scipy) evaluations used to pin the oracle."""
from __future__ import annotations

import functools

import numpy as np

from paper_1510_05613_amd import scenes
from oracle import Oracle, render_fn


def down_camera(W=160, H=120, f=100.0, cx=79.5, cy=59.5, height=1.0, delta=0.01):
    """Camera ``height`` metres above the world origin looking straight down:
    camera x = world x, camera y = -world y, camera z = -world z."""
    M = np.array([[1, 0, 0, 0], [0, -1, 0, 0], [0, 0, -1, height]], np.float32)
    return scenes.Sensor(W, H, f, f, cx, cy, M, delta)


def single_pose_table(x=0.0, y=0.0, theta=0.0):
    return np.array([[x, y, np.cos(theta), np.sin(theta)]], np.float32)


def unit_planes():
    return np.array([[0, 0, 1, 1e3]], np.float32)


def plane_grid_mesh(n, size, z, jitter=0.0, rng=None):
    """A horizontal n x n grid of quads (2 triangles each) at height z, facing +z."""
    xs = np.linspace(-size / 2, size / 2, n + 1)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    V = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], 1)
    if jitter > 0:
        interior = (np.abs(V[:, 0]) < size / 2 - 1e-9) & (np.abs(V[:, 1]) < size / 2 - 1e-9)
        V[interior, :2] += rng.uniform(-jitter, jitter, size=(interior.sum(), 2))
    T = []
    for i in range(n):
        for j in range(n):
            a, b = i * (n + 1) + j, (i + 1) * (n + 1) + j
            c, d = (i + 1) * (n + 1) + j + 1, i * (n + 1) + j + 1
            T += [[a, b, c], [a, c, d]]
    T = np.array(T)
    # counter-clockwise seen from +z (above)
    n_ = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    flip = n_[:, 2] < 0
    T[flip, 1], T[flip, 2] = T[flip, 2].copy(), T[flip, 1].copy()
    return V.astype(np.float32), T.astype(np.int32)


def triangle_library(V, T):
    """Every triangle as a mesh of its own (so per-triangle coverage can be counted)."""
    meshes = []
    for t in T:
        meshes.append(scenes.Mesh(V[t].astype(np.float32), np.array([[0, 1, 2]], np.int32),
                                  unit_planes(), "tri"))
    return scenes.Library(meshes)


@functools.lru_cache(maxsize=None)
def c1_library():
    return scenes.make_library("c1")


@functools.lru_cache(maxsize=None)
def c1_scene(i):
    return scenes.make_scene(1, i, render_fn, c1_library())


@functools.lru_cache(maxsize=None)
def c2_library():
    return scenes.make_library("c2")


@functools.lru_cache(maxsize=None)
def c2_scene(i):
    return scenes.make_scene(2, i, render_fn, c2_library())


@functools.lru_cache(maxsize=None)
def c3_library():
    return scenes.make_library("c3")


@functools.lru_cache(maxsize=None)
def c5_scene(i):
    return scenes.make_scene(5, i, render_fn, c3_library())


# ----------------------------------------------------------------------------
# independent evaluation of Eq.(1)-(4) on the oracle's depth images (KD-tree
# nearest neighbours instead of pixel windows; numpy half-space tests)
# ----------------------------------------------------------------------------

def backproject_image(sensor, D):
    H, W = D.shape
    v, u = np.nonzero(np.isfinite(D) & (D > 0))
    z = D[v, u].astype(np.float64)
    x = (u - np.float64(sensor.cx)) * z / np.float64(sensor.fx)
    y = (v - np.float64(sensor.cy)) * z / np.float64(sensor.fy)
    return np.stack([x, y, z], 1), v * W + u


def observed_points(sensor, depth_obs):
    D = depth_obs.astype(np.float64)
    D[D <= 0] = np.inf
    return backproject_image(sensor, D)


def world_from_cam(sensor, P):
    M = sensor.cam_from_world.astype(np.float64)
    R, t = M[:, :3], M[:, 3]
    return (np.linalg.inv(R) @ (P - t).T).T


def vol_margin(mesh, pose_row, Pw):
    x, y, c, s = [np.float64(v) for v in pose_row]
    n2 = c * c + s * s
    dx, dy = Pw[:, 0] - x, Pw[:, 1] - y
    obj = np.stack([(c * dx + s * dy) / n2, (-s * dx + c * dy) / n2, Pw[:, 2]], 1)
    pl = mesh.planes.astype(np.float64)
    return (obj @ pl[:, :3].T - pl[:, 3]).max(1)


def min_dist(A, B):
    from scipy.spatial import cKDTree

    if len(A) == 0:
        return np.zeros(0)
    if len(B) == 0:
        return np.full(len(A), np.inf)
    d, _ = cKDTree(B).query(A, k=1)
    return d


def independent_edge_cost(scene_like, depth_obs, par_mesh, par_pose, cand_mesh, cand_pose, K,
                          o: Oracle):
    """(valid, cost, comps, n_near) of one successor, from the oracle's per-object
    renders but with every count taken by KD-tree / numpy."""
    sensor, lib, poses = scene_like.sensor, scene_like.library, scene_like.poses
    delta = np.float64(np.float32(sensor.delta))
    D_par = np.full((sensor.H, sensor.W), np.inf)
    if len(par_mesh):
        Dp = o.render_objects(par_mesh, par_pose)
        D_par = Dp.min(0)
    D_o = o.render_objects([cand_mesh], [cand_pose])[0]
    both = np.isfinite(D_o) & np.isfinite(D_par)
    if np.any(D_o[both] < D_par[both]):
        return False, -1, None, 0
    dR = np.where(np.isfinite(D_par), np.inf, D_o)
    I, _ = observed_points(sensor, depth_obs)
    Iw = world_from_cam(sensor, I)
    Q, _ = backproject_image(sensor, dR)
    n_near = 0
    d_r = min_dist(Q, I)
    n_near += int(np.sum(np.abs(d_r - delta) <= 1e-6))
    dJr = int(np.sum(d_r * d_r > delta * delta))
    vm = vol_margin(lib.meshes[cand_mesh], poses[cand_pose], Iw)
    n_near += int(np.sum(np.abs(vm) <= 1e-6))
    inV = vm <= 0
    d_o = min_dist(I[inV], Q)
    n_near += int(np.sum(np.abs(d_o - delta) <= 1e-6))
    dJo = int(np.sum(d_o * d_o > delta * delta))
    res = 0
    if len(par_mesh) + 1 == K:
        RK = np.where(np.isfinite(D_par), D_par, dR)
        QK, _ = backproject_image(sensor, RK)
        inAny = inV.copy()
        for m, p in zip(par_mesh, par_pose):
            vmp = vol_margin(lib.meshes[m], poses[p], Iw)
            n_near += int(np.sum(np.abs(vmp) <= 1e-6))
            inAny |= vmp <= 0
        d_k = min_dist(I[~inAny], QK)
        n_near += int(np.sum(np.abs(d_k - delta) <= 1e-6))
        res = int(np.sum(d_k * d_k > delta * delta))
    S = int(np.isfinite(D_o).sum())
    return True, dJr + dJo + res, (S, len(Q), dJr, dJo, res), n_near


def independent_near_counts(scene_like, depth_obs, par_mesh, par_pose, cand_mesh, cand_pose, K,
                            o: Oracle, band=1e-6):
    """Upper bounds, by KD-tree and numpy, of the oracle's three flags for one
    successor: (depth tie, near-delta count, near-volume count).
      - tie: some pixel where candidate and parent depths are both finite and within
        `band` (the flag_valid rule);
      - near-delta: points whose distance to the cloud they are tested against lies
        within `band` of delta, over the sets the oracle tests: dR against I; the
        observed points inside or near V(O) against dR; at the goal level the points
        outside (or near) the candidate's and the parents' volumes against R_K;
      - near-volume: observed points within `band` of the candidate's volume
        boundary, plus (goal level) those within `band` of a parent's.
    The oracle counts only the points whose flip would change the edge cost, so its
    counts must not exceed these."""
    sensor, lib, poses = scene_like.sensor, scene_like.library, scene_like.poses
    delta = np.float64(np.float32(sensor.delta))
    D_par = np.full((sensor.H, sensor.W), np.inf)
    if len(par_mesh):
        D_par = o.render_objects(par_mesh, par_pose).min(0)
    D_o = o.render_objects([cand_mesh], [cand_pose])[0]
    both = np.isfinite(D_o) & np.isfinite(D_par)
    tie = bool(np.any(np.abs(D_o[both] - D_par[both]) <= band))
    dR = np.where(np.isfinite(D_par), np.inf, D_o)
    I, _ = observed_points(sensor, depth_obs)
    Iw = world_from_cam(sensor, I)
    Q, _ = backproject_image(sensor, dR)
    near = lambda d: np.abs(d - delta) <= band  # noqa: E731
    n_delta = int(near(min_dist(Q, I)).sum())
    vm = vol_margin(lib.meshes[cand_mesh], poses[cand_pose], Iw)
    inV, nearV = vm <= 0, np.abs(vm) <= band
    n_vol = int(nearV.sum())
    n_delta += int(near(min_dist(I[inV | nearV], Q)).sum())
    if len(par_mesh) + 1 == K:
        inVp = np.zeros(len(I), bool)
        nearVp = np.zeros(len(I), bool)
        for m, p in zip(par_mesh, par_pose):
            vmp = vol_margin(lib.meshes[m], poses[p], Iw)
            n_vol += int((np.abs(vmp) <= band).sum())
            inVp |= vmp <= 0
            nearVp |= np.abs(vmp) <= band
        tested = (~inV & ~inVp) | (nearV & ~inVp) | (nearVp & ~inV)
        RK = np.where(np.isfinite(D_par), D_par, dR)
        QK, _ = backproject_image(sensor, RK)
        n_delta += int(near(min_dist(I[tested], QK)).sum())
    return tie, n_delta, n_vol
