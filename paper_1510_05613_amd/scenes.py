"""Seeded synthetic tabletop scenes for PERCH (arXiv:1510.05613).

The paper evaluates on a tabletop RGB-D occlusion dataset (Sec. V-A) that is not
available here; these seeded scenes stand in for it with the same structure:
household-sized convex objects resting on a table, 2-6 per scene, seen by a depth
camera with known intrinsics and pose (Sec. III assumptions), objects varying
only in (x, y, yaw), mutual occlusion, and a 3-DoF pose grid (Sec. V-B).

This module generates inputs only.  It holds none of the method's arithmetic:
wherever a scene needs a depth image (checking that an order satisfying the
non-occlusion constraint exists, measuring an occlusion fraction, making the
observed depth) it calls the ``render`` callback it is given, which returns one
stand-alone depth image per object (+inf where uncovered).  The tests pass the CPU
oracle's renderer; the benchmark passes the GPU library's renderer.

Conventions: world z up with the table top at z = 0; camera frame x right, y
down, z forward; pixel (u, v) = (column, row) with centres at integers; depth is
camera Z.  A pose (x, y, theta) places model point m at
(cos t m_x - sin t m_y + x, sin t m_x + cos t m_y + y, m_z).
"""
from __future__ import annotations

import dataclasses
import heapq
import math
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------

CONFIGS: Dict[int, dict] = {
    1: dict(name="plain-160x120", W=160, H=120, f=131.0, table=(0.6, 0.6), lib="c1",
            K=(2, 2), grid=0.05, n_yaw=8, delta=0.01, occlusion=None, cam_height=1.0),
    2: dict(name="plain-640x480", W=640, H=480, f=525.0, table=(1.0, 1.0), lib="c2",
            K=(3, 3), grid=0.02, n_yaw=16, delta=0.005, occlusion=("pair", 0.18, 0.22),
            cam_height=1.0),
    3: dict(name="batched-64x640x480", W=640, H=480, f=525.0, table=(1.0, 1.0), lib="c3",
            K=(2, 5), grid=0.02, n_yaw=16, delta=0.005, occlusion=None, cam_height=1.0,
            n_scenes=64),
    4: dict(name="learned-160x120", W=160, H=120, f=131.0, table=(0.6, 0.6), lib="c1",
            K=(2, 2), grid=0.05, n_yaw=8, delta=0.01, occlusion=None, cam_height=1.0),
    5: dict(name="full-640x480", W=640, H=480, f=525.0, table=(1.5, 1.0), lib="c3",
            K=(6, 6), grid=0.01, n_yaw=32, delta=0.005, occlusion=("heavy", 0.30, 0.70),
            cam_height=None),
}

LIBRARIES = {
    # (family, triangle target) per mesh; extents per axis ~ U[lo, hi] metres
    "c1": dict(meshes=[("box", 500), ("cyl", 500), ("hull", 500)], ext=(0.05, 0.15)),
    "c2": dict(meshes=[("box", 2000), ("cyl", 2500), ("hull", 3000), ("box", 3500),
                       ("cyl", 4000), ("hull", 5000)], ext=(0.05, 0.25)),
    "c3": dict(meshes=[("box", 200), ("cyl", 300), ("hull", 500), ("box", 800),
                       ("cyl", 1200), ("hull", 2000), ("box", 3000), ("cyl", 5000),
                       ("hull", 8000), ("box", 12000), ("cyl", 16000), ("hull", 20000)],
               ext=(0.05, 0.25)),
}
LIBRARY_SEED = {"c1": 1999, "c2": 2999, "c3": 3999}


# ----------------------------------------------------------------------------
# data classes
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Mesh:
    verts: np.ndarray   # (V, 3) float32, model frame, z_min = 0, x/y AABB centred
    tris: np.ndarray    # (T, 3) int32, closed, outward counter-clockwise
    planes: np.ndarray  # (F, 4) float32 (unit n, d): solid = {n.p <= d}
    family: str


@dataclasses.dataclass
class Library:
    meshes: List[Mesh]

    def flat(self):
        """Concatenated arrays with offsets (mesh m owns [off[m], off[m+1]))."""
        v_off = np.cumsum([0] + [len(m.verts) for m in self.meshes]).astype(np.int32)
        t_off = np.cumsum([0] + [len(m.tris) for m in self.meshes]).astype(np.int32)
        f_off = np.cumsum([0] + [len(m.planes) for m in self.meshes]).astype(np.int32)
        verts = np.ascontiguousarray(np.concatenate([m.verts for m in self.meshes]), np.float32)
        tris = np.ascontiguousarray(np.concatenate([m.tris for m in self.meshes]), np.int32)
        planes = np.ascontiguousarray(np.concatenate([m.planes for m in self.meshes]),
                                      np.float32)
        return v_off, t_off, f_off, verts, tris, planes


@dataclasses.dataclass
class Sensor:
    W: int
    H: int
    fx: float
    fy: float
    cx: float
    cy: float
    cam_from_world: np.ndarray  # (3, 4) float32
    delta: float


@dataclasses.dataclass
class Grid:
    x0: float
    y0: float
    step: float
    nx: int
    ny: int
    n_yaw: int

    @property
    def P(self) -> int:
        return self.nx * self.ny * self.n_yaw

    def index(self, ix: int, iy: int, k: int) -> int:
        return (ix * self.ny + iy) * self.n_yaw + k

    def unindex(self, p: int):
        k = p % self.n_yaw
        r = p // self.n_yaw
        return r // self.ny, r % self.ny, k

    def table(self) -> np.ndarray:
        """(P, 4) float32 rows (x, y, cos theta, sin theta); cell centres, yaw 2 pi k / n."""
        ix, iy, k = np.meshgrid(np.arange(self.nx), np.arange(self.ny), np.arange(self.n_yaw),
                                indexing="ij")
        x = self.x0 + (ix.ravel() + 0.5) * self.step
        y = self.y0 + (iy.ravel() + 0.5) * self.step
        th = 2.0 * np.pi * k.ravel() / self.n_yaw
        return np.ascontiguousarray(np.stack([x, y, np.cos(th), np.sin(th)], 1), np.float32)


@dataclasses.dataclass
class Scene:
    config: int
    seed: int
    sensor: Sensor
    library: Library
    grid: Grid
    poses: np.ndarray      # (P, 4) float32
    obj_mesh: np.ndarray   # (K,) int32, the known multiset
    gt_pose: np.ndarray    # (K,) int32 pose index of obj_mesh[k]
    gt_order: np.ndarray   # (K,) indices into obj_mesh: an order meeting the constraint
    depth_obs: np.ndarray  # (H, W) float32 metres, 0 = no return
    table: tuple

    @property
    def K(self) -> int:
        return len(self.obj_mesh)


RenderFn = Callable[[Sensor, Library, np.ndarray, Sequence[int], Sequence[int]], np.ndarray]


# ----------------------------------------------------------------------------
# camera rig
# ----------------------------------------------------------------------------

def look_at(eye, target) -> np.ndarray:
    """cam_from_world (3x4) of a camera at ``eye`` looking at ``target``, no roll,
    x right / y down / z forward."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    up = np.array([0.0, 0.0, 1.0])
    x = np.cross(z, up)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    t = -R @ eye
    return np.concatenate([R, t[:, None]], 1)


def make_sensor(cfg: dict) -> Sensor:
    W, H, f = cfg["W"], cfg["H"], cfg["f"]
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    if cfg["cam_height"] is not None:
        h = cfg["cam_height"]
        M = look_at((0.0, -h, h), (0.0, 0.0, 0.0))
    else:
        # 45 degree pitch; height and back-offset grown until every table corner
        # projects at least 10 px inside the image
        tx, ty = cfg["table"][0] / 2, cfg["table"][1] / 2
        corners = np.array([[sx * tx, sy * ty, 0.0, 1.0] for sx in (-1, 1) for sy in (-1, 1)])
        h = 1.0
        while True:
            M = look_at((0.0, -h, h), (0.0, 0.0, 0.0))
            pc = corners @ M.T
            u = f * pc[:, 0] / pc[:, 2] + cx
            v = f * pc[:, 1] / pc[:, 2] + cy
            if (u.min() >= 10 and u.max() <= W - 1 - 10 and v.min() >= 10
                    and v.max() <= H - 1 - 10):
                break
            h += 0.01
    return Sensor(W, H, f, f, cx, cy, np.ascontiguousarray(M, np.float32), cfg["delta"])


def make_grid(cfg: dict) -> Grid:
    Lx, Ly = cfg["table"]
    step = cfg["grid"]
    nx, ny = int(round(Lx / step)), int(round(Ly / step))
    return Grid(-Lx / 2, -Ly / 2, step, nx, ny, cfg["n_yaw"])


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------

def _orient_outward(V: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Makes every triangle counter-clockwise seen from outside (convex solid)."""
    c = V.mean(0)
    a, b, d = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    n = np.cross(b - a, d - a)
    flip = np.einsum("ij,ij->i", n, (a + b + d) / 3 - c) < 0
    T = T.copy()
    T[flip, 1], T[flip, 2] = T[flip, 2].copy(), T[flip, 1].copy()
    return T


def _refine(V: np.ndarray, T: np.ndarray, target: int):
    """Longest-edge bisection until the mesh has >= target triangles.  Each split
    inserts the edge midpoint and splits both triangles sharing the edge, so the
    mesh stays closed and the surface is unchanged."""
    V = [tuple(v) for v in V]
    T = [list(t) for t in T]
    edges: Dict[tuple, set] = {}

    def key(a, b):
        return (a, b) if a < b else (b, a)

    def add_tri(ti):
        t = T[ti]
        for k in range(3):
            edges.setdefault(key(t[k], t[(k + 1) % 3]), set()).add(ti)

    def length(e):
        a, b = np.array(V[e[0]]), np.array(V[e[1]])
        return float(np.linalg.norm(a - b))

    for ti in range(len(T)):
        add_tri(ti)
    heap = [(-length(e), e) for e in edges]
    heapq.heapify(heap)
    while len(T) < target and heap:
        _, e = heapq.heappop(heap)
        if e not in edges or len(edges[e]) != 2:
            continue
        a, b = e
        m = len(V)
        V.append(tuple((np.array(V[a]) + np.array(V[b])) / 2.0))
        for ti in list(edges[e]):
            t = T[ti]
            for k in range(3):
                if key(t[k], t[(k + 1) % 3]) == e:
                    break
            x, y, z = t[k], t[(k + 1) % 3], t[(k + 2) % 3]
            for kk in range(3):
                ed = key(t[kk], t[(kk + 1) % 3])
                edges[ed].discard(ti)
                if not edges[ed]:
                    del edges[ed]
            T[ti] = [x, m, z]
            T.append([m, y, z])
            add_tri(ti)
            add_tri(len(T) - 1)
        for ed in (key(a, m), key(m, b)):
            heapq.heappush(heap, (-length(ed), ed))
        for ti in edges.get(key(a, m), ()):  # the new edges towards the opposite vertices
            for kk in range(3):
                ed = key(T[ti][kk], T[ti][(kk + 1) % 3])
                if m in ed:
                    heapq.heappush(heap, (-length(ed), ed))
        for ti in edges.get(key(m, b), ()):
            for kk in range(3):
                ed = key(T[ti][kk], T[ti][(kk + 1) % 3])
                if m in ed:
                    heapq.heappush(heap, (-length(ed), ed))
    return np.array(V, np.float64), np.array(T, np.int64)


def make_box(ext, target: int) -> Mesh:
    ex, ey, ez = ext
    x, y = ex / 2, ey / 2
    V = np.array([[-x, -y, 0], [x, -y, 0], [x, y, 0], [-x, y, 0],
                  [-x, -y, ez], [x, -y, ez], [x, y, ez], [-x, y, ez]], np.float64)
    T = np.array([[0, 2, 1], [0, 3, 2], [4, 5, 6], [4, 6, 7], [0, 1, 5], [0, 5, 4],
                  [1, 2, 6], [1, 6, 5], [2, 3, 7], [2, 7, 6], [3, 0, 4], [3, 4, 7]])
    T = _orient_outward(V, T)
    V, T = _refine(V, T, target)
    T = _orient_outward(V, T)
    planes = np.array([[1, 0, 0, x], [-1, 0, 0, x], [0, 1, 0, y], [0, -1, 0, y],
                       [0, 0, 1, ez], [0, 0, -1, 0]], np.float64)
    return Mesh(V.astype(np.float32), T.astype(np.int32), planes.astype(np.float32), "box")


def make_cylinder(ext, n_sides: int, target: int) -> Mesh:
    r = ext[0] / 2
    h = ext[2]
    phi = 2 * np.pi * np.arange(n_sides) / n_sides
    ring = np.stack([r * np.cos(phi), r * np.sin(phi)], 1)
    V = np.concatenate([np.c_[ring, np.zeros(n_sides)], np.c_[ring, np.full(n_sides, h)],
                        [[0, 0, 0], [0, 0, h]]])
    cb, ct = 2 * n_sides, 2 * n_sides + 1
    T = []
    for k in range(n_sides):
        k1 = (k + 1) % n_sides
        T += [[k, k1, n_sides + k1], [k, n_sides + k1, n_sides + k], [cb, k1, k],
              [ct, n_sides + k, n_sides + k1]]
    T = _orient_outward(V, np.array(T))
    V, T = _refine(V, T, target)
    T = _orient_outward(V, T)
    mid = phi + np.pi / n_sides
    planes = np.concatenate([np.c_[np.cos(mid), np.sin(mid), np.zeros(n_sides),
                                   np.full(n_sides, r * np.cos(np.pi / n_sides))],
                             [[0, 0, 1, h], [0, 0, -1, 0]]])
    return Mesh(V.astype(np.float32), T.astype(np.int32), planes.astype(np.float32), "cyl")


def make_hull(ext, rng: np.random.Generator, target: int, n_points: int = 64) -> Mesh:
    from scipy.spatial import ConvexHull

    pts = rng.uniform([-ext[0] / 2, -ext[1] / 2, 0.0], [ext[0] / 2, ext[1] / 2, ext[2]],
                      size=(n_points, 3))
    hull = ConvexHull(pts)
    used = np.unique(hull.simplices)
    remap = -np.ones(len(pts), np.int64)
    remap[used] = np.arange(len(used))
    V = pts[used]
    T = remap[hull.simplices]
    eq = hull.equations  # n.x + off <= 0 inside, unit outward n
    # model origin: x/y AABB centre, z_min = 0
    shift = -np.array([(V[:, 0].min() + V[:, 0].max()) / 2, (V[:, 1].min() + V[:, 1].max()) / 2,
                       V[:, 2].min()])
    V = V + shift
    d = -eq[:, 3] + eq[:, :3] @ shift
    planes = np.unique(np.round(np.c_[eq[:, :3], d], 12), axis=0)
    T = _orient_outward(V, T)
    V, T = _refine(V, T, target)
    T = _orient_outward(V, T)
    return Mesh(V.astype(np.float32), T.astype(np.int32), planes.astype(np.float32), "hull")


def make_library(name: str) -> Library:
    spec = LIBRARIES[name]
    rng = np.random.default_rng(LIBRARY_SEED[name])
    lo, hi = spec["ext"]
    meshes = []
    for fam, target in spec["meshes"]:
        ext = rng.uniform(lo, hi, size=3)
        if fam == "box":
            meshes.append(make_box(ext, target))
        elif fam == "cyl":
            meshes.append(make_cylinder(ext, int(rng.integers(32, 65)), target))
        else:
            meshes.append(make_hull(ext, rng, target))
    return Library(meshes)


def footprint_radius(mesh: Mesh) -> float:
    return float(np.sqrt((mesh.verts[:, :2].astype(np.float64) ** 2).sum(1)).max())


def footprint_polygon(mesh: Mesh) -> np.ndarray:
    """Counter-clockwise convex hull of the mesh's vertices projected on the table
    (Andrew's monotone chain)."""
    pts = sorted(set(map(tuple, np.round(mesh.verts[:, :2].astype(np.float64), 9))))
    if len(pts) < 3:
        return np.array(pts)

    def half(seq):
        h = []
        for q in seq:
            while len(h) >= 2 and ((h[-1][0] - h[-2][0]) * (q[1] - h[-2][1]) -
                                   (h[-1][1] - h[-2][1]) * (q[0] - h[-2][0])) <= 0:
                h.pop()
            h.append(q)
        return h

    lo, hi = half(pts), half(pts[::-1])
    return np.array(lo[:-1] + hi[:-1])


def _placed_polygon(poly: np.ndarray, pose: np.ndarray) -> np.ndarray:
    c, s = float(pose[2]), float(pose[3])
    R = np.array([[c, -s], [s, c]])
    return poly @ R.T + np.asarray(pose[:2], np.float64)


def _polygons_apart(a: np.ndarray, b: np.ndarray, gap: float) -> bool:
    """Separating-axis test: some edge normal of a or b separates them by > gap."""
    for P in (a, b):
        e = np.roll(P, -1, axis=0) - P
        n = np.stack([e[:, 1], -e[:, 0]], 1)
        n /= np.linalg.norm(n, axis=1, keepdims=True)
        pa, pb = a @ n.T, b @ n.T
        if np.any(pa.min(0) - pb.max(0) > gap) or np.any(pb.min(0) - pa.max(0) > gap):
            return True
    return False


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------

def _occlusion_matrix(D: np.ndarray) -> np.ndarray:
    """occ[a, b]: some pixel has object a strictly in front of object b."""
    K = len(D)
    occ = np.zeros((K, K), bool)
    for a in range(K):
        for b in range(K):
            if a != b:
                occ[a, b] = bool(np.any((D[a] < D[b]) & np.isfinite(D[b])))
    return occ


def _front_to_back_order(occ: np.ndarray) -> Optional[np.ndarray]:
    """An insertion order in which no object is added in front of an earlier one
    (occluders first), or None if "a occludes b" has a cycle."""
    K = len(occ)
    indeg = occ.sum(0).astype(int)
    order, done = [], np.zeros(K, bool)
    for _ in range(K):
        free = [a for a in range(K) if not done[a] and indeg[a] == 0]
        if not free:
            return None
        a = free[0]
        done[a] = True
        order.append(a)
        indeg -= occ[a].astype(int)
    return np.array(order, np.int32)


def _hidden_fraction(D: np.ndarray, a: int) -> float:
    """Fraction of object a's stand-alone silhouette hidden by the other objects."""
    sil = np.isfinite(D[a])
    if not sil.any():
        return 0.0
    others = np.min(np.delete(D, a, axis=0), axis=0) if len(D) > 1 else np.full_like(D[a], np.inf)
    return float((sil & (others < D[a])).sum() / sil.sum())


def _in_view(D: np.ndarray) -> bool:
    """Every object has a non-empty silhouette not touching the image border."""
    for d in D:
        m = np.isfinite(d)
        if not m.any() or m[0].any() or m[-1].any() or m[:, 0].any() or m[:, -1].any():
            return False
    return True


def make_scene(config: int, index: int, render: RenderFn, library: Optional[Library] = None,
               max_tries: int = 20000, overrides: Optional[dict] = None) -> Scene:
    """Scene ``index`` of ``config`` (seed 1000 config + index); ``overrides``
    replaces configuration entries (e.g. K) for small test variants."""
    cfg = dict(CONFIGS[config])
    if overrides:
        cfg.update(overrides)
    seed = 1000 * config + index
    rng = np.random.default_rng(seed)
    lib = library if library is not None else make_library(cfg["lib"])
    sensor = make_sensor(cfg)
    grid = make_grid(cfg)
    poses = grid.table()
    kmin, kmax = cfg["K"]
    K = int(rng.integers(kmin, kmax + 1))
    mesh_ids = rng.choice(len(lib.meshes), size=K,
                          replace=K > len(lib.meshes)).astype(np.int32)
    radii = np.array([footprint_radius(lib.meshes[m]) for m in mesh_ids])
    occl = cfg["occlusion"]

    def random_pose():
        return int(rng.integers(grid.P))

    def pose_xy(p):
        return poses[p, :2].astype(np.float64)

    def separated(ps, k, p):
        return all(np.linalg.norm(pose_xy(p) - pose_xy(ps[i])) > radii[k] + radii[i] + 1e-3
                   for i in range(len(ps)))

    for _ in range(max_tries):
        ps: List[int] = []
        if occl is not None and occl[0] == "pair":
            # object 0 (A) is partly hidden behind object 1 (B); B is nearer the camera
            ps.append(random_pose())
            DA = render(sensor, lib, mesh_ids[:1], ps[:1], poses)
            if not _in_view(DA):
                continue
            ok = False
            ia, ja, ka = grid.unindex(ps[0])
            for _t in range(400):
                ib = ia + int(rng.integers(-8, 9))
                jb = ja - int(rng.integers(2, 16))
                if not (0 <= ib < grid.nx and 0 <= jb < grid.ny):
                    continue
                pb = grid.index(ib, jb, int(rng.integers(grid.n_yaw)))
                if not separated(ps, 1, pb):
                    continue
                D = render(sensor, lib, mesh_ids[:2], [ps[0], pb], poses)
                if _in_view(D[1:]) and occl[1] <= _hidden_fraction(D, 0) <= occl[2]:
                    ps.append(pb)
                    ok = True
                    break
            if not ok:
                continue
        if occl is not None and occl[0] == "heavy":
            # one or two front objects, then each further object behind a placed one
            # (larger y is farther from the camera) at a lateral offset, kept only
            # when the part of it the placed objects hide is inside the range
            n_front = int(rng.integers(1, 3))
            polys = [footprint_polygon(lib.meshes[m]) for m in mesh_ids]

            def apart(k, p):  # footprints (convex hulls) at least 1 mm apart
                return all(_polygons_apart(_placed_polygon(polys[k], poses[p]),
                                           _placed_polygon(polys[i], poses[q]), 1e-3)
                           for i, q in enumerate(ps))

            for k in range(K):
                for _t in range(300):
                    if k < n_front:
                        p = random_pose()
                    else:
                        i = int(rng.integers(k))
                        ia, ja, _ = grid.unindex(ps[i])
                        reach = (radii[i] + radii[k]) / grid.step
                        half = max(1, int(reach / 2))
                        ib = ia + int(rng.integers(-half, half + 1))
                        jb = ja + int(rng.integers(1, int(np.ceil(reach)) + 2))
                        if not (0 <= ib < grid.nx and 0 <= jb < grid.ny):
                            continue
                        p = grid.index(ib, jb, int(rng.integers(grid.n_yaw)))
                    if not apart(k, p):
                        continue
                    if k >= n_front:
                        # the new object, and any earlier one it now hides, in range
                        D = render(sensor, lib, mesh_ids[:k + 1], ps + [p], poses)
                        fr = [_hidden_fraction(D, a) for a in range(k + 1)]
                        if not (occl[1] <= fr[k] <= occl[2]):
                            continue
                        if any(0.0 < f < occl[1] or f > occl[2] for f in fr):
                            continue
                    ps.append(p)
                    break
                if len(ps) < k + 1:
                    break
        else:
            for k in range(len(ps), K):
                for _t in range(1000):
                    p = random_pose()
                    if separated(ps, k, p):
                        ps.append(p)
                        break
        if len(ps) < K:
            continue
        D = render(sensor, lib, mesh_ids, ps, poses)
        if not _in_view(D):
            continue
        occm = _occlusion_matrix(D)
        order = _front_to_back_order(occm)
        if order is None:
            continue
        if occl is not None and occl[0] == "heavy":
            occluded = [k for k in range(K) if occm[:, k].any()]
            if len(occluded) < 4:
                continue
            if not all(occl[1] <= _hidden_fraction(D, k) <= occl[2] for k in occluded):
                continue
        gt = np.min(D, axis=0)
        depth = np.zeros(gt.shape, np.float32)
        hit = np.isfinite(gt)
        noisy = gt[hit] + rng.normal(0.0, 0.002, size=int(hit.sum()))
        depth[hit] = (np.round(noisy * 1000.0) / 1000.0).astype(np.float32)
        return Scene(config, seed, sensor, lib, grid, poses, mesh_ids,
                     np.array(ps, np.int32), order, depth, cfg["table"])
    raise RuntimeError(f"no scene found for config {config} index {index}")


def noise_free_observation(scene: Scene, render: RenderFn) -> np.ndarray:
    """The ground-truth render quantised to 1 mm with no noise (the ideal case)."""
    D = render(scene.sensor, scene.library, scene.obj_mesh, scene.gt_pose, scene.poses)
    gt = np.min(D, axis=0)
    out = np.zeros(gt.shape, np.float32)
    hit = np.isfinite(gt)
    out[hit] = (np.round(gt[hit] * 1000.0) / 1000.0).astype(np.float32)
    return out


def pose_subset_around(scene: Scene, radius_cells: int, yaw_stride: int = 1) -> np.ndarray:
    """Pose indices within ``radius_cells`` grid cells of any ground-truth pose,
    every ``yaw_stride``-th yaw (always including the ground-truth yaws); used for
    tiny searches that must include the ground truth."""
    g = scene.grid
    keep = set()
    gts = [g.unindex(int(p)) for p in scene.gt_pose]
    yaws = set(range(0, g.n_yaw, yaw_stride)) | {k for (_, _, k) in gts}
    for (ix, iy, _) in gts:
        for dx in range(-radius_cells, radius_cells + 1):
            for dy in range(-radius_cells, radius_cells + 1):
                jx, jy = ix + dx, iy + dy
                if 0 <= jx < g.nx and 0 <= jy < g.ny:
                    for k in yaws:
                        keep.add(g.index(jx, jy, k))
    return np.array(sorted(keep), np.int32)


def offgrid_truth(scene: Scene, render: RenderFn, shift: float = 0.4, seed: int = 0):
    """The scene's objects moved off the pose grid: each ground-truth pose shifted
    by a random fraction (up to ``shift`` of a cell in x and y, and of a yaw step)
    of the grid spacing, the observation re-rendered from those poses with the
    generator's noise recipe (N(0, 2 mm), quantised to 1 mm).  Returns (true poses
    (K, 4) float32, depth_obs).  The nearest grid pose of each object stays its
    ground-truth pose; the grid can no longer express the scene exactly, which is
    what the local ICP of Sec. IV-E compensates for."""
    rng = np.random.default_rng(10_000 + scene.seed + seed)
    g = scene.grid
    true = []
    for p in scene.gt_pose:
        x, y, c, s = (float(v) for v in scene.poses[int(p)])
        dx, dy, dk = rng.uniform(-shift, shift, 3)
        th = np.arctan2(s, c) + dk * 2.0 * np.pi / g.n_yaw
        true.append([x + dx * g.step, y + dy * g.step, np.cos(th), np.sin(th)])
    true = np.asarray(true, np.float32)
    poses = np.concatenate([scene.poses, true]).astype(np.float32)
    idx = np.arange(len(scene.poses), len(poses), dtype=np.int32)
    D = render(scene.sensor, scene.library, scene.obj_mesh, idx, poses)
    gt = np.min(D, axis=0)
    depth = np.zeros(gt.shape, np.float32)
    hit = np.isfinite(gt)
    noisy = gt[hit] + rng.normal(0.0, 0.002, size=int(hit.sum()))
    depth[hit] = (np.round(noisy * 1000.0) / 1000.0).astype(np.float32)
    return true, depth


def chessboard_scene(render: RenderFn, seed: int = 0) -> Scene:
    """A chessboard-like stand-in for the paper's twelve-piece run (Sec. V-C): an
    8 x 8 board of 4 cm squares with the pose grid on the square centres (8 yaws),
    twelve pieces of three kinds — eight pawns (cylinders, rotationally symmetric),
    two rooks (square towers) and two kings (tall cylinders, symmetric) — the
    pieces on the first rank, the pawns on the second, seen from in front of the
    first rank (the pieces hide parts of the pawns).  640 x 480, delta = 7.5 mm as
    in that run; the observation uses the generator's noise recipe.  The seed
    shuffles the files of the first-rank pieces and the pawns' yaws are 0."""
    rng = np.random.default_rng(20_000 + seed)
    lib = Library([make_cylinder((0.030, 0.030, 0.045), 48, 400),   # pawn
                   make_box((0.032, 0.032, 0.060), 300),             # rook
                   make_cylinder((0.036, 0.036, 0.090), 48, 600)])   # king
    cfg = dict(W=640, H=480, f=525.0, table=(0.32, 0.32), delta=0.0075, cam_height=0.45)
    sensor = make_sensor(cfg)
    grid = Grid(-0.16, -0.16, 0.04, 8, 8, 8)
    poses = grid.table()
    files = rng.permutation(8)[:4]  # first-rank files of rook, rook, king, king
    mesh_ids = [0] * 8 + [1, 1, 2, 2]
    gt = [grid.index(ix, 1, 0) for ix in range(8)]
    gt += [grid.index(int(f), 0, 0) for f in files]
    mesh_ids = np.array(mesh_ids, np.int32)
    gt = np.array(gt, np.int32)
    D = render(sensor, lib, mesh_ids, gt, poses)
    if not _in_view(D):
        raise RuntimeError("chessboard pieces out of view")
    order = _front_to_back_order(_occlusion_matrix(D))
    if order is None:
        raise RuntimeError("chessboard occlusion has a cycle")
    depth_gt = np.min(D, axis=0)
    depth = np.zeros(depth_gt.shape, np.float32)
    hit = np.isfinite(depth_gt)
    noisy = depth_gt[hit] + rng.normal(0.0, 0.002, size=int(hit.sum()))
    depth[hit] = (np.round(noisy * 1000.0) / 1000.0).astype(np.float32)
    return Scene(0, 20_000 + seed, sensor, lib, grid, poses, mesh_ids, gt, order, depth,
                 cfg["table"])
