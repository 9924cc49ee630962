"""ctypes wrapper of the CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path never imports it.  The oracle is
the scalar FP64 definition of PERCH's successor evaluation (arXiv:1510.05613,
Sec. III-IV); see ``perch_oracle.c`` for the passages each step follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PERCH_ORACLE_LIB: another build of the same source (the sanitizer test's)
LIB_PATH = os.environ.get("PERCH_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "perch_oracle.c")]


def build(force: bool = True) -> str:
    """Compiles liboracle.so with gcc (float32 vertex stage needs no contraction)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O3", "-march=x86-64-v2", "-std=c11", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp,
               *SOURCES, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Sensor(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("cam_from_world", C.c_float * 12), ("delta", C.c_float)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(_Sensor), P, C.c_int32, P, P, P, P, P, P, C.c_int32,
                                 P, C.c_int32, P]
        L.orc_destroy.argtypes = [P]
        L.orc_set_mode.argtypes = [P, C.c_int32, C.c_int32]
        L.orc_num_points.argtypes = [P]
        L.orc_vertex_stage.argtypes = [P, C.c_int32, C.c_int32, P, P]
        L.orc_render_objects.argtypes = [P, C.c_int32, P, P, C.c_int32, P]
        L.orc_eval.argtypes = [P, C.c_int32, P, P, C.c_int32, P, P, P, P, P, P]
        L.orc_jtree.argtypes = [P, C.c_int32, P, P, P]
        L.orc_overlap.argtypes = [P, C.c_int32, P, P, C.c_int32, P, P, P, P, P]
        L.orc_icp_step.argtypes = [C.c_int32, P, P, P, P]
        L.orc_set_symmetric.argtypes = [P, C.c_int32, C.c_int32]
        L.orc_icp.argtypes = [P, C.c_int32, P, P, C.c_int32, P, P, C.c_int32, C.c_double, P, P,
                              P, P]
        for f in (L.orc_search_exhaustive, L.orc_search_ucs, L.orc_bruteforce_joint):
            f.argtypes = [P, C.c_int32, P, P, P, P]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1))


class Oracle:
    """One scene: sensor, observed depth (optional), mesh library, pose table and
    the known multiset of K mesh ids."""

    def __init__(self, sensor, library, poses: np.ndarray, obj_mesh: Sequence[int] = (),
                 depth_obs: Optional[np.ndarray] = None, nthreads: int = 1,
                 radius_mode: int = 0):
        L = lib()
        s = _Sensor()
        s.width, s.height = int(sensor.W), int(sensor.H)
        s.fx, s.fy, s.cx, s.cy = sensor.fx, sensor.fy, sensor.cx, sensor.cy
        M = np.asarray(sensor.cam_from_world, np.float32).reshape(-1)
        for i in range(12):
            s.cam_from_world[i] = float(M[i])
        s.delta = float(sensor.delta)
        self.sensor = sensor
        self._keep = list(library.flat())
        v_off, t_off, f_off, verts, tris, planes = self._keep
        self.poses = np.ascontiguousarray(poses, np.float32)
        self.obj_mesh = _i32(obj_mesh)
        self.depth = None if depth_obs is None else np.ascontiguousarray(depth_obs, np.float32)
        self.K = len(self.obj_mesh)
        h = L.orc_create(C.byref(s), _ptr(self.depth), len(library.meshes), _ptr(v_off),
                         _ptr(t_off), _ptr(f_off), _ptr(verts), _ptr(tris), _ptr(planes),
                         len(self.poses), _ptr(self.poses), self.K, _ptr(self.obj_mesh))
        if not h:
            raise ValueError("orc_create rejected the scene")
        self.h = C.c_void_p(h)
        self.set_mode(radius_mode, nthreads)

    @classmethod
    def from_scene(cls, scene, depth_obs: Optional[np.ndarray] = None, **kw) -> "Oracle":
        d = scene.depth_obs if depth_obs is None else depth_obs
        return cls(scene.sensor, scene.library, scene.poses, scene.obj_mesh, d, **kw)

    def close(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_mode(self, radius_mode: int = 0, nthreads: int = 1):
        if lib().orc_set_mode(self.h, radius_mode, nthreads) != 0:
            raise ValueError("bad mode")

    def set_symmetric(self, mesh: int, symmetric: bool = True):
        """Searches try a symmetric mesh only at the first pose per (x, y)."""
        if lib().orc_set_symmetric(self.h, int(mesh), int(bool(symmetric))):
            raise RuntimeError("orc_set_symmetric failed")

    @property
    def n_points(self) -> int:
        return lib().orc_num_points(self.h)

    def vertex_stage(self, mesh: int, pose: int):
        nv = int(self._keep[0][mesh + 1] - self._keep[0][mesh])
        cam = np.zeros((nv, 3), np.float32)
        uv = np.zeros((nv, 2), np.int32)
        rc = lib().orc_vertex_stage(self.h, mesh, pose, _ptr(cam), _ptr(uv))
        if rc:
            raise RuntimeError(f"orc_vertex_stage failed ({rc})")
        return cam, uv

    def render_objects(self, mesh, pose, cull: bool = True) -> np.ndarray:
        m, p = _i32(mesh), _i32(pose)
        out = np.empty((len(m), self.sensor.H, self.sensor.W), np.float64)
        rc = lib().orc_render_objects(self.h, len(m), _ptr(m), _ptr(p), int(cull), _ptr(out))
        if rc:
            raise RuntimeError(f"orc_render_objects failed ({rc})")
        return out

    def eval(self, parent_mesh, parent_pose, cand_mesh, cand_pose):
        """Edge costs of successors of one parent.  Returns (status, cost, comps, flags)."""
        pm, pp = _i32(parent_mesh), _i32(parent_pose)
        cm, cp = _i32(cand_mesh), _i32(cand_pose)
        n = len(cm)
        st = np.zeros(n, np.int32)
        cost = np.zeros(n, np.int32)
        comps = np.zeros((n, 5), np.int32)
        flags = np.zeros((n, 3), np.int32)
        rc = lib().orc_eval(self.h, len(pm), _ptr(pm), _ptr(pp), n, _ptr(cm), _ptr(cp), _ptr(st),
                            _ptr(cost), _ptr(comps), _ptr(flags))
        if rc:
            raise RuntimeError(f"orc_eval failed ({rc})")
        return st, cost, comps, flags

    def overlap(self, parent_mesh, parent_pose, cand_mesh, cand_pose):
        """Overlap heuristic (Sec. IV-C) of the parent and of each child.
        Returns (h_parent, h_child (n,), flags (n,))."""
        pm, pp = _i32(parent_mesh), _i32(parent_pose)
        cm, cp = _i32(cand_mesh), _i32(cand_pose)
        n = len(cm)
        hp = np.zeros(1, np.int64)
        hc = np.zeros(n, np.int64)
        fl = np.zeros(n, np.int32)
        rc = lib().orc_overlap(self.h, len(pm), _ptr(pm), _ptr(pp), n, _ptr(cm), _ptr(cp),
                               _ptr(hp), _ptr(hc), _ptr(fl))
        if rc:
            raise RuntimeError(f"orc_overlap failed ({rc})")
        return int(hp[0]), hc, fl

    def icp(self, parent_mesh, parent_pose, cand_mesh, cand_pose, iters: int = 10,
            radius: float = 0.02):
        """Local ICP (Sec. IV-E) of each candidate under the parent.  Returns
        (poses (n, 4) float64 (x, y, cos, sin), n_match (n,), status (n,), flags (n,))."""
        pm, pp = _i32(parent_mesh), _i32(parent_pose)
        cm, cp = _i32(cand_mesh), _i32(cand_pose)
        n = len(cm)
        out = np.zeros((max(n, 1), 4), np.float64)
        nm = np.zeros(max(n, 1), np.int32)
        st = np.zeros(max(n, 1), np.int32)
        fl = np.zeros(max(n, 1), np.int32)
        rc = lib().orc_icp(self.h, len(pm), _ptr(pm), _ptr(pp), n, _ptr(cm), _ptr(cp),
                           int(iters), float(radius), _ptr(out), _ptr(nm), _ptr(st), _ptr(fl))
        if rc:
            raise RuntimeError(f"orc_icp failed ({rc})")
        return out[:n], nm[:n], st[:n], fl[:n]

    def jtree(self, mesh, pose) -> dict:
        m, p = _i32(mesh), _i32(pose)
        out = np.zeros(6, np.int64)
        rc = lib().orc_jtree(self.h, len(m), _ptr(m), _ptr(p), _ptr(out))
        if rc:
            raise RuntimeError(f"orc_jtree failed ({rc})")
        return dict(valid=bool(out[0]), J_tree=int(out[1]), J_raw=int(out[2]),
                    n_flag_delta=int(out[3]), n_flag_vol=int(out[4]), flag_valid=bool(out[5]))

    def _search(self, fn, pose_subset):
        sub = None if pose_subset is None else _i32(pose_subset)
        bm = np.zeros(max(self.K, 1), np.int32)
        bp = np.zeros(max(self.K, 1), np.int32)
        stats = np.zeros(4, np.int64)
        rc = fn(self.h, 0 if sub is None else len(sub), _ptr(sub), _ptr(bm), _ptr(bp),
                _ptr(stats))
        if rc < 0:
            raise RuntimeError(f"search failed ({rc})")
        return dict(found=(rc == 0), mesh=bm, pose=bp, cost=int(stats[0]),
                    n_eval=int(stats[1]), n_expanded=int(stats[2]), n_goal=int(stats[3]))

    def search_exhaustive(self, pose_subset=None):
        return self._search(lib().orc_search_exhaustive, pose_subset)

    def search_ucs(self, pose_subset=None):
        return self._search(lib().orc_search_ucs, pose_subset)

    def bruteforce_joint(self, pose_subset=None):
        r = self._search(lib().orc_bruteforce_joint, pose_subset)
        r["n_valid"] = r.pop("n_eval")
        return r


def icp_step(a, p, nrm):
    """(phi, tx, ty): the linearised point-to-plane step for pairs a (n, 3) -> p
    (n, 3) with unit normals nrm (n, 3) at p, world frame."""
    a = np.ascontiguousarray(a, np.float64).reshape(-1, 3)
    p = np.ascontiguousarray(p, np.float64).reshape(-1, 3)
    nrm = np.ascontiguousarray(nrm, np.float64).reshape(-1, 3)
    out = np.zeros(3, np.float64)
    rc = lib().orc_icp_step(len(a), _ptr(a), _ptr(p), _ptr(nrm), _ptr(out))
    if rc:
        raise RuntimeError(f"orc_icp_step failed ({rc})")
    return tuple(float(v) for v in out)


def render_fn(sensor, library, mesh_ids, pose_idx, poses) -> np.ndarray:
    """Renderer callback for the scene generator: stand-alone depth per object."""
    o = Oracle(sensor, library, poses)
    try:
        return o.render_objects(mesh_ids, pose_idx)
    finally:
        o.close()
