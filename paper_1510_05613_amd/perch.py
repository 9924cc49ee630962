"""Python binding of libperch.so (the C ABI in include/perch.h).

Argument marshalling only: every step of PERCH's successor evaluation runs in the
HIP kernels of libperch.so.  torch supplies device memory (tensors on the GPU) and
the HIP stream.  There is no CPU path: if the library is missing, or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libperch.so")

PERCH_SUCC_VALID = 1
PERCH_SUCC_INVALID = 0
PERCH_SUCC_NEAR_PLANE = -2
PERCH_SUCC_TOO_WIDE = -3
PERCH_SUCC_BAD_INPUT = -4

# the public symbols declared in include/perch.h
EXPORTS = ("perch_create", "perch_destroy", "perch_set_observation", "perch_add_mesh",
           "perch_set_poses", "perch_set_objects", "perch_eval_successors",
           "perch_eval_successors_noalloc", "perch_set_parent",
           "perch_eval_children", "perch_overlap_gain", "perch_set_pose_arena",
           "perch_set_symmetric",
           "perch_get_poses", "perch_icp_children", "perch_render", "perch_set_tuning",
           "perch_get_info",
           "perch_search", "perch_batch_create", "perch_batch_destroy",
           "perch_batch_set_parents", "perch_batch_eval", "perch_batch_set_tuning",
           "perch_batch_autotune",
           "perch_autotune", "perch_cnn_create", "perch_cnn_destroy", "perch_cnn_param_count",
           "perch_cnn_set_params", "perch_cnn_get_params", "perch_cnn_crops", "perch_cnn_predict",
           "perch_cnn_predict_scene",
           "perch_cnn_set_crop_step",
           "perch_rank_children", "perch_cnn_train_step", "perch_cnn_gradients",
           "perch_posenet_create", "perch_posenet_destroy", "perch_posenet_param_count",
           "perch_posenet_set_params", "perch_posenet_get_params", "perch_cnn_crops_step",
           "perch_posenet_predict", "perch_posenet_train_step", "perch_posenet_gradients",
           "perch_posenet_estimate", "perch_last_error")

SEARCH_EXHAUSTIVE, SEARCH_UCS, SEARCH_FOCAL, SEARCH_LEARNED, SEARCH_MHA = 0, 1, 2, 3, 4
SEARCH_LEARNED_MHA = 5
MAX_OBJECTS = 16  # PERCH_MAX_OBJECTS


class PerchError(RuntimeError):
    pass


class _Sensor(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("cam_from_world", C.c_float * 12), ("delta", C.c_float)]


class PerchObject(C.Structure):
    _fields_ = [("mesh_id", C.c_int32), ("pose_idx", C.c_int32)]


class PerchParent(C.Structure):
    _fields_ = [("ctx", C.c_int32), ("j", C.c_int32), ("objs", PerchObject * MAX_OBJECTS)]


class _Tuning(C.Structure):
    _fields_ = [("threads", C.c_int32), ("tile_px", C.c_int32), ("radius_mode", C.c_int32),
                ("cell_over_delta", C.c_float), ("ms", C.c_float)]


class _BatchTuning(C.Structure):
    _fields_ = [("threads", C.c_int32), ("tile_px", C.c_int32), ("radius_mode", C.c_int32),
                ("cell_over_delta", C.c_float), ("ms", C.c_float), ("default_ms", C.c_float)]


class PerchPosePrior(C.Structure):
    _fields_ = [("mesh_id", C.c_int32), ("x", C.c_float), ("y", C.c_float),
                ("theta", C.c_float)]


class _SearchOpts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("w", C.c_float), ("anytime", C.c_int32),
                ("budget_s", C.c_double), ("budget_expansions", C.c_int64),
                ("pose_subset", C.c_void_p), ("n_pose_subset", C.c_int32),
                ("cnn", C.c_void_p), ("topk", C.c_int32), ("icp_iters", C.c_int32),
                ("icp_radius", C.c_float), ("priors", C.c_void_p), ("n_priors", C.c_int32),
                ("prior_rad_m", C.c_float), ("prior_slot_m", C.c_float), ("batch", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("objs", PerchObject * MAX_OBJECTS), ("K", C.c_int32), ("found", C.c_int32),
                ("cost", C.c_int64), ("edge_cost", C.c_int32 * MAX_OBJECTS),
                ("n_expanded", C.c_int64),
                ("n_evaluated", C.c_int64), ("n_invalid", C.c_int64), ("t_total_s", C.c_double),
                ("t_best_s", C.c_double), ("lower_bound", C.c_int64),
                ("n_evaluated_best", C.c_int64), ("n_merged", C.c_int64),
                ("n_trace", C.c_int32), ("trace_t", C.c_double * 64),
                ("trace_cost", C.c_int64 * 64), ("trace_lb", C.c_int64 * 64)]


_lib = None


def load(path: str = LIB_PATH):
    """Loads libperch.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise PerchError(f"{path} is missing: build it with paper_1510_05613_amd.build.build()")
    L = C.CDLL(path)
    P, I32 = C.c_void_p, C.c_int32
    L.perch_create.argtypes = [C.POINTER(_Sensor), P, C.POINTER(P)]
    L.perch_destroy.argtypes = [P]
    L.perch_destroy.restype = None
    L.perch_set_observation.argtypes = [P, P]
    L.perch_add_mesh.argtypes = [P, I32, P, I32, P, I32, P, I32]
    L.perch_set_poses.argtypes = [P, P, I32]
    L.perch_set_objects.argtypes = [P, P, I32]
    L.perch_eval_successors.argtypes = [P, P, I32, P, I32, P, P, P]
    L.perch_eval_successors_noalloc.argtypes = [P, P, I32, P, I32, P, P, P]
    L.perch_set_parent.argtypes = [P, P, I32]
    L.perch_eval_children.argtypes = [P, P, I32, P, P, P]
    L.perch_render.argtypes = [P, P, I32, I32, P]
    L.perch_overlap_gain.argtypes = [P, P, I32, P, P, P]
    L.perch_set_pose_arena.argtypes = [P, I32]
    L.perch_set_symmetric.argtypes = [P, I32, I32]
    L.perch_get_poses.argtypes = [P, I32, I32, P]
    L.perch_icp_children.argtypes = [P, P, I32, I32, C.c_float, P, P, P]
    L.perch_set_tuning.argtypes = [P, I32, I32, C.c_float, I32]
    L.perch_get_info.argtypes = [P, C.POINTER(I32), C.POINTER(I32)]
    L.perch_search.argtypes = [P, C.POINTER(_SearchOpts), C.POINTER(_Result)]
    L.perch_autotune.argtypes = [P, P, I32, P, I32, I32, C.c_char_p, C.POINTER(_Tuning)]
    L.perch_cnn_create.argtypes = [I32, I32, I32, P, C.POINTER(P)]
    L.perch_cnn_destroy.argtypes = [P]
    L.perch_cnn_destroy.restype = None
    L.perch_cnn_param_count.argtypes = [P]
    L.perch_cnn_set_params.argtypes = [P, P, C.c_int64]
    L.perch_cnn_get_params.argtypes = [P, P, C.c_int64]
    L.perch_cnn_crops.argtypes = [P, P, I32, P]
    L.perch_cnn_set_crop_step.argtypes = [P, I32]
    L.perch_cnn_predict.argtypes = [P, P, I32, P, I32, P]
    L.perch_cnn_predict_scene.argtypes = [P, P, P, I32, P, I32, P]
    L.perch_rank_children.argtypes = [P, P, I32, I32, P, I32, P, P, P]
    L.perch_cnn_train_step.argtypes = [P, P, I32, P, P, I32, C.c_float, C.POINTER(C.c_float)]
    L.perch_cnn_gradients.argtypes = [P, P, I32, P, P, I32, P, C.POINTER(C.c_float)]
    L.perch_posenet_create.argtypes = [I32, I32, I32, I32, P, C.POINTER(P)]
    L.perch_posenet_destroy.argtypes = [P]
    L.perch_posenet_destroy.restype = None
    L.perch_posenet_param_count.argtypes = [P]
    L.perch_posenet_param_count.restype = C.c_int64
    L.perch_posenet_set_params.argtypes = [P, P, C.c_int64]
    L.perch_posenet_get_params.argtypes = [P, P, C.c_int64]
    L.perch_cnn_crops_step.argtypes = [P, P, I32, I32, P]
    L.perch_posenet_predict.argtypes = [P, P, I32, P, I32, P]
    L.perch_posenet_train_step.argtypes = [P, P, I32, P, P, I32, C.c_float,
                                           C.POINTER(C.c_float)]
    L.perch_posenet_gradients.argtypes = [P, P, I32, P, P, I32, P, C.POINTER(C.c_float)]
    L.perch_posenet_estimate.argtypes = [P, P, I32, P, C.c_float, C.c_float, P, P, I32, P, I32,
                                         C.POINTER(I32)]
    L.perch_batch_create.argtypes = [P, I32, P, C.POINTER(P)]
    L.perch_batch_destroy.argtypes = [P]
    L.perch_batch_destroy.restype = None
    L.perch_batch_set_parents.argtypes = [P, P, I32]
    L.perch_batch_eval.argtypes = [P, P, I32, P, P, P]
    L.perch_batch_set_tuning.argtypes = [P, I32, I32, I32, I32]
    L.perch_batch_autotune.argtypes = [P, P, I32, I32, C.c_char_p, C.POINTER(_BatchTuning)]
    L.perch_cnn_param_count.restype = C.c_int64
    L.perch_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("perch_destroy", "perch_batch_destroy", "perch_cnn_destroy",
                        "perch_cnn_param_count", "perch_posenet_destroy",
                        "perch_posenet_param_count", "perch_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        msg = load().perch_last_error().decode(errors="replace")
        raise PerchError(f"perch error {rc}: {msg}")


def _objects(objs) -> C.Array:
    arr = (PerchObject * max(1, len(objs)))()
    for k, (m, p) in enumerate(objs):
        arr[k].mesh_id = int(m)
        arr[k].pose_idx = int(p)
    return arr


def _dev_ptr(t, dtype_name: str, numel: Optional[int] = None) -> int:
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise PerchError("expected a GPU tensor")
    if str(t.dtype) != f"torch.{dtype_name}" or not t.is_contiguous():
        raise PerchError(f"expected a contiguous {dtype_name} tensor, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise PerchError(f"tensor has {t.numel()} elements, need {numel}")
    return t.data_ptr()


class Context:
    """One scene on one GPU: sensor, observation, mesh library, pose table, objects."""

    def __init__(self, sensor, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise PerchError("no GPU: libperch.so has no CPU path")
        L = load()
        s = _Sensor()
        s.width, s.height = int(sensor.W), int(sensor.H)
        s.fx, s.fy, s.cx, s.cy = sensor.fx, sensor.fy, sensor.cx, sensor.cy
        M = np.asarray(sensor.cam_from_world, np.float32).reshape(-1)
        for i in range(12):
            s.cam_from_world[i] = float(M[i])
        s.delta = float(sensor.delta)
        self.sensor = sensor
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(L.perch_create(C.byref(s), C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.H, self.W = int(sensor.H), int(sensor.W)
        self.K = 0

    def close(self):
        if getattr(self, "h", None):
            load().perch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_observation(self, depth):
        _check(load().perch_set_observation(self.h, _dev_ptr(depth, "float32", self.H * self.W)))

    def add_mesh(self, mesh_id: int, verts, tris, planes):
        v = np.ascontiguousarray(verts, np.float32)
        t = np.ascontiguousarray(tris, np.int32)
        p = np.ascontiguousarray(planes, np.float32)
        _check(load().perch_add_mesh(self.h, mesh_id, v.ctypes.data, len(v), t.ctypes.data,
                                     len(t), p.ctypes.data, len(p)))

    def set_poses(self, poses):
        p = np.ascontiguousarray(poses, np.float32)
        _check(load().perch_set_poses(self.h, p.ctypes.data, len(p)))

    def set_objects(self, mesh_ids: Sequence[int]):
        m = np.ascontiguousarray(mesh_ids, np.int32)
        _check(load().perch_set_objects(self.h, m.ctypes.data, len(m)))
        self.K = len(m)

    def set_tuning(self, threads: int = 0, tile_px: int = 0, cell_over_delta: float = 0.0,
                   radius_mode: int = -1):
        """Kernel knobs: threads per successor, z-tile pixels (-1 = sized
        automatically), voxel cell / delta, radius mode; 0 (radius_mode -1) keeps the
        current value.  Results do not depend on them."""
        _check(load().perch_set_tuning(self.h, threads, tile_px, cell_over_delta, radius_mode))

    def autotune(self, parent, cands, reps: int = 3, cache_path: Optional[str] = None) -> dict:
        """Times the kernel settings on a calibration batch and applies the fastest."""
        t = _Tuning()
        _check(load().perch_autotune(
            self.h, C.cast(_objects(parent), C.c_void_p), len(parent),
            _dev_ptr(cands, "int32", 2 * cands.shape[0]), cands.shape[0], reps,
            None if cache_path is None else cache_path.encode(), C.byref(t)))
        return dict(threads=t.threads, tile_px=t.tile_px, radius_mode=t.radius_mode,
                    cell_over_delta=t.cell_over_delta, ms=t.ms)

    def info(self):
        n, h = C.c_int32(), C.c_int32()
        _check(load().perch_get_info(self.h, C.byref(n), C.byref(h)))
        return dict(n_points=n.value, halo=h.value)

    def eval_successors(self, parent, cands, cost, status, comps=None):
        """parent: sequence of (mesh, pose); cands: int32 GPU tensor (n, 2); outputs:
        int32 GPU tensors (n,), (n,), and optionally (n, 5).  Asynchronous."""
        n = cands.shape[0]
        par = _objects(parent)
        _check(load().perch_eval_successors(
            self.h, C.cast(par, C.c_void_p), len(parent), _dev_ptr(cands, "int32", 2 * n), n,
            _dev_ptr(cost, "int32", n), _dev_ptr(status, "int32", n),
            None if comps is None else _dev_ptr(comps, "int32", 5 * n)))

    def eval_successors_noalloc(self, parent, cands, cost, status, comps=None):
        """eval_successors without device allocation: the parent buffers are the
        library's fixed per-GPU array (shared by every such call on the GPU)."""
        n = cands.shape[0]
        par = _objects(parent)
        _check(load().perch_eval_successors_noalloc(
            self.h, C.cast(par, C.c_void_p), len(parent), _dev_ptr(cands, "int32", 2 * n), n,
            _dev_ptr(cost, "int32", n), _dev_ptr(status, "int32", n),
            None if comps is None else _dev_ptr(comps, "int32", 5 * n)))

    def set_parent(self, parent):
        """Materialises the parent state R_j (and U at the goal level)."""
        _check(load().perch_set_parent(self.h, C.cast(_objects(parent), C.c_void_p),
                                       len(parent)))

    def eval_children(self, cands, cost, status, comps=None):
        """Successors of the parent last set; same tensors as eval_successors."""
        n = cands.shape[0]
        _check(load().perch_eval_children(
            self.h, _dev_ptr(cands, "int32", 2 * n), n, _dev_ptr(cost, "int32", n),
            _dev_ptr(status, "int32", n),
            None if comps is None else _dev_ptr(comps, "int32", 5 * n)))

    def overlap_gain(self, cands, cost, status, gain):
        """Successors of the parent last set (as eval_children) and, per successor,
        the observed points its volume adds to the parent's V_j (the decrease of the
        overlap heuristic, Sec. IV-C; -1 when not valid).  Asynchronous."""
        n = cands.shape[0]
        _check(load().perch_overlap_gain(
            self.h, _dev_ptr(cands, "int32", 2 * n), n, _dev_ptr(cost, "int32", n),
            _dev_ptr(status, "int32", n), _dev_ptr(gain, "int32", n)))

    def evaluate(self, parent, cands, with_comps: bool = True):
        """Convenience: allocates outputs, evaluates and returns GPU tensors."""
        import torch

        n = cands.shape[0]
        dev = cands.device
        cost = torch.empty(n, dtype=torch.int32, device=dev)
        status = torch.empty(n, dtype=torch.int32, device=dev)
        comps = torch.empty((n, 5), dtype=torch.int32, device=dev) if with_comps else None
        self.eval_successors(parent, cands, cost, status, comps)
        return status, cost, comps

    def set_symmetric(self, mesh_id: int, symmetric: bool = True):
        """The searches try a rotationally symmetric mesh once per (x, y)."""
        _check(load().perch_set_symmetric(self.h, int(mesh_id), int(bool(symmetric))))

    def set_pose_arena(self, capacity: int):
        """Room for `capacity` ICP-adjusted poses after the grid (empties it)."""
        _check(load().perch_set_pose_arena(self.h, int(capacity)))

    def get_poses(self, first: int, n: int) -> np.ndarray:
        """Poses [first, first + n) of the table (grid, then arena), (n, 4) float32."""
        out = np.zeros((max(n, 1), 4), np.float32)
        _check(load().perch_get_poses(self.h, int(first), int(n), out.ctypes.data))
        return out[:n]

    def rank_children(self, pred, n_poses: int, allow, k: int, mesh_ids, pose_ids):
        """The learned search's ranking step: (k, 2) int32 GPU tensor of (mesh, pose)
        for the k smallest of the n_meshes x n_poses predictions pred (float32 GPU
        tensor, child u * n_poses + b), ties by child index, mesh positions with
        allow[u] == 0 last; mesh_ids / pose_ids: int32 GPU tensors."""
        import torch

        allow = np.ascontiguousarray(allow, np.int32)
        n_meshes = len(allow)
        n = n_meshes * int(n_poses)
        out = torch.empty((max(int(k), 1), 2), dtype=torch.int32, device="cuda")
        _check(load().perch_rank_children(self.h, _dev_ptr(pred, "float32", n), int(n_poses),
                                          n_meshes, allow.ctypes.data, int(k),
                                          _dev_ptr(mesh_ids, "int32", n_meshes),
                                          _dev_ptr(pose_ids, "int32", int(n_poses)),
                                          out.data_ptr()))
        return out[:int(k)]

    def icp_children(self, cands, adjusted, n_match, status, iters: int = 10,
                     radius: float = 0.02):
        """Local ICP (Sec. IV-E) of the successors of the parent last set: cands and
        adjusted int32 GPU tensors (n, 2) (adjusted = (mesh, arena pose index)),
        n_match and status int32 GPU tensors (n,).  Asynchronous."""
        n = cands.shape[0]
        _check(load().perch_icp_children(
            self.h, _dev_ptr(cands, "int32", 2 * n), n, int(iters), float(radius),
            _dev_ptr(adjusted, "int32", 2 * n), _dev_ptr(n_match, "int32", n),
            _dev_ptr(status, "int32", n)))

    def search(self, mode: int = SEARCH_UCS, w: float = 1.0, anytime: bool = False,
               budget_s: float = 0.0, budget_expansions: int = 0, pose_subset=None,
               cnn: "Optional[Cnn]" = None, topk: int = 64, icp_iters: int = 0,
               icp_radius: float = 0.02, priors=None, prior_rad_m: float = 0.0,
               prior_slot_m: float = 0.0, batch: int = 1) -> dict:
        """Tree search of Alg. 1 on this scene (synchronous).  Returns the goal in
        insertion order plus its canonical (sorted) form, cost and statistics."""
        o = _SearchOpts()
        o.mode, o.w, o.anytime = int(mode), float(w), int(bool(anytime))
        o.budget_s, o.budget_expansions = float(budget_s), int(budget_expansions)
        o.cnn = None if cnn is None else cnn.h.value
        o.topk = int(topk)
        o.icp_iters, o.icp_radius = int(icp_iters), float(icp_radius)
        o.batch = int(batch)
        pri = None
        if priors is not None and len(priors):  # [(mesh, x, y, theta), ...]
            pri = (PerchPosePrior * len(priors))()
            for k, (m, x, y, th) in enumerate(priors):
                pri[k].mesh_id, pri[k].x, pri[k].y, pri[k].theta = int(m), x, y, th
            o.priors, o.n_priors = C.cast(pri, C.c_void_p), len(priors)
        o.prior_rad_m, o.prior_slot_m = float(prior_rad_m), float(prior_slot_m)
        sub = None
        if pose_subset is not None:
            sub = np.ascontiguousarray(pose_subset, np.int32)
            o.pose_subset, o.n_pose_subset = sub.ctypes.data, len(sub)
        r = _Result()
        rc = load().perch_search(self.h, C.byref(o), C.byref(r))
        if rc not in (0, -6):
            _check(rc)
        objs = [(r.objs[k].mesh_id, r.objs[k].pose_idx) for k in range(r.K)] if r.found else []
        return dict(found=bool(r.found), budget_exhausted=(rc == -6), objs=objs,
                    canonical=sorted(objs), cost=int(r.cost),
                    edge_cost=[int(r.edge_cost[k]) for k in range(r.K)] if r.found else [],
                    n_expanded=int(r.n_expanded), n_evaluated=int(r.n_evaluated),
                    n_invalid=int(r.n_invalid), t_total_s=float(r.t_total_s),
                    t_best_s=float(r.t_best_s), lower_bound=int(r.lower_bound),
                    n_evaluated_best=int(r.n_evaluated_best), n_merged=int(r.n_merged),
                    trace=[(float(r.trace_t[k]), int(r.trace_cost[k]), int(r.trace_lb[k]))
                           for k in range(r.n_trace)])

    def render(self, objs, composite: bool = True):
        """Depth images (+inf = empty) of objects [(mesh, pose), ...]."""
        import torch

        n = len(objs)
        shape = (self.H, self.W) if composite else (n, self.H, self.W)
        out = torch.empty(shape, dtype=torch.float32, device="cuda")
        _check(load().perch_render(self.h, C.cast(_objects(objs), C.c_void_p), n,
                                   1 if composite else 0, out.data_ptr()))
        return out


class Batch:
    """Successors of many parents of many scenes in one persistent, graph-replayed
    launch (work items (parent slot, mesh, pose, 0) as an int32 GPU tensor (n, 4))."""

    def __init__(self, contexts, stream=None):
        import torch

        self.contexts = list(contexts)  # keeps them alive
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        arr = (C.c_void_p * len(self.contexts))(*[c.h.value for c in self.contexts])
        h = C.c_void_p()
        _check(load().perch_batch_create(C.cast(arr, C.c_void_p), len(self.contexts),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().perch_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, threads: int = 0, tile_px: int = 0, use_graph: int = -1, grid: int = -1):
        _check(load().perch_batch_set_tuning(self.h, threads, tile_px, use_graph, grid))

    def autotune(self, items, reps: int = 3, cache_path: Optional[str] = None) -> dict:
        """Times the batched launch's settings on the calibration work list `items`
        (int32 GPU tensor (n, 4)) over the parents last set, applies the fastest
        (outputs bit-identical across settings) and returns it with the time of the
        setting in force before."""
        t = _BatchTuning()
        n = items.shape[0]
        _check(load().perch_batch_autotune(self.h, _dev_ptr(items, "int32", 4 * n), n, reps,
                                           None if cache_path is None else cache_path.encode(),
                                           C.byref(t)))
        return dict(threads=t.threads, tile_px=t.tile_px, radius_mode=t.radius_mode,
                    cell_over_delta=t.cell_over_delta, ms=t.ms, default_ms=t.default_ms)

    def set_parents(self, parents):
        """parents: list of (context index, [(mesh, pose), ...])."""
        arr = (PerchParent * max(1, len(parents)))()
        for k, (ci, objs) in enumerate(parents):
            arr[k].ctx = int(ci)
            arr[k].j = len(objs)
            for o, (m, p) in enumerate(objs):
                arr[k].objs[o].mesh_id = int(m)
                arr[k].objs[o].pose_idx = int(p)
        _check(load().perch_batch_set_parents(self.h, C.cast(arr, C.c_void_p), len(parents)))

    def eval(self, items, cost, status, comps=None):
        n = items.shape[0]
        _check(load().perch_batch_eval(
            self.h, _dev_ptr(items, "int32", 4 * n), n, _dev_ptr(cost, "int32", n),
            _dev_ptr(status, "int32", n),
            None if comps is None else _dev_ptr(comps, "int32", 5 * n)))


# flat parameter order of the network (sizes depend on the number of meshes)
CNN_TENSORS = ("cW0", "cb0", "cW1", "cb1", "cW2", "cb2", "cW3", "cb3", "emb", "hW1", "hb1",
               "hw2", "hb2")


def cnn_shapes(n_mesh: int):
    shp = {}
    cin = 2
    for l in range(4):
        shp[f"cW{l}"] = (32, 3, 3, cin)
        shp[f"cb{l}"] = (32,)
        cin = 32
    shp.update(emb=(n_mesh, 16), hW1=(64, 82), hb1=(64,), hw2=(64,), hb2=(1,))
    return shp


class Cnn:
    """The learned successor-cost network on the GPU (inference and training)."""

    def __init__(self, n_mesh: int, max_crops: int = 256, max_pairs: int = 8192, stream=None):
        import torch

        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.n_mesh = n_mesh
        h = C.c_void_p()
        _check(load().perch_cnn_create(n_mesh, max_crops, max_pairs,
                                       C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.n_params = int(load().perch_cnn_param_count(self.h))
        self.crop_step = 1

    def close(self):
        if getattr(self, "h", None):
            load().perch_cnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, params: dict) -> np.ndarray:
        shp = cnn_shapes(self.n_mesh)
        return np.concatenate([np.asarray(params[k], np.float32).reshape(-1) for k in CNN_TENSORS])

    def unpack(self, flat: np.ndarray) -> dict:
        out, o = {}, 0
        for k in CNN_TENSORS:
            s = cnn_shapes(self.n_mesh)[k]
            n = int(np.prod(s))
            out[k] = flat[o:o + n].reshape(s)
            o += n
        return out

    def set_params(self, params):
        flat = np.ascontiguousarray(self.pack(params) if isinstance(params, dict) else params,
                                    np.float32)
        _check(load().perch_cnn_set_params(self.h, flat.ctypes.data, self.n_params))

    def get_params(self) -> dict:
        flat = np.zeros(self.n_params, np.float32)
        _check(load().perch_cnn_get_params(self.h, flat.ctypes.data, self.n_params))
        return self.unpack(flat)

    def set_crop_step(self, step: int):
        """Pixel step of the crops the learned search takes for this network."""
        _check(load().perch_cnn_set_crop_step(self.h, int(step)))
        self.crop_step = int(step)

    @staticmethod
    def crops(ctx: "Context", xy, step: int = 1):
        """bfloat16 crops (as an int16 GPU tensor n x 64 x 64 x 2) of ctx's parent, one
        sample every `step` pixels."""
        import torch

        xy = np.ascontiguousarray(xy, np.float32).reshape(-1, 2)
        out = torch.empty((len(xy), 64, 64, 2), dtype=torch.int16, device="cuda")
        if step == 1:
            _check(load().perch_cnn_crops(ctx.h, xy.ctypes.data, len(xy), out.data_ptr()))
        else:
            _check(load().perch_cnn_crops_step(ctx.h, xy.ctypes.data, len(xy), int(step),
                                               out.data_ptr()))
        return out

    @staticmethod
    def pairs(crop, mesh, cos_yaw, sin_yaw):
        """int32 GPU tensor (n, 4) of (crop, mesh, cos bits, sin bits)."""
        import torch

        a = np.zeros((len(crop), 4), np.int32)
        a[:, 0] = crop
        a[:, 1] = mesh
        a[:, 2] = np.asarray(cos_yaw, np.float32).view(np.int32)
        a[:, 3] = np.asarray(sin_yaw, np.float32).view(np.int32)
        return torch.as_tensor(a).cuda()

    def predict(self, crops, pairs):
        import torch

        out = torch.empty(pairs.shape[0], dtype=torch.float32, device="cuda")
        _check(load().perch_cnn_predict(self.h, crops.data_ptr(), crops.shape[0], pairs.data_ptr(),
                                        pairs.shape[0], out.data_ptr()))
        return out

    def predict_scene(self, ctx, xy, pairs):
        """predict() of the crops Cnn.crops(ctx, xy, self.crop_step) would make, sampled
        inside the network's first kernel (perch_cnn_predict_scene)."""
        import torch

        xy = np.ascontiguousarray(xy, np.float32).reshape(-1, 2)
        out = torch.empty(pairs.shape[0], dtype=torch.float32, device="cuda")
        _check(load().perch_cnn_predict_scene(self.h, ctx.h, xy.ctypes.data, len(xy),
                                              pairs.data_ptr(), pairs.shape[0], out.data_ptr()))
        return out

    def train_step(self, crops, pairs, target, lr: float, want_loss: bool = True):
        loss = C.c_float(0.0)
        _check(load().perch_cnn_train_step(self.h, crops.data_ptr(), crops.shape[0],
                                           pairs.data_ptr(), _dev_ptr(target, "float32"),
                                           pairs.shape[0], lr,
                                           C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def gradients(self, crops, pairs, target):
        g = np.zeros(self.n_params, np.float32)
        loss = C.c_float(0.0)
        _check(load().perch_cnn_gradients(self.h, crops.data_ptr(), crops.shape[0],
                                          pairs.data_ptr(), _dev_ptr(target, "float32"),
                                          pairs.shape[0], g.ctypes.data, C.byref(loss)))
        return loss.value, self.unpack(g)


# flat parameter order of the pose regressor (sizes depend on meshes and yaw bins)
POSENET_TENSORS = ("cW0", "cb0", "cW1", "cb1", "cW2", "cb2", "cW3", "cb3", "emb", "W1", "b1",
                   "W2", "b2")


def posenet_shapes(n_mesh: int, n_yaw: int):
    shp = {}
    cin = 2
    for l in range(4):
        shp[f"cW{l}"] = (32, 3, 3, cin)
        shp[f"cb{l}"] = (32,)
        cin = 32
    shp.update(emb=(n_mesh, 16), W1=(64, 80), b1=(64,), W2=(3 + n_yaw, 64), b2=(3 + n_yaw,))
    return shp


class PoseNet:
    """The per-object pose regressor on the GPU (inference, estimates, training)."""

    def __init__(self, n_mesh: int, n_yaw: int, max_crops: int = 256, max_pairs: int = 2048,
                 stream=None):
        import torch

        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.n_mesh, self.n_yaw = n_mesh, n_yaw
        self.max_crops, self.max_pairs = max_crops, max_pairs
        h = C.c_void_p()
        _check(load().perch_posenet_create(n_mesh, n_yaw, max_crops, max_pairs,
                                           C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.n_params = int(load().perch_posenet_param_count(self.h))

    def close(self):
        if getattr(self, "h", None):
            load().perch_posenet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, params: dict) -> np.ndarray:
        return np.concatenate([np.asarray(params[k], np.float32).reshape(-1)
                               for k in POSENET_TENSORS])

    def unpack(self, flat: np.ndarray) -> dict:
        out, o = {}, 0
        shp = posenet_shapes(self.n_mesh, self.n_yaw)
        for k in POSENET_TENSORS:
            n = int(np.prod(shp[k]))
            out[k] = flat[o:o + n].reshape(shp[k])
            o += n
        return out

    def set_params(self, params):
        flat = np.ascontiguousarray(self.pack(params) if isinstance(params, dict) else params,
                                    np.float32)
        _check(load().perch_posenet_set_params(self.h, flat.ctypes.data, self.n_params))

    def get_params(self) -> dict:
        flat = np.zeros(self.n_params, np.float32)
        _check(load().perch_posenet_get_params(self.h, flat.ctypes.data, self.n_params))
        return self.unpack(flat)

    @staticmethod
    def crops(ctx: "Context", xy, step: int = 1):
        """bfloat16 crops (int16 GPU tensor n x 64 x 64 x 2) of ctx's parent, one sample
        every `step` pixels."""
        import torch

        xy = np.ascontiguousarray(xy, np.float32).reshape(-1, 2)
        out = torch.empty((len(xy), 64, 64, 2), dtype=torch.int16, device="cuda")
        _check(load().perch_cnn_crops_step(ctx.h, xy.ctypes.data, len(xy), int(step),
                                           out.data_ptr()))
        return out

    @staticmethod
    def pairs(crop, mesh):
        """int32 GPU tensor (n, 2) of (crop, mesh)."""
        import torch

        a = np.stack([np.asarray(crop, np.int32), np.asarray(mesh, np.int32)], 1)
        return torch.as_tensor(np.ascontiguousarray(a)).cuda()

    @staticmethod
    def targets(t):
        """float32 GPU tensor (n, 5) of (label, dx, dy, yaw bin, period)."""
        import torch

        return torch.as_tensor(np.ascontiguousarray(t, np.float32).reshape(-1, 5)).cuda()

    def predict(self, crops, pairs):
        import torch

        out = torch.empty((pairs.shape[0], 3 + self.n_yaw), dtype=torch.float32, device="cuda")
        _check(load().perch_posenet_predict(self.h, crops.data_ptr(), crops.shape[0],
                                            _dev_ptr(pairs, "int32", 2 * pairs.shape[0]),
                                            pairs.shape[0], out.data_ptr()))
        return out

    def predict_scene(self, ctx, xy, pairs):
        """predict() of the crops Cnn.crops(ctx, xy, self.crop_step) would make, sampled
        inside the network's first kernel (perch_cnn_predict_scene)."""
        import torch

        xy = np.ascontiguousarray(xy, np.float32).reshape(-1, 2)
        out = torch.empty(pairs.shape[0], dtype=torch.float32, device="cuda")
        _check(load().perch_cnn_predict_scene(self.h, ctx.h, xy.ctypes.data, len(xy),
                                              pairs.data_ptr(), pairs.shape[0], out.data_ptr()))
        return out

    def train_step(self, crops, pairs, target, lr: float, want_loss: bool = True):
        loss = C.c_float(0.0)
        _check(load().perch_posenet_train_step(self.h, crops.data_ptr(), crops.shape[0],
                                               _dev_ptr(pairs, "int32", 2 * pairs.shape[0]),
                                               _dev_ptr(target, "float32", 5 * pairs.shape[0]),
                                               pairs.shape[0], lr,
                                               C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def gradients(self, crops, pairs, target):
        g = np.zeros(self.n_params, np.float32)
        loss = C.c_float(0.0)
        _check(load().perch_posenet_gradients(self.h, crops.data_ptr(), crops.shape[0],
                                              _dev_ptr(pairs, "int32", 2 * pairs.shape[0]),
                                              _dev_ptr(target, "float32", 5 * pairs.shape[0]),
                                              pairs.shape[0], g.ctypes.data, C.byref(loss)))
        return loss.value, self.unpack(g)

    def estimate(self, crops, anchor_xy, spacing: float, meshes, counts, nms_m: float):
        """[(mesh, x, y, theta), ...] from one crop per anchor (perch_posenet_estimate)."""
        xy = np.ascontiguousarray(anchor_xy, np.float32).reshape(-1, 2)
        m = np.ascontiguousarray(meshes, np.int32)
        c = np.ascontiguousarray(counts, np.int32)
        cap = int(c.sum())
        out = (PerchPosePrior * max(1, cap))()
        n = C.c_int32(0)
        _check(load().perch_posenet_estimate(self.h, crops.data_ptr(), len(xy), xy.ctypes.data,
                                             float(spacing), float(nms_m), m.ctypes.data,
                                             c.ctypes.data, len(m), out, cap, C.byref(n)))
        return [(int(out[k].mesh_id), float(out[k].x), float(out[k].y), float(out[k].theta))
                for k in range(n.value)]


def context_from_scene(scene, depth=None, stream=None) -> Context:
    """Context loaded with a generated scene (observation on the GPU)."""
    import torch

    ctx = Context(scene.sensor, stream)
    for m, mesh in enumerate(scene.library.meshes):
        ctx.add_mesh(m, mesh.verts, mesh.tris, mesh.planes)
    ctx.set_poses(scene.poses)
    ctx.set_objects(scene.obj_mesh)
    d = scene.depth_obs if depth is None else depth
    ctx.set_observation(torch.as_tensor(np.ascontiguousarray(d, np.float32)).cuda())
    return ctx


class GpuRenderer:
    """Renderer callback for the scene generator, backed by perch_render."""

    def __init__(self):
        self._cache = {}

    def __call__(self, sensor, library, mesh_ids, pose_idx, poses):
        key = (id(sensor), id(library), id(poses))
        ctx = self._cache.get(key)
        if ctx is None:
            ctx = Context(sensor)
            for m, mesh in enumerate(library.meshes):
                ctx.add_mesh(m, mesh.verts, mesh.tris, mesh.planes)
            ctx.set_poses(poses)
            self._cache = {key: ctx}
        D = ctx.render(list(zip(mesh_ids, pose_idx)), composite=False)
        return D.double().cpu().numpy()
