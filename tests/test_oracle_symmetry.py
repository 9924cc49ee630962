"""Pins of the oracle's searches with rotationally symmetric objects and with
replicated instances (Sec. IV-E: a symmetric object only needs (x, y); identical
objects are one mesh id placed several times).  Tree search (exhaustive and
uniform-cost) must equal brute force over joint assignments under the same pose
restriction, the restriction must try exactly one pose per (x, y) cell, and a
replicated scene must be searched over sets, not orders."""
import numpy as np
import pytest

from oracle import Oracle, render_fn
from paper_1510_05613_amd import scenes
from tests import helpers as H


def _xy_first(sc, sub):
    """First pose of sub at each distinct (x, y), in sub order (the rule)."""
    seen, out = set(), []
    for p in sub:
        key = (float(sc.poses[p, 0]), float(sc.poses[p, 1]))
        if key not in seen:
            seen.add(key)
            out.append(int(p))
    return np.array(out, np.int32)


@pytest.mark.parametrize("scene_idx", [0, 1])
def test_symmetric_mesh_search_equals_bruteforce(scene_idx):
    sc = H.c1_scene(scene_idx)
    sub = scenes.pose_subset_around(sc, 1, yaw_stride=1)
    o = Oracle.from_scene(sc, nthreads=8)
    m_sym = int(sc.obj_mesh[0])
    o.set_symmetric(m_sym)
    ex, bf, uc = o.search_exhaustive(sub), o.bruteforce_joint(sub), o.search_ucs(sub)
    assert ex["found"] and bf["found"] and uc["found"]
    assert ex["cost"] == bf["cost"] == uc["cost"]
    assert np.array_equal(ex["mesh"], bf["mesh"]) and np.array_equal(ex["pose"], bf["pose"])
    # the symmetric mesh sits at the first pose of its (x, y) cell
    allowed = set(_xy_first(sc, sub).tolist())
    for m, p in zip(ex["mesh"], ex["pose"]):
        if int(m) == m_sym:
            assert int(p) in allowed
    # evaluation count of the exhaustive tree: the root tries |L(a)| + |L(b)|
    # children; every valid child of one mesh is expanded over the other's list
    a, b = int(sc.obj_mesh[0]), int(sc.obj_mesh[1])
    La, Lb = _xy_first(sc, sub), sub
    st_a, *_ = o.eval([], [], np.full(len(La), a), La)
    st_b, *_ = o.eval([], [], np.full(len(Lb), b), Lb)
    expect = len(La) + len(Lb) + int(st_a.sum()) * len(Lb) + int(st_b.sum()) * len(La)
    assert ex["n_eval"] == expect
    # unrestricted: more evaluations, and a cost no higher
    o.set_symmetric(m_sym, False)
    full = o.search_exhaustive(sub)
    assert full["n_eval"] > ex["n_eval"] and full["cost"] <= ex["cost"]


def test_xy_restriction_keeps_one_pose_per_cell():
    sc = H.c1_scene(0)
    g = sc.grid
    L = _xy_first(sc, np.arange(g.P, dtype=np.int32))
    assert len(L) == g.nx * g.ny
    assert all(g.unindex(int(p))[2] == 0 for p in L)  # yaw index 0 comes first per cell


def _replicated_scene(idx):
    lib = H.c1_library()
    one = scenes.Library([lib.meshes[2]])  # a single hull, placed twice
    return scenes.make_scene(1, 200 + idx, render_fn, one, overrides=dict(K=(2, 2)))


@pytest.mark.parametrize("idx", [0, 1])
def test_replicated_instances_are_searched_as_sets(idx):
    """Two identical objects: the known multiset holds one mesh id twice.  The
    tree search places 'the' mesh twice and equals brute force; uniform-cost search
    merges the two orders of one pair of poses (canonical states), so it evaluates
    fewer successors than the exhaustive tree."""
    sc = _replicated_scene(idx)
    assert sc.obj_mesh[0] == sc.obj_mesh[1]
    sub = scenes.pose_subset_around(sc, 1, yaw_stride=2)
    o = Oracle.from_scene(sc, nthreads=8)
    ex, bf, uc = o.search_exhaustive(sub), o.bruteforce_joint(sub), o.search_ucs(sub)
    assert ex["cost"] == bf["cost"] == uc["cost"]
    # the exhaustive tree: n roots, each valid root expanded over n poses
    st, *_ = o.eval([], [], np.zeros(len(sub), np.int32), sub)
    assert ex["n_eval"] == len(sub) + int(st.sum()) * len(sub)
    assert uc["n_eval"] <= ex["n_eval"]
