"""The learned search mode (a focal search whose inadmissible queue holds the
network's top-k children, Sec. IV-C) and the network's checkpoints.  Whatever the
network predicts, the anchor queue and the lazy blocks keep the search complete:
run to the end it returns the exhaustive optimum, and stopped at the focal bound
it returns a goal within w of it (Theorem 2)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1510_05613_amd import learn, perch, scenes  # noqa: E402

CKPT = os.path.join(os.path.dirname(learn.__file__), "weights", "c4_cnn.npz")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    perch.load()


_LIB = {}


def held_out_scene(k):
    lib = _LIB.setdefault("c1", scenes.make_library("c1"))
    return scenes.make_scene(4, learn.HELD_OUT_FIRST + k, perch.GpuRenderer(), library=lib)


def random_net(seed=5):
    net = perch.Cnn(3, max_crops=144, max_pairs=3 * 1152)
    net.set_params(learn.init_params(3, seed))
    return net


def test_checkpoint_round_trip(tmp_path):
    net = random_net(3)
    path = str(tmp_path / "net.npz")
    learn.save(net, path, steps=0)
    back = learn.load(path, max_crops=144, max_pairs=3 * 1152)
    a, b = net.get_params(), back.get_params()
    assert set(a) == set(b) == set(perch.CNN_TENSORS)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    sc = held_out_scene(0)
    ctx = perch.context_from_scene(sc)
    ctx.set_parent([])
    crops = perch.Cnn.crops(ctx, learn.cell_centres(sc.grid))
    g = sc.grid
    cell = np.arange(g.P) // g.n_yaw
    pairs = perch.Cnn.pairs(cell, np.zeros(g.P, np.int32), sc.poses[:, 2], sc.poses[:, 3])
    assert torch.equal(net.predict(crops, pairs), back.predict(crops, pairs))


def test_learned_search_needs_a_network():
    sc = held_out_scene(0)
    ctx = perch.context_from_scene(sc)
    with pytest.raises(perch.PerchError):
        ctx.search(perch.SEARCH_LEARNED, w=2.0)


LEARNED_MODES = [perch.SEARCH_LEARNED, perch.SEARCH_LEARNED_MHA]


@pytest.mark.parametrize("mode", LEARNED_MODES)
@pytest.mark.parametrize("k", [0, 1, 2])
@pytest.mark.parametrize("topk", [1, 64])
def test_learned_anytime_reaches_the_exhaustive_optimum(k, topk, mode):
    """Any network, any k: run until the anchor's bound meets the incumbent, the
    learned search (with or without the h_overlap queue) returns the optimum of
    the whole tree."""
    sc = held_out_scene(k)
    ctx = perch.context_from_scene(sc)
    ex = ctx.search(perch.SEARCH_EXHAUSTIVE)
    r = ctx.search(mode, w=2.0, anytime=True, cnn=random_net(k), topk=topk)
    assert r["found"] and not r["budget_exhausted"]
    assert r["cost"] == ex["cost"]
    assert r["lower_bound"] >= r["cost"]  # the search proved its goal optimal
    assert sum(r["edge_cost"]) == r["cost"]
    assert 0 <= r["n_evaluated_best"] <= r["n_evaluated"]


@pytest.mark.parametrize("mode", LEARNED_MODES)
@pytest.mark.parametrize("w", [1.0, 1.5, 3.0])
def test_learned_first_goal_within_w(w, mode):
    sc = held_out_scene(3)
    ctx = perch.context_from_scene(sc)
    opt = ctx.search(perch.SEARCH_UCS)["cost"]
    r = ctx.search(mode, w=w, anytime=False, cnn=random_net(1), topk=32)
    assert r["found"]
    assert r["cost"] <= w * opt + 1e-9
    assert r["lower_bound"] <= opt


def test_learned_budget_keeps_incumbent():
    sc = held_out_scene(4)
    ctx = perch.context_from_scene(sc)
    r = ctx.search(perch.SEARCH_LEARNED, w=3.0, anytime=True, budget_expansions=3,
                   cnn=random_net(2), topk=16)
    assert r["budget_exhausted"] or r["lower_bound"] >= r["cost"]
    assert r["n_expanded"] <= 3
    if r["found"]:
        assert r["cost"] >= r["lower_bound"]


@pytest.mark.skipif(not os.path.exists(CKPT), reason="no trained checkpoint")
def test_trained_network_finds_the_best_scene_sooner():
    """Config-4 gain test on held-out scenes: evaluations until the exhaustive
    optimum is first held, learned (trained network) against the plain exhaustive
    search and against the same learned search with a random-init network."""
    net = learn.load(CKPT, max_crops=144, max_pairs=3 * 1152)
    ctrl = random_net(0)
    ln, pl, rc = [], [], []
    for k in range(20):
        sc = held_out_scene(k)
        ctx = perch.context_from_scene(sc)
        ex = ctx.search(perch.SEARCH_EXHAUSTIVE)
        a = ctx.search(perch.SEARCH_LEARNED, w=3.0, anytime=True, cnn=net, topk=64)
        b = ctx.search(perch.SEARCH_LEARNED, w=3.0, anytime=True, cnn=ctrl, topk=64)
        assert a["cost"] == b["cost"] == ex["cost"]
        ln.append(a["n_evaluated_best"])
        rc.append(b["n_evaluated_best"])
        pl.append(ex["n_evaluated_best"])
    assert np.median(ln) < np.median(pl)
    assert np.median(ln) < np.median(rc)


def batched_net(seed, B):
    net = perch.Cnn(3, max_crops=144 * B, max_pairs=3 * 1152 * B)
    net.set_params(learn.init_params(3, seed))
    return net


@pytest.mark.parametrize("B", [2, 8])
@pytest.mark.parametrize("k", [0, 1])
@pytest.mark.parametrize("topk", [1, 64])
def test_learned_batched_anytime_reaches_the_exhaustive_optimum(k, topk, B):
    """Several states per step (one batched exact launch per step): run to the end,
    the search still returns the optimum of the whole tree, proved by its bound."""
    sc = held_out_scene(k)
    ctx = perch.context_from_scene(sc)
    ex = ctx.search(perch.SEARCH_EXHAUSTIVE)
    r = ctx.search(perch.SEARCH_LEARNED, w=2.0, anytime=True, cnn=batched_net(k, B), topk=topk,
                   batch=B)
    assert r["found"] and not r["budget_exhausted"]
    assert r["cost"] == ex["cost"]
    assert r["lower_bound"] >= r["cost"]
    assert sum(r["edge_cost"]) == r["cost"]
    # the path re-evaluates to its edge costs through the single-parent entry point
    objs = r["objs"]
    for j in range(len(objs)):
        c = torch.as_tensor(np.array([objs[j]], np.int32)).cuda()
        st, cost, _ = ctx.evaluate(objs[:j], c)
        torch.cuda.synchronize()
        assert int(st[0]) == 1 and int(cost[0]) == r["edge_cost"][j]


@pytest.mark.parametrize("w", [1.0, 3.0])
def test_learned_batched_first_goal_within_w(w):
    sc = held_out_scene(3)
    ctx = perch.context_from_scene(sc)
    opt = ctx.search(perch.SEARCH_UCS)["cost"]
    r = ctx.search(perch.SEARCH_LEARNED, w=w, anytime=False, cnn=batched_net(1, 4), topk=32,
                   batch=4)
    assert r["found"]
    assert r["cost"] <= w * opt + 1e-9
    assert r["lower_bound"] <= opt


def test_learned_batched_needs_network_capacity():
    """A network sized for one state per step is refused for a batched search (the
    crops of B states do not fit), and h_overlap is a single-state queue."""
    sc = held_out_scene(0)
    ctx = perch.context_from_scene(sc)
    with pytest.raises(perch.PerchError):
        ctx.search(perch.SEARCH_LEARNED, w=2.0, anytime=True, cnn=random_net(0), batch=4)
    with pytest.raises(perch.PerchError):
        ctx.search(perch.SEARCH_LEARNED_MHA, w=2.0, anytime=True, cnn=batched_net(0, 4), batch=4)


def test_crop_step_is_the_networks_and_keeps_the_optimum():
    """A network's crop step reaches the learned search's crops (strided crops equal
    perch_cnn_crops_step's), bad steps are refused, and the search stays exact."""
    net = random_net(3)
    assert net.crop_step == 1
    with pytest.raises(perch.PerchError):
        net.set_crop_step(0)
    with pytest.raises(perch.PerchError):
        net.set_crop_step(65)
    net.set_crop_step(3)
    sc = held_out_scene(2)
    ctx = perch.context_from_scene(sc)
    ctx.set_parent([])
    xy = learn.cell_centres(sc.grid)[:5]
    a = perch.Cnn.crops(ctx, xy, 3).cpu().numpy()
    b = perch.PoseNet.crops(ctx, xy, 3).cpu().numpy()
    assert np.array_equal(a, b)
    assert not np.array_equal(a, perch.Cnn.crops(ctx, xy).cpu().numpy())
    ex = ctx.search(perch.SEARCH_EXHAUSTIVE)
    r = ctx.search(perch.SEARCH_LEARNED, w=2.0, anytime=True, cnn=net, topk=16)
    assert r["found"] and r["cost"] == ex["cost"] and r["lower_bound"] >= r["cost"]
