"""The learned search's ranking step (Sec. IV-C: only the children the learned
heuristic ranks best reach the inadmissible queue), through the C ABI, against
its plain definition: the first k entries of a stable ascending sort of the
predictions, with the children of meshes already placed ranked as +inf and -0
equal to +0.  Up to 8192 children one workgroup selects them; beyond that
workgroups select each 8192-child chunk's k best and one more selection merges
them while those candidates fit it, and a device radix sort does the rest; every
path is covered, with heavy ties, signed zeros, masks and k up to the selection's
limit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1510_05613_amd import perch  # noqa: E402
from tests import helpers as H  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    perch.load()
    return perch.context_from_scene(H.c1_scene(0))


def _expected(pred, n_poses, allow, k, mesh_ids, pose_ids):
    """First k of a stable argsort of the masked predictions, as (mesh, pose)."""
    p = pred.astype(np.float32).copy()
    p[p == 0] = 0.0  # -0 ranks with +0
    for u, a in enumerate(allow):
        if not a:
            p[u * n_poses:(u + 1) * n_poses] = np.inf
    idx = np.argsort(p, kind="stable")[:k]
    return np.stack([mesh_ids[idx // n_poses], pose_ids[idx % n_poses]], 1)


def _preds(rng, n, kind):
    if kind == "normal":
        return rng.normal(size=n).astype(np.float32)
    if kind == "ties":  # a handful of values, signed zeros among them
        return rng.choice(np.array([0.25, 1.0, -0.0, 0.0, 3.0, -2.0], np.float32), size=n)
    # a learned cost: log(1 + cost) of integer costs, many exact repeats
    return np.log1p(rng.integers(0, 40, size=n)).astype(np.float32)


CASES = [
    # (n_meshes, n_poses, k, allow, kind)
    (1, 1, 1, (1,), "normal"),
    (1, 7, 7, (1,), "ties"),
    (2, 1152, 64, (1, 1), "costs"),  # the 160 x 120 learned scenes' child count
    (2, 1152, 64, (0, 1), "costs"),  # one mesh placed already
    (3, 700, 1024, (1, 0, 1), "ties"),
    (8, 1024, 1024, (1, 1, 0, 1, 1, 1, 1, 0), "normal"),  # n = 8192, the limit
    (8, 1024, 8192, (1,) * 8, "ties"),  # k above the selection's limit: sorted
    (1, 8193, 64, (1,), "ties"),  # one child over the limit: two chunks
    (1, 8292, 200, (1,), "ties"),  # the second chunk holds fewer children than k
    (5, 20000, 400, (1, 0, 1, 1, 0), "ties"),  # 13 chunks, heavy ties across them
    (3, 40000, 256, (1, 0, 1), "costs"),  # the 640 x 480 scenes' child count
    (3, 40000, 1024, (1, 1, 1), "costs"),  # too many chunk candidates: sorted
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-k{c[2]}-{c[4]}" for c in CASES])
def test_rank_children_equals_stable_sort(ctx, case):
    nm, P, k, allow, kind = case
    rng = np.random.default_rng(nm * 100003 + P + k)
    pred = _preds(rng, nm * P, kind)
    mesh_ids = rng.permutation(16)[:nm].astype(np.int32)
    pose_ids = rng.permutation(max(P, 1) * 3)[:P].astype(np.int32)
    d_pred = torch.as_tensor(pred).cuda()
    got = ctx.rank_children(d_pred, P, allow, k, torch.as_tensor(mesh_ids).cuda(),
                            torch.as_tensor(pose_ids).cuda()).cpu().numpy()
    exp = _expected(pred, P, allow, k, mesh_ids, pose_ids)
    assert got.shape == exp.shape
    bad = np.nonzero((got != exp).any(1))[0]
    assert len(bad) == 0, f"first mismatch at rank {bad[0]}: {got[bad[0]]} vs {exp[bad[0]]}"
    # the predictions are read only, masked children included
    assert np.array_equal(d_pred.cpu().numpy().view(np.uint32), pred.view(np.uint32))


def test_rank_children_rejects_bad_sizes(ctx):
    P = 16
    d_pred = torch.zeros(P * 9, dtype=torch.float32, device="cuda")
    ids = torch.arange(P, dtype=torch.int32, device="cuda")
    with pytest.raises(perch.PerchError):
        ctx.rank_children(d_pred, P, (1,), 0, ids, ids)  # k = 0
    with pytest.raises(perch.PerchError):
        ctx.rank_children(d_pred, P, (1,), P + 1, ids, ids)  # k > n
    with pytest.raises(perch.PerchError):
        ctx.rank_children(d_pred, P, (1,) * 9, 4, ids, ids)  # more than 8 meshes
