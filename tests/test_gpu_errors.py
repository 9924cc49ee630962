"""Error paths of the C ABI on the GPU: an allocation refused under the
library's device-memory cap (PERCH_DEVICE_MEM_CAP) comes back as PERCH_E_OOM with
a message, leaves the context usable once the cap allows it, and never reaches
the kernels."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1510_05613_amd import perch  # noqa: E402
from tests import helpers as H  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    perch.load()


def test_allocation_over_the_cap_is_perch_e_oom(monkeypatch):
    sc = H.c1_scene(0)
    depth = torch.as_tensor(np.ascontiguousarray(sc.depth_obs, np.float32)).cuda()
    ctx = perch.Context(sc.sensor)
    for m, mesh in enumerate(sc.library.meshes):
        ctx.add_mesh(m, mesh.verts, mesh.tris, mesh.planes)
    ctx.set_objects(sc.obj_mesh)
    # a cap below what the observation's buffers need: refused as out of memory
    monkeypatch.setenv("PERCH_DEVICE_MEM_CAP", "1024")
    with pytest.raises(perch.PerchError, match=r"perch error -2: .*ensure"):
        ctx.set_poses(sc.poses)
    monkeypatch.delenv("PERCH_DEVICE_MEM_CAP")
    # the same context works once the cap allows it
    ctx.set_poses(sc.poses)
    ctx.set_observation(depth)
    first = sc.gt_order[0]
    cands = torch.as_tensor(np.array([[int(sc.obj_mesh[first]), int(sc.gt_pose[first])]],
                                     np.int32)).cuda()
    st, cost, _ = ctx.evaluate([], cands)
    torch.cuda.synchronize()
    assert int(st[0]) == 1 and int(cost[0]) >= 0
    # a cap reached in the middle of a search: the search reports OOM, not a crash
    monkeypatch.setenv("PERCH_DEVICE_MEM_CAP", "1")
    with pytest.raises(perch.PerchError, match=r"perch error -2"):
        ctx.search(perch.SEARCH_UCS)
    monkeypatch.delenv("PERCH_DEVICE_MEM_CAP")
    assert ctx.search(perch.SEARCH_UCS)["found"]
    ctx.close()
