"""bake_normals_noalloc through the C ABI: the forward bake with no device
allocation (the library's fixed per-GPU scratch array instead of a caller
workspace) gives bitwise the maps and hit ids of bake_normals with a
workspace, on consecutive calls of different sizes that share the array."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from synth import Asset, make_config  # noqa: E402
from synth import meshes as M  # noqa: E402


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_26137_amd.bake as bake
    bake.lib()
    return bake


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _near_limit_asset():
    # 327,680 high-poly faces onto 5,120 at 512^2: a workspace of ~126 MiB,
    # just under the array's 128 MiB
    lV, lF = M.icosphere(4)
    hV, hF = M.icosphere(7)
    U = M.unit_directions(hV)
    hiV = M.displace(U, M.noise_radius(U, 3, 4, 0.03))
    hiF = hF.astype(np.int32)
    return Asset("noise_L7_L4_512", hiV, hiF, M.vertex_normals(hiV, hiF), lV.astype(np.float32),
                 lF.astype(np.int32), M.face_grid_atlas(lF.shape[0], 512), res=512, max_dist=0.12)


def _same(B, a, dilate):
    t = B.to_device(a)
    ref = B.bake_normals(*t, a.res, a.max_dist, dilate_passes=dilate)
    m = torch.full((a.res, a.res, 3), float("nan"), device="cuda")
    h = torch.full((a.res, a.res), -7, dtype=torch.int32, device="cuda")
    B.bake_normals_noalloc(*t, a.res, a.max_dist, m, h, dilate_passes=dilate)
    torch.cuda.synchronize()
    assert ref.status() == 0
    ok_map = torch.equal(m.view(torch.int32), ref.map.view(torch.int32))
    ok_hit = torch.equal(h, ref.hit)
    covered = int((ref.hit != B.BAKE_UNCOVERED).sum())
    say(f"[gpu] {a.name}: no-alloc bake equal to the workspace bake: map {ok_map}, hit {ok_hit}"
        f" ({covered} covered texels)")
    assert covered > 0
    assert ok_map and ok_hit


def test_noalloc_equals_workspace_bake_on_two_calls(B):
    big = _near_limit_asset()
    small = make_config(1)  # 5,120 faces onto 80 at 128^2
    assert B.workspace_size(*(x.shape[0] for x in (big.hi_V, big.hi_F, big.lo_V, big.lo_F)), big.res) \
        <= B.NOALLOC_BYTES
    _same(B, big, 2)
    _same(B, small, 2)   # second call, smaller input, on the same array
    _same(B, big, 0)     # and back: nothing of the earlier calls leaks into a later one


def test_noalloc_rejects_a_bake_beyond_the_array(B):
    a = make_config(1)
    t = B.to_device(a)
    m = torch.empty((4096, 4096, 3), device="cuda")
    h = torch.empty((4096, 4096), dtype=torch.int32, device="cuda")
    with pytest.raises(B.BakeError) as e:
        B.bake_normals_noalloc(*t, 4096, a.max_dist, m, h)
    assert e.value.code == B.BAKE_E_WORKSPACE
