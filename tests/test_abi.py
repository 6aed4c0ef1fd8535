"""C-ABI contract checks that need no GPU: the library loads, exports every
function declared in include/bake.h, and rejects bad arguments on the host
with the documented codes before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bake.h")


@pytest.fixture(scope="module")
def B():
    import paper_2605_26137_amd.bake as bake
    if not os.path.exists(bake.LIB_PATH):
        from paper_2605_26137_amd import build
        build.build()
    bake.lib()
    return bake


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(bake_[a-z_0-9]+)\s*\(", src, re.M)))


def test_every_declared_symbol_is_exported(B):
    names = declared_functions()
    assert len(names) >= 10, names
    L = C.CDLL(B.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B._EXPORTS), set(names) ^ set(B._EXPORTS)


def test_version_and_defaults(B):
    assert "gfx950" in B.version()
    o = B.make_options()
    assert o.dilate_passes == 2 and o.flags == 0 and o.trav_mode == -1


def test_workspace_size_grows_with_inputs(B):
    s1 = B.workspace_size(2562, 5120, 42, 80, 128)
    s2 = B.workspace_size(655362, 1310720, 10242, 20480, 2048)
    assert 0 < s1 < s2
    assert s1 % 256 == 0 and s2 % 256 == 0
    save = B.workspace_size(2562, 5120, 42, 80, 128, B.make_options(save=True))
    assert save >= s1 + 16 * 128 * 128


@pytest.mark.parametrize("res", [0, 3, 100, 32768, -4])
def test_bad_res_is_unsupported(B, res):
    with pytest.raises(B.BakeError) as e:
        B.workspace_size(10, 10, 10, 10, res)
    assert e.value.code == B.BAKE_E_UNSUPPORTED


def test_negative_and_inconsistent_counts(B):
    for args in [(-1, 1, 1, 1), (1, -1, 1, 1), (0, 5, 3, 1), (3, 1, 0, 4)]:
        with pytest.raises(B.BakeError) as e:
            B.workspace_size(*args, 64)
        assert e.value.code == B.BAKE_E_INVALID_ARG


def _call(B, **over):
    """bake_normals with fake (never dereferenced) device pointers."""
    fake = C.c_void_p(0x1000)
    a = dict(hi_V=fake, nhv=3, hi_F=fake, nhf=1, hi_N=fake, lo_V=fake, nlv=3, lo_F=fake, nlf=1,
             lo_UV=fake, res=16, max_dist=0.1, out_map=fake, out_hit=fake, opt=None,
             ws=C.c_void_p(0x100000), ws_bytes=1 << 40, stream=None)
    a.update(over)
    return B.lib().bake_normals(a["hi_V"], a["nhv"], a["hi_F"], a["nhf"], a["hi_N"], a["lo_V"],
                                a["nlv"], a["lo_F"], a["nlf"], a["lo_UV"], a["res"], a["max_dist"],
                                a["out_map"], a["out_hit"], a["opt"], a["ws"], a["ws_bytes"],
                                a["stream"])


@pytest.mark.parametrize("over,code", [
    (dict(hi_V=None), -1), (dict(hi_N=None), -1), (dict(hi_F=None), -1), (dict(lo_V=None), -1),
    (dict(lo_F=None), -1), (dict(lo_UV=None), -1), (dict(out_map=None), -1), (dict(out_hit=None), -1),
    (dict(max_dist=0.0), -1), (dict(max_dist=-1.0), -1), (dict(max_dist=float("inf")), -1),
    (dict(max_dist=float("nan")), -1), (dict(res=12), -2), (dict(nhv=-2), -1),
    (dict(ws=None), -3), (dict(ws=C.c_void_p(0x100010)), -3), (dict(ws_bytes=1000), -3),
])
def test_host_validation_codes(B, over, code):
    rc = _call(B, **over)
    assert rc == code, B.lib().bake_last_error()
    assert B.lib().bake_last_error()


@pytest.mark.parametrize("field,val", [("dilate_passes", -1), ("dilate_passes", 65), ("flags", 64),
                                       ("trav_block", 96), ("trav_stack", 12), ("trav_mode", 4), ("trav_mode", -2)])
def test_bad_options(B, field, val):
    o = B.make_options()
    setattr(o, field, val)
    rc = _call(B, opt=C.byref(o))
    assert rc == B.BAKE_E_INVALID_ARG


def test_backward_requires_saved_state_and_stage_times_require_timing(B):
    buf = (C.c_float * 6)()
    assert B.lib().bake_stage_times(buf, 6) == B.BAKE_E_STATE


def test_workspace_views(B):
    o, b = B.workspace_view(2562, 5120, 42, 80, 128, B.VIEW_RAYS)
    assert o % 256 == 0 and b == 16 * 128 * 128
    with pytest.raises(B.BakeError):
        B.workspace_view(2562, 5120, 42, 80, 128, B.VIEW_HITS)
    o2, _ = B.workspace_view(2562, 5120, 42, 80, 128, B.VIEW_HITS, B.make_options(save=True))
    assert o2 % 256 == 0


def test_product_does_not_reach_the_oracle():
    """The GPU package never imports the oracle (no CPU fallback path)."""
    pkg = os.path.join(ROOT, "paper_2605_26137_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dp, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "liboracle" not in txt, f


# ---- batches ---------------------------------------------------------------

def _asset(B, **over):
    """bake_asset with fake (never dereferenced) device pointers."""
    fake = 0x1000
    a = B.BakeAsset()
    a.hi_V, a.n_hi_v, a.hi_F, a.n_hi_f, a.hi_N = fake, 3, fake, 1, fake
    a.lo_V, a.n_lo_v, a.lo_F, a.n_lo_f, a.lo_UV = fake, 3, fake, 1, fake
    a.res, a.max_dist = 16, 0.1
    a.out_map, a.out_hit = fake, fake
    for k, v in over.items():
        setattr(a, k, v)
    return a


def _arr(B, assets):
    arr = (B.BakeAsset * len(assets))()
    for i, a in enumerate(assets):
        arr[i] = a
    return arr


def test_batch_of_one_has_the_single_layout(B):
    for sizes, save in [((2562, 5120, 42, 80, 128), False), ((655362, 1310720, 10242, 20480, 2048), True)]:
        a = _asset(B, n_hi_v=sizes[0], n_hi_f=sizes[1], n_lo_v=sizes[2], n_lo_f=sizes[3], res=sizes[4])
        o = B.make_options(save=save)
        b = C.c_size_t(0)
        assert B.lib().bake_batch_workspace_size(_arr(B, [a]), 1, C.byref(o), C.byref(b)) == 0
        assert b.value == B.workspace_size(*sizes, o)


def test_batch_workspace_grows_with_assets(B):
    one = C.c_size_t(0)
    two = C.c_size_t(0)
    a = _asset(B, n_hi_v=2562, n_hi_f=5120, n_lo_v=42, n_lo_f=80, res=128)
    assert B.lib().bake_batch_workspace_size(_arr(B, [a]), 1, None, C.byref(one)) == 0
    assert B.lib().bake_batch_workspace_size(_arr(B, [a, a]), 2, None, C.byref(two)) == 0
    assert one.value < two.value < 2 * one.value + (1 << 20)


@pytest.mark.parametrize("n", [0, -1, 65537])
def test_batch_bad_count(B, n):
    b = C.c_size_t(0)
    arr = _arr(B, [_asset(B)])
    assert B.lib().bake_batch_workspace_size(arr, n, None, C.byref(b)) == B.BAKE_E_INVALID_ARG
    assert B.lib().bake_batch_workspace_size(None, 1, None, C.byref(b)) == B.BAKE_E_INVALID_ARG


@pytest.mark.parametrize("over,code", [
    (dict(res=12), -2), (dict(n_hi_f=-1), -1), (dict(max_dist=0.0), -1), (dict(out_map=None), -1),
    (dict(out_hit=None), -1), (dict(hi_V=None), -1), (dict(lo_UV=None), -1),
])
def test_batch_validation_codes(B, over, code):
    arr = _arr(B, [_asset(B), _asset(B, **over)])
    rc = B.lib().bake_normals_batched(arr, 2, None, C.c_void_p(0x100000), 1 << 40, None)
    assert rc == code, B.lib().bake_last_error()
    assert "asset 1" in B.lib().bake_last_error().decode() or code == -2 or "n_hi_f" in str(over)


def test_batch_rejects_shared_rgb8_and_small_workspace(B):
    arr = _arr(B, [_asset(B), _asset(B)])
    o = B.make_options(rgb8_ptr=0x2000)
    assert B.lib().bake_normals_batched(arr, 2, C.byref(o), C.c_void_p(0x100000), 1 << 40, None) == -1
    assert B.lib().bake_normals_batched(arr, 2, None, C.c_void_p(0x100000), 4096, None) == B.BAKE_E_WORKSPACE
    assert B.lib().bake_normals_batched(arr, 2, None, C.c_void_p(0x100010), 1 << 40, None) == B.BAKE_E_WORKSPACE


def test_batch_backward_without_saved_forward(B):
    arr = _arr(B, [_asset(B, grad_map=0x3000, grad_lo_V=0x4000)])
    rc = B.lib().bake_normals_batched_backward(arr, 1, C.c_void_p(0x7000000), 1 << 40, None)
    assert rc == B.BAKE_E_STATE
    arr = _arr(B, [_asset(B, grad_lo_V=0x4000)])  # gradient wanted without grad_map
    rc = B.lib().bake_normals_batched_backward(arr, 1, C.c_void_p(0x7000000), 1 << 40, None)
    assert rc == B.BAKE_E_INVALID_ARG


def test_autotune_argument_checks(B):
    arr = _arr(B, [_asset(B)])
    best = B.BakeOptions()
    assert B.lib().bake_autotune(arr, 1, None, 0, C.c_void_p(0x100000), 1 << 40, None, C.byref(best),
                                 None) == B.BAKE_E_INVALID_ARG
    assert B.lib().bake_autotune(arr, 1, None, 3, C.c_void_p(0x100000), 1 << 40, None, None,
                                 None) == B.BAKE_E_INVALID_ARG


def _vis_call(B, **over):
    """bake_visibility with fake (never dereferenced) device pointers."""
    fake = C.c_void_p(0x1000)
    a = dict(V=fake, F=fake, nv=3, nf=1, eyes=fake, nviews=4, target=(C.c_float * 3)(0, 0, 0),
             tan_half=0.5, res=16, t_far=5.0, flags=0, vis=fake, ext=fake, fh=None,
             ws=C.c_void_p(0x100000), ws_bytes=1 << 40, stream=None)
    a.update(over)
    return B.lib().bake_visibility(a["V"], a["F"], a["nv"], a["nf"], a["eyes"], a["nviews"], a["target"],
                                   a["tan_half"], a["res"], a["t_far"], a["flags"], a["vis"], a["ext"],
                                   a["fh"], a["ws"], a["ws_bytes"], a["stream"])


@pytest.mark.parametrize("over,code", [
    (dict(V=None), -1), (dict(F=None), -1), (dict(vis=None), -1), (dict(eyes=None), -1),
    (dict(target=None), -1), (dict(nviews=0), -1), (dict(res=0), -1), (dict(res=16385), -1),
    (dict(tan_half=0.0), -1), (dict(tan_half=float("inf")), -1), (dict(t_far=float("nan")), -1),
    (dict(t_far=-1.0), -1), (dict(flags=1), -1), (dict(nv=-1), -1), (dict(nf=1 << 30), -2),
    (dict(ws=None), -3), (dict(ws=C.c_void_p(0x100010)), -3), (dict(ws_bytes=1000), -3),
    (dict(target=(C.c_float * 3)(0, float("inf"), 0)), -1),
])
def test_visibility_host_validation_codes(B, over, code):
    rc = _vis_call(B, **over)
    assert rc == code, B.lib().bake_last_error()
    assert B.lib().bake_last_error()


def test_visibility_workspace_size(B):
    a = B.visibility_workspace_size(1000, 2000)
    b = B.visibility_workspace_size(2000, 4000)
    assert 0 < a < b and a % 256 == 0
    with pytest.raises(B.BakeError):
        B.visibility_workspace_size(-1, 5)


def _map_call(B, **over):
    """bake_view_maps with fake (never dereferenced) device pointers."""
    fake = C.c_void_p(0x1000)
    a = dict(V=fake, F=fake, UV=fake, nv=3, nf=1, res=16, eyes=fake, nviews=4, target=(C.c_float * 3)(0, 0, 0),
             tan_half=0.5, img=64, t_far=5.0, tol=1e-3, flags=0, uv=fake, inc=fake, dep=None,
             ws=C.c_void_p(0x100000), ws_bytes=1 << 40, stream=None)
    a.update(over)
    return B.lib().bake_view_maps(a["V"], a["F"], a["UV"], a["nv"], a["nf"], a["res"], a["eyes"], a["nviews"],
                                  a["target"], a["tan_half"], a["img"], a["t_far"], a["tol"], a["flags"], a["uv"],
                                  a["inc"], a["dep"], a["ws"], a["ws_bytes"], a["stream"])


@pytest.mark.parametrize("over,code", [
    (dict(V=None), -1), (dict(F=None), -1), (dict(UV=None), -1), (dict(eyes=None), -1), (dict(target=None), -1),
    (dict(uv=None), -1), (dict(inc=None), -1), (dict(nviews=0), -1), (dict(img=0), -1), (dict(res=12), -2),
    (dict(tan_half=-1.0), -1), (dict(t_far=float("inf")), -1), (dict(tol=-1e-3), -1), (dict(tol=float("nan")), -1),
    (dict(flags=1), -1), (dict(ws=None), -3), (dict(ws_bytes=1000), -3),
])
def test_view_maps_host_validation_codes(B, over, code):
    rc = _map_call(B, **over)
    assert rc == code, B.lib().bake_last_error()


def test_view_maps_workspace_size(B):
    a = B.view_maps_workspace_size(1000, 2000, 256, 10, 256)
    b = B.view_maps_workspace_size(1000, 2000, 256, 10, 512)
    assert 0 < a < b and a % 256 == 0


def _qem_call(B, **over):
    """bake_qem_simplify with fake (never dereferenced) device pointers."""
    fake = C.c_void_p(0x1000)
    a = dict(V=fake, F=fake, nv=4, nf=4, target=4, rho=0.25, rounds=10, flags=0, Vo=fake, Fo=fake,
             counts=(C.c_int64 * 2)(), nr=C.pointer(C.c_int32(0)), stats=None, tms=None,
             ws=C.c_void_p(0x100000), ws_bytes=1 << 40, stream=None)
    a.update(over)
    return B.lib().bake_qem_simplify(a["V"], a["F"], a["nv"], a["nf"], a["target"], a["rho"], a["rounds"],
                                     a["flags"], a["Vo"], a["Fo"], a["counts"], a["nr"], a["stats"], a["tms"],
                                     a["ws"], a["ws_bytes"], a["stream"])


@pytest.mark.parametrize("over,code", [
    (dict(V=None), -1), (dict(F=None), -1), (dict(Vo=None), -1), (dict(Fo=None), -1), (dict(counts=None), -1),
    (dict(nr=None), -1), (dict(target=3), -1), (dict(rho=0.0), -1), (dict(rho=1.5), -1),
    (dict(rho=float("nan")), -1), (dict(rounds=-1), -1), (dict(flags=2), -1), (dict(nv=-1), -1),
    (dict(nf=1 << 28), -2), (dict(ws=None), -3), (dict(ws=C.c_void_p(0x100010)), -3), (dict(ws_bytes=1000), -3),
])
def test_qem_host_validation_codes(B, over, code):
    rc = _qem_call(B, **over)
    assert rc == code, B.lib().bake_last_error()
    assert B.lib().bake_last_error()


def test_qem_edges_host_validation_codes(B):
    fake = C.c_void_p(0x1000)
    n = C.c_int64(0)
    L = B.lib()
    names = ["V", "F", "nv", "nf", "flags", "cap", "E", "ok", "fc", "cost", "p", "Q", "n", "ws", "ws_bytes", "s"]
    base = [fake, fake, 4, 4, 0, 12, fake, fake, fake, fake, fake, None, C.byref(n), C.c_void_p(0x100000), 1 << 40,
            None]
    for name, v, code in (("n", None, -1), ("cap", -1, -1), ("E", None, -1), ("nf", 1 << 28, -2),
                          ("flags", 2, -1), ("ws", None, -3), ("ws_bytes", 100, -3)):
        args = list(base)
        args[names.index(name)] = v
        assert L.bake_qem_edges(*args) == code, (name, v, L.bake_last_error())


def test_qem_workspace_size(B):
    a = B.qem_workspace_size(1000, 2000)
    b = B.qem_workspace_size(2000, 4000)
    assert 0 < a < b and a % 256 == 0
    with pytest.raises(B.BakeError):
        B.qem_workspace_size(-1, 5)
    with pytest.raises(B.BakeError):
        B.qem_workspace_size(10, 1 << 28)


def _noalloc(B, nhv, nhf, nlv, nlf, res, opt=None):
    fake = C.c_void_p(0x1000)
    return B.lib().bake_normals_noalloc(fake, nhv, fake, nhf, fake, fake, nlv, fake, nlf, fake, res,
                                        C.c_float(0.1), fake, fake, opt, None)


def test_noalloc_host_checks(B):
    """bake_normals_noalloc refuses, before touching the device, a bake larger
    than its scratch array and the flags whose state it could not hand back."""
    assert B.NOALLOC_BYTES == 128 << 20
    assert _noalloc(B, 655362, 1310720, 10242, 20480, 2048) == B.BAKE_E_WORKSPACE
    assert b"BAKE_NOALLOC_BYTES" in B.lib().bake_last_error()
    for kw in (dict(save=True), dict(timing=True), dict(count=True)):
        o = B.make_options(**kw)
        assert _noalloc(B, 2562, 5120, 42, 80, 128, C.byref(o)) == B.BAKE_E_INVALID_ARG
    assert _noalloc(B, 2562, 5120, 42, 80, 100) == B.BAKE_E_UNSUPPORTED
