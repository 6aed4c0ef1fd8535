"""Python binding of the gfx950 normal baker (libbake.so, C ABI in include/bake.h).

Argument marshalling only: every step of the bake runs in the HIP kernels of
libbake.so.  PyTorch provides device memory and the stream.  If the library
is missing, importing works but every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbake.so")

BAKE_OK = 0
BAKE_E_INVALID_ARG = -1
BAKE_E_UNSUPPORTED = -2
BAKE_E_WORKSPACE = -3
BAKE_E_INDEX = -4
BAKE_E_HIP = -5
BAKE_E_STATE = -6

BAKE_MISS = -1
BAKE_UNRELIABLE = -2
BAKE_UNCOVERED = -3

BAKE_STATUS_LO_INDEX = 1
BAKE_STATUS_HI_INDEX = 2
BAKE_STATUS_BAD_UV = 4
BAKE_STATUS_NONFINITE = 8
BAKE_STATUS_INTERNAL = 16
BAKE_STATUS_STATE = 32

BAKE_QUERY_RAY = 0
BAKE_QUERY_CLOSEST = 1
QUERIES = {"ray": BAKE_QUERY_RAY, "closest": BAKE_QUERY_CLOSEST}

BAKE_FLAG_SAVE = 1
BAKE_FLAG_TIMING = 2
BAKE_FLAG_COUNT = 4
BAKE_FLAG_ONE_STREAM = 8
BAKE_FLAG_ONE_QUEUE = 16

(VIEW_RAYS, VIEW_HITS, VIEW_FACEMAP, VIEW_LO_N, VIEW_SORTED, VIEW_NODES, VIEW_LEAVES, VIEW_FACE_T,
 VIEW_SORTED_IDX) = range(9)

STAGES = ("lo_prep", "raster", "bvh_build", "traverse", "dilate", "forward")


class BakeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bake error {code}: {msg}")
        self.code = code


class BakeOptions(C.Structure):
    _fields_ = [
        ("dilate_passes", C.c_int32),
        ("flags", C.c_uint32),
        ("out_rgb8", C.c_void_p),
        ("trav_block", C.c_int32),
        ("trav_stack", C.c_int32),
        ("trav_mode", C.c_int32),
        ("query", C.c_int32),
        ("reserved", C.c_int32 * 3),
    ]


class BakeAsset(C.Structure):
    """One asset of a batch (struct bake_asset)."""
    _fields_ = [
        ("hi_V", C.c_void_p), ("n_hi_v", C.c_int64),
        ("hi_F", C.c_void_p), ("n_hi_f", C.c_int64),
        ("hi_N", C.c_void_p),
        ("lo_V", C.c_void_p), ("n_lo_v", C.c_int64),
        ("lo_F", C.c_void_p), ("n_lo_f", C.c_int64),
        ("lo_UV", C.c_void_p),
        ("res", C.c_int32), ("max_dist", C.c_float),
        ("out_map", C.c_void_p), ("out_hit", C.c_void_p), ("out_rgb8", C.c_void_p),
        ("grad_map", C.c_void_p), ("grad_lo_V", C.c_void_p), ("grad_hi_N", C.c_void_p),
    ]


_lib = None

_EXPORTS = {
    "bake_default_options": (None, [C.c_void_p]),
    "bake_workspace_size": (C.c_int32, [C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_int32,
                                        C.c_void_p, C.POINTER(C.c_size_t)]),
    "bake_normals": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                 C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                 C.c_int32, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_size_t, C.c_void_p]),
    "bake_normals_noalloc": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                         C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                         C.c_int32, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p]),
    "bake_normals_backward": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                          C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                          C.c_int32, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_size_t, C.c_void_p]),
    "bake_sq_loss": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_size_t, C.c_void_p]),
    "bake_query_status": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_uint32)]),
    "bake_read_counter": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_int64)]),
    "bake_workspace_view": (C.c_int32, [C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_int32,
                                        C.c_void_p, C.c_int32, C.POINTER(C.c_size_t),
                                        C.POINTER(C.c_size_t)]),
    "bake_batch_workspace_size": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_size_t)]),
    "bake_normals_batched": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t,
                                         C.c_void_p]),
    "bake_normals_batched_backward": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t,
                                                  C.c_void_p]),
    "bake_read_asset_counter": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                            C.POINTER(C.c_int64)]),
    "bake_autotune": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t,
                                  C.c_void_p, C.c_void_p, C.POINTER(C.c_float)]),
    "bake_visibility_workspace_size": (C.c_int32, [C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
    "bake_visibility": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_int32,
                                    C.POINTER(C.c_float), C.c_float, C.c_int32, C.c_float, C.c_uint32,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "bake_view_maps_workspace_size": (C.c_int32, [C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                                  C.POINTER(C.c_size_t)]),
    "bake_view_maps": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int32,
                                   C.c_void_p, C.c_int32, C.POINTER(C.c_float), C.c_float, C.c_int32, C.c_float,
                                   C.c_float, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_size_t, C.c_void_p]),
    "bake_qem_workspace_size": (C.c_int32, [C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
    "bake_qem_simplify": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_double,
                                      C.c_int32, C.c_uint32, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int32), C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                      C.c_void_p]),
    "bake_qem_edges": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_uint32, C.c_int64,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.POINTER(C.c_int64), C.c_void_p, C.c_size_t, C.c_void_p]),
    "bake_stage_times": (C.c_int32, [C.POINTER(C.c_float), C.c_int32]),
    "bake_stage_history": (C.c_int32, [C.POINTER(C.c_float), C.c_int32]),
    "bake_last_error": (C.c_char_p, []),
    "bake_version": (C.c_char_p, []),
}


def lib():
    """Load libbake.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2605_26137_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc < 0:
        raise BakeError(rc, lib().bake_last_error().decode())
    return rc


def make_options(dilate_passes=2, save=False, timing=False, rgb8_ptr=0, trav_block=0,
                 trav_stack=0, trav_mode=-1, count=False, query="ray", one_stream=False,
                 one_queue=False) -> BakeOptions:
    o = BakeOptions()
    lib().bake_default_options(C.byref(o))
    o.dilate_passes = int(dilate_passes)
    o.flags = ((BAKE_FLAG_SAVE if save else 0) | (BAKE_FLAG_TIMING if timing else 0)
               | (BAKE_FLAG_COUNT if count else 0) | (BAKE_FLAG_ONE_STREAM if one_stream else 0)
               | (BAKE_FLAG_ONE_QUEUE if one_queue else 0))
    o.out_rgb8 = rgb8_ptr or None
    o.trav_block = int(trav_block)
    o.trav_stack = int(trav_stack)
    o.trav_mode = int(trav_mode)
    o.query = QUERIES[query]
    return o


def workspace_size(n_hi_v, n_hi_f, n_lo_v, n_lo_f, res, opts: Optional[BakeOptions] = None) -> int:
    b = C.c_size_t(0)
    _check(lib().bake_workspace_size(int(n_hi_v), int(n_hi_f), int(n_lo_v), int(n_lo_f), int(res),
                                     C.byref(opts) if opts is not None else None, C.byref(b)))
    return b.value


def workspace_view(n_hi_v, n_hi_f, n_lo_v, n_lo_f, res, which, opts=None):
    o = C.c_size_t(0)
    b = C.c_size_t(0)
    _check(lib().bake_workspace_view(int(n_hi_v), int(n_hi_f), int(n_lo_v), int(n_lo_f), int(res),
                                     C.byref(opts) if opts is not None else None, int(which),
                                     C.byref(o), C.byref(b)))
    return o.value, b.value


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_handle(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev_tensor(x, dtype, name, shape_tail=None):
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if x.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU (got {x.device})")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {x.dtype})")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(x.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} has shape {tuple(x.shape)}, expected [n, {shape_tail}]")
    return x


@dataclass
class BakeResult:
    map: torch.Tensor          # [res, res, 3] f32
    hit: torch.Tensor          # [res, res] i32
    rgb8: Optional[torch.Tensor]
    workspace: torch.Tensor
    opts: BakeOptions
    sizes: tuple               # (n_hi_v, n_hi_f, n_lo_v, n_lo_f, res)

    def view(self, which, dtype=torch.uint8):
        o, b = workspace_view(*self.sizes, which, self.opts)
        return self.workspace[o:o + b].view(dtype)

    def counter(self, which: int, stream=None) -> int:
        v = C.c_int64(0)
        _check(lib().bake_read_counter(_ptr(self.workspace), int(which), _stream_handle(stream),
                                       C.byref(v)))
        return v.value

    def ray_count(self, stream=None) -> int:
        return self.counter(0, stream)

    def test_counts(self, stream=None):
        """(box tests, triangle tests) of a bake made with count=True."""
        return self.counter(1, stream), self.counter(2, stream)

    def wave_trips(self, stream=None) -> int:
        """Traversal loop trips of whole 64-lane waves (a bake made with
        count=True): (box / 2 + tri) / (64 trips) is the useful-lane fraction."""
        return self.counter(3, stream)

    def status(self, stream=None) -> int:
        v = C.c_uint32(0)
        _check(lib().bake_query_status(_ptr(self.workspace), _stream_handle(stream), C.byref(v)))
        return v.value


def bake_normals(hi_V, hi_F, hi_N, lo_V, lo_F, lo_UV, res: int, max_dist: float, *,
                 dilate_passes: int = 2, rgb8: bool = False, save: bool = False,
                 timing: bool = False, trav_block: int = 0, trav_stack: int = 0,
                 trav_mode: int = -1, count: bool = False, query: str = "ray",
                 one_stream: bool = False, one_queue: bool = False,
                 workspace: Optional[torch.Tensor] = None,
                 out_map: Optional[torch.Tensor] = None, out_hit: Optional[torch.Tensor] = None,
                 stream=None) -> BakeResult:
    """Bake a tangent-space normal map of the high-poly onto the low-poly's UV
    atlas.  Inputs are GPU tensors: hi_V [Vh,3] f32, hi_F [Fh,3] i32, hi_N [Vh,3]
    f32, lo_V [Vl,3] f32, lo_F [Fl,3] i32, lo_UV [Fl,3,2] f32.  query: "ray"
    (two-sided ray along the interpolated normal) or "closest" (closest point
    of the high-poly within max_dist, forward only).  one_stream: run every
    stage on the caller's stream (no second stream beside the BVH build; the
    backward of a saved bake follows), with the same results bit for bit."""
    hi_V = _dev_tensor(hi_V, torch.float32, "hi_V", (3,))
    hi_F = _dev_tensor(hi_F, torch.int32, "hi_F", (3,))
    hi_N = _dev_tensor(hi_N, torch.float32, "hi_N", (3,))
    lo_V = _dev_tensor(lo_V, torch.float32, "lo_V", (3,))
    lo_F = _dev_tensor(lo_F, torch.int32, "lo_F", (3,))
    lo_UV = _dev_tensor(lo_UV, torch.float32, "lo_UV", (3, 2))
    if hi_N.shape[0] != hi_V.shape[0]:
        raise ValueError("hi_N and hi_V must have the same number of rows")
    if lo_UV.shape[0] != lo_F.shape[0]:
        raise ValueError("lo_UV and lo_F must have the same number of rows")
    dev = hi_V.device
    sizes = (hi_V.shape[0], hi_F.shape[0], lo_V.shape[0], lo_F.shape[0], int(res))
    rgb = torch.empty((res, res, 3), dtype=torch.uint8, device=dev) if rgb8 else None
    opts = make_options(dilate_passes, save, timing, rgb.data_ptr() if rgb is not None else 0,
                        trav_block, trav_stack, trav_mode, count, query, one_stream, one_queue)
    nbytes = workspace_size(*sizes, opts)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    if out_map is None:
        out_map = torch.empty((res, res, 3), dtype=torch.float32, device=dev)
    if out_hit is None:
        out_hit = torch.empty((res, res), dtype=torch.int32, device=dev)
    _check(lib().bake_normals(
        _ptr(hi_V), sizes[0], _ptr(hi_F), sizes[1], _ptr(hi_N), _ptr(lo_V), sizes[2], _ptr(lo_F),
        sizes[3], _ptr(lo_UV), int(res), float(max_dist), _ptr(out_map), _ptr(out_hit),
        C.byref(opts), _ptr(workspace), workspace.numel(), _stream_handle(stream)))
    r = BakeResult(out_map, out_hit, rgb, workspace, opts, sizes)
    r.max_dist = float(max_dist)
    return r


NOALLOC_BYTES = 128 << 20  # BAKE_NOALLOC_BYTES


def bake_normals_noalloc(hi_V, hi_F, hi_N, lo_V, lo_F, lo_UV, res: int, max_dist: float,
                         out_map: torch.Tensor, out_hit: torch.Tensor, *, dilate_passes: int = 2,
                         out_rgb8: Optional[torch.Tensor] = None, trav_block: int = 0, trav_stack: int = 0,
                         trav_mode: int = -1, query: str = "ray", stream=None) -> None:
    """bake_normals into caller-allocated out_map [res,res,3] f32 and out_hit
    [res,res] i32 (and optionally out_rgb8 [res,res,3] u8) with no device
    allocation at all: the library's fixed per-GPU scratch array stands in
    for the workspace (include/bake.h, bake_normals_noalloc: its size limit,
    and calls that overlap on one GPU race)."""
    hi_V = _dev_tensor(hi_V, torch.float32, "hi_V", (3,))
    hi_F = _dev_tensor(hi_F, torch.int32, "hi_F", (3,))
    hi_N = _dev_tensor(hi_N, torch.float32, "hi_N", (3,))
    lo_V = _dev_tensor(lo_V, torch.float32, "lo_V", (3,))
    lo_F = _dev_tensor(lo_F, torch.int32, "lo_F", (3,))
    lo_UV = _dev_tensor(lo_UV, torch.float32, "lo_UV", (3, 2))
    out_map = _dev_tensor(out_map, torch.float32, "out_map")
    out_hit = _dev_tensor(out_hit, torch.int32, "out_hit")
    if tuple(out_map.shape) != (res, res, 3) or tuple(out_hit.shape) != (res, res):
        raise ValueError(f"out_map must be [{res},{res},3] and out_hit [{res},{res}]")
    if out_rgb8 is not None:
        out_rgb8 = _dev_tensor(out_rgb8, torch.uint8, "out_rgb8")
        if tuple(out_rgb8.shape) != (res, res, 3):
            raise ValueError(f"out_rgb8 must be [{res},{res},3]")
    if hi_N.shape[0] != hi_V.shape[0] or lo_UV.shape[0] != lo_F.shape[0]:
        raise ValueError("hi_N / hi_V or lo_UV / lo_F row counts differ")
    opts = make_options(dilate_passes, False, False, out_rgb8.data_ptr() if out_rgb8 is not None else 0,
                        trav_block, trav_stack, trav_mode, False, query, True)
    _check(lib().bake_normals_noalloc(
        _ptr(hi_V), hi_V.shape[0], _ptr(hi_F), hi_F.shape[0], _ptr(hi_N), _ptr(lo_V), lo_V.shape[0],
        _ptr(lo_F), lo_F.shape[0], _ptr(lo_UV), int(res), float(max_dist), _ptr(out_map), _ptr(out_hit),
        C.byref(opts), _stream_handle(stream)))


def bake_normals_backward(result: BakeResult, inputs, grad_map, need_lo=True, need_hi=True,
                          stream=None, out_lo=None, out_hi=None):
    """Gradients of a loss on the pre-dilation map w.r.t. lo_V and hi_N, for a
    forward `result` made with save=True on the same `inputs` (the six tensors
    given to bake_normals, same order).  Returns (grad_lo_V, grad_hi_N); an
    entry is None when not requested.  out_lo / out_hi: optional preallocated
    outputs."""
    hi_V, hi_F, hi_N, lo_V, lo_F, lo_UV = inputs
    res = result.sizes[4]
    g = _dev_tensor(grad_map.contiguous(), torch.float32, "grad_map")
    if tuple(g.shape) != (res, res, 3):
        raise ValueError(f"grad_map must be [{res},{res},3]")
    glo = (out_lo if out_lo is not None else torch.empty_like(lo_V)) if need_lo else None
    ghi = (out_hi if out_hi is not None else torch.empty_like(hi_N)) if need_hi else None
    for t, ref, name in ((glo, lo_V, "out_lo"), (ghi, hi_N, "out_hi")):
        if t is not None:
            _dev_tensor(t, torch.float32, name)
            if t.shape != ref.shape:
                raise ValueError(f"{name} must have shape {tuple(ref.shape)}")
    _check(lib().bake_normals_backward(
        _ptr(hi_V), hi_V.shape[0], _ptr(hi_F), hi_F.shape[0], _ptr(hi_N), _ptr(lo_V), lo_V.shape[0],
        _ptr(lo_F), lo_F.shape[0], _ptr(lo_UV), int(res), float(result.max_dist), _ptr(g), _ptr(glo),
        _ptr(ghi), _ptr(result.workspace), result.workspace.numel(), _stream_handle(stream)))
    return glo, ghi


def sq_loss(map_, target, want_grad=True, stream=None, out_loss=None, out_grad=None, scratch=None):
    """(sum (map - target)^2 as a 1-element tensor, 2 (map - target) or None).
    out_loss / out_grad / scratch: optional preallocated buffers."""
    m = _dev_tensor(map_.contiguous(), torch.float32, "map")
    t = _dev_tensor(target.contiguous(), torch.float32, "target")
    if m.shape != t.shape:
        raise ValueError("map and target shapes differ")
    n = m.numel()
    loss = out_loss if out_loss is not None else torch.empty(1, dtype=torch.float32, device=m.device)
    grad = (out_grad if out_grad is not None else torch.empty_like(m)) if want_grad else None
    need = 4 * ((n + 255) // 256 + 1)
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(need, dtype=torch.uint8, device=m.device)
    _check(lib().bake_sq_loss(_ptr(m), _ptr(t), n, _ptr(grad), _ptr(loss), _ptr(scratch),
                              scratch.numel(), _stream_handle(stream)))
    return loss, grad


class BakeNormals(torch.autograd.Function):
    """Differentiable bake: map = BakeNormals.apply(lo_V, hi_N, hi_V, hi_F, lo_F,
    lo_UV, res, max_dist[, dilate_passes]).  Gradients flow to lo_V and hi_N
    with the hit selection held fixed; the hit-id map is returned as a second,
    non-differentiable output.  dilate_passes defaults to 0 so that every
    differentiable texel is a traced one."""

    @staticmethod
    def forward(ctx, lo_V, hi_N, hi_V, hi_F, lo_F, lo_UV, res, max_dist, dilate_passes=0):
        r = bake_normals(hi_V, hi_F, hi_N, lo_V, lo_F, lo_UV, res, max_dist,
                         dilate_passes=dilate_passes, save=True)
        r.max_dist = float(max_dist)
        ctx.result = r
        ctx.inputs = (hi_V, hi_F, hi_N, lo_V, lo_F, lo_UV)
        ctx.mark_non_differentiable(r.hit)
        return r.map, r.hit

    @staticmethod
    def backward(ctx, grad_map, grad_hit):
        glo, ghi = bake_normals_backward(ctx.result, ctx.inputs, grad_map,
                                         need_lo=ctx.needs_input_grad[0],
                                         need_hi=ctx.needs_input_grad[1])
        return glo, ghi, None, None, None, None, None, None, None


class BakeBatch:
    """Many assets baked by one launch sequence (bake_normals_batched).

    `assets` is a list of (hi_V, hi_F, hi_N, lo_V, lo_F, lo_UV, res, max_dist)
    with GPU tensors as for bake_normals.  The batch owns its outputs (maps[i],
    hits[i], rgb8[i]), its gradient buffers (grad_maps[i] in, grad_lo_V[i] /
    grad_hi_N[i] out) and its workspace, at fixed addresses, so forward() and
    backward() can be recorded into a CUDA/HIP graph (capture()) and replayed.
    Every asset's results are bitwise those of a single bake_normals call."""

    def __init__(self, assets, *, save=False, dilate_passes=2, rgb8=False, trav_block=0,
                 trav_stack=0, trav_mode=-1, need_lo=True, need_hi=True, query="ray", one_queue=False):
        if not assets:
            raise ValueError("empty batch")
        self.inputs = []
        self.maps, self.hits, self.rgb8 = [], [], []
        self.grad_maps, self.grad_lo_V, self.grad_hi_N = [], [], []
        self.n = len(assets)
        self.save = bool(save)
        self._arr = (BakeAsset * self.n)()
        for i, a in enumerate(assets):
            hi_V, hi_F, hi_N, lo_V, lo_F, lo_UV, res, max_dist = a
            hi_V = _dev_tensor(hi_V, torch.float32, "hi_V", (3,))
            hi_F = _dev_tensor(hi_F, torch.int32, "hi_F", (3,))
            hi_N = _dev_tensor(hi_N, torch.float32, "hi_N", (3,))
            lo_V = _dev_tensor(lo_V, torch.float32, "lo_V", (3,))
            lo_F = _dev_tensor(lo_F, torch.int32, "lo_F", (3,))
            lo_UV = _dev_tensor(lo_UV, torch.float32, "lo_UV", (3, 2))
            if hi_N.shape[0] != hi_V.shape[0] or lo_UV.shape[0] != lo_F.shape[0]:
                raise ValueError(f"asset {i}: inconsistent row counts")
            dev = hi_V.device
            res = int(res)
            self.inputs.append((hi_V, hi_F, hi_N, lo_V, lo_F, lo_UV, res, float(max_dist)))
            m = torch.empty((res, res, 3), dtype=torch.float32, device=dev)
            h = torch.empty((res, res), dtype=torch.int32, device=dev)
            r8 = torch.empty((res, res, 3), dtype=torch.uint8, device=dev) if rgb8 else None
            gm = torch.zeros((res, res, 3), dtype=torch.float32, device=dev) if save else None
            glo = torch.empty_like(lo_V) if (save and need_lo) else None
            ghi = torch.empty_like(hi_N) if (save and need_hi) else None
            self.maps.append(m)
            self.hits.append(h)
            self.rgb8.append(r8)
            self.grad_maps.append(gm)
            self.grad_lo_V.append(glo)
            self.grad_hi_N.append(ghi)
            e = self._arr[i]
            e.hi_V, e.n_hi_v = hi_V.data_ptr(), hi_V.shape[0]
            e.hi_F, e.n_hi_f = hi_F.data_ptr(), hi_F.shape[0]
            e.hi_N = hi_N.data_ptr()
            e.lo_V, e.n_lo_v = lo_V.data_ptr(), lo_V.shape[0]
            e.lo_F, e.n_lo_f = lo_F.data_ptr(), lo_F.shape[0]
            e.lo_UV = lo_UV.data_ptr()
            e.res, e.max_dist = res, float(max_dist)
            e.out_map, e.out_hit = m.data_ptr(), h.data_ptr()
            e.out_rgb8 = r8.data_ptr() if r8 is not None else None
            e.grad_map = gm.data_ptr() if gm is not None else None
            e.grad_lo_V = glo.data_ptr() if glo is not None else None
            e.grad_hi_N = ghi.data_ptr() if ghi is not None else None
        self.device = self.inputs[0][0].device
        self.opts = make_options(dilate_passes, save, False, 0, trav_block, trav_stack, trav_mode,
                                 query=query, one_queue=one_queue)
        b = C.c_size_t(0)
        _check(lib().bake_batch_workspace_size(self._arr, self.n, C.byref(self.opts), C.byref(b)))
        self.workspace = torch.empty(b.value, dtype=torch.uint8, device=self.device)

    def set_traversal(self, block=0, stack=0, mode=-1):
        self.opts.trav_block, self.opts.trav_stack, self.opts.trav_mode = int(block), int(stack), int(mode)

    def forward(self, timing=False, count=False, stream=None):
        o = BakeOptions.from_buffer_copy(self.opts)
        o.flags |= (BAKE_FLAG_TIMING if timing else 0) | (BAKE_FLAG_COUNT if count else 0)
        _check(lib().bake_normals_batched(self._arr, self.n, C.byref(o), _ptr(self.workspace),
                                          self.workspace.numel(), _stream_handle(stream)))

    def backward(self, stream=None):
        """Gradients from grad_maps[i] into grad_lo_V[i] / grad_hi_N[i] (needs save=True)."""
        if not self.save:
            raise BakeError(BAKE_E_STATE, "batch was made without save=True")
        _check(lib().bake_normals_batched_backward(self._arr, self.n, _ptr(self.workspace),
                                                   self.workspace.numel(), _stream_handle(stream)))

    def capture(self, backward=None):
        """Record forward (+ backward when the batch saves) into a CUDA graph;
        returns the torch.cuda.CUDAGraph (replay() runs the whole batch)."""
        backward = self.save if backward is None else backward
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            self.forward()
            if backward:
                self.backward()
        torch.cuda.current_stream(self.device).wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            self.forward()
            if backward:
                self.backward()
        return g

    def counter(self, asset: int, which: int, stream=None) -> int:
        v = C.c_int64(0)
        _check(lib().bake_read_asset_counter(_ptr(self.workspace), int(asset), int(which),
                                             _stream_handle(stream), C.byref(v)))
        return v.value

    def ray_counts(self, stream=None):
        return [self.counter(i, 0, stream) for i in range(self.n)]

    def status(self, stream=None) -> int:
        v = C.c_uint32(0)
        _check(lib().bake_query_status(_ptr(self.workspace), _stream_handle(stream), C.byref(v)))
        return v.value

    def size_class(self) -> str:
        """Key of the autotuner cache: asset count and the rounded log2 of the
        batch's texel and high-poly triangle totals."""
        import math
        tex = sum(a[6] * a[6] for a in self.inputs)
        tri = sum(a[1].shape[0] for a in self.inputs)
        return f"n{self.n}-tex2^{round(math.log2(max(tex, 1)))}-tri2^{round(math.log2(max(tri, 1)))}"


TRAV_CONFIGS = [(b, s, m) for b in (64, 128, 256) for s in (8, 16, 32) for m in (0, 1, 2, 3)]


def autotune(batch: BakeBatch, reps: int = 3, cache_path: Optional[str] = None, stream=None) -> dict:
    """Time every traversal configuration on `batch` (bake_autotune), set the
    fastest on the batch and, with cache_path, store it in the JSON cache under
    the batch's size class.  Returns {"block", "stack", "mode", "ms": {...}}."""
    import json
    best = BakeOptions()
    ms = (C.c_float * len(TRAV_CONFIGS))()
    _check(lib().bake_autotune(batch._arr, batch.n, C.byref(batch.opts), int(reps), _ptr(batch.workspace),
                               batch.workspace.numel(), _stream_handle(stream), C.byref(best), ms))
    out = {"block": best.trav_block, "stack": best.trav_stack, "mode": best.trav_mode,
           "ms": {f"{b}/{s}/{m}": float(ms[i]) for i, (b, s, m) in enumerate(TRAV_CONFIGS)}}
    batch.set_traversal(best.trav_block, best.trav_stack, best.trav_mode)
    if cache_path:
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[batch.size_class()] = out
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return out


def apply_tuning(batch: BakeBatch, cache_path: str) -> bool:
    """Set the cached traversal configuration of the batch's size class, if any."""
    import json
    if not os.path.exists(cache_path):
        return False
    with open(cache_path) as f:
        e = json.load(f).get(batch.size_class())
    if not e:
        return False
    batch.set_traversal(e["block"], e["stack"], e["mode"])
    return True


def bake_batched(assets, **kw) -> BakeBatch:
    """Bake a list of assets in one launch sequence; returns the BakeBatch
    (maps / hits per asset)."""
    b = BakeBatch(assets, **kw)
    b.forward()
    return b


def stage_times() -> dict:
    """Per-stage GPU times (ms) of the last bake on this thread made with timing=True."""
    buf = (C.c_float * len(STAGES))()
    n = _check(lib().bake_stage_times(buf, len(STAGES)))
    return {STAGES[k]: float(buf[k]) for k in range(n)}


def stage_history(max_bakes: int = 64):
    """[n, 6] per-stage ms of up to the 64 most recent timed bakes, oldest first."""
    import numpy as np
    buf = (C.c_float * (6 * max_bakes))()
    n = _check(lib().bake_stage_history(buf, int(max_bakes)))
    return np.frombuffer(buf, dtype=np.float32, count=6 * n).reshape(n, 6).copy()


def version() -> str:
    return lib().bake_version().decode()


def to_device(asset, device="cuda"):
    """numpy Asset arrays -> GPU tensors in the layout the bake expects."""
    import numpy as np
    f = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
    return (f(asset.hi_V, np.float32), f(asset.hi_F, np.int32), f(asset.hi_N, np.float32),
            f(asset.lo_V, np.float32), f(asset.lo_F, np.int32), f(asset.lo_UV, np.float32))


# ---------------------------------------------------------------------------
# Hidden-face removal (Sec. 6.2)
# ---------------------------------------------------------------------------

VIS_STAGES = ("setup", "bvh_build", "rays", "flood_fill", "unused", "total")


def visibility_workspace_size(n_v: int, n_f: int) -> int:
    out = C.c_size_t(0)
    _check(lib().bake_visibility_workspace_size(int(n_v), int(n_f), C.byref(out)))
    return out.value


@dataclass
class VisibilityResult:
    visible: torch.Tensor               # [n_f] bool: some camera ray's first hit
    exterior: torch.Tensor              # [n_f] bool: visible or reached by the flood fill
    first_hit: Optional[torch.Tensor]   # [n_views, res, res] i32 (-1: no hit) when asked for
    workspace: torch.Tensor

    def counter(self, which: int, stream=None) -> int:
        v = C.c_int64(0)
        _check(lib().bake_read_counter(_ptr(self.workspace), int(which), _stream_handle(stream),
                                       C.byref(v)))
        return v.value

    def status(self, stream=None) -> int:
        v = C.c_uint32(0)
        _check(lib().bake_query_status(_ptr(self.workspace), _stream_handle(stream), C.byref(v)))
        return v.value


def visibility(V, F, eyes, target, tan_half: float, res: int, t_far: float, *, first_hit: bool = False,
               count: bool = False, timing: bool = False, workspace: Optional[torch.Tensor] = None,
               out: Optional[tuple] = None, stream=None) -> VisibilityResult:
    """The hidden-face pass on GPU tensors V [n_v,3] f32, F [n_f,3] i32 and
    eyes [n_views,3] f32 (camera positions); target: 3 floats (the point every
    camera looks at).  out: optional preallocated (visible u8 [n_f], exterior
    u8 [n_f])."""
    V = _dev_tensor(V, torch.float32, "V", (3,))
    F = _dev_tensor(F, torch.int32, "F", (3,))
    eyes = _dev_tensor(eyes, torch.float32, "eyes", (3,))
    dev = V.device
    nv, nf, nviews = V.shape[0], F.shape[0], eyes.shape[0]
    if workspace is None:
        workspace = torch.empty(visibility_workspace_size(nv, nf), dtype=torch.uint8, device=dev)
    if out is None:
        vis = torch.empty(nf, dtype=torch.uint8, device=dev)
        ext = torch.empty(nf, dtype=torch.uint8, device=dev)
    else:
        vis, ext = out
    fh = torch.empty((nviews, res, res), dtype=torch.int32, device=dev) if first_hit else None
    tg = (C.c_float * 3)(*[float(x) for x in target])
    flags = (BAKE_FLAG_COUNT if count else 0) | (BAKE_FLAG_TIMING if timing else 0)
    _check(lib().bake_visibility(_ptr(V), _ptr(F), nv, nf, _ptr(eyes), nviews, tg, float(tan_half), int(res),
                                 float(t_far), flags, _ptr(vis), _ptr(ext), _ptr(fh), _ptr(workspace),
                                 workspace.numel(), _stream_handle(stream)))
    return VisibilityResult(vis.view(torch.bool), ext.view(torch.bool), fh, workspace)


# ---------------------------------------------------------------------------
# Backprojection precompute (Sec. 7.4, TextureGen Postprocessing)
# ---------------------------------------------------------------------------

MAP_STAGES = ("gbuffer", "bvh_build", "depth_rays", "maps", "unused", "total")


def view_maps_workspace_size(n_v: int, n_f: int, res: int, n_views: int, img_res: int) -> int:
    out = C.c_size_t(0)
    _check(lib().bake_view_maps_workspace_size(int(n_v), int(n_f), int(res), int(n_views), int(img_res),
                                               C.byref(out)))
    return out.value


@dataclass
class ViewMapsResult:
    uv: torch.Tensor               # [n_views, res, res, 2] image coordinates (col, row); (-1, -1) outside
    inc: torch.Tensor              # [n_views, res, res] incidence after the visibility test
    depth: Optional[torch.Tensor]  # [n_views, img_res, img_res] first-hit distances of the pixel rays when asked for
    workspace: torch.Tensor

    def counter(self, which: int, stream=None) -> int:
        v = C.c_int64(0)
        _check(lib().bake_read_counter(_ptr(self.workspace), int(which), _stream_handle(stream),
                                       C.byref(v)))
        return v.value


def view_maps(V, F, UV, res: int, eyes, target, tan_half: float, img_res: int, t_far: float, depth_tol: float, *,
              depth: bool = False, timing: bool = False, count: bool = False,
              workspace: Optional[torch.Tensor] = None,
              out: Optional[tuple] = None, stream=None) -> ViewMapsResult:
    """The backprojection precompute on GPU tensors V [n_v,3] f32, F [n_f,3]
    i32, UV [n_f,3,2] f32 and eyes [n_views,3] f32 (target: 3 floats).
    out: optional preallocated (uv [n_views,res,res,2] f32, inc [n_views,res,res] f32)."""
    V = _dev_tensor(V, torch.float32, "V", (3,))
    F = _dev_tensor(F, torch.int32, "F", (3,))
    UV = _dev_tensor(UV, torch.float32, "UV", (3, 2))
    eyes = _dev_tensor(eyes, torch.float32, "eyes", (3,))
    dev = V.device
    nv, nf, k = V.shape[0], F.shape[0], eyes.shape[0]
    if workspace is None:
        workspace = torch.empty(view_maps_workspace_size(nv, nf, res, k, img_res), dtype=torch.uint8, device=dev)
    if out is None:
        uv = torch.empty((k, res, res, 2), dtype=torch.float32, device=dev)
        inc = torch.empty((k, res, res), dtype=torch.float32, device=dev)
    else:
        uv, inc = out
    dep = torch.empty((k, img_res, img_res), dtype=torch.float32, device=dev) if depth else None
    tg = (C.c_float * 3)(*[float(x) for x in target])
    flags = (BAKE_FLAG_TIMING if timing else 0) | (BAKE_FLAG_COUNT if count else 0)
    _check(lib().bake_view_maps(_ptr(V), _ptr(F), _ptr(UV), nv, nf, int(res), _ptr(eyes), k, tg, float(tan_half),
                                int(img_res), float(t_far), float(depth_tol), flags, _ptr(uv), _ptr(inc), _ptr(dep),
                                _ptr(workspace), workspace.numel(), _stream_handle(stream)))
    return ViewMapsResult(uv, inc, dep, workspace)



# ---------------------------------------------------------------------------
# Mesh simplification (Sec. 6.1)
# ---------------------------------------------------------------------------

BAKE_QEM_MIDPOINT = 1


def qem_workspace_size(n_v: int, n_f: int) -> int:
    out = C.c_size_t(0)
    _check(lib().bake_qem_workspace_size(int(n_v), int(n_f), C.byref(out)))
    return out.value


@dataclass
class QemEdges:
    edges: torch.Tensor   # [ne, 2] i32, v0 < v1 in (v0, v1) order
    valid: torch.Tensor   # [ne] bool: the collapse is allowed
    faces: torch.Tensor   # [ne] i32: faces on the edge
    cost: torch.Tensor    # [ne] f64
    p: torch.Tensor       # [ne, 3] f64 placement
    Q: torch.Tensor       # [n_v, 10] f64 vertex quadrics


def qem_edges(V, F, *, midpoint: bool = False, workspace: Optional[torch.Tensor] = None, stream=None) -> QemEdges:
    """Every edge of the mesh (GPU tensors V [n_v,3] f32, F [n_f,3] i32) with
    its collapse evaluated, as the first simplification round sees it."""
    V = _dev_tensor(V, torch.float32, "V", (3,))
    F = _dev_tensor(F, torch.int32, "F", (3,))
    dev = V.device
    nv, nf = V.shape[0], F.shape[0]
    if workspace is None:
        workspace = torch.empty(qem_workspace_size(nv, nf), dtype=torch.uint8, device=dev)
    cap = 3 * nf
    E = torch.empty((cap, 2), dtype=torch.int32, device=dev)
    ok = torch.empty(cap, dtype=torch.uint8, device=dev)
    fc = torch.empty(cap, dtype=torch.int32, device=dev)
    cost = torch.empty(cap, dtype=torch.float64, device=dev)
    P = torch.empty((cap, 3), dtype=torch.float64, device=dev)
    Q = torch.empty((nv, 10), dtype=torch.float64, device=dev)
    n = C.c_int64(0)
    _check(lib().bake_qem_edges(_ptr(V), _ptr(F), nv, nf, BAKE_QEM_MIDPOINT if midpoint else 0, cap, _ptr(E),
                                _ptr(ok), _ptr(fc), _ptr(cost), _ptr(P), _ptr(Q), C.byref(n), _ptr(workspace),
                                workspace.numel(), _stream_handle(stream)))
    k = n.value
    return QemEdges(E[:k], ok[:k].bool(), fc[:k], cost[:k], P[:k], Q)


@dataclass
class QemResult:
    V: torch.Tensor        # [n_v', 3] f32
    F: torch.Tensor        # [n_f', 3] i32
    rounds: int
    stats: "numpy.ndarray"  # [rounds, 4]: edges, allowed edges, collapses, faces after the round
    times_ms: Optional[tuple] = None  # (per-edge evaluation launches summed, whole call) when timed


def qem_simplify(V, F, target: int, *, rho: float = 0.25, max_rounds: int = 1000, midpoint: bool = False,
                 timing: bool = False, workspace: Optional[torch.Tensor] = None, out: Optional[tuple] = None,
                 stream=None) -> QemResult:
    """Simplify the mesh (GPU tensors V [n_v,3] f32, F [n_f,3] i32) to `target`
    faces by rounds of quadric edge collapses (blocking).  out: optional
    preallocated (V_out [n_v,3] f32, F_out [n_f,3] i32)."""
    import numpy as np
    V = _dev_tensor(V, torch.float32, "V", (3,))
    F = _dev_tensor(F, torch.int32, "F", (3,))
    dev = V.device
    nv, nf = V.shape[0], F.shape[0]
    if workspace is None:
        workspace = torch.empty(qem_workspace_size(nv, nf), dtype=torch.uint8, device=dev)
    if out is None:
        Vo = torch.empty((nv, 3), dtype=torch.float32, device=dev)
        Fo = torch.empty((nf, 3), dtype=torch.int32, device=dev)
    else:
        Vo, Fo = out
    counts = (C.c_int64 * 2)()
    rounds = C.c_int32(0)
    stats = np.zeros((max(int(max_rounds), 1), 4), np.int64)
    tms = (C.c_float * 2)() if timing else None
    _check(lib().bake_qem_simplify(_ptr(V), _ptr(F), nv, nf, int(target), float(rho), int(max_rounds),
                                   BAKE_QEM_MIDPOINT if midpoint else 0, _ptr(Vo), _ptr(Fo), counts,
                                   C.byref(rounds), stats.ctypes.data, tms, _ptr(workspace), workspace.numel(),
                                   _stream_handle(stream)))
    r = rounds.value
    return QemResult(Vo[:counts[0]], Fo[:counts[1]], r, stats[:r], (tms[0], tms[1]) if timing else None)
