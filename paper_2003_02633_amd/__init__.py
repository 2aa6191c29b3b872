"""MI355X-native inline 3-vector compression (Trojak & Witherden, arXiv 2003.02633).

Thin Python binding over the C ABI of ``libvc.so`` (declared in ``include/vc.h``
and ``include/vc_ext.h``).  Every function here only marshals arguments --
device pointers of torch tensors and the current HIP stream -- and calls the
library; all computation runs in the library's HIP kernels.  If the library is
not built, every call raises (there is no CPU fallback).

PyTorch is used for device memory and streams only.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvc.so")

VC_SUCCESS = 0
STATUS = {0: "VC_SUCCESS", 1: "VC_ERROR_INVALID_VALUE", 2: "VC_ERROR_MISALIGNED",
          3: "VC_ERROR_UNSUPPORTED_CODEC", 4: "VC_ERROR_LAUNCH", 5: "VC_ERROR_HIP",
          6: "VC_ERROR_OUT_OF_MEMORY", 7: "VC_ERROR_OVERLAP"}
LAYOUTS = {"0,7,22-17-18": 0, "0,7,23-17-17": 1, "0,8,23-16-17": 2, "1,8,23-16-16": 3}
MODES = {"plain": 0, "tanh": 1, "cos": 2, "frac": 3}
OPS = {"axpy": 0, "dot": 1, "norm2": 2, "encode": 3}


class VcError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}")
        self.status = status


class vc_codec(C.Structure):
    """Mirror of ``vc_codec`` in include/vc.h."""
    _fields_ = [("struct_size", C.c_uint32), ("layout", C.c_uint32), ("mode", C.c_uint32),
                ("mag_round", C.c_uint32), ("compand_mask", C.c_uint32), ("gamma", C.c_float),
                ("frac_P", C.c_uint64), ("precision", C.c_uint32), ("reserved0", C.c_uint32)]


class vc_segment(C.Structure):
    """Mirror of ``vc_segment`` in include/vc.h."""
    _fields_ = [("op", C.c_uint32), ("alpha", C.c_float), ("n", C.c_uint64), ("a", C.c_void_p),
                ("b", C.c_void_p), ("out", C.c_void_p)]


_lib = None
_vp = C.c_void_p
_SIGS = {
    "vc_codec_init": ([C.POINTER(vc_codec), C.c_char_p], C.c_int),
    "vc_encode": ([C.POINTER(vc_codec), _vp, _vp, C.c_size_t, _vp], C.c_int),
    "vc_decode": ([C.POINTER(vc_codec), _vp, _vp, C.c_size_t, _vp], C.c_int),
    "vc_axpy": ([C.POINTER(vc_codec), C.c_float, _vp, _vp, _vp, C.c_size_t, _vp], C.c_int),
    "vc_dot": ([C.POINTER(vc_codec), _vp, _vp, C.c_size_t, _vp, _vp], C.c_int),
    "vc_norm2": ([C.POINTER(vc_codec), _vp, C.c_size_t, _vp, _vp], C.c_int),
    "vc_dot_noalloc": ([C.POINTER(vc_codec), _vp, _vp, C.c_size_t, _vp, _vp], C.c_int),
    "vc_fused_apply": ([C.POINTER(vc_codec), _vp, C.c_int, C.c_int, _vp, _vp, C.c_size_t, _vp], C.c_int),
    "vc_batch_plan_create": ([C.POINTER(_vp), C.POINTER(vc_codec), C.POINTER(vc_segment), C.c_int, _vp],
                             C.c_int),
    "vc_batch_plan_run": ([_vp, _vp], C.c_int),
    "vc_batch_plan_run_separate": ([_vp, _vp], C.c_int),
    "vc_batch_plan_destroy": ([_vp], C.c_int),
    "vc_status_string": ([C.c_int], C.c_char_p),
    "vc_version": ([], C.c_char_p),
    "vcx_axpy_dump": ([C.POINTER(vc_codec), C.c_float, _vp, _vp, _vp, _vp, C.c_size_t, _vp], C.c_int),
    "vcb_axpy_f32": ([C.c_float, _vp, _vp, _vp, C.c_size_t, _vp], C.c_int),
    "vcb_axpy_bf16x4": ([C.c_float, _vp, _vp, _vp, C.c_size_t, _vp], C.c_int),
    "vcb_axpy_f16x4": ([C.c_float, _vp, _vp, _vp, C.c_size_t, _vp], C.c_int),
    "vcb_copy": ([_vp, _vp, C.c_size_t, _vp], C.c_int),
    "vcx_inline_params": ([C.POINTER(vc_codec), _vp, C.c_size_t], C.c_int),
    "vcx_inline_params_size": ([], C.c_size_t),
    "vcx_set_stream_config": ([C.c_int, C.c_int, C.c_int, C.c_int], C.c_int),
    "vcx_get_stream_config": ([C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
    "vcx_load_tuning": ([C.c_char_p], C.c_int),
    "vcx_batch_plan_run_separate_graph": ([_vp, _vp], C.c_int),
    "vcx_batch_plan_info": ([_vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint32)], C.c_int),
    "vcx_set_batch_config": ([C.c_int, C.c_int, C.c_int], C.c_int),
    "vcx_get_batch_config": ([C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
    "vcx_set_apply_mode": ([C.c_int], C.c_int),
    "vcx_get_apply_mode": ([], C.c_int),
    "vc_flux_div_tp": ([C.POINTER(vc_codec), _vp, C.c_int, C.c_int, _vp, _vp, C.c_size_t, _vp], C.c_int),
    "vcb_flux_div_tp_f32": ([_vp, C.c_int, C.c_int, _vp, _vp, C.c_size_t, _vp], C.c_int),
    "vc_gather_decode": ([C.POINTER(vc_codec), _vp, C.c_size_t, _vp, C.c_size_t, _vp, _vp], C.c_int),
    "vc_scatter_encode": ([C.POINTER(vc_codec), _vp, _vp, C.c_size_t, _vp, C.c_size_t, _vp], C.c_int),
    "vcb_gather_f32": ([_vp, C.c_size_t, _vp, C.c_size_t, _vp, _vp], C.c_int),
    "vcx_error_hist": ([C.POINTER(vc_codec), _vp, C.c_size_t, _vp, C.c_int, _vp, _vp, _vp], C.c_int),
}


def lib():
    """Load libvc.so (built in-tree by ``python -m paper_2003_02633_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2003_02633_amd.build`")
        # torch first: its HIP runtime is then the one libvc.so binds to.  Loaded the other way
        # round, the process holds two HIP runtimes, and the library's finds no device.
        _torch()
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(st: int, where: str):
    if st != VC_SUCCESS:
        raise VcError(st, where)


PRECISIONS = {"f64": 0, "f32": 1}


def codec(layout: str = "0,7,22-17-18", mode: str = "plain", gamma: float = 0.5, P: int = 1 << 17,
          compand: str = "both", precision: str = "f64", mag_round: str = "rne") -> vc_codec:
    c = vc_codec()
    _check(lib().vc_codec_init(C.byref(c), layout.encode()), "vc_codec_init")
    c.precision = PRECISIONS[precision]
    c.mode = MODES[mode]
    c.mag_round = {"rne": 0, "trunc": 1}[mag_round]
    c.gamma = float(gamma)
    c.frac_P = int(P)
    c.compand_mask = {"both": 3, "phi": 1, "theta": 2, "none": 0}[compand]
    return c


def _torch():
    import torch
    return torch


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _require(t, dtype, what):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{what}: expected a contiguous CUDA tensor of {dtype}")


def vc_encode(c: vc_codec, xyz, out=None, stream=None):
    """codes[N] (int64 holding uint64 bit patterns) of float32 vectors xyz[N, 3]."""
    torch = _torch()
    _require(xyz, torch.float32, "vc_encode xyz")
    n = xyz.numel() // 3
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=xyz.device)
    _require(out, torch.int64, "vc_encode out")
    _check(lib().vc_encode(C.byref(c), _ptr(xyz), _ptr(out), n, _stream(stream)), "vc_encode")
    return out


def vc_decode(c: vc_codec, codes, out=None, stream=None):
    torch = _torch()
    _require(codes, torch.int64, "vc_decode codes")
    n = codes.numel()
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=codes.device)
    _require(out, torch.float32, "vc_decode out")
    _check(lib().vc_decode(C.byref(c), _ptr(codes), _ptr(out), n, _stream(stream)), "vc_decode")
    return out


def vc_axpy(c: vc_codec, alpha: float, a, b, out=None, stream=None):
    torch = _torch()
    _require(a, torch.int64, "vc_axpy a")
    _require(b, torch.int64, "vc_axpy b")
    n = a.numel()
    if b.numel() != n:
        raise ValueError("vc_axpy: a and b differ in length")
    if out is None:
        out = torch.empty_like(a)
    _check(lib().vc_axpy(C.byref(c), float(alpha), _ptr(a), _ptr(b), _ptr(out), n, _stream(stream)), "vc_axpy")
    return out


def vcx_axpy_dump(c: vc_codec, alpha: float, a, b, out=None, c32=None, stream=None):
    torch = _torch()
    n = a.numel()
    if out is None:
        out = torch.empty_like(a)
    if c32 is None:
        c32 = torch.empty((n, 3), dtype=torch.float32, device=a.device)
    _check(lib().vcx_axpy_dump(C.byref(c), float(alpha), _ptr(a), _ptr(b), _ptr(out), _ptr(c32), n,
                               _stream(stream)), "vcx_axpy_dump")
    return out, c32


def vc_dot(c: vc_codec, a, b, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty(1, dtype=torch.float32, device=a.device)
    _check(lib().vc_dot(C.byref(c), _ptr(a), _ptr(b), a.numel(), _ptr(out), _stream(stream)), "vc_dot")
    return out


def vc_dot_noalloc(c: vc_codec, a, b, out, stream=None):
    """vc_dot through the allocation-free entry point; ``out`` (one device float) is required."""
    torch = _torch()
    _require(out, torch.float32, "vc_dot_noalloc out")
    _check(lib().vc_dot_noalloc(C.byref(c), _ptr(a), _ptr(b), a.numel(), _ptr(out), _stream(stream)),
           "vc_dot_noalloc")
    return out


def vc_norm2(c: vc_codec, a, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty(1, dtype=torch.float32, device=a.device)
    _check(lib().vc_norm2(C.byref(c), _ptr(a), a.numel(), _ptr(out), _stream(stream)), "vc_norm2")
    return out


def vc_fused_apply(c: vc_codec, M, U, out=None, stream=None):
    """out[e] = M @ decode(U[e]); M [rows, cols] float32, U [n_elem, cols] codes."""
    torch = _torch()
    _require(M, torch.float32, "vc_fused_apply M")
    _require(U, torch.int64, "vc_fused_apply U")
    rows, cols = M.shape
    n_elem = U.numel() // cols
    if out is None:
        out = torch.empty((n_elem, rows, 3), dtype=torch.float32, device=U.device)
    _check(lib().vc_fused_apply(C.byref(c), _ptr(M), rows, cols, _ptr(U), _ptr(out), n_elem, _stream(stream)),
           "vc_fused_apply")
    return out


def vcb_axpy_f32(alpha, a, b, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty_like(a)
    _check(lib().vcb_axpy_f32(float(alpha), _ptr(a), _ptr(b), _ptr(out), a.numel(), _stream(stream)),
           "vcb_axpy_f32")
    return out


def vcb_axpy_h4(kind: str, alpha, a, b, out=None, stream=None):
    """kind 'bf16' or 'f16'; a, b: int16/uint16 tensors [N, 4]."""
    if out is None:
        out = _torch().empty_like(a)
    f = lib().vcb_axpy_bf16x4 if kind == "bf16" else lib().vcb_axpy_f16x4
    _check(f(float(alpha), _ptr(a), _ptr(b), _ptr(out), a.numel() // 4, _stream(stream)), f"vcb_axpy_{kind}x4")
    return out


def vcb_copy(src, dst, stream=None):
    nbytes = src.numel() * src.element_size()
    _check(lib().vcb_copy(_ptr(src), _ptr(dst), nbytes, _stream(stream)), "vcb_copy")
    return dst


def vc_flux_div_tp(c: vc_codec, d, F, out=None, stream=None):
    """Alg. (fr_fdiv_comp) on hexahedra: d float32 [3][q][q] (device), F int64 codes
    [n_elem][q^3][np] (device); returns float32 [n_elem][q^3][np]."""
    torch = _torch()
    _require(d, torch.float32, "vc_flux_div_tp d")
    _require(F, torch.int64, "vc_flux_div_tp F")
    q = d.shape[-1]
    ne, ns, npq = F.shape
    if out is None:
        out = torch.empty((ne, ns, npq), dtype=torch.float32, device=F.device)
    _check(lib().vc_flux_div_tp(C.byref(c), _ptr(d), q, npq, _ptr(F), _ptr(out), ne, _stream(stream)),
           "vc_flux_div_tp")
    return out


def vcb_flux_div_tp_f32(d, F, out=None, stream=None):
    """uncompressed baseline: F float32 [n_elem][q^3][np][3]"""
    torch = _torch()
    q = d.shape[-1]
    ne, ns, npq, _ = F.shape
    if out is None:
        out = torch.empty((ne, ns, npq), dtype=torch.float32, device=F.device)
    _check(lib().vcb_flux_div_tp_f32(_ptr(d), q, npq, _ptr(F), _ptr(out), ne, _stream(stream)),
           "vcb_flux_div_tp_f32")
    return out


def vc_gather_decode(c: vc_codec, codes, idx, out=None, stream=None):
    """out[i] = decode(codes[idx[i]]); codes int64 [n_src], idx int32 [n] (device)"""
    torch = _torch()
    _require(codes, torch.int64, "vc_gather_decode codes")
    _require(idx, torch.int32, "vc_gather_decode idx")
    n = idx.numel()
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=idx.device)
    _check(lib().vc_gather_decode(C.byref(c), _ptr(codes), codes.numel(), _ptr(idx), n, _ptr(out), _stream(stream)),
           "vc_gather_decode")
    return out


def vc_scatter_encode(c: vc_codec, xyz, idx, codes, stream=None):
    """codes[idx[i]] = encode(xyz[i])"""
    torch = _torch()
    _require(xyz, torch.float32, "vc_scatter_encode xyz")
    _require(idx, torch.int32, "vc_scatter_encode idx")
    _require(codes, torch.int64, "vc_scatter_encode codes")
    _check(lib().vc_scatter_encode(C.byref(c), _ptr(xyz), _ptr(idx), idx.numel(), _ptr(codes), codes.numel(),
                                   _stream(stream)), "vc_scatter_encode")
    return codes


def vcb_gather_f32(src, idx, out=None, stream=None):
    torch = _torch()
    n = idx.numel()
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=idx.device)
    _check(lib().vcb_gather_f32(_ptr(src), src.numel() // 3, _ptr(idx), n, _ptr(out), _stream(stream)),
           "vcb_gather_f32")
    return out


def error_hist(c: vc_codec, xyz, edges, stream=None):
    """(counts [3, nedges+1] int64, excluded, stats [3, 3] = (sum, sum of squares, max)) of the
    codec's errors over the float32 vectors xyz [N, 3] (device); edges: float64 device tensor."""
    torch = _torch()
    _require(xyz, torch.float32, "error_hist xyz")
    _require(edges, torch.float64, "error_hist edges")
    ne = edges.numel()
    counts = torch.empty(3 * (ne + 1) + 1, dtype=torch.int64, device=xyz.device)
    stats = torch.empty(9, dtype=torch.float64, device=xyz.device)
    _check(lib().vcx_error_hist(C.byref(c), _ptr(xyz), xyz.numel() // 3, _ptr(edges), ne, _ptr(counts),
                                _ptr(stats), _stream(stream)), "vcx_error_hist")
    cnt = counts.cpu()
    return cnt[:-1].reshape(3, ne + 1), int(cnt[-1]), stats.cpu().reshape(3, 3)


def set_stream_config(block: int, vpt: int, nt: int, precision: str = "both"):
    """axpy launch configuration for one encoder precision ("f64", "f32") or both"""
    p = -1 if precision == "both" else PRECISIONS[precision]
    _check(lib().vcx_set_stream_config(p, block, vpt, nt), "vcx_set_stream_config")


def get_stream_config(precision: str = "f64"):
    b, v, t = C.c_int(), C.c_int(), C.c_int()
    _check(lib().vcx_get_stream_config(PRECISIONS[precision], C.byref(b), C.byref(v), C.byref(t)),
           "vcx_get_stream_config")
    return b.value, v.value, t.value


def set_batch_config(ua: int, ud: int, un: int):
    """tile shape of batch plans created from now on (default codec): code pairs per lane for
    axpy (1, 2), dot (2, 4, 8) and norm2 (4, 8, 16) tiles"""
    _check(lib().vcx_set_batch_config(ua, ud, un), "vcx_set_batch_config")


def get_batch_config():
    a, d, n = C.c_int(), C.c_int(), C.c_int()
    _check(lib().vcx_get_batch_config(C.byref(a), C.byref(d), C.byref(n)), "vcx_get_batch_config")
    return a.value, d.value, n.value


APPLY_MODES = {"auto": 0, "fp32": 1}


def set_apply_mode(mode: str):
    """matrix cores of vc_fused_apply: 'auto' (bf16 cores with three-part splits where the
    operator fits the LDS, else FP32) or 'fp32' (always the FP32 cores)"""
    _check(lib().vcx_set_apply_mode(APPLY_MODES[mode]), "vcx_set_apply_mode")


def get_apply_mode() -> str:
    m = lib().vcx_get_apply_mode()
    return {v: k for k, v in APPLY_MODES.items()}[m]


def _seg_ptr(seg, key):
    """device address of a segment operand: a tensor, a raw integer address, or None"""
    v = seg.get(key)
    if v is None:
        return None
    return int(v) if isinstance(v, int) else v.data_ptr()


class BatchPlan:
    """Persistent batched launch over a segment table (see vc_batch_plan_create)."""

    def __init__(self, c: vc_codec, segments, stream=None):
        arr = (vc_segment * len(segments))()
        for i, s in enumerate(segments):
            arr[i] = vc_segment(OPS[s["op"]], float(s.get("alpha", 1.0)), int(s["n"]),
                                _seg_ptr(s, "a"), _seg_ptr(s, "b"),
                                _seg_ptr(s, "out"))
        self._keep = segments
        self._c = c
        self.plan = C.c_void_p()
        _check(lib().vc_batch_plan_create(C.byref(self.plan), C.byref(c), arr, len(segments), _stream(stream)),
               "vc_batch_plan_create")

    def run(self, stream=None):
        _check(lib().vc_batch_plan_run(self.plan, _stream(stream)), "vc_batch_plan_run")

    def run_separate(self, stream=None):
        _check(lib().vc_batch_plan_run_separate(self.plan, _stream(stream)), "vc_batch_plan_run_separate")

    def run_separate_graph(self, stream=None):
        _check(lib().vcx_batch_plan_run_separate_graph(self.plan, _stream(stream)),
               "vcx_batch_plan_run_separate_graph")

    def info(self):
        """(tiles walked by the persistent kernel, its grid size)"""
        t, g = C.c_uint64(), C.c_uint32()
        _check(lib().vcx_batch_plan_info(self.plan, C.byref(t), C.byref(g)), "vcx_batch_plan_info")
        return t.value, g.value

    def close(self):
        if self.plan:
            lib().vc_batch_plan_destroy(self.plan)
            self.plan = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
