"""CPU oracle for the inline 3-vector compression of arXiv 2003.02633.

TEST INFRASTRUCTURE ONLY.  A plain FP64/integer C implementation (``vco.c``)
written from the paper, wrapped with ctypes and numpy.  Only ``tests/``, the
smoke check and the CPU-baseline leg of ``bench.py`` may import this package;
the product library (``paper_2003_02633_amd``) never imports it and shares no
code with it.

Pinning status of each function is listed in ``oracle/README.md``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

PLAIN, TANH, COS, FRAC = 0, 1, 2, 3
RNE, TRUNC = 0, 1
COMP_PHI, COMP_THETA = 1, 2

# <s,e,m>-p-t layouts of §2.2-2.3 with their exponent biases
LAYOUTS = {
    "0,7,22-17-18": (0, 7, 22, 17, 18, 80),
    "0,7,23-17-17": (0, 7, 23, 17, 17, 80),
    "0,8,23-16-17": (0, 8, 23, 16, 17, 127),
    "1,8,23-16-16": (1, 8, 23, 16, 16, 127),
}
MODES = {"plain": PLAIN, "tanh": TANH, "cos": COS, "frac": FRAC}


class Codec(C.Structure):
    _fields_ = [("s", C.c_int), ("e", C.c_int), ("m", C.c_int), ("p", C.c_int), ("t", C.c_int),
                ("bias", C.c_int), ("mode", C.c_int), ("mag_round", C.c_int),
                ("compand_mask", C.c_int), ("gamma", C.c_double), ("P", C.c_uint64)]

    def __repr__(self):  # pragma: no cover - debugging aid
        return (f"Codec(<{self.s},{self.e},{self.m}>-{self.p}-{self.t}, b={self.bias}, "
                f"mode={self.mode}, mag={self.mag_round}, mask={self.compand_mask}, "
                f"gamma={self.gamma}, P={self.P})")


class Detail(C.Structure):
    _fields_ = [("Q_theta", C.c_double), ("w_theta", C.c_double), ("Q_phi", C.c_double),
                ("w_phi", C.c_double), ("n_theta", C.c_int64), ("n_phi", C.c_int64),
                ("r", C.c_double), ("mid_rel", C.c_double), ("saturated", C.c_int),
                ("flushed", C.c_int)]


_lib = None


def lib():
    """Load liboracle.so, building it with gcc if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER
        cp = C.POINTER(Codec)
        L.vco_check.argtypes = [cp]
        L.vco_check.restype = C.c_int
        for f in ("vco_nmax_theta", "vco_nmax_phi", "vco_frac_T"):
            getattr(L, f).argtypes = [cp]
            getattr(L, f).restype = C.c_uint64
        L.vco_encode.argtypes = [cp, C.c_float, C.c_float, C.c_float]
        L.vco_encode.restype = C.c_uint64
        L.vco_encode_detail.argtypes = [cp, C.c_float, C.c_float, C.c_float, P(Detail)]
        L.vco_encode_detail.restype = C.c_uint64
        L.vco_decode64.argtypes = [cp, C.c_uint64, P(C.c_double)]
        L.vco_decode.argtypes = [cp, C.c_uint64, P(C.c_float)]
        L.vco_rn32_fma.argtypes = [C.c_float, C.c_float, C.c_float]
        L.vco_rn32_fma.restype = C.c_float
        L.vco_round_norm.argtypes = [C.c_float, C.c_float, C.c_float, C.c_int, C.c_double, P(C.c_int)]
        L.vco_round_norm.restype = C.c_double
        L.vco_exact_sign.argtypes = [P(C.c_double), C.c_int]
        L.vco_exact_sign.restype = C.c_int
        vp = C.c_void_p
        L.vco_encode_batch.argtypes = [cp, vp, vp, C.c_size_t, C.c_int]
        L.vco_encode_detail_batch.argtypes = [cp, vp, vp, vp, vp, C.c_size_t, C.c_int]
        L.vco_decode_batch.argtypes = [cp, vp, vp, C.c_size_t, C.c_int]
        L.vco_decode64_batch.argtypes = [cp, vp, vp, C.c_size_t, C.c_int]
        L.vco_axpy_batch.argtypes = [cp, C.c_float, vp, vp, vp, vp, vp, C.c_size_t, C.c_int]
        L.vco_dot.argtypes = [cp, vp, vp, C.c_size_t, C.c_int]
        L.vco_dot.restype = C.c_double
        L.vco_norm2.argtypes = [cp, vp, C.c_size_t, C.c_int]
        L.vco_norm2.restype = C.c_double
        L.vco_apply.argtypes = [cp, vp, C.c_int, C.c_int, vp, vp, C.c_size_t, C.c_int]
        L.vco_max_threads.restype = C.c_int
        L.vco_flux_div.argtypes = [cp, vp, C.c_int, C.c_int, vp, vp, C.c_size_t, C.c_int]
        L.vco_error_hist.argtypes = [cp, vp, C.c_size_t, vp, C.c_int, vp, vp, C.c_int]
        _lib = L
    return _lib


def codec(layout: str = "0,7,22-17-18", mode: str = "plain", gamma: float = 0.5, P: int = 0,
          mag_round: str = "rne", compand: str = "both", bias: int | None = None,
          fields: tuple | None = None) -> Codec:
    """Build a codec.  ``fields`` = (s, e, m, p, t) overrides ``layout`` (tiny test layouts)."""
    if fields is not None:
        s, e, m, p, t = fields
        b = bias if bias is not None else (1 << (e - 1)) - 1
    else:
        s, e, m, p, t, b = LAYOUTS[layout]
        if bias is not None:
            b = bias
    mask = {"both": COMP_PHI | COMP_THETA, "phi": COMP_PHI, "theta": COMP_THETA, "none": 0}[compand]
    c = Codec(s, e, m, p, t, b, MODES[mode], RNE if mag_round == "rne" else TRUNC, mask,
              float(gamma), int(P))
    rc = lib().vco_check(C.byref(c))
    if rc != 0:
        raise ValueError(f"invalid oracle codec parameters (code {rc}): {c!r}")
    return c


def nmax(c: Codec) -> tuple[int, int]:
    """(n_theta_max, n_phi_max)"""
    return int(lib().vco_nmax_theta(C.byref(c))), int(lib().vco_nmax_phi(C.byref(c)))


def frac_T(c: Codec) -> int:
    return int(lib().vco_frac_T(C.byref(c)))


def _f32xyz(xyz) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32).reshape(-1, 3))
    return a


def _u64(w) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(w).astype(np.uint64, copy=False).reshape(-1))


def encode(c: Codec, xyz, threads: int = 0) -> np.ndarray:
    a = _f32xyz(xyz)
    out = np.empty(a.shape[0], dtype=np.uint64)
    lib().vco_encode_batch(C.byref(c), a.ctypes.data, out.ctypes.data, a.shape[0], threads)
    return out


def encode_detail(c: Codec, xyz, threads: int = 0):
    """codes, q5 [N,5] = (Q_theta, w_theta, Q_phi, w_phi, mid_rel), flags (bit0 sat, bit1 flush)"""
    a = _f32xyz(xyz)
    n = a.shape[0]
    out = np.empty(n, dtype=np.uint64)
    q5 = np.empty((n, 5), dtype=np.float64)
    fl = np.empty(n, dtype=np.int32)
    lib().vco_encode_detail_batch(C.byref(c), a.ctypes.data, out.ctypes.data, q5.ctypes.data,
                                  fl.ctypes.data, n, threads)
    return out, q5, fl


def encode_one(c: Codec, x: float, y: float, z: float) -> int:
    return int(lib().vco_encode(C.byref(c), x, y, z))


def detail_one(c: Codec, x: float, y: float, z: float) -> tuple[int, Detail]:
    d = Detail()
    w = lib().vco_encode_detail(C.byref(c), x, y, z, C.byref(d))
    return int(w), d


def decode(c: Codec, w, threads: int = 0) -> np.ndarray:
    w = _u64(w)
    out = np.empty((w.shape[0], 3), dtype=np.float32)
    lib().vco_decode_batch(C.byref(c), w.ctypes.data, out.ctypes.data, w.shape[0], threads)
    return out


def decode64(c: Codec, w, threads: int = 0) -> np.ndarray:
    w = _u64(w)
    out = np.empty((w.shape[0], 3), dtype=np.float64)
    lib().vco_decode64_batch(C.byref(c), w.ctypes.data, out.ctypes.data, w.shape[0], threads)
    return out


def axpy(c: Codec, alpha: float, a, b, threads: int = 0, want_c32: bool = False,
         want_c64: bool = False):
    """codes of alpha*a + b; optionally the single-precision pre-encode sum and the FP64 sum
    of the exactly decoded operands."""
    a = _u64(a)
    b = _u64(b)
    n = a.shape[0]
    out = np.empty(n, dtype=np.uint64)
    c32 = np.empty((n, 3), dtype=np.float32) if want_c32 else None
    c64 = np.empty((n, 3), dtype=np.float64) if want_c64 else None
    lib().vco_axpy_batch(C.byref(c), float(alpha), a.ctypes.data, b.ctypes.data, out.ctypes.data,
                         None if c32 is None else c32.ctypes.data,
                         None if c64 is None else c64.ctypes.data, n, threads)
    res = [out]
    if want_c32:
        res.append(c32)
    if want_c64:
        res.append(c64)
    return res[0] if len(res) == 1 else tuple(res)


def dot(c: Codec, a, b, threads: int = 0) -> float:
    a = _u64(a)
    b = _u64(b)
    return float(lib().vco_dot(C.byref(c), a.ctypes.data, b.ctypes.data, a.shape[0], threads))


def norm2(c: Codec, a, threads: int = 0) -> float:
    a = _u64(a)
    return float(lib().vco_norm2(C.byref(c), a.ctypes.data, a.shape[0], threads))


def apply(c: Codec, M, U, threads: int = 0) -> np.ndarray:
    """out[e] = M @ decode(U[e]) in FP64; M [rows, cols] f32, U [n_elem, cols] codes."""
    M = np.ascontiguousarray(np.asarray(M, dtype=np.float32))
    rows, cols = M.shape
    U = np.ascontiguousarray(np.asarray(U).astype(np.uint64, copy=False).reshape(-1, cols))
    out = np.empty((U.shape[0], rows, 3), dtype=np.float64)
    lib().vco_apply(C.byref(c), M.ctypes.data, rows, cols, U.ctypes.data, out.ctypes.data,
                    U.shape[0], threads)
    return out


def flux_div(c: Codec, D, F, threads: int = 0) -> np.ndarray:
    """Alg. (fr_fdiv_comp) in FP64: D [3 ns][ns] (as float32), F codes [n_elem][ns][np];
    returns [n_elem][ns][np]."""
    D = np.ascontiguousarray(np.asarray(D, dtype=np.float32))
    ns = D.shape[1]
    assert D.shape[0] == 3 * ns
    F = np.ascontiguousarray(np.asarray(F).astype(np.uint64, copy=False))
    ne, ns2, npq = F.shape
    assert ns2 == ns
    out = np.empty((ne, ns, npq), dtype=np.float64)
    lib().vco_flux_div(C.byref(c), D.ctypes.data, ns, npq, F.ctypes.data, out.ctypes.data, ne, threads)
    return out


def log_edges(lo_exp: float = -12.0, hi_exp: float = -2.0, per_decade: int = 10) -> np.ndarray:
    """histogram edges 10^(lo + i / per_decade), i = 0 .. (hi - lo) per_decade, in FP64"""
    k = int(round((hi_exp - lo_exp) * per_decade))
    return 10.0 ** (lo_exp + np.arange(k + 1, dtype=np.float64) / per_decade)


ERROR_KINDS = ("vector", "angle", "magnitude")


def error_hist(c: Codec, xyz, edges, threads: int = 0):
    """(counts [3, nedges+1], excluded, stats [3, 3] = (sum, sum of squares, max)) of the codec's
    errors over xyz (see vco_error_hist)."""
    a = _f32xyz(xyz)
    edges = np.ascontiguousarray(edges, dtype=np.float64)
    ne = edges.shape[0]
    counts = np.zeros(3 * (ne + 1) + 1, dtype=np.uint64)
    stats = np.zeros(9, dtype=np.float64)
    lib().vco_error_hist(C.byref(c), a.ctypes.data, a.shape[0], edges.ctypes.data, ne, counts.ctypes.data,
                         stats.ctypes.data, threads)
    return counts[:-1].reshape(3, ne + 1), int(counts[-1]), stats.reshape(3, 3)


def rn32_fma(alpha: float, a: float, b: float) -> float:
    return float(lib().vco_rn32_fma(alpha, a, b))


def round_norm(x: float, y: float, z: float, prec: int, min_spacing: float = 0.0):
    tie = C.c_int(0)
    r = lib().vco_round_norm(x, y, z, prec, min_spacing, C.byref(tie))
    return float(r), bool(tie.value)


def exact_sign(values) -> int:
    arr = (C.c_double * len(values))(*values)
    return int(lib().vco_exact_sign(arr, len(values)))


def max_threads() -> int:
    return int(lib().vco_max_threads())


def fields(c: Codec, w):
    """Split codes into (E, M, n_phi, n_theta) following the layout (n_p split for FRAC)."""
    w = _u64(w)
    pt = c.p + c.t
    E = (w >> np.uint64(c.m + pt)) & np.uint64((1 << c.e) - 1)
    M = (w >> np.uint64(pt)) & np.uint64((1 << c.m) - 1)
    low = w & np.uint64((1 << pt) - 1)
    if c.mode == FRAC:
        T = np.uint64(frac_T(c))
        nph = low // T
        nth = low % T
    else:
        nth = low & np.uint64((1 << c.t) - 1)
        nph = low >> np.uint64(c.t)
    return E, M, nph, nth
