"""ctypes loader of the CPU emulation build of the device codec (test infrastructure)."""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vc_hostemu.cpp")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libvcemu.so")
_lib = None


def build():
    os.makedirs(OUT_DIR, exist_ok=True)
    root = os.path.join(HERE, "..", "..")
    deps = [SRC, os.path.join(root, "paper_2003_02633_amd", "csrc", "vc_params.hpp")] + \
        [os.path.join(root, "include", f) for f in ("vc_device.hpp", "vc_coeffs.inc", "vc.h")]
    if os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(d) for d in deps):
        return LIB
    # a private temporary per process, then an atomic rename: parallel test workers may build at
    # the same time, and each loads a complete library
    tmp = f"{LIB}.tmp{os.getpid()}"
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        vp = C.c_void_p
        L.emu_encode.argtypes = [vp, vp, vp, C.c_size_t]
        L.emu_decode.argtypes = [vp, vp, vp, C.c_size_t]
        L.emu_dot_pair.argtypes = [vp, vp, vp, vp, C.c_size_t]
        L.emu_magnitude_checked.argtypes = [vp, vp, vp, C.c_size_t]
        L.emu_exact_norm.argtypes = [C.c_float, C.c_float, C.c_float, C.c_int, C.c_int,
                                     C.POINTER(C.c_uint32), C.POINTER(C.c_int)]
        _lib = L
    return _lib


def encode(codec, xyz):
    a = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32).reshape(-1, 3))
    out = np.empty(a.shape[0], dtype=np.uint64)
    st = lib().emu_encode(C.addressof(codec), a.ctypes.data, out.ctypes.data, a.shape[0])
    if st:
        raise RuntimeError(f"emu_encode status {st}")
    return out


def decode(codec, w):
    w = np.ascontiguousarray(np.asarray(w).astype(np.uint64).reshape(-1))
    out = np.empty((w.shape[0], 3), dtype=np.float32)
    st = lib().emu_decode(C.addressof(codec), w.ctypes.data, out.ctypes.data, w.shape[0])
    if st:
        raise RuntimeError(f"emu_decode status {st}")
    return out


def magnitude_checked(codec, w):
    """per-code magnitude as the norm kernels take it (NaN past a fractional split's P T levels)"""
    w = np.ascontiguousarray(np.asarray(w).astype(np.uint64).reshape(-1))
    out = np.empty(w.shape[0], dtype=np.float32)
    st = lib().emu_magnitude_checked(C.addressof(codec), w.ctypes.data, out.ctypes.data, w.shape[0])
    if st:
        raise RuntimeError(f"emu_magnitude_checked status {st}")
    return out


def dot_pair(codec, wa, wb):
    """per-pair decode(a) . decode(b) as the kernels form it (spherical form)"""
    wa = np.ascontiguousarray(np.asarray(wa).astype(np.uint64).reshape(-1))
    wb = np.ascontiguousarray(np.asarray(wb).astype(np.uint64).reshape(-1))
    out = np.empty(wa.shape[0], dtype=np.float32)
    st = lib().emu_dot_pair(C.addressof(codec), wa.ctypes.data, wb.ctypes.data, out.ctypes.data, wa.shape[0])
    if st:
        raise RuntimeError(f"emu_dot_pair status {st}")
    return out


def exact_norm(x, y, z, prec, keep_sub=False):
    j = C.c_uint32()
    g = C.c_int()
    lib().emu_exact_norm(x, y, z, prec, int(keep_sub), C.byref(j), C.byref(g))
    return j.value, g.value
