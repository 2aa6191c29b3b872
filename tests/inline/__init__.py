"""Build and load a user kernel written against include/vc_inline.hpp (test infrastructure)."""
import ctypes as C
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "user_kernels.hip")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libvcuser.so")
_lib = None


def build():
    """hipcc the user kernel with the library's flags, linked against libvc.so (found next to
    this file's tree through a relative run path)"""
    from paper_2003_02633_amd import build as B
    os.makedirs(OUT_DIR, exist_ok=True)
    libdir = os.path.join(ROOT, "paper_2003_02633_amd")
    cmd = [B.HIPCC, *B.COMMON, "-shared", SRC, "-L", libdir, "-lvc",
           "-Wl,-rpath,$ORIGIN/../../../paper_2003_02633_amd", "-o", f"{LIB}.tmp{os.getpid()}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for the inline user kernel:\n" + r.stderr[-3000:])
    os.replace(f"{LIB}.tmp{os.getpid()}", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB)
        vp = C.c_void_p
        L.user_roundtrip.argtypes = [vp, vp, vp, vp, vp, C.c_size_t, vp]
        L.user_roundtrip.restype = C.c_int
        _lib = L
    return _lib
