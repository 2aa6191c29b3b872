"""C-ABI checks that need no GPU: the library loads, exports every symbol the public headers
declare, and rejects invalid arguments synchronously (before any device work)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2003_02633_amd as vc
from tests.conftest import ROOT


def _declared_symbols():
    names = set()
    for h in ("vc.h", "vc_ext.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(vc[bx]?_[a-z0-9_]+)\s*\(", txt):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(vc.LIB_PATH):
        pytest.fail("libvc.so is not built (run python -m paper_2003_02633_amd.build)")
    return vc.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), f"missing export {n}"


def test_binding_covers_declared_symbols():
    declared = set(_declared_symbols())
    assert declared <= set(vc._SIGS), declared - set(vc._SIGS)


def test_status_strings_and_version(lib):
    assert lib.vc_status_string(0) == b"VC_SUCCESS"
    assert lib.vc_status_string(7) == b"VC_ERROR_OVERLAP"
    assert lib.vc_version().startswith(b"libvc")


def test_codec_init_layouts(lib):
    for name, idx in vc.LAYOUTS.items():
        c = vc.codec(name)
        assert c.layout == idx and c.struct_size == C.sizeof(vc.vc_codec)
    c = vc.vc_codec()
    assert lib.vc_codec_init(C.byref(c), b"0,9,22-16-17") == 3


def _fake(addr):
    return C.c_void_p(addr)


def test_validation_errors_without_device_work(lib):
    c = vc.codec()
    P = C.byref(c)
    n = 16
    # NULL data with n > 0
    assert lib.vc_encode(P, None, _fake(0x10000), n, None) == 1
    assert lib.vc_axpy(P, 1.0, None, _fake(0x10000), _fake(0x20000), n, None) == 1
    # misaligned codes
    assert lib.vc_decode(P, _fake(0x10004), _fake(0x20000), n, None) == 2
    assert lib.vc_axpy(P, 1.0, _fake(0x10001), _fake(0x20000), _fake(0x30000), n, None) == 2
    # partial overlap of output and input (exact aliasing is allowed)
    assert lib.vc_axpy(P, 1.0, _fake(0x10000), _fake(0x20000), _fake(0x10008), n, None) == 7
    assert lib.vc_encode(P, _fake(0x10000), _fake(0x10010), n, None) == 7
    # n == 0 is a no-op even with NULL pointers
    assert lib.vc_encode(P, None, None, 0, None) == 0
    assert lib.vc_axpy(P, 1.0, None, None, None, 0, None) == 0
    # bad codec
    bad = vc.codec()
    bad.struct_size = 3
    assert lib.vc_encode(C.byref(bad), _fake(0x10000), _fake(0x20000), n, None) == 1
    bad = vc.codec(mode="frac", P=1)
    assert lib.vc_encode(C.byref(bad), _fake(0x10000), _fake(0x20000), n, None) == 1
    bad = vc.codec(mode="tanh", gamma=5.0)
    assert lib.vc_encode(C.byref(bad), _fake(0x10000), _fake(0x20000), n, None) == 3
    # companding with the single-precision encoder is accepted; validation alone (n == 0) builds
    # none of its boundary tables, so it needs no device
    for mode in ("tanh", "cos"):
        ok = vc.codec(mode=mode, precision="f32")
        assert lib.vc_encode(C.byref(ok), None, None, 0, None) == 0
        assert lib.vc_axpy(C.byref(ok), 1.0, None, None, None, 0, None) == 0
    bad = vc.codec("0,8,23-16-17", mode="tanh")
    assert lib.vc_encode(C.byref(bad), _fake(0x10000), _fake(0x20000), n, None) == 3
    bad = vc.codec()
    bad.mag_round = 2                                  # no such magnitude rounding
    assert lib.vc_encode(C.byref(bad), _fake(0x10000), _fake(0x20000), n, None) == 3
    # the truncating magnitude is accepted with every layout, mode and encoder precision
    # (validation only: n == 0)
    for layout in ("0,7,22-17-18", "0,7,23-17-17", "0,8,23-16-17", "1,8,23-16-16"):
        for prec in ("f64", "f32"):
            ok = vc.codec(layout, precision=prec, mag_round="trunc")
            assert lib.vc_encode(C.byref(ok), None, None, 0, None) == 0
    ok = vc.codec(mode="frac", P=163840, mag_round="trunc")
    assert lib.vc_axpy(C.byref(ok), 1.0, None, None, None, 0, None) == 0
    # reductions need an output
    assert lib.vc_dot(P, _fake(0x10000), _fake(0x20000), n, None, None) == 1
    assert lib.vc_dot_noalloc(P, _fake(0x10000), _fake(0x20000), n, None, None) == 1
    assert lib.vc_dot_noalloc(P, _fake(0x10000), None, n, _fake(0x30000), None) == 1
    assert lib.vc_dot_noalloc(P, _fake(0x10004), _fake(0x20000), n, _fake(0x30000), None) == 2
    assert lib.vc_dot_noalloc(P, _fake(0x10000), _fake(0x20000), n, _fake(0x30002), None) == 2
    # baselines
    assert lib.vcb_copy(_fake(0x10000), _fake(0x20008), 64, None) == 2
    assert lib.vcb_axpy_f32(1.0, None, None, None, 0, None) == 0


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(vc, "_lib", None)
    monkeypatch.setattr(vc, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        vc.lib()


def _seg(op, n, a, b, out, alpha=1.0):
    return vc.vc_segment(vc.OPS[op], alpha, n, a, b, out)


def _create(lib, segs):
    arr = (vc.vc_segment * len(segs))(*segs)
    plan = C.c_void_p()
    st = lib.vc_batch_plan_create(C.byref(plan), C.byref(vc.codec()), arr, len(segs), None)
    assert not plan.value
    return st


def test_batch_plan_validation_without_device_work(lib):
    K = 1 << 20
    # unknown op
    assert _create(lib, [vc.vc_segment(9, 1.0, 4, 0x10000, 0x20000, 0x30000)]) == 1
    # NULL operand / output
    assert _create(lib, [_seg("axpy", 4, None, 0x20000, 0x30000)]) == 1
    assert _create(lib, [_seg("dot", 0, None, None, None)]) == 1
    # misaligned
    assert _create(lib, [_seg("norm2", 4, 0x10004, None, 0x30000)]) == 2
    assert _create(lib, [_seg("encode", 4, 0x10002, None, 0x30000)]) == 2
    # in-segment partial overlap
    assert _create(lib, [_seg("axpy", 16, 0x10000, 0x20000 + K, 0x10008)]) == 7
    # one segment writes what another reads, or two write the same memory
    assert _create(lib, [_seg("axpy", 16, 0x10000, 0x20000, 0x30000),
                         _seg("norm2", 16, 0x30000 + 64, None, 0x40000)]) == 7
    assert _create(lib, [_seg("encode", 16, 0x10000, None, 0x30000),
                         _seg("dot", 16, 0x50000, 0x60000, 0x30000 + 120)]) == 7
    # nseg bounds and plan pointer
    arr = (vc.vc_segment * 1)(_seg("norm2", 4, 0x10000, None, 0x30000))
    plan = C.c_void_p()
    assert lib.vc_batch_plan_create(C.byref(plan), C.byref(vc.codec()), arr, -1, None) == 1
    assert lib.vc_batch_plan_create(None, C.byref(vc.codec()), arr, 1, None) == 1
    assert lib.vc_batch_plan_run(None, None) == 1
    assert lib.vc_batch_plan_destroy(None) == 0


def test_apply_validation_without_device_work(lib):
    P = C.byref(vc.codec())
    f = _fake
    assert lib.vc_fused_apply(P, f(0x10000), 0, 4, f(0x20000), f(0x30000), 8, None) == 1
    assert lib.vc_fused_apply(P, f(0x10000), 257, 4, f(0x20000), f(0x30000), 8, None) == 1
    assert lib.vc_fused_apply(P, f(0x10000), 16, 0, f(0x20000), f(0x30000), 8, None) == 1
    # operator too large for LDS staging: 4*ceil(200/4)*160 floats
    assert lib.vc_fused_apply(P, f(0x10000), 160, 200, f(0x20000), f(0x30000), 8, None) == 1
    assert lib.vc_fused_apply(P, f(0x10000), 150, 125, None, f(0x30000), 8, None) == 1
    assert lib.vc_fused_apply(P, f(0x10000), 150, 125, f(0x20004), f(0x30000), 8, None) == 2
    assert lib.vc_fused_apply(P, None, 150, 125, None, None, 0, None) == 0
    # companding is built into the apply for the default layout only
    bad = vc.codec(layout="0,7,23-17-17", mode="tanh")
    assert lib.vc_fused_apply(C.byref(bad), f(0x10000), 16, 4, f(0x20000), f(0x30000), 8, None) == 3


def test_tuning_cache_parsing(lib, tmp_path):
    saved = {p: vc.get_stream_config(p) for p in ("f64", "f32")}
    saved_batch = vc.get_batch_config()
    try:
        f = tmp_path / "tune.txt"
        f.write_text("# comment\naxpy f64 block=256 vpt=2 nt=0\n")
        assert lib.vcx_load_tuning(str(f).encode()) == 0
        assert vc.get_stream_config("f64") == (256, 2, 0)
        assert vc.get_stream_config("f32") == saved["f32"]
        f.write_text("axpy block=128 vpt=4 nt=1\n")
        assert lib.vcx_load_tuning(str(f).encode()) == 0
        assert vc.get_stream_config("f64") == vc.get_stream_config("f32") == (128, 4, 1)
        f.write_text("axpy f16 block=128 vpt=4 nt=1\n")
        assert lib.vcx_load_tuning(str(f).encode()) == 1
        assert lib.vcx_set_stream_config(-1, 100, 2, 1) == 3
        assert lib.vcx_set_stream_config(-1, 256, 3, 1) == 3
        assert lib.vcx_set_stream_config(-1, 128, 8, 1) == 3       # 8 per thread needs >= 256 threads
        assert lib.vcx_set_stream_config(0, 512, 8, 1) == 0       # VC_PREC_F64
        assert vc.get_stream_config("f64") == (512, 8, 1)
        assert lib.vcx_load_tuning(str(tmp_path / "missing").encode()) == 1
        # the batch tile shape
        f.write_text("batch ua=1 ud=4 un=8\n")
        assert lib.vcx_load_tuning(str(f).encode()) == 0
        assert vc.get_batch_config() == (1, 4, 8)
        f.write_text("batch ua=3 ud=4 un=8\n")
        assert lib.vcx_load_tuning(str(f).encode()) == 3
        assert vc.get_batch_config() == (1, 4, 8)
        assert lib.vcx_set_batch_config(2, 3, 4) == 3 and lib.vcx_set_batch_config(2, 2, 32) == 3
    finally:
        vc.set_batch_config(*saved_batch)
        for p, (b, v, t) in saved.items():
            vc.set_stream_config(b, v, t, p)
    assert vc.get_stream_config("f64") == saved["f64"]


def test_inline_params(lib):
    """the constants block of the inline device API: size checked, codec validated"""
    size = lib.vcx_inline_params_size()
    assert 64 <= size <= 4096
    buf = C.create_string_buffer(size)
    assert lib.vcx_inline_params(C.byref(vc.codec()), buf, size) == 0
    assert lib.vcx_inline_params(C.byref(vc.codec()), buf, size - 8) == 1
    assert lib.vcx_inline_params(C.byref(vc.codec()), None, size) == 1
    bad = vc.codec()
    bad.mode = 9                                        # no such mode
    assert lib.vcx_inline_params(C.byref(bad), buf, size) == 3
    assert lib.vcx_inline_params(C.byref(vc.codec()), buf, size) == 0
    # the first fields are n_theta_max and n_phi_max of the default layout
    nt, npm = np.frombuffer(buf.raw[:8], dtype=np.uint32)
    assert (nt, npm) == ((1 << 18) - 1, (1 << 17) - 1)


def test_tanh_fits_cached_per_gamma(lib):
    """the tanh map's polynomial fits (milliseconds each) are cached per gamma: interleaved codecs
    of several gammas get the same constants as when first resolved, and resolving is cheap"""
    import time
    size = lib.vcx_inline_params_size()

    def params(g):
        buf = C.create_string_buffer(size)
        assert lib.vcx_inline_params(C.byref(vc.codec(mode="tanh", gamma=g)), buf, size) == 0
        return buf.raw
    gammas = [0.5, 1.0, 0.25, 0.8125]
    first = {g: params(g) for g in gammas}
    assert len(set(first.values())) == len(gammas)
    for _ in range(3):
        for g in reversed(gammas):
            assert params(g) == first[g]
    t0 = time.perf_counter()
    for _ in range(2000):
        params(1.0)
    assert time.perf_counter() - t0 < 1.0


def test_error_hist_validation_without_device_work(lib):
    P = C.byref(vc.codec())
    f = _fake
    assert lib.vcx_error_hist(P, f(0x10000), 8, f(0x20000), 0, f(0x30000), f(0x40000), None) == 1
    assert lib.vcx_error_hist(P, f(0x10000), 8, f(0x20000), 257, f(0x30000), f(0x40000), None) == 1
    assert lib.vcx_error_hist(P, None, 8, f(0x20000), 10, f(0x30000), f(0x40000), None) == 1
    assert lib.vcx_error_hist(P, f(0x10000), 8, f(0x20004), 10, f(0x30000), f(0x40000), None) == 2
    assert lib.vcx_error_hist(P, f(0x10000), 8, f(0x20000), 10, f(0x30004), f(0x40000), None) == 2


def test_flux_div_validation_without_device_work(lib):
    P = C.byref(vc.codec())
    f = _fake
    assert lib.vc_flux_div_tp(P, f(0x10000), 7, 5, f(0x20000), f(0x80000000), 4, None) == 1
    assert lib.vc_flux_div_tp(P, f(0x10000), 5, 0, f(0x20000), f(0x80000000), 4, None) == 1
    assert lib.vc_flux_div_tp(P, f(0x10000), 5, 5, f(0x20004), f(0x80000000), 4, None) == 2
    assert lib.vc_flux_div_tp(P, f(0x10000), 5, 5, f(0x20000), f(0x20000 + 64), 4, None) == 7
    assert lib.vc_flux_div_tp(P, None, 5, 5, f(0x20000), f(0x80000000), 4, None) == 1
    assert lib.vc_flux_div_tp(P, None, 5, 5, None, None, 0, None) == 0
    assert lib.vcb_flux_div_tp_f32(f(0x10000), 5, 5, f(0x20002), f(0x80000000), 4, None) == 2


def test_gather_scatter_validation_without_device_work(lib):
    P = C.byref(vc.codec())
    f = _fake
    assert lib.vc_gather_decode(P, f(0x10000), 16, f(0x20000), 8, None, None) == 1
    assert lib.vc_gather_decode(P, f(0x10004), 16, f(0x20000), 8, f(0x80000000), None) == 2
    assert lib.vc_gather_decode(P, f(0x10000), 16, f(0x20000), 8, f(0x10000 + 8), None) == 7
    assert lib.vc_gather_decode(P, None, 0, None, 0, None, None) == 0
    assert lib.vc_scatter_encode(P, f(0x10000), f(0x20002), 8, f(0x30000), 8, None) == 2
    assert lib.vc_scatter_encode(P, f(0x10000), f(0x20000), 8, f(0x10000 + 16), 8, None) == 7
    assert lib.vcb_gather_f32(f(0x10000), 16, None, 8, f(0x30000), None) == 1


def test_vc_log_lines_without_device_work():
    """VC_LOG=1 makes each core entry point report its codec, size, launch configuration and
    status on stderr; unset, nothing is written (validation-only calls, no GPU needed)"""
    import subprocess
    import sys
    code = ("import ctypes as C, paper_2003_02633_amd as vc\n"
            "L = vc.lib(); c = vc.codec(mag_round='trunc')\n"
            "L.vc_encode(C.byref(c), None, None, 0, None)\n"
            "L.vc_axpy(C.byref(vc.codec()), C.c_float(1.0), None, C.c_void_p(0x1000), C.c_void_p(0x2000), 16, None)\n"
            "L.vc_norm2(C.byref(c), None, 0, None, None)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for val, expect in (("1", True), ("0", False), (None, False)):
        env = {k: v for k, v in os.environ.items() if k != "VC_LOG"}
        if val is not None:
            env["VC_LOG"] = val
        r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 0, r.stderr
        lines = [l for l in r.stderr.splitlines() if l.startswith("[vc] ")]
        if not expect:
            assert lines == []
            continue
        assert len(lines) == 3, r.stderr
        assert lines[0] == "[vc] vc_encode n=0 layout=0 mode=0 mag_round=1 precision=0 -> VC_SUCCESS"
        assert lines[1].startswith("[vc] vc_axpy n=16 layout=0 mode=0 mag_round=0 precision=0 block=")
        assert lines[1].endswith("-> VC_ERROR_INVALID_VALUE")
        assert lines[2].startswith("[vc] vc_norm2 n=0 ") and lines[2].endswith("-> VC_ERROR_INVALID_VALUE")   # needs d_out


def test_env_tuning_applied_once_under_concurrent_first_calls(tmp_path):
    """$VC_TUNE_CACHE is applied exactly once, by whichever thread calls vc_axpy first, while
    other threads change and read the configuration (validation-only calls, no GPU needed)"""
    import subprocess
    import sys
    f = tmp_path / "tune.txt"
    f.write_text("axpy f64 block=256 vpt=8 nt=0\n")
    code = (
        "import ctypes as C, threading, paper_2003_02633_amd as vc\n"
        "L = vc.lib(); c = vc.codec(); seen = set(); errs = []; d0 = vc.get_stream_config('f64')\n"
        "def axpy():\n"
        "    for _ in range(200):\n"
        "        if L.vc_axpy(C.byref(c), C.c_float(1.0), None, None, None, 0, None) != 0: errs.append('axpy')\n"
        "def reader():\n"
        "    for _ in range(200): seen.add(vc.get_stream_config('f64'))\n"
        "ts = [threading.Thread(target=axpy) for _ in range(4)] + [threading.Thread(target=reader) for _ in range(4)]\n"
        "[t.start() for t in ts]; [t.join() for t in ts]\n"
        "assert not errs, errs\n"
        "assert vc.get_stream_config('f64') == (256, 8, 0), vc.get_stream_config('f64')\n"
        "assert seen <= {d0, (256, 8, 0)}, seen\n"
        "vc.set_stream_config(512, 4, 1, 'f64')\n"
        "L.vc_axpy(C.byref(c), C.c_float(1.0), None, None, None, 0, None)\n"
        "assert vc.get_stream_config('f64') == (512, 4, 1)   # not re-applied\n"
        "print('ok')\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, VC_TUNE_CACHE=str(f))
    env.pop("VC_LOG", None)
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-2000:]
