"""The allocation-free dot (vc_dot_noalloc) against vc_dot and the oracle, through the C ABI.

Two calls in a row on one device, the second with a smaller input, so the second reads partials
the first call left in the shared device array only where it wrote them itself: both calls must
equal vc_dot on the same operands bit for bit (same kernels, same fixed reduction order) and the
oracle's FP64 dot within 4e-6 sum |a_hat| |b_hat| (the dot tolerance of the parity tests).
"""
import ctypes as C
import sys

import numpy as np
import pytest

import oracle as O
import paper_2003_02633_amd as vc
from paper_2003_02633_amd import inputs

pytestmark = pytest.mark.gpu


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


def test_dot_noalloc_matches_dot_and_oracle():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    c, co = vc.codec(), O.codec()
    lib = vc.lib()
    for n, seed in ((3_000_017, 41), (65_547, 43), (0, 0)):
        say(f"case: vc_dot_noalloc n={n}")
        wa = O.encode(co, inputs.gaussian_with_edges(max(n - 11, 0), seed)[:n]) if n else np.zeros(0, np.uint64)
        wb = O.encode(co, inputs.gaussian_with_edges(max(n - 11, 0), seed + 1)[:n]) if n else np.zeros(0, np.uint64)
        ta = torch.from_numpy(wa.view(np.int64)).to("cuda")
        tb = torch.from_numpy(wb.view(np.int64)).to("cuda")
        out_na = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        out_ref = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        st = lib.vc_dot_noalloc(C.byref(c), C.c_void_p(ta.data_ptr()), C.c_void_p(tb.data_ptr()), n,
                                C.c_void_p(out_na.data_ptr()), stream)
        assert st == vc.VC_SUCCESS, lib.vc_status_string(st)
        vc.vc_dot(c, ta, tb, out=out_ref)
        torch.cuda.synchronize()
        got, ref = float(out_na.cpu()[0]), float(out_ref.cpu()[0])
        exact = O.dot(co, wa, wb) if n else 0.0
        if n:
            A, B = O.decode64(co, wa), O.decode64(co, wb)
            scale = float((np.linalg.norm(A, axis=1) * np.linalg.norm(B, axis=1)).sum())
        else:
            scale = 0.0
        say(f"n={n}: noalloc {got:.9e} vc_dot {ref:.9e} oracle {exact:.9e}")
        assert np.float32(got).tobytes() == np.float32(ref).tobytes()
        assert abs(got - exact) <= 4e-6 * scale
