"""The public inline device API (include/vc_inline.hpp) used from a kernel of the caller's own:
its codes and decoded vectors equal the library's entry points bit for bit, and its dot product
of two codes matches the oracle's FP64 dot product of the decoded vectors."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_2003_02633_amd as vc
import tests.inline as U
from paper_2003_02633_amd import inputs

pytestmark = pytest.mark.gpu


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    vc.lib()
    U.lib()
    return torch


@pytest.mark.parametrize("n", [1, 1000, 65547])
def test_user_kernel_matches_library(torch_dev, n):
    import ctypes as C
    torch = torch_dev
    say(f"case: inline user kernel n={n}")
    c, co = vc.codec(), O.codec()
    x = inputs.gaussian_with_edges(max(n, 16), 3)[:n]
    tx = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    codes = torch.empty(n, dtype=torch.int64, device="cuda")
    back = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    dots = torch.empty(n, dtype=torch.float32, device="cuda")
    st = U.lib().user_roundtrip(C.byref(c), tx.data_ptr(), codes.data_ptr(), back.data_ptr(), dots.data_ptr(), n,
                                torch.cuda.current_stream().cuda_stream)
    assert st == 0
    ref_codes = vc.vc_encode(c, tx)
    ref_back = vc.vc_decode(c, ref_codes)
    torch.cuda.synchronize()
    assert torch.equal(codes, ref_codes)
    assert torch.equal(torch.nan_to_num(back, nan=7.0), torch.nan_to_num(ref_back, nan=7.0))
    w = codes.cpu().numpy().view(np.uint64)
    wj = np.concatenate([w[1:], w[-1:]])
    A, B = O.decode64(co, w), O.decode64(co, wj)
    ref = np.einsum("ij,ij->i", A, B)
    scale = np.linalg.norm(A, axis=1) * np.linalg.norm(B, axis=1)
    got = dots.cpu().numpy().astype(np.float64)
    ok = np.isfinite(ref)
    assert np.all(np.isnan(got[~ok]))
    assert np.all(np.abs(got[ok] - ref[ok]) <= 2e-6 * scale[ok]), np.max(np.abs(got[ok] - ref[ok]) / np.maximum(scale[ok], 1e-300))
