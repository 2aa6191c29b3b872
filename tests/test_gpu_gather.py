"""GPU parity of indexed decode / encode (vc_gather_decode, vc_scatter_encode).

gather: out[i] against the oracle's decode of codes[idx[i]], within 1e-6 r_hat per component (the
decode contract), out-of-range indices give NaN; it also equals vc_decode of the gathered codes
bit for bit.  scatter of a permutation: the codes equal vc_encode of the permuted inputs bit for
bit, and follow the encode contract against the oracle."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_2003_02633_amd as vc
from paper_2003_02633_amd import inputs
from tests.parity import classify, decode_err

pytestmark = pytest.mark.gpu


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    vc.lib()
    return torch


@pytest.mark.parametrize("n_src,n", [(100_003, 65_537), (17, 1000), (1, 5)])
def test_gather_decode(torch_dev, n_src, n):
    torch = torch_dev
    say(f"case: gather n_src={n_src} n={n}")
    c, co = vc.codec(), O.codec()
    w = O.encode(co, inputs.sphere_loguniform(n_src, 31))
    g = np.random.default_rng(32)
    idx = g.integers(0, n_src, n).astype(np.int32)
    idx[::97] = n_src + 5            # out of range
    tw = torch.from_numpy(w.view(np.int64)).to("cuda")
    ti = torch.from_numpy(idx).to("cuda")
    got = vc.vc_gather_decode(c, tw, ti).cpu().numpy()
    bad = idx >= n_src
    assert np.isnan(got[bad]).all()
    err, nan_ok = decode_err(co, w[idx[~bad]], got[~bad])
    say(f"gather decode max err/r = {err:.3e}")
    assert nan_ok and err <= 1e-6
    ref = vc.vc_decode(c, tw[torch.from_numpy(idx[~bad].astype(np.int64)).to("cuda")]).cpu().numpy()
    assert np.array_equal(ref, got[~bad])


def test_scatter_encode_permutation(torch_dev):
    torch = torch_dev
    say("case: scatter permutation")
    c, co = vc.codec(), O.codec()
    n = 50_001
    x = inputs.gaussian_with_edges(n - 11, 33)
    perm = np.random.default_rng(34).permutation(n).astype(np.int32)
    tx = torch.from_numpy(x).to("cuda")
    codes = torch.zeros(n, dtype=torch.int64, device="cuda")
    vc.vc_scatter_encode(c, tx, torch.from_numpy(perm).to("cuda"), codes)
    got = codes.cpu().numpy().view(np.uint64)
    # codes[perm[i]] = encode(x[i])  <=>  codes = encode(x[inv])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(n, dtype=np.int32)
    xs = x[inv]
    ref = vc.vc_encode(c, torch.from_numpy(xs).to("cuda")).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, ref)
    res = classify(co, xs, got)
    assert res["other"] == 0
