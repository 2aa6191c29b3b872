"""GPU parity of the compressed flux divergence (vc_flux_div_tp) against the oracle's Alg.
(fr_fdiv_comp) in FP64, with the dense operator expanded from the same float32 1D factors.

Two checks per output k:
- against the oracle: |gpu - oracle| <= 2e-6 sum_{j,c} |D[c ns + j][k]| ||X_jp|| + 1e-30.  The decode
  contract bounds each decoded component's error by 1e-6 of the vector's norm (not of the component),
  so the weight is the norm ||X_jp||; the single-precision accumulation of the 3 q terms adds under
  1e-6 of the sum of their magnitudes.
- against the GPU's own decode (vc_decode of the same codes, contracted in FP64): the difference is
  the kernel's single-precision sum alone, <= (3 q + 2) 2^-24 sum |D| |X^gpu_jpc| + 1e-30.  A wrong
  element, a stale prefetched group or a reused LDS slot gives an O(1) error here.
"""
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


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    vc.lib()
    return torch


def factors(q, h=(0.3, 0.5, 0.7)):
    return np.stack([inputs.fr_derivative_1d(q - 1, hc) for hc in h]).astype(np.float32)   # [3][q][q]


def dense(d32):
    q = d32.shape[-1]
    eye = np.eye(q, dtype=np.float64)
    d = d32.astype(np.float64)
    return np.concatenate([np.kron(eye, np.kron(eye, d[0])), np.kron(eye, np.kron(d[1], eye)),
                           np.kron(d[2], np.kron(eye, eye))]).astype(np.float32)


def _flux(ne, q, npq, seed):
    if npq == 5:
        return inputs.euler_flux_tgv(ne, q - 1, grid=(8, 8, 8) if ne <= 512 else (32, 32, 32))
    g = np.random.default_rng(seed)
    return (g.standard_normal((ne, q ** 3, npq, 3)) * 10.0 ** g.uniform(-2, 2, (ne, q ** 3, npq, 1))).astype(np.float32)


def _check(torch, c, co, q, npq, ne, seed, label):
    d32 = factors(q)
    F = _flux(ne, q, npq, seed)
    W = O.encode(co, F.reshape(-1, 3)).reshape(ne, q ** 3, npq)
    td = torch.from_numpy(d32).to("cuda")
    tW = torch.from_numpy(W.view(np.int64)).to("cuda")
    got = vc.vc_flux_div_tp(c, td, tW).cpu().numpy().astype(np.float64)
    Xg = vc.vc_decode(c, tW.reshape(-1)).cpu().numpy().astype(np.float64).reshape(ne, q ** 3, npq, 3)
    D = dense(d32)
    ref = O.flux_div(co, D, W)
    X = O.decode64(co, W.reshape(-1)).reshape(ne, q ** 3, npq, 3)
    ns = q ** 3
    D64 = D.astype(np.float64).reshape(3, ns, ns)
    absD = np.abs(D64)
    scale = np.einsum("cjk,ejp->ekp", absD, np.linalg.norm(X, axis=-1), optimize=True)
    ratio = (np.abs(got - ref) / (2e-6 * scale + 1e-30)).max()
    own = np.einsum("cjk,ejpc->ekp", D64, Xg, optimize=True)
    own_scale = np.einsum("cjk,ejpc->ekp", absD, np.abs(Xg), optimize=True)
    own_ratio = (np.abs(got - own) / ((3 * q + 2) * 2.0 ** -24 * own_scale + 1e-30)).max()
    say(f"{label} q={q} np={npq} ne={ne}: max err/tol {ratio:.3f} (oracle), {own_ratio:.3f} (own decode)")
    assert ratio <= 1.0
    assert own_ratio <= 1.0
    return F, got


@pytest.mark.parametrize("q,npq,ne", [(5, 5, 64), (5, 5, 63), (5, 5, 1), (5, 5, 3), (2, 1, 100), (3, 3, 37),
                                      (4, 5, 20), (6, 8, 9), (6, 1, 17), (5, 8, 11),
                                      # more element groups than resident workgroups: every
                                      # workgroup walks several groups (prefetch, LDS reuse), with
                                      # a ragged last group
                                      (5, 5, 12001), (3, 3, 40001)])
def test_flux_div_tp_matches_oracle(torch_dev, q, npq, ne):
    say(f"case: flux div q={q} np={npq} ne={ne}")
    _check(torch_dev, vc.codec(), O.codec(), q, npq, ne, q * 100 + npq, "plain")


@pytest.mark.parametrize("mode,kw", [("frac", {"P": 163840}), ("tanh", {"gamma": 0.5}), ("cos", {})])
def test_flux_div_tp_variants(torch_dev, mode, kw):
    say(f"case: flux div variant {mode}")
    _check(torch_dev, vc.codec(mode=mode, **kw), O.codec(mode=mode, **kw), 5, 5, 40, 7, mode)


def test_flux_div_tp_f32_baseline(torch_dev):
    """the same kernel on float32 fluxes against the FP64 dense divergence of those floats"""
    torch = torch_dev
    say("case: flux div f32 baseline")
    q, npq, ne = 5, 5, 50
    d32 = factors(q)
    F = inputs.euler_flux_tgv(ne, q - 1, grid=(8, 8, 8))
    got = vc.vcb_flux_div_tp_f32(torch.from_numpy(d32).to("cuda"), torch.from_numpy(F).to("cuda")).cpu().numpy()
    D = dense(d32).astype(np.float64).reshape(3, q ** 3, q ** 3)
    ref = np.einsum("cjk,ejpc->ekp", D, F.astype(np.float64))
    scale = np.einsum("cjk,ejpc->ekp", np.abs(D), np.abs(F.astype(np.float64)))
    assert (np.abs(got - ref) <= 1e-6 * scale + 1e-30).all()


def test_flux_div_tp_rejects(torch_dev):
    torch = torch_dev
    c = vc.codec()
    d = torch.zeros((3, 7, 7), dtype=torch.float32, device="cuda")
    W = torch.zeros((2, 343, 5), dtype=torch.int64, device="cuda")
    with pytest.raises(vc.VcError):
        vc.vc_flux_div_tp(c, d, W)
