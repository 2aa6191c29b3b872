"""GPU error statistics (vcx_error_hist, FP64 on the GPU) against the oracle's histograms.

Contract: the GPU encodes with the library's encoder, so its codes may differ from the oracle's
by one level inside the one-ulp window (counted here as n_diff).  Each such vector can move one
count per histogram, so per histogram sum |h_gpu - h_oracle| <= 2 n_diff; the sums differ by at
most n_diff times the largest per-vector error change (< 4e-5) plus 1e-9 relative (the two FP64
decodes differ in their sincospi/atan2 implementations by ~1e-16 of |x|); the vectors
left out (zero, non-finite, flushed, saturated) agree exactly.
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


def _compare(torch, layout, mode, kw, xyz, label):
    okw = {k: v for k, v in kw.items() if k != "precision"}
    c, co = vc.codec(layout, mode=mode, **kw), O.codec(layout, mode=mode, **okw)
    edges = O.log_edges()
    tx = torch.from_numpy(np.ascontiguousarray(xyz)).to("cuda")
    te = torch.from_numpy(edges).to("cuda")
    hg, exg, sg = vc.error_hist(c, tx, te)
    hg, sg = hg.numpy().astype(np.int64), sg.numpy()
    ho, exo, so = O.error_hist(co, xyz, edges)
    ho = ho.astype(np.int64)
    wg = vc.vc_encode(c, tx).cpu().numpy().view(np.uint64)
    wo = O.encode(co, xyz)
    n_diff = int((wg != wo).sum())
    n = int(ho[0].sum())
    say(f"{label}: n={n} excluded={exo} n_diff={n_diff} mean vec err gpu {sg[0, 0] / max(n, 1):.6e} "
        f"oracle {so[0, 0] / max(n, 1):.6e}; hist L1 {[int(np.abs(hg[k] - ho[k]).sum()) for k in range(3)]}")
    assert exg == exo
    for k in range(3):
        assert int(hg[k].sum()) == n
        assert int(np.abs(hg[k] - ho[k]).sum()) <= 2 * n_diff
        # the two FP64 decodes use different sincospi/atan2 implementations: x_hat differs by
        # ~1e-16 |x|, so each error value by ~1e-11 relative; 1e-9 relative covers it
        assert abs(sg[k, 0] - so[k, 0]) <= n_diff * 4e-5 + 1e-9 * abs(so[k, 0])
        assert abs(sg[k, 2] - so[k, 2]) <= (4e-5 if n_diff else 1e-9 * so[k, 2] + 1e-300)
    return sg / max(n, 1)


CODECS = [("0,7,22-17-18", "plain", {"precision": "f64"}),
          ("0,7,22-17-18", "plain", {"precision": "f32"}),
          ("0,7,22-17-18", "frac", {"P": 163840, "precision": "f64"}),
          ("0,7,22-17-18", "tanh", {"gamma": 0.5, "precision": "f64"}),
          ("0,7,22-17-18", "cos", {"precision": "f64"}),
          ("0,8,23-16-17", "plain", {"precision": "f64"}),
          ("1,8,23-16-16", "plain", {"precision": "f64"}),
          ("0,7,22-17-18", "plain", {"precision": "f64", "mag_round": "trunc"})]


@pytest.mark.parametrize("layout,mode,kw", CODECS)
def test_error_hist_matches_oracle(torch_dev, layout, mode, kw):
    say(f"case: error hist {layout} {mode} {kw}")
    xs = {"gauss+edges": inputs.gaussian_with_edges((1 << 17) - 11, 71),
          "sphere_log": inputs.sphere_loguniform(100_003, 72),
          "vmf_k1000_z": inputs.vmf(1 << 16, 1000.0, seed=73)}
    for name, xyz in xs.items():
        _compare(torch_dev, layout, mode, kw, xyz, f"{layout} {mode} {name}")


def test_error_hist_anisotropy(torch_dev):
    """§2.2: the theta step shrinks on the sphere by sin(phi), so directions clustered at the z pole
    (vMF, kappa = 1000 about +z) have smaller errors than ones clustered on the equator."""
    say("case: error hist anisotropy")
    pole = _compare(torch_dev, "0,7,22-17-18", "plain", {}, inputs.vmf(1 << 16, 1000.0, seed=74), "pole")
    equ = _compare(torch_dev, "0,7,22-17-18", "plain", {},
                   inputs.vmf(1 << 16, 1000.0, mean=(1.0, 0.0, 0.0), seed=75), "equator")
    assert pole[0, 0] < 0.8 * equ[0, 0]


def test_error_hist_empty_and_small(torch_dev):
    torch = torch_dev
    c = vc.codec()
    te = torch.from_numpy(O.log_edges()).to("cuda")
    h, ex, s = vc.error_hist(c, torch.empty((0, 3), dtype=torch.float32, device="cuda"), te)
    assert int(h.sum()) == 0 and ex == 0 and float(s.abs().sum()) == 0.0
    _compare(torch, "0,7,22-17-18", "plain", {}, inputs.gaussian(257, 76), "n=257")
