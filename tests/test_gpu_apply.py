"""GPU parity of the fused decode + MFMA apply (vc_fused_apply) against the FP64 oracle.

Tolerance per output entry: |out_gpu - out_oracle| <= 1e-5 * sum_j |M_ij| |u_j|, where u_j are
the exactly decoded vectors (single-precision decode error ~3e-7 |u| plus FP32 accumulation).
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
    assert torch.cuda.is_available()
    vc.lib()
    return torch


@pytest.fixture
def apply_mode(torch_dev):
    """sets the apply's matrix cores for one test ('auto': split-bf16 where it fits, 'fp32')"""
    yield vc.set_apply_mode
    vc.set_apply_mode("auto")


def _run(torch, c, M, U, offset=0):
    """offset > 0 places the output `offset` floats into a buffer (a 4-byte aligned output)"""
    tM = torch.from_numpy(np.ascontiguousarray(M)).to("cuda")
    tU = torch.from_numpy(np.ascontiguousarray(U).view(np.int64)).to("cuda")
    out = None
    if offset:
        n = U.shape[0] * M.shape[0] * 3
        out = torch.full((n + offset,), float("nan"), dtype=torch.float32, device="cuda")[offset:]
        out = out.view(U.shape[0], M.shape[0], 3)
    out = vc.vc_fused_apply(c, tM, tU, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _check(co, M, U, got, label):
    ref = O.apply(co, M, U)
    X = O.decode64(co, U.reshape(-1)).reshape(U.shape[0], U.shape[1], 3)
    scale = np.einsum("ij,ej->ei", np.abs(M.astype(np.float64)), np.linalg.norm(X, axis=2))
    err = np.abs(got.astype(np.float64) - ref).max(axis=2)
    ratio = (err / np.maximum(1e-5 * scale, 1e-300)).max()
    say(f"{label}: max err / tol = {ratio:.3f}")
    assert ratio <= 1.0


@pytest.mark.parametrize("rows,cols,n_elem", [(150, 125, 1000), (150, 125, 17), (1, 1, 5), (16, 4, 33),
                                              (32, 8, 64), (47, 125, 100), (256, 20, 40), (150, 125, 1),
                                              # 2,054 tiles on 256 workgroups of 8 waves: one full round
                                              # and 6 tiles spread over the workgroups' first waves
                                              (16, 4, 16 * 2054 - 13),
                                              # M (76 KB) and 8 waves' whole-element staging (98 KB)
                                              # exceed the LDS: the 16-row block staging runs
                                              (256, 68, 41),
                                              # on 256 workgroups (2,048 waves): 2,048 tiles, the last
                                              # one partial, all in the full round
                                              (32, 8, 16 * 2048 - 5),
                                              # one full round and 100 tiles left over, cut into 5
                                              # units of 2 row blocks each
                                              (150, 8, 16 * 2148 - 3),
                                              # 500 tiles left over: 5 units each would give some
                                              # waves two, so they stay whole
                                              (150, 8, 16 * 2548 - 7)])
@pytest.mark.parametrize("mode", ["auto", "fp32"])
def test_apply_shapes(torch_dev, apply_mode, rows, cols, n_elem, mode):
    apply_mode(mode)
    say(f"case: apply rows={rows} cols={cols} n_elem={n_elem} cores={mode}")
    c, co = vc.codec(), O.codec()
    M = inputs.uniform_matrix(rows, cols, 2)
    U = O.encode(co, inputs.gaussian(n_elem * cols, 7)).reshape(n_elem, cols)
    _check(co, M, U, _run(torch_dev, c, M, U), f"apply {rows}x{cols} E={n_elem} {mode}")


@pytest.mark.parametrize("offset", [1, 2, 4])
def test_apply_output_alignment(torch_dev, offset):
    """Outputs 4, 8 and 16 bytes into a buffer: element staging needs 16-byte alignment, the
    block staging's pair stores 8; the others take the single-float stores."""
    say(f"case: apply 150x125 E=70 output offset {offset} floats")
    c, co = vc.codec(), O.codec()
    M = inputs.uniform_matrix(150, 125, 2)
    U = O.encode(co, inputs.gaussian(70 * 125, 9)).reshape(70, 125)
    _check(co, M, U, _run(torch_dev, c, M, U, offset), f"apply offset {offset}")


@pytest.mark.parametrize("mode", ["auto", "fp32"])
def test_apply_tgv_field(torch_dev, apply_mode, mode):
    """The fused-apply workload: TGV velocity at p = 4 solution points (sampled elements)."""
    apply_mode(mode)
    say(f"case: apply tgv 4000 elements cores={mode}")
    c, co = vc.codec(), O.codec()
    M = inputs.uniform_matrix(150, 125, 2)
    vel = inputs.tgv_elements(4000, 4, seed=0)
    U = O.encode(co, vel.reshape(-1, 3)).reshape(4000, 125)
    _check(co, M, U, _run(torch_dev, c, M, U), "apply tgv")


def test_apply_rejects_oversize(torch_dev):
    c = vc.codec()
    import torch
    M = torch.zeros((256, 256), dtype=torch.float32, device="cuda")
    U = torch.zeros((4, 256), dtype=torch.int64, device="cuda")
    with pytest.raises(vc.VcError):
        vc.vc_fused_apply(c, M, U)


def test_apply_split_bf16_dynamic_range(torch_dev, apply_mode):
    """Operator entries and vector magnitudes over many binades (the three bf16 parts of each
    operand carry its 24 significant bits at any exponent): the bf16 cores still meet the FP32
    bound, and agree with the FP32 cores to the same bound."""
    say("case: apply 150x125 E=300 wide dynamic range, both cores")
    c, co = vc.codec(), O.codec()
    rng = np.random.default_rng(11)
    M = (inputs.uniform_matrix(150, 125, 2) * np.exp2(rng.integers(-30, 30, (150, 125)))).astype(np.float32)
    X = inputs.sphere_loguniform(300 * 125, 12)
    U = O.encode(co, X).reshape(300, 125)
    apply_mode("auto")
    got_bf = _run(torch_dev, c, M, U)
    _check(co, M, U, got_bf, "apply wide range, bf16 cores")
    apply_mode("fp32")
    got_32 = _run(torch_dev, c, M, U)
    _check(co, M, U, got_32, "apply wide range, FP32 cores")


def test_apply_mode_validation(torch_dev):
    with pytest.raises(vc.VcError):
        vc.lib()  # (loads the library)
        vc._check(vc.lib().vcx_set_apply_mode(7), "vcx_set_apply_mode")
    assert vc.get_apply_mode() == "auto"


@pytest.mark.parametrize("mode", ["auto", "fp32"])
@pytest.mark.parametrize("kw", [{"mode": "tanh", "gamma": 0.5}, {"mode": "cos"}, {"mode": "frac", "P": 163840}],
                         ids=["tanh", "cos", "frac"])
def test_apply_codec_variants(torch_dev, apply_mode, kw, mode):
    """The apply decodes with the codec's own inverse maps (companding, fractional split)."""
    apply_mode(mode)
    say(f"case: apply 150x125 E=200 codec {kw} cores={mode}")
    c, co = vc.codec(**kw), O.codec(**kw)
    M = inputs.uniform_matrix(150, 125, 2)
    U = O.encode(co, inputs.gaussian(200 * 125, 13)).reshape(200, 125)
    _check(co, M, U, _run(torch_dev, c, M, U), f"apply {kw} {mode}")
