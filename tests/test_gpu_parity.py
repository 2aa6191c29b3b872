"""GPU parity: the HIP kernels (through the C ABI) against the CPU oracle.

Contract:
  * encode: codes equal the oracle's bit for bit, except an angle level may differ by one
    where the exact level coordinate is within one single-precision ulp of the angle of the
    boundary (counted); magnitude fields exact.
  * decode: |x_gpu - x_oracle| <= 1e-6 r_hat per component; zero/reserved codes exact/NaN.
  * axpy (layered): the fused kernel's codes equal the GPU encode of its own pre-encode
    single-precision sum (dumped by the verification variant of the same kernel); those codes
    follow the encode rule against the oracle; decoding them recovers the FP64 sum of the
    exactly decoded operands within the codec error bound.
  * dot / norm2: within 4e-6 of sum |a||b| (resp. sum |a|^2) of the FP64 oracle.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import paper_2003_02633_amd as vc
from paper_2003_02633_amd import inputs
from tests.parity import classify, decode_abs_err, decode_err, describe_bad, random_codes

pytestmark = pytest.mark.gpu

ALPHA = float(np.float32(0.7))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    vc.lib()
    return torch


def up(torch, arr):
    arr = np.ascontiguousarray(arr)
    if arr.dtype == np.uint64:
        arr = arr.view(np.int64)
    return torch.from_numpy(arr).to("cuda")


def down(t, u64=False):
    a = t.cpu().numpy()
    return a.view(np.uint64) if u64 else a


def gpu_encode(torch, c, xyz):
    out = vc.vc_encode(c, up(torch, xyz.astype(np.float32)))
    torch.cuda.synchronize()
    return down(out, True)


def _summary(res):
    return {k: v for k, v in res.items() if not isinstance(v, np.ndarray)}


# ----------------------------------------------------------------------------- encode
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_encode_config1(torch_dev, prec):
    """N = 65,536 N(0,1) vectors plus the axis/zero/extreme edge cases."""
    say(f"case: encode config1 N=65547 {prec}")
    c, co = vc.codec(precision=prec), O.codec()
    xyz = inputs.gaussian_with_edges(65536, 0)
    dev = gpu_encode(torch_dev, c, xyz)
    res = classify(co, xyz, dev)
    say(f"encode config1: {_summary(res)}")
    assert res["other"] == 0, describe_bad(co, xyz, dev, res)
    # the 11 edge cases are exact (axis ties, zero, flush, saturation)
    assert np.array_equal(dev[-11:], res["ref"][-11:])


VARIANTS = []
for _prec in ("f64", "f32"):
    VARIANTS += [(lay, "plain", {"precision": _prec}) for lay in
                 ("0,7,22-17-18", "0,7,23-17-17", "0,8,23-16-17", "1,8,23-16-16")]
    VARIANTS += [("0,7,22-17-18", "frac", {"P": P, "precision": _prec})
                 for P in (1 << 16, 1 << 17, 163840, 1 << 18)]
# companding with either encoder (the single-precision one settles its levels with the
# library's boundary tables)
VARIANTS += [("0,7,22-17-18", "tanh", {"gamma": 0.5, "precision": p}) for p in ("f64", "f32")]
VARIANTS += [("0,7,22-17-18", "tanh", {"gamma": 1.0, "precision": p}) for p in ("f64", "f32")]
VARIANTS += [("0,7,22-17-18", "cos", {"precision": p}) for p in ("f64", "f32")]
# companding of one angle only (the kernels' run-time mask path; both angles is compiled apart)
COMPAND_ONE = [("0,7,22-17-18", m, dict(kw, precision=p, compand=a))
               for m, kw in (("tanh", {"gamma": 0.5}), ("cos", {})) for a in ("phi", "theta")
               for p in ("f64", "f32")]
VARIANTS += COMPAND_ONE
# the paper-literal truncating magnitude (§2.3): float32 norm, trailing mantissa bit dropped
VARIANTS += [("0,7,22-17-18", "plain", {"precision": p, "mag_round": "trunc"}) for p in ("f64", "f32")]
VARIANTS += [("0,7,22-17-18", "frac", {"P": 163840, "precision": "f32", "mag_round": "trunc"}),
             ("0,7,22-17-18", "tanh", {"gamma": 0.5, "precision": "f64", "mag_round": "trunc"}),
             ("0,8,23-16-17", "plain", {"precision": "f64", "mag_round": "trunc"})]


@pytest.mark.parametrize("layout,mode,kw", VARIANTS)
def test_encode_decode_variants(torch_dev, layout, mode, kw):
    say(f"case: variant {layout} {mode} {kw}")
    okw = {k: v for k, v in kw.items() if k != "precision"}
    c, co = vc.codec(layout, mode=mode, **kw), O.codec(layout, mode=mode, **okw)
    for name, xyz in [("sphere_log", inputs.sphere_loguniform(1 << 18, 1)),
                      ("vmf_pole", inputs.vmf(1 << 16, 1000.0, seed=5)),
                      ("gauss", inputs.gaussian_with_edges(1 << 16, 3))]:
        dev = gpu_encode(torch_dev, c, xyz)
        res = classify(co, xyz, dev)
        say(f"  {name}: {_summary(res)}")
        assert res["other"] == 0, describe_bad(co, xyz, dev, res)
        w = O.encode(co, xyz)
        d = vc.vc_decode(c, up(torch_dev, w))
        torch_dev.cuda.synchronize()
        err, nan_ok = decode_err(co, w, down(d))
        say(f"  {name}: decode max err/r = {err:.3e}")
        assert nan_ok and err <= 1e-6


def test_encode_nonfinite_and_zero_grid(torch_dev):
    """every combination of NaN, +-inf, +-0, 1 and 3e38 in three components, for every codec:
    a NaN or infinity in any component gives the reserved code, the zero vector the zero code,
    the rest the oracle's codes (within the window)"""
    v = np.array([np.nan, np.inf, -np.inf, 0.0, -0.0, 1.0, 3e38], dtype=np.float32)
    xyz = np.ascontiguousarray(np.stack(np.meshgrid(v, v, v, indexing="ij"), axis=-1).reshape(-1, 3))
    bad = ~np.isfinite(xyz).all(axis=1)
    zero = (xyz == 0).all(axis=1)
    for layout, mode, kw in VARIANTS:
        okw = {k: v for k, v in kw.items() if k != "precision"}
        c, co = vc.codec(layout, mode=mode, **kw), O.codec(layout, mode=mode, **okw)
        dev = gpu_encode(torch_dev, c, xyz)
        ref = O.encode(co, xyz)
        assert np.array_equal(dev[bad], ref[bad]) and len(set(ref[bad].tolist())) == 1, (layout, mode, kw)
        assert (dev[zero] == 0).all(), (layout, mode, kw)
        res = classify(co, xyz, dev)
        assert res["other"] == 0, (layout, mode, kw, describe_bad(co, xyz, dev, res))
    say(f"non-finite grid: {len(VARIANTS)} codecs, {int(bad.sum())} non-finite and {int(zero.sum())} zero vectors each")


def test_decode_arbitrary_codes_every_codec(torch_dev):
    """every 64-bit word (subnormal magnitudes of the e = 8 layouts, reserved exponents,
    fractional-split fields beyond P T) decodes as the oracle decodes it: NaN exactly where the
    oracle gives NaN, values within 1e-6 r_hat + 2^-149"""
    w = random_codes(1 << 18, 18)
    for layout, mode, kw in VARIANTS:
        okw = {k: v for k, v in kw.items() if k != "precision"}
        c, co = vc.codec(layout, mode=mode, **kw), O.codec(layout, mode=mode, **okw)
        d = vc.vc_decode(c, up(torch_dev, w))
        torch_dev.cuda.synchronize()
        excess = decode_abs_err(co, w, down(d))
        assert excess <= 0.0, (layout, mode, kw, excess)
    say(f"arbitrary codes: {len(VARIANTS)} codecs x {len(w)} words decode within tolerance")


def test_decode_random_codes(torch_dev):
    """Every valid code (random fields) plus zero and reserved codes."""
    say("case: decode random codes")
    c, co = vc.codec(), O.codec()
    g = np.random.default_rng(7)
    n = 1 << 18
    E = g.integers(1, 127, n, dtype=np.uint64)
    M = g.integers(0, 1 << 22, n, dtype=np.uint64)
    P = g.integers(0, 1 << 17, n, dtype=np.uint64)
    T = g.integers(0, 1 << 18, n, dtype=np.uint64)
    w = (E << np.uint64(57)) | (M << np.uint64(35)) | (P << np.uint64(18)) | T
    w[:4] = [0, 127 << 57, (127 << 57) | 12345, 1 << 57]
    d = down(vc.vc_decode(c, up(torch_dev, w)))
    err, nan_ok = decode_err(co, w, d)
    say(f"decode random codes: max err/r = {err:.3e}")
    assert nan_ok and err <= 1e-6
    assert (d[0] == 0).all() and np.isnan(d[1]).all() and np.isnan(d[2]).all()


# ----------------------------------------------------------------------------- axpy
def _axpy_operands(n, seed_a, seed_b):
    xa = inputs.gaussian_with_edges(n, seed_a)
    xb = inputs.gaussian_with_edges(n, seed_b)
    xb[-11:-4] = -xa[-11:-4]          # negated axes/zero: a + b hits exact zero
    return xa, xb


def _level_stretch(mode, n_max, gamma=0.5):
    """largest quantisation error of a companded angle (normalised u in [-1, 1]) over the uniform
    half step 1/n_max.  §2.5: the levels are uniform in h = 2 n/n_max - 1 and decode to
    u = atanh(tanh(gamma) h)/gamma (tanh) or (2/pi) asin(h) (cosine); rounding is to the nearest
    level in h, so a value decodes to its level from anywhere up to the midpoints in h on either
    side, which lie farther than half a step in u where the map is flat (the cosine map's ends)."""
    h = 2.0 * np.arange(n_max + 1, dtype=np.float64) / n_max - 1.0
    hm = 0.5 * (h[1:] + h[:-1])

    def u_of(x):
        if mode == "tanh":
            return np.arctanh(np.tanh(gamma) * x) / gamma
        return (2.0 / np.pi) * np.arcsin(np.clip(x, -1.0, 1.0))
    u, um = u_of(h), u_of(hm)
    worst = max((um - u[:-1]).max(), (u[1:] - um).max())
    return float(worst / (1.0 / n_max))


def _check_axpy(torch, c, co, wa, wb, alpha, label, mag_err=2.0 ** -23, stretch=(1.0, 1.0)):
    ta, tb = up(torch, wa), up(torch, wb)
    out = vc.vc_axpy(c, alpha, ta, tb)
    out2, c32 = vc.vcx_axpy_dump(c, alpha, ta, tb)
    torch.cuda.synchronize()
    wc, wc2, c32 = down(out, True), down(out2, True), down(c32)
    # 1. fused kernel == verification variant == GPU encode of the pre-encode sum
    assert np.array_equal(wc, wc2)
    assert np.array_equal(wc, gpu_encode(torch, c, c32))
    # 2. encode rule against the oracle on the same single-precision sums
    res = classify(co, c32, wc)
    say(f"{label}: encode-of-sum {_summary(res)}")
    assert res["other"] == 0, describe_bad(co, c32, wc, res)
    # 3. end to end vs the FP64 sum of the exactly decoded operands
    A64, B64 = O.decode64(co, wa), O.decode64(co, wb)
    c64 = alpha * A64 + B64
    got = O.decode64(co, wc)
    nrm = np.linalg.norm(c64, axis=1)
    scale = alpha * np.linalg.norm(A64, axis=1) + np.linalg.norm(B64, axis=1)
    ok = (nrm > 2.0 ** -70) & (nrm < 1e14)
    nt, npm = O.nmax(co)
    codec_bound = math.hypot(math.pi / nt * stretch[0], math.pi / (2 * npm) * stretch[1]) + mag_err
    err = np.linalg.norm(got - c64, axis=1)[ok]
    allowed = codec_bound * nrm[ok] + (4 * 2.0 ** -24 + 1e-6) * scale[ok]
    say(f"{label}: max end-to-end err/allowed = {(err / allowed).max():.3f}")
    assert (err <= allowed).all()
    # exact zeros: a + b == 0 exactly where b = -a
    z = np.all(c64 == 0, axis=1)
    assert (wc[z] == 0).all()
    # 4. field-wise agreement with the oracle's own axpy (reported)
    ref = O.axpy(co, alpha, wa, wb)
    same = np.mean(ref == wc)
    say(f"{label}: identical to oracle axpy codes: {same * 100:.4f} %")
    return wc


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_axpy_config1(torch_dev, prec):
    """c = a + b (alpha = 1) and alpha = 0.7 on the N(0,1) + edge-case operands."""
    say(f"case: axpy config1 {prec}")
    c, co = vc.codec(precision=prec), O.codec()
    xa, xb = _axpy_operands(65536, 0, 1)
    wa, wb = O.encode(co, xa), O.encode(co, xb)
    _check_axpy(torch_dev, c, co, wa, wb, 1.0, "axpy config1 alpha=1")
    _check_axpy(torch_dev, c, co, wa, wb, ALPHA, "axpy config1 alpha=0.7")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("mode,kw", [("tanh", {"gamma": 0.5}), ("tanh", {"gamma": 1.0}), ("cos", {}),
                                     ("tanh", {"gamma": 0.5, "compand": "phi"}),
                                     ("cos", {"compand": "theta"})])
def test_axpy_companded(torch_dev, mode, kw, prec):
    """the companded codecs' axpy (both angles, and one angle only) under the layered contract,
    with either encoder"""
    say(f"case: axpy {mode} {kw} {prec}")
    c, co = vc.codec(mode=mode, precision=prec, **kw), O.codec(mode=mode, **kw)
    xa, xb = _axpy_operands(65536, 4, 5)
    wa, wb = O.encode(co, xa), O.encode(co, xb)
    nt, npm = O.nmax(co)
    mask = kw.get("compand", "both")
    g = kw.get("gamma", 0.5)
    st = _level_stretch(mode, nt, g) if mask in ("both", "theta") else 1.0
    sp = _level_stretch(mode, npm, g) if mask in ("both", "phi") else 1.0
    _check_axpy(torch_dev, c, co, wa, wb, ALPHA, f"axpy {mode} {kw}", stretch=(st, sp))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_axpy_arbitrary_codes(torch_dev, prec):
    """operands of arbitrary 64-bit words (reserved exponents among them, so NaN sums): the fused
    kernel equals its verification variant and the GPU encode of its own single-precision sums,
    and those codes follow the encode rule against the oracle (reserved code for NaN sums)"""
    torch = torch_dev
    say(f"case: axpy arbitrary codes {prec}")
    c, co = vc.codec(precision=prec), O.codec()
    n = (1 << 16) + 7
    wa, wb = random_codes(n, 31), random_codes(n, 32)
    ta, tb = up(torch, wa), up(torch, wb)
    out = vc.vc_axpy(c, ALPHA, ta, tb)
    out2, c32 = vc.vcx_axpy_dump(c, ALPHA, ta, tb)
    torch.cuda.synchronize()
    wc, wc2, c32 = down(out, True), down(out2, True), down(c32)
    assert np.array_equal(wc, wc2)
    assert np.array_equal(wc, gpu_encode(torch, c, c32))
    res = classify(co, c32, wc)
    nan_sums = int((~np.isfinite(c32).all(axis=1)).sum())
    say(f"axpy arbitrary codes {prec}: {_summary(res)}, {nan_sums} non-finite sums")
    assert nan_sums > 0 and res["other"] == 0, describe_bad(co, c32, wc, res)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_axpy_truncating_magnitude(torch_dev, prec):
    """the paper-literal magnitude: nearest-even at 24 bits, the last of them dropped, so the
    magnitude error is below 2^-22 + 2^-24 of the norm"""
    say(f"case: axpy truncating magnitude {prec}")
    c, co = vc.codec(precision=prec, mag_round="trunc"), O.codec(mag_round="trunc")
    xa, xb = _axpy_operands(65536, 20, 21)
    wa, wb = O.encode(co, xa), O.encode(co, xb)
    _check_axpy(torch_dev, c, co, wa, wb, ALPHA, "axpy trunc alpha=0.7", mag_err=2.0 ** -22 + 2.0 ** -24)
    # the codes differ from the nearest-even codec's on about a quarter of the sums
    wr = down(vc.vc_axpy(vc.codec(precision=prec), ALPHA, up(torch_dev, wa), up(torch_dev, wb)), True)
    wt = down(vc.vc_axpy(c, ALPHA, up(torch_dev, wa), up(torch_dev, wb)), True)
    frac = float(np.mean(wr != wt))
    say(f"axpy trunc vs rne: {frac * 100:.2f} % of codes differ")
    assert 0.15 < frac < 0.35


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 2, 3, 511, 512, 513, 1023, 1025, 4099])
def test_axpy_ragged_and_unaligned(torch_dev, n, prec):
    say(f"case: axpy ragged n={n} {prec}")
    torch = torch_dev
    c, co = vc.codec(precision=prec), O.codec()
    xa, xb = inputs.sphere_loguniform(n + 1, 11), inputs.sphere_loguniform(n + 1, 12)
    wa, wb = O.encode(co, xa), O.encode(co, xb)
    ref_gpu = _check_axpy(torch, c, co, wa[:n], wb[:n], ALPHA, f"axpy n={n}")
    # element offset 1: 8-byte aligned but not 16-byte aligned -> scalar path
    ta, tb = up(torch, wa), up(torch, wb)
    out = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    vc.vc_axpy(c, ALPHA, ta[1:], tb[1:], out[1:])
    torch.cuda.synchronize()
    got = down(out, True)
    assert got[0] == 0
    ref_shift = _check_axpy(torch, c, co, wa[1:], wb[1:], ALPHA, f"axpy n={n} offset")
    assert np.array_equal(got[1:], ref_shift)
    # in-place (c aliases a)
    vc.vc_axpy(c, ALPHA, ta[:n], tb[:n], ta[:n])
    torch.cuda.synchronize()
    assert np.array_equal(down(ta, True)[:n], ref_gpu)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_axpy_every_launch_config(torch_dev, prec):
    """Every launch configuration the autotuner may pick gives the codes of the default one, on
    several whole tiles plus a ragged tail (and those codes follow the encode rule)."""
    from paper_2003_02633_amd import tune
    say(f"case: axpy launch configurations {prec}")
    torch = torch_dev
    c, co = vc.codec(precision=prec), O.codec()
    n = 3 * 2 * 512 * 4 + 77
    xa, xb = inputs.sphere_loguniform(n, 21), inputs.sphere_loguniform(n, 22)
    wa, wb = O.encode(co, xa), O.encode(co, xb)
    ref = _check_axpy(torch, c, co, wa, wb, ALPHA, f"axpy default config {prec}")
    ta, tb = up(torch, wa), up(torch, wb)
    saved = vc.get_stream_config(prec)
    try:
        for blk, vpt, nt in tune.CONFIGS:
            vc.set_stream_config(blk, vpt, nt, prec)
            out = torch.zeros(n, dtype=torch.int64, device="cuda")
            vc.vc_axpy(c, ALPHA, ta, tb, out)
            torch.cuda.synchronize()
            assert np.array_equal(down(out, True), ref), (blk, vpt, nt)
    finally:
        vc.set_stream_config(*saved, prec)


def test_encode_decode_ragged_unaligned(torch_dev):
    torch = torch_dev
    c, co = vc.codec(), O.codec()
    for n in (1, 3, 4, 5, 1021, 4096 + 7):
        say(f"case: encode/decode ragged n={n}")
        xyz = inputs.sphere_loguniform(n + 1, 13)
        t = up(torch, xyz)
        codes = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
        vc.vc_encode(c, t[1:], codes[1:])                  # 12-byte offset: scalar path
        codes_a = vc.vc_encode(c, t[:n].contiguous())      # aligned path
        torch.cuda.synchronize()
        res = classify(co, xyz[1:], down(codes, True)[1:])
        assert res["other"] == 0
        res = classify(co, xyz[:n], down(codes_a, True))
        assert res["other"] == 0
        w = O.encode(co, xyz)
        tw = up(torch, w)
        out = torch.zeros((n + 1) * 3, dtype=torch.float32, device="cuda")
        vc.vc_decode(c, tw[1:], out[3:].view(n, 3))
        torch.cuda.synchronize()
        err, nan_ok = decode_err(co, w[1:], down(out)[3:].reshape(n, 3))
        assert nan_ok and err <= 1e-6 and (down(out)[:3] == 0).all()


def test_zero_length_and_empty(torch_dev):
    torch = torch_dev
    c = vc.codec()
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    assert vc.vc_axpy(c, 1.0, e, e).numel() == 0
    out = vc.vc_norm2(c, e)
    torch.cuda.synchronize()
    assert float(out.cpu()[0]) == 0.0


# ----------------------------------------------------------------------------- reductions
@pytest.mark.parametrize("n", [1, 1000, 65547, 1 << 20])
def test_dot_norm2(torch_dev, n):
    say(f"case: dot/norm2 n={n}")
    torch = torch_dev
    c, co = vc.codec(), O.codec()
    wa = O.encode(co, inputs.gaussian_with_edges(n, 21)[:n])
    wb = O.encode(co, inputs.gaussian_with_edges(n, 22)[:n])
    ta, tb = up(torch, wa), up(torch, wb)
    d = float(vc.vc_dot(c, ta, tb).cpu()[0])
    s = float(vc.vc_norm2(c, ta).cpu()[0])
    ref_d, ref_s = O.dot(co, wa, wb), O.norm2(co, wa)
    A, B = O.decode64(co, wa), O.decode64(co, wb)
    scale = float((np.linalg.norm(A, axis=1) * np.linalg.norm(B, axis=1)).sum())
    say(f"dot n={n}: gpu {d:.9e} oracle {ref_d:.9e}; norm2 gpu {s:.9e} oracle {ref_s:.9e}")
    assert abs(d - ref_d) <= 4e-6 * scale
    assert abs(s - ref_s) <= 4e-6 * ref_s
    # operands one code in (8-byte but not 16-byte aligned: the one-code-per-load path)
    if n > 1:
        ta2, tb2 = up(torch, np.concatenate([wa[:1], wa])), up(torch, np.concatenate([wb[:1], wb]))
        d2 = float(vc.vc_dot(c, ta2[1:], tb2[1:]).cpu()[0])
        s2 = float(vc.vc_norm2(c, ta2[1:]).cpu()[0])
        assert abs(d2 - ref_d) <= 4e-6 * scale
        assert abs(s2 - ref_s) <= 4e-6 * ref_s


# ----------------------------------------------------------------------------- fractional split
def _frac_codes(P, T, n, seed):
    """<0,7,22> codes whose 35-bit field n_p covers [0, P T] and a little past it: uniform draws,
    exact multiples of T and their neighbours, the range ends"""
    g = np.random.default_rng(seed)
    lim = P * T
    k = g.integers(1, P, n // 4, dtype=np.uint64)
    npf = np.concatenate([g.integers(0, lim + (lim >> 6), n // 4, dtype=np.uint64), k * np.uint64(T),
                          k * np.uint64(T) - np.uint64(1), k * np.uint64(T) + np.uint64(1),
                          np.array([0, 1, T - 1, T, lim - T, lim - 1, lim, lim + 1], dtype=np.uint64)])
    E = g.integers(1, 127, npf.size, dtype=np.uint64)
    M = g.integers(0, 1 << 22, npf.size, dtype=np.uint64)
    return (E << np.uint64(57)) | (M << np.uint64(35)) | npf


@pytest.mark.parametrize("P", [163840, 12_000_000, (1 << 24) - 3, 1 << 24])
def test_frac_decode_large_P(torch_dev, P):
    """Eq. (q_split) with up to 2^24 phi levels: the decode's quotient n_p / T and remainder
    match the oracle's integer division for every accepted P (decoded values within 1e-6 r_hat,
    NaN exactly past P T); encoding round-trips on the same codec follow the encode rule"""
    say(f"case: frac decode P={P}")
    c, co = vc.codec(mode="frac", P=P), O.codec(mode="frac", P=P)
    T = O.frac_T(co)
    w = _frac_codes(P, T, 1 << 18, P % 997)
    d = down(vc.vc_decode(c, up(torch_dev, w)))
    assert decode_abs_err(co, w, d) <= 0.0
    x = inputs.sphere_loguniform(1 << 16, 3)
    dev = gpu_encode(torch_dev, c, x)
    res = classify(co, x, dev)
    assert res["other"] == 0, describe_bad(co, x, dev, res)


@pytest.mark.parametrize("mode,kw", [("plain", {}), ("frac", {"P": 163840}), ("frac", {"P": 1 << 24})])
def test_norm2_dot_of_codes_against_oracle(torch_dev, mode, kw):
    """norm2 = sum |decode(w)|^2 and dot over valid codes of every field value, and NaN where
    some code decodes to NaN (fractional-split fields past P T), as in the oracle"""
    torch = torch_dev
    say(f"case: norm2/dot codes {mode} {kw}")
    c, co = vc.codec(mode=mode, **kw), O.codec(mode=mode, **kw)
    if mode == "frac":
        T = O.frac_T(co)
        w = _frac_codes(kw["P"], T, 1 << 16, 5)
        valid = (w & np.uint64((1 << 35) - 1)) < np.uint64(kw["P"] * T)
    else:
        g = np.random.default_rng(6)
        n = 1 << 16
        w = (g.integers(1, 127, n, dtype=np.uint64) << np.uint64(57)) | \
            (g.integers(0, 1 << 57, n, dtype=np.uint64))
        valid = np.ones(n, dtype=bool)
    wv = w[valid]
    wb = np.roll(wv, 1)
    for codes, expect_nan in ((wv, False), (w, not valid.all())):
        s = float(vc.vc_norm2(c, up(torch, codes)).cpu()[0])
        ref = O.norm2(co, codes)
        if expect_nan:
            assert math.isnan(s) and math.isnan(ref)
        else:
            assert abs(s - ref) <= 4e-6 * ref, (s, ref)
    dv = float(vc.vc_dot(c, up(torch, wv), up(torch, wb)).cpu()[0])
    A, B = O.decode64(co, wv), O.decode64(co, wb)
    scale = float((np.linalg.norm(A, axis=1) * np.linalg.norm(B, axis=1)).sum())
    assert abs(dv - O.dot(co, wv, wb)) <= 4e-6 * scale
