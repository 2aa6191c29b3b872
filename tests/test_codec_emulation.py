"""CPU emulation of the device codec (vc_device.hpp compiled for the host) against the oracle.

The emulation runs the kernels' exact integer and double-float logic with FP64-based
stand-ins for the hardware transcendentals, so these tests check the codec's
algorithm on any machine before it runs on the GPU.  The GPU tests repeat the
same comparisons with the real kernels.
"""
import math

import numpy as np
import pytest

import oracle as O
import paper_2003_02633_amd as vc
import tests.hostemu as H
from paper_2003_02633_amd import inputs
from tests.exact import exact_sq_norm, round_sqrt
from tests.parity import classify, decode_abs_err, decode_err, describe_bad, random_codes

from fractions import Fraction

VARIANTS = []
for _prec in ("f64", "f32"):
    VARIANTS += [
        ("0,7,22-17-18", "plain", {"precision": _prec}),
        ("0,7,23-17-17", "plain", {"precision": _prec}),
        ("0,8,23-16-17", "plain", {"precision": _prec}),
        ("1,8,23-16-16", "plain", {"precision": _prec}),
        ("0,7,22-17-18", "frac", {"P": 1 << 16, "precision": _prec}),
        ("0,7,22-17-18", "frac", {"P": 163840, "precision": _prec}),
        ("0,7,22-17-18", "frac", {"P": 1 << 18, "precision": _prec}),
        ("0,7,22-17-18", "frac", {"P": 100003, "precision": _prec}),
    ]
    _m = []
    VARIANTS += [
        pytest.param("0,7,22-17-18", "tanh", {"gamma": 0.5, "precision": _prec}, marks=_m),
        pytest.param("0,7,22-17-18", "tanh", {"gamma": 1.0, "precision": _prec}, marks=_m),
        pytest.param("0,7,22-17-18", "cos", {"precision": _prec}, marks=_m),
    ]
    # companding of one angle only
    VARIANTS += [pytest.param("0,7,22-17-18", m, dict(kw, precision=_prec, compand=a), marks=_m)
                 for m, kw in (("tanh", {"gamma": 0.5}), ("cos", {})) for a in ("phi", "theta")]
    # the paper-literal truncating magnitude (§2.3); only the 22-bit mantissa drops a bit
    VARIANTS += [
        ("0,7,22-17-18", "plain", {"precision": _prec, "mag_round": "trunc"}),
        ("0,7,22-17-18", "frac", {"P": 163840, "precision": _prec, "mag_round": "trunc"}),
        pytest.param("0,7,22-17-18", "tanh", {"gamma": 0.5, "precision": _prec, "mag_round": "trunc"}, marks=_m),
        ("0,8,23-16-17", "plain", {"precision": _prec, "mag_round": "trunc"}),
    ]


def _pair(layout, mode, kw):
    c = vc.codec(layout, mode=mode, **kw)
    okw = {k: v for k, v in kw.items() if k != "precision"}
    co = O.codec(layout, mode=mode, **okw)
    return c, co


def _workloads():
    g = np.random.default_rng(9)
    crafted = np.array([[1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0], [0, 0, 0], [1, 0, 1], [0, 1, 1],
                        [0, -1, -1], [3, 4, 0], [-3, 4, 12], [-1, -1e-30, 0], [1e10, -1e-30, 0],
                        [-1e10, -1e-30, 0], [0, 0, -0.0], [-0.0, -0.0, 1], [1e-40, -1e-41, 0]],
                       dtype=np.float32)
    tiny = (g.standard_normal((2000, 3)) * 1e-39).astype(np.float32)
    # magnitudes at and around the ends of every layout's range (flush, smallest code, the
    # rounding midpoint below 2^47 that saturates, IEEE subnormals and overflow for e = 8)
    radii = [2.0 ** -81, 2.0 ** -80, 2.0 ** -80 * (1 + 2.0 ** -23), 2.0 ** -79 * (1 - 2.0 ** -24), 2.0 ** -79,
             1.5 * 2.0 ** -79, 2.0 ** 46 * (2 - 2.0 ** -22), 2.0 ** 46 * (2 - 2.0 ** -23),
             2.0 ** 46 * (2 - 2.0 ** -24), 2.0 ** 47, 1e20, 3.0e38, 1.1754944e-38, 1e-40, 1.4e-45, 2.0 ** -126,
             2.0 ** -127 * 1.5, 2.0 ** 127 * (2 - 2.0 ** -23)]
    dirs = np.array([[1, 0, 0], [0.6, 0.8, 0], [0, 0, -1], [1, 2, 3]], dtype=np.float64)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    with np.errstate(over="ignore"):
        limits = (np.array(radii)[:, None, None] * dirs[None]).reshape(-1, 3).astype(np.float32)
    limits = limits[np.isfinite(limits).all(axis=1)]
    # norms beyond the largest float: saturate in the e = 8 layouts
    limits = np.concatenate([limits, np.array([[3e38, 3e38, 0], [3.4e38, 1e38, -1e38], [-2e38, 2e38, 2e38]],
                                              dtype=np.float32)])
    return [("gauss", inputs.gaussian_with_edges(20000, 0)), ("sphere_log", inputs.sphere_loguniform(60000, 1)),
            ("crafted", crafted), ("tiny", tiny), ("vmf_pole", inputs.vmf(20000, 1000.0, seed=5)),
            ("limits", limits), ("ties24", _ties24()), ("nonfinite", _nonfinite())]


def _nonfinite():
    """every combination of NaN, +-inf, 0 and 1 in three components (the finite ones included):
    non-finite input gives the reserved code, the zero vector the zero code"""
    v = np.array([np.nan, np.inf, -np.inf, 0.0, -0.0, 1.0, 3e38], dtype=np.float32)
    g = np.stack(np.meshgrid(v, v, v, indexing="ij"), axis=-1).reshape(-1, 3)
    return np.ascontiguousarray(g)


def _ties24():
    """vectors whose norm is an odd 25-bit integer (times a power of two): exact ties of the
    nearest-even rounding at 24 bits, from Pythagorean triples (m^2 - n^2, 2mn, m^2 + n^2)"""
    out = []
    for m in range(4096, 5793, 29):
        n0 = math.isqrt(max(m * m - (1 << 24), 0)) + 1
        for n in range(n0, n0 + 4):
            a, b, c = m * m - n * n, 2 * m * n, m * m + n * n
            if (m - n) % 2 == 0 or not (1 << 24) <= c < (1 << 25) or a >= (1 << 24) or b >= (1 << 24):
                continue
            for e in (-60, -10, 0, 20):
                s = 2.0 ** e
                out += [(a * s, b * s, 0.0), (-b * s, 0.0, a * s), (0.0, a * s, -b * s)]
    xyz = np.array(out, dtype=np.float32)
    assert np.array_equal(xyz.astype(np.float64), np.array(out))   # exactly representable
    return xyz


@pytest.mark.parametrize("layout,mode,kw", VARIANTS)
def test_emulated_encode_matches_oracle(layout, mode, kw):
    c, co = _pair(layout, mode, kw)
    for name, xyz in _workloads():
        dev = H.encode(c, xyz)
        res = classify(co, xyz, dev)
        assert res["other"] == 0, f"{name}:\n" + describe_bad(co, xyz, dev, res)
        # within-window level differences are rare (design error ~1e-4 level units) on the drawn
        # workloads.  The non-finite grid and the crafted vectors are mostly axis and 45-degree
        # directions; for some level counts (fractional split, n_max = 2 mod 4) the diagonals lie
        # exactly on a level tie, which the encoder (angles from their half-angle tangents, exact
        # on the axes only) may resolve either way inside the window
        if name not in ("nonfinite", "crafted"):
            assert res["pm1_theta"] + res["pm1_phi"] <= max(2, 2e-3 * res["n"]), res


@pytest.mark.parametrize("layout,mode,kw", VARIANTS)
def test_emulated_decode_matches_oracle(layout, mode, kw):
    c, co = _pair(layout, mode, kw)
    w = O.encode(co, inputs.sphere_loguniform(50000, 2))
    err, nan_ok = decode_err(co, w, H.decode(c, w))
    assert nan_ok and err <= 1e-6


@pytest.mark.parametrize("layout,mode,kw", VARIANTS)
def test_emulated_decode_of_arbitrary_codes(layout, mode, kw):
    """every 64-bit word decodes as the oracle decodes it: NaN exactly for the reserved exponent
    (and fractional-split fields beyond the P T levels), values within 1e-6 r_hat + 2^-149"""
    c, co = _pair(layout, mode, kw)
    w = random_codes(200_000, 17)
    assert decode_abs_err(co, w, H.decode(c, w)) <= 0.0


@pytest.mark.parametrize("layout,mode,kw", [v for v in VARIANTS if not hasattr(v, "marks") or not v.marks])
def test_emulated_dot_pair_matches_oracle(layout, mode, kw):
    """The kernels' dot product of two codes, taken in spherical form (the angle difference from
    the level counts), against the FP64 dot product of the oracle's decodes, per pair."""
    c, co = _pair(layout, mode, kw)
    xa, xb = inputs.sphere_loguniform(20000, 31), inputs.sphere_loguniform(20000, 32)
    wa, wb = O.encode(co, xa), O.encode(co, xb)
    wb[:50] = wa[:50]                                  # equal angles (theta difference zero)
    wa[50:60] = 0                                      # the zero code
    got = H.dot_pair(c, wa, wb).astype(np.float64)
    A, B = O.decode64(co, wa), O.decode64(co, wb)
    ref = np.einsum("ij,ij->i", A, B)
    scale = np.linalg.norm(A, axis=1) * np.linalg.norm(B, axis=1)
    assert np.all(got[50:60] == 0.0)
    assert np.all(np.abs(got - ref) <= 1e-6 * scale), np.max(np.abs(got - ref) / np.maximum(scale, 1e-300))


def test_ties24_are_ties():
    """the tie workload holds exact midpoints of the 24-bit rounding (checked in exact arithmetic)"""
    xyz = _ties24()
    assert len(xyz) > 50
    for x, y, z in xyz[::7]:
        S = exact_sq_norm(float(x), float(y), float(z))
        r = Fraction(math.isqrt(S.numerator), math.isqrt(S.denominator))
        assert r * r == S
        e = math.floor(math.log2(r))
        q = r / Fraction(2) ** (e - 24)          # 25 significant bits, odd last bit
        assert q.denominator == 1 and q.numerator % 2 == 1


def test_truncation_is_nearest_even_for_23bit_mantissas():
    """the library resolves VC_MAG_TRUNC to nearest-even where the mantissa has 23 bits, since
    no bit is dropped; the oracle's paper-literal truncation gives the same codes there"""
    xs = np.concatenate([w for _, w in _workloads()])
    for layout in ("0,7,23-17-17", "0,8,23-16-17", "1,8,23-16-16"):
        ct, cr = O.codec(layout, mag_round="trunc"), O.codec(layout)
        assert np.array_equal(O.encode(ct, xs), O.encode(cr, xs)), layout
    # the 22-bit mantissa does differ: in units of its grid step, with r in [k, k + 1), nearest-even
    # gives k + 1 above k + 1/2 and truncation only from k + 3/4 (where the 24-bit rounding
    # carries), so a quarter of the norms land on different codes
    ct, cr = O.codec(mag_round="trunc"), O.codec()
    d = O.encode(ct, xs) != O.encode(cr, xs)
    assert 0.2 < d.mean() < 0.3


def test_single_product_level_reciprocals():
    """Uniform levels have n_max = 2^k - 1 (k = 16..18), whose reciprocal (and half of it) rounds
    to float32 within 2^-32 relative, so the decode's single product loses nothing measurable."""
    for k in (16, 17, 18):
        for r in (1.0 / ((1 << k) - 1), 1.0 / (2.0 * ((1 << k) - 1))):
            assert abs(float(np.float32(r)) - r) / r <= 2.0 ** -32


def test_emulated_exact_norm_path():
    """The exact integer magnitude path (taken near rounding midpoints) is exact."""
    g = np.random.default_rng(10)
    cases = list(g.standard_normal((300, 3)).astype(np.float32) * np.float32(3.7))
    for k in range(30):
        m = np.float32(((1 << 23) + 2 * k + 1) * 2.0 ** -23)
        cases += [(m, 0, 0), (m, np.float32(2.0 ** -70), 0), (np.float32(1e-39), np.float32(-3e-40), 0)]
    for x, y, z in cases:
        x, y, z = float(np.float32(x)), float(np.float32(y)), float(np.float32(z))
        for prec, keep in ((23, False), (24, False), (24, True)):
            j, gexp = H.exact_norm(x, y, z, prec, keep)
            S = exact_sq_norm(x, y, z)
            ref = round_sqrt(S, prec, Fraction(1, 1 << 149) if keep else None)
            assert Fraction(j) * Fraction(2) ** gexp == ref, (x, y, z, prec, keep)


def _frac_quotient_codes(P, T, n, seed):
    """codes of the <0,7,22> layout whose low 35-bit field n_p covers the valid range [0, P T):
    uniform draws, exact multiples of T (remainder zero, where an estimate of n_p / T from below
    truncates one short), their neighbours, and the ends of the range"""
    g = np.random.default_rng(seed)
    lim = P * T
    k = g.integers(1, P, n // 4, dtype=np.uint64)
    npf = np.concatenate([g.integers(0, lim, n // 4, dtype=np.uint64), k * np.uint64(T),
                          k * np.uint64(T) - np.uint64(1), k * np.uint64(T) + np.uint64(1),
                          np.array([0, 1, T - 1, T, lim - T, lim - 1, lim, lim + 1], dtype=np.uint64)])
    E = g.integers(1, 127, npf.size, dtype=np.uint64)
    M = g.integers(0, 1 << 22, npf.size, dtype=np.uint64)
    return (E << np.uint64(57)) | (M << np.uint64(35)) | npf


@pytest.mark.parametrize("P", [163840, 1 << 20, 1 << 22, 12_000_000, 16_000_001, (1 << 24) - 3, 1 << 24])
def test_emulated_frac_decode_large_P(P):
    """Fractional split (§2.4, Eq. q_split) with up to 2^24 phi levels: n_phi = floor(n_p / T) and
    n_theta = n_p mod T decode as the oracle's integer division does, including n_p at multiples
    of T, for every n_phi_max + 1 the library accepts (P <= 2^24)"""
    c, co = _pair("0,7,22-17-18", "frac", {"P": P})
    T = O.frac_T(co)
    w = _frac_quotient_codes(P, T, 200_000, P % 1000)
    assert decode_abs_err(co, w, H.decode(c, w)) <= 0.0
    # the round trip through the encoder stays on valid fields
    assert decode_abs_err(co, w[:20000], H.decode(c, w[:20000])) <= 0.0


def test_emulated_norm2_magnitude_frac_limit():
    """norm2's magnitude of a fractional-split code is NaN past the P T levels, as its decode is"""
    c, co = _pair("0,7,22-17-18", "frac", {"P": 163840})
    T = O.frac_T(co)
    w = _frac_quotient_codes(163840, T, 4000, 3)
    ref = O.decode64(co, w)
    mag = H.magnitude_checked(c, w)
    assert np.array_equal(np.isnan(mag), np.isnan(ref).any(axis=1))
    fin = ~np.isnan(mag)
    assert np.allclose(mag[fin].astype(np.float64), np.linalg.norm(ref[fin], axis=1), rtol=1e-6, atol=0)
