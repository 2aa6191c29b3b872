"""Code-level comparison of device (or emulated) codes with the oracle.

Rule: codes must equal the oracle's bit for bit, except
that an angle field may differ by exactly one level when the exact level
coordinate lies within one single-precision ulp of the angle (expressed in
level units) of the boundary between the two levels.  Such cases are counted.
The magnitude fields must match exactly.
"""
from __future__ import annotations

import numpy as np

import oracle as O


def _base(nmax: int) -> int:
    return (nmax + 1) // 2 if nmax % 2 else nmax // 2


def classify(co, xyz, dev_codes, threads: int = 0):
    """Return a dict of counts and boolean masks comparing dev codes with the oracle."""
    xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32).reshape(-1, 3))
    dev = np.asarray(dev_codes).astype(np.uint64).reshape(-1)
    ref, q5, flags = O.encode_detail(co, xyz, threads)
    Er, Mr, Pr, Tr = O.fields(co, ref)
    Ed, Md, Pd, Td = O.fields(co, dev)
    nt_max, np_max = O.nmax(co)
    same = ref == dev
    mag_ok = (Er == Ed) & (Mr == Md)
    dt = Td.astype(np.int64) - Tr.astype(np.int64)
    dp = Pd.astype(np.int64) - Pr.astype(np.int64)
    bt = np.maximum(Td, Tr).astype(np.int64) - _base(nt_max)
    bp = np.maximum(Pd, Pr).astype(np.int64) - _base(np_max)
    win_t = np.abs(q5[:, 0] - bt) <= q5[:, 1]
    win_p = np.abs(q5[:, 2] - bp) <= q5[:, 3]
    ok_t = (dt == 0) | ((np.abs(dt) == 1) & win_t)
    ok_p = (dp == 0) | ((np.abs(dp) == 1) & win_p)
    ok = same | (mag_ok & ok_t & ok_p)
    return {
        "n": int(ref.size),
        "identical": int(same.sum()),
        "pm1_theta": int(((np.abs(dt) == 1) & win_t & mag_ok).sum()),
        "pm1_phi": int(((np.abs(dp) == 1) & win_p & mag_ok).sum()),
        "mag_mismatch": int((~mag_ok).sum()),
        "other": int((~ok).sum()),
        "bad_mask": ~ok,
        "ref": ref,
    }


def describe_bad(co, xyz, dev_codes, res, limit: int = 8) -> str:
    xyz = np.asarray(xyz, dtype=np.float32).reshape(-1, 3)
    idx = np.nonzero(res["bad_mask"])[0][:limit]
    if idx.size == 0:
        return ""
    dev = np.asarray(dev_codes).astype(np.uint64).reshape(-1)
    lines = []
    _, q5, _ = O.encode_detail(co, xyz[idx])
    for k, i in enumerate(idx):
        r = int(res["ref"][i])
        d = int(dev[i])
        lines.append(f"i={i} x={xyz[i].tolist()} ref={r:#018x} dev={d:#018x} "
                     f"Q_t={q5[k,0]:.6f} w_t={q5[k,1]:.2e} Q_p={q5[k,2]:.6f} w_p={q5[k,3]:.2e}")
    return "\n".join(lines)


def decode_err(co, codes, dev_xyz):
    """max over vectors of max_k |x_dev - x_oracle| / r_hat (r_hat = |oracle decode|)."""
    ref = O.decode64(co, codes)
    dev = np.asarray(dev_xyz, dtype=np.float64).reshape(-1, 3)
    r = np.linalg.norm(ref, axis=1)
    fin = np.isfinite(ref).all(axis=1)
    err = np.abs(dev - ref).max(axis=1)
    rel = np.where(r > 0, err / np.where(r > 0, r, 1), err)
    nan_ok = np.array_equal(np.isnan(dev).any(axis=1), ~fin)
    return float(rel[fin].max(initial=0.0)), nan_ok


def random_codes(n, seed):
    """n arbitrary 64-bit codes (every field random: subnormal magnitudes of the e = 8 layouts,
    reserved exponents, fractional-split fields beyond P T) plus the zero and all-ones words"""
    g = np.random.default_rng(seed)
    w = g.integers(0, 1 << 32, n, dtype=np.uint64) << np.uint64(32) | g.integers(0, 1 << 32, n, dtype=np.uint64)
    w[:4] = [0, (1 << 64) - 1, 1 << 57, 127 << 57]
    return w


def decode_abs_err(co, w, dev):
    """max over components of |x_dev - x_oracle| - (1e-6 r_hat + 2^-149): positive means out of
    tolerance.  The float32 outputs of a subnormal-magnitude vector cannot be closer than the
    subnormal spacing 2^-149, whatever r_hat is."""
    ref = O.decode64(co, w)
    dev = np.asarray(dev, dtype=np.float64).reshape(-1, 3)
    fin = np.isfinite(ref).all(axis=1)
    assert np.array_equal(np.isnan(dev).any(axis=1), ~fin)
    r = np.linalg.norm(ref[fin], axis=1)
    return float((np.abs(dev[fin] - ref[fin]).max(axis=1) - (1e-6 * r + 2.0 ** -149)).max(initial=-1.0))
