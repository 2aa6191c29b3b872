"""Error characterisation of the codec on the GPU (FP64 error norms, vcx_error_hist): the sweeps
of §2.3-§2.5 at up to 10^8 samples per point.

The statistic is the paper's Eq. (stat): e_i = |x_i - x_hat_i|, its mean and standard deviation
(on the unit sphere and ball the radius-normalised error the kernel reports equals e_i for
|x| = 1, and the mean of the normalised error is the radius-invariant quantity of §2.3).

  layouts   §2.3: <0,8,23>-16-17, <0,7,23>-17-17, <0,7,22>-17-18 (angle-uniform sampling)
  table     §3 Table (C++_error), double/double rows: S^2 and [-1,1]^3
  frac      §2.4 Fig. (frac_1718): P = n_phi_max + 1 from 2^16 to 2^18 (35-bit split)
  tanh      §2.5: gamma in (0, 1], sigma(e) relative to uniform quantisation
  radius    §2.3: normalised mean over radii 1e-8 .. 1e8

Usage (on the GPU):  python -m paper_2003_02633_amd.sweeps [--n N] [--json FILE]
"""
from __future__ import annotations

import argparse
import json
import math
import sys

EDGES = None


def _edges(torch):
    global EDGES
    if EDGES is None:
        import numpy as np
        EDGES = torch.from_numpy(10.0 ** (-12.0 + np.arange(101, dtype=np.float64) / 10)).to("cuda")
    return EDGES


def stats(vc, c, kind: str, n: int, seed: int, radius: float = 1.0, chunk: int = 1 << 24):
    """mean, sigma (Eq. stat, N - 1 normalisation) and max of the normalised vector error over n
    samples of ``kind``, accumulated in FP64 over chunks"""
    import torch

    from paper_2003_02633_amd import inputs

    s1 = s2 = 0.0
    mx = 0.0
    m = 0
    for i, s in enumerate(range(0, n, chunk)):
        k = min(chunk, n - s)
        x = inputs.sampler_torch(kind, k, seed * 1000 + i, radius=radius)
        try:
            h, ex, st = vc.error_hist(c, x, _edges(torch))
        except vc.VcError as e:
            raise RuntimeError(f"{kind} chunk {i} ({k} vectors): {e}; "
                               f"torch reserved {torch.cuda.memory_reserved() / 2**30:.1f} GiB") from e
        cnt = int(h[0].sum())
        s1 += float(st[0, 0])
        s2 += float(st[0, 1])
        mx = max(mx, float(st[0, 2]))
        m += cnt
        del x
    mean = s1 / m
    var = (s2 - m * mean * mean) / (m - 1)
    return {"n": m, "mean": mean, "sigma": math.sqrt(max(var, 0.0)), "max": mx}


def run(n: int = 10 ** 8, log=print):
    import paper_2003_02633_amd as vc

    out = {"n_per_point": n}
    out["layouts"] = {lay: stats(vc, vc.codec(lay), "angles", n, 11)
                      for lay in ("0,8,23-16-17", "0,7,23-17-17", "0,7,22-17-18")}
    log(f"layouts: { {k: v['mean'] for k, v in out['layouts'].items()} }")
    out["table_cpp_error"] = {kind: stats(vc, vc.codec(), kind, n, 12) for kind in ("sphere", "cube")}
    log(f"table: { {k: (v['mean'], v['max']) for k, v in out['table_cpp_error'].items()} }")
    frac = {}
    for e2 in [16 + i / 4 for i in range(9)]:
        P = int(round(2 ** e2))
        frac[P] = stats(vc, vc.codec(mode="frac", P=P), "sphere", n, 13)
    out["frac"] = frac
    log(f"frac: { {k: round(v['mean'] * 1e6, 4) for k, v in frac.items()} }")
    base = stats(vc, vc.codec(), "sphere", n, 14)
    tanh = {}
    for g in (0.1, 0.25, 0.5, 0.75, 1.0):
        r = stats(vc, vc.codec(mode="tanh", gamma=g), "sphere", n, 14)
        r["sigma_reduction"] = 1.0 - r["sigma"] / base["sigma"]
        tanh[g] = r
    out["tanh"] = {"uniform": base, **{str(k): v for k, v in tanh.items()}}
    log(f"tanh sigma reduction: { {k: round(v['sigma_reduction'], 4) for k, v in tanh.items()} }")
    out["radius"] = {r: stats(vc, vc.codec(), "sphere", n, 15, radius=r)["mean"] for r in (1e-8, 1e-4, 1.0, 1e4, 1e8)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=float, default=1e8)
    ap.add_argument("--json", default=None)
    a = ap.parse_args()
    res = run(int(a.n), log=lambda m: print(m, file=sys.stderr, flush=True))
    txt = json.dumps(res, default=str)
    if a.json:
        with open(a.json, "w") as f:
            f.write(txt)
    print(txt, flush=True)


if __name__ == "__main__":
    main()
