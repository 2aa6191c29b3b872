"""Autotuner for the streaming compressed axpy (block size, vectors per thread, non-temporal) and
for the tile shape of the batched persistent kernel (code pairs per lane of axpy, dot and norm2
tiles).

Sweeps every launch configuration the library is built with on a workload of N vectors
(default 2^27, the benchmark size), checks that all configurations produce bit-identical
codes, and writes the fastest one as a tuning cache:

    axpy <f64|f32> block=<B> vpt=<V> nt=<T>
    batch ua=<A> ud=<D> un=<N>

The library applies the file named by $VC_TUNE_CACHE on first use, and
``vcx_load_tuning(path)`` applies any cache explicitly.

Usage (on the GPU):  python -m paper_2003_02633_amd.tune [--n N] [--out FILE] [--precision f64|f32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "mi355x_axpy.txt")
CONFIGS = [(b, v, t) for b in (128, 256, 512) for v in (2, 4, 8) for t in (1, 0) if v < 8 or b >= 256]


def _settle(torch, fn, ms: float):
    """back-to-back untimed calls for `ms` of wall time: the GPU clocks drop within milliseconds
    of idle and take tens of milliseconds of load to come back, so each configuration is timed
    only after its own warm-up by time"""
    import time

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()


def sweep(n: int = 1 << 27, precision: str = "f64", steps: int = 20, settle_ms: float = 150.0, log=print):
    import torch

    import paper_2003_02633_amd as vc
    from paper_2003_02633_amd import inputs

    c = vc.codec(precision=precision)
    a = vc.vc_encode(c, inputs.sphere_loguniform_torch(n, 0))
    b = vc.vc_encode(c, inputs.sphere_loguniform_torch(n, 1))
    out = torch.empty_like(a)
    ref = None
    results = []
    saved = vc.get_stream_config(precision)
    try:
        for (blk, vpt, nt) in CONFIGS:
            vc.set_stream_config(blk, vpt, nt, precision)
            _settle(torch, lambda: vc.vc_axpy(c, 0.7, a, b, out), settle_ms)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                vc.vc_axpy(c, 0.7, a, b, out)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            chk = out[:: max(1, n // (1 << 20))].clone()
            if ref is None:
                ref = chk
            same = bool(torch.equal(chk, ref))
            results.append({"block": blk, "vpt": vpt, "nt": nt, "ms": ms, "gvecs": n / ms / 1e6, "identical": same})
            log(f"[tune] block={blk} vpt={vpt} nt={nt}: {ms:.4f} ms  {n / ms / 1e6:.1f} Gvec/s  identical={same}")
    finally:
        vc.set_stream_config(*saved, precision)
    if not all(r["identical"] for r in results):
        raise RuntimeError("launch configurations disagree")
    return results


BATCH_CONFIGS = [(ua, ud, un) for ua in (1, 2) for ud in (2, 4, 8) for un in (4, 8, 16)]
BATCH_BYTES = {"axpy": 24, "dot": 16, "norm2": 8, "encode": 20}


def sweep_batch(precision: str = "f64", steps: int = 20, settle_ms: float = 150.0, log=print):
    """every tile shape on the 64-segment plan of the benchmark (lengths floor(10^U[3, 7]),
    seed 3, a shuffled round robin of axpy / dot / norm2 / encode); the axpy and encode codes
    must be bit-identical across shapes (the reductions' order differs)"""
    import torch

    import paper_2003_02633_amd as vc
    from paper_2003_02633_amd import inputs

    c = vc.codec(precision=precision)
    lengths, ops = inputs.segments(nseg=64, seed=3, lo_exp=3.0, hi_exp=7.0)
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    segs, algo = [], 0.0
    for n, op in zip(lengths, ops):
        n = int(n)
        x = torch.randn((n, 3), generator=g, dtype=torch.float32, device="cuda")
        if op == "encode":
            segs.append({"op": op, "n": n, "a": x, "out": torch.empty(n, dtype=torch.int64, device="cuda")})
        else:
            a = vc.vc_encode(c, x)
            b = vc.vc_encode(c, torch.randn((n, 3), generator=g, dtype=torch.float32, device="cuda")) \
                if op in ("axpy", "dot") else None
            out = torch.empty(n, dtype=torch.int64, device="cuda") if op == "axpy" else \
                torch.empty(1, dtype=torch.float32, device="cuda")
            segs.append({"op": op, "n": n, "a": a, "b": b, "out": out, "alpha": 0.7})
        algo += BATCH_BYTES[op] * n
    saved = vc.get_batch_config()
    results, ref = [], None
    try:
        for cfg in BATCH_CONFIGS:
            vc.set_batch_config(*cfg)
            plan = vc.BatchPlan(c, segs)
            _settle(torch, plan.run, settle_ms)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                plan.run()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            codes = [s["out"][:: max(1, s["n"] // 4096)].clone() for s in segs if s["op"] in ("axpy", "encode")]
            if ref is None:
                ref = codes
            same = all(bool(torch.equal(x, y)) for x, y in zip(codes, ref))
            plan.close()
            results.append({"ua": cfg[0], "ud": cfg[1], "un": cfg[2], "ms": ms, "GBs": algo / (ms * 1e-3) / 1e9,
                            "identical": same})
            log(f"[tune] batch ua={cfg[0]} ud={cfg[1]} un={cfg[2]}: {ms * 1e3:.1f} us  "
                f"{algo / (ms * 1e-3) / 1e9:.0f} GB/s  identical={same}")
    finally:
        vc.set_batch_config(*saved)
    if not all(r["identical"] for r in results):
        raise RuntimeError("batch tile shapes disagree")
    return results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1 << 27)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--json", default=None, help="also write all timings here")
    args = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)
    res = sweep(args.n, args.precision, log=log)
    best = min(res, key=lambda r: r["ms"])
    bres = sweep_batch(args.precision, log=log)
    bbest = min(bres, key=lambda r: r["ms"])
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        f.write(f"# compressed axpy launch configuration, N={args.n}, encoder {args.precision}, "
                f"{best['gvecs']:.1f} Gvec/s\n")
        f.write(f"axpy {args.precision} block={best['block']} vpt={best['vpt']} nt={best['nt']}\n")
        f.write(f"# batch tile shape, 64-segment plan, {bbest['GBs']:.0f} GB/s\n")
        f.write(f"batch ua={bbest['ua']} ud={bbest['ud']} un={bbest['un']}\n")
    if args.json:
        with open(args.json, "w") as f:
            json.dump({"n": args.n, "precision": args.precision, "results": res, "best": best,
                       "batch_results": bres, "batch_best": bbest}, f, indent=1)
    print(json.dumps({"best": best, "batch_best": bbest}), flush=True)


if __name__ == "__main__":
    main()
