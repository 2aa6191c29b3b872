#!/usr/bin/env python3
"""Benchmark of the compressed 3-vector axpy on one MI355X.

Workload (one "step" = one pass of the whole hot path = one launch of the fused
decode-FMA-encode kernel): c = alpha*a + b on N = 2^27 compressed 3-vectors
(<0,7,22>-17-18 codes, 1 GiB per operand), directions uniform on S^2, magnitudes
log-uniform on [1e-6, 1e6], alpha = 0.7.  Inputs are generated and encoded on the
GPU before timing, so they are resident in HBM.  Before the W warm-up steps the same
launch runs untimed for 200 ms of wall time (the GPU clocks take tens of milliseconds of
load to ramp); then exactly K steps are timed with HIP events.

Prints one JSON line: metric/value (Gvec/s of the compressed axpy), the HBM
roofline of that kernel, the CPU oracle timed on the host on a bounded sample, and
side-by-side figures: uncompressed FP32 / BF16 / FP16 axpy on the same GPU, a copy
kernel (attainable bandwidth), encode/decode/dot/norm2, and the codec variants.

Usage: python bench.py [--steps K] [--warmup W] [--n N] [--quick] [--no-cpu]
       python bench.py --pmc-run     (launch copy + axpy once each, for rocprofv3 --pmc)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E spec
ALPHA = 0.699999988079071      # float32(0.7)
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "axpy_n2p27_traffic.txt")
PROFILE_VALU = os.path.join(ROOT, "profiles", "axpy_n2p27_valu.txt")
KERNEL_SOURCES = ["include/vc_device.hpp", "paper_2003_02633_amd/csrc/vc_stream.hip",
                  "include/vc_coeffs.inc"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _code_only(text: str) -> str:
    """C++ source without its comments and blank space: what the compiler sees"""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_hash() -> str:
    """hash of the axpy kernel's sources (comments and layout ignored): the counters in profiles/
    count for the current build only while it matches"""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def _read_profile(path: str, n: int):
    """key = value lines of a committed rocprofv3 summary, if it was taken on the current kernel
    sources and this N; otherwise None."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_hash") != kernel_hash():
        return None
    if "n_vectors" in kv and int(kv["n_vectors"]) != n:
        return None
    return kv


def read_traffic(n: int):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary (FETCH_SIZE + WRITE_SIZE,
    calibrated on a copy kernel), or None when the kernel changed since it was taken."""
    kv = _read_profile(PROFILE_TRAFFIC, n)
    try:
        return float(kv["traffic_bytes_per_launch"]) if kv else None
    except (KeyError, ValueError):
        return None


def read_valu(n: int):
    """VALU figures of the same kernel (SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU), or None."""
    kv = _read_profile(PROFILE_VALU, n)
    try:
        return {"valu_instr_per_vector": float(kv["valu_instr_per_vector"]),
                "valu_busy_frac": float(kv["valu_busy_frac"])} if kv else None
    except (KeyError, ValueError):
        return None


# VALU issue ceiling of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions per second
# (a wave64 instruction occupies a SIMD16 for 4 cycles; packed FP32 is compiled out)
VALU_PEAK_LANE_INSTR_PER_S = 256 * 4 * 16 * 2.4e9


def valu_view(v, n: int, ms: float):
    """The ALU side of the roofline: the profiled VALU instructions per vector times the vectors
    per second of this run, against the issue ceiling (busy fraction from the same profile)."""
    if not v:
        return None
    rate = v["valu_instr_per_vector"] * n / (ms * 1e-3)
    return dict(v, achieved_lane_instr_per_s=rate, peak_lane_instr_per_s=VALU_PEAK_LANE_INSTR_PER_S,
                issue_frac=rate / VALU_PEAK_LANE_INSTR_PER_S)


# Side-by-side timings warm up by time, not count: the clocks drop within milliseconds of idle
# (host-side set-up between measurements) and take tens of milliseconds of load to come back up.
WX = None
SETTLE_MS = 200.0


def settle(torch, fn, ms: float = None):
    """back-to-back untimed calls of fn(), checked every 8, until `ms` (SETTLE_MS) of wall time
    has passed: brings the GPU clocks up before anything is timed"""
    import time

    limit = SETTLE_MS if ms is None else ms
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < limit:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()


# codec variants of the axpy timed beside the headline codec (and launched once each by --pmc-run
# variants): fractional split (§2.4), companding (§2.5), the truncating magnitude (§2.3), and the
# single-precision encoder's companding (level-boundary tables)
VARIANTS = (("frac_P2^16", {"mode": "frac", "P": 1 << 16}),
            ("frac_P163840", {"mode": "frac", "P": 163840}),
            ("frac_P2^18", {"mode": "frac", "P": 1 << 18}),
            ("tanh_g0.5", {"mode": "tanh", "gamma": 0.5}),
            ("cos", {"mode": "cos"}),
            ("trunc_magnitude", {"mag_round": "trunc"}),
            ("tanh_g0.5_f32encoder", {"mode": "tanh", "gamma": 0.5, "precision": "f32"}),
            ("cos_f32encoder", {"mode": "cos", "precision": "f32"}))


def timed(torch, fn, steps: int, warmup) -> float:
    """Average milliseconds per call of fn() (all work on torch's current stream), after `warmup`
    untimed calls, or (warmup None) untimed calls for at least SETTLE_MS."""
    import time

    if warmup is None:
        settle(torch, fn)
    else:
        for _ in range(warmup):
            fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def host_info(torch) -> dict:
    """the machine the record comes from: CPU model, cores this process may use, GPU name"""
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "cores_available": cores, "gpu": torch.cuda.get_device_name(0)}


def cpu_baseline(torch, wa_dev, wb_dev, target_s: float = 15.0):
    """Time the oracle's compressed axpy on the host, all cores, on a bounded sample: the first n
    vectors of the benchmark operands (at most 2^25, 0.75 GiB of codes), passed over repeatedly
    until about target_s seconds of CPU work have been timed."""
    import math

    import numpy as np

    import oracle as O

    co = O.codec()
    threads = O.max_threads()
    n_cal = 1 << 18
    wa = wa_dev[:n_cal].cpu().numpy().view(np.uint64)
    wb = wb_dev[:n_cal].cpu().numpy().view(np.uint64)
    t = time.perf_counter()
    O.axpy(co, ALPHA, wa, wb, threads)
    rate = n_cal / max(time.perf_counter() - t, 1e-6)
    n = int(min(wa_dev.numel(), 1 << 25, max(n_cal, rate * target_s)))
    reps = max(1, math.ceil(rate * target_s / n))
    wa = wa_dev[:n].cpu().numpy().view(np.uint64)
    wb = wb_dev[:n].cpu().numpy().view(np.uint64)
    t = time.perf_counter()
    for _ in range(reps):
        O.axpy(co, ALPHA, wa, wb, threads)
    dt = time.perf_counter() - t
    return {"value": reps * n / dt / 1e9, "unit": "Gvec/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} vectors of the benchmark operands, {reps} passes; oracle compressed axpy "
                      f"(decode both, single-rounded FMA, encode), OpenMP over {threads} threads, {dt:.1f} s"}


def sample_error(torch, vc, c, wa, wb, wc, nsample: int = 1 << 20, seed: int = 5):
    """Max normalised error |decode(c) - (alpha a_hat + b_hat)| / |alpha a_hat + b_hat| over a seeded
    sample: the three codes decoded by the library (single precision; its decode error, under
    3e-7 |x| per component, is a few per cent of the codec's), the sum and the error norms in FP64
    on the host."""
    import numpy as np

    n = wa.numel()
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    idx = torch.randint(0, n, (min(nsample, n),), generator=g).to(wa.device)
    A = vc.vc_decode(c, wa[idx].contiguous()).double().cpu().numpy()
    B = vc.vc_decode(c, wb[idx].contiguous()).double().cpu().numpy()
    got = vc.vc_decode(c, wc[idx].contiguous()).double().cpu().numpy()
    c64 = float(ALPHA) * A + B
    nrm = np.linalg.norm(c64, axis=1)
    scale = float(ALPHA) * np.linalg.norm(A, axis=1) + np.linalg.norm(B, axis=1)
    ok = nrm > 0
    err = np.linalg.norm(got - c64, axis=1)
    return {"max_rel_err": float((err[ok] / nrm[ok]).max()),
            "mean_rel_err": float((err[ok] / nrm[ok]).mean()),
            "max_err_over_operand_scale": float((err[ok] / scale[ok]).max()),
            "sample": int(idx.numel()), "decode": "library (single precision)"}


def bench_apply(torch, vc, inputs, k: int):
    """Fused decode + operator apply: 200,000 p = 4 hexahedral elements (125 solution points
    each) of a Taylor-Green velocity field, operator 150 x 125 with entries U[-1, 1]."""
    import numpy as np

    E, rows, cols = 200_000, 150, 125
    c = vc.codec()
    vel = inputs.tgv_elements(E, 4, seed=0)
    U = vc.vc_encode(c, torch.from_numpy(vel.reshape(-1, 3)).to("cuda"))
    del vel
    M = torch.from_numpy(inputs.uniform_matrix(rows, cols, 2)).to("cuda")
    out = torch.empty((E, rows, 3), dtype=torch.float32, device="cuda")
    # the default cores (bf16 with three-part splits, FP32-accurate), then the FP32 cores
    ms = timed(torch, lambda: vc.vc_fused_apply(c, M, U.view(E, cols), out), k, WX)
    vc.set_apply_mode("fp32")
    try:
        ms32 = timed(torch, lambda: vc.vc_fused_apply(c, M, U.view(E, cols), out), k, WX)
    finally:
        vc.set_apply_mode("auto")
    flop = 2.0 * rows * cols * 3 * E
    byts = 8.0 * cols * E + 12.0 * rows * E
    # issued matrix work: the operator padded to 16-row blocks and 32-wide K steps, six bf16
    # part products per FP32 product
    flop_bf = 6 * 2.0 * (16 * ((rows + 15) // 16)) * (32 * ((cols + 31) // 32)) * 3 * E
    del U, M, out
    return {"elements": E, "rows": rows, "cols": cols, "ms": ms, "cores": "bf16, three-part split (FP32 accuracy)",
            "TFLOPs": flop / (ms * 1e-3) / 1e12, "frac_fp32_mfma_peak": flop / (ms * 1e-3) / 157.3e12,
            "bf16_issued_TFLOPs": flop_bf / (ms * 1e-3) / 1e12,
            "frac_bf16_mfma_peak": flop_bf / (ms * 1e-3) / 2.5e15,
            "GBs": byts / (ms * 1e-3) / 1e9, "bound": "mfma", "bf16_mfma_floor_us": flop_bf / 2.5e15 * 1e6,
            "fp32_cores": {"ms": ms32, "TFLOPs": flop / (ms32 * 1e-3) / 1e12, "mfma_floor_us": flop / 157.3e12 * 1e6},
            "hbm_floor_us": byts / 8e12 * 1e6}


ANISO_CODECS = (("plain", {}), ("tanh_g0.5", {"mode": "tanh", "gamma": 0.5}), ("cos", {"mode": "cos"}),
                ("frac_P2^16", {"mode": "frac", "P": 1 << 16}), ("frac_P163840", {"mode": "frac", "P": 163840}),
                ("frac_P2^18", {"mode": "frac", "P": 1 << 18}))


def _compact_hist(counts):
    """nonzero span of a histogram: [index of the first nonzero bin, counts up to the last]"""
    nz = [i for i, v in enumerate(counts) if v]
    if not nz:
        return [0, []]
    return [nz[0], [int(v) for v in counts[nz[0]:nz[-1] + 1]]]


def bench_anisotropy(torch, vc, inputs, n: int = 1 << 25):
    """Codec error statistics on the GPU (FP64 error norms) for von Mises-Fisher directions,
    kappa in {1, 10, 100, 1000}, mean +z and (1,1,1)/sqrt(3), lognormal magnitudes, for every
    codec variant: mean / max / rms of the three error measures and the histograms of the angular
    and magnitude errors (bins 10^(-12 + i/10); bin 0 counts errors below 1e-12)."""
    import numpy as np

    edges_np = 10.0 ** (-12.0 + np.arange(101, dtype=np.float64) / 10)
    edges = torch.from_numpy(edges_np).to("cuda")
    codecs = [(name, vc.codec(**kw)) for name, kw in ANISO_CODECS]
    res = {"n": n, "edges": "10^(-12 + i/10), i = 0..100", "kinds": ["|x_hat-x|/|x|", "angle(x, x_hat)", "|r_hat-r|/r"],
           "hist_format": "[first nonzero bin, counts...] of the angle and magnitude histograms",
           "codecs": {name: {} for name, _ in codecs}}
    for kappa in (1.0, 10.0, 100.0, 1000.0):
        for mname, mean in (("z", (0.0, 0.0, 1.0)), ("diag", (1.0, 1.0, 1.0))):
            x = inputs.vmf_torch(n, kappa, mean, seed=int(kappa) + (0 if mname == "z" else 7))
            torch.cuda.synchronize()
            for name, c in codecs:
                t0 = time.perf_counter()
                h, ex, st = vc.error_hist(c, x, edges)
                ms = (time.perf_counter() - t0) * 1e3
                m = int(h[0].sum())
                st = st.numpy()
                res["codecs"][name][f"kappa{int(kappa)}_{mname}"] = {
                    "mean": [float(v) for v in st[:, 0] / m], "max": [float(v) for v in st[:, 2]],
                    "rms": [float(v) for v in np.sqrt(st[:, 1] / m)], "excluded": ex, "ms": round(ms, 3),
                    "hist_angle": _compact_hist(h[1].tolist()), "hist_magnitude": _compact_hist(h[2].tolist())}
            del x
    return res


def storage_error(torch, vc, c_codec, a32, b32, wc, outs, nsample: int = 1 << 20, seed: int = 6):
    """Error of each storage format's axpy result against the FP64 axpy of the float32 inputs
    (alpha a + b), over a seeded sample: normalised vector error |c_hat - c|/|c|, the angle between
    c_hat and c, and |(|c_hat| - |c|)|/|c|; mean and max, computed in FP64 on the host.  `outs` maps
    a format to its result (float tensor [N, 3] or [N, 4]); the codec's result is decoded by the
    library (single precision).  Non-finite results (FP16 overflow) are counted and left out of
    the statistics."""
    import numpy as np

    n = a32.shape[0]
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    idx = torch.randint(0, n, (min(nsample, n),), generator=g).to(a32.device)
    a = a32[idx].double().cpu().numpy()
    b = b32[idx].double().cpu().numpy()
    c = float(ALPHA) * a + b
    nrm = np.linalg.norm(c, axis=1)
    res = {"sample": int(idx.numel()), "truth": "alpha a + b in FP64 from the float32 inputs"}
    got = {"codec": vc.vc_decode(c_codec, wc[idx].contiguous()).double().cpu().numpy()}
    for k, t in outs.items():
        got[k] = t[idx][:, :3].double().cpu().numpy()
    for k, v in got.items():
        fin = np.isfinite(v).all(axis=1) & (nrm > 0)
        e = np.linalg.norm(v - c, axis=1)[fin] / nrm[fin]
        vn = np.linalg.norm(v[fin], axis=1)
        cosang = np.clip(np.einsum("ij,ij->i", v[fin], c[fin]) / np.maximum(vn * nrm[fin], 1e-300), -1.0, 1.0)
        ang = np.arccos(cosang)
        mag = np.abs(vn - nrm[fin]) / nrm[fin]
        res[k] = {"vector_mean": float(e.mean()), "vector_max": float(e.max()), "angle_mean": float(ang.mean()),
                  "angle_max": float(ang.max()), "magnitude_mean": float(mag.mean()), "magnitude_max": float(mag.max()),
                  "nonfinite_fraction": float(1.0 - fin.mean())}
    return res


def bench_flux_div(torch, vc, inputs, k: int, grid=(64, 64, 64), p: int = 4):
    """Divergence of the Taylor-Green Euler flux (step 10 of the FR right-hand side, Alg.
    fr_fdiv_comp) on a grid of p = 4 hexahedra: compressed flux codes vs the same kernel on
    float32 fluxes.  Algorithmic bytes per element: 125 x 5 codes (5,000 B) or 125 x 5 x 3 floats
    (7,500 B) in, 125 x 5 floats (2,500 B) out -- the 9.77 KiB and ratio 0.75 of Table (mem_usage),
    step 10, k = 4."""
    import math

    import numpy as np

    n = grid[0] * grid[1] * grid[2]
    q = p + 1
    c = vc.codec()
    d = torch.from_numpy(np.stack([inputs.fr_derivative_1d(p, 2 * math.pi / g) for g in grid]).astype(np.float32)).to("cuda")
    F = inputs.euler_flux_tgv(n, p, grid=grid, device="cuda")
    W = vc.vc_encode(c, F.view(-1, 3)).view(n, q ** 3, 5)
    out = torch.empty((n, q ** 3, 5), dtype=torch.float32, device="cuda")
    # alternate the two kernels over several rounds and keep the medians (the pair shares the GPU
    # with nothing else, but single short timings of either vary by a few per cent)
    mc, mu = [], []
    for _ in range(5):
        mc.append(timed(torch, lambda: vc.vc_flux_div_tp(c, d, W, out), k, WX))
        mu.append(timed(torch, lambda: vc.vcb_flux_div_tp_f32(d, F, out), k, WX))
    ms_c, ms_u = float(np.median(mc)), float(np.median(mu))
    bc, bu = 7500.0 * n, 10000.0 * n
    del F, W, out
    return {"elements": n, "p": p, "equations": 5, "compressed_ms": ms_c, "uncompressed_ms": ms_u,
            "speedup": ms_u / ms_c, "ideal_speedup_bytes": bu / bc,
            "compressed_GBs": bc / (ms_c * 1e-3) / 1e9, "uncompressed_GBs": bu / (ms_u * 1e-3) / 1e9}


def bench_gather(torch, vc, k: int, n: int = 1 << 26):
    """Indexed decode out[i] = decode(codes[idx[i]]) vs the float32 gather of the same vectors, for
    the identity, face-sized blocks (25 consecutive points, the flux points of one face of a p = 4
    hexahedron) in shuffled order, and a random permutation."""
    c = vc.codec()
    g = torch.Generator(device="cuda")
    g.manual_seed(41)
    x = torch.randn((n, 3), generator=g, dtype=torch.float32, device="cuda")
    w = vc.vc_encode(c, x)
    out = torch.empty_like(x)
    nb = n // 25
    blocks = torch.randperm(nb, generator=g, device="cuda").to(torch.int32)
    face = (blocks[:, None] * 25 + torch.arange(25, device="cuda", dtype=torch.int32)[None]).reshape(-1)
    pats = {"identity": torch.arange(n, device="cuda", dtype=torch.int32),
            "face_blocks": torch.cat([face, torch.arange(nb * 25, n, device="cuda", dtype=torch.int32)]),
            "random": torch.randperm(n, generator=g, device="cuda").to(torch.int32)}
    res = {"n": n}
    for name, idx in pats.items():
        ms_c = timed(torch, lambda: vc.vc_gather_decode(c, w, idx, out), k, WX)
        ms_f = timed(torch, lambda: vc.vcb_gather_f32(x, idx, out), k, WX)
        res[name] = {"compressed_ms": ms_c, "float_ms": ms_f, "speedup": ms_f / ms_c,
                     "compressed_gvecs": n / (ms_c * 1e-3) / 1e9}
    del x, w, out, pats
    return res


BYTES_PER_VEC = {"axpy": 24, "dot": 16, "norm2": 8, "encode": 20}


def bench_batch(torch, vc, inputs, k: int, precision: str):
    """64 segments of lengths floor(10^U[3, 7]) (seed 3), a shuffled round robin of axpy (alpha
    0.7), dot, norm2 and encode: one persistent graph-replayed kernel vs separate launches vs
    separate launches captured in one graph."""
    lengths, ops = inputs.segments(nseg=64, seed=3, lo_exp=3.0, hi_exp=7.0)
    c = vc.codec(precision=precision)
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
            segs.append({"op": op, "n": n, "a": a, "b": b, "out": out, "alpha": ALPHA})
        del x
        algo += BYTES_PER_VEC[op] * n
    torch.cuda.synchronize()
    plan = vc.BatchPlan(c, segs)
    tiles, grid = plan.info()
    res = {"segments": len(segs), "vectors": int(sum(int(n) for n in lengths)), "tiles": tiles, "grid": grid,
           "algorithmic_bytes": algo}
    for name, fn in (("persistent_graph", plan.run), ("separate_launches", plan.run_separate),
                     ("separate_launches_graph", plan.run_separate_graph)):
        ms = timed(torch, fn, k, WX)
        res[name] = {"ms": ms, "GBs": algo / (ms * 1e-3) / 1e9}
    plan.close()
    del segs
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=50,
                    help="untimed launches first; the clocks take tens of milliseconds of load to settle")
    ap.add_argument("--n", type=int, default=1 << 27)
    ap.add_argument("--quick", action="store_true", help="skip the side-by-side extras")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--pmc-run", nargs="?", const="axpy", default=None, choices=["axpy", "variants", "apply", "fdiv", "gather", "all"],
                    help="launch the copy kernel (counter calibration) and the selected kernels once "
                         "(axpy by default) for rocprofv3 --pmc")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"],
                    help="encoder arithmetic of the headline codec")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (--gpus {args.gpus} requested); "
              "the method is data-parallel over independent vectors (each GPU would take a contiguous "
              "range), but no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2003_02633_amd as vc
    from paper_2003_02633_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    vc.lib()
    N = args.n
    dev = torch.device("cuda:0")
    c = vc.codec(precision=args.precision)
    log(f"generating inputs N={N}")
    a32 = inputs.sphere_loguniform_torch(N, 0, dev)
    b32 = inputs.sphere_loguniform_torch(N, 1, dev)
    wa = vc.vc_encode(c, a32)
    wb = vc.vc_encode(c, b32)
    wc = torch.empty_like(wa)
    torch.cuda.synchronize()

    if args.pmc_run:
        # the copy kernel over 12 N bytes each way (calibration of the byte counters), then one
        # launch of each selected kernel: the axpy, the fused apply, the flux divergence
        # (compressed and float32) or the indexed gathers
        cp_src = torch.empty(N * 3, dtype=torch.float32, device=dev)
        cp_src.copy_(a32.view(-1))
        cp_dst = torch.empty_like(cp_src)
        vc.vcb_copy(cp_src, cp_dst)
        torch.cuda.synchronize()
        del cp_src, cp_dst
        if args.pmc_run in ("axpy", "all"):
            vc.vc_axpy(c, ALPHA, wa, wb, wc)
            torch.cuda.synchronize()
        if args.pmc_run in ("variants", "all"):
            # the headline codec with the other encoder precision, then each codec variant
            other = "f32" if args.precision == "f64" else "f64"
            vc.vc_axpy(vc.codec(precision=other), ALPHA, wa, wb, wc)
            for _name, kw in VARIANTS:
                cv = vc.codec(**dict({"precision": args.precision}, **kw))
                va_, vb_ = vc.vc_encode(cv, a32), vc.vc_encode(cv, b32)
                vc.vc_axpy(cv, ALPHA, va_, vb_, wc)
                torch.cuda.synchronize()
                del va_, vb_
        if args.pmc_run in ("apply", "all"):
            bench_apply(torch, vc, inputs, 1)
        if args.pmc_run in ("fdiv", "all"):
            bench_flux_div(torch, vc, inputs, 1)
        if args.pmc_run in ("gather", "all"):
            bench_gather(torch, vc, 1)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_run": args.pmc_run, "n_vectors": N, "copy_bytes_each_way": N * 12,
                          "kernel_hash": kernel_hash()}), flush=True)
        return

    log(f"timing compressed axpy: clock settle {SETTLE_MS:.0f} ms, warmup {args.warmup}, steps {args.steps}")
    step = lambda: vc.vc_axpy(c, ALPHA, wa, wb, wc)
    # the clocks ramp over tens of milliseconds of load: untimed launches for SETTLE_MS of wall
    # time first, then the W warm-up launches, then exactly the K timed ones
    settle(torch, step)
    ms = timed(torch, step, args.steps, args.warmup)
    gvecs = N / (ms * 1e-3) / 1e9
    achieved = 24.0 * N / (ms * 1e-3) / 1e9
    log(f"compressed axpy: {ms:.3f} ms/step, {gvecs:.2f} Gvec/s, {achieved:.0f} GB/s")

    err = sample_error(torch, vc, c, wa, wb, wc)
    log(f"sample error: {err}")

    extras = {"host": host_info(torch)}
    if not args.quick:
        k = max(3, args.steps // 4)
        # uncompressed FP32 axpy over the same vectors (36 B/vec)
        c32 = torch.empty_like(a32)
        ms_f32 = timed(torch, lambda: vc.vcb_axpy_f32(ALPHA, a32, b32, c32), k, WX)
        extras["fp32_axpy"] = {"gvecs": N / (ms_f32 * 1e-3) / 1e9, "ms": ms_f32,
                               "GBs": 36.0 * N / (ms_f32 * 1e-3) / 1e9}
        extras["speedup_vs_fp32"] = ms_f32 / ms
        log(f"fp32 axpy: {ms_f32:.3f} ms -> speedup {ms_f32 / ms:.3f}")
        stored = {"fp32": c32}
        # bf16 / fp16 storage padded to 4 x 16 bit (8 B/vec, the bytes of a code)
        for kind, dt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
            ha = torch.zeros((N, 4), dtype=dt, device=dev)
            hb = torch.zeros((N, 4), dtype=dt, device=dev)
            ha[:, :3] = a32
            hb[:, :3] = b32
            hc = torch.empty_like(ha)
            iv = (ha.view(torch.int16), hb.view(torch.int16), hc.view(torch.int16))
            ms_h = timed(torch, lambda: vc.vcb_axpy_h4(kind, ALPHA, *iv), k, WX)
            rec = {"gvecs": N / (ms_h * 1e-3) / 1e9, "ms": ms_h, "GBs": 24.0 * N / (ms_h * 1e-3) / 1e9}
            if kind == "f16":
                big = (a32.abs() > 65504).any(dim=1).sum().item()
                small = ((a32.abs() < 6.1e-5) & (a32 != 0)).any(dim=1).sum().item()
                rec["overflow_fraction"] = big / N
                rec["subnormal_fraction"] = small / N
            extras[f"{kind}x4_axpy"] = rec
            log(f"{kind}x4 axpy: {ms_h:.3f} ms")
            stored[f"{kind}x4"] = hc
            del ha, hb, iv
        # storage error of each format's axpy against FP64 (sampled, on the host)
        extras["storage_error_vs_fp64"] = storage_error(torch, vc, c, a32, b32, wc, stored)
        log(f"storage error: { {k: v['vector_max'] for k, v in extras['storage_error_vs_fp64'].items() if isinstance(v, dict)} }")
        del stored, c32
        # attainable bandwidth: copy of 2 x 12 N bytes
        src = a32.view(-1)
        dst = torch.empty_like(src)
        ms_cp = timed(torch, lambda: vc.vcb_copy(src, dst), k, WX)
        copy_gbs = 2.0 * 12 * N / (ms_cp * 1e-3) / 1e9
        extras["copy"] = {"GBs": copy_gbs, "ms": ms_cp, "bytes": 24 * N}
        extras["axpy_frac_of_copy_bw"] = achieved / copy_gbs
        del dst
        # encode / decode / reductions of the same data
        ms_enc = timed(torch, lambda: vc.vc_encode(c, a32, wc), k, WX)
        xyz = torch.empty_like(a32)
        ms_dec = timed(torch, lambda: vc.vc_decode(c, wa, xyz), k, WX)
        del xyz
        out1 = torch.empty(1, dtype=torch.float32, device=dev)
        ms_dot = timed(torch, lambda: vc.vc_dot(c, wa, wb, out1), k, WX)
        ms_n2 = timed(torch, lambda: vc.vc_norm2(c, wa, out1), k, WX)
        extras["encode"] = {"gvecs": N / (ms_enc * 1e-3) / 1e9, "GBs": 20.0 * N / (ms_enc * 1e-3) / 1e9}
        extras["decode"] = {"gvecs": N / (ms_dec * 1e-3) / 1e9, "GBs": 20.0 * N / (ms_dec * 1e-3) / 1e9}
        extras["dot"] = {"gvecs": N / (ms_dot * 1e-3) / 1e9, "GBs": 16.0 * N / (ms_dot * 1e-3) / 1e9}
        extras["norm2"] = {"gvecs": N / (ms_n2 * 1e-3) / 1e9, "GBs": 8.0 * N / (ms_n2 * 1e-3) / 1e9}
        log(f"encode {ms_enc:.3f} ms, decode {ms_dec:.3f} ms, dot {ms_dot:.3f} ms, norm2 {ms_n2:.3f} ms")
        # the other encoder precision on the same operands
        other = "f32" if args.precision == "f64" else "f64"
        co_ = vc.codec(precision=other)
        ms_o = timed(torch, lambda: vc.vc_axpy(co_, ALPHA, wa, wb, wc), k, WX)
        extras[f"axpy_encoder_{other}"] = {"gvecs": N / (ms_o * 1e-3) / 1e9, "ms": ms_o,
                                           "GBs": 24.0 * N / (ms_o * 1e-3) / 1e9,
                                           "speedup_vs_fp32": extras["fp32_axpy"]["ms"] / ms_o}
        log(f"axpy with {other} encoder: {ms_o:.3f} ms")
        # codec variants of the same axpy
        var = {}
        for name, kw in VARIANTS:
            kw = dict({"precision": args.precision}, **kw)
            cv = vc.codec(**kw)
            va_ = vc.vc_encode(cv, a32)
            vb_ = vc.vc_encode(cv, b32)
            msv = timed(torch, lambda: vc.vc_axpy(cv, ALPHA, va_, vb_, wc), k, WX)
            var[name] = {"gvecs": N / (msv * 1e-3) / 1e9, "GBs": 24.0 * N / (msv * 1e-3) / 1e9}
            log(f"variant {name}: {msv:.3f} ms")
            del va_, vb_
        extras["variants_axpy"] = var
        log("fused apply (200,000 elements, 150 x 125)")
        extras["fused_apply"] = bench_apply(torch, vc, inputs, k)
        log(f"fused apply: {extras['fused_apply']}")
        log("flux divergence (TGV Euler flux, 64^3 p=4 hexahedra)")
        extras["flux_div"] = bench_flux_div(torch, vc, inputs, k)
        log(f"flux divergence: {extras['flux_div']}")
        log("indexed gather (2^26 vectors)")
        extras["gather"] = bench_gather(torch, vc, k)
        log(f"gather: {extras['gather']}")
        log("anisotropy error statistics (vMF, 2^25 vectors each)")
        extras["anisotropy"] = bench_anisotropy(torch, vc, inputs)
        log("anisotropy (mean vector error, kappa 1 / 1000 about +z): " + ", ".join(
            f"{name}: {cases['kappa1_z']['mean'][0]:.3e} / {cases['kappa1000_z']['mean'][0]:.3e}"
            for name, cases in extras["anisotropy"]["codecs"].items()))
        log("batched segments (64 segments, 10^3..10^7 vectors)")
        extras["batch"] = bench_batch(torch, vc, inputs, k, args.precision)
        log(f"batch: {extras['batch']}")
        extras["paper_titanv_speedup_context"] = 1.5
        torch.cuda.synchronize()
        # restore the plain result for consistency
        vc.vc_axpy(c, ALPHA, wa, wb, wc)

    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(torch, wa, wb)
        log(f"cpu oracle: {cpu}")

    rec = {
        "metric": "compressed vs FP32 axpy: Gvec/s, effective HBM GB/s (% peak), max rel err",
        "value": gvecs,
        "unit": "Gvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "compressed axpy c = 0.7 a + b, N = 2^27 3-vectors, <0,7,22>-17-18 codes, "
                               "directions uniform on S^2, |x| log-uniform [1e-6, 1e6]",
                   "n_vectors": N, "codec": "0,7,22-17-18 plain RNE", "alpha": ALPHA,
                   "encoder_precision": args.precision},
        "effective_GBs": achieved,
        "pct_hbm_peak": 100.0 * achieved / HBM_PEAK_GBS,
        "error": err,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": read_traffic(N),
                     "algorithmic_bytes_per_launch": 24 * N, "copy_GBs": extras.get("copy", {}).get("GBs"),
                     "valu": valu_view(read_valu(N), N, ms)},
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
