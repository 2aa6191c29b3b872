"""GPU parity of the batched persistent launch (vc_batch_plan_*) over a segment table.

Contract:
  * axpy segments: against the oracle, in the layered form of the single-call axpy: the codes
    follow the encode rule (bit-exact up to counted one-level differences inside the one-ulp
    window) on the single-precision sums alpha decode(a) + decode(b) of the same operands, and
    decoding them recovers the FP64 sum of the oracle's exact decodes within the codec bound;
  * encode segments: the encode rule against the oracle on the segment's own input;
  * both: also bit-identical to the single-call entry points (vc_axpy, vc_encode) on the same
    operands -- the persistent kernel runs the same per-vector codec;
  * dot / norm2 segments: within 4e-6 of sum |a||b| (resp. sum |a|^2) of the FP64 oracle;
    deterministic (two replays agree bit for bit); an empty segment gives exactly 0;
  * graph replays: every replay, with eager work in between, rewrites the same results;
  * the separate-launch paths (plain and graph-captured) agree with each other bit for bit.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import paper_2003_02633_amd as vc
from paper_2003_02633_amd import inputs
from tests.parity import classify, describe_bad

pytestmark = pytest.mark.gpu

ALPHA = float(np.float32(0.7))


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    vc.lib()
    return torch


def up(torch, arr, pad=0):
    """device copy of arr; with pad > 0 the data starts `pad` elements into the allocation
    (breaks 16-byte alignment and exercises the scalar path)"""
    arr = np.ascontiguousarray(arr)
    if arr.dtype == np.uint64:
        arr = arr.view(np.int64)
    t = torch.from_numpy(arr.reshape(-1)).to("cuda")
    if pad:
        big = torch.empty(t.numel() + pad, dtype=t.dtype, device="cuda")
        big[pad:] = t
        t = big[pad:]
    return t


def build_segments(torch, co, lengths, ops, pad_every=0):
    """device segments plus host copies of their operands"""
    segs, host = [], []
    for i, (n, op) in enumerate(zip(lengths, ops)):
        n = int(n)
        pad = 1 if (pad_every and i % pad_every == pad_every - 1) else 0
        if op == "encode":
            x = inputs.gaussian_with_edges(n - 11, 100 + i) if n >= 11 else inputs.gaussian(n, 100 + i)
            ta = up(torch, x, 3 * pad)
            out = torch.empty(max(n, 1), dtype=torch.int64, device="cuda")
            segs.append({"op": op, "n": n, "a": ta, "out": out})
            host.append({"x": x})
            continue
        wa = O.encode(co, inputs.gaussian(n, 200 + i))
        wb = O.encode(co, inputs.gaussian(n, 300 + i)) if op in ("axpy", "dot") else None
        ta = up(torch, wa, pad) if n else torch.empty(1, dtype=torch.int64, device="cuda")
        tb = (up(torch, wb, pad) if n else torch.empty(1, dtype=torch.int64, device="cuda")) \
            if wb is not None else None
        if op == "axpy":
            out = torch.empty(max(n, 1), dtype=torch.int64, device="cuda")
        else:
            out = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        segs.append({"op": op, "n": n, "a": ta, "b": tb, "out": out, "alpha": ALPHA})
        host.append({"wa": wa, "wb": wb})
    return segs, host


def expected_codes(torch, c, segs):
    """per axpy/encode segment: the single-call entry point's result, and for axpy segments the
    single-precision sums alpha decode(a) + decode(b) of the same operands (the verification
    variant of the axpy kernel writes them)"""
    exp, sums = {}, {}
    for i, s in enumerate(segs):
        if s["n"] == 0:
            continue
        if s["op"] == "axpy":
            exp[i] = vc.vc_axpy(c, ALPHA, s["a"], s["b"]).cpu()
            _, c32 = vc.vcx_axpy_dump(c, ALPHA, s["a"], s["b"])
            sums[i] = c32.cpu().numpy()
        elif s["op"] == "encode":
            exp[i] = vc.vc_encode(c, s["a"].view(-1, 3)).cpu()
    torch.cuda.synchronize()
    exp["sums"] = sums
    return exp


def check_codes_against_oracle(co, s, h, got, c32, label):
    """the oracle side of an axpy / encode segment's codes"""
    codes = got.numpy().view(np.uint64)
    if s["op"] == "encode":
        res = classify(co, h["x"], codes)
        assert res["other"] == 0, f"{label}: encode segment\n" + describe_bad(co, h["x"], codes, res)
        return
    res = classify(co, c32, codes)
    assert res["other"] == 0, f"{label}: axpy segment\n" + describe_bad(co, c32, codes, res)
    A64, B64 = O.decode64(co, h["wa"]), O.decode64(co, h["wb"])
    c64 = ALPHA * A64 + B64
    dec = O.decode64(co, codes)
    nrm = np.linalg.norm(c64, axis=1)
    scale = ALPHA * np.linalg.norm(A64, axis=1) + np.linalg.norm(B64, axis=1)
    ok = (nrm > 2.0 ** -70) & (nrm < 1e14)
    nt, npm = O.nmax(co)
    bound = (math.hypot(math.pi / nt, math.pi / (2 * npm)) + MAG_ERR[co.mag_round]) * nrm[ok] \
        + (4 * 2.0 ** -24 + 1e-6) * scale[ok]
    assert (np.linalg.norm(dec - c64, axis=1)[ok] <= bound).all(), f"{label}: axpy end-to-end bound"


# magnitude error of nearest-even at 23 bits, and of the paper's truncation (24 bits, one dropped)
MAG_ERR = {O.RNE: 2.0 ** -23, O.TRUNC: 2.0 ** -22 + 2.0 ** -24}


def check_results(torch, co, segs, host, exp, label, oracle_codes=True):
    torch.cuda.synchronize()
    red = {}
    for i, s in enumerate(segs):
        n = s["n"]
        if s["op"] in ("axpy", "encode"):
            if n == 0:
                continue
            got = s["out"][:n].cpu()
            assert torch.equal(got, exp[i]), f"{label}: segment {i} ({s['op']}, n={n}) differs"
            if oracle_codes:
                check_codes_against_oracle(co, s, host[i], got, exp["sums"].get(i), f"{label} segment {i}")
        else:
            v = float(s["out"].cpu()[0])
            red[i] = v
            if n == 0:
                assert v == 0.0, f"{label}: empty {s['op']} segment {i} gave {v}"
                continue
            if s["op"] == "dot":
                ref = O.dot(co, host[i]["wa"], host[i]["wb"])
                A, B = O.decode64(co, host[i]["wa"]), O.decode64(co, host[i]["wb"])
                scale = float((np.linalg.norm(A, axis=1) * np.linalg.norm(B, axis=1)).sum())
            else:
                ref = O.norm2(co, host[i]["wa"])
                scale = ref
            assert abs(v - ref) <= 4e-6 * scale, f"{label}: {s['op']} segment {i} n={n}: {v} vs {ref}"
    return red


def clobber(torch, segs):
    for s in segs:
        if s["op"] in ("axpy", "encode"):
            s["out"].fill_(-1)
        else:
            s["out"].fill_(float("nan"))


# edge segments: empty of every op, single vectors, and one vector either side of the tile sizes
EDGE_LENGTHS = [0, 0, 0, 0, 1, 1, 1, 1, 511, 512, 513, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097,
                8191, 8192, 8193, 8193]
EDGE_OPS = ["axpy", "dot", "norm2", "encode"] * 6


def expected_tiles(lengths, ops, cfg):
    """tiles of a plan: 512 ua vectors per axpy tile, 512 ud per dot, 512 un per norm2, 1024 per
    encode tile"""
    ua, ud, un = cfg
    size = {"axpy": 512 * ua, "dot": 512 * ud, "norm2": 512 * un, "encode": 1024}
    return sum((int(n) + size[op] - 1) // size[op] for n, op in zip(lengths, ops))


def test_batch_every_tile_shape(torch_dev):
    """the mixed segments under every tile shape the autotuner chooses from: codes bit-identical to
    the single-call entry points (and to the oracle's rule), reductions within the tolerance"""
    from paper_2003_02633_amd import tune
    torch = torch_dev
    lengths, ops = inputs.segments(nseg=24, seed=5, lo_exp=3.0, hi_exp=4.5)
    lengths, ops = list(lengths) + EDGE_LENGTHS, list(ops) + EDGE_OPS
    c, co = vc.codec(), O.codec()
    segs, host = build_segments(torch, co, lengths, ops, pad_every=7)
    exp = expected_codes(torch, c, segs)
    saved = vc.get_batch_config()
    try:
        for cfg in tune.BATCH_CONFIGS:
            say(f"case: batch tile shape {cfg}")
            vc.set_batch_config(*cfg)
            plan = vc.BatchPlan(c, segs)
            assert plan.info()[0] == expected_tiles(lengths, ops, cfg)
            clobber(torch, segs)
            plan.run()
            check_results(torch, co, segs, host, exp, f"shape {cfg}", oracle_codes=cfg == tune.BATCH_CONFIGS[0])
            plan.close()
    finally:
        vc.set_batch_config(*saved)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_mixed_segments(torch_dev, precision):
    torch = torch_dev
    lengths, ops = inputs.segments(nseg=64, seed=3, lo_exp=3.0, hi_exp=5.0)
    # edge segments: empty of every op, single vectors, one tile +- 1, unaligned operands
    lengths, ops = list(lengths) + EDGE_LENGTHS, list(ops) + EDGE_OPS
    say(f"case: batch precision={precision} nseg={len(lengths)} total={int(np.sum(lengths))}")
    c, co = vc.codec(precision=precision), O.codec()
    segs, host = build_segments(torch, co, lengths, ops, pad_every=5)
    exp = expected_codes(torch, c, segs)
    plan = vc.BatchPlan(c, segs)
    tiles, grid = plan.info()
    say(f"plan: {tiles} tiles, grid {grid}")
    assert tiles == expected_tiles(lengths, ops, vc.get_batch_config())

    clobber(torch, segs)
    plan.run()
    first = check_results(torch, co, segs, host, exp, "persistent")
    for rep in range(3):
        clobber(torch, segs)
        scratch = vc.vc_norm2(c, segs[-2]["a"])   # eager library work between replays
        torch.cuda.synchronize()
        del scratch
        plan.run()
        again = check_results(torch, co, segs, host, exp, f"replay {rep}", oracle_codes=False)
        assert again == first, "reductions not deterministic across replays"

    clobber(torch, segs)
    plan.run_separate()
    sep = check_results(torch, co, segs, host, exp, "separate", oracle_codes=False)
    for rep in range(2):
        clobber(torch, segs)
        plan.run_separate_graph()
        sep_g = check_results(torch, co, segs, host, exp, f"separate graph {rep}", oracle_codes=False)
        assert sep_g == sep
    plan.close()


def test_batch_in_place_axpy(torch_dev):
    torch = torch_dev
    say("case: batch in-place axpy")
    c, co = vc.codec(), O.codec()
    n = 5000
    wa = O.encode(co, inputs.gaussian(n, 41))
    wb = O.encode(co, inputs.gaussian(n, 42))
    ta, tb = up(torch, wa), up(torch, wb)
    ref = vc.vc_axpy(c, ALPHA, ta, tb).cpu()
    plan = vc.BatchPlan(c, [{"op": "axpy", "n": n, "a": ta, "b": tb, "out": ta, "alpha": ALPHA}])
    plan.run()
    torch.cuda.synchronize()
    assert torch.equal(ta.cpu(), ref)
    plan.close()


@pytest.mark.parametrize("kw", [{"mode": "frac", "P": 163840}, {"mag_round": "trunc"}])
def test_batch_variant_codec(torch_dev, kw):
    """fractional split and truncating-magnitude codecs through the persistent kernel"""
    torch = torch_dev
    say(f"case: batch {kw}")
    c, co = vc.codec(**kw), O.codec(**kw)
    lengths, ops = [3000, 7001, 20000, 1], ["axpy", "encode", "dot", "norm2"]
    segs, host = build_segments(torch, co, lengths, ops)
    exp = expected_codes(torch, c, segs)
    plan = vc.BatchPlan(c, segs)
    plan.run()
    check_results(torch, co, segs, host, exp, "frac")
    plan.close()


def test_batch_empty_plan(torch_dev):
    plan = vc.BatchPlan(vc.codec(), [])
    plan.run()
    plan.run_separate()
    plan.run_separate_graph()
    assert plan.info() == (0, 1)
    plan.close()
