"""Parity at the benchmark's full sizes, in the launch configurations bench.py times, on sampled
outputs the oracle computes one by one (and properties that hold at any size).

  axpy     N = 2^27, directions uniform on S^2, |x| = 10^U[-6, 6], alpha = RN32(0.7), the tuned
           launch of vc_axpy, for the plain codec (both encoders), the variants and the
           truncating magnitude
  apply    200,000 p = 4 elements of the Taylor-Green field, operator 150 x 125
  batch    64 segments of floor(10^U[3, 7]) vectors, axpy / dot / norm2 / encode
  errhist  2^25 von Mises-Fisher vectors (kappa 1000 about +z), against the oracle's histogram
  fdiv     64^3 p = 4 hexahedra of the Taylor-Green Euler flux (the persistent launch with about
           70 element groups per workgroup), 2,000 sampled elements against the oracle
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
N = 1 << 27
SAMPLE = 1 << 20


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    vc.lib()
    return torch


@pytest.fixture(scope="module")
def operands(torch_dev):
    a32 = inputs.sphere_loguniform_torch(N, 0)
    b32 = inputs.sphere_loguniform_torch(N, 1)
    yield a32, b32
    del a32, b32


def _sample(torch, n, seed):
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    return torch.randint(0, n, (min(SAMPLE, n),), generator=g).to("cuda")


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("label,kw", [("plain-f64", {"precision": "f64"}), ("plain-f32", {"precision": "f32"}),
                                      ("frac163840", {"mode": "frac", "P": 163840}),
                                      ("tanh0.5", {"mode": "tanh", "gamma": 0.5}), ("cos", {"mode": "cos"}),
                                      ("tanh0.5-f32", {"mode": "tanh", "gamma": 0.5, "precision": "f32"}),
                                      ("cos-f32", {"mode": "cos", "precision": "f32"}),
                                      ("trunc", {"mag_round": "trunc"}),
                                      ("trunc-f32", {"mag_round": "trunc", "precision": "f32"})])
def test_axpy_full_size(torch_dev, operands, label, kw):
    torch = torch_dev
    say(f"case: full-size axpy {label} N=2^27")
    a32, b32 = operands
    okw = {k: v for k, v in kw.items() if k != "precision"}
    c, co = vc.codec(**kw), O.codec(**okw)
    wa, wb = vc.vc_encode(c, a32), vc.vc_encode(c, b32)
    wc = vc.vc_axpy(c, ALPHA, wa, wb)                 # the launch bench.py times
    wd, c32 = vcx_dump(torch, c, wa, wb)              # the verification variant, same arithmetic
    idx = _sample(torch, N, 7)
    sa, sb, sc, sd, s32 = _u64(wa[idx]), _u64(wb[idx]), _u64(wc[idx]), _u64(wd[idx]), c32[idx].cpu().numpy()
    del wd, c32
    # the timed launch equals the verification variant bit for bit
    assert np.array_equal(sc, sd)
    # the codes follow the encode rule against the oracle on the same single-precision sums
    res = classify(co, s32, sc)
    say(f"{label}: identical {res['identical']}/{res['n']}, +-1 theta {res['pm1_theta']}, phi {res['pm1_phi']}")
    assert res["other"] == 0, describe_bad(co, s32, sc, res)
    # end to end against the FP64 sum of the exactly decoded operands
    A64, B64 = O.decode64(co, sa), O.decode64(co, sb)
    c64 = ALPHA * A64 + B64
    got = O.decode64(co, sc)
    nrm = np.linalg.norm(c64, axis=1)
    scale = ALPHA * np.linalg.norm(A64, axis=1) + np.linalg.norm(B64, axis=1)
    ok = (nrm > 2.0 ** -70) & (nrm < 1e14)
    nt, npm = O.nmax(co)
    # companded codecs (§2.5): the level spacing is the uniform one divided by h'(u); for
    # h(u) = tanh(g u)/tanh(g) the smallest slope is g sech^2(g)/tanh(g), at |u| = 1
    stretch = 1.0
    if kw.get("mode") == "tanh":
        g = kw["gamma"]
        stretch = g / (math.cosh(g) ** 2 * math.tanh(g))
    elif kw.get("mode") == "cos":
        stretch = None
    err = np.linalg.norm(got - c64, axis=1)[ok]
    # magnitude: nearest-even at 23 bits, or (truncation) nearest-even at 24 then one bit dropped
    mag = 2.0 ** -22 + 2.0 ** -24 if kw.get("mag_round") == "trunc" else 2.0 ** -23
    if stretch is not None:
        bound = (math.hypot(math.pi / nt, math.pi / (2 * npm)) / stretch + mag) * nrm[ok] \
            + (4 * 2.0 ** -24 + 1e-6) * scale[ok]
        say(f"{label}: max end-to-end err/allowed {(err / bound).max():.3f}")
        assert (err <= bound).all()
    else:
        # the cosine map h(u) = sin(pi u / 2) is stationary at the ends of the angle ranges
        # (u = +-1), where its level spacing has no useful bound; inside, the spacing of each angle
        # is the uniform one divided by h'(u) = (pi/2) cos(pi u / 2), taken at |u| + 1e-3 (the
        # level's width and the sum's rounding move u by far less).  Every vector with both angles
        # at |u| <= 0.95 is held to Eq. (v_error) with those spacings.
        cc = c64[ok]
        th = np.arctan2(cc[:, 1], cc[:, 0])
        ph = np.arctan2(np.hypot(cc[:, 0], cc[:, 1]), cc[:, 2])
        ut, up_ = np.abs(th / math.pi), np.abs(2 * ph / math.pi - 1)
        inner = (ut <= 0.95) & (up_ <= 0.95)
        slope = lambda u: (math.pi / 2) * np.cos(math.pi / 2 * np.minimum(u + 1e-3, 1.0))
        et = math.pi / nt / slope(ut) * np.sin(ph)
        ep = math.pi / (2 * npm) / slope(up_)
        bound = (np.hypot(et, ep) + mag) * nrm[ok] + (4 * 2.0 ** -24 + 1e-6) * scale[ok]
        say(f"{label}: interior {int(inner.sum())}/{inner.size}, max end-to-end err/allowed "
            f"{(err[inner] / bound[inner]).max():.3f}")
        assert inner.sum() > 0.8 * inner.size
        assert (err[inner] <= bound[inner]).all()
        assert np.isfinite(got[ok]).all()


def vcx_dump(torch, c, wa, wb):
    out, c32 = vc.vcx_axpy_dump(c, ALPHA, wa, wb)
    torch.cuda.synchronize()
    return out, c32


def test_apply_full_size(torch_dev):
    """200,000 elements in the benchmark's launch; 2,000 sampled elements against the oracle"""
    torch = torch_dev
    say("case: full-size apply 200,000 elements")
    E, rows, cols = 200_000, 150, 125
    c, co = vc.codec(), O.codec()
    vel = inputs.tgv_elements(E, 4, seed=0)
    W = vc.vc_encode(c, torch.from_numpy(vel.reshape(-1, 3)).to("cuda")).view(E, cols)
    del vel
    M = inputs.uniform_matrix(rows, cols, 2)
    out = vc.vc_fused_apply(c, torch.from_numpy(M).to("cuda"), W)
    g = np.random.default_rng(5)
    el = np.sort(g.choice(E, 2000, replace=False))
    Ws = W[torch.from_numpy(el).to("cuda")].cpu().numpy().view(np.uint64)
    got = out[torch.from_numpy(el).to("cuda")].cpu().numpy().astype(np.float64)
    ref = O.apply(co, M, Ws)
    X = O.decode64(co, Ws.reshape(-1)).reshape(len(el), cols, 3)
    scale = np.einsum("ij,ej->ei", np.abs(M.astype(np.float64)), np.linalg.norm(X, axis=2))
    ratio = (np.abs(got - ref).max(axis=2) / (1e-5 * scale)).max()
    say(f"apply full size: max err/tol {ratio:.3f}")
    assert ratio <= 1.0


def test_batch_full_size(torch_dev):
    """the 64-segment plan (about 5e7 vectors): at sampled positions the codes equal the
    single-call entry points and follow the encode rule against the oracle; reductions match
    the oracle"""
    torch = torch_dev
    say("case: full-size batch 64 segments")
    lengths, ops = inputs.segments(nseg=64, seed=3, lo_exp=3.0, hi_exp=7.0)
    c, co = vc.codec(), O.codec()
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    segs = []
    for n, op in zip(lengths, ops):
        n = int(n)
        x = torch.randn((n, 3), generator=g, dtype=torch.float32, device="cuda")
        if op == "encode":
            segs.append({"op": op, "n": n, "a": x, "out": torch.empty(n, dtype=torch.int64, device="cuda")})
            continue
        a = vc.vc_encode(c, x)
        b = vc.vc_encode(c, torch.randn((n, 3), generator=g, dtype=torch.float32, device="cuda")) \
            if op in ("axpy", "dot") else None
        out = torch.empty(n, dtype=torch.int64, device="cuda") if op == "axpy" else \
            torch.empty(1, dtype=torch.float32, device="cuda")
        segs.append({"op": op, "n": n, "a": a, "b": b, "out": out, "alpha": ALPHA})
    plan = vc.BatchPlan(c, segs)
    plan.run()
    torch.cuda.synchronize()
    for i, s in enumerate(segs):
        n = s["n"]
        if s["op"] in ("axpy", "encode"):
            idx = _sample(torch, n, 100 + i)
            ref = vc.vc_axpy(c, ALPHA, s["a"], s["b"]) if s["op"] == "axpy" else vc.vc_encode(c, s["a"])
            assert torch.equal(s["out"][idx], ref[idx]), (i, s["op"], n)
            del ref
            # the sampled codes against the oracle: the encode rule on the segment's input, or on
            # the single-precision sums of the same operands (the axpy's verification variant)
            got = _u64(s["out"][idx])
            if s["op"] == "encode":
                xin = s["a"][idx].cpu().numpy()
            else:
                _, c32 = vc.vcx_axpy_dump(c, ALPHA, s["a"], s["b"])
                xin = c32[idx].cpu().numpy()
                del c32
            res = classify(co, xin, got)
            assert res["other"] == 0, (i, s["op"], describe_bad(co, xin, got, res))
        else:
            wa = _u64(s["a"])
            v = float(s["out"].cpu()[0])
            if s["op"] == "dot":
                wb = _u64(s["b"])
                refv = O.dot(co, wa, wb)
                A, B = O.decode64(co, wa), O.decode64(co, wb)
                scale = float((np.linalg.norm(A, axis=1) * np.linalg.norm(B, axis=1)).sum())
            else:
                refv = O.norm2(co, wa)
                scale = refv
            assert abs(v - refv) <= 4e-6 * scale, (i, s["op"], n, v, refv)
    plan.close()


def test_errhist_full_size(torch_dev):
    """2^25 vMF vectors (kappa 1000 about +z): the GPU histograms against the oracle's on the same
    vectors, within the counted one-level code differences"""
    torch = torch_dev
    say("case: full-size error histogram 2^25")
    n = 1 << 25
    c, co = vc.codec(), O.codec()
    x = inputs.vmf_torch(n, 1000.0, (0.0, 0.0, 1.0), seed=1000)
    edges = O.log_edges()
    hg, exg, sg = vc.error_hist(c, x, torch.from_numpy(edges).to("cuda"))
    xs = x.cpu().numpy()
    ho, exo, so = O.error_hist(co, xs, edges)
    n_diff = int((_u64(vc.vc_encode(c, x)) != O.encode(co, xs)).sum())
    hg = hg.numpy().astype(np.int64)
    ho = ho.astype(np.int64)
    say(f"errhist full size: n_diff {n_diff}, hist L1 {[int(np.abs(hg[k] - ho[k]).sum()) for k in range(3)]}")
    assert exg == exo
    for k in range(3):
        assert int(np.abs(hg[k] - ho[k]).sum()) <= 2 * n_diff
        assert abs(float(sg[k, 0]) - so[k, 0]) <= n_diff * 4e-5 + 1e-9 * abs(so[k, 0])


def test_flux_div_full_size(torch_dev):
    """Alg. (fr_fdiv_comp) on 64^3 p = 4 hexahedra, the benchmark's launch: each persistent
    workgroup walks many element groups (next-group loads in flight, LDS reused across groups).
    The codes are the oracle's encoding of the generated flux.  2,000 sampled elements are checked
    against the oracle's dense FP64 algorithm (2e-6 sum |D| ||X||: the decode contract bounds a
    component's error by 1e-6 of the vector's norm) and against the FP64 contraction of the GPU's own
    decode of the same codes ((3 q + 2) 2^-24 sum |D| |X|: the kernel's single-precision sum alone)"""
    torch = torch_dev
    say("case: full-size flux divergence 64^3 p=4")
    grid, p = (64, 64, 64), 4
    q, npq = p + 1, 5
    ne, ns = grid[0] * grid[1] * grid[2], (p + 1) ** 3
    c, co = vc.codec(), O.codec()
    d32 = np.stack([inputs.fr_derivative_1d(p, 2 * math.pi / gc) for gc in grid]).astype(np.float32)
    F = inputs.euler_flux_tgv(ne, p, grid=grid, device="cuda").cpu().numpy()
    Wh = O.encode(co, F.reshape(-1, 3)).reshape(ne, ns, npq)
    del F
    W = torch.from_numpy(Wh.view(np.int64)).to("cuda")
    out = vc.vc_flux_div_tp(c, torch.from_numpy(d32).to("cuda"), W)
    g = np.random.default_rng(64)
    el = np.sort(g.choice(ne, 2000, replace=False))
    # the first and last elements (first and last groups of the walk) always among them
    el = np.unique(np.concatenate([el, [0, 1, ne - 2, ne - 1]]))
    ti = torch.from_numpy(el).to("cuda")
    got = out[ti].cpu().numpy().astype(np.float64)
    Xg = vc.vc_decode(c, W[ti].reshape(-1)).cpu().numpy().astype(np.float64).reshape(len(el), ns, npq, 3)
    Ws = Wh[el]
    del W, out, Wh
    eye = np.eye(q, dtype=np.float64)
    dd = d32.astype(np.float64)
    D = np.concatenate([np.kron(eye, np.kron(eye, dd[0])), np.kron(eye, np.kron(dd[1], eye)),
                        np.kron(dd[2], np.kron(eye, eye))]).astype(np.float32)
    ref = O.flux_div(co, D, Ws)
    X = O.decode64(co, Ws.reshape(-1)).reshape(len(el), ns, npq, 3)
    D64 = D.astype(np.float64).reshape(3, ns, ns)
    absD = np.abs(D64)
    scale = np.einsum("cjk,ejp->ekp", absD, np.linalg.norm(X, axis=-1), optimize=True)
    ratio = (np.abs(got - ref) / (2e-6 * scale + 1e-30)).max()
    own = np.einsum("cjk,ejpc->ekp", D64, Xg, optimize=True)
    own_scale = np.einsum("cjk,ejpc->ekp", absD, np.abs(Xg), optimize=True)
    own_ratio = (np.abs(got - own) / ((3 * q + 2) * 2.0 ** -24 * own_scale + 1e-30)).max()
    say(f"flux div full size: {len(el)} sampled elements, max err/tol {ratio:.3f} (oracle), "
        f"{own_ratio:.3f} (own decode)")
    assert ratio <= 1.0
    assert own_ratio <= 1.0
