"""Seeded synthetic inputs for the compression workloads.

This module only draws random numbers and lays them out; it contains none of
the codec's arithmetic, so the GPU path and the CPU oracle can both be fed from
it without sharing any of the method.

All draws use numpy's PCG64 in FP64 and round to FP32 at the end.  Large draws
are produced in fixed-size chunks from one generator, so a given (seed, n)
always yields the same array.

Workloads (shapes and distributions follow the paper's test settings: the unit ball of
§2.2/§3, the streaming kernel of §5 and the flux-reconstruction fields of §4):
  * ``gaussian_with_edges``  -- N(0,1) components plus axis/zero/extreme cases
  * ``sphere_loguniform``    -- directions uniform on S^2, |x| log-uniform
  * ``unit_sphere`` / ``unit_cube`` -- the unit-ball samplers of §2.2 and §3
  * ``angle_uniform``        -- theta, phi drawn uniformly (§2.3 averages)
  * ``vmf``                  -- von Mises-Fisher directions (Wood's method), lognormal |x|
  * ``tgv_elements``         -- Taylor-Green velocity at Gauss-Legendre points of hex elements
  * ``uniform_matrix``       -- U[-1,1] operator entries
  * ``segments``             -- uneven segment table for the batched launch
  * ``fr_derivative_1d`` / ``fr_div_operator`` -- nodal derivative operators of a hexahedral
    flux-reconstruction element (tensor-product Lagrange basis on Gauss-Legendre points)
  * ``euler_flux_tgv``       -- Euler flux rows (5 x 3 per point) of the Taylor-Green initial state
"""
from __future__ import annotations

import math

import numpy as np

CHUNK = 1 << 22


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _normal_rows(g: np.random.Generator, n: int, out: np.ndarray | None = None) -> np.ndarray:
    """n x 3 standard normals in FP64, drawn chunk by chunk."""
    res = np.empty((n, 3), dtype=np.float64) if out is None else out
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        res[s:e] = g.standard_normal((e - s, 3))
    return res


def edge_cases() -> np.ndarray:
    """Axis vectors, the zero vector and two extreme magnitudes along +x and (1,2,3)/sqrt(14)."""
    d = np.array([1.0, 2.0, 3.0]) / np.sqrt(14.0)
    rows = [
        (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1), (0, 0, 0),
        (1e-30, 0, 0), (1e30, 0, 0), tuple(1e-30 * d), tuple(1e30 * d),
    ]
    return np.array(rows, dtype=np.float64).astype(np.float32)


def gaussian_with_edges(n: int = 65536, seed: int = 0) -> np.ndarray:
    """n vectors with i.i.d. N(0,1) components followed by ``edge_cases()`` (n + 11 rows)."""
    g = _rng(seed)
    body = _normal_rows(g, n).astype(np.float32)
    return np.concatenate([body, edge_cases()], axis=0)


def gaussian(n: int, seed: int) -> np.ndarray:
    return _normal_rows(_rng(seed), n).astype(np.float32)


def _normalise(v: np.ndarray) -> np.ndarray:
    nrm = np.sqrt((v * v).sum(axis=1, keepdims=True))
    nrm[nrm == 0] = 1.0
    return v / nrm


def sphere_loguniform(n: int, seed: int, lo_exp: float = -6.0, hi_exp: float = 6.0) -> np.ndarray:
    """Directions uniform on S^2 (normalised Gaussians), |x| = 10^U[lo_exp, hi_exp]."""
    g = _rng(seed)
    out = np.empty((n, 3), dtype=np.float32)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        d = _normalise(g.standard_normal((e - s, 3)))
        r = 10.0 ** g.uniform(lo_exp, hi_exp, size=(e - s, 1))
        out[s:e] = (d * r).astype(np.float32)
    return out


def unit_sphere(n: int, seed: int) -> np.ndarray:
    """Points uniform on the unit sphere, generated in FP64 and rounded to FP32 (§2.2)."""
    g = _rng(seed)
    return _normalise(_normal_rows(g, n)).astype(np.float32)


def unit_cube(n: int, seed: int) -> np.ndarray:
    """Points uniform in [-1, 1]^3 (§3)."""
    g = _rng(seed)
    return g.uniform(-1.0, 1.0, size=(n, 3)).astype(np.float32)


def angle_uniform(n: int, seed: int, radius: float = 1.0) -> np.ndarray:
    """theta ~ U[-pi, pi), phi ~ U[0, pi), fixed radius, mapped to Cartesian in FP64."""
    g = _rng(seed)
    th = g.uniform(-np.pi, np.pi, size=n)
    ph = g.uniform(0.0, np.pi, size=n)
    v = np.stack([np.cos(th) * np.sin(ph), np.sin(th) * np.sin(ph), np.cos(ph)], axis=1)
    return (radius * v).astype(np.float32)


def _rotation_to(mean: np.ndarray) -> np.ndarray:
    """Rotation matrix taking +z to the unit vector ``mean``."""
    mu = np.asarray(mean, dtype=np.float64)
    mu = mu / np.linalg.norm(mu)
    zhat = np.array([0.0, 0.0, 1.0])
    v = np.cross(zhat, mu)
    s = np.linalg.norm(v)
    cth = float(zhat @ mu)
    if s < 1e-15:
        return np.eye(3) if cth > 0 else np.diag([1.0, -1.0, -1.0])
    vx = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])
    return np.eye(3) + vx + vx @ vx * ((1 - cth) / (s * s))


def vmf(n: int, kappa: float, mean=(0.0, 0.0, 1.0), seed: int = 0, sigma: float = 2.0) -> np.ndarray:
    """von Mises-Fisher directions on S^2 about ``mean`` (Wood 1994 for p = 3:
    w = 1 + ln(xi + (1 - xi) e^{-2 kappa}) / kappa, uniform azimuth), magnitudes
    lognormal(0, sigma)."""
    g = _rng(seed)
    R = _rotation_to(np.asarray(mean, dtype=np.float64))
    out = np.empty((n, 3), dtype=np.float32)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        m = e - s
        xi = g.uniform(0.0, 1.0, size=m)
        w = 1.0 + np.log(xi + (1.0 - xi) * np.exp(-2.0 * kappa)) / kappa
        w = np.clip(w, -1.0, 1.0)
        az = g.uniform(0.0, 2.0 * np.pi, size=m)
        sw = np.sqrt(np.maximum(0.0, 1.0 - w * w))
        d = np.stack([sw * np.cos(az), sw * np.sin(az), w], axis=1) @ R.T
        r = np.exp(sigma * g.standard_normal(m))[:, None]
        out[s:e] = (d * r).astype(np.float32)
    return out


def vmf_torch(n: int, kappa: float, mean=(0.0, 0.0, 1.0), seed: int = 0, sigma: float = 2.0, device="cuda"):
    """GPU-side draw of the ``vmf`` distribution (torch's seeded Philox generator), FP64 then FP32."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    R = torch.from_numpy(_rotation_to(np.asarray(mean, dtype=np.float64))).to(device)
    xi = torch.rand(n, generator=g, dtype=torch.float64, device=device)
    w = 1.0 + torch.log(xi + (1.0 - xi) * math.exp(-2.0 * kappa)) / kappa
    w = w.clamp(-1.0, 1.0)
    az = 2.0 * math.pi * torch.rand(n, generator=g, dtype=torch.float64, device=device)
    sw = torch.sqrt(torch.clamp(1.0 - w * w, min=0.0))
    d = torch.stack([sw * torch.cos(az), sw * torch.sin(az), w], dim=1) @ R.T
    r = torch.exp(sigma * torch.randn(n, generator=g, dtype=torch.float64, device=device))[:, None]
    return (d * r).to(torch.float32).contiguous()


def sampler_torch(kind: str, n: int, seed: int, device="cuda", radius: float = 1.0):
    """GPU-side draws (torch's seeded Philox) of the unit-ball samplers: ``sphere`` (uniform on
    S^2: normalised FP64 Gaussians), ``cube`` (uniform in [-1, 1]^3) and ``angles`` (theta, phi
    uniform on [-pi, pi) x [0, pi)), scaled by ``radius``, rounded to FP32 [n, 3]."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    if kind == "sphere":
        d = torch.randn((n, 3), generator=g, dtype=torch.float64, device=device)
        v = d / torch.linalg.vector_norm(d, dim=1, keepdim=True).clamp_min(1e-300)
    elif kind == "cube":
        v = 2.0 * torch.rand((n, 3), generator=g, dtype=torch.float64, device=device) - 1.0
    elif kind == "angles":
        th = (2.0 * torch.rand(n, generator=g, dtype=torch.float64, device=device) - 1.0) * math.pi
        ph = torch.rand(n, generator=g, dtype=torch.float64, device=device) * math.pi
        v = torch.stack([torch.cos(th) * torch.sin(ph), torch.sin(th) * torch.sin(ph), torch.cos(ph)], dim=1)
    else:
        raise ValueError(kind)
    return (radius * v).to(torch.float32).contiguous()


def gauss_legendre_nodes(k: int) -> np.ndarray:
    x, _ = np.polynomial.legendre.leggauss(k)
    return x


def tgv_elements(n_elem: int = 200_000, p: int = 4, grid=(100, 50, 40), seed: int = 0,
                 noise: float = 1e-3) -> np.ndarray:
    """Velocity u = (sin x cos y cos z, -cos x sin y cos z, 0) plus N(0, noise^2) per
    component, at the (p+1)^3 Gauss-Legendre solution points of hexahedral elements
    tiling [0, 2 pi]^3 (``grid`` elements per direction).  Returns [n_elem, (p+1)^3, 3] FP32."""
    nx, ny, nz = grid
    if nx * ny * nz < n_elem:
        raise ValueError("grid holds fewer elements than requested")
    g = _rng(seed)
    q = p + 1
    xi = 0.5 * (gauss_legendre_nodes(q) + 1.0)  # in [0, 1]
    npts = q ** 3
    out = np.empty((n_elem, npts, 3), dtype=np.float32)
    L = 2.0 * np.pi
    hx, hy, hz = L / nx, L / ny, L / nz
    a, b, c = np.meshgrid(xi, xi, xi, indexing="ij")
    a, b, c = a.ravel(), b.ravel(), c.ravel()
    step = 8192
    for s in range(0, n_elem, step):
        e = min(n_elem, s + step)
        idx = np.arange(s, e)
        ix, iy, iz = idx % nx, (idx // nx) % ny, idx // (nx * ny)
        X = (ix[:, None] + a[None, :]) * hx
        Y = (iy[:, None] + b[None, :]) * hy
        Z = (iz[:, None] + c[None, :]) * hz
        u = np.sin(X) * np.cos(Y) * np.cos(Z)
        v = -np.cos(X) * np.sin(Y) * np.cos(Z)
        w = np.zeros_like(u)
        vel = np.stack([u, v, w], axis=2) + noise * g.standard_normal((e - s, npts, 3))
        out[s:e] = vel.astype(np.float32)
    return out


def fr_derivative_1d(p: int, h: float = 2.0) -> np.ndarray:
    """d[a][b] = l_a'(x_b): derivative of the Lagrange basis polynomial a at Gauss-Legendre node b,
    on an element of width h (reference width 2).  FP64, [p+1][p+1]."""
    x = gauss_legendre_nodes(p + 1)
    q = x.size
    w = np.array([1.0 / np.prod([x[i] - x[m] for m in range(q) if m != i]) for i in range(q)])
    d = np.empty((q, q))
    for a in range(q):
        for b in range(q):
            d[a, b] = (w[a] / w[b]) / (x[b] - x[a]) if a != b else sum(1.0 / (x[a] - x[m]) for m in range(q) if m != a)
    return d * (2.0 / h)


def fr_div_operator(p: int, h=(2.0, 2.0, 2.0)) -> np.ndarray:
    """Dense divergence operator of a hexahedral element, D[c n_s + j][k] = d l_j / d x_c at point
    k, for the tensor-product basis; point index j = jx + q jy + q^2 jz, q = p + 1, n_s = q^3.
    FP64, [3 n_s][n_s]."""
    q = p + 1
    ns = q ** 3
    d = [fr_derivative_1d(p, hc) for hc in h]
    eye = np.eye(q)
    # kron order: the fastest index (x) is the last factor
    Dx = np.kron(eye, np.kron(eye, d[0]))
    Dy = np.kron(eye, np.kron(d[1], eye))
    Dz = np.kron(d[2], np.kron(eye, eye))
    return np.concatenate([Dx, Dy, Dz], axis=0).reshape(3 * ns, ns)


def euler_flux_tgv(n_elem: int, p: int = 4, grid=(64, 64, 64), gamma: float = 1.4, U0: float = 1.0,
                   rho0: float = 1.0, p0: float = 100.0, device=None):
    """Inviscid flux rows of the Taylor-Green initial state (sec. 4, TGV: velocity U0 (f(x,y,z),
    -f(y,x,z), 0), f = sin x cos y cos z, pressure p0 + rho0 U0^2/16 (cos 2x + cos 2y)(2 + cos 2z),
    density from p rho0/p0) at the Gauss-Legendre solution points of hexahedral elements tiling
    [0, 2 pi]^3 with ``grid`` elements per direction (element e at ix = e % gx, iy = (e / gx) % gy,
    iz = e / (gx gy)), as the five rows of Eq. (eulerF):
        (rho u, rho v, rho w), (rho u^2 + p, rho u v, rho u w), (rho u v, rho v^2 + p, rho v w),
        (rho u w, rho v w, rho w^2 + p), (u (E + p), v (E + p), w (E + p)),
    E = p / (gamma - 1) + rho |u|^2 / 2.  Returns float32 [n_elem][(p+1)^3][5][3] (a torch tensor on
    ``device`` when given, else numpy).  Computed in FP64."""
    import torch

    gx, gy, gz = grid
    if gx * gy * gz < n_elem:
        raise ValueError("grid holds fewer elements than requested")
    dev = torch.device(device) if device is not None else torch.device("cpu")
    q = p + 1
    xi = torch.from_numpy(0.5 * (gauss_legendre_nodes(q) + 1.0)).to(dev)
    a = xi.view(1, 1, q).expand(q, q, q).reshape(-1)
    b = xi.view(1, q, 1).expand(q, q, q).reshape(-1)
    c = xi.view(q, 1, 1).expand(q, q, q).reshape(-1)
    L = 2.0 * math.pi
    out = torch.empty((n_elem, q ** 3, 5, 3), dtype=torch.float32, device=dev)
    step = 1 << 14
    for s in range(0, n_elem, step):
        e = torch.arange(s, min(n_elem, s + step), device=dev, dtype=torch.float64)
        ix, iy, iz = torch.remainder(e, gx), torch.remainder(torch.floor(e / gx), gy), torch.floor(e / (gx * gy))
        X = (ix[:, None] + a[None]) * (L / gx)
        Y = (iy[:, None] + b[None]) * (L / gy)
        Z = (iz[:, None] + c[None]) * (L / gz)
        u = U0 * torch.sin(X) * torch.cos(Y) * torch.cos(Z)
        v = -U0 * torch.sin(Y) * torch.cos(X) * torch.cos(Z)
        w = torch.zeros_like(u)
        pr = p0 + rho0 * U0 * U0 / 16.0 * (torch.cos(2 * X) + torch.cos(2 * Y)) * (2.0 + torch.cos(2 * Z))
        rho = pr * rho0 / p0
        En = pr / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
        rows = [(rho * u, rho * v, rho * w),
                (rho * u * u + pr, rho * u * v, rho * u * w),
                (rho * u * v, rho * v * v + pr, rho * v * w),
                (rho * u * w, rho * v * w, rho * w * w + pr),
                (u * (En + pr), v * (En + pr), w * (En + pr))]
        blk = torch.stack([torch.stack(r, dim=-1) for r in rows], dim=-2)
        out[s:s + blk.shape[0]] = blk.to(torch.float32)
    return out if device is not None else out.numpy()


def uniform_matrix(rows: int = 150, cols: int = 125, seed: int = 2) -> np.ndarray:
    return _rng(seed).uniform(-1.0, 1.0, size=(rows, cols)).astype(np.float32)


def segments(nseg: int = 64, seed: int = 3, lo_exp: float = 3.0, hi_exp: float = 7.0,
             ops=("axpy", "dot", "norm2", "encode")):
    """Segment lengths floor(10^U[lo, hi]) and a shuffled round-robin op assignment."""
    g = _rng(seed)
    lengths = np.floor(10.0 ** g.uniform(lo_exp, hi_exp, size=nseg)).astype(np.int64)
    tags = np.array([ops[i % len(ops)] for i in range(nseg)])
    g.shuffle(tags)
    return lengths, list(tags)


def sphere_loguniform_torch(n: int, seed: int, device="cuda", lo_exp: float = -6.0, hi_exp: float = 6.0,
                            chunk: int = 1 << 24):
    """GPU-side draw of the ``sphere_loguniform`` distribution (torch's seeded Philox generator):
    directions = normalised FP64 Gaussians, |x| = 10^U[lo_exp, hi_exp], rounded to FP32.
    Used for the large benchmark inputs, which are generated where they are consumed."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = torch.empty((n, 3), dtype=torch.float32, device=device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        d = torch.randn((e - s, 3), generator=g, dtype=torch.float64, device=device)
        d = d / torch.linalg.vector_norm(d, dim=1, keepdim=True).clamp_min(1e-300)
        r = torch.pow(10.0, torch.empty((e - s, 1), dtype=torch.float64, device=device).uniform_(
            lo_exp, hi_exp, generator=g))
        out[s:e] = (d * r).to(torch.float32)
    return out
