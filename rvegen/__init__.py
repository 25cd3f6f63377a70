"""Seeded synthetic RVE (representative volume element) generators.

This module only produces voxel conductivity arrays.  It holds none of the
solver's arithmetic: both the GPU path (through its tests and benchmark) and the
CPU oracle consume the arrays it returns, and neither imports the other.

Conventions shared by every generator:

* arrays are C-contiguous ``float64`` of shape ``(n0, n1, n2)``; user dim 0 is
  called ``x`` and is the default load axis;
* voxel ``(i, j, k)`` has its centre at ``(i + 1/2, j + 1/2, k + 1/2)`` in voxel
  units; a voxel belongs to a shape when its centre lies inside the closed
  shape (the centre-in-shape rule the paper uses for its center-ball RVE,
  Section "Investigations on the TPFA scheme");
* shapes are clipped by the RVE boundary (no periodic wrap);
* randomness comes only from ``numpy.random.default_rng(seed)`` (PCG64), so a
  given seed gives the same array on every machine.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "center_ball",
    "spheres_rsa",
    "spheroids",
    "grf_lognormal",
    "series_laminate",
    "parallel_laminate",
    "random_two_phase",
    "channels",
    "CONFIGS",
    "make_config",
]


def _box(lo: float, hi: float, n: int) -> tuple[int, int]:
    """Voxel index range whose centres may fall inside [lo, hi]."""
    a = max(0, int(math.floor(lo - 0.5)))
    b = min(n, int(math.ceil(hi - 0.5)) + 1)
    return a, b


def center_ball(n: int | tuple[int, int, int], kappa_inc: float,
                radius: float = 0.25, kappa_matrix: float = 1.0) -> np.ndarray:
    """Ball of radius ``radius`` (fraction of the unit cube) at the cube centre.

    This is the paper's center-ball RVE (Section "Investigations on the TPFA
    scheme", the piecewise K with kappa_inc inside the ball of radius 1/4):
    a voxel takes ``kappa_inc`` when its centre, mapped to the unit cube, lies
    in the closed ball.
    """
    shape = (n, n, n) if isinstance(n, int) else tuple(n)
    c = [(np.arange(m) + 0.5) / m - 0.5 for m in shape]
    d2 = c[0][:, None, None] ** 2 + c[1][None, :, None] ** 2 + c[2][None, None, :] ** 2
    out = np.full(shape, float(kappa_matrix))
    out[d2 <= radius * radius] = float(kappa_inc)
    return out


class _CellGrid:
    """Uniform hash grid of sphere centres for the non-overlap test."""

    def __init__(self, cell: float):
        self.cell = cell
        self.cells: dict[tuple[int, int, int], list[int]] = {}
        self.pts: list[tuple[float, float, float]] = []

    def key(self, p):
        return (int(p[0] // self.cell), int(p[1] // self.cell), int(p[2] // self.cell))

    def near(self, p, dmin2: float) -> bool:
        kx, ky, kz = self.key(p)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for idx in self.cells.get((kx + dx, ky + dy, kz + dz), ()):
                        q = self.pts[idx]
                        if (p[0] - q[0]) ** 2 + (p[1] - q[1]) ** 2 + (p[2] - q[2]) ** 2 < dmin2:
                            return True
        return False

    def add(self, p):
        self.cells.setdefault(self.key(p), []).append(len(self.pts))
        self.pts.append(p)


def spheres_rsa(n: int, radius: float, seed: int, count: int | None = None,
                target_vf: float | None = None, kappa_matrix: float = 1.0,
                kappa_inc: float = 10.0, max_attempts: int = 5_000_000):
    """Random sequential addition of non-overlapping spheres in an n^3 grid.

    Centres are uniform in [0, n)^3; a candidate is accepted when its centre is
    at least 2*radius from every accepted centre.  Stops after ``count``
    spheres, or once the realised voxel volume fraction reaches ``target_vf``.
    Returns ``(kappa, info)`` with ``info = {"spheres": m, "vf": realised}``.
    """
    if (count is None) == (target_vf is None):
        raise ValueError("give exactly one of count / target_vf")
    rng = np.random.default_rng(seed)
    kap = np.full((n, n, n), float(kappa_matrix))
    inside = np.zeros((n, n, n), dtype=bool)
    grid = _CellGrid(2.0 * radius)
    dmin2 = (2.0 * radius) ** 2
    r2 = radius * radius
    n_in = 0
    attempts = 0
    total = n ** 3
    while True:
        if count is not None and len(grid.pts) >= count:
            break
        if target_vf is not None and n_in >= target_vf * total:
            break
        attempts += 1
        if attempts > max_attempts:
            raise RuntimeError("sphere packing did not reach its target")
        p = tuple(float(v) for v in rng.uniform(0.0, n, size=3))
        if grid.near(p, dmin2):
            continue
        grid.add(p)
        sl = []
        axes = []
        for d in range(3):
            a, b = _box(p[d] - radius, p[d] + radius, n)
            sl.append(slice(a, b))
            axes.append(np.arange(a, b) + 0.5 - p[d])
        d2 = axes[0][:, None, None] ** 2 + axes[1][None, :, None] ** 2 + axes[2][None, None, :] ** 2
        m = d2 <= r2
        sub = inside[tuple(sl)]
        n_in += int(np.count_nonzero(m & ~sub))
        sub |= m
    kap[inside] = float(kappa_inc)
    return kap, {"spheres": len(grid.pts), "vf": n_in / total}


def spheroids(n: int, semi_axes=(12.0, 3.0, 3.0), target_vf: float = 0.25, seed: int = 2,
              kappa_matrix: float = 1.0, kappa_inc: float = 100.0):
    """Overlapping prolate spheroids with uniformly random axis directions.

    The long axis ``u`` is a normalised Gaussian vector (uniform on the
    sphere); centres are uniform in [0, n)^3.  A voxel centre ``x`` is inside
    when ``((d.u)/A)^2 + (|d - (d.u)u| / B)^2 <= 1`` with ``d = x - centre``.
    Spheroids are added until the realised volume fraction reaches
    ``target_vf``.  Returns ``(kappa, info)``.
    """
    A, B, _ = (float(v) for v in semi_axes)
    rng = np.random.default_rng(seed)
    inside = np.zeros((n, n, n), dtype=bool)
    total = n ** 3
    n_in = 0
    m_count = 0
    while n_in < target_vf * total:
        c = rng.uniform(0.0, n, size=3)
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        ext = [A * abs(u[d]) + B * math.sqrt(max(0.0, 1.0 - u[d] ** 2)) for d in range(3)]
        sl, ax = [], []
        for d in range(3):
            a, b = _box(c[d] - ext[d], c[d] + ext[d], n)
            sl.append(slice(a, b))
            ax.append(np.arange(a, b) + 0.5 - c[d])
        dx = ax[0][:, None, None]
        dy = ax[1][None, :, None]
        dz = ax[2][None, None, :]
        t = dx * u[0] + dy * u[1] + dz * u[2]
        perp2 = dx * dx + dy * dy + dz * dz - t * t
        m = (t / A) ** 2 + perp2 / (B * B) <= 1.0
        sub = inside[tuple(sl)]
        n_in += int(np.count_nonzero(m & ~sub))
        sub |= m
        m_count += 1
    kap = np.full((n, n, n), float(kappa_matrix))
    kap[inside] = float(kappa_inc)
    return kap, {"spheroids": m_count, "vf": n_in / total}


def grf_lognormal(n: int, sigma2: float = 1.0, ell: float = 8.0, seed: int = 3,
                  clip_contrast: float = 1e3, dtype=np.float32):
    """Log-normal conductivity ``exp(g)`` from a Gaussian random field ``g``.

    ``g`` has an exponential covariance ``sigma2 * exp(-r / ell)`` and is made by
    spectral synthesis on a periodic grid of edge ``2n`` (cropped to ``n``):
    white noise is filtered by ``sqrt(S(k))`` with the exponential-covariance
    spectrum ``S(k) = 8 pi sigma2 ell^3 / (1 + k^2 ell^2)^2``; the sample is then
    shifted and scaled to mean 0 and variance ``sigma2`` and clipped to
    ``+-ln(clip_contrast)/2`` so that max/min <= clip_contrast.
    """
    m = 2 * n
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((m, m, m))
    f = np.fft.rfftn(noise)
    del noise
    k1 = 2.0 * np.pi * np.fft.fftfreq(m)
    k3 = 2.0 * np.pi * np.fft.rfftfreq(m)
    kk = k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + k3[None, None, :] ** 2
    spec = 8.0 * np.pi * sigma2 * ell ** 3 / (1.0 + kk * ell * ell) ** 2
    f *= np.sqrt(spec)
    del kk, spec
    g = np.fft.irfftn(f, s=(m, m, m), axes=(0, 1, 2))[:n, :n, :n]
    del f
    g = (g - g.mean()) / g.std() * math.sqrt(sigma2)
    half = 0.5 * math.log(clip_contrast)
    g = np.clip(g, -half, half)
    return np.ascontiguousarray(np.exp(g).astype(dtype))


def series_laminate(shape, layer_kappa, axis: int = 0) -> np.ndarray:
    """Conductivity that varies only along ``axis`` (one value per layer)."""
    layer_kappa = np.asarray(layer_kappa, dtype=np.float64)
    assert layer_kappa.shape == (shape[axis],)
    bshape = [1, 1, 1]
    bshape[axis] = shape[axis]
    return np.ascontiguousarray(np.broadcast_to(layer_kappa.reshape(bshape), shape).astype(np.float64))


def parallel_laminate(shape, plane_kappa, axis: int = 0) -> np.ndarray:
    """Conductivity that is constant along ``axis`` (``plane_kappa`` varies across it)."""
    plane_kappa = np.asarray(plane_kappa, dtype=np.float64)
    rest = [s for d, s in enumerate(shape) if d != axis]
    assert plane_kappa.shape == tuple(rest)
    return np.ascontiguousarray(np.broadcast_to(np.expand_dims(plane_kappa, axis), shape).astype(np.float64))


def random_two_phase(shape, seed: int, kappa=(1.0, 10.0), p: float = 0.3) -> np.ndarray:
    """Independent Bernoulli(p) voxels taking kappa[1], else kappa[0]."""
    rng = np.random.default_rng(seed)
    return np.where(rng.random(shape) < p, float(kappa[1]), float(kappa[0]))


def channels(n: int, cells: int, psi: float, dtype=np.float64):
    """Periodic channel cells with orthotropic conductivity (Section "Other
    experiments", fig:channels-cell): the unit cell holds three orthogonal
    square bars, each spanning the cell along one axis with its cross-section
    (3/8, 5/8)^2 in the other two; inside a bar K = diag(2^psi, 5^psi, 10^psi),
    elsewhere diag(0.01, 0.1, 1).  The RVE (0,1)^3 repeats the cell `cells`
    times per axis and is sampled at the n^3 voxel centres.  Returns the
    conductivity along user axes 0, 1, 2 (x, y, z)."""
    c = np.modf((np.arange(n) + 0.5) / n * cells)[0]        # fractional cell coordinate per index
    mid = (c > 3 / 8) & (c < 5 / 8)
    X, Y, Z = mid[:, None, None], mid[None, :, None], mid[None, None, :]
    bar = (Y & Z) | (X & Z) | (X & Y)
    out = []
    for inside, outside in zip((2.0 ** psi, 5.0 ** psi, 10.0 ** psi), (0.01, 0.1, 1.0)):
        out.append(np.where(bar, inside, outside).astype(dtype))
    return tuple(out)


@dataclass
class RVEConfig:
    name: str
    n: int
    desc: str
    rtol: float
    kwargs: dict = field(default_factory=dict)


#: The benchmark/parity workloads (sizes, value distributions and structure
#: follow the paper's experiments; every geometry is synthetic and seeded).
CONFIGS = {
    "spheres32": RVEConfig("spheres32", 32, "32^3, 12 non-overlapping r=4 spheres, kappa 1/10", 1e-10,
                           dict(radius=4.0, count=12, seed=1, kappa_inc=10.0)),
    "spheroids128": RVEConfig("spheroids128", 128, "128^3 prolate 12x3x3 fibres, vf>=0.25, kappa 1/100", 1e-6,
                              dict(semi_axes=(12.0, 3.0, 3.0), target_vf=0.25, seed=2, kappa_inc=100.0)),
    "grf256": RVEConfig("grf256", 256, "256^3 log-normal GRF, exp covariance l=8 var=1, contrast<=1e3", 1e-6,
                        dict(sigma2=1.0, ell=8.0, seed=3, clip_contrast=1e3)),
    "spheres512": RVEConfig("spheres512", 512, "512^3 r=10 non-overlapping spheres to vf>=0.26, kappa 1/100", 1e-6,
                            dict(radius=10.0, target_vf=0.26, seed=4, kappa_inc=100.0)),
    "spheres512_2000": RVEConfig("spheres512_2000", 512, "512^3 2000 r=10 non-overlapping spheres, kappa 1/100", 1e-6,
                                 dict(radius=10.0, count=2000, seed=4, kappa_inc=100.0)),
}


def grf_ensemble_specs(count: int = 64, meta_seed: int = 5, edges=(48, 64, 96, 128, 160),
                       base_seed: int = 5000):
    """Specifications of an ensemble of log-normal GRF RVEs of mixed sizes.

    Per RVE ``i``: edge uniform over ``edges``, variance ``sigma2 ~ U[0.5, 2]``,
    correlation length ``ell ~ U[4, 16]``, field seed ``base_seed + i`` (the
    draws come from one generator seeded with ``meta_seed``)."""
    rng = np.random.default_rng(meta_seed)
    out = []
    for i in range(count):
        n = int(edges[int(rng.integers(len(edges)))])
        sigma2 = float(rng.uniform(0.5, 2.0))
        ell = float(rng.uniform(4.0, 16.0))
        out.append(dict(index=i, n=n, sigma2=sigma2, ell=ell, seed=base_seed + i))
    return out


def grf_ensemble(count: int = 64, meta_seed: int = 5, edges=(48, 64, 96, 128, 160), dtype=np.float32):
    """The conductivity arrays of :func:`grf_ensemble_specs` (contrast <= 1e3)."""
    specs = grf_ensemble_specs(count, meta_seed, edges)
    return [grf_lognormal(s["n"], s["sigma2"], s["ell"], s["seed"], 1e3, dtype) for s in specs], specs


def make_config(name: str, n: int | None = None):
    """Build the conductivity array of a named workload (optionally at another edge ``n``)."""
    cfg = CONFIGS[name]
    n = cfg.n if n is None else n
    if name.startswith("spheres"):
        return spheres_rsa(n, **cfg.kwargs)
    if name.startswith("spheroids"):
        return spheroids(n, **cfg.kwargs)
    if name.startswith("grf"):
        return grf_lognormal(n, **cfg.kwargs), {}
    raise KeyError(name)
