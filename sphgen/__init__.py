"""Seeded synthetic particle sets for the SPH density path.

This module only draws inputs: positions, masses, initial smoothing lengths,
group offsets and cotangents.  It holds none of the density method's
arithmetic, so both the CPU oracle and the GPU library can be fed from it
without sharing any of the computation.

The paper measures on a Gadget snapshot (81^3 dark-matter plus 81^3 gas
particles, Sec. II-C) that is not available; these generators stand in for it:
uniform periodic boxes, mixtures of Plummer spheres over a uniform background
(halo/sub-halo density contrast), and many isolated Plummer groups (the
friends-of-friends groups Subfind works on, Sec. II-B).

Every generator uses ``numpy.random.Generator(PCG64(seed))`` and returns plain
float64 NumPy arrays in the caller's (unsorted) order.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "ParticleSet",
    "default_h_init",
    "uniform",
    "lattice",
    "plummer_radii",
    "plummer_mixture",
    "group_sizes",
    "group_volume",
    "groups",
    "doubled",
    "with_duplicates",
    "cotangent",
    "config",
]


@dataclass
class ParticleSet:
    """Positions, masses and initial smoothing lengths in caller order.

    ``offsets`` is ``None`` for one periodic set, else an int64 CSR array of
    G+1 entries delimiting isolated groups (group g owns
    ``[offsets[g], offsets[g+1])``).
    """

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    m: np.ndarray
    h_init: np.ndarray
    periodic: bool
    box: float
    n_target: float
    n_tol: float
    offsets: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def pos(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.x, self.y, self.z, self.m, self.h_init):
            h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
        if self.offsets is not None:
            h.update(np.ascontiguousarray(self.offsets, dtype=np.int64).tobytes())
        return h.hexdigest()


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def default_h_init(n: int, volume: float) -> float:
    """Initial smoothing length 2 (V/N)^(1/3): twice the mean spacing."""
    return 2.0 * (volume / n) ** (1.0 / 3.0)


def uniform(n: int, seed: int, box: float = 1.0, n_target: float = 64.0,
            n_tol: float = 2.0, h_init: float | None = None) -> ParticleSet:
    """N particles uniform-random in the periodic cube [0, box)^3, equal masses 1/N."""
    rng = _rng(seed)
    p = rng.random((n, 3)) * box
    p = np.where(p >= box, np.nextafter(box, 0.0), p)
    h0 = default_h_init(n, box ** 3) if h_init is None else float(h_init)
    return ParticleSet(
        x=np.ascontiguousarray(p[:, 0]), y=np.ascontiguousarray(p[:, 1]),
        z=np.ascontiguousarray(p[:, 2]), m=np.full(n, 1.0 / n),
        h_init=np.full(n, h0), periodic=True, box=float(box),
        n_target=float(n_target), n_tol=float(n_tol),
        meta={"kind": "uniform", "seed": seed},
    )


def lattice(nside: int, box: float = 1.0, h: float = 0.1, n_target: float = 64.0,
            n_tol: float = 2.0, jitter_seed: int | None = None) -> ParticleSet:
    """Simple cubic lattice of nside^3 points at cell centres of a periodic box.

    Points are listed in a shuffled order when ``jitter_seed`` is given (the
    positions stay exact lattice sites), else x-major.
    """
    a = box / nside
    g = (np.arange(nside, dtype=np.float64) + 0.5) * a
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = X.ravel(), Y.ravel(), Z.ravel()
    n = x.shape[0]
    if jitter_seed is not None:
        order = _rng(jitter_seed).permutation(n)
        x, y, z = x[order], y[order], z[order]
    return ParticleSet(
        x=np.ascontiguousarray(x), y=np.ascontiguousarray(y), z=np.ascontiguousarray(z),
        m=np.full(n, 1.0 / n), h_init=np.full(n, float(h)), periodic=True,
        box=float(box), n_target=float(n_target), n_tol=float(n_tol),
        meta={"kind": "lattice", "nside": nside},
    )


def plummer_radii(rng: np.random.Generator, k: int, a: float,
                  mass_cut: float = 0.99) -> np.ndarray:
    """Radii of a Plummer sphere of scale radius ``a``, truncated at ``mass_cut``.

    The enclosed-mass fraction of a Plummer sphere is r^3/(r^2+a^2)^(3/2);
    inverting it for a uniform draw U gives r = a (U^(-2/3) - 1)^(-1/2).
    Truncation at 99% of the mass bounds r by about 12.2 a.
    """
    u = rng.random(k) * mass_cut
    u = np.maximum(u, 1e-300)
    return a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)


def _isotropic(rng: np.random.Generator, k: int) -> np.ndarray:
    mu = rng.random(k) * 2.0 - 1.0
    phi = rng.random(k) * (2.0 * np.pi)
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return np.stack([s * np.cos(phi), s * np.sin(phi), mu], axis=1)


def _powerlaw(rng: np.random.Generator, k: int, lo: float, hi: float,
              slope: float) -> np.ndarray:
    """Draws from dN/dx proportional to x^slope on [lo, hi] by inverse CDF."""
    u = rng.random(k)
    if abs(slope + 1.0) < 1e-12:
        return lo * (hi / lo) ** u
    e = slope + 1.0
    return (lo ** e + u * (hi ** e - lo ** e)) ** (1.0 / e)


def _largest_remainder(weights: np.ndarray, total: int) -> np.ndarray:
    w = weights / weights.sum() * total
    base = np.floor(w).astype(np.int64)
    rem = total - int(base.sum())
    if rem > 0:
        order = np.argsort(-(w - base), kind="stable")
        base[order[:rem]] += 1
    return base


def plummer_mixture(n: int, n_spheres: int, seed: int, box: float = 1.0,
                    bg_frac: float = 0.3, a_range=(0.005, 0.05),
                    mass_range=(1.0, 1000.0), mass_slope: float = -2.0,
                    contrast_cap: float | None = None, n_target: float = 64.0,
                    n_tol: float = 2.0) -> ParticleSet:
    """Plummer spheres over a uniform background in a periodic cube.

    Sphere masses follow dN/dM ~ M^slope on ``mass_range``; particle counts are
    proportional to M and sum to round((1-bg_frac) N) by largest remainder.
    Scale radii are log-uniform on ``a_range``.  With ``contrast_cap`` the
    central number-density contrast 3 n_s / (4 pi a^3 N) (box volume 1) is
    bounded by raising a.  Centres are uniform; positions wrap periodically.
    Input order is shuffled.
    """
    rng = _rng(seed)
    n_sph_tot = int(round((1.0 - bg_frac) * n))
    n_bg = n - n_sph_tot
    masses = _powerlaw(rng, n_spheres, mass_range[0], mass_range[1], mass_slope)
    counts = _largest_remainder(masses, n_sph_tot)
    loga = rng.random(n_spheres) * (np.log(a_range[1]) - np.log(a_range[0])) + np.log(a_range[0])
    a = np.exp(loga) * box
    if contrast_cap is not None:
        a_min = (3.0 * counts / (4.0 * np.pi * contrast_cap * n)) ** (1.0 / 3.0) * box
        a = np.maximum(a, a_min)
    centres = rng.random((n_spheres, 3)) * box
    parts = []
    for s in range(n_spheres):
        k = int(counts[s])
        if k == 0:
            continue
        r = plummer_radii(rng, k, a[s])
        parts.append(centres[s] + r[:, None] * _isotropic(rng, k))
    parts.append(rng.random((n_bg, 3)) * box)
    p = np.concatenate(parts, axis=0)
    p = np.mod(p, box)
    p = np.where(p >= box, np.nextafter(box, 0.0), p)
    p = p[rng.permutation(n)]
    h0 = default_h_init(n, box ** 3)
    return ParticleSet(
        x=np.ascontiguousarray(p[:, 0]), y=np.ascontiguousarray(p[:, 1]),
        z=np.ascontiguousarray(p[:, 2]), m=np.full(n, 1.0 / n),
        h_init=np.full(n, h0), periodic=True, box=float(box),
        n_target=float(n_target), n_tol=float(n_tol),
        meta={"kind": "plummer_mixture", "seed": seed, "n_spheres": n_spheres,
              "sphere_counts": counts, "scale_radii": a},
    )


def group_sizes(n_groups: int, seed: int, lo: int = 32, hi: int = 131072,
                slope: float = -2.0) -> np.ndarray:
    """Group sizes from dN/dn ~ n^slope on [lo, hi], rounded down to integers."""
    rng = _rng(seed)
    s = np.floor(_powerlaw(rng, n_groups, float(lo), float(hi), slope)).astype(np.int64)
    return np.clip(s, lo, hi)


def group_volume(p: np.ndarray) -> float:
    """Bounding-box volume of an (k, 3) point set: the product of the extents,
    each at least 2^-16 of the largest (the largest taken as 1 when all are 0)."""
    ext = p.max(axis=0) - p.min(axis=0)
    e = float(ext.max())
    if not e > 0.0:
        e = 1.0
    return float(np.prod(np.maximum(ext, e * 2.0 ** -16)))


def groups(n_groups: int, seed: int, lo: int = 32, hi: int = 131072,
           slope: float = -2.0, a_range=(0.005, 0.05), n_target: float = 32.0,
           n_tol: float = 1.0, sizes: np.ndarray | None = None) -> ParticleSet:
    """Independent isolated Plummer groups, concatenated with CSR offsets.

    Each group is one Plummer sphere (random log-uniform scale radius) centred
    at a random point of the unit cube.  Masses are equal, 1/N_total.  The
    initial smoothing length of a group is 2 (V_g / n_g)^(1/3) with V_g the
    volume of the group's bounding box.
    """
    if sizes is None:
        sizes = group_sizes(n_groups, seed, lo, hi, slope)
    rng = _rng(seed + 1_000_003)
    sizes = np.asarray(sizes, dtype=np.int64)
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    n = int(offsets[-1])
    x = np.empty(n)
    y = np.empty(n)
    z = np.empty(n)
    h0 = np.empty(n)
    for g, k in enumerate(sizes):
        k = int(k)
        a = float(np.exp(rng.random() * (np.log(a_range[1]) - np.log(a_range[0])) + np.log(a_range[0])))
        c = rng.random(3)
        p = c + plummer_radii(rng, k, a)[:, None] * _isotropic(rng, k)
        sl = slice(int(offsets[g]), int(offsets[g + 1]))
        x[sl], y[sl], z[sl] = p[:, 0], p[:, 1], p[:, 2]
        if k == 0:
            continue
        h0[sl] = default_h_init(k, group_volume(p))
    return ParticleSet(
        x=x, y=y, z=z, m=np.full(n, 1.0 / n), h_init=h0, periodic=False,
        box=1.0, n_target=float(n_target), n_tol=float(n_tol), offsets=offsets,
        meta={"kind": "groups", "seed": seed, "sizes": sizes},
    )


def doubled(ps: ParticleSet) -> ParticleSet:
    """Every particle twice at the same position (copies 2i and 2i+1 of
    particle i), each of half the mass, with the target count and its band
    doubled.  Groups stay contiguous (offsets doubled)."""
    rep = lambda a: np.ascontiguousarray(np.repeat(np.asarray(a, dtype=np.float64), 2))
    return ParticleSet(
        x=rep(ps.x), y=rep(ps.y), z=rep(ps.z), m=rep(ps.m) * 0.5, h_init=rep(ps.h_init),
        periodic=ps.periodic, box=ps.box, n_target=2.0 * ps.n_target,
        n_tol=2.0 * ps.n_tol,
        offsets=None if ps.offsets is None else np.asarray(ps.offsets, dtype=np.int64) * 2,
        meta={**ps.meta, "doubled": True},
    )


def with_duplicates(ps: ParticleSet, n_dup: int, seed: int) -> ParticleSet:
    """A periodic set with ``n_dup`` distinct particles, drawn at random, given
    a second particle at exactly the same position (appended after the
    originals); all masses 1/N of the new count."""
    if ps.offsets is not None:
        raise ValueError("with_duplicates takes one periodic set")
    src = np.sort(_rng(seed).choice(ps.n, size=n_dup, replace=False))
    cat = lambda a: np.ascontiguousarray(np.concatenate([a, a[src]]))
    n = ps.n + n_dup
    return ParticleSet(
        x=cat(ps.x), y=cat(ps.y), z=cat(ps.z), m=np.full(n, 1.0 / n),
        h_init=cat(ps.h_init), periodic=True, box=ps.box, n_target=ps.n_target,
        n_tol=ps.n_tol, meta={**ps.meta, "duplicates": n_dup, "dup_seed": seed,
                              "dup_of": src},
    )


def cotangent(n: int, seed: int) -> np.ndarray:
    """Standard-normal cotangent on rho (one value per particle)."""
    return _rng(seed).standard_normal(n)


def config(name: str, scale: float = 1.0) -> ParticleSet:
    """The named benchmark inputs.

    ``uniform4096``: 4096 uniform particles, h_init 0.125, N_t = 64 +- 2.
    ``clustered2^20``: 2^20 particles, 200 Plummer spheres + 30% background,
    N_t = 64 +- 2.  ``clustered2^24``: 2^24 particles, 2000 spheres, contrast
    at most 1e5, N_t = 64 +- 1.  ``groups10k``: 10,000 isolated groups with
    sizes ~ n^-2 on [32, 131072], N_t = 32 +- 1 (about 2.2e6 particles).
    ``groups10k_a1554``: the same with sizes ~ n^-1.554, the slope whose
    expected total is the ~1.6e7 particles the group-finding workload is
    quoted at (the literal slope -2 gives ~2.7e6).  ``scale`` < 1 shrinks the
    particle counts (test-sized variants keep the same recipe).
    """
    if name == "uniform4096":
        return uniform(int(4096 * scale), seed=1, n_target=64.0, n_tol=2.0,
                       h_init=0.125 if scale == 1.0 else None)
    if name == "clustered2^20":
        n = int((1 << 20) * scale)
        return plummer_mixture(n, max(1, int(round(200 * min(1.0, scale * 8)))), seed=2,
                               n_target=64.0, n_tol=2.0)
    if name == "clustered2^24":
        n = int((1 << 24) * scale)
        return plummer_mixture(n, max(1, int(round(2000 * min(1.0, scale * 8)))), seed=3,
                               contrast_cap=1e5, n_target=64.0, n_tol=1.0)
    if name == "groups10k":
        g = max(1, int(round(10000 * scale)))
        return groups(g, seed=4, n_target=32.0, n_tol=1.0)
    if name == "groups10k_a1554":
        g = max(1, int(round(10000 * scale)))
        return groups(g, seed=4, slope=-1.554, n_target=32.0, n_tol=1.0)
    raise KeyError(name)
