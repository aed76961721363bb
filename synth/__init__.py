"""Seeded synthetic particle sets for the HOP hot path.

This module only draws particle positions (and padded flags for subvolumes);
it contains none of the halo finder's arithmetic.  Both the CPU oracle tests
and the GPU path consume the arrays it returns, so every parity check runs on
bit-identical inputs.

The paper measures on ENZO dark-matter snapshots (D128, D512, D1024, 2048^3;
section 5) that are not available here.  The recipes below stand in for them:
clustered boxes made of NFW clumps on a uniform background, a Zel'dovich-like
displaced lattice, and padded non-periodic subvolumes shaped like one Parallel
HOP task's share (section 3.1).  Positions are quantised to an integer grid of
2^21 cells per axis, so squared distances are exact integers.

Conventions
-----------
* Unit box [0, 1)^3 -> uint32 grid coordinate ``floor(x * 2^21) mod 2^21``.
* After drawing, storage order is shuffled with the same seeded generator, so
  the particle index carries no spatial information.
* All draws use ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GRID_BITS = 21
GRID = 1 << GRID_BITS

__all__ = [
    "GRID_BITS", "GRID", "Particles", "quantise", "nfw_clumped_box",
    "zeldovich_box", "uniform_box", "lattice_box", "perturbed_lattice_box",
    "padded_subvolume", "subvolume_batch", "config", "tiny_case",
    "CONFIG_SIZES",
]


@dataclass
class Particles:
    """A particle set ready for the halo finder.

    pos:          uint32 [n, 3] grid coordinates, all < 2^grid_bits
    periodic:     True for a whole periodic box, False for a subvolume frame
    mean_density: particles per grid-unit^3 of the *global* volume
    padded:       uint8 [n] (1 = padding particle) or None
    """
    pos: np.ndarray
    periodic: bool
    mean_density: float
    padded: np.ndarray | None = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def quantise(x: np.ndarray, grid_bits: int = GRID_BITS) -> np.ndarray:
    """Unit-box float coordinates -> uint32 grid coordinates (periodic wrap)."""
    g = 1 << grid_bits
    q = np.floor(np.asarray(x, dtype=np.float64) * g).astype(np.int64)
    q %= g
    return q.astype(np.uint32)


# ---------------------------------------------------------------------------
# NFW clump sampling
# ---------------------------------------------------------------------------

def _nfw_m(x):
    return np.log1p(x) - x / (1.0 + x)


def _nfw_invert(t, c, iters=100):
    """Solve m(x) = t*m(c) for x in (0, c], vectorised safeguarded Newton.

    Converges to ~1e-13 relative in a handful of iterations; a bracket keeps
    every step inside (lo, hi).
    """
    target = t * _nfw_m(c)
    lo = np.zeros_like(c)
    hi = c.copy()
    # small-x start: m(x) ~ x^2/2
    x = np.minimum(np.sqrt(2.0 * target), 0.5 * c)
    x = np.where(x <= 0, 0.5 * c, x)
    for _ in range(iters):
        f = _nfw_m(x) - target
        lo = np.where(f < 0, x, lo)
        hi = np.where(f > 0, x, hi)
        fp = x / (1.0 + x) ** 2
        with np.errstate(divide="ignore", invalid="ignore"):
            xn = x - f / fp
        bad = ~np.isfinite(xn) | (xn < lo) | (xn > hi)
        xn = np.where(bad, 0.5 * (lo + hi), xn)
        done = np.max(np.abs(xn - x) / np.maximum(c, 1e-300)) < 1e-13
        x = xn
        if done:
            break
    return x


def _split_counts(weights: np.ndarray, total: int) -> np.ndarray:
    """Integer counts proportional to weights summing to total (largest remainders)."""
    if total <= 0 or weights.size == 0:
        return np.zeros(weights.size, dtype=np.int64)
    share = weights / weights.sum() * total
    base = np.floor(share).astype(np.int64)
    rem = total - int(base.sum())
    if rem > 0:
        order = np.argsort(-(share - base), kind="stable")
        base[order[:rem]] += 1
    return base


def _clump_points(rng, n_total_box, counts, centres, cmin=5.0, cmax=15.0):
    """Draw NFW particles for clumps with given counts and centres (unit box).

    r_vir = (3 n_k / (4 pi 200 N))^(1/3): mean overdensity 200 relative to the
    box's mean particle density, which fixes r_vir proportional to M^(1/3).
    Concentrations c ~ U[cmin, cmax]; radii by inverting the enclosed-mass
    profile; isotropic directions.
    """
    k = counts.size
    conc = rng.uniform(cmin, cmax, size=k)
    rvir = (3.0 * counts / (4.0 * math.pi * 200.0 * n_total_box)) ** (1.0 / 3.0)
    owner = np.repeat(np.arange(k), counts)
    m = owner.size
    u = rng.random(m)
    c_p = conc[owner]
    x = _nfw_invert(u, c_p)
    r = x / c_p * rvir[owner]
    # isotropic direction
    cz = rng.uniform(-1.0, 1.0, size=m)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=m)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    d = np.empty((m, 3))
    d[:, 0] = sz * np.cos(ph)
    d[:, 1] = sz * np.sin(ph)
    d[:, 2] = cz
    pts = centres[owner] + d * r[:, None]
    return pts, {"conc": conc, "rvir": rvir}


def _powerlaw_masses(rng, k, slope=-1.9, mmin=1.0, mmax=1000.0):
    """Inverse-CDF draws from dN/dM ~ M^slope on [mmin, mmax]."""
    a = slope + 1.0  # -0.9
    u = rng.random(k)
    lo, hi = mmin ** a, mmax ** a
    return (lo + u * (hi - lo)) ** (1.0 / a)


def nfw_clumped_box(n: int, n_clumps: int, seed: int, clump_frac: float = 0.7,
                    name: str = "") -> Particles:
    """Periodic box: clump_frac of n in NFW clumps, the rest uniform."""
    rng = np.random.default_rng(seed)
    n_clump = int(round(clump_frac * n))
    masses = _powerlaw_masses(rng, n_clumps)
    counts = _split_counts(masses, n_clump)
    centres = rng.random((n_clumps, 3))
    pts, meta = _clump_points(rng, n, counts, centres)
    bg = rng.random((n - n_clump, 3))
    allp = np.concatenate([pts, bg], axis=0)
    pos = quantise(allp)
    perm = rng.permutation(n)
    pos = np.ascontiguousarray(pos[perm])
    return Particles(pos=pos, periodic=True, mean_density=n / float(GRID) ** 3,
                     name=name or f"nfw_{n}_{n_clumps}_s{seed}",
                     meta={"counts": counts, **meta})


def zeldovich_box(n_side: int, seed: int, n_clumps: int = 5000,
                  clump_frac: float = 0.3, rms_cells: float = 0.5,
                  name: str = "") -> Particles:
    """Lattice displaced by a Gaussian field with P(k) ~ k^-2, plus NFW clumps.

    psi(k) = i k delta(k) / k^2 (Zel'dovich), scaled so that the 3-D rms
    displacement is rms_cells lattice spacings.  Then a seeded clump_frac of
    the particles is re-drawn into n_clumps NFW clumps, so the count stays
    n_side^3.
    """
    rng = np.random.default_rng(seed)
    ns = n_side
    n = ns ** 3
    white = rng.standard_normal((ns, ns, ns))
    wk = np.fft.rfftn(white)
    kx = np.fft.fftfreq(ns)[:, None, None]
    ky = np.fft.fftfreq(ns)[None, :, None]
    kz = np.fft.rfftfreq(ns)[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    amp = k2 ** (-0.5)          # sqrt(P(k)) with P ~ k^-2
    amp[0, 0, 0] = 0.0
    dk = wk * amp
    del wk, white
    disp = np.empty((n, 3), dtype=np.float64)
    for ax, kk in enumerate((kx, ky, kz)):
        comp = np.fft.irfftn(1j * kk * dk / k2, s=(ns, ns, ns), axes=(0, 1, 2))
        disp[:, ax] = comp.reshape(-1)
        del comp
    del dk
    rms = math.sqrt(float(np.mean(np.sum(disp * disp, axis=1))))
    if rms > 0:
        disp *= rms_cells / rms
    g = np.arange(ns, dtype=np.float64)
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    x = (lat + 0.5 + disp) / ns
    del lat, disp
    n_clump = int(round(clump_frac * n))
    sel = rng.permutation(n)[:n_clump]
    masses = _powerlaw_masses(rng, n_clumps)
    counts = _split_counts(masses, n_clump)
    centres = rng.random((n_clumps, 3))
    pts, meta = _clump_points(rng, n, counts, centres)
    x[sel] = pts
    pos = quantise(x)
    del x
    perm = rng.permutation(n)
    pos = np.ascontiguousarray(pos[perm])
    return Particles(pos=pos, periodic=True, mean_density=n / float(GRID) ** 3,
                     name=name or f"zeldovich_{ns}_s{seed}", meta=meta)


def uniform_box(n: int, seed: int) -> Particles:
    rng = np.random.default_rng(seed)
    pos = quantise(rng.random((n, 3)))
    return Particles(pos=pos, periodic=True, mean_density=n / float(GRID) ** 3,
                     name=f"uniform_{n}_s{seed}")


def lattice_box(n_side: int, seed: int | None = None) -> Particles:
    """Perfect simple-cubic lattice, spacing 2^21/n_side (n_side a power of 2)."""
    a = GRID // n_side
    g = np.arange(n_side, dtype=np.int64) * a
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    if seed is not None:
        lat = lat[np.random.default_rng(seed).permutation(lat.shape[0])]
    return Particles(pos=np.ascontiguousarray(lat.astype(np.uint32)), periodic=True,
                     mean_density=lat.shape[0] / float(GRID) ** 3,
                     name=f"lattice_{n_side}")


def perturbed_lattice_box(n_side: int, seed: int, jitter: float = 0.1) -> Particles:
    """Lattice with independent uniform jitter of +-jitter spacing per axis."""
    rng = np.random.default_rng(seed)
    g = np.arange(n_side, dtype=np.float64)
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    x = (lat + 0.5 + rng.uniform(-jitter, jitter, size=lat.shape)) / n_side
    pos = quantise(x)[rng.permutation(lat.shape[0])]
    return Particles(pos=np.ascontiguousarray(pos), periodic=True,
                     mean_density=pos.shape[0] / float(GRID) ** 3,
                     name=f"plattice_{n_side}_s{seed}")


# ---------------------------------------------------------------------------
# Padded subvolumes (one task's share in the paper's decomposition)
# ---------------------------------------------------------------------------

def padded_subvolume(n: int, seed: int, box_clumps_per_particle: float = 2000.0 / 2 ** 21,
                     clump_frac: float = 0.7, pad_frac: float = 0.1) -> Particles:
    """A non-periodic padded cube in its own 2^21 frame.

    The frame is the padded cube; the local cube is its central 1/(1+2*pad)
    part, so the padding shell is pad_frac of the local side on each face.
    Clumps follow the config-2 recipe scaled to n: K = max(1, round(n * c))
    clumps, with centres uniform in the frame and draws falling outside the
    frame rejected and redrawn.  Particles outside the local cube are padded.
    mean_density is n / 2^63, the frame's own mean density.
    """
    rng = np.random.default_rng(seed)
    k = max(1, int(round(box_clumps_per_particle * n)))
    n_clump = int(round(clump_frac * n))
    masses = _powerlaw_masses(rng, k)
    counts = _split_counts(masses, n_clump)
    centres = rng.random((k, 3))
    pts, _ = _clump_points(rng, n, counts, centres)
    # reject out-of-frame draws, refill from the same clumps
    for _ in range(64):
        bad = np.any((pts < 0.0) | (pts >= 1.0), axis=1)
        if not bad.any():
            break
        nb = int(bad.sum())
        owner = np.repeat(np.arange(k), counts)[bad]
        sub_counts = np.bincount(owner, minlength=k)
        redo, _ = _clump_points(rng, n, sub_counts, centres)
        pts[bad] = redo
    pts = np.clip(pts, 0.0, np.nextafter(1.0, 0.0))
    bg = rng.random((n - n_clump, 3))
    x = np.concatenate([pts, bg], axis=0)
    lo = pad_frac / (1.0 + 2.0 * pad_frac)
    hi = 1.0 - lo
    padded = np.any((x < lo) | (x >= hi), axis=1).astype(np.uint8)
    pos = np.minimum(np.floor(x * GRID), GRID - 1).astype(np.uint32)
    perm = rng.permutation(n)
    return Particles(pos=np.ascontiguousarray(pos[perm]), periodic=False,
                     mean_density=n / float(GRID) ** 3,
                     padded=np.ascontiguousarray(padded[perm]),
                     name=f"subvol_{n}_s{seed}")


def subvolume_batch(n_sub: int = 64, seed: int = 4000, median: float = 250_000.0,
                    sigma: float = 0.668, nmin: int = 50_000, nmax: int = 2_000_000,
                    scale: float = 1.0) -> list[Particles]:
    """Lognormal-sized padded subvolumes; seeds seed+s.  scale shrinks sizes."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(np.log(median) + sigma * rng.standard_normal(n_sub))
    sizes = np.clip(sizes, nmin, nmax) * scale
    sizes = np.maximum(sizes.astype(np.int64), 128)
    return [padded_subvolume(int(s), seed + i) for i, s in enumerate(sizes)]


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

CONFIG_SIZES = {1: 32_768, 2: 2_097_152, 3: 16_777_216, 5: 134_217_728}


def config(k: int, seed: int | None = None) -> Particles | list[Particles]:
    """The five workloads: 1..3 and 5 are periodic boxes, 4 is a subvolume batch."""
    if k == 1:
        return nfw_clumped_box(32_768, 20, seed if seed is not None else 1,
                               name="nfw32k_20clumps")
    if k == 2:
        return nfw_clumped_box(2_097_152, 2000, seed if seed is not None else 2,
                               name="nfw2m_2000clumps")
    if k == 3:
        return zeldovich_box(256, seed if seed is not None else 3,
                             name="zeldovich16m_5000clumps")
    if k == 4:
        return subvolume_batch(seed=seed if seed is not None else 4000)
    if k == 5:
        return nfw_clumped_box(134_217_728, 40_000, seed if seed is not None else 5,
                               name="nfw134m_40000clumps")
    raise ValueError(f"unknown config {k}")


def tiny_case(kind: str, n: int, seed: int) -> Particles:
    """Small inputs for brute-force checks: uniform, clustered, lattice, plattice."""
    if kind == "uniform":
        return uniform_box(n, seed)
    if kind == "clustered":
        return nfw_clumped_box(n, max(1, n // 400), seed)
    if kind == "lattice":
        side = round(n ** (1.0 / 3.0))
        return lattice_box(side, seed)
    if kind == "plattice":
        side = round(n ** (1.0 / 3.0))
        return perturbed_lattice_box(side, seed)
    raise ValueError(kind)
