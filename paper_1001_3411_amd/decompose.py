"""Spatial decomposition of a periodic box into padded subvolumes for the
batched call (the paper's section 3.1 and its load-balancing and
directional-padding subsections): the host-side front end that turns one
box into the per-task inputs of ``HopContext.run_batch``.

* Load balancing: the task count's prime factors, largest first, give the
  cutting rounds; a round cuts every current subvolume into that many
  slabs holding equal numbers of a random subsample of the particles,
  cycling the axis x, y, z like a kd-tree (a power of two is plain
  bisection).
* Padding (Eq. 1): L_p = s (N_dens V / N)^(1/3) for a subvolume of volume V
  holding N particles.  Directional padding: for each face, the particles
  of the subvolume within L_p of that face give the spacing near it,
  L_face = s (N_dens V_face / N_face)^(1/3) with V_face the volume of that
  slab.
* Each subvolume is then cut out of the box with its six paddings
  (periodic wrap), moved to a frame of its own starting at the padded
  box's low corner, and its padding particles flagged.

Coordinates are integers in [0, 2^grid_bits); every box bound is an
integer.  This is host logic (NumPy) on the caller's particles; the
search and everything after it run in the HIP kernels of the batched call.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = ["prime_factors", "cut_boxes", "paddings", "Decomposition", "decompose"]


def prime_factors(p: int) -> list[int]:
    """Prime factors of p, largest first (with multiplicity)."""
    if p < 1:
        raise ValueError("task count must be >= 1")
    out, f = [], 2
    while f * f <= p:
        while p % f == 0:
            out.append(f)
            p //= f
        f += 1
    if p > 1:
        out.append(p)
    return sorted(out, reverse=True)


def cut_boxes(sample: np.ndarray, n_tasks: int, grid_bits: int = 21) -> np.ndarray:
    """Boxes [n_tasks][2][3] (lo, hi; hi exclusive) of the load-balanced
    decomposition of [0, 2^grid_bits)^3 computed on the sample points."""
    G = 1 << grid_bits
    sample = np.asarray(sample, dtype=np.int64)
    regions = [(np.zeros(3, np.int64), np.full(3, G, np.int64), sample)]
    for r, k in enumerate(prime_factors(n_tasks)):
        dim = r % 3
        nxt = []
        for lo, hi, pts in regions:
            srt = np.sort(pts[:, dim])
            m = srt.size
            edges = [int(lo[dim])]
            for j in range(1, k):
                if m == 0:
                    c = int(lo[dim] + (hi[dim] - lo[dim]) * j // k)
                else:
                    a = srt[min(m - 1, max(0, (j * m) // k - 1))]
                    b = srt[min(m - 1, (j * m) // k)]
                    c = int((a + b + 1) // 2)  # between the two sample points
                c = min(max(c, edges[-1] + 1), int(hi[dim]) - (k - j))
                edges.append(c)
            edges.append(int(hi[dim]))
            for j in range(k):
                l2, h2 = lo.copy(), hi.copy()
                l2[dim], h2[dim] = edges[j], edges[j + 1]
                sel = (pts[:, dim] >= edges[j]) & (pts[:, dim] < edges[j + 1])
                nxt.append((l2, h2, pts[sel]))
        regions = nxt
    return np.array([[lo, hi] for lo, hi, _ in regions], dtype=np.int64)


def _in_box(pos, lo, hi):
    return np.all((pos >= lo) & (pos < hi), axis=1)


def paddings(pos: np.ndarray, boxes: np.ndarray, n_dens: int = 64, safety: float = 1.5,
             directional: bool = True) -> np.ndarray:
    """Padding widths [n_tasks][2][3] (below lo, above hi per axis), integer
    grid units rounded up, from Eq. (1) and, if directional, per face."""
    pos = np.asarray(pos, dtype=np.int64)
    out = np.zeros((len(boxes), 2, 3), np.int64)
    for t, (lo, hi) in enumerate(boxes):
        inside = pos[_in_box(pos, lo, hi)]
        n = max(inside.shape[0], 1)
        V = float(np.prod((hi - lo).astype(np.float64)))
        lp = safety * (n_dens * V / n) ** (1.0 / 3.0)
        for side in (0, 1):
            for d in range(3):
                width = float(hi[d] - lo[d])
                L = lp
                if directional:
                    t_slab = min(lp, width)
                    if side == 0:
                        sel = inside[:, d] < lo[d] + t_slab
                    else:
                        sel = inside[:, d] >= hi[d] - t_slab
                    nf = int(np.count_nonzero(sel))
                    area = V / width
                    if nf > 0:
                        L = safety * (n_dens * area * t_slab / nf) ** (1.0 / 3.0)
                out[t, side, d] = int(np.ceil(L))
    return out


@dataclass
class Decomposition:
    boxes: np.ndarray     # [T][2][3] local (core) boxes, hi exclusive
    pads: np.ndarray      # [T][2][3] padding below lo and above hi
    offsets: np.ndarray   # [T+1] row ranges of the concatenated batch
    pos: np.ndarray       # [rows][3] uint32, each subvolume in its own frame
    padded: np.ndarray    # [rows] uint8, 1 = padding particle
    index: np.ndarray     # [rows] int64, the particle's index in the box
    origin: np.ndarray    # [T][3] frame origin (padded low corner) in box units


def decompose(pos: np.ndarray, n_tasks: int, grid_bits: int = 21, n_dens: int = 64,
              safety: float = 1.5, sample_frac: float = 0.03, seed: int = 0,
              directional: bool = True) -> Decomposition:
    """Load-balanced, padded subvolumes of a periodic box, ready for the
    batched call (run each as a non-periodic frame with the box's mean
    density)."""
    G = 1 << grid_bits
    pos = np.ascontiguousarray(pos, dtype=np.uint32)
    n = pos.shape[0]
    rng = np.random.default_rng(seed)
    m = max(1, min(n, int(round(sample_frac * n))))
    sample = pos[rng.choice(n, m, replace=False)]
    boxes = cut_boxes(sample, n_tasks, grid_bits)
    pads = paddings(pos, boxes, n_dens, safety, directional)
    p64 = pos.astype(np.int64)
    rows_pos, rows_pad, rows_idx, offs, origins = [], [], [], [0], []
    for t in range(len(boxes)):
        lo, hi = boxes[t]
        org = lo - pads[t, 0]
        span = (hi - lo) + pads[t, 0] + pads[t, 1]
        if np.any(span >= G):
            raise ValueError("padding wider than the box: use more particles or fewer tasks")
        rel = np.mod(p64 - org, G)
        sel = np.all(rel < span, axis=1)
        idx = np.flatnonzero(sel)
        core = _in_box(p64[idx], lo, hi)
        rows_pos.append(rel[idx].astype(np.uint32))
        rows_pad.append((~core).astype(np.uint8))
        rows_idx.append(idx)
        offs.append(offs[-1] + idx.size)
        origins.append(np.mod(org, G))
    return Decomposition(boxes=boxes, pads=pads, offsets=np.array(offs, np.int64),
                         pos=np.concatenate(rows_pos), padded=np.concatenate(rows_pad),
                         index=np.concatenate(rows_idx), origin=np.array(origins, np.int64))
