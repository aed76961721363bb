"""Per-halo statistics of the HOP output -- test infrastructure only.

Only the test suite may import this module.  The paper lists, as each
task's output besides the group membership, a halo's particle count,
centre of mass, maximum radius and bulk velocity (section 3.1, output
step; section 5).  It gives no formulas; this is the reading used here,
written out plainly in FP64 and exact integers:

* members of halo g: the particles with group == g (padded particles carry
  -1 and belong to none);
* offsets are integer displacements from the halo's peak particle, taken
  as the minimum image in a periodic box of side G = 2^grid_bits (the
  representative in [-G/2, G/2)), plain differences otherwise, so that a
  halo straddling the boundary is unwrapped;
* centre of mass (unit masses): the peak's position plus m = (sum of the
  offsets) / count, the sum exact in integers and the quotient one
  correctly rounded FP64 division; wrapped into [0, G) when periodic;
* maximum radius: the largest member distance from the centre,
  sqrt((dx - mx)^2 + (dy - my)^2 + (dz - mz)^2) with every difference,
  product and sum rounded to FP64 in that order (x + y first) and a
  correctly rounded square root;
* bulk velocity: the mean member velocity, the FP64 sum of the velocities
  taken in index order divided by the count.
"""
import numpy as np

__all__ = ["halo_stats"]


def _offsets(pos, peak_pos, grid_bits, periodic):
    d = pos.astype(np.int64) - peak_pos.astype(np.int64)
    if periodic:
        G = np.int64(1) << grid_bits
        d = np.mod(d, G)
        d = np.where(d >= G // 2, d - G, d)
    return d


def halo_stats(pos, group, peak, grid_bits=21, periodic=True, vel=None):
    """pos [n][3] uint32, group [n] int32 (-1 = none), peak [G] int32 (the
    peak particle of each halo).  Returns count [G] int64, com [G][3] f64,
    rmax [G] f64 and, when vel ([n][3] float32) is given, vbulk [G][3] f64."""
    pos = np.ascontiguousarray(pos, dtype=np.uint32)
    group = np.asarray(group, dtype=np.int64)
    peak = np.asarray(peak, dtype=np.int64)
    ng = peak.size
    mem = np.flatnonzero(group >= 0)
    g = group[mem]
    d = _offsets(pos[mem], pos[peak[g]], grid_bits, periodic)
    count = np.bincount(g, minlength=ng).astype(np.int64)
    s = np.zeros((ng, 3), np.int64)
    for k in range(3):
        np.add.at(s[:, k], g, d[:, k])
    m = s.astype(np.float64) / count[:, None].astype(np.float64)
    com = pos[peak].astype(np.float64) + m
    if periodic:
        G = float(1 << grid_bits)
        com = np.where(com < 0.0, com + G, com)
        com = np.where(com >= G, com - G, com)
    e = d.astype(np.float64) - m[g]
    r = np.sqrt((e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1]) + e[:, 2] * e[:, 2])
    rmax = np.zeros(ng, np.float64)
    np.maximum.at(rmax, g, r)
    out = {"count": count, "com": com, "rmax": rmax}
    if vel is not None:
        v = np.asarray(vel, dtype=np.float32).astype(np.float64)
        vs = np.zeros((ng, 3), np.float64)
        for k in range(3):
            # index order: bincount accumulates sequentially over the input
            vs[:, k] = np.bincount(g, weights=v[mem, k], minlength=ng)
        out["vbulk"] = vs / count[:, None].astype(np.float64)
        out["vabs"] = np.stack([np.bincount(g, weights=np.abs(v[mem, k]), minlength=ng)
                                for k in range(3)], axis=1)
    return out
