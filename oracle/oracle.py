"""ctypes wrapper of the C oracle (test infrastructure only).

Every function takes and returns NumPy arrays.  Semantics follow the paper's
section 2 (HOP) and section 3.1 (per-task rules); the C source states the
readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

__all__ = [
    "lib", "knn", "density", "norm", "hop", "chains", "saddles", "merge", "labels",
    "run", "run_lite", "Lite", "stages", "subhalos", "Subhalos", "OracleResult", "LiteResult", "num_threads",
    "set_threads", "HopParams",
]

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        i64, i32, f64, vp = C.c_int64, C.c_int, C.c_double, C.c_void_p
        L.orc_knn_brute.argtypes = [i64, vp, vp, i32, i32, i32, vp, i64, vp, vp]
        L.orc_knn_kdtree.argtypes = [i64, vp, vp, i32, i32, i32, vp, i64, vp, vp]
        L.orc_density.argtypes = [i64, i32, vp, f64, vp]
        L.orc_norm.argtypes = [f64]
        L.orc_norm.restype = f64
        L.orc_hop.argtypes = [i64, i32, i32, vp, vp, vp, vp, i32, vp]
        L.orc_chains.argtypes = [i64, vp, vp, vp, f64, vp, vp, vp, vp, vp]
        L.orc_saddles.argtypes = [i64, i32, i32, vp, vp, vp, vp, i32, vp, vp, vp, i64, vp]
        L.orc_merge.argtypes = [i64, vp, i64, vp, vp, vp, f64, f64, vp]
        L.orc_labels.argtypes = [i64, vp, i64, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp]
        L.orc_run.argtypes = [i64, vp, vp, vp, i32, i32, i32, i32, i32, i32, f64, f64, f64, f64,
                              i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_run_lite.argtypes = [i64, vp, vp, vp, i32, i32, i32, i32, i32, i32, i32, f64, f64,
                                   f64, f64, i32, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                   vp, vp]
        L.orc_lite_begin.argtypes = [i64, vp, vp, i32, i32, i32, i32, i32, f64]
        L.orc_lite_begin.restype = vp
        L.orc_lite_query.argtypes = [vp, i64, i64, vp, vp, vp, vp]
        L.orc_lite_end.argtypes = [vp]
        L.orc_lite_end.restype = None
        L.orc_stages.argtypes = [i64, vp, vp, i32, i32, i32, f64, f64, f64, i32, vp, vp, vp, vp,
                                 vp, vp, vp, vp, vp, vp]
        L.orc_subhalos.argtypes = [i64, i32, i32, vp, vp, vp, i64, vp, vp, i32, f64, vp, vp, vp,
                                   vp, vp, vp, vp]
        L.orc_num_threads.restype = i32
        L.orc_set_threads.argtypes = [i32]
        L.orc_set_threads.restype = None
        _LIB = L
    return _LIB


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    lib().orc_set_threads(int(n))


@dataclass
class HopParams:
    """HOP parameters (section 4.1 and Table 2 of the paper)."""
    n_dens: int = 64
    n_hop: int = 16
    n_merge: int = 4
    k_store: int = 64
    delta_outer: float = 80.0
    delta_saddle: float = 200.0
    delta_peak: float = 240.0
    grid_bits: int = 21


def knn(pos, k, periodic=True, ids=None, queries=None, method="kdtree", grid_bits=21):
    """Neighbour lists (self first, then by (d^2, id, index)) and their d^2."""
    pos = _c(pos, np.uint32)
    n = pos.shape[0]
    q = _c(queries, np.int64)
    nq = n if q is None else q.shape[0]
    nbr = np.empty((nq, k), np.int32)
    d2 = np.empty((nq, k), np.int64)
    f = lib().orc_knn_kdtree if method == "kdtree" else lib().orc_knn_brute
    _check(f(n, _p(pos), _p(_c(ids, np.int64)), int(periodic), grid_bits, k, _p(q), nq,
             _p(nbr), _p(d2)), "knn")
    return nbr, d2


def norm(mean_density: float) -> float:
    return float(lib().orc_norm(mean_density))


def density(d2, mean_density):
    d2 = _c(d2, np.int64)
    nq, k = d2.shape
    out = np.empty(nq, np.float64)
    _check(lib().orc_density(nq, k, _p(d2), float(mean_density), _p(out)), "density")
    return out


def hop(nbr, dens, n_hop, ids=None, padded=None, padded_rules=False):
    nbr = _c(nbr, np.int32)
    n, ks = nbr.shape
    out = np.empty(n, np.int32)
    _check(lib().orc_hop(n, ks, n_hop, _p(nbr), _p(_c(dens, np.float64)), _p(_c(ids, np.int64)),
                         _p(_c(padded, np.uint8)), int(padded_rules), _p(out)), "hop")
    return out


def chains(hop_, dens, delta_outer, ids=None):
    hop_ = _c(hop_, np.int32)
    n = hop_.shape[0]
    root = np.empty(n, np.int32)
    chain_of = np.empty(n, np.int32)
    croot = np.empty(max(n, 1), np.int32)
    cpeak = np.empty(max(n, 1), np.float64)
    nc = np.zeros(1, np.int64)
    _check(lib().orc_chains(n, _p(hop_), _p(_c(dens, np.float64)), _p(_c(ids, np.int64)),
                            float(delta_outer), _p(root), _p(chain_of), _p(croot), _p(cpeak),
                            _p(nc)), "chains")
    c = int(nc[0])
    return root, chain_of, croot[:c].copy(), cpeak[:c].copy()


def saddles(nbr, dens, chain_of, n_merge, padded=None, padded_rules=False):
    nbr = _c(nbr, np.int32)
    n, ks = nbr.shape
    cap = n * max(n_merge - 1, 1) + 1
    lo = np.empty(cap, np.int32)
    hi = np.empty(cap, np.int32)
    s = np.empty(cap, np.float64)
    ne = np.zeros(1, np.int64)
    _check(lib().orc_saddles(n, ks, n_merge, _p(nbr), _p(_c(dens, np.float64)),
                             _p(_c(chain_of, np.int32)), _p(_c(padded, np.uint8)),
                             int(padded_rules), _p(lo), _p(hi), _p(s), cap, _p(ne)), "saddles")
    e = int(ne[0])
    return lo[:e].copy(), hi[:e].copy(), s[:e].copy()


def merge(chain_peak, e_lo, e_hi, e_s, delta_saddle, delta_peak):
    cp = _c(chain_peak, np.float64)
    nc = cp.shape[0]
    out = np.empty(max(nc, 1), np.int32)
    e_lo, e_hi, e_s = _c(e_lo, np.int32), _c(e_hi, np.int32), _c(e_s, np.float64)
    _check(lib().orc_merge(nc, _p(cp), e_lo.shape[0], _p(e_lo), _p(e_hi), _p(e_s),
                           float(delta_saddle), float(delta_peak), _p(out)), "merge")
    return out[:nc].copy()


def labels(chain_of, chain_root, chain_peak, chain_halo, ids=None, padded=None,
           padded_rules=False):
    chain_of = _c(chain_of, np.int32)
    n = chain_of.shape[0]
    nc = len(chain_root)
    group = np.empty(n, np.int32)
    ng = np.zeros(1, np.int64)
    cap = max(nc, 1)
    gc = np.empty(cap, np.int64)
    gp = np.empty(cap, np.int32)
    gd = np.empty(cap, np.float64)
    _check(lib().orc_labels(n, _p(chain_of), nc, _p(_c(chain_root, np.int32)),
                            _p(_c(chain_peak, np.float64)), _p(_c(chain_halo, np.int32)),
                            _p(_c(ids, np.int64)), _p(_c(padded, np.uint8)), int(padded_rules),
                            _p(group), _p(ng), _p(gc), _p(gp), _p(gd)), "labels")
    g = int(ng[0])
    return group, gc[:g].copy(), gp[:g].copy(), gd[:g].copy()


@dataclass
class OracleResult:
    density: np.ndarray
    nbr: np.ndarray
    hop: np.ndarray
    root: np.ndarray
    chain_of: np.ndarray
    group: np.ndarray
    g_count: np.ndarray
    g_peak: np.ndarray
    g_peak_dens: np.ndarray
    n_chains: int
    n_edges: int
    n_groups: int


def run(pos, periodic=True, mean_density=None, params: HopParams | None = None, ids=None,
        padded=None, padded_rules=False, search="kdtree") -> OracleResult:
    """The whole pipeline: density, links, chains, boundaries, merge, labels."""
    p = params or HopParams()
    pos = _c(pos, np.uint32)
    n = pos.shape[0]
    if mean_density is None:
        mean_density = n / float(1 << (3 * p.grid_bits))
    dens = np.empty(n, np.float64)
    nbr = np.empty((n, p.k_store), np.int32)
    hop_ = np.empty(n, np.int32)
    root = np.empty(n, np.int32)
    chain_of = np.empty(n, np.int32)
    group = np.empty(n, np.int32)
    gc = np.empty(max(n, 1), np.int64)
    gp = np.empty(max(n, 1), np.int32)
    gd = np.empty(max(n, 1), np.float64)
    counts = np.zeros(3, np.int64)
    _check(lib().orc_run(n, _p(pos), _p(_c(ids, np.int64)), _p(_c(padded, np.uint8)),
                         int(periodic), p.grid_bits, p.n_dens, p.n_hop, p.n_merge, p.k_store,
                         p.delta_outer, p.delta_saddle, p.delta_peak, float(mean_density),
                         int(padded_rules), 1 if search == "kdtree" else 0,
                         _p(dens), _p(nbr), _p(hop_), _p(root), _p(chain_of), _p(group),
                         _p(gc), _p(gp), _p(gd), _p(counts)), "run")
    g = int(counts[2])
    return OracleResult(dens, nbr, hop_, root, chain_of, group, gc[:g].copy(), gp[:g].copy(),
                        gd[:g].copy(), int(counts[0]), int(counts[1]), g)


@dataclass
class LiteResult:
    density: np.ndarray
    nbr: np.ndarray        # [n][k_keep] list heads
    row_hash: np.ndarray   # [n] uint64 fingerprint of the first k_store entries
    r2max: np.ndarray      # [n] d^2 to the N_dens-th entry
    hop: np.ndarray
    root: np.ndarray
    chain_of: np.ndarray
    group: np.ndarray
    g_count: np.ndarray
    g_peak: np.ndarray
    g_peak_dens: np.ndarray
    n_chains: int
    n_edges: int
    n_groups: int


def run_lite(pos, periodic=True, mean_density=None, params: HopParams | None = None, ids=None,
             padded=None, padded_rules=False, k_keep=16, chunk=1 << 20) -> LiteResult:
    """orc_run in bounded memory: list heads, row fingerprints, all other outputs."""
    p = params or HopParams()
    pos = _c(pos, np.uint32)
    n = pos.shape[0]
    if mean_density is None:
        mean_density = n / float(1 << (3 * p.grid_bits))
    dens = np.empty(n, np.float64)
    nbr = np.empty((n, k_keep), np.int32)
    rh = np.empty(n, np.uint64)
    r2 = np.empty(n, np.int64)
    hop_ = np.empty(n, np.int32)
    root = np.empty(n, np.int32)
    chain_of = np.empty(n, np.int32)
    group = np.empty(n, np.int32)
    gc = np.empty(max(n, 1), np.int64)
    gp = np.empty(max(n, 1), np.int32)
    gd = np.empty(max(n, 1), np.float64)
    counts = np.zeros(3, np.int64)
    _check(lib().orc_run_lite(n, _p(pos), _p(_c(ids, np.int64)), _p(_c(padded, np.uint8)),
                              int(periodic), p.grid_bits, p.n_dens, p.n_hop, p.n_merge,
                              p.k_store, int(k_keep), p.delta_outer, p.delta_saddle,
                              p.delta_peak, float(mean_density), int(padded_rules), int(chunk),
                              _p(dens), _p(nbr), _p(rh), _p(r2), _p(hop_), _p(root),
                              _p(chain_of), _p(group), _p(gc), _p(gp), _p(gd), _p(counts)),
           "run_lite")
    g = int(counts[2])
    return LiteResult(dens, nbr, rh, r2, hop_, root, chain_of, group, gc[:g].copy(),
                      gp[:g].copy(), gd[:g].copy(), int(counts[0]), int(counts[1]), g)


def stages(nbr, dens, params: HopParams | None = None, ids=None, padded=None,
           padded_rules=False):
    """Stages 3-7 (links, chains, boundaries, merge, labels) from densities and
    the first list columns; returns (hop, root, chain_of, group, g_count,
    g_peak, g_peak_dens, n_chains, n_edges, n_groups)."""
    p = params or HopParams()
    nbr = _c(nbr, np.int32)
    n, kc = nbr.shape
    hop_ = np.empty(n, np.int32)
    root = np.empty(n, np.int32)
    chain_of = np.empty(n, np.int32)
    group = np.empty(n, np.int32)
    gc = np.empty(max(n, 1), np.int64)
    gp = np.empty(max(n, 1), np.int32)
    gd = np.empty(max(n, 1), np.float64)
    counts = np.zeros(3, np.int64)
    _check(lib().orc_stages(n, _p(_c(ids, np.int64)), _p(_c(padded, np.uint8)), p.n_hop,
                            p.n_merge, kc, p.delta_outer, p.delta_saddle, p.delta_peak,
                            int(padded_rules), _p(_c(dens, np.float64)), _p(nbr), _p(hop_),
                            _p(root), _p(chain_of), _p(group), _p(gc), _p(gp), _p(gd),
                            _p(counts)), "stages")
    g = int(counts[2])
    return (hop_, root, chain_of, group, gc[:g].copy(), gp[:g].copy(), gd[:g].copy(),
            int(counts[0]), int(counts[1]), g)


class Lite:
    """Incremental bounded-memory pipeline: the kd-tree is built on creation,
    query(c0, c1) searches the particles at tree positions [c0, c1), and
    finish() runs the later stages.  Outputs fill the arrays held here."""

    def __init__(self, pos, periodic=True, mean_density=None, params: HopParams | None = None,
                 ids=None, k_keep=16):
        self.p = params or HopParams()
        self.pos = _c(pos, np.uint32)
        self.ids = _c(ids, np.int64)
        self.n = n = self.pos.shape[0]
        if mean_density is None:
            mean_density = n / float(1 << (3 * self.p.grid_bits))
        self.density = np.empty(n, np.float64)
        self.nbr = np.empty((n, k_keep), np.int32)
        self.row_hash = np.empty(n, np.uint64)
        self.r2max = np.empty(n, np.int64)
        self.h = lib().orc_lite_begin(n, _p(self.pos), _p(self.ids), int(periodic),
                                      self.p.grid_bits, self.p.n_dens, self.p.k_store,
                                      int(k_keep), float(mean_density))
        if not self.h:
            raise RuntimeError("oracle lite_begin failed")

    def query(self, c0, c1):
        _check(lib().orc_lite_query(self.h, int(c0), int(c1), _p(self.density), _p(self.nbr),
                                    _p(self.row_hash), _p(self.r2max)), "lite_query")

    def close(self):
        if self.h:
            lib().orc_lite_end(self.h)
            self.h = None

    def finish(self, padded=None, padded_rules=False):
        self.close()
        return stages(self.nbr, self.density, self.p, ids=self.ids, padded=padded,
                      padded_rules=padded_rules)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Subhalos:
    sub: np.ndarray        # [n_levels][n] structure number per level or -1
    t_off: np.ndarray      # [n_levels + 1] table offsets
    count: np.ndarray
    peak: np.ndarray
    peak_dens: np.ndarray
    parent: np.ndarray
    n_sym: int             # symmetric chain boundaries


def subhalos(nbr, dens, chain_of, n_chains, levels, n_merge=4, alpha=0.0, ids=None) -> Subhalos:
    """Subhalos at ascending levels (the readings are in the C source)."""
    nbr = _c(nbr, np.int32)
    n, kc = nbr.shape
    lv = np.ascontiguousarray(np.asarray(levels, dtype=np.float64))
    L = lv.size
    cap = max(L * int(n_chains), 1)
    sub = np.empty((L, n), np.int32)
    t_off = np.zeros(L + 1, np.int64)
    cnt = np.empty(cap, np.int64)
    pk = np.empty(cap, np.int32)
    pd = np.empty(cap, np.float64)
    par = np.empty(cap, np.int32)
    ns = np.zeros(1, np.int64)
    _check(lib().orc_subhalos(n, kc, int(n_merge), _p(nbr), _p(_c(dens, np.float64)),
                              _p(_c(chain_of, np.int32)), int(n_chains), _p(_c(ids, np.int64)),
                              _p(lv), L, float(alpha), _p(sub), _p(t_off), _p(cnt), _p(pk), _p(pd),
                              _p(par), _p(ns)), "subhalos")
    g = int(t_off[-1])
    return Subhalos(sub, t_off, cnt[:g].copy(), pk[:g].copy(), pd[:g].copy(), par[:g].copy(),
                    int(ns[0]))
