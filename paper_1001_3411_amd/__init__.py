"""MI355X HOP hot path: Python binding of the C ABI in include/hop.h.

The binding only marshals arguments: every stage runs in the HIP kernels of
libhop.so.  PyTorch supplies device memory and the current stream.  Loading
fails loudly when the library has not been built (run
``__graft_entry__.build()`` or ``python paper_1001_3411_amd/build.py``).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

__all__ = [
    "LIB_PATH", "load", "HopParams", "HopError", "HopContext", "HOP_PERIODIC",
    "HOP_DENSITY_FP32", "HOP_PADDED_RULES", "HOP_LEARNED_RADIUS", "HOP_RADIUS_MLP",
    "HOP_RADIUS_ANALYTIC", "HOP_MLP_PARAMS", "exported_symbols",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhop.so")

HOP_PERIODIC = 0x1
HOP_DENSITY_FP32 = 0x2
HOP_LEARNED_RADIUS = 0x8
HOP_RADIUS_MLP = 1
HOP_RADIUS_ANALYTIC = 2
HOP_MLP_PARAMS = 6017
HOP_PADDED_RULES = 0x4

ERRORS = {-1: "HOP_ERR_ARG", -2: "HOP_ERR_RANGE", -3: "HOP_ERR_DEGENERATE",
          -4: "HOP_ERR_CAPACITY", -5: "HOP_ERR_NOMEM", -6: "HOP_ERR_HIP"}


class HopError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Params(C.Structure):
    _fields_ = [("n_dens", C.c_int32), ("n_hop", C.c_int32), ("n_merge", C.c_int32),
                ("k_store", C.c_int32), ("delta_outer", C.c_double),
                ("delta_saddle", C.c_double), ("delta_peak", C.c_double),
                ("mean_density", C.c_double), ("grid_bits", C.c_uint32), ("flags", C.c_uint32)]


class _GroupInfo(C.Structure):
    _fields_ = [("count", C.c_int64), ("peak", C.c_int32), ("reserved", C.c_int32),
                ("peak_density", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("ms_sort", C.c_double), ("ms_knn", C.c_double), ("n", C.c_int64),
                ("nodes_visited", C.c_int64), ("leaves_scanned", C.c_int64),
                ("ms_radius", C.c_double), ("misses", C.c_int64), ("redo_buckets", C.c_int64),
                ("premerged", C.c_int64), ("insert_iterations", C.c_int64),
                ("offered", C.c_int64)]


@dataclass
class HopParams:
    """Section 4.1 / Table 2 parameters; defaults are the paper's thresholds
    (80, 2.5x, 3x) with N_dens = 64, N_hop = 16, N_merge = 4."""
    n_dens: int = 64
    n_hop: int = 16
    n_merge: int = 4
    k_store: int = 64
    delta_outer: float = 80.0
    delta_saddle: float = 200.0
    delta_peak: float = 240.0
    mean_density: float = 0.0
    grid_bits: int = 21
    periodic: bool = True
    padded_rules: bool = False
    density_fp32: bool = False
    learned_radius: bool = False

    def c(self) -> _Params:
        flags = (HOP_PERIODIC if self.periodic else 0) | \
                (HOP_PADDED_RULES if self.padded_rules else 0) | \
                (HOP_DENSITY_FP32 if self.density_fp32 else 0) | \
                (HOP_LEARNED_RADIUS if self.learned_radius else 0)
        return _Params(self.n_dens, self.n_hop, self.n_merge, self.k_store, self.delta_outer,
                       self.delta_saddle, self.delta_peak, self.mean_density, self.grid_bits,
                       flags)


class _Tuning(C.Structure):
    _fields_ = [("front_cap", C.c_int32), ("persistent_waves", C.c_int32),
                ("xcd_queues", C.c_int32), ("largest_first", C.c_int32),
                ("hash_slots", C.c_int32)]


_LIB = None


def load():
    """Load libhop.so; raises if it is missing (there is no fallback path)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    L.hop_params_default.argtypes = [C.POINTER(_Params)]
    L.hop_params_default.restype = None
    L.hop_ctx_create.argtypes = [C.c_int, C.POINTER(vp)]
    L.hop_ctx_destroy.argtypes = [vp]
    L.hop_ctx_destroy.restype = None
    L.hop_last_error.argtypes = [vp]
    L.hop_last_error.restype = C.c_char_p
    L.hop_density.argtypes = [vp, i64, vp, vp, C.POINTER(_Params), vp, vp, vp]
    L.hop_link.argtypes = [vp, i64, vp, vp, vp, vp, C.POINTER(_Params), vp, vp]
    L.hop_density_link.argtypes = [vp, i64, vp, vp, vp, C.POINTER(_Params), vp, vp, vp, vp]
    L.hop_groups.argtypes = [vp, i64, vp, vp, vp, C.POINTER(_Params), vp, vp,
                             C.POINTER(i32), vp]
    L.hop_merge.argtypes = [vp, i64, vp, vp, vp, vp, i32, vp, vp, C.POINTER(_Params), vp,
                            C.POINTER(i32), vp, vp]
    L.hop_halo_stats.argtypes = [vp, i64, vp, vp, vp, i32, vp, C.POINTER(_Params), vp, vp, vp, vp]
    L.hop_halo_stats_noalloc.argtypes = [vp, i64, vp, vp, vp, i32, vp, C.POINTER(_Params), vp,
                                         vp, vp, vp]
    L.hop_stitch.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, C.POINTER(_Params), i32, i64, vp,
                             vp, vp, vp, vp, C.POINTER(i32), C.POINTER(i32), vp, vp]
    L.hop_subhalos.argtypes = [vp, i64, vp, vp, vp, i32, vp, C.POINTER(_Params), i32, vp,
                               C.c_double, vp, vp, vp, vp]
    L.hop_run_batch.argtypes = [vp, i32, vp, vp, vp, vp, C.POINTER(_Params), vp, vp, vp, vp, vp,
                                vp, vp, vp, vp, vp, vp]
    f32 = C.c_float
    L.hop_radius_cell_bits.argtypes = [i64, C.c_uint32, f32]
    L.hop_radius_dataset.argtypes = [vp, i64, vp, vp, C.POINTER(_Params), i32, vp, vp, vp]
    L.hop_mlp_grad.argtypes = [vp, i64, vp, vp, vp, i32, vp, vp, vp, vp]
    L.hop_mlp_train.argtypes = [vp, i64, vp, vp, vp, i32, i32, i32, f32, f32, f32, f32, vp, vp,
                                vp, vp, vp]
    L.hop_radius_load.argtypes = [vp, i32, vp, f32, f32, vp]
    L.hop_radius_predict.argtypes = [vp, i64, vp, i32, vp, vp]
    L.hop_set_tuning.argtypes = [vp, C.POINTER(_Tuning)]
    L.hop_get_tuning.argtypes = [vp, C.POINTER(_Tuning)]
    L.hop_sync.argtypes = [vp, vp]
    L.hop_set_profiling.argtypes = [vp, C.c_int]
    L.hop_get_stats.argtypes = [vp, C.POINTER(_Stats)]
    _LIB = L
    return L


def exported_symbols():
    """Names of the C functions declared in include/hop.h."""
    import re
    hdr = os.path.join(os.path.dirname(HERE), "include", "hop.h")
    with open(hdr) as f:
        txt = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?(hop_\w+)\s*\(", txt, re.M)))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class HopContext:
    """One library context on one device (scratch memory lives here)."""

    def __init__(self, device: int = 0):
        import torch
        self._torch = torch
        self.lib = load()
        self.device = device
        h = C.c_void_p()
        rc = self.lib.hop_ctx_create(device, C.byref(h))
        if rc != 0:
            raise HopError(rc, "hop_ctx_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.hop_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ------------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            raise HopError(rc, self.lib.hop_last_error(self.h).decode())

    def _stream(self, stream):
        if stream is None:
            stream = self._torch.cuda.current_stream(self.device)
        return C.c_void_p(stream.cuda_stream)

    def _dev(self, t, dtype):
        torch = self._torch
        if t is None:
            return None
        if not isinstance(t, torch.Tensor):
            import numpy as np
            a = np.ascontiguousarray(t)
            if a.dtype == np.uint32:
                a = a.view(np.int32)  # same bits; the ABI reads uint32
            t = torch.from_numpy(a)
        return t.to(device=f"cuda:{self.device}", dtype=dtype).contiguous()

    # -- stages -------------------------------------------------------------
    def density(self, pos, params: HopParams | None = None, ids=None, want_nbr=True,
                stream=None):
        torch = self._torch
        p = params or HopParams()
        pos = self._dev(pos, torch.int32).view(torch.int32)
        n = pos.shape[0]
        ids = self._dev(ids, torch.int64)
        dens = torch.empty(n, dtype=torch.float64, device=pos.device)
        nbr = torch.empty((n, p.k_store), dtype=torch.int32, device=pos.device) if want_nbr else None
        cp = p.c()
        self._check(self.lib.hop_density(self.h, n, _ptr(pos), _ptr(ids), C.byref(cp), _ptr(dens),
                                         _ptr(nbr), self._stream(stream)))
        return dens, nbr

    def density_link(self, pos, params: HopParams | None = None, ids=None, padded=None,
                     want_nbr=True, stream=None):
        """hop_density_link: (density, nbr or None, hop) in one call."""
        torch = self._torch
        p = params or HopParams()
        pos = self._dev(pos, torch.int32).view(torch.int32)
        n = pos.shape[0]
        dens = torch.empty(n, dtype=torch.float64, device=pos.device)
        nbr = torch.empty((n, p.k_store), dtype=torch.int32, device=pos.device) if want_nbr else None
        hop = torch.empty(n, dtype=torch.int32, device=pos.device)
        cp = p.c()
        # converted inputs stay referenced until the call has enqueued its
        # work: a temporary freed earlier could be handed to the next one
        ids_d, pad_d = self._dev(ids, torch.int64), self._dev(padded, torch.uint8)
        self._check(self.lib.hop_density_link(self.h, n, _ptr(pos), _ptr(ids_d), _ptr(pad_d),
                                              C.byref(cp), _ptr(dens), _ptr(nbr), _ptr(hop),
                                              self._stream(stream)))
        return dens, nbr, hop

    def link(self, nbr, dens, params: HopParams | None = None, ids=None, padded=None,
             stream=None):
        torch = self._torch
        p = params or HopParams()
        n = nbr.shape[0]
        hop = torch.empty(n, dtype=torch.int32, device=nbr.device)
        cp = p.c()
        ids_d, pad_d = self._dev(ids, torch.int64), self._dev(padded, torch.uint8)
        self._check(self.lib.hop_link(self.h, n, _ptr(nbr), _ptr(dens), _ptr(ids_d), _ptr(pad_d),
                                      C.byref(cp), _ptr(hop), self._stream(stream)))
        return hop

    def groups(self, hop, dens, params: HopParams | None = None, ids=None, stream=None):
        torch = self._torch
        p = params or HopParams()
        n = hop.shape[0]
        root = torch.empty(n, dtype=torch.int32, device=hop.device)
        chain_of = torch.empty(n, dtype=torch.int32, device=hop.device)
        nc = C.c_int32(0)
        cp = p.c()
        ids_d = self._dev(ids, torch.int64)
        self._check(self.lib.hop_groups(self.h, n, _ptr(hop), _ptr(dens), _ptr(ids_d), C.byref(cp),
                                        _ptr(root), _ptr(chain_of), C.byref(nc),
                                        self._stream(stream)))
        return root, chain_of, int(nc.value)

    def merge(self, nbr, dens, root, chain_of, n_chains, params: HopParams | None = None,
              ids=None, padded=None, want_table=True, stream=None):
        torch = self._torch
        p = params or HopParams()
        n = nbr.shape[0]
        group = torch.empty(n, dtype=torch.int32, device=nbr.device)
        table = None
        if want_table:
            table = torch.empty((max(n_chains, 1), 3), dtype=torch.int64, device=nbr.device)
        ng = C.c_int32(0)
        cp = p.c()
        ids_d, pad_d = self._dev(ids, torch.int64), self._dev(padded, torch.uint8)
        self._check(self.lib.hop_merge(self.h, n, _ptr(nbr), _ptr(dens), _ptr(root),
                                       _ptr(chain_of), n_chains, _ptr(ids_d), _ptr(pad_d),
                                       C.byref(cp), _ptr(group), C.byref(ng), _ptr(table),
                                       self._stream(stream)))
        g = int(ng.value)
        out = {"group": group, "n_groups": g}
        if want_table:
            t = table[:g]
            out["table"] = t
            out["g_count"] = t[:, 0].clone()
            out["g_peak"] = (t[:, 1] & 0xFFFFFFFF).to(torch.int32)
            out["g_peak_dens"] = t[:, 2].contiguous().view(torch.float64)
        return out

    def stitch(self, offsets, index, padded, batch, n, params: HopParams | None = None,
               premerge=False, task_densities=False, stream=None):
        """hop_stitch: whole-box chains and halos from the rows of a batched
        run (batch = run_batch() output; offsets host, index/padded per row).
        Returns device box arrays and the group table."""
        import numpy as np
        torch = self._torch
        p = params or HopParams()
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        idx_d = self._dev(index, torch.int64)
        pad_d = self._dev(padded, torch.uint8)
        dev = batch["density"].device
        out = {k: torch.empty(n, dtype=torch.int32, device=dev)
               for k in ("hop", "root", "chain_of", "group")}
        out["density"] = torch.empty(n, dtype=torch.float64, device=dev)
        table = torch.empty((max(int(off[-1]), 1), 3), dtype=torch.int64, device=dev)
        nc, ng = C.c_int32(0), C.c_int32(0)
        cp = p.c()
        self._check(self.lib.hop_stitch(self.h, off.size - 1, off.ctypes.data_as(C.c_void_p),
                                        _ptr(idx_d), _ptr(pad_d), _ptr(batch["density"]),
                                        _ptr(batch["nbr"]), _ptr(batch["hop"]), C.byref(cp),
                                        (1 if premerge else 0) | (2 if task_densities else 0),
                                        int(n), _ptr(out["density"]),
                                        _ptr(out["hop"]), _ptr(out["root"]), _ptr(out["chain_of"]),
                                        _ptr(out["group"]), C.byref(nc), C.byref(ng), _ptr(table),
                                        self._stream(stream)))
        g = int(ng.value)
        t = table[:g]
        out.update(n_chains=int(nc.value), n_groups=g, table=t, g_count=t[:, 0].clone(),
                   g_peak=(t[:, 1] & 0xFFFFFFFF).to(torch.int32),
                   g_peak_dens=t[:, 2].contiguous().view(torch.float64))
        return out

    def halo_stats(self, pos, group, table, params: HopParams | None = None, vel=None,
                   stream=None):
        """hop_halo_stats: per-halo centre of mass, maximum radius and (with
        vel) bulk velocity; table is merge()["table"]."""
        torch = self._torch
        p = params or HopParams()
        pos_d = self._dev(pos, torch.int32).view(torch.int32)
        vel_d = self._dev(vel, torch.float32)
        n = pos_d.shape[0]
        ng = table.shape[0]
        dev = pos_d.device
        com = torch.empty((max(ng, 1), 3), dtype=torch.float64, device=dev)
        rmax = torch.empty(max(ng, 1), dtype=torch.float64, device=dev)
        vbulk = torch.empty((max(ng, 1), 3), dtype=torch.float64, device=dev) if vel is not None else None
        cp = p.c()
        self._check(self.lib.hop_halo_stats(self.h, n, _ptr(pos_d), _ptr(vel_d), _ptr(group), ng,
                                            _ptr(table), C.byref(cp), _ptr(com), _ptr(rmax),
                                            _ptr(vbulk), self._stream(stream)))
        out = {"com": com[:ng], "rmax": rmax[:ng]}
        if vbulk is not None:
            out["vbulk"] = vbulk[:ng]
        return out

    def subhalos(self, nbr, dens, chain_of, n_chains, levels, params: HopParams | None = None,
                 alpha=0.0, ids=None, stream=None):
        """hop_subhalos: structure numbers per level [L][n] (device), host
        table offsets [L+1], and the device table [count, peak, parent,
        peak density] per structure."""
        import numpy as np
        torch = self._torch
        p = params or HopParams()
        lv = np.ascontiguousarray(np.asarray(levels, dtype=np.float64))
        L = lv.size
        n = nbr.shape[0]
        sub = torch.empty((L, n), dtype=torch.int32, device=nbr.device)
        t_off = np.zeros(L + 1, np.int64)
        table = torch.empty((max(L * n_chains, 1), 3), dtype=torch.int64, device=nbr.device)
        cp = p.c()
        ids_d = self._dev(ids, torch.int64)
        self._check(self.lib.hop_subhalos(self.h, n, _ptr(nbr), _ptr(dens), _ptr(chain_of),
                                          int(n_chains), _ptr(ids_d), C.byref(cp), L,
                                          lv.ctypes.data_as(C.c_void_p), float(alpha), _ptr(sub),
                                          t_off.ctypes.data_as(C.c_void_p), _ptr(table),
                                          self._stream(stream)))
        g = int(t_off[-1])
        t = table[:g]
        return {"sub": sub, "t_off": t_off.tolist(), "count": t[:, 0].clone(),
                "peak": (t[:, 1] & 0xFFFFFFFF).to(torch.int32),
                "parent": (t[:, 1] >> 32).to(torch.int32),
                "peak_dens": t[:, 2].contiguous().view(torch.float64)}

    def sync(self, stream=None):
        self._check(self.lib.hop_sync(self.h, self._stream(stream)))

    def run(self, pos, params: HopParams | None = None, ids=None, padded=None, stream=None,
            fused=True):
        """All four stages; returns a dict of device tensors.  fused: density
        and links in one hop_density_link call (else hop_density, hop_link)."""
        p = params or HopParams()
        if fused:
            dens, nbr, hop = self.density_link(pos, p, ids=ids, padded=padded, stream=stream)
        else:
            dens, nbr = self.density(pos, p, ids=ids, stream=stream)
            hop = self.link(nbr, dens, p, ids=ids, padded=padded, stream=stream)
        root, chain_of, nc = self.groups(hop, dens, p, ids=ids, stream=stream)
        out = self.merge(nbr, dens, root, chain_of, nc, p, ids=ids, padded=padded,
                         stream=stream)
        out.update(density=dens, nbr=nbr, hop=hop, root=root, chain_of=chain_of, n_chains=nc)
        return out

    def run_batch(self, pos, offsets, params: HopParams | None = None, padded=None,
                  mean_density=None, stream=None):
        """The whole path for concatenated independent subvolumes (one call).

        pos: [n][3] coordinates of all subvolumes, subvolume s at rows
        offsets[s]:offsets[s+1]; padded: [n] flags or None; mean_density:
        one value per subvolume or None (each subvolume's own count).
        Returns device tensors with every index and number local to its
        subvolume, and host lists n_chains, n_groups, group_off.
        """
        import numpy as np
        torch = self._torch
        p = params or HopParams()
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        n_sub = off.size - 1
        pos = self._dev(pos, torch.int32).view(torch.int32)
        n = pos.shape[0]
        if n_sub < 1 or int(off[-1]) != n:
            raise HopError(-1, "offsets must end at the particle count")
        dev = pos.device
        padded = self._dev(padded, torch.uint8)
        md = None
        if mean_density is not None:
            md = np.ascontiguousarray(np.asarray(mean_density, dtype=np.float64))
            if md.size != n_sub:
                raise HopError(-1, "one mean density per subvolume")
        out = {
            "density": torch.empty(n, dtype=torch.float64, device=dev),
            "nbr": torch.empty((n, p.k_store), dtype=torch.int32, device=dev),
            "hop": torch.empty(n, dtype=torch.int32, device=dev),
            "root": torch.empty(n, dtype=torch.int32, device=dev),
            "chain_of": torch.empty(n, dtype=torch.int32, device=dev),
            "group": torch.empty(n, dtype=torch.int32, device=dev),
        }
        table = torch.empty((max(n, 1), 3), dtype=torch.int64, device=dev)
        nch = np.zeros(n_sub, np.int32)
        ngr = np.zeros(n_sub, np.int32)
        goff = np.zeros(n_sub + 1, np.int64)
        cp = p.c()
        hp = lambda a: None if a is None else C.c_void_p(a.ctypes.data)
        self._check(self.lib.hop_run_batch(
            self.h, n_sub, hp(off), _ptr(pos), _ptr(padded), hp(md), C.byref(cp),
            _ptr(out["density"]), _ptr(out["nbr"]), _ptr(out["hop"]), _ptr(out["root"]),
            _ptr(out["chain_of"]), _ptr(out["group"]), hp(nch), hp(ngr), _ptr(table), hp(goff),
            self._stream(stream)))
        g = int(goff[-1])
        t = table[:g]
        out["g_count"] = t[:, 0].clone()
        out["g_peak"] = (t[:, 1] & 0xFFFFFFFF).to(torch.int32)
        out["g_peak_dens"] = t[:, 2].contiguous().view(torch.float64)
        out.update(n_chains=nch.tolist(), n_groups=ngr.tolist(), group_off=goff.tolist(),
                   offsets=off.tolist())
        return out

    # -- learned search radius ----------------------------------------------
    def radius_dataset(self, pos, params: HopParams, cell_bits: int, nbr=None, stream=None):
        """Features [n][27] and (with nbr) targets [n] as float32 tensors."""
        torch = self._torch
        pos = self._dev(pos, torch.int32).view(torch.int32)
        n = pos.shape[0]
        feats = torch.empty((n, 27), dtype=torch.float32, device=pos.device)
        target = torch.empty(n, dtype=torch.float32, device=pos.device) if nbr is not None else None
        cp = params.c()
        self._check(self.lib.hop_radius_dataset(self.h, n, _ptr(pos), _ptr(nbr), C.byref(cp),
                                                int(cell_bits), _ptr(feats), _ptr(target),
                                                self._stream(stream)))
        return feats, target

    def mlp_grad(self, feats, target, w, batch=None, idx=None, stream=None):
        """(gradient [6017], loss) of the mean squared error over `batch` rows."""
        torch = self._torch
        if idx is not None:
            idx = idx.to(device=feats.device, dtype=torch.int32).contiguous()
            batch = idx.numel()
        batch = int(batch if batch is not None else feats.shape[0])
        grad = torch.empty(HOP_MLP_PARAMS, dtype=torch.float32, device=feats.device)
        loss = torch.empty(1, dtype=torch.float32, device=feats.device)
        self._check(self.lib.hop_mlp_grad(self.h, feats.shape[0], _ptr(feats), _ptr(target),
                                          _ptr(idx), batch, _ptr(w), _ptr(grad), _ptr(loss),
                                          self._stream(stream)))
        return grad, float(loss.item())

    def mlp_train(self, feats, target, w, m, v, idx, steps, batch, first_step=1, lr=1e-3,
                  beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        """Adam steps in place on w, m, v; returns the per-step losses."""
        torch = self._torch
        loss = torch.empty(max(int(steps), 1), dtype=torch.float32, device=feats.device)
        if idx is not None:
            idx = idx.to(device=feats.device, dtype=torch.int32).contiguous()
        self._check(self.lib.hop_mlp_train(self.h, feats.shape[0], _ptr(feats), _ptr(target),
                                           _ptr(idx), int(steps), int(batch), int(first_step),
                                           lr, beta1, beta2, eps, _ptr(w), _ptr(m), _ptr(v),
                                           _ptr(loss), self._stream(stream)))
        return loss[:int(steps)]

    def radius_load(self, kind, w=None, margin=0.0, occupancy=8.0, stream=None):
        self._check(self.lib.hop_radius_load(self.h, int(kind), _ptr(w), float(margin),
                                             float(occupancy), self._stream(stream)))

    def radius_predict(self, feats, n_dens=64, stream=None):
        torch = self._torch
        out = torch.empty(feats.shape[0], dtype=torch.float32, device=feats.device)
        self._check(self.lib.hop_radius_predict(self.h, feats.shape[0], _ptr(feats), int(n_dens),
                                                _ptr(out), self._stream(stream)))
        return out

    def set_tuning(self, **kw):
        """Change launch settings (front_cap, persistent_waves, xcd_queues,
        largest_first, hash_slots); results never depend on them."""
        t = _Tuning()
        self._check(self.lib.hop_get_tuning(self.h, C.byref(t)))
        for k, v in kw.items():
            if k not in dict(_Tuning._fields_):
                raise KeyError(k)
            setattr(t, k, int(v))
        self._check(self.lib.hop_set_tuning(self.h, C.byref(t)))

    def tuning(self) -> dict:
        t = _Tuning()
        self._check(self.lib.hop_get_tuning(self.h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in _Tuning._fields_}

    def set_profiling(self, on: bool):
        self._check(self.lib.hop_set_profiling(self.h, int(on)))

    def stats(self) -> dict:
        s = _Stats()
        self._check(self.lib.hop_get_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in _Stats._fields_}
