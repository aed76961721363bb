"""CPU-side checks of the C ABI: the library builds, loads, and exports every
function that include/hop.h declares.  No compute call is made here."""
import ctypes
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_declares_the_stage_entry_points():
    import paper_1001_3411_amd as hop
    names = hop.exported_symbols()
    for want in ("hop_density", "hop_link", "hop_groups", "hop_merge", "hop_ctx_create",
                 "hop_ctx_destroy", "hop_last_error", "hop_params_default", "hop_sync"):
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_1001_3411_amd as hop
    lib = hop.load()
    for name in hop.exported_symbols():
        assert hasattr(lib, name), name


def test_params_default_matches_paper_defaults():
    import paper_1001_3411_amd as hop
    lib = hop.load()
    p = hop._Params()
    lib.hop_params_default(ctypes.byref(p))
    assert (p.n_dens, p.n_hop, p.n_merge, p.k_store) == (64, 16, 4, 64)
    assert (p.delta_outer, p.delta_saddle, p.delta_peak) == (80.0, 200.0, 240.0)
    assert p.delta_saddle == 2.5 * p.delta_outer and p.delta_peak == 3 * p.delta_outer
    assert p.grid_bits == 21 and p.flags == hop.HOP_PERIODIC


def test_null_context_is_rejected_without_device():
    import paper_1001_3411_amd as hop
    lib = hop.load()
    p = hop._Params()
    lib.hop_params_default(ctypes.byref(p))
    assert lib.hop_density(None, 100, None, None, ctypes.byref(p), None, None, None) == -1
    assert lib.hop_link(None, 100, None, None, None, None, ctypes.byref(p), None, None) == -1
    assert lib.hop_density_link(None, 100, None, None, None, ctypes.byref(p), None, None, None,
                                None) == -1
    assert lib.hop_halo_stats(None, 100, None, None, None, 1, None, ctypes.byref(p), None, None,
                              None, None) == -1
    assert lib.hop_stitch(None, 1, None, None, None, None, None, None, ctypes.byref(p), 0, 100,
                          None, None, None, None, None, None, None, None, None) == -1
    assert lib.hop_last_error(None) == b"no context"


def test_no_cpu_fallback_in_binding():
    # the binding must not import the oracle or compute anything on the host
    src = open(os.path.join(ROOT, "paper_1001_3411_amd", "__init__.py")).read()
    assert "oracle" not in src.replace("no fallback", "")
    assert "numpy" not in src.split("def _dev")[0]


def test_radius_cell_bits_rule():
    """Cells of side 2^cb hold about 8 particles on average."""
    from paper_1001_3411_amd.radius import cell_bits_for
    assert cell_bits_for(2 ** 24) == 14      # 128^3 cells
    assert cell_bits_for(2 ** 27) == 13      # 256^3 cells
    assert cell_bits_for(2 ** 15) == 17      # 16^3 cells
    assert cell_bits_for(10, 21) == 20       # never fewer than 2 cells per axis
    assert cell_bits_for(2 ** 40, 21) == 12  # never more than 2^9 per axis
    with pytest.raises(ValueError):
        cell_bits_for(0)
