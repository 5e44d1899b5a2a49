"""CPU checks of the C ABI: the library loads, exports every function that
include/harp.h declares, and rejects bad arguments synchronously (no GPU
work is enqueued for a rejected call, so these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "harp.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_][a-z_0-9]*)\s*\(", txt, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_1702_03781_amd import _lib
    return _lib.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["harp_fit", "harp_fill", "reduced_factor", "reduced_solve", "embedded_patterns",
              "harp_port_rhs", "harp_port_admittance", "harp_model_bytes", "harp_fit_ws",
              "reduced_factor_ws", "reduced_solve_ws", "embedded_patterns_ws", "harp_status_str",
              "harp_version"]:
        assert n in names


def test_library_exports_every_declared_symbol(L):
    for n in _declared():
        assert hasattr(L, n), n


def test_binding_signatures_cover_header():
    from paper_1702_03781_amd import _lib
    assert sorted(_lib.SIGNATURES) == _declared()


def test_status_strings(L):
    for s in range(0, -7, -1):
        assert L.harp_status_str(s)
    assert L.harp_version() >= 100


def test_model_bytes_layout(L):
    # header 256 + aligned sections
    nb = L.harp_model_bytes(8, 64, 12, 6)
    ncoef = 8 * 8 * 25 * 7
    a = lambda b: (b + 255) & ~255  # noqa: E731
    assert nb == 256 + a(ncoef * 16) + a(ncoef * 8) + a(64 * 16) + a(8 * 16) + a(8 * 64 * 64)
    assert L.harp_model_bytes(0, 64, 12, 6) == 0


def test_argument_errors_are_synchronous(L):
    from paper_1702_03781_amd import _lib
    HARP_E_ARG, HARP_E_WORKSPACE = -1, -6
    # null pointers / bad sizes: rejected before any launch
    assert L.harp_fill(None, 256, 1, 8, 6, 12, None, None, 16, 0.0, 0, None, 128, 0, None, 0, 0,
                       None, None) == HARP_E_ARG
    el = _lib.HarpElement(4, 32, 0, 0.02)
    assert L.harp_fit(ctypes.byref(el), 1e8, 6, 6, 1.5, 28, 14, None, 0, None, 0, None) == HARP_E_ARG
    el = _lib.HarpElement(4, 32, 1, 0.02)
    # n_alpha odd -> invalid
    assert L.harp_fit(ctypes.byref(el), 1e8, 6, 6, 1.5, 27, 14, 1, 1 << 20, 1, 1 << 20,
                      None) == HARP_E_ARG
    # workspace too small
    assert L.harp_fit(ctypes.byref(el), 1e8, 6, 6, 1.5, 28, 14, 1, 1 << 20, 1, 16,
                      None) == HARP_E_WORKSPACE
    ws = ctypes.c_size_t()
    assert L.harp_fit_ws(4, 32, 6, 6, 28, 14, ctypes.byref(ws)) == 0 and ws.value > 0


def test_new_entry_points_reject_bad_arguments_synchronously(L):
    """Batch, port and fill limits are checked on the host before anything is
    enqueued (placeholder pointers are never dereferenced)."""
    HARP_E_ARG = -1
    # systems without descriptors
    assert L.harp_fill_systems(1, 256, 1, 8, 6, 12, 1, 1, 16, None, 1, 2, 0.0, 1, 1, 16, 256, None, 0, 0, 1,
                               None) == HARP_E_ARG
    assert L.harp_port_rhs_systems(1, 256, 1, 8, None, 1, 2, 2, 1, 16, 32, None) == HARP_E_ARG
    assert L.harp_port_admittance_systems(1, 256, 1, 8, None, 1, 2, 2, 1, 16, 32, 1, 2, 4, None) == HARP_E_ARG
    # more than 64 MBFs
    assert L.harp_fill(1, 256, 1, 65, 6, 12, 1, 1, 2, 0.0, 1, 1, 130, 0, None, 0, 0, 1, None) == HARP_E_ARG
    assert L.harp_port_admittance(1, 256, 1, 65, 2, 1, 130, 260, 1, 2, 4, None) == HARP_E_ARG
    # coefficients of one source MBF beyond 64 KB (64 MBFs, p_max 8, Q 6, complex128)
    assert L.harp_fill(1, 256, 1, 64, 6, 8, 1, 1, 2, 0.0, 1, 1, 128, 0, None, 0, 0, 1, None) == HARP_E_ARG
    # ports beyond the padded port count are refused by the kernels' descriptors,
    # a zero port count by the host
    assert L.harp_port_rhs_systems(1, 256, 1, 8, 1, 1, 2, 0, 1, 16, 0, None) == HARP_E_ARG


def test_refinement_matrix_precision_flag_is_checked(L):
    """harp_refine.z_complex64 must be 0 (complex128 Z) or 1 (complex64 Z,
    widened in the residual); anything else is refused before the workspace
    check and before any launch (placeholder pointers)."""
    from paper_1702_03781_amd._lib import HarpRefine
    HARP_E_ARG, HARP_E_WORKSPACE = -1, -6
    for flag, want in ((2, HARP_E_ARG), (-1, HARP_E_ARG), (1, HARP_E_WORKSPACE), (0, HARP_E_WORKSPACE)):
        ref = HarpRefine(1, 16, 256, 1e-10, 3, None, flag)
        st = L.reduced_solve(16, 1, 1, 0, 1, 16, 256, 1, 1, 1 << 30, 1, 16, 16, 1, 16, 16,
                             ctypes.byref(ref), None, None, 0, None)
        assert st == want, (flag, st)


def test_tuning_table_validation(L):
    """The kernel tuning table: valid entries round-trip, infeasible panel
    widths and unordered entries are refused, an empty table restores the
    defaults.  Host only (no device work)."""
    import ctypes

    from paper_1702_03781_amd._lib import HarpTuningEntry

    def put(rows):
        arr = (HarpTuningEntry * max(1, len(rows)))(*[HarpTuningEntry(*r) for r in rows])
        return L.harp_set_tuning(arr, len(rows))

    assert put([(1024, 8, 4, 256), (2048, 16, 8, 1024), (8192, 4, 2, 4096)]) == 0
    out = (HarpTuningEntry * 8)()
    n = ctypes.c_int32()
    assert L.harp_get_tuning(out, 8, ctypes.byref(n)) == 0 and n.value == 3
    assert [(e.max_order, e.panel_width_c64, e.panel_width_c128, e.small_grid_wgs) for e in out[:3]] == \
        [(1024, 8, 4, 256), (2048, 16, 8, 1024), (8192, 4, 2, 4096)]
    # complex64: 16 columns (two blocks of 8) up to 4096 rows, the first block
    # re-read from memory above 2048; 8192 rows would need four blocks of 4
    assert put([(4096, 16, 4, 1024)]) == 0
    assert put([(8192, 16, 2, 1024)]) == -1
    assert put([(8192, 8, 2, 1024)]) == 0           # two blocks of 4 at 8 rows per thread
    assert put([(4096, 8, 8, 1024)]) == -1           # complex128 width 8 has no configuration past 2048 rows
    assert put([(2048, 8, 4, 1024), (1024, 8, 4, 1024)]) == -1   # not ascending
    assert put([(2048, 3, 4, 1024)]) == -1
    assert put([]) == 0
    assert L.harp_get_tuning(out, 8, ctypes.byref(n)) == 0 and n.value == 0
    d = HarpTuningEntry()
    assert L.harp_default_tuning(2048, ctypes.byref(d)) == 0 and (d.panel_width_c64, d.panel_width_c128) == (16, 8)
    assert L.harp_default_tuning(4096, ctypes.byref(d)) == 0 and (d.panel_width_c64, d.panel_width_c128) == (16, 4)
    assert L.harp_default_tuning(8192, ctypes.byref(d)) == 0 and (d.panel_width_c64, d.panel_width_c128) == (8, 2)
