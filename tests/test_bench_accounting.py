"""The benchmark's flop and roofline accounting (host arithmetic only).

The method flops that the reported roofline charges are pinned here against
operation counts of the textbook algorithms, and the class attribution and
the roofline against small hand-built timer records.
"""
import json
import math
import os

import pytest

import bench


def _lu_muladds(n):
    """Complex multiply-adds of right-looking Gaussian elimination on an n x n
    matrix (the rank-1 updates of the trailing block), counted by loop."""
    return sum((n - k - 1) ** 2 for k in range(n))


def _trsv_muladds(n):
    """Complex multiply-adds of one forward plus one back substitution."""
    return 2 * sum(k for k in range(n))


@pytest.mark.parametrize("n", [64, 512, 2048])
def test_lu_flops_match_the_elimination_count(n):
    # 8 real flops per complex multiply-add; the count is
    # (n-1) n (2n-1) / 6 = n^3/3 - n^2/2 + n/6, the charge its leading term
    w = bench.method_flops(n, 1, [0], refined=False)
    counted = 8.0 * _lu_muladds(n)
    assert math.isclose(w["lu"] - counted, 8.0 * (n * n / 2.0 - n / 6.0), rel_tol=1e-9)


@pytest.mark.parametrize("n,nrhs", [(64, 3), (2048, 256)])
def test_solve_and_residual_flops_match_their_counts(n, nrhs):
    w = bench.method_flops(n, nrhs, [0])
    # the count is n (n-1) per right-hand side, the charge n^2
    counted = 8.0 * _trsv_muladds(n) * nrhs
    assert w["solves"] - counted == 8.0 * n * nrhs
    # the residual b - Z x: n^2 complex multiply-adds per right-hand side
    assert w["residuals"] == 8.0 * n * n * nrhs


def test_refinement_sweeps_scale_solves_and_residuals():
    n, nrhs = 100, 7
    one = bench.method_flops(n, nrhs, [0])
    w = bench.method_flops(n, nrhs, [0, 1, 3])
    # one initial solve plus one per correction; one check more than corrections
    assert w["solves"] == one["solves"] * (1 + 2 + 4)
    assert w["residuals"] == one["residuals"] * (1 + 2 + 4)
    assert w["lu"] == 3 * one["lu"]
    plain = bench.method_flops(n, nrhs, [5, 5], refined=False)
    assert plain["residuals"] == 0.0 and plain["solves"] == 2 * one["solves"]


def test_residual_update_takes_the_first_check_after_a_correction():
    # against a complex64 matrix the check after the first correction is a
    # complex64 update; every other check stays an FP64 residual
    n, nrhs = 100, 7
    per = 8.0 * n * n * nrhs
    w = bench.method_flops(n, nrhs, [0, 1, 3], residual_update=True)
    assert w["residual_updates"] == 2 * per                 # the two systems that corrected
    assert w["residuals"] == (1 + 1 + 3) * per              # checks 0, and 2..k
    plain = bench.method_flops(n, nrhs, [0, 1, 3])
    assert plain["residual_updates"] == 0.0 and plain["residuals"] == (1 + 2 + 4) * per
    assert w["residuals"] + w["residual_updates"] == plain["residuals"]


def _prof(**ms):
    classes = ("fill", "gemm_c64", "gemm_c128", "getf2", "trsm_lower", "trsm_upper", "rank_update")
    p = {k: {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0} for k in classes}
    for k, v in ms.items():
        p[k].update(v)
    return p


def test_attribution_conserves_the_method_flops():
    work = bench.method_flops(256, 16, [1, 2])
    prof = _prof(getf2={"ms": 1.0, "launches": 4, "flops": 3.0e6},
                 rank_update={"ms": 0.5, "launches": 4, "flops": 1.0e6})
    steps, fill = 3, 5.0e8
    a = bench.attribute_method_flops(prof, steps, work, fill)
    wu = bench.method_flops(256, 16, [1, 2], residual_update=True)
    au = bench.attribute_method_flops(prof, steps, wu, fill)
    assert math.isclose(sum(au.values()), sum(a.values()), rel_tol=1e-14)   # moved, not lost
    assert math.isclose(au["gemm_c64"] - a["gemm_c64"], wu["residual_updates"] * steps, rel_tol=1e-12)
    total = (work["lu"] + work["solves"] + work["residuals"] + work["residual_updates"] + fill) * steps
    assert math.isclose(sum(a.values()), total, rel_tol=1e-14)
    assert a["gemm_c128"] == work["residuals"] * steps
    # the plain path has no residual class; the FP64 GEMMs carry the LU
    p = bench.attribute_method_flops(prof, steps, bench.method_flops(256, 16, [0, 0], refined=False),
                                     fill, refined=False)
    assert "gemm_c64" not in p and p["gemm_c128"] > 0


def test_roofline_takes_the_dominant_class_and_its_own_peak():
    prof = _prof(gemm_c64={"ms": 8.0, "launches": 100, "flops": 1.0},
                 gemm_c128={"ms": 4.0, "launches": 10, "flops": 1.0},
                 fill={"ms": 1.0, "launches": 1, "flops": 1.0})
    mflops = {"gemm_c64": 6.0e11, "gemm_c128": 1.0e11, "fill": 1.0e10}
    r = bench.roofline_from_prof(prof, 2, mflops, fill32=True)
    assert r["kernel"] == "gemm_c64" and r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["peak"] == 157.3
    assert math.isclose(r["achieved"], 6.0e11 / 8.0e-3 / 1e12, rel_tol=1e-14)
    assert math.isclose(r["frac"], r["achieved"] / 157.3, rel_tol=1e-14)
    assert math.isclose(r["avg_launch_ms"], 0.08, rel_tol=1e-14)
    assert r["launches_per_step"] == 50
    # the FP64 class prices against the FP64 matrix-core peak; a dominant
    # fill against the vector peak of its own precision
    prof["gemm_c128"]["ms"] = 9.0
    assert bench.roofline_from_prof(prof, 2, mflops)["peak"] == 78.6
    prof["fill"]["ms"] = 10.0
    assert bench.roofline_from_prof(prof, 2, mflops, fill32=True)["peak"] == 157.3
    r64 = bench.roofline_from_prof(prof, 2, mflops, fill32=False)
    assert r64["bound"] == "alu" and r64["peak"] == 78.6


def test_stored_traffic_is_reported_only_for_unchanged_sources():
    tf = os.path.join(bench.ROOT, "profiles", "traffic.json")
    if not os.path.exists(tf):
        pytest.skip("no stored counter figures")
    stored = json.load(open(tf))
    prof = _prof(gemm_c64={"ms": 1.0, "launches": 1, "flops": 1.0})
    r = bench.roofline_from_prof(prof, 1, {"gemm_c64": 1.0e9}, stored_traffic=True)
    t = stored.get("gemm_c64")
    fresh = t is not None and t.get("source_sha") == bench._sha(bench.KERNEL_SOURCES["gemm_c64"])
    assert r["traffic"] == (t["hbm_bytes_per_launch"] if fresh else None)


def test_stored_traffic_belongs_to_the_station_sweep_only():
    # the stored counters were taken on the station sweep's launches; other
    # workloads (batched, large, tessellated) report no traffic
    prof = _prof(gemm_c64={"ms": 1.0, "launches": 1, "flops": 1.0})
    assert bench.roofline_from_prof(prof, 1, {"gemm_c64": 1.0e9})["traffic"] is None


def test_step_roofs_of_the_station_sweep():
    # 16 frequencies, n = 2048, 256 ports, one correction each
    work = bench.method_flops(2048, 256, [1] * 16)
    fill = 4.0e11
    r32 = bench.step_roofs(work, fill, fill32=True)
    r64 = bench.step_roofs(work, fill, fill32=False)
    lu = (work["lu"] + work["solves"]) / 157.3e12 * 1e3
    res = work["residuals"] / 78.6e12 * 1e3
    assert math.isclose(r32["lu_and_solves_ms"], lu, rel_tol=1e-14)
    assert math.isclose(r32["residuals_ms"], res, rel_tol=1e-14)
    assert math.isclose(r64["fill_ms"] / r32["fill_ms"], 157.3 / 78.6, rel_tol=1e-14)
    assert math.isclose(r32["ms"], lu + res + r32["fill_ms"], rel_tol=1e-14)
    plain = bench.step_roofs(bench.method_flops(2048, 256, [0] * 16, refined=False), fill, refined=False)
    assert plain["residuals_ms"] == 0.0
    assert math.isclose(plain["lu_and_solves_ms"] / 1e3 * 78.6e12,
                        16 * (8.0 * 2048 ** 3 / 3 + 8.0 * 2048 ** 2 * 256), rel_tol=1e-14)


def _eq4_entry_flops(P, Q):
    """Real flops of one Eq. 4 entry by Horner's rule: for each of the 2P+1
    angular orders, Q steps in t (a complex value times a real t, plus a
    complex coefficient: 4 flops), then one complex multiply by e^{j p alpha}
    added into the sum (8 flops)."""
    flops = 0
    for _ in range(-P, P + 1):
        for _ in range(Q):
            flops += 2 + 2
        flops += 6 + 2
    return flops


@pytest.mark.parametrize("P,Q", [(0, 0), (5, 3), (12, 6)])
def test_fill_flops_per_entry(P, Q):
    # additive over models, times the antenna pairs and the MBF blocks
    assert bench.fill_flops_of([P], Q, 1, 1) == _eq4_entry_flops(P, Q)
    assert bench.fill_flops_of([P, P + 2], Q, 10, 4) == \
        (_eq4_entry_flops(P, Q) + _eq4_entry_flops(P + 2, Q)) * 10 * 16


def test_fill_flops_of_known_orders():
    assert bench.fill_flops_of([5], 3, 1, 1) == 2.0 * 11 * 10
    assert bench.fill_flops_of([5, 7], 3, 10, 4) == (2.0 * 11 * 10 + 2.0 * 15 * 10) * 10 * 16


def _fwd_muladds_from(n, f):
    """Complex multiply-adds of a forward substitution whose right-hand side
    is zero above row f: rows f..n-1, each against the rows before it from f."""
    return sum(i - f for i in range(f, n))


@pytest.mark.parametrize("n,f", [(64, 0), (64, 17), (2048, 256), (2048, 2048)])
def test_sparse_first_solve_charge(n, f):
    # the first forward substitution of a column starting at row f is charged
    # 4 (n - f)^2, the leading term of its count (n - f)(n - f - 1)/2
    dense = bench.method_flops(n, 1, [1])
    sparse = bench.method_flops(n, 1, [1], first_rows=[[f]])
    charged_fwd = 4.0 * n * n - (dense["solves"] - sparse["solves"])
    assert charged_fwd == 4.0 * (n - f) ** 2
    assert charged_fwd - 8.0 * _fwd_muladds_from(n, f) == 4.0 * (n - f)
    assert sparse["lu"] == dense["lu"] and sparse["residuals"] == dense["residuals"]


def test_first_rows_follow_the_row_exchanges():
    torch = pytest.importorskip("torch")
    # rows 0..5; columns start at rows 1, 4 and nowhere
    B = torch.zeros((1, 6, 3), dtype=torch.complex128)
    B[0, 1, 0] = 1.0
    B[0, 5, 0] = 2.0
    B[0, 4, 1] = 1.0j
    # step 0 exchanges rows 0 and 4, step 1 rows 1 and 5: P B puts row 4 at
    # 0 and row 5 at 1, row 0 at 4 and row 1 at 5
    ipiv = [[4, 5, 2, 3, 4, 5]]
    f = bench.rhs_first_rows(ipiv, B)
    assert f.tolist() == [[1, 0, 6]]
    assert bench.rhs_first_rows([[0, 1, 2, 3, 4, 5]], B).tolist() == [[1, 4, 6]]
