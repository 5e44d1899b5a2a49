#!/usr/bin/env python3
"""Benchmark of the reduced-MBF array solver hot path on one MI355X.

One step = the whole hot path over one batch: for the 256-element station
(8 MBFs of 64 dipole samples per element, n = 2048 unknowns) at 16
frequencies 50-350 MHz, fill every reduced matrix from the HARP models
(Eq. 4), excite every port (256 right-hand sides per frequency), factor and
solve (complex64 on the matrix cores), refine in FP64, and form the port
admittances.  The HARP models are built once before timing (they are reused
for any layout) and all inputs are resident in HBM when the timed region
starts.

Output: one JSON line (see the keys below).  `value` is port solves per second
of the refined path, whose results are checked against the plain complex128
GPU path (relative error <= 1e-6 required) before timing.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {  # MI355X published dense peaks
    "hbm_gbs": 8000.0,
    "fp32_mfma_tflops": 157.3,
    "fp64_mfma_tflops": 78.6,
    "fp64_vector_tflops": 78.6,
    "fp32_vector_tflops": 157.3,
}
REL_GATE = 1e-6


def _sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# sources whose change invalidates the stored HBM counter figures of a kernel
# class (the GEMM launches' shapes come from the LU driver)
KERNEL_SOURCES = {
    "gemm_c64": ["paper_1702_03781_amd/csrc/cgemm.hpp", "paper_1702_03781_amd/csrc/lu.hip"],
    "gemm_c128": ["paper_1702_03781_amd/csrc/cgemm.hpp", "paper_1702_03781_amd/csrc/lu.hip"],
    "fill": ["paper_1702_03781_amd/csrc/fill.hip"],
    "rank_update": ["paper_1702_03781_amd/csrc/lu.hip"],
}


def _say(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _host():
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:  # pragma: no cover
        pass
    return {"cpu_model": cpu_model, "nproc": os.cpu_count()}


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def _rel(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _port_rel(a, b):
    import numpy as np
    return float((np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max())


def cpu_baseline(wl, freq_idx, X_gpu=None, Y_gpu=None, min_seconds=10.0, max_passes=4):
    """The FP64 oracle (its own model fit, Eq. 4 fill, LAPACK solve with one
    right-hand side per port, admittances) over whole passes of a sample of
    the workload's frequencies on this host's cores, and the GPU results of
    the same frequencies against it (X_gpu, Y_gpu: [n_freq] host arrays)."""
    import numpy as np

    from oracle import fill as ofill, fit as ofit, solve as osolve
    models = [ofit.fit(wl.freqs[i], wl.elem.samples, wl.P[i], wl.Q, wl.r_min,
                       wire_radius=wl.elem.wire_radius) for i in freq_idx]
    t0 = time.perf_counter()
    passes = 0
    last = {}
    while True:                      # whole passes over the sample, ~10 s of CPU work
        for i, m in zip(freq_idx, models):
            Z = ofill.fill(m, wl.x, wl.y, wl.ri)
            X = osolve.solve(Z, osolve.port_rhs(m.w, wl.n_ant))
            Y = osolve.admittance(X, m.w, wl.n_ant)
            last[i] = (X, Y)
        passes += 1
        if time.perf_counter() - t0 >= min_seconds or passes >= max_passes:
            break
    dt = time.perf_counter() - t0
    # the same work for one frequency on one thread
    one_thread = None
    try:
        from threadpoolctl import threadpool_limits
        m = models[0]
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            Z = ofill.fill(m, wl.x, wl.y, wl.ri)
            X = osolve.solve(Z, osolve.port_rhs(m.w, wl.n_ant))
            osolve.admittance(X, m.w, wl.n_ant)
            one_thread = wl.n_ant / (time.perf_counter() - t1)
    except Exception:  # pragma: no cover
        one_thread = None
    acc = None
    if X_gpu is not None:
        ex = {float(wl.freqs[i]): _port_rel(X_gpu[i], last[i][0]) for i in freq_idx}
        ey = {float(wl.freqs[i]): _rel(Y_gpu[i], last[i][1]) for i in freq_idx}
        acc = {"max_rel_err_X_per_port": max(ex.values()), "max_rel_err_Y": max(ey.values()),
               "per_freq_X": {f"{k / 1e6:.0f} MHz": v for k, v in ex.items()},
               "per_freq_Y": {f"{k / 1e6:.0f} MHz": v for k, v in ey.items()},
               "gate": REL_GATE,
               "ok": max(ex.values()) <= REL_GATE and max(ey.values()) <= REL_GATE,
               "note": "GPU path (GPU model build, fill, complex64 LU, FP64 refinement) against the "
                       "oracle (its own FP64 model fit, Eq. 4 fill, LAPACK) on the same seeded inputs"}
    return {
        "value": passes * len(freq_idx) * wl.n_ant / dt,
        "unit": "port solves/s",
        "cores": int(_blas_threads()),
        "kind": "oracle",
        "sample": (f"{passes} pass(es) over {len(freq_idx)} of the {len(wl.freqs)} frequencies "
                   f"({', '.join(f'{wl.freqs[i] / 1e6:.0f}' for i in freq_idx)} MHz): "
                   f"oracle Eq. 4 fill + LAPACK zgesv with {wl.n_ant} RHS + admittances, "
                   f"{dt:.1f} s wall"),
        "seconds": dt,
        "one_thread_port_solves_per_s": one_thread,
        "host": _host(),
    }, acc


def cpu_small16():
    """The oracle on the 16-element case (n = 64, 16 ports), repeated ~1 s."""
    from oracle import fill as ofill, fit as ofit, solve as osolve
    from workloads import workload
    wl = workload("small16")
    m = ofit.fit(wl.freqs[0], wl.elem.samples, wl.P[0], wl.Q, wl.r_min, wire_radius=wl.elem.wire_radius)
    t0 = time.perf_counter()
    reps = 0
    while time.perf_counter() - t0 < 1.0:
        Z = ofill.fill(m, wl.x, wl.y)
        X = osolve.solve(Z, osolve.port_rhs(m.w, wl.n_ant))
        osolve.admittance(X, m.w, wl.n_ant)
        reps += 1
    dt = time.perf_counter() - t0
    return {"value": reps * wl.n_ant / dt, "unit": "port solves/s", "cores": int(_blas_threads()),
            "kind": "oracle", "sample": f"{reps} repetitions of the 16-element case (n = 64, 16 ports)"}


def class_rates(prof, steps):
    """Per kernel class: time and launches per step, and the algorithmic
    rates its timers give (flops and bytes that the library attaches)."""
    out = {}
    for k, v in prof.items():
        if v["launches"] == 0:
            continue
        sec = v["ms"] * 1e-3
        out[k] = {"ms_per_step": round(v["ms"] / steps, 4), "launches_per_step": v["launches"] / steps,
                  "avg_launch_us": round(1e3 * v["ms"] / v["launches"], 2),
                  "tflops": round(v["flops"] / sec / 1e12, 2) if v["flops"] > 0 else None,
                  "gbs": round(v["bytes"] / sec / 1e9, 1) if v["bytes"] > 0 else None}
    return out


def method_flops(n, nrhs, iters, refined=True, first_rows=None, residual_update=False):
    """Algorithmic flops of one pass of the solver over len(iters) systems of
    order n with nrhs right-hand sides: LU 8n^3/3 each; triangular solves
    8 n^2 nrhs per solve (one initial solve plus one per correction); the
    residuals 8 n^2 nrhs each (one per check: one more than corrections), in
    FP64, except, with residual_update (a complex64 matrix), the check after
    the first correction: a complex64 update R - Z D ("residual_updates").
    first_rows ([systems][nrhs], optional): the first non-zero row f of each
    column of P B; the first forward substitution of such a column starts
    there, 4 (n - f)^2 flops instead of 4 n^2 (the sparse right-hand sides of
    port excitations)."""
    lu = len(iters) * 8.0 * n ** 3 / 3.0
    saved = 0.0
    if first_rows is not None:
        import numpy as np
        f = np.asarray(first_rows, dtype=np.float64)
        assert f.shape == (len(iters), nrhs)
        saved = float(np.sum(4.0 * (n * n - (n - f) ** 2)))
    if not refined:
        return {"lu": lu, "solves": len(iters) * 8.0 * n * n * nrhs - saved, "residuals": 0.0,
                "residual_updates": 0.0}
    solves = sum(1 + it for it in iters) * 8.0 * n * n * nrhs - saved
    per = 8.0 * n * n * nrhs
    upd = sum(1 for it in iters if it >= 1) if residual_update else 0
    resid = (sum(1 + it for it in iters) - upd) * per
    return {"lu": lu, "solves": solves, "residuals": resid, "residual_updates": upd * per}


def rhs_first_rows(ipiv, B):
    """First non-zero row of each column of P B, per system (n where a column
    is zero): ipiv [systems][n] (host or torch; the row exchanged with row i
    at step i, 0-based), B a torch tensor [systems][n][nrhs] on any device
    (masked there; only the pivots and the result cross to the host)."""
    import numpy as np
    import torch
    piv = ipiv.cpu().numpy() if isinstance(ipiv, torch.Tensor) else np.asarray(ipiv)
    ns, n = piv.shape
    out = np.empty((ns, B.shape[2]), dtype=np.int64)
    for s in range(ns):
        perm = np.arange(n)
        for i, p in enumerate(piv[s]):
            if p != i:
                perm[i], perm[p] = perm[p], perm[i]
        nz = B[s].index_select(0, torch.from_numpy(perm).to(B.device)) != 0
        first = torch.where(nz.any(0), nz.to(torch.int32).argmax(0), torch.full_like(nz[0], n, dtype=torch.int64))
        out[s] = first.cpu().numpy()
    return out


def attribute_method_flops(prof, steps, work, fill_flops_step, refined=True):
    """Method flops per kernel class over the timed steps: the FP32 (or FP64)
    matrix-core class takes the LU and solve flops that the panel and rank-w
    update kernels do not do themselves, and the complex64 residual updates;
    the FP64 class of the refined path the FP64 residuals; the fill its Eq. 4
    flops."""
    lu_cls = "gemm_c64" if refined else "gemm_c128"
    other = prof["getf2"]["flops"] + prof["rank_update"]["flops"]
    out = {lu_cls: (work["lu"] + work["solves"] + work.get("residual_updates", 0.0)) * steps - other,
           "getf2": prof["getf2"]["flops"], "rank_update": prof["rank_update"]["flops"],
           "fill": fill_flops_step * steps}
    if refined:
        out["gemm_c128"] = work["residuals"] * steps
    return out


def roofline_from_prof(prof, steps, mflops, fill32=False, stored_traffic=False):
    """Roofline of the kernel class with the largest summed time, from the
    library's dispatch-attached kernel timers, charged with the method's own
    flops (mflops: per class over the timed steps; fill32: the fill runs in
    FP32).  stored_traffic: report the HBM bytes per launch stored in
    profiles/traffic.json (counters taken on the station sweep, so only that
    workload's launches match them; null while the sources differ)."""
    cand = {k: v for k, v in prof.items() if k in ("fill", "gemm_c64", "gemm_c128", "getf2",
                                                    "trsm_lower", "trsm_upper", "rank_update")}
    dom = max(cand, key=lambda k: cand[k]["ms"])
    pd = prof[dom]
    launches = max(1, pd["launches"])
    avg_ms = pd["ms"] / launches
    if dom == "fill":
        bound, unit = "alu", "TFLOP/s"
        peak = PEAK["fp32_vector_tflops"] if fill32 else PEAK["fp64_vector_tflops"]
        achieved = mflops["fill"] / (pd["ms"] * 1e-3) / 1e12
    elif dom in ("gemm_c64", "gemm_c128"):
        bound = "mfma"
        peak = PEAK["fp32_mfma_tflops"] if dom == "gemm_c64" else PEAK["fp64_mfma_tflops"]
        unit = "TFLOP/s"
        achieved = mflops[dom] / (pd["ms"] * 1e-3) / 1e12
    elif dom == "getf2":
        bound, peak, unit = "alu", PEAK["fp32_vector_tflops"], "TFLOP/s"
        achieved = pd["flops"] / (pd["ms"] * 1e-3) / 1e12
    elif dom == "rank_update":
        bound, peak, unit = "hbm", PEAK["hbm_gbs"], "GB/s"
        achieved = pd["bytes"] / (pd["ms"] * 1e-3) / 1e9
    else:
        bound, peak, unit, achieved = "latency", None, "TFLOP/s", None
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if stored_traffic and os.path.exists(tf) and dom in KERNEL_SOURCES:
        try:
            t = json.load(open(tf)).get(dom)
            if t and t.get("source_sha") == _sha(KERNEL_SOURCES[dom]):
                traffic = t.get("hbm_bytes_per_launch")
        except Exception:
            traffic = None
    return {
        "kernel": dom,
        "bound": bound,
        "achieved": achieved,
        "peak": peak,
        "unit": unit,
        "frac": (achieved / peak) if (achieved and peak) else None,
        "traffic": traffic,
        "launches_per_step": pd["launches"] / steps,
        "avg_launch_ms": avg_ms,
        "algorithmic_flops_per_launch": mflops.get(dom, pd["flops"]) / launches,
        "algorithmic_bytes_per_launch": pd["bytes"] / launches,
        "flops_charged": "method flops: LU 8n^3/3 and triangular solves 8n^2 N_rhs per solve (measured "
                         "sweep count; the first forward substitution 4(n-f)^2 per column from its first "
                         "non-zero row f of P B), less the panel and rank-w kernels' own; residual 8n^2 "
                         "N_rhs per check (FP64, or on the FP32 matrix cores for the complex64 update after "
                         "the first correction); fill 2(2P+1)(2Q+4) per model-evaluated entry",
    }


def step_roofs(work, fill_flops, refined=True, fill32=False):
    """Time of one step if every part ran at its roof: FP32 matrix cores for
    the complex64 LU, solves and residual updates (FP64 for the plain path),
    FP64 matrix cores for the FP64 residuals, FP64 vector units for the fill
    (FP32 vector units for the complex64 fill)."""
    lu_peak = PEAK["fp32_mfma_tflops"] if refined else PEAK["fp64_mfma_tflops"]
    t_lu = (work["lu"] + work["solves"] + work.get("residual_updates", 0.0)) / (lu_peak * 1e12)
    t_res = work["residuals"] / (PEAK["fp64_mfma_tflops"] * 1e12)
    fill_peak = PEAK["fp32_vector_tflops"] if fill32 else PEAK["fp64_vector_tflops"]
    t_fill = fill_flops / (fill_peak * 1e12)
    return {"ms": 1e3 * (t_lu + t_res + t_fill), "lu_and_solves_ms": 1e3 * t_lu,
            "residuals_ms": 1e3 * t_res, "fill_ms": 1e3 * t_fill}


def fill_flops_of(P_list, Q, n_ant_pairs, n_mbf):
    """2(2P+1)(2Q+4) flops per model-evaluated entry, summed over models."""
    return sum(2.0 * (2 * P + 1) * (2 * Q + 4) for P in P_list) * n_ant_pairs * n_mbf ** 2


def bench_batched(args, api, torch, dev):
    """48 station layouts of 64-512 elements, each at 8 of the 16 sweep
    frequencies (384 systems, n = 528-4056), reusing the 16 models; one step
    is one replay of the HIP graph that holds every group's fill, excitation,
    factorisation, refined solve and admittances (--no-graph: eager, the
    refinement reporting to the host once per group)."""
    import numpy as np

    from workloads import batched_layouts, workload

    wl = workload("station_sweep")        # element and frequency sweep whose models the layouts reuse
    samples = api.to_device_samples(wl.elem.samples, dev)
    models = [api.harp_fit(samples, wl.elem.wire_radius, f, P, wl.Q, wl.r_min)
              for f, P in zip(wl.freqs, wl.P)]
    mb = api.stack_models(models)
    layouts = batched_layouts()
    # the planner's cost model measured on this GPU (one group per point)
    cost, cost_points = api.autotune_batch_costs(mb)
    S = api.BatchSolver(mb, layouts, tol=args.tol, streams=args.streams, cost=cost, graph=not args.no_graph,
                        fill=args.fill)
    # kernel choices (panel width, GEMM tile switch) per group order, timed on this GPU
    tuning, tuning_points = api.autotune_kernels([(g.n, len(g.members), g.n_ports_pad) for g in S.groups])
    S.tuning = tuning
    _say(f"batched: plan of {len(S.groups)} groups, kernel tuning of {len(tuning)} orders")
    S.step()                              # raises on a domain error or a zero pivot
    torch.cuda.synchronize()
    conv = all(r["converged"] for r in S.reports)
    # accuracy gate on the smallest, a middle and the largest system: the
    # refined batch against the plain complex128 GPU path of that layout alone
    sizes = np.array(S.n_ant)
    picks = [int(np.argmin(sizes)), int(np.argsort(sizes)[len(sizes) // 2]), int(np.argmax(sizes))]
    rel_x = rel_y = 0.0
    for s in picks:
        li, f = S.layout_of[s]
        x, y, _ = layouts[li]
        P = api.StationSolver(api.stack_models([models[f]]), torch.from_numpy(x).to(dev),
                              torch.from_numpy(y).to(dev), "plain")
        Xp, Yp = P.step()
        X, Y, _, _ = S.system(s)
        rel_x = max(rel_x, float(torch.linalg.norm(X - Xp[0]) / torch.linalg.norm(Xp[0])))
        rel_y = max(rel_y, float(torch.linalg.norm(Y - Yp[0]) / torch.linalg.norm(Yp[0])))
        del P, Xp, Yp
    accuracy_ok = conv and rel_x <= REL_GATE and rel_y <= REL_GATE

    for _ in range(args.warmup):
        S.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S.step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    iters = sorted({r["iters"] for r in S.reports})

    # kernel-class timers need eager launches: a timed pass of the eager path
    E = api.BatchSolver(mb, layouts, tol=args.tol, streams=args.streams, cost=cost,
                        tuning=tuning, fill=args.fill) if not args.no_graph else S
    E.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E.step()
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3
    api.prof_enable(True)
    t0 = time.perf_counter()
    E.step()
    torch.cuda.synchronize()
    ms_instr = (time.perf_counter() - t0) * 1e3
    prof = api.prof_read()
    api.prof_enable(False)
    e_iters = [E.reports[s]["iters"] for s in range(E.n_systems)]
    e_first = [rhs_first_rows(g.ipiv, g.B) for g in E.groups]
    del E
    fill_flops_step = 0.0
    lu = solves = resid = upd = 0.0
    for g, first in zip(S.groups, e_first):
        w = method_flops(g.n, g.n_ports_pad, [e_iters[m] for m in g.members], first_rows=first,
                         residual_update=args.fill == "c64")
        lu, solves, resid = lu + w["lu"], solves + w["solves"], resid + w["residuals"]
        upd += w["residual_updates"]
    for s in range(S.n_systems):
        li, f = S.layout_of[s]
        na_s = S.n_ant[s]
        fill_flops_step += fill_flops_of([wl.P[f]], wl.Q, na_s * (na_s - 1), wl.elem.n_mbf)
    work = {"lu": lu, "solves": solves, "residuals": resid, "residual_updates": upd}
    mfl = attribute_method_flops(prof, 1, work, fill_flops_step, refined=True)
    for v in prof.values():
        v["ms_per_step"] = v["ms"]
    roofline = roofline_from_prof(prof, 1, mfl, fill32=args.fill == "c64")
    roof = step_roofs(work, fill_flops_step, fill32=args.fill == "c64")

    nm = wl.elem.n_mbf
    port_solves = float(sum(S.n_ant))
    entries = float(sum((nm * v) ** 2 for v in S.n_ant))
    padded = float(sum(len(g.members) * g.n ** 2 for g in S.groups))
    out = {
        "metric": "reduced-Z entries/s + port solves/s at rel err 1e-6 vs FP64 plain path",
        "value": port_solves / (ms * 1e-3),
        "unit": "port solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_step_eager": ms_eager,
        "ms_per_step_with_kernel_timers": ms_instr,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64",
        "data": "synthetic",
        "config": {
            "workload": ("batched layouts: 48 station layouts of 64-512 elements (disk radius "
                         "19 m x sqrt(N_a/256), 1.5 m min spacing), 8 MBFs x 64 dipole samples, 8 of "
                         "16 frequencies 50-350 MHz each (384 systems, n = 528-4056, N_a ports each); "
                         "grouped and padded, complex64 LU on MFMA + FP64 refinement, "
                         + ("complex64 fill" if args.fill == "c64" else "FP64 fill")),
            "systems": S.n_systems, "groups": [(len(g.members), g.n) for g in S.groups],
            "streams": args.streams, "refine_tol": args.tol, "graph": not args.no_graph,
            "graph_sweep_budget": S.sweeps if not args.no_graph else None,
            "padded_over_real_entries": padded / entries,
            "plan_cost_model": {"t_group_s": cost[0], "t_order_s": cost[1], "t_system_s": cost[2],
                                "measured": cost_points},
            "kernel_tuning": tuning,
            "kernel_tuning_default_differs": [e for e in tuning if
                                              (e["panel_width_c64"], e["small_grid_wgs"]) !=
                                              (api.default_tuning(e["max_order"])["panel_width_c64"], 1024)],
        },
        "reduced_z_entries_per_s_whole_step": entries / (ms * 1e-3),
        "accuracy": {"max_rel_err_X_vs_plain": rel_x, "max_rel_err_Y_vs_plain": rel_y,
                     "all_converged": conv, "gate": REL_GATE, "ok": accuracy_ok,
                     "refine_iters": iters, "checked_systems": picks},
        "phases_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in prof.items()},
        "kernel_classes": class_rates(prof, 1),
        "roofline": roofline,
        "step_roofline": {**{k: round(v, 3) for k, v in roof.items()}, "measured_ms": ms, "frac": roof["ms"] / ms},
        "cpu_baseline": None,
    }
    if args.cpu_freqs > 0:
        # the oracle on the three checked systems (each its own model fit,
        # fill, LAPACK solve and admittances), and the GPU batch against it
        from oracle import fill as ofill, fit as ofit, solve as osolve
        t_cpu, ports, ex, ey = 0.0, 0, 0.0, 0.0
        for s in picks:
            li, f = S.layout_of[s]
            x, y, _ = layouts[li]
            m = ofit.fit(wl.freqs[f], wl.elem.samples, wl.P[f], wl.Q, wl.r_min, wire_radius=wl.elem.wire_radius)
            t0 = time.perf_counter()
            Zo = ofill.fill(m, x, y)
            Xo = osolve.solve(Zo, osolve.port_rhs(m.w, x.size))
            Yo = osolve.admittance(Xo, m.w, x.size)
            t_cpu += time.perf_counter() - t0
            ports += x.size
            X, Y, _, _ = S.system(s)
            ex = max(ex, _port_rel(X.cpu().numpy(), Xo))
            ey = max(ey, _rel(Y.cpu().numpy(), Yo))
        out["cpu_baseline"] = {"value": ports / t_cpu, "unit": "port solves/s", "cores": int(_blas_threads()),
                               "kind": "oracle",
                               "sample": f"the smallest, a middle and the largest system ({ports} ports): oracle "
                                         f"Eq. 4 fill + LAPACK zgesv + admittances, {t_cpu:.1f} s",
                               "host": _host()}
        out["accuracy"]["vs_oracle"] = {"max_rel_err_X_per_port": ex, "max_rel_err_Y": ey,
                                        "ok": ex <= REL_GATE and ey <= REL_GATE}
        out["accuracy"]["ok"] = accuracy_ok and ex <= REL_GATE and ey <= REL_GATE
    api.set_tuning(None)
    print(json.dumps(out), flush=True)


def bench_large(args, api, torch, dev):
    """The large array alone: 1024 elements (38 m disk), 8 MBFs, 200 MHz,
    radius of influence 12 m, n = 8192, 1024 ports; fill, complex64 LU, solve,
    FP64 refinement and admittances per step; the oracle on one pass."""
    import numpy as np

    from workloads import workload
    wl = workload("large1024")
    samples = api.to_device_samples(wl.elem.samples, dev)
    model = api.harp_fit(samples, wl.elem.wire_radius, wl.freqs[0], wl.P[0], wl.Q, wl.r_min)
    mb = api.stack_models([model])
    S = api.StationSolver(mb, torch.from_numpy(wl.x).to(dev), torch.from_numpy(wl.y).to(dev),
                          "refined32" if args.fill == "c64" else "refined", tol=args.tol, ri=wl.ri)
    S.step()
    for _ in range(args.warmup):
        S.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S.step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    names = ["fill_and_excitation", "factor", "solve_and_refine", "admittance"]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    S.step(events=ev)
    torch.cuda.synchronize()
    ph = {k: ev[i].elapsed_time(ev[i + 1]) for i, k in enumerate(names)}
    api.prof_enable(True)
    S.step()
    torch.cuda.synchronize()
    prof = api.prof_read()
    api.prof_enable(False)
    it = [r["iters"] for r in S.reports]
    first = rhs_first_rows(S.ipiv, S.B)
    n = wl.n
    fill_flops = fill_flops_of(wl.P, wl.Q, int(np.count_nonzero(
        (np.hypot(wl.x[:, None] - wl.x[None, :], wl.y[:, None] - wl.y[None, :]) <= wl.ri))) - wl.n_ant, wl.elem.n_mbf)
    work = method_flops(n, wl.n_ant, it, first_rows=first, residual_update=args.fill == "c64")
    mfl = attribute_method_flops(prof, 1, work, fill_flops)
    for v in prof.values():
        v["ms_per_step"] = v["ms"]
    f32 = args.fill == "c64"
    roof = step_roofs(work, fill_flops, fill32=f32)
    out = {
        "metric": "reduced-Z entries/s + port solves/s at rel err 1e-6 vs FP64 plain path",
        "value": wl.n_ant / (ms * 1e-3), "unit": "port solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64+f64", "data": "synthetic",
        "config": {"workload": "large array: 1024 elements (38 m disk, 1.5 m min spacing), 8 MBFs x 64 dipole "
                               "samples, 200 MHz, radius of influence 12 m, n = 8192, 1024 ports; complex64 LU "
                               "on MFMA + FP64 refinement, " + ("complex64 fill" if f32 else "FP64 fill"),
                   "P": wl.P[0], "Q": wl.Q, "refine_tol": args.tol, "fill": args.fill},
        "reduced_z_entries_per_s": n * n / (prof["fill"]["ms"] * 1e-3) if prof["fill"]["ms"] > 0 else None,
        "phase_ms": {k: round(v, 3) for k, v in ph.items()}, "refine_iters": it,
        "kernel_classes": class_rates(prof, 1), "roofline": roofline_from_prof(prof, 1, mfl, fill32=f32),
        "step_roofline": {**{k: round(v, 3) for k, v in roof.items()}, "measured_ms": ms, "frac": roof["ms"] / ms},
        "cpu_baseline": None,
    }
    if args.cpu_freqs > 0:
        cb, acc = cpu_baseline(wl, [0], S.X.cpu().numpy(), S.Y.cpu().numpy(), min_seconds=0.0, max_passes=1)
        out["cpu_baseline"] = cb
        out["accuracy_vs_oracle"] = acc
    print(json.dumps(out), flush=True)


def bench_tessellated(args, api, torch, dev):
    """The 1024-element array (38 m disk, 8 MBFs, 200 MHz) by the overlapping-
    subarray tessellation (every cell's subarray one system of a batch, inner
    ports only) against the full refined solve of the whole array (n = 8192,
    1024 ports); EEP error of the tessellation over 128 directions."""
    import numpy as np

    from workloads import directions, workload

    wl = workload("large1024")
    samples = api.to_device_samples(wl.elem.samples, dev)
    model = api.harp_fit(samples, wl.elem.wire_radius, wl.freqs[0], wl.P[0], wl.Q, wl.r_min)
    mb = api.stack_models([model])
    th, ph = directions(128, seed=9)
    tht, pht = torch.from_numpy(th).to(dev), torch.from_numpy(ph).to(dev)
    x, y = torch.from_numpy(wl.x).to(dev), torch.from_numpy(wl.y).to(dev)
    T = api.TessellatedSolver(mb, wl.x, wl.y, [0], args.r_in, args.r_ext, tol=args.tol, streams=args.streams)
    full = api.StationSolver(mb, x, y, "refined", tol=args.tol)

    def timed(step):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps

    ms_t = timed(T.step)
    ms_f = timed(full.step)
    E = T.patterns([model], 0, tht, pht)
    Ef = api.embedded_patterns(model, x, y, full.X, tht, pht)
    err = ((E - Ef).abs().pow(2).sum(dim=(1, 2)).sqrt() / Ef.abs().pow(2).sum(dim=(1, 2)).sqrt()).cpu().numpy()
    conv = all(r["converged"] for r in T.batch.reports) and all(r["converged"] for r in full.reports)
    sizes = [len(c.members) for c in T.cells]
    out = {
        "metric": "reduced-Z entries/s + port solves/s at rel err 1e-6 vs FP64 plain path",
        "value": wl.n_ant / (ms_t * 1e-3),
        "unit": "port solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_t,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64",
        "data": "synthetic",
        "config": {
            "workload": ("tessellated large array: 1024 elements (38 m disk, 1.5 m min spacing), 8 MBFs x 64 "
                         "dipole samples, 200 MHz; hexagonal cells R_in = %g m, extension R_ext = %g m, every "
                         "subarray one system of a batch with its inner ports excited; complex64 LU + FP64 "
                         "refinement" % (args.r_in, args.r_ext)),
            "cells": len(T.cells), "subarray_sizes": [min(sizes), max(sizes), float(np.mean(sizes))],
            "groups": [(len(g.members), g.n) for g in T.batch.groups], "refine_tol": args.tol,
        },
        "full_solve_ms": ms_f,
        "speedup_over_full_solve": ms_f / ms_t,
        "eep_rel_err_vs_full": {"mean": float(err.mean()), "max": float(err.max()), "directions": 128},
        "all_converged": conv,
        "cpu_baseline": None,
    }
    if args.cpu_freqs > 0:
        # the oracle's tessellated solve of the same array (its own model fit,
        # every cell's fill and LAPACK solve), and the GPU's ports against it
        from oracle import fit as ofit
        from oracle import tessellation as otess
        mo = ofit.fit(wl.freqs[0], wl.elem.samples, wl.P[0], wl.Q, wl.r_min, wire_radius=wl.elem.wire_radius)
        t0 = time.perf_counter()
        per, _ = otess.solve_tessellated(mo, wl.x, wl.y, args.r_in, args.r_ext)
        dt = time.perf_counter() - t0
        ex = ey = 0.0
        for a in range(wl.n_ant):
            mem, Xg, Yg = T.port(a, 0)
            mo_mem, Xo, Yo = per[a]
            ex = max(ex, _rel(Xg.cpu().numpy(), Xo))
            ey = max(ey, _rel(Yg.cpu().numpy(), Yo))
        out["cpu_baseline"] = {"value": wl.n_ant / dt, "unit": "port solves/s", "cores": int(_blas_threads()),
                               "kind": "oracle", "sample": f"the oracle's tessellated solve of the whole array "
                                                           f"({len(T.cells)} cells, {wl.n_ant} ports), {dt:.1f} s",
                               "host": _host()}
        out["accuracy_vs_oracle"] = {"max_rel_err_X_per_port": ex, "max_rel_err_Y_per_port": ey,
                                     "ok": ex <= REL_GATE and ey <= REL_GATE}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-10, help="FP64 refinement tolerance")
    ap.add_argument("--cpu-freqs", type=int, default=16,
                    help="frequencies of the station sweep in the CPU-baseline sample (0: skip every CPU leg)")
    ap.add_argument("--no-plain", action="store_true", help="skip timing the plain FP64 path")
    ap.add_argument("--fill", choices=["c64", "c128"], default="c64",
                    help="station sweep: precision of the timed fill and of the residual's matrix (c64: "
                         "complex64 fill, FP64 residual against it; c128: FP64 fill); the other is timed "
                         "beside it")
    ap.add_argument("--no-large", action="store_true", help="skip the large-array (n = 8192) steps")
    ap.add_argument("--workload", choices=["station", "batched", "large", "tessellated"], default="station",
                    help="station: the 16-frequency station sweep (default); batched: 48 unequal "
                         "layouts x 8 frequencies; large: the 1024-element array (n = 8192) alone; "
                         "tessellated: the 1024-element array by overlapping "
                         "subarrays against its full solve")
    ap.add_argument("--r-in", type=float, default=6.0, help="tessellation inner radius (m)")
    ap.add_argument("--r-ext", type=float, default=6.0, help="tessellation extension (m)")
    ap.add_argument("--streams", type=int, default=4, help="HIP streams of the batched and tessellated workloads")
    ap.add_argument("--no-graph", action="store_true", help="batched workload: eager launches instead of a HIP graph")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB three times (the reference kernel that "
                         "scales the HBM byte counters) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU: the batch of frequencies is the "
                                   "unit of work and multi-GPU sharding is not implemented "
                                   "(see DESIGN.md); run with --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1702_03781_amd import api
    from workloads import workload

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU available"}))
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                          "copies": 3}))
        return
    if args.workload == "batched":
        return bench_batched(args, api, torch, dev)
    if args.workload == "tessellated":
        return bench_tessellated(args, api, torch, dev)
    if args.workload == "large":
        return bench_large(args, api, torch, dev)
    wl = workload("station_sweep")
    n, na, nf = wl.n, wl.n_ant, len(wl.freqs)

    # HARP models (built once, reused for any layout), inputs resident in HBM
    samples = api.to_device_samples(wl.elem.samples, dev)
    models = [api.harp_fit(samples, wl.elem.wire_radius, f, P, wl.Q, wl.r_min)
              for f, P in zip(wl.freqs, wl.P)]
    mb = api.stack_models(models)
    x = torch.from_numpy(wl.x).to(dev)
    y = torch.from_numpy(wl.y).to(dev)
    torch.cuda.synchronize()

    _say("station sweep: models built")
    mode = "refined32" if args.fill == "c64" else "refined"
    alt_mode = "refined" if mode == "refined32" else "refined32"
    fill32 = mode == "refined32"
    ref = api.StationSolver(mb, x, y, mode, tol=args.tol)
    plain = api.StationSolver(mb, x, y, "plain")

    # accuracy gate: refined path vs the plain FP64 GPU path (the oracle
    # comparison follows in the CPU leg); step() raises on a fill domain error
    # or a zero pivot
    Xr, Yr = ref.step()
    Xp, Yp = plain.step()
    torch.cuda.synchronize()
    d = (Xr - Xp).abs().pow(2).sum(dim=(1, 2)).sqrt() / Xp.abs().pow(2).sum(dim=(1, 2)).sqrt()
    dy = (Yr - Yp).abs().pow(2).sum(dim=(1, 2)).sqrt() / Yp.abs().pow(2).sum(dim=(1, 2)).sqrt()
    rel_x, rel_y = float(d.max()), float(dy.max())
    accuracy_ok = rel_x <= REL_GATE and rel_y <= REL_GATE
    X_host, Y_host = Xr.cpu().numpy(), Yr.cpu().numpy()

    def timed(solver, steps):
        for _ in range(args.warmup):
            solver.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            solver.step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    _say(f"accuracy vs plain: X {rel_x:.2e}, Y {rel_y:.2e}; timing")
    # timed region (refined path), uninstrumented; an event after every step
    # (recorded on the stream, no synchronisation) gives per-step durations
    for _ in range(args.warmup):
        ref.step()
    torch.cuda.synchronize()
    step_ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    step_ev[0].record()
    for i in range(args.steps):
        ref.step()
        step_ev[i + 1].record()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    per_step = sorted(step_ev[i].elapsed_time(step_ev[i + 1]) for i in range(args.steps))
    iters = [r["iters"] for r in ref.reports]
    first_ref = rhs_first_rows(ref.ipiv, ref.B)

    # phases (fill + excitation, factorisation, solve + refinement, admittances)
    # from events at the phase boundaries of a few more steps
    phase_names = ["fill_and_excitation", "factor", "solve_and_refine", "admittance"]
    phase_ms = dict.fromkeys(phase_names, 0.0)
    n_phase = max(1, min(5, args.steps))
    for _ in range(n_phase):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ref.step(events=ev)
        torch.cuda.synchronize()
        for i, k in enumerate(phase_names):
            phase_ms[k] += ev[i].elapsed_time(ev[i + 1]) / n_phase

    # the same steps again with the library's kernel-class HIP-event timers
    # (each launch bracketed on its own stream) for the per-kernel roofline
    api.prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ref.step()
    torch.cuda.synchronize()
    ms_instr = (time.perf_counter() - t0) * 1e3 / args.steps
    prof = api.prof_read()
    sites = api.prof_read_sites()
    api.prof_enable(False)

    _say(f"refined {ms:.3f} ms per step; kernel timers done")
    ms_plain = None if args.no_plain else timed(plain, max(3, args.steps // 4))
    first_plain = rhs_first_rows(plain.ipiv, plain.B)
    # the other precision of the fill and residual matrix, for comparison
    alt = api.StationSolver(mb, x, y, alt_mode, tol=args.tol)
    Xa, Ya = alt.step()
    torch.cuda.synchronize()
    da = (Xa - Xp).abs().pow(2).sum(dim=(1, 2)).sqrt() / Xp.abs().pow(2).sum(dim=(1, 2)).sqrt()
    dya = (Ya - Yp).abs().pow(2).sum(dim=(1, 2)).sqrt() / Yp.abs().pow(2).sum(dim=(1, 2)).sqrt()
    ms_alt = timed(alt, max(3, args.steps // 2))
    ev_alt = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    alt.step(events=ev_alt)
    torch.cuda.synchronize()
    alt_block = {"mode": ("complex64 fill, FP64 residual against the complex64 matrix" if alt_mode == "refined32"
                          else "FP64 fill (complex128 residual matrix plus its complex64 rounding)"),
                 "ms_per_step": ms_alt, "port_solves_per_s": nf * na / (ms_alt * 1e-3),
                 "fill_and_excitation_ms": ev_alt[0].elapsed_time(ev_alt[1]),
                 "max_rel_err_X_vs_plain": float(da.max()), "max_rel_err_Y_vs_plain": float(dya.max())}
    del alt, Xa, Ya, plain, Xp, Yp
    torch.cuda.empty_cache()

    # embedded element patterns (Eqs. 5-6) of every port at 110 MHz over the
    # adjoint configuration's 1024 directions: one dense FP64 product of the
    # pattern operator (2 x 1024 rows, n columns) with the 256 port solutions
    from workloads import directions
    th, ph = directions(1024, seed=304)
    tht, pht = torch.from_numpy(th).to(dev), torch.from_numpy(ph).to(dev)
    fi = int(np.argmin(np.abs(wl.freqs - 110e6)))
    Xf = ref.X[fi]
    api.embedded_patterns(models[fi], x, y, Xf, tht, pht)
    torch.cuda.synchronize()
    pe = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 10
    pe[0].record()
    for _ in range(reps):
        api.embedded_patterns(models[fi], x, y, Xf, tht, pht)
    pe[1].record()
    torch.cuda.synchronize()
    ms_pat = pe[0].elapsed_time(pe[1]) / reps
    pat_flops = 8.0 * (2 * 1024) * na * n
    patterns = {"workload": "110 MHz, 1024 directions, 256 ports (n = 2048)", "ms": ms_pat,
                "gemm_flops": pat_flops, "tflops": pat_flops / (ms_pat * 1e-3) / 1e12,
                "frac_fp64_mfma_whole_call": pat_flops / (ms_pat * 1e-3) / 1e12 / PEAK["fp64_mfma_tflops"],
                "note": "whole call (MBF radiation vectors, operator build, product) against the product's "
                        "FP64 matrix-core roof"}

    # algorithmic work per step and the method flops of each kernel class
    fill_flops_step = fill_flops_of(wl.P, wl.Q, na * (na - 1), wl.elem.n_mbf)


    work = method_flops(n, na, iters, refined=True, first_rows=first_ref, residual_update=fill32)
    mfl = attribute_method_flops(prof, args.steps, work, fill_flops_step, refined=True)
    for v in prof.values():
        v["ms_per_step"] = v["ms"] / args.steps
    roofline = roofline_from_prof(prof, args.steps, mfl, fill32=fill32, stored_traffic=True)
    roof_ref = step_roofs(work, fill_flops_step, refined=True, fill32=fill32)
    work_plain = method_flops(n, na, [0] * nf, refined=False, first_rows=first_plain)
    roof_plain = step_roofs(work_plain, fill_flops_step, refined=False)
    t_fill = prof["fill"]["ms_per_step"] * 1e-3

    port_solves = nf * na
    value = port_solves / (ms * 1e-3)
    out = {
        "metric": "reduced-Z entries/s + port solves/s at rel err 1e-6 vs FP64 plain path",
        "value": value,
        "unit": "port solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_step_median": per_step[len(per_step) // 2],
        "ms_per_step_min": per_step[0],
        "ms_per_step_with_kernel_timers": ms_instr,
        "phase_ms_per_step": {k: round(v, 4) for k, v in phase_ms.items()},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64",
        "data": "synthetic",
        "config": {
            "workload": ("station sweep: 256 elements (19 m disk, 1.5 m min spacing), 8 MBFs x 64 "
                         "dipole samples, 16 frequencies 50-350 MHz, n = 2048, 256 ports each; "
                         + ("complex64 fill (FP32 evaluation, FP64 phase argument), complex64 LU on MFMA, "
                            "FP64 refinement against the complex64 matrix" if fill32 else
                            "FP64 fill, complex64 LU on MFMA, FP64 refinement against the complex128 matrix")),
            "n_ant": na, "n_mbf": wl.elem.n_mbf, "n_freq": nf, "n": n, "rhs_per_freq": na,
            "P": list(wl.P), "Q": wl.Q, "refine_tol": args.tol, "fill": args.fill,
        },
        # entries/s over the fill's own time (the fill kernel's timers); the
        # port solves over the factorisation and solve phases
        "reduced_z_entries_per_s": nf * n * n / t_fill if t_fill > 0 else None,
        "reduced_z_entries_per_s_whole_step": nf * n * n / (ms * 1e-3),
        "port_solves_per_s_factor_and_solve": port_solves / ((phase_ms["factor"] + phase_ms["solve_and_refine"])
                                                              * 1e-3),
        "accuracy": {"max_rel_err_X_vs_plain": rel_x, "max_rel_err_Y_vs_plain": rel_y,
                     "gate": REL_GATE, "ok": accuracy_ok, "refine_iters": iters},
        "plain_fp64": None if ms_plain is None else {
            "ms_per_step": ms_plain, "port_solves_per_s": port_solves / (ms_plain * 1e-3),
            "speedup_refined_over_plain": ms_plain / ms,
            "step_at_roofs_ms": roof_plain["ms"], "step_roof_frac": roof_plain["ms"] / ms_plain},
        "step_roofline": {**{k: round(v, 4) for k, v in roof_ref.items()}, "measured_ms": ms,
                          "frac": roof_ref["ms"] / ms,
                          "parts": ("FP32 matrix cores: LU + solves (+ complex64 residual updates); "
                                    "FP64 matrix cores: FP64 residuals; "
                                    + ("FP32 vector: fill" if fill32 else "FP64 vector: fill"))},
        "phases_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in prof.items()},
        "kernel_classes": class_rates(prof, args.steps),
        "gemm_sites": class_rates(sites, args.steps),
        "patterns": patterns,
        "other_fill_precision": alt_block,
        "roofline": roofline,
        "paper_context": {"fill_s": 10.0, "solve_s": 12.6, "eeps_s": 6.0,
                          "hardware": "Intel Core i7-3770 3.4 GHz (desktop)",
                          "workload": "SKA station, 256 SKALA elements, 20 MBFs, 110 MHz, one "
                                      "frequency (Table II); not this workload"},
        "cpu_baseline": None,
    }
    del ref, Xr, Yr
    torch.cuda.empty_cache()

    # the large array (1024 elements, 38 m, 200 MHz, radius of influence 12 m,
    # n = 8192, 1024 ports): a few refined steps on the same launch path
    large = None
    if not args.no_large:
        _say("large array")
        wl5 = workload("large1024")
        model5 = api.harp_fit(samples, wl5.elem.wire_radius, wl5.freqs[0], wl5.P[0], wl5.Q, wl5.r_min)
        mb5 = api.stack_models([model5])
        S5 = api.StationSolver(mb5, torch.from_numpy(wl5.x).to(dev), torch.from_numpy(wl5.y).to(dev), mode,
                               tol=args.tol, ri=wl5.ri)
        ms5 = timed(S5, 3)
        ev5 = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        S5.step(events=ev5)
        torch.cuda.synchronize()
        ph5 = {k: ev5[i].elapsed_time(ev5[i + 1]) for i, k in enumerate(phase_names)}
        it5 = [r["iters"] for r in S5.reports]
        n5 = wl5.n
        large = {"workload": "large array: 1024 elements (38 m disk), 8 MBFs x 64 samples, 200 MHz, radius of "
                             "influence 12 m, n = 8192, 1024 ports; complex64 LU + FP64 refinement, "
                             + ("complex64 fill" if fill32 else "FP64 fill"),
                 "steps": 3, "ms_per_step": ms5, "port_solves_per_s": wl5.n_ant / (ms5 * 1e-3),
                 "reduced_z_entries_per_s": n5 * n5 / (ph5["fill_and_excitation"] * 1e-3),
                 "phase_ms": {k: round(v, 3) for k, v in ph5.items()}, "refine_iters": it5,
                 "step_at_roofs_ms": step_roofs(method_flops(n5, wl5.n_ant, it5,
                                                             first_rows=rhs_first_rows(S5.ipiv, S5.B),
                                                             residual_update=fill32),
                                                0.0, fill32=fill32)["ms"]}
        X5, Y5 = S5.X[0].cpu().numpy(), S5.Y[0].cpu().numpy()
        del S5
        torch.cuda.empty_cache()
    out["large_array"] = large

    if args.cpu_freqs > 0:
        _say("CPU baseline (oracle)")
        k = min(args.cpu_freqs, nf)
        idx = sorted(set(int(round(i)) for i in np.linspace(0, nf - 1, k)))
        out["cpu_baseline"], acc = cpu_baseline(wl, idx, X_host, Y_host)
        out["accuracy"]["vs_oracle"] = acc
        out["accuracy"]["ok"] = accuracy_ok and acc["ok"]
        out["cpu_baseline_small16"] = cpu_small16()
        if large is not None:
            wl5 = workload("large1024")
            cb5, acc5 = cpu_baseline(wl5, [0], X5[None], Y5[None], min_seconds=0.0, max_passes=1)
            cb5["sample"] = "one pass of the large array (n = 8192, 1024 ports; fill within RI 12 m): " + \
                            cb5["sample"].split(": ", 1)[1]
            large["cpu_baseline"] = cb5
            large["accuracy_vs_oracle"] = acc5
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
