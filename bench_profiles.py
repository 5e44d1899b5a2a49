"""Summaries of the benchmark's rocprofv3 runs for profiles/ (text) and the
per-launch HBM bytes that bench.py reports as roofline.traffic.

Collect, from the repository root on the GPU host, into one directory OUT
(each counter set in a run of its own; the copy runs calibrate the byte
counters against a plain device copy of 1 GiB):

  cd /tmp && export TMPDIR=/tmp
  for C in FETCH_SIZE WRITE_SIZE; do
    rocprofv3 --pmc $C --output-format csv -d OUT/pmc.$C.copy -o run -- python3 REPO/bench.py --calibrate-copy
    rocprofv3 --pmc $C --output-format csv -d OUT/pmc.$C.bench -o run -- \
        python3 REPO/bench.py --steps 2 --warmup 1 --cpu-freqs 0 --no-plain
  done
  rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_INSTS_VALU_MFMA_MOPS_F64 \
      --output-format csv -d OUT/pmc.MFMA.bench -o run -- python3 REPO/bench.py --steps 2 --warmup 1 --cpu-freqs 0 --no-plain
  rocprofv3 --kernel-trace --stats -d OUT/prof -o run -- python3 REPO/bench.py --steps 5 --warmup 1 --cpu-freqs 0 \
      --no-plain > OUT/prof.log

then: python bench_profiles.py station OUT [bench.json of an untraced `python bench.py` run]

Other workloads (one kernel trace each, summarised into profiles/NAME_kernel_trace.txt):

  rocprofv3 --kernel-trace --stats -d OUT -o run -- python3 REPO/bench.py --workload batched --steps 2 --warmup 1
  python bench_profiles.py trace OUT batched_layouts "TITLE" "COMMAND"
"""
import collections
import csv
import json
import os
import re
import sqlite3
import sys

R = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, R)
import bench  # noqa: E402

P = os.path.join(R, "profiles")

PMC_CMD = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 240 rocprofv3 --pmc {C} --output-format csv "
           "-d <out> -o run -- python3 /root/repo/bench.py --steps 2 --warmup 1 --cpu-freqs 0 --no-plain")
COPY_CMD = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 120 rocprofv3 --pmc {C} --output-format csv "
            "-d <out> -o run -- python3 /root/repo/bench.py --calibrate-copy")
MFMA_CMD = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 240 rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES "
            "GRBM_GUI_ACTIVE SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_INSTS_VALU_MFMA_MOPS_F64 --output-format csv -d <out> "
            "-o run -- python3 /root/repo/bench.py --steps 2 --warmup 1 --cpu-freqs 0 --no-plain")
TRACE_CMD = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats -d <out> -o run -- "
             "python3 /root/repo/bench.py --steps 5 --warmup 1 --cpu-freqs 0 --no-plain")
SIMDS = 256 * 4


def short(nm):
    nm = re.sub(r"\(anonymous namespace\)::", "", nm)
    nm = nm.split("(")[0].replace("void ", "").replace("harp::", "")
    return nm


def kclass(nm):
    s = short(nm)
    if s.startswith("cgemm_kernel<float"):
        return "gemm_c64"
    if s.startswith("cgemm_kernel<double"):
        return "gemm_c128"
    if s.startswith("getf2_kernel"):
        return "getf2"
    if s.startswith("laswp_kernel"):
        return "trsm_lower"
    if s.startswith("rank_update_kernel"):
        return "rank_update"
    if s.startswith("fill_kernel"):
        return "fill"
    return None


def pmc(G, C, what):
    rows = list(csv.DictReader(open(os.path.join(G, f"pmc.{C}.{what}", "run_counter_collection.csv"))))
    per = collections.defaultdict(list)
    for r in rows:
        per[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return per



def station(G, bench_json=None):
    """Summaries of the station sweep: HBM counters, kernel trace, MFMA counters
    and profiles/traffic.json."""
    # copy calibration: counter KiB read for a copy of exactly 1 GiB in, 1 GiB out
    cal = {}
    for C in ("FETCH_SIZE", "WRITE_SIZE"):
        v = pmc(G, C, "copy")["__amd_rocclr_copyBuffer"]
        cal[C] = {"kib_per_copy": sum(v) / len(v), "copies": len(v),
                  "factor": (sum(v) / len(v)) * 1024.0 / float(1 << 30)}

    fetch, write = pmc(G, "FETCH_SIZE", "bench"), pmc(G, "WRITE_SIZE", "bench")
    lines = []
    lines.append("HBM traffic of the hot-path kernels, station sweep (16 frequencies x n = 2048, 256 ports;")
    lines.append("complex64 LU + FP64 refinement), MI355X, rocprofv3 derived counters FETCH_SIZE / WRITE_SIZE")
    lines.append("(KiB per dispatch), one counter per run.")
    lines.append("")
    lines.append("Commands (one per counter C in FETCH_SIZE, WRITE_SIZE):")
    lines.append("  " + PMC_CMD)
    lines.append("  " + COPY_CMD)
    lines.append("")
    lines.append("Calibration: a plain device copy of 1 GiB (1048576 KiB read, 1048576 KiB written):")
    for C, c in cal.items():
        lines.append(f"  {C:10s} reads {c['kib_per_copy']:12.1f} KiB per copy -> scale factor {c['factor']:.4f} "
                     f"(true bytes = counter bytes / factor)")
    lines.append("")
    lines.append(f"{'kernel':58s} {'dispatches':>10s} {'fetch KiB':>12s} {'write KiB':>12s} {'HBM MB/disp':>12s}")
    lines.append(f"{'':58s} {'':>10s} {'(raw, avg)':>12s} {'(raw, avg)':>12s} {'(scaled)':>12s}")
    classes = collections.defaultdict(lambda: [0, 0.0, 0.0])
    for k in sorted(fetch, key=lambda k: -sum(fetch[k])):
        f, w = fetch[k], write.get(k, [])
        if not w:
            continue
        fa, wa = sum(f) / len(f), sum(w) / len(w)
        mb = (fa * 1024 / cal["FETCH_SIZE"]["factor"] + wa * 1024 / cal["WRITE_SIZE"]["factor"]) / 1e6
        if sum(f) + sum(w) > 1e5:
            lines.append(f"{k[:58]:58s} {len(f):10d} {fa:12.1f} {wa:12.1f} {mb:12.2f}")
        kc = kclass(k)
        if kc:
            classes[kc][0] += len(f)
            classes[kc][1] += sum(f) * 1024 / cal["FETCH_SIZE"]["factor"]
            classes[kc][2] += sum(w) * 1024 / cal["WRITE_SIZE"]["factor"]
    lines.append("")
    lines.append("Per kernel class (all tile variants of the class; the benchmark's roofline uses these):")
    traffic = {}
    for kc, (nd, fb, wb) in sorted(classes.items()):
        per = (fb + wb) / nd
        lines.append(f"  {kc:10s} dispatches {nd:6d}  fetch {fb / nd / 1e6:10.2f} MB  write {wb / nd / 1e6:10.2f} MB"
                     f"  HBM bytes per launch {per / 1e6:10.2f} MB")
        if kc in bench.KERNEL_SOURCES:
            traffic[kc] = {"hbm_bytes_per_launch": per, "fetch_bytes_per_launch": fb / nd,
                           "write_bytes_per_launch": wb / nd, "dispatches": nd,
                           "source_sha": bench._sha(bench.KERNEL_SOURCES[kc]),
                           "scale": {"FETCH_SIZE": cal["FETCH_SIZE"]["factor"], "WRITE_SIZE": cal["WRITE_SIZE"]["factor"]}}
    open(os.path.join(P, "hotpath_station_sweep_hbm_counters.txt"), "w").write("\n".join(lines) + "\n")

    # kernel trace summary
    db = sqlite3.connect(os.path.join(G, "prof", "run_results.db"))
    rows = db.execute("select name, start, end from kernels order by start").fetchall()
    st = collections.defaultdict(list)
    for nm, s, e in rows:
        st[short(nm)].append((e - s) / 1e3)
    tot = sum(sum(v) for v in st.values())
    bl = [l for l in open(os.path.join(G, "prof.log")) if l.startswith("{")]
    bj = json.loads(bl[-1]) if bl else {}
    out = []
    out.append("Kernel trace of the benchmark, station sweep (16 frequencies x n = 2048, 256 ports), MI355X.")
    out.append("Command:")
    out.append("  " + TRACE_CMD)
    out.append("(the run covers model builds, the accuracy check, warm-up, 5 uninstrumented and 5 kernel-timed steps)")
    out.append("")
    out.append(f"{'kernel':64s} {'calls':>6s} {'avg_us':>9s} {'total_ms':>9s} {'pct':>6s}")
    for k, v in sorted(st.items(), key=lambda kv: -sum(kv[1]))[:30]:
        out.append(f"{k[:64]:64s} {len(v):6d} {sum(v) / len(v):9.2f} {sum(v) / 1e3:9.3f} {100 * sum(v) / tot:6.1f}")
    out.append("")
    cls = collections.defaultdict(list)
    for k, v in st.items():
        for nm in [k]:
            kc = kclass(nm)
            if kc:
                cls[kc] += v
    out.append("Per class over the whole trace (average launch duration):")
    for kc, v in sorted(cls.items()):
        out.append(f"  {kc:10s} launches {len(v):6d}  avg {sum(v) / len(v) / 1e3:.4f} ms")
    # matrix-core work per class: the MFMA flops the hardware counted (512 per
    # MOPS unit) against the algorithmic flops bench.py charges, and the MFMA pipe
    # busy cycles over the traced launch duration at the 2.4 GHz peak clock
    mf = os.path.join(G, "pmc.MFMA.bench", "run_counter_collection.csv")
    if os.path.exists(mf):
        acc = collections.defaultdict(lambda: collections.defaultdict(float))
        disp = collections.defaultdict(set)
        for r in csv.DictReader(open(mf)):
            kc = kclass(r["Kernel_Name"])
            if kc is None:
                continue
            disp[kc].add(r["Dispatch_Id"])
            acc[kc][r["Counter_Name"]] += float(r["Counter_Value"])
        out.append("")
        out.append("Matrix cores per class, from " + MFMA_CMD + ":")
        out.append("  hardware MFMA flops = SQ_INSTS_VALU_MFMA_MOPS_{F32,F64} x 512; busy = SQ_VALU_MFMA_BUSY_CYCLES "
                   "/ (1024 SIMDs x 2.4 GHz x traced average launch)")
        for kc in ("gemm_c64", "gemm_c128"):
            if kc not in acc or not cls.get(kc):
                continue
            a, nd = acc[kc], max(1, len(disp[kc]))
            fl = (a.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) + a.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0)) * 512 / nd
            busy = a.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / nd
            dur = sum(cls[kc]) / len(cls[kc]) * 1e-6
            util = busy / (SIMDS * 2.4e9 * dur)
            out.append(f"  {kc:10s} dispatches {nd:6d}  hardware MFMA flops per dispatch {fl / 1e9:8.3f} G  "
                       f"MFMA busy over the traced duration {100 * util:5.1f} %")
            if kc in traffic:
                traffic[kc]["hw_mfma_flops_per_dispatch"] = fl
    # achieved HBM bandwidth per class: counter bytes per launch over the traced
    # average launch duration, against the 8 TB/s peak
    if traffic:
        out.append("")
        out.append("HBM bandwidth per class (counter bytes per launch / traced average launch; peak 8000 GB/s):")
        for kc in sorted(traffic):
            if not cls.get(kc):
                continue
            dur = sum(cls[kc]) / len(cls[kc]) * 1e-6
            gbs = traffic[kc]["hbm_bytes_per_launch"] / dur / 1e9
            out.append(f"  {kc:10s} {traffic[kc]['hbm_bytes_per_launch'] / 1e6:10.2f} MB per launch in "
                       f"{dur * 1e3:8.4f} ms -> {gbs:8.1f} GB/s ({100 * gbs / 8000:5.1f} % of peak)")
            traffic[kc]["achieved_gbs"] = gbs
    def bench_line(j, what):
        rf = j.get("roofline", {})
        out.append(f"  {what}: ms_per_step {j.get('ms_per_step'):.3f}  dominant class {rf.get('kernel')}  "
                   f"avg_launch_ms {rf.get('avg_launch_ms'):.4f}  achieved {rf.get('achieved'):.2f} {rf.get('unit')}"
                   f"  launches_per_step {rf.get('launches_per_step')}")


    if bench_json:
        sj = [l for l in open(bench_json) if l.startswith("{")]
        out.append("")
        out.append("The benchmark's live kernel timers (HIP events attached to each dispatch, kernel-timed steps):")
        bench_line(json.loads(sj[-1]), "python bench.py (no tracer)")
        if bj:
            bench_line(bj, "the traced command above   ")
            out.append("  (under the tracer the dispatch-attached events also carry the tracer's per-dispatch work;")
            out.append("   the tracer's own kernel durations above are the figure to compare with the untraced run)")
    # one step window: from the last-but-one to the last dual fill launch
    idx = [i for i, r in enumerate(rows) if "fill_kernel" in r[0] and "true" in r[0]]
    if len(idx) >= 2:
        seg = rows[idx[-2]:idx[-1]]
        busy = collections.defaultdict(float)
        for nm, s, e in seg:
            busy[kclass(nm) or "other"] += (e - s) / 1e6
        span = (rows[idx[-1]][1] - rows[idx[-2]][1]) / 1e6
        out.append("")
        out.append(f"One kernel-timed step under the tracer: span {span:.2f} ms, busy per class (ms): " +
                   ", ".join(f"{k} {v:.2f}" for k, v in sorted(busy.items(), key=lambda kv: -kv[1])))
    open(os.path.join(P, "hotpath_station_sweep_kernel_trace.txt"), "w").write("\n".join(out) + "\n")
    json.dump(traffic, open(os.path.join(P, "traffic.json"), "w"), indent=1)
    print("\n".join(lines[-8:]))
    print("\n".join(out[-12:]))



def trace(G, name, title, command):
    """profiles/<name>_kernel_trace.txt from the kernel trace of one run
    (rocprofv3 --kernel-trace --stats ... -d G -o run): the kernels by total
    time and the per-class launch counts and averages."""
    db = sqlite3.connect(os.path.join(G, "run_results.db"))
    rows = db.execute("select name, start, end from kernels order by start").fetchall()
    st = collections.defaultdict(list)
    for nm, s0, e0 in rows:
        st[short(nm)].append((e0 - s0) / 1e3)
    tot = sum(sum(v) for v in st.values())
    out = [title, "Command:", "  " + command, ""]
    out.append(f"{'kernel':64s} {'calls':>6s} {'avg_us':>9s} {'total_ms':>9s} {'pct':>6s}")
    for k, v in sorted(st.items(), key=lambda kv: -sum(kv[1]))[:30]:
        out.append(f"{k[:64]:64s} {len(v):6d} {sum(v) / len(v):9.2f} {sum(v) / 1e3:9.3f} {100 * sum(v) / tot:6.1f}")
    cls = collections.defaultdict(list)
    for k, v in st.items():
        kc = kclass(k)
        if kc:
            cls[kc] += v
    out.append("")
    out.append("Per class over the whole trace:")
    for kc, v in sorted(cls.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"  {kc:12s} launches {len(v):7d}  avg {sum(v) / len(v) / 1e3:8.4f} ms  total {sum(v) / 1e3:9.2f} ms")
    open(os.path.join(P, f"{name}_kernel_trace.txt"), "w").write("\n".join(out) + "\n")
    print("\n".join(out[:20]))


if __name__ == "__main__":
    if sys.argv[1] == "station":
        station(os.path.abspath(sys.argv[2]), sys.argv[3] if len(sys.argv) > 3 else None)
    elif sys.argv[1] == "trace":
        trace(os.path.abspath(sys.argv[2]), sys.argv[3], sys.argv[4], sys.argv[5])
    else:
        raise SystemExit("usage: bench_profiles.py station OUT [bench.json] | trace OUT NAME TITLE COMMAND")
