"""rocprofv3 passes over the benchmark and their text summaries.

    python -m paper_2504_12004_amd.profiling run [--out DIR]
    python -m paper_2504_12004_amd.profiling summarize [--out DIR] [--write profiles]

`run` starts each profiler pass as a child process (this process never touches
the GPU): a kernel trace with statistics of a short benchmark run, the HBM
byte counters FETCH_SIZE and WRITE_SIZE of the same run (one pass each), and
the same two counters over a plain 1 GiB device copy, which gives the factors
that turn counter readings into bytes.  `summarize` reads the rocpd databases
the passes wrote and writes a markdown summary plus a small JSON with the
per-launch HBM bytes of the dominant kernel, tagged with a hash of the kernel
sources so that a later change of the kernel invalidates it.
"""
import argparse
import hashlib
import json
import os
import re
import sqlite3
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ("paper_2504_12004_amd/csrc/loglik_kernels.hip", "paper_2504_12004_amd/csrc/sbv_internal.h",
                  "paper_2504_12004_amd/build.py")
BENCH_ARGS = ["--steps", "10", "--warmup", "2", "--no-cpu-baseline", "--fit-evals", "0", "--large-steps", "0"]
COUNTER_BENCH_ARGS = ["--steps", "3", "--warmup", "1", "--no-cpu-baseline", "--fit-evals", "0", "--large-steps", "0"]
# shader-sequencer counters, at most 8 per pass
SQ_PASSES = {
    "sq_a": ["SQ_INSTS_VALU", "SQ_INSTS_MFMA", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_ACTIVE_INST_VALU",
             "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_BUSY_CU_CYCLES", "SQ_WAVE_CYCLES"],
    "sq_b": ["SQ_WAIT_INST_ANY", "SQ_WAIT_ANY", "SQ_WAIT_INST_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS",
             "SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_CYCLES", "SQ_WAVES"],
}


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


LARGE_BENCH_ARGS = ["--steps", "1", "--warmup", "1", "--no-cpu-baseline", "--fit-evals", "0", "--large-steps", "2"]


def passes(out, workload="uneven_1m"):
    py = sys.executable
    bench = os.path.join(ROOT, "bench.py")
    if workload == "m400_5m":
        # the m = 400, n = 5e6 leg: kernel trace and the two HBM byte counters
        # (the copy calibration is shared with the headline workload's passes)
        return [
            ("trace", 600, ["rocprofv3", "--kernel-trace", "--stats", "-d", f"{out}/trace", "-o", "bench", "--",
                            py, bench] + LARGE_BENCH_ARGS),
            ("fetch", 600, ["rocprofv3", "--pmc", "FETCH_SIZE", "-d", f"{out}/fetch", "-o", "bench", "--",
                            py, bench] + LARGE_BENCH_ARGS),
            ("write", 600, ["rocprofv3", "--pmc", "WRITE_SIZE", "-d", f"{out}/write", "-o", "bench", "--",
                            py, bench] + LARGE_BENCH_ARGS),
            ("copy_fetch", 200, ["rocprofv3", "--pmc", "FETCH_SIZE", "-d", f"{out}/copy_fetch", "-o", "copy", "--",
                                 py, bench, "--copy-calibration"]),
            ("copy_write", 200, ["rocprofv3", "--pmc", "WRITE_SIZE", "-d", f"{out}/copy_write", "-o", "copy", "--",
                                 py, bench, "--copy-calibration"]),
        ]
    return [
        ("trace", 400, ["rocprofv3", "--kernel-trace", "--stats", "-d", f"{out}/trace", "-o", "bench", "--",
                        py, bench] + BENCH_ARGS),
        ("fetch", 400, ["rocprofv3", "--pmc", "FETCH_SIZE", "-d", f"{out}/fetch", "-o", "bench", "--",
                        py, bench] + COUNTER_BENCH_ARGS),
        ("write", 400, ["rocprofv3", "--pmc", "WRITE_SIZE", "-d", f"{out}/write", "-o", "bench", "--",
                        py, bench] + COUNTER_BENCH_ARGS),
        ("copy_fetch", 200, ["rocprofv3", "--pmc", "FETCH_SIZE", "-d", f"{out}/copy_fetch", "-o", "copy", "--",
                             py, bench, "--copy-calibration"]),
        ("copy_write", 200, ["rocprofv3", "--pmc", "WRITE_SIZE", "-d", f"{out}/copy_write", "-o", "copy", "--",
                             py, bench, "--copy-calibration"]),
    ] + [(name, 400, ["rocprofv3", "--pmc"] + ctrs + ["-d", f"{out}/{name}", "-o", "bench", "--", py, bench]
          + COUNTER_BENCH_ARGS) for name, ctrs in SQ_PASSES.items()]


def run(out, workload="uneven_1m"):
    os.makedirs(out, exist_ok=True)
    env = dict(os.environ, TMPDIR="/tmp")
    for name, limit, cmd in passes(out, workload):
        print(f"[prof] {name}: {' '.join(cmd)}", flush=True)
        with open(f"{out}/{name}.out", "w") as fo, open(f"{out}/{name}.err", "w") as fe:
            try:
                rc = subprocess.run(["timeout", "-s", "KILL", str(limit)] + cmd, cwd=ROOT, env=env, stdout=fo,
                                    stderr=fe).returncode
            except OSError as e:
                print(f"[prof] {name} could not start: {e}", flush=True)
                return 1
        print(f"[prof] {name} exit {rc}", flush=True)
        if rc != 0:
            return rc
    with open(f"{out}/commands.json", "w") as f:
        json.dump({n: " ".join(c).replace(ROOT + "/", "").replace(sys.executable, "python")
                   for n, _, c in passes(out, workload)}, f, indent=1)
    return 0


def _db(path):
    for root, _, files in os.walk(path):
        for fn in files:
            if fn.endswith("_results.db"):
                return sqlite3.connect(os.path.join(root, fn))
    raise FileNotFoundError(f"no rocpd database under {path}")


def _groups(con):
    """(kernel name, grid size) -> list of (dispatch id, duration ns)."""
    g = {}
    for name, grid, dur, did in con.execute(
            "select name, grid_x * grid_y * grid_z, duration, dispatch_id from kernels order by dispatch_id"):
        g.setdefault((name, grid), []).append((did, dur))
    return g


def _counter(con, counter):
    """(kernel name, grid size) -> list of per-dispatch counter values."""
    g = {}
    for name, grid, val in con.execute(
            "select kernel_name, grid_size, value from counters_collection where counter_name = ? "
            "order by dispatch_id", (counter,)):
        g.setdefault((name, grid), []).append(val)
    return g


def _short(name, n=110):
    return name if len(name) <= n else name[:n - 3] + "..."


def summarize(out, write_dir):
    cmds = {}
    if os.path.exists(f"{out}/commands.json"):
        with open(f"{out}/commands.json") as f:
            cmds = json.load(f)
    tr = _db(f"{out}/trace")
    groups = _groups(tr)
    # dominant launch group of the FP64 evaluation: largest total time
    hot = [k for k in groups if "k_block_loglik<double" in k[0]]
    dom = max(hot, key=lambda k: sum(d for _, d in groups[k]))
    durs = [d for _, d in groups[dom]]
    avg_ms = sum(durs) / len(durs) / 1e6
    top = list(tr.execute("select name, total_calls, total_duration, average, percentage from top_kernels "
                          "order by total_duration desc limit 12"))
    fetch = _counter(_db(f"{out}/fetch"), "FETCH_SIZE")
    write = _counter(_db(f"{out}/write"), "WRITE_SIZE")
    cf = _counter(_db(f"{out}/copy_fetch"), "FETCH_SIZE")
    cw = _counter(_db(f"{out}/copy_write"), "WRITE_SIZE")
    copy_bytes = 1 << 30
    # the plain copy: the launch group that reads the most (the fill that
    # initialises the source writes 1 GiB too, but reads nothing)
    ck = max(cf, key=lambda k: sum(cf[k]) / len(cf[k]))
    f_copy_kib = sum(cf[ck]) / len(cf[ck])
    w_copy_kib = sum(cw[ck]) / len(cw[ck])
    f_scale = copy_bytes / (f_copy_kib * 1024)
    w_scale = copy_bytes / (w_copy_kib * 1024)
    fk = fetch.get(dom, [])
    wk = write.get(dom, [])
    fetch_b = sum(fk) / len(fk) * 1024 * f_scale if fk else None
    write_b = sum(wk) / len(wk) * 1024 * w_scale if wk else None
    traffic = (fetch_b + write_b) if fk and wk else None
    bench_line = None
    if os.path.exists(f"{out}/trace.out"):
        with open(f"{out}/trace.out") as f:
            for line in f:
                if line.startswith("{"):
                    bench_line = json.loads(line)
    res = {
        "kernel": dom[0], "grid_threads": dom[1], "launches": len(durs), "avg_launch_ms": avg_ms,
        "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b, "bytes_per_launch": traffic,
        "fetch_scale": f_scale, "write_scale": w_scale, "copy_kernel": ck[0],
        "kernel_source_hash": kernel_source_hash(),
        "bench_avg_launch_ms": bench_line["roofline"]["avg_launch_ms"] if bench_line else None,
    }
    os.makedirs(write_dir, exist_ok=True)
    with open(os.path.join(write_dir, "k_block_loglik_uneven_1m_traffic.json"), "w") as f:
        json.dump(res, f, indent=1)
    L = []
    L.append("# k_block_loglik on uneven_1m (n = 1e6, d = 10, K = 49981, m = 200, FP64)\n")
    L.append("Made by `python -m paper_2504_12004_amd.profiling run` then `... summarize`, which ran:\n")
    for k in ("trace", "fetch", "write", "copy_fetch", "copy_write") + tuple(SQ_PASSES):
        if k in cmds:
            L.append(f"- {k}: `{cmds[k].replace(ROOT + '/', '').replace(sys.executable, 'python')}`")
    L.append("")
    L.append("## Kernel trace (rocprofv3 --kernel-trace --stats), top kernels by total time\n")
    L.append("| kernel | calls | total ms | avg ms | % |")
    L.append("|---|---|---|---|---|")
    for name, calls, tot, avg, pct in top:
        # the top_kernels view reports microseconds
        L.append(f"| `{_short(name)}` | {calls} | {tot / 1e3:.3f} | {avg / 1e3:.4f} | {pct:.1f} |")
    L.append("")
    L.append("Per-name averages mix every size bucket that launches the same kernel (and the autotuner's")
    L.append("trial launches); the dominant launch group below is one kernel at one grid size.\n")
    L.append("## Dominant launch group\n")
    L.append(f"- kernel: `{dom[0]}`")
    L.append(f"- grid: {dom[1]} threads, {len(durs)} launches, average {avg_ms:.3f} ms "
             f"(min {min(durs) / 1e6:.3f}, max {max(durs) / 1e6:.3f})")
    if bench_line:
        L.append(f"- the benchmark's own HIP-event average for this bucket in the same run: "
                 f"{bench_line['roofline']['avg_launch_ms']:.3f} ms")
    L.append("")
    L.append("## HBM bytes (rocprofv3 --pmc, one counter per pass)\n")
    L.append(f"- plain 1 GiB copy (`{_short(ck[0], 60)}`): FETCH_SIZE {f_copy_kib:.0f} KiB, "
             f"WRITE_SIZE {w_copy_kib:.0f} KiB -> scale factors {f_scale:.3f} (fetch), {w_scale:.3f} (write)")
    if fk:
        L.append(f"- dominant group FETCH_SIZE: {sum(fk) / len(fk):.0f} KiB per launch over {len(fk)} launches "
                 f"-> {fetch_b / 1e9:.3f} GB")
    if wk:
        L.append(f"- dominant group WRITE_SIZE: {sum(wk) / len(wk):.0f} KiB per launch over {len(wk)} launches "
                 f"-> {write_b / 1e9:.3f} GB")
    if traffic:
        L.append(f"- HBM traffic per launch: {traffic / 1e9:.3f} GB; at the trace's average duration that is "
                 f"{traffic / (avg_ms * 1e-3) / 1e9:.0f} GB/s of the 8000 GB/s peak")
    L.append(f"- kernel source hash: `{res['kernel_source_hash']}`")
    sq = {}
    for name, ctrs in SQ_PASSES.items():
        if not os.path.isdir(f"{out}/{name}"):
            continue
        con = _db(f"{out}/{name}")
        for c in ctrs:
            v = _counter(con, c).get(dom, [])
            if v:
                sq[c] = sum(v) / len(v)
    if sq:
        L.append("")
        L.append("## Shader-sequencer counters of the dominant launch group (per launch)\n")
        L.append("| counter | value |")
        L.append("|---|---|")
        for c, v in sq.items():
            L.append(f"| {c} | {v:.4g} |")
        if "SQ_VALU_MFMA_BUSY_CYCLES" in sq and "SQ_BUSY_CU_CYCLES" in sq and sq["SQ_BUSY_CU_CYCLES"] > 0:
            L.append(f"\nSQ_VALU_MFMA_BUSY_CYCLES / SQ_BUSY_CU_CYCLES = "
                     f"{sq['SQ_VALU_MFMA_BUSY_CYCLES'] / sq['SQ_BUSY_CU_CYCLES']:.3f}")
        res["sq"] = sq
        with open(os.path.join(write_dir, "k_block_loglik_uneven_1m_traffic.json"), "w") as f:
            json.dump(res, f, indent=1)
    with open(os.path.join(write_dir, "k_block_loglik_uneven_1m.md"), "w") as f:
        f.write("\n".join(L) + "\n")
    print("\n".join(L))
    return 0


def summarize_large(out, write_dir):
    """Summary of the m = 400 leg: the prefix-elimination kernel and the
    trailing register kernel of the large path, per evaluation."""
    cmds = {}
    if os.path.exists(f"{out}/commands.json"):
        with open(f"{out}/commands.json") as f:
            cmds = json.load(f)
    tr = _db(f"{out}/trace")
    bench_line = None
    if os.path.exists(f"{out}/trace.out"):
        with open(f"{out}/trace.out") as f:
            for line in f:
                if line.startswith("{"):
                    bench_line = json.loads(line)
    big = bench_line["extra"]["m400_5m"] if bench_line else None
    # kernels of the large path in FP64: the prefix-elimination kernel and the
    # register kernel in large-block mode (last template flag true), forward
    # (GRAD false) or gradient (GRAD true).  A prefix launch belongs to the
    # register launch that follows it.  FP32 evaluations also launch the FP64
    # pair over their fallback list, which is empty unless a block lost
    # positive definiteness: such launches end within microseconds and are
    # counted apart.
    rows = list(tr.execute("select name, duration from kernels order by dispatch_id"))

    def kind(name):
        if "k_block_prefix<double" in name:
            return "prefix"
        if "k_block_loglik<double, 17, 8, false, false, false, true" in name:
            return "trailing"
        if "k_block_loglik<double, 17, 8, true, false, false, true" in name:
            return "trailing_grad"
        return None
    empty_ns = 50e3
    per, n_empty, pending = {}, {}, []
    for name, dur in rows:
        k = kind(name)
        if k == "prefix":
            pending.append(dur)
            continue
        if k is None:
            continue
        pk = "prefix" if k == "trailing" else "prefix_grad"
        for dp in pending:
            if dp < empty_ns:
                n_empty[pk] = n_empty.get(pk, 0) + 1
            else:
                per.setdefault(pk, []).append(dp)
        pending = []
        if dur < empty_ns:
            n_empty[k] = n_empty.get(k, 0) + 1
        else:
            per.setdefault(k, []).append(dur)
    fetch = _counter(_db(f"{out}/fetch"), "FETCH_SIZE")
    write = _counter(_db(f"{out}/write"), "WRITE_SIZE")
    cf = _counter(_db(f"{out}/copy_fetch"), "FETCH_SIZE")
    cw = _counter(_db(f"{out}/copy_write"), "WRITE_SIZE")
    ck = max(cf, key=lambda k: sum(cf[k]) / len(cf[k]))
    f_scale = (1 << 30) / (sum(cf[ck]) / len(cf[ck]) * 1024)
    w_scale = (1 << 30) / (sum(cw[ck]) / len(cw[ck]) * 1024)

    def bytes_of(counter, scale, k):
        v = [x for (name, _), vals in counter.items() if kind(name) == k for x in vals]
        return sum(v) * 1024 * scale if v else None
    m = re.search(r"--large-steps (\d+)", cmds.get("trace", ""))
    evals = int(m.group(1)) + 1 if m else None
    L = ["# Large-set path on m400_5m (n = 5e6, d = 10, K = 2.5e5, m = 400, FP64)\n",
         "Made by `python -m paper_2504_12004_amd.profiling run --workload m400_5m` then "
         "`... summarize --workload m400_5m`, which ran:\n"]
    for k in ("trace", "fetch", "write", "copy_fetch", "copy_write"):
        if k in cmds:
            L.append(f"- {k}: `{cmds[k]}`")
    L += ["", f"The trace holds {evals} FP64 forward evaluations (1 warm-up + the timed ones) and as many",
          "gradient evaluations, each of them one window after another of prefix + register launches.",
          f"FP32 evaluations launch the FP64 pair over their (empty) fallback lists: launches under "
          f"{empty_ns / 1e3:.0f} us", "are counted apart and left out of the averages. The counter runs "
          "repeat the same command; their bytes", "(scaled by the copy-kernel calibration) are split over "
          "the non-empty launches, prefix bytes over", "forward and gradient prefix launches alike (the "
          "prefix kernel does the same work in both).", "",
          "| kernel | launches | empty | avg ms | ms per evaluation | FETCH GB/launch | WRITE GB/launch |",
          "|---|---|---|---|---|---|---|"]
    res = {"kernel_source_hash": kernel_source_hash(), "evaluations": evals}
    n_pref = len(per.get("prefix", [])) + len(per.get("prefix_grad", []))
    for k, label in (("prefix", "k_block_prefix<double, 8> (forward)"),
                     ("prefix_grad", "k_block_prefix<double, 8> (gradient)"),
                     ("trailing", "k_block_loglik<double, 17, 8, forward, large-block mode>"),
                     ("trailing_grad", "k_block_loglik<double, 17, 8, gradient, large-block mode>")):
        d = per.get(k, [])
        ck_ = "prefix" if k.startswith("prefix") else k
        nl = n_pref if ck_ == "prefix" else len(d)
        fb, wb = bytes_of(fetch, f_scale, ck_), bytes_of(write, w_scale, ck_)
        fpl = fb / nl if fb and nl else None
        wpl = wb / nl if wb and nl else None
        avg = sum(d) / max(len(d), 1) / 1e6
        per_eval = sum(d) / 1e6 / evals if evals else None
        L.append(f"| `{label}` | {len(d)} | {n_empty.get(k, 0)} | {avg:.3f} | "
                 f"{'%.1f' % per_eval if per_eval is not None else '-'} | "
                 f"{'%.3f' % (fpl / 1e9) if fpl else '-'} | {'%.3f' % (wpl / 1e9) if wpl else '-'} |")
        res[k] = {"launches": len(d), "empty_launches": n_empty.get(k, 0), "total_ms": sum(d) / 1e6,
                  "avg_ms": avg, "ms_per_eval": per_eval, "fetch_bytes_per_launch": fpl,
                  "write_bytes_per_launch": wpl}
    if big:
        L += ["", f"- benchmark (same run): FP64 {big['fp64']['ms_per_eval']:.1f} ms per evaluation, "
              f"{big['algorithmic_tflop_per_eval']:.3f} TFLOP algorithmic per evaluation, "
              f"{big['fp64']['total_algorithmic_tflops']:.2f} TFLOP/s = "
              f"{big['fp64']['total_algorithmic_tflops'] / 78.6:.3f} of the FP64 peak"]
    os.makedirs(write_dir, exist_ok=True)
    with open(os.path.join(write_dir, "k_block_large_m400_5m.md"), "w") as f:
        f.write("\n".join(L) + "\n")
    with open(os.path.join(write_dir, "k_block_large_m400_5m.json"), "w") as f:
        json.dump(res, f, indent=1)
    print("\n".join(L))
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["run", "summarize", "all"])
    ap.add_argument("--out", default=None)
    ap.add_argument("--write", default=os.path.join(ROOT, "profiles"))
    ap.add_argument("--workload", choices=["uneven_1m", "m400_5m"], default="uneven_1m")
    a = ap.parse_args()
    out = a.out or os.path.join(ROOT, "prof_raw" if a.workload == "uneven_1m" else "prof_raw_m400")
    rc = 0
    if a.what in ("run", "all"):
        rc = run(out, a.workload)
    if rc == 0 and a.what in ("summarize", "all"):
        rc = summarize(out, a.write) if a.workload == "uneven_1m" else summarize_large(out, a.write)
    sys.exit(rc)


if __name__ == "__main__":
    main()
