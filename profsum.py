"""Summaries of rocprofv3 CSV output for the pair pipeline and the contractions.

Measurement harness beside bench.py (not part of the library):

    python profsum.py --workload W --trace DIR --fetch DIR --write DIR \
        --copy-fetch DIR --copy-write DIR --bench-json FILE --out profiles
    python profsum.py --workload W --trace DIR --bench-json FILE --out profiles
    python profsum.py --workload W --mfma DIR --out profiles
    python profsum.py --workload W --sq DIR DIR DIR --out profiles

DIR are rocprofv3 output directories (``--output-format csv``): a
``--kernel-trace --stats`` run of ``bench.py``, two ``--pmc`` runs of
``bench.py`` (FETCH_SIZE, then WRITE_SIZE) and the same two counters on
``bench.py --calibrate-copy`` (the plain copy kernel, 2 GiB).  Writes
``pair_pipeline_W_kernel_trace.md``, ``pair_pipeline_W_hbm_counters.md`` and
``pair_pipeline_W_traffic.json`` (calibrated HBM bytes per launch, tagged with
the digest of the kernel sources they were measured on; bench.py reports them
only while the sources still have that digest).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os

COPY_BYTES = 2 << 30
ROOT = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("exchange_kernels.hpp", "fft_core.hpp", "px_internal.hpp", "exchange_inst.hip",
                  "pair_transpose.hip")
WORKLOAD_TEXT = {"large96": "large96 workload (96^3 grid, 1536 orbitals)",
                 "mid72": "mid72 workload (72^3 grid, 512 orbitals)",
                 "mixed96": "mixed96 workload (96^3 grid, 1536 orbitals, full occupation matrix)",
                 "mixed72": "mixed72 workload (72^3 grid, 512 orbitals, full occupation matrix)"}


def source_digest():
    """Digest of the pair-pipeline kernel sources with comments and blank lines
    removed: counter figures measured on other code are not reported."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, "paper_2501_03061_amd", "csrc", name)).read()
        text = re.sub(r"//[^\n]*", "", text)
        lines = [l.strip() for l in text.splitlines() if l.strip()]
        h.update(("\n".join(lines) + "\n").encode())
    return h.hexdigest()


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"pair_pipeline_{workload}_traffic.json")


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary of
    this workload, or None when that summary was taken on different kernel
    code (or does not exist)."""
    try:
        rec = json.load(open(traffic_file(workload)))
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != source_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["read_bytes"] + k["write_bytes"]


def _csv(d, suffix):
    hits = glob.glob(os.path.join(d, f"*{suffix}"))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} in {d}")
    return list(csv.DictReader(open(hits[0])))


def _per_kernel(d):
    agg = collections.defaultdict(list)
    for r in _csv(d, "counter_collection.csv"):
        agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def _short(name):
    # "void px::pass3_inv_xy_acc<float, 72, ...>(...)" -> "pass3_inv_xy_acc"; the staged
    # form of pass 3 (FP32 at 72^3-96^3) counts as pass 3
    base = name.split("(")[0].split("<")[0]
    short = base.split("::")[-1].replace("void ", "").strip()
    return "pass3_inv_xy_acc" if short == "pass3_staged" else short


def summarize(trace, fetch, write, copy_fetch, copy_write, bench_json, out, commands, workload):
    summarize_trace(trace, bench_json, out, commands, workload)
    summarize_hbm(fetch, write, copy_fetch, copy_write, out, commands, workload)


def summarize_trace(trace, bench_json, out, commands, workload):
    os.makedirs(out, exist_ok=True)
    rec = json.loads(open(bench_json).read().strip().splitlines()[-1])
    stats = _csv(trace, "kernel_stats.csv")
    lines = [f"# Kernel trace: exchange/ACE hot path, {WORKLOAD_TEXT[workload]}", "",
             "Command ($REPO: the repository root, $OUT: the raw output folder; one MI355X):", "", "```", commands["trace"], "```", "",
             f"The bench run inside the profiler printed: value {rec['value']:.4g} pair-solves/s, "
             f"{rec['ms_per_step']:.1f} ms/step (FP32 form, Hermitian-pair mode); FP64 form "
             f"{rec['extra'].get('fp64_pair_solves_per_s', float('nan')):.4g} pair-solves/s.", "",
             "Per-pass averages measured by bench.py with HIP events over the timed region (FP32 form):", "",
             "| pass | avg per launch (us) | launches per step | ms per step | model GB/s |",
             "|---|---|---|---|---|"]
    for k, v in rec["extra"]["passes"].items():
        lines.append(f"| {k} | {v['avg_us']:.1f} | {v['launches_per_step']} | {v['ms_per_step']:.1f} | "
                     f"{v['model_GBps']:.0f} |")
    # the same passes in the trace: FP32 instantiations of each pass merged by
    # dispatch count (pass 3 runs with and without the kept v_ij)
    merged = collections.defaultdict(lambda: [0, 0.0])
    for r in stats:
        if "<float" in r["Name"] and _short(r["Name"]) in rec["extra"]["passes"]:
            m = merged[_short(r["Name"])]
            m[0] += int(r["Calls"])
            m[1] += float(r["TotalDurationNs"])
    lines += ["", "The same passes in the trace (FP32 instantiations, dispatch-weighted average over "
              "every call of the run):", "",
              "| pass | calls | trace avg (us) | bench HIP-event avg (us) | ratio |", "|---|---|---|---|---|"]
    for k, v in rec["extra"]["passes"].items():
        if k in merged and merged[k][0]:
            t = merged[k][1] / merged[k][0] / 1e3
            lines.append(f"| {k} | {merged[k][0]} | {t:.1f} | {v['avg_us']:.1f} | {t / v['avg_us']:.3f} |")
    lines += ["", "Top kernels (`kernel_stats.csv`, whole run: warmup, timed FP32 steps, FP64 comparison):", "",
              "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in stats[:18]:
        name = r["Name"] if len(r["Name"]) < 90 else r["Name"][:90] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.1f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    open(os.path.join(out, f"pair_pipeline_{workload}_kernel_trace.md"), "w").write("\n".join(lines) + "\n")


def summarize_stages(trace, bench_json, out, command, workload):
    """Kernel trace of the mixed-state time steps: the bench's stage times
    (HIP events inside its timed steps) beside the trace's kernels."""
    os.makedirs(out, exist_ok=True)
    rec = json.loads(open(bench_json).read().strip().splitlines()[-1])
    stats = _csv(trace, "kernel_stats.csv")
    ex = rec["extra"]
    steps = ex["checks"]["steps_taken"]
    lines = [f"# Kernel trace: mixed-state time steps, {WORKLOAD_TEXT[workload]}", "",
             "Command ($REPO: the repository root, $OUT: the raw output folder; one MI355X):", "",
             "```", command, "```", "",
             f"The run inside the profiler: {steps} time steps (the first untimed) after the initial "
             f"diagonalisation and rotation; {rec['ms_per_step']:.1f} ms per timed step.", "",
             "Stages of the timed step (bench.py, HIP events on the library's stream):", "",
             "| stage | ms | bound | rate | fraction of peak |", "|---|---|---|---|---|"]
    for name, st in ex["stages"].items():
        rate, frac = "", ""
        if st.get("bound") == "mfma":
            rate, frac = f"{st['TFLOPs']:.1f} TFLOP/s", f"{st['frac']:.3f} of {st['peak_TFLOPs']}"
        elif st.get("bound") == "hbm":
            rate, frac = f"{st['GBps']:.0f} GB/s", f"{st['frac']:.3f} of 8000"
        elif st.get("bound") == "alu":
            rate = f"{st['TFLOPs']:.1f} TFLOP/s, {st['GBps']:.0f} GB/s"
            frac = f"{st['frac']:.3f} of {st['peak_TFLOPs']} (HBM {st['hbm_frac']:.3f})"
        lines.append(f"| {name} | {st['ms']:.2f} | {st.get('bound', 'pipeline')} | {rate} | {frac} |")
    lines += ["", "Kernels (`kernel_stats.csv`, the whole run; the Jacobi launches include the no-op "
              "launches after convergence, which return at once):", "",
              "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in stats[:26]:
        name = r["Name"] if len(r["Name"]) < 90 else r["Name"][:90] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.1f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    fam = collections.defaultdict(float)
    for r in stats:
        name = r["Name"].replace("(anonymous namespace)::", "")
        short = name.split("(")[0].split("<")[0].split("::")[-1].replace("void ", "").strip()
        fam[short] += float(r["TotalDurationNs"]) / 1e6
    diag = (fam["bj_solve_k"] + fam["bj_apply_k"] + fam["eig_norm_part_k"] + fam["eig_conv_k"] +
            fam["eig_init_k"] + fam["eig_rank_k"] + fam["eig_permute_k"]) / (steps + 1)
    # the z pass of the fine-grid density runs as xc contractions over the n2 planes of
    # one orbital: those dispatches have ceil(n2 / 64) workgroup columns, the other xc
    # contractions (over all orbitals) many more
    n2 = rec["config"]["grid"][2]
    zpass = 0.0
    for r in _csv(trace, "kernel_trace.csv"):
        if "gemm_xc_k" in r["Kernel_Name"] and int(r["Grid_Size_Y"]) == (n2 + 63) // 64:
            zpass += (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) / 1e6
    fine = (fam["interp_x_k"] + fam["interp_strided_k"] + fam["density_acc_k"] + fam["interp_table_k"] +
            fam["interp_matrix_k"] + zpass) / steps
    lines += ["", f"Per diagonalisation in the trace ({steps + 1} of them): {diag:.1f} ms "
              f"(bench: {ex['stages']['sigma_diagonalize']['ms']:.1f} ms); density kernel "
              f"{fam['density_k'] / steps:.2f} ms per call (bench: {ex['stages']['density']['ms']:.2f} ms); "
              f"density on the fine grid {fine:.1f} ms per step (bench: "
              f"{ex['stages']['density_fine']['ms']:.1f} ms)."]
    open(os.path.join(out, f"mixed_steps_{workload}_kernel_trace.md"), "w").write("\n".join(lines) + "\n")


def summarize_hbm(fetch, write, copy_fetch, copy_write, out, commands, workload):
    fc, wc = _per_kernel(copy_fetch), _per_kernel(copy_write)
    ck = [k for k in fc if "stream_copy" in k][0]
    f_copy = sum(fc[ck]) / len(fc[ck])
    w_copy = sum(wc[ck]) / len(wc[ck])
    ff = COPY_BYTES / 1024 / f_copy
    wf = COPY_BYTES / 1024 / w_copy
    fb, wb = _per_kernel(fetch), _per_kernel(write)
    lines = [f"# HBM traffic counters: pair pipeline, {WORKLOAD_TEXT[workload]}", "",
             "Commands ($REPO: the repository root, $OUT: the raw output folder; each counter in a run of its own):", "", "```"] + commands["pmc"] + ["```", "",
             f"Calibration with the plain copy kernel (`px_stream_copy`, 2 GiB read and 2 GiB written per "
             f"launch): FETCH_SIZE reads {f_copy:,.0f} KiB per launch (factor {ff:.3f} to bytes read), "
             f"WRITE_SIZE {w_copy:,.0f} KiB (factor {wf:.3f}).", "",
             "Per dispatch, averaged over the launches of one FP32 step:", "",
             "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read GB | write GB | read+write GB |",
             "|---|---|---|---|---|---|---|"]
    kernels = {}
    for k in sorted(fb, key=lambda k: -sum(fb[k])):
        if k not in wb:
            continue
        f = sum(fb[k]) / len(fb[k])
        w = sum(wb[k]) / len(wb[k])
        if f + w < 1000:
            continue
        rb, wbts = f * ff * 1024, w * wf * 1024
        name = k if len(k) < 80 else k[:80] + "..."
        lines.append(f"| `{name}` | {len(fb[k])} | {f:,.0f} | {w:,.0f} | {rb / 1e9:.3f} | "
                     f"{wbts / 1e9:.3f} | {(rb + wbts) / 1e9:.3f} |")
        if "float" in k and _short(k).startswith("pass"):
            # instantiations of one pass (e.g. pass 3 with and without the kept
            # v_ij) merge into a dispatch-weighted average per launch
            d = len(fb[k])
            prev = kernels.get(_short(k))
            if prev:
                n = prev["dispatches"] + d
                rb = (prev["read_bytes"] * prev["dispatches"] + rb * d) / n
                wbts = (prev["write_bytes"] * prev["dispatches"] + wbts * d) / n
                d, k = n, prev["name"] + " + " + k
            kernels[_short(k)] = dict(read_bytes=rb, write_bytes=wbts, dispatches=d, name=k)
    open(os.path.join(out, f"pair_pipeline_{workload}_hbm_counters.md"), "w").write("\n".join(lines) + "\n")
    json.dump(dict(source_digest=source_digest(), fetch_factor=ff, write_factor=wf,
                   kernels=kernels, note="FP32 form, bytes per dispatch averaged over one step"),
              open(os.path.join(out, f"pair_pipeline_{workload}_traffic.json"), "w"), indent=1)


def summarize_mfma(mfma, out, command, workload):
    """MFMA counters of the contractions (one --pmc run of bench.py): flops
    from SQ_INSTS_VALU_MFMA_MOPS_* (512 flops each), MFMA busy fraction from
    SQ_VALU_MFMA_BUSY_CYCLES over 4 SIMDs x SQ_BUSY_CU_CYCLES, and the rate
    over the dispatch duration recorded with the counters."""
    rows = collections.defaultdict(lambda: collections.defaultdict(list))
    durs = collections.defaultdict(dict)
    for r in _csv(mfma, "counter_collection.csv"):
        k = r["Kernel_Name"]
        if "gemm_x" not in k:   # the MFMA contractions (xhy, xc)
            continue
        rows[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
        durs[k][r["Dispatch_Id"]] = (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) * 1e-9
    lines = [f"# MFMA counters: complex contractions, {WORKLOAD_TEXT[workload]}", "",
             "Command ($REPO: the repository root, $OUT: the raw output folder; one MI355X):", "", "```", command, "```", "",
             "Each row groups the dispatches of one kernel with the same flop count (the xi = W U "
             "contraction of the ACE build uses only the upper-triangular U, about half the flops of "
"a dense one). GFLOP = SQ_INSTS_VALU_MFMA_MOPS x 512 (the flops the matrix cores execute); "
             "MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (4 SIMDs x SQ_BUSY_CU_CYCLES); rate = GFLOP / "
             "dispatch duration; peaks 157.3 TFLOP/s (FP32 MFMA) and 78.6 TFLOP/s (FP64 MFMA). A "
             "complex product takes three real MFMAs (Gauss), so the usual count of a complex "
             "contraction (8 real flops per complex multiply-add) is 4/3 of the executed flops: "
             "the last columns give that complex-equivalent rate.", "",
             "| kernel | dispatches | GFLOP per dispatch | avg duration (ms) | TFLOP/s | % of peak | MFMA busy "
             "| complex-equivalent TFLOP/s | % of peak |",
             "|---|---|---|---|---|---|---|---|---|"]
    for k, cs in rows.items():
        mops = cs.get("SQ_INSTS_VALU_MFMA_MOPS_F32", []) if "float" in k else cs.get("SQ_INSTS_VALU_MFMA_MOPS_F64", [])
        busy, cu = cs.get("SQ_VALU_MFMA_BUSY_CYCLES", []), cs.get("SQ_BUSY_CU_CYCLES", [])
        d = list(durs[k].values())
        if not (mops and busy and cu and len(d) == len(mops)):
            continue
        peak = 157.3 if "float" in k else 78.6
        groups = collections.defaultdict(list)
        for i, m in enumerate(mops):
            groups[round(m / 1e6)].append(i)
        name = _short(k) + ("<float>" if "float" in k else "<double>")
        for g, idx in sorted(groups.items()):
            gf = g * 1e6 * 512 / 1e9
            dt = sum(d[i] for i in idx) / len(idx)
            frac = sum(busy[i] / (4 * cu[i]) for i in idx) / len(idx)
            tf = gf / dt / 1e3
            lines.append(f"| `{name}` | {len(idx)} | {gf:.0f} | {dt * 1e3:.2f} | {tf:.1f} | "
                         f"{100 * tf / peak:.0f} % | {100 * frac:.0f} % | {tf * 4 / 3:.1f} | "
                         f"{100 * tf * 4 / 3 / peak:.0f} % |")
    open(os.path.join(out, f"gemm_{workload}_mfma_counters.md"), "w").write("\n".join(lines) + "\n")


def summarize_sq(dirs, out, commands, workload):
    """SQ / TA / TCP counters of the pair-pipeline passes and the contractions
    (FP32 form, one bench step), per dispatch, with ratios whose units cancel:
    VALU issue share = SQ_INSTS_VALU / SQ_BUSY_CU_CYCLES (a wave64 VALU
    instruction holds its SIMD 4 cycles and a CU has 4 SIMDs; both counters are
    summed over CUs), wait share = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES (both per
    wave), LDS bank-conflict share = SQ_LDS_BANK_CONFLICT / SQ_BUSY_CU_CYCLES,
    TA busy share = TA_TA_BUSY / SQ_BUSY_CU_CYCLES, and the mean L2 read
    latency seen by the vector L1 = TCP_TCC_READ_REQ_LATENCY / TCP_TCC_READ_REQ."""
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in dirs:
        for r in _csv(d, "counter_collection.csv"):
            k = r["Kernel_Name"]
            if "float" not in k or not (_short(k).startswith("pass") or "gemm_" in k):
                continue
            agg[_short(k)][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = [f"# SQ / TA / TCP counters: pair pipeline and contractions, {WORKLOAD_TEXT[workload]} (FP32 form)", "",
             "Commands ($REPO: the repository root, $OUT: the raw output folder; one counter group per "
             "run):", "", "```"] + commands + ["```", "",
             "Per dispatch, averaged over the dispatches of one FP32 bench step (instantiations of a "
             "pass merged). VALU issue share = SQ_INSTS_VALU / SQ_BUSY_CU_CYCLES (a wave64 VALU "
             "instruction holds its SIMD 4 cycles, a CU has 4 SIMDs, both counters are summed over "
             "CUs); wait share = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES (time waves spend at s_waitcnt); "
             "LDS conflict share = SQ_LDS_BANK_CONFLICT / SQ_BUSY_CU_CYCLES; TA busy = TA_TA_BUSY / "
             "SQ_BUSY_CU_CYCLES; L2 latency = TCP_TCC_READ_REQ_LATENCY / TCP_TCC_READ_REQ (cycles).", "",
             "| kernel | dispatches | VALU instr. per wave | VALU issue share | wait share | LDS conflict "
             "share | TA busy | L2 read latency (cycles) |", "|---|---|---|---|---|---|---|---|"]
    order = ["pass1_fwd_xy", "pass2_z_kernel", "pass3_inv_xy_acc", "pass4_transpose_acc", "gemm_xhy_k",
             "gemm_xc_k"]

    def avg(cs, c):
        v = cs.get(c, [])
        return sum(v) / len(v) if v else float("nan")

    for k in order:
        if k not in agg:
            continue
        cs = agg[k]
        busy = avg(cs, "SQ_BUSY_CU_CYCLES")
        lines.append(
            f"| `{k}<float>` | {len(cs.get('SQ_INSTS_VALU', []))} | "
            f"{avg(cs, 'SQ_INSTS_VALU') / avg(cs, 'SQ_WAVES'):.0f} | "
            f"{100 * avg(cs, 'SQ_INSTS_VALU') / busy:.0f} % | "
            f"{100 * avg(cs, 'SQ_WAIT_INST_ANY') / avg(cs, 'SQ_WAVE_CYCLES'):.0f} % | "
            f"{100 * avg(cs, 'SQ_LDS_BANK_CONFLICT') / busy:.1f} % | "
            f"{100 * avg(cs, 'TA_TA_BUSY') / busy:.0f} % | "
            f"{avg(cs, 'TCP_TCC_READ_REQ_LATENCY') / avg(cs, 'TCP_TCC_READ_REQ'):.0f} |")
    open(os.path.join(out, f"pair_pipeline_{workload}_sq_counters.md"), "w").write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    for a in ("trace", "fetch", "write", "copy-fetch", "copy-write", "bench-json"):
        ap.add_argument("--" + a)
    ap.add_argument("--workload", default="large96", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--mfma", help="rocprofv3 --pmc run with the MFMA counters (contractions)")
    ap.add_argument("--sq", nargs="+", help="rocprofv3 --pmc runs with the SQ / TA / TCP counter groups")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    args = ap.parse_args()
    w = args.workload
    # $REPO: the repository root; $OUT: a folder for the raw rocprofv3 output
    pre = "cd /tmp && export TMPDIR=/tmp"
    one = f"--workload {w} --steps 1 --warmup 0"
    if args.sq:
        groups = ["SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS "
                  "SQ_WAIT_INST_LDS SQ_WAIT_ANY SQ_INSTS_VALU",
                  "SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_VMEM SQ_INST_LEVEL_VMEM SQ_INSTS_LDS "
                  "SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY SQ_INSTS_SALU SQ_BUSY_CU_CYCLES",
                  "TA_TA_BUSY TA_ADDR_STALLED_BY_TC_CYCLES TCP_TCC_READ_REQ_LATENCY TCP_TCC_READ_REQ"]
        summarize_sq(args.sq, args.out, [pre] + [
            f"timeout -s KILL 300 rocprofv3 --pmc {g} --output-format csv -d $OUT/pmc_sq{i + 1} -o run -- "
            f"python3 $REPO/bench.py {one} --no-fp64 --no-cpu" for i, g in enumerate(groups)], w)
        if not (args.trace or args.mfma):
            return
    if args.mfma:
        summarize_mfma(args.mfma, args.out, pre + "\ntimeout -s KILL 400 rocprofv3 --pmc "
                       "SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_VALU_MFMA_BUSY_CYCLES "
                       "SQ_BUSY_CU_CYCLES --output-format csv -d $OUT/pmc_mfma_bench -o run -- "
                       f"python3 $REPO/bench.py {one} --no-cpu", w)
        if not args.trace:
            return
    if w.startswith("mixed"):
        summarize_stages(args.trace, args.bench_json, args.out,
                         pre + "\nrocprofv3 --kernel-trace --stats --output-format csv -d $OUT/trace_" + w +
                         f" -o run -- python3 $REPO/bench.py --workload {w} --steps 1 --warmup 1 --no-cpu", w)
        return
    commands = {
        "trace": pre + "\nrocprofv3 --kernel-trace --stats --output-format csv -d $OUT/trace_bench "
                       f"-o run -- python3 $REPO/bench.py --workload {w}",
        "pmc": [pre] + [
            f"timeout -s KILL {t} rocprofv3 --pmc {c} --output-format csv -d $OUT/{d} -o run -- "
            f"python3 $REPO/bench.py {a}"
            for t, c, d, a in ((120, "FETCH_SIZE", "pmc_fetch_copy", "--calibrate-copy"),
                               (120, "WRITE_SIZE", "pmc_write_copy", "--calibrate-copy"),
                               (400, "FETCH_SIZE", "pmc_fetch_bench", f"{one} --no-fp64 --no-cpu"),
                               (400, "WRITE_SIZE", "pmc_write_bench", f"{one} --no-fp64 --no-cpu"))],
    }
    if args.fetch:
        summarize(args.trace, args.fetch, args.write, args.copy_fetch, args.copy_write, args.bench_json,
                  args.out, commands, w)
    else:  # kernel trace only
        summarize_trace(args.trace, args.bench_json, args.out, commands, w)


if __name__ == "__main__":
    main()
