#!/usr/bin/env python
"""Throughput of the exchange / ACE hot path on one MI355X.

One step is one pass of the whole path over the resident synthetic instance:
  staging of Psi and Phi_n to complex64 (FP32 form),
  ACE build: W = Vx Psi through the fused pair pipeline (N^2 pair solves),
    M = dV Psi^H W, Hermitisation, FP64 Cholesky of -M, U = L^-H, xi = W U,
  4 PT-IM-style fixed-point iterations with the ACE operator and FP64 residuals.
The headline value is logical pair solves per second of whole steps.  The
plain FP64 form of the same step is timed after the headline run for the
precision/speed comparison, and the CPU oracle is timed on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pair_pipeline_mid72_traffic.json")
KERNEL_SOURCES = ("exchange_kernels.hpp", "fft_core.hpp", "px_internal.hpp", "exchange_inst.hip",
                  "pair_transpose.hip")


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


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when that summary was taken on different kernel code."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != source_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["read_bytes"] + k["write_bytes"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_inputs(cfg):
    import numpy as np
    import torch
    from paper_2501_03061_amd import inputs
    t0 = time.perf_counter()
    inst = inputs.make_instance(cfg["n"], cfg["L"], cfg["n_orb"], cfg["kT"], seed=cfg["seed"])
    z = inputs.noise_block(inst.n, inst.L, inst.n_orb, seed=1001)
    phi_n = inst.psi + 1e-3 * z
    del z
    psi_d = torch.from_numpy(inst.psi).cuda()
    phi_d = torch.from_numpy(phi_n).cuda()
    occ_d = torch.from_numpy(inst.occ).cuda()
    del phi_n
    log(f"inputs generated in {time.perf_counter() - t0:.1f}s "
        f"(frac. occupations 0.01<f<0.99: {float(np.mean((inst.occ > 0.01) & (inst.occ < 0.99))):.3f})")
    return inst, psi_d, phi_d, occ_d


class Step:
    """One pass of the hot path in one precision form, buffers preallocated."""

    def __init__(self, ctx, cell, psi64, phi64, occ, kern, fp32, n_iter=4):
        import torch
        from paper_2501_03061_amd import px
        self.ctx, self.cell, self.fp32, self.n_iter = ctx, cell, fp32, n_iter
        self.psi64, self.phi64, self.occ, self.kern = psi64, phi64, occ, kern
        dt = torch.complex64 if fp32 else torch.complex128
        n = psi64.shape[0]
        dev = psi64.device
        self.psi = torch.empty(psi64.shape, dtype=dt, device=dev) if fp32 else psi64
        self.phi = torch.empty(phi64.shape, dtype=dt, device=dev) if fp32 else phi64
        self.xi = torch.empty(psi64.shape, dtype=dt, device=dev)
        self.out = torch.empty(phi64.shape, dtype=dt, device=dev)
        self.M = torch.empty((n, n), dtype=torch.complex128, device=dev)
        self.ex = torch.zeros(1, dtype=torch.float64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.res = torch.zeros(n_iter, dtype=torch.float64, device=dev)
        prec = px.PX_PREC_FP32 if fp32 else px.PX_PREC_FP64
        need = max(ctx.workspace_bytes(px.PX_OP_ACE_BUILD, cell, prec, n),
                   ctx.workspace_bytes(px.PX_OP_PTIM_LOOP, cell, prec, n, n))
        ctx.ensure_workspace(need)

    def __call__(self):
        c = self.ctx
        if self.fp32:
            c.px_convert_c128_to_c64(self.psi64, self.psi)
            c.px_convert_c128_to_c64(self.phi64, self.phi)
        c.px_ace_build(self.cell, self.psi, self.occ, self.kern, xi=self.xi, M=self.M,
                       e_x=self.ex, status=self.status)
        c.px_ptim_exchange_loop(self.cell, self.xi, self.phi, self.n_iter, DT_ALPHA,
                                out=self.out, residuals=self.res)


# Time step 50 as in atomic units of time times the hybrid mixing fraction 0.25.
DT_ALPHA = 50.0 / 24.188843265857 * 0.25


def ace_stages(prof, ace):
    """Per ACE build (ms): pair pipeline (passes 1-4), M contraction,
    factorisation (Hermitise, Cholesky, inverse), xi contraction."""
    calls = max(1, ace["calls"])
    return dict(pair_pipeline=sum(p["ms"] for p in prof) / calls, M_contraction=ace["M"] / calls,
                factorization=ace["factor"] / calls, xi_contraction=ace["xi"] / calls, builds=ace["calls"])


def run_steps(step, k):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(k):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / k


def copy_bandwidth(ctx, nbytes=2 << 30, reps=5):
    """Plain copy of nbytes (read + write = 2*nbytes moved) with the library's copy kernel."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    ctx.px_stream_copy(src, dst)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.px_stream_copy(src, dst)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del src, dst
    return dict(copy_bytes=nbytes, copy_GBps=2 * nbytes / dt / 1e9, copy_ms=dt * 1e3)


def cpu_baseline(inst, kern_np, seconds):
    """The oracle as it stands on a bounded sample: a few output columns of
    W = Vx Psi against all orbitals."""
    import numpy as np
    import oracle
    cols = 1
    t0 = time.perf_counter()
    oracle.exchange_apply(inst.psi, inst.occ, inst.psi[:cols], kern_np)
    t1 = time.perf_counter() - t0
    more = max(0, min(inst.n_orb - 1, int(seconds / max(t1, 1e-3)) - 1))
    t2 = 0.0
    if more:
        t0 = time.perf_counter()
        oracle.exchange_apply(inst.psi, inst.occ, inst.psi[cols:cols + more], kern_np)
        t2 = time.perf_counter() - t0
    pairs = (cols + more) * inst.n_orb
    return dict(value=pairs / (t1 + t2), unit="pair-solves/s", cores=os.cpu_count(), kind="oracle",
                sample=f"{cols + more} output orbitals x {inst.n_orb} density orbitals "
                       f"({pairs} pair solves) of the same instance, {t1 + t2:.1f}s, "
                       f"scipy.fft workers={os.cpu_count()}")


def bench_batch48(args):
    """48 uneven instances (grids {32,40,48,64}^3, 32..256 orbitals): FP32 ACE
    builds of all of them in one batched, graph-replayed call, against the
    same builds one instance at a time (FP32 and plain FP64)."""
    import torch
    from paper_2501_03061_amd import inputs, px
    ctx = px.Context(0)
    t0 = time.perf_counter()
    recipe = inputs.batch_recipe()
    insts, args64 = [], []
    for r in recipe:
        inst = inputs.make_instance(r["n"], r["L"], r["n_orb"], r["kT"], seed=r["seed"])
        cell = px.Cell(inst.L, inst.n)
        args64.append(dict(cell=cell, psi=torch.from_numpy(inst.psi).cuda(),
                           occ=torch.from_numpy(inst.occ).cuda(), kern=ctx.px_kernel_hse(cell, 0.106)))
        insts.append((inst.n[0], inst.n_orb))
        del inst
    log(f"batch48 inputs in {time.perf_counter() - t0:.1f}s")
    args32 = [dict(a, psi=ctx.px_convert_c128_to_c64(a["psi"])) for a in args64]
    for a in args32:
        a["out"] = torch.empty_like(a["psi"])
        a["status"] = torch.zeros(1, dtype=torch.int32, device="cuda")
    blocks = {}
    for n in sorted(set(i[0] for i in insts)):
        k = max((i for i, x in enumerate(insts) if x[0] == n), key=lambda i: insts[i][1])
        blocks[n] = ctx.px_autotune(args32[k]["cell"], args32[k]["psi"], args32[k]["occ"], args32[k]["kern"])
    log(f"autotuned blocks {blocks}")
    pairs = sum(n_orb * n_orb for _, n_orb in insts)

    def batched():
        ctx.px_exchange_apply_batched(args32, ace=True)
    for _ in range(max(1, args.warmup)):
        batched()                                  # first call captures the graph
    torch.cuda.synchronize()
    ms_b = 1e3 * run_steps(batched, args.steps)
    ctx.px_sync()

    def single(a_list):
        def f():
            for a in a_list:
                ctx.px_ace_build(a["cell"], a["psi"], a["occ"], a["kern"], xi=a.get("out"),
                                 status=a.get("status"))
        return f
    ms_1 = 1e3 * run_steps(single(args32), 1)
    for a in args64:
        a["out"] = torch.empty_like(a["psi"])
        a["status"] = torch.zeros(1, dtype=torch.int32, device="cuda")
    single(args64)()
    torch.cuda.synchronize()
    ms_64 = 1e3 * run_steps(single(args64), 1)
    ctx.px_sync()
    rec = {
        "metric": "exchange pair-solves/s + ACE build s, FP32-batched vs FP64 at <=2e-5 err",
        "value": pairs / (ms_b * 1e-3), "unit": "pair-solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_b, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch48: 48 instances, grids {32,40,48,64}^3, 32..256 orbitals, "
                               "kT 0.005..0.05 Ha, L = 0.28 n bohr; FP32 ACE builds, batched + graph",
                   "pairs_per_step": pairs},
        "extra": {"autotuned_blocks": blocks, "single_fp32_ms": ms_1, "single_fp64_ms": ms_64,
                  "single_fp32_pair_solves_per_s": pairs / (ms_1 * 1e-3),
                  "single_fp64_pair_solves_per_s": pairs / (ms_64 * 1e-3),
                  "speedup_batched_fp32_vs_single_fp64": ms_64 / ms_b},
    }
    ctx.close()
    return rec


def bench_large96(args):
    """The large single-GPU share (96^3, 1536 orbitals, kT 0.03): one step of
    each form (staging, ACE build, 4 PT-IM-style ACE iterations), timed after
    one untimed step, and the ACE builds alone; FP32 against FP64 errors."""
    import torch
    from paper_2501_03061_amd import inputs, px
    cfg = inputs.CONFIGS["large96"]
    inst, psi64, phi64, occ = build_inputs(cfg)
    n = inst.n_orb
    cell = px.Cell(inst.L, inst.n)
    ctx = px.Context(0)
    kern = ctx.px_kernel_hse(cell, cfg["mu"])
    pairs = n * n
    res = {}
    steps = {}
    for name, fp32 in (("fp32", True), ("fp64", False)):
        st = Step(ctx, cell, psi64, phi64, occ, kern, fp32=fp32)
        st()
        torch.cuda.synchronize()
        ms = 1e3 * run_steps(st, 1)

        def ace_only():
            if fp32:
                ctx.px_convert_c128_to_c64(psi64, st.psi)
            ctx.px_ace_build(cell, st.psi, occ, kern, xi=st.xi, M=st.M, e_x=st.ex, status=st.status)
        ace_s = run_steps(ace_only, 1)
        st()
        torch.cuda.synchronize()
        ctx.px_sync()
        res[name] = dict(ms_per_step=ms, pair_solves_per_s=pairs / (ms * 1e-3), ace_build_s=ace_s)
        log(f"large96 {name}: step {ms:.0f} ms, ACE build {ace_s:.2f} s")
        steps[name] = st
        if not fp32:
            continue
        # keep only what the comparison needs before the FP64 buffers are allocated
        st.psi = st.phi = None
        torch.cuda.empty_cache()
    s32, s64 = steps["fp32"], steps["fp64"]

    def rel(a, b):
        return float(torch.linalg.vector_norm((a.to(torch.complex128) - b).flatten()) /
                     torch.linalg.vector_norm(b.flatten()))
    ex32, ex64 = float(s32.ex.item()), float(s64.ex.item())
    errs = dict(M=rel(s32.M, s64.M), e_x=abs(ex32 - ex64) / abs(ex64), ptim_out=rel(s32.out, s64.out),
                residuals_fp32=[float(x) for x in s32.res.cpu()],
                residuals_fp64=[float(x) for x in s64.res.cpu()])
    rec = {
        "metric": "exchange pair-solves/s + ACE build s, FP32-batched vs FP64 at <=2e-5 err",
        "value": res["fp32"]["pair_solves_per_s"], "unit": "pair-solves/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": res["fp32"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "large96: cubic cell L=27 bohr, 96^3 grid, 1536 complex orbitals, "
                               "Fermi-Dirac kT=0.03 Ha; step = staging + ACE build (2359296 pair "
                               "solves) + 4 PT-IM-style ACE iterations",
                   "grid": [96, 96, 96], "n_orbitals": n, "pairs_per_step": pairs},
        "extra": {"fp32": res["fp32"], "fp64": res["fp64"],
                  "speedup_fp32_vs_fp64": res["fp64"]["ms_per_step"] / res["fp32"]["ms_per_step"],
                  "e_x_fp64": ex64, "err_fp32_vs_fp64": errs},
    }
    ctx.close()
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--workload", default="mid72", choices=["mid72", "batch48", "large96"],
                    help="mid72 (default, the headline): one 72^3 x 512 instance; batch48: the "
                         "48-instance uneven batch in the batched form; large96: the 96^3 x 1536 "
                         "single-GPU share, one step per form (several minutes)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the plain copy kernel (2 GiB, 5 launches) and print its bandwidth")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the exchange shards by orbital columns; see the design notes). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2501_03061_amd import inputs, px

    if args.calibrate_copy:
        ctx = px.Context(0)
        print(json.dumps(copy_bandwidth(ctx, reps=5)), flush=True)
        return
    if args.workload == "batch48":
        print(json.dumps(bench_batch48(args)), flush=True)
        return
    if args.workload == "large96":
        print(json.dumps(bench_large96(args)), flush=True)
        return

    cfg = inputs.CONFIGS["mid72"]
    inst, psi64, phi64, occ = build_inputs(cfg)
    n = inst.n_orb
    cell = px.Cell(inst.L, inst.n)
    ctx = px.Context(0)
    kern = ctx.px_kernel_hse(cell, cfg["mu"])

    copy = copy_bandwidth(ctx)
    log(f"copy kernel: {copy['copy_GBps']:.0f} GB/s")
    step32 = Step(ctx, cell, psi64, phi64, occ, kern, fp32=True)
    for _ in range(args.warmup):
        step32()
    torch.cuda.synchronize()
    ctx.px_sync()
    ctx.px_profile_read(reset=True)
    ctx.px_profile_read_ace(reset=True)
    ctx.px_set_profiling(True)
    ms_step = 1e3 * run_steps(step32, args.steps)
    ctx.px_set_profiling(False)
    prof = ctx.px_profile_read(reset=True)
    ace_prof = ctx.px_profile_read_ace(reset=True)
    ctx.px_sync()
    pairs = n * n
    value = pairs / (ms_step * 1e-3)
    log(f"fp32 step {ms_step:.1f} ms -> {value:.4g} pair-solves/s")

    # ACE build alone (FP32 form including staging), for the second half of the metric
    def ace_only():
        ctx.px_convert_c128_to_c64(psi64, step32.psi)
        ctx.px_ace_build(cell, step32.psi, occ, kern, xi=step32.xi, M=step32.M, e_x=step32.ex,
                         status=step32.status)
    ace_s32 = run_steps(ace_only, 1)

    # pipeline roofline: dominant pass of the pair pipeline
    names = ["pass1_fwd_xy", "pass2_z_kernel", "pass3_inv_xy_acc", "pass4_transpose_acc"]
    dom = max(range(4), key=lambda k: prof[k]["ms"])
    pd = prof[dom]
    achieved = pd["bytes"] / (pd["ms"] * 1e-3) / 1e9
    pipe_ms = sum(p["ms"] for p in prof)
    pipe_gbps = sum(p["bytes"] for p in prof) / (pipe_ms * 1e-3) / 1e9

    extra = dict(
        copy_kernel_GBps=copy["copy_GBps"],
        ace_build_s_fp32=ace_s32,
        pair_pipeline_ms_per_step=pipe_ms / args.steps,
        pair_pipeline_model_GBps=pipe_gbps,
        passes={names[k]: dict(avg_us=1e3 * prof[k]["ms"] / max(1, prof[k]["launches"]),
                               launches_per_step=prof[k]["launches"] // args.steps,
                               GBps=prof[k]["bytes"] / (prof[k]["ms"] * 1e-3) / 1e9)
                for k in range(4) if prof[k]["launches"] > 0},
        ace_build_stages_fp32_ms=ace_stages(prof, ace_prof),
        e_x_fp32=float(step32.ex.item()),
        residuals_fp32=[float(x) for x in step32.res.cpu()],
    )

    if not args.no_fp64:
        step64 = Step(ctx, cell, psi64, phi64, occ, kern, fp32=False)
        step64()
        torch.cuda.synchronize()
        ms64 = 1e3 * run_steps(step64, args.fp64_steps)
        ace_s64 = run_steps(lambda: ctx.px_ace_build(cell, psi64, occ, kern, xi=step64.xi, M=step64.M,
                                                     e_x=step64.ex, status=step64.status), 1)
        ctx.px_sync()
        # stage breakdown of one more (profiled) FP64 build
        ctx.px_profile_read(reset=True)
        ctx.px_profile_read_ace(reset=True)
        ctx.px_set_profiling(True)
        ctx.px_ace_build(cell, psi64, occ, kern, xi=step64.xi, M=step64.M, e_x=step64.ex,
                         status=step64.status)
        ctx.px_set_profiling(False)
        stages64 = ace_stages(ctx.px_profile_read(reset=True), ctx.px_profile_read_ace(reset=True))
        step32()
        torch.cuda.synchronize()
        ctx.px_sync()

        def rel(a, b):
            return float(torch.linalg.vector_norm((a.to(torch.complex128) - b).flatten()) /
                         torch.linalg.vector_norm(b.flatten()))
        ex64, ex32 = float(step64.ex.item()), float(step32.ex.item())
        extra.update(
            fp64_pair_solves_per_s=pairs / (ms64 * 1e-3),
            fp64_ms_per_step=ms64,
            ace_build_s_fp64=ace_s64,
            ace_build_stages_fp64_ms=stages64,
            speedup_fp32_vs_fp64=(pairs / (ms_step * 1e-3)) / (pairs / (ms64 * 1e-3)),
            err_fp32_vs_fp64=dict(M=rel(step32.M, step64.M), e_x=abs(ex32 - ex64) / abs(ex64),
                                  xi=rel(step32.xi, step64.xi),
                                  ptim_out=rel(step32.out, step64.out),
                                  residuals=[float(a) for a in step64.res.cpu()]),
        )
        log(f"fp64 step {ms64:.1f} ms; errors {extra['err_fp32_vs_fp64']}")
        del step64

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(inst, kern.cpu().numpy(), args.cpu_seconds)
        log(f"cpu oracle: {cpu['value']:.4g} pair-solves/s on {cpu['cores']} threads")

    rec = {
        "metric": "exchange pair-solves/s + ACE build s, FP32-batched vs FP64 at <=2e-5 err",
        "value": value,
        "unit": "pair-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "mid72: cubic cell L=20 bohr, 72^3 grid, 512 complex orbitals (10 Ha sphere, "
                        "QR-orthonormalised), Fermi-Dirac kT=0.02 Ha, HSE mu=0.106; FP32 bulk with FP64 "
                        "G=0/energy/reductions/Cholesky; step = staging + ACE build (262144 pair solves) "
                        "+ 4 PT-IM-style ACE iterations",
            "grid": [72, 72, 72], "n_orbitals": n, "pairs_per_step": pairs,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": measured_traffic(names[dom]),
            "kernel": names[dom],
            "per_unit_bytes": pd["bytes"] / max(1, pd["launches"]),
            "unit_desc": "algorithmic bytes per launch: 2*N_g*8 B per pair of the launch's chunk "
                         "(its share of the 6*N_g*b pair model), plus N_g*8 B per pair for the kept "
                         "v_ij when pass 3 runs an off-diagonal block of the Hermitian-pair mode",
        },
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(rec), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
