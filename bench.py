#!/usr/bin/env python
"""Throughput of the exchange / ACE hot path on one MI355X.

One step is one pass of the whole path over the resident synthetic instance:
  staging of Psi to complex64 (FP32 form),
  ACE build: W = Vx Psi through the fused pair pipeline (N^2 logical pair
    solves, N(N+1)/2 physical ones in the Hermitian-pair mode),
    M = dV Psi^H W, Hermitisation, FP64 Cholesky of -M, U = L^-H, xi = W U,
  staging of Phi_n = Psi + 1e-3 Z to complex64 (FP32 form),
  4 PT-IM-style fixed-point iterations with the ACE operator and FP64 residuals.
The headline value is logical pair solves per second of whole steps on the
large single-GPU share (96^3 grid, 1536 orbitals).  The plain FP64 form of the
same step is timed after the headline run for the precision/speed comparison,
and the CPU oracle is timed on a bounded sample of the same instance.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
                    [--workload large96|mid72|batch48|mixed72|mixed96]

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "exchange pair-solves/s + ACE build s, FP32-batched vs FP64 at <=2e-5 err"
PASS_NAMES = ["pass1_fwd_xy", "pass2_z_kernel", "pass3_inv_xy_acc", "pass4_transpose_acc"]
# Time step 50 as in atomic units of time times the hybrid mixing fraction 0.25.
DT_ALPHA = 50.0 / 24.188843265857 * 0.25

WORKLOAD_TEXT = {
    "large96": "large96: cubic cell L=27 bohr, 96^3 grid, 1536 complex orbitals (10 Ha sphere, "
               "QR-orthonormalised), Fermi-Dirac kT=0.03 Ha, HSE mu=0.106; FP32 bulk with FP64 "
               "G=0/energy/reductions/Cholesky; step = staging + ACE build (2359296 logical pair "
               "solves, Hermitian-pair mode) + 4 PT-IM-style ACE iterations on Phi = Psi + 1e-3 Z",
    "mid72": "mid72: cubic cell L=20 bohr, 72^3 grid, 512 complex orbitals (10 Ha sphere, "
             "QR-orthonormalised), Fermi-Dirac kT=0.02 Ha, HSE mu=0.106; FP32 bulk with FP64 "
             "G=0/energy/reductions/Cholesky; step = staging + ACE build (262144 logical pair "
             "solves, Hermitian-pair mode) + 4 PT-IM-style ACE iterations on Phi = Psi + 1e-3 Z",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def build_inputs(cfg):
    import numpy as np
    import torch
    from paper_2501_03061_amd import inputs
    t0 = time.perf_counter()
    inst = inputs.make_instance(cfg["n"], cfg["L"], cfg["n_orb"], cfg["kT"], seed=cfg["seed"])
    psi_d = torch.from_numpy(inst.psi).cuda()
    z = inputs.noise_block(inst.n, inst.L, inst.n_orb, seed=1001)
    z *= 1e-3
    z += inst.psi
    phi_d = torch.from_numpy(z).cuda()
    del z
    occ_d = torch.from_numpy(inst.occ).cuda()
    log(f"inputs generated in {time.perf_counter() - t0:.1f}s "
        f"(occupations 0.1<f<0.9: {float(np.mean((inst.occ > 0.1) & (inst.occ < 0.9))):.3f}, "
        f"0.01<f<0.99: {float(np.mean((inst.occ > 0.01) & (inst.occ < 0.99))):.3f})")
    return inst, psi_d, phi_d, occ_d


class Step:
    """One pass of the hot path in one precision form, buffers preallocated.
    With events, a CUDA event pair brackets the staging of Psi plus the ACE
    build (the "ACE build s" half of the metric) on the current stream, which
    is the stream the library's calls are enqueued on."""

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
        self.events = []

    def __call__(self, record=False):
        import torch
        c = self.ctx
        if record:
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record()
        if self.fp32:
            c.px_convert_c128_to_c64(self.psi64, self.psi)
        c.px_ace_build(self.cell, self.psi, self.occ, self.kern, xi=self.xi, M=self.M,
                       e_x=self.ex, status=self.status)
        if record:
            e[1].record()
        if self.fp32:
            c.px_convert_c128_to_c64(self.phi64, self.phi)
        c.px_ptim_exchange_loop(self.cell, self.xi, self.phi, self.n_iter, DT_ALPHA,
                                out=self.out, residuals=self.res)
        if record:
            e[2].record()
            self.events.append(e)

    def event_times(self):
        """Per recorded step: (staging + ACE build ms, whole step ms)."""
        out = [(e[0].elapsed_time(e[1]), e[0].elapsed_time(e[2])) for e in self.events]
        self.events = []
        return out


def run_steps(step, k, record=False):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(k):
        step(record) if record else step()
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
    """The oracle as it stands on a bounded sample of the same instance: whole
    output columns of W = Vx Psi (each column pairs one orbital with all N),
    scipy.fft with all host threads; then the same oracle with one FFT thread
    on a 64-pair piece of one column."""
    import oracle
    import oracle.exchange as oex
    threads = oex._WORKERS
    t0 = time.perf_counter()
    oracle.exchange_apply(inst.psi, inst.occ, inst.psi[:1], kern_np)
    t1 = time.perf_counter() - t0
    more = max(0, min(inst.n_orb - 1, int(seconds / max(t1, 1e-3)) - 1))
    t2 = 0.0
    if more:
        t0 = time.perf_counter()
        oracle.exchange_apply(inst.psi, inst.occ, inst.psi[1:1 + more], kern_np)
        t2 = time.perf_counter() - t0
    pairs = (1 + more) * inst.n_orb
    # one thread: 64 density orbitals against one output orbital
    oex._WORKERS = 1
    try:
        t0 = time.perf_counter()
        oracle.exchange_apply(inst.psi[:64], inst.occ[:64], inst.psi[:1], kern_np)
        t3 = time.perf_counter() - t0
    finally:
        oex._WORKERS = threads
    return dict(value=pairs / (t1 + t2), unit="pair-solves/s", cores=threads, kind="oracle",
                sample=f"{1 + more} output orbital(s) x {inst.n_orb} density orbitals "
                       f"({pairs} pair solves) of the same instance, {t1 + t2:.1f}s, "
                       f"scipy.fft workers={threads}, host CPU: {cpu_model()}",
                one_thread_value=64 / t3, one_thread_sample="64 pair solves (one output orbital "
                f"x 64 density orbitals), scipy.fft workers=1, {t3:.1f}s")


def roofline_fields(prof, ace, steps, pairs_phys, ng, b, copy_gbps):
    """Roofline of the dominant pass (HIP-event durations over the timed
    region) and of the whole pair pipeline, both with the 6*N_g*b model."""
    dom = max(range(4), key=lambda k: prof[k]["ms"])
    pd = prof[dom]
    per_launch = pd["bytes"] / max(1, pd["launches"])
    avg_s = pd["ms"] * 1e-3 / max(1, pd["launches"])
    achieved = per_launch / avg_s / 1e9
    pipe_ms = sum(p["ms"] for p in prof)
    model_bytes = pairs_phys * 6.0 * ng * b * steps
    pipe_gbps = model_bytes / (pipe_ms * 1e-3) / 1e9
    # bytes the Hermitian-pair mode moves beyond the model: the kept v_ij,
    # written by pass 3 and read back by pass 4
    extra_bytes = pairs_phys * ng * b * steps + prof[3]["bytes"]
    passes = {}
    for k in range(4):
        if prof[k]["launches"] == 0:
            continue
        passes[PASS_NAMES[k]] = dict(
            avg_us=1e3 * prof[k]["ms"] / prof[k]["launches"],
            launches_per_step=prof[k]["launches"] // steps,
            ms_per_step=prof[k]["ms"] / steps,
            model_GBps=prof[k]["bytes"] / (prof[k]["ms"] * 1e-3) / 1e9)
    roof = {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBPS, "traffic": None, "kernel": PASS_NAMES[dom],
        "per_unit_bytes": per_launch,
        "unit_desc": "algorithmic bytes per launch of the dominant pass: 2*N_g*b per pair "
                     "solved in the launch (its share of the 6*N_g*b pair model), b = 8 B "
                     "(complex64); the kept v_ij of the Hermitian-pair mode is not counted",
    }
    pipeline = dict(ms_per_step=pipe_ms / steps, model_GBps=pipe_gbps,
                    model_frac=pipe_gbps / HBM_PEAK_GBPS,
                    model_plus_kept_v_GBps=(model_bytes + extra_bytes) / (pipe_ms * 1e-3) / 1e9,
                    copy_kernel_GBps=copy_gbps,
                    desc="physical pair solves x 6*N_g*b over the summed pass times of the "
                         "pair pipeline; model_plus_kept_v adds the v_ij that the Hermitian-pair "
                         "mode writes in pass 3 and reads in pass 4")
    stages = dict(pair_pipeline_ms=pipe_ms / max(1, ace["calls"]),
                  M_contraction_ms=ace["M"] / max(1, ace["calls"]),
                  factorization_ms=ace["factor"] / max(1, ace["calls"]),
                  xi_contraction_ms=ace["xi"] / max(1, ace["calls"]),
                  build_ms=ace["build"] / max(1, ace["calls"]), builds=ace["calls"])
    return dom, roof, pipeline, passes, stages


def bench_single(args, workload):
    import torch
    from paper_2501_03061_amd import inputs, px
    import profsum
    cfg = inputs.CONFIGS[workload]
    inst, psi64, phi64, occ = build_inputs(cfg)
    n = inst.n_orb
    cell = px.Cell(inst.L, inst.n)
    ng = cell.ng
    ctx = px.Context(0)
    kern = ctx.px_kernel_hse(cell, cfg["mu"])
    pairs = n * n
    pairs_phys = n * (n + 1) // 2

    copy = copy_bandwidth(ctx)
    log(f"copy kernel: {copy['copy_GBps']:.0f} GB/s")
    step32 = Step(ctx, cell, psi64, phi64, occ, kern, fp32=True)
    for k in range(args.warmup):
        step32()
        log(f"warmup step {k + 1}/{args.warmup}")
    torch.cuda.synchronize()
    ctx.px_sync()
    ctx.px_profile_read(reset=True)
    ctx.px_profile_read_ace(reset=True)
    ctx.px_set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step32(True)
        if args.steps > 3:
            log(f"timed step {k + 1}/{args.steps}")
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.perf_counter() - t0) / args.steps
    ctx.px_set_profiling(False)
    prof = ctx.px_profile_read(reset=True)
    ace = ctx.px_profile_read_ace(reset=True)
    ctx.px_sync()
    ev32 = step32.event_times()
    value = pairs / (ms_step * 1e-3)
    log(f"fp32 step {ms_step:.1f} ms -> {value:.4g} pair-solves/s")
    dom, roof, pipeline, passes, stages = roofline_fields(prof, ace, args.steps, pairs_phys, ng, 8,
                                                          copy["copy_GBps"])
    roof["traffic"] = profsum.measured_traffic(workload, PASS_NAMES[dom])
    if roof["traffic"] is not None:
        # the same launch priced by its counter-measured HBM bytes
        avg_s = prof[dom]["ms"] * 1e-3 / max(1, prof[dom]["launches"])
        roof["measured_GBps"] = roof["traffic"] / avg_s / 1e9
        roof["measured_frac"] = roof["measured_GBps"] / HBM_PEAK_GBPS
    ace_s = [a * 1e-3 for a, _ in ev32]
    extra = dict(
        logical_pair_solves_per_step=pairs, physical_pair_solves_per_step=pairs_phys,
        physical_pair_solves_per_s=pairs_phys / (ms_step * 1e-3),
        ace_build_s_fp32=statistics.median(ace_s), ace_build_s_fp32_all=ace_s,
        step_ms_median=statistics.median(s for _, s in ev32),
        pair_pipeline=pipeline, passes=passes, ace_build_stages_fp32=stages,
        e_x_fp32=float(step32.ex.item()), residuals_fp32=[float(x) for x in step32.res.cpu()],
        gpu=torch.cuda.get_device_name(0),
    )

    if not args.no_fp64:
        step64 = Step(ctx, cell, psi64, phi64, occ, kern, fp32=False)
        step64()
        torch.cuda.synchronize()
        log("fp64 warmup step done")
        ms64 = 1e3 * run_steps(step64, args.fp64_steps, record=True)
        ctx.px_sync()
        ev64 = step64.event_times()
        ace64 = [a * 1e-3 for a, _ in ev64]

        def rel(a, b):
            return float(torch.linalg.vector_norm((a.to(torch.complex128) - b).flatten()) /
                         torch.linalg.vector_norm(b.flatten()))
        ex64, ex32 = float(step64.ex.item()), float(step32.ex.item())
        errs = dict(M=rel(step32.M, step64.M), e_x=abs(ex32 - ex64) / abs(ex64),
                    xi=rel(step32.xi, step64.xi), ptim_out=rel(step32.out, step64.out),
                    residuals_fp64=[float(a) for a in step64.res.cpu()])
        extra.update(
            fp64_pair_solves_per_s=pairs / (ms64 * 1e-3),
            fp64_physical_pair_solves_per_s=pairs_phys / (ms64 * 1e-3),
            fp64_ms_per_step=ms64, fp64_steps=args.fp64_steps,
            fp64_step_ms_all=[s for _, s in ev64],
            ace_build_s_fp64=statistics.median(ace64),
            speedup_fp32_vs_fp64=ms64 / ms_step,
            speedup_fp32_vs_fp64_ace_build=statistics.median(ace64) / statistics.median(ace_s),
            err_fp32_vs_fp64=errs, e_x_fp64=ex64,
        )
        log(f"fp64 step {ms64:.1f} ms; errors {errs}")
        step64 = None
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(inst, kern.cpu().numpy(), args.cpu_seconds)
        log(f"cpu oracle: {cpu['value']:.4g} pair-solves/s on {cpu['cores']} threads "
            f"({cpu['one_thread_value']:.3g} on one)")

    rec = {
        "metric": METRIC, "value": value, "unit": "pair-solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[workload], "grid": list(inst.n), "n_orbitals": n,
                   "pairs_per_step": pairs},
        "roofline": roof, "cpu_baseline": cpu, "extra": extra,
    }
    ctx.close()
    return rec


class MixedStep:
    """Exchange-only finite-temperature PT-IM time steps with a full occupation
    matrix, in one precision form, buffers preallocated.  The state is
    (Phi, sigma) with the diagonal form (phi = Phi Q, d) of sigma = Q D Q^H;
    one step is
      the ACE build of Vx[Phi sigma Phi^H] on (phi, d) (pair pipeline, M,
        Cholesky, xi),
      the PT-IM step (Eq. 4-7 with the projector and the sigma commutator,
        n_iter fixed-point iterations, FP64 residuals) -> (Phi', sigma'),
      the diagonalisation of sigma' (FP64 blocked Jacobi) and phi' = Phi' Q',
      the density of the new state, sum_i d'_i |phi'_i|^2, on the wavefunction
        grid and on the twice-finer charge-density grid,
    so that one diagonalisation per step serves both the density of the new
    state and the exchange operator of the next step.  Each call advances the
    state by one step.  Events on the current stream (the library's stream)
    bracket the stages."""

    def __init__(self, ctx, cell, phi64, sigma, kern, fp32, n_iter=4):
        import torch
        from paper_2501_03061_amd import px
        self.ctx, self.cell, self.fp32, self.n_iter, self.kern = ctx, cell, fp32, n_iter, kern
        dt = torch.complex64 if fp32 else torch.complex128
        n = phi64.shape[0]
        dev = phi64.device
        mk = lambda: torch.empty(phi64.shape, dtype=dt, device=dev)  # noqa: E731
        self.phi = [mk(), mk()]          # Phi of the current and the next state
        self.rot = [mk(), mk()]          # phi = Phi Q of the current and the next state
        self.xi = mk()
        self.sigma = [sigma.clone(), torch.empty_like(sigma)]
        self.Q = torch.empty_like(sigma)
        self.d = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(2)]
        self.res = torch.zeros((2, n_iter), dtype=torch.float64, device=dev)
        self.ex = torch.zeros(1, dtype=torch.float64, device=dev)
        self.st_ace = torch.zeros(1, dtype=torch.int32, device=dev)
        self.st_step = torch.zeros(1, dtype=torch.int32, device=dev)
        self.st_eig = torch.zeros(1, dtype=torch.int32, device=dev)
        self.rho = torch.empty((cell.n[2], cell.n[1], cell.n[0]), dtype=torch.float64, device=dev)
        self.rho_f = torch.empty((2 * cell.n[2], 2 * cell.n[1], 2 * cell.n[0]), dtype=torch.float64,
                                 device=dev)
        prec = px.PX_PREC_FP32 if fp32 else px.PX_PREC_FP64
        need = max(ctx.workspace_bytes(px.PX_OP_ACE_BUILD, cell, prec, n),
                   ctx.workspace_bytes(px.PX_OP_PTIM_STEP, cell, prec, n, n),
                   ctx.workspace_bytes(px.PX_OP_SIGMA_DIAG, cell, prec, n),
                   ctx.workspace_bytes(px.PX_OP_ROTATE, cell, prec, n),
                   ctx.workspace_bytes(px.PX_OP_DENSITY_FINE, cell, prec, n))
        ctx.ensure_workspace(need)
        self.cur = 0
        # the diagonal form of the initial state (outside the steps)
        if fp32:
            ctx.px_convert_c128_to_c64(phi64, self.phi[0])
        else:
            self.phi[0].copy_(phi64)
        ctx.px_sigma_diagonalize(self.sigma[0], Q=self.Q, d=self.d[0], status=self.st_eig)
        ctx.px_rotate_orbitals(cell, self.phi[0], self.Q, out=self.rot[0])
        self.events = []

    def __call__(self, record=False):
        import torch
        c, a, b = self.ctx, self.cur, 1 - self.cur
        if record:
            e = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
            e[0].record()
        c.px_ace_build(self.cell, self.rot[a], self.d[a], self.kern, xi=self.xi, e_x=self.ex,
                       status=self.st_ace)
        if record:
            e[1].record()
        c.px_ptim_step(self.cell, self.xi, self.phi[a], self.sigma[a], self.n_iter, DT_ALPHA,
                       phi_out=self.phi[b], sigma_out=self.sigma[b], residuals=self.res,
                       status=self.st_step)
        if record:
            e[2].record()
        c.px_sigma_diagonalize(self.sigma[b], Q=self.Q, d=self.d[b], status=self.st_eig)
        if record:
            e[3].record()
        c.px_rotate_orbitals(self.cell, self.phi[b], self.Q, out=self.rot[b])
        if record:
            e[4].record()
        c.px_density(self.cell, self.rot[b], self.d[b], rho=self.rho)
        if record:
            e[5].record()
        c.px_density_fine(self.cell, self.rot[b], self.d[b], rho=self.rho_f)
        if record:
            e[6].record()
            self.events.append(e)
        self.cur = b

    STAGES = ("ace_build", "ptim_step", "sigma_diagonalize", "rotation", "density", "density_fine")

    def stage_times(self):
        """Per recorded step: ms of each stage in STAGES."""
        out = [[e[k].elapsed_time(e[k + 1]) for k in range(len(self.STAGES))] for e in self.events]
        self.events = []
        return out

    def status(self):
        return [int(self.st_ace.item()), int(self.st_step.item()), int(self.st_eig.item())]


def time_call(fn, reps=3):
    """Median ms of fn() over reps calls, each bracketed by events on the current stream."""
    import torch
    fn()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return statistics.median(ts)


MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}


def bench_mixed(args, workload):
    """The rows after the exchange/ACE path (the occupation-matrix front end,
    the PT-IM step with the projector, the density) in exchange-only
    finite-temperature time steps on the resident instance of the same size as
    the single-instance workloads, FP32 form; stage rooflines from the event
    timings of each stage inside the timed steps."""
    import numpy as np
    import torch
    from paper_2501_03061_amd import inputs, px
    cfg = inputs.CONFIGS[MIXED_BASE[workload]]
    inst, psi64, phi64, occ = build_inputs(cfg)
    del psi64
    n = inst.n_orb
    sigma_h = inputs.occupation_matrix(inst.occ, seed=cfg["seed"] + 7)
    sigma = torch.from_numpy(sigma_h).cuda()
    cell = px.Cell(inst.L, inst.n)
    ng = cell.ng
    ctx = px.Context(0)
    kern = ctx.px_kernel_hse(cell, cfg["mu"])
    step = MixedStep(ctx, cell, phi64, sigma, kern, fp32=True)
    if args.no_fp64:
        del phi64
        torch.cuda.empty_cache()
    for k in range(max(1, args.warmup)):
        step()
        log(f"mixed warmup step {k + 1}")
    torch.cuda.synchronize()
    ctx.px_sync()
    ctx.px_profile_read(reset=True)
    ctx.px_profile_read_ace(reset=True)
    ctx.px_set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(True)
        log(f"mixed timed step {k + 1}/{args.steps}")
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.perf_counter() - t0) / args.steps
    ctx.px_set_profiling(False)
    prof = ctx.px_profile_read(reset=True)
    ace = ctx.px_profile_read_ace(reset=True)
    ctx.px_sync()
    stages = step.stage_times()
    med = {name: statistics.median(s[k] for s in stages) for k, name in enumerate(MixedStep.STAGES)}
    pairs = n * n
    pairs_phys = n * (n + 1) // 2
    dom, roof, pipeline, passes, ace_stages = roofline_fields(prof, ace, args.steps, pairs_phys, ng, 8, 0.0)
    pipeline.pop("copy_kernel_GBps", None)
    peak = MFMA_PEAK_TFLOPS["f32"]
    rot_flops = 8.0 * n * n * ng
    # per PT-IM iteration: C = dV xi^H mid and Y = -xi C (8 n^2 N_g each), S on
    # its upper tiles (about 4 n^2 N_g), Z = -mid X (8 n^2 N_g)
    it_flops = 28.0 * n * n * ng
    dens_bytes = n * ng * 8 + ng * 8
    fine_flops = 4.0 * n * ng * (cell.n[0] + 2 * cell.n[1] + 4 * cell.n[2])
    fine_bytes = 25.0 * n * ng * 8 + 2.0 * 8 * ng * 8 * ((n + 15) // 16)

    def mfma(ms, flops, desc):
        return dict(ms=ms, bound="mfma", flops=flops, TFLOPs=flops / (ms * 1e-3) / 1e12, peak_TFLOPs=peak,
                    frac=flops / (ms * 1e-3) / 1e12 / peak, desc=desc)
    stage_roof = {
        "ace_build": dict(ms=med["ace_build"], stages=ace_stages,
                          desc="ACE build on (phi, d): pair pipeline, M, Cholesky, xi"),
        "ptim_step": dict(mfma(med["ptim_step"], it_flops * step.n_iter,
                               "per iteration 28 n^2 N_g flops (xi^H mid, xi C, S on its upper tiles, "
                               "mid X) on FP32 MFMA; Hm = -C^H C and the sigma algebra in FP64"),
                          iterations=step.n_iter),
        "sigma_diagonalize": dict(ms=med["sigma_diagonalize"], bound="latency",
                                  desc=f"FP64 blocked cyclic Jacobi, {n} x {n}: per sweep "
                                       f"{2 * ((n + 15) // 16 + ((n + 15) // 16) % 2) - 2} small launches"),
        "rotation": mfma(med["rotation"], rot_flops, "phi = Phi Q, 8 n^2 N_g flops, FP32 MFMA"),
        "density": dict(ms=med["density"], bound="hbm", bytes=dens_bytes,
                        GBps=dens_bytes / (med["density"] * 1e-3) / 1e9,
                        frac=dens_bytes / (med["density"] * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                        desc="sum_i d_i |phi_i|^2: n N_g b read + 8 N_g written (FP64)"),
        "density_fine": dict(ms=med["density_fine"], bound="alu", flops=fine_flops, bytes=fine_bytes,
                             TFLOPs=fine_flops / (med["density_fine"] * 1e-3) / 1e12, peak_TFLOPs=157.3,
                             frac=fine_flops / (med["density_fine"] * 1e-3) / 1e12 / 157.3,
                             GBps=fine_bytes / (med["density_fine"] * 1e-3) / 1e9,
                             hbm_frac=fine_bytes / (med["density_fine"] * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                             desc="orbitals interpolated axis by axis to the 2x grid: the odd fine points of "
                                  "each axis n MACs each, 4 flops (n0 + 2 n1 + 4 n2) N_g per orbital (x and y "
                                  "on the FP32 vector units, z on the matrix cores); 25 N_g b of traffic per "
                                  "orbital; squares summed in FP64; peak is the chip's FP32 vector rate"),
    }
    res = step.res.cpu().numpy()
    a = step.cur
    sig_now = step.sigma[a].cpu().numpy()
    rot_plane = step.rot[a][:, :1].to(torch.complex128).cpu().numpy()   # for the CPU sample
    d_now = step.d[a].cpu().numpy()
    rho_int = float(step.rho.sum().item()) * cell.dV
    checks = dict(trace_sigma_0=float(np.trace(sigma_h).real), trace_sigma_now=float(np.trace(sig_now).real),
                  hermitian_defect_sigma_now=float(np.abs(sig_now - sig_now.conj().T).max()),
                  integral_rho=rho_int, e_x=float(step.ex.item()),
                  residuals_phi_last_step=[float(x) for x in res[0]],
                  residuals_sigma_last_step=[float(x) for x in res[1]], status=step.status(),
                  steps_taken=max(1, args.warmup) + args.steps)
    log(f"mixed step {ms_step:.1f} ms: stages {[round(med[k], 2) for k in MixedStep.STAGES]} ms; "
        f"checks {checks}")
    fp64 = None
    if not args.no_fp64:
        # the plain FP64 form from the same initial state over the same number of
        # steps: its speed, and the FP32 form's deviation from it per result
        taken = checks["steps_taken"]
        keep = dict(phi=step.phi[a].clone(), sigma=step.sigma[a].clone(), rho=step.rho.clone(),
                    rho_fine=step.rho_f.clone(), e_x=float(step.ex.item()))
        step = None
        torch.cuda.empty_cache()
        step64 = MixedStep(ctx, cell, phi64, sigma, kern, fp32=False)
        del phi64
        torch.cuda.empty_cache()
        n_timed = max(1, min(args.fp64_steps, taken - 1))
        for k in range(taken - n_timed):
            step64()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(n_timed):
            step64(True)
        torch.cuda.synchronize()
        ms64 = 1e3 * (time.perf_counter() - t1) / n_timed
        st64 = step64.stage_times()
        med64 = {name: statistics.median(s[k] for s in st64) for k, name in enumerate(MixedStep.STAGES)}
        b = step64.cur

        def rel(x, y):
            return float(torch.linalg.vector_norm((x.to(y.dtype) - y).flatten()) /
                         torch.linalg.vector_norm(y.flatten()))
        ex64 = float(step64.ex.item())
        fp64 = dict(ms_per_step=ms64, steps_timed=n_timed, stage_ms_median=med64,
                    speedup_fp32_vs_fp64=ms64 / ms_step,
                    stage_speedup={k: med64[k] / med[k] for k in MixedStep.STAGES},
                    err_fp32_vs_fp64=dict(phi=rel(keep["phi"], step64.phi[b]),
                                          sigma=rel(keep["sigma"], step64.sigma[b]),
                                          rho=rel(keep["rho"], step64.rho),
                                          rho_fine=rel(keep["rho_fine"], step64.rho_f),
                                          e_x=abs(keep["e_x"] - ex64) / abs(ex64)),
                    desc=f"both forms advanced {taken} steps from the same state; errors of the "
                         "FP32 state after them relative to the FP64 one")
        log(f"mixed fp64 step {ms64:.1f} ms; FP32 vs FP64 {fp64['err_fp32_vs_fp64']}")
        step64 = None
        torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(inst, kern.cpu().numpy(), args.cpu_seconds)
        import oracle
        t1 = time.perf_counter()
        oracle.sigma_eig(sig_now)
        t_eig = time.perf_counter() - t1
        rot_h = rot_plane
        t1 = time.perf_counter()
        oracle.density(rot_h, d_now)
        t_rho = (time.perf_counter() - t1) * inst.n[2]
        cpu["stage_samples"] = dict(sigma_eig_s=t_eig, density_s_scaled=t_rho,
                                    desc="oracle sigma_eig (LAPACK) at full n; oracle density on one "
                                         "z-plane, times the number of planes")
    rec = {
        "metric": METRIC, "value": pairs / (ms_step * 1e-3), "unit": "pair-solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": MIXED_TEXT[workload], "grid": list(inst.n), "n_orbitals": n,
                   "pairs_per_step": pairs},
        "roofline": roof, "cpu_baseline": cpu,
        "extra": {"stage_ms_median": med, "stages": stage_roof, "pair_pipeline": pipeline, "passes": passes,
                  "physical_pair_solves_per_s": pairs_phys / (ms_step * 1e-3), "checks": checks,
                  "fp64": fp64, "gpu": torch.cuda.get_device_name(0)},
    }
    ctx.close()
    return rec


MIXED_BASE = {"mixed72": "mid72", "mixed96": "large96"}
MIXED_TEXT = {
    k: f"{k}: the {v} instance (Phi_0 = Psi + 1e-3 Z) with a full occupation matrix sigma_0 = "
       "V diag(f) V^H (V unitary, I + 0.1 noise), advanced by exchange-only PT-IM time steps; "
       "step = ACE build of Vx[sigma] on the diagonal form (phi = Phi Q, d) + PT-IM step with "
       "projector and sigma commutator (4 iterations) + diagonalisation of the new sigma (FP64 "
       "Jacobi) + phi' = Phi' Q' + density of the new state on the wavefunction grid and on the "
       "twice-finer charge-density grid; FP32 bulk"
    for k, v in MIXED_BASE.items()}


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
        "metric": METRIC, "value": pairs / (ms_b * 1e-3), "unit": "pair-solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_b, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch48: 48 instances, grids {32,40,48,64}^3, 32..256 orbitals, "
                               "kT 0.005..0.05 Ha, L = 0.28 n bohr; FP32 ACE builds, batched + graph",
                   "pairs_per_step": pairs},
        "extra": {"autotuned_blocks": blocks, "single_fp32_ms": ms_1, "single_fp64_ms": ms_64,
                  "single_fp32_pair_solves_per_s": pairs / (ms_1 * 1e-3),
                  "single_fp64_pair_solves_per_s": pairs / (ms_64 * 1e-3),
                  "speedup_batched_fp32_vs_single_fp32": ms_1 / ms_b,
                  "speedup_batched_fp32_vs_single_fp64": ms_64 / ms_b},
    }
    ctx.close()
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--workload", default="large96",
                    choices=["large96", "mid72", "batch48", "mixed72", "mixed96"],
                    help="large96 (default, the headline): the 96^3 x 1536 single-GPU share; "
                         "mid72: one 72^3 x 512 instance; batch48: the 48-instance uneven batch "
                         "in the batched form; mixed72 / mixed96: a finite-temperature step with "
                         "a full occupation matrix (sigma front end, PT-IM step, density)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the plain copy kernel (2 GiB, 5 launches) and print its bandwidth")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the exchange "
              "would shard by orbital columns, with a ring of orbital blocks). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    from paper_2501_03061_amd import px

    if args.calibrate_copy:
        ctx = px.Context(0)
        print(json.dumps(copy_bandwidth(ctx, reps=5)), flush=True)
        return
    if args.workload == "batch48":
        print(json.dumps(bench_batch48(args)), flush=True)
        return
    if args.workload in MIXED_BASE:
        print(json.dumps(bench_mixed(args, args.workload)), flush=True)
        return
    print(json.dumps(bench_single(args, args.workload)), flush=True)


if __name__ == "__main__":
    main()
