"""Batched form: many uneven instances in one call (task-table launches,
Hermitian-pair block schedule, HIP graph replay) and the autotuner."""
import os

import numpy as np
import pytest

import oracle
from paper_2501_03061_amd import inputs, px
from _gpu import banner, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

FP64_TOL, FP32_TOL, FP32_EX_TOL = 1e-11, 2e-5, 1e-7


def _make(specs, fp32, ctx):
    import torch
    out = []
    for (n, n_orb, kT, seed) in specs:
        L = 0.28 * n
        inst = inputs.make_instance(n, L, n_orb, kT, seed=seed)
        cell = px.Cell(inst.L, inst.n)
        psi = to_dev(inst.psi)
        if fp32:
            psi = ctx.px_convert_c128_to_c64(psi)
        out.append(dict(inst=inst, cell=cell, psi=psi, occ=to_dev(inst.occ),
                        kern=ctx.px_kernel_hse(cell, 0.106),
                        e_x=torch.zeros(1, dtype=torch.float64, device="cuda")))
    return out


SPECS = [(16, 11, 0.02, 1), (24, 37, 0.01, 2), (16, 5, 0.05, 3), (32, 20, 0.03, 4),
         (24, 16, 0.02, 5), (32, 45, 0.005, 6)]


@pytest.mark.parametrize("fp32", [False, True])
def test_batched_exchange_matches_oracle(px_ctx, fp32):
    banner(f"batched exchange fp32={fp32}")
    import torch
    insts = _make(SPECS, fp32, px_ctx)
    prec = px.PX_PREC_FP32 if fp32 else px.PX_PREC_FP64
    for d in insts:                       # small blocks: several diagonals per instance
        px_ctx.set_tuning(d["cell"], prec, 8, 8)
    try:
        outs, _ = px_ctx.px_exchange_apply_batched(
            [dict(cell=d["cell"], psi=d["psi"], occ=d["occ"], kern=d["kern"], e_x=d["e_x"]) for d in insts])
        torch.cuda.synchronize()
    finally:
        for d in insts:
            px_ctx.set_tuning(d["cell"], prec, 0, 0)
    for d, out in zip(insts, outs):
        inst = d["inst"]
        K = oracle.kernel_hse(inst.n, inst.L, 0.106)
        ref = oracle.exchange_apply(inst.psi, inst.occ, inst.psi, K)
        ex = oracle.exchange_energy_gspace(inst.psi, inst.occ, K, inst.omega)
        err, eerr = relerr(to_host(out), ref), abs(float(d["e_x"].item()) - ex) / abs(ex)
        print(f"n={inst.n[0]} N={inst.n_orb}: vx {err:.2e} e_x {eerr:.2e}")
        assert err < (FP32_TOL if fp32 else FP64_TOL)
        assert eerr < (FP32_EX_TOL if fp32 else FP64_TOL)


def test_batched_graph_replay_is_deterministic(px_ctx):
    """Replays of the cached graph, with eager work in between, give bitwise
    the same result as the first launch and as direct (uncaptured) enqueue."""
    banner("batched graph replay")
    import torch
    insts = _make(SPECS[:4], True, px_ctx)
    args = [dict(cell=d["cell"], psi=d["psi"], occ=d["occ"], kern=d["kern"], e_x=d["e_x"]) for d in insts]
    outs = [torch.empty_like(d["psi"]) for d in insts]
    for a, o in zip(args, outs):
        a["out"] = o
    px_ctx.px_exchange_apply_batched(args)
    torch.cuda.synchronize()
    first = [o.clone() for o in outs]
    ex0 = [float(d["e_x"].item()) for d in insts]
    for rep in range(3):
        for o in outs:
            o.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()      # eager work between replays
        px_ctx.px_exchange_apply_batched(args)
        torch.cuda.synchronize()
        del junk
        for a, b in zip(outs, first):
            assert torch.equal(a, b), f"replay {rep} differs"
        assert [float(d["e_x"].item()) for d in insts] == ex0
    px_ctx.px_set_graph(False)
    try:
        for o in outs:
            o.zero_()
        px_ctx.px_exchange_apply_batched(args)
        torch.cuda.synchronize()
    finally:
        px_ctx.px_set_graph(True)
    for a, b in zip(outs, first):
        assert torch.equal(a, b)


def test_batched_ace_replays_bitwise(px_ctx):
    """ACE mode with the tails on the side streams: graph replays (eager work
    in between) and direct enqueue give bitwise the same xi, M and e_x as the
    first call (same kernels and task order, fixed-order sums)."""
    banner("batched ace replays")
    import torch
    insts = _make(SPECS, True, px_ctx)
    args = []
    for d in insts:
        n = d["inst"].n_orb
        d["M"] = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
        args.append(dict(cell=d["cell"], psi=d["psi"], occ=d["occ"], kern=d["kern"], e_x=d["e_x"], M=d["M"],
                         out=torch.empty_like(d["psi"])))
        px_ctx.set_tuning(d["cell"], px.PX_PREC_FP32, 8, 8)

    def run():
        for a in args:
            a["out"].zero_()
            a["M"].zero_()
        _, stats = px_ctx.px_exchange_apply_batched(args, ace=True)
        px_ctx.px_sync()
        assert all(int(st.item()) == 0 for st in stats)
        return [(a["out"].clone(), a["M"].clone(), float(a["e_x"].item())) for a in args]

    try:
        ref = run()
        for rep in range(3):
            junk = torch.randn(1 << 20, device="cuda").sum()      # eager work between replays
            got = run()
            del junk
            for (x, m, e), (x0, m0, e0) in zip(got, ref):
                assert torch.equal(x, x0) and torch.equal(m, m0) and e == e0, f"replay {rep} differs"
        px_ctx.px_set_graph(False)
        got = run()
        for (x, m, e), (x0, m0, e0) in zip(got, ref):
            assert torch.equal(x, x0) and torch.equal(m, m0) and e == e0
    finally:
        px_ctx.px_set_graph(True)
        for d in insts:
            px_ctx.set_tuning(d["cell"], px.PX_PREC_FP32, 0, 0)


@pytest.mark.parametrize("blk", [0, 8])
@pytest.mark.parametrize("fp32", [False, True])
def test_batched_ace_matches_oracle(px_ctx, fp32, blk):
    """ACE tails: with the default blocks every instance completes in its
    size's first wave (one tail group per size); with 8 x 8 blocks instances
    complete in different waves, so several groups of different sizes run on
    both side streams while later waves are still in flight."""
    banner(f"batched ace fp32={fp32} blk={blk}")
    import torch
    insts = _make(SPECS, fp32, px_ctx)
    prec = px.PX_PREC_FP32 if fp32 else px.PX_PREC_FP64
    args = []
    for d in insts:
        n = d["inst"].n_orb
        d["M"] = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
        args.append(dict(cell=d["cell"], psi=d["psi"], occ=d["occ"], kern=d["kern"], e_x=d["e_x"], M=d["M"]))
        px_ctx.set_tuning(d["cell"], prec, blk, blk)
    try:
        xis, stats = px_ctx.px_exchange_apply_batched(args, ace=True)
        px_ctx.px_sync()
    finally:
        for d in insts:
            px_ctx.set_tuning(d["cell"], prec, 0, 0)
    tol = FP32_TOL if fp32 else FP64_TOL
    for d, xi, st in zip(insts, xis, stats):
        inst = d["inst"]
        assert int(st.item()) == 0
        K = oracle.kernel_hse(inst.n, inst.L, 0.106)
        dV = inst.omega / inst.ng
        r = oracle.ace_build(inst.psi, inst.occ, K, dV)
        print(f"n={inst.n[0]} N={inst.n_orb}: M {relerr(to_host(d['M']), r['M']):.2e} "
              f"xi {relerr(to_host(xi), r['xi']):.2e}")
        assert relerr(to_host(d["M"]), r["M"]) < tol
        assert relerr(to_host(xi), r["xi"]) < tol
        ex = oracle.exchange_energy_gspace(inst.psi, inst.occ, K, inst.omega)
        assert abs(float(d["e_x"].item()) - ex) / abs(ex) < (FP32_EX_TOL if fp32 else FP64_TOL)


def test_autotune_and_cache(px_ctx, tmp_path):
    banner("autotune")
    import torch
    d = _make([(32, 40, 0.02, 9)], True, px_ctx)[0]
    path = str(tmp_path / "tune.jsonl")
    best = px_ctx.px_autotune(d["cell"], d["psi"], d["occ"], d["kern"], cache_path=path)
    assert best in (16, 24, 32, 48, 64, 96, 128, 192, 256)
    lines = open(path).read().strip().splitlines()
    assert len(lines) == 1 and f'"block": {best}' in lines[0]
    assert '"p2": 0' in lines[0] or '"p2": 1' in lines[0]
    assert '"48/1"' in lines[0]        # both pass-2 configurations, blocks up to the first B >= n
    # results with the tuned block equal the untuned ones to FP32 tolerance
    tuned = to_host(px_ctx.px_exchange_apply(d["cell"], d["psi"], d["occ"], d["psi"], d["kern"]))
    px_ctx.set_tuning(d["cell"], px.PX_PREC_FP32, 0, 0)
    plain = to_host(px_ctx.px_exchange_apply(d["cell"], d["psi"], d["occ"], d["psi"], d["kern"]))
    assert relerr(tuned, plain) < 1e-6
    assert px_ctx.px_load_tuning(path) == 1
    px_ctx.set_tuning(d["cell"], px.PX_PREC_FP32, 0, 0)
    torch.cuda.synchronize()
