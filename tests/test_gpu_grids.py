"""Non-cubic grids: the wavefunction grids of the paper's 768- and 1536-atom
cells (Sec. VI), 60 x 60 x 90 and 60 x 90 x 120 with x fastest, on
orthorhombic cells with three different edge lengths.  Against the oracle:
the kernel table, the exchange application with its energy, the ACE build in
the Hermitian-pair mode with diagonal, off-diagonal and ragged blocks, and a
batch that mixes both grids with a cubic instance.  Tolerances as for the
cubic grids: FP64 1e-11; FP32 2e-5 (E_x 1e-7)."""
import numpy as np
import pytest

import oracle
from paper_2501_03061_amd import inputs, px
from _gpu import banner, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

FP64_TOL, FP32_TOL, FP32_EX_TOL = 1e-11, 2e-5, 1e-7
SHAPES = [((60, 60, 90), 7), ((60, 90, 120), 6)]
MU = 0.106


def _inst(n, n_orb, seed):
    return inputs.make_instance(n, tuple(0.28 * m for m in n), n_orb, kT=0.04, seed=seed)


def _dev_block(ctx, psi, fp32):
    d = to_dev(psi)
    return ctx.px_convert_c128_to_c64(d) if fp32 else d


@pytest.mark.parametrize("n", [s for s, _ in SHAPES])
def test_kernel_hse_noncubic(px_ctx, n):
    banner(f"kernel_hse grid {n}")
    L = tuple(0.28 * m for m in n)
    k = to_host(px_ctx.px_kernel_hse(px.Cell(L, n), MU))
    ref = oracle.kernel_hse(n, L, MU)
    assert k.shape == (n[2], n[1], n[0])
    assert np.abs(k - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("n,n_orb", SHAPES)
def test_exchange_noncubic(px_ctx, n, n_orb, fp32):
    import torch
    banner(f"exchange grid {n} N={n_orb} fp32={fp32}")
    inst = _inst(n, n_orb, seed=71)
    K = oracle.kernel_hse(inst.n, inst.L, MU)
    ref = oracle.exchange_apply(inst.psi, inst.occ, inst.psi, K)
    ex = oracle.exchange_energy_gspace(inst.psi, inst.occ, K, inst.omega)
    cell = px.Cell(inst.L, inst.n)
    p = _dev_block(px_ctx, inst.psi, fp32)
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    out = px_ctx.px_exchange_apply(cell, p, to_dev(inst.occ), p, px_ctx.px_kernel_hse(cell, MU), e_x=e)
    torch.cuda.synchronize()
    err, eerr = relerr(to_host(out), ref), abs(float(e.item()) - ex) / abs(ex)
    print(f"grid {n} fp32={fp32}: vx {err:.2e} e_x {eerr:.2e}", flush=True)
    assert err < (FP32_TOL if fp32 else FP64_TOL)
    assert eerr < (FP32_EX_TOL if fp32 else FP64_TOL)


@pytest.mark.parametrize("fp32", [False, True])
def test_ace_build_noncubic(px_ctx, fp32):
    """60 x 90 x 120, 7 orbitals in 3 x 3 blocks (3, 3, 1): triangular diagonal
    blocks, kept v_ij below the diagonal, a ragged last block."""
    import torch
    banner(f"ace build grid 60x90x120 fp32={fp32}")
    inst = _inst((60, 90, 120), 7, seed=72)
    K = oracle.kernel_hse(inst.n, inst.L, MU)
    dV = inst.omega / inst.ng
    r = oracle.ace_build(inst.psi, inst.occ, K, dV)
    ex = oracle.exchange_energy_gspace(inst.psi, inst.occ, K, inst.omega)
    cell = px.Cell(inst.L, inst.n)
    prec = px.PX_PREC_FP32 if fp32 else px.PX_PREC_FP64
    px_ctx.set_tuning(cell, prec, 3, 3)
    try:
        M = torch.zeros((7, 7), dtype=torch.complex128, device="cuda")
        e = torch.zeros(1, dtype=torch.float64, device="cuda")
        xi, st = px_ctx.px_ace_build(cell, _dev_block(px_ctx, inst.psi, fp32), to_dev(inst.occ),
                                     px_ctx.px_kernel_hse(cell, MU), M=M, e_x=e)
        px_ctx.px_sync()
    finally:
        px_ctx.set_tuning(cell, prec, 0, 0)
    tol = FP32_TOL if fp32 else FP64_TOL
    em, ex_ = relerr(to_host(M), r["M"]), relerr(to_host(xi), r["xi"])
    eerr = abs(float(e.item()) - ex) / abs(ex)
    print(f"ace 60x90x120 fp32={fp32}: M {em:.2e} xi {ex_:.2e} E_x {eerr:.2e}", flush=True)
    assert int(st.item()) == 0
    assert em < tol and ex_ < tol
    assert eerr < (FP32_EX_TOL if fp32 else FP64_TOL)


def test_batched_mixed_grids(px_ctx):
    """FP32 ACE builds of both non-cubic grids and a cubic one in one batched
    call (waves grouped by grid), each against the oracle."""
    banner("batched ace mixed grids")
    specs = [((60, 60, 90), 5, 81), ((32, 32, 32), 9, 82), ((60, 90, 120), 6, 83)]
    args, refs = [], []
    for n, n_orb, seed in specs:
        inst = _inst(n, n_orb, seed)
        K = oracle.kernel_hse(inst.n, inst.L, MU)
        refs.append(oracle.ace_build(inst.psi, inst.occ, K, inst.omega / inst.ng)["xi"])
        cell = px.Cell(inst.L, inst.n)
        args.append(dict(cell=cell, psi=_dev_block(px_ctx, inst.psi, True), occ=to_dev(inst.occ),
                         kern=px_ctx.px_kernel_hse(cell, MU)))
    xis, stats = px_ctx.px_exchange_apply_batched(args, ace=True)
    px_ctx.px_sync()
    for (n, _, _), xi, st, ref in zip(specs, xis, stats, refs):
        err = relerr(to_host(xi), ref)
        print(f"batched grid {n}: xi {err:.2e}", flush=True)
        assert int(st.item()) == 0
        assert err < FP32_TOL
