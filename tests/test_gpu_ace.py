"""GPU parity of px_ace_build and px_ace_apply against the CPU oracle, the
ACE exactness property, and the Cholesky breakdown path."""
import numpy as np
import pytest

import oracle
from paper_2501_03061_amd import inputs, px
from _gpu import banner, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

FP64_TOL, FP32_TOL, FP32_EX_TOL = 1e-11, 2e-5, 1e-7


@pytest.fixture(scope="module")
def toy():
    c = inputs.CONFIGS["toy24"]
    inst = inputs.make_instance(c["n"], c["L"], c["n_orb"], c["kT"], seed=c["seed"])
    K = oracle.kernel_hse(inst.n, inst.L, c["mu"])
    dV = inst.omega / inst.ng
    r = oracle.ace_build(inst.psi, inst.occ, K, dV)
    r["ex"] = oracle.exchange_energy_gspace(inst.psi, inst.occ, K, inst.omega)
    return inst, K, dV, r


def _build(ctx, inst, kd, fp32):
    import torch
    cell = px.Cell(inst.L, inst.n)
    psi = to_dev(inst.psi)
    if fp32:
        psi = ctx.px_convert_c128_to_c64(psi)
    n = inst.n_orb
    M = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    xi, st = ctx.px_ace_build(cell, psi, to_dev(inst.occ), kd, M=M, e_x=e)
    ctx.px_sync()
    return cell, psi, xi, to_host(M), float(e.item()), int(st.item())


@pytest.mark.parametrize("fp32", [False, True])
def test_ace_build_toy24(px_ctx, toy, fp32):
    inst, K, dV, r = toy
    banner(f"ace build toy24 fp32={fp32}")
    cell = px.Cell(inst.L, inst.n)
    kd = px_ctx.px_kernel_hse(cell, 0.106)
    cell, psi, xi, M, e, st = _build(px_ctx, inst, kd, fp32)
    assert st == 0
    tol = FP32_TOL if fp32 else FP64_TOL
    em, ex_, ee = relerr(M, r["M"]), relerr(to_host(xi), r["xi"]), abs(e - r["ex"]) / abs(r["ex"])
    print(f"ace fp32={fp32}: M {em:.3e} xi {ex_:.3e} E_x {ee:.3e}")
    assert em < tol
    assert ex_ < tol
    assert ee < (FP32_EX_TOL if fp32 else FP64_TOL)
    # operator action on span(Psi): V_ACE Psi = W = Vx Psi
    y = to_host(px_ctx.px_ace_apply(cell, xi, psi))
    assert relerr(y, r["W"]) < tol


@pytest.mark.parametrize("fp32", [False, True])
def test_ace_apply_random_block(px_ctx, toy, fp32):
    inst, K, dV, r = toy
    banner(f"ace apply toy24 fp32={fp32}")
    rng = np.random.default_rng(11)
    phi = rng.standard_normal((5,) + inst.psi.shape[1:]) + 1j * rng.standard_normal((5,) + inst.psi.shape[1:])
    cell = px.Cell(inst.L, inst.n)
    xi = to_dev(r["xi"])
    ph = to_dev(phi)
    if fp32:
        xi, ph = px_ctx.px_convert_c128_to_c64(xi), px_ctx.px_convert_c128_to_c64(ph)
    y = to_host(px_ctx.px_ace_apply(cell, xi, ph))
    ref = oracle.ace_apply(r["xi"], phi, dV)
    assert relerr(y, ref) < (FP32_TOL if fp32 else FP64_TOL)


def test_ace_build_larger_n_ragged_tiles(px_ctx):
    """n = 70 orbitals: GEMM tiles of 64 leave a ragged edge; 32^3 grid."""
    banner("ace build n=70 grid 32")
    inst = inputs.make_instance(32, 9.0, 70, kT=0.03, seed=5)
    K = oracle.kernel_hse(inst.n, inst.L, 0.106)
    dV = inst.omega / inst.ng
    r = oracle.ace_build(inst.psi, inst.occ, K, dV)
    cell = px.Cell(inst.L, inst.n)
    cell, psi, xi, M, e, st = _build(px_ctx, inst, to_dev(K), False)
    assert st == 0
    assert relerr(M, r["M"]) < FP64_TOL
    assert relerr(to_host(xi), r["xi"]) < FP64_TOL


def test_ace_cholesky_breakdown_reported(px_ctx, toy):
    """A negated kernel makes M positive semidefinite: -M has no Cholesky
    factor, the status word names column 1 and px_sync raises."""
    inst, K, dV, r = toy
    banner("ace cholesky breakdown")
    import torch
    cell = px.Cell(inst.L, inst.n)
    psi = to_dev(inst.psi)
    xi, st = px_ctx.px_ace_build(cell, psi, to_dev(inst.occ), to_dev(-K))
    with pytest.raises(px.PxError) as ei:
        px_ctx.px_sync()
    assert ei.value.status == px.PX_ERR_NOT_POSITIVE_DEFINITE
    assert "ace_build: -M is not positive definite (Cholesky breakdown at column 1)" in str(ei.value)
    assert int(st.item()) == 1
    # latched until cleared
    with pytest.raises(px.PxError):
        px_ctx.px_sync()
    px_ctx.px_clear_error()
    px_ctx.px_sync()
    torch.cuda.synchronize()


@pytest.mark.parametrize("fp32", [False, True])
def test_ptim_loop_matches_oracle(px_ctx, toy, fp32):
    """Exchange-only implicit-midpoint fixed point with V_ACE matches the
    oracle loop, iterate and FP64 residuals.  The FP32 form runs the loop on
    the complex64 copies of xi and Phi_n (its contractions in FP32, the
    residual norms in FP64) and meets 2e-5 on the iterate.  A residual is a
    norm of the difference of two iterates over the norm of one, so each
    R_k can move by at most about twice the iterates' relative error: the
    FP32 residuals are compared with an absolute bound of 4e-5, and R_0
    (about 0.1 here) to 1e-4 relative."""
    inst, K, dV, r = toy
    banner(f"ptim loop toy24 fp32={fp32}")
    cell = px.Cell(inst.L, inst.n)
    z = inputs.noise_block(inst.n, inst.L, inst.n_orb, seed=1001)
    phi_n = inst.psi + 1e-3 * z
    ref_phi, ref_res = oracle.ptim_exchange_loop(r["xi"], phi_n, dV, n_iter=4)
    xi_d, phi_d = to_dev(r["xi"]), to_dev(phi_n)
    if fp32:
        xi_d, phi_d = px_ctx.px_convert_c128_to_c64(xi_d), px_ctx.px_convert_c128_to_c64(phi_d)
    out, res = px_ctx.px_ptim_exchange_loop(cell, xi_d, phi_d, 4, oracle.DT_50AS * oracle.ALPHA)
    err, res_h = relerr(to_host(out), ref_phi), to_host(res)
    print(f"ptim loop fp32={fp32}: iterate err {err:.2e}, residuals {res_h} oracle {ref_res}")
    if not fp32:
        assert err < FP64_TOL
        assert np.allclose(res_h, ref_res, rtol=1e-9, atol=1e-15)
    else:
        assert err < FP32_TOL
        assert np.all(np.abs(res_h - np.asarray(ref_res)) < 2 * FP32_TOL)
        assert abs(res_h[0] - ref_res[0]) < 1e-4 * ref_res[0]
        assert np.all(np.diff(res_h) < 0)


@pytest.mark.parametrize("sym", [False, True])
@pytest.mark.parametrize("fp32", [False, True])
def test_ace_build_symmetry_modes_ragged_blocks(px_ctx, fp32, sym):
    """n = 70 on a 24^3 grid with 16x16 blocks: blocks of 16, 16, 16, 16, 6 give
    off-diagonal, diagonal and ragged blocks in the Hermitian-pair mode."""
    banner(f"ace symmetry={sym} fp32={fp32}")
    inst = inputs.make_instance(24, 10.0, 70, kT=0.04, seed=7)
    K = oracle.kernel_hse(inst.n, inst.L, 0.106)
    dV = inst.omega / inst.ng
    r = oracle.ace_build(inst.psi, inst.occ, K, dV)
    ex = oracle.exchange_energy_gspace(inst.psi, inst.occ, K, inst.omega)
    cell = px.Cell(inst.L, inst.n)
    prec = px.PX_PREC_FP32 if fp32 else px.PX_PREC_FP64
    px_ctx.set_tuning(cell, prec, 16, 16)
    px_ctx.px_set_symmetry(sym)
    try:
        cell, psi, xi, M, e, st = _build(px_ctx, inst, to_dev(K), fp32)
        y = to_host(px_ctx.px_ace_apply(cell, xi, psi))
    finally:
        px_ctx.px_set_symmetry(True)
        px_ctx.set_tuning(cell, prec, 0, 0)
    tol = FP32_TOL if fp32 else FP64_TOL
    assert st == 0
    print(f"sym={sym} fp32={fp32}: M {relerr(M, r['M']):.2e} W {relerr(y, r['W']):.2e} "
          f"E_x {abs(e - ex) / abs(ex):.2e}")
    assert relerr(M, r["M"]) < tol
    assert relerr(y, r["W"]) < tol
    assert relerr(to_host(xi), r["xi"]) < tol
    assert abs(e - ex) < (FP32_EX_TOL if fp32 else FP64_TOL) * abs(ex)


def test_ace_build_profiling_stages(px_ctx, toy):
    """Profiling mode: per-pass and per-stage times of one build are reported,
    and the profiled build gives the same result as an unprofiled one."""
    inst, K, dV, r = toy
    banner("ace build profiling stages")
    cell = px.Cell(inst.L, inst.n)
    kd = px_ctx.px_kernel_hse(cell, 0.106)
    _, _, xi0, M0, _, _ = _build(px_ctx, inst, kd, False)
    px_ctx.px_profile_read(reset=True)
    px_ctx.px_profile_read_ace(reset=True)
    px_ctx.px_set_profiling(True)
    try:
        _, _, xi1, M1, _, st = _build(px_ctx, inst, kd, False)
    finally:
        px_ctx.px_set_profiling(False)
    passes = px_ctx.px_profile_read(reset=True)
    stages = px_ctx.px_profile_read_ace(reset=True)
    assert st == 0
    assert stages["calls"] == 1
    assert stages["M"] > 0 and stages["factor"] > 0 and stages["xi"] > 0
    assert all(p["launches"] > 0 and p["ms"] > 0 for p in passes[:3])
    assert np.array_equal(M0, M1)
    assert np.array_equal(to_host(xi0), to_host(xi1))
    assert px_ctx.px_profile_read_ace()["calls"] == 0


@pytest.mark.parametrize("sym", [False, True])
def test_ace_build_non_even_kernel(px_ctx, sym):
    """A real kernel with K(G) != K(-G) (the HSE kernel times 1 + 0.3 sin of a
    lattice phase).  Hermitian-pair mode off: M equals the oracle's.  On: the
    documented behaviour, i.e. pairs (i, j <= i) use K and the transposed
    pairs use K(-G); the oracle side builds that W orbital by orbital."""
    import torch
    banner(f"ace non-even kernel sym={sym}")
    inst = inputs.make_instance(16, 6.5, 7, kT=0.05, seed=17)
    n = inst.n_orb
    K0 = oracle.kernel_hse(inst.n, inst.L, 0.106)
    iz, iy, ix = np.meshgrid(*(np.arange(m) for m in inst.n[::-1]), indexing="ij")
    K = K0 * (1.0 + 0.3 * np.sin(2 * np.pi * (ix / inst.n[0] + 2 * iy / inst.n[1] + 3 * iz / inst.n[2])))
    Kref = K[(-iz) % inst.n[2], (-iy) % inst.n[1], (-ix) % inst.n[0]]
    assert np.abs(K - Kref).max() > 0.01 * np.abs(K).max()      # K(0) = pi / mu^2 dominates the max
    dV = inst.omega / inst.ng
    if sym:
        W = np.empty_like(inst.psi)
        for i in range(n):
            w = oracle.exchange_apply(inst.psi[:i + 1], inst.occ[:i + 1], inst.psi[i:i + 1], K)
            if i + 1 < n:
                w = w + oracle.exchange_apply(inst.psi[i + 1:], inst.occ[i + 1:], inst.psi[i:i + 1], Kref)
            W[i] = w[0]
    else:
        W = oracle.exchange_apply(inst.psi, inst.occ, inst.psi, K)
    Mref = dV * (inst.psi.reshape(n, -1).conj() @ W.reshape(n, -1).T)
    Mref = 0.5 * (Mref + Mref.conj().T)
    cell = px.Cell(inst.L, inst.n)
    px_ctx.set_tuning(cell, px.PX_PREC_FP64, 4, 4)       # diagonal, off-diagonal and ragged blocks
    px_ctx.px_set_symmetry(sym)
    try:
        M = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
        xi, st = px_ctx.px_ace_build(cell, to_dev(inst.psi), to_dev(inst.occ), to_dev(K), M=M)
        px_ctx.px_sync()
    finally:
        px_ctx.px_set_symmetry(True)
        px_ctx.set_tuning(cell, px.PX_PREC_FP64, 0, 0)
    err = relerr(to_host(M), Mref)
    print(f"non-even kernel sym={sym}: M {err:.2e}", flush=True)
    assert err < FP64_TOL
    if not sym:
        assert int(st.item()) == 0
        assert relerr(to_host(M), oracle.ace_build(inst.psi, inst.occ, K, dV)["M"]) < FP64_TOL
