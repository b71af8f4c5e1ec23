"""GPU parity of the occupation-matrix front end (Sec. IV-A-1, Eq. 11-13) and
the density (Sec. III-C, Eq. 12) against the CPU oracle.

* px_sigma_diagonalize: eigenvalues against LAPACK's, Q D Q^H against sigma,
  Q unitary; spectra with degenerate and tiny eigenvalues, odd and even n.
* px_exchange_apply_sigma: against the oracle's triple loop of Eq. 10 on tiny
  inputs (every (k, i, j) pair solve done directly), and against the oracle's
  diagonalised form on a 24^3 instance with Phi as the target.
* px_density / px_density_sigma: against the oracle's density (diagonal form)
  and its double sum over sigma.
Tolerances: FP64 form 1e-11 relative (1e-12 for the density and the
eigenvalues); FP32 form 2e-5.
"""
import numpy as np
import pytest

import oracle
from paper_2501_03061_amd import inputs, px
from _gpu import banner, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

FP64_TOL, FP32_TOL = 1e-11, 2e-5


def _unitary(rng, n):
    q, r = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _sigma(rng, n, degenerate=False):
    d = rng.uniform(0.0, 1.0, n)
    if degenerate and n >= 4:
        d[1] = d[0]
        d[3] = 1e-13
    U = _unitary(rng, n)
    return U @ np.diag(d) @ U.conj().T


@pytest.mark.parametrize("n", [1, 2, 7, 33, 64, 201, 600])
def test_sigma_diagonalize(px_ctx, n):
    import torch
    banner(f"sigma diagonalize n={n}")
    rng = np.random.default_rng(40 + n)
    sigma = _sigma(rng, n, degenerate=True)
    Q, d, st = px_ctx.px_sigma_diagonalize(to_dev(sigma))
    px_ctx.px_sync()
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    Qh, dh = to_host(Q), to_host(d)
    dref, _ = oracle.sigma_eig(sigma)
    scale = max(1.0, float(np.abs(dref).max()))
    print(f"n={n}: eigenvalue err {np.abs(dh - dref).max():.2e}, rebuild "
          f"{relerr(Qh @ np.diag(dh) @ Qh.conj().T, sigma):.2e}", flush=True)
    assert np.abs(dh - dref).max() < 1e-12 * scale
    assert np.all(np.diff(dh) >= 0)
    assert np.abs(Qh.conj().T @ Qh - np.eye(n)).max() < 1e-12
    assert relerr(Qh @ np.diag(dh) @ Qh.conj().T, sigma) < 1e-12


@pytest.mark.parametrize("n,kT", [(512, 0.02), (1536, 0.03)])
def test_sigma_diagonalize_fermi_dirac(px_ctx, n, kT):
    """The occupation matrices of the mixed-state workloads: Fermi-Dirac
    spectra, whose eigenvalues crowd exponentially close to 0 and 1 (Jacobi's
    slow case: quadratic convergence only once the off-diagonal norm is below
    those gaps)."""
    import torch
    banner(f"sigma diagonalize Fermi-Dirac n={n}")
    e = np.sort(np.random.default_rng(n).uniform(-0.5, 0.5, n))
    sigma = inputs.occupation_matrix(inputs.fermi_dirac(e, kT), seed=n + 1)
    Q, d, st = px_ctx.px_sigma_diagonalize(to_dev(sigma))
    px_ctx.px_sync()
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    Qh, dh = to_host(Q), to_host(d)
    dref, _ = oracle.sigma_eig(sigma)
    rebuild = relerr((Qh * dh) @ Qh.conj().T, sigma)
    print(f"n={n}: eigenvalue err {np.abs(dh - dref).max():.2e}, rebuild {rebuild:.2e}", flush=True)
    # Jacobi stops at an off-diagonal norm of 64 eps sqrt(n) ||sigma||; Q carries
    # the rounding of about 20 sweeps of rotations: O(n eps) after normalisation
    tol = 20 * n * np.finfo(float).eps
    assert np.abs(dh - dref).max() < 1e-11
    assert np.abs(Qh.conj().T @ Qh - np.eye(n)).max() < tol
    assert rebuild < tol


def test_sigma_diagonalize_diagonal_and_zero(px_ctx):
    """Already diagonal (no rotation at all) and all-zero sigma."""
    import torch
    banner("sigma diagonalize trivial")
    for sigma in (np.diag([0.3, 0.1, 0.9, 0.5]).astype(np.complex128), np.zeros((5, 5), np.complex128)):
        Q, d, st = px_ctx.px_sigma_diagonalize(to_dev(sigma))
        px_ctx.px_sync()
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        assert np.array_equal(to_host(d), np.sort(np.diag(sigma).real))
        Qh = to_host(Q)
        assert np.abs(np.abs(Qh) - np.abs(Qh).round()).max() == 0.0   # a permutation


@pytest.mark.parametrize("fp32", [False, True])
def test_exchange_sigma_vs_triple_loop(px_ctx, fp32):
    """Eq. 10 directly (N^3 pair solves in the oracle) on a 16^3 grid."""
    banner(f"exchange sigma vs triple loop fp32={fp32}")
    rng = np.random.default_rng(7)
    inst = inputs.make_instance(16, 6.0, 4, kT=0.05, seed=31)
    Phi = inst.psi
    tgt = inputs.noise_block(inst.n, inst.L, 3, seed=32)
    sigma = _sigma(rng, 4)
    K = oracle.kernel_hse(inst.n, inst.L, 0.106)
    ref = oracle.exchange_apply_sigma(Phi, sigma, tgt, K)
    cell = px.Cell(inst.L, inst.n)
    P, T = to_dev(Phi), to_dev(tgt)
    if fp32:
        P, T = px_ctx.px_convert_c128_to_c64(P), px_ctx.px_convert_c128_to_c64(T)
    out, st = px_ctx.px_exchange_apply_sigma(cell, P, to_dev(sigma), T, to_dev(K))
    px_ctx.px_sync()
    assert int(st.item()) == 0
    err = relerr(to_host(out), ref)
    print(f"exchange sigma fp32={fp32}: err vs Eq. 10 triple loop {err:.2e}", flush=True)
    assert err < (FP32_TOL if fp32 else FP64_TOL)


@pytest.mark.parametrize("fp32", [False, True])
def test_exchange_sigma_toy24_on_phi(px_ctx, fp32):
    """24^3, 16 orbitals, sigma with the Fermi-Dirac spectrum in a random
    basis, target Phi itself; against the oracle's diagonalised form."""
    banner(f"exchange sigma toy24 fp32={fp32}")
    c = inputs.CONFIGS["toy24"]
    inst = inputs.make_instance(c["n"], c["L"], c["n_orb"], 0.05, seed=c["seed"])
    rng = np.random.default_rng(8)
    U = _unitary(rng, inst.n_orb)
    sigma = U @ np.diag(inst.occ) @ U.conj().T
    K = oracle.kernel_hse(inst.n, inst.L, c["mu"])
    d, Q = oracle.sigma_eig(sigma)
    ref = oracle.exchange_apply(oracle.rotate(inst.psi, Q), d, inst.psi, K)
    cell = px.Cell(inst.L, inst.n)
    P = to_dev(inst.psi)
    if fp32:
        P = px_ctx.px_convert_c128_to_c64(P)
    out, st = px_ctx.px_exchange_apply_sigma(cell, P, to_dev(sigma), P, px_ctx.px_kernel_hse(cell, c["mu"]))
    px_ctx.px_sync()
    assert int(st.item()) == 0
    err = relerr(to_host(out), ref)
    print(f"exchange sigma toy24 fp32={fp32}: err {err:.2e}", flush=True)
    assert err < (FP32_TOL if fp32 else FP64_TOL)


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("n,L,N", [(24, 10.0, 16), (40, 11.2, 37)])
def test_density(px_ctx, fp32, n, L, N):
    import torch
    banner(f"density n={n} N={N} fp32={fp32}")
    inst = inputs.make_instance(n, L, N, kT=0.03, seed=50 + n)
    rng = np.random.default_rng(9)
    sigma = _sigma(rng, N)
    cell = px.Cell(inst.L, inst.n)
    P = to_dev(inst.psi)
    psi = inst.psi
    if fp32:
        P = px_ctx.px_convert_c128_to_c64(P)
        psi = to_host(P).astype(np.complex128)        # the oracle on the rounded orbitals
    rho = to_host(px_ctx.px_density(cell, P, to_dev(inst.occ)))
    rho_s, st = px_ctx.px_density_sigma(cell, P, to_dev(sigma))
    px_ctx.px_sync()
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    ref = oracle.density(psi, inst.occ)
    ref_s = oracle.density_sigma(psi, sigma)
    e1, e2 = relerr(rho, ref), relerr(to_host(rho_s), ref_s)
    print(f"density fp32={fp32}: occupations {e1:.2e}, sigma {e2:.2e}", flush=True)
    assert e1 < 1e-12
    assert e2 < (FP32_TOL if fp32 else 1e-12)


@pytest.mark.parametrize("fp32", [False, True])
def test_rotate_orbitals(px_ctx, fp32):
    """phi = Phi Q against the oracle's rotation (Eq. 11), with Q from the
    library's diagonalisation; the FP32 form against the oracle on the rounded
    Phi and Q."""
    import torch
    banner(f"rotate orbitals fp32={fp32}")
    rng = np.random.default_rng(12)
    inst = inputs.make_instance(24, 10.0, 37, kT=0.05, seed=43)
    sigma = _sigma(rng, 37)
    cell = px.Cell(inst.L, inst.n)
    Q, d, st = px_ctx.px_sigma_diagonalize(to_dev(sigma))
    P = to_dev(inst.psi)
    if fp32:
        P = px_ctx.px_convert_c128_to_c64(P)
    out = to_host(px_ctx.px_rotate_orbitals(cell, P, Q))
    px_ctx.px_sync()
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    Qh = to_host(Q)
    if fp32:
        base, Qr = to_host(P).astype(np.complex128), Qh.astype(np.complex64).astype(np.complex128)
    else:
        base, Qr = inst.psi, Qh
    err = relerr(out, oracle.rotate(base, Qr))
    print(f"rotate fp32={fp32}: {err:.2e}", flush=True)
    assert err < (2e-6 if fp32 else 1e-13)


@pytest.mark.parametrize("fp32", [False, True])
def test_ace_build_sigma(px_ctx, fp32):
    """ACE operator of a full occupation matrix on a 16^3 grid with 6 orbitals
    and a random sigma with eigenvalues in [0, 1]:
    * V_ACE Phi = Vx[sigma] Phi against the oracle's Eq. 10 triple loop
      (exactness on span(Phi));
    * V_ACE on vectors outside span(Phi) against the oracle's ACE built on
      (Phi Q, d) (xi xi^H does not depend on the phases of Q);
    * e_x against (1/2) dV Tr(sigma Phi^H Vx[sigma] Phi) from the triple loop."""
    import torch
    banner(f"ace build sigma fp32={fp32}")
    rng = np.random.default_rng(11)
    inst = inputs.make_instance(16, 6.0, 6, kT=0.05, seed=41)
    Phi = inst.psi
    sigma = _sigma(rng, 6)
    K = oracle.kernel_hse(inst.n, inst.L, 0.106)
    dV = inst.omega / inst.ng
    vx_phi = oracle.exchange_apply_sigma(Phi, sigma, Phi, K)
    A = dV * Phi.reshape(6, -1).conj() @ vx_phi.reshape(6, -1).T        # A_ki = dV <Phi_k|Vx Phi_i>
    e_ref = 0.5 * float(np.trace(sigma @ A).real)
    d, Q = oracle.sigma_eig(sigma)
    r = oracle.ace_build(oracle.rotate(Phi, Q), d, K, dV)
    X = inputs.noise_block(inst.n, inst.L, 3, seed=42)
    ref_x = oracle.ace_apply(r["xi"], X, dV)
    cell = px.Cell(inst.L, inst.n)
    P, Xd = to_dev(Phi), to_dev(X)
    if fp32:
        P, Xd = px_ctx.px_convert_c128_to_c64(P), px_ctx.px_convert_c128_to_c64(Xd)
    e_x = torch.zeros(1, dtype=torch.float64, device="cuda")
    xi, st = px_ctx.px_ace_build_sigma(cell, P, to_dev(sigma), to_dev(K), e_x=e_x)
    px_ctx.px_sync()
    assert to_host(st).tolist() == [0, 0]
    on_span = to_host(px_ctx.px_ace_apply(cell, xi, P))
    off_span = to_host(px_ctx.px_ace_apply(cell, xi, Xd))
    torch.cuda.synchronize()
    e1, e2 = relerr(on_span, vx_phi), relerr(off_span, ref_x)
    e3 = abs(float(e_x.item()) - e_ref) / abs(e_ref)
    print(f"ace build sigma fp32={fp32}: V_ACE Phi vs Eq. 10 {e1:.2e}, outside span {e2:.2e}, "
          f"e_x {e3:.2e}", flush=True)
    tol = FP32_TOL if fp32 else FP64_TOL
    assert e1 < tol and e2 < tol
    assert e3 < (1e-7 if fp32 else FP64_TOL)


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("n,L,N", [(16, 8.0, 5), ((24, 16, 20), (9.0, 6.0, 7.5), 37), ((60, 60, 90), (16.8, 16.8, 25.2), 18)])
def test_density_fine(px_ctx, fp32, n, L, N):
    """The density on the twice-finer charge-density grid against the oracle's
    zero-padded transforms: cubic, orthorhombic (any even grid, no FFT plan
    needed) and the paper's 768-atom wavefunction grid; 37 orbitals cross the
    16-orbital chunks with a ragged tail.  The FP32 form against the oracle on
    the rounded orbitals."""
    import torch
    banner(f"density fine n={n} N={N} fp32={fp32}")
    inst = inputs.make_instance(n, L, N, kT=0.03, seed=70 + N)
    cell = px.Cell(inst.L, inst.n)
    P = to_dev(inst.psi)
    base = inst.psi
    if fp32:
        P = px_ctx.px_convert_c128_to_c64(P)
        base = to_host(P).astype(np.complex128)
    occ = to_dev(inst.occ)
    rf = to_host(px_ctx.px_density_fine(cell, P, occ))
    rc = to_host(px_ctx.px_density(cell, P, occ))
    torch.cuda.synchronize()
    ref = oracle.density_fine(base, inst.occ)
    err = float(np.abs(rf - ref).max() / np.abs(ref).max())
    ec = float(np.abs(rf[::2, ::2, ::2] - rc).max() / np.abs(rc).max())
    print(f"density fine n={n} fp32={fp32}: vs oracle {err:.2e}, even points vs px_density {ec:.2e}",
          flush=True)
    assert err < (FP32_TOL if fp32 else 1e-12)
    assert ec < (FP32_TOL if fp32 else 1e-13)
