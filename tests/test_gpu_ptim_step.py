"""GPU parity of px_ptim_step, the exchange-only PT-IM step with the projector
of Eq. 5 and the occupation-matrix commutator of Eq. 6 (Eq. 4-7), against the
CPU oracle: iterates Phi and sigma and both residual sequences, on a toy
instance with non-orthogonal Phi_n and a random Hermitian sigma_n, on ragged
sizes, and on plane waves, where Phi must stay put and sigma follow the
scalar implicit-midpoint recursion.  Tolerances: FP64 1e-11; FP32 2e-5 on
Phi and sigma, residuals within twice that."""
import numpy as np
import pytest

import oracle
from paper_2501_03061_amd import inputs, px
from _gpu import banner, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

FP64_TOL, FP32_TOL = 1e-11, 2e-5
DTA = oracle.DT_50AS * oracle.ALPHA


def _herm(rng, n):
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return X @ X.conj().T / n


def _case(n_grid, L, n_orb, n_phi, seed):
    inst = inputs.make_instance(n_grid, L, n_orb, kT=0.04, seed=seed)
    K = oracle.kernel_hse(inst.n, inst.L, 0.106)
    dV = inst.omega / inst.ng
    r = oracle.ace_build(inst.psi, inst.occ, K, dV)
    z = inputs.noise_block(inst.n, inst.L, n_phi, seed=seed + 1)
    phi_n = inst.psi[:n_phi] + 0.3 * z
    sig = _herm(np.random.default_rng(seed + 2), n_phi)
    return inst, r, dV, phi_n, sig


def _run(ctx, inst, xi, phi_n, sig, n_iter, fp32):
    import torch
    cell = px.Cell(inst.L, inst.n)
    x, p = to_dev(xi), to_dev(phi_n)
    if fp32:
        x, p = ctx.px_convert_c128_to_c64(x), ctx.px_convert_c128_to_c64(p)
    po, so, res, st = ctx.px_ptim_step(cell, x, p, to_dev(sig), n_iter, DTA)
    ctx.px_sync()
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return to_host(po), to_host(so), to_host(res)


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("grid,L,n_orb,n_phi", [(24, 10.0, 16, 8), (32, 9.0, 70, 37)])
def test_ptim_step_matches_oracle(px_ctx, fp32, grid, L, n_orb, n_phi):
    banner(f"ptim step grid {grid} n={n_orb} n_phi={n_phi} fp32={fp32}")
    inst, r, dV, phi_n, sig = _case(grid, L, n_orb, n_phi, seed=60 + grid)
    ref_p, ref_s, ref_rp, ref_rs = oracle.ptim_step(r["xi"], phi_n, sig, dV, n_iter=4)
    po, so, res = _run(px_ctx, inst, r["xi"], phi_n, sig, 4, fp32)
    ep, es = relerr(po, ref_p), relerr(so, ref_s)
    print(f"ptim step fp32={fp32}: Phi {ep:.2e} sigma {es:.2e}; residuals Phi {res[0]} "
          f"(oracle {ref_rp}), sigma {res[1]} (oracle {ref_rs})", flush=True)
    if fp32:
        assert ep < FP32_TOL and es < FP32_TOL
        assert np.all(np.abs(res[0] - ref_rp) < 2 * FP32_TOL)
        assert np.all(np.abs(res[1] - ref_rs) < 2 * FP32_TOL)
    else:
        assert ep < FP64_TOL and es < FP64_TOL
        assert np.allclose(res[0], ref_rp, rtol=1e-9, atol=1e-15)
        assert np.allclose(res[1], ref_rs, rtol=1e-9, atol=1e-15)
    # trace and Hermiticity of sigma are kept (FP64 algebra in both forms)
    assert abs(np.trace(so) - np.trace(sig)) < 1e-12 * abs(np.trace(sig))
    assert np.linalg.norm(so - so.conj().T) < 1e-12 * np.linalg.norm(so)


def test_ptim_step_plane_waves(px_ctx):
    """Plane waves: V_ACE Phi lies in span(Phi), so the projected update
    vanishes and Phi stays; sigma_ij follows the scalar midpoint recursion with
    omega_ij = alpha (lam_i - lam_j)."""
    banner("ptim step plane waves")
    n, L, mu = 24, 7.0, 0.15
    ms = [(0, 0, 0), (1, 1, 0), (-2, 0, 3), (5, -4, 1)]
    occ = np.array([1.0, 0.6, 0.3, 0.1])
    psi = inputs.plane_wave_orbitals(n, L, ms)
    K = oracle.kernel_hse((n, n, n), (L, L, L), mu)
    dV = L ** 3 / n ** 3
    r = oracle.ace_build(psi, occ, K, dV)
    lam = np.real(np.diag(r["M"]))
    sig = _herm(np.random.default_rng(5), 4)

    class _I:
        pass
    inst = _I()
    inst.L, inst.n = (L, L, L), (n, n, n)
    po, so, res = _run(px_ctx, inst, r["xi"], psi, sig, 6, False)
    w = oracle.ALPHA * (lam[:, None] - lam[None, :])
    s = sig.copy()
    for _ in range(6):
        s = sig - 1j * oracle.DT_50AS * w * (sig + s) / 2
    print(f"plane waves: Phi moved {relerr(po, psi):.2e}, sigma err {relerr(so, s):.2e}", flush=True)
    assert relerr(po, psi) < FP64_TOL
    assert relerr(so, s) < FP64_TOL
    assert np.all(res[0] < 1e-12)
