"""Oracle: the Fock exchange operator with fractional occupations, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (readings of points the paper leaves open):
  * grid layout [orb][n2][n1][n0], x = n0 fastest; G = 2*pi*m/L per axis with
    the signed frequency m = i if i < n/2 else i - n;
  * forward FFT exp(-iG.r) unnormalised, inverse exp(+iG.r) scaled by 1/N_g
    (NumPy's convention).  With a real, even kernel K(G) = K(-G) the operator
    does not depend on the sign convention;
  * Vx carries the minus sign of Eq. (10) (the accumulation step printed in
    Algorithm 2 lacks it); the mixing fraction alpha of Eq. (8) and any spin
    factor are not applied;
  * the operator is the discrete one on the full wavefunction grid: no
    dealiasing, no projection onto the cutoff sphere, no screening of small
    occupations.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft

_WORKERS = max(1, os.cpu_count() or 1)


def _fftn(a):
    return sfft.fftn(a, axes=(-3, -2, -1), workers=_WORKERS)


def _ifftn(a):
    return sfft.ifftn(a, axes=(-3, -2, -1), workers=_WORKERS)


def signed_freq(n: int) -> np.ndarray:
    """Signed frequency of FFT index i: i for i < n/2, else i - n."""
    i = np.arange(n)
    return np.where(i < n / 2.0, i, i - n)


def g2_grid(n, L) -> np.ndarray:
    """|G|^2 on the FFT grid, shape [n2][n1][n0]."""
    n0, n1, n2 = n
    gx = 2.0 * math.pi * signed_freq(n0) / L[0]
    gy = 2.0 * math.pi * signed_freq(n1) / L[1]
    gz = 2.0 * math.pi * signed_freq(n2) / L[2]
    return gz[:, None, None] ** 2 + gy[None, :, None] ** 2 + gx[None, None, :] ** 2


def kernel_hse(n, L, mu: float) -> np.ndarray:
    """Screened interaction K(G) of the HSE06 functional (Sec. II-B leaves the
    kernel as "possibly screened"; Sec. VI uses HSE06).

    K(G) = 4*pi*(1 - exp(-G^2/(4 mu^2)))/G^2 for G != 0, evaluated with expm1,
    and its G -> 0 limit pi/mu^2 at G = 0.  This is the Fourier transform of
    erfc(mu*r)/r.
    """
    g2 = g2_grid(n, L)
    out = np.empty_like(g2)
    nz = g2 > 0
    out[nz] = 4.0 * math.pi * (-np.expm1(-g2[nz] / (4.0 * mu * mu))) / g2[nz]
    out[~nz] = math.pi / (mu * mu)
    return out


def pair_potential(rho: np.ndarray, K: np.ndarray) -> np.ndarray:
    """v = IFFT[K * FFT(rho)]: the Poisson-type solve behind one orbital pair
    (the forward FFT, kernel multiply and inverse FFT of Algorithm 2)."""
    return _ifftn(K * _fftn(rho))


def exchange_apply(psi, occ, phi, K, chunk=64):
    """(Vx phi_i)(r) = -sum_j f_j psi_j(r) IFFT[K FFT(conj(psi_j) phi_i)](r).

    Eq. (13) with the occupation-matrix eigenvalues d_j written as f_j: the
    double loop over orbital pairs.  psi [Npsi][n2][n1][n0], occ [Npsi],
    phi [Nphi][n2][n1][n0], K [n2][n1][n0]; returns [Nphi][n2][n1][n0].
    The sum over j runs in blocks of ``chunk`` orbitals to bound memory.
    """
    psi = np.asarray(psi, dtype=np.complex128)
    phi = np.asarray(phi, dtype=np.complex128)
    occ = np.asarray(occ, dtype=np.float64)
    out = np.zeros(phi.shape, dtype=np.complex128)
    for i in range(phi.shape[0]):
        acc = np.zeros(phi.shape[1:], dtype=np.complex128)
        for a in range(0, psi.shape[0], chunk):
            pj = psi[a:a + chunk]
            rho = np.conj(pj) * phi[i][None]
            v = pair_potential(rho, K[None])
            acc -= np.einsum("j,jzyx->zyx", occ[a:a + chunk], pj * v)
        out[i] = acc
    return out


def exchange_energy_real(psi, occ, vx_psi, dV) -> float:
    """E_x = 1/2 sum_i f_i Re <psi_i | Vx psi_i>, <a|b> = dV sum_r conj(a) b.

    The paper's convergence test uses the exchange energy without a formula;
    this is the standard definition for the operator of Eq. (13), with alpha
    and spin not applied.
    """
    ip = dV * np.einsum("izyx,izyx->i", np.conj(psi), vx_psi).real
    return 0.5 * float(np.dot(occ, ip))


def exchange_energy_gspace(psi, occ, K, omega) -> float:
    """Same energy summed over pairs in reciprocal space:
    E_x = -1/2 Omega sum_{i,j} f_i f_j sum_G K(G) |FFT(conj(psi_j) psi_i)/N_g|^2."""
    ng = psi[0].size
    e = 0.0
    for i in range(psi.shape[0]):
        rho_hat = _fftn(np.conj(psi) * psi[i][None]) / ng
        s = np.einsum("zyx,jzyx->j", K, (rho_hat * np.conj(rho_hat)).real)
        e += occ[i] * float(np.dot(occ, s))
    return -0.5 * omega * e


def exchange_apply_sigma(phi_basis, sigma, phi, K):
    """Mixed-state Vx with a full Hermitian occupation matrix, Eq. (10):

    (Vx phi_j)(r) = -sum_{i,k} sigma_ik phi_i(r) IFFT[K FFT(conj(phi_k) phi_j)](r),

    as the triple loop over (k, i, j) of Algorithm 2 (with Eq. (10)'s sign):
    N^3 pair solves.  Only for tiny inputs.
    """
    n = phi_basis.shape[0]
    out = np.zeros(phi.shape, dtype=np.complex128)
    for k in range(n):
        for i in range(n):
            for j in range(phi.shape[0]):
                tmp = pair_potential(np.conj(phi_basis[k]) * phi[j], K)
                out[j] -= sigma[i, k] * tmp * phi_basis[i]
    return out
