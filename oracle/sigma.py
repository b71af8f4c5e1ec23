"""Oracle: the occupation matrix sigma, its diagonalisation and the density, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. II-A writes the density matrix of a mixed state as P = Phi sigma Phi^*
with a Hermitian occupation matrix sigma.  Sec. IV-A-1 diagonalises it,
sigma = Q D Q^* (Eq. 11), so that with phi = Phi Q the density matrix becomes
sum_i d_i phi_i phi_i^* (Eq. 12) and the exchange operator the double sum of
Eq. 13.  Sec. III-C gives the charge density of PT-IM as
rho(r) = sum_{i,j} phi_i(r) sigma_ij phi_j^*(r).  Sec. VI evaluates the
exchange on the wavefunction grid and the charge density on a grid twice as
fine per axis (120 x 180 x 240 for the 60 x 90 x 120 wavefunction grid).
"""
from __future__ import annotations

import numpy as np


def _flat(a):
    a = np.asarray(a)
    return a.reshape(a.shape[0], -1)


def sigma_eig(sigma):
    """sigma = Q diag(d) Q^H for a Hermitian sigma (Eq. 11), d ascending.

    LAPACK's Hermitian eigensolver (numpy.linalg.eigh) on (sigma + sigma^H)/2;
    column k of Q is the eigenvector of d[k].  Returns (d, Q).
    """
    s = np.asarray(sigma, dtype=np.complex128)
    d, Q = np.linalg.eigh(0.5 * (s + s.conj().T))
    return d, Q


def rotate(phi_basis, Q):
    """phi = Phi Q: orbital b of the result is sum_a Q[a][b] Phi_a (Eq. 11's basis)."""
    P = _flat(np.asarray(phi_basis, dtype=np.complex128))
    return (np.asarray(Q).T @ P).reshape(np.asarray(phi_basis).shape)


def density_sigma(phi_basis, sigma):
    """rho(r) = sum_{i,j} Phi_i(r) sigma_ij conj(Phi_j(r)) (Sec. III-C): the
    double sum, N^2 products per grid point.  Real for a Hermitian sigma; the
    real part is returned."""
    P = _flat(np.asarray(phi_basis, dtype=np.complex128))
    s = np.asarray(sigma, dtype=np.complex128)
    rho = np.einsum("ir,ij,jr->r", P, s, P.conj(), optimize=True)
    return rho.real.reshape(np.asarray(phi_basis).shape[1:])


def density(phi, occ):
    """rho(r) = sum_i occ_i |phi_i(r)|^2: the density of Eq. 12's diagonal
    form (N products per grid point)."""
    P = _flat(np.asarray(phi, dtype=np.complex128))
    rho = np.asarray(occ, dtype=np.float64) @ (P.real ** 2 + P.imag ** 2)
    return rho.reshape(np.asarray(phi).shape[1:])


def _pad_axis(c, axis):
    """Zero-pads the unnormalised DFT coefficients c along one even axis of
    length n to length 2n: frequencies 0 .. n/2-1 and -n/2+1 .. -1 keep their
    coefficients, the Nyquist coefficient (index n/2, frequency +-n/2 on the
    coarse grid) is split evenly between +n/2 and -n/2 of the fine grid."""
    c = np.moveaxis(c, axis, 0)
    n = c.shape[0]
    if n % 2:
        raise ValueError("even axis lengths only")
    h = n // 2
    out = np.zeros((2 * n,) + c.shape[1:], dtype=np.complex128)
    out[:h] = c[:h]                      # 0 .. n/2-1
    out[2 * n - h + 1:] = c[h + 1:]      # -n/2+1 .. -1
    out[h] = 0.5 * c[h]                  # +n/2
    out[2 * n - h] = 0.5 * c[h]          # -n/2
    return np.moveaxis(out, 0, axis)


def density_fine(phi, occ):
    """The density of Eq. 12's diagonal form on the grid twice as fine per
    axis (the charge-density grid of Sec. VI): each orbital is Fourier-
    interpolated onto the fine grid (its spectrum zero-padded by _pad_axis,
    one axis after the other), then rho_f = sum_i occ_i |phi_i^f|^2.
    phi [N][n2][n1][n0] with even n0, n1, n2; returns [2 n2][2 n1][2 n0]."""
    phi = np.asarray(phi, dtype=np.complex128)
    occ = np.asarray(occ, dtype=np.float64)
    n2, n1, n0 = phi.shape[1:]
    rho = np.zeros((2 * n2, 2 * n1, 2 * n0))
    for i in range(phi.shape[0]):
        c = np.fft.fftn(phi[i])           # unnormalised forward transform
        for axis in range(3):
            c = _pad_axis(c, axis)
        f = np.fft.ifftn(c) * 8.0         # ifftn divides by 8 N_g; the coarse inverse by N_g
        rho += occ[i] * (f.real ** 2 + f.imag ** 2)
    return rho
