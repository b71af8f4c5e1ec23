"""Oracle: the occupation matrix sigma, its diagonalisation and the density, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. II-A writes the density matrix of a mixed state as P = Phi sigma Phi^*
with a Hermitian occupation matrix sigma.  Sec. IV-A-1 diagonalises it,
sigma = Q D Q^* (Eq. 11), so that with phi = Phi Q the density matrix becomes
sum_i d_i phi_i phi_i^* (Eq. 12) and the exchange operator the double sum of
Eq. 13.  Sec. III-C gives the charge density of PT-IM as
rho(r) = sum_{i,j} phi_i(r) sigma_ij phi_j^*(r).
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
