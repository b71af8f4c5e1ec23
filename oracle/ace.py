"""Oracle: adaptively compressed exchange (ACE), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (14) states the defining property of the ACE operator, W_i = Vx phi_i =
V_ACE phi_i, and its low-rank form V_ACE(r,r') = -sum_k xi_k(r) conj(xi_k(r'))
(the conjugate is missing in the printed equation; rank N).  The construction
itself is deferred by the paper to the ACE literature; the steps used here are
the standard ones:

    W = Vx Psi,  M = dV Psi^H W,  M <- (M + M^H)/2,  -M = L L^H  (lower, real
    positive diagonal),  xi = W L^{-H},  V_ACE phi = -xi (dV xi^H phi).

With the dV-weighted inner product V_ACE Psi = W holds exactly.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

from .exchange import exchange_apply

# Time step of the paper's propagation, 50 attoseconds in atomic units of time
# (1 a.u. = 24.188843265857 as), and the hybrid mixing fraction of Eq. (8).
DT_50AS = 50.0 / 24.188843265857
ALPHA = 0.25


def _flat(a):
    return a.reshape(a.shape[0], -1)


def ace_build(psi, occ, K, dV):
    """Returns dict(W, M, L, xi, herm_defect) for orbitals psi [N][n2][n1][n0]."""
    psi = np.asarray(psi, dtype=np.complex128)
    W = exchange_apply(psi, occ, psi, K)
    Wf, Pf = _flat(W), _flat(psi)
    M = dV * (np.conj(Pf) @ Wf.T)          # M[a][b] = dV sum_r conj(psi_a) W_b
    herm_defect = np.linalg.norm(M - M.conj().T) / np.linalg.norm(M)
    M = 0.5 * (M + M.conj().T)
    L = np.linalg.cholesky(-M)             # lower, positive real diagonal
    # xi (as N_g x N columns) = W L^{-H}  <=>  xi^H = L^{-1} W^H
    xiH = solve_triangular(L, np.conj(Wf), lower=True)
    xi = np.conj(xiH).reshape(psi.shape)
    return dict(W=W, M=M, L=L, xi=xi, herm_defect=float(herm_defect))


def ace_apply(xi, phi, dV):
    """Y = V_ACE phi = -xi (dV xi^H phi); xi [N][...], phi [Nphi][...]."""
    Xf, Ff = _flat(np.asarray(xi)), _flat(np.asarray(phi, dtype=np.complex128))
    C = dV * (np.conj(Xf) @ Ff.T)          # [N][Nphi]
    Y = -(C.T @ Xf)                        # Y[c] = -sum_a C[a][c] xi_a
    return Y.reshape(np.asarray(phi).shape)


def ptim_exchange_loop(xi, phi_n, dV, n_iter=4, dt=DT_50AS, alpha=ALPHA):
    """Exchange-only implicit-midpoint fixed point with the ACE operator.

    The orbital update of Eq. (6) with the midpoint of Eq. (4), keeping only
    the alpha*Vx part of H (Eq. 8) and no projector, iterated as the fixed
    point x = T(x) of Eq. (7):

        Phi^(k+1) = Phi_n - i dt alpha V_ACE (Phi_n + Phi^(k))/2,  Phi^(0) = Phi_n,

    with the relative residual R_k = ||Phi^(k+1) - Phi^(k)||_F / ||Phi^(k+1)||_F.
    Returns (Phi^(n_iter), [R_0 .. R_{n_iter-1}]).
    """
    phi_n = np.asarray(phi_n, dtype=np.complex128)
    cur = phi_n.copy()
    res = []
    for _ in range(n_iter):
        mid = 0.5 * (phi_n + cur)
        nxt = phi_n - 1j * dt * alpha * ace_apply(xi, mid, dV)
        res.append(float(np.linalg.norm(nxt - cur) / np.linalg.norm(nxt)))
        cur = nxt
    return cur, res
