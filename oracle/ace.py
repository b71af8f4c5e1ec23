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


def ptim_step(xi, phi_n, sigma_n, dV, n_iter=4, dt=DT_50AS, alpha=ALPHA):
    """Exchange-only PT-IM step with the projection and the occupation matrix.

    The scheme of Eq. (6) at the midpoints of Eq. (4), with the projector of
    Eq. (5) and H reduced to its exchange part alpha * V_ACE (Eq. 8, V_ACE of
    Eq. 14), iterated as the fixed point x = T(x) of Eq. (7) on
    x = (Phi_{n+1}, sigma_{n+1}) from the guess x^(0) = (Phi_n, sigma_n):

        Phi_mid   = (Phi_n + Phi^(k)) / 2,   sigma_mid = (sigma_n + sigma^(k)) / 2
        Y         = alpha V_ACE Phi_mid                       (H Phi_mid)
        S         = dV Phi_mid^H Phi_mid,    Hm = dV Phi_mid^H Y   (Phi^* H Phi)
        Phi^(k+1)   = Phi_n   - i dt (Y - Phi_mid S^{-1} Hm)     ((I - P~) H Phi_mid)
        sigma^(k+1) = sigma_n - i dt (Hm sigma_mid - sigma_mid Hm)

    P~ Y = Phi (Phi^* Phi)^{-1} Phi^* Y of Eq. (5); the dV weights of S and of
    Phi^H Y cancel there, and make Hm the matrix of H in the continuous inner
    product.  Residuals R_k = ||x^(k+1) - x^(k)|| / ||x^(k+1)|| (Frobenius),
    separately for Phi and sigma.  xi [N][...], phi_n [Nphi][...] orbitals,
    sigma_n [Nphi][Nphi].  Returns (Phi^(n_iter), sigma^(n_iter),
    [R_Phi,0 ..], [R_sigma,0 ..]).  Anderson mixing, the other terms of H and
    the final orthogonalisation of Algorithm 1 are not part of this step.
    """
    phi_n = np.asarray(phi_n, dtype=np.complex128)
    sigma_n = np.asarray(sigma_n, dtype=np.complex128)
    shape = phi_n.shape
    Pn = _flat(phi_n)
    cur_p, cur_s = Pn.copy(), sigma_n.copy()
    res_p, res_s = [], []
    for _ in range(n_iter):
        mid = 0.5 * (Pn + cur_p)
        smid = 0.5 * (sigma_n + cur_s)
        Y = alpha * _flat(ace_apply(xi, mid.reshape(shape), dV))
        S = dV * (np.conj(mid) @ mid.T)            # S[a][b] = dV <mid_a | mid_b>
        Hm = dV * (np.conj(mid) @ Y.T)             # Hm[a][b] = dV <mid_a | Y_b>
        # P~ Y: column b of Y projected on span(mid), mid (S^{-1} Hm)
        X = np.linalg.solve(S, Hm)
        PY = X.T @ mid                             # row b = sum_a X[a][b] mid_a
        nxt_p = Pn - 1j * dt * (Y - PY)
        nxt_s = sigma_n - 1j * dt * (Hm @ smid - smid @ Hm)
        res_p.append(float(np.linalg.norm(nxt_p - cur_p) / np.linalg.norm(nxt_p)))
        res_s.append(float(np.linalg.norm(nxt_s - cur_s) / np.linalg.norm(nxt_s)))
        cur_p, cur_s = nxt_p, nxt_s
    return cur_p.reshape(shape), cur_s, res_p, res_s
