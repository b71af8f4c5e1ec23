"""Seeded synthetic inputs for the exchange / ACE path.

This module builds the *inputs* of the problem only: band-limited,
orthonormal plane-wave orbitals on a periodic real-space grid, Fermi-Dirac
occupations, plain plane waves and perturbation fields.  It contains none of
the arithmetic of the exchange operator or of ACE; both the CPU oracle and the
HIP library consume what it returns.

Shapes follow the library's layout: an orbital block is a C-ordered array
``[n_orb][n2][n1][n0]`` (x = n0 fastest) of complex values.  Orbitals are
normalised so that ``dV * sum_r |psi(r)|^2 = 1`` with ``dV = Omega / N_g``.

Recipe (the paper's workloads are silicon supercells at a 10 Ha cutoff, HSE06
and 8000 K, Sec. VI; here smooth random fields of the same cutoff, kernel and
temperature range stand in for them):

* G-vectors of the grid, ``G = 2*pi*m/L`` per axis with the signed frequency
  ``m`` of each FFT index, kept where ``|G|^2/2 <= ecut``;
* ``C = rng.standard_normal((N_pw, N)) + 1j*rng.standard_normal((N_pw, N))``,
  reduced Householder QR, ``psi = (N_g/sqrt(Omega)) * ifftn(Q placed on grid)``;
* then ``eps = sort(rng.uniform(-0.5, 0.5, N))`` Ha and
  ``f = 1/(1+exp(eps/kT))`` (chemical potential 0).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np
import scipy.fft as _sfft
from scipy.special import expit

__all__ = [
    "Instance", "signed_freq", "sphere_indices", "random_orbitals",
    "fermi_dirac", "make_instance", "plane_wave_orbitals", "noise_block",
    "batch_recipe", "occupation_matrix", "CONFIGS",
]


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def signed_freq(n: int) -> np.ndarray:
    """Signed frequency of FFT index m: m if m < n/2 else m - n."""
    m = np.arange(n)
    return np.where(m < n / 2.0, m, m - n)


def sphere_indices(n: tuple[int, int, int], L: tuple[float, float, float],
                   ecut: float) -> np.ndarray:
    """Flat C-order indices ([z][y][x]) of grid G-vectors with |G|^2/2 <= ecut."""
    n0, n1, n2 = n
    gx = 2.0 * math.pi * signed_freq(n0) / L[0]
    gy = 2.0 * math.pi * signed_freq(n1) / L[1]
    gz = 2.0 * math.pi * signed_freq(n2) / L[2]
    g2 = (gz[:, None, None] ** 2 + gy[None, :, None] ** 2 + gx[None, None, :] ** 2)
    return np.flatnonzero(0.5 * g2.ravel() <= ecut)


def random_orbitals(n, L, n_orb, ecut, rng, out=None, chunk=64):
    """Orthonormal random band-limited orbitals, [n_orb][n2][n1][n0] complex128.

    ``out`` may be a preallocated complex128 array (e.g. pinned host memory) of
    that shape; it is filled in chunks of ``chunk`` orbitals so that large
    blocks never need a second full-size temporary.
    """
    n0, n1, n2 = n
    ng = n0 * n1 * n2
    omega = L[0] * L[1] * L[2]
    idx = sphere_indices(n, L, ecut)
    if len(idx) < n_orb:
        raise ValueError(f"{len(idx)} plane waves inside the cutoff < {n_orb} orbitals")
    c = rng.standard_normal((len(idx), n_orb)) + 1j * rng.standard_normal((len(idx), n_orb))
    q, _ = np.linalg.qr(c, mode="reduced")
    del c
    if out is None:
        out = np.empty((n_orb, n2, n1, n0), dtype=np.complex128)
    scale = ng / math.sqrt(omega)
    for a in range(0, n_orb, chunk):
        b = min(n_orb, a + chunk)
        g = np.zeros((b - a, ng), dtype=np.complex128)
        g[:, idx] = q[:, a:b].T
        blk = _sfft.ifftn(g.reshape(b - a, n2, n1, n0), axes=(1, 2, 3), workers=_workers())
        blk *= scale
        out[a:b] = blk
    return out


def fermi_dirac(eps: np.ndarray, kT: float) -> np.ndarray:
    """f = 1/(1+exp(eps/kT)) evaluated without overflow, chemical potential 0."""
    return expit(-np.asarray(eps, dtype=np.float64) / kT)


@dataclass
class Instance:
    n: tuple[int, int, int]          # grid (n0, n1, n2), n0 = x fastest
    L: tuple[float, float, float]    # orthorhombic edge lengths, bohr
    psi: np.ndarray                  # [N][n2][n1][n0] complex128
    occ: np.ndarray                  # [N] float64 occupations in [0, 1]
    eps: np.ndarray                  # [N] float64 eigenvalues behind occ, Ha
    kT: float
    seed: int

    @property
    def n_orb(self) -> int:
        return self.psi.shape[0]

    @property
    def ng(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def omega(self) -> float:
        return self.L[0] * self.L[1] * self.L[2]


def make_instance(n, L, n_orb, kT, seed=0, ecut=10.0, out=None) -> Instance:
    """One seeded instance: orbitals first, then eigenvalues, from one generator."""
    if isinstance(n, int):
        n = (n, n, n)
    if isinstance(L, (int, float)):
        L = (float(L),) * 3
    rng = np.random.default_rng(seed)
    psi = random_orbitals(n, L, n_orb, ecut, rng, out=out)
    eps = np.sort(rng.uniform(-0.5, 0.5, n_orb))
    return Instance(n=tuple(n), L=tuple(float(x) for x in L), psi=psi,
                    occ=fermi_dirac(eps, kT), eps=eps, kT=kT, seed=seed)


def plane_wave_orbitals(n, L, ms) -> np.ndarray:
    """psi_j(r) = exp(i k_j.r)/sqrt(Omega), k_j = 2*pi*m_j/L, for integer triples m_j."""
    if isinstance(n, int):
        n = (n, n, n)
    if isinstance(L, (int, float)):
        L = (float(L),) * 3
    n0, n1, n2 = n
    omega = L[0] * L[1] * L[2]
    x = np.arange(n0)[None, None, :] / n0
    y = np.arange(n1)[None, :, None] / n1
    z = np.arange(n2)[:, None, None] / n2
    out = np.empty((len(ms), n2, n1, n0), dtype=np.complex128)
    for j, (mx, my, mz) in enumerate(ms):
        out[j] = np.exp(2j * math.pi * (mx * x + my * y + mz * z)) / math.sqrt(omega)
    return out


def noise_block(n, L, n_orb, seed, ecut=10.0, chunk=64) -> np.ndarray:
    """Band-limited random fields (same sphere as the orbitals), each column
    scaled to dV-norm 1, not orthogonalised.  Coefficients are drawn orbital
    by orbital (real parts, then imaginary parts) from one generator."""
    if isinstance(n, int):
        n = (n, n, n)
    if isinstance(L, (int, float)):
        L = (float(L),) * 3
    n0, n1, n2 = n
    ng = n0 * n1 * n2
    dv = L[0] * L[1] * L[2] / ng
    rng = np.random.default_rng(seed)
    idx = sphere_indices(n, L, ecut)
    out = np.empty((n_orb, n2, n1, n0), dtype=np.complex128)
    for a in range(0, n_orb, chunk):
        b = min(n_orb, a + chunk)
        g = np.zeros((b - a, ng), dtype=np.complex128)
        for k in range(b - a):
            g[k, idx] = rng.standard_normal(len(idx)) + 1j * rng.standard_normal(len(idx))
        f = _sfft.ifftn(g.reshape(b - a, n2, n1, n0), axes=(1, 2, 3), workers=_workers())
        norms = np.sqrt(dv * np.einsum("kzyx,kzyx->k", f.conj(), f).real)
        out[a:b] = f / norms[:, None, None, None]
    return out


def batch_recipe(n_inst=48, seed=0, sizes=(32, 40, 48, 64), n_range=(32, 256),
                 kT_range=(0.005, 0.05), spacing=0.28):
    """Parameters of the uneven batch: a master generator draws (n, N, kT) per
    instance; instance s is then generated with seed s and L = spacing*n."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_inst):
        n = int(rng.choice(sizes))
        n_orb = int(rng.integers(n_range[0], n_range[1] + 1))
        kT = float(rng.uniform(*kT_range))
        out.append(dict(n=n, L=spacing * n, n_orb=n_orb, kT=kT, seed=s))
    return out


def occupation_matrix(occ, seed, mix=0.1) -> np.ndarray:
    """A full Hermitian occupation matrix with the spectrum occ, standing for
    sigma some time steps into a run (it starts diagonal and develops
    coherences): sigma = V diag(occ) V^H with V the unitary factor of the QR of
    I + mix * (A + iB) / sqrt(2 n), A and B standard normal from one generator
    (column phases fixed so that diag(R) > 0).  complex128 [n][n]."""
    occ = np.asarray(occ, dtype=np.float64)
    n = occ.shape[0]
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    q, r = np.linalg.qr(np.eye(n) + mix * g / math.sqrt(2.0 * n))
    d = np.diag(r)
    q = q * (d / np.abs(d))
    sigma = (q * occ) @ q.conj().T
    return (sigma + sigma.conj().T) / 2


# The five workloads: grids, cells, orbital counts and temperatures.
CONFIGS = {
    "toy24": dict(n=24, L=10.0, n_orb=16, kT=0.01, mu=0.106, seed=0),
    "mid72": dict(n=72, L=20.0, n_orb=512, kT=0.02, mu=0.106, seed=0),
    "large96": dict(n=96, L=27.0, n_orb=1536, kT=0.03, mu=0.106, seed=0),
}
