"""Thin ctypes binding of libpx (include/px.h).

Argument marshalling only: every array argument is a torch tensor that lives
on the GPU (device memory and the current stream come from PyTorch); its data
pointer, sizes and the stream handle are passed to the C entry point of the
same name.  Nothing here computes any part of the method, and there is no
fallback: if libpx.so is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpx.so")

PX_OK, PX_ERR_INVALID_ARG, PX_ERR_UNSUPPORTED_GRID, PX_ERR_WORKSPACE, PX_ERR_DEVICE, \
    PX_ERR_NOT_POSITIVE_DEFINITE, PX_ERR_NOT_CONVERGED = range(7)
PX_PREC_FP64, PX_PREC_FP32 = 0, 1
PX_OP_EXCHANGE, PX_OP_ACE_BUILD, PX_OP_ACE_APPLY, PX_OP_PTIM_LOOP = 0, 1, 2, 3
PX_OP_EXCHANGE_SIGMA, PX_OP_SIGMA_DIAG, PX_OP_DENSITY_SIGMA, PX_OP_PTIM_STEP = 4, 5, 6, 7
PX_OP_ACE_BUILD_SIGMA, PX_OP_ROTATE, PX_OP_DENSITY_FINE = 8, 9, 10

STATUS_NAMES = {0: "PX_OK", 1: "PX_ERR_INVALID_ARG", 2: "PX_ERR_UNSUPPORTED_GRID",
                3: "PX_ERR_WORKSPACE", 4: "PX_ERR_DEVICE", 5: "PX_ERR_NOT_POSITIVE_DEFINITE",
                6: "PX_ERR_NOT_CONVERGED"}

# Every function declared in include/px.h, with its ctypes signature.
_vp, _i32, _sz, _dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.c_double


class PxCell(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3), ("n", ctypes.c_int32 * 3)]


_cellp = ctypes.POINTER(PxCell)


class PxInstance(ctypes.Structure):
    _fields_ = [("cell", PxCell), ("n", ctypes.c_int32), ("psi", ctypes.c_void_p),
                ("occ", ctypes.c_void_p), ("kernel_G", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("e_x", ctypes.c_void_p), ("M", ctypes.c_void_p), ("status", ctypes.c_void_p)]


_instp = ctypes.POINTER(PxInstance)
SIGNATURES = {
    "px_abi_version": (_i32, []),
    "px_create": (_i32, [_i32, ctypes.POINTER(_vp)]),
    "px_destroy": (None, [_vp]),
    "px_last_error": (ctypes.c_char_p, [_vp]),
    "px_grid_supported": (_i32, [_cellp, _i32]),
    "px_workspace_bytes": (_sz, [_vp, _i32, _cellp, _i32, _i32, _i32]),
    "px_set_workspace": (_i32, [_vp, _vp, _sz]),
    "px_set_tuning": (_i32, [_vp, _cellp, _i32, _i32, _i32]),
    "px_kernel_hse": (_i32, [_vp, _cellp, _dbl, _vp, _vp]),
    "px_convert_c128_to_c64": (_i32, [_vp, _sz, _vp, _vp, _vp]),
    "px_stream_copy": (_i32, [_vp, _vp, _vp, _sz, _vp]),
    "px_exchange_apply": (_i32, [_vp, _cellp, _i32, _i32, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "px_ace_build": (_i32, [_vp, _cellp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "px_ace_apply": (_i32, [_vp, _cellp, _i32, _i32, _vp, _i32, _vp, _vp, _vp]),
    "px_ace_apply_noalloc": (_i32, [_vp, _cellp, _i32, _i32, _vp, _i32, _vp, _vp, _vp]),
    "px_ptim_exchange_loop": (_i32, [_vp, _cellp, _i32, _i32, _vp, _i32, _vp, _i32, _dbl, _vp, _vp, _vp]),
    "px_sigma_diagonalize": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "px_exchange_apply_sigma": (_i32, [_vp, _cellp, _i32, _i32, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "px_density": (_i32, [_vp, _cellp, _i32, _i32, _vp, _vp, _vp, _vp]),
    "px_density_sigma": (_i32, [_vp, _cellp, _i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "px_density_fine": (_i32, [_vp, _cellp, _i32, _i32, _vp, _vp, _vp, _vp]),
    "px_ptim_step": (_i32, [_vp, _cellp, _i32, _i32, _vp, _i32, _vp, _vp, _i32, _dbl, _vp, _vp, _vp,
                            _vp, _vp]),
    "px_ace_build_sigma": (_i32, [_vp, _cellp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "px_rotate_orbitals": (_i32, [_vp, _cellp, _i32, _i32, _vp, _vp, _vp, _vp]),
    "px_set_symmetry": (_i32, [_vp, _i32]),
    "px_set_profiling": (_i32, [_vp, _i32]),
    "px_profile_read_ace": (_i32, [_vp, ctypes.POINTER(_dbl), ctypes.POINTER(ctypes.c_int64), _i32]),
    "px_profile_read": (_i32, [_vp, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl),
                               ctypes.POINTER(ctypes.c_int64), _i32]),
    "px_workspace_bytes_batched": (_sz, [_vp, _i32, _instp, _i32, _i32]),
    "px_exchange_apply_batched": (_i32, [_vp, _i32, _instp, _i32, _i32, _vp]),
    "px_set_batch_capacity": (_i32, [_vp, _sz]),
    "px_set_graph": (_i32, [_vp, _i32]),
    "px_autotune": (_i32, [_vp, _cellp, _i32, _i32, _vp, _vp, _vp, _vp, ctypes.c_char_p,
                           ctypes.POINTER(_i32), _vp]),
    "px_load_tuning": (_i32, [_vp, ctypes.c_char_p, ctypes.POINTER(_i32)]),
    "px_sync": (_i32, [_vp, _vp]),
    "px_clear_error": (None, [_vp]),
}

_lib = None


class PxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load_library(path: str = LIB_PATH):
    """Loads libpx.so once; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libpx.so not found at {path}: run __graft_entry__.build() "
                          "(or python -m paper_2501_03061_amd.csrc.build) first")
    # PyTorch brings its own HIP runtime; load it before libpx so that both use
    # the same one (a second runtime loaded first does not see the GPU)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


@dataclass(frozen=True)
class Cell:
    """Orthorhombic cell: edge lengths L (bohr) and grid n = (n0, n1, n2), n0 = x."""
    L: tuple
    n: tuple

    @staticmethod
    def cubic(n: int, L: float) -> "Cell":
        return Cell((float(L),) * 3, (int(n),) * 3)

    def c(self) -> PxCell:
        return PxCell((ctypes.c_double * 3)(*self.L), (ctypes.c_int32 * 3)(*self.n))

    @property
    def ng(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def omega(self) -> float:
        return self.L[0] * self.L[1] * self.L[2]

    @property
    def dV(self) -> float:
        return self.omega / self.ng


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _prec(dtype) -> int:
    import torch
    if dtype == torch.complex128:
        return PX_PREC_FP64
    if dtype == torch.complex64:
        return PX_PREC_FP32
    raise TypeError(f"orbital blocks must be complex128 or complex64, got {dtype}")


def _check_block(name, t, cell: Cell, dtype=None):
    if t is None:
        raise ValueError(f"{name} is required")
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous device tensor")
    if t.dim() != 4 or tuple(t.shape[1:]) != (cell.n[2], cell.n[1], cell.n[0]):
        raise ValueError(f"{name} must have shape [orb][n2][n1][n0], got {tuple(t.shape)}")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")


def _check_dev(name, t, dtype, numel=None, at_least=None, required=True):
    """A contiguous device tensor of dtype holding numel (or at least at_least)
    elements; None passes a null pointer where the argument is optional.  The
    library reads every pointer on the device: a host tensor here would fault
    the GPU instead of raising."""
    if t is None:
        if required:
            raise ValueError(f"{name} is required")
        return
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    if at_least is not None and t.numel() < at_least:
        raise ValueError(f"{name} must have at least {at_least} elements, got {t.numel()}")


def _check_inputs(cell: "Cell", n, occ=None, kern=None, e_x=None, M=None, status=None, nstatus=1):
    """The occupations (FP64, n), the kernel table (FP64, N_g) and the optional
    FP64 energy, complex128 n x n Gram matrix and int32 status words."""
    import torch
    if occ is not False:
        _check_dev("occ", occ, torch.float64, at_least=n)
    if kern is not False:
        _check_dev("kern", kern, torch.float64, numel=cell.ng)
    _check_dev("e_x", e_x, torch.float64, at_least=1, required=False)
    _check_dev("M", M, torch.complex128, numel=n * n, required=False)
    _check_dev("status", status, torch.int32, at_least=nstatus, required=False)


class Context:
    """A px_context plus a caller-owned workspace tensor grown on demand."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        h = ctypes.c_void_p()
        st = self.lib.px_create(int(device), ctypes.byref(h))
        if st != PX_OK:
            raise PxError(st, "px_create failed")
        self.h = h
        self.device = device
        self.ws = None

    def close(self):
        if self.h:
            self.lib.px_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != PX_OK:
            raise PxError(st, self.lib.px_last_error(self.h).decode())

    def last_error(self) -> str:
        return self.lib.px_last_error(self.h).decode()

    # ------------------------------------------------------------ workspace
    def workspace_bytes(self, op, cell: Cell, prec, n_psi, n_phi=0) -> int:
        return int(self.lib.px_workspace_bytes(self.h, op, ctypes.byref(cell.c()), prec, n_psi, n_phi))

    def ensure_workspace(self, nbytes: int):
        import torch
        if nbytes <= 0:
            raise PxError(PX_ERR_INVALID_ARG, "invalid problem for workspace sizing")
        if self.ws is None or self.ws.numel() < nbytes:
            if self.ws is not None:
                self.ws = None
                torch.cuda.synchronize(self.device)
                torch.cuda.empty_cache()
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")
        self._check(self.lib.px_set_workspace(self.h, _ptr(self.ws), self.ws.numel()))

    def set_tuning(self, cell: Cell, prec, ic: int, jc: int):
        self._check(self.lib.px_set_tuning(self.h, ctypes.byref(cell.c()), prec, ic, jc))

    # ------------------------------------------------------------ entry points
    def px_kernel_hse(self, cell: Cell, mu: float, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((cell.n[2], cell.n[1], cell.n[0]), dtype=torch.float64,
                              device=f"cuda:{self.device}")
        _check_dev("out", out, torch.float64, numel=cell.ng)
        self._check(self.lib.px_kernel_hse(self.h, ctypes.byref(cell.c()), float(mu), _ptr(out),
                                           _stream(stream)))
        return out

    def px_convert_c128_to_c64(self, src, dst=None, stream=None):
        import torch
        if src.dtype != torch.complex128 or not src.is_contiguous():
            raise TypeError("src must be a contiguous complex128 tensor")
        _check_dev("src", src, torch.complex128)
        if dst is None:
            dst = torch.empty(src.shape, dtype=torch.complex64, device=src.device)
        _check_dev("dst", dst, torch.complex64, at_least=src.numel())
        self._check(self.lib.px_convert_c128_to_c64(self.h, src.numel(), _ptr(src), _ptr(dst),
                                                    _stream(stream)))
        return dst

    def px_stream_copy(self, src, dst, stream=None):
        nbytes = src.numel() * src.element_size()
        if dst.numel() * dst.element_size() < nbytes:
            raise ValueError("dst smaller than src")
        self._check(self.lib.px_stream_copy(self.h, _ptr(src), _ptr(dst), nbytes, _stream(stream)))
        return dst

    def px_exchange_apply(self, cell: Cell, psi, occ, phi, kern, out=None, e_x=None,
                          stream=None):
        import torch
        prec = _prec(psi.dtype)
        _check_block("psi", psi, cell)
        _check_block("phi", phi, cell, psi.dtype)
        _check_inputs(cell, psi.shape[0], occ, kern, e_x)
        if out is None:
            out = torch.empty_like(phi)
        _check_block("out", out, cell, psi.dtype)
        self.ensure_workspace(self.workspace_bytes(PX_OP_EXCHANGE, cell, prec, psi.shape[0], phi.shape[0]))
        self._check(self.lib.px_exchange_apply(
            self.h, ctypes.byref(cell.c()), prec, psi.shape[0], _ptr(psi), _ptr(occ),
            phi.shape[0], _ptr(phi), _ptr(kern), _ptr(out), _ptr(e_x), _stream(stream)))
        return out

    def px_ace_build(self, cell: Cell, psi, occ, kern, xi=None, M=None, e_x=None, status=None,
                     stream=None):
        import torch
        prec = _prec(psi.dtype)
        _check_block("psi", psi, cell)
        dev = psi.device
        if xi is None:
            xi = torch.empty_like(psi)
        if status is None:
            status = torch.zeros(1, dtype=torch.int32, device=dev)
        _check_block("xi", xi, cell, psi.dtype)
        _check_inputs(cell, psi.shape[0], occ, kern, e_x, M, status)
        self.ensure_workspace(self.workspace_bytes(PX_OP_ACE_BUILD, cell, prec, psi.shape[0]))
        self._check(self.lib.px_ace_build(
            self.h, ctypes.byref(cell.c()), prec, psi.shape[0], _ptr(psi), _ptr(occ), _ptr(kern),
            _ptr(xi), _ptr(M), _ptr(e_x), _ptr(status), _stream(stream)))
        return xi, status

    def px_ace_apply(self, cell: Cell, xi, phi, out=None, stream=None):
        import torch
        prec = _prec(xi.dtype)
        _check_block("xi", xi, cell)
        _check_block("phi", phi, cell, xi.dtype)
        if out is None:
            out = torch.empty_like(phi)
        _check_block("out", out, cell, xi.dtype)
        self.ensure_workspace(self.workspace_bytes(PX_OP_ACE_APPLY, cell, prec, xi.shape[0], phi.shape[0]))
        self._check(self.lib.px_ace_apply(
            self.h, ctypes.byref(cell.c()), prec, xi.shape[0], _ptr(xi), phi.shape[0], _ptr(phi),
            _ptr(out), _stream(stream)))
        return out

    def px_ace_apply_noalloc(self, cell: Cell, xi, phi, out=None, stream=None):
        """px_ace_apply with the library's static scratch instead of the workspace."""
        import torch
        prec = _prec(xi.dtype)
        _check_block("xi", xi, cell)
        _check_block("phi", phi, cell, xi.dtype)
        if out is None:
            out = torch.empty_like(phi)
        _check_block("out", out, cell, xi.dtype)
        self._check(self.lib.px_ace_apply_noalloc(
            self.h, ctypes.byref(cell.c()), prec, xi.shape[0], _ptr(xi), phi.shape[0], _ptr(phi),
            _ptr(out), _stream(stream)))
        return out

    def px_ptim_exchange_loop(self, cell: Cell, xi, phi_n, n_iter: int, dt_alpha: float,
                              out=None, residuals=None, stream=None):
        import torch
        prec = _prec(xi.dtype)
        _check_block("xi", xi, cell)
        _check_block("phi_n", phi_n, cell, xi.dtype)
        if out is None:
            out = torch.empty_like(phi_n)
        if residuals is None:
            residuals = torch.zeros(n_iter, dtype=torch.float64, device=phi_n.device)
        _check_block("out", out, cell, xi.dtype)
        _check_dev("residuals", residuals, torch.float64, at_least=max(int(n_iter), 0))
        self.ensure_workspace(self.workspace_bytes(PX_OP_PTIM_LOOP, cell, prec, xi.shape[0], phi_n.shape[0]))
        self._check(self.lib.px_ptim_exchange_loop(
            self.h, ctypes.byref(cell.c()), prec, xi.shape[0], _ptr(xi), phi_n.shape[0],
            _ptr(phi_n), int(n_iter), float(dt_alpha), _ptr(out), _ptr(residuals), _stream(stream)))
        return out, residuals

    def _status(self, status, device):
        import torch
        if status is None:
            status = torch.zeros(1, dtype=torch.int32, device=device)
        return status

    def _sigma(self, sigma, n):
        import torch
        if sigma.dtype != torch.complex128 or not sigma.is_cuda or not sigma.is_contiguous() \
                or tuple(sigma.shape) != (n, n):
            raise ValueError(f"sigma must be a contiguous complex128 device tensor of shape ({n}, {n})")

    def px_sigma_diagonalize(self, sigma, Q=None, d=None, status=None, stream=None):
        """sigma = Q diag(d) Q^H; returns (Q, d, status)."""
        import torch
        n = sigma.shape[0]
        self._sigma(sigma, n)
        if Q is None:
            Q = torch.empty_like(sigma)
        if d is None:
            d = torch.empty(n, dtype=torch.float64, device=sigma.device)
        status = self._status(status, sigma.device)
        _check_dev("Q", Q, torch.complex128, numel=n * n)
        _check_dev("d", d, torch.float64, at_least=n)
        _check_dev("status", status, torch.int32, at_least=1)
        cell = Cell.cubic(16, 1.0)
        self.ensure_workspace(self.workspace_bytes(PX_OP_SIGMA_DIAG, cell, PX_PREC_FP64, n))
        self._check(self.lib.px_sigma_diagonalize(self.h, n, _ptr(sigma), _ptr(Q), _ptr(d),
                                                  _ptr(status), _stream(stream)))
        return Q, d, status

    def px_exchange_apply_sigma(self, cell: Cell, phi_basis, sigma, tgt, kern, out=None, status=None,
                                stream=None):
        """Vx[Phi sigma Phi^H] applied to tgt (Eq. 10 via Eq. 11-13); returns (out, status)."""
        import torch
        prec = _prec(phi_basis.dtype)
        _check_block("phi_basis", phi_basis, cell)
        _check_block("tgt", tgt, cell, phi_basis.dtype)
        n = phi_basis.shape[0]
        self._sigma(sigma, n)
        if out is None:
            out = torch.empty_like(tgt)
        status = self._status(status, tgt.device)
        _check_block("out", out, cell, phi_basis.dtype)
        _check_inputs(cell, n, False, kern, status=status)
        self.ensure_workspace(self.workspace_bytes(PX_OP_EXCHANGE_SIGMA, cell, prec, n, tgt.shape[0]))
        self._check(self.lib.px_exchange_apply_sigma(
            self.h, ctypes.byref(cell.c()), prec, n, _ptr(phi_basis), _ptr(sigma), tgt.shape[0],
            _ptr(tgt), _ptr(kern), _ptr(out), _ptr(status), _stream(stream)))
        return out, status

    def px_density(self, cell: Cell, phi, occ, rho=None, stream=None):
        """rho(r) = sum_i occ_i |phi_i(r)|^2 (FP64, shape [n2][n1][n0])."""
        import torch
        prec = _prec(phi.dtype)
        _check_block("phi", phi, cell)
        if rho is None:
            rho = torch.empty((cell.n[2], cell.n[1], cell.n[0]), dtype=torch.float64, device=phi.device)
        _check_inputs(cell, phi.shape[0], occ, False)
        _check_dev("rho", rho, torch.float64, numel=cell.ng)
        self._check(self.lib.px_density(self.h, ctypes.byref(cell.c()), prec, phi.shape[0], _ptr(phi),
                                        _ptr(occ), _ptr(rho), _stream(stream)))
        return rho

    def px_density_fine(self, cell: Cell, phi, occ, rho=None, stream=None):
        """rho on the grid twice as fine per axis (FP64, shape [2 n2][2 n1][2 n0])."""
        import torch
        prec = _prec(phi.dtype)
        _check_block("phi", phi, cell)
        if rho is None:
            rho = torch.empty((2 * cell.n[2], 2 * cell.n[1], 2 * cell.n[0]), dtype=torch.float64,
                              device=phi.device)
        _check_inputs(cell, phi.shape[0], occ, False)
        _check_dev("rho", rho, torch.float64, numel=8 * cell.ng)
        self.ensure_workspace(self.workspace_bytes(PX_OP_DENSITY_FINE, cell, prec, phi.shape[0]))
        self._check(self.lib.px_density_fine(self.h, ctypes.byref(cell.c()), prec, phi.shape[0], _ptr(phi),
                                             _ptr(occ), _ptr(rho), _stream(stream)))
        return rho

    def px_density_sigma(self, cell: Cell, phi_basis, sigma, rho=None, status=None, stream=None):
        """rho(r) = sum_ij Phi_i sigma_ij conj(Phi_j); returns (rho, status)."""
        import torch
        prec = _prec(phi_basis.dtype)
        _check_block("phi_basis", phi_basis, cell)
        n = phi_basis.shape[0]
        self._sigma(sigma, n)
        if rho is None:
            rho = torch.empty((cell.n[2], cell.n[1], cell.n[0]), dtype=torch.float64,
                              device=phi_basis.device)
        status = self._status(status, phi_basis.device)
        _check_dev("rho", rho, torch.float64, numel=cell.ng)
        _check_dev("status", status, torch.int32, at_least=1)
        self.ensure_workspace(self.workspace_bytes(PX_OP_DENSITY_SIGMA, cell, prec, n))
        self._check(self.lib.px_density_sigma(self.h, ctypes.byref(cell.c()), prec, n, _ptr(phi_basis),
                                              _ptr(sigma), _ptr(rho), _ptr(status), _stream(stream)))
        return rho, status

    def px_rotate_orbitals(self, cell: Cell, phi_basis, Q, out=None, stream=None):
        """phi = Phi Q (orbital b = sum_a Q[a][b] Phi_a)."""
        import torch
        prec = _prec(phi_basis.dtype)
        _check_block("phi_basis", phi_basis, cell)
        n = phi_basis.shape[0]
        self._sigma(Q, n)
        if out is None:
            out = torch.empty_like(phi_basis)
        _check_block("out", out, cell, phi_basis.dtype)
        self.ensure_workspace(self.workspace_bytes(PX_OP_ROTATE, cell, prec, n))
        self._check(self.lib.px_rotate_orbitals(self.h, ctypes.byref(cell.c()), prec, n, _ptr(phi_basis),
                                                _ptr(Q), _ptr(out), _stream(stream)))
        return out

    def px_ace_build_sigma(self, cell: Cell, phi_basis, sigma, kern, xi=None, M=None, e_x=None,
                           status=None, stream=None):
        """ACE operator of Vx[Phi sigma Phi^H] (Eq. 14 on (Phi Q, d)); returns
        (xi, status [2]: diagonalisation, Cholesky)."""
        import torch
        prec = _prec(phi_basis.dtype)
        _check_block("phi_basis", phi_basis, cell)
        n = phi_basis.shape[0]
        self._sigma(sigma, n)
        if xi is None:
            xi = torch.empty_like(phi_basis)
        if status is None:
            status = torch.zeros(2, dtype=torch.int32, device=phi_basis.device)
        elif status.numel() < 2 or status.dtype != torch.int32:
            raise ValueError("status must hold two int32 words")
        _check_block("xi", xi, cell, phi_basis.dtype)
        _check_inputs(cell, n, False, kern, e_x, M, status, nstatus=2)
        self.ensure_workspace(self.workspace_bytes(PX_OP_ACE_BUILD_SIGMA, cell, prec, n))
        self._check(self.lib.px_ace_build_sigma(
            self.h, ctypes.byref(cell.c()), prec, n, _ptr(phi_basis), _ptr(sigma), _ptr(kern),
            _ptr(xi), _ptr(M), _ptr(e_x), _ptr(status), _stream(stream)))
        return xi, status

    def px_ptim_step(self, cell: Cell, xi, phi_n, sigma_n, n_iter: int, dt_alpha: float,
                     phi_out=None, sigma_out=None, residuals=None, status=None, stream=None):
        """Exchange-only PT-IM step with projector and sigma; returns
        (phi_out, sigma_out, residuals [2][n_iter], status)."""
        import torch
        prec = _prec(xi.dtype)
        _check_block("xi", xi, cell)
        _check_block("phi_n", phi_n, cell, xi.dtype)
        m = phi_n.shape[0]
        self._sigma(sigma_n, m)
        if phi_out is None:
            phi_out = torch.empty_like(phi_n)
        if sigma_out is None:
            sigma_out = torch.empty_like(sigma_n)
        if residuals is None:
            residuals = torch.zeros((2, n_iter), dtype=torch.float64, device=phi_n.device)
        status = self._status(status, phi_n.device)
        _check_block("phi_out", phi_out, cell, xi.dtype)
        _check_dev("sigma_out", sigma_out, torch.complex128, numel=m * m)
        _check_dev("residuals", residuals, torch.float64, at_least=2 * max(int(n_iter), 0))
        _check_dev("status", status, torch.int32, at_least=1)
        self.ensure_workspace(self.workspace_bytes(PX_OP_PTIM_STEP, cell, prec, xi.shape[0], m))
        self._check(self.lib.px_ptim_step(
            self.h, ctypes.byref(cell.c()), prec, xi.shape[0], _ptr(xi), m, _ptr(phi_n), _ptr(sigma_n),
            int(n_iter), float(dt_alpha), _ptr(phi_out), _ptr(sigma_out), _ptr(residuals), _ptr(status),
            _stream(stream)))
        return phi_out, sigma_out, residuals, status

    def px_set_profiling(self, enable: bool):
        self._check(self.lib.px_set_profiling(self.h, 1 if enable else 0))

    def px_set_symmetry(self, enable: bool):
        self._check(self.lib.px_set_symmetry(self.h, 1 if enable else 0))

    def px_profile_read(self, reset: bool = False):
        """Per pass (1, 2, 3, 4): dict(ms=total event ms, bytes=algorithmic bytes, launches=n)."""
        ms = (ctypes.c_double * 4)()
        by = (ctypes.c_double * 4)()
        la = (ctypes.c_int64 * 4)()
        self._check(self.lib.px_profile_read(self.h, ms, by, la, 1 if reset else 0))
        return [dict(ms=ms[k], bytes=by[k], launches=la[k]) for k in range(4)]

    def px_profile_read_ace(self, reset: bool = False):
        """ACE build stages while profiling: dict(M=ms, factor=ms, xi=ms, build=ms of the
        whole builds, calls=n)."""
        ms = (ctypes.c_double * 4)()
        calls = ctypes.c_int64()
        self._check(self.lib.px_profile_read_ace(self.h, ms, ctypes.byref(calls), 1 if reset else 0))
        return dict(M=ms[0], factor=ms[1], xi=ms[2], build=ms[3], calls=calls.value)

    def px_exchange_apply_batched(self, instances, ace=False, stream=None):
        """instances: list of dicts with cell (Cell), psi, occ, kern and optional
        out, e_x, M, status (torch device tensors).  Returns the list of outputs
        (Vx psi, or xi with ace=True) and the status tensors (ace)."""
        import torch
        if not instances:
            raise ValueError("need at least one instance")
        prec = _prec(instances[0]["psi"].dtype)
        arr = (PxInstance * len(instances))()
        outs, stats = [], []
        for k, d in enumerate(instances):
            cell, psi = d["cell"], d["psi"]
            _check_block(f"instances[{k}].psi", psi, cell, instances[0]["psi"].dtype)
            out = d.get("out")
            if out is None:
                out = torch.empty_like(psi)
            st = d.get("status")
            if ace and st is None:
                st = torch.zeros(1, dtype=torch.int32, device=psi.device)
            _check_block(f"instances[{k}].out", out, cell, psi.dtype)
            _check_inputs(cell, psi.shape[0], d.get("occ"), d.get("kern"), d.get("e_x"), d.get("M"), st)
            outs.append(out)
            stats.append(st)
            arr[k] = PxInstance(cell.c(), psi.shape[0], psi.data_ptr(), d["occ"].data_ptr(),
                                d["kern"].data_ptr(), out.data_ptr(),
                                d["e_x"].data_ptr() if d.get("e_x") is not None else None,
                                d["M"].data_ptr() if d.get("M") is not None else None,
                                st.data_ptr() if st is not None else None)
        need = int(self.lib.px_workspace_bytes_batched(self.h, len(instances), arr, prec, int(ace)))
        self.ensure_workspace(need)
        self._check(self.lib.px_exchange_apply_batched(self.h, len(instances), arr, prec, int(ace),
                                                       _stream(stream)))
        return outs, stats

    def px_set_graph(self, enable: bool):
        self._check(self.lib.px_set_graph(self.h, 1 if enable else 0))

    def px_set_batch_capacity(self, nbytes: int):
        self._check(self.lib.px_set_batch_capacity(self.h, int(nbytes)))

    def px_autotune(self, cell: Cell, psi, occ, kern, out=None, cache_path=None, stream=None):
        """Returns the fastest square pair block for this grid and precision
        (also applied to the context)."""
        import torch
        prec = _prec(psi.dtype)
        _check_block("psi", psi, cell)
        if out is None:
            out = torch.empty_like(psi)
        _check_block("out", out, cell, psi.dtype)
        _check_inputs(cell, psi.shape[0], occ, kern)
        need = max(self.workspace_bytes(PX_OP_EXCHANGE, cell, prec, psi.shape[0], psi.shape[0]), 1)
        # room for the largest candidate block (256 x 256 pair slabs, or as
        # many as 64 GiB hold; larger candidates are skipped)
        b = psi.element_size()
        blk = min(256, psi.shape[0])
        need = max(need, min(blk * blk * cell.ng * b, 64 << 30) + (256 << 20))
        self.ensure_workspace(need)
        best = ctypes.c_int32(0)
        self._check(self.lib.px_autotune(self.h, ctypes.byref(cell.c()), prec, psi.shape[0],
                                         _ptr(psi), _ptr(occ), _ptr(kern), _ptr(out),
                                         cache_path.encode() if cache_path else None,
                                         ctypes.byref(best), _stream(stream)))
        return best.value

    def px_load_tuning(self, path: str) -> int:
        n = ctypes.c_int32(0)
        self._check(self.lib.px_load_tuning(self.h, path.encode(), ctypes.byref(n)))
        return n.value

    def px_sync(self, stream=None):
        """Raises PxError(PX_ERR_NOT_POSITIVE_DEFINITE) after a failed ACE build."""
        self._check(self.lib.px_sync(self.h, _stream(stream)))

    def px_clear_error(self):
        self.lib.px_clear_error(self.h)
