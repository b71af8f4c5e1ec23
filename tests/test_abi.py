"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/px.h, and rejects bad arguments before enqueuing work."""
import ctypes
import os
import re

import pytest

from paper_2501_03061_amd import px

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "px.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(px_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return px.load_library()


def test_header_declares_the_three_entry_points():
    names = _declared_functions()
    for n in ("px_exchange_apply", "px_ace_build", "px_ace_apply"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert names, "no declarations parsed"
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding marshals exactly the declared set
    assert sorted(px.SIGNATURES) == names


def test_abi_version(lib):
    assert lib.px_abi_version() == 1


@pytest.fixture()
def ctx(lib):
    h = ctypes.c_void_p()
    assert lib.px_create(0, ctypes.byref(h)) == px.PX_OK
    yield h
    lib.px_destroy(h)


def _cell(n=24, L=10.0):
    return px.Cell.cubic(n, L).c()


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first


def test_grid_support(lib):
    for n in (16, 24, 32, 40, 48, 60, 64, 72, 80, 96):
        assert lib.px_grid_supported(ctypes.byref(_cell(n)), 0) == 1
    for n in (7, 11, 25, 100):
        assert lib.px_grid_supported(ctypes.byref(_cell(n)), 0) == 0
    noncubic = px.Cell((1.0, 1.0, 1.0), (24, 24, 32)).c()
    assert lib.px_grid_supported(ctypes.byref(noncubic), 0) == 0
    # the non-cubic grids with compiled pipelines (x, y, z), and not their transposes
    for n in ((60, 60, 90), (60, 90, 120)):
        assert lib.px_grid_supported(ctypes.byref(px.Cell((1.0, 1.0, 1.0), n).c()), 0) == 1
    for n in ((90, 60, 60), (120, 90, 60), (60, 120, 90)):
        assert lib.px_grid_supported(ctypes.byref(px.Cell((1.0, 1.0, 1.0), n).c()), 0) == 0


def test_create_rejects_negative_device(lib):
    h = ctypes.c_void_p()
    assert lib.px_create(-1, ctypes.byref(h)) == px.PX_ERR_INVALID_ARG


def _exchange(lib, ctx, cell, n_psi=4, n_phi=4, psi=FAKE, occ=FAKE, phi=FAKE, kern=FAKE,
              out=ctypes.c_void_p(0x2000), e_x=None, prec=0):
    return lib.px_exchange_apply(ctx, ctypes.byref(cell), prec, n_psi, psi, occ, n_phi, phi,
                                 kern, out, e_x, None)


def test_exchange_validation(lib, ctx):
    c = _cell()
    assert _exchange(lib, ctx, c, psi=None) == px.PX_ERR_INVALID_ARG
    assert _exchange(lib, ctx, c, n_psi=0) == px.PX_ERR_INVALID_ARG
    assert _exchange(lib, ctx, c, n_phi=-3) == px.PX_ERR_INVALID_ARG
    assert _exchange(lib, ctx, c, prec=7) == px.PX_ERR_INVALID_ARG
    assert _exchange(lib, ctx, c, out=FAKE) == px.PX_ERR_INVALID_ARG        # aliases psi
    assert _exchange(lib, ctx, _cell(7)) == px.PX_ERR_UNSUPPORTED_GRID
    bad = px.Cell((10.0, -1.0, 10.0), (24, 24, 24)).c()
    assert _exchange(lib, ctx, bad) == px.PX_ERR_INVALID_ARG
    # energy needs phi == psi and equal counts
    ex = ctypes.c_void_p(0x3000)
    assert _exchange(lib, ctx, c, phi=ctypes.c_void_p(0x4000), e_x=ex) == px.PX_ERR_INVALID_ARG
    assert _exchange(lib, ctx, c, n_phi=3, e_x=ex) == px.PX_ERR_INVALID_ARG
    # orbital blocks are read with 16-byte vector loads
    assert _exchange(lib, ctx, c, psi=ctypes.c_void_p(0x1008), phi=ctypes.c_void_p(0x1008)) == px.PX_ERR_INVALID_ARG
    assert _exchange(lib, ctx, c, out=ctypes.c_void_p(0x2008)) == px.PX_ERR_INVALID_ARG
    # no workspace attached
    assert _exchange(lib, ctx, c) == px.PX_ERR_WORKSPACE
    assert b"workspace" in lib.px_last_error(ctx)


def test_workspace_sizes(lib, ctx):
    c = _cell(72, 20.0)
    ng = 72 ** 3
    b64 = lib.px_workspace_bytes(ctx, px.PX_OP_EXCHANGE, ctypes.byref(c), 0, 512, 512)
    b32 = lib.px_workspace_bytes(ctx, px.PX_OP_EXCHANGE, ctypes.byref(c), 1, 512, 512)
    # default chunk: 32 x 16 pair slabs dominate
    assert b64 >= 256 * ng * 16 and b32 >= 256 * ng * 8 and b32 < b64
    ace = lib.px_workspace_bytes(ctx, px.PX_OP_ACE_BUILD, ctypes.byref(c), 0, 512, 0)
    assert ace >= b64 + 512 * ng * 16             # plus W
    assert lib.px_workspace_bytes(ctx, px.PX_OP_EXCHANGE, ctypes.byref(c), 0, 0, 4) == 0
    # tuning changes the chunk
    assert lib.px_set_tuning(ctx, ctypes.byref(c), 0, 8, 4) == px.PX_OK
    small = lib.px_workspace_bytes(ctx, px.PX_OP_EXCHANGE, ctypes.byref(c), 0, 512, 512)
    assert small < b64
    assert lib.px_set_tuning(ctx, ctypes.byref(c), 0, 0, 0) == px.PX_OK
    assert lib.px_workspace_bytes(ctx, px.PX_OP_EXCHANGE, ctypes.byref(c), 0, 512, 512) == b64
    assert lib.px_set_tuning(ctx, ctypes.byref(c), 0, -1, 4) == px.PX_ERR_INVALID_ARG


def test_set_workspace_alignment(lib, ctx):
    assert lib.px_set_workspace(ctx, ctypes.c_void_p(0x1001), 1024) == px.PX_ERR_INVALID_ARG
    assert lib.px_set_workspace(ctx, ctypes.c_void_p(0x10000), 1024) == px.PX_OK


def test_ace_validation(lib, ctx):
    c = _cell()
    st = ctypes.c_void_p(0x5000)
    f = lib.px_ace_build
    assert f(ctx, ctypes.byref(c), 0, 0, FAKE, FAKE, FAKE, ctypes.c_void_p(0x6000), None, None, st, None) == px.PX_ERR_INVALID_ARG
    assert f(ctx, ctypes.byref(c), 0, 4, FAKE, FAKE, FAKE, ctypes.c_void_p(0x6000), None, None, None, None) == px.PX_ERR_INVALID_ARG
    assert f(ctx, ctypes.byref(c), 0, 4, FAKE, FAKE, FAKE, FAKE, None, None, st, None) == px.PX_ERR_INVALID_ARG
    assert f(ctx, ctypes.byref(_cell(7)), 0, 4, FAKE, FAKE, FAKE, ctypes.c_void_p(0x6000), None, None, st, None) == px.PX_ERR_UNSUPPORTED_GRID
    assert f(ctx, ctypes.byref(c), 0, 4, FAKE, FAKE, FAKE, ctypes.c_void_p(0x6000), None, None, st, None) == px.PX_ERR_WORKSPACE
    g = lib.px_ace_apply
    assert g(ctx, ctypes.byref(c), 0, 4, FAKE, 2, ctypes.c_void_p(0x7000), ctypes.c_void_p(0x7000), None) == px.PX_ERR_INVALID_ARG
    assert g(ctx, ctypes.byref(c), 0, 4, None, 2, ctypes.c_void_p(0x7000), ctypes.c_void_p(0x8000), None) == px.PX_ERR_INVALID_ARG
    assert g(ctx, ctypes.byref(c), 0, 4, FAKE, 2, ctypes.c_void_p(0x7008), ctypes.c_void_p(0x8000), None) == px.PX_ERR_INVALID_ARG
    assert f(ctx, ctypes.byref(c), 1, 4, ctypes.c_void_p(0x1008), FAKE, FAKE, ctypes.c_void_p(0x6000), None, None, st, None) == px.PX_ERR_INVALID_ARG
    assert g(ctx, ctypes.byref(c), 0, 4, FAKE, 2, ctypes.c_void_p(0x7000), ctypes.c_void_p(0x8000), None) == px.PX_ERR_WORKSPACE


def test_contraction_entry_points_reject_odd_grids_in_fp32(lib, ctx):
    """ACE application and the PT-IM-style loop read FP32 blocks two complex64
    values per 16-byte load: an odd N_g would misalign every second orbital and
    let a load straddle two orbitals, so such grids are refused (FP64 is fine)."""
    odd = px.Cell((5.0, 5.0, 5.0), (5, 5, 5)).c()      # N_g = 125
    even = px.Cell((5.0, 5.0, 5.0), (6, 5, 5)).c()     # N_g = 150: no FFT plan, but contractions work
    g = lib.px_ace_apply
    a, b, o = FAKE, ctypes.c_void_p(0x7000), ctypes.c_void_p(0x8000)
    assert g(ctx, ctypes.byref(odd), 1, 4, a, 2, b, o, None) == px.PX_ERR_UNSUPPORTED_GRID
    assert g(ctx, ctypes.byref(odd), 0, 4, a, 2, b, o, None) == px.PX_ERR_WORKSPACE
    assert g(ctx, ctypes.byref(even), 1, 4, a, 2, b, o, None) == px.PX_ERR_WORKSPACE
    h = lib.px_ptim_exchange_loop
    res = ctypes.c_void_p(0x9000)
    assert h(ctx, ctypes.byref(odd), 1, 4, a, 2, b, 3, 0.5, o, res, None) == px.PX_ERR_UNSUPPORTED_GRID
    assert h(ctx, ctypes.byref(odd), 0, 4, a, 2, b, 3, 0.5, o, res, None) == px.PX_ERR_WORKSPACE
    wb = lib.px_workspace_bytes
    assert wb(ctx, px.PX_OP_ACE_APPLY, ctypes.byref(odd), 1, 4, 2) == 0
    assert wb(ctx, px.PX_OP_PTIM_LOOP, ctypes.byref(odd), 1, 4, 2) == 0
    assert wb(ctx, px.PX_OP_ACE_APPLY, ctypes.byref(odd), 0, 4, 2) > 0
    assert wb(ctx, px.PX_OP_ACE_APPLY, ctypes.byref(even), 1, 4, 2) > 0
    # the FFT entry points need a compiled plan
    assert wb(ctx, px.PX_OP_EXCHANGE, ctypes.byref(even), 0, 4, 2) == 0
    assert wb(ctx, px.PX_OP_ACE_BUILD, ctypes.byref(even), 0, 4, 0) == 0


def test_kernel_and_convert_validation(lib, ctx):
    c = _cell()
    assert lib.px_kernel_hse(ctx, ctypes.byref(c), 0.0, FAKE, None) == px.PX_ERR_INVALID_ARG
    assert lib.px_kernel_hse(ctx, ctypes.byref(c), 0.106, None, None) == px.PX_ERR_INVALID_ARG
    assert lib.px_convert_c128_to_c64(ctx, 10, None, FAKE, None) == px.PX_ERR_INVALID_ARG
    assert lib.px_convert_c128_to_c64(ctx, 10, ctypes.c_void_p(0x1010), ctypes.c_void_p(0x2000), None) == px.PX_ERR_INVALID_ARG


def _inst(n=24, n_orb=4, psi=FAKE, out=ctypes.c_void_p(0x9000), status=None):
    return px.PxInstance(px.Cell.cubic(n, 10.0).c(), n_orb, psi, FAKE, FAKE, out, None, None, status)


def test_batched_validation(lib, ctx):
    arr = (px.PxInstance * 2)(_inst(), _inst(32))
    f = lib.px_exchange_apply_batched
    assert f(ctx, 0, arr, 0, 0, None) == px.PX_ERR_INVALID_ARG
    assert f(ctx, 2, None, 0, 0, None) == px.PX_ERR_INVALID_ARG
    assert f(ctx, 2, arr, 5, 0, None) == px.PX_ERR_INVALID_ARG
    bad = (px.PxInstance * 2)(_inst(), _inst(7))
    assert f(ctx, 2, bad, 0, 0, None) == px.PX_ERR_UNSUPPORTED_GRID
    alias = (px.PxInstance * 1)(_inst(out=FAKE))
    assert f(ctx, 1, alias, 0, 0, None) == px.PX_ERR_INVALID_ARG
    # ACE mode needs a status word per instance
    assert f(ctx, 2, arr, 0, 1, None) == px.PX_ERR_INVALID_ARG
    assert f(ctx, 2, arr, 0, 0, None) == px.PX_ERR_WORKSPACE
    need = lib.px_workspace_bytes_batched(ctx, 2, arr, 0, 0)
    assert need > 0
    assert lib.px_workspace_bytes_batched(ctx, 2, bad, 0, 0) == 0
    with_ace = (px.PxInstance * 2)(_inst(status=FAKE), _inst(32, status=FAKE))
    assert lib.px_workspace_bytes_batched(ctx, 2, with_ace, 0, 1) > need


def test_load_tuning_cache(lib, ctx, tmp_path):
    """The cache lines written by the autotuner set the context's pair block."""
    c = _cell(72, 20.0)
    base = lib.px_workspace_bytes(ctx, px.PX_OP_EXCHANGE, ctypes.byref(c), 1, 512, 512)
    path = tmp_path / "tune.jsonl"
    path.write_text(
        '{"arch": "gfx950", "n": [72, 72, 72], "prec": "fp32", "n_orb": 512, "block": 8, "us_per_pair": 1.0}\n'
        'not json at all\n'
        '{"arch": "gfx950", "n": [48, 48, 48], "prec": "fp64", "n_orb": 100, "block": 16, "us_per_pair": 2.0}\n')
    n = ctypes.c_int32(0)
    assert lib.px_load_tuning(ctx, str(path).encode(), ctypes.byref(n)) == px.PX_OK
    assert n.value == 2
    tuned = lib.px_workspace_bytes(ctx, px.PX_OP_EXCHANGE, ctypes.byref(c), 1, 512, 512)
    assert tuned < base                       # 8 x 8 pair block instead of the default
    assert lib.px_load_tuning(ctx, b"/nonexistent/file", None) == px.PX_ERR_INVALID_ARG
    # the pass-2 configuration of a line: at 96^3 the default has two x-sections per
    # plane (twice the energy-partial slots of configuration 1)
    c96 = _cell(96, 27.0)
    path.write_text('{"n": [96, 96, 96], "prec": "fp32", "block": 32, "p2": 0}\n')
    assert lib.px_load_tuning(ctx, str(path).encode(), None) == px.PX_OK
    w0 = lib.px_workspace_bytes(ctx, px.PX_OP_EXCHANGE, ctypes.byref(c96), 1, 64, 64)
    path.write_text('{"n": [96, 96, 96], "prec": "fp32", "block": 32, "p2": 1}\n')
    assert lib.px_load_tuning(ctx, str(path).encode(), None) == px.PX_OK
    w1 = lib.px_workspace_bytes(ctx, px.PX_OP_EXCHANGE, ctypes.byref(c96), 1, 64, 64)
    assert w1 < w0
    # px_set_tuning keeps the configuration
    assert lib.px_set_tuning(ctx, ctypes.byref(c96), 1, 32, 32) == px.PX_OK
    assert lib.px_workspace_bytes(ctx, px.PX_OP_EXCHANGE, ctypes.byref(c96), 1, 64, 64) == w1


def test_sigma_and_density_validation(lib, ctx):
    c = _cell()
    st = ctypes.c_void_p(0x5000)
    S, Q, d = ctypes.c_void_p(0x6000), ctypes.c_void_p(0x7000), ctypes.c_void_p(0x8000)
    f = lib.px_sigma_diagonalize
    assert f(ctx, 0, S, Q, d, st, None) == px.PX_ERR_INVALID_ARG
    assert f(ctx, 4, S, S, d, st, None) == px.PX_ERR_INVALID_ARG        # Q aliases sigma
    assert f(ctx, 4, S, Q, d, None, None) == px.PX_ERR_INVALID_ARG      # status required
    assert f(ctx, 4, ctypes.c_void_p(0x6008), Q, d, st, None) == px.PX_ERR_INVALID_ARG
    assert f(ctx, 4, S, Q, d, st, None) == px.PX_ERR_WORKSPACE
    g = lib.px_exchange_apply_sigma
    phi, tgt, kern, out = ctypes.c_void_p(0x9000), ctypes.c_void_p(0xa000), FAKE, ctypes.c_void_p(0xb000)
    assert g(ctx, ctypes.byref(c), 0, 4, phi, S, 2, tgt, kern, out, st, None) == px.PX_ERR_WORKSPACE
    assert g(ctx, ctypes.byref(c), 0, 4, phi, S, 2, tgt, kern, phi, st, None) == px.PX_ERR_INVALID_ARG
    assert g(ctx, ctypes.byref(c), 0, 4, phi, S, 2, tgt, kern, out, None, None) == px.PX_ERR_INVALID_ARG
    assert g(ctx, ctypes.byref(_cell(7)), 0, 4, phi, S, 2, tgt, kern, out, st, None) == px.PX_ERR_UNSUPPORTED_GRID
    assert g(ctx, ctypes.byref(c), 0, 0, phi, S, 2, tgt, kern, out, st, None) == px.PX_ERR_INVALID_ARG
    h = lib.px_density
    rho = ctypes.c_void_p(0xc000)
    assert h(ctx, ctypes.byref(c), 0, 0, phi, d, rho, None) == px.PX_ERR_INVALID_ARG
    assert h(ctx, ctypes.byref(c), 0, 4, None, d, rho, None) == px.PX_ERR_INVALID_ARG
    assert h(ctx, ctypes.byref(c), 0, 4, phi, d, ctypes.c_void_p(0xc004), None) == px.PX_ERR_INVALID_ARG
    odd = px.Cell((5.0, 5.0, 5.0), (5, 5, 5)).c()
    assert h(ctx, ctypes.byref(odd), 1, 4, phi, d, rho, None) == px.PX_ERR_UNSUPPORTED_GRID
    k = lib.px_density_sigma
    assert k(ctx, ctypes.byref(c), 0, 4, phi, S, rho, st, None) == px.PX_ERR_WORKSPACE
    assert k(ctx, ctypes.byref(c), 0, 4, phi, S, rho, None, None) == px.PX_ERR_INVALID_ARG
    wb = lib.px_workspace_bytes
    assert wb(ctx, px.PX_OP_SIGMA_DIAG, ctypes.byref(c), 0, 64, 0) >= 2 * 64 * 64 * 16
    ws = wb(ctx, px.PX_OP_EXCHANGE_SIGMA, ctypes.byref(c), 1, 16, 5)
    assert ws >= 16 * 24 ** 3 * 8 + 2 * 16 * 16 * 16    # phi = Phi Q plus the Jacobi arrays
    assert wb(ctx, px.PX_OP_EXCHANGE_SIGMA, ctypes.byref(_cell(7)), 0, 16, 5) == 0
    assert wb(ctx, px.PX_OP_DENSITY_SIGMA, ctypes.byref(c), 0, 16, 0) >= 16 * 24 ** 3 * 16


def test_ptim_step_validation(lib, ctx):
    c = _cell()
    f = lib.px_ptim_step
    xi, p, s, po, so = (ctypes.c_void_p(a) for a in (0x1000, 0x2000, 0x3000, 0x4000, 0x5000))
    res, st = ctypes.c_void_p(0x6000), ctypes.c_void_p(0x7000)

    def call(n=4, n_phi=3, n_iter=2, **kw):
        a = dict(xi=xi, p=p, s=s, po=po, so=so, res=res, st=st)
        a.update(kw)
        return f(ctx, ctypes.byref(c), 0, n, a["xi"], n_phi, a["p"], a["s"], n_iter, 0.5, a["po"], a["so"],
                 a["res"], a["st"], None)
    assert call(n_iter=0) == px.PX_ERR_INVALID_ARG
    assert call(n_iter=65) == px.PX_ERR_INVALID_ARG
    assert call(n_phi=0) == px.PX_ERR_INVALID_ARG
    assert call(st=None) == px.PX_ERR_INVALID_ARG
    assert call(po=p) == px.PX_ERR_INVALID_ARG
    assert call(so=s) == px.PX_ERR_INVALID_ARG
    assert call(s=ctypes.c_void_p(0x3008)) == px.PX_ERR_INVALID_ARG
    assert call() == px.PX_ERR_WORKSPACE
    wb = lib.px_workspace_bytes
    assert wb(ctx, px.PX_OP_PTIM_STEP, ctypes.byref(c), 1, 16, 8) >= 5 * 8 * 24 ** 3 * 8
    assert wb(ctx, px.PX_OP_PTIM_STEP, ctypes.byref(c), 1, 16, 0) == 0


def test_ace_build_sigma_validation(lib, ctx):
    c = _cell()
    f = lib.px_ace_build_sigma
    phi, s, kern, xi, st = (ctypes.c_void_p(a) for a in (0x1000, 0x2000, 0x3000, 0x4000, 0x5000))

    def call(n=4, cell=c, **kw):
        a = dict(phi=phi, s=s, kern=kern, xi=xi, st=st)
        a.update(kw)
        return f(ctx, ctypes.byref(cell), 0, n, a["phi"], a["s"], a["kern"], a["xi"], None, None,
                 a["st"], None)
    assert call(n=0) == px.PX_ERR_INVALID_ARG
    assert call(st=None) == px.PX_ERR_INVALID_ARG
    assert call(kern=None) == px.PX_ERR_INVALID_ARG
    assert call(xi=phi) == px.PX_ERR_INVALID_ARG                  # xi aliases Phi
    assert call(s=ctypes.c_void_p(0x2008)) == px.PX_ERR_INVALID_ARG  # sigma misaligned
    assert call(cell=_cell(7)) == px.PX_ERR_UNSUPPORTED_GRID
    assert call() == px.PX_ERR_WORKSPACE
    wb = lib.px_workspace_bytes
    ace = wb(ctx, px.PX_OP_ACE_BUILD, ctypes.byref(c), 1, 16, 0)
    # the ACE build's workspace plus phi = Phi Q, Q and the Jacobi arrays
    assert wb(ctx, px.PX_OP_ACE_BUILD_SIGMA, ctypes.byref(c), 1, 16, 0) >= ace + 16 * 24 ** 3 * 8 + 16 * 16 * 16
    assert wb(ctx, px.PX_OP_ACE_BUILD_SIGMA, ctypes.byref(_cell(7)), 1, 16, 0) == 0


def test_rotate_orbitals_validation(lib, ctx):
    c = _cell()
    f = lib.px_rotate_orbitals
    phi, Q, out = (ctypes.c_void_p(a) for a in (0x1000, 0x2000, 0x3000))
    assert f(ctx, ctypes.byref(c), 1, 0, phi, Q, out, None) == px.PX_ERR_INVALID_ARG
    assert f(ctx, ctypes.byref(c), 1, 4, phi, None, out, None) == px.PX_ERR_INVALID_ARG
    assert f(ctx, ctypes.byref(c), 1, 4, phi, Q, phi, None) == px.PX_ERR_INVALID_ARG      # aliasing
    assert f(ctx, ctypes.byref(c), 1, 4, phi, ctypes.c_void_p(0x2008), out, None) == px.PX_ERR_INVALID_ARG
    odd = px.Cell((5.0, 5.0, 5.0), (5, 5, 5)).c()
    assert f(ctx, ctypes.byref(odd), 1, 4, phi, Q, out, None) == px.PX_ERR_UNSUPPORTED_GRID
    assert f(ctx, ctypes.byref(c), 1, 4, phi, Q, out, None) == px.PX_ERR_WORKSPACE         # FP32: Q in complex64
    assert lib.px_workspace_bytes(ctx, px.PX_OP_ROTATE, ctypes.byref(c), 1, 16, 0) >= 16 * 16 * 8


def test_density_fine_validation(lib, ctx):
    c = _cell()
    f = lib.px_density_fine
    phi, occ, rho = (ctypes.c_void_p(a) for a in (0x1000, 0x2000, 0x3000))
    assert f(ctx, ctypes.byref(c), 1, 0, phi, occ, rho, None) == px.PX_ERR_INVALID_ARG
    assert f(ctx, ctypes.byref(c), 1, 4, phi, None, rho, None) == px.PX_ERR_INVALID_ARG
    assert f(ctx, ctypes.byref(c), 1, 4, phi, occ, ctypes.c_void_p(0x3004), None) == px.PX_ERR_INVALID_ARG
    odd = px.Cell((5.0, 5.0, 5.0), (6, 6, 5)).c()
    assert f(ctx, ctypes.byref(odd), 1, 4, phi, occ, rho, None) == px.PX_ERR_UNSUPPORTED_GRID
    big = px.Cell((5.0, 5.0, 5.0), (8, 128, 8)).c()
    assert f(ctx, ctypes.byref(big), 1, 4, phi, occ, rho, None) == px.PX_ERR_UNSUPPORTED_GRID
    assert f(ctx, ctypes.byref(c), 1, 4, phi, occ, rho, None) == px.PX_ERR_WORKSPACE
    wb = lib.px_workspace_bytes
    assert wb(ctx, px.PX_OP_DENSITY_FINE, ctypes.byref(c), 1, 4, 0) >= 10 * 24 ** 3 * 8 * 16
    assert wb(ctx, px.PX_OP_DENSITY_FINE, ctypes.byref(odd), 0, 4, 0) == 0


class _DevTensor:
    """Stands in for a device tensor in the binding's argument checks (no GPU here)."""

    def __init__(self, dtype, numel, cuda=True, contiguous=True):
        self.dtype, self._n, self.is_cuda, self._c = dtype, numel, cuda, contiguous

    def numel(self):
        return self._n

    def is_contiguous(self):
        return self._c


def test_binding_rejects_host_and_mis_sized_arguments():
    import torch
    cell = px.Cell.cubic(24, 10.0)
    ok = dict(occ=_DevTensor(torch.float64, 4), kern=_DevTensor(torch.float64, cell.ng))
    px._check_inputs(cell, 4, **ok)
    px._check_inputs(cell, 4, **ok, e_x=None, M=None, status=None)
    with pytest.raises(ValueError, match="device tensor"):      # a host array would fault the GPU
        px._check_inputs(cell, 4, occ=torch.ones(4, dtype=torch.float64), kern=ok["kern"])
    with pytest.raises(ValueError, match="required"):
        px._check_inputs(cell, 4, occ=None, kern=ok["kern"])
    with pytest.raises(TypeError):
        px._check_inputs(cell, 4, occ=_DevTensor(torch.float32, 4), kern=ok["kern"])
    with pytest.raises(ValueError, match="at least 4"):
        px._check_inputs(cell, 4, occ=_DevTensor(torch.float64, 3), kern=ok["kern"])
    with pytest.raises(ValueError, match=f"{cell.ng} elements"):
        px._check_inputs(cell, 4, occ=ok["occ"], kern=_DevTensor(torch.float64, cell.ng - 1))
    with pytest.raises(ValueError, match="16 elements"):
        px._check_inputs(cell, 4, **ok, M=_DevTensor(torch.complex128, 15))
    with pytest.raises(ValueError, match="at least 2"):
        px._check_inputs(cell, 4, **ok, status=_DevTensor(torch.int32, 1), nstatus=2)
    with pytest.raises(ValueError, match="contiguous"):
        px._check_dev("rho", _DevTensor(torch.float64, cell.ng, contiguous=False), torch.float64)
    px._check_inputs(cell, 4, False, ok["kern"])                 # occupations not taken
