"""CPU-side checks of the C ABI library: it loads, exports every declared symbol,
rejects bad arguments before touching a device, and its scalar math (compiled for
the host from the kernels' own source) agrees with the oracle."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest
import torch

from oracle import lanczos as olz
from oracle import probes as opr
from oracle import spme as osp
from oracle import tensors as otz
from paper_2307_02278_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(not os.path.exists(L.LIB_PATH),
                                reason="libmbd.so not built (run __graft_entry__.build())")


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mbdh?_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(L.LIB_PATH)
    names = _declared("mbd.h")
    assert "mbd_plan_create" in names and "mbd_execute" in names
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in L.SIGNATURES}
    assert set(names) == bound


def test_hostcheck_exports_every_declared_symbol():
    lib = C.CDLL(L.HOSTCHECK_PATH)
    names = _declared("mbd_hostcheck.h")
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == {s[0] for s in L.HOSTCHECK_SIGNATURES}


def test_status_strings_and_grid_support():
    lib = L.lib()
    assert lib.mbd_status_string(0) == b"ok"
    assert lib.mbd_status_string(L.MBD_E_GRID) == b"unsupported grid"
    for k in (8, 16, 18, 20, 24, 30, 48, 80, 96, 128):
        assert lib.mbd_grid_supported(k) == 1
    for k in (7, 14, 22, 130, 256):
        assert lib.mbd_grid_supported(k) == 0


def _args(n=4, cell=(20.0, 20.0, 20.0)):
    s = L.MbdSystem()
    s.n_atoms = n
    fake = 0x1000  # never dereferenced: validation fails (or no device) first
    s.pos = s.alpha = s.omega = s.r_vdw = fake
    for i in range(9):
        s.cell[i] = 0.0
    for a in range(3):
        s.cell[4 * a] = cell[a]
    p = L.MbdParams()
    p.damp_beta, p.damp_d, p.ewald_tau, p.real_cutoff, p.damp_tol = 0.83, 6.0, 0.2, 12.0, 0.0
    for a in range(3):
        p.grid[a] = 16
    p.spline_order, p.n_probes, p.n_steps, p.block = 6, 4, 10, 4
    p.seed, p.precision, p.reorth, p.want_forces, p.deterministic = 1, 0, 0, 0, 0
    return s, p


def _create(s, p, nsys=1):
    h = C.c_void_p()
    arr = (L.MbdSystem * nsys)(*([s] * nsys))
    code = L.lib().mbd_plan_create(C.byref(h), arr, nsys, C.byref(p), None)
    return code, h


@pytest.mark.parametrize("mutate,code", [
    (lambda s, p: setattr(p, "damp_beta", -1.0), L.MBD_E_ARG),
    (lambda s, p: setattr(p, "damp_d", 0.0), L.MBD_E_ARG),
    (lambda s, p: setattr(p, "real_cutoff", float("nan")), L.MBD_E_ARG),
    (lambda s, p: setattr(p, "spline_order", 5), L.MBD_E_ARG),
    (lambda s, p: setattr(p, "n_probes", 0), L.MBD_E_ARG),
    (lambda s, p: setattr(p, "n_steps", 0), L.MBD_E_ARG),
    (lambda s, p: setattr(p, "n_steps", 100000), L.MBD_E_ARG),
    (lambda s, p: setattr(p, "block", 3), L.MBD_E_ARG),
    (lambda s, p: setattr(p, "precision", 7), L.MBD_E_ARG),
    (lambda s, p: setattr(p, "reorth", 9), L.MBD_E_ARG),
    (lambda s, p: setattr(p, "want_forces", 2), L.MBD_E_ARG),
    (lambda s, p: (setattr(p, "want_forces", 1), setattr(p, "block", 2)), L.MBD_E_ARG),
    (lambda s, p: setattr(p, "krylov_block", 3), L.MBD_E_ARG),
    (lambda s, p: setattr(p, "krylov_block", 8), L.MBD_E_ARG),      # block 4 < 8
    (lambda s, p: (setattr(p, "krylov_block", 4), setattr(p, "n_probes", 6)), L.MBD_E_ARG),
    (lambda s, p: (setattr(p, "krylov_block", 2), setattr(p, "reorth", 2)), L.MBD_E_ARG),
    (lambda s, p: (setattr(p, "krylov_block", 4), setattr(p, "want_forces", 1)), L.MBD_E_ARG),
    (lambda s, p: (setattr(p, "krylov_block", 4), setattr(p, "n_steps", 200)), L.MBD_E_ARG),
    (lambda s, p: (setattr(p, "krylov_block", 4), setattr(s, "n_atoms", 1)), L.MBD_E_ARG),
    (lambda s, p: setattr(s, "n_atoms", 0), L.MBD_E_ARG),
    (lambda s, p: setattr(s, "pos", None), L.MBD_E_ARG),
    (lambda s, p: [s.cell.__setitem__(3 + c, s.cell[c]) for c in range(3)], L.MBD_E_CELL),
    (lambda s, p: s.cell.__setitem__(0, -3.0), L.MBD_E_CELL),
    (lambda s, p: p.grid.__setitem__(0, 14), L.MBD_E_GRID),
    (lambda s, p: p.grid.__setitem__(1, 10), L.MBD_E_GRID),  # supported but < 2p
    (lambda s, p: setattr(p, "tune", 3), L.MBD_E_ARG),
    (lambda s, p: (setattr(p, "tune", 2), setattr(p.shape, "pair_subsets", 3)), L.MBD_E_ARG),
    (lambda s, p: (setattr(p, "tune", 2), setattr(p.shape, "grid_chunk", 8)), L.MBD_E_ARG),
    (lambda s, p: (setattr(p, "tune", 2), setattr(p.shape, "grid_chunk", 3)), L.MBD_E_ARG),
    (lambda s, p: (setattr(p, "tune", 2), setattr(p.shape, "overlap", 3)), L.MBD_E_ARG),
    (lambda s, p: (setattr(p, "tune", 2), setattr(p.shape, "pair_wg_per_cu", -1)), L.MBD_E_ARG),
    (lambda s, p: (setattr(p, "tune", 2), setattr(p.shape, "gather_waves", 6)), L.MBD_E_ARG),
    (lambda s, p: (setattr(p, "tune", 2), setattr(p.shape, "spread_mode", 2)), L.MBD_E_ARG),
    (lambda s, p: (setattr(p, "tune", 2), setattr(p.shape, "pair_mode", 3)), L.MBD_E_ARG),
])
def test_invalid_arguments_fail_before_device_work(mutate, code):
    s, p = _args()
    mutate(s, p)
    got, h = _create(s, p)
    assert got == code
    assert not h.value
    assert L.lib().mbd_last_error()


def test_valid_arguments_without_gpu_report_no_device():
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    s, p = _args()
    got, h = _create(s, p)
    assert got == L.MBD_E_NODEVICE
    assert not h.value


def test_null_handles_are_rejected():
    lib = L.lib()
    assert lib.mbd_execute(None, None, None, None) == L.MBD_E_ARG
    assert lib.mbd_matvec(None, 0, None, None, 1, 15) == L.MBD_E_ARG
    assert lib.mbd_plan_destroy(None) == L.MBD_OK
    prm = L.MbdScsParams(15, 0.6, 1e-10, 100)
    assert lib.mbd_scs(None, 0, C.byref(prm), None, None, None, None, None) == L.MBD_E_ARG
    assert lib.mbd_status_string(L.MBD_E_NOCONV) == b"iterative solve did not converge"


@pytest.mark.parametrize("n", [1, 2, 5, 15, 31])
def test_hostcheck_gauss_legendre_matches_numpy(n):
    h = L.hostcheck()
    x, w = (C.c_double * n)(), (C.c_double * n)()
    h.mbdh_gauss_legendre(n, x, w)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(np.array(x[:]), xr, rtol=0, atol=1e-15)
    assert np.allclose(np.array(w[:]), wr, rtol=1e-12, atol=0)
    assert abs(sum(w[:]) - 2.0) < 1e-14


# --- kernel scalar math on the host vs the oracle ---------------------------------

def test_hostcheck_splitmix_matches_oracle():
    h = L.hostcheck()
    for seed, n in [(0, 0), (12345, 17), (2 ** 63 + 5, 10 ** 9)]:
        assert h.mbdh_splitmix(seed, n) == int(opr.splitmix64(seed, [n])[0])


@pytest.mark.parametrize("p", [4, 6, 8])
def test_hostcheck_bspline_matches_oracle(p):
    h = L.hostcheck()
    th = (C.c_double * p)()
    dth = (C.c_double * p)()
    for w in (0.0, 0.123, 0.5, 0.999999):
        assert h.mbdh_bspline(p, w, th, dth) == 0
        x = torch.tensor([w + t for t in range(p)], dtype=torch.float64)
        assert np.allclose(list(th), osp.bspline(p, x).numpy(), atol=1e-15)
        assert np.allclose(list(dth), osp.bspline_deriv(p, x).numpy(), atol=1e-14)
    assert h.mbdh_bspline(5, 0.1, th, dth) == -1


def _oracle_direct(r, tau, S, d):
    A, B = otz.radial_direct(torch.tensor([r], dtype=torch.float64), tau,
                             torch.tensor([S], dtype=torch.float64), d)
    return float(A[0]), float(B[0])


@pytest.mark.parametrize("prec,tol", [(0, 1e-13), (1, 2e-6)])
def test_hostcheck_direct_kernel_matches_oracle(prec, tol):
    h = L.hostcheck()
    A = C.c_double()
    B = C.c_double()
    tau, d = 0.2223, 6.0
    for S in (5.15, 5.98):
        for r in np.concatenate([np.linspace(1.6, 4.0, 13), np.linspace(4.0, 25.0, 40)]):
            h.mbdh_direct_kernel(prec, r * r, tau, 1.0 / S, d, C.byref(A), C.byref(B))
            Ao, Bo = _oracle_direct(r, tau, S, d)
            # compare the eigenvalues A and A - B r^2 of the 3x3 tensor; where the erfc part
            # and the damping tail cancel, the floor is 1e-3 of the bare tensor 1/r^3
            scale = max(abs(Ao), abs(Ao - Bo * r * r)) + (1e-3 / r ** 3 if prec == 1 else 0.0)
            assert abs(A.value - Ao) <= tol * scale, (r, A.value, Ao)
            assert abs((A.value - B.value * r * r) - (Ao - Bo * r * r)) <= tol * scale, r


def test_hostcheck_direct_kernel_short_range_series():
    """The single-precision short-range path (Taylor series of the erf part)."""
    h = L.hostcheck()
    A = C.c_double()
    B = C.c_double()
    tau, d, S = 0.35, 6.0, 5.5
    for r in (0.6, 1.0, 1.4):
        h.mbdh_direct_kernel(1, r * r, tau, 1.0 / S, d, C.byref(A), C.byref(B))
        Ao, Bo = _oracle_direct(r, tau, S, d)
        scale = max(abs(Ao), abs(Ao - Bo * r * r))
        assert abs(A.value - Ao) <= 2e-6 * scale
        assert abs(B.value - Bo) * r * r <= 2e-6 * scale


@pytest.mark.parametrize("n", [1, 2, 5, 17, 50])
def test_hostcheck_tridiagonal_quadrature_matches_eigh(n):
    h = L.hostcheck()
    rng = np.random.default_rng(n)
    a = rng.uniform(0.2, 0.6, n)
    b = rng.uniform(0.01, 0.1, max(n - 1, 0))
    q = C.c_double()
    tmin = C.c_double()
    ok = h.mbdh_tridiag_quadrature((C.c_double * n)(*a), (C.c_double * max(n - 1, 1))(*b), n,
                                   C.byref(q), C.byref(tmin))
    assert ok == 1
    qo, theta, _ = olz.quadrature(torch.tensor(a), torch.tensor(b))
    assert q.value == pytest.approx(float(qo), rel=1e-13)
    assert tmin.value == pytest.approx(float(theta.min()), rel=1e-12)


def test_hostcheck_tridiagonal_flags_indefinite():
    h = L.hostcheck()
    a = [0.5, -0.3, 0.4]
    b = [0.1, 0.2]
    q = C.c_double()
    tmin = C.c_double()
    h.mbdh_tridiag_quadrature((C.c_double * 3)(*a), (C.c_double * 2)(*b), 3, C.byref(q),
                              C.byref(tmin))
    assert tmin.value < 0


@pytest.mark.parametrize("p", [4, 6, 8])
def test_hostcheck_bspline_second_derivative(p):
    """M_p'' from the kernels' recursion against central differences of the oracle's M_p'."""
    h = L.hostcheck()
    th, dth, ddth = (C.c_double * p)(), (C.c_double * p)(), (C.c_double * p)()
    eps = 1e-6
    # away from the knots, where M_p''' (p = 4) jumps and central differences lose O(eps)
    for w in (0.13, 0.27, 0.5, 0.93):
        assert h.mbdh_bspline2(p, w, th, dth, ddth) == 0
        x = torch.tensor([w + t for t in range(p)], dtype=torch.float64)
        fd = (osp.bspline_deriv(p, x + eps) - osp.bspline_deriv(p, x - eps)) / (2 * eps)
        assert np.allclose(list(ddth), fd.numpy(), atol=1e-8)
        assert np.allclose(list(th), osp.bspline(p, x).numpy(), atol=1e-15)
        assert np.allclose(list(dth), osp.bspline_deriv(p, x).numpy(), atol=1e-14)


def test_hostcheck_direct_kernel_radial_derivatives():
    """A'(r)/r and B'(r)/r of the direct-space kernel against autograd of the oracle's
    radial functions."""
    h = L.hostcheck()
    A, B, dA, dB = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    tau, d = 0.2223, 6.0
    for S in (5.15, 5.98):
        for r in np.concatenate([np.linspace(1.6, 4.0, 7), np.linspace(4.0, 25.0, 15)]):
            h.mbdh_direct_kernel_grad(r * r, tau, 1.0 / S, d, C.byref(A), C.byref(B),
                                      C.byref(dA), C.byref(dB))
            rt = torch.tensor([r], dtype=torch.float64, requires_grad=True)
            Ao, Bo = otz.radial_direct(rt, tau, torch.tensor([S], dtype=torch.float64), d)
            (gA,) = torch.autograd.grad(Ao.sum(), rt, retain_graph=True)
            (gB,) = torch.autograd.grad(Bo.sum(), rt)
            sa = abs(float(gA[0])) / r + 1e-12 / r ** 4
            sb = abs(float(gB[0])) / r + 1e-12 / r ** 6
            assert dA.value == pytest.approx(float(gA[0]) / r, rel=1e-9, abs=1e-9 * sa), r
            assert dB.value == pytest.approx(float(gB[0]) / r, rel=1e-9, abs=1e-9 * sb), r


@pytest.mark.parametrize("n", [1, 2, 7, 30])
def test_hostcheck_tridiagonal_adjoint_matches_autograd(n):
    """dQ/da_k and dQ/db_k of the Gauss quadrature (tridiagonal eigenvectors plus
    Daleckii-Krein divided differences) against autograd through the oracle's eigh."""
    h = L.hostcheck()
    rng = np.random.default_rng(100 + n)
    a = rng.uniform(0.2, 0.6, n)
    b = rng.uniform(0.01, 0.1, max(n - 1, 0))
    ab, bb = (C.c_double * n)(), (C.c_double * n)()
    ok = h.mbdh_tridiag_adjoint((C.c_double * n)(*a), (C.c_double * max(n - 1, 1))(*b), n,
                                ab, bb)
    assert ok == 1
    at = torch.tensor(a, requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    q, _, _ = olz.quadrature(at, bt)
    grads = torch.autograd.grad(q, [at, bt] if n > 1 else [at])
    assert np.allclose(list(ab), grads[0].numpy(), rtol=1e-9, atol=1e-12)
    assert bb[0] == 0.0
    if n > 1:
        assert np.allclose(list(bb)[1:], grads[1].numpy(), rtol=1e-9, atol=1e-12)


def test_hostcheck_scs_kernel_matches_oracle():
    """The screening tensor of the GPU solver (host build of the same source) against the
    oracle's (1 - f) T_GG, on both sides of the 7-sigma switch to the bare tensor."""
    from oracle import scs as osc
    h = L.hostcheck()
    for r, sig2, S, d in [(2.0, 1.7, 5.0, 6.0), (4.5, 2.9, 5.4, 6.0), (9.0, 0.8, 5.8, 6.0),
                          (16.0, 1.2, 6.2, 6.0), (3.1, 9.0, 4.0, 8.0)]:
        A, B = C.c_double(), C.c_double()
        h.mbdh_scs_kernel(r * r, sig2, S, d, C.byref(A), C.byref(B))
        rt = torch.tensor(r, dtype=torch.float64)
        Ag, Bg = osc.radial_gauss(rt, torch.tensor(sig2, dtype=torch.float64).sqrt())
        g = float(otz.one_minus_fermi(rt, S, d))
        assert A.value == pytest.approx(g * float(Ag), rel=1e-13)
        assert B.value == pytest.approx(g * float(Bg), rel=1e-13)
