"""ctypes front end of the FP64 CPU oracle (``fsic_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The test suite, the package smoke check and the
benchmark's CPU-baseline leg are the only users.  The GPU library never
imports this module and this module imports nothing from the GPU library.

Every function follows the definitions of Diaz et al., arXiv 2108.01186:
Eq. 1 (PZ-SIC energy), Eq. 5 (orbital SIC potential), Eq. 6-8 (Fermi orbitals
and the transformation matrix), Sec. I.B (Loewdin orthonormalisation), Sec. II.A (the
finite-difference Poisson problem with multipole Dirichlet values), Sec. II.B
(cubic interpolation at the FODs), Sec. II.C / Eq. 13 (Slater-averaged SIC
potential), Eq. 9-11 (FOD gradient).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fsic_oracle.c")
LIB = os.path.join(HERE, "liboracle_fsic.so")

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math: IEEE semantics)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=HERE)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.orc_multipole_potential.restype = ctypes.c_double
        L.orc_xc_pol.restype = None
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _grid(n, origin):
    return np.asarray(n, dtype=np.int32).copy(), _f64(origin)


class OracleError(RuntimeError):
    CODES = {-1: "bad argument", -2: "FOD interpolation stencil leaves the grid",
             -3: "FOD in vacuum", -4: "singular overlap matrix", -5: "CG did not converge"}

    def __init__(self, code):
        self.code = code
        super().__init__(f"oracle status {code}: {self.CODES.get(code, '?')}")


def _check(st, allow_noconv=False):
    if st == 0 or (allow_noconv and st == -5):
        return st
    raise OracleError(st)


def fd_coeffs(p: int) -> np.ndarray:
    c = np.zeros(p + 1)
    _check(lib().orc_fd_coeffs(p, _d(c)))
    return c


def apply_laplacian(u: np.ndarray, h: float, p: int) -> np.ndarray:
    """L u, zero Dirichlet ghosts; u has shape (nz, ny, nx)."""
    u = _f64(u)
    n = np.array([u.shape[2], u.shape[1], u.shape[0]], dtype=np.int32)
    out = np.empty_like(u)
    _check(lib().orc_apply_laplacian(_i(n), ctypes.c_double(h), p, _d(u), _d(out)))
    return out


def hamiltonian(psi: np.ndarray, v: np.ndarray, h: float, p: int = 6) -> np.ndarray:
    """-1/2 L psi + v psi for psi of shape (count, nz, ny, nx), v of shape (nz, ny, nx)."""
    psi = _f64(psi)
    v = _f64(v)
    n = np.array([psi.shape[3], psi.shape[2], psi.shape[1]], dtype=np.int32)
    out = np.empty_like(psi)
    _check(lib().orc_hamiltonian(_i(n), ctypes.c_double(h), p, psi.shape[0], _d(psi), _d(v), _d(out)))
    return out


def solid_harmonics(lmax: int, x: float, y: float, z: float) -> np.ndarray:
    out = np.zeros((lmax + 1) ** 2)
    _check(lib().orc_solid_harmonics(lmax, ctypes.c_double(x), ctypes.c_double(y),
                                     ctypes.c_double(z), _d(out)))
    return out


def multipole_moments(rho, n, h, origin, lmax):
    n, origin = _grid(n, origin)
    rho = _f64(rho)
    Q = np.zeros((lmax + 1) ** 2)
    _check(lib().orc_multipole_moments(_i(n), ctypes.c_double(h), _d(origin), lmax, _d(rho), _d(Q)))
    return Q


def multipole_potential(Q, n, h, origin, lmax, x, y, z):
    n, origin = _grid(n, origin)
    Q = _f64(Q)
    return lib().orc_multipole_potential(_i(n), ctypes.c_double(h), _d(origin), lmax, _d(Q),
                                         ctypes.c_double(x), ctypes.c_double(y), ctypes.c_double(z))


def poisson(rho, n, h, origin, p=6, lmax=6, tol=1e-13, maxit=20000, transpose=False):
    """Hartree potential v = A rho (or A^T rho); returns (v, iters, relres)."""
    n, origin = _grid(n, origin)
    rho = _f64(rho)
    v = np.zeros_like(rho)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    fn = lib().orc_poisson_transpose if transpose else lib().orc_poisson
    _check(fn(_i(n), ctypes.c_double(h), _d(origin), p, lmax, _d(rho), ctypes.c_double(tol),
              maxit, _d(v), ctypes.byref(it), ctypes.byref(rr)))
    return v, it.value, rr.value


def orbital_terms(rho, n, h, origin, p=6, lmax=6, tol=1e-13, maxit=20000, rho_floor=1e-30):
    """(U, X, iters, relres) of one orbital density: Hartree and LSDA terms of Eq. 1."""
    n, origin = _grid(n, origin)
    rho = _f64(rho)
    U, X, rr = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    it = ctypes.c_int(0)
    _check(lib().orc_orbital_terms(_i(n), ctypes.c_double(h), _d(origin), p, lmax,
                                   ctypes.c_double(tol), maxit, ctypes.c_double(rho_floor),
                                   _d(rho), ctypes.byref(U), ctypes.byref(X), ctypes.byref(it),
                                   ctypes.byref(rr)))
    return U.value, X.value, it.value, rr.value


def xc_pol(rho, rho_floor=1e-30):
    """(eps_x, eps_c, v_x, v_c) at full spin polarisation, elementwise."""
    rho = np.atleast_1d(_f64(rho))
    out = np.zeros((4,) + rho.shape)
    ex, ec, vx, vc = (ctypes.c_double() for _ in range(4))
    L = lib()
    for idx, r in np.ndenumerate(rho):
        L.orc_xc_pol(ctypes.c_double(r), ctypes.c_double(rho_floor), ctypes.byref(ex),
                     ctypes.byref(ec), ctypes.byref(vx), ctypes.byref(vc))
        out[(0,) + idx] = ex.value
        out[(1,) + idx] = ec.value
        out[(2,) + idx] = vx.value
        out[(3,) + idx] = vc.value
    return out


def interp(psi, n, h, origin, a):
    """values u[N] and gradients du[N,3] of the cubic interpolant at point a."""
    n, origin = _grid(n, origin)
    psi = _f64(psi)
    N = psi.shape[0]
    a = _f64(a)
    u = np.zeros(N)
    du = np.zeros((N, 3))
    _check(lib().orc_interp(_i(n), ctypes.c_double(h), _d(origin), N, _d(psi), _d(a), _d(u), _d(du)))
    return u, du


def grid_gradient(f, n, h):
    """per-node difference gradient (3, M) of one field (Sec. II.B)."""
    n = np.asarray(n, dtype=np.int32).copy()
    f = _f64(f).reshape(-1)
    g = np.zeros((3, f.size))
    _check(lib().orc_grid_gradient(_i(n), ctypes.c_double(h), _d(f), _d(g)))
    return g


def interp_fdgrad(psi, n, h, origin, a):
    """values u[N] and interpolated per-node difference gradients du[N,3] at a."""
    n, origin = _grid(n, origin)
    psi = _f64(psi)
    N = psi.shape[0]
    a = _f64(a)
    u = np.zeros(N)
    du = np.zeros((N, 3))
    _check(lib().orc_interp_fdgrad(_i(n), ctypes.c_double(h), _d(origin), N, _d(psi), _d(a), _d(u),
                                   _d(du)))
    return u, du


def jacobi_eig(A):
    A = _f64(A)
    N = A.shape[0]
    lam = np.zeros(N)
    U = np.zeros((N, N))
    _check(lib().orc_jacobi_eig(N, _d(A), _d(lam), _d(U)))
    return lam, U


class SpinResult:
    """Outputs of one spin channel."""

    def __init__(self, N, M):
        self.e = 0.0
        self.U = np.zeros(N)
        self.X = np.zeros(N)
        self.vsic = np.zeros(M)
        self.T = np.zeros((N, N))
        self.S = np.zeros((N, N))
        self.Z = np.zeros((N, N))
        self.phi = np.zeros((N, M))
        self.v = np.zeros((N, M))
        self.iters = np.zeros(N, dtype=np.int32)
        self.relres = np.zeros(N)


def sic_spin(psi, fod, n, h, origin, p=6, lmax=6, tol=1e-13, maxit=20000, vscale=1.0,
             rho_floor=1e-30, keep_fields=True):
    """One spin channel: E_spin = -sum_i (U_i + X_i), V_SIC, intermediates."""
    n, origin = _grid(n, origin)
    psi = _f64(psi).reshape(psi.shape[0], -1)
    fod = _f64(fod).reshape(-1, 3)
    N, M = psi.shape
    r = SpinResult(N, M if keep_fields else 1)
    e = ctypes.c_double(0.0)
    null = ctypes.POINTER(ctypes.c_double)()
    st = lib().orc_sic_spin(
        _i(n), ctypes.c_double(h), _d(origin), p, lmax, ctypes.c_double(tol), maxit,
        ctypes.c_double(vscale), ctypes.c_double(rho_floor), N, _d(psi), _d(fod),
        ctypes.byref(e), _d(r.U), _d(r.X), _d(r.vsic) if keep_fields else null,
        _d(r.T), _d(r.S), _d(r.Z), _d(r.phi) if keep_fields else null,
        _d(r.v) if keep_fields else null, _i(r.iters), _d(r.relres))
    _check(st)
    r.e = e.value
    if not keep_fields:
        r.vsic = r.phi = r.v = None
    return r


def flo_spin(psi, fod, n, h, origin, rho_floor=1e-30):
    """Fermi-Loewdin orbitals of one spin channel: (phi, T, S, Z)."""
    n, origin = _grid(n, origin)
    psi = _f64(psi).reshape(psi.shape[0], -1)
    fod = _f64(fod).reshape(-1, 3)
    N, M = psi.shape
    phi = np.zeros((N, M))
    T = np.zeros((N, N)); S = np.zeros((N, N)); Z = np.zeros((N, N))
    _check(lib().orc_flo_spin(_i(n), ctypes.c_double(h), _d(origin), ctypes.c_double(rho_floor),
                              N, _d(psi), _d(fod), _d(phi), _d(T), _d(S), _d(Z)))
    return phi, T, S, Z


def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(n):
    """Threads of the oracle's parallel loops from here on (OpenMP)."""
    lib().orc_set_num_threads(int(n))


def sic_grad_spin(psi, fod, n, h, origin, p=6, lmax=6, tol=1e-13, maxit=20000, rho_floor=1e-30,
                  fd_gradient=False, eq9=False):
    """dE_SIC/da for one spin channel, shape (N, 3).  fd_gradient: grad psi at
    the FODs from interpolated per-node differences (Sec. II.B) instead of the
    interpolant's derivative; eq9: the Eq. 9 form with V_k = -(v_k + vxc_k)
    instead of the exact derivative of the discrete energy."""
    n, origin = _grid(n, origin)
    psi = _f64(psi).reshape(psi.shape[0], -1)
    fod = _f64(fod).reshape(-1, 3)
    N = psi.shape[0]
    g = np.zeros((N, 3))
    st = lib().orc_sic_grad_spin_mode(_i(n), ctypes.c_double(h), _d(origin), p, lmax,
                                      ctypes.c_double(tol), maxit, ctypes.c_double(rho_floor), N,
                                      _d(psi), _d(fod), int(bool(fd_gradient)), int(bool(eq9)), _d(g))
    _check(st)
    return g


def sic_system(sysd, p=6, lmax=6, tol=1e-13, maxit=20000, vscale=1.0, rho_floor=1e-30,
               keep_fields=True):
    """Both spin channels of a synthetic system (see the input generator):
    returns (E_SIC, [SpinResult per spin])."""
    out = []
    e = 0.0
    for s in range(sysd.nspin):
        r = sic_spin(np.asarray(sysd.psi[s]), np.asarray(sysd.fod[s]), sysd.n, sysd.h, sysd.origin,
                     p, lmax, tol, maxit, vscale, rho_floor, keep_fields)
        e += r.e
        out.append(r)
    return e, out
