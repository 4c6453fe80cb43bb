"""Python binding of the gfx950 FLOSIC SIC library (``libfsic.so``).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  The names mirror ``include/fsic.h``.  PyTorch supplies device
memory and the current HIP stream.

The library must be built (``python -m paper_2108_01186_amd.build`` or
``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libfsic.so")

if not os.path.exists(LIBPATH):
    raise ImportError(f"{LIBPATH} is missing: build the HIP library first "
                      "(python -m paper_2108_01186_amd.build)")

_lib = ctypes.CDLL(LIBPATH)

# --------------------------------------------------------------------------
# C structures (include/fsic.h)
# --------------------------------------------------------------------------

FSIC_OK, FSIC_EINVAL, FSIC_ENOMEM, FSIC_EHIP, FSIC_ENONORTHO, FSIC_EVACUUM, \
    FSIC_EBOUNDARY, FSIC_ESINGULAR, FSIC_ENOCONV, FSIC_ENOTAPE = range(10)
FSIC_FP64, FSIC_MIXED = 0, 1
FSIC_CG, FSIC_PCG, FSIC_AAR = 0, 1, 2
FSIC_WANT_VSIC, FSIC_KEEP_TAPE, FSIC_ALLOW_NONORTHO, FSIC_PROFILE, FSIC_FP32_ORBITALS = 1, 2, 4, 8, 16
FSIC_GRAPHS = 32
FSIC_PAPER_GRADIENT, FSIC_EQ9_FORCES, FSIC_DIRECT_BC = 64, 128, 256


class fsic_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("h", ctypes.c_double), ("origin", ctypes.c_double * 3)]


class fsic_opts(ctypes.Structure):
    _fields_ = [("fd_order", ctypes.c_int32), ("lmax", ctypes.c_int32), ("solver", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("vsic_scale", ctypes.c_double),
                ("rho_floor", ctypes.c_double), ("s_eig_floor", ctypes.c_double),
                ("flags", ctypes.c_uint32)]


class fsic_system(ctypes.Structure):
    _fields_ = [("grid", fsic_grid), ("nspin", ctypes.c_int32), ("nocc", ctypes.c_int32 * 2),
                ("psi", ctypes.c_void_p * 2), ("fod", ctypes.c_void_p * 2),
                ("vsic", ctypes.c_void_p * 2)]


class fsic_stats(ctypes.Structure):
    _fields_ = [("nsolves", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("total_iters", ctypes.c_int64), ("outer_refinements", ctypes.c_int32),
                ("max_relres", ctypes.c_double), ("cond_S_max", ctypes.c_double),
                ("min_rho_fod", ctypes.c_double), ("max_nonortho", ctypes.c_double),
                ("ms_phase", ctypes.c_double * 8),
                ("sweep_launches", ctypes.c_int32), ("update_launches", ctypes.c_int32),
                ("sweep_ms", ctypes.c_double), ("sweep_bytes", ctypes.c_double),
                ("update_ms", ctypes.c_double), ("update_bytes", ctypes.c_double),
                ("precond_launches", ctypes.c_int32), ("precond_ms", ctypes.c_double),
                ("precond_bytes", ctypes.c_double), ("precond_flops", ctypes.c_double),
                ("stencil_cpt", ctypes.c_int32), ("stencil_depth", ctypes.c_int32),
                ("stencil_blocks", ctypes.c_int64), ("tune_ms", ctypes.c_double),
                ("resid_launches", ctypes.c_int32), ("resid_ms", ctypes.c_double),
                ("resid_bytes", ctypes.c_double), ("graph_captures", ctypes.c_int32),
                ("precond_layout", ctypes.c_int32), ("precond_tune_ms", ctypes.c_double),
                ("npoisson", ctypes.c_int32), ("basis_solves", ctypes.c_int32), ("basis_ms", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "ms_phase"}
        d["ms_phase"] = list(self.ms_phase)
        return d


_P = ctypes.POINTER
_vp = ctypes.c_void_p
_dp = _P(ctypes.c_double)
_ip = _P(ctypes.c_int32)


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


fsic_default_opts = _sig("fsic_default_opts", ctypes.c_int, [_P(fsic_opts)])
fsic_create = _sig("fsic_create", ctypes.c_int, [_P(_vp), _P(fsic_opts), _vp])
fsic_set_opts = _sig("fsic_set_opts", ctypes.c_int, [_vp, _P(fsic_opts)])
fsic_forward = _sig("fsic_forward", ctypes.c_int,
                    [_vp, ctypes.c_int32, _P(fsic_system), _dp, _dp, _dp, _P(fsic_stats)])
fsic_backward = _sig("fsic_backward", ctypes.c_int, [_vp, _dp, _P(_dp), _P(fsic_stats)])
fsic_forward_backward = _sig("fsic_forward_backward", ctypes.c_int,
                             [_vp, ctypes.c_int32, _P(fsic_system), _dp, _dp, _dp, _dp, _P(_dp),
                              _P(fsic_stats), _P(fsic_stats)])
fsic_status_string = _sig("fsic_status_string", ctypes.c_char_p, [ctypes.c_int])
fsic_last_error = _sig("fsic_last_error", ctypes.c_char_p, [_vp])
fsic_destroy = _sig("fsic_destroy", None, [_vp])
fsic_op_laplacian = _sig("fsic_op_laplacian", ctypes.c_int,
                         [_ip, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp])
fsic_op_laplacian_f32 = _sig("fsic_op_laplacian_f32", ctypes.c_int,
                             [_ip, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp])
fsic_op_xc = _sig("fsic_op_xc", ctypes.c_int,
                  [ctypes.c_int64, _vp, ctypes.c_double, _vp, _vp, _vp, _vp, _vp])
fsic_op_hamiltonian = _sig("fsic_op_hamiltonian", ctypes.c_int,
                           [_ip, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp])
fsic_op_poisson = _sig("fsic_op_poisson", ctypes.c_int,
                       [_P(fsic_grid), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp,
                        ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _ip, _dp,
                        _vp])
fsic_op_invsqrt = _sig("fsic_op_invsqrt", ctypes.c_int,
                       [ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp])
fsic_op_flo = _sig("fsic_op_flo", ctypes.c_int,
                   [_P(fsic_grid), ctypes.c_int32, _vp, _dp, ctypes.c_double, _vp, _vp, _vp, _vp,
                    _vp, _vp])
fsic_op_flo_noalloc = _sig("fsic_op_flo_noalloc", ctypes.c_int,
                           [_P(fsic_grid), ctypes.c_int32, _vp, _dp, ctypes.c_double, _vp, _vp, _vp,
                            _vp, _vp, _vp])
fsic_op_interp = _sig("fsic_op_interp", ctypes.c_int,
                      [_P(fsic_grid), ctypes.c_int32, ctypes.c_int32, _vp, _dp, ctypes.c_int32, _vp,
                       _vp, _vp])

EXPORTED = ["fsic_default_opts", "fsic_create", "fsic_set_opts", "fsic_forward", "fsic_backward",
            "fsic_forward_backward",
            "fsic_status_string", "fsic_last_error", "fsic_destroy", "fsic_op_laplacian",
            "fsic_op_laplacian_f32", "fsic_op_xc", "fsic_op_poisson", "fsic_op_invsqrt",
            "fsic_op_hamiltonian", "fsic_op_interp",
            "fsic_op_flo", "fsic_op_flo_noalloc"]


class FsicError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        msg = fsic_status_string(status).decode()
        super().__init__(f"fsic status {status} ({msg})" + (f": {detail}" if detail else ""))


def _check(st, ctx=None, allow=()):
    if st != FSIC_OK and st not in allow:
        detail = fsic_last_error(ctx).decode() if ctx else ""
        raise FsicError(st, detail)
    return st


# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def default_opts(**kw) -> fsic_opts:
    o = fsic_opts()
    _check(fsic_default_opts(ctypes.byref(o)))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": FSIC_FP64, "mixed": FSIC_MIXED}[v]
        if k == "solver" and isinstance(v, str):
            v = {"cg": FSIC_CG, "pcg": FSIC_PCG, "aar": FSIC_AAR}[v]
        setattr(o, k, v)
    return o


def make_grid(n, h, origin) -> fsic_grid:
    g = fsic_grid()
    for d in range(3):
        g.n[d] = int(n[d])
        g.origin[d] = float(origin[d])
    g.h = float(h)
    return g


class Context:
    """Owns an fsic_ctx bound to a HIP stream (torch's current stream by default)."""

    def __init__(self, opts: Optional[fsic_opts] = None, stream=None, **kw):
        self.opts = opts if opts is not None else default_opts(**kw)
        self._h = ctypes.c_void_p()
        self._stream = _stream_ptr(stream)
        _check(fsic_create(ctypes.byref(self._h), ctypes.byref(self.opts), self._stream))
        self._keep = []
        self.stats = None
        # the context holds one tape (the last forward pass); every forward
        # pass gets a new generation number so a backward pass can tell
        # whether the tape is still its own
        self.generation = 0

    def close(self):
        if self._h:
            fsic_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_opts(self, **kw):
        for k, v in kw.items():
            if k == "precision" and isinstance(v, str):
                v = {"fp64": FSIC_FP64, "mixed": FSIC_MIXED}[v]
            if k == "solver" and isinstance(v, str):
                v = {"cg": FSIC_CG, "pcg": FSIC_PCG, "aar": FSIC_AAR}[v]
            setattr(self.opts, k, v)
        self.generation += 1  # the library drops the tape with new options
        _check(fsic_set_opts(self._h, ctypes.byref(self.opts)), self._h)

    def _systems(self, systems):
        nsys = len(systems)
        arr = (fsic_system * nsys)()
        keep = []
        norb = 0
        for k, s in enumerate(systems):
            arr[k].grid = make_grid(s["n"], s["h"], s["origin"])
            nspin = len(s["psi"])
            arr[k].nspin = nspin
            for sp in range(nspin):
                psi = s["psi"][sp]
                fod = np.ascontiguousarray(np.asarray(s["fod"][sp], dtype=np.float64).reshape(-1, 3))
                if psi.dtype != _torch().float64:
                    raise TypeError("psi must be float64")
                if psi.shape[0] != fod.shape[0]:
                    raise ValueError("psi rows and FODs differ in number")
                arr[k].nocc[sp] = psi.shape[0]
                arr[k].psi[sp] = _dev_ptr(psi).value
                arr[k].fod[sp] = fod.ctypes.data
                keep.append(fod)
                vs = (s.get("vsic") or [None, None])[sp]
                arr[k].vsic[sp] = _dev_ptr(vs).value if vs is not None else None
                norb += psi.shape[0]
        return arr, keep, norb

    def forward(self, systems: Sequence[dict], allow_noconv=False):
        """systems: dicts with n, h, origin, psi (list of device (N, M) float64
        tensors), fod (list of host (N, 3) arrays), vsic (list of device (M,)
        tensors or None).  Returns (E_SIC per system, U, X, stats)."""
        nsys = len(systems)
        arr, keep, norb = self._systems(systems)
        e = np.zeros(nsys)
        U = np.zeros(norb)
        X = np.zeros(norb)
        st = fsic_stats()
        status = fsic_forward(self._h, nsys, arr, e.ctypes.data_as(_dp), U.ctypes.data_as(_dp),
                              X.ctypes.data_as(_dp), ctypes.byref(st))
        self.generation += 1
        _check(status, self._h, allow=(FSIC_ENOCONV,) if allow_noconv else ())
        self._keep = keep
        self.stats = st.as_dict()
        return e, U, X, self.stats

    def forward_backward(self, systems: Sequence[dict], grad_e=None):
        """forward() and backward() of the same systems in one library call
        (needs FSIC_KEEP_TAPE).  Returns (E_SIC, U, X, dE/da per system as in
        backward(), forward stats, backward stats)."""
        nsys = len(systems)
        arr, keep, norb = self._systems(systems)
        nocc = [[int(p.shape[0]) for p in s["psi"]] for s in systems]
        e = np.zeros(nsys)
        U = np.zeros(norb)
        X = np.zeros(norb)
        outs = [np.zeros((sum(no), 3)) for no in nocc]
        ptrs = (_dp * nsys)(*[o.ctypes.data_as(_dp) for o in outs])
        ge = None
        if grad_e is not None:
            ge = np.ascontiguousarray(np.asarray(grad_e, dtype=np.float64).reshape(nsys))
        stf, stb = fsic_stats(), fsic_stats()
        status = fsic_forward_backward(self._h, nsys, arr, e.ctypes.data_as(_dp),
                                       U.ctypes.data_as(_dp), X.ctypes.data_as(_dp),
                                       ge.ctypes.data_as(_dp) if ge is not None else None, ptrs,
                                       ctypes.byref(stf), ctypes.byref(stb))
        self.generation += 1
        _check(status, self._h)
        self._keep = keep
        self.stats = stb.as_dict()
        return e, U, X, self._split(outs, nocc), stf.as_dict(), self.stats

    @staticmethod
    def _split(outs, nocc_per_system):
        res = []
        for o, no in zip(outs, nocc_per_system):
            parts, b = [], 0
            for n in no:
                parts.append(o[b:b + n])
                b += n
            res.append(parts)
        return res

    def backward(self, nocc_per_system: Sequence[Sequence[int]], grad_e=None):
        """Returns, per system, dE/da as an array (nspin, N, 3) (ragged spins
        as a list)."""
        nsys = len(nocc_per_system)
        outs = [np.zeros((sum(no), 3)) for no in nocc_per_system]
        ptrs = (_dp * nsys)(*[o.ctypes.data_as(_dp) for o in outs])
        ge = None
        if grad_e is not None:
            ge = np.ascontiguousarray(np.asarray(grad_e, dtype=np.float64).reshape(nsys))
        st = fsic_stats()
        _check(fsic_backward(self._h, ge.ctypes.data_as(_dp) if ge is not None else None, ptrs,
                             ctypes.byref(st)), self._h)
        self.stats = st.as_dict()
        return self._split(outs, nocc_per_system)


# --------------------------------------------------------------------------
# operator-level calls
# --------------------------------------------------------------------------

def op_laplacian(u, h: float, fd_order: int = 12, stream=None):
    """L u for u of shape (count, nz, ny, nx) (or (nz, ny, nx)), zero ghosts."""
    torch = _torch()
    squeeze = u.dim() == 3
    if squeeze:
        u = u.unsqueeze(0)
    u = u.contiguous()
    out = torch.empty_like(u)
    n = (ctypes.c_int32 * 3)(u.shape[3], u.shape[2], u.shape[1])
    fn = fsic_op_laplacian if u.dtype == torch.float64 else fsic_op_laplacian_f32
    _check(fn(n, h, fd_order, u.shape[0], _dev_ptr(u), _dev_ptr(out), _stream_ptr(stream)))
    return out[0] if squeeze else out


def op_xc(rho, rho_floor: float = 1e-30, stream=None):
    torch = _torch()
    rho = rho.contiguous()
    outs = [torch.empty_like(rho) for _ in range(4)]
    _check(fsic_op_xc(rho.numel(), _dev_ptr(rho), rho_floor, *[_dev_ptr(o) for o in outs],
                      _stream_ptr(stream)))
    return outs


def op_hamiltonian(psi, v, n, h: float, fd_order: int = 12, stream=None):
    """-1/2 L psi + v psi for device psi (count, M) and v (M,), float64."""
    torch = _torch()
    psi = psi.contiguous()
    v = v.contiguous()
    count = psi.shape[0] if psi.dim() > 1 else 1
    out = torch.empty_like(psi)
    nn = (ctypes.c_int32 * 3)(*[int(x) for x in n])
    _check(fsic_op_hamiltonian(nn, h, fd_order, count, _dev_ptr(psi), _dev_ptr(v), _dev_ptr(out),
                               _stream_ptr(stream)))
    return out


def op_poisson(rho, n, h, origin, fd_order=12, lmax=6, tol=1e-10, max_iter=20000,
               precision="fp64", solver="cg", stream=None):
    """Hartree potentials of densities rho (count, M) on one grid."""
    torch = _torch()
    rho = rho.contiguous()
    count = rho.shape[0] if rho.dim() > 1 else 1
    v = torch.empty_like(rho)
    g = make_grid(n, h, origin)
    it = np.zeros(count, dtype=np.int32)
    rr = np.zeros(count)
    prec = {"fp64": FSIC_FP64, "mixed": FSIC_MIXED}[precision] if isinstance(precision, str) else precision
    solv = {"cg": FSIC_CG, "pcg": FSIC_PCG, "aar": FSIC_AAR}[solver] if isinstance(solver, str) else solver
    _check(fsic_op_poisson(ctypes.byref(g), fd_order, lmax, count, _dev_ptr(rho), _dev_ptr(v), tol,
                           max_iter, prec, solv, it.ctypes.data_as(_ip), rr.ctypes.data_as(_dp),
                           _stream_ptr(stream)))
    return v, it, rr


def op_invsqrt(S, stream=None):
    """S^{-1/2} and eigenvalues of SPD matrices S (count, N, N)."""
    torch = _torch()
    S = S.contiguous()
    squeeze = S.dim() == 2
    if squeeze:
        S = S.unsqueeze(0)
    Z = torch.empty_like(S)
    lam = torch.empty(S.shape[0], S.shape[1], dtype=S.dtype, device=S.device)
    _check(fsic_op_invsqrt(S.shape[1], S.shape[0], _dev_ptr(S), _dev_ptr(Z), _dev_ptr(lam),
                           _stream_ptr(stream)))
    return (Z[0], lam[0]) if squeeze else (Z, lam)


def op_interp(psi, pts, n, h, origin, fd_gradient=False, stream=None):
    """psi_a(p_k) (K x N) and its gradient (K x N x 3) at K points: the
    cubic interpolant's derivative, or (fd_gradient) the interpolated
    per-node first differences."""
    torch = _torch()
    psi = psi.contiguous()
    N = psi.shape[0]
    pts = np.ascontiguousarray(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
    K = pts.shape[0]
    u = torch.empty(K, N, dtype=torch.float64, device=psi.device)
    du = torch.empty(K, N, 3, dtype=torch.float64, device=psi.device)
    g = make_grid(n, h, origin)
    _check(fsic_op_interp(ctypes.byref(g), N, K, _dev_ptr(psi), pts.ctypes.data_as(_dp),
                          int(bool(fd_gradient)), _dev_ptr(u), _dev_ptr(du), _stream_ptr(stream)))
    return u, du


def op_flo(psi, fod, n, h, origin, rho_floor=1e-30, stream=None, noalloc=False):
    """T, G, S, Z (N x N) and the Fermi-Loewdin orbitals phi (N x M) of one
    channel; noalloc: through fsic_op_flo_noalloc (the library allocates
    nothing; the outputs here are still torch tensors)."""
    torch = _torch()
    psi = psi.contiguous()
    N = psi.shape[0]
    fod = np.ascontiguousarray(np.asarray(fod, dtype=np.float64).reshape(N, 3))
    mats = [torch.empty(N, N, dtype=torch.float64, device=psi.device) for _ in range(4)]
    phi = torch.empty_like(psi)
    g = make_grid(n, h, origin)
    fn = fsic_op_flo_noalloc if noalloc else fsic_op_flo
    _check(fn(ctypes.byref(g), N, _dev_ptr(psi), fod.ctypes.data_as(_dp), rho_floor,
              *[_dev_ptr(m) for m in mats], _dev_ptr(phi), _stream_ptr(stream)))
    return (*mats, phi)


# --------------------------------------------------------------------------
# one-call convenience for a synthetic System (see synth.py)
# --------------------------------------------------------------------------

def system_dict(sysobj, vsic=True):
    torch = _torch()
    d = {"n": sysobj.n, "h": sysobj.h, "origin": sysobj.origin,
         "psi": list(sysobj.psi), "fod": list(sysobj.fod)}
    if vsic:
        d["vsic"] = [torch.empty(sysobj.M, dtype=torch.float64, device=p.device) for p in sysobj.psi]
    return d


def sic_energy(sysobjs, opts: Optional[fsic_opts] = None, ctx: Optional[Context] = None, **kw):
    """E_SIC and V_SIC of synthetic systems whose psi already lives on the GPU."""
    own = ctx is None
    if own:
        ctx = Context(opts, **kw)
    dicts = [system_dict(s) for s in sysobjs]
    e, U, X, st = ctx.forward(dicts)
    out = dict(e=e, U=U, X=X, stats=st, vsic=[d["vsic"] for d in dicts])
    if own:
        ctx.close()
    return out


# --------------------------------------------------------------------------
# autograd: E_SIC(FODs) with the library's adjoint as the backward pass
# --------------------------------------------------------------------------

def _make_autograd():
    torch = _torch()

    class FlosicSIC(torch.autograd.Function):
        """E_SIC of one system as a function of its FOD positions.

        forward(fctx, grid, psis, *fods) -> (E_SIC, *V_SIC)
          fctx:  a Context (its KEEP_TAPE flag is turned on)
          grid:  (n, h, origin)
          psis:  tuple of device (N_s, M) float64 orbitals (must stay unchanged
                 until backward runs)
          fods:  one host (N_s, 3) float64 tensor per spin channel
        V_SIC outputs are not differentiable; the gradient of E_SIC with
        respect to each FOD tensor comes from fsic_backward.  The context
        keeps the tape of its last forward pass only: when another forward
        pass ran on it since this one (two geometries before one backward),
        backward first repeats this forward pass (same inputs, same result).
        """

        @staticmethod
        def forward(actx, fctx, grid, psis, *fods):
            if not (fctx.opts.flags & FSIC_KEEP_TAPE):
                fctx.set_opts(flags=fctx.opts.flags | FSIC_KEEP_TAPE)
            n, h, origin = grid
            vs = [torch.empty(p.shape[1], dtype=torch.float64, device=p.device) for p in psis]
            d = {"n": n, "h": h, "origin": origin, "psi": list(psis),
                 "fod": [f.detach().cpu().numpy().copy() for f in fods], "vsic": vs}
            e, U, X, st = fctx.forward([d])
            actx.fctx = fctx
            actx.generation = fctx.generation
            actx.nocc = [p.shape[0] for p in psis]
            actx.psis = psis
            actx.inputs = dict(d, vsic=None)
            actx.mark_non_differentiable(*vs)
            return (torch.tensor(e[0], dtype=torch.float64), *vs)

        @staticmethod
        def backward(actx, gE, *gV):
            for g in gV:
                if g is not None and bool(torch.any(g != 0)):
                    raise RuntimeError("V_SIC is not differentiable in this library")
            fctx = actx.fctx
            if fctx.generation != actx.generation:
                # the tape belongs to a later forward pass: rebuild this one
                if not (fctx.opts.flags & FSIC_KEEP_TAPE):
                    fctx.set_opts(flags=fctx.opts.flags | FSIC_KEEP_TAPE)
                fctx.forward([actx.inputs])
                actx.generation = fctx.generation
            res = fctx.backward([actx.nocc], grad_e=[float(gE)])
            grads = [torch.tensor(r, dtype=torch.float64) for r in res[0]]
            return (None, None, None, *grads)

    return FlosicSIC


_FLOSIC = None


def flosic_sic(fctx: Context, n, h, origin, psis, fods):
    """Differentiable E_SIC (and V_SIC per spin) of one system; fods are host
    float64 tensors, typically with requires_grad=True."""
    global _FLOSIC
    if _FLOSIC is None:
        _FLOSIC = _make_autograd()
    out = _FLOSIC.apply(fctx, (tuple(n), float(h), tuple(origin)), tuple(psis), *fods)
    return out[0], list(out[1:])
