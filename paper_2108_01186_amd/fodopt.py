"""FOD optimisation: minimise E_SIC over the Fermi-orbital descriptors.

The FOD positions a_i are variational parameters of FLOSIC: they are moved
until the FOD forces -dE_SIC/da_i vanish (Sec. I.B, Eq. 9-11; the paper
relaxes them to 1e-3 Ha/Bohr per FOD).  This module drives that loop on the
device: every energy and gradient comes from the library (one forward pass,
one adjoint pass), and the host only runs a limited-memory BFGS update with
a backtracking line search on the 3N coordinates of each spin channel.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

from . import fsic as F


@dataclasses.dataclass
class FodOptResult:
    fods: List[np.ndarray]        # optimised FODs per spin, (N, 3) each
    energy: float                 # E_SIC at the optimised FODs (Ha)
    max_force: float              # max over FODs of |dE/da_i| (Ha/Bohr)
    steps: int                    # accepted L-BFGS steps
    evaluations: int              # forward + backward passes
    history: List[float]          # E_SIC after each accepted step (first: initial)
    converged: bool


def _max_force(g: np.ndarray) -> float:
    return float(np.sqrt((g.reshape(-1, 3) ** 2).sum(axis=1)).max()) if g.size else 0.0


def optimize_fods(ctx: F.Context, n, h: float, origin, psi: Sequence, fods: Sequence,
                  ftol: float = 1e-3, max_steps: int = 50, memory: int = 8,
                  max_move: float = 0.2, verbose: bool = False) -> FodOptResult:
    """L-BFGS on E_SIC(a) for one system.

    psi: per spin, device (N_s, M) float64 tensors; fods: per spin, (N_s, 3)
    starting positions (Bohr).  Stops when every FOD force is below ftol
    (Ha/Bohr) or after max_steps accepted steps.  Steps are capped at
    max_move Bohr per coordinate; a step that would carry an FOD's
    interpolation stencil off the grid, into vacuum, or raise the energy is
    shortened (backtracking, factor 1/2)."""
    nocc = [int(p.shape[0]) for p in psi]
    shapes = [(k, 3) for k in nocc]
    x = np.concatenate([np.asarray(f, dtype=np.float64).reshape(-1) for f in fods])
    base = {"n": n, "h": h, "origin": np.asarray(origin, dtype=np.float64), "psi": list(psi)}
    if not (ctx.opts.flags & F.FSIC_KEEP_TAPE):
        ctx.set_opts(flags=ctx.opts.flags | F.FSIC_KEEP_TAPE)
    nevals = 0

    def split(v):
        out, o = [], 0
        for k in nocc:
            out.append(v[o:o + 3 * k].reshape(k, 3).copy())
            o += 3 * k
        return out

    def evaluate(v):
        nonlocal nevals
        nevals += 1
        e = ctx.forward([dict(base, fod=split(v))])[0][0]
        g = ctx.backward([nocc])[0]
        return float(e), np.concatenate([gi.reshape(-1) for gi in g])

    e, g = evaluate(x)
    hist = [e]
    S, Y = [], []
    steps = 0
    while _max_force(g) >= ftol and steps < max_steps:
        # two-loop recursion: d = -H g
        q = g.copy()
        alph = []
        for s_, y_ in reversed(list(zip(S, Y))):
            rho = 1.0 / float(y_ @ s_)
            a = rho * float(s_ @ q)
            alph.append((rho, a))
            q -= a * y_
        if S:
            q *= float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1])
        for (s_, y_), (rho, a) in zip(zip(S, Y), reversed(alph)):
            b = rho * float(y_ @ q)
            q += (a - b) * s_
        d = -q
        if float(d @ g) >= 0.0:  # not a descent direction: restart from steepest descent
            S.clear(); Y.clear()
            d = -g
        big = float(np.abs(d).max())
        if big > max_move:
            d *= max_move / big
        t = 1.0
        accepted = False
        for _ in range(20):
            xn = x + t * d
            try:
                en, gn = evaluate(xn)
            except F.FsicError:
                t *= 0.5  # FOD stencil off the grid or in vacuum: shorter step
                continue
            if en <= e + 1e-4 * t * float(d @ g):
                accepted = True
                break
            t *= 0.5
        if not accepted:
            break
        s_, y_ = xn - x, gn - g
        if float(s_ @ y_) > 1e-12 * float(np.linalg.norm(s_) * np.linalg.norm(y_)):
            S.append(s_); Y.append(y_)
            if len(S) > memory:
                S.pop(0); Y.pop(0)
        x, e, g = xn, en, gn
        steps += 1
        hist.append(e)
        if verbose:
            print(f"[fodopt] step {steps}: E_SIC = {e:.10f} Ha, max force = {_max_force(g):.2e} Ha/Bohr",
                  flush=True)
    return FodOptResult(fods=split(x), energy=e, max_force=_max_force(g), steps=steps,
                        evaluations=nevals, history=hist, converged=_max_force(g) < ftol)
