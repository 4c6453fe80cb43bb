"""Seeded synthetic molecule-shaped inputs for the SIC path.

This module is the one thing the GPU library's tests and the CPU oracle's
tests share.  It draws random numbers and evaluates Gaussian primitives; it
holds none of the SIC method's arithmetic (no Fermi orbitals, no overlap of
Fermi orbitals, no Poisson solve, no exchange-correlation).

Recipe (the paper's molecules, pseudopotentials and FODs are not available,
so these stand in for them):
  * grid: n^3 nodes, spacing h, node-centred box: origin = -h (n-1)/2;
  * atoms: uniform in a central cube (a given edge, else the central third of
    the box);
  * Gaussians: Gaussian g sits on atom g mod n_atoms; its type is uniform in
    {s, p_x, p_y, p_z}; its exponent is log-uniform on [0.3, 3.0] Bohr^-2; the
    primitive is (x - X)^l exp(-alpha |r - R|^2), normalised on the grid;
  * Kohn-Sham orbitals per spin: psi_raw = C g with C ~ N(0, 1) of shape
    (N, N_g), then made orthonormal on the grid (dV psi psi^T = I) by the
    symmetric (Loewdin) transformation G^{-1/2};
  * FODs: FOD i of spin up at atom i, of spin down at atom offset + i, plus
    independent N(0, 0.3^2) jitter on each coordinate; the jitter is redrawn
    (seed + 1000 k) if an FOD lands where the grid density at the nearest node
    is below 1e-8.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

try:  # torch only as an array backend (device memory)
    import torch
except ImportError:  # pragma: no cover
    torch = None


@dataclasses.dataclass
class System:
    name: str
    n: tuple            # (nx, ny, nz)
    h: float
    origin: np.ndarray  # (3,)
    nocc: tuple         # orbitals per spin
    psi: list           # per spin: (N, M) float64 (torch tensor or numpy array)
    fod: list           # per spin: (N, 3) float64 numpy array
    atoms: np.ndarray
    seed: int

    @property
    def nspin(self) -> int:
        return len(self.nocc)

    @property
    def M(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])


# Workloads, named by their shapes.  Seeds are 2108 + 100 k (+ instance).
WORKLOADS = {
    # 40^3 grid, h = 0.3 Bohr, 5 atoms in the central 4 Bohr cube, 12 Gaussians,
    # one spin channel with 5 orbitals.
    "mol40": dict(n=40, h=0.3, n_atoms=5, n_gauss=12, nocc=(5,), atom_box=4.0,
                  down_offset=0, seed=2108),
    # 96^3 grid, h = 0.2 Bohr, 16 atoms, 48 Gaussians, 16 + 15 orbitals.
    "mol96": dict(n=96, h=0.2, n_atoms=16, n_gauss=48, nocc=(16, 15), atom_box=None,
                  down_offset=0, seed=2208),
    # 128^3 grid, h = 0.2 Bohr, 64 Gaussian centres, 32 + 32 orbitals; the
    # spin-down FODs sit at centres 32..63.
    "mol128": dict(n=128, h=0.2, n_atoms=64, n_gauss=64, nocc=(32, 32), atom_box=None,
                   down_offset=32, seed=2408),
    # 192^3 grid, h = 0.15 Bohr, 200 Gaussian centres in a 20 Bohr cube,
    # 100 + 100 orbitals; spin-down FODs at centres 100..199.
    "mol192": dict(n=192, h=0.15, n_atoms=200, n_gauss=200, nocc=(100, 100), atom_box=20.0,
                   down_offset=100, seed=2508),
}

BATCH24_SEED = 2308


def _backend(device):
    if device is None or device == "numpy":
        return None
    if torch is None:
        raise RuntimeError("torch is required for device generation")
    return torch.device(device)


def _coords(n, h, origin, dev):
    if dev is None:
        axes = [origin[d] + h * np.arange(n[d], dtype=np.float64) for d in range(3)]
        return axes
    return [torch.tensor(origin[d], dtype=torch.float64, device=dev)
            + h * torch.arange(n[d], dtype=torch.float64, device=dev) for d in range(3)]


def _gaussians(n, h, origin, centres, kinds, alphas, dev):
    """(N_g, M) Gaussian primitives normalised on the grid."""
    xs, ys, zs = _coords(n, h, origin, dev)
    M = n[0] * n[1] * n[2]
    dV = h ** 3
    ng = len(kinds)
    if dev is None:
        out = np.empty((ng, M))
    else:
        out = torch.empty((ng, M), dtype=torch.float64, device=dev)
    for g in range(ng):
        X, Y, Z = centres[g]
        a = alphas[g]
        if dev is None:
            ex = np.exp(-a * (xs - X) ** 2)
            ey = np.exp(-a * (ys - Y) ** 2)
            ez = np.exp(-a * (zs - Z) ** 2)
            fx = (xs - X) * ex if kinds[g] == 1 else ex
            fy = (ys - Y) * ey if kinds[g] == 2 else ey
            fz = (zs - Z) * ez if kinds[g] == 3 else ez
            f = (fz[:, None, None] * fy[None, :, None] * fx[None, None, :]).reshape(-1)
            f /= math.sqrt(dV * float(f @ f))
        else:
            ex = torch.exp(-a * (xs - X) ** 2)
            ey = torch.exp(-a * (ys - Y) ** 2)
            ez = torch.exp(-a * (zs - Z) ** 2)
            fx = (xs - X) * ex if kinds[g] == 1 else ex
            fy = (ys - Y) * ey if kinds[g] == 2 else ey
            fz = (zs - Z) * ez if kinds[g] == 3 else ez
            f = (fz[:, None, None] * fy[None, :, None] * fx[None, None, :]).reshape(-1)
            f = f / torch.sqrt(dV * torch.dot(f, f))
        out[g] = f
    return out


def _orthonormalise(raw, dV, dev):
    """psi = G^{-1/2} raw with G = dV raw raw^T (two passes for round-off)."""
    psi = raw
    for _ in range(2):
        if dev is None:
            G = dV * (psi @ psi.T)
            w, V = np.linalg.eigh(G)
            Zm = (V / np.sqrt(w)) @ V.T
            psi = Zm @ psi
        else:
            G = dV * (psi @ psi.T)
            Gc = G.cpu().numpy()
            w, V = np.linalg.eigh(Gc)
            Zm = torch.tensor((V / np.sqrt(w)) @ V.T, dtype=torch.float64, device=dev)
            psi = Zm @ psi
    return psi


def _nearest_density(psi, n, h, origin, a, dev):
    idx = [int(round((a[d] - origin[d]) / h)) for d in range(3)]
    idx = [min(max(idx[d], 0), n[d] - 1) for d in range(3)]
    m = (idx[2] * n[1] + idx[1]) * n[0] + idx[0]
    col = psi[:, m]
    if dev is not None:
        col = col.cpu().numpy()
    return float(np.sum(col ** 2))


def make_molecule(name: str, n: int, h: float, n_atoms: int, n_gauss: int, nocc: Sequence[int],
                  seed: int, atom_box: Optional[float] = None, down_offset: int = 0,
                  device=None, jitter: float = 0.3) -> System:
    """One synthetic molecule following the recipe in the module docstring."""
    dev = _backend(device)
    rng = np.random.Generator(np.random.PCG64(seed))
    nn = (n, n, n)
    origin = np.full(3, -h * (n - 1) / 2.0)
    L = (n - 1) * h
    edge = atom_box if atom_box is not None else L / 3.0
    atoms = rng.uniform(-edge / 2.0, edge / 2.0, size=(n_atoms, 3))
    kinds = rng.integers(0, 4, size=n_gauss)
    alphas = np.exp(rng.uniform(math.log(0.3), math.log(3.0), size=n_gauss))
    centres = atoms[np.arange(n_gauss) % n_atoms]
    g = _gaussians(nn, h, origin, centres, kinds, alphas, dev)
    dV = h ** 3
    psis = []
    for s, N in enumerate(nocc):
        C = rng.standard_normal((N, n_gauss))
        if dev is None:
            raw = C @ g
        else:
            raw = torch.tensor(C, dtype=torch.float64, device=dev) @ g
        psis.append(_orthonormalise(raw, dV, dev))
    del g
    fods = []
    for s, N in enumerate(nocc):
        off = 0 if s == 0 else down_offset
        base = atoms[(off + np.arange(N)) % n_atoms]
        k = 0
        while True:
            jr = np.random.Generator(np.random.PCG64(seed + 1000 * k + 17 * (s + 1)))
            f = base + jr.normal(0.0, jitter, size=(N, 3))
            dens = min(_nearest_density(psis[s], nn, h, origin, f[i], dev) for i in range(N))
            if dens >= 1e-8 or k >= 20:
                break
            k += 1
        fods.append(np.ascontiguousarray(f))
    return System(name=name, n=nn, h=h, origin=origin, nocc=tuple(nocc), psi=psis, fod=fods,
                  atoms=atoms, seed=seed)


def make_workload(name: str, device=None) -> System:
    w = WORKLOADS[name]
    return make_molecule(name, w["n"], w["h"], w["n_atoms"], w["n_gauss"], w["nocc"], w["seed"],
                         atom_box=w["atom_box"], down_offset=w["down_offset"], device=device)


def batch24_specs(count: int = 24, seed: int = BATCH24_SEED) -> List[dict]:
    """Uneven systems: n ~ U{48..128}, h ~ U[0.2, 0.3], N_up ~ U{2..40},
    N_down = N_up - Bernoulli(1/2), N_g = ceil(2.4 N_up), one atom per
    spin-up orbital."""
    specs = []
    for k in range(count):
        rng = np.random.Generator(np.random.PCG64(seed + k))
        n = int(rng.integers(48, 129))
        h = float(rng.uniform(0.2, 0.3))
        nup = int(rng.integers(2, 41))
        ndn = nup - int(rng.integers(0, 2))
        specs.append(dict(name=f"batch24_{k}", n=n, h=h, n_atoms=nup,
                          n_gauss=int(math.ceil(2.4 * nup)), nocc=(nup, ndn),
                          seed=seed + 10000 + k))
    return specs


def make_batch24(device=None, count: int = 24) -> List[System]:
    return [make_molecule(s["name"], s["n"], s["h"], s["n_atoms"], s["n_gauss"], s["nocc"],
                          s["seed"], device=device) for s in batch24_specs(count)]


def gaussian_charge(n: int, h: float, sigma: float, centre=(0.0, 0.0, 0.0), q: float = 1.0):
    """Normalised Gaussian charge q (2 pi sigma^2)^{-3/2} exp(-|r-c|^2 / (2 sigma^2))
    sampled on the node-centred n^3 grid (shape (n, n, n), z slowest)."""
    origin = -h * (n - 1) / 2.0
    x = origin + h * np.arange(n)
    dx = x - centre[0]
    dy = x - centre[1]
    dz = x - centre[2]
    r2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
    return q * (2 * math.pi * sigma ** 2) ** -1.5 * np.exp(-r2 / (2 * sigma ** 2))
