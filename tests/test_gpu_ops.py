"""Operator-level parity of the HIP kernels against the CPU oracle, through
the C ABI: the star Laplacian (FP64 and FP32), the LSDA pointwise kernel,
the device Jacobi S^{-1/2}, and the multipole-BC Poisson solver."""
import copy
import math

import numpy as np
import pytest

from paper_2108_01186_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def F():
    from paper_2108_01186_amd import fsic
    return fsic


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("shape,fd_order", [((29, 37, 45), 12), ((16, 16, 16), 12), ((20, 33, 70), 8),
                                            ((9, 10, 11), 2), ((40, 40, 40), 12), ((17, 48, 33), 6)])
def test_laplacian_fp64(torch_cuda, F, oracle, shape, fd_order):
    torch = torch_cuda
    _say(f"laplacian fp64 shape={shape} order={fd_order}")
    rng = np.random.default_rng(sum(shape) + fd_order)
    u = rng.standard_normal((2,) + shape)
    h = 0.27
    out = F.op_laplacian(torch.tensor(u, device="cuda"), h, fd_order).cpu().numpy()
    for f in range(2):
        ref = oracle.apply_laplacian(u[f], h, fd_order // 2)
        err = np.abs(out[f] - ref).max() / np.abs(ref).max()
        assert err < 1e-14, err


def test_laplacian_fp32(torch_cuda, F, oracle):
    torch = torch_cuda
    _say("laplacian fp32 (23,31,50)")
    rng = np.random.default_rng(5)
    u = rng.standard_normal((23, 31, 50))
    h = 0.2
    out = F.op_laplacian(torch.tensor(u, device="cuda", dtype=torch.float32), h, 12).cpu().numpy()
    ref = oracle.apply_laplacian(u.astype(np.float32).astype(np.float64), h, 6)
    # FP32 sum of 37 terms of magnitude ~ |c_0| max|u| / h^2: rounding ~ 1e-6 relative
    assert np.abs(out - ref).max() / np.abs(ref).max() < 2e-6


def test_xc_pointwise(torch_cuda, F, oracle):
    torch = torch_cuda
    _say("xc pointwise")
    rho = np.concatenate([[0.0, 1e-40, 1e-30, 2e-30], np.logspace(-14, 3, 400)])
    outs = [o.cpu().numpy() for o in F.op_xc(torch.tensor(rho, device="cuda"))]
    ref = oracle.xc_pol(rho)
    for k in range(4):
        err = np.abs(outs[k] - ref[k]) / np.maximum(np.abs(ref[k]), 1e-300)
        assert np.all(err < 1e-13), (k, err.max())
    assert np.all(outs[0][:3] == 0)


@pytest.mark.parametrize("N", [1, 2, 5, 16, 31, 64, 100])
def test_invsqrt(torch_cuda, F, N):
    torch = torch_cuda
    _say(f"invsqrt N={N}")
    rng = np.random.default_rng(N)
    B = rng.standard_normal((N, N))
    S = B @ B.T / N + 0.05 * np.eye(N)
    Z, lam = F.op_invsqrt(torch.tensor(S, device="cuda"))
    Z = Z.cpu().numpy()
    w, V = np.linalg.eigh(S)
    Zref = (V / np.sqrt(w)) @ V.T
    assert np.abs(Z - Zref).max() < 1e-11 * np.abs(Zref).max() * max(1, np.linalg.cond(S) / 1e3)
    assert np.allclose(np.sort(lam.cpu().numpy()), w, rtol=1e-12, atol=1e-13)
    assert np.abs(Z @ S @ Z - np.eye(N)).max() < 1e-11 * np.linalg.cond(S)


@pytest.mark.parametrize("n,h,precision,solver", [(40, 0.3, "fp64", "cg"), (33, 0.25, "fp64", "cg"),
                                                   (40, 0.3, "mixed", "cg"), (40, 0.3, "fp64", "pcg"),
                                                   (33, 0.25, "fp64", "pcg"), (40, 0.3, "mixed", "pcg"),
                                                   (40, 0.3, "fp64", "aar"), (33, 0.25, "fp64", "aar")])
def test_poisson_vs_oracle(torch_cuda, F, oracle, n, h, precision, solver):
    torch = torch_cuda
    _say(f"poisson n={n} h={h} {precision} {solver}")
    origin = np.full(3, -h * (n - 1) / 2)
    rhos = [synth.gaussian_charge(n, h, 0.8, centre=(0.5, -0.3, 0.2)),
            synth.gaussian_charge(n, h, 0.6, centre=(-1.0, 0.7, -0.4))
            + 0.3 * synth.gaussian_charge(n, h, 1.1, centre=(1.2, 0.0, 0.9))]
    rho = np.stack([r.reshape(-1) for r in rhos])
    v, it, rr = F.op_poisson(torch.tensor(rho, device="cuda"), (n, n, n), h, origin, tol=1e-12,
                             precision=precision, solver=solver)
    v = v.cpu().numpy()
    assert np.all(rr <= 1e-12), rr
    if solver == "pcg":
        assert np.all(it < 40), it  # the spectral preconditioner leaves only the face corrections
    for f in range(2):
        ref, _, _ = oracle.poisson(rho[f], (n, n, n), h, origin)
        # |dv| <= ||K^{-1}|| ||r||: relative 1e-12 residual leaves ~1e-10 in v
        assert np.abs(v[f] - ref).max() < 1e-9 * np.abs(ref).max(), np.abs(v[f] - ref).max()
        U = 0.5 * h ** 3 * rho[f] @ v[f]
        Uref = 0.5 * h ** 3 * rho[f] @ ref
        assert abs(U - Uref) < 1e-10


@pytest.mark.parametrize("lmax", [0, 3, 8])
def test_poisson_multipole_orders(torch_cuda, F, oracle, lmax):
    """Boundary values at other multipole orders (Sec. II.A): the harmonic
    tiles of the moment and ghost contractions change with lmax (one to six
    16-row tiles); off-centre charges on a non-cubic grid make every order
    matter.  Against the oracle at the same order."""
    torch = torch_cuda
    n = (37, 29, 45)
    h = 0.3
    _say(f"poisson lmax={lmax} {n}")
    origin = np.array([-h * (m - 1) / 2 for m in n])
    axes = [origin[d] + h * np.arange(n[d]) for d in range(3)]
    rhos = []
    for c, s in (((1.1, -0.6, 0.9), 0.7), ((-0.8, 0.9, -1.3), 0.5), ((0.3, 0.2, -0.1), 0.9)):
        r2 = ((axes[2][:, None, None] - c[2]) ** 2 + (axes[1][None, :, None] - c[1]) ** 2
              + (axes[0][None, None, :] - c[0]) ** 2)
        rhos.append((np.exp(-r2 / (2 * s * s)) / (2 * np.pi * s * s) ** 1.5).reshape(-1))
    rho = np.stack(rhos)
    v, it, rr = F.op_poisson(torch.tensor(rho, device="cuda"), n, h, origin, lmax=lmax, tol=1e-12,
                             precision="mixed", solver="pcg")
    v = v.cpu().numpy()
    assert np.all(rr <= 1e-12), rr
    for f in range(len(rhos)):
        ref, _, _ = oracle.poisson(rho[f], n, h, origin, lmax=lmax)
        assert np.abs(v[f] - ref).max() < 1e-9 * np.abs(ref).max(), (f, np.abs(v[f] - ref).max())


@pytest.mark.parametrize("precision,n", [("fp64", (37, 29, 45)), ("mixed", (37, 29, 45)),
                                         ("fp64", (136, 21, 18)), ("mixed", (19, 150, 17)),
                                         ("fp64", (190, 14, 12)), ("mixed", (12, 13, 185)),
                                         ("fp64", (230, 9, 10)), ("mixed", (230, 9, 10))])
def test_pcg_non_cubic_grid(torch_cuda, F, oracle, precision, n):
    """Preconditioned solve on a box with a different node count per axis
    (ragged tiles of every sine transform), against the oracle.  The longest
    axis picks the transform variant: <= 128 nodes 128-column split-bf16
    panels, 136-150 64-column ones, 185-190 the bf16 sine matrix without its
    low part; no variant fits 230 nodes in LDS, so that batch is solved by
    plain CG (same tolerance, many more iterations)."""
    torch = torch_cuda
    _say(f"pcg non-cubic {precision} {n}")
    h = 0.28
    origin = np.array([-h * (m - 1) / 2 for m in n])
    axes = [origin[d] + h * np.arange(n[d]) for d in range(3)]
    r2 = ((axes[2][:, None, None] - 0.3) ** 2 + (axes[1][None, :, None] + 0.2) ** 2
          + (axes[0][None, None, :] - 0.5) ** 2)
    rho = (np.exp(-r2 / (2 * 0.7 ** 2)) + 0.2 * np.exp(-r2 / 3.0)).reshape(1, -1)
    v, it, rr = F.op_poisson(torch.tensor(rho, device="cuda"), n, h, origin, tol=1e-12,
                             precision=precision, solver="pcg")
    assert rr[0] <= 1e-12, (rr, it)
    assert (it[0] < 40) == (max(n) <= 208), (rr, it)
    ref, _, _ = oracle.poisson(rho[0], n, h, origin)
    assert np.abs(v.cpu().numpy()[0] - ref).max() < 1e-9 * np.abs(ref).max()


_POISSON_REF = {}


@pytest.mark.parametrize("fused", ["0", "1"])
@pytest.mark.parametrize("n", [(40, 40, 40), (37, 29, 45), (12, 13, 185), (96, 64, 50)])
def test_pcg_fused_and_five_pass_transforms(torch_cuda, F, oracle, n, fused, monkeypatch):
    """The preconditioner with both in-plane transforms fused per z plane (the
    default where the plane fits in LDS) and with five separate passes
    (FSIC_DST_XY=0): vector and single-value plane access, equal and unequal
    in-plane axes, a long z axis beside a small plane; both reach the
    tolerance in a few iterations and agree with the oracle."""
    torch = torch_cuda
    _say(f"pcg transforms fused={fused} {n}")
    monkeypatch.setenv("FSIC_DST_XY", fused)
    h = 0.3
    origin = np.array([-h * (m - 1) / 2 for m in n])
    axes = [origin[d] + h * np.arange(n[d]) for d in range(3)]
    r2 = ((axes[2][:, None, None] + 0.4) ** 2 + (axes[1][None, :, None] - 0.1) ** 2
          + (axes[0][None, None, :] - 0.3) ** 2)
    rho = np.stack([np.exp(-r2 / (2 * 0.8 ** 2)).reshape(-1), (np.exp(-r2 / 2.5) * (1 + 0.3 * np.cos(r2))).reshape(-1)])
    v, it, rr = F.op_poisson(torch.tensor(rho, device="cuda"), n, h, origin, tol=1e-12,
                             precision="fp64", solver="pcg")
    assert max(rr) <= 1e-12 and max(it) < 40, (rr, it)
    v = v.cpu().numpy()
    for k in range(2):
        if (n, k) not in _POISSON_REF:
            _POISSON_REF[n, k] = oracle.poisson(rho[k], n, h, origin)[0]
        ref = _POISSON_REF[n, k]
        assert np.abs(v[k] - ref).max() < 1e-9 * np.abs(ref).max(), k


@pytest.mark.parametrize("fused", ["0", "1"])
@pytest.mark.parametrize("n", [(37, 29, 45), (96, 64, 50), (12, 13, 185)])
def test_aar_non_cubic_grid(torch_cuda, F, oracle, n, fused, monkeypatch):
    """Alternating Anderson-Richardson with the sine-transform preconditioner
    (both transform layouts) on unequal axes and several densities at once:
    the FP64 residual meets the tolerance within a few tens of iterations and
    the potentials match the oracle."""
    torch = torch_cuda
    _say(f"aar fused={fused} {n}")
    monkeypatch.setenv("FSIC_DST_XY", fused)
    h = 0.3
    origin = np.array([-h * (m - 1) / 2 for m in n])
    axes = [origin[d] + h * np.arange(n[d]) for d in range(3)]
    r2 = ((axes[2][:, None, None] + 0.4) ** 2 + (axes[1][None, :, None] - 0.1) ** 2
          + (axes[0][None, None, :] - 0.3) ** 2)
    rho = np.stack([np.exp(-r2 / (2 * 0.8 ** 2)).reshape(-1), (np.exp(-r2 / 2.5) * (1 + 0.3 * np.cos(r2))).reshape(-1)])
    v, it, rr = F.op_poisson(torch.tensor(rho, device="cuda"), n, h, origin, tol=1e-12,
                             precision="fp64", solver="aar")
    assert max(rr) <= 1e-12 and max(it) < 60, (rr, it)
    v = v.cpu().numpy()
    for k in range(2):
        if (n, k) not in _POISSON_REF:
            _POISSON_REF[n, k] = oracle.poisson(rho[k], n, h, origin)[0]
        ref = _POISSON_REF[n, k]
        assert np.abs(v[k] - ref).max() < 1e-9 * np.abs(ref).max(), k


def test_aar_needs_fp64(torch_cuda, F):
    with pytest.raises(F.FsicError):
        F.Context(precision="mixed", solver="aar")


def test_poisson_gaussian_closed_form(torch_cuda, F):
    torch = torch_cuda
    _say("poisson gaussian self-energy")
    n, h, sigma = 40, 0.3, 1.0
    rho = synth.gaussian_charge(n, h, sigma).reshape(1, -1)
    v, it, rr = F.op_poisson(torch.tensor(rho, device="cuda"), (n, n, n), h,
                             np.full(3, -h * (n - 1) / 2), tol=1e-12)
    U = 0.5 * h ** 3 * float(rho[0] @ v.cpu().numpy()[0])
    assert abs(U - 1 / (2 * math.sqrt(math.pi) * sigma)) < 2e-9


@pytest.mark.parametrize("fd_gradient", [False, True])
def test_interp_vs_oracle(torch_cuda, F, oracle, fd_gradient):
    """psi and grad psi at points (Sec. II.B) against the oracle, with points
    whose stencils touch the first and last node of each axis (where the
    per-node differences turn one-sided) on a non-cubic grid."""
    torch = torch_cuda
    _say(f"interp fd_gradient={fd_gradient}")
    rng = np.random.default_rng(5)
    n, h = (13, 17, 11), 0.3
    origin = np.array([-1.0, 0.5, -2.0])
    N = 7
    psi = rng.normal(size=(N, n[0] * n[1] * n[2]))
    cells = [(1, 1, 1), (n[0] - 3, n[1] - 3, n[2] - 3), (1, n[1] - 3, 4), (5, 1, n[2] - 3),
             (2, 7, 2), (n[0] - 4, 3, 5)]
    pts = np.array([origin + h * (np.array(c) + rng.uniform(0, 1, 3)) for c in cells]
                   + [origin + h * rng.uniform([1, 1, 1], [n[0] - 2, n[1] - 2, n[2] - 2]) for _ in range(10)])
    u, du = F.op_interp(torch.tensor(psi, device="cuda"), pts, n, h, origin, fd_gradient=fd_gradient)
    u, du = u.cpu().numpy(), du.cpu().numpy()
    for k, p in enumerate(pts):
        ru, rdu = (oracle.interp_fdgrad if fd_gradient else oracle.interp)(psi, n, h, origin, p)
        assert np.abs(u[k] - ru).max() < 1e-13, k
        assert np.abs(du[k] - rdu).max() < 1e-12, (k, np.abs(du[k] - rdu).max())
    bad = origin + h * np.array([[0.5, 3.2, 3.2]])  # cell 0: stencil leaves the grid
    with pytest.raises(F.FsicError):
        F.op_interp(torch.tensor(psi, device="cuda"), bad, n, h, origin, fd_gradient=fd_gradient)


@pytest.mark.parametrize("case", ["mol40", "n20", "n45", "n70"])
def test_fermi_loewdin_orbitals(torch_cuda, F, oracle, mol40, case):
    """T (Eq. 8), the FO overlap S, S^{-1/2} and the FLOs against the oracle;
    n20 spans two 16-wide matrix-core tiles with a ragged tail, n45 and n70
    take the staged products (three and five tiles: the symmetric Gram splits
    its tile triangle over the waves by rows)."""
    torch = torch_cuda
    _say(f"flo {case}")
    sizes = {"n20": (36, 20, 91), "n45": (36, 45, 92), "n70": (40, 70, 93)}
    if case == "mol40":
        s = mol40
    else:
        nn, N, seed = sizes[case]
        s = synth.make_molecule(case, nn, 0.3, N, int(np.ceil(2.4 * N)), (N,), seed=seed)
    psi = np.asarray(s.psi[0])
    N = psi.shape[0]
    T, G, S, Z, phi = F.op_flo(torch.tensor(psi, device="cuda"), s.fod[0], s.n, s.h, s.origin)
    if case in ("mol40", "n20"):
        r = oracle.sic_spin(psi, s.fod[0], s.n, s.h, s.origin, keep_fields=True)
        rphi, rT, rS, rZ = r.phi, r.T, r.S, r.Z
    else:  # the FLO stage alone: no Poisson solves of 45 or 70 orbitals
        rphi, rT, rS, rZ = oracle.flo_spin(psi, s.fod[0], s.n, s.h, s.origin)
    T, G, S, Z, phi = (x.cpu().numpy() for x in (T, G, S, Z, phi))
    assert np.abs(T - rT).max() < 1e-12
    assert np.abs(G - np.eye(N)).max() < 1e-12
    assert np.abs(S - rS).max() < 1e-12
    cond = np.linalg.cond(rS)
    assert np.abs(Z - rZ).max() < 1e-13 * cond * np.abs(rZ).max()
    assert np.abs(phi - rphi).max() < 1e-13 * cond * np.abs(rphi).max()


@pytest.mark.parametrize("n,fd_order", [((37, 29, 45), 12), ((40, 40, 40), 8)])
def test_hamiltonian_vs_oracle(torch_cuda, F, oracle, n, fd_order):
    """-1/2 L psi + v psi on three orbitals with a random potential (ragged
    tiles, two stencil orders), against the oracle."""
    torch = torch_cuda
    _say(f"hamiltonian {n} order {fd_order}")
    rng = np.random.default_rng(7)
    M = n[0] * n[1] * n[2]
    psi = rng.standard_normal((3, M))
    v = rng.standard_normal(M)
    h = 0.27
    out = F.op_hamiltonian(torch.tensor(psi, device="cuda"), torch.tensor(v, device="cuda"), n, h,
                           fd_order=fd_order).cpu().numpy()
    ref = oracle.hamiltonian(psi.reshape(3, n[2], n[1], n[0]), v.reshape(n[2], n[1], n[0]), h,
                             p=fd_order // 2).reshape(3, M)
    assert np.abs(out - ref).max() < 1e-12 * np.abs(ref).max()


def test_hamiltonian_with_sic_potential(torch_cuda, F, oracle, mol40):
    """H psi with the Slater-averaged V_SIC of a forward pass as the potential."""
    torch = torch_cuda
    _say("hamiltonian with V_SIC")
    s = mol40
    psi = torch.tensor(np.asarray(s.psi[0]), device="cuda")
    sd = copy.copy(s)
    sd.psi = [psi]
    out = F.sic_energy([sd])
    vs = out["vsic"][0][0]
    hp = F.op_hamiltonian(psi, vs, s.n, s.h).cpu().numpy()
    ref = oracle.hamiltonian(np.asarray(s.psi[0]).reshape(5, *s.n[::-1]),
                             vs.cpu().numpy().reshape(*s.n[::-1]), s.h).reshape(5, -1)
    assert np.abs(hp - ref).max() < 1e-12 * np.abs(ref).max()
