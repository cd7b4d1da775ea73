"""Pins of the oracle fixed point (Algorithm 1).

P7: on tiny grids the converged fields equal a direct least-squares solve of
    the discrete finite-difference equilibrium D(u^f + u*) = 0 on the kept
    nodes, assembled column by column (random two-phase elastic problems,
    random per-face, per-component BCs, both schemes, both Green operators).
P8: a homogeneous body under affine-compatible BCs converges to the exact
    affine field (the FD gradient of an affine field is exact).
P9: a periodic two-phase laminate with layers on node planes reproduces the
    analytic laminate strains (continuity of traction, mean strain imposed).
P10: <sigma> does not depend on lambda0, mu0, the Green operator or the
    Anderson settings (within the solver tolerance).
P11: a homogeneous J2 body under uniaxial stress (u_z Dirichlet on z faces,
    all other faces / components Neumann) follows the bilinear closed form.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dt, fd, solver
from oracle.laws import MaterialSet


def _residual_operator(prob):
    pl = solver.Plan(prob)
    mats = MaterialSet(prob.materials, np.asarray(prob.mat_id).transpose(2, 1, 0))
    state = mats.init_state(pl.nppv, pl.n)
    step = prob.steps[0]
    us = pl.ustar(step.c, step.G, step.H)

    def D_of(uf):
        gu = pl.grad(uf) + pl.grad(us)
        eps = 0.5 * (gu + np.swapaxes(gu, -1, -2))
        sig, _ = mats.stress(eps, state, 1.0)
        return pl.div(sig), eps, sig

    return pl, D_of


def _direct_solve(prob):
    pl, D_of = _residual_operator(prob)
    shape = (3,) + tuple(v + 1 for v in pl.n)
    idx = [np.argwhere(pl.kept[q]) for q in range(3)]
    cols = [(q, tuple(i)) for q in range(3) for i in idx[q]]
    rows = cols
    z = np.zeros(shape)
    D0 = D_of(z)[0]
    b = -np.array([D0[q][i] for q, i in rows])
    A = np.zeros((len(rows), len(cols)))
    for c, (q, i) in enumerate(cols):
        e = np.zeros(shape)
        e[q][i] = 1.0
        for qq in range(3):
            fd.zero_dismissed(e[qq], pl.exts[qq])
        Dc = D_of(e)[0]
        A[:, c] = [Dc[qq][ii] for qq, ii in rows] + b
    x = np.linalg.lstsq(A, b, rcond=1e-12)[0]
    uf = np.zeros(shape)
    for (q, i), v in zip(cols, x):
        uf[q][i] = v
    for q in range(3):
        fd.zero_dismissed(uf[q], pl.exts[q])
    D, eps, sig = D_of(uf)
    return eps, sig, np.abs(A @ x - b).max()


@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
@pytest.mark.parametrize("seed", range(4))
def test_fixed_point_equals_direct_solve(scheme, seed):
    rng = np.random.default_rng(1000 + seed)
    n = (4, 3, 5) if seed % 2 else (3, 4, 4)
    prob = W.random_small_problem(rng, n=n, scheme=scheme, tol=1e-12)
    prob.green = seed % 2
    eps_d, sig_d, res = _direct_solve(prob)
    assert res < 1e-10
    r = solver.solve(prob)
    assert r["converged"][0]
    sig = r["sig"]
    ref = np.stack([sig_d[..., i, j] for (i, j) in solver.VOIGT]).transpose(0, 1, 4, 3, 2)
    scale = np.abs(ref).max()
    np.testing.assert_allclose(sig, ref, atol=1e-8 * scale)


@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
def test_homogeneous_affine(scheme):
    n = (6, 5, 7)
    bc = np.full((3, 3, 2), W.N, dtype=np.int32)
    bc[2, 2, :] = W.D
    bc[:, 1, :] = W.P
    lam, mu = W.iso_from_E_nu(2.0, 0.3)
    G = np.zeros((3, 3)); G[2, 2] = 1e-3
    prob = W.Problem(n=n, h=1.0, bc=bc, scheme=scheme, green=W.GREEN_B0, lambda0=lam,
                     mu0=mu, materials=[W.mat_iso(lam, mu)],
                     mat_id=np.zeros((n[2], n[1], n[0]), dtype=np.int32),
                     steps=[W.step_affine(G)], tol=1e-12, max_iter=500)
    r = solver.solve(prob)
    assert r["converged"][0]
    # y periodic with <eps_yy> = 0: plane strain in y, free contraction in x
    nu = 0.3
    exp = np.array([-nu / (1 - nu) * 1e-3, 0.0, 1e-3, 0, 0, 0])
    for a in range(6):
        np.testing.assert_allclose(r["eps"][a], exp[a], atol=1e-13)
    np.testing.assert_allclose(r["sig"][2], 2.0 / (1 - nu ** 2) * 1e-3, rtol=1e-10)


@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
def test_periodic_laminate(scheme):
    n = (4, 3, 8)
    k = 3                                     # voxels 0..k-1 along z are phase 1
    ids = np.zeros((n[2], n[1], n[0]), dtype=np.int32)
    ids[:k] = 1
    mA = W.iso_from_E_nu(1.0, 0.3)
    mB = W.iso_from_E_nu(7.0, 0.2)
    E = np.array([[1e-3, 2e-4, -3e-4], [2e-4, -5e-4, 4e-4], [-3e-4, 4e-4, 8e-4]])
    prob = W.Problem(n=n, h=1.0, bc=np.zeros((3, 3, 2), dtype=np.int32), scheme=scheme,
                     green=W.GREEN_B0, lambda0=max(mA[0], mB[0]), mu0=max(mA[1], mB[1]),
                     materials=[W.mat_iso(*mA), W.mat_iso(*mB)], mat_id=ids,
                     steps=[W.step_affine(E)], tol=1e-12, max_iter=2000)
    r = solver.solve(prob)
    assert r["converged"][0]
    # analytic: eps_k = E + sym(a_k x e3), f_B a_B + f_A a_A = 0, traction continuous
    fB, fA = k / n[2], 1 - k / n[2]

    def C(lam, mu):
        d = np.eye(3)
        return lam * np.einsum("ij,kl->ijkl", d, d) + mu * (np.einsum("ik,jl->ijkl", d, d)
                                                             + np.einsum("il,jk->ijkl", d, d))
    CA, CB = C(*mA), C(*mB)
    e3 = np.array([0.0, 0.0, 1.0])

    def trac(Cm, a):
        eps = E + 0.5 * (np.outer(a, e3) + np.outer(e3, a))
        return np.einsum("ijkl,kl->ij", Cm, eps) @ e3

    # linear in aA (aB = -fA/fB aA): solve trac(CA, aA) = trac(CB, aB)
    M = np.zeros((3, 3)); rhs = trac(CB, np.zeros(3)) - trac(CA, np.zeros(3))
    for j in range(3):
        a = np.zeros(3); a[j] = 1.0
        M[:, j] = (trac(CA, a) - trac(CA, 0 * a)) - (trac(CB, -fA / fB * a) - trac(CB, 0 * a))
    aA = np.linalg.solve(M, rhs)
    aB = -fA / fB * aA
    for zsl, a in ((slice(0, k), aB), (slice(k, None), aA)):
        eps = E + 0.5 * (np.outer(a, e3) + np.outer(e3, a))
        for c, (i, j) in enumerate(solver.VOIGT):
            np.testing.assert_allclose(r["eps"][c][:, zsl], eps[i, j], atol=1e-12)


def test_invariance_to_reference_medium_and_acceleration():
    rng = np.random.default_rng(77)
    base = W.random_small_problem(rng, n=(5, 6, 4), scheme=W.TETRA2, tol=1e-11)
    ref = solver.solve(base)["macro_sigma"][0]
    variants = []
    for lam_f, mu_f, green, depth, period in ((0.5, 1.3, 0, 4, 3), (2.0, 0.8, 0, 1, 3),
                                              (1.0, 1.0, 1, 3, 2), (1.0, 2.0, 0, 4, 2)):
        p = W.random_small_problem(np.random.default_rng(77), n=(5, 6, 4), scheme=W.TETRA2,
                                   tol=1e-11)
        p.lambda0 *= lam_f; p.mu0 *= mu_f; p.green = green
        p.aa_depth = depth; p.aa_period = period
        variants.append(solver.solve(p)["macro_sigma"][0])
    for v in variants:
        np.testing.assert_allclose(v, ref, atol=1e-9 * np.abs(ref).max())


def test_j2_uniaxial_stress_bilinear():
    n = (3, 3, 4)
    E, nu, sy0, H = 70.0, 0.33, 0.1, 1.0
    lam, mu = W.iso_from_E_nu(E, nu)
    bc = np.full((3, 3, 2), W.N, dtype=np.int32)
    bc[2, 2, :] = W.D
    steps = []
    ez = np.linspace(0, 5e-3, 11)[1:]
    for e in ez:
        s = W.LoadStep(); s.G[2, 2] = e
        steps.append(s)
    prob = W.Problem(n=n, h=1.0, bc=bc, scheme=W.HEX1, green=W.GREEN_B0, lambda0=lam,
                     mu0=mu, materials=[W.mat_j2(lam, mu, sy0, H)],
                     mat_id=np.zeros((n[2], n[1], n[0]), dtype=np.int32), steps=steps,
                     tol=1e-12, max_iter=800)
    r = solver.solve(prob)
    assert all(r["converged"])
    ey = sy0 / E
    Et = E * H / (E + H)
    for t, e in enumerate(ez):
        exact = E * e if e <= ey else sy0 + Et * (e - ey)
        assert r["macro_sigma"][t][2] == pytest.approx(exact, rel=1e-9)
        assert abs(r["macro_sigma"][t][0]) < 1e-9


def test_mixed_control_uniaxial_stress_j2():
    """C3's boundary conditions on a homogeneous J2 body: x, y periodic, z faces
    u_z Dirichlet / u_x, u_y Neumann, <sigma_xx> = <sigma_yy> = 0 enforced by
    the mixed update -> uniaxial stress, bilinear closed form."""
    n = (3, 4, 4)
    E, nu, sy0, H = 70.0, 0.33, 0.1, 1.0
    lam, mu = W.iso_from_E_nu(E, nu)
    bc = np.zeros((3, 3, 2), dtype=np.int32)
    bc[0, 2, :] = W.N; bc[1, 2, :] = W.N; bc[2, 2, :] = W.D
    steps = []
    ez = np.linspace(0, 4e-3, 9)[1:]
    for e in ez:
        s = W.LoadStep(); s.G[2, 2] = e
        s.mixed_mask = np.array([1, 1, 0, 0, 0, 0], dtype=np.int32)
        steps.append(s)
    prob = W.Problem(n=n, h=1.0, bc=bc, scheme=W.HEX1, green=W.GREEN_B0, lambda0=lam,
                     mu0=mu, materials=[W.mat_j2(lam, mu, sy0, H)],
                     mat_id=np.zeros((n[2], n[1], n[0]), dtype=np.int32), steps=steps,
                     tol=1e-11, max_iter=800)
    r = solver.solve(prob)
    assert all(r["converged"])
    ey = sy0 / E
    Et = E * H / (E + H)
    for t, e in enumerate(ez):
        exact = E * e if e <= ey else sy0 + Et * (e - ey)
        assert r["macro_sigma"][t][2] == pytest.approx(exact, rel=1e-8)
        assert abs(r["macro_sigma"][t][0]) < 1e-10 * exact


@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
def test_cantilever_beam_theory(scheme):
    """P14 (approximate): the cantilever under a uniform load on its top face
    (Sec. 3.1.1, Eq. analytical_sol_bending_elastic_own_weight) deflects as
    beam theory predicts to within the shear-deformation and discretisation
    gap of a coarse 40 x 4 x 4 grid (about 7 % HEX1, 2 % TETRA2)."""
    n = (40, 4, 4)
    prob = W.cantilever(n=n, t2=1e-3, scheme=scheme, tol=1e-8)
    r = solver.solve(prob)
    assert r["converged"][0]
    lam, mu = 120.0, 80.0
    E = mu * (3 * lam + 2 * mu) / (lam + mu)
    I = n[2] * n[1] ** 3 / 12.0
    L = n[0]
    tip = -1e-3 * n[2] * L ** 4 / (8.0 * E * I)
    uy = r["u"][1][n[2] // 2, n[1] // 2, -1]
    assert 0.97 < uy / tip < 1.10
    # the load is carried: the clamped face reacts the applied force
    assert r["macro_sigma"][0][5] != 0.0


@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
@pytest.mark.parametrize("seed", range(3))
def test_c0_fixed_point_equals_b0(scheme, seed):
    """P10 for the C0 operator: on normal-mixed conditions (Eq. SGO_BCs) the
    C0-preconditioned iteration converges to the same discrete equilibrium as
    the B0 one (stress field and <sigma>), and to the direct solve."""
    rng = np.random.default_rng(400 + seed)
    choice = rng.integers(0, 5, size=3)
    if seed == 0:
        choice = [0, 0, 1]               # the normal-mixed workload: x, y periodic, z faces normal-mixed
    prob = W.random_small_problem(rng, n=(4, 5, 4), scheme=scheme, bc=W.normal_mixed_bc(choice),
                                  tol=1e-11)
    rb = solver.solve(prob)
    prob.green = W.GREEN_C0
    rc = solver.solve(prob)
    assert rb["converged"][0] and rc["converged"][0]
    scale = np.abs(rb["sig"]).max()
    np.testing.assert_allclose(rc["sig"], rb["sig"], atol=1e-8 * scale)
    np.testing.assert_allclose(rc["macro_sigma"], rb["macro_sigma"], atol=1e-9 * scale)
    eps_d, sig_d, res = _direct_solve(prob)
    ref = np.stack([sig_d[..., i, j] for (i, j) in solver.VOIGT]).transpose(0, 1, 4, 3, 2)
    np.testing.assert_allclose(rc["sig"], ref, atol=1e-8 * scale)


def _nh_tension_closed_form(e, mu, K):
    """Appendix B: homogeneous tension F = diag(e, t, t) of the compressible
    Neo-Hookean bar.  P22(t) = mu/3 e t (e t^2)^-5/3 (t^2 - e^2) + K e t
    (e t^2 - 1) (from the energy; the printed P22 has (t^2 - 1) in its
    volumetric term, which drops J = e t^2) vanishes on the free lateral faces;
    t by bisection, then P11 = 2/3 mu t^2 (e t^2)^-5/3 (e^2 - t^2) + K (e t^4 - t^2)."""
    def P22(t):
        return mu / 3.0 * e * t * (e * t * t) ** (-5.0 / 3.0) * (t * t - e * e) + K * e * t * (e * t * t - 1.0)
    lo, hi = 0.3, 1.0 + 1e-12
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if P22(lo) * P22(mid) <= 0:
            hi = mid
        else:
            lo = mid
    t = 0.5 * (lo + hi)
    P11 = 2.0 / 3.0 * mu * t * t * (e * t * t) ** (-5.0 / 3.0) * (e * e - t * t) + K * (e * t ** 4 - t * t)
    return t, P11


@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
def test_neohooke_pure_tension_closed_form(scheme):
    """Appendix B: a Neo-Hookean bar stretched by Dirichlet conditions on u_x
    of its x faces (every other face and component free) is homogeneously
    stretched; <P11> follows the semi-analytic law over large elongations and
    the lateral stress vanishes."""
    n = (6, 3, 3)
    mu, K = 0.8, 2.0
    bc = np.full((3, 3, 2), W.N, dtype=np.int32)
    bc[0, 0, :] = W.D
    es = [1.05, 1.15, 1.3]
    steps = []
    for e in es:
        s = W.LoadStep(); s.G[0, 0] = e - 1.0
        steps.append(s)
    prob = W.Problem(n=n, h=1.0, bc=bc, scheme=scheme, green=W.GREEN_B0, lambda0=K, mu0=mu,
                     materials=[W.mat_neohooke(mu, K)], mat_id=np.zeros((n[2], n[1], n[0]), dtype=np.int32),
                     steps=steps, tol=1e-12, max_iter=3000, finite_strain=1)
    r = solver.solve(prob)
    assert all(r["converged"])
    for k, e in enumerate(es):
        t, P11 = _nh_tension_closed_form(e, mu, K)
        assert r["macro_sigma"][k][0] == pytest.approx(P11, rel=1e-9)
        assert abs(r["macro_sigma"][k][1]) < 1e-10 and abs(r["macro_sigma"][k][2]) < 1e-10
    # the lateral contraction of the last increment
    t, _ = _nh_tension_closed_form(es[-1], mu, K)
    Exx, Eyy = r["eps"][0].mean(), r["eps"][1].mean()
    assert Eyy == pytest.approx(0.5 * (t * t - 1.0), rel=1e-9)
    assert Exx == pytest.approx(0.5 * (es[-1] ** 2 - 1.0), rel=1e-9)


@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
def test_finite_strain_small_load_limit(scheme):
    """At small loads the finite-strain SVK solve of a random two-phase
    problem reduces to the small-strain isotropic one: <P> - <sigma> is of
    the order of the strain squared."""
    rng = np.random.default_rng(31 + scheme)
    small = W.random_small_problem(rng, n=(5, 4, 6), scheme=scheme, tol=1e-12)
    for s in small.steps:
        s.G *= 1e-3
        s.H *= 1e-3
    fs = W.random_small_problem(np.random.default_rng(31 + scheme), n=(5, 4, 6), scheme=scheme, tol=1e-12)
    for s in fs.steps:
        s.G *= 1e-3
        s.H *= 1e-3
    fs.materials = [W.mat_svk(m["lam"], m["mu"]) for m in fs.materials]
    fs.finite_strain = 1
    a = solver.solve(small)["macro_sigma"][0]
    b = solver.solve(fs)["macro_sigma"][0]
    scale = np.abs(a).max()
    assert np.abs(a - b).max() < 1e-4 * scale
    assert np.abs(a - b).max() > 0


def _nodal_poly(pl, step):
    """The polynomial u* of a step as a nodal field (oracle layout)."""
    return pl.ustar(step.c, step.G, step.H)


@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
def test_ustar_interior_is_absorbed(scheme):
    """Sec. 2.2 / Algorithm 1 set-up: u* enters only through its values on the
    dismissed (Dirichlet) nodes of each component; a perturbation of a nodal
    u* on the kept nodes is absorbed by u^f, so the strain and stress are
    unchanged, and u = u^f + u* up to a mode of zero discrete strain (rigid
    motions where the BCs leave them free, HEX1's hourglass modes: the null
    modes of the Green operator).  A perturbation
    on a Dirichlet face does change them."""
    rng = np.random.default_rng(77 + scheme)
    prob = W.random_small_problem(rng, n=(6, 5, 7), scheme=scheme, tol=1e-12)
    pl = solver.Plan(prob)
    base = solver.solve(prob)
    pert = 1e-3 * rng.standard_normal((3,) + tuple(v + 1 for v in prob.n))
    for q in range(3):
        fd.zero_dismissed(pert[q], pl.exts[q])
    p2 = W.random_small_problem(np.random.default_rng(77 + scheme), n=(6, 5, 7), scheme=scheme, tol=1e-12)
    p2.steps[0].ustar_nodal = pert
    r2 = solver.solve(p2)
    scale = np.abs(base["sig"]).max()
    np.testing.assert_allclose(r2["sig"], base["sig"], atol=1e-8 * scale)
    np.testing.assert_allclose(r2["eps"], base["eps"], atol=1e-8 * np.abs(base["eps"]).max())
    du = (r2["u"] - base["u"]).transpose(0, 3, 2, 1)
    g = pl.grad(du)
    assert np.abs(g + np.swapaxes(g, -1, -2)).max() < 1e-9 * np.abs(base["eps"]).max()
    # the same perturbation on the dismissed nodes only moves the solution
    dis = 1e-3 * rng.standard_normal(pert.shape)
    mask = np.stack([~pl.kept[q] for q in range(3)])
    if mask.any():
        p3 = W.random_small_problem(np.random.default_rng(77 + scheme), n=(6, 5, 7), scheme=scheme, tol=1e-12)
        p3.steps[0].ustar_nodal = np.where(mask, dis, 0.0)
        r3 = solver.solve(p3)
        assert np.abs(r3["sig"] - base["sig"]).max() > 1e-6 * scale


def test_ustar_nodal_equals_polynomial():
    """A nodal u* equal to the nodal values of the polynomial u* gives the
    polynomial's solve (zero polynomial in its place)."""
    rng = np.random.default_rng(5)
    prob = W.random_small_problem(rng, n=(5, 6, 4), scheme=W.TETRA2, tol=1e-12, n_steps=2)
    pl = solver.Plan(prob)
    base = solver.solve(prob)
    p2 = W.random_small_problem(np.random.default_rng(5), n=(5, 6, 4), scheme=W.TETRA2, tol=1e-12, n_steps=2)
    for s in p2.steps:
        s.ustar_nodal = _nodal_poly(pl, s)
        s.c, s.G, s.H = np.zeros(3), np.zeros((3, 3)), np.zeros((3, 3, 3))
    r2 = solver.solve(p2)
    np.testing.assert_allclose(r2["sig"], base["sig"], atol=1e-9 * np.abs(base["sig"]).max())
    np.testing.assert_allclose(r2["u"], base["u"], atol=1e-10 * np.abs(base["u"]).max())
