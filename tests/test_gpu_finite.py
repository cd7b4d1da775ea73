"""The Lagrangian finite-strain formulation on the GPU (Sec. 2.2: F = 1 +
grad u, P = F Pi with the Saint Venant-Kirchhoff and compressible
Neo-Hookean laws, the divergence taken of the first Piola-Kirchhoff stress)
against the oracle through the C ABI; the Neo-Hookean pure-tension case of
Appendix B against its semi-analytic solution."""
import numpy as np
import pytest

import workloads as W
from oracle import fd, solver as osolver
from oracle.laws import MaterialSet
from tests.gpu_util import rel_err, xyz_nodes_from_zyx, zyx_nodes_from_xyz
from tests.test_oracle_solver import _nh_tension_closed_form

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2607_05929_amd import binding
    binding.lib()
    return binding


def _fs_problem(rng, n, scheme, law, load=40.0, bc=None, tol=1e-10, n_steps=1):
    """A random two-phase problem of the small parity family, turned into a
    finite-strain one: the phases become SVK or Neo-Hookean solids with the
    same Lame constants and the load is scaled up to a few per cent strain."""
    prob = W.random_small_problem(rng, n=n, scheme=scheme, bc=bc, tol=tol, n_steps=n_steps)
    mats = []
    for m in prob.materials:
        if law == "svk":
            mats.append(W.mat_svk(m["lam"], m["mu"]))
        else:
            mats.append(W.mat_neohooke(m["mu"], m["lam"] + 2.0 * m["mu"] / 3.0))
    prob.materials = mats
    prob.finite_strain = 1
    for s in prob.steps:
        s.G = s.G * load
        s.H = s.H * load
    return prob


def _oracle_residual(prob, pl, uf, step):
    mats = MaterialSet(prob.materials, np.asarray(prob.mat_id).transpose(2, 1, 0))
    gu = pl.grad(uf) + pl.grad(pl.ustar(step.c, step.G, step.H))
    F = np.eye(3) + np.swapaxes(gu, -1, -2)
    S = np.swapaxes(mats.pk1(F), -1, -2)
    D = pl.div(S) + pl.div_applied(getattr(step, "traction", np.zeros((3, 2, 3))))
    err = osolver.equilibrium_error(pl, D, S)
    mP = S.mean(axis=(0, 1, 2, 3)).T
    macro = np.array([mP[i, j] for (i, j) in osolver.VOIGT])
    return D, err, macro


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
@pytest.mark.parametrize("law", ["svk", "nh"])
@pytest.mark.parametrize("n", [(9, 7, 8), (40, 17, 35)])
def test_fs_residual_matches_oracle(B, prec, scheme, law, n):
    """One residual evaluation (strain, first Piola-Kirchhoff stress,
    divergence, error and <P>) on a random displacement, grids spanning
    several tiles with ragged tails."""
    rng = np.random.default_rng(11 + 5 * scheme + n[0] + (law == "nh"))
    prob = _fs_problem(rng, n, scheme, law)
    pl = osolver.Plan(prob)
    uf = 2e-2 * rng.standard_normal((3,) + tuple(v + 1 for v in n))
    for q in range(3):
        fd.zero_dismissed(uf[q], pl.exts[q])
    step = prob.steps[0]
    Dref, err_ref, mref = _oracle_residual(prob, pl, uf, step)
    gp = B.Plan(prob, prec=prec)
    D, err, macro = gp.residual(zyx_nodes_from_xyz(uf), step)
    gp.close()
    D = xyz_nodes_from_zyx(D)
    kept = np.stack(pl.kept)
    e = rel_err(D[kept], Dref[kept])
    print(f"fs residual n={n} scheme={scheme} law={law} prec={prec} D {e:.2e} err {err:.6e}/{err_ref:.6e} "
          f"macro {rel_err(macro, mref):.2e}", flush=True)
    assert np.all(D[~kept] == 0)
    assert e < (1e-12 if prec == W.FP64 else 2e-5)
    assert err == pytest.approx(err_ref, rel=1e-10 if prec == W.FP64 else 1e-4)
    assert rel_err(macro, mref) < (1e-12 if prec == W.FP64 else 1e-6)


@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
@pytest.mark.parametrize("law", ["svk", "nh"])
def test_fs_solve_matches_oracle(B, scheme, law):
    """Full solves (two increments) in FP64 and FP32-mixed: <P> per increment,
    the displacement, the Green-Lagrange strain and the Cauchy stress."""
    rng = np.random.default_rng(23 + scheme + 2 * (law == "nh"))
    prob = _fs_problem(rng, (9, 8, 7), scheme, law, n_steps=2)
    ref = osolver.solve(prob)
    assert all(ref["converged"])
    got = B.solve(prob, prec=W.FP64)
    print(f"fs solve scheme={scheme} law={law} iters gpu {got['iters']} oracle {ref['iters']}", flush=True)
    assert all(got["converged"])
    assert rel_err(got["macro_sigma"], ref["macro_sigma"]) < 1e-8
    assert rel_err(got["u"], ref["u"]) < 1e-7
    assert rel_err(got["eps"], ref["eps"]) < 1e-7
    assert rel_err(got["sig"], ref["sig"]) < 1e-7
    prob.tol = 1e-6
    got32 = B.solve(prob, prec=W.FP32_MIXED)
    e32 = rel_err(got32["macro_sigma"], ref["macro_sigma"])
    print(f"fs solve fp32 iters {got32['iters']} macro err {e32:.2e}", flush=True)
    assert all(got32["converged"]) and e32 < 1e-5


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
def test_fs_neohooke_pure_tension(B, prec, scheme):
    """Appendix B: a Neo-Hookean bar stretched by u_x Dirichlet conditions on
    its x faces, every other face and component free, up to 30 % elongation:
    <P_11> against the semi-analytic law, vanishing lateral stress, and the
    lateral Green-Lagrange strain from the closed-form contraction."""
    n = (12, 5, 6)
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
                     steps=steps, tol=1e-11 if prec == W.FP64 else 1e-7, max_iter=5000, finite_strain=1)
    r = B.solve(prob, prec=prec)
    assert all(r["converged"])
    bar = 1e-9 if prec == W.FP64 else 1e-6
    for k, e in enumerate(es):
        t, P11 = _nh_tension_closed_form(e, mu, K)
        print(f"nh tension scheme={scheme} prec={prec} e={e} P11 {r['macro_sigma'][k][0]:.12f} closed {P11:.12f} "
              f"iters {r['iters'][k]}", flush=True)
        assert r["macro_sigma"][k][0] == pytest.approx(P11, rel=bar)
        assert np.abs(r["macro_sigma"][k][1:]).max() < bar * abs(P11)
    t, _ = _nh_tension_closed_form(es[-1], mu, K)
    assert r["eps"][1].mean() == pytest.approx(0.5 * (t * t - 1.0), rel=bar)
    assert r["eps"][0].mean() == pytest.approx(0.5 * (es[-1] ** 2 - 1.0), rel=bar)


@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
def test_fs_c0_solve_matches_oracle(B, scheme):
    """The C0 operator in its finite-strain form (C0 acting on the full
    gradient) on a normal-mixed problem, against the oracle."""
    rng = np.random.default_rng(41 + scheme)
    prob = _fs_problem(rng, (8, 7, 9), scheme, "nh", bc=W.normal_mixed_bc((1, 3, 0)))
    prob.green = W.GREEN_C0
    ref = osolver.solve(prob)
    got = B.solve(prob, prec=W.FP64)
    print(f"fs c0 scheme={scheme} iters gpu {got['iters']} oracle {ref['iters']}", flush=True)
    assert all(ref["converged"]) and all(got["converged"])
    assert rel_err(got["macro_sigma"], ref["macro_sigma"]) < 1e-8
    assert rel_err(got["sig"], ref["sig"]) < 1e-7


def test_fs_with_tractions_matches_oracle(B):
    """Finite strain with applied tractions on the Neumann faces (the
    applied stress enters the divergence as in the small-strain case)."""
    rng = np.random.default_rng(57)
    prob = _fs_problem(rng, (9, 7, 8), W.TETRA2, "svk")
    for q in range(3):
        if not np.any(prob.bc[q] == W.N):
            prob.bc[q, q % 3] = [W.N, W.D]
    T = np.zeros((3, 2, 3))
    for q in range(3):
        for i in range(3):
            for a in range(2):
                if prob.bc[q, i, a] == W.N:
                    T[i, a, q] = rng.uniform(-2e-2, 2e-2)
    prob.steps[0].traction = T
    ref = osolver.solve(prob)
    got = B.solve(prob, prec=W.FP64)
    print(f"fs tractions iters gpu {got['iters']} oracle {ref['iters']}", flush=True)
    assert all(ref["converged"]) and all(got["converged"])
    assert rel_err(got["macro_sigma"], ref["macro_sigma"]) < 1e-8
    assert rel_err(got["u"], ref["u"]) < 1e-7


def test_fs_batch_matches_single_solves(B):
    """A batch of finite-strain solves of different sizes and laws equals
    the one-at-a-time solves; a batch mixing formulations is refused."""
    rng = np.random.default_rng(71)
    probs = [_fs_problem(rng, n, W.HEX1, law) for n, law in
             [((9, 8, 7), "svk"), ((16, 12, 10), "nh"), ((7, 7, 7), "nh")]]
    res = B.batch_solve(probs, prec=W.FP64)
    for p, r in zip(probs, res):
        one = B.solve(p, prec=W.FP64, fields=False)
        assert r["rc"] == 0
        assert rel_err(r["macro_sigma"], one["macro_sigma"]) < 1e-12
    small = W.random_small_problem(rng, n=(6, 5, 7))
    with pytest.raises(B.FmError, match="formulation"):
        B.batch_solve([probs[0], small], prec=W.FP64)


def test_fs_rejects_mismatched_laws(B):
    rng = np.random.default_rng(5)
    prob = _fs_problem(rng, (6, 5, 7), W.HEX1, "svk")
    prob.materials = [W.mat_iso(1.0, 1.0), W.mat_iso(2.0, 1.0)]
    with pytest.raises(B.FmError, match="finite-strain"):
        B.Plan(prob, prec=W.FP64)
