"""Non-vanishing Neumann conditions on the GPU (Sec. 2.2, applied stress P*
on the mirror voxels of a loaded face), against the oracle through the C ABI,
and the cantilever under a uniformly distributed load of Sec. 3.1.1 against
the beam-theory deflection (an approximate check: beam theory neglects shear
deformation and the grid is coarse)."""
import numpy as np
import pytest

import workloads as W
from oracle import fd, solver as osolver
from oracle.laws import MaterialSet
from tests.gpu_util import rel_err, xyz_nodes_from_zyx, zyx_nodes_from_xyz

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2607_05929_amd import binding
    binding.lib()
    return binding


def _traction_problem(rng, n, scheme, law):
    prob = W.random_small_problem(rng, n=n, scheme=scheme, law=law)
    for q in range(3):                       # at least one Neumann face per component
        if not np.any(prob.bc[q] == W.N):
            prob.bc[q, q % 3] = [W.N, W.D]
    T = np.zeros((3, 2, 3))
    for q in range(3):
        for i in range(3):
            for a in range(2):
                if prob.bc[q, i, a] == W.N:
                    T[i, a, q] = rng.uniform(-1e-3, 1e-3)
    prob.steps[0].traction = T
    return prob


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
@pytest.mark.parametrize("n", [(9, 7, 8), (40, 17, 35)])
def test_residual_with_tractions(B, prec, scheme, n):
    rng = np.random.default_rng(31 + 7 * scheme + n[0])
    prob = _traction_problem(rng, n, scheme, "cubic")
    pl = osolver.Plan(prob)
    uf = 1e-3 * rng.standard_normal((3,) + tuple(v + 1 for v in n))
    for q in range(3):
        fd.zero_dismissed(uf[q], pl.exts[q])
    step = prob.steps[0]
    mats = MaterialSet(prob.materials, np.asarray(prob.mat_id).transpose(2, 1, 0))
    gu = pl.grad(uf) + pl.grad(pl.ustar(step.c, step.G, step.H))
    eps = 0.5 * (gu + np.swapaxes(gu, -1, -2))
    sig, _ = mats.stress(eps, mats.init_state(pl.nppv, pl.n), step.dt)
    Dref = pl.div(sig) + pl.div_applied(step.traction)
    gp = B.Plan(prob, prec=prec)
    D, err, macro = gp.residual(zyx_nodes_from_xyz(uf), step)
    gp.close()
    D = xyz_nodes_from_zyx(D)
    kept = np.stack(pl.kept)
    e = rel_err(D[kept], Dref[kept])
    err_ref = osolver.equilibrium_error(pl, Dref, sig)
    print(f"traction residual n={n} scheme={scheme} prec={prec} D err={e:.2e} eq. err {err:.6e} vs {err_ref:.6e}",
          flush=True)
    assert np.all(D[~kept] == 0.0)
    assert e < (1e-10 if prec == W.FP64 else 5e-5)
    assert abs(err - err_ref) / err_ref < (1e-12 if prec == W.FP64 else 1e-5)


@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
def test_cantilever_matches_oracle(B, scheme):
    prob = W.cantilever(n=(40, 4, 4), t2=1e-3, scheme=scheme, n_steps=2, tol=1e-9)
    ref = osolver.solve(prob)
    got = B.solve(prob, prec=W.FP64)
    print(f"cantilever scheme={scheme} iters gpu {got['iters']} oracle {ref['iters']}", flush=True)
    assert all(got["converged"])
    assert rel_err(got["u"], ref["u"]) < 1e-7
    assert rel_err(got["sig"], ref["sig"]) < 1e-6
    assert rel_err(got["macro_sigma"], ref["macro_sigma"]) < 1e-7
    prob.tol = 1e-6
    got32 = B.solve(prob, prec=W.FP32_MIXED)
    e32 = rel_err(got32["u"], ref["u"])
    print(f"cantilever fp32 iters {got32['iters']} u err {e32:.2e}", flush=True)
    assert all(got32["converged"]) and e32 < 1e-4


def _beam_deflection(n, t2, lam=120.0, mu=80.0):
    E = mu * (3 * lam + 2 * mu) / (lam + mu)
    L, w, hh = n[0], n[2], n[1]
    I = w * hh ** 3 / 12.0
    x = np.arange(n[0] + 1.0)
    return -t2 * w / (E * I) * (L ** 2 * x ** 2 / 4 - L * x ** 3 / 6 + x ** 4 / 24)


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
def test_cantilever_beam_theory(B, prec, scheme):
    """Sec. 3.1.1 at its grid (100 x 10 x 10 voxels): the neutral-axis
    deflection follows the beam formula within the shear-deformation gap."""
    n = (100, 10, 10)
    prob = W.cantilever(n=n, t2=1e-4, scheme=scheme, n_steps=3, tol=1e-6)
    got = B.solve(prob, prec=prec)
    assert all(got["converged"])
    uy = got["u"][1]                         # (z, y, x)
    mid = 0.5 * (uy[n[2] // 2, n[1] // 2, :] + uy[n[2] // 2, n[1] // 2, :])
    beam = _beam_deflection(n, 1e-4)
    r_tip, r_mid = mid[-1] / beam[-1], mid[n[0] // 2] / beam[n[0] // 2]
    print(f"cantilever 100x10x10 scheme={scheme} prec={prec} iters {got['iters']} tip ratio {r_tip:.4f} "
          f"mid ratio {r_mid:.4f}", flush=True)
    assert abs(r_tip - 1) < 0.05 and abs(r_mid - 1) < 0.06
