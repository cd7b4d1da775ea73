"""The C0 discrete Green operator on the GPU (Sec. 2.6.1, small-strain form of
Appendix A) against the oracle, which applies the paper's formulas to the
virtually extended fields with a plain 3D DFT; and solves with it."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import fd, solver as osolver
from tests.gpu_util import rel_err, xyz_nodes_from_zyx, zyx_nodes_from_xyz

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2607_05929_amd import binding
    binding.lib()
    return binding


def _c0_problem(rng, n, scheme, choice, law="iso", n_steps=1):
    prob = W.random_small_problem(rng, n=n, scheme=scheme, bc=W.normal_mixed_bc(choice), law=law,
                                  n_steps=n_steps)
    prob.green = W.GREEN_C0
    return prob


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
def test_c0_green_all_patterns(B, prec, scheme):
    """Every one of the 125 normal-mixed patterns (5 pairs per axis)."""
    rng = np.random.default_rng(90 + scheme)
    n = (6, 5, 7)
    worst = 0.0
    for choice in itertools.product(range(5), repeat=3):
        prob = _c0_problem(rng, n, scheme, choice)
        pl = osolver.Plan(prob)
        x = rng.standard_normal((3,) + tuple(v + 1 for v in n))
        for q in range(3):
            fd.zero_dismissed(x[q], pl.exts[q])
        ref = -pl.green_apply(x)
        gp = B.Plan(prob, prec=prec)
        got = xyz_nodes_from_zyx(gp.apply_green(zyx_nodes_from_xyz(x)))
        gp.close()
        e = rel_err(got, ref)
        worst = max(worst, e)
        assert e < (1e-11 if prec == W.FP64 else 2e-5), (choice, e)
    print(f"c0 green all patterns scheme={scheme} prec={prec} worst {worst:.2e}", flush=True)


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
@pytest.mark.parametrize("shape,choice", [((33, 20, 17), (0, 0, 1)), ((64, 48, 40), (1, 2, 3)),
                                          ((40, 64, 24), (4, 0, 2))])
def test_c0_green_larger_grids(B, prec, shape, choice):
    rng = np.random.default_rng(sum(shape))
    for scheme in (W.HEX1, W.TETRA2):
        prob = _c0_problem(rng, shape, scheme, choice)
        pl = osolver.Plan(prob)
        x = rng.standard_normal((3,) + tuple(v + 1 for v in shape))
        for q in range(3):
            fd.zero_dismissed(x[q], pl.exts[q])
        ref = -pl.green_apply(x)
        gp = B.Plan(prob, prec=prec)
        got = xyz_nodes_from_zyx(gp.apply_green(zyx_nodes_from_xyz(x)))
        gp.close()
        e = rel_err(got, ref)
        print(f"c0 green shape={shape} choice={choice} scheme={scheme} prec={prec} err {e:.2e}", flush=True)
        assert e < (1e-11 if prec == W.FP64 else 2e-5)


def test_c0_rejects_non_normal_mixed(B):
    rng = np.random.default_rng(3)
    prob = W.config_polycrystal_bending(nv=16, n_grains=4)
    prob.green = W.GREEN_C0
    with pytest.raises(B.FmError, match="normal-mixed"):
        B.Plan(prob, prec=W.FP64)


@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
@pytest.mark.parametrize("law", ["iso", "j2"])
def test_c0_solve_matches_oracle(B, scheme, law):
    rng = np.random.default_rng(17 + scheme + (law == "j2"))
    prob = _c0_problem(rng, (9, 8, 7), scheme, (0, 1, 2), law=law, n_steps=3 if law == "j2" else 1)
    prob.tol = 1e-10
    ref = osolver.solve(prob)
    got = B.solve(prob, prec=W.FP64)
    print(f"c0 solve scheme={scheme} law={law} iters gpu {got['iters']} oracle {ref['iters']}", flush=True)
    assert all(got["converged"])
    assert rel_err(got["sig"], ref["sig"]) < 1e-7
    assert rel_err(got["macro_sigma"], ref["macro_sigma"]) < 1e-8
    prob.tol = 1e-6
    got32 = B.solve(prob, prec=W.FP32_MIXED)
    e32 = rel_err(got32["macro_sigma"], ref["macro_sigma"])
    print(f"c0 solve fp32 iters {got32['iters']} macro err {e32:.2e}", flush=True)
    assert all(got32["converged"]) and e32 < 1e-5


def test_c0_normal_mixed_workload_iterations(B):
    """The normal-mixed elastoplastic workload (x, y periodic; z faces u_z
    Dirichlet, u_x, u_y Neumann; <sigma_xx> = <sigma_yy> = 0) at 64^3, first
    six increments: the C0 and B0 operators reach the same macroscopic stress;
    the iteration counts of both are recorded."""
    prob = W.config_j2_inclusions(nv=64, n_steps=20, eps_final=2e-2, prec=W.FP64)
    prob.steps = prob.steps[:6]
    r_b0 = B.solve(prob, prec=W.FP64, fields=False)
    prob.green = W.GREEN_C0
    r_c0 = B.solve(prob, prec=W.FP64, fields=False)
    r_c032 = B.solve(prob, prec=W.FP32_MIXED, fields=False)
    print(f"normal-mixed J2 64^3 iterations B0 {r_b0['iters']} C0 {r_c0['iters']} C0 fp32 {r_c032['iters']}",
          flush=True)
    assert all(r_b0["converged"]) and all(r_c0["converged"]) and all(r_c032["converged"])
    zz0, zz1 = r_b0["macro_sigma"][:, 2], r_c0["macro_sigma"][:, 2]
    assert rel_err(zz1, zz0) < 1e-5
    assert rel_err(r_c032["macro_sigma"][:, 2], zz0) < 1e-5
