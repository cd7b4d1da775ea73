"""fm_solve_static, the allocation-free solve on the library's static device
scratch, against fm_solve on a caller workspace: the same kernels, so the
results are bitwise equal; two calls in a row (the second on a smaller grid,
over the contents the first left in the scratch), both precisions; a
workspace beyond the scratch is refused."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2607_05929_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
def test_static_solve_equals_workspace_solve(B, prec):
    rng = np.random.default_rng(808)
    first = W.random_small_problem(rng, n=(24, 20, 22), scheme=W.TETRA2, law="cubic", tol=1e-8, n_steps=2)
    second = W.random_small_problem(rng, n=(12, 10, 9), scheme=W.HEX1, law="j2", tol=1e-8, n_steps=3)
    for prob in (first, second):
        prob.tol = 1e-8 if prec == W.FP64 else 1e-6
        got = B.solve_static(prob, prec=prec)
        ref = B.solve(prob, prec=prec)
        print(f"static solve n={prob.n} prec={prec} iters {got['iters']} workspace {ref['iters']}", flush=True)
        assert got["rc"] == ref["rc"] == 0
        assert got["iters"] == ref["iters"]
        np.testing.assert_array_equal(got["macro_sigma"], ref["macro_sigma"])
        np.testing.assert_array_equal(got["u"], ref["u"])
        np.testing.assert_array_equal(got["sig"], ref["sig"])


def test_static_solve_refuses_large_grid(B):
    prob = W.config_polycrystal_bending(nv=96, n_grains=8)
    with pytest.raises(B.FmError, match="static scratch"):
        B.solve_static(prob, prec=W.FP64)
