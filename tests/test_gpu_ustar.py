"""A nodal u* field in the load steps (Sec. 2.2, Algorithm 1 set-up: the
prescribed displacement need not be a polynomial) on the GPU, against the
oracle through the C ABI: solves over two increments with different fields,
the residual entry point, a batch and the server."""
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


def _nodal_problem(rng, n, scheme, n_steps=2, tol=1e-10, law="iso"):
    prob = W.random_small_problem(rng, n=n, scheme=scheme, n_steps=n_steps, tol=tol, law=law)
    N = tuple(v + 1 for v in n)
    for t, s in enumerate(prob.steps):
        s.ustar_nodal = 1e-3 * (t + 1) * rng.standard_normal((3,) + N)
    return prob


@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
@pytest.mark.parametrize("law", ["iso", "j2"])
def test_nodal_solve_matches_oracle(B, scheme, law):
    rng = np.random.default_rng(200 + 3 * scheme + (law == "j2"))
    prob = _nodal_problem(rng, (8, 7, 9), scheme, law=law)
    ref = osolver.solve(prob)
    assert all(ref["converged"])
    got = B.solve(prob, prec=W.FP64)
    print(f"nodal u* scheme={scheme} law={law} iters gpu {got['iters']} oracle {ref['iters']}", flush=True)
    assert all(got["converged"])
    assert rel_err(got["macro_sigma"], ref["macro_sigma"]) < 1e-8
    assert rel_err(got["sig"], ref["sig"]) < 1e-7
    assert rel_err(got["u"], ref["u"]) < 1e-7
    prob.tol = 1e-6
    got32 = B.solve(prob, prec=W.FP32_MIXED)
    e32 = rel_err(got32["macro_sigma"], ref["macro_sigma"])
    print(f"nodal u* fp32 iters {got32['iters']} macro err {e32:.2e}", flush=True)
    assert all(got32["converged"]) and e32 < 1e-5


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
def test_nodal_residual_matches_oracle(B, prec):
    rng = np.random.default_rng(31)
    n = (24, 17, 20)
    prob = _nodal_problem(rng, n, W.TETRA2, n_steps=1)
    pl = osolver.Plan(prob)
    step = prob.steps[0]
    uf = 1e-3 * rng.standard_normal((3,) + tuple(v + 1 for v in n))
    for q in range(3):
        fd.zero_dismissed(uf[q], pl.exts[q])
    mats = MaterialSet(prob.materials, np.asarray(prob.mat_id).transpose(2, 1, 0))
    gu = pl.grad(uf) + pl.grad(pl.ustar(step.c, step.G, step.H, step.ustar_nodal))
    eps = 0.5 * (gu + np.swapaxes(gu, -1, -2))
    sig, _ = mats.stress(eps, mats.init_state(pl.nppv, pl.n), step.dt)
    Dref = pl.div(sig)
    gp = B.Plan(prob, prec=prec)
    D, err, macro = gp.residual(zyx_nodes_from_xyz(uf), step)
    gp.close()
    D = xyz_nodes_from_zyx(D)
    kept = np.stack(pl.kept)
    e = rel_err(D[kept], Dref[kept])
    print(f"nodal u* residual prec={prec} D err {e:.2e}", flush=True)
    assert e < (1e-12 if prec == W.FP64 else 2e-5)


def test_nodal_batch_and_server_equal_alone(B):
    rng = np.random.default_rng(47)
    probs = [_nodal_problem(rng, n, W.HEX1, tol=1e-8) for n in [(9, 8, 7), (12, 10, 11)]]
    probs.append(W.random_small_problem(rng, n=(7, 7, 7), tol=1e-8))
    alone = [B.solve(p, prec=W.FP64, fields=False) for p in probs]
    res = B.batch_solve(probs, prec=W.FP64)
    for r, a in zip(res, alone):
        assert r["rc"] == 0
        assert rel_err(r["macro_sigma"], a["macro_sigma"]) < 1e-12
    srv = B.Server(arena_bytes=1 << 30, max_active=4)
    tickets = [srv.submit(p, arrival_s=0.0, prec=W.FP64) for p in probs]
    for _ in range(20000):
        srv.step(8, 0.0)
        if all(srv.poll(t)[0] == 2 for t in tickets):
            break
    for t, a in zip(tickets, alone):
        served = srv.result(t)
        assert rel_err(served["macro_sigma"], a["macro_sigma"]) < 1e-12
    srv.close()
