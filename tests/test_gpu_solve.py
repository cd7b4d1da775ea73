"""End-to-end GPU solves against the FP64 oracle (through the C ABI).

Tolerances: FP64 solves converged to tol agree with the oracle to ~tol on
the fields (both are within tol of the same discrete fixed point); the FP32
path is held to the 1e-5 relative macroscopic-stress target and to 1e-4 on
the local stress fields.
"""
import numpy as np
import pytest

import workloads as W
from oracle import solver as osolver
from tests.gpu_util import rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2607_05929_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def inclusion32():
    prob = W.config_inclusion32()
    return prob, osolver.solve(prob)


def test_inclusion32_fp64(B, inclusion32):
    prob, ref = inclusion32
    got = B.solve(prob, prec=W.FP64)
    print(f"inclusion32 fp64 iters gpu {got['iters']} oracle {ref['iters']}", flush=True)
    assert got["converged"][0]
    assert rel_err(got["macro_sigma"], ref["macro_sigma"]) < 1e-7
    assert rel_err(got["sig"], ref["sig"]) < 1e-6
    assert rel_err(got["u"], ref["u"]) < 1e-6


def test_inclusion32_fp32(B, inclusion32):
    prob, ref = inclusion32
    p = W.config_inclusion32()
    p.tol = 1e-6
    got = B.solve(p, prec=W.FP32_MIXED)
    e = rel_err(got["macro_sigma"], ref["macro_sigma"])
    print(f"inclusion32 fp32 iters {got['iters']} macro rel err {e:.2e}", flush=True)
    assert got["converged"][0]
    assert e < 1e-5
    assert rel_err(got["sig"], ref["sig"]) < 1e-4


@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
@pytest.mark.parametrize("seed", [11, 12])
def test_small_fp32(B, scheme, seed):
    rng = np.random.default_rng(seed)
    prob = W.random_small_problem(rng, n=(12, 10, 14), scheme=scheme, tol=1e-7,
                                  law="cubic" if seed == 12 else "iso")
    ref = osolver.solve(prob)
    prob.tol = 1e-6
    got = B.solve(prob, prec=W.FP32_MIXED)
    e = rel_err(got["macro_sigma"], ref["macro_sigma"])
    print(f"small fp32 scheme={scheme} seed={seed} iters {got['iters']} macro err {e:.2e}", flush=True)
    assert got["converged"][0]
    assert e < 1e-5


def _j2_problem():
    prob = W.config_j2_inclusions(nv=12, seed=3, n_steps=4, eps_final=6e-3, tol=1e-9,
                                  phi=0.15, rmin=2.0, rmax=3.0, prec=W.FP64)
    return prob


def test_j2_mixed_fp64(B):
    prob = _j2_problem()
    ref = osolver.solve(prob)
    got = B.solve(prob, prec=W.FP64)
    print(f"j2 fp64 iters gpu {got['iters']} oracle {ref['iters']}", flush=True)
    assert all(got["converged"]) and all(ref["converged"])
    assert rel_err(got["macro_sigma"], ref["macro_sigma"]) < 1e-7
    assert rel_err(got["sig"], ref["sig"]) < 1e-6
    # the mixed control reached <sigma_xx> = <sigma_yy> = 0
    assert np.abs(got["macro_sigma"][:, :2]).max() < 1e-8 * np.abs(got["macro_sigma"][:, 2]).max()
    # plasticity is active in the last increments
    assert got["macro_sigma"][-1, 2] < 0.9 * 70.0 * 6e-3


def test_j2_mixed_fp32(B):
    prob = _j2_problem()
    ref = osolver.solve(prob)
    prob.tol = 1e-6
    got = B.solve(prob, prec=W.FP32_MIXED)
    e = rel_err(got["macro_sigma"][:, 2], ref["macro_sigma"][:, 2])
    print(f"j2 fp32 iters {got['iters']} macro zz err {e:.2e}", flush=True)
    assert all(got["converged"])
    assert e < 1e-5


def test_j2_fp32_converges_like_fp64(B):
    """Precision policy for plastic solves: with the FP64 strain and law the
    FP32-mixed path converges in about the FP64 iteration counts (an FP32
    strain made the yield switch chatter and the increments stall), and the
    macroscopic stress agrees with the FP64 path."""
    prob = W.config_j2_inclusions(nv=96, n_steps=6, eps_final=6e-3)
    r32 = B.solve(prob, prec=W.FP32_MIXED, fields=False)
    r64 = B.solve(prob, prec=W.FP64, fields=False)
    print(f"j2 96^3 iters fp32 {r32['iters']} fp64 {r64['iters']}", flush=True)
    assert all(r32["converged"]) and all(r64["converged"])
    for a, b in zip(r32["iters"], r64["iters"]):
        assert a <= 1.5 * b + 10
    zz32, zz64 = r32["macro_sigma"][:, 2], r64["macro_sigma"][:, 2]
    assert rel_err(zz32, zz64) < 1e-5
    assert np.abs(r32["macro_sigma"][:, :2]).max() < 1e-5 * np.abs(zz64).max()


def _cp_problem(prec):
    rng = np.random.default_rng(55)
    prob = W.cp_polycrystal(rng, 8, 4, prec=prec, n_steps=3, eps_max=4e-3, tol=1e-9)
    return prob


def test_cp_fp64(B):
    prob = _cp_problem(W.FP64)
    ref = osolver.solve(prob)
    got = B.solve(prob, prec=W.FP64)
    print(f"cp fp64 iters gpu {got['iters']} oracle {ref['iters']}", flush=True)
    assert all(got["converged"])
    assert rel_err(got["macro_sigma"], ref["macro_sigma"]) < 1e-6
    assert rel_err(got["sig"], ref["sig"]) < 1e-5


def test_cp_fp32(B):
    prob = _cp_problem(W.FP64)
    ref = osolver.solve(prob)
    prob.tol = 1e-6
    got = B.solve(prob, prec=W.FP32_MIXED)
    e = rel_err(got["macro_sigma"], ref["macro_sigma"])
    print(f"cp fp32 iters {got['iters']} macro err {e:.2e}", flush=True)
    assert all(got["converged"])
    assert e < 1e-5


def _batch_problems():
    rng = np.random.default_rng(4)
    sizes = [8, 12, 16, 10, 14, 8]
    return [W.random_rve(rng, n, prec=W.FP32_MIXED, tol=1e-6) for n in sizes]


def test_batch_equals_alone(B):
    probs = _batch_problems()
    res = B.batch_solve(probs, fields=True)
    for p, r in zip(probs, res):
        alone = B.solve(p, prec=W.FP32_MIXED)
        print(f"long-pencil member n={p.n} rc {r['rc']} iters {r['iters']} alone {alone['iters']} "
              f"{alone['converged']}", flush=True)
        assert r["rc"] == 0
        assert r["iters"] == alone["iters"]
        np.testing.assert_array_equal(r["sig"], alone["sig"])
    # and against the oracle for two of them
    for k in (0, 3):
        p = probs[k]
        ref = osolver.solve(p)
        e = rel_err(res[k]["macro_sigma"], ref["macro_sigma"])
        print(f"batch member {k} macro err vs oracle {e:.2e}", flush=True)
        assert e < 1e-5


def test_autotuned_batch_matches_untuned(B):
    """Plans autotuned one at a time (small plans' passes timed with their
    tiles repeated to fill the device) run together as one batch: every
    member converges to the untuned batch's result, and a 24^3 member (48-
    and 24-point pencils: 16-lane wavefront kernels, generic DFT) matches the
    oracle."""
    rng = np.random.default_rng(9)
    probs = _batch_problems() + [W.random_rve(rng, n, prec=W.FP32_MIXED, tol=1e-6) for n in (24, 48)]
    plans = [B.Plan(p, W.FP32_MIXED) for p in probs]
    try:
        for pl in plans:
            info = pl.autotune(n_iter=2)
            assert all(c >= 0 for c in info["choice"])
        res = B.batch_solve(probs, plans=plans)
    finally:
        for pl in plans:
            pl.close()
    ref = B.batch_solve(probs, prec=W.FP32_MIXED)
    for p, r, q in zip(probs, res, ref):
        e = rel_err(r["macro_sigma"], q["macro_sigma"])
        print(f"tuned batch member n={p.n} iters {r['iters']} untuned {q['iters']} macro diff {e:.2e}", flush=True)
        assert r["rc"] == 0 and q["rc"] == 0
        assert e < 1e-5
    k = len(_batch_problems())
    oref = osolver.solve(probs[k])
    e = rel_err(res[k]["macro_sigma"], oref["macro_sigma"])
    print(f"tuned 24^3 member macro err vs oracle {e:.2e}", flush=True)
    assert e < 1e-5


def test_batch_fp64_finishing_equals_alone(B):
    """Members of the batched family (32^3) that move their real-space step
    to FP64 near the FP32 rounding floor, batched with members that do not:
    the FP64 real-space kernel of the group (blocks scanning their tiles 256
    at a time for solves that need it) gives every member exactly its own
    solve's iterations and stress."""
    probs = [p for p in W.config_batch(count=64) if p.n[0] == 32][:6]
    alone = [B.solve(p, prec=W.FP32_MIXED, log_capacity=4000) for p in probs]
    used = [any(e["rs_fp64"] for e in a["log"]) for a in alone]
    print(f"fp64 finishing per member {used} iters {[a['iters'] for a in alone]}", flush=True)
    assert any(used) and not all(used)
    res = B.batch_solve(probs, prec=W.FP32_MIXED, fields=True)
    for p, r, a in zip(probs, res, alone):
        assert r["rc"] == 0
        assert r["iters"] == a["iters"]
        np.testing.assert_array_equal(r["sig"], a["sig"])


def test_batch_long_pencils_equals_alone(B):
    """A batch whose solves put 512-point pencils on different axes: the
    persistent pipelined pass kernels take work items of several solves in
    one launch; every member equals its own solve bitwise, and the oracle.
    (These thin grids converge slowly; their FP32 error floor lies between
    1e-6 and 1e-5, so the FP32 solves stop at 1e-5 and the oracle, solved to
    1e-8, is matched to 1e-4 on the macroscopic stress.)"""
    rng = np.random.default_rng(21)
    shapes = [(256, 6, 5), (6, 256, 5), (5, 6, 256), (6, 256, 6)]
    probs = []
    for k, sh in enumerate(shapes):
        p = W.random_small_problem(rng, n=sh, scheme=(W.HEX1, W.TETRA2)[k % 2], tol=1e-5,
                                   law=("iso", "cubic")[k % 2], prec=W.FP32_MIXED)
        p.max_iter = 2000
        long_ax = int(np.argmax(sh))
        for q in range(3):
            # N/N (DCT-I) or D/D (DST-I) on the long axis: 512-point pencils
            p.bc[q][long_ax] = [W.N, W.N] if (q + k) % 2 == 0 else [W.D, W.D]
        probs.append(p)
    res = B.batch_solve(probs, fields=True)
    for p, r in zip(probs, res):
        alone = B.solve(p, prec=W.FP32_MIXED)
        print(f"long-pencil member n={p.n} rc {r['rc']} iters {r['iters']} alone {alone['iters']} "
              f"{alone['converged']}", flush=True)
        assert r["rc"] == 0
        assert r["iters"] == alone["iters"]
        np.testing.assert_array_equal(r["sig"], alone["sig"])
    for k in (0, 2):
        probs[k].tol = 1e-8
        ref = osolver.solve(probs[k])
        e = rel_err(res[k]["macro_sigma"], ref["macro_sigma"])
        print(f"long-pencil batch member {k} macro err vs oracle {e:.2e}", flush=True)
        assert e < 1e-4


def test_server_mix_equals_alone(B):
    probs = _batch_problems()[:5]
    srv = B.Server(arena_bytes=256 << 20, max_active=3)
    tickets = []
    now = 0.0
    # staggered arrivals: submit two, advance, submit the rest while they run
    for k, p in enumerate(probs):
        tickets.append(srv.submit(p, arrival_s=now))
        if k == 1:
            srv.step(4, now)
            now += 0.001
    for _ in range(2000):
        srv.step(8, now)
        now += 0.001
        if all(srv.poll(t)[0] == 2 for t in tickets):
            break
    st = srv.stats()
    print(f"server stats {st}", flush=True)
    assert st["completed"] == len(probs)
    assert st["arena_in_use"] == 0
    for t, p in zip(tickets, probs):
        alone = B.solve(p, prec=W.FP32_MIXED, fields=False)
        got = srv.result(t)
        np.testing.assert_array_equal(got["macro_sigma"], alone["macro_sigma"])
        assert got["iters"] == alone["iters"]
    srv.close()


def test_graph_launch_equals_direct(B):
    """Captured-graph iteration chunks reproduce direct launches bitwise:
    one plan solved repeatedly (every chunk graph replayed many times, with
    host reads and syncs between replays), both precisions, and a batch."""
    rng = np.random.default_rng(77)
    probs = [W.random_small_problem(rng, n=(9, 8, 7), scheme=s, law=law, tol=1e-9, n_steps=2)
             for s, law in ((W.HEX1, "cubic"), (W.TETRA2, "j2"))]
    try:
        for prec in (W.FP64, W.FP32_MIXED):
            for p in probs:
                B.set_graph_launch(False)
                ref = B.solve(p, prec=prec)
                B.set_graph_launch(True)
                plan = B.Plan(p, prec)
                for rep in range(3):
                    plan.reset()
                    got = plan.solve()
                    assert got["iters"] == ref["iters"], (rep, got["iters"], ref["iters"])
                    np.testing.assert_array_equal(got["macro_sigma"], ref["macro_sigma"])
                    np.testing.assert_array_equal(got["u"], ref["u"])
                    np.testing.assert_array_equal(got["sig"], ref["sig"])
                plan.close()
        batch = _batch_problems()[:4]
        B.set_graph_launch(False)
        ref = B.batch_solve(batch)
        B.set_graph_launch(True)
        got = B.batch_solve(batch)
        for a, b in zip(got, ref):
            assert a["iters"] == b["iters"]
            np.testing.assert_array_equal(a["macro_sigma"], b["macro_sigma"])
    finally:
        B.set_graph_launch(True)


def test_autotune_then_solve_matches_oracle(B, inclusion32):
    """fm_autotune times every applicable transform kernel per axis pass and
    keeps the fastest; the tuned plan still reproduces the oracle."""
    prob, ref = inclusion32
    plan = B.Plan(prob, W.FP64)
    info = plan.autotune(n_iter=3)
    print(f"autotune choice {info['choice']}\n{info['ms']}", flush=True)
    assert all(c >= 0 for c in info["choice"])
    for pass_, c in enumerate(info["choice"]):
        t = info["ms"][c, pass_]
        assert t > 0 and t <= info["ms"][:, pass_][info["ms"][:, pass_] > 0].min() + 1e-12
    r = plan.solve()
    plan.close()
    assert all(r["converged"])
    e = rel_err(r["macro_sigma"], ref["macro_sigma"])
    es = rel_err(r["sig"], ref["sig"])
    print(f"autotuned inclusion32 macro err {e:.2e} sigma err {es:.2e}", flush=True)
    assert e < 1e-7 and es < 1e-6


def test_server_admission_near_full_arena(B):
    """An arena that holds one request's workspace but not its batch
    descriptors refuses the request at submission; an arena with room for one
    request at a time (plus descriptors) serves a stream of them one after
    the other without error."""
    import ctypes as C
    probs = _batch_problems()[:3]
    for p in probs:
        p.n = (16, 16, 16)
        p.mat_id = np.zeros((16, 16, 16), dtype=np.int32)
        p.mat_id[4:10, 4:10, 4:10] = 1
    d = B.plan_desc(probs[0], W.FP32_MIXED)
    ws = int(B.lib().fm_workspace_bytes(C.byref(d)))
    stage = 4 * 16 ** 3
    tight = B.Server(arena_bytes=ws + stage + 4096, max_active=4)
    with pytest.raises(B.FmError, match="never fit"):
        tight.submit(probs[0], arrival_s=0.0, prec=W.FP32_MIXED)
    tight.close()
    srv = B.Server(arena_bytes=ws + stage + (2 << 20), max_active=4)
    tickets = [srv.submit(p, arrival_s=0.0, prec=W.FP32_MIXED) for p in probs]
    for _ in range(4000):
        srv.step(8, 0.0)
        if all(srv.poll(t)[0] == 2 for t in tickets):
            break
    st = srv.stats()
    print(f"near-full arena stats {st}", flush=True)
    assert st["completed"] == 3 and st["arena_in_use"] == 0
    for t, p in zip(tickets, probs):
        alone = B.solve(p, prec=W.FP32_MIXED, fields=False)
        np.testing.assert_array_equal(srv.result(t)["macro_sigma"], alone["macro_sigma"])
    srv.close()


def test_server_cp_mix_equals_alone(B):
    """The served law: crystal-plasticity torsion-bending requests of
    different sizes and grain counts, arriving while others run, each give
    the result of their lone solve (same device arithmetic, bitwise) and
    converge every increment."""
    rng = np.random.default_rng(5)
    probs = [W.cp_polycrystal(rng, nv, g, prec=W.FP32_MIXED, n_steps=3, eps_max=4e-3)
             for nv, g in ((8, 3), (12, 5), (10, 4), (16, 6))]
    srv = B.Server(arena_bytes=512 << 20, max_active=3)
    tickets = []
    now = 0.0
    for k, p in enumerate(probs):
        tickets.append(srv.submit(p, arrival_s=now, prec=W.FP32_MIXED))
        srv.step(3, now)                     # later requests arrive while earlier ones run
        now += 0.001
    for _ in range(4000):
        srv.step(4, now)
        now += 0.001
        if all(srv.poll(t)[0] == 2 for t in tickets):
            break
    st = srv.stats()
    print(f"cp server stats {st}", flush=True)
    assert st["completed"] == len(probs)
    for t, p in zip(tickets, probs):
        alone = B.solve(p, prec=W.FP32_MIXED, fields=False)
        got = srv.result(t)
        print(f"cp served n={p.n} iters {got['iters']} alone {alone['iters']}", flush=True)
        assert all(alone["converged"])
        assert got["iters"] == alone["iters"]
        np.testing.assert_array_equal(got["macro_sigma"], alone["macro_sigma"])
    srv.close()
