"""The five workload configurations at (or near) their full size against the
FP64 oracle's stored results (tests/golden/*.json, written by
tests/golden/make_config_goldens.py, which calls only the oracle).

Bars: FP32-mixed and FP64 solves stopped at the configuration's tolerance
(1e-6 unless stated) reach the oracle's macroscopic stress, solved to 1e-8,
within 1e-5 relative to its largest component; the stress at the sampled
integration points agrees in relative L2 to 1e-4 (FP32-mixed) and 1e-5
(FP64) -- both sides are within the tolerance of the same discrete fixed
point, and the local stress of a converged iterate deviates from it by about
the tolerance times the local stiffness contrast.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import rel_err

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def B():
    from paper_2607_05929_amd import binding
    binding.lib()
    return binding


def _sampled_sigma(sig, vox):
    """sig (6, nppv, z, y, x) at voxels (x, y, z) -> (count, nppv, 6)."""
    return np.array([[[sig[c, ip, z, y, x] for c in range(6)] for ip in range(sig.shape[1])] for x, y, z in vox])


def _l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
def test_inclusion32_against_golden(B, prec):
    g = _golden("inclusion32.json")
    prob = W.config_inclusion32()
    prob.tol = 1e-8 if prec == W.FP64 else 1e-6
    r = B.solve(prob, prec=prec)
    em = rel_err(r["macro_sigma"], g["macro_sigma"])
    es = _l2(_sampled_sigma(r["sig"], g["voxels_xyz"]), g["sigma"])
    print(f"inclusion32 prec={prec} iters {r['iters']} macro {em:.2e} sigma L2 {es:.2e}", flush=True)
    assert all(r["converged"])
    assert em < (1e-7 if prec == W.FP64 else 1e-5)
    assert es < (1e-6 if prec == W.FP64 else 1e-4)


def test_batch_members_against_golden(B):
    """Eight of the first 64 solves of the batched configuration, among them
    the high-contrast ones whose FP32 residual converges slowest: one
    FP32-mixed batch and FP64 one at a time, both at tol 1e-6."""
    g = _golden("batch_members.json")
    probs = W.config_batch(count=64, prec=W.FP32_MIXED)
    sel = [probs[m["index"]] for m in g["members"]]
    res32 = B.batch_solve(sel, prec=W.FP32_MIXED)
    for m, p, r in zip(g["members"], sel, res32):
        r64 = B.solve(p, prec=W.FP64, fields=False)
        e32 = rel_err(r["macro_sigma"], m["macro_sigma"])
        e64 = rel_err(r64["macro_sigma"], m["macro_sigma"])
        print(f"batch member {m['index']} n={p.n[0]} iters fp32 {r['iters']} fp64 {r64['iters']} oracle "
              f"{m['iters']} macro err fp32 {e32:.2e} fp64 {e64:.2e}", flush=True)
        assert r["rc"] == 0 and all(r64["converged"])
        assert e32 < 1e-5 and e64 < 1e-5


def test_cp32_served_against_golden(B):
    """A 32^3 request of the serving configuration (crystal plasticity,
    10 torsion-bending increments) served in FP32-mixed and solved in FP64:
    <sigma> of every increment against the oracle's."""
    from tests.golden.make_config_goldens import cp_request
    g = _golden("cp32.json")
    prob = cp_request()
    srv = B.Server(arena_bytes=1 << 30, max_active=4)
    t = srv.submit(prob, arrival_s=0.0, prec=W.FP32_MIXED)
    for _ in range(20000):
        srv.step(8, 0.0)
        if srv.poll(t)[0] == 2:
            break
    served = srv.result(t)
    srv.close()
    r64 = B.solve(prob, prec=W.FP64)
    e32 = rel_err(served["macro_sigma"], g["macro_sigma"])
    e64 = rel_err(r64["macro_sigma"], g["macro_sigma"])
    es64 = _l2(_sampled_sigma(r64["sig"], g["voxels_xyz"]), g["sigma"])
    print(f"cp32 iters served {served['iters']} fp64 {r64['iters']} oracle {g['iters']} macro err served "
          f"{e32:.2e} fp64 {e64:.2e} fp64 sigma L2 {es64:.2e}", flush=True)
    assert e32 < 1e-5 and e64 < 1e-5
    assert es64 < 1e-5


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLD, "j2_inclusions64.json")),
                    reason="oracle golden of the 64^3 elastoplastic workload not generated")
@pytest.mark.parametrize("green", [W.GREEN_B0, W.GREEN_C0])
def test_j2_64_against_golden(B, green):
    """The normal-mixed elastoplastic workload at a 64^3 downscale, all 20
    increments, FP32-mixed and FP64 at tol 1e-6, with the B0 and the C0
    operator: <sigma> per increment against the oracle's."""
    g = _golden("j2_inclusions64.json")
    prob = W.config_j2_inclusions(nv=64, prec=W.FP64)
    prob.green = green
    for prec in (W.FP64, W.FP32_MIXED):
        r = B.solve(prob, prec=prec, fields=False)
        e = rel_err(r["macro_sigma"], g["macro_sigma"])
        print(f"j2 64^3 green={green} prec={prec} iters {r['iters']} macro err {e:.2e}", flush=True)
        assert all(r["converged"])
        assert e < 1e-5


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLD, "polycrystal256.json")),
                    reason="oracle golden of the 256^3 polycrystal not generated")
@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
def test_polycrystal256_against_golden(B, prec):
    """The benchmarked 256^3 polycrystal in the launch configuration the
    benchmark times: <sigma>, the stress at 1024 sampled voxels (corners,
    edges and faces of the box included, where the mirror rules act) and the
    displacement at 256 sampled nodes."""
    g = _golden("polycrystal256.json")
    prob = W.config_polycrystal_bending(nv=256)
    r = B.solve(prob, prec=prec)
    em = rel_err(r["macro_sigma"], g["macro_sigma"])
    es = _l2(_sampled_sigma(r["sig"], g["voxels_xyz"]), g["sigma"])
    u = np.array([[r["u"][q, z, y, x] for q in range(3)] for x, y, z in g["nodes_xyz"]])
    eu = rel_err(u, g["u"])
    print(f"polycrystal256 prec={prec} iters {r['iters']} oracle {g['iters']} macro {em:.2e} sigma L2 {es:.2e} "
          f"u {eu:.2e}", flush=True)
    assert all(r["converged"])
    assert em < 1e-5
    assert es < (1e-5 if prec == W.FP64 else 1e-4)
    assert eu < 1e-5
