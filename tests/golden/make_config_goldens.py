"""Writes the oracle goldens of the five workload configurations.

Every value stored here comes from the FP64 oracle (``oracle/``) run on the
seeded problem descriptions of ``workloads``; nothing is read from the HIP
library.  Run on a CPU host (the 256^3 polycrystal takes about 90 minutes
and ~25 GB of memory):

    python tests/golden/make_config_goldens.py poly256 j2_64 batch cp32 inclusion32

Outputs (JSON, next to this script):

* ``polycrystal256.json`` -- 256^3 Voronoi polycrystal (500 grains, seed 2),
  cubic elasticity, bending, TETRA2, B0, solved to tol 1e-8: <sigma>, the
  iteration count, the stress at both integration points of 1024 sampled
  voxels (corners, edges and faces of the box included) and the displacement
  at 256 sampled nodes.
* ``j2_inclusions64.json`` -- the elastoplastic workload at a 64^3 downscale
  (same sphere radii 6-12 voxels, 20 % volume fraction, seed 3), 20
  increments to eps_zz = 2e-2 with <sigma_xx> = <sigma_yy> = 0, HEX1, tol
  1e-8: <sigma> and iterations per increment.
* ``batch_members.json`` -- eight of the first 64 solves of the batched
  configuration (seed 4), among them the high-contrast members whose FP32
  residual converges slowest, solved to tol 1e-8: <sigma>.
* ``cp32.json`` -- one 32^3 request of the serving configuration (FCC
  crystal plasticity, 10 torsion-bending increments, TETRA2), tol 1e-8:
  <sigma> per increment and the stress at 256 sampled voxels.
* ``inclusion32.json`` -- the 32^3 inclusion workload at tol 1e-10: <sigma>
  and the stress at 256 sampled voxels.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import solver as osolver  # noqa: E402

BATCH_MEMBERS = [0, 1, 3, 12, 16, 21, 39, 63]


def sample_voxels(n, count, seed):
    """Voxel indices (x, y, z): the 8 corners, the 12 edge midpoints, the 6
    face centres, then uniform random voxels."""
    rng = np.random.default_rng(seed)
    n1, n2, n3 = n
    pts = []
    for x in (0, n1 - 1):
        for y in (0, n2 - 1):
            for z in (0, n3 - 1):
                pts.append((x, y, z))
    mx, my, mz = n1 // 2, n2 // 2, n3 // 2
    for a in (0, n1 - 1):
        for b in (0, n2 - 1):
            pts.append((a, b, mz))
    for a in (0, n1 - 1):
        for c in (0, n3 - 1):
            pts.append((a, my, c))
    for b in (0, n2 - 1):
        for c in (0, n3 - 1):
            pts.append((mx, b, c))
    pts += [(0, my, mz), (n1 - 1, my, mz), (mx, 0, mz), (mx, n2 - 1, mz), (mx, my, 0), (mx, my, n3 - 1)]
    while len(pts) < count:
        pts.append((int(rng.integers(0, n1)), int(rng.integers(0, n2)), int(rng.integers(0, n3))))
    return np.array(pts[:count], dtype=np.int64)


def sample_nodes(n, count, seed):
    rng = np.random.default_rng(seed)
    N = [v + 1 for v in n]
    pts = [(0, 0, 0), (N[0] - 1, N[1] - 1, N[2] - 1), (0, N[1] // 2, N[2] // 2), (N[0] - 1, N[1] // 2, N[2] // 2)]
    while len(pts) < count:
        pts.append(tuple(int(rng.integers(0, v)) for v in N))
    return np.array(pts[:count], dtype=np.int64)


def write(name, data):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(data, f, indent=None, separators=(",", ":"))
    print(f"wrote {path}", flush=True)


def progress(tag):
    t0 = time.time()

    def cb(t, m, err):
        print(f"[{tag}] step {t} iter {m} err {err:.3e} ({time.time() - t0:.0f} s)", flush=True)
    return cb


def stress_samples(r, vox):
    """sig[c][ip][z][y][x] at the sampled voxels -> list of [n_ppv][6]."""
    sig = r["sig"]
    return [[[float(sig[c, ip, z, y, x]) for c in range(6)] for ip in range(sig.shape[1])]
            for x, y, z in vox]


def poly256():
    prob = W.config_polycrystal_bending(nv=256, tol=1e-8)
    prob.max_iter = 400
    r = osolver.solve(prob, callback=progress("poly256"))
    vox = sample_voxels(prob.n, 1024, seed=256)
    nodes = sample_nodes(prob.n, 256, seed=257)
    u = r["u"]
    write("polycrystal256.json", {
        "workload": "256^3 Voronoi polycrystal, 500 grains (seed 2), cubic 168/121/75 GPa, bending "
                    "kappa 1e-4, Dirichlet x faces, Neumann y, z; TETRA2, B0 (121, 75)",
        "oracle_tol": prob.tol, "iters": r["iters"], "converged": r["converged"],
        "macro_sigma": r["macro_sigma"].tolist(),
        "voxels_xyz": vox.tolist(), "sigma": stress_samples(r, vox),
        "nodes_xyz": nodes.tolist(),
        "u": [[float(u[q, z, y, x]) for q in range(3)] for x, y, z in nodes],
    })


def j2_64():
    prob = W.config_j2_inclusions(nv=64, tol=1e-8, prec=W.FP64)
    prob.max_iter = 5000
    r = osolver.solve(prob, callback=progress("j2_64"))
    write("j2_inclusions64.json", {
        "workload": "64^3 downscale of the elastoplastic workload: elastic spheres (E 400 GPa, nu 0.2, "
                    "radius 6-12 voxels, 20 % volume fraction, seed 3) in a J2 matrix (E 70 GPa, "
                    "nu 0.33, sy0 0.1 GPa, H 1 GPa); 20 increments to eps_zz 2e-2, <sigma_xx> = "
                    "<sigma_yy> = 0; HEX1, B0",
        "oracle_tol": prob.tol, "iters": r["iters"], "converged": r["converged"],
        "macro_sigma": r["macro_sigma"].tolist(), "G": r["G"].tolist(),
    })


def batch():
    probs = W.config_batch(count=64, prec=W.FP64)
    out = []
    for k in BATCH_MEMBERS:
        p = probs[k]
        p.tol = 1e-8
        p.max_iter = 5000
        r = osolver.solve(p, callback=progress(f"batch{k}") if k == BATCH_MEMBERS[0] else None)
        print(f"batch member {k} n={p.n} iters {r['iters']}", flush=True)
        out.append({"index": k, "n": list(p.n), "iters": r["iters"], "converged": r["converged"],
                    "macro_sigma": r["macro_sigma"].tolist()})
    write("batch_members.json", {
        "workload": "first 64 draws of the batched configuration (seed 4): members " + str(BATCH_MEMBERS),
        "oracle_tol": 1e-8, "members": out})


def cp_request():
    """The serving configuration's first draw with the grid size forced to
    32^3: same seed-5 stream of grain counts and orientations."""
    reqs = W.serving_stream(count=1, sizes=(32,), prec=W.FP64)
    return reqs[0].problem


def cp32():
    prob = cp_request()
    prob.tol = 1e-8
    prob.max_iter = 3000
    r = osolver.solve(prob, callback=progress("cp32"))
    vox = sample_voxels(prob.n, 256, seed=32)
    write("cp32.json", {
        "workload": "32^3 request of the serving configuration (seed 5 stream, first draw): FCC crystal "
                    "plasticity polycrystal, torsion-bending, 10 increments; TETRA2, B0 (121, 75)",
        "grains": len(prob.materials), "oracle_tol": prob.tol, "iters": r["iters"],
        "converged": r["converged"], "macro_sigma": r["macro_sigma"].tolist(),
        "voxels_xyz": vox.tolist(), "sigma": stress_samples(r, vox),
    })


def inclusion32():
    prob = W.config_inclusion32()
    prob.tol = 1e-10
    r = osolver.solve(prob)
    vox = sample_voxels(prob.n, 256, seed=33)
    write("inclusion32.json", {
        "workload": "32^3 inclusion (R 8, E 1 / 10, nu 0.3), eps_zz 1e-3 by Dirichlet z faces, Neumann x, "
                    "periodic y; HEX1, B0 with the mean moduli",
        "oracle_tol": prob.tol, "iters": r["iters"], "converged": r["converged"],
        "macro_sigma": r["macro_sigma"].tolist(), "voxels_xyz": vox.tolist(),
        "sigma": stress_samples(r, vox)})


JOBS = {"poly256": poly256, "j2_64": j2_64, "batch": batch, "cp32": cp32, "inclusion32": inclusion32}

if __name__ == "__main__":
    for name in sys.argv[1:] or list(JOBS):
        JOBS[name]()
