"""Full-size checks on the 256^3 polycrystal (the benchmarked workload, the
launch configuration bench.py times), on samples the oracle evaluates one by
one and on properties that hold at any size.

* FP32-mixed and FP64 solves both converge and their macroscopic stresses
  agree to 1e-5 relative (the FP32-mixed accuracy target).
* Strain and stress at sampled voxels: the oracle's stencil applied to the
  GPU displacement reproduces the GPU strain at every integration point, and
  the oracle's law applied to that strain reproduces the GPU stress (FP64
  round-off for the FP64 path; FP32 for the FP32 path).
* Equilibrium at sampled interior nodes: the oracle's divergence of the GPU
  stress is negligible against the stress scale (a converged solution of the
  discrete equations, err < 1e-6 in the RMS sense).
"""
import numpy as np
import pytest

import workloads as W
from oracle import fd
from oracle.laws import MaterialSet
from tests.gpu_util import rel_err

pytestmark = pytest.mark.gpu

VOIGT = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


@pytest.fixture(scope="module")
def runs():
    from paper_2607_05929_amd import binding as B
    B.lib()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    prob = W.config_polycrystal_bending(nv=256)
    out = {}
    for prec in (W.FP64, W.FP32_MIXED):
        p = B.Plan(prob, prec=prec)
        out[prec] = p.solve(fields=True)
        p.close()
        print(f"fullsize prec={prec} iters={out[prec]['iters']} converged={out[prec]['converged']}", flush=True)
    return prob, out


def _tensor(v6):
    """Voigt (tensor shears) -> 3x3, last axis first."""
    t = np.zeros(v6.shape[1:] + (3, 3))
    for k, (i, j) in enumerate(VOIGT):
        t[..., i, j] = v6[k]
        t[..., j, i] = v6[k]
    return t


def test_fullsize_converged_and_fp32_matches_fp64(runs):
    prob, out = runs
    r64, r32 = out[W.FP64], out[W.FP32_MIXED]
    assert all(r64["converged"]) and all(r32["converged"])
    m64, m32 = r64["macro_sigma"][-1], r32["macro_sigma"][-1]
    d = rel_err(m32, m64)
    print(f"fullsize <sigma> FP32 vs FP64 rel diff {d:.2e}", flush=True)
    assert d < 1e-5


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
def test_fullsize_sampled_strain_and_stress(runs, prec):
    prob, out = runs
    r = out[prec]
    u, eps, sig = r["u"], r["eps"], r["sig"]          # zyx layouts
    n1, n2, n3 = prob.n
    rng = np.random.default_rng(11)
    vox = np.stack([rng.integers(0, n1, 256), rng.integers(0, n2, 256), rng.integers(0, n3, 256)], axis=1)
    vox[:8] = [[0, 0, 0], [n1 - 1, 0, 0], [0, n2 - 1, 0], [0, 0, n3 - 1],
               [n1 - 1, n2 - 1, n3 - 1], [n1 // 2, 0, n3 // 2], [0, n2 // 2, n3 - 1], [n1 - 1, n2 // 2, 0]]
    mat_id = np.asarray(prob.mat_id)
    e_ref, e_gpu, s_gpu, ids = [], [], [], []
    for x, y, z in vox:
        patch = u[:, z:z + 2, y:y + 2, x:x + 2].transpose(0, 3, 2, 1)    # (3, 2, 2, 2) xyz
        g = fd.gradient(patch, prob.scheme, prob.h)                       # (nppv, 1, 1, 1, 3, 3)
        e_ref.append(0.5 * (g + np.swapaxes(g, -1, -2))[:, 0, 0, 0])
        e_gpu.append(_tensor(eps[:, :, z, y, x]))                         # (nppv, 3, 3)
        s_gpu.append(_tensor(sig[:, :, z, y, x]))
        ids.append(mat_id[z, y, x])
    e_ref, e_gpu, s_gpu = map(np.array, (e_ref, e_gpu, s_gpu))           # (samples, nppv, 3, 3)
    # the oracle law on the GPU strain, all samples as one (samples, 1, 1) grid
    mats = MaterialSet(prob.materials, np.array(ids).reshape(-1, 1, 1))
    E = np.swapaxes(e_gpu, 0, 1)[:, :, None, None]                        # (nppv, samples, 1, 1, 3, 3)
    st = mats.init_state(E.shape[0], (len(ids), 1, 1))
    sref, _ = mats.stress(E, st, prob.steps[0].dt)
    s_ref = np.swapaxes(sref[:, :, 0, 0], 0, 1)
    de, ds = rel_err(e_gpu, e_ref), rel_err(s_gpu, s_ref)
    print(f"fullsize sampled prec={prec} strain err {de:.2e} stress err {ds:.2e}", flush=True)
    tol = 1e-10 if prec == W.FP64 else 2e-5
    assert de < tol and ds < tol


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
def test_fullsize_sampled_equilibrium(runs, prec):
    prob, out = runs
    sig = out[prec]["sig"]
    n1, n2, n3 = prob.n
    rng = np.random.default_rng(12)
    nodes = np.stack([rng.integers(1, n1, 64), rng.integers(1, n2, 64), rng.integers(1, n3, 64)], axis=1)
    s_rms = np.sqrt(np.mean(np.sum(_tensor(sig[:, :, ::8, ::8, ::8].reshape(6, -1)) ** 2, axis=(-1, -2))))
    ext = [[("P", "P")] * 3] * 3     # interior nodes: the extension of the patch is not used
    worst = 0.0
    for x, y, z in nodes:
        S = _tensor(sig[:, :, z - 1:z + 1, y - 1:y + 1, x - 1:x + 1].reshape(6, -1)).reshape(
            sig.shape[1], 2, 2, 2, 3, 3).transpose(0, 3, 2, 1, 4, 5)        # (nppv, 2, 2, 2, 3, 3) xyz
        D = fd.divergence(S, ext, prob.scheme, prob.h)[:, 1, 1, 1]
        worst = max(worst, float(np.abs(D).max()) * prob.h / s_rms)
    print(f"fullsize equilibrium prec={prec} max |D| h / sigma_rms = {worst:.2e}", flush=True)
    assert worst < 1e-4


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
def test_fullsize_sampled_equilibrium_on_faces(runs, prec):
    """Equilibrium at sampled nodes on the traction-free y and z faces, their
    edges and the corners they share, where the mirror rules act (the
    x faces carry Dirichlet conditions: their nodes are dismissed): the
    oracle's divergence of the GPU stress, with the problem's own extension
    along the face normals, is negligible against the stress scale."""
    from oracle import dt as odt
    prob, out = runs
    sig = out[prec]["sig"]
    n1, n2, n3 = prob.n
    bc = np.asarray(prob.bc)
    rng = np.random.default_rng(13)
    s_rms = np.sqrt(np.mean(np.sum(_tensor(sig[:, :, ::8, ::8, ::8].reshape(6, -1)) ** 2, axis=(-1, -2))))
    cases = []
    for _ in range(24):
        x = int(rng.integers(1, n1))
        y, z = int(rng.integers(1, n2)), int(rng.integers(1, n3))
        kind = rng.integers(0, 3)
        if kind == 0:
            y = int(rng.choice([0, n2]))
        elif kind == 1:
            z = int(rng.choice([0, n3]))
        else:
            y, z = int(rng.choice([0, n2])), int(rng.choice([0, n3]))
        cases.append((x, y, z))
    worst = 0.0
    for x, y, z in cases:
        # voxel patch around the node, clipped at the faces; the node's index in the patch
        lo = [x - 1, max(y - 1, 0), max(z - 1, 0)]
        hi = [x + 1, min(y + 1, n2), min(z + 1, n3)]
        idx = [1, y - lo[1], z - lo[2]]
        ext = []
        for q in range(3):
            e = [(odt.EXT_P, odt.EXT_P)]
            for a, J, n in ((1, y, n2), (2, z, n3)):
                if J in (0, n):   # the face's own extension on both sides of the (thin) patch
                    side = odt.ext_of_bc(bc[q, a, 0 if J == 0 else 1])
                    e.append((side, side))
                else:
                    e.append((odt.EXT_P, odt.EXT_P))
            ext.append(e)
        blk = sig[:, :, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        shp = blk.shape[2:]
        S = _tensor(blk.reshape(6, -1)).reshape((sig.shape[1],) + shp + (3, 3)).transpose(0, 3, 2, 1, 4, 5)
        D = fd.divergence(S, ext, prob.scheme, prob.h)[:, idx[0], idx[1], idx[2]]
        worst = max(worst, float(np.abs(D).max()) * prob.h / s_rms)
    print(f"fullsize face equilibrium prec={prec} max |D| h / sigma_rms = {worst:.2e}", flush=True)
    assert worst < 1e-4
