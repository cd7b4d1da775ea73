"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances: FP64 results agree with the oracle to round-off (1e-10 relative
on fields, derived from the condition of the transforms and stencils); the
FP32-mixed path stores fields in FP32 (unit round-off 6e-8), so single
operator applications agree to 1e-5 relative and converged macroscopic
stresses to the 1e-5 target of the FP32 mode.
"""
import zlib

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
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return binding


def _cases():
    out = []
    rng = np.random.default_rng(2024)
    sizes = [(5, 4, 6), (8, 7, 9), (16, 12, 10), (33, 20, 17)]
    for k, n in enumerate(sizes):
        for scheme in (W.HEX1, W.TETRA2):
            out.append((int(rng.integers(1 << 30)), n, scheme, k % 2))
    return out


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
@pytest.mark.parametrize("seed,n,scheme,green", _cases())
def test_green_apply(B, prec, seed, n, scheme, green):
    rng = np.random.default_rng(seed)
    prob = W.random_small_problem(rng, n=n, scheme=scheme)
    prob.green = green
    pl = osolver.Plan(prob)
    x = rng.standard_normal((3,) + tuple(v + 1 for v in n))
    for q in range(3):
        fd.zero_dismissed(x[q], pl.exts[q])
    ref = -pl.green_apply(x)
    gp = B.Plan(prob, prec=prec)
    got = xyz_nodes_from_zyx(gp.apply_green(zyx_nodes_from_xyz(x)))
    gp.close()
    tol = 1e-11 if prec == W.FP64 else 2e-5
    print(f"green n={n} scheme={scheme} green={green} prec={prec} err={rel_err(got, ref):.2e}", flush=True)
    assert rel_err(got, ref) < tol


# Grids whose pencil lengths L = 64 E reach every wavefront-kernel variant
# (E = 1, 2, 3, 4, 5, 6, 8, 12) on the x, y and z axes, for each transform kind;
# the 512-point DFT shapes reach the E = 8 periodic (r2c and complex) kernels.
# The 16-, 32-, 48- and 96-point pencils (n = 8, 16, 24, 48; DFT and the
# doubled DTT lengths) take the kernels with two or four pencils per
# wavefront (32 / 16 lanes each), also on the x passes with their wider tiles;
# the 96-cell y and z axes reach the FP32 kind-specific kernels of 96- and
# 192-point pencils on complex (post-r2c) data.
WAVE_SHAPES = [(256, 6, 5), (6, 256, 5), (5, 6, 256), (96, 160, 6), (192, 7, 128), (64, 32, 384),
               (512, 5, 6), (6, 512, 5), (5, 6, 512),
               (48, 16, 5), (16, 48, 7), (5, 24, 48), (24, 7, 16), (8, 48, 24), (6, 96, 5), (5, 6, 96)]
BC_PATTERNS = {
    "P": [W.P, W.P], "N": [W.N, W.N], "D": [W.D, W.D], "ND": [W.N, W.D], "DN": [W.D, W.N],
}


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
@pytest.mark.parametrize("shape", WAVE_SHAPES)
@pytest.mark.parametrize("pattern", ["P", "N", "D", "mix"])
def test_green_apply_wave_lengths(B, prec, shape, pattern):
    rng = np.random.default_rng(zlib.crc32(repr((shape, pattern)).encode()))
    prob = W.random_small_problem(rng, n=shape, scheme=W.TETRA2 if pattern == "mix" else W.HEX1)
    bc = np.zeros((3, 3, 2), dtype=np.int32)
    names = list(BC_PATTERNS)
    for q in range(3):
        for i in range(3):
            key = pattern if pattern != "mix" else names[(q + 2 * i) % len(names)]
            bc[q, i] = BC_PATTERNS[key]
    prob.bc = bc
    pl = osolver.Plan(prob)
    x = rng.standard_normal((3,) + tuple(v + 1 for v in shape))
    for q in range(3):
        fd.zero_dismissed(x[q], pl.exts[q])
    ref = -pl.green_apply(x)
    gp = B.Plan(prob, prec=prec)
    got = xyz_nodes_from_zyx(gp.apply_green(zyx_nodes_from_xyz(x)))
    gp.close()
    tol = 1e-11 if prec == W.FP64 else 2e-5
    print(f"green-wave shape={shape} pattern={pattern} prec={prec} err={rel_err(got, ref):.2e}", flush=True)
    assert rel_err(got, ref) < tol


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
@pytest.mark.parametrize("law", ["iso", "cubic", "j2", "cp"])
@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
def test_residual(B, prec, law, scheme):
    rng = np.random.default_rng(7 + 13 * scheme + 101 * ["iso", "cubic", "j2", "cp"].index(law))
    n = (9, 7, 8)
    prob = W.random_small_problem(rng, n=n, scheme=scheme, law=law)
    pl = osolver.Plan(prob)
    uf = 1e-3 * rng.standard_normal((3,) + tuple(v + 1 for v in n))
    for q in range(3):
        fd.zero_dismissed(uf[q], pl.exts[q])
    step = prob.steps[0]
    mats = MaterialSet(prob.materials, np.asarray(prob.mat_id).transpose(2, 1, 0))
    state = mats.init_state(pl.nppv, pl.n)
    us = pl.ustar(step.c, step.G, step.H)
    gu = pl.grad(uf) + pl.grad(us)
    eps = 0.5 * (gu + np.swapaxes(gu, -1, -2))
    sig, _ = mats.stress(eps, state, step.dt)
    Dref = pl.div(sig)
    gp = B.Plan(prob, prec=prec)
    D, err, macro = gp.residual(zyx_nodes_from_xyz(uf), step)
    gp.close()
    D = xyz_nodes_from_zyx(D)
    # FP32-mixed: the plastic laws run in FP64 and store their stress in FP32,
    # elastic ones run in FP32; either way D carries the FP32 rounding of the
    # stresses it sums (unit round-off 6e-8 times the stencil's cancellation)
    tol = 1e-10 if prec == W.FP64 else 5e-5
    # compare at the kept nodes (periodic duplicates and Dirichlet nodes carry no equation)
    kept = np.stack(pl.kept)
    e = rel_err(D[kept], Dref[kept])
    assert np.all(D[~kept] == 0.0)
    ms = sig.mean(axis=(0, 1, 2, 3))
    mref = np.array([ms[i, j] for (i, j) in osolver.VOIGT])
    err_ref = osolver.equilibrium_error(pl, Dref, sig)
    e_err = abs(err - err_ref) / err_ref
    print(f"residual law={law} scheme={scheme} prec={prec} D err={e:.2e} macro err={rel_err(macro, mref):.2e} "
          f"eq. error {err:.6e} vs {err_ref:.6e}", flush=True)
    assert e < tol
    assert rel_err(macro, mref) < (1e-12 if prec == W.FP64 else 1e-5)
    assert e_err < (1e-12 if prec == W.FP64 else 1e-5)


def _bc_pattern(rng, pattern):
    """Boundary codes [q][axis][side] for the multi-tile residual cases."""
    bc = np.zeros((3, 3, 2), dtype=np.int32)
    if pattern == "P":
        return bc
    if pattern in ("D", "N"):
        bc[:] = W.D if pattern == "D" else W.N
        return bc
    for q in range(3):
        for i in range(3):
            if pattern == "mixwrap" and i == q:
                continue                       # u_q periodic along axis q only
            bc[q, i, 0] = rng.integers(1, 3)
            bc[q, i, 1] = rng.integers(1, 3)
    return bc


# Grids spanning several stress-divergence tiles (31 x 7 node columns, 16
# layers): ragged last tiles, a one-column tile (63 nodes), a one-layer
# z chunk (17 nodes), one tile exactly (31 nodes).
TILE_SHAPES = [(40, 17, 35), (62, 13, 33), (30, 6, 16)]


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_MIXED])
@pytest.mark.parametrize("pattern", ["P", "D", "N", "mix", "mixwrap"])
@pytest.mark.parametrize("shape", TILE_SHAPES)
def test_residual_tiles(B, prec, pattern, shape):
    seed = zlib.crc32(f"{shape}{pattern}".encode())
    rng = np.random.default_rng(seed)
    scheme = W.TETRA2 if seed % 2 else W.HEX1
    prob = W.random_small_problem(rng, n=shape, scheme=scheme, law="cubic",
                                  bc=_bc_pattern(rng, pattern))
    pl = osolver.Plan(prob)
    uf = 1e-3 * rng.standard_normal((3,) + tuple(v + 1 for v in shape))
    for q in range(3):
        fd.zero_dismissed(uf[q], pl.exts[q])
    step = prob.steps[0]
    mats = MaterialSet(prob.materials, np.asarray(prob.mat_id).transpose(2, 1, 0))
    state = mats.init_state(pl.nppv, pl.n)
    gu = pl.grad(uf) + pl.grad(pl.ustar(step.c, step.G, step.H))
    eps = 0.5 * (gu + np.swapaxes(gu, -1, -2))
    sig, _ = mats.stress(eps, state, step.dt)
    Dref = pl.div(sig)
    gp = B.Plan(prob, prec=prec)
    D, err, macro = gp.residual(zyx_nodes_from_xyz(uf), step)
    gp.close()
    D = xyz_nodes_from_zyx(D)
    kept = np.stack(pl.kept)
    e = rel_err(D[kept], Dref[kept])
    ms = sig.mean(axis=(0, 1, 2, 3))
    mref = np.array([ms[i, j] for (i, j) in osolver.VOIGT])
    print(f"residual-tiles shape={shape} pattern={pattern} scheme={scheme} prec={prec} "
          f"D err={e:.2e} macro err={rel_err(macro, mref):.2e}", flush=True)
    assert np.all(D[~kept] == 0.0)
    assert e < (1e-10 if prec == W.FP64 else 5e-5)
    assert rel_err(macro, mref) < (1e-12 if prec == W.FP64 else 1e-5)


@pytest.mark.parametrize("scheme", [W.HEX1, W.TETRA2])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_small_solve_fp64(B, scheme, seed):
    rng = np.random.default_rng(500 + seed)
    prob = W.random_small_problem(rng, n=(7, 6, 9), scheme=scheme, tol=1e-10,
                                  law="iso" if seed != 3 else "cubic")
    prob.green = seed % 2
    ref = osolver.solve(prob)
    got = B.solve(prob, prec=W.FP64)
    print(f"solve scheme={scheme} seed={seed} iters gpu={got['iters']} oracle={ref['iters']}", flush=True)
    assert got["converged"][0]
    assert rel_err(got["sig"], ref["sig"]) < 1e-7
    assert rel_err(got["eps"], ref["eps"]) < 1e-7
    assert rel_err(got["macro_sigma"], ref["macro_sigma"]) < 1e-8
