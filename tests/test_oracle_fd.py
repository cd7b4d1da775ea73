"""Pins of the oracle stencils and Green operators.

P4: real-space second derivatives (with the symmetry / periodicity extensions
    of the fields) equal the spectral multiply by -|xi|^2 and -|xi_q|^2 for all
    125 per-axis transform combinations and both schemes: the cross-validation
    of Sec. 3.2 (Discrete derivation), relative squared error below 1e-13.
P5: Green(L0 u) = u for fields without null-mode content.
P6: the divergence of the stress equals the nodal force of an independently
    assembled finite-element operator (HEX1: one-point trilinear hexahedron;
    TETRA2: two inscribed linear tetrahedra, each weighted by half the voxel),
    times 2 per symmetric (Neumann) face the node lies on.
Null-mode counts on a periodic 8^3 grid (HEX1: 23, TETRA2: 2).
"""
import itertools

import numpy as np
import pytest

from oracle import dt, fd, green

EXT_OF_KIND = {dt.DFT: ("P", "P"), dt.DCT1: ("S", "S"), dt.DST1: ("A", "A"),
               dt.DCT3: ("S", "A"), dt.DST3: ("A", "S")}


def _random_field(rng, kinds, n):
    u = rng.standard_normal(tuple(v + 1 for v in n))
    fd.zero_dismissed(u, [EXT_OF_KIND[k] for k in kinds])
    return u


def _real_second(u, kinds, n, scheme, h, mode):
    """mode 'lap': sum_l D_l D_l u; mode q: D_q D_q u (as component-q term)."""
    ext3 = [[EXT_OF_KIND[k] for k in kinds]] * 3
    U = np.zeros((3,) + u.shape)
    U[0] = u
    g = fd.gradient(U, scheme, h)            # (nppv, n1, n2, n3, l, q)
    w = np.zeros((3, 3))
    if mode == "lap":
        w[:, 0] = 1.0
    else:
        w[mode, 0] = 1.0
    return fd.divergence(g * w, ext3, scheme, h)[0]


def _spectral_second(u, kinds, n, scheme, h, mode):
    tot, comp = green.xi_components(kinds, n, scheme, h)
    mult = tot if mode == "lap" else comp[mode]
    return dt.inverse_3d(-mult * dt.forward_3d(u, kinds), kinds, n)


@pytest.mark.parametrize("scheme", [0, 1])
def test_cross_validation_all_combinations(scheme):
    rng = np.random.default_rng(11 + scheme)
    n = (4, 5, 6)
    h = 0.7
    worst = 0.0
    for kinds in itertools.product(range(5), repeat=3):
        u = _random_field(rng, kinds, n)
        sl = np.ix_(*[dt.kept_nodes(kinds[i], n[i]) for i in range(3)])
        for mode in ("lap", 0, 1, 2):
            a = _real_second(u, kinds, n, scheme, h, mode)[sl]
            b = _spectral_second(u, kinds, n, scheme, h, mode)[sl]
            rel = np.sum((a - b) ** 2) / max(np.sum(b ** 2), 1e-300)
            worst = max(worst, rel)
    assert worst < 1e-13, worst


@pytest.mark.parametrize("scheme", [0, 1])
def test_green_inverts_L0(scheme):
    from oracle.solver import Plan
    import workloads as W
    rng = np.random.default_rng(5)
    for trial in range(12):
        prob = W.random_small_problem(rng, n=(5, 4, 6), scheme=scheme)
        prob.green = trial % 2
        pl = Plan(prob)
        x = rng.standard_normal((3, 6, 5, 7))
        for q in range(3):
            fd.zero_dismissed(x[q], pl.exts[q])
        u = pl.green_apply(x)          # has no null-mode content by construction
        back = pl.green_apply(pl.L0(u))
        np.testing.assert_allclose(back, u, atol=1e-12 * np.abs(u).max())


def test_null_mode_counts_periodic_8():
    n = (8, 8, 8)
    kinds = [dt.DFT] * 3
    assert int(green.null_mask(kinds, n, 0).sum()) == 23
    assert int(green.null_mask(kinds, n, 1).sum()) == 2
    # the index-space mask agrees with a floating-point zero test here
    tot, _ = green.xi_components(kinds, n, 0, 1.0)
    assert np.all((tot < 1e-20) == green.null_mask(kinds, n, 0))


# ---------------------------------------------------------------- P6: FE assembly
def _tet_grads(pts):
    """Gradients of the 4 linear shape functions of a tetrahedron."""
    A = np.hstack([np.ones((4, 1)), pts])
    inv = np.linalg.inv(A)
    return inv[1:].T              # (4 nodes, 3)


def _fe_force(u, Cvox, n, h, scheme, periodic):
    """Internal nodal force f_a = sum_e w_e B_a^T sigma_e on a (possibly periodic) grid."""
    N = tuple(v + 1 for v in n)
    f = np.zeros((3,) + N)
    corners = list(itertools.product((0, 1), repeat=3))
    if scheme == 0:
        sets = [(corners, np.array([[(2 * a[i] - 1) / (4.0 * h) for i in range(3)] for a in corners]), 1.0)]
    else:
        even = [c for c in corners if sum(c) % 2 == 0]
        odd = [c for c in corners if sum(c) % 2 == 1]
        sets = []
        for tet in (even, odd):
            pts = np.array(tet, dtype=float) * h
            sets.append((tet, _tet_grads(pts), 0.5))
    for j1, j2, j3 in itertools.product(range(n[0]), range(n[1]), range(n[2])):
        C = Cvox[j1, j2, j3]
        for nodes, B, wt in sets:
            idx = [(j1 + a[0], j2 + a[1], j3 + a[2]) for a in nodes]
            gu = np.zeros((3, 3))             # gu[l, q] = d u_q / d x_l
            for (i1, i2, i3), b in zip(idx, B):
                gu += np.outer(b, u[:, i1, i2, i3])
            eps = 0.5 * (gu + gu.T)
            sig = np.einsum("ijkl,kl->ij", C, eps)
            for (i1, i2, i3), b in zip(idx, B):
                f[:, i1, i2, i3] += wt * h ** 3 * (sig.T @ b)
    for i in range(3):                        # fold periodic duplicates
        if periodic[i]:
            s0 = [slice(None)] * 4; s0[i + 1] = 0
            sn = [slice(None)] * 4; sn[i + 1] = -1
            f[tuple(s0)] += f[tuple(sn)]
            f[tuple(sn)] = f[tuple(s0)]
    return f


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_divergence_equals_fe_assembly(scheme, seed):
    from oracle.laws import iso_tensor
    rng = np.random.default_rng(40 + seed)
    n = (3, 4, 3)
    h = 1.3
    types = [int(v) for v in rng.integers(0, 3, size=3)]   # per axis P / S / A for all comps
    extmap = {0: ("P", "P"), 1: ("S", "S"), 2: ("A", "A")}
    if seed == 2:
        types = [1, 1, 0]
    ext = [extmap[t] for t in types]
    ext3 = [ext] * 3
    u = rng.standard_normal((3,) + tuple(v + 1 for v in n))
    for q in range(3):
        fd.zero_dismissed(u[q], ext)
    lam = rng.uniform(0.5, 2.0, size=n)
    mu = rng.uniform(0.5, 2.0, size=n)
    Cvox = np.array([iso_tensor(l, m) for l, m in zip(lam.ravel(), mu.ravel())]).reshape(n + (3, 3, 3, 3))
    g = fd.gradient(u, scheme, h)
    eps = 0.5 * (g + np.swapaxes(g, -1, -2))
    sig = np.einsum("xyzijkl,rxyzkl->rxyzij", Cvox, eps)
    D = fd.divergence(sig, ext3, scheme, h)
    f = _fe_force(u, Cvox, n, h, scheme, [t == 0 for t in types])
    # weight: 2 per symmetric face the node lies on
    w = np.ones(tuple(v + 1 for v in n))
    for i in range(3):
        if ext[i][0] == "S":
            s = [slice(None)] * 3; s[i] = 0; w[tuple(s)] *= 2.0
        if ext[i][1] == "S":
            s = [slice(None)] * 3; s[i] = -1; w[tuple(s)] *= 2.0
    for q in range(3):
        keep = fd.kept_mask(ext, n)
        np.testing.assert_allclose(D[q][keep], (-f[q] / h ** 3 * w)[keep], atol=1e-12)
