"""Pins of the oracle stencils and Green operators.

P4: real-space second derivatives (with the symmetry / periodicity extensions
    of the fields) equal the spectral multiply by -|xi|^2 and -|xi_q|^2 for all
    125 per-axis transform combinations and both schemes: the cross-validation
    of Sec. 2.7.3 (Discrete derivation), relative squared error below 1e-13.
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
    """Internal nodal force f_a = sum_e w_e B_a^T sigma_e on a (possibly periodic) grid.
    ``periodic[i]`` (one flag per axis, all components) or ``periodic[q][i]``
    (per component: the test functions of component q are periodic along i)."""
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
    per = np.broadcast_to(np.asarray(periodic, dtype=bool), (3, 3))
    for q in range(3):
        for i in range(3):                    # fold periodic duplicates
            if per[q, i]:
                s0 = [q, slice(None), slice(None), slice(None)]; s0[i + 1] = 0
                sn = [q, slice(None), slice(None), slice(None)]; sn[i + 1] = -1
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


PAIRS = [("P", "P"), ("S", "S"), ("A", "A"), ("S", "A"), ("A", "S")]


def _face_weight(ext, n):
    """2 per symmetric (Neumann) face a node of this component lies on."""
    w = np.ones(tuple(v + 1 for v in n))
    for i in range(3):
        if ext[i][0] == "S":
            s = [slice(None)] * 3; s[i] = 0; w[tuple(s)] *= 2.0
        if ext[i][1] == "S":
            s = [slice(None)] * 3; s[i] = -1; w[tuple(s)] *= 2.0
    return w


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("seed", range(6))
def test_divergence_equals_fe_assembly_per_component(scheme, seed):
    """P6 with every extension pair of Table 1 (P/P, S/S, A/A, S/A, A/S) drawn
    per component and per axis, so that an axis can be periodic for one
    component and mirror-extended for another (the per-component mixed
    conditions of the inclusion and normal-mixed workloads), on an anisotropic
    random material (the shear columns of the stress are non-zero)."""
    from oracle.laws import cubic_tensor, quat_to_rot, rotate4
    rng = np.random.default_rng(700 + seed)
    n = (3, 4, 3) if seed % 2 else (4, 3, 3)
    h = 0.9
    ext3 = [[PAIRS[int(rng.integers(0, 5))] for i in range(3)] for q in range(3)]
    if seed == 0:          # inclusion workload: N on x, P on y, D on z for every component
        ext3 = [[("S", "S"), ("P", "P"), ("A", "A")]] * 3
    if seed == 1:          # normal-mixed workload: x, y periodic; u_z D, u_x, u_y N on z
        ext3 = [[("P", "P"), ("P", "P"), ("S", "S")], [("P", "P"), ("P", "P"), ("S", "S")],
                [("P", "P"), ("P", "P"), ("A", "A")]]
    if seed == 2:          # the S/A and A/S pairs on every axis, crossed between components
        ext3 = [[("S", "A"), ("A", "S"), ("S", "A")], [("A", "S"), ("S", "A"), ("P", "P")],
                [("S", "A"), ("P", "P"), ("A", "S")]]
    u = rng.standard_normal((3,) + tuple(v + 1 for v in n))
    for q in range(3):
        fd.zero_dismissed(u[q], ext3[q])
    C0 = cubic_tensor(1.68, 1.21, 0.75)
    Cvox = np.empty(n + (3, 3, 3, 3))
    for idx in itertools.product(*[range(v) for v in n]):
        Cvox[idx] = rotate4(C0 * rng.uniform(0.5, 2.0), quat_to_rot(rng.standard_normal(4)))
    g = fd.gradient(u, scheme, h)
    eps = 0.5 * (g + np.swapaxes(g, -1, -2))
    sig = np.einsum("xyzijkl,rxyzkl->rxyzij", Cvox, eps)
    assert np.abs(sig[..., 0, 1]).max() > 1e-3
    D = fd.divergence(sig, ext3, scheme, h)
    per = [[ext3[q][i][0] == "P" for i in range(3)] for q in range(3)]
    f = _fe_force(u, Cvox, n, h, scheme, per)
    for q in range(3):
        keep = fd.kept_mask(ext3[q], n)
        w = _face_weight(ext3[q], n)
        np.testing.assert_allclose(D[q][keep], (-f[q] / h ** 3 * w)[keep], atol=1e-12)
        for i in range(3):                 # anti-symmetric faces carry no equation
            for side, idx in ((0, 0), (1, -1)):
                if ext3[q][i][side] == "A":
                    sl = [slice(None)] * 3; sl[i] = idx
                    assert np.all(D[q][tuple(sl)] == 0.0)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("seed", range(3))
def test_equilibrium_error_from_fe_assembly(scheme, seed):
    """The oracle's equilibrium error of the first iterate (u^f = 0, affine
    u*: uniform strain E in every voxel) equals h sqrt(sum_kept D^2 / sum_ip
    w_ip |sigma|_F^2) built from the independently assembled FE nodal forces
    (D = -f / h^3, times 2 per symmetric face) and the stress C(x) : E."""
    import workloads as W
    from oracle import solver as osolver
    from oracle.laws import iso_tensor
    rng = np.random.default_rng(900 + seed)
    n = (4, 3, 5)
    prob = W.random_small_problem(rng, n=n, scheme=scheme)
    E = rng.uniform(-1e-3, 1e-3, (3, 3))
    prob.steps = [W.step_affine(E)]
    prob.max_iter = 0
    prob.h = 1.3
    r = osolver.solve(prob)
    err_oracle = r["log"][0]["err"]
    pl = osolver.Plan(prob)
    ids = np.asarray(prob.mat_id).transpose(2, 1, 0)
    Cvox = np.empty(n + (3, 3, 3, 3))
    for idx in itertools.product(*[range(v) for v in n]):
        m = prob.materials[ids[idx]]
        Cvox[idx] = iso_tensor(m["lam"], m["mu"])
    us = pl.ustar(prob.steps[0].c, prob.steps[0].G, prob.steps[0].H)
    per = [[pl.exts[q][i][0] == "P" for i in range(3)] for q in range(3)]
    f = _fe_force(us, Cvox, n, prob.h, scheme, per)
    sD = 0.0
    for q in range(3):
        keep = fd.kept_mask(pl.exts[q], n)
        sD += float(np.sum(((-f[q] / prob.h ** 3) * _face_weight(pl.exts[q], n))[keep] ** 2))
    Es = 0.5 * (E + E.T)
    sig = np.einsum("xyzijkl,kl->xyzij", Cvox, Es)
    sS = float(np.sum(sig * sig))          # every integration point of a voxel carries this stress
    ref = prob.h * np.sqrt(sD / sS)
    assert ref > 0
    assert err_oracle == pytest.approx(ref, rel=1e-12)


def _fe_face_load(T, n, h, per):
    """Consistent nodal forces of uniform face tractions T[i, a, q]: every
    face cell (area h^2) gives a quarter of t_q h^2 to each of its corners;
    periodic duplicates folded per component like the internal forces."""
    N = tuple(v + 1 for v in n)
    f = np.zeros((3,) + N)
    for i in range(3):
        j, k = [a for a in range(3) if a != i]
        for a in (0, 1):
            for q in range(3):
                t = T[i, a, q]
                if t == 0:
                    continue
                for cj in range(n[j]):
                    for ck in range(n[k]):
                        for dj in (0, 1):
                            for dk in (0, 1):
                                idx = [0, 0, 0]
                                idx[i] = 0 if a == 0 else n[i]
                                idx[j] = cj + dj
                                idx[k] = ck + dk
                                f[(q,) + tuple(idx)] += 0.25 * t * h * h
    perm = np.broadcast_to(np.asarray(per, dtype=bool), (3, 3))
    for q in range(3):
        for i in range(3):
            if perm[q, i]:
                s0 = [q, slice(None), slice(None), slice(None)]; s0[i + 1] = 0
                sn = [q, slice(None), slice(None), slice(None)]; sn[i + 1] = -1
                f[tuple(s0)] += f[tuple(sn)]
                f[tuple(sn)] = f[tuple(s0)]
    return f


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("seed", range(4))
def test_applied_traction_equals_fe_face_load(scheme, seed):
    """Non-vanishing Neumann conditions (Sec. 2.2): div_d sigma + D*, with P*
    on the mirror voxels of the loaded faces, equals the FE residual of the
    internal forces minus the consistent nodal forces of the face tractions
    (times 2 per symmetric face), at every kept node."""
    from oracle.laws import cubic_tensor, quat_to_rot, rotate4
    rng = np.random.default_rng(1100 + seed)
    n = (3, 4, 3)
    h = 1.1
    ext3 = [[PAIRS[int(rng.integers(0, 5))] for i in range(3)] for q in range(3)]
    if seed == 0:        # the cantilever: clamped x = 0, every other face free
        ext3 = [[("A", "S"), ("S", "S"), ("S", "S")]] * 3
    T = np.zeros((3, 2, 3))
    for q in range(3):
        for i in range(3):
            for a in range(2):
                if ext3[q][i][a] == "S":
                    T[i, a, q] = rng.uniform(-1.0, 1.0)
    assert np.count_nonzero(T) > 0
    u = rng.standard_normal((3,) + tuple(v + 1 for v in n))
    for q in range(3):
        fd.zero_dismissed(u[q], ext3[q])
    C0 = cubic_tensor(1.68, 1.21, 0.75)
    Cvox = np.empty(n + (3, 3, 3, 3))
    for idx in itertools.product(*[range(v) for v in n]):
        Cvox[idx] = rotate4(C0 * rng.uniform(0.5, 2.0), quat_to_rot(rng.standard_normal(4)))
    g = fd.gradient(u, scheme, h)
    eps = 0.5 * (g + np.swapaxes(g, -1, -2))
    sig = np.einsum("xyzijkl,rxyzkl->rxyzij", Cvox, eps)
    D = fd.divergence(sig, ext3, scheme, h) + fd.applied_divergence(T, ext3, scheme, h, n)
    per = [[ext3[q][i][0] == "P" for i in range(3)] for q in range(3)]
    f = _fe_force(u, Cvox, n, h, scheme, per) - _fe_face_load(T, n, h, per)
    for q in range(3):
        keep = fd.kept_mask(ext3[q], n)
        np.testing.assert_allclose(D[q][keep], (-f[q] / h ** 3 * _face_weight(ext3[q], n))[keep], atol=1e-12)


@pytest.mark.parametrize("finite", [False, True])
@pytest.mark.parametrize("scheme", [0, 1])
def test_c0_green_inverts_L0(scheme, finite):
    """P5 for the C0 operator (Sec. 2.6.1, Appendix A): on the virtually
    extended fields its Green operator inverts div_d(C0 : grad^s_d u) (small
    strain; div_d(C0 : grad_d u) for finite strain), the
    real-space operator with the mirror rules, off the null modes, for every
    normal-mixed condition pattern (5 pairs per axis for the normal component,
    the opposite pair for the tangential ones: the 125 cases of Eq. SGO_BCs)."""
    import workloads as W
    from oracle.solver import Plan
    rng = np.random.default_rng(60 + scheme)
    n = (4, 5, 3)
    worst = 0.0
    for choice in itertools.product(range(5), repeat=3):
        prob = W.random_small_problem(rng, n=n, scheme=scheme, bc=W.normal_mixed_bc(choice))
        prob.green = W.GREEN_C0
        prob.finite_strain = int(finite)
        prob.lambda0, prob.mu0 = rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0)
        pl = Plan(prob)
        x = rng.standard_normal((3,) + tuple(v + 1 for v in n))
        for q in range(3):
            fd.zero_dismissed(x[q], pl.exts[q])
        u = pl.green_apply(x)               # no null-mode content by construction
        back = pl.green_apply(pl.L0(u))
        worst = max(worst, float(np.abs(back - u).max() / np.abs(u).max()))
    assert worst < 1e-11, worst


def test_c0_rejects_non_normal_mixed():
    import workloads as W
    from oracle.solver import Plan
    rng = np.random.default_rng(1)
    bc = W.normal_mixed_bc((1, 0, 2))
    bc[1, 0] = [W.N, W.N]                   # tangential u_y on the x faces made Neumann like u_x
    prob = W.random_small_problem(rng, n=(4, 4, 4), bc=bc)
    prob.green = W.GREEN_C0
    with pytest.raises(ValueError):
        Plan(prob)
    # a bending pattern (every component Dirichlet on the x faces) is not normal-mixed either
    bc = np.full((3, 3, 2), W.N, dtype=np.int32)
    bc[:, 0, :] = W.D
    prob = W.random_small_problem(rng, n=(4, 4, 4), bc=bc)
    prob.green = W.GREEN_C0
    with pytest.raises(ValueError):
        Plan(prob)


def _fe_force_of_field(S, n, h, scheme, per):
    """FE nodal force f_a,q = sum_e w_e sum_l B_a,l S_lq of a given per-point
    tensor field S[r, x, y, z, l, q] (not necessarily symmetric)."""
    N = tuple(v + 1 for v in n)
    f = np.zeros((3,) + N)
    corners = list(itertools.product((0, 1), repeat=3))
    if scheme == 0:
        sets = [(0, corners, np.array([[(2 * a[i] - 1) / (4.0 * h) for i in range(3)] for a in corners]), 1.0)]
    else:
        even = [c for c in corners if sum(c) % 2 == 0]
        odd = [c for c in corners if sum(c) % 2 == 1]
        sets = [(r, tet, _tet_grads(np.array(tet, dtype=float) * h), 0.5) for r, tet in enumerate((even, odd))]
    for j1, j2, j3 in itertools.product(range(n[0]), range(n[1]), range(n[2])):
        for r, nodes, B, wt in sets:
            Sv = S[r, j1, j2, j3]
            for a, b in zip(nodes, B):
                f[:, j1 + a[0], j2 + a[1], j3 + a[2]] += wt * h ** 3 * (Sv.T @ b)
    perm = np.broadcast_to(np.asarray(per, dtype=bool), (3, 3))
    for q in range(3):
        for i in range(3):
            if perm[q, i]:
                s0 = [q, slice(None), slice(None), slice(None)]; s0[i + 1] = 0
                sn = [q, slice(None), slice(None), slice(None)]; sn[i + 1] = -1
                f[tuple(s0)] += f[tuple(sn)]
                f[tuple(sn)] = f[tuple(s0)]
    return f


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("seed", range(3))
def test_divergence_of_nonsymmetric_field_equals_fe_assembly(scheme, seed):
    """P6 for the finite-strain divergence: a random non-symmetric per-point
    field (first Piola-Kirchhoff stresses are not symmetric), every Table 1
    pair per component and axis; the column-wise mirror rules make the
    divergence equal the FE nodal force (times 2 per symmetric face)."""
    rng = np.random.default_rng(1300 + seed)
    n = (3, 4, 3)
    h = 0.8
    ext3 = [[PAIRS[int(rng.integers(0, 5))] for i in range(3)] for q in range(3)]
    S = rng.standard_normal((fd.n_ppv(scheme),) + n + (3, 3))
    D = fd.divergence(S, ext3, scheme, h)
    per = [[ext3[q][i][0] == "P" for i in range(3)] for q in range(3)]
    f = _fe_force_of_field(S, n, h, scheme, per)
    for q in range(3):
        keep = fd.kept_mask(ext3[q], n)
        np.testing.assert_allclose(D[q][keep], (-f[q] / h ** 3 * _face_weight(ext3[q], n))[keep], atol=1e-12)
