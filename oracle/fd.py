"""HEX1 and TETRA2 finite-difference derivatives (Sec. 2.5).

Arrays are indexed [j1, j2, j3] (x, y, z).  A node field has shape
(n1+1, n2+1, n3+1); a voxel field (one value per voxel centre) has shape
(n1, n2, n3).

``cell_derivs`` evaluates the stencils of Eqs. D1HG-D3HG (HEX1) and
D1T1T2G-D3T1T2G (TETRA2) on a field F of shape (N1, N2, N3), giving values at
the (N1-1, N2-1, N3-1) cell centres.  By Remark 1 the same stencils map a
voxel field padded with one ghost voxel per side to the nodes, so gradient
(node -> voxel) and divergence (voxel -> node) share this one function.

``pad_voxel_pair`` fills the ghost voxels from the extension of the equation
component q along each axis (Eq. Continuous_der_symmetry_per applied to the
columns of the stress, Eq. GeneralBCtobesolved): periodic faces wrap; at a
mirror face the value is +/- the inner voxel, with + iff (u_q symmetric and
l != i) or (u_q anti-symmetric and l == i), and for TETRA2 the mirror swaps the
two tetrahedra (Sec. 2.5.2, reflection maps T1 onto T2).
"""
from __future__ import annotations

import numpy as np

from . import dt as _dt


def _corner(F, a, b, c):
    n1, n2, n3 = F.shape
    return F[a:n1 - 1 + a, b:n2 - 1 + b, c:n3 - 1 + c]


def cell_derivs(F: np.ndarray, scheme: int, h: float):
    """Return derivatives at cell centres.

    HEX1  -> array (3, N1-1, N2-1, N3-1): D_i^H F for i = 1, 2, 3.
    TETRA2-> array (2, 3, ...): [r][i] = D_i^{T_{r+1}} F.
    """
    c = {(a, b, cc): _corner(F, a, b, cc) for a in (0, 1) for b in (0, 1) for cc in (0, 1)}
    if scheme == 0:
        d1 = (c[1, 0, 0] - c[0, 0, 0] + c[1, 1, 0] - c[0, 1, 0]
              + c[1, 0, 1] - c[0, 0, 1] + c[1, 1, 1] - c[0, 1, 1]) / (4.0 * h)
        d2 = (c[0, 1, 0] - c[0, 0, 0] + c[1, 1, 0] - c[1, 0, 0]
              + c[0, 1, 1] - c[0, 0, 1] + c[1, 1, 1] - c[1, 0, 1]) / (4.0 * h)
        d3 = (c[0, 0, 1] - c[0, 0, 0] + c[1, 0, 1] - c[1, 0, 0]
              + c[0, 1, 1] - c[0, 1, 0] + c[1, 1, 1] - c[1, 1, 0]) / (4.0 * h)
        return np.stack([d1, d2, d3])
    t1 = np.stack([
        (c[1, 1, 0] - c[0, 1, 1] + c[1, 0, 1] - c[0, 0, 0]) / (2.0 * h),
        (c[1, 1, 0] - c[0, 0, 0] + c[0, 1, 1] - c[1, 0, 1]) / (2.0 * h),
        (c[0, 1, 1] - c[0, 0, 0] + c[1, 0, 1] - c[1, 1, 0]) / (2.0 * h),
    ])
    t2 = np.stack([
        (c[1, 0, 0] - c[0, 0, 1] + c[1, 1, 1] - c[0, 1, 0]) / (2.0 * h),
        (c[0, 1, 0] - c[1, 0, 0] + c[1, 1, 1] - c[0, 0, 1]) / (2.0 * h),
        (c[0, 0, 1] - c[0, 1, 0] + c[1, 1, 1] - c[1, 0, 0]) / (2.0 * h),
    ])
    return np.stack([t1, t2])


def n_ppv(scheme: int) -> int:
    return 1 if scheme == 0 else 2


def gradient(u: np.ndarray, scheme: int, h: float) -> np.ndarray:
    """Gradient of a node vector field u[q] at the integration points.

    Returns grad[r, ..., l, q] = D_l u_q at ip r (r = 0 for HEX1; r = 0, 1 for
    the T1 / T2 points of TETRA2), shape (n_ppv, n1, n2, n3, 3, 3).
    """
    outs = []
    for q in range(3):
        d = cell_derivs(u[q], scheme, h)
        if scheme == 0:
            d = d[None]
        outs.append(d)               # (n_ppv, 3[l], n1, n2, n3)
    g = np.stack(outs, axis=2)       # (n_ppv, 3[l], 3[q], n1, n2, n3)
    return np.moveaxis(np.moveaxis(g, 1, -1), 1, -1)   # (n_ppv, n1, n2, n3, l, q)


def mirror_sign(ext: str, l: int, i: int) -> float:
    if ext == _dt.EXT_S:
        return 1.0 if l != i else -1.0
    return 1.0 if l == i else -1.0


def pad_voxel_pair(A: np.ndarray, B, exts, l: int):
    """Pad voxel fields with one ghost voxel per side along each axis.

    A (and B for TETRA2: A = T1 values, B = T2 values) hold the column entry
    S_lq of a voxel tensor field; ``exts[i] = (left, right)`` are the
    extensions of the displacement component q along axis i.
    """
    for i in range(3):
        left, right = exts[i]
        n = A.shape[i]

        def take(X, idx):
            return np.take(X, [idx], axis=i)

        if left == _dt.EXT_P:
            gA_l, gA_r = take(A, n - 1), take(A, 0)
            gB_l, gB_r = (take(B, n - 1), take(B, 0)) if B is not None else (None, None)
        else:
            sl = mirror_sign(left, l, i)
            sr = mirror_sign(right, l, i)
            if B is None:
                gA_l, gA_r = sl * take(A, 0), sr * take(A, n - 1)
                gB_l = gB_r = None
            else:
                gA_l, gA_r = sl * take(B, 0), sr * take(B, n - 1)
                gB_l, gB_r = sl * take(A, 0), sr * take(A, n - 1)
        A2 = np.concatenate([gA_l, A, gA_r], axis=i)
        B2 = np.concatenate([gB_l, B, gB_r], axis=i) if B is not None else None
        A, B = A2, B2
    return A, B


def divergence(S: np.ndarray, ext3, scheme: int, h: float) -> np.ndarray:
    """Divergence at the nodes of a voxel tensor field S[r, j1, j2, j3, l, q]
    (derivative contracted with the first index: (div S)_q = sum_l D_l S_lq).

    ``ext3[q][i] = (left, right)`` extension of u_q along axis i.
    HEX1: D_q = sum_l D_l^H S_lq.
    TETRA2: D_q = 1/2 sum_l (D_l^{T2} S^{T1}_lq + D_l^{T1} S^{T2}_lq), the
    crossed combination of the TETRA2 Laplacian (Eq. laplacian_tetra2).
    Returns (3, n1+1, n2+1, n3+1); dismissed (anti-symmetric face) nodes are 0.
    """
    n1, n2, n3 = S.shape[1:4]
    out = np.zeros((3, n1 + 1, n2 + 1, n3 + 1))
    for q in range(3):
        acc = np.zeros((n1 + 1, n2 + 1, n3 + 1))
        for l in range(3):
            if scheme == 0:
                Ap, _ = pad_voxel_pair(S[0, ..., l, q], None, ext3[q], l)
                acc += cell_derivs(Ap, 0, h)[l]
            else:
                Ap, Bp = pad_voxel_pair(S[0, ..., l, q], S[1, ..., l, q], ext3[q], l)
                dA = cell_derivs(Ap, 1, h)
                dB = cell_derivs(Bp, 1, h)
                acc += 0.5 * (dA[1, l] + dB[0, l])
        out[q] = acc
        zero_dismissed(out[q], ext3[q])
    return out


def zero_dismissed(f: np.ndarray, exts) -> None:
    """Set anti-symmetric face nodes to zero; copy periodic node 0 to node n."""
    for i in range(3):
        left, right = exts[i]
        sl = [slice(None)] * 3
        if left == _dt.EXT_P:
            s0 = list(sl); s0[i] = 0
            sn = list(sl); sn[i] = -1
            f[tuple(sn)] = f[tuple(s0)]
            continue
        if left == _dt.EXT_A:
            s0 = list(sl); s0[i] = 0
            f[tuple(s0)] = 0.0
        if right == _dt.EXT_A:
            sn = list(sl); sn[i] = -1
            f[tuple(sn)] = 0.0


def kept_mask(exts, n) -> np.ndarray:
    """Boolean node mask of the kept nodes of one component (Tab. 1 ranges)."""
    m = np.ones((n[0] + 1, n[1] + 1, n[2] + 1), dtype=bool)
    for i in range(3):
        kind = _dt.pair_kind(*exts[i])
        keep = np.zeros(n[i] + 1, dtype=bool)
        keep[_dt.kept_nodes(kind, n[i])] = True
        shape = [1, 1, 1]; shape[i] = n[i] + 1
        m &= keep.reshape(shape)
    return m


def applied_divergence(T: np.ndarray, ext3, scheme: int, h: float, n) -> np.ndarray:
    """D* = div_d P* of the applied stress of non-vanishing Neumann conditions
    (Sec. 2.2, Fig. NeumannBC): P* vanishes at every voxel of the grid; on the
    mirror voxels across a face S_{i a} where u_q is Neumann, its entry P*_iq
    is twice the face value that the traction prescribes, P_iq (-1)^(a+1) =
    T*_q, so that P* interpolated to the face equals it.  T[i, a, q] is
    uniform over the face, so the whole mirror layer (edges and corners of
    the padded grid included) carries the same value.  The stencils are those
    of the divergence; dismissed nodes are 0."""
    n1, n2, n3 = n
    out = np.zeros((3, n1 + 1, n2 + 1, n3 + 1))
    for q in range(3):
        acc = np.zeros((n1 + 1, n2 + 1, n3 + 1))
        for i in range(3):
            if not np.any(T[i, :, q]):
                continue
            A = np.zeros((n1 + 2, n2 + 2, n3 + 2))
            for a in (0, 1):
                if T[i, a, q] == 0:
                    continue
                if ext3[q][i][a] != _dt.EXT_S:
                    raise ValueError("a traction needs a Neumann condition of that component on that face")
                sl = [slice(None)] * 3
                sl[i] = 0 if a == 0 else -1
                A[tuple(sl)] = 2.0 * (-1.0) ** (a + 1) * T[i, a, q]
            if scheme == 0:
                acc += cell_derivs(A, 0, h)[i]
            else:
                d = cell_derivs(A, 1, h)
                acc += 0.5 * (d[1, i] + d[0, i])
        out[q] = acc
        zero_dismissed(out[q], ext3[q])
    return out
