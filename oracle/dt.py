"""Discrete transforms of Table 1 (Sec. 2.4, Tab. BCsSymmetriesDTTDFT).

A node field along one axis has values g[j], j = 0..n (n voxels, n+1 nodes).
The pair of extensions at the two ends picks the transform:

    P/P  DFT      kept j = 0..n-1          xi_k = 2 pi k / n        k = 0..n-1
    S/S  DCT-I    kept j = 0..n            xi_k = pi k / n          k = 0..n
    A/A  DST-I    kept j = 1..n-1          xi_k = pi (k+1) / n      k = 0..n-2
    S/A  DCT-III  kept j = 0..n-1          xi_k = pi (k+1/2) / n    k = 0..n-1
    A/S  DST-III  kept j = 1..n            xi_k = pi (k+1/2) / n    k = 0..n-1

``brute_matrix`` writes the sums of Table 1 out literally (O(n^2));
``forward_1d`` / ``inverse_1d`` evaluate the same transforms with scipy.fft
(the unnormalised DCT/DST types 1 and 3 are exactly Table 1's sums; the
inverses are DCT-I/(2n), DST-I/(2n), DCT-II/(2n), DST-II/(2n), IDFT).
``extension`` builds the virtually extended periodic field E of Table 1 and
``ext_dft_index`` / ``alpha`` give the link DFT(E)[mapped k] = alpha DT(G)[k].
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

DFT, DCT1, DST1, DCT3, DST3 = 0, 1, 2, 3, 4
NAMES = {DFT: "DFT", DCT1: "DCT-I", DST1: "DST-I", DCT3: "DCT-III", DST3: "DST-III"}

# extension codes of the fluctuation displacement at one face
EXT_P, EXT_A, EXT_S = "P", "A", "S"


def ext_of_bc(code: int) -> str:
    """Periodic -> P, Dirichlet -> anti-symmetric, Neumann -> symmetric
    (Sec. 2.2, Eq. GeneralBCtobesolved)."""
    return {0: EXT_P, 1: EXT_A, 2: EXT_S}[int(code)]


def pair_kind(left: str, right: str) -> int:
    if left == EXT_P or right == EXT_P:
        if not (left == EXT_P and right == EXT_P):
            raise ValueError("periodicity must hold on both opposite faces")
        return DFT
    return {("S", "S"): DCT1, ("A", "A"): DST1, ("S", "A"): DCT3, ("A", "S"): DST3}[(left, right)]


def kind_of_bc(bc_left: int, bc_right: int) -> int:
    return pair_kind(ext_of_bc(bc_left), ext_of_bc(bc_right))


def kept_nodes(kind: int, n: int) -> np.ndarray:
    return {DFT: np.arange(0, n), DCT1: np.arange(0, n + 1), DST1: np.arange(1, n),
            DCT3: np.arange(0, n), DST3: np.arange(1, n + 1)}[kind]


def n_freq(kind: int, n: int) -> int:
    return {DFT: n, DCT1: n + 1, DST1: n - 1, DCT3: n, DST3: n}[kind]


def freqs(kind: int, n: int) -> np.ndarray:
    k = np.arange(n_freq(kind, n), dtype=np.float64)
    if kind == DFT:
        return 2.0 * np.pi * k / n
    if kind == DCT1:
        return np.pi * k / n
    if kind == DST1:
        return np.pi * (k + 1.0) / n
    return np.pi * (k + 0.5) / n


def symmetry_factor(kind: int) -> int:
    return {DFT: 1, DCT1: 2, DST1: 2, DCT3: 4, DST3: 4}[kind]


def alpha(kind: int) -> complex:
    return {DFT: 1.0, DCT1: 1.0, DST1: -1j, DCT3: 2.0, DST3: -2j}[kind]


def ext_dft_index(kind: int, k: np.ndarray) -> np.ndarray:
    """Index of the extended field's DFT that carries DT(G)[k] (Tab. 1, col. 3)."""
    k = np.asarray(k)
    return {DFT: k, DCT1: k, DST1: k + 1, DCT3: 2 * k + 1, DST3: 2 * k + 1}[kind]


def end_extensions(kind: int):
    return {DFT: (EXT_P, EXT_P), DCT1: (EXT_S, EXT_S), DST1: (EXT_A, EXT_A),
            DCT3: (EXT_S, EXT_A), DST3: (EXT_A, EXT_S)}[kind]


def extension(g: np.ndarray, kind: int) -> np.ndarray:
    """Virtually extended periodic field E built from the n+1 node values g
    (Fig. Symmetries): reflect about node 0 / node n with the sign of the
    extension; the period is S_f * n."""
    n = len(g) - 1
    if kind == DFT:
        return g[:n].astype(np.complex128)
    sf = symmetry_factor(kind)
    L = sf * n
    left, right = end_extensions(kind)
    sl = 1.0 if left == EXT_S else -1.0
    sr = 1.0 if right == EXT_S else -1.0
    e = np.zeros(L, dtype=np.complex128)
    # fill by repeated reflection: value at integer position x in [0, L)
    for x in range(L):
        # unfold x into [0, n] with accumulated sign
        sign = 1.0
        y = x
        # reduce modulo the full period first
        y %= L
        # map into [-n, ... ] via reflections about 0 and n
        # walk: positions beyond n reflect about n, negative reflect about 0
        while y > n or y < 0:
            if y > n:
                y = 2 * n - y
                sign *= sr
            else:
                y = -y
                sign *= sl
        val = g[y]
        # anti-symmetric ends force the node value on that face to zero
        if (y == 0 and left == EXT_A) or (y == n and right == EXT_A):
            val = 0.0
        e[x] = sign * val
    return e


def brute_matrix(kind: int, n: int) -> np.ndarray:
    """Matrix M (n_freq x (n+1)) with DT(G) = M @ g, the sums of Table 1."""
    m = n_freq(kind, n)
    xi = freqs(kind, n)
    M = np.zeros((m, n + 1), dtype=np.complex128)
    j = np.arange(n + 1, dtype=np.float64)
    for k in range(m):
        if kind == DFT:
            w = np.exp(-1j * xi[k] * j)
            w[n] = 0.0
        elif kind == DCT1:
            wt = 2.0 - (j == 0) - (j == n)
            w = wt * np.cos(xi[k] * j)
        elif kind == DST1:
            w = 2.0 * np.sin(xi[k] * j)
            w[0] = 0.0
            w[n] = 0.0
        elif kind == DCT3:
            wt = 2.0 - (j == 0)
            w = wt * np.cos(xi[k] * j)
            w[n] = 0.0
        else:  # DST3
            wt = 2.0 - (j == n)
            w = wt * np.sin(xi[k] * j)
            w[0] = 0.0
        M[k] = w
    return M


def forward_1d(g: np.ndarray, kind: int, axis: int) -> np.ndarray:
    """Transform the node values along ``axis`` (length n+1) to the spectral
    coefficients of Table 1 (length n_freq).  Works on real or complex data."""
    g = np.moveaxis(np.asarray(g), axis, -1)
    n = g.shape[-1] - 1
    if kind == DFT:
        out = np.fft.fft(g[..., :n], axis=-1)
    elif kind == DCT1:
        out = sfft.dct(g, type=1, axis=-1)
    elif kind == DST1:
        out = sfft.dst(g[..., 1:n], type=1, axis=-1)
    elif kind == DCT3:
        out = sfft.dct(g[..., :n], type=3, axis=-1)
    else:
        out = sfft.dst(g[..., 1:], type=3, axis=-1)
    return np.moveaxis(out, -1, axis)


def inverse_1d(G: np.ndarray, kind: int, axis: int, n: int) -> np.ndarray:
    """Inverse of ``forward_1d``; returns all n+1 node values with the
    dismissed points filled (anti-symmetric face nodes = 0, periodic node n =
    node 0) as in Sec. 2.7.2 (Domain decomposition and discrete transformations)."""
    G = np.moveaxis(np.asarray(G), axis, -1)
    shape = G.shape[:-1] + (n + 1,)
    dtype = np.result_type(G.dtype, np.float64)
    out = np.zeros(shape, dtype=dtype)
    if kind == DFT:
        v = np.fft.ifft(G, axis=-1)
        if not np.iscomplexobj(G):
            v = v.real
        out = out.astype(v.dtype)
        out[..., :n] = v
        out[..., n] = v[..., 0]
    elif kind == DCT1:
        out[...] = sfft.idct(G, type=1, axis=-1)
    elif kind == DST1:
        out[..., 1:n] = sfft.idst(G, type=1, axis=-1)
    elif kind == DCT3:
        out[..., :n] = sfft.idct(G, type=3, axis=-1)
    else:
        out[..., 1:] = sfft.idst(G, type=3, axis=-1)
    return np.moveaxis(out, -1, axis)


def forward_3d(g: np.ndarray, kinds) -> np.ndarray:
    """3D transform of a node field indexed [j1, j2, j3] (axis i <-> e_{i+1})."""
    out = g
    for ax in range(3):
        out = forward_1d(out, kinds[ax], ax)
    return out


def inverse_3d(G: np.ndarray, kinds, n) -> np.ndarray:
    out = G
    for ax in (2, 1, 0):
        out = inverse_1d(out, kinds[ax], ax, n[ax])
    if np.iscomplexobj(out):
        out = out.real
    return out
