"""Modified frequencies and the B0 / 2mu0 discrete Green operators (Sec. 2.6).

For component q the frequencies along axis i are those of the transform its
extension selects (Tab. 1).  With s_i = sin(xi_i / 2), c_i = cos(xi_i / 2):

HEX1 (Eq. modified_freq_hex1):
    xi_H = (2/h) (s1 c2 c3, c1 s2 c3, c1 c2 s3)
TETRA2 (Eq. freq_TETRA2), xi_T2 = conj(xi_T1):
    xi_T1 = (2/h) [(s1 c2 c3, c1 s2 c3, c1 c2 s3) - i (c1 s2 s3, s1 c2 s3, s1 s2 c3)]

B0 operator (Eqs. NSGO2_HEX1, NSGO2_TETRA2), no sum on q:
    u_q = - p_q / (2 mu0 |xi|^2 + lambda0 |xi_q|^2)
2mu0 operator (Eqs. NSGO1_HEX1, NSGO1_TETRA2): the same with lambda0 = 0.
Where the denominator is null the result is set to 0 (end of Sec. 2.6.3).
Nullity is decided in index space (cos(pi/2) is not 0 in floating point):
an axis is at xi = 0 for (DFT or DCT-I, k = 0) and at xi = pi for
(DFT, k = n/2 with n even) or (DCT-I, k = n); HEX1 vanishes when all three
axes are at 0 or at least two are at pi, TETRA2 when all three are at 0 or
all three at pi.
"""
from __future__ import annotations

import numpy as np

from . import dt as _dt


def axis_tables(kind: int, n: int):
    xi = _dt.freqs(kind, n)
    s = np.sin(0.5 * xi)
    c = np.cos(0.5 * xi)
    k = np.arange(len(xi))
    at0 = np.zeros(len(xi), dtype=bool)
    atpi = np.zeros(len(xi), dtype=bool)
    if kind in (_dt.DFT, _dt.DCT1):
        at0[0] = True
    if kind == _dt.DFT and n % 2 == 0:
        atpi[n // 2] = True
    if kind == _dt.DCT1:
        atpi[n] = True
    # exact values where the index says so
    s[at0] = 0.0; c[at0] = 1.0
    s[atpi] = 1.0; c[atpi] = 0.0
    return s, c, at0, atpi


def _grid(arrs):
    a, b, c = arrs
    return a[:, None, None], b[None, :, None], c[None, None, :]


def xi_components(kinds, n, scheme: int, h: float):
    """Return (|xi|^2, [|xi_i|^2 for i]) as 3D arrays over the spectral grid."""
    tabs = [axis_tables(kinds[i], n[i]) for i in range(3)]
    s1, s2, s3 = _grid([t[0] for t in tabs])
    c1, c2, c3 = _grid([t[1] for t in tabs])
    f = (2.0 / h) ** 2
    real = [s1 * c2 * c3, c1 * s2 * c3, c1 * c2 * s3]
    if scheme == 0:
        comp = [f * r ** 2 for r in real]
    else:
        imag = [c1 * s2 * s3, s1 * c2 * s3, s1 * s2 * c3]
        comp = [f * (r ** 2 + m ** 2) for r, m in zip(real, imag)]
    comp = [np.broadcast_to(x, (len(tabs[0][0]), len(tabs[1][0]), len(tabs[2][0]))) for x in comp]
    return comp[0] + comp[1] + comp[2], comp


def null_mask(kinds, n, scheme: int) -> np.ndarray:
    tabs = [axis_tables(kinds[i], n[i]) for i in range(3)]
    z1, z2, z3 = _grid([t[2] for t in tabs])
    p1, p2, p3 = _grid([t[3] for t in tabs])
    allz = z1 & z2 & z3
    npi = p1.astype(int) + p2.astype(int) + p3.astype(int)
    if scheme == 0:
        m = allz | (npi >= 2)
    else:
        m = allz | (npi == 3)
    shape = tuple(len(t[0]) for t in tabs)
    return np.broadcast_to(m, shape)


def denominator(kinds, n, q: int, scheme: int, h: float, lam0: float, mu0: float,
                green: int) -> np.ndarray:
    tot, comp = xi_components(kinds, n, scheme, h)
    lam = lam0 if green == 0 else 0.0
    return 2.0 * mu0 * tot + lam * comp[q]


def apply(p_hat: np.ndarray, kinds, n, q, scheme, h, lam0, mu0, green) -> np.ndarray:
    den = denominator(kinds, n, q, scheme, h, lam0, mu0, green)
    mask = null_mask(kinds, n, scheme)
    out = np.zeros_like(p_hat)
    ok = ~mask
    out[ok] = -p_hat[ok] / den[ok]
    return out


# ---------------------------------------------------------------------------
# C0 discrete Green operator (Sec. 2.6.1, small-strain form of Appendix A)
# ---------------------------------------------------------------------------
OPPOSITE = {_dt.DFT: _dt.DFT, _dt.DCT1: _dt.DST1, _dt.DST1: _dt.DCT1,
            _dt.DCT3: _dt.DST3, _dt.DST3: _dt.DCT3}


def c0_compatible(kinds) -> bool:
    """Eq. SGO_BCs ("normal-mixed" conditions): along every axis a, the
    extension of the normal component u_a is the opposite of that of the two
    tangential components (periodic stays periodic), so that p and u^f share
    one extension.  ``kinds[q][a]`` is the Table 1 transform of u_q along a."""
    for a in range(3):
        for q in range(3):
            if q != a and kinds[q][a] != OPPOSITE[kinds[a][a]]:
                return False
    return True


def _extension_map(kind: int, n: int):
    """Index into the n+1 node values and sign of every position of the
    virtually extended periodic field (Table 1, Fig. Symmetries); sign 0 where
    the extension is forced to zero."""
    probe = np.arange(1, n + 2, dtype=np.float64)
    e = _dt.extension(probe, kind).real
    idx = np.where(e == 0, 0, np.abs(e).astype(np.int64) - 1)
    return idx, np.sign(e)


def _extend3(g, kinds, n):
    maps = [_extension_map(kinds[a], n[a]) for a in range(3)]
    E = g[np.ix_(maps[0][0], maps[1][0], maps[2][0])]
    return E * maps[0][1][:, None, None] * maps[1][1][None, :, None] * maps[2][1][None, None, :]


def c0_apply(p, kinds, n, scheme: int, h: float, lam0: float, mu0: float, finite: bool = False) -> np.ndarray:
    """u^f = DGO(p) of the C0 reference medium on
    the virtually extended periodic fields: every component of p (node
    field, shape (3, n1+1, n2+1, n3+1)) is extended with its own symmetries
    (identical periods along each axis under Eq. SGO_BCs), transformed by a
    plain 3D DFT, mapped to u^f by the formulas of Appendix A with the
    modified frequencies of the scheme (HEX1: Eq. modified_freq_hex1; TETRA2:
    xi_T2 of Eq. freq_TETRA2), transformed back and restricted to the nodes.
    Small strain (C0 on the symmetric gradient): the formulas of Appendix A;
    finite strain (C0 on the gradient): Eqs. FourierSGO_HEX1 and
    FourierSGO_TETRA2_1/_2, i.e. the same with mu0 -> 2 mu0 in the leading
    factor and mu0 + lambda0 -> lambda0 in the coupling.  Null modes (|xi| =
    0, decided in index space) give 0."""
    if not c0_compatible(kinds):
        raise ValueError("the C0 operator needs normal-mixed boundary conditions (Eq. SGO_BCs)")
    Ps = [np.fft.fftn(_extend3(p[q], kinds[q], n)) for q in range(3)]
    shape = Ps[0].shape
    xs, at0, atpi = [], [], []
    for a in range(3):
        L = shape[a]
        m = np.arange(L)
        xs.append(2.0 * np.pi * m / L)
        at0.append(m == 0)
        atpi.append((m == L // 2) if L % 2 == 0 else np.zeros(L, dtype=bool))
    g = [np.meshgrid(*[v for v in arrs], indexing="ij") for arrs in (xs,)][0]
    s = [np.sin(0.5 * x) for x in g]
    c = [np.cos(0.5 * x) for x in g]
    z = np.meshgrid(*at0, indexing="ij")
    pi = np.meshgrid(*atpi, indexing="ij")
    for a in range(3):                      # exact values where the index says so
        s[a] = np.where(z[a], 0.0, np.where(pi[a], 1.0, s[a]))
        c[a] = np.where(z[a], 1.0, np.where(pi[a], 0.0, c[a]))
    f = 2.0 / h
    re = [f * s[0] * c[1] * c[2], f * c[0] * s[1] * c[2], f * c[0] * c[1] * s[2]]
    allz = z[0] & z[1] & z[2]
    npi = pi[0].astype(int) + pi[1].astype(int) + pi[2].astype(int)
    U = [np.zeros(shape, dtype=np.complex128) for _ in range(3)]
    if scheme == 0:
        null = allz | (npi >= 2)
        ok = ~null
        xi2 = re[0] ** 2 + re[1] ** 2 + re[2] ** 2
        pd = Ps[0] * re[0] + Ps[1] * re[1] + Ps[2] * re[2]
        lead = 2.0 * mu0 if finite else mu0
        k = (lam0 if finite else mu0 + lam0) / (2.0 * mu0 + lam0)
        for q in range(3):
            U[q][ok] = -(Ps[q][ok] - k * pd[ok] * re[q][ok] / xi2[ok]) / (lead * xi2[ok])
    else:
        null = allz | (npi == 3)
        ok = ~null
        im = [f * c[0] * s[1] * s[2], f * s[0] * c[1] * s[2], f * s[0] * s[1] * c[2]]
        xi = [re[a] + 1j * im[a] for a in range(3)]           # xi_T2 = conj(xi_T1)
        xib = [np.conj(v) for v in xi]
        xi2 = sum(np.abs(v) ** 2 for v in xi)
        zz = xi[0] ** 2 + xi[1] ** 2 + xi[2] ** 2             # xi . xi
        zzb = np.conj(zz)
        lead = 2.0 * mu0 if finite else mu0
        cb = 0.5 * (lam0 if finite else mu0 + lam0)
        ca = (lead + cb) * xi2
        Ds = ca ** 2 - (cb * np.abs(zz)) ** 2
        px = Ps[0] * xi[0] + Ps[1] * xi[1] + Ps[2] * xi[2]    # p . xi
        pxb = Ps[0] * xib[0] + Ps[1] * xib[1] + Ps[2] * xib[2]
        with np.errstate(divide="ignore", invalid="ignore"):
            p1 = (-ca * px + cb * zz * pxb) / Ds
            p2 = (cb * zzb * px - ca * pxb) / Ds
        for q in range(3):
            U[q][ok] = -(Ps[q][ok] + cb * (p1[ok] * xib[q][ok] + p2[ok] * xi[q][ok])) / (lead * xi2[ok])
    out = np.zeros_like(p)
    for q in range(3):
        e = np.fft.ifftn(U[q]).real
        sl = tuple(slice(0, min(n[a] + 1, shape[a])) for a in range(3))
        r = e[sl]
        full = np.zeros(tuple(v + 1 for v in n))
        full[:r.shape[0], :r.shape[1], :r.shape[2]] = r
        out[q] = full
    return out
