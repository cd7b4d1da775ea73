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
