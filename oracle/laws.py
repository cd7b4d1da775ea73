"""Constitutive laws of the oracle (small strain), vectorised over points.

* Isotropic elasticity sigma = 2 mu eps + lambda tr(eps) 1 (Sec. 3.1; the
  factor 2 on mu follows the C0 reference medium of Eq. TF_C0_behavior).
* Cubic elasticity (C11, C12, C44) rotated from crystal to sample frame by a
  unit quaternion; the paper's copper moduli (Sec. 3.3).
* J2 plasticity with linear isotropic hardening sy = sy0 + H p, closed-form
  radial return (von Mises yield and normality rule as in Sec. 3.2, small
  strain, with a hardening slope).
* FCC crystal viscoplasticity, small strain: 12 {111}<110> systems (Sec. 3.3),
  power-law rate gdot = gdot0 |tau/tau_c|^n sign(tau), Voce hardening of a
  common CRSS tau_c(Gamma) = tau0 + (taus - tau0)(1 - exp(-theta0 Gamma /
  (taus - tau0))), backward Euler solved by Newton on (sigma, dGamma).

Tensors are full 3x3 arrays in the last two axes; Mandel vectors use the
order (11, 22, 33, 23, 13, 12) with sqrt(2) on the shears.
"""
from __future__ import annotations

import itertools

import numpy as np

LAW_ISO, LAW_ANISO, LAW_J2, LAW_CP, LAW_SVK, LAW_NEOHOOKE = 0, 1, 2, 3, 4, 5
SQ2 = np.sqrt(2.0)
_MANDEL_IJ = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def quat_to_rot(q) -> np.ndarray:
    w, x, y, z = np.asarray(q, dtype=np.float64) / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def cubic_tensor(C11, C12, C44) -> np.ndarray:
    d = np.eye(3)
    C = (C12 * np.einsum("ij,kl->ijkl", d, d)
         + C44 * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))
    for a in range(3):
        C[a, a, a, a] += C11 - C12 - 2.0 * C44
    return C


def rotate4(C, R) -> np.ndarray:
    return np.einsum("ia,jb,kc,ld,abcd->ijkl", R, R, R, R, C)


def iso_tensor(lam, mu) -> np.ndarray:
    d = np.eye(3)
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def to_mandel(T: np.ndarray) -> np.ndarray:
    return np.stack([T[..., 0, 0], T[..., 1, 1], T[..., 2, 2], SQ2 * T[..., 1, 2],
                     SQ2 * T[..., 0, 2], SQ2 * T[..., 0, 1]], axis=-1)


def from_mandel(v: np.ndarray) -> np.ndarray:
    T = np.empty(v.shape[:-1] + (3, 3))
    T[..., 0, 0] = v[..., 0]; T[..., 1, 1] = v[..., 1]; T[..., 2, 2] = v[..., 2]
    T[..., 1, 2] = T[..., 2, 1] = v[..., 3] / SQ2
    T[..., 0, 2] = T[..., 2, 0] = v[..., 4] / SQ2
    T[..., 0, 1] = T[..., 1, 0] = v[..., 5] / SQ2
    return T


def mandel_matrix(C: np.ndarray) -> np.ndarray:
    M = np.empty((6, 6))
    w = [1, 1, 1, SQ2, SQ2, SQ2]
    for a, (i, j) in enumerate(_MANDEL_IJ):
        for b, (k, l) in enumerate(_MANDEL_IJ):
            M[a, b] = w[a] * w[b] * C[i, j, k, l]
    return M


def fcc_slip_systems():
    """12 {111}<110> systems: unit normals n and directions m with m . n = 0."""
    normals = [np.array(v, dtype=np.float64) / np.sqrt(3.0)
               for v in ((1, 1, 1), (-1, 1, 1), (1, -1, 1), (1, 1, -1))]
    dirs = []
    for a, b in itertools.combinations(range(3), 2):
        for sb in (1.0, -1.0):
            v = np.zeros(3); v[a] = 1.0; v[b] = sb
            dirs.append(v / np.sqrt(2.0))
    ms, ns = [], []
    for nrm in normals:
        for d in dirs:
            if abs(np.dot(nrm, d)) < 1e-12:
                ms.append(d); ns.append(nrm)
    assert len(ms) == 12
    return np.array(ms), np.array(ns)


def voce(Gamma, tau0, taus, theta0):
    return tau0 + (taus - tau0) * (1.0 - np.exp(-theta0 * Gamma / (taus - tau0)))


def voce_slope(Gamma, tau0, taus, theta0):
    return theta0 * np.exp(-theta0 * Gamma / (taus - tau0))


def cp_update(eps_M, epn_M, Gn, Cm, Pm, prm, dt, tol=1e-10, max_newton=100):
    """Backward-Euler FCC crystal viscoplasticity for a batch of points.

    eps_M, epn_M: (N, 6) Mandel total strain at t_{n+1} and plastic strain at
    t_n; Gn: (N,) accumulated slip at t_n; Cm: (6, 6) Mandel stiffness; Pm:
    (12, 6) Mandel Schmid tensors sym(m x n).  Unknowns y = (sigma_M, dGamma):

        R_sigma = C^-1 sigma - (eps - ep_n) + dt sum_s gdot_s P_s = 0
        R_Gamma = dGamma - dt sum_s |gdot_s| = 0

    Newton from the elastic predictor with backtracking on the scaled residual
    norm.  Returns sigma_M, ep_M, Gamma at t_{n+1}.
    """
    g0, nexp, tau0, taus, th0 = prm
    Sm = np.linalg.inv(Cm)
    N = eps_M.shape[0]
    ee = eps_M - epn_M
    sig = ee @ Cm.T
    dG = np.zeros(N)
    e_scale = np.maximum(np.abs(ee).max(axis=1), 1e-9)

    def resid(idx, s, d):
        tc = voce(Gn[idx] + d, tau0, taus, th0)
        tau = s @ Pm.T
        r = tau / tc[:, None]
        gd = g0 * np.abs(r) ** nexp * np.sign(r)
        Rs = s @ Sm.T - ee[idx] + dt * gd @ Pm
        Rg = d - dt * np.abs(gd).sum(axis=1)
        nr = np.maximum(np.abs(Rs).max(axis=1), np.abs(Rg)) / e_scale[idx]
        return Rs, Rg, tau, tc, gd, nr

    allidx = np.arange(N)
    Rs, Rg, tau, tc, gd, nr = resid(allidx, sig, dG)
    for _ in range(max_newton):
        act = np.nonzero(nr >= tol)[0]
        if act.size == 0:
            break
        s, d = sig[act], dG[act]
        t, c, g = tau[act], tc[act], gd[act]
        hG = voce_slope(Gn[act] + d, tau0, taus, th0)
        a = nexp * g0 * np.abs(t / c[:, None]) ** (nexp - 1.0) / c[:, None]
        J = np.zeros((act.size, 7, 7))
        J[:, :6, :6] = Sm[None] + dt * np.einsum("ns,si,sj->nij", a, Pm, Pm)
        J[:, :6, 6] = -dt * np.einsum("ns,si->ni", nexp * g / c[:, None] * hG[:, None], Pm)
        J[:, 6, :6] = -dt * np.einsum("ns,si->ni", np.sign(t) * a, Pm)
        J[:, 6, 6] = 1.0 + dt * (nexp * np.abs(g) / c[:, None]).sum(axis=1) * hG
        R = np.concatenate([Rs[act], Rg[act][:, None]], axis=1)
        step = np.linalg.solve(J, R[..., None])[..., 0]
        lam = np.ones(act.size)
        n_old = nr[act]
        for _ls in range(40):
            s_new = s - lam[:, None] * step[:, :6]
            d_new = np.maximum(d - lam * step[:, 6], 0.0)
            out = resid(act, s_new, d_new)
            bad = ~(out[5] < n_old) & (lam > 1e-8)
            if not bad.any():
                break
            lam = np.where(bad, 0.5 * lam, lam)
        sig[act], dG[act] = s_new, d_new
        Rs[act], Rg[act], tau[act], tc[act], gd[act], nr[act] = out
    if np.any(nr >= tol):
        raise RuntimeError("crystal plasticity update did not converge")
    ep = epn_M + dt * gd @ Pm
    return sig, ep, Gn + dG


def j2_update(eps, epn, pn, lam, mu, sy0, H):
    """Radial return for J2 with linear isotropic hardening (full tensors).

    Trial sigma = C:(eps - ep_n); yield f = q_tr - (sy0 + H p_n) with
    q = sqrt(3/2 s:s); if f > 0: dp = f / (3 mu + H), s = s_tr (1 - 3 mu dp /
    q_tr), ep = ep_n + 3/2 dp s_tr / q_tr.
    """
    ee = eps - epn
    tr = np.trace(ee, axis1=-2, axis2=-1)
    sig = 2.0 * mu * ee + lam * tr[..., None, None] * np.eye(3)
    s = sig - (np.trace(sig, axis1=-2, axis2=-1) / 3.0)[..., None, None] * np.eye(3)
    q = np.sqrt(1.5 * np.einsum("...ij,...ij->...", s, s))
    f = q - (sy0 + H * pn)
    plast = f > 0.0
    dp = np.where(plast, f / (3.0 * mu + H), 0.0)
    qs = np.where(plast, q, 1.0)
    fac = np.where(plast, 1.0 - 3.0 * mu * dp / qs, 1.0)
    sig_new = sig - s + fac[..., None, None] * s
    ep = epn + (1.5 * dp / qs)[..., None, None] * s
    return sig_new, ep, pn + dp


# ---------------------------------------------------------------------------
# Finite strain (Lagrangian formulation of Sec. 2.2): F = 1 + grad u,
# E = (F^T F - 1) / 2, second Piola-Kirchhoff Pi = d psi / dE, first P = F Pi.
# ---------------------------------------------------------------------------
def svk_pk1(F, lam, mu):
    """Saint Venant-Kirchhoff (Sec. 3.1.2): Pi = lam tr(E) 1 + 2 mu E (the
    factor 2 on mu as for the small-strain law, reading R6); P = F Pi."""
    E = 0.5 * (np.einsum("...ki,...kj->...ij", F, F) - np.eye(3))
    tr = np.trace(E, axis1=-2, axis2=-1)
    Pi = lam * tr[..., None, None] * np.eye(3) + 2.0 * mu * E
    return F @ Pi


def neohooke_pk1(F, mu, K):
    """Compressible Neo-Hookean of Appendix B, psi = mu/2 (J^-2/3 tr(F F^T) - 3)
    + K/2 (J - 1)^2, differentiated with respect to F:
    P = mu J^-2/3 (F - tr(F F^T)/3 F^-T) + K (J - 1) J F^-T."""
    J = np.linalg.det(F)
    Finv_T = np.swapaxes(np.linalg.inv(F), -1, -2)
    I1 = np.einsum("...ij,...ij->...", F, F)
    return (mu * J[..., None, None] ** (-2.0 / 3.0) * (F - (I1 / 3.0)[..., None, None] * Finv_T)
            + (K * (J - 1.0) * J)[..., None, None] * Finv_T)


class MaterialSet:
    """Per-voxel material table for the oracle.

    ``materials`` is the list of table entries of ``workloads`` (law code plus
    parameters); ``mat_id`` is indexed [j1, j2, j3].
    """

    def __init__(self, materials, mat_id):
        self.materials = materials
        self.mat_id = mat_id
        self.C = []
        self.P = []
        ms, ns = fcc_slip_systems()
        for m in materials:
            law = m["law"]
            if law in (LAW_SVK, LAW_NEOHOOKE):
                self.C.append(None)
                self.P.append(None)
            elif law in (LAW_ISO, LAW_J2):
                self.C.append(iso_tensor(m["lam"], m["mu"]))
                self.P.append(None)
            else:
                R = quat_to_rot(m["quat"])
                self.C.append(rotate4(cubic_tensor(m["C11"], m["C12"], m["C44"]), R))
                if law == LAW_CP:
                    mm = ms @ R.T
                    nn = ns @ R.T
                    Ps = 0.5 * (np.einsum("si,sj->sij", mm, nn) + np.einsum("si,sj->sij", nn, mm))
                    self.P.append(to_mandel(Ps))
                else:
                    self.P.append(None)
        self.masks = [mat_id == k for k in range(len(materials))]

    def pk1(self, F):
        """First Piola-Kirchhoff stress P[..., q, J] of the hyperelastic laws
        for the deformation gradient F[..., q, J] at the points (finite strain)."""
        P = np.zeros_like(F)
        for k, m in enumerate(self.materials):
            mk = self.masks[k]
            if not mk.any():
                continue
            if m["law"] == LAW_SVK:
                P[:, mk] = svk_pk1(F[:, mk], m["lam"], m["mu"])
            elif m["law"] == LAW_NEOHOOKE:
                P[:, mk] = neohooke_pk1(F[:, mk], m["mu"], m["K"])
            else:
                raise ValueError("finite-strain solves take the SVK and Neo-Hookean laws")
        return P

    def has_state(self) -> bool:
        return any(m["law"] in (LAW_J2, LAW_CP) for m in self.materials)

    def init_state(self, nppv, n):
        shp = (nppv,) + tuple(n)
        return {"ep": np.zeros(shp + (3, 3)), "p": np.zeros(shp)}

    def stress(self, eps, state, dt):
        """eps: (n_ppv, n1, n2, n3, 3, 3) symmetric strain at the points.
        Returns sigma (same shape) and the trial state at t_{n+1}."""
        sig = np.zeros_like(eps)
        new = {"ep": state["ep"].copy(), "p": state["p"].copy()}
        for k, m in enumerate(self.materials):
            mk = self.masks[k]
            if not mk.any():
                continue
            e = eps[:, mk]                      # (nppv, cnt, 3, 3)
            law = m["law"]
            if law in (LAW_ISO, LAW_ANISO):
                sig[:, mk] = np.einsum("ijkl,...kl->...ij", self.C[k], e)
            elif law == LAW_J2:
                s, ep, p = j2_update(e, state["ep"][:, mk], state["p"][:, mk],
                                     m["lam"], m["mu"], m["sy0"], m["H"])
                sig[:, mk] = s
                new["ep"][:, mk] = ep
                new["p"][:, mk] = p
            else:
                shp = e.shape[:2]
                eM = to_mandel(e).reshape(-1, 6)
                epM = to_mandel(state["ep"][:, mk]).reshape(-1, 6)
                Gn = state["p"][:, mk].reshape(-1)
                prm = (m["gdot0"], m["n"], m["tau0"], m["taus"], m["theta0"])
                sM, epM2, G2 = cp_update(eM, epM, Gn, mandel_matrix(self.C[k]), self.P[k], prm, dt)
                sig[:, mk] = from_mandel(sM.reshape(shp + (6,)))
                new["ep"][:, mk] = from_mandel(epM2.reshape(shp + (6,)))
                new["p"][:, mk] = G2.reshape(shp)
        return sig, new
