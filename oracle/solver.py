"""Algorithm 1 (algFFT) of the paper, written out step by step in FP64.

For every load increment (the set-up steps of Algorithm 1): update u* and
its discrete gradient, the divergence D* of the applied stress of the
Neumann faces that carry a traction (Sec. 2.2), and predict u^f from the
previous increment; then iterate (the loop of Algorithm 1):

  * strain at the integration points, grad_d u = grad_d u^f + grad_d u*
  * stress from the behaviour law
  * D = div_d P + D*
  * equilibrium error, Eq. equilibrium_condition
  * stop if below the tolerance
  * p = div_d(R0 : grad_d u^f) - D
  * Anderson acceleration on p
  * DTs of the accelerated p, Green operator, inverse DTs -> u^f

Readings where the paper is silent or garbled:
  * error  = h sqrt( sum_kept |D|^2 / sum_ip w_ip |sigma|_F^2 ), w_ip = 1/n_ppv
    (squared L2 norms; the printed ratio of norms is not dimensionless);
  * Anderson (Sec. 2.3 applies it every second or third iteration with a
    history of four pairs, without further detail):
    type-II Anderson on the Green input x with g_m = p_m, f_m = g_m - x_{m-1},
    the last ``aa_depth`` pairs, applied when m >= 2 and m % aa_period == 0,
    weights minimising |sum a_j f_j|^2 with sum a_j = 1 (normal equations,
    ridge 1e-14 trace, skipped if the Cholesky pivots differ by more than a
    factor 1e12 in square), history cleared at every increment; before the
    first iteration x_{-1} = L0(u^f_0) so that u^f_0 = Green(x_{-1});
  * R0 = B0 (or 2 mu0 when lambda0 = 0) acts on the non-symmetric gradient;
  * mixed control (Sec. 3.2, NMBC1 loading): after each iteration the
    stress-controlled Voigt components of sym(G) move by
    C0|_SS^{-1} (Sigma*_S - <sigma>_S) with the isotropic lambda0, mu0;
    an increment also requires max_S |<sigma>_S - Sigma*_S| <= tol |<sigma>|.
"""
from __future__ import annotations

import numpy as np

from . import dt as _dt
from . import fd as _fd
from . import green as _green
from .laws import MaterialSet

VOIGT = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


class Plan:
    def __init__(self, prob):
        self.n = tuple(int(v) for v in prob.n)
        self.h = float(prob.h)
        self.scheme = int(prob.scheme)
        self.nppv = _fd.n_ppv(self.scheme)
        self.lam0 = float(prob.lambda0)
        self.mu0 = float(prob.mu0)
        self.green = int(prob.green)
        self.fs = bool(getattr(prob, "finite_strain", 0))
        bc = np.asarray(prob.bc)
        self.exts = [[(_dt.ext_of_bc(bc[q, i, 0]), _dt.ext_of_bc(bc[q, i, 1])) for i in range(3)]
                     for q in range(3)]
        self.kinds = [[_dt.pair_kind(*self.exts[q][i]) for i in range(3)] for q in range(3)]
        if self.green == 2 and not _green.c0_compatible(self.kinds):
            raise ValueError("the C0 Green operator needs normal-mixed boundary conditions (Eq. SGO_BCs)")
        self.kept = [_fd.kept_mask(self.exts[q], self.n) for q in range(3)]
        n1, n2, n3 = self.n
        j = [np.arange(self.n[i] + 1) * self.h for i in range(3)]
        self.X = np.meshgrid(j[0], j[1], j[2], indexing="ij")

    # -- operators -----------------------------------------------------------
    def ustar(self, c, G, H, nodal=None):
        """u* at the nodes (Algorithm 1 set-up): the quadratic polynomial
        c + G x + x.H.x / 2, plus an optional nodal field (3, N1, N2, N3)."""
        X = self.X
        u = np.zeros((3,) + X[0].shape)
        for q in range(3):
            u[q] = c[q]
            for l in range(3):
                u[q] += G[q, l] * X[l]
                for m in range(3):
                    u[q] += 0.5 * H[q, l, m] * X[l] * X[m]
        if nodal is not None:
            u += np.asarray(nodal, dtype=np.float64)
        return u

    def grad(self, u):
        return _fd.gradient(u, self.scheme, self.h)

    def div(self, S):
        return _fd.divergence(S, self.exts, self.scheme, self.h)

    def div_applied(self, T):
        """D* = div_d P* for the face tractions T[axis, face, component] (0 when none)."""
        T = np.asarray(T, dtype=np.float64)
        if not np.any(T):
            return 0.0
        return _fd.applied_divergence(T, self.exts, self.scheme, self.h, self.n)

    def L0(self, u):
        """div_d(R0 : grad_d u): R0 = B0 (2 mu0 grad u + lambda0 grad u . I) or
        2 mu0 (lambda0 = 0) on the non-symmetric gradient; R0 = C0 on the
        symmetric gradient for the C0 operator (small strain, Sec. 2.6.1)."""
        g = self.grad(u)
        if self.green == 2:
            tr = np.trace(g, axis1=-2, axis2=-1)
            if self.fs:          # finite strain: C0 on the gradient (Eq. TF_C0_behavior)
                tau0 = 2.0 * self.mu0 * g + self.lam0 * tr[..., None, None] * np.eye(3)
            else:                # small strain: C0 on the symmetric gradient (Appendix A)
                tau0 = self.mu0 * (g + np.swapaxes(g, -1, -2)) + self.lam0 * tr[..., None, None] * np.eye(3)
            return self.div(tau0)
        lam = self.lam0 if self.green == 0 else 0.0
        tau0 = g * (2.0 * self.mu0 + lam * np.eye(3))    # factor on entry (l, q)
        return self.div(tau0)

    def green_apply(self, x):
        if self.green == 2:
            u = _green.c0_apply(x, self.kinds, self.n, self.scheme, self.h, self.lam0, self.mu0, finite=self.fs)
            for q in range(3):
                _fd.zero_dismissed(u[q], self.exts[q])
            return u
        u = np.zeros_like(x)
        for q in range(3):
            xh = _dt.forward_3d(x[q], self.kinds[q])
            uh = _green.apply(xh, self.kinds[q], self.n, q, self.scheme, self.h,
                              self.lam0, self.mu0, self.green)
            u[q] = _dt.inverse_3d(uh, self.kinds[q], self.n)
            _fd.zero_dismissed(u[q], self.exts[q])
        return u

    def dot_kept(self, a, b):
        return float(sum(np.sum(a[q][self.kept[q]] * b[q][self.kept[q]]) for q in range(3)))


def equilibrium_error(pl: Plan, D: np.ndarray, sig: np.ndarray) -> float:
    """Eq. equilibrium_condition read with squared L2 norms (the printed ratio
    of norms is not dimensionless): h sqrt(sum over each component's kept
    nodes of D^2 / sum over the integration points of w_ip |sigma|_F^2), with
    w_ip = 1 / n_ppv.  A stress-free body has error 0 if D vanishes, else inf."""
    sD = pl.dot_kept(D, D)
    sS = float(np.sum(sig * sig)) / pl.nppv
    if sS > 0:
        return pl.h * np.sqrt(sD / sS)
    return 0.0 if sD == 0 else np.inf


def anderson_weights(F: np.ndarray):
    k = F.shape[0]
    Fr = F + 1e-14 * np.trace(F) * np.eye(k)
    try:
        L = np.linalg.cholesky(Fr)
    except np.linalg.LinAlgError:
        return None
    d = np.diag(L) ** 2
    if d.min() <= 1e-12 * d.max():
        return None
    y = np.linalg.solve(Fr, np.ones(k))
    return y / y.sum()


def c0_voigt(lam0, mu0):
    C = np.zeros((6, 6))
    C[:3, :3] = lam0
    for a in range(3):
        C[a, a] += 2.0 * mu0
    for a in range(3, 6):
        C[a, a] = 2.0 * mu0
    return C


def solve(prob, callback=None):
    """Run Algorithm 1 on a ``workloads.Problem``.  Returns a dict with the
    outputs in the library layout (x fastest): u (3, n3+1, n2+1, n1+1),
    eps and sig (6, n_ppv, n3, n2, n1) in Voigt order, per-step macroscopic
    stress, iteration counts, convergence flags and the iteration log."""
    pl = Plan(prob)
    n = pl.n
    mats = MaterialSet(prob.materials, np.asarray(prob.mat_id).transpose(2, 1, 0))
    state = mats.init_state(pl.nppv, n)
    uf = np.zeros((3, n[0] + 1, n[1] + 1, n[2] + 1))
    nvox = n[0] * n[1] * n[2]
    log, macro, iters, conv, Gs = [], [], [], [], []
    C0 = c0_voigt(pl.lam0, pl.mu0)
    fs = bool(getattr(prob, "finite_strain", 0))
    for t, step in enumerate(prob.steps):
        G = np.array(step.G, dtype=np.float64).copy()
        if t > 0 and np.any(step.mixed_mask) and len(Gs):
            Gprev = Gs[-1]
            for a in np.nonzero(step.mixed_mask)[0]:
                i, j = VOIGT[a]
                G[i, j] = Gprev[i, j]
                G[j, i] = Gprev[j, i]
        S_idx = np.nonzero(step.mixed_mask)[0]
        Dstar = pl.div_applied(getattr(step, "traction", np.zeros((3, 2, 3))))
        hist = []
        x_prev = pl.L0(uf)
        converged = False
        m = 0
        while True:
            us = pl.ustar(step.c, G, step.H, getattr(step, "ustar_nodal", None))
            gu = pl.grad(uf) + pl.grad(us)            # gu[..., l, q] = D_l u_q
            if fs:
                # Lagrangian finite strain (Sec. 2.2): F[q, J] = delta + D_J u_q,
                # P = F Pi; the divergence contracts the derivative index of
                # S[l, q] = P[q, l], column-wise mirror rules as for sigma
                F = np.eye(3) + np.swapaxes(gu, -1, -2)
                P = mats.pk1(F)
                sig = np.swapaxes(P, -1, -2)
                trial = state
            else:
                eps = 0.5 * (gu + np.swapaxes(gu, -1, -2))
                sig, trial = mats.stress(eps, state, step.dt)
            Dv = pl.div(sig) + Dstar
            err = equilibrium_error(pl, Dv, sig)
            ms = sig.mean(axis=(0, 1, 2, 3))
            if fs:
                ms = ms.T                                # <P>[q, J]
            mvo = np.array([ms[i, j] for (i, j) in VOIGT])
            mixed_ok = True
            if S_idx.size:
                r = step.mixed_target[S_idx] - mvo[S_idx]
                mixed_ok = np.max(np.abs(r)) <= prob.tol * np.linalg.norm(ms)
            log.append({"step": t, "iter": m, "err": err, "macro_sigma": mvo.copy()})
            if callback is not None:
                callback(t, m, err)
            if err < prob.tol and mixed_ok:
                converged = True
                break
            if m >= prob.max_iter:
                break
            if S_idx.size:
                dE = np.linalg.solve(C0[np.ix_(S_idx, S_idx)], r)
                for a, v in zip(S_idx, dE):
                    i, j = VOIGT[a]
                    if i == j:
                        G[i, i] += v
                    else:
                        G[i, j] += v
                        G[j, i] += v
            p = pl.L0(uf) - Dv
            g = p
            f = g - x_prev
            hist.append((g, f))
            hist = hist[-prob.aa_depth:]
            aa = False
            x = g
            if m >= 2 and m % prob.aa_period == 0 and len(hist) >= 2:
                k = len(hist)
                F = np.array([[pl.dot_kept(hist[a][1], hist[b][1]) for b in range(k)]
                              for a in range(k)])
                al = anderson_weights(F)
                if al is not None:
                    x = sum(al[a] * hist[a][0] for a in range(k))
                    aa = True
            log[-1]["aa"] = aa
            uf = pl.green_apply(x)
            x_prev = x
            m += 1
        state = trial
        Gs.append(G.copy())
        macro.append(mvo)
        iters.append(m)
        conv.append(converged)
    us = pl.ustar(prob.steps[-1].c, Gs[-1], prob.steps[-1].H, getattr(prob.steps[-1], "ustar_nodal", None))
    u = uf + us
    if fs:
        # outputs of a finite-strain solve: Green-Lagrange strain and Cauchy stress
        F = np.eye(3) + np.swapaxes(gu, -1, -2)
        P = np.swapaxes(sig, -1, -2)
        eps = 0.5 * (np.einsum("...ki,...kj->...ij", F, F) - np.eye(3))
        sig = (P @ np.swapaxes(F, -1, -2)) / np.linalg.det(F)[..., None, None]

    def vox_out(T):
        out = np.empty((6, pl.nppv, n[2], n[1], n[0]))
        for a, (i, j) in enumerate(VOIGT):
            out[a] = T[..., i, j].transpose(0, 3, 2, 1)
        return out

    return {
        "u": u.transpose(0, 3, 2, 1).copy(),
        "uf": uf.transpose(0, 3, 2, 1).copy(),
        "eps": vox_out(eps),
        "sig": vox_out(sig),
        "macro_sigma": np.array(macro),
        "iters": iters,
        "converged": conv,
        "G": np.array(Gs),
        "log": log,
        "nvox": nvox,
    }
