"""Pins of the oracle behaviour laws.

P11: J2 with linear hardening under monotonic pure shear follows the
     closed-form bilinear response tau = mu gamma, then slope mu H / (H + 3 mu).
P12: crystal plasticity, [001] single crystal under uniaxial strain: by the
     cubic symmetry only the 8 systems with Schmid product 1/sqrt(6) slip, by
     equal amounts, which reduces backward Euler to one scalar equation solved
     here by bisection, with the Voce CRSS integrated from its hardening rate.
P13: rotated cubic stiffness keeps its rotation invariants (bulk modulus,
     Frobenius norm), and the 12 FCC systems are unit, orthogonal, {111}<110>.
     Unrotated, its entries are the textbook ones (sigma_11 = C11 eps_11,
     sigma_22 = C12 eps_11, sigma_12 = 2 C44 eps_12); rotated, the Young's
     modulus along a sample direction d follows the closed form of cubic
     crystals in the crystal-frame direction cosines of d (which fixes the
     crystal -> sample sense of the quaternion).
Voce: tau_c(Gamma) solves d tau_c / d Gamma = theta0 (taus - tau_c) /
     (taus - tau0), tau_c(0) = tau0 (integrated numerically here).
Frame: rotating the strain and the crystal together rotates the stress, the
     plastic strain and leaves the accumulated slip unchanged (CP and cubic).
"""
import numpy as np
import pytest

from oracle import laws


def test_cubic_rotation_invariants():
    rng = np.random.default_rng(0)
    C = laws.cubic_tensor(168.0, 121.0, 75.0)
    for _ in range(5):
        q = rng.standard_normal(4)
        R = laws.quat_to_rot(q)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert np.linalg.det(R) == pytest.approx(1.0)
        Cr = laws.rotate4(C, R)
        K = np.einsum("iijj->", Cr) / 9.0
        assert K == pytest.approx((168.0 + 2 * 121.0) / 3.0)
        assert np.linalg.norm(Cr) == pytest.approx(np.linalg.norm(C))
        # major and minor symmetries
        np.testing.assert_allclose(Cr, Cr.transpose(2, 3, 0, 1), atol=1e-10)
        np.testing.assert_allclose(Cr, Cr.transpose(1, 0, 2, 3), atol=1e-10)


def test_fcc_systems():
    m, n = laws.fcc_slip_systems()
    np.testing.assert_allclose(np.linalg.norm(m, axis=1), 1.0)
    np.testing.assert_allclose(np.linalg.norm(n, axis=1), 1.0)
    np.testing.assert_allclose(np.sum(m * n, axis=1), 0.0, atol=1e-15)
    assert np.allclose(np.abs(n) * np.sqrt(3.0), 1.0)
    np.testing.assert_allclose(np.sort(np.abs(m) * np.sqrt(2.0), axis=1), np.tile([0.0, 1.0, 1.0], (12, 1)), atol=1e-14)
    # no duplicate system up to sign
    keys = {tuple(np.round(np.sign(m[s][np.argmax(np.abs(m[s]))]) * np.concatenate([m[s], n[s]]), 6))
            for s in range(12)}
    assert len(keys) == 12


def test_j2_pure_shear_closed_form():
    E, nu, sy0, H = 70.0, 0.33, 0.1, 1.0
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    ty = sy0 / np.sqrt(3.0)
    gy = ty / mu
    ep = np.zeros((3, 3))
    p = 0.0
    for g in np.linspace(0.0, 8.0 * gy, 41)[1:]:
        eps = np.zeros((3, 3)); eps[0, 1] = eps[1, 0] = 0.5 * g
        sig, ep, p = laws.j2_update(eps[None], ep[None], np.array([p]), lam, mu, sy0, H)
        sig, ep, p = sig[0], ep[0], float(p[0])
        exact = mu * g if g <= gy else ty + mu * H / (H + 3 * mu) * (g - gy)
        assert sig[0, 1] == pytest.approx(exact, rel=1e-12)
        assert abs(sig[0, 0]) < 1e-12 and abs(sig[2, 2]) < 1e-12


def _voce_ode(G, tau0, taus, th0, steps=4000):
    """tau_c(G) by RK4 on d tau / d Gamma = th0 (taus - tau) / (taus - tau0)
    from tau(0) = tau0 (the Voce hardening rate, not its closed form)."""
    if G == 0.0:
        return tau0
    f = lambda t: th0 * (taus - t) / (taus - tau0)
    h = G / steps
    t = tau0
    for _ in range(steps):
        k1 = f(t); k2 = f(t + 0.5 * h * k1); k3 = f(t + 0.5 * h * k2); k4 = f(t + h * k3)
        t += h * (k1 + 2 * k2 + 2 * k3 + k4) / 6.0
    return t


def test_voce_against_hardening_rate():
    tau0, taus, th0 = 0.05, 0.15, 0.3
    for G in (0.0, 1e-3, 0.05, 0.3, 2.0):
        ref = _voce_ode(G, tau0, taus, th0)
        assert laws.voce(G, tau0, taus, th0) == pytest.approx(ref, rel=1e-12, abs=1e-15)
        # the slope is the hardening rate at that CRSS
        assert laws.voce_slope(G, tau0, taus, th0) == pytest.approx(th0 * (taus - ref) / (taus - tau0),
                                                                     rel=1e-10)


def _scalar_cp_root(e, C11, C12, gdot0, nexp, tau0, taus, th0, dt, Gn=0.0):
    """gamma = dt gdot0 (tau/tau_c)^n with tau = (C11-C12)(e - 12 gamma/sqrt6)/sqrt6
    and tau_c the Voce CRSS at Gn + 8 gamma; bisection in gamma."""
    s6 = np.sqrt(6.0)

    def F(g):
        tau = (C11 - C12) * (e - 12.0 * g / s6) / s6
        tc = _voce_ode(Gn + 8.0 * g, tau0, taus, th0, steps=400)
        return g - dt * gdot0 * np.sign(tau) * abs(tau / tc) ** nexp

    lo, hi = 0.0, e * s6 / 12.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if F(mid) > 0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("e", [2e-4, 8e-4, 2e-3])
def test_cp_001_uniaxial_strain(e):
    C11, C12, C44 = 168.0, 121.0, 75.0
    prm = (1e-3, 20.0, 0.05, 0.15, 0.3)
    Cm = laws.mandel_matrix(laws.cubic_tensor(C11, C12, C44))
    m, n = laws.fcc_slip_systems()
    P = 0.5 * (np.einsum("si,sj->sij", m, n) + np.einsum("si,sj->sij", n, m))
    Pm = laws.to_mandel(P)
    eps = np.zeros((3, 3)); eps[2, 2] = e
    sM, epM, G = laws.cp_update(laws.to_mandel(eps)[None], np.zeros((1, 6)), np.zeros(1),
                                Cm, Pm, prm, 1.0)
    g = _scalar_cp_root(e, C11, C12, *prm, 1.0)
    assert G[0] == pytest.approx(8.0 * g, rel=1e-8)
    ep = laws.from_mandel(epM[0])
    assert ep[2, 2] == pytest.approx(8.0 * g / np.sqrt(6.0), rel=1e-8)
    sig = laws.from_mandel(sM[0])
    tau = (C11 - C12) * (e - 12.0 * g / np.sqrt(6.0)) / np.sqrt(6.0)
    assert (sig[2, 2] - sig[0, 0]) / np.sqrt(6.0) == pytest.approx(tau, rel=1e-8)


def test_cubic_entries_unrotated():
    C11, C12, C44 = 168.0, 121.0, 75.0
    C = laws.cubic_tensor(C11, C12, C44)
    e = np.zeros((3, 3)); e[0, 0] = 1e-3
    sig = np.einsum("ijkl,kl->ij", C, e)
    assert sig[0, 0] == pytest.approx(C11 * 1e-3) and sig[1, 1] == pytest.approx(C12 * 1e-3)
    assert sig[2, 2] == pytest.approx(C12 * 1e-3) and abs(sig[0, 1]) < 1e-15
    for (i, j) in ((0, 1), (0, 2), (1, 2)):
        e = np.zeros((3, 3)); e[i, j] = e[j, i] = 1e-3      # tensor shear strain
        sig = np.einsum("ijkl,kl->ij", C, e)
        assert sig[i, j] == pytest.approx(2.0 * C44 * 1e-3)
        assert np.count_nonzero(np.abs(sig) > 1e-14) == 2


def _young_closed_form(C11, C12, C44, l):
    """1/E = S11 - 2 (S11 - S12 - S44/2)(l1^2 l2^2 + l2^2 l3^2 + l3^2 l1^2),
    crystal-frame direction cosines l, engineering-shear compliances."""
    det = (C11 - C12) * (C11 + 2.0 * C12)
    S11 = (C11 + C12) / det
    S12 = -C12 / det
    S44 = 1.0 / C44
    G = l[0] ** 2 * l[1] ** 2 + l[1] ** 2 * l[2] ** 2 + l[2] ** 2 * l[0] ** 2
    return 1.0 / (S11 - 2.0 * (S11 - S12 - 0.5 * S44) * G)


def test_cubic_directional_young_modulus():
    C11, C12, C44 = 168.0, 121.0, 75.0
    rng = np.random.default_rng(3)
    # the textbook extremes: E[100] and E[111]
    C = laws.cubic_tensor(C11, C12, C44)
    Sm = np.linalg.inv(laws.mandel_matrix(C))
    for d, ref in ((np.array([1.0, 0, 0]), _young_closed_form(C11, C12, C44, [1, 0, 0])),
                   (np.ones(3) / np.sqrt(3.0), 1.0 / (1.0 / 3.0 * ((C11 + 2 * C12) ** -1)
                                                      + 1.0 / (3.0 * C44)))):
        eps = laws.from_mandel(Sm @ laws.to_mandel(np.outer(d, d)))
        assert 1.0 / (d @ eps @ d) == pytest.approx(ref, rel=1e-12)
    for _ in range(6):
        q = rng.standard_normal(4)
        R = laws.quat_to_rot(q)                    # crystal -> sample
        Cs = laws.rotate4(C, R)
        Ss = np.linalg.inv(laws.mandel_matrix(Cs))
        d = rng.standard_normal(3); d /= np.linalg.norm(d)
        eps = laws.from_mandel(Ss @ laws.to_mandel(np.outer(d, d)))
        E = 1.0 / (d @ eps @ d)
        assert E == pytest.approx(_young_closed_form(C11, C12, C44, R.T @ d), rel=1e-10)


def test_quaternion_rotation_sense():
    """quat (cos t/2, 0, 0, sin t/2) turns e_x towards e_y by t about z."""
    t = 0.7
    R = laws.quat_to_rot([np.cos(t / 2), 0.0, 0.0, np.sin(t / 2)])
    np.testing.assert_allclose(R @ np.array([1.0, 0, 0]), [np.cos(t), np.sin(t), 0.0], atol=1e-15)
    R = laws.quat_to_rot([np.cos(t / 2), np.sin(t / 2), 0.0, 0.0])
    np.testing.assert_allclose(R @ np.array([0, 1.0, 0]), [0.0, np.cos(t), np.sin(t)], atol=1e-15)


@pytest.mark.parametrize("law", ["cp", "cubic"])
def test_frame_equivariance(law):
    """sigma(R eps R^T; crystal rotated by R) = R sigma(eps; crystal unrotated) R^T,
    and the same for the plastic strain; the accumulated slip is unchanged."""
    import workloads as W
    rng = np.random.default_rng(9)
    q = rng.standard_normal(4); q /= np.linalg.norm(q)
    R = laws.quat_to_rot(q)
    prm = dict(gdot0=1e-3, nexp=20.0, tau0=0.05, taus=0.15, theta0=0.3)
    if law == "cp":
        rot = W.mat_cp(168.0, 121.0, 75.0, q, **prm)
        ident = W.mat_cp(168.0, 121.0, 75.0, [1.0, 0, 0, 0], **prm)
    else:
        rot = W.mat_cubic(168.0, 121.0, 75.0, q)
        ident = W.mat_cubic(168.0, 121.0, 75.0, [1.0, 0, 0, 0])
    ids = np.zeros((1, 1, 1), dtype=np.int32)
    ms_r = laws.MaterialSet([rot], ids)
    ms_i = laws.MaterialSet([ident], ids)
    e = rng.uniform(-2e-3, 2e-3, (3, 3)); e = 0.5 * (e + e.T)
    eps_r = (R @ e @ R.T)[None, None, None, None]
    eps_i = e[None, None, None, None]
    st_r, st_i = ms_r.init_state(1, (1, 1, 1)), ms_i.init_state(1, (1, 1, 1))
    for _ in range(3):                            # three increments of the same strain path
        sr, nr = ms_r.stress(eps_r, st_r, 1.0)
        si, ni = ms_i.stress(eps_i, st_i, 1.0)
        np.testing.assert_allclose(sr[0, 0, 0, 0], R @ si[0, 0, 0, 0] @ R.T, atol=1e-12)
        np.testing.assert_allclose(nr["ep"][0, 0, 0, 0], R @ ni["ep"][0, 0, 0, 0] @ R.T, atol=1e-14)
        assert nr["p"][0, 0, 0, 0] == pytest.approx(ni["p"][0, 0, 0, 0], rel=1e-9, abs=1e-15)
        st_r, st_i = nr, ni
        eps_r = eps_r * 1.5; eps_i = eps_i * 1.5
    if law == "cp":
        assert ni["p"][0, 0, 0, 0] > 0                 # slip happened


def _fd_pk1(psi, F, h=1e-6):
    """P = d psi / dF by central differences of the strain energy."""
    P = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            Fp = F.copy(); Fp[i, j] += h
            Fm = F.copy(); Fm[i, j] -= h
            P[i, j] = (psi(Fp) - psi(Fm)) / (2 * h)
    return P


def test_finite_strain_laws_derive_from_their_energies():
    """P of the SVK and Neo-Hookean laws = d psi / dF of the energies written
    out here (SVK: lam/2 tr(E)^2 + mu tr(E^2); Neo-Hookean, Appendix B:
    mu/2 (J^-2/3 tr(F F^T) - 3) + K/2 (J - 1)^2), at random deformations."""
    rng = np.random.default_rng(12)
    lam, mu, K = 1.2, 0.8, 2.5

    def psi_svk(F):
        E = 0.5 * (F.T @ F - np.eye(3))
        return 0.5 * lam * np.trace(E) ** 2 + mu * np.trace(E @ E)

    def psi_nh(F):
        J = np.linalg.det(F)
        return 0.5 * mu * (J ** (-2.0 / 3.0) * np.trace(F @ F.T) - 3.0) + 0.5 * K * (J - 1.0) ** 2

    for _ in range(5):
        F = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
        np.testing.assert_allclose(laws.svk_pk1(F, lam, mu), _fd_pk1(psi_svk, F), atol=1e-7)
        np.testing.assert_allclose(laws.neohooke_pk1(F, mu, K), _fd_pk1(psi_nh, F), atol=1e-7)
    # objectivity: P(Q F) = Q P(F) for a rotation Q
    Q = laws.quat_to_rot(rng.standard_normal(4))
    F = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
    np.testing.assert_allclose(laws.neohooke_pk1(Q @ F, mu, K), Q @ laws.neohooke_pk1(F, mu, K), atol=1e-12)
    np.testing.assert_allclose(laws.svk_pk1(Q @ F, lam, mu), Q @ laws.svk_pk1(F, lam, mu), atol=1e-12)
