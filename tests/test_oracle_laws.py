"""Pins of the oracle behaviour laws.

P11: J2 with linear hardening under monotonic pure shear follows the
     closed-form bilinear response tau = mu gamma, then slope mu H / (H + 3 mu).
P12: crystal plasticity, [001] single crystal under uniaxial strain: by the
     cubic symmetry only the 8 systems with Schmid product 1/sqrt(6) slip, by
     equal amounts, which reduces backward Euler to one scalar equation solved
     here by bisection.
P13: rotated cubic stiffness keeps its rotation invariants (bulk modulus,
     Frobenius norm), and the 12 FCC systems are unit, orthogonal, {111}<110>.
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


def _scalar_cp_root(e, C11, C12, gdot0, nexp, tau0, taus, th0, dt, Gn=0.0):
    """gamma = dt gdot0 (tau/tau_c)^n with tau = (C11-C12)(e - 12 gamma/sqrt6)/sqrt6
    and tau_c = voce(Gn + 8 gamma); bisection in gamma."""
    s6 = np.sqrt(6.0)

    def F(g):
        tau = (C11 - C12) * (e - 12.0 * g / s6) / s6
        tc = laws.voce(Gn + 8.0 * g, tau0, taus, th0)
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
