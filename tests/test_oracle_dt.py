"""Pins of the oracle transforms against Table 1 (Sec. 2.4, Tab. BCsSymmetriesDTTDFT).

P1: DT(G) = alpha^-1 DFT(E)[mapped k] on the explicitly built extension E.
P2: the O(n^2) sums written out from Table 1 equal the scipy-based transforms.
P3: round trip iDT(DT(G)) = G on the kept nodes (Sec. 2.7.2 validation recipe).
"""
import numpy as np
import pytest

from oracle import dt

KINDS = [dt.DFT, dt.DCT1, dt.DST1, dt.DCT3, dt.DST3]
SIZES = [1, 2, 3, 4, 5, 7, 8, 12, 31, 32, 33]


def _rand_nodes(rng, kind, n, cplx=False):
    g = rng.standard_normal(n + 1)
    if cplx:
        g = g + 1j * rng.standard_normal(n + 1)
    # dismissed entries are not part of the field
    keep = np.zeros(n + 1, dtype=bool)
    keep[dt.kept_nodes(kind, n)] = True
    g = np.where(keep, g, 0.0)
    return g


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", SIZES)
def test_extension_identity(kind, n):
    if kind == dt.DST1 and n < 2:
        pytest.skip("DST-I needs n >= 2")
    rng = np.random.default_rng(100 + n + 7 * kind)
    g = _rand_nodes(rng, kind, n)
    E = dt.extension(g, kind)
    assert len(E) == dt.symmetry_factor(kind) * n
    Ehat = np.fft.fft(E)
    Gt = dt.forward_1d(g, kind, 0)
    k = np.arange(dt.n_freq(kind, n))
    np.testing.assert_allclose(Ehat[dt.ext_dft_index(kind, k)], dt.alpha(kind) * Gt,
                               rtol=0, atol=1e-12 * max(1.0, np.abs(Ehat).max()))


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", SIZES)
def test_bruteforce_sums(kind, n):
    if kind == dt.DST1 and n < 2:
        pytest.skip("DST-I needs n >= 2")
    rng = np.random.default_rng(200 + n + 7 * kind)
    for cplx in (False, True):
        g = _rand_nodes(rng, kind, n, cplx)
        M = dt.brute_matrix(kind, n)
        np.testing.assert_allclose(dt.forward_1d(g, kind, 0), M @ g, rtol=0,
                                   atol=1e-13 * max(1.0, n) * np.abs(g).max())


def test_alpha_and_symmetry_factor_golden():
    """Table 1 third column, stored with its citation in tests/golden."""
    import json, os
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_alpha.json")
    with open(path) as f:
        gold = json.load(f)
    names = {"PP": dt.DFT, "SS": dt.DCT1, "AA": dt.DST1, "SA": dt.DCT3, "AS": dt.DST3}
    for key, row in gold["rows"].items():
        kind = names[key]
        assert dt.symmetry_factor(kind) == row["S_f"]
        a = complex(row["alpha_re"], row["alpha_im"])
        assert dt.alpha(kind) == a
        assert list(dt.ext_dft_index(kind, np.arange(3))) == row["mapped_first3"]
        assert dt.NAMES[kind] == row["transform"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", [2, 3, 5, 8, 16, 33])
def test_round_trip(kind, n):
    rng = np.random.default_rng(300 + n + kind)
    g = _rand_nodes(rng, kind, n)
    back = dt.inverse_1d(dt.forward_1d(g, kind, 0), kind, 0, n)
    keep = dt.kept_nodes(kind, n)
    np.testing.assert_allclose(back[keep], g[keep], atol=1e-12)


def test_inverse_equals_matrix_inverse():
    """The inverse transform equals the inverse of the Table 1 matrix restricted
    to the kept nodes (independent of scipy's inverse routines)."""
    rng = np.random.default_rng(7)
    for kind in KINDS:
        for n in (4, 7, 10):
            keep = dt.kept_nodes(kind, n)
            M = dt.brute_matrix(kind, n)[:, keep]
            G = rng.standard_normal(dt.n_freq(kind, n))
            ref = np.linalg.solve(M, G)
            got = dt.inverse_1d(G.astype(complex) if kind == dt.DFT else G, kind, 0, n)[keep]
            np.testing.assert_allclose(got, ref, atol=1e-11)


@pytest.mark.parametrize("seed", range(6))
def test_round_trip_3d_all_combinations(seed):
    rng = np.random.default_rng(seed)
    n = tuple(int(v) for v in rng.integers(2, 9, size=3))
    for _ in range(8):
        kinds = [int(v) for v in rng.integers(0, 5, size=3)]
        g = rng.standard_normal(tuple(v + 1 for v in n))
        G = dt.forward_3d(g, kinds)
        back = dt.inverse_3d(G, kinds, n)
        sl = np.ix_(*[dt.kept_nodes(kinds[i], n[i]) for i in range(3)])
        np.testing.assert_allclose(back[sl], g[sl], atol=1e-11)
