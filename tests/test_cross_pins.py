"""Pins of the bin-bin cross-correlation oracle (Sec. II.B.i, Sec. III.C.i)
against the hand-worked lag fixture, loop brute force, the sum rule that
returns Eq. 17, and the zero-lag symmetry.  Mutation tests plant plausible
mistakes in copies of the oracle and show that a pin rejects each one."""
import numpy as np

import oracle
import synth
from oracle import cross as ox
from tests import _golden


def _lags_fixture():
    g = _golden.read("gkma_lags.txt")
    a = np.array([float(x) for x in g["Jb"][0]])
    b = np.array([float(x) for x in g["Jt"][0]])
    S = a.size
    Jb = np.zeros((S, 3, 2))
    Jb[:, 0, 0] = a            # bin 0, x
    Jb[:, 1, 1] = b            # bin 1, y
    return g, Jb


def test_golden_cross_pair():
    """Bin 0's x series is the fixture's modal series and bin 1's y series its
    second series, so C[tau, 0, 1, x, y] is the hand-worked correlation."""
    g, Jb = _lags_fixture()
    L = len(g["corr"][0])
    C = ox.gkma_cross_correlation(Jb, L)
    np.testing.assert_allclose(C[:, 0, 1, 0, 1], [float(x) for x in g["corr"][0]], rtol=0, atol=1e-15)
    mask = np.ones(C.shape, bool)
    mask[:, 0, 1, 0, 1] = False
    mask[:, 0, 0, 0, 0] = False
    mask[:, 1, 1, 1, 1] = False
    mask[:, 1, 0, 1, 0] = False
    assert np.all(C[mask] == 0)


def test_brute_force_loops():
    rng = np.random.default_rng(8)
    Jb = rng.standard_normal((6, 3, 3))
    np.testing.assert_allclose(ox.gkma_cross_correlation(Jb, 8), ox.gkma_cross_correlation_loops(Jb.tolist(), 8),
                               rtol=1e-13, atol=1e-15)


def test_sum_over_second_bin_is_eq17():
    """Every mode binned and a complete basis: the binned currents sum to the
    Eq. 10 total, so the sum over b2 is the GKMA correlation with the total."""
    lat = synth.BlochLattice((3, 3, 2))
    E = lat.eig_matrix()
    m = synth.masses(lat.n_atoms, "natural", 4)
    v, W = synth.gen_steps(4, m, 0, 9)
    bins = oracle.bin_of_mode(lat.frequencies, 4, 0.0, lat.f_max)
    assert np.all(bins >= 0)
    d = oracle.run_dense(E, m, v, W, bins, 4, corr_len=5)
    C = ox.gkma_cross_correlation(d["Jb"], 5)
    np.testing.assert_allclose(C.sum(axis=2), d["corr"], rtol=1e-11, atol=1e-14)


def test_zero_lag_symmetry():
    rng = np.random.default_rng(9)
    Jb = rng.standard_normal((11, 3, 4))
    C = ox.gkma_cross_correlation(Jb, 3)
    np.testing.assert_allclose(C[0], C[0].transpose(1, 0, 3, 2), rtol=1e-14, atol=1e-15)
    assert not np.allclose(C[1], C[1].transpose(1, 0, 3, 2))


def test_mutation_swapped_bins_fails_golden():
    g, Jb = _lags_fixture()
    L = len(g["corr"][0])
    bad = ox.gkma_cross_correlation(Jb, L).transpose(0, 2, 1, 4, 3)      # <J_b2(t+tau) J_b(t)>
    assert not np.allclose(bad[:, 0, 1, 0, 1], [float(x) for x in g["corr"][0]], atol=1e-12)


def test_mutation_normalised_by_S_fails_golden():
    g, Jb = _lags_fixture()
    L = len(g["corr"][0])
    S = Jb.shape[0]
    bad = ox.gkma_cross_correlation(Jb, L) * (S - np.arange(L))[:, None, None, None, None] / S
    assert not np.allclose(bad[:, 0, 1, 0, 1], [float(x) for x in g["corr"][0]], atol=1e-12)
