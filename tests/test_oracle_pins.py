"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these checks re-types the oracle's formulas: each compares it with a
hand-worked value, a closed form, an invariant of the method, an independent
library route (FFT), or a statistical expectation of the synthetic inputs.
The mutation tests at the end plant plausible mistakes in copies of the
oracle's functions and show that some pin here rejects each one.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from tests import _golden


def _f(x):
    return float(x)


# ------------------------------------------------------------ hand-worked
def _two_atom_inputs():
    g = _golden.read("two_atom_chain.txt")
    m = np.array([_f(x) for x in g["mass"][0]])
    v = np.zeros((1, 2, 3))
    for row in g["v"]:
        v[0, int(row[0])] = [_f(x) for x in row[1:]]
    W = np.zeros((1, 2, 3, 3))
    for row in g["W"]:
        W[0, int(row[0]), "xyz".index(row[1])] = [_f(x) for x in row[2:]]
    return g, m, v, W


def test_two_atom_chain_basis_is_the_hand_basis():
    E = synth.BlochLattice((2, 1, 1)).eig_matrix()
    s = 1 / math.sqrt(2)
    hand = np.zeros((6, 6))
    for f, phi in enumerate([(s, s), (s, -s)]):
        for a in range(3):
            hand[a, 3 * f + a] = phi[0]
            hand[3 + a, 3 * f + a] = phi[1]
    assert np.array_equal(E, hand)


def test_two_atom_chain_golden():
    g, m, v, W = _two_atom_inputs()
    E = synth.BlochLattice((2, 1, 1)).eig_matrix()
    u = oracle.mass_weighted_velocity(m, v)
    xdot = oracle.modal_velocity(E, u)[0]
    want_x = np.array([_f(r[1]) for r in g["xdot_sqrt2"]]) / math.sqrt(2)
    np.testing.assert_allclose(xdot, want_x, rtol=0, atol=1e-14)
    Jn = oracle.modal_currents(E, m, v, W)[0]            # [3, M]
    want_Jn = np.array([[_f(x) for x in r[1:]] for r in g["Jn"]])  # [M, 3]
    np.testing.assert_allclose(Jn.T, want_Jn, rtol=0, atol=1e-13)
    bins = np.array([int(b) for b in g["bins"][0]])
    Jb = oracle.binned_current(Jn[None], bins, 2)[0]     # [3, nb]
    want_Jb = np.array([[_f(x) for x in r[1:]] for r in g["Jb"]])
    np.testing.assert_allclose(Jb.T, want_Jb, rtol=0, atol=1e-13)
    Jt = oracle.total_heat_current(v, W)[0]
    np.testing.assert_allclose(Jt, [_f(x) for x in g["total"][0]], rtol=0, atol=1e-14)
    ke = 0.5 * float(xdot @ xdot)
    assert abs(ke - _f(g["kinetic"][0][0])) < 1e-12


def test_gkma_lags_golden():
    g = _golden.read("gkma_lags.txt")
    Jb = np.array([_f(x) for x in g["Jb"][0]])
    Jt = np.array([_f(x) for x in g["Jt"][0]])
    S = Jb.size
    Jb3 = np.zeros((S, 3, 1)); Jb3[:, 0, 0] = Jb
    Jt3 = np.zeros((S, 3)); Jt3[:, 0] = Jt
    L = len(g["corr"][0])
    C = oracle.gkma_correlation(Jb3, Jt3, L)
    np.testing.assert_allclose(C[:, 0, 0, 0], [_f(x) for x in g["corr"][0]], rtol=0, atol=1e-15)
    assert np.all(C[:, 0, 1:, :] == 0) and np.all(C[:, 0, :, 1:] == 0)
    G = oracle.gkma_running_integral(C, 1.0)
    np.testing.assert_allclose(G[:, 0, 0, 0], [_f(x) for x in g["integral"][0]], rtol=0, atol=1e-15)
    np.testing.assert_array_equal(oracle.correlation_counts(S, L), [4, 3, 2, 1, 0])


def test_hnema_average_golden():
    """Eq. 19 numerator on the hand-worked series: the mean over all S samples
    (an S - 1 denominator or a dropped sample gives another fraction)."""
    g = _golden.read("gkma_lags.txt")
    Jb = np.array([_f(x) for x in g["Jb"][0]])
    Jt = np.array([_f(x) for x in g["Jt"][0]])
    S = Jb.size
    Jb3 = np.zeros((S, 3, 2))
    Jb3[:, 1, 0] = Jb
    Jb3[:, 2, 1] = Jt
    avg = oracle.hnema_average(Jb3)
    want = np.zeros((2, 3))
    want[0, 1] = _f(g["mean_Jb"][0][0])
    want[1, 2] = _f(g["mean_Jt"][0][0])
    np.testing.assert_array_equal(avg, want)


def test_mutation_hnema_sample_count_fails_golden():
    g = _golden.read("gkma_lags.txt")
    Jb = np.array([_f(x) for x in g["Jb"][0]])
    assert Jb.sum() / (Jb.size - 1) != _f(g["mean_Jb"][0][0])


def test_single_atom_identity_basis_brute_force():
    """N = 1: the basis is the identity, masses cancel, J_alpha^mu = W^{mu alpha} v^alpha."""
    E = synth.BlochLattice((1, 1, 1)).eig_matrix()
    assert np.array_equal(E, np.eye(3))
    rng = np.random.default_rng(5)
    m = np.array([17.0])
    v = rng.standard_normal((3, 1, 3))
    W = rng.standard_normal((3, 1, 3, 3))
    Jn = oracle.modal_currents(E, m, v, W)
    for s in range(3):
        for mu in range(3):
            for a in range(3):
                assert abs(Jn[s, mu, a] - W[s, 0, mu, a] * v[s, 0, a]) < 1e-15


# --------------------------------------------------------------- invariants
def _case(dims=(4, 3, 2), mass_kind="natural", S=6, seed=3, nb=12):
    lat = synth.BlochLattice(dims)
    E = lat.eig_matrix()
    m = synth.masses(lat.n_atoms, mass_kind, seed)
    v, W = synth.gen_steps(seed, m, 0, S)
    bins = oracle.bin_of_mode(lat.frequencies, nb, 0.0, lat.f_max)
    return lat, E, m, v, W, bins, nb


@pytest.mark.parametrize("dims", [(4, 3, 2), (3, 3, 3), (4, 4, 4)])
def test_basis_orthonormal_and_complete(dims):
    E = synth.BlochLattice(dims).eig_matrix()
    n = E.shape[0]
    assert np.abs(E.T @ E - np.eye(n)).max() < 1e-13
    assert np.abs(E @ E.T - np.eye(n)).max() < 1e-13


@pytest.mark.parametrize("dims", [(4, 3, 2), (3, 3, 3)])
def test_completeness_modal_sum_is_total_current(dims):
    """Eq. 14 (completeness) + Eq. 10: the modal currents sum to the total."""
    lat, E, m, v, W, bins, nb = _case(dims)
    out = oracle.run_dense(E, m, v, W, bins, nb)
    np.testing.assert_allclose(out["Jn"].sum(axis=2), out["Jt"], rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(out["Jb"].sum(axis=2), out["Jt"], rtol=1e-12, atol=1e-16)


def test_completeness_with_dense_random_basis():
    rng_E = synth.random_orthonormal(3 * 10, seed=11)
    m = synth.masses(10, "natural", 2)
    v, W = synth.gen_steps(2, m, 0, 4)
    Jn = oracle.modal_currents(rng_E, m, v, W)
    np.testing.assert_allclose(Jn.sum(axis=2), oracle.total_heat_current(v, W), rtol=1e-12, atol=1e-16)


def test_kinetic_energy_parseval():
    """Eq. 13 with an orthonormal basis: sum_n Xdot_n^2 / 2 = sum_i m_i |v_i|^2 / 2."""
    lat, E, m, v, W, bins, nb = _case((4, 3, 2))
    xdot = oracle.modal_velocity(E, oracle.mass_weighted_velocity(m, v))
    ke_modes = 0.5 * (xdot ** 2).sum(axis=1)
    ke_atoms = 0.5 * (m[None, :, None] * v.astype(np.float64) ** 2).sum(axis=(1, 2))
    np.testing.assert_allclose(ke_modes, ke_atoms, rtol=1e-12)


def test_harmonic_round_trip_eq14():
    """Prescribe Xdot_n(t), build v by Eq. 14, project back by Eq. 13."""
    n_atoms = 8
    E = synth.random_orthonormal(3 * n_atoms, seed=4)      # not symmetric
    assert np.abs(E - E.T).max() > 0.1
    m = synth.masses(n_atoms, "natural", 9)
    rng = np.random.default_rng(1)
    amp = rng.uniform(0.5, 2.0, 3 * n_atoms)
    omega = rng.uniform(0.01, 0.2, 3 * n_atoms)
    phase = rng.uniform(0, 2 * np.pi, 3 * n_atoms)
    t = np.arange(10.0)
    xdot = amp[None, :] * np.cos(omega[None, :] * t[:, None] + phase[None, :])
    # Eq. 14: v_i = m_i^{-1/2} sum_n e_{i,n} Xdot_n
    v = ((E @ xdot.T).T).reshape(10, n_atoms, 3) / np.sqrt(m)[None, :, None]
    back = oracle.modal_velocity(E, oracle.mass_weighted_velocity(m, v))
    np.testing.assert_allclose(back, xdot, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("dims", [(4, 3, 2), (6, 4, 2), (5, 3, 1)])
def test_fft_special_case(dims):
    """Dense oracle vs the Parseval/FFT form of the binned current."""
    lat, E, m, v, W, bins, nb = _case(dims, nb=9)
    dense = oracle.run_dense(E, m, v, W, bins, nb)["Jb"]
    kb = oracle.bin_of_mode(lat.kpoint_frequencies().ravel(), nb, 0.0, lat.f_max).reshape(lat.dims)
    fft = oracle.binned_current_fft(lat.dims, m, v, W, kb, nb)
    scale = np.abs(dense).max()
    assert np.abs(dense - fft).max() < 1e-13 * scale


def test_invariance_mode_permutation_and_degenerate_rotation():
    lat, E, m, v, W, bins, nb = _case((4, 4, 2), nb=7)
    ref = oracle.run_dense(E, m, v, W, bins, nb)["Jb"]
    rng = np.random.default_rng(7)
    perm = rng.permutation(E.shape[1])
    got = oracle.run_dense(E[:, perm], m, v, W, bins[perm], nb)["Jb"]
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-15)
    # rotate inside each bin's subspace: P_b = E_b E_b^T is unchanged
    E2 = E.copy()
    for b in range(nb):
        sel = np.nonzero(bins == b)[0]
        if sel.size > 1:
            E2[:, sel] = E[:, sel] @ synth.random_orthonormal(sel.size, seed=b)
    got = oracle.run_dense(E2, m, v, W, bins, nb)["Jb"]
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-15)


def test_bilinearity_and_single_bin():
    lat, E, m, v, W, bins, nb = _case((4, 3, 2))
    v = v.astype(np.float64); W = W.astype(np.float64)
    ref = oracle.run_dense(E, m, v, W, bins, nb)["Jb"]
    np.testing.assert_allclose(oracle.run_dense(E, m, 2.5 * v, W, bins, nb)["Jb"], 2.5 * ref, rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(oracle.run_dense(E, m, v, -3.0 * W, bins, nb)["Jb"], -3.0 * ref, rtol=1e-12, atol=1e-16)
    one = oracle.run_dense(E, m, v, W, np.zeros_like(bins), 1)
    np.testing.assert_allclose(one["Jb"][:, :, 0], one["Jt"], rtol=1e-12, atol=1e-16)


def test_transposed_virial_is_detected_by_eq10():
    """A nonsymmetric W with only W^{xy}: J^x = W^{xy} v^y, J^y = 0."""
    v = np.zeros((1, 1, 3)); v[0, 0] = [0.0, 2.0, 0.0]
    W = np.zeros((1, 1, 3, 3)); W[0, 0, 0, 1] = 3.0
    np.testing.assert_array_equal(oracle.total_heat_current(v, W)[0], [6.0, 0.0, 0.0])
    Jn = oracle.modal_currents(np.eye(3), np.array([5.0]), v, W)[0]
    np.testing.assert_allclose(Jn.sum(axis=1), [6.0, 0.0, 0.0], atol=1e-15)


# ------------------------------------------------------------- statistics
def test_statistical_equipartition_and_zero_lag_correlation():
    """iid inputs: E[Xdot_n^2] = k_B T (mass-weighted units);
    E[C_b^{mu nu}(0)] = delta_{mu nu} sigma_W^2 sigma_v^2 n_b (uniform mass)."""
    lat = synth.BlochLattice((4, 4, 4))
    E = lat.eig_matrix()
    m = synth.masses(lat.n_atoms)
    S = 3000
    v, W = synth.gen_steps(21, m, 0, S)
    xdot = oracle.modal_velocity(E, oracle.mass_weighted_velocity(m, v))
    kT = synth.KB_EV_PER_K * 300.0 / synth.AMU_A2_PER_FS2_IN_EV
    mean = (xdot ** 2).mean()
    se = (xdot ** 2).std() / math.sqrt(xdot.size)
    assert abs(mean - kT) < 5 * se
    nb = 5
    bins = oracle.bin_of_mode(lat.frequencies, nb, 0.0, lat.f_max)
    out = oracle.run_dense(E, m, v, W, bins, nb, corr_len=3)
    sv2 = synth.velocity_sigma(m[:1], 300.0)[0] ** 2
    nbins = np.bincount(bins, minlength=nb)
    C0 = out["corr"][0]                                   # [nb, 3, 3]
    for b in range(nb):
        if nbins[b] == 0:
            assert np.all(C0[b] == 0)
            continue
        prod = out["Jb"][:, :, b][:, :, None] * out["Jt"][:, None, :]
        se = prod.std(axis=0) / math.sqrt(S)
        want = np.eye(3) * sv2 * nbins[b]
        assert np.all(np.abs(C0[b] - want) < 5 * se + 1e-12)
        # lag 1: zero mean
        prod1 = out["Jb"][1:, :, b][:, :, None] * out["Jt"][:-1, None, :]
        se1 = prod1.std(axis=0) / math.sqrt(S - 1)
        assert np.all(np.abs(out["corr"][1][b]) < 5 * se1)
    # HNEMA average of zero-mean iid currents: mean 0, std sqrt(sv2 n_b / S)
    for b in range(nb):
        if nbins[b]:
            sd = math.sqrt(sv2 * nbins[b] / S)
            assert np.all(np.abs(out["hnema"][b]) < 5 * sd)


# ------------------------------------------------------------------ GKMA
def _series(S=40, nb=3, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((S, 3, nb)), rng.standard_normal((S, 3))


def test_gkma_sum_rule_eq18():
    lat, E, m, v, W, bins, nb = _case((4, 3, 2), S=30)
    out = oracle.run_dense(E, m, v, W, bins, nb, corr_len=8)
    np.testing.assert_allclose(out["corr"].sum(axis=1), out["hcacf"], rtol=1e-11, atol=1e-18)


def test_gkma_correlation_matches_fft_route():
    """Direct lag sums vs a zero-padded FFT cross-correlation (Wiener-Khinchin)."""
    Jb, Jt = _series(S=50, nb=2)
    L = 20
    C = oracle.gkma_correlation(Jb, Jt, L)
    S = Jb.shape[0]
    n = 2 * S
    Fb = np.fft.rfft(Jb, n=n, axis=0)
    Ft = np.fft.rfft(Jt, n=n, axis=0)
    for b in range(2):
        for mu in range(3):
            for nu in range(3):
                raw = np.fft.irfft(Fb[:, mu, b] * np.conj(Ft[:, nu]), n=n)[:L]
                np.testing.assert_allclose(C[:, b, mu, nu], raw / (S - np.arange(L)), rtol=1e-10, atol=1e-12)


def test_gkma_lag_direction_pulse():
    S, s0, s1 = 20, 12, 5
    Jb = np.zeros((S, 3, 1)); Jb[s0, 1, 0] = 1.0
    Jt = np.zeros((S, 3)); Jt[s1, 2] = 1.0
    C = oracle.gkma_correlation(Jb, Jt, 10)
    nz = np.argwhere(C != 0)
    assert nz.tolist() == [[s0 - s1, 0, 1, 2]]
    assert C[s0 - s1, 0, 1, 2] == 1.0 / (S - (s0 - s1))


def test_gkma_origin_count_normalisation():
    S = 9
    C = oracle.gkma_correlation(np.ones((S, 3, 2)), np.ones((S, 3)), 12)
    assert np.all(C[:S] == 1.0) and np.all(C[S:] == 0.0)


def test_trapezoid_integral_closed_form():
    tau0, w0, dt = 50.0, 0.07, 0.5
    t = np.arange(0, 400) * dt
    c = np.exp(-t / tau0) * np.cos(w0 * t)
    G = oracle.gkma_running_integral(c[:, None, None, None], dt)[:, 0, 0, 0]
    a = 1.0 / tau0
    exact = (a + np.exp(-a * t) * (w0 * np.sin(w0 * t) - a * np.cos(w0 * t))) / (a * a + w0 * w0)
    # trapezoid error bound: t * dt^2 / 12 * max|c''|
    bound = t * dt ** 2 / 12.0 * (a + w0) ** 2
    assert np.all(np.abs(G - exact) <= bound + 1e-15)


# --------------------------------------------------------------- binning
def test_bin_edges_ties_clamp_and_exclusion():
    nb, lo, hi = 4, 0.0, 8.0        # delta = 2
    f = np.array([0.0, 1.999, 2.0, np.nextafter(2.0, 0), 7.999, 8.0, -0.1, 8.1, 5.0])
    got = oracle.bin_of_mode(f, nb, lo, hi)
    np.testing.assert_array_equal(got, [0, 0, 1, 1, 3, 3, -1, -1, 2])
    assert np.all(oracle.bin_of_mode(f[:6], 1, lo, hi) == 0)


def test_bins_of_degenerate_modes_agree():
    """k, -k and axis permutations carry identical frequencies, hence bins."""
    lat = synth.BlochLattice((6, 6, 6))
    kf = lat.kpoint_frequencies()
    assert np.array_equal(kf, np.transpose(kf, (1, 0, 2)))
    assert np.array_equal(kf, np.transpose(kf, (2, 1, 0)))
    neg = kf[(-np.arange(6)) % 6][:, (-np.arange(6)) % 6][:, :, (-np.arange(6)) % 6]
    assert np.array_equal(kf, neg)
    b = oracle.bin_of_mode(lat.frequencies, 37, 0.0, lat.f_max)
    assert np.all(b[0::3] == b[1::3]) and np.all(b[1::3] == b[2::3])


def test_frequency_constants():
    lat = synth.BlochLattice((4, 4, 4))
    assert abs(lat.omega0 - 0.05861241) < 1e-8
    assert abs(lat.f_max - 32.31471) < 1e-5
    assert abs(lat.frequencies.max() - lat.f_max) < 1e-12
    assert len(np.unique(np.round(lat.frequencies, 9))) == 7
    assert abs(synth.velocity_sigma(np.array([28.0855]), 300.0)[0] - 2.980140e-3) < 1e-9


def test_kappa_prefactors_units():
    # 1 eV A/fs over (1 K * 1 A^3 * 1/A) = 1 eV/(fs A K) = 1.602176634e6 W/(m K)
    assert abs(oracle.hnema_kappa(1.0, 1.0, 1.0, 1.0) - 1.602176634e6) < 1e-3
    k = oracle.gkma_kappa(1.0, 300.0, 1000.0)
    assert abs(k - 1.602176634e6 / (8.617333262e-5 * 9e4 * 1e3)) < 1e-6


def test_streaming_equals_dense():
    lat, E, m, v, W, bins, nb = _case((4, 3, 2), S=17)
    dense = oracle.run_dense(E, m, v, W, bins, nb, corr_len=5, dt=0.5)
    so = oracle.StreamingOracle(lambda r0, n: lat.eig_rows(r0, n), m, bins, nb, corr_len=5, dt=0.5, row_chunk=13)
    for a, b in [(0, 5), (5, 6), (6, 17)]:
        so.push(v[a:b], W[a:b])
    got = so.read()
    for key in ("hnema", "hnema_total", "corr", "hcacf", "integral"):
        np.testing.assert_allclose(got[key], dense[key], rtol=1e-12, atol=1e-18)


# ------------------------------------------------------------- mutations
def _mut_virial_transposed(m, W):
    W = np.asarray(W, dtype=np.float64)
    S, N, _, _ = W.shape
    w = W / np.sqrt(m)[None, :, None, None]
    return np.ascontiguousarray(w.transpose(0, 3, 1, 2)).reshape(S, 3, 3 * N)


def test_mutation_transposed_virial_fails_golden():
    g, m, v, W = _two_atom_inputs()
    E = synth.BlochLattice((2, 1, 1)).eig_matrix()
    xdot = oracle.modal_velocity(E, oracle.mass_weighted_velocity(m, v))
    A = oracle.virial_projection(E, _mut_virial_transposed(m, W))
    Jb = oracle.binned_current(oracle.modal_heat_current(xdot, A), [0, 0, 0, 1, 1, 1], 2)[0]
    want = np.array([[_f(x) for x in r[1:]] for r in g["Jb"]])
    assert np.abs(Jb.T - want).max() > 0.1


def test_mutation_missing_sqrt_mass_fails_kinetic_energy():
    lat, E, m, v, W, bins, nb = _case((4, 3, 2))
    S, N, _ = v.shape
    xdot = oracle.modal_velocity(E, v.astype(np.float64).reshape(S, 3 * N))
    ke_atoms = 0.5 * (m[None, :, None] * v.astype(np.float64) ** 2).sum(axis=(1, 2))
    assert np.abs(0.5 * (xdot ** 2).sum(axis=1) / ke_atoms - 1).max() > 0.5


def test_mutation_transposed_basis_fails_round_trip():
    n_atoms = 8
    E = synth.random_orthonormal(3 * n_atoms, seed=4)
    m = synth.masses(n_atoms, "natural", 9)
    xdot = np.random.default_rng(2).standard_normal((3, 3 * n_atoms))
    v = ((E @ xdot.T).T).reshape(3, n_atoms, 3) / np.sqrt(m)[None, :, None]
    back = oracle.mass_weighted_velocity(m, v) @ E.T      # E instead of E^T
    assert np.abs(back - xdot).max() > 0.1


def test_mutation_swapped_lag_or_wrong_normalisation_fails_golden():
    g = _golden.read("gkma_lags.txt")
    Jb = np.array([_f(x) for x in g["Jb"][0]])
    Jt = np.array([_f(x) for x in g["Jt"][0]])
    want = np.array([_f(x) for x in g["corr"][0]])
    S, L = Jb.size, want.size
    swapped = [sum(Jt[s] * Jb[s - t] for s in range(t, S)) / (S - t) if t < S else 0 for t in range(L)]
    by_S = [sum(Jb[s] * Jt[s - t] for s in range(t, S)) / S if t < S else 0 for t in range(L)]
    assert np.abs(np.array(swapped) - want).max() > 0.1
    assert np.abs(np.array(by_S) - want).max() > 0.1


def test_mutation_rectangle_rule_fails_closed_form():
    tau0, w0, dt = 50.0, 0.07, 0.5
    t = np.arange(0, 400) * dt
    c = np.exp(-t / tau0) * np.cos(w0 * t)
    G = np.concatenate([[0.0], np.cumsum(c[:-1]) * dt])    # left rectangle
    a = 1.0 / tau0
    exact = (a + np.exp(-a * t) * (w0 * np.sin(w0 * t) - a * np.cos(w0 * t))) / (a * a + w0 * w0)
    bound = t * dt ** 2 / 12.0 * (a + w0) ** 2
    assert np.any(np.abs(G - exact) > bound + 1e-15)


def test_mutation_ties_down_fails_edge_test():
    f = np.array([2.0, np.nextafter(2.0, 0)])
    delta = 2.0
    down = [min(math.floor(x / delta), 3) for x in f]
    assert down != list(oracle.bin_of_mode(f, 4, 0.0, 8.0))
