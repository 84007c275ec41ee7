"""Pins of the SHC oracle (Sec. II.C, Eqs. 20-23) against the hand-worked
fixture, brute force, the Eq. 10 sum rule and closed forms of the transform.
Mutation tests plant a plausible mistake in a copy of the oracle and show
that a pin rejects it."""
import math

import numpy as np
import pytest

import oracle
from oracle import shc as osh
from tests import _golden


def _fixture():
    g = _golden.read("shc_two_atoms.txt")
    S = 3
    v = np.zeros((S, 2, 3))
    W = np.zeros((S, 2, 3, 3))
    W[:, 0, 0, 1] = [float(x) for x in g["W0xy"][0]]
    v[:, 0, 0] = [float(x) for x in g["v0x"][0]]
    v[:, 0, 1] = [float(x) for x in g["v0y"][0]]
    W[:, 1, 2, 0] = [float(x) for x in g["W1zx"][0]]
    v[:, 1, 0] = [float(x) for x in g["v1x"][0]]
    K = np.array([[float(x) for x in g[k][0]] for k in ("Kx", "Ky", "Kz")]).T      # [tau, mu]
    spec = {k: np.array([float(x) for x in g[k][0]]) for k in ("spec_w0", "spec_wpi2", "spec_hann_w0")}
    return v, W, K, spec


def test_golden_correlation_and_transform():
    v, W, K, spec = _fixture()
    got = oracle.shc_correlation(v, W, 3)
    assert np.allclose(got, K, rtol=0, atol=1e-15)
    assert np.allclose(oracle.shc_spectrum(got, 1.0, [0.0])[0], spec["spec_w0"], atol=1e-15)
    assert np.allclose(oracle.shc_spectrum(got, 1.0, [math.pi / 2])[0], spec["spec_wpi2"], atol=1e-14)
    assert np.allclose(oracle.shc_spectrum(got, 1.0, [0.0], window=True)[0], spec["spec_hann_w0"], atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1])
def test_brute_force_loops(seed):
    rng = np.random.default_rng(seed)
    S, N, L = 6, 3, 8            # more lags than samples: the last ones have no origin
    v = rng.standard_normal((S, N, 3))
    W = rng.standard_normal((S, N, 3, 3))
    a = oracle.shc_correlation(v, W, L)
    b = osh.shc_correlation_loops(v.tolist(), W.tolist(), L)
    assert np.allclose(a, b, rtol=1e-13, atol=1e-15)
    assert np.all(a[S:] == 0.0)


def test_zero_lag_is_the_eq10_current_time_average():
    """The paper: Eq. 21 reduces to the heat current of Eq. 10 at t = 0."""
    rng = np.random.default_rng(3)
    S, N = 40, 17
    v = rng.standard_normal((S, N, 3))
    W = rng.standard_normal((S, N, 3, 3))
    K = oracle.shc_correlation(v, W, 5)
    Jt = oracle.total_heat_current(v, W)                 # [S, 3], Eq. 10 per step
    assert np.allclose(K[0], Jt.mean(axis=0), rtol=1e-13, atol=1e-14)


def test_lag_direction_pulse():
    """A virial at step 2 and a velocity at step 5 correlate at lag 3 only."""
    S, N = 8, 1
    v = np.zeros((S, N, 3))
    W = np.zeros((S, N, 3, 3))
    W[2, 0, 1, 2] = 1.5          # W^{yz}
    v[5, 0, 2] = 2.0             # v^z
    K = oracle.shc_correlation(v, W, 6)
    expect = np.zeros((6, 3))
    expect[3, 1] = 1.5 * 2.0 / (S - 3)
    assert np.array_equal(K, expect)


def test_transform_of_a_delta_is_flat():
    K = np.zeros((9, 3))
    K[0] = [1.0, -2.0, 0.5]
    om = np.linspace(0.0, 3.0, 7)
    out = oracle.shc_spectrum(K, 0.5, om)
    assert np.allclose(out, 0.5 * K[0][None, :], rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", [2, 5, 64])
def test_transform_of_a_constant_closed_form(n):
    """K = 1 on n lags: trapezoid of the even extension = Dirichlet kernel minus
    the half-weighted end points, dt [sin((n - 1/2) x) / sin(x / 2) - cos((n - 1) x)],
    x = omega dt; at omega = 0 it is 2 (n - 1) dt.  With the Hann window the
    omega = 0 value is (n - 1) dt."""
    dt = 0.7
    K = np.ones((n, 3))
    om = np.array([0.0, 0.3, 1.1, 2.9])
    got = oracle.shc_spectrum(K, dt, om)[:, 0]
    x = om * dt
    with np.errstate(invalid="ignore", divide="ignore"):
        d = np.where(x == 0, 2 * n - 1, np.sin((n - 0.5) * x) / np.sin(x / 2))
    expect = dt * (d - np.cos((n - 1) * x))
    assert np.allclose(got, expect, rtol=1e-12, atol=1e-12)
    assert math.isclose(got[0], 2 * (n - 1) * dt, rel_tol=1e-14)
    hann = oracle.shc_spectrum(K, dt, [0.0], window=True)[0, 0]
    assert math.isclose(hann, (n - 1) * dt, rel_tol=1e-13, abs_tol=1e-13)


def test_kappa_prefactor():
    Kw = np.array([[2.0, 4.0, 6.0]])
    assert np.allclose(oracle.shc_kappa(Kw, 10.0, 300.0, 0.5), 2 * Kw / (10.0 * 300.0 * 0.5))


# ------------------------------------------------------------------ mutations
def _mut_transposed(v, W, n):
    return oracle.shc_correlation(v, np.swapaxes(W, 2, 3), n)


def _mut_virial_late(v, W, n):
    S = v.shape[0]
    K = np.zeros((n, 3))
    for tau in range(min(n, S)):
        K[tau] = np.tensordot(W[tau:], v[: S - tau], axes=([0, 1, 3], [0, 1, 2])) / (S - tau)
    return K


def _mut_norm_S(v, W, n):
    S = v.shape[0]
    return oracle.shc_correlation(v, W, n) * (S - np.arange(n))[:, None] / S


@pytest.mark.parametrize("mut", [_mut_transposed, _mut_virial_late, _mut_norm_S])
def test_mutations_fail_the_golden(mut):
    v, W, K, _ = _fixture()
    assert not np.allclose(mut(v, W, 3), K, atol=1e-12)


def test_mutation_rectangle_rule_fails_the_closed_form():
    n, dt = 5, 1.0
    K = np.ones((n, 3))
    c = np.full(n, 2.0)
    c[0] = 1.0                                       # end point weighted 2, not 1
    rect = dt * (np.cos(np.outer([0.0], np.arange(n)) * dt) * c) @ K
    assert not math.isclose(rect[0, 0], 2 * (n - 1) * dt)


def test_package_shc_kappa_units():
    """1 eV A over 1 A^3, 1 K, 1/A: 2 eV/(A K) = 3.204e-9 J/(m K) per hertz of
    f; times 1e12 per THz."""
    from paper_2102_03691_amd.physics import shc_kappa
    assert math.isclose(shc_kappa(1.0, 1.0, 1.0, 1.0), 2 * 1.602176634e-9 * 1e12, rel_tol=1e-15)


def test_package_shc_kappa_sum_rule():
    """The spectral kappa integrates over f to the HNEMD total: Eq. 21 at lag 0
    is the time average of the Eq. 10 current, so int_0^{f_Nyquist} kappa(f) df
    equals hnema_kappa(K(0)) (Eq. 19 with the same T, V, F_e).  K is an
    exponential sampled every fs; the transform of the sampled lags has
    int_0^{pi/dt} K~ d omega / pi = c_0 K(0) exactly, and a trapezoid over
    omega with N panels integrates cos(omega tau dt) exactly for tau < 2N."""
    from paper_2102_03691_amd.physics import hnema_kappa, shc_kappa
    dt, n, T, V, Fe = 1.0, 400, 300.0, 1.7e4, 2e-4
    K = np.exp(-np.arange(n) / 37.0)[:, None] * np.array([[0.8, -0.1, 0.05]])
    n_panels = 4000
    omega = np.linspace(0.0, np.pi / dt, n_panels + 1)          # rad per fs, up to Nyquist
    Kw = oracle.shc_spectrum(K, dt, omega)
    f_thz = omega / (2 * np.pi) * 1e3                           # 1/fs -> THz
    dens = shc_kappa(Kw, T, V, Fe)
    total = ((dens[1:] + dens[:-1]) * 0.5 * np.diff(f_thz)[:, None]).sum(axis=0)
    assert np.allclose(total, hnema_kappa(K[0], T, V, Fe), rtol=1e-11, atol=0)


# ------------------------------------------------------- motion-direction split
def test_golden_directional_split():
    """The fixture's only virial entries are W_0^{xy} and W_1^{zx}: K^x comes from
    atom 0 moving along y and K^z from atom 1 moving along x; every other
    (mu, nu) pair is zero, although v_0^x is nonzero."""
    v, W, K, _ = _fixture()
    Kd = oracle.shc_correlation_directional(v, W, 3)
    expect = np.zeros((3, 3, 3))
    expect[:, 0, 1] = K[:, 0]
    expect[:, 2, 0] = K[:, 2]
    assert np.allclose(Kd, expect, rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", [2, 3])
def test_directional_sums_to_eq21_and_matches_loops(seed):
    rng = np.random.default_rng(seed)
    S, N, L = 7, 4, 9
    v = rng.standard_normal((S, N, 3))
    W = rng.standard_normal((S, N, 3, 3))
    Kd = oracle.shc_correlation_directional(v, W, L)
    assert np.allclose(Kd.sum(axis=2), oracle.shc_correlation(v, W, L), rtol=1e-13, atol=1e-15)
    # brute force per direction: only the nu column of W and the nu component of v
    for nu in range(3):
        Wn = np.zeros_like(W)
        Wn[:, :, :, nu] = W[:, :, :, nu]
        assert np.allclose(Kd[:, :, nu], osh.shc_correlation_loops(v.tolist(), Wn.tolist(), L), rtol=1e-13, atol=1e-15)


def test_mutation_directional_wrong_velocity_component_fails_golden():
    v, W, K, _ = _fixture()
    S = v.shape[0]
    bad = np.zeros((3, 3, 3))
    for tau in range(3):
        # velocity component mu instead of nu
        bad[tau] = np.einsum("simn,sim->mn", W[: S - tau], v[tau:]) / (S - tau)
    expect = np.zeros((3, 3, 3))
    expect[:, 0, 1] = K[:, 0]
    expect[:, 2, 0] = K[:, 2]
    assert not np.allclose(bad, expect, atol=1e-12)
