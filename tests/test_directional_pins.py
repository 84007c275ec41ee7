"""Pins of the direction-resolved oracle (Sec. II, remark after Eq. 10; closing
remark of Sec. II.C) against the hand-worked two-atom chain, the completeness
of the basis, the sum rule over motion directions and the polarisation
structure of a Bloch basis.  Mutation tests plant plausible mistakes in copies
of the oracle and show that a pin rejects each one."""
import numpy as np
import pytest

import oracle
import synth
from oracle import directional as od
from tests import _golden


def _two_atom():
    g = _golden.read("two_atom_chain.txt")
    m = np.array([float(x) for x in g["mass"][0]])
    v = np.zeros((1, 2, 3))
    for row in g["v"]:
        v[0, int(row[0])] = [float(x) for x in row[1:]]
    W = np.zeros((1, 2, 3, 3))
    for row in g["W"]:
        W[0, int(row[0]), "xyz".index(row[1])] = [float(x) for x in row[2:]]
    return g, m, v, W


def test_golden_total_split():
    g, m, v, W = _two_atom()
    want = np.array([[float(x) for x in r[1:]] for r in g["total_dir"]])
    got = od.total_heat_current_directional(v, W)[0]
    assert np.array_equal(got, want)
    assert np.array_equal(got.sum(axis=1), [float(x) for x in g["total"][0]])


def test_golden_modal_split_follows_polarisation():
    """On the chain's basis mode (f, alpha) moves the atoms along alpha only, so
    its whole current sits in motion direction nu = alpha (hand-worked J_n^mu)."""
    g, m, v, W = _two_atom()
    E = synth.BlochLattice((2, 1, 1)).eig_matrix()
    Jd = od.modal_currents_directional(E, m, v, W)[0]            # [mu, nu, M]
    want_Jn = np.array([[float(x) for x in r[1:]] for r in g["Jn"]])   # [M, mu]
    for n in range(6):
        for nu in range(3):
            expect = want_Jn[n] if nu == n % 3 else np.zeros(3)
            np.testing.assert_allclose(Jd[:, nu, n], expect, rtol=0, atol=1e-13)


def _dense_case(N=9, S=5, seed=4):
    E = synth.random_orthonormal(3 * N, seed=seed)
    m = synth.masses(N, "natural", seed)
    v, W = synth.gen_steps(seed, m, 0, S)
    return E, m, v, W


def test_completeness_gives_the_split_total():
    """Eq. 14 completeness: sum_n e_{i,n}^nu e_{j,n}^alpha = delta_ij delta_{nu alpha},
    so the split modal currents of a dense basis sum over modes to J^{mu nu}."""
    E, m, v, W = _dense_case()
    Jd = od.modal_currents_directional(E, m, v, W)
    np.testing.assert_allclose(Jd.sum(axis=3), od.total_heat_current_directional(v, W), rtol=1e-12, atol=1e-14)


def test_sum_over_motion_directions_is_eq16():
    E, m, v, W = _dense_case(seed=6)
    Jd = od.modal_currents_directional(E, m, v, W)
    np.testing.assert_allclose(Jd.sum(axis=2), oracle.modal_currents(E, m, v, W), rtol=1e-12, atol=1e-15)


def test_run_dense_outputs_sum_to_the_plain_outputs():
    lat = synth.BlochLattice((3, 2, 2))
    E = synth.random_orthonormal(3 * lat.n_atoms, seed=2)
    m = synth.masses(lat.n_atoms, "natural", 2)
    v, W = synth.gen_steps(2, m, 0, 7)
    bins = oracle.bin_of_mode(lat.frequencies, 5, 0.0, lat.f_max)
    d = od.run_dense_directional(E, m, v, W, bins, 5, corr_len=4, dt=0.5)
    p = oracle.run_dense(E, m, v, W, bins, 5, corr_len=4, dt=0.5)
    np.testing.assert_allclose(d["hnema_dir"].sum(axis=2), p["hnema"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(d["hnema_total_dir"].sum(axis=1), p["hnema_total"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(d["corr_dir"].sum(axis=3), p["corr"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(d["integral_dir"].sum(axis=3), p["integral"], rtol=1e-12, atol=1e-15)


def test_polarisation_bins_of_a_bloch_basis():
    """With bins = polarisation of the Bloch mode, bin alpha holds motion along
    alpha only: every other direction of its correlation is exactly zero."""
    lat = synth.BlochLattice((3, 2, 2))
    E = lat.eig_matrix()
    m = synth.masses(lat.n_atoms, "natural", 1)
    v, W = synth.gen_steps(1, m, 0, 6)
    bins = np.arange(lat.n_modes) % 3
    d = od.run_dense_directional(E, m, v, W, bins, 3, corr_len=3)
    p = oracle.run_dense(E, m, v, W, bins, 3, corr_len=3)
    for b in range(3):
        for nu in range(3):
            if nu != b:
                assert np.all(np.abs(d["corr_dir"][:, b, :, nu, :]) < 1e-15)
                assert np.all(np.abs(d["hnema_dir"][b, :, nu]) < 1e-15)
        np.testing.assert_allclose(d["corr_dir"][:, b, :, b, :], p["corr"][:, b], rtol=1e-12, atol=1e-15)


# ------------------------------------------------------------------ mutations
def _mut_wrong_dof(E, m, v, W):
    """Mask on the current direction mu instead of the motion direction nu."""
    xdot = oracle.modal_velocity(E, oracle.mass_weighted_velocity(m, v))
    S, N = v.shape[:2]
    out = np.zeros((S, 3, 3, E.shape[1]))
    inv = 1.0 / np.sqrt(m)
    for nu in range(3):
        w = np.zeros((S, 3, N, 3))
        for mu in range(3):
            w[:, mu, :, mu] = W[:, :, mu, nu] * inv[None, :]
        A = oracle.virial_projection(E, w.reshape(S, 3, 3 * N))
        out[:, :, nu, :] = A * xdot[:, None, :]
    return out


def _mut_transposed(E, m, v, W):
    return od.modal_currents_directional(E, m, v, np.swapaxes(W, 2, 3))


@pytest.mark.parametrize("mut", [_mut_wrong_dof, _mut_transposed])
def test_mutations_fail_completeness(mut):
    E, m, v, W = _dense_case()
    got = mut(E, m, v, W).sum(axis=3)
    assert not np.allclose(got, od.total_heat_current_directional(v, W), rtol=1e-6, atol=1e-9)


def test_mutation_transposed_total_fails_golden():
    g, m, v, W = _two_atom()
    want = np.array([[float(x) for x in r[1:]] for r in g["total_dir"]])
    assert not np.array_equal(od.total_heat_current_directional(v, np.swapaxes(W, 2, 3))[0], want)


def test_bench_plane_wave_split_reference_equals_dense_split():
    """The benchmark's direction-split reference (FFT form per polarisation: a
    plane-wave mode of polarisation nu moves atoms along nu only) equals the
    dense split oracle on the same lattice basis and bins."""
    import bench
    lat = synth.BlochLattice((3, 3, 2))
    m = synth.masses(lat.n_atoms)
    v, W = synth.gen_steps(3, m, 0, 16)
    nb = 7
    ref = bench.lattice_reference(lat, m, v, W, nb, 5, 0)
    bins = oracle.bin_of_mode(lat.frequencies, nb, 0.0, lat.f_max)
    d = od.run_dense_directional(lat.eig_matrix(), m, v, W, bins, nb, 0, 1.0)
    scale = np.abs(d["hnema_dir"]).max()
    assert scale > 0
    assert np.abs(ref["hnema_dir"] - d["hnema_dir"]).max() <= 1e-13 * scale
    assert np.abs(ref["hnema_dir"].sum(axis=2) - ref["hnema"]).max() <= 1e-13 * scale
