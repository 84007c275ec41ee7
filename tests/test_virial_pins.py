"""Pins of the per-atom virial oracle (oracle/virial.py; Sec. II.A, Eqs. 1-12)
against what the mathematics and the published potential fix, not against
the oracle itself:
  * the perfect diamond crystal: every site energy equals a scalar closed form
    of Tersoff's expression (four neighbours at a sqrt(3)/4, all angles with
    cos = -1/3), close to the -4.63 eV per atom Tersoff fitted for Si;
    forces vanish by symmetry;
  * partial derivatives dU_i/dr_ij against central finite differences of the
    site energy (with the exponential term switched on and atoms inside the
    cutoff's switching shell), forces against the gradient of the total energy;
  * the total virial of Eq. 8 summed over atoms equals Eq. 5 (pair forces of
    Eq. 4) and Eq. 2 summed, and equals minus the strain derivative of the
    energy; it is symmetric while the per-atom tensors are not;
  * the two-body limit (beta = 0): per-atom W of Eq. 8 equals Eq. 2 and is
    symmetric;
  * Eq. 9 equals Eq. 10 and Eq. 11 equals Eq. 12 (loops against the compact
    forms);
  * mutations (partials with the wrong atom, a dropped three-body term, the
    transposed virial in Eq. 10 or Eq. 12) each fail one of the pins.
"""
import math

import numpy as np
import pytest

import synth
from oracle import virial as ov


def _si():
    return ov.tersoff_si()


def _exp_on():
    """The Si parameters with the exponential term switched on (l3 = 1.3258, m = 3,
    Tersoff's 1988 Si(B) value of l3) so that its derivative is exercised."""
    p = ov.tersoff_si()
    p.update(lambda3=1.3258)
    return p


def _config(kind, seed=0):
    if kind == "displaced":
        return synth.diamond((2, 2, 2), sigma=0.08, seed=seed)
    if kind == "switching":
        # expanded lattice: nearest neighbours at 2.73 A, inside R - D < r < R + D
        return synth.diamond((2, 2, 2), a=6.3, sigma=0.04, seed=seed)
    raise ValueError(kind)


def test_perfect_diamond_closed_form_and_published_energy():
    p = _si()
    a = synth.SI_LATTICE_A
    pos, box = synth.diamond((2, 2, 2), a=a)
    U = ov.site_energies(pos, box, p, ov.neighbor_lists(pos, box, p["R"] + p["D"]))
    # closed form of one site: 4 bonds of length r, each with 3 other bonds at cos = -1/3
    r = a * math.sqrt(3.0) / 4.0
    t = -1.0 / 3.0 - p["h"]
    g = 1.0 + p["c"] ** 2 / p["d"] ** 2 - p["c"] ** 2 / (p["d"] ** 2 + t * t)
    zeta = 3.0 * g
    b = (1.0 + (p["beta"] * zeta) ** p["n"]) ** (-1.0 / (2.0 * p["n"]))
    u = 0.5 * 4.0 * (p["A"] * math.exp(-p["lambda1"] * r) - b * p["B"] * math.exp(-p["lambda2"] * r))
    np.testing.assert_allclose(U, u, rtol=1e-13, atol=0)
    assert abs(u - (-4.63)) < 0.01          # Tersoff's fitted cohesive energy of diamond Si


def test_perfect_diamond_forces_vanish():
    p = _si()
    pos, box = synth.diamond((2, 2, 2))
    nl = ov.neighbor_lists(pos, box, p["R"] + p["D"])
    assert all(len(x) == 4 for x in nl)
    F = ov.forces(pos, box, p, nl)
    assert np.abs(F).max() < 1e-11


def _fd_site_partial(pos, box, p, nl, i, j, h=1e-5):
    """dU_i/dr_ij by central differences of U_i in the position of j (only r_ij changes)."""
    g = np.zeros(3)
    for a in range(3):
        pp, pm = pos.copy(), pos.copy()
        pp[j, a] += h
        pm[j, a] -= h
        g[a] = (ov.site_energies(pp, box, p, nl)[i] - ov.site_energies(pm, box, p, nl)[i]) / (2 * h)
    return g


@pytest.mark.parametrize("kind,params", [("displaced", _si), ("switching", _si), ("displaced", _exp_on),
                                         ("switching", _exp_on)])
def test_partials_match_finite_differences(kind, params):
    p = params()
    pos, box = _config(kind, seed=3)
    nl = ov.neighbor_lists(pos, box, p["R"] + p["D"])
    Dp = ov.site_energy_partials(pos, box, p, nl)
    rng = np.random.default_rng(5)
    scale = max(np.abs(d).max() for d in Dp if len(d))
    for i in rng.choice(len(nl), size=5, replace=False):
        for s, j in enumerate(nl[i][:3]):
            fd = _fd_site_partial(pos, box, p, nl, i, j)
            np.testing.assert_allclose(Dp[i][s], fd, rtol=0, atol=2e-8 * scale)


def test_switching_shell_is_exercised():
    p = _si()
    pos, box = _config("switching", seed=3)
    r = [np.linalg.norm(ov.min_image(pos[j] - pos[i], box)) for i in range(8) for j in
         ov.neighbor_lists(pos, box, p["R"] + p["D"])[i]]
    inside = [x for x in r if p["R"] - p["D"] < x < p["R"] + p["D"]]
    assert len(inside) >= len(r) // 2 and max(r) < p["R"] + p["D"]


def test_forces_are_minus_the_energy_gradient():
    p = _exp_on()
    pos, box = _config("displaced", seed=4)
    nl = ov.neighbor_lists(pos, box, p["R"] + p["D"])
    F = ov.forces(pos, box, p, nl)
    h = 1e-5
    for i in (0, 17, 45):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, a] += h
            pm[i, a] -= h
            g = (ov.site_energies(pp, box, p, nl).sum() - ov.site_energies(pm, box, p, nl).sum()) / (2 * h)
            assert abs(F[i, a] + g) < 2e-8 * np.abs(F).max()
    assert np.abs(F.sum(axis=0)).max() < 1e-10 * np.abs(F).max()   # translation invariance


@pytest.mark.parametrize("kind", ["displaced", "switching"])
def test_total_virial_eq8_equals_eq5_and_eq2(kind):
    p = _exp_on()
    pos, box = _config(kind, seed=6)
    nl = ov.neighbor_lists(pos, box, p["R"] + p["D"])
    W = ov.per_atom_virial(pos, box, p, nl)
    W5 = ov.total_virial_eq5(pos, box, p, nl)
    W2 = ov.per_atom_virial_eq2(pos, box, p, nl)
    s = np.abs(W5).max()
    np.testing.assert_allclose(W.sum(axis=0), W5, rtol=0, atol=1e-12 * s)
    np.testing.assert_allclose(W2.sum(axis=0), W5, rtol=0, atol=1e-12 * s)
    # many-body: the per-atom tensors are not symmetric and differ from Eq. 2, the total is symmetric
    asym = np.abs(W - W.transpose(0, 2, 1)).max() / np.abs(W).max()
    assert asym > 1e-2
    assert np.abs(W - W2).max() > 1e-2 * np.abs(W).max()
    np.testing.assert_allclose(W5, W5.T, rtol=0, atol=1e-12 * s)


def _strain_energy(pos, box, p, nl, mu, eps):
    q, b = pos.copy(), box.copy()
    q[:, mu] *= 1.0 + eps
    b[mu] *= 1.0 + eps
    return ov.site_energies(q, b, p, nl).sum()


def test_total_virial_is_minus_the_strain_derivative():
    """r -> (1 + eps) r along axis mu: dE/deps = sum_j sum_i r_ji^mu (dU_j/dr_ji)^mu = -W^{mu mu}."""
    p = _exp_on()
    pos, box = _config("displaced", seed=7)
    nl = ov.neighbor_lists(pos, box, p["R"] + p["D"])
    W = ov.per_atom_virial(pos, box, p, nl).sum(axis=0)
    h = 1e-6
    for mu in range(3):
        d = (_strain_energy(pos, box, p, nl, mu, h) - _strain_energy(pos, box, p, nl, mu, -h)) / (2 * h)
        assert abs(d + W[mu, mu]) < 1e-6 * np.abs(W).max()


def test_two_body_limit_per_atom_virial_is_eq2_and_symmetric():
    p = _si()
    p.update(beta=0.0)          # b_ij = 1: a pair potential
    pos, box = _config("switching", seed=8)
    nl = ov.neighbor_lists(pos, box, p["R"] + p["D"])
    W = ov.per_atom_virial(pos, box, p, nl)
    W2 = ov.per_atom_virial_eq2(pos, box, p, nl)
    s = np.abs(W).max()
    np.testing.assert_allclose(W, W2, rtol=0, atol=1e-13 * s)
    np.testing.assert_allclose(W, W.transpose(0, 2, 1), rtol=0, atol=1e-13 * s)
    # pair closed form of the site energy
    U = ov.site_energies(pos, box, p, nl)
    for i in (0, 9):
        acc = 0.0
        for j in nl[i]:
            r = np.linalg.norm(ov.min_image(pos[j] - pos[i], box))
            fc, _ = ov.cutoff_fn(r, p["R"], p["D"])
            acc += 0.5 * fc * (p["A"] * math.exp(-p["lambda1"] * r) - p["B"] * math.exp(-p["lambda2"] * r))
        assert abs(U[i] - acc) < 1e-13 * abs(acc)


def test_eq9_equals_eq10_and_eq11_equals_eq12():
    p = _exp_on()
    pos, box = _config("switching", seed=9)
    nl = ov.neighbor_lists(pos, box, p["R"] + p["D"])
    m = synth.masses(len(nl), "natural", 1)
    v = synth.thermal_velocities(m, 300.0, 2)
    W = ov.per_atom_virial(pos, box, p, nl)
    J9 = ov.heat_current_eq9(pos, box, v, p, nl)
    J10 = ov.heat_current_eq10(W, v)
    np.testing.assert_allclose(J10, J9, rtol=0, atol=1e-13 * np.abs(J9).max())
    U = ov.site_energies(pos, box, p, nl)
    E = ov.atom_energies(U, m, v)
    fe = np.array([2e-4, -1e-4, 5e-5])
    F11 = ov.hnemd_force_eq11(pos, box, E, fe, p, nl)
    F12 = ov.hnemd_force_eq12(E, W, fe)
    np.testing.assert_allclose(F12, F11, rtol=0, atol=1e-13 * np.abs(F11).max())
    # the kinetic part of E_i: m v^2 / 2 in eV (1 amu A^2/fs^2 = 103.6427 eV)
    assert abs(ov.KE_UNIT - 103.642697) < 1e-6


def test_evaluate_bundles_the_same_quantities():
    p = _si()
    pos, box = _config("displaced", seed=10)
    m = synth.masses(len(pos))
    v = synth.thermal_velocities(m, 300.0, 3)
    fe = np.array([1e-4, 0.0, 0.0])
    out = ov.evaluate(pos, box, v, m, fe, p)
    nl = out["nl"]
    np.testing.assert_array_equal(out["W"], ov.per_atom_virial(pos, box, p, nl))
    np.testing.assert_array_equal(out["Fext"], ov.hnemd_force_eq12(out["E"], out["W"], fe))


def test_sampled_atoms_equal_the_whole_system():
    """evaluate_atoms (each atom on its own, for sampling large systems) gives the
    same bits as the whole-system functions."""
    p = _exp_on()
    pos, box = synth.diamond((3, 3, 3), sigma=0.08, seed=2)
    m = synth.masses(len(pos), "natural", 1)
    v = synth.thermal_velocities(m, 300.0, 1)
    fe = np.array([1e-4, 2e-5, -3e-5])
    full = ov.evaluate(pos, box, v, m, fe, p)
    idx = [0, 7, 100, 215]
    sub = ov.evaluate_atoms(pos, box, v, m, fe, p, idx)
    for k in ("U", "F", "W", "Fext"):
        np.testing.assert_array_equal(sub[k], full[k][idx])


# ------------------------------------------------------------------ mutations
def test_mutation_partials_of_the_wrong_atom_fail_the_strain_pin():
    """Using dU_i/dr_ij in place of dU_j/dr_ji flips the sign of the total (Eq. 6)."""
    p = _exp_on()
    pos, box = _config("displaced", seed=7)
    nl = ov.neighbor_lists(pos, box, p["R"] + p["D"])
    Dp = ov.site_energy_partials(pos, box, p, nl)
    Wbad = np.zeros((3, 3))
    for i in range(len(nl)):
        for s, j in enumerate(nl[i]):
            Wbad += np.outer(ov.min_image(pos[j] - pos[i], box), Dp[i][s])
    h = 1e-6
    d = (_strain_energy(pos, box, p, nl, 0, h) - _strain_energy(pos, box, p, nl, 0, -h)) / (2 * h)
    assert abs(d + Wbad[0, 0]) > 1e-2 * abs(d)


def test_mutation_dropped_three_body_term_fails_finite_differences():
    p = _si()
    pos, box = _config("displaced", seed=3)
    nl = ov.neighbor_lists(pos, box, p["R"] + p["D"])
    # partials of the bond-order-free bracket only (the b_ij derivative dropped)
    i, s = 5, 0
    j = nl[i][s]
    _, b, _ = ov.bond_terms(pos, box, p, nl)
    rv = ov.min_image(pos[j] - pos[i], box)
    r = np.linalg.norm(rv)
    fc, dfc = ov.cutoff_fn(r, p["R"], p["D"])
    fr, fa = p["A"] * math.exp(-p["lambda1"] * r), p["B"] * math.exp(-p["lambda2"] * r)
    bad = 0.5 * (dfc * (fr - b[i][s] * fa) + fc * (-p["lambda1"] * fr + p["lambda2"] * b[i][s] * fa)) * rv / r
    fd = _fd_site_partial(pos, box, p, nl, i, j)
    assert np.abs(bad - fd).max() > 1e-3 * np.abs(fd).max()


def test_mutation_transposed_virial_fails_eq9_and_eq11():
    p = _exp_on()
    pos, box = _config("switching", seed=9)
    nl = ov.neighbor_lists(pos, box, p["R"] + p["D"])
    m = synth.masses(len(nl))
    v = synth.thermal_velocities(m, 300.0, 2)
    W = ov.per_atom_virial(pos, box, p, nl)
    J9 = ov.heat_current_eq9(pos, box, v, p, nl)
    assert np.abs(ov.heat_current_eq10(W.transpose(0, 2, 1), v) - J9).max() > 1e-3 * np.abs(J9).max()
    E = ov.atom_energies(ov.site_energies(pos, box, p, nl), m, v)
    fe = np.array([2e-4, -1e-4, 5e-5])
    F11 = ov.hnemd_force_eq11(pos, box, E, fe, p, nl)
    Fbad = E[:, None] * fe[None, :] + np.einsum("imn,n->im", W, fe)
    assert np.abs(Fbad - F11).max() > 1e-3 * np.abs(F11 - E[:, None] * fe[None, :]).max()


def test_package_parameters_are_the_published_ones():
    """The package's tersoff_si() (what users pass to ModalVirial) holds the same
    published numbers as the oracle's, each written from Tersoff's paper."""
    from paper_2102_03691_amd.physics import tersoff_si
    assert tersoff_si() == ov.tersoff_si()
