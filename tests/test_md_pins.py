"""Pins of the oracle's NVE molecular dynamics (oracle.virial.md_nve; velocity
Verlet with the Tersoff forces, the paper's 1 fs production time step,
Sec. III.A), from properties the integrator must have rather than from its
own formulas:
  * second order: the total-energy error over the same 40 fs falls fourfold
    when the time step halves, and stays below 1e-4 eV per atom at 1 fs;
  * time reversibility: n steps, velocities reversed, n steps back to the
    start (to round-off);
  * momentum conservation (the forces sum to zero);
  * free flight: atoms out of each other's range move on straight lines,
    x(t) = x0 + v t (mod the box), at constant velocity;
mutations (a full kick in place of each half kick; the second half kick with
the old force) fail a pin each.  The NVT integrator with the HNEMD driving
force (oracle.virial.md_nvt_hnemd) is pinned at the end of the file."""
import numpy as np
import pytest

import synth
from oracle import virial as ov


def _case(seed=1):
    p = ov.tersoff_si()
    pos, box = synth.diamond((2, 2, 2), sigma=0.05, seed=seed)
    m = synth.masses(len(pos))
    return p, pos, box, m, synth.thermal_velocities(m, 300.0, seed + 1)


def _energy_error(run, dt, T=40.0):
    p, pos, box, m, v0 = _case()
    E = run(pos, v0, m, box, p, dt, int(round(T / dt)))["E"]
    return np.abs(E - E[0]).max() / len(pos)


def test_energy_error_is_second_order():
    e1, e2 = _energy_error(ov.md_nve, 1.0), _energy_error(ov.md_nve, 0.5)
    assert e1 < 1e-4
    assert 3.5 < e1 / e2 < 4.5, e1 / e2


def _reversal_error(run, n=30):
    p, pos, box, m, v0 = _case(3)
    r = run(pos, v0, m, box, p, 1.0, n)
    b = run(r["pos"][-1], -r["vel"][-1], m, box, p, 1.0, n)
    dx = np.abs(ov.min_image(b["pos"][-1] - np.mod(pos, box), box)).max()
    dv = np.abs(-b["vel"][-1] - v0).max()
    return dx, dv


def test_time_reversible():
    dx, dv = _reversal_error(ov.md_nve)
    assert dx < 1e-12 and dv < 1e-12


def test_momentum_conserved():
    p, pos, box, m, v0 = _case(5)
    r = ov.md_nve(pos, v0, m, box, p, 1.0, 20)
    P0 = (m[:, None] * v0).sum(axis=0)
    for v in r["vel"]:
        assert np.abs((m[:, None] * v).sum(axis=0) - P0).max() <= 1e-12 * np.abs(m[:, None] * v0).sum()


def test_free_flight():
    p = ov.tersoff_si()
    box = np.array([20.0, 21.0, 22.0])
    pos = np.array([[1.0, 2.0, 3.0], [11.0, 12.5, 14.0], [5.0, 17.0, 9.0]])   # > R + D apart, also across the walls
    m = np.array([28.0855, 27.9769, 29.9738])
    v0 = np.array([[0.01, -0.02, 0.005], [-0.03, 0.004, 0.02], [0.0, 0.05, -0.04]])
    n, dt = 400, 1.0
    r = ov.md_nve(pos, v0, m, box, p, dt, n)
    assert np.all(r["vel"] == v0) and np.all(r["W"] == 0.0)
    want = np.mod(pos + n * dt * v0, box)
    assert np.abs(ov.min_image(r["pos"][-1] - want, box)).max() < 1e-12
    assert np.all(r["E"] == r["E"][0])


def _mut_full_kicks(pos, vel, mass, box, p, dt, n_steps):
    """Euler-like: a full kick before and after the drift."""
    box = np.asarray(box, dtype=np.float64)
    x, v = np.mod(np.array(pos, dtype=float), box), np.array(vel, dtype=float)
    inv = 1.0 / (np.asarray(mass) * ov.KE_UNIT)
    out = {"pos": [], "vel": [], "E": []}
    nl = ov.neighbor_lists(x, box, p["R"] + p["D"])
    F = ov.forces(x, box, p, nl)
    out["E"].append(float(ov.site_energies(x, box, p, nl).sum() + 0.5 * (mass * (v * v).sum(1)).sum() * ov.KE_UNIT))
    for _ in range(n_steps):
        v = v + dt * F * inv[:, None]
        x = np.mod(x + dt * v, box)
        nl = ov.neighbor_lists(x, box, p["R"] + p["D"])
        F = ov.forces(x, box, p, nl)
        out["pos"].append(x)
        out["vel"].append(v)
        out["E"].append(float(ov.site_energies(x, box, p, nl).sum() + 0.5 * (mass * (v * v).sum(1)).sum() * ov.KE_UNIT))
    return {k: np.array(val) for k, val in out.items()}


def _mut_stale_force(pos, vel, mass, box, p, dt, n_steps):
    """The second half kick with the force of the old positions."""
    box = np.asarray(box, dtype=np.float64)
    x, v = np.mod(np.array(pos, dtype=float), box), np.array(vel, dtype=float)
    inv = 1.0 / (np.asarray(mass) * ov.KE_UNIT)
    out = {"pos": [], "vel": [], "E": [0.0]}
    F = ov.forces(x, box, p, ov.neighbor_lists(x, box, p["R"] + p["D"]))
    for _ in range(n_steps):
        v = v + 0.5 * dt * F * inv[:, None]
        x = np.mod(x + dt * v, box)
        v = v + 0.5 * dt * F * inv[:, None]
        F = ov.forces(x, box, p, ov.neighbor_lists(x, box, p["R"] + p["D"]))
        out["pos"].append(x)
        out["vel"].append(v)
        out["E"].append(0.0)
    return {k: np.array(val) for k, val in out.items()}


def test_mutations_fail():
    e1, e2 = _energy_error(_mut_full_kicks, 1.0), _energy_error(_mut_full_kicks, 0.5)
    assert not (e1 < 1e-4 and 3.5 < e1 / e2 < 4.5)
    dx, dv = _reversal_error(_mut_stale_force)
    assert dx > 1e-9 or dv > 1e-9


# ---------------------------------------------------------------------------
# NVT with the HNEMD driving force (oracle.virial.md_nvt_hnemd): pins from
# what the integrator must do, not from its formulas:
#   * no driving force and a thermostat too slow to act (tau -> infinity):
#     the NVE trajectory bit for bit;
#   * no driving force: the extended energy K + U + Q xi^2/2 + g k_B T eta is
#     a constant of the motion, its error second order in the time step;
#   * the driving force: Newton's third law makes the interatomic forces sum
#     to zero, so the total momentum changes only by the summed driving force,
#     F_e sum_i E_i + F_e . sum_i W_i, whose virial part is the total virial of
#     Eq. 5 (computed independently of the per-atom tensors);
#   * the thermostat pulls a hot start towards the set temperature.

def _nvt(dt, T_fs, fe=(0.0, 0.0, 0.0), temp=300.0, tau=20.0, v_temp=300.0, seed=1):
    p, pos, box, m, _ = _case(seed)
    v0 = synth.thermal_velocities(m, v_temp, seed + 1)
    return ov.md_nvt_hnemd(pos, v0, m, box, p, dt, int(round(T_fs / dt)), fe, temp, tau), (p, pos, box, m, v0)


def test_nvt_without_thermostat_or_drive_is_nve():
    out, (p, pos, box, m, v0) = _nvt(1.0, 10, tau=1e30)
    ref = ov.md_nve(pos, v0, m, box, p, 1.0, 10)
    assert np.array_equal(out["pos"], ref["pos"]) and np.array_equal(out["vel"], ref["vel"])
    assert np.all(np.abs(out["xi"]) < 1e-40)


def test_nvt_extended_energy_is_conserved_to_second_order():
    errs = []
    for dt in (1.0, 0.5):
        out, (_, pos, _, _, _) = _nvt(dt, 20, tau=10.0, v_temp=600.0)
        H = out["H"]
        errs.append(np.abs(H - H[0]).max() / len(pos))
    assert errs[0] < 5e-4                      # eV per atom, against a cohesive energy of about 4.6 eV
    assert 3.5 < errs[0] / errs[1] < 4.5, errs


def test_nvt_driving_force_moves_the_momentum_by_its_sum():
    fe = np.array([2e-3, -1e-3, 0.5e-3])
    out, (p, pos, box, m, v0) = _nvt(1.0, 20, fe=fe, tau=1e30)
    x = np.concatenate([[np.mod(pos, box)], out["pos"]])
    v = np.concatenate([[v0], out["vel"]])

    def drive(k):   # F_e sum_i E_i + F_e . (total virial, Eq. 5), at state k
        nl = ov.neighbor_lists(x[k], box, p["R"] + p["D"])
        E = float(ov.site_energies(x[k], box, p, nl).sum()) + 0.5 * float((m * (v[k] ** 2).sum(axis=1)).sum()) * ov.KE_UNIT
        return E * fe + fe @ ov.total_virial_eq5(x[k], box, p, nl)

    d = np.array([drive(k) for k in range(len(x))])
    dP_pred = (0.5 * (d[:-1] + d[1:])).sum(axis=0) * 1.0 / ov.KE_UNIT     # trapezoid over the steps, amu A/fs
    dP = (m[:, None] * (v[-1] - v[0])).sum(axis=0)
    assert np.abs(dP - dP_pred).max() < 2e-2 * np.abs(dP_pred).max(), (dP, dP_pred)
    # and with the drive reversed the momentum moves the other way
    out_r, _ = _nvt(1.0, 20, fe=-fe, tau=1e30)
    dP_r = (m[:, None] * (out_r["vel"][-1] - v[0])).sum(axis=0)
    assert np.abs(dP_r + dP).max() < 0.1 * np.abs(dP).max()


def test_nvt_thermostat_cools_a_hot_start():
    out, (_, _, _, m, _) = _nvt(1.0, 60, tau=10.0, v_temp=900.0)
    kin = 0.5 * (m[None, :, None] * out["vel"] ** 2).sum(axis=(1, 2)) * ov.KE_UNIT
    T_late = 2.0 * kin[30:].mean() / (3 * len(m) * ov.K_B)
    assert 150.0 < T_late < 500.0, T_late
