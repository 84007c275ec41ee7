"""Per-atom virial, heat current and HNEMD driving force of a many-body
potential (Sec. II.A, Eqs. 1-12): the plain FP64 oracle.

TEST INFRASTRUCTURE ONLY (see oracle.modal): imported by the tests, the
package smoke check and the benchmark's oracle leg, never by the library.

What the paper fixes (Sec. II.A):
  * the potential is a sum of site energies, U = sum_i U_i, and U_i depends on
    the relative positions r_ij = r_j - r_i (Eq. 3) of atom i's neighbours;
  * the force on i is sum_j F_ij with F_ij = dU_i/dr_ij - dU_j/dr_ji (Eq. 4);
  * the per-atom virial is W_i = sum_{j != i} r_ij (x) dU_j/dr_ji (Eq. 8), i.e.
    W_i^{mu nu} = sum_j r_ij^mu (dU_j/dr_ji)^nu, and it sums to the total
    virial of Eq. 5 (written with the pair forces of Eq. 4);
  * the potential part of the per-atom heat current is
    J_i = sum_j r_ij (dU_j/dr_ji . v_i) (Eq. 9) = W_i v_i (Eq. 10);
  * the HNEMD driving force is
    F_i^ext = E_i F_e + sum_j (dU_j/dr_ji (x) r_ij) . F_e (Eq. 11)
            = E_i F_e + F_e . W_i (Eq. 12), E_i the total energy of atom i.

The site energies are those of Tersoff's bond-order potential (Phys. Rev. B
38, 9902 (1988); the paper's "original Tersoff" for Si, Sec. III.A):
  U_i  = 1/2 sum_{j != i} f_C(r_ij) [A exp(-l1 r_ij) - b_ij B exp(-l2 r_ij)]
  b_ij = (1 + beta^n zeta_ij^n)^(-1/(2n))
  zeta_ij = sum_{k != i, j} f_C(r_ik) g(cos theta_ijk) exp(l3^m (r_ij - r_ik)^m)
  g(c) = gamma (1 + c0^2/d^2 - c0^2 / (d^2 + (c - h)^2))          (c0: the "c" parameter)
  f_C(r) = 1 below R - D, 1/2 - 1/2 sin(pi/2 (r - R)/D) inside, 0 above R + D,
where cos theta_ijk is the angle between r_ij and r_ik.  U_i depends only on
the vectors r_ij of atom i's neighbours, which is what Eq. 8 needs; its
partials dU_i/dr_ij are written out below by the chain rule, with every
r_ij treated as an independent variable.

Periodic orthorhombic box, minimum image (the box must exceed twice the
cutoff R + D).  Units: A, eV, amu, fs (1 amu A^2/fs^2 = KE_UNIT eV).
Everything is float64; loops are plain Python over atoms and neighbours.
"""
from __future__ import annotations

import math

import numpy as np

# 1 amu * (A/fs)^2 in eV, from CODATA: 1.66053906660e-27 kg * 1e10 m^2/s^2 / 1.602176634e-19 J
KE_UNIT = 1.66053906660e-27 * 1e10 / 1.602176634e-19


def tersoff_si() -> dict:
    """Tersoff's published parameters for silicon (Si(C) of the 1988 paper)."""
    return dict(A=1830.8, B=471.18, lambda1=2.4799, lambda2=1.7322, lambda3=0.0, m=3, beta=1.1e-6, n=0.78734,
                c=1.0039e5, d=16.217, h=-0.59825, gamma=1.0, R=2.85, D=0.15)


def min_image(d: np.ndarray, box) -> np.ndarray:
    box = np.asarray(box, dtype=np.float64)
    return d - box * np.round(d / box)


def neighbor_lists(pos, box, cutoff: float):
    """For each atom i the ascending list of j != i with |r_ij| < cutoff (brute force)."""
    pos = np.asarray(pos, dtype=np.float64)
    out = []
    for i in range(pos.shape[0]):
        r = np.linalg.norm(min_image(pos - pos[i], box), axis=1)
        out.append([int(j) for j in np.nonzero(r < cutoff)[0] if j != i])
    return out


def cutoff_fn(r: float, R: float, D: float):
    """f_C and its derivative d f_C / d r."""
    if r < R - D:
        return 1.0, 0.0
    if r > R + D:
        return 0.0, 0.0
    x = 0.5 * math.pi * (r - R) / D
    return 0.5 - 0.5 * math.sin(x), -0.25 * math.pi / D * math.cos(x)


def angle_fn(c: float, p):
    """g(cos theta) and dg / d cos theta."""
    c0sq, dsq = p["c"] ** 2, p["d"] ** 2
    t = c - p["h"]
    den = dsq + t * t
    return p["gamma"] * (1.0 + c0sq / dsq - c0sq / den), p["gamma"] * c0sq * 2.0 * t / (den * den)


def exp_fn(x: float, p):
    """exp(l3^m x^m) and its derivative in x."""
    m, l3 = p["m"], p["lambda3"]
    e = math.exp((l3 ** m) * (x ** m))
    return e, e * m * (l3 ** m) * (x ** (m - 1))


def _vec(pos, box, i, j):
    return min_image(np.asarray(pos[j], dtype=np.float64) - np.asarray(pos[i], dtype=np.float64), box)


def _bond_terms_one(pos, box, p, i, js):
    """zeta_ij, b_ij and db_ij/dzeta_ij for the neighbours js of atom i."""
    rv = [_vec(pos, box, i, j) for j in js]
    rn = [float(np.linalg.norm(x)) for x in rv]
    zi, bi, dbi = [], [], []
    for s in range(len(js)):
        z = 0.0
        for q in range(len(js)):
            if q == s:
                continue
            fc, _ = cutoff_fn(rn[q], p["R"], p["D"])
            cos = float(rv[s] @ rv[q]) / (rn[s] * rn[q])
            g, _ = angle_fn(cos, p)
            e, _ = exp_fn(rn[s] - rn[q], p)
            z += fc * g * e
        n, beta = p["n"], p["beta"]
        bz = (beta * z) ** n
        bb = (1.0 + bz) ** (-0.5 / n)
        # d b / d zeta = -1/2 beta^n zeta^(n-1) (1 + (beta zeta)^n)^(-1/(2n) - 1), zero at zeta = 0
        dbb = 0.0 if z == 0.0 else -0.5 * bz / z * (1.0 + bz) ** (-0.5 / n - 1.0)
        zi.append(z)
        bi.append(bb)
        dbi.append(dbb)
    return zi, bi, dbi


def bond_terms(pos, box, p, nl):
    """zeta_ij, b_ij and db_ij/dzeta_ij for every neighbour j of every atom i:
    lists indexed [i][s] for j = nl[i][s]."""
    out = [_bond_terms_one(pos, box, p, i, nl[i]) for i in range(len(nl))]
    return [o[0] for o in out], [o[1] for o in out], [o[2] for o in out]


def _site_energy_one(pos, box, p, i, js):
    _, b, _ = _bond_terms_one(pos, box, p, i, js)
    acc = []
    for s, j in enumerate(js):
        r = float(np.linalg.norm(_vec(pos, box, i, j)))
        fc, _ = cutoff_fn(r, p["R"], p["D"])
        acc.append(fc * (p["A"] * math.exp(-p["lambda1"] * r) - b[s] * p["B"] * math.exp(-p["lambda2"] * r)))
    return 0.5 * math.fsum(acc)


def site_energies(pos, box, p, nl) -> np.ndarray:
    """U_i of the Tersoff form above, [N]."""
    return np.array([_site_energy_one(pos, box, p, i, nl[i]) for i in range(len(nl))], dtype=np.float64)


def _site_partials_one(pos, box, p, i, js) -> np.ndarray:
    """dU_i/dr_ij for the neighbours js of atom i, [len(js), 3] (see site_energy_partials)."""
    _, b, db = _bond_terms_one(pos, box, p, i, js)
    nj = len(js)
    rv = [_vec(pos, box, i, j) for j in js]
    rn = [float(np.linalg.norm(x)) for x in rv]
    fc = [cutoff_fn(r, p["R"], p["D"]) for r in rn]
    a = [fc[q][0] * p["B"] * math.exp(-p["lambda2"] * rn[q]) for q in range(nj)]

    def dcos_drij(s, q):
        # derivative of cos theta between r_s and r_q with respect to r_s
        c = float(rv[s] @ rv[q]) / (rn[s] * rn[q])
        return rv[q] / (rn[s] * rn[q]) - c * rv[s] / (rn[s] ** 2), c

    D = np.zeros((nj, 3))
    for s in range(nj):
        r, u = rn[s], rv[s] / rn[s]
        fcs, dfcs = fc[s]
        fr, dfr = p["A"] * math.exp(-p["lambda1"] * r), -p["lambda1"] * p["A"] * math.exp(-p["lambda1"] * r)
        fa, dfa = p["B"] * math.exp(-p["lambda2"] * r), -p["lambda2"] * p["B"] * math.exp(-p["lambda2"] * r)
        grad = 0.5 * (dfcs * (fr - b[s] * fa) + fcs * (dfr - b[s] * dfa)) * u
        # k = j: every term l != j of zeta_ij depends on r_ij
        dz = np.zeros(3)
        for q in range(nj):
            if q == s:
                continue
            dc, c = dcos_drij(s, q)
            g, dg = angle_fn(c, p)
            e, de = exp_fn(rn[s] - rn[q], p)
            dz += fc[q][0] * (dg * dc * e + g * de * u)
        grad -= 0.5 * a[s] * db[s] * dz
        # k != j: the term l = j of zeta_ik
        for q in range(nj):
            if q == s:
                continue
            dc, c = dcos_drij(s, q)      # cos theta_ikj, differentiated in r_ij
            g, dg = angle_fn(c, p)
            e, de = exp_fn(rn[q] - rn[s], p)
            dzq = dfcs * g * e * u + fcs * dg * dc * e - fcs * g * de * u
            grad -= 0.5 * a[q] * db[q] * dzq
        D[s] = grad
    return D


def site_energy_partials(pos, box, p, nl):
    """dU_i/dr_ij for every neighbour j = nl[i][s]: list [i] of arrays [len(nl[i]), 3].

    With a_ik = f_C(r_ik) B exp(-l2 r_ik) and V_ij the pair bracket,
      dU_i/dr_ij = 1/2 dV_ij/dr_ij (b_ij held fixed)
                   - 1/2 sum_k a_ik (db_ik/dzeta_ik) dzeta_ik/dr_ij,
    where k runs over all neighbours of i: zeta_ij depends on r_ij through every
    term of its sum, zeta_ik (k != j) through its term l = j.
    """
    return [_site_partials_one(pos, box, p, i, nl[i]) for i in range(len(nl))]


def _partial(Dp, nl, j, i):
    """dU_j/dr_ji from the partials of atom j."""
    return Dp[j][nl[j].index(i)]


def per_atom_virial(pos, box, p, nl) -> np.ndarray:
    """Eq. 8: W_i^{mu nu} = sum_{j != i} r_ij^mu (dU_j/dr_ji)^nu, [N, 3, 3]."""
    Dp = site_energy_partials(pos, box, p, nl)
    W = np.zeros((len(nl), 3, 3))
    for i in range(len(nl)):
        for j in nl[i]:
            W[i] += np.outer(_vec(pos, box, i, j), _partial(Dp, nl, j, i))
    return W


def forces(pos, box, p, nl) -> np.ndarray:
    """Eq. 4 summed over the neighbours: F_i = sum_j (dU_i/dr_ij - dU_j/dr_ji), [N, 3]."""
    Dp = site_energy_partials(pos, box, p, nl)
    F = np.zeros((len(nl), 3))
    for i in range(len(nl)):
        for s, j in enumerate(nl[i]):
            F[i] += Dp[i][s] - _partial(Dp, nl, j, i)
    return F


def total_virial_eq5(pos, box, p, nl) -> np.ndarray:
    """Eq. 5: W = -1/2 sum_i sum_j r_ij (x) F_ij, with the F_ij of Eq. 4."""
    Dp = site_energy_partials(pos, box, p, nl)
    W = np.zeros((3, 3))
    for i in range(len(nl)):
        for s, j in enumerate(nl[i]):
            W -= 0.5 * np.outer(_vec(pos, box, i, j), Dp[i][s] - _partial(Dp, nl, j, i))
    return W


def per_atom_virial_eq2(pos, box, p, nl) -> np.ndarray:
    """Eq. 2, the earlier per-atom virial: -1/2 sum_j r_ij (x) F_ij, [N, 3, 3]."""
    Dp = site_energy_partials(pos, box, p, nl)
    W = np.zeros((len(nl), 3, 3))
    for i in range(len(nl)):
        for s, j in enumerate(nl[i]):
            W[i] -= 0.5 * np.outer(_vec(pos, box, i, j), Dp[i][s] - _partial(Dp, nl, j, i))
    return W


def heat_current_eq9(pos, box, vel, p, nl) -> np.ndarray:
    """Eq. 9: J_i = sum_j r_ij (dU_j/dr_ji . v_i), [N, 3] (loops)."""
    Dp = site_energy_partials(pos, box, p, nl)
    vel = np.asarray(vel, dtype=np.float64)
    J = np.zeros((len(nl), 3))
    for i in range(len(nl)):
        for j in nl[i]:
            J[i] += _vec(pos, box, i, j) * float(_partial(Dp, nl, j, i) @ vel[i])
    return J


def heat_current_eq10(W, vel) -> np.ndarray:
    """Eq. 10: J_i^mu = sum_nu W_i^{mu nu} v_i^nu, [N, 3]."""
    return np.einsum("imn,in->im", np.asarray(W, dtype=np.float64), np.asarray(vel, dtype=np.float64))


def atom_energies(U, mass, vel) -> np.ndarray:
    """E_i = U_i + m_i |v_i|^2 / 2 (kinetic part converted to eV)."""
    vel = np.asarray(vel, dtype=np.float64)
    return np.asarray(U, dtype=np.float64) + 0.5 * np.asarray(mass, dtype=np.float64) * (vel * vel).sum(axis=1) * KE_UNIT


def hnemd_force_eq11(pos, box, E, fe, p, nl) -> np.ndarray:
    """Eq. 11: F_i^ext = E_i F_e + sum_j (dU_j/dr_ji (x) r_ij) . F_e, [N, 3] (loops)."""
    Dp = site_energy_partials(pos, box, p, nl)
    fe = np.asarray(fe, dtype=np.float64)
    F = np.zeros((len(nl), 3))
    for i in range(len(nl)):
        F[i] = E[i] * fe
        for j in nl[i]:
            F[i] += np.outer(_partial(Dp, nl, j, i), _vec(pos, box, i, j)) @ fe
    return F


def hnemd_force_eq12(E, W, fe) -> np.ndarray:
    """Eq. 12: F_i^ext = E_i F_e + F_e . W_i, (F_e . W_i)^nu = sum_mu F_e^mu W_i^{mu nu}."""
    fe = np.asarray(fe, dtype=np.float64)
    return np.asarray(E, dtype=np.float64)[:, None] * fe[None, :] + np.einsum("m,imn->in", fe, W)


def evaluate_atoms(pos, box, vel, mass, fe, p, atoms) -> dict:
    """The quantities of evaluate() for the listed atoms only, each computed on
    its own: the neighbour lists of the atom and of its neighbours by brute
    force, then U_i, F_i (Eq. 4), W_i (Eq. 8) and F_i^ext (Eq. 12).  For
    sampling systems too large for the whole-system functions."""
    pos = np.asarray(pos, dtype=np.float64)
    rc = p["R"] + p["D"]
    lists = {}

    def nl_of(i):
        if i not in lists:
            r = np.linalg.norm(min_image(pos - pos[i], box), axis=1)
            lists[i] = [int(j) for j in np.nonzero(r < rc)[0] if j != i]
        return lists[i]

    fe = np.asarray(fe, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    out = {k: [] for k in ("U", "F", "W", "Fext")}
    for i in atoms:
        js = nl_of(int(i))
        Di = _site_partials_one(pos, box, p, int(i), js)
        U = _site_energy_one(pos, box, p, int(i), js)
        F = np.zeros(3)
        W = np.zeros((3, 3))
        for s, j in enumerate(js):
            jl = nl_of(j)
            dji = _site_partials_one(pos, box, p, j, jl)[jl.index(int(i))]
            F += Di[s] - dji
            W += np.outer(_vec(pos, box, int(i), j), dji)
        E = U + 0.5 * float(mass[i]) * float(vel[i] @ vel[i]) * KE_UNIT
        out["U"].append(U)
        out["F"].append(F)
        out["W"].append(W)
        out["Fext"].append(E * fe + fe @ W)
    return {k: np.array(v) for k, v in out.items()}


def evaluate(pos, box, vel, mass, fe, p, nl=None) -> dict:
    """Everything the device computes for one configuration: U, F, W (Eq. 8),
    per-atom heat current (Eq. 10) and F^ext (Eq. 12)."""
    if nl is None:
        nl = neighbor_lists(pos, box, p["R"] + p["D"])
    U = site_energies(pos, box, p, nl)
    W = per_atom_virial(pos, box, p, nl)
    E = atom_energies(U, mass, vel)
    return {"U": U, "F": forces(pos, box, p, nl), "W": W, "J": heat_current_eq10(W, vel),
            "Fext": hnemd_force_eq12(E, W, fe), "E": E, "nl": nl}


def md_nve(pos, vel, mass, box, p, dt: float, n_steps: int) -> dict:
    """NVE molecular dynamics with the forces above, by velocity Verlet (the
    paper's production runs are NVE with a 1 fs time step, Sec. III.A; it names
    no integrator).  One step, with a = F / (m KE_UNIT) in A/fs^2:
        v <- v + dt/2 a(x);   x <- x + dt v (wrapped into the box);   v <- v + dt/2 a(x).
    The neighbour lists are rebuilt from scratch at every step.  Returns, for
    every step s = 1 .. n_steps, the positions, velocities and per-atom virials
    (Eq. 8) after the step, and the total energy sum_i U_i + m_i |v_i|^2 / 2
    before the first step (index 0) and after each step."""
    box = np.asarray(box, dtype=np.float64)
    x = np.mod(np.array(pos, dtype=np.float64), box)
    v = np.array(vel, dtype=np.float64)
    m = np.asarray(mass, dtype=np.float64)
    inv_mk = 1.0 / (m * KE_UNIT)

    def state(x):
        nl = neighbor_lists(x, box, p["R"] + p["D"])
        return forces(x, box, p, nl), nl

    def energy(x, v, nl):
        return float(site_energies(x, box, p, nl).sum() + 0.5 * (m * (v * v).sum(axis=1)).sum() * KE_UNIT)

    F, nl = state(x)
    out = {"pos": [], "vel": [], "W": [], "E": [energy(x, v, nl)]}
    for _ in range(n_steps):
        v = v + 0.5 * dt * F * inv_mk[:, None]
        x = np.mod(x + dt * v, box)
        F, nl = state(x)
        v = v + 0.5 * dt * F * inv_mk[:, None]
        out["pos"].append(x.copy())
        out["vel"].append(v.copy())
        out["W"].append(per_atom_virial(x, box, p, nl))
        out["E"].append(energy(x, v, nl))
    return {k: np.array(val) for k, val in out.items()}


# Boltzmann constant in eV/K (CODATA 2018, exact)
K_B = 8.617333262e-5


def md_nvt_hnemd(pos, vel, mass, box, p, dt: float, n_steps: int, fe, temperature: float, tau: float,
                 xi: float = 0.0, eta: float = 0.0) -> dict:
    """NVT molecular dynamics with the HNEMD driving force on every atom, the
    protocol of the paper's HNEMA and SHC runs (Sec. III.A: 300 K, a 1 fs time
    step, a Nose-Hoover thermostat; the driving force of Eq. 12).  One
    thermostat variable xi with mass Q = g k_B T tau^2 (g = 3N), its time
    integral eta, and a time-reversible splitting of each step:
        xi += dt/2 G;   v *= exp(-xi dt/2);   eta += dt/2 xi
        v += dt/2 a;    x += dt v (wrapped);  v += dt/2 a
        v *= exp(-xi dt/2);   eta += dt/2 xi;   xi += dt/2 G
    with G = (2K - g k_B T) / Q for the kinetic energy K of the velocities at
    that point, and a = (F + F_ext) / (m KE_UNIT), F_ext = E_i F_e + F_e . W_i
    (Eq. 12) with E_i from the velocities at the force evaluation (after the
    first half kick).  Neighbour lists are rebuilt at every evaluation.
    Returns, for every step, the positions, velocities and per-atom virials
    after it, xi and eta after it, and the extended energy
    K + U + Q xi^2 / 2 + g k_B T eta before the first step (index 0) and after
    each step: a constant of the motion when fe = 0."""
    box = np.asarray(box, dtype=np.float64)
    x = np.mod(np.array(pos, dtype=np.float64), box)
    v = np.array(vel, dtype=np.float64)
    m = np.asarray(mass, dtype=np.float64)
    fe = np.asarray(fe, dtype=np.float64)
    inv_mk = 1.0 / (m * KE_UNIT)
    g = 3 * len(m)
    gkt = g * K_B * temperature
    Q = gkt * tau * tau

    def kinetic(v):
        return 0.5 * float((m * (v * v).sum(axis=1)).sum()) * KE_UNIT

    def state(x, v):
        nl = neighbor_lists(x, box, p["R"] + p["D"])
        U = site_energies(x, box, p, nl)
        W = per_atom_virial(x, box, p, nl)
        F = forces(x, box, p, nl) + hnemd_force_eq12(atom_energies(U, m, v), W, fe)
        return F, U, W

    F, U, _ = state(x, v)
    out = {"pos": [], "vel": [], "W": [], "xi": [], "eta": [],
           "H": [kinetic(v) + float(U.sum()) + 0.5 * Q * xi * xi + gkt * eta]}
    for _ in range(n_steps):
        xi += 0.5 * dt * (2.0 * kinetic(v) - gkt) / Q
        v = v * math.exp(-0.5 * dt * xi)
        eta += 0.5 * dt * xi
        v = v + 0.5 * dt * F * inv_mk[:, None]
        x = np.mod(x + dt * v, box)
        F, U, W = state(x, v)
        v = v + 0.5 * dt * F * inv_mk[:, None]
        v = v * math.exp(-0.5 * dt * xi)
        eta += 0.5 * dt * xi
        xi += 0.5 * dt * (2.0 * kinetic(v) - gkt) / Q
        out["pos"].append(x.copy())
        out["vel"].append(v.copy())
        out["W"].append(W)
        out["xi"].append(xi)
        out["eta"].append(eta)
        out["H"].append(kinetic(v) + float(U.sum()) + 0.5 * Q * xi * xi + gkt * eta)
    return {k: np.array(val) for k, val in out.items()}
