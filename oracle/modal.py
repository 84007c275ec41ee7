"""FP64 CPU oracle of the modal heat-current path (HNEMA and GKMA).

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
package smoke check and the CPU-baseline leg of the benchmark may import it;
the library never does, and it imports nothing from the library.

Every function follows one passage of Gabourie, Fan, Ala-Nissila and Pop,
"Spectral Decomposition of Thermal Conductivity: Comparing Velocity
Decomposition Methods in Homogeneous Molecular Dynamics Simulations"
(arXiv:2102.03691), cited by section and equation.  Arithmetic is float64
throughout; matrix products use numpy (BLAS dgemm), time sums use
``math.fsum`` where the sum is the definition itself.

Array conventions (the paper uses none; these are this project's):
  E      [3N, M]      eigenvectors, E[3*i+alpha, n] = e_{i,n}^alpha (real)
  m      [N]          masses
  v      [S, N, 3]    velocities v_i^alpha at each step
  W      [S, N, 3, 3] per-atom virials, W[s, i, mu, nu] = W_i^{mu nu}
  bins   [M]          bin index of each mode, -1 = mode excluded
Outputs carry the Cartesian index mu of the heat current.

Readings where the paper is silent:
  * e* = e: only real bases are used (Eq. 13).
  * (W . v)^mu = sum_nu W^{mu nu} v^nu, i.e. the virial's first index is the
    heat-current direction (Eq. 8 defines W_i as r_ij (outer) dU_j/dr_ji and
    Eq. 9 contracts the second factor with v_i).
  * The total current in the Green-Kubo correlation is Eq. 10 evaluated
    directly, not the mode sum.
  * Time-origin average at lag tau uses every available origin, S - tau.
  * The later time belongs to the modal current: <J_b^mu(t+tau) J^nu(t)>.
  * The running integral is the trapezoid rule with G(0) = 0.
  * Uniform frequency bins: width (f_hi - f_lo)/nb, half-open, ties go up,
    f == f_hi falls in the last bin, frequencies outside [f_lo, f_hi] are
    excluded.
"""
from __future__ import annotations

import math

import numpy as np

# Constants for the kappa prefactors (owned here; the generators keep their own).
KB_EV_PER_K = 8.617333262e-5
_EV_J = 1.602176634e-19      # J per eV
_A_M = 1e-10                 # m per Angstrom
_FS_S = 1e-15                # s per fs


# --------------------------------------------------------------- Eq. 13 / 16
def mass_weighted_velocity(m: np.ndarray, v: np.ndarray) -> np.ndarray:
    """u[s, 3i+alpha] = sqrt(m_i) v_i^alpha(s): the factor of Eq. 13."""
    v = np.asarray(v, dtype=np.float64)
    S, N, _ = v.shape
    return (np.sqrt(np.asarray(m, dtype=np.float64))[None, :, None] * v).reshape(S, 3 * N)


def mass_scaled_virial(m: np.ndarray, W: np.ndarray) -> np.ndarray:
    """w[s, mu, 3i+nu] = W_i^{mu nu}(s) / sqrt(m_i): the bracket of Eq. 16.

    Row mu of W_i, divided by sqrt(m_i), is the vector that Eq. 16 contracts
    with the eigenvector e_{i,n}.
    """
    W = np.asarray(W, dtype=np.float64)
    S, N, _, _ = W.shape
    w = W / np.sqrt(np.asarray(m, dtype=np.float64))[None, :, None, None]
    # [S, N, mu, nu] -> [S, mu, N, nu] -> [S, mu, 3N]
    return np.ascontiguousarray(w.transpose(0, 2, 1, 3)).reshape(S, 3, 3 * N)


def modal_velocity(E: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Eq. 13: Xdot[s, n] = sum_i sqrt(m_i) e_{i,n} . v_i(s) = sum_j E[j, n] u[s, j]."""
    return np.asarray(u, dtype=np.float64) @ np.asarray(E, dtype=np.float64)


def virial_projection(E: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Eq. 16 bracket: A[s, mu, n] = sum_i (W_i . e_{i,n})^mu / sqrt(m_i)."""
    return np.asarray(w, dtype=np.float64) @ np.asarray(E, dtype=np.float64)


def modal_heat_current(xdot: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Eq. 16: J_n^mu(s) = A[s, mu, n] * Xdot[s, n], shape [S, 3, M]."""
    return A * xdot[:, None, :]


def modal_currents(E, m, v, W) -> np.ndarray:
    """Eqs. 13 and 16 chained: per-mode heat current, shape [S, 3, M]."""
    xdot = modal_velocity(E, mass_weighted_velocity(m, v))
    A = virial_projection(E, mass_scaled_virial(m, W))
    return modal_heat_current(xdot, A)


# ------------------------------------------------------------------- Eq. 10
def total_heat_current(v: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Eq. 10 summed over atoms: J^mu(s) = sum_i sum_nu W_i^{mu nu} v_i^nu. [S, 3]"""
    v = np.asarray(v, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    return np.einsum("simn,sin->sm", W, v)


# ------------------------------------------------------ frequency binning
def bin_of_mode(freq: np.ndarray, n_bins: int, f_lo: float, f_hi: float) -> np.ndarray:
    """Uniform frequency bins (Sec. III.A: bins of fixed width over the spectrum).

    b = min(floor((f - f_lo) / delta + 1e-9), nb - 1) with delta = (f_hi - f_lo)/nb,
    evaluated in float64.  The 1e-9 bin-width nudge sends frequencies that sit
    on an edge up to rounding into the upper bin.  Frequencies below f_lo or
    above f_hi get -1 (excluded).
    """
    if n_bins < 1 or not (f_hi > f_lo):
        raise ValueError("need n_bins >= 1 and f_hi > f_lo")
    f = np.asarray(freq, dtype=np.float64)
    delta = (f_hi - f_lo) / n_bins
    out = np.empty(f.shape[0], dtype=np.int32)
    for n in range(f.shape[0]):
        if not (f_lo <= f[n] <= f_hi):
            out[n] = -1
            continue
        b = math.floor((f[n] - f_lo) / delta + 1e-9)
        out[n] = min(b, n_bins - 1)
    return out


def binned_current(Jn: np.ndarray, bins: np.ndarray, n_bins: int) -> np.ndarray:
    """Sum of modal currents over the modes of each bin: J_b^mu(s). [S, 3, nb]"""
    Jn = np.asarray(Jn, dtype=np.float64)
    S = Jn.shape[0]
    out = np.zeros((S, 3, n_bins), dtype=np.float64)
    for b in range(n_bins):
        sel = np.nonzero(np.asarray(bins) == b)[0]
        if sel.size:
            out[:, :, b] = Jn[:, :, sel].sum(axis=2)
    return out


# ------------------------------------------------------------------ HNEMA
def hnema_average(Jb: np.ndarray) -> np.ndarray:
    """Eq. 19 numerator: time average <J_b^mu> over all S samples, [nb, 3].

    Each element is a correctly rounded sum (math.fsum) divided by S.
    """
    Jb = np.asarray(Jb, dtype=np.float64)
    S, _, nb = Jb.shape
    out = np.empty((nb, 3), dtype=np.float64)
    for b in range(nb):
        for mu in range(3):
            out[b, mu] = math.fsum(Jb[:, mu, b]) / S
    return out


def hnema_kappa(avg_ev_a_per_fs: np.ndarray, temperature: float, volume_a3: float,
                fe_per_a: float) -> np.ndarray:
    """Eq. 19 solved for the driven column: kappa_b^{mu x} = <J_b^mu> / (T V F_e).

    Inputs in eV*A/fs, K, A^3 and 1/A; output in W/(m K).
    """
    k = np.asarray(avg_ev_a_per_fs) / (temperature * volume_a3 * fe_per_a)  # eV/(fs A K)
    return k * _EV_J / (_FS_S * _A_M)


# ------------------------------------------------------------------- GKMA
def gkma_correlation(Jb: np.ndarray, Jt: np.ndarray, corr_len: int) -> np.ndarray:
    """Eq. 17 integrand: C[tau, b, mu, nu] = <J_b^mu(t + tau) J^nu(t)>.

    The bracket averages over every time origin available at that lag:
    C(tau) = 1/(S - tau) * sum_{s = tau}^{S-1} J_b^mu(s) J^nu(s - tau).
    Lags with no origin (tau >= S) are zero.  Shape [L, nb, 3, 3].
    """
    Jb = np.asarray(Jb, dtype=np.float64)
    Jt = np.asarray(Jt, dtype=np.float64)
    S, _, nb = Jb.shape
    out = np.zeros((corr_len, nb, 3, 3), dtype=np.float64)
    for tau in range(min(corr_len, S)):
        late = Jb[tau:]                  # J_b(s),        s = tau .. S-1
        early = Jt[: S - tau]            # J(s - tau)
        # sum over the origins s of late[s, mu, b] * early[s, nu] -> [mu, b, nu]
        prod = np.tensordot(late, early, axes=([0], [0]))
        out[tau] = prod.transpose(1, 0, 2) / (S - tau)
    return out


def correlation_counts(n_samples: int, corr_len: int) -> np.ndarray:
    """Number of time origins at each lag: max(S - tau, 0)."""
    return np.maximum(n_samples - np.arange(corr_len), 0).astype(np.int64)


def gkma_running_integral(C: np.ndarray, dt: float) -> np.ndarray:
    """Eq. 17 integral over tau by the trapezoid rule, G(0) = 0.

    G(tau) = G(tau - 1) + dt * (C(tau - 1) + C(tau)) / 2 along axis 0.
    """
    C = np.asarray(C, dtype=np.float64)
    G = np.zeros_like(C)
    for tau in range(1, C.shape[0]):
        G[tau] = G[tau - 1] + dt * 0.5 * (C[tau - 1] + C[tau])
    return G


def gkma_kappa(G_ev2_a2_per_fs: np.ndarray, temperature: float, volume_a3: float) -> np.ndarray:
    """Eq. 17 prefactor: kappa = G / (k_B T^2 V); G in (eV A/fs)^2 fs, out W/(m K)."""
    k = np.asarray(G_ev2_a2_per_fs) / (KB_EV_PER_K * temperature ** 2 * volume_a3)
    # (eV A / fs)^2 * fs / (eV/K * K^2 * A^3) = eV / (fs A K)
    return k * _EV_J / (_FS_S * _A_M)


# ------------------------------------------------------------ full runs
def run_dense(E, m, v, W, bins, n_bins, corr_len=0, dt=1.0):
    """Whole path on one trajectory: returns a dict of every output.

    Jn  [S, 3, M]   modal currents (Eq. 16)
    Jb  [S, 3, nb]  binned modal currents
    Jt  [S, 3]      total current (Eq. 10)
    hnema [nb, 3], hnema_total [3]   time averages (Eq. 19 numerator)
    corr [L, nb, 3, 3], hcacf [L, 3, 3], integral [L, nb, 3, 3] (Eq. 17)
    """
    Jn = modal_currents(E, m, v, W)
    Jb = binned_current(Jn, bins, n_bins)
    Jt = total_heat_current(v, W)
    out = {"Jn": Jn, "Jb": Jb, "Jt": Jt,
           "hnema": hnema_average(Jb),
           "hnema_total": hnema_average(Jt[:, :, None])[0]}
    if corr_len:
        C = gkma_correlation(Jb, Jt, corr_len)
        out["corr"] = C
        out["hcacf"] = gkma_correlation(Jt[:, :, None], Jt, corr_len)[:, 0]
        out["integral"] = gkma_running_integral(C, dt)
        out["counts"] = correlation_counts(Jb.shape[0], corr_len)
    return out


class StreamingOracle:
    """The same definitions applied to a trajectory that arrives in pieces.

    Keeps J_b(s) and J(s) for every sample pushed (float64), so the outputs
    are exactly those of :func:`run_dense` on the concatenated trajectory.
    E may be given as a callable ``rows(mode0, n) -> E^T rows`` for bases too
    large to hold; rows are then consumed in chunks of ``row_chunk`` modes.
    """

    def __init__(self, E, m, bins, n_bins, corr_len=0, dt=1.0, row_chunk=4096):
        self.E = E
        self.m = np.asarray(m, dtype=np.float64)
        self.bins = np.asarray(bins)
        self.n_bins = int(n_bins)
        self.corr_len = int(corr_len)
        self.dt = float(dt)
        self.row_chunk = row_chunk
        self._Jb = []
        self._Jt = []

    def _modal_binned(self, v, W):
        u = mass_weighted_velocity(self.m, v)
        w = mass_scaled_virial(self.m, W)
        if callable(self.E):
            M = self.bins.shape[0]
            Jb = np.zeros((u.shape[0], 3, self.n_bins))
            for r0 in range(0, M, self.row_chunk):
                rows = self.E(r0, min(self.row_chunk, M - r0))      # [r, 3N] = E^T rows
                Ec = rows.T
                Jn = modal_heat_current(modal_velocity(Ec, u), virial_projection(Ec, w))
                bsel = self.bins[r0:r0 + Ec.shape[1]]
                for b in np.unique(bsel[bsel >= 0]):
                    Jb[:, :, b] += Jn[:, :, bsel == b].sum(axis=2)
            return Jb
        Jn = modal_heat_current(modal_velocity(self.E, u), virial_projection(self.E, w))
        return binned_current(Jn, self.bins, self.n_bins)

    def push(self, v, W):
        self._Jb.append(self._modal_binned(v, W))
        self._Jt.append(total_heat_current(v, W))

    @property
    def Jb(self):
        return np.concatenate(self._Jb, axis=0)

    @property
    def Jt(self):
        return np.concatenate(self._Jt, axis=0)

    def read(self):
        Jb, Jt = self.Jb, self.Jt
        out = {"Jb": Jb, "Jt": Jt, "hnema": hnema_average(Jb),
               "hnema_total": hnema_average(Jt[:, :, None])[0], "n_samples": Jb.shape[0]}
        if self.corr_len:
            C = gkma_correlation(Jb, Jt, self.corr_len)
            out["corr"] = C
            out["hcacf"] = gkma_correlation(Jt[:, :, None], Jt, self.corr_len)[:, 0]
            out["integral"] = gkma_running_integral(C, self.dt)
            out["counts"] = correlation_counts(Jb.shape[0], self.corr_len)
        return out
