"""FP64 CPU oracle of the direction-resolved modal heat current.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the plain reference the
GPU library is checked against.  Only the test suite, the package smoke check
and the CPU-baseline leg of the benchmark may import it; the library never
does, and it imports nothing from the library.

Sec. II (the remark after Eq. 10) notes that the per-atom form of the heat
current splits by the Cartesian direction of the atoms' motion: the mu
component of W_i . v_i is a sum over nu of W_i^{mu nu} v_i^nu, one term per
motion direction.  The closing remark of Sec. II.C carries the same split to
every method's mode- or frequency-resolved result (in-plane against
out-of-plane motion for 2D materials, Sec. III.A.ii).  For the modal current
of Eq. 16 the split keeps the modal velocity of Eq. 13 whole and restricts the
virial bracket to the nu column of W_i and the nu component of e_{i,n}:

    J_n^{mu nu}(s) = Xdot_n(s) sum_i m_i^{-1/2} W_i^{mu nu}(s) e_{i,n}^nu,

so that sum_nu J_n^{mu nu} = J_n^mu.  The total of Eq. 10 splits alike:
J^{mu nu}(s) = sum_i W_i^{mu nu}(s) v_i^nu(s).

Readings:
  * nu is the second virial index, the one contracted with the motion
    (Eq. 10 convention of ``oracle.modal``).
  * The GKMA correlation of a split current keeps the total current whole:
    C[tau, b, mu, nu, mu2] = <J_b^{mu nu}(t + tau) J^{mu2}(t)>, so that the sum
    over nu is the Eq. 17 integrand.

Array conventions as in ``oracle.modal``; split outputs put the motion
direction nu right after the heat-current direction mu.
"""
from __future__ import annotations

import numpy as np

from . import modal


def masked_virial(m: np.ndarray, W: np.ndarray, nu: int) -> np.ndarray:
    """w_nu[s, mu, 3i+alpha] = W_i^{mu nu}(s) / sqrt(m_i) if alpha == nu else 0:
    the Eq. 16 bracket vector restricted to motion direction nu."""
    W = np.asarray(W, dtype=np.float64)
    S, N, _, _ = W.shape
    w = np.zeros((S, 3, N, 3), dtype=np.float64)
    inv = 1.0 / np.sqrt(np.asarray(m, dtype=np.float64))
    # [S, N, mu] -> [S, mu, N], placed in the alpha == nu slot
    w[:, :, :, nu] = (W[:, :, :, nu] * inv[None, :, None]).transpose(0, 2, 1)
    return w.reshape(S, 3, 3 * N)


def modal_currents_directional(E, m, v, W) -> np.ndarray:
    """J_n^{mu nu}(s), shape [S, 3 (mu), 3 (nu), M]."""
    xdot = modal.modal_velocity(E, modal.mass_weighted_velocity(m, v))          # Eq. 13, [S, M]
    out = []
    for nu in range(3):
        A = modal.virial_projection(E, masked_virial(m, W, nu))                # [S, 3, M]
        out.append(modal.modal_heat_current(xdot, A))
    return np.stack(out, axis=2)


def total_heat_current_directional(v: np.ndarray, W: np.ndarray) -> np.ndarray:
    """J^{mu nu}(s) = sum_i W_i^{mu nu}(s) v_i^nu(s), shape [S, 3, 3]."""
    v = np.asarray(v, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    return np.einsum("simn,sin->smn", W, v)


def binned_directional(Jn_dir: np.ndarray, bins: np.ndarray, n_bins: int) -> np.ndarray:
    """Bin sums of the split currents: [S, 3, 3, M] -> [S, 3, 3, nb]."""
    return np.stack([modal.binned_current(Jn_dir[:, :, nu, :], bins, n_bins) for nu in range(3)], axis=2)


def hnema_average_directional(Jb_dir: np.ndarray) -> np.ndarray:
    """Eq. 19 numerator per motion direction: [S, 3, 3, nb] -> [nb, 3 (mu), 3 (nu)]."""
    return np.stack([modal.hnema_average(Jb_dir[:, :, nu, :]) for nu in range(3)], axis=2)


def gkma_correlation_directional(Jb_dir: np.ndarray, Jt: np.ndarray, corr_len: int) -> np.ndarray:
    """<J_b^{mu nu}(t + tau) J^{mu2}(t)>: [L, nb, 3 (mu), 3 (nu), 3 (mu2)]."""
    return np.stack([modal.gkma_correlation(Jb_dir[:, :, nu, :], Jt, corr_len) for nu in range(3)], axis=3)


def run_dense_directional(E, m, v, W, bins, n_bins, corr_len=0, dt=1.0):
    """Every split output on one trajectory:
    hnema_dir [nb, 3, 3], hnema_total_dir [3, 3] (time average of J^{mu nu}),
    corr_dir / integral_dir [L, nb, 3, 3, 3]."""
    Jn = modal_currents_directional(E, m, v, W)
    Jb = binned_directional(Jn, bins, n_bins)
    Jt = modal.total_heat_current(v, W)
    Jtd = total_heat_current_directional(v, W)
    out = {"Jb_dir": Jb, "hnema_dir": hnema_average_directional(Jb),
           "hnema_total_dir": hnema_average_directional(Jtd[:, :, :, None])[0]}
    if corr_len:
        C = gkma_correlation_directional(Jb, Jt, corr_len)
        out["corr_dir"] = C
        out["integral_dir"] = modal.gkma_running_integral(C, dt)
    return out
