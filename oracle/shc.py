"""FP64 CPU oracle of the spectral heat current (SHC), Sec. II.C, Eqs. 20-23.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the plain reference the
GPU library is checked against.  Only the test suite, the package smoke check
and the CPU-baseline leg of the benchmark may import it; the library never
does, and it imports nothing from the library.

Array conventions as in ``oracle.modal``: v [S, N, 3], W [S, N, 3, 3] with
W[s, i, mu, nu] = W_i^{mu nu}.

Readings where the paper is silent:
  * Eq. 21 uses the virial convention of Eq. 10, (W . v)^mu = sum_nu W^{mu nu}
    v^nu, so that K(0) is the Eq. 10 current, as the paper states.
  * The virial is taken at the time origin and the velocity at the later time,
    K(tau) = <W(s) . v(s + tau)> (Eq. 20 has the virial factors at time 0 and
    the momentum at time t).
  * The steady-state average uses every available origin at each lag:
    K(tau) = 1/(S - tau) sum_{s=0}^{S-1-tau} sum_i W_i(s) . v_i(s + tau).
  * Eq. 22 integrates over the whole time axis while K is sampled for t >= 0
    only: K is extended evenly, K(-t) = K(t), and the integral over
    [-(n-1) dt, (n-1) dt] is the trapezoid rule, so
      K~(omega) = dt [K(0) + 2 sum_{tau=1}^{n-2} w_tau K(tau) cos(omega tau dt)
                      + w_{n-1} K(n-1) cos(omega (n-1) dt)]
    with the window w = 1, or the Hann window w_tau = (1 + cos(pi tau/(n-1)))/2
    when asked for (a finite correlation time needs one to damp ringing; the
    paper names none).  The result is real.
"""
from __future__ import annotations

import math

import numpy as np


def shc_correlation(v: np.ndarray, W: np.ndarray, n_lags: int) -> np.ndarray:
    """Eq. 21: K[tau, mu] = <sum_i (W_i(s) . v_i(s + tau))^mu> over the S - tau
    origins s.  Lags with no origin (tau >= S) are zero.  Shape [n_lags, 3]."""
    v = np.asarray(v, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    S = v.shape[0]
    K = np.zeros((n_lags, 3), dtype=np.float64)
    for tau in range(min(n_lags, S)):
        early = W[: S - tau]             # W_i^{mu nu}(s)
        late = v[tau:]                   # v_i^nu(s + tau)
        # sum over origins s, atoms i and the contracted index nu -> [mu]
        K[tau] = np.tensordot(early, late, axes=([0, 1, 3], [0, 1, 2])) / (S - tau)
    return K


def shc_correlation_directional(v: np.ndarray, W: np.ndarray, n_lags: int) -> np.ndarray:
    """Eq. 21 split by the direction nu of the atoms' motion (Sec. II, remark
    after Eq. 10; closing remark of Sec. II.C):
    K[tau, mu, nu] = <sum_i W_i^{mu nu}(s) v_i^nu(s + tau)> over the S - tau
    origins; the sum over nu is Eq. 21.  Shape [n_lags, 3, 3].

    For each (mu, nu) the Gram matrix G[s, s'] = sum_i W_i^{mu nu}(s) v_i^nu(s')
    is one matrix product; the lag-tau sum over origins is its tau-th upper
    diagonal, sum_s G[s, s + tau]."""
    v = np.asarray(v, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    S = v.shape[0]
    K = np.zeros((n_lags, 3, 3), dtype=np.float64)
    for mu in range(3):
        for nu in range(3):
            G = np.ascontiguousarray(W[:, :, mu, nu]) @ np.ascontiguousarray(v[:, :, nu]).T    # [S, S]
            for tau in range(min(n_lags, S)):
                K[tau, mu, nu] = np.trace(G, offset=tau) / (S - tau)
    return K


def shc_weights(n_lags: int, window: bool = False) -> np.ndarray:
    """Weights c_tau of the even-extension trapezoid rule (times the Hann window
    when ``window``): c_0 = 1, c_tau = 2 inside, c_{n-1} = 1."""
    c = np.full(n_lags, 2.0)
    c[0] = 1.0
    if n_lags > 1:
        c[-1] = 1.0
    if window and n_lags > 1:
        tau = np.arange(n_lags, dtype=np.float64)
        c = c * 0.5 * (1.0 + np.cos(np.pi * tau / (n_lags - 1)))
    return c


def shc_spectrum(K: np.ndarray, dt: float, omega: np.ndarray, window: bool = False) -> np.ndarray:
    """Eq. 22 on the sampled lags: K~[w, mu] = dt sum_tau c_tau K[tau, mu]
    cos(omega_w tau dt).  omega in radians per unit of dt.  Shape [n_omega, 3]."""
    K = np.asarray(K, dtype=np.float64)
    omega = np.asarray(omega, dtype=np.float64)
    n = K.shape[0]
    c = shc_weights(n, window)
    tau = np.arange(n, dtype=np.float64)
    phase = np.cos(np.outer(omega, tau) * dt)            # [n_omega, n_lags]
    return dt * (phase * c) @ K


def shc_kappa(Kw: np.ndarray, volume: float, temperature: float, fe: float) -> np.ndarray:
    """Eq. 23: kappa(omega) = 2 K~(omega) / (V T F_e), in the units of the
    inputs (the caller converts)."""
    return 2.0 * np.asarray(Kw, dtype=np.float64) / (volume * temperature * fe)


def shc_correlation_loops(v, W, n_lags):
    """Eq. 21 written out with Python loops, for tiny inputs only."""
    S, N = len(v), len(v[0])
    K = [[0.0, 0.0, 0.0] for _ in range(n_lags)]
    for tau in range(min(n_lags, S)):
        for mu in range(3):
            terms = []
            for s in range(S - tau):
                for i in range(N):
                    for nu in range(3):
                        terms.append(float(W[s][i][mu][nu]) * float(v[s + tau][i][nu]))
            K[tau][mu] = math.fsum(terms) / (S - tau)
    return np.array(K)
