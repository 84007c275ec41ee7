"""FP64 CPU oracle of the bin-bin (mode-mode) cross-correlation of modal heat
currents.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the plain reference the
GPU library is checked against.  Only the test suite, the package smoke check
and the CPU-baseline leg of the benchmark may import it; the library never
does, and it imports nothing from the library.

Sec. II.B.i notes that cross-correlations of modal heat currents resolve
mode-mode interactions beyond each mode's total contribution of Eq. 17, and
Sec. III.C.i that the modal currents GKMA produces allow them (HNEMA does
not).  The paper computes none; the definition here puts a second binned
modal current where Eq. 17 has the total current:

    C[tau, b, b2, mu, nu] = <J_b^mu(t + tau) J_b2^nu(t)>,

with the time-origin average, lag direction and origin count of
``oracle.modal.gkma_correlation`` (the readings stated there).
With every mode binned and a complete basis, the sum over b2 is the Eq. 17
integrand, since the binned currents then sum to the Eq. 10 total.
"""
from __future__ import annotations

import numpy as np


def gkma_cross_correlation(Jb: np.ndarray, corr_len: int) -> np.ndarray:
    """Jb [S, 3, nb] binned modal currents -> C [L, nb, nb, 3, 3] as above.
    Lags with no origin (tau >= S) are zero."""
    Jb = np.asarray(Jb, dtype=np.float64)
    S, _, nb = Jb.shape
    out = np.zeros((corr_len, nb, nb, 3, 3), dtype=np.float64)
    for tau in range(min(corr_len, S)):
        late = Jb[tau:]                  # J_b^mu(s),        s = tau .. S-1
        early = Jb[: S - tau]            # J_b2^nu(s - tau)
        # sum over the origins: [mu, b] x [nu, b2] -> [mu, b, nu, b2]
        prod = np.tensordot(late, early, axes=([0], [0]))
        out[tau] = prod.transpose(1, 3, 0, 2) / (S - tau)
    return out


def gkma_cross_correlation_loops(Jb, corr_len):
    """The same with Python loops, for tiny inputs only."""
    S, _, nb = len(Jb), len(Jb[0]), len(Jb[0][0])
    out = np.zeros((corr_len, nb, nb, 3, 3))
    for tau in range(min(corr_len, S)):
        for b in range(nb):
            for b2 in range(nb):
                for mu in range(3):
                    for nu in range(3):
                        acc = 0.0
                        for s in range(tau, S):
                            acc += float(Jb[s][mu][b]) * float(Jb[s - tau][nu][b2])
                        out[tau, b, b2, mu, nu] = acc / (S - tau)
    return out
