"""FFT form of the binned modal current for the real Bloch basis.

TEST INFRASTRUCTURE ONLY (see oracle.modal).

For a basis made of real plane waves on a periodic L1 x L2 x L3 grid (any
orthonormal real basis spanning, per frequency bin, the plane waves of the
k-points in that bin), Eq. 16 summed over the modes of a bin is

    J_b^mu = u^T P_b w^mu,   P_b = projector onto the bin's modes,

and P_b is diagonal in the discrete Fourier basis.  With U_alpha(k) and
Wmu_alpha(k) the unnormalised DFTs (numpy.fft.fftn) of u and w^mu over the
grid, Parseval gives

    J_b^mu = (1/N) sum_{k in b} sum_alpha Re(conj(U_alpha(k)) Wmu_alpha(k)).

This reduces the dense O(N^2) projection to an O(N log N) library FFT, so it
can check binned currents at sizes the dense oracle cannot hold.  It does not
assume anything about how the basis is ordered or rotated inside a bin.
"""
from __future__ import annotations

import numpy as np


def binned_current_fft(dims, m, v, W, kbin, n_bins) -> np.ndarray:
    """J_b^mu(s) for every step, shape [S, 3, nb].

    dims  (L1, L2, L3); atom i = (a*L2 + b)*L3 + c
    m     [N] masses; v [S, N, 3]; W [S, N, 3, 3] with W[s, i, mu, nu]
    kbin  [L1, L2, L3] bin of each k-point (-1 = excluded)
    """
    L1, L2, L3 = dims
    m = np.asarray(m, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    S, N, _ = v.shape
    sq = np.sqrt(m)
    u = (sq[None, :, None] * v).reshape(S, L1, L2, L3, 3)
    w = (W / sq[None, :, None, None]).reshape(S, L1, L2, L3, 3, 3)   # [..., mu, nu]
    U = np.fft.fftn(u, axes=(1, 2, 3))
    out = np.zeros((S, 3, n_bins), dtype=np.float64)
    flat_bins = np.asarray(kbin).reshape(-1)
    for mu in range(3):
        Wm = np.fft.fftn(w[..., mu, :], axes=(1, 2, 3))
        dens = np.real(np.conj(U) * Wm).sum(axis=-1).reshape(S, -1) / N   # [S, K]
        for b in range(n_bins):
            sel = flat_bins == b
            if sel.any():
                out[:, mu, b] = dens[:, sel].sum(axis=1)
    return out
