"""Scalar prefactors that turn the library's outputs into thermal conductivity.

Eq. 19: kappa_b^{mu nu} F_e^nu = <J_b^mu> / (T V), so for a driving force
along one axis kappa_b^{mu x} = <J_b^mu> / (T V F_e).
Eq. 17: kappa_b^{mu nu}(tau) = G_b^{mu nu}(tau) / (k_B T^2 V), G the running
integral of the modal-current / total-current correlation.
Eq. 23: kappa(omega) = 2 K~(omega) / (V T F_e), K~ the transform of the SHC
virial-velocity correlation (eV A/fs integrated over fs: eV A), a density per
unit of frequency f = omega / (2 pi).
Units: eV, Angstrom, fs, K in; W/(m K) out.
"""
KB_EV_PER_K = 8.617333262e-5
_EV_PER_FS_A_K_IN_W_PER_M_K = 1.602176634e-19 / (1e-15 * 1e-10)


def hnema_kappa(avg, temperature, volume_a3, fe_per_a):
    """kappa from an HNEMA average <J> (eV A/fs) for a drive F_e (1/A)."""
    return avg / (temperature * volume_a3 * fe_per_a) * _EV_PER_FS_A_K_IN_W_PER_M_K


def gkma_kappa(integral, temperature, volume_a3):
    """kappa(tau) from the GKMA running integral ((eV A/fs)^2 fs)."""
    return integral / (KB_EV_PER_K * temperature ** 2 * volume_a3) * _EV_PER_FS_A_K_IN_W_PER_M_K


def shc_kappa(Kw, temperature, volume_a3, fe_per_a):
    """Spectral kappa per unit of frequency (W m^-1 K^-1 THz^-1) from the SHC
    transform K~(omega) (eV A) for a drive F_e (1/A).

    Eq. 23's kappa(omega) = 2 K~(omega) / (V T F_e) is a density in
    d omega / (2 pi) = d f: K~ is even in omega and integrates over
    d omega / (2 pi) to K(0), the time average of the Eq. 10 current, so
    int_0^inf kappa(omega) d f = K(0) / (V T F_e), the HNEMD total.  In
    eV / (A K) it is already per hertz of f (1 eV / (A K) = 1.602e-9 J / (m K)
    = 1.602e-9 W m^-1 K^-1 Hz^-1); times 1e12 per THz."""
    per_hz = 2.0 * Kw / (volume_a3 * temperature * fe_per_a)             # eV / (A K)
    return per_hz * (1.602176634e-19 / 1e-10) * 1e12


def tersoff_si() -> dict:
    """Tersoff's published silicon parameters (Phys. Rev. B 38, 9902 (1988);
    the paper's Si potential, Sec. III.A), in the form ModalVirial takes:
    eV, 1/A and A."""
    return dict(A=1830.8, B=471.18, lambda1=2.4799, lambda2=1.7322, lambda3=0.0, m=3, beta=1.1e-6, n=0.78734,
                c=1.0039e5, d=16.217, h=-0.59825, gamma=1.0, R=2.85, D=0.15)
