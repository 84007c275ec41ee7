"""Seeded synthetic inputs for the modal heat-current path.

This module produces the *inputs* of the method and nothing else: an
orthonormal eigenvector basis with its mode frequencies, atomic masses, and
per-step atomic velocities and per-atom virials.  It holds none of the
method's arithmetic (no projection, no heat current, no binning, no time
average or correlation).  Both the FP64 oracle and the GPU library consume
what it produces; it imports neither of them.

Stand-ins for the paper's inputs (Sec. III.A): the paper projects MD
trajectories of CNT, graphene and Si onto harmonic lattice-dynamics
eigenvectors.  Neither the MD engine nor the relaxed structures exist here,
so the basis is the closed-form real Bloch basis of a monatomic simple-cubic
lattice with nearest-neighbour springs (Sec. II.B allows "any valid basis"),
velocities are Maxwell-Boltzmann Gaussians at the target temperature, and
virials are iid Gaussian nonsymmetric 3x3 tensors (Eq. 10 needs all nine
components).

Units: amu, Angstrom, fs, eV.  Frequencies are in THz.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from functools import cached_property

import numpy as np

# Physical constants owned by the generators (the library needs none; the
# oracle keeps its own copies for the kappa prefactors).
KB_EV_PER_K = 8.617333262e-5            # Boltzmann constant, eV/K
AMU_A2_PER_FS2_IN_EV = 103.642697       # 1 amu*A^2/fs^2 expressed in eV
SI_MASS_AMU = 28.0855                   # natural Si standard atomic weight
SI_ISOTOPES = ((27.9769265, 0.922), (28.9764947, 0.047), (29.9737702, 0.031))


def _lex_less(a, b) -> bool:
    return tuple(a) < tuple(b)


@dataclass(frozen=True)
class BlochLattice:
    """Monatomic simple-cubic lattice of L1 x L2 x L3 periodic cells.

    Atom i sits at integer position (a, b, c) with i = (a*L2 + b)*L3 + c.
    Degree of freedom j = 3*i + alpha (alpha = x, y, z).

    The basis is built from scalar real plane waves phi_f(r):
      * for each k-index n = (n1, n2, n3), 0 <= n_a < L_a, pair n with its
        conjugate nbar = (-n) mod L; the lexicographically smaller one is the
        representative;
      * self-conjugate n (n == nbar): phi = cos(2 pi n.r / L) / sqrt(N);
      * otherwise two functions, cos then sin, each scaled by sqrt(2/N).
    Functions are ordered by representative (lexicographic), cos before sin.
    Mode m = 3*f + alpha is phi_f(r_i) on dof 3*i + alpha and zero on the
    other two polarisations.  The 3N modes are orthonormal and complete.

    Frequencies (nearest-neighbour springs K, mass m):
      omega(n) = 2 sqrt(K/m) sqrt(sum_a sin^2(pi n_a / L_a)),
    the same for all three polarisations.  sin^2 is evaluated on the folded
    index min(n_a, L_a - n_a) and the three terms are summed in sorted order,
    so k, -k and axis permutations give bit-identical frequencies.
    """

    dims: tuple
    mass: float = SI_MASS_AMU
    spring: float = 10.0          # eV / A^2
    lattice_constant: float = 2.715  # A, edge of one simple-cubic cell

    def __post_init__(self):
        d = tuple(int(x) for x in self.dims)
        if len(d) != 3 or min(d) < 1:
            raise ValueError("dims must be three positive integers")
        object.__setattr__(self, "dims", d)

    @property
    def n_atoms(self) -> int:
        L1, L2, L3 = self.dims
        return L1 * L2 * L3

    @property
    def n_modes(self) -> int:
        return 3 * self.n_atoms

    @property
    def volume(self) -> float:
        """Cell volume in A^3 (N cells of edge ``lattice_constant``)."""
        return float(self.n_atoms) * self.lattice_constant ** 3

    # ------------------------------------------------------------------ basis
    @cached_property
    def functions(self):
        """(kvec [F,3] int64, kind [F] int8, norm [F] float64).

        kind: 0 = self-conjugate cosine, 1 = cosine of a pair, 2 = sine.
        """
        L1, L2, L3 = self.dims
        N = self.n_atoms
        ks, kinds, norms = [], [], []
        for n1 in range(L1):
            for n2 in range(L2):
                for n3 in range(L3):
                    n = (n1, n2, n3)
                    nb = ((-n1) % L1, (-n2) % L2, (-n3) % L3)
                    if n == nb:
                        ks.append(n); kinds.append(0); norms.append(1.0 / math.sqrt(N))
                    elif _lex_less(n, nb):
                        s = math.sqrt(2.0 / N)
                        ks.append(n); kinds.append(1); norms.append(s)
                        ks.append(n); kinds.append(2); norms.append(s)
        k = np.asarray(ks, dtype=np.int64).reshape(-1, 3)
        assert k.shape[0] == N
        return k, np.asarray(kinds, dtype=np.int8), np.asarray(norms, dtype=np.float64)

    @cached_property
    def positions(self) -> np.ndarray:
        """Integer cell coordinates [N, 3] in atom order."""
        L1, L2, L3 = self.dims
        a, b, c = np.meshgrid(np.arange(L1), np.arange(L2), np.arange(L3), indexing="ij")
        return np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1).astype(np.int64)

    def _phases(self, kvec: np.ndarray) -> np.ndarray:
        """Exact integer phase numerators p, theta = 2 pi p / (L1 L2 L3), shape [F, N]."""
        L1, L2, L3 = self.dims
        r = self.positions
        w = np.array([L2 * L3, L1 * L3, L1 * L2], dtype=np.int64)
        p = (kvec * w) @ r.T
        return np.mod(p, L1 * L2 * L3)

    def scalar_functions(self, f0: int, nf: int) -> np.ndarray:
        """phi_f(r_i) for f in [f0, f0+nf), shape [nf, N] float64."""
        k, kind, norm = self.functions
        sl = slice(f0, f0 + nf)
        theta = self._phases(k[sl]).astype(np.float64) * (2.0 * math.pi / self.n_atoms)
        out = np.where((kind[sl] == 2)[:, None], np.sin(theta), np.cos(theta))
        return out * norm[sl, None]

    def eig_rows(self, mode0: int, n_rows: int) -> np.ndarray:
        """Rows mode0..mode0+n_rows-1 of E^T: shape [n_rows, 3N] float64.

        Row m holds e_{i,m}^alpha at column 3*i + alpha.
        """
        if mode0 < 0 or n_rows < 0 or mode0 + n_rows > self.n_modes:
            raise ValueError("row range outside the basis")
        N = self.n_atoms
        out = np.zeros((n_rows, 3 * N), dtype=np.float64)
        if n_rows == 0:
            return out
        f_lo = mode0 // 3
        f_hi = (mode0 + n_rows - 1) // 3 + 1
        phi = self.scalar_functions(f_lo, f_hi - f_lo)
        for r in range(n_rows):
            m = mode0 + r
            f, alpha = divmod(m, 3)
            out[r, alpha::3] = phi[f - f_lo]
        return out

    def eig_matrix(self) -> np.ndarray:
        """Full E, shape [3N (dof), 3N (mode)], float64 (small lattices only)."""
        return np.ascontiguousarray(self.eig_rows(0, self.n_modes).T)

    def eig_rows_torch(self, mode0: int, n_rows: int, device="cuda"):
        """Same rows as :meth:`eig_rows`, generated with torch on ``device``.

        Used to feed large bases straight into device memory without an FP64
        host copy.  Values agree with :meth:`eig_rows` to float64 rounding.
        """
        import torch

        N = self.n_atoms
        L1, L2, L3 = self.dims
        k, kind, norm = self.functions
        f_lo = mode0 // 3
        f_hi = (mode0 + n_rows - 1) // 3 + 1
        kk = torch.as_tensor(k[f_lo:f_hi], device=device)
        w = torch.tensor([L2 * L3, L1 * L3, L1 * L2], dtype=torch.int64, device=device)
        r = torch.as_tensor(self.positions, device=device)
        kw = kk * w
        p = kw[:, 0:1] * r[None, :, 0] + kw[:, 1:2] * r[None, :, 1] + kw[:, 2:3] * r[None, :, 2]
        p = torch.remainder(p, N).to(torch.float64) * (2.0 * math.pi / N)
        is_sin = torch.as_tensor(kind[f_lo:f_hi] == 2, device=device)[:, None]
        phi = torch.where(is_sin, torch.sin(p), torch.cos(p)) * torch.as_tensor(
            norm[f_lo:f_hi], device=device)[:, None]
        out = torch.zeros((n_rows, 3 * N), dtype=torch.float64, device=device)
        m = torch.arange(mode0, mode0 + n_rows, device=device)
        f = torch.div(m, 3, rounding_mode="floor") - f_lo
        alpha = m % 3
        cols = 3 * torch.arange(N, device=device)[None, :] + alpha[:, None]
        out.scatter_(1, cols, phi[f])
        return out

    # ------------------------------------------------------------ frequencies
    @property
    def omega0(self) -> float:
        """sqrt(K/m) in rad/fs."""
        return math.sqrt(self.spring / (self.mass * AMU_A2_PER_FS2_IN_EV))

    def _freq_of_k(self, kvec: np.ndarray) -> np.ndarray:
        L = np.asarray(self.dims, dtype=np.int64)
        folded = np.minimum(kvec, L - kvec)
        s2 = np.sin(np.pi * folded.astype(np.float64) / L.astype(np.float64)) ** 2
        s2 = np.sort(s2, axis=1)
        tot = (s2[:, 0] + s2[:, 1]) + s2[:, 2]
        omega = 2.0 * self.omega0 * np.sqrt(tot)          # rad/fs
        return omega * (1000.0 / (2.0 * math.pi))          # THz

    @cached_property
    def frequencies(self) -> np.ndarray:
        """Mode frequencies in THz, shape [3N], in mode order."""
        k, _, _ = self.functions
        return np.repeat(self._freq_of_k(k), 3)

    def kpoint_frequencies(self) -> np.ndarray:
        """Frequency of every k-index of the full grid, shape [L1, L2, L3]."""
        L1, L2, L3 = self.dims
        n = np.stack(np.meshgrid(np.arange(L1), np.arange(L2), np.arange(L3),
                                 indexing="ij"), axis=-1).reshape(-1, 3)
        return self._freq_of_k(n).reshape(L1, L2, L3)

    @property
    def f_max(self) -> float:
        """Upper edge of the spectrum: all three sin^2 terms equal to one."""
        tot = (1.0 + 1.0) + 1.0
        return 2.0 * self.omega0 * math.sqrt(tot) * (1000.0 / (2.0 * math.pi))


# ---------------------------------------------------------------- masses
def masses(n_atoms: int, kind: str = "uniform", seed: int = 0) -> np.ndarray:
    """Atomic masses in amu: 'uniform' Si or the natural-Si isotope mix."""
    if kind == "uniform":
        return np.full(n_atoms, SI_MASS_AMU, dtype=np.float64)
    if kind == "natural":
        rng = np.random.default_rng([seed, 0x5151])
        iso = np.array([m for m, _ in SI_ISOTOPES])
        p = np.array([w for _, w in SI_ISOTOPES])
        return iso[rng.choice(len(iso), size=n_atoms, p=p / p.sum())]
    raise ValueError(kind)


def velocity_sigma(mass_amu: np.ndarray, temperature: float) -> np.ndarray:
    """Maxwell-Boltzmann standard deviation per component, A/fs."""
    return np.sqrt(KB_EV_PER_K * temperature / (np.asarray(mass_amu) * AMU_A2_PER_FS2_IN_EV))


# ------------------------------------------------------------ trajectories
def gen_steps(seed: int, mass_amu: np.ndarray, step0: int, n_steps: int,
              temperature: float = 300.0, w_sigma: float = 1.0):
    """Velocities and virials for steps [step0, step0 + n_steps).

    Returns (v [n, N, 3] float32 in A/fs, W [n, N, 3, 3] float32 in eV) with
    W[s, i, mu, nu] the per-atom virial component W_i^{mu nu}.  Each step has
    its own PCG64 stream seeded by (seed, step), so any range can be drawn
    independently and chunking does not change the values.  Draws are made
    in float64 and rounded once to float32; consumers that work in float64
    promote the rounded values.
    """
    m = np.asarray(mass_amu, dtype=np.float64)
    N = m.shape[0]
    sig = velocity_sigma(m, temperature)[:, None]
    v = np.empty((n_steps, N, 3), dtype=np.float32)
    W = np.empty((n_steps, N, 3, 3), dtype=np.float32)
    for s in range(n_steps):
        rng = np.random.Generator(np.random.PCG64([seed, step0 + s]))
        v[s] = (rng.standard_normal((N, 3)) * sig).astype(np.float32)
        W[s] = (rng.standard_normal((N, 3, 3)) * w_sigma).astype(np.float32)
    return v, W


def gen_steps_torch(seed: int, mass_amu, n_steps: int, temperature: float = 300.0,
                    w_sigma: float = 1.0, device="cuda"):
    """Large trajectories drawn directly in device memory with torch.

    Same distributions as :func:`gen_steps` but a different random stream;
    for throughput runs whose inputs are too large to draw on the host.
    """
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    m = torch.as_tensor(np.asarray(mass_amu, dtype=np.float64), device=device)
    sig = torch.sqrt(KB_EV_PER_K * temperature / (m * AMU_A2_PER_FS2_IN_EV)).to(torch.float32)
    N = m.shape[0]
    v = torch.randn((n_steps, N, 3), generator=g, device=device, dtype=torch.float32) * sig[None, :, None]
    W = torch.randn((n_steps, N, 3, 3), generator=g, device=device, dtype=torch.float32) * w_sigma
    return v, W


def random_orthonormal(n: int, seed: int) -> np.ndarray:
    """A dense random orthonormal n x n matrix (QR of a Gaussian), float64."""
    rng = np.random.default_rng([seed, 0x0E0E])
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))[None, :]


# ------------------------------------------------------------ atomic structures
SI_LATTICE_A = 5.432                    # diamond-cubic Si lattice constant, A


def diamond(cells, a: float = SI_LATTICE_A, sigma: float = 0.0, seed: int = 0):
    """Diamond-cubic crystal of cells = (n1, n2, n3) conventional cells (8 atoms
    each) in a periodic orthorhombic box, every atom displaced by an iid
    Gaussian of standard deviation sigma (A) per component.

    Returns (pos [N, 3] float64 in [0, box), box [3] float64).  Atom order:
    cell (c1, c2, c3) row-major, then the 8 basis sites."""
    n1, n2, n3 = cells
    basis = np.array([[0, 0, 0], [0, 2, 2], [2, 0, 2], [2, 2, 0],
                      [1, 1, 1], [1, 3, 3], [3, 1, 3], [3, 3, 1]], dtype=np.float64) * (a / 4.0)
    c = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), axis=-1).reshape(-1, 3)
    pos = (c[:, None, :] * a + basis[None, :, :]).reshape(-1, 3)
    box = np.array([n1, n2, n3], dtype=np.float64) * a
    if sigma > 0:
        rng = np.random.Generator(np.random.PCG64([seed, 0xD1A3]))
        pos = pos + rng.standard_normal(pos.shape) * sigma
    return np.mod(pos, box), box


def thermal_velocities(mass_amu: np.ndarray, temperature: float, seed: int) -> np.ndarray:
    """Maxwell-Boltzmann velocities [N, 3] float64 (A/fs), one PCG64 stream per seed."""
    rng = np.random.Generator(np.random.PCG64([seed, 0x7E10]))
    m = np.asarray(mass_amu, dtype=np.float64)
    return rng.standard_normal((m.shape[0], 3)) * velocity_sigma(m, temperature)[:, None]


# --------------------------------------------------------------- workloads
@dataclass(frozen=True)
class Workload:
    """One synthetic workload: lattice, run length, batching and binning."""
    name: str
    dims: tuple
    n_steps: int
    t_block: int
    n_bins: int
    corr_len: int = 0
    seed: int = 0
    temperature: float = 300.0

    @property
    def lattice(self) -> BlochLattice:
        return BlochLattice(self.dims)

    @property
    def n_atoms(self) -> int:
        return int(np.prod(self.dims))


WORKLOADS = {
    # 4x4x4 simple cubic, 64 atoms / 192 modes, 1000 steps, 100 bins
    "sc4_hnema": Workload("sc4_hnema", (4, 4, 4), 1000, 1, 100),
    # 16^3, 4096 atoms / 12288 modes, 10^4 steps, per-step (T=1), 500 bins
    "sc16_hnema_t1": Workload("sc16_hnema_t1", (16, 16, 16), 10000, 1, 500),
    # 48x48x4 slab, 9216 atoms / 27648 modes, 2*10^4 steps, T=128, 1000 bins
    "slab48_hnema_t128": Workload("slab48_hnema_t128", (48, 48, 4), 20000, 128, 1000),
    # 4x4x1500 rod, 24000 atoms / 72000 modes, 5*10^4 steps, T=256, L=2000, 1000 bins
    "rod1500_gkma_t256": Workload("rod1500_gkma_t256", (4, 4, 1500), 50000, 256, 1000, 2000),
}

# Uneven batch: 16 simple-cubic systems with edge lengths drawn by seed.
UNEVEN_EDGES = (8, 10, 12, 14, 16, 20)


def uneven_batch(seed: int = 0, n_systems: int = 16):
    """[(edge, method)] for the uneven serving-style batch; method 1=HNEMA, 2=GKMA."""
    rng = np.random.Generator(np.random.PCG64([seed, 0xBA7C]))
    edges = rng.choice(UNEVEN_EDGES, size=n_systems)
    meth = rng.choice([1, 2], size=n_systems)
    return [(int(e), int(mm)) for e, mm in zip(edges, meth)]
