"""Motion-direction split (Sec. II, remark after Eq. 10; closing remark of
Sec. II.C) on the GPU against the FP64 oracle, through the C ABI.  T-batched
contexts run it as one contraction per block over a
direction-major operand (the three per-direction brackets are the
contraction's thirds of K), in every precision; the per-step path runs one
contraction per direction.

The basis is a dense random orthonormal matrix (540 x 540 for 180 atoms), so
every mode moves every atom in every direction and the split is not the
trivial polarisation split of a Bloch basis.  Bars as for the unsplit path:
relative L2 per output array, float32 1e-5, split-BF16 1e-4, e4m3 hi/lo 1e-2;
the float64 Eq. 10 totals 1e-12."""
import numpy as np
import pytest

import oracle
import synth
from oracle import directional as od
from tests._cases import TOL, announce, log, rel

pytestmark = pytest.mark.gpu

HNEMA, GKMA, DIR = 1, 2, 4
FP32, BF16X3, FP8, FP8X3 = 0, 1, 2, 3
BAR = {FP32: TOL[0], BF16X3: TOL[1], FP8X3: 1e-2, FP8: 6e-2}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


class DenseCase:
    def __init__(self, dims=(6, 6, 5), S=300, nb=23, seed=5):
        self.lat = synth.BlochLattice(dims)
        N = self.lat.n_atoms
        self.E = synth.random_orthonormal(3 * N, seed=seed)
        self.m = synth.masses(N, "natural", seed)
        self.v, self.W = synth.gen_steps(seed, self.m, 0, S)
        self.nb = nb
        self.bins = oracle.bin_of_mode(self.lat.frequencies, nb, 0.0, self.lat.f_max)
        self._ref = {}

    def oracle(self, corr_len=0, dt=1.0):
        key = (corr_len, dt)
        if key not in self._ref:
            d = od.run_dense_directional(self.E, self.m, self.v, self.W, self.bins, self.nb, corr_len, dt)
            p = oracle.run_dense(self.E, self.m, self.v, self.W, self.bins, self.nb, corr_len, dt)
            d.update({k: p[k] for k in p if k in ("hnema", "hnema_total", "corr", "integral", "hcacf")})
            self._ref[key] = d
        return self._ref[key]

    def context(self, methods, prec, T, corr_len=0, dt=1.0, schedule=0):
        from paper_2102_03691_amd import ModalHC
        h = ModalHC(0)
        h.load_system(self.m, self.lat.frequencies)
        h.set_bins(self.nb, self.bins)
        h.configure(methods=methods, precision=prec, t_block=T, corr_len=corr_len, dt=dt, schedule=schedule)
        M = self.E.shape[1]
        for r0 in range(0, M, 128):
            h.load_eigvec_rows(r0, np.ascontiguousarray(self.E[:, r0:r0 + 128].T))
        h.finalize()
        return h

    def push(self, h, splits):
        s0 = 0
        for n in splits:
            h.push(self.v[s0:s0 + n], self.W[s0:s0 + n])
            s0 += n
        assert s0 == self.v.shape[0]


@pytest.fixture(scope="module")
def dense():
    return DenseCase()


@pytest.mark.parametrize("prec,T,sched", [(FP32, 1, 0), (FP32, 64, 1), (BF16X3, 128, 3), (BF16X3, 96, 2),
                                          (FP8X3, 64, 1), (FP8, 128, 0)])
def test_hnema_split(dense, prec, T, sched):
    announce(f"directional hnema prec={prec} T={T} sched={sched}")
    ref = dense.oracle()
    h = dense.context(HNEMA | DIR, prec, T, schedule=sched)
    h.set_timing(True)
    dense.push(h, [1, 150, 149])
    launches, _ = h.kernel_timing()
    # T-batched: one contraction per block over the direction-major operand
    # (the per-step path runs one per direction)
    if T > 1:
        assert launches == sum(-(-n // T) for n in (1, 150, 149)), launches
    avg_d, tot_d, n = h.read_hnema_dir()
    avg, tot, n2 = h.read_hnema()
    h.close()
    e = {"rel_hnema_dir": rel(avg_d, ref["hnema_dir"]), "rel_hnema_sum": rel(avg, ref["hnema"]),
         "rel_total_dir": rel(tot_d, ref["hnema_total_dir"]), "rel_total": rel(tot, ref["hnema_total"])}
    log(f"dense540_dir_hnema_p{prec}_T{T}_s{sched}", **e)
    assert n == n2 == 300
    assert e["rel_hnema_dir"] <= BAR[prec] and e["rel_hnema_sum"] <= BAR[prec]
    assert e["rel_total_dir"] <= 1e-12 and e["rel_total"] <= 1e-12


@pytest.mark.parametrize("prec,T,sched", [(FP32, 1, 0), (BF16X3, 64, 1), (BF16X3, 128, 3), (FP8X3, 64, 2),
                                          (FP8, 128, 0)])
def test_gkma_split(dense, prec, T, sched):
    announce(f"directional gkma prec={prec} T={T} sched={sched}")
    L, dt = 30, 0.5
    ref = dense.oracle(L, dt)
    h = dense.context(HNEMA | GKMA | DIR, prec, T, corr_len=L, dt=dt, schedule=sched)
    dense.push(h, [77, 1, 150, 72])
    gd = h.read_gkma_dir()
    g = h.read_gkma()
    avg_d, _, _ = h.read_hnema_dir()
    h.close()
    e = {"rel_corr_dir": rel(gd["corr"], ref["corr_dir"]), "rel_integral_dir": rel(gd["integral"], ref["integral_dir"]),
         "rel_corr_sum": rel(g["corr"], ref["corr"]), "rel_integral_sum": rel(g["integral"], ref["integral"]),
         "rel_hcacf": rel(g["hcacf"], ref["hcacf"]), "rel_hnema_dir": rel(avg_d, ref["hnema_dir"])}
    log(f"dense540_dir_gkma_p{prec}_T{T}_s{sched}", **e)
    assert gd["n_samples"] == g["n_samples"] == 300
    for k in ("rel_corr_dir", "rel_integral_dir", "rel_corr_sum", "rel_integral_sum", "rel_hnema_dir"):
        assert e[k] <= BAR[prec], k
    assert e["rel_hcacf"] <= 1e-12


def test_split_save_restore_and_determinism(dense):
    """Bitwise: one run equals a run saved halfway and resumed in a new context."""
    announce("directional save/restore bf16x3 T=64")
    L = 12
    a = dense.context(HNEMA | GKMA | DIR, BF16X3, 64, corr_len=L)
    dense.push(a, [300])
    ra, ga = a.read_hnema_dir(), a.read_gkma_dir()
    a.close()
    b = dense.context(HNEMA | GKMA | DIR, BF16X3, 64, corr_len=L)
    b.push(dense.v[:128], dense.W[:128])
    state = b.save_state()
    b.close()
    c = dense.context(HNEMA | GKMA | DIR, BF16X3, 64, corr_len=L)
    c.load_state(state)
    c.push(dense.v[128:], dense.W[128:])
    rc, gc = c.read_hnema_dir(), c.read_gkma_dir()
    c.close()
    assert np.array_equal(ra[0], rc[0]) and np.array_equal(ra[1], rc[1])
    assert np.array_equal(ga["corr"], gc["corr"]) and np.array_equal(ga["integral"], gc["integral"])


def test_split_unsupported_paths(dense):
    from paper_2102_03691_amd import MhcError, ModalGroup
    announce("directional unsupported paths")
    h = dense.context(GKMA | DIR, BF16X3, 64, corr_len=4)
    h.push(dense.v[:64], dense.W[:64])
    with pytest.raises(MhcError) as ei:
        h.read_block_currents(8)
    assert ei.value.status == 5
    with pytest.raises(MhcError) as ei:
        h.read_hnema_dir()                         # HNEMA not enabled
    assert ei.value.status == 2
    h.close()
    p = dense.context(HNEMA, BF16X3, 64)
    with pytest.raises(MhcError) as ei:
        p.read_hnema_dir()                         # split not enabled
    assert ei.value.status == 2
    p.close()


def test_split_with_mode_subset_and_excluded_modes():
    """M < 3N modes (the first 400 of a dense 540 x 540 basis) and an explicit
    bin map that excludes every seventh mode (-1): split outputs against the
    split oracle on the same subset and map."""
    from paper_2102_03691_amd import ModalHC
    announce("directional mode subset + excluded modes fp32 T=64")
    c = DenseCase(seed=9)
    M, nb, L = 400, 9, 16
    E = c.E[:, :M]
    bins = (np.arange(M) * 7) % nb
    bins[::7] = -1
    ref = od.run_dense_directional(E, c.m, c.v, c.W, bins, nb, L, 1.0)
    h = ModalHC(0)
    h.load_system(c.m, c.lat.frequencies[:M])
    h.set_bins(nb, bins)
    h.configure(methods=HNEMA | GKMA | DIR, precision=FP32, t_block=64, corr_len=L, dt=1.0)
    for r0 in range(0, M, 100):
        h.load_eigvec_rows(r0, np.ascontiguousarray(E[:, r0:r0 + 100].T))
    h.finalize()
    c.push(h, [200, 100])
    avg_d, _, n = h.read_hnema_dir()
    gd = h.read_gkma_dir()
    h.close()
    e1, e2 = rel(avg_d, ref["hnema_dir"]), rel(gd["corr"], ref["corr_dir"])
    log("dense540_dir_subset400_excl", rel_hnema_dir=e1, rel_corr_dir=e2)
    assert n == 300 and e1 <= BAR[FP32] and e2 <= BAR[FP32]
