"""Degenerate and boundary shapes on the GPU against the FP64 oracle, through
the C ABI: one atom (three zero-frequency modes), one bin (every mode: the
bin's current is the Eq. 10 total), one lag, more lags than samples (those
lags stay zero), a one-mode subset, a block longer than the whole
trajectory, empty pushes and reads before any sample; and a group that holds
a one-atom system beside larger ones.  Bars as for the other parity tests
(relative L2 per output array: float32 1e-5, split-BF16 1e-4; float64 totals
1e-12)."""
import numpy as np
import pytest

import oracle
import synth
from tests._cases import TOL, announce, log, rel

pytestmark = pytest.mark.gpu

HNEMA, GKMA = 1, 2
FP32, BF16X3 = 0, 1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


class Tiny:
    """A lattice, its first M modes, explicit bins mode % nb, S samples."""

    def __init__(self, dims, M, nb, S, seed):
        self.lat = synth.BlochLattice(dims)
        N = self.lat.n_atoms
        self.M = 3 * N if M is None else M
        self.E = self.lat.eig_matrix()[:, :self.M]
        self.freq = np.asarray(self.lat.frequencies[:self.M], dtype=np.float64)
        self.m = synth.masses(N, "natural", seed)
        self.v, self.W = synth.gen_steps(seed, self.m, 0, S)
        self.nb = nb
        self.bins = (np.arange(self.M) % nb).astype(np.int32)

    def oracle(self, L):
        return oracle.run_dense(self.E, self.m, self.v, self.W, self.bins, self.nb, corr_len=L, dt=1.0)

    def context(self, methods, prec, T, L, stream=None):
        from paper_2102_03691_amd import ModalHC
        h = ModalHC(0, stream=stream)
        h.load_system(self.m, self.freq)
        h.set_bins(self.nb, self.bins)
        h.configure(methods=methods, precision=prec, t_block=T, corr_len=L, dt=1.0)
        h.load_eigvec_rows(0, np.ascontiguousarray(self.E.T))
        h.finalize()
        return h


# name: dims, M (None: all 3N), nb, L, T, precision, S, push sizes
CASES = {
    "one_atom_fp32_lags_past_samples": ((1, 1, 1), None, 3, 100, 32, FP32, 70, [1, 0, 69]),
    "one_atom_bf16x3_one_bin": ((1, 1, 1), None, 1, 5, 64, BF16X3, 70, [70]),
    "one_atom_per_step": ((1, 1, 1), None, 3, 10, 1, FP32, 20, [7, 13]),
    "one_bin_sum_rule": ((4, 3, 3), None, 1, 8, 64, BF16X3, 150, [150]),
    "one_lag": ((4, 3, 3), None, 7, 1, 32, FP32, 100, [33, 0, 67]),
    "one_mode": ((4, 3, 3), 1, 1, 12, 64, BF16X3, 90, [90]),
    "block_longer_than_run": ((4, 3, 3), None, 5, 20, 512, BF16X3, 37, [37]),
}


@pytest.mark.parametrize("name", list(CASES))
def test_edge_case(name):
    dims, M, nb, L, T, prec, S, splits = CASES[name]
    announce(f"edge {name}")
    c = Tiny(dims, M, nb, S, seed=31)
    ref = c.oracle(L)
    h = c.context(HNEMA | GKMA, prec, T, L)
    # reads before any sample: zero averages and correlations, S = 0
    avg0, tot0, n0 = h.read_hnema()
    g0 = h.read_gkma()
    assert n0 == 0 and g0["n_samples"] == 0
    assert not avg0.any() and not tot0.any() and not g0["corr"].any() and not g0["hcacf"].any()
    s0 = 0
    for n in splits:
        h.push(c.v[s0:s0 + n], c.W[s0:s0 + n])
        s0 += n
    assert s0 == S
    avg, tot, n_h = h.read_hnema()
    g = h.read_gkma()
    h.close()
    bar = TOL[0] if prec == FP32 else TOL[1]
    e = {"rel_hnema": rel(avg, ref["hnema"]), "rel_corr": rel(g["corr"], ref["corr"]),
         "rel_integral": rel(g["integral"], ref["integral"]), "rel_total": rel(tot, ref["hnema_total"]),
         "rel_hcacf": rel(g["hcacf"], ref["hcacf"])}
    log(f"edge_{name}", **e)
    assert n_h == S and g["n_samples"] == S
    for k in ("rel_hnema", "rel_corr", "rel_integral"):
        assert e[k] <= bar, k
    assert e["rel_total"] <= 1e-12 and e["rel_hcacf"] <= 1e-12
    if L > S:
        # no origin pairs at lags >= S: exactly zero on both sides
        assert not g["corr"][S:].any() and not g["hcacf"][S:].any()
        assert not ref["corr"][S:].any()
    if nb == 1 and c.M == 3 * c.lat.n_atoms:
        # a complete basis in one bin: the bin's current is the Eq. 10 total
        assert rel(avg[0], tot) <= bar


def test_group_with_a_one_atom_system():
    """A group of a one-atom system, a 12-atom system and a 36-atom system
    (graph replay), pushed in uneven pieces, against the oracle per system."""
    import torch
    from paper_2102_03691_amd import ModalGroup
    announce("edge group with a one-atom system")
    S, L, T = 64 * 2 + 9, 16, 64
    systems = [Tiny((1, 1, 1), None, 2, S, seed=41), Tiny((3, 2, 2), None, 4, S, seed=42),
               Tiny((4, 3, 3), None, 6, S, seed=43)]
    # one explicit stream: a null handle (torch's default stream) gives every
    # context a stream of its own, and a group needs them to share one
    stream = torch.cuda.Stream()
    hs = [c.context(HNEMA | GKMA, BF16X3, T, L, stream=stream.cuda_stream) for c in systems]
    grp = ModalGroup(hs, graph=True, autotune=False)
    dev = [(torch.as_tensor(c.v, device="cuda:0"), torch.as_tensor(c.W, device="cuda:0")) for c in systems]
    s0 = 0
    for n in (70, 0, 58, 9):
        grp.push([v[s0:s0 + n] for v, _ in dev], [W[s0:s0 + n] for _, W in dev])
        s0 += n
    assert s0 == S
    for i, (c, h) in enumerate(zip(systems, hs)):
        ref = c.oracle(L)
        avg, tot, n = h.read_hnema()
        g = h.read_gkma()
        e = {"rel_hnema": rel(avg, ref["hnema"]), "rel_corr": rel(g["corr"], ref["corr"]),
             "rel_total": rel(tot, ref["hnema_total"])}
        log(f"edge_group_sys{i}", **e)
        assert n == S and g["n_samples"] == S
        assert e["rel_hnema"] <= TOL[1] and e["rel_corr"] <= TOL[1] and e["rel_total"] <= 1e-12
    grp.close()
    for h in hs:
        h.close()


def test_maximum_lags():
    """corr_len = 65536, the largest the API takes, on a small system: the
    first 300 lags against the oracle, every later lag exactly zero."""
    announce("edge maximum lags (65536) fp32 T=64")
    L, S = 65536, 300
    c = Tiny((2, 2, 2), None, 2, S, seed=51)
    ref = c.oracle(L)
    h = c.context(HNEMA | GKMA, FP32, 64, L)
    h.push(c.v[:100], c.W[:100])
    h.push(c.v[100:], c.W[100:])
    g = h.read_gkma()
    h.close()
    e = {"rel_corr": rel(g["corr"][:S], ref["corr"][:S]), "rel_integral": rel(g["integral"], ref["integral"]),
         "rel_hcacf": rel(g["hcacf"], ref["hcacf"])}
    log("edge_max_lags", **e)
    assert g["corr"].shape[0] == L and g["n_samples"] == S
    assert e["rel_corr"] <= TOL[0] and e["rel_integral"] <= TOL[0] and e["rel_hcacf"] <= 1e-12
    assert not g["corr"][S:].any() and not g["hcacf"][S:].any()


def test_maximum_bins():
    """n_bins = 2^20, the largest the API takes, with the 108 modes of a
    4x3x3 lattice spread over it (the last bin included): the bins that hold
    modes against the oracle on the same map compacted to those bins (a
    bin's current does not depend on its label), every other bin exactly
    zero, for HNEMA and a two-lag GKMA."""
    announce("edge maximum bins (2^20) bf16x3 T=32")
    nb, L, S = 1 << 20, 2, 96
    c = Tiny((4, 3, 3), None, 1, S, seed=52)
    bins = ((np.arange(c.M) * 9973) % nb).astype(np.int32)
    bins[0] = nb - 1
    used, compact = np.unique(bins, return_inverse=True)
    ref = oracle.run_dense(c.E, c.m, c.v, c.W, compact.astype(np.int32), len(used), corr_len=L, dt=1.0)
    c.nb, c.bins = nb, bins
    h = c.context(HNEMA | GKMA, BF16X3, 32, L)
    h.push(c.v, c.W)
    avg, tot, n = h.read_hnema()
    g = h.read_gkma()
    h.close()
    empty = np.ones(nb, bool)
    empty[used] = False
    e = {"rel_hnema": rel(avg[used], ref["hnema"]), "rel_corr": rel(g["corr"][:, used], ref["corr"]),
         "rel_total": rel(tot, ref["hnema_total"])}
    log("edge_max_bins", **e)
    assert n == S and avg.shape == (nb, 3) and g["corr"].shape == (L, nb, 3, 3)
    assert e["rel_hnema"] <= TOL[1] and e["rel_corr"] <= TOL[1] and e["rel_total"] <= 1e-12
    assert not avg[empty].any() and not g["corr"][:, empty].any()
