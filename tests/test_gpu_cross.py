"""Bin-bin cross-correlations of the modal currents (Sec. II.B.i, Sec. III.C.i)
on the GPU against the FP64 oracle, through the C ABI.

6x6x5 simple cubic (540 modes, ragged padding), 6 frequency bins covering
every mode, L = 24 lags; relative L2 bars as for the GKMA correlation
(float32 1e-5, split-BF16 1e-4, e4m3 hi/lo 1e-2)."""
import numpy as np
import pytest

import oracle
from oracle import cross as ox
from tests._cases import TOL, Case, announce, log, rel, run_library

pytestmark = pytest.mark.gpu

HNEMA, GKMA, DIR, CROSS = 1, 2, 4, 8
FP32, BF16X3, FP8, FP8X3 = 0, 1, 2, 3
BAR = {FP32: TOL[0], BF16X3: TOL[1], FP8X3: 1e-2, FP8: 6e-2}
NB, L, DT = 6, 24, 0.5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def case():
    c = Case((6, 6, 5), 300, mass_kind="natural", seed=12)
    ref = c.oracle(NB, corr_len=L, dt=DT)
    ref["cross"] = ox.gkma_cross_correlation(ref["Jb"], L)
    ref["cross_integral"] = oracle.gkma_running_integral(ref["cross"], DT)
    c.ref = ref
    return c


@pytest.mark.parametrize("prec,T,sched", [(FP32, 1, 0), (FP32, 96, 2), (BF16X3, 64, 3), (BF16X3, 128, 1),
                                          (FP8X3, 128, 0), (FP8, 64, 1)])
def test_cross_parity(case, prec, T, sched):
    announce(f"cross prec={prec} T={T} sched={sched}")
    got = run_library(case, NB, HNEMA | GKMA | CROSS, prec, T, corr_len=L, dt=DT, splits=[77, 1, 150, 72],
                      schedule=sched, keep=True)
    h = got["handle"]
    x = h.read_gkma_cross()
    h.close()
    ref = case.ref
    e = {"rel_cross": rel(x["corr"], ref["cross"]), "rel_cross_integral": rel(x["integral"], ref["cross_integral"]),
         "rel_corr": rel(got["corr"], ref["corr"]), "rel_cross_sum_vs_corr": rel(x["corr"].sum(axis=2), got["corr"])}
    log(f"6x6x5_cross_p{prec}_T{T}_s{sched}", **e)
    assert x["n_samples"] == 300
    assert e["rel_cross"] <= BAR[prec] and e["rel_cross_integral"] <= BAR[prec] and e["rel_corr"] <= BAR[prec]
    # every mode is binned: the sum over the second bin is the correlation with the Eq. 10 total
    assert e["rel_cross_sum_vs_corr"] <= BAR[prec]


def test_cross_save_restore_and_group(case):
    """Bitwise: one single-context run, a run saved after two blocks and resumed
    in a new context, and a grouped push (graph replay) of the same system."""
    import torch
    from paper_2102_03691_amd import ModalGroup, ModalHC
    announce("cross save/restore + group bf16x3 T=64")

    def ctx(stream=None):
        h = ModalHC(0, stream=stream)
        h.load_system(case.m, case.freq)
        h.set_bins_uniform(NB, 0.0, case.lat.f_max)
        h.configure(methods=GKMA | CROSS, precision=BF16X3, t_block=64, corr_len=L, dt=DT, schedule=1)
        h.load_eigvec_rows(0, case.lat.eig_rows(0, case.n_modes))
        h.finalize()
        return h

    a = ctx()
    a.push(case.v, case.W)
    ra = a.read_gkma_cross()
    a.close()
    b = ctx()
    b.push(case.v[:128], case.W[:128])
    st = b.save_state()
    b.close()
    c = ctx()
    c.load_state(st)
    c.push(case.v[128:], case.W[128:])
    rc = c.read_gkma_cross()
    c.close()
    assert np.array_equal(ra["corr"], rc["corr"]) and np.array_equal(ra["integral"], rc["integral"])
    stream = torch.cuda.current_stream().cuda_stream
    g1 = ctx(stream)
    grp = ModalGroup([g1], graph=True, autotune=False)
    v = torch.as_tensor(case.v, device="cuda:0")
    W = torch.as_tensor(case.W, device="cuda:0")
    grp.push([v], [W])
    rg = g1.read_gkma_cross()
    grp.close()
    g1.close()
    assert np.array_equal(ra["corr"], rg["corr"])


def test_cross_invalid_configurations(case):
    from paper_2102_03691_amd import MhcError, ModalHC
    h = ModalHC(0)
    h.load_system(case.m, case.freq)
    h.set_bins_uniform(NB, 0.0, case.lat.f_max)
    with pytest.raises(MhcError) as ei:
        h.configure(methods=HNEMA | CROSS, precision=FP32, t_block=64)
    assert ei.value.status == 1
    with pytest.raises(MhcError) as ei:
        h.configure(methods=GKMA | CROSS | DIR, precision=FP32, t_block=64, corr_len=4)
    assert ei.value.status == 5
    h.configure(methods=GKMA, precision=FP32, t_block=64, corr_len=4)
    h.load_eigvec_rows(0, case.lat.eig_rows(0, case.n_modes))
    h.finalize()
    with pytest.raises(MhcError) as ei:
        h.read_gkma_cross()
    assert ei.value.status == 2
    h.close()


def test_cross_with_excluded_modes():
    """An explicit bin map that leaves out a third of the modes (-1): the cross
    correlations of the remaining bins against the oracle (the sum rule to the
    total no longer holds, parity does)."""
    from paper_2102_03691_amd import ModalHC
    announce("cross excluded modes bf16x3 T=64")
    c = Case((5, 4, 4), 200, mass_kind="natural", seed=13)
    nb, L = 5, 12
    bins = oracle.bin_of_mode(c.freq, nb, 0.0, c.lat.f_max)
    bins[np.arange(c.n_modes) % 3 == 1] = -1
    ref = c.oracle(nb, corr_len=L, bins=bins)
    C = ox.gkma_cross_correlation(ref["Jb"], L)
    got = run_library(c, nb, GKMA | CROSS, BF16X3, 64, corr_len=L, bins=bins, keep=True)
    h = got["handle"]
    x = h.read_gkma_cross()
    h.close()
    e = rel(x["corr"], C)
    log("5x4x4_cross_excluded", rel_cross=e)
    assert x["n_samples"] == 200 and e <= BAR[BF16X3]
