"""GPU path vs the FP64 oracle, element by element, through the C ABI.

Sizes are chosen so the oracle finishes in seconds while the kernels still
see several row tiles, several column tiles and a ragged tail in both the
mode and the dof dimension (e.g. 6x6x5: 540 modes -> 768 padded slots, 540
dofs -> 576 padded).  Tolerances are the relative L2 norms per output array
(float32: 1e-5, split-bf16: 1e-4); the total current of Eq. 10 is float64.
"""
import numpy as np
import pytest

from tests._cases import TOL, Case, announce, log, rel, run_library

pytestmark = pytest.mark.gpu

HNEMA, GKMA = 1, 2
FP32, BF16X3 = 0, 1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_03691_amd import library
    library()


@pytest.fixture(scope="module")
def small():
    return Case((6, 6, 5), 300, mass_kind="natural", seed=1)


def test_sc4_per_step_fp32_hnema():
    """4x4x4 simple cubic, 64 atoms, 192 modes, 1000 steps, 100 bins, per-step FP32."""
    announce("sc4 per-step fp32 hnema")
    c = Case((4, 4, 4), 1000, seed=0)
    ref = c.oracle(100)
    got = run_library(c, 100, HNEMA, FP32, 1, splits=[1, 255, 256, 488])
    e = rel(got["hnema"], ref["hnema"])
    et = rel(got["hnema_total"], ref["hnema_total"])
    log("sc4_per_step_fp32_hnema", rel_hnema=e, rel_total=et)
    assert got["n_samples"] == 1000
    assert e <= TOL[FP32] and et <= 1e-12


@pytest.mark.parametrize("prec", [FP32, BF16X3])
@pytest.mark.parametrize("T,sched", [(32, 1), (64, 1), (96, 1), (128, 1), (256, 1), (32, 2), (64, 2), (96, 2),
                                     (128, 2), (256, 2), (32, 3), (64, 3), (256, 3)])
def test_batched_hnema(small, prec, T, sched):
    """sched 1 = one tile per work-group, 2 = stream-K (split tiles + fixup),
    3 = lockstep split (tiles of the last round cut along k)."""
    announce(f"batched hnema prec={prec} T={T} sched={sched}")
    ref = small.oracle(23)
    got = run_library(small, 23, HNEMA, prec, T, schedule=sched)
    e = rel(got["hnema"], ref["hnema"])
    log(f"6x6x5_hnema_p{prec}_T{T}_s{sched}", rel_hnema=e, rel_total=rel(got["hnema_total"], ref["hnema_total"]))
    assert e <= TOL[prec]
    assert rel(got["hnema_total"], ref["hnema_total"]) <= 1e-12


@pytest.mark.parametrize("prec,T,sched", [(FP32, 1, 0), (FP32, 64, 1), (FP32, 128, 2), (BF16X3, 96, 2),
                                          (BF16X3, 128, 1), (BF16X3, 256, 2)])
def test_gkma(small, prec, T, sched):
    announce(f"gkma prec={prec} T={T} sched={sched}")
    L, dt = 40, 0.5
    ref = small.oracle(23, corr_len=L, dt=dt)
    got = run_library(small, 23, GKMA | HNEMA, prec, T, corr_len=L, dt=dt, splits=[77, 1, 150, 72], schedule=sched)
    ec, ei, eh = rel(got["corr"], ref["corr"]), rel(got["integral"], ref["integral"]), rel(got["hcacf"], ref["hcacf"])
    e0 = rel(got["corr"][0], ref["corr"][0])
    eh2 = rel(got["hnema"], ref["hnema"])
    log(f"6x6x5_gkma_p{prec}_T{T}_s{sched}", rel_corr=ec, rel_corr_tau0=e0, rel_integral=ei, rel_hcacf=eh, rel_hnema=eh2)
    assert ec <= TOL[prec] and ei <= TOL[prec] and eh2 <= TOL[prec]
    assert eh <= 1e-12
    assert got["n_samples"] == 300


def test_side_stream_device_inputs(small):
    """A context on a stream other than torch's current one, fed device tensors
    that torch makes on its current stream and frees right after each call:
    the binding orders the context stream after the producer and keeps the
    memory from being reused until it has been read."""
    import torch
    from paper_2102_03691_amd import ModalHC
    announce("side-stream device inputs bf16x3 T=64")
    ref = small.oracle(23)
    side = torch.cuda.Stream()
    h = ModalHC(0, stream=side.cuda_stream)
    h.load_system(small.m, small.freq)
    h.set_bins_uniform(23, 0.0, small.lat.f_max)
    h.configure(methods=HNEMA, precision=BF16X3, t_block=64)
    for r0 in range(0, small.n_modes, 97):
        n = min(97, small.n_modes - r0)
        rows = small.lat.eig_rows_torch(r0, n, device="cuda:0") * 1.0     # produced on the current stream
        h.load_eigvec_rows(r0, rows)
        del rows
    h.finalize()
    s0 = 0
    for n in (64, 64, 100, 72):
        v = torch.as_tensor(small.v[s0:s0 + n], device="cuda:0") * 1.0
        W = torch.as_tensor(small.W[s0:s0 + n], device="cuda:0") * 1.0
        h.push(v, W)
        del v, W
        s0 += n
    got, tot, n = h.read_hnema()
    h.close()
    e = rel(got, ref["hnema"])
    log("6x6x5_side_stream_bf16x3_T64", rel_hnema=e)
    assert n == 300 and e <= TOL[BF16X3]
    assert rel(tot, ref["hnema_total"]) <= 1e-12


def test_block_currents_elementwise(small):
    from paper_2102_03691_amd import ModalHC  # noqa: F401
    announce("block currents elementwise bf16x3 T=128")
    ref = small.oracle(23)
    out = run_library(small, 23, GKMA, BF16X3, 128, corr_len=4, keep=True)
    h = out["handle"]
    last = 300 - 256
    jb = h.read_block_currents(last)                    # [t, nb, 3]
    want = ref["Jb"][256:].transpose(0, 2, 1)          # [t, nb, 3]
    e = rel(jb, want)
    scale = np.abs(want).max()
    log("6x6x5_block_currents_bf16x3", rel=e, max_abs_over_scale=float(np.abs(jb - want).max() / scale))
    h.close()
    assert e <= TOL[BF16X3]
    assert np.abs(jb - want).max() <= 1e-3 * scale


def test_mode_subset_and_explicit_bins():
    announce("mode subset + explicit bins fp32 T=64")
    c = Case((5, 4, 4), 130, mass_kind="natural", seed=4, n_modes=200)
    rng = np.random.default_rng(0)
    bins = rng.integers(-1, 9, size=200).astype(np.int32)
    ref = c.oracle(9, bins=bins)
    got = run_library(c, 9, HNEMA, FP32, 64, bins=bins)
    e = rel(got["hnema"], ref["hnema"])
    log("5x4x4_subset200_fp32", rel_hnema=e)
    assert e <= TOL[FP32]


@pytest.mark.parametrize("sched", [1, 2, 3])
def test_block_split_invariance_and_determinism(small, sched):
    announce(f"split invariance + determinism bf16x3 T=64 sched={sched}")
    a = run_library(small, 23, HNEMA | GKMA, BF16X3, 64, corr_len=16, schedule=sched)
    b = run_library(small, 23, HNEMA | GKMA, BF16X3, 64, corr_len=16, schedule=sched)
    for k in ("hnema", "corr", "integral", "hcacf"):
        assert np.array_equal(a[k], b[k]), k
    c = run_library(small, 23, HNEMA | GKMA, BF16X3, 64, corr_len=16, splits=[1, 7, 64, 228], schedule=sched)
    for k in ("hnema", "corr", "hcacf"):
        assert rel(c[k], a[k]) <= 1e-5, k
    # host pushes of several blocks overlap each copy with the previous block's kernels; device inputs
    # of the same blocks give the same bits
    d = run_library(small, 23, HNEMA | GKMA, BF16X3, 64, corr_len=16, schedule=sched, device_inputs=True)
    for k in ("hnema", "corr", "integral", "hcacf"):
        assert np.array_equal(d[k], a[k]), k


def test_save_and_restore_is_bitwise(small):
    from paper_2102_03691_amd import ModalHC
    announce("save/restore fp32 T=32 gkma+hnema")
    full = run_library(small, 23, HNEMA | GKMA, FP32, 32, corr_len=24, splits=[150, 150], keep=True)
    h1 = full.pop("handle")
    h1.close()
    part = run_library(Case((6, 6, 5), 150, mass_kind="natural", seed=1), 23, HNEMA | GKMA, FP32, 32, corr_len=24,
                       keep=True)
    hp = part["handle"]
    blob = hp.save_state()
    hp.close()
    h2 = ModalHC(0)
    h2.load_system(small.m, small.freq)
    h2.set_bins_uniform(23, 0.0, small.lat.f_max)
    h2.configure(methods=HNEMA | GKMA, precision=FP32, t_block=32, corr_len=24)
    h2.load_eigvec_rows(0, small.lat.eig_rows(0, small.n_modes))
    h2.finalize()
    h2.load_state(blob)
    h2.push(small.v[150:], small.W[150:])
    avg, tot, n = h2.read_hnema()
    g = h2.read_gkma()
    h2.close()
    assert n == 300
    assert np.array_equal(avg, full["hnema"])
    assert np.array_equal(g["corr"], full["corr"])
    assert np.array_equal(g["hcacf"], full["hcacf"])


def test_error_paths_on_gpu(small):
    from paper_2102_03691_amd import MhcError, ModalHC
    announce("error paths")
    h = ModalHC(0)
    with pytest.raises(MhcError) as ei:
        h.finalize()
    assert ei.value.status == 2
    h.load_system(small.m, small.freq)
    h.set_bins_uniform(5, 0.0, small.lat.f_max)
    with pytest.raises(MhcError) as ei:
        h.configure(methods=HNEMA, precision=BF16X3, t_block=1)
    assert ei.value.status == 5
    with pytest.raises(MhcError) as ei:
        h.configure(methods=HNEMA, precision=FP32, t_block=48)
    assert ei.value.status == 1
    h.configure(methods=HNEMA, precision=FP32, t_block=32, check_finite=True)
    h.load_eigvec_rows(0, small.lat.eig_rows(0, 10))
    with pytest.raises(MhcError) as ei:
        h.configure(methods=HNEMA, precision=FP32, t_block=32)
    assert ei.value.status == 2
    with pytest.raises(MhcError) as ei:
        h.finalize()
    assert ei.value.status == 2
    h.load_eigvec_rows(10, small.lat.eig_rows(10, small.n_modes - 10))
    h.finalize()
    v = small.v[:2].copy()
    v[1, 3, 1] = np.nan
    with pytest.raises(MhcError) as ei:
        h.push(v, small.W[:2])
    assert ei.value.status == 6
    avg, tot, n = h.read_hnema()
    assert n == 0 and np.all(avg == 0)
    with pytest.raises(MhcError) as ei:
        h.read_gkma()
    assert ei.value.status == 2
    h.close()


FP8, FP8X3 = 2, 3


@pytest.mark.parametrize("prec,T,sched", [(FP8X3, 64, 1), (FP8X3, 128, 2), (FP8X3, 96, 1), (FP8, 64, 1),
                                          (FP8, 128, 2)])
def test_fp8(small, prec, T, sched):
    """e4m3 with per-mode and per-(channel, step) scales.  FP8X3 (hi/lo, three
    products) must meet the 1e-2 gate; single-term FP8 is reported with its
    measured error (4.1-4.6e-2 here), bounded at 6e-2 so that a regression of
    its accuracy fails; it is not expected to meet 1e-2."""
    announce(f"fp8 prec={prec} T={T} sched={sched}")
    L = 24
    ref = small.oracle(23, corr_len=L)
    got = run_library(small, 23, GKMA | HNEMA, prec, T, corr_len=L, splits=[100, 200], schedule=sched)
    e = {"rel_hnema": rel(got["hnema"], ref["hnema"]), "rel_corr": rel(got["corr"], ref["corr"]),
         "rel_integral": rel(got["integral"], ref["integral"]), "rel_hcacf": rel(got["hcacf"], ref["hcacf"])}
    log(f"6x6x5_fp8_p{prec}_T{T}_s{sched}", **e)
    bound = 1e-2 if prec == FP8X3 else 6e-2
    assert e["rel_hnema"] <= bound and e["rel_corr"] <= bound and e["rel_integral"] <= bound
    assert e["rel_hcacf"] <= 1e-12


@pytest.mark.parametrize("dims,prec,T,n_steps", [((8, 8, 4), BF16X3, 64, 200), ((8, 8, 4), FP32, 32, 200),
                                                 ((12, 12, 8), FP8X3, 128, 200), ((16, 16, 8), BF16X3, 512, 512)])
def test_split_schedule(dims, prec, T, n_steps):
    """Lockstep split with several pieces per tile: 8x8x4 has 24 k-stages and
    3 tiles (3 pieces each, so the fixed-order sum of pieces 2.. runs); the
    12x12x8 FP8X3 case cuts 28 tiles into 6 pieces; 16x16x8 at T = 512 has
    192 tiles, more than half the CUs, so its tiles get a main piece and a
    tail piece, three tails per spare work-group.  Checked against the oracle,
    against the one-tile-per-work-group schedule, and for bitwise
    repeatability."""
    announce(f"split schedule dims={dims} prec={prec} T={T}")
    c = Case(dims, n_steps, mass_kind="natural", seed=5)
    nb = 37
    ref = c.oracle(nb)
    a = run_library(c, nb, HNEMA, prec, T, schedule=3, row_chunk=512)
    b = run_library(c, nb, HNEMA, prec, T, schedule=3, row_chunk=512)
    t = run_library(c, nb, HNEMA, prec, T, schedule=1, row_chunk=512)
    e = rel(a["hnema"], ref["hnema"])
    et = rel(a["hnema"], t["hnema"])
    log(f"{dims[0]}x{dims[1]}x{dims[2]}_split_p{prec}_T{T}", rel_hnema=e, rel_vs_tiles=et)
    assert np.array_equal(a["hnema"], b["hnema"])
    tol = TOL.get(prec, 1e-2)
    assert e <= tol and et <= tol


def test_last_schedule_reports_the_split_used(small):
    """mhc_last_schedule tells which work split ran; on the 6x6x5 case (3 tiles
    of 20 k-stages on a 256-CU device) AUTO resolves to the lockstep split."""
    announce("last schedule query")
    for asked, expect in ((1, 1), (2, 2), (3, 3), (0, 3)):
        got = run_library(small, 23, HNEMA, BF16X3, 64, schedule=asked, keep=True)
        h = got.pop("handle")
        assert h.last_schedule() == expect, (asked, h.last_schedule())
        h.close()
    got = run_library(small, 23, HNEMA, FP32, 1, keep=True)
    h = got.pop("handle")
    assert h.last_schedule() == 0
    h.close()
