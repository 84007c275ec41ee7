"""mhc_push_noalloc (the allocation-free push) against mhc_push on device
inputs, through the C ABI: the same system, configuration and inputs pushed
into two contexts, one through each entry point, two calls in a row (the
second with fewer steps), then a second, smaller system on the same device
(the scratch keeps the previous call's contents).  The work split is the same,
so the results are compared bit for bit, and both against the FP64 oracle at
the precision's bar."""
import numpy as np
import pytest

from tests._cases import TOL, Case, announce, log, rel

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


def _ctx(case, nb, methods, prec, T, L, sched):
    from paper_2102_03691_amd import ModalHC
    h = ModalHC(0)
    h.load_system(case.m, case.freq)
    h.set_bins_uniform(nb, 0.0, case.lat.f_max)
    h.configure(methods=methods, precision=prec, t_block=T, corr_len=L, dt=0.5, schedule=sched)
    h.load_eigvec_rows(0, case.lat.eig_rows(0, case.n_modes))
    h.finalize()
    return h


DIR = 4


def _reads(h, methods):
    out = {}
    if methods & HNEMA:
        out["hnema"], out["hnema_total"], out["n"] = h.read_hnema()
    if methods & GKMA:
        g = h.read_gkma()
        out.update(corr=g["corr"], integral=g["integral"], hcacf=g["hcacf"], n=g["n_samples"])
    if methods & DIR:
        out["hnema_dir"], out["hnema_total_dir"], _ = h.read_hnema_dir()
        gd = h.read_gkma_dir()
        out["corr_dir"], out["integral_dir"] = gd["corr"], gd["integral"]
    return out


@pytest.mark.parametrize("prec,T,sched,split", [(BF16X3, 64, 3, False), (BF16X3, 96, 2, False),
                                                (FP32, 128, 3, False), (BF16X3, 128, 1, False),
                                                (FP32, 1, 0, False), (BF16X3, 64, 0, True)])
def test_noalloc_push_matches_push(prec, T, sched, split):
    """split: the motion-direction split in its one-contraction form, whose
    bracket slots also live in the scratch."""
    import torch
    announce(f"noalloc push prec={prec} T={T} sched={sched} split={split}")
    methods = HNEMA | GKMA | (DIR if split else 0)
    L, nb = 40, 23
    for dims, splits, seed in [((6, 6, 5), [230, 70], 1), ((4, 4, 3), [150, 37], 2)]:
        case = Case(dims, sum(splits), mass_kind="natural", seed=seed)
        ref = case.oracle(nb, corr_len=L, dt=0.5)
        v = torch.as_tensor(case.v, device="cuda:0")
        W = torch.as_tensor(case.W, device="cuda:0")
        a = _ctx(case, nb, methods, prec, T, L, sched)
        b = _ctx(case, nb, methods, prec, T, L, sched)
        s0 = 0
        for n in splits:                       # two calls, the second smaller
            a.push(v[s0:s0 + n], W[s0:s0 + n])
            b.push_noalloc(v[s0:s0 + n], W[s0:s0 + n])
            s0 += n
        assert a.last_schedule() == b.last_schedule()
        ra, rb = _reads(a, methods), _reads(b, methods)
        bytes_a, bytes_b = a.device_bytes(), b.device_bytes()
        a.close()
        b.close()
        assert ra["n"] == rb["n"] == s0
        assert bytes_a == bytes_b
        for k in ra:
            np.testing.assert_array_equal(rb[k], ra[k], err_msg=k)
        e_h, e_c = rel(rb["hnema"], ref["hnema"]), rel(rb["corr"], ref["corr"])
        e_i = rel(rb["integral"], ref["integral"])
        log(f"noalloc_{dims[0]}x{dims[1]}x{dims[2]}_p{prec}_T{T}_s{sched}", rel_hnema=e_h, rel_corr=e_c,
            rel_integral=e_i)
        assert e_h <= TOL[prec] and e_c <= TOL[prec] and e_i <= TOL[prec]
        assert rel(rb["hnema_total"], ref["hnema_total"]) <= 1e-12
        assert rel(rb["hcacf"], ref["hcacf"]) <= 1e-12


def test_noalloc_push_rejects_bad_arguments():
    import torch
    from paper_2102_03691_amd import library
    lib = library()
    assert lib.mhc_push_noalloc(None, 1, None, None) == 1
    case = Case((4, 4, 3), 64, seed=3)
    h = _ctx(case, 7, HNEMA, BF16X3, 64, 0, 0)
    v = torch.as_tensor(case.v, device="cuda:0")
    assert lib.mhc_push_noalloc(h._h, -1, v.data_ptr(), v.data_ptr()) == 1
    assert lib.mhc_push_noalloc(h._h, 4, None, v.data_ptr()) == 1
    assert lib.mhc_push_noalloc(h._h, 0, None, None) == 0
    h.close()
