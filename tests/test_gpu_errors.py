"""Error paths on the GPU, through the C ABI: non-finite device inputs with
check_finite (single and grouped pushes), and a basis larger than the
device's memory (MHC_ERR_OOM with nothing kept, the context still usable).
None of these makes a kernel fault: the checks run before any accumulation,
and a failed hipMalloc only returns an error."""
import numpy as np
import pytest

from tests._cases import TOL, Case, announce, rel

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


def _ctx(case, nb, methods, prec, T, L=0, check=True, stream=None):
    from paper_2102_03691_amd import ModalHC
    h = ModalHC(0, stream=stream)
    h.load_system(case.m, case.freq)
    h.set_bins_uniform(nb, 0.0, case.lat.f_max)
    h.configure(methods=methods, precision=prec, t_block=T, corr_len=L, dt=1.0, check_finite=check)
    h.load_eigvec_rows(0, case.lat.eig_rows(0, case.n_modes))
    h.finalize()
    return h


@pytest.mark.parametrize("prec,T", [(BF16X3, 64), (FP32, 1)])
def test_device_nonfinite_input_is_rejected_before_accumulation(prec, T):
    import torch
    from paper_2102_03691_amd import MhcError
    announce(f"non-finite device input prec={prec} T={T}")
    c = Case((4, 4, 3), 200, seed=5)
    v = torch.as_tensor(c.v, device="cuda:0")
    W = torch.as_tensor(c.W, device="cuda:0")
    good = _ctx(c, 9, HNEMA | GKMA, prec, T, L=12)
    h = _ctx(c, 9, HNEMA | GKMA, prec, T, L=12)
    good.push(v[:100], W[:100])
    h.push(v[:100], W[:100])
    for bad_kind, idx in [("nan", (37, 5, 2)), ("inf", (0, 0, 0)), ("-inf", (99, 47, 1))]:
        bv = v[100:].clone()
        bW = W[100:].clone()
        val = {"nan": float("nan"), "inf": float("inf"), "-inf": float("-inf")}[bad_kind]
        if bad_kind == "nan":
            bv[idx] = val
        else:
            bW[idx + (2,)] = val
        with pytest.raises(MhcError) as ei:
            h.push(bv, bW)
        assert ei.value.status == 6
    assert h.read_hnema()[2] == 100                  # nothing of the rejected pushes was accumulated
    good.push(v[100:], W[100:])
    h.push(v[100:], W[100:])
    a, b = good.read_hnema(), h.read_hnema()
    ga, gb = good.read_gkma(), h.read_gkma()
    assert a[2] == b[2] == 200
    np.testing.assert_array_equal(b[0], a[0])
    np.testing.assert_array_equal(gb["corr"], ga["corr"])
    ref = c.oracle(9, corr_len=12)
    assert rel(b[0], ref["hnema"]) <= TOL[prec] and rel(gb["corr"], ref["corr"]) <= TOL[prec]
    good.close()
    h.close()


@pytest.mark.parametrize("device_inputs", [True, False])
def test_group_push_checks_member_inputs(device_inputs):
    import torch
    from paper_2102_03691_amd import MhcError, ModalGroup
    announce(f"grouped non-finite check device_inputs={device_inputs}")
    cases = [Case((4, 4, 3), 128, seed=6), Case((3, 3, 3), 128, seed=7)]
    stream = torch.cuda.Stream()                     # grouped contexts share one stream
    hs = [_ctx(cases[0], 7, HNEMA, BF16X3, 64, check=False, stream=stream.cuda_stream),
          _ctx(cases[1], 5, GKMA, BF16X3, 64, L=8, check=True, stream=stream.cuda_stream)]
    g = ModalGroup(hs, graph=False, autotune=False)
    vs = [c.v.copy() for c in cases]
    Ws = [c.W.copy() for c in cases]
    Ws[1][70, 3, 1, 2] = np.nan                      # second block of the checked system
    if device_inputs:
        vs = [torch.as_tensor(x, device="cuda:0") for x in vs]
        Ws = [torch.as_tensor(x, device="cuda:0") for x in Ws]
    with pytest.raises(MhcError) as ei:
        g.push(vs, Ws)
    assert ei.value.status == 6
    assert hs[0].read_hnema()[2] == 0 and hs[1].read_gkma()["n_samples"] == 0   # no system advanced
    # a non-finite value in an unchecked system is not looked for
    vs2 = [c.v.copy() for c in cases]
    Ws2 = [c.W.copy() for c in cases]
    if device_inputs:
        vs2 = [torch.as_tensor(x, device="cuda:0") for x in vs2]
        Ws2 = [torch.as_tensor(x, device="cuda:0") for x in Ws2]
    g.push(vs2, Ws2)
    assert hs[0].read_hnema()[2] == 128 and hs[1].read_gkma()["n_samples"] == 128
    g.close()
    for h in hs:
        h.close()


def test_basis_larger_than_device_memory_is_oom():
    """A split-BF16 basis of 95000 atoms (285000 modes) needs about 325 GB, more
    than the 288 GB of HBM: the first row load returns MHC_ERR_OOM, keeps no
    device memory, and the context is not put in an error state (the same
    call fails the same way again; other contexts on the device work)."""
    from paper_2102_03691_amd import MhcError, ModalHC
    announce("basis larger than device memory")
    N = 95000
    h = ModalHC(0)
    h.load_system(np.full(N, 28.0855), np.linspace(0.0, 30.0, 3 * N))
    h.set_bins_uniform(10, 0.0, 30.0)
    h.configure(methods=HNEMA, precision=BF16X3, t_block=128)
    before = h.device_bytes()
    row = np.zeros((1, 3 * N))
    row[0, 0] = 1.0
    for _ in range(2):
        with pytest.raises(MhcError) as ei:
            h.load_eigvec_rows(0, row)
        assert ei.value.status == 3
        assert h.device_bytes() == before
    with pytest.raises(MhcError) as ei:            # still loading: finalize is a state error, not a HIP error
        h.finalize()
    assert ei.value.status == 2
    h.close()
    c = Case((4, 4, 3), 64, seed=8)
    small = _ctx(c, 7, HNEMA, BF16X3, 64, check=False)
    small.push(c.v, c.W)
    assert rel(small.read_hnema()[0], c.oracle(7)["hnema"]) <= TOL[BF16X3]
    small.close()
