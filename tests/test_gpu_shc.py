"""Spectral heat current (Sec. II.C, Eqs. 21-22) on the GPU against the FP64
oracle, through the C ABI.  The device forms the float32 inputs' products
exactly in float64 and sums in float64, so the bar is 1e-12 relative (L2 per
output array); summation order differs from numpy's, nothing else."""
import numpy as np
import pytest

import oracle
import synth
from tests._cases import announce, log, rel

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _inputs(n_atoms, S, seed):
    m = synth.masses(n_atoms, "natural", seed)
    return synth.gen_steps(seed, m, 0, S)


def _run(n_atoms, v, W, n_lags, T, splits, device_inputs):
    import torch
    from paper_2102_03691_amd import ModalSHC
    h = ModalSHC(n_atoms, n_lags, T)
    if device_inputs:
        v = torch.as_tensor(v, device="cuda:0")
        W = torch.as_tensor(W, device="cuda:0")
    s0 = 0
    for n in splits:
        h.push(v[s0:s0 + n], W[s0:s0 + n])
        s0 += n
    assert s0 == v.shape[0]
    K, S = h.read()
    return h, K, S


@pytest.mark.parametrize("n_atoms,S,n_lags,T,splits,dev", [
    (37, 300, 70, 64, [1, 63, 100, 136], False),           # ragged dofs (111), ragged lag tile, uneven pushes
    (200, 500, 130, 128, [500], True),                     # lags longer than a block: history across blocks
    (64, 40, 100, 64, [17, 23], True),                     # more lags than samples: empty lags are zero
    (1000, 700, 256, 256, [256, 256, 188], True),          # several dof ranges per work-group split
])
def test_shc_correlation_parity(n_atoms, S, n_lags, T, splits, dev):
    announce(f"shc N={n_atoms} S={S} L={n_lags} T={T}")
    v, W = _inputs(n_atoms, S, seed=n_atoms + S)
    h, K, n = _run(n_atoms, v, W, n_lags, T, splits, dev)
    ref = oracle.shc_correlation(v, W, n_lags)
    e = rel(K, ref)
    e0 = rel(K[0], oracle.total_heat_current(v, W).mean(axis=0))
    log(f"shc_N{n_atoms}_S{S}_L{n_lags}_T{T}", rel_K=e, rel_K0_vs_eq10=e0)
    assert n == S
    assert e <= TOL and e0 <= TOL
    if n_lags > S:
        assert np.all(K[S:] == 0.0)
    # the motion-direction split, accumulated alongside
    Kd, nd = h.read_dir()
    ref_d = oracle.shc_correlation_directional(v, W, n_lags)
    ed = rel(Kd, ref_d)
    log(f"shc_dir_N{n_atoms}_S{S}_L{n_lags}_T{T}", rel_K_dir=ed)
    assert nd == S and ed <= TOL
    # K is the device's in-order float64 sum of the three split components
    assert np.array_equal(K, (Kd[:, :, 0] + Kd[:, :, 1]) + Kd[:, :, 2])
    assert rel(Kd.sum(axis=2), K) <= 1e-14
    # transform of the device correlation against the oracle's transform of the oracle's correlation
    om = np.linspace(0.0, np.pi / 2.0, 33)
    for window in (False, True):
        Kw = h.spectrum(om, 2.0, window)
        ref_w = oracle.shc_spectrum(ref, 2.0, om, window)
        ew = rel(Kw, ref_w)
        Kwd = h.spectrum_dir(om, 2.0, window)
        ref_wd = oracle.shc_spectrum(ref_d.reshape(n_lags, 9), 2.0, om, window).reshape(-1, 3, 3)
        ewd = rel(Kwd, ref_wd)
        log(f"shc_spectrum_N{n_atoms}_w{int(window)}", rel_Kw=ew, rel_Kw_dir=ewd)
        assert ew <= 1e-11 and ewd <= 1e-11
    h.close()


def test_shc_determinism_split_invariance_and_reset():
    announce("shc determinism / reset")
    n_atoms, S, L, T = 120, 400, 90, 64
    v, W = _inputs(n_atoms, S, seed=7)
    h1, K1, _ = _run(n_atoms, v, W, L, T, [S], True)
    h2, K2, _ = _run(n_atoms, v, W, L, T, [S], True)
    assert np.array_equal(K1, K2)
    h3, K3, _ = _run(n_atoms, v, W, L, T, [5, 100, 1, 294], True)
    assert rel(K3, K1) <= 1e-13
    # the same blocks pushed from host memory (copies overlapped with the kernels): bitwise equal
    h5, K5, _ = _run(n_atoms, v, W, L, T, [S], False)
    assert np.array_equal(K5, K1)
    h5.close()
    # reset, then a different run: only the new samples count
    import torch
    v2, W2 = _inputs(n_atoms, 150, seed=8)
    h1.reset()
    h1.push(torch.as_tensor(v2, device="cuda:0"), torch.as_tensor(W2, device="cuda:0"))
    K4, n4 = h1.read()
    assert n4 == 150
    assert rel(K4, oracle.shc_correlation(v2, W2, L)) <= TOL
    for h in (h1, h2, h3):
        h.close()


def test_shc_save_restore_is_bitwise():
    """A run saved after 128 samples (a block boundary) and resumed in a new
    object equals the uninterrupted run bit for bit (lags reach back across
    the saved point); saved mid-block, it agrees to rounding."""
    import torch
    from paper_2102_03691_amd import ModalSHC
    announce("shc save/restore")
    n_atoms, S, L, T = 150, 300, 90, 64
    v, W = _inputs(n_atoms, S, seed=31)
    dv, dW = torch.as_tensor(v, device="cuda:0"), torch.as_tensor(W, device="cuda:0")
    a = ModalSHC(n_atoms, L, T)
    a.push(dv, dW)
    Ka, Kda = a.read()[0], a.read_dir()[0]
    b = ModalSHC(n_atoms, L, T)
    b.push(dv[:128], dW[:128])
    st = b.save_state()
    b.close()
    c = ModalSHC(n_atoms, L, T)
    c.load_state(st)
    c.push(dv[128:], dW[128:])
    Kc, n = c.read()
    assert n == S and np.array_equal(Ka, Kc) and np.array_equal(Kda, c.read_dir()[0])
    assert rel(Kc, oracle.shc_correlation(v, W, L)) <= TOL
    e = ModalSHC(n_atoms, L, T)
    e.push(dv[:130], dW[:130])
    st2 = e.save_state()
    e.close()
    f = ModalSHC(n_atoms, L, T)
    f.load_state(st2)
    f.push(dv[130:], dW[130:])
    assert rel(f.read()[0], Ka) <= 1e-13
    f.close()
    d = ModalSHC(n_atoms, L + 1, T)
    from paper_2102_03691_amd import MhcError
    with pytest.raises(MhcError):
        d.load_state(st)
    for h in (a, c, d):
        h.close()


def test_shc_invalid_arguments():
    from paper_2102_03691_amd import MhcError, ModalSHC
    with pytest.raises(MhcError):
        ModalSHC(10, 0, 64)
    with pytest.raises(MhcError):
        ModalSHC(10, 8, 96)
    h = ModalSHC(10, 8, 64)
    with pytest.raises(MhcError):
        h.spectrum([0.0], -1.0)
    with pytest.raises(MhcError):
        h.spectrum([float("nan")], 1.0)
    # before any sample, and after an empty push: S = 0 and every lag zero
    K, n = h.read()
    assert n == 0 and not K.any()
    v, W = _inputs(10, 3, seed=3)
    h.push(v[:0], W[:0])
    K, n = h.read()
    assert n == 0 and not K.any()
    h.push(v, W)
    K, n = h.read()
    assert n == 3 and rel(K, oracle.shc_correlation(v, W, 8)) <= TOL
    assert not K[3:].any()
    # timing events around every k-th block; k < 0 is an error
    with pytest.raises(MhcError) as ei:
        h.set_timing(-1)
    assert ei.value.status == 1
    for k, timed in ((3, 3), (1, 7)):
        h.set_timing(k)
        for _ in range(7):
            h.push(v, W)
        launches, ms = h.kernel_timing()
        assert launches == timed and ms > 0.0
    h.set_timing(False)
    h.close()


def test_shc_paper_shaped_size():
    """8000 atoms (the paper's Si and CNT sizes, Sec. III.A), 250 lags (500 fs
    at a 2 fs sample interval, Sec. III.A.i), T = 256, 600 samples."""
    announce("shc 8000 atoms L=250 T=256")
    n_atoms, S, L, T = 8000, 600, 250, 256
    v, W = _inputs(n_atoms, S, seed=11)
    h, K, n = _run(n_atoms, v, W, L, T, [256, 256, 88], True)
    ref = oracle.shc_correlation(v, W, L)
    e = rel(K, ref)
    Kd, _ = h.read_dir()
    ed = rel(Kd, oracle.shc_correlation_directional(v, W, L))
    log("shc_N8000_S600_L250_T256", rel_K=e, rel_K_dir=ed)
    assert n == S and e <= TOL and ed <= TOL
    h.close()


def test_shc_maximum_lags_and_block():
    """n_lags = 4096 and t_block = 1024, the largest the API takes, on 10
    atoms: 2100 samples pushed from host memory in one call (two full blocks
    and a partial one, copies overlapped), K and the direction split against
    the oracle, every lag past the run exactly zero."""
    announce("shc 10 atoms L=4096 T=1024")
    n_atoms, S, L, T = 10, 2100, 4096, 1024
    v, W = _inputs(n_atoms, S, seed=13)
    h, K, n = _run(n_atoms, v, W, L, T, [S], False)
    Kd, _ = h.read_dir()
    h.close()
    e = rel(K, oracle.shc_correlation(v, W, L))
    ed = rel(Kd, oracle.shc_correlation_directional(v, W, L))
    log("shc_N10_S2100_L4096_T1024", rel_K=e, rel_K_dir=ed)
    assert n == S and K.shape == (L, 3) and e <= TOL and ed <= TOL
    assert not K[S:].any() and not Kd[S:].any()


def test_shc_group_same_bits_as_single_pushes():
    """Grouped SHC (mhc_shc_group_*): five systems of uneven size and lag
    count (16, 133, 1000, 2051 and 8000 atoms; 7, 64, 250, 130 and 250 lags;
    T = 256), the small ones fused into one launch per kernel and the
    8000-atom one on its own launches, pushed together — device inputs in two
    pushes of 300 and 220 steps (partial blocks), then host inputs of 80
    steps — end with every system's K and split K bit-equal to pushing it
    alone, and K within the 1e-12 bar of the oracle (checked on the four
    smaller systems)."""
    import torch
    from paper_2102_03691_amd import ModalSHC, SHCGroup
    announce("shc group of 5 uneven systems")
    sizes, lags, T = (16, 133, 1000, 2051, 8000), (7, 64, 250, 130, 250), 256
    pieces = ((0, 300, True), (300, 520, True), (520, 600, False))
    data = [_inputs(n, 600, seed=500 + n) for n in sizes]
    side = torch.cuda.Stream()                   # one stream for all (a null stream would give each its own)
    stream = side.cuda_stream
    grouped = [ModalSHC(n, L, T, stream=stream) for n, L in zip(sizes, lags)]
    alone = [ModalSHC(n, L, T, stream=stream) for n, L in zip(sizes, lags)]
    g = SHCGroup(grouped)
    for a, b, dev in pieces:
        if dev:
            vs = [torch.as_tensor(v[a:b], device="cuda:0") for v, _ in data]
            Ws = [torch.as_tensor(W[a:b], device="cuda:0") for _, W in data]
        else:
            vs = [v[a:b] for v, _ in data]
            Ws = [W[a:b] for _, W in data]
        g.push(vs, Ws)
        for h, v, W in zip(alone, vs, Ws):
            h.push(v, W)
    torch.cuda.synchronize()
    for k, (n, L) in enumerate(zip(sizes, lags)):
        Kg, Sg = grouped[k].read()
        Ka, Sa = alone[k].read()
        Kdg, _ = grouped[k].read_dir()
        Kda, _ = alone[k].read_dir()
        assert Sg == Sa == 600
        assert np.array_equal(Kg, Ka) and np.array_equal(Kdg, Kda)
        if n <= 2051:
            v, W = data[k]
            e = rel(Kg, oracle.shc_correlation(v, W, L))
            log(f"shc_group_N{n}_L{L}", rel_K=e)
            assert e <= TOL
    g.close()
    for h in grouped + alone:
        h.close()


def test_shc_group_errors():
    import torch
    from paper_2102_03691_amd import MhcError, ModalSHC, SHCGroup
    announce("shc group errors")
    side = torch.cuda.Stream()
    stream = side.cuda_stream
    a = ModalSHC(50, 10, 64, stream=stream)
    b = ModalSHC(50, 10, 128, stream=stream)
    with pytest.raises(MhcError) as ei:          # different t_block
        SHCGroup([a, b])
    assert ei.value.status == 1
    with pytest.raises(MhcError) as ei:          # the same system twice
        SHCGroup([a, a])
    assert ei.value.status == 1
    c = ModalSHC(50, 10, 64, stream=0)           # a null stream: the object owns a stream of its own
    with pytest.raises(MhcError) as ei:
        SHCGroup([a, c])
    assert ei.value.status == 1
    for h in (a, b, c):
        h.close()


def test_shc_group_of_large_systems_only():
    """A group whose systems all fill the GPU by themselves (two of 8000 atoms,
    250 lags, T = 256): nothing is fused, each runs its own launches inside the
    grouped push; the sums equal single pushes bit for bit."""
    import torch
    from paper_2102_03691_amd import ModalSHC, SHCGroup
    announce("shc group of large systems only")
    side = torch.cuda.Stream()
    stream = side.cuda_stream
    data = [_inputs(8000, 300, seed=900 + k) for k in range(2)]
    grouped = [ModalSHC(8000, 250, 256, stream=stream) for _ in data]
    alone = [ModalSHC(8000, 250, 256, stream=stream) for _ in data]
    g = SHCGroup(grouped)
    vs = [torch.as_tensor(v, device="cuda:0") for v, _ in data]
    Ws = [torch.as_tensor(W, device="cuda:0") for _, W in data]
    g.push(vs, Ws)
    g.push([v[:0] for v in vs], [W[:0] for W in Ws])   # nothing to push
    for h, v, W in zip(alone, vs, Ws):
        h.push(v, W)
    torch.cuda.synchronize()
    for hg, ha in zip(grouped, alone):
        (Kg, Sg), (Ka, Sa) = hg.read(), ha.read()
        assert Sg == Sa == 300 and np.array_equal(Kg, Ka)
    g.close()
    for h in grouped + alone:
        h.close()
