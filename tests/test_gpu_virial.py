"""Per-atom virial, forces and HNEMD driving force on the GPU (mhc_virial_*,
Sec. II.A, Eqs. 4, 8, 10, 12) against the FP64 oracle, element by element,
through the C ABI:
  * neighbour lists bit for bit (counts and sorted indices);
  * site energies, forces, W (float64), Fext within 1e-12 of the largest
    reference element per array (float64 on both sides; only the summation
    order and the device's exp / pow / sincos differ), W32 within one float32
    rounding of the oracle's W;
  * the displaced crystal, the expanded crystal whose bonds sit inside the
    cutoff's switching shell, the exponential term switched on (m = 3 and 1),
    a non-cubic box, a liquid-like cell with 2 to 8 bonds per atom, lists
    built with a skin (extra pairs contribute zero),
    the paper's 8000-atom Si at full size; bitwise repeatability; the
    neighbour-overflow error;
  * the float32 W fed to the modal-current push on the device, against the
    oracle's modal path on the oracle's W."""
import numpy as np
import pytest

import oracle
import synth
from oracle import virial as ov
from tests._cases import TOL, announce, log, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_03691_amd import library
    library()


def _params(kind):
    p = ov.tersoff_si()
    if kind == "exp3":
        p.update(lambda3=1.3258, m=3)
    elif kind == "exp1":
        p.update(lambda3=0.7, m=1)
    return p


def _device(pos, box, mass, vel, fe, p, max_nb=16, skin=0.0, runs=1):
    import torch
    from paper_2102_03691_amd import ModalVirial
    v = ModalVirial(mass, box, p, max_neighbors=max_nb, skin=skin)
    pt = torch.as_tensor(pos, device="cuda:0")
    vt = torch.as_tensor(vel, device="cuda:0")
    v.neighbors(pt)
    counts, lists = v.read_neighbors()
    outs = []
    for _ in range(runs):
        o = v.compute(pt, vt, fe)
        torch.cuda.synchronize()
        outs.append({k: t.cpu().numpy() for k, t in o.items()})
    v.close()
    return outs, counts, lists


def _compare(tag, got, ref):
    e = {}
    for k in ("U", "F", "W", "Fext"):
        scale = np.abs(ref[k]).max()
        e[k] = float(np.abs(got[k] - ref[k]).max() / scale)
    w32 = ref["W"].astype(np.float32)
    assert np.all(w32 != 0)
    ulp = np.spacing(np.abs(w32)).astype(np.float64)
    e["W32_ulps"] = float((np.abs(got["W32"].astype(np.float64) - w32.astype(np.float64)) / ulp).max())
    log(f"virial_{tag}", **e)
    for k in ("U", "F", "W", "Fext"):
        assert e[k] <= 1e-12, (k, e[k])
    assert e["W32_ulps"] <= 1.0


CASES = [("displaced_si", (2, 2, 2), 5.432, 0.08, "si"), ("switching_si", (2, 2, 2), 6.3, 0.04, "si"),
         ("displaced_exp3", (3, 2, 4), 5.432, 0.1, "exp3"), ("switching_exp1", (3, 3, 3), 6.3, 0.05, "exp1"),
         ("displaced_si_1000", (5, 5, 5), 5.432, 0.06, "si")]


@pytest.mark.parametrize("tag,cells,a,sigma,pk", CASES)
def test_virial_matches_oracle(tag, cells, a, sigma, pk):
    announce(f"virial {tag}")
    p = _params(pk)
    pos, box = synth.diamond(cells, a=a, sigma=sigma, seed=11)
    m = synth.masses(len(pos), "natural", 2)
    vel = synth.thermal_velocities(m, 300.0, 4)
    fe = np.array([1.5e-4, -0.7e-4, 0.4e-4])
    ref = ov.evaluate(pos, box, vel, m, fe, p)
    (got,), counts, lists = _device(pos, box, m, vel, fe, p)
    want_c = np.array([len(x) for x in ref["nl"]], dtype=np.int32)
    np.testing.assert_array_equal(counts, want_c)
    for i, js in enumerate(ref["nl"]):
        np.testing.assert_array_equal(lists[i, : len(js)], js)
        assert np.all(lists[i, len(js):] == -1)
    _compare(tag, got, ref)
    # the per-atom tensors are not symmetric (many-body), their sum is
    assert np.abs(got["W"] - got["W"].transpose(0, 2, 1)).max() > 1e-2 * np.abs(got["W"]).max()


def test_liquid_like_cell_five_to_eight_bonds():
    """64 atoms at random (at least 2.2 A apart) in a 10.9 A cube: 2 to 8 pairs
    inside R + D per atom, 43 atoms with more than 4, so the site kernel runs
    4 lanes x 2 slots per atom with the second slot round active in some waves
    and not in others (the sums keep the list order: results as with one slot
    per lane)."""
    announce("virial liquid-like cell, 5-8 bonds")
    rng = np.random.default_rng(1)
    box = np.array([10.9, 10.9, 10.9])
    pos = []
    while len(pos) < 64:
        x = rng.uniform(0.0, 10.9, 3)
        if all(np.linalg.norm(ov.min_image(x - q, box)) >= 2.2 for q in pos):
            pos.append(x)
    pos = np.array(pos)
    p = _params("exp3")
    m = synth.masses(len(pos), "natural", 3)
    vel = synth.thermal_velocities(m, 300.0, 7)
    fe = np.array([1e-4, 2e-4, -1e-4])
    ref = ov.evaluate(pos, box, vel, m, fe, p)
    want_c = np.array([len(x) for x in ref["nl"]])
    assert want_c.min() >= 2 and want_c.max() == 8 and (want_c > 4).sum() >= 40
    outs, counts, _ = _device(pos, box, m, vel, fe, p, runs=2)
    np.testing.assert_array_equal(counts, want_c)
    _compare("liquid64", outs[0], ref)
    for k in outs[0]:
        np.testing.assert_array_equal(outs[0][k], outs[1][k])


def test_skin_lists_give_the_same_results():
    """Lists built with a 1 A skin hold most of the 12 second neighbours (at
    3.84 A, displaced) besides the 4 bonds; pairs beyond R + D contribute
    exactly zero."""
    announce("virial with a neighbour skin")
    p = _params("exp3")
    pos, box = synth.diamond((3, 3, 3), sigma=0.07, seed=12)
    m = synth.masses(len(pos))
    vel = synth.thermal_velocities(m, 300.0, 5)
    fe = np.array([2e-4, 0.0, 0.0])
    ref = ov.evaluate(pos, box, vel, m, fe, p)
    (got,), counts, _ = _device(pos, box, m, vel, fe, p, max_nb=24, skin=1.0)
    assert counts.min() >= 4 and counts.mean() > 12
    _compare("skin1", got, ref)


def test_bitwise_repeatable_and_overflow_error():
    import torch
    from paper_2102_03691_amd import MhcError, ModalVirial
    announce("virial repeatability and overflow")
    p = _params("si")
    pos, box = synth.diamond((3, 3, 3), sigma=0.05, seed=13)
    m = synth.masses(len(pos))
    vel = synth.thermal_velocities(m, 300.0, 6)
    outs, _, _ = _device(pos, box, m, vel, np.array([1e-4, 1e-4, 0.0]), p, runs=2)
    for k in outs[0]:
        np.testing.assert_array_equal(outs[0][k], outs[1][k])
    v = ModalVirial(m, box, p, max_neighbors=3)
    pt = torch.as_tensor(pos, device="cuda:0")
    with pytest.raises(MhcError) as ei:
        v.neighbors(pt)
    assert ei.value.status == 1 and "4 neighbours" in str(ei.value)
    with pytest.raises(MhcError) as ei:
        v.compute(pt)
    assert ei.value.status == 2
    v.close()
    with pytest.raises(MhcError) as ei:          # box too small for the cutoff
        ModalVirial(m[:8], np.array([5.432, 5.432, 5.432]), p)
    assert ei.value.status == 1


@pytest.mark.timeout(600)
def test_si8000_full_size():
    """The paper's 8000-atom Si (10 x 10 x 10 conventional cells, Sec. III.C.ii),
    thermal displacements; every atom against the oracle."""
    announce("virial si8000 full size")
    p = _params("si")
    pos, box = synth.diamond((10, 10, 10), sigma=0.06, seed=14)
    m = synth.masses(len(pos), "natural", 3)
    vel = synth.thermal_velocities(m, 300.0, 7)
    fe = np.array([1e-4, 0.0, 0.0])
    (got,), counts, _ = _device(pos, box, m, vel, fe, p)
    ref = ov.evaluate(pos, box, vel, m, fe, p)
    np.testing.assert_array_equal(counts, [len(x) for x in ref["nl"]])
    _compare("si8000", got, ref)


@pytest.mark.parametrize("prec,T", [(1, 64), (0, 1)])
def test_device_virials_feed_the_modal_push(prec, T):
    """64 displaced configurations of 64 Si atoms: the device's float32 W of each
    configuration written into one block buffer and pushed (with the
    configurations' velocities) into an HNEMA + GKMA context with a dense random
    orthonormal basis; against the oracle's modal path on the oracle's W."""
    import torch
    from paper_2102_03691_amd import GKMA, HNEMA, ModalHC, ModalVirial
    announce(f"virial -> modal push prec={prec} T={T}")
    p = _params("exp3")
    S, nb, L = 64, 6, 10
    pos0, box = synth.diamond((2, 2, 2))
    N = len(pos0)
    m = synth.masses(N, "natural", 4)
    E = synth.random_orthonormal(3 * N, 21)
    freq = np.linspace(0.0, 15.0, 3 * N)
    rng = np.random.default_rng(31)
    vir = ModalVirial(m, box, p, max_neighbors=16, skin=0.6)
    vblk = torch.empty((S, N, 3), dtype=torch.float32, device="cuda:0")
    wblk = torch.empty((S, N, 3, 3), dtype=torch.float32, device="cuda:0")
    v_host = np.empty((S, N, 3), dtype=np.float32)
    W_ref = np.empty((S, N, 3, 3))
    configs = []
    for s in range(S):
        pos = np.mod(pos0 + rng.standard_normal(pos0.shape) * 0.05, box)
        vel = synth.thermal_velocities(m, 300.0, 100 + s)
        pt = torch.as_tensor(pos, device="cuda:0")
        if s % 16 == 0:
            vir.neighbors(pt)            # rebuilt every 16 configurations; the skin covers the moves
        vir.compute(pt, want=(), out={"W32": wblk[s]})
        v_host[s] = vel.astype(np.float32)
        vblk[s] = torch.as_tensor(v_host[s], device="cuda:0")
        nl = ov.neighbor_lists(pos, box, p["R"] + p["D"])
        W_ref[s] = ov.per_atom_virial(pos, box, p, nl)
        configs.append((pos, nl))
    torch.cuda.synchronize()
    vir.close()
    W32 = W_ref.astype(np.float32)
    np.testing.assert_allclose(wblk.cpu().numpy(), W32, rtol=0, atol=float(np.spacing(np.abs(W32).max())))
    h = ModalHC(0)
    h.load_system(m, freq)
    h.set_bins_uniform(nb, 0.0, 15.0)
    h.configure(methods=HNEMA | GKMA, precision=prec, t_block=T, corr_len=L, dt=1.0)
    h.load_eigvec_rows(0, np.ascontiguousarray(E.T))
    h.finalize()
    h.push(vblk, wblk)
    avg, tot, n = h.read_hnema()
    g = h.read_gkma()
    h.close()
    bins = oracle.bin_of_mode(freq, nb, 0.0, 15.0)
    ref = oracle.run_dense(E, m, v_host, W32, bins, nb, corr_len=L)
    e = {"hnema": rel(avg, ref["hnema"]), "corr": rel(g["corr"], ref["corr"]), "total": rel(tot, ref["hnema_total"])}
    log(f"virial_to_push_p{prec}_T{T}", **e)
    assert n == S and e["hnema"] <= TOL[prec] and e["corr"] <= TOL[prec]
    # the Eq. 10 total of the push against the oracle's Eq. 9 current (float32 W and v): the two
    # float32 virials may differ by one rounding (2^-24 relative) per element, so the totals agree
    # to 2^-24 sum |W||v| (plus float64 rounding)
    Wv = np.abs(W32.astype(np.float64)) * np.abs(v_host.astype(np.float64))[:, :, None, :]
    bound = 2.0 ** -24 * Wv.sum(axis=(1, 3)).mean(axis=0) + 1e-12 * np.abs(ref["hnema_total"]).max()
    J9 = np.mean([ov.heat_current_eq9(pos_s, box, v_host[s].astype(np.float64), p, nl_s).sum(axis=0)
                  for s, (pos_s, nl_s) in enumerate(configs)], axis=0)
    assert np.all(np.abs(tot - ref["hnema_total"]) <= bound)
    assert np.all(np.abs(tot - J9) <= bound + 2.0 ** -24 * np.abs(J9))
