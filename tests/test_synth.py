"""The seeded generators: reproducibility, chunk independence, distributions."""
import numpy as np

import synth


def test_steps_do_not_depend_on_chunking():
    m = synth.masses(20, "natural", 1)
    v, W = synth.gen_steps(7, m, 0, 9)
    v2, W2 = synth.gen_steps(7, m, 4, 5)
    assert np.array_equal(v[4:], v2) and np.array_equal(W[4:], W2)
    assert v.dtype == np.float32 and W.dtype == np.float32


def test_velocity_distribution():
    m = synth.masses(500)
    v, W = synth.gen_steps(3, m, 0, 40)
    sig = synth.velocity_sigma(m[:1], 300.0)[0]
    assert abs(v.std() / sig - 1) < 0.02
    assert abs(W.std() - 1) < 0.02
    # nonsymmetric virials
    assert np.abs(W - np.swapaxes(W, -1, -2)).max() > 0.5


def test_rows_match_full_matrix_and_torch():
    lat = synth.BlochLattice((3, 4, 2))
    E = lat.eig_matrix()
    assert np.array_equal(lat.eig_rows(7, 11), E[:, 7:18].T)
    t = lat.eig_rows_torch(7, 11, device="cpu").numpy()
    assert np.abs(t - E[:, 7:18].T).max() < 1e-15


def test_natural_masses_mix():
    m = synth.masses(20000, "natural", 0)
    frac28 = np.mean(np.abs(m - 27.9769265) < 1e-6)
    assert abs(frac28 - 0.922) < 0.01


def test_uneven_batch_is_seeded():
    a = synth.uneven_batch(0)
    assert a == synth.uneven_batch(0) and len(a) == 16
    assert all(e in synth.UNEVEN_EDGES and mm in (1, 2) for e, mm in a)
