"""Shared helpers of the GPU parity tests: drive the library through the C ABI
and compute the oracle's answer on the same seeded inputs."""
import json
import os
import sys

import numpy as np

import oracle
import synth

TOL = {0: 1e-5, 1: 1e-4}          # relative L2 per output array: FP32, split-BF16


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def rel_max(a, b) -> float:
    """max |a - b| / max |b|: the max-abs-normalised companion of rel()."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mb = np.abs(b).max() if b.size else 0.0
    return float(np.abs(a - b).max() / mb) if mb > 0 else float(np.abs(a).max() if a.size else 0.0)


def log(case: str, **vals):
    """Print (and optionally append to $MHC_PARITY_LOG) one measured error record."""
    rec = {"case": case, **vals}
    print("PARITY", json.dumps(rec), flush=True)
    path = os.environ.get("MHC_PARITY_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps(rec) + "\n")


def announce(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


class Case:
    def __init__(self, dims, n_steps, mass_kind="uniform", seed=0, n_modes=None):
        self.lat = synth.BlochLattice(dims)
        self.m = synth.masses(self.lat.n_atoms, mass_kind, seed)
        self.v, self.W = synth.gen_steps(seed, self.m, 0, n_steps)
        self.n_modes = n_modes or self.lat.n_modes
        self.freq = self.lat.frequencies[: self.n_modes]

    def oracle_bins(self, nb):
        return oracle.bin_of_mode(self.freq, nb, 0.0, self.lat.f_max)

    def oracle(self, nb, corr_len=0, dt=1.0, bins=None):
        E = self.lat.eig_matrix()[:, : self.n_modes]
        b = self.oracle_bins(nb) if bins is None else bins
        return oracle.run_dense(E, self.m, self.v, self.W, b, nb, corr_len=corr_len, dt=dt)


def run_library(case: Case, nb, methods, precision, t_block, corr_len=0, dt=1.0, splits=None, bins=None,
                row_chunk=97, keep=False, schedule=0, device_inputs=False):
    from paper_2102_03691_amd import ModalHC, HNEMA, GKMA
    h = ModalHC(0)
    h.load_system(case.m, case.freq)
    if bins is None:
        h.set_bins_uniform(nb, 0.0, case.lat.f_max)
    else:
        h.set_bins(nb, bins)
    h.configure(methods=methods, precision=precision, t_block=t_block, corr_len=corr_len, dt=dt,
                schedule=schedule)
    for r0 in range(0, case.n_modes, row_chunk):
        n = min(row_chunk, case.n_modes - r0)
        h.load_eigvec_rows(r0, case.lat.eig_rows(r0, n))
    h.finalize()
    S = case.v.shape[0]
    splits = splits or [S]
    v, W = case.v, case.W
    if device_inputs:
        import torch
        v = torch.as_tensor(v, device="cuda:0")
        W = torch.as_tensor(W, device="cuda:0")
    s0 = 0
    for n in splits:
        h.push(v[s0:s0 + n], W[s0:s0 + n])
        s0 += n
    assert s0 == S
    out = {}
    if methods & HNEMA:
        out["hnema"], out["hnema_total"], out["n_samples"] = h.read_hnema()
    if methods & GKMA:
        g = h.read_gkma()
        out.update(g)
    if keep:
        out["handle"] = h
    else:
        h.close()
    return out
