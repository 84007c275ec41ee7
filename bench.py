"""Throughput of the modal heat-current hot path on one MI355X.

One bench step = one pass of the whole path over one block of T sampled MD
steps: input prep -> projection GEMM with fused modal-current epilogue ->
frequency binning -> float64 HNEMA accumulation (and, for GKMA workloads,
the float64 correlation update).  Inputs are generated in device memory
before the timed region.

Metric: atom*mode*steps/s = N_atoms * N_modes * (MD steps processed) / time.

Prints one JSON line: the metric, its value and unit, steps and warm-up, the
workload's configuration, the roofline of the dominant kernel (achieved
algorithmic FLOP/s or bytes/s against the MI355X peak -- 24 FLOP per
atom*mode*step, the method's own work; the split precisions issue three
products, reported beside it as frac_issued -- and the HBM bytes per launch
from the rocprofv3 summary while its kernel sources are unchanged), the
relative error of one seeded block of the same workload against the FP64
oracle, and the FP64 oracle timed on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "modal heat-current atom*mode*steps/s, split-BF16 vs FP32 at ≤1e-4 rel err"

# MI355X published peaks
PEAK_BF16_FLOPS = 2.5e15
PEAK_FP32_MFMA_FLOPS = 157.3e12
PEAK_HBM_BPS = 8.0e12

WORKLOADS = {
    # name: (dims, t_block, precision, methods, n_bins, corr_len, default bench steps)
    "slab48x48x4_hnema_bf16x3_t128": ((48, 48, 4), 128, 1, 1, 1000, 0, 156),
    "slab48x48x4_hnema_fp32_t128": ((48, 48, 4), 128, 0, 1, 1000, 0, 20),
    "sc16_hnema_fp32_t1": ((16, 16, 16), 1, 0, 1, 500, 0, 40),
    "rod4x4x1500_gkma_bf16x3_t256": ((4, 4, 1500), 256, 1, 3, 1000, 2000, 195),
    "rod4x4x1500_gkma_fp32_t256": ((4, 4, 1500), 256, 0, 3, 1000, 2000, 20),
    # shaped like the paper's speed test (Sec. III.C.ii): 8000 atoms, the modal current
    # every step, 3 bins of 8000 modes (equal mode counts in frequency order)
    "sc20_3bins_fp32_t1": ((20, 20, 20), 1, 0, 1, 3, 0, 8),
    # the motion-direction split (methods HNEMA | DIRECTIONAL) on the slab
    "slab48x48x4_hnema_dir_bf16x3_t128": ((48, 48, 4), 128, 1, 5, 1000, 0, 60),
}
COUNT_BINS = {"sc20_3bins_fp32_t1"}
DEFAULT = "slab48x48x4_hnema_bf16x3_t128"

# Uneven serving-style batch: 16 simple-cubic systems, edges and methods drawn by seed
# from {8,10,12,14,16,20} and {HNEMA, GKMA}; T = 64, 5000 steps each (78 full blocks).
GROUP_WORKLOADS = {
    "uneven16_fp8x3_t64": 3, "uneven16_fp8_t64": 2, "uneven16_bf16x3_t64": 1, "uneven16_fp32_t64": 0,
}
GROUP_NB, GROUP_L, GROUP_T, GROUP_STEPS = 500, 1000, 64, 78
PEAK_FP8_FLOPS = 5.0e15

# Spectral heat current (no eigenvectors): 8000 atoms (the paper's Si and CNT
# sizes), 250 lags (500 fs at a 2 fs sample interval), T = 256 steps per block.
SHC_WORKLOADS = {"shc8000_l250_t256": (8000, 250, 256, 40)}     # atoms, lags, T, default blocks
# grouped SHC: independent runs of uneven size (seeded draw of 16 sizes in 512 .. 8000 atoms), lags, T, blocks
SHC_GROUP_WORKLOADS = {"shc_group16_l250_t256": (16, 512, 8000, 250, 256, 20),
                       "shc_group64_small_l250_t256": (64, 216, 1000, 250, 256, 20)}
SHC_METRIC = "spectral heat current atom*lag*steps/s (float64 virial-velocity correlation)"
PEAK_FP64_FLOPS = 78.6e12

# Per-atom virial, forces and HNEMD force of Tersoff Si from positions (the
# inputs of the modal current, Sec. II.A): diamond crystals of n^3 conventional
# cells with thermal displacements; one bench step = one evaluation of every
# atom (neighbour lists built before the timed region, as an MD code rebuilds
# them every few steps).  8000 atoms is the paper's speed-test size.
VIRIAL_WORKLOADS = {"si8000_virial": ((10, 10, 10), 200), "si512k_virial": ((40, 40, 40), 100)}
# NVE velocity-Verlet steps on the device with the same forces, each step writing its
# float32 v and W (the push inputs); lists with a 1 A skin rebuilt every 50 steps
MD_WORKLOADS = {"si8000_md": ((10, 10, 10), 400), "si512k_md": ((40, 40, 40), 200)}
# the paper's SHC run on its 8000-atom Si block (Sec. III.A): NVT at 300 K with the HNEMD driving force
# |F_e| = 0.1 / um along x, the SHC correlation over 250 lags computed on the fly; blocks of T steps
# Tersoff workloads: HIP events around every TIMED_EVERY-th evaluation inside
# the timed region (at 8000 atoms recording them at each one costs about as
# much as the kernels they time)
TIMED_EVERY = 16
# SHC: events around every 4th block (two events cost about 3% of a 0.26 ms block)
TIMED_EVERY_SHC = 4
# cells, lags, T, default blocks, independent runs (each on a stream of its own, driven by a host thread of its own)
HNEMD_WORKLOADS = {"si8000_hnemd_shc": ((10, 10, 10), 250, 256, 4, 1),
                   "si8000x8_hnemd_shc": ((10, 10, 10), 250, 256, 4, 8)}
MD_METRIC = "NVE molecular dynamics (velocity Verlet, Tersoff Si, float64) atom*steps/s incl. push inputs"
VIRIAL_METRIC = "per-atom virial (Eq. 8) + forces + HNEMD force (Eq. 12) atom*steps/s, float64 Tersoff Si"


# Algorithmic work of the modal current per atom*mode*step: 3 FMAs of the
# projection (Eq. 13) and 9 of the virial bracket (Eq. 16).  The split
# precisions (split-BF16, e4m3 hi/lo) issue three products of that size.
FLOP_PER_UNIT = 24.0
ISSUED_PER_UNIT = {0: 24.0, 1: 72.0, 2: 24.0, 3: 72.0}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# HBM traffic of the dominant kernel comes from the committed rocprofv3 counter
# summaries (profiles/*.md: FETCH_SIZE and WRITE_SIZE passes, scaled by the
# plain-copy calibration).  It is reported only while the kernel sources hash
# to the value recorded with the counters; otherwise it is null.
def _sources_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(workload, kernel):
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        rec = {}
        with open(path) as fh:
            for line in fh:
                if line.startswith("- ") and ": " in line:
                    k, v = line[2:].strip().split(": ", 1)
                    rec[k] = v
        if rec.get("workload") != workload or rec.get("kernel") != kernel:
            continue
        try:
            if _sources_sha256(rec["kernel-sources"].split()) == rec["source-sha256"]:
                return float(rec["hbm-bytes-per-launch"])
        except (KeyError, OSError, ValueError):
            pass
    return None


def count_bins(freq, nb):
    """Bins of equal mode counts in frequency order (stable for equal frequencies)."""
    import numpy as np
    order = np.argsort(np.asarray(freq), kind="stable")
    bins = np.empty(len(order), dtype=np.int32)
    bins[order] = (np.arange(len(order)) * nb) // len(order)
    return bins


def make_context(lat, t_block, precision, methods, nb, corr_len, device=0, schedule=0, bins=None):
    import torch
    import synth
    from paper_2102_03691_amd import ModalHC
    h = ModalHC(device)
    m = synth.masses(lat.n_atoms)
    h.load_system(m, lat.frequencies)
    if bins is None:
        h.set_bins_uniform(nb, 0.0, lat.f_max)
    else:
        h.set_bins(nb, bins)
    h.configure(methods=methods, precision=precision, t_block=t_block, corr_len=corr_len, dt=1.0,
                schedule=schedule)
    M = lat.n_modes
    chunk = max(1, min(M, (512 << 20) // (8 * 3 * lat.n_atoms)))
    for r0 in range(0, M, chunk):
        n = min(chunk, M - r0)
        rows = lat.eig_rows_torch(r0, n, device=f"cuda:{device}")
        h.load_eigvec_rows(r0, rows)
        del rows
    torch.cuda.synchronize()
    h.finalize()
    return h, m


def time_pushes(h, blocks_v, blocks_W, n_warm, n_steps):
    import torch
    for i in range(n_warm):
        h.push(blocks_v[i % len(blocks_v)], blocks_W[i % len(blocks_W)])
    h.synchronize()
    h.kernel_timing()                       # drop warm-up launches
    h.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_steps):
        j = (n_warm + i) % len(blocks_v)
        h.push(blocks_v[j], blocks_W[j])
    h.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, kms = h.kernel_timing()
    h.set_timing(False)
    return t1 - t0, launches, kms


def cpu_baseline(dims, t_block, nb, budget_s=15.0, bins=None):
    """The FP64 oracle on a bounded sample of the same workload.

    Same lattice and block length; the oracle's Eq. 13/16 projection and the
    binning are applied to consecutive chunks of modes (rows of E^T), block
    after block of T steps, until about ``budget_s`` seconds of CPU work have
    been timed.  The oracle's cost is linear in the number of modes and of
    steps, so the rate carries over to the whole run.  Generating the
    eigenvector rows and the inputs is input preparation, not timed.
    """
    import oracle
    import synth
    lat = synth.BlochLattice(dims)
    m = synth.masses(lat.n_atoms)
    T = max(t_block, 128)
    if bins is None:
        bins = oracle.bin_of_mode(lat.frequencies, nb, 0.0, lat.f_max)
    rows_per = min(lat.n_modes, 2048)
    done_units, spent, n_rows, n_blocks = 0, 0.0, 0, 0
    while spent < budget_s and n_blocks < 64:
        v, W = synth.gen_steps(n_blocks, m, n_blocks * T, T)
        r0 = 0
        while r0 < lat.n_modes and spent < budget_s:
            n = min(rows_per, lat.n_modes - r0)
            Ec = lat.eig_rows(r0, n).T                     # [3N, n] columns of E
            t0 = time.perf_counter()
            Jn = oracle.modal_currents(Ec, m, v, W)
            oracle.binned_current(Jn, bins[r0:r0 + n], nb)
            spent += time.perf_counter() - t0
            done_units += lat.n_atoms * n * T
            n_rows += n
            r0 += n
        n_blocks += 1
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count()
    return {"value": done_units / spent, "unit": "atom*mode*steps/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{n_rows} mode rows x {T} steps over {n_blocks} block(s) of the same lattice "
                      f"({lat.n_modes} modes; float64 numpy/BLAS), {spent:.1f} s of CPU work"}


def cpu_baseline_one_core(dims, t_block, nb, budget_s=6.0, bins=None):
    """The same oracle sample with the BLAS pool limited to one thread (the
    paper's comparisons are against single CPU cores, Sec. III.C.ii)."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:
        return None
    with threadpool_limits(limits=1):
        r = cpu_baseline(dims, t_block, nb, budget_s=budget_s, bins=bins)
    r["cores"] = 1
    return r


def _rel(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def lattice_reference(lat, m, v, W, nb, methods, L):
    """The FP64 oracle's binned currents (FFT form, exact for the plane-wave
    basis) of seeded inputs, and its HNEMA average / GKMA correlation."""
    import oracle
    kb = oracle.bin_of_mode(lat.kpoint_frequencies().ravel(), nb, 0.0, lat.f_max).reshape(lat.dims)
    Jb = oracle.binned_current_fft(lat.dims, m, v, W, kb, nb)
    ref = {}
    if methods & 1:
        ref["hnema"] = oracle.hnema_average(Jb)
    if (methods & 1) and (methods & 4):
        # direction split: a plane-wave mode of polarisation nu moves atoms along
        # nu only, so J_b^{mu nu} is the FFT-form current of v^nu and W^{. nu} alone
        import numpy as np
        hd = np.zeros((nb, 3, 3))
        for nu in range(3):
            vm = np.zeros_like(v)
            vm[..., nu] = v[..., nu]
            Wm = np.zeros_like(W)
            Wm[..., :, nu] = W[..., :, nu]
            hd[:, :, nu] = oracle.hnema_average(oracle.binned_current_fft(lat.dims, m, vm, Wm, kb, nb))
        ref["hnema_dir"] = hd
    if methods & 2:
        ref["corr"] = oracle.gkma_correlation(Jb, oracle.total_heat_current(v, W), L)
    return ref


def library_errors(h, ref):
    out = {}
    if "hnema" in ref:
        out["hnema"] = _rel(h.read_hnema()[0], ref["hnema"])
    if "hnema_dir" in ref:
        out["hnema_dir"] = _rel(h.read_hnema_dir()[0], ref["hnema_dir"])
    if "corr" in ref:
        out["corr"] = _rel(h.read_gkma()["corr"], ref["corr"])
    return out


def accuracy_vs_oracle(h, lat, m, methods, nb, L, steps):
    """Relative L2 error of the timed context on one seeded block: the context
    is reset, fed ``steps`` seeded MD steps (device inputs) and read; the
    reference is the FP64 oracle on the same float32 inputs."""
    import torch
    import synth
    h.reset()
    v, W = synth.gen_steps(7, m, 0, steps)
    h.push(torch.as_tensor(v, device="cuda:0"), torch.as_tensor(W, device="cuda:0"))
    h.synchronize()
    out = library_errors(h, lattice_reference(lat, m, v, W, nb, methods, L))
    out.update(oracle="binned_current_fft (FFT form of the FP64 oracle, exact for the plane-wave basis)",
               sample=f"{steps} seeded MD steps (float32 inputs) through the timed context after a reset",
               norm="relative L2 per output array")
    return out


def run_shc(args):
    """SHC virial-velocity correlation (Eq. 21) in float64, inputs resident in HBM."""
    import torch
    import oracle
    import synth
    from paper_2102_03691_amd import ModalSHC
    N, L, T, blocks = SHC_WORKLOADS[args.workload]
    K = args.steps or blocks
    m = synth.masses(N)
    n_blocks = max(1, min(K + args.warmup, 16))
    v, W = synth.gen_steps_torch(3, m, n_blocks * T, device="cuda:0")
    h = ModalSHC(N, L, T)
    for j in range(args.warmup):
        b = j % n_blocks
        h.push(v[b * T:(b + 1) * T], W[b * T:(b + 1) * T])
    h.synchronize()
    h.set_timing(TIMED_EVERY_SHC)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(K):
        b = (args.warmup + j) % n_blocks
        h.push(v[b * T:(b + 1) * T], W[b * T:(b + 1) * T])
    h.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, kms = h.kernel_timing()
    acc = None
    if not args.no_cpu_baseline:
        log("accuracy: one seeded block against the FP64 oracle")
        h.reset()
        vc, Wc = synth.gen_steps(7, m, 0, T)
        h.push(torch.as_tensor(vc, device="cuda:0"), torch.as_tensor(Wc, device="cuda:0"))
        acc = {"K": _rel(h.read()[0], oracle.shc_correlation(vc, Wc, L)),
               "oracle": "shc_correlation (FP64)", "sample": f"{T} seeded samples after a reset",
               "norm": "relative L2 per output array"}
    h.close()
    units_per_block = float(N) * L * T
    avg_ms = kms / max(launches, 1)
    flops = 18.0 * units_per_block                    # 9 FMAs per atom, lag and step
    # float64 matrix-core products (v_mfma_f64_16x16x4f64): bound by the dense FP64 MFMA rate; the
    # algorithmic count leaves out the off-diagonal products of the Gram tiles
    roof = {"bound": "mfma", "achieved": flops / (avg_ms * 1e-3) / 1e12, "peak": PEAK_FP64_FLOPS / 1e12,
            "unit": "TFLOP/s", "traffic": profiled_traffic(args.workload, "k_shc_gram"), "kernel": "k_shc_gram",
            "avg_launch_ms": avg_ms,
            "launches": launches, "timed_every": TIMED_EVERY_SHC}
    roof["frac"] = roof["achieved"] / roof["peak"]
    out = {"metric": SHC_METRIC, "value": units_per_block * K / wall, "unit": "atom*lag*steps/s", "n_gpus": 1,
           "steps": K, "warmup": args.warmup, "ms_per_step": wall / K * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": args.workload, "atoms": N, "lags": L, "md_steps_per_step": T, "t_block": T,
                      "precision": "float32 inputs, products and sums in float64", "parallelism": "single GPU"},
           "roofline": roof}
    if acc is not None:
        out["rel_err_vs_oracle"] = acc
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        vc, Wc = synth.gen_steps(0, m, 0, T)
        t0 = time.perf_counter()
        oracle.shc_correlation(vc, Wc, L)
        spent = time.perf_counter() - t0
        # the oracle sums each lag over the S - tau origins of the sample
        work = float(N) * sum(T - tau for tau in range(L))
        try:
            from threadpoolctl import threadpool_info
            cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        except Exception:
            cores = os.cpu_count()
        out["cpu_baseline"] = {"value": work / spent, "unit": "atom*lag*steps/s", "cores": int(cores),
                               "kind": "oracle",
                               "sample": f"{T} samples x {L} lags x {N} atoms (float64 numpy tensordot), "
                                         f"{spent:.1f} s of CPU work"}
    return out


def run_shc_group(args):
    """Grouped SHC (mhc_shc_group_*): 16 independent systems of uneven size, one
    launch per kernel and block for all of them, inputs resident in HBM; the
    same systems pushed one after another are timed beside it."""
    import numpy as np
    import torch
    import oracle
    import synth
    from paper_2102_03691_amd import ModalSHC, SHCGroup
    n_sys, n_lo, n_hi, L, T, blocks = SHC_GROUP_WORKLOADS[args.workload]
    K = args.steps or blocks
    sizes = [int(x) for x in np.random.default_rng(2102).integers(n_lo, n_hi + 1, n_sys)]
    n_blocks = max(1, min(K + args.warmup, 8))
    side = torch.cuda.Stream()
    stream = side.cuda_stream
    data = []
    for q, n in enumerate(sizes):
        data.append(synth.gen_steps_torch(40 + q, synth.masses(n), n_blocks * T, device="cuda:0"))
    torch.cuda.synchronize()

    def timed(push_block):
        for j in range(args.warmup):
            push_block(j % n_blocks)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(K):
            push_block((args.warmup + j) % n_blocks)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    hs = [ModalSHC(n, L, T, stream=stream) for n in sizes]
    g = SHCGroup(hs)
    wall = timed(lambda b: g.push([v[b * T:(b + 1) * T] for v, _ in data], [W[b * T:(b + 1) * T] for _, W in data]))
    solo = [ModalSHC(n, L, T, stream=stream) for n in sizes]

    def one_by_one(b):
        for h, (v, W) in zip(solo, data):
            h.push(v[b * T:(b + 1) * T], W[b * T:(b + 1) * T])
    wall_seq = timed(one_by_one)
    acc = None
    if not args.no_cpu_baseline:
        log("accuracy: one seeded block of the smallest system against the FP64 oracle")
        q = int(np.argmin(sizes))
        for h in hs:
            h.reset()
        vc, Wc = synth.gen_steps(7, synth.masses(sizes[q]), 0, T)
        ins_v = [v[:T] for v, _ in data]
        ins_W = [W[:T] for _, W in data]
        ins_v[q] = torch.as_tensor(vc, device="cuda:0")
        ins_W[q] = torch.as_tensor(Wc, device="cuda:0")
        g.push(ins_v, ins_W)
        acc = {"K": _rel(hs[q].read()[0], oracle.shc_correlation(vc, Wc, L)),
               "oracle": "shc_correlation (FP64)", "sample": f"{T} seeded samples of the {sizes[q]}-atom system",
               "norm": "relative L2 per output array"}
    g.close()
    for h in hs + solo:
        h.close()
    units_per_block = float(sum(sizes)) * L * T
    flops = 18.0 * units_per_block
    ms = wall / K * 1e3
    roof = {"bound": "mfma", "achieved": flops / (ms * 1e-3) / 1e12, "peak": PEAK_FP64_FLOPS / 1e12,
            "unit": "TFLOP/s", "traffic": profiled_traffic(args.workload, "k_shc_gram_group"),
            "kernel": "k_shc_gram_group",
            "achieved_from": "wall time per block (ring, products and sums of all systems)"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    out = {"metric": SHC_METRIC, "value": units_per_block * K / wall, "unit": "atom*lag*steps/s", "n_gpus": 1,
           "steps": K, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": args.workload, "systems": sizes, "lags": L, "md_steps_per_step": T,
                      "t_block": T, "precision": "float32 inputs, products and sums in float64",
                      "parallelism": "single GPU"},
           "roofline": roof,
           "one_by_one": {"ms_per_step": wall_seq / K * 1e3, "value": units_per_block * K / wall_seq,
                          "note": "the same systems pushed one after another (mhc_shc_push each)"}}
    if acc is not None:
        out["rel_err_vs_oracle"] = acc
    return out


def run_hnemd_shc(args):
    """The SHC method end to end on the device: NVT molecular dynamics with the
    HNEMD driving force (Nose-Hoover, Eq. 12 on every atom) writing every
    step's float32 v and W, pushed block by block into the SHC correlation.
    With several independent runs (the paper averages many, Sec. III.A), each
    has its own contexts on a stream of its own, advanced by a host thread of
    its own (the library calls release the interpreter lock), so that the
    runs' launches overlap on the GPU; the value counts every run's steps."""
    import threading
    import numpy as np
    import torch
    import synth
    from paper_2102_03691_amd import ModalSHC, ModalVirial, tersoff_si
    cells, L, T, blocks, R = HNEMD_WORKLOADS[args.workload]
    K = args.steps or blocks
    fe = (1e-5, 0.0, 0.0)                   # 0.1 / um along x
    TEMP, TAU, REBUILD = 300.0, 100.0, 50
    runs = []
    for r in range(R):
        # one run: torch's current stream; several: a new stream each (default priority)
        s = torch.cuda.current_stream() if R == 1 else torch.cuda.Stream()
        handle = None if R == 1 else s.cuda_stream
        with torch.cuda.stream(s):
            pos, box = synth.diamond(cells, sigma=0.06, seed=1 + r)
            N = len(pos)
            m = synth.masses(N, "natural", 1)
            vel = synth.thermal_velocities(m, 300.0, 1 + r)
            run = {"stream": s, "vir": ModalVirial(m, box, tersoff_si(), max_neighbors=24, skin=1.0, stream=handle),
                   "shc": ModalSHC(N, L, T, stream=handle),
                   "pt": torch.as_tensor(np.mod(pos, box), device="cuda:0"),
                   "vt": torch.as_tensor(vel, device="cuda:0").clone(),
                   "v32": torch.empty((T, N, 3), dtype=torch.float32, device="cuda:0"),
                   "W32": torch.empty((T, N, 3, 3), dtype=torch.float32, device="cuda:0"), "th": (0.0, 0.0)}
            run["vir"].neighbors(run["pt"])
        runs.append(run)

    def advance(run, n, errors):
        try:
            with torch.cuda.stream(run["stream"]):
                for _ in range(n):
                    run["th"] = run["vir"].md_nvt(run["pt"], run["vt"], 1.0, T, fe, TEMP, TAU, thermostat=run["th"],
                                                  rebuild=REBUILD, v32=run["v32"], W32=run["W32"])
                    run["shc"].push(run["v32"], run["W32"])
                run["shc"].synchronize()
        except Exception as e:    # re-raised by the caller
            errors.append(e)

    def advance_all(n):
        errors = []
        if R == 1:
            advance(runs[0], n, errors)
        else:
            threads = [threading.Thread(target=advance, args=(run, n, errors)) for run in runs]
            for t in threads:
                t.start()
            for t in threads:
                t.join()
        if errors:
            raise errors[0]

    advance_all(args.warmup)
    for run in runs:
        run["shc"].reset()
    vir, shc, vt = runs[0]["vir"], runs[0]["shc"], runs[0]["vt"]   # timing and end state: the first run
    vir.set_timing(TIMED_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    advance_all(K)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    th = runs[0]["th"]
    launches, site_ms, gather_ms = vir.kernel_timing()
    vir.set_timing(False)
    Kc, n_samples = shc.read()
    kin = 0.5 * float((torch.as_tensor(m, device="cuda:0") * (vt * vt).sum(dim=1)).sum()) * 103.64269652680505
    site_avg = site_ms / max(launches, 1)
    n_b = np.full(N, 4.0)
    flops = float((65.0 * n_b + 79.0 * n_b * (n_b - 1.0) + n_b).sum())
    roof = {"bound": "alu", "achieved": flops / (site_avg * 1e-3) / 1e12, "peak": PEAK_FP64_FLOPS / 1e12,
            "unit": "TFLOP/s", "work": "65 float64 ops per bond + 79 per ordered pair of bonds (4 bonds per Si atom)",
            "flop_per_launch": flops, "traffic": None, "kernel": "k_tersoff_site", "avg_launch_ms": site_avg,
            "launches": launches, "timed_every": TIMED_EVERY, "gather_kernel_avg_ms": gather_ms / max(launches, 1)}
    roof["frac"] = roof["achieved"] / roof["peak"]
    res = {"metric": "HNEMD (NVT + driving force) MD with the SHC correlation on the fly, atom*steps/s",
           "value": R * N * T * K / wall, "unit": "atom*steps/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
           "ms_per_step": wall / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": args.workload, "atoms": N, "cells": list(cells), "potential": "Tersoff Si",
                      "dt_fs": 1.0, "md_steps_per_step": T, "lags": L, "fe_per_A": list(fe), "temperature_K": TEMP,
                      "thermostat_tau_fs": TAU, "skin_A": 1.0, "rebuild_every": REBUILD, "independent_runs": R,
                      "parallelism": "single GPU" if R == 1 else f"single GPU, {R} runs on {R} streams"},
           "roofline": roof,
           "end_state": {"temperature_K": 2.0 * kin / (3 * N * 8.617333262e-5), "xi_per_fs": th[0],
                         "K0_x_eV_A_per_fs": float(Kc[0, 0]), "samples": n_samples}}
    if not args.no_cpu_baseline:
        import oracle
        import oracle.virial as ov
        log("accuracy: NVT + drive and the SHC of its steps against the oracle on a 64-atom cut")
        spos, sbox = synth.diamond((2, 2, 2), sigma=0.06, seed=1)
        sm = synth.masses(len(spos), "natural", 1)
        svel = synth.thermal_velocities(sm, 300.0, 1)
        sfe = (2e-3, 0.0, 0.0)
        ref = ov.md_nvt_hnemd(spos, svel, sm, sbox, ov.tersoff_si(), 1.0, 64, sfe, TEMP, 20.0)
        sv = ModalVirial(sm, sbox, tersoff_si(), max_neighbors=24, skin=1.0)
        ss = ModalSHC(len(spos), 16, 64)
        sp = torch.as_tensor(np.mod(spos, sbox), device="cuda:0")
        svt = torch.as_tensor(svel, device="cuda:0").clone()
        sv32 = torch.empty((64, len(spos), 3), dtype=torch.float32, device="cuda:0")
        sW32 = torch.empty((64, len(spos), 3, 3), dtype=torch.float32, device="cuda:0")
        sv.neighbors(sp)
        sv.md_nvt(sp, svt, 1.0, 64, sfe, TEMP, 20.0, v32=sv32, W32=sW32)
        ss.push(sv32, sW32)
        Kd, _ = ss.read()
        Kr = oracle.shc_correlation(ref["vel"].astype(np.float32), ref["W"].astype(np.float32), 16)
        res["rel_err_vs_oracle"] = {
            "pos_A": float(np.abs(ov.min_image(sp.cpu().numpy() - ref["pos"][-1], sbox)).max()),
            "vel": float(np.abs(svt.cpu().numpy() - ref["vel"][-1]).max() / np.abs(ref["vel"][-1]).max()),
            "shc_K": _rel(Kd, Kr),
            "oracle": "oracle.virial.md_nvt_hnemd, then oracle.shc_correlation of its float32 v and W",
            "sample": "64 atoms (2x2x2 cells), 64 steps, 16 lags",
            "norm": "max |diff| (A) / max |diff| / max |ref| / relative L2"}
        sv.close()
        ss.close()
        log("cpu baseline (oracle)")
        t0 = time.perf_counter()
        done = 0
        while time.perf_counter() - t0 < 12.0:
            ov.md_nvt_hnemd(spos, svel, sm, sbox, ov.tersoff_si(), 1.0, 10, sfe, TEMP, 20.0)
            done += 10
        spent = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": len(spos) * done / spent, "unit": "atom*steps/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{done} NVT + drive steps of the 64-atom cut (pure Python float64, lists "
                                         f"rebuilt every step; the SHC correlation not included), {spent:.1f} s"}
    for run in runs:
        run["vir"].close()
        run["shc"].close()
    return res


def run_virial(args):
    """Tersoff Si: per-atom virial, forces, site energies, float32 W and HNEMD
    force for every atom per step, inputs resident in HBM."""
    import numpy as np
    import torch
    import synth
    from paper_2102_03691_amd import ModalVirial
    cells, default_steps = VIRIAL_WORKLOADS[args.workload]
    K = args.steps or default_steps
    pos, box = synth.diamond(cells, sigma=0.06, seed=1)
    N = len(pos)
    m = synth.masses(N, "natural", 1)
    vel = synth.thermal_velocities(m, 300.0, 1)
    fe = np.array([1e-4, 0.0, 0.0])
    params = dict(A=1830.8, B=471.18, lambda1=2.4799, lambda2=1.7322, lambda3=0.0, m=3, beta=1.1e-6, n=0.78734,
                  c=1.0039e5, d=16.217, h=-0.59825, gamma=1.0, R=2.85, D=0.15)     # Tersoff Si
    vir = ModalVirial(m, box, params, max_neighbors=8, skin=0.0)
    pt = torch.as_tensor(pos, device="cuda:0")
    vt = torch.as_tensor(vel, device="cuda:0")
    out = {k: torch.empty(sh, dtype=torch.float32 if k == "W32" else torch.float64, device="cuda:0")
           for k, sh in (("U", (N,)), ("F", (N, 3)), ("W", (N, 3, 3)), ("W32", (N, 3, 3)), ("Fext", (N, 3)))}
    max_found = vir.neighbors(pt)     # the first call also loads the kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        vir.neighbors(pt)
    nb_ms = (time.perf_counter() - t0) * 1e3 / 5
    for _ in range(args.warmup):
        vir.compute(pt, vt, fe, out=out)
    vir.synchronize()
    vir.set_timing(TIMED_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        vir.compute(pt, vt, fe, out=out)
    vir.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, site_ms, gather_ms = vir.kernel_timing()
    vir.set_timing(False)
    counts, _ = vir.read_neighbors()
    site_avg, gather_avg = site_ms / max(launches, 1), gather_ms / max(launches, 1)
    # Dominant kernel: the site kernel, bound by float64 vector arithmetic.  Its
    # algorithmic operations, from the formulas (exp, pow, sqrt and a division
    # count one each): 65 per neighbour pair (pair vector and minimum image,
    # |r| and 1/|r|, f_C, f_R, f_A, b_ij and db/dzeta, the pair energy, the
    # radial part and the assembly of dU_i/dr_ij) and 79 per ordered pair of
    # neighbours (the zeta term: cos theta, g, product; the derivative: cos theta,
    # its gradient, g and g', the dzeta_ij and dzeta_ik terms), plus the U_i sum.
    n_i = counts.astype(np.float64)
    flops = float((65.0 * n_i + 79.0 * n_i * (n_i - 1.0) + n_i).sum())
    roof = {"bound": "alu", "achieved": flops / (site_avg * 1e-3) / 1e12, "peak": PEAK_FP64_FLOPS / 1e12,
            "unit": "TFLOP/s", "work": "65 float64 ops per neighbour pair + 79 per ordered pair of neighbours",
            "flop_per_launch": flops, "traffic": profiled_traffic(args.workload, "k_tersoff_site"),
            "kernel": "k_tersoff_site", "avg_launch_ms": site_avg, "launches": launches, "timed_every": TIMED_EVERY,
            "gather_kernel_avg_ms": gather_avg}
    roof["frac"] = roof["achieved"] / roof["peak"]
    # the gather kernel is bound by HBM: the pair partials written by the site
    # kernel (read twice, 24 B per pair each), the lists (8 B per pair + 4 B),
    # positions, velocities, masses and U (64 B) and the outputs (156 B)
    gb = float((48.0 * n_i + 8.0 * n_i + 4.0 + 64.0 + 156.0).sum())
    roof["gather_hbm_GBps"] = gb / (gather_avg * 1e-3) / 1e9
    res = {"metric": VIRIAL_METRIC, "value": N * K / wall, "unit": "atom*steps/s", "n_gpus": 1, "steps": K,
           "warmup": args.warmup, "ms_per_step": wall / K * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": args.workload, "atoms": N, "cells": list(cells), "potential": "Tersoff Si",
                      "neighbors_per_atom": 4, "max_found": max_found, "neighbor_build_ms": nb_ms,
                      "outputs": "U, F, W (f64 and f32), F_ext", "parallelism": "single GPU"},
           "roofline": roof}
    if not args.no_cpu_baseline:
        import oracle.virial as ov
        log("accuracy: sampled atoms against the FP64 oracle")
        got = {k: t.cpu().numpy() for k, t in out.items()}
        rng = np.random.default_rng(3)
        idx = np.sort(rng.choice(N, size=48, replace=False))
        ref = ov.evaluate_atoms(pos, box, vel, m, fe, ov.tersoff_si(), idx)
        res["rel_err_vs_oracle"] = {
            **{k: float(np.abs(got[k][idx] - ref[k]).max() / np.abs(ref[k]).max()) for k in ("U", "F", "W", "Fext")},
            "oracle": "oracle.virial.evaluate_atoms (FP64, each sampled atom on its own)",
            "sample": "48 random atoms of the timed configuration", "norm": "max |diff| / max |ref| per array"}
        log("cpu baseline (oracle)")
        t0 = time.perf_counter()
        done = 0
        while time.perf_counter() - t0 < 12.0:
            ov.evaluate_atoms(pos, box, vel, m, fe, ov.tersoff_si(), rng.choice(N, size=16, replace=False))
            done += 16
        spent = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": done / spent, "unit": "atom*steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"{done} random atoms evaluated one by one (pure Python float64, brute-force "
                                         f"neighbour search included), {spent:.1f} s"}
    vir.close()
    return res


def run_md(args):
    """NVE molecular dynamics on the device: K velocity-Verlet steps of 1 fs
    (the paper's time step), every step's float32 v and W written as push
    inputs; inputs resident in HBM."""
    import numpy as np
    import torch
    import synth
    from paper_2102_03691_amd import ModalVirial
    cells, default_steps = MD_WORKLOADS[args.workload]
    K = args.steps or default_steps
    pos, box = synth.diamond(cells, sigma=0.06, seed=1)
    N = len(pos)
    m = synth.masses(N, "natural", 1)
    vel = synth.thermal_velocities(m, 300.0, 1)
    params = dict(A=1830.8, B=471.18, lambda1=2.4799, lambda2=1.7322, lambda3=0.0, m=3, beta=1.1e-6, n=0.78734,
                  c=1.0039e5, d=16.217, h=-0.59825, gamma=1.0, R=2.85, D=0.15)     # Tersoff Si
    REBUILD = 50
    vir = ModalVirial(m, box, params, max_neighbors=24, skin=1.0)
    pt = torch.as_tensor(np.mod(pos, box), device="cuda:0")
    vt = torch.as_tensor(vel, device="cuda:0").clone()
    v32 = torch.empty((K, N, 3), dtype=torch.float32, device="cuda:0")
    W32 = torch.empty((K, N, 3, 3), dtype=torch.float32, device="cuda:0")
    vir.neighbors(pt)

    def energy():
        vir.neighbors(pt)
        U = vir.compute(pt, want=("U",))["U"]
        return float(U.sum()) + 0.5 * float((torch.as_tensor(m, device="cuda:0") * (vt * vt).sum(dim=1)).sum()) * 103.64269652680505

    E0 = energy()
    if args.warmup:
        vir.md(pt, vt, 1.0, args.warmup, rebuild=REBUILD)
    vir.synchronize()
    vir.set_timing(TIMED_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vir.md(pt, vt, 1.0, K, rebuild=REBUILD, v32=v32, W32=W32)
    vir.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, site_ms, gather_ms = vir.kernel_timing()
    vir.set_timing(False)
    E1 = energy()
    counts, _ = vir.read_neighbors()
    n_i = counts.astype(np.float64)
    site_avg = site_ms / max(launches, 1)
    # the site kernel's algorithmic operations (as for the per-atom virial workloads),
    # counted for the pairs within R + D only (the skin's extra pairs are skipped work)
    n_b = np.full(N, 4.0)
    flops = float((65.0 * n_b + 79.0 * n_b * (n_b - 1.0) + n_b).sum())
    roof = {"bound": "alu", "achieved": flops / (site_avg * 1e-3) / 1e12, "peak": PEAK_FP64_FLOPS / 1e12,
            "unit": "TFLOP/s", "work": "65 float64 ops per bond + 79 per ordered pair of bonds (4 bonds per Si atom)",
            "flop_per_launch": flops, "traffic": profiled_traffic(args.workload, "k_tersoff_site"),
            "kernel": "k_tersoff_site", "avg_launch_ms": site_avg, "launches": launches, "timed_every": TIMED_EVERY,
            "gather_kernel_avg_ms": gather_ms / max(launches, 1), "listed_neighbors_mean": float(n_i.mean())}
    roof["frac"] = roof["achieved"] / roof["peak"]
    res = {"metric": MD_METRIC, "value": N * K / wall, "unit": "atom*steps/s", "n_gpus": 1, "steps": K,
           "warmup": args.warmup, "ms_per_step": wall / K * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": args.workload, "atoms": N, "cells": list(cells), "potential": "Tersoff Si",
                      "dt_fs": 1.0, "skin_A": 1.0, "rebuild_every": REBUILD,
                      "outputs": "positions, velocities (f64); per step v and W in f32 (push inputs)",
                      "parallelism": "single GPU"},
           "roofline": roof,
           "energy_drift_eV_per_atom": abs(E1 - E0) / N}
    if not args.no_cpu_baseline:
        import oracle.virial as ov
        log("accuracy: the first steps against the FP64 oracle integrator on a 64-atom cut of the workload")
        spos, sbox = synth.diamond((2, 2, 2), sigma=0.06, seed=1)
        sm = synth.masses(len(spos), "natural", 1)
        svel = synth.thermal_velocities(sm, 300.0, 1)
        ref = ov.md_nve(spos, svel, sm, sbox, ov.tersoff_si(), 1.0, 10)
        sv = ModalVirial(sm, sbox, params, max_neighbors=24, skin=1.0)
        sp = torch.as_tensor(np.mod(spos, sbox), device="cuda:0")
        svt = torch.as_tensor(svel, device="cuda:0").clone()
        sv.neighbors(sp)
        sv.md(sp, svt, 1.0, 10)
        torch.cuda.synchronize()
        res["rel_err_vs_oracle"] = {
            "pos_A": float(np.abs(ov.min_image(sp.cpu().numpy() - ref["pos"][-1], sbox)).max()),
            "vel": float(np.abs(svt.cpu().numpy() - ref["vel"][-1]).max() / np.abs(ref["vel"][-1]).max()),
            "oracle": "oracle.virial.md_nve (FP64 velocity Verlet)", "sample": "64 atoms (2x2x2 cells), 10 steps",
            "norm": "max |diff| (A) / max |diff| / max |ref|"}
        sv.close()
        log("cpu baseline (oracle)")
        t0 = time.perf_counter()
        done = 0
        while time.perf_counter() - t0 < 12.0:
            ov.md_nve(spos, svel, sm, sbox, ov.tersoff_si(), 1.0, 20)
            done += 20
        spent = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": len(spos) * done / spent, "unit": "atom*steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"{done} steps of the 64-atom cut (pure Python float64 forces, lists rebuilt "
                                         f"every step), {spent:.1f} s"}
    vir.close()
    return res


def run_group(args, prec):
    """The uneven batch as one grouped push per block (graph replay, autotuned tiles)."""
    import torch
    import synth
    from paper_2102_03691_amd import GKMA, HNEMA, ModalGroup, ModalHC
    K = args.steps or GROUP_STEPS
    batch = synth.uneven_batch(0)
    stream = torch.cuda.Stream()
    handle = stream.cuda_stream
    systems, inputs, units_per_block, lats = [], [], 0.0, []
    log(f"uneven batch: edges {[e for e, _ in batch]}, methods {[m for _, m in batch]}")
    n_blocks = None
    for i, (edge, meth) in enumerate(batch):
        lat = synth.BlochLattice((edge, edge, edge))
        m = synth.masses(lat.n_atoms)
        h = ModalHC(0, stream=handle)
        h.load_system(m, lat.frequencies)
        h.set_bins_uniform(GROUP_NB, 0.0, lat.f_max)
        methods = HNEMA if meth == 1 else GKMA
        h.configure(methods=methods, precision=prec, t_block=GROUP_T, corr_len=GROUP_L, dt=1.0)
        M = lat.n_modes
        chunk = max(1, min(M, (512 << 20) // (8 * 3 * lat.n_atoms)))
        for r0 in range(0, M, chunk):
            n = min(chunk, M - r0)
            h.load_eigvec_rows(r0, lat.eig_rows_torch(r0, n, device="cuda:0"))
        torch.cuda.synchronize()
        h.finalize()
        systems.append(h)
        lats.append((lat, m, methods))
        units_per_block += float(lat.n_atoms) * M * GROUP_T
        if n_blocks is None:
            n_blocks = max(1, min(K + args.warmup, 8))
        v, W = synth.gen_steps_torch(100 + i, m, n_blocks * GROUP_T, device="cuda:0")
        inputs.append((v, W))
    torch.cuda.synchronize()
    grp = ModalGroup(systems, graph=not args.no_graph, autotune=True)

    def block(j):
        b = j % n_blocks
        grp.push([v[b * GROUP_T:(b + 1) * GROUP_T] for v, _ in inputs],
                 [W[b * GROUP_T:(b + 1) * GROUP_T] for _, W in inputs])

    for j in range(args.warmup):
        block(j)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(K):
        block(args.warmup + j)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = grp.info()
    # roofline of the grouped contraction: a few eager blocks with HIP events
    grp.set_timing(True)
    for j in range(4):
        block(j)
    launches, kms = grp.kernel_timing()
    grp.set_timing(False)
    avg_ms = kms / max(launches, 1)
    peak = {0: PEAK_FP32_MFMA_FLOPS, 1: PEAK_BF16_FLOPS, 2: PEAK_FP8_FLOPS, 3: PEAK_FP8_FLOPS}[prec]
    achieved = FLOP_PER_UNIT * units_per_block / (avg_ms * 1e-3)
    issued = ISSUED_PER_UNIT[prec] * units_per_block / (avg_ms * 1e-3)
    roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak, "work": "24 FLOP per atom*mode*step (Eq. 13: 3 FMAs; Eq. 16 bracket: 9 FMAs)",
            "achieved_issued": issued / 1e12, "frac_issued": issued / peak,
            "traffic": profiled_traffic(args.workload, "k_gemm_group"),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
            "kernel": "k_gemm_group", "avg_launch_ms": avg_ms,
            "launches": launches, "tile_shape": info["tile_shape"], "autotuned_ms": info["tuned_ms"]}
    acc = None
    if not args.no_cpu_baseline:
        # one grouped block of seeded inputs against the oracle, per system
        log("accuracy: one seeded grouped block against the FP64 oracle")
        for h in systems:
            h.reset()
        host = [synth.gen_steps(200 + i, m, 0, GROUP_T) for i, (_, m, _) in enumerate(lats)]
        grp.push([torch.as_tensor(v, device="cuda:0") for v, _ in host],
                 [torch.as_tensor(W, device="cuda:0") for _, W in host])
        torch.cuda.synchronize()
        worst = {}
        for h, (lat, m, meth), (v, W) in zip(systems, lats, host):
            for k, e in library_errors(h, lattice_reference(lat, m, v, W, GROUP_NB, meth, GROUP_L)).items():
                worst[k] = max(worst.get(k, 0.0), e)
        acc = {**{f"{k}_worst_system": e for k, e in worst.items()},
               "oracle": "binned_current_fft (FFT form of the FP64 oracle, exact for the plane-wave basis)",
               "sample": f"one grouped block of {GROUP_T} seeded MD steps per system after a reset",
               "norm": "relative L2 per output array"}
    grp.close()
    for h in systems:
        h.close()
    return {"metric": METRIC, "value": units_per_block * K / wall, "unit": "atom*mode*steps/s", "n_gpus": 1,
            "steps": K, "warmup": args.warmup, "ms_per_step": wall / K * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": {0: "f32", 1: "bf16x3", 2: "fp8", 3: "fp8x3"}[prec],
            "data": "synthetic",
            "config": {"workload": args.workload, "systems": [[e, m] for e, m in batch],
                       "md_steps_per_step": GROUP_T, "t_block": GROUP_T, "bins": GROUP_NB, "corr_len": GROUP_L,
                       "precision": {0: "fp32", 1: "split-bf16 three products", 2: "e4m3 one product",
                                     3: "e4m3 hi/lo three products"}[prec]
                       + ", per-mode / per-(channel, step) scales for e4m3; fp64 bins and time sums",
                       "launch": "grouped persistent contraction, "
                                 + ("eager launches" if args.no_graph else "HIP graph replay") + ", autotuned tile shape",
                       "parallelism": "single GPU"},
            "roofline": roof, **({"rel_err_vs_oracle": acc} if acc is not None else {})}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT,
                    choices=sorted(WORKLOADS) + sorted(GROUP_WORKLOADS) + sorted(SHC_WORKLOADS)
                    + sorted(SHC_GROUP_WORKLOADS)
                    + sorted(VIRIAL_WORKLOADS) + sorted(MD_WORKLOADS) + sorted(HNEMD_WORKLOADS))
    ap.add_argument("--schedule", type=int, default=0, choices=[0, 1, 2, 3],
                    help="work split of the T-batched contraction: 0 auto, 1 tiles, 2 stream-K, 3 split")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (CPU baseline timing and the accuracy check of one seeded block)")
    ap.add_argument("--no-fp32-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="grouped workloads: launch each block eagerly")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="GiB copied by a plain device copy before the workload (to calibrate HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding over several GPUs is not "
              "implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    if args.copy_probe > 0:
        n = int(args.copy_probe * (1 << 30)) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: 3 copies of {n * 4} bytes")
        del src, dst
    if args.workload in GROUP_WORKLOADS:
        print(json.dumps(run_group(args, GROUP_WORKLOADS[args.workload])), flush=True)
        return
    if args.workload in SHC_WORKLOADS:
        print(json.dumps(run_shc(args)), flush=True)
        return
    if args.workload in SHC_GROUP_WORKLOADS:
        print(json.dumps(run_shc_group(args)), flush=True)
        return
    if args.workload in VIRIAL_WORKLOADS:
        print(json.dumps(run_virial(args)), flush=True)
        return
    if args.workload in MD_WORKLOADS:
        print(json.dumps(run_md(args)), flush=True)
        return
    if args.workload in HNEMD_WORKLOADS:
        print(json.dumps(run_hnemd_shc(args)), flush=True)
        return
    dims, t_block, prec, methods, nb, L, default_steps = WORKLOADS[args.workload]
    K = args.steps or default_steps
    lat = synth.BlochLattice(dims)
    N, M = lat.n_atoms, lat.n_modes
    log(f"workload {args.workload}: N={N} M={M} T={t_block} prec={prec} steps={K} warmup={args.warmup}")
    bins = count_bins(lat.frequencies, nb) if args.workload in COUNT_BINS else None
    h, m = make_context(lat, t_block, prec, methods, nb, L, schedule=args.schedule, bins=bins)
    md_per_step = t_block if t_block > 1 else 256      # per-step path: 256 MD steps per launch
    # inputs resident in HBM before the timed region (distinct block per bench step, cycled if huge)
    bytes_per_block = md_per_step * N * 12 * 4
    n_blocks = max(1, min(K + args.warmup, int(24e9 // bytes_per_block)))
    v, W = synth.gen_steps_torch(1, m, n_blocks * md_per_step, device="cuda:0")
    bv = [v[i * md_per_step:(i + 1) * md_per_step] for i in range(n_blocks)]
    bW = [W[i * md_per_step:(i + 1) * md_per_step] for i in range(n_blocks)]
    log(f"inputs: {n_blocks} blocks resident ({n_blocks * bytes_per_block / 1e9:.2f} GB)")
    wall, launches, kms = time_pushes(h, bv, bW, args.warmup, K)
    sched_used = h.last_schedule()
    units = float(N) * M * md_per_step * K
    value = units / wall
    avg_ms = kms / max(launches, 1)
    units_per_launch = float(N) * M * md_per_step
    if t_block > 1:
        peak = PEAK_BF16_FLOPS if prec == 1 else PEAK_FP32_MFMA_FLOPS
        flops = FLOP_PER_UNIT * units_per_launch
        issued = ISSUED_PER_UNIT[prec] * units_per_launch
        roof = {"bound": "mfma", "achieved": flops / (avg_ms * 1e-3) / 1e12, "peak": peak / 1e12,
                "unit": "TFLOP/s", "work": "24 FLOP per atom*mode*step (Eq. 13: 3 FMAs; Eq. 16 bracket: 9 FMAs)",
                "achieved_issued": issued / (avg_ms * 1e-3) / 1e12, "frac_issued": issued / (avg_ms * 1e-3) / peak}
    else:
        byts = 12.0 * units_per_launch               # E streamed once per MD step: 3 dofs x 4 B per atom*mode
        roof = {"bound": "hbm", "achieved": byts / (avg_ms * 1e-3) / 1e9, "peak": PEAK_HBM_BPS / 1e9, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    kernel = "k_gemv_f32" if t_block == 1 else {1: "k_gemm", 2: "k_gemm", 3: "k_gemm_split"}.get(sched_used, "k_gemm")
    if t_block > 1 and (methods & 4) and prec in (0, 1):
        kernel = "k_gemm_dir"          # the direction split as one contraction
    roof["traffic"] = profiled_traffic(args.workload, kernel)
    roof["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)"
    roof["kernel"] = kernel
    roof["avg_launch_ms"] = avg_ms
    roof["launches"] = launches
    del bv, bW, v, W
    acc = None
    if not args.no_cpu_baseline:
        if bins is None:
            log("accuracy: one seeded block against the FP64 oracle")
            acc = accuracy_vs_oracle(h, lat, m, methods, nb, L, md_per_step if t_block > 1 else 128)
        else:
            acc = {"skipped": "bins of equal mode counts split k-points, which the FFT form of the oracle cannot "
                              "represent; the dense oracle does not fit this basis"}
    h.close()
    torch.cuda.empty_cache()

    out = {"metric": METRIC, "value": value, "unit": "atom*mode*steps/s", "n_gpus": 1, "steps": K,
           "warmup": args.warmup, "ms_per_step": wall / K * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": {0: "f32", 1: "bf16x3"}[prec], "data": "synthetic",
           "config": {"workload": args.workload, "atoms": N, "modes": M, "md_steps_per_step": md_per_step,
                      "t_block": t_block,
                      "bins": nb if bins is None else f"{nb} of equal mode counts in frequency order",
                      "corr_len": L,
                      "schedule": {0: "auto", 1: "tiles", 2: "stream-K", 3: "split"}[args.schedule]
                      + ("" if t_block == 1 else
                         " -> " + {1: "tiles", 2: "stream-K", 3: "split"}.get(sched_used, "?")),
                      "precision": {0: "fp32 operands, fp32 accumulate",
                                    1: "split-bf16 hi*hi+hi*lo+lo*hi, fp32 accumulate"}[prec]
                      + "; fp64 bins and time sums",
                      "parallelism": "single GPU"},
           "roofline": roof}
    if acc is not None:
        out["rel_err_vs_oracle"] = acc

    if not args.no_fp32_baseline and not (prec == 0 and t_block == 1):
        log("plain per-step FP32 path on the same lattice")
        h2, m2 = make_context(lat, 1, 0, 1, nb, 0, bins=bins)
        n_md = 256
        v2, W2 = synth.gen_steps_torch(2, m2, n_md, device="cuda:0")
        wall2, l2, k2 = time_pushes(h2, [v2], [W2], 0, 1)
        h2.close()
        del v2, W2
        torch.cuda.empty_cache()
        v_fp32 = float(N) * M * n_md / wall2
        out["fp32_per_step"] = {"value": v_fp32, "unit": "atom*mode*steps/s", "md_steps": n_md,
                                "ms_per_md_step": wall2 / n_md * 1e3,
                                "hbm_GBps": 12.0 * N * M * n_md / (k2 * 1e-3) / 1e9 if k2 > 0 else None}
        out["speedup_vs_fp32_per_step"] = value / v_fp32

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(dims, t_block, nb, bins=bins)
        log("cpu baseline on one core (oracle)")
        one = cpu_baseline_one_core(dims, t_block, nb, bins=bins)
        if one is not None:
            out["cpu_baseline_one_core"] = one
            out["speedup_vs_one_cpu_core"] = value / one["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
