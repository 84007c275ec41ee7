"""The C ABI used from a C99 program on the GPU: the program (tests/c/abi_run.c)
loads a system, pushes host samples in uneven pieces and reads HNEMA and GKMA
results through include/mhc.h alone; the results are checked against the FP64
oracle (split-BF16 bar 1e-4, float64 totals 1e-12)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2102_03691_amd import _lib
from tests._cases import TOL, Case, announce, log, rel

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    # device_count() does not initialise the HIP runtime in this process: the
    # C program is started as a child process and is then the device's only user
    import torch
    if torch.cuda.device_count() == 0:
        pytest.skip("no GPU")


def _write_case(c, nb, L, T, prec, bins, case):
    N, M, S = c.lat.n_atoms, c.n_modes, c.v.shape[0]
    with open(case, "wb") as fh:
        fh.write(np.array([N, M, S], dtype=np.int64).tobytes())
        fh.write(np.array([nb, L, T, prec], dtype=np.int32).tobytes())
        fh.write(np.ascontiguousarray(c.m, dtype=np.float64).tobytes())
        fh.write(np.ascontiguousarray(c.freq, dtype=np.float64).tobytes())
        fh.write(np.ascontiguousarray(bins, dtype=np.int32).tobytes())
        fh.write(np.ascontiguousarray(c.lat.eig_rows(0, M), dtype=np.float64).tobytes())
        fh.write(np.ascontiguousarray(c.v, dtype=np.float32).tobytes())
        fh.write(np.ascontiguousarray(c.W, dtype=np.float32).tobytes())


def _check_output(c, nb, L, bins, out, tag):
    S = c.v.shape[0]
    raw = np.fromfile(out, dtype=np.float64)
    k = 0
    avg = raw[k:k + nb * 3].reshape(nb, 3); k += nb * 3
    tot = raw[k:k + 3]; k += 3
    corr = raw[k:k + L * nb * 9].reshape(L, nb, 3, 3); k += L * nb * 9
    hcacf = raw[k:k + L * 9].reshape(L, 3, 3); k += L * 9
    n = int(raw[k:k + 1].view(np.int64)[0])
    ref = c.oracle(nb, corr_len=L, bins=bins)
    e = {"rel_hnema": rel(avg, ref["hnema"]), "rel_corr": rel(corr, ref["corr"]),
         "rel_total": rel(tot, ref["hnema_total"]), "rel_hcacf": rel(hcacf, ref["hcacf"])}
    log(tag, **e)
    assert n == S
    assert e["rel_hnema"] <= TOL[1] and e["rel_corr"] <= TOL[1]
    assert e["rel_total"] <= 1e-12 and e["rel_hcacf"] <= 1e-12


def _case():
    c = Case((5, 4, 3), 150, mass_kind="natural", seed=21)
    nb, L, T, prec = 11, 10, 64, 1
    return c, nb, L, T, prec, oracle.bin_of_mode(c.freq, nb, 0.0, c.lat.f_max)


def test_c_program_through_the_abi(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    announce("C program through the ABI, bf16x3 T=64")
    c, nb, L, T, prec, bins = _case()
    case = tmp_path / "case.bin"
    _write_case(c, nb, L, T, prec, bins, case)
    exe = tmp_path / "abi_run"
    lib = _lib.library_path()
    subprocess.run([gcc, "-std=c99", "-O2", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c", "abi_run.c"), lib, "-Wl,-rpath," + os.path.dirname(lib),
                    "-o", str(exe)], check=True)
    out = tmp_path / "out.bin"
    r = subprocess.run([str(exe), str(case), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    _check_output(c, nb, L, bins, out, "c_abi_5x4x3_bf16x3_T64")


SAN_DIR = os.path.join(ROOT, "tests", "c", "build")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")


def test_c_programs_under_host_sanitizers(tmp_path):
    """The same program and the error-path driver (tests/c/abi_errors.c: corrupted
    saved states, bad arguments of every object) linked against the host
    AddressSanitizer + UndefinedBehaviorSanitizer build of the C ABI."""
    run_exe, err_exe = os.path.join(SAN_DIR, "abi_run_asan"), os.path.join(SAN_DIR, "abi_errors_asan")
    if not (os.path.exists(run_exe) and os.path.exists(err_exe)):
        pytest.skip("sanitized drivers not built (paper_2102_03691_amd._build.build_sanitized)")
    announce("C programs under host ASan + UBSan")
    r = subprocess.run([err_exe], capture_output=True, text=True, timeout=120, env=SAN_ENV)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "abi_errors: ok" in r.stdout and "no device" not in r.stdout
    c, nb, L, T, prec, bins = _case()
    case = tmp_path / "case.bin"
    _write_case(c, nb, L, T, prec, bins, case)
    out = tmp_path / "out.bin"
    r = subprocess.run([run_exe, str(case), str(out)], capture_output=True, text=True, timeout=120, env=SAN_ENV)
    assert r.returncode == 0, r.stderr
    _check_output(c, nb, L, bins, out, "c_abi_asan_5x4x3_bf16x3_T64")
