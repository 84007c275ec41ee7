"""The C ABI without a GPU: the library loads, exports every declared entry
point, validates arguments, and its host-only bin rule matches the oracle's."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_2102_03691_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mhc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mhc_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = _lib.library()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_abi_version_and_status_strings():
    lib = _lib.library()
    assert lib.mhc_abi_version() == 1
    for code, name in _lib._STATUS.items():
        assert lib.mhc_status_string(code).decode() == name


@pytest.mark.parametrize("dims,nb", [((4, 4, 4), 100), ((16, 16, 16), 500), ((48, 48, 4), 1000),
                                     ((6, 6, 6), 37), ((10, 10, 10), 500)])
def test_uniform_bins_match_oracle_exactly(dims, nb):
    lat = synth.BlochLattice(dims)
    f = lat.frequencies
    got = _lib.bins_uniform(f, nb, 0.0, lat.f_max)
    want = oracle.bin_of_mode(f, nb, 0.0, lat.f_max)
    np.testing.assert_array_equal(got, want)


def test_uniform_bins_edges_and_exclusion():
    f = np.array([0.0, 1.999, 2.0, np.nextafter(2.0, 0), 7.999, 8.0, -0.1, 8.1, 5.0])
    np.testing.assert_array_equal(_lib.bins_uniform(f, 4, 0.0, 8.0), oracle.bin_of_mode(f, 4, 0.0, 8.0))


def test_uniform_bins_rejects_bad_arguments():
    f = np.ones(3)
    for nb, lo, hi in [(0, 0.0, 1.0), (4, 1.0, 1.0), (4, 2.0, 1.0), (4, 0.0, float("nan"))]:
        with pytest.raises(_lib.MhcError):
            _lib.bins_uniform(f, nb, lo, hi)


def test_null_context_and_null_pointers_are_invalid_arg():
    lib = _lib.library()
    assert lib.mhc_load_system(None, 1, None, 1, None) == 1
    assert lib.mhc_push(None, 1, None, None, 0) == 1
    assert lib.mhc_finalize(None) == 1
    assert lib.mhc_read_hnema_dir(None, None, None, None) == 1
    assert lib.mhc_read_gkma_dir(None, None, None, None) == 1
    assert lib.mhc_create(0, None, None) == 1
    assert lib.mhc_destroy(None) == 0


def test_create_without_gpu_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = _lib.library()
    h = C.c_void_p()
    assert lib.mhc_create(0, None, C.byref(h)) == 4
    assert h.value is None
    assert b"HIP" in lib.mhc_last_error(None) or len(lib.mhc_last_error(None)) > 0


def test_shc_entry_points_validate_before_touching_a_device():
    lib = _lib.library()
    h = C.c_void_p()
    assert lib.mhc_shc_create(0, None, 10, 0, 64, C.byref(h)) == 1        # no lags
    assert lib.mhc_shc_create(0, None, 10, 8, 100, C.byref(h)) == 1       # t_block not a multiple of 64
    assert lib.mhc_shc_create(0, None, 0, 8, 64, C.byref(h)) == 1         # no atoms
    assert lib.mhc_shc_create(0, None, 10, 8, 64, None) == 1
    assert lib.mhc_shc_push(None, 1, None, None, 0) == 1
    assert lib.mhc_shc_read(None, None, None) == 1
    assert lib.mhc_shc_destroy(None) == 0


def test_shc_create_without_gpu_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = _lib.library()
    h = C.c_void_p()
    assert lib.mhc_shc_create(0, None, 10, 8, 64, C.byref(h)) == 4
    assert h.value is None


def test_header_compiles_as_c_and_links(tmp_path):
    """include/mhc.h is plain C: a C99 program that uses it builds against the
    library and runs its host-only helpers (no GPU needed)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lib = _lib.library_path()
    src = tmp_path / "use_mhc.c"
    src.write_text(r'''
#include <stdio.h>
#include "mhc.h"
int main(void) {
  double f[4] = {0.5, 1.5, 2.5, 3.5};
  int32_t b[4];
  mhc_status st = mhc_bins_uniform(4, f, 2, 0.0, 4.0, b);
  mhc_run_config cfg = {MHC_HNEMA | MHC_GKMA | MHC_DIRECTIONAL, MHC_PREC_BF16X3, 128, 10, 1.0, 0, MHC_SCHED_AUTO, {0, 0}};
  printf("%d %d %d %d %d %d %s\n", (int)st, b[0], b[1], b[2], b[3], mhc_abi_version(), mhc_status_string(MHC_ERR_STATE));
  return cfg.t_block == 128 ? 0 : 1;
}
''')
    exe = tmp_path / "use_mhc"
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(root, "include"), str(src), lib,
                    "-Wl,-rpath," + os.path.dirname(lib), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    assert out[:5] == ["0", "0", "0", "1", "1"] and out[5] == "1" and out[6] == "MHC_ERR_STATE"


def test_header_compiles_as_cpp_and_links(tmp_path):
    """The same program as C++17: the header's extern "C" guards give the
    library's unmangled symbols."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lib = _lib.library_path()
    src = tmp_path / "use_mhc.cpp"
    src.write_text(r'''
#include <cstdio>
#include "mhc.h"
int main() {
  const double f[4] = {0.5, 1.5, 2.5, 3.5};
  int32_t b[4];
  const mhc_status st = mhc_bins_uniform(4, f, 2, 0.0, 4.0, b);
  mhc_ctx* ctx = nullptr;
  const mhc_status bad = mhc_push(ctx, 1, nullptr, nullptr, 0);
  std::printf("%d %d %d %d %d %d\n", (int)st, b[0], b[1], b[2], b[3], (int)bad);
  return 0;
}
''')
    exe = tmp_path / "use_mhc_cpp"
    subprocess.run([gxx, "-std=c++17", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(root, "include"),
                    str(src), lib, "-Wl,-rpath," + os.path.dirname(lib), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    assert out == ["0", "0", "0", "1", "1", "1"]


def test_bench_refuses_several_gpus():
    """bench.py runs on one GPU: --gpus above 1 exits with status 2 and a message, before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in (r.stdout + r.stderr)


def test_c_abi_driver_builds(tmp_path):
    """tests/c/abi_run.c (the C99 program the GPU test runs through the ABI)
    compiles with -Wall -Werror and links against the library."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lib = _lib.library_path()
    subprocess.run([gcc, "-std=c99", "-O2", "-Wall", "-Werror", "-I", os.path.join(root, "include"),
                    os.path.join(root, "tests", "c", "abi_run.c"), lib, "-Wl,-rpath," + os.path.dirname(lib),
                    "-o", str(tmp_path / "abi_run")], check=True)
    assert (tmp_path / "abi_run").exists()


def test_virial_create_validates_arguments_without_a_gpu():
    """mhc_virial_create checks its arguments before any HIP call."""
    import ctypes as C
    from oracle import virial as ov
    lib = _lib.library()
    p = ov.tersoff_si()
    good = dict(A=p["A"], B=p["B"], lambda1=p["lambda1"], lambda2=p["lambda2"], lambda3=0.0, m=3, reserved=0,
                beta=p["beta"], n=p["n"], c=p["c"], d=p["d"], h=p["h"], gamma=1.0, R=p["R"], D=p["D"])
    m = np.full(8, 28.0855)
    box = np.full(3, 10.0)
    out = C.c_void_p()

    def create(mass=m, bx=box, max_nb=16, skin=0.0, **kw):
        tp = _lib.TersoffParams(**{**good, **kw})
        return lib.mhc_virial_create(0, None, len(mass), mass.ctypes.data, bx.ctypes.data, C.byref(tp), max_nb,
                                     skin, C.byref(out))

    assert create(bx=np.full(3, 5.9)) == 1                      # box edge below 2 (R + D)
    assert b"twice" in lib.mhc_virial_last_error(None)
    assert create(skin=2.0) == 1                                # 2 (R + D + skin) = 10 is not below the box
    assert create(m=2) == 1
    assert create(reserved=1) == 1
    assert create(D=0.0) == 1
    assert create(max_nb=0) == 1 and create(max_nb=65) == 1
    assert create(mass=np.array([28.0, -1.0])) == 1
    assert create(n=float("nan")) == 1
    assert lib.mhc_virial_create(0, None, 8, None, box.ctypes.data, None, 16, 0.0, C.byref(out)) == 1
    assert lib.mhc_virial_destroy(None) == 0
    assert lib.mhc_virial_compute(None, None, None, None, None, None, None, None, None) == 1
