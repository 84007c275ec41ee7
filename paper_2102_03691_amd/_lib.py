"""ctypes binding of libmodalhc (include/mhc.h): argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import _build

HNEMA, GKMA, DIRECTIONAL, CROSS = 1, 2, 4, 8
PREC_FP32, PREC_BF16X3, PREC_FP8, PREC_FP8X3 = 0, 1, 2, 3
SCHED_AUTO, SCHED_TILES, SCHED_STREAMK, SCHED_SPLIT = 0, 1, 2, 3
GROUP_GRAPH, GROUP_AUTOTUNE = 1, 2

_STATUS = {0: "MHC_OK", 1: "MHC_ERR_INVALID_ARG", 2: "MHC_ERR_STATE", 3: "MHC_ERR_OOM",
           4: "MHC_ERR_HIP", 5: "MHC_ERR_UNSUPPORTED", 6: "MHC_ERR_NONFINITE"}


class MhcError(RuntimeError):
    """A library call returned a status other than MHC_OK."""

    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class RunConfig(C.Structure):
    _fields_ = [("methods", C.c_int32), ("precision", C.c_int32), ("t_block", C.c_int32),
                ("corr_len", C.c_int32), ("dt", C.c_double), ("check_finite", C.c_int32),
                ("schedule", C.c_int32), ("reserved", C.c_int32 * 2)]


class TersoffParams(C.Structure):
    _fields_ = [("A", C.c_double), ("B", C.c_double), ("lambda1", C.c_double), ("lambda2", C.c_double),
                ("lambda3", C.c_double), ("m", C.c_int32), ("reserved", C.c_int32), ("beta", C.c_double),
                ("n", C.c_double), ("c", C.c_double), ("d", C.c_double), ("h", C.c_double), ("gamma", C.c_double),
                ("R", C.c_double), ("D", C.c_double)]


_lib = None


def library_path() -> str:
    return _build.LIB


def library():
    """Load libmodalhc.so (built in-tree by _build.build()); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2102_03691_amd._build.build(); "
                           "there is no fallback path")
    try:
        # torch, when present, loads its HIP runtime first, so that the
        # library binds to the same runtime instead of a second copy
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "mhc_create": (i32, [C.c_int, vp, P(vp)]),
        "mhc_destroy": (i32, [vp]),
        "mhc_last_error": (C.c_char_p, [vp]),
        "mhc_status_string": (C.c_char_p, [i32]),
        "mhc_abi_version": (C.c_int, []),
        "mhc_load_system": (i32, [vp, i64, vp, i64, vp]),
        "mhc_set_bins": (i32, [vp, i32, vp]),
        "mhc_set_bins_uniform": (i32, [vp, i32, dbl, dbl]),
        "mhc_bins_uniform": (i32, [i64, vp, i32, dbl, dbl, vp]),
        "mhc_configure": (i32, [vp, P(RunConfig)]),
        "mhc_load_eigvec_rows": (i32, [vp, i64, i64, vp, C.c_int]),
        "mhc_finalize": (i32, [vp]),
        "mhc_push": (i32, [vp, i32, vp, vp, C.c_int]),
        "mhc_push_noalloc": (i32, [vp, i32, vp, vp]),
        "mhc_synchronize": (i32, [vp]),
        "mhc_read_hnema": (i32, [vp, vp, vp, P(i64)]),
        "mhc_read_gkma": (i32, [vp, vp, vp, vp, P(i64)]),
        "mhc_read_hnema_dir": (i32, [vp, vp, vp, P(i64)]),
        "mhc_read_gkma_dir": (i32, [vp, vp, vp, P(i64)]),
        "mhc_read_gkma_cross": (i32, [vp, vp, vp, P(i64)]),
        "mhc_read_block_currents": (i32, [vp, i32, vp]),
        "mhc_reset": (i32, [vp]),
        "mhc_save_state": (i32, [vp, vp, P(C.c_size_t)]),
        "mhc_load_state": (i32, [vp, vp, C.c_size_t]),
        "mhc_set_timing": (i32, [vp, C.c_int]),
        "mhc_kernel_timing": (i32, [vp, P(i64), P(dbl)]),
        "mhc_device_bytes": (i32, [vp, P(i64)]),
        "mhc_last_schedule": (i32, [vp, P(i32)]),
        "mhc_shc_create": (i32, [C.c_int, vp, i64, i32, i32, P(vp)]),
        "mhc_shc_destroy": (i32, [vp]),
        "mhc_shc_last_error": (C.c_char_p, [vp]),
        "mhc_shc_push": (i32, [vp, i32, vp, vp, C.c_int]),
        "mhc_shc_read": (i32, [vp, vp, P(i64)]),
        "mhc_shc_spectrum": (i32, [vp, i32, vp, dbl, i32, vp]),
        "mhc_shc_read_dir": (i32, [vp, vp, P(i64)]),
        "mhc_shc_save_state": (i32, [vp, vp, P(C.c_size_t)]),
        "mhc_shc_load_state": (i32, [vp, vp, C.c_size_t]),
        "mhc_shc_spectrum_dir": (i32, [vp, i32, vp, dbl, i32, vp]),
        "mhc_shc_reset": (i32, [vp]),
        "mhc_shc_synchronize": (i32, [vp]),
        "mhc_shc_set_timing": (i32, [vp, C.c_int]),
        "mhc_shc_kernel_timing": (i32, [vp, P(i64), P(dbl)]),
        "mhc_shc_group_create": (i32, [P(vp), i32, P(vp)]),
        "mhc_shc_group_destroy": (i32, [vp]),
        "mhc_shc_group_last_error": (C.c_char_p, [vp]),
        "mhc_shc_group_push": (i32, [vp, i32, P(vp), P(vp), C.c_int]),
        "mhc_virial_create": (i32, [C.c_int, vp, i64, vp, vp, P(TersoffParams), i32, dbl, P(vp)]),
        "mhc_virial_destroy": (i32, [vp]),
        "mhc_virial_last_error": (C.c_char_p, [vp]),
        "mhc_virial_neighbors": (i32, [vp, vp, P(i32)]),
        "mhc_virial_read_neighbors": (i32, [vp, vp, vp]),
        "mhc_virial_compute": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "mhc_virial_synchronize": (i32, [vp]),
        "mhc_virial_set_timing": (i32, [vp, C.c_int]),
        "mhc_virial_kernel_timing": (i32, [vp, P(i64), P(dbl), P(dbl)]),
        "mhc_virial_md": (i32, [vp, vp, vp, dbl, i32, i32, vp, vp, vp]),
        "mhc_virial_md_nvt": (i32, [vp, vp, vp, dbl, i32, i32, vp, dbl, dbl, vp, vp, vp, vp]),
        "mhc_group_create": (i32, [P(vp), i32, i32, P(vp)]),
        "mhc_group_destroy": (i32, [vp]),
        "mhc_group_last_error": (C.c_char_p, [vp]),
        "mhc_group_push": (i32, [vp, i32, P(vp), P(vp), C.c_int]),
        "mhc_group_info": (i32, [vp, P(i32), P(dbl), P(i64)]),
        "mhc_group_set_timing": (i32, [vp, C.c_int]),
        "mhc_group_kernel_timing": (i32, [vp, P(i64), P(dbl)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return library().mhc_status_string(status).decode()


def _ptr(a) -> int:
    return a.ctypes.data if isinstance(a, np.ndarray) else int(a.data_ptr())


def bins_uniform(freq, n_bins: int, f_lo: float, f_hi: float) -> np.ndarray:
    """Host-only bin map (no GPU): the rule mhc_set_bins_uniform applies."""
    f = np.ascontiguousarray(freq, dtype=np.float64)
    out = np.empty(f.shape[0], dtype=np.int32)
    st = library().mhc_bins_uniform(f.shape[0], _ptr(f), int(n_bins), float(f_lo), float(f_hi), _ptr(out))
    if st:
        raise MhcError(st, "mhc_bins_uniform")
    return out


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


class _StreamUse:
    """Stream ordering of device tensors handed to a context whose stream is not
    torch's current one: the context stream waits for the work queued so far on
    the current stream (which produced the tensors), and each tensor is recorded
    on the context stream so that torch's caching allocator does not hand its
    memory out again before the context has read it."""

    def __init__(self, device: int, handle: int):
        self.device = int(device)
        self.handle = int(handle)
        self._stream = None

    def __call__(self, *tensors):
        import torch
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream == self.handle:
            return
        if self._stream is None:
            dflt = torch.cuda.default_stream(self.device)
            self._stream = dflt if dflt.cuda_stream == self.handle else \
                torch.cuda.ExternalStream(self.handle, device=self.device)
        self._stream.wait_stream(cur)
        for t in tensors:
            t.record_stream(self._stream)


class ModalHC:
    """One system (basis, bins, configuration, accumulators) on one GPU.

    Device inputs are torch tensors on the context's device (passed by
    pointer); host inputs are numpy arrays.  By default work is queued on
    torch's current stream of that device, so it orders with torch ops.  With
    another stream, each call that takes device tensors first makes that stream
    wait for torch's current stream and records the tensors on it.
    """

    def __init__(self, device: int = 0, stream=None):
        self._lib = library()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        h = C.c_void_p()
        st = self._lib.mhc_create(int(device), C.c_void_p(int(stream) if stream else 0), C.byref(h))
        if st:
            raise MhcError(st, self._lib.mhc_last_error(None).decode())
        self._h = h
        self._use = _StreamUse(device, int(stream) if stream else 0)
        self.device = device
        self.nb = None
        self.n_atoms = None
        self.cfg = None

    # -- plumbing
    def _check(self, st, what):
        if st:
            raise MhcError(st, f"{what}: {self._lib.mhc_last_error(self._h).decode()}")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mhc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- loading
    def load_system(self, mass, freq):
        m = np.ascontiguousarray(mass, dtype=np.float64)
        f = np.ascontiguousarray(freq, dtype=np.float64)
        self._check(self._lib.mhc_load_system(self._h, m.shape[0], _ptr(m), f.shape[0], _ptr(f)), "load_system")
        self.n_atoms = m.shape[0]
        self.n_modes = f.shape[0]

    def set_bins(self, n_bins, bins):
        b = np.ascontiguousarray(bins, dtype=np.int32)
        self._check(self._lib.mhc_set_bins(self._h, int(n_bins), _ptr(b)), "set_bins")
        self.nb = int(n_bins)

    def set_bins_uniform(self, n_bins, f_lo, f_hi):
        self._check(self._lib.mhc_set_bins_uniform(self._h, int(n_bins), float(f_lo), float(f_hi)), "set_bins_uniform")
        self.nb = int(n_bins)

    def configure(self, methods=HNEMA, precision=PREC_FP32, t_block=1, corr_len=0, dt=1.0, check_finite=False,
                  schedule=SCHED_AUTO):
        cfg = RunConfig(int(methods), int(precision), int(t_block), int(corr_len), float(dt), int(bool(check_finite)),
                        int(schedule))
        self._check(self._lib.mhc_configure(self._h, C.byref(cfg)), "configure")
        self.cfg = dict(methods=methods, precision=precision, t_block=t_block, corr_len=corr_len, dt=dt,
                        schedule=schedule)

    def load_eigvec_rows(self, mode0, rows):
        """rows: E^T rows [n, 3N] float64, numpy (host) or torch (device)."""
        if _is_torch(rows):
            assert rows.dtype.is_floating_point and rows.element_size() == 8 and rows.is_contiguous()
            self._use(rows)
            self._check(self._lib.mhc_load_eigvec_rows(self._h, int(mode0), rows.shape[0], _ptr(rows), 1),
                        "load_eigvec_rows")
        else:
            r = np.ascontiguousarray(rows, dtype=np.float64)
            self._check(self._lib.mhc_load_eigvec_rows(self._h, int(mode0), r.shape[0], _ptr(r), 0),
                        "load_eigvec_rows")

    def finalize(self):
        self._check(self._lib.mhc_finalize(self._h), "finalize")

    # -- stepping
    def push(self, v, W):
        """v [S, N, 3] and W [S, N, 3, 3] float32 (numpy host or torch device)."""
        if _is_torch(v):
            assert v.is_contiguous() and W.is_contiguous() and v.element_size() == 4 and W.element_size() == 4
            assert v.shape[0] == W.shape[0] and v.numel() == v.shape[0] * self.n_atoms * 3
            assert W.numel() == W.shape[0] * self.n_atoms * 9
            self._use(v, W)
            self._check(self._lib.mhc_push(self._h, v.shape[0], _ptr(v), _ptr(W), 1), "push")
        else:
            vv = np.ascontiguousarray(v, dtype=np.float32)
            WW = np.ascontiguousarray(W, dtype=np.float32)
            assert vv.shape[0] == WW.shape[0] and vv.size == vv.shape[0] * self.n_atoms * 3
            assert WW.size == WW.shape[0] * self.n_atoms * 9
            self._check(self._lib.mhc_push(self._h, vv.shape[0], _ptr(vv), _ptr(WW), 0), "push")

    def push_noalloc(self, v, W):
        """mhc_push_noalloc: v [S, N, 3] and W [S, N, 3, 3] float32 torch tensors on the context's device."""
        assert _is_torch(v) and _is_torch(W) and v.is_cuda and W.is_cuda
        assert v.is_contiguous() and W.is_contiguous() and v.element_size() == 4 and W.element_size() == 4
        assert v.shape[0] == W.shape[0] and v.numel() == v.shape[0] * self.n_atoms * 3
        assert W.numel() == W.shape[0] * self.n_atoms * 9
        self._use(v, W)
        self._check(self._lib.mhc_push_noalloc(self._h, v.shape[0], _ptr(v), _ptr(W)), "push_noalloc")

    def synchronize(self):
        self._check(self._lib.mhc_synchronize(self._h), "synchronize")

    # -- reading
    def read_hnema(self):
        avg = np.empty((self.nb, 3), dtype=np.float64)
        tot = np.empty(3, dtype=np.float64)
        n = C.c_int64()
        self._check(self._lib.mhc_read_hnema(self._h, _ptr(avg), _ptr(tot), C.byref(n)), "read_hnema")
        return avg, tot, n.value

    def read_gkma(self):
        L = int(self.cfg["corr_len"])
        corr = np.empty((L, self.nb, 3, 3), dtype=np.float64)
        integ = np.empty_like(corr)
        hc = np.empty((L, 3, 3), dtype=np.float64)
        n = C.c_int64()
        self._check(self._lib.mhc_read_gkma(self._h, _ptr(corr), _ptr(integ), _ptr(hc), C.byref(n)), "read_gkma")
        return {"corr": corr, "integral": integ, "hcacf": hc, "n_samples": n.value}

    def read_hnema_dir(self):
        """Split by the atoms' motion direction: (avg [nb, 3 mu, 3 nu], total [3 mu, 3 nu], S)."""
        avg = np.empty((self.nb, 3, 3), dtype=np.float64)
        tot = np.empty((3, 3), dtype=np.float64)
        n = C.c_int64()
        self._check(self._lib.mhc_read_hnema_dir(self._h, _ptr(avg), _ptr(tot), C.byref(n)), "read_hnema_dir")
        return avg, tot, n.value

    def read_gkma_dir(self):
        """<J_b^{mu nu}(t + tau) J^{mu2}(t)> and its running integral, [L, nb, 3 mu, 3 nu, 3 mu2]."""
        L = int(self.cfg["corr_len"])
        corr = np.empty((L, self.nb, 3, 3, 3), dtype=np.float64)
        integ = np.empty_like(corr)
        n = C.c_int64()
        self._check(self._lib.mhc_read_gkma_dir(self._h, _ptr(corr), _ptr(integ), C.byref(n)), "read_gkma_dir")
        return {"corr": corr, "integral": integ, "n_samples": n.value}

    def read_gkma_cross(self):
        """<J_b^mu(t + tau) J_b2^nu(t)> and its running integral, [L, nb, nb, 3 mu, 3 nu]."""
        L = int(self.cfg["corr_len"])
        corr = np.empty((L, self.nb, self.nb, 3, 3), dtype=np.float64)
        integ = np.empty_like(corr)
        n = C.c_int64()
        self._check(self._lib.mhc_read_gkma_cross(self._h, _ptr(corr), _ptr(integ), C.byref(n)), "read_gkma_cross")
        return {"corr": corr, "integral": integ, "n_samples": n.value}

    def read_block_currents(self, t_count):
        out = np.empty((t_count, self.nb, 3), dtype=np.float64)
        self._check(self._lib.mhc_read_block_currents(self._h, int(t_count), _ptr(out)), "read_block_currents")
        return out

    def reset(self):
        self._check(self._lib.mhc_reset(self._h), "reset")

    def save_state(self) -> bytes:
        n = C.c_size_t()
        self._check(self._lib.mhc_save_state(self._h, None, C.byref(n)), "save_state")
        buf = C.create_string_buffer(n.value)
        self._check(self._lib.mhc_save_state(self._h, buf, C.byref(n)), "save_state")
        return buf.raw[: n.value]

    def load_state(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        self._check(self._lib.mhc_load_state(self._h, buf, len(data)), "load_state")

    # -- diagnostics
    def set_timing(self, enable=True):
        self._check(self._lib.mhc_set_timing(self._h, int(bool(enable))), "set_timing")

    def kernel_timing(self):
        n = C.c_int64()
        ms = C.c_double()
        self._check(self._lib.mhc_kernel_timing(self._h, C.byref(n), C.byref(ms)), "kernel_timing")
        return n.value, ms.value

    def device_bytes(self):
        b = C.c_int64()
        self._check(self._lib.mhc_device_bytes(self._h, C.byref(b)), "device_bytes")
        return b.value

    def last_schedule(self):
        """Work split of the last T-batched contraction (SCHED_TILES/_STREAMK/_SPLIT; 0 before any)."""
        s = C.c_int32()
        self._check(self._lib.mhc_last_schedule(self._h, C.byref(s)), "last_schedule")
        return s.value


class ModalGroup:
    """Several ModalHC systems advanced together (mhc_group_*).

    The systems must share one device, one stream, the precision and t_block.
    """

    def __init__(self, systems, graph=True, autotune=True):
        self._lib = library()
        self.systems = list(systems)
        arr = (C.c_void_p * len(self.systems))(*[s._h.value for s in self.systems])
        h = C.c_void_p()
        flags = (GROUP_GRAPH if graph else 0) | (GROUP_AUTOTUNE if autotune else 0)
        st = self._lib.mhc_group_create(arr, len(self.systems), flags, C.byref(h))
        if st:
            why = {1: "the systems must be distinct and share one device, one stream (contexts created with a "
                      "null stream each own a stream of their own), the precision and t_block",
                   2: "every system must be finalized, with t_block > 1",
                   5: "systems with the motion-direction split cannot be grouped"}.get(st, "")
            raise MhcError(st, f"mhc_group_create: {why}" if why else "mhc_group_create")
        self._h = h

    def _check(self, st, what):
        if st:
            raise MhcError(st, f"{what}: {self._lib.mhc_group_last_error(self._h).decode()}")

    def push(self, vs, Ws):
        """vs[i], Ws[i]: system i's [S, N_i, 3] and [S, N_i, 3, 3] float32 (all torch or all numpy)."""
        n = len(self.systems)
        S = vs[0].shape[0]
        dev = _is_torch(vs[0])
        keep = []
        for i, sysm in enumerate(self.systems):
            v, W = vs[i], Ws[i]
            assert v.shape[0] == S and W.shape[0] == S
            if dev:
                assert v.is_contiguous() and W.is_contiguous()
                assert v.numel() == S * sysm.n_atoms * 3 and W.numel() == S * sysm.n_atoms * 9
                keep += [v, W]
            else:
                v = np.ascontiguousarray(v, dtype=np.float32)
                W = np.ascontiguousarray(W, dtype=np.float32)
                assert v.size == S * sysm.n_atoms * 3 and W.size == S * sysm.n_atoms * 9
                keep += [v, W]
            vs_i, Ws_i = (v, W)
            if i == 0:
                pv = (C.c_void_p * n)()
                pW = (C.c_void_p * n)()
            pv[i] = _ptr(vs_i)
            pW[i] = _ptr(Ws_i)
        if dev:
            # the systems share one stream: one wait on torch's stream for all inputs
            self.systems[0]._use(*keep)
        self._check(self._lib.mhc_group_push(self._h, S, pv, pW, 1 if dev else 0), "group_push")

    def info(self):
        shape = C.c_int32()
        ms = (C.c_double * 3)()
        nt = C.c_int64()
        self._check(self._lib.mhc_group_info(self._h, C.byref(shape), ms, C.byref(nt)), "group_info")
        return {"tile_shape": shape.value, "tuned_ms": list(ms), "n_tiles": nt.value}

    def set_timing(self, enable=True):
        self._check(self._lib.mhc_group_set_timing(self._h, int(bool(enable))), "group_set_timing")

    def kernel_timing(self):
        n = C.c_int64()
        ms = C.c_double()
        self._check(self._lib.mhc_group_kernel_timing(self._h, C.byref(n), C.byref(ms)), "group_kernel_timing")
        return n.value, ms.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mhc_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ModalSHC:
    """Spectral heat current (mhc_shc_*): the virial-velocity correlation of
    Eq. 21 over n_lags lags and its transform (Eq. 22); no eigenvectors.

    Inputs as for ModalHC.push (torch device tensors or numpy host arrays);
    work is queued on torch's current stream by default."""

    def __init__(self, n_atoms: int, n_lags: int, t_block: int = 256, device: int = 0, stream=None):
        self._lib = library()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        h = C.c_void_p()
        st = self._lib.mhc_shc_create(int(device), C.c_void_p(int(stream) if stream else 0), int(n_atoms),
                                      int(n_lags), int(t_block), C.byref(h))
        if st:
            raise MhcError(st, self._lib.mhc_shc_last_error(None).decode())
        self._h = h
        self._use = _StreamUse(device, int(stream) if stream else 0)
        self.n_atoms, self.n_lags, self.t_block = int(n_atoms), int(n_lags), int(t_block)

    def _check(self, st, what):
        if st:
            raise MhcError(st, f"{what}: {self._lib.mhc_shc_last_error(self._h).decode()}")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mhc_shc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def push(self, v, W):
        """v [S, N, 3] and W [S, N, 3, 3] float32 (numpy host or torch device)."""
        if _is_torch(v):
            assert v.is_contiguous() and W.is_contiguous() and v.element_size() == 4 and W.element_size() == 4
            assert v.shape[0] == W.shape[0] and v.numel() == v.shape[0] * self.n_atoms * 3
            assert W.numel() == W.shape[0] * self.n_atoms * 9
            self._use(v, W)
            self._check(self._lib.mhc_shc_push(self._h, v.shape[0], _ptr(v), _ptr(W), 1), "shc push")
        else:
            vv = np.ascontiguousarray(v, dtype=np.float32)
            WW = np.ascontiguousarray(W, dtype=np.float32)
            assert vv.shape[0] == WW.shape[0] and vv.size == vv.shape[0] * self.n_atoms * 3
            assert WW.size == WW.shape[0] * self.n_atoms * 9
            self._check(self._lib.mhc_shc_push(self._h, vv.shape[0], _ptr(vv), _ptr(WW), 0), "shc push")

    def read(self):
        """(K [n_lags, 3] float64, number of samples)."""
        K = np.empty((self.n_lags, 3), dtype=np.float64)
        n = C.c_int64()
        self._check(self._lib.mhc_shc_read(self._h, _ptr(K), C.byref(n)), "shc read")
        return K, n.value

    def spectrum(self, omega, dt: float, window: bool = False):
        """Eq. 22 on the sampled lags at the angular frequencies omega: [n_omega, 3]."""
        om = np.ascontiguousarray(omega, dtype=np.float64).ravel()
        out = np.empty((om.shape[0], 3), dtype=np.float64)
        self._check(self._lib.mhc_shc_spectrum(self._h, om.shape[0], _ptr(om), float(dt), int(bool(window)),
                                               _ptr(out)), "shc spectrum")
        return out

    def read_dir(self):
        """Split by the atoms' motion direction: (K [n_lags, 3 mu, 3 nu], number of samples)."""
        K = np.empty((self.n_lags, 3, 3), dtype=np.float64)
        n = C.c_int64()
        self._check(self._lib.mhc_shc_read_dir(self._h, _ptr(K), C.byref(n)), "shc read_dir")
        return K, n.value

    def spectrum_dir(self, omega, dt: float, window: bool = False):
        """Eq. 22 of each split component: [n_omega, 3 mu, 3 nu]."""
        om = np.ascontiguousarray(omega, dtype=np.float64).ravel()
        out = np.empty((om.shape[0], 3, 3), dtype=np.float64)
        self._check(self._lib.mhc_shc_spectrum_dir(self._h, om.shape[0], _ptr(om), float(dt), int(bool(window)),
                                                   _ptr(out)), "shc spectrum_dir")
        return out

    def reset(self):
        self._check(self._lib.mhc_shc_reset(self._h), "shc reset")

    def save_state(self) -> bytes:
        n = C.c_size_t()
        self._check(self._lib.mhc_shc_save_state(self._h, None, C.byref(n)), "shc save_state")
        buf = C.create_string_buffer(n.value)
        self._check(self._lib.mhc_shc_save_state(self._h, buf, C.byref(n)), "shc save_state")
        return buf.raw[: n.value]

    def load_state(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        self._check(self._lib.mhc_shc_load_state(self._h, buf, len(data)), "shc load_state")

    def synchronize(self):
        self._check(self._lib.mhc_shc_synchronize(self._h), "shc synchronize")

    def set_timing(self, enable=True):
        """False / 0: off; True / 1: time every block; k > 1: every k-th."""
        self._check(self._lib.mhc_shc_set_timing(self._h, int(enable)), "shc set_timing")

    def kernel_timing(self):
        n = C.c_int64()
        ms = C.c_double()
        self._check(self._lib.mhc_shc_kernel_timing(self._h, C.byref(n), C.byref(ms)), "shc kernel_timing")
        return n.value, ms.value


class SHCGroup:
    """Several ModalSHC systems advanced by one launch per kernel and block
    (mhc_shc_group_*).  The systems must share one device, one stream and
    t_block; their sizes and lag counts may differ."""

    def __init__(self, systems):
        self._lib = library()
        self.systems = list(systems)
        arr = (C.c_void_p * len(self.systems))(*[s._h.value for s in self.systems])
        h = C.c_void_p()
        st = self._lib.mhc_shc_group_create(arr, len(self.systems), C.byref(h))
        if st:
            raise MhcError(st, f"mhc_shc_group_create: {self._lib.mhc_shc_group_last_error(None).decode()}")
        self._h = h

    def _check(self, st, what):
        if st:
            raise MhcError(st, f"{what}: {self._lib.mhc_shc_group_last_error(self._h).decode()}")

    def push(self, vs, Ws):
        """vs[i], Ws[i]: system i's [S, N_i, 3] and [S, N_i, 3, 3] float32 (all torch or all numpy)."""
        n = len(self.systems)
        S = vs[0].shape[0]
        dev = _is_torch(vs[0])
        keep = []
        pv = (C.c_void_p * n)()
        pW = (C.c_void_p * n)()
        for i, sysm in enumerate(self.systems):
            v, W = vs[i], Ws[i]
            assert v.shape[0] == S and W.shape[0] == S
            if dev:
                assert v.is_contiguous() and W.is_contiguous() and v.element_size() == 4 and W.element_size() == 4
            else:
                v = np.ascontiguousarray(v, dtype=np.float32)
                W = np.ascontiguousarray(W, dtype=np.float32)
            n_v = v.numel() if dev else v.size
            n_W = W.numel() if dev else W.size
            assert n_v == S * sysm.n_atoms * 3 and n_W == S * sysm.n_atoms * 9
            keep += [v, W]
            pv[i] = _ptr(v)
            pW[i] = _ptr(W)
        if dev:
            self.systems[0]._use(*keep)   # one stream: one wait on torch's stream for all inputs
        self._check(self._lib.mhc_shc_group_push(self._h, S, pv, pW, 1 if dev else 0), "shc group push")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mhc_shc_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ModalVirial:
    """Per-atom virial, forces and HNEMD driving force of a Tersoff potential
    (mhc_virial_*): positions in, the W input of the modal-current push out.

    params: dict with the keys of mhc_tersoff_params (A, B, lambda1, lambda2,
    lambda3, m, beta, n, c, d, h, gamma, R, D).  Positions, velocities and
    outputs are float64 torch tensors on the device (W32 float32)."""

    def __init__(self, mass, box, params: dict, max_neighbors: int = 16, skin: float = 0.0, device: int = 0,
                 stream=None):
        self._lib = library()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        m = np.ascontiguousarray(mass, dtype=np.float64)
        b = np.ascontiguousarray(box, dtype=np.float64)
        assert b.shape == (3,)
        tp = TersoffParams(**{k: params[k] for k in ("A", "B", "lambda1", "lambda2", "lambda3", "beta", "n", "c", "d",
                                                      "h", "gamma", "R", "D")}, m=int(params["m"]), reserved=0)
        h = C.c_void_p()
        st = self._lib.mhc_virial_create(int(device), C.c_void_p(int(stream) if stream else 0), m.shape[0], _ptr(m),
                                         _ptr(b), C.byref(tp), int(max_neighbors), float(skin), C.byref(h))
        if st:
            raise MhcError(st, self._lib.mhc_virial_last_error(None).decode())
        self._h = h
        self._use = _StreamUse(device, int(stream) if stream else 0)
        self.n_atoms, self.max_neighbors, self.device = m.shape[0], int(max_neighbors), device

    def _check(self, st, what):
        if st:
            raise MhcError(st, f"{what}: {self._lib.mhc_virial_last_error(self._h).decode()}")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mhc_virial_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _dev(self, t, dtype_size, shape_tail):
        assert _is_torch(t) and t.is_cuda and t.is_contiguous() and t.element_size() == dtype_size
        assert t.numel() == self.n_atoms * shape_tail
        return _ptr(t)

    def neighbors(self, pos) -> int:
        """Build the lists from pos [N, 3] (float64 device tensor); returns the largest count."""
        p = self._dev(pos, 8, 3)
        self._use(pos)
        mx = C.c_int32()
        self._check(self._lib.mhc_virial_neighbors(self._h, p, C.byref(mx)), "virial neighbors")
        return mx.value

    def read_neighbors(self):
        counts = np.empty(self.n_atoms, dtype=np.int32)
        lists = np.empty((self.n_atoms, self.max_neighbors), dtype=np.int32)
        self._check(self._lib.mhc_virial_read_neighbors(self._h, _ptr(counts), _ptr(lists)), "virial read_neighbors")
        return counts, lists

    def compute(self, pos, vel=None, fe=None, want=("U", "F", "W", "W32", "Fext"), out=None):
        """One evaluation; returns {name: tensor} for the names in want (or the
        preallocated tensors given in out, e.g. a step slice of a W32 block)."""
        import torch
        N = self.n_atoms
        out = dict(out or {})
        shapes = {"U": (N,), "F": (N, 3), "W": (N, 3, 3), "W32": (N, 3, 3), "Fext": (N, 3)}
        for k in want:
            if k not in out:
                out[k] = torch.empty(shapes[k], dtype=torch.float32 if k == "W32" else torch.float64,
                                     device=pos.device)
        ptrs = {}
        for k, t in out.items():
            ptrs[k] = self._dev(t, 4 if k == "W32" else 8, {"U": 1, "F": 3, "W": 9, "W32": 9, "Fext": 3}[k])
        p = self._dev(pos, 8, 3)
        vp = self._dev(vel, 8, 3) if vel is not None else None
        f = None
        if fe is not None:
            fa = np.ascontiguousarray(fe, dtype=np.float64)
            assert fa.shape == (3,)
            f = _ptr(fa)
        self._use(*[t for t in (pos, vel) if t is not None], *out.values())
        self._check(self._lib.mhc_virial_compute(self._h, p, vp, f, ptrs.get("U"), ptrs.get("F"), ptrs.get("W"),
                                                 ptrs.get("W32"), ptrs.get("Fext")), "virial compute")
        return out

    def md(self, pos, vel, dt, n_steps, rebuild=0, v32=None, W32=None, F=None):
        """n_steps velocity-Verlet steps of dt fs on the device tensors pos and vel
        (float64 [N][3], updated in place); per step the float32 velocities and
        virials go to v32 [n_steps][N][3] and W32 [n_steps][N][3][3] (device
        tensors or None), the push's inputs for those steps; the lists are
        rebuilt every `rebuild` steps (0: never)."""
        N = self.n_atoms
        p = self._dev(pos, 8, 3)
        vp = self._dev(vel, 8, 3)
        ptr = {}
        for name, t, es, per in (("v32", v32, 4, 3 * n_steps), ("W32", W32, 4, 9 * n_steps), ("F", F, 8, 3)):
            if t is not None:
                if not (_is_torch(t) and t.is_cuda and t.is_contiguous() and t.element_size() == es
                        and t.numel() == N * per):
                    raise ValueError(f"{name} must be a contiguous device tensor of {N * per} "
                                     f"{'float32' if es == 4 else 'float64'} values")
                ptr[name] = _ptr(t)
        self._use(pos, vel, *[t for t in (v32, W32, F) if t is not None])
        self._check(self._lib.mhc_virial_md(self._h, p, vp, float(dt), int(n_steps), int(rebuild), ptr.get("v32"),
                                            ptr.get("W32"), ptr.get("F")), "virial md")

    def md_nvt(self, pos, vel, dt, n_steps, fe, temperature, tau, thermostat=(0.0, 0.0), rebuild=0, v32=None,
               W32=None, F=None):
        """As md, under a Nose-Hoover thermostat (temperature K, time tau fs) with
        the HNEMD driving force fe (1/A, 3 values; None: no drive) on every atom
        (mhc_virial_md_nvt).  thermostat: (xi, eta) at entry; returns them at the end."""
        N = self.n_atoms
        p = self._dev(pos, 8, 3)
        vp = self._dev(vel, 8, 3)
        ptr = {}
        for name, t, es, per in (("v32", v32, 4, 3 * n_steps), ("W32", W32, 4, 9 * n_steps), ("F", F, 8, 3)):
            if t is not None:
                if not (_is_torch(t) and t.is_cuda and t.is_contiguous() and t.element_size() == es
                        and t.numel() == N * per):
                    raise ValueError(f"{name} must be a contiguous device tensor of {N * per} "
                                     f"{'float32' if es == 4 else 'float64'} values")
                ptr[name] = _ptr(t)
        fe_arr = None if fe is None else np.ascontiguousarray(fe, dtype=np.float64)
        if fe_arr is not None and fe_arr.size != 3:
            raise ValueError("fe must hold 3 values")
        th = np.ascontiguousarray(thermostat, dtype=np.float64).copy()
        if th.size != 2:
            raise ValueError("thermostat must hold (xi, eta)")
        self._use(pos, vel, *[t for t in (v32, W32, F) if t is not None])
        self._check(self._lib.mhc_virial_md_nvt(self._h, p, vp, float(dt), int(n_steps), int(rebuild),
                                                None if fe_arr is None else _ptr(fe_arr), float(temperature),
                                                float(tau), _ptr(th), ptr.get("v32"), ptr.get("W32"), ptr.get("F")),
                    "virial md_nvt")
        return float(th[0]), float(th[1])

    def synchronize(self):
        self._check(self._lib.mhc_virial_synchronize(self._h), "virial synchronize")

    def set_timing(self, enable=True):
        """False / 0: off; True / 1: time every evaluation; k > 1: every k-th."""
        self._check(self._lib.mhc_virial_set_timing(self._h, int(enable)), "virial set_timing")

    def kernel_timing(self):
        """(evaluations, summed site-kernel ms, summed gather-kernel ms) since the last call."""
        n = C.c_int64()
        ms_site = C.c_double()
        ms_gather = C.c_double()
        self._check(self._lib.mhc_virial_kernel_timing(self._h, C.byref(n), C.byref(ms_site), C.byref(ms_gather)),
                    "virial kernel_timing")
        return n.value, ms_site.value, ms_gather.value
