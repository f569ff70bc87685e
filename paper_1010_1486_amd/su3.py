"""Python binding of the SU(3) heat bath of libsu2 (the C ABI in include/su3.h).

Argument marshalling only: the Cabibbo-Marinari updates and the measurements
run in the library's HIP kernels, on torch's current stream of the chosen
device.  There is no fallback: the calls raise if libsu2.so is missing.
"""
import ctypes
import os
import re

import numpy as np

from . import su2 as _su2
from .su2 import SU2_COLD, SU2_HOT, SU2Error, lib  # noqa: F401

HEADER3 = os.path.join(os.path.dirname(_su2.HERE), "include", "su3.h")

_vp = ctypes.c_void_p
_i32, _u32, _u64, _sz, _d, _int = (ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64,
                                   ctypes.c_size_t, ctypes.c_double, ctypes.c_int)
_SIGS3 = {
    "su3_links_bytes": (_sz, [_vp]),
    "su3_init": (_int, [_vp, _vp, _d, _u64, _int, _vp]),
    "su3_destroy": (_int, [_vp]),
    "su3_heatbath_sweep": (_int, [_vp, _i32, _i32, _vp]),
    "su3_reunitarize": (_int, [_vp]),
    "su3_plaquette": (_int, [_vp, _vp]),
    "su3_polyakov": (_int, [_vp, _vp]),
    "su3_get_links": (_int, [_vp, _vp]),
    "su3_set_links": (_int, [_vp, _vp]),
    "su3_get_sweep": (_int, [_vp, _vp]),
    "su3_set_sweep": (_int, [_vp, _u32]),
    "su3_set_beta": (_int, [_vp, _d]),
    "su3_set_launch": (_int, [_vp, _int, _int, _int, _int, _int]),
    "su3_links_device": (_int, [_vp, _vp, _vp]),
    "su3_synchronize": (_int, [_vp]),
    "su3_test_pass": (_int, [_vp, _int, _int]),
    "su3_test_or_pass": (_int, [_vp, _int, _int]),
    "su3_overrelax": (_int, [_vp, _i32]),
    "su3_test_read_links": (_int, [_vp, ctypes.c_int64, _vp, _int, _vp]),
    "su3_capture_sweeps": (_int, [_vp, _i32, _i32, _int, _vp, ctypes.c_int64]),
    "su3_replay_sweeps": (_int, [_vp, _i32]),
    "su3_set_replica": (_int, [_vp, _u32]),
    "su3_batch_init": (_int, [_vp, _i32, _vp, _vp, _u64, _int, _vp]),
    "su3_batch_destroy": (_int, [_vp]),
    "su3_batch_size": (_int, [_vp, _vp]),
    "su3_batch_heatbath_sweep": (_int, [_vp, _i32, _i32, _vp]),
    "su3_batch_overrelax": (_int, [_vp, _i32]),
    "su3_batch_reunitarize": (_int, [_vp]),
    "su3_batch_plaquette": (_int, [_vp, _vp]),
    "su3_batch_polyakov": (_int, [_vp, _vp]),
    "su3_batch_get_links": (_int, [_vp, _i32, _vp]),
    "su3_batch_set_links": (_int, [_vp, _i32, _vp]),
    "su3_batch_get_sweep": (_int, [_vp, _vp]),
    "su3_batch_set_sweep": (_int, [_vp, _u32]),
    "su3_batch_set_launch": (_int, [_vp, _int, _int, _int, _int, _int]),
    "su3_batch_synchronize": (_int, [_vp]),
}
_bound = False


def lib3():
    """libsu2.so with the SU(3) signatures set (raises if it has not been built)."""
    global _bound
    l = lib()
    if not _bound:
        for name, (res, args) in _SIGS3.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return l


def header_functions3():
    """Names of the functions declared in include/su3.h."""
    with open(HEADER3) as f:
        text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
    return sorted(set(re.findall(r"\b(su3_[a-z0-9_]+)\s*\(", text)))


def _check(rc):
    return _su2._check(rc)


def _p(a):
    return a.ctypes.data_as(_vp)


def su3_links_bytes(dims):
    return lib3().su3_links_bytes(_p(_su2._dims(dims)))


class Lattice3:
    """An SU(3) lattice (library-owned device memory) on torch's current stream
    of the device.  Links are exchanged as complex128 arrays (V, 4, 3, 3).  The
    lattice is created on `device`; later calls expect it to be the current
    device (as on a one-GPU machine, or inside torch.cuda.device(device))."""

    def __init__(self, dims, beta, seed, start=SU2_COLD, device="cuda:0"):
        import torch
        self.dims = [int(d) for d in dims]
        self.volume = int(np.prod(self.dims))
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        h = _vp()
        with torch.cuda.device(self.device):  # the context belongs to this device
            _check(lib3().su3_init(ctypes.byref(h), _p(_su2._dims(self.dims)), float(beta),
                                   int(seed), int(start), _vp(self.stream.cuda_stream)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None:
            lib3().su3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def heatbath_sweep(self, n, reunit_every=0, history=False):
        """n sweeps; with history, returns the plaquette after each one."""
        hist = np.zeros(max(int(n), 1)) if history else None
        _check(lib3().su3_heatbath_sweep(self.h, int(n), int(reunit_every),
                                         None if hist is None else _p(hist)))
        return hist[:n] if history else None

    def capture(self, n, reunit_every=0, hist=None):
        """Record n heat-bath sweeps as a graph (su3_capture_sweeps); hist: FP64
        device tensor of plaquette rows (None: no measurement).  The k-th replay
        writes rows k*n.. and replays past its last row are refused."""
        rows = 0
        if hist is not None:
            import torch
            assert hist.dtype == torch.float64 and hist.is_contiguous()
            rows = hist.numel()
        _check(lib3().su3_capture_sweeps(self.h, int(n), int(reunit_every),
                                         0 if hist is None else 1,
                                         None if hist is None else _vp(hist.data_ptr()),
                                         int(rows)))

    def replay(self, count):
        _check(lib3().su3_replay_sweeps(self.h, int(count)))

    def overrelax(self, n):
        """n microcanonical over-relaxation sweeps (the action is unchanged)."""
        _check(lib3().su3_overrelax(self.h, int(n)))

    def reunitarize(self):
        _check(lib3().su3_reunitarize(self.h))

    def plaquette(self):
        out = ctypes.c_double()
        _check(lib3().su3_plaquette(self.h, ctypes.byref(out)))
        return out.value

    def polyakov(self):
        """(Re, Im) of the mean of Tr L / 3 and the mean of |Tr L / 3|."""
        out = np.zeros(3)
        _check(lib3().su3_polyakov(self.h, _p(out)))
        return float(out[0]), float(out[1]), float(out[2])

    def get_links(self):
        out = np.empty((self.volume, 4, 3, 3), dtype=np.complex128)
        _check(lib3().su3_get_links(self.h, _p(out)))
        return out

    def set_links(self, links):
        a = np.ascontiguousarray(links, dtype=np.complex128).reshape(self.volume, 4, 3, 3)
        _check(lib3().su3_set_links(self.h, _p(a)))

    @property
    def sweep(self):
        out = ctypes.c_uint32()
        _check(lib3().su3_get_sweep(self.h, ctypes.byref(out)))
        return out.value

    def set_sweep(self, s):
        _check(lib3().su3_set_sweep(self.h, int(s)))

    def set_beta(self, b):
        _check(lib3().su3_set_beta(self.h, float(b)))

    def set_replica(self, r):
        _check(lib3().su3_set_replica(self.h, int(r)))

    def set_launch(self, block=256, remap=1, snake=1, tile_z=0, tile_t=0):
        _check(lib3().su3_set_launch(self.h, int(block), int(remap), int(snake), int(tile_z),
                                     int(tile_t)))

    def synchronize(self):
        _check(lib3().su3_synchronize(self.h))

    def test_pass(self, mu, parity):
        _check(lib3().su3_test_pass(self.h, int(mu), int(parity)))

    def test_read_links(self, sites, mu):
        """U_mu at the given sites as complex128 (n, 3, 3), without the whole field."""
        s = np.ascontiguousarray(sites, dtype=np.int64)
        out = np.empty((s.size, 3, 3), dtype=np.complex128)
        _check(lib3().su3_test_read_links(self.h, s.size, _p(s), int(mu), _p(out)))
        return out

    def test_or_pass(self, mu, parity):
        _check(lib3().su3_test_or_pass(self.h, int(mu), int(parity)))


class Batch3:
    """n SU(3) replicas of one lattice size (su3_batch), coupling betas[r] and
    Philox replica id r, on torch's current stream of the device; every pass
    is one launch for all replicas."""

    def __init__(self, dims, betas, seed, start=SU2_COLD, device="cuda:0"):
        import torch
        self.dims = [int(d) for d in dims]
        self.volume = int(np.prod(self.dims))
        b = np.ascontiguousarray(betas, dtype=np.float64).ravel()
        self.n = int(b.size)
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        h = _vp()
        with torch.cuda.device(self.device):
            _check(lib3().su3_batch_init(ctypes.byref(h), self.n, _p(_su2._dims(self.dims)),
                                         _p(b), int(seed), int(start),
                                         _vp(self.stream.cuda_stream)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None:
            lib3().su3_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def heatbath_sweep(self, n, reunit_every=0, history=False):
        """n sweeps of every replica; with history, the plaquettes (n, replicas)."""
        hist = np.zeros((max(int(n), 1), self.n)) if history else None
        _check(lib3().su3_batch_heatbath_sweep(self.h, int(n), int(reunit_every),
                                               None if hist is None else _p(hist)))
        return hist[:n] if history else None

    def overrelax(self, n):
        _check(lib3().su3_batch_overrelax(self.h, int(n)))

    def reunitarize(self):
        _check(lib3().su3_batch_reunitarize(self.h))

    def plaquette(self):
        out = np.zeros(self.n)
        _check(lib3().su3_batch_plaquette(self.h, _p(out)))
        return out

    def polyakov(self):
        """(replicas, 3): Re and Im of the mean of Tr L / 3, mean of |Tr L / 3|."""
        out = np.zeros((self.n, 3))
        _check(lib3().su3_batch_polyakov(self.h, _p(out)))
        return out

    def get_links(self, r):
        out = np.empty((self.volume, 4, 3, 3), dtype=np.complex128)
        _check(lib3().su3_batch_get_links(self.h, int(r), _p(out)))
        return out

    def set_links(self, r, links):
        a = np.ascontiguousarray(links, dtype=np.complex128).reshape(self.volume, 4, 3, 3)
        _check(lib3().su3_batch_set_links(self.h, int(r), _p(a)))

    @property
    def sweep(self):
        out = ctypes.c_uint32()
        _check(lib3().su3_batch_get_sweep(self.h, ctypes.byref(out)))
        return out.value

    def set_sweep(self, s):
        _check(lib3().su3_batch_set_sweep(self.h, int(s)))

    def set_launch(self, block=256, remap=1, snake=1, tile_z=0, tile_t=0):
        _check(lib3().su3_batch_set_launch(self.h, int(block), int(remap), int(snake),
                                           int(tile_z), int(tile_t)))

    def synchronize(self):
        _check(lib3().su3_batch_synchronize(self.h))
