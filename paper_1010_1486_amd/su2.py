"""Python binding of libsu2 (the C ABI in include/su2.h).

Argument marshalling only: every step of the heat bath and of the
measurements runs in the library's HIP kernels.  torch provides device memory
(caller-owned buffers passed to su2_init_ext) and the stream (torch's current
stream on the chosen device).  If libsu2.so has not been built this module
raises on first use; there is no fallback.
"""
import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsu2.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "su2.h")

SU2_OK, SU2_EINVAL, SU2_EODD, SU2_ENOMEM, SU2_EHIP, SU2_ESTATE, SU2_ERANGE = 0, -1, -2, -3, -4, -5, -6
SU2_COLD, SU2_HOT = 0, 1
SU2_KP, SU2_LEARNED, SU2_KP_OR = 0, 1, 2
SU2_MEAS_PLAQ, SU2_MEAS_POLY = 1, 2

_ERR_NAMES = {SU2_EINVAL: "SU2_EINVAL", SU2_EODD: "SU2_EODD", SU2_ENOMEM: "SU2_ENOMEM",
              SU2_EHIP: "SU2_EHIP", SU2_ESTATE: "SU2_ESTATE", SU2_ERANGE: "SU2_ERANGE"}


class SU2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

_vp = ctypes.c_void_p
_i32, _u32, _i64, _u64, _sz, _d, _int = (ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64,
                                         ctypes.c_uint64, ctypes.c_size_t, ctypes.c_double,
                                         ctypes.c_int)
_SIGS = {
    "su2_last_error": (ctypes.c_char_p, []),
    "su2_links_bytes": (_sz, [_vp]),
    "su2_scratch_bytes": (_sz, [_vp]),
    "su2_init": (_int, [_vp, _vp, _d, _u64, _int]),
    "su2_init_ext": (_int, [_vp, _vp, _d, _u64, _int, _vp, _sz, _vp, _sz, _vp]),
    "su2_init_f64": (_int, [_vp, _vp, _d, _u64, _int, _vp]),
    "su2_wilson_loops": (_int, [_vp, _int, _int, _vp]),
    "su2_is_f64": (_int, [_vp, _vp]),
    "su2_get_links_f64": (_int, [_vp, _vp]),
    "su2_set_links_f64": (_int, [_vp, _vp]),
    "su2_destroy": (_int, [_vp]),
    "su2_heatbath_sweep": (_int, [_vp, _i32, _int]),
    "su2_sweep_measure": (_int, [_vp, _i32, _int, _i32, _int, _vp]),
    "su2_reunitarize": (_int, [_vp]),
    "su2_plaquette": (_int, [_vp, _vp]),
    "su2_polyakov": (_int, [_vp, _vp, _vp]),
    "su2_get_links": (_int, [_vp, _vp]),
    "su2_set_links": (_int, [_vp, _vp]),
    "su2_get_sweep": (_int, [_vp, _vp]),
    "su2_set_sweep": (_int, [_vp, _u32]),
    "su2_set_beta": (_int, [_vp, _d]),
    "su2_set_replica": (_int, [_vp, _u32]),
    "su2_links_device": (_int, [_vp, _vp, _vp]),
    "su2_set_hb_overrelax": (_int, [_vp, _i32]),
    "su2_batch_set_hb_overrelax": (_int, [_vp, _i32]),
    "su2_set_reunit_fused": (_int, [_vp, _int]),
    "su2_batch_set_reunit_fused": (_int, [_vp, _int]),
    "su2_sweep_measure_static": (_int, [_vp, _vp, _d, _u64, _u32, _i32, _i32, _int, _vp, _vp]),
    "su2_synchronize": (_int, [_vp]),
    "su2_set_launch": (_int, [_vp, _int, _int, _int, _int, _int]),
    "su2_autotune": (_int, [_vp, ctypes.c_char_p, _int, _vp]),
    "su2_get_launch": (_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "su2_batch_get_launch": (_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "su2_capture_sweeps": (_int, [_vp, _i32, _int, _i32, _int, _vp, _i64]),
    "su2_replay_sweeps": (_int, [_vp, _i32]),
    "su2_batch_init": (_int, [_vp, _i32, _vp, _vp, _vp, _u64, _vp]),
    "su2_batch_destroy": (_int, [_vp]),
    "su2_batch_size": (_int, [_vp, _vp]),
    "su2_batch_sweep": (_int, [_vp, _i32, _int]),
    "su2_batch_sweep_measure": (_int, [_vp, _i32, _int, _i32, _int, _vp]),
    "su2_batch_capture": (_int, [_vp, _i32, _int, _i32, _int, _vp, _i64]),
    "su2_batch_replay": (_int, [_vp, _i32]),
    "su2_batch_observables": (_int, [_vp, _vp, _vp, _vp]),
    "su2_batch_get_links": (_int, [_vp, _i32, _vp]),
    "su2_batch_set_links": (_int, [_vp, _i32, _vp]),
    "su2_batch_set_launch": (_int, [_vp, _int, _int, _int, _int, _int]),
    "su2_batch_autotune": (_int, [_vp, ctypes.c_char_p, _int, _vp]),
    "su2_batch_synchronize": (_int, [_vp]),
    "su2_batch_get_accept_stats": (_int, [_vp, _vp, _vp, _int]),
    "su2_batch_set_proposal": (_int, [_vp, _vp]),
    "su2_test_philox": (_int, [_vp, _i64, _u64, _vp]),
    "su2_test_heatbath_links": (_int, [_vp, _i64, _d, _u64, _u32, _u32, _u32, _vp, _vp]),
    "su2_test_pass": (_int, [_vp, _int, _int, _int]),
    "su2_test_gauge_transform": (_int, [_vp, _u64]),
    "su2_test_stream_pass": (_int, [_vp, _int, _int, _vp]),
    "su2_test_index_map": (_int, [_vp, _int, _int, _int, _vp]),
    "su2_test_queue_plan": (_int, [_i32, _vp, _int, _i32, _i32, _i32, _u32, _int, _int, _vp]),
    "su2_test_batch_spin_limit": (_int, [_vp, _u32]),
    "su2_nn_num_params": (_int, []),
    "su2_nn_create": (_int, [_vp, _vp, _u64, _vp]),
    "su2_nn_destroy": (_int, [_vp]),
    "su2_nn_get_params": (_int, [_vp, _vp]),
    "su2_nn_set_params": (_int, [_vp, _vp]),
    "su2_nn_sample_data": (_int, [_vp, _i64, _d, _d, _u64]),
    "su2_nn_set_data": (_int, [_vp, _i64, _vp, _vp]),
    "su2_nn_get_data": (_int, [_vp, _vp, _vp, _vp]),
    "su2_nn_loss_grad": (_int, [_vp, _i64, _i32, _vp, _vp]),
    "su2_nn_train": (_int, [_vp, _i32, _i32, _d, _vp]),
    "su2_nn_train_cosine": (_int, [_vp, _i32, _i32, _d, _d, _vp]),
    "su2_nn_build_table": (_int, [_vp]),
    "su2_nn_get_table": (_int, [_vp, _vp]),
    "su2_set_proposal": (_int, [_vp, _vp]),
    "su2_get_accept_stats": (_int, [_vp, _vp, _vp, _int]),
    "su2_test_learned_links": (_int, [_vp, _vp, _vp, _i64, _d, _u64, _u32, _u32, _u32, _d,
                                      _vp, _vp]),
    "su2_set_overrelax": (_int, [_vp, _d]),
    "su2_batch_set_overrelax": (_int, [_vp, _d]),
}


def lib():
    """Load libsu2.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no CPU fallback)")
        # torch brings its own HIP runtime (same soname).  Loading it first
        # makes libsu2 bind to that runtime, so tensors, streams and kernels
        # share one runtime; loading libsu2 first would put a second HIP
        # runtime into the process and torch's device initialisation fails.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


def header_functions():
    """Names of the functions declared in include/su2.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(su2_[a-z0-9_]+)\s*\(", text)))


def _check(rc):
    if rc != SU2_OK:
        raise SU2Error(rc, lib().su2_last_error().decode())
    return rc


def _p(a):
    return a.ctypes.data_as(_vp)


def _dims(dims):
    d = np.ascontiguousarray(dims, dtype=np.int32)
    if d.shape != (4,):
        raise ValueError("dims must have 4 entries")
    return d


# ---------------------------------------------------------------- raw names
def su2_links_bytes(dims):
    return lib().su2_links_bytes(_p(_dims(dims)))


def su2_scratch_bytes(dims):
    return lib().su2_scratch_bytes(_p(_dims(dims)))


def su2_init(dims, beta, seed, start):
    """Context with library-owned memory and stream; returns an opaque handle."""
    h = _vp()
    _check(lib().su2_init(ctypes.byref(h), _p(_dims(dims)), float(beta), int(seed), int(start)))
    return h


def su2_init_ext(dims, beta, seed, start, links_ptr, links_bytes, scratch_ptr, scratch_bytes,
                 stream):
    h = _vp()
    _check(lib().su2_init_ext(ctypes.byref(h), _p(_dims(dims)), float(beta), int(seed),
                              int(start), _vp(links_ptr), links_bytes, _vp(scratch_ptr),
                              scratch_bytes, _vp(stream)))
    return h


def su2_destroy(h):
    _check(lib().su2_destroy(h))


def su2_heatbath_sweep(h, nsweeps, mode=SU2_KP):
    _check(lib().su2_heatbath_sweep(h, int(nsweeps), int(mode)))


def su2_sweep_measure(h, nsweeps, mode, reunit_every, meas, dev_history_ptr):
    _check(lib().su2_sweep_measure(h, int(nsweeps), int(mode), int(reunit_every), int(meas),
                                   _vp(dev_history_ptr)))


def su2_reunitarize(h):
    _check(lib().su2_reunitarize(h))


def su2_plaquette(h):
    v = ctypes.c_double()
    _check(lib().su2_plaquette(h, ctypes.byref(v)))
    return v.value


def su2_polyakov(h):
    s, a = ctypes.c_double(), ctypes.c_double()
    _check(lib().su2_polyakov(h, ctypes.byref(s), ctypes.byref(a)))
    return s.value, a.value


def su2_get_links(h, volume):
    out = np.empty((volume, 4, 4), dtype=np.float32)
    _check(lib().su2_get_links(h, _p(out)))
    return out


def su2_set_links(h, links):
    a = np.ascontiguousarray(links, dtype=np.float32)
    _check(lib().su2_set_links(h, _p(a)))


def su2_get_sweep(h):
    v = ctypes.c_uint32()
    _check(lib().su2_get_sweep(h, ctypes.byref(v)))
    return v.value


def su2_set_sweep(h, sweep):
    _check(lib().su2_set_sweep(h, int(sweep)))


def su2_set_beta(h, beta):
    _check(lib().su2_set_beta(h, float(beta)))


def su2_set_replica(h, replica):
    _check(lib().su2_set_replica(h, int(replica)))


def su2_synchronize(h):
    _check(lib().su2_synchronize(h))


def su2_set_launch(h, block, flags, tile_z=0, tile_t=0, grid_cap=0):
    _check(lib().su2_set_launch(h, int(block), int(flags), int(tile_z), int(tile_t),
                                int(grid_cap)))


def su2_get_launch(h, batch=False):
    v = [ctypes.c_int() for _ in range(5)]
    fn = lib().su2_batch_get_launch if batch else lib().su2_get_launch
    _check(fn(h, *[ctypes.byref(x) for x in v]))
    return dict(zip(("block", "flags", "tile_z", "tile_t", "grid_cap"), (x.value for x in v)))


def su2_autotune(h, cache_path=None, mode=SU2_KP):
    us = ctypes.c_double()
    _check(lib().su2_autotune(h, None if cache_path is None else cache_path.encode(), int(mode),
                              ctypes.byref(us)))
    return us.value


def su2_capture_sweeps(h, nsweeps, mode=SU2_KP, reunit_every=0, meas=0, dev_history_ptr=None,
                       history_rows=0):
    _check(lib().su2_capture_sweeps(h, int(nsweeps), int(mode), int(reunit_every), int(meas),
                                    _vp(dev_history_ptr), int(history_rows)))


def su2_replay_sweeps(h, count):
    _check(lib().su2_replay_sweeps(h, int(count)))


def su2_sweep_measure_static(links, dims, beta, seed, sweep0, nsweeps, reunit_every=0,
                             meas=SU2_MEAS_PLAQ, hist=None, stream=None):
    """Allocation-free sweeps on caller-owned device links (torch uint8 or
    float32 tensor of su2_links_bytes(dims) bytes in the library's device
    layout): returns the FP64 (nsweeps, 3) history tensor.  hist, if given,
    is used instead of a new tensor (nothing is then allocated)."""
    import torch
    d = np.ascontiguousarray(dims, np.int32)
    assert links.is_cuda and links.numel() * links.element_size() >= su2_links_bytes(dims)
    if hist is None:
        hist = torch.zeros((max(int(nsweeps), 1), 3), dtype=torch.float64, device=links.device)
    assert hist.dtype == torch.float64 and hist.is_contiguous() and hist.numel() >= 3 * nsweeps
    if stream is None:
        stream = torch.cuda.current_stream(links.device)
    with torch.cuda.device(links.device):
        _check(lib().su2_sweep_measure_static(_vp(links.data_ptr()), _p(d), float(beta),
                                              int(seed), int(sweep0), int(nsweeps),
                                              int(reunit_every), int(meas),
                                              _vp(hist.data_ptr()), _vp(stream.cuda_stream)))
    return hist


def su2_links_device(h):
    p, s = _vp(), _vp()
    _check(lib().su2_links_device(h, ctypes.byref(p), ctypes.byref(s)))
    return p.value, s.value


def su2_test_philox(ctr, seed):
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(c)
    _check(lib().su2_test_philox(_p(c), c.shape[0], int(seed), _p(out)))
    return out


def su2_test_heatbath_links(V, beta, seed, sweep, mu, replica=0, want_trials=False):
    v = np.ascontiguousarray(V, dtype=np.float32).reshape(-1, 4)
    out = np.empty_like(v)
    nt = np.empty(v.shape[0], dtype=np.int32) if want_trials else None
    _check(lib().su2_test_heatbath_links(_p(v), v.shape[0], float(beta), int(seed), int(sweep),
                                         int(mu), int(replica), _p(out),
                                         _p(nt) if nt is not None else None))
    return (out, nt) if want_trials else out


def su2_test_pass(h, mu, parity, mode=SU2_KP):
    _check(lib().su2_test_pass(h, int(mu), int(parity), int(mode)))


def su2_test_index_map(dims, parity, tile_z=0, tile_t=0):
    d = _dims(dims)
    vh = int(np.prod(d.astype(np.int64))) // 2
    out = np.empty((vh, 9), dtype=np.uint32)
    _check(lib().su2_test_index_map(_p(d), int(tile_z), int(tile_t), int(parity), _p(out)))
    return out


def su2_test_queue_plan(dims, block, nsweeps, reunit_every=0, first_sweep=0, meas=0,
                        rows=False, queues=8):
    """Host-side check of the work-queue schedule; returns the items run."""
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32).reshape(-1, 4))
    items = ctypes.c_int64()
    _check(lib().su2_test_queue_plan(len(d), _p(d), int(block), int(queues), int(nsweeps),
                                     int(reunit_every), int(first_sweep), int(meas), int(rows),
                                     ctypes.byref(items)))
    return items.value


def su2_test_stream_pass(h, mu, parity, out_ptr):
    _check(lib().su2_test_stream_pass(h, int(mu), int(parity), _vp(out_ptr)))


def su2_test_gauge_transform(h, seed):
    _check(lib().su2_test_gauge_transform(h, int(seed)))


NN_NPARAM, NN_ROWS, NN_ROW = 2671, 64, 48


def su2_nn_create(params=None, seed=0, stream=None):
    h = _vp()
    pa = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().su2_nn_create(ctypes.byref(h), None if pa is None else _p(pa), int(seed),
                               _vp(stream)))
    return h


def su2_nn_destroy(h):
    _check(lib().su2_nn_destroy(h))


def su2_nn_get_params(h):
    out = np.empty(NN_NPARAM, dtype=np.float32)
    _check(lib().su2_nn_get_params(h, _p(out)))
    return out


def su2_nn_set_params(h, params):
    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().su2_nn_set_params(h, _p(a)))


def su2_nn_sample_data(h, n, alpha_lo, alpha_hi, seed):
    _check(lib().su2_nn_sample_data(h, int(n), float(alpha_lo), float(alpha_hi), int(seed)))


def su2_nn_set_data(h, alpha, a0):
    a = np.ascontiguousarray(alpha, dtype=np.float32)
    x = np.ascontiguousarray(a0, dtype=np.float32)
    _check(lib().su2_nn_set_data(h, a.size, _p(a), _p(x)))


def su2_nn_get_data(h):
    n = ctypes.c_int64()
    _check(lib().su2_nn_get_data(h, ctypes.byref(n), None, None))
    a = np.empty(n.value, dtype=np.float32)
    x = np.empty(n.value, dtype=np.float32)
    _check(lib().su2_nn_get_data(h, ctypes.byref(n), _p(a), _p(x)))
    return a, x


def su2_nn_loss_grad(h, offset, batch):
    loss = ctypes.c_double()
    g = np.empty(NN_NPARAM, dtype=np.float32)
    _check(lib().su2_nn_loss_grad(h, int(offset), int(batch), ctypes.byref(loss), _p(g)))
    return loss.value, g


def su2_nn_train(h, steps, batch, lr):
    hist = np.empty(max(int(steps), 1), dtype=np.float64)
    _check(lib().su2_nn_train(h, int(steps), int(batch), float(lr), _p(hist)))
    return hist[:steps]


def su2_nn_train_cosine(h, steps, batch, lr0, lr1):
    hist = np.empty(max(int(steps), 1), dtype=np.float64)
    _check(lib().su2_nn_train_cosine(h, int(steps), int(batch), float(lr0), float(lr1), _p(hist)))
    return hist[:steps]


def su2_nn_build_table(h):
    _check(lib().su2_nn_build_table(h))


def su2_nn_get_table(h):
    out = np.empty((NN_ROWS, NN_ROW), dtype=np.float32)
    _check(lib().su2_nn_get_table(h, _p(out)))
    return out


def su2_set_proposal(ctx, nn):
    _check(lib().su2_set_proposal(ctx, nn))


def su2_get_accept_stats(ctx, reset=False):
    p, a = ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().su2_get_accept_stats(ctx, ctypes.byref(p), ctypes.byref(a), int(reset)))
    return p.value, a.value


def su2_test_learned_links(nn, V, Uold, beta, seed, sweep, mu, replica=0, or_width=-1.0):
    v = np.ascontiguousarray(V, dtype=np.float32).reshape(-1, 4)
    u = np.ascontiguousarray(Uold, dtype=np.float32).reshape(-1, 4)
    out = np.empty_like(v)
    acc = np.empty(v.shape[0], dtype=np.int32)
    _check(lib().su2_test_learned_links(nn, _p(v), _p(u), v.shape[0], float(beta), int(seed),
                                        int(sweep), int(mu), int(replica), float(or_width),
                                        _p(out), _p(acc)))
    return out, acc


class NN:
    """Learned-proposal network held by the library (su2_nn)."""

    def __init__(self, params=None, seed=0, stream=None):
        self.h = su2_nn_create(params, seed, stream)

    def close(self):
        if getattr(self, "h", None) is not None:
            su2_nn_destroy(self.h)
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

    params = property(lambda self: su2_nn_get_params(self.h))

    def set_params(self, p):
        su2_nn_set_params(self.h, p)

    def sample_data(self, n, alpha_lo=0.5, alpha_hi=30.0, seed=0):
        su2_nn_sample_data(self.h, n, alpha_lo, alpha_hi, seed)

    def set_data(self, alpha, a0):
        su2_nn_set_data(self.h, alpha, a0)

    def data(self):
        return su2_nn_get_data(self.h)

    def loss_grad(self, offset, batch):
        return su2_nn_loss_grad(self.h, offset, batch)

    def train(self, steps, batch, lr=1e-3, lr_end=None):
        """Adam steps; with lr_end, a cosine schedule from lr down to lr_end."""
        if lr_end is None:
            return su2_nn_train(self.h, steps, batch, lr)
        return su2_nn_train_cosine(self.h, steps, batch, lr, lr_end)

    def build_table(self):
        su2_nn_build_table(self.h)

    def table(self):
        return su2_nn_get_table(self.h)

    def test_links(self, V, Uold, beta, seed, sweep, mu, replica=0, or_width=-1.0):
        return su2_test_learned_links(self.h, V, Uold, beta, seed, sweep, mu, replica, or_width)


# ------------------------------------------------------------ convenience
class Lattice:
    """A lattice whose links and scratch are torch tensors on a GPU, run on
    torch's current stream of that device (su2_init_ext).  The context is
    created with `device` current; later calls expect it to be the current
    device (as on a one-GPU machine, or inside torch.cuda.device(device))."""

    def __init__(self, dims, beta, seed, start=SU2_COLD, device="cuda:0"):
        import torch
        self.torch = torch
        self.dims = [int(d) for d in dims]
        self.volume = int(np.prod(self.dims))
        self.device = torch.device(device)
        lb, sb = su2_links_bytes(self.dims), su2_scratch_bytes(self.dims)
        if lb == 0:
            raise SU2Error(SU2_EODD, f"invalid extents {self.dims}")
        self.links_t = torch.empty(lb, dtype=torch.uint8, device=self.device)
        self.scratch_t = torch.empty(sb, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):  # the context belongs to this device
            self.h = su2_init_ext(self.dims, beta, seed, start, self.links_t.data_ptr(), lb,
                                  self.scratch_t.data_ptr(), sb, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "h", None) is not None:
            su2_destroy(self.h)
            self.h = None
        self._proposal = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def heatbath_sweep(self, n, mode=SU2_KP):
        su2_heatbath_sweep(self.h, n, mode)

    def sweep_measure(self, n, mode=SU2_KP, reunit_every=0, meas=SU2_MEAS_PLAQ, hist=None):
        torch = self.torch
        if hist is None:
            hist = torch.zeros((max(n, 1), 3), dtype=torch.float64, device=self.device)
        su2_sweep_measure(self.h, n, mode, reunit_every, meas, hist.data_ptr())
        return hist

    def reunitarize(self):
        su2_reunitarize(self.h)

    def plaquette(self):
        return su2_plaquette(self.h)

    def polyakov(self):
        return su2_polyakov(self.h)

    def get_links(self):
        return su2_get_links(self.h, self.volume)

    def set_links(self, links):
        su2_set_links(self.h, links)

    @property
    def sweep(self):
        return su2_get_sweep(self.h)

    def set_sweep(self, s):
        su2_set_sweep(self.h, s)

    def set_beta(self, b):
        su2_set_beta(self.h, b)

    def set_replica(self, r):
        su2_set_replica(self.h, r)

    def set_launch(self, block, flags=1, tile_z=0, tile_t=0, grid_cap=0):
        """flags: bit 0 XCD remap, bit 1 disables the alternating pass order, bit 2
        disables the whole-sweep kernel of small lattices."""
        su2_set_launch(self.h, block, flags, tile_z, tile_t, grid_cap)

    def autotune(self, cache_path=None, mode=SU2_KP):
        return su2_autotune(self.h, cache_path, mode)

    def launch(self):
        return su2_get_launch(self.h)

    def capture(self, nsweeps, mode=SU2_KP, reunit_every=0, meas=0, hist=None):
        """hist: FP64 device tensor of shape (rows, 3); the k-th replay writes rows
        k*nsweeps.. and replays past its last row are refused."""
        rows = 0
        if hist is not None:
            assert hist.dtype == self.torch.float64 and hist.is_contiguous()
            rows = hist.numel() // 3
        su2_capture_sweeps(self.h, nsweeps, mode, reunit_every, meas,
                           None if hist is None else hist.data_ptr(), rows)

    def replay(self, count):
        su2_replay_sweeps(self.h, count)

    def synchronize(self):
        su2_synchronize(self.h)

    def test_pass(self, mu, parity, mode=SU2_KP):
        su2_test_pass(self.h, mu, parity, mode)

    def test_stream_pass(self, mu, parity, out):
        """out: float32 device tensor of at least 2 V elements."""
        assert out.dtype == self.torch.float32 and out.numel() >= 2 * int(np.prod(self.dims))
        su2_test_stream_pass(self.h, mu, parity, out.data_ptr())

    def test_gauge_transform(self, seed):
        su2_test_gauge_transform(self.h, seed)

    def set_proposal(self, nn):
        """Attach nn (None detaches); the lattice keeps nn alive while attached."""
        su2_set_proposal(self.h, None if nn is None else nn.h)
        self._proposal = nn

    def wilson_loops(self, rmax, tmax):
        """W(R, T) for R = 1..rmax, T = 1..tmax as an (rmax, tmax) array."""
        out = np.zeros(rmax * tmax)
        _check(lib().su2_wilson_loops(self.h, int(rmax), int(tmax), _p(out)))
        return out.reshape(rmax, tmax)

    def set_overrelax(self, width):
        """width < 0: independence proposal; 0..1: over-relaxed learned proposal."""
        _check(lib().su2_set_overrelax(self.h, float(width)))

    def set_hb_overrelax(self, n_or):
        """Over-relaxation sweeps after each heat-bath sweep in SU2_KP_OR mode."""
        _check(lib().su2_set_hb_overrelax(self.h, int(n_or)))

    def set_reunit_fused(self, on=True):
        """Reunitarise inside the last pass stage of a reunitarisation sweep."""
        _check(lib().su2_set_reunit_fused(self.h, int(on)))

    def accept_stats(self, reset=False):
        return su2_get_accept_stats(self.h, reset)


class Lattice64(Lattice):
    """A lattice with FP64 links (library-owned device memory) run on torch's
    current stream of the device (su2_init_f64).  get_links returns float64."""

    def __init__(self, dims, beta, seed, start=SU2_COLD, device="cuda:0"):
        import torch
        self.torch = torch
        self.dims = [int(d) for d in dims]
        self.volume = int(np.prod(self.dims))
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        h = _vp()
        with torch.cuda.device(self.device):  # the context belongs to this device
            _check(lib().su2_init_f64(ctypes.byref(h), _p(_dims(self.dims)), float(beta),
                                      int(seed), int(start), _vp(self.stream.cuda_stream)))
        self.h = h

    def get_links(self):
        out = np.empty((self.volume, 4, 4), dtype=np.float64)
        _check(lib().su2_get_links_f64(self.h, _p(out)))
        return out

    def set_links(self, links):
        a = np.ascontiguousarray(links, dtype=np.float64).reshape(self.volume, 4, 4)
        _check(lib().su2_set_links_f64(self.h, _p(a)))


class Batch:
    """n replicas (su2_batch) on torch's current stream of the device."""

    def __init__(self, dims, betas, starts, seed, device="cuda:0"):
        import torch  # noqa: F811
        self.torch = torch
        self.device = torch.device(device)
        d = np.ascontiguousarray(dims, dtype=np.int32).reshape(-1, 4)
        self.n = d.shape[0]
        self.dims = [list(map(int, x)) for x in d]
        b = np.ascontiguousarray(np.broadcast_to(np.asarray(betas, np.float64), (self.n,)))
        st = np.ascontiguousarray(np.broadcast_to(np.asarray(starts, np.int32), (self.n,)))
        self.betas = b.copy()
        self.stream = torch.cuda.current_stream(self.device)
        h = _vp()
        with torch.cuda.device(self.device):  # the batch belongs to this device
            _check(lib().su2_batch_init(ctypes.byref(h), self.n, _p(d), _p(b), _p(st),
                                        int(seed), _vp(self.stream.cuda_stream)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None:
            _check(lib().su2_batch_destroy(self.h))
            self.h = None
        self._proposal = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def sweep(self, n, mode=SU2_KP):
        _check(lib().su2_batch_sweep(self.h, int(n), int(mode)))

    def _hist(self, rows, hist):
        if hist is None:
            hist = self.torch.zeros((max(rows, 1), self.n, 3), dtype=self.torch.float64,
                                    device=self.device)
        return hist

    def sweep_measure(self, n, mode=SU2_KP, reunit_every=0, meas=SU2_MEAS_PLAQ, hist=None):
        hist = self._hist(n, hist)
        _check(lib().su2_batch_sweep_measure(self.h, int(n), int(mode), int(reunit_every),
                                             int(meas), _vp(hist.data_ptr())))
        return hist

    def capture(self, n, mode=SU2_KP, reunit_every=0, meas=0, hist=None):
        """hist: FP64 device tensor of shape (rows, replicas, 3); the k-th replay
        writes rows k*n.. and replays past its last row are refused."""
        rows = 0
        if hist is not None:
            import torch
            assert hist.dtype == torch.float64 and hist.is_contiguous()
            rows = hist.numel() // (3 * self.n)
        _check(lib().su2_batch_capture(self.h, int(n), int(mode), int(reunit_every), int(meas),
                                       None if hist is None else _vp(hist.data_ptr()),
                                       int(rows)))

    def replay(self, count):
        _check(lib().su2_batch_replay(self.h, int(count)))

    def observables(self):
        p, s, a = np.empty(self.n), np.empty(self.n), np.empty(self.n)
        _check(lib().su2_batch_observables(self.h, _p(p), _p(s), _p(a)))
        return p, s, a

    def get_links(self, r):
        V = int(np.prod(self.dims[r]))
        out = np.empty((V, 4, 4), dtype=np.float32)
        _check(lib().su2_batch_get_links(self.h, int(r), _p(out)))
        return out

    def set_links(self, r, links):
        a = np.ascontiguousarray(links, dtype=np.float32)
        _check(lib().su2_batch_set_links(self.h, int(r), _p(a)))

    def set_launch(self, block, flags=1, tile_z=0, tile_t=0, grid_cap=0):
        _check(lib().su2_batch_set_launch(self.h, int(block), int(flags), int(tile_z),
                                          int(tile_t), int(grid_cap)))

    def launch(self):
        return su2_get_launch(self.h, batch=True)

    def test_spin_limit(self, polls):
        _check(lib().su2_test_batch_spin_limit(self.h, int(polls)))

    def autotune(self, cache_path=None, mode=SU2_KP):
        us = ctypes.c_double()
        _check(lib().su2_batch_autotune(self.h, None if cache_path is None else
                                        cache_path.encode(), int(mode), ctypes.byref(us)))
        return us.value

    def synchronize(self):
        _check(lib().su2_batch_synchronize(self.h))

    def set_proposal(self, nn):
        """Attach nn (None detaches); the batch keeps nn alive while attached."""
        _check(lib().su2_batch_set_proposal(self.h, None if nn is None else nn.h))
        self._proposal = nn

    def set_overrelax(self, width):
        """width < 0: independence proposal; 0..1: over-relaxed learned proposal."""
        _check(lib().su2_batch_set_overrelax(self.h, float(width)))

    def set_hb_overrelax(self, n_or):
        """Over-relaxation sweeps after each heat-bath sweep in SU2_KP_OR mode."""
        _check(lib().su2_batch_set_hb_overrelax(self.h, int(n_or)))

    def set_reunit_fused(self, on=True):
        """Reunitarise inside the last pass stage of a reunitarisation sweep."""
        _check(lib().su2_batch_set_reunit_fused(self.h, int(on)))

    def accept_stats(self, reset=False):
        p = np.zeros(self.n, dtype=np.uint64)
        a = np.zeros(self.n, dtype=np.uint64)
        _check(lib().su2_batch_get_accept_stats(self.h, _p(p), _p(a), int(reset)))
        return p, a
