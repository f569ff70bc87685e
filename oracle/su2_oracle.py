"""ctypes wrapper over the FP64 CPU oracle (oracle/su2_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  It shares no code with the GPU library.

Link arrays are float64 numpy arrays of shape (V, 4, 4) = [site][mu][component]
with site s = x + Nx*(y + Ny*(z + Nz*t)); the same canonical order the GPU
library uses for its host exchange format.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIB
    if _build.stale():
        _build.build()
    lib = ctypes.CDLL(path)
    c_u64, c_u32, c_i64, c_int, c_d = (ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64,
                                       ctypes.c_int, ctypes.c_double)
    vp = ctypes.c_void_p
    sig = {
        "orc_philox4x32_10": (None, [_u32p, _u32p, _u32p]),
        "orc_philox_batch": (None, [c_i64, _u32p, c_u64, _u32p]),
        "orc_uniform": (c_d, [c_u32]),
        "orc_uniform18": (c_d, [c_u32]),
        "orc_qmul_batch": (None, [c_i64, _f64p, _f64p, _f64p]),
        "orc_check_dims": (c_int, [_i32p]),
        "orc_volume": (c_i64, [_i32p]),
        "orc_parity": (c_int, [_i32p, c_i64]),
        "orc_shift": (c_i64, [_i32p, c_i64, c_int, c_int]),
        "orc_staple": (None, [_i32p, _f64p, c_i64, c_int, _f64p]),
        "orc_hot_link": (None, [c_i64, c_int, c_u64, c_u32, _f64p]),
        "orc_hot_staple": (None, [_i32p, c_i64, c_int, c_u64, c_u32, _f64p]),
        "orc_sample_delta_batch": (None, [c_i64, _f64p, c_u64, _u32p, c_u32, c_u32, c_u32,
                                          _f64p, vp, vp]),
        "orc_heatbath_link": (None, [_f64p, c_d, c_u64, c_u32, c_u32, c_u32, c_u32, _f64p, vp]),
        "orc_pass": (None, [_i32p, _f64p, c_int, c_int, c_u32, c_d, c_u64, c_u32, c_int, c_u64,
                            vp]),
        "orc_sweeps": (None, [_i32p, _f64p, ctypes.c_int32, c_u32, c_d, c_u64, c_u32,
                              ctypes.c_int32, c_int, vp, vp, vp]),
        "orc_init": (None, [_i32p, _f64p, c_int, c_u64, c_u32]),
        "orc_overrelax_link": (None, [_f64p, _f64p, _f64p]),
        "orc_or_pass": (None, [_i32p, _f64p, c_int, c_int]),
        "orc_sweeps_or": (None, [_i32p, _f64p, ctypes.c_int32, ctypes.c_int32, c_u32, c_d, c_u64,
                                 c_u32, ctypes.c_int32, c_int, vp, vp]),
        "orc_reunitarize": (None, [_i32p, _f64p]),
        "orc_plaquette": (c_d, [_i32p, _f64p]),
        "orc_staple_action": (c_d, [_i32p, _f64p]),
        "orc_polyakov": (None, [_i32p, _f64p, ctypes.POINTER(c_d), ctypes.POINTER(c_d)]),
        "orc_gauge_transform": (None, [_i32p, _f64p, c_u64, c_u32]),
        "orc_wilson_loops": (None, [_i32p, _f64p, c_int, c_int, _f64p]),
        "orc_haar_from_block": (None, [_u32p, _f64p]),
        "orc_max_threads": (c_int, []),
        "orc_nn_feature": (c_d, [c_d]),
        "orc_nn_data": (None, [c_i64, c_d, c_d, c_u64, _f64p, _f64p]),
        "orc_nn_forward": (None, [_f32p, c_d, _f64p]),
        "orc_spline_from_raw": (None, [_f64p, _f64p, _f64p, _f64p]),
        "orc_spline_fwd": (c_d, [_f64p, _f64p, _f64p, c_d, ctypes.POINTER(c_d)]),
        "orc_spline_inv": (c_d, [_f64p, _f64p, _f64p, c_d, ctypes.POINTER(c_d)]),
        "orc_nn_table": (None, [_f32p, _f64p]),
        "orc_table_row": (c_int, [c_d, ctypes.POINTER(c_d)]),
        "orc_table_knots": (None, [_f64p, c_int, _f64p, _f64p, _f64p]),
        "orc_learned_link": (None, [_f64p, _f64p, _f64p, c_d, c_u64, c_u32, c_u32, c_u32, c_u32,
                                    c_d, _f64p, _f64p, ctypes.POINTER(c_int)]),
        "orc_learned_pass": (None, [_i32p, _f64p, _f64p, c_int, c_int, c_u32, c_d, c_u64, c_u32,
                                    c_d, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _dims(dims):
    d = np.ascontiguousarray(dims, dtype=np.int32)
    assert d.shape == (4,)
    return d


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


TAG_TRIAL, TAG_RESERVED, TAG_HOT, TAG_GAUGE, TAG_LEARN, TAG_TRAIN, TAG_BETA = range(7)


def word2(mu, tag, replica=0):
    return (mu | (tag << 2) | (replica << 6)) & 0xFFFFFFFF


def philox(counters, seed):
    """Philox4x32-10 of an (n, 4) uint32 counter array under a 64-bit key."""
    c = np.ascontiguousarray(counters, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(c)
    _load().orc_philox_batch(c.shape[0], c, np.uint64(seed), out)
    return out


def uniform(words):
    w = np.asarray(words, dtype=np.uint64)
    return (2.0 * (w >> np.uint64(9)).astype(np.float64) + 1.0) * 2.0 ** -24


def qmul(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1, 4)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1, 4)
    out = np.empty_like(a)
    _load().orc_qmul_batch(a.shape[0], a, b, out)
    return out


def volume(dims):
    return int(np.prod(np.asarray(dims, dtype=np.int64)))


def check_dims(dims):
    return _load().orc_check_dims(_dims(dims)) == 0


def parity(dims, s):
    return _load().orc_parity(_dims(dims), int(s))


def shift(dims, s, mu, step):
    return _load().orc_shift(_dims(dims), int(s), int(mu), int(step))


def new_links(dims):
    return np.zeros((volume(dims), 4, 4), dtype=np.float64)


def init(dims, start, seed, replica=0):
    U = new_links(dims)
    _load().orc_init(_dims(dims), U, int(start), np.uint64(seed), int(replica))
    return U


def staple(dims, U, s, mu):
    out = np.zeros(4)
    _load().orc_staple(_dims(dims), _c(U), int(s), int(mu), out)
    return out


def hot_link(s, mu, seed, replica=0):
    """U_mu(s) of the hot start, computed on its own."""
    out = np.zeros(4)
    _load().orc_hot_link(int(s), int(mu), np.uint64(seed), int(replica), out)
    return out


def hot_staple(dims, s, mu, seed, replica=0):
    """Staple sum at (s, mu) of the hot-start configuration, without the lattice."""
    out = np.zeros(4)
    _load().orc_hot_staple(_dims(dims), int(s), int(mu), np.uint64(seed), int(replica), out)
    return out


def _c(U):
    assert U.dtype == np.float64 and U.flags["C_CONTIGUOUS"]
    return U


def sample_delta(alpha, seed, site, sweep, mu, replica=0):
    """Exact a0 sampler; returns (delta = 1 - a0, trials, margin) arrays."""
    a = np.ascontiguousarray(alpha, dtype=np.float64).ravel()
    s = np.ascontiguousarray(np.broadcast_to(np.asarray(site, dtype=np.uint32), a.shape))
    delta = np.empty_like(a)
    ntr = np.empty(a.shape, dtype=np.int32)
    mar = np.empty_like(a)
    _load().orc_sample_delta_batch(a.size, a, np.uint64(seed), s, int(sweep), int(mu),
                                   int(replica), delta, _ptr(ntr), _ptr(mar))
    return delta, ntr, mar


def heatbath_link(V, beta, seed, site, sweep, mu, replica=0):
    out = np.zeros(4)
    m = ctypes.c_double()
    _load().orc_heatbath_link(np.ascontiguousarray(V, dtype=np.float64), float(beta),
                              np.uint64(seed), int(site), int(sweep), int(mu), int(replica), out,
                              ctypes.byref(m))
    return out, m.value


def do_pass(dims, U, mu, par, sweep, beta, seed, replica=0, order=0, order_seed=0,
            want_margin=False):
    margin = np.full(volume(dims), np.inf) if want_margin else None
    _load().orc_pass(_dims(dims), _c(U), int(mu), int(par), int(sweep), float(beta),
                     np.uint64(seed), int(replica), int(order), np.uint64(order_seed),
                     _ptr(margin))
    return margin


def sweeps(dims, U, nsweeps, sweep0, beta, seed, replica=0, reunit_every=0, nthreads=1,
           measure=False, want_margin=False):
    """Returns (plaquette, Polyakov) histories with measure=True, then, with
    want_margin=True, each link's smallest decision margin ((V, 4) array)."""
    ph = np.zeros(nsweeps) if measure else None
    lh = np.zeros(nsweeps) if measure else None
    margin = np.full((volume(dims), 4), np.inf) if want_margin else None
    _load().orc_sweeps(_dims(dims), _c(U), int(nsweeps), int(sweep0), float(beta),
                       np.uint64(seed), int(replica), int(reunit_every), int(nthreads),
                       _ptr(ph), _ptr(lh), _ptr(margin))
    out = ((ph, lh) if measure else ()) + ((margin,) if want_margin else ())
    return out if len(out) > 1 else (out[0] if out else None)


def overrelax_link(V, U):
    out = np.zeros(4)
    _load().orc_overrelax_link(np.ascontiguousarray(V, np.float64),
                               np.ascontiguousarray(U, np.float64), out)
    return out


def or_pass(dims, U, mu, par):
    _load().orc_or_pass(_dims(dims), _c(U), int(mu), int(par))


def sweeps_or(dims, U, nsweeps, n_or, sweep0, beta, seed, replica=0, reunit_every=0, nthreads=1,
              measure=False):
    """Compound sweeps (heat bath, then n_or over-relaxation sweeps)."""
    ph = np.zeros(nsweeps) if measure else None
    lh = np.zeros(nsweeps) if measure else None
    _load().orc_sweeps_or(_dims(dims), _c(U), int(nsweeps), int(n_or), int(sweep0), float(beta),
                          np.uint64(seed), int(replica), int(reunit_every), int(nthreads),
                          _ptr(ph), _ptr(lh))
    return (ph, lh) if measure else None


def reunitarize(dims, U):
    _load().orc_reunitarize(_dims(dims), _c(U))


def plaquette(dims, U):
    return _load().orc_plaquette(_dims(dims), _c(U))


def staple_action(dims, U):
    return _load().orc_staple_action(_dims(dims), _c(U))


def polyakov(dims, U):
    s, a = ctypes.c_double(), ctypes.c_double()
    _load().orc_polyakov(_dims(dims), _c(U), ctypes.byref(s), ctypes.byref(a))
    return s.value, a.value


def wilson_loops(dims, U, rmax, tmax):
    """W(R, T), R = 1..rmax, T = 1..tmax, as an (rmax, tmax) array."""
    out = np.zeros(rmax * tmax)
    _load().orc_wilson_loops(_dims(dims), _c(U), int(rmax), int(tmax), out)
    return out.reshape(rmax, tmax)


def gauge_transform(dims, U, seed, replica=0):
    _load().orc_gauge_transform(_dims(dims), _c(U), np.uint64(seed), int(replica))


def haar_from_words(w):
    out = np.zeros(4)
    _load().orc_haar_from_block(np.ascontiguousarray(w, dtype=np.uint32), out)
    return out


def max_threads():
    return _load().orc_max_threads()


# ------------------------------------------------------- learned proposal
NN_NPARAM, NN_OUT, NN_BINS, NN_ROWS, NN_ROW = 2671, 47, 16, 64, 48
ALPHA_LO, ALPHA_HI = 0.5, 30.0


def nn_feature(alpha):
    return _load().orc_nn_feature(float(alpha))


def nn_forward(params, f):
    out = np.zeros(NN_OUT)
    _load().orc_nn_forward(np.ascontiguousarray(params, np.float32), float(f), out)
    return out


def spline_from_raw(raw):
    x, y, d = np.zeros(17), np.zeros(17), np.zeros(17)
    _load().orc_spline_from_raw(np.ascontiguousarray(raw, np.float64), x, y, d)
    return x, y, d


def spline_fwd(knots, xv):
    ld = ctypes.c_double()
    g = _load().orc_spline_fwd(*knots, float(xv), ctypes.byref(ld))
    return g, ld.value


def spline_inv(knots, u):
    ld = ctypes.c_double()
    x = _load().orc_spline_inv(*knots, float(u), ctypes.byref(ld))
    return x, ld.value


def nn_table(params):
    t = np.zeros((NN_ROWS, NN_ROW))
    _load().orc_nn_table(np.ascontiguousarray(params, np.float32), t)
    return t


def table_row(alpha):
    m = ctypes.c_double()
    j = _load().orc_table_row(float(alpha), ctypes.byref(m))
    return j, m.value


def table_knots(table, row):
    x, y, d = np.zeros(17), np.zeros(17), np.zeros(17)
    _load().orc_table_knots(np.ascontiguousarray(table, np.float64), int(row), x, y, d)
    return x, y, d


def learned_link(V, Uold, table, beta, seed, site, sweep, mu, replica=0, or_width=-1.0):
    """Returns (new link, margins (mh, row, range), accepted 1 / 0 / -1 fallback).
    or_width < 0: independence proposal; else the over-relaxed proposal."""
    out = np.zeros(4)
    m = np.zeros(3)
    acc = ctypes.c_int()
    _load().orc_learned_link(np.ascontiguousarray(V, np.float64),
                             np.ascontiguousarray(Uold, np.float64),
                             np.ascontiguousarray(table, np.float64), float(beta),
                             np.uint64(seed), int(site), int(sweep), int(mu), int(replica),
                             float(or_width), out, m, ctypes.byref(acc))
    return out, m, acc.value


def learned_pass(dims, U, table, mu, par, sweep, beta, seed, replica=0, or_width=-1.0):
    """Returns (margins (V, 3), accepted (V,)) for the updated sites."""
    margin = np.full((volume(dims), 3), np.inf)
    acc = np.full(volume(dims), -2, dtype=np.int32)
    _load().orc_learned_pass(_dims(dims), _c(U), np.ascontiguousarray(table, np.float64),
                             int(mu), int(par), int(sweep), float(beta), np.uint64(seed),
                             int(replica), float(or_width), _ptr(margin), _ptr(acc))
    return margin, acc


def nn_data(n, lo, hi, seed):
    a, x = np.zeros(n), np.zeros(n)
    _load().orc_nn_data(int(n), float(lo), float(hi), np.uint64(seed), a, x)
    return a, x
