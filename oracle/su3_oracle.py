"""ctypes wrapper over the FP64 SU(3) CPU oracle (oracle/su3_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  It shares no code with the GPU library.

Link arrays are complex128 numpy arrays of shape (V, 4, 3, 3) = [site][mu][row][col]
with site s = x + Nx*(y + Ny*(z + Nz*t)); the same order the GPU library uses
for its host exchange format (there as interleaved float64 re/im pairs).
"""
import ctypes

import numpy as np

from . import su2_oracle as _o2

_lib = None
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_c128p = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = _o2._load()
    c_u64, c_u32, c_i64, c_int, c_d = (ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64,
                                       ctypes.c_int, ctypes.c_double)
    vp = ctypes.c_void_p
    pd = ctypes.POINTER(c_d)
    sig = {
        "orc3_staple": (None, [_i32p, _c128p, c_i64, c_int, _c128p]),
        "orc3_heatbath_link": (None, [_c128p, _c128p, c_d, c_u64, c_u32, c_u32, c_u32, c_u32,
                                      _c128p, pd]),
        "orc3_pass": (None, [_i32p, _c128p, c_int, c_int, c_u32, c_d, c_u64, c_u32, c_int, vp]),
        "orc3_sweeps": (None, [_i32p, _c128p, ctypes.c_int32, c_u32, c_d, c_u64, c_u32,
                               ctypes.c_int32, c_int, vp, vp]),
        "orc3_init": (None, [_i32p, _c128p, c_int, c_u64, c_u32]),
        "orc3_reunitarize": (None, [_i32p, _c128p]),
        "orc3_plaquette": (c_d, [_i32p, _c128p]),
        "orc3_polyakov": (None, [_i32p, _c128p, pd, pd, pd]),
        "orc3_staple_action": (c_d, [_i32p, _c128p]),
        "orc3_gauge_transform": (None, [_i32p, _c128p, c_u64, c_u32]),
        "orc3_link_chain": (None, [_c128p, c_d, c_i64, c_u64, _c128p, vp]),
        "orc3_overrelax_link": (None, [_c128p, _c128p, _c128p]),
        "orc3_hot_link": (None, [c_i64, c_int, c_u64, c_u32, _c128p]),
        "orc3_hot_staple": (None, [_i32p, c_i64, c_int, c_u64, c_u32, _c128p]),
        "orc3_or_pass": (None, [_i32p, _c128p, c_int, c_int, c_int]),
        "orc3_sweeps_or": (None, [_i32p, _c128p, ctypes.c_int32, ctypes.c_int32, c_u32, c_d,
                                  c_u64, c_u32, ctypes.c_int32, c_int, vp, vp]),
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


def _links(U, dims):
    assert U.dtype == np.complex128 and U.flags.c_contiguous
    assert U.shape == (_o2.volume(dims), 4, 3, 3)
    return U


def _m3(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    assert a.shape == (3, 3)
    return a


def new_links(dims):
    return np.zeros((_o2.volume(dims), 4, 3, 3), dtype=np.complex128)


def init(dims, start, seed, replica=0):
    """start 0: unit links; 1: Haar-random links."""
    U = new_links(dims)
    _load().orc3_init(_dims(dims), U, int(start), np.uint64(seed), replica)
    return U


def staple(dims, U, s, mu):
    A = np.zeros((3, 3), dtype=np.complex128)
    _load().orc3_staple(_dims(dims), _links(U, dims), int(s), int(mu), A)
    return A


def heatbath_link(U, A, beta, seed, site, sweep, mu, replica=0):
    """One Cabibbo-Marinari update (three SU(2) subgroup draws); returns
    (new link, smallest decision margin of the three samplers)."""
    out = np.zeros((3, 3), dtype=np.complex128)
    m = ctypes.c_double()
    _load().orc3_heatbath_link(_m3(U), _m3(A), float(beta), np.uint64(seed), site, sweep, mu,
                               replica, out, ctypes.byref(m))
    return out, m.value


def pass_(dims, U, mu, parity, sweep, beta, seed, replica=0, nthreads=1, margin=None):
    if margin is not None:
        assert margin.dtype == np.float64 and margin.shape == (_o2.volume(dims),)
    _load().orc3_pass(_dims(dims), _links(U, dims), mu, parity, sweep, float(beta),
                      np.uint64(seed), replica, int(nthreads),
                      None if margin is None else margin.ctypes.data_as(ctypes.c_void_p))


def sweeps(dims, U, nsweeps, sweep0, beta, seed, replica=0, reunit_every=0, nthreads=1,
           history=False):
    """nsweeps sweeps in place; with history, returns (plaquette, Re Polyakov) per sweep."""
    ph = np.zeros(nsweeps) if history else None
    lh = np.zeros(nsweeps) if history else None
    _load().orc3_sweeps(_dims(dims), _links(U, dims), nsweeps, sweep0, float(beta),
                        np.uint64(seed), replica, reunit_every, int(nthreads),
                        None if ph is None else ph.ctypes.data_as(ctypes.c_void_p),
                        None if lh is None else lh.ctypes.data_as(ctypes.c_void_p))
    return (ph, lh) if history else None


def hot_link(s, mu, seed, replica=0):
    """U_mu(s) of the hot start, computed on its own."""
    out = np.zeros((3, 3), dtype=np.complex128)
    _load().orc3_hot_link(int(s), int(mu), np.uint64(seed), int(replica), out)
    return out


def hot_staple(dims, s, mu, seed, replica=0):
    """Staple sum at (s, mu) of the hot-start configuration, without the lattice."""
    out = np.zeros((3, 3), dtype=np.complex128)
    _load().orc3_hot_staple(_dims(dims), int(s), int(mu), np.uint64(seed), int(replica), out)
    return out


def overrelax_link(U, A):
    """Microcanonical over-relaxation of one link with staple sum A."""
    out = np.zeros((3, 3), dtype=np.complex128)
    _load().orc3_overrelax_link(_m3(U), _m3(A), out)
    return out


def or_pass(dims, U, mu, parity, nthreads=1):
    _load().orc3_or_pass(_dims(dims), _links(U, dims), mu, parity, int(nthreads))


def sweeps_or(dims, U, nsweeps, n_or, sweep0, beta, seed, replica=0, reunit_every=0, nthreads=1,
              history=False):
    """nsweeps heat-bath sweeps, each followed by n_or over-relaxation sweeps;
    with history, returns (plaquette, Re Polyakov) after each heat-bath sweep's group."""
    ph = np.zeros(nsweeps) if history else None
    lh = np.zeros(nsweeps) if history else None
    _load().orc3_sweeps_or(_dims(dims), _links(U, dims), nsweeps, n_or, sweep0, float(beta),
                           np.uint64(seed), replica, reunit_every, int(nthreads),
                           None if ph is None else ph.ctypes.data_as(ctypes.c_void_p),
                           None if lh is None else lh.ctypes.data_as(ctypes.c_void_p))
    return (ph, lh) if history else None


def reunitarize(dims, U):
    _load().orc3_reunitarize(_dims(dims), _links(U, dims))


def plaquette(dims, U):
    return _load().orc3_plaquette(_dims(dims), _links(U, dims))


def polyakov(dims, U):
    """(Re, Im) of the mean of Tr L / 3, and the mean of |Tr L / 3|."""
    re, im, mag = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _load().orc3_polyakov(_dims(dims), _links(U, dims), ctypes.byref(re), ctypes.byref(im),
                          ctypes.byref(mag))
    return re.value, im.value, mag.value


def staple_action(dims, U):
    return _load().orc3_staple_action(_dims(dims), _links(U, dims))


def gauge_transform(dims, U, seed, replica=0):
    _load().orc3_gauge_transform(_dims(dims), _links(U, dims), np.uint64(seed), replica)


def link_chain(A, beta, nsteps, seed, U0=None):
    """Markov chain of one link under a fixed staple A; returns (end link,
    (nsteps, 2) complex array of [Tr(U A), Tr U] after every step)."""
    U = np.eye(3, dtype=np.complex128) if U0 is None else _m3(U0).copy()
    obs = np.zeros((int(nsteps), 2), dtype=np.complex128)
    _load().orc3_link_chain(_m3(A), float(beta), int(nsteps), np.uint64(seed), U,
                            obs.ctypes.data_as(ctypes.c_void_p))
    return U, obs
