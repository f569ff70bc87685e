"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/su2.h declares, and rejects bad arguments before any
device work."""
import ctypes

import numpy as np
import pytest

import paper_1010_1486_amd as su2


def test_library_exports_every_declared_function():
    lib = su2.lib()
    names = su2.header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_sizes():
    assert su2.su2_links_bytes([4, 4, 4, 4]) == 64 * 256
    assert su2.su2_links_bytes([48, 48, 48, 48]) == 64 * 48 ** 4
    assert su2.su2_links_bytes([3, 4, 4, 4]) == 0
    assert su2.su2_links_bytes([512, 512, 512, 4]) == 0  # V/2 = 2^28: out of range
    assert su2.su2_links_bytes([1 << 30] * 4) == 0  # no overflow
    assert su2.su2_links_bytes([512, 512, 512, 2]) == 64 * 512 ** 3 * 2
    assert su2.su2_scratch_bytes([4, 4, 4, 4]) >= 256


@pytest.mark.parametrize("dims", [[3, 4, 4, 4], [4, 4, 4, 5], [0, 4, 4, 4], [4, 1, 4, 4]])
def test_odd_or_small_extents_rejected(dims):
    with pytest.raises(su2.SU2Error) as e:
        su2.su2_init(dims, 2.3, 1, su2.SU2_COLD)
    assert e.value.code == su2.SU2_EODD


def test_bad_arguments_rejected():
    # the samplers need alpha = beta k >= 0
    for beta in (float("nan"), float("inf"), -0.5, -1e-300):
        with pytest.raises(su2.SU2Error) as e:
            su2.su2_init([4, 4, 4, 4], beta, 1, su2.SU2_COLD)
        assert e.value.code == su2.SU2_EINVAL
    with pytest.raises(su2.SU2Error) as e:
        su2.su2_test_heatbath_links(np.ones((2, 4), np.float32), -1.0, 1, 0, 0)
    assert e.value.code == su2.SU2_EINVAL
    with pytest.raises(su2.SU2Error) as e:
        su2.su2_init([4, 4, 4, 4], 2.0, 1, 7)
    assert e.value.code == su2.SU2_EINVAL
    for dims in ([2048, 2048, 2048, 2], [512, 512, 512, 4]):  # V/2 >= 2^28
        with pytest.raises(su2.SU2Error) as e:
            su2.su2_init(dims, 2.0, 1, su2.SU2_COLD)
        assert e.value.code == su2.SU2_ERANGE
    lib = su2.lib()
    assert lib.su2_init(None, None, 1.0, 1, 0) == su2.SU2_EINVAL
    assert lib.su2_heatbath_sweep(None, 1, 0) == su2.SU2_EINVAL
    assert lib.su2_plaquette(None, None) == su2.SU2_EINVAL
    assert lib.su2_destroy(None) == su2.SU2_EINVAL
    assert b"NULL" in lib.su2_last_error()
    h = ctypes.c_void_p()
    d = np.array([4, 4, 4, 4], np.int32)
    rc = lib.su2_init_ext(ctypes.byref(h), d.ctypes.data_as(ctypes.c_void_p), 2.0, 1, 0,
                          None, 0, None, 0, None)
    assert rc == su2.SU2_EINVAL
    rc = lib.su2_init_ext(ctypes.byref(h), d.ctypes.data_as(ctypes.c_void_p), 2.0, 1, 0,
                          ctypes.c_void_p(4096), 16, ctypes.c_void_p(8192), 16, None)
    assert rc == su2.SU2_ENOMEM
    assert lib.su2_test_stream_pass(None, 0, 0, None) == su2.SU2_EINVAL
    assert lib.su2_nn_train_cosine(None, 10, 64, 1e-3, 1e-5, None) == su2.SU2_EINVAL
    assert lib.su2_test_philox(None, -1, 0, None) == su2.SU2_EINVAL
    assert lib.su2_test_philox(None, 0, 0, None) == su2.SU2_OK


@pytest.mark.parametrize("dims,tiles", [
    ([2, 2, 2, 2], (0, 0)), ([4, 4, 4, 4], (0, 0)), ([4, 6, 2, 8], (2, 4)),
    ([8, 6, 8, 10], (8, 2)), ([12, 10, 8, 6], (4, 2)), ([6, 4, 12, 16], (4, 16)),
    ([48, 4, 48, 8], (16, 8))], ids=str)
def test_pass_index_map_matches_oracle_neighbours(orc, dims, tiles):
    """The pass kernel's traversal (tiled (z,t)-plane order, magic-number
    division, additive neighbour offsets) evaluated on the host: every site of
    the parity is visited exactly once and every neighbour index equals the
    oracle's periodic shift."""
    V = int(np.prod(dims))
    for par in (0, 1):
        m = su2.su2_test_index_map(dims, par, *tiles).astype(np.int64)
        sites = m[:, 0]
        assert np.array_equal(np.sort(sites), np.sort(
            [s for s in range(V) if orc.parity(dims, s) == par]))
        for row in m[:: max(1, len(m) // 400)]:
            s = int(row[0])
            for d in range(4):
                assert row[1 + 2 * d] == orc.shift(dims, s, d, +1) >> 1
                assert row[2 + 2 * d] == orc.shift(dims, s, d, -1) >> 1
        assert m[:, 1:].max() < V // 2


def test_index_map_rejects_bad_tiles():
    with pytest.raises(su2.SU2Error):
        su2.su2_test_index_map([4, 4, 6, 4], 0, tile_z=4)
    with pytest.raises(su2.SU2Error):
        su2.su2_test_index_map([4, 4, 4, 4], 0, tile_t=3)


REPLICAS64 = [[8 + 2 * (r % 7)] * 4 for r in range(64)]


@pytest.mark.parametrize("queues", [1, 3, 8])
@pytest.mark.parametrize("dims,block,ns,reunit,first,meas,rows", [
    ([[4, 4, 4, 4]], 256, 7, 0, 0, 0, False),
    ([[48, 48, 48, 48]], 256, 2, 2, 1, 3, True),
    ([[8, 6, 8, 16], [4, 4, 4, 8], [6, 6, 6, 4]], 64, 13, 4, 3, 3, True),
    ([[8, 6, 8, 16], [4, 4, 4, 8], [6, 6, 6, 4]], 128, 9, 3, 0, 1, True),
    ([[2, 2, 2, 2], [16, 16, 16, 16]], 192, 6, 1, 0, 2, True),
    (REPLICAS64, 256, 5, 10, 8, 1, True),
    (REPLICAS64, 128, 3, 0, 0, 3, False),
], ids=["4^4", "48^4", "three-mixed", "three-plaq", "reunit-every-sweep", "replicas64",
        "replicas64-nomeas"])
def test_work_queue_schedule(dims, block, ns, reunit, first, meas, rows, queues):
    """The persistent work-queue launch run on the host one item at a time in
    ticket order, queue by queue: the replicas' slots tile the queues, every
    item's wait target counts exactly its replica's earlier items (no
    deadlock, no early start), the stage kinds follow the sweep schedule and
    every sweep of every replica ends."""
    items = su2.su2_test_queue_plan(dims, block, ns, reunit, first, meas, rows, queues)
    nb = [-(-int(np.prod(d)) // 2 // block) for d in dims]
    per_sweep = 8 + (1 if rows and meas & 2 else 0)
    n_reunit = sum(1 for j in range(first, first + ns) if reunit and (j + 1) % reunit == 0)
    extra = n_reunit * (1 + (1 if rows and meas & 1 else 0))
    assert items == sum(nb) * (per_sweep * ns + extra)


def test_work_queue_schedule_rejects_bad_arguments():
    with pytest.raises(su2.SU2Error):
        su2.su2_test_queue_plan([[4, 4, 4, 4]], 100, 2)
    with pytest.raises(su2.SU2Error):
        su2.su2_test_queue_plan([[4, 4, 4, 5]], 256, 2)
    with pytest.raises(su2.SU2Error) as e:
        su2.su2_test_queue_plan([[48, 48, 48, 48]], 64, 100000)
    assert e.value.code == su2.SU2_ERANGE
    with pytest.raises(su2.SU2Error):
        su2.su2_test_queue_plan([[4, 4, 4, 4]], 256, 2, queues=17)


def test_library_exports_every_su3_function():
    lib = su2.lib3()
    names = su2.header_functions3()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_su3_sizes_and_bad_arguments():
    from paper_1010_1486_amd import su3
    assert su3.su3_links_bytes([4, 4, 4, 4]) == 192 * 256
    assert su3.su3_links_bytes([48, 48, 48, 48]) == 192 * 48 ** 4
    assert su3.su3_links_bytes([3, 4, 4, 4]) == 0
    assert su3.su3_links_bytes([512, 512, 512, 4]) == 0
    lib = su2.lib3()
    h = ctypes.c_void_p()
    d = np.array([4, 4, 4, 5], dtype=np.int32)
    assert lib.su3_init(ctypes.byref(h), d.ctypes.data_as(ctypes.c_void_p), 6.0, 1, 0,
                        None) == su2.SU2_EODD
    d = np.array([4, 4, 4, 4], dtype=np.int32)
    for beta in (float("nan"), -6.0):
        assert lib.su3_init(ctypes.byref(h), d.ctypes.data_as(ctypes.c_void_p), beta, 1, 0,
                            None) == su2.SU2_EINVAL
    assert lib.su3_init(ctypes.byref(h), d.ctypes.data_as(ctypes.c_void_p), 6.0, 1, 7,
                        None) == su2.SU2_EINVAL
    assert lib.su3_init(None, d.ctypes.data_as(ctypes.c_void_p), 6.0, 1, 0, None) == su2.SU2_EINVAL
    for call in (lambda: lib.su3_destroy(None), lambda: lib.su3_reunitarize(None),
                 lambda: lib.su3_heatbath_sweep(None, 1, 0, None),
                 lambda: lib.su3_test_pass(None, 0, 0), lambda: lib.su3_synchronize(None),
                 lambda: lib.su3_set_replica(None, 1)):
        assert call() == su2.SU2_EINVAL


def test_su3_batch_bad_arguments():
    """su3_batch_init checks n, the couplings, the extents and its pointers
    before any device work (no GPU needed), and every batch call refuses a
    NULL batch."""
    lib = su2.lib3()
    h = ctypes.c_void_p()
    d = np.array([4, 4, 4, 4], dtype=np.int32)
    dp = d.ctypes.data_as(ctypes.c_void_p)
    betas = np.array([5.5, 5.7, 6.0])
    bp = betas.ctypes.data_as(ctypes.c_void_p)
    for n in (0, -1, 65536):
        assert lib.su3_batch_init(ctypes.byref(h), n, dp, bp, 1, 0, None) == su2.SU2_EINVAL
    assert lib.su3_batch_init(ctypes.byref(h), 3, dp, None, 1, 0, None) == su2.SU2_EINVAL
    assert lib.su3_batch_init(None, 3, dp, bp, 1, 0, None) == su2.SU2_EINVAL
    assert lib.su3_batch_init(ctypes.byref(h), 3, dp, bp, 1, 7, None) == su2.SU2_EINVAL
    for bad in (float("nan"), -1.0, float("inf")):
        b2 = np.array([5.5, bad, 6.0])
        assert lib.su3_batch_init(ctypes.byref(h), 3, dp, b2.ctypes.data_as(ctypes.c_void_p),
                                  1, 0, None) == su2.SU2_EINVAL
    d5 = np.array([4, 4, 4, 5], dtype=np.int32)
    assert lib.su3_batch_init(ctypes.byref(h), 3, d5.ctypes.data_as(ctypes.c_void_p), bp, 1, 0,
                              None) == su2.SU2_EODD
    assert h.value is None
    out = np.zeros(8)
    op = out.ctypes.data_as(ctypes.c_void_p)
    for call in (lambda: lib.su3_batch_destroy(None), lambda: lib.su3_batch_size(None, op),
                 lambda: lib.su3_batch_heatbath_sweep(None, 1, 0, None),
                 lambda: lib.su3_batch_overrelax(None, 1), lambda: lib.su3_batch_reunitarize(None),
                 lambda: lib.su3_batch_plaquette(None, op), lambda: lib.su3_batch_polyakov(None, op),
                 lambda: lib.su3_batch_get_links(None, 0, op),
                 lambda: lib.su3_batch_set_links(None, 0, op),
                 lambda: lib.su3_batch_get_sweep(None, op), lambda: lib.su3_batch_set_sweep(None, 0),
                 lambda: lib.su3_batch_set_launch(None, 256, 1, 1, 0, 0),
                 lambda: lib.su3_batch_synchronize(None)):
        assert call() == su2.SU2_EINVAL


def test_no_exception_leaves_the_c_abi():
    """Every extern "C" entry point defined in the runtime sources runs its body
    inside the exception barrier (SU2_API_BEGIN ... SU2_API_END), so host-side
    allocation failures come back as SU2_ENOMEM, never as an exception."""
    import os
    import re
    csrc = os.path.join(os.path.dirname(su2.__file__), "csrc")
    seen = 0
    for f in ("su2_runtime.cpp", "su3_runtime.cpp", "su2_static.hip"):
        lines = open(os.path.join(csrc, f)).read().split("\n")
        for i, l in enumerate(lines):
            if re.match(r"^(int|size_t) (su2_|su3_)\w+\(", l):
                j = lines.index("{", i)
                k = lines.index("}", j)
                assert lines[j + 1].strip() == "SU2_API_BEGIN", (f, l)
                assert lines[k - 1].strip().startswith("SU2_API_END"), (f, l)
                seen += 1
    exported = set(su2.header_functions()) | set(su2.header_functions3())
    assert seen >= len(exported) - 1  # su2_last_error only reads a string


def test_static_sweeps_reject_bad_arguments_before_device_work():
    """su2_sweep_measure_static checks its arguments before it touches a
    device (these calls need no GPU)."""
    lib = su2.lib()
    fake = ctypes.c_void_p(16)  # never dereferenced: the checks come first
    good = np.array([4, 4, 4, 4], np.int32)
    odd = np.array([4, 4, 4, 5], np.int32)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    f = lib.su2_sweep_measure_static
    assert f(None, p(good), 2.0, 1, 0, 1, 0, 1, fake, None) == su2.SU2_EINVAL
    assert f(fake, p(good), 2.0, 1, 0, 1, 0, 1, None, None) == su2.SU2_EINVAL
    assert f(fake, p(odd), 2.0, 1, 0, 1, 0, 1, fake, None) == su2.SU2_EODD
    assert f(fake, p(good), -1.0, 1, 0, 1, 0, 1, fake, None) == su2.SU2_EINVAL
    assert f(fake, p(good), 2.0, 1, 0, -1, 0, 1, fake, None) == su2.SU2_EINVAL
    assert f(fake, p(good), 2.0, 1, 0, 1, 0, 8, fake, None) == su2.SU2_EINVAL
    big = np.array([512, 512, 512, 4], np.int32)  # V/2 = 2^28
    assert f(fake, p(big), 2.0, 1, 0, 1, 0, 1, fake, None) == su2.SU2_ERANGE
