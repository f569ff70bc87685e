"""Pins of the oracle's quaternion algebra, Philox and uniform mapping.

Quaternion algebra: U = a0 + i a.sigma (Sec. 2) checked against explicit 2x2
complex matrices; Philox4x32-10 against rocRAND's independent host-side
implementation of the same published generator.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

SIG = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]),
       np.array([[1, 0], [0, -1]], complex)]


def mat(a):
    return a[0] * np.eye(2) + 1j * sum(a[i + 1] * SIG[i] for i in range(3))


def test_qmul_matches_2x2_matrices(orc):
    rng = np.random.default_rng(11)
    a = rng.standard_normal((200, 4))
    b = rng.standard_normal((200, 4))
    c = orc.qmul(a, b)
    for i in range(200):
        np.testing.assert_allclose(mat(c[i]), mat(a[i]) @ mat(b[i]), atol=1e-13)


def test_trace_det_and_adjoint(orc):
    rng = np.random.default_rng(12)
    a = rng.standard_normal((50, 4))
    for q in a:
        m = mat(q)
        assert np.isclose(np.trace(m).real / 2, q[0], atol=1e-14)
        assert np.isclose(np.linalg.det(m).real, (q * q).sum(), atol=1e-12)
        qd = q * np.array([1, -1, -1, -1])
        np.testing.assert_allclose(mat(qd), m.conj().T, atol=1e-14)
    u = a / np.linalg.norm(a, axis=1, keepdims=True)
    ud = u * np.array([1, -1, -1, -1])
    np.testing.assert_allclose(orc.qmul(u, ud), np.tile([1, 0, 0, 0], (50, 1)), atol=1e-14)


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available to build the rocRAND reference")
    src = os.path.join(os.path.dirname(__file__), "pins", "rocrand_philox_ref.cpp")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-o", exe, src],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(13)
    n = 2000
    seeds = rng.integers(0, 2 ** 64, n, dtype=np.uint64)
    ctr = rng.integers(0, 2 ** 32, (n, 4), dtype=np.uint64).astype(np.uint32)
    seeds[:4] = [0, 1, 2 ** 64 - 1, 0x123456789ABCDEF0]
    ctr[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 2, 3, 4], [5308415, 1999, 0x1C3, 7]]
    lines = "\n".join(f"{s} {c[0]} {c[1]} {c[2]} {c[3]}" for s, c in zip(seeds, ctr))
    out = subprocess.run([rocrand_ref], input=lines, capture_output=True, text=True,
                         check=True).stdout.split()
    ref = np.array(out, dtype=np.uint64).reshape(n, 4).astype(np.uint32)
    mine = np.concatenate([orc.philox(ctr[i:i + 1], int(seeds[i])) for i in range(n)])
    np.testing.assert_array_equal(mine, ref)


def test_uniform_mapping_exact_open_interval(orc):
    w = np.array([0, 1, 511, 512, 0x7FFFFFFF, 0xFFFFFFFF, 0xFFFFFE00], dtype=np.uint32)
    u = orc.uniform(w)
    assert u.min() > 0 and u.max() < 1
    assert u[0] == 2.0 ** -24 and u[5] == 1 - 2.0 ** -24
    np.testing.assert_array_equal(u.astype(np.float32).astype(np.float64), u)
    for wi, ui in zip(w, u):
        assert orc._load().orc_uniform(int(wi)) == ui
    # 23 random bits: distinct words differing only below bit 9 map together
    assert orc.uniform(np.array([1024 + 3], np.uint32))[0] == orc.uniform(np.array([1024], np.uint32))[0]
