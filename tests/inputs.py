"""Seeded synthetic inputs shared by the oracle side and the GPU side of tests.

Holds none of the method's arithmetic: only numpy random draws of link
configurations, staples and coupling values, in the canonical host layout
float32 [t][z][y][x][mu][c] (flattened as (V, 4, 4)).
"""
import numpy as np


def volume(dims):
    return int(np.prod(np.asarray(dims, dtype=np.int64)))


def random_links(dims, seed, spread=None):
    """Unit quaternions as float32 (V, 4, 4).

    spread=None: isotropic (Gaussian 4-vector normalised).
    spread=eps : identity plus Gaussian noise of width eps, normalised; mimics a
                 thermalised weak-coupling configuration.
    """
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((volume(dims), 4, 4))
    if spread is not None:
        g *= spread
        g[..., 0] += 1.0
    g /= np.linalg.norm(g, axis=-1, keepdims=True)
    return g.astype(np.float32)


def as_f64(links32):
    return np.ascontiguousarray(links32, dtype=np.float64)


def random_staples(n, seed, kmin=0.05, kmax=6.0):
    """Staple sums V with |V| log-uniform in [kmin, kmax] (float32, (n, 4))."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 4))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    k = np.exp(rng.uniform(np.log(kmin), np.log(kmax), n))
    return (d * k[:, None]).astype(np.float32)


def log_uniform(n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n))


def random_su3_links(dims, seed, spread=None):
    """SU(3) links as complex128 (V, 4, 3, 3).

    spread=None: Haar (QR of a complex Gaussian matrix, phases of R's diagonal
                 moved into Q, det divided out by a cube root).
    spread=eps : the same decomposition of identity plus complex Gaussian noise
                 of width eps; mimics an ordered configuration.
    """
    rng = np.random.default_rng(seed)
    n = volume(dims) * 4
    z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2)
    if spread is not None:
        z = np.eye(3) + spread * z
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    q = q * (np.linalg.det(q) ** (-1.0 / 3.0))[:, None, None]
    return np.ascontiguousarray(q.reshape(volume(dims), 4, 3, 3))
