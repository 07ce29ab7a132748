"""Seeded random inputs for parity tests (no method arithmetic here)."""
import numpy as np


def random_active_set(n, fill, seed, blob=True):
    """Sorted unique row-major linear keys on the grid ``n``.

    ``blob=True`` draws an ellipsoidal blob (the shape a thresholded smooth
    packet has) with holes and a scattering of isolated points, so fibers
    come in mixed lengths with gaps.  ``blob=False`` draws uniformly.
    """
    rng = np.random.default_rng(seed)
    n = [int(v) for v in n]
    total = int(np.prod(n))
    if not blob:
        m = max(1, int(round(fill * total)))
        keys = rng.choice(total, size=m, replace=False)
        return np.sort(keys).astype(np.uint64)
    grids = np.meshgrid(*[np.arange(v) for v in n], indexing="ij")
    centre = [rng.uniform(0.3, 0.7) * (v - 1) for v in n]
    radius = [max(1.0, rng.uniform(0.3, 0.6) * v) for v in n]
    r2 = sum(((g - c) / r) ** 2 for g, c, r in zip(grids, centre, radius))
    mask = r2 <= 1.0
    mask &= rng.random(mask.shape) > 0.15          # holes inside the blob
    mask |= rng.random(mask.shape) < 0.02          # isolated outliers
    keys = np.flatnonzero(mask.ravel())
    if keys.size == 0:
        keys = np.array([rng.integers(total)])
    return keys.astype(np.uint64)


def random_complex(m, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return (scale * (rng.standard_normal(m) + 1j * rng.standard_normal(m))).astype(np.complex128)


def random_dense_factor(nk, seed, hermitian=False):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((nk, nk)) + 1j * rng.standard_normal((nk, nk))
    if hermitian:
        a = a + a.conj().T
    return a.astype(np.complex128)
