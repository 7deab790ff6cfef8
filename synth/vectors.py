"""Seeded random batches of response orbitals (operator unit tests only)."""
import numpy as np


def random_batch(sys, seed: int, scale: float = 1.0) -> np.ndarray:
    """Complex Gaussian batch [nks, nbnd, npwx] on the k+q spheres, zero in
    the padding beyond npw_kq."""
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal((sys.nks, sys.nbnd, sys.npwx))
         + 1j * rng.standard_normal((sys.nks, sys.nbnd, sys.npwx))) * scale
    for k in range(sys.nks):
        x[k, :, int(sys.npw_kq[k]):] = 0.0
    return x
