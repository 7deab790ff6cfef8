"""Write the oracle's first steps on the large cell with its valence states.

The file `cfg5_oracle_reference.npz` holds what the FP64 oracle computes on
the 96^3 cell (simple cubic a = 20.5 bohr, ecut 25 Ha, 64 wells with 256 s/p
projectors, 128 bands, 4 k-points, q = (0.2, 0.1, 0) 2 pi/a, TDDFT with the
Perdew-Zunger kernel), its valence states the lowest 128 eigenpairs of every
sphere (synth, block Davidson to a residual of 1e-10):

  beta[50], z[50]       the first 50 pseudo-Hermitian Lanczos coefficients
                        (Sec. 2.5)
  et_k, et_kq           the band energies (128 valence and 2 more at k+q)
  npw_k, npw_kq, n0_sum ... of the inputs (a reader detects a drift), and the
                        integral of the ground-state density (2 N_b)

Only `oracle/` and `synth/` are called.  Run from the repository root:
    python tests/golden/make_cfg5_reference.py [threads]
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
from threadpoolctl import threadpool_limits  # noqa: E402

import oracle.pw as opw  # noqa: E402
from oracle import lanczos  # noqa: E402
from oracle.liouvillian import Liouvillian  # noqa: E402
from synth import config_system  # noqa: E402

STEPS = 50
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg5_oracle_reference.npz")


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 1
    t0 = time.perf_counter()
    s = config_system("cfg5")
    print(f"system built in {time.perf_counter() - t0:.0f} s", flush=True)
    opw.FFT_WORKERS = threads
    with threadpool_limits(threads):
        L = Liouvillian(s)
        t0 = time.perf_counter()
        r = lanczos.run(L, STEPS)
        print(f"{r.steps} steps ({r.status}) in {time.perf_counter() - t0:.0f} s", flush=True)
    if r.steps != STEPS:
        raise RuntimeError(f"the recursion stopped at step {r.steps}: {r.status}")
    np.savez_compressed(OUT, beta=r.beta, z=r.z, et_k=np.asarray(s.et_k),
                        et_kq=np.asarray(s.et_kq), npw_k=np.asarray(s.npw_k),
                        npw_kq=np.asarray(s.npw_kq),
                        n0_sum=np.float64(np.sum(s.n0_r) * s.omega / np.prod(s.nr)))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
