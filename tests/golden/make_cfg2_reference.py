"""Write the oracle's reference recursion of the 48^3 benchmark cell.

The file `cfg2_oracle_reference.npz` holds what the FP64 oracle computes on
the 48^3 cell (simple cubic a = 10.26 bohr, ecut 25 Ha, 8 wells with 32 s/p
projectors, 16 bands, 8 k-points, q = 0.2 (2 pi/a) [100], TDDFT with the
Perdew-Zunger kernel):

  beta[3000], z[3000]   the pseudo-Hermitian Lanczos coefficients (Sec. 2.5)
                        of 3000 steps; the first M of them are the
                        coefficients of an M-step recursion
  loss_300, loss_1000, loss_3000
                        -Im eps^-1 on 2000 frequencies in [0, 2] Ha with
                        eta = 0.01 Ha from the first 300, 1000 and 3000
                        coefficients (eqs. post_processing,
                        def_inv_microscopic_diel_tensor)
  et_k, et_kq, npw_k, npw_kq
                        the input system's band energies and sphere sizes,
                        so that a reader detects a drift of the inputs

Only `oracle/` and `synth/` are called.  Run from the repository root:
    python tests/golden/make_cfg2_reference.py [threads]
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
from threadpoolctl import threadpool_limits  # noqa: E402

import oracle.pw as opw  # noqa: E402
from oracle import lanczos, spectrum  # noqa: E402
from oracle.liouvillian import Liouvillian  # noqa: E402
from synth import config_system  # noqa: E402

STEPS = 3000
CUTS = (300, 1000, 3000)
OMEGA = np.linspace(0.0, 2.0, 2000)
ETA = 0.01
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg2_oracle_reference.npz")


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 1
    opw.FFT_WORKERS = threads
    s = config_system("cfg2")
    with threadpool_limits(threads):
        L = Liouvillian(s)
        t0 = time.perf_counter()
        r = lanczos.run(L, STEPS)
        print(f"{r.steps} steps ({r.status}) in {time.perf_counter() - t0:.0f} s", flush=True)
    if r.steps != STEPS:
        raise RuntimeError(f"the recursion stopped at step {r.steps}: {r.status}")
    out = dict(beta=r.beta, z=r.z, omega=OMEGA, eta=np.float64(ETA),
               et_k=np.asarray(s.et_k), et_kq=np.asarray(s.et_kq),
               npw_k=np.asarray(s.npw_k), npw_kq=np.asarray(s.npw_kq))
    for m in CUTS:
        out[f"loss_{m}"] = spectrum.spectrum(r.beta, r.z, OMEGA, ETA, s.omega, s.qcart, m=m)[2]
    np.savez_compressed(OUT, **out)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
