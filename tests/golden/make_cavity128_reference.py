"""Write tests/golden/cavity128_ra1e6_d3q7_2500.npz with the CPU oracle.

The 128^3 cavity at Ra = 1e6, Pr = 0.71, u0 = 0.05, D3Q7 scalar, started
from rest, advanced 2500 steps: the same physical time (t u0 / L) as 10,000
steps of the 512^3 cavity.  The shear rate is 1.937 here, outside the
linear stability range of the default rate set, so both this run and the
512^3 runs it is compared with use the stable set: bulk rate 1, Maxwellian
fourth-order equilibrium, c_sphi^2 = 1/4 (the same Ra, Pr and u0, hence the
same continuum problem).  Stored: the macroscopic fields (rho, ux, uy, uz,
T, float32) on the mid-planes y = 64 and z = 64 (0-based cell indices), the
points the 512^3 fields are compared at after averaging each 4x4x4 block.

Only the oracle is called.  Runtime: several CPU hours (OpenMP threads from
ORACLE_THREADS, default all cores).  With GOLDEN_CHECKPOINT set to a file
path the state is saved there every 500 steps and a run resumes from it.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402

N, RA, STEPS = 128, 1e6, 2500
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cavity128_ra1e6_d3q7_2500.npz")


def main():
    threads = O.set_threads(int(os.environ.get("ORACLE_THREADS", "0")) or (os.cpu_count() or 1))
    p = O.cavity_params(N, RA, omega_bulk=1.0, fourth_maxwell=1, cs2T=0.25)
    F, G = O.rest_state(p)
    done, chunk = 0, 100
    ckpt = os.environ.get("GOLDEN_CHECKPOINT")
    if ckpt and os.path.exists(ckpt):
        z = np.load(ckpt)
        F, G, done = z["F"].copy(), z["G"].copy(), int(z["done"])
        print(f"resumed at step {done}", flush=True)
    t0 = time.time()
    while done < STEPS:
        k = min(chunk, STEPS - done)
        F, G, mac = O.run(p, k, F, G)
        done += k
        if not np.all(np.isfinite(mac)):
            raise SystemExit(f"non-finite fields after {done} steps")
        print(f"{done}/{STEPS} steps, {time.time() - t0:.0f} s, {threads} threads", flush=True)
        if ckpt and done % 500 == 0 and done < STEPS:
            np.savez(ckpt + ".tmp.npz", F=F, G=G, done=done)
            os.replace(ckpt + ".tmp.npz", ckpt)
    np.savez_compressed(
        OUT, steps=STEPS, n=N, Ra=RA, plane_y=64, plane_z=64,
        y64=mac[:, :, 64, :].astype(np.float32), z64=mac[:, 64, :, :].astype(np.float32),
        fields=np.array(["rho", "ux", "uy", "uz", "T"]),
        rates=np.array(["omega_bulk=1", "fourth_maxwell=1", "cs2_T=0.25"]))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
