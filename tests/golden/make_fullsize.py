"""Write the stored oracle results of the full-size parity tests.

    python tests/golden/make_fullsize.py [c3] [c5]

Runs the FP64 CPU oracle (oracle/, nothing else) on the seeded full-size
workloads and stores summaries of the final state (tests/helpers.py,
state_summary: per-block L1 norms, sums and seeded random projections of
every variable, plus the state at 4096 seeded cells) with the per-step time
steps:
  * c3: 3D ideal MHD, 4096 uneven blocks 32^3:16^3:8^3 with fixed faces,
        10 SSPRK(5,4) steps at CFL 0.4  -> fullsize_c3_10.npz
  * c5: 3D ideal MHD, 256^3 periodic in 4096 blocks of 16^3,
        100 SSPRK(5,4) steps at CFL 0.4 -> fullsize_c5_100.npz
The oracle needs about 40 GB of host memory and an hour (c5) on 8 cores.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from helpers import input_digest, state_summary  # noqa: E402
from paper_1407_2052_amd import inputs  # noqa: E402

CASES = {
    "c3": ("fullsize_c3_10.npz", lambda: inputs.uneven_3d(), 10),
    "c5": ("fullsize_c5_100.npz", lambda: inputs.mhd_turbulence_3d(), 100),
}


def make(name):
    fname, gen, nsteps = CASES[name]
    t0 = time.time()
    bs = gen()
    digest = input_digest(bs)
    print(f"{name}: input {digest[:16]}, {bs.interior_cells()} cells, {nsteps} steps", flush=True)
    out, dts = oracle.run(bs, oracle.SSPRK54, nsteps, cfl=0.4)
    del bs
    summ = state_summary(out, out.u)
    meta = {"case": name, "scheme": "SSPRK(5,4)", "cfl": 0.4, "nsteps": nsteps, "input_sha256": digest,
            "oracle_threads": oracle.num_threads(), "seconds": round(time.time() - t0, 1)}
    np.savez(os.path.join(HERE, fname), dts=dts, meta=np.array(json.dumps(meta)), **summ)
    print(f"{name}: wrote {fname} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        make(name)
