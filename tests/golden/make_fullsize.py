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
  * c4grad: 2D Euler, 256^2 periodic in 256 blocks of 16^2, 200 SSPRK(5,4)
        steps at the fixed dt 0.4 / sum_d c_max,d(U_0)/dx_d; the gradient of
        J = 1/2 sum (rho_N - rho*)^2 with respect to U_0 by the oracle's
        reverse mode -> fullsize_c4_grad200.npz (every interior entry)
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


def make_c4grad():
    t0 = time.time()
    bs = inputs.hydro_random_2d()
    target = inputs.hydro_target_density()
    _, cm = oracle.rhs(bs)
    dt = 0.4 / sum(cm[d] / bs.dx[0, d] for d in range(2))
    out, _ = oracle.run(bs, oracle.SSPRK54, 200, dt=dt)
    lam_n = []
    for b in range(bs.nb):
        x = np.zeros(bs.padded_shape(b))
        bs.interior(b, x)[0] = out.interior(b)[0] - target[b]
        lam_n.append(x)
    lam0 = oracle.run_vjp(bs, lam_n, oracle.SSPRK54, 200, dt)
    grad = np.stack([bs.interior(b, lam0[b]) for b in range(bs.nb)])
    meta = {"case": "c4grad", "scheme": "SSPRK(5,4)", "nsteps": 200, "dt": dt, "input_sha256": input_digest(bs),
            "oracle_threads": oracle.num_threads(), "seconds": round(time.time() - t0, 1)}
    np.savez(os.path.join(HERE, "fullsize_c4_grad200.npz"), grad=grad, meta=np.array(json.dumps(meta)))
    print(f"c4grad: wrote fullsize_c4_grad200.npz in {time.time() - t0:.0f} s", flush=True)


def make(name):
    if name == "c4grad":
        return make_c4grad()
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
    for name in (sys.argv[1:] or list(CASES) + ["c4grad"]):
        make(name)
