"""Write the operation-count records of the stage (the operation figures of
the rooflines), counted by the oracle.

    python oracle/count_ops.py

Runs one SSPRK(5,4) step of the oracle with its counting scalar on 64 blocks
of the 4096-block uneven 3D MHD list (32^3:16^3:8^3 = 9:18:37, the list's
size mix), once with MP5's published early exit and once in its median form
(no early exit; the same values for eps = 0), and forms per-unit averages:
one cell's primitive recovery, flux and split along one direction; one
reconstruction (with its share of the pair sum); one cell-variable-direction
of the conservative difference; one cell's c_max contribution; one cell's
stage combination.  The method's work per cell and stage is then

    ndim x (flux unit + 2 nvar x reconstruction unit + nvar x difference unit)
    + stage unit + c_max unit

(each cell's flux evaluated once per direction, one interface per cell and
direction), counted as arithmetic operations (+, -, *, /, sqrt; the oracle
forms no fused multiply-add) and, separately, as comparisons and selections
(min, max, minmod, median, |x|, branch tests).  The same counts are taken
on 16 blocks of the 256^3 periodic 3D MHD list, on the 2D Euler 256^2 list
and on the 2D MHD 512^2 list.  Writes profiles/oracle_op_count_mhd3d_uneven4096.json, read by
bench.py.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1407_2052_amd import inputs  # noqa: E402

OUT = os.path.join(ROOT, "profiles", "oracle_op_count_mhd3d_uneven4096.json")


def sample_blocks(bs, counts=(9, 18, 37), seed=11):
    rng = np.random.default_rng(seed)
    sizes = bs.n[:, 0]
    idx = []
    for s, k in zip((32, 16, 8), counts):
        pool = np.where(sizes == s)[0]
        idx.extend(rng.choice(pool, k, replace=False).tolist())
    idx = np.array(sorted(idx))
    sub = bs.copy()
    sub.u = [bs.u[i] for i in idx]
    sub.n, sub.dx, sub.xlo, sub.nbr = bs.n[idx], bs.dx[idx], bs.xlo[idx], bs.nbr[idx]
    return sub


def per_cell_stage(c, ndim, nvar):
    unit = {k: {"ops": v["ops"] / v["units"], "cmp": v["cmp"] / v["units"]} for k, v in c.items() if v["units"]}
    out = {}
    for kind in ("ops", "cmp"):
        out[kind] = (ndim * (unit["flux"][kind] + 2 * nvar * unit["recon"][kind] + nvar * unit["diff"][kind])
                     + unit["stage"][kind] + unit["cmax"][kind])
    return unit, out


def record(bs, workload, sample):
    rec = {"workload": workload, "sample": sample, "per_cell_stage": {}, "units": {}}
    for form, median in (("early_exit", False), ("median_form", True)):
        c = oracle.count_ops(bs, oracle.SSPRK54, median_form=median)
        unit, tot = per_cell_stage(c, bs.ndim, bs.nvar)
        rec["per_cell_stage"][form] = {"flops": round(tot["ops"], 1), "comparisons": round(tot["cmp"], 1)}
        rec["units"][form] = {k: {"flops": round(v["ops"], 3), "comparisons": round(v["cmp"], 3)}
                              for k, v in unit.items()}
        rec["units"][form]["counts"] = {k: v["units"] for k, v in c.items()}
        print(workload[:40], form, rec["per_cell_stage"][form], flush=True)
    return rec


def main():
    out = {"convention": "arithmetic ops: +, -, *, /, sqrt one each (no fused multiply-add in the oracle); "
                         "comparisons and selections counted apart; per cell and stage = ndim x (flux unit + "
                         "2 nvar x reconstruction unit + nvar x difference unit) + stage unit + c_max unit"}
    bs = sample_blocks(inputs.uneven_3d())
    out["mhd3d_uneven4096"] = record(bs, "3D ideal MHD, 4096 uneven blocks 32^3:16^3:8^3, SSPRK(5,4) + MP5",
                                     f"{bs.nb} blocks (9:18:37), {bs.interior_cells()} cells, one step")
    full = inputs.mhd_turbulence_3d(N=64, block=16)
    out["mhd3d_periodic256"] = record(full, "3D ideal MHD, 256^3 periodic in 16^3 blocks, SSPRK(5,4) + MP5",
                                      "the same recipe on 64^3 (64 blocks of 16^3), one step")
    h2 = inputs.hydro_random_2d()
    out["euler2d_256"] = record(h2, "2D Euler, 256^2 periodic in 16^2 blocks, SSPRK(5,4) + MP5",
                                f"the whole list ({h2.interior_cells()} cells), one step")
    ot = inputs.orszag_tang_2d(512, 16)
    out["mhd2d_512"] = record(ot, "2D ideal MHD, smooth Orszag-Tang data, 512^2 periodic in 16^2 blocks, "
                                  "SSPRK(5,4) + MP5", f"the whole list ({ot.interior_cells()} cells), one step")
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
