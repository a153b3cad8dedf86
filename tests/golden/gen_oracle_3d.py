"""Write oracle_3d.json: observables of the FP64 oracle on the 64^3 D3Q19
drop and lens workloads, the reference of the 3D accuracy tests of the
16-bit population storage.  Calls only the oracle (inputs from the seeded
workload generators).

    python tests/golden/gen_oracle_3d.py      # a few minutes on 8 cores
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from helpers import lens_angles, pressure  # noqa: E402
from paper_1906_03065_amd import workloads as W  # noqa: E402

DROP = dict(n=64, R=16.0, steps=1500)
LENS = dict(n=64, R=16.0, mobility=0.5, steps=4000)
KAP = (0.02, 0.02, 0.02)


def drop_dp(fields, n):
    """Pressure in the central 4^3 block minus that in the corner 4^3 block
    (periodic box: the corners are the farthest from the drop)."""
    p = pressure(fields, KAP)
    c = n // 2
    return float(p[c - 2:c + 2, c - 2:c + 2, c - 2:c + 2].mean() - p[0:4, 0:4, 0:4].mean())


def lens_slice_angles(fields, n):
    """Cap angles of the lens in the plane y = (n-1)/2 (mean of the two
    middle planes), from circle fits to the C3 = 1/2 contour."""
    c3 = fields["c3"]
    mid = 0.5 * (c3[:, n // 2 - 1, :] + c3[:, n // 2, :])
    return [float(a) for a in lens_angles(mid, (n - 1) / 2.0)]


def run(w, steps):
    s = oracle.Sim(w["params"])
    f = w["fields"]
    s.set_fields(f["rho"], f["phi"], f["psi"], f.get("u"))
    s.step(steps)
    return s.fields()


def main():
    oracle.build(force=False)
    threads = oracle.set_threads(0)
    out = {"generator": "tests/golden/gen_oracle_3d.py", "threads": threads}
    f = run(W.sphere3d(n=DROP["n"], R=DROP["R"], kappa=KAP), DROP["steps"])
    out["drop"] = dict(DROP, dp=drop_dp(f, DROP["n"]), mass_c3=float(f["c3"].sum()))
    print("drop", out["drop"], flush=True)
    f = run(W.lens3d(n=LENS["n"], R=LENS["R"], kappa=KAP, mobility=LENS["mobility"]), LENS["steps"])
    out["lens"] = dict(LENS, angles=lens_slice_angles(f, LENS["n"]))
    print("lens", out["lens"], flush=True)
    with open(os.path.join(HERE, "oracle_3d.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
