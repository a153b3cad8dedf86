"""Capsule at a fluid-fluid interface (Sec. 4.1): Taylor deformation sweeps.

The capsule of Sec. 4.1 (R = 20 in a periodic 12R x 6R box, alpha 2,
kappa_c 1e-2) relaxes to its mechanical equilibrium under its strain and
bending energies and the three surface tensions.  The paper sweeps kappa_3
in a symmetric (kappa_1 = kappa_2 = 8e-3) and an asymmetric (kappa_1 = 8e-3,
kappa_2 = 2e-3) case for six (kappa_s, kappa_b) pairs and reports the Taylor
deformation D = (L - B) / (L + B), L and B the major and minor axes.  All
runs step together as one batch on the GPU until D changes by less than a
tolerance over a window of steps.

    python -m paper_1906_03065_amd.taylor [--stride S] [--max-steps N] [--out FILE]
    python -m paper_1906_03065_amd.taylor --compare SWEEP.json REFERENCE.json

The second form prints, for every case of a sweep's output, D against the D
of the same case in a reference file of the same layout (a list `runs` of
records with symmetric, kappa3, kappa_s, kappa_b and D).
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import lbib
from . import workloads as W


def taylor_deformation(X: np.ndarray) -> float:
    """D = (L - B) / (L + B) of a closed polygon: L and B are its extents
    along the principal axes of the area's second moment (the axes of the
    equivalent ellipse)."""
    P = np.asarray(X, dtype=np.float64)[:, :2]
    Q = np.roll(P, -1, axis=0)
    # triangle fan from the origin: signed areas and their moments
    a = 0.5 * (P[:, 0] * Q[:, 1] - Q[:, 0] * P[:, 1])
    A = a.sum()
    c = (a[:, None] * (P + Q)).sum(0) / (3.0 * A)
    P, Q = P - c, Q - c
    a = 0.5 * (P[:, 0] * Q[:, 1] - Q[:, 0] * P[:, 1])
    # second moment of a triangle (0, p, q): a/6 (p p^T + q q^T + (p q^T + q p^T)/2)
    M = np.zeros((2, 2))
    for i in range(2):
        for j in range(2):
            M[i, j] = (a * (P[:, i] * P[:, j] + Q[:, i] * Q[:, j] + 0.5 * (P[:, i] * Q[:, j] + Q[:, i] * P[:, j]))).sum() / 6.0
    _, V = np.linalg.eigh(M)
    proj = P @ V
    ext = proj.max(0) - proj.min(0)
    L, B = float(ext.max()), float(ext.min())
    return (L - B) / (L + B)


def case_list(stride: int = 1, which: str = "both"):
    """(symmetric, kappa_3, kappa_s, kappa_b) of the sweeps, every stride-th
    kappa_3."""
    out = []
    sets = []
    if which in ("both", "sym"):
        sets.append((True, W.TAYLOR_KAPPA3_SYM))
    if which in ("both", "asym"):
        sets.append((False, W.TAYLOR_KAPPA3_ASYM))
    for sym, k3s in sets:
        for k3 in k3s[::stride]:
            for ks, kb in W.TAYLOR_MODULI:
                out.append((sym, k3, ks, kb))
    return out


def run_sweep(cases, max_steps: int = 100000, every: int = 1000, window: int = 20000, tol: float = 1e-4,
              device="cuda:0", log: bool = True, force_form: int = 1):
    """Step all cases as one batch for max_steps steps.  A run counts as at
    equilibrium from the first check at which its D has changed by less than
    tol over the last `window` steps; every run is measured to the end."""
    ws = [W.taylor2d(k3, ks, kb, symmetric=sym) for sym, k3, ks, kb in cases]
    for w in ws:
        w["params"]["force_form"] = int(force_form)
    nodes = sum(w["params"]["nx"] * w["params"]["ny"] for w in ws)
    b = lbib.Batch.from_workloads(ws, device=device)
    hist = [[] for _ in ws]
    trace = [[] for _ in ws]  # D every 10 checks
    eq_step = [-1] * len(ws)
    D = [None] * len(ws)
    live = set(range(len(ws)))
    step = 0
    t0 = time.perf_counter()
    while step < max_steps:
        b.step(every)
        step += every
        allx = b.markers()
        for k in range(len(ws)):
            D[k] = taylor_deformation(allx[k][0])
            if step % (10 * every) == 0:
                trace[k].append(round(D[k], 6))
            h = hist[k]
            h.append((step, D[k]))
            while h and h[0][0] < step - window:
                h.pop(0)
            if k in live and h[0][0] == step - window and abs(D[k] - h[0][1]) < tol:
                eq_step[k] = step
                live.discard(k)
        if log and step % (20 * every) == 0:
            print(f"  step {step}: {len(ws) - len(live)} of {len(ws)} at equilibrium", flush=True)
    b.synchronize()
    wall = time.perf_counter() - t0
    rc = b.check()
    X = b.markers()
    b.close()
    out = []
    for k, (sym, k3, ks, kb) in enumerate(cases):
        k1, k2, _ = ws[k]["params"]["kappa"]
        out.append(dict(symmetric=sym, kappa3=k3, kappa_s=ks, kappa_b=kb, D=D[k], equilibrium_step=eq_step[k],
                        g12_g13=(k1 + k2) / (k1 + k3), g13_g23=(k1 + k3) / (k2 + k3), D_every=10 * every,
                        D_trace=trace[k],
                        X=[[round(float(a), 6), round(float(c), 6)] for a, c in X[k][0][:, :2]]))
    return dict(runs=out, steps_run=step, wall_s=wall, check=int(rc), nodes=nodes,
                mlups=nodes * step / wall / 1e6, tol=tol, window=window, force_form=int(force_form))


def compare(sweep: dict, reference: dict):
    """Per-case relative difference of D between two result files; returns
    the rows and a summary per tension set."""
    key = lambda r: (bool(r["symmetric"]), round(float(r["kappa3"]), 6), float(r["kappa_s"]), float(r["kappa_b"]))
    ref = {key(r): r["D"] for r in reference["runs"]}
    rows = []
    for r in sweep["runs"]:
        d_ref = ref.get(key(r))
        if d_ref is not None:
            rows.append(key(r) + (r["D"], d_ref, r["D"] / d_ref - 1.0))
    summ = {}
    for sym in (True, False):
        e = np.array([abs(x[6]) for x in rows if x[0] == sym])
        if e.size:
            summ["sym" if sym else "asym"] = dict(cases=int(e.size), median=float(np.median(e)),
                                                  mean=float(e.mean()), max=float(e.max()),
                                                  within_10pct=int((e < 0.10).sum()))
    return rows, summ


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--compare", nargs=2, metavar=("SWEEP", "REFERENCE"))
    ap.add_argument("--stride", type=int, default=1, help="every stride-th kappa_3 of each sweep")
    ap.add_argument("--which", default="both", choices=["both", "sym", "asym"])
    ap.add_argument("--max-steps", type=int, default=100000)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--window", type=int, default=20000)
    ap.add_argument("--force-form", type=int, default=1, choices=[0, 1])
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    if a.compare:
        rows, summ = compare(json.load(open(a.compare[0])), json.load(open(a.compare[1])))
        for x in rows:
            print(f"{'sym ' if x[0] else 'asym'} k3 {x[1]:.4f} ks {x[2]:6g} kb {x[3]:6g}  D {x[4]:.4f}  "
                  f"reference {x[5]:.4f}  rel {x[6]:+.3f}")
        print(json.dumps(summ))
        return
    res = run_sweep(case_list(a.stride, a.which), max_steps=a.max_steps, tol=a.tol, window=a.window,
                    force_form=a.force_form)
    for r in res["runs"]:
        print(f"{'sym ' if r['symmetric'] else 'asym'} k3 {r['kappa3']:.4f} ks {r['kappa_s']:6g} "
              f"kb {r['kappa_b']:6g}  D {r['D']:.5f}  equilibrium at step {r['equilibrium_step']}", flush=True)
    print(f"{res['steps_run']} steps of {len(res['runs'])} runs in {res['wall_s']:.1f} s "
          f"({res['mlups']:.0f} MLUPS), check {res['check']}", flush=True)
    if a.out:
        json.dump(res, open(a.out, "w"))


if __name__ == "__main__":
    main()
