"""Learned warm start of 2D capsule-at-interface relaxations.

Parameter sets (kappa_1..3, shear and bending moduli, radius) map to the
equilibrium shape coefficients of the capsule (shape.py): the training data
come from batched runs of the solver to equilibrium, a small MLP (mlp.py,
hand-written HIP kernels) learns the map, and a warm-started run begins
from the predicted shape -- markers on the predicted curve, concentration
fields built around it, rest lengths those of the undeformed circle -- while
the cold start begins from the circle.  Equilibrium: the shape coefficients
drift by less than `tol` over the last 1000 steps (checked every 250
steps), or the step cap.
"""
from __future__ import annotations

import math

import numpy as np

from . import lbib, shape
from . import workloads as W

SEED = W.SEED_BASE + 4


def param_sets(count: int, seed: int = SEED) -> list:
    """The parameter distribution of the batched capsule workload: kappa_m
    U[0.01, 0.05], shear modulus log-U[1e-3, 1e-1], bending log-U[1e-5,
    1e-3], and the radius drawn as there, R ~ U[12, min(48, n/4)] with the
    lattice side n = 16 U_int[6, 32].  The run itself uses a lattice of side
    2R + 44 (rounded up to 16, side()), whose walls stand 22 nodes from the
    capsule: the side n only shapes the radius distribution."""
    g = W.rng(seed)
    out = []
    for _ in range(count):
        kap = g.uniform(0.01, 0.05, 3)
        ks = float(10 ** g.uniform(-3, -1))
        kb = float(10 ** g.uniform(-5, -3))
        n = 16 * int(g.integers(6, 33))
        R = float(g.uniform(12.0, min(48.0, 0.25 * n)))
        out.append(dict(kappa=[float(k) for k in kap], kappa_s=ks, kappa_b=kb, R=R))
    return out


def features(ps: dict) -> np.ndarray:
    """Network input: kappa_1..3, log10 kappa_s, log10 kappa_b, R."""
    return np.array([*ps["kappa"], math.log10(ps["kappa_s"]), math.log10(ps["kappa_b"]), ps["R"]])


def side(R: float) -> int:
    return int(16 * math.ceil((2.0 * R + 44.0) / 16.0))


def n_markers(R: float) -> int:
    return int(min(384, max(64, math.ceil(2 * math.pi * R / 0.8))))


def cold_workload(ps: dict, seed: int = 0) -> dict:
    n = side(ps["R"])
    w = W.capsule_at_interface(nx=n, ny=n, R=ps["R"], n_markers=n_markers(ps["R"]), kappa=ps["kappa"],
                               kappa_s=ps["kappa_s"], kappa_b=ps["kappa_b"], wall_y=1, mobility=0.1,
                               perturb=1e-4, seed=seed)
    w["R"] = ps["R"]
    return w


def warm_workload(ps: dict, coef: np.ndarray, seed: int = 0) -> dict:
    """The cold workload with the capsule (markers and C fields) reshaped to
    the shape coef; the rest lengths stay those of the circle."""
    w = cold_workload(ps, seed)
    p = w["params"]
    n, ny = p["nx"], p["ny"]
    R = ps["R"]
    m = w["membranes"][0]
    nm = len(m["X"])
    xc = n / 2.0
    y0 = (ny - 1) / 2.0
    X = shape.markers(np.asarray(coef, dtype=np.float64), R, xc, y0, nm)
    x, y = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(ny, dtype=np.float64))
    C3 = W.tanh_profile(shape.signed_distance(X, x, y), p["alpha"])
    below = 0.5 * (1.0 - np.tanh((y - y0) / (2.0 * p["alpha"])))
    C1 = (1.0 - C3) * below
    C2 = 1.0 - C1 - C3
    w["fields"] = W.fields_from_C(C1, C2, C3, 1e-4, seed)
    rest = np.full(nm, 2.0 * R * math.sin(math.pi / nm))
    w["membranes"] = [dict(X=X, tris=None, kappa_s=m["kappa_s"], kappa_b=m["kappa_b"], rest=rest)]
    w["name"] = "warm_" + w["name"]
    return w


def run_batched(workloads: list, max_steps: int, tol: float = 1e-3, every: int = 250,
                window: int = 1000, device="cuda:0", log: bool = True, retire: bool = True,
                batch_max: int = 256):
    """Run every workload in batches of up to batch_max members until its
    shape coefficients drift by less than tol over `window` steps, or
    max_steps.  With `retire`, a batch whose live members have fallen to half
    or less is rebuilt from them alone (each one's state carried over by a
    checkpoint), so members at equilibrium stop costing steps.  Returns
    (coefficients at equilibrium or at the cap, steps to equilibrium or -1,
    wall seconds per batch)."""
    import time

    coefs = [None] * len(workloads)
    steps = [-1] * len(workloads)
    walls = []
    for b0 in range(0, len(workloads), batch_max):
        idx = list(range(b0, min(b0 + batch_max, len(workloads))))
        meta = {i: dict(R=workloads[i]["R"], y0=(workloads[i]["params"]["ny"] - 1) / 2.0, hist=[]) for i in idx}
        t0 = time.perf_counter()
        b = lbib.Batch.from_workloads([workloads[i] for i in idx], device=device)
        members = list(idx)  # workload index of each batch member
        live = set(idx)
        step = 0
        rebuilds = 0
        while live and step < max_steps:
            b.step(every)
            step += every
            allx = b.markers()
            for k, i in enumerate(members):
                if i not in live:
                    continue
                c = shape.coefficients(allx[k][0], meta[i]["R"], meta[i]["y0"])
                h = meta[i]["hist"]
                h.append((step, c))
                while h and h[0][0] < step - window:
                    h.pop(0)
                coefs[i] = c
                if h[0][0] == step - window and np.abs(c - h[0][1]).max() < tol:
                    steps[i] = step
                    live.discard(i)
            if retire and live and 2 * len(live) <= len(members):
                keep = [k for k, i in enumerate(members) if i in live]
                blobs = [b[k].save() for k in keep]
                nb = lbib.Batch.from_workloads([workloads[members[k]] for k in keep], device=device)
                for j, blob in enumerate(blobs):
                    nb[j].load(blob)
                b.close()
                b = nb
                members = [members[k] for k in keep]
                rebuilds += 1
        b.synchronize()
        walls.append(time.perf_counter() - t0)
        b.close()
        if log:
            done = sum(steps[i] > 0 for i in idx)
            print(f"  batch {b0 // batch_max}: {len(idx)} runs, {done} at equilibrium, {walls[-1]:.1f} s, "
                  f"{rebuilds} rebuilds", flush=True)
    return coefs, steps, walls


def run_single(w: dict, max_steps: int, tol: float = 1e-3, every: int = 250, window: int = 1000,
               device="cuda:0"):
    """One simulation alone (its own handle) until equilibrium or the cap:
    (coefficients, steps or -1, wall seconds)."""
    import time

    import torch

    s = lbib.from_workload(w, device=device)
    R, y0 = w["R"], (w["params"]["ny"] - 1) / 2.0
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step, reached, c = 0, -1, None
    while step < max_steps:
        s.step(every)
        step += every
        c = shape.coefficients(s.membrane(0)["X"], R, y0)
        hist.append((step, c))
        while hist and hist[0][0] < step - window:
            hist.pop(0)
        if hist[0][0] == step - window and np.abs(c - hist[0][1]).max() < tol:
            reached = step
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.close()
    return c, reached, wall


def polygon_gap(A: np.ndarray, B: np.ndarray) -> float:
    """Largest distance from a vertex of A to polygon B."""
    P = B
    Q = np.roll(B, -1, axis=0)
    best = np.full(len(A), np.inf)
    for a, b in zip(P, Q):
        e = b - a
        t = np.clip(((A - a) @ e) / (e @ e), 0.0, 1.0)
        best = np.minimum(best, np.hypot(*(A - a - t[:, None] * e).T))
    return float(best.max())


def _gen_files(out: str) -> list:
    import glob
    import os

    return sorted(glob.glob(os.path.join(out, "gen_*.npz")))


def generate(first: int, count: int, cap: int, tol: float, out: str) -> str:
    """Cold runs of parameter sets [first, first + count) to equilibrium with
    the batched solver; their final coefficients and steps go to
    out/gen_<first>_<count>.npz."""
    import os
    import time

    ps = param_sets(first + count)[first:]
    ws = [cold_workload(p, seed=first + k) for k, p in enumerate(ps)]
    t0 = time.perf_counter()
    coefs, steps, walls = run_batched(ws, cap, tol)
    wall = time.perf_counter() - t0
    path = os.path.join(out, f"gen_{first:05d}_{count:05d}.npz")
    np.savez(path, first=first, X=np.array([features(p) for p in ps]), Y=np.array(coefs),
             steps=np.array(steps), wall=wall, nodes=np.array([w["params"]["nx"] * w["params"]["ny"] for w in ws]))
    print(f"generated sets {first}..{first + count - 1} in {wall:.1f} s, "
          f"{sum(s > 0 for s in steps)} at equilibrium -> {path}", flush=True)
    return path


def main():
    """Generate equilibria with the batched solver (in chunks), train the
    network on the device on the runs that reached equilibrium, and compare
    warm and cold starts on held-out parameter sets at equal batching."""
    import argparse
    import json
    import os
    import time

    from . import mlp

    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["generate", "train", "evaluate"])
    ap.add_argument("--train", type=int, default=4096)
    ap.add_argument("--test", type=int, default=256)
    ap.add_argument("--first", type=int, default=0, help="generate: first parameter set")
    ap.add_argument("--count", type=int, default=1024, help="generate: parameter sets in this chunk")
    ap.add_argument("--cap", type=int, default=30000)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--epochs", type=int, default=3000)
    ap.add_argument("--single", type=int, default=16, help="held-out sets also run alone (wall time)")
    ap.add_argument("--out", default="warmstart_out")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    if args.what == "generate":
        generate(args.first, args.count, args.cap, args.tol, args.out)
        return
    if args.what == "train":
        X, Y, S, wall = [], [], [], 0.0
        for f in _gen_files(args.out):
            d = np.load(f)
            first = int(d["first"])
            n = min(len(d["steps"]), max(0, args.train - first))
            X.append(d["X"][:n])
            Y.append(d["Y"][:n])
            S.append(d["steps"][:n])
            wall += float(d["wall"])
        X, Y, S = np.concatenate(X), np.concatenate(Y), np.concatenate(S)
        ok = S > 0  # equilibria only: runs that hit the step cap are left out
        model, hist = mlp.train(X[ok], Y[ok], epochs=args.epochs)
        model.save(os.path.join(args.out, "warmstart_mlp.npz"))
        info = {"train_sets": int(len(S)), "train_rows_at_equilibrium": int(ok.sum()), "generation_seconds": wall,
                "train_loss": hist[-1][1], "loss_history": hist, "epochs": args.epochs}
        json.dump(info, open(os.path.join(args.out, "warmstart_train.json"), "w"), indent=1)
        print(json.dumps({k: v for k, v in info.items() if k != "loss_history"}), flush=True)
        return
    # evaluate: held-out sets, warm and cold, each batched the same way
    model = mlp.WarmStartModel.load(os.path.join(args.out, "warmstart_mlp.npz"))
    ps_all = param_sets(args.train + args.test)
    test = list(range(args.train, args.train + args.test))
    ps = [ps_all[i] for i in test]
    X = np.array([features(p) for p in ps])
    pred = model.predict(X)
    cws = [cold_workload(p, seed=i) for p, i in zip(ps, test)]
    wws = [warm_workload(p, pred[k], seed=i) for k, (p, i) in enumerate(zip(ps, test))]
    t0 = time.perf_counter()
    wcoefs, wsteps, _ = run_batched(wws, args.cap, args.tol)
    t_warm = time.perf_counter() - t0
    t0 = time.perf_counter()
    ccoefs, csteps, _ = run_batched(cws, args.cap, args.tol)
    t_cold = time.perf_counter() - t0
    single = []
    for k in range(min(args.single, len(cws))):
        single.append(run_single(cws[k], args.cap, args.tol))
        print(f"  single run {k}: {single[-1][1]} steps, {single[-1][2]:.1f} s", flush=True)
    cs, wsx = np.array(csteps), np.array(wsteps)
    both = (cs > 0) & (wsx > 0)
    pred_err = np.abs(pred - np.array(ccoefs)).max(1)
    shape_err = np.abs(np.array(wcoefs) - np.array(ccoefs)).max(1)
    gaps = []
    for k, p in enumerate(ps):
        cw = cws[k]
        nm = len(cw["membranes"][0]["X"])
        xc, y0 = cw["params"]["nx"] / 2.0, (cw["params"]["ny"] - 1) / 2.0
        A = shape.markers(np.array(wcoefs[k]), p["R"], xc, y0, nm)
        B = shape.markers(np.array(ccoefs[k]), p["R"], xc, y0, nm)
        gaps.append(polygon_gap(A, B) / p["R"])
    R = np.array([p["R"] for p in ps])
    res = {
        "test": len(test), "cap": args.cap, "tol": args.tol, "radius_range": [float(R.min()), float(R.max())],
        "cold_steps_median": float(np.median(cs[cs > 0])) if (cs > 0).any() else None,
        "warm_steps_median": float(np.median(wsx[wsx > 0])) if (wsx > 0).any() else None,
        "cold_reached": int((cs > 0).sum()), "warm_reached": int((wsx > 0).sum()),
        "steps_ratio_median_both": float(np.median(wsx[both] / cs[both])) if both.any() else None,
        "warm_faster_of_both": int((wsx[both] < cs[both]).sum()), "both_reached": int(both.sum()),
        "cold_batched_seconds": t_cold, "warm_batched_seconds": t_warm,
        "wall_ratio_warm_over_cold_batched": t_warm / t_cold,
        "cold_single_seconds_per_run": float(np.mean([s_[2] for s_ in single])) if single else None,
        "cold_single_runs": len(single),
        "prediction_error_max_coef_median": float(np.median(pred_err)),
        "final_shape_error_max_coef_median": float(np.median(shape_err)),
        "final_shape_error_max_coef_p90": float(np.percentile(shape_err, 90)),
        "final_max_marker_distance_over_R_median": float(np.median(gaps)),
        "final_max_marker_distance_over_R_max": float(np.max(gaps)),
        "cold_steps": csteps, "warm_steps": wsteps,
    }
    with open(os.path.join(args.out, "warmstart_eval.json"), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps({k: v for k, v in res.items() if not isinstance(v, list)}), flush=True)


if __name__ == "__main__":
    main()
