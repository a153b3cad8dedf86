"""Benchmark of the ternary LB + IBM step on one MI355X.

Workload (default): 2048 x 2048 D2Q9 in FP32, walls in y, a flat C1/C2
interface carrying 16 capsules of radius 24..64 with 256..512 markers each,
kappa_m uniform in [0.01, 0.05] (seeded).  A step is one pass of the whole
method: coupling profile and forces, membrane forces, spreading, the fused
lattice kernel, interpolation and marker update.  Inputs are resident in HBM
before the timed region.

With --workload c3: 256^3 D3Q19 in FP32 (or 16-bit storage), walls in z,
two icosphere capsules of radius 40 (5120 triangles each) bridged by C2 on a
flat C1/C2 interface.

With --workload c4: 64 capsule-at-interface D2Q9 runs of seeded sizes
96^2..512^2 (FP32) stepped as one batch (one launch per phase, the step
replayed from a hipGraph, lattice-kernel shapes from the autotuner), against
the same 64 simulations stepped one after another.

Prints one JSON line: whole-step MLUPS, the lattice update's HBM roofline
fraction (algorithmic bytes / kernel time from HIP events on the library's
stream over the timed region; 216 B per update for D2Q9 FP32, the bytes the
storage format actually moves reported beside it) and the CPU oracle's rate
on a bounded sample of the same workload, on all host threads and on one.
D2Q9 runs take the divergence form of the force (the library's default)
unless --force-form 0 asks for the potential form.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_lb2d_d2q9_2048_traffic.json")


def measured_traffic(storage: str, size: int, force_form: int):
    """HBM bytes per fused-kernel launch from the committed rocprofv3 counter
    runs (FETCH_SIZE, WRITE_SIZE scaled by a plain copy), or None when the
    kernel sources changed since they were taken or the workload differs."""
    import hashlib

    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    src = b"".join(open(os.path.join(ROOT, "paper_1906_03065_amd", "csrc", f), "rb").read()
                   for f in ("k_lb.h", "store.h"))
    if hashlib.sha256(src).hexdigest()[:16] != rec.get("source_sha256_16"):
        return None
    if storage != "fp32" or size != 2048 or force_form != rec.get("force_form", 0):
        return None
    return rec["traffic_bytes_per_launch"]


def alg_bytes_per_lup(storage: str, Q: int = 9) -> int:
    """Algorithmic bytes per lattice update: the three population sets read
    once and written once, 4 bytes per population in FP32, 8 in FP64, and 2
    per moving population plus 4 per rest population in the 16-bit formats
    (216 B for D2Q9 FP32, 456 B for D3Q19 FP32)."""
    if storage == "fp32":
        return 2 * 3 * Q * 4
    if storage == "fp64":
        return 2 * 3 * Q * 8
    return 2 * (3 * (Q - 1) * 2 + 3 * 4)


def stored_bytes_per_lup(storage: str, Q: int = 9) -> int:
    """Bytes per lattice update the storage format actually moves: the FP32
    format keeps g_0 and h_0 in FP64 (232 B for D2Q9), the 16-bit formats
    keep f_0 in FP32 and g_0, h_0 in FP64 (136 B for D2Q9)."""
    if storage == "fp32":
        return 2 * ((3 * Q - 2) * 4 + 2 * 8)
    if storage == "fp64":
        return 2 * 3 * Q * 8
    return 2 * (3 * (Q - 1) * 2 + 4 + 2 * 8)


def host_info() -> dict:
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def cpu_baseline(w, budget_s: float, note: str = "", single_s: float = 8.0):
    """The oracle as it stands, on the given lattice, for about budget_s on
    all the host threads it uses, then for about single_s on one thread."""
    import oracle

    oracle.build(force=False)
    # the same coupling band as the library's run (the oracle's r_cut <= 0
    # would mean no band at all)
    po = dict(w["params"])
    if po.get("r_cut", 0.0) <= 0.0:
        po["r_cut"] = 17.0 * po.get("alpha", 1.0)

    def timed(threads, budget):
        used = oracle.set_threads(threads)
        s = oracle.Sim(po)
        for m in w["membranes"]:
            s.add_membrane(m["X"], m.get("tris"), m["kappa_s"], m["kappa_b"])
        f = w["fields"]
        s.set_fields(f["rho"], f["phi"], f["psi"], f.get("u"))
        n = 0
        t0 = time.perf_counter()
        while True:
            s.step(1)
            n += 1
            el = time.perf_counter() - t0
            if el >= budget or n >= 200:
                break
        return s.N * n / el / 1e6, n, el, used

    p = w["params"]
    dims = f"{p['nx']}x{p['ny']}" + (f"x{p['nz']}" if p.get("lattice", 0) == 1 else "")
    v, n, el, threads = timed(0, budget_s)
    v1, n1, el1, _ = timed(1, single_s)
    oracle.set_threads(0)
    return {"value": v, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{n} full steps of the {note or 'same'} {dims} workload "
                      f"({el:.1f} s, FP64, {threads} OpenMP threads)",
            "single_thread": {"value": v1, "unit": "MLUPS", "cores": 1,
                              "sample": f"{n1} full steps of the same ({el1:.1f} s, FP64, 1 thread)"},
            "host": host_info()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16", "bf16", "fp64"])
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4"],
                    help="c2: 2048^2 D2Q9 with 16 capsules; c3: 256^3 D3Q19 with two capsules; "
                         "c4: batch of 64 D2Q9 capsule runs")
    ap.add_argument("--size", type=int, default=0, help="lattice side (default 2048 / 256)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--block-x", type=int, default=0, help="fused kernel lanes per workgroup")
    ap.add_argument("--seg", type=int, default=0, help="fused kernel rows per workgroup")
    ap.add_argument("--nxcd", type=int, default=0, help="L2 domains workgroups are dealt to")
    ap.add_argument("--ring", type=int, default=0, help="register ring depth (3 or 4)")
    ap.add_argument("--overlap-steps", type=int, default=-1,
                    help="D2Q9: steps timed afterwards with the overlapped step order (default "
                         "steps/4; 0 skips them, e.g. for a profile of the single-stream kernel)")
    ap.add_argument("--force-form", type=int, default=1, choices=[0, 1],
                    help="D2Q9: thermodynamic force in divergence (1, the default) or potential (0) form")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (source + destination "
                         "traffic 2*MIB MiB per launch), --steps times, to scale counters")
    args = ap.parse_args()
    if args.calib_copy:
        import torch

        a = torch.empty(args.calib_copy * (1 << 20) // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_mib": args.calib_copy, "launches": args.steps}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "domain decomposition is a design, not part of this build", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c4":
        bench_batch(args)
        return

    import torch

    from paper_1906_03065_amd import lbib
    from paper_1906_03065_amd import workloads as W

    d3 = args.workload == "c3"
    size = args.size or (256 if d3 else 2048)
    w = W.c3(n=size) if d3 else W.c2(n=size)
    form = 0 if d3 else args.force_form  # D3Q19 has the potential form only
    w["params"]["force_form"] = form
    g = lbib.from_workload(w, storage=args.storage, device="cuda:0")
    g.set_launch(args.block_x, args.seg, args.nxcd, args.ring)
    N = g.N
    g.step(args.warmup)
    torch.cuda.synchronize()
    g.timing(1)  # HIP events around the fused lattice kernel only
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = g.timing_read()
    g.timing(0)
    rc = g.check()
    if rc != 0:
        print(f"state check failed after the run: {lbib.STATUS.get(rc, rc)}", file=sys.stderr)
        sys.exit(3)
    el = t1 - t0
    mlups = N * args.steps / el / 1e6
    lb_ms = tm["lb"] / max(tm["steps"], 1)
    Q = 19 if d3 else 9
    bpl = alg_bytes_per_lup(args.storage, Q)
    stored = stored_bytes_per_lup(args.storage, Q)
    achieved = bpl * N / (lb_ms * 1e-3) / 1e9
    out = {
        "metric": "MLUPS & % HBM roofline; wall time to equilibrium, warm-start vs plain",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el * 1e3 / args.steps, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": (f"D3Q19 {size}^3, walls in z, two icosphere capsules (R {size / 6.4:g}, "
                                f"{len(w['membranes'][0]['tris'])} triangles each) bridged by C2, "
                                f"flat C1/C2 interface, {args.storage} populations" if d3 else
                                f"D2Q9 {size}x{size}, walls in y, 16 capsules "
                                f"(R 24-64, {sum(len(m['X']) for m in w['membranes'])} markers), "
                                f"flat C1/C2 interface, {args.storage} populations"),
                   "force_form": "divergence" if form else "potential",
                   "nodes": N, "capsules": len(w["membranes"]),
                   "markers": sum(len(m["X"]) for m in w["membranes"])},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if d3 else measured_traffic(args.storage, size, form),
                     "kernel": "k_mom3d + k_lb3d" if d3 else "k_lb2d", "kernel_ms": round(lb_ms, 5),
                     "bytes_per_lup": bpl,
                     "stored_bytes_per_lup": stored,
                     "achieved_stored": round(stored * N / (lb_ms * 1e-3) / 1e9, 1),
                     "kernel_share_of_step": round(lb_ms / (el * 1e3 / args.steps), 4),
                     "launch": g.get_launch()},
    }
    k2 = max(args.steps // 4, 1) if args.overlap_steps < 0 else args.overlap_steps
    if not d3 and k2 > 0:
        # the same lattice with the regions away from the membranes on a second
        # stream beside the membrane kernels (a scheduling option, bitwise the
        # same results); the roofline above stays the single-stream kernel's
        g.set_overlap(1)
        g.step(max(args.warmup // 4, 1))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        g.step(k2)
        torch.cuda.synchronize()
        el2 = time.perf_counter() - t2
        g.set_overlap(0)
        out["overlap_on"] = {"value": round(N * k2 / el2 / 1e6, 2), "unit": "MLUPS",
                             "ms_per_step": round(el2 * 1e3 / k2, 6), "steps": k2,
                             "what": "lattice regions away from the membranes on a second stream beside "
                                     "the membrane kernels (lbib_set_overlap)"}
    if not args.no_cpu:
        if d3:
            # the oracle's brute-force mesh distances make a 256^3 step take
            # minutes: time it on the same workload generated at 64^3
            out["cpu_baseline"] = cpu_baseline(W.c3(n=64), args.cpu_seconds, "same two-capsule")
        else:
            out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """Batched c4 workload: aggregate MLUPS of the batch and of the same 64
    simulations stepped one after another."""
    import torch

    from paper_1906_03065_amd import autotune, lbib
    from paper_1906_03065_amd import workloads as W

    ws = W.c4()
    NT = sum(w["params"]["nx"] * w["params"]["ny"] for w in ws)
    tuned = autotune.tune(ws, steps=20)  # untimed; cached per GPU architecture
    b = lbib.Batch.from_workloads(ws)
    autotune.apply(b, tuned)
    b.step(args.warmup)
    b.synchronize()
    t0 = time.perf_counter()
    b.step(args.steps)
    b.synchronize()
    el = time.perf_counter() - t0
    graph = b.graph()
    rc = b.check()
    if rc != 0:
        print(f"state check failed after the run: {lbib.STATUS.get(rc, rc)}", file=sys.stderr)
        sys.exit(3)
    shapes = {c: b.get_launch(c) for c in range(3)}
    b.close()
    del b
    # the same simulations, each its own handle, stepped one after another
    sims = [lbib.from_workload(w) for w in ws]
    for s in sims:
        s.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for s in sims:
            s.step(1)
    torch.cuda.synchronize()
    el_seq = time.perf_counter() - t0
    mlups = NT * args.steps / el / 1e6
    mlups_seq = NT * args.steps / el_seq / 1e6
    bpl = alg_bytes_per_lup("fp32")
    achieved = bpl * NT / (el / args.steps) / 1e9
    out = {
        "metric": "MLUPS & % HBM roofline; wall time to equilibrium, warm-start vs plain",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el * 1e3 / args.steps, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"batch of {len(ws)} D2Q9 capsule-at-interface runs, sides 96..512, "
                               f"{NT} nodes in total, fp32 populations, one launch per phase, "
                               f"hipGraph replay {'on' if graph else 'off'}",
                   "nodes": NT, "members": len(ws), "tuned_shapes": shapes},
        "sequential": {"value": round(mlups_seq, 2), "unit": "MLUPS",
                       "ms_per_step": round(el_seq * 1e3 / args.steps, 6),
                       "what": "the same 64 simulations as separate handles, stepped one after another"},
        "speedup_vs_sequential": round(mlups / mlups_seq, 3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "whole batched step (all phases)", "bytes_per_lup": bpl},
    }
    if not args.no_cpu:
        big = max(ws, key=lambda w: w["params"]["nx"] * w["params"]["ny"])
        out["cpu_baseline"] = cpu_baseline(big, args.cpu_seconds, "largest member's")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
