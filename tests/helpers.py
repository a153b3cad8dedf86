"""Shared helpers of the GPU parity tests: run the oracle and the HIP
library on the same seeded workload and compare."""
import numpy as np

FIELDS = ("rho", "c1", "c2", "c3", "ux", "uy")


def normwise(a, b):
    """max |a - b| / max |b| (the field error measure of the parity bar)."""
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def run_oracle(orc, w):
    s = orc.Sim(w["params"])
    for m in w["membranes"]:
        s.add_membrane(m["X"], m.get("tris"), m["kappa_s"], m["kappa_b"])
    f = w["fields"]
    s.set_fields(f["rho"], f["phi"], f["psi"], f.get("u"))
    return s


def run_gpu(w, storage="fp32", **kw):
    from paper_1906_03065_amd import lbib

    return lbib.from_workload(w, storage=storage, **kw)


def compare(g, o, D=2):
    fg, fo = g.fields(), o.fields()
    keys = FIELDS if D == 2 else FIELDS + ("uz",)
    return {k: normwise(fg[k], fo[k]) for k in keys}


def marker_err(g, o, n_mem):
    e = 0.0
    for i in range(n_mem):
        e = max(e, float(np.abs(g.membrane(i)["X"] - o.membrane(i)["X"]).max()))
    return e
