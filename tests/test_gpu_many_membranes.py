"""A 2D simulation holding more membranes than a coupling workgroup has
lanes (300 small capsules, 256 lanes): the membranes beyond the first 256
reach each tile's list in a second pass.  FP64 parity with the oracle, and
bitwise the same results with the coupling cache on or off."""
import numpy as np
import pytest

from helpers import compare, marker_err, run_gpu, run_oracle
from paper_1906_03065_amd import workloads as W

pytestmark = pytest.mark.gpu


def _capsule_grid(cols=20, rows=15, spacing=20.0, R=2.5, n_markers=16, r_cut=3.0, seed=31):
    """cols x rows capsules of fluid 3 (radius R, n_markers each) on a flat
    C1/C2 interface, walls in y.  With r_cut = 3 a grown box reaches 6.5
    from a capsule's centre, and a tile takes a membrane whose grown box
    meets the square of half-width 8 sqrt 2 around its centre: with centres
    20 apart a tile takes at most two per axis, four in all (the most whose
    band data a tile keeps)."""
    nx, ny = int(cols * spacing), int(rows * spacing)
    g = np.random.default_rng(seed)
    p = W.base_params(nx, ny, wall_y=1, kappa=(0.02, 0.03, 0.015), alpha=1.0, kappa_c=0.01, r_cut=r_cut)
    x = np.arange(nx, dtype=np.float64)[None, :] * np.ones((ny, 1))
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    C3 = np.zeros((ny, nx))
    mem = []
    for j in range(rows):
        for i in range(cols):
            cx = (i + 0.5) * spacing + g.uniform(-0.3, 0.3)
            cy = (j + 0.5) * spacing + g.uniform(-0.3, 0.3)
            C3 += W.tanh_profile(R - np.hypot(x - cx, y - cy), 1.0)
            mem.append(dict(X=W.circle_markers(cx, cy, R, n_markers), tris=None, kappa_s=0.02, kappa_b=1e-4))
    below = 0.5 * (1.0 - np.tanh((y - 0.5 * (ny - 1)) / 2.0))
    C1 = (1.0 - C3) * below
    C2 = 1.0 - C1 - C3
    fields = W.fields_from_C(C1, C2, C3, 1e-4, seed)
    return dict(params=p, fields=fields, membranes=mem, name=f"capsule_grid_{nx}x{ny}")


def test_many_membranes_fp64_parity(orc):
    """300 membranes, FP64: fields and markers within 1e-9 of the oracle
    after one and four steps."""
    w = _capsule_grid()
    assert len(w["membranes"]) == 300
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    for n in (1, 4):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o)
        xe = marker_err(g, o, len(w["membranes"]))
        print(f"300 membranes fp64 step {n}", {k: f"{v:.2e}" for k, v in errs.items()}, f"markers {xe:.2e}",
              flush=True)
        for k, v in errs.items():
            assert v < 1e-9, (n, k, v)
        assert xe < 1e-9
    assert g.check() == 0


def test_many_membranes_cache_bitwise():
    """300 membranes, FP32, 30 steps: the coupling cache changes nothing."""
    w = _capsule_grid(seed=32)
    a = run_gpu(w, "fp32")
    b = run_gpu(w, "fp32")
    b.set_coupling_cache(0)
    a.step(30)
    b.step(30)
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    for i in range(len(w["membranes"])):
        for q in ("X", "U", "F"):
            assert np.array_equal(a.membrane(i)[q], b.membrane(i)[q]), (i, q)
    assert a.check() == 0
