"""Capillary bridge between two capsules (Sec. 4.2) on the GPU: the full
240 x 120 set-up against the FP64 oracle, and the batched sweep's runs kept
mirror-symmetric."""
import numpy as np
import pytest

from helpers import compare, marker_err, run_gpu, run_oracle
from paper_1906_03065_amd import bridge
from paper_1906_03065_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kappa1", [1e-3, 9e-3])
def test_fp64_parity_bridge(orc, kappa1):
    """Two capsules, the bridge of fluid 2, periodic in both directions, alpha
    2, band 24: the FP64 kernels match the oracle to round-off.  The set-up
    is shifted by (0.37, 0.21) of a node: centred on nodes, the capsule
    centres' exact ties between opposite segments would be decided by each
    side's rounding (both choices are correct)."""
    w = W.bridge2d(kappa1=kappa1, kappa_s=1e-2, offset=(0.37, 0.21))
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    for n in (1, 40):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o)
        print(f"fp64 bridge k1={kappa1} step {n}", {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
        for k, v in errs.items():
            assert v < 1e-9, (n, k, v)
        assert marker_err(g, o, 2) < 1e-9


def test_bridge_sweep_short_symmetric():
    """Two runs of the sweep (soft and stiff membrane) stepped as one batch
    for 6000 steps: the two capsules of each run keep the same aspect ratio
    (the set-up is a mirror image about x = 6R), the soft capsule deforms
    more than the stiff one, and the state check passes."""
    res = bridge.run_sweep(kappa1s=(9e-3,), kappa_ss=(1e-3, 1.0), max_steps=6000, every=500, window=2000,
                           tol=1e-12, log=False)
    assert res["check"] == 0
    soft, stiff = res["runs"]
    for r in (soft, stiff):
        assert abs(r["aspect_left"] - r["aspect_right"]) < 1e-4, r
    assert abs(soft["aspect_left"] - 1.0) > abs(stiff["aspect_left"] - 1.0)
