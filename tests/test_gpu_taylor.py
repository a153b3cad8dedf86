"""Capsule at a fluid-fluid interface (Sec. 4.1) on the GPU: FP64 parity
with the oracle on the paper's set-up (symmetric and asymmetric tensions),
and equilibrium Taylor deformations of a few cases against the
sharp-interface reference (tests/golden/taylor_sharp.json, written by
tests/golden/gen_taylor_sharp.py from oracle/sharp.py)."""
import json
import os

import numpy as np
import pytest

from helpers import compare, marker_err, run_gpu, run_oracle
from paper_1906_03065_amd import taylor as T
from paper_1906_03065_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "taylor_sharp.json")


@pytest.mark.parametrize("case", [(True, 5e-4, 1e-3, 1e-2), (False, 8e-3, 1e-1, 1e-4)])
def test_fp64_parity_taylor_setup(orc, case):
    sym, k3, ks, kb = case
    # off the lattice's symmetry lines: with a band wider than R, nodes on a
    # mirror line of the capsule are equidistant from two segments
    w = W.taylor2d(k3, ks, kb, symmetric=sym, offset=(0.37, 0.21))
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    for n in (1, 50):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o)
        print(f"taylor {case} step {n}", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
        for k, v in errs.items():
            assert v < 1e-9, (n, k, v)
        assert marker_err(g, o, 1) < 1e-9


def test_equilibrium_deformation_against_sharp_interface():
    """Five cases (both tension sets, stiff to soft) stepped as a batch in
    the divergence force form for 150 000 steps: D within 12 % of the
    sharp-interface value.  (The paper reports under 10 % against its
    finite-element model; the sharp reference here lets the contact points
    slide freely, and these runs are still relaxing slowly at 150 000 steps:
    the full sweeps reach a median difference of 6 % at 300 000.)"""
    ref = {(r["symmetric"], r["kappa3"], r["kappa_s"], r["kappa_b"]): r["D"]
           for r in json.load(open(GOLDEN))["runs"]}
    cases = [(True, 5e-4, 1e-1, 1e-4), (True, 5e-3, 1e-2, 1e-4), (True, 1e-2, 1e-3, 1e-2),
             (False, 5e-4, 1e-1, 1e-2), (False, 8e-3, 1e-3, 1e-4)]
    res = T.run_sweep(cases, max_steps=150000, log=True, force_form=1)
    assert res["check"] == 0
    for r, c in zip(res["runs"], cases):
        d_ref = ref[c]
        print(c, f"D {r['D']:.4f} sharp {d_ref:.4f} rel {r['D'] / d_ref - 1:+.3f}", flush=True)
        assert r["D"] == pytest.approx(d_ref, rel=0.12)
