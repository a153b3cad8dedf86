"""What the trained warm-start network gains over the plain method: on
held-out parameter sets (never seen in training), runs started from the
predicted shape reach the equilibrium criterion in fewer steps than runs
started from the circle, and settle to nearby shapes.  The network was
trained by the project's own kernels on equilibria from the batched solver
(paper_1906_03065_amd/data/warmstart_mlp.npz, written by
`python -m paper_1906_03065_amd.warmstart`)."""
import os

import numpy as np
import pytest

from paper_1906_03065_amd import mlp, shape
from paper_1906_03065_amd import warmstart as WS

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1906_03065_amd",
                       "data", "warmstart_mlp.npz")
TRAIN = 4096  # the first parameter sets of the seeded stream were the training set


def test_warm_start_beats_cold_start():
    model = mlp.WarmStartModel.load(WEIGHTS)
    ps = WS.param_sets(TRAIN + 24)[TRAIN:]
    X = np.array([WS.features(p) for p in ps])
    pred = model.predict(X)
    cold = [WS.cold_workload(p, seed=TRAIN + k) for k, p in enumerate(ps)]
    warm = [WS.warm_workload(p, pred[k], seed=TRAIN + k) for k, p in enumerate(ps)]
    cc, cs, _ = WS.run_batched(cold, 24000)
    wc, wsx, _ = WS.run_batched(warm, 24000)
    cs, wsx = np.array(cs), np.array(wsx)
    cap = 24000
    cs_c = np.where(cs > 0, cs, cap)
    ws_c = np.where(wsx > 0, wsx, cap)
    print("cold", cs.tolist(), "\nwarm", wsx.tolist(), flush=True)
    # steps to equilibrium (runs that hit the cap count as the cap)
    assert np.median(ws_c) < 0.75 * np.median(cs_c)
    assert (wsx > 0).sum() >= (cs > 0).sum()
    # the network's prediction is close to the cold run's final shape
    perr = np.abs(pred - np.array(cc)).max(1)
    print("prediction error (max |coef|) median", np.median(perr), flush=True)
    assert np.median(perr) < 0.03
    # and the two starts settle to nearby shapes (a few per cent of R)
    gaps = []
    for k, p in enumerate(ps):
        w = cold[k]
        n = len(w["membranes"][0]["X"])
        xc, y0 = w["params"]["nx"] / 2.0, (w["params"]["ny"] - 1) / 2.0
        A = shape.markers(np.array(wc[k]), p["R"], xc, y0, n)
        B = shape.markers(np.array(cc[k]), p["R"], xc, y0, n)
        gaps.append(WS.polygon_gap(A, B) / p["R"])
    print("final gap / R median", np.median(gaps), "max", np.max(gaps), flush=True)
    assert np.median(gaps) < 0.08
