"""Unequal mobilities on the GPU (Sec. 2.6 names M_phi = 3 M_psi): the decay
rates of small sinusoidal phi and psi perturbations in a bulk phase against
the linearised Cahn-Hilliard closed form, and FP64 parity with the oracle on
a capsule at an interface with M_phi = 3 M_psi and relaxation times != 1."""
import pytest

from helpers import ch_rate, compare, decay_rate, marker_err, run_gpu, run_oracle
from paper_1906_03065_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage,amp,tol", [("fp64", 1e-5, 2e-3), ("fp32", 1e-3, 5e-3)])
@pytest.mark.parametrize("mode", ["phi", "psi"])
@pytest.mark.parametrize("mob", [(0.3, 0.1), (0.1, 0.3)])
def test_mode_decay_rates(storage, amp, tol, mode, mob):
    w = W.mode_decay(mode, mobility=mob, amp=amp)
    r = decay_rate(run_gpu(w, storage), mode)
    pred = ch_rate(w["params"], mode)
    print(storage, mode, mob, f"rate {r:.6e} closed form {pred:.6e} ratio {r / pred:.5f}", flush=True)
    assert r == pytest.approx(pred, rel=tol)


@pytest.mark.parametrize("wall_y", [0, 1])
def test_fp64_parity_unequal_mobilities(orc, wall_y):
    w = W.capsule_at_interface(nx=150, ny=83, R=12.0, n_markers=72, centre=(40.3, 41.2), wall_y=wall_y,
                               tau=0.9, tau_phi=0.8, tau_psi=1.3, mobility=(0.3, 0.1),
                               kappa=(0.02, 0.03, 0.015), seed=12)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    o.step(100)
    g.step(100)
    errs = compare(g, o)
    print(f"fp64 M_phi = 3 M_psi wall={wall_y}", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v < 1e-9, (k, v)
    assert marker_err(g, o, 1) < 1e-9
