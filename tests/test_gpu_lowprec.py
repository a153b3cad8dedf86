"""16-bit population storage (moving populations in half or bfloat16 with
the weights subtracted, rest populations in FP32): mass conservation and the
observables against the FP64 oracle, as the bar for reduced precision asks
(contact angle within 0.5 degrees, Laplace pressure within 1 %)."""
import numpy as np
import pytest

from helpers import lens_angles, normwise, pressure, run_gpu, run_oracle
from paper_1906_03065_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_mass_conservation_16bit(storage):
    """The rounding of the moving populations goes into the rest population
    of the same node, so the masses stay fixed to FP32 round-off."""
    w = W.c1()
    g = run_gpu(w, storage)
    m0 = np.array(g.energy()["mass"])
    g.step(500)
    m1 = np.array(g.energy()["mass"])
    print(storage, "mass drift", (m1 - m0) / m0, flush=True)
    assert np.abs((m1 - m0) / m0).max() < 1e-6


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_laplace_pressure_16bit(orc, storage):
    """Drop of C3 in C1: the pressure jump of the 16-bit run is within 1 % of
    the FP64 oracle's."""
    kap = (0.02, 0.02, 0.02)
    w = W.drop(n=64, R=12.0, kappa=kap, alpha=1.0)
    o = run_oracle(orc, w)
    g = run_gpu(w, storage)
    o.step(3000)
    g.step(3000)
    dps = []
    for s in (o, g):
        f = s.fields()
        p = pressure(f, kap)
        dps.append(p[29:34, 29:34].mean() - p[0:3, 0:3].mean())
    print(storage, "dp oracle", dps[0], "gpu", dps[1], flush=True)
    assert abs(dps[1] / dps[0] - 1) < 0.01


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_lens_angle_16bit(orc, storage):
    """Liquid lens: the cap angles of the 16-bit run are within 0.5 degrees
    of the FP64 oracle's after 10000 steps."""
    w = W.lens(nx=128, ny=80, R=16.0, kappa=(0.02, 0.02, 0.02), alpha=1.0, mobility=0.5)
    o = run_oracle(orc, w)
    g = run_gpu(w, storage)
    o.step(10000)
    g.step(10000)
    ao = lens_angles(o.fields()["c3"], 39.5)
    ag = lens_angles(g.fields()["c3"], 39.5)
    print(storage, "angles oracle", ao, "gpu", ag, flush=True)
    assert abs(ag[0] - ao[0]) < 0.5 and abs(ag[1] - ao[1]) < 0.5


def test_fp16_capsule_close_to_oracle(orc):
    """Capsule at an interface, 200 steps in half storage: fields and markers
    stay close to the FP64 oracle (reported; the bar is on observables)."""
    w = W.c1()
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp16")
    o.step(200)
    g.step(200)
    fo, fg = o.fields(), g.fields()
    errs = {k: normwise(fg[k], fo[k]) for k in ("rho", "c1", "c2", "c3", "ux", "uy")}
    print("fp16 c1 step 200", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert max(errs[k] for k in ("rho", "c1", "c2", "c3")) < 1e-3
    assert np.abs(g.membrane(0)["X"] - o.membrane(0)["X"]).max() < 1e-2
