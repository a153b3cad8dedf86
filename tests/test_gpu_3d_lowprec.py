"""16-bit population storage on D3Q19 against the FP64 oracle at 64^3: the
Laplace pressure of a drop within 1 % and the cap angles of a lens within
0.5 degrees.  The oracle's observables are stored in golden/oracle_3d.json,
written by golden/gen_oracle_3d.py (the oracle alone; minutes of CPU at
64^3, so not rerun per test); the observable recipes are shared with it."""
import json
import os

import numpy as np
import pytest

from golden.gen_oracle_3d import DROP, KAP, LENS, drop_dp, lens_slice_angles
from helpers import run_gpu
from paper_1906_03065_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_3d.json")))


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "bf16"])
def test_laplace_pressure_3d(storage):
    """C3 drop (R = 16) in C1, 64^3 periodic, 1500 steps: the pressure jump
    is within 1 % of the oracle's (FP64 and FP32 far closer)."""
    w = W.sphere3d(n=DROP["n"], R=DROP["R"], kappa=KAP)
    g = run_gpu(w, storage)
    g.step(DROP["steps"])
    f = g.fields()
    dp = drop_dp(f, DROP["n"])
    ref = GOLDEN["drop"]["dp"]
    print(storage, "dp gpu", dp, "oracle", ref, "rel", dp / ref - 1, flush=True)
    assert abs(dp / ref - 1) < (1e-9 if storage == "fp64" else 1e-4 if storage == "fp32" else 0.01)
    m3 = float(f["c3"].sum())
    # every storage format conserves each set's mass: the 16-bit formats keep
    # g_0 and h_0 in FP64 like the FP32 one, so no rest-population update is
    # rounded away
    print(storage, "c3 mass rel", m3 / GOLDEN["drop"]["mass_c3"] - 1, flush=True)
    assert abs(m3 / GOLDEN["drop"]["mass_c3"] - 1) < (1e-9 if storage == "fp64" else 1e-6)


@pytest.mark.parametrize("storage", ["fp64", "fp16", "bf16"])
def test_lens_angles_3d(storage):
    """C3 lens on a flat C1/C2 interface, 64^3 with walls in z, 4000 steps:
    cap angles in the mid plane within 0.5 degrees of the oracle's."""
    w = W.lens3d(n=LENS["n"], R=LENS["R"], kappa=KAP, mobility=LENS["mobility"])
    g = run_gpu(w, storage)
    g.step(LENS["steps"])
    a = lens_slice_angles(g.fields(), LENS["n"])
    ref = GOLDEN["lens"]["angles"]
    print(storage, "angles gpu", a, "oracle", ref, flush=True)
    tol = 1e-6 if storage == "fp64" else 0.5
    assert abs(a[0] - ref[0]) < tol and abs(a[1] - ref[1]) < tol


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_mass_conservation_16bit_3d(storage):
    """Masses of the 16-bit D3Q19 path stay fixed to FP32 round-off."""
    w = W.capsule3d(n=32, R=7.0, subdiv=2, two=False, bridge=False)
    g = run_gpu(w, storage)
    m0 = np.array(g.energy()["mass"])
    g.step(300)
    m1 = np.array(g.energy()["mass"])
    print(storage, "mass drift", (m1 - m0) / m0, flush=True)
    assert np.abs((m1 - m0) / m0).max() < 1e-6
