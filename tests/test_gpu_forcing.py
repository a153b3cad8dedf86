"""GPU checks of the external force density of eq. ForcingTermLBE and of the
BGK relaxation at tau != 1, against the same closed forms that pin the
oracle (see test_oracle_relaxation.py) and against the oracle itself."""
import numpy as np
import pytest

from helpers import compare, marker_err, normwise, run_gpu, run_oracle
from paper_1906_03065_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage,tau", [("fp64", 1.0), ("fp64", 0.8), ("fp32", 1.0)])
def test_uniform_force_closed_form(orc, storage, tau):
    """A fluid at rest under a uniform force density: after T steps the
    bare velocity is T f_ext and every marker has moved f_ext T (T + 2) / 2
    (the v* reading), on the GPU as in the oracle."""
    T = 10
    w = W.forced_fluid(tau=tau)
    g = run_gpu(w, storage)
    fext = np.array(w["params"]["fext"][:2])
    X0 = g.membrane(0)["X"].copy()
    g.step(T)
    f = g.fields()
    tol = 1e-10 if storage == "fp64" else 1e-5
    for a, key in enumerate(("ux", "uy")):
        assert np.abs(f[key] / (T * fext[a]) - 1.0).max() < tol, key
    disp = g.membrane(0)["X"] - X0
    want = fext * T * (T + 2) / 2.0
    print(storage, tau, "displacement", disp[0], "closed form", want, flush=True)
    assert np.abs(disp - want).max() < tol * np.abs(want).max()
    o = run_oracle(orc, w)
    o.step(T)
    fo = o.fields()
    # one bulk phase: C1 = 1 and C2 = C3 = 0 up to round-off, compared
    # absolutely; the velocities relative to their size
    for k in ("rho", "c1", "c2", "c3"):
        assert np.abs(f[k] - fo[k]).max() < (1e-13 if storage == "fp64" else 1e-6), k
    for k in ("ux", "uy"):
        assert normwise(f[k], fo[k]) < (1e-12 if storage == "fp64" else 1e-5), k
    assert marker_err(g, o, 1) < (1e-14 if storage == "fp64" else 1e-9)


@pytest.mark.parametrize("fext", [(2e-6, -1e-6)])
def test_external_force_with_capsule_parity(orc, fext):
    """The force enters every node's forcing, the velocities and the marker
    reading: a capsule at an interface under a small uniform force, walls in
    y, tau != 1, FP64 against the oracle after 1, 10 and 80 steps."""
    w = W.capsule_at_interface(nx=72, ny=66, R=12.0, n_markers=80, centre=(35.3, 32.6), tau=0.9, seed=21)
    w["params"]["fext"] = list(fext)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    for n in (1, 10, 80):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o)
        print("fext", fext, "capsule step", n, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
        for k, v in errs.items():
            assert v < 1e-9, (n, k, v)
        assert marker_err(g, o, 1) < 1e-9


def test_external_force_rejected_values():
    from paper_1906_03065_amd import lbib

    g = run_gpu(W.forced_fluid(fext=(0.0, 0.0)), "fp32")
    for bad in ((float("nan"), 0.0, 0.0), (0.0, float("inf"), 0.0), (0.0, 0.0, 1e-6)):
        with pytest.raises(lbib.LbibError) as e:
            g.set_external_force(*bad)
        assert e.value.code == lbib.EINVAL


@pytest.mark.parametrize("tau", [0.8, 1.3])
def test_shear_wave_viscosity_gpu(orc, tau):
    """The shear wave decays at nu k^2, nu = (tau - 1/2)/3, within 1 % on the
    GPU (FP64 and FP32), and the FP64 field matches the oracle's."""
    ny = 128
    w = W.shear_wave(ny=ny, tau=tau)
    nu, k = (tau - 0.5) / 3.0, 2.0 * np.pi / ny
    for storage in ("fp64", "fp32"):
        g = run_gpu(w, storage)
        t, a = [], []
        for n in range(0, 2401, 300):
            g.step(n - g.steps_done)
            t.append(n)
            a.append(2.0 * float(np.mean(g.fields()["ux"] * np.sin(2.0 * np.pi * np.arange(ny) / ny)[:, None])))
        rate = -np.polyfit(t[1:], np.log(a[1:]), 1)[0]
        print(storage, tau, "rate / nu k^2", rate / (nu * k * k), flush=True)
        assert abs(rate / (nu * k * k) - 1.0) < 1e-2
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    o.step(600)
    g.step(600)
    fg, fo = g.fields(), o.fields()
    for key in ("rho", "c1", "c2", "c3"):
        assert np.abs(fg[key] - fo[key]).max() < 1e-13, key
    amp = np.abs(fo["ux"]).max()  # u_y is zero up to round-off: both against the wave's amplitude
    for key in ("ux", "uy"):
        assert np.abs(fg[key] - fo[key]).max() < 1e-10 * amp, key
