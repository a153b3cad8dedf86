"""Oracle pins of the BGK relaxation of f at tau != 1 and of the marker
velocity reading, against closed forms (no GPU).

  * A shear wave u_x = U sin(k y) in one bulk phase decays at nu k^2 with
    the kinematic viscosity nu = eta / rho = c_s^2 (tau - 1/2) of eq.
    RelaxationTimes (c_s^2 = 1/3).  Relaxing with tau in place of 1/tau, or
    dropping the 1/2, changes the rate by far more than the 1 % bar.
  * A fluid at rest under a uniform force density f_ext (eq. ForcingTermLBE)
    stays uniform and at equilibrium; the exact-difference forcing of eq.
    LBE adds f_ext to the momentum every step, so the bare velocity after t
    steps is u = t f_ext / rho.  The marker velocity read at t+1 is
    v* = u(t+1) + f(t) / (2 rho(t+1)) (eqs. Interpolation, ActualFluidVel
    with the force of step t), i.e. (t + 3/2) f_ext / rho, and the Peskin
    kernel interpolates a uniform field exactly, so after T Euler updates
    (eq. UpdatedXl) every marker has moved by f_ext T (T + 2) / (2 rho).
    Without the half-force term the displacement would be
    f_ext T (T + 1) / 2, with a doubled one f_ext T (T + 3) / 2.
"""
import numpy as np
import pytest

from paper_1906_03065_amd import workloads as W


def _amplitude(f, ny):
    y = np.arange(ny)
    return 2.0 * float(np.mean(f["ux"] * np.sin(2.0 * np.pi * y / ny)[:, None]))


@pytest.mark.parametrize("tau", [0.8, 1.3])
def test_shear_wave_viscosity(orc, tau):
    ny = 128
    w = W.shear_wave(ny=ny, tau=tau)
    s = orc.Sim(w["params"])
    f = w["fields"]
    s.set_fields(f["rho"], f["phi"], f["psi"], f["u"])
    t, a = [], []
    for n in range(0, 2401, 300):
        s.step(n - s.steps_done)
        t.append(n)
        a.append(_amplitude(s.fields(), ny))
    # skip the first 300 steps (the equilibrium start has no viscous stress)
    rate = -np.polyfit(t[1:], np.log(a[1:]), 1)[0]
    nu = (tau - 0.5) / 3.0
    k = 2.0 * np.pi / ny
    print(f"tau {tau}: rate {rate:.6e}, nu k^2 {nu * k * k:.6e}, ratio {rate / (nu * k * k):.5f}")
    assert abs(rate / (nu * k * k) - 1.0) < 1e-2


@pytest.mark.parametrize("tau", [1.0, 0.8])
def test_uniform_force_velocity_and_marker_reading(orc, tau):
    T = 10
    w = W.forced_fluid(tau=tau)
    g = np.array(w["params"]["fext"][:2])
    s = orc.Sim(w["params"])
    m = w["membranes"][0]
    s.add_membrane(m["X"], None, 0.0, 0.0)
    f = w["fields"]
    s.set_fields(f["rho"], f["phi"], f["psi"])
    X0 = s.membrane(0)["X"].copy()
    s.step(T)
    out = s.fields()
    assert np.abs(out["rho"] - 1.0).max() < 1e-14
    for a, key in enumerate(("ux", "uy")):
        assert np.abs(out[key] - T * g[a]).max() < 1e-12 * abs(T * g[a])
    disp = s.membrane(0)["X"] - X0
    want = g * T * (T + 2) / 2.0
    assert np.abs(disp - want).max() < 1e-10 * np.abs(want).max(), (disp[0], want)
    # the readings the pin rules out differ by f_ext T / 2
    assert np.abs(want - g * T * (T + 1) / 2.0).max() > 1e4 * np.abs(disp - want).max()
    mv = s.membrane(0)["U"]
    assert np.abs(mv - g * (T - 1 + 1.5)).max() < 1e-10 * np.abs(g).max() * T
