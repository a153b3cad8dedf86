"""GPU parity of unequal component densities (eq. MassDensity, the extension
the paper names in Sec. 5) against the oracle: the concentration map, the
chemical potentials through it, the pressure tensor's congruent kappa
matrix, the lattice pressure of the number density and the energy readout.
Density ratios 2 to 3, D2Q9 and D3Q19; the oracle's own pins are in
test_oracle_densities.py.

FP64 storage is held to the parity bar of the equal-density tests.  FP32
storage is held to looser bars: the format keeps f_i - w_i rho0 (rho0 =
(M1 + M2)/2), which is small for the moving populations in every phase, but
the rest population then carries the density contrast, f_0 - w_0 rho0 ~
a phi + b psi (up to 0.75 here), so each step rounds a node's mass at
2^-25 x 0.75 ~ 2e-8 where equal densities round at ~1e-11 (f_0 - w_0 ~ 1e-3).
That noise in rho is a pressure noise c_s^2 drho, which moves the fluid:
after a few hundred steps the FP32 fields sit ~3e-5 (concentrations) and
~5e-4 of max|u| (velocities) from the FP64 oracle, against ~1e-7 and ~1e-6
with equal densities on the same set-up.  The FP32 bars below are those
figures with a margin of 2 to 4."""
import numpy as np
import pytest

from helpers import compare, marker_err, normwise, normwise_dev, run_gpu, run_oracle
from paper_1906_03065_amd import workloads as W

pytestmark = pytest.mark.gpu

MW = (2.5, 1.0, 1.5)


def _capsule(form, tau=0.8):
    w = W.capsule_at_interface(nx=72, ny=66, R=12.0, n_markers=80, centre=(35.3, 32.6), tau=tau, tau_phi=1.3,
                               seed=23, mw=MW)
    w["params"]["force_form"] = form
    return w


@pytest.mark.parametrize("form", [1, 0])
def test_capsule_parity_fp64(orc, form):
    """A capsule at a C1/C2 interface with M = (2.5, 1, 1.5), walls in y,
    tau and tau_phi != 1: FP64 against the oracle after 1, 10 and 150 steps
    (fields and markers)."""
    w = _capsule(form)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    for n in (1, 10, 150):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o)
        errs["rho_dev"] = normwise_dev(g.fields()["rho"], o.fields()["rho"])
        print("form", form, "step", n, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
        for k, v in errs.items():
            assert v < 1e-9, (n, k, v)
        assert marker_err(g, o, 1) < 1e-9


def test_capsule_parity_fp32(orc):
    """The same capsule in FP32 storage (divergence form) after 300 steps,
    to the FP32 bars of this file (see the module docstring)."""
    w = _capsule(1)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp32")
    o.step(300)
    g.step(300)
    fg, fo = g.fields(), o.fields()
    errs = {k: normwise(fg[k], fo[k]) for k in ("c1", "c2", "c3", "ux", "uy")}
    errs["rho_dev"] = normwise_dev(fg["rho"], fo["rho"])
    merr = marker_err(g, o, 1)
    print("fp32 step 300", {k: f"{v:.2e}" for k, v in errs.items()}, "markers", merr, flush=True)
    for k in ("c1", "c2", "c3", "rho_dev"):
        assert errs[k] < 1e-4, (k, errs[k])
    for k in ("ux", "uy"):
        assert errs[k] < 2e-3, (k, errs[k])
    # markers move with that velocity error, ~7e-7 per step: a few 1e-4
    # lattice units after 300 steps
    assert merr < 5e-4


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_flat_interface_ratio_3(orc, storage):
    """C1 three times denser than C2, periodic in y: after 4000 steps the
    GPU's profile, densities and flow match the oracle's (the oracle's own
    pins fix the tanh profile, the tension and the bulk densities 3 and 1)."""
    w = W.flat(nx=2, ny=64, kappa=(0.02, 0.03, 0.02), alpha=2.0, wall_y=0, mw=(3.0, 1.0, 1.0))
    o = run_oracle(orc, w)
    g = run_gpu(w, storage)
    o.step(4000)
    g.step(4000)
    fg, fo = g.fields(), o.fields()
    # FP32: over 4000 steps the rounding of the rest population (2e-8 per
    # step, see the module docstring) moves each interface by ~1e-3 nodes,
    # which on a density step of 2 over ~8 nodes is ~2e-4 in rho
    tol = 1e-10 if storage == "fp64" else 5e-4
    errs = {k: float(np.abs(fg[k] - fo[k]).max()) for k in ("rho", "c1", "c2")}
    # the flow is the interface's residual current, ~1e-6: compared absolutely
    du = np.abs(fg["uy"] - fo["uy"]).max()
    print(storage, errs, "max |u| oracle", np.abs(fo["uy"]).max(), "max |du|", du, flush=True)
    for k, v in errs.items():
        assert v < tol, (k, v)
    assert du < (1e-14 if storage == "fp64" else 1e-6)
    assert abs(fg["rho"].max() - 3.0) < 2e-3 and abs(fg["rho"].min() - 1.0) < 2e-3


def test_energy_parity(orc):
    """Masses and energies with component densities: p_ideal is the ideal gas
    of the number density, c_s^2 (M1 + M2)/2 sum n ln n."""
    w = _capsule(1)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    o.step(20)
    g.step(20)
    eo, eg = o.energy(), g.energy()
    print("energies", eg, eo, flush=True)
    for k in ("F_bulk", "F_grad", "E_c", "E_s", "E_b", "E_kin"):
        assert abs(eg[k] - eo[k]) <= 1e-9 * max(abs(eo[k]), 1e-12), k
    # M_b n ln n / 3 with n ~ 1 is a sum of terms near zero: bounded, as in
    # the equal-density test, by the round-off of n (1e-14 per node)
    assert abs(eg["p_ideal"] - eo["p_ideal"]) <= 1e-14 * 72 * 66 * 0.5 * (MW[0] + MW[1])
    np.testing.assert_allclose(eg["mass"], eo["mass"], rtol=1e-12)


def test_fp32_mass_conservation():
    """Every component's mass stays constant in FP32 storage."""
    g = run_gpu(_capsule(1), "fp32")
    m0 = np.array(g.energy()["mass"])
    g.step(500)
    m1 = np.array(g.energy()["mass"])
    print("mass drift", (m1 - m0) / m0, flush=True)
    assert np.abs((m1 - m0) / m0).max() < 1e-6


def test_equal_densities_unchanged():
    """Setting the densities to 1 explicitly is the default model bit for bit."""
    w = W.c1()
    a = run_gpu(w, "fp32")
    from paper_1906_03065_amd import lbib

    b = lbib.Sim(w["params"], storage="fp32", membranes=w["membranes"])
    b.set_densities(1.0, 1.0, 1.0)
    for m in w["membranes"]:
        b.add_membrane(m["X"], None, m["kappa_s"], m["kappa_b"])
    f = w["fields"]
    b.set_fields(f["rho"], f["phi"], f["psi"], f.get("u"))
    a.step(30)
    b.step(30)
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k


def test_densities_rejected_and_checkpoint():
    """Bad values, a set state and a checkpoint of other densities are refused."""
    from paper_1906_03065_amd import lbib

    w = _capsule(1)
    g = run_gpu(w, "fp32")
    for bad in ((0.0, 1.0, 1.0), (1.0, -2.0, 1.0), (1.0, 1.0, float("nan"))):
        with pytest.raises(lbib.LbibError) as e:
            g.set_densities(*bad)
        assert e.value.code == lbib.EINVAL
    with pytest.raises(lbib.LbibError) as e:
        g.set_densities(1.0, 1.0, 1.0)  # the fields are set
    assert e.value.code == lbib.ESTATE
    g.step(2)
    blob = g.save()
    w2 = _capsule(1)
    w2["params"]["mw"] = [2.0, 1.0, 1.5]
    h = run_gpu(w2, "fp32")
    with pytest.raises(lbib.LbibError) as e:
        h.load(blob)
    assert e.value.code == lbib.EINVAL
    same = run_gpu(_capsule(1), "fp32")
    same.load(blob)
    assert same.steps_done == 2


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_drop3d_parity(orc, storage):
    """D3Q19 (potential form): a C3 drop above a C2 layer in C1 with
    M = (2, 1, 3), a wall in z, tau != 1, against the oracle after 1, 10
    and 60 steps; energies at the end."""
    w = W.drop3d(tau=0.8, tau_psi=1.2, mw=(2.0, 1.0, 3.0))
    o = run_oracle(orc, w)
    g = run_gpu(w, storage)
    allerr = []
    for n in (1, 10, 60):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o, D=3)
        errs["rho_dev"] = normwise_dev(g.fields()["rho"], o.fields()["rho"])
        print("3d", storage, "step", n, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
        allerr.append((n, errs))
    for n, errs in allerr:
        for k, v in errs.items():
            if storage == "fp64":
                assert v < 1e-9, (n, k, v)
            else:  # the FP32 bars of this file (module docstring)
                assert v < (2e-3 if k in ("ux", "uy", "uz") else 1e-4), (n, k, v)
    if storage == "fp64":
        eo, eg = o.energy(), g.energy()
        for k in ("F_bulk", "F_grad", "E_kin"):
            assert abs(eg[k] - eo[k]) <= 1e-9 * max(abs(eo[k]), 1e-12), k
        assert abs(eg["p_ideal"] - eo["p_ideal"]) <= 1e-14 * g.N * 1.5
        np.testing.assert_allclose(eg["mass"], eo["mass"], rtol=1e-12)


def test_batch_member_matches_single():
    """A batch member with component densities steps bit for bit like the
    same simulation alone."""
    from paper_1906_03065_amd import lbib

    ws = [_capsule(1), W.capsule_at_interface(nx=64, ny=60, R=10.0, n_markers=72, seed=5, mw=(1.0, 2.0, 1.0))]
    single = [run_gpu(w, "fp32") for w in ws]
    b = lbib.Batch.from_workloads(ws)
    b.step(25)
    for s in single:
        s.step(25)
    for m, s in zip(b.members, single):
        fm, fs = m.fields(), s.fields()
        for k in fs:
            assert np.array_equal(fm[k], fs[k]), k
