"""GPU parity: the HIP library against the FP64 oracle on the same seeded
inputs, element by element over whole fields (D2Q9)."""
import numpy as np
import pytest

from helpers import compare, marker_err, normwise, rho_dev_err, run_gpu, run_oracle
from paper_1906_03065_amd import workloads as W

pytestmark = pytest.mark.gpu


def _report(tag, errs):
    print(tag, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)


def test_fp64_parity_c1(orc):
    """128x128 capsule at an interface (periodic x, walls y): FP64 kernels
    match the oracle to round-off at steps 0, 1, 10 and 200."""
    w = W.c1()
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    for n in (0, 1, 10, 200):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o)
        _report(f"fp64 c1 step {n}", errs)
        for k, v in errs.items():
            assert v < 1e-9, (n, k, v)
        assert marker_err(g, o, 1) < 1e-9


def test_fp64_parity_c1_no_band_2000_steps(orc):
    """The C1 workload for its full 2000 steps against the oracle's profile
    of eq. Iprofile with no band at all.  The library runs with a band of
    40 alpha, beyond which (1 + tanh(d/2 alpha))/2 is exactly 0 or 1 in FP64,
    so the truncation is below FP64 resolution: fields and markers agree to
    round-off at steps 0, 1, 10, 1000 and 2000; rho is also measured against
    its own variation (max |rho - mean rho|)."""
    o = run_oracle(orc, W.c1(), untruncated=True)
    g = run_gpu(W.c1(r_cut=40.0), "fp64")
    for n in (0, 1, 10, 1000, 2000):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o)
        rd = rho_dev_err(g, o)
        _report(f"fp64 c1 no band step {n} (rho_dev {rd:.2e})", errs)
        for k, v in errs.items():
            assert v < 1e-9, (n, k, v)
        assert rd < 1e-7, (n, rd)
        assert marker_err(g, o, 1) < 1e-9


def test_fp32_parity_c1_default_band_vs_no_band(orc):
    """The library at its defaults (FP32, band 17 alpha) against the oracle
    with no band, after 1000 steps: within the FP32 bar of 1e-5.  The band's
    own effect (the profile's tail beyond 17 alpha, e^-17 = 4e-8) is of
    order 1e-7 in the velocities, far below it."""
    w = W.c1()
    o = run_oracle(orc, w, untruncated=True)
    g = run_gpu(w, "fp32")
    o.step(1000)
    g.step(1000)
    errs = compare(g, o)
    rd = rho_dev_err(g, o)
    _report(f"fp32 c1 default band vs no band step 1000 (rho_dev {rd:.2e})", errs)
    for k, v in errs.items():
        assert v <= 1e-5, (k, v)
    assert rd < 1e-2, rd
    assert marker_err(g, o, 1) < 1e-4


def test_fp32_parity_c1_1000_steps(orc):
    """FP32 storage and arithmetic: max relative error <= 1e-5 on rho, u and
    C_m after 1000 steps (normwise: max |a-b| / max |b|)."""
    w = W.c1()
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp32")
    o.step(1000)
    g.step(1000)
    errs = compare(g, o)
    _report("fp32 c1 step 1000", errs)
    for k, v in errs.items():
        assert v <= 1e-5, (k, v)
    assert marker_err(g, o, 1) < 1e-4


@pytest.mark.parametrize("wall_y", [0, 1])
def test_fp64_parity_ragged_two_capsules_taus(orc, wall_y):
    """Ragged lattice (several 60-column strips plus a tail, segments plus a
    tail), two capsules, tau != 1 (tau = 1 hides BGK errors)."""
    nx, ny = 150, 83
    w = W.capsule_at_interface(nx=nx, ny=ny, R=12.0, n_markers=72, centre=(40.3, 41.2),
                               wall_y=wall_y, tau=0.8, tau_phi=1.3, tau_psi=0.9,
                               kappa=(0.02, 0.03, 0.015), seed=5)
    w["membranes"].append(dict(X=W.circle_markers(110.6, 40.1, 10.0, 60), tris=None,
                               kappa_s=0.05, kappa_b=1e-3))
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    for n in (1, 60):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o)
        _report(f"fp64 ragged wall={wall_y} step {n}", errs)
        for k, v in errs.items():
            assert v < 1e-9, (n, k, v)
        assert marker_err(g, o, 2) < 1e-9


def test_fp64_parity_no_membrane(orc):
    """Pure ternary fluid (a drop, no markers): the lattice path alone."""
    w = W.drop(n=70, R=14.0)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    o.step(100)
    g.step(100)
    errs = compare(g, o)
    _report("fp64 drop", errs)
    for k, v in errs.items():
        assert v < 1e-10, (k, v)


def test_energy_parity(orc):
    """FP64 reductions: energies and masses against the oracle's."""
    w = W.c1()
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    o.step(20)
    g.step(20)
    eo, eg = o.energy(), g.energy()
    print("energies", eg, eo, flush=True)
    for k in ("F_bulk", "F_grad", "E_c", "E_s", "E_b", "E_kin"):
        assert abs(eg[k] - eo[k]) <= 1e-9 * max(abs(eo[k]), 1e-12), k
    # sum rho ln rho / 3 moves by ~1/3 per unit of total mass, which the two
    # sides carry to ~1e-15 relative: bound it by the mass round-off
    assert abs(eg["p_ideal"] - eo["p_ideal"]) <= 1e-14 * 128 * 128
    np.testing.assert_allclose(eg["mass"], eo["mass"], rtol=1e-12)


def test_fp32_mass_conservation():
    """Masses stay constant on the GPU in FP32 (moving populations shifted)."""
    w = W.c1()
    g = run_gpu(w, "fp32")
    m0 = np.array(g.energy()["mass"])
    g.step(500)
    m1 = np.array(g.energy()["mass"])
    print("mass drift", (m1 - m0) / m0, flush=True)
    assert np.abs((m1 - m0) / m0).max() < 1e-6


def test_determinism_and_checkpoint():
    """Bitwise reproducible runs; save/load resumes bitwise."""
    w = W.c1()
    a = run_gpu(w, "fp32")
    a.step(40)
    blob = a.save()
    a.step(40)
    fa = a.fields()
    b = run_gpu(w, "fp32")
    b.step(80)
    fb = b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    c = run_gpu(w, "fp32")
    c.load(blob)
    c.step(40)
    fc = c.fields()
    for k in fa:
        assert np.array_equal(fa[k], fc[k]), k
    assert np.array_equal(a.membrane(0)["X"], c.membrane(0)["X"])


def test_checkpoint_mismatch_refused():
    """A checkpoint from a simulation of another lattice size, storage format
    or force form (with the same marker count) is refused and the handle is
    left as it was."""
    from paper_1906_03065_amd import lbib

    w = W.c1()
    a = run_gpu(w, "fp32")
    a.step(3)
    blob = a.save()
    others = [run_gpu(W.c1(nx=120), "fp32"), run_gpu(w, "fp16"), run_gpu(w, "fp32")]
    others[2].set_force_form(0)  # the potential form (the default is the divergence form)
    for b in others:
        before = b.fields()["rho"].copy()
        with pytest.raises(lbib.LbibError) as e:
            b.load(blob)
        assert e.value.code == lbib.EINVAL
        assert b.steps_done == 0 and np.array_equal(b.fields()["rho"], before)
    with pytest.raises(lbib.LbibError):
        a.load(blob[:-8])  # truncated
    a.load(blob)
    assert a.steps_done == 3


def test_failure_injection_nonfinite():
    """A NaN forced into a population from the host is reported by lbib_check."""
    from paper_1906_03065_amd import lbib

    w = W.c1()
    g = run_gpu(w, "fp32")
    g.step(2)
    assert g.check() == 0
    g.poke(0, 12345, float("nan"))
    g.step(1)
    assert g.check() == -4


def test_c2_fullsize_fp32_vs_oracle(orc):
    """2048x2048 with 16 capsules (the throughput workload, same launch
    shape as the benchmark): two steps, every node against the oracle."""
    w = W.c2()
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp32")
    o.step(2)
    g.step(2)
    errs = compare(g, o)
    _report("fp32 c2 step 2", errs)
    for k, v in errs.items():
        assert v <= 1e-5, (k, v)
    assert marker_err(g, o, 16) < 1e-6


@pytest.mark.parametrize("wall_y", [1, 0])
def test_fp64_parity_band_near_period(orc, wall_y):
    """Capsule band (r_cut + 1 around the ring) nearly as wide as the
    periodic lattice: tiles that straddle the antipode of the capsule hold
    nodes of two periodic images and are searched node by node."""
    w = W.capsule_at_interface(nx=80, ny=82, R=18.5, n_markers=144, centre=(37.3, 40.2),
                               wall_y=wall_y, seed=9)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    for n in (1, 30):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o)
        _report(f"fp64 band near period wall={wall_y} step {n}", errs)
        for k, v in errs.items():
            assert v < 1e-9, (n, k, v)
        assert marker_err(g, o, 1) < 1e-9
    assert g.check() == 0


def test_fp64_parity_partial_tile_at_periodic_edge(orc):
    """72 columns (the last 16-wide tile holds 8), capsule centre at x =
    35.3: the last tile's nodes are within 36 of the centre but its nominal
    centre (x = 71.5) is not, so the tile must be placed by its nodes' image.
    Band nodes at x = 64 must get the tanh tail of the profile."""
    w = W.capsule_at_interface(nx=72, ny=66, R=12.0, n_markers=80, centre=(35.3, 32.6), tau=0.9, seed=21)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    for n in (1, 80):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o)
        _report(f"fp64 partial edge tile step {n}", errs)
        for k, v in errs.items():
            assert v < 1e-9, (n, k, v)
        assert marker_err(g, o, 1) < 1e-9


@pytest.mark.parametrize("r_cut", [4.0, 8.0])
def test_fp64_parity_band_widths(orc, r_cut):
    """Bands narrower than the default 17: with r_cut = 4 every band node of
    a sub-tile is searched exactly (no node is provably beyond the band from
    its sub-tile centre); with r_cut = 8 the capsule interior beyond the
    band takes the side of its sub-tile centres, wave by wave and node by
    node.  Both must give the oracle's profile and forces."""
    w = W.c1(r_cut=r_cut, R=16.0, n_markers=100)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    for n in (1, 40):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o)
        _report(f"fp64 r_cut={r_cut} step {n}", errs)
        for k, v in errs.items():
            assert v < 1e-9, (n, k, v)
        assert marker_err(g, o, 1) < 1e-9
