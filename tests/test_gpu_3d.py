"""GPU parity on D3Q19: the HIP library against the FP64 oracle on the same
seeded inputs, element by element over whole fields and marker sets."""
import numpy as np
import pytest

from helpers import compare, marker_err, run_gpu, run_oracle
from paper_1906_03065_amd import workloads as W

pytestmark = pytest.mark.gpu


def _report(tag, errs):
    print(tag, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)


@pytest.mark.parametrize("walls", [(0, 1), (1, 1), (0, 0)])
def test_fp64_parity_drop3d_ragged(orc, walls):
    """No membrane, ragged box (x, y not multiples of the 16-node tile, z not
    a multiple of the plane segment), walls in y and/or z or none, tau != 1."""
    wy, wz = walls
    w = W.drop3d(nx=21, ny=19, nz=13, R=5.0, wall_y=wy, wall_z=wz, tau=0.8, tau_phi=1.3,
                 tau_psi=0.9, u0=(2e-3, -1e-3, 5e-4))
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    for n in (0, 1, 60):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o, D=3)
        _report(f"fp64 drop3d walls={walls} step {n}", errs)
        for k, v in errs.items():
            assert v < 1e-10, (n, k, v)


def test_fp64_parity_small_segments(orc):
    """Plane segments of 5 in a 30-plane box (several segments and a tail,
    alternating march direction) give the oracle's fields."""
    w = W.drop3d(nx=34, ny=18, nz=30, R=6.0, wall_y=1, wall_z=1)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    g.set_launch(seg=5)
    o.step(40)
    g.step(40)
    errs = compare(g, o, D=3)
    _report("fp64 drop3d seg 5", errs)
    for k, v in errs.items():
        assert v < 1e-10, (k, v)


def test_fp32_parity_drop3d_1000_steps(orc):
    """FP32 storage: max relative error <= 1e-5 on rho, u and C_m after 1000
    steps (normwise)."""
    w = W.drop3d(nx=20, ny=20, nz=20, R=6.0, wall_y=0, wall_z=1)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp32")
    o.step(1000)
    g.step(1000)
    errs = compare(g, o, D=3)
    _report("fp32 drop3d step 1000", errs)
    for k, v in errs.items():
        assert v <= 1e-5, (k, v)


def _capsule(n=24, R=6.0, subdiv=2, two=False, **kw):
    return W.capsule3d(n=n, R=R, subdiv=subdiv, two=two, bridge=two, **kw)


def test_fp64_parity_capsule3d(orc):
    """One icosphere capsule (320 triangles) on the C1/C2 interface, walls in
    z, tau != 1: fields and marker positions match the oracle."""
    w = _capsule(tau=0.85, kappa_b=5e-3)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    for n in (1, 40):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o, D=3)
        _report(f"fp64 capsule3d step {n}", errs)
        for k, v in errs.items():
            assert v < 1e-9, (n, k, v)
        assert marker_err(g, o, 1) < 1e-10
        Fo, Fg = o.membrane(0)["F"], g.membrane(0)["F"]
        assert np.abs(Fg - Fo).max() <= 1e-9 * np.abs(Fo).max()


def test_fp64_parity_partial_tile_at_periodic_edge_3d(orc):
    """36^3 (the last 8-wide tile in x and y holds 4 nodes), one capsule of
    radius 6 centred at x = 17.2, band 8.9: the last tile's nodes lie
    within half a period of the capsule but its nominal centre (35.5) does
    not, so the tile must be placed by its nodes' image; its nodes at
    x = 32 are in the band."""
    w = W.capsule3d(n=36, R=6.0, subdiv=2, two=False, bridge=False, r_cut=8.9, shift=(-1.1, 0.0, 0.0))
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    for n in (1, 20):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o, D=3)
        _report(f"fp64 capsule3d partial edge tile step {n}", errs)
        for k, v in errs.items():
            assert v < 1e-9, (n, k, v)
        assert marker_err(g, o, 1) < 1e-10


def test_fp64_energy_parity_capsule3d(orc):
    """Free-energy sums, coupling, strain and bending energies (FP64 on the
    GPU) agree with the oracle."""
    w = _capsule(kappa_b=5e-3)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    o.step(15)
    g.step(15)
    eo, eg = o.energy(), g.energy()
    print("oracle", eo, "\ngpu", eg, flush=True)
    for k in ("F_bulk", "F_grad", "E_c", "E_s", "E_b", "E_kin"):
        assert abs(eg[k] - eo[k]) <= 1e-9 * max(abs(eo[k]), 1e-12), k
    for a, b in zip(eg["mass"], eo["mass"]):
        assert abs(a - b) <= 1e-12 * abs(b)


def test_fp32_parity_capsule3d_200_steps(orc):
    """FP32 storage with a membrane: fields within 1e-5 and markers within
    1e-5 lattice units after 200 steps."""
    w = _capsule()
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp32")
    o.step(200)
    g.step(200)
    errs = compare(g, o, D=3)
    _report("fp32 capsule3d step 200", errs)
    for k, v in errs.items():
        assert v <= 1e-5, (k, v)
    assert marker_err(g, o, 1) < 1e-5


def test_fp64_parity_two_capsules_64(orc):
    """The 3D workload's shape at 64^3: two icosphere capsules (1280
    triangles each, R = 10) with a C2 bridge, r_cut = 17 (the coupling band
    wraps close to the antipode of each capsule in x and y)."""
    w = W.capsule3d(n=64, R=10.0, subdiv=3)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    o.step(2)
    g.step(2)
    errs = compare(g, o, D=3)
    _report("fp64 two capsules 64^3 step 2", errs)
    for k, v in errs.items():
        assert v < 1e-10, (k, v)
    assert marker_err(g, o, 2) < 1e-12
    assert g.check() == 0


def test_fp32_launch_shapes_bitwise_3d():
    """Different plane segments and tile shapes (16 x 16, 32 x 8, 64 x 4
    nodes) and repeated runs give bitwise identical FP32 results
    (fixed-point force sums, no order-dependent reductions)."""
    w = _capsule()
    ref = None
    for tx, seg in ((0, 0), (0, 3), (0, 7), (0, 24), (32, 0), (64, 0), (64, 5)):
        g = run_gpu(w, "fp32")
        if seg or tx:
            g.set_launch(block_x=tx, seg=seg)
        g.step(30)
        f = g.fields()
        X = g.membrane(0)["X"]
        if ref is None:
            ref = (f, X)
            continue
        for k in f:
            assert np.array_equal(f[k], ref[0][k]), (tx, seg, k)
        assert np.array_equal(X, ref[1]), (tx, seg)


@pytest.mark.parametrize("tx", [32, 64])
def test_fp64_parity_wide_tiles(orc, tx):
    """Tiles of 32 x 8 and 64 x 4 nodes on a box whose sides are not
    multiples of them (partial tiles in x and y, walls in y and z) give the
    oracle's fields."""
    w = W.drop3d(nx=70, ny=13, nz=11, R=4.0, wall_y=1, wall_z=1, tau=0.8)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    g.set_launch(block_x=tx)
    o.step(30)
    g.step(30)
    errs = compare(g, o, D=3)
    _report(f"fp64 drop3d tiles {tx}", errs)
    for k, v in errs.items():
        assert v < 1e-10, (k, v)
    from paper_1906_03065_amd import lbib
    with pytest.raises(lbib.LbibError):
        g.set_launch(block_x=48)


def test_mass_conservation_fp32_3d():
    """Every component's mass is conserved by the FP32 path (relative drift
    at the FP32 rounding level over 500 steps)."""
    w = _capsule()
    g = run_gpu(w, "fp32")
    m0 = np.array(g.energy()["mass"])
    g.step(500)
    m1 = np.array(g.energy()["mass"])
    print("mass drift", (m1 - m0) / m0, flush=True)
    assert np.all(np.abs(m1 - m0) <= 1e-6 * np.abs(m0))


def test_fp64_parity_dense_mesh(orc):
    """A 5120-triangle capsule of radius 6 in a 32^3 box: every tile near the
    capsule sees more candidate triangles than the per-tile id list holds,
    so the whole-mesh FP64 search runs; fields and markers match."""
    w = W.capsule3d(n=32, R=6.0, subdiv=4, two=False, bridge=False, r_cut=8.0)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    o.step(2)
    g.step(2)
    errs = compare(g, o, D=3)
    _report("fp64 dense mesh step 2", errs)
    for k, v in errs.items():
        assert v < 1e-10, (k, v)
    assert marker_err(g, o, 1) < 1e-12
