"""The coupling-profile search with and without the per-node cache of the
closest membrane element (lbib_set_coupling_cache; ring segments in 2D,
triangles in 3D): a cached element is used only while a bound proves a full
search would pick it, so both give bitwise the same fields, markers, marker
velocities and forces."""
import numpy as np
import pytest

from helpers import run_gpu
from paper_1906_03065_amd import lbib
from paper_1906_03065_amd import workloads as W

pytestmark = pytest.mark.gpu


def _same(a, b, n_mem):
    fa, fb = a.fields(), b.fields()
    for k in fa:
        if not np.array_equal(fa[k], fb[k]):
            return k, float(np.abs(fa[k] - fb[k]).max())
    for i in range(n_mem):
        ma, mb = a.membrane(i), b.membrane(i)
        for q in ("X", "U", "F"):
            if not np.array_equal(ma[q], mb[q]):
                return f"{q}{i}", float(np.abs(ma[q] - mb[q]).max())
    return None


def _two_moving_capsules(wall_y):
    w = W.capsule_at_interface(nx=150, ny=83, R=12.0, n_markers=72, centre=(40.3, 41.2), wall_y=wall_y,
                               tau=0.8, tau_phi=1.3, tau_psi=0.9, kappa=(0.02, 0.03, 0.015), seed=5)
    w["membranes"].append(dict(X=W.circle_markers(110.6, 40.1, 10.0, 60), tris=None, kappa_s=0.05,
                               kappa_b=1e-3))
    # a uniform force drives the capsules across the lattice, so cached
    # segments keep expiring
    w["params"]["fext"] = [3e-6, 1e-6]
    return w


@pytest.mark.parametrize("storage,wall_y", [("fp64", 1), ("fp32", 0), ("fp32", 1)])
def test_cache_bitwise_moving_capsules(storage, wall_y):
    w = _two_moving_capsules(wall_y)
    a = run_gpu(w, storage)
    b = run_gpu(w, storage)
    b.set_coupling_cache(0)
    for n in (1, 50, 400):
        a.step(n - a.steps_done)
        b.step(n - b.steps_done)
        bad = _same(a, b, 2)
        print(storage, wall_y, "step", n, "cache on vs off:", bad or "bitwise equal", flush=True)
        assert bad is None, (n, bad)
    X = a.membrane(0)["X"]
    print("capsule 0 moved", float(np.abs(X.mean(0) - w["membranes"][0]["X"].mean(0)).max()), flush=True)


def test_cache_bitwise_galilean_frame():
    """A capsule carried at U = 1e-2 on a periodic lattice (about four lattice
    units in 400 steps), the potential form as well."""
    w = W.capsule_at_interface(nx=96, ny=90, R=14.0, n_markers=100, centre=(40.3, 44.7), wall_y=0,
                               u0=1e-2, seed=8)
    for form in (1, 0):
        w["params"]["force_form"] = form
        a = run_gpu(w, "fp32")
        b = run_gpu(w, "fp32")
        b.set_coupling_cache(0)
        a.step(400)
        b.step(400)
        bad = _same(a, b, 1)
        print("form", form, "galilean cache on vs off:", bad or "bitwise equal", flush=True)
        assert bad is None, bad


def test_cache_bitwise_c2():
    """The 2048 x 2048 benchmark workload, 30 steps."""
    w = W.c2()
    a = run_gpu(w, "fp32")
    b = run_gpu(w, "fp32")
    b.set_coupling_cache(0)
    a.step(30)
    b.step(30)
    bad = _same(a, b, len(w["membranes"]))
    assert bad is None, bad


def test_cache_bitwise_batch_and_rules():
    ws = [_two_moving_capsules(1), W.capsule_at_interface(nx=300, ny=64, R=11.0, n_markers=88,
                                                          centre=(83.4, 31.7), seed=33)]
    a = lbib.Batch.from_workloads(ws)
    b = lbib.Batch.from_workloads(ws)
    b.set_coupling_cache(0)
    a.step(120)
    b.step(120)
    for k, w in enumerate(ws):
        bad = _same(a[k], b[k], len(w["membranes"]))
        assert bad is None, (k, bad)
    g = run_gpu(W.c1(), "fp32")
    with pytest.raises(lbib.LbibError):
        g.set_coupling_cache(2)


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_cache_bitwise_moving_capsules_3d(storage):
    """Two icosphere capsules (1280 triangles each) bridged on an interface,
    walls in z, driven across the box by a uniform force so that cached
    triangles keep expiring: cache on and off bitwise equal."""
    w = W.capsule3d(n=40, R=8.0, subdiv=3, tau=0.85, shift=(0.3, 0.2, 0.1))
    w["params"]["fext"] = [4e-6, 2e-6, 1e-6]
    a = run_gpu(w, storage)
    b = run_gpu(w, storage)
    b.set_coupling_cache(0)
    for n in (1, 30, 150):
        a.step(n - a.steps_done)
        b.step(n - b.steps_done)
        bad = _same(a, b, 2)
        print(storage, "3d step", n, "cache on vs off:", bad or "bitwise equal", flush=True)
        assert bad is None, (n, bad)


def test_cache_bitwise_c3():
    """The 256^3 two-capsule benchmark workload, 8 steps."""
    w = W.c3()
    a = run_gpu(w, "fp32")
    b = run_gpu(w, "fp32")
    b.set_coupling_cache(0)
    a.step(8)
    b.step(8)
    bad = _same(a, b, len(w["membranes"]))
    assert bad is None, bad
