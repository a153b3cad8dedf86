"""The overlapped D2Q9 step (lattice regions away from the membranes on a
second stream beside the membrane kernels, the rest after them in short
pieces) against the single-stream step: every node is updated by the same
arithmetic, so fields, markers and forces must agree bitwise, in both
forms of the force."""
import numpy as np
import pytest

from helpers import run_gpu
from paper_1906_03065_amd import workloads as W

pytestmark = pytest.mark.gpu


def _form(w, form=0):
    w["params"]["force_form"] = form
    return w


def _state(g):
    f = g.fields()
    mem = [g.membrane(i) for i in range(len(g.mem_sizes))]
    return f, mem


def _same(a, b):
    fa, ma = a
    fb, mb = b
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    for x, y in zip(ma, mb):
        for k in x:
            assert np.array_equal(x[k], y[k]), k


def _ragged(form=0):
    w = W.capsule_at_interface(nx=300, ny=259, R=22.0, n_markers=176, centre=(80.3, 129.2), wall_y=1,
                               tau=0.8, tau_phi=1.3, tau_psi=0.9, kappa=(0.02, 0.03, 0.015), seed=21)
    w["membranes"].append(dict(X=W.circle_markers(220.6, 100.1, 15.0, 120), tris=None, kappa_s=0.05,
                               kappa_b=1e-3))
    return _form(w, form)


@pytest.mark.parametrize("storage,form", [("fp32", 0), ("fp64", 0), ("fp16", 0), ("fp32", 1), ("fp64", 1)])
def test_overlap_bitwise_ragged(storage, form):
    """300 x 259 lattice (ragged strips and segments), two capsules, walls
    in y: 80 steps with the overlap forced on equal 80 steps without."""
    w = _ragged(form)
    a = run_gpu(w, storage)
    a.set_overlap(0)
    b = run_gpu(w, storage)
    b.set_overlap(1)
    a.step(80)
    b.step(80)
    _same(_state(a), _state(b))
    assert b.check() == 0


def test_overlap_bitwise_periodic_and_shapes():
    """Periodic in y (regions wrap), launch shapes varied on the overlapped
    side: 192 lanes with ring 4, then 64 lanes with short segments."""
    w = _form(W.capsule_at_interface(nx=256, ny=192, R=30.0, n_markers=236, centre=(128.0, 20.5), wall_y=0,
                                          seed=23))
    ref = run_gpu(w, "fp32")
    ref.set_overlap(0)
    ref.step(40)
    for bx, seg, ring in ((192, 0, 4), (64, 7, 3)):
        g = run_gpu(w, "fp32")
        g.set_overlap(1)
        g.set_launch(bx, seg, 0, ring)
        g.step(40)
        _same(_state(ref), _state(g))


@pytest.mark.parametrize("form", [0, 1])
def test_overlap_full_size_c2(form):
    """The 2048 x 2048 benchmark lattice with the overlap on against the
    default single-stream step, five steps."""
    w = _form(W.c2(), form)
    a = run_gpu(w, "fp32")
    b = run_gpu(w, "fp32")
    b.set_overlap(1)
    a.step(5)
    b.step(5)
    _same(_state(a), _state(b))


def test_overlap_rejects_bad_values():
    w = W.c1()
    g = run_gpu(w, "fp32")
    for v in (2, -2):
        with pytest.raises(RuntimeError):
            g.set_overlap(v)
    g.set_overlap(1)  # the divergence form (the default)
    g.step(3)
    g.set_force_form(0)
    g.step(3)
    assert g.check() == 0
