"""Hyperelastic strain laws of 2D rings on the GPU (the paper's law, eq.
DiscreteSE, and the neo-Hookean and Skalak laws it names): FP64 parity with
the oracle on stretched capsules at an interface (fields, markers, energies),
the Laplace law of a prestressed ring for each law, batch members with their
own laws equal to single runs, and the argument rules."""
import numpy as np
import pytest

from helpers import compare, marker_err, ring_laplace, run_gpu, run_oracle
from paper_1906_03065_amd import lbib
from paper_1906_03065_amd import workloads as W

pytestmark = pytest.mark.gpu


def _stretched(law, wall_y=1, lam0=1.15):
    """Capsule at an interface whose rest lengths are the chords / lam0, plus
    a second, compressed capsule (rest lengths chords * 1.1)."""
    w = W.capsule_at_interface(nx=150, ny=83, R=12.0, n_markers=72, centre=(40.3, 41.2), wall_y=wall_y,
                               tau=0.9, kappa=(0.02, 0.03, 0.015), kappa_s=0.05, seed=21)
    m = w["membranes"][0]
    m["rest"] = np.linalg.norm(np.roll(m["X"], -1, axis=0) - m["X"], axis=1) / lam0
    m["law"] = law
    X2 = W.circle_markers(110.6, 40.1, 10.0, 60)
    w["membranes"].append(dict(X=X2, tris=None, kappa_s=0.05, kappa_b=1e-3, law=law,
                               rest=np.linalg.norm(np.roll(X2, -1, axis=0) - X2, axis=1) * 1.1))
    return w


@pytest.mark.parametrize("wall_y", [0, 1])
@pytest.mark.parametrize("law", [0, 1, 2])
def test_fp64_parity_strain_laws(orc, law, wall_y):
    w = _stretched(law, wall_y)
    o = run_oracle(orc, w)
    g = run_gpu(w, "fp64")
    for n in (1, 80):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o)
        print(f"law {law} wall={wall_y} step {n}", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
        for k, v in errs.items():
            assert v < 1e-9, (n, k, v)
        assert marker_err(g, o, 2) < 1e-9
    eo, eg = o.energy(), g.energy()
    print(f"law {law}: E_s gpu {eg['E_s']:.12e} oracle {eo['E_s']:.12e}", flush=True)
    assert abs(eg["E_s"] - eo["E_s"]) <= 1e-10 * abs(eo["E_s"])
    assert abs(eg["E_b"] - eo["E_b"]) <= 1e-10 * abs(eo["E_b"])


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("law", [0, 1, 2])
def test_prestressed_ring_laplace_law(storage, law):
    """A ring stretched by 1.25 in a uniform fluid: pressure jump = T(lam)/R
    after 6000 steps (T from the general membrane laws at plane strain)."""
    w = W.prestressed_ring(law)
    g = run_gpu(w, storage)
    g.step(6000)
    dp, pred = ring_laplace(g, w)
    print(storage, law, f"dp {dp:.6e} T/R {pred:.6e} ratio {dp / pred:.5f}", flush=True)
    assert dp == pytest.approx(pred, rel=3e-3)


def test_batch_members_with_their_own_laws():
    """A batch of three stretched capsules, one per law: every member bitwise
    equal to its single run."""
    ws = [_stretched(law) for law in (0, 1, 2)]
    b = lbib.Batch.from_workloads(ws)
    b.step(40)
    b.synchronize()
    assert b.check() == 0
    for k, w in enumerate(ws):
        s = run_gpu(w, "fp32")
        s.step(40)
        for q in ("X", "U", "F"):
            for i in range(2):
                assert np.array_equal(b[k].membrane(i)[q], s.membrane(i)[q]), (k, q, i)
        fb, fs = b[k].fields(), s.fields()
        for key in fb:
            assert np.array_equal(fb[key], fs[key]), (k, key)


def test_membrane_law_rules():
    g = run_gpu(_stretched(0), "fp32")
    for bad in ((0, 3), (0, -1), (2, 1)):
        with pytest.raises(lbib.LbibError):
            g.set_membrane_law(*bad)
    g.set_membrane_law(1, 2)
    s3 = run_gpu(W.capsule3d(n=32, R=6.0, subdiv=1, two=False, bridge=False), "fp32")
    with pytest.raises(lbib.LbibError):
        s3.set_membrane_law(0, 1)  # the laws are defined for 2D rings
    s3.set_membrane_law(0, 0)
