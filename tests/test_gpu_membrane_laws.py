"""Hyperelastic strain laws of 2D rings on the GPU (the paper's law, eq.
DiscreteSE, and the neo-Hookean and Skalak laws it names): FP64 parity with
the oracle on stretched capsules at an interface (fields, markers, energies),
the Laplace law of a prestressed ring for each law, batch members with their
own laws equal to single runs, and the argument rules."""
import numpy as np
import pytest

from helpers import compare, marker_err, oracle_params, ring_laplace, run_gpu, run_oracle
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
        s3.set_membrane_law(0, 3)
    s3.set_membrane_law(0, 1)  # triangle law on a mesh
    s3.set_membrane_law(0, 0)


def _edge_keys_sorted(T):
    return sorted({(min(int(t[k]), int(t[(k + 1) % 3])), max(int(t[k]), int(t[(k + 1) % 3])))
                   for t in T for k in range(3)})


def _edge_keys_first_seen(T):
    seen = []
    got = set()
    for t in T:
        for k in range(3):
            key = (min(int(t[k]), int(t[(k + 1) % 3])), max(int(t[k]), int(t[(k + 1) % 3])))
            if key not in got:
                got.add(key)
                seen.append(key)
    return seen


@pytest.mark.parametrize("law", [1, 2])
def test_fp64_parity_mesh_laws(orc, law):
    """D3Q19 capsule whose mesh starts stretched by 1.1 (rest lengths of the
    edges / 1.1), triangle law 1 or 2, walls in z: FP64 fields, markers and
    strain energy against the oracle after 1 and 15 steps."""
    w = W.capsule3d(n=36, R=7.0, subdiv=2, two=False, bridge=False, kappa_s=0.02, kappa_b=1e-3)
    m = w["membranes"][0]
    X, T = m["X"], np.asarray(m["tris"])
    length = {k: np.linalg.norm(X[k[0]] - X[k[1]]) / 1.1 for k in _edge_keys_sorted(T)}
    o = orc.Sim(oracle_params(w["params"]))
    o.add_membrane(X, T, m["kappa_s"], m["kappa_b"])
    o.set_rest(0, [length[k] for k in _edge_keys_first_seen(T)])
    o.set_membrane_law(0, law)
    f = w["fields"]
    o.set_fields(f["rho"], f["phi"], f["psi"], f.get("u"))
    from paper_1906_03065_amd import lbib as L
    g = L.Sim(w["params"], storage="fp64", membranes=w["membranes"])
    g.add_membrane(X, T, m["kappa_s"], m["kappa_b"], [length[k] for k in _edge_keys_sorted(T)])
    g.set_membrane_law(0, law)
    g.set_fields(f["rho"], f["phi"], f["psi"], f.get("u"))
    for n in (1, 15):
        o.step(n - o.steps_done)
        g.step(n - g.steps_done)
        errs = compare(g, o, D=3)
        print(f"mesh law {law} step {n}", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
        for k, v in errs.items():
            assert v < 1e-9, (n, k, v)
        assert marker_err(g, o, 1) < 1e-9
    eo, eg = o.energy(), g.energy()
    print(f"mesh law {law}: E_s gpu {eg['E_s']:.12e} oracle {eo['E_s']:.12e}", flush=True)
    assert abs(eg["E_s"] - eo["E_s"]) <= 1e-10 * abs(eo["E_s"])
    Fg, Fo = g.membrane(0)["F"], o.membrane(0)["F"]
    assert np.abs(Fg - Fo).max() <= 1e-9 * np.abs(Fo).max()


def _mesh_area_volume(X, T):
    P0, P1, P2 = X[T[:, 0]], X[T[:, 1]], X[T[:, 2]]
    A = 0.5 * np.linalg.norm(np.cross(P1 - P0, P2 - P0), axis=1).sum()
    V = np.einsum("ij,ij->i", P0, np.cross(P1, P2)).sum() / 6.0
    return A, V


def _w_sphere(law, lam, G):
    """Energy per rest area at equibiaxial stretch lam from the general
    membrane laws: neo-Hookean G/2 (l1^2 + l2^2 + (l1 l2)^-2 - 3), Skalak
    G/4 (I1^2 + 2 I1 - 2 I2 + C I2^2) with C = 1."""
    if law == 1:
        return 0.5 * G * (2 * lam ** 2 + lam ** -4 - 3)
    I1, I2 = 2 * lam ** 2 - 2, lam ** 4 - 1
    return 0.25 * G * (I1 ** 2 + 2 * I1 - 2 * I2 + I2 ** 2)


@pytest.mark.parametrize("law", [1, 2])
def test_prestressed_mesh_laplace_law(law):
    """A closed mesh stretched by 1.2 in a uniform fluid settles where the
    pressure jump balances its membrane stress: dp = dE/dV = A0 W'(lam) /
    (3 lam^2 V0) for uniform scaling (A0, V0 the rest mesh's area and
    volume), each triangle law against the general law."""
    w = W.prestressed_mesh(law)
    m = w["membranes"][0]
    T = np.asarray(m["tris"])
    g = run_gpu(w, "fp32")
    g.step(6000)
    assert g.check() == 0
    X = g.membrane(0)["X"]
    A_r, V_r = _mesh_area_volume(m["X"] / 1.2, T)  # rest mesh (a scaled copy)
    lam = (_mesh_area_volume(X, T)[1] / V_r) ** (1.0 / 3.0)
    h = 1e-6
    dW = (_w_sphere(law, lam + h, m["kappa_s"]) - _w_sphere(law, lam - h, m["kappa_s"])) / (2 * h)
    pred = A_r * dW / (3 * lam ** 2 * V_r)
    n = w["params"]["nx"]
    f = g.fields()
    dp = (f["rho"][n // 2, n // 2, n // 2] - f["rho"][0, 0, 0]) / 3.0
    print(f"law {law}: lam {lam:.5f} dp {dp:.6e} predicted {pred:.6e} ratio {dp / pred:.4f}", flush=True)
    assert dp == pytest.approx(pred, rel=0.02)
