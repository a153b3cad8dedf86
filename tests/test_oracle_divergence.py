"""Pins of the oracle's divergence-form free-energy force (eq. ForceFE with
the pressure tensor of Appendix A).  The tensor is checked against the
continuum Gibbs-Duhem identity div p' = sum_q q grad mu_q, with the chemical
potentials that are themselves pinned to the free energy, and its bulk part
against numerical derivatives of the bulk energy; the lattice force against
exact momentum conservation on a periodic lattice and against the potential
form on smooth fields."""
import numpy as np
import pytest

import oracle as O
from paper_1906_03065_amd import workloads as W

P = dict(nx=8, ny=8, kappa=[0.013, 0.021, 0.034], alpha=1.7, kappa_c=0.0)
CS2 = 1.0 / 3.0


def _fields(x, y):
    """Smooth analytic rho, phi, psi with exact gradients and Laplacians."""
    spec = [(1.0, 0.02, 0.3, 0.7, 0.2), (0.1, 0.4, 0.5, -0.4, 1.1), (0.3, 0.25, -0.6, 0.35, 0.4)]
    q, g, l = np.zeros(3), np.zeros((3, 3)), np.zeros(3)
    for k, (a, b, kx, ky, ph) in enumerate(spec):
        s, c = np.sin(kx * x + ph), np.cos(ky * y)
        q[k] = a + b * s * c
        g[k, 0] = b * kx * np.cos(kx * x + ph) * c
        g[k, 1] = -b * ky * s * np.sin(ky * y)
        l[k] = -b * (kx * kx + ky * ky) * s * c
    return q, g, l


def _mu(x, y):
    q, g, l = _fields(x, y)
    out = np.zeros(3)
    O.lib().orc_mu(O.C.byref(O.make_params(P)), q[0], q[1], q[2], l[0], l[1], l[2], q[2],
                   out.ctypes.data_as(O._dp))
    return out


@pytest.mark.parametrize("pt", [(0.3, 1.1), (2.2, -0.7), (-1.4, 0.25)])
def test_gibbs_duhem(pt):
    """div p'(x) = rho grad mu_rho + phi grad mu_phi + psi grad mu_psi at a
    point, both sides by central differences of exact-derivative fields."""
    x, y = pt
    h = 1e-4
    div = np.zeros(2)
    for b, (dx, dy) in enumerate(((h, 0.0), (0.0, h))):
        Pp = O.pressure_tensor(P, *_fields(x + dx, y + dy))
        Pm = O.pressure_tensor(P, *_fields(x - dx, y - dy))
        div += (Pp[:2, b] - Pm[:2, b]) / (2 * h)
    q, _, _ = _fields(x, y)
    gm = np.stack([(_mu(x + h, y) - _mu(x - h, y)) / (2 * h), (_mu(x, y + h) - _mu(x, y - h)) / (2 * h)], 1)
    rhs = (q[:, None] * gm).sum(0)
    # central differences of step 1e-4 carry ~1e-8 relative truncation error;
    # a wrong coefficient or sign anywhere in p' is off at order one
    assert np.abs(div - rhs).max() < 1e-6 * np.abs(rhs).max(), (div, rhs)


def test_bulk_pressure_from_energy():
    """With no gradients p' = p_b' I, p_b' = sum_q q df_b/dq - f_b, the
    derivatives of f_b = sum_m kappa_m/2 C_m^2 (1 - C_m)^2 taken numerically
    in (rho, phi, psi)."""
    k = P["kappa"]

    def fb(q):
        C = (0.5 * (q[0] + q[1] - q[2]), 0.5 * (q[0] - q[1] - q[2]), q[2])
        return sum(0.5 * km * c * c * (1 - c) ** 2 for km, c in zip(k, C))

    rng = np.random.default_rng(3)
    for _ in range(5):
        q = np.array([1.0 + rng.uniform(-0.1, 0.1), rng.uniform(-1, 1), rng.uniform(0, 1)])
        h = 1e-6
        d = np.array([(fb(q + h * e) - fb(q - h * e)) / (2 * h) for e in np.eye(3)])
        pb = (q * d).sum() - fb(q)
        Pt = O.pressure_tensor(P, q, np.zeros((3, 3)), np.zeros(3))
        assert Pt[0, 0] == pytest.approx(pb, rel=1e-8, abs=1e-14)
        assert Pt[1, 1] == Pt[0, 0] and Pt[0, 1] == 0.0


def _sim(w, form):
    p = dict(w["params"])
    p["force_form"] = form
    s = O.Sim(p)
    f = w["fields"]
    s.set_fields(f["rho"], f["phi"], f["psi"])
    return s


def test_divergence_form_conserves_momentum():
    """On a periodic lattice the lattice divergence telescopes: the force of
    a liquid lens sums to zero (round-off), where the potential form's does
    not."""
    w = W.capsule_at_interface(nx=64, ny=48, R=12.0, n_markers=8, kappa=(0.02, 0.03, 0.015), kappa_c=0.0,
                               wall_y=0, perturb=0.0)
    s = _sim(w, 1)
    Fd = s.fe_force(1)
    Fp = s.fe_force(0)
    scale = np.abs(Fd).max()
    assert scale > 1e-6
    assert np.abs(Fd.sum(0)).max() < 1e-13 * Fd.shape[0] * scale
    assert np.abs(Fp.sum(0)).max() > 1e3 * np.abs(Fd.sum(0)).max()


def test_divergence_and_potential_forms_agree_on_smooth_fields():
    """Both forms discretise the same continuum force: on well-resolved fields
    they agree to the stencils' second order."""
    for n in (32, 64):
        x, y = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float))
        k = 2 * np.pi / n
        rho = 1.0 + 0.01 * np.sin(k * x) * np.cos(k * y)
        phi = 0.5 * np.sin(k * x + 0.3)
        psi = 0.4 + 0.3 * np.cos(k * y + 0.7)
        w = dict(params=W.base_params(n, n, kappa=(0.02, 0.03, 0.01), alpha=1.0, kappa_c=0.0),
                 fields=dict(rho=rho, phi=phi, psi=psi))
        s = _sim(w, 1)
        d = np.abs(s.fe_force(1) - s.fe_force(0)).max() / np.abs(s.fe_force(0)).max()
        if n == 32:
            d32 = d
    assert d < 0.35 * d32 and d < 5e-3, (d32, d)
