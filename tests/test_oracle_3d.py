"""Pins of the oracle's D3Q19 / triangle-mesh path (the paper states the 3D
extension is direct; the mesh law is the reading recorded with the oracle)."""
import numpy as np
import pytest

from paper_1906_03065_amd import workloads as W


def _sphere_sim(orc, n=24, R=7.0, subdiv=3, kc=0.01, centre=None, rc=0.0):
    p = W.base_params(n, n, n, lattice=1, kappa=(0.02,) * 3, alpha=1.0, kappa_c=kc, r_cut=rc)
    s = orc.Sim(p)
    V, T = W.icosphere(subdiv)
    c = np.array(centre if centre is not None else (n / 2 + 0.31, n / 2 - 0.17, n / 2 + 0.23))
    X = V * R + c
    s.add_membrane(X, T, 0.0, 0.0)
    return s, X, T, c


def test_mesh_profile_matches_sphere(orc):
    """eq. Iprofile with d the signed distance to the triangle mesh: close to
    the tanh profile of the exact sphere distance (the mesh lies inside the
    sphere by at most its chord sag), 1 deep inside and 0 far outside."""
    n, R = 24, 7.0
    s, X, T, c = _sphere_sim(orc, n=n, R=R, subdiv=3)
    I, Fc, Ec = s.coupling(np.zeros(s.shape))
    z, y, x = np.meshgrid(*(np.arange(n, dtype=float),) * 3, indexing="ij")
    d = R - np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    ref = W.tanh_profile(d, 1.0)
    e = np.linalg.norm(X[T[:, 1]] - X[T[:, 0]], axis=1).max()
    sag = R - np.sqrt(R ** 2 - (e / np.sqrt(3)) ** 2)
    assert np.abs(I - ref).max() < 0.26 * sag + 1e-12
    assert I.min() >= 0.0 and I.max() <= 1.0
    assert I[0, 0, 0] < 1e-4


def test_mesh_inside_parity_matches_sphere(orc):
    """Inside/outside far from the mesh (beyond r_cut, I is exactly 0 or 1)
    follows the sphere."""
    n, R = 24, 8.0
    s, X, T, c = _sphere_sim(orc, n=n, R=R, subdiv=2, rc=2.0)
    I, _, _ = s.coupling(np.zeros(s.shape))
    z, y, x = np.meshgrid(*(np.arange(n, dtype=float),) * 3, indexing="ij")
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    assert np.all(I[r < R - 3.5] == 1.0)
    assert np.all(I[r > R + 2.5] == 0.0)


def test_mesh_coupling_force_is_energy_gradient(orc):
    """eq. DiscreteCF in 3D: the coupling force is -dE_c/dX by central
    differences of eq. DiscreteCE at fixed psi."""
    n, R = 16, 4.0
    V, T = W.icosphere(1)
    g = np.random.default_rng(12)
    c = np.array([7.6, 8.3, 7.9])
    X = V * R + c + g.normal(scale=0.1, size=V.shape)
    p = W.base_params(n, n, n, lattice=1, kappa=(0.02,) * 3, alpha=1.0, kappa_c=0.05)
    z, y, x = np.meshgrid(*(np.arange(n, dtype=float),) * 3, indexing="ij")
    psi = W.tanh_profile(R + 0.6 - np.sqrt((x - 8) ** 2 + (y - 8) ** 2 + (z - 8) ** 2), 1.0)

    def coup(Xm):
        s = orc.Sim(p)
        s.add_membrane(Xm, T, 0.0, 0.0)
        return s.coupling(psi)

    _, Fc, _ = coup(X)
    h = 1e-6
    G = np.zeros_like(X)
    for v in range(len(X)):
        for a in range(3):
            Xp = X.copy(); Xp[v, a] += h
            Xm = X.copy(); Xm[v, a] -= h
            G[v, a] = (coup(Xp)[2] - coup(Xm)[2]) / (2 * h)
    np.testing.assert_allclose(Fc, -G, atol=3e-6 * np.abs(Fc).max())


def test_spread_interp_3d(orc):
    """Spreading and interpolation with the tensor-product kernel are adjoint
    and interpolate linear fields exactly (3D)."""
    p = W.base_params(20, 18, 16, lattice=1, kappa=(0.02,) * 3, alpha=1.0)
    s = orc.Sim(p)
    g = np.random.default_rng(13)
    X = g.uniform([3, 3, 3], [16, 14, 12], size=(25, 3))
    F = g.normal(size=(25, 3))
    v = g.normal(size=s.shape + (3,))
    fib = s.spread(X, F)
    U = s.interp(X, v)
    assert abs((fib * v).sum() - (F * U).sum()) < 1e-11
    np.testing.assert_allclose(fib.reshape(-1, 3).sum(0), F.sum(0), atol=1e-12)
    z, y, x = np.meshgrid(np.arange(16.0), np.arange(18.0), np.arange(20.0), indexing="ij")
    lin = np.stack([0.3 * x - 0.1 * z, 0.2 * y + 0.4 * z, x - y], -1)
    U = s.interp(X, lin)
    ref = np.stack([0.3 * X[:, 0] - 0.1 * X[:, 2], 0.2 * X[:, 1] + 0.4 * X[:, 2], X[:, 0] - X[:, 1]], 1)
    np.testing.assert_allclose(U, ref, atol=1e-12)


def test_mass_conservation_3d(orc):
    """D3Q19 with a membrane and walls in z: every component is conserved."""
    w = W.capsule3d(n=20, R=5.0, subdiv=2, two=False, bridge=False, wall_z=1)
    s = orc.Sim(w["params"])
    for m in w["membranes"]:
        s.add_membrane(m["X"], m["tris"], m["kappa_s"], m["kappa_b"])
    f = w["fields"]
    s.set_fields(f["rho"], f["phi"], f["psi"])
    m0 = np.array(s.energy()["mass"])
    s.step(40)
    m1 = np.array(s.energy()["mass"])
    np.testing.assert_allclose(m1, m0, rtol=1e-13)


@pytest.mark.slow
def test_laplace_law_3d(orc):
    """A C3 drop in C1 in 3D holds dp = 2 gamma_13 / R."""
    n, R = 32, 9.0
    kap = (0.02, 0.02, 0.02)
    p = W.base_params(n, n, n, lattice=1, kappa=kap, alpha=1.0, kappa_c=0.0, mobility=0.1)
    z, y, x = np.meshgrid(*(np.arange(n, dtype=float),) * 3, indexing="ij")
    c = (n - 1) / 2
    C3 = W.tanh_profile(R - np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2), 1.0)
    f = W.fields_from_C(1 - C3, np.zeros_like(C3), C3)
    s = orc.Sim(p)
    s.set_fields(f["rho"], f["phi"], f["psi"])
    s.step(1500)
    fl = s.fields()
    Cs = [fl["c1"], fl["c2"], fl["c3"]]
    pr = fl["rho"] / 3.0
    for k, cc in zip(kap, Cs):
        pr = pr + cc * k * cc * (1 - cc) * (1 - 2 * cc) - 0.5 * k * cc * cc * (1 - cc) ** 2
    dp = pr[14:18, 14:18, 14:18].mean() - pr[0:2, 0:2, 0:2].mean()
    Rm = (3 * fl["c3"].sum() / (4 * np.pi)) ** (1 / 3)
    gamma = 1.0 * (kap[0] + kap[2]) / 6
    assert abs(dp * Rm / (2 * gamma) - 1) < 0.04, (dp * Rm, 2 * gamma)
