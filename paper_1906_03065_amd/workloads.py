"""Seeded synthetic inputs shared by the GPU library's tests and benchmark and
by the CPU oracle's tests.

This module builds parameter dictionaries, initial macroscopic fields and
initial membrane marker sets.  It holds none of the method's arithmetic: no
equilibria, stencils, chemical potentials, forces or kernels.  Initial fields
are diffuse tanh profiles of analytic distances (circles, spheres, planes),
the shape the paper uses for every interface (Sec. 2.5, eq. CmProfile), and
markers are points placed evenly on circles or on icosphere meshes.

Workloads (the paper publishes no datasets; these stand in for its geometries):
  * ``capsule_at_interface``: one capsule of fluid 3 centred on a flat C1/C2
    interface (Sec. 4.1, Fig. 1a), the paper's benchmark configuration.
  * ``c1``: 128x128, periodic x, walls in y, R = 20, 128 markers, kappa 0.02,
    alpha 1, mobility 0.1, +-1e-4 perturbation: the FP64 parity workload.
  * ``c2``: 2048x2048 with 16 capsules of radius 24..64 on a flat interface,
    kappa_m uniform in [0.01, 0.05]: the FP32 throughput workload.
  * ``lens``: a pure liquid lens (no membrane) for the Neumann-angle check.
  * ``drop``: a C3 drop in C1 for the Laplace-law check.
  * ``flat``: a flat C1/C2 interface for the tanh-profile / tension checks.
  * ``capsule3d`` / ``c3``: D3Q19 icosphere capsules with a C3 bridge.
  * ``c4``: 64 capsule-at-interface runs of seeded uneven sizes.
  * ``bridge2d``: two capsules joined by a capillary bridge of fluid 2 in a
    periodic 12R x 6R box (Sec. 4.2), the paper's second workload.
Seeds: ``1906030650 + k`` for workload k unless a seed is given.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 1906030650


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def base_params(nx, ny, nz=1, lattice=0, wall_y=0, wall_z=0, kappa=(0.02, 0.02, 0.02), alpha=1.0,
                kappa_c=0.01, tau=1.0, tau_phi=1.0, tau_psi=1.0, mobility=None, gamma=1.0,
                r_cut=0.0, force_form=None) -> dict:
    """Parameter dictionary.  ``mobility`` M sets Gamma = M/(tau - 1/2) for both
    order parameters (eq. RelaxationTimes), or a pair (M_phi, M_psi) sets each
    (Sec. 2.6 names M_phi = 3 M_psi); otherwise ``gamma`` is used.
    ``force_form``: the thermodynamic force of eq. ForceFE as the divergence
    of the pressure tensor (1, the default on D2Q9) or in its potential form
    (0, the only form on D3Q19)."""
    if force_form is None:
        force_form = 1 if lattice == 0 else 0
    gphi = gpsi = gamma
    if mobility is not None:
        m_phi, m_psi = (mobility, mobility) if np.isscalar(mobility) else mobility
        gphi = m_phi / (tau_phi - 0.5)
        gpsi = m_psi / (tau_psi - 0.5)
    return dict(lattice=lattice, nx=int(nx), ny=int(ny), nz=int(nz), wall_y=int(wall_y),
                wall_z=int(wall_z), tau=float(tau), tau_phi=float(tau_phi), tau_psi=float(tau_psi),
                gamma_phi=float(gphi), gamma_psi=float(gpsi),
                kappa=[float(k) for k in kappa], alpha=float(alpha), kappa_c=float(kappa_c),
                r_cut=float(r_cut), force_form=int(force_form))


def tanh_profile(d, alpha):
    """(1 + tanh(d / 2 alpha)) / 2 of a signed distance d (eq. CmProfile)."""
    return 0.5 * (1.0 + np.tanh(np.asarray(d, dtype=np.float64) / (2.0 * alpha)))


def circle_markers(cx, cy, R, n, phase=None):
    """n markers evenly spaced counter-clockwise on a circle, marker l at angle
    (2 l + 1) pi / n by default.  The half-step phase keeps the polygon
    symmetric under both axis mirrors while no vertex lies on the vertical
    axis, so lattice nodes on that axis have a unique closest membrane point."""
    if phase is None:
        phase = np.pi / n
    t = phase + 2.0 * np.pi * np.arange(n) / n
    return np.stack([cx + R * np.cos(t), cy + R * np.sin(t)], axis=1)


def _grid2(nx, ny):
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y


def _min_image(dx, n):
    return dx - n * np.round(dx / n)


def fields_from_C(C1, C2, C3, perturb=0.0, seed=0, u=None, mw=(1.0, 1.0, 1.0)):
    """rho, phi, psi from concentrations (eq. VariableTransform), after adding a
    seeded uniform perturbation in [-perturb, perturb] to every C_m.  With
    component densities mw, rho is the mass density sum_m mw_m C_m (eq.
    MassDensity)."""
    C1, C2, C3 = (np.array(c, dtype=np.float64) for c in (C1, C2, C3))
    if perturb:
        g = rng(seed)
        C1 = C1 + g.uniform(-perturb, perturb, C1.shape)
        C2 = C2 + g.uniform(-perturb, perturb, C2.shape)
        C3 = C3 + g.uniform(-perturb, perturb, C3.shape)
    rho = mw[0] * C1 + mw[1] * C2 + mw[2] * C3
    out = dict(rho=rho, phi=C1 - C2, psi=C3)
    if u is not None:
        out["u"] = [np.full(rho.shape, float(c)) for c in u]
    return out


def capsule_at_interface(nx=128, ny=128, R=20.0, n_markers=128, centre=None, y0=None,
                         kappa=(0.02, 0.02, 0.02), alpha=1.0, kappa_c=0.01, kappa_s=0.01,
                         kappa_b=1e-4, wall_y=1, mobility=0.1, tau=1.0, tau_phi=1.0, tau_psi=1.0,
                         perturb=1e-4, seed=SEED_BASE, u0=None, r_cut=0.0, mw=(1.0, 1.0, 1.0)):
    """One capsule of fluid 3 centred on a flat C1/C2 interface at y = y0
    (C1 below, C2 above), in a box periodic in x (Sec. 4.1).  ``mw``:
    component densities (all 1 in the paper)."""
    if centre is None:
        centre = (nx / 2.0, (ny - 1) / 2.0)
    if y0 is None:
        y0 = centre[1]
    p = base_params(nx, ny, wall_y=wall_y, kappa=kappa, alpha=alpha, kappa_c=kappa_c, tau=tau,
                    tau_phi=tau_phi, tau_psi=tau_psi, mobility=mobility, r_cut=r_cut)
    x, y = _grid2(nx, ny)
    dx = _min_image(x - centre[0], nx)
    dy = y - centre[1] if wall_y else _min_image(y - centre[1], ny)
    C3 = tanh_profile(R - np.hypot(dx, dy), alpha)
    below = 0.5 * (1.0 - np.tanh((y - y0) / (2.0 * alpha)))
    if not wall_y:
        # periodic in y: a second interface half a box away keeps C1 a band
        dyy = _min_image(y - y0 + ny / 4.0, ny)
        below = tanh_profile(ny / 4.0 - np.abs(dyy), alpha)
    C1 = (1.0 - C3) * below
    C2 = 1.0 - C1 - C3
    fields = fields_from_C(C1, C2, C3, perturb, seed, u=(u0 if u0 is None else (u0, 0.0)), mw=mw)
    if tuple(mw) != (1.0, 1.0, 1.0):
        p["mw"] = [float(m) for m in mw]
    mem = [dict(X=circle_markers(centre[0], centre[1], R, n_markers), tris=None,
                kappa_s=kappa_s, kappa_b=kappa_b)]
    return dict(params=p, fields=fields, membranes=mem, name=f"capsule_at_interface_{nx}x{ny}")


def c1(seed=SEED_BASE + 0, **kw):
    """128x128 D2Q9, periodic x / walls y, lower half C1, upper half C2, one
    capsule R = 20 of 128 markers (shear modulus 0.01, bending 1e-4), tau 1,
    kappa 0.02 x3, alpha 1, mobility 0.1, +-1e-4 perturbation."""
    args = dict(nx=128, ny=128, R=20.0, n_markers=128, kappa=(0.02, 0.02, 0.02), alpha=1.0,
                kappa_c=0.01, kappa_s=0.01, kappa_b=1e-4, wall_y=1, mobility=0.1, perturb=1e-4,
                seed=seed)
    args.update(kw)
    w = capsule_at_interface(**args)
    w["name"] = "c1_capsule_128x128"
    return w


def c2(seed=SEED_BASE + 1, n=2048, n_caps=16, with_fields=True):
    """n x n D2Q9 (FP32 throughput workload), walls in y, flat C1/C2 interface
    at y0 = (n-1)/2, n_caps capsules with radii U[24, 64] laid left to right
    with equal gaps, markers clamp(ceil(2 pi R / 0.8), 256, 512), kappa_m
    U[0.01, 0.05], shear 0.01, bending 1e-4, alpha 1, mobility 0.1."""
    g = rng(seed)
    scale = n / 2048.0
    while True:
        R = g.uniform(24.0, 64.0, n_caps) * min(1.0, scale)
        gap = (n - 2.0 * R.sum()) / n_caps
        if gap >= 8.0:
            break
    kappa = g.uniform(0.01, 0.05, 3)
    y0 = (n - 1) / 2.0
    p = base_params(n, n, wall_y=1, kappa=kappa, alpha=1.0, kappa_c=0.01, mobility=0.1)
    cx = []
    pos = gap / 2.0
    for r in R:
        cx.append(pos + r)
        pos += 2.0 * r + gap
    mems = []
    for k in range(n_caps):
        nm = int(min(512, max(256, math.ceil(2.0 * math.pi * R[k] / 0.8))))
        mems.append(dict(X=circle_markers(cx[k], y0, R[k], nm), tris=None, kappa_s=0.01,
                         kappa_b=1e-4))
    w = dict(params=p, membranes=mems, name=f"c2_{n_caps}caps_{n}x{n}")
    if with_fields:
        x, y = _grid2(n, n)
        C3 = np.zeros((n, n))
        for k in range(n_caps):
            C3 += tanh_profile(R[k] - np.hypot(_min_image(x - cx[k], n), y - y0), 1.0)
        C3 = np.minimum(C3, 1.0)
        below = 0.5 * (1.0 - np.tanh((y - y0) / 2.0))
        C1 = (1.0 - C3) * below
        C2 = 1.0 - C1 - C3
        w["fields"] = fields_from_C(C1, C2, C3, 1e-4, seed)
    return w


def mode_decay(mode, nx=96, ny=4, mobility=(0.3, 0.1), kappa=(0.05, 0.05, 0.08), alpha=1.0, tau_phi=0.8,
               tau_psi=1.3, amp=1e-5):
    """A uniform bulk phase with a small sinusoidal perturbation along x, one
    wavelength over the periodic box, for the decay rates of the order
    parameters (Sec. 2.6 mobilities): mode "phi" perturbs phi in the C3 bulk,
    mode "psi" perturbs psi in the C1 bulk (at fixed rho and phi).  No
    membrane, no coupling."""
    p = base_params(nx, ny, wall_y=0, kappa=kappa, alpha=alpha, kappa_c=0.0, tau_phi=tau_phi,
                    tau_psi=tau_psi, mobility=mobility)
    x, _ = _grid2(nx, ny)
    s = amp * np.sin(2.0 * np.pi * x / nx)
    rho = np.ones((ny, nx))
    if mode == "phi":
        phi, psi = s, np.ones((ny, nx))
    elif mode == "psi":
        phi, psi = np.ones((ny, nx)), s
    else:
        raise ValueError(mode)
    return dict(params=p, fields=dict(rho=rho, phi=phi, psi=psi), membranes=[],
                name=f"mode_decay_{mode}_{nx}x{ny}")


def prestressed_ring(law=0, n=64, R=12.0, n_markers=64, kappa_s=0.05, lam0=1.25, kappa=(1e-4, 1e-4, 1e-4)):
    """A ring of markers on a circle of radius R in a uniform fluid (C1, no
    coupling) whose rest lengths are the chords divided by lam0, so that it
    starts stretched by lam0 and pulls inward; strain law `law` (0 eq.
    DiscreteSE, 1 neo-Hookean, 2 Skalak).  Small kappa_m keep the non-ideal
    pressure negligible against the ring's pressure jump."""
    p = base_params(n, n, kappa=kappa, kappa_c=0.0, mobility=0.1)
    X = circle_markers(n / 2.0, n / 2.0, R, n_markers)
    rest = np.linalg.norm(np.roll(X, -1, axis=0) - X, axis=1) / lam0
    f = dict(rho=np.ones((n, n)), phi=np.ones((n, n)), psi=np.zeros((n, n)))
    mem = [dict(X=X, tris=None, kappa_s=kappa_s, kappa_b=0.0, rest=rest, law=int(law))]
    return dict(params=p, fields=f, membranes=mem, name=f"prestressed_ring_law{law}_{n}x{n}")


def shear_wave(ny=128, nx=4, U=1e-4, tau=1.0, kappa=(0.02, 0.02, 0.02), alpha=1.0, mobility=0.1):
    """A single bulk phase (C1 = 1) on a periodic nx x ny lattice carrying a
    small shear wave u_x = U sin(2 pi y / ny), u_y = 0: the wave decays at
    nu k^2 with the kinematic viscosity nu of eq. RelaxationTimes."""
    p = base_params(nx, ny, wall_y=0, kappa=kappa, alpha=alpha, kappa_c=0.0, tau=tau, mobility=mobility)
    _, y = _grid2(nx, ny)
    one = np.ones((ny, nx))
    f = fields_from_C(one, 0.0 * one, 0.0 * one)
    f["u"] = [U * np.sin(2.0 * np.pi * y / ny), 0.0 * one]
    return dict(params=p, fields=f, membranes=[], name=f"shear_wave_{nx}x{ny}_tau{tau:g}")


def forced_fluid(n=24, fext=(1e-5, -5e-6), tau=1.0, R=2.0, n_markers=12, kappa=(0.02, 0.02, 0.02)):
    """A single bulk phase (C1 = 1) at rest on a periodic n x n lattice under
    a uniform external force density f_ext (eq. ForcingTermLBE), with a
    force-free ring of markers (no stiffness, no coupling) carried by the
    fluid.  The coupling band is 1 (there is no coupling), so the ring's
    tile band fits the small periodic box."""
    p = base_params(n, n, wall_y=0, kappa=kappa, kappa_c=0.0, tau=tau, mobility=0.1, r_cut=1.0)
    p["fext"] = [float(v) for v in fext]
    one = np.ones((n, n))
    mem = [dict(X=circle_markers(n / 2.0 + 0.3, n / 2.0 - 0.2, R, n_markers), tris=None, kappa_s=0.0,
                kappa_b=0.0)]
    return dict(params=p, fields=fields_from_C(one, 0.0 * one, 0.0 * one), membranes=mem,
                name=f"forced_fluid_{n}x{n}_tau{tau:g}")


def flat(nx=4, ny=64, kappa=(0.02, 0.02, 0.02), alpha=1.0, mobility=0.1, wall_y=1, seed=None,
         mw=(1.0, 1.0, 1.0)):
    """Flat C1/C2 interface at y = (ny-1)/2, C1 below; no membrane.  ``mw``:
    component densities (all 1 in the paper)."""
    p = base_params(nx, ny, wall_y=wall_y, kappa=kappa, alpha=alpha, kappa_c=0.0, mobility=mobility)
    p["mw"] = [float(m) for m in mw]
    x, y = _grid2(nx, ny)
    y0 = (ny - 1) / 2.0
    if wall_y:
        C1 = 0.5 * (1.0 - np.tanh((y - y0) / (2.0 * alpha)))
    else:
        C1 = tanh_profile(ny / 4.0 - np.abs(_min_image(y - y0 + ny / 4.0, ny)), alpha)
    C2 = 1.0 - C1
    C3 = np.zeros_like(C1)
    return dict(params=p, fields=fields_from_C(C1, C2, C3, mw=mw), membranes=[], name="flat")


def drop(n=64, R=12.0, kappa=(0.02, 0.02, 0.02), alpha=1.0, mobility=0.1, mw=(1.0, 1.0, 1.0)):
    """C3 drop of radius R in C1, fully periodic box, no membrane.  ``mw``:
    component densities (all 1 in the paper)."""
    p = base_params(n, n, wall_y=0, kappa=kappa, alpha=alpha, kappa_c=0.0, mobility=mobility)
    p["mw"] = [float(m) for m in mw]
    x, y = _grid2(n, n)
    c = (n - 1) / 2.0
    C3 = tanh_profile(R - np.hypot(x - c, y - c), alpha)
    C1 = 1.0 - C3
    C2 = np.zeros_like(C1)
    return dict(params=p, fields=fields_from_C(C1, C2, C3, mw=mw), membranes=[], name="drop")


def lens(nx=120, ny=80, R=20.0, kappa=(0.02, 0.02, 0.02), alpha=1.0, mobility=0.1):
    """Pure liquid lens (Sec. 4.1, filled squares of Fig. 2): a circular C3 drop
    on a flat C1/C2 interface, walls in y, no membrane."""
    w = capsule_at_interface(nx=nx, ny=ny, R=R, n_markers=8, kappa=kappa, alpha=alpha, kappa_c=0.0,
                             wall_y=1, mobility=mobility, perturb=0.0)
    w["membranes"] = []
    w["name"] = "lens"
    return w


# ---------------------------------------------------------------------------
# 3D inputs
# ---------------------------------------------------------------------------
def icosphere(subdiv: int):
    """Unit icosphere: 10*4^k + 2 vertices, 20*4^k triangles, counter-clockwise
    seen from outside."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t),
         (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    V = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]

        nf = []
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = nf
    return np.array(V), np.array(F, dtype=np.int32)


def capsule3d(n=64, R=10.0, subdiv=3, kappa=(0.02, 0.02, 0.02), alpha=1.0, kappa_c=0.01,
              kappa_s=0.01, kappa_b=1e-3, mobility=0.1, two=True, bridge=True, perturb=1e-4,
              seed=SEED_BASE + 2, wall_z=1, r_cut=0.0, tau=1.0, shift=(0.0, 0.0, 0.0)):
    """D3Q19 box n^3 (periodic x, y; walls in z when wall_z): C2 below
    z0 = (n-1)/2, C1 above; two icosphere capsules of fluid 3 (radius R) side
    by side on the interface with a C2 bridge between them.  READING of the
    bridge: component 3 is reserved for capsule interiors by the coupling
    energy, so the bridge is component 2."""
    p = base_params(n, n, n, lattice=1, wall_y=0, wall_z=wall_z, kappa=kappa, alpha=alpha,
                    kappa_c=kappa_c, mobility=mobility, r_cut=r_cut, tau=tau)
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64),) * 3, indexing="ij")
    z0 = (n - 1) / 2.0
    yc = (n - 1) / 2.0 + 0.25
    if two:
        centres = [(n / 2.0 - 1.25 * R + 0.3, yc, z0 + 0.15), (n / 2.0 + 1.25 * R + 0.3, yc, z0 + 0.15)]
    else:
        centres = [(n / 2.0 + 0.3, yc, z0 + 0.15)]
    centres = [(c[0] + shift[0], c[1] + shift[1], c[2] + shift[2]) for c in centres]
    V, F = icosphere(subdiv)
    C3 = np.zeros(x.shape)
    mems = []
    for c in centres:
        d = R - np.sqrt(_min_image(x - c[0], n) ** 2 + _min_image(y - c[1], n) ** 2 + (z - c[2]) ** 2)
        C3 += tanh_profile(d, alpha)
        mems.append(dict(X=V * R + np.array(c), tris=F, kappa_s=kappa_s, kappa_b=kappa_b))
    C3 = np.minimum(C3, 1.0)
    below = 0.5 * (1.0 - np.tanh((z - z0) / (2.0 * alpha)))
    C2 = (1.0 - C3) * below
    if two and bridge:
        # a C2 column between the capsules, of half-width 0.6 R
        dxb = np.abs(x - n / 2.0 - 0.3) - 0.25 * R
        dyb = np.abs(y - yc) - 0.6 * R
        dzb = np.abs(z - z0) - 0.6 * R
        inside_box = -np.maximum(np.maximum(dxb, dyb), dzb)
        C2 = np.maximum(C2, (1.0 - C3) * tanh_profile(inside_box, alpha))
    C1 = 1.0 - C2 - C3
    return dict(params=p, fields=fields_from_C(C1, C2, C3, perturb, seed), membranes=mems,
                name=f"capsule3d_{n}")


def prestressed_mesh(law=1, n=40, R=10.0, subdiv=3, kappa_s=0.02, lam0=1.2, kappa=(1e-4, 1e-4, 1e-4)):
    """An icosphere mesh of radius R in a uniform fluid (C1, no coupling,
    periodic n^3 box) whose edge rest lengths are its edge lengths / lam0, so
    that it starts stretched equibiaxially by lam0; strain law `law`.  The
    rest lengths are listed per edge in (lower vertex, higher vertex) order."""
    # no coupling: a narrow band keeps the mesh's band inside the period
    p = base_params(n, n, n, lattice=1, kappa=kappa, kappa_c=0.0, mobility=0.1, r_cut=3.0)
    V, F = icosphere(subdiv)
    X = V * R + np.array([n / 2.0 + 0.3, n / 2.0 + 0.2, n / 2.0 + 0.1])
    keys = sorted({(min(int(t[k]), int(t[(k + 1) % 3])), max(int(t[k]), int(t[(k + 1) % 3])))
                   for t in F for k in range(3)})
    rest = np.array([np.linalg.norm(X[a] - X[b]) / lam0 for a, b in keys])
    f = dict(rho=np.ones((n, n, n)), phi=np.ones((n, n, n)), psi=np.zeros((n, n, n)))
    mem = [dict(X=X, tris=F, kappa_s=kappa_s, kappa_b=0.0, rest=rest, law=int(law))]
    return dict(params=p, fields=f, membranes=mem, name=f"prestressed_mesh_law{law}_{n}")


def drop3d(nx=24, ny=22, nz=20, R=6.0, wall_y=0, wall_z=1, kappa=(0.02, 0.03, 0.025), alpha=1.0,
           mobility=0.1, tau=1.0, tau_phi=1.0, tau_psi=1.0, u0=None, perturb=1e-4,
           seed=SEED_BASE + 4, mw=(1.0, 1.0, 1.0)):
    """D3Q19 box: a C3 sphere of radius R in C1, above a C2 layer of a third
    of the height (no membrane).  ``mw``: component densities (all 1 in the
    paper)."""
    p = base_params(nx, ny, nz, lattice=1, wall_y=wall_y, wall_z=wall_z, kappa=kappa, alpha=alpha,
                    kappa_c=0.0, mobility=mobility, tau=tau, tau_phi=tau_phi, tau_psi=tau_psi)
    if tuple(mw) != (1.0, 1.0, 1.0):
        p["mw"] = [float(m) for m in mw]
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    c = (nx / 2.0 + 0.2, ny / 2.0 - 0.3, 0.6 * nz)
    C3 = tanh_profile(R - np.sqrt(_min_image(x - c[0], nx) ** 2 + _min_image(y - c[1], ny) ** 2 +
                                  (z - c[2]) ** 2), alpha)
    C2 = (1.0 - C3) * 0.5 * (1.0 - np.tanh((z - nz / 3.0) / (2.0 * alpha)))
    C1 = 1.0 - C2 - C3
    return dict(params=p, fields=fields_from_C(C1, C2, C3, perturb, seed, u=u0, mw=mw), membranes=[],
                name=f"drop3d_{nx}x{ny}x{nz}")


def sphere3d(n=64, R=16.0, kappa=(0.02, 0.02, 0.02), alpha=1.0, mobility=0.1):
    """D3Q19 n^3, periodic: a C3 sphere of radius R centred in C1 (no C2)."""
    p = base_params(n, n, n, lattice=1, wall_y=0, wall_z=0, kappa=kappa, alpha=alpha, kappa_c=0.0,
                    mobility=mobility)
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64),) * 3, indexing="ij")
    c = (n - 1) / 2.0
    C3 = tanh_profile(R - np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2), alpha)
    return dict(params=p, fields=fields_from_C(1.0 - C3, np.zeros_like(C3), C3), membranes=[],
                name=f"sphere3d_{n}")


def lens3d(n=64, R=16.0, kappa=(0.02, 0.02, 0.02), alpha=1.0, mobility=0.1, wall_z=1):
    """D3Q19 n^3: a C3 sphere centred on a flat C1/C2 interface at
    z0 = (n-1)/2 (C1 below, C2 above), periodic in x and y."""
    p = base_params(n, n, n, lattice=1, wall_y=0, wall_z=wall_z, kappa=kappa, alpha=alpha,
                    kappa_c=0.0, mobility=mobility)
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64),) * 3, indexing="ij")
    c = (n - 1) / 2.0
    C3 = tanh_profile(R - np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2), alpha)
    C1 = (1.0 - C3) * 0.5 * (1.0 - np.tanh((z - c) / (2.0 * alpha)))
    C2 = 1.0 - C1 - C3
    return dict(params=p, fields=fields_from_C(C1, C2, C3), membranes=[], name=f"lens3d_{n}")


def c3(n=256, **kw):
    """D3Q19 at n^3 with two icosphere capsules of radius n/6.4 (40 at 256^3,
    10 at 64^3) and 5120 triangles, bridged by C2 between them."""
    R = n / 6.4
    return capsule3d(n=n, R=R, subdiv=4, **kw)


def c4(seed=SEED_BASE + 3, count=64):
    """Batch of capsule-at-interface runs: square sides 16*U_int[6, 32], radius
    U[12, min(48, n/4)], markers clamp(ceil(2 pi R/0.8), 64, 384), kappa_m
    U[0.01, 0.05], shear log-U[1e-3, 1e-1], bending log-U[1e-5, 1e-3]."""
    g = rng(seed)
    out = []
    for k in range(count):
        n = 16 * int(g.integers(6, 33))
        R = float(g.uniform(12.0, min(48.0, 0.25 * n)))
        nm = int(min(384, max(64, math.ceil(2 * math.pi * R / 0.8))))
        kap = g.uniform(0.01, 0.05, 3)
        ks = float(10 ** g.uniform(-3, -1))
        kb = float(10 ** g.uniform(-5, -3))
        w = capsule_at_interface(nx=n, ny=n, R=R, n_markers=nm, kappa=kap, alpha=1.0, kappa_c=0.01,
                                 kappa_s=ks, kappa_b=kb, wall_y=1, mobility=0.1, perturb=1e-4,
                                 seed=seed * 1000 + k)
        w["name"] = f"c4_{k}_{n}"
        out.append(w)
    return out


# the three tension ratios of the capillary-bridge study (Sec. 4.2): kappa_1
# with kappa_2 = 3e-3 and kappa_3 = 6e-3
# capsule at a fluid-fluid interface (Sec. 4.1): kappa_3 sweeps of the
# symmetric (kappa_1 = kappa_2 = 8e-3) and asymmetric (kappa_1 = 8e-3,
# kappa_2 = 2e-3) cases, and the (kappa_s, kappa_b) pairs
TAYLOR_KAPPA3_SYM = tuple(round(5e-4 * k, 6) for k in range(1, 21))
TAYLOR_KAPPA3_ASYM = tuple(round(5e-4 * k, 6) for k in range(1, 17))
TAYLOR_MODULI = ((1e-3, 1e-4), (1e-3, 1e-2), (1e-2, 1e-4), (1e-2, 1e-2), (1e-1, 1e-4), (1e-1, 1e-2))


def taylor2d(kappa3, kappa_s, kappa_b, symmetric=True, R=20.0, n_markers=160, alpha=2.0, kappa_c=1e-2,
             mobility=0.1, seed=SEED_BASE + 7, offset=(0.0, 0.0), u0=None):
    """Capsule at a fluid-fluid interface as in Sec. 4.1: an initially
    circular capsule of radius R at the centre of a 12R x 6R box periodic in
    both directions, on a flat C1/C2 interface (C1 below), alpha 2, kappa_c
    1e-2; kappa_1 = kappa_2 = 8e-3 (symmetric) or kappa_1 = 8e-3, kappa_2 =
    2e-3 (asymmetric).  The band is 12 alpha wide, so that the band of a
    deformed capsule fits in the 6R-high box.  `offset` moves the capsule
    and the interface off the lattice's symmetry lines; `u0` gives every
    fluid an initial horizontal velocity (the moving frames of Sec. 4.1)."""
    kappa = (8e-3, 8e-3 if symmetric else 2e-3, float(kappa3))
    nx, ny = int(12 * R), int(6 * R)
    centre = (nx / 2.0 + offset[0], (ny - 1) / 2.0 + offset[1])
    w = capsule_at_interface(nx=nx, ny=ny, R=R, n_markers=n_markers, kappa=kappa, centre=centre,
                             alpha=alpha, kappa_c=kappa_c, kappa_s=kappa_s, kappa_b=kappa_b, wall_y=0,
                             mobility=mobility, seed=seed, r_cut=12.0 * alpha, u0=u0)
    w["name"] = f"taylor_{'sym' if symmetric else 'asym'}_k3_{kappa3:g}_ks_{kappa_s:g}_kb_{kappa_b:g}"
    return w


BRIDGE_KAPPA1 = (1e-3, 3e-3, 9e-3)
BRIDGE_KAPPA_S = (1e-4, 1e-3, 1e-2, 1e-1, 1.0)


def bridge2d(kappa1=3e-3, kappa_s=1e-2, R=20.0, n_markers=160, kappa_b=1e-2, kappa_c=1e-2, alpha=2.0,
             mobility=0.1, offset=(0.0, 0.0)):
    """Capillary bridge between two capsules (Sec. 4.2, Fig. 1b): a periodic
    12R x 6R box of fluid 1; capsules of fluid 3 with radius R centred at
    (9R/2, 3R) and (15R/2, 3R); between them a rectangle of fluid 2, 2S = R
    wide and H_b = 31R/10 high, centred in the box.  kappa_2 = 3e-3,
    kappa_3 = 6e-3, alpha = 2, kappa_b = kappa_c = 1e-2 as in the paper; the
    rectangle's diffuse edge is the product of two tanh profiles.  No
    perturbation: the set-up is mirror-symmetric about x = 6R.  ``offset``
    shifts the whole set-up off the lattice (a node at a capsule centre is
    equidistant from opposite membrane segments, and with a band wider than
    R such exact ties are decided by the last bit of each implementation's
    rounding)."""
    nx, ny = int(round(12 * R)), int(round(6 * R))
    # band 12 alpha: the profile is saturated to 6e-6 there, and an elongated
    # capsule's band (height + 2 reach) still fits the 6R-high periodic box
    p = base_params(nx, ny, wall_y=0, kappa=(kappa1, 3e-3, 6e-3), alpha=alpha, kappa_c=kappa_c,
                    mobility=mobility, r_cut=12.0 * alpha)
    x, y = _grid2(nx, ny)
    ox, oy = (float(v) for v in offset)
    centres = ((4.5 * R + ox, 3.0 * R + oy), (7.5 * R + ox, 3.0 * R + oy))
    C3 = np.zeros((ny, nx))
    for cx, cy in centres:
        C3 += tanh_profile(R - np.hypot(_min_image(x - cx, nx), _min_image(y - cy, ny)), alpha)
    half_w, half_h = 0.5 * R, 0.5 * 3.1 * R
    rect = tanh_profile(half_w - np.abs(_min_image(x - 6.0 * R - ox, nx)), alpha) * \
        tanh_profile(half_h - np.abs(_min_image(y - 3.0 * R - oy, ny)), alpha)
    C2 = rect * (1.0 - C3)
    C1 = 1.0 - C2 - C3
    mems = [dict(X=circle_markers(cx, cy, R, n_markers), tris=None, kappa_s=float(kappa_s),
                 kappa_b=float(kappa_b)) for cx, cy in centres]
    return dict(params=p, fields=fields_from_C(C1, C2, C3), membranes=mems, R=float(R),
                name=f"bridge2d_k1_{kappa1:g}_ks_{kappa_s:g}")


def aspect_ratio(X):
    """L_c / H_c of a capsule from its markers (n, 2): horizontal extent over
    vertical extent."""
    X = np.asarray(X, dtype=np.float64)
    return float((X[:, 0].max() - X[:, 0].min()) / (X[:, 1].max() - X[:, 1].min()))

