"""Shared helpers of the GPU parity tests: run the oracle and the HIP
library on the same seeded workload and compare."""
import numpy as np

FIELDS = ("rho", "c1", "c2", "c3", "ux", "uy")


def normwise(a, b):
    """max |a - b| / max |b| (the field error measure of the parity bar)."""
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def normwise_dev(a, b):
    """max |a - b| / max |b - mean(b)|: the error of a field measured against
    its variation (rho is 1 up to ~1e-3, so normwise() against max |rho|
    would be an absolute bar)."""
    den = np.abs(b - b.mean()).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


GPU_DEFAULT_BAND = 17.0  # the library's coupling band for r_cut <= 0, in units of alpha


def oracle_params(p, untruncated=False):
    """Parameters for the oracle.  The oracle takes r_cut <= 0 as no band at
    all (the profile of eq. Iprofile everywhere); the library as a band of
    17 alpha.  By default the oracle is given the library's band, so the
    comparison checks the same reading; untruncated=True keeps the paper's
    profile with no band."""
    q = dict(p)
    if not untruncated and q.get("r_cut", 0.0) <= 0.0:
        q["r_cut"] = GPU_DEFAULT_BAND * q.get("alpha", 1.0)
    return q


def run_oracle(orc, w, untruncated=False):
    s = orc.Sim(oracle_params(w["params"], untruncated))
    for m in w["membranes"]:
        i = s.add_membrane(m["X"], m.get("tris"), m["kappa_s"], m["kappa_b"])
        if m.get("rest") is not None:
            s.set_rest(i, m["rest"])
        if m.get("law", 0):
            s.set_membrane_law(i, m["law"])
    f = w["fields"]
    s.set_fields(f["rho"], f["phi"], f["psi"], f.get("u"))
    return s


def run_gpu(w, storage="fp32", **kw):
    from paper_1906_03065_amd import lbib

    return lbib.from_workload(w, storage=storage, **kw)


def compare(g, o, D=2):
    fg, fo = g.fields(), o.fields()
    keys = FIELDS if D == 2 else FIELDS + ("uz",)
    return {k: normwise(fg[k], fo[k]) for k in keys}


def rho_dev_err(g, o):
    """error of rho measured against the variation of the oracle's rho"""
    return normwise_dev(g.fields()["rho"], o.fields()["rho"])


def marker_err(g, o, n_mem):
    e = 0.0
    for i in range(n_mem):
        e = max(e, float(np.abs(g.membrane(i)["X"] - o.membrane(i)["X"]).max()))
    return e


def pressure(f, kap):
    """p = sum_m C_m dF/dC_m - f + c_s^2 rho with the Landau energy (the
    bulk pressure definition), evaluated from concentration fields."""
    C = [f["c1"], f["c2"], f["c3"]]
    p = f["rho"] / 3.0
    for k, c in zip(kap, C):
        p = p + c * k * c * (1 - c) * (1 - 2 * c) - 0.5 * k * c * c * (1 - c) ** 2
    return p


def contour(c3, level=0.5):
    """Points where a 2D field crosses level, from row and column scans."""
    pts = []
    a = c3 - level
    for y in range(a.shape[0]):
        r = a[y]
        for i in np.where(np.sign(r[:-1]) != np.sign(r[1:]))[0]:
            pts.append((i + r[i] / (r[i] - r[i + 1]), y))
    for x in range(a.shape[1]):
        c = a[:, x]
        for i in np.where(np.sign(c[:-1]) != np.sign(c[1:]))[0]:
            pts.append((x, i + c[i] / (c[i] - c[i + 1])))
    return np.array(pts)


def lens_angles(c3, y0, margin=4.0):
    """Cap angles of a lens at y = y0 from circle fits to the C3 = 1/2 contour
    above and below the interface."""
    P = contour(c3)

    def circ(Q):
        A = np.c_[2 * Q[:, 0], 2 * Q[:, 1], np.ones(len(Q))]
        s = np.linalg.lstsq(A, (Q ** 2).sum(1), rcond=None)[0]
        return s[0], s[1], np.sqrt(s[2] + s[0] ** 2 + s[1] ** 2)

    _, yu, ru = circ(P[P[:, 1] > y0 + margin])
    _, yd, rd = circ(P[P[:, 1] < y0 - margin])
    return np.degrees(np.arccos((y0 - yu) / ru)), np.degrees(np.arccos((yd - y0) / rd))


def mode_amplitude(f, mode):
    """Amplitude of the sin(2 pi x / nx) component of phi = C1 - C2 (mode
    "phi") or psi = C3 (mode "psi") on the first row."""
    q = (f["c1"] - f["c2"]) if mode == "phi" else f["c3"]
    nx = q.shape[1]
    return 2.0 * float(np.mean(q[0] * np.sin(2.0 * np.pi * np.arange(nx) / nx)))


def decay_rate(sim, mode, steps=3600, every=450, skip=2):
    """Exponential decay rate per step of a mode_decay workload's perturbation,
    fitted to its amplitude every `every` steps after the first `skip`."""
    t, a = [], []
    for n in range(0, steps + 1, every):
        sim.step(n - sim.steps_done)
        t.append(n)
        a.append(abs(mode_amplitude(sim.fields(), mode)))
    return -float(np.polyfit(t[skip:], np.log(a[skip:]), 1)[0])


def ch_rate(p, mode, density_response=True):
    """Decay rate of a small sin(k x) perturbation in a bulk phase from the
    linearised Cahn-Hilliard equation dq/dt = M lap mu_q (Sec. 2.6), with
    M = Gamma (tau - 1/2) and the chemical potentials of the Landau energy:
    about C = 0 or 1, d/dC [C (1 - C)(1 - 2C)] = 1, so each concentration's
    b_m = kappa_m (1 + alpha^2 K) dC_m, where K = 2 (1 - cos k) is the
    isotropic Laplacian stencil's eigenvalue for a wave along x.
      phi in the C3 bulk: dC1 = -dC2 = dphi/2, mu_phi = (b1 - b2)/2 gives
      rate = M_phi K (kappa1 + kappa2)/4 (1 + alpha^2 K); with kappa1 =
      kappa2 no other field is driven.
      psi in the C1 bulk (phi fixed, kappa1 = kappa2): dC1 = dC2 =
      (drho - dpsi)/2, so mu_rho = A (drho - dpsi) with A = (kappa1 +
      kappa2)/4 (1 + alpha^2 K); the fluid balances it with its pressure,
      c_s^2 grad drho = -grad mu_rho, i.e. drho = 3 A dpsi / (1 + 3 A), and
      mu_psi = b3 - (b1 + b2)/2 = [kappa3 (1 + alpha^2 K) + A / (1 + 3 A)] dpsi.
    density_response=False drops the pressure balance (drho = 0)."""
    nx = p["nx"]
    K = 2.0 * (1.0 - np.cos(2.0 * np.pi / nx))
    k1, k2, k3 = p["kappa"]
    a2 = p["alpha"] ** 2
    if mode == "phi":
        M = p["gamma_phi"] * (p["tau_phi"] - 0.5)
        return M * K * (k1 + k2) / 4.0 * (1.0 + a2 * K)
    M = p["gamma_psi"] * (p["tau_psi"] - 0.5)
    A = (k1 + k2) / 4.0 * (1.0 + a2 * K)
    extra = A / (1.0 + 3.0 * A) if density_response else A
    return M * K * (k3 * (1.0 + a2 * K) + extra)


def ring_law_tension(law, ks, lam):
    """dW/dlam of the ring strain laws, from the general membrane laws at
    plane strain: neo-Hookean G/2 (l1^2 + l2^2 + (l1 l2)^-2 - 3) with G = ks/4,
    Skalak G/4 (I1^2 + 2 I1 - 2 I2 + C I2^2) with G (1 + C) = ks/2, and the
    paper's ks/2 (lam - 1)^2, differentiated by hand at l2 = 1."""
    if law == 1:
        return ks / 4.0 * (lam - lam ** -3)
    if law == 2:
        return ks / 2.0 * (lam ** 3 - lam)
    return ks * (lam - 1.0)


def ring_laplace(sim, w, n_markers_mem=0):
    """(pressure jump across a prestressed ring measured between the box
    centre and corner, T(lam)/R from its current mean radius)."""
    f = sim.fields()
    n = w["params"]["nx"]
    m = w["membranes"][0]
    X = sim.membrane(0)["X"][:, :2]
    Rm = float(np.linalg.norm(X - n / 2.0, axis=1).mean())
    R0 = float(np.linalg.norm(m["X"] - n / 2.0, axis=1).mean())
    lam = Rm / R0 * float(np.mean(np.linalg.norm(np.roll(m["X"], -1, axis=0) - m["X"], axis=1) / m["rest"]))
    dp = (f["rho"][n // 2, n // 2] - f["rho"][0, 0]) / 3.0
    return dp, ring_law_tension(m["law"], m["kappa_s"], lam) / Rm
