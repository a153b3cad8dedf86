"""Plain FP64 CPU oracle of the ternary free-energy LB + IBM step.

TEST INFRASTRUCTURE ONLY.  The oracle checks the HIP library against the
paper (Pepona et al., "Modelling ternary fluids in contact with elastic
membranes").  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product package never
does.  It shares no code with the HIP path: the C source ``orc.c`` is built
on its own with ``gcc`` into ``liborc.so`` and bound here with ctypes.

Every function of ``orc.c`` cites the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

# built with no fast-math and no contraction, so every operation rounds as written
CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
          "-ffp-contract=off", "-Wall", "-Wno-unused-function"]


def build(force: bool = True) -> str:
    """Compile ``orc.c`` into ``liborc.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("lattice", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("wall_y", C.c_int), ("wall_z", C.c_int),
                ("tau", C.c_double), ("tau_phi", C.c_double), ("tau_psi", C.c_double),
                ("gamma_phi", C.c_double), ("gamma_psi", C.c_double),
                ("kappa1", C.c_double), ("kappa2", C.c_double), ("kappa3", C.c_double),
                ("alpha", C.c_double), ("kappa_c", C.c_double), ("r_cut", C.c_double),
                ("force_form", C.c_int), ("fext", C.c_double * 3), ("mw", C.c_double * 3)]


class Energy(C.Structure):
    _fields_ = [("mass", C.c_double * 3), ("F_bulk", C.c_double), ("F_grad", C.c_double),
                ("E_c", C.c_double), ("E_s", C.c_double), ("E_b", C.c_double),
                ("E_kin", C.c_double), ("p_ideal", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "mass"}
        d["mass"] = list(self.mass)
        return d


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(Params)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_add_membrane.argtypes = [C.c_void_p, C.c_int, _dp, C.c_int, _ip, C.c_double, C.c_double]
        L.orc_set_fields.argtypes = [C.c_void_p] + [_dp] * 6
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_steps_done.restype = C.c_long
        L.orc_steps_done.argtypes = [C.c_void_p]
        L.orc_get_fields.argtypes = [C.c_void_p] + [_dp] * 7
        L.orc_get_membrane.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
        L.orc_energy.argtypes = [C.c_void_p, C.POINTER(Energy)]
        L.orc_peskin.restype = C.c_double
        L.orc_peskin.argtypes = [C.c_double]
        L.orc_lattice.argtypes = [C.c_int, _ip, _ip, _dp]
        L.orc_feq.argtypes = [C.c_int, C.c_double, _dp, _dp]
        L.orc_geq.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _dp, _dp]
        L.orc_mu.argtypes = [C.POINTER(Params)] + [C.c_double] * 7 + [_dp]
        L.orc_mu_general.argtypes = [C.POINTER(Params)] + [C.c_double] * 7 + [_dp]
        L.orc_concentrations.argtypes = [C.POINTER(Params), C.c_double, C.c_double, C.c_double, _dp]
        L.orc_collide.argtypes = [C.POINTER(Params), _dp, _dp, C.c_double, C.c_double, _dp]
        L.orc_grad_lap.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_ring_forces.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, _dp, _dp, _dp]
        L.orc_ring_forces_law.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_int, _dp, _dp,
                                          _dp]
        L.orc_set_membrane_law.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.orc_mesh_forces_law.argtypes = [C.c_int, _dp, C.c_int, _ip, _dp, C.c_double, C.c_double, C.c_int,
                                          _dp, _dp, _dp]
        L.orc_set_rest.argtypes = [C.c_void_p, C.c_int, _dp]
        L.orc_mesh_forces.argtypes = [C.c_int, _dp, C.c_int, _ip, _dp, C.c_double, C.c_double,
                                      _dp, _dp, _dp]
        L.orc_coupling.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.orc_spread.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
        L.orc_interp.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
        L.orc_pressure_tensor.argtypes = [C.POINTER(Params), C.c_int, _dp, _dp, _dp, _dp]
        L.orc_fe_force.argtypes = [C.c_void_p, C.c_int, _dp]
        _lib = L
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def make_params(p: dict) -> Params:
    return Params(int(p.get("lattice", 0)), int(p["nx"]), int(p["ny"]), int(p.get("nz", 1)),
                  int(p.get("wall_y", 0)), int(p.get("wall_z", 0)),
                  float(p.get("tau", 1.0)), float(p.get("tau_phi", 1.0)), float(p.get("tau_psi", 1.0)),
                  float(p.get("gamma_phi", 1.0)), float(p.get("gamma_psi", 1.0)),
                  float(p["kappa"][0]), float(p["kappa"][1]), float(p["kappa"][2]),
                  float(p.get("alpha", 1.0)), float(p.get("kappa_c", 0.0)), float(p.get("r_cut", 0.0)),
                  int(p.get("force_form", 0)),
                  (C.c_double * 3)(*[float(v) for v in (list(p.get("fext", ())) + [0.0, 0.0, 0.0])[:3]]),
                  (C.c_double * 3)(*[float(v) for v in (list(p.get("mw", ())) + [1.0, 1.0, 1.0])[:3]]))


def pressure_tensor(p: dict, q, g, l, D: int = 2):
    """Pressure tensor p' of Appendix A (no ideal gas) at one point: q the
    three values (rho, phi, psi), g their gradients (3 x 3, row q), l their
    Laplacians.  Returns a 3 x 3 array."""
    prm = make_params(p)
    P = np.zeros(9)
    gg = np.zeros((3, 3))
    gg[:, :np.asarray(g).shape[1]] = np.asarray(g, dtype=np.float64)
    if lib().orc_pressure_tensor(C.byref(prm), int(D), _d(_f64(q)), _d(np.ascontiguousarray(gg.reshape(-1))),
                                  _d(_f64(l)), _d(P)):
        raise ValueError("orc_pressure_tensor failed")
    return P.reshape(3, 3)


def set_threads(n: int = 0) -> int:
    return lib().orc_set_threads(int(n))


class Sim:
    """One oracle simulation.  ``p`` is the parameter dict used across the
    project (keys of :class:`Params`, with ``kappa`` a 3-list)."""

    def __init__(self, p: dict):
        self.p = dict(p)
        self.params = make_params(p)
        self.D = 3 if self.params.lattice == 1 else 2
        self.shape = (self.params.nz, self.params.ny, self.params.nx) if self.D == 3 else \
            (self.params.ny, self.params.nx)
        self.N = int(np.prod(self.shape))
        self.h = lib().orc_create(C.byref(self.params))
        if not self.h:
            raise ValueError("orc_create rejected the parameters")
        self.mem_sizes = []

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def add_membrane(self, X, tris=None, kappa_s=0.0, kappa_b=0.0) -> int:
        X = _f64(X).reshape(-1, self.D)
        n = X.shape[0]
        if tris is None:
            r = lib().orc_add_membrane(self.h, n, _d(X), 0, None, kappa_s, kappa_b)
        else:
            t = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
            r = lib().orc_add_membrane(self.h, n, _d(X), t.shape[0], t.ctypes.data_as(_ip),
                                       kappa_s, kappa_b)
        if r < 0:
            raise ValueError(f"orc_add_membrane failed ({r})")
        self.mem_sizes.append(n)
        return r

    def set_membrane_law(self, id: int, law: int):
        """Strain law of ring id: 0 eq. DiscreteSE, 1 neo-Hookean, 2 Skalak."""
        if lib().orc_set_membrane_law(self.h, int(id), int(law)):
            raise ValueError("orc_set_membrane_law failed")

    def set_rest(self, id: int, rest):
        """Rest lengths of membrane id: 2D one per segment l -> l+1; 3D one
        per edge in order of first appearance over the triangles' edges."""
        rest = _f64(rest).reshape(-1)
        if (self.D == 2 and rest.size != self.mem_sizes[id]) or lib().orc_set_rest(self.h, int(id), _d(rest)):
            raise ValueError("orc_set_rest failed")

    def set_fields(self, rho, phi, psi, u=None):
        rho, phi, psi = (_f64(a).reshape(-1) for a in (rho, phi, psi))
        comps = [None, None, None]
        if u is not None:
            for a in range(self.D):
                comps[a] = _f64(u[a]).reshape(-1)
        r = lib().orc_set_fields(self.h, _d(rho), _d(phi), _d(psi), *(_d(c) for c in comps))
        if r:
            raise ValueError(f"orc_set_fields failed ({r})")

    def step(self, n: int = 1):
        if lib().orc_step(self.h, int(n)):
            raise RuntimeError("orc_step failed")

    @property
    def steps_done(self) -> int:
        return lib().orc_steps_done(self.h)

    def fields(self) -> dict:
        out = {k: np.empty(self.N) for k in ("rho", "c1", "c2", "c3", "ux", "uy", "uz")}
        lib().orc_get_fields(self.h, *(_d(out[k]) for k in ("rho", "c1", "c2", "c3", "ux", "uy", "uz")))
        res = {k: v.reshape(self.shape) for k, v in out.items()}
        if self.D == 2:
            res.pop("uz")
        return res

    def membrane(self, i: int) -> dict:
        n = self.mem_sizes[i]
        X, U, F = (np.empty((n, self.D)) for _ in range(3))
        lib().orc_get_membrane(self.h, i, _d(X), _d(U), _d(F))
        return {"X": X, "U": U, "F": F}

    def energy(self) -> dict:
        e = Energy()
        lib().orc_energy(self.h, C.byref(e))
        return e.as_dict()

    # ---- pieces for unit pins ----
    def fe_force(self, form: int):
        """Free-energy force of the current populations (no coupling or
        membrane force): form 0 potential, 1 divergence of the pressure
        tensor; shape (N, 3)."""
        F = np.zeros(3 * self.N)
        if lib().orc_fe_force(self.h, int(form), _d(F)):
            raise ValueError("orc_fe_force failed")
        return F.reshape(self.N, 3)

    def grad_lap(self, q):
        q = _f64(q).reshape(-1)
        g = np.empty(self.N * self.D)
        l = np.empty(self.N)
        lib().orc_grad_lap(self.h, _d(q), _d(g), _d(l))
        return g.reshape(self.shape + (self.D,)), l.reshape(self.shape)

    def coupling(self, psi):
        psi = _f64(psi).reshape(-1)
        I = np.empty(self.N)
        nm = sum(self.mem_sizes)
        Fc = np.empty(max(nm, 1) * 3)
        E = C.c_double(0.0)
        lib().orc_coupling(self.h, _d(psi), _d(I), _d(Fc), C.byref(E))
        return I.reshape(self.shape), Fc[: 3 * nm].reshape(-1, 3)[:, : self.D], E.value

    def spread(self, X, F):
        X = _f64(X).reshape(-1, self.D)
        F = _f64(F).reshape(-1, self.D)
        out = np.empty(self.N * self.D)
        lib().orc_spread(self.h, X.shape[0], _d(X), _d(F), _d(out))
        return out.reshape(self.shape + (self.D,))

    def interp(self, X, v):
        X = _f64(X).reshape(-1, self.D)
        v = _f64(v).reshape(-1)
        U = np.empty(X.shape[0] * self.D)
        lib().orc_interp(self.h, X.shape[0], _d(X), _d(v), _d(U))
        return U.reshape(-1, self.D)


def peskin(r: float) -> float:
    return lib().orc_peskin(float(r))


def lattice(kind: int = 0):
    Q = C.c_int(0)
    c = np.zeros(19 * 3, dtype=np.int32)
    w = np.zeros(19)
    lib().orc_lattice(kind, C.byref(Q), c.ctypes.data_as(_ip), _d(w))
    q = Q.value
    return c[: 3 * q].reshape(q, 3).copy(), w[:q].copy()


def feq(kind, rho, u):
    c, w = lattice(kind)
    out = np.empty(len(w))
    uu = np.zeros(3)
    uu[: len(u)] = u
    lib().orc_feq(kind, float(rho), _d(uu), _d(out))
    return out


def geq(kind, q, mu, Gamma, v):
    c, w = lattice(kind)
    out = np.empty(len(w))
    vv = np.zeros(3)
    vv[: len(v)] = v
    lib().orc_geq(kind, float(q), float(mu), float(Gamma), _d(vv), _d(out))
    return out


def mu(p: dict, rho, phi, psi, lap_rho, lap_phi, lap_psi, I=0.0):
    out = np.empty(3)
    prm = make_params(p)
    lib().orc_mu(C.byref(prm), rho, phi, psi, lap_rho, lap_phi, lap_psi, I, _d(out))
    return out


def mu_general(p: dict, rho, phi, psi, lap_rho, lap_phi, lap_psi, I=0.0):
    out = np.empty(3)
    prm = make_params(p)
    lib().orc_mu_general(C.byref(prm), rho, phi, psi, lap_rho, lap_phi, lap_psi, I, _d(out))
    return out


def concentrations(p: dict, rho, phi, psi):
    out = np.empty(3)
    prm = make_params(p)
    lib().orc_concentrations(C.byref(prm), rho, phi, psi, _d(out))
    return out


def collide(p: dict, pops, F, mu_phi, mu_psi):
    """One collision of a node's populations pops = (f, g, h), each length Q."""
    prm = make_params(p)
    pin = np.ascontiguousarray(np.concatenate([np.asarray(x, float) for x in pops]))
    q = pin.size // 3
    FF = np.zeros(3)
    FF[: len(F)] = F
    out = np.empty(3 * q)
    lib().orc_collide(C.byref(prm), _d(pin), _d(FF), float(mu_phi), float(mu_psi), _d(out))
    return out[:q], out[q:2 * q], out[2 * q:]


def ring_forces(X, rest, kappa_s, kappa_b, law=0):
    X = _f64(X).reshape(-1, 2)
    n = X.shape[0]
    rest = _f64(rest).reshape(-1)
    F = np.empty((n, 2))
    es, eb = C.c_double(), C.c_double()
    r = lib().orc_ring_forces_law(n, _d(X), _d(rest), kappa_s, kappa_b, int(law), _d(F), C.byref(es),
                                  C.byref(eb))
    if r:
        raise ValueError("orc_ring_forces failed")
    return F, es.value, eb.value


def mesh_forces(X, tris, rest_edge, kappa_s, kappa_b, law=0):
    X = _f64(X).reshape(-1, 3)
    t = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    rest_edge = _f64(rest_edge).reshape(-1)
    F = np.empty((X.shape[0], 3))
    es, eb = C.c_double(), C.c_double()
    r = lib().orc_mesh_forces_law(X.shape[0], _d(X), t.shape[0], t.ctypes.data_as(_ip), _d(rest_edge),
                                  kappa_s, kappa_b, int(law), _d(F), C.byref(es), C.byref(eb))
    if r:
        raise ValueError("orc_mesh_forces failed")
    return F, es.value, eb.value
