"""ctypes binding of the HIP library ``liblbib.so`` (C ABI in include/lbib.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch supplies the device workspace (one uint8 tensor) and
the stream.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbib.so")

D2Q9, D3Q19 = 0, 1
FP32, FP16, BF16, FP64 = 0, 1, 2, 3
STORAGE = {"fp32": FP32, "fp16": FP16, "bf16": BF16, "fp64": FP64}

OK, EINVAL, ENOMEM, EHIP, ENONFINITE, EUNSTABLE, ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS = {0: "LBIB_OK", -1: "LBIB_EINVAL", -2: "LBIB_ENOMEM", -3: "LBIB_EHIP",
          -4: "LBIB_ENONFINITE", -5: "LBIB_EUNSTABLE", -6: "LBIB_ESTATE"}


class LbibError(RuntimeError):
    def __init__(self, fn, code):
        self.code = code
        super().__init__(f"{fn} failed: {STATUS.get(code, code)}")


class Params(C.Structure):
    _fields_ = [("lattice", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("wall_y", C.c_int), ("wall_z", C.c_int),
                ("tau", C.c_double), ("tau_phi", C.c_double), ("tau_psi", C.c_double),
                ("gamma_phi", C.c_double), ("gamma_psi", C.c_double),
                ("kappa", C.c_double * 3), ("alpha", C.c_double), ("kappa_c", C.c_double),
                ("r_cut", C.c_double), ("storage", C.c_int), ("max_markers", C.c_int),
                ("max_elems", C.c_int), ("max_membranes", C.c_int)]


class Energies(C.Structure):
    _fields_ = [("mass", C.c_double * 3), ("F_bulk", C.c_double), ("F_grad", C.c_double),
                ("E_c", C.c_double), ("E_s", C.c_double), ("E_b", C.c_double),
                ("E_kin", C.c_double), ("p_ideal", C.c_double)]


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_fp = C.POINTER(C.c_float)
_vp = C.c_void_p

# (name, restype, argtypes) of every entry point declared in include/lbib.h
SIGNATURES = [
    ("lbib_workspace_bytes", C.c_int, [C.POINTER(Params), C.POINTER(C.c_size_t)]),
    ("lbib_create", C.c_int, [C.POINTER(Params), _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    ("lbib_add_membrane", C.c_int, [_vp, C.c_int, _dp, C.c_int, _ip, C.c_double, C.c_double, _ip]),
    ("lbib_set_fields", C.c_int, [_vp, _dp, _dp, _dp, _dp, _dp, _dp]),
    ("lbib_step", C.c_int, [_vp, C.c_int]),
    ("lbib_get_fields", C.c_int, [_vp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
    ("lbib_get_membrane", C.c_int, [_vp, C.c_int, _dp, _dp, _dp]),
    ("lbib_energy", C.c_int, [_vp, C.POINTER(Energies)]),
    ("lbib_check", C.c_int, [_vp]),
    ("lbib_device_view", C.c_int, [_vp, C.c_int, C.POINTER(_vp), C.POINTER(C.c_size_t)]),
    ("lbib_save", C.c_int, [_vp, _vp, C.POINTER(C.c_size_t)]),
    ("lbib_load", C.c_int, [_vp, _vp, C.c_size_t]),
    ("lbib_timing_enable", C.c_int, [_vp, C.c_int]),
    ("lbib_timing_read", C.c_int, [_vp, _dp, C.c_int, _ip]),
    ("lbib_set_launch", C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int]),
    ("lbib_set_overlap", C.c_int, [_vp, C.c_int]),
    ("lbib_set_force_form", C.c_int, [_vp, C.c_int]),
    ("lbib_set_external_force", C.c_int, [_vp, C.c_double, C.c_double, C.c_double]),
    ("lbib_set_coupling_cache", C.c_int, [_vp, C.c_int]),
    ("lbib_set_densities", C.c_int, [_vp, C.c_double, C.c_double, C.c_double]),
    ("lbib_get_launch", C.c_int, [_vp, _ip, _ip, _ip, _ip]),
    ("lbib_steps_done", C.c_longlong, [_vp]),
    ("lbib_debug_poke", C.c_int, [_vp, C.c_int, C.c_longlong, C.c_double]),
    ("lbib_strerror", C.c_char_p, [C.c_int]),
    ("lbib_destroy", None, [_vp]),
    ("lbib_set_rest", C.c_int, [_vp, C.c_int, _dp]),
    ("lbib_set_membrane_law", C.c_int, [_vp, C.c_int, C.c_int]),
    ("lbib_batch_workspace_bytes", C.c_int, [C.c_int, _vp, C.POINTER(C.c_size_t)]),
    ("lbib_batch_create", C.c_int, [C.c_int, _vp, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    ("lbib_batch_member", C.c_int, [_vp, C.c_int, C.POINTER(_vp)]),
    ("lbib_batch_set_launch", C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int]),
    ("lbib_batch_get_launch", C.c_int, [_vp, C.c_int, _ip, _ip, _ip, _ip]),
    ("lbib_batch_graph", C.c_int, [_vp, C.c_int, _ip]),
    ("lbib_mlp_param_count", C.c_int, []),
    ("lbib_mlp_workspace_bytes", C.c_int, [C.c_int, C.POINTER(C.c_size_t)]),
    ("lbib_mlp_create", C.c_int, [C.c_int, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    ("lbib_mlp_set_params", C.c_int, [_vp, _fp]),
    ("lbib_mlp_get_params", C.c_int, [_vp, _fp]),
    ("lbib_mlp_forward", C.c_int, [_vp, _vp, C.c_int, _vp]),
    ("lbib_mlp_gradient", C.c_int, [_vp, _vp, _vp, C.c_int, C.POINTER(C.c_double), _fp]),
    ("lbib_mlp_adam_step", C.c_int, [_vp, _vp, _vp, C.c_int, C.c_float, C.c_float, C.c_float, C.c_float,
                                     C.POINTER(C.c_double)]),
    ("lbib_mlp_destroy", None, [_vp]),
    ("lbib_mlp_forward_noalloc", C.c_int, [_vp, _vp, C.c_int, _vp, _vp]),
]


def lib():
    """Load liblbib.so (built by paper_1906_03065_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import "
                               "__graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _chk(fn, code):
    if code != 0:
        raise LbibError(fn, code)


def _d(a):
    return None if a is None else a.ctypes.data_as(_dp)


def make_params(p: dict, storage="fp32", max_markers=None, max_membranes=None, max_elems=None,
                membranes=()) -> Params:
    if isinstance(storage, str):
        storage = STORAGE[storage]
    if max_markers is None:
        max_markers = sum(len(m["X"]) for m in membranes)
    if max_elems is None:
        max_elems = sum(len(m["tris"]) for m in membranes if m.get("tris") is not None)
    if max_membranes is None:
        max_membranes = len(membranes)
    k = p["kappa"]
    return Params(int(p.get("lattice", 0)), int(p["nx"]), int(p["ny"]), int(p.get("nz", 1)),
                  int(p.get("wall_y", 0)), int(p.get("wall_z", 0)),
                  float(p.get("tau", 1.0)), float(p.get("tau_phi", 1.0)), float(p.get("tau_psi", 1.0)),
                  float(p.get("gamma_phi", 1.0)), float(p.get("gamma_psi", 1.0)),
                  (C.c_double * 3)(float(k[0]), float(k[1]), float(k[2])),
                  float(p.get("alpha", 1.0)), float(p.get("kappa_c", 0.0)), float(p.get("r_cut", 0.0)),
                  int(storage), int(max_markers), int(max_elems), int(max_membranes))


def workspace_bytes(prm: Params) -> int:
    n = C.c_size_t(0)
    _chk("lbib_workspace_bytes", lib().lbib_workspace_bytes(C.byref(prm), C.byref(n)))
    return n.value


class Sim:
    """One GPU simulation.  ``p`` is the project's parameter dict (see
    workloads.base_params); ``membranes`` sizes the marker capacity."""

    def __init__(self, p: dict, storage="fp32", membranes=(), device="cuda:0", stream=None,
                 max_markers=None, max_membranes=None, max_elems=None):
        import torch

        self.torch = torch
        self.p = dict(p)
        self.prm = make_params(p, storage, max_markers, max_membranes, max_elems, membranes=membranes)
        self.D = 3 if self.prm.lattice == D3Q19 else 2
        self.shape = ((self.prm.nz, self.prm.ny, self.prm.nx) if self.D == 3
                      else (self.prm.ny, self.prm.nx))
        self.N = int(np.prod(self.shape))
        self.device = torch.device(device)
        nbytes = workspace_bytes(self.prm)
        # torch's caching allocator returns blocks aligned to at least 512 bytes
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = _vp()
        _chk("lbib_create", lib().lbib_create(C.byref(self.prm), _vp(self.ws.data_ptr()), nbytes,
                                              _vp(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.mem_sizes = []
        if self.D == 2:
            # the library's D2Q9 default is the divergence form (1)
            self.set_force_form(int(p.get("force_form", 1)))
        if any(p.get("fext", ())):
            self.set_external_force(*p["fext"])
        if tuple(p.get("mw", (1.0, 1.0, 1.0))) != (1.0, 1.0, 1.0):
            self.set_densities(*p["mw"])

    @classmethod
    def _member(cls, batch, h, p: dict):
        """Wrap member handle h of a Batch (owned by the batch)."""
        self = cls.__new__(cls)
        self.torch = batch.torch
        self.p = dict(p)
        self.prm = None
        self.D = 2
        self.shape = (int(p["ny"]), int(p["nx"]))
        self.N = int(np.prod(self.shape))
        self.device = batch.device
        self.ws = None
        self.stream = batch.stream
        self.h = h
        self.mem_sizes = []
        self.owner = batch
        return self

    def close(self):
        if getattr(self, "owner", None) is not None:
            self.h = None  # freed with its batch
            return
        if getattr(self, "h", None):
            lib().lbib_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_membrane(self, X, tris=None, kappa_s=0.0, kappa_b=0.0, rest=None) -> int:
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, self.D)
        mid = C.c_int(-1)
        if tris is None:
            rc = lib().lbib_add_membrane(self.h, X.shape[0], _d(X), 0, None, kappa_s, kappa_b,
                                         C.byref(mid))
        else:
            t = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
            rc = lib().lbib_add_membrane(self.h, X.shape[0], _d(X), t.shape[0],
                                         t.ctypes.data_as(_ip), kappa_s, kappa_b, C.byref(mid))
        _chk("lbib_add_membrane", rc)
        self.mem_sizes.append(X.shape[0])
        if rest is not None:
            self.set_rest(mid.value, rest)
        return mid.value

    def set_membrane_law(self, i: int, law: int):
        """Strain law of ring i: 0 eq. DiscreteSE, 1 neo-Hookean, 2 Skalak."""
        _chk("lbib_set_membrane_law", lib().lbib_set_membrane_law(self.h, int(i), int(law)))

    def set_rest(self, i: int, rest):
        r = np.ascontiguousarray(rest, dtype=np.float64).reshape(-1)
        _chk("lbib_set_rest", lib().lbib_set_rest(self.h, int(i), _d(r)))

    def set_fields(self, rho, phi, psi, u=None):
        arr = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in (rho, phi, psi)]
        uu = [None, None, None]
        if u is not None:
            for a in range(self.D):
                uu[a] = np.ascontiguousarray(u[a], dtype=np.float64).reshape(-1)
        _chk("lbib_set_fields", lib().lbib_set_fields(self.h, *(_d(a) for a in arr),
                                                      *(_d(a) for a in uu)))

    def step(self, n=1):
        _chk("lbib_step", lib().lbib_step(self.h, int(n)))

    @property
    def steps_done(self) -> int:
        return lib().lbib_steps_done(self.h)

    def fields(self) -> dict:
        keys = ("rho", "c1", "c2", "c3", "ux", "uy", "uz")
        out = {k: np.empty(self.N) for k in keys}
        if self.D == 2:
            out["uz"] = None
        _chk("lbib_get_fields", lib().lbib_get_fields(self.h, *(_d(out[k]) for k in keys)))
        return {k: v.reshape(self.shape) for k, v in out.items() if v is not None}

    def membrane(self, i: int) -> dict:
        n = self.mem_sizes[i]
        X, U, F = (np.empty((n, self.D)) for _ in range(3))
        _chk("lbib_get_membrane", lib().lbib_get_membrane(self.h, i, _d(X), _d(U), _d(F)))
        return {"X": X, "U": U, "F": F}

    def energy(self) -> dict:
        e = Energies()
        _chk("lbib_energy", lib().lbib_energy(self.h, C.byref(e)))
        d = {k: getattr(e, k) for k, _ in Energies._fields_ if k != "mass"}
        d["mass"] = list(e.mass)
        return d

    def check(self) -> int:
        return lib().lbib_check(self.h)

    def save(self) -> bytes:
        n = C.c_size_t(0)
        _chk("lbib_save", lib().lbib_save(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _chk("lbib_save", lib().lbib_save(self.h, buf, C.byref(n)))
        return buf.raw[: n.value]

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _chk("lbib_load", lib().lbib_load(self.h, buf, len(blob)))

    def poke(self, field: int, idx: int, value: float):
        _chk("lbib_debug_poke", lib().lbib_debug_poke(self.h, field, int(idx), float(value)))

    def set_launch(self, block_x=0, seg=0, nxcd=0, ring=0):
        _chk("lbib_set_launch", lib().lbib_set_launch(self.h, int(block_x), int(seg), int(nxcd),
                                                      int(ring)))

    def set_overlap(self, on: int = -1):
        """D2Q9: 1 runs the lattice regions away from the membranes on a second
        stream beside the membrane kernels, 0 (the default) keeps one stream,
        -1 lets the library choose (currently 0)."""
        _chk("lbib_set_overlap", lib().lbib_set_overlap(self.h, int(on)))

    def set_force_form(self, form: int):
        """D2Q9: 1 (the default) the divergence form of the thermodynamic
        force (minus the divergence of the non-ideal pressure tensor, plus the
        coupling term), 0 its potential form."""
        _chk("lbib_set_force_form", lib().lbib_set_force_form(self.h, int(form)))

    def set_coupling_cache(self, on: int):
        """D2Q9: 1 (the default) keeps each node's closest membrane segment
        between steps (re-evaluated, not searched, while provably still the
        closest), 0 searches every step; the results are bitwise the same."""
        _chk("lbib_set_coupling_cache", lib().lbib_set_coupling_cache(self.h, int(on)))

    def set_external_force(self, fx=0.0, fy=0.0, fz=0.0):
        """Uniform external force density f_ext of eq. ForcingTermLBE."""
        _chk("lbib_set_external_force", lib().lbib_set_external_force(self.h, float(fx), float(fy), float(fz)))

    def set_densities(self, m1=1.0, m2=1.0, m3=1.0):
        """D2Q9: component densities of eq. MassDensity (all 1 in the paper);
        before set_fields."""
        _chk("lbib_set_densities", lib().lbib_set_densities(self.h, float(m1), float(m2), float(m3)))

    def get_launch(self):
        a, b, c, d = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        _chk("lbib_get_launch", lib().lbib_get_launch(self.h, C.byref(a), C.byref(b), C.byref(c),
                                                      C.byref(d)))
        return {"block_x": a.value, "seg": b.value, "nxcd": c.value, "ring": d.value}

    def timing(self, mask: int = 15):
        """Time the phases in ``mask`` (bit 0 lattice kernel, 1 coupling,
        2 membrane forces + spreading, 3 interpolation); 0 switches off."""
        _chk("lbib_timing_enable", lib().lbib_timing_enable(self.h, int(mask)))

    def timing_read(self):
        """Summed milliseconds per phase: lattice kernel, coupling, membrane
        forces + spreading, interpolation; and the number of steps timed."""
        ms = np.zeros(4)
        n = C.c_int(0)
        _chk("lbib_timing_read", lib().lbib_timing_read(self.h, _d(ms), 4, C.byref(n)))
        return {"lb": ms[0], "coupling": ms[1], "membrane": ms[2], "interp": ms[3],
                "steps": n.value}

    def device_view(self, field: int):
        ptr, n = _vp(), C.c_size_t(0)
        _chk("lbib_device_view", lib().lbib_device_view(self.h, field, C.byref(ptr), C.byref(n)))
        return ptr.value, n.value


class Batch:
    """n independent D2Q9 simulations (FP32) stepped together: one launch
    per phase over all members, the step replayed from a hipGraph.  The
    batch runs on its own (capturable) stream unless one is given."""

    def __init__(self, params: list, membranes: list = None, device="cuda:0", stream=None):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        n = len(params)
        forms = {int(p.get("force_form", 1)) for p in params}
        if len(forms) > 1:
            raise LbibError("lbib_batch_create", EINVAL)  # one force form per batch
        membranes = membranes or [()] * n
        arr = (Params * n)(*[make_params(p, "fp32", membranes=m) for p, m in zip(params, membranes)])
        self._prms = arr
        nb = C.c_size_t(0)
        _chk("lbib_batch_workspace_bytes", lib().lbib_batch_workspace_bytes(n, C.byref(arr), C.byref(nb)))
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        h = _vp()
        _chk("lbib_batch_create", lib().lbib_batch_create(n, C.byref(arr), _vp(self.ws.data_ptr()), nb.value,
                                                          _vp(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.members = []
        for k in range(n):
            mh = _vp()
            _chk("lbib_batch_member", lib().lbib_batch_member(self.h, k, C.byref(mh)))
            self.members.append(Sim._member(self, mh, params[k]))
            if any(params[k].get("fext", ())):
                self.members[-1].set_external_force(*params[k]["fext"])
            if tuple(params[k].get("mw", (1.0, 1.0, 1.0))) != (1.0, 1.0, 1.0):
                self.members[-1].set_densities(*params[k]["mw"])
        self.set_force_form(forms.pop())

    def set_force_form(self, form: int):
        """Force form of every member (see Sim.set_force_form); the next step
        captures the batch's graphs again."""
        _chk("lbib_set_force_form", lib().lbib_set_force_form(self.h, int(form)))

    def set_coupling_cache(self, on: int):
        """Coupling-search cache of every member (see Sim.set_coupling_cache)."""
        _chk("lbib_set_coupling_cache", lib().lbib_set_coupling_cache(self.h, int(on)))

    def __len__(self):
        return len(self.members)

    def __getitem__(self, k) -> Sim:
        return self.members[k]

    def step(self, n=1):
        _chk("lbib_step", lib().lbib_step(self.h, int(n)))

    def check(self) -> int:
        return lib().lbib_check(self.h)

    def set_launch(self, size_class=-1, block_x=0, seg=0, ring=0):
        _chk("lbib_batch_set_launch", lib().lbib_batch_set_launch(self.h, int(size_class), int(block_x),
                                                                  int(seg), int(ring)))

    def get_launch(self, size_class: int) -> dict:
        a, b, c, d = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        _chk("lbib_batch_get_launch", lib().lbib_batch_get_launch(self.h, int(size_class), C.byref(a),
                                                                  C.byref(b), C.byref(c), C.byref(d)))
        return {"block_x": a.value, "seg": b.value, "ring": c.value, "members": d.value}

    def graph(self, on: int = -1) -> int:
        """Switch graph replay on (1) or off (0); returns whether the last
        step replayed a graph."""
        a = C.c_int(0)
        _chk("lbib_batch_graph", lib().lbib_batch_graph(self.h, int(on), C.byref(a)))
        return a.value

    def synchronize(self):
        self.stream.synchronize()

    def markers(self) -> list:
        """Marker positions of every member's membranes, [(n, 2)] per member
        and membrane, gathered on the device and copied in one transfer."""
        t = self.torch
        if not hasattr(self, "_views"):
            base = self.ws.data_ptr()
            self._views = []
            for m in self.members:
                ptr, n = m.device_view(2)
                off = ptr - base
                self._views.append(self.ws[off:off + 8 * n].view(t.float64).view(-1, 3))
        with t.cuda.stream(self.stream):
            allx = t.cat(self._views).cpu().numpy()
        out, o = [], 0
        for m in self.members:
            mk = []
            for n in m.mem_sizes:
                mk.append(allx[o:o + n, :2].copy())
                o += n
            out.append(mk)
        return out

    def close(self):
        if getattr(self, "h", None):
            for m in self.members:
                m.h = None
            lib().lbib_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @classmethod
    def from_workloads(cls, ws: list, device="cuda:0", stream=None) -> "Batch":
        b = cls([w["params"] for w in ws], [w["membranes"] for w in ws], device=device, stream=stream)
        for m, w in zip(b.members, ws):
            for mem in w["membranes"]:
                i = m.add_membrane(mem["X"], mem.get("tris"), mem["kappa_s"], mem["kappa_b"], mem.get("rest"))
                if mem.get("law", 0):
                    m.set_membrane_law(i, mem["law"])
            f = w["fields"]
            m.set_fields(f["rho"], f["phi"], f["psi"], f.get("u"))
        return b


class Mlp:
    """The warm-start network's device state (parameters, Adam moments,
    activations for up to batch_max rows) in a torch-owned workspace."""

    def __init__(self, batch_max: int, device="cuda:0", stream=None):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.batch_max = int(batch_max)
        nb = C.c_size_t(0)
        _chk("lbib_mlp_workspace_bytes", lib().lbib_mlp_workspace_bytes(self.batch_max, C.byref(nb)))
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = _vp()
        _chk("lbib_mlp_create", lib().lbib_mlp_create(self.batch_max, _vp(self.ws.data_ptr()), nb.value,
                                                      _vp(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.nparam = lib().lbib_mlp_param_count()

    def set_params(self, p):
        a = np.ascontiguousarray(p, dtype=np.float32).reshape(-1)
        assert a.size == self.nparam
        _chk("lbib_mlp_set_params", lib().lbib_mlp_set_params(self.h, a.ctypes.data_as(_fp)))

    def params(self) -> np.ndarray:
        a = np.empty(self.nparam, dtype=np.float32)
        _chk("lbib_mlp_get_params", lib().lbib_mlp_get_params(self.h, a.ctypes.data_as(_fp)))
        return a

    def _dev(self, a, cols):
        t = self.torch
        x = t.as_tensor(np.ascontiguousarray(a, dtype=np.float32)) if not t.is_tensor(a) else a
        x = x.to(self.device, dtype=t.float32).contiguous()
        assert x.dim() == 2 and x.shape[1] == cols and 1 <= x.shape[0] <= self.batch_max
        return x

    def forward(self, x):
        """y [B][32] (torch tensor on the device) for inputs x [B][6]."""
        x = self._dev(x, 6)
        y = self.torch.empty((x.shape[0], 32), dtype=self.torch.float32, device=self.device)
        _chk("lbib_mlp_forward", lib().lbib_mlp_forward(self.h, _vp(x.data_ptr()), x.shape[0], _vp(y.data_ptr())))
        return y

    def gradient(self, x, t):
        """(loss, gradient) of the batch (host FP64 loss, FP32 gradient)."""
        x, t = self._dev(x, 6), self._dev(t, 32)
        loss = C.c_double(0)
        g = np.empty(self.nparam, dtype=np.float32)
        _chk("lbib_mlp_gradient", lib().lbib_mlp_gradient(self.h, _vp(x.data_ptr()), _vp(t.data_ptr()),
                                                          x.shape[0], C.byref(loss), g.ctypes.data_as(_fp)))
        return loss.value, g

    def adam_step(self, x, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, want_loss=False):
        x, t = self._dev(x, 6), self._dev(t, 32)
        loss = C.c_double(0)
        _chk("lbib_mlp_adam_step", lib().lbib_mlp_adam_step(self.h, _vp(x.data_ptr()), _vp(t.data_ptr()),
                                                            x.shape[0], lr, beta1, beta2, eps,
                                                            C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def close(self):
        if getattr(self, "h", None):
            lib().lbib_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_forward_noalloc(params_dev, x_dev, y_dev, stream=None):
    """lbib_mlp_forward_noalloc on torch tensors already on the device:
    params_dev (float32, lbib_mlp_param_count()), x_dev [B][6], y_dev [B][32]
    (contiguous float32).  Allocates nothing; returns nothing."""
    import torch

    st = stream if stream is not None else torch.cuda.current_stream(x_dev.device)
    _chk("lbib_mlp_forward_noalloc", lib().lbib_mlp_forward_noalloc(
        _vp(params_dev.data_ptr()), _vp(x_dev.data_ptr()), int(x_dev.shape[0]), _vp(y_dev.data_ptr()),
        _vp(st.cuda_stream)))


def from_workload(w: dict, storage="fp32", device="cuda:0", **kw) -> Sim:
    """Create a GPU simulation from a workloads.* dictionary."""
    s = Sim(w["params"], storage=storage, membranes=w["membranes"], device=device, **kw)
    for m in w["membranes"]:
        i = s.add_membrane(m["X"], m.get("tris"), m["kappa_s"], m["kappa_b"], m.get("rest"))
        if m.get("law", 0):
            s.set_membrane_law(i, m["law"])
    f = w["fields"]
    s.set_fields(f["rho"], f["phi"], f["psi"], f.get("u"))
    return s
