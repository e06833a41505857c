"""Thin Python binding of libmdg (include/mdg.h): argument marshalling only.

Every computation runs in the native library (host setup in C++, the stage
operator in HIP kernels on gfx950). PyTorch is used only to own the device
workspace and to supply the HIP stream. If ``libmdg.so`` has not been built,
loading fails loudly; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdg.so")

MDG_OK, MDG_E_ARG, MDG_E_MESH, MDG_E_HIP, MDG_E_OOM, MDG_E_STATE, MDG_E_UNSTABLE, MDG_E_UNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7)
MDG_FP64, MDG_FP32 = 0, 1
MDG_CENTRAL, MDG_UPWIND = 0, 1
MDG_RK4 = 0
MDG_LEAPFROG = 1

_STATUS = {0: "MDG_OK", -1: "MDG_E_ARG", -2: "MDG_E_MESH", -3: "MDG_E_HIP", -4: "MDG_E_OOM",
           -5: "MDG_E_STATE", -6: "MDG_E_UNSTABLE", -7: "MDG_E_UNSUPPORTED"}


class MdgError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


_LAUNCH = {"auto": 0, "persistent": 1, "per_tile": 2}


class mdg_options(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("precision", ctypes.c_int32), ("flux", ctypes.c_int32),
                ("integrator", ctypes.c_int32), ("dt", ctypes.c_double), ("cfl", ctypes.c_double),
                ("tile", ctypes.c_int32), ("mixed", ctypes.c_int32), ("sip_alpha", ctypes.c_double),
                ("monitor", ctypes.c_int32), ("mfma", ctypes.c_int32), ("launch", ctypes.c_int32)]


class mdg_info(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("nmodes", ctypes.c_int32), ("nfacemodes", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flux", ctypes.c_int32), ("tile_size", ctypes.c_int32),
                ("n_elements", ctypes.c_int64), ("n_faces_interior", ctypes.c_int64),
                ("n_faces_boundary", ctypes.c_int64), ("n_pml", ctypes.c_int64),
                ("n_tiles", ctypes.c_int64), ("n_halo", ctypes.c_int64),
                ("dt", ctypes.c_double), ("time", ctypes.c_double),
                ("bytes_per_stage", ctypes.c_double), ("flops_per_stage", ctypes.c_double),
                ("workspace_bytes", ctypes.c_int64), ("n_instances", ctypes.c_int64),
                ("n_dipoles", ctypes.c_int64), ("order_h", ctypes.c_int32), ("nmodes_h", ctypes.c_int32)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_VP = ctypes.c_void_p
_S = ctypes.c_int32

SIGNATURES = {
    "mdg_create": (_S, [ctypes.POINTER(mdg_options), ctypes.POINTER(_VP)]),
    "mdg_destroy": (None, [_VP]),
    "mdg_last_error": (ctypes.c_char_p, [_VP]),
    "mdg_set_mesh": (_S, [_VP, ctypes.c_int64, _D, ctypes.c_int64, _I64]),
    "mdg_set_material": (_S, [_VP, _D, _D]),
    "mdg_set_pml": (_S, [_VP, _D]),
    "mdg_set_dipoles": (_S, [_VP, ctypes.c_int32, _D, _D, _D]),
    "mdg_set_instances": (_S, [_VP, ctypes.c_int32, _I64]),
    "mdg_set_instance_dipoles": (_S, [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _D, _D, _D]),
    "mdg_workspace_size": (_S, [_VP, ctypes.POINTER(ctypes.c_size_t)]),
    "mdg_bind_workspace": (_S, [_VP, _VP, ctypes.c_size_t, _VP]),
    "mdg_set_state": (_S, [_VP, _D, _D, _D, _D, ctypes.c_double]),
    "mdg_get_state": (_S, [_VP, _D, _D, _D, _D, _D]),
    "mdg_set_sip_state": (_S, [_VP, _D]),
    "mdg_get_sip_state": (_S, [_VP, _D]),
    "mdg_projection_points": (_S, [_VP, ctypes.c_int32, _I64, _D]),
    "mdg_project": (_S, [_VP, ctypes.c_int32, _D, _D, ctypes.c_double]),
    "mdg_step": (_S, [_VP, ctypes.c_int64, _VP]),
    "mdg_step_graph": (_S, [_VP, ctypes.c_int64, ctypes.c_int32, _VP]),
    "mdg_rhs": (_S, [_VP, _D, _D, _D, _D, ctypes.c_double, _D, _D, _D, _D]),
    "mdg_rhs_sip": (_S, [_VP, _D, _D, _D, _D, _D, ctypes.c_double, _D, _D, _D, _D, _D]),
    "mdg_energy": (_S, [_VP, _D]),
    "mdg_energy_instances": (_S, [_VP, _D]),
    "mdg_adjoint_probe_energy": (_S, [_VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _I64, _D, _D, _VP]),
    "mdg_probe_energy": (_S, [_VP, ctypes.c_int64, ctypes.c_int32, _I64, _D, _VP]),
    "mdg_probe_energy_noalloc": (_S, [_VP, ctypes.c_int64, ctypes.c_int32, _I64, _D, _VP]),
    "mdg_query": (_S, [_VP, ctypes.POINTER(mdg_info)]),
}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmdg.so (built in-tree by ``paper_2002_08733_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libmdg.so not found at {path}: build it with "
                          "`python -m paper_2002_08733_amd.build` (no fallback exists)")
    # PyTorch ships its own HIP runtime with the same soname as the system one.
    # Load and initialise it first so that libmdg binds to the runtime that owns
    # the device memory and streams it is handed (one runtime per process).
    try:
        import torch
        torch.cuda.is_available()
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _dptr(a):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        a = a.reshape(shape)
    return a


class Solver:
    """One libmdg handle. Methods mirror the C entry points one to one."""

    def __init__(self, order, precision="fp64", flux="central", dt=0.0, cfl=0.3, tile=0, integrator="rk4",
                 mixed=False, sip_alpha=0.0, monitor=0, mfma=False, launch="auto"):
        """order: polynomial order of h (and of e, unless mixed: then e is one
        order higher, the paper's pairing). sip_alpha > 0 adds the SIP
        surface unknown (central flux). monitor >= 2: step() checks the
        energy every `monitor` steps (see mdg_options.monitor). mfma: the
        volume term as BF16x3 MFMA products (FP32, RK4, order <= 3). launch:
        "auto", "persistent" or "per_tile" (see mdg_options.launch)."""
        self.lib = load_library()
        if integrator not in ("rk4", "leapfrog"):
            raise ValueError("integrator must be 'rk4' or 'leapfrog'")
        o = mdg_options(order=order, precision=MDG_FP32 if precision == "fp32" else MDG_FP64,
                        flux=MDG_UPWIND if flux == "upwind" else MDG_CENTRAL,
                        integrator=MDG_RK4 if integrator == "rk4" else MDG_LEAPFROG, dt=float(dt), cfl=float(cfl),
                        tile=int(tile), mixed=1 if mixed else 0, sip_alpha=float(sip_alpha), monitor=int(monitor),
                        mfma=1 if mfma else 0, launch=_LAUNCH[launch])
        h = _VP()
        st = self.lib.mdg_create(ctypes.byref(o), ctypes.byref(h))
        if st != MDG_OK:
            raise MdgError(st, self.lib.mdg_last_error(None).decode())
        self.h = h
        self.order = order
        pe = order + (1 if mixed else 0)
        self.nmodes = (pe + 1) * (pe + 2) * (pe + 3) // 6  # of e (and p)
        self.nmodes_h = (order + 1) * (order + 2) * (order + 3) // 6  # of h (and q)
        self.nfacemodes = (order + 1) * (order + 2) // 2  # of the SIP unknown (order of h)
        self.nt = 0
        self._ws = None

    # -------------------------------------------------------------- helpers
    def _chk(self, st):
        if st != MDG_OK:
            raise MdgError(st, self.lib.mdg_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.mdg_destroy(self.h)
            self.h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _shape(self):
        return (self.nt, 3, self.nmodes)

    def _shape_h(self):
        return (self.nt, 3, self.nmodes_h)

    # ----------------------------------------------------------------- setup
    def set_mesh(self, verts, tets):
        v = _f64(verts)
        t = np.ascontiguousarray(tets, dtype=np.int64)
        self._chk(self.lib.mdg_set_mesh(self.h, v.shape[0], _dptr(v), t.shape[0], t.ctypes.data_as(_I64)))
        self.nt = t.shape[0]

    def set_material(self, eps=None, mu=None):
        e, m = _f64(eps), _f64(mu)
        self._chk(self.lib.mdg_set_material(self.h, _dptr(e), _dptr(m)))

    def set_pml(self, omega=None):
        w = _f64(omega)
        self._chk(self.lib.mdg_set_pml(self.h, _dptr(w)))

    def set_dipoles(self, pos, direction, wave, instance=None):
        p, d, w = _f64(pos), _f64(direction), _f64(wave)
        n = 0 if p is None else p.reshape(-1, 3).shape[0]
        if instance is None:
            self._chk(self.lib.mdg_set_dipoles(self.h, n, _dptr(p), _dptr(d), _dptr(w)))
        else:
            ins = np.ascontiguousarray(instance, dtype=np.int32)
            self._chk(self.lib.mdg_set_instance_dipoles(
                self.h, n, ins.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dptr(p), _dptr(d), _dptr(w)))

    def set_instances(self, first):
        """Element ranges [first[i], first[i+1]) of independent instances."""
        f = np.ascontiguousarray(first, dtype=np.int64)
        self._chk(self.lib.mdg_set_instances(self.h, len(f) - 1, f.ctypes.data_as(_I64)))

    def workspace_size(self):
        n = ctypes.c_size_t()
        self._chk(self.lib.mdg_workspace_size(self.h, ctypes.byref(n)))
        return n.value

    def bind_workspace(self, tensor=None, stream=None):
        """Bind device memory: a CUDA/HIP torch tensor (kept alive here) or None
        to let the library allocate it."""
        ptr, nbytes = None, 0
        if tensor is not None:
            ptr = tensor.data_ptr()
            nbytes = tensor.numel() * tensor.element_size()
        self._chk(self.lib.mdg_bind_workspace(self.h, ptr, nbytes, stream))
        self._ws = tensor

    def bind_torch_workspace(self, device="cuda"):
        import torch
        n = self.workspace_size()
        ws = torch.empty(n, dtype=torch.uint8, device=device)
        self.bind_workspace(ws, torch.cuda.current_stream(ws.device).cuda_stream)
        return ws

    # ----------------------------------------------------------------- state
    def set_state(self, E, H, P=None, Q=None, t=0.0):
        s, sh = self._shape(), self._shape_h()
        E, H, P, Q = _f64(E, s), _f64(H, sh), _f64(P, s), _f64(Q, sh)
        self._chk(self.lib.mdg_set_state(self.h, _dptr(E), _dptr(H), _dptr(P), _dptr(Q), float(t)))

    def get_state(self, aux=False):
        s, sh = self._shape(), self._shape_h()
        E, H = np.empty(s), np.empty(sh)
        P = np.empty(s) if aux else None
        Q = np.empty(sh) if aux else None
        t = ctypes.c_double()
        self._chk(self.lib.mdg_get_state(self.h, _dptr(E), _dptr(H), _dptr(P), _dptr(Q), ctypes.byref(t)))
        return (E, H, P, Q, t.value) if aux else (E, H, t.value)

    def set_sip_state(self, S):
        """SIP unknown S[nt][4][2][NF] (see mdg_set_sip_state)."""
        S = _f64(S, (self.nt, 4, 2, self.nfacemodes))
        self._chk(self.lib.mdg_set_sip_state(self.h, _dptr(S)))

    def get_sip_state(self):
        S = np.empty((self.nt, 4, 2, self.nfacemodes))
        self._chk(self.lib.mdg_get_sip_state(self.h, _dptr(S)))
        return S

    def projection_points(self, q):
        n = ctypes.c_int64()
        self._chk(self.lib.mdg_projection_points(self.h, q, ctypes.byref(n), None))
        x = np.empty((self.nt, n.value, 3))
        self._chk(self.lib.mdg_projection_points(self.h, q, ctypes.byref(n), _dptr(x)))
        return x

    def project(self, q, Evals=None, Hvals=None, t=0.0):
        E, H = _f64(Evals), _f64(Hvals)
        self._chk(self.lib.mdg_project(self.h, q, _dptr(E), _dptr(H), float(t)))

    # ------------------------------------------------------------------- run
    def step(self, nsteps=1, stream=None):
        self._chk(self.lib.mdg_step(self.h, int(nsteps), stream))

    def step_graph(self, nsteps, steps_per_graph, stream):
        self._chk(self.lib.mdg_step_graph(self.h, int(nsteps), int(steps_per_graph), stream))

    def rhs(self, E, H, P=None, Q=None, t=0.0, aux=False):
        s, sh = self._shape(), self._shape_h()
        E, H, P, Q = _f64(E, s), _f64(H, sh), _f64(P, s), _f64(Q, sh)
        dE, dH = np.empty(s), np.empty(sh)
        dP = np.empty(s) if aux else None
        dQ = np.empty(sh) if aux else None
        self._chk(self.lib.mdg_rhs(self.h, _dptr(E), _dptr(H), _dptr(P), _dptr(Q), float(t),
                                   _dptr(dE), _dptr(dH), _dptr(dP), _dptr(dQ)))
        return (dE, dH, dP, dQ) if aux else (dE, dH)

    def rhs_sip(self, E, H, S=None, P=None, Q=None, t=0.0, aux=False):
        """Operator with the SIP unknown: (dE, dH, dS) or, with aux, (dE, dH, dS, dP, dQ)."""
        s, sh, ss = self._shape(), self._shape_h(), (self.nt, 4, 2, self.nfacemodes)
        E, H, S, P, Q = _f64(E, s), _f64(H, sh), _f64(S, ss), _f64(P, s), _f64(Q, sh)
        dE, dH, dS = np.empty(s), np.empty(sh), np.empty(ss)
        dP = np.empty(s) if aux else None
        dQ = np.empty(sh) if aux else None
        self._chk(self.lib.mdg_rhs_sip(self.h, _dptr(E), _dptr(H), _dptr(S), _dptr(P), _dptr(Q), float(t),
                                       _dptr(dE), _dptr(dH), _dptr(dS), _dptr(dP), _dptr(dQ)))
        return (dE, dH, dS, dP, dQ) if aux else (dE, dH, dS)

    def energy(self):
        w = ctypes.c_double()
        self._chk(self.lib.mdg_energy(self.h, ctypes.byref(w)))
        return w.value

    def probe_energy(self, nsteps, probes, stream=None):
        """J = sum_n dt sum_probes ||e^n||^2 over nsteps steps from the current state."""
        pr = np.ascontiguousarray(probes, dtype=np.int64)
        J = ctypes.c_double()
        self._chk(self.lib.mdg_probe_energy(self.h, int(nsteps), len(pr), pr.ctypes.data_as(_I64),
                                            ctypes.byref(J), stream))
        return J.value

    def probe_energy_noalloc(self, nsteps, probes, stream=None):
        """probe_energy through the entry point that allocates no device memory."""
        pr = np.ascontiguousarray(probes, dtype=np.int64)
        J = ctypes.c_double()
        self._chk(self.lib.mdg_probe_energy_noalloc(self.h, int(nsteps), len(pr), pr.ctypes.data_as(_I64),
                                                    ctypes.byref(J), stream))
        return J.value

    def adjoint_probe_energy(self, nsteps, every, probes, stream=None):
        """(J, dJ/deps[nt]): probe energy over nsteps steps from the current
        state and its gradient by the checkpointed discrete adjoint."""
        pr = np.ascontiguousarray(probes, dtype=np.int64)
        J = ctypes.c_double()
        g = np.empty(self.nt)
        self._chk(self.lib.mdg_adjoint_probe_energy(self.h, int(nsteps), int(every), len(pr),
                                                    pr.ctypes.data_as(_I64), ctypes.byref(J), _dptr(g), stream))
        return J.value, g

    def energy_instances(self):
        n = self.query()["n_instances"]
        w = np.empty(n)
        self._chk(self.lib.mdg_energy_instances(self.h, _dptr(w)))
        return w

    def query(self):
        i = mdg_info()
        self._chk(self.lib.mdg_query(self.h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in mdg_info._fields_}
