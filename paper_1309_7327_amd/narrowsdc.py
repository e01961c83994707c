"""Thin ctypes binding of libnarrowsdc.so (argument marshalling only).

Every computation runs in the HIP kernels of the library; torch tensors only
provide device memory and the current HIP stream.  Importing this module on a
machine without the built library raises immediately: there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnarrowsdc.so")

SDC_OK, SDC_EINVAL, SDC_ENOMECH, SDC_EHIP, SDC_ETEMP, SDC_ENOMEM = 0, -1, -2, -3, -4, -5
RHS_HYP, RHS_DIFF, RHS_REACT, RHS_AD, RHS_ALL = 1, 2, 4, 3, 7
NG = 4

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run paper_1309_7327_amd/build.py "
                      "(or __graft_entry__.build()); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)


class BoxDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("ng", ctypes.c_int),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("nonperiodic", ctypes.c_int)]


class MechanismDesc(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int), ("nr", ctypes.c_int),
                ("W", ctypes.c_void_p), ("nasa", ctypes.c_void_p),
                ("Tlo", ctypes.c_double), ("Thi", ctypes.c_double),
                ("A", ctypes.c_void_p), ("b", ctypes.c_void_p), ("Ea", ctypes.c_void_p),
                ("nu_f", ctypes.c_void_p), ("nu_r", ctypes.c_void_p), ("Le", ctypes.c_void_p),
                ("mu_ref", ctypes.c_double), ("T_ref", ctypes.c_double), ("mu_exp", ctypes.c_double),
                ("Pr", ctypes.c_double), ("bulk_ratio", ctypes.c_double),
                ("m47", ctypes.c_double), ("m48", ctypes.c_double)]


class Scheme(ctypes.Structure):
    _fields_ = [("n_coarse", ctypes.c_int), ("sweeps", ctypes.c_int), ("n_fine", ctypes.c_int),
                ("fine_repeat", ctypes.c_int), ("mode", ctypes.c_int)]


_vp, _ip, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
_SIGS = {
    "sdc_context_create": [ctypes.POINTER(_vp), _ip],
    "sdc_context_destroy": [_vp],
    "set_mechanism": [_vp, ctypes.POINTER(MechanismDesc)],
    "sdc_species_supported": [_ip],
    "prim_to_cons": [_vp, ctypes.POINTER(BoxDesc), _vp, _vp, _vp, _vp, _vp, _vp],
    "rhs_eval": [_vp, ctypes.POINTER(BoxDesc), _vp, _vp, ctypes.c_uint, _vp],
    "rhs_eval_static": [_vp, ctypes.POINTER(BoxDesc), _vp, _vp, ctypes.c_uint, _vp],
    "sdc_workspace_size": [_vp, _ip, ctypes.POINTER(BoxDesc), ctypes.POINTER(Scheme),
                           ctypes.POINTER(ctypes.c_size_t)],
    "sdc_step": [_vp, ctypes.POINTER(BoxDesc), _vp, _d, _ip, ctypes.POINTER(Scheme), _vp,
                 ctypes.c_size_t, _vp],
    "sdc_step_batched": [_vp, _ip, ctypes.POINTER(BoxDesc), ctypes.POINTER(_vp), _d, _ip,
                         ctypes.POINTER(Scheme), _vp, ctypes.c_size_t, _vp],
    "last_status": [_vp, _vp],
    "sdc_set_tiles": [_vp, _ip, _ip, _ip, _ip, _ip, _ip, _ip],
    "sdc_set_graph": [_vp, _ip],
    "sdc_autotune": [_vp, _ip, ctypes.POINTER(BoxDesc), ctypes.POINTER(_vp), _vp, ctypes.c_size_t, _vp,
                     ctypes.POINTER(ctypes.c_int)],
    "rhs_vjp": [_vp, ctypes.POINTER(BoxDesc), _vp, _vp, _vp, _vp, ctypes.c_uint, _vp],
    "set_log_prefactors": [_vp, _vp],
    "set_reference_species": [_vp, _ip],
    "sdc_set_residual_exit": [_vp, ctypes.c_double],
    "set_wide_stencil": [_vp, _ip],
    "sdc_set_fused_fine": [_vp, _ip],
    "sdc_residual_history": [_vp, _ip, _vp, _vp, _vp],
    "sdc_vjp_workspace_size": [_vp, ctypes.POINTER(BoxDesc), ctypes.POINTER(Scheme), _ip,
                               ctypes.POINTER(ctypes.c_size_t)],
    "sdc_step_vjp": [_vp, ctypes.POINTER(BoxDesc), _vp, _d, _ip, ctypes.POINTER(Scheme), _vp, _vp, _vp,
                     _vp, ctypes.c_size_t, _vp],
    "sdc_profile_enable": [_vp, _ip],
    "sdc_profile_read": [_vp, _vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)],
}
for _name, _args in _SIGS.items():
    getattr(_lib, _name).argtypes = _args
    getattr(_lib, _name).restype = ctypes.c_int
_lib.last_error_message.argtypes = [_vp]
_lib.last_error_message.restype = ctypes.c_char_p
_lib.sdc_kernel_name.argtypes = [_ip]
_lib.sdc_kernel_name.restype = ctypes.c_char_p

EXPORTS = list(_SIGS) + ["last_error_message", "sdc_kernel_name"]


class NarrowSDCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"narrowsdc error {code}: {msg}")
        self.code = code


def box(nx, ny, nz, dx, dy=None, dz=None, nonperiodic=0):
    """nonperiodic: bit d (1 x, 2 y, 4 z) for physical boundaries along d."""
    return BoxDesc(nx, ny, nz, NG, dx, dx if dy is None else dy, dx if dz is None else dz, int(nonperiodic))


def scheme(n_coarse=4, sweeps=6, n_fine=0, fine_repeat=1, mode=1):
    return Scheme(n_coarse, sweeps, n_fine, fine_repeat, mode)


def species_supported(ns):
    """Whether the library's kernels were compiled for ``ns`` species."""
    return bool(_lib.sdc_species_supported(int(ns)))


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    import torch
    if isinstance(t, torch.Tensor):
        assert t.is_cuda and t.is_contiguous() and t.dtype == torch.float64, "device FP64 contiguous tensor expected"
        return ctypes.c_void_p(t.data_ptr())
    return ctypes.c_void_p(int(t))


class Context:
    """A library context on one HIP device."""

    def __init__(self, device=0):
        h = ctypes.c_void_p()
        rc = _lib.sdc_context_create(ctypes.byref(h), device)
        if rc != SDC_OK:
            raise NarrowSDCError(rc, "context creation failed")
        self.h = h
        self.ns = None
        self._mech_keep = None

    def close(self):
        if self.h:
            _lib.sdc_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != SDC_OK:
            raise NarrowSDCError(rc, _lib.last_error_message(self.h).decode())

    def set_mechanism(self, mech):
        k = dict(W=np.ascontiguousarray(mech["W"], np.float64),
                 nasa=np.ascontiguousarray(mech["nasa"], np.float64),
                 A=np.ascontiguousarray(mech["A"], np.float64),
                 b=np.ascontiguousarray(mech["b"], np.float64),
                 Ea=np.ascontiguousarray(mech["Ea"], np.float64),
                 nu_f=np.ascontiguousarray(mech["nu_f"], np.int32),
                 nu_r=np.ascontiguousarray(mech["nu_r"], np.int32),
                 Le=np.ascontiguousarray(mech["Le"], np.float64))
        d = MechanismDesc(int(mech["ns"]), int(mech["nr"]), k["W"].ctypes.data, k["nasa"].ctypes.data,
                          mech["Tlo"], mech["Thi"], k["A"].ctypes.data, k["b"].ctypes.data,
                          k["Ea"].ctypes.data, k["nu_f"].ctypes.data, k["nu_r"].ctypes.data,
                          k["Le"].ctypes.data, mech["mu_ref"], mech["T_ref"], mech["mu_exp"],
                          mech["Pr"], mech["bulk_ratio"], mech["m47"], mech["m48"])
        self._check(_lib.set_mechanism(self.h, ctypes.byref(d)))
        self.ns = int(mech["ns"])

    def prim_to_cons(self, bx, p, T, Y, u, U, stream=None):
        self._check(_lib.prim_to_cons(self.h, ctypes.byref(bx), _ptr(p), _ptr(T), _ptr(Y), _ptr(u),
                                      _ptr(U), _stream(stream)))

    def rhs_eval(self, bx, U, dUdt, parts=RHS_ALL, stream=None):
        self._check(_lib.rhs_eval(self.h, ctypes.byref(bx), _ptr(U), _ptr(dUdt), parts, _stream(stream)))

    def rhs_eval_static(self, bx, U, dUdt, parts=RHS_ALL, stream=None):
        """rhs_eval with the library's static scratch array (no device
        allocation in the call; see the header for the size limit)."""
        self._check(_lib.rhs_eval_static(self.h, ctypes.byref(bx), _ptr(U), _ptr(dUdt), parts,
                                         _stream(stream)))

    def workspace_size(self, boxes, sch):
        arr = (BoxDesc * len(boxes))(*boxes)
        n = ctypes.c_size_t()
        self._check(_lib.sdc_workspace_size(self.h, len(boxes), arr, ctypes.byref(sch), ctypes.byref(n)))
        return n.value

    def sdc_step(self, bx, U, dt, nsteps, sch, ws, ws_bytes, stream=None):
        self._check(_lib.sdc_step(self.h, ctypes.byref(bx), _ptr(U), dt, nsteps, ctypes.byref(sch),
                                  _ptr(ws) if ws is not None else None, ws_bytes, _stream(stream)))

    def sdc_step_batched(self, boxes, Us, dt, nsteps, sch, ws, ws_bytes, stream=None):
        arr = (BoxDesc * len(boxes))(*boxes)
        ptrs = (ctypes.c_void_p * len(Us))(*[_ptr(u).value for u in Us])
        self._check(_lib.sdc_step_batched(self.h, len(boxes), arr, ptrs, dt, nsteps, ctypes.byref(sch),
                                          _ptr(ws), ws_bytes, _stream(stream)))

    def last_status(self, stream=None):
        return _lib.last_status(self.h, _stream(stream))

    def check_status(self, stream=None):
        self._check(self.last_status(stream))

    def set_tiles(self, interior=(0, 0, 0), stored=(0, 0, 0), grid_cap=0):
        self._check(_lib.sdc_set_tiles(self.h, *interior, *stored, grid_cap))

    def set_graph(self, enable=True):
        self._check(_lib.sdc_set_graph(self.h, 1 if enable else 0))

    def autotune(self, boxes, Us, ws, ws_bytes, stream=None):
        arr = (BoxDesc * len(boxes))(*boxes)
        ptrs = (ctypes.c_void_p * len(Us))(*[_ptr(u).value for u in Us])
        ch = (ctypes.c_int * 4)()
        self._check(_lib.sdc_autotune(self.h, len(boxes), arr, ptrs, _ptr(ws), ws_bytes, _stream(stream), ch))
        return tuple(ch)

    def rhs_vjp(self, bx, U, dUdt_bar, U_bar, lnA_bar=None, parts=RHS_ALL, stream=None):
        """U_bar += (d rhs/dU)^T dUdt_bar; lnA_bar += (d rhs/d lnA)^T dUdt_bar."""
        self._check(_lib.rhs_vjp(self.h, ctypes.byref(bx), _ptr(U), _ptr(dUdt_bar), _ptr(U_bar),
                                 _ptr(lnA_bar), parts, _stream(stream)))

    def set_wide_stencil(self, enable=True):
        """Second derivatives with the wide stencil D(a D u) (Section 2.2)
        instead of the narrow one."""
        self._check(_lib.set_wide_stencil(self.h, 1 if enable else 0))

    def set_fused_fine(self, enable=True):
        """Multirate fine sub-steps in one kernel where the scheme and
        mechanism allow it (results are identical either way)."""
        self._check(_lib.sdc_set_fused_fine(self.h, 1 if enable else 0))

    def set_residual_exit(self, ratio=0.0):
        """0: K sweeps per step; ratio > 1: skip a step's remaining sweeps once
        successive residuals of eq. (residual) shrink by less than ratio."""
        self._check(_lib.sdc_set_residual_exit(self.h, float(ratio)))

    def residual_history(self):
        """(residuals measured by the last sdc_step call, sweeps it performed)."""
        n, sw = ctypes.c_int(), ctypes.c_int()
        self._check(_lib.sdc_residual_history(self.h, 0, None, ctypes.byref(n), ctypes.byref(sw)))
        out = np.zeros(max(n.value, 1))
        self._check(_lib.sdc_residual_history(self.h, n.value, ctypes.c_void_p(out.ctypes.data), ctypes.byref(n),
                                              ctypes.byref(sw)))
        return out[:n.value], sw.value

    def set_reference_species(self, k=-1):
        """-1: correction-velocity species diffusion (default); k >= 0:
        reference species k (Section 2.1)."""
        self._check(_lib.set_reference_species(self.h, int(k)))

    def set_log_prefactors(self, lnA):
        a = np.ascontiguousarray(lnA, dtype=np.float64)
        self._check(_lib.set_log_prefactors(self.h, ctypes.c_void_p(a.ctypes.data)))

    def vjp_workspace_size(self, bx, sch, nsteps):
        n = ctypes.c_size_t()
        self._check(_lib.sdc_vjp_workspace_size(self.h, ctypes.byref(bx), ctypes.byref(sch), nsteps,
                                                ctypes.byref(n)))
        return n.value

    def sdc_step_vjp(self, bx, U0, dt, nsteps, sch, UN_bar, U0_bar, lnA_bar, ws, ws_bytes, stream=None):
        self._check(_lib.sdc_step_vjp(self.h, ctypes.byref(bx), _ptr(U0), dt, nsteps, ctypes.byref(sch),
                                      _ptr(UN_bar), _ptr(U0_bar), _ptr(lnA_bar), _ptr(ws), ws_bytes,
                                      _stream(stream)))

    def profile(self, enable=True):
        self._check(_lib.sdc_profile_enable(self.h, 1 if enable else 0))

    def profile_read(self, stream=None):
        """{kernel name: (total ms, launches)} since the last read."""
        tot = (ctypes.c_double * 32)()
        cnt = (ctypes.c_int * 32)()
        n = _lib.sdc_profile_read(self.h, _stream(stream), tot, cnt)
        if n < 0:
            self._check(n)
        return {_lib.sdc_kernel_name(i).decode(): (tot[i], cnt[i]) for i in range(n) if cnt[i] > 0}


# ------------------------------------------------------------- helpers
def ghosted_shape(nU, nz, ny, nx):
    return (nU, nz + 2 * NG, ny + 2 * NG, nx + 2 * NG)


def interior(U):
    """Interior view of a ghosted [nU][nz+8][ny+8][nx+8] array."""
    return U[:, NG:-NG, NG:-NG, NG:-NG]


def workspace(ctx, boxes, sch, device="cuda"):
    import torch
    n = ctx.workspace_size(boxes, sch)
    return torch.empty(max(n // 8, 1), dtype=torch.float64, device=device), n
