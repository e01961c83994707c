"""Oracle: plain CPU FP64 reference (TEST INFRASTRUCTURE ONLY).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use this package.  It shares no code with the HIP library.

``liboracle.so`` is built from ``oracle.cpp`` with g++ (-O2, no FP
contraction, OpenMP); the Python side only marshals arrays.  Time stepping
(spectral deferred corrections) is in :mod:`oracle.sdc`.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

HYP, DIFF, REACT = 1, 2, 4
AD = HYP | DIFF
ALL = HYP | DIFF | REACT


def build(force=False):
    src = os.path.join(HERE, "oracle.cpp")
    deps = [src, os.path.join(HERE, "oracle.h"), os.path.join(HERE, "dual.hpp")]
    if not force and os.path.exists(LIB_PATH) and \
            os.path.getmtime(LIB_PATH) >= max(os.path.getmtime(d) for d in deps):
        return LIB_PATH
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", src, "-o", LIB_PATH + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _OMech(ctypes.Structure):
    _fields_ = [
        ("ns", ctypes.c_int), ("nr", ctypes.c_int),
        ("W", ctypes.c_void_p), ("nasa", ctypes.c_void_p),
        ("Tlo", ctypes.c_double), ("Thi", ctypes.c_double),
        ("A", ctypes.c_void_p), ("b", ctypes.c_void_p), ("Ea", ctypes.c_void_p),
        ("nu_f", ctypes.c_void_p), ("nu_r", ctypes.c_void_p), ("Le", ctypes.c_void_p),
        ("mu_ref", ctypes.c_double), ("T_ref", ctypes.c_double), ("mu_exp", ctypes.c_double),
        ("Pr", ctypes.c_double), ("bulk_ratio", ctypes.c_double),
        ("m47", ctypes.c_double), ("m48", ctypes.c_double),
        ("ref_species", ctypes.c_int), ("wide_stencil", ctypes.c_int),
        ("nonperiodic", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.c_void_p
        L.oracle_d1_point.restype = ctypes.c_double
        L.oracle_d1_point.argtypes = [dp, ctypes.c_double]
        L.oracle_narrow_point.restype = ctypes.c_double
        L.oracle_narrow_point.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.oracle_narrow_matrix.argtypes = [ctypes.c_double, ctypes.c_double, dp]
        L.oracle_narrow6_matrix.argtypes = [ctypes.c_double, dp]
        L.oracle_d1_periodic.argtypes = [ctypes.c_int, dp, ctypes.c_double, dp]
        L.oracle_d1_line.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_int, dp]
        L.oracle_narrow_line.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, dp]
        L.oracle_narrow4_matrix.argtypes = [dp]
        L.oracle_narrow_periodic.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, dp]
        L.oracle_heat2d.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, dp]
        L.oracle_species_thermo.argtypes = [dp, ctypes.c_double, dp, dp, dp]
        L.oracle_rate_constants.argtypes = [dp, ctypes.c_double, dp, dp]
        L.oracle_prim_to_cons.argtypes = [dp, ctypes.c_long, dp, dp, dp, dp, dp]
        L.oracle_cons_to_prim.argtypes = [dp, ctypes.c_long, dp, dp]
        L.oracle_production.argtypes = [dp, ctypes.c_long, dp, dp]
        L.oracle_sound_speed.argtypes = [dp, ctypes.c_long, dp, dp]
        L.oracle_rhs.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, dp, ctypes.c_uint, dp, ctypes.c_int]
        L.oracle_rhs_cells.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, dp, ctypes.c_uint,
                                       ctypes.c_int, dp, dp, ctypes.c_int]
        L.oracle_rhs_jvp.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, dp, dp, dp, ctypes.c_uint,
                                     dp, dp, ctypes.c_int]
        L.oracle_rhs_jvp_cells.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, dp, dp, dp, ctypes.c_uint,
                                           ctypes.c_int, dp, dp, ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Mechanism:
    """Holds contiguous copies of a mechanism dict and its C descriptor.
    ref_species: -1 for the correction-velocity form of the species
    diffusion, k >= 0 for reference species k (Section 2.1).  wide: the
    wide stencil D(a D u) instead of the narrow one for the second-derivative
    terms (Section 2.2).  nonperiodic: bit d set for physical boundaries at
    both ends of direction d, with the boundary stencils of Section 2.5."""

    def __init__(self, mech, ref_species=-1, wide=False, nonperiodic=0):
        self.mech = mech
        self.ns = int(mech["ns"])
        self.nr = int(mech["nr"])
        self._keep = dict(
            W=_f64(mech["W"]), nasa=_f64(mech["nasa"]), A=_f64(mech["A"]), b=_f64(mech["b"]),
            Ea=_f64(mech["Ea"]), Le=_f64(mech["Le"]),
            nu_f=np.ascontiguousarray(mech["nu_f"], dtype=np.int32),
            nu_r=np.ascontiguousarray(mech["nu_r"], dtype=np.int32))
        k = self._keep
        self.c = _OMech(
            self.ns, self.nr, _ptr(k["W"]).value, _ptr(k["nasa"]).value, mech["Tlo"], mech["Thi"],
            _ptr(k["A"]).value, _ptr(k["b"]).value, _ptr(k["Ea"]).value,
            _ptr(k["nu_f"]).value, _ptr(k["nu_r"]).value, _ptr(k["Le"]).value,
            mech["mu_ref"], mech["T_ref"], mech["mu_exp"], mech["Pr"], mech["bulk_ratio"],
            mech["m47"], mech["m48"], int(ref_species), int(bool(wide)), int(nonperiodic))
        self.ref_species = int(ref_species)
        self.wide = bool(wide)
        self.nonperiodic = int(nonperiodic)

    @property
    def ref(self):
        return ctypes.byref(self.c)


def _check(st, what):
    if st != 0:
        raise RuntimeError(f"oracle {what} failed with status {st}")


# ----------------------------------------------------------------- stencils
def narrow_matrix(m47, m48):
    M = np.zeros((8, 8))
    lib().oracle_narrow_matrix(m47, m48, _ptr(M))
    return M


def narrow6_matrix(m36):
    M = np.zeros((6, 6))
    lib().oracle_narrow6_matrix(m36, _ptr(M))
    return M


def d1_point(f9, dx):
    f9 = _f64(f9)
    return lib().oracle_d1_point(_ptr(f9), dx)


def narrow_point(a9, u9, dx, m47, m48):
    a9, u9 = _f64(a9), _f64(u9)
    return lib().oracle_narrow_point(_ptr(a9), _ptr(u9), dx, m47, m48)


def narrow4_matrix():
    M = np.zeros((4, 4))
    lib().oracle_narrow4_matrix(_ptr(M))
    return M


def d1_line(f, dx, kind):
    """First derivative on a line with physical boundaries at both ends
    (kind 0 advection, 1 diffusion closures)."""
    f = _f64(f)
    out = np.zeros_like(f)
    lib().oracle_d1_line(len(f), _ptr(f), dx, int(kind), _ptr(out))
    return out


def narrow_line(a, u, dx, m47, m48):
    """d/dx(a du/dx) on a line with physical boundaries at both ends."""
    a, u = _f64(a), _f64(u)
    out = np.zeros_like(u)
    lib().oracle_narrow_line(len(u), _ptr(a), _ptr(u), dx, m47, m48, _ptr(out))
    return out


def d1_periodic(f, dx):
    f = _f64(f)
    out = np.zeros_like(f)
    lib().oracle_d1_periodic(len(f), _ptr(f), dx, _ptr(out))
    return out


def narrow_periodic(a, u, dx, m47, m48):
    a, u = _f64(a), _f64(u)
    out = np.zeros_like(u)
    lib().oracle_narrow_periodic(len(u), _ptr(a), _ptr(u), dx, m47, m48, _ptr(out))
    return out


def heat2d(a, b, u, dx, m47, m48):
    a, b, u = _f64(a), _f64(b), _f64(u)
    out = np.zeros_like(u)
    lib().oracle_heat2d(u.shape[0], _ptr(a), _ptr(b), _ptr(u), dx, m47, m48, _ptr(out))
    return out


# ----------------------------------------------------------- thermochemistry
def species_thermo(om, T):
    cp, h, s = (np.zeros(om.ns) for _ in range(3))
    lib().oracle_species_thermo(om.ref, T, _ptr(cp), _ptr(h), _ptr(s))
    return cp, h, s


def rate_constants(om, T):
    kf, kr = np.zeros(om.nr), np.zeros(om.nr)
    lib().oracle_rate_constants(om.ref, T, _ptr(kf), _ptr(kr))
    return kf, kr


def prim_to_cons(om, prim):
    p = _f64(prim["p"])
    shape = p.shape
    n = p.size
    T = _f64(prim["T"])
    Y = _f64(prim["Y"])
    u = _f64(prim["u"])
    U = np.zeros((5 + om.ns,) + shape)
    _check(lib().oracle_prim_to_cons(om.ref, n, _ptr(p), _ptr(T), _ptr(Y), _ptr(u), _ptr(U)),
           "prim_to_cons")
    return U


def cons_to_prim(om, U):
    U = _f64(U)
    n = U[0].size
    out = np.zeros((6,) + U.shape[1:])
    _check(lib().oracle_cons_to_prim(om.ref, n, _ptr(U), _ptr(out)), "cons_to_prim")
    return out


def sound_speed(om, U):
    U = _f64(U)
    n = U[0].size
    out = np.zeros(U.shape[1:])
    _check(lib().oracle_sound_speed(om.ref, n, _ptr(U), _ptr(out)), "sound_speed")
    return out


def production(om, U):
    U = _f64(U)
    n = U[0].size
    out = np.zeros((om.ns,) + U.shape[1:])
    _check(lib().oracle_production(om.ref, n, _ptr(U), _ptr(out)), "production")
    return out


# ------------------------------------------------------------ right-hand side
def rhs(om, U, dx, parts=ALL, nthreads=0):
    """U: interior state [nU][nz][ny][nx]; dx scalar or (dx, dy, dz)."""
    U = _f64(U)
    nU, nz, ny, nx = U.shape
    assert nU == 5 + om.ns
    h = np.broadcast_to(np.asarray(dx, dtype=np.float64), (3,))
    out = np.zeros_like(U)
    _check(lib().oracle_rhs(om.ref, nx, ny, nz, h[0], h[1], h[2], _ptr(U), parts, _ptr(out),
                            nthreads), "rhs")
    return out


def rhs_cells(om, U, dx, cells, parts=ALL, nthreads=0):
    """RHS at listed interior cells (array [n][3] of x, y, z) -> [n][nU]."""
    U = _f64(U)
    nU, nz, ny, nx = U.shape
    h = np.broadcast_to(np.asarray(dx, dtype=np.float64), (3,))
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    out = np.zeros((len(cells), nU))
    _check(lib().oracle_rhs_cells(om.ref, nx, ny, nz, h[0], h[1], h[2], _ptr(U), parts,
                                  len(cells), _ptr(cells), _ptr(out), nthreads), "rhs_cells")
    return out


def rhs_jvp(om, U, dx, wU, wA=None, parts=ALL, nthreads=0):
    """(rhs(U), d rhs/dU . wU + d rhs/d lnA . wA) by forward-mode dual numbers."""
    U = _f64(U)
    wU = _f64(wU)
    nU, nz, ny, nx = U.shape
    h = np.broadcast_to(np.asarray(dx, dtype=np.float64), (3,))
    out = np.zeros_like(U)
    jvp = np.zeros_like(U)
    wA = _f64(wA) if wA is not None else None
    _check(lib().oracle_rhs_jvp(om.ref, nx, ny, nz, h[0], h[1], h[2], _ptr(U), _ptr(wU),
                                _ptr(wA), parts, _ptr(out), _ptr(jvp), nthreads), "rhs_jvp")
    return out, jvp


def rhs_jvp_cells(om, U, dx, wU, cells, wA=None, parts=ALL, nthreads=0):
    """d rhs/dU . wU + d rhs/d lnA . wA at listed interior cells ([n][3] of
    x, y, z) -> [n][nU]."""
    U = _f64(U)
    wU = _f64(wU)
    nU, nz, ny, nx = U.shape
    h = np.broadcast_to(np.asarray(dx, dtype=np.float64), (3,))
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    jvp = np.zeros((len(cells), nU))
    wA = _f64(wA) if wA is not None else None
    _check(lib().oracle_rhs_jvp_cells(om.ref, nx, ny, nz, h[0], h[1], h[2], _ptr(U), _ptr(wU),
                                      _ptr(wA), parts, len(cells), _ptr(cells), _ptr(jvp), nthreads),
           "rhs_jvp_cells")
    return jvp
