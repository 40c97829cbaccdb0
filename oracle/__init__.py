"""CPU oracle for the hydro step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never touches it, and the two share no code.

The arithmetic lives in ``hydro_ref.c`` (plain C, FP64, -ffp-contract=off);
this module builds and loads it with ctypes and marshals numpy arrays.
The functions follow the method described in Sec. II ("Solvers"): PPM
reconstruction at 26 quadrature points, central-upwind (Kurganov-Tadmor)
face flux with Newton-Cotes (Simpson) quadrature, finite-volume divergence.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hydro_ref.c")
SUBGRID_SIZES = (8, 16)     # interior cells per dimension; 8 is the default

CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra"]
# The sanitizer build (HYDRO_REF_SANITIZE=1 in the environment): address and
# undefined-behaviour checks, every finding fatal.  A process that loads it
# must have the address-sanitizer runtime preloaded (LD_PRELOAD).
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer", "-g"]


def sanitized() -> bool:
    return os.environ.get("HYDRO_REF_SANITIZE", "") == "1"


def lib_path(n: int = 8, san: bool | None = None) -> str:
    san = sanitized() if san is None else san
    base = "libhydro_ref" + ("" if n == 8 else f"_n{n}") + ("_san" if san else "")
    return os.path.join(_HERE, base + ".so")


def build(force: bool = False, n: int | None = None, san: bool | None = None) -> str:
    """Compile the oracle with gcc into ``oracle/libhydro_ref.so`` (subgrid
    size 8) and ``libhydro_ref_n16.so`` (size 16), or their ``_san``
    sanitizer builds; returns the size-n path."""
    san = sanitized() if san is None else san
    for m in (SUBGRID_SIZES if n is None else (n,)):
        path = lib_path(m, san)
        if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            tmp = path + ".tmp"
            subprocess.run(["gcc", *CFLAGS, *(SAN_FLAGS if san else []), f"-DREF_N={m}", "-o",
                            tmp, _SRC, "-lm"], check=True)
            os.replace(tmp, path)
    return lib_path(8 if n is None else n, san)


_COUNT_SRC = os.path.join(_HERE, "count_build.cpp")
_COUNT_LIB = os.path.join(_HERE, "libhydro_ref_count.so")
_count_lib = None


def build_count(force: bool = False) -> str:
    """Compile the operation-counting build of the oracle (count_build.cpp
    includes hydro_ref.c unchanged; subgrid size 8)."""
    if (force or not os.path.exists(_COUNT_LIB)
            or os.path.getmtime(_COUNT_LIB) < max(os.path.getmtime(_SRC),
                                                  os.path.getmtime(_COUNT_SRC))):
        tmp = _COUNT_LIB + ".tmp"
        subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                        "-fno-fast-math", "-Wall", "-DREF_N=8", "-o", tmp, _COUNT_SRC, "-lm"],
                       check=True)
        os.replace(tmp, _COUNT_LIB)
    return _COUNT_LIB


def count_lib():
    global _count_lib
    if _count_lib is None:
        L = ctypes.CDLL(build_count())
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        P, B = ctypes.POINTER(Params), ctypes.POINTER(Batch)
        L.hydro_ref_step.argtypes = [P, B, dp, dp, dp, ip]
        L.hydro_ref_step.restype = ctypes.c_int
        L.hydro_ref_ppm1d.argtypes = [dp, dp, dp]
        L.hydro_ref_ppm1d.restype = ctypes.c_int
        L.hydro_ref_state_flux.argtypes = [P, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, ip]
        L.hydro_ref_state_flux.restype = ctypes.c_int
        L.hydro_ref_face.argtypes = [P, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, ip]
        L.hydro_ref_face.restype = ctypes.c_int
        L.hydro_ref_flops.argtypes = []
        L.hydro_ref_flops.restype = ctypes.c_ulonglong
        L.hydro_ref_flops_reset.argtypes = []
        _count_lib = L
    return _count_lib


def counted(fn_name, *args):
    """Call an entry point of the counting build; returns (return code,
    operations counted during the call)."""
    L = count_lib()
    L.hydro_ref_flops_reset()
    rc = getattr(L, fn_name)(*args)
    return rc, int(L.hydro_ref_flops())


def step_flops(U_in, offset, h, n_species, fstride, dt, gamma=5.0 / 3.0, de_switch=1e-3,
               flags=0):
    """One stage in the counting build: (U_out, amax, status, operations)."""
    U_in = _f64(U_in)
    ba = _BatchArgs(offset, h, n_species, fstride)
    U_out = U_in.copy()
    n = len(ba.offset)
    amax = np.zeros(n)
    status = np.zeros(n, dtype=np.int32)
    prm = params(gamma, de_switch, dt, flags)
    rc, ops = counted("hydro_ref_step", ctypes.byref(prm), ctypes.byref(ba.struct), _dp(U_in),
                      _dp(U_out), _dp(amax), status.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    assert rc == 0, rc
    return U_out, amax, status, ops


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("de_switch", ctypes.c_double),
                ("dt", ctypes.c_double), ("flags", ctypes.c_uint32)]


class Batch(ctypes.Structure):
    _fields_ = [("n_sub", ctypes.c_int32), ("fstride", ctypes.c_int32),
                ("offset", ctypes.POINTER(ctypes.c_int64)),
                ("h", ctypes.POINTER(ctypes.c_double)),
                ("n_species", ctypes.POINTER(ctypes.c_int32))]


_libs = {}


def lib(n: int = 8):
    if n not in _libs:
        assert n in SUBGRID_SIZES, n
        L = ctypes.CDLL(build(n=n))
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lp = ctypes.POINTER(ctypes.c_int64)
        P, B = ctypes.POINTER(Params), ctypes.POINTER(Batch)
        L.hydro_ref_ppm1d.argtypes = [dp, dp, dp]
        L.hydro_ref_ppm1d_cw.argtypes = [P, dp, dp, dp, dp, ctypes.c_int, dp, dp]
        L.hydro_ref_state_flux.argtypes = [P, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, ip]
        L.hydro_ref_face.argtypes = [P, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, ip]
        L.hydro_ref_reconstruct.argtypes = [P, B, dp, dp, lp]
        L.hydro_ref_flux.argtypes = [P, B, dp, lp, dp, lp, dp, ip]
        L.hydro_ref_divergence.argtypes = [P, B, dp, lp, dp, dp]
        L.hydro_ref_step.argtypes = [P, B, dp, dp, dp, ip]
        L.hydro_ref_tau_resync.argtypes = [P, B, dp]
        L.hydro_ref_q_elems.argtypes = [ctypes.c_int]
        L.hydro_ref_q_elems.restype = ctypes.c_int64
        L.hydro_ref_f_elems.argtypes = [ctypes.c_int]
        L.hydro_ref_f_elems.restype = ctypes.c_int64
        L.hydro_ref_subgrid_n.argtypes = []
        L.hydro_ref_subgrid_n.restype = ctypes.c_int
        assert L.hydro_ref_subgrid_n() == n
        for name in ("hydro_ref_ppm1d", "hydro_ref_ppm1d_cw", "hydro_ref_state_flux", "hydro_ref_face",
                     "hydro_ref_reconstruct", "hydro_ref_flux", "hydro_ref_divergence",
                     "hydro_ref_step", "hydro_ref_tau_resync"):
            getattr(L, name).restype = ctypes.c_int
        _libs[n] = L
    return _libs[n]


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


KT_SYMMETRIC = 1   # flags bit: one speed max(|u_n| + c) for both directions
VELOCITY = 2       # flags bit: PPM of v = s / rho; point momentum = rho_q * v_q
STEEPEN = 4        # flags bit: Colella-Woodward contact steepening (density)
FLATTEN = 8        # flags bit: Colella-Woodward flattening in strong compressions


def params(gamma=5.0 / 3.0, de_switch=1e-3, dt=0.0, flags=0):
    return Params(float(gamma), float(de_switch), float(dt), int(flags))


class _BatchArgs:
    """Keeps the metadata arrays alive while a call runs."""

    def __init__(self, offset, h, n_species, fstride):
        self.offset = np.ascontiguousarray(offset, dtype=np.int64)
        self.h = np.ascontiguousarray(h, dtype=np.float64)
        self.n_species = np.ascontiguousarray(n_species, dtype=np.int32)
        n = len(self.offset)
        self.struct = Batch(n, int(fstride),
                            self.offset.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            self.h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            self.n_species.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))


def ppm1d(u):
    """PPM on five values u_{-2..2}; returns (q+, q-) of the middle cell."""
    u = _f64(u)
    assert u.shape == (5,)
    qp, qm = ctypes.c_double(), ctypes.c_double()
    rc = lib().hydro_ref_ppm1d(_dp(u), ctypes.byref(qp), ctypes.byref(qm))
    assert rc == 0
    return qp.value, qm.value


def ppm1d_cw(u, rho, p, un, is_density, flags, gamma=5.0 / 3.0):
    """PPM of one line with the Colella-Woodward options in `flags`; rho, p
    and un are the densities, pressures and line velocities of the same five
    cells.  Returns (q+, q-)."""
    arrs = [_f64(x) for x in (u, rho, p, un)]
    assert all(a.shape == (5,) for a in arrs)
    qp, qm = ctypes.c_double(), ctypes.c_double()
    prm = params(gamma, flags=flags)
    rc = lib().hydro_ref_ppm1d_cw(ctypes.byref(prm), *[_dp(a) for a in arrs], int(is_density),
                                  ctypes.byref(qp), ctypes.byref(qm))
    assert rc == 0
    return qp.value, qm.value


def state_flux(V, axis, gamma=5.0 / 3.0, de_switch=1e-3):
    """Physical flux F(V) along axis, normal velocity, sound speed, pressure, status."""
    V = _f64(V)
    nf = V.shape[0]
    F = np.zeros(nf)
    un, cs, p = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    st = ctypes.c_int32()
    prm = params(gamma, de_switch)
    rc = lib().hydro_ref_state_flux(ctypes.byref(prm), nf, axis, _dp(V), _dp(F),
                                    ctypes.byref(un), ctypes.byref(cs), ctypes.byref(p),
                                    ctypes.byref(st))
    assert rc == 0
    return F, un.value, cs.value, p.value, st.value


def face(VL, VR, axis, gamma=5.0 / 3.0, de_switch=1e-3, flags=0):
    """Central-upwind Simpson-averaged flux of one face from [9][nf] states."""
    VL, VR = _f64(VL), _f64(VR)
    assert VL.shape == VR.shape and VL.shape[0] == 9
    nf = VL.shape[1]
    Fbar = np.zeros(nf)
    a = ctypes.c_double()
    st = ctypes.c_int32()
    prm = params(gamma, de_switch, flags=flags)
    rc = lib().hydro_ref_face(ctypes.byref(prm), nf, axis, _dp(VL), _dp(VR), _dp(Fbar),
                              ctypes.byref(a), ctypes.byref(st))
    assert rc == 0
    return Fbar, a.value, st.value


def q_elems(n_species, n=8):
    return int(lib(n).hydro_ref_q_elems(int(n_species)))


def f_elems(n_species, n=8):
    return int(lib(n).hydro_ref_f_elems(int(n_species)))


def packed_offsets(sizes):
    off = np.zeros(len(sizes), dtype=np.int64)
    if len(sizes) > 1:
        off[1:] = np.cumsum(np.asarray(sizes[:-1], dtype=np.int64))
    return off


def reconstruct(U, offset, h, n_species, fstride, gamma=5.0 / 3.0, de_switch=1e-3, flags=0,
                n=8):
    """Q for every subgrid, packed; returns (Q, q_offset).  n: subgrid size."""
    U = _f64(U)
    ba = _BatchArgs(offset, h, n_species, fstride)
    q_off = packed_offsets([q_elems(ns, n) for ns in ba.n_species])
    total = int(q_off[-1] + q_elems(ba.n_species[-1], n)) if len(q_off) else 0
    Q = np.zeros(total)
    prm = params(gamma, de_switch, flags=flags)
    rc = lib(n).hydro_ref_reconstruct(ctypes.byref(prm), ctypes.byref(ba.struct), _dp(U), _dp(Q),
                                     q_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    assert rc == 0, rc
    return Q, q_off


def flux(Q, q_offset, offset, h, n_species, fstride, gamma=5.0 / 3.0, de_switch=1e-3, flags=0,
         n=8):
    """Face fluxes; returns (F, f_offset, amax, status)."""
    Q = _f64(Q)
    q_offset = np.ascontiguousarray(q_offset, dtype=np.int64)
    ba = _BatchArgs(offset, h, n_species, fstride)
    f_off = packed_offsets([f_elems(ns, n) for ns in ba.n_species])
    total = int(f_off[-1] + f_elems(ba.n_species[-1], n)) if len(f_off) else 0
    F = np.zeros(total)
    amax = np.zeros(len(ba.offset))
    status = np.zeros(len(ba.offset), dtype=np.int32)
    prm = params(gamma, de_switch, flags=flags)
    rc = lib(n).hydro_ref_flux(ctypes.byref(prm), ctypes.byref(ba.struct), _dp(Q),
                              q_offset.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(F),
                              f_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(amax),
                              status.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    assert rc == 0, rc
    return F, f_off, amax, status


def divergence(F, f_offset, U_in, offset, h, n_species, fstride, dt,
               gamma=5.0 / 3.0, de_switch=1e-3, n=8):
    """U_out from face fluxes; ghosts of U_out are copied from U_in."""
    F, U_in = _f64(F), _f64(U_in)
    f_offset = np.ascontiguousarray(f_offset, dtype=np.int64)
    ba = _BatchArgs(offset, h, n_species, fstride)
    U_out = U_in.copy()
    prm = params(gamma, de_switch, dt)
    rc = lib(n).hydro_ref_divergence(ctypes.byref(prm), ctypes.byref(ba.struct), _dp(F),
                                    f_offset.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    _dp(U_in), _dp(U_out))
    assert rc == 0, rc
    return U_out


def step(U_in, offset, h, n_species, fstride, dt, gamma=5.0 / 3.0, de_switch=1e-3, flags=0,
         n=8):
    """One forward-Euler hydro stage; returns (U_out, amax, status).

    Ghost cells of U_out are copies of U_in (the step never writes them)."""
    U_in = _f64(U_in)
    ba = _BatchArgs(offset, h, n_species, fstride)
    U_out = U_in.copy()
    nsub = len(ba.offset)
    amax = np.zeros(nsub)
    status = np.zeros(nsub, dtype=np.int32)
    prm = params(gamma, de_switch, dt, flags)
    rc = lib(n).hydro_ref_step(ctypes.byref(prm), ctypes.byref(ba.struct), _dp(U_in),
                              _dp(U_out), _dp(amax),
                              status.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    assert rc == 0, rc
    return U_out, amax, status


def step_threaded(U_in, offset, h, n_species, fstride, dt, threads=None, **kw):
    """oracle.step over disjoint slices of the batch in threads (the C calls
    release the interpreter lock, and the oracle keeps no global state); the
    result is the single-threaded one, subgrid by subgrid."""
    from concurrent.futures import ThreadPoolExecutor
    offset = np.ascontiguousarray(offset, dtype=np.int64)
    h = np.ascontiguousarray(h, dtype=np.float64)
    n_species = np.ascontiguousarray(n_species, dtype=np.int32)
    n = len(offset)
    threads = threads or min(16, os.cpu_count() or 1)
    U_in = _f64(U_in)
    U_out = U_in.copy()
    amax = np.zeros(n)
    status = np.zeros(n, dtype=np.int32)
    bounds = np.linspace(0, n, min(threads, max(n, 1)) + 1).astype(int)

    def run(lo, hi):
        if hi <= lo:
            return
        ba = _BatchArgs(offset[lo:hi], h[lo:hi], n_species[lo:hi], fstride)
        prm = params(kw.get("gamma", 5.0 / 3.0), kw.get("de_switch", 1e-3), dt, kw.get("flags", 0))
        st = np.zeros(hi - lo, dtype=np.int32)
        am = np.zeros(hi - lo)
        # outputs go straight into U_out: the slices' interiors are disjoint
        rc = lib(kw.get("n", 8)).hydro_ref_step(
            ctypes.byref(prm), ctypes.byref(ba.struct), _dp(U_in), _dp(U_out), _dp(am),
            st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        assert rc == 0, rc
        amax[lo:hi] = am
        status[lo:hi] = st

    lib(kw.get("n", 8))
    with ThreadPoolExecutor(len(bounds) - 1) as ex:
        list(ex.map(lambda i: run(bounds[i], bounds[i + 1]), range(len(bounds) - 1)))
    return U_out, amax, status


def tau_resync(U, offset, h, n_species, fstride, gamma=5.0 / 3.0, de_switch=1e-3, n=8):
    """Copy of U with the entropy tracer of every interior cell reset to
    e_i^(1/gamma) where e_i >= de_switch * E."""
    U = _f64(U).copy()
    ba = _BatchArgs(offset, h, n_species, fstride)
    prm = params(gamma, de_switch)
    rc = lib(n).hydro_ref_tau_resync(ctypes.byref(prm), ctypes.byref(ba.struct), _dp(U))
    assert rc == 0, rc
    return U


def raw_call(name, *args):
    """Direct access for argument-validation tests."""
    return getattr(lib(), name)(*args)
