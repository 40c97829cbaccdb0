"""Python binding of the gfx950 hydro library (ctypes over include/hydro.h).

Argument marshalling only: every stage of the hydro step runs in the HIP
kernels of ``libhydro.so``.  PyTorch provides device memory and streams.
If the library has not been built the calls raise; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhydro.so")

EXPORTS = [
    "hydro_reconstruct", "hydro_flux", "hydro_divergence", "hydro_step",
    "hydro_q_elems", "hydro_f_elems", "hydro_strerror",
    "hydro_variant_count", "hydro_variant_name", "hydro_step_variant",
    "hydro_autotune", "hydro_selected_variant",
    "hydro_plan_create", "hydro_plan_set_dt", "hydro_plan_launch", "hydro_plan_destroy",
    "hydro_fill_ghosts", "hydro_rate", "hydro_cfl_dt", "hydro_rk_update",
    "hydro_rk3_create", "hydro_rk3_launch", "hydro_rk3_destroy", "hydro_tau_resync",
    "hydro_rk_stage", "hydro_step_io", "hydro_workspace_bytes", "hydro_subgrid_n",
    "hydro_step_gather", "hydro_step_noalloc", "hydro_copy_blocks",
]

STATUS_RHO, STATUS_P, STATUS_NONFINITE, STATUS_BADMETA = 1, 2, 4, 8
KT_SYMMETRIC = 1   # params flag: one face speed max(|u_n| + c) for both directions
VELOCITY = 2       # params flag: PPM of v = s / rho; point momentum = rho_q v_q
STEEPEN = 4        # params flag: Colella-Woodward contact steepening of the density
FLATTEN = 8        # params flag: Colella-Woodward flattening in strong compressions


class HydroError(RuntimeError):
    pass


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("de_switch", ctypes.c_double),
                ("dt", ctypes.c_double), ("flags", ctypes.c_uint32)]


class Batch(ctypes.Structure):
    _fields_ = [("n_sub", ctypes.c_int32), ("fstride", ctypes.c_int32),
                ("offset", ctypes.c_void_p), ("h", ctypes.c_void_p),
                ("n_species", ctypes.c_void_p)]


class GhostMap(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("mode", ctypes.c_void_p)]


SUBGRID_SIZES = (8, 16)
_libs = {}


def lib_path(n: int = 8) -> str:
    return LIB_PATH if n == 8 else os.path.join(_PKG, f"libhydro_n{n}.so")


def lib(n: int = 8):
    """Load the library for subgrid size n: libhydro.so (8) or libhydro_n16.so
    (raises if it is missing: the product has no CPU path)."""
    if n not in _libs:
        if n not in SUBGRID_SIZES:
            raise HydroError(f"no library for subgrid size {n}; built sizes: {SUBGRID_SIZES}")
        path = lib_path(n)
        if not os.path.exists(path):
            raise HydroError(f"{path} is not built; run python -m paper_2210_06439_amd.build")
        L = ctypes.CDLL(path)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        P, B = ctypes.POINTER(Params), ctypes.POINTER(Batch)
        L.hydro_reconstruct.argtypes = [P, B, vp, vp, vp, vp]
        L.hydro_flux.argtypes = [P, B, vp, vp, vp, vp, vp, vp, vp]
        L.hydro_divergence.argtypes = [P, B, vp, vp, vp, vp, vp]
        L.hydro_step.argtypes = [P, B, vp, vp, vp, vp, vp]
        L.hydro_step_noalloc.argtypes = [P, B, vp, vp, vp, vp, vp]
        L.hydro_step_variant.argtypes = [P, B, vp, vp, vp, vp, ctypes.c_int, vp]
        L.hydro_autotune.argtypes = [P, B, vp, vp, vp, vp, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_float), vp]
        L.hydro_selected_variant.argtypes = [ctypes.c_int, ctypes.c_int]
        L.hydro_q_elems.argtypes = [ctypes.c_int]
        L.hydro_q_elems.restype = i64
        L.hydro_f_elems.argtypes = [ctypes.c_int]
        L.hydro_f_elems.restype = i64
        L.hydro_workspace_bytes.argtypes = []
        L.hydro_workspace_bytes.restype = i64
        L.hydro_subgrid_n.argtypes = []
        L.hydro_subgrid_n.restype = ctypes.c_int
        L.hydro_strerror.argtypes = [ctypes.c_int]
        L.hydro_strerror.restype = ctypes.c_char_p
        L.hydro_variant_name.argtypes = [ctypes.c_int]
        L.hydro_variant_name.restype = ctypes.c_char_p
        L.hydro_plan_create.argtypes = [P, B, vp, vp, vp, vp, vp, ctypes.POINTER(vp)]
        L.hydro_plan_set_dt.argtypes = [vp, ctypes.c_double]
        L.hydro_plan_launch.argtypes = [vp, vp]
        L.hydro_plan_destroy.argtypes = [vp]
        G, dbl = ctypes.POINTER(GhostMap), ctypes.c_double
        L.hydro_fill_ghosts.argtypes = [B, G, vp, vp, vp]
        L.hydro_rate.argtypes = [P, B, vp, vp, vp, vp, vp]
        L.hydro_cfl_dt.argtypes = [B, vp, dbl, dbl, vp, vp]
        L.hydro_rk_update.argtypes = [B, dbl, vp, dbl, vp, vp, vp, vp, vp]
        L.hydro_rk3_create.argtypes = [P, B, G, vp, vp, vp, vp, vp, vp, vp, dbl, dbl, vp,
                                       ctypes.POINTER(vp)]
        L.hydro_rk3_launch.argtypes = [vp, ctypes.c_int, vp]
        L.hydro_rk3_destroy.argtypes = [vp]
        L.hydro_tau_resync.argtypes = [P, B, vp, vp]
        L.hydro_rk_stage.argtypes = [P, B, vp, vp, vp, dbl, dbl, vp, vp, vp, vp]
        L.hydro_step_io.argtypes = [P, B, vp, vp, vp, vp, vp, vp]
        L.hydro_step_gather.argtypes = [P, B, G, vp, vp, vp, vp, vp]
        L.hydro_copy_blocks.argtypes = [vp, i64, vp, vp, i64, vp, vp, ctypes.c_int, i64, vp]
        if L.hydro_subgrid_n() != n:
            raise HydroError(f"{path} reports subgrid size {L.hydro_subgrid_n()}, not {n}")
        _libs[n] = L
        del i32
    return _libs[n]


def check(rc: int) -> int:
    if rc < 0:
        raise HydroError(f"hydro call failed ({rc}): {lib().hydro_strerror(rc).decode()}")
    return rc


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def params(gamma=5.0 / 3.0, de_switch=1e-3, dt=0.0, flags=0) -> Params:
    return Params(float(gamma), float(de_switch), float(dt), int(flags))


def q_elems(n_species: int, n: int = 8) -> int:
    return int(lib(n).hydro_q_elems(int(n_species)))


def f_elems(n_species: int, n: int = 8) -> int:
    return int(lib(n).hydro_f_elems(int(n_species)))


def variant_count() -> int:
    return int(lib().hydro_variant_count())


def variant_name(v: int) -> str:
    return lib().hydro_variant_name(int(v)).decode()


class DeviceBatch:
    """A batch of subgrids resident on the GPU: field buffer + metadata."""

    def __init__(self, U, offset, h, n_species, fstride, n: int = 8):
        import torch
        dev = torch.device("cuda")
        self.U = torch.as_tensor(U, dtype=torch.float64).to(dev)
        self.offset = torch.as_tensor(np.asarray(offset, dtype=np.int64)).to(dev)
        self.h = torch.as_tensor(np.asarray(h, dtype=np.float64)).to(dev)
        self.n_species = torch.as_tensor(np.asarray(n_species, dtype=np.int32)).to(dev)
        self.n_species_host = np.asarray(n_species, dtype=np.int32).copy()
        self.fstride = int(fstride)
        self.n = int(n)                 # subgrid size: which library the batch is for
        self.n_sub = int(len(self.n_species_host))
        self.struct = Batch(self.n_sub, self.fstride, self.offset.data_ptr(),
                            self.h.data_ptr(), self.n_species.data_ptr())

    @classmethod
    def from_inputs(cls, b):
        return cls(b.U, b.offset, b.h, b.n_species, b.fstride)

    def view(self, start: int, count: int) -> Batch:
        """Metadata of subgrids [start, start+count) (device pointer arithmetic)."""
        return Batch(int(count), self.fstride,
                     self.offset.data_ptr() + 8 * start, self.h.data_ptr() + 8 * start,
                     self.n_species.data_ptr() + 4 * start)

    def q_layout(self):
        sizes = [q_elems(ns, self.n) for ns in self.n_species_host]
        return _packed(sizes)

    def f_layout(self):
        sizes = [f_elems(ns, self.n) for ns in self.n_species_host]
        return _packed(sizes)


def _packed(sizes):
    import torch
    off = np.zeros(len(sizes), dtype=np.int64)
    if len(sizes) > 1:
        off[1:] = np.cumsum(np.asarray(sizes[:-1], dtype=np.int64))
    total = int(off[-1] + sizes[-1]) if len(sizes) else 0
    return torch.as_tensor(off).cuda(), total


def reconstruct(prm: Params, batch: Batch, U, Q, q_offset, stream=None, n: int = 8):
    check(lib(n).hydro_reconstruct(ctypes.byref(prm), ctypes.byref(batch), _ptr(U), _ptr(Q),
                                  _ptr(q_offset), _stream(stream)))


def flux(prm: Params, batch: Batch, Q, q_offset, F, f_offset, amax, status=None, stream=None,
         n: int = 8):
    check(lib(n).hydro_flux(ctypes.byref(prm), ctypes.byref(batch), _ptr(Q), _ptr(q_offset),
                           _ptr(F), _ptr(f_offset), _ptr(amax), _ptr(status), _stream(stream)))


def divergence(prm: Params, batch: Batch, F, f_offset, U_in, U_out, stream=None, n: int = 8):
    check(lib(n).hydro_divergence(ctypes.byref(prm), ctypes.byref(batch), _ptr(F),
                                 _ptr(f_offset), _ptr(U_in), _ptr(U_out), _stream(stream)))


def step(prm: Params, batch: Batch, U_in, U_out, amax, status=None, variant=None, stream=None):
    if variant is None:
        check(lib().hydro_step(ctypes.byref(prm), ctypes.byref(batch), _ptr(U_in), _ptr(U_out),
                               _ptr(amax), _ptr(status), _stream(stream)))
    else:
        check(lib().hydro_step_variant(ctypes.byref(prm), ctypes.byref(batch), _ptr(U_in),
                                       _ptr(U_out), _ptr(amax), _ptr(status), int(variant),
                                       _stream(stream)))


def step_noalloc(prm: Params, batch: Batch, U_in, U_out, amax, status=None, stream=None):
    """hydro_step without any device allocation (fixed scratch in the library;
    at most NOALLOC_MAX_SUB subgrids)."""
    check(lib().hydro_step_noalloc(ctypes.byref(prm), ctypes.byref(batch), _ptr(U_in),
                                   _ptr(U_out), _ptr(amax), _ptr(status), _stream(stream)))


NOALLOC_MAX_SUB = 65536
ESCRATCH = -4


def step_io(prm: Params, batch: Batch, out_offset, U_in, U_out, amax, status=None, stream=None):
    """Fused step writing subgrid s at out_offset[s] of U_out (which may be U_in
    when the output regions do not overlap the input regions)."""
    check(lib().hydro_step_io(ctypes.byref(prm), ctypes.byref(batch), _ptr(out_offset),
                              _ptr(U_in), _ptr(U_out), _ptr(amax), _ptr(status),
                              _stream(stream)))


def copy_blocks(src, src_row, dst, dst_row0, dst_row1=None, row_elems=None, stream=None):
    """Rows src_row[i] of src (row_elems doubles each) into rows dst_row0[i]
    and dst_row1[i] of dst; src and dst are flat float64 device tensors, the
    row indices int64 device tensors of one length."""
    n = int(src_row.numel())
    if row_elems is None:
        raise HydroError("row_elems is required")
    for t in (dst_row0, dst_row1):
        if t is not None and int(t.numel()) != n:
            raise HydroError("row index arrays differ in length")
    check(lib().hydro_copy_blocks(_ptr(src), int(src.numel()) // int(row_elems), _ptr(src_row),
                                  _ptr(dst), int(dst.numel()) // int(row_elems), _ptr(dst_row0),
                                  _ptr(dst_row1), n, int(row_elems), _stream(stream)))


def autotune(prm: Params, batch: Batch, U_in, U_out, amax, status=None, reps=3, stream=None):
    """Time every launch variant on this batch; returns (best, times_ms)."""
    n = variant_count()
    times = (ctypes.c_float * n)()
    best = check(lib().hydro_autotune(ctypes.byref(prm), ctypes.byref(batch), _ptr(U_in),
                                      _ptr(U_out), _ptr(amax), _ptr(status), int(reps), times,
                                      _stream(stream)))
    return best, [float(t) for t in times]


def selected_variant(n_sub: int) -> int:
    return int(lib().hydro_selected_variant(int(n_sub), 5))


class Plan:
    """A fused step recorded into a hipGraph; replay with launch()."""

    def __init__(self, prm: Params, batch: Batch, U_in, U_out, amax, status=None, stream=None):
        self._h = ctypes.c_void_p()
        check(lib().hydro_plan_create(ctypes.byref(prm), ctypes.byref(batch), _ptr(U_in),
                                      _ptr(U_out), _ptr(amax), _ptr(status), _stream(stream),
                                      ctypes.byref(self._h)))

    def set_dt(self, dt: float):
        check(lib().hydro_plan_set_dt(self._h, float(dt)))

    def launch(self, stream=None):
        check(lib().hydro_plan_launch(self._h, _stream(stream)))

    def close(self):
        if self._h:
            lib().hydro_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- device-resident time integration ----------------------------------------

def box_ghost_map(nx: int, ny: int, nz: int, periodic=(True, True, True)):
    """Ghost map (src, mode), int32 [n*27] each, of an nx x ny x nz box of
    subgrids numbered s = (kz*ny + ky)*nx + kx.  Along an axis that is not
    periodic, directions that leave the box are zero-gradient (outflow)."""
    n = nx * ny * nz
    src = np.zeros((n, 27), dtype=np.int32)
    mode = np.zeros((n, 27), dtype=np.int32)
    dims = (nx, ny, nz)
    for s in range(n):
        kx, ky, kz = s % nx, (s // nx) % ny, s // (nx * ny)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    slot = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)
                    pos, m = [], 0
                    for a, (k, d) in enumerate(((kx, dx), (ky, dy), (kz, dz))):
                        t = k + d
                        if 0 <= t < dims[a]:
                            pos.append(t)
                        elif periodic[a]:
                            pos.append(t % dims[a])
                        else:
                            pos.append(k)
                            m |= 1 << a
                    src[s, slot] = (pos[2] * ny + pos[1]) * nx + pos[0]
                    mode[s, slot] = m
    return src.reshape(-1), mode.reshape(-1)


class DeviceGhostMap:
    def __init__(self, src, mode):
        import torch
        self.src = torch.as_tensor(np.asarray(src, dtype=np.int32)).cuda()
        self.mode = torch.as_tensor(np.asarray(mode, dtype=np.int32)).cuda()
        self.struct = GhostMap(self.src.data_ptr(), self.mode.data_ptr())


def fill_ghosts(batch: Batch, gmap: DeviceGhostMap, U, status=None, stream=None, n: int = 8):
    check(lib(n).hydro_fill_ghosts(ctypes.byref(batch), ctypes.byref(gmap.struct), _ptr(U),
                                  _ptr(status), _stream(stream)))


def step_gather(prm: Params, batch: Batch, gmap: DeviceGhostMap, U_in, U_out, amax, status=None,
                stream=None):
    """Fused step reading ghost cells through the ghost map (no fill pass)."""
    check(lib().hydro_step_gather(ctypes.byref(prm), ctypes.byref(batch), ctypes.byref(gmap.struct),
                                  _ptr(U_in), _ptr(U_out), _ptr(amax), _ptr(status),
                                  _stream(stream)))


def rate(prm: Params, batch: Batch, U_in, R, amax, status=None, stream=None):
    check(lib().hydro_rate(ctypes.byref(prm), ctypes.byref(batch), _ptr(U_in), _ptr(R),
                           _ptr(amax), _ptr(status), _stream(stream)))


def cfl_dt(batch: Batch, amax, cfl, t_end, clock, stream=None, n: int = 8):
    check(lib(n).hydro_cfl_dt(ctypes.byref(batch), _ptr(amax), float(cfl), float(t_end),
                             _ptr(clock), _stream(stream)))


def rk_stage(prm: Params, batch: Batch, U_in, U_out, U0, a, b, clock, amax, status=None,
             stream=None):
    """Fused stage: U_out = a U0 + b (U_in + dt L(U_in)), dt = clock[1] (device)."""
    check(lib().hydro_rk_stage(ctypes.byref(prm), ctypes.byref(batch), _ptr(U_in), _ptr(U_out),
                               _ptr(U0), float(a), float(b), _ptr(clock), _ptr(amax),
                               _ptr(status), _stream(stream)))


def rk_update(batch: Batch, a, U0, b, Uk, R, clock, U_out, stream=None, n: int = 8):
    check(lib(n).hydro_rk_update(ctypes.byref(batch), float(a), _ptr(U0), float(b), _ptr(Uk),
                                _ptr(R), _ptr(clock), _ptr(U_out), _stream(stream)))


class RK3:
    """SSP-RK3 steps with device ghost fill and device CFL, one hipGraph per
    step.  Owns the work buffers, amax, status and the clock {t, dt}."""

    def __init__(self, prm: Params, db: "DeviceBatch", gmap: DeviceGhostMap, U, cfl=0.4,
                 t_end=float("inf"), stream=None):
        import torch
        self.db, self.gmap, self.U = db, gmap, U
        self.U1 = torch.zeros_like(U)
        self.U2 = torch.zeros_like(U)
        self.R = torch.zeros_like(U)
        self.amax = torch.zeros(db.n_sub, dtype=torch.float64, device=U.device)
        self.status = torch.zeros(db.n_sub, dtype=torch.int32, device=U.device)
        self.clock = torch.zeros(3, dtype=torch.float64, device=U.device)
        self._h = ctypes.c_void_p()
        check(lib().hydro_rk3_create(ctypes.byref(prm), ctypes.byref(db.struct),
                                     ctypes.byref(gmap.struct), _ptr(U), _ptr(self.U1),
                                     _ptr(self.U2), _ptr(self.R), _ptr(self.amax),
                                     _ptr(self.status), _ptr(self.clock), float(cfl),
                                     float(t_end), _stream(stream), ctypes.byref(self._h)))

    def launch(self, n_steps=1, stream=None):
        check(lib().hydro_rk3_launch(self._h, int(n_steps), _stream(stream)))

    def run_to_end(self, chunk=16, max_launches=1_000_000, stream=None):
        """Replay until a step finds the clock at t_end (checked every `chunk`
        replays); returns the number of steps that advanced time."""
        import torch
        launched = 0
        while launched < max_launches:
            self.launch(chunk, stream)
            launched += chunk
            torch.cuda.synchronize()
            if self.clock[1].item() == 0.0:
                break
        return int(self.clock[2].item())

    def close(self):
        if self._h:
            lib().hydro_rk3_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tau_resync(prm: Params, batch: Batch, U, stream=None, n: int = 8):
    """Entropy tracer reset to e_i^(1/gamma) where e_i >= de_switch * E (in place)."""
    check(lib(n).hydro_tau_resync(ctypes.byref(prm), ctypes.byref(batch), _ptr(U),
                                 _stream(stream)))
