"""ctypes binding of libpic (include/pic.h): argument marshalling only.

Every step of the particle cycle and the field update runs in the HIP
library; this module only converts arguments, supplies device memory from
PyTorch's caching allocator and passes PyTorch's current HIP stream.  It
raises if the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_ENOMEM, PIC_EHIP, PIC_ESTATE, PIC_ERANGE, PIC_ENAN = 0, -1, -2, -3, -4, -5, -6
FROZEN_FIELDS, NO_DEPOSIT, CHARGE_CHECK, TRACK_IDS, TIMING, GLOBAL_KERNEL = 1, 2, 4, 8, 16, 32
SEPARATE_SPECIES = 64
TIMING_ADJOINT = 65536  # pic_timing tag offset of the adjoint particle kernel
POINT, TWO_BODY, MULTI_SHELL = 0, 1, 2  # species kinds
ERR_NAN, ERR_RANGE = 1, 2

_NAMES = {PIC_EINVAL: "PIC_EINVAL", PIC_ENOMEM: "PIC_ENOMEM", PIC_EHIP: "PIC_EHIP",
          PIC_ESTATE: "PIC_ESTATE", PIC_ERANGE: "PIC_ERANGE", PIC_ENAN: "PIC_ENAN"}


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class PicLaser(C.Structure):
    _fields_ = [("a0", C.c_double), ("omega", C.c_double), ("t_env", C.c_double),
                ("waist", C.c_double), ("yc", C.c_double), ("zc", C.c_double),
                ("phase", C.c_double), ("t_delay", C.c_double),
                ("pol", C.c_int32), ("reserved", C.c_int32), ("angle", C.c_double),
                ("n_env", C.c_int32), ("reserved2", C.c_int32), ("env", C.c_double * 64)]


class PicConfig(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("precision", C.c_int32), ("pad", C.c_int32),
                ("max_probe_steps", C.c_int32), ("n", C.c_int64 * 3), ("dx", C.c_double * 3),
                ("dt", C.c_double), ("bc_lo", C.c_int32 * 3), ("bc_hi", C.c_int32 * 3),
                ("tile", C.c_int32 * 3), ("sort_every", C.c_int32), ("flags", C.c_uint32),
                ("reserved", C.c_int32), ("re_norm", C.c_double), ("laser", PicLaser)]


class PicSpeciesDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("q1", C.c_double),
                ("m1", C.c_double), ("q2", C.c_double), ("m2", C.c_double),
                ("weight", C.c_double), ("omega_c", C.c_double), ("a_c", C.c_double),
                ("nu", C.c_double), ("nu_per_omega", C.c_double), ("capacity", C.c_int64)]


class PicDiag(C.Structure):
    _fields_ = [("step", C.c_int64), ("time", C.c_double), ("field_energy", C.c_double),
                ("kinetic_energy", C.c_double), ("momentum", C.c_double * 3),
                ("div_l2", C.c_double), ("div_max", C.c_double), ("rho_l2", C.c_double),
                ("n_particles", C.c_int64), ("error_word", C.c_uint32), ("reserved", C.c_uint32),
                ("n_outside_tile", C.c_int64), ("n_far", C.c_int64)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class PicAllocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


_lib = None

# (name, restype, argtypes) of every entry point in include/pic.h
_P, _D = C.c_void_p, C.POINTER(C.c_double)
class PicGrad(C.Structure):
    _fields_ = [("d_omega_c", _D), ("d_nu", _D), ("d_env", _D), ("d_E", _D), ("d_B", _D)]


SIGNATURES = [
    ("pic_create", C.c_int, [C.POINTER(PicConfig), C.POINTER(PicAllocator), _P, C.POINTER(_P)]),
    ("pic_add_species", C.c_int, [_P, C.POINTER(PicSpeciesDesc), C.POINTER(C.c_int32)]),
    ("pic_add_multishell", C.c_int, [_P, C.POINTER(PicSpeciesDesc), C.c_int32, _D, _D, _D, _D,
                                     C.POINTER(C.c_int32)]),
    ("pic_load_particles", C.c_int, [_P, C.c_int32, C.c_int64, _D, _D, _D, _D, _D, _D]),
    ("pic_load_particles_device", C.c_int, [_P, C.c_int32, C.c_int64, _P, _P, _P, _P, _P, _P]),
    ("pic_load_fields", C.c_int, [_P, _D, _D]),
    ("pic_step", C.c_int, [_P, C.c_int32]),
    ("pic_diagnostics", C.c_int, [_P, C.POINTER(PicDiag)]),
    ("pic_read_fields", C.c_int, [_P, _D, _D, _D]),
    ("pic_count", C.c_int, [_P, C.c_int32, C.POINTER(C.c_int64)]),
    ("pic_read_particles", C.c_int, [_P, C.c_int32, C.POINTER(C.c_int32), _D, _D, _D, _D,
                                     C.POINTER(C.c_int64)]),
    ("pic_read_particles_range", C.c_int, [_P, C.c_int32, C.c_int64, C.c_int64,
                                           C.POINTER(C.c_int32), _D, _D, _D, _D, _D, _D,
                                           C.POINTER(C.c_int64)]),
    ("pic_rho", C.c_int, [_P, _D]),
    ("pic_rho_static", C.c_int, [_P, _D]),
    ("pic_set_probes", C.c_int, [_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    ("pic_read_probes", C.c_int, [_P, _D, C.POINTER(C.c_int64)]),
    ("pic_timing", C.c_int, [_P, C.c_int32, _D, C.POINTER(C.c_int64), C.c_int32]),
    ("pic_grad_forward", C.c_int, [_P, C.c_int32, C.c_int32]),
    ("pic_grad_backward", C.c_int, [_P, _D, C.POINTER(PicGrad)]),
    ("pic_read_grad_particles", C.c_int, [_P, C.c_int32, _D, _D, _D, _D]),
    ("pic_save_state", C.c_int, [_P, _P, C.POINTER(C.c_size_t)]),
    ("pic_load_state", C.c_int, [_P, _P, C.c_size_t]),
    ("pic_last_error", C.c_char_p, [_P]),
    ("pic_destroy", None, [_P]),
    ("pic_version", C.c_char_p, []),
]


def load_library(path: str = LIB_PATH):
    """Load libpic.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpic.so not found at {path}; build it with __graft_entry__.build()")
    lib = C.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a.reshape(shape) if shape is not None else a


class TorchDeviceMemory:
    """Device allocator backed by PyTorch tensors (the caching allocator)."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device
        self.live = {}

        def _alloc(nbytes, user):
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            except Exception:
                return None
            p = t.data_ptr()
            self.live[p] = t
            return p

        def _free(ptr, user):
            self.live.pop(int(ptr) if ptr else 0, None)

        self._alloc_cb = ALLOC_FN(_alloc)
        self._free_cb = FREE_FN(_free)
        self.struct = PicAllocator(self._alloc_cb, self._free_cb, None)

    @property
    def bytes(self):
        return sum(t.numel() for t in self.live.values())


class Simulation:
    """One libpic context on the current HIP device and stream."""

    def __init__(self, grid, precision: int = 64, flags: int = 0, tile=None, sort_every: int = 0,
                 max_probe_steps: int = 0, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libpic needs a HIP device (torch.cuda.is_available() is False)")
        self.lib = load_library()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.mem = TorchDeviceMemory(self.device)
        cfg = PicConfig()
        cfg.ndim = grid.ndim
        cfg.precision = int(precision)
        cfg.pad = int(grid.pad)
        cfg.max_probe_steps = int(max_probe_steps)
        for d in range(3):
            cfg.n[d] = int(grid.n[d]) if d < grid.ndim else 1
            cfg.dx[d] = float(grid.dx[d]) if d < grid.ndim else 1.0
            cfg.bc_lo[d] = int(grid.bc_lo[d])
            cfg.bc_hi[d] = int(grid.bc_hi[d])
            cfg.tile[d] = int(tile[d]) if tile is not None and d < len(tile) else 0
        cfg.dt = float(grid.dt)
        cfg.sort_every = int(sort_every)
        cfg.flags = int(flags)
        cfg.re_norm = float(grid.re_norm)
        las = grid.laser
        cfg.laser = PicLaser(las.a0, las.omega, las.t_env, las.waist, las.yc, las.zc, las.phase,
                             las.t_delay, int(las.pol), 0, float(getattr(las, "angle", 0.0)))
        env = tuple(getattr(las, "env", ()) or ())
        if len(env) > 64:
            raise ValueError("at most 64 envelope coefficients")
        cfg.laser.n_env = len(env)
        for k, v in enumerate(env):
            cfg.laser.env[k] = float(v)
        self.cfg = cfg
        self.grid = grid
        self.ndim = grid.ndim
        self.precision = precision
        self.shape = tuple(int(grid.n[d]) if d < grid.ndim else 1 for d in range(3))
        self.ncell = int(np.prod(self.shape))
        ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.pic_create(C.byref(cfg), C.byref(self.mem.struct),
                                     C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if rc != PIC_OK:
            raise PicError(rc, self.lib.pic_last_error(None).decode())
        self.ctx = ctx
        self.nprobe = 0
        self.species = []
        self._grad_steps = 0  # steps of the last completed grad_forward

    def _check(self, rc):
        if rc != PIC_OK:
            raise PicError(rc, self.lib.pic_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.pic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- setup
    def add_species(self, sp, capacity: int) -> int:
        if int(sp.kind) == MULTI_SHELL:
            sh = np.asarray(sp.shells, dtype=np.float64).reshape(-1, 4)
            cols = [np.ascontiguousarray(sh[:, j]) for j in range(4)]
            d = PicSpeciesDesc(MULTI_SHELL, 0, sp.q1, sp.m1, 0.0, 0.0, sp.weight, 0.0, 0.0, sp.nu,
                               0.0, int(capacity))
            sid = C.c_int32()
            self._check(self.lib.pic_add_multishell(self.ctx, C.byref(d), int(sh.shape[0]),
                                                    *[_dp(v) for v in cols], C.byref(sid)))
            self.species.append(sp)
            return sid.value
        d = PicSpeciesDesc(int(sp.kind), 0, sp.q1, sp.m1, sp.q2, sp.m2, sp.weight, sp.omega_c,
                           sp.a_c if sp.a_c is not None else math.inf, sp.nu, sp.nu_per_omega,
                           int(capacity))
        sid = C.c_int32()
        self._check(self.lib.pic_add_species(self.ctx, C.byref(d), C.byref(sid)))
        self.species.append(sp)
        return sid.value

    def _nshell(self, sid: int) -> int:
        sp = self.species[sid]
        return len(sp.shells) if int(sp.kind) == MULTI_SHELL else 1

    def load_particles(self, sid: int, parts) -> None:
        n = parts.n
        K = self._nshell(sid)
        x = _f64(parts.x, (n, self.ndim))
        u1 = _f64(parts.u1, (n, 3))
        delta = _f64(parts.delta, (n, 3 * K))
        u2 = _f64(parts.u2, (n, 3 * K))
        wc = _f64(parts.omega_c, (n,))
        w = _f64(parts.weight, (n,))
        self._check(self.lib.pic_load_particles(self.ctx, sid, n, _dp(x), _dp(delta), _dp(u1),
                                                _dp(u2), _dp(wc), _dp(w)))

    def load_particles_device(self, sid: int, x, u1, delta=None, u2=None, omega_c=None,
                              weight=None) -> None:
        """Append particles from FP64 torch tensors on the context's device."""
        import torch
        n = int(x.shape[0])
        keep = []

        def ptr(t, cols):
            if t is None:
                return None
            t = t.to(device=self.device, dtype=torch.float64).contiguous()
            if t.numel() != n * cols:
                raise ValueError("particle array has the wrong size")
            keep.append(t)
            return C.c_void_p(t.data_ptr())

        K = self._nshell(sid)  # a multi-shell species: 3 K values of delta and u2
        args = [ptr(x, self.ndim), ptr(delta, 3 * K), ptr(u1, 3), ptr(u2, 3 * K),
                ptr(omega_c, 1), ptr(weight, 1)]
        torch.cuda.current_stream(self.device).synchronize()
        self._check(self.lib.pic_load_particles_device(self.ctx, sid, n, *args))
        del keep

    @classmethod
    def from_workload(cls, wl, precision: Optional[int] = None, flags: int = 0, **kw):
        sim = cls(wl.grid, precision=precision or wl.precision, flags=flags, **kw)
        for sp, parts in wl.species:
            sid = sim.add_species(sp, parts.n)
            sim.load_particles(sid, parts)
        if wl.probes and kw.get("max_probe_steps", 0) > 0:
            sim.set_probes(wl.probes)
        return sim

    def load_fields(self, E, B):
        E = _f64(E, (3, self.ncell))
        B = _f64(B, (3, self.ncell))
        self._check(self.lib.pic_load_fields(self.ctx, _dp(E), _dp(B)))

    def set_probes(self, probes):
        comp = np.array([p[0] for p in probes], dtype=np.int32)
        idx = np.array([list(p[1]) for p in probes], dtype=np.int64).reshape(-1, 3)
        self._check(self.lib.pic_set_probes(self.ctx, len(probes),
                                            comp.ctypes.data_as(C.POINTER(C.c_int32)),
                                            idx.ctypes.data_as(C.POINTER(C.c_int64))))
        self.nprobe = len(probes)

    # ------------------------------------------------------------------ run
    def step(self, n: int = 1):
        self._check(self.lib.pic_step(self.ctx, int(n)))

    def diagnostics(self, check: bool = True) -> dict:
        d = PicDiag()
        rc = self.lib.pic_diagnostics(self.ctx, C.byref(d))
        if check:
            self._check(rc)
        return {"step": d.step, "time": d.time, "field_energy": d.field_energy,
                "kinetic_energy": d.kinetic_energy, "momentum": list(d.momentum),
                "div_l2": d.div_l2, "div_max": d.div_max, "rho_l2": d.rho_l2,
                "n_particles": d.n_particles, "error_word": d.error_word,
                "n_outside_tile": d.n_outside_tile, "n_far": d.n_far, "status": rc}

    def fields(self):
        E = np.zeros((3, self.ncell))
        B = np.zeros((3, self.ncell))
        J = np.zeros((3, self.ncell))
        self._check(self.lib.pic_read_fields(self.ctx, _dp(E), _dp(B), _dp(J)))
        return E, B, J

    def fields_E(self):
        """E only (3 x ncell), for grids where E, B and J at once would not fit
        the host."""
        E = np.zeros((3, self.ncell))
        self._check(self.lib.pic_read_fields(self.ctx, _dp(E), None, None))
        return E

    def count(self, sid: int) -> int:
        n = C.c_int64()
        self._check(self.lib.pic_count(self.ctx, sid, C.byref(n)))
        return n.value

    def particles(self, sid: int, ids: bool = False) -> dict:
        n = self.count(sid)
        K = self._nshell(sid)
        cell = np.zeros((n, 3), dtype=np.int32)
        off = np.zeros((n, 3))
        delta = np.zeros((n, 3 * K))
        u1 = np.zeros((n, 3))
        u2 = np.zeros((n, 3 * K))
        idv = np.zeros(n, dtype=np.int64) if ids else None
        self._check(self.lib.pic_read_particles(
            self.ctx, sid, cell.ctypes.data_as(C.POINTER(C.c_int32)), _dp(off), _dp(delta),
            _dp(u1), _dp(u2), idv.ctypes.data_as(C.POINTER(C.c_int64)) if ids else None))
        nd = self.ndim
        out = {"cell": cell[:, :nd].copy(), "off": off[:, :nd].copy(), "delta": delta,
               "u1": u1, "u2": u2}
        if ids:
            out["id"] = idv
        return out

    def particles_range(self, sid: int, start: int, count: int, ids: bool = False) -> dict:
        """Particles start .. start+count-1 in storage order (see
        pic_read_particles_range), with omega_c and weight."""
        K = self._nshell(sid)
        cell = np.zeros((count, 3), dtype=np.int32)
        off, u1 = np.zeros((count, 3)), np.zeros((count, 3))
        delta, u2 = np.zeros((count, 3 * K)), np.zeros((count, 3 * K))
        wc, w = np.zeros(count), np.zeros(count)
        idv = np.zeros(count, dtype=np.int64) if ids else None
        self._check(self.lib.pic_read_particles_range(
            self.ctx, sid, int(start), int(count), cell.ctypes.data_as(C.POINTER(C.c_int32)),
            _dp(off), _dp(delta), _dp(u1), _dp(u2), _dp(wc), _dp(w),
            idv.ctypes.data_as(C.POINTER(C.c_int64)) if ids else None))
        nd = self.ndim
        out = {"cell": cell[:, :nd].copy(), "off": off[:, :nd].copy(), "delta": delta,
               "u1": u1, "u2": u2, "omega_c": wc, "weight": w}
        if ids:
            out["id"] = idv
        return out

    def rho(self):
        r = np.zeros(self.ncell)
        self._check(self.lib.pic_rho(self.ctx, _dp(r)))
        return r

    def rho_static(self):
        """pic_rho computed in the library's static device array (no
        allocation during the call)."""
        r = np.zeros(self.ncell)
        self._check(self.lib.pic_rho_static(self.ctx, _dp(r)))
        return r

    def probes(self):
        n = C.c_int64()
        self._check(self.lib.pic_read_probes(self.ctx, None, C.byref(n)))
        out = np.zeros((self.nprobe, n.value))
        self._check(self.lib.pic_read_probes(self.ctx, _dp(out), C.byref(n)))
        return out

    # ------------------------------------------------------- gradient run
    def grad_forward(self, nsteps: int, checkpoint_every: int) -> None:
        """Advance nsteps as step() does (no tile sorts), recording the
        probes and keeping a checkpoint every `checkpoint_every` steps."""
        self._grad_steps = 0
        self._check(self.lib.pic_grad_forward(self.ctx, int(nsteps), int(checkpoint_every)))
        self._grad_steps = int(nsteps)

    def grad_backward(self, dprobe, fields: bool = False) -> dict:
        """Gradients from the cotangent of the probe values of the last
        grad_forward run (nprobe x nsteps): d_omega_c, d_nu per species,
        d_env per envelope coefficient, and (fields=True) d_E, d_B at the
        start of the run (3 x ncell each)."""
        ns = len(self.species)
        dp = None
        if self.nprobe:
            dp = _f64(dprobe)
            # the library reads nprobe x nsteps values of the last run (and
            # refuses with PIC_ESTATE when there is none)
            if self._grad_steps and dp.size != self.nprobe * self._grad_steps:
                raise ValueError(f"dprobe must hold {self.nprobe} x {self._grad_steps} values")
            if not self._grad_steps:
                dp = np.zeros(self.nprobe)
        out = {"d_omega_c": np.zeros(ns), "d_nu": np.zeros(ns),
               "d_env": np.zeros(max(int(self.cfg.laser.n_env), 0))}
        if fields:
            out["d_E"] = np.zeros((3, self.ncell))
            out["d_B"] = np.zeros((3, self.ncell))
        g = PicGrad(_dp(out["d_omega_c"]), _dp(out["d_nu"]),
                    _dp(out["d_env"]) if out["d_env"].size else None,
                    _dp(out.get("d_E")), _dp(out.get("d_B")))
        self._check(self.lib.pic_grad_backward(self.ctx, _dp(dp), C.byref(g)))
        return out

    def grad_particles(self, sid: int) -> dict:
        """dL/d(state at the start of the run) of one species, in the run's
        storage order (that of particles(sid) after grad_forward)."""
        n = self.count(sid)
        two = self.species[sid].kind == 1  # two-body
        out = {"x": np.zeros((n, self.ndim)), "u1": np.zeros((n, 3))}
        if two:
            out["delta"] = np.zeros((n, 3))
            out["u2"] = np.zeros((n, 3))
        self._check(self.lib.pic_read_grad_particles(self.ctx, int(sid), _dp(out["x"]),
                                                     _dp(out.get("delta")), _dp(out["u1"]),
                                                     _dp(out.get("u2"))))
        return out

    # ------------------------------------------------ checkpoint / restart
    def save_state(self) -> np.ndarray:
        """The context's state as a host byte array (pic_save_state)."""
        n = C.c_size_t(0)
        self._check(self.lib.pic_save_state(self.ctx, None, C.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        self._check(self.lib.pic_save_state(self.ctx, C.c_void_p(buf.ctypes.data), C.byref(n)))
        return buf[: n.value]

    def load_state(self, buf) -> None:
        """Replace the context's state by one saved from a context of the
        same configuration and species (pic_load_state)."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self.lib.pic_load_state(self.ctx, C.c_void_p(buf.ctypes.data),
                                            C.c_size_t(buf.size)))

    def timing(self, species: int = -1, reset: bool = True):
        """(total ms, dispatches) of the main particle kernel of one species
        (-1: all); the tiled kernel counts one dispatch per tile colour."""
        ms = C.c_double()
        nl = C.c_int64()
        self._check(self.lib.pic_timing(self.ctx, int(species), C.byref(ms), C.byref(nl),
                                        int(reset)))
        return ms.value, nl.value
