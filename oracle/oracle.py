"""ctypes wrapper of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY.  Accepts the plain workload description objects
(grid / species / particles with the attribute names used by the seeded
input module) by duck typing; it imports nothing from the HIP package.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_LIB = os.path.join(HERE, "liboracle.so")

FROZEN_FIELDS = 1
NO_DEPOSIT = 2
CHARGE_CHECK = 4
MULTI_SHELL = 2  # species kind: nucleus + bound clouds with one bond each


class _Config(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32), ("pol", C.c_int32), ("pad", C.c_int32),
        ("max_probe_steps", C.c_int32),
        ("n", C.c_int64 * 3), ("dx", C.c_double * 3), ("dt", C.c_double),
        ("bc_lo", C.c_int32 * 3), ("bc_hi", C.c_int32 * 3),
        ("flags", C.c_uint32), ("reserved", C.c_uint32),
        ("a0", C.c_double), ("omega", C.c_double), ("t_env", C.c_double),
        ("waist", C.c_double), ("yc", C.c_double), ("zc", C.c_double),
        ("phase", C.c_double), ("t_delay", C.c_double), ("angle", C.c_double),
        ("n_env", C.c_int32), ("reserved2", C.c_int32), ("env", C.c_double * 64),
    ]


class _Diag(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("time", C.c_double), ("field_energy", C.c_double),
        ("kinetic_energy", C.c_double), ("momentum", C.c_double * 3),
        ("div_l2", C.c_double), ("div_max", C.c_double), ("rho_l2", C.c_double),
        ("n_particles", C.c_int64), ("error_word", C.c_uint32), ("reserved", C.c_uint32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(ORACLE_LIB):
        from .build import build
        build()
    lib = C.CDLL(ORACLE_LIB)
    P = C.c_void_p
    D = C.POINTER(C.c_double)
    lib.or_create.restype = P
    lib.or_create.argtypes = [C.POINTER(_Config)]
    lib.or_destroy.argtypes = [P]
    lib.or_add_species.restype = C.c_int
    lib.or_add_species.argtypes = [P, C.c_int] + [C.c_double] * 10 + [C.c_int64]
    lib.or_add_multishell.restype = C.c_int
    lib.or_add_multishell.argtypes = ([P, C.c_double, C.c_double, C.c_int, D, D, D, D] +
                                      [C.c_double] * 3 + [C.c_int64])
    lib.or_load_particles.restype = C.c_int
    lib.or_load_particles.argtypes = [P, C.c_int, C.c_int64, D, D, D, D, D, D]
    lib.or_load_fields.argtypes = [P, D, D]
    lib.or_step.argtypes = [P, C.c_int]
    lib.or_step.restype = C.c_int
    lib.or_diagnostics.argtypes = [P, C.POINTER(_Diag)]
    lib.or_read_fields.argtypes = [P, D, D, D]
    lib.or_read_particles.argtypes = [P, C.c_int, C.POINTER(C.c_int32), D, D, D, D]
    lib.or_count.restype = C.c_int64
    lib.or_count.argtypes = [P, C.c_int]
    lib.or_rho.argtypes = [P, D]
    lib.or_gather.argtypes = [P, C.POINTER(C.c_int32), D, D, D]
    lib.or_set_probes.argtypes = [P, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
    lib.or_set_probes.restype = C.c_int
    lib.or_read_probes.argtypes = [P, D, C.POINTER(C.c_int64)]
    lib.or_split_momentum.argtypes = [C.c_double] * 4 + [D, D, D]
    lib.or_ac_from_omega.restype = C.c_double
    lib.or_ac_from_omega.argtypes = [C.c_double] * 6
    _lib = lib
    return lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def split_momentum(q1, m1, q2, m2, uc):
    lib = _load()
    uc = _f64(uc, (3,))
    u1 = np.zeros(3)
    u2 = np.zeros(3)
    lib.or_split_momentum(q1, m1, q2, m2, _dp(uc), _dp(u1), _dp(u2))
    return u1, u2


def ac_from_omega(q1, m1, q2, m2, omega_c, re_norm):
    return _load().or_ac_from_omega(q1, m1, q2, m2, omega_c, re_norm)


class Oracle:
    """One oracle simulation.  `grid` carries ndim, n, dx, dt, bc_lo, bc_hi,
    pad, laser (a0, omega, t_env, waist, yc, zc, phase, t_delay, pol) and
    re_norm."""

    def __init__(self, grid, flags: int = 0, max_probe_steps: int = 0):
        lib = _load()
        self.lib = lib
        cfg = _Config()
        cfg.ndim = grid.ndim
        las = grid.laser
        cfg.pol = int(las.pol)
        cfg.pad = int(grid.pad)
        cfg.max_probe_steps = int(max_probe_steps)
        for d in range(3):
            cfg.n[d] = int(grid.n[d]) if d < grid.ndim else 1
            cfg.dx[d] = float(grid.dx[d]) if d < grid.ndim else 1.0
            cfg.bc_lo[d] = int(grid.bc_lo[d])
            cfg.bc_hi[d] = int(grid.bc_hi[d])
        cfg.dt = float(grid.dt)
        cfg.flags = int(flags)
        cfg.a0, cfg.omega, cfg.t_env = las.a0, las.omega, las.t_env
        cfg.waist, cfg.yc, cfg.zc = las.waist, las.yc, las.zc
        cfg.phase, cfg.t_delay = las.phase, las.t_delay
        cfg.angle = getattr(las, "angle", 0.0)
        env = tuple(getattr(las, "env", ()) or ())
        if len(env) > 64:
            raise ValueError("oracle: at most 64 envelope coefficients")
        cfg.n_env = len(env)
        for k, v in enumerate(env):
            cfg.env[k] = float(v)
        self.cfg = cfg
        self.grid = grid
        self.ndim = grid.ndim
        self.shape = tuple(int(grid.n[d]) if d < grid.ndim else 1 for d in range(3))
        self.ncell = int(np.prod(self.shape))
        self.ctx = lib.or_create(C.byref(cfg))
        if not self.ctx:
            raise ValueError("oracle: invalid grid")
        self.species = []

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.or_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- setup
    def add_species(self, sp, capacity: int) -> int:
        if int(sp.kind) == MULTI_SHELL:
            return self._add_multishell(sp, capacity)
        # a_c = 0: each ion's a_c from its own omega_c (derived in the C oracle)
        a_c = sp.a_c if sp.a_c is not None else math.inf
        sid = self.lib.or_add_species(self.ctx, int(sp.kind), sp.q1, sp.m1, sp.q2, sp.m2,
                                      sp.weight, sp.omega_c, a_c, sp.nu, sp.nu_per_omega,
                                      float(self.grid.re_norm), int(capacity))
        if sid < 0:
            raise ValueError("oracle: add_species failed (omega_c <= 0, a_c < 0, or a "
                             "derived a_c without re_norm > 0)")
        self.species.append(sp)
        return sid

    def _add_multishell(self, sp, capacity: int) -> int:
        sh = np.asarray(sp.shells, dtype=np.float64).reshape(-1, 4)
        qk, mk, wk, ak = (np.ascontiguousarray(sh[:, j]) for j in range(4))
        sid = self.lib.or_add_multishell(self.ctx, sp.q1, sp.m1, int(sh.shape[0]), _dp(qk),
                                         _dp(mk), _dp(wk), _dp(ak), sp.weight, sp.nu,
                                         float(self.grid.re_norm), int(capacity))
        if sid < 0:
            raise ValueError("oracle: add_multishell failed (1..4 shells, m > 0, q != 0, "
                             "omega_c > 0, a_c >= 0; a derived a_c needs re_norm > 0)")
        self.species.append(sp)
        return sid

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
        rc = self.lib.or_load_particles(self.ctx, sid, n, _dp(x), _dp(delta), _dp(u1), _dp(u2),
                                        _dp(wc), _dp(w))
        if rc != 0:
            raise ValueError(f"oracle: load_particles failed ({rc})")

    @classmethod
    def from_workload(cls, wl, flags: int = 0, max_probe_steps: int = 0):
        o = cls(wl.grid, flags=flags, max_probe_steps=max_probe_steps)
        for sp, parts in wl.species:
            sid = o.add_species(sp, parts.n)
            o.load_particles(sid, parts)
        if wl.probes and max_probe_steps > 0:
            o.set_probes(wl.probes)
        return o

    def load_fields(self, E, B):
        E = _f64(E, (3, self.ncell))
        B = _f64(B, (3, self.ncell))
        self.lib.or_load_fields(self.ctx, _dp(E), _dp(B))

    def set_probes(self, probes):
        comp = np.array([p[0] for p in probes], dtype=np.int32)
        idx = np.array([list(p[1]) for p in probes], dtype=np.int64).reshape(-1, 3)
        rc = self.lib.or_set_probes(self.ctx, len(probes),
                                    comp.ctypes.data_as(C.POINTER(C.c_int32)),
                                    idx.ctypes.data_as(C.POINTER(C.c_int64)))
        if rc != 0:
            raise ValueError("oracle: bad probes")
        self.nprobe = len(probes)

    # ----------------------------------------------------------------- run
    def step(self, n: int = 1):
        rc = self.lib.or_step(self.ctx, int(n))
        if rc != 0:
            raise RuntimeError("oracle: step failed")

    def diagnostics(self) -> dict:
        d = _Diag()
        self.lib.or_diagnostics(self.ctx, C.byref(d))
        return {
            "step": d.step, "time": d.time, "field_energy": d.field_energy,
            "kinetic_energy": d.kinetic_energy, "momentum": list(d.momentum),
            "div_l2": d.div_l2, "div_max": d.div_max, "rho_l2": d.rho_l2,
            "n_particles": d.n_particles, "error_word": d.error_word,
        }

    def fields(self):
        E = np.zeros((3, self.ncell))
        B = np.zeros((3, self.ncell))
        J = np.zeros((3, self.ncell))
        self.lib.or_read_fields(self.ctx, _dp(E), _dp(B), _dp(J))
        return E, B, J

    def particles(self, sid: int) -> dict:
        n = self.lib.or_count(self.ctx, sid)
        K = self._nshell(sid)
        cell = np.zeros((n, 3), dtype=np.int32)
        off = np.zeros((n, 3))
        delta = np.zeros((n, 3 * K))
        u1 = np.zeros((n, 3))
        u2 = np.zeros((n, 3 * K))
        self.lib.or_read_particles(self.ctx, sid, cell.ctypes.data_as(C.POINTER(C.c_int32)),
                                   _dp(off), _dp(delta), _dp(u1), _dp(u2))
        nd = self.ndim
        return {"cell": cell[:, :nd].copy(), "off": off[:, :nd].copy(), "delta": delta,
                "u1": u1, "u2": u2}

    def rho(self):
        r = np.zeros(self.ncell)
        self.lib.or_rho(self.ctx, _dp(r))
        return r

    def gather(self, cell, off):
        cl = np.zeros(3, dtype=np.int32)
        of = np.zeros(3)
        cl[: self.ndim] = cell
        of[: self.ndim] = off
        E = np.zeros(3)
        B = np.zeros(3)
        self.lib.or_gather(self.ctx, cl.ctypes.data_as(C.POINTER(C.c_int32)), _dp(of),
                           _dp(E), _dp(B))
        return E, B

    def probes(self):
        n = C.c_int64(0)
        self.lib.or_read_probes(self.ctx, None, C.byref(n))
        out = np.zeros((self.nprobe, n.value))
        self.lib.or_read_probes(self.ctx, _dp(out), C.byref(n))
        return out
