"""Parity at the full size of the benchmark (512 x 256 x 256 cells, 8 two-body
ions and 8 electrons per cell, 530 million macro-particles) in the launch
configuration bench.py times.  The oracle cannot advance the whole system,
so it advances sampled particles one by one: a full-grid oracle holding only
the sampled particles, with the same fields frozen and no deposit, must move
them exactly as the GPU moved them in its coupled step (the push of a
particle depends only on its own state and on the fields at its nodes).
The whole-system property checked at full size is charge continuity.  The
3D mixed-precision case (1024 x 1024 x 512 cells, 537 million ions) is
checked the same way, each sampled range on a window of the grid.  The 2D
Bragg case (4096^2 cells, 457 ions) is small enough in particles for the
oracle to advance the whole system at its full size.
"""
import math
import sys

import numpy as np
import pytest

from oracle import Oracle
from oracle.oracle import FROZEN_FIELDS as O_FROZEN, NO_DEPOSIT as O_NODEP
from paper_2208_08038_amd.inputs import Particles

pytestmark = pytest.mark.gpu

CELLS = (512, 256, 256)
PPC = 8
SAMPLE_RANGES = 16
SAMPLE_LEN = 128


@pytest.fixture(scope="module")
def pic():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2208_08038_amd import pic as P
    P.load_library()
    return P


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _smooth_fields(shape, dx, amp=0.05):
    """E, B (3, ncell) with x fastest: separable sines of a few wavelengths,
    a different phase and direction mix per component."""
    nx, ny, nz = shape
    i = np.arange(nx) * dx
    j = np.arange(ny) * dx
    k = np.arange(nz) * dx
    Lx, Ly, Lz = nx * dx, ny * dx, nz * dx
    out = []
    for c in range(6):
        fx = np.sin(2 * math.pi * (c + 1) * i / Lx + 0.3 * c)
        fy = np.cos(2 * math.pi * (1 + c % 3) * j / Ly + 0.7 * c)
        fz = np.cos(2 * math.pi * (1 + c % 2) * k / Lz + 1.1 * c)
        v = amp * (1.0 - 0.3 * (c >= 3)) * np.multiply.outer(np.multiply.outer(fz, fy), fx)
        out.append(v.reshape(-1))
    return np.stack(out[:3]), np.stack(out[3:])


def _check(ref, got, tol, what):
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(ref - got).max() / scale
    assert err < tol, f"{what}: relative error {err:.3e} (tolerance {tol:.0e})"
    return err


@pytest.mark.parametrize("precision", [32, 64])
def test_full_size_sampled_particles_and_continuity(pic, precision):
    import bench
    _say(f"case: full-size slab {CELLS} ppc={PPC} fp{precision}: load")
    sim, meta, sid_i, sid_e, _ = bench.ionised_slab_simulation(
        CELLS, PPC, precision, pic.TRACK_IDS | pic.CHARGE_CHECK)
    grid = meta.grid
    dx = grid.dx[0]
    E, B = _smooth_fields(CELLS, dx)
    if precision == 32:  # the oracle starts from the values the GPU holds
        E, B = E.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
    sim.load_fields(E, B)
    rng = np.random.default_rng(2208)
    before, starts = {}, {}
    for sid in (sid_i, sid_e):
        n = sim.count(sid)
        starts[sid] = np.sort(rng.integers(0, n - SAMPLE_LEN, SAMPLE_RANGES))
        before[sid] = [sim.particles_range(sid, s0, SAMPLE_LEN, ids=True) for s0 in starts[sid]]
    _say(f"case: full-size fp{precision}: one coupled step")
    sim.step(1)
    d = sim.diagnostics()
    assert d["error_word"] == 0 and d["status"] == 0
    # Charge continuity over the whole grid after the step.  Esirkepov's
    # deposit conserves charge exactly, so the residual is rounding: each
    # body moves the charge |q W| / (dV dt) per unit of shape change, and the
    # shape changes carry an error of order eps |x| (|x| < 2 cells).  A node
    # sees the bodies of 27 cells, so |residual| < 27 * 8 * eps * (gross
    # charge rate of one cell), and its RMS over the grid stays below eps
    # times that rate.  The slab is near neutral (79 - 78 per ion, ions
    # against electrons), so the net rate rho_l2 is far below the gross one.
    eps = 2.0 ** -24 if precision == 32 else 2.0 ** -53
    dv = dx ** 3
    gross = sum(PPC * sp.weight * (abs(sp.q1) + (abs(sp.q2) if sp.kind == 1 else 0.0))
                for sp, _ in meta.species) / (dv * grid.dt)
    ncell = CELLS[0] * CELLS[1] * CELLS[2]
    assert d["rho_l2"] > 0
    assert d["div_max"] < 27 * 8 * eps * gross, (d, gross)
    assert d["div_l2"] / math.sqrt(ncell) < eps * gross, (d, gross)
    after = {sid: [sim.particles_range(sid, s0, SAMPLE_LEN, ids=True) for s0 in starts[sid]]
             for sid in (sid_i, sid_e)}
    species = [meta.species[0][0], meta.species[1][0]]
    sim.close()
    del sim
    import torch
    torch.cuda.empty_cache()  # the next full-size case needs the memory

    _say(f"case: full-size fp{precision}: oracle on the sampled particles")
    o = Oracle(grid, flags=O_FROZEN | O_NODEP)
    cat = {}
    for sid, sp in zip((sid_i, sid_e), species):
        b = {k: np.concatenate([r[k] for r in before[sid]]) for k in before[sid][0]}
        a = {k: np.concatenate([r[k] for r in after[sid]]) for k in after[sid][0]}
        assert np.array_equal(a["id"], b["id"]), "a step without a sort kept the storage order"
        x = (b["cell"] + b["off"]) * dx
        two = sp.kind == 1
        parts = Particles(x=x, u1=b["u1"], delta=b["delta"] if two else None,
                          u2=b["u2"] if two else None, omega_c=b["omega_c"] if two else None)
        osid = o.add_species(sp, parts.n)
        o.load_particles(osid, parts)
        cat[osid] = (two, a)
    o.load_fields(E, B)
    o.step(1)
    tol = 2e-5 if precision == 32 else 1e-11
    for osid, (two, a) in cat.items():
        r = o.particles(osid)
        pos_err = np.abs((r["cell"] + r["off"]) - (a["cell"] + a["off"])).max()
        assert pos_err < (2e-6 if precision == 32 else 1e-11), f"position error {pos_err:.3e} cells"
        errs = {"position (cells)": pos_err, "u1": _check(r["u1"], a["u1"], tol, "u1")}
        if two:
            errs["u2"] = _check(r["u2"], a["u2"], tol, "u2")
            errs["delta"] = _check(r["delta"], a["delta"], tol, "delta")
        _say(f"fp{precision} {'ions' if two else 'electrons'} ({len(r['u1'])} sampled): " +
             ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    _say(f"fp{precision} continuity: div_max {d['div_max']:.3e} (bound "
         f"{27 * 8 * eps * gross:.3e}), rms {d['div_l2'] / math.sqrt(ncell):.3e} "
         f"(bound {eps * gross:.3e}), rho_l2 {d['rho_l2']:.3e}")
    o.close()


def _smooth_fields_2d(shape, dx, amp=0.05):
    """E, B (3, ncell) on a 2D grid, x fastest: separable sines of a few
    wavelengths per component."""
    nx, ny = shape
    i = np.arange(nx) * dx
    j = np.arange(ny) * dx
    Lx, Ly = nx * dx, ny * dx
    out = []
    for c in range(6):
        fx = np.sin(2 * math.pi * (c + 1) * i / Lx + 0.3 * c)
        fy = np.cos(2 * math.pi * (1 + c % 3) * j / Ly + 0.7 * c)
        out.append((amp * (1.0 - 0.3 * (c >= 3)) * np.multiply.outer(fy, fx)).reshape(-1))
    return np.stack(out[:3]), np.stack(out[3:])


@pytest.mark.parametrize("precision", [64, 32])
def test_full_size_bragg_case(pic, precision):
    """The 2D Bragg case at its full size (4096^2 cells, the gold lattice of
    the central 1024^2 cells, the x-min laser, Mur faces) in the launch
    configuration bench.py times: from smooth fields, 12 coupled steps of the
    whole system on the GPU and in the oracle (which starts from the state
    the GPU holds after its load): fields and every ion."""
    from paper_2208_08038_amd.inputs import bragg_2d
    _say(f"case: full-size bragg 4096^2 fp{precision}")
    steps = 12
    wl = bragg_2d(steps=steps, precision=precision)
    g = wl.grid
    dx = g.dx[0]
    E, B = _smooth_fields_2d(g.n[:2], dx)
    if precision == 32:
        E, B = E.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
    s = pic.Simulation.from_workload(wl, precision=precision, flags=pic.TRACK_IDS)
    s.load_fields(E, B)
    n = s.count(0)
    st = s.particles_range(0, 0, n, ids=True)
    order = np.argsort(st["id"])
    sp = wl.species[0][0]
    parts = Particles(x=(st["cell"][order] + st["off"][order]) * dx, u1=st["u1"][order],
                      delta=st["delta"][order], u2=st["u2"][order])
    o = Oracle(g)
    osid = o.add_species(sp, n)
    o.load_particles(osid, parts)
    o.load_fields(E, B)
    s.step(steps)
    assert s.diagnostics()["error_word"] == 0
    _say(f"case: full-size bragg fp{precision}: oracle, {steps} steps")
    o.step(steps)
    Eo, Bo, Jo = o.fields()
    Eg, Bg, Jg = s.fields()
    tol = 1e-12 if precision == 64 else 2e-5
    errs = {}
    for name, got, ref in (("E", Eg, Eo), ("B", Bg, Bo), ("J", Jg, Jo)):
        errs[name] = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
        assert errs[name] < tol, (name, errs[name])
    r = o.particles(osid)
    a = s.particles(0, ids=True)
    a = {k: v[np.argsort(a["id"])] for k, v in a.items()}
    pos_err = np.abs((r["cell"] + r["off"]) - (a["cell"] + a["off"])).max()
    assert pos_err < (2e-6 if precision == 32 else 1e-11), pos_err
    if precision == 64:
        assert np.array_equal(r["cell"], a["cell"])
    errs["u1"] = _check(r["u1"], a["u1"], tol, "u1")
    errs["u2"] = _check(r["u2"], a["u2"], tol, "u2")
    errs["delta"] = _check(r["delta"], a["delta"], tol, "delta")
    _say(f"fp{precision} bragg full size: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()) +
         f", positions {pos_err:.2e} cells")
    s.close()
    o.close()


MP_CELLS = (1024, 1024, 512)
MP_RANGES = 12


def _smooth_factors(shape, dx, amp=0.05):
    """Per component c of E, B: (scale, fx, fy, fz), the separable factors
    of _smooth_fields, so that a window of the grid takes exactly the values
    of the whole."""
    nx, ny, nz = shape
    i, j, k = np.arange(nx) * dx, np.arange(ny) * dx, np.arange(nz) * dx
    Lx, Ly, Lz = nx * dx, ny * dx, nz * dx
    return [(amp * (1.0 - 0.3 * (c >= 3)),
             np.sin(2 * math.pi * (c + 1) * i / Lx + 0.3 * c),
             np.cos(2 * math.pi * (1 + c % 3) * j / Ly + 0.7 * c),
             np.cos(2 * math.pi * (1 + c % 2) * k / Lz + 1.1 * c)) for c in range(6)]


def _fields_from(factors, lo, shape, f32):
    """E, B (3, ncell), x fastest, on the cells lo .. lo + shape."""
    n = shape[0] * shape[1] * shape[2]
    E, B = np.empty((3, n)), np.empty((3, n))
    for c, (a, fx, fy, fz) in enumerate(factors):
        v = a * np.multiply.outer(np.multiply.outer(fz[lo[2]:lo[2] + shape[2]],
                                                    fy[lo[1]:lo[1] + shape[1]]),
                                  fx[lo[0]:lo[0] + shape[0]])
        if f32:  # the values the FP32 run holds
            v = v.astype(np.float32).astype(np.float64)
        (E if c < 3 else B)[c % 3] = v.reshape(-1)
    return E, B


@pytest.mark.parametrize("precision", [32, 64])
def test_full_size_mixed_precision_case(pic, precision):
    """The 3D mixed-precision case at its full size (1024 x 1024 x 512 cells,
    536,870,912 two-body ions) in the launch configuration bench.py times:
    from smooth fields, one coupled step of the whole system; sampled ranges
    of ions against the oracle, each on a window of the grid around its
    particles with the same field values (frozen fields, no deposit: a
    particle's push depends only on the fields at its nodes), and the charge
    continuity of the whole grid."""
    import dataclasses

    import bench
    import torch
    _say(f"case: full-size mixed precision {MP_CELLS} fp{precision}: load")
    sim, sid, meta, total, wmax, _ = bench.mixed_precision_simulation(
        MP_CELLS, precision, pic.TRACK_IDS | pic.CHARGE_CHECK)
    grid, sp = meta.grid, meta.species[0][0]
    dx = grid.dx[0]
    factors = _smooth_factors(MP_CELLS, dx)
    E, B = _fields_from(factors, (0, 0, 0), MP_CELLS, precision == 32)
    sim.load_fields(E, B)
    del E, B
    rng = np.random.default_rng(4)
    ranges = []
    while len(ranges) < MP_RANGES:
        s0 = int(rng.integers(0, total - SAMPLE_LEN))
        b = sim.particles_range(sid, s0, SAMPLE_LEN, ids=True)
        lo = b["cell"].min(axis=0) - 4
        hi = b["cell"].max(axis=0) + 5
        if np.all(lo >= 0) and np.all(hi <= np.array(MP_CELLS)):  # away from the periodic seams
            ranges.append((s0, b, lo, hi))
    _say(f"case: full-size mixed precision fp{precision}: one coupled step")
    sim.step(1)
    d = sim.diagnostics()
    assert d["error_word"] == 0 and d["status"] == 0
    eps = 2.0 ** -24 if precision == 32 else 2.0 ** -53
    gross = 4 * wmax * (abs(sp.q1) + abs(sp.q2)) / (dx ** 3 * grid.dt)
    ncell = MP_CELLS[0] * MP_CELLS[1] * MP_CELLS[2]
    assert d["rho_l2"] > 0
    assert d["div_max"] < 27 * 8 * eps * gross, (d, gross)
    assert d["div_l2"] / math.sqrt(ncell) < eps * gross, (d, gross)
    after = [sim.particles_range(sid, s0, SAMPLE_LEN, ids=True) for s0, _, _, _ in ranges]
    sim.close()
    del sim
    torch.cuda.empty_cache()

    _say(f"case: full-size mixed precision fp{precision}: oracle windows")
    tol = 2e-5 if precision == 32 else 1e-11
    worst = {"position (cells)": 0.0, "u1": 0.0, "u2": 0.0, "delta": 0.0}
    P = (0, 0, 0)  # periodic window (its seams lie beyond every stencil of its particles)
    for (s0, b, lo, hi), a in zip(ranges, after):
        assert np.array_equal(a["id"], b["id"]), "a step without a sort kept the storage order"
        shape = tuple(int(v) for v in hi - lo)
        wg = dataclasses.replace(grid, n=shape, bc_lo=P, bc_hi=P)
        o = Oracle(wg, flags=O_FROZEN | O_NODEP)
        parts = Particles(x=(b["cell"] - lo + b["off"]) * dx, u1=b["u1"], delta=b["delta"],
                          u2=b["u2"], omega_c=b["omega_c"], weight=b["weight"])
        osid = o.add_species(sp, parts.n)
        o.load_particles(osid, parts)
        o.load_fields(*_fields_from(factors, tuple(int(v) for v in lo), shape, precision == 32))
        o.step(1)
        r = o.particles(osid)
        pos = np.abs((r["cell"] + r["off"]) - (a["cell"] - lo + a["off"])).max()
        assert pos < (2e-6 if precision == 32 else 1e-11), f"position error {pos:.3e} cells"
        worst["position (cells)"] = max(worst["position (cells)"], pos)
        for key in ("u1", "u2", "delta"):
            worst[key] = max(worst[key], _check(r[key], a[key], tol, key))
        o.close()
    _say(f"fp{precision} mixed precision full size ({MP_RANGES} x {SAMPLE_LEN} ions): " +
         ", ".join(f"{k} {v:.2e}" for k, v in worst.items()) +
         f"; continuity div_max {d['div_max']:.3e} (bound {27 * 8 * eps * gross:.3e})")


def test_full_size_gradient_run(pic):
    """The gradient run at the size bench.py measures (2D 2048 x 1024 cells,
    6,291,456 two-body ions, 1024 steps, checkpoints every 32): FP32 adjoint
    gradients of the transmitted-pulse loss with respect to omega_c, nu and
    one envelope coefficient against central differences (h = 1e-3
    relative) of the FP64 forward, within 1e-4."""
    import torch
    from paper_2208_08038_amd.inputs import adjoint_slab
    from paper_2208_08038_amd.objectives import transmitted_loss, transmitted_parts
    import _adjoint as A
    wl = adjoint_slab(2, (2048, 1024))
    ny, dt, dy = wl.grid.n[1], wl.grid.dt, wl.grid.dx[1]
    _say(f"case: full-size gradient run, {wl.species[0][1].n} ions, {wl.steps} steps: fp32 adjoint")
    sim = pic.Simulation.from_workload(wl, precision=32, max_probe_steps=wl.steps)
    sim.grad_forward(wl.steps, 32)
    series = torch.tensor(sim.probes(), requires_grad=True)
    e_ref = float(transmitted_parts(series.detach(), ny, dt, dy)[0])
    L = transmitted_loss(series, ny, dt, dy, e_ref=e_ref)
    (cot,) = torch.autograd.grad(L, series)
    g = sim.grad_backward(cot.numpy())
    assert sim.diagnostics()["error_word"] == 0
    sim.close()

    def loss(s):
        return float(transmitted_loss(s, ny, dt, dy, e_ref=e_ref))
    sp = wl.species[0][0]
    env = np.array(wl.grid.laser.env)
    k = 32

    def env_k(v):
        e = env.copy()
        e[k] = v
        return A.with_params(wl, env=e)
    for name, adj, make, x0 in (
            ("omega_c", g["d_omega_c"][0], lambda v: A.with_params(wl, omega_c=v), sp.omega_c),
            ("nu", g["d_nu"][0], lambda v: A.with_params(wl, nu=v), sp.nu),
            (f"env[{k}]", g["d_env"][k], env_k, env[k])):
        _say(f"case: full-size gradient run: fp64 central differences in {name}")
        fd = A.central_fd(lambda w: A.gpu_series(pic, w), loss, make, x0, 1e-3 * abs(x0))
        rel = abs(adj - fd) / abs(fd)
        _say(f"full size d/d{name}: fp32 adjoint {adj:.8e}, fp64 FD {fd:.8e}, rel {rel:.2e}")
        assert rel < 1e-4, name
