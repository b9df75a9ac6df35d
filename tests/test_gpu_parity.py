"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
identical seeded inputs.  Tolerances: integer state (cells, sort order)
bit-exact; FP64 fields within relative L2 1e-12; FP32 fields within 2e-5.
"""
import dataclasses
import math
import sys

import numpy as np
import pytest

from _parity import match_by_id, random_fields, random_workload, rel_l2, small_grid
from oracle import Oracle
from oracle.oracle import CHARGE_CHECK as O_CHARGE, FROZEN_FIELDS as O_FROZEN
from paper_2208_08038_amd.inputs import (LASER, OPEN, PERIODIC, POINT, TWO_BODY, Grid, Laser,
                                         Particles, Species, neutral_medium_1d)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2208_08038_amd import pic as P
    P.load_library()  # raises if libpic.so is missing
    return P


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _both(wl, P, precision, oflags=0, pflags=0, **kw):
    o = Oracle.from_workload(wl, flags=oflags)
    s = P.Simulation.from_workload(wl, precision=precision, flags=pflags | P.TRACK_IDS, **kw)
    return o, s


def _compare_particles(o, s, wl, tol, exact_cells=True):
    worst = 0.0
    for sid, (sp, parts) in enumerate(wl.species):
        ref = o.particles(sid)
        got = match_by_id(s.particles(sid, ids=True), s.particles(sid, ids=True)["id"])
        if exact_cells:
            assert np.array_equal(ref["cell"], got["cell"]), "cell indices differ"
        # compare absolute positions in cell units (robust to a face crossing)
        pr = ref["cell"] + ref["off"]
        pg = got["cell"] + got["off"]
        worst = max(worst, np.max(np.abs(pr - pg)) if pr.size else 0.0)
        keys = ["u1"] + (["u2", "delta"] if sp.kind == TWO_BODY else [])
        for k in keys:
            scale = max(np.abs(ref[k]).max(), 1e-300)
            err = np.abs(ref[k] - got[k]).max() / scale
            assert err < tol, f"{k}: relative error {err:.3e}"
    assert worst < tol * 10, f"position error {worst:.3e} cells"


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_one_step_frozen_fields_fp64(pic, ndim):
    """Gather + force + Boris + move + deposit of one step on random ions and
    electrons in a frozen random field: particles and J match the oracle."""
    _say(f"case: one step frozen fp64 ndim={ndim}")
    wl = random_workload(ndim, 37, 29, seed=10 + ndim)
    o, s = _both(wl, pic, 64, oflags=O_FROZEN, pflags=pic.FROZEN_FIELDS)
    rng = np.random.default_rng(ndim)
    E, B = random_fields(rng, o.ncell)
    o.load_fields(E, B)
    s.load_fields(E, B)
    o.step(1)
    s.step(1)
    assert s.diagnostics()["error_word"] == 0
    _compare_particles(o, s, wl, 1e-12)
    _, _, Jo = o.fields()
    _, _, Jg = s.fields()
    assert rel_l2(Jg, Jo) < 1e-12


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_one_step_tiny_brute_force(pic, ndim):
    """At most 8 particles, including ones next to cell faces and at rest."""
    _say(f"case: tiny brute force ndim={ndim}")
    wl = random_workload(ndim, 5, 3, seed=99 + ndim, shape=(9, 8, 7)[:ndim])
    sp, parts = wl.species[0]
    parts.x[0, 0] = 3.0 * wl.grid.dx[0]            # exactly on a face
    parts.x[1, 0] = (4.0 - 1e-13) * wl.grid.dx[0]  # just below a face
    parts.u1[2] = 0.0
    parts.u2[2] = 0.0
    o, s = _both(wl, pic, 64, oflags=O_FROZEN, pflags=pic.FROZEN_FIELDS)
    rng = np.random.default_rng(5)
    E, B = random_fields(rng, o.ncell)
    o.load_fields(E, B)
    s.load_fields(E, B)
    o.step(1)
    s.step(1)
    _compare_particles(o, s, wl, 1e-12)
    assert rel_l2(s.fields()[2], o.fields()[2]) < 1e-12


@pytest.mark.parametrize("ndim", [2, 3])
def test_coupled_periodic_fp64(pic, ndim):
    """20 self-consistent steps (particles + Yee) in a periodic box."""
    _say(f"case: coupled periodic fp64 ndim={ndim}")
    wl = random_workload(ndim, 300, 300, seed=20 + ndim)
    o, s = _both(wl, pic, 64, sort_every=3)
    o.step(20)
    s.step(20)
    assert o.diagnostics()["error_word"] == 0, "oracle run left the valid range"
    Eo, Bo, Jo = o.fields()
    Eg, Bg, Jg = s.fields()
    assert rel_l2(Eg, Eo) < 1e-12
    assert rel_l2(Bg, Bo) < 1e-12
    assert rel_l2(Jg, Jo) < 1e-12
    _compare_particles(o, s, wl, 1e-11)
    assert s.diagnostics()["error_word"] == 0


@pytest.mark.parametrize("ndim,shape,n,precision", [(2, (240, 192), 8, 64), (3, (64, 64, 48), 5, 64),
                                                    (3, (64, 64, 48), 5, 32)])
def test_sparse_tiles_coupled(pic, ndim, shape, n, precision):
    """A few particles in a large box (fewer than a quarter of the tiles of
    one colour): the tiled launches visit only the occupied tiles, listed
    again after every sort; 12 coupled steps with fast particles crossing
    tiles match the oracle."""
    _say(f"case: sparse tiles ndim={ndim} fp{precision}")
    wl = random_workload(ndim, n, n, seed=40 + ndim, shape=shape, vmax_ion=0.6, vmax_el=0.95)
    o, s = _both(wl, pic, precision)
    o.step(12)
    s.step(12)
    d = s.diagnostics()
    assert d["error_word"] == 0
    tol = 1e-12 if precision == 64 else 2e-5
    Eo, Bo, Jo = o.fields()
    Eg, Bg, Jg = s.fields()
    assert rel_l2(Eg, Eo) < tol
    assert rel_l2(Bg, Bo) < tol
    _compare_particles(o, s, wl, 1e-11 if precision == 64 else 1e-4, exact_cells=precision == 64)


def _relativistic(wl, seed):
    """Give every particle a random direction and gamma in [2, 8] (ion
    centres, both bodies kept at their loaded momentum difference) or
    [2, 20] (free electrons)."""
    rng = np.random.default_rng(seed)
    for sp, p in wl.species:
        n = p.u1.shape[0]
        d = rng.normal(size=(n, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        g = rng.uniform(2.0, 8.0 if sp.kind == TWO_BODY else 20.0, n)
        u = d * np.sqrt(g * g - 1.0)[:, None]
        if sp.kind == TWO_BODY:
            p.u2 = u + (p.u2 - p.u1)
        p.u1 = u


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_relativistic_coupled(pic, ndim):
    """15 self-consistent steps with every particle at gamma 2 - 20: FP64
    follows the oracle to round-off, FP32 fields within its tolerance."""
    _say(f"case: relativistic coupled ndim={ndim}")
    wl = random_workload(ndim, 300, 300, seed=60 + ndim, weight=0.001)
    _relativistic(wl, 70 + ndim)
    o, s = _both(wl, pic, 64, sort_every=3)
    o.step(15)
    s.step(15)
    assert o.diagnostics()["error_word"] == 0, "oracle run left the valid range"
    assert s.diagnostics()["error_word"] == 0
    Eo, Bo, Jo = o.fields()
    Eg, Bg, Jg = s.fields()
    assert rel_l2(Eg, Eo) < 1e-12 and rel_l2(Bg, Bo) < 1e-12 and rel_l2(Jg, Jo) < 1e-12
    _compare_particles(o, s, wl, 1e-11)
    s32 = pic.Simulation.from_workload(wl, precision=32)
    s32.step(15)
    assert s32.diagnostics()["error_word"] == 0
    Eg, Bg, _ = s32.fields()
    assert rel_l2(Eg, Eo) < 2e-5 and rel_l2(Bg, Bo) < 2e-5


@pytest.mark.parametrize("tile", [(8, 8, 8), (8, 8, 6), (6, 8, 8), (5, 5, 5), (16, 8, 6)])
def test_tile_shapes(pic, tile):
    """Other tile shapes (partial tiles at the upper faces, two workgroups
    per CU where the LDS footprint allows): FP64 follows the oracle,
    FP32 within its tolerance."""
    _say(f"case: tile shape {tile}")
    wl = random_workload(3, 300, 300, seed=24)
    o, s = _both(wl, pic, 64, sort_every=3, tile=tile)
    o.step(10)
    s.step(10)
    assert o.diagnostics()["error_word"] == 0, "oracle run left the valid range"
    Eo, Bo, Jo = o.fields()
    Eg, Bg, Jg = s.fields()
    assert rel_l2(Eg, Eo) < 1e-12 and rel_l2(Bg, Bo) < 1e-12 and rel_l2(Jg, Jo) < 1e-12
    _compare_particles(o, s, wl, 1e-11)
    s32 = pic.Simulation.from_workload(wl, precision=32, sort_every=3, tile=tile)
    s32.step(10)
    Eg, Bg, _ = s32.fields()
    assert rel_l2(Eg, Eo) < 2e-5 and rel_l2(Bg, Bo) < 2e-5
    assert s.diagnostics()["error_word"] == 0 and s32.diagnostics()["error_word"] == 0


def test_open_faces_laser_walls_fp64(pic):
    """2D box with Mur faces, a Gaussian laser entering at x-min, reflecting
    particle walls: fields and particles follow the oracle."""
    _say("case: open faces + laser 2d fp64")
    wl = random_workload(2, 200, 200, seed=31, shape=(40, 24), dx=(0.2, 0.2), bc=OPEN,
                         vmax_el=0.9)
    g = wl.grid
    g.bc_lo = (LASER, OPEN, PERIODIC)
    g.laser = Laser(a0=0.05, omega=1.0, t_env=4 * math.pi, waist=2.0, yc=12 * 0.2, pol=1)
    o, s = _both(wl, pic, 64, sort_every=2)
    o.step(60)
    s.step(60)
    assert o.diagnostics()["error_word"] == 0, "oracle run left the valid range"
    assert s.diagnostics()["error_word"] == 0
    Eo, Bo, _ = o.fields()
    Eg, Bg, _ = s.fields()
    assert rel_l2(Eg, Eo) < 1e-12
    assert rel_l2(Bg, Bo) < 1e-12
    _compare_particles(o, s, wl, 1e-11)


@pytest.mark.parametrize("prec", [64, 32])
def test_open_faces_laser_3d(pic, prec):
    """3D box with Mur faces on x (a Gaussian laser entering at x-min) and y,
    periodic z (the boundaries of the slab workloads, with open y faces
    too): fields and particles follow the oracle."""
    _say(f"case: open faces + laser 3d fp{prec}")
    wl = random_workload(3, 300, 300, seed=37, shape=(70, 20, 40), dx=(0.2, 0.2, 0.2), bc=OPEN,
                         vmax_el=0.9)
    g = wl.grid
    g.bc_lo = (LASER, OPEN, PERIODIC)
    g.bc_hi = (OPEN, OPEN, PERIODIC)
    g.laser = Laser(a0=0.05, omega=1.0, t_env=4 * math.pi, waist=1.5, yc=10 * 0.2,
                    zc=20 * 0.2, pol=1)
    o, s = _both(wl, pic, prec, sort_every=2)
    o.step(50)
    s.step(50)
    assert o.diagnostics()["error_word"] == 0, "oracle run left the valid range"
    assert s.diagnostics()["error_word"] == 0
    Eo, Bo, _ = o.fields()
    Eg, Bg, _ = s.fields()
    tol = 1e-12 if prec == 64 else 2e-5
    assert rel_l2(Eg, Eo) < tol
    assert rel_l2(Bg, Bo) < tol
    assert np.abs(Eo).max() > 1e-4  # the pulse is in the box
    if prec == 64:
        _compare_particles(o, s, wl, 1e-11)


def test_charge_continuity_gpu(pic):
    """(rho^{n+1} - rho^n)/dt + div J = 0 on the GPU: round-off in FP64,
    reported (and small) in FP32."""
    for prec, tol in [(64, 1e-12), (32, 1e-5)]:
        _say(f"case: continuity precision={prec}")
        wl = random_workload(3, 400, 400, seed=41)
        s = pic.Simulation.from_workload(wl, precision=prec, flags=pic.CHARGE_CHECK)
        s.step(3)
        d = s.diagnostics()
        assert d["rho_l2"] > 0
        assert d["div_l2"] < tol * d["rho_l2"], (prec, d)


def test_fp32_against_fp64_oracle(pic):
    """FP32 path (cell + FP32 offset, stored delta) against the FP64 oracle."""
    _say("case: fp32 vs oracle 3d")
    wl = random_workload(3, 300, 300, seed=51)
    o = Oracle.from_workload(wl)
    s = pic.Simulation.from_workload(wl, precision=32)
    o.step(10)
    s.step(10)
    Eo, Bo, Jo = o.fields()
    Eg, Bg, Jg = s.fields()
    assert rel_l2(Eg, Eo) < 2e-5
    assert rel_l2(Bg, Bo) < 2e-5


@pytest.mark.parametrize("shape,tile,n", [((24, 16, 16), (4, 4, 4), 3000),
                                          ((160, 160, 80), (5, 5, 5), 60000),
                                          ((320, 320, 160), (5, 5, 5), 200000)])
def test_stable_tile_sort_permutation(pic, shape, tile, n):
    """The device sort orders particles by tile, stably: the new order is
    the stable argsort of the tile keys of the previous order (one radix
    pass for 96 tiles, two 7-bit passes for 16384, two 9-bit passes for
    131072)."""
    _say(f"case: tile sort permutation {shape} tile {tile}")
    wl = random_workload(3, n, 0, seed=61, shape=shape, vmax_ion=0.9)
    s = pic.Simulation.from_workload(wl, precision=64, flags=pic.TRACK_IDS, sort_every=1,
                                     tile=tile)
    s.step(1)                       # no sort on the first step after a load
    before = s.particles(0, ids=True)
    s.step(1)                       # sorts by the cells of `before`, then pushes
    after = s.particles(0, ids=True)
    c = before["cell"]
    nt = tuple(-(-shape[d] // tile[d]) for d in range(3))
    key = c[:, 0] // tile[0] + nt[0] * (c[:, 1] // tile[1] + nt[1] * (c[:, 2] // tile[2]))
    expect = before["id"][np.argsort(key, kind="stable")]
    assert np.array_equal(after["id"], expect)


def _load_order(cells, prev_ids, tile, nt):
    """Expected order after a load: by tile, then by the rank of the
    particle within its cell in the previous order (clamped at 255), then
    by the cell's index within the tile (x fastest), then stably."""
    nd = cells.shape[1]
    t = list(tile) + [1] * (3 - nd)
    c = np.zeros((len(cells), 3), dtype=np.int64)
    c[:, :nd] = cells
    n_t = list(nt) + [1] * (3 - nd)
    tid = c[:, 0] // t[0] + n_t[0] * (c[:, 1] // t[1] + n_t[1] * (c[:, 2] // t[2]))
    local = c[:, 0] % t[0] + t[0] * (c[:, 1] % t[1] + t[1] * (c[:, 2] % t[2]))
    ckey = tid * (t[0] * t[1] * t[2]) + local
    order = np.argsort(ckey, kind="stable")
    sk = ckey[order]
    rank = np.empty(len(ckey), dtype=np.int64)
    rank[order] = np.arange(len(sk)) - np.searchsorted(sk, sk, side="left")
    rank = np.minimum(rank, 255)
    return prev_ids[np.lexsort((np.arange(len(ckey)), local, rank, tid))]


@pytest.mark.parametrize("ndim,shape,tile", [(3, (24, 16, 16), (8, 8, 6)),
                                             (2, (48, 36), (12, 12)),
                                             (1, (600,), (256,))])
def test_load_order_within_tiles(pic, ndim, shape, tile):
    """The first sort after a host load orders each tile by the particles'
    rank within their cell (first particle of every cell, then every cell's
    second, ...) and by cell within a rank, whatever the load order; 300
    particles in one cell check the rank clamp at 255.  Later sorts keep
    the order stable (test_stable_tile_sort_permutation)."""
    _say(f"case: load order {ndim}d {shape} tile {tile}")
    n = {3: 20000, 2: 15000, 1: 6000}[ndim]
    wl = random_workload(ndim, n, 0, seed=67, shape=shape, vmax_ion=0.3)
    sp, parts = wl.species[0]
    x = np.array(parts.x, copy=True)
    dx = np.array(wl.grid.dx[:ndim])
    rng = np.random.default_rng(5)
    c0 = np.array([s // 2 for s in shape], float)
    x[:300] = (c0 + rng.uniform(0.2, 0.8, (300, ndim))) * dx
    # cell-major clumps: the next 3000 particles sorted by cell
    blk = x[300:3300]
    x[300:3300] = blk[np.lexsort(tuple(np.floor(blk[:, d] / dx[d]) for d in range(ndim)))]
    wl = dataclasses.replace(wl, species=[(sp, dataclasses.replace(parts, x=x))])
    s = pic.Simulation.from_workload(wl, precision=64, flags=pic.TRACK_IDS, tile=tile)
    before = s.particles(0, ids=True)   # host loader's tile order, before the device sort
    s.step(1)                           # ordering sort, then the push
    after = s.particles(0, ids=True)
    nt = tuple(-(-shape[d] // tile[d]) for d in range(ndim))
    assert np.array_equal(after["id"], _load_order(before["cell"], before["id"], tile, nt))
    assert s.diagnostics()["error_word"] == 0
    s.close()


def test_load_order_device_loader(pic):
    """Device loads sort at once into the same order (ranks counted in the
    load order)."""
    import torch
    _say("case: load order device loader 3d")
    shape, tile = (24, 16, 16), (8, 8, 6)
    wl = random_workload(3, 30000, 0, seed=71, shape=shape, vmax_ion=0.3)
    sp, parts = wl.species[0]
    dx = np.array(wl.grid.dx)
    x = np.array(parts.x, copy=True)
    x = x[np.lexsort(tuple(np.floor(x[:, d] / dx[d]) for d in range(3)))]   # cell-major
    s = pic.Simulation(wl.grid, precision=32, flags=pic.TRACK_IDS, tile=tile)
    sid = s.add_species(sp, parts.n)
    dev = torch.device("cuda", 0)
    s.load_particles_device(sid, torch.tensor(x, device=dev), torch.tensor(parts.u1, device=dev),
                            delta=torch.tensor(parts.delta, device=dev),
                            u2=torch.tensor(parts.u2, device=dev),
                            omega_c=torch.tensor(parts.omega_c, device=dev),
                            weight=torch.tensor(parts.weight, device=dev))
    after = s.particles(0, ids=True)
    cells = np.empty_like(after["cell"])
    cells[after["id"]] = after["cell"]       # cells in load order
    nt = tuple(-(-shape[d] // tile[d]) for d in range(3))
    assert np.array_equal(after["id"], _load_order(cells, np.arange(parts.n), tile, nt))
    s.close()


def test_bragg_case_fp64_fp32(pic):
    """Reduced Bragg case (Sec. 3.2 geometry, 512^2 cells, 700 steps): GPU
    fields match the oracle (FP64 1e-12, FP32 2e-5 relative L2); the FP32
    scattered field (run with ions minus run without) against the oracle's
    is reported and keeps the Bragg direction 2 theta_B."""
    import math
    from _bragg import bragg_case, scattered_direction
    _say("case: bragg 2d reduced")
    wl = bragg_case(1.5)
    ovac = Oracle(wl.grid)
    ovac.step(wl.steps)
    omed = Oracle.from_workload(wl)
    omed.step(wl.steps)
    Eo = omed.fields()[0]
    es_ref = Eo[2] - ovac.fields()[0][2]
    for prec, tol in ((64, 1e-12), (32, 2e-5)):
        vac = pic.Simulation(wl.grid, precision=prec)
        vac.step(wl.steps)
        med = pic.Simulation.from_workload(wl, precision=prec)
        med.step(wl.steps)
        Eg = med.fields()[0]
        assert rel_l2(Eg, Eo) < tol
        es = Eg[2] - vac.fields()[0][2]
        err = rel_l2(es, es_ref)
        angle, kmean, contrast = scattered_direction(wl, es)
        _say(f"bragg fp{prec}: field rel L2 {rel_l2(Eg, Eo):.2e}, scattered field rel L2 "
             f"{err:.2e}, direction {angle:.2f} deg")
        assert err < (1e-10 if prec == 64 else 2e-4)
        expect = 2 * math.degrees(math.asin(1.0 / 3.0))
        assert abs(angle - expect) < math.degrees(1.0 / 16.0)
        assert med.diagnostics()["error_word"] == 0


def _gpu_series(pic, wl, probes, with_medium, prec):
    if with_medium:
        s = pic.Simulation.from_workload(wl, precision=prec, max_probe_steps=wl.steps)
    else:
        s = pic.Simulation(wl.grid, precision=prec, max_probe_steps=wl.steps)
    s.set_probes([(1, (p, 0, 0)) for p in probes])
    s.step(wl.steps)
    assert s.diagnostics()["error_word"] == 0
    return s.probes()


def test_sec31_observables_gpu(pic):
    """Group velocity (w_c = 2.5) and reflection phase (opaque medium,
    w_c = 0.8) on the GPU: probe series against the oracle's (FP64 relative
    L2 1e-12, FP32 2e-5) and the observables against the Sec. 3.1 closed
    forms (as for the oracle pins)."""
    import _sec31 as S31
    _say("case: sec 3.1 group velocity and reflection")
    wl, probes = S31.group_velocity_case(2.5)
    ref = Oracle.from_workload(wl, max_probe_steps=wl.steps)
    ref.set_probes([(1, (p, 0, 0)) for p in probes])
    ref.step(wl.steps)
    pr_o = ref.probes()
    wr, (pp,) = S31.reflection_case(0.8)
    rv = Oracle(wr.grid, max_probe_steps=wr.steps)
    rm = Oracle.from_workload(wr, max_probe_steps=wr.steps)
    for o in (rv, rm):
        o.set_probes([(1, (pp, 0, 0))])
        o.step(wr.steps)
    for prec, tol in ((64, 1e-12), (32, 2e-5)):
        pr = _gpu_series(pic, wl, probes, True, prec)
        assert rel_l2(pr, pr_o) < tol
        v = S31.measured_group_velocity(wl, probes, pr)
        assert abs(v / S31.group_velocity_theory(2.5) - 1.0) < 1e-3
        vac = _gpu_series(pic, wr, (pp,), False, prec)[0]
        med = _gpu_series(pic, wr, (pp,), True, prec)[0]
        assert rel_l2(med, rm.probes()[0]) < tol and rel_l2(vac, rv.probes()[0]) < tol
        r = S31.measured_reflection(wr, pp, vac, med)
        assert abs(np.angle(r) - np.angle(S31.reflection_theory(0.8))) < 0.01
        _say(f"fp{prec}: v_g {v:.5f} (theory {S31.group_velocity_theory(2.5):.5f}), "
             f"reflection phase {np.angle(r):.4f} (theory "
             f"{np.angle(S31.reflection_theory(0.8)):.4f})")


def test_refraction_gpu(pic):
    """Oblique plane wave (30 degrees, E along z) into the medium, 2D: GPU
    probe series against the oracle's (FP64 1e-12, FP32 2e-5) and the
    refraction angle against Snell's law (0.2 degrees), as for the oracle."""
    import math
    import _sec31 as S31
    _say("case: refraction 2d")
    wl, vac, med = S31.refraction_case(2.0)
    probes = [(2, (x, 32, 0)) for x in vac + med]
    o = Oracle.from_workload(wl, max_probe_steps=wl.steps)
    o.set_probes(probes)
    o.step(wl.steps)
    pr_o = o.probes()
    n = math.sqrt(S31.eps_r(2.0))
    for prec, tol in ((64, 1e-12), (32, 2e-5)):
        s = pic.Simulation.from_workload(wl, precision=prec, max_probe_steps=wl.steps)
        s.set_probes(probes)
        s.step(wl.steps)
        assert s.diagnostics()["error_word"] == 0
        pr = s.probes()
        assert rel_l2(pr, pr_o) < tol
        km = S31.measured_kx(wl, med, pr[len(vac):])
        theta_t = math.degrees(math.atan2(0.5, km))
        _say(f"fp{prec}: refraction angle {theta_t:.3f} deg (Snell "
             f"{math.degrees(math.asin(0.5 / n)):.3f}), probes rel L2 {rel_l2(pr, pr_o):.2e}")
        assert abs(theta_t - math.degrees(math.asin(0.5 / n))) < 0.2


def test_neutral_medium_case_fp64(pic):
    """The full 1D neutral-medium case (2048 cells, 16k two-body ions,
    1000 steps): fields and probes match the oracle."""
    _say("case: neutral_medium_1d full fp64")
    wl = neutral_medium_1d()
    o = Oracle.from_workload(wl, max_probe_steps=wl.steps)
    s = pic.Simulation.from_workload(wl, precision=64, max_probe_steps=wl.steps,
                                     flags=pic.TRACK_IDS)
    o.step(wl.steps)
    s.step(wl.steps)
    Eo, Bo, _ = o.fields()
    Eg, Bg, _ = s.fields()
    assert rel_l2(Eg, Eo) < 1e-12
    assert rel_l2(Bg, Bo) < 1e-12
    assert np.max(np.abs(s.probes() - o.probes())) < 1e-12 * np.abs(o.probes()).max()
    ref = o.particles(0)
    got = s.particles(0, ids=True)
    got = match_by_id(got, got["id"])
    assert np.array_equal(ref["cell"], got["cell"])


def test_edge_cases(pic):
    """Empty species, a single particle, ragged counts."""
    _say("case: edge cases")
    for n in [0, 1, 255, 257]:
        wl = random_workload(2, n, n, seed=70 + n)
        o, s = _both(wl, pic, 64)
        o.step(2)
        s.step(2)
        assert rel_l2(s.fields()[0], o.fields()[0]) < 1e-12 if n else True
        assert s.diagnostics()["n_particles"] == 2 * n


def test_load_errors(pic):
    """Invalid inputs are rejected at load with the documented codes."""
    _say("case: load errors")
    g = small_grid(1, (16,), (0.3,), bc=OPEN)
    s = pic.Simulation(g, precision=64)
    sid = s.add_species(Species(TWO_BODY, 2.0, 10.0, -1.0, 1.0, omega_c=1.0, a_c=math.inf), 4)
    bad_u = Particles(x=np.array([[1.5]]), u1=np.array([[np.nan, 0, 0]]))
    with pytest.raises(pic.PicError) as e:
        s.load_particles(sid, bad_u)
    assert e.value.code == pic.PIC_ENAN
    # the cloud beyond the particle wall (3 cells in)
    bad_d = Particles(x=np.array([[3.5 * 0.3]]), u1=np.zeros((1, 3)),
                      delta=np.array([[1.0 * 0.3, 0, 0]]))
    with pytest.raises(pic.PicError) as e:
        s.load_particles(sid, bad_d)
    assert e.value.code == pic.PIC_ERANGE
    # far apart but inside: accepted (each body has its own position)
    s.load_particles(sid, Particles(x=np.array([[8.0 * 0.3]]), u1=np.zeros((1, 3)),
                                    delta=np.array([[3.0 * 0.3, 0.7, 0]])))
    many = Particles(x=np.ones((5, 1)) * 1.5, u1=np.zeros((5, 3)))
    with pytest.raises(pic.PicError) as e:
        s.load_particles(sid, many)
    assert e.value.code == pic.PIC_ENOMEM
    # per-particle omega_c: positive, and not with a fixed finite a_c
    s2 = pic.Simulation(g, precision=64)
    fixed = s2.add_species(Species(TWO_BODY, 2.0, 10.0, -1.0, 1.0, omega_c=1.0, a_c=0.2), 4)
    with pytest.raises(pic.PicError) as e:
        s2.load_particles(fixed, Particles(x=np.array([[1.5]]), u1=np.zeros((1, 3)),
                                           omega_c=np.array([1.0])))
    assert e.value.code == pic.PIC_EINVAL
    harm = s2.add_species(Species(TWO_BODY, 2.0, 10.0, -1.0, 1.0, omega_c=1.0, a_c=math.inf), 4)
    with pytest.raises(pic.PicError) as e:
        s2.load_particles(harm, Particles(x=np.array([[1.5]]), u1=np.zeros((1, 3)),
                                          omega_c=np.array([-1.0])))
    assert e.value.code == pic.PIC_EINVAL
    with pytest.raises(pic.PicError) as e:
        s2.add_species(Species(TWO_BODY, 2.0, 10.0, -1.0, 1.0, omega_c=1.0, a_c=-0.5), 1)
    assert e.value.code == pic.PIC_EINVAL


def test_device_error_word(pic):
    """A momentum that overflows during a step (a field of 1e308 in a frozen
    grid) raises PIC_ENAN at the next diagnostics: the kernel flags it, the
    particle stops, nothing faults."""
    _say("case: device error word")
    g = small_grid(1, (16,), (0.3,), bc=OPEN)
    s = pic.Simulation(g, precision=64, flags=pic.FROZEN_FIELDS)
    sid = s.add_species(Species(TWO_BODY, 2.0, 10.0, -1.0, 1.0, omega_c=1.0, a_c=math.inf), 1)
    s.load_particles(sid, Particles(x=np.array([[8.4 * 0.3]]), u1=np.zeros((1, 3)),
                                    u2=np.zeros((1, 3)), delta=np.zeros((1, 3))))
    E = np.zeros((3, 16))
    E[1] = 1e308  # kicks of ~5e306 per step: the momentum overflows within 40 steps
    s.load_fields(E, np.zeros((3, 16)))
    s.step(40)
    d = s.diagnostics(check=False)
    assert d["status"] == pic.PIC_ENAN
    assert d["error_word"] & pic.ERR_NAN


def test_timing_events(pic):
    _say("case: timing")
    wl = random_workload(3, 1000, 1000, seed=80)
    # tiled kernel, ions and electrons in one launch per tile colour (2^3)
    # and step, counted for the two-body species
    s = pic.Simulation.from_workload(wl, precision=32, flags=pic.TIMING)
    s.step(3)
    ms0, n0 = s.timing(species=0, reset=False)
    ms1, n1 = s.timing(species=1, reset=False)
    ms, n = s.timing()
    assert n0 == 3 * 8 and n1 == 0 and n == n0 and ms == ms0 > 0
    # one launch per species: one timed dispatch per colour, species and step
    s = pic.Simulation.from_workload(wl, precision=32, flags=pic.TIMING | pic.SEPARATE_SPECIES)
    s.step(3)
    ms0, n0 = s.timing(species=0, reset=False)
    ms, n = s.timing()
    assert n0 == 3 * 8 and n == 2 * n0 and ms >= ms0 > 0
    # global kernel: one dispatch per species and step
    s = pic.Simulation.from_workload(wl, precision=32, flags=pic.TIMING | pic.GLOBAL_KERNEL)
    s.step(3)
    ms, n = s.timing()
    assert n == 6 and ms > 0


def test_device_loader_matches_host_loader(pic):
    """Loading the same FP64 arrays from device memory gives the same state
    as the host loader: cells, offsets and delta bit-identical, momenta
    (through the Sec. 2 split of a charged ion's momentum) to round-off."""
    import torch
    _say("case: device loader vs host loader")
    for prec in (64, 32):
        wl = random_workload(3, 2000, 1000, seed=91)
        sp, parts = wl.species[0]
        parts.u2 = None          # exercise the split
        parts.delta = None
        a = pic.Simulation.from_workload(wl, precision=prec, flags=pic.TRACK_IDS)
        b = pic.Simulation(wl.grid, precision=prec, flags=pic.TRACK_IDS)
        for s_, p_ in wl.species:
            sid = b.add_species(s_, p_.n)
            t = lambda v: None if v is None else torch.from_numpy(v).cuda()
            b.load_particles_device(sid, t(p_.x), t(p_.u1), delta=t(p_.delta), u2=t(p_.u2),
                                    omega_c=t(p_.omega_c), weight=t(p_.weight))
        for sid in range(2):
            ga = a.particles(sid, ids=True)
            gb = b.particles(sid, ids=True)
            ga = match_by_id(ga, ga["id"])
            gb = match_by_id(gb, gb["id"])
            for k in ("cell", "off", "delta"):
                assert np.array_equal(ga[k], gb[k]), (prec, sid, k)
            # the split's Newton iteration may contract multiply-adds differently
            for k in ("u1", "u2"):
                scale = max(np.abs(ga[k]).max(), 1e-300)
                assert np.abs(ga[k] - gb[k]).max() <= 2e-15 * scale * (1 if prec == 64 else 1e9)


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_particles_outside_their_tile(pic, ndim):
    """Fast electrons with a long sort interval leave their tiles; those
    particles take the HBM path and the result still matches the oracle."""
    _say(f"case: drift out of tiles ndim={ndim}")
    wl = random_workload(ndim, 200, 600, seed=140 + ndim, shape=(40, 24, 20)[:ndim],
                         vmax_el=0.95)
    o, s = _both(wl, pic, 64, sort_every=1000, tile=(8, 8, 8)[:ndim])
    o.step(12)
    s.step(12)
    d = s.diagnostics()
    assert d["n_outside_tile"] > 0
    assert o.diagnostics()["error_word"] == 0
    Eo, Bo, Jo = o.fields()
    Eg, Bg, Jg = s.fields()
    assert rel_l2(Eg, Eo) < 1e-12
    assert rel_l2(Jg, Jo) < 1e-12
    _compare_particles(o, s, wl, 1e-11)


def test_adaptive_sort_policy(pic):
    """Default sort policy with hot electrons: the species is re-sorted once
    enough of it was advanced outside its tile (the storage order changes),
    and the coupled run still follows the oracle."""
    _say("case: adaptive sort policy")
    wl = random_workload(3, 400, 3000, seed=91, shape=(24, 24, 16), vmax_el=0.95)
    o, s = _both(wl, pic, 64)
    first = s.particles(1, ids=True)["id"].copy()
    o.step(12)
    s.step(12)
    assert o.diagnostics()["error_word"] == 0, "oracle run left the valid range"
    later = s.particles(1, ids=True)["id"]
    assert not np.array_equal(first, later), "no sort of the electrons in 12 steps"
    Eo, Bo, Jo = o.fields()
    Eg, Bg, Jg = s.fields()
    assert rel_l2(Eg, Eo) < 1e-12 and rel_l2(Bg, Bo) < 1e-12
    _compare_particles(o, s, wl, 1e-11)


def test_fp32_current_patch_fixed_point(pic):
    """FP32 work accumulates each tile's current in 64-bit fixed point: the
    sum does not depend on the order of the LDS atomics, so two identical
    FP32 steps give bit-identical J (no particle leaves its tile in a first
    step after a load, so no global atomics are involved); a tile with more
    than 32768 particles (the rest go to the outside-tile kernel) still
    follows the oracle."""
    _say("case: fp32 fixed-point patch")
    wl = random_workload(3, 600, 600, seed=101)
    J = []
    for _ in range(2):
        s = pic.Simulation.from_workload(wl, precision=32)
        s.step(1)
        assert s.diagnostics()["n_outside_tile"] == 0
        J.append(s.fields()[2])
    assert np.array_equal(J[0], J[1])
    # crowded tile: 40000 electrons in the first 8x8x6 tile
    g = small_grid(3, (16, 16, 12), (0.3, 0.25, 0.2))
    rng = np.random.default_rng(7)
    n = 40000
    x = rng.random((n, 3)) * np.array([8 * 0.3, 8 * 0.25, 6 * 0.2])
    parts = Particles(x=x, u1=rng.normal(0.0, 0.05, (n, 3)))
    sp = Species(POINT, -1.0, 1.0, 0.0, 0.0, weight=1e-4)
    from paper_2208_08038_amd.inputs import Workload
    wc = Workload("crowded", g, [(sp, parts)], 2, 32)
    o = Oracle.from_workload(wc)
    s = pic.Simulation.from_workload(wc, precision=32)
    o.step(2)
    s.step(2)
    assert s.diagnostics()["error_word"] == 0
    Eo, Bo, Jo = o.fields()
    Eg, Bg, Jg = s.fields()
    assert rel_l2(Eg, Eo) < 2e-5 and rel_l2(Jg, Jo) < 2e-5


@pytest.mark.parametrize("precision,tol", [(64, 1e-13), (32, 1e-6)])
def test_shared_launch_matches_separate(pic, precision, tol):
    """Ions and electrons advanced in one launch per tile colour (the
    default for a two-body and a point species) against one launch per
    species (PIC_FLAG_SEPARATE_SPECIES): the same fields and particles up
    to the order of the FP64 patch sums, or, for FP32 work, the fixed-point
    quantum of the shared patch scale (which moves a few FP32 results by an
    ulp); 3D, 2D and 1D, with particles leaving their tiles (fast electrons,
    no sort for 4 steps)."""
    for ndim in (3, 2, 1):
        _say(f"case: shared launch {ndim}d fp{precision}")
        wl = random_workload(ndim, 1500, 1500, seed=113 + ndim, vmax_el=0.95)
        out = []
        for flags in (pic.TRACK_IDS, pic.TRACK_IDS | pic.SEPARATE_SPECIES):
            s = pic.Simulation.from_workload(wl, precision=precision, flags=flags, sort_every=1000)
            s.step(4)
            d = s.diagnostics()
            assert d["error_word"] == 0
            out.append((s.fields(), [s.particles(k, ids=True) for k in range(2)],
                        d["n_outside_tile"]))
            s.close()
        (fa, pa, na), (fb, pb, nb) = out
        assert na == nb and (na > 0 or ndim == 1)
        for x, y in zip(fa, fb):
            assert rel_l2(x, y) < tol
        for k in range(2):
            ia, ib = np.argsort(pa[k]["id"]), np.argsort(pb[k]["id"])
            assert np.array_equal(pa[k]["cell"][ia], pb[k]["cell"][ib])
            for key in ("off", "u1"):
                a_, b_ = pa[k][key][ia], pb[k][key][ib]
                assert np.max(np.abs(a_ - b_) / np.maximum(1.0, np.abs(b_))) < tol


def test_shared_launch_empty_partner(pic):
    """A shared launch whose two-body species holds no particle yet (a load
    of zero ions with per-particle weights, so no weight bounds its terms)
    takes the electrons' patch scale: the same current as one launch per
    species."""
    _say("case: shared launch, empty ion species")
    wl = random_workload(3, 0, 1200, seed=131)
    el_sp, el = wl.species[0]
    ion_sp = Species(TWO_BODY, 5.0, 40.0, -3.0, 3.0, weight=0.005, omega_c=2.0, a_c=0.0,
                     nu=0.05, name="ion")
    z3 = np.zeros((0, 3))
    empty = Particles(x=z3, u1=z3, u2=z3, delta=z3, omega_c=np.zeros(0), weight=np.zeros(0))
    wl = dataclasses.replace(wl, species=[(ion_sp, empty), (el_sp, el)])
    J = []
    for flags in (0, pic.SEPARATE_SPECIES):
        s = pic.Simulation.from_workload(wl, precision=32, flags=flags)
        s.step(2)
        assert s.diagnostics()["error_word"] == 0
        J.append(s.fields()[2])
        s.close()
    assert np.max(np.abs(J[0])) > 0
    assert rel_l2(J[0], J[1]) < 1e-6


def test_global_kernel_option(pic):
    """The HBM-gather / global-atomic kernel (PIC_FLAG_GLOBAL_KERNEL) agrees
    with the oracle too."""
    _say("case: global kernel option 3d")
    wl = random_workload(3, 300, 300, seed=150)
    o, s = _both(wl, pic, 64, pflags=pic.GLOBAL_KERNEL)
    o.step(8)
    s.step(8)
    assert rel_l2(s.fields()[0], o.fields()[0]) < 1e-12
    _compare_particles(o, s, wl, 1e-11)


@pytest.fixture(scope="module")
def mixed_case():
    """The mixed-precision case (Bragg geometry in 3D, lattice-modulated
    per-particle weights) at reduced size, and its FP64 oracle run."""
    from paper_2208_08038_amd.inputs import mixed_precision_3d
    wl = mixed_precision_3d(n=(80, 12, 12), slab=(20, 44), ppc=1, steps=220, cycles=2)
    o = Oracle.from_workload(wl)
    o.step(wl.steps)
    assert o.diagnostics()["error_word"] == 0
    ref = o.fields()
    o.close()
    return wl, ref


@pytest.mark.parametrize("precision", [64, 32])
def test_mixed_precision_case(pic, mixed_case, precision):
    """Per-step charge-continuity residual (FP64 compensated reduction) and
    the final fields, whole grid and the transmitted region behind the
    slab, against the FP64 oracle."""
    wl, (Eo, Bo, _) = mixed_case
    _say(f"case: mixed-precision 3D fp{precision}, {wl.species[0][1].n} ions, {wl.steps} steps")
    s = pic.Simulation.from_workload(wl, precision=precision, flags=pic.CHARGE_CHECK)
    sp = wl.species[0][0]
    dx = wl.grid.dx[0]
    ncell = int(np.prod(wl.grid.n))
    # rounding of the continuity residual scales with the largest charge
    # rate of a cell: the site-modulated weights peak far above their mean
    wmax = float(np.max(wl.species[0][1].weight))
    gross = wmax * (abs(sp.q1) + abs(sp.q2)) / (dx ** 3 * wl.grid.dt)
    eps = 2.0 ** -24 if precision == 32 else 2.0 ** -53
    worst = 0.0
    for _ in range(wl.steps):
        s.step(1)
        d = s.diagnostics()
        assert d["error_word"] == 0
        worst = max(worst, d["div_l2"] / math.sqrt(ncell))
    assert worst < eps * gross, (worst, eps * gross)
    Eg, Bg, _ = s.fields()
    s.close()
    tol = 1e-12 if precision == 64 else 2e-5
    nx, ny, nz = wl.grid.n
    behind = (slice(None), slice(None), slice(48, nx - 4))

    def region(F):
        return F.reshape(3, nz, ny, nx)[(slice(None),) + behind]
    errs = {"E": rel_l2(Eg, Eo), "B": rel_l2(Bg, Bo),
            "E transmitted": rel_l2(region(Eg), region(Eo))}
    _say(f"fp{precision}: per-step residual RMS max {worst:.3e} (bound {eps * gross:.3e}); " +
         ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v < tol, k
