"""GPU: multi-shell ions (a nucleus and up to four bound clouds, one bond
each; the extension named in the paper's summary) against the FP64 oracle:
coupled runs in 1D-3D with periodic and open faces (walls mirroring each
body), FP32 to its rounding, the FP64 diagnostics, charge continuity,
checkpoint/restart, and the refusals."""
import dataclasses
import math
import sys

import numpy as np
import pytest

from _parity import match_by_id, rel_l2, small_grid
from oracle.oracle import CHARGE_CHECK as O_CHECK
from oracle.oracle import Oracle
from paper_2208_08038_amd.inputs import (MULTI_SHELL, OPEN, PERIODIC, POINT, Particles, Species,
                                         Workload, multishell_medium_1d)

pytestmark = pytest.mark.gpu


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


SHELLS = ((-2.0, 2.0, 1.7, 0.0), (-3.0, 3.0, 0.9, math.inf), (-1.0, 1.0, 2.6, 0.0))


def shell_workload(ndim, n_ion, n_el, seed, K=3, bc=PERIODIC, vmax=0.2, spread=0.08):
    """Random multi-shell ions (K clouds; net charge +2) and electrons, every
    body between the walls when the faces are open."""
    rng = np.random.default_rng(seed)
    shape = (23, 17, 13)[:ndim]
    dx = (0.3, 0.25, 0.2)[:ndim]
    g = small_grid(ndim, shape, dx, bc=bc, re_norm=2e-3)
    shells = SHELLS[:K]
    q0 = 2.0 - sum(s[0] for s in shells)
    sp = Species(MULTI_SHELL, q0, 60.0, weight=0.004, nu=0.05, shells=shells, name="ms")
    pad = g.pad + 0.6 if bc == OPEN else 0.0
    lo = np.array([pad] * ndim)
    hi = np.array([s - pad for s in shape], float)
    x = (lo + (hi - lo) * rng.random((n_ion, ndim))) * np.array(dx)
    u = rng.normal(size=(n_ion, 3)) * vmax / math.sqrt(3)
    u1 = u
    u2 = np.tile(u, (1, K)) + rng.normal(scale=0.02, size=(n_ion, 3 * K))
    delta = rng.uniform(-spread, spread, (n_ion, 3 * K)) * min(dx)
    species = [(sp, Particles(x=x, u1=u1, delta=delta, u2=u2))]
    if n_el:
        el = Species(POINT, -1.0, 1.0, weight=0.004, name="e")
        xe = (lo + (hi - lo) * rng.random((n_el, ndim))) * np.array(dx)
        species.append((el, Particles(x=xe, u1=rng.normal(scale=0.3, size=(n_el, 3)))))
    return Workload(f"shells{ndim}d", g, species, steps=1, precision=64)


def _run_both(pic, wl, precision, steps, oflags=0, pflags=0):
    o = Oracle.from_workload(wl, flags=oflags)
    s = pic.Simulation.from_workload(wl, precision=precision, flags=pflags | pic.TRACK_IDS)
    o.step(steps)
    s.step(steps)
    return o, s


def _compare(o, s, wl, tol, exact_cells=True):
    for sid, (sp, parts) in enumerate(wl.species):
        ref = o.particles(sid)
        got = s.particles(sid, ids=True)
        got = match_by_id(got, got["id"])
        if exact_cells:
            assert np.array_equal(ref["cell"], got["cell"])
        pr, pg = ref["cell"] + ref["off"], got["cell"] + got["off"]
        assert np.abs(pr - pg).max() < 10 * tol
        keys = ["u1"] + (["u2", "delta"] if sp.kind == MULTI_SHELL else [])
        for k in keys:
            scale = max(np.abs(ref[k]).max(), 1e-300)
            err = np.abs(ref[k] - got[k]).max() / scale
            assert err < tol, f"species {sid} {k}: {err:.3e}"


@pytest.mark.parametrize("ndim,bc", [(1, PERIODIC), (2, PERIODIC), (3, PERIODIC), (2, OPEN),
                                     (3, OPEN)])
def test_shells_coupled_fp64(pic, ndim, bc):
    _say(f"case: shells coupled fp64 ndim={ndim} bc={bc}")
    wl = shell_workload(ndim, 60, 60, seed=70 + ndim + 5 * bc, bc=bc)
    o, s = _run_both(pic, wl, 64, 20)
    assert o.diagnostics()["error_word"] == 0
    assert s.diagnostics()["error_word"] == 0
    Eo, Bo, Jo = o.fields()
    Eg, Bg, Jg = s.fields()
    assert rel_l2(Eg, Eo) < 1e-12 and rel_l2(Bg, Bo) < 1e-12 and rel_l2(Jg, Jo) < 1e-12
    _compare(o, s, wl, 1e-11)
    do, dg = o.diagnostics(), s.diagnostics()
    for k in ("field_energy", "kinetic_energy"):
        assert abs(dg[k] - do[k]) <= 1e-12 * abs(do[k]), k
    pm = np.array(do["momentum"])
    assert np.abs(np.array(dg["momentum"]) - pm).max() <= 1e-12 * np.abs(pm).max()


@pytest.mark.parametrize("ndim", [2, 3])
def test_shells_tiled_fp32_far_clouds(pic, ndim):
    """FP32 (one workgroup per tile with an LDS current patch once sorted)
    against the FP64 oracle with clouds up to 2.5 smallest cell widths from
    their nucleus on a periodic grid of several tiles: bodies in the tile's cells deposit
    into the patch, bodies in other tiles or across a periodic face go to
    the planes directly."""
    _say(f"case: shells tiled fp32 far ndim={ndim}")
    wl = shell_workload(ndim, 80, 40, seed=130 + ndim, K=2, spread=2.5)
    o, s = _run_both(pic, wl, 32, 10)
    assert s.diagnostics()["error_word"] == 0
    Eo, Bo, Jo = o.fields()
    Eg, Bg, Jg = s.fields()
    errs = (rel_l2(Eg, Eo), rel_l2(Bg, Bo), rel_l2(Jg, Jo))
    _say(f"fp32 tiled far ndim={ndim}: E {errs[0]:.2e} B {errs[1]:.2e} J {errs[2]:.2e}")
    assert max(errs) < 2e-5
    _compare(o, s, wl, 5e-5, exact_cells=False)


def test_shells_large_tiles_take_the_hbm_kernel(pic):
    """Tiles too large for the LDS of the tiled kernels (16^3 and 24^3 cells
    in 3D FP64): the context advances every species from HBM with global
    atomics, and a multi-shell species' step and charge density still match
    the oracle."""
    _say("case: shells with large tiles")
    wl = shell_workload(3, 60, 60, seed=150, K=2)
    for tile in ((16, 16, 16), (24, 24, 24)):
        o = Oracle.from_workload(wl)
        s = pic.Simulation.from_workload(wl, precision=64, flags=pic.TRACK_IDS, tile=tile)
        o.step(6)
        s.step(6)
        assert s.diagnostics()["error_word"] == 0
        Eo, Bo, Jo = o.fields()
        Eg, Bg, Jg = s.fields()
        assert rel_l2(Eg, Eo) < 1e-12 and rel_l2(Jg, Jo) < 1e-12
        _compare(o, s, wl, 1e-11)
        ro = o.rho()
        assert np.abs(s.rho() - ro).max() < 1e-12 * np.abs(ro).max()
        s.close()


@pytest.mark.parametrize("K", [1, 2, 4])
def test_shells_count_fp32(pic, K):
    """FP32 against the FP64 oracle for 1, 2 and 4 clouds (2D, open faces)."""
    _say(f"case: shells fp32 K={K}")
    shells4 = SHELLS + ((-1.5, 1.5, 1.2, math.inf),)
    wl = shell_workload(2, 50, 50, seed=90 + K, K=min(K, 3), bc=OPEN)
    if K == 4:
        sp, parts = wl.species[0]
        rng = np.random.default_rng(3)
        sp = dataclasses.replace(sp, shells=shells4, q1=2.0 - sum(s[0] for s in shells4))
        parts = dataclasses.replace(
            parts, delta=np.hstack([parts.delta, rng.uniform(-0.01, 0.01, (parts.n, 3))]),
            u2=np.hstack([parts.u2, parts.u1]))
        wl = dataclasses.replace(wl, species=[(sp, parts)] + wl.species[1:])
    o, s = _run_both(pic, wl, 32, 15)
    assert s.diagnostics()["error_word"] == 0
    Eo, Bo, Jo = o.fields()
    Eg, Bg, Jg = s.fields()
    errs = (rel_l2(Eg, Eo), rel_l2(Bg, Bo), rel_l2(Jg, Jo))
    _say(f"fp32 K={K}: E {errs[0]:.2e} B {errs[1]:.2e} J {errs[2]:.2e}")
    assert max(errs) < 2e-5
    _compare(o, s, wl, 5e-5, exact_cells=False)


def test_shells_charge_continuity(pic):
    """The GPU continuity residual of a coupled 3D multi-shell run stays at
    rounding level against rho (each body deposits its own current)."""
    _say("case: shells continuity")
    wl = shell_workload(3, 80, 80, seed=5, bc=OPEN)
    s = pic.Simulation.from_workload(wl, precision=64, flags=pic.CHARGE_CHECK)
    s.step(6)
    d = s.diagnostics()
    assert d["error_word"] == 0 and d["rho_l2"] > 0
    assert d["div_l2"] < 1e-11 * d["rho_l2"]


def test_shells_restart(pic):
    """Save after 7 steps, restore into a new context, run to 16: equal to
    the uninterrupted run to FP64 rounding (cells exact)."""
    _say("case: shells restart")
    wl = shell_workload(2, 40, 40, seed=8, bc=OPEN)
    a = pic.Simulation.from_workload(wl, precision=64, flags=pic.TRACK_IDS)
    a.step(16)
    b = pic.Simulation.from_workload(wl, precision=64, flags=pic.TRACK_IDS)
    b.step(7)
    buf = b.save_state()
    b.close()
    c = pic.Simulation(wl.grid, precision=64, flags=pic.TRACK_IDS)
    for sp, parts in wl.species:
        c.add_species(sp, parts.n)
    c.load_state(buf)
    c.step(9)
    Ea, Ba, _ = a.fields()
    Ec, Bc, _ = c.fields()
    assert rel_l2(Ec, Ea) < 1e-13 and rel_l2(Bc, Ba) < 1e-13
    pa = a.particles(0, ids=True)
    pc = c.particles(0, ids=True)
    pa, pc = match_by_id(pa, pa["id"]), match_by_id(pc, pc["id"])
    assert np.array_equal(pa["cell"], pc["cell"])
    for k in ("delta", "u2", "u1"):
        assert np.abs(pa[k] - pc[k]).max() <= 1e-13 * np.abs(pa[k]).max()


def test_shells_refusals(pic):
    """Per-particle omega_c (host and device loads) and gradient runs refuse
    a multi-shell species (PIC_EINVAL); a body outside the walls is
    PIC_ERANGE from either loader; a bad shell is refused at creation."""
    _say("case: shells refusals")
    import torch
    wl = shell_workload(2, 10, 0, seed=9, bc=OPEN)
    sp, parts = wl.species[0]
    s = pic.Simulation(wl.grid, precision=64)
    sid = s.add_species(sp, 100)
    with pytest.raises(pic.PicError) as e:
        s.load_particles(sid, dataclasses.replace(parts, omega_c=np.full(parts.n, 2.0)))
    assert e.value.code == pic.PIC_EINVAL
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    with pytest.raises(pic.PicError) as e:
        s.load_particles_device(sid, dev(parts.x), dev(parts.u1), delta=dev(parts.delta),
                                u2=dev(parts.u2), omega_c=dev(np.full(parts.n, 2.0)))
    assert e.value.code == pic.PIC_EINVAL
    far = parts.delta.copy()
    far[0, 0] = 40.0 * wl.grid.dx[0]  # cloud 1 of ion 0 beyond the wall
    with pytest.raises(pic.PicError) as e:
        s.load_particles(sid, dataclasses.replace(parts, delta=far))
    assert e.value.code == pic.PIC_ERANGE
    with pytest.raises(pic.PicError) as e:
        s.load_particles_device(sid, dev(parts.x), dev(parts.u1), delta=dev(far),
                                u2=dev(parts.u2))
    assert e.value.code == pic.PIC_ERANGE
    assert s.count(sid) == 0
    s.load_particles(sid, parts)
    with pytest.raises(pic.PicError) as e:
        s.grad_forward(4, 2)
    assert e.value.code == pic.PIC_EINVAL
    bad = dataclasses.replace(sp, shells=((-2.0, 0.0, 1.0, 0.0),))
    with pytest.raises(pic.PicError) as e:
        s.add_species(bad, 10)
    assert e.value.code == pic.PIC_EINVAL


@pytest.mark.parametrize("precision", [64, 32])
def test_shells_device_loader_matches_host_loader(pic, precision):
    """The same arrays loaded from host and from device memory give the same
    state (matched by load index: cells, offsets, displacements and
    momenta equal), and the same fields after 8 steps (to rounding: the
    loaders order the particles differently, so the current sums
    differ in order)."""
    _say(f"case: shells device loader fp{precision}")
    import torch
    wl = shell_workload(3, 200, 0, seed=11, K=3, bc=OPEN)
    sp, parts = wl.species[0]
    a = pic.Simulation(wl.grid, precision=precision, flags=pic.TRACK_IDS)
    ia = a.add_species(sp, parts.n)
    a.load_particles(ia, parts)
    b = pic.Simulation(wl.grid, precision=precision, flags=pic.TRACK_IDS)
    ib = b.add_species(sp, parts.n)
    dev = lambda x: torch.tensor(x, dtype=torch.float64, device="cuda")
    b.load_particles_device(ib, dev(parts.x), dev(parts.u1), delta=dev(parts.delta),
                            u2=dev(parts.u2))
    pa, pb = a.particles(ia, ids=True), b.particles(ib, ids=True)
    pa, pb = match_by_id(pa, pa["id"]), match_by_id(pb, pb["id"])
    for k in ("cell", "off", "delta", "u1", "u2"):
        assert np.array_equal(pa[k], pb[k]), k
    a.step(8)
    b.step(8)
    Ea, Ba, _ = a.fields()
    Eb, Bb, _ = b.fields()
    tol = 1e-12 if precision == 64 else 1e-5
    assert rel_l2(Eb, Ea) < tol and rel_l2(Bb, Ba) < tol


def test_multishell_medium_probes_fp64(pic):
    """The two-shell medium of the permittivity pin on the GPU: its E_y
    probes follow the oracle's over the whole run (FP64)."""
    _say("case: multi-shell medium probes")
    wl = multishell_medium_1d()
    o = Oracle.from_workload(wl, max_probe_steps=wl.steps)
    o.step(wl.steps)
    s = pic.Simulation.from_workload(wl, precision=64, max_probe_steps=wl.steps)
    s.step(wl.steps)
    assert s.diagnostics()["error_word"] == 0
    po, pg = o.probes(), s.probes()
    assert pg.shape == po.shape
    assert np.abs(pg - po).max() < 1e-10 * np.abs(po).max()
