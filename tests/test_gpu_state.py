"""GPU: checkpoint and restart through the C ABI (pic_save_state /
pic_load_state).  Run K steps, save, destroy, create a new context, load,
run N - K more: the result equals N steps in one run, bit for bit where the
run itself is reproducible (FP32: the fixed-point current patch with every
particle in its tile), to rounding otherwise (FP64 LDS and global atomics
add in a varying order; two uninterrupted FP64 runs differ as much)."""
import dataclasses
import math
import sys

import numpy as np
import pytest

from _parity import random_workload, small_grid
from paper_2208_08038_amd.inputs import (LASER, OPEN, PERIODIC, Laser, neutral_medium_1d)

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


def _laser_workload(ndim, seed):
    """Random ions (own omega_c and weights) and electrons between walls,
    open x faces with a laser entering at x-min (so the Mur history is part
    of the state)."""
    wl = random_workload(ndim, 400, 400, seed=seed, bc=OPEN)
    g = wl.grid
    lo = (LASER,) + tuple(g.bc_lo[1:])
    las = Laser(a0=0.05, omega=1.0, t_env=4 * math.pi, waist=0.0, pol=1)
    g = dataclasses.replace(g, bc_lo=lo, laser=las)
    return dataclasses.replace(wl, grid=g)


def _state(sim):
    E, B, J = sim.fields()
    parts = [sim.particles(k, ids=True) for k in range(len(sim.species))]
    return E, B, J, parts


def _run(pic, wl, precision, steps, **kw):
    s = pic.Simulation.from_workload(wl, precision=precision, flags=pic.TRACK_IDS, **kw)
    s.step(steps)
    return s


def _restart(pic, wl, precision, k, n, **kw):
    a = _run(pic, wl, precision, k, **kw)
    buf = a.save_state()
    before = _state(a)
    a.close()
    b = pic.Simulation(wl.grid, precision=precision, flags=pic.TRACK_IDS, **kw)
    for sp, parts in wl.species:
        b.add_species(sp, parts.n)
    b.load_state(buf)
    after = _state(b)
    # the restored state reads back exactly as saved, and saves identically
    for x, y in zip(before[:3], after[:3]):
        assert np.array_equal(x, y)
    for p, q in zip(before[3], after[3]):
        for key in p:
            assert np.array_equal(p[key], q[key]), key
    assert np.array_equal(b.save_state(), buf)
    b.step(n - k)
    return b


def _max_rel(x, y):
    return np.abs(x - y).max() / max(np.abs(y).max(), 1e-300)


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_restart_fp32_bit_identical(pic, ndim):
    """FP32 with a sort before every step (every particle in its tile, so
    the fixed-point current patch makes the run reproducible): the restarted
    run equals the uninterrupted one bit for bit."""
    _say(f"case: restart fp32 ndim={ndim}")
    wl = _laser_workload(ndim, 500 + ndim)
    a = _run(pic, wl, 32, 14, sort_every=1)
    b = _restart(pic, wl, 32, 6, 14, sort_every=1)
    assert a.diagnostics()["n_outside_tile"] == 0
    sa, sb = _state(a), _state(b)
    for x, y in zip(sa[:3], sb[:3]):
        assert np.array_equal(x, y)
    for p, q in zip(sa[3], sb[3]):
        for key in p:
            assert np.array_equal(p[key], q[key]), key
    assert a.diagnostics()["step"] == b.diagnostics()["step"] == 14


@pytest.mark.parametrize("ndim", [2, 3])
def test_restart_fp64_to_rounding(pic, ndim):
    """FP64 with the adaptive sort: the restarted run agrees with the
    uninterrupted one to FP64 rounding (cells bit-exact), as closely as two
    uninterrupted runs agree with each other."""
    _say(f"case: restart fp64 ndim={ndim}")
    wl = _laser_workload(ndim, 600 + ndim)
    a = _run(pic, wl, 64, 16)
    a2 = _run(pic, wl, 64, 16)
    b = _restart(pic, wl, 64, 7, 16)
    sa, sa2, sb = _state(a), _state(a2), _state(b)
    for i in range(3):
        assert _max_rel(sb[i], sa[i]) < 1e-13
    for p, q in zip(sa[3], sb[3]):
        assert np.array_equal(p["cell"], q["cell"])
        assert np.array_equal(p["id"], q["id"])
        for key in ("off", "u1", "u2", "delta"):
            assert _max_rel(q[key], p[key]) < 1e-13, key
    assert _max_rel(sa2[0], sa[0]) < 1e-13


def test_restart_neutral_medium_probes(pic):
    """The Sec. 3.1 medium (laser through the open x-min face, 1D FP64):
    200 + 200 steps through a restart give the fields of 400 steps."""
    _say("case: restart neutral medium")
    wl = neutral_medium_1d(cells=512, steps=400)
    a = _run(pic, wl, 64, 400)
    b = _restart(pic, wl, 64, 200, 400)
    Ea, Ba, _, _ = _state(a)
    Eb, Bb, _, _ = _state(b)
    assert _max_rel(Eb, Ea) < 1e-13 and _max_rel(Bb, Ba) < 1e-13
    assert np.abs(Ea).max() > 1e-4  # the pulse is in the box


def test_load_state_refuses_a_different_context(pic):
    """A state goes back only into a context of the same grid, precision,
    flags and species."""
    _say("case: load_state refusals")
    wl = random_workload(2, 50, 50, seed=7)
    a = _run(pic, wl, 64, 2)
    buf = a.save_state()
    other = dataclasses.replace(wl.grid, n=(wl.grid.n[0] + 1,) + tuple(wl.grid.n[1:]))
    b = pic.Simulation(other, precision=64, flags=pic.TRACK_IDS)
    for sp, parts in wl.species:
        b.add_species(sp, parts.n)
    with pytest.raises(pic.PicError) as e:
        b.load_state(buf)
    assert e.value.code == pic.PIC_EINVAL
    c = pic.Simulation(wl.grid, precision=32, flags=pic.TRACK_IDS)
    with pytest.raises(pic.PicError) as e:
        c.load_state(buf)
    assert e.value.code == pic.PIC_EINVAL
    d = pic.Simulation(wl.grid, precision=64, flags=pic.TRACK_IDS)
    for sp, parts in wl.species:
        d.add_species(sp, 10)  # capacity below the state's
    with pytest.raises(pic.PicError) as e:
        d.load_state(buf)
    assert e.value.code == pic.PIC_ENOMEM
    with pytest.raises(pic.PicError) as e:
        a.load_state(buf[:-8])
    assert e.value.code == pic.PIC_EINVAL
