"""GPU: the allocation-free entry point pic_rho_static against pic_rho,
through the C ABI, on two calls in a row (the second on a smaller grid),
with no device allocation during the calls."""
import sys

import numpy as np
import pytest

from _parity import random_workload, small_grid
from paper_2208_08038_amd.inputs import POINT, Particles, Species

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


def _check(pic, sim):
    import torch
    ref = sim.rho()
    live = len(sim.mem.live)
    torch.cuda.synchronize()
    # cumulative count of allocations through torch's caching allocator
    before = torch.cuda.memory_stats()["allocation.all.allocated"]
    got = sim.rho_static()
    assert len(sim.mem.live) == live  # no call to the context's allocator
    assert torch.cuda.memory_stats()["allocation.all.allocated"] == before
    scale = np.abs(ref).max()
    assert scale > 0
    # FP64 atomics add in a varying order: equal to rounding
    assert np.abs(got - ref).max() <= 1e-13 * scale
    return got


@pytest.mark.parametrize("precision", [64, 32])
def test_rho_static_matches_rho_twice(pic, precision):
    _say(f"case: rho_static precision={precision}")
    big = random_workload(3, 3000, 2000, seed=31, shape=(40, 36, 30))
    small = random_workload(2, 500, 300, seed=32, shape=(20, 14))
    a = pic.Simulation.from_workload(big, precision=precision)
    a.step(2)
    _check(pic, a)
    b = pic.Simulation.from_workload(small, precision=precision)
    b.step(3)
    got = _check(pic, b)
    assert got.size == 20 * 14
    # the second call left nothing of the first (larger) one behind
    assert np.array_equal(got, b.rho_static()) or np.abs(got - b.rho()).max() <= \
        1e-13 * np.abs(got).max()


def test_rho_static_refuses_a_grid_beyond_the_array(pic):
    _say("case: rho_static too large")
    g = small_grid(3, (160, 160, 160), (0.3, 0.3, 0.3))
    s = pic.Simulation(g, precision=32)
    s.add_species(Species(POINT, -1.0, 1.0, weight=1.0), 1)
    with pytest.raises(pic.PicError) as e:
        s.rho_static()
    assert e.value.code == pic.PIC_EINVAL
