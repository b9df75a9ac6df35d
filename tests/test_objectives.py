"""The transmitted-pulse objective of the gradient runs on closed-form
series (CPU): the phase of a pure sinusoid, the Poynting flux of a plane
wave, and numpy / torch agreement."""
import math

import numpy as np

from paper_2208_08038_amd.objectives import transmitted_loss, transmitted_parts


def _series(ny, nsteps, dt, phi0, amp=1.0):
    t = (np.arange(nsteps) + 1) * dt
    ey = amp * np.cos(t + phi0)
    rows = np.concatenate([np.tile(ey, (ny, 1)), np.tile(ey, (ny, 1)), np.tile(ey, (ny, 1))])
    return rows, t


def test_phase_and_flux_of_a_sinusoid():
    ny, dt = 3, 2 * math.pi / 40
    nsteps = 400  # ten periods exactly
    s, t = _series(ny, nsteps, dt, 0.7, amp=2.0)
    e_t, re, im = transmitted_parts(s, ny, dt, dy=0.5)
    # E_y B_z = 4 cos^2: mean 2 over whole periods
    assert abs(e_t - 2.0 * nsteps * dt * ny * 0.5) < 1e-9
    # sum_n exp(i t_n) cos(t_n + phi0) = N/2 exp(-i phi0) over whole periods
    assert abs(math.atan2(im, re) + 0.7) < 1e-12
    assert abs(transmitted_loss(s, ny, dt, dy=0.5, e_ref=e_t) - (1.0 - 0.7)) < 1e-12


def test_numpy_and_torch_agree():
    import torch
    rng = np.random.default_rng(1)
    s = rng.normal(size=(6, 50))
    a = transmitted_loss(s, 2, 0.1, dy=0.3, e_ref=0.7)
    b = transmitted_loss(torch.tensor(s), 2, 0.1, dy=0.3, e_ref=0.7)
    assert abs(a - float(b)) < 1e-12
