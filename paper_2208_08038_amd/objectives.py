"""Objective of the gradient run: the pulse transmitted through the probe
plane behind the medium, from the probe series of `inputs.adjoint_slab`
(rows: E_y(x_p, j), B_z(x_p - 1, j), B_z(x_p, j) over the ny points j of the
plane (ny = n_y n_z in 3D, dy the area of one point); one column per step).

    L = E_T / E_ref + phi_T
    E_T   = sum_n sum_j E_y B_z dt dy     (Poynting flux through the plane,
            B_z averaged onto the E_y node)
    phi_T = arg sum_n exp(i omega t_n) sum_j E_y   (phase at the laser frequency)

Works on numpy arrays and on torch tensors (then differentiable by
autograd); the probe series is small, this is not hot-path work.
"""
import math


def transmitted_parts(series, ny, dt, dy=1.0, omega=1.0, t0=0.0):
    """(E_T, Re D, Im D) of a probe series (3 ny rows)."""
    try:
        import torch
        is_torch = isinstance(series, torch.Tensor)
    except ImportError:  # pragma: no cover
        is_torch = False
    ey = series[0:ny]
    bz = 0.5 * (series[ny:2 * ny] + series[2 * ny:3 * ny])
    e_t = (ey * bz).sum() * dt * dy
    nsteps = series.shape[1]
    if is_torch:
        import torch
        t = t0 + (torch.arange(nsteps, dtype=series.dtype, device=series.device) + 1) * dt
        s = ey.sum(dim=0)
        return e_t, (s * torch.cos(omega * t)).sum(), (s * torch.sin(omega * t)).sum()
    import numpy as np
    t = t0 + (np.arange(nsteps) + 1) * dt
    s = ey.sum(axis=0)
    return e_t, float((s * np.cos(omega * t)).sum()), float((s * np.sin(omega * t)).sum())


def transmitted_loss(series, ny, dt, dy=1.0, omega=1.0, e_ref=1.0, t0=0.0):
    """L = E_T / e_ref + phi_T (see the module docstring)."""
    e_t, re, im = transmitted_parts(series, ny, dt, dy, omega, t0)
    try:
        import torch
        if isinstance(series, torch.Tensor):
            return e_t / e_ref + torch.atan2(im, re)
    except ImportError:  # pragma: no cover
        pass
    return float(e_t) / e_ref + math.atan2(im, re)
