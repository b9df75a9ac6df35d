"""Reduced Bragg-scattering case (Sec. 3.2 geometry) and the direction of
its scattered wave, shared by the oracle pin and the GPU comparison."""
import math

import numpy as np

from paper_2208_08038_amd.inputs import bragg_2d


def bragg_case(d_over_lambda, precision=64):
    """512^2 cells of lambda/32, a 256^2-cell region of a square lattice of
    two-body ions (lattice constant d) tilted by the Bragg angle
    asin(lambda / 2d) to a 6-cycle pulse travelling along +x, polarised out
    of the plane, a0 = 1e-4; 700 steps."""
    wl = bragg_2d(cells=512, slab=256, steps=700, d_over_lambda=d_over_lambda, cycles=6,
                  waist_lambda=4.0, a0=1e-4, weight_scale=10.0, precision=precision)
    wl.grid.laser.pol = 2
    return wl


def scattered_direction(wl, ez_scattered):
    """Spatial spectrum of the scattered E_z on the ring |k| ~ omega, away
    from the forward direction: (angle from +x of the strongest lobe, as
    its intensity-weighted centroid in degrees; its mean |k|; its peak over
    the peak of the mirror direction)."""
    n = wl.grid.n[0]
    es = np.asarray(ez_scattered).reshape(n, n)  # [y, x]
    power = np.abs(np.fft.fftshift(np.fft.fft2(es))) ** 2
    k = np.fft.fftshift(np.fft.fftfreq(n, d=wl.grid.dx[0])) * 2 * math.pi
    ky, kx = np.meshgrid(k, k, indexing="ij")
    kr = np.hypot(kx, ky)
    phi = np.degrees(np.arctan2(ky, kx))
    ring = (kr > 0.8) & (kr < 1.2) & (kx > 0) & (np.abs(phi) > 12.0)
    peak = phi.flat[np.argmax(np.where(ring, power, 0.0))]
    lobe = ring & (np.abs(phi - peak) < 12.0)
    w = power[lobe]
    angle = math.degrees(math.atan2((ky[lobe] * w).sum(), (kx[lobe] * w).sum()))
    kmean = (kr[lobe] * w).sum() / w.sum()
    mirror = power[ring & (np.abs(phi + angle) < 6.0)].max()
    return angle, kmean, w.max() / mirror
