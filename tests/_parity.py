"""Helpers shared by the GPU parity tests: build the same seeded workload in
the oracle and in the HIP library, advance both, and compare."""
import math

import numpy as np

from paper_2208_08038_amd.inputs import (OPEN, PERIODIC, POINT, TWO_BODY, Grid, Particles,
                                         Species, Workload)


def rel_l2(a, b):
    a = np.asarray(a, float).ravel()
    b = np.asarray(b, float).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def small_grid(ndim, shape, dx, cfl_frac=0.9, bc=PERIODIC, laser=None, re_norm=1e-3):
    n3 = tuple(list(shape) + [1] * (3 - ndim))
    dx3 = tuple(list(dx) + [1.0] * (3 - ndim))
    bcs = tuple([bc] * ndim + [PERIODIC] * (3 - ndim))
    cfl = 1.0 / math.sqrt(sum(1.0 / d ** 2 for d in dx))
    g = Grid(ndim, n3, dx3, cfl_frac * cfl, bcs, bcs, re_norm=re_norm)
    if laser is not None:
        g.laser = laser
    return g


def random_workload(ndim, n_ion, n_el, seed, shape=None, dx=None, bc=PERIODIC, vmax_ion=0.3,
                    vmax_el=0.9, per_particle=True, nu=0.05, harmonic=False, weight=0.005):
    """Random two-body ions and free electrons in a small box (parity cases)."""
    rng = np.random.default_rng(seed)
    shape = shape or (23, 17, 13)[:ndim]
    dx = dx or (0.3, 0.25, 0.2)[:ndim]
    g = small_grid(ndim, shape, dx, bc=bc)
    pad = g.pad if bc == OPEN else 0
    species = []

    def pos(n, margin=0.0):
        lo = np.array([pad + margin] * ndim, float)
        hi = np.array([s - pad - margin for s in shape], float)
        return (lo + (hi - lo) * rng.random((n, ndim))) * np.array(dx)

    def mom(n, vmax):
        u = rng.normal(size=(n, 3))
        u *= (vmax / np.linalg.norm(u, axis=1))[:, None] * rng.random((n, 1))
        return u / np.sqrt(1 - np.sum(u * u, axis=1))[:, None]

    if n_ion:
        sp = Species(TWO_BODY, 5.0, 40.0, -3.0, 3.0, weight=weight, omega_c=2.0,
                     a_c=math.inf if harmonic else 0.0, nu=nu, name="ion")
        u = mom(n_ion, vmax_ion)
        # both bodies between the walls: the cloud sits up to 0.1 cell off the centre
        parts = Particles(x=pos(n_ion, 0.15 if bc == OPEN else 0.0), u1=u,
                          u2=u + rng.normal(scale=1e-3, size=u.shape),
                          delta=rng.uniform(-0.1, 0.1, (n_ion, 3)) * min(dx),
                          omega_c=rng.uniform(1.0, 3.0, n_ion) if per_particle else None,
                          weight=rng.uniform(0.5, 1.5, n_ion) * weight if per_particle else None)
        species.append((sp, parts))
    if n_el:
        sp = Species(POINT, -1.0, 1.0, weight=weight, name="e")
        species.append((sp, Particles(x=pos(n_el), u1=mom(n_el, vmax_el))))
    return Workload(f"random{ndim}d", g, species, steps=1, precision=64)


def random_fields(rng, ncell, e=0.05, b=0.05):
    return rng.normal(size=(3, ncell)) * e, rng.normal(size=(3, ncell)) * b


def match_by_id(state, ids):
    """Reorder a GPU particle state (device order) into load order."""
    order = np.argsort(ids, kind="stable")
    return {k: v[order] for k, v in state.items() if k != "id"}
