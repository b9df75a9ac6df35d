"""GPU tests of the gradient run (adjoint of the step, checkpointed reverse
sweep) through the C ABI.

* Transposes: with no particles and no laser the probes are a linear map
  A of the initial fields, so <w, A x> must equal <A^T w, x> for random
  x, w (exact up to rounding; catches any wrong index, sign or order in
  the transposed Yee, Mur and guard operations).  The probes are also
  linear in the spline coefficients of the laser envelope.
* Particles: adjoint gradients with respect to omega_c, nu, envelope
  coefficients and the initial particle state against central finite
  differences of the FP64 forward (GPU), and against central finite
  differences of the FP64 oracle.
* The autograd bridge (ProbeSeries) with the transmitted-pulse loss.
"""
import math
import sys

import numpy as np
import pytest

import _adjoint as A
from paper_2208_08038_amd.inputs import Laser

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


def _rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("precision", [64, 32])
def test_field_adjoint_is_the_transpose(pic, ndim, precision):
    _say(f"case: field transpose {ndim}D fp{precision}")
    grid = A.vacuum_grid(ndim)
    sim = pic.Simulation(grid, precision=precision, max_probe_steps=64)
    rng = np.random.default_rng(11 + ndim)
    E0 = rng.normal(size=(3, sim.ncell))
    B0 = rng.normal(size=(3, sim.ncell))
    if precision == 32:
        E0, B0 = E0.astype(np.float32).astype(np.float64), B0.astype(np.float32).astype(np.float64)
    sim.load_fields(E0, B0)
    nprobe = 40
    probes = [(int(rng.integers(0, 6)), tuple(int(rng.integers(0, grid.n[d])) for d in range(3)))
              for _ in range(nprobe)]
    sim.set_probes(probes)
    nsteps, K = 25, 6
    sim.grad_forward(nsteps, K)
    y = sim.probes()
    w = rng.normal(size=y.shape)
    g = sim.grad_backward(w, fields=True)
    lhs = float((w * y).sum())
    rhs = float((g["d_E"] * E0).sum() + (g["d_B"] * B0).sum())
    tol = 1e-12 if precision == 64 else 2e-5
    _say(f"<w, A x> = {lhs:.15e}, <A^T w, x> = {rhs:.15e}, rel {_rel(lhs, rhs):.2e}")
    assert _rel(lhs, rhs) < tol
    # the context continues from the end of the run
    d = sim.diagnostics()
    assert d["step"] == nsteps
    sim.close()


@pytest.mark.parametrize("ndim", [1, 2])
def test_envelope_gradient_of_the_linear_probes(pic, ndim):
    """In vacuum the probes are linear in the spline coefficients: the
    adjoint must give sum w * (probes of the unit coefficient k)."""
    _say(f"case: envelope gradient {ndim}D")
    ncoef = 6
    rng = np.random.default_rng(5)
    env = rng.uniform(0.2, 1.0, ncoef)
    t_env = 2.5 * A.TWO_PI
    las = dict(a0=1e-3, omega=1.0, t_env=t_env, pol=1)
    if ndim == 2:
        las.update(waist=4.0, yc=8 * A.TWO_PI / 16.0)
    grid = A.vacuum_grid(ndim, Laser(env=tuple(env), **las))
    probes = [(c, (i, j, 0)) for c in (1, 5) for i in (10, 30) for j in ((3, 9) if ndim == 2 else (0,))]
    nsteps = 70

    def run(e):
        g2 = A.vacuum_grid(ndim, Laser(env=tuple(e), **las))
        s = pic.Simulation(g2, precision=64, max_probe_steps=nsteps)
        s.set_probes(probes)
        s.grad_forward(nsteps, 16)
        return s
    sim = run(env)
    y = sim.probes()
    w = rng.normal(size=y.shape)
    g = sim.grad_backward(w)
    sim.close()
    for k in range(ncoef):
        e1 = np.zeros(ncoef)
        e1[k] = 1.0
        s = run(e1)
        yk = s.probes()
        s.close()
        ref = float((w * yk).sum())
        _say(f"env[{k}]: adjoint {g['d_env'][k]:.12e}, direct {ref:.12e}")
        assert _rel(g["d_env"][k], ref) < 1e-10


def _loss_w(w):
    return lambda series: float((w * series).sum())


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_parameter_gradients_match_finite_differences(pic, ndim):
    """FP64 adjoint against central differences of the FP64 GPU forward:
    omega_c, nu and two envelope coefficients; random cotangent."""
    _say(f"case: parameter FD {ndim}D")
    wl = A.small_case(ndim)
    rng = np.random.default_rng(3)
    sim = pic.Simulation.from_workload(wl, precision=64, max_probe_steps=wl.steps)
    sim.grad_forward(wl.steps, 32)
    y = sim.probes()
    w = rng.normal(size=y.shape)
    g = sim.grad_backward(w)
    sim.close()
    loss = _loss_w(w)
    series = lambda x: A.gpu_series(pic, x)
    sp = wl.species[0][0]
    checks = [
        ("omega_c", g["d_omega_c"][0], lambda v: A.with_params(wl, omega_c=v), sp.omega_c, 1e-4),
        ("nu", g["d_nu"][0], lambda v: A.with_params(wl, nu=v), sp.nu, 1e-3),
    ]
    env = np.array(wl.grid.laser.env)
    for k in (2, 5):
        def make(v, k=k):
            e = env.copy()
            e[k] = v
            return A.with_params(wl, env=e)
        checks.append((f"env[{k}]", g["d_env"][k], make, env[k], 1e-3))
    for name, adj, make, x0, hrel in checks:
        fd = A.richardson_fd(series, loss, make, x0, hrel * max(abs(x0), 1e-3))
        _say(f"{ndim}D {name}: adjoint {adj:.10e}, FD {fd:.10e}, rel {_rel(adj, fd):.2e}")
        assert _rel(adj, fd) < 2e-7, name


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_particle_state_gradient_matches_finite_differences(pic, ndim):
    """Warm ions (both bodies with random momenta) and a softened bond with
    |delta| up to a_c / 3 (anharmonic): the adjoint with respect
    to one ion's initial u1, u2, delta and position against
    Richardson-extrapolated central differences of the FP64 forward."""
    _say(f"case: particle-state FD {ndim}D")
    wl = A.small_case(ndim, a0=3e-3, thermal=2e-3, a_c=0.03)
    sp, parts = wl.species[0]
    rng = np.random.default_rng(9)
    parts = A.with_particles(wl, delta=rng.uniform(-0.01, 0.01, (parts.n, 3))).species[0][1]
    wl = A.with_particles(wl, delta=parts.delta)
    sim = pic.Simulation.from_workload(wl, precision=64, flags=pic.TRACK_IDS,
                                       max_probe_steps=wl.steps)
    sim.grad_forward(wl.steps, 40)
    ids = sim.particles(0, ids=True)["id"]  # the run's storage order
    y = sim.probes()
    w = rng.normal(size=y.shape)
    sim.grad_backward(w)
    gp = sim.grad_particles(0)
    sim.close()
    loss = _loss_w(w)
    series = lambda x: A.gpu_series(pic, x)
    # the ion whose momentum matters most for the probes
    slot = int(np.argmax(np.abs(gp["u1"]).sum(axis=1)))
    pid = int(ids[slot])
    _say(f"ion {pid} (slot {slot})")
    for key, comp, h in (("u1", 0, 1e-6), ("u1", 1, 1e-6), ("u2", 1, 1e-6), ("delta", 1, 2e-7),
                         ("x", 0, 1e-5)):
        arr = {"u1": parts.u1, "u2": parts.u2, "delta": parts.delta, "x": parts.x}[key]

        def make(v, arr=arr, key=key, comp=comp):
            a = np.array(arr, dtype=np.float64, copy=True)
            a[pid, comp] = v
            return A.with_particles(wl, **{key: a})
        fd = A.richardson_fd(series, loss, make, float(arr[pid, comp]), h)
        adj = float(gp[key][slot, comp])
        _say(f"{ndim}D d/d{key}[{comp}]: adjoint {adj:.10e}, FD {fd:.10e}, rel {_rel(adj, fd):.2e}")
        assert _rel(adj, fd) < 2e-6, (key, comp)


@pytest.mark.parametrize("ndim", [1, 3])
def test_particle_state_gradient_relativistic(pic, ndim):
    """Ions drifting across the laser at gamma up to 1.56 (a common
    transverse momentum of 0.5 - 1.2 on both bodies, so that the Jacobian
    of v = u / gamma is far from the identity): the adjoint with respect to
    one ion's initial u1, u2, delta and position against
    Richardson-extrapolated central differences of the FP64 forward."""
    _say(f"case: relativistic particle-state FD {ndim}D")
    wl = A.small_case(ndim, a0=3e-3, thermal=2e-3, a_c=0.03)
    sp, parts = wl.species[0]
    rng = np.random.default_rng(11)
    n = parts.n
    ang = rng.uniform(0.0, 2.0 * math.pi, n)
    mag = rng.uniform(0.5, 1.2, n)
    uc = np.stack([0.02 * rng.normal(size=n), mag * np.cos(ang), mag * np.sin(ang)], 1)
    wl = A.with_particles(wl, u1=parts.u1 + uc, u2=parts.u2 + uc,
                          delta=rng.uniform(-0.01, 0.01, (n, 3)))
    parts = wl.species[0][1]
    sim = pic.Simulation.from_workload(wl, precision=64, flags=pic.TRACK_IDS,
                                       max_probe_steps=wl.steps)
    sim.grad_forward(wl.steps, 40)
    ids = sim.particles(0, ids=True)["id"]
    y = sim.probes()
    w = rng.normal(size=y.shape)
    sim.grad_backward(w)
    gp = sim.grad_particles(0)
    sim.close()
    loss = _loss_w(w)
    series = lambda x: A.gpu_series(pic, x)
    slot = int(np.argmax(np.abs(gp["u1"]).sum(axis=1)))
    pid = int(ids[slot])
    gam = math.sqrt(1.0 + parts.u1[pid] @ parts.u1[pid])
    _say(f"ion {pid} (slot {slot}), gamma {gam:.3f}")
    assert gam > 1.1
    for key, comp, h in (("u1", 0, 1e-6), ("u1", 1, 1e-6), ("u2", 2, 1e-6), ("delta", 1, 2e-7),
                         ("x", 0, 1e-5)):
        arr = {"u1": parts.u1, "u2": parts.u2, "delta": parts.delta, "x": parts.x}[key]

        def make(v, arr=arr, key=key, comp=comp):
            a = np.array(arr, dtype=np.float64, copy=True)
            a[pid, comp] = v
            return A.with_particles(wl, **{key: a})
        fd = A.richardson_fd(series, loss, make, float(arr[pid, comp]), h)
        adj = float(gp[key][slot, comp])
        _say(f"{ndim}D d/d{key}[{comp}]: adjoint {adj:.10e}, FD {fd:.10e}, rel {_rel(adj, fd):.2e}")
        assert _rel(adj, fd) < 2e-6, (key, comp)


@pytest.mark.parametrize("ndim,precision", [(1, 64), (1, 32), (3, 64), (3, 32)])
def test_gradients_against_the_oracle(pic, ndim, precision):
    """The 1D and 3D cases' gradients with respect to omega_c, nu and an
    envelope coefficient, from the library's adjoint (FP64 and FP32),
    against central finite differences of the FP64 oracle."""
    _say(f"case: adjoint vs oracle FD {ndim}D fp{precision}")
    from paper_2208_08038_amd.objectives import transmitted_loss, transmitted_parts
    wl = A.small_case(ndim)
    ny = len(wl.probes) // 3
    dt = wl.grid.dt
    dy = wl.grid.dx[0] ** (ndim - 1)
    e_ref = float(transmitted_parts(A.oracle_series(wl), ny, dt, dy)[0])

    def loss(series):
        return transmitted_loss(series, ny, dt, dy, e_ref=e_ref)
    import torch
    sim = pic.Simulation.from_workload(wl, precision=precision, max_probe_steps=wl.steps)
    sim.grad_forward(wl.steps, 50)
    y = torch.tensor(sim.probes(), requires_grad=True)
    L = transmitted_loss(y, ny, dt, dy, e_ref=e_ref)
    (w,) = torch.autograd.grad(L, y)
    g = sim.grad_backward(w.numpy())
    sim.close()
    sp = wl.species[0][0]
    env = np.array(wl.grid.laser.env)

    def env_k(v, k=3):
        e = env.copy()
        e[k] = v
        return A.with_params(wl, env=e)
    checks = [("omega_c", g["d_omega_c"][0], lambda v: A.with_params(wl, omega_c=v), sp.omega_c, 1e-4),
              ("nu", g["d_nu"][0], lambda v: A.with_params(wl, nu=v), sp.nu, 1e-2),
              ("env[3]", g["d_env"][3], env_k, env[3], 1e-3)]
    tol = 1e-6 if precision == 64 else 1e-4
    for name, adj, make, x0, hrel in checks:
        fd = A.richardson_fd(A.oracle_series, loss, make, x0, hrel * abs(x0))
        _say(f"fp{precision} {name}: adjoint {adj:.10e}, oracle FD {fd:.10e}, rel {_rel(adj, fd):.2e}")
        assert _rel(adj, fd) < tol, name


def test_autograd_bridge(pic):
    """torch.autograd through ProbeSeries and the transmitted-pulse loss
    gives the same gradients as FD of the same composite (2D case)."""
    _say("case: autograd bridge 2D")
    import torch
    from paper_2208_08038_amd.autograd import ProbeSeries
    from paper_2208_08038_amd.objectives import transmitted_loss, transmitted_parts
    wl = A.small_case(2)
    ny = wl.grid.n[1]
    dt, dy = wl.grid.dt, wl.grid.dx[1]

    def builder(omega_c, nu, env):
        w2 = A.with_params(wl, omega_c=omega_c, nu=nu, env=env)
        return pic.Simulation.from_workload(w2, precision=64, max_probe_steps=w2.steps)

    sp = wl.species[0][0]
    wc = torch.tensor(sp.omega_c, dtype=torch.float64, requires_grad=True)
    nu = torch.tensor(sp.nu, dtype=torch.float64, requires_grad=True)
    env = torch.tensor(wl.grid.laser.env, dtype=torch.float64, requires_grad=True)
    series = ProbeSeries.apply(wc, nu, env, builder, wl.steps, 25)
    e_ref = float(transmitted_parts(series.detach(), ny, dt, dy)[0])
    L = transmitted_loss(series, ny, dt, dy, e_ref=e_ref)
    gwc, gnu, genv = torch.autograd.grad(L, (wc, nu, env))

    def loss(s):
        return float(transmitted_loss(s, ny, dt, dy, e_ref=e_ref))
    fd = A.richardson_fd(lambda x: A.gpu_series(pic, x), loss,
                         lambda v: A.with_params(wl, omega_c=v), sp.omega_c, 1e-4 * sp.omega_c)
    _say(f"autograd d/d omega_c {float(gwc):.10e}, FD {fd:.10e}")
    assert _rel(float(gwc), fd) < 2e-6
    e = np.array(wl.grid.laser.env)
    k = 4
    fde = A.richardson_fd(lambda x: A.gpu_series(pic, x), loss,
                          lambda v: A.with_params(wl, env=np.concatenate([e[:k], [v], e[k + 1:]])),
                          e[k], 1e-3 * e[k])
    _say(f"autograd d/d env[{k}] {float(genv[k]):.10e}, FD {fde:.10e}")
    assert _rel(float(genv[k]), fde) < 2e-6
    assert math.isfinite(float(gnu))


def test_gradient_run_errors(pic):
    """Call-order and configuration errors of the gradient run come back as
    error codes, and a failed call leaves the context usable."""
    _say("case: gradient-run errors")
    s = pic.Simulation(A.vacuum_grid(1), precision=64, max_probe_steps=8)
    s.set_probes([(1, (5, 0, 0))])
    with pytest.raises(pic.PicError) as e:  # backward before any forward run
        s.grad_backward(np.zeros((1, 4)))
    assert e.value.code == pic.PIC_ESTATE
    with pytest.raises(pic.PicError) as e:  # no room for 9 more probe records
        s.grad_forward(9, 3)
    assert e.value.code == pic.PIC_EINVAL
    with pytest.raises(pic.PicError) as e:
        s.grad_forward(4, 0)
    assert e.value.code == pic.PIC_EINVAL
    s.grad_forward(4, 2)
    s.step(1)  # the context moved on: the run can no longer be reversed
    with pytest.raises(pic.PicError) as e:
        s.grad_backward(np.zeros((1, 4)))
    assert e.value.code == pic.PIC_ESTATE
    s.grad_forward(2, 1)
    s.load_fields(np.zeros((3, s.ncell)), np.zeros((3, s.ncell)))  # so does a load
    with pytest.raises(pic.PicError) as e:
        s.grad_backward(np.zeros((1, 2)))
    assert e.value.code == pic.PIC_ESTATE
    s.close()
    sf = pic.Simulation(A.vacuum_grid(2), precision=32, flags=pic.FROZEN_FIELDS,
                        max_probe_steps=8)
    with pytest.raises(pic.PicError) as e:
        sf.grad_forward(2, 1)
    assert e.value.code == pic.PIC_EINVAL
    sf.close()


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_gradients_with_free_electrons(pic, ndim):
    """Ions of charge +1 and warm free electrons (the point-particle adjoint
    kernel): parameter gradients and one electron's initial momentum and
    position against Richardson central differences of the FP64 forward."""
    _say(f"case: gradients with free electrons {ndim}D")
    wl = A.with_electrons(A.small_case(ndim, a0=3e-3))
    rng = np.random.default_rng(17)
    sim = pic.Simulation.from_workload(wl, precision=64, flags=pic.TRACK_IDS,
                                       max_probe_steps=wl.steps)
    sim.grad_forward(wl.steps, 40)
    ids = sim.particles(1, ids=True)["id"]
    y = sim.probes()
    w = rng.normal(size=y.shape)
    g = sim.grad_backward(w)
    ge = sim.grad_particles(1)
    sim.close()
    loss = _loss_w(w)
    series = lambda x: A.gpu_series(pic, x)
    sp = wl.species[0][0]
    env = np.array(wl.grid.laser.env)
    checks = [("omega_c", g["d_omega_c"][0], lambda v: A.with_params(wl, omega_c=v), sp.omega_c, 1e-4),
              ("env[4]", g["d_env"][4],
               lambda v: A.with_params(wl, env=np.concatenate([env[:4], [v], env[5:]])), env[4], 1e-3)]
    for name, adj, make, x0, hrel in checks:
        fd = A.richardson_fd(series, loss, make, x0, hrel * abs(x0))
        _say(f"{ndim}D {name}: adjoint {adj:.10e}, FD {fd:.10e}, rel {_rel(adj, fd):.2e}")
        assert _rel(adj, fd) < 2e-7, name
    parts = wl.species[1][1]
    # each derivative on the electron where it matters most (a nearly
    # cancelling derivative is not a fair finite-difference target: the
    # B-spline is only C1 at the knots the electron crosses)
    for key, comp, h in (("u1", 0, 1e-6), ("u1", 1, 1e-6), ("x", 0, 1e-5)):
        slot = int(np.argmax(np.abs(ge[key][:, comp])))
        pid = int(ids[slot])
        arr = {"u1": parts.u1, "x": parts.x}[key]

        def make(v, arr=arr, key=key, comp=comp):
            a = np.array(arr, dtype=np.float64, copy=True)
            a[pid, comp] = v
            return A.with_particles(wl, species=1, **{key: a})
        fd = A.richardson_fd(series, loss, make, float(arr[pid, comp]), h)
        adj = float(ge[key][slot, comp])
        _say(f"{ndim}D electron {pid} d/d{key}[{comp}]: adjoint {adj:.10e}, FD {fd:.10e}, "
             f"rel {_rel(adj, fd):.2e}")
        assert _rel(adj, fd) < 2e-6, (key, comp)


def test_backward_is_repeatable_and_linear(pic):
    """One forward run, three reverse sweeps: the context is restored after
    each, so the gradients are linear in the cotangent and the run can be
    reversed again (2D case with ions, FP64)."""
    _say("case: repeated reverse sweeps")
    wl = A.small_case(2)
    sim = pic.Simulation.from_workload(wl, precision=64, max_probe_steps=wl.steps)
    sim.grad_forward(wl.steps, 32)
    rng = np.random.default_rng(2)
    y = sim.probes()
    w1, w2 = rng.normal(size=y.shape), rng.normal(size=y.shape)
    g1 = sim.grad_backward(w1, fields=True)
    g2 = sim.grad_backward(w2, fields=True)
    g12 = sim.grad_backward(w1 + 2.0 * w2, fields=True)
    for k in ("d_omega_c", "d_nu", "d_env", "d_E", "d_B"):
        ref = g1[k] + 2.0 * g2[k]
        err = np.abs(g12[k] - ref).max() / max(np.abs(ref).max(), 1e-300)
        _say(f"{k}: linearity error {err:.2e}")
        assert err < 1e-11, k
    assert sim.diagnostics()["step"] == wl.steps
    sim.close()
