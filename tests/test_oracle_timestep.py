"""Pins of the oracle's drop / surfactant time step (Sec. 3, Algorithm 1).

Each pin is fixed by the mathematics, not by retyping the oracle:
- spherical harmonics are Laplace-Beltrami eigenfunctions on a sphere,
  L Y_n^m = -n(n+1)/R^2 Y_n^m (Sec. 3.2.1);
- the Laplace-Beltrami of any field integrates to zero over a closed surface;
- div_s x = 2 (trace of the tangential projector) and div_s(Omega x x) = 0;
- the surface gradient of a linear function a.x is the tangential part of a;
- the IMEX stage system on a sphere is the diagonal preconditioner itself;
- one step of a uniformly expanding sphere has a closed form (midpoint and
  IMEX stages written out by hand), including both error estimates;
- the midpoint rule is second order in a linear flow (exact solution by the
  matrix exponential);
- the scheme's conservation error is third order in dt (a description whose
  nodes carry the printed fE would be first order).
"""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O
import workloads as W
from oracle import timestep as T

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _scalar(rng, p, A=0.3, mean=1.0):
    return W.scalar_field(rng, p, A, 1.0, mean)


def _deg(p):
    n = np.zeros((O.ncoef(p), 2))
    for l in range(p + 1):
        for m in range(l + 1):
            n[l * (l + 1) // 2 + m] = l
    return n


def test_laplace_beltrami_sphere_eigenfunctions():
    p, R = 7, 1.3
    xc = W.sphere(p, R, (0.2, -0.1, 0.3))
    g = _scalar(np.random.default_rng(1), p)
    n = _deg(p)
    lg = T.lb_coef(p, xc, g, 2 * p)
    ref = -n * (n + 1) / R ** 2 * g
    assert np.abs(lg - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("q_factor,tol", [(2, 1e-9), (4, 1e-13)])
def test_laplace_beltrami_integrates_to_zero(q_factor, tol):
    rng = np.random.default_rng(7)
    p = 8
    xc = W.perturbed_sphere(rng, p, 1.0, (0.1, -0.2, 0.05), 0.05)
    g = _scalar(rng, p)
    q = q_factor * p
    lg = T.laplace_beltrami(p, xc, g, q)
    I = O.surface_integral(p, xc, q, lg.ravel())
    Ia = O.surface_integral(p, xc, q, np.abs(lg).ravel())
    assert abs(I) <= tol * Ia


def test_surface_divergence_of_position_and_rotation():
    rng = np.random.default_rng(8)
    p = 9
    xc = W.perturbed_sphere(rng, p, 1.1, (0.0, 0.3, -0.2), 0.08)
    assert np.abs(T.surface_div(p, xc, xc, 2 * p) - 2.0).max() <= 1e-12
    Om = np.array([0.3, -0.7, 0.5])
    uc = np.stack([Om[1] * xc[2] - Om[2] * xc[1], Om[2] * xc[0] - Om[0] * xc[2], Om[0] * xc[1] - Om[1] * xc[0]])
    assert np.abs(T.surface_div(p, xc, uc, 2 * p)).max() <= 1e-12


def test_surface_gradient_of_linear_function():
    rng = np.random.default_rng(9)
    p = 8
    xc = W.perturbed_sphere(rng, p, 1.0, (0.1, 0.1, 0.1), 0.06)
    a = np.array([0.4, -1.1, 0.7])
    gc = a[0] * xc[0] + a[1] * xc[1] + a[2] * xc[2]
    q = 2 * p
    grad = T.surface_grad(p, xc, gc, q)
    x, nrm, Wd, K = O.geometry(p, xc, q)
    an = a @ nrm
    ref = a[:, None] - an[None, :] * nrm
    assert np.abs(grad.reshape(3, -1) - ref).max() <= 1e-12


def test_imex_stage_on_sphere_is_the_preconditioner():
    p, R, c = 6, 0.8, 0.05
    xc = W.sphere(p, R)
    b = _scalar(np.random.default_rng(3), p)
    y = T.imex_solve(p, xc, b, c, 2 * p)
    assert np.abs(y - b / T.sphere_preconditioner(p, R, c)).max() <= 1e-13 * np.abs(b).max()


def test_uniform_expansion_step_closed_form():
    """u = a x on a sphere centred at 0 with uniform surfactant: every stage by hand."""
    p, a, dt, R0, G0 = 4, 0.3, 0.1, 1.0, 1.7
    xc = W.sphere(p, R0)
    gc = np.zeros((O.ncoef(p), 2))
    gc[0, 0] = np.sqrt(4 * np.pi) * G0
    sys = O.System([O.Drop(p, xc, 1.0, gc=gc)])
    new, rep = T.time_step(sys, dt, Pe=10.0, tol=1e-3, velocity=lambda s: [a * d.xc for d in s.drops])
    sx = 1 + a * dt + (a * dt) ** 2 / 2          # midpoint: x0 + dt a (x0 + dt/2 a x0)
    sg = 1 - 2 * a * dt + 2 * (a * dt) ** 2      # Gamma0 + dt (-2a) Gamma0 (1 - a dt)
    assert np.abs(new.drops[0].xc - sx * xc).max() <= 1e-13
    assert np.abs(new.drops[0].gc - sg * gc).max() <= 1e-12 * G0
    assert rep["err_drop"] == pytest.approx(((a * dt) ** 2 / 2) / sx, rel=1e-12)
    assert rep["err_surf"] == pytest.approx(abs(sx ** 2 * sg - 1.0), rel=1e-9)
    err = max(rep["err_drop"], rep["err_surf"])
    assert rep["dt_next"] == pytest.approx(dt * (0.9e-3 / err) ** 0.5, rel=1e-12)
    assert rep["accepted"] == (err < 1e-3)


def _linear_flow_step(p, G, xc, dt, nsteps, gc=None, Pe=np.inf):
    sys = O.System([O.Drop(p, xc, 1.0, gc=gc)])
    vel = lambda s: [np.einsum("cd,d...->c...", G, d.xc) for d in s.drops]
    reps = []
    for _ in range(nsteps):
        sys, rep = T.time_step(sys, dt, Pe=Pe, tol=0.0, velocity=vel)
        reps.append(rep)
    return sys, reps


def test_midpoint_rule_is_second_order_in_a_linear_flow():
    rng = np.random.default_rng(11)
    p = 6
    xc = W.perturbed_sphere(rng, p, 1.0, (0.2, 0.0, -0.1), 0.05)
    G = np.array([[0.5, 0.3, 0.0], [-0.2, -0.25, 0.1], [0.0, 0.4, -0.25]])
    Tend = 0.4
    exact = np.einsum("cd,d...->c...", expm(G * Tend), xc)
    errs = []
    for n in (4, 8, 16):
        sys, _ = _linear_flow_step(p, G, xc, Tend / n, n)
        errs.append(np.abs(sys.drops[0].xc - exact).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


def test_conservation_error_is_third_order():
    rng = np.random.default_rng(12)
    p = 6
    xc = W.perturbed_sphere(rng, p, 1.0, (0.0, 0.0, 0.0), 0.05)
    gc = _scalar(rng, p, A=0.2, mean=1.0)
    G = np.array([[0.6, 0.2, 0.0], [0.0, -0.3, 0.3], [0.1, 0.0, -0.3]])
    errs = []
    for dt in (0.08, 0.04):
        _, reps = _linear_flow_step(p, G, xc, dt, 1, gc=gc, Pe=5.0)
        errs.append(reps[0]["err_surf"])
    assert 6.5 < errs[0] / errs[1] < 9.5, errs
