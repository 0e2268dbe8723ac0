"""Oracle for the coupled drop / insoluble-surfactant time step (Sec. 3).

Test infrastructure, like the rest of oracle/: plain FP64 numpy on top of the
oracle's own transforms (synth / analyze), surface integral and velocity solve.
Nothing here is used by the product path.

What one step computes (Algorithm 1 with the explicit midpoint rule of the
drop-evolution tableaus and the second-order IMEX scheme of Sec. 3.2):

    u0  = velocity(x0, Gamma0)
    xh  = x0 + dt/2 u0
    Gh  : (I - dt/(2 Pe) L_xh) Gh = Gamma0 + dt/2 fE(x0, u0, Gamma0)
    uh  = velocity(xh, Gh)
    x1  = x0 + dt uh
    G1  = Gamma0 + dt (fE(xh, uh, Gh) + L_xh Gh / Pe)

with fI = L Gamma / Pe (L the Laplace-Beltrami operator of the surface) and
the error estimates of Sec. 3: drop = midpoint against the lower-order row of
the tableau (explicit Euler, x0 + dt u0); surfactant = the local conservation
error of the total surfactant on each drop.  The new step size is
dt (0.9 tol / err)^(1/2) (Algorithm 1).

Readings (each listed in the design doc):
- The algorithm box writes the full step as x^(t+dt/2) + dt u^(t+dt/2); the
  midpoint tableau (weights 0, 1) gives x^t + dt u^(t+dt/2), used here.
- The drop nodes move with the full velocity (dx/dt = u, Sec. 1.2), so the
  surfactant value carried by a node changes by the material rate
  fE = -Gamma div_s u = -div_s(Gamma u_s) - 2 K Gamma (u.n) + u_s . grad_s Gamma.
  The printed fE omits the last term, which belongs to a description whose
  nodes move normally; with nodes moving with u it would not conserve mass,
  while the conservation error of Sec. 3.2 presumes a scheme that does.
- Norms: the drop error is the relative 2-norm of the position coefficients
  of all drops; the surfactant error is the largest relative change of the
  total surfactant over the drops.
- Surface operators are evaluated on the de-aliasing grid of degree U_geom p
  and analysed back to degree p (Sec. 1.3).
"""
from __future__ import annotations

import copy

import numpy as np

from . import System, analyze, ncoef, surface_integral, synth, volume

_DER = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]


def _fields(p, c, q, ders):
    """Grid values of the derivatives `ders` of a (ncomp, ncoef, 2) expansion."""
    c = np.asarray(c, dtype=float)
    if c.ndim == 2:
        c = c[None]
    return {d: np.stack([synth(p, c[k], q, *d) for k in range(c.shape[0])]) for d in ders}


def _metric(X):
    """Inverse metric (g^tt, g^tp, g^pp) and area element W from x_theta, x_phi."""
    xt, xp = X[(1, 0)], X[(0, 1)]
    G = np.sum(xt * xt, axis=0)
    F = np.sum(xt * xp, axis=0)
    E = np.sum(xp * xp, axis=0)
    W2 = E * G - F * F
    return E / W2, -F / W2, G / W2, np.sqrt(W2)


def surface_div(p, xc, uc, q):
    """div_s u on the degree-q grid: g^{ij} x_i . u_j (tangential trace of grad u)."""
    X = _fields(p, xc, q, [(1, 0), (0, 1)])
    U = _fields(p, uc, q, [(1, 0), (0, 1)])
    gtt, gtp, gpp, _ = _metric(X)
    xt, xp, ut, up = X[(1, 0)], X[(0, 1)], U[(1, 0)], U[(0, 1)]
    dot = lambda a, b: np.sum(a * b, axis=0)
    return gtt * dot(xt, ut) + gtp * (dot(xt, up) + dot(xp, ut)) + gpp * dot(xp, up)


def surface_grad(p, xc, gc, q):
    """grad_s g on the degree-q grid, Cartesian components (3, q+1, 2q)."""
    X = _fields(p, xc, q, [(1, 0), (0, 1)])
    Gf = _fields(p, gc, q, [(1, 0), (0, 1)])
    gtt, gtp, gpp, _ = _metric(X)
    gt, gp = Gf[(1, 0)][0], Gf[(0, 1)][0]
    return (gtt * gt + gtp * gp) * X[(1, 0)] + (gtp * gt + gpp * gp) * X[(0, 1)]


def laplace_beltrami(p, xc, gc, q):
    """Laplace-Beltrami of g on the degree-q grid: g^{ij} (g_ij - x_ij . grad_s g),
    the surface Hessian traced with the inverse metric (the Christoffel term is
    the tangential part of the second derivatives of x)."""
    X = _fields(p, xc, q, _DER)
    Gf = _fields(p, gc, q, _DER)
    gtt, gtp, gpp, _ = _metric(X)
    gt, gp = Gf[(1, 0)][0], Gf[(0, 1)][0]
    grad = (gtt * gt + gtp * gp) * X[(1, 0)] + (gtp * gt + gpp * gp) * X[(0, 1)]
    h = lambda d: Gf[d][0] - np.sum(X[d] * grad, axis=0)
    return gtt * h((2, 0)) + 2.0 * gtp * h((1, 1)) + gpp * h((0, 2))


def f_explicit(p, xc, uc, gc, q):
    """Coefficients of fE = -Gamma div_s u (material rate at nodes moving with u)."""
    gam = synth(p, gc, q)
    return analyze(-gam * surface_div(p, xc, uc, q), q, p)


def lb_coef(p, xc, gc, q):
    """Galerkin Laplace-Beltrami: coefficients of L g to degree p."""
    return analyze(laplace_beltrami(p, xc, gc, q), q, p)


def mass(p, xc, gc, q):
    """Total surfactant int Gamma dS by the regular rule on the degree-q grid."""
    return surface_integral(p, xc, q, synth(p, gc, q).ravel())


def imex_solve(p, xc, b, c, q):
    """Solve (I - c L) y = b for y in coefficient space (dense matrix of the
    Galerkin operator, one column per coefficient entry)."""
    n = 2 * ncoef(p)
    A = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = e - c * lb_coef(p, xc, e.reshape(-1, 2), q).ravel()
    return np.linalg.solve(A, np.asarray(b, dtype=float).ravel()).reshape(-1, 2)


def sphere_preconditioner(p, R, c):
    """Diagonal of I - c L on a sphere of radius R: 1 + c n (n + 1) / R^2 (Sec. 3.2.1)."""
    d = np.zeros((ncoef(p), 2))
    for n in range(p + 1):
        for m in range(n + 1):
            d[n * (n + 1) // 2 + m] = 1.0 + c * n * (n + 1) / R ** 2
    return d


def _velocity(sys):
    u, _, _ = sys.solve()
    return u


def time_step(sys: System, dt: float, Pe: float, tol: float, velocity=None):
    """One coupled step from the state held in `sys` (drop coefficients xc and
    surfactant coefficients gc). Returns (new System, report dict); the new
    System holds the stepped state (whether or not the step is accepted)."""
    vel = velocity or _velocity
    q = lambda d: sys.opt.U_geom * d.p
    surf = all(d.gc is not None for d in sys.drops)
    diff = surf and np.isfinite(Pe) and Pe > 0
    x0 = [np.asarray(d.xc, dtype=float) for d in sys.drops]
    g0 = [np.asarray(d.gc, dtype=float) for d in sys.drops] if surf else None
    u0 = vel(sys)
    rep = {}
    # half step
    half = copy.deepcopy(sys)
    half._cache = {}
    fE0, m0 = [], []
    for i, d in enumerate(sys.drops):
        half.drops[i].xc = x0[i] + 0.5 * dt * u0[i]
        if surf:
            fE0.append(f_explicit(d.p, x0[i], u0[i], g0[i], q(d)))
            m0.append(mass(d.p, x0[i], g0[i], q(d)))
            b = g0[i] + 0.5 * dt * fE0[i]
            half.drops[i].gc = imex_solve(d.p, half.drops[i].xc, b, 0.5 * dt / Pe, q(d)) if diff else b
    uh = vel(half)
    # full step
    new = copy.deepcopy(sys)
    new._cache = {}
    m1 = []
    for i, d in enumerate(sys.drops):
        new.drops[i].xc = x0[i] + dt * uh[i]
        if surf:
            xh, gh = half.drops[i].xc, half.drops[i].gc
            kE = f_explicit(d.p, xh, uh[i], gh, q(d))
            kI = lb_coef(d.p, xh, gh, q(d)) / Pe if diff else 0.0
            new.drops[i].gc = g0[i] + dt * (kE + kI)
            m1.append(mass(d.p, new.drops[i].xc, new.drops[i].gc, q(d)))
    x1 = np.concatenate([d.xc.ravel() for d in new.drops])
    xe = np.concatenate([(x0[i] + dt * u0[i]).ravel() for i in range(len(sys.drops))])
    err_drop = float(np.linalg.norm(x1 - xe) / np.linalg.norm(x1))
    err_surf = float(max(abs(b - a) / abs(a) for a, b in zip(m0, m1))) if surf else 0.0
    err = max(err_drop, err_surf)
    accepted = tol <= 0 or err < tol
    dt_next = dt * (0.9 * tol / err) ** 0.5 if (tol > 0 and err > 0) else dt
    rep.update(err_drop=err_drop, err_surf=err_surf, accepted=accepted, dt_next=dt_next,
               mass0=m0, mass1=m1, u0=u0, uh=uh)
    return new, rep


def radius(p, xc):
    """Volume-equivalent radius (3V / 4 pi)^(1/3)."""
    return (3.0 * volume(p, xc, p) / (4.0 * np.pi)) ** (1.0 / 3.0)
