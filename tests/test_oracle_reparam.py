"""Pins of the oracle's angle reparametrization (Sec. 4, Algorithm 2).

Fixed by the method, not by retyping it:
- the standard grid on a sphere is a fixed point (only degree-1 modes, so the
  filtered gradient vanishes);
- the nodes move along the surface: a surfactant that is a linear function of
  the position, Gamma = c + a.x, stays exactly that function of the new
  nodes (both are evaluations of the same initial expansions at the same
  angles), and the enclosed volume is kept to spectral accuracy;
- a small pseudo-time step moves each node by dtau w to first order
  (w = -(I - n n) grad E), which pins the 2x2 solve for the angle velocities
  and its signs;
- the filtered residual max |g| decreases under the iteration.
"""
import numpy as np

import oracle as O
import workloads as W
from oracle import reparam as RP


def twisted_sphere(p, beta, a, R=1.0, c=(0.0, 0.0, 0.0)):
    """Degree-p expansion of a sphere with a distorted parametrization:
    theta -> theta + a sin 2 theta, phi -> phi + beta cos theta."""
    th, ph = RP.grid_angles(p)
    th2 = th + a * np.sin(2 * th)
    ph2 = ph + beta * np.cos(th)
    X = np.stack([R * np.sin(th2) * np.cos(ph2) + c[0], R * np.sin(th2) * np.sin(ph2) + c[1],
                  R * np.cos(th2) + c[2]])
    return np.stack([O.analyze(X[k].reshape(p + 1, 2 * p), p, p) for k in range(3)])


def linear_gamma(xc, a, c0):
    g = a[0] * xc[0] + a[1] * xc[1] + a[2] * xc[2]
    g[0, 0] += np.sqrt(4 * np.pi) * c0
    return g


def test_standard_sphere_is_a_fixed_point():
    p = 8
    xc = W.sphere(p, 1.3, (0.1, 0.2, -0.3))
    gc = linear_gamma(xc, (0.2, -0.1, 0.4), 1.0)
    xn, gn, rep = RP.reparametrize(p, xc, gc, U_rep=2, P_cut=1e-3, imax=5)
    assert rep["gnorm"][0] <= 1e-13
    assert np.abs(xn - xc).max() <= 1e-13
    assert np.abs(gn - gc).max() <= 1e-13


def test_linear_surfactant_follows_the_nodes_and_volume_is_kept():
    p = 10
    xc = twisted_sphere(p, 0.4, 0.15, 1.1, (0.2, 0.0, 0.1))
    a, c0 = np.array([0.3, -0.2, 0.5]), 1.0
    gc = linear_gamma(xc, a, c0)
    xn, gn, rep = RP.reparametrize(p, xc, gc, U_rep=2, P_cut=1e-3, imax=12)
    assert rep["moves"] == 11
    assert np.abs(gn - linear_gamma(xn, a, c0)).max() <= 1e-12
    V0, V1 = O.volume(p, xc), O.volume(p, xn)
    assert abs(V1 / V0 - 1.0) <= 1e-9       # truncation from degree U_rep p back to p sets the level
    assert rep["gnorm"][-1] < 0.05 * rep["gnorm"][0]


def test_small_pseudo_step_moves_nodes_by_w():
    p = 8
    xc = twisted_sphere(p, 0.3, 0.1)
    q = 2 * p
    x0 = RP.pad(xc, p, q)
    th, ph = RP.grid_angles(q)
    X, Xt, Xp = RP._eval(q, x0, th, ph)
    _, _, g = RP._gradient(q, X, Xt, Xp, 1e-3)
    dtau = 1e-6
    _, _, rep = RP.reparametrize(p, xc, None, U_rep=2, P_cut=1e-3, imax=2, dtau=dtau)
    X1 = rep["x_nodes"]
    dx = (X1 - X) / dtau
    assert np.abs(dx - (-g)).max() <= 1e-4 * np.abs(g).max()


def test_ncutoff_rule():
    p = 6
    xc = W.sphere(p)
    assert RP.ncutoff(p, xc, 1e-3) == 2          # only degree 1: N2(2) = 0
    xd = xc.copy()
    xd[0, 5 * 6 // 2 + 2, 0] = 1e-2              # a degree-5 mode
    N1 = sum(np.sqrt(np.sum(xd[:, e, :] ** 2)) * (1 if m == 0 else 2)
             for n in range(1, p + 1) for m in range(n + 1) for e in [n * (n + 1) // 2 + m])
    frac = 2 * 1e-2 / N1
    assert RP.ncutoff(p, xd, frac * 1.01) == 2
    assert RP.ncutoff(p, xd, frac * 0.99) == 6
