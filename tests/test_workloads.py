"""Checks of the synthetic input generators against their stated recipes.

The generators build coefficients in closed form; these tests synthesize them
with the oracle and compare with the geometric definition of each shape.
"""
import numpy as np

import workloads as W


def _points(orc, p, xc, q):
    return np.stack([orc.synth(p, xc[k], q).ravel() for k in range(3)], -1)


def test_sphere_coefficients_give_unit_sphere(orc):
    x = _points(orc, 6, W.sphere(6, 1.7, (0.3, -0.2, 1.0)), 6)
    assert np.allclose(np.linalg.norm(x - [0.3, -0.2, 1.0], axis=1), 1.7, atol=1e-14)


def test_p2_spheroid_radius_and_deformation(orc):
    """r = R (1 + eps P_2(cos theta_body)) at every node; eps = 4/9 gives the
    Taylor deformation (L - B)/(L + B) = 0.3."""
    eps, R, p, q = 4.0 / 9.0, 1.3, 8, 12
    x = _points(orc, p, W.p2_spheroid(p, R, eps), q)
    r = np.linalg.norm(x, axis=1)
    u = x[:, 2] / r
    assert np.abs(r - R * (1 + eps * 0.5 * (3 * u ** 2 - 1))).max() < 1e-13
    L, Bm = R * (1 + eps), R * (1 - eps / 2)
    assert abs((L - Bm) / (L + Bm) - 0.3) < 1e-15
    # eps = 0 is the sphere
    assert np.abs(W.p2_spheroid(p, 1.0, 0.0) - W.sphere(p)).max() < 1e-15


def test_rotated_coefficients_rotate_the_surface(orc):
    rng = np.random.default_rng(11)
    Q = W.random_rotation(rng)
    assert np.allclose(Q @ Q.T, np.eye(3), atol=1e-14) and abs(np.linalg.det(Q) - 1) < 1e-14
    p = 6
    xc = W.p2_spheroid(p, 1.0, 0.3) + W.perturbation(rng, p, 0.05)
    a = _points(orc, p, xc, p)
    b = _points(orc, p, W.rotate_coefficients(xc, Q), p)
    assert np.abs(b - a @ Q.T).max() < 1e-14


def test_scalar_field_is_real_and_has_mean(orc):
    rng = np.random.default_rng(3)
    g = W.scalar_field(rng, 10, 0.05, 2.0, 1.0)
    f = orc.synth(10, g, 10)
    assert abs(orc.surface_integral(10, W.sphere(10), 10, f.ravel()) / (4 * np.pi) - 1.0) < 1e-13
    assert np.all(g[[W.idx(n, 0) for n in range(11)], 1] == 0.0)


def test_deformed_drops_pairs_and_gap(orc):
    """One pair at low degree: noise-free surfaces placed 0.1 apart (sampled),
    noisy drops do not overlap, and the pair sits at the lattice origin."""
    wl = W.deformed_drops(npairs=1, p=10, A=0.0)
    a, b = wl.drops
    assert np.allclose(a.centre + b.centre, 0.0)
    pa = _points(orc, 10, a.xc, 40)
    pb = _points(orc, 10, b.xc, 40)
    d = np.sqrt(((pa[:, None, :] - pb[None, :, :]) ** 2).sum(-1)).min()
    assert 0.1 <= d < 0.115
    assert wl.eos == 1 and a.lam == 3.0
