"""Parity of the nearest-region special quadrature (Sec. 2.3) with the oracle.

Both sides take the closest point by damped Newton from the nearest node,
the exterior limit at it from the source drop's self-interaction expansion,
regular-rule values at x* + h sqrt(l) d and Lagrange interpolation; the
tolerance is the FP64 one, per drop and component:
||gpu - oracle||_inf <= 1e-10 ||oracle||_inf.
"""
import numpy as np
import pytest

import workloads as W
from test_parity_gpu import TOL, coef_err, ctx_for, osys, random_coef, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_02156_amd as B
    return B


def close_drops(rng, specs, A=0.05):
    return [W.DropSpec(p, W.perturbed_sphere(rng, p, 1.0, c0, A), lam) for p, c0, lam in specs]


def test_near_rule_single_and_double_layer_three_drops(B, orc):
    """Degrees 8, 10, 9 at gaps well inside h: Omega_2 items from every drop,
    single layer of the force, raw double layer and the Galerkin operator."""
    print("near rule three drops", flush=True)
    rng = np.random.default_rng(71)
    drops = close_drops(rng, [(8, (0, 0, 0), 2.0), (10, (2.1, 0.1, 0), 1.0), (9, (0.6, 2.05, 0.2), 4.0)])
    wl = W.Workload("near3", drops, eos=0, A_tilde=5.0, U_tilde=3)
    c = ctx_for(B, wl, near_rule=1, near_L=8)
    s = osys(orc, wl, near_rule=1, near_L=8)
    reg, _ = c.regions()
    assert (reg == 2).sum() > 10
    u = c.single_layer()
    for i in range(3):
        ref = -s.layer(i, [s.force(j) for j in range(3)], 0) / (8 * np.pi)
        assert rel_err(u[i], ref) <= TOL, i
    us = [random_coef(rng, d.p, 3) for d in drops]
    D = c.double_layer(us, mode=0)
    for i in range(3):
        assert rel_err(D[i], s.layer(i, us, 1) / (4 * np.pi)) <= TOL, i
    A = c.double_layer(us, mode=1)
    ref = s.split(s.matvec(np.concatenate([x.ravel() for x in us])))
    for i in range(3):
        assert coef_err(A[i], ref[i]) <= TOL, i
    c.close()


@pytest.mark.parametrize("L", [4, 8])
def test_near_rule_rigid_motion_of_two_close_spheres(B, L):
    """Constant density, two unit spheres 0.05 apart at p = 12 (about h/5):
    the exterior double layer vanishes, so every target sees 4 pi e from its
    own sphere; the special quadrature holds this to 1e-5, the Omega_1 rule
    does not."""
    print(f"near rule rigid motion L={L}", flush=True)
    p = 12
    drops = [W.DropSpec(p, W.sphere(p, 1.0, (0, 0, 0)), 2.0), W.DropSpec(p, W.sphere(p, 1.0, (2.05, 0, 0)), 2.0)]
    wl = W.Workload("spheres", drops, eos=0, A_tilde=5.0, U_tilde=4)
    e = np.array([0.2, -0.7, 0.4])
    u = np.zeros((3, B.ncoef(p), 2))
    u[:, 0, 0] = e * np.sqrt(4 * np.pi)
    errs = {}
    for rule in (0, 1):
        c = ctx_for(B, wl, near_rule=rule, near_L=L)
        D = c.double_layer([u, u], mode=0)  # sum_j D_j[u] / (4 pi)
        errs[rule] = max(np.abs(D[i] - e).max() for i in range(2))
        c.close()
    assert errs[1] <= 1e-5
    assert errs[0] > 100 * errs[1]


def test_near_rule_velocity_solve_two_close_drops(B, orc):
    """Full velocity solve (lambda 1 and 5, linear EOS) of two p = 10 drops
    about h/3 apart with the special quadrature, against the oracle's solve."""
    print("near rule velocity solve", flush=True)
    rng = np.random.default_rng(72)
    drops = close_drops(rng, [(10, (0, 0, 0), 1.0), (10, (2.09, 0, 0.05), 5.0)])
    for d in drops:
        d.gc = np.zeros((B.ncoef(10), 2))
        d.gc[0, 0] = np.sqrt(4 * np.pi)
        d.gc[W.idx(2, 0), 0] = 0.2
    wl = W.Workload("near2", drops, eos=1, E=0.5, xs=0.6, A_tilde=5.0, U_tilde=4, gmres_tol=1e-12)
    c = ctx_for(B, wl, near_rule=1)
    reg, _ = c.regions()
    assert (reg == 2).any()
    ug, rep = c.eval_velocity(coefficients=True)
    s = osys(orc, wl, near_rule=1)
    uo, _, _ = s.solve(tol=1e-12)
    for i in range(2):
        assert coef_err(ug[i], uo[i]) <= 1e-9, i
    c.close()
