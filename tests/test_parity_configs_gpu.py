"""Parity at full workload sizes: the 64-drop far-field configuration
(p = 16, every pair on the 2x grid) and the 16 deformed drops (p = 48, close
pairs, full velocity solve), on outputs sampled where the oracle can compute
them one by one, and on properties that hold at any size.

Tolerance (FP64 path): per component, max |gpu - oracle| over the sampled
targets <= 1e-10 max |oracle| over the same targets.
"""
import numpy as np
import pytest

import workloads as W
from test_parity_gpu import TOL, coef_err, ctx_for, osys, random_coef

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_02156_amd as B
    return B


def _check(got, ref):
    scale = np.abs(ref).max(axis=0)
    err = (np.abs(got - ref).max(axis=0) / scale).max()
    assert err <= TOL, err


def _decaying_density(rng, p, nf=3):
    c = random_coef(rng, p, nf)
    for n in range(p + 1):
        c[:, n * (n + 1) // 2:(n + 1) * (n + 2) // 2] *= (1.0 + n) ** -2
    return c


@pytest.fixture(scope="module")
def many(B):
    wl = W.many_drops()
    c = ctx_for(B, wl)
    yield wl, c
    c.close()


def test_many_drops_regions_all_upsampled(B, many):
    """A_tilde = 1e30: every (target, other drop) pair is Omega_1 or Omega_2."""
    print("64 drops regions", flush=True)
    wl, c = many
    reg, dist = c.regions()
    T = reg.shape[0]
    own = np.repeat(np.arange(64), B.npts(16))
    other = np.ones_like(reg, dtype=bool)
    other[np.arange(T), own] = False
    assert np.all(reg[other] >= 1)
    assert np.all(dist[other] > 0)


def test_many_drops_single_and_double_layer_sampled(B, orc, many):
    print("64 drops SL + DL sampled", flush=True)
    wl, c = many
    rng = np.random.default_rng(33)
    s = osys(orc, wl)
    nd = len(wl.drops)
    u = c.single_layer()
    dens = [_decaying_density(rng, 16) for _ in range(nd)]
    D = c.double_layer(dens, mode=0)
    forces = [s.force(j) for j in range(nd)]
    for i in rng.choice(nd, 4, replace=False):
        tg = np.sort(rng.choice(B.npts(16), 12, replace=False))
        _check(u[i][tg], -s.layer(i, forces, 0, targets=tg) / (8 * np.pi))
        _check(D[i][tg], s.layer(i, dens, 1, targets=tg) / (4 * np.pi))


@pytest.fixture(scope="module")
def deformed(B):
    wl = W.deformed_drops()
    c = ctx_for(B, wl)
    yield wl, c
    c.close()


def test_deformed_drops_force_and_regions(B, orc, deformed):
    print("16 deformed drops p=48 force, regions", flush=True)
    wl, c = deformed
    s = osys(orc, wl)
    fg = c.force()
    for i in (0, 7, 15):
        assert coef_err(fg[i], s.force(i)) <= TOL
    reg, dist = c.regions()
    n = B.npts(48)
    for i, j in ((0, 1), (9, 8)):
        r, d = s.regions(i, j)
        assert np.array_equal(reg[i * n:(i + 1) * n, j], r)
        assert np.abs(dist[i * n:(i + 1) * n, j] - d).max() <= 1e-13
    assert (reg == 1).any()


def test_deformed_drops_layers_sampled(B, orc, deformed):
    """Single layer of the interfacial force and raw double layer of a smooth
    random density at targets near the partner drop (Omega_1) and far away."""
    print("16 deformed drops p=48 SL + DL sampled", flush=True)
    wl, c = deformed
    rng = np.random.default_rng(55)
    s = osys(orc, wl)
    nd = len(wl.drops)
    u = c.single_layer()
    dens = [_decaying_density(rng, 48) for _ in range(nd)]
    D = c.double_layer(dens, mode=0)
    reg, _ = c.regions()
    n = B.npts(48)
    forces = [s.force(j) for j in range(nd)]
    for i in (0, 13):
        partner = i ^ 1
        r = reg[i * n:(i + 1) * n, partner]
        near = np.nonzero(r != 0)[0]
        far = np.nonzero(r == 0)[0]
        tg = np.sort(np.concatenate([rng.choice(near, 6, replace=False), rng.choice(far, 6, replace=False)]))
        _check(u[i][tg], -s.layer(i, forces, 0, targets=tg) / (8 * np.pi))
        _check(D[i][tg], s.layer(i, dens, 1, targets=tg) / (4 * np.pi))


def test_deformed_drops_solve_residual(B, deformed):
    """Full velocity solve at p = 48: the returned coefficients satisfy
    A u = P[2 u_inf - S/(4 pi)] to the GMRES tolerance, with A applied by
    the double-layer entry point (mode 1) and the right-hand side assembled
    from the single-layer entry point and the analysis transform (each checked
    against the oracle above and in the transform tests)."""
    print("16 deformed drops p=48 solve", flush=True)
    wl, c = deformed
    uc, rep = c.eval_velocity(coefficients=True)
    assert rep.gmres_residual <= wl.gmres_tol
    Au = c.double_layer(uc, mode=1)
    sl = c.single_layer()
    b = []
    for i, p in enumerate(c.ps):
        g = np.ascontiguousarray((2.0 * sl[i]).T.reshape(-1))
        out = np.zeros(3 * 2 * B.ncoef(p))
        B.bim_sh_analyze(c.h, p, p, 3, g, out)
        b.append(out.reshape(3, -1, 2))
    r = np.concatenate([(a - bb).ravel() for a, bb in zip(Au, b)])
    bn = np.linalg.norm(np.concatenate([bb.ravel() for bb in b]))
    assert np.linalg.norm(r) <= 2 * wl.gmres_tol * bn
