"""Mixed precision (precision = BIM_PREC_MIXED): the direct pair sums in FP32
arithmetic, every other step in FP64.

Bar: 1e-5 of the largest value, per output, against the FP64 oracle on
sampled targets and against the FP64 GPU path on every target (the FP32
pair sums round each pair to about 1e-7 relative; runs of 16 sources are
summed in FP32 and accumulated in FP64). The error is also required to be
above FP64 rounding, so the FP32 kernel is known to have run.
"""
import numpy as np
import pytest

import workloads as W
from test_parity_gpu import ctx_for, osys, random_coef

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_02156_amd as B
    return B


def _density(rng, p):
    c = random_coef(rng, p, 3)
    for n in range(p + 1):
        c[:, n * (n + 1) // 2:(n + 1) * (n + 2) // 2] *= (1.0 + n) ** -2
    return c


def _rel(got, ref):
    return np.abs(np.asarray(got) - np.asarray(ref)).max() / np.abs(ref).max()


def _flat(xs):
    return np.concatenate([np.ravel(x) for x in xs])


def test_mixed_two_drops_against_oracle(B, orc):
    """The two-drop p = 32 workload (gap 0.2: Omega_1 pairs on the upsampled
    grid and Omega_2 targets), sampled targets of both drops."""
    print("mixed: two drops p=32 vs oracle", flush=True)
    wl = W.two_drops()
    rng = np.random.default_rng(61)
    c = ctx_for(B, wl, precision=B.BIM_PREC_MIXED)
    s = osys(orc, wl)
    dens = [_density(rng, 32) for _ in wl.drops]
    u = c.single_layer()
    D = c.double_layer(dens, mode=0)
    forces = [s.force(j) for j in range(2)]
    for i in (0, 1):
        tg = np.sort(rng.choice(B.npts(32), 8, replace=False))
        assert _rel(u[i][tg], -s.layer(i, forces, 0, targets=tg) / (8 * np.pi)) <= TOL32
        assert _rel(D[i][tg], s.layer(i, dens, 1, targets=tg) / (4 * np.pi)) <= TOL32
    c.close()


def test_mixed_many_drops_against_fp64(B):
    """The 64-drop workload, every target, single and double layer."""
    print("mixed: 64 drops vs FP64", flush=True)
    wl = W.many_drops()
    rng = np.random.default_rng(62)
    dens = [_density(rng, 16) for _ in wl.drops]
    res = {}
    for prec in (B.BIM_PREC_FP64, B.BIM_PREC_MIXED):
        c = ctx_for(B, wl, precision=prec)
        res[prec] = (_flat(c.single_layer()), _flat(c.double_layer(dens, mode=0)))
        c.close()
    for k in range(2):
        e = _rel(res[B.BIM_PREC_MIXED][k], res[B.BIM_PREC_FP64][k])
        print("layer", k, "rel err", e, flush=True)
        assert 1e-12 < e <= TOL32


def test_mixed_velocity_solve(B):
    """Full velocity solve of the two-drop workload in both precisions."""
    print("mixed: velocity solve", flush=True)
    wl = W.two_drops()
    out = {}
    for prec in (B.BIM_PREC_FP64, B.BIM_PREC_MIXED):
        c = ctx_for(B, wl, precision=prec)
        u, rep = c.eval_velocity(coefficients=True)
        out[prec] = (_flat(u), rep.gmres_iterations)
        c.close()
    e = _rel(out[B.BIM_PREC_MIXED][0], out[B.BIM_PREC_FP64][0])
    print("solve rel err", e, flush=True)
    assert 1e-12 < e <= TOL32
    assert abs(out[B.BIM_PREC_MIXED][1] - out[B.BIM_PREC_FP64][1]) <= 1


@pytest.mark.parametrize("eps", [1e-12, 1e-8])
def test_mixed_with_fast_summation(B, eps):
    """Mixed precision and the fast summation together (the far pairs by the
    multipole method, the near pairs in FP32), with the truncation bound at
    the FP64 level and at 1e-8 (below the mixed form's 1e-5 bar)."""
    print("mixed + fast summation, eps", eps, flush=True)
    wl = W.many_drops(nd=16, p=12, box=14.0, gap=0.4, seed=46)
    cd = ctx_for(B, wl)
    ud, _ = cd.eval_velocity(coefficients=True)
    cd.close()
    cm = ctx_for(B, wl, precision=B.BIM_PREC_MIXED, fmm_order=24, fmm_eps=eps)
    um, rm = cm.eval_velocity(coefficients=True)
    cm.close()
    assert rm.n_fmm_pairs > 0
    e = _rel(_flat(um), _flat(ud))
    print("rel err", e, flush=True)
    assert e <= TOL32
