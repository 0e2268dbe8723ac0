"""Mixed precision (precision = BIM_PREC_MIXED): the direct pair sums in FP32
arithmetic; the operator's density synthesis and the analyses (operator
output, right-hand side) as FP32 matrix-core contractions with FP32
accumulation; rotation, the singular rule, the single layer's force
density and GMRES in FP64.

Bar: 1e-5 per output, where an output is one drop and one component:
||gpu - ref||_inf / ||ref||_inf over that drop's targets (sampled ones
against the FP64 oracle, all of them against the FP64 GPU path). The FP32
pair sums round each pair to about 1e-7 relative; runs of sources are summed
in FP32 and accumulated in FP64. The error is also required to be above
FP64 rounding, so the FP32 kernel is known to have run. Each test prints
the per-output error it measured.
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


def _rel_out(got, ref):
    """Largest per-drop, per-component relative error; got/ref: per drop,
    arrays (targets, 3) of grid values or (3, ncoef, 2) of coefficients."""
    e = 0.0
    for g, r in zip(got, ref):
        g, r = np.asarray(g), np.asarray(r)
        if g.ndim == 2:
            g, r = g.T, r.T
        for c in range(3):
            e = max(e, float(np.abs(g[c] - r[c]).max() / np.abs(r[c]).max()))
    return e


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
    es, ed = 0.0, 0.0
    for i in (0, 1):
        tg = np.sort(rng.choice(B.npts(32), 8, replace=False))
        es = max(es, _rel_out([u[i][tg]], [-s.layer(i, forces, 0, targets=tg) / (8 * np.pi)]))
        ed = max(ed, _rel_out([D[i][tg]], [s.layer(i, dens, 1, targets=tg) / (4 * np.pi)]))
    print("per-output error SL", es, "DL", ed, flush=True)
    assert 1e-12 < es <= TOL32 and ed <= TOL32
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
        res[prec] = (c.single_layer(), c.double_layer(dens, mode=0))
        c.close()
    for k in range(2):
        e = _rel_out(res[B.BIM_PREC_MIXED][k], res[B.BIM_PREC_FP64][k])
        print("layer", k, "per-output error", e, flush=True)
        assert 1e-12 < e <= TOL32


def test_mixed_two_drops_solve_against_oracle_solution(B, orc):
    """The two-drop p = 32 solve in the mixed form against the oracle's
    stored solution (GMRES 1e-12, written by the oracle only): velocity
    coefficients per drop and component."""
    print("mixed: two drops p=32 solve vs oracle solution", flush=True)
    from test_parity_gpu import GOLDEN_C2
    ref = np.load(GOLDEN_C2)
    wl = W.two_drops()
    c = ctx_for(B, wl, precision=B.BIM_PREC_MIXED)
    uc, rep = c.eval_velocity(coefficients=True)
    c.close()
    uo = osys(orc, wl).split(ref["u"])
    e = _rel_out(uc, uo)
    print("per-output error", e, flush=True)
    assert 1e-12 < e <= TOL32


def test_mixed_many_drops_operator_and_solve_against_fp64(B):
    """The 64-drop workload: the full operator A u in coefficients (FP32
    density synthesis and analysis) and the solved velocity on the grid,
    mixed against FP64, per drop and component. (The error of this velocity
    is set by the FP32 pair sums of the single layer: with the transforms in
    FP64 it is the same to two digits.)"""
    print("mixed: 64 drops operator and solve vs FP64", flush=True)
    wl = W.many_drops()
    rng = np.random.default_rng(63)
    dens = [_density(rng, 16) for _ in wl.drops]
    res = {}
    for prec in (B.BIM_PREC_FP64, B.BIM_PREC_MIXED):
        c = ctx_for(B, wl, precision=prec)
        res[prec] = (c.double_layer(dens, mode=1), c.eval_velocity()[0])
        c.close()
    for k, name in ((0, "operator"), (1, "velocity")):
        e = _rel_out(res[B.BIM_PREC_MIXED][k], res[B.BIM_PREC_FP64][k])
        print(name, "per-output error", e, flush=True)
        assert 1e-12 < e <= TOL32


def test_mixed_velocity_solve(B):
    """Full velocity solve of the two-drop workload in both precisions."""
    print("mixed: velocity solve", flush=True)
    wl = W.two_drops()
    out = {}
    for prec in (B.BIM_PREC_FP64, B.BIM_PREC_MIXED):
        c = ctx_for(B, wl, precision=prec)
        u, rep = c.eval_velocity(coefficients=True)
        out[prec] = (u, rep.gmres_iterations)
        c.close()
    e = _rel_out(out[B.BIM_PREC_MIXED][0], out[B.BIM_PREC_FP64][0])
    print("solve per-output error", e, flush=True)
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
    e = _rel_out(um, ud)
    print("per-output error", e, flush=True)
    assert e <= TOL32


@pytest.fixture(scope="module")
def deformed_both(B):
    """The 16 deformed drops p = 48: single layer, raw double layer of a smooth
    random density and the full velocity solve, in FP64 and mixed."""
    wl = W.deformed_drops()
    rng = np.random.default_rng(57)
    dens = [_density(rng, 48) for _ in wl.drops]
    out = {}
    for prec in (B.BIM_PREC_FP64, B.BIM_PREC_MIXED):
        c = ctx_for(B, wl, precision=prec)
        sl, dl = c.single_layer(), c.double_layer(dens, mode=0)
        u, rep = c.eval_velocity()
        reg, _ = c.regions() if prec == B.BIM_PREC_MIXED else (None, None)
        op = c.double_layer(dens, mode=1)
        out[prec] = (sl, dl, u, rep, reg, op)
        c.close()
    return wl, dens, out


def test_mixed_deformed_drops_every_target_against_fp64(B, deformed_both):
    """Every target of the 16 deformed drops: single layer, double layer, the
    solved velocity and the full operator in coefficients of the mixed form
    against the FP64 form."""
    print("mixed: 16 deformed drops p=48 vs FP64", flush=True)
    wl, dens, out = deformed_both
    m, d = out[B.BIM_PREC_MIXED], out[B.BIM_PREC_FP64]
    for k, name in ((0, "SL"), (1, "DL"), (2, "velocity"), (5, "operator")):
        e = _rel_out(m[k], d[k])
        print(name, "per-output error", e, flush=True)
        assert 1e-12 < e <= TOL32
    assert abs(m[3].gmres_iterations - d[3].gmres_iterations) <= 1


def test_mixed_deformed_drops_sampled_against_oracle(B, orc, deformed_both):
    """Sampled targets of two drops, near their partner (Omega_1) and far:
    the mixed single and double layer against the FP64 oracle."""
    print("mixed: 16 deformed drops p=48 vs oracle, sampled", flush=True)
    wl, dens, out = deformed_both
    sl, dl, _, _, reg, _ = out[B.BIM_PREC_MIXED]
    rng = np.random.default_rng(58)
    s = osys(orc, wl)
    n = B.npts(48)
    forces = [s.force(j) for j in range(len(wl.drops))]
    es, ed = 0.0, 0.0
    for i in (0, 13):
        r = reg[i * n:(i + 1) * n, i ^ 1]
        near, far = np.nonzero(r != 0)[0], np.nonzero(r == 0)[0]
        tg = np.sort(np.concatenate([rng.choice(near, 4, replace=False), rng.choice(far, 4, replace=False)]))
        es = max(es, _rel_out([sl[i][tg]], [-s.layer(i, forces, 0, targets=tg) / (8 * np.pi)]))
        ed = max(ed, _rel_out([dl[i][tg]], [s.layer(i, dens, 1, targets=tg) / (4 * np.pi)]))
    print("per-output error SL", es, "DL", ed, flush=True)
    assert 1e-12 < es <= TOL32 and ed <= TOL32


@pytest.mark.parametrize("which", ["many_drops", "deformed_drops"])
def test_mixed_matrix_core_transforms_at_full_size(B, which):
    """The 64-drop and the 16-deformed-drop workloads with the FP32
    matrix-core transforms forced (xform_path 2; timing may pick the scalar
    ones): the Galerkin operator in coefficients and the solved velocity
    against the FP64 GPU path with scalar transforms (itself held to the
    oracle at 1e-10), per drop and component."""
    print(f"mixed, FP32 matrix-core transforms forced: {which}", flush=True)
    wl = W.many_drops() if which == "many_drops" else W.deformed_drops()
    p = wl.drops[0].p
    rng = np.random.default_rng(64)
    dens = [_density(rng, p) for _ in wl.drops]
    res = {}
    for prec, path in ((B.BIM_PREC_FP64, 1), (B.BIM_PREC_MIXED, 2)):
        c = ctx_for(B, wl, precision=prec, xform_path=path)
        op = c.double_layer(dens, mode=1)
        u, rep = c.eval_velocity()
        assert rep.xform_matrix_cores == (3 if path == 2 else 0)
        res[prec] = (op, u)
        c.close()
    for k, name in ((0, "operator"), (1, "velocity")):
        e = _rel_out(res[B.BIM_PREC_MIXED][k], res[B.BIM_PREC_FP64][k])
        print(name, "per-output error", e, flush=True)
        assert 1e-12 < e <= TOL32
