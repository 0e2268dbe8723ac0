"""Matrix-core transforms of value fields (Sec. 1.1 synthesis, Sec. 2.1
analysis): the Legendre and Fourier sums as batched 16x16x4 contractions.

FP64 (plain context): 1e-10 of the field's largest value (synthesis) or
largest coefficient (analysis) against the FP64 oracle. FP32 (mixed
context: FP32 operands and accumulation): the same per-field measure at most
1e-5 and above 1e-12 (so the FP32 kernels are known to have run). Sizes cover
ragged tiles in every dimension: degrees and grids that are not multiples of
the 16-row and 4-deep tiles, odd q, field counts above one 16-field tile,
and the largest degree and grid the kernels take (p = 63; analysis q = 63).
Each test prints the error it measured.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-5


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_02156_amd as B
    return B


def _coef(rng, p, nf):
    c = rng.standard_normal((nf, (p + 1) * (p + 2) // 2, 2))
    c[..., [n * (n + 1) // 2 for n in range(p + 1)], 1] = 0.0   # m = 0: real
    return c


def _synth(B, orc, prec, p, q, nf, seed):
    rng = np.random.default_rng(seed)
    coef = _coef(rng, p, nf)
    c = B.Context(precision=prec)
    g = np.zeros(nf * B.npts(q))
    B.bim_sh_synthesize(c.h, p, q, nf, np.ascontiguousarray(coef.reshape(-1)), 0, 0, g)
    c.close()
    g = g.reshape(nf, -1)
    e = 0.0
    for f in range(nf):
        ref = orc.synth(p, coef[f], q, 0, 0).ravel()
        e = max(e, float(np.abs(g[f] - ref).max() / np.abs(ref).max()))
    return e


def _anal(B, orc, prec, q, p, nf, seed):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((nf, B.npts(q)))
    c = B.Context(precision=prec)
    out = np.zeros(nf * 2 * B.ncoef(p))
    B.bim_sh_analyze(c.h, q, p, nf, np.ascontiguousarray(g.reshape(-1)), out)
    c.close()
    out = out.reshape(nf, -1, 2)
    e = 0.0
    for f in range(nf):
        ref = orc.analyze(g[f], q, p)
        e = max(e, float(np.abs(out[f] - ref).max() / np.abs(ref).max()))
    return e


SYN = [(0, 1, 1), (1, 1, 2), (5, 5, 3), (17, 17, 5), (13, 39, 17), (31, 62, 6), (40, 120, 3), (63, 63, 2),
       (63, 126, 1)]
ANA = [(1, 1, 2), (5, 5, 3), (17, 17, 17), (33, 20, 5), (45, 30, 2), (63, 63, 3)]


@pytest.mark.parametrize("p,q,nf", SYN)
def test_synthesis_fp64(B, orc, p, q, nf):
    e = _synth(B, orc, B.BIM_PREC_FP64, p, q, nf, 300 + p + q + nf)
    print(f"synthesis FP64 p={p} q={q} nf={nf}: {e:.2e}", flush=True)
    assert e <= TOL64


@pytest.mark.parametrize("q,p,nf", ANA)
def test_analysis_fp64(B, orc, q, p, nf):
    e = _anal(B, orc, B.BIM_PREC_FP64, q, p, nf, 400 + p + q + nf)
    print(f"analysis FP64 q={q} p={p} nf={nf}: {e:.2e}", flush=True)
    assert e <= TOL64


@pytest.mark.parametrize("p,q,nf", SYN[2:])
def test_synthesis_fp32(B, orc, p, q, nf):
    e = _synth(B, orc, B.BIM_PREC_MIXED, p, q, nf, 500 + p + q + nf)
    print(f"synthesis FP32 p={p} q={q} nf={nf}: {e:.2e}", flush=True)
    assert 1e-12 < e <= TOL32


@pytest.mark.parametrize("q,p,nf", ANA[1:])
def test_analysis_fp32(B, orc, q, p, nf):
    e = _anal(B, orc, B.BIM_PREC_MIXED, q, p, nf, 600 + p + q + nf)
    print(f"analysis FP32 q={q} p={p} nf={nf}: {e:.2e}", flush=True)
    assert 1e-12 < e <= TOL32


def test_round_trip_fp64(B):
    """Synthesis then analysis on the same degree-p grid returns the
    coefficients (Im at m = q kept zero: the grid cannot hold it)."""
    p, nf = 29, 4
    rng = np.random.default_rng(77)
    coef = _coef(rng, p, nf)
    coef[:, p * (p + 1) // 2 + p, 1] = 0.0
    c = B.Context()
    g = np.zeros(nf * B.npts(p))
    B.bim_sh_synthesize(c.h, p, p, nf, np.ascontiguousarray(coef.reshape(-1)), 0, 0, g)
    out = np.zeros(nf * 2 * B.ncoef(p))
    B.bim_sh_analyze(c.h, p, p, nf, g, out)
    c.close()
    e = np.abs(out.reshape(coef.shape) - coef).max() / np.abs(coef).max()
    print(f"round trip p={p}: {e:.2e}", flush=True)
    assert e <= 1e-12


def _mixed_degree_drops():
    """Three drops of degrees 12, 12 and 10 (two degree groups), lambda 1.5,
    3 and 0.5, gap about 0.4."""
    import workloads as W
    rng = np.random.default_rng(91)
    ds = [W.DropSpec(12, W.perturbed_sphere(rng, 12, 1.0, (0.0, 0.0, 0.0), 0.1), 1.5),
          W.DropSpec(12, W.perturbed_sphere(rng, 12, 0.9, (2.4, 0.3, 0.0), 0.1), 3.0),
          W.DropSpec(10, W.perturbed_sphere(rng, 10, 0.8, (0.2, 2.3, 0.4), 0.1), 0.5)]
    return ds


def _rel(a, b):
    e = 0.0
    for x, y in zip(a, b):
        x, y = np.asarray(x), np.asarray(y)
        if x.ndim == 2:
            x, y = x.T, y.T
        for c in range(3):
            e = max(e, float(np.abs(x[c] - y[c]).max() / np.abs(y[c]).max()))
    return e


@pytest.mark.parametrize("which", ["two_drops", "mixed_degrees"])
def test_operator_and_solve_paths_agree_fp64(B, which):
    """The Galerkin operator A u in coefficients and the solved velocity with
    the scalar transforms (xform_path 1) and the matrix-core ones (2), FP64:
    the same per drop and component to 1e-12 (only the summation order of the
    transforms differs). The report names the path in use."""
    import workloads as W
    from test_parity_gpu import random_coef
    print(f"transform paths agree: {which}", flush=True)
    drops = W.two_drops().drops if which == "two_drops" else _mixed_degree_drops()
    rng = np.random.default_rng(92)
    dens = [random_coef(rng, d.p, 3) for d in drops]
    out = {}
    for path in (1, 2):
        c = B.Context(xform_path=path)
        c.set_drops([d.p for d in drops], [d.xc for d in drops], [d.lam for d in drops])
        c.set_tension(None, 0, sigma0=1.0)
        op = c.double_layer(dens, mode=1)
        u, rep = c.eval_velocity()
        out[path] = (op, u)
        assert rep.xform_matrix_cores == (3 if path == 2 else 0)
        c.close()
    for k, name in ((0, "operator"), (1, "velocity")):
        e = _rel(out[2][k], out[1][k])
        print(name, e, flush=True)
        assert e <= 1e-12


def test_mixed_matrix_core_solve_against_oracle_solution(B, orc):
    """The two-drop p = 32 solve in the mixed form with the FP32 matrix-core
    transforms forced (xform_path 2) against the oracle's stored solution:
    per drop and component at most 1e-5."""
    import workloads as W
    from test_parity_gpu import GOLDEN_C2, ctx_for, osys
    print("mixed matrix-core transforms: two drops p=32 solve vs oracle", flush=True)
    ref = np.load(GOLDEN_C2)
    wl = W.two_drops()
    c = ctx_for(B, wl, precision=B.BIM_PREC_MIXED, xform_path=2)
    uc, rep = c.eval_velocity(coefficients=True)
    c.close()
    assert rep.xform_matrix_cores == 3
    e = _rel(uc, osys(orc, wl).split(ref["u"]))
    print("per-output error", e, flush=True)
    assert 1e-12 < e <= TOL32
