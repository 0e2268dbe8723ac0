"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerance (FP64 path): per drop and component, ||gpu - oracle||_inf <= 1e-10
||oracle||_inf; outputs that vanish analytically are normalised by the term
scale instead (stated per test). Same seeded inputs on both sides
(``workloads``).
"""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10
GOLDEN_C2 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "two_drops_p32_solution.npz")


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_02156_amd as B
    return B


def ctx_for(B, wl, **kw):
    opts = dict(A_tilde=wl.A_tilde, U_tilde=wl.U_tilde, U_sing=wl.U_sing, U_geom=wl.U_geom,
                gmres_tol=wl.gmres_tol)
    opts.update(kw)
    c = B.Context(**opts)
    c.set_drops([d.p for d in wl.drops], [d.xc for d in wl.drops], [d.lam for d in wl.drops])
    if wl.eos != 0:
        c.set_tension([d.gc for d in wl.drops], wl.eos, wl.E, wl.xs, wl.sigma0)
    else:
        c.set_tension(None, 0, sigma0=wl.sigma0)
    return c


def osys(orc, wl, **kw):
    o = orc.Options(A_tilde=wl.A_tilde, U_tilde=wl.U_tilde, U_sing=wl.U_sing, U_geom=wl.U_geom,
                    eos=wl.eos, E=wl.E, xs=wl.xs, sigma0=wl.sigma0, gmres_tol=wl.gmres_tol)
    for k, v in kw.items():
        setattr(o, k, v)
    return orc.System([orc.Drop(d.p, d.xc, d.lam, d.gc) for d in wl.drops], o)


def rel_err(a, b, scale=None):
    """max over components of ||a_c - b_c||_inf / ||b_c||_inf (or / scale)."""
    a = np.asarray(a).reshape(-1, 3) if a.ndim != 3 else a
    out = 0.0
    for c in range(3):
        den = scale if scale is not None else np.abs(b[..., c]).max()
        out = max(out, np.abs(a[..., c] - b[..., c]).max() / den)
    return out


def coef_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def random_coef(rng, p, nf):
    c = rng.standard_normal((nf, (p + 1) * (p + 2) // 2, 2))
    c[..., [n * (n + 1) // 2 for n in range(p + 1)], 1] = 0.0
    c[..., p * (p + 1) // 2 + p, 1] = 0.0
    return c


# --- transforms -----------------------------------------------------------------

@pytest.mark.parametrize("p,q", [(2, 2), (7, 7), (13, 26), (16, 16), (32, 32), (32, 128), (48, 48)])
def test_synthesis_all_derivatives(B, orc, p, q):
    print(f"synthesis p={p} q={q}", flush=True)
    rng = np.random.default_rng(100 + p + q)
    nf = 3
    coef = random_coef(rng, p, nf)
    c = B.Context()
    for dt, dp in [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]:
        g = np.zeros(nf * B.npts(q))
        B.bim_sh_synthesize(c.h, p, q, nf, np.ascontiguousarray(coef.reshape(-1)), dt, dp, g)
        g = g.reshape(nf, -1)
        for f in range(nf):
            ref = orc.synth(p, coef[f], q, dt, dp).ravel()
            assert np.abs(g[f] - ref).max() <= TOL * np.abs(ref).max(), (dt, dp, f)
    c.close()


@pytest.mark.parametrize("q,p", [(2, 2), (9, 9), (16, 16), (26, 13), (64, 32), (96, 48)])
def test_analysis(B, orc, q, p):
    print(f"analysis q={q} p={p}", flush=True)
    rng = np.random.default_rng(200 + p + q)
    nf = 2
    g = rng.standard_normal((nf, B.npts(q)))
    c = B.Context()
    out = np.zeros(nf * 2 * B.ncoef(p))
    B.bim_sh_analyze(c.h, q, p, nf, np.ascontiguousarray(g.reshape(-1)), out)
    out = out.reshape(nf, -1, 2)
    for f in range(nf):
        ref = orc.analyze(g[f], q, p)
        assert coef_err(out[f], ref) <= TOL
    c.close()


def test_transforms_on_device_tensors(B, orc):
    import torch
    p, q = 12, 24
    rng = np.random.default_rng(7)
    coef = random_coef(rng, p, 1)
    c = B.Context()
    dc = torch.tensor(coef.reshape(-1), device="cuda", dtype=torch.float64)
    dg = torch.zeros(B.npts(q), device="cuda", dtype=torch.float64)
    B.bim_sh_synthesize(c.h, p, q, 1, dc, 1, 0, dg)
    B.bim_synchronize(c.h)
    ref = orc.synth(p, coef[0], q, 1, 0).ravel()
    assert np.abs(dg.cpu().numpy() - ref).max() <= TOL * np.abs(ref).max()
    c.close()


# --- geometry, force, regions -----------------------------------------------------

@pytest.mark.parametrize("p", [8, 13])
def test_force_linear_eos(B, orc, p):
    print(f"force p={p}", flush=True)
    wl = W.two_drops(p=p)
    c = ctx_for(B, wl)
    fg = c.force()
    s = osys(orc, wl)
    for i in range(2):
        assert coef_err(fg[i], s.force(i)) <= TOL
    c.close()


def test_force_langmuir_and_uniform(B, orc):
    wl = W.two_drops(p=10)
    wl.eos, wl.E, wl.xs = 2, 0.3, 0.4
    c = ctx_for(B, wl)
    fg = c.force()
    s = osys(orc, wl)
    for i in range(2):
        assert coef_err(fg[i], s.force(i)) <= TOL
    c.set_tension(None, 0, sigma0=1.7)
    fg = c.force()
    s = osys(orc, wl, eos=0, sigma0=1.7)
    for i in range(2):
        assert coef_err(fg[i], s.force(i)) <= TOL
    c.close()


def test_regions_and_distances(B, orc):
    wl = W.many_drops(nd=5, p=8, box=6.0, gap=0.15, seed=31)
    wl.A_tilde, wl.U_tilde = 5.0, 3
    c = ctx_for(B, wl)
    reg, dist = c.regions()
    s = osys(orc, wl)
    off = 0
    for i, di in enumerate(wl.drops):
        n = B.npts(di.p)
        for j in range(len(wl.drops)):
            if j == i:
                assert np.all(reg[off:off + n, j] == -1)
                continue
            r, d = s.regions(i, j)
            assert np.abs(dist[off:off + n, j] - d).max() <= 1e-12 * max(1.0, d.max())
            h = s.h(j)
            near = (np.abs(d - h) < 1e-9 * h) | (np.abs(d - wl.A_tilde * h) < 1e-9 * h)
            assert np.array_equal(reg[off:off + n, j][~near], r[~near])
        off += n
    assert (reg == 1).any() and (reg == 0).any()
    c.close()


# --- single layer ------------------------------------------------------------------

@pytest.mark.parametrize("path", [0, 1, 2])
def test_single_layer_one_drop_p16(B, orc, path):
    """Single drop p = 16: every grid target against the oracle's pole rule
    (fused kernel and per-application rotation path)."""
    print(f"single layer p=16 path={path}", flush=True)
    wl = W.single_drop(p=16)
    c = ctx_for(B, wl, singular_path=path)
    u = c.single_layer()[0]
    s = osys(orc, wl)
    ref = -s.layer(0, [s.force(0)], 0) / (8 * np.pi)
    assert rel_err(u, ref) <= TOL
    c.close()


def test_single_layer_unperturbed_sphere_is_zero(B, orc):
    """Uniform tension on a sphere: u = 0; error normalised by the term scale."""
    wl = W.single_drop(p=16, perturbed=False)
    c = ctx_for(B, wl)
    u = c.single_layer()[0]
    scale = 2.0 * 16 * np.pi / 3 / (8 * np.pi)   # |S[const 2]| / 8 pi on a unit sphere
    assert np.abs(u).max() <= 1e-12 * scale
    c.close()


@pytest.mark.parametrize("p", [3, 9, 14])
def test_single_layer_with_prescribed_density_odd_and_small_degrees(B, orc, p):
    print(f"single layer prescribed p={p}", flush=True)
    rng = np.random.default_rng(300 + p)
    wl = W.single_drop(p=p, seed=5 + p)
    fcoef = random_coef(rng, p, 3)
    c = ctx_for(B, wl)
    u = c.single_layer([fcoef])[0]
    s = osys(orc, wl)
    ref = -s.layer(0, [fcoef], 0) / (8 * np.pi)
    assert rel_err(u, ref) <= TOL
    c.close()


def test_single_layer_three_drops_mixed_regions(B, orc):
    """Three drops with degrees 6, 8, 11: Omega_0 on the standard grid and
    Omega_1/2 on the upsampled grid, several target tiles and ragged tails."""
    print("single layer three drops", flush=True)
    rng = np.random.default_rng(41)
    drops = []
    for p, c0 in [(6, (0, 0, 0)), (8, (2.25, 0.2, 0)), (11, (0.8, 2.3, 0.4))]:
        drops.append(W.DropSpec(p, W.perturbed_sphere(rng, p, 1.0, c0, 0.05), 1.0))
    wl = W.Workload("three", drops, eos=0, A_tilde=5.0, U_tilde=3)
    c = ctx_for(B, wl)
    u = c.single_layer()
    s = osys(orc, wl)
    for i in range(3):
        ref = -s.layer(i, [s.force(j) for j in range(3)], 0) / (8 * np.pi)
        assert rel_err(u[i], ref) <= TOL, i
    reg, _ = c.regions()
    assert (reg == 1).any() or (reg == 2).any()
    c.close()


# --- double layer -----------------------------------------------------------------

@pytest.mark.parametrize("path", [0, 1, 2])
def test_double_layer_raw_three_drops(B, orc, path):
    print(f"double layer raw path={path}", flush=True)
    rng = np.random.default_rng(42)
    drops = []
    for p, c0, lam in [(7, (0, 0, 0), 2.0), (9, (2.3, 0.1, 0), 1.0), (8, (0.5, 2.4, 0.3), 4.0)]:
        drops.append(W.DropSpec(p, W.perturbed_sphere(rng, p, 1.0, c0, 0.05), lam))
    wl = W.Workload("three", drops, eos=0, A_tilde=5.0, U_tilde=3)
    us = [random_coef(rng, d.p, 3) for d in drops]
    c = ctx_for(B, wl, singular_path=path)
    D = c.double_layer(us, mode=0)
    s = osys(orc, wl)
    for i in range(3):
        ref = s.layer(i, us, 1) / (4 * np.pi)
        assert rel_err(D[i], ref) <= TOL, i
    # Galerkin operator (mode 1): (lambda_i + 1) u_i - P_i[sum_j (lambda_j - 1)/(4 pi) D_j[u]]
    A = c.double_layer(us, mode=1)
    ref = s.split(s.matvec(np.concatenate([u.ravel() for u in us])))
    for i in range(3):
        assert coef_err(A[i], ref[i]) <= TOL, i
    # the target-drop reading of lambda
    c2 = ctx_for(B, wl, lambda_rule=1, singular_path=path)
    A2 = c2.double_layer(us, mode=1)
    s2 = osys(orc, wl, lambda_rule=1)
    ref2 = s2.split(s2.matvec(np.concatenate([u.ravel() for u in us])))
    for i in range(3):
        assert coef_err(A2[i], ref2[i]) <= TOL, i
    c.close()
    c2.close()


@pytest.mark.parametrize("p,us", [(5, 1), (11, 2), (24, 1)])
def test_singular_path_single_and_double_layer_degrees(B, orc, p, us):
    """The default singular path (the batched pipeline) for an odd singular
    grid (p = 5, qs = 5: no longitude pairs folded in the Fourier stage), an
    upsampled one (U_sing = 2) and an even one: single layer and raw double
    layer against the oracle."""
    print(f"singular path p={p} U_sing={us}", flush=True)
    rng = np.random.default_rng(500 + p)
    wl = W.single_drop(p=p, seed=60 + p)
    wl.U_sing = us
    fc = random_coef(rng, p, 3)
    uc = random_coef(rng, p, 3)
    c = ctx_for(B, wl)
    S = c.single_layer([fc])[0]
    D = c.double_layer([uc], mode=0)[0]
    s = osys(orc, wl)
    assert rel_err(S, -s.layer(0, [fc], 0) / (8 * np.pi)) <= TOL
    assert rel_err(D, s.layer(0, [uc], 1) / (4 * np.pi)) <= TOL
    c.close()


def test_high_degree_uses_rotation_path(B, orc):
    """p = 53 exceeds the fused kernel's register and LDS budget: the
    per-application path runs; checked at sampled targets."""
    print("p=53 fallback", flush=True)
    rng = np.random.default_rng(53)
    wl = W.single_drop(p=53, seed=53)
    uc = random_coef(rng, 53, 3)
    c = ctx_for(B, wl)
    D = c.double_layer([uc], mode=0)[0]
    s = osys(orc, wl)
    tg = np.sort(rng.choice(B.npts(53), 24, replace=False))
    ref = s.layer(0, [uc], 1, targets=tg) / (4 * np.pi)
    assert np.all(np.abs(D[tg] - ref).max(axis=0) <= TOL * np.abs(ref).max(axis=0))
    c.close()


def test_double_layer_identity_on_gpu(B, orc):
    """D[const] / 4 pi = const on every drop (Sec. 2.3.1), spheres resolved at U = 8."""
    p = 8
    drops = [W.DropSpec(p, W.sphere(p, 1.0, (0, 0, 0)), 2.0), W.DropSpec(p, W.sphere(p, 0.9, (2.4, 0.1, 0)), 3.0)]
    wl = W.Workload("spheres", drops, A_tilde=1e30, U_tilde=8)
    e = np.array([0.2, 0.5, -0.3])
    u = np.zeros((3, B.ncoef(p), 2))
    u[:, 0, 0] = e * np.sqrt(4 * np.pi)
    c = ctx_for(B, wl)
    D = c.double_layer([u, u], mode=0)
    for i in range(2):
        assert np.abs(D[i] - e).max() < 1e-12
    c.close()


# --- full velocity -------------------------------------------------------------------

def test_eval_velocity_lambda_one_matches_single_layer(B, orc):
    wl = W.single_drop(p=12)
    c = ctx_for(B, wl)
    uc, rep = c.eval_velocity(coefficients=True)
    s = osys(orc, wl)
    ref, it, _ = s.solve()
    assert coef_err(uc[0], ref[0]) <= TOL
    assert rep.gmres_iterations == 0
    c.close()


@pytest.mark.parametrize("path", [0, 1, 2])
def test_eval_velocity_two_drops_gmres(B, orc, path):
    """Two drops (p = 8, lambda 1 and 5), linear equation of state; GMRES to
    1e-12 on both sides; solutions agree to 1e-10."""
    print(f"eval velocity two drops path={path}", flush=True)
    wl = W.two_drops(p=8)
    wl.gmres_tol = 1e-12
    c = ctx_for(B, wl, singular_path=path)
    uc, rep = c.eval_velocity(coefficients=True)
    s = osys(orc, wl)
    ref, it, hist = s.solve()
    for i in range(2):
        assert coef_err(uc[i], ref[i]) <= TOL, i
    assert rep.gmres_iterations > 0 and rep.gmres_residual <= 1e-12
    ug, _ = c.eval_velocity(coefficients=False)
    refg = s.velocity_grid(ref)
    for i in range(2):
        assert rel_err(ug[i], refg[i]) <= TOL
    c.close()


def test_hadamard_rybczynski_on_gpu(B, orc):
    """Closed form of a translating drop, through the GPU operator: the RHS of
    a prescribed force f = alpha (e.(x-c)) n, solved with lambda = 5."""
    p, R, alpha, lam = 8, 1.2, 0.7, 5.0
    c0 = np.array([0.1, 0.2, -0.3])
    xc = W.sphere(p, R, c0)
    x, n, Wa, K = orc.geometry(p, xc, p)
    e = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    f = (alpha * ((x.T - c0) @ e))[:, None] * n.T
    fc = np.stack([orc.analyze(f[:, k], p, p) for k in range(3)])
    wl = W.Workload("hr", [W.DropSpec(p, xc, lam)], gmres_tol=1e-13)
    c = ctx_for(B, wl)
    # GPU single layer of the prescribed force -> rhs, then the GPU operator in GMRES is
    # exercised through eval_velocity's machinery via double_layer mode 1 on the exact answer
    V = -(2 / 3) * alpha * R ** 2 * (1 + lam) / (2 + 3 * lam)
    nn = n.T
    ex = V * e[None, :] - V * (e[None, :] - nn * (nn @ e)[:, None]) / (2 * (1 + lam))
    exc = np.stack([orc.analyze(ex[:, k], p, p) for k in range(3)])
    Au = c.double_layer([exc], mode=1)[0]
    Sg = c.single_layer([fc])[0]                     # -S/(8 pi)
    bg = np.stack([orc.analyze(2 * Sg[:, k], p, p) for k in range(3)])  # -S/(4 pi) projected
    assert np.abs(Au - bg).max() < 1e-12
    c.close()


def test_two_drops_p32_sampled_singular_and_pairs(B, orc):
    """The full two-drop workload (p = 32, gap 0.2, U = 4): force, regions,
    the single layer and the raw double layer of a random density at 96
    sampled targets per drop."""
    print("two drops p=32 sampled", flush=True)
    wl = W.two_drops()
    c = ctx_for(B, wl)
    fg = c.force()
    s = osys(orc, wl)
    for i in range(2):
        assert coef_err(fg[i], s.force(i)) <= TOL
    u = c.single_layer()
    rng = np.random.default_rng(9)
    dens = [random_coef(rng, 32, 3) for _ in range(2)]
    D = c.double_layer(dens, mode=0)
    reg, _ = c.regions()
    for i in range(2):
        n = B.npts(32)
        r = reg[i * n:(i + 1) * n, 1 - i]
        near = np.nonzero(r != 0)[0]
        far = np.nonzero(r == 0)[0]
        tg = np.sort(np.concatenate([rng.choice(near, 48, replace=False), rng.choice(far, 48, replace=False)]))
        ref = -s.layer(i, [s.force(0), s.force(1)], 0, targets=tg) / (8 * np.pi)
        got = u[i][tg]
        scale = np.abs(ref).max(axis=0)
        assert np.all(np.abs(got - ref).max(axis=0) <= TOL * scale)
        refd = s.layer(i, dens, 1, targets=tg) / (4 * np.pi)
        assert np.all(np.abs(D[i][tg] - refd).max(axis=0) <= TOL * np.abs(refd).max(axis=0))
    c.close()


@pytest.mark.slow
def test_two_drops_p32_solve_matches_oracle_solution(B, orc):
    """Full two-drop solve (p = 32, lambda 1 and 5), both sides to GMRES tol
    1e-12: the GPU coefficients match the oracle's solution per drop and
    component to 1e-10, and the GPU solution's residual under the oracle's
    right-hand side and operator is <= 1e-10 ||b||. The oracle's b and
    solution are stored by tests/golden/make_two_drops_p32.py (oracle only);
    the residual takes one oracle operator application here."""
    print("two drops p=32 solve vs oracle solution", flush=True)
    ref = np.load(GOLDEN_C2)
    wl = W.two_drops()
    c = ctx_for(B, wl, gmres_tol=1e-12)
    uc, rep = c.eval_velocity(coefficients=True)
    c.close()
    assert rep.gmres_residual <= 1e-12
    s = osys(orc, wl)
    uo = s.split(ref["u"])
    for i in range(2):
        for comp in range(3):
            assert np.abs(uc[i][comp] - uo[i][comp]).max() <= TOL * np.abs(uo[i][comp]).max()
    b = ref["b"]
    r = s.matvec(np.concatenate([u.ravel() for u in uc])) - b
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b)


def test_invalid_inputs_rejected(B):
    c = B.Context()
    xc = W.sphere(8)
    with pytest.raises(B.BimError) as e:
        c.set_drops([1], [W.sphere(1)], [1.0])
    assert e.value.status == B.BIM_EINVAL
    bad = xc.copy()
    bad[0, 3, 0] = np.nan
    with pytest.raises(B.BimError) as e:
        c.set_drops([8], [bad], [1.0])
    assert e.value.status == B.BIM_EINVAL
    with pytest.raises(B.BimError) as e:
        c.set_drops([8], [xc], [-1.0])
    assert e.value.status == B.BIM_EINVAL
    with pytest.raises(B.BimError) as e:
        c.single_layer()
    assert e.value.status == B.BIM_ESTATE
    c.close()


def test_gmres_maxit_reports_noconv(B):
    wl = W.two_drops(p=8)
    c = ctx_for(B, wl, gmres_maxit=1, gmres_tol=1e-14)
    out, rep = c.eval_velocity(coefficients=True, allow_noconv=True)
    assert rep.gmres_iterations == 1 and rep.gmres_residual > 1e-14
    with pytest.raises(B.BimError) as e:
        c.eval_velocity(coefficients=True)
    assert e.value.status == B.BIM_ENOCONV
    c.close()


def test_gmres_restarts_reach_the_same_solution(B):
    """GMRES(m) with short restart cycles (m = 5 and 2) against the
    unrestarted solve on the two-drop p = 8 workload. Every cycle recomputes
    the residual b - A x and reuses the Krylov storage and the two slots of the
    residual estimates, so the solutions must agree to the solve tolerance."""
    print("gmres restarts", flush=True)
    wl = W.two_drops(p=8)
    ref, it0 = None, 0
    for m in (50, 5, 2):
        c = ctx_for(B, wl, gmres_restart=m, gmres_tol=1e-12, gmres_maxit=400)
        u, rep = c.eval_velocity(coefficients=True)
        c.close()
        x = np.concatenate([np.ravel(v) for v in u])
        print("restart", m, "iterations", rep.gmres_iterations, flush=True)
        if ref is None:
            ref, it0 = x, rep.gmres_iterations
        else:
            assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()
            assert rep.gmres_iterations >= it0


@pytest.mark.parametrize("nd", [1, 2])
def test_inverted_drop_is_rejected(B, nd):
    """A drop whose parametrization is turned inside out (x mirrored, so the
    enclosed volume is negative) is reported as invalid by the evaluation,
    alone (no drop pairs) and next to a valid drop (drop pairs)."""
    print("inverted drop, nd", nd, flush=True)
    bad = W.sphere(8).copy()
    bad[0] *= -1.0
    xs = [bad] if nd == 1 else [bad, W.sphere(8, 1.0, (3.0, 0.0, 0.0))]
    c = B.Context()
    c.set_drops([8] * nd, xs, [1.0] * nd)
    c.set_tension(None, 0)
    with pytest.raises(B.BimError) as e:
        c.eval_velocity()
    assert e.value.status == B.BIM_EINVAL and "volume" in str(e.value)
    c.close()


def test_context_recovers_after_a_rejected_evaluation(B):
    """An evaluation rejected midway (an inverted drop next to a valid one,
    found after the singular pipeline has been started on the context's
    second stream) leaves the context usable: the next evaluation of valid
    drops equals a fresh context's bit for bit."""
    print("recovery after a rejected evaluation", flush=True)
    bad = W.sphere(8).copy()
    bad[0] *= -1.0
    good = [W.sphere(8, 1.0, (0.0, 0.0, 0.0)), W.sphere(8, 0.9, (2.6, 0.3, 0.0))]
    lam = [2.0, 5.0]

    def ev(c):
        c.set_drops([8, 8], good, lam)
        c.set_tension(None, 0)
        return c.eval_velocity(coefficients=True)[0]

    c = B.Context(pair_tune=0, xform_path=1)
    c.set_drops([8, 8], [bad, good[1]], lam)
    c.set_tension(None, 0)
    with pytest.raises(B.BimError) as e:
        c.eval_velocity()
    assert e.value.status == B.BIM_EINVAL
    u = ev(c)
    c.close()
    c = B.Context(pair_tune=0, xform_path=1)
    ref = ev(c)
    c.close()
    assert all(np.array_equal(a, b) for a, b in zip(u, ref))
