"""The no-allocation variant of the double-layer operator
(bim_apply_double_layer_noalloc, static device scratch for the pair partial
sums) against bim_apply_double_layer, through the C ABI, on two calls in a
row, the second on a smaller input; plus its error paths.

Bar: FP64, 1e-10 per drop and component (the same kernels in the same order
run, so the outputs are expected to be bit-identical; the test requires the
parity bar and reports equality).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_02156_amd as B
    return B


def _case(B, ps, centres, lams, seed):
    import torch
    rng = np.random.default_rng(seed)
    xs = [W.perturbed_sphere(rng, p, 1.0, c, 0.05) for p, c in zip(ps, centres)]
    ctx = B.Context()
    ctx.set_drops(ps, xs, lams)
    ctx.set_tension(None, 0, sigma0=1.0)
    dens = []
    for p in ps:
        d = rng.standard_normal((3, B.ncoef(p), 2))
        d[..., [n * (n + 1) // 2 for n in range(p + 1)], 1] = 0.0
        d[..., p * (p + 1) // 2 + p, 1] = 0.0
        dens.append(d)
    u = torch.tensor(B.pack_coefficients(dens), dtype=torch.float64, device="cuda")
    return ctx, u


def _per_output_err(a, b, ps, grid):
    a, b = a.reshape(3, -1), b.reshape(3, -1)
    e, o = 0.0, 0
    for p in ps:
        n = B_npts(p) if grid else 2 * (p + 1) * (p + 2) // 2
        for c in range(3):
            e = max(e, float(np.abs(a[c, o:o + n] - b[c, o:o + n]).max() / np.abs(b[c, o:o + n]).max()))
        o += n
    return e


def B_npts(p):
    return 2 * p * (p + 1)


@pytest.mark.parametrize("mode", [0, 1])
def test_noalloc_matches_the_allocating_operator_twice(B, mode):
    import torch
    cases = [([12, 12, 10], [(0, 0, 0), (2.25, 0, 0), (0.5, 2.4, 0.3)], [2.0, 5.0, 0.5], 71),
             ([8, 8], [(0, 0, 0), (2.3, 0.2, 0)], [3.0, 1.5], 72)]   # second call: a smaller input
    for ps, cs, lams, seed in cases:
        print(f"no-alloc operator mode {mode}, degrees {ps}", flush=True)
        ctx, u = _case(B, ps, cs, lams, seed)
        n = 3 * (sum(B_npts(p) for p in ps) if mode == 0 else sum((p + 1) * (p + 2) for p in ps))
        ref = torch.zeros(n, dtype=torch.float64, device="cuda")
        got = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        B.bim_apply_double_layer(ctx.h, u, ref, mode)       # prepares the context (allocates)
        torch.cuda.synchronize()
        rc = B.lib().bim_apply_double_layer_noalloc(ctx.h, u.data_ptr(), got.data_ptr(), mode)
        assert rc == B.BIM_OK, B.lib().bim_last_error(ctx.h)
        torch.cuda.synchronize()
        a, b = got.cpu().numpy(), ref.cpu().numpy()
        e = _per_output_err(a, b, ps, mode == 0)
        print("per-output error", e, "bit-identical", bool(np.array_equal(a, b)), flush=True)
        assert e <= 1e-10
        ctx.close()


def test_noalloc_error_paths(B):
    """A context that has not applied the operator yet is rejected before
    anything runs (BIM_ESTATE); null pointers and a bad mode are BIM_EINVAL."""
    import torch
    print("no-alloc error paths", flush=True)
    ctx, u = _case(B, [8, 8], [(0, 0, 0), (2.3, 0.2, 0)], [3.0, 1.5], 73)
    out = torch.zeros(3 * 2 * B_npts(8), dtype=torch.float64, device="cuda")
    assert B.lib().bim_apply_double_layer_noalloc(ctx.h, u.data_ptr(), out.data_ptr(), 0) == B.BIM_ESTATE
    assert B.lib().bim_apply_double_layer_noalloc(ctx.h, None, out.data_ptr(), 0) == B.BIM_EINVAL
    assert B.lib().bim_apply_double_layer_noalloc(ctx.h, u.data_ptr(), out.data_ptr(), 2) == B.BIM_EINVAL
    B.bim_apply_double_layer(ctx.h, u, out, 0)
    # prepared for mode 0 only: mode 1 needs its own work list
    out1 = torch.zeros(3 * 2 * 90, dtype=torch.float64, device="cuda")
    assert B.lib().bim_apply_double_layer_noalloc(ctx.h, u.data_ptr(), out1.data_ptr(), 1) == B.BIM_ESTATE
    assert B.lib().bim_apply_double_layer_noalloc(ctx.h, u.data_ptr(), out.data_ptr(), 0) == B.BIM_OK
    torch.cuda.synchronize()
    ctx.close()


def test_noalloc_operator_replayed_from_a_graph(B):
    """The allocation-free operator captured once in a HIP graph (torch's graph
    capture on the context's stream) and replayed four times, with a new
    density written in place (eager) between replays: every replay equals
    the eager operator on the same density."""
    import torch
    print("no-alloc operator in a graph", flush=True)
    s = torch.cuda.Stream()
    rng = np.random.default_rng(74)
    ps = [10, 10]
    xs = [W.perturbed_sphere(rng, p, 1.0, c, 0.05) for p, c in zip(ps, [(0, 0, 0), (2.3, 0.1, 0)])]
    ctx = B.Context(stream=s.cuda_stream)
    ctx.set_drops(ps, xs, [2.0, 4.0])
    ctx.set_tension(None, 0, sigma0=1.0)

    def dens():
        out = []
        for p in ps:
            d = rng.standard_normal((3, B.ncoef(p), 2))
            d[..., [n * (n + 1) // 2 for n in range(p + 1)], 1] = 0.0
            d[..., p * (p + 1) // 2 + p, 1] = 0.0
            out.append(d)
        return torch.tensor(B.pack_coefficients(out), dtype=torch.float64, device="cuda")

    n = 3 * sum(B_npts(p) for p in ps)
    u = dens()
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    ref = torch.zeros(n, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(s):
        B.bim_apply_double_layer(ctx.h, u, ref, 0)        # prepares the context
        assert B.lib().bim_apply_double_layer_noalloc(ctx.h, u.data_ptr(), out.data_ptr(), 0) == B.BIM_OK
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rc = B.lib().bim_apply_double_layer_noalloc(ctx.h, u.data_ptr(), out.data_ptr(), 0)
    assert rc == B.BIM_OK, B.lib().bim_last_error(ctx.h)
    for r in range(4):
        u.copy_(dens())                                     # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            B.bim_apply_double_layer(ctx.h, u, ref, 0)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        e = _per_output_err(a, b, ps, True)
        print("replay", r, "per-output error", e, "bit-identical", bool(np.array_equal(a, b)), flush=True)
        assert e <= 1e-10
    del g
    ctx.close()
