"""Request server: results in the mix equal results alone, admission by the
memory budget, error paths.

Requests are independent drop systems from the serving stream (1-8 drops of
one degree in {8, 16, 24, 32}, lambda in {1, 2, 5}, uniform tension). Each
result of a request run concurrently with others must equal the same request
run alone on a plain context with the server's options (the pair work
shape by its rule, pair_tune = 0; scalar transforms, xform_path = 1) bit
for bit: every sum on the path has a
fixed order, so overlapping work on the device changes nothing.
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


def _requests(n, pmax=24):
    return [r for r in W.serving_requests(n=4 * n) if r.p <= pmax][:n]


def _alone(B, req):
    c = B.Context(pair_tune=0, xform_path=1)
    c.set_drops([d.p for d in req.drops], [d.xc for d in req.drops], [d.lam for d in req.drops])
    c.set_tension(None, 0, sigma0=1.0)
    u, rep = c.eval_velocity()
    c.close()
    return u


def test_results_in_the_mix_equal_results_alone(B):
    print("server mix vs alone", flush=True)
    reqs = _requests(10)
    srv = B.Server(slots=4)
    ids = [srv.submit([d.p for d in r.drops], [d.xc for d in r.drops], [d.lam for d in r.drops]) for r in reqs]
    got = [srv.wait(i) for i in ids]
    srv.close()
    for r, (u, rep, t) in zip(reqs, got):
        ref = _alone(B, r)
        for a, b in zip(u, ref):
            assert np.array_equal(a, b)
        assert t[2] >= t[1] > 0.0


def test_budget_admits_one_request_at_a_time(B):
    """A budget below any request's estimate runs them one at a time: the
    service intervals (measured from the common submission instant) do not
    overlap."""
    print("server tiny budget", flush=True)
    reqs = _requests(5, pmax=16)
    srv = B.Server(slots=4, hbm_budget_gb=1e-9)
    ids = [srv.submit([d.p for d in r.drops], [d.xc for d in r.drops], [d.lam for d in r.drops]) for r in reqs]
    times = [srv.wait(i)[2] for i in ids]
    srv.close()
    iv = sorted((q, q + s) for q, s, _ in times)
    for (a0, a1), (b0, b1) in zip(iv, iv[1:]):
        assert b0 >= a1 - 1.0   # ms; submissions are within a millisecond of each other


def test_server_error_paths(B):
    srv = B.Server(slots=1)
    r = _requests(1, pmax=32)[0]
    with pytest.raises(B.BimError) as e:
        srv.submit([1], [W.sphere(1)], [1.0])
    assert e.value.status == B.BIM_EINVAL
    rid = srv.submit([d.p for d in r.drops], [d.xc for d in r.drops], [d.lam for d in r.drops])
    res = srv.wait(rid, timeout=0.0)
    if res is None:        # not finished at the poll: wait for it
        res = srv.wait(rid)
    assert res is not None
    assert B.lib().bim_server_wait(srv.h, 987654321, 0.0, None, None, None) == B.BIM_EINVAL
    srv.close()


def test_independent_systems_in_one_context(B):
    """Two systems occupying the same region of space, set as independent
    systems of one context: each gets the result it has alone (no
    interaction leaks across systems), to the GMRES tolerance."""
    print("independent systems", flush=True)
    r1, r2 = _requests(2, pmax=16)
    a1, a2 = _alone(B, r1), _alone(B, r2)
    drops = r1.drops + r2.drops
    c = B.Context(gmres_tol=1e-12)
    c.set_drops([d.p for d in drops], [d.xc for d in drops], [d.lam for d in drops])
    c.set_systems([0] * len(r1.drops) + [1] * len(r2.drops))
    c.set_tension(None, 0, sigma0=1.0)
    reg, _ = c.regions()
    n1 = sum(B.npts(d.p) for d in r1.drops)
    assert np.all(reg[:n1, len(r1.drops):] == -2) and np.all(reg[n1:, :len(r1.drops)] == -2)
    u, rep = c.eval_velocity()
    c.close()
    for got, ref in zip(u, a1 + a2):
        assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()


def test_batched_server_results_match_alone(B):
    """max_batch 8: queued requests run together as independent systems;
    every result matches the request alone to 1e-8 (both meet the GMRES
    tolerance 1e-10 on their own system)."""
    print("batched server", flush=True)
    reqs = _requests(12)
    srv = B.Server(slots=2, max_batch=8)
    ids = [srv.submit([d.p for d in r.drops], [d.xc for d in r.drops], [d.lam for d in r.drops]) for r in reqs]
    got = [srv.wait(i) for i in ids]
    srv.close()
    for r, (u, rep, t) in zip(reqs, got):
        assert rep.gmres_residual <= 1e-10
        ref = _alone(B, r)
        for a, b in zip(u, ref):
            assert np.abs(a - b).max() <= 1e-8 * np.abs(b).max()


def _small_and_large_systems():
    """A nearly spherical drop under uniform tension (its right-hand side is
    about 1e-8 of the other's) and a strongly perturbed two-drop system."""
    rng = np.random.default_rng(17)
    p = 12
    small = [W.DropSpec(p, W.perturbed_sphere(rng, p, 1.0, (0.0, 0.0, 0.0), 1e-8), 5.0)]
    large = [W.DropSpec(p, W.perturbed_sphere(rng, p, 1.0, (10.0, 0.0, 0.0), 0.15), 2.0),
             W.DropSpec(p, W.perturbed_sphere(rng, p, 0.9, (12.3, 0.4, 0.0), 0.15), 5.0)]
    return small, large


def _alone_drops(B, drops):
    c = B.Context(pair_tune=0, xform_path=1)
    c.set_drops([d.p for d in drops], [d.xc for d in drops], [d.lam for d in drops])
    c.set_tension(None, 0, sigma0=1.0)
    u, rep = c.eval_velocity()
    c.close()
    return u, rep


def test_joint_solve_meets_every_systems_tolerance(B):
    """Independent systems solved together: a system whose right-hand side is
    tiny next to another's would need a joint tolerance below what rounding
    lets GMRES reach. The joint solve stops at the floor, checks each
    system's own residual and corrects the ones above gmres_tol: both
    converge, and each matches its result alone (1e-8, both at 1e-10)."""
    print("joint solve small + large rhs", flush=True)
    small, large = _small_and_large_systems()
    ref = _alone_drops(B, small)[0] + _alone_drops(B, large)[0]
    drops = small + large
    c = B.Context()
    c.set_drops([d.p for d in drops], [d.xc for d in drops], [d.lam for d in drops])
    c.set_systems([0, 1, 1])
    c.set_tension(None, 0, sigma0=1.0)
    u, rep = c.eval_velocity()
    c.close()
    assert rep.gmres_residual <= 1e-10
    for got, r in zip(u, ref):
        assert np.abs(got - r).max() <= 1e-8 * np.abs(r).max()


def test_batched_server_small_and_large_requests(B):
    """The same pair as requests of a batching server (one slot, batches of
    two; a first request holds the slot while the pair queues): both are
    served with status OK and match their results alone."""
    print("batched server small + large rhs", flush=True)
    small, large = _small_and_large_systems()
    first = _requests(1, pmax=16)[0]
    srv = B.Server(slots=1, max_batch=2)
    ids = [srv.submit([d.p for d in r], [d.xc for d in r], [d.lam for d in r])
           for r in (first.drops, small, large)]
    got = [srv.wait(i) for i in ids]
    srv.close()
    for drops, (u, rep, t) in zip((small, large), got[1:]):
        assert rep.gmres_residual <= 1e-10
        ref = _alone_drops(B, drops)[0]
        for a, b in zip(u, ref):
            assert np.abs(a - b).max() <= 1e-8 * np.abs(b).max()


def test_served_results_match_the_oracle(B, orc):
    """Requests of degree 8 served concurrently (server and oracle both to
    GMRES tol 1e-12): every served velocity matches the oracle's solve per
    drop and component to 1e-10."""
    print("served vs oracle", flush=True)
    reqs = [r for r in W.serving_requests(n=64) if r.p == 8 and 2 <= len(r.drops) <= 3][:3]
    assert len(reqs) == 3
    srv = B.Server(slots=3, gmres_tol=1e-12)
    ids = [srv.submit([d.p for d in r.drops], [d.xc for d in r.drops], [d.lam for d in r.drops]) for r in reqs]
    got = [srv.wait(i) for i in ids]
    srv.close()
    for r, (u, rep, t) in zip(reqs, got):
        s = orc.System([orc.Drop(d.p, d.xc, d.lam) for d in r.drops], orc.Options(gmres_tol=1e-12))
        uc, it, hist = s.solve()
        ref = s.velocity_grid(uc)
        for a, b in zip(u, ref):
            for c in range(3):
                assert np.abs(a[:, c] - b[:, c]).max() <= 1e-10 * np.abs(b[:, c]).max()


def test_mixed_results_in_the_mix_equal_results_alone(B):
    """The serving stream's form (FP32 far field, FP64 singular steps and
    GMRES): results in the mix equal the same request alone bit for bit."""
    print("server mix vs alone, mixed precision", flush=True)
    reqs = _requests(8)
    srv = B.Server(slots=4, precision=B.BIM_PREC_MIXED)
    ids = [srv.submit([d.p for d in r.drops], [d.xc for d in r.drops], [d.lam for d in r.drops]) for r in reqs]
    got = [srv.wait(i) for i in ids]
    srv.close()
    for r, (u, rep, t) in zip(reqs, got):
        c = B.Context(precision=B.BIM_PREC_MIXED, pair_tune=0, xform_path=1)
        c.set_drops([d.p for d in r.drops], [d.xc for d in r.drops], [d.lam for d in r.drops])
        c.set_tension(None, 0, sigma0=1.0)
        ref, _ = c.eval_velocity()
        c.close()
        for a, b in zip(u, ref):
            assert np.array_equal(a, b)


def test_full_queue_refuses_requests(B):
    """max_queue 2 with one slot: while a large first request runs, the
    submits beyond two waiting requests are refused with BIM_EBUSY (the
    server sheds load instead of growing its queue); every accepted request
    is served."""
    print("server max_queue", flush=True)
    big = [r for r in W.serving_requests(n=256) if r.p == 32 and len(r.drops) >= 6][0]
    small = _requests(8, pmax=16)
    srv = B.Server(slots=1, max_queue=2)
    ids, refused = [], 0
    for r in [big] + small:
        try:
            ids.append(srv.submit([d.p for d in r.drops], [d.xc for d in r.drops], [d.lam for d in r.drops]))
        except B.BimError as e:
            assert e.status == B.BIM_EBUSY
            refused += 1
    got = [srv.wait(i) for i in ids]
    srv.close()
    assert refused >= 1 and len(ids) <= 1 + 2 + 1
    for u, rep, t in got:
        assert rep.gmres_residual <= 1e-10
