"""The C-ABI library loads on a CPU-only machine, exports every declared
symbol, and its host-side tables agree with the independent oracle tables."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "bim.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(bim_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def B():
    import paper_1707_02156_amd as B
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libbim.so not built (run __graft_entry__.build())")
    return B


def test_every_declared_symbol_is_exported(B):
    L = B.lib()
    syms = declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(B.EXPORTS), "binding and header disagree"


def test_status_strings_and_defaults(B):
    assert B.bim_version() >= 100
    assert B.lib().bim_status_string(B.BIM_ENOCONV).decode() == "GMRES did not converge"
    o = B.bim_default_options()
    assert o.A_tilde == 5.0 and o.U_tilde == 4 and o.U_sing == 1 and o.U_geom == 2
    assert o.gmres_tol == 1e-10 and o.gmres_restart == 50 and o.precision == B.BIM_PREC_FP64
    assert o.near_rule == 1 and o.near_L == 8 and o.fmm_order == 0 and o.fmm_eps == 1e-10
    assert o.pair_tune == 1 and o.xform_path == 0 and o.pipe_budget_gb == 8.0
    assert B.lib().bim_status_string(B.BIM_EBUSY).decode() == "server queue full"
    import ctypes
    so = B.bim_server_options()
    assert B.lib().bim_server_default_options(ctypes.byref(so)) == B.BIM_OK
    assert so.slots == 3 and so.max_batch == 1 and so.max_queue == 0
    assert so.opt.pair_tune == 0 and so.opt.xform_path == 1 and so.opt.pipe_budget_gb == 0.75


def test_invalid_options_rejected_without_device(B):
    import ctypes
    o = B.bim_default_options(precision=2)
    h = ctypes.c_void_p()
    assert B.lib().bim_create(ctypes.byref(o), ctypes.byref(h)) == B.BIM_EINVAL
    o = B.bim_default_options(U_tilde=0)
    assert B.lib().bim_create(ctypes.byref(o), ctypes.byref(h)) == B.BIM_EINVAL
    for bad in (dict(near_rule=2), dict(near_L=1), dict(near_L=17), dict(fmm_order=1), dict(fmm_order=31),
                dict(fmm_order=8, fmm_eps=0.0), dict(fmm_order=8, fmm_eps=1.0), dict(xform_path=3),
                dict(xform_path=-1), dict(pipe_budget_gb=0.0), dict(pipe_budget_gb=float("nan"))):
        o = B.bim_default_options(**bad)
        assert B.lib().bim_create(ctypes.byref(o), ctypes.byref(h)) == B.BIM_EINVAL
    assert B.lib().bim_destroy(None) == B.BIM_EINVAL


@pytest.mark.parametrize("q", [1, 8, 32, 96, 192])
def test_host_gauss_legendre_vs_oracle(B, orc, q):
    t, w = B.bim_host_gauss_legendre(q)
    to, wo = orc.gauss_legendre(q)
    assert np.abs(t - to).max() < 2e-15
    assert np.abs(w - wo).max() < 2e-15


@pytest.mark.parametrize("t", [0.97, 0.31, -0.55])
def test_host_legendre_vs_oracle(B, orc, t):
    nmax = 48
    P, D1, D2 = B.bim_host_legendre(nmax, t)
    Po, D1o, D2o = orc.legendre_dtheta(nmax, t)
    n = np.array([k for k in range(nmax + 1) for _ in range(k + 1)], dtype=float)
    assert np.abs(P - Po).max() < 1e-13
    assert np.all(np.abs(D1 - D1o) <= 1e-13 * (1 + n))
    assert np.all(np.abs(D2 - D2o) <= 1e-13 * (1 + n) ** 2)


@pytest.mark.parametrize("n", [1, 7, 24, 48])
def test_host_wigner_vs_oracle_appendix_b(B, orc, n):
    """Jacobi-recurrence tables vs the Appendix B sum in __float128."""
    for beta in [0.05, 0.9, np.pi / 2, 2.7, 3.1]:
        d = B.bim_host_wigner_d(n, beta)
        assert np.abs(d - orc.wigner_d(n, beta)).max() < 5e-14


def test_host_wigner_unitary_at_degree_64(B):
    for beta in [0.02, 1.0, 3.12]:
        d = B.bim_host_wigner_d(64, beta)
        assert np.abs(d @ d.T - np.eye(129)).max() < 1e-12


def test_create_fails_cleanly_without_gpu(B):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(B.BimError) as e:
        B.bim_create()
    assert e.value.status == B.BIM_EDEVICE
