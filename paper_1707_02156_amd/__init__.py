"""Python binding of the gfx950 Stokes layer-potential library (libbim.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/bim.h``. Functions carry the
names of the C entry points. Arrays are numpy arrays (host memory) or
torch CUDA tensors (device memory, passed by ``data_ptr()``); torch is used
for device memory and streams only.

If the library is missing the import raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbim.so")

BIM_OK, BIM_EINVAL, BIM_ENOMEM, BIM_EDEVICE, BIM_ENOCONV, BIM_ESTATE, BIM_EAGAIN, BIM_EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
BIM_MEM_HOST, BIM_MEM_DEVICE = 0, 1
BIM_EOS_UNIFORM, BIM_EOS_LINEAR, BIM_EOS_LANGMUIR = 0, 1, 2
BIM_PREC_FP64, BIM_PREC_MIXED = 0, 1


class bim_options(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("A_tilde", ctypes.c_double),
        ("U_tilde", ctypes.c_int),
        ("U_sing", ctypes.c_int),
        ("U_geom", ctypes.c_int),
        ("lambda_rule", ctypes.c_int),
        ("gmres_tol", ctypes.c_double),
        ("gmres_restart", ctypes.c_int),
        ("gmres_maxit", ctypes.c_int),
        ("singular_path", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("near_rule", ctypes.c_int),
        ("near_L", ctypes.c_int),
        ("fmm_order", ctypes.c_int),
        ("fmm_eps", ctypes.c_double),
        ("pair_tune", ctypes.c_int),
        ("xform_path", ctypes.c_int),
        ("pipe_budget_gb", ctypes.c_double),
    ]


class bim_server_options(ctypes.Structure):
    _fields_ = [
        ("slots", ctypes.c_int),
        ("hbm_budget_gb", ctypes.c_double),
        ("opt", bim_options),
        ("max_batch", ctypes.c_int),
        ("max_batch_drops", ctypes.c_int),
        ("max_queue", ctypes.c_int),
    ]


class bim_report(ctypes.Structure):
    _fields_ = [
        ("gmres_iterations", ctypes.c_int),
        ("gmres_residual", ctypes.c_double),
        ("n_targets", ctypes.c_int),
        ("n_omega1", ctypes.c_int),
        ("n_omega2", ctypes.c_int),
        ("n_matvec", ctypes.c_int),
        ("ms_total", ctypes.c_double),
        ("n_fmm_pairs", ctypes.c_int),
        ("fmm_order", ctypes.c_int),
        ("pair_targets_per_lane", ctypes.c_int),
        ("pair_sources_per_item", ctypes.c_int),
        ("xform_matrix_cores", ctypes.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class bim_step_report(ctypes.Structure):
    _fields_ = [
        ("dt_next", ctypes.c_double),
        ("err_drop", ctypes.c_double),
        ("err_surf", ctypes.c_double),
        ("mass0", ctypes.c_double),
        ("mass1", ctypes.c_double),
        ("accepted", ctypes.c_int),
        ("gmres_velocity", ctypes.c_int * 2),
        ("gmres_imex", ctypes.c_int),
        ("ms_total", ctypes.c_double),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["gmres_velocity"] = list(self.gmres_velocity)
        d["accepted"] = bool(self.accepted)
        return d


class bim_rep_report(ctypes.Structure):
    _fields_ = [
        ("moves", ctypes.c_int),
        ("ncut_min", ctypes.c_int),
        ("gnorm", ctypes.c_double),
        ("ms_total", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double

EXPORTS = {
    "bim_version": ([], _i),
    "bim_status_string": ([_i], ctypes.c_char_p),
    "bim_default_options": ([ctypes.POINTER(bim_options)], _i),
    "bim_create": ([ctypes.POINTER(bim_options), ctypes.POINTER(_vp)], _i),
    "bim_destroy": ([_vp], _i),
    "bim_last_error": ([_vp], ctypes.c_char_p),
    "bim_set_drops": ([_vp, _i, _vp, _vp, _vp, _i], _i),
    "bim_set_tension": ([_vp, _vp, _i, _d, _d, _d, _i], _i),
    "bim_set_systems": ([_vp, _vp], _i),
    "bim_set_farfield": ([_vp, _vp, _vp], _i),
    "bim_force": ([_vp, _vp, _i], _i),
    "bim_regions": ([_vp, _vp, _vp, _i], _i),
    "bim_single_layer": ([_vp, _vp, _vp, _i], _i),
    "bim_apply_double_layer": ([_vp, _vp, _vp, _i, _i], _i),
    "bim_apply_double_layer_noalloc": ([_vp, _vp, _vp, _i], _i),
    "bim_eval_velocity": ([_vp, _vp, _i, ctypes.POINTER(bim_report)], _i),
    "bim_time_step": ([_vp, _d, _d, _d, ctypes.POINTER(bim_step_report)], _i),
    "bim_get_state": ([_vp, _vp, _vp, _i], _i),
    "bim_reparametrize": ([_vp, _i, _d, _d, _i, _d, ctypes.POINTER(bim_rep_report)], _i),
    "bim_sh_synthesize": ([_vp, _i, _i, _i, _vp, _i, _i, _vp, _i], _i),
    "bim_sh_analyze": ([_vp, _i, _i, _i, _vp, _vp, _i], _i),
    "bim_synchronize": ([_vp], _i),
    "bim_profile": ([_vp, _i], _i),
    "bim_profile_select": ([_vp, ctypes.c_char_p], _i),
    "bim_profile_query": ([_vp, ctypes.c_char_p, _vp, _vp, _vp, _vp], _i),
    "bim_host_gauss_legendre": ([_i, _vp, _vp], _i),
    "bim_host_legendre": ([_i, _d, _vp, _vp, _vp], _i),
    "bim_host_wigner_d": ([_i, _d, _vp], _i),
    "bim_server_default_options": ([ctypes.POINTER(bim_server_options)], _i),
    "bim_server_create": ([ctypes.POINTER(bim_server_options), ctypes.POINTER(_vp)], _i),
    "bim_server_destroy": ([_vp], _i),
    "bim_server_submit": ([_vp, _i, _vp, _vp, _vp, _vp, _i, _d, _d, _d, _i, ctypes.POINTER(ctypes.c_uint64)], _i),
    "bim_server_wait": ([_vp, ctypes.c_uint64, _d, _vp, ctypes.POINTER(bim_report), _vp], _i),
    "bim_server_footprint": ([ctypes.POINTER(bim_options), _i, _vp, ctypes.POINTER(_d)], _i),
}

_lib = None


def lib():
    """Load libbim.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1707_02156_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in EXPORTS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


class BimError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _ptr(a):
    """(pointer, mem_kind) of a numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None, BIM_MEM_HOST
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data, BIM_MEM_HOST
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr(), (BIM_MEM_DEVICE if a.is_cuda else BIM_MEM_HOST)
    raise TypeError(f"unsupported array type {type(a)}")


def _check(ctx, rc, allow=()):
    if rc != BIM_OK and rc not in allow:
        msg = lib().bim_last_error(ctx).decode() if ctx else lib().bim_status_string(rc).decode()
        raise BimError(rc, msg)
    return rc


# ---- one function per C entry point ----------------------------------------

def bim_version():
    return lib().bim_version()


def bim_default_options(**kw):
    o = bim_options()
    lib().bim_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "stream":
            v = ctypes.c_void_p(v)
        setattr(o, k, v)
    return o


def bim_create(opt=None, **kw):
    o = opt or bim_default_options(**kw)
    h = ctypes.c_void_p()
    rc = lib().bim_create(ctypes.byref(o), ctypes.byref(h))
    _check(None, rc)
    return h


def bim_destroy(ctx):
    return lib().bim_destroy(ctx)


def bim_last_error(ctx):
    return lib().bim_last_error(ctx).decode()


def bim_set_drops(ctx, p, xcoef, lam):
    p = np.ascontiguousarray(p, dtype=np.int32)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    xp, mk = _ptr(xcoef)
    return _check(ctx, lib().bim_set_drops(ctx, len(p), p.ctypes.data, xp, lam.ctypes.data, mk))


def bim_set_tension(ctx, gamma_coef, eos, E=0.0, xs=0.0, sigma0=1.0):
    gp, mk = _ptr(gamma_coef)
    return _check(ctx, lib().bim_set_tension(ctx, gp, eos, E, xs, sigma0, mk))


def bim_set_farfield(ctx, U0, gradU):
    U0 = np.ascontiguousarray(U0, dtype=np.float64)
    gU = np.ascontiguousarray(gradU, dtype=np.float64).reshape(9)
    return _check(ctx, lib().bim_set_farfield(ctx, U0.ctypes.data, gU.ctypes.data))


def bim_force(ctx, out):
    op, mk = _ptr(out)
    return _check(ctx, lib().bim_force(ctx, op, mk))


def bim_regions(ctx, regions, dist=None):
    rp, mk = _ptr(regions)
    dp, _ = _ptr(dist)
    return _check(ctx, lib().bim_regions(ctx, rp, dp, mk))


def bim_single_layer(ctx, f_coef, out):
    op, mk = _ptr(out)
    fp, _ = _ptr(f_coef)
    return _check(ctx, lib().bim_single_layer(ctx, fp, op, mk))


def bim_apply_double_layer(ctx, u_coef, out, mode):
    up, mk = _ptr(u_coef)
    op, _ = _ptr(out)
    return _check(ctx, lib().bim_apply_double_layer(ctx, up, op, mode, mk))


def bim_apply_double_layer_noalloc(ctx, u_coef, out, mode):
    """bim_apply_double_layer without device allocation (device tensors only)."""
    up, mk = _ptr(u_coef)
    op, mo = _ptr(out)
    if mk != BIM_MEM_DEVICE or mo != BIM_MEM_DEVICE:
        raise ValueError("bim_apply_double_layer_noalloc takes device tensors")
    return _check(ctx, lib().bim_apply_double_layer_noalloc(ctx, up, op, mode))


def bim_eval_velocity(ctx, out, coefficients=False, allow_noconv=False):
    op, mk = _ptr(out)
    kind = (1 if coefficients else 0) | (2 if mk == BIM_MEM_DEVICE else 0)
    rep = bim_report()
    rc = lib().bim_eval_velocity(ctx, op, kind, ctypes.byref(rep))
    _check(ctx, rc, allow=(BIM_ENOCONV,) if allow_noconv else ())
    return rep


def bim_sh_synthesize(ctx, p, q, nf, coef, dt, dp, grid):
    cp, mk = _ptr(coef)
    gp, _ = _ptr(grid)
    return _check(ctx, lib().bim_sh_synthesize(ctx, p, q, nf, cp, dt, dp, gp, mk))


def bim_sh_analyze(ctx, q, p, nf, grid, coef):
    gp, mk = _ptr(grid)
    cp, _ = _ptr(coef)
    return _check(ctx, lib().bim_sh_analyze(ctx, q, p, nf, gp, cp, mk))


def bim_synchronize(ctx):
    return _check(ctx, lib().bim_synchronize(ctx))


def bim_profile(ctx, enable):
    return _check(ctx, lib().bim_profile(ctx, int(enable)))


def bim_profile_select(ctx, names=None):
    """Time only the named kernels (iterable of names; None = all)."""
    arg = None if not names else ",".join(names).encode()
    return _check(ctx, lib().bim_profile_select(ctx, arg))


def bim_profile_query(ctx, name):
    n = ctypes.c_int()
    ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(ctx, lib().bim_profile_query(ctx, name.encode(), ctypes.addressof(n), ctypes.addressof(ms),
                                        ctypes.addressof(fl), ctypes.addressof(by)))
    return {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}


def bim_host_gauss_legendre(q):
    t = np.zeros(q + 1)
    w = np.zeros(q + 1)
    _check(None, lib().bim_host_gauss_legendre(q, t.ctypes.data, w.ctypes.data))
    return t, w


def bim_host_legendre(nmax, t):
    n = (nmax + 1) * (nmax + 2) // 2
    P, D1, D2 = np.zeros(n), np.zeros(n), np.zeros(n)
    _check(None, lib().bim_host_legendre(nmax, float(t), P.ctypes.data, D1.ctypes.data, D2.ctypes.data))
    return P, D1, D2


def bim_host_wigner_d(n, beta):
    d = np.zeros((2 * n + 1) ** 2)
    _check(None, lib().bim_host_wigner_d(n, float(beta), d.ctypes.data))
    return d.reshape(2 * n + 1, 2 * n + 1)


# ---- layout helpers ----------------------------------------------------------

def ncoef(p):
    return (p + 1) * (p + 2) // 2


def npts(q):
    return 2 * q * (q + 1)


def pack_coefficients(fields):
    """Component-major multi-drop array from per-drop (3, ncoef(p), 2) arrays."""
    return np.ascontiguousarray(np.concatenate(
        [np.concatenate([np.asarray(f[c], dtype=np.float64).reshape(-1) for f in fields]) for c in range(3)]))


def pack_scalar(fields):
    return np.ascontiguousarray(np.concatenate([np.asarray(f, dtype=np.float64).reshape(-1) for f in fields]))


def unpack_grid(arr, ps):
    """Split a component-major grid array [3][sum N(p)] into per-drop (N(p), 3)."""
    arr = np.asarray(arr).reshape(3, -1)
    out, o = [], 0
    for p in ps:
        n = npts(p)
        out.append(arr[:, o:o + n].T.copy())
        o += n
    return out


def unpack_coefficients(arr, ps):
    arr = np.asarray(arr).reshape(3, -1)
    out, o = [], 0
    for p in ps:
        n = 2 * ncoef(p)
        out.append(arr[:, o:o + n].reshape(3, ncoef(p), 2).copy())
        o += n
    return out


class Context:
    """A bim context holding a set of drops (thin owner of the C handle)."""

    def __init__(self, **opts):
        self.h = bim_create(**opts)
        self.ps = []

    def close(self):
        if self.h:
            bim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_drops(self, ps, xcoefs, lams):
        self.ps = list(ps)
        bim_set_drops(self.h, ps, pack_coefficients(xcoefs), lams)

    def set_systems(self, system_of_drop):
        sy = np.ascontiguousarray(system_of_drop, dtype=np.int32)
        _check(self.h, lib().bim_set_systems(self.h, sy.ctypes.data))

    def set_tension(self, gammas, eos, E=0.0, xs=0.0, sigma0=1.0):
        g = pack_scalar(gammas) if gammas is not None else None
        bim_set_tension(self.h, g, eos, E, xs, sigma0)

    def ntargets(self):
        return sum(npts(p) for p in self.ps)

    def ncoef_total(self):
        return sum(2 * ncoef(p) for p in self.ps)

    def force(self):
        out = np.zeros(3 * self.ncoef_total())
        bim_force(self.h, out)
        return unpack_coefficients(out, self.ps)

    def single_layer(self, fcoefs=None):
        out = np.zeros(3 * self.ntargets())
        f = pack_coefficients(fcoefs) if fcoefs is not None else None
        bim_single_layer(self.h, f, out)
        return unpack_grid(out, self.ps)

    def double_layer(self, ucoefs, mode=0):
        u = pack_coefficients(ucoefs)
        if mode == 0:
            out = np.zeros(3 * self.ntargets())
            bim_apply_double_layer(self.h, u, out, 0)
            return unpack_grid(out, self.ps)
        out = np.zeros(3 * self.ncoef_total())
        bim_apply_double_layer(self.h, u, out, 1)
        return unpack_coefficients(out, self.ps)

    def regions(self):
        T, nd = self.ntargets(), len(self.ps)
        reg = np.zeros(T * nd, dtype=np.int8)
        dist = np.zeros(T * nd)
        bim_regions(self.h, reg, dist)
        return reg.reshape(T, nd), dist.reshape(T, nd)

    def eval_velocity(self, coefficients=False, allow_noconv=False):
        n = 3 * (self.ncoef_total() if coefficients else self.ntargets())
        out = np.zeros(n)
        rep = bim_eval_velocity(self.h, out, coefficients, allow_noconv)
        res = unpack_coefficients(out, self.ps) if coefficients else unpack_grid(out, self.ps)
        return res, rep

    def time_step(self, dt, Pe=float("inf"), tol=0.0):
        """One coupled drop / surfactant step (bim_time_step); returns the report
        as a dict (dt_next, err_drop, err_surf, mass0, mass1, accepted, ...)."""
        rep = bim_step_report()
        _check(self.h, lib().bim_time_step(self.h, float(dt), float(Pe), float(tol), ctypes.byref(rep)))
        return rep.as_dict()

    def reparametrize(self, U_rep=2, P_cut=1e-3, eps=1e-10, imax=30, dtau=1.0):
        """Angle reparametrization of every drop (bim_reparametrize); returns the report."""
        rep = bim_rep_report()
        _check(self.h, lib().bim_reparametrize(self.h, int(U_rep), float(P_cut), float(eps), int(imax),
                                               float(dtau), ctypes.byref(rep)))
        return rep.as_dict()

    def state(self, surfactant=True):
        """(per-drop position coefficients, per-drop surfactant coefficients or None)."""
        nc = self.ncoef_total()
        x = np.zeros(3 * nc)
        g = np.zeros(nc) if surfactant else None
        _check(self.h, lib().bim_get_state(self.h, x.ctypes.data, g.ctypes.data if surfactant else None, 0))
        xs = unpack_coefficients(x, self.ps)
        if not surfactant:
            return xs, None
        gs, o = [], 0
        for p in self.ps:
            n = 2 * ncoef(p)
            gs.append(g[o:o + n].reshape(ncoef(p), 2).copy())
            o += n
        return xs, gs


class Server:
    """Request server (bim_server_*): submit independent drop systems, wait
    for their velocities. Options: slots, hbm_budget_gb, and any context
    option by name."""

    def __init__(self, slots=3, hbm_budget_gb=64.0, max_batch=1, max_batch_drops=128, max_queue=0, **opts):
        so = bim_server_options()
        _check(None, lib().bim_server_default_options(ctypes.byref(so)))
        so.slots = slots
        so.hbm_budget_gb = hbm_budget_gb
        so.max_batch = max_batch
        so.max_batch_drops = max_batch_drops
        so.max_queue = max_queue
        for k, v in opts.items():
            setattr(so.opt, k, v)
        h = ctypes.c_void_p()
        _check(None, lib().bim_server_create(ctypes.byref(so), ctypes.byref(h)))
        self.h = h
        self._sizes = {}

    def close(self):
        if self.h:
            lib().bim_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, ps, xcoefs, lams, gammas=None, eos=BIM_EOS_UNIFORM, E=0.0, xs=0.0, sigma0=1.0,
               coefficients=False):
        p = np.ascontiguousarray(ps, dtype=np.int32)
        x = np.ascontiguousarray(pack_coefficients(xcoefs))
        lam = np.ascontiguousarray(lams, dtype=np.float64)
        g = np.ascontiguousarray(pack_scalar(gammas)) if gammas is not None else None
        rid = ctypes.c_uint64()
        _check(None, lib().bim_server_submit(self.h, len(p), p.ctypes.data, x.ctypes.data, lam.ctypes.data,
                                             g.ctypes.data if g is not None else None, int(eos), float(E),
                                             float(xs), float(sigma0), int(bool(coefficients)), ctypes.byref(rid)))
        n = 3 * (sum(2 * ncoef(q) for q in p) if coefficients else sum(npts(q) for q in p))
        self._sizes[rid.value] = (n, list(p), coefficients)
        return rid.value

    def wait(self, rid, timeout=-1.0, allow_noconv=False):
        """(velocity per drop, report, (queue, service, total) ms), or None if
        not finished within the timeout."""
        n, ps, coef = self._sizes[rid]
        out = np.zeros(n)
        rep = bim_report()
        t = np.zeros(3)
        st = lib().bim_server_wait(self.h, ctypes.c_uint64(rid), float(timeout), out.ctypes.data, ctypes.byref(rep),
                                   t.ctypes.data)
        if st == BIM_EAGAIN:
            return None
        del self._sizes[rid]
        if st != BIM_OK and not (allow_noconv and st == BIM_ENOCONV):
            raise BimError(st, f"request {rid} failed with status {st}")
        res = unpack_coefficients(out, ps) if coef else unpack_grid(out, ps)
        return res, rep, tuple(t)

