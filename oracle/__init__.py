"""Plain FP64 CPU oracle for the Stokes layer-potential hot path.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The product
library (``paper_1707_02156_amd``) never imports it and shares no code with it.

The low-level steps (grid, Legendre functions, synthesis, analysis, Wigner-d
rotation, geometry, force, singular and regular quadrature) live in
``bim_oracle.c`` (plain C, FP64, OpenMP over targets). This module loads that
library with ctypes and composes the system-level operator in plain numpy:

* region split by node distance (Sec. 2.3, regions Omega_0/1/2),
* right-hand side ``2 u_inf - (1/4pi) sum_j S_j[f]`` of the boundary integral
  equation of Sec. 1,
* the Galerkin second-kind operator of Sec. 1.2 and its textbook GMRES solve.

Paper: C. Sorgentone, A.-K. Tornberg, arXiv:1707.02156.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "bim_oracle.c")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile ``bim_oracle.c`` into ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", _SRC,
               "-o", _LIB_PATH + ".tmp", "-lquadmath", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_gauss_legendre.argtypes = [ctypes.c_int, _dp, _dp]
        L.orc_legendre.argtypes = [ctypes.c_int, ctypes.c_double, _dp]
        L.orc_legendre_dtheta.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
        L.orc_synth.argtypes = [ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
        L.orc_analyze.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp]
        L.orc_eval_point.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double]
        L.orc_eval_point.restype = ctypes.c_double
        L.orc_eval_points_d.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int, _dp]
        L.orc_wigner_d.argtypes = [ctypes.c_int, ctypes.c_double, _dp]
        L.orc_rotate.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_geometry.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, _dp, _dp]
        L.orc_surface_integral.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp]
        L.orc_surface_integral.restype = ctypes.c_double
        L.orc_volume.argtypes = [ctypes.c_int, _dp, ctypes.c_int]
        L.orc_volume.restype = ctypes.c_double
        L.orc_force.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int, _dp]
        L.orc_singular.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int, _ip, _dp]
        L.orc_singular.restype = ctypes.c_int
        L.orc_regular.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.orc_regular.restype = ctypes.c_int
        L.orc_min_node_distance.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp, _dp]
        L.orc_eval_point_d.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_int]
        L.orc_eval_point_d.restype = ctypes.c_double
        L.orc_closest_point.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_closest_point.restype = ctypes.c_int
        L.orc_nearest_node.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp, _ip]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def ncoef(p: int) -> int:
    return (p + 1) * (p + 2) // 2


def npts(q: int) -> int:
    return 2 * q * (q + 1)


def num_threads() -> int:
    return int(lib().orc_num_threads())


# --------------------------------------------------------------------------
# Low-level wrappers (each cites the passage its C routine follows).
# Coefficient arrays: shape (ncoef(p), 2) for a scalar, (3, ncoef(p), 2) for a
# vector field; [..., 0] = Re, [..., 1] = Im of f_n^m at index n(n+1)/2 + m.
# --------------------------------------------------------------------------

def gauss_legendre(q: int):
    """Gauss-Legendre nodes (descending) and weights, q+1 points (Sec. 2.1)."""
    t = np.zeros(q + 1)
    w = np.zeros(q + 1)
    lib().orc_gauss_legendre(q, _p(t), _p(w))
    return t, w


def legendre(nmax: int, t: float):
    """Normalized associated Legendre functions by the Appendix A recursions."""
    P = np.zeros(ncoef(nmax))
    lib().orc_legendre(nmax, float(t), _p(P))
    return P


def legendre_dtheta(nmax: int, t: float):
    P = legendre(nmax, t)
    D1 = np.zeros_like(P)
    D2 = np.zeros_like(P)
    lib().orc_legendre_dtheta(nmax, float(t), _p(P), _p(D1), _p(D2))
    return P, D1, D2


def synth(p: int, c, q: int, dt: int = 0, dp: int = 0):
    """Grid values (q+1, 2q) of a degree-p field or of a derivative (Sec. 1.1, App. A)."""
    c = _c(c)
    out = np.zeros((q + 1) * 2 * q)
    lib().orc_synth(p, _p(c), q, dt, dp, _p(out))
    return out.reshape(q + 1, 2 * q)


def analyze(f, q: int, p: int):
    """Coefficients to degree p from grid values on the degree-q grid (Sec. 2.1)."""
    f = _c(f)
    c = np.zeros((ncoef(p), 2))
    lib().orc_analyze(q, _p(f), p, _p(c))
    return c


def eval_point(p: int, c, theta: float, phi: float) -> float:
    c = _c(c)
    return float(lib().orc_eval_point(p, _p(c), float(theta), float(phi)))


def wigner_d(n: int, beta: float):
    """Appendix B small-d matrix, full (2n+1)^2, rows m' and columns m from -n."""
    d = np.zeros((2 * n + 1) * (2 * n + 1))
    lib().orc_wigner_d(n, float(np.cos(beta)), _p(d))
    return d.reshape(2 * n + 1, 2 * n + 1)


def rotate(p: int, c, beta: float, alpha: float):
    """Coefficients of f'(s) = f(R_z(alpha) R_y(beta) s) (Appendix B, gamma = 0)."""
    c = _c(c)
    out = np.zeros((ncoef(p), 2))
    lib().orc_rotate(p, _p(c), float(beta), float(alpha), _p(out))
    return out


def geometry(p: int, xc, q: int):
    """Grid geometry of a degree-p surface on the degree-q grid (Table 2, readings)."""
    xc = _c(xc)
    n = npts(q)
    x = np.zeros(3 * n)
    nr = np.zeros(3 * n)
    W = np.zeros(n)
    K = np.zeros(n)
    lib().orc_geometry(p, _p(xc), q, _p(x), _p(nr), _p(W), _p(K))
    return x.reshape(3, n), nr.reshape(3, n), W, K


def surface_integral(p: int, xc, q: int, g=None) -> float:
    xc = _c(xc)
    gp = _p(_c(g)) if g is not None else ctypes.cast(None, _dp)
    return float(lib().orc_surface_integral(p, _p(xc), q, gp))


def volume(p: int, xc, q: int | None = None) -> float:
    xc = _c(xc)
    return float(lib().orc_volume(p, _p(xc), q if q is not None else p))


def force(p: int, xc, gc=None, eos: int = 0, E: float = 0.0, xs: float = 0.0,
          sigma0: float = 1.0, ugeom: int = 2):
    """Force coefficients f = 2 sigma K n - grad_gamma sigma (Sec. 1, Sec. 1.3)."""
    xc = _c(xc)
    fc = np.zeros((3, ncoef(p), 2))
    gp = _p(_c(gc)) if gc is not None else ctypes.cast(None, _dp)
    lib().orc_force(p, _p(xc), gp, int(eos), float(E), float(xs), float(sigma0), int(ugeom), _p(fc))
    return fc


def singular(p: int, xc, dc, kind: int, targets=None, qs: int | None = None):
    """Pole-rule self-integral at grid targets (Sec. 2.2 Theorem 1, App. B).

    kind 0: int f.G ds; kind 1: int u.T.n ds. Returns (nt, 3)."""
    xc = _c(xc)
    dc = _c(dc)
    if targets is None:
        targets = np.arange(npts(p))
    tg = _c(targets, np.int32)
    out = np.zeros((len(tg), 3))
    rc = lib().orc_singular(p, qs if qs is not None else p, _p(xc), _p(dc), int(kind), len(tg),
                            tg.ctypes.data_as(_ip), _p(out))
    if rc != 0:
        raise ValueError("orc_singular failed")
    return out


def regular(ps: int, q: int, xc, dc, kind: int, x0):
    """Regular rule on the degree-q grid of a degree-ps source drop (Sec. 2.1, 2.3)."""
    xc = _c(xc)
    dc = _c(dc)
    x0 = _c(np.asarray(x0).reshape(-1, 3))
    out = np.zeros_like(x0)
    if len(x0) == 0:
        return out
    rc = lib().orc_regular(ps, q, _p(xc), _p(dc), int(kind), len(x0), _p(x0), _p(out))
    if rc != 0:
        raise ValueError("orc_regular failed")
    return out


def eval_point_d(p: int, c, theta: float, phi: float, dt: int = 0, dp: int = 0) -> float:
    """d^dt/dtheta^dt d^dp/dphi^dp of a real degree-p expansion at one point."""
    return lib().orc_eval_point_d(p, _p(_c(c)), float(theta), float(phi), int(dt), int(dp))


def eval_points_d(p: int, c, theta, phi, dt: int = 0, dp: int = 0):
    """eval_point_d at arrays of angles (vectorised over points in C)."""
    th = _c(theta)
    ph = _c(phi)
    out = np.zeros(len(th))
    lib().orc_eval_points_d(p, _p(_c(c)), len(th), _p(th), _p(ph), int(dt), int(dp), _p(out))
    return out


def closest_point(p: int, xc, x0, theta0: float, phi0: float):
    """Closest point of a drop to x0 (Sec. 2.3): Newton on the gradient of
    |x(theta, phi) - x0|^2 / 2 with a Levenberg-Marquardt shift. Returns
    (theta, phi, x_star (3,), iterations)."""
    res = np.zeros(5)
    x0 = _c(np.asarray(x0, dtype=float).reshape(3))
    it = lib().orc_closest_point(p, _p(_c(xc)), _p(x0), float(theta0), float(phi0), _p(res))
    return res[0], res[1], res[2:5].copy(), it


def nearest_node(ps: int, xc, x0):
    """Index j*2ps + k of the nearest node of the degree-ps grid to each target."""
    x0 = _c(np.asarray(x0).reshape(-1, 3))
    idx = np.zeros(len(x0), dtype=np.int32)
    if len(x0):
        lib().orc_nearest_node(ps, _p(_c(xc)), len(x0), _p(x0), idx.ctypes.data_as(_ip))
    return idx


def lagrange(s_nodes, values, s):
    """Value at s of the polynomial through (s_nodes[l], values[l]) (values may
    be vectors), in Lagrange form."""
    s_nodes = np.asarray(s_nodes, dtype=float)
    values = np.asarray(values, dtype=float)
    out = np.zeros(values.shape[1:])
    for l in range(len(s_nodes)):
        w = 1.0
        for m in range(len(s_nodes)):
            if m != l:
                w *= (s - s_nodes[m]) / (s_nodes[l] - s_nodes[m])
        out = out + w * values[l]
    return out


def min_node_distance(ps: int, xc, x0):
    xc = _c(xc)
    x0 = _c(np.asarray(x0).reshape(-1, 3))
    d = np.zeros(len(x0))
    if len(x0):
        lib().orc_min_node_distance(ps, _p(xc), len(x0), _p(x0), _p(d))
    return d


# --------------------------------------------------------------------------
# System level: drops, regions, operators, GMRES.
# --------------------------------------------------------------------------

@dataclass
class Options:
    A_tilde: float = 5.0      # Omega_1 threshold in units of h (Sec. 2.3 test: 5h)
    U_tilde: int = 4          # Omega_1 upsampling factor (Sec. 5 two-drop runs)
    U_sing: int = 1           # singular grid degree = U_sing * p
    U_geom: int = 2           # de-aliasing grid degree for the force = U_geom * p
    eos: int = 0              # 0 uniform sigma0, 1 linear, 2 Langmuir
    E: float = 0.0
    xs: float = 0.0
    sigma0: float = 1.0
    U0: tuple = (0.0, 0.0, 0.0)
    gradU: tuple = (0.0,) * 9
    lambda_rule: int = 0      # 0: source-drop lambda_j, 1: target-drop lambda_i
    near_rule: int = 1        # Omega_2 targets: 0 the Omega_1 rule, 1 the special quadrature of Sec. 2.3
    near_L: int = 8           # interpolation points x_l = x* + h sqrt(l) d, l = 1..L (Sec. 5: L = 8)
    gmres_tol: float = 1e-10
    gmres_restart: int = 50
    gmres_maxit: int = 500


@dataclass
class Drop:
    p: int
    xc: np.ndarray            # (3, ncoef(p), 2)
    lam: float = 1.0
    gc: np.ndarray | None = None  # (ncoef(p), 2) surfactant coefficients
    fc: np.ndarray | None = None  # prescribed force coefficients (3, ncoef(p), 2), else from tension


@dataclass
class System:
    drops: list
    opt: Options = field(default_factory=Options)

    def __post_init__(self):
        self._cache = {}

    # geometry ----------------------------------------------------------
    def nodes(self, i):
        key = ("nodes", i)
        if key not in self._cache:
            d = self.drops[i]
            x, n, W, K = geometry(d.p, d.xc, d.p)
            self._cache[key] = x.T.copy()
        return self._cache[key]

    def radius(self, i):
        d = self.drops[i]
        V = volume(d.p, d.xc, d.p)
        return (3.0 * V / (4.0 * np.pi)) ** (1.0 / 3.0)

    def h(self, i):
        """Grid size h = R pi / (p + 1) of the source drop (Sec. 2.3)."""
        return self.radius(i) * np.pi / (self.drops[i].p + 1)

    def force(self, i):
        key = ("force", i)
        if key not in self._cache:
            d = self.drops[i]
            o = self.opt
            if d.fc is not None:
                self._cache[key] = np.asarray(d.fc, dtype=float)
            else:
                self._cache[key] = force(d.p, d.xc, d.gc, o.eos, o.E, o.xs, o.sigma0, o.U_geom)
        return self._cache[key]

    # regions -----------------------------------------------------------
    def regions(self, i, j):
        """Region of every grid target of drop i w.r.t. source drop j (Sec. 2.3):
        0 = Omega_0 (dist > A h_j), 1 = Omega_1 (h_j < dist <= A h_j),
        2 = Omega_2 (dist <= h_j). Also returns the distances."""
        key = ("regions", i, j)
        if key not in self._cache:
            x0 = self.nodes(i)
            dist = min_node_distance(self.drops[j].p, self.drops[j].xc, x0)
            hj = self.h(j)
            reg = np.where(dist > self.opt.A_tilde * hj, 0, np.where(dist > hj, 1, 2)).astype(np.int32)
            self._cache[key] = (reg, dist)
        return self._cache[key]

    # layer potentials --------------------------------------------------
    def _pair(self, i, j, dens, kind, targets):
        """Sum over the nodes of source drop j at targets (indices) of drop i."""
        reg, _ = self.regions(i, j)
        x0 = self.nodes(i)[targets]
        r = reg[targets]
        out = np.zeros((len(targets), 3))
        dj = self.drops[j]
        far = np.nonzero(r == 0)[0]
        special = self.opt.near_rule == 1
        near = np.nonzero((r == 1) | ((r == 2) & (not special)))[0]
        nearest = np.nonzero((r == 2) & special)[0]
        if len(far):
            out[far] = regular(dj.p, dj.p, dj.xc, dens, kind, x0[far])
        if len(near):
            out[near] = regular(dj.p, self.opt.U_tilde * dj.p, dj.xc, dens, kind, x0[near])
        for a in nearest:
            out[a] = self.nearest_value(j, dens, kind, x0[a])
        return out

    # nearest region (Sec. 2.3) ------------------------------------------
    def closest(self, j, x0):
        """Closest point on drop j to x0 by Newton from the nearest grid node."""
        dj = self.drops[j]
        k = int(nearest_node(dj.p, dj.xc, x0)[0])
        t, _ = gauss_legendre(dj.p)
        th0 = np.arccos(t[k // (2 * dj.p)])
        ph0 = np.pi * (k % (2 * dj.p)) / dj.p
        return closest_point(dj.p, dj.xc, x0, th0, ph0)

    def self_coefficients(self, j, dens, kind):
        """The self-interaction of drop j at its own grid nodes (singular rule),
        analysed to a degree-p expansion: the on-surface value anywhere."""
        key = ("selfcoef", j, kind, hash(np.asarray(dens).tobytes()))
        if key not in self._cache:
            dj = self.drops[j]
            v = singular(dj.p, dj.xc, dens, kind, None, self.opt.U_sing * dj.p)
            self._cache[key] = np.stack([analyze(v[:, c], dj.p, dj.p) for c in range(3)])
        return self._cache[key]

    def nearest_value(self, j, dens, kind, x0):
        """Layer potential of drop j at x0 in its nearest region (Sec. 2.3):
        closest point x*, the exterior limit at x* from the self-interaction
        expansion (the double layer jumps by -4 pi u(x*) from its on-surface
        value to the exterior side), regular-rule values at x_l = x* + h sqrt(l) d
        (d the unit vector from x* to x0), and Lagrange interpolation in the
        distance along d."""
        dj = self.drops[j]
        th, ph, xs, _ = self.closest(j, x0)
        dvec = np.asarray(x0) - xs
        s0 = np.linalg.norm(dvec)
        d = dvec / s0
        sc = self.self_coefficients(j, dens, kind)
        v0 = np.array([eval_point_d(dj.p, sc[c], th, ph) for c in range(3)])
        if kind == 1:
            u = np.asarray(dens).reshape(3, -1, 2)
            v0 = v0 - 4.0 * np.pi * np.array([eval_point_d(dj.p, u[c], th, ph) for c in range(3)])
        hj = self.h(j)
        L = self.opt.near_L
        sl = hj * np.sqrt(np.arange(1, L + 1))
        xl = xs[None, :] + sl[:, None] * d[None, :]
        dist = min_node_distance(dj.p, dj.xc, xl)
        vals = np.zeros((L, 3))
        far = dist > self.opt.A_tilde * hj
        if far.any():
            vals[far] = regular(dj.p, dj.p, dj.xc, dens, kind, xl[far])
        if (~far).any():
            vals[~far] = regular(dj.p, self.opt.U_tilde * dj.p, dj.xc, dens, kind, xl[~far])
        return lagrange(np.concatenate([[0.0], sl]), np.vstack([v0[None, :], vals]), s0)

    def layer(self, i, dens_list, kind, targets=None, weights=None):
        """sum_j weights[j] * (int f.G or int u.T.n over drop j) at targets of drop i."""
        di = self.drops[i]
        if targets is None:
            targets = np.arange(npts(di.p))
        targets = np.asarray(targets)
        out = np.zeros((len(targets), 3))
        for j, dj in enumerate(self.drops):
            wj = 1.0 if weights is None else weights[j]
            if wj == 0.0:
                continue
            if j == i:
                out += wj * singular(dj.p, dj.xc, dens_list[j], kind, targets,
                                     self.opt.U_sing * dj.p)
            else:
                out += wj * self._pair(i, j, dens_list[j], kind, targets)
        return out

    def dl_weights(self, i):
        """Per-source weight (lambda - 1) / (4 pi) of the double layer on drop i's
        equation; lambda of the source drop j (rule 0) or of the target drop i."""
        lam = np.array([d.lam for d in self.drops])
        if self.opt.lambda_rule == 0:
            return (lam - 1.0) / (4.0 * np.pi)
        return np.full(len(lam), (lam[i] - 1.0) / (4.0 * np.pi))

    def u_inf(self, x):
        U0 = np.asarray(self.opt.U0, dtype=float)
        gU = np.asarray(self.opt.gradU, dtype=float).reshape(3, 3)
        return U0[None, :] + x @ gU.T

    def rhs_grid(self, i, targets=None):
        """b = 2 u_inf - (1/4pi) sum_j int f.G ds at grid targets of drop i (Sec. 1)."""
        di = self.drops[i]
        if targets is None:
            targets = np.arange(npts(di.p))
        f = [self.force(j) for j in range(len(self.drops))]
        S = self.layer(i, f, 0, targets)
        return 2.0 * self.u_inf(self.nodes(i)[targets]) - S / (4.0 * np.pi)

    # Galerkin operator ---------------------------------------------------
    def sizes(self):
        return [3 * ncoef(d.p) * 2 for d in self.drops]

    def split(self, v):
        out, o = [], 0
        for d, s in zip(self.drops, self.sizes()):
            out.append(v[o:o + s].reshape(3, ncoef(d.p), 2))
            o += s
        return out

    def project(self, i, grid_vals):
        """Analysis (Sec. 2.1) of a grid vector field (npts, 3) of drop i."""
        p = self.drops[i].p
        return np.stack([analyze(grid_vals[:, c], p, p) for c in range(3)])

    def dl_grid(self, i, ucoefs, targets=None):
        """sum_j w_j int u.T.n ds over drop j, at grid targets of drop i."""
        return self.layer(i, ucoefs, 1, targets, self.dl_weights(i))

    def matvec(self, v):
        """Second-kind Galerkin operator (Sec. 1.2):
        (A u)_i = (lambda_i + 1) u_i - P_i[ sum_j (lambda_j - 1)/(4pi) D_j[u] ]."""
        us = self.split(v)
        out = []
        for i, d in enumerate(self.drops):
            g = self.dl_grid(i, us)
            out.append(((d.lam + 1.0) * us[i] - self.project(i, g)).ravel())
        return np.concatenate(out)

    def rhs(self):
        return np.concatenate([self.project(i, self.rhs_grid(i)).ravel() for i in range(len(self.drops))])

    def solve(self, tol=None, restart=None, maxit=None):
        """Galerkin solve of the second-kind equation (Sec. 1.2) by GMRES.
        Returns (u coefficients per drop, iterations, relative residual history)."""
        o = self.opt
        b = self.rhs()
        if all(d.lam == 1.0 for d in self.drops):
            x = b / 2.0
            return self.split(x), 0, [0.0]
        x, it, hist = gmres(self.matvec, b, tol or o.gmres_tol, restart or o.gmres_restart,
                            maxit or o.gmres_maxit)
        return self.split(x), it, hist

    def velocity_grid(self, ucoefs):
        """Grid values of the velocity from its coefficients (synthesis)."""
        out = []
        for d, uc in zip(self.drops, ucoefs):
            out.append(np.stack([synth(d.p, uc[c], d.p).ravel() for c in range(3)], axis=1))
        return out


def gmres(A, b, tol, restart, maxit):
    """Restarted GMRES with modified Gram-Schmidt and Givens rotations, x0 = 0,
    stopping when ||b - A x|| <= tol ||b|| (Euclidean norm)."""
    n = len(b)
    x = np.zeros(n)
    bn = np.linalg.norm(b)
    hist = [1.0]
    if bn == 0.0:
        return x, 0, hist
    it = 0
    while it < maxit:
        r = b - A(x) if it > 0 else b.copy()
        beta = np.linalg.norm(r)
        if beta <= tol * bn:
            break
        m = restart
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k_done = 0
        for k in range(m):
            w = A(V[k])
            for l in range(k + 1):
                H[l, k] = np.dot(V[l], w)
                w = w - H[l, k] * V[l]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] != 0.0:
                V[k + 1] = w / H[k + 1, k]
            for l in range(k):
                t = cs[l] * H[l, k] + sn[l] * H[l + 1, k]
                H[l + 1, k] = -sn[l] * H[l, k] + cs[l] * H[l + 1, k]
                H[l, k] = t
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k] = H[k, k] / den
            sn[k] = H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            it += 1
            k_done = k + 1
            hist.append(abs(g[k + 1]) / bn)
            if abs(g[k + 1]) <= tol * bn or it >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done])
        x = x + V[:k_done].T @ y
        if hist[-1] <= tol:
            break
    return x, it, hist
