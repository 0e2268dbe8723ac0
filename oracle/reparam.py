"""Oracle for the angle reparametrization of a drop surface (Sec. 4, Algorithm 2).

Test infrastructure, like the rest of oracle/: plain FP64 numpy on top of the
oracle's transforms and point evaluation; not used by the product path.

The surface keeps its initial expansion x0 (upsampled to degree q = U_rep p);
only the parameter angles of the grid nodes move. One pseudo-time iteration,
from the current angles (theta*, phi*) of every node of the degree-q grid:
  X = x0(theta*, phi*), X_t, X_p its angle derivatives there;
  x~ = analysis of X (degree q); n_cut adaptive (eq. for n_cutoff with the
  threshold P_cut); grad E = sum_{n >= n_cut} x~_n^m Y_n^m on the grid
  (perfect low-pass filter);
  w = -(I - n n) grad E, n = X_t x X_p / |X_t x X_p|;
  A alpha = b, A = [[X_t.X_t, X_t.X_p], [X_t.X_p, X_p.X_p]], b = (w.X_t, w.X_p);
  (theta*, phi*) += dtau alpha (forward Euler);
then x~ and g = (I - n n) grad E at the new angles; stop when max |g| < eps
or after i_max - 1 moves. Finally x~ and Gamma~ = Gamma0(theta*, phi*) are
analysed on the degree-q grid and truncated to degree p.

Readings (each listed in the design doc):
- grad E of the spectral energy sum a_nm |x_n^m|^2 is the filtered field
  sum a_nm x_n^m Y_n^m (its L2 gradient up to a factor 2, absorbed in dtau).
- The chain rule is applied to the fixed initial expansion: X_t, X_p are the
  derivatives of x0 at the current angles.
- |x_n^m| is the Euclidean norm of the 3-vector coefficient; the sum over
  m = -n..n counts m > 0 twice (real fields).
- No l in 2..q below the threshold: n_cut = q + 1 (nothing is filtered).
- Angles leaving [0, pi] are taken across the pole: theta -> -theta or
  2 pi - theta, phi -> phi + pi (the same surface point).
- ||g|| is the largest Euclidean norm of g over the nodes.
- The paper's values: U_rep = 2, dtau = 1, i_max = 30; P_cut and eps are
  not stated and are inputs.
"""
from __future__ import annotations

import numpy as np

from . import analyze, eval_points_d, gauss_legendre, ncoef, synth


def pad(c, p, q):
    """Coefficients of degree p zero-padded to degree q (last two axes (ncoef, 2))."""
    c = np.asarray(c, dtype=float)
    out = np.zeros(c.shape[:-2] + (ncoef(q), 2))
    out[..., :ncoef(p), :] = c
    return out


def truncate(c, q, p):
    return np.asarray(c)[..., :ncoef(p), :].copy()


def ncutoff(q, xc, P_cut):
    """Adaptive cutoff: the smallest l in 2..q with N2(l)/N1 < P_cut, where
    N2(l) = sum_{n >= l} sum_{|m| <= n} |x_n^m| and N1 = N2(1)."""
    xc = np.asarray(xc, dtype=float)
    mag = np.zeros(q + 1)
    for n in range(q + 1):
        for m in range(n + 1):
            e = n * (n + 1) // 2 + m
            v = np.sqrt(np.sum(xc[:, e, :] ** 2))
            mag[n] += v if m == 0 else 2.0 * v
    N1 = mag[1:].sum()
    for l in range(2, q + 1):
        if mag[l:].sum() < P_cut * N1:
            return l
    return q + 1


def highpass(xc, q, ncut):
    out = np.array(xc, dtype=float)
    out[:, :ncoef(ncut - 1), :] = 0.0      # degrees n < ncut
    return out


def grid_angles(q):
    t, _ = gauss_legendre(q)
    th = np.arccos(np.asarray(t))          # ascending theta (descending t)
    if th[0] > th[-1]:
        th = th[::-1]
    ph = np.pi * np.arange(2 * q) / q
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    return TH.ravel(), PH.ravel()


def _eval(q, c3, th, ph):
    """Values and angle derivatives of a 3-component degree-q expansion."""
    X = np.stack([eval_points_d(q, c3[k], th, ph, 0, 0) for k in range(3)])
    Xt = np.stack([eval_points_d(q, c3[k], th, ph, 1, 0) for k in range(3)])
    Xp = np.stack([eval_points_d(q, c3[k], th, ph, 0, 1) for k in range(3)])
    return X, Xt, Xp


def _wrap(th, ph):
    th = th.copy()
    ph = ph.copy()
    lo = th < 0.0
    th[lo] = -th[lo]
    ph[lo] += np.pi
    hi = th > np.pi
    th[hi] = 2.0 * np.pi - th[hi]
    ph[hi] += np.pi
    return th, np.mod(ph, 2.0 * np.pi)


def _gradient(q, X, Xt, Xp, P_cut):
    """x~ coefficients, n_cut, and g = (I - n n) grad E at the nodes."""
    xt_c = np.stack([analyze(X[k].reshape(q + 1, 2 * q), q, q) for k in range(3)])
    nc = ncutoff(q, xt_c, P_cut)
    hp = highpass(xt_c, q, nc)
    gE = np.stack([synth(q, hp[k], q).ravel() for k in range(3)])
    N = np.cross(Xt.T, Xp.T).T
    n = N / np.linalg.norm(N, axis=0)
    g = gE - n * np.sum(n * gE, axis=0)
    return xt_c, nc, g


def reparametrize(p, xc, gc=None, U_rep=2, P_cut=1e-3, eps=1e-10, imax=30, dtau=1.0):
    """Algorithm 2 on one drop. Returns (x coefficients (3, ncoef(p), 2),
    Gamma coefficients or None, report)."""
    q = U_rep * p
    x0 = pad(xc, p, q)
    g0 = pad(gc, p, q) if gc is not None else None
    th, ph = grid_angles(q)
    X, Xt, Xp = _eval(q, x0, th, ph)
    xt_c, nc, g = _gradient(q, X, Xt, Xp, P_cut)
    hist = [float(np.linalg.norm(g, axis=0).max())]
    moves = 0
    i = 0
    while True:
        i += 1
        if i >= imax:
            break
        w = -g
        A00 = np.sum(Xt * Xt, axis=0)
        A01 = np.sum(Xt * Xp, axis=0)
        A11 = np.sum(Xp * Xp, axis=0)
        b0 = np.sum(w * Xt, axis=0)
        b1 = np.sum(w * Xp, axis=0)
        det = A00 * A11 - A01 * A01
        at = (A11 * b0 - A01 * b1) / det
        ap = (A00 * b1 - A01 * b0) / det
        th, ph = _wrap(th + dtau * at, ph + dtau * ap)
        moves += 1
        X, Xt, Xp = _eval(q, x0, th, ph)
        xt_c, nc, g = _gradient(q, X, Xt, Xp, P_cut)
        hist.append(float(np.linalg.norm(g, axis=0).max()))
        if hist[-1] < eps:
            break
    x_new = truncate(xt_c, q, p)
    g_new = None
    if g0 is not None:
        G = eval_points_d(q, g0, th, ph, 0, 0)
        g_new = truncate(analyze(G.reshape(q + 1, 2 * q), q, q), q, p)
    return x_new, g_new, {"moves": moves, "gnorm": hist, "ncut": nc, "theta": th, "phi": ph,
                          "x_nodes": X}
