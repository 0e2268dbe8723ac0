"""Seeded synthetic drop configurations (inputs only; no method arithmetic).

Shared by the oracle tests, the HIP parity tests and the benchmark. Every
generator returns plain numpy arrays in the coefficient layout used by both
sides: a real field of degree p is (ncoef(p), 2) with complex index
n(n+1)/2 + m (m >= 0) and [..., 0] = Re, [..., 1] = Im; a vector field is
(3, ncoef(p), 2). The spherical-harmonic basis is orthonormal with the
Condon-Shortley phase, so the unit sphere is

    x = -sqrt(2 pi/3) R  at (n, m) = (1, 1)           (real part)
    y =  sqrt(2 pi/3) R  at (1, 1)                    (imaginary part)
    z =  sqrt(4 pi/3) R  at (1, 0)
    centre c:  sqrt(4 pi) c  at (0, 0).

Random numbers come from numpy's PCG64 with the seed stated per workload.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SQ2PI3 = np.sqrt(2.0 * np.pi / 3.0)
SQ4PI3 = np.sqrt(4.0 * np.pi / 3.0)
SQ4PI = np.sqrt(4.0 * np.pi)


def ncoef(p: int) -> int:
    return (p + 1) * (p + 2) // 2


def idx(n: int, m: int) -> int:
    return n * (n + 1) // 2 + m


@dataclass
class DropSpec:
    p: int
    xc: np.ndarray                 # (3, ncoef(p), 2)
    lam: float = 1.0
    gc: np.ndarray | None = None   # (ncoef(p), 2) or None
    centre: np.ndarray = field(default_factory=lambda: np.zeros(3))
    radius: float = 1.0


@dataclass
class Workload:
    name: str
    drops: list
    eos: int = 0            # 0 uniform, 1 linear, 2 Langmuir
    E: float = 0.0
    xs: float = 0.0
    sigma0: float = 1.0
    A_tilde: float = 5.0
    U_tilde: int = 4
    U_sing: int = 1
    U_geom: int = 2
    U0: tuple = (0.0, 0.0, 0.0)
    gradU: tuple = (0.0,) * 9
    gmres_tol: float = 1e-10
    notes: str = ""


def sphere(p: int, R: float = 1.0, c=(0.0, 0.0, 0.0)) -> np.ndarray:
    xc = np.zeros((3, ncoef(p), 2))
    xc[0, idx(1, 1), 0] = -SQ2PI3 * R
    xc[1, idx(1, 1), 1] = SQ2PI3 * R
    xc[2, idx(1, 0), 0] = SQ4PI3 * R
    for k in range(3):
        xc[k, 0, 0] = SQ4PI * c[k]
    return xc


def _draw_layout(p: int, lmin: int):
    """Destinations of the normal draws of one component, in draw order:
    for l = lmin..p: (l, 0) real, then (l, m) real and imaginary for m = 1..l."""
    key = (p, lmin)
    if key not in _LAYOUT:
        idx, part, lv = [], [], []
        for l in range(lmin, p + 1):
            idx.append(idx_(l, 0)); part.append(0); lv.append(l)
            for m in range(1, l + 1):
                idx += [idx_(l, m), idx_(l, m)]; part += [0, 1]; lv += [l, l]
        _LAYOUT[key] = (np.array(idx), np.array(part), np.array(lv, dtype=float))
    return _LAYOUT[key]


_LAYOUT = {}


def idx_(n: int, m: int) -> int:
    return n * (n + 1) // 2 + m


def perturbation(rng: np.random.Generator, p: int, A: float, lmin: int = 2, power: float = 3.0) -> np.ndarray:
    """Random coefficients N(0,1) A l^-power for lmin <= l <= p on each Cartesian
    component; m = 0 real, m > 0 complex with Re and Im each of variance
    (A l^-power)^2 / 2; Im at m = p zero so the field is representable on the
    degree-p grid. Draw order: component, then l, then (m = 0), (m, Re, Im)."""
    d = np.zeros((3, ncoef(p), 2))
    ii, pp, lv = _draw_layout(p, lmin)
    if len(ii) == 0:
        return d
    scale = A * lv ** (-power)
    half = ii != np.array([idx_(int(l), 0) for l in lv])
    for k in range(3):
        z = rng.standard_normal(len(ii)) * scale
        z[half] = z[half] / np.sqrt(2.0)
        d[k, ii, pp] = z
    d[:, idx_(p, p), 1] = 0.0 if p >= lmin else d[:, idx_(p, p), 1]
    return d


def perturbed_sphere(rng, p, R, c, A):
    """Unit sphere plus perturbation, scaled by R, translated by c."""
    xc = (sphere(p, 1.0) + perturbation(rng, p, A)) * R
    for k in range(3):
        xc[k, 0, 0] += SQ4PI * c[k]
    return xc


def perturbation_bound(d: np.ndarray) -> float:
    """Upper bound of max |dx| over the sphere for a perturbation field d
    (3, ncoef, 2): per component, the sum of coefficient moduli (doubled for
    m > 0) times the sup norm sqrt((2l+1)/4pi) of the basis function."""
    p = int(round((np.sqrt(8 * d.shape[1] + 1) - 3) / 2))
    n = np.concatenate([[l] * (l + 1) for l in range(p + 1)])
    m = np.concatenate([np.arange(l + 1) for l in range(p + 1)])
    w = np.where(m == 0, 1.0, 2.0) * np.sqrt((2 * n + 1) / (4 * np.pi))
    tot = (np.hypot(d[..., 0], d[..., 1]) * w).sum(axis=1)
    return float(np.sqrt(np.sum(tot ** 2)))


def random_centres(rng, radii_bound, box_lo, box_hi, gap, max_tries=200000):
    """Random sequential addition: centre i uniform in [lo_i, hi_i]^3, accepted
    when the bounding-sphere gap to every accepted centre is >= gap."""
    cs = []
    for i, b in enumerate(radii_bound):
        for _ in range(max_tries):
            c = rng.uniform(box_lo[i], box_hi[i], size=3)
            if all(np.linalg.norm(c - cj) - b - radii_bound[j] >= gap for j, cj in enumerate(cs)):
                cs.append(c)
                break
        else:
            raise RuntimeError("random sequential addition failed")
    return np.array(cs)


# ----------------------------------------------------------------------------
# The five workloads.
# ----------------------------------------------------------------------------

def single_drop(p=16, A=0.05, seed=1, perturbed=True) -> Workload:
    """One drop of degree p (default 16): unit sphere plus N(0,1) 0.05 l^-3
    perturbations, lambda 1, uniform tension 1; single-layer velocity at all
    grid points."""
    rng = np.random.default_rng(seed)
    xc = perturbed_sphere(rng, p, 1.0, (0, 0, 0), A) if perturbed else sphere(p)
    return Workload(name=f"single_drop_p{p}", drops=[DropSpec(p, xc, 1.0)], eos=0, sigma0=1.0,
                    notes="uniform tension 1, lambda 1")


def two_drops(p=32, A=0.1, gap=0.2, lams=(1.0, 5.0), seed=2) -> Workload:
    """Two drops of degree p (default 32), perturbations N(0,1) 0.1 l^-3,
    centres 2 + gap apart along x, lambda (1, 5), surfactant
    Gamma = 1 + 0.2 Y_2^0 with the linear equation of state sigma = 1 - E xs Gamma
    (E = 0.5, xs = 0.6), Omega_1 upsampling 4, GMRES tolerance 1e-10."""
    rng = np.random.default_rng(seed)
    drops = []
    for i, c in enumerate([(0.0, 0.0, 0.0), (2.0 + gap, 0.0, 0.0)]):
        xc = perturbed_sphere(rng, p, 1.0, c, A)
        gc = np.zeros((ncoef(p), 2))
        gc[idx(0, 0), 0] = SQ4PI
        gc[idx(2, 0), 0] = 0.2
        drops.append(DropSpec(p, xc, lams[i], gc, np.array(c, float), 1.0))
    return Workload(name=f"two_drops_p{p}", drops=drops, eos=1, E=0.5, xs=0.6, A_tilde=5.0, U_tilde=4,
                    gmres_tol=1e-10, notes="gap 0.2 nominal; Gamma = 1 + 0.2 Y_2^0; sigma = 1 - 0.3 Gamma")


def many_drops(nd=64, p=16, A=0.05, box=12.0, gap=0.3, seed=3) -> Workload:
    """nd drops (default 64) of degree p (default 16), radii U[0.8, 1.2],
    centres uniform in a cube of side 12 by random sequential addition with
    bounding-sphere gap >= 0.3 (restricting centres to [R, 12 - R]^3 would need
    a packing beyond the jamming limit of sequential addition), lambda uniform
    in {1, 2, 5}, uniform tension; every pair on the 2x upsampled grid
    (Omega_1 everywhere)."""
    rng = np.random.default_rng(seed)
    R = rng.uniform(0.8, 1.2, size=nd)
    perts = [perturbation(rng, p, A) for _ in range(nd)]
    shapes = [sphere(p) + d for d in perts]
    bounds = [r * (1.0 + perturbation_bound(d)) for d, r in zip(perts, R)]
    lo = [0.0] * nd
    hi = [box] * nd
    cs = random_centres(rng, bounds, lo, hi, gap)
    lams = rng.choice([1.0, 2.0, 5.0], size=nd)
    drops = []
    for i in range(nd):
        xc = shapes[i] * R[i]
        for k in range(3):
            xc[k, 0, 0] += SQ4PI * cs[i, k]
        drops.append(DropSpec(p, xc, float(lams[i]), None, cs[i], float(R[i])))
    return Workload(name=f"many_drops_n{nd}_p{p}", drops=drops, eos=0, sigma0=1.0, A_tilde=1e30, U_tilde=2,
                    notes="all pairs on the 2x upsampled grid")


def random_rotation(rng) -> np.ndarray:
    """Uniformly distributed rotation matrix (QR of a Gaussian matrix with the
    sign convention that makes the factorisation unique, determinant +1)."""
    Q, Rm = np.linalg.qr(rng.standard_normal((3, 3)))
    Q = Q * np.sign(np.diag(Rm))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def p2_spheroid(p: int, R: float, eps: float) -> np.ndarray:
    """Body-frame surface r(theta) = R (1 + eps P_2(cos theta)) s_hat, exactly a
    degree-3 expansion. With u = cos(theta):
      z = R [(1 + 2 eps/5) P_1(u) + (3 eps/5) P_3(u)]
      sin(theta) (1 + eps P_2(u)) = -(1 - eps/5) P_1^1(u) - (eps/5) P_3^1(u)
    (P_n^m with the Condon-Shortley phase), converted to the orthonormal basis
    with the factors sqrt((2n+1)/(4 pi) (n-m)!/(n+m)!)."""
    xc = np.zeros((3, ncoef(p), 2))
    N10, N30 = np.sqrt(3 / (4 * np.pi)), np.sqrt(7 / (4 * np.pi))
    N11, N31 = np.sqrt(3 / (8 * np.pi)), np.sqrt(7 / (48 * np.pi))
    c1 = -(1.0 - eps / 5.0) / N11
    c3 = -(eps / 5.0) / N31
    # x = h(theta) cos(phi): real part of the m = 1 coefficient is c_n / 2
    xc[0, idx(1, 1), 0] = c1 / 2
    xc[0, idx(3, 1), 0] = c3 / 2
    # y = h(theta) sin(phi): imaginary part -c_n / 2
    xc[1, idx(1, 1), 1] = -c1 / 2
    xc[1, idx(3, 1), 1] = -c3 / 2
    xc[2, idx(1, 0), 0] = (1.0 + 2.0 * eps / 5.0) / N10
    xc[2, idx(3, 0), 0] = (3.0 * eps / 5.0) / N30
    return xc * R


def p2_surface_points(R: float, eps: float, Q: np.ndarray, c, nt: int = 96, nphi: int = 192) -> np.ndarray:
    """Points of the rotated, translated spheroid c + Q r(theta) s_hat on a
    uniform (theta, phi) sample; used only to place drops."""
    th = (np.arange(nt) + 0.5) * np.pi / nt
    ph = np.arange(nphi) * 2 * np.pi / nphi
    T, P = np.meshgrid(th, ph, indexing="ij")
    r = R * (1.0 + eps * 0.5 * (3 * np.cos(T) ** 2 - 1))
    s = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(-1, 3)
    return (r.reshape(-1, 1) * s) @ Q.T + np.asarray(c, float)


def rotate_coefficients(xc: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """Rigid rotation of the surface: every coefficient triple (x, y, z)_n^m is
    multiplied by Q (real and imaginary parts alike)."""
    return np.einsum("ij,jkr->ikr", Q, xc)


def scalar_field(rng, p: int, A: float, power: float, mean: float) -> np.ndarray:
    """Real scalar expansion: mean at l = 0 (times sqrt(4 pi)), N(0,1) A l^-power
    for 1 <= l <= p, split over Re/Im like perturbation(); Im at m = p zero."""
    g = np.zeros((ncoef(p), 2))
    g[0, 0] = SQ4PI * mean
    for l in range(1, p + 1):
        s = A * l ** (-power)
        g[idx(l, 0), 0] = rng.standard_normal() * s
        for m in range(1, l + 1):
            g[idx(l, m), 0] = rng.standard_normal() * s / np.sqrt(2.0)
            g[idx(l, m), 1] = rng.standard_normal() * s / np.sqrt(2.0)
            if m == p:
                g[idx(l, m), 1] = 0.0
    return g


def deformed_drops(npairs=8, p=48, eps=4.0 / 9.0, A=0.05, gap=0.1, spacing=8.0, lam=3.0, seed=5) -> Workload:
    """2 npairs drops (default 16) of degree p (default 48): P_2 spheroids with
    eps = 4/9, i.e. Taylor deformation (L - B)/(L + B) = 0.3, each randomly
    oriented, plus N(0,1) 0.05 l^-3 noise; lambda 3. Drops come in pairs whose
    centres sit on a 2x2x2 lattice of spacing 8; within a pair the separation
    along a random direction is bisected until the noise-free surfaces are 0.1
    apart (sampled surfaces). Surfactant Gamma = 1 + sum_{l>=1} N(0,1) 0.05 l^-2
    Y_l^m of degree p with the linear equation of state sigma = 1 - 0.3 Gamma."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    drops = []
    lattice = [np.array([i, j, k], float) * spacing for i in range(2) for j in range(2) for k in range(2)]
    for pc in lattice[:npairs]:
        Qa, Qb = random_rotation(rng), random_rotation(rng)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        pa = p2_surface_points(1.0, eps, Qa, (0, 0, 0))
        tree = cKDTree(pa[pa @ d > 0])           # the half of A that faces B
        pb0 = p2_surface_points(1.0, eps, Qb, (0, 0, 0))
        pb0 = pb0[pb0 @ d < 0]                   # the half of B that faces A
        lo, hi = 0.5, 2.0 * (1.0 + eps) + gap + 1.0
        for _ in range(44):
            mid = 0.5 * (lo + hi)
            dist = tree.query(pb0 + mid * d, k=1, distance_upper_bound=4.0 * gap)[0].min()
            if dist > gap:
                hi = mid
            else:
                lo = mid
        sep = hi
        for Q, c in ((Qa, pc - 0.5 * sep * d), (Qb, pc + 0.5 * sep * d)):
            xc = rotate_coefficients(p2_spheroid(p, 1.0, eps), Q) + perturbation(rng, p, A)
            for k in range(3):
                xc[k, 0, 0] += SQ4PI * c[k]
            gc = scalar_field(rng, p, 0.05, 2.0, 1.0)
            drops.append(DropSpec(p, xc, lam, gc, c, 1.0))
    return Workload(name=f"deformed_drops_n{2 * npairs}_p{p}", drops=drops, eos=1, E=0.5, xs=0.6, A_tilde=5.0,
                    U_tilde=4, gmres_tol=1e-10,
                    notes="P2 spheroids eps 4/9 (D = 0.3), pairs 0.1 apart (noise-free), lambda 3")


@dataclass
class Request:
    arrival: float          # seconds after the start of the stream (rate 1; scale by 1 / rate)
    drops: list             # DropSpec list
    p: int


def serving_requests(n=2048, A=0.05, gap=0.2, seed=4):
    """A stream of n independent drop systems with Poisson arrivals (unit rate:
    exponential gaps of mean 1, to be divided by the target rate). Each has
    N_d ~ U{1..8} drops of one degree p ~ U{8, 16, 24, 32}, unit radius, N(0,1)
    0.05 l^-3 perturbations, lambda per drop ~ U{1, 2, 5}, centres by random
    sequential addition in a cube of side 4 N_d^(1/3) + 2 with bounding-sphere
    gap >= 0.2; uniform tension 1."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(n):
        t += rng.exponential(1.0)
        nd = int(rng.integers(1, 9))
        p = int(rng.choice([8, 16, 24, 32]))
        perts = [perturbation(rng, p, A) for _ in range(nd)]
        bounds = [1.0 + perturbation_bound(d) for d in perts]
        side = 4.0 * nd ** (1.0 / 3.0) + 2.0
        cs = random_centres(rng, bounds, [0.0] * nd, [side] * nd, gap)
        lams = rng.choice([1.0, 2.0, 5.0], size=nd)
        drops = []
        for i in range(nd):
            xc = sphere(p) + perts[i]
            for k in range(3):
                xc[k, 0, 0] += SQ4PI * cs[i, k]
            drops.append(DropSpec(p, xc, float(lams[i]), None, cs[i], 1.0))
        out.append(Request(t, drops, p))
    return out
