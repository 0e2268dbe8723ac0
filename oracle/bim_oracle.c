/*
 * bim_oracle.c -- plain, slow FP64 CPU oracle for the Stokes layer potentials
 * over spherical-harmonic drop surfaces, written from
 *   C. Sorgentone, A.-K. Tornberg, "A highly accurate boundary integral
 *   equation method for surfactant-laden drops in 3D" (arXiv:1707.02156).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline of the benchmark may load this library. The product path (the HIP
 * library) never calls it, and the two share no code, tables or headers.
 *
 * Everything is FP64 except the Wigner small-d matrices, which follow the
 * explicit sum of Appendix B evaluated in __float128 (the sum cancels
 * catastrophically in FP64 beyond degree ~24) and are then rounded to double.
 *
 * Conventions (readings of the paper, each one pinned by a test):
 *  - Grid of degree q: q+1 Gauss-Legendre nodes t_j in cos(theta), ordered
 *    with theta ascending (t descending), times 2q uniform phi_k = pi k / q
 *    (Sec. 2.1; the weight pi/q of the regular rule fixes 2q points).
 *  - Basis Y_n^m = Ptilde_n^m(cos theta) e^{i m phi}, orthonormal with the
 *    Condon-Shortley phase (Sec. 1.1, Appendix A).
 *  - A real field is stored by its m >= 0 coefficients as interleaved
 *    (re, im) doubles at complex index n(n+1)/2 + m; f_n^{-m} = (-1)^m conj f_n^m
 *    (Sec. 1.2).
 *  - Analysis halves the weight of |m| = q, where sin(q phi) vanishes on the
 *    grid (discrete orthogonality of Sec. 2.1 fails only for that pair).
 *  - Outward normal n = x_theta x x_phi / W, mean curvature
 *    K = -(EN - 2FM + GL) / (2 W^2) (= +1/R on a sphere), Table 2 with the
 *    labels of the two curvatures exchanged and the normal flipped outward.
 *  - Singular rule (Sec. 2.2, Theorem 1): node weight
 *    (pi/q) w_j^G [sum_{n<=q} P_n(t_j)] 2 sin(theta_j/2) / sin(theta_j),
 *    i.e. 1/sin(theta) counted once.
 *  - Rotation (Appendix B) with gamma = 0: the rotated field is
 *    f'(s) = f(R_z(phi_k) R_y(theta_j) s), whose coefficients are
 *    f'^mu_n = sum_nu e^{i nu phi_k} d_n^{nu,mu}(theta_j) f_n^nu, with d the
 *    Appendix B matrix read with (m', m) := (nu, mu).
 */
#include <math.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

static inline int tri(int n, int m) { return n * (n + 1) / 2 + m; }
static inline int ncoef(int p) { return (p + 1) * (p + 2) / 2; }

int orc_num_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------
 * Gauss-Legendre nodes and weights on [-1, 1] (Sec. 2.1): Newton's method on
 * the Legendre polynomial P_{N}, N = q + 1, evaluated by Bonnet's recursion.
 * Nodes are returned descending in t, i.e. ascending in theta = acos t.
 * ---------------------------------------------------------------------- */
void orc_gauss_legendre(int q, double *t, double *w)
{
    const int N = q + 1;
    for (int i = 0; i < N; ++i) {
        double x = cos(M_PI * (i + 0.75) / (N + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= N; ++k) {
                double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            if (N == 1) { p1 = x; p0 = 1.0; }
            /* derivative of P_N from (x^2 - 1) P_N' = N (x P_N - P_{N-1}) */
            dp = N * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        /* recompute the derivative at the converged node */
        {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= N; ++k) {
                double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            if (N == 1) { p1 = x; p0 = 1.0; }
            dp = N * (x * p1 - p0) / (x * x - 1.0);
        }
        t[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

/* ------------------------------------------------------------------------
 * Normalized associated Legendre functions Ptilde_n^m(t), 0 <= m <= n <= nmax,
 * by the four recursions of Appendix A. P[tri(n,m)].
 * ---------------------------------------------------------------------- */
void orc_legendre(int nmax, double t, double *P)
{
    const double s = sqrt(fmax(0.0, 1.0 - t * t));
    P[tri(0, 0)] = sqrt(1.0 / (4.0 * M_PI));
    for (int m = 1; m <= nmax; ++m)
        P[tri(m, m)] = -sqrt(1.0 + 1.0 / (2.0 * m)) * s * P[tri(m - 1, m - 1)];
    for (int m = 0; m < nmax; ++m)
        P[tri(m + 1, m)] = sqrt(2.0 * m + 3.0) * t * P[tri(m, m)];
    for (int m = 0; m <= nmax; ++m)
        for (int n = m + 2; n <= nmax; ++n) {
            double a = sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
            double b = -sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) /
                             (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
            P[tri(n, m)] = a * (t * P[tri(n - 1, m)] + b * P[tri(n - 2, m)]);
        }
}

/* theta-derivatives of Ptilde_n^m(cos theta) at an interior node t = cos theta.
 * First derivative from the t-derivative identity
 *   (1 - t^2) dPtilde_n^m/dt = sqrt((2n+1)(n^2-m^2)/(2n-1)) Ptilde_{n-1}^m - n t Ptilde_n^m
 * and d/dtheta = -sin(theta) d/dt; second derivative from the associated
 * Legendre equation  P'' = -cot(theta) P' - (n(n+1) - m^2/sin^2 theta) P.
 * (Appendix A prints these derivatives with garbles; this is the reading.) */
void orc_legendre_dtheta(int nmax, double t, const double *P, double *D1, double *D2)
{
    const double s = sqrt(1.0 - t * t);
    const double cot = t / s;
    for (int m = 0; m <= nmax; ++m)
        for (int n = m; n <= nmax; ++n) {
            double prev = (n - 1 >= m) ? P[tri(n - 1, m)] : 0.0;
            double c = (n > m) ? sqrt((2.0 * n + 1.0) * ((double)n * n - (double)m * m) / (2.0 * n - 1.0)) : 0.0;
            double d1 = -(c * prev - n * t * P[tri(n, m)]) / s;
            D1[tri(n, m)] = d1;
            if (D2)
                D2[tri(n, m)] = -cot * d1 - (n * (n + 1.0) - (double)m * m / (s * s)) * P[tri(n, m)];
        }
}

/* Legendre polynomial sum  sum_{n=0}^{q} P_n(t)  (Theorem 1 weights). */
static double legendre_poly_sum(int q, double t)
{
    double p0 = 1.0, p1 = t, sum = 1.0;
    if (q >= 1) sum += t;
    for (int k = 2; k <= q; ++k) {
        double pk = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
        sum += pk;
    }
    return sum;
}

/* ------------------------------------------------------------------------
 * A grid of degree q with Legendre tables for degrees up to nmax.
 * ---------------------------------------------------------------------- */
typedef struct {
    int q, nmax, nth, nph;
    double *t, *w, *th, *ph;
    double *P, *D1, *D2; /* [j][tri(n,m)] */
} grid_t;

static void grid_init(grid_t *g, int q, int nmax)
{
    g->q = q;
    g->nmax = nmax;
    g->nth = q + 1;
    g->nph = 2 * q;
    g->t = malloc(sizeof(double) * g->nth);
    g->w = malloc(sizeof(double) * g->nth);
    g->th = malloc(sizeof(double) * g->nth);
    g->ph = malloc(sizeof(double) * g->nph);
    orc_gauss_legendre(q, g->t, g->w);
    for (int j = 0; j < g->nth; ++j) g->th[j] = acos(g->t[j]);
    for (int k = 0; k < g->nph; ++k) g->ph[k] = M_PI * k / q;
    const int nc = ncoef(nmax);
    g->P = malloc(sizeof(double) * nc * g->nth);
    g->D1 = malloc(sizeof(double) * nc * g->nth);
    g->D2 = malloc(sizeof(double) * nc * g->nth);
    for (int j = 0; j < g->nth; ++j) {
        orc_legendre(nmax, g->t[j], g->P + (size_t)j * nc);
        orc_legendre_dtheta(nmax, g->t[j], g->P + (size_t)j * nc, g->D1 + (size_t)j * nc,
                            g->D2 + (size_t)j * nc);
    }
}

static void grid_free(grid_t *g)
{
    free(g->t); free(g->w); free(g->th); free(g->ph);
    free(g->P); free(g->D1); free(g->D2);
}

/* ------------------------------------------------------------------------
 * Synthesis (Sec. 1.1, eq. of the truncated expansion; Appendix A for the
 * derivatives): values of the degree-p real field c, or of its derivative
 * d^dt/dtheta^dt d^dp/dphi^dp, at every node of the degree-q grid g.
 * out[j * 2q + k]. The double sum over (n, m) is evaluated with the m-sum
 * outermost: for each latitude and order, sum over n, then over m.
 * ---------------------------------------------------------------------- */
static void synth_on_grid(int p, const double *c, const grid_t *g, int dt, int dp, double *out)
{
    const int nc = ncoef(g->nmax);
    double *Gr = malloc(sizeof(double) * (p + 1));
    double *Gi = malloc(sizeof(double) * (p + 1));
    for (int j = 0; j < g->nth; ++j) {
        const double *L = (dt == 0 ? g->P : dt == 1 ? g->D1 : g->D2) + (size_t)j * nc;
        for (int m = 0; m <= p; ++m) {
            double sr = 0.0, si = 0.0;
            for (int n = m; n <= p; ++n) {
                sr += c[2 * tri(n, m)] * L[tri(n, m)];
                si += c[2 * tri(n, m) + 1] * L[tri(n, m)];
            }
            Gr[m] = sr;
            Gi[m] = si;
        }
        for (int k = 0; k < g->nph; ++k) {
            double v = 0.0;
            for (int m = 0; m <= p; ++m) {
                /* Re[(i m)^dp G_m e^{i m phi}] */
                double cr = cos(m * g->ph[k]), sn = sin(m * g->ph[k]);
                double ar = Gr[m], ai = Gi[m];
                for (int r = 0; r < dp; ++r) { double tr = -m * ai; ai = m * ar; ar = tr; }
                double re = ar * cr - ai * sn;
                v += (m == 0 ? 1.0 : 2.0) * re;
            }
            out[(size_t)j * g->nph + k] = v;
        }
    }
    free(Gr);
    free(Gi);
}

/* Analysis, the discrete transform of Sec. 2.1 with weight (pi/q) w_j^G:
 * coefficients up to degree p of the field f sampled on the degree-q grid.
 * The weight of order m = q is halved (reading, see the header). */
static void analyze_on_grid(const grid_t *g, const double *f, int p, double *c)
{
    const int nc = ncoef(g->nmax);
    const int q = g->q;
    memset(c, 0, sizeof(double) * 2 * ncoef(p));
    for (int m = 0; m <= p; ++m) {
        for (int j = 0; j < g->nth; ++j) {
            double Fr = 0.0, Fi = 0.0;
            for (int k = 0; k < g->nph; ++k) {
                Fr += f[(size_t)j * g->nph + k] * cos(m * g->ph[k]);
                Fi -= f[(size_t)j * g->nph + k] * sin(m * g->ph[k]);
            }
            double wj = M_PI / q * g->w[j] * (m == q ? 0.5 : 1.0);
            const double *L = g->P + (size_t)j * nc;
            for (int n = m; n <= p; ++n) {
                c[2 * tri(n, m)] += wj * L[tri(n, m)] * Fr;
                c[2 * tri(n, m) + 1] += wj * L[tri(n, m)] * Fi;
            }
        }
    }
}

void orc_synth(int p, const double *c, int q, int dt, int dp, double *out)
{
    grid_t g;
    grid_init(&g, q, p);
    synth_on_grid(p, c, &g, dt, dp, out);
    grid_free(&g);
}

void orc_analyze(int q, const double *f, int p, double *c)
{
    grid_t g;
    grid_init(&g, q, p);
    analyze_on_grid(&g, f, p, c);
    grid_free(&g);
}

/* Point evaluation of a degree-p real field at (theta, phi), direct sum. */
double orc_eval_point(int p, const double *c, double theta, double phi)
{
    double *P = malloc(sizeof(double) * ncoef(p));
    orc_legendre(p, cos(theta), P);
    double v = 0.0;
    for (int n = 0; n <= p; ++n)
        for (int m = 0; m <= n; ++m) {
            double re = c[2 * tri(n, m)] * cos(m * phi) - c[2 * tri(n, m) + 1] * sin(m * phi);
            v += (m == 0 ? 1.0 : 2.0) * re * P[tri(n, m)];
        }
    free(P);
    return v;
}

/* ------------------------------------------------------------------------
 * Wigner small-d (Appendix B), explicit sum in __float128:
 * d_n^{m',m}(beta) for -n <= m', m <= n, beta given by cos(beta).
 * ---------------------------------------------------------------------- */
static __float128 qfact[512];
static int qfact_ready = 0;

static void qfact_init(void)
{
    if (qfact_ready) return;
    qfact[0] = 1.0Q;
    for (int i = 1; i < 512; ++i) qfact[i] = qfact[i - 1] * (__float128)i;
    qfact_ready = 1;
}

static double wigner_appB(int n, int mp, int m, const __float128 *cpow, const __float128 *spow)
{
    int s0 = (m - mp > 0) ? m - mp : 0;
    int s1 = (n + m < n - mp) ? n + m : n - mp;
    __float128 S = 0.0Q;
    for (int s = s0; s <= s1; ++s) {
        __float128 term = cpow[2 * (n - s) + m - mp] * spow[2 * s - m + mp] /
                          (qfact[n + m - s] * qfact[s] * qfact[mp - m + s] * qfact[n - mp - s]);
        S += (s & 1) ? -term : term;
    }
    __float128 pre = sqrtq(qfact[n + mp] * qfact[n - mp] * qfact[n + m] * qfact[n - m]);
    if ((mp - m) & 1) pre = -pre;
    return (double)(pre * S);
}

/* Full (2n+1)^2 matrix, d[(m'+n)(2n+1) + (m+n)], at cos(beta) = t. */
void orc_wigner_d(int n, double t, double *d)
{
    qfact_init();
    __float128 tq = (__float128)t;
    __float128 cb = sqrtq((1.0Q + tq) / 2.0Q), sb = sqrtq((1.0Q - tq) / 2.0Q);
    __float128 *cpow = malloc(sizeof(__float128) * (4 * n + 2));
    __float128 *spow = malloc(sizeof(__float128) * (4 * n + 2));
    cpow[0] = spow[0] = 1.0Q;
    for (int k = 1; k < 4 * n + 2; ++k) { cpow[k] = cpow[k - 1] * cb; spow[k] = spow[k - 1] * sb; }
    for (int mp = -n; mp <= n; ++mp)
        for (int m = -n; m <= n; ++m)
            d[(mp + n) * (2 * n + 1) + (m + n)] = wigner_appB(n, mp, m, cpow, spow);
    free(cpow);
    free(spow);
}

/* Per-degree cache of d_n^{nu,mu}(theta_j), nu in [-n,n], mu in [0,n], for every
 * latitude of the degree-p grid (the only rotations the singular rule needs). */
typedef struct { int p; double *d; size_t *off; } wig_cache_t;
static wig_cache_t wcache[8];
static int wcache_n = 0;

static size_t wig_lat_size(int p)
{
    size_t s = 0;
    for (int n = 0; n <= p; ++n) s += (size_t)(2 * n + 1) * (n + 1);
    return s;
}

static const wig_cache_t *wigner_tables(int p, const double *t)
{
    for (int i = 0; i < wcache_n; ++i)
        if (wcache[i].p == p) return &wcache[i];
    qfact_init();
    wig_cache_t *wc = &wcache[wcache_n % 8];
    if (wcache_n >= 8) { free(wc->d); free(wc->off); }
    wc->p = p;
    wc->off = malloc(sizeof(size_t) * (p + 2));
    wc->off[0] = 0;
    for (int n = 0; n <= p; ++n) wc->off[n + 1] = wc->off[n] + (size_t)(2 * n + 1) * (n + 1);
    const size_t per = wig_lat_size(p);
    wc->d = malloc(sizeof(double) * per * (p + 1));
#pragma omp parallel for schedule(dynamic)
    for (int j = 0; j <= p; ++j) {
        __float128 tq = (__float128)t[j];
        __float128 cb = sqrtq((1.0Q + tq) / 2.0Q), sb = sqrtq((1.0Q - tq) / 2.0Q);
        __float128 *cpow = malloc(sizeof(__float128) * (4 * p + 2));
        __float128 *spow = malloc(sizeof(__float128) * (4 * p + 2));
        cpow[0] = spow[0] = 1.0Q;
        for (int k = 1; k < 4 * p + 2; ++k) { cpow[k] = cpow[k - 1] * cb; spow[k] = spow[k - 1] * sb; }
        double *dj = wc->d + per * j;
        for (int n = 0; n <= p; ++n)
            for (int nu = -n; nu <= n; ++nu)
                for (int mu = 0; mu <= n; ++mu)
                    dj[wc->off[n] + (size_t)(nu + n) * (n + 1) + mu] = wigner_appB(n, nu, mu, cpow, spow);
        free(cpow);
        free(spow);
    }
    ++wcache_n;
    return wc;
}

/* Rotation of a degree-p real field so that the point (theta_j, phi) of the
 * degree-p grid moves to the north pole (Appendix B, gamma = 0). */
static void rotate_with(int p, const double *c, const double *dj, const size_t *off, double phi, double *out)
{
    for (int n = 0; n <= p; ++n)
        for (int mu = 0; mu <= n; ++mu) {
            double sr = 0.0, si = 0.0;
            for (int nu = -n; nu <= n; ++nu) {
                int a = nu < 0 ? -nu : nu;
                double fr = c[2 * tri(n, a)], fi = c[2 * tri(n, a) + 1];
                if (nu < 0) { /* f_n^{-a} = (-1)^a conj(f_n^a) */
                    double sg = (a & 1) ? -1.0 : 1.0;
                    fr = sg * fr;
                    fi = -sg * fi;
                }
                double cr = cos(nu * phi), sn = sin(nu * phi);
                double d = dj[off[n] + (size_t)(nu + n) * (n + 1) + mu];
                sr += d * (cr * fr - sn * fi);
                si += d * (sn * fr + cr * fi);
            }
            out[2 * tri(n, mu)] = sr;
            out[2 * tri(n, mu) + 1] = si;
        }
}

/* Rotation about an arbitrary (beta, alpha) via the full App-B matrices; used
 * by the pin tests (resample-and-evaluate brute force). */
void orc_rotate(int p, const double *c, double beta, double alpha, double *out)
{
    for (int n = 0; n <= p; ++n) {
        double *d = malloc(sizeof(double) * (2 * n + 1) * (2 * n + 1));
        orc_wigner_d(n, cos(beta), d);
        for (int mu = 0; mu <= n; ++mu) {
            double sr = 0.0, si = 0.0;
            for (int nu = -n; nu <= n; ++nu) {
                int a = nu < 0 ? -nu : nu;
                double fr = c[2 * tri(n, a)], fi = c[2 * tri(n, a) + 1];
                if (nu < 0) {
                    double sg = (a & 1) ? -1.0 : 1.0;
                    fr = sg * fr;
                    fi = -sg * fi;
                }
                double cr = cos(nu * alpha), sn = sin(nu * alpha);
                double dd = d[(nu + n) * (2 * n + 1) + (mu + n)];
                sr += dd * (cr * fr - sn * fi);
                si += dd * (sn * fr + cr * fi);
            }
            out[2 * tri(n, mu)] = sr;
            out[2 * tri(n, mu) + 1] = si;
        }
        free(d);
    }
}

/* ------------------------------------------------------------------------
 * Geometry on a grid (Table 2, with the readings of the header).
 * xc: 3 components, each 2*ncoef(p) doubles. Outputs per node (may be NULL):
 * W, N = x_theta x x_phi (3 comps, = W n), K (mean curvature), and
 * the metric (E, F, G) and the tangents.
 * ---------------------------------------------------------------------- */
typedef struct {
    int n;
    double *x[3], *xt[3], *xp[3], *xtt[3], *xtp[3], *xpp[3];
} surf_t;

static void surf_synth(surf_t *s, int p, const double *xc, const grid_t *g, int second)
{
    const int nn = g->nth * g->nph;
    const int stride = 2 * ncoef(p);
    s->n = nn;
    for (int c = 0; c < 3; ++c) {
        s->x[c] = malloc(sizeof(double) * nn);
        s->xt[c] = malloc(sizeof(double) * nn);
        s->xp[c] = malloc(sizeof(double) * nn);
        synth_on_grid(p, xc + c * stride, g, 0, 0, s->x[c]);
        synth_on_grid(p, xc + c * stride, g, 1, 0, s->xt[c]);
        synth_on_grid(p, xc + c * stride, g, 0, 1, s->xp[c]);
        if (second) {
            s->xtt[c] = malloc(sizeof(double) * nn);
            s->xtp[c] = malloc(sizeof(double) * nn);
            s->xpp[c] = malloc(sizeof(double) * nn);
            synth_on_grid(p, xc + c * stride, g, 2, 0, s->xtt[c]);
            synth_on_grid(p, xc + c * stride, g, 1, 1, s->xtp[c]);
            synth_on_grid(p, xc + c * stride, g, 0, 2, s->xpp[c]);
        } else {
            s->xtt[c] = s->xtp[c] = s->xpp[c] = NULL;
        }
    }
}

static void surf_free(surf_t *s)
{
    for (int c = 0; c < 3; ++c) {
        free(s->x[c]); free(s->xt[c]); free(s->xp[c]);
        free(s->xtt[c]); free(s->xtp[c]); free(s->xpp[c]);
    }
}

static inline void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Per-node geometry from a synthesized surface (first and second forms). */
static void node_geometry(const surf_t *s, int i, double *W, double *nrm, double *K,
                          double *E_, double *F_, double *G_, double *xt, double *xp)
{
    double a[3], b[3];
    for (int c = 0; c < 3; ++c) { a[c] = s->xt[c][i]; b[c] = s->xp[c][i]; }
    double E = dot3(b, b), F = dot3(b, a), G = dot3(a, a);
    double w = sqrt(E * G - F * F);
    double N[3];
    cross3(a, b, N); /* x_theta x x_phi: outward */
    double n[3] = {N[0] / w, N[1] / w, N[2] / w};
    if (W) *W = w;
    if (nrm) { nrm[0] = n[0]; nrm[1] = n[1]; nrm[2] = n[2]; }
    if (K) {
        double xpp[3], xtp[3], xtt[3];
        for (int c = 0; c < 3; ++c) { xpp[c] = s->xpp[c][i]; xtp[c] = s->xtp[c][i]; xtt[c] = s->xtt[c][i]; }
        double L = dot3(xpp, n), M = dot3(xtp, n), Nn = dot3(xtt, n);
        *K = -(E * Nn - 2.0 * F * M + G * L) / (2.0 * w * w);
    }
    if (E_) *E_ = E;
    if (F_) *F_ = F;
    if (G_) *G_ = G;
    if (xt) { xt[0] = a[0]; xt[1] = a[1]; xt[2] = a[2]; }
    if (xp) { xp[0] = b[0]; xp[1] = b[1]; xp[2] = b[2]; }
}

/* Geometry of a degree-p surface on the degree-q grid. Arrays of (q+1)*2q:
 * x (3), n (3), W, K. Any output may be NULL. */
void orc_geometry(int p, const double *xc, int q, double *x, double *nrm, double *W, double *K)
{
    grid_t g;
    grid_init(&g, q, p);
    surf_t s;
    surf_synth(&s, p, xc, &g, 1);
    for (int i = 0; i < s.n; ++i) {
        double w, n[3], k;
        node_geometry(&s, i, &w, n, &k, NULL, NULL, NULL, NULL, NULL);
        for (int c = 0; c < 3; ++c) {
            if (x) x[(size_t)c * s.n + i] = s.x[c][i];
            if (nrm) nrm[(size_t)c * s.n + i] = n[c];
        }
        if (W) W[i] = w;
        if (K) K[i] = k;
    }
    surf_free(&s);
    grid_free(&g);
}

/* Regular quadrature (Sec. 2.1) of a grid function g times the area element
 * over the degree-q grid: sum_jk (pi/q) w_j^G / sin(theta_j) g_jk W_jk. */
double orc_surface_integral(int p, const double *xc, int q, const double *gfun)
{
    grid_t g;
    grid_init(&g, q, p);
    surf_t s;
    surf_synth(&s, p, xc, &g, 0);
    double acc = 0.0;
    for (int j = 0; j < g.nth; ++j)
        for (int k = 0; k < g.nph; ++k) {
            int i = j * g.nph + k;
            double w;
            node_geometry(&s, i, &w, NULL, NULL, NULL, NULL, NULL, NULL, NULL);
            acc += M_PI / q * g.w[j] / sin(g.th[j]) * (gfun ? gfun[i] : 1.0) * w;
        }
    surf_free(&s);
    grid_free(&g);
    return acc;
}

/* Enclosed volume V = (1/3) int x . n dS by the regular rule on the degree-q grid. */
double orc_volume(int p, const double *xc, int q)
{
    grid_t g;
    grid_init(&g, q, p);
    surf_t s;
    surf_synth(&s, p, xc, &g, 0);
    double acc = 0.0;
    for (int j = 0; j < g.nth; ++j)
        for (int k = 0; k < g.nph; ++k) {
            int i = j * g.nph + k;
            double a[3], b[3], N[3], x[3];
            for (int c = 0; c < 3; ++c) { a[c] = s.xt[c][i]; b[c] = s.xp[c][i]; x[c] = s.x[c][i]; }
            cross3(a, b, N);
            acc += M_PI / q * g.w[j] / sin(g.th[j]) * dot3(x, N) / 3.0;
        }
    surf_free(&s);
    grid_free(&g);
    return acc;
}

/* ------------------------------------------------------------------------
 * Interfacial force (Sec. 1, jump condition; equation of state of Sec. 1):
 *   f = 2 sigma K n - grad_gamma sigma,
 *   grad_gamma sigma = [(G s_phi - F s_theta) x_phi + (E s_theta - F s_phi) x_theta] / W^2,
 * with E, F, G of Table 2. Computed on the degree-(ugeom*p) grid and analysed
 * back to degree p (Sec. 1.3: upsample, non-linear operation, downsample).
 * eos: 0 uniform sigma = sigma0; 1 linear sigma = 1 - E xs Gamma;
 *      2 Langmuir sigma = 1 + E ln(1 - xs Gamma).
 * gc (Gamma coefficients, degree p) is ignored for eos 0.
 * ---------------------------------------------------------------------- */
void orc_force(int p, const double *xc, const double *gc, int eos, double E, double xs,
               double sigma0, int ugeom, double *fc)
{
    const int q = ugeom * p;
    grid_t g;
    grid_init(&g, q, p);
    surf_t s;
    surf_synth(&s, p, xc, &g, 1);
    const int nn = s.n;
    double *gam = calloc(nn, sizeof(double)), *gt = calloc(nn, sizeof(double)), *gp = calloc(nn, sizeof(double));
    if (eos != 0) {
        synth_on_grid(p, gc, &g, 0, 0, gam);
        synth_on_grid(p, gc, &g, 1, 0, gt);
        synth_on_grid(p, gc, &g, 0, 1, gp);
    }
    double *f[3];
    for (int c = 0; c < 3; ++c) f[c] = malloc(sizeof(double) * nn);
    for (int i = 0; i < nn; ++i) {
        double w, n[3], K, Em, Fm, Gm, xt[3], xp[3];
        node_geometry(&s, i, &w, n, &K, &Em, &Fm, &Gm, xt, xp);
        double sig, dsig; /* sigma and d sigma / d Gamma */
        if (eos == 0) { sig = sigma0; dsig = 0.0; }
        else if (eos == 1) { sig = 1.0 - E * xs * gam[i]; dsig = -E * xs; }
        else { sig = 1.0 + E * log(1.0 - xs * gam[i]); dsig = -E * xs / (1.0 - xs * gam[i]); }
        double st = dsig * gt[i], sp = dsig * gp[i];
        for (int c = 0; c < 3; ++c) {
            double grad = ((Gm * sp - Fm * st) * xp[c] + (Em * st - Fm * sp) * xt[c]) / (w * w);
            f[c][i] = 2.0 * sig * K * n[c] - grad;
        }
    }
    for (int c = 0; c < 3; ++c) analyze_on_grid(&g, f[c], p, fc + (size_t)c * 2 * ncoef(p));
    for (int c = 0; c < 3; ++c) free(f[c]);
    free(gam); free(gt); free(gp);
    surf_free(&s);
    grid_free(&g);
}

/* ------------------------------------------------------------------------
 * Stokeslet and stresslet contributions (Sec. 1, below the integral equation):
 *   G = I/r + xh xh / r^3,  T = -6 xh xh xh / r^5,  xh = x0 - x.
 * SL accumulates  wt * G f ;  DL accumulates  wt_N * (-6) xh (xh.u)(xh.N) / r^5
 * where N = W n is the non-normalized normal and the weight excludes W.
 * ---------------------------------------------------------------------- */
static inline void add_sl(const double *x0, const double *x, const double *f, double wt, double *acc)
{
    double h[3] = {x0[0] - x[0], x0[1] - x[1], x0[2] - x[2]};
    double r2 = dot3(h, h), r = sqrt(r2);
    double hf = dot3(h, f);
    for (int c = 0; c < 3; ++c) acc[c] += wt * (f[c] / r + h[c] * hf / (r2 * r));
}

static inline void add_dl(const double *x0, const double *x, const double *u, const double *N, double wt, double *acc)
{
    double h[3] = {x0[0] - x[0], x0[1] - x[1], x0[2] - x[2]};
    double r2 = dot3(h, h), r = sqrt(r2);
    double hu = dot3(h, u), hn = dot3(h, N);
    double r5 = r2 * r2 * r;
    for (int c = 0; c < 3; ++c) acc[c] += wt * (-6.0) * h[c] * hu * hn / r5;
}

/* ------------------------------------------------------------------------
 * Singular self-integral (Sec. 2.2, Theorem 1 + Appendix B).
 * For each listed target (flat index j*2p + k on the degree-p grid of the
 * drop), rotate x and the density so the target is at the north pole,
 * synthesize on the degree-qs grid, and apply the pole rule.
 * kind 0: SL  int f . G ds       (dens = f coefficients)
 * kind 1: DL  int u . T . n ds   (dens = u coefficients)
 * out[t*3 + c]. Coefficient arrays are 3 components of 2*ncoef(p) doubles.
 * ---------------------------------------------------------------------- */
int orc_singular(int p, int qs, const double *xc, const double *dc, int kind, int nt, const int *tgt, double *out)
{
    if (qs < p) return -1;
    const int stride = 2 * ncoef(p);
    double *tp = malloc(sizeof(double) * (p + 1)), *wp = malloc(sizeof(double) * (p + 1));
    orc_gauss_legendre(p, tp, wp);
    const wig_cache_t *wc = wigner_tables(p, tp);
    const size_t per = wig_lat_size(p);
    grid_t gs;
    grid_init(&gs, qs, p);
    double *omega = malloc(sizeof(double) * gs.nth);
    for (int j = 0; j < gs.nth; ++j)
        omega[j] = M_PI / qs * gs.w[j] * legendre_poly_sum(qs, gs.t[j]) * 2.0 * sin(gs.th[j] / 2.0) / sin(gs.th[j]);
#pragma omp parallel for schedule(dynamic)
    for (int it = 0; it < nt; ++it) {
        const int j = tgt[it] / (2 * p), k = tgt[it] % (2 * p);
        const double phi = M_PI * k / p;
        const double *dj = wc->d + per * j;
        double *rx = malloc(sizeof(double) * 3 * stride), *rd = malloc(sizeof(double) * 3 * stride);
        for (int c = 0; c < 3; ++c) {
            rotate_with(p, xc + c * stride, dj, wc->off, phi, rx + c * stride);
            rotate_with(p, dc + c * stride, dj, wc->off, phi, rd + c * stride);
        }
        /* pole value of the rotated surface = the target x0 */
        double x0[3] = {0, 0, 0};
        for (int c = 0; c < 3; ++c)
            for (int n = 0; n <= p; ++n) x0[c] += rx[c * stride + 2 * tri(n, 0)] * sqrt((2.0 * n + 1.0) / (4.0 * M_PI));
        surf_t s;
        surf_synth(&s, p, rx, &gs, 0);
        const int nn = s.n;
        double *dv[3];
        for (int c = 0; c < 3; ++c) {
            dv[c] = malloc(sizeof(double) * nn);
            synth_on_grid(p, rd + c * stride, &gs, 0, 0, dv[c]);
        }
        double acc[3] = {0, 0, 0};
        for (int jj = 0; jj < gs.nth; ++jj)
            for (int kk = 0; kk < gs.nph; ++kk) {
                int i = jj * gs.nph + kk;
                double x[3] = {s.x[0][i], s.x[1][i], s.x[2][i]};
                double a[3] = {s.xt[0][i], s.xt[1][i], s.xt[2][i]};
                double b[3] = {s.xp[0][i], s.xp[1][i], s.xp[2][i]};
                double N[3];
                cross3(a, b, N);
                double d[3] = {dv[0][i], dv[1][i], dv[2][i]};
                if (kind == 0) add_sl(x0, x, d, omega[jj] * sqrt(dot3(N, N)), acc);
                else add_dl(x0, x, d, N, omega[jj], acc);
            }
        for (int c = 0; c < 3; ++c) out[it * 3 + c] = acc[c];
        for (int c = 0; c < 3; ++c) free(dv[c]);
        surf_free(&s);
        free(rx);
        free(rd);
    }
    free(omega);
    grid_free(&gs);
    free(tp);
    free(wp);
    return 0;
}

/* ------------------------------------------------------------------------
 * Regular quadrature (Sec. 2.1) of the SL or DL kernel of a degree-ps source
 * drop on its degree-q grid (q = ps: standard grid; q = U ps: upsampled grid,
 * Sec. 2.3 region Omega_1), evaluated at arbitrary targets x0[t*3 + c].
 * ---------------------------------------------------------------------- */
int orc_regular(int ps, int q, const double *xc, const double *dc, int kind, int nt, const double *x0, double *out)
{
    if (q < ps) return -1;
    const int stride = 2 * ncoef(ps);
    grid_t g;
    grid_init(&g, q, ps);
    surf_t s;
    surf_synth(&s, ps, xc, &g, 0);
    const int nn = s.n;
    double *dv[3];
    for (int c = 0; c < 3; ++c) {
        dv[c] = malloc(sizeof(double) * nn);
        synth_on_grid(ps, dc + c * stride, &g, 0, 0, dv[c]);
    }
#pragma omp parallel for schedule(static)
    for (int it = 0; it < nt; ++it) {
        double acc[3] = {0, 0, 0};
        for (int jj = 0; jj < g.nth; ++jj) {
            double wj = M_PI / q * g.w[jj] / sin(g.th[jj]);
            for (int kk = 0; kk < g.nph; ++kk) {
                int i = jj * g.nph + kk;
                double x[3] = {s.x[0][i], s.x[1][i], s.x[2][i]};
                double a[3] = {s.xt[0][i], s.xt[1][i], s.xt[2][i]};
                double b[3] = {s.xp[0][i], s.xp[1][i], s.xp[2][i]};
                double N[3];
                cross3(a, b, N);
                double d[3] = {dv[0][i], dv[1][i], dv[2][i]};
                if (kind == 0) add_sl(x0 + 3 * it, x, d, wj * sqrt(dot3(N, N)), acc);
                else add_dl(x0 + 3 * it, x, d, N, wj, acc);
            }
        }
        for (int c = 0; c < 3; ++c) out[it * 3 + c] = acc[c];
    }
    for (int c = 0; c < 3; ++c) free(dv[c]);
    surf_free(&s);
    grid_free(&g);
    return 0;
}

/* Distance from each target to the nearest node of the degree-ps grid of a
 * drop (the node-based distance a cell list yields, Sec. 2.3). */
void orc_min_node_distance(int ps, const double *xc, int nt, const double *x0, double *dist)
{
    double *x = malloc(sizeof(double) * 3 * (ps + 1) * 2 * ps);
    orc_geometry(ps, xc, ps, x, NULL, NULL, NULL);
    const int nn = (ps + 1) * 2 * ps;
#pragma omp parallel for schedule(static)
    for (int it = 0; it < nt; ++it) {
        double best = INFINITY;
        for (int i = 0; i < nn; ++i) {
            double h[3] = {x0[3 * it] - x[i], x0[3 * it + 1] - x[nn + i], x0[3 * it + 2] - x[2 * nn + i]};
            double r = sqrt(dot3(h, h));
            if (r < best) best = r;
        }
        dist[it] = best;
    }
    free(x);
}

/* ------------------------------------------------------------------------
 * Nearest region (Sec. 2.3): closest point on a drop by Newton's method on
 * the gradient of F = |x(theta, phi) - x0|^2 / 2, with the Levenberg-Marquardt
 * shift mu I added to the Hessian when a step does not decrease F (the
 * footnote of Sec. 2.3).
 * ---------------------------------------------------------------------- */

/* d^dt/dtheta^dt d^dp/dphi^dp of a real field at one point (dt <= 2). */
double orc_eval_point_d(int p, const double *c, double theta, double phi, int dt, int dp)
{
    const int nc = ncoef(p);
    double *P = malloc(sizeof(double) * 3 * nc);
    double *D1 = P + nc, *D2 = P + 2 * nc;
    orc_legendre(p, cos(theta), P);
    orc_legendre_dtheta(p, cos(theta), P, D1, D2);
    const double *L = dt == 0 ? P : (dt == 1 ? D1 : D2);
    double v = 0.0;
    for (int n = 0; n <= p; ++n)
        for (int m = 0; m <= n; ++m) {
            /* (i m)^dp e^{i m phi} (re + i im), real part */
            double cr = c[2 * tri(n, m)], ci = c[2 * tri(n, m) + 1];
            double er = cos(m * phi), ei = sin(m * phi);
            double zr = cr * er - ci * ei, zi = cr * ei + ci * er;
            for (int k = 0; k < dp; ++k) {
                double t = -m * zi;
                zi = m * zr;
                zr = t;
            }
            v += (m == 0 ? 1.0 : 2.0) * zr * L[tri(n, m)];
        }
    free(P);
    return v;
}

/* The same at n points (theta[i], phi[i]) into out[i]. */
void orc_eval_points_d(int p, const double *c, int n, const double *theta, const double *phi, int dt, int dp,
                       double *out)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) out[i] = orc_eval_point_d(p, c, theta[i], phi[i], dt, dp);
}

static void surface_point(int p, const double *xc, double th, double ph, double out[6][3])
{
    const int nc2 = 2 * ncoef(p);
    static const int DT[6] = {0, 1, 0, 2, 1, 0}, DP[6] = {0, 0, 1, 0, 1, 2};
    for (int f = 0; f < 6; ++f)
        for (int c = 0; c < 3; ++c) out[f][c] = orc_eval_point_d(p, xc + c * nc2, th, ph, DT[f], DP[f]);
}

/* Closest point of drop (p, xc) to x0 from the start (th0, ph0). Returns the
 * number of iterations; res = {theta, phi, x*[3]}. */
int orc_closest_point(int p, const double *xc, const double *x0, double th0, double ph0, double *res)
{
    double th = th0, ph = ph0, mu = 0.0;
    double S[6][3];
    surface_point(p, xc, th, ph, S);
    double r[3] = {S[0][0] - x0[0], S[0][1] - x0[1], S[0][2] - x0[2]};
    double F = 0.5 * dot3(r, r);
    int it = 0, converged = 0;
    for (; it < 100 && !converged; ++it) {
        const double g0 = dot3(r, S[1]), g1 = dot3(r, S[2]);
        const double H00 = dot3(S[1], S[1]) + dot3(r, S[3]);
        const double H01 = dot3(S[1], S[2]) + dot3(r, S[4]);
        const double H11 = dot3(S[2], S[2]) + dot3(r, S[5]);
        const double scale = dot3(S[1], S[1]) + dot3(S[2], S[2]);
        int accepted = 0;
        for (int tries = 0; tries < 40 && !accepted; ++tries) {
            const double a = H00 + mu * scale, b = H01, d = H11 + mu * scale;
            const double det = a * d - b * b;
            if (!(det > 0.0) || !(a > 0.0)) {  /* not a descent system: raise the shift */
                mu = mu == 0.0 ? 1e-6 : 10.0 * mu;
                continue;
            }
            const double s0 = -(d * g0 - b * g1) / det, s1 = -(a * g1 - b * g0) / det;
            double Sn[6][3];
            surface_point(p, xc, th + s0, ph + s1, Sn);
            double rn[3] = {Sn[0][0] - x0[0], Sn[0][1] - x0[1], Sn[0][2] - x0[2]};
            const double Fn = 0.5 * dot3(rn, rn);
            /* near the minimum F changes by less than its rounding: take the
             * small Newton steps without the decrease test */
            const int local = mu == 0.0 && fabs(s0) + fabs(s1) < 1e-8;
            if (Fn <= F || local) {
                th += s0;
                ph += s1;
                memcpy(S, Sn, sizeof(S));
                memcpy(r, rn, sizeof(r));
                F = Fn;
                mu = mu * 0.1 < 1e-12 ? 0.0 : mu * 0.1;
                accepted = 1;
                converged = fabs(s0) + fabs(s1) < 1e-15;
            } else {
                mu = mu == 0.0 ? 1e-6 : 10.0 * mu;
            }
        }
        if (!accepted) break;  /* no decrease at any shift: at the minimum to rounding */
    }
    res[0] = th;
    res[1] = ph;
    res[2] = S[0][0];
    res[3] = S[0][1];
    res[4] = S[0][2];
    return it;
}

/* Index of the nearest node of the degree-ps grid of a drop to each target. */
void orc_nearest_node(int ps, const double *xc, int nt, const double *x0, int *idx)
{
    double *x = malloc(sizeof(double) * 3 * (ps + 1) * 2 * ps);
    orc_geometry(ps, xc, ps, x, NULL, NULL, NULL);
    const int nn = (ps + 1) * 2 * ps;
#pragma omp parallel for schedule(static)
    for (int it = 0; it < nt; ++it) {
        double best = INFINITY;
        int bi = 0;
        for (int i = 0; i < nn; ++i) {
            double h[3] = {x0[3 * it] - x[i], x0[3 * it + 1] - x[nn + i], x0[3 * it + 2] - x[2 * nn + i]};
            double r = dot3(h, h);
            if (r < best) {
                best = r;
                bi = i;
            }
        }
        idx[it] = bi;
    }
    free(x);
}
