// Nearest-region quadrature (Sec. 2.3) on gfx950, FP64.
//
// A target x0 of drop i whose nearest node of source drop j lies within h_j
// (region Omega_2) gets drop j's contribution from:
//   1. the closest point x* = x_j(theta*, phi*): Newton's method on the
//      gradient of |x_j(theta, phi) - x0|^2 / 2 from the nearest node, with a
//      Levenberg-Marquardt shift mu I when a step does not decrease the
//      distance (the footnote of Sec. 2.3);
//   2. the on-surface value at x* from the expansion of drop j's
//      self-interaction (singular rule at its own nodes, analysed); for the
//      double layer the exterior limit, on-surface value - 4 pi u(x*);
//   3. regular-rule values at x_l = x* + h_j sqrt(l) d, l = 1..L, d the unit
//      vector from x* to x0 (standard grid beyond A h_j, else upsampled);
//   4. Lagrange interpolation in the distance along d, evaluated at |x0 - x*|.
//
// One wavefront per (target, source drop) item. Surface points and their
// derivatives: lane m carries order m of the normalized associated Legendre
// functions (three-term recursion in n), the theta-derivatives come from the
// ladder identity of Appendix A (d/dtheta P_n^m = sqrt((n-m)(n+m+1)) P_n^{m+1}
// + m cot(theta) P_n^m, the neighbour lane holding P_n^{m+1}) and its
// derivative; sums over m by butterfly reductions, so every lane holds the
// same totals and the Newton iteration runs uniformly.
#include "internal.hpp"

#include <hip/hip_runtime.h>

namespace bim {

static constexpr double kPiN = 3.14159265358979323846;

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Surface point and derivatives of a degree-p drop at (th, ph):
// S[0] x, S[1] x_theta, S[2] x_phi, S[3] x_theta theta, S[4] x_theta phi,
// S[5] x_phi phi. Coefficients of component c at xc + c * cs. If Pst is set,
// lanes also store Ptilde_n^m(cos th) at Pst[tri(n, m)].
__device__ void surf_eval(int p, const double *__restrict__ xc, long cs, double th, double ph, double S[6][3],
                          double *Pst)
{
    const int m = threadIdx.x & 63;
    const double t = cos(th), s = sin(th), cot = t / s, is2 = 1.0 / (s * s);
    double pmm = 1.0 / sqrt(4.0 * kPiN);
    for (int k = 1; k <= m; ++k) pmm *= -sqrt((2.0 * k + 1.0) / (2.0 * k)) * s;
    double Pm1 = 0.0, Pm2 = 0.0;
    double G[3][3][2] = {};  // [kind][component][re, im]
    for (int n = 0; n <= p; ++n) {
        double P = 0.0;
        if (n == m) {
            P = pmm;
        } else if (n == m + 1) {
            P = sqrt(2.0 * m + 3.0) * t * pmm;
        } else if (n > m + 1) {
            const double an = sqrt((2.0 * n + 1.0) * (2.0 * n - 1.0) / ((double)(n - m) * (n + m)));
            const double bn = sqrt((2.0 * n + 1.0) * (double)(n + m - 1) * (n - m - 1) /
                                   ((2.0 * n - 3.0) * (double)(n - m) * (n + m)));
            P = an * t * Pm1 - bn * Pm2;
        }
        Pm2 = Pm1;
        Pm1 = P;
        const double lad = n > m ? sqrt((double)(n - m) * (n + m + 1)) : 0.0;
        double Pup = __shfl_down(P, 1, 64);
        if (m + 1 > n) Pup = 0.0;
        const double D1 = lad * Pup + m * cot * P;
        double D1up = __shfl_down(D1, 1, 64);
        if (m + 1 > n) D1up = 0.0;
        const double D2 = lad * D1up - m * is2 * P + m * cot * D1;
        if (n >= m) {
            const int e = n * (n + 1) / 2 + m;
            if (Pst) Pst[e] = P;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double cr = xc[c * cs + 2 * e], ci = xc[c * cs + 2 * e + 1];
                G[0][c][0] = fma(cr, P, G[0][c][0]);
                G[0][c][1] = fma(ci, P, G[0][c][1]);
                G[1][c][0] = fma(cr, D1, G[1][c][0]);
                G[1][c][1] = fma(ci, D1, G[1][c][1]);
                G[2][c][0] = fma(cr, D2, G[2][c][0]);
                G[2][c][1] = fma(ci, D2, G[2][c][1]);
            }
        }
    }
    double sm, cm;
    sincos(m * ph, &sm, &cm);
    const double w = m ? 2.0 : 1.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // Re(g e^{i m phi}) = gr cm - gi sm; Re(i m g e^{i m phi}) = -m (gr sm + gi cm)
        const double r0 = G[0][c][0] * cm - G[0][c][1] * sm, i0 = G[0][c][0] * sm + G[0][c][1] * cm;
        const double r1 = G[1][c][0] * cm - G[1][c][1] * sm, i1 = G[1][c][0] * sm + G[1][c][1] * cm;
        const double r2 = G[2][c][0] * cm - G[2][c][1] * sm;
        S[0][c] = wave_sum(w * r0);
        S[1][c] = wave_sum(w * r1);
        S[2][c] = wave_sum(-w * m * i0);
        S[3][c] = wave_sum(w * r2);
        S[4][c] = wave_sum(-w * m * i1);
        S[5][c] = wave_sum(-w * (double)m * m * r0);
    }
}

__device__ __forceinline__ double dot3d(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Setup of every item: closest point, interpolation points and their grid
// (0 standard, 1 upsampled), Legendre values at x*.
__global__ __launch_bounds__(64) void k_near_setup(NearArgs a)
{
    const int it = blockIdx.x;
    if (it >= a.n) return;
    const int lane = threadIdx.x;
    const NearItem I = a.items[it];
    const int j = I.j, p = a.dp[j];
    const double *xc = a.xc + a.dcoff[j];
    const long cs = a.Ctot;
    const double x0[3] = {a.tx[I.t], a.tx[a.T + I.t], a.tx[2 * a.T + I.t]};
    // nearest node of drop j (ties: lowest index)
    const int nn = 2 * p * (p + 1), o = a.dtoff[j];
    double best = 1e300;
    int bi = 0;
    for (int k = lane; k < nn; k += 64) {
        const double hx = x0[0] - a.tx[o + k], hy = x0[1] - a.tx[a.T + o + k], hz = x0[2] - a.tx[2 * a.T + o + k];
        const double r2 = hx * hx + hy * hy + hz * hz;
        if (r2 < best) {
            best = r2;
            bi = k;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob < best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
        }
    }
    double th = acos(a.gl_t[a.gl_off[j] + bi / (2 * p)]);
    double ph = kPiN * (bi % (2 * p)) / p;
    // Newton with the Levenberg-Marquardt shift
    double S[6][3], Sn[6][3];
    surf_eval(p, xc, cs, th, ph, S, nullptr);
    double r[3] = {S[0][0] - x0[0], S[0][1] - x0[1], S[0][2] - x0[2]};
    double F = 0.5 * dot3d(r, r), mu = 0.0;
    bool converged = false;
    for (int iter = 0; iter < 100 && !converged; ++iter) {
        const double g0 = dot3d(r, S[1]), g1 = dot3d(r, S[2]);
        const double H00 = dot3d(S[1], S[1]) + dot3d(r, S[3]);
        const double H01 = dot3d(S[1], S[2]) + dot3d(r, S[4]);
        const double H11 = dot3d(S[2], S[2]) + dot3d(r, S[5]);
        const double scale = dot3d(S[1], S[1]) + dot3d(S[2], S[2]);
        bool accepted = false;
        for (int tries = 0; tries < 40 && !accepted; ++tries) {
            const double aa = H00 + mu * scale, bb = H01, dd = H11 + mu * scale;
            const double det = aa * dd - bb * bb;
            if (!(det > 0.0) || !(aa > 0.0)) {
                mu = mu == 0.0 ? 1e-6 : 10.0 * mu;
                continue;
            }
            const double s0 = -(dd * g0 - bb * g1) / det, s1 = -(aa * g1 - bb * g0) / det;
            surf_eval(p, xc, cs, th + s0, ph + s1, Sn, nullptr);
            double rn[3] = {Sn[0][0] - x0[0], Sn[0][1] - x0[1], Sn[0][2] - x0[2]};
            const double Fn = 0.5 * dot3d(rn, rn);
            const bool local = mu == 0.0 && fabs(s0) + fabs(s1) < 1e-8;
            if (Fn <= F || local) {
                th += s0;
                ph += s1;
#pragma unroll
                for (int q = 0; q < 6; ++q)
#pragma unroll
                    for (int c = 0; c < 3; ++c) S[q][c] = Sn[q][c];
                r[0] = rn[0];
                r[1] = rn[1];
                r[2] = rn[2];
                F = Fn;
                mu = mu * 0.1 < 1e-12 ? 0.0 : mu * 0.1;
                accepted = true;
                converged = fabs(s0) + fabs(s1) < 1e-15;
            } else {
                mu = mu == 0.0 ? 1e-6 : 10.0 * mu;
            }
        }
        if (!accepted) break;
    }
    // Legendre values at x* for the on-surface evaluations
    surf_eval(p, xc, cs, th, ph, S, a.Pst + (long)it * a.ldp);
    const double dv[3] = {x0[0] - S[0][0], x0[1] - S[0][1], x0[2] - S[0][2]};
    const double s0 = sqrt(dot3d(dv, dv));
    const double d[3] = {dv[0] / s0, dv[1] / s0, dv[2] / s0};
    if (lane == 0) {
        a.par[4 * it] = th;
        a.par[4 * it + 1] = ph;
        a.par[4 * it + 2] = s0;
        a.par[4 * it + 3] = (double)bi;
    }
    const double hj = a.hj[j];
    for (int l = 1; l <= a.L; ++l) {
        const double sl = hj * sqrt((double)l);
        const double xl[3] = {S[0][0] + sl * d[0], S[0][1] + sl * d[1], S[0][2] + sl * d[2]};
        double dm = 1e300;
        for (int k = lane; k < nn; k += 64) {
            const double hx = xl[0] - a.tx[o + k], hy = xl[1] - a.tx[a.T + o + k], hz = xl[2] - a.tx[2 * a.T + o + k];
            dm = fmin(dm, hx * hx + hy * hy + hz * hz);
        }
        dm = sqrt(wave_min(dm));
        const long v = (long)it * a.L + (l - 1);
        if (lane == 0) {
            a.vx[v] = xl[0];
            a.vx[a.V + v] = xl[1];
            a.vx[2 * a.V + v] = xl[2];
            a.vreg[v] = dm > a.A * hj ? 0 : 1;
        }
    }
}

// Interpolation: value at x* from the self-interaction expansion (minus
// 4 pi u(x*) for the double layer), the L regular-rule values, Lagrange in the
// distance; the weighted result of item `it` goes to out[c * n + it] (the
// items of a target are added to it afterwards in item order).
__global__ __launch_bounds__(64) void k_near_interp(NearArgs a, int kind, const double *__restrict__ selfc,
                                                   const double *__restrict__ dens, const double *__restrict__ vacc,
                                                   const double *__restrict__ wts, double *__restrict__ out)
{
    const int it = blockIdx.x;
    if (it >= a.n) return;
    const double wi = wts[it];
    if (wi == 0.0) {  // the item's slot still takes its (zero) contribution
        if (threadIdx.x < 3) out[threadIdx.x * a.n + it] = 0.0;
        return;
    }
    const int m = threadIdx.x;
    const NearItem I = a.items[it];
    const int j = I.j, p = a.dp[j];
    const double ph = a.par[4 * it + 1], s0 = a.par[4 * it + 2];
    const double *P = a.Pst + (long)it * a.ldp;
    const long co = a.dcoff[j], cs = a.Ctot;
    double sm, cm;
    sincos(m * ph, &sm, &cm);
    const double w = m ? 2.0 : 1.0;
    double v0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double gr = 0.0, gi = 0.0, ur = 0.0, ui = 0.0;
        for (int n = m; n <= p; ++n) {
            const int e = n * (n + 1) / 2 + m;
            const double Pe = P[e];
            gr = fma(selfc[c * cs + co + 2 * e], Pe, gr);
            gi = fma(selfc[c * cs + co + 2 * e + 1], Pe, gi);
            if (kind == 1) {
                ur = fma(dens[c * cs + co + 2 * e], Pe, ur);
                ui = fma(dens[c * cs + co + 2 * e + 1], Pe, ui);
            }
        }
        double val = w * (gr * cm - gi * sm);
        if (kind == 1) val -= 4.0 * kPiN * w * (ur * cm - ui * sm);
        v0[c] = wave_sum(m <= p ? val : 0.0);
    }
    if (m != 0) return;
    const int L = a.L;
    const double hj = a.hj[j];
    // nodes s_0 = 0, s_l = h sqrt(l); weights of the Lagrange basis at s0
    double sn[kNearMaxL + 1];
    sn[0] = 0.0;
    for (int l = 1; l <= L; ++l) sn[l] = hj * sqrt((double)l);
    double res[3] = {0.0, 0.0, 0.0};
    for (int l = 0; l <= L; ++l) {
        double b = 1.0;
        for (int q = 0; q <= L; ++q)
            if (q != l) b *= (s0 - sn[q]) / (sn[l] - sn[q]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = l == 0 ? v0[c] : vacc[c * a.V + (long)it * L + (l - 1)];
            res[c] = fma(b, v, res[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c * a.n + it] = wi * res[c];
}

void launch_near_setup(hipStream_t st, const NearArgs &a)
{
    if (a.n <= 0) return;
    hipLaunchKernelGGL(k_near_setup, dim3(a.n), dim3(64), 0, st, a);
}

void launch_near_interp(hipStream_t st, const NearArgs &a, int kind, const double *selfc, const double *dens,
                        const double *vacc, const double *wts, double *out)
{
    if (a.n <= 0) return;
    hipLaunchKernelGGL(k_near_interp, dim3(a.n), dim3(64), 0, st, a, kind, selfc, dens, vacc, wts, out);
}

}  // namespace bim
