// Surface operators of the surfactant equation (Sec. 1.1, Sec. 3.2) on the
// de-aliasing grid, one batched launch for all drops.
//
// Per grid point, from synthesized fields (positions and their first and
// second parameter derivatives, the surfactant concentration Gamma and its
// derivatives, the velocity and its first derivatives):
//   metric      E = x_phi.x_phi, F = x_theta.x_phi, G = x_theta.x_theta, W^2 = EG - F^2,
//               inverse metric g^tt = E/W^2, g^tp = -F/W^2, g^pp = G/W^2;
//   div_s u   = g^ij x_i . u_j                      (tangential trace of grad u);
//   grad_s g  = (g^tt g_t + g^tp g_p) x_t + (g^tp g_t + g^pp g_p) x_p;
//   LB g      = g^ij (g_ij - x_ij . grad_s g)       (surface Hessian traced;
//               x_ij . grad_s g is the Christoffel term);
//   fE        = -Gamma div_s u                      (material rate at nodes moving with u).
// Integrals by the regular rule (Sec. 2.1), w_j = (pi/q) w_j^G / sin theta_j:
//   mass   += w_j W Gamma,   volume += w_j (x_t x x_p) . x / 3.
#include "internal.hpp"

#include <hip/hip_runtime.h>

namespace bim {

__global__ __launch_bounds__(256) void k_surf_terms(SurfJobs jobs)
{
    const SurfJob &J = jobs.j[blockIdx.y];
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double mloc = 0.0, vloc = 0.0;
    if (i < J.np) {
        const long np = J.np;
        auto X = [&](int f, int c) { return J.syn[((long)f * 3 + c) * np + i]; };  // x fields f = 0..5
        auto Gm = [&](int f) { return J.syn[(18L + f) * np + i]; };               // Gamma fields
        double xt[3], xp[3];
        for (int c = 0; c < 3; ++c) {
            xt[c] = X(1, c);
            xp[c] = X(2, c);
        }
        const double E = xp[0] * xp[0] + xp[1] * xp[1] + xp[2] * xp[2];
        const double F = xt[0] * xp[0] + xt[1] * xp[1] + xt[2] * xp[2];
        const double G = xt[0] * xt[0] + xt[1] * xt[1] + xt[2] * xt[2];
        const double W2 = E * G - F * F;
        const double gtt = E / W2, gtp = -F / W2, gpp = G / W2;
        const double W = sqrt(W2);
        const double w = J.wreg[i / (2 * J.q)];
        if (J.vol) {
            const double N0 = xt[1] * xp[2] - xt[2] * xp[1], N1 = xt[2] * xp[0] - xt[0] * xp[2],
                         N2 = xt[0] * xp[1] - xt[1] * xp[0];
            vloc = w * (N0 * X(0, 0) + N1 * X(0, 1) + N2 * X(0, 2)) / 3.0;
        }
        if (J.gam) {
            const double g0 = Gm(0);
            if (J.mass) mloc = w * W * g0;
            if (J.fE) {
                // u fields at 24 + 3 f + c, f = 0 (u), 1 (u_t), 2 (u_p)
                auto U = [&](int f, int c) { return J.syn[(24L + 3 * f + c) * np + i]; };
                double tu = 0.0, tp = 0.0, pu = 0.0, pp = 0.0;  // x_t.u_t, x_t.u_p, x_p.u_t, x_p.u_p
                for (int c = 0; c < 3; ++c) {
                    tu = fma(xt[c], U(1, c), tu);
                    tp = fma(xt[c], U(2, c), tp);
                    pu = fma(xp[c], U(1, c), pu);
                    pp = fma(xp[c], U(2, c), pp);
                }
                const double divu = gtt * tu + gtp * (tp + pu) + gpp * pp;
                J.fE[i] = -g0 * divu;
            }
            if (J.lg) {
                const double gt = Gm(1), gp = Gm(2);
                const double at = gtt * gt + gtp * gp, ap = gtp * gt + gpp * gp;
                double grad[3];
                for (int c = 0; c < 3; ++c) grad[c] = at * xt[c] + ap * xp[c];
                auto h = [&](int f) {  // second derivative f (3: tt, 4: tp, 5: pp) less the Christoffel term
                    return Gm(f) - (X(f, 0) * grad[0] + X(f, 1) * grad[1] + X(f, 2) * grad[2]);
                };
                J.lg[i] = gtt * h(3) + 2.0 * gtp * h(4) + gpp * h(5);
            }
        }
    }
    if (J.mass || J.vol) {
        // wavefront sums, one atomic per wavefront
        for (int o = 32; o > 0; o >>= 1) {
            mloc += __shfl_down(mloc, o, 64);
            vloc += __shfl_down(vloc, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            if (J.mass && mloc != 0.0) atomicAdd(J.mass, mloc);
            if (J.vol && vloc != 0.0) atomicAdd(J.vol, vloc);
        }
    }
}

void launch_surf_terms(hipStream_t st, const SurfJob *jobs, int n)
{
    for (int o = 0; o < n; o += kMaxSurfJobs) {
        SurfJobs b{};
        b.n = n - o < kMaxSurfJobs ? n - o : kMaxSurfJobs;
        long maxnp = 0;
        for (int i = 0; i < b.n; ++i) {
            b.j[i] = jobs[o + i];
            maxnp = b.j[i].np > maxnp ? b.j[i].np : maxnp;
        }
        hipLaunchKernelGGL(k_surf_terms, dim3((unsigned)((maxnp + 255) / 256), b.n), dim3(256), 0, st, b);
    }
}

// y = d * x (elementwise; y may alias x)
__global__ void k_mul(long n, const double *__restrict__ d, const double *x, double *y)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = d[i] * x[i];
}

void launch_mul(hipStream_t st, long n, const double *d, const double *x, double *y)
{
    hipLaunchKernelGGL(k_mul, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, d, x, y);
}

// out = a x + b y (out may alias x or y)
__global__ void k_axpby(long n, double a, const double *x, double b, const double *y, double *out)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a * x[i] + b * y[i];
}

void launch_axpby(hipStream_t st, long n, double a, const double *x, double b, const double *y, double *out)
{
    hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, x, b, y, out);
}

// ----------------------------------------------------------------------------
// Angle reparametrization (Sec. 4, Algorithm 2)
// ----------------------------------------------------------------------------
constexpr int kRepMaxF = 3;
constexpr double kPiS = 3.14159265358979323846;

__device__ inline double wave_add(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Values and angle derivatives of nf <= 3 real expansions of degree q
// (component f at coef + f * cstride) at nodes (theta_i, phi_i), theta in
// [0, pi]. One wavefront per node; lanes take the orders m = lane, lane + 64,
// ...; each runs the orthonormal associated-Legendre recursion in n (Sec. 1.1)
// and the theta derivative from the same order,
//   dP_n^m/dtheta = (n cos(theta) P_n^m - sqrt((2n+1)(n^2-m^2)/(2n-1)) P_{n-1}^m) / sin(theta);
// the order sums are wavefront sums. out[(3 f + d) N + i]: d = 0 value,
// 1 d/dtheta, 2 d/dphi.
__global__ __launch_bounds__(256) void k_rep_eval(int q, int nf, const double *__restrict__ coef, long cstride,
                                                  const double *__restrict__ th, const double *__restrict__ ph,
                                                  long N, double *__restrict__ out)
{
    const long i = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;  // node (one per wavefront)
    const int lane = threadIdx.x & 63;
    if (i >= N) return;                                                 // the whole wavefront
    const double t = cos(th[i]), s = sin(th[i]), phi = ph[i];
    double acc[kRepMaxF][3] = {};
    for (int m0 = 0; m0 <= q; m0 += 64) {
        const int m = m0 + lane;
        if (m > q) continue;
        double pmm = 1.0 / sqrt(4.0 * kPiS);
        for (int k = 1; k <= m; ++k) pmm *= -sqrt((2.0 * k + 1.0) / (2.0 * k)) * s;
        double G[kRepMaxF][2][2] = {};  // [field][value, d_theta][re, im]
        double Pm1 = 0.0, Pm2 = 0.0;
        for (int n = m; n <= q; ++n) {
            double P;
            if (n == m) {
                P = pmm;
            } else if (n == m + 1) {
                P = sqrt(2.0 * m + 3.0) * t * pmm;
            } else {
                const double an = sqrt((2.0 * n + 1.0) * (2.0 * n - 1.0) / ((double)(n - m) * (n + m)));
                const double bn = sqrt((2.0 * n + 1.0) * (double)(n + m - 1) * (n - m - 1) /
                                       ((2.0 * n - 3.0) * (double)(n - m) * (n + m)));
                P = an * t * Pm1 - bn * Pm2;
            }
            const double D =
                (n * t * P - (n > m ? sqrt((2.0 * n + 1.0) * (double)(n - m) * (n + m) / (2.0 * n - 1.0)) * Pm1
                                    : 0.0)) / s;
            Pm2 = Pm1;
            Pm1 = P;
            const long e = (long)n * (n + 1) / 2 + m;
            for (int f = 0; f < nf; ++f) {
                const double cr = coef[f * cstride + 2 * e], ci = coef[f * cstride + 2 * e + 1];
                G[f][0][0] = fma(cr, P, G[f][0][0]);
                G[f][0][1] = fma(ci, P, G[f][0][1]);
                G[f][1][0] = fma(cr, D, G[f][1][0]);
                G[f][1][1] = fma(ci, D, G[f][1][1]);
            }
        }
        double sm, cm;
        sincos(m * phi, &sm, &cm);
        const double w = m ? 2.0 : 1.0;
        for (int f = 0; f < nf; ++f) {
            // Re(g e^{i m phi}) and Re(i m g e^{i m phi})
            acc[f][0] += w * (G[f][0][0] * cm - G[f][0][1] * sm);
            acc[f][1] += w * (G[f][1][0] * cm - G[f][1][1] * sm);
            acc[f][2] += -w * m * (G[f][0][0] * sm + G[f][0][1] * cm);
        }
    }
    for (int f = 0; f < nf; ++f)
        for (int d = 0; d < 3; ++d) {
            const double v = wave_add(acc[f][d]);
            if (lane == 0) out[(3L * f + d) * N + i] = v;
        }
}

// g = (I - n n) grad E at every node, n = X_t x X_p / |X_t x X_p|; gmax holds
// the largest |g| as the bits of a non-negative double (ordered like unsigned
// integers). E: k_rep_eval output for the 3 position components; gE [3][N].
__global__ void k_rep_grad(long N, const double *__restrict__ E, const double *__restrict__ gE,
                           double *__restrict__ g, unsigned long long *gmax)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double mag = 0.0;
    if (i < N) {
        double xt[3], xp[3], v[3];
        for (int c = 0; c < 3; ++c) {
            xt[c] = E[(3L * c + 1) * N + i];
            xp[c] = E[(3L * c + 2) * N + i];
            v[c] = gE[c * N + i];
        }
        double n[3] = {xt[1] * xp[2] - xt[2] * xp[1], xt[2] * xp[0] - xt[0] * xp[2], xt[0] * xp[1] - xt[1] * xp[0]};
        const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int c = 0; c < 3; ++c) n[c] /= nn;
        const double vn = n[0] * v[0] + n[1] * v[1] + n[2] * v[2];
        for (int c = 0; c < 3; ++c) {
            const double gc = v[c] - vn * n[c];
            g[c * N + i] = gc;
            mag = fma(gc, gc, mag);
        }
        mag = sqrt(mag);
    }
    for (int o = 32; o > 0; o >>= 1) mag = fmax(mag, __shfl_xor(mag, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(gmax, (unsigned long long)__double_as_longlong(mag));
}

// One forward-Euler step of the angles: w = -g, A alpha = (w.X_t, w.X_p) with
// A the metric of the initial expansion at the node; theta, phi += dtau alpha,
// taken back into theta in [0, pi] across the pole (phi + pi) and phi mod 2 pi.
__global__ void k_rep_move(long N, const double *__restrict__ E, const double *__restrict__ g, double dtau,
                           double *__restrict__ th, double *__restrict__ ph)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double a00 = 0.0, a01 = 0.0, a11 = 0.0, b0 = 0.0, b1 = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double xt = E[(3L * c + 1) * N + i], xp = E[(3L * c + 2) * N + i], w = -g[c * N + i];
        a00 = fma(xt, xt, a00);
        a01 = fma(xt, xp, a01);
        a11 = fma(xp, xp, a11);
        b0 = fma(w, xt, b0);
        b1 = fma(w, xp, b1);
    }
    const double det = a00 * a11 - a01 * a01;
    double t = th[i] + dtau * (a11 * b0 - a01 * b1) / det;
    double p = ph[i] + dtau * (a00 * b1 - a01 * b0) / det;
    if (t < 0.0) {
        t = -t;
        p += kPiS;
    } else if (t > kPiS) {
        t = 2.0 * kPiS - t;
        p += kPiS;
    }
    p = fmod(p, 2.0 * kPiS);
    if (p < 0.0) p += 2.0 * kPiS;
    th[i] = t;
    ph[i] = p;
}

void launch_rep_eval(hipStream_t st, int q, int nf, const double *coef, long cstride, const double *th,
                     const double *ph, long N, double *out)
{
    hipLaunchKernelGGL(k_rep_eval, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, st, q, nf, coef, cstride, th, ph, N,
                       out);
}

void launch_rep_grad(hipStream_t st, long N, const double *E, const double *gE, double *g, unsigned long long *gmax)
{
    hipLaunchKernelGGL(k_rep_grad, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, N, E, gE, g, gmax);
}

void launch_rep_move(hipStream_t st, long N, const double *E, const double *g, double dtau, double *th, double *ph)
{
    hipLaunchKernelGGL(k_rep_move, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, N, E, g, dtau, th, ph);
}

}  // namespace bim
