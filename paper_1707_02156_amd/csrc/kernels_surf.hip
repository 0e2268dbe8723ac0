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

#include <algorithm>

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
constexpr int kRepMaxDeg = 64;  // degree bound of the reparametrization grid (U_rep p)
constexpr double kPiS = 3.14159265358979323846;

// Values and angle derivatives of NF (1 or 3) real expansions of degree q
// at nodes (theta_i, phi_i), theta in [0, pi], from the orthonormal
// associated-Legendre recursion in n at fixed order m (Sec. 1.1),
//   P_m^m = c_m sin^m(theta),  P_{m+1}^m = sqrt(2m+3) cos(theta) P_m^m,
//   P_n^m = a_nm cos(theta) P_{n-1}^m - b_nm P_{n-2}^m,
// and the theta derivative from the same order,
//   dP_n^m/dtheta = (n cos(theta) P_n^m - d_nm P_{n-1}^m) / sin(theta),
//   d_nm = sqrt((2n+1)(n^2-m^2)/(2n-1))  (d_mm = 0).
// The expansions are first packed (k_rep_pack) into order-major records
// rec[(off(m) + n - m) RS], off(m) = m(q+1) - m(m-1)/2, RS = 4 + 2 NF:
//   {a, b, d, n, re_0, im_0, ..., re_{NF-1}, im_{NF-1}},
// with (a, b) = (0, -1) at n = m and (sqrt(2m+3), 0) at n = m + 1, so that
// one recursion P = a t P_{n-1} - b P_{n-2} started from (P_{m-1}, P_{m-2})
// = (0, c_m sin^m) covers every n. The expansions are fixed while the nodes
// move, so the packing is done once per set of expansions.
// Batched over drops of one degree (blockIdx.y = drop b of the batch): the
// expansions of drop b start at coef + b NF cstride, its records at
// rec + b R RS. The evaluation, gradient and move kernels take the same
// batch index, with the nodes of drop b at th/ph + b ang_bs and its
// outputs at the per-drop strides given below.
template <int NF>
__global__ void k_rep_pack(int q, const double *__restrict__ coef, long cstride, const double *__restrict__ hdr,
                           double *__restrict__ rec)
{
    constexpr int RS = 4 + 2 * NF;
    const long nc = (long)(q + 1) * (q + 2) / 2;
    const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nc) return;
    coef += (long)blockIdx.y * NF * cstride;
    rec += (long)blockIdx.y * nc * RS;
    int m = 0;
    long off = 0;
    while (off + (q + 1 - m) <= j) off += q + 1 - m++;
    const int n = m + (int)(j - off);
    const long e = (long)n * (n + 1) / 2 + m;
    double *r = rec + j * RS;
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = hdr[4 * j + k];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        r[4 + 2 * f] = coef[f * cstride + 2 * e];
        r[5 + 2 * f] = coef[f * cstride + 2 * e + 1];
    }
}

// Evaluation: lanes take nodes (64 per block); the orders are split into
// kRepWaves runs of whole orders with about equal record counts (order m
// goes to run floor(off(m) kRepWaves / R), R = (q+1)(q+2)/2), one per
// wavefront of the block. The records of a wavefront's orders are
// wavefront-uniform, read through scalar loads. The order sums of the runs
// are added in LDS in a fixed order, within the block (a split of the orders
// over several blocks needs device-scope fences for the cross-block sum,
// which cost more than the added parallelism gains).
// out[(3 f + d) N + i] (+ b 3 NF N for drop b): d = 0 value, 1 d/dtheta,
// 2 d/dphi.
constexpr int kRepWaves = 16;
static_assert(kRepWaves % 2 == 0, "two-phase block sum");

template <int NF>
__global__ __launch_bounds__(64 * kRepWaves) void k_rep_eval(int q, const double *__restrict__ rec,
                                                             const double *__restrict__ cmt,
                                                             const double *__restrict__ th,
                                                             const double *__restrict__ ph, long ang_bs, long N,
                                                             double *__restrict__ out)
{
    constexpr int RS = 4 + 2 * NF, NO = 3 * NF;
    __shared__ double red[kRepWaves / 2][NO][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long grp = blockIdx.x;
    const long R = (long)(q + 1) * (q + 2) / 2;
    rec += (long)blockIdx.y * R * RS;
    th += (long)blockIdx.y * ang_bs;
    ph += (long)blockIdx.y * ang_bs;
    out += (long)blockIdx.y * NO * N;
    const long i = grp * 64 + lane, ic = i < N ? i : N - 1;  // lanes past N evaluate node N - 1, store nothing
    const double t = cos(th[ic]), s = sin(th[ic]), is = 1.0 / s, phi = ph[ic];
    double acc[NF][3] = {};
    bool first = true;
    double spow = 1.0, cm = 1.0, sm = 0.0, c1 = 1.0, s1 = 0.0;  // sin^m, e^{i m phi}, e^{i phi}
    long off = 0;
    for (int m = 0; m <= q; off += q + 1 - m, ++m) {
        if ((off * kRepWaves) / R != w) continue;
        if (first) {  // the run's first order: sin^m by binary powers, e^{i m phi} directly
            double b = s;
            for (int k = m; k; k >>= 1, b *= b)
                if (k & 1) spow *= b;
            sincos(m * phi, &sm, &cm);
            sincos(phi, &s1, &c1);
            first = false;
        } else {  // the next order of the run
            spow *= s;
            const double c = cm * c1 - sm * s1;
            sm = sm * c1 + cm * s1;
            cm = c;
        }
        const double *r = rec + off * RS;
        double Pm1 = 0.0, Pm2 = cmt[m] * spow;
        double G[NF][2][2] = {};  // [field][value, d_theta * sin][re, im]
#pragma unroll 2
        for (int n = m; n <= q; ++n, r += RS) {
            const double P = fma(r[0] * t, Pm1, -r[1] * Pm2);
            const double Dp = fma(r[3] * t, P, -r[2] * Pm1);
            Pm2 = Pm1;
            Pm1 = P;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                G[f][0][0] = fma(r[4 + 2 * f], P, G[f][0][0]);
                G[f][0][1] = fma(r[5 + 2 * f], P, G[f][0][1]);
                G[f][1][0] = fma(r[4 + 2 * f], Dp, G[f][1][0]);
                G[f][1][1] = fma(r[5 + 2 * f], Dp, G[f][1][1]);
            }
        }
        const double wt = m ? 2.0 : 1.0;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            // Re(g e^{i m phi}) and Re(i m g e^{i m phi})
            acc[f][0] += wt * (G[f][0][0] * cm - G[f][0][1] * sm);
            acc[f][1] += wt * is * (G[f][1][0] * cm - G[f][1][1] * sm);
            acc[f][2] += -wt * m * (G[f][0][0] * sm + G[f][0][1] * cm);
        }
    }
    // block sum: the upper half of the wavefronts stores, the lower half adds
    constexpr int H = kRepWaves / 2;
    if (w >= H) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int d = 0; d < 3; ++d) red[w - H][3 * f + d][lane] = acc[f][d];
    }
    __syncthreads();
    if (w < H) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int d = 0; d < 3; ++d) red[w][3 * f + d][lane] += acc[f][d];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < NO * 64; idx += blockDim.x) {
        const int k = idx >> 6, l = idx & 63;
        double v = 0.0;
        for (int u = 0; u < H; ++u) v += red[u][k][l];
        const long node = grp * 64 + l;
        if (node < N) out[k * N + node] = v;
    }
}

// g = (I - n n) grad E at every node, n = X_t x X_p / |X_t x X_p|; gmax holds
// the largest |g| as the bits of a non-negative double (ordered like unsigned
// integers). E: k_rep_eval output for the 3 position components; gE [3][N].
// Drop b of a batch: E + 9 N b, gE and g + 3 N b, gmax + b.
__global__ void k_rep_grad(long N, const double *__restrict__ E, const double *__restrict__ gE,
                           double *__restrict__ g, unsigned long long *gmax)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    E += 9 * N * blockIdx.y;
    gE += 3 * N * blockIdx.y;
    g += 3 * N * blockIdx.y;
    gmax += blockIdx.y;
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
// With check set the step is skipped once the previous residual max |g|
// (gmax) is below eps (the iteration has stopped); moves counts the steps taken.
// Drop b of a batch: E + 9 N b, g + 3 N b, th/ph + ang_bs b, gmax and moves + b.
__global__ void k_rep_move(long N, const double *__restrict__ E, const double *__restrict__ g, double dtau,
                           double *__restrict__ th, double *__restrict__ ph, long ang_bs,
                           const unsigned long long *gmax, double eps, int check, int *moves)
{
    gmax += blockIdx.y;
    if (check && __longlong_as_double((long long)gmax[0]) < eps) return;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    E += 9 * N * blockIdx.y;
    g += 3 * N * blockIdx.y;
    th += ang_bs * blockIdx.y;
    ph += ang_bs * blockIdx.y;
    moves += blockIdx.y;
    if (i == 0) moves[0] += 1;
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

void launch_rep_pack(hipStream_t st, int q, int nf, int nb, const double *coef, long cstride, const double *hdr,
                     double *rec)
{
    const long nc = (long)(q + 1) * (q + 2) / 2;
    const dim3 grid((unsigned)((nc + 255) / 256), (unsigned)nb);
    if (nf == 3)
        hipLaunchKernelGGL(k_rep_pack<3>, grid, dim3(256), 0, st, q, coef, cstride, hdr, rec);
    else
        hipLaunchKernelGGL(k_rep_pack<1>, grid, dim3(256), 0, st, q, coef, cstride, hdr, rec);
}

void launch_rep_eval(hipStream_t st, int q, int nf, int nb, const double *rec, const double *cm, const double *th,
                     const double *ph, long ang_bs, long N, double *out)
{
    const dim3 grid((unsigned)((N + 63) / 64), (unsigned)nb);
    if (nf == 3)
        hipLaunchKernelGGL(k_rep_eval<3>, grid, dim3(64 * kRepWaves), 0, st, q, rec, cm, th, ph, ang_bs, N, out);
    else
        hipLaunchKernelGGL(k_rep_eval<1>, grid, dim3(64 * kRepWaves), 0, st, q, rec, cm, th, ph, ang_bs, N, out);
}

void launch_rep_grad(hipStream_t st, int nb, long N, const double *E, const double *gE, double *g,
                     unsigned long long *gmax)
{
    hipLaunchKernelGGL(k_rep_grad, dim3((unsigned)((N + 255) / 256), (unsigned)nb), dim3(256), 0, st, N, E, gE, g,
                       gmax);
}

void launch_rep_move(hipStream_t st, int nb, long N, const double *E, const double *g, double dtau, double *th,
                     double *ph, long ang_bs, const unsigned long long *gmax, double eps, int check, int *moves)
{
    hipLaunchKernelGGL(k_rep_move, dim3((unsigned)((N + 255) / 256), (unsigned)nb), dim3(256), 0, st, N, E, g, dtau,
                       th, ph, ang_bs, gmax, eps, check, moves);
}

// Adaptive cutoff and filter in one block: mag_n = sum_{|m| <= n} |x_n^m|
// (3-vector norm, m > 0 twice), n_cut = the smallest l in 2..q whose tail
// sum_{n >= l} mag_n is below P_cut sum_{n >= 1} mag_n (q + 1 when none);
// hp = xt with the degrees n < n_cut zeroed; clears gmax for the gradient.
// Each thread holds up to kRepCutPer coefficients (3 components) in
// registers from one coalesced pass; the per-degree sums, their tails and
// the search run from LDS in a fixed order (no atomics on the sums).
// One block per drop of a batch: drop b at xt and hp + 3 cs b, ncut and
// gmax + b.
constexpr int kRepCutThreads = 1024, kRepCutPer = 3;  // tri(kRepMaxDeg + 1) <= 3072
static_assert((kRepMaxDeg + 1) * (kRepMaxDeg + 2) / 2 <= kRepCutThreads * kRepCutPer, "cutoff kernel size");

__global__ __launch_bounds__(kRepCutThreads) void k_rep_cut(int q, const double *__restrict__ xt, long cs,
                                                            double P_cut, double *__restrict__ hp, int *ncut,
                                                            unsigned long long *gmax)
{
    __shared__ double v[kRepCutThreads * kRepCutPer];
    __shared__ double mag[kRepMaxDeg + 1], tail[kRepMaxDeg + 2];
    __shared__ int snc;
    const int tid = threadIdx.x;
    const int nc = (q + 1) * (q + 2) / 2;
    xt += 3 * cs * blockIdx.x;
    hp += 3 * cs * blockIdx.x;
    ncut += blockIdx.x;
    gmax += blockIdx.x;
    double2 x[kRepCutPer][3];
    int deg[kRepCutPer];
#pragma unroll
    for (int k = 0; k < kRepCutPer; ++k) {
        const int e = tid + k * kRepCutThreads;
        deg[k] = -1;
        if (e < nc) {
            int n = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
            while (n * (n + 1) / 2 > e) --n;
            while ((n + 1) * (n + 2) / 2 <= e) ++n;
            deg[k] = n;
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                x[k][c] = *reinterpret_cast<const double2 *>(xt + c * cs + 2L * e);
                s += x[k][c].x * x[k][c].x + x[k][c].y * x[k][c].y;
            }
            v[e] = (e == n * (n + 1) / 2 ? 1.0 : 2.0) * sqrt(s);
        }
    }
    if (tid == 0) snc = q + 1;
    __syncthreads();
    if (tid <= q) {
        double a = 0.0;
        for (int m = 0; m <= tid; ++m) a += v[tid * (tid + 1) / 2 + m];
        mag[tid] = a;
    }
    __syncthreads();
    if (tid >= 1 && tid <= q) {
        double t = 0.0;
        for (int n = tid; n <= q; ++n) t += mag[n];
        tail[tid] = t;
    }
    __syncthreads();
    if (tid >= 2 && tid <= q && tail[tid] < P_cut * tail[1]) atomicMin(&snc, tid);
    __syncthreads();
    const int l = snc;
    if (tid == 0) {
        ncut[0] = l;
        gmax[0] = 0ull;
    }
#pragma unroll
    for (int k = 0; k < kRepCutPer; ++k) {
        if (deg[k] < 0) continue;
        const long e = tid + k * kRepCutThreads;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            *reinterpret_cast<double2 *>(hp + c * cs + 2 * e) = deg[k] >= l ? x[k][c] : double2{0.0, 0.0};
    }
}

void launch_rep_cut(hipStream_t st, int q, int nb, const double *xt, long cs, double P_cut, double *hp, int *ncut,
                    unsigned long long *gmax)
{
    if (q < 1 || q > kRepMaxDeg || (cs & 1)) return;  // the host validates q = U_rep p <= 64, cs = (q+1)(q+2)
    hipLaunchKernelGGL(k_rep_cut, dim3((unsigned)nb), dim3(kRepCutThreads), 0, st, q, xt, cs, P_cut, hp, ncut, gmax);
}

}  // namespace bim
