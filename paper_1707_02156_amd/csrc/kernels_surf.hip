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

}  // namespace bim
