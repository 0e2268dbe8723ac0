// Fused singular self-integral kernel (gfx950, FP64).
//
// One workgroup per grid target of a drop. For the target (theta_j, phi_k):
//   R. rotation of the expansion so the target is at the north pole
//      (Appendix B, gamma = 0), for x and (single layer) the density f, into LDS;
//   then, for blocks of JB latitudes of the rotated degree-qs grid:
//   L. Legendre sums G = sum_n C^mu_n Ptilde_n^mu(t_j') (and d/dtheta for x);
//   F. Fourier sums at the 2qs longitudes, using the symmetries
//      phi -> -phi and phi -> phi + pi (four points per cosine/sine pair);
//   K. the kernels of the Theorem 1 pole rule (Sec. 2.2) with weight
//      omega_j' = (pi/qs) w_j' [sum_{n<=qs} P_n(t_j')] 2 sin(theta_j'/2)/sin(theta_j'):
//      SL  omega W (f/r + xh (xh.f)/r^3), accumulated per thread;
//      DL  the six distinct entries of -6 omega xh xh (xh.N)/r^5 (N = x_theta x x_phi);
//   and for the double layer the adjoint transforms
//   FA. Fourier analysis of the six kernel fields on the rotated grid,
//   LA. Legendre analysis accumulated in registers over the latitude blocks,
//   after the last block
//   AR. adjoint rotation: the rows of the linear map u -> D_self[u](target)
//      in the coefficient layout of u (6 symmetric 3x3 blocks).
// So the double layer of the drop on itself becomes a stored matrix
// M[t][pair][2 ncoef(p)], applied to any density by k_dl_apply.
#include "internal.hpp"

#include <hip/hip_runtime.h>

#include <mutex>

#include <algorithm>

namespace bim {

static constexpr double kInvSqrt4Pi_s = 0.28209479177387814347;

struct SingArgs {
    int p, qs, nt;
    // rotation tables of the degree-p target grid, per latitude: A+ and A-
    // ([nu][mu] in blocks per n), and their transposes ([mu][nu])
    const double *Ap, *Am, *ApT, *AmT;
    const double *csp;       // cos/sin of the degree-p grid: [2][2p]
    const double *xc;        // x coefficients of the drop, component stride xstride
    long xstride;
    const double *dc;        // density coefficients (single layer), stride dstride
    long dstride;
    const double *L;         // singular grid tables [3][qs+1][ncoef(p)] (Ptilde, d/dtheta, -)
    const double *wsing;     // omega_j' [qs+1]
    double *out_sl;          // [3][ostride] single-layer sums (added, times scale)
    long ostride;
    double scale;
    double *M;               // double-layer rows [nt][6][2 ncoef(p)]
};

__device__ __forceinline__ void decode_tri(int e, int &n, int &m)
{
    int nn = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while ((nn + 1) * (nn + 2) / 2 <= e) ++nn;
    while (nn * (nn + 1) / 2 > e) --nn;
    n = nn;
    m = e - nn * (nn + 1) / 2;
}

// LDS footprint in doubles of one workgroup.
__host__ __device__ inline long sing_lds_doubles(int p, int qs, int JB, bool SL, bool DL)
{
    const long nc = ncoef(p), P1 = p + 1;
    const long coefs = (SL ? 12 : 6) * nc;
    const long creg = DL ? (coefs > 12 * nc ? coefs : 12 * nc) : coefs;
    const long ntypes = SL ? 9 : 6;
    long gsz = (long)JB * ntypes * P1 * 2;
    if (DL && (long)JB * 6 * P1 * 2 > gsz) gsz = (long)JB * 6 * P1 * 2;
    const long vsz = (long)JB * 2 * qs * 12;
    const long misc = 2 * P1 + 8 + 3 * 16;
    return creg + gsz + vsz + misc;
}

// threads per workgroup: 1024 for the single layer alone (16 wavefronts hide
// the latency of the table reads), 512 when the double-layer rows are built
// (their register accumulators need up to 256 VGPRs per lane)
template <bool SL, bool DL> struct SingThreads { static constexpr int value = DL ? 512 : 1024; };

template <bool SL, bool DL, int JB, int NB>
__global__ __launch_bounds__(DL ? 512 : 1024) void k_sing_fused(SingArgs a)
{
    constexpr int NTH = SingThreads<SL, DL>::value;
    extern __shared__ double lds[];
    const int p = a.p, qs = a.qs;
    const int nc = ncoef(p), P1 = p + 1, nk = 2 * qs;
    const int t = blockIdx.x;
    const int j = t / (2 * p), k = t % (2 * p);
    const int tid = threadIdx.x;

    // ---- LDS carve-up (doubles)
    const long coefs = (SL ? 12 : 6) * (long)nc;
    const long creg = DL ? (coefs > 12L * nc ? coefs : 12L * nc) : coefs;
    double *Cx = lds;                       // [3][nc][2]
    double *Cf = lds + 6L * nc;             // [3][nc][2] (SL)
    constexpr int NTYPES = SL ? 9 : 6;
    long gsz = (long)JB * NTYPES * P1 * 2;
    if (DL && (long)JB * 6 * P1 * 2 > gsz) gsz = (long)JB * 6 * P1 * 2;
    double *G = lds + creg;                 // [JB][type][P1][2]; aliased by Fa [JB][6][P1][2]
    double *V = G + gsz;                    // [JB][2qs][12]
    double *ph = V + (long)JB * nk * 12;    // cos/sin(nu phi_k) [P1][2]
    double *x0s = ph + 2 * P1;              // [3] (+pad)
    double *red = x0s + 8;                  // [3][16]

    // ---- phases of the target longitude
    for (int nu = tid; nu <= p; nu += NTH) {
        const int e = (int)(((long)nu * k) % (2 * p));
        ph[2 * nu] = a.csp[e];
        ph[2 * nu + 1] = a.csp[2 * p + e];
    }
    __syncthreads();

    // ---- R: rotation into LDS
    {
        const size_t lat = rot_lat_size(p) * j;
        const int nf = SL ? 6 : 3;
        for (int it = tid; it < nf * nc; it += NTH) {
            const int f = it / nc, e = it % nc;
            int n, mu;
            decode_tri(e, n, mu);
            const double *c = (f < 3) ? a.xc + f * a.xstride : a.dc + (f - 3) * a.dstride;
            const double *ap = a.Ap + lat + rot_off(n) + mu;
            const double *am = a.Am + lat + rot_off(n) + mu;
            double re = 0.0, im = 0.0;
            const int b0 = n * (n + 1) / 2;
            for (int nu = 0; nu <= n; ++nu) {
                const double cr = c[2 * (b0 + nu)], ci = c[2 * (b0 + nu) + 1];
                const double cc = ph[2 * nu], ss = ph[2 * nu + 1];
                re = fma(ap[nu * (n + 1)], cr * cc - ci * ss, re);
                im = fma(am[nu * (n + 1)], cr * ss + ci * cc, im);
            }
            double *dst = (f < 3) ? Cx + 2L * (f * nc + e) : Cf + 2L * ((f - 3) * nc + e);
            dst[0] = re;
            dst[1] = im;
        }
    }
    __syncthreads();
    if (tid < 3) {
        double s = 0.0;
        for (int n = 0; n <= p; ++n) s += Cx[2 * (tid * nc + n * (n + 1) / 2)] * sqrt(2.0 * n + 1.0) * kInvSqrt4Pi_s;
        x0s[tid] = s;
    }
    __syncthreads();
    const double X0 = x0s[0], Y0 = x0s[1], Z0 = x0s[2];

    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    double Bre[DL ? NB : 1], Bim[DL ? NB : 1];
#pragma unroll
    for (int r = 0; r < (DL ? NB : 1); ++r) { Bre[r] = 0.0; Bim[r] = 0.0; }

    const bool even = (qs & 1) == 0;
    const int nkk = even ? qs / 2 + 1 : qs;   // Fourier items per latitude and component
    const double dphi = 3.14159265358979323846 / qs;

    for (int jb0 = 0; jb0 <= qs; jb0 += JB) {
        const int nb = min(JB, qs + 1 - jb0);
        // ---- L: Legendre sums for the block
        for (int it = tid; it < nb * P1 * 3; it += NTH) {
            const int c = it % 3;
            const int r = it / 3;
            const int mu = r % P1, b = r / P1;
            const double *Lp = a.L + (long)(jb0 + b) * nc;
            const double *Ld = a.L + ((long)(qs + 1) + jb0 + b) * nc;
            double xr = 0, xi = 0, dr = 0, di = 0, fr = 0, fi = 0;
            for (int n = mu; n <= p; ++n) {
                const int e = n * (n + 1) / 2 + mu;
                const double l0 = Lp[e], l1 = Ld[e];
                const double cr = Cx[2 * (c * nc + e)], ci = Cx[2 * (c * nc + e) + 1];
                xr = fma(cr, l0, xr);
                xi = fma(ci, l0, xi);
                dr = fma(cr, l1, dr);
                di = fma(ci, l1, di);
                if (SL) {
                    const double gr = Cf[2 * (c * nc + e)], gi = Cf[2 * (c * nc + e) + 1];
                    fr = fma(gr, l0, fr);
                    fi = fma(gi, l0, fi);
                }
            }
            double *g = G + 2L * ((b * NTYPES) * P1 + mu);
            g[2L * (c * P1)] = xr;
            g[2L * (c * P1) + 1] = xi;
            g[2L * ((3 + c) * P1)] = dr;
            g[2L * ((3 + c) * P1) + 1] = di;
            if (SL) {
                g[2L * ((6 + c) * P1)] = fr;
                g[2L * ((6 + c) * P1) + 1] = fi;
            }
        }
        __syncthreads();
        // ---- F: Fourier sums -> point values V[b][k'][field]
        // fields: 0-2 x, 3-5 x_theta, 6-8 x_phi, 9-11 f
        for (int it = tid; it < nb * nkk * 3; it += NTH) {
            const int c = it % 3;
            const int r = it / 3;
            const int kk = r % nkk, b = r / nkk;
            const double *gx = G + 2L * ((b * NTYPES + c) * P1);
            const double *gd = G + 2L * ((b * NTYPES + 3 + c) * P1);
            const double *gf = G + 2L * ((b * NTYPES + 6 + c) * P1);
            double sn, cs;
            sincos(dphi * kk, &sn, &cs);
            double cm = 1.0, sm = 0.0;  // cos, sin of mu phi
            // [0] x, [1] x_theta, [2] f: C even, C odd, S even, S odd ; x_phi: A even/odd, B even/odd
            double CE[3] = {0, 0, 0}, CO[3] = {0, 0, 0}, SE[3] = {0, 0, 0}, SO[3] = {0, 0, 0};
            double AE = 0, AO = 0, BE = 0, BO = 0;
            for (int mu = 0; mu <= p; ++mu) {
                const double w = mu ? 2.0 : 1.0;
                const double xr = w * gx[2 * mu], xi = w * gx[2 * mu + 1];
                const double dr = w * gd[2 * mu], di = w * gd[2 * mu + 1];
                double fr = 0.0, fi = 0.0;
                if (SL) { fr = w * gf[2 * mu]; fi = w * gf[2 * mu + 1]; }
                if (mu & 1) {
                    CO[0] = fma(xr, cm, CO[0]); SO[0] = fma(xi, sm, SO[0]);
                    CO[1] = fma(dr, cm, CO[1]); SO[1] = fma(di, sm, SO[1]);
                    if (SL) { CO[2] = fma(fr, cm, CO[2]); SO[2] = fma(fi, sm, SO[2]); }
                    AO = fma(-mu * xi, cm, AO);
                    BO = fma(-mu * xr, sm, BO);
                } else {
                    CE[0] = fma(xr, cm, CE[0]); SE[0] = fma(xi, sm, SE[0]);
                    CE[1] = fma(dr, cm, CE[1]); SE[1] = fma(di, sm, SE[1]);
                    if (SL) { CE[2] = fma(fr, cm, CE[2]); SE[2] = fma(fi, sm, SE[2]); }
                    AE = fma(-mu * xi, cm, AE);
                    BE = fma(-mu * xr, sm, BE);
                }
                const double c2 = cm * cs - sm * sn;
                sm = fma(sm, cs, cm * sn);
                cm = c2;
            }
            double *Vb = V + (long)b * nk * 12;
            // point values of field set at phi, -phi, phi + pi, pi - phi
            auto put = [&](int kp, double s1, double s2) {
                // s1 = +1 for phi / phi+pi (cosine terms minus sine terms), s2 = +1 for no pi shift
                double *v = Vb + (long)kp * 12;
                v[c] = (CE[0] - s1 * SE[0]) + s2 * (CO[0] - s1 * SO[0]);
                v[3 + c] = (CE[1] - s1 * SE[1]) + s2 * (CO[1] - s1 * SO[1]);
                v[6 + c] = (AE + s1 * BE) + s2 * (AO + s1 * BO);
                if (SL) v[9 + c] = (CE[2] - s1 * SE[2]) + s2 * (CO[2] - s1 * SO[2]);
            };
            if (even) {
                put(kk, 1.0, 1.0);
                put(kk + qs, 1.0, -1.0);
                if (kk != 0 && kk != qs / 2) {
                    put(nk - kk, -1.0, 1.0);
                    put(qs - kk, -1.0, -1.0);
                }
            } else {
                put(kk, 1.0, 1.0);
                put(kk + qs, 1.0, -1.0);
            }
        }
        __syncthreads();
        // ---- K: kernels at the points of the block
        for (int it = tid; it < nb * nk; it += NTH) {
            const int b = it / nk;
            double *v = V + (long)it * 12;
            const double om = a.wsing[jb0 + b];
            const double xt0 = v[3], xt1 = v[4], xt2 = v[5];
            const double xp0 = v[6], xp1 = v[7], xp2 = v[8];
            const double N0 = xt1 * xp2 - xt2 * xp1;
            const double N1 = xt2 * xp0 - xt0 * xp2;
            const double N2 = xt0 * xp1 - xt1 * xp0;
            const double h0 = X0 - v[0], h1 = Y0 - v[1], h2 = Z0 - v[2];
            const double r2 = h0 * h0 + h1 * h1 + h2 * h2;
            const double ri = rsqrt(r2);
            if (SL) {
                const double f0 = v[9], f1 = v[10], f2 = v[11];
                const double hf = h0 * f0 + h1 * f1 + h2 * f2;
                const double Wr = om * sqrt(N0 * N0 + N1 * N1 + N2 * N2) * ri;
                const double q = hf * ri * ri;
                acc0 = fma(Wr, f0 + h0 * q, acc0);
                acc1 = fma(Wr, f1 + h1 * q, acc1);
                acc2 = fma(Wr, f2 + h2 * q, acc2);
            }
            if (DL) {
                const double hn = h0 * N0 + h1 * N1 + h2 * N2;
                const double r2i = ri * ri;
                const double s = -6.0 * om * hn * r2i * r2i * ri;
                v[0] = s * h0 * h0;
                v[1] = s * h0 * h1;
                v[2] = s * h0 * h2;
                v[3] = s * h1 * h1;
                v[4] = s * h1 * h2;
                v[5] = s * h2 * h2;
            }
        }
        if (DL) {
            __syncthreads();
            // ---- FA: Fourier analysis of the six kernel fields -> Fa[b][pair][mu] = (sum K cos, sum K sin)
            double *Fa = G;
            for (int it = tid; it < nb * 6 * P1; it += NTH) {
                const int mu = it % P1;
                const int r = it / P1;
                const int pr = r % 6, b = r / 6;
                const double *Vb = V + (long)b * nk * 12 + pr;
                double sn, cs;
                sincos(dphi * mu, &sn, &cs);
                double ck = 1.0, sk = 0.0;  // cos, sin of mu phi_kk
                const double sg = (mu & 1) ? -1.0 : 1.0;
                double fc = 0.0, fs = 0.0;
                for (int kk = 0; kk < nkk; ++kk) {
                    double K1, K2, K3, K4;
                    if (even) {
                        K1 = Vb[(long)kk * 12];
                        K3 = Vb[(long)(kk + qs) * 12];
                        if (kk != 0 && kk != qs / 2) {
                            K2 = Vb[(long)(nk - kk) * 12];
                            K4 = Vb[(long)(qs - kk) * 12];
                        } else {
                            K2 = 0.0;
                            K4 = 0.0;
                        }
                    } else {
                        K1 = Vb[(long)kk * 12];
                        K3 = Vb[(long)(kk + qs) * 12];
                        K2 = 0.0;
                        K4 = 0.0;
                    }
                    fc = fma(ck, (K1 + K2) + sg * (K3 + K4), fc);
                    fs = fma(sk, (K1 - K2) + sg * (K3 - K4), fs);
                    const double c2 = ck * cs - sk * sn;
                    sk = fma(sk, cs, ck * sn);
                    ck = c2;
                }
                Fa[2L * ((b * 6 + pr) * P1 + mu)] = fc;
                Fa[2L * ((b * 6 + pr) * P1 + mu) + 1] = fs;
            }
            __syncthreads();
            // ---- LA: Legendre analysis into registers
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                const int idx = tid + NTH * r;
                if (idx < 6 * nc) {
                    const int pr = idx / nc, e = idx % nc;
                    int n, mu;
                    decode_tri(e, n, mu);
                    (void)n;
                    double sr = Bre[r], si = Bim[r];
                    for (int b = 0; b < nb; ++b) {
                        const double l = a.L[(long)(jb0 + b) * nc + e];
                        const double *f = Fa + 2L * ((b * 6 + pr) * P1 + mu);
                        sr = fma(l, f[0], sr);
                        si = fma(l, f[1], si);
                    }
                    Bre[r] = sr;
                    Bim[r] = si;
                }
            }
        }
        __syncthreads();
    }

    if (SL) {
        for (int o = 32; o > 0; o >>= 1) {
            acc0 += __shfl_down(acc0, o, 64);
            acc1 += __shfl_down(acc1, o, 64);
            acc2 += __shfl_down(acc2, o, 64);
        }
        const int wv = tid >> 6;
        if ((tid & 63) == 0) {
            red[wv] = acc0;
            red[16 + wv] = acc1;
            red[32 + wv] = acc2;
        }
        __syncthreads();
        if (tid < 3) {
            double s = 0.0;
            for (int w = 0; w < NTH / 64; ++w) s += red[16 * tid + w];
            a.out_sl[tid * a.ostride + t] += a.scale * s;
        }
    }
    if (DL) {
        // a_mu = w_mu sum_j' P F_c, b_mu = -w_mu sum_j' P F_s, stored over the coefficient region
        double *Bl = lds;  // [6][nc][2]
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int idx = tid + NTH * r;
            if (idx < 6 * nc) {
                const int e = idx % nc;
                int n, mu;
                decode_tri(e, n, mu);
                (void)n;
                const double w = mu ? 2.0 : 1.0;
                Bl[2L * idx] = w * Bre[r];
                Bl[2L * idx + 1] = -w * Bim[r];
            }
        }
        __syncthreads();
        // ---- AR: adjoint rotation -> rows of the double-layer map
        const size_t lat = rot_lat_size(p) * j;
        double *Mt = a.M + (long)t * 6 * 2 * nc;
        for (int it = tid; it < 6 * nc; it += NTH) {
            const int pr = it / nc, e = it % nc;
            int n, nu;
            decode_tri(e, n, nu);
            const double *apt = a.ApT + lat + rot_off(n) + nu;
            const double *amt = a.AmT + lat + rot_off(n) + nu;
            const double *bp = Bl + 2L * (pr * nc + n * (n + 1) / 2);
            double al = 0.0, be = 0.0;
            for (int mu = 0; mu <= n; ++mu) {
                al = fma(apt[mu * (n + 1)], bp[2 * mu], al);
                be = fma(amt[mu * (n + 1)], bp[2 * mu + 1], be);
            }
            const double cc = ph[2 * nu], ss = ph[2 * nu + 1];
            Mt[(long)pr * 2 * nc + 2 * e] = al * cc + be * ss;
            Mt[(long)pr * 2 * nc + 2 * e + 1] = -al * ss + be * cc;
        }
    }
}

// out_c[t] += w * sum_{c'} sum_e M[t][pair(c,c')][e] u_{c'}[e], one wavefront per target.
// One target row: (o0, o1, o2) = M_t (u0, u1, u2) over the six symmetric pair
// rows of length nc2 (even; rows and densities 16-byte aligned), read as
// double2 by one wavefront, two iterations of loads in flight per lane.
__device__ inline void dl_row(const double *__restrict__ Mt, const double *__restrict__ u, long ustride, int nc2,
                              int lane, double &o0, double &o1, double &o2)
{
    const int h = nc2 >> 1;
    const double2 *M0 = reinterpret_cast<const double2 *>(Mt), *M1 = M0 + h, *M2 = M1 + h, *M3 = M2 + h,
                  *M4 = M3 + h, *M5 = M4 + h;
    const double2 *U0 = reinterpret_cast<const double2 *>(u), *U1 = reinterpret_cast<const double2 *>(u + ustride),
                  *U2 = reinterpret_cast<const double2 *>(u + 2 * ustride);
    o0 = o1 = o2 = 0.0;
#pragma unroll 2
    for (int e = lane; e < h; e += 64) {
        const double2 a = U0[e], b = U1[e], c = U2[e];
        const double2 m00 = M0[e], m01 = M1[e], m02 = M2[e], m11 = M3[e], m12 = M4[e], m22 = M5[e];
        o0 = fma(m00.x, a.x, fma(m01.x, b.x, fma(m02.x, c.x, o0)));
        o1 = fma(m01.x, a.x, fma(m11.x, b.x, fma(m12.x, c.x, o1)));
        o2 = fma(m02.x, a.x, fma(m12.x, b.x, fma(m22.x, c.x, o2)));
        o0 = fma(m00.y, a.y, fma(m01.y, b.y, fma(m02.y, c.y, o0)));
        o1 = fma(m01.y, a.y, fma(m11.y, b.y, fma(m12.y, c.y, o1)));
        o2 = fma(m02.y, a.y, fma(m12.y, b.y, fma(m22.y, c.y, o2)));
    }
    for (int o = 32; o > 0; o >>= 1) {
        o0 += __shfl_down(o0, o, 64);
        o1 += __shfl_down(o1, o, 64);
        o2 += __shfl_down(o2, o, 64);
    }
}

__global__ __launch_bounds__(256) void k_dl_apply(int nt, int nc2, const double *__restrict__ M,
                                                  const double *__restrict__ u, long ustride, double w,
                                                  double *__restrict__ out, long ostride)
{
    const int wv = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wv >= nt) return;
    double o0, o1, o2;
    dl_row(M + (long)wv * 6 * nc2, u, ustride, nc2, lane, o0, o1, o2);
    if (lane == 0) {
        out[wv] += w * o0;
        out[ostride + wv] += w * o1;
        out[2 * ostride + wv] += w * o2;
    }
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
template <bool SL, bool DL, int JB, int NB> static void launch_one(hipStream_t st, const SingArgs &a, size_t lds)
{
    auto fn = k_sing_fused<SL, DL, JB, NB>;
    static std::once_flag once;  // concurrent callers wait until the limit is set
    std::call_once(once, [&] {
        (void)hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
    });
    hipLaunchKernelGGL(fn, dim3(a.nt), dim3(SingThreads<SL, DL>::value), lds, st, a);
}

// Register-resident adjoint accumulators per thread for the double-layer rows.
static inline long dl_entries(int p, int nth) { return (6L * ncoef(p) + nth - 1) / nth; }

template <bool SL, bool DL, int NB> static bool launch_nb(hipStream_t st, const SingArgs &a, int jbmax)
{
    for (int jb : {8, 4, 2, 1}) {
        if (jb > jbmax) continue;
        const long need = sing_lds_doubles(a.p, a.qs, jb, SL, DL) * 8;
        if (need > 163840) continue;
        if (jb == 8) launch_one<SL, DL, 8, NB>(st, a, need);
        else if (jb == 4) launch_one<SL, DL, 4, NB>(st, a, need);
        else if (jb == 2) launch_one<SL, DL, 2, NB>(st, a, need);
        else launch_one<SL, DL, 1, NB>(st, a, need);
        return true;
    }
    return false;
}

template <bool SL, bool DL> static bool launch_sl_dl(hipStream_t st, const SingArgs &a)
{
    if constexpr (!DL) {
        return launch_nb<SL, DL, 1>(st, a, 8);
    } else {
        const long need = dl_entries(a.p, 512);
        if (need <= 2) return launch_nb<SL, DL, 2>(st, a, 8);
        if (need <= 4) return launch_nb<SL, DL, 4>(st, a, 8);
        if (need <= 7) return launch_nb<SL, DL, 7>(st, a, 8);
        if (need <= 11) return launch_nb<SL, DL, 11>(st, a, 4);
        if constexpr (!SL) {
            if (need <= 15) return launch_nb<SL, DL, 15>(st, a, 4);
            if (need <= 17) return launch_nb<SL, DL, 17>(st, a, 4);
        }
        return false;
    }
}

// Returns false when the degree does not fit the fused kernel (caller falls back).
bool launch_sing_fused(hipStream_t st, bool sl, bool dl, const SingArgs &a)
{
    if (sl && dl) return launch_sl_dl<true, true>(st, a);
    if (sl) return launch_sl_dl<true, false>(st, a);
    if (dl) return launch_sl_dl<false, true>(st, a);
    return true;
}

// Whether the fused kernel handles this degree (single layer, double-layer rows, or both at once).
bool sing_fused_fits(int p, int qs, bool sl, bool dl)
{
    bool lds_ok = false;
    for (int jb : {4, 2, 1})
        if (sing_lds_doubles(p, qs, jb, sl, dl) * 8 <= 163840) lds_ok = true;
    if (!lds_ok) return false;
    if (!dl) return true;
    return dl_entries(p, 512) <= (sl ? 11 : 17);
}

// Stored rows of several drops in one launch: block (target group, job).
__global__ __launch_bounds__(256) void k_dl_apply_multi(DlJobs jobs, long ustride, long ostride)
{
    const DlJob &J = jobs.j[blockIdx.y];
    const int wv = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wv >= J.nt) return;
    double o0, o1, o2;
    dl_row(J.M + (long)wv * 6 * J.nc2, J.u, ustride, J.nc2, lane, o0, o1, o2);
    if (lane == 0) {
        J.out[wv] += J.w * o0;
        J.out[ostride + wv] += J.w * o1;
        J.out[2 * ostride + wv] += J.w * o2;
    }
}

void launch_dl_apply_multi(hipStream_t st, const DlJob *jobs, int n, long ustride, long ostride)
{
    for (int o = 0; o < n; o += kMaxDlJobs) {
        DlJobs b{};
        b.n = std::min(kMaxDlJobs, n - o);
        int maxnt = 0;
        for (int i = 0; i < b.n; ++i) {
            b.j[i] = jobs[o + i];
            maxnt = std::max(maxnt, jobs[o + i].nt);
        }
        hipLaunchKernelGGL(k_dl_apply_multi, dim3((unsigned)(((long)maxnt * 64 + 255) / 256), b.n), dim3(256), 0, st,
                           b, ustride, ostride);
    }
}

void launch_dl_apply(hipStream_t st, int nt, int nc2, const double *M, const double *u, long ustride, double w,
                     double *out, long ostride)
{
    const long threads = (long)nt * 64;
    hipLaunchKernelGGL(k_dl_apply, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, nt, nc2, M, u, ustride,
                       w, out, ostride);
}

}  // namespace bim
