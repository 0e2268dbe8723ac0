// Fast summation of the far drop pairs of the regular pair sums (Sec. 2.1,
// 2.3; the cost the paper names for large systems, Sec. 6): a drop-level
// fast multipole method on the Laplace kernel.
//
// Both Stokes kernels of the pair sums are rebuilt from four harmonic
// potentials H_0..H_3 about a common origin o (the target drop's centre):
//   u_i(x) = H_i(x) - (x - o)_j d_i H_j(x) + d_i H_3(x).
// Single layer (weights q = wW f at the source nodes):
//   H_j = sum q_j / r (j < 3), H_3 = sum ((y - o).q) / r.
// Double layer (-6 h (h.u)(h.wN) / r^5, density u, weighted normal wN):
//   dipole potentials with moments m_j = -(u_j wN + wN_j u) (j < 3) and
//   m_3 = -((y - o).u wN + (y - o).wN u), a dipole m at y giving m.h / r^3.
// Harmonics (scaled solid harmonics, m >= 0 stored, index tri(n,m) =
// n(n+1)/2 + m, values at m < 0 by X_n^{-m} = (-1)^m conj(X_n^m)):
//   regular   U_0^0 = 1, U_m^m = -(x+iy)/(2m) U_{m-1}^{m-1},
//             U_n^m = ((2n-1) z U_{n-1}^m - r^2 U_{n-2}^m) / ((n+m)(n-m));
//   irregular T_0^0 = 1/r, T_m^m = -(2m-1)(x+iy)/r^2 T_{m-1}^{m-1},
//             T_n^m = ((2n-1) z T_{n-1}^m - ((n-1)^2 - m^2) T_{n-2}^m) / r^2;
//   1/|x - y| = sum_{n,m} conj(U_n^m(y)) T_n^m(x)  (|y| < |x|);
//   d_z U_n^m = U_{n-1}^m, (d_x + i d_y) U_n^m = U_{n-1}^{m+1},
//   (d_x - i d_y) U_n^m = -U_{n-1}^{m-1}.
// Multipole about the source centre c_s (P2M):
//   M_n^m = sum q conj(U_n^m(y - c_s)) + conj(m.grad U_n^m(y - c_s)).
// Local expansion about the target centre c_t (M2L), D = c_t - c_s:
//   L_k^l = (-1)^k sum_{n,m} M_n^m T_{n+k}^{m+l}(D),  H(c_t + xi) = sum L_k^l conj(U_k^l(xi));
// H_3 is moved to the origin c_t by H_3 += sum_j (c_s - c_t)_j H_j before
// the translation. The truncation error of a pair with source radius a_s,
// target radius a_t is bounded by a constant times rho^(P+1),
// rho = (a_s + a_t) / |D| (the host applies the method to a pair only when
// rho^(P+1) <= eps).
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace bim {

__device__ inline int ftri(int n, int m) { return n * (n + 1) / 2 + m; }

// ---- regular harmonics of the source nodes, stored once per geometry -------
// Y[(s) * ntri + tri(n,m)] = U_n^m(y_s - c) for the ns nodes of a source grid,
// as double2, or float2 in the mixed-precision form (the multipoles are still
// accumulated in FP64).
template <class YT>
__global__ void k_fmm_ytab(const FmmSrcJob *__restrict__ jobs, int P, const double *__restrict__ cen,
                           YT *__restrict__ Y)
{
    const FmmSrcJob j = jobs[blockIdx.y];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= j.ns) return;
    const int ntri = (P + 1) * (P + 2) / 2;
    const double *c = cen + 4 * j.slot;
    const long g = j.off + s;
    const double x = j.x[g] - c[0], y = j.x[j.stride + g] - c[1], z = j.x[2 * j.stride + g] - c[2];
    const double r2 = x * x + y * y + z * z;
    YT *out = Y + (j.yoff + (long)s * ntri);
    double dre = 1.0, dim = 0.0;  // U_m^m
    for (int m = 0; m <= P; ++m) {
        if (m) {
            const double f = -0.5 / m, ar = f * x, ai = f * y;
            const double t = dre * ar - dim * ai;
            dim = dre * ai + dim * ar;
            dre = t;
        }
        double p1r = dre, p1i = dim, p2r = 0.0, p2i = 0.0;
        out[ftri(m, m)] = YT{(decltype(YT::x))dre, (decltype(YT::x))dim};
        for (int n = m + 1; n <= P; ++n) {
            const double inv = 1.0 / ((double)(n + m) * (n - m)), a = (2 * n - 1) * z;
            const double ur = (a * p1r - r2 * p2r) * inv, ui = (a * p1i - r2 * p2i) * inv;
            out[ftri(n, m)] = YT{(decltype(YT::x))ur, (decltype(YT::x))ui};
            p2r = p1r;
            p2i = p1i;
            p1r = ur;
            p1i = ui;
        }
    }
}

// ---- per-source weights of one application --------------------------------
// SL: W[s][c] = q_c (c < 3), q_3 = (y - c_s).q, q = wW f.
// DL: W[s][3c..3c+2] = (a, Re b, Im b) of moment m_c: a = m_z, b = (m_x + i m_y)/2.
__global__ void k_fmm_srcw(const FmmSrcJob *__restrict__ jobs, int kind, const double *__restrict__ cen,
                           double *__restrict__ W)
{
    const FmmSrcJob j = jobs[blockIdx.y];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= j.ns) return;
    const double *c = cen + 4 * j.slot;
    const long g = j.off + s, st = j.stride;
    const double yp[3] = {j.x[g] - c[0], j.x[st + g] - c[1], j.x[2 * st + g] - c[2]};
    const double d[3] = {j.d[g], j.d[st + g], j.d[2 * st + g]};
    double *w = W + (j.woff + (long)s * (kind == 0 ? 4 : 12));
    if (kind == 0) {
        const double ww = j.wW[g];
        const double q[3] = {ww * d[0], ww * d[1], ww * d[2]};
        w[0] = q[0];
        w[1] = q[1];
        w[2] = q[2];
        w[3] = yp[0] * q[0] + yp[1] * q[1] + yp[2] * q[2];
    } else {
        const double n[3] = {j.wN[g], j.wN[st + g], j.wN[2 * st + g]};
        const double yu = yp[0] * d[0] + yp[1] * d[1] + yp[2] * d[2];
        const double yn = yp[0] * n[0] + yp[1] * n[1] + yp[2] * n[2];
        for (int ch = 0; ch < 4; ++ch) {
            double m[3];
            for (int k = 0; k < 3; ++k)
                m[k] = ch < 3 ? -(d[ch] * n[k] + n[ch] * d[k]) : -(yu * n[k] + yn * d[k]);
            w[3 * ch] = m[2];
            w[3 * ch + 1] = 0.5 * m[0];
            w[3 * ch + 2] = 0.5 * m[1];
        }
    }
}

// ---- P2M: partial multipoles of source chunks ------------------------------
// Block (chunk, job): thread = coefficient tri(n,m); sums over the chunk's
// kFmmChunk sources; part[(job chunk base + chunk)][c][tri].
template <int KIND, class YT>
__global__ __launch_bounds__(kFmmThreads) void k_fmm_p2m(const FmmSrcJob *__restrict__ jobs, int P,
                                                         const YT *__restrict__ Y, const double *__restrict__ W,
                                                         double2 *__restrict__ part)
{
    const FmmSrcJob j = jobs[blockIdx.y];
    const int chunk = blockIdx.x;
    const int s0 = chunk * kFmmChunk;
    if (s0 >= j.ns) return;
    const int s1 = min(j.ns, s0 + kFmmChunk);
    const int ntri = (P + 1) * (P + 2) / 2;
    const int e = threadIdx.x;
    if (e >= ntri) return;
    int n = 0;
    while ((n + 1) * (n + 2) / 2 <= e) ++n;
    const int m = e - n * (n + 1) / 2;
    double ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
    const YT *Yc = Y + j.yoff;
    constexpr int NW = KIND == 0 ? 4 : 12;
    const double *Wc = W + j.woff;
    if (KIND == 0) {
        for (int s = s0; s < s1; ++s) {
            const YT uy = Yc[(long)s * ntri + e];
            const double2 u = make_double2(uy.x, uy.y);
            const double *w = Wc + (long)s * NW;
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {  // q conj(U)
                ar[ch] = fma(w[ch], u.x, ar[ch]);
                ai[ch] = fma(-w[ch], u.y, ai[ch]);
            }
        }
    } else if (n > 0) {
        // conj(m.grad U_n^m) = a conj(U_{n-1}^m) + b conj(U_{n-1}^{m+1}) - conj(b) conj(U_{n-1}^{m-1})
        const bool hp = m + 1 <= n - 1, hm = m <= n - 1;
        const int e0 = ftri(n - 1, min(m, n - 1)), ep = ftri(n - 1, min(m + 1, n - 1)),
                  em = ftri(n - 1, m > 0 ? m - 1 : 1 <= n - 1 ? 1 : 0);
        for (int s = s0; s < s1; ++s) {
            const YT *yr = Yc + (long)s * ntri;
            const YT y0 = yr[e0], yp = yr[ep], ym = yr[em];
            const double2 u0 = hm ? make_double2(y0.x, y0.y) : make_double2(0.0, 0.0);
            const double2 up = hp ? make_double2(yp.x, yp.y) : make_double2(0.0, 0.0);
            double2 um;  // conj(U_{n-1}^{m-1}); at m = 0 conj(U^{-1}) = -U^{1}
            if (m > 0) {
                um = make_double2(ym.x, -ym.y);
            } else if (n - 1 >= 1) {
                um = make_double2(-ym.x, -ym.y);
            } else {
                um = make_double2(0.0, 0.0);
            }
            const double *w = Wc + (long)s * NW;
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                const double a = w[3 * ch], br = w[3 * ch + 1], bi = w[3 * ch + 2];
                // a conj(u0)
                double re = a * u0.x, im = -a * u0.y;
                // b conj(up)
                re = fma(br, up.x, fma(bi, up.y, re));
                im = fma(bi, up.x, fma(-br, up.y, im));
                // - conj(b) um
                re = fma(-br, um.x, fma(-bi, um.y, re));
                im = fma(bi, um.x, fma(-br, um.y, im));
                ar[ch] += re;
                ai[ch] += im;
            }
        }
    }
    double2 *o = part + (long)(j.pbase + chunk) * 4 * ntri;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) o[ch * ntri + e] = make_double2(ar[ch], ai[ch]);
}

// Multipoles of every order: Mf[slot][n^2 + n + m][c], |m| <= n, from the
// sum of the job's partial chunks (in order) and M_n^{-m} = (-1)^m conj(M_n^m).
__global__ void k_fmm_msum(const FmmSrcJob *__restrict__ jobs, int P, const double2 *__restrict__ part,
                           double2 *__restrict__ Mf)
{
    const FmmSrcJob j = jobs[blockIdx.y];
    const int ntri = (P + 1) * (P + 2) / 2, nsq = (P + 1) * (P + 1);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * nsq) return;
    const int ch = i & 3, f = i >> 2;
    int n = 0;
    while ((n + 1) * (n + 1) <= f) ++n;
    const int m = f - n * n - n, ma = m < 0 ? -m : m;
    const int e = ch * ntri + ftri(n, ma);
    const int nch = (j.ns + kFmmChunk - 1) / kFmmChunk;
    double re = 0.0, im = 0.0;
    for (int k = 0; k < nch; ++k) {
        const double2 v = part[(long)(j.pbase + k) * 4 * ntri + e];
        re += v.x;
        im += v.y;
    }
    if (m < 0) {
        im = -im;
        if (ma & 1) {
            re = -re;
            im = -im;
        }
    }
    Mf[(long)j.slot * 4 * nsq + i] = make_double2(re, im);
}

// ---- M2L per far drop pair ----------------------------------------------------
// Block per pair; thread = output coefficient tri(k,l), k <= the pair's
// order Q (coefficients above it are zero). The irregular harmonics of D up
// to degree 2Q, every order, are built in LDS (lane = order); the multipole
// coefficients are wavefront-uniform (scalar loads). Output:
// Lp[pair][c][tri] = w (-1)^k sum_{n<=Q,|m|<=n} M'_c T_{n+k}^{m+l}(D), with
// channel 3 moved to the target origin.
__global__ __launch_bounds__(kFmmThreads) void k_fmm_m2l(const FmmPair *__restrict__ pairs, int P,
                                                         const double *__restrict__ cen_s,
                                                         const double *__restrict__ cen_t,
                                                         const double2 *__restrict__ Mf, double2 *__restrict__ Lp)
{
    extern __shared__ double2 th[];  // T_N^mu(D) at N^2 + N + mu, N <= 2Q
    const FmmPair pr = pairs[blockIdx.x];
    const int Q = pr.order;
    const double *cs = cen_s + 4 * pr.src, *ct = cen_t + 4 * pr.tgt;
    const double Dx = ct[0] - cs[0], Dy = ct[1] - cs[1], Dz = ct[2] - cs[2];
    const double r2 = Dx * Dx + Dy * Dy + Dz * Dz, ir2 = 1.0 / r2;
    const int Q2 = 2 * Q;
    for (int mm = threadIdx.x; mm <= Q2; mm += blockDim.x) {
        double dre = sqrt(ir2), dim = 0.0;  // T_0^0 = 1/r
        for (int k = 1; k <= mm; ++k) {
            const double f = -(2 * k - 1) * ir2, ar = f * Dx, ai = f * Dy;
            const double t = dre * ar - dim * ai;
            dim = dre * ai + dim * ar;
            dre = t;
        }
        const double sg = (mm & 1) ? -1.0 : 1.0;  // T_N^{-mm} = (-1)^mm conj(T_N^mm)
        double p1r = dre, p1i = dim, p2r = 0.0, p2i = 0.0;
        for (int n = mm; n <= Q2; ++n) {
            double tr, ti;
            if (n == mm) {
                tr = dre;
                ti = dim;
            } else {
                const double a = (2 * n - 1) * Dz, b = (double)(n - 1) * (n - 1) - (double)mm * mm;
                tr = (a * p1r - b * p2r) * ir2;
                ti = (a * p1i - b * p2i) * ir2;
                p2r = p1r;
                p2i = p1i;
                p1r = tr;
                p1i = ti;
            }
            th[n * n + n + mm] = make_double2(tr, ti);
            if (mm) th[n * n + n - mm] = make_double2(sg * tr, -sg * ti);
        }
    }
    __syncthreads();
    const int ntri = (P + 1) * (P + 2) / 2, nsq = (P + 1) * (P + 1);
    const int e = threadIdx.x;
    if (e >= ntri) return;
    int k = 0;
    while ((k + 1) * (k + 2) / 2 <= e) ++k;
    const int l = e - k * (k + 1) / 2;
    double2 *o = Lp + (long)blockIdx.x * 4 * ntri;
    if (k > Q) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) o[ch * ntri + e] = make_double2(0.0, 0.0);
        return;
    }
    const double2 *Ms = Mf + (long)pr.src * 4 * nsq;
    double ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
    for (int n = 0; n <= Q; ++n) {
        const int N = n + k;
        const double2 *trow = th + (N * N + N + l);  // T_N^{m+l} at trow[m]
        const double2 *mrow = Ms + 4 * (n * n + n);  // M_n^m, 4 channels, at mrow[4 m]
        for (int m = -n; m <= n; ++m) {
            const double2 t = trow[m];
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                const double2 mv = mrow[4 * m + ch];
                ar[ch] = fma(mv.x, t.x, fma(-mv.y, t.y, ar[ch]));
                ai[ch] = fma(mv.x, t.y, fma(mv.y, t.x, ai[ch]));
            }
        }
    }
    const double sg = (k & 1) ? -pr.w : pr.w;
    const double sx = cs[0] - ct[0], sy = cs[1] - ct[1], sz = cs[2] - ct[2];
    ar[3] += sx * ar[0] + sy * ar[1] + sz * ar[2];
    ai[3] += sx * ai[0] + sy * ai[1] + sz * ai[2];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) o[ch * ntri + e] = make_double2(sg * ar[ch], sg * ai[ch]);
}

// L[t][c][tri] = sum of the partial local expansions of the target's pairs
// (pairs sorted by target, [poff[t], poff[t+1])), in order.
__global__ void k_fmm_lsum(int nt, int P, const int *__restrict__ poff, const double2 *__restrict__ Lp,
                           double2 *__restrict__ L)
{
    const int t = blockIdx.y;
    const int ntri = (P + 1) * (P + 2) / 2;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt || i >= 4 * ntri) return;
    double re = 0.0, im = 0.0;
    for (int p = poff[t]; p < poff[t + 1]; ++p) {
        const double2 v = Lp[(long)p * 4 * ntri + i];
        re += v.x;
        im += v.y;
    }
    L[(long)t * 4 * ntri + i] = make_double2(re, im);
}

// ---- L2P: velocity at the target nodes ---------------------------------------
// Coefficients of the 15 real fields evaluated at the targets, per target
// slot and tri(k,l): f = 0..2 H_c, 3..6 d_x H_c, 7..10 d_y H_c, 11..14 d_z H_c,
// with U = U_k^l(xi), xi = x - c_t, each field = sum_{k, l >= 0} Re(C_f conj(U)):
//   H_c:     L_c[k][l]
//   d_z H_c: L_c[k+1][l]
//   d_x H_c: (L_c[k+1][l-1] - L_c[k+1][l+1]) / 2
//   d_y H_c: i (L_c[k+1][l-1] + L_c[k+1][l+1]) / 2
// (L[k+1][-1] = -conj(L[k+1][1])), times 2 for l > 0 (the l < 0 terms of a
// real field are the conjugates of the l > 0 terms).
constexpr int kFmmFields = 15, kL2pWaves = 8;

__global__ void k_fmm_lderiv(int nt, int P, const double2 *__restrict__ L, double2 *__restrict__ C)
{
    const int t = blockIdx.y;
    const int ntri = (P + 1) * (P + 2) / 2;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt || e >= ntri) return;
    int k = 0;
    while ((k + 1) * (k + 2) / 2 <= e) ++k;
    const int l = e - k * (k + 1) / 2;
    const double wl = l ? 2.0 : 1.0;
    const double2 *Lt = L + (long)t * 4 * ntri;
    double2 *o = C + ((long)t * ntri + e) * kFmmFields;
    for (int ch = 0; ch < 3; ++ch) {
        const double2 v = Lt[ch * ntri + e];
        o[ch] = make_double2(wl * v.x, wl * v.y);
    }
    for (int ch = 0; ch < 4; ++ch) {
        double2 gx = make_double2(0.0, 0.0), gy = gx, gz = gx;
        if (k < P) {
            const double2 Z = Lt[ch * ntri + ftri(k + 1, l)], B = Lt[ch * ntri + ftri(k + 1, l + 1)];
            double2 A = Lt[ch * ntri + ftri(k + 1, l > 0 ? l - 1 : 1)];
            if (l == 0) A.x = -A.x;
            gx = make_double2(0.5 * wl * (A.x - B.x), 0.5 * wl * (A.y - B.y));
            gy = make_double2(-0.5 * wl * (A.y + B.y), 0.5 * wl * (A.x + B.x));
            gz = make_double2(wl * Z.x, wl * Z.y);
        }
        o[3 + ch] = gx;
        o[7 + ch] = gy;
        o[11 + ch] = gz;
    }
}

// Block: 64 targets of one target slot (lane = target), its kL2pWaves
// wavefronts taking runs of whole columns l with about equal term counts
// (column l goes to wavefront floor(off(l) kL2pWaves / ntri), off(l) = terms of
// the columns before it); the coefficients are wavefront-uniform (scalar
// loads); the fields are summed over the wavefronts in LDS in a fixed order;
// out[i][t] += H_i - xi_j d_i H_j + d_i H_3.
__global__ __launch_bounds__(64 * kL2pWaves) void k_fmm_l2p(const FmmTgtJob *__restrict__ jobs, int P,
                                                            const double *__restrict__ cen_t,
                                                            const double2 *__restrict__ C,
                                                            const double *__restrict__ tx, long tstride,
                                                            double *__restrict__ out, long ostride)
{
    constexpr int H = kL2pWaves / 2;
    __shared__ double red[H][kFmmFields][64];
    const FmmTgtJob jb = jobs[blockIdx.y];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i0 = blockIdx.x * 64;
    if (i0 >= jb.n) return;
    const int i = i0 + lane, ii = i < jb.n ? i : jb.n - 1;
    const long t = jb.off + ii;
    const double *c = cen_t + 4 * jb.slot;
    const double x = tx[t] - c[0], y = tx[tstride + t] - c[1], z = tx[2 * tstride + t] - c[2];
    const double r2 = x * x + y * y + z * z;
    const int ntri = (P + 1) * (P + 2) / 2;
    const double2 *Ct = C + (long)jb.slot * ntri * kFmmFields;
    double f[kFmmFields];
#pragma unroll
    for (int q = 0; q < kFmmFields; ++q) f[q] = 0.0;
    double dre = 1.0, dim = 0.0;  // U_l^l
    int off = 0;
    for (int l = 0; l <= P; off += P + 1 - l, ++l) {
        if (l) {
            const double g = -0.5 / l, ar = g * x, ai = g * y;
            const double tt = dre * ar - dim * ai;
            dim = dre * ai + dim * ar;
            dre = tt;
        }
        if ((off * kL2pWaves) / ntri != w) continue;
        double p1r = dre, p1i = dim, p2r = 0.0, p2i = 0.0;
        for (int k = l; k <= P; ++k) {
            double ur = p1r, ui = p1i;
            if (k > l) {
                const double inv = 1.0 / ((double)(k + l) * (k - l)), a = (2 * k - 1) * z;
                ur = (a * p1r - r2 * p2r) * inv;
                ui = (a * p1i - r2 * p2i) * inv;
                p2r = p1r;
                p2i = p1i;
                p1r = ur;
                p1i = ui;
            }
            const double2 *cr = Ct + (long)ftri(k, l) * kFmmFields;
#pragma unroll
            for (int q = 0; q < kFmmFields; ++q) f[q] = fma(cr[q].x, ur, fma(cr[q].y, ui, f[q]));
        }
    }
    if (w >= H)
#pragma unroll
        for (int q = 0; q < kFmmFields; ++q) red[w - H][q][lane] = f[q];
    __syncthreads();
    if (w < H)
#pragma unroll
        for (int q = 0; q < kFmmFields; ++q) red[w][q][lane] += f[q];
    __syncthreads();
    if (w != 0 || i >= jb.n) return;
#pragma unroll
    for (int q = 0; q < kFmmFields; ++q) {
        double v = 0.0;
        for (int u = 0; u < H; ++u) v += red[u][q][lane];
        f[q] = v;
    }
    const double xi[3] = {x, y, z};
    for (int d = 0; d < 3; ++d) {
        const double *g = f + 3 + 4 * d;  // d_d H_0..3
        const double v = f[d] - (xi[0] * g[0] + xi[1] * g[1] + xi[2] * g[2]) + g[3];
        out[d * ostride + t] += v;
    }
}

// ---- launchers ------------------------------------------------------------------
void launch_fmm_ytab(hipStream_t st, const FmmSrcJob *jobs, int njobs, int maxns, int P, const double *cen, void *Y,
                     bool f32)
{
    if (!njobs || !maxns) return;
    if (f32)
        hipLaunchKernelGGL(k_fmm_ytab<float2>, dim3((maxns + 127) / 128, njobs), dim3(128), 0, st, jobs, P, cen,
                           (float2 *)Y);
    else
        hipLaunchKernelGGL(k_fmm_ytab<double2>, dim3((maxns + 127) / 128, njobs), dim3(128), 0, st, jobs, P, cen,
                           (double2 *)Y);
}

void launch_fmm_p2m(hipStream_t st, const FmmSrcJob *jobs, int njobs, int maxns, int kind, int P, const double *cen,
                    const void *Y, bool f32, double *W, double2 *part, double2 *M)
{
    if (!njobs || !maxns) return;
    hipLaunchKernelGGL(k_fmm_srcw, dim3((maxns + 255) / 256, njobs), dim3(256), 0, st, jobs, kind, cen, W);
    const int nch = (maxns + kFmmChunk - 1) / kFmmChunk;
    const dim3 g(nch, njobs), b(kFmmThreads);
    if (f32) {
        const float2 *Yf = (const float2 *)Y;
        if (kind == 0)
            hipLaunchKernelGGL((k_fmm_p2m<0, float2>), g, b, 0, st, jobs, P, Yf, W, part);
        else
            hipLaunchKernelGGL((k_fmm_p2m<1, float2>), g, b, 0, st, jobs, P, Yf, W, part);
    } else {
        const double2 *Yd = (const double2 *)Y;
        if (kind == 0)
            hipLaunchKernelGGL((k_fmm_p2m<0, double2>), g, b, 0, st, jobs, P, Yd, W, part);
        else
            hipLaunchKernelGGL((k_fmm_p2m<1, double2>), g, b, 0, st, jobs, P, Yd, W, part);
    }
    const int nsq = (P + 1) * (P + 1);
    hipLaunchKernelGGL(k_fmm_msum, dim3((4 * nsq + 255) / 256, njobs), dim3(256), 0, st, jobs, P, part, M);
}

size_t fmm_m2l_lds(int P) { return (size_t)(2 * P + 1) * (2 * P + 1) * sizeof(double2); }

void launch_fmm_m2l(hipStream_t st, int npairs, const FmmPair *pairs, int P, const double *cen_s, const double *cen_t,
                    const double2 *M, double2 *Lp, int nt, const int *poff, double2 *L)
{
    if (!npairs) return;
    hipLaunchKernelGGL(k_fmm_m2l, dim3(npairs), dim3(kFmmThreads), fmm_m2l_lds(P), st, pairs, P, cen_s, cen_t, M, Lp);
    const int ntri = (P + 1) * (P + 2) / 2;
    hipLaunchKernelGGL(k_fmm_lsum, dim3((4 * ntri + 255) / 256, nt), dim3(256), 0, st, nt, P, poff, Lp, L);
}

void launch_fmm_l2p(hipStream_t st, int njobs, const FmmTgtJob *jobs, int maxn, int P, const double *cen_t,
                    const double2 *L, double2 *C, const double *tx, long tstride, double *out, long ostride)
{
    if (!njobs || !maxn) return;
    const int ntri = (P + 1) * (P + 2) / 2;
    hipLaunchKernelGGL(k_fmm_lderiv, dim3((ntri + 255) / 256, njobs), dim3(256), 0, st, njobs, P, L, C);
    hipLaunchKernelGGL(k_fmm_l2p, dim3((maxn + 63) / 64, njobs), dim3(64 * kL2pWaves), 0, st, jobs, P, cen_t, C, tx,
                       tstride, out, ostride);
}

}  // namespace bim
