// Singular self-integral as a batched pipeline over all grid targets of a drop
// (gfx950, FP64). Same quadrature as the fused kernel (Sec. 2.2, Theorem 1,
// Appendix B), reorganised so the Legendre stages are dense contractions on
// the matrix cores:
//
//   R  k_rot_mfma  rotation of x (and the single-layer density) for every
//                  target of a latitude, per degree n (Appendix B, gamma = 0), as
//                  GEMMs on the matrix cores; output by order mu:
//                  B^mu[n - mu][col], col = target*6 + comp*2 + re/im
//   L  k_leg_mfma  G^mu = T^mu B^mu on v_mfma_f64_16x16x4f64, T^mu the Legendre
//                  rows [Ptilde_n^mu(t_j'); dPtilde_n^mu/dtheta(t_j')] of the rotated grid
//   FK k_fk        Fourier sums at the rotated longitudes (symmetries phi -> -phi,
//                  phi -> phi + pi), the pole-rule kernels, per-latitude partial sums;
//                  for the double layer the six stresslet fields and their Fourier
//                  analysis Fa^mu[j'][target*12 + pair*2 + re/im]
//   LA k_leg_mfma  Legendre analysis Bt^mu = (Ptilde^mu)^T Fa^mu (same kernel)
//   AR k_adjrot_mfma adjoint rotation (matrix cores) -> rows of the stored double layer
//                  M[t][pair][2 ncoef(p)] (applied by k_dl_apply)
//
// Layouts: a triangle-ordered operand stores order mu as the rows n = mu..p at
// row offset koff(mu) = mu (p+1) - mu (mu-1)/2, each row NC doubles wide.
#include "internal.hpp"

#include <hip/hip_runtime.h>

#include <mutex>

namespace bim {

typedef double d4_t __attribute__((ext_vector_type(4)));

__host__ __device__ inline long koff(int mu, int P1) { return (long)mu * P1 - (long)mu * (mu - 1) / 2; }

// ----------------------------------------------------------------------------
// R: rotation on the matrix cores. Block (n, latitude j), 256 threads. For the
// 2p targets k of latitude j and the nf fields f (x, then the density):
//   Re f'^mu_n(k, f) = sum_nu A+_{nu mu} Re g^nu,  Im f'^mu_n = sum_nu A-_{nu mu} Im g^nu,
//   g^nu = e^{i nu phi_k} c^nu_{n,f},
// two GEMMs (mu x nu) x (nu x col), col = k nf + f, on v_mfma_f64_16x16x4f64:
// A = A+/- from LDS (zero padded to a multiple of 16), B = g formed in
// registers per lane, one 16-column tile per wavefront at a time.
// Output by order mu: B^mu[koff(mu) + n - mu][t*6 + comp*2 + re/im].
// ----------------------------------------------------------------------------
// Stage the N1 x N1 blocks of A+ and A- at lat into LDS ([nu][mu], NP x NP,
// zero padded, row stride NS), the loads of four rounds issued before their
// stores.
__device__ inline void stage_rot(const double *__restrict__ Ap, const double *__restrict__ Am, size_t lat, int N1,
                                 int NP, int NS, double *sAp, double *sAm)
{
    for (int i0 = threadIdx.x; i0 < NP * NP; i0 += 1024) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + 256 * u, nu = i / NP, mu = i % NP;
            const bool in = i < NP * NP && nu < N1 && mu < N1;
            a[u] = in ? Ap[lat + nu * N1 + mu] : 0.0;
            b[u] = in ? Am[lat + nu * N1 + mu] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + 256 * u;
            if (i < NP * NP) {
                const int nu = i / NP, mu = i % NP;
                sAp[nu * NS + mu] = a[u];
                sAm[nu * NS + mu] = b[u];
            }
        }
    }
}

constexpr int kRotMaxPad = 64;  // degree p <= 63

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_rot_mfma(int p, const double *__restrict__ Ap, const double *__restrict__ Am,
                                                  const double *__restrict__ csp, const double *__restrict__ xc0,
                                                  long xstride, const double *__restrict__ dc0, long dstride,
                                                  PipeDrops pd, int u0, double *__restrict__ Bx,
                                                  double *__restrict__ Bd, long NC)
{
    extern __shared__ double sm[];
    const int ug = u0 + blockIdx.y, dr = ug / (p + 1);
    const int n = blockIdx.x, j = ug % (p + 1);
    const double *xc = xc0 + pd.coff[dr];
    const double *dc = dc0 ? dc0 + pd.coff[dr] : nullptr;
    const int N1 = n + 1, nk = 2 * p, P1 = p + 1;
    const int nf = dc ? 6 : 3;
    const int MT = (N1 + 15) / 16, NP = MT * 16, NS = NP + 1, KS = (N1 + 3) / 4;
    double *sAp = sm;                  // [nu][mu], NP x NP, zero padded, row stride NS
    double *sAm = sAp + NP * NS;
    double *sC = sAm + NP * NS;        // [f][nu][re,im]
    double *sCS = sC + nf * N1 * 2;    // cos, sin of the target longitudes [2][nk]
    const size_t lat = rot_lat_size(p) * j + rot_off(n);
    stage_rot(Ap, Am, lat, N1, NP, NS, sAp, sAm);
    const int b0 = n * (n + 1) / 2;
    for (int i = threadIdx.x; i < nf * N1; i += 256) {
        const int f = i / N1, nu = i % N1;
        const double *c = (f < 3) ? xc + f * xstride : dc + (f - 3) * dstride;
        sC[2 * i] = c[2 * (b0 + nu)];
        sC[2 * i + 1] = c[2 * (b0 + nu) + 1];
    }
    for (int i = threadIdx.x; i < 2 * nk; i += 256) sCS[i] = csp[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r16 = lane & 15, k4 = lane >> 4;
    const int ncol = nk * nf, NT = (ncol + 15) / 16;
    for (int nt = wv; nt < NT; nt += 4) {
        const int col = nt * 16 + r16;
        const bool cok = col < ncol;
        const int k = cok ? col / nf : 0, f = cok ? col % nf : 0;
        const double *cf = sC + 2 * f * N1;
        d4_t ap[4], am[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) ap[m] = am[m] = (d4_t){0, 0, 0, 0};
        // e = nu k mod nk, stepped by 4k as nu advances by 4
        int e = (k4 * k) % nk;
        const int step = (4 * k) % nk;
        for (int ks = 0; ks < KS; ++ks) {
            const int nu = ks * 4 + k4;
            double gr = 0.0, gi = 0.0;
            if (cok && nu < N1) {
                const double cr = cf[2 * nu], ci = cf[2 * nu + 1];
                const double cs = sCS[e], sn = sCS[nk + e];
                gr = cr * cs - ci * sn;
                gi = fma(cr, sn, ci * cs);
            }
            e += step;
            if (e >= nk) e -= nk;
            const double *pa = sAp + nu * NS + r16, *pm = sAm + nu * NS + r16;
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (m < MT) {
                    ap[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[m * 16], gr, ap[m], 0, 0, 0);
                    am[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(pm[m * 16], gi, am[m], 0, 0, 0);
                }
        }
        if (!cok) continue;
        const int t = blockIdx.y * nk + k;
        double *dst = (f < 3) ? Bx : Bd;
        const int ff = f < 3 ? f : f - 3;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            if (m < MT)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int mu = m * 16 + 4 * v + k4;
                    if (mu <= n) {
                        double *o = dst + (koff(mu, P1) + (n - mu)) * NC + (long)t * 6 + ff * 2;
                        o[0] = ap[m][v];
                        o[1] = am[m][v];
                    }
                }
    }
}

// ----------------------------------------------------------------------------
// L / LA: batched contraction on the matrix cores.
//   OUT^b[r][col] = sum_k TAB^b[r][k] IN^b[k][col],  b = 0..nb-1,
// with per-batch rows R_b, depth K_b and row offsets; TAB^b row-major R_b x K_b
// at tab_off[b]. Block: all rows of one batch x 64 columns (4 wavefronts x 16).
// ----------------------------------------------------------------------------
struct LegBatch {
    int R, K;          // rows, depth
    long tab_off;      // TAB offset (doubles)
    long in_row;       // first IN row
    long out_row;      // first OUT row
};

template <int MT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_leg_mfma(const LegBatch *__restrict__ bt, const double *__restrict__ tab,
                                                  const double *__restrict__ in, double *__restrict__ out, long NC)
{
    __shared__ double sT[MT * 16 * 53];   // rows padded to MT*16, depth padded to 4 (up to 52), odd row stride
    const LegBatch b = bt[blockIdx.y];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long col = (long)blockIdx.x * 64 + wv * 16 + (lane & 15);
    const bool cok = col < NC;
    const int Kp = (b.K + 3) & ~3, Ks = Kp + 1;
    const int kl = lane >> 4;
    // every B value of the lane loaded before the first product (13 depth
    // steps at most): one memory latency per block instead of one per step
    constexpr int KS = 13;
    double bv[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int k = 4 * s + kl;
        bv[s] = (cok && k < b.K) ? in[(b.in_row + k) * NC + col] : 0.0;
    }
    // stage the table block, zero padded: sT[r][k], r < MT*16, k < Kp, row
    // stride Ks; the loads of eight rounds issued before their stores
    for (int i0 = threadIdx.x; i0 < MT * 16 * Kp; i0 += 8 * 256) {
        double tv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + 256 * u, r = i / Kp, k = i % Kp;
            tv[u] = (i < MT * 16 * Kp && r < b.R && k < b.K) ? tab[b.tab_off + (long)r * b.K + k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + 256 * u;
            if (i < MT * 16 * Kp) sT[(i / Kp) * Ks + i % Kp] = tv[u];
        }
    }
    __syncthreads();
    d4_t acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = (d4_t){0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        if (4 * s >= Kp) break;
        const int k = 4 * s + kl;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const double av = sT[(m * 16 + (lane & 15)) * Ks + k];
            acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[s], acc[m], 0, 0, 0);
        }
    }
    if (!cok) return;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = m * 16 + 4 * v + kl;
            if (r < b.R) out[(b.out_row + r) * NC + col] = acc[m][v];
        }
}

// ----------------------------------------------------------------------------
// FK: Fourier sums and kernels. Block: TG consecutive targets x one rotated
// latitude j'. Gx rows: j' (Ptilde) and Q1 + j' (d/dtheta); Gd row j'.
// SL: partial[t][j'][3] += omega W (f/r + xh (xh.f)/r^3) summed over the longitudes.
// DL: Fa^mu[j'][t*12 + pair*2 + {cos, sin}] of the six stresslet fields.
// ----------------------------------------------------------------------------
// point records of 12 fields padded to an odd number of doubles, so that
// lanes reading consecutive points hit distinct LDS banks
constexpr int kVS = 13;
// Each target's block of point records starts 6 doubles (12 banks) further
// round the LDS banks than the previous one: the Fourier-analysis stage reads
// the same point of up to 4 targets x 6 stresslet fields in one instruction,
// and with blocks a multiple of 32 doubles apart (2 qs 13 is, for even qs)
// those 24 reads fell on 6 bank pairs.
__host__ __device__ inline long fk_vt(int nk) { return (long)nk * kVS + ((6 - (long)nk * kVS % 32) % 32 + 32) % 32; }

// 1/sqrt(x) to full double precision: hardware estimate plus one third-order
// correction (relative error of the estimate e -> O(e^3))
__device__ inline double rsq_full(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}

template <bool SL, bool DL, int TG, int FQ>
__global__ __launch_bounds__(256) void k_fk(int p, int qs, int nt, const double *__restrict__ Gx,
                                            const double *__restrict__ Gd, long NC6,
                                            const double *__restrict__ wsing, const double *__restrict__ cs,
                                            const double *__restrict__ X0, double *__restrict__ part,
                                            double *__restrict__ Fa, long NC12)
{
    extern __shared__ double sm[];
    const int P1 = p + 1, Q1 = qs + 1, nk = 2 * qs;
    const int jr = blockIdx.y;
    const int t0 = blockIdx.x * TG;
    const int ntg = min(TG, nt - t0);
    // sG[tg][mu][type 0..3][c][re,im] ; type 0 x, 1 x_theta, 2 x_phi (= i mu x), 3 density
    constexpr int NTY = SL ? 4 : 3;
    double *sG = sm;
    const long gsz = (long)TG * P1 * NTY * 6;
    const long VT = fk_vt(nk);
    double *V = sG + gsz;                    // [tg][k'][kVS] at tg VT: 12 fields, padded
    double *sCS = V + (long)TG * VT + TG * 3;  // cos, sin of pi e / qs, e < 2 qs
    for (int e = threadIdx.x; e < 2 * nk; e += 256) sCS[e] = cs[e];
    // ---- load G (weights w_mu applied; x_phi built from x). All loads of a
    // thread are issued before the first LDS store (P1 <= 52: at most 5
    // rounds of 3 values), so the block waits for one memory latency.
    constexpr int kGR = (52 * TG * 6 + 255) / 256;
    double lx[kGR], lt[kGR], ld[kGR];
#pragma unroll
    for (int u = 0; u < kGR; ++u) {
        const int i = threadIdx.x + 256 * u;
        lx[u] = lt[u] = ld[u] = 0.0;
        if (i < P1 * ntg * 6) {
            const int e = i % 6, r = i / 6;
            const int tg = r % ntg, mu = r / ntg;
            const long colx = (long)(t0 + tg) * 6 + e;
            lx[u] = Gx[((long)mu * 2 * Q1 + jr) * NC6 + colx];
            lt[u] = Gx[((long)mu * 2 * Q1 + Q1 + jr) * NC6 + colx];
            if (SL) ld[u] = Gd[((long)mu * Q1 + jr) * NC6 + colx];
        }
    }
#pragma unroll
    for (int u = 0; u < kGR; ++u) {
        const int i = threadIdx.x + 256 * u;
        if (i < P1 * ntg * 6) {
            const int e = i % 6;           // c*2 + re/im
            const int r = i / 6;
            const int tg = r % ntg, mu = r / ntg;
            const double w = mu ? 2.0 : 1.0;
            double *g = sG + ((long)(tg * P1 + mu) * NTY) * 6;
            g[e] = w * lx[u];
            g[6 + e] = w * lt[u];
            if (SL) g[18 + e] = w * ld[u];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < P1 * ntg * 3; i += 256) {
        const int c = i % 3;
        const int r = i / 3;
        const int tg = r % ntg, mu = r / ntg;
        double *g = sG + ((long)(tg * P1 + mu) * NTY) * 6;
        // (i mu) (gr + i gi) = (-mu gi) + i (mu gr)
        g[12 + 2 * c] = -mu * g[2 * c + 1];
        g[12 + 2 * c + 1] = mu * g[2 * c];
    }
    __syncthreads();
    const bool even = (qs & 1) == 0;
    const int nkk = even ? qs / 2 + 1 : qs;
    // ---- F: point values. cos/sin(mu phi) by the three-term recurrence
    // c_{mu+1} = 2 cos(phi) c_mu - c_{mu-1} (same for sin), error O(p^2 eps).
    // A thread takes the points kk and kk + H of one (target, component): each
    // G value read from LDS feeds both.
    const int H = (nkk + 1) / 2;
    for (int it = threadIdx.x; it < ntg * H * 3; it += 256) {
        const int c = it % 3;
        const int r = it / 3;
        const int kp = r % H, tg = r / H;
        const int kq[2] = {kp, kp + H};
        const bool two = kp + H < nkk;
        const double *g = sG + (long)tg * P1 * NTY * 6 + 2 * c;
        double tc[2], c0[2], s0[2], cm1[2], sm1[2];
        double CE[2][NTY], CO[2][NTY], SE[2][NTY], SO[2][NTY];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int kb = min(kq[b], nkk - 1);
            const double c1 = sCS[kb], s1 = sCS[nk + kb];
            tc[b] = 2.0 * c1;
            c0[b] = 1.0;
            s0[b] = 0.0;
            cm1[b] = c1;  // orders mu and mu - 1
            sm1[b] = -s1;
#pragma unroll
            for (int q = 0; q < NTY; ++q) { CE[b][q] = 0; CO[b][q] = 0; SE[b][q] = 0; SO[b][q] = 0; }
        }
        // Two register sets of G values (orders mu, mu + 1), filled alternately:
        // the next two orders are read while the current ones are summed.
        // Indexes are clamped to p; values past the last order are never used.
        double ac[NTY], as[NTY], aoc[NTY], aos[NTY], bc[NTY], bs[NTY], boc[NTY], bos[NTY];
        auto gload = [&](int m, double *gc, double *gs) {
            const double *gm = g + (long)m * NTY * 6;
#pragma unroll
            for (int q = 0; q < NTY; ++q) { gc[q] = gm[6 * q]; gs[q] = gm[6 * q + 1]; }
        };
        // orders mu (even) and mu + 1 (odd) added; the recurrences advance by two
        auto step = [&](const double *ec, const double *es, const double *oc, const double *os) {
#pragma unroll
            for (int q = 0; q < NTY; ++q)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    CE[b][q] = fma(ec[q], c0[b], CE[b][q]);
                    SE[b][q] = fma(es[q], s0[b], SE[b][q]);
                }
            double c1n[2], s1n[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                c1n[b] = fma(tc[b], c0[b], -cm1[b]);
                s1n[b] = fma(tc[b], s0[b], -sm1[b]);
            }
#pragma unroll
            for (int q = 0; q < NTY; ++q)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    CO[b][q] = fma(oc[q], c1n[b], CO[b][q]);
                    SO[b][q] = fma(os[q], s1n[b], SO[b][q]);
                }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                cm1[b] = c1n[b];
                sm1[b] = s1n[b];
                c0[b] = fma(tc[b], c1n[b], -c0[b]);
                s0[b] = fma(tc[b], s1n[b], -s0[b]);
            }
        };
        auto last_even = [&](const double *ec, const double *es) {
#pragma unroll
            for (int q = 0; q < NTY; ++q)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    CE[b][q] = fma(ec[q], c0[b], CE[b][q]);
                    SE[b][q] = fma(es[q], s0[b], SE[b][q]);
                }
        };
        gload(0, ac, as);
        gload(min(1, p), aoc, aos);
        int mu = 0;
#pragma unroll 1
        for (; mu + 3 <= p; mu += 4) {
            gload(mu + 2, bc, bs);
            gload(mu + 3, boc, bos);
            __builtin_amdgcn_sched_barrier(0);
            step(ac, as, aoc, aos);
            __builtin_amdgcn_sched_barrier(0);
            gload(min(mu + 4, p), ac, as);
            gload(min(mu + 5, p), aoc, aos);
            __builtin_amdgcn_sched_barrier(0);
            step(bc, bs, boc, bos);
            __builtin_amdgcn_sched_barrier(0);
        }
        // the set a holds orders mu and mu + 1 (clamped)
        if (mu + 1 <= p) {
            step(ac, as, aoc, aos);
            mu += 2;
            if (mu <= p) {
                gload(mu, bc, bs);
                last_even(bc, bs);
            }
        } else if (mu <= p) {
            last_even(ac, as);
        }
        double *Vb = V + (long)tg * VT;
        // value(phi) = (CE - SE) + (CO - SO); at -phi the sine terms flip; at phi + pi the odd orders flip
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            if (b == 1 && !two) break;
            const int kk = kq[b];
            auto put = [&](int kpt, double f1, double f2) {
                double *v = Vb + (long)kpt * kVS;
                v[c] = (CE[b][0] - f1 * SE[b][0]) + f2 * (CO[b][0] - f1 * SO[b][0]);
                v[3 + c] = (CE[b][1] - f1 * SE[b][1]) + f2 * (CO[b][1] - f1 * SO[b][1]);
                v[6 + c] = (CE[b][2] - f1 * SE[b][2]) + f2 * (CO[b][2] - f1 * SO[b][2]);
                if (SL) v[9 + c] = (CE[b][3] - f1 * SE[b][3]) + f2 * (CO[b][3] - f1 * SO[b][3]);
            };
            put(kk, 1.0, 1.0);
            put(kk + qs, 1.0, -1.0);
            if (even && kk != 0 && kk != qs / 2) {
                put(nk - kk, -1.0, 1.0);
                put(qs - kk, -1.0, -1.0);
            }
        }
    }
    __syncthreads();
    // ---- K: kernels
    const double om = wsing[jr];
    for (int it = threadIdx.x; it < ((ntg * nk + 63) & ~63); it += 256) {
        const bool ok = it < ntg * nk;
        const int tg = ok ? it / nk : 0;
        double *v = V + (long)tg * VT + (long)(ok ? it % nk : 0) * kVS;
        const int t = t0 + tg;
        double e0 = 0.0, e1 = 0.0, e2 = 0.0;
        if (ok) {
            const double xt0 = v[3], xt1 = v[4], xt2 = v[5];
            const double xp0 = v[6], xp1 = v[7], xp2 = v[8];
            const double N0 = xt1 * xp2 - xt2 * xp1;
            const double N1 = xt2 * xp0 - xt0 * xp2;
            const double N2 = xt0 * xp1 - xt1 * xp0;
            const double h0 = X0[3 * t] - v[0], h1 = X0[3 * t + 1] - v[1], h2 = X0[3 * t + 2] - v[2];
            const double r2 = h0 * h0 + h1 * h1 + h2 * h2;
            const double ri = rsq_full(r2);
            if (SL) {
                const double f0 = v[9], f1 = v[10], f2 = v[11];
                const double hf = h0 * f0 + h1 * f1 + h2 * f2;
                const double n2 = N0 * N0 + N1 * N1 + N2 * N2;
                const double Wr = om * (n2 * rsq_full(n2)) * ri;
                const double q = hf * ri * ri;
                e0 = Wr * fma(h0, q, f0);
                e1 = Wr * fma(h1, q, f1);
                e2 = Wr * fma(h2, q, f2);
            }
            if (DL) {
                const double hn = h0 * N0 + h1 * N1 + h2 * N2;
                const double r2i = ri * ri;
                const double sc = -6.0 * om * hn * r2i * r2i * ri;
                v[0] = sc * h0 * h0;
                v[1] = sc * h0 * h1;
                v[2] = sc * h0 * h2;
                v[3] = sc * h1 * h1;
                v[4] = sc * h1 * h2;
                v[5] = sc * h2 * h2;
            }
        }
        if (SL && ok) {  // f is read; its slots take the point's contribution
            v[9] = e0;
            v[10] = e1;
            v[11] = e2;
        }
    }
    __syncthreads();
    if (SL) {
        // sums over the longitudes in a fixed order (run to run identical):
        // 16 lanes per (target, component), lane l adds the points l, l + 16,
        // ..., then a butterfly over the 16 lanes
        for (int i0 = 0; i0 < ntg * 48; i0 += 256) {
            const int i = i0 + threadIdx.x;
            const bool act = i < ntg * 48;
            const int g = act ? i >> 4 : 0, l = i & 15;
            const int tg = g / 3, cc = g % 3;
            double sum = 0.0;
            if (act)
                for (int k = l; k < nk; k += 16) sum += V[(long)tg * VT + (long)k * kVS + 9 + cc];
            for (int o = 8; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 16);
            if (act && l == 0) part[((long)(t0 + tg) * Q1 + jr) * 3 + cc] = sum;
        }
    }
    if (DL) {
        // ---- FA: Fourier analysis of the six stresslet fields. One item = FQ
        // orders of one parity (mu = base + 2q), sharing the symmetric
        // combinations of the four points kk, -kk, kk + qs, qs - kk; FQ is
        // the smallest that lets one pass of the block's threads take every
        // item (a second, mostly idle pass would cost a whole item's time).
        const int nE = p / 2 + 1, nO = (p + 1) / 2;
        const int NGe = (nE + FQ - 1) / FQ, NG = NGe + (nO + FQ - 1) / FQ;
        for (int it = threadIdx.x; it < NG * ntg * 6; it += 256) {
            const int pr = it % 6;
            const int r = it / 6;
            const int tg = r % ntg, gidx = r / ntg;
            const bool odd = gidx >= NGe;
            const int base = odd ? 2 * FQ * (gidx - NGe) + 1 : 2 * FQ * gidx;
            const double sg = odd ? -1.0 : 1.0;
            const double *Vb = V + (long)tg * VT + pr;
            double tq[FQ], cq[FQ], sq[FQ], cp[FQ], sp[FQ], fc[FQ], fs[FQ];
#pragma unroll
            for (int q = 0; q < FQ; ++q) {
                const int mu = min(base + 2 * q, p);
                const double c1 = sCS[mu], s1 = sCS[nk + mu];
                tq[q] = 2.0 * c1;
                cq[q] = 1.0;
                sq[q] = 0.0;
                cp[q] = c1;
                sp[q] = -s1;
                fc[q] = 0.0;
                fs[q] = 0.0;
            }
            for (int kk = 0; kk < nkk; ++kk) {
                const double K1 = Vb[(long)kk * kVS];
                const double K3 = Vb[(long)(kk + qs) * kVS];
                double K2 = 0.0, K4 = 0.0;
                if (even && kk != 0 && kk != qs / 2) {
                    K2 = Vb[(long)(nk - kk) * kVS];
                    K4 = Vb[(long)(qs - kk) * kVS];
                }
                const double A = fma(sg, K3 + K4, K1 + K2);
                const double Bv = fma(sg, K3 - K4, K1 - K2);
#pragma unroll
                for (int q = 0; q < FQ; ++q) {
                    fc[q] = fma(cq[q], A, fc[q]);
                    fs[q] = fma(sq[q], Bv, fs[q]);
                    const double cn = fma(tq[q], cq[q], -cp[q]), sn = fma(tq[q], sq[q], -sp[q]);
                    cp[q] = cq[q];
                    sp[q] = sq[q];
                    cq[q] = cn;
                    sq[q] = sn;
                }
            }
#pragma unroll
            for (int q = 0; q < FQ; ++q) {
                const int mu = base + 2 * q;
                if (mu <= p) {
                    double *o = Fa + ((long)mu * Q1 + jr) * NC12 + (long)(t0 + tg) * 12 + pr * 2;
                    o[0] = fc[q];
                    o[1] = fs[q];
                }
            }
        }
    }
}

// part[t][j'][3] summed over j' into out (scaled, added); column t belongs to
// unit u0 + t / nk of the pass.
__global__ void k_sum_part(int nt, int Q1, int nk, int P1, const double *__restrict__ part, PipeDrops pd, int u0,
                           double scale, double *__restrict__ out, long ostride)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt * 3) return;
    const int t = i / 3, c = i % 3;
    double s = 0.0;
    for (int j = 0; j < Q1; ++j) s += part[((long)t * Q1 + j) * 3 + c];
    const int ug = u0 + t / nk;
    out[c * ostride + pd.toff[ug / P1] + (long)(ug % P1) * nk + t % nk] += scale * s;
}

// Pole values x0 of every target: sum_n Re x'^0_n sqrt((2n+1)/4pi) from the
// mu = 0 block of the rotated x (col = t*6 + c*2).
__global__ void k_pole(int p, int nt, const double *__restrict__ Bx, long NC, double *__restrict__ X0)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt * 3) return;
    const int t = i / 3, c = i % 3;
    double s = 0.0;
    for (int n = 0; n <= p; ++n) s += Bx[(long)n * NC + (long)t * 6 + 2 * c] * sqrt((2.0 * n + 1.0) / (4.0 * 3.14159265358979323846));
    X0[3 * t + c] = s;
}

// ----------------------------------------------------------------------------
// AR: adjoint rotation on the matrix cores. Block (n, latitude j), 256 threads.
// a_mu = w_mu Bt^mu[n][.. cos], b_mu = -w_mu Bt^mu[n][.. sin] (w_0 = 1, else 2);
// alpha_nu = sum_mu A+_{nu mu} a_mu, beta_nu = sum_mu A-_{nu mu} b_mu as two GEMMs
// (nu x mu) x (mu x col), col = k*6 + pair over the 2p targets of the latitude;
// both results of one (nu, col) land in the same lane, which writes
// M[t][pair][2 tri(n,nu)] = alpha cos(nu phi_k) + beta sin, [+1] = -alpha sin + beta cos.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_adjrot_mfma(int p, const double *__restrict__ Ap,
                                                     const double *__restrict__ Am, const double *__restrict__ csp,
                                                     const double *__restrict__ Bt, long NC12, PipeDrops pd,
                                                     int u0)
{
    extern __shared__ double sm[];
    const int ug = u0 + blockIdx.y, dr = ug / (p + 1);
    const int n = blockIdx.x, j = ug % (p + 1);
    double *__restrict__ M = pd.M[dr];
    const int N1 = n + 1, nk = 2 * p, P1 = p + 1;
    const int MT = (N1 + 15) / 16, NP = MT * 16, NS = NP + 1, KS = (N1 + 3) / 4;
    double *sAp = sm;                  // [nu][mu], NP x NP, zero padded, row stride NS
    double *sAm = sAp + NP * NS;
    double *sCS = sAm + NP * NS;       // [2][nk]
    const size_t lat = rot_lat_size(p) * j + rot_off(n);
    stage_rot(Ap, Am, lat, N1, NP, NS, sAp, sAm);
    for (int i = threadIdx.x; i < 2 * nk; i += 256) sCS[i] = csp[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r16 = lane & 15, k4 = lane >> 4;
    const int ncol = nk * 6, NT = (ncol + 15) / 16;
    const int nc2 = 2 * ncoef(p);
    for (int nt = wv; nt < NT; nt += 4) {
        const int col = nt * 16 + r16;
        const bool cok = col < ncol;
        const int k = cok ? col / 6 : 0, pr = cok ? col % 6 : 0;
        const long tcol = (long)(blockIdx.y * nk + k) * 12 + pr * 2;
        d4_t al[4], be[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) al[m] = be[m] = (d4_t){0, 0, 0, 0};
        // the next depth step's B operand is loaded while this one's products run
        auto bload = [&](int ks) {
            const int mu = ks * 4 + k4;
            return (cok && mu < N1) ? *reinterpret_cast<const double2 *>(Bt + (koff(mu, P1) + (n - mu)) * NC12 + tcol)
                                    : make_double2(0.0, 0.0);
        };
        double2 vn = bload(0);
        for (int ks = 0; ks < KS; ++ks) {
            const int mu = ks * 4 + k4;
            const double2 v = vn;
            if (ks + 1 < KS) vn = bload(ks + 1);
            const double w = mu ? 2.0 : 1.0;
            const double av = w * v.x, bv = -w * v.y;
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (m < MT) {
                    const int nu = m * 16 + r16;
                    al[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(sAp[nu * NS + mu], av, al[m], 0, 0, 0);
                    be[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(sAm[nu * NS + mu], bv, be[m], 0, 0, 0);
                }
        }
        if (!cok) continue;
        const long tg = (long)j * nk + k;  // target index within the drop
        double *Mt = M + (tg * 6 + pr) * nc2 + n * (n + 1);
#pragma unroll
        for (int m = 0; m < 4; ++m)
            if (m < MT)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int nu = m * 16 + 4 * v + k4;
                    if (nu <= n) {
                        const int e = (int)(((long)nu * k) % nk);
                        const double cc = sCS[e], ss = sCS[nk + e];
                        const double a_ = al[m][v], b_ = be[m][v];
                        *reinterpret_cast<double2 *>(Mt + 2 * nu) =
                            make_double2(fma(a_, cc, b_ * ss), fma(-a_, ss, b_ * cc));
                    }
                }
    }
}

// ============================================================================
// launchers
// ============================================================================
static inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

// allow up to 160 KB of dynamic LDS for the kernels that size it by degree
// (once per process, before any of them is launched: server worker threads
// reach this concurrently, and call_once makes the others wait until it is set)
void pipe_set_lds_limits()
{
    static std::once_flag once;
    std::call_once(once, [] {
        for (const void *fn : {(const void *)k_fk<true, true, 4, 2>, (const void *)k_fk<true, true, 4, 3>,
                               (const void *)k_fk<true, true, 4, 4>, (const void *)k_fk<true, true, 4, 5>,
                               (const void *)k_fk<true, true, 4, 7>, (const void *)k_fk<true, false, 4, 4>,
                               (const void *)k_fk<false, true, 4, 2>, (const void *)k_fk<false, true, 4, 3>,
                               (const void *)k_fk<false, true, 4, 4>, (const void *)k_fk<false, true, 4, 5>,
                               (const void *)k_fk<false, true, 4, 7>})
            (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
    });
}

void launch_rot2(hipStream_t st, int p, const double *Ap, const double *Am, const double *csp, const double *xc,
                 long xstride, const double *dc, long dstride, const PipeDrops &pd, int u0, int nunits,
                 double *Bx, double *Bd, long NC)
{
    const int P1 = p + 1, nk = 2 * p, NP = (P1 + 15) / 16 * 16;
    const int nf = dc ? 6 : 3;
    const size_t lds = (size_t)(2 * NP * (NP + 1) + nf * P1 * 2 + 2 * nk) * sizeof(double);
    hipLaunchKernelGGL(k_rot_mfma, dim3(P1, nunits), dim3(256), lds, st, p, Ap, Am, csp, xc, xstride, dc, dstride,
                       pd, u0, Bx, Bd, NC);
}

size_t rot_lds_bytes(int p)
{
    const int P1 = p + 1, NP = (P1 + 15) / 16 * 16;
    return P1 > kRotMaxPad ? (size_t)1 << 40 : (size_t)(2 * NP * (NP + 1) + 6 * P1 * 2 + 4 * p) * sizeof(double);
}

void launch_leg_mfma(hipStream_t st, int nbatch, int maxrows, const void *batches, const double *tab, const double *in,
                     double *out, long NC)
{
    const dim3 grid(cdiv(NC, 64), nbatch);
    const LegBatch *b = static_cast<const LegBatch *>(batches);
    const int MT = (maxrows + 15) / 16;
    switch (MT) {
    case 1: hipLaunchKernelGGL(k_leg_mfma<1>, grid, dim3(256), 0, st, b, tab, in, out, NC); break;
    case 2: hipLaunchKernelGGL(k_leg_mfma<2>, grid, dim3(256), 0, st, b, tab, in, out, NC); break;
    case 3: hipLaunchKernelGGL(k_leg_mfma<3>, grid, dim3(256), 0, st, b, tab, in, out, NC); break;
    case 4: hipLaunchKernelGGL(k_leg_mfma<4>, grid, dim3(256), 0, st, b, tab, in, out, NC); break;
    case 5: hipLaunchKernelGGL(k_leg_mfma<5>, grid, dim3(256), 0, st, b, tab, in, out, NC); break;
    case 6: hipLaunchKernelGGL(k_leg_mfma<6>, grid, dim3(256), 0, st, b, tab, in, out, NC); break;
    default: hipLaunchKernelGGL(k_leg_mfma<7>, grid, dim3(256), 0, st, b, tab, in, out, NC); break;
    }
}

int leg_mfma_max_rows() { return 7 * 16; }
int leg_mfma_max_depth() { return 52; }

size_t fk_lds_bytes(int p, int qs, bool sl, int tg)
{
    const int nty = sl ? 4 : 3;
    return ((size_t)tg * (p + 1) * nty * 6 + (size_t)tg * fk_vt(2 * qs) + (size_t)tg * 3 + 4 * (size_t)qs) *
           sizeof(double);
}

void launch_fk(hipStream_t st, bool sl, bool dl, int p, int qs, int nt, const double *Gx, const double *Gd, long NC6,
               const double *wsing, const double *cs, const double *X0, double *part, double *Fa, long NC12)
{
    constexpr int TG = 4;
    const dim3 grid(cdiv(nt, TG), qs + 1);
    const size_t lds = fk_lds_bytes(p, qs, sl, TG);
    // orders per item of the stresslet analysis: the smallest with every item
    // in one pass of the 256 threads
    const int nE = p / 2 + 1, nO = (p + 1) / 2;
    int fq = 7;
    for (int q : {2, 3, 4, 5, 7})
        if (((nE + q - 1) / q + (nO + q - 1) / q) * TG * 6 <= 256) {
            fq = q;
            break;
        }
    auto go = [&](auto fqc) {
        constexpr int FQ = decltype(fqc)::value;
        if (sl && dl)
            hipLaunchKernelGGL((k_fk<true, true, TG, FQ>), grid, dim3(256), lds, st, p, qs, nt, Gx, Gd, NC6, wsing, cs,
                               X0, part, Fa, NC12);
        else if (sl)
            hipLaunchKernelGGL((k_fk<true, false, TG, 4>), grid, dim3(256), lds, st, p, qs, nt, Gx, Gd, NC6, wsing, cs,
                               X0, part, Fa, NC12);
        else
            hipLaunchKernelGGL((k_fk<false, true, TG, FQ>), grid, dim3(256), lds, st, p, qs, nt, Gx, Gd, NC6, wsing, cs,
                               X0, part, Fa, NC12);
    };
    switch (fq) {
    case 2: go(std::integral_constant<int, 2>()); break;
    case 3: go(std::integral_constant<int, 3>()); break;
    case 4: go(std::integral_constant<int, 4>()); break;
    case 5: go(std::integral_constant<int, 5>()); break;
    default: go(std::integral_constant<int, 7>()); break;
    }
}

void launch_sum_part(hipStream_t st, int nt, int Q1, int nk, int P1, const double *part, const PipeDrops &pd, int u0,
                     double scale, double *out, long ostride)
{
    hipLaunchKernelGGL(k_sum_part, dim3(cdiv((long)nt * 3, 256)), dim3(256), 0, st, nt, Q1, nk, P1, part, pd, u0, scale,
                       out, ostride);
}

void launch_pole(hipStream_t st, int p, int nt, const double *Bx, long NC, double *X0)
{
    hipLaunchKernelGGL(k_pole, dim3(cdiv((long)nt * 3, 256)), dim3(256), 0, st, p, nt, Bx, NC, X0);
}

void launch_adjrot(hipStream_t st, int p, const double *Ap, const double *Am, const double *csp, const double *Bt,
                   long NC12, const PipeDrops &pd, int u0, int nunits)
{
    const int P1 = p + 1, nk = 2 * p, NP = (P1 + 15) / 16 * 16;
    const size_t lds = (size_t)(2 * NP * (NP + 1) + 2 * nk) * sizeof(double);
    hipLaunchKernelGGL(k_adjrot_mfma, dim3(P1, nunits), dim3(256), lds, st, p, Ap, Am, csp, Bt, NC12, pd, u0);
}

}  // namespace bim
