// Batched spherical-harmonic transforms (gfx950, FP64).
//
// Synthesis (Sec. 1.1, derivatives by Appendix A) and analysis (Sec. 2.1)
// for many (drop, grid, field) jobs in one launch; the job list travels in the
// kernel arguments.
//
// Synthesis block = (job, latitude j, range of 64 longitudes): Legendre sums G[c][kind][m] =
// sum_n c_n^m L_kind(t_j) for the kinds the requested derivatives need, into
// LDS; then each thread forms points k and k + q of one output field with the
// even/odd split e^{i m (phi + pi)} = (-1)^m e^{i m phi}.
// Analysis block = (job, component, chunk of four orders m): F[j][m] =
// sum_k v_jk e^{-i m phi_k} into LDS, then f_n^m = sum_j (pi/q) w_j h_m
// Ptilde_n^m(t_j) F[j][m] with h_q = 1/2 (grids up to q = 512).
#include "internal.hpp"

#include <hip/hip_runtime.h>

namespace bim {

// derivative sets (d/dtheta order, d/dphi order) by mask bit
__constant__ int kDt[6] = {0, 1, 0, 2, 1, 0};
__constant__ int kDp[6] = {0, 0, 1, 0, 1, 2};

struct SynJob {
    const double *coef;   // component c at coef + c * cstride
    const double *L;      // Legendre tables [3][q+1][ldn]
    double *out;          // field f, component c at out + f * fstride + c * ostride
    long cstride, ostride, fstride;
    int p, q, ldn, ncomp, mask;
};

constexpr int kMaxSynJobs = 20;
struct SynJobs {
    int n;
    double *zero[2];  // optional ranges cleared by the launch (accumulators of the pass that follows)
    long nzero[2];
    SynJob j[kMaxSynJobs];
};

constexpr int kSynK = 64;  // longitudes k <= q/2 (and their images k + q, -k, q - k) per synthesis block

__global__ __launch_bounds__(256) void k_synth_batch(SynJobs jobs)
{
    __shared__ double G[3 * 3 * 65 * 2];  // [c][kind][m][re,im]
    {
        const long nb = (long)gridDim.x * gridDim.y * gridDim.z;
        const long bid = ((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        for (int z = 0; z < 2; ++z)
            if (jobs.zero[z])
                for (long i = bid * 256 + threadIdx.x; i < jobs.nzero[z]; i += nb * 256) jobs.zero[z][i] = 0.0;
    }
    const SynJob &J = jobs.j[blockIdx.y];
    const int j = blockIdx.x;
    const int k0 = blockIdx.z * kSynK;
    const int H = J.q / 2 + 1;  // longitudes k <= q/2; the others by symmetry
    if (j > J.q || k0 >= H) return;
    const int kn = min(kSynK, H - k0);
    const int p = J.p, P1 = p + 1, q = J.q, nk = 2 * q;
    int kinds = 0;  // bit 0: Ptilde, 1: d/dtheta, 2: d2/dtheta2
    for (int b = 0; b < 6; ++b)
        if (J.mask >> b & 1) kinds |= 1 << kDt[b];
    const int nq = J.q + 1;
    for (int it = threadIdx.x; it < J.ncomp * 3 * P1; it += 256) {
        const int m = it % P1;
        const int r = it / P1;
        const int kind = r % 3, c = r / 3;
        if (!(kinds >> kind & 1)) continue;
        const double *cf = J.coef + c * J.cstride;
        const double *Lj = J.L + ((long)kind * nq + j) * J.ldn;
        double sr = 0.0, si = 0.0;
        int e = m * (m + 1) / 2 + m;
#pragma unroll 4
        for (int n = m; n <= p; ++n) {
            const double l = Lj[e];
            sr = fma(cf[2 * e], l, sr);
            si = fma(cf[2 * e + 1], l, si);
            e += n + 1;
        }
        G[2 * ((c * 3 + kind) * P1 + m)] = sr;
        G[2 * ((c * 3 + kind) * P1 + m) + 1] = si;
    }
    __syncthreads();
    int nout = 0, fidx[6];
    for (int b = 0; b < 6; ++b)
        if (J.mask >> b & 1) fidx[nout++] = b;
    const double dphi = 3.14159265358979323846 / q;
    for (int it = threadIdx.x; it < J.ncomp * nout * kn; it += 256) {
        const int k = k0 + it % kn;
        const int r = it / kn;
        const int fo = r % nout, c = r / nout;
        const int b = fidx[fo], dt = kDt[b], dp = kDp[b];
        const double *g = G + 2 * ((c * 3 + dt) * P1);
        double sn, cs;
        sincos(dphi * k, &sn, &cs);
        // cosine and sine sums kept apart (C - S at phi, C + S at -phi) and
        // split by the parity of m (the odd orders flip at phi + pi)
        double cm = 1.0, sm = 0.0, ce = 0.0, co = 0.0, se = 0.0, so = 0.0;
        for (int m = 0; m <= p; ++m) {
            double ar = g[2 * m], ai = g[2 * m + 1];
            if (dp == 1) {
                const double t = -m * ai;
                ai = m * ar;
                ar = t;
            } else if (dp == 2) {
                ar *= -(double)m * m;
                ai *= -(double)m * m;
            }
            const double w = m ? 2.0 : 1.0;
            const double vc = w * ar * cm, vs = w * ai * sm;
            if (m & 1) {
                co += vc;
                so += vs;
            } else {
                ce += vc;
                se += vs;
            }
            const double c2 = cm * cs - sm * sn;
            sm = fma(sm, cs, cm * sn);
            cm = c2;
        }
        double *o = J.out + fo * J.fstride + c * J.ostride + (long)j * nk;
        o[k] = (ce - se) + (co - so);      // phi_k
        o[k + q] = (ce - se) - (co - so);  // phi_k + pi
        if (k > 0 && 2 * k != q) {
            o[nk - k] = (ce + se) + (co + so);  // -phi_k
            o[q - k] = (ce + se) - (co + so);   // pi - phi_k
        }
    }
}

constexpr int kMaxAnaJobs = 24;
struct AnaJobs {
    int n;
    AnaJob j[kMaxAnaJobs];
};

constexpr int kAnaMC = 4;  // orders m per analysis block

// block = (job, component x chunk of kAnaMC orders)
__global__ __launch_bounds__(256) void k_anal_batch(AnaJobs jobs)
{
    __shared__ double F[513 * kAnaMC * 2];  // [j][m - m0][re,im]
    const AnaJob &J = jobs.j[blockIdx.y];
    const int p = J.p, P1 = p + 1, q = J.q, nj = q + 1, nk = 2 * q;
    const int nch = (P1 + kAnaMC - 1) / kAnaMC;
    const int c = blockIdx.x / nch, ch = blockIdx.x % nch;
    if (c >= J.ncomp) return;
    const int m0 = ch * kAnaMC, mc = min(kAnaMC, P1 - m0);
    const double *v = J.v + c * J.vstride;
    const double dphi = 3.14159265358979323846 / q;
    for (int it = threadIdx.x; it < nj * mc; it += 256) {
        const int mm = it % mc, j = it / mc;
        const int m = m0 + mm;
        const double *row = v + (long)j * nk;
        double sn, cs;
        sincos(dphi * m, &sn, &cs);
        double ck = 1.0, sk = 0.0, fr = 0.0, fi = 0.0;
        // 16 longitudes per step: their loads are issued together (the loads do
        // not depend on the recurrence, but a shorter step waits on each batch)
#pragma unroll 16
        for (int k = 0; k < nk; ++k) {
            fr = fma(row[k], ck, fr);
            fi = fma(-row[k], sk, fi);
            const double c2 = ck * cs - sk * sn;
            sk = fma(sk, cs, ck * sn);
            ck = c2;
        }
        F[2 * (j * kAnaMC + mm)] = fr;
        F[2 * (j * kAnaMC + mm) + 1] = fi;
    }
    __syncthreads();
    double *out = J.coef + c * J.cstride;
    // coefficients (n, m) with m0 <= m < m0 + mc, n = m..p
    int cnt = 0;
    for (int mm = 0; mm < mc; ++mm) cnt += P1 - (m0 + mm);
    for (int it = threadIdx.x; it < cnt; it += 256) {
        int mm = 0, r = it;
        while (r >= P1 - (m0 + mm)) { r -= P1 - (m0 + mm); ++mm; }
        const int m = m0 + mm, n = m + r;
        const int e = n * (n + 1) / 2 + m;
        const double h = (m == q) ? 0.5 : 1.0;
        double sr = 0.0, si = 0.0;
#pragma unroll 8
        for (int j = 0; j < nj; ++j) {
            const double w = J.wq[j] * J.L[(long)j * J.ldn + e] * h;
            sr = fma(w, F[2 * (j * kAnaMC + mm)], sr);
            si = fma(w, F[2 * (j * kAnaMC + mm) + 1], si);
        }
        if (J.cx) {  // Galerkin combine: csc x - P[...]
            const double *x = J.cx + c * J.cstride;
            out[2 * e] = fma(J.csc, x[2 * e], -sr);
            out[2 * e + 1] = fma(J.csc, x[2 * e + 1], -si);
        } else {
            out[2 * e] = sr;
            out[2 * e + 1] = si;
        }
    }
}

// ----------------------------------------------------------------------------
// host side: job collectors that flush full batches
// ----------------------------------------------------------------------------
void launch_synth_batch(hipStream_t st, const SynJob *jobs, int n, double *z0, long nz0, double *z1, long nz1)
{
    for (int o = 0; o < n; o += kMaxSynJobs) {
        SynJobs b{};
        b.n = std::min(kMaxSynJobs, n - o);
        if (o == 0) {
            b.zero[0] = nz0 > 0 ? z0 : nullptr;
            b.nzero[0] = nz0;
            b.zero[1] = nz1 > 0 ? z1 : nullptr;
            b.nzero[1] = nz1;
        }
        int maxq = 0;
        for (int i = 0; i < b.n; ++i) {
            b.j[i] = jobs[o + i];
            maxq = std::max(maxq, jobs[o + i].q);
        }
        hipLaunchKernelGGL(k_synth_batch, dim3(maxq + 1, b.n, (maxq / 2 + 1 + kSynK - 1) / kSynK), dim3(256), 0, st, b);
    }
}

size_t anal_batch_lds(int p, int q) { return q <= 512 ? 0 : (size_t)1 << 40; }

void launch_anal_batch(hipStream_t st, const AnaJob *jobs, int n)
{
    for (int o = 0; o < n; o += kMaxAnaJobs) {
        AnaJobs b{};
        b.n = std::min(kMaxAnaJobs, n - o);
        int maxblk = 0;
        for (int i = 0; i < b.n; ++i) {
            b.j[i] = jobs[o + i];
            const int nch = (jobs[o + i].p + 1 + kAnaMC - 1) / kAnaMC;
            maxblk = std::max(maxblk, jobs[o + i].ncomp * nch);
        }
        hipLaunchKernelGGL(k_anal_batch, dim3(maxblk, b.n), dim3(256), 0, st, b);
    }
}

// ----------------------------------------------------------------------------
// Matrix-core transforms of value fields: the Legendre and Fourier sums of
// synthesis (Sec. 1.1) and analysis (Sec. 2.1) as batched contractions on
// v_mfma_f64_16x16x4f64 (FP64) or v_mfma_f32_16x16x4f32 (FP32 operands and
// accumulation, the mixed form). Columns are (field, re/im) pairs, col = 2 f
// + ri, of every field of a job (one degree group of drops, or the fields of
// a stand-alone call); the intermediate G is [m][j][col].
//   synthesis, Legendre:  G[m][j][col] = sum_{n=m..p} Ptilde_n^m(t_j) c_n^m[col]
//   synthesis, Fourier:   v[f][j][k] = E + O, v[f][j][k + q] = E - O (k < q),
//       E (O) = sum over even (odd) m of w_m (Re G cos m phi_k - Im G sin m phi_k),
//       w_0 = 1, w_m = 2: the orders m < 0 of a real field, and the shift
//       by pi flipping the odd orders
//   analysis, Fourier:    G[m][j][col] = sum_{k<q} (v_k + (-1)^m v_{k+q}) (cos, -sin)(m phi_k)
//   analysis, Legendre:   c_n^m = sum_j (pi/q) w_j h_m Ptilde_n^m(t_j) G[m][j],
//       h_q = 1/2 (the Nyquist order of the 2q-point grid), then
//       y = csc[f] x + sgn c.
// Operand layout of both 16x16x4 instructions: lane l holds A[l & 15][l >> 4]
// and B[l >> 4][l & 15]; accumulator element v of lane l is row 4 v + (l >> 4)
// (FP64) or 4 (l >> 4) + v (FP32) of column l & 15.
// ----------------------------------------------------------------------------
typedef double xd4 __attribute__((ext_vector_type(4)));
typedef float xf4 __attribute__((ext_vector_type(4)));

template <typename TY> struct Mma;
template <> struct Mma<double> {
    typedef xd4 acc;
    __device__ static acc run(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <> struct Mma<float> {
    typedef xf4 acc;
    __device__ static acc run(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

struct XJobs {
    int n;
    double *zero[2];  // synthesis: optional ranges cleared by the launch
    long nzero[2];
    XJob j[kMaxXJobs];
};

constexpr int kXRows = 64;   // rows per Legendre block (four 16-row tiles)
constexpr int kXDepth = 64;  // largest depth of a Legendre block (degree or latitudes)
constexpr int kXSteps = kXDepth / 4;  // K steps of 4 at most; every operand a lane needs is loaded before the first
                                      // product (one memory latency per kernel, not one per step)

// Legendre stage of synthesis. Block: (64 columns, order m x latitude chunk
// of kXRows, job); the table block T[r][k] = Ptilde_{m+k}^m(t_{r0+r}) staged
// in LDS (row stride odd), zero padded.
template <typename TY>
__global__ __launch_bounds__(256) void k_xs_leg(XJobs J, const double *__restrict__ x)
{
    __shared__ TY sT[kXRows * (kXDepth + 1)];
    {
        const long nb = (long)gridDim.x * gridDim.y * gridDim.z;
        const long bid = ((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        for (int z = 0; z < 2; ++z)
            if (J.zero[z])
                for (long i = bid * 256 + threadIdx.x; i < J.nzero[z]; i += nb * 256) J.zero[z][i] = 0.0;
    }
    const XJob &b = J.j[blockIdx.z];
    const int p = b.p, nq = b.q + 1, NC = 2 * b.nf;
    const int nch = (nq + kXRows - 1) / kXRows;
    const int m = blockIdx.y / nch, r0 = (blockIdx.y % nch) * kXRows;
    const int c0 = blockIdx.x * 64;
    if (m > p || c0 >= NC) return;
    const int K = p - m + 1, Kp = (K + 3) & ~3, Ks = Kp + 1;
    const int lane = threadIdx.x & 63, kl = lane >> 4, l16 = lane & 15;
    const int col = c0 + (threadIdx.x >> 6) * 16 + l16;
    const bool cok = col < NC;
    const long cbase = cok ? b.cb[col] : 0;
    TY bv[kXSteps];
#pragma unroll
    for (int s = 0; s < kXSteps; ++s) {
        const int k = 4 * s + kl;
        bv[s] = (cok && k < K) ? (TY)x[cbase + 2 * tri(m + k, m)] : (TY)0;
    }
    TY tv[kXRows * kXDepth / 256];
#pragma unroll
    for (int u = 0; u < kXRows * kXDepth / 256; ++u) {
        const int i = threadIdx.x + 256 * u, r = i / Kp, k = i % Kp, j = r0 + r;
        tv[u] = (i < kXRows * Kp && j < nq && k < K) ? (TY)b.L[(long)j * b.ldn + tri(m + k, m)] : (TY)0;
    }
#pragma unroll
    for (int u = 0; u < kXRows * kXDepth / 256; ++u) {
        const int i = threadIdx.x + 256 * u;
        if (i < kXRows * Kp) sT[(i / Kp) * Ks + i % Kp] = tv[u];
    }
    __syncthreads();
    const int nt = min(4, (nq - r0 + 15) / 16);  // row tiles holding latitudes
    typename Mma<TY>::acc acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = (typename Mma<TY>::acc){0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < kXSteps; ++s) {
        if (4 * s >= Kp) break;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (t < nt) acc[t] = Mma<TY>::run(sT[(t * 16 + l16) * Ks + 4 * s + kl], bv[s], acc[t]);
    }
    if (!cok) return;
    TY *G = (TY *)b.G;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = r0 + t * 16 + Mma<TY>::row(lane, v);
            if (t < nt && j < nq) G[((long)m * nq + j) * NC + col] = acc[t][v];
        }
}

// Fourier stage of synthesis. Wavefront: (16 fields x 16 longitudes k < q,
// latitude j, job); K steps over (m, m + 2) x (re, im), the even orders into
// E, the odd ones into O.
template <typename TY>
__global__ __launch_bounds__(256) void k_xs_fourier(XJobs J)
{
    const XJob &b = J.j[blockIdx.z];
    const int p = b.p, q = b.q, nq = q + 1, NC = 2 * b.nf, j = blockIdx.y;
    const int nkt = (q + 15) / 16, nft = (b.nf + 15) / 16;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= nq || tile >= nkt * nft) return;
    const int ft = tile / nkt, kt = tile % nkt;
    const int lane = threadIdx.x & 63, kl = lane >> 4, l16 = lane & 15;
    const int fa = ft * 16 + l16, kb = kt * 16 + l16;  // A row (field), B column (longitude)
    const bool fok = fa < b.nf, kok = kb < q;
    const TY *G = (const TY *)b.G + (long)j * NC + 2 * fa + (kl & 1);
    const TY *Tr = (const TY *)b.trig + (long)(kl & 1) * q + kb;
    const long ms = (long)nq * NC;
    TY ae[kXSteps], be[kXSteps], ao[kXSteps], bo[kXSteps];
#pragma unroll
    for (int s = 0; s < kXSteps; ++s) {
        const int me = 4 * s + 2 * (kl >> 1), mo = me + 1;
        ae[s] = (fok && me <= p) ? G[me * ms] : (TY)0;
        be[s] = (kok && me <= p) ? Tr[(long)2 * me * q] : (TY)0;
        ao[s] = (fok && mo <= p) ? G[mo * ms] : (TY)0;
        bo[s] = (kok && mo <= p) ? Tr[(long)2 * mo * q] : (TY)0;
    }
    typename Mma<TY>::acc E = {0, 0, 0, 0}, O = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < kXSteps; ++s) {
        if (4 * s > p) break;
        E = Mma<TY>::run(ae[s], be[s], E);
        O = Mma<TY>::run(ao[s], bo[s], O);
    }
    const int kc = kt * 16 + l16;
    if (kc >= q) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int f = ft * 16 + Mma<TY>::row(lane, v);
        if (f < b.nf) {
            double *o = b.grid + b.gb[f] + (long)j * 2 * q;
            o[kc] = (double)E[v] + (double)O[v];
            o[kc + q] = (double)E[v] - (double)O[v];
        }
    }
}

// Fourier stage of analysis. Wavefront: (8 orders of one parity x (re, im),
// 16 fields, latitude j, job); K runs over the longitudes k < q with the
// values folded as v_k + v_{k+q} (even orders) or v_k - v_{k+q} (odd).
template <typename TY>
__global__ __launch_bounds__(256) void k_xa_fourier(XJobs J)
{
    const XJob &b = J.j[blockIdx.z];
    const int p = b.p, q = b.q, nq = q + 1, NC = 2 * b.nf, j = blockIdx.y;
    const int rt0 = (p / 2 + 1 + 7) / 8, rt1 = ((p + 1) / 2 + 7) / 8;  // row tiles of the even / odd orders
    const int nft = (b.nf + 15) / 16;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= nq || tile >= (rt0 + rt1) * nft) return;
    const int rt = tile / nft, ft = tile % nft;
    const int par = rt < rt0 ? 0 : 1, mt = rt < rt0 ? rt : rt - rt0;
    const int lane = threadIdx.x & 63, kl = lane >> 4, l16 = lane & 15;
    const int ma = 2 * (mt * 8 + (l16 >> 1)) + par;  // A row: order, part l16 & 1
    const int fb = ft * 16 + l16;                     // B column: field
    const bool aok = ma <= p, bok = fb < b.nf;
    const TY *Tr = (const TY *)b.trig + (long)(2 * ma + (l16 & 1)) * q;
    const double *v = b.grid + (bok ? b.gb[fb] : 0) + (long)j * 2 * q;
    const double sg = par ? -1.0 : 1.0;
    TY av[kXSteps], bv[kXSteps];
#pragma unroll
    for (int s = 0; s < kXSteps; ++s) {
        const int k = 4 * s + kl;
        const bool kok = k < q;
        av[s] = (aok && kok) ? Tr[k] : (TY)0;
        bv[s] = (bok && kok) ? (TY)(v[k] + sg * v[k + q]) : (TY)0;
    }
    typename Mma<TY>::acc acc = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < kXSteps; ++s) {
        if (4 * s >= q) break;
        acc = Mma<TY>::run(av[s], bv[s], acc);
    }
    if (!bok) return;
    TY *G = (TY *)b.G;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = Mma<TY>::row(lane, e);
        const int m = 2 * (mt * 8 + (r >> 1)) + par;
        if (m <= p) G[((long)m * nq + j) * NC + 2 * fb + (r & 1)] = acc[e];
    }
}

// Legendre stage of analysis with the combine. Block: (64 columns, order m,
// job); rows n - m (up to kXRows), depth the q + 1 latitudes (up to
// kXDepth); the weighted table Ta[r][k] = (pi/q) w_k h_m Ptilde_{m+r}^m(t_k)
// staged in LDS.
template <typename TY>
__global__ __launch_bounds__(256) void k_xa_leg(XJobs J, const double *__restrict__ x, double *__restrict__ y,
                                                double sgn)
{
    __shared__ TY sT[kXRows * (kXDepth + 1)];
    const XJob &b = J.j[blockIdx.z];
    const int p = b.p, q = b.q, nq = q + 1, NC = 2 * b.nf, m = blockIdx.y;
    const int c0 = blockIdx.x * 64;
    if (m > p || c0 >= NC) return;
    const int R = p - m + 1, Kp = (nq + 3) & ~3, Ks = Kp + 1;
    const double h = m == q ? 0.5 : 1.0;
    const int lane = threadIdx.x & 63, kl = lane >> 4, l16 = lane & 15;
    const int col = c0 + (threadIdx.x >> 6) * 16 + l16;
    const bool cok = col < NC;
    const TY *G = (const TY *)b.G + (long)m * nq * NC + col;
    TY bv[kXSteps];
#pragma unroll
    for (int s = 0; s < kXSteps; ++s) {
        const int k = 4 * s + kl;
        bv[s] = (cok && k < nq) ? G[(long)k * NC] : (TY)0;
    }
    TY tv[kXRows * kXDepth / 256];
#pragma unroll
    for (int u = 0; u < kXRows * kXDepth / 256; ++u) {
        const int i = threadIdx.x + 256 * u, r = i / Kp, k = i % Kp;
        tv[u] = (i < kXRows * Kp && r < R && k < nq) ? (TY)(b.wq[k] * h * b.L[(long)k * b.ldn + tri(m + r, m)])
                                                     : (TY)0;
    }
#pragma unroll
    for (int u = 0; u < kXRows * kXDepth / 256; ++u) {
        const int i = threadIdx.x + 256 * u;
        if (i < kXRows * Kp) sT[(i / Kp) * Ks + i % Kp] = tv[u];
    }
    __syncthreads();
    const int nt = min(4, (R + 15) / 16);
    typename Mma<TY>::acc acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = (typename Mma<TY>::acc){0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < kXSteps; ++s) {
        if (4 * s >= Kp) break;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (t < nt) acc[t] = Mma<TY>::run(sT[(t * 16 + l16) * Ks + 4 * s + kl], bv[s], acc[t]);
    }
    if (!cok) return;
    const long cbase = b.cb[col];
    const double cs = b.csc ? b.csc[col >> 1] : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = t * 16 + Mma<TY>::row(lane, v);
            if (t < nt && r < R) {
                const long e = cbase + 2 * tri(m + r, m);
                y[e] = (b.csc ? cs * x[e] : 0.0) + sgn * (double)acc[t][v];
            }
        }
}

bool xform_fits(int p, int q, bool analysis)
{
    return p >= 0 && p < kXDepth && q >= p && q >= 1 && q <= 1024 && (!analysis || q + 1 <= kXDepth);
}

static XJobs xjobs(const XJob *jobs, int n)
{
    XJobs b{};
    b.n = n;
    for (int i = 0; i < n; ++i) b.j[i] = jobs[i];
    return b;
}

template <typename TY>
static void xsynth(hipStream_t st, const XJob *jobs, int n, const double *x, double *z0, long nz0, double *z1, long nz1)
{
    XJobs b = xjobs(jobs, n);
    b.zero[0] = nz0 > 0 ? z0 : nullptr;
    b.nzero[0] = nz0;
    b.zero[1] = nz1 > 0 ? z1 : nullptr;
    b.nzero[1] = nz1;
    int cblk = 1, mch = 1, tiles = 1, lat = 1;
    for (int i = 0; i < n; ++i) {
        const XJob &j = jobs[i];
        cblk = std::max(cblk, (2 * j.nf + 63) / 64);
        mch = std::max(mch, (j.p + 1) * ((j.q + 1 + kXRows - 1) / kXRows));
        tiles = std::max(tiles, ((j.q + 15) / 16) * ((j.nf + 15) / 16));
        lat = std::max(lat, j.q + 1);
    }
    hipLaunchKernelGGL(k_xs_leg<TY>, dim3(cblk, mch, n), dim3(256), 0, st, b, x);
    b.zero[0] = b.zero[1] = nullptr;
    hipLaunchKernelGGL(k_xs_fourier<TY>, dim3((tiles + 3) / 4, lat, n), dim3(256), 0, st, b);
}

template <typename TY>
static void xanal(hipStream_t st, const XJob *jobs, int n, const double *x, double *y, double sgn)
{
    const XJobs b = xjobs(jobs, n);
    int cblk = 1, m1 = 1, tiles = 1, lat = 1;
    for (int i = 0; i < n; ++i) {
        const XJob &j = jobs[i];
        cblk = std::max(cblk, (2 * j.nf + 63) / 64);
        m1 = std::max(m1, j.p + 1);
        tiles = std::max(tiles, ((j.p / 2 + 1 + 7) / 8 + ((j.p + 1) / 2 + 7) / 8) * ((j.nf + 15) / 16));
        lat = std::max(lat, j.q + 1);
    }
    hipLaunchKernelGGL(k_xa_fourier<TY>, dim3((tiles + 3) / 4, lat, n), dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_xa_leg<TY>, dim3(cblk, m1, n), dim3(256), 0, st, b, x, y, sgn);
}

// Synthesis of the jobs' value fields from the coefficient vector x (FP32
// operands when f32); the ranges z0[nz0], z1[nz1] are cleared by the launch.
void launch_xsynth(hipStream_t st, bool f32, const XJob *jobs, int n, const double *x, double *z0, long nz0,
                   double *z1, long nz1)
{
    for (int o = 0; o < n; o += kMaxXJobs) {
        const int k = std::min(kMaxXJobs, n - o);
        if (f32)
            xsynth<float>(st, jobs + o, k, x, o == 0 ? z0 : nullptr, o == 0 ? nz0 : 0, o == 0 ? z1 : nullptr,
                          o == 0 ? nz1 : 0);
        else
            xsynth<double>(st, jobs + o, k, x, o == 0 ? z0 : nullptr, o == 0 ? nz0 : 0, o == 0 ? z1 : nullptr,
                           o == 0 ? nz1 : 0);
    }
}

// Analysis of the jobs' grid fields into y = csc x + sgn c (no x term for a
// job without csc).
void launch_xanal(hipStream_t st, bool f32, const XJob *jobs, int n, const double *x, double *y, double sgn)
{
    for (int o = 0; o < n; o += kMaxXJobs) {
        const int k = std::min(kMaxXJobs, n - o);
        if (f32)
            xanal<float>(st, jobs + o, k, x, y, sgn);
        else
            xanal<double>(st, jobs + o, k, x, y, sgn);
    }
}

}  // namespace bim
