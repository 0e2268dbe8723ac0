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

}  // namespace bim
