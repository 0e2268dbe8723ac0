// gfx950 kernels of the Stokes layer-potential path (FP64).
//
// Data layouts (device):
//   coefficient triangle of a real field: (re, im) doubles at complex index
//     n(n+1)/2 + m, m >= 0;
//   Legendre tables of a degree-q grid: L[kind][j][tri(n, m)], kind 0 = Ptilde,
//     1 = d/dtheta, 2 = d^2/dtheta^2, j = 0..q (theta ascending);
//   grid values: [field][j * 2q + k];
//   cos/sin table of a degree-q grid: cs[i] = cos(pi i / q), cs[2q + i] = sin(pi i / q).
#include "internal.hpp"

#include <hip/hip_runtime.h>

#include <type_traits>

namespace bim {

static constexpr double kInvSqrt4Pi = 0.28209479177387814347;

// ----------------------------------------------------------------------------
// Analysis (Sec. 2.1, weight (pi/q) w_j, half weight at m = q):
// stage 1 (Fourier):  F[f][j][m] = sum_k v[f][j][k] e^{-i m phi_k}, m = 0..p
// stage 2 (Legendre): c_f[n,m] = sum_j wq_j h_m Ptilde_n^m(t_j) F[f][j][m]
// ----------------------------------------------------------------------------
__global__ void k_anal_fourier(int p, int q, const double *__restrict__ v, long vstride,
                               const double *__restrict__ cs, int nf, double *__restrict__ F)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nj = q + 1, nk = 2 * q;
    const long total = (long)nf * nj * (p + 1);
    if (idx >= total) return;
    const int m = idx % (p + 1);
    const long r = idx / (p + 1);
    const int j = r % nj;
    const int f = r / nj;
    const double *g = v + f * vstride + (long)j * nk;
    double sr = 0.0, si = 0.0;
    int e = 0;
    for (int k = 0; k < nk; ++k) {
        sr = fma(g[k], cs[e], sr);
        si = fma(-g[k], cs[nk + e], si);
        e += m;
        if (e >= nk) e -= nk;
    }
    F[2 * idx] = sr;
    F[2 * idx + 1] = si;
}

__global__ void k_anal_leg(int p, int q, int ldn, const double *__restrict__ L, const double *__restrict__ wq,
                           int nf, const double *__restrict__ F, double *__restrict__ coef, long cstride)
{
    const int nc = ncoef(p);
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)nf * nc;
    if (idx >= total) return;
    const int e = idx % nc;
    const int f = idx / nc;
    int n = (int)((sqrt(8.0 * e + 1.0) - 1.0) / 2.0);
    while (tri(n + 1, 0) <= e) ++n;
    while (tri(n, 0) > e) --n;
    const int m = e - tri(n, 0);
    const int nj = q + 1;
    const double h = (m == q) ? 0.5 : 1.0;
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < nj; ++j) {
        const double w = wq[j] * L[(long)j * ldn + e] * h;
        const double *Fj = F + 2 * ((long)(f * nj + j) * (p + 1) + m);
        sr = fma(w, Fj[0], sr);
        si = fma(w, Fj[1], si);
    }
    coef[f * cstride + 2 * e] = sr;
    coef[f * cstride + 2 * e + 1] = si;
}

// ----------------------------------------------------------------------------
// Geometry and interfacial force on the de-aliasing grid (Table 2 with the
// outward normal n = x_theta x x_phi / W and mean curvature
// K = -(E N - 2 F M + G L)/(2 W^2); Sec. 1 force f = 2 sigma K n - grad sigma).
// syn: 21 fields [x(3), xt(3), xp(3), xtt(3), xtp(3), xpp(3), Gam, Gam_t, Gam_p].
// ----------------------------------------------------------------------------
__global__ void k_force(int npt, const double *__restrict__ syn, int eos, double E, double xs, double sigma0,
                        double *__restrict__ f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npt) return;
    auto F = [&](int fld) { return syn[(long)fld * npt + i]; };
    const double at[3] = {F(3), F(4), F(5)};
    const double ap[3] = {F(6), F(7), F(8)};
    const double Em = ap[0] * ap[0] + ap[1] * ap[1] + ap[2] * ap[2];
    const double Fm = ap[0] * at[0] + ap[1] * at[1] + ap[2] * at[2];
    const double Gm = at[0] * at[0] + at[1] * at[1] + at[2] * at[2];
    const double W2 = Em * Gm - Fm * Fm;
    const double W = sqrt(W2);
    double n[3] = {at[1] * ap[2] - at[2] * ap[1], at[2] * ap[0] - at[0] * ap[2], at[0] * ap[1] - at[1] * ap[0]};
    n[0] /= W; n[1] /= W; n[2] /= W;
    const double Lm = F(15) * n[0] + F(16) * n[1] + F(17) * n[2];
    const double Mm = F(12) * n[0] + F(13) * n[1] + F(14) * n[2];
    const double Nm = F(9) * n[0] + F(10) * n[1] + F(11) * n[2];
    const double K = -(Em * Nm - 2.0 * Fm * Mm + Gm * Lm) / (2.0 * W2);
    double sig, ds;
    if (eos == 0) { sig = sigma0; ds = 0.0; }
    else if (eos == 1) { sig = 1.0 - E * xs * F(18); ds = -E * xs; }
    else { const double g = 1.0 - xs * F(18); sig = 1.0 + E * log(g); ds = -E * xs / g; }
    const double st = ds * F(19), sp = ds * F(20);
    const double cpn = (Gm * sp - Fm * st) / W2, ctn = (Em * st - Fm * sp) / W2;
    for (int c = 0; c < 3; ++c) f[(long)c * npt + i] = 2.0 * sig * K * n[c] - (cpn * ap[c] + ctn * at[c]);
}

// ----------------------------------------------------------------------------
// Quadrature nodes of drop grids (one job per drop and grid, all in one
// launch) on a degree-q grid: positions, the weighted
// non-normalized normal wN = w_j (x_theta x x_phi), the weighted area element
// wW = w_j |x_theta x x_phi|, w_j = (pi/q) w_j^G / sin theta_j (Sec. 2.1).
// The enclosed volume (1/3) sum wN . x of the job's grid goes to vol as one
// partial sum per wavefront, vol[i / 64] for the wavefront of node i (vol may
// be null); k_vol_sum adds them in order.
// syn: 9 fields [x(3), xt(3), xp(3)], npt = 2q(q+1).
// ----------------------------------------------------------------------------
// Jobs of one launch (blockIdx.y = job): the grids of all drops at once.
__global__ void k_nodes(NodeJobs jobs)
{
    const NodeJob &J = jobs.j[blockIdx.y];
    const int q = J.q;
    const int npt = npts(q);
    if ((int)(blockIdx.x * blockDim.x) >= npt) return;  // the whole block is past this grid
    const double *__restrict__ syn = J.syn;
    double *__restrict__ sx = J.sx;
    double *__restrict__ swN = J.swN;
    const long sstride = J.sstride;
    double *vol = J.vol;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double contrib = 0.0;
    if (i < npt) {
        auto F = [&](int fld) { return syn[(long)fld * npt + i]; };
        const double w = J.wreg[i / (2 * q)];
        const double at[3] = {F(3), F(4), F(5)};
        const double ap[3] = {F(6), F(7), F(8)};
        const double N[3] = {at[1] * ap[2] - at[2] * ap[1], at[2] * ap[0] - at[0] * ap[2], at[0] * ap[1] - at[1] * ap[0]};
        for (int c = 0; c < 3; ++c) {
            sx[c * sstride + i] = F(c);
            swN[c * sstride + i] = w * N[c];
        }
        J.swW[i] = w * sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        contrib = w * (N[0] * F(0) + N[1] * F(1) + N[2] * F(2)) / 3.0;
    }
    if (vol) {
        // wavefront reduction, one partial per wavefront (fixed order)
        for (int o = 32; o > 0; o >>= 1) contrib += __shfl_down(contrib, o, 64);
        const int w0 = blockIdx.x * blockDim.x + (threadIdx.x & ~63);
        if ((threadIdx.x & 63) == 0 && w0 < npt) vol[w0 >> 6] = contrib;
    }
}

// ----------------------------------------------------------------------------
// Region split (Sec. 2.3): for every target t and source drop j != drop(t),
// the distance to the nearest node of j's degree-p grid, compared with
// A_tilde h_j and h_j. reg[t * nd + j] = 0 / 1 / 2, -1 for the own drop.
// Pass 1 (thread per pair): the bounds |x0 - c_j| -/+ b_j of the nearest-node
// distance (b_j = the largest node distance from the drop's centre c_j) decide
// pairs whose region they already fix; the others go to a list. Pass 2 (wavefront per
// listed pair): the nearest-node distance and the region.
// ----------------------------------------------------------------------------
__global__ void k_classify_bound(int T, int nd, const double *__restrict__ tx, long tstride,
                                 const int *__restrict__ tdrop, const int *__restrict__ sys,
                                 const double *__restrict__ cb /*[nd][4]*/, const double *__restrict__ hj, double A,
                                 int exact, int8_t *__restrict__ reg, double *__restrict__ dist,
                                 int *__restrict__ list, int *__restrict__ count)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)T * nd) return;
    const int j = idx % nd;
    const int t = idx / nd;
    if (tdrop[t] == j) {
        reg[idx] = -1;
        if (dist) dist[idx] = 0.0;
        return;
    }
    if (sys[tdrop[t]] != sys[j]) {  // drops of independent systems do not interact
        reg[idx] = -2;
        if (dist) dist[idx] = 0.0;
        return;
    }
    bool scan = exact != 0;
    if (!scan) {
        const double dx = tx[t] - cb[4 * j], dy = tx[tstride + t] - cb[4 * j + 1], dz = tx[2 * tstride + t] - cb[4 * j + 2];
        const double dc = sqrt(dx * dx + dy * dy + dz * dz);
        const double lb = dc - cb[4 * j + 3], ub = dc + cb[4 * j + 3];  // bounds of the nearest-node distance
        const double h = hj[j];
        if (lb > A * h) {
            reg[idx] = 0;
            if (dist) dist[idx] = lb;
        } else if (lb > h && ub <= A * h) {
            reg[idx] = 1;
            if (dist) dist[idx] = lb;
        } else {
            scan = true;
        }
    }
    if (scan) list[atomicAdd(count, 1)] = (int)idx;
}

// One list item (target t, drop j) = idx = t nd + j, on one wavefront: the
// distance from the target to the nearest node of drop j and its region.
__device__ inline void classify_scan_item(int idx, int nd, const double *__restrict__ tx, long tstride,
                                          const double *__restrict__ sx, long sstride,
                                          const int *__restrict__ noff, const int *__restrict__ ncnt,
                                          const double *__restrict__ hj, double A, int8_t *__restrict__ reg,
                                          double *__restrict__ dist)
{
    const int lane = threadIdx.x & 63;
    const int j = idx % nd;
    const int t = idx / nd;
    const double x0 = tx[t], y0 = tx[tstride + t], z0 = tx[2 * tstride + t];
    double best = 1e300;
    const int o = noff[j], c = ncnt[j];
    for (int s = lane; s < c; s += 64) {
        const double dx = x0 - sx[o + s], dy = y0 - sx[sstride + o + s], dz = z0 - sx[2 * sstride + o + s];
        best = fmin(best, dx * dx + dy * dy + dz * dz);
    }
    for (int off = 32; off > 0; off >>= 1) best = fmin(best, __shfl_down(best, off, 64));
    if (lane == 0) {
        const double d = sqrt(best);
        const double h = hj[j];
        reg[idx] = (d > A * h) ? 0 : (d > h ? 1 : 2);
        if (dist) dist[idx] = d;
    }
}

__global__ __launch_bounds__(256) void k_classify_scan(const int *__restrict__ count, const int *__restrict__ list,
                                                       int nd, const double *__restrict__ tx, long tstride,
                                                       const double *__restrict__ sx, long sstride,
                                                       const int *__restrict__ noff, const int *__restrict__ ncnt,
                                                       const double *__restrict__ hj, double A,
                                                       int8_t *__restrict__ reg, double *__restrict__ dist)
{
    // the list length is read on the device (written by k_classify_bound), so
    // the host need not wait for it; wavefronts stride over the list
    const int n = count[0];
    const int nw = (gridDim.x * blockDim.x) >> 6;
    for (int wv = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; wv < n; wv += nw)
        classify_scan_item(list[wv], nd, tx, tstride, sx, sstride, noff, ncnt, hj, A, reg, dist);
}

// Centre (mean node position) and bounding radius of each drop's standard nodes.
__global__ __launch_bounds__(256) void k_drop_bounds(int nd, const double *__restrict__ sx, long sstride,
                                                     const int *__restrict__ noff, const int *__restrict__ ncnt,
                                                     double *__restrict__ cb)
{
    __shared__ double red[4][4];
    const int j = blockIdx.x;
    const int o = noff[j], c = ncnt[j];
    double s[3] = {0, 0, 0};
    for (int i = threadIdx.x; i < c; i += 256)
        for (int k = 0; k < 3; ++k) s[k] += sx[k * sstride + o + i];
    for (int k = 0; k < 3; ++k) {
        for (int off = 32; off > 0; off >>= 1) s[k] += __shfl_down(s[k], off, 64);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = s[k];
    }
    __syncthreads();
    double cen[3];
    for (int k = 0; k < 3; ++k) cen[k] = (red[k][0] + red[k][1] + red[k][2] + red[k][3]) / c;
    double m = 0.0;
    for (int i = threadIdx.x; i < c; i += 256) {
        const double dx = sx[o + i] - cen[0], dy = sx[sstride + o + i] - cen[1], dz = sx[2 * sstride + o + i] - cen[2];
        m = fmax(m, dx * dx + dy * dy + dz * dz);
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[3][threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double mm = fmax(fmax(red[3][0], red[3][1]), fmax(red[3][2], red[3][3]));
        cb[4 * j] = cen[0];
        cb[4 * j + 1] = cen[1];
        cb[4 * j + 2] = cen[2];
        // bounding radius, enlarged by a relative 1e-12 so the bound stays rigorous under rounding
        cb[4 * j + 3] = sqrt(mm) * (1.0 + 1e-12) + 1e-300;
    }
}

// ----------------------------------------------------------------------------
// Rotation of the expansion so that each grid target of a drop is at the
// north pole (Appendix B with gamma = 0):
//   Re f'^mu_n = sum_nu A+_{nu mu}(theta_j) Re(e^{i nu phi_k} f_n^nu)
//   Im f'^mu_n = sum_nu A-_{nu mu}(theta_j) Im(e^{i nu phi_k} f_n^nu)
// R[t][field][tri(n,mu)] complex for fields 0..2 (x) and 3..5 (density).
// ----------------------------------------------------------------------------
__global__ void k_rotate(int p, int nt, const double *__restrict__ Ap, const double *__restrict__ Am,
                         const double *__restrict__ cs, const double *__restrict__ xc, long xstride,
                         const double *__restrict__ dc, long dstride, double *__restrict__ R)
{
    const int nc = ncoef(p);
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nt * 6 * nc) return;
    const int e = idx % nc;
    const long r = idx / nc;
    const int f = r % 6;
    const int t = r / 6;
    int n = (int)((sqrt(8.0 * e + 1.0) - 1.0) / 2.0);
    while (tri(n + 1, 0) <= e) ++n;
    while (tri(n, 0) > e) --n;
    const int mu = e - tri(n, 0);
    const int j = t / (2 * p), k = t % (2 * p);
    const int nk = 2 * p;
    const double *c = (f < 3) ? xc + f * xstride : dc + (f - 3) * dstride;
    const size_t base = rot_lat_size(p) * j + rot_off(n);
    const double *ap = Ap + base, *am = Am + base;
    double re = 0.0, im = 0.0;
    int ph = 0;
    for (int nu = 0; nu <= n; ++nu) {
        const double cr = c[2 * tri(n, nu)], ci = c[2 * tri(n, nu) + 1];
        const double cc = cs[ph], ss = cs[nk + ph];
        re = fma(ap[nu * (n + 1) + mu], cr * cc - ci * ss, re);
        im = fma(am[nu * (n + 1) + mu], cr * ss + ci * cc, im);
        ph += k;
        if (ph >= nk) ph -= nk;
    }
    R[2 * idx] = re;
    R[2 * idx + 1] = im;
}

// ----------------------------------------------------------------------------
// Singular self-integral (Sec. 2.2, Theorem 1) at every grid target of one
// drop, one workgroup per target. On the degree-qs rotated grid:
//   Q = sum_{j',k'} omega_{j'} K(x0, x'_{j'k'}) rho'_{j'k'} W'_{j'k'},
//   omega_{j'} = (pi/qs) w^G_{j'} [sum_{n<=qs} P_n(t_{j'})] 2 sin(theta_{j'}/2) / sin(theta_{j'}),
// K the Stokeslet (kind 0, density f) or the stresslet (kind 1, density u).
// Stage A: Legendre sums G = sum_n C^mu_n L_n^mu(t_{j'}) for JB latitudes into LDS
// (9 sums: x, dx/dtheta, density); stage B: Fourier sums at k' and k'+qs
// (even/odd orders) and the kernel, accumulated per thread; then a block reduction.
// ----------------------------------------------------------------------------
template <int JB>
__global__ __launch_bounds__(256) void k_singular(int p, int qs, int kind, const double *__restrict__ R,
                                                  const double *__restrict__ Ls, int ldn,
                                                  const double *__restrict__ wsing,
                                                  const double *__restrict__ cs, double *__restrict__ out,
                                                  long ostride, double scale)
{
    extern __shared__ double G[];  // [JB][9][p+1][2]
    __shared__ double x0s[3];
    __shared__ double red[3][4];
    const int t = blockIdx.x;
    const int nc = ncoef(p);
    const int nk = 2 * qs;
    const double *Rt = R + (long)t * 6 * nc * 2;
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int n = 0; n <= p; ++n) s += Rt[2 * (threadIdx.x * nc + tri(n, 0))] * sqrt(2.0 * n + 1.0) * kInvSqrt4Pi;
        x0s[threadIdx.x] = s;
    }
    __syncthreads();
    const double x0 = x0s[0], y0 = x0s[1], z0 = x0s[2];
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    const int P1 = p + 1;
    for (int jb0 = 0; jb0 <= qs; jb0 += JB) {
        const int nb = min(JB, qs + 1 - jb0);
        // stage A
        for (int idx = threadIdx.x; idx < 9 * P1; idx += blockDim.x) {
            const int type = idx / P1, mu = idx % P1;
            const int field = (type < 6) ? type % 3 : type - 3;
            const int kl = (type >= 3 && type < 6) ? 1 : 0;
            const double *C = Rt + 2 * field * nc;
            double sr[JB], si[JB];
#pragma unroll
            for (int b = 0; b < JB; ++b) { sr[b] = 0.0; si[b] = 0.0; }
            const double *Lb = Ls + ((long)kl * (qs + 1) + jb0) * ldn;
            for (int n = mu; n <= p; ++n) {
                const double cr = C[2 * tri(n, mu)], ci = C[2 * tri(n, mu) + 1];
#pragma unroll
                for (int b = 0; b < JB; ++b) {
                    if (b < nb) {
                        const double l = Lb[(long)b * ldn + tri(n, mu)];
                        sr[b] = fma(cr, l, sr[b]);
                        si[b] = fma(ci, l, si[b]);
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < JB; ++b)
                if (b < nb) {
                    G[2 * ((b * 9 + type) * P1 + mu)] = sr[b];
                    G[2 * ((b * 9 + type) * P1 + mu) + 1] = si[b];
                }
        }
        __syncthreads();
        // stage B
        for (int idx = threadIdx.x; idx < nb * qs; idx += blockDim.x) {
            const int b = idx / qs, kp = idx % qs;
            const double *Gb = G + 2 * b * 9 * P1;
            double ev[12], od[12];
#pragma unroll
            for (int i = 0; i < 12; ++i) { ev[i] = 0.0; od[i] = 0.0; }
            int e = 0;
            for (int mu = 0; mu <= p; ++mu) {
                const double c = cs[e], s = cs[nk + e];
                const double wm = mu ? 2.0 : 1.0;
                double v[12];
#pragma unroll
                for (int ty = 0; ty < 9; ++ty) {
                    const double gr = Gb[2 * (ty * P1 + mu)], gi = Gb[2 * (ty * P1 + mu) + 1];
                    v[ty] = wm * (gr * c - gi * s);
                }
#pragma unroll
                for (int c3 = 0; c3 < 3; ++c3) {
                    const double gr = Gb[2 * (c3 * P1 + mu)], gi = Gb[2 * (c3 * P1 + mu) + 1];
                    v[9 + c3] = -wm * mu * (gi * c + gr * s);
                }
                if (mu & 1) {
#pragma unroll
                    for (int i = 0; i < 12; ++i) od[i] += v[i];
                } else {
#pragma unroll
                    for (int i = 0; i < 12; ++i) ev[i] += v[i];
                }
                e += kp;
                if (e >= nk) e -= nk;
            }
            const double om = wsing[jb0 + b];
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const double sg = side ? -1.0 : 1.0;
                double v[12];
#pragma unroll
                for (int i = 0; i < 12; ++i) v[i] = ev[i] + sg * od[i];
                // v: x(0..2), x_theta(3..5), density(6..8), x_phi(9..11)
                const double Nx = v[4] * v[11] - v[5] * v[10];
                const double Ny = v[5] * v[9] - v[3] * v[11];
                const double Nz = v[3] * v[10] - v[4] * v[9];
                const double hx = x0 - v[0], hy = y0 - v[1], hz = z0 - v[2];
                const double r2 = hx * hx + hy * hy + hz * hz;
                const double rinv = 1.0 / sqrt(r2);
                const double hd = hx * v[6] + hy * v[7] + hz * v[8];
                if (kind == 0) {
                    const double Wd = om * sqrt(Nx * Nx + Ny * Ny + Nz * Nz) * rinv;
                    const double r2i = rinv * rinv;
                    acc0 += Wd * (v[6] + hx * hd * r2i);
                    acc1 += Wd * (v[7] + hy * hd * r2i);
                    acc2 += Wd * (v[8] + hz * hd * r2i);
                } else {
                    const double hn = hx * Nx + hy * Ny + hz * Nz;
                    const double r5i = rinv * rinv * rinv * rinv * rinv;
                    const double s = -6.0 * om * hd * hn * r5i;
                    acc0 += s * hx;
                    acc1 += s * hy;
                    acc2 += s * hz;
                }
            }
        }
        __syncthreads();
    }
    // block reduction (256 threads = 4 wavefronts)
    for (int o = 32; o > 0; o >>= 1) {
        acc0 += __shfl_down(acc0, o, 64);
        acc1 += __shfl_down(acc1, o, 64);
        acc2 += __shfl_down(acc2, o, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[0][wv] = acc0; red[1][wv] = acc1; red[2][wv] = acc2; }
    __syncthreads();
    if (threadIdx.x < 3) {
        const double s = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
        out[threadIdx.x * ostride + t] += scale * s;
    }
}

// ----------------------------------------------------------------------------
// Pair sums (Sec. 1 kernels by the regular rule of Sec. 2.1 on the standard
// or upsampled grid of a source drop, Sec. 2.3).
//   kind 0 (SL): sum wW G(x0, x) f = sum wW (f / r + h (h.f) / r^3);
//   kind 1 (DL): sum -6 h (h.u)(h.wN) / r^5,   h = x0 - x.
// One wavefront per work item: up to 64 T targets, T per lane, against a run
// of sources of one grid. The sources are the same for every lane, so they
// are read through the scalar data path (constant address space: SGPR
// operands of the VALU instructions) and each one feeds T pairs per lane,
// with no LDS staging and no barriers. Item i of a launch writes w * sum for
// each of its target slots into its own block of the partial buffer,
// part[(item0 + i) * 3 * tile + c * tile + slot]; k_pair_gather then adds the
// slots of each target in a fixed order, so the sums do not depend on
// scheduling. Items of whole tiles run with T = the tile's targets per lane,
// the remainder items of a target set (flag kPairSmall) with T = 1, in the
// same launch.
// ----------------------------------------------------------------------------
constexpr int kPairWaves = 4;  // wavefronts (independent items) per block

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) double cdouble;
typedef const __attribute__((address_space(4))) f32x4 cf32x4;
__device__ inline cdouble *scalar_ptr(const double *p) { return (cdouble *)p; }
__device__ inline cf32x4 *scalar_ptr(const float4 *p) { return (cf32x4 *)p; }

// Target a of an item, clamped to the item's last target (surplus lanes
// evaluate a duplicate and their slot is never read).
__device__ inline int pair_target(const PairWork &w, const int *__restrict__ tlist, int a)
{
    a = a < w.ntgt ? a : w.ntgt - 1;
    return (w.pad & kPairContig) ? w.tlist_off + a : tlist[w.tlist_off + a];
}

// One pair of the sums above (FP64): adds target (X, Y, Z)'s term of the
// source (px, py, pz, u, m) to (A0, A1, A2). u = wW f (SL) or the density,
// m = wN (DL).
template <int KIND>
__device__ inline void pair64(double X, double Y, double Z, double px, double py, double pz, double u0, double u1,
                              double u2, double m0, double m1, double m2, double &A0, double &A1, double &A2)
{
    const double hx = X - px, hy = Y - py, hz = Z - pz;
    const double r2 = fma(hz, hz, fma(hy, hy, hx * hx));
    // y = the hardware reciprocal square root of r2 (r2 > 0 for every pair of
    // distinct drops; overlapping drops are rejected at input), relative error
    // d below 5.3e-8 (measured over twelve decades), refined to the accuracy
    // of the sums (1e-10 and below) by the first-order correction of the
    // power the kernel needs: with e = r2 y^2 - 1 = 2 d + d^2,
    //   r^-1 = y (1 + e)^(-1/2) ~ y (1 - e/2)          (SL; one Newton step),
    //   r^-5 = y^5 (1 + e)^(-5/2) ~ y^5 (1 - 5 e / 2)  (DL),
    // leaving relative errors of 3/8 e^2 and 35/8 e^2 (below 5e-14): 4 and 6
    // FP64 instructions on top of the estimate.
    const double y = __builtin_amdgcn_rsq(r2);
    const double hd = fma(hz, u2, fma(hy, u1, hx * u0));
    if (KIND == 0) {
        const double e = fma(-r2 * y, y, 1.0);
        const double ri = fma(y * e, 0.5, y);
        const double q = hd * ri * ri;
        A0 = fma(ri, fma(hx, q, u0), A0);
        A1 = fma(ri, fma(hy, q, u1), A1);
        A2 = fma(ri, fma(hz, q, u2), A2);
    } else {
        const double hn = fma(hz, m2, fma(hy, m1, hx * m0));
        const double z = y * y;
        const double e = fma(r2, z, -1.0);
        const double y5 = z * z * y;
        const double sc = (hd * hn) * fma(y5 * -2.5, e, y5);
        A0 = fma(sc, hx, A0);
        A1 = fma(sc, hy, A1);
        A2 = fma(sc, hz, A2);
    }
}

// One item of the FP64 sums with T targets per lane and U independent
// accumulators per target: consecutive sources alternate between them
// (independent work for one lane when T is small), added in a fixed order at
// the end. With one target per lane the kernel takes 8 (its 8 steps of 9
// source values overflow the scalar registers into vector lanes, and it is
// still the faster of 4 and 8 on the two-drop workload it serves).
template <int KIND, int T, int U>
__device__ inline void pair_item64(const PairWork &w, int item, int tile, const int *__restrict__ tlist,
                                   const double *__restrict__ tx, long tstride, const PairSrc &g0,
                                   const PairSrc &g1, double *__restrict__ part)
{
    const int lane = threadIdx.x & 63;
    double X[T], Y[T], Z[T], A0[T][U], A1[T][U], A2[T][U];
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int t = pair_target(w, tlist, lane + 64 * k);
        X[k] = tx[t];
        Y[k] = tx[tstride + t];
        Z[k] = tx[2 * tstride + t];
#pragma unroll
        for (int v = 0; v < U; ++v) A0[k][v] = A1[k][v] = A2[k][v] = 0.0;
    }
    const PairSrc &G = (w.pad & 1) ? g1 : g0;
    const long st = G.stride, o = w.src_off;
    cdouble *sx = scalar_ptr(G.x + o), *sy = scalar_ptr(G.x + st + o), *sz = scalar_ptr(G.x + 2 * st + o);
    cdouble *d0 = scalar_ptr(G.d + o), *d1 = scalar_ptr(G.d + st + o), *d2 = scalar_ptr(G.d + 2 * st + o);
    cdouble *n0 = scalar_ptr((KIND == 0 ? G.wW : G.wN) + o), *n1 = scalar_ptr(G.wN + st + o),
            *n2 = scalar_ptr(G.wN + 2 * st + o);
    auto step = [&](int s, int v) {
        const double px = sx[s], py = sy[s], pz = sz[s];
        double u0 = d0[s], u1 = d1[s], u2 = d2[s], m0 = 0.0, m1 = 0.0, m2 = 0.0;
        if (KIND == 0) {
            const double ww = n0[s];
            u0 *= ww;
            u1 *= ww;
            u2 *= ww;
        } else {
            m0 = n0[s];
            m1 = n1[s];
            m2 = n2[s];
        }
#pragma unroll
        for (int k = 0; k < T; ++k)
            pair64<KIND>(X[k], Y[k], Z[k], px, py, pz, u0, u1, u2, m0, m1, m2, A0[k][v], A1[k][v], A2[k][v]);
    };
    int s = 0;
    if (U == 1) {
#pragma unroll 2
        for (; s < w.nsrc; ++s) step(s, 0);
    } else {
        for (; s + U <= w.nsrc; s += U)
#pragma unroll
            for (int v = 0; v < U; ++v) step(s + v, v);
        for (; s < w.nsrc; ++s) step(s, 0);
    }
    const double sw = KIND == 0 ? w.w : -6.0 * w.w;
    double *out = part + (long)item * (3 * tile) + lane;
#pragma unroll
    for (int k = 0; k < T; ++k) {
#pragma unroll
        for (int v = 1; v < U; ++v) {
            A0[k][0] += A0[k][v];
            A1[k][0] += A1[k][v];
            A2[k][0] += A2[k][v];
        }
        out[64 * k] = sw * A0[k][0];
        out[tile + 64 * k] = sw * A1[k][0];
        out[2 * tile + 64 * k] = sw * A2[k][0];
    }
}

// Items [0, nwork) of a work list: whole tiles (ntgt <= 64 T; a ragged last
// tile of a target set repeats its last target in the surplus slots) with T
// targets per lane, remainder items (flag kPairSmall, at most 64 targets)
// with one. The item index is uniform over the wavefront, so the branch is.
template <int KIND, int T>
__global__ __launch_bounds__(64 * kPairWaves) __attribute__((amdgpu_waves_per_eu(T == 1 ? 1 : 6, 8))) void k_pair(const PairWork *__restrict__ work, int nwork, int item0,
                                                         int tile, const int *__restrict__ tlist,
                                                         const double *__restrict__ tx, long tstride, PairSrc g0,
                                                         PairSrc g1, double *__restrict__ part)
{
    const int item = __builtin_amdgcn_readfirstlane(blockIdx.x * kPairWaves + (threadIdx.x >> 6));
    if (item >= nwork) return;
    const PairWork w = work[item];
    if (T > 1 && (w.pad & kPairSmall))
        pair_item64<KIND, 1, (T >= 4 ? 2 : 4)>(w, item0 + item, tile, tlist, tx, tstride, g0, g1, part);
    else
        pair_item64<KIND, T, (T >= 4 ? 1 : 8 / T)>(w, item0 + item, tile, tlist, tx, tstride, g0, g1, part);
}

// FP32 source records of the mixed form, three float4 per node at the node's
// index: position relative to its drop's centre (mean node) and the density
// terms,
//   DL (x, y, z, u0) (u1, u2, wN0, wN1) (wN2, -, -, -)
//   SL (x, y, z, wW f0) (wW f1, wW f2, -, -) (-)
// Job b covers nodes [off, off + n) of drop `drop`.
template <int KIND>
__global__ void k_pair_pack32(const PackJob *__restrict__ jobs, PairSrc G, const double *__restrict__ cb,
                              float4 *__restrict__ rec)
{
    const PackJob jb = jobs[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= jb.n) return;
    const long s = jb.off + i, st = G.stride;
    const double *c = cb + 4 * jb.drop;
    const float px = (float)(G.x[s] - c[0]), py = (float)(G.x[st + s] - c[1]), pz = (float)(G.x[2 * st + s] - c[2]);
    float4 *r = rec + 3 * s;
    if (KIND == 0) {
        const double ww = G.wW[s];
        r[0] = make_float4(px, py, pz, (float)(ww * G.d[s]));
        r[1] = make_float4((float)(ww * G.d[st + s]), (float)(ww * G.d[2 * st + s]), 0.f, 0.f);
    } else {
        r[0] = make_float4(px, py, pz, (float)G.d[s]);
        r[1] = make_float4((float)G.d[st + s], (float)G.d[2 * st + s], (float)G.wN[s], (float)G.wN[st + s]);
        r[2] = make_float4((float)G.wN[2 * st + s], 0.f, 0.f, 0.f);
    }
}

// The same pair sums in FP32 arithmetic (precision BIM_PREC_MIXED) from the
// packed records: targets are taken relative to the source drop's centre in
// FP64 and rounded to FP32, so the differences h keep FP32 relative accuracy
// for every distance; 1/r from the single-precision reciprocal square root
// (about 1 ulp); runs of kPairRun sources are summed in FP32 and added into
// FP64 accumulators.
constexpr int kPairRun = 16;

template <int KIND, int T>
__device__ inline void pair_item32(const PairWork &w, int item, int tile, const int *__restrict__ tlist,
                                   const double *__restrict__ tx, long tstride, const float4 *__restrict__ rec0,
                                   const float4 *__restrict__ rec1, const double *__restrict__ cb, int nd,
                                   double *__restrict__ part)
{
    const int lane = threadIdx.x & 63;
    const double *c = cb + 4 * (w.pair % nd);
    const double c0 = c[0], c1 = c[1], c2 = c[2];
    float X[T], Y[T], Z[T];
    double A0[T], A1[T], A2[T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int t = pair_target(w, tlist, lane + 64 * k);
        X[k] = (float)(tx[t] - c0);
        Y[k] = (float)(tx[tstride + t] - c1);
        Z[k] = (float)(tx[2 * tstride + t] - c2);
        A0[k] = A1[k] = A2[k] = 0.0;
    }
    cf32x4 *r = scalar_ptr(((w.pad & 1) ? rec1 : rec0) + 3L * w.src_off);
    for (int r0 = 0; r0 < w.nsrc; r0 += kPairRun) {
        const int r1 = min(w.nsrc, r0 + kPairRun);
        float B0[T], B1[T], B2[T];
#pragma unroll
        for (int k = 0; k < T; ++k) B0[k] = B1[k] = B2[k] = 0.f;
#pragma unroll 2
        for (int s = r0; s < r1; ++s) {
            const f32x4 p0 = r[3 * s], p1 = r[3 * s + 1];
            f32x4 p2 = p1;
            if (KIND == 1) p2 = r[3 * s + 2];
#pragma unroll
            for (int k = 0; k < T; ++k) {
                const float hx = X[k] - p0.x, hy = Y[k] - p0.y, hz = Z[k] - p0.z;
                const float r2 = fmaf(hz, hz, fmaf(hy, hy, hx * hx));
                const float ri = __builtin_amdgcn_rsqf(r2);
                const float hd = fmaf(hz, p1.y, fmaf(hy, p1.x, hx * p0.w));
                if (KIND == 0) {
                    const float q = hd * ri * ri;
                    B0[k] = fmaf(ri, fmaf(hx, q, p0.w), B0[k]);
                    B1[k] = fmaf(ri, fmaf(hy, q, p1.x), B1[k]);
                    B2[k] = fmaf(ri, fmaf(hz, q, p1.y), B2[k]);
                } else {
                    const float hn = fmaf(hz, p2.x, fmaf(hy, p1.w, hx * p1.z));
                    const float r2i = ri * ri;
                    const float sc = (hd * hn) * (r2i * r2i * ri);
                    B0[k] = fmaf(sc, hx, B0[k]);
                    B1[k] = fmaf(sc, hy, B1[k]);
                    B2[k] = fmaf(sc, hz, B2[k]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < T; ++k) {
            A0[k] += (double)B0[k];
            A1[k] += (double)B1[k];
            A2[k] += (double)B2[k];
        }
    }
    const double sw = KIND == 0 ? w.w : -6.0 * w.w;
    double *out = part + (long)item * (3 * tile) + lane;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        out[64 * k] = sw * A0[k];
        out[tile + 64 * k] = sw * A1[k];
        out[2 * tile + 64 * k] = sw * A2[k];
    }
}

// Items of a work list as k_pair takes them (remainder items with one target
// per lane), the sums of the FP32 records.
template <int KIND, int T>
__global__ __launch_bounds__(64 * kPairWaves) void k_pair32(const PairWork *__restrict__ work, int nwork, int item0,
                                                           int tile, const int *__restrict__ tlist,
                                                           const double *__restrict__ tx, long tstride,
                                                           const float4 *__restrict__ rec0,
                                                           const float4 *__restrict__ rec1,
                                                           const double *__restrict__ cb, int nd,
                                                           double *__restrict__ part)
{
    const int item = __builtin_amdgcn_readfirstlane(blockIdx.x * kPairWaves + (threadIdx.x >> 6));
    if (item >= nwork) return;
    const PairWork w = work[item];
    if (T > 1 && (w.pad & kPairSmall))
        pair_item32<KIND, 1>(w, item0 + item, tile, tlist, tx, tstride, rec0, rec1, cb, nd, part);
    else
        pair_item32<KIND, T>(w, item0 + item, tile, tlist, tx, tstride, rec0, rec1, cb, nd, part);
}

// out[c][t] (+)= the pair sums of target t from the partial buffer, added in
// a fixed order, so the result does not depend on scheduling. Items over a
// contiguous tile of targets are listed once per tile: the slots of target t
// are tent[e] + t for e in [toff[k], toff[k+1]), k = tile_of[t] (tile_of may
// be null: no such items). Items over an index list are listed per target:
// slots ent[e], e in [off[t], off[t+1]). Each slot holds three components at
// stride `tile`. One wavefront per target: lane l adds the entries l, l + 64,
// ... of the two lists in turn, then a butterfly over the lanes. Targets
// with no slot are left alone.
__global__ __launch_bounds__(256) void k_pair_gather(int nt, int tile, const int *__restrict__ tile_of,
                                                     const int *__restrict__ toff, const int *__restrict__ tent,
                                                     const int *__restrict__ off, const int *__restrict__ ent,
                                                     const double *__restrict__ part, double *__restrict__ out,
                                                     long ostride, int add)
{
    const int t = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (t >= nt) return;
    int k0 = 0, k1 = 0;
    if (tile_of) {
        const int k = tile_of[t];
        k0 = toff[k];
        k1 = toff[k + 1];
    }
    const int e0 = off[t], e1 = off[t + 1];
    if (k0 == k1 && e0 == e1) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int e = k0 + lane; e < k1; e += 64) {
        const double *p = part + ((long)tent[e] + t);
        s0 += p[0];
        s1 += p[tile];
        s2 += p[2 * tile];
    }
    for (int e = e0 + lane; e < e1; e += 64) {
        const double *p = part + (long)ent[e];
        s0 += p[0];
        s1 += p[tile];
        s2 += p[2 * tile];
    }
    for (int o = 32; o > 0; o >>= 1) {
        s0 += __shfl_xor(s0, o, 64);
        s1 += __shfl_xor(s1, o, 64);
        s2 += __shfl_xor(s2, o, 64);
    }
    if (lane == 0) {
        if (add) {
            s0 += out[t];
            s1 += out[ostride + t];
            s2 += out[2 * ostride + t];
        }
        out[t] = s0;
        out[ostride + t] = s1;
        out[2 * ostride + t] = s2;
    }
}

// ----------------------------------------------------------------------------
// Pointwise combinations and GMRES vector kernels (FP64).
// ----------------------------------------------------------------------------
// b = 2 (U0 + gradU x) + a * s, over T targets (component-major)
__global__ void k_rhs(int T, const double *__restrict__ tx, long tstride, const double *__restrict__ s, double a,
                      double U00, double U01, double U02, const double *__restrict__ gU, double *__restrict__ b)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const double x = tx[t], y = tx[tstride + t], z = tx[2 * tstride + t];
    const double U0[3] = {U00, U01, U02};
    for (int c = 0; c < 3; ++c) {
        const double ui = U0[c] + gU[3 * c] * x + gU[3 * c + 1] * y + gU[3 * c + 2] * z;
        b[c * tstride + t] = 2.0 * ui + a * s[c * tstride + t];
    }
}

// y = a x + b y; with b = 0, y is written without being read (it may hold
// anything, NaN included)
__global__ void k_scale_add(long n, double a, const double *__restrict__ x, double b, double *__restrict__ y)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];
}

// y_i = s_i * x_i - y_i with s_i = (lambda_drop(i) + 1): the Galerkin operator
// (lambda + 1) u - P[D u], entries grouped by a per-entry scale array.
__global__ void k_op_combine(long n, const double *__restrict__ sc, const double *__restrict__ x, double *__restrict__ y)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = sc[i] * x[i] - y[i];
}

// ----------------------------------------------------------------------------
// Gram-Schmidt passes of the Arnoldi step. A block owns kGsChunk entries of w
// (kGsR per lane, in registers); its four wavefronts split the basis vectors
// (i = wave, wave + 4, ...) so that each lane has few dependent loads in flight.
// Block partial sums go to part[i][b]; the last block to finish (ticket on
// cnt) adds them in block order, so results do not depend on scheduling, and
// resets cnt for the next launch.
//   UPD:  w -= sum_{i<kv} hin[i] V_i
//   !NRM: hout[i] = V_i . w for i < kv
//   NRM:  hacc[i] += hin[i] for i < kv (UPD only) and hacc[kv] = ||w||
// ----------------------------------------------------------------------------
constexpr int kGsR = 4, kGsChunk = 64 * kGsR;
constexpr int kGsMaxVectors = 256;  // Krylov vectors; the Givens staging below needs 3 (kv - 1) + 2 doubles of sacc
static_assert(3 * (kGsMaxVectors - 1) + 2 <= 4 * kGsChunk, "Givens staging exceeds the LDS buffer");

template <bool UPD, bool NRM>
__global__ __launch_bounds__(256) void k_gs(long n, int kv, const double *__restrict__ V, long ld,
                                            const double *__restrict__ hin, double *__restrict__ w,
                                            double *__restrict__ part, unsigned *__restrict__ cnt,
                                            double *__restrict__ hout, GivensArgs ga, double *__restrict__ vout)
{
    __shared__ double sacc[4][kGsChunk];
    __shared__ bool last;
    const int nb = gridDim.x, b = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long e0 = (long)b * kGsChunk + lane;
    double x[kGsR];
    bool ok[kGsR];
    long eo[kGsR];  // entry read from each basis vector: lanes past n read entry 0 and weigh it by zero
#pragma unroll
    for (int r = 0; r < kGsR; ++r) {
        const long e = e0 + r * 64;
        ok[r] = e < n;
        eo[r] = ok[r] ? e : 0;
        x[r] = ok[r] ? w[e] : 0.0;
    }
    // the basis loads are unconditional, so that a wavefront has all of them
    // in flight at once (a guarded load waits before the next is issued)
    if (UPD) {
        double acc[kGsR] = {};
#pragma unroll 4
        for (int i = wv; i < kv; i += 4) {
            const double hi = hin[i];
            const double *Vi = V + i * ld;
#pragma unroll
            for (int r = 0; r < kGsR; ++r) acc[r] = fma(hi, Vi[eo[r]], acc[r]);
        }
#pragma unroll
        for (int r = 0; r < kGsR; ++r) sacc[wv][r * 64 + lane] = acc[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kGsR; ++r) {
            const int j = r * 64 + lane;
            x[r] = ok[r] ? x[r] - ((sacc[0][j] + sacc[1][j]) + (sacc[2][j] + sacc[3][j])) : 0.0;
            if (wv == 0 && ok[r]) w[e0 + r * 64] = x[r];
        }
    }
    if (NRM) {
        if (wv == 0) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < kGsR; ++r) s = fma(x[r], x[r], s);
            for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
            if (lane == 0) part[b] = s;
        }
    } else {
#pragma unroll 2
        for (int i = wv; i < kv; i += 4) {
            const double *Vi = V + i * ld;
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < kGsR; ++r) s = fma(Vi[eo[r]], x[r], s);
            for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
            if (lane == 0) part[(long)i * nb + b] = s;
        }
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(cnt, 1u) == (unsigned)(nb - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    // Sum i of nsum: G threads add its block partials in a fixed strided
    // order, then a butterfly inside the group (G divides the wavefront)
    const int nsum = NRM ? 1 : kv;
    __shared__ double snrm;
    {
        int G = 64;
        while (G > 1 && G * nsum > 256) G >>= 1;
        const int i = threadIdx.x / G, g = threadIdx.x % G;
        double s = 0.0;
        if (i < nsum) {
            const double *pi = part + (long)i * nb;
            for (int q = g; q < nb; q += G) s += __hip_atomic_load(pi + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        for (int o = G >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (i < nsum && g == 0) {
            if (NRM) {
                hout[kv] = sqrt(s);
                snrm = sqrt(s);
            } else {
                hout[i] = s;
            }
        }
    }
    if (NRM && vout) {
        // v = w / ||w|| (zero norm: v = 0). The acquire fence above invalidated
        // this unit's L1, so plain loads see the other blocks' w.
        __syncthreads();
        const double t = snrm, ti = t > 0.0 ? 1.0 / t : 0.0;
        // n is even and both vectors 16-byte aligned; 16 loads in flight per thread
        const double2 *w2 = reinterpret_cast<const double2 *>(w);
        double2 *v2 = reinterpret_cast<double2 *>(vout);
#pragma unroll 16
        for (long e = threadIdx.x; e < n / 2; e += 256) {
            const double2 a = w2[e];
            v2[e] = make_double2(a.x * ti, a.y * ti);
        }
    }
    if (NRM && UPD && !ga.H)
        for (int i = threadIdx.x; i < kv; i += 256) hout[i] += hin[i];
    if (NRM && UPD && ga.H) {
        // h[i] += hin[i] (i < kv), then the Givens update of the least-squares
        // problem for column k = kv - 1: previous rotations on the new column
        // of H (h[0..k+1], kept as it is for the normalisation that follows),
        // then the rotation that zeroes h[k+1]; g updated and the residual
        // estimate |g[k+1]| / ||b|| stored. The column, the previous rotations
        // and g[k] are staged in LDS in one round of loads (sacc is free by
        // now), so the sequential sweep does not wait on a global load per
        // rotation.
        const int kc = kv - 1;
        double *scol = &sacc[0][0], *scs = scol + kc + 2, *ssn = scs + kc;  // 3 kc + 2 < 4 kGsChunk
        __shared__ double sgk;
        __syncthreads();  // snrm set, sacc free
        for (int l = threadIdx.x; l < kv; l += 256) {
            const double v = hout[l] + hin[l];
            hout[l] = v;
            scol[l] = v;
        }
        for (int l = threadIdx.x; l < kc; l += 256) {
            scs[l] = ga.cs[l];
            ssn[l] = ga.sn[l];
        }
        if (threadIdx.x == 0) {
            scol[kv] = snrm;
            sgk = ga.g[kc];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double cur = scol[0];  // entry l of the column after rotations 0..l-1
            for (int l = 0; l < kc; ++l) {
                const double nx = scol[l + 1];
                scol[l] = scs[l] * cur + ssn[l] * nx;
                cur = -ssn[l] * cur + scs[l] * nx;
            }
            const double hk1 = scol[kc + 1];
            const double den = hypot(cur, hk1);
            const double cr = den > 0.0 ? cur / den : 1.0, sr = den > 0.0 ? hk1 / den : 0.0;
            ga.cs[kc] = cr;
            ga.sn[kc] = sr;
            scol[kc] = den;
            scol[kc + 1] = 0.0;
            ga.g[kc + 1] = -sr * sgk;
            ga.g[kc] = cr * sgk;
            ga.res[0] = fabs(ga.g[kc + 1]) / ga.bnorm;  // host-visible memory
            __threadfence_system();
            ga.res[1] = ga.stamp;  // the host reads the estimate once it sees this step's stamp
            __threadfence_system();
        }
        __syncthreads();
        double *col = ga.H + (long)kc * ga.ldH;  // column kc of R, rows 0..kc+1
        for (int l = threadIdx.x; l <= kc + 1; l += 256) col[l] = scol[l];
    }
    if (threadIdx.x == 0) atomicExch(cnt, 0u);
}

// y = R^-1 g for the leading k x k block of the upper triangular R stored by
// columns (leading dimension ldH); one thread (k is at most the restart length).
__global__ void k_backsub(int k, const double *__restrict__ H, long ldH, const double *__restrict__ g,
                          double *__restrict__ y)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int l = k - 1; l >= 0; --l) {
        double s = g[l];
        for (int q = l + 1; q < k; ++q) s -= H[(long)q * ldH + l] * y[q];
        y[l] = s / H[(long)l * ldH + l];
    }
}

// v = w / nrm[0] (v may alias w); a zero norm leaves v = 0
__global__ void k_gs_scale(long n, const double *__restrict__ w, const double *__restrict__ nrm, double *v)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const double t = nrm[0];
    v[e] = t > 0.0 ? w[e] / t : 0.0;
}

// x += sum_i y[i] V_i
__global__ void k_lincomb(long n, int k, const double *__restrict__ V, long ld, const double *__restrict__ y,
                          double *__restrict__ x)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double s = x[e];
    for (int i = 0; i < k; ++i) s = fma(y[i], V[i * ld + e], s);
    x[e] = s;
}

// ============================================================================
// Host launchers
// ============================================================================
static inline unsigned nblk(long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

void launch_analyze(hipStream_t st, int q, int p, int nmax, const double *L, const double *wq, const double *cs,
                    int nf, const double *v, long vstride, double *F, double *coef, long cstride)
{
    const long n1 = (long)nf * (q + 1) * (p + 1);
    hipLaunchKernelGGL(k_anal_fourier, dim3(nblk(n1)), dim3(256), 0, st, p, q, v, vstride, cs, nf, F);
    const long n2 = (long)nf * ncoef(p);
    hipLaunchKernelGGL(k_anal_leg, dim3(nblk(n2)), dim3(256), 0, st, p, q, ncoef(nmax), L, wq, nf, F, coef,
                       cstride);
}

void launch_force(hipStream_t st, int npt, const double *syn, int eos, double E, double xs, double sigma0, double *f)
{
    hipLaunchKernelGGL(k_force, dim3(nblk(npt)), dim3(256), 0, st, npt, syn, eos, E, xs, sigma0, f);
}

void launch_nodes(hipStream_t st, const NodeJob *jobs, int n)
{
    for (int o = 0; o < n; o += kMaxNodeJobs) {
        NodeJobs b{};
        b.n = std::min(kMaxNodeJobs, n - o);
        long maxp = 0;
        for (int k = 0; k < b.n; ++k) {
            b.j[k] = jobs[o + k];
            maxp = std::max(maxp, (long)npts(jobs[o + k].q));
        }
        hipLaunchKernelGGL(k_nodes, dim3(nblk(maxp), b.n), dim3(256), 0, st, b);
    }
}

// vol[i] = sum of the wavefront partials part[off[i] .. off[i+1]) in order.
__global__ void k_vol_sum(int nd, const double *__restrict__ part, const int *__restrict__ off, double *__restrict__ vol)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd) return;
    double s = 0.0;
    for (int e = off[i]; e < off[i + 1]; ++e) s += part[e];
    vol[i] = s;
}

void launch_vol_sum(hipStream_t st, int nd, const double *part, const int *off, double *vol)
{
    hipLaunchKernelGGL(k_vol_sum, dim3(nblk(nd)), dim3(256), 0, st, nd, part, off, vol);
}

// Grid spacing of each drop, h_i = R_i pi / (p_i + 1) with R_i the radius of
// the sphere of the drop's volume (hfac_i = pi / (p_i + 1)); bad[0] = 1 when a
// volume is not positive and finite (h_i = 0 then), else 0. One block.
__global__ __launch_bounds__(256) void k_drop_h(int nd, const double *__restrict__ vol,
                                                const double *__restrict__ hfac, double *__restrict__ hj, int *bad)
{
    int b = 0;
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
        const double v = vol[i];
        const bool ok = v > 0.0 && isfinite(v);
        b |= !ok;
        hj[i] = ok ? cbrt(3.0 * v / (4.0 * 3.14159265358979323846)) * hfac[i] : 0.0;
    }
    b = __syncthreads_or(b);
    if (threadIdx.x == 0) bad[0] = b;
}

void launch_drop_h(hipStream_t st, int nd, const double *vol, const double *hfac, double *hj, int *bad)
{
    hipLaunchKernelGGL(k_drop_h, dim3(1), dim3(256), 0, st, nd, vol, hfac, hj, bad);
}

void launch_drop_bounds(hipStream_t st, int nd, const double *sx, long sstride, const int *noff, const int *ncnt,
                        double *cb)
{
    hipLaunchKernelGGL(k_drop_bounds, dim3(nd), dim3(256), 0, st, nd, sx, sstride, noff, ncnt, cb);
}

void launch_classify_bound(hipStream_t st, int T, int nd, const double *tx, long tstride, const int *tdrop,
                           const int *sys, const double *cb, const double *hj, double A, int exact, int8_t *reg,
                           double *dist, int *list, int *count)
{
    hipLaunchKernelGGL(k_classify_bound, dim3(nblk((long)T * nd)), dim3(256), 0, st, T, nd, tx, tstride, tdrop, sys,
                       cb, hj, A, exact, reg, dist, list, count);
}

// count: device-side list length, at most nmax
void launch_classify_scan(hipStream_t st, const int *count, long nmax, const int *list, int nd, const double *tx,
                          long tstride, const double *sx, long sstride, const int *noff, const int *ncnt,
                          const double *hj, double A, int8_t *reg, double *dist)
{
    if (nmax <= 0) return;
    const long waves = std::min<long>(nmax, 8192);
    hipLaunchKernelGGL(k_classify_scan, dim3(nblk(waves * 64)), dim3(256), 0, st, count, list, nd, tx, tstride, sx,
                       sstride, noff, ncnt, hj, A, reg, dist);
}

void launch_rotate(hipStream_t st, int p, const double *Ap, const double *Am, const double *cs, const double *xc,
                   long xstride, const double *dc, long dstride, double *R)
{
    const int nt = npts(p);
    hipLaunchKernelGGL(k_rotate, dim3(nblk((long)nt * 6 * ncoef(p))), dim3(256), 0, st, p, nt, Ap, Am, cs, xc,
                       xstride, dc, dstride, R);
}

int singular_lds_bytes(int p, int jb) { return jb * 9 * (p + 1) * 2 * (int)sizeof(double); }

void launch_singular(hipStream_t st, int p, int qs, int kind, const double *R, const double *Ls, int ldn,
                     const double *wsing, const double *cs, double *out, long ostride, double scale)
{
    const int nt = npts(p);
    if (p <= 48) {
        hipLaunchKernelGGL(k_singular<8>, dim3(nt), dim3(256), singular_lds_bytes(p, 8), st, p, qs, kind, R, Ls, ldn,
                           wsing, cs, out, ostride, scale);
    } else {
        hipLaunchKernelGGL(k_singular<4>, dim3(nt), dim3(256), singular_lds_bytes(p, 4), st, p, qs, kind, R, Ls, ldn,
                           wsing, cs, out, ostride, scale);
    }
}

template <int KIND, int T>
static void pair_one(hipStream_t st, int n, const PairWork *work, int item0, int tile, const int *tlist,
                     const double *tx, long tstride, const PairSrc &g0, const PairSrc &g1, double *part,
                     const float4 *rec0, const float4 *rec1, const double *cb32, int nd)
{
    if (n <= 0) return;
    const dim3 grid((n + kPairWaves - 1) / kPairWaves), block(64 * kPairWaves);
    if (rec0)
        hipLaunchKernelGGL((k_pair32<KIND, T>), grid, block, 0, st, work, n, item0, tile, tlist, tx, tstride, rec0,
                           rec1, cb32, nd, part);
    else
        hipLaunchKernelGGL((k_pair<KIND, T>), grid, block, 0, st, work, n, item0, tile, tlist, tx, tstride, g0, g1,
                           part);
}

// Items [0, n) of a work list with T targets per lane (1, 2 or 4); their
// partial blocks of 3 tile doubles start at block item0.
void launch_pair(hipStream_t st, int kind, int T, int n, const PairWork *work, int item0, int tile, const int *tlist,
                 const double *tx, long tstride, const PairSrc &g0, const PairSrc &g1, double *part,
                 const float4 *rec0, const float4 *rec1, const double *cb32, int nd)
{
    auto go = [&](auto k) {
        constexpr int K = decltype(k)::value;
        if (T == 4)
            pair_one<K, 4>(st, n, work, item0, tile, tlist, tx, tstride, g0, g1, part, rec0, rec1, cb32, nd);
        else if (T == 2)
            pair_one<K, 2>(st, n, work, item0, tile, tlist, tx, tstride, g0, g1, part, rec0, rec1, cb32, nd);
        else
            pair_one<K, 1>(st, n, work, item0, tile, tlist, tx, tstride, g0, g1, part, rec0, rec1, cb32, nd);
    };
    if (kind == 0)
        go(std::integral_constant<int, 0>());
    else
        go(std::integral_constant<int, 1>());
}

void launch_pair_pack32(hipStream_t st, int kind, const void *jobs, int njobs, int maxn, const PairSrc &g,
                        const double *cb, float4 *rec)
{
    if (njobs <= 0 || maxn <= 0) return;
    const dim3 grid((maxn + 255) / 256, njobs);
    if (kind == 0)
        hipLaunchKernelGGL(k_pair_pack32<0>, grid, dim3(256), 0, st, (const PackJob *)jobs, g, cb, rec);
    else
        hipLaunchKernelGGL(k_pair_pack32<1>, grid, dim3(256), 0, st, (const PackJob *)jobs, g, cb, rec);
}

void launch_pair_gather(hipStream_t st, int nt, int tile, const int *tile_of, const int *toff, const int *tent,
                        const int *off, const int *ent, const double *part, double *out, long ostride, bool add)
{
    if (nt <= 0) return;
    hipLaunchKernelGGL(k_pair_gather, dim3((nt + 3) / 4), dim3(256), 0, st, nt, tile, tile_of, toff, tent, off, ent,
                       part, out, ostride, add ? 1 : 0);
}

void launch_rhs(hipStream_t st, int T, const double *tx, long tstride, const double *s, double a, const double *U0,
                const double *gU_dev, double *b)
{
    hipLaunchKernelGGL(k_rhs, dim3(nblk(T)), dim3(256), 0, st, T, tx, tstride, s, a, U0[0], U0[1], U0[2], gU_dev, b);
}

void launch_scale_add(hipStream_t st, long n, double a, const double *x, double b, double *y)
{
    hipLaunchKernelGGL(k_scale_add, dim3(nblk(n)), dim3(256), 0, st, n, a, x, b, y);
}

void launch_op_combine(hipStream_t st, long n, const double *sc, const double *x, double *y)
{
    hipLaunchKernelGGL(k_op_combine, dim3(nblk(n)), dim3(256), 0, st, n, sc, x, y);
}

long gs_blocks(long n) { return (n + kGsChunk - 1) / kGsChunk; }
int gs_max_vectors() { return kGsMaxVectors; }
constexpr long kGsFuseScale = 64;  // blocks up to which the last block also writes the scaled vector

// pass 1 of classical Gram-Schmidt: h[i] = V_i . w, i < kv
void launch_gs_dots(hipStream_t st, long n, int kv, const double *V, long ld, double *w, double *part,
                    unsigned *cnt, double *h)
{
    hipLaunchKernelGGL((k_gs<false, false>), dim3(gs_blocks(n)), dim3(256), 0, st, n, kv, V, ld, nullptr, w, part,
                       cnt, h, GivensArgs{}, nullptr);
}

// w -= V h1, then h2[i] = V_i . w
void launch_gs_update_dots(hipStream_t st, long n, int kv, const double *V, long ld, const double *h1, double *w,
                           double *part, unsigned *cnt, double *h2)
{
    hipLaunchKernelGGL((k_gs<true, false>), dim3(gs_blocks(n)), dim3(256), 0, st, n, kv, V, ld, h1, w, part, cnt,
                       h2, GivensArgs{}, nullptr);
}

// w -= V h2, h[i] += h2[i], h[kv] = ||w||; with kv = 0 just h[0] = ||w||.
// With ga.H set (kv > 0) the last block also applies the Givens update.
// vout (if set) receives w / ||w||.
void launch_gs_update_norm(hipStream_t st, long n, int kv, const double *V, long ld, const double *h2, double *w,
                           double *part, unsigned *cnt, double *h, const GivensArgs &ga, double *vout)
{
    const long nb = gs_blocks(n);
    const bool al = n % 2 == 0 && (((uintptr_t)w | (uintptr_t)vout) & 15) == 0;
    double *vk = nb <= kGsFuseScale && al ? vout : nullptr;
    if (kv > 0)
        hipLaunchKernelGGL((k_gs<true, true>), dim3(nb), dim3(256), 0, st, n, kv, V, ld, h2, w, part, cnt, h, ga, vk);
    else
        hipLaunchKernelGGL((k_gs<false, true>), dim3(nb), dim3(256), 0, st, n, 0, V, ld, nullptr, w, part, cnt, h,
                           GivensArgs{}, vk);
    if (vout && !vk) hipLaunchKernelGGL(k_gs_scale, dim3(nblk(n)), dim3(256), 0, st, n, w, h + kv, vout);
}

void launch_backsub(hipStream_t st, int k, const double *H, long ldH, const double *g, double *y)
{
    hipLaunchKernelGGL(k_backsub, dim3(1), dim3(64), 0, st, k, H, ldH, g, y);
}

void launch_gs_scale(hipStream_t st, long n, const double *w, const double *nrm, double *v)
{
    hipLaunchKernelGGL(k_gs_scale, dim3(nblk(n)), dim3(256), 0, st, n, w, nrm, v);
}

void launch_lincomb(hipStream_t st, long n, int k, const double *V, long ld, const double *y, double *x)
{
    hipLaunchKernelGGL(k_lincomb, dim3(nblk(n)), dim3(256), 0, st, n, k, V, ld, y, x);
}

}  // namespace bim
