// Internal declarations shared by the host code and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace bim {

// complex index of (n, m), m >= 0, in a degree-p coefficient triangle
inline __host__ __device__ int tri(int n, int m) { return n * (n + 1) / 2 + m; }
inline __host__ __device__ int ncoef(int p) { return (p + 1) * (p + 2) / 2; }
inline __host__ __device__ int npts(int q) { return 2 * q * (q + 1); }
// offset of degree n in a per-latitude rotation table: sum_{k<n} (k+1)^2
inline __host__ __device__ size_t rot_off(int n) { return (size_t)n * (n + 1) * (2 * n + 1) / 6; }
inline __host__ __device__ size_t rot_lat_size(int p) { return rot_off(p + 1); }

// ---- host tables (tables.cpp) ----
void gauss_legendre(int q, std::vector<double> &t, std::vector<double> &w);
void legendre_table(int nmax, double t, double *P, double *D1, double *D2);
void wigner_table(int nmax, double beta, std::vector<double> &d);
void rotation_tables(int p, const std::vector<double> &theta, std::vector<double> &Ap, std::vector<double> &Am);
double legendre_sum(int q, double t);

// ---- device-side work descriptors ----
// Quadrature nodes of one drop's grid (k_nodes): the 9 synthesized fields
// syn, the latitude weights wreg, the outputs at stride sstride and the
// volume accumulator vol (nullptr: not accumulated).
struct NodeJob {
    const double *syn, *wreg;
    double *sx, *swN, *swW, *vol;
    long sstride;
    int q;
};
constexpr int kMaxNodeJobs = 32;
struct NodeJobs {
    int n;
    NodeJob j[kMaxNodeJobs];
};

// Pair sums: a work item is one wavefront's run of sources of one grid
// against up to 64 T targets (T per lane: the launch's T for whole tiles, 1
// for the remainders of a target set).
struct PairWork {
    int tlist_off;  // first entry in the target index list, or the first target (kPairContig)
    int ntgt;       // targets in this item (<= 64 T)
    int src_off;    // first source node in the source arrays
    int nsrc;       // source nodes in this item
    int pair;       // target drop * n_drops + source drop
    int pad;        // bit 0: source grid (0 standard, 1 upsampled); kPairContig: targets
                    // tlist_off .. tlist_off + ntgt - 1, no index list; kPairSmall: a
                    // remainder item (<= 64 targets, one per lane)
    double w;       // weight applied to the sum
};
constexpr int kPairContig = 2;
constexpr int kPairSmall = 4;

// Device state of the GMRES least-squares problem (Givens rotations applied
// on the device): R by columns, rotations, right-hand side g, and the
// residual estimate |g[k+1]| / ||b|| of the latest column.
struct GivensArgs {
    double *H = nullptr;
    long ldH = 0;
    double *cs = nullptr, *sn = nullptr, *g = nullptr, *res = nullptr;  // res: {estimate, stamp}
    double bnorm = 1.0;
    double stamp = 0.0;  // written to res[1] after the estimate
};

// Drops of one degree in a pass of the batched singular pipeline (kernel
// argument). Latitude unit g = drop * (p+1) + j covers the 2p targets of
// latitude j of that drop; a chunk of units starts at unit u0 and puts unit
// u0 + y at columns y * 2p + k.
constexpr int kPipeMaxDrops = 64;
struct PipeDrops {
    int n;
    long coff[kPipeMaxDrops];   // coefficient offset (inside a component block)
    long toff[kPipeMaxDrops];   // global index of the first target
    double *M[kPipeMaxDrops];   // stored double-layer rows (or null)
};

// Stored double-layer rows of one drop applied to a density: out[c][t] +=
// w sum_pairs M[t][pair] . u (k_dl_apply_multi takes several drops).
// One analysis job of the batched kernel: grid values -> coefficients of
// degree p for ncomp components; with cx set the output is csc * cx - P[v]
// (the Galerkin combine of the second-kind operator) instead of P[v].
struct AnaJob {
    const double *v;      // component c grid at v + c * vstride
    const double *L;      // Legendre tables [3][q+1][ldn] (kind 0 used)
    const double *wq;     // (pi/q) w_j
    double *coef;         // component c at coef + c * cstride
    long vstride, cstride;
    int p, q, ldn, ncomp;
    const double *cx;     // optional: coefficients combined into the output (same layout as coef)
    double csc;
};

// Matrix-core transforms of value fields (kernels_xform.hip): nf fields of
// degree p on the degree-q grid. Field f's coefficients (complex n-major
// triangle, (re, im) interleaved) start at cb[2 f] (real parts) and cb[2 f +
// 1] (imaginary parts) inside the coefficient vector, its grid values [j][k]
// (2q longitudes per latitude) at gb[f] inside the grid array.
struct XJob {
    const long *cb;     // [2 nf]
    const long *gb;     // [nf]
    const double *csc;  // analysis: [nf] factor of x in the output (nullptr: none)
    const double *L;    // Ptilde_n^m(t_j) at L[j * ldn + tri(n, m)]
    const double *wq;   // analysis: (pi/q) w_j
    const void *trig;   // [2 (p+1)][q] (the job's type): synthesis w_m (cos, -sin)(m phi_k), analysis (cos, -sin)
    void *G;            // intermediate [p+1][q+1][2 nf] (the job's type)
    double *grid;       // synthesis output, analysis input
    int p, q, nf, ldn;
};
constexpr int kMaxXJobs = 8;

// One drop of the surface-operator kernel (kernels_surf.hip). syn holds, per
// grid point (np of them): x fields f = 0..5 (value, d_theta, d_phi,
// d_theta^2, d_theta d_phi, d_phi^2) x 3 components at (3 f + c) np; Gamma
// fields f = 0..5 at (18 + f) np (when gam); u fields f = 0..2 x 3
// components at (24 + 3 f + c) np (when fE is set).
struct SurfJob {
    const double *syn;
    const double *wreg;   // regular-rule weight per latitude (pi/q) w_j / sin theta_j
    double *fE, *lg;      // grid outputs: -Gamma div_s u, Laplace-Beltrami of Gamma (optional)
    double *mass, *vol;   // accumulated int Gamma dS and enclosed volume (optional)
    long np;
    int q, gam;           // grid degree; Gamma fields present
};
constexpr int kMaxSurfJobs = 32;
struct SurfJobs {
    int n;
    SurfJob j[kMaxSurfJobs];
};

struct DlJob {
    const double *M;
    const double *u;   // density coefficients of the drop, component stride ustride
    double *out;       // first target of the drop, component stride ostride
    double w;
    int nt, nc2;
};
constexpr int kMaxDlJobs = 32;
struct DlJobs {
    int n;
    DlJob j[kMaxDlJobs];
};

// Nearest-region items: a grid target t (global index) of drop i whose
// nearest node of source drop j is within h_j.
struct NearItem {
    int t, i, j, pad;
};
constexpr int kNearMaxL = 16;  // interpolation points per item, at most

struct NearArgs {
    const NearItem *items;
    int n;                      // items
    const int *dp;              // degree per drop
    const long *dcoff;          // coefficient offset per drop (inside a component block)
    const int *dtoff;           // first standard-grid node per drop
    const double *hj;           // h per drop
    const double *xc;           // drop coefficients [3][Ctot]
    long Ctot;
    const double *tx;           // standard-grid nodes (= grid targets) [3][T]
    long T;
    const double *gl_t;         // Gauss-Legendre nodes cos(theta_j) of each drop's grid
    const int *gl_off;          // per drop: first entry in gl_t
    int L;                      // interpolation points
    double A;                   // Omega_1 threshold in units of h
    double *par;                // per item: theta*, phi*, |x0 - x*|, nearest node
    double *vx;                 // interpolation points [3][V], V = n L
    long V;
    int8_t *vreg;               // their grid: 0 standard, 1 upsampled
    double *Pst;                // Ptilde_n^m(cos theta*) per item, stride ldp
    long ldp;
};

// One source grid for the pair sums: component-major arrays [3][stride].
struct PairSrc {
    const double *x, *wN, *wW, *d;
    long stride;
};
// Nodes [off, off + n) of drop `drop` in one source grid (FP32 record packing).
struct PackJob {
    long off;
    int n, drop;
};

// Fast summation of far drop pairs (kernels_fmm.hip). Expansion order P <=
// kFmmMaxOrder; 4 channels; local expansions and partial multipoles keep
// m >= 0 ((P+1)(P+2)/2 complex per channel), the multipoles used by the
// translation all orders, channel fastest ((P+1)^2 x 4 complex).
constexpr int kFmmMaxOrder = 30, kFmmThreads = 512, kFmmChunk = 128;
static_assert((kFmmMaxOrder + 1) * (kFmmMaxOrder + 2) / 2 <= kFmmThreads, "one thread per coefficient");

// One source grid of one drop (a multipole slot): nodes [off, off + ns) of
// component-major arrays with the given stride; regular-harmonic table at
// Y + yoff (ns x ntri), per-source weights at W + woff (ns x 4 or 12),
// partial multipoles from chunk pbase on.
struct FmmSrcJob {
    const double *x, *d, *wW, *wN;
    long stride, off, yoff, woff;
    int ns, slot, pbase, drop;
};

// A far pair: multipole slot src translated to target slot tgt with weight
// w, truncated at degree order (<= P) in both expansions.
struct FmmPair {
    int src, tgt, order, pad;
    double w;
};

// Target nodes [off, off + n) (global target indices) of target slot.
struct FmmTgtJob {
    long off;
    int n, slot;
};

}  // namespace bim
