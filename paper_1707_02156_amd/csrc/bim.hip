// Context and C ABI of the Stokes layer-potential library (see include/bim.h).
//
// One call of bim_eval_velocity runs, on the context stream:
//   1. nodes: synthesis of x, x_theta, x_phi on the standard (degree p) and
//      upsampled (degree U_tilde p) grid of every drop -> positions, weighted
//      normals and area elements, enclosed volume (Sec. 2.1);
//   2. force: synthesis on the degree U_geom p grid, f = 2 sigma K n - grad sigma,
//      analysis to degree p (Sec. 1, Sec. 1.3);
//   3. regions: node distance of every target to every other drop (Sec. 2.3),
//      compacted into pair work lists on the host (one device-to-host copy);
//   4. single layer: rotated-pole singular rule per drop (Sec. 2.2, App. B) and
//      pair sums on the standard / upsampled grids;
//   5. right-hand side 2 u_inf - S/(4 pi), Galerkin projection (Sec. 1.2), and
//      GMRES on (lambda+1) u - P[sum_j (lambda_j - 1)/(4 pi) D_j[u]] when any
//      lambda != 1.
#include "internal.hpp"
#include "../../include/bim.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

namespace bim {

void launch_analyze(hipStream_t st, int q, int p, int nmax, const double *L, const double *wq, const double *cs,
                    int nf, const double *v, long vstride, double *F, double *coef, long cstride);
void launch_force(hipStream_t st, int npt, const double *syn, int eos, double E, double xs, double sigma0, double *f);
void launch_nodes(hipStream_t st, const NodeJob *jobs, int n);
void launch_vol_sum(hipStream_t st, int nd, const double *part, const int *off, double *vol);
void launch_drop_bounds(hipStream_t st, int nd, const double *sx, long sstride, const int *noff, const int *ncnt,
                        double *cb);
void launch_classify_bound(hipStream_t st, int T, int nd, const double *tx, long tstride, const int *tdrop,
                           const int *sys, const double *cb, const double *hj, double A, int exact, int8_t *reg,
                           double *dist, int *list, int *count);
void launch_drop_h(hipStream_t st, int nd, const double *vol, const double *hfac, double *hj, int *bad);
void launch_classify_scan(hipStream_t st, const int *count, long nmax, const int *list, int nd, const double *tx,
                          long tstride,
                          const double *sx, long sstride, const int *noff, const int *ncnt, const double *hj, double A,
                          int8_t *reg, double *dist);
void launch_rotate(hipStream_t st, int p, const double *Ap, const double *Am, const double *cs, const double *xc,
                   long xstride, const double *dc, long dstride, double *R);
void launch_singular(hipStream_t st, int p, int qs, int kind, const double *R, const double *Ls, int ldn,
                     const double *wsing, const double *cs, double *out, long ostride, double scale);
void launch_near_setup(hipStream_t st, const NearArgs &a);
void launch_near_interp(hipStream_t st, const NearArgs &a, int kind, const double *selfc, const double *dens,
                        const double *vacc, const double *wts, double *out);
void launch_pair(hipStream_t st, int kind, int T, int n, const PairWork *work, int item0, int tile, const int *tlist,
                 const double *tx, long tstride, const PairSrc &g0, const PairSrc &g1, double *part,
                 const float4 *rec0 = nullptr, const float4 *rec1 = nullptr, const double *cb32 = nullptr, int nd = 0);
void launch_pair_pack32(hipStream_t st, int kind, const void *jobs, int njobs, int maxn, const PairSrc &g,
                        const double *cb, float4 *rec);
void launch_pair_gather(hipStream_t st, int nt, int tile, const int *tile_of, const int *toff, const int *tent,
                        const int *off, const int *ent, const double *part, double *out, long ostride, bool add);
struct SingArgs {
    int p, qs, nt;
    const double *Ap, *Am, *ApT, *AmT;
    const double *csp;
    const double *xc;
    long xstride;
    const double *dc;
    long dstride;
    const double *L;
    const double *wsing;
    double *out_sl;
    long ostride;
    double scale;
    double *M;
};
bool launch_sing_fused(hipStream_t st, bool sl, bool dl, const SingArgs &a);
struct LegBatchH {
    int R, K;
    long tab_off, in_row, out_row;
};
size_t rot_lds_bytes(int p);
void launch_rot2(hipStream_t st, int p, const double *Ap, const double *Am, const double *csp, const double *xc,
                 long xstride, const double *dc, long dstride, const PipeDrops &pd, int u0, int nunits,
                 double *Bx, double *Bd, long NC);
void launch_leg_mfma(hipStream_t st, int nbatch, int maxrows, const void *batches, const double *tab, const double *in,
                     double *out, long NC);
int leg_mfma_max_rows();
int leg_mfma_max_depth();
size_t fk_lds_bytes(int p, int qs, bool sl, int tg);
void launch_fk(hipStream_t st, bool sl, bool dl, int p, int qs, int nt, const double *Gx, const double *Gd, long NC6,
               const double *wsing, const double *cs, const double *X0, double *part, double *Fa, long NC12);
void launch_sum_part(hipStream_t st, int nt, int Q1, int nk, int P1, const double *part, const PipeDrops &pd, int u0,
                     double scale, double *out, long ostride);
void launch_pole(hipStream_t st, int p, int nt, const double *Bx, long NC, double *X0);
void launch_adjrot(hipStream_t st, int p, const double *Ap, const double *Am, const double *csp, const double *Bt,
                   long NC12, const PipeDrops &pd, int u0, int nunits);
void launch_dl_apply_multi(hipStream_t st, const DlJob *jobs, int n, long ustride, long ostride);
void pipe_set_lds_limits();
struct SynJob {
    const double *coef;
    const double *L;
    double *out;
    long cstride, ostride, fstride;
    int p, q, ldn, ncomp, mask;
};
void launch_synth_batch(hipStream_t st, const SynJob *jobs, int n, double *z0 = nullptr, long nz0 = 0,
                        double *z1 = nullptr, long nz1 = 0);
void launch_anal_batch(hipStream_t st, const AnaJob *jobs, int n);
size_t anal_batch_lds(int p, int q);
bool xform_fits(int p, int q, bool analysis);
void launch_xsynth(hipStream_t st, bool f32, const XJob *jobs, int n, const double *x, double *z0, long nz0,
                   double *z1, long nz1);
void launch_xanal(hipStream_t st, bool f32, const XJob *jobs, int n, const double *x, double *y, double sgn);
bool sing_fused_fits(int p, int qs, bool sl, bool dl);
void launch_dl_apply(hipStream_t st, int nt, int nc2, const double *M, const double *u, long ustride, double w,
                     double *out, long ostride);
void launch_rhs(hipStream_t st, int T, const double *tx, long tstride, const double *s, double a, const double *U0,
                const double *gU_dev, double *b);
void launch_scale_add(hipStream_t st, long n, double a, const double *x, double b, double *y);
void launch_op_combine(hipStream_t st, long n, const double *sc, const double *x, double *y);
long gs_blocks(long n);
int gs_max_vectors();
void launch_gs_dots(hipStream_t st, long n, int kv, const double *V, long ld, double *w, double *part,
                    unsigned *cnt, double *h);
void launch_gs_update_dots(hipStream_t st, long n, int kv, const double *V, long ld, const double *h1, double *w,
                           double *part, unsigned *cnt, double *h2);
void launch_gs_update_norm(hipStream_t st, long n, int kv, const double *V, long ld, const double *h2, double *w,
                           double *part, unsigned *cnt, double *h, const GivensArgs &ga = GivensArgs{},
                           double *vout = nullptr);
void launch_backsub(hipStream_t st, int k, const double *H, long ldH, const double *g, double *y);
void launch_gs_scale(hipStream_t st, long n, const double *w, const double *nrm, double *v);
void launch_surf_terms(hipStream_t st, const SurfJob *jobs, int n);
void launch_mul(hipStream_t st, long n, const double *d, const double *x, double *y);
void launch_axpby(hipStream_t st, long n, double a, const double *x, double b, const double *y, double *out);
void launch_rep_pack(hipStream_t st, int q, int nf, int nb, const double *coef, long cstride, const double *hdr,
                     double *rec);
void launch_rep_eval(hipStream_t st, int q, int nf, int nb, const double *rec, const double *cm, const double *th,
                     const double *ph, long ang_bs, long N, double *out);
void launch_rep_grad(hipStream_t st, int nb, long N, const double *E, const double *gE, double *g,
                     unsigned long long *gmax);
void launch_rep_move(hipStream_t st, int nb, long N, const double *E, const double *g, double dtau, double *th,
                     double *ph, long ang_bs, const unsigned long long *gmax, double eps, int check, int *moves);
void launch_rep_cut(hipStream_t st, int q, int nb, const double *xt, long cs, double P_cut, double *hp, int *ncut,
                    unsigned long long *gmax);
void launch_lincomb(hipStream_t st, long n, int k, const double *V, long ld, const double *y, double *x);
void launch_fmm_ytab(hipStream_t st, const FmmSrcJob *jobs, int njobs, int maxns, int P, const double *cen, void *Y,
                     bool f32);
void launch_fmm_p2m(hipStream_t st, const FmmSrcJob *jobs, int njobs, int maxns, int kind, int P, const double *cen,
                    const void *Y, bool f32, double *W, double2 *part, double2 *M);
void launch_fmm_m2l(hipStream_t st, int npairs, const FmmPair *pairs, int P, const double *cen_s, const double *cen_t,
                    const double2 *M, double2 *Lp, int nt, const int *poff, double2 *L);
void launch_fmm_l2p(hipStream_t st, int njobs, const FmmTgtJob *jobs, int maxn, int P, const double *cen_t,
                    const double2 *L, double2 *C, const double *tx, long tstride, double *out, long ostride);

static const double kPi = 3.14159265358979323846;

struct Error {
    int code;
    std::string msg;
};

#define HIPC(expr)                                                                                 \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            throw Error{e_ == hipErrorOutOfMemory ? BIM_ENOMEM : BIM_EDEVICE,                      \
                        std::string(#expr) + ": " + hipGetErrorString(e_)};                         \
    } while (0)

#define REQUIRE(cond, code, msg) \
    do {                         \
        if (!(cond)) throw Error{code, msg}; \
    } while (0)

// Set while an entry point that must not allocate device memory runs on
// this thread (bim_apply_double_layer_noalloc): DBuf::ensure then fails with
// BIM_ESTATE instead of allocating.
static thread_local bool t_no_alloc = false;

// Device buffer owned by a context.
struct DBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    void release()
    {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    void ensure(size_t b)
    {
        if (b <= bytes && ptr) return;
        if (t_no_alloc)
            throw Error{BIM_ESTATE, "the call would allocate device memory (" + std::to_string(b) +
                                        " bytes): apply bim_apply_double_layer once to these drops first"};
        const bool regrow = ptr != nullptr;
        release();
        if (b == 0) b = 8;
        // grow with slack: freeing device memory waits for the whole device,
        // so a context reused for inputs of varying size should rarely regrow
        if (regrow) b += b / 4;
        HIPC(hipMalloc(&ptr, b));
        bytes = b;
    }
    double *d() const { return static_cast<double *>(ptr); }
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Host vectors in pinned memory: the lists uploaded at every evaluation are
// copied from them without staging, so an upload neither waits for the work
// ahead of it in the stream nor makes the device wait for the host. Their
// storage is kept across evaluations (cleared, refilled, grown rarely).
template <class T> struct PinnedAlloc {
    using value_type = T;
    PinnedAlloc() = default;
    template <class U> PinnedAlloc(const PinnedAlloc<U> &) {}
    T *allocate(size_t n)
    {
        void *p = nullptr;
        if (hipHostMalloc(&p, std::max<size_t>(1, n) * sizeof(T)) != hipSuccess) throw std::bad_alloc();
        return static_cast<T *>(p);
    }
    void deallocate(T *p, size_t) { (void)hipHostFree(p); }
    template <class U> bool operator==(const PinnedAlloc<U> &) const { return true; }
    template <class U> bool operator!=(const PinnedAlloc<U> &) const { return false; }
};
template <class T> using HVec = std::vector<T, PinnedAlloc<T>>;

// Tables of a degree-q grid with Legendre functions up to degree nmax.
struct GridTab {
    int q = 0, nmax = 0;
    DBuf L, wq, wreg, wsing, cs;
    DBuf xtrig[2][2];  // matrix-core Fourier tables [analysis][FP32]
    std::vector<double> t, w, th;
};

struct RotTab {
    int p = 0;
    DBuf Ap, Am, ApT, AmT;
};

struct Drop {
    int p;
    double lam;
    long coff;  // offset (doubles) inside one component block of coefficients
    long toff;  // offset of its standard-grid nodes
    long uoff;  // offset of its upsampled-grid nodes
    int qu, qg, qs;
};

struct Ctx {
    bim_options opt{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // second stream: the singular pipeline of the single-layer pass runs on
    // it while the context's stream classifies the regions and the host
    // builds the pair lists; the context's stream waits for ev_join before
    // the pipeline's results are used
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool join_pending = false;
    std::string err;

    int nd = 0;
    std::vector<Drop> drops;
    long Ctot = 0;  // doubles per component block of coefficients
    long T = 0;     // standard-grid nodes (targets) over all drops
    long S1 = 0;    // upsampled nodes over all drops

    int eos = BIM_EOS_UNIFORM;
    double E = 0.0, xs = 0.0, sigma0 = 1.0;
    bool have_gamma = false;
    double U0[3] = {0, 0, 0}, gradU[9] = {0};

    DBuf xc, gc, fc, gU;
    DBuf tx, s0N, s0W, s0d;        // standard-grid nodes [3][T]
    DBuf s1x, s1N, s1W, s1d;       // upsampled nodes [3][S1]
    DBuf tdrop, vol, hj, noff, ncnt, hfac, hbad;
    DBuf volpart, voloff;  // per-wavefront partial volumes of the standard grids, and each drop's first
    std::vector<int> voloff_h;
    DBuf unoff, uncnt, cbnd1;  // upsampled grids: node offsets, counts, centres and radii
    std::vector<int> sys_h;  // independent system of each drop (bim_set_systems)
    DBuf sysd;
    DBuf reg, dist, cbnd, clist, ccount;
    bool regions_exact = false;  // distances of every pair computed (bim_regions with dist)
    DBuf tlist;
    std::vector<int> tlist_h;         // host image of tlist
    std::vector<PairWork> w0h, w1h;   // pair work templates (weights per pass)
    int pair_ch = 0;                  // sources per pair work item (0: from the pair count)
    int pair_T_fix = 0;               // targets per lane of whole tiles (0: from the pair count)
    int pair_T = 4;                   // targets per lane of the whole-tile pair items in use
    bool pair_tuned = false;          // pair_T_fix / pair_ch chosen by tune_pairs for these drops
    double npairs_direct = 0.0;       // direct pairs of one application (the last build_lists)
    DBuf pair_part;                   // partial sums of the pair work items [item][3][64 pair_T]
    double *part_override = nullptr;  // the no-allocation scratch in place of pair_part (during such a call)
    DBuf pack_jobs, rec32_0, rec32_1; // FP32 source records of the mixed form
    std::vector<PackJob> pack_h;
    int pack_n0 = 0, pack_n1 = 0, pack_max0 = 0, pack_max1 = 0;
    // fixed-order reduction lists of a pair work list (k_pair_gather): per
    // target tile for the items over contiguous tiles, per target for the
    // items over index lists
    struct Gather {
        HVec<int> h_toff, h_tent, h_off, h_ent;
        DBuf toff, tent, off, ent;
        long nt = 0;
    };
    // target tiles of the contiguous pair items: tile of each target, first
    // target of each tile
    std::vector<int> tile_of_h, tile_start_h;
    DBuf tile_of;
    struct WList {
        std::vector<double> wt;
        // stale: built for earlier regions; refilled in place (its buffers
        // kept) by the next request for a weight table
        bool stale = false;
        // host images the device copies are made from (kept for the list's
        // lifetime, so no upload waits; declared before the device buffers,
        // whose release waits for the device, so they outlive any copy)
        HVec<PairWork> h_items;
        HVec<double> h_nw;
        HVec<FmmPair> h_fp;
        DBuf d;
        int n = 0;           // items: whole tiles first, then the remainder items
        double pairs = 0.0;  // target-source pairs per application
        Gather g;
        DBuf nw;             // weight of each nearest-region item
        DBuf fp;             // far pairs of the fast summation with their weights
    };
    std::vector<std::unique_ptr<WList>> wlists;
    std::vector<int8_t> reg_h;
    int n_om1 = 0, n_om2 = 0;
    // fast summation of far drop pairs (opt.fmm_order != 0): multipole slots
    // (drop, source grid), target slots (drops), pairs grouped by target slot
    struct Fmm {
        int P = 0;
        std::vector<FmmSrcJob> src;
        std::vector<FmmTgtJob> tgt;
        std::vector<FmmPair> pairs;  // weights set per weight table
        std::vector<int> pair_ij;    // i * nd + j of each pair
        std::vector<int> poff;       // pairs of target slot t: [poff[t], poff[t+1])
        int maxns = 0, maxnt = 0;
        long nsrc = 0, ntgt = 0, nchunks = 0;
        double m2l_flops = 0.0;  // algorithmic flops of the translations of one application
        DBuf dsrc, dtgt, dpoff, cen_s, cen_t, Y, W, part, M, Lp, L, C;
        void reset(int order)  // a new plan (device buffers kept for reuse)
        {
            P = order;
            src.clear();
            tgt.clear();
            pairs.clear();
            pair_ij.clear();
            poff.clear();
            maxns = maxnt = 0;
            nsrc = ntgt = nchunks = 0;
            m2l_flops = 0.0;
        }
    } fmm;
    int fmm_tuned = -1;  // order chosen by tune_fmm (fmm_order = -1), -1 before tuning
    // nearest-region items (near_rule 1) and their interpolation points
    std::vector<NearItem> near_h;
    std::vector<char> near_src;                 // drops that are the source of an item
    DBuf near_items, near_par, near_vx, near_vreg, near_Pst, near_vacc, near_self, near_selfc;
    DBuf near_dp, near_dcoff, near_dtoff, near_glt, near_gloff;
    DBuf near_work, near_tl;
    Gather near_g;        // interpolation points: slots of the pair items
    Gather near_tg;       // grid targets: their items' interpolated values, near_res [3][items]
    DBuf near_res;
    int near_nwork = 0;
    long near_ldp = 0;
    double near_pairs = 0.0;
    DBuf acc, tmp, bvec, scl;      // [3][T] accumulators, [3][Ctot] vectors
    DBuf acc2;                     // [3][T] the single-layer pipeline's part when it runs on the second stream
    DBuf synbuf, Gbuf, Rbuf, Fbuf, fgrid;
    // per drop: stored singular double-layer rows. The buffers are kept
    // (grown, never freed) when new drops are set: freeing device memory
    // waits for the whole device and a fresh large allocation is slow, which
    // a server slot would pay at every request
    std::vector<std::unique_ptr<DBuf>> Mdl;
    // pinned host images of the per-drop tables set_drops uploads
    HVec<int> h_tdrop, h_noff, h_ncnt, h_unoff, h_uncnt, h_sys;
    HVec<double> h_xc, h_hfac, h_scl, h_gU;
    std::vector<char> Mok;
    DBuf V, hbuf, ybuf, wvec, xsol, rvec, gspart, gscnt, givbuf;
    DBuf bcorr, xcorr;  // per-system corrections of a joint solve
    // time step: states, stage velocities and surfactant terms, surface fields and outputs
    DBuf ts_x0, ts_g0, ts_u0, ts_uh, ts_xh, ts_gh, ts_fe, ts_ki, ts_ke, ts_sinv, ts_w, ts_lw, ts_z, ts_syn, ts_grid,
        ts_acc;
    // reparametrization: initial expansions, current coefficients, node angles, evaluations
    DBuf rp_x0, rp_g0, rp_xt, rp_hp, rp_ang, rp_E, rp_gE, rp_g, rp_gmax, rp_rec;
    std::map<int, std::unique_ptr<DBuf>> rp_tab;  // Legendre recursion coefficients per degree
    double *hhost = nullptr;       // pinned
    double *hres = nullptr;        // pinned, coherent: GMRES residual estimates and their stamps, written by the device
    double gm_seq = 0.0;           // stamp of the latest enqueued GMRES step (exact integer)

    bool nodes_ok = false, force_ok = false, regions_ok = false;

    // kernel timing with HIP events on the context stream (bim_profile)
    struct ProfEntry {
        int launches = 0;
        double ms = 0.0, flops = 0.0, bytes = 0.0;
        std::vector<std::pair<hipEvent_t, hipEvent_t>> pend;
    };
    bool prof_on = false;
    std::map<std::string, ProfEntry> prof;
    std::set<std::string> prof_sel;  // kernels timed with events (empty = all)
    std::vector<hipEvent_t> evpool;
    std::map<std::pair<int, int>, std::unique_ptr<GridTab>> grids;
    std::map<int, std::unique_ptr<RotTab>> rots;

    // matrix-core transforms of value fields: one plan per degree group of
    // the drops (their three components as fields), built on first use after
    // bim_set_drops, and plans of stand-alone calls by (p, q, nf)
    struct XPlan {
        int p = 0, qu = 0, nf = 0;
        std::vector<long> h_cb, h_gb0, h_gb1;  // coefficient offsets [2 nf], standard / upsampled grid offsets [nf]
        std::vector<double> h_csc;             // lambda + 1 per field
        DBuf cb, gb0, gb1, csc;
    };
    std::vector<std::unique_ptr<XPlan>> xplans;
    std::map<std::tuple<int, int, int>, std::unique_ptr<XPlan>> xfields;
    DBuf xG;  // their intermediate [m][j][col]
    int xmode[2][2] = {{-1, -1}, {-1, -1}};  // [synthesis, analysis][FP32]: 1 matrix cores, 0 scalar, -1 undecided

    // batched singular pipeline: contraction tables per (p, qs) and work buffers
    struct PipeTab {
        DBuf syn, ana, bsx, bsd, ban;  // tables and batch descriptors
        int maxrows_syn = 0, maxrows_ana = 0;
    };
    std::map<std::pair<int, int>, std::unique_ptr<PipeTab>> pipes;
    DBuf pBx, pBd, pGx, pGd, pPart, pX0, pFa, pBt;

    ~Ctx()
    {
        pipes.clear();
        for (auto &kv : prof)
            for (auto &pr : kv.second.pend) {
                (void)hipEventDestroy(pr.first);
                (void)hipEventDestroy(pr.second);
            }
        for (auto e : evpool) (void)hipEventDestroy(e);
        grids.clear();
        rots.clear();
        if (hhost) (void)hipHostFree(hhost);
        if (hres) (void)hipHostFree(hres);
        if (side) {
            (void)hipStreamSynchronize(side);
            (void)hipStreamDestroy(side);
        }
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

// --------------------------------------------------------------------------
// kernel timing
// --------------------------------------------------------------------------
static hipEvent_t prof_event(Ctx &c)
{
    if (!c.evpool.empty()) {
        hipEvent_t e = c.evpool.back();
        c.evpool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPC(hipEventCreate(&e));
    return e;
}

// Brackets the launches issued in its scope with events when profiling is on;
// records the algorithmic flops and bytes of those launches.
struct ProfScope {
    Ctx &c;
    Ctx::ProfEntry *e = nullptr;
    hipEvent_t a = nullptr;
    hipStream_t st;
    ProfScope(Ctx &cc, const char *name, double flops, double bytes, hipStream_t s = nullptr)
        : c(cc), st(s ? s : cc.stream)
    {
        if (!c.prof_on) return;
        Ctx::ProfEntry *pe = &c.prof[name];
        pe->flops += flops;
        pe->bytes += bytes;
        pe->launches += 1;
        if (!c.prof_sel.empty() && !c.prof_sel.count(name)) return;
        e = pe;
        a = prof_event(c);
        HIPC(hipEventRecord(a, st));
    }
    ~ProfScope()
    {
        if (!e) return;
        hipEvent_t b = prof_event(c);
        if (hipEventRecord(b, st) == hipSuccess) e->pend.emplace_back(a, b);
    }
};

static void prof_drain(Ctx &c)
{
    HIPC(hipStreamSynchronize(c.stream));
    if (c.side) HIPC(hipStreamSynchronize(c.side));
    for (auto &kv : c.prof) {
        for (auto &pr : kv.second.pend) {
            float ms = 0.0f;
            HIPC(hipEventElapsedTime(&ms, pr.first, pr.second));
            kv.second.ms += ms;
            c.evpool.push_back(pr.first);
            c.evpool.push_back(pr.second);
        }
        kv.second.pend.clear();
    }
}

// Algorithmic work of the fused singular kernel per target.
static double sing_flops_per_target(int p, int qs, bool sl, bool dl)
{
    const double nc = ncoef(p), P1 = p + 1, Q1 = qs + 1, KK = qs / 2 + 1, NP = npts(qs);
    const double rot = (double)rot_lat_size(p);
    const double nx = sl ? 6.0 : 3.0;
    double f = nx * nc * 6.0 + nx * rot * 4.0;                     // phases + rotation
    f += (sl ? 9.0 : 6.0) * Q1 * nc * 4.0;                          // Legendre sums
    f += (sl ? 12.0 : 9.0) * Q1 * KK * P1 * 4.0;                    // Fourier sums
    if (sl) f += NP * 35.0;                                         // single-layer kernel
    if (dl) {
        f += NP * 40.0;                                             // stresslet fields
        f += 6.0 * Q1 * P1 * KK * 10.0;                             // Fourier analysis
        f += 6.0 * nc * Q1 * 4.0;                                   // Legendre analysis
        f += 6.0 * rot * 4.0 + 6.0 * nc * 6.0;                      // adjoint rotation
    }
    return f;
}

// --------------------------------------------------------------------------
// tables
// --------------------------------------------------------------------------
static GridTab &grid(Ctx &c, int q, int nmax)
{
    auto key = std::make_pair(q, nmax);
    auto it = c.grids.find(key);
    if (it != c.grids.end()) return *it->second;
    auto g = std::make_unique<GridTab>();
    g->q = q;
    g->nmax = nmax;
    gauss_legendre(q, g->t, g->w);
    g->th.resize(q + 1);
    const int nc = ncoef(nmax);
    std::vector<double> L((size_t)3 * (q + 1) * nc), wq(q + 1), wreg(q + 1), wsing(q + 1), cs(4 * q);
    for (int j = 0; j <= q; ++j) {
        g->th[j] = std::acos(g->t[j]);
        legendre_table(nmax, g->t[j], &L[(size_t)j * nc], &L[((size_t)(q + 1) + j) * nc],
                       &L[((size_t)2 * (q + 1) + j) * nc]);
        const double s = std::sin(g->th[j]);
        wq[j] = kPi / q * g->w[j];
        wreg[j] = wq[j] / s;
        wsing[j] = wq[j] * legendre_sum(q, g->t[j]) * 2.0 * std::sin(g->th[j] / 2.0) / s;
    }
    for (int i = 0; i < 2 * q; ++i) {
        cs[i] = std::cos(kPi * i / q);
        cs[2 * q + i] = std::sin(kPi * i / q);
    }
    auto up = [&](DBuf &b, const std::vector<double> &v) {
        b.ensure(v.size() * sizeof(double));
        HIPC(hipMemcpyAsync(b.ptr, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
        HIPC(hipStreamSynchronize(c.stream));
    };
    up(g->L, L);
    up(g->wq, wq);
    up(g->wreg, wreg);
    up(g->wsing, wsing);
    up(g->cs, cs);
    auto &ref = *g;
    c.grids[key] = std::move(g);
    return ref;
}

static RotTab &rot(Ctx &c, int p)
{
    auto it = c.rots.find(p);
    if (it != c.rots.end()) return *it->second;
    auto r = std::make_unique<RotTab>();
    r->p = p;
    GridTab &g = grid(c, p, p);
    std::vector<double> Ap, Am;
    rotation_tables(p, g.th, Ap, Am);
    // transposed blocks ([mu][nu] per degree) for the adjoint rotation
    std::vector<double> ApT(Ap.size()), AmT(Am.size());
    const size_t per = rot_lat_size(p);
    for (int j = 0; j <= p; ++j)
        for (int n = 0; n <= p; ++n)
            for (int a = 0; a <= n; ++a)
                for (int b = 0; b <= n; ++b) {
                    const size_t o = per * j + rot_off(n);
                    ApT[o + (size_t)b * (n + 1) + a] = Ap[o + (size_t)a * (n + 1) + b];
                    AmT[o + (size_t)b * (n + 1) + a] = Am[o + (size_t)a * (n + 1) + b];
                }
    auto up = [&](DBuf &b, const std::vector<double> &v) {
        b.ensure(v.size() * sizeof(double));
        HIPC(hipMemcpyAsync(b.ptr, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
        HIPC(hipStreamSynchronize(c.stream));
    };
    up(r->Ap, Ap);
    up(r->Am, Am);
    up(r->ApT, ApT);
    up(r->AmT, AmT);
    auto &ref = *r;
    c.rots[p] = std::move(r);
    return ref;
}

// --------------------------------------------------------------------------
// transforms on the context stream
// --------------------------------------------------------------------------
// Synthesis job: ncomp components of a degree-p field on the degree-q grid,
// derivative sets by mask bit (0 value, 1 d/dtheta, 2 d/dphi, 3 d2/dtheta2,
// 4 d2/dtheta dphi, 5 d2/dphi2); field f (f-th set bit), component c written
// at out + f * fstride + c * ostride.
static SynJob syn_job(Ctx &c, int p, int q, int ncomp, const double *coef, long cstride, int mask, double *out,
                      long ostride, long fstride)
{
    GridTab &g = grid(c, q, p);
    SynJob j;
    j.coef = coef;
    j.L = g.L.d();
    j.out = out;
    j.cstride = cstride;
    j.ostride = ostride;
    j.fstride = fstride;
    j.p = p;
    j.q = q;
    j.ldn = ncoef(p);
    j.ncomp = ncomp;
    j.mask = mask;
    return j;
}

// Batched synthesis; the optional ranges z0[nz0], z1[nz1] are cleared by the
// same launch (stream-ordered before everything enqueued after it).
static void syn_run(Ctx &c, const std::vector<SynJob> &jobs, double *z0 = nullptr, long nz0 = 0,
                    double *z1 = nullptr, long nz1 = 0)
{
    if (jobs.empty()) {
        if (nz0 > 0) HIPC(hipMemsetAsync(z0, 0, nz0 * sizeof(double), c.stream));
        if (nz1 > 0) HIPC(hipMemsetAsync(z1, 0, nz1 * sizeof(double), c.stream));
        return;
    }
    double fl = 0.0, by = 0.0;
    for (auto &j : jobs) {
        const int nout = __builtin_popcount(j.mask);
        fl += (double)j.ncomp * (j.q + 1) * ncoef(j.p) * 4.0 * 2 + (double)j.ncomp * nout * npts(j.q) * (j.p + 1) * 4.0;
        by += (double)j.ncomp * (2.0 * ncoef(j.p) + nout * npts(j.q)) * 8.0;
    }
    ProfScope ps(c, "synthesis", fl, by);
    launch_synth_batch(c.stream, jobs.data(), (int)jobs.size(), z0, nz0, z1, nz1);
}

static void synth(Ctx &c, int p, int q, int nf, const double *coef, long cstride, int dt, int dp, double *out,
                  long ostride)
{
    int bit = 0;
    for (int b = 0; b < 6; ++b) {
        static const int kt[6] = {0, 1, 0, 2, 1, 0}, kp[6] = {0, 0, 1, 0, 1, 2};
        if (kt[b] == dt && kp[b] == dp) bit = b;
    }
    std::vector<SynJob> jobs;
    // more than 3 fields: one job per field (a job holds up to 3 components)
    for (int f = 0; f < nf; f += 3)
        jobs.push_back(syn_job(c, p, q, std::min(3, nf - f), coef + f * cstride, cstride, 1 << bit, out + f * ostride,
                               ostride, 0));
    syn_run(c, jobs);
}

static AnaJob ana_job(Ctx &c, int q, int p, int ncomp, const double *v, long vstride, double *coef, long cstride)
{
    GridTab &g = grid(c, q, p);
    AnaJob j;
    j.v = v;
    j.L = g.L.d();
    j.wq = g.wq.d();
    j.coef = coef;
    j.vstride = vstride;
    j.cstride = cstride;
    j.p = p;
    j.q = q;
    j.ldn = ncoef(p);
    j.ncomp = ncomp;
    j.cx = nullptr;
    j.csc = 0.0;
    return j;
}

static void ana_run(Ctx &c, const std::vector<AnaJob> &jobs)
{
    if (jobs.empty()) return;
    double fl = 0.0, by = 0.0;
    std::vector<AnaJob> fit;
    for (auto &j : jobs) {
        fl += (double)j.ncomp * ((j.q + 1) * ncoef(j.p) * 4.0 + (double)npts(j.q) * (j.p + 1) * 4.0);
        by += (double)j.ncomp * (2.0 * ncoef(j.p) + npts(j.q)) * 8.0;
        if (anal_batch_lds(j.p, j.q) <= 163840) {
            fit.push_back(j);
        } else {  // grids too large for one block's LDS: two-stage kernels
            GridTab &g = grid(c, j.q, j.p);
            c.Fbuf.ensure((size_t)j.ncomp * (j.q + 1) * (j.p + 1) * 2 * sizeof(double));
            launch_analyze(c.stream, j.q, j.p, j.p, g.L.d(), g.wq.d(), g.cs.d(), j.ncomp, j.v, j.vstride, c.Fbuf.d(),
                           j.coef, j.cstride);
        }
    }
    ProfScope ps(c, "analysis", fl, by);
    launch_anal_batch(c.stream, fit.data(), (int)fit.size());
}

static void analyze(Ctx &c, int q, int p, int nf, const double *v, long vstride, double *coef, long cstride)
{
    std::vector<AnaJob> jobs;
    for (int f = 0; f < nf; f += 3)
        jobs.push_back(ana_job(c, q, p, std::min(3, nf - f), v + f * vstride, vstride, coef + f * cstride, cstride));
    ana_run(c, jobs);
}

// per-drop offsets into the node and force synthesis buffers
static void syn_layout(const Ctx &c, std::vector<long> &o0, std::vector<long> &o1, std::vector<long> &og, long &tot)
{
    o0.resize(c.nd);
    o1.resize(c.nd);
    og.resize(c.nd);
    tot = 0;
    for (int i = 0; i < c.nd; ++i) {
        const Drop &d = c.drops[i];
        o0[i] = tot;
        tot += 9L * npts(d.p);
        o1[i] = tot;
        tot += 9L * npts(d.qu);
        og[i] = tot;
        tot += 21L * npts(d.qg);
    }
}

static void build_nodes(Ctx &c)
{
    if (c.nodes_ok) return;
    std::vector<long> o0, o1, og;
    long tot;
    syn_layout(c, o0, o1, og, tot);
    c.synbuf.ensure((size_t)tot * sizeof(double));
    c.vol.ensure(c.nd * sizeof(double));
    c.voloff_h.assign(c.nd + 1, 0);
    for (int i = 0; i < c.nd; ++i) c.voloff_h[i + 1] = c.voloff_h[i] + (npts(c.drops[i].p) + 63) / 64;
    c.volpart.ensure((size_t)c.voloff_h[c.nd] * sizeof(double));
    c.voloff.ensure((size_t)(c.nd + 1) * sizeof(int));
    HIPC(hipMemcpyAsync(c.voloff.ptr, c.voloff_h.data(), (c.nd + 1) * sizeof(int), hipMemcpyHostToDevice, c.stream));
    std::vector<SynJob> jobs;
    for (int i = 0; i < c.nd; ++i) {
        const Drop &d = c.drops[i];
        const double *x = c.xc.d() + d.coff;
        const long n0 = npts(d.p), n1 = npts(d.qu);
        jobs.push_back(syn_job(c, d.p, d.p, 3, x, c.Ctot, 0x7, c.synbuf.d() + o0[i], n0, 3 * n0));
        jobs.push_back(syn_job(c, d.p, d.qu, 3, x, c.Ctot, 0x7, c.synbuf.d() + o1[i], n1, 3 * n1));
    }
    syn_run(c, jobs);
    std::vector<NodeJob> nj;
    for (int i = 0; i < c.nd; ++i) {
        const Drop &d = c.drops[i];
        nj.push_back(NodeJob{c.synbuf.d() + o0[i], grid(c, d.p, d.p).wreg.d(), c.tx.d() + d.toff, c.s0N.d() + d.toff,
                             c.s0W.d() + d.toff, c.volpart.d() + c.voloff_h[i], c.T, d.p});
        nj.push_back(NodeJob{c.synbuf.d() + o1[i], grid(c, d.qu, d.p).wreg.d(), c.s1x.d() + d.uoff,
                             c.s1N.d() + d.uoff, c.s1W.d() + d.uoff, nullptr, c.S1, d.qu});
    }
    launch_nodes(c.stream, nj.data(), (int)nj.size());
    launch_vol_sum(c.stream, c.nd, c.volpart.d(), c.voloff.as<int>(), c.vol.d());
    c.nodes_ok = true;
}

static void build_force(Ctx &c)
{
    if (c.force_ok) return;
    std::vector<long> o0, o1, og;
    long tot;
    syn_layout(c, o0, o1, og, tot);
    c.synbuf.ensure((size_t)tot * sizeof(double));
    std::vector<SynJob> jobs;
    long fmax = 0;
    for (int i = 0; i < c.nd; ++i) {
        const Drop &d = c.drops[i];
        const long np = npts(d.qg);
        double *s = c.synbuf.d() + og[i];
        jobs.push_back(syn_job(c, d.p, d.qg, 3, c.xc.d() + d.coff, c.Ctot, 0x3f, s, np, 3 * np));
        if (c.eos != BIM_EOS_UNIFORM)
            jobs.push_back(syn_job(c, d.p, d.qg, 1, c.gc.d() + d.coff, 0, 0x7, s + 18 * np, 0, np));
        fmax += 3 * np;
    }
    syn_run(c, jobs);
    c.fgrid.ensure((size_t)fmax * sizeof(double));
    std::vector<AnaJob> ajobs;
    long fo = 0;
    for (int i = 0; i < c.nd; ++i) {
        const Drop &d = c.drops[i];
        const long np = npts(d.qg);
        launch_force(c.stream, (int)np, c.synbuf.d() + og[i], c.eos, c.E, c.xs, c.sigma0, c.fgrid.d() + fo);
        ajobs.push_back(ana_job(c, d.qg, d.p, 3, c.fgrid.d() + fo, np, c.fc.d() + d.coff, c.Ctot));
        fo += 3 * np;
    }
    ana_run(c, ajobs);
    c.force_ok = true;
}

// Regions and pair work lists (Sec. 2.3).
// Nearest-region items: closest points, interpolation points and their grids
// (one device pass), then the work list of the interpolation points against
// the source drop of each item (standard or upsampled grid).
static NearArgs near_args(Ctx &c)
{
    NearArgs a{};
    a.items = c.near_items.as<NearItem>();
    a.n = (int)c.near_h.size();
    a.dp = c.near_dp.as<int>();
    a.dcoff = c.near_dcoff.as<long>();
    a.dtoff = c.near_dtoff.as<int>();
    a.hj = c.hj.d();
    a.xc = c.xc.d();
    a.Ctot = c.Ctot;
    a.tx = c.tx.d();
    a.T = c.T;
    a.gl_t = c.near_glt.d();
    a.gl_off = c.near_gloff.as<int>();
    a.L = c.opt.near_L;
    a.A = c.opt.A_tilde;
    a.par = c.near_par.d();
    a.vx = c.near_vx.d();
    a.V = (long)a.n * a.L;
    a.vreg = c.near_vreg.as<int8_t>();
    a.Pst = c.near_Pst.d();
    a.ldp = c.near_ldp;
    return a;
}

// Work-item shape of the pair sums from the pairs of one application:
// targets per lane T of the whole tiles (2; 1 when even the shortest source
// runs would leave fewer than kPairItemsMin items, as for two drops of
// degree 32, where more, smaller items fill the chip better) and the
// sources per item: about kPairItemsTarget items per application (about 28
// wavefronts per SIMD: shorter items balance the tail better, down to where
// the per-item set-up and partial writes start to show), a multiple of 64
// between 64 and 4096. pair_ch > 0 fixes the sources per item.
constexpr double kPairItemsTarget = 28672.0, kPairItemsMin = 8192.0;
static void pair_shape(Ctx &c, double pairs, int &T, int &ch)
{
    T = c.pair_T_fix > 0 ? c.pair_T_fix : pairs / (64.0 * 2 * 64) < kPairItemsMin ? 1 : 2;
    if (c.pair_ch > 0) {
        ch = c.pair_ch;
        return;
    }
    long n = (long)std::ceil(pairs / (64.0 * T * kPairItemsTarget) / 64.0) * 64;
    ch = (int)std::min<long>(4096, std::max<long>(64, n));
}

// Targets of the next item of a target set with r targets left: a whole
// tile of 64 T targets while that many remain; a shorter tail as one ragged
// whole tile when its 64-target pieces would fill T of them anyway (r > 64
// (T - 1)), else as 64-target remainder items (whole = false).
static int pair_chunk(int T, int r, bool &whole)
{
    whole = r > 64 * (T - 1);
    return std::min(whole ? 64 * T : 64, r);
}

// Items of (target set, source range): whole tiles of 64 T targets, the rest
// in remainder items of one target per lane (flag kPairSmall), each split
// into runs of ch sources; appended to w.
static void pair_items(std::vector<PairWork> &w, int tl_off, int cnt, bool contig, long soff, int ns, int pair,
                       int grid, int T, int ch, double wt)
{
    for (int a = 0; a < cnt;) {
        bool whole = true;
        const int sz = pair_chunk(T, cnt - a, whole);
        for (int b = 0; b < ns; b += ch) {
            PairWork pw;
            pw.tlist_off = tl_off + a;
            pw.ntgt = sz;
            pw.src_off = (int)(soff + b);
            pw.nsrc = std::min(ch, ns - b);
            pw.pair = pair;
            pw.pad = grid | (contig ? kPairContig : 0) | (whole ? 0 : kPairSmall);
            pw.w = wt;
            w.push_back(pw);
        }
        a += sz;
    }
}

// Reduction lists of the items over nt targets (k_pair_gather), for partial
// blocks of 3 tile doubles per item, uploaded to g: an item over a
// contiguous tile k adds its base slot minus the tile's first target to tile
// k's list; an item over an index list adds the slot of each of its targets
// to that target's list. Both in item order.
template <class Items>
static void gather_lists(Ctx &c, const Items &items, const std::vector<int> &tl, long nt, bool tiles, int tile,
                         Ctx::Gather &g)
{
    REQUIRE((double)items.size() * 3 * tile < 2147483647.0, BIM_ENOMEM, "too many pair work items");
    const size_t ntile = tiles ? c.tile_start_h.size() : 0;
    g.nt = nt;
    g.h_toff.assign(ntile + 1, 0);
    g.h_off.assign(nt + 1, 0);
    for (const PairWork &w : items) {
        if (w.pad & kPairContig) {
            REQUIRE(tiles, BIM_EDEVICE, "contiguous pair item without target tiles");
            ++g.h_toff[c.tile_of_h[w.tlist_off] + 1];
        } else {
            for (int a = 0; a < w.ntgt; ++a) ++g.h_off[tl[w.tlist_off + a] + 1];
        }
    }
    for (size_t k = 0; k < ntile; ++k) g.h_toff[k + 1] += g.h_toff[k];
    for (long t = 0; t < nt; ++t) g.h_off[t + 1] += g.h_off[t];
    g.h_tent.resize(g.h_toff[ntile]);
    g.h_ent.resize(g.h_off[nt]);
    std::vector<int> tpos(g.h_toff.begin(), g.h_toff.end() - 1), pos(g.h_off.begin(), g.h_off.end() - 1);
    for (size_t it = 0; it < items.size(); ++it) {
        const PairWork &w = items[it];
        const int base = (int)it * 3 * tile;
        if (w.pad & kPairContig) {
            const int k = c.tile_of_h[w.tlist_off];
            REQUIRE(c.tile_start_h[k] == w.tlist_off, BIM_EDEVICE, "pair item not aligned to its target tile");
            g.h_tent[tpos[k]++] = base - w.tlist_off;
        } else {
            for (int a = 0; a < w.ntgt; ++a) g.h_ent[pos[tl[w.tlist_off + a]]++] = base + a;
        }
    }
    auto up = [&](DBuf &d, const HVec<int> &h) {
        d.ensure(std::max<size_t>(1, h.size()) * sizeof(int));
        if (!h.empty()) HIPC(hipMemcpyAsync(d.ptr, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice, c.stream));
    };
    up(g.toff, g.h_toff);
    up(g.tent, g.h_tent);
    up(g.off, g.h_off);
    up(g.ent, g.h_ent);
    c.pair_part.ensure(std::max<size_t>(1, items.size()) * 3 * tile * sizeof(double));
}

// Target tiles of each drop's consecutive targets, split as pair_items
// splits a contiguous target set.
static void target_tiles(Ctx &c, int T)
{
    c.tile_of_h.resize(std::max<long>(1, c.T));
    c.tile_start_h.clear();
    for (const Drop &d : c.drops) {
        const int nt = npts(d.p);
        for (int a = 0; a < nt;) {
            bool whole = true;
            const int sz = pair_chunk(T, nt - a, whole);
            c.tile_start_h.push_back((int)(d.toff + a));
            for (int b = a; b < a + sz; ++b) c.tile_of_h[d.toff + b] = (int)c.tile_start_h.size() - 1;
            a += sz;
        }
    }
    c.tile_of.ensure(c.tile_of_h.size() * sizeof(int));
    HIPC(hipMemcpyAsync(c.tile_of.ptr, c.tile_of_h.data(), c.tile_of_h.size() * sizeof(int), hipMemcpyHostToDevice,
                        c.stream));
}

static void near_setup(Ctx &c)
{
    c.near_src.assign(c.nd, 0);
    c.near_nwork = 0;
    c.near_pairs = 0.0;
    const int n = (int)c.near_h.size();
    if (n == 0) return;
    for (const NearItem &it : c.near_h) c.near_src[it.j] = 1;
    const int L = c.opt.near_L;
    const long V = (long)n * L;
    int pmax = 0;
    std::vector<int> dp(c.nd), dtoff(c.nd), gloff(c.nd);
    std::vector<long> dcoff(c.nd);
    std::vector<double> glt;
    for (int i = 0; i < c.nd; ++i) {
        const Drop &d = c.drops[i];
        dp[i] = d.p;
        dtoff[i] = (int)d.toff;
        dcoff[i] = d.coff;
        gloff[i] = (int)glt.size();
        GridTab &g = grid(c, d.p, d.p);
        glt.insert(glt.end(), g.t.begin(), g.t.end());
        pmax = std::max(pmax, d.p);
    }
    REQUIRE(pmax <= 63, BIM_EINVAL, "the nearest-region rule supports degrees up to 63");
    c.near_ldp = ncoef(pmax);
    c.near_items.ensure(n * sizeof(NearItem));
    c.near_dp.ensure(c.nd * sizeof(int));
    c.near_dtoff.ensure(c.nd * sizeof(int));
    c.near_gloff.ensure(c.nd * sizeof(int));
    c.near_dcoff.ensure(c.nd * sizeof(long));
    c.near_glt.ensure(glt.size() * sizeof(double));
    c.near_par.ensure((size_t)n * 4 * sizeof(double));
    c.near_vx.ensure((size_t)3 * V * sizeof(double));
    c.near_vreg.ensure((size_t)V);
    c.near_Pst.ensure((size_t)n * c.near_ldp * sizeof(double));
    c.near_vacc.ensure((size_t)3 * V * sizeof(double));
    c.near_self.ensure((size_t)3 * c.T * sizeof(double));
    c.near_selfc.ensure((size_t)3 * c.Ctot * sizeof(double));
    HIPC(hipMemcpyAsync(c.near_items.ptr, c.near_h.data(), n * sizeof(NearItem), hipMemcpyHostToDevice, c.stream));
    HIPC(hipMemcpyAsync(c.near_dp.ptr, dp.data(), c.nd * sizeof(int), hipMemcpyHostToDevice, c.stream));
    HIPC(hipMemcpyAsync(c.near_dtoff.ptr, dtoff.data(), c.nd * sizeof(int), hipMemcpyHostToDevice, c.stream));
    HIPC(hipMemcpyAsync(c.near_gloff.ptr, gloff.data(), c.nd * sizeof(int), hipMemcpyHostToDevice, c.stream));
    HIPC(hipMemcpyAsync(c.near_dcoff.ptr, dcoff.data(), c.nd * sizeof(long), hipMemcpyHostToDevice, c.stream));
    HIPC(hipMemcpyAsync(c.near_glt.ptr, glt.data(), glt.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
    launch_near_setup(c.stream, near_args(c));
    std::vector<int8_t> vreg(V);
    HIPC(hipMemcpyAsync(vreg.data(), c.near_vreg.ptr, V, hipMemcpyDeviceToHost, c.stream));
    HIPC(hipStreamSynchronize(c.stream));
    // work list: interpolation points grouped by (source drop, grid)
    std::vector<int> tl;
    std::vector<PairWork> w;
    std::vector<std::pair<int, int>> runs;  // (start in tl, count) per (source drop, grid)
    double npairs = 0.0;
    for (int j = 0; j < c.nd; ++j) {
        if (!c.near_src[j]) continue;
        const Drop &dj = c.drops[j];
        for (int g = 0; g < 2; ++g) {
            const int start = (int)tl.size();
            for (int it = 0; it < n; ++it) {
                if (c.near_h[it].j != j) continue;
                for (int l = 0; l < L; ++l)
                    if (vreg[(long)it * L + l] == g) tl.push_back(it * L + l);
            }
            runs.emplace_back(start, (int)tl.size() - start);
            npairs += (double)runs.back().second * (g == 0 ? npts(dj.p) : npts(dj.qu));
        }
    }
    int Tn = 1, CH = 64;
    pair_shape(c, npairs, Tn, CH);
    size_t r = 0;
    for (int j = 0; j < c.nd; ++j) {
        if (!c.near_src[j]) continue;
        const Drop &dj = c.drops[j];
        for (int g = 0; g < 2; ++g, ++r) {
            const long soff = g == 0 ? dj.toff : dj.uoff;
            const int ns = g == 0 ? npts(dj.p) : npts(dj.qu);
            pair_items(w, runs[r].first, runs[r].second, false, soff, ns, j, g, 1, CH, 1.0);
        }
    }
    for (const PairWork &pw : w) c.near_pairs += (double)pw.ntgt * pw.nsrc;
    c.near_tl.ensure(std::max<size_t>(1, tl.size()) * sizeof(int));
    c.near_work.ensure(std::max<size_t>(1, w.size()) * sizeof(PairWork));
    if (!tl.empty())
        HIPC(hipMemcpyAsync(c.near_tl.ptr, tl.data(), tl.size() * sizeof(int), hipMemcpyHostToDevice, c.stream));
    if (!w.empty())
        HIPC(hipMemcpyAsync(c.near_work.ptr, w.data(), w.size() * sizeof(PairWork), hipMemcpyHostToDevice, c.stream));
    gather_lists(c, w, tl, V, false, 64, c.near_g);
    {
        // each item's interpolated value goes to its grid target, items in order
        Ctx::Gather &g = c.near_tg;
        g.nt = c.T;
        g.h_off.assign(c.T + 1, 0);
        for (const NearItem &it : c.near_h) ++g.h_off[it.t + 1];
        for (long t = 0; t < c.T; ++t) g.h_off[t + 1] += g.h_off[t];
        g.h_ent.resize(n);
        std::vector<int> pos(g.h_off.begin(), g.h_off.end() - 1);
        for (int it = 0; it < n; ++it) g.h_ent[pos[c.near_h[it].t]++] = it;
        g.off.ensure((c.T + 1) * sizeof(int));
        g.ent.ensure(std::max<size_t>(1, n) * sizeof(int));
        HIPC(hipMemcpyAsync(g.off.ptr, g.h_off.data(), (c.T + 1) * sizeof(int), hipMemcpyHostToDevice, c.stream));
        HIPC(hipMemcpyAsync(g.ent.ptr, g.h_ent.data(), n * sizeof(int), hipMemcpyHostToDevice, c.stream));
        c.near_res.ensure((size_t)3 * n * sizeof(double));
    }
    HIPC(hipStreamSynchronize(c.stream));
    c.near_nwork = (int)w.size();
}

// Device side of the fast-summation plan built by build_regions: job and
// centre arrays, work buffers, and the regular harmonics of every source
// grid's nodes about its centre (fixed while the geometry is).
static void fmm_setup(Ctx &c, const std::vector<double> &cb0, const std::vector<double> &cb1)
{
    Ctx::Fmm &F = c.fmm;
    const int P = F.P, ntri = (P + 1) * (P + 2) / 2;
    std::vector<double> cs(4 * F.src.size()), ct(4 * F.tgt.size());
    for (auto &sj : F.src) {
        const bool up = sj.x == c.s1x.d();
        for (int k = 0; k < 4; ++k) cs[4 * sj.slot + k] = (up ? cb1 : cb0)[4 * sj.drop + k];
        sj.yoff = F.nsrc * ntri;
        sj.woff = F.nsrc * 12;
        sj.pbase = (int)F.nchunks;
        F.nsrc += sj.ns;
        F.nchunks += (sj.ns + kFmmChunk - 1) / kFmmChunk;
        F.maxns = std::max(F.maxns, sj.ns);
    }
    for (auto &tj : F.tgt) {
        int i = 0;
        while (c.drops[i].toff != tj.off) ++i;
        for (int k = 0; k < 4; ++k) ct[4 * tj.slot + k] = cb0[4 * i + k];
        F.ntgt += tj.n;
        F.maxnt = std::max(F.maxnt, tj.n);
    }
    F.poff.push_back((int)F.pairs.size());
    const size_t cb = (size_t)4 * ntri * sizeof(double2);
    F.dsrc.ensure(F.src.size() * sizeof(FmmSrcJob));
    F.dtgt.ensure(F.tgt.size() * sizeof(FmmTgtJob));
    F.dpoff.ensure(F.poff.size() * sizeof(int));
    F.cen_s.ensure(cs.size() * sizeof(double));
    F.cen_t.ensure(ct.size() * sizeof(double));
    const bool f32 = c.opt.precision == BIM_PREC_MIXED;
    F.Y.ensure((size_t)F.nsrc * ntri * (f32 ? sizeof(float2) : sizeof(double2)));
    F.W.ensure((size_t)F.nsrc * 12 * sizeof(double));
    F.part.ensure((size_t)F.nchunks * cb);
    F.M.ensure(F.src.size() * 4 * (P + 1) * (P + 1) * sizeof(double2));
    F.Lp.ensure(F.pairs.size() * cb);
    F.L.ensure(F.tgt.size() * cb);
    F.C.ensure(F.tgt.size() * ntri * 15 * sizeof(double2));
    HIPC(hipMemcpyAsync(F.dsrc.ptr, F.src.data(), F.src.size() * sizeof(FmmSrcJob), hipMemcpyHostToDevice, c.stream));
    HIPC(hipMemcpyAsync(F.dtgt.ptr, F.tgt.data(), F.tgt.size() * sizeof(FmmTgtJob), hipMemcpyHostToDevice, c.stream));
    HIPC(hipMemcpyAsync(F.dpoff.ptr, F.poff.data(), F.poff.size() * sizeof(int), hipMemcpyHostToDevice, c.stream));
    HIPC(hipMemcpyAsync(F.cen_s.ptr, cs.data(), cs.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
    HIPC(hipMemcpyAsync(F.cen_t.ptr, ct.data(), ct.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
    launch_fmm_ytab(c.stream, F.dsrc.as<FmmSrcJob>(), (int)F.src.size(), F.maxns, P, F.cen_s.d(), F.Y.ptr, f32);
    HIPC(hipStreamSynchronize(c.stream));
}

// Work lists of the pair sums for fast-summation order P (0: every pair
// summed directly): the direct items of both grids, the nearest-region items
// and the fast-summation plan. cb0, cb1: centres and bounding radii of the
// standard and upsampled nodes of every drop (read when P > 0).
static void build_lists(Ctx &c, int P, const std::vector<double> &cb0, const std::vector<double> &cb1)
{
    // far drop pairs for the fast summation: every target of i in the same
    // region (0 or 1) with respect to j, and the truncation bound
    // rho^(P+1) <= eps, rho = (a_i + a_j) / |c_i - c_j| (bounding radii of the
    // target nodes and of the source grid the region selects)
    // grid of a far pair (-1: summed directly); order: the smallest degree
    // Q <= P with rho^(Q+1) <= eps, used by that pair's translation
    // uni[i * nd + j]: the region shared by all targets of i with respect to
    // j, or -4 (one sweep over the regions in memory order)
    std::vector<int8_t> uni;
    {
        uni.resize((size_t)c.nd * c.nd);
        for (int i = 0; i < c.nd; ++i) {
            const Drop &di = c.drops[i];
            int8_t *u = &uni[(size_t)i * c.nd];
            const int8_t *row = &c.reg_h[di.toff * c.nd];
            for (int j = 0; j < c.nd; ++j) u[j] = row[j];
            for (int t = 1; t < npts(di.p); ++t) {
                row = &c.reg_h[(di.toff + t) * c.nd];
                for (int j = 0; j < c.nd; ++j) u[j] = row[j] == u[j] ? u[j] : (int8_t)-4;
            }
        }
    }
    auto far_grid = [&](int i, int j, int &order) -> int {
        if (P <= 0) return -1;
        const int8_t r0 = uni[(size_t)i * c.nd + j];
        if (r0 != 0 && r0 != 1) return -1;
        const double *cs = (r0 == 0 ? cb0.data() : cb1.data()) + 4 * j, *ct = cb0.data() + 4 * i;
        const double D = std::sqrt((ct[0] - cs[0]) * (ct[0] - cs[0]) + (ct[1] - cs[1]) * (ct[1] - cs[1]) +
                                   (ct[2] - cs[2]) * (ct[2] - cs[2]));
        const double rho = (cs[3] + ct[3]) / D;
        if (!(rho < 1.0 && std::pow(rho, P + 1) <= c.opt.fmm_eps)) return -1;
        order = 2;
        while (order < P && std::pow(rho, order + 1) > c.opt.fmm_eps) ++order;
        return r0;
    };
    Ctx::Fmm &F = c.fmm;
    F.reset(P);
    std::map<std::pair<int, int>, int> sslot;
    std::map<int, int> tslot;
    // work lists: for each (target drop i, source drop j != i): Omega_0 targets
    // against j's standard grid, Omega_1/2 targets against j's upsampled grid
    std::vector<int> tl, k0, k1;
    std::vector<PairWork> w0, w1;
    std::vector<NearItem> near;
    // (target set, source range) segments, split into work items once the
    // total pair count (and with it the items' source run) is known
    struct Seg {
        int tl_off, cnt;
        bool contig;
        long soff;
        int ns, pair, grid;
    };
    std::vector<Seg> segs;
    double npairs = 0.0;
    c.n_om1 = c.n_om2 = 0;
    for (int i = 0; i < c.nd; ++i) {
        const Drop &di = c.drops[i];
        const int nti = npts(di.p);
        for (int j = 0; j < c.nd; ++j) {
            if (j == i || c.sys_h[i] != c.sys_h[j]) continue;
            const Drop &dj = c.drops[j];
            int forder = 0;
            const int fg = far_grid(i, j, forder);
            if (fg >= 0) {
                if (fg == 1) c.n_om1 += nti;
                const auto ks = std::make_pair(j, fg);
                if (!sslot.count(ks)) {
                    const int sl = (int)F.src.size();
                    sslot[ks] = sl;
                    FmmSrcJob sj{};
                    sj.x = fg == 0 ? c.tx.d() : c.s1x.d();
                    sj.d = fg == 0 ? c.s0d.d() : c.s1d.d();
                    sj.wW = fg == 0 ? c.s0W.d() : c.s1W.d();
                    sj.wN = fg == 0 ? c.s0N.d() : c.s1N.d();
                    sj.stride = fg == 0 ? c.T : c.S1;
                    sj.off = fg == 0 ? dj.toff : dj.uoff;
                    sj.ns = fg == 0 ? npts(dj.p) : npts(dj.qu);
                    sj.slot = sl;
                    sj.drop = j;
                    F.src.push_back(sj);
                }
                if (!tslot.count(i)) {
                    const int sl = (int)F.tgt.size();
                    tslot[i] = sl;
                    F.tgt.push_back(FmmTgtJob{di.toff, nti, sl});
                    F.poff.push_back((int)F.pairs.size());
                }
                F.pairs.push_back(FmmPair{sslot[ks], tslot[i], forder, 0, 0.0});
                const double nt = (forder + 1) * (forder + 2) / 2;
                F.m2l_flops += nt * (forder + 1) * (forder + 1) * 32.0;
                F.pair_ij.push_back(i * c.nd + j);
                continue;
            }
            const int8_t ru = uni[(size_t)i * c.nd + j];
            if (ru == 0 || ru == 1) {
                // every target of i in one region: items over the contiguous
                // target range, no index list
                if (ru == 1) c.n_om1 += nti;
                const long soff = ru == 0 ? dj.toff : dj.uoff;
                const int ns = ru == 0 ? npts(dj.p) : npts(dj.qu);
                segs.push_back(Seg{(int)di.toff, nti, true, soff, ns, i * c.nd + j, ru});
                npairs += (double)nti * ns;
                continue;
            }
            // one pass over i's targets: region 0 to the standard grid, 1 (and 2 by
            // the Omega_1 rule) to the upsampled grid, 2 by the special rule to the
            // nearest-region items
            k0.clear();
            k1.clear();
            for (int t = 0; t < nti; ++t) {
                const int8_t r = c.reg_h[(di.toff + t) * c.nd + j];
                const int tg = (int)(di.toff + t);
                if (r == 0) {
                    k0.push_back(tg);
                    continue;
                }
                if (r == 1) ++c.n_om1;
                if (r == 2) ++c.n_om2;
                if (r == 2 && c.opt.near_rule == 1)
                    near.push_back(NearItem{tg, i, j, 0});
                else
                    k1.push_back(tg);
            }
            for (int kind = 0; kind < 2; ++kind) {
                const int start = (int)tl.size();
                const std::vector<int> &kl = kind == 0 ? k0 : k1;
                tl.insert(tl.end(), kl.begin(), kl.end());
                const int cnt = (int)kl.size();
                const long soff = kind == 0 ? dj.toff : dj.uoff;
                const int ns = kind == 0 ? npts(dj.p) : npts(dj.qu);
                if (cnt == 0) continue;
                segs.push_back(Seg{start, cnt, false, soff, ns, i * c.nd + j, kind});
                npairs += (double)cnt * ns;
            }
        }
    }
    int CH = 64;
    pair_shape(c, npairs, c.pair_T, CH);
    c.npairs_direct = npairs;
    target_tiles(c, c.pair_T);
    for (const Seg &g : segs)
        pair_items(g.grid == 0 ? w0 : w1, g.tl_off, g.cnt, g.contig, g.soff, g.ns, g.pair, g.grid, c.pair_T, CH, 0.0);
    c.tlist.ensure(std::max<size_t>(1, tl.size()) * sizeof(int));
    if (!tl.empty())
        HIPC(hipMemcpyAsync(c.tlist.ptr, tl.data(), tl.size() * sizeof(int), hipMemcpyHostToDevice, c.stream));
    HIPC(hipStreamSynchronize(c.stream));
    c.tlist_h = std::move(tl);
    if (!F.pairs.empty()) fmm_setup(c, cb0, cb1);
    c.w0h = std::move(w0);
    c.w1h = std::move(w1);
    for (auto &e : c.wlists) e->stale = true;
    c.near_h = std::move(near);
}

static void run_pairs(Ctx &c, int kind, const std::vector<double> &wt);

// Order of the fast summation chosen by timing (fmm_order = -1): the
// double-layer pair pass (direct items plus fast summation, unit weights)
// is timed with events at each candidate order and with every pair direct;
// the fastest wins. For a given fmm_eps every far pair meets the same
// truncation bound at any order, so the choice changes the cost, not the
// accuracy. The accumulator is cleared afterwards.
static int tune_fmm(Ctx &c, const std::vector<double> &cb0, const std::vector<double> &cb1)
{
    static const int cand[] = {0, 8, 12, 16, 20, 24, 30};
    const std::vector<double> ones((size_t)c.nd * c.nd, 1.0);
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    int best = 0;
    float tbest = 0.0f;
    for (int P : cand) {
        build_lists(c, P, cb0, cb1);
        if (P > 0 && c.fmm.pairs.empty()) continue;  // no far pair at this order: the same as direct
        run_pairs(c, 1, ones);  // warm-up
        HIPC(hipEventRecord(e0, c.stream));
        run_pairs(c, 1, ones);
        HIPC(hipEventRecord(e1, c.stream));
        HIPC(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIPC(hipEventElapsedTime(&ms, e0, e1));
        if (P == 0 || ms < tbest) {
            tbest = ms;
            best = P;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPC(hipMemsetAsync(c.acc.ptr, 0, (size_t)3 * c.T * sizeof(double), c.stream));
    return best;
}

// Work-item shape of the pair sums chosen by timing (option pair_tune):
// targets per lane T in {1, 2, 4} and sources per item ch in {ch0/2, ch0,
// 2 ch0} (ch0 the pair-count rule's choice for that T), double-layer pair
// passes (unit weights, after a warm-up pass) timed with HIP events on the
// context stream, two rounds over the candidates, the faster of each
// candidate's two counted. The rule's own shape is kept unless a candidate
// beats it by more than kTuneMargin (a single pass varies by a few percent
// run to run; a smaller gain is not worth a shape chosen on noise). The
// choice depends on the
// problem's shape only, so it is cached for the process under (direct pairs
// of an application to two significant digits, targets, order of the fast
// summation): later contexts of the same shape reuse it without timing, and
// contexts that time the same shape concurrently all adopt the first result
// stored, so results in one process do not depend on which context tuned.
struct PairShapeKey {
    long mant, targets;  // pairs = mant 10^expo, mant in [10, 99]
    int expo, P;
    bool operator<(const PairShapeKey &o) const
    {
        return std::tie(mant, expo, targets, P) < std::tie(o.mant, o.expo, o.targets, o.P);
    }
};
static std::mutex g_shape_mu;
static std::map<PairShapeKey, std::pair<int, int>> g_shapes;
constexpr float kTuneMargin = 0.03f;

static void tune_pairs(Ctx &c, int P, const std::vector<double> &cb0, const std::vector<double> &cb1)
{
    c.pair_T_fix = 0;
    c.pair_ch = 0;
    build_lists(c, P, cb0, cb1);
    c.pair_tuned = true;
    if (c.npairs_direct <= 0.0) return;
    const int expo = (int)std::floor(std::log10(c.npairs_direct)) - 1;
    const PairShapeKey key{(long)std::llround(c.npairs_direct / std::pow(10.0, expo)), c.T, expo, P};
    {
        std::lock_guard<std::mutex> lk(g_shape_mu);
        auto it = g_shapes.find(key);
        if (it != g_shapes.end()) {
            c.pair_T_fix = it->second.first;
            c.pair_ch = it->second.second;
            return;
        }
    }
    const std::vector<double> ones((size_t)c.nd * c.nd, 1.0);
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    int rT = 0, rch = 0;  // the rule's shape
    c.pair_T_fix = 0;
    c.pair_ch = 0;
    pair_shape(c, c.npairs_direct, rT, rch);
    std::vector<std::pair<int, int>> cand;
    for (int T : {4, 2, 1}) {
        int T0 = T, ch0 = 64;
        c.pair_T_fix = T;
        c.pair_ch = 0;
        pair_shape(c, c.npairs_direct, T0, ch0);
        for (int ch : {ch0 / 2, ch0, 2 * ch0}) {
            ch = std::min(4096, std::max(64, ch / 64 * 64));
            if (std::find(cand.begin(), cand.end(), std::make_pair(T, ch)) == cand.end()) cand.emplace_back(T, ch);
        }
    }
    if (std::find(cand.begin(), cand.end(), std::make_pair(rT, rch)) == cand.end()) cand.emplace_back(rT, rch);
    std::vector<float> best(cand.size(), 0.0f);
    for (int round = 0; round < 2; ++round)
        for (size_t k = 0; k < cand.size(); ++k) {
            c.pair_T_fix = cand[k].first;
            c.pair_ch = cand[k].second;
            build_lists(c, P, cb0, cb1);
            if (round == 0) run_pairs(c, 1, ones);  // warm-up
            HIPC(hipEventRecord(e0, c.stream));
            run_pairs(c, 1, ones);
            HIPC(hipEventRecord(e1, c.stream));
            HIPC(hipEventSynchronize(e1));
            float ms = 0.0f;
            HIPC(hipEventElapsedTime(&ms, e0, e1));
            best[k] = round == 0 ? ms : std::min(best[k], ms);
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPC(hipMemsetAsync(c.acc.ptr, 0, (size_t)3 * c.T * sizeof(double), c.stream));
    size_t kr = std::find(cand.begin(), cand.end(), std::make_pair(rT, rch)) - cand.begin(), kb = kr;
    for (size_t k = 0; k < cand.size(); ++k)
        if (best[k] < best[kb]) kb = k;
    if (!(best[kb] < (1.0f - kTuneMargin) * best[kr])) kb = kr;
    const int bestT = cand[kb].first, bestch = cand[kb].second;
    std::lock_guard<std::mutex> lk(g_shape_mu);
    const auto it = g_shapes.emplace(key, std::make_pair(bestT, bestch)).first;  // the first stored wins
    c.pair_T_fix = it->second.first;
    c.pair_ch = it->second.second;
}

static void build_regions(Ctx &c)
{
    if (c.regions_ok) return;
    build_nodes(c);
    // grid spacings from the volumes on the device; the volume check is read
    // back with the regions (or on its own when there are no drop pairs)
    c.hj.ensure(c.nd * sizeof(double));
    c.hbad.ensure(sizeof(int));
    launch_drop_h(c.stream, c.nd, c.vol.d(), c.hfac.d(), c.hj.d(), c.hbad.as<int>());
    int bad = 0;
    auto check_volumes = [&]() {
        if (!bad) return;
        std::vector<double> vol(c.nd);
        HIPC(hipMemcpyAsync(vol.data(), c.vol.ptr, c.nd * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        HIPC(hipStreamSynchronize(c.stream));
        for (int i = 0; i < c.nd; ++i)
            REQUIRE(vol[i] > 0.0 && std::isfinite(vol[i]), BIM_EINVAL,
                    "drop " + std::to_string(i) + " has non-positive volume");
    };
    const long nreg = c.T * c.nd;
    c.reg.ensure(nreg);
    c.dist.ensure(nreg * sizeof(double));
    c.cbnd.ensure(4 * c.nd * sizeof(double));
    c.clist.ensure(std::max<long>(1, nreg) * sizeof(int));
    c.ccount.ensure(sizeof(int));
    {
        ProfScope ps(c, "classify", 0.0, 0.0);
        launch_drop_bounds(c.stream, c.nd, c.tx.d(), c.T, c.noff.as<int>(), c.ncnt.as<int>(), c.cbnd.d());
        if (c.opt.fmm_order != 0) {
            c.cbnd1.ensure(4 * c.nd * sizeof(double));
            launch_drop_bounds(c.stream, c.nd, c.s1x.d(), c.S1, c.unoff.as<int>(), c.uncnt.as<int>(), c.cbnd1.d());
        }
        HIPC(hipMemsetAsync(c.ccount.ptr, 0, sizeof(int), c.stream));
        launch_classify_bound(c.stream, (int)c.T, c.nd, c.tx.d(), c.T, c.tdrop.as<int>(), c.sysd.as<int>(),
                              c.cbnd.d(), c.hj.d(),
                              c.opt.A_tilde, c.regions_exact ? 1 : 0, c.reg.as<int8_t>(), c.dist.d(),
                              c.clist.as<int>(), c.ccount.as<int>());
    }
    // drops that interact (two drops of one system); without any, the bound
    // kernel has already written every region (own drop -1, other system -2)
    // and there is nothing to scan or to list
    bool pairs = false;
    for (int i = 0; i < c.nd && !pairs; ++i)
        for (int j = i + 1; j < c.nd; ++j)
            if (c.sys_h[i] == c.sys_h[j]) {
                pairs = true;
                break;
            }
    if (pairs) {
        {
            ProfScope ps(c, "classify", 0.0, 0.0);
            launch_classify_scan(c.stream, c.ccount.as<int>(), nreg, c.clist.as<int>(), c.nd, c.tx.d(), c.T, c.tx.d(),
                                 c.T, c.noff.as<int>(), c.ncnt.as<int>(), c.hj.d(), c.opt.A_tilde,
                                 c.reg.as<int8_t>(), c.dist.d());
        }
        c.reg_h.resize(nreg);
        HIPC(hipMemcpyAsync(c.reg_h.data(), c.reg.ptr, nreg, hipMemcpyDeviceToHost, c.stream));
        HIPC(hipMemcpyAsync(&bad, c.hbad.ptr, sizeof(int), hipMemcpyDeviceToHost, c.stream));
        HIPC(hipStreamSynchronize(c.stream));
    } else {
        c.reg_h.assign(nreg, -1);  // not read without pairs
        HIPC(hipMemcpyAsync(&bad, c.hbad.ptr, sizeof(int), hipMemcpyDeviceToHost, c.stream));
        HIPC(hipStreamSynchronize(c.stream));
    }
    check_volumes();
    std::vector<double> cb0, cb1;
    if (c.opt.fmm_order != 0 && pairs) {
        cb0.resize(4 * c.nd);
        cb1.resize(4 * c.nd);
        HIPC(hipMemcpyAsync(cb0.data(), c.cbnd.ptr, cb0.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        HIPC(hipMemcpyAsync(cb1.data(), c.cbnd1.ptr, cb1.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        HIPC(hipStreamSynchronize(c.stream));
    }
    int P = pairs ? c.opt.fmm_order : 0;
    if (P < 0) {
        if (c.fmm_tuned < 0) c.fmm_tuned = tune_fmm(c, cb0, cb1);
        P = c.fmm_tuned;
    }
    if (c.opt.pair_tune && pairs && !c.pair_tuned) tune_pairs(c, P, cb0, cb1);
    build_lists(c, P, cb0, cb1);
    near_setup(c);
    c.regions_ok = true;
}

// Device work lists for a weight table wt[i * nd + j] (items of zero weight
// dropped), cached per table.
static Ctx::WList &work_lists(Ctx &c, const std::vector<double> &wt)
{
    for (auto &e : c.wlists)
        if (!e->stale && e->wt == wt) return *e;
    // refill a stale list (the one of this table if there is one): its
    // device buffers and pinned host images are kept, so a new evaluation
    // of the same drops allocates and frees nothing here
    Ctx::WList *e = nullptr;
    for (auto &x : c.wlists)
        if (x->stale && (!e || x->wt == wt)) e = x.get();
    if (!e) {
        c.wlists.push_back(std::make_unique<Ctx::WList>());
        e = c.wlists.back().get();
    }
    e->stale = false;
    e->wt = wt;
    e->pairs = 0.0;
    HVec<PairWork> &keep = e->h_items;
    keep.clear();
    keep.reserve(c.w0h.size() + c.w1h.size());
    for (int small = 0; small < 2; ++small) {  // whole-tile items first, then the remainders
        for (int u = 0; u < 2; ++u)
            for (PairWork pw : (u == 0 ? c.w0h : c.w1h)) {
                if (((pw.pad & kPairSmall) != 0) != (small != 0)) continue;
                pw.w = wt[pw.pair];
                if (pw.w != 0.0) {
                    keep.push_back(pw);
                    e->pairs += (double)pw.ntgt * pw.nsrc;
                }
            }
    }
    e->d.ensure(std::max<size_t>(1, keep.size()) * sizeof(PairWork));
    if (!keep.empty())
        HIPC(hipMemcpyAsync(e->d.ptr, keep.data(), keep.size() * sizeof(PairWork), hipMemcpyHostToDevice, c.stream));
    e->n = (int)keep.size();
    gather_lists(c, keep, c.tlist_h, c.T, true, 64 * c.pair_T, e->g);
    if (!c.near_h.empty()) {
        HVec<double> &nw = e->h_nw;
        nw.resize(c.near_h.size());
        for (size_t it = 0; it < nw.size(); ++it) nw[it] = wt[(size_t)c.near_h[it].i * c.nd + c.near_h[it].j];
        e->nw.ensure(nw.size() * sizeof(double));
        HIPC(hipMemcpyAsync(e->nw.ptr, nw.data(), nw.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
    }
    if (!c.fmm.pairs.empty()) {
        HVec<FmmPair> &fp = e->h_fp;
        fp.assign(c.fmm.pairs.begin(), c.fmm.pairs.end());
        for (size_t k = 0; k < fp.size(); ++k) fp[k].w = wt[c.fmm.pair_ij[k]];
        e->fp.ensure(fp.size() * sizeof(FmmPair));
        HIPC(hipMemcpyAsync(e->fp.ptr, fp.data(), fp.size() * sizeof(FmmPair), hipMemcpyHostToDevice, c.stream));
    }
    return *e;
}

// Far drop pairs by the fast summation (plan of build_regions), added into
// acc: per-source weights and multipoles of every source grid, one
// translation per pair with its weight, the local expansions summed per
// target drop, then evaluated at its nodes.
static void run_fmm(Ctx &c, int kind, Ctx::WList &L)
{
    Ctx::Fmm &F = c.fmm;
    if (F.pairs.empty()) return;
    const int P = F.P;
    const double ntri = (P + 1) * (P + 2) / 2;
    // algorithmic flops: P2M 8 (SL) or 48 (DL) per source and coefficient;
    // M2L 32 per coefficient pair at the pair's order (4 channels, complex);
    // L2P 60 per target and coefficient
    const double fl = (double)F.nsrc * ntri * (kind == 0 ? 8.0 : 48.0) + F.m2l_flops + (double)F.ntgt * ntri * 60.0;
    ProfScope ps(c, "fmm", fl, 0.0);
    launch_fmm_p2m(c.stream, F.dsrc.as<FmmSrcJob>(), (int)F.src.size(), F.maxns, kind, P, F.cen_s.d(), F.Y.ptr,
                   c.opt.precision == BIM_PREC_MIXED, F.W.d(), (double2 *)F.part.ptr, (double2 *)F.M.ptr);
    launch_fmm_m2l(c.stream, (int)F.pairs.size(), L.fp.as<FmmPair>(), P, F.cen_s.d(), F.cen_t.d(),
                   (const double2 *)F.M.ptr, (double2 *)F.Lp.ptr, (int)F.tgt.size(), F.dpoff.as<int>(),
                   (double2 *)F.L.ptr);
    launch_fmm_l2p(c.stream, (int)F.tgt.size(), F.dtgt.as<FmmTgtJob>(), F.maxnt, P, F.cen_t.d(),
                   (const double2 *)F.L.ptr, (double2 *)F.C.ptr, c.tx.d(), c.T, c.acc.d(), c.T);
}

// Pair sums with weight table wt, added into acc: one launch over the items
// of both source grids.
// FP32 source records of both grids for the mixed form (every drop's nodes,
// relative to its centre), from the current densities.
static void pack32(Ctx &c, int kind, const PairSrc &g0, const PairSrc &g1)
{
    if (c.pack_h.empty()) {
        for (int g = 0; g < 2; ++g)
            for (int j = 0; j < c.nd; ++j) {
                const Drop &d = c.drops[j];
                const int n = g == 0 ? npts(d.p) : npts(d.qu);
                c.pack_h.push_back(PackJob{g == 0 ? d.toff : d.uoff, n, j});
                (g == 0 ? c.pack_max0 : c.pack_max1) = std::max(g == 0 ? c.pack_max0 : c.pack_max1, n);
            }
        c.pack_n0 = c.pack_n1 = c.nd;
        c.pack_jobs.ensure(c.pack_h.size() * sizeof(PackJob));
        HIPC(hipMemcpyAsync(c.pack_jobs.ptr, c.pack_h.data(), c.pack_h.size() * sizeof(PackJob),
                            hipMemcpyHostToDevice, c.stream));
        c.rec32_0.ensure((size_t)std::max<long>(1, c.T) * 3 * sizeof(float4));
        c.rec32_1.ensure((size_t)std::max<long>(1, c.S1) * 3 * sizeof(float4));
    }
    launch_pair_pack32(c.stream, kind, c.pack_jobs.as<PackJob>(), c.pack_n0, c.pack_max0, g0, c.cbnd.d(),
                       c.rec32_0.as<float4>());
    launch_pair_pack32(c.stream, kind, c.pack_jobs.as<PackJob>() + c.pack_n0, c.pack_n1, c.pack_max1, g1, c.cbnd.d(),
                       c.rec32_1.as<float4>());
}

static void run_pairs(Ctx &c, int kind, const std::vector<double> &wt)
{
    Ctx::WList &L = work_lists(c, wt);
    const double fpp = kind == 0 ? 29.0 : 30.0;  // flops per pair (SL / DL)
    const PairSrc g0{c.tx.d(), c.s0N.d(), c.s0W.d(), c.s0d.d(), c.T};
    const PairSrc g1{c.s1x.d(), c.s1N.d(), c.s1W.d(), c.s1d.d(), c.S1};
    if (L.n > 0) {
        const bool f32 = c.opt.precision == BIM_PREC_MIXED;
        if (f32) {  // (allocates the record buffers on first use: their addresses are taken after it)
            ProfScope ps(c, "pair_pack", 0.0, 0.0);
            pack32(c, kind, g0, g1);
        }
        const float4 *r0 = f32 ? c.rec32_0.as<float4>() : nullptr, *r1 = f32 ? c.rec32_1.as<float4>() : nullptr;
        REQUIRE(!f32 || (r0 && r1), BIM_EDEVICE, "FP32 source records missing");
        const int tile = 64 * c.pair_T;
        double *part = c.part_override ? c.part_override : c.pair_part.d();
        {
            // whole tiles first, the remainder items after them (they fill the launch's tail)
            ProfScope ps(c, kind == 0 ? "pair_sl" : "pair_dl", L.pairs * fpp, 0.0);
            launch_pair(c.stream, kind, c.pair_T, L.n, L.d.as<PairWork>(), 0, tile, c.tlist.as<int>(), c.tx.d(), c.T,
                        g0, g1, part, r0, r1, c.cbnd.d(), c.nd);
        }
        {
            ProfScope ps(c, "pair_gather", 0.0, 8.0 * 3.0 * ((double)L.g.h_tent.size() * tile + L.g.h_ent.size()));
            launch_pair_gather(c.stream, (int)c.T, tile, c.tile_of.as<int>(), L.g.toff.as<int>(), L.g.tent.as<int>(),
                               L.g.off.as<int>(), L.g.ent.as<int>(), part, c.acc.d(), c.T, true);
        }
    }
    run_fmm(c, kind, L);
}

// Nearest-region items (Sec. 2.3): the self-interaction grids of their source
// drops (in near_self) analysed, the regular rule at the interpolation points,
// then interpolation to the targets, weighted and added into acc.
static void run_near(Ctx &c, int kind, const double *dens, const std::vector<double> &wt)
{
    if (c.near_h.empty()) return;
    Ctx::WList &L = work_lists(c, wt);
    std::vector<AnaJob> jobs;
    for (int j = 0; j < c.nd; ++j) {
        if (!c.near_src[j]) continue;
        const Drop &d = c.drops[j];
        jobs.push_back(ana_job(c, d.p, d.p, 3, c.near_self.d() + d.toff, c.T, c.near_selfc.d() + d.coff, c.Ctot));
    }
    ana_run(c, jobs);
    // every interpolation point belongs to one item list (its grid), so the
    // gather below writes all of near_vacc
    const long V = (long)c.near_h.size() * c.opt.near_L;
    double *part = c.part_override ? c.part_override : c.pair_part.d();
    const double fpp = kind == 0 ? 29.0 : 30.0;
    ProfScope ps(c, "near", c.near_pairs * fpp, 0.0);
    const PairSrc g0{c.tx.d(), c.s0N.d(), c.s0W.d(), c.s0d.d(), c.T};
    const PairSrc g1{c.s1x.d(), c.s1N.d(), c.s1W.d(), c.s1d.d(), c.S1};
    launch_pair(c.stream, kind, 1, c.near_nwork, c.near_work.as<PairWork>(), 0, 64, c.near_tl.as<int>(), c.near_vx.d(),
                V, g0, g1, part);
    launch_pair_gather(c.stream, (int)V, 64, nullptr, nullptr, nullptr, c.near_g.off.as<int>(),
                       c.near_g.ent.as<int>(), part, c.near_vacc.d(), V, false);
    launch_near_interp(c.stream, near_args(c), kind, c.near_selfc.d(), dens, c.near_vacc.d(), L.nw.d(),
                       c.near_res.d());
    launch_pair_gather(c.stream, (int)c.T, (int)c.near_h.size(), nullptr, nullptr, nullptr, c.near_tg.off.as<int>(),
                       c.near_tg.ent.as<int>(), c.near_res.d(), c.acc.d(), c.T, true);
}

// --------------------------------------------------------------------------
// matrix-core transforms of value fields (kernels_xform.hip), FP32 operands in
// the mixed form
// --------------------------------------------------------------------------
// Fourier table of grid g for orders m <= g.nmax: [2 m + ri][k], k < q, the
// values (cos, -sin)(m pi k / q), times w_m (1 at m = 0, else 2) for synthesis.
static const void *xtrig(Ctx &c, GridTab &g, bool analysis, bool f32)
{
    DBuf &b = g.xtrig[analysis][f32];
    if (b.ptr) return b.ptr;
    const int q = g.q, p = g.nmax;
    std::vector<double> t((size_t)2 * (p + 1) * q);
    for (int m = 0; m <= p; ++m) {
        const double w = analysis || m == 0 ? 1.0 : 2.0;
        for (int k = 0; k < q; ++k) {
            const double a = kPi * (double)(((long)m * k) % (2L * q)) / q;
            t[(size_t)(2 * m) * q + k] = w * std::cos(a);
            t[(size_t)(2 * m + 1) * q + k] = -w * std::sin(a);
        }
    }
    if (f32) {
        const std::vector<float> f(t.begin(), t.end());
        b.ensure(f.size() * sizeof(float));
        HIPC(hipMemcpyAsync(b.ptr, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, c.stream));
    } else {
        b.ensure(t.size() * sizeof(double));
        HIPC(hipMemcpyAsync(b.ptr, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
    }
    HIPC(hipStreamSynchronize(c.stream));
    return b.ptr;
}

static void xplan_upload(Ctx &c, Ctx::XPlan &pl)
{
    auto up = [&](DBuf &d, const void *h, size_t bytes) {
        d.ensure(std::max<size_t>(8, bytes));
        if (bytes) HIPC(hipMemcpyAsync(d.ptr, h, bytes, hipMemcpyHostToDevice, c.stream));
    };
    up(pl.cb, pl.h_cb.data(), pl.h_cb.size() * sizeof(long));
    up(pl.gb0, pl.h_gb0.data(), pl.h_gb0.size() * sizeof(long));
    up(pl.gb1, pl.h_gb1.data(), pl.h_gb1.size() * sizeof(long));
    up(pl.csc, pl.h_csc.data(), pl.h_csc.size() * sizeof(double));
    HIPC(hipStreamSynchronize(c.stream));
}

// Plans of the drops: drops of equal degree (and upsampled degree) in one
// plan, the fields (drop, component) in drop order.
static std::vector<std::unique_ptr<Ctx::XPlan>> &xplans(Ctx &c)
{
    if (!c.xplans.empty()) return c.xplans;
    for (int i = 0; i < c.nd; ++i) {
        const Drop &d = c.drops[i];
        Ctx::XPlan *pl = nullptr;
        for (auto &e : c.xplans)
            if (e->p == d.p && e->qu == d.qu) pl = e.get();
        if (!pl) {
            c.xplans.push_back(std::make_unique<Ctx::XPlan>());
            pl = c.xplans.back().get();
            pl->p = d.p;
            pl->qu = d.qu;
        }
        for (int cc = 0; cc < 3; ++cc) {
            pl->h_cb.push_back(cc * c.Ctot + d.coff);
            pl->h_cb.push_back(cc * c.Ctot + d.coff + 1);
            pl->h_gb0.push_back(cc * c.T + d.toff);
            pl->h_gb1.push_back(cc * c.S1 + d.uoff);
            pl->h_csc.push_back(d.lam + 1.0);
            ++pl->nf;
        }
    }
    for (auto &e : c.xplans) xplan_upload(c, *e);
    return c.xplans;
}

// Plan of a stand-alone call: nf fields of degree p, consecutive
// coefficient blocks of 2 ncoef(p) doubles and grids of N(q) values.
static Ctx::XPlan &xfield_plan(Ctx &c, int p, int q, int nf)
{
    auto &e = c.xfields[std::make_tuple(p, q, nf)];
    if (e) return *e;
    e = std::make_unique<Ctx::XPlan>();
    e->p = p;
    e->qu = q;
    e->nf = nf;
    for (int f = 0; f < nf; ++f) {
        e->h_cb.push_back((long)f * 2 * ncoef(p));
        e->h_cb.push_back((long)f * 2 * ncoef(p) + 1);
        e->h_gb0.push_back((long)f * npts(q));
    }
    xplan_upload(c, *e);
    return *e;
}

static bool xform_drops_ok(const Ctx &c, bool analysis)
{
    for (const Drop &d : c.drops)
        if (!xform_fits(d.p, analysis ? d.p : d.qu, analysis)) return false;
    return true;
}

static XJob xjob(Ctx &c, Ctx::XPlan &pl, int q, const DBuf &gb, double *gridv, bool analysis, bool combine,
                 bool f32, size_t &goff)
{
    GridTab &g = grid(c, q, pl.p);
    XJob j{};
    j.cb = pl.cb.as<long>();
    j.gb = gb.as<long>();
    j.csc = combine ? pl.csc.d() : nullptr;
    j.L = g.L.d();
    j.wq = g.wq.d();
    j.trig = xtrig(c, g, analysis, f32);
    j.G = reinterpret_cast<void *>(goff);  // offset inside xG until the buffer is sized
    j.grid = gridv;
    j.p = pl.p;
    j.q = q;
    j.nf = pl.nf;
    j.ldn = ncoef(pl.p);
    const size_t bytes = (size_t)(pl.p + 1) * (q + 1) * 2 * pl.nf * (f32 ? sizeof(float) : sizeof(double));
    goff += (bytes + 255) / 256 * 256;
    return j;
}

static void xjobs_place(Ctx &c, std::vector<XJob> &jobs, size_t goff)
{
    c.xG.ensure(std::max<size_t>(256, goff));
    for (XJob &j : jobs) j.G = static_cast<char *>(c.xG.ptr) + reinterpret_cast<size_t>(j.G);
}

// Synthesis of value fields on the grids named by the jobs, FP32 operands
// when f32 (flops and bytes as the scalar path counts them).
static void xsynth_run(Ctx &c, std::vector<XJob> &jobs, size_t goff, const double *x, bool f32,
                       double *z0 = nullptr, long nz0 = 0, double *z1 = nullptr, long nz1 = 0)
{
    xjobs_place(c, jobs, goff);
    double fl = 0.0, by = 0.0;
    for (const XJob &j : jobs) {
        fl += (double)j.nf * (j.q + 1) * ncoef(j.p) * 8.0 + (double)j.nf * npts(j.q) * (j.p + 1) * 4.0;
        by += (double)j.nf * (2.0 * ncoef(j.p) + npts(j.q)) * 8.0;
    }
    ProfScope ps(c, "synthesis", fl, by);
    launch_xsynth(c.stream, f32, jobs.data(), (int)jobs.size(), x, z0, nz0, z1, nz1);
}

static void xanal_run(Ctx &c, std::vector<XJob> &jobs, size_t goff, const double *x, double *y, double sgn,
                      bool f32)
{
    xjobs_place(c, jobs, goff);
    double fl = 0.0, by = 0.0;
    for (const XJob &j : jobs) {
        fl += (double)j.nf * ((j.q + 1) * ncoef(j.p) * 4.0 + (double)npts(j.q) * (j.p + 1) * 4.0);
        by += (double)j.nf * (2.0 * ncoef(j.p) + npts(j.q)) * 8.0;
    }
    ProfScope ps(c, "analysis", fl, by);
    launch_xanal(c.stream, f32, jobs.data(), (int)jobs.size(), x, y, sgn);
}

// Path of the value-field transforms of the drops (option xform_path): the
// matrix-core kernels or the scalar ones; with xform_path 0 both are timed
// (run(false) scalar, run(true) matrix cores; each run is complete and
// repeatable, and the caller runs the chosen path once more), two rounds
// after a warm-up, with HIP events on the context stream, the faster of
// each path's two counted; the matrix cores are taken when faster by more
// than kTuneMargin. The choice is kept for the context and, under the
// problem's shape (kind, precision, degrees and field counts of the plans),
// for the process: the first stored wins, so concurrent contexts of one
// shape agree and their results do not depend on which of them timed.
static std::mutex g_xmode_mu;
static std::map<std::vector<long>, int> g_xmodes;

template <class Run> static bool xform_mfma(Ctx &c, int kind, bool f32, Run &&run)
{
    int &mode = c.xmode[kind][f32];
    if (!xform_drops_ok(c, kind == 1)) return (mode = 0) == 1;
    if (c.opt.xform_path != 0) return (mode = c.opt.xform_path == 2 ? 1 : 0) == 1;
    if (mode >= 0) return mode == 1;
    std::vector<long> key{kind, f32 ? 1 : 0};
    for (auto &pl : xplans(c)) key.insert(key.end(), {pl->p, pl->qu, pl->nf});
    {
        std::lock_guard<std::mutex> lk(g_xmode_mu);
        auto it = g_xmodes.find(key);
        if (it != g_xmodes.end()) return (mode = it->second) == 1;
    }
    REQUIRE(!t_no_alloc, BIM_ESTATE, "transform path not chosen yet: call the allocating entry point first");
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    float best[2] = {0.0f, 0.0f};
    run(false);
    run(true);
    for (int round = 0; round < 2; ++round)
        for (int m = 0; m < 2; ++m) {
            HIPC(hipEventRecord(e0, c.stream));
            run(m == 1);
            HIPC(hipEventRecord(e1, c.stream));
            HIPC(hipEventSynchronize(e1));
            float ms = 0.0f;
            HIPC(hipEventElapsedTime(&ms, e0, e1));
            best[m] = round == 0 ? ms : std::min(best[m], ms);
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const int pick = best[1] < (1.0f - kTuneMargin) * best[0] ? 1 : 0;
    std::lock_guard<std::mutex> lk(g_xmode_mu);
    return (mode = g_xmodes.emplace(key, pick).first->second) == 1;
}

// Standard-grid values gridv [3][T] of every drop to coefficients: y =
// (lambda + 1) x - P[gridv] with combine, else y = P[gridv]; FP32 operands in
// the mixed form.
static void xanal_drops(Ctx &c, const double *gridv, const double *x, double *y, bool combine)
{
    const bool f32 = c.opt.precision == BIM_PREC_MIXED;
    std::vector<XJob> jobs;
    size_t goff = 0;
    for (auto &pl : xplans(c))
        jobs.push_back(xjob(c, *pl, pl->p, pl->gb0, const_cast<double *>(gridv), true, combine, f32, goff));
    xanal_run(c, jobs, goff, x, y, combine ? -1.0 : 1.0, f32);
}

// Density values (3 components, coefficients dens [3][Ctot]) on the standard
// and upsampled nodes of the drops whose flag is set (the matrix-core path
// writes every drop's). f32: FP32 operands in the mixed form (the density of
// the double-layer operator); the force density of the single layer stays
// FP64: its layer is the sum of terms that nearly cancel for a drop close to
// equilibrium, and FP32 node values would set the error of that small sum.
static void density_nodes(Ctx &c, const double *dens, const std::vector<char> &need, bool f32, double *z0 = nullptr,
                          long nz0 = 0, double *z1 = nullptr, long nz1 = 0)
{
    f32 = f32 && c.opt.precision == BIM_PREC_MIXED;
    auto run = [&](bool mfma) {
        if (mfma) {
            std::vector<XJob> xj;
            size_t goff = 0;
            for (auto &pl : xplans(c)) {
                xj.push_back(xjob(c, *pl, pl->p, pl->gb0, c.s0d.d(), false, false, f32, goff));
                xj.push_back(xjob(c, *pl, pl->qu, pl->gb1, c.s1d.d(), false, false, f32, goff));
            }
            xsynth_run(c, xj, goff, dens, f32, z0, nz0, z1, nz1);
            return;
        }
        std::vector<SynJob> jobs;
        for (int i = 0; i < c.nd; ++i) {
            if (!need[i]) continue;
            const Drop &d = c.drops[i];
            jobs.push_back(syn_job(c, d.p, d.p, 3, dens + d.coff, c.Ctot, 0x1, c.s0d.d() + d.toff, c.T, 0));
            jobs.push_back(syn_job(c, d.p, d.qu, 3, dens + d.coff, c.Ctot, 0x1, c.s1d.d() + d.uoff, c.S1, 0));
        }
        syn_run(c, jobs, z0, nz0, z1, nz1);
    };
    run(xform_mfma(c, 0, f32, run));
}

// Singular self-integral of drop i with density coefficients dens [3][Ctot]
// (kind 0 SL, 1 DL), added into acc with the given scale: rotation of the
// expansion per target, then the fused quadrature (per-application path).
static void run_singular(Ctx &c, int i, int kind, const double *dens, double scale, double *out = nullptr)
{
    const Drop &d = c.drops[i];
    RotTab &r = rot(c, d.p);
    GridTab &gp = grid(c, d.p, d.p);
    GridTab &gs = grid(c, d.qs, d.p);
    const long nc = ncoef(d.p);
    c.Rbuf.ensure((size_t)npts(d.p) * 6 * nc * 2 * sizeof(double));
    {
        ProfScope ps(c, "sing_rotate", (double)npts(d.p) * 6.0 * rot_lat_size(d.p) * 4.0, 0.0);
        launch_rotate(c.stream, d.p, r.Ap.d(), r.Am.d(), gp.cs.d(), c.xc.d() + d.coff, c.Ctot, dens + d.coff,
                      c.Ctot, c.Rbuf.d());
    }
    {
        ProfScope ps(c, "sing_v1", 0.0, 0.0);
        launch_singular(c.stream, d.p, d.qs, kind, c.Rbuf.d(), gs.L.d(), (int)nc, gs.wsing.d(), gs.cs.d(),
                        (out ? out : c.acc.d()) + d.toff, c.T, scale);
    }
}

// --------------------------------------------------------------------------
// batched singular pipeline (kernels_pipe.hip)
// --------------------------------------------------------------------------
static Ctx::PipeTab &pipe_tables(Ctx &c, int p, int qs)
{
    auto key = std::make_pair(p, qs);
    auto it = c.pipes.find(key);
    if (it != c.pipes.end()) return *it->second;
    auto t = std::make_unique<Ctx::PipeTab>();
    GridTab &g = grid(c, qs, p);
    const int P1 = p + 1, Q1 = qs + 1, nc = ncoef(p);
    std::vector<double> P((size_t)Q1 * nc), D((size_t)Q1 * nc);
    for (int j = 0; j < Q1; ++j) legendre_table(p, g.t[j], &P[(size_t)j * nc], &D[(size_t)j * nc], nullptr);
    // synthesis: per mu, rows [Ptilde(t_j'); dPtilde/dtheta(t_j')] (2 Q1), depth n = mu..p
    std::vector<double> syn, ana;
    std::vector<LegBatchH> bx, bd, ba;
    long koffm = 0;
    for (int mu = 0; mu < P1; ++mu) {
        const int K = P1 - mu;
        LegBatchH h{2 * Q1, K, (long)syn.size(), koffm, (long)mu * 2 * Q1};
        for (int r = 0; r < 2 * Q1; ++r)
            for (int kk = 0; kk < K; ++kk) {
                const int n = mu + kk, j = r % Q1;
                syn.push_back(r < Q1 ? P[(size_t)j * nc + tri(n, mu)] : D[(size_t)j * nc + tri(n, mu)]);
            }
        bx.push_back(h);
        LegBatchH hd{Q1, K, h.tab_off, koffm, (long)mu * Q1};
        bd.push_back(hd);
        // analysis: rows n = mu..p, depth j' = 0..qs
        LegBatchH ha{K, Q1, (long)ana.size(), (long)mu * Q1, koffm};
        for (int kk = 0; kk < K; ++kk)
            for (int j = 0; j < Q1; ++j) ana.push_back(P[(size_t)j * nc + tri(mu + kk, mu)]);
        ba.push_back(ha);
        koffm += K;
    }
    auto up = [&](DBuf &b, const void *src, size_t bytes) {
        b.ensure(bytes);
        HIPC(hipMemcpyAsync(b.ptr, src, bytes, hipMemcpyHostToDevice, c.stream));
        HIPC(hipStreamSynchronize(c.stream));
    };
    up(t->syn, syn.data(), syn.size() * sizeof(double));
    up(t->ana, ana.data(), ana.size() * sizeof(double));
    up(t->bsx, bx.data(), bx.size() * sizeof(LegBatchH));
    up(t->bsd, bd.data(), bd.size() * sizeof(LegBatchH));
    up(t->ban, ba.data(), ba.size() * sizeof(LegBatchH));
    t->maxrows_syn = 2 * Q1;
    t->maxrows_ana = P1;
    auto &ref = *t;
    c.pipes[key] = std::move(t);
    return ref;
}

static bool pipe_fits(int p, int qs)
{
    return 2 * (qs + 1) <= leg_mfma_max_rows() && (p + 1) <= leg_mfma_max_depth() &&
           (qs + 1) <= leg_mfma_max_depth() && fk_lds_bytes(p, qs, true, 4) <= 163840 && rot_lds_bytes(p) <= 163840;
}

// Singular pass of a group of drops of one degree (and singular grid) through
// the batched pipeline: single layer of dens added into acc (sl) and/or the
// stored double-layer rows of each drop (dl). Chunks are sets of (drop,
// latitude) units sized by a memory budget for the intermediates.
// st: the stream of the launches (the context's by default); acc_out: where
// the single layer's longitude sums are added (acc by default).
static void run_pipe_group(Ctx &c, const std::vector<int> &ids, bool sl, bool dl, const double *dens,
                           hipStream_t st = nullptr, double *acc_out = nullptr)
{
    if (ids.empty()) return;
    if (!st) st = c.stream;
    if (!acc_out) acc_out = c.acc.d();
    const Drop &d0 = c.drops[ids[0]];
    const int p = d0.p, qs = d0.qs, P1 = p + 1, Q1 = qs + 1, nk = 2 * p, nc = ncoef(p);
    RotTab &r = rot(c, p);
    GridTab &gp = grid(c, p, p);
    GridTab &gs = grid(c, qs, p);
    Ctx::PipeTab &pt = pipe_tables(c, p, qs);
    pipe_set_lds_limits();
    REQUIRE((int)ids.size() <= kPipeMaxDrops, BIM_EINVAL, "too many drops in one pipeline pass");
    PipeDrops pd{};
    pd.n = (int)ids.size();
    for (int q = 0; q < pd.n; ++q) {
        const int i = ids[q];
        const Drop &d = c.drops[i];
        pd.coff[q] = d.coff;
        pd.toff[q] = d.toff;
        pd.M[q] = nullptr;
        if (dl) {
            if ((int)c.Mdl.size() < c.nd) {
                c.Mdl.resize(c.nd);
                c.Mok.resize(c.nd, 0);
            }
            if (!c.Mdl[i]) c.Mdl[i] = std::make_unique<DBuf>();
            c.Mdl[i]->ensure((size_t)npts(p) * 6 * 2 * nc * sizeof(double));
            pd.M[q] = c.Mdl[i]->d();
        }
    }
    // units per chunk from a memory budget for the intermediates
    const double per_lat = (double)nk * 8.0 *
                           ((double)nc * 6 * (sl ? 2 : 1) + (double)P1 * 2 * Q1 * 6 + (sl ? (double)P1 * Q1 * 6 : 0.0) +
                            (dl ? (double)P1 * Q1 * 12 + (double)nc * 12 : 0.0) + Q1 * 3 + 3);
    const double budget = c.opt.pipe_budget_gb * 1024.0 * 1024 * 1024;
    const int nu = pd.n * P1;
    const int nj = std::max(1, std::min(nu, (int)(budget / per_lat)));
    const long NTc = (long)nj * nk;
    c.pBx.ensure((size_t)nc * NTc * 6 * 8);
    if (sl) c.pBd.ensure((size_t)nc * NTc * 6 * 8);
    c.pGx.ensure((size_t)P1 * 2 * Q1 * NTc * 6 * 8);
    if (sl) c.pGd.ensure((size_t)P1 * Q1 * NTc * 6 * 8);
    c.pPart.ensure((size_t)NTc * Q1 * 3 * 8);
    c.pX0.ensure((size_t)NTc * 3 * 8);
    if (dl) {
        c.pFa.ensure((size_t)P1 * Q1 * NTc * 12 * 8);
        c.pBt.ensure((size_t)nc * NTc * 12 * 8);
    }
    const double rotlat = (double)rot_lat_size(p);
    for (int u0 = 0; u0 < nu; u0 += nj) {
        const int nuc = std::min(nj, nu - u0);
        const long nt = (long)nuc * nk, NC6 = nt * 6, NC12 = nt * 12;
        {
            ProfScope ps(c, "pipe_rotate", nt * (sl ? 6.0 : 3.0) * rotlat * 4.0, nt * (sl ? 2.0 : 1.0) * nc * 6 * 8.0, st);
            launch_rot2(st, p, r.Ap.d(), r.Am.d(), gp.cs.d(), c.xc.d(), c.Ctot, sl ? dens : nullptr, c.Ctot,
                        pd, u0, nuc, c.pBx.d(), sl ? c.pBd.d() : nullptr, NC6);
            launch_pole(st, p, (int)nt, c.pBx.d(), NC6, c.pX0.d());
        }
        {
            ProfScope ps(c, "pipe_legendre", 2.0 * 2 * Q1 * nc * NC6 + (sl ? 2.0 * Q1 * nc * NC6 : 0.0),
                         8.0 * ((double)nc * NC6 * (sl ? 2 : 1) + (double)P1 * 2 * Q1 * NC6 + (sl ? (double)P1 * Q1 * NC6 : 0.0)), st);
            launch_leg_mfma(st, P1, pt.maxrows_syn, pt.bsx.ptr, pt.syn.d(), c.pBx.d(), c.pGx.d(), NC6);
            if (sl) launch_leg_mfma(st, P1, Q1, pt.bsd.ptr, pt.syn.d(), c.pBd.d(), c.pGd.d(), NC6);
        }
        {
            // algorithmic flops per target: each real field column of the
            // rotated grid as a length-2qs FFT per latitude, 2.5 n log2 n with
            // n = 2 qs, over qs + 1 latitudes (x, x_theta, x_phi and, for the
            // single layer, f: 12 or 9 columns; the stresslet analysis: 6),
            // plus the pointwise kernels (35 flops per node SL, 40 DL). The
            // kernel itself evaluates the Fourier sums directly with the
            // phi -> -phi symmetry (more flops), which this count ignores.
            const double NP = npts(qs), n2 = 2.0 * qs;
            const double fft = 2.5 * n2 * std::log2(n2) * Q1;
            double fl = fft * (sl ? 12.0 : 9.0) + (sl ? NP * 35.0 : 0.0);
            if (dl) fl += NP * 40.0 + 6.0 * fft;
            ProfScope ps(c, "pipe_fourier", nt * fl,
                         8.0 * ((double)P1 * (sl ? 3 : 2) * Q1 * NC6 + (dl ? (double)P1 * Q1 * NC12 : 0.0)), st);
            launch_fk(st, sl, dl, p, qs, (int)nt, c.pGx.d(), sl ? c.pGd.d() : nullptr, NC6, gs.wsing.d(),
                      gs.cs.d(), c.pX0.d(), c.pPart.d(), dl ? c.pFa.d() : nullptr, NC12);
            if (sl) launch_sum_part(st, (int)nt, Q1, nk, P1, c.pPart.d(), pd, u0, 1.0, acc_out, c.T);
        }
        if (dl) {
            {
                ProfScope ps(c, "pipe_legendre", 2.0 * Q1 * nc * NC12, 8.0 * ((double)P1 * Q1 * NC12 + (double)nc * NC12), st);
                launch_leg_mfma(st, P1, pt.maxrows_ana, pt.ban.ptr, pt.ana.d(), c.pFa.d(), c.pBt.d(), NC12);
            }
            {
                ProfScope ps(c, "pipe_adjrot", nt * 6.0 * rotlat * 4.0, 8.0 * ((double)nc * NC12 + (double)nt * 6 * 2 * nc), st);
                launch_adjrot(st, p, r.Ap.d(), r.Am.d(), gp.cs.d(), c.pBt.d(), NC12, pd, u0, nuc);
            }
        }
    }
    HIPC(hipGetLastError());
    if (dl)
        for (int i : ids) c.Mok[i] = 1;
}

// Drops grouped by (degree, singular grid degree), in drop order.
static std::vector<std::vector<int>> pipe_groups(const Ctx &c, const std::vector<int> &ids)
{
    std::map<std::pair<int, int>, std::vector<int>> g;
    for (int i : ids) g[{c.drops[i].p, c.drops[i].qs}].push_back(i);
    std::vector<std::vector<int>> out;
    for (auto &kv : g)
        for (size_t a = 0; a < kv.second.size(); a += kPipeMaxDrops)
            out.emplace_back(kv.second.begin() + a,
                             kv.second.begin() + std::min(kv.second.size(), a + (size_t)kPipeMaxDrops));
    return out;
}

static bool use_fused(const Ctx &c, const Drop &d, bool sl, bool dl)
{
    return c.opt.singular_path == 2 && sing_fused_fits(d.p, d.qs, sl, dl);
}

static bool use_pipe(const Ctx &c, const Drop &d) { return c.opt.singular_path == 0 && pipe_fits(d.p, d.qs); }

// Fused singular pass of drop i: single layer of dens added into acc (if sl),
// and/or the stored double-layer rows of the drop (if dl).
static void run_fused(Ctx &c, int i, bool sl, bool dl, const double *dens)
{
    const Drop &d = c.drops[i];
    RotTab &r = rot(c, d.p);
    GridTab &gp = grid(c, d.p, d.p);
    GridTab &gs = grid(c, d.qs, d.p);
    SingArgs a{};
    a.p = d.p;
    a.qs = d.qs;
    a.nt = npts(d.p);
    a.Ap = r.Ap.d();
    a.Am = r.Am.d();
    a.ApT = r.ApT.d();
    a.AmT = r.AmT.d();
    a.csp = gp.cs.d();
    a.xc = c.xc.d() + d.coff;
    a.xstride = c.Ctot;
    a.dc = sl ? dens + d.coff : nullptr;
    a.dstride = c.Ctot;
    a.L = gs.L.d();
    a.wsing = gs.wsing.d();
    a.out_sl = c.acc.d() + d.toff;
    a.ostride = c.T;
    a.scale = 1.0;
    a.M = nullptr;
    if (dl) {
        if ((int)c.Mdl.size() < c.nd) {
            c.Mdl.resize(c.nd);
            c.Mok.resize(c.nd, 0);
        }
        if (!c.Mdl[i]) c.Mdl[i] = std::make_unique<DBuf>();
        c.Mdl[i]->ensure((size_t)npts(d.p) * 6 * 2 * ncoef(d.p) * sizeof(double));
        a.M = c.Mdl[i]->d();
    }
    {
        const double nt = npts(d.p);
        ProfScope ps(c, "sing_fused", nt * sing_flops_per_target(d.p, d.qs, sl, dl),
                     dl ? nt * 6.0 * 2.0 * ncoef(d.p) * 8.0 : 0.0);
        REQUIRE(launch_sing_fused(c.stream, sl, dl, a), BIM_EDEVICE, "fused singular kernel does not fit");
    }
    HIPC(hipGetLastError());
    if (dl) c.Mok[i] = 1;
}

static bool dl_matrix_ready(const Ctx &c, int i) { return i < (int)c.Mok.size() && c.Mok[i]; }

// Weighted double-layer sum sum_j w(i,j) D_j[u] at all targets into acc.
static std::vector<double> dl_weights(const Ctx &c)
{
    std::vector<double> wt((size_t)c.nd * c.nd);
    for (int i = 0; i < c.nd; ++i)
        for (int j = 0; j < c.nd; ++j) {
            const double lam = c.opt.lambda_rule == 0 ? c.drops[j].lam : c.drops[i].lam;
            wt[(size_t)i * c.nd + j] = (lam - 1.0) / (4.0 * kPi);
        }
    return wt;
}

static void double_layer_grid(Ctx &c, const double *ucoef, const std::vector<double> &wt)
{
    build_regions(c);
    std::vector<char> need(c.nd, 0), selfraw(c.nd, 0);
    for (int j = 0; j < c.nd; ++j)
        for (int i = 0; i < c.nd; ++i)
            if (wt[(size_t)i * c.nd + j] != 0.0) need[j] = 1;
    for (const NearItem &it : c.near_h)
        if (wt[(size_t)it.i * c.nd + it.j] != 0.0) selfraw[it.j] = 1;
    // acc (and near_self) cleared by the density synthesis launch
    density_nodes(c, ucoef, need, true, c.acc.d(), 3 * c.T, c.near_h.empty() ? nullptr : c.near_self.d(),
                  c.near_h.empty() ? 0 : 3 * c.T);
    // stored rows: build those missing (pipeline drops grouped by degree)
    std::vector<int> build;
    for (int i = 0; i < c.nd; ++i) {
        const Drop &d = c.drops[i];
        if ((wt[(size_t)i * c.nd + i] != 0.0 || selfraw[i]) && use_pipe(c, d) && !dl_matrix_ready(c, i))
            build.push_back(i);
    }
    for (auto &g : pipe_groups(c, build)) run_pipe_group(c, g, false, true, nullptr);
    std::vector<DlJob> jobs;
    double dfl = 0.0, dby = 0.0;
    for (int i = 0; i < c.nd; ++i) {
        const double w = wt[(size_t)i * c.nd + i];
        if (w == 0.0 && !selfraw[i]) continue;
        const Drop &d = c.drops[i];
        // the raw self-interaction goes to near_self when an item interpolates from it
        double *dst = selfraw[i] ? c.near_self.d() : c.acc.d();
        const double ws = selfraw[i] ? 1.0 : w;
        if (use_pipe(c, d) || use_fused(c, d, false, true)) {
            if (!dl_matrix_ready(c, i)) run_fused(c, i, false, true, nullptr);
            const double nt = npts(d.p), nc2 = 2.0 * ncoef(d.p);
            dfl += nt * 18.0 * nc2;
            dby += nt * 6.0 * nc2 * 8.0 + 3.0 * nc2 * 8.0;
            jobs.push_back(DlJob{c.Mdl[i]->d(), ucoef + d.coff, dst + d.toff, ws, npts(d.p), 2 * ncoef(d.p)});
        } else {
            run_singular(c, i, 1, ucoef, ws, dst);
        }
    }
    if (!jobs.empty()) {
        ProfScope ps(c, "dl_apply", dfl, dby);
        launch_dl_apply_multi(c.stream, jobs.data(), (int)jobs.size(), c.Ctot, c.T);
    }
    for (int i = 0; i < c.nd; ++i) {
        const double w = wt[(size_t)i * c.nd + i];
        if (!selfraw[i] || w == 0.0) continue;
        const Drop &d = c.drops[i];
        for (int cc = 0; cc < 3; ++cc)
            launch_scale_add(c.stream, npts(d.p), w, c.near_self.d() + cc * c.T + d.toff, 1.0,
                             c.acc.d() + cc * c.T + d.toff);
    }
    run_pairs(c, 1, wt);
    run_near(c, 1, ucoef, wt);
}

// Whether two drops of one system interact (there are pair sums).
static bool drop_pairs(const Ctx &c)
{
    for (int i = 0; i < c.nd; ++i)
        for (int j = i + 1; j < c.nd; ++j)
            if (c.sys_h[i] == c.sys_h[j]) return true;
    return false;
}

// Whether a choice by timing (pair work shape, fast-summation order,
// transform path) is still to be made: its timed launches must not share the
// device with other work.
static bool timing_pending(const Ctx &c)
{
    const bool f32 = c.opt.precision == BIM_PREC_MIXED;
    if (c.opt.xform_path == 0 && (c.xmode[0][f32] < 0 || c.xmode[1][f32] < 0)) return true;
    if (!drop_pairs(c)) return false;
    return (c.opt.pair_tune && !c.pair_tuned) || (c.opt.fmm_order < 0 && c.fmm_tuned < 0);
}

// The context's stream waits for the work of the second stream (a no-op
// when nothing is pending there).
static void join_side(Ctx &c)
{
    if (!c.join_pending) return;
    c.join_pending = false;
    HIPC(hipStreamWaitEvent(c.stream, c.ev_join, 0));
}

// Orders the second stream after the work enqueued so far on the context's
// stream (creating the stream and its events on first use).
static void fork_side(Ctx &c)
{
    join_side(c);
    if (!c.side) {
        HIPC(hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking));
        HIPC(hipEventCreateWithFlags(&c.ev_fork, hipEventDisableTiming));
        HIPC(hipEventCreateWithFlags(&c.ev_join, hipEventDisableTiming));
    }
    HIPC(hipEventRecord(c.ev_fork, c.stream));
    HIPC(hipStreamWaitEvent(c.side, c.ev_fork, 0));
}

// Single layer of fcoef at all targets into acc. with_dl[i] also builds the
// stored double-layer rows of drop i in the same pass; wt_dl: the weights of
// the double-layer operator that will follow, whose pair lists are built
// while the device runs the pipeline.
//
// The singular pipeline needs neither the regions nor the node densities.
// When the regions are still to be built, it runs on the second stream,
// adding into acc2, while the context's stream classifies the regions and
// the host builds the pair lists (with no timing pending, whose launches
// must have the device to themselves). acc then starts as a copy of acc2:
// the same values, added in the same order, as when the pipeline adds into a
// cleared acc on the context's stream.
static void single_layer_grid(Ctx &c, const double *fcoef, const std::vector<char> *with_dl = nullptr,
                              const std::vector<double> *wt_dl = nullptr)
{
    // pipeline drops grouped by degree, separately with and without the rows
    std::vector<int> with_rows, without_rows;
    for (int i = 0; i < c.nd; ++i) {
        if (!use_pipe(c, c.drops[i])) continue;
        const bool dl = with_dl && (*with_dl)[i] && !dl_matrix_ready(c, i);
        (dl ? with_rows : without_rows).push_back(i);
    }
    const bool side = !c.regions_ok && !(with_rows.empty() && without_rows.empty()) && !timing_pending(c);
    const size_t accb = (size_t)3 * c.T * sizeof(double);
    if (side) {
        c.acc2.ensure(accb);
        fork_side(c);
        HIPC(hipMemsetAsync(c.acc2.ptr, 0, accb, c.side));
        for (auto &g : pipe_groups(c, with_rows)) run_pipe_group(c, g, true, true, fcoef, c.side, c.acc2.d());
        for (auto &g : pipe_groups(c, without_rows)) run_pipe_group(c, g, true, false, fcoef, c.side, c.acc2.d());
        HIPC(hipEventRecord(c.ev_join, c.side));
        c.join_pending = true;
    }
    build_regions(c);
    std::vector<double> wt((size_t)c.nd * c.nd, 1.0);
    if (side) {
        (void)work_lists(c, wt);  // uploads enqueued now run beside the pipeline
        if (wt_dl) (void)work_lists(c, *wt_dl);
    }
    std::vector<char> need(c.nd, 1);
    density_nodes(c, fcoef, need, false, c.acc.d(), 3 * c.T);  // acc cleared by the same launch
    if (side) {
        join_side(c);
        HIPC(hipMemcpyAsync(c.acc.ptr, c.acc2.ptr, accb, hipMemcpyDeviceToDevice, c.stream));
    } else {
        for (auto &g : pipe_groups(c, with_rows)) run_pipe_group(c, g, true, true, fcoef);
        for (auto &g : pipe_groups(c, without_rows)) run_pipe_group(c, g, true, false, fcoef);
    }
    for (int i = 0; i < c.nd; ++i) {
        const Drop &d = c.drops[i];
        const bool dl = with_dl && (*with_dl)[i] && !dl_matrix_ready(c, i);
        if (use_pipe(c, d)) {
            continue;
        } else if (use_fused(c, d, true, dl)) {
            run_fused(c, i, true, dl, fcoef);             // both in one pass
        } else if (use_fused(c, d, true, false)) {
            run_fused(c, i, true, false, fcoef);          // rows built on first use
        } else {
            run_singular(c, i, 0, fcoef, 1.0);
        }
    }
    if (!c.near_h.empty())
        HIPC(hipMemcpyAsync(c.near_self.ptr, c.acc.ptr, 3 * c.T * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
    run_pairs(c, 0, wt);
    run_near(c, 0, fcoef, wt);
}

// analysis of grid vectors [3][T] into coefficients [3][Ctot]
static void project(Ctx &c, const double *grid_vals, double *coef)
{
    auto run = [&](bool mfma) {
        if (mfma) {
            xanal_drops(c, grid_vals, nullptr, coef, false);
            return;
        }
        std::vector<AnaJob> jobs;
        for (int i = 0; i < c.nd; ++i) {
            const Drop &d = c.drops[i];
            jobs.push_back(ana_job(c, d.p, d.p, 3, grid_vals + d.toff, c.T, coef + d.coff, c.Ctot));
        }
        ana_run(c, jobs);
    };
    run(xform_mfma(c, 1, c.opt.precision == BIM_PREC_MIXED, run));
}

static void synth_grid_all(Ctx &c, const double *coef, double *grid_vals)
{
    std::vector<SynJob> jobs;
    for (int i = 0; i < c.nd; ++i) {
        const Drop &d = c.drops[i];
        jobs.push_back(syn_job(c, d.p, d.p, 3, coef + d.coff, c.Ctot, 0x1, grid_vals + d.toff, c.T, 0));
    }
    syn_run(c, jobs);
}

// y = A x, the Galerkin second-kind operator (coefficients [3][Ctot]).
static void apply_operator(Ctx &c, const double *x, double *y, const std::vector<double> &wt)
{
    double_layer_grid(c, x, wt);
    // y = (lambda + 1) x - P[acc]: the combine rides on the analysis (the
    // scalar one when every drop's grid fits it)
    auto run = [&](bool mfma) {
        if (mfma) {
            xanal_drops(c, c.acc.d(), x, y, true);
            return;
        }
        std::vector<AnaJob> jobs;
        bool fused = true;
        for (int i = 0; i < c.nd; ++i) {
            const Drop &d = c.drops[i];
            AnaJob j = ana_job(c, d.p, d.p, 3, c.acc.d() + d.toff, c.T, y + d.coff, c.Ctot);
            j.cx = x + d.coff;
            j.csc = d.lam + 1.0;
            fused = fused && anal_batch_lds(d.p, d.p) <= 163840;
            jobs.push_back(j);
        }
        if (fused) {
            ana_run(c, jobs);
        } else {
            std::vector<AnaJob> pj;
            for (int i = 0; i < c.nd; ++i) {
                const Drop &d = c.drops[i];
                pj.push_back(ana_job(c, d.p, d.p, 3, c.acc.d() + d.toff, c.T, y + d.coff, c.Ctot));
            }
            ana_run(c, pj);
            launch_op_combine(c.stream, 3 * c.Ctot, c.scl.d(), x, y);
        }
    };
    run(xform_mfma(c, 1, c.opt.precision == BIM_PREC_MIXED, run));
}

// --------------------------------------------------------------------------
// GMRES (restarted, classical Gram-Schmidt with one re-orthogonalisation,
// Givens rotations and back substitution on the device). The residual
// estimate of each Arnoldi step reaches the host through pinned memory once
// the step's stamp is there. While steps are short the host enqueues step k
// + 1 before it reads the estimate of step k, so the device never waits for
// the host, and a step enqueued after convergence is discarded; once a step
// takes longer than kAheadMs the host reads each estimate first (the device
// then waits for the host's next launches, some 20 us per step, which is
// less than the one discarded step it saves).
// --------------------------------------------------------------------------
constexpr double kAheadMs = 1.0;
using OpFn = std::function<void(const double *, double *)>;

static int gmres_op(Ctx &c, long n, const OpFn &apply, const double *b, double *x, double tol, int &iters,
                    double &relres, int &nmv)
{
    const int m = std::max(1, std::min(c.opt.gmres_restart, gs_max_vectors() - 1));
    const long ldH = m + 2;
    c.V.ensure((size_t)(m + 1) * n * sizeof(double));
    c.hbuf.ensure((size_t)(2 * (m + 2)) * sizeof(double));
    c.ybuf.ensure((size_t)(m + 2) * sizeof(double));
    c.wvec.ensure((size_t)n * sizeof(double));
    c.rvec.ensure((size_t)n * sizeof(double));
    c.gspart.ensure((size_t)gs_blocks(n) * (m + 2) * sizeof(double));
    c.givbuf.ensure((size_t)(ldH * m + 3 * (m + 2)) * sizeof(double));
    if (!c.gscnt.ptr) {
        c.gscnt.ensure(sizeof(unsigned));
        HIPC(hipMemsetAsync(c.gscnt.ptr, 0, sizeof(unsigned), c.stream));
    }
    if (!c.hhost) HIPC(hipHostMalloc((void **)&c.hhost, 4 * 256 * sizeof(double)));
    double *V = c.V.d(), *h = c.hbuf.d(), *h2 = h + (m + 2), *w = c.wvec.d(), *part = c.gspart.d();
    unsigned *cnt = (unsigned *)c.gscnt.ptr;
    GivensArgs ga;
    ga.H = c.givbuf.d();
    ga.ldH = ldH;
    ga.cs = ga.H + ldH * m;
    ga.sn = ga.cs + (m + 2);
    ga.g = ga.sn + (m + 2);
    // residual estimates of the two latest steps: coherent pinned host memory
    // that the Givens step writes directly, each slot {estimate, stamp}; the
    // host waits for the step's stamp (no event in the stream between steps)
    if (!c.hres) {
        HIPC(hipHostMalloc((void **)&c.hres, 4 * sizeof(double), hipHostMallocCoherent));
        std::fill(c.hres, c.hres + 4, 0.0);
    }
    double *resdev = nullptr;
    HIPC(hipHostGetDevicePointer((void **)&resdev, c.hres, 0));
    HIPC(hipMemsetAsync(x, 0, n * sizeof(double), c.stream));
    // ||b|| is the first residual norm (r = b at x = 0: the same kernel and
    // summation order), read with it
    double bn = 0.0;
    iters = 0;
    nmv = 0;
    relres = 0.0;
    double *gh = c.hhost + 256;  // host image of g at a restart
    volatile double *resh = c.hres;
    bool first = true;
    while (true) {
        // r = b - A x
        if (first) {
            HIPC(hipMemcpyAsync(c.rvec.ptr, b, n * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
        } else {
            apply(x, c.rvec.d());
            ++nmv;
            launch_scale_add(c.stream, n, 1.0, b, -1.0, c.rvec.d());
        }
        launch_gs_update_norm(c.stream, n, 0, nullptr, n, nullptr, c.rvec.d(), part, cnt, h, GivensArgs{}, V);
        HIPC(hipMemcpyAsync(c.hhost, h, sizeof(double), hipMemcpyDeviceToHost, c.stream));
        HIPC(hipStreamSynchronize(c.stream));
        const double beta = c.hhost[0];
        if (first) {
            bn = beta;
            ga.bnorm = bn;
            if (bn == 0.0) return BIM_OK;
        }
        first = false;
        relres = beta / bn;
        if (relres <= tol) return BIM_OK;
        if (iters >= c.opt.gmres_maxit) return BIM_ENOCONV;
        std::fill(gh, gh + m + 2, 0.0);
        gh[0] = beta;
        HIPC(hipMemcpyAsync(ga.g, gh, (m + 2) * sizeof(double), hipMemcpyHostToDevice, c.stream));
        const int kmax = std::min(m, c.opt.gmres_maxit - iters);
        int kdone = 0;
        bool conv = false;
        // step k: Arnoldi vector k + 1, column k of R, residual estimate and
        // the step's stamp -> resh[2 (k & 1)], resh[2 (k & 1) + 1]
        double stamp[2] = {0.0, 0.0};
        auto step = [&](int k) {
            apply(V + (long)k * n, w);
            GivensArgs gk = ga;
            gk.res = resdev + 2 * (k & 1);  // written by the device into pinned host memory
            gk.stamp = stamp[k & 1] = (c.gm_seq += 1.0);
            launch_gs_dots(c.stream, n, k + 1, V, n, w, part, cnt, h);
            launch_gs_update_dots(c.stream, n, k + 1, V, n, h, w, part, cnt, h2);
            launch_gs_update_norm(c.stream, n, k + 1, V, n, h2, w, part, cnt, h, gk, V + (long)(k + 1) * n);
        };
        // the estimate of step k once its stamp has arrived; a stream that
        // ends or fails without it is an error (no unbounded wait)
        auto wait_step = [&](int k) {
            volatile double *st = resh + 2 * (k & 1) + 1;
            for (long spin = 1; *st != stamp[k & 1]; ++spin) {
                if (spin % 256 != 0) continue;
                const hipError_t q = hipStreamQuery(c.stream);
                if (q == hipErrorNotReady) continue;
                HIPC(q);
                if (*st != stamp[k & 1]) throw Error{BIM_EDEVICE, "GMRES step finished without its residual estimate"};
            }
            std::atomic_thread_fence(std::memory_order_acquire);
            return resh[2 * (k & 1)];
        };
        int next = 0;  // the next step to enqueue
        auto enqueue_to = [&](int k) {
            while (next <= k && next < kmax) step(next++);
        };
        enqueue_to(0);
        auto t_prev = std::chrono::steady_clock::now();
        double t_step = 0.0;  // host-observed duration of the latest step, ms
        for (int k = 0; k < kmax; ++k) {
            enqueue_to(k);                                        // (already there when enqueued ahead)
            if (k == 0 || t_step < kAheadMs) enqueue_to(k + 1);  // one step ahead while steps are short
            const double r = wait_step(k);
            const auto t_now = std::chrono::steady_clock::now();
            t_step = std::chrono::duration<double, std::milli>(t_now - t_prev).count();
            t_prev = t_now;
            ++iters;
            ++nmv;
            kdone = k + 1;
            relres = r;
            if (r <= tol) {
                conv = true;
                break;
            }
        }
        // x += V y with R y = g over the completed steps (stream-ordered for
        // what follows: a converged solve returns without waiting for it)
        launch_backsub(c.stream, kdone, ga.H, ldH, ga.g, c.ybuf.d());
        launch_lincomb(c.stream, n, kdone, V, n, c.ybuf.d(), x);
        if (conv) return BIM_OK;
        HIPC(hipStreamSynchronize(c.stream));
        if (iters >= c.opt.gmres_maxit) return BIM_ENOCONV;
    }
}

// GMRES on the second-kind operator of the velocity (coefficients [3][Ctot])
static int gmres(Ctx &c, const double *b, double *x, const std::vector<double> &wt, double tol, int &iters,
                 double &relres, int &nmv)
{
    return gmres_op(
        c, 3 * c.Ctot, [&](const double *u, double *y) { apply_operator(c, u, y, wt); }, b, x, tol, iters, relres,
        nmv);
}

// --------------------------------------------------------------------------
// helpers for inputs / outputs
// --------------------------------------------------------------------------
static void copy_in(Ctx &c, void *dst, const void *src, size_t bytes, int mem_kind)
{
    if (bytes == 0) return;
    HIPC(hipMemcpyAsync(dst, src, bytes, mem_kind == BIM_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        c.stream));
    if (mem_kind != BIM_MEM_DEVICE) HIPC(hipStreamSynchronize(c.stream));
}

static void copy_out(Ctx &c, void *dst, const void *src, size_t bytes, int mem_kind)
{
    if (bytes == 0) return;
    HIPC(hipMemcpyAsync(dst, src, bytes, mem_kind == BIM_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        c.stream));
    if (mem_kind != BIM_MEM_DEVICE) HIPC(hipStreamSynchronize(c.stream));
}

static void invalidate(Ctx &c)
{
    c.nodes_ok = c.force_ok = c.regions_ok = false;
    c.regions_exact = false;
    c.pack_h.clear();
    c.pack_max0 = c.pack_max1 = 0;
    std::fill(c.Mok.begin(), c.Mok.end(), 0);
}

static void require_drops(Ctx &c) { REQUIRE(c.nd > 0, BIM_ESTATE, "no drops set (call bim_set_drops first)"); }

template <class F> static int guarded(Ctx *c, F &&f)
{
    if (!c) return BIM_EINVAL;
    try {
        HIPC(hipSetDevice(c->device));
        // work left on the second stream by a call that failed midway is
        // ordered before anything this call enqueues
        join_side(*c);
        int rc = f();
        if (rc == BIM_OK) c->err.clear();
        return rc;
    } catch (const Error &e) {
        c->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        c->err = "host allocation failed";
        return BIM_ENOMEM;
    } catch (const std::exception &e) {
        c->err = e.what();
        return BIM_EDEVICE;
    } catch (...) {
        c->err = "unknown error";
        return BIM_EDEVICE;
    }
}

}  // namespace bim

using namespace bim;

struct bim_ctx_s {
    Ctx c;
};

extern "C" {

int bim_version(void) { return 100; }

const char *bim_status_string(int s)
{
    switch (s) {
    case BIM_OK: return "ok";
    case BIM_EINVAL: return "invalid argument";
    case BIM_ENOMEM: return "out of memory";
    case BIM_EDEVICE: return "device error";
    case BIM_ENOCONV: return "GMRES did not converge";
    case BIM_ESTATE: return "invalid call order";
    case BIM_EAGAIN: return "request not finished";
    case BIM_EBUSY: return "server queue full";
    default: return "unknown status";
    }
}

int bim_default_options(bim_options *o)
{
    if (!o) return BIM_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->device = 0;
    o->precision = BIM_PREC_FP64;
    o->A_tilde = 5.0;
    o->U_tilde = 4;
    o->U_sing = 1;
    o->U_geom = 2;
    o->lambda_rule = 0;
    o->gmres_tol = 1e-10;
    o->gmres_restart = 50;
    o->gmres_maxit = 500;
    o->singular_path = 0;
    o->stream = nullptr;
    o->near_rule = 1;
    o->near_L = 8;
    o->fmm_order = 0;
    o->fmm_eps = 1e-10;
    o->pair_tune = 1;
    o->xform_path = 0;
    o->pipe_budget_gb = 8.0;
    return BIM_OK;
}

// --------------------------------------------------------------------------
// Scratch of bim_apply_double_layer_noalloc: the partial sums of the pair
// work items (the buffer pair_part of the other entry points), in a
// file-scope device array. Every GPU the library runs on holds its own copy
// until the process ends; its device address is looked up once per device
// (in bim_create, with the device current) and kept in g_scratch.
// --------------------------------------------------------------------------
constexpr size_t kScratchDoubles = (size_t)1 << 25;  // 256 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch[kMaxDevices];
static bool g_scratch_tried[kMaxDevices];

// The device address of `scratch` on the current device `dev` (nullptr if the
// lookup failed or dev is out of range).
static double *scratch_on(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_tried[dev]) {
        g_scratch_tried[dev] = true;
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch[dev] = static_cast<double *>(p);
        else (void)hipGetLastError();
    }
    return g_scratch[dev];
}

int bim_create(const bim_options *opt, bim_ctx *out)
{
    if (!opt || !out) return BIM_EINVAL;
    *out = nullptr;
    if ((opt->precision != BIM_PREC_FP64 && opt->precision != BIM_PREC_MIXED) || opt->U_tilde < 1 || opt->U_sing < 1 || opt->U_geom < 1 ||
        !(opt->A_tilde >= 0.0) || !(opt->gmres_tol > 0.0) || opt->gmres_restart < 1 || opt->gmres_maxit < 0 ||
        (opt->lambda_rule != 0 && opt->lambda_rule != 1) || (opt->singular_path < 0 || opt->singular_path > 2) ||
        (opt->near_rule != 0 && opt->near_rule != 1) || opt->near_L < 2 || opt->near_L > kNearMaxL ||
        (opt->fmm_order != 0 && opt->fmm_order != -1 && (opt->fmm_order < 2 || opt->fmm_order > kFmmMaxOrder)) ||
        !(opt->fmm_eps > 0.0 && opt->fmm_eps < 1.0) || opt->xform_path < 0 || opt->xform_path > 2 ||
        !(opt->pipe_budget_gb > 0.0 && opt->pipe_budget_gb < 1e6))
        return BIM_EINVAL;
    bim_ctx h = nullptr;
    try {
        h = new bim_ctx_s();
    } catch (...) {
        return BIM_ENOMEM;
    }
    Ctx &c = h->c;
    c.opt = *opt;
    c.device = opt->device;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || opt->device < 0 || opt->device >= ndev) {
        delete h;
        return BIM_EDEVICE;
    }
    if (hipSetDevice(opt->device) != hipSuccess) {
        delete h;
        return BIM_EDEVICE;
    }
    (void)scratch_on(opt->device);  // once per device: the no-allocation entry point's scratch
    if (opt->stream) {
        c.stream = static_cast<hipStream_t>(opt->stream);
    } else {
        // non-blocking: no implicit ordering with the null stream, so that
        // contexts on other threads never wait for each other
        if (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess) {
            delete h;
            return BIM_EDEVICE;
        }
        c.own_stream = true;
    }
    *out = h;
    return BIM_OK;
}

int bim_destroy(bim_ctx h)
{
    if (!h) return BIM_EINVAL;
    (void)hipSetDevice(h->c.device);
    if (h->c.stream) (void)hipStreamSynchronize(h->c.stream);
    delete h;
    return BIM_OK;
}

const char *bim_last_error(bim_ctx h) { return h ? h->c.err.c_str() : "null context"; }

int bim_synchronize(bim_ctx h)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        HIPC(hipStreamSynchronize(h->c.stream));
        return BIM_OK;
    });
}

int bim_set_drops(bim_ctx h, int n_drops, const int *p, const double *xcoef, const double *lambda, int mem_kind)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        REQUIRE(n_drops >= 1 && p && xcoef && lambda, BIM_EINVAL, "bim_set_drops: null argument or no drops");
        REQUIRE(mem_kind == BIM_MEM_HOST || mem_kind == BIM_MEM_DEVICE, BIM_EINVAL, "bad mem_kind");
        c.fmm_tuned = -1;  // a new system: choose the fast-summation order again
        c.pair_tuned = false;
        c.pair_T_fix = c.pair_ch = 0;
        std::vector<Drop> ds(n_drops);
        long coff = 0, toff = 0, uoff = 0;
        for (int i = 0; i < n_drops; ++i) {
            REQUIRE(p[i] >= 2 && p[i] <= 64, BIM_EINVAL, "degree p out of range [2, 64]");
            REQUIRE(std::isfinite(lambda[i]) && lambda[i] >= 0.0, BIM_EINVAL, "lambda must be finite and >= 0");
            ds[i].p = p[i];
            ds[i].lam = lambda[i];
            ds[i].coff = coff;
            ds[i].toff = toff;
            ds[i].uoff = uoff;
            ds[i].qu = c.opt.U_tilde * p[i];
            ds[i].qg = c.opt.U_geom * p[i];
            ds[i].qs = c.opt.U_sing * p[i];
            REQUIRE(ds[i].qu <= 512 && ds[i].qg <= 512 && ds[i].qs <= 256, BIM_EINVAL, "grid degree too large");
            coff += 2L * ncoef(p[i]);
            toff += npts(p[i]);
            uoff += npts(ds[i].qu);
        }
        // validate coefficients on the host
        std::vector<double> hx((size_t)3 * coff);
        if (mem_kind == BIM_MEM_DEVICE) {
            HIPC(hipMemcpyAsync(hx.data(), xcoef, hx.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
            HIPC(hipStreamSynchronize(c.stream));
        } else {
            std::memcpy(hx.data(), xcoef, hx.size() * sizeof(double));
        }
        for (double v : hx) REQUIRE(std::isfinite(v), BIM_EINVAL, "non-finite surface coefficient");
        c.nd = n_drops;
        c.drops = ds;
        c.xplans.clear();
        for (auto &row : c.xmode) row[0] = row[1] = -1;
        if ((int)c.Mdl.size() < n_drops) c.Mdl.resize(n_drops);
        c.Mok.assign(n_drops, 0);
        c.Ctot = coff;
        c.T = toff;
        c.S1 = uoff;
        // uploads from pinned host images: enqueued without waiting, all
        // complete at the synchronisation that ends this call
        auto up = [&](DBuf &d, auto &img) {
            d.ensure(std::max<size_t>(1, img.size()) * sizeof(img[0]));
            if (!img.empty())
                HIPC(hipMemcpyAsync(d.ptr, img.data(), img.size() * sizeof(img[0]), hipMemcpyHostToDevice, c.stream));
        };
        c.h_xc.assign(hx.begin(), hx.end());
        up(c.xc, c.h_xc);
        c.gc.ensure((size_t)coff * sizeof(double));
        HIPC(hipMemsetAsync(c.gc.ptr, 0, (size_t)coff * sizeof(double), c.stream));
        c.fc.ensure((size_t)3 * coff * sizeof(double));
        c.eos = BIM_EOS_UNIFORM;
        c.sigma0 = 1.0;
        c.E = c.xs = 0.0;
        c.have_gamma = false;
        c.tx.ensure((size_t)3 * c.T * sizeof(double));
        c.s0N.ensure((size_t)3 * c.T * sizeof(double));
        c.s0W.ensure((size_t)c.T * sizeof(double));
        c.s0d.ensure((size_t)3 * c.T * sizeof(double));
        c.s1x.ensure((size_t)3 * c.S1 * sizeof(double));
        c.s1N.ensure((size_t)3 * c.S1 * sizeof(double));
        c.s1W.ensure((size_t)c.S1 * sizeof(double));
        c.s1d.ensure((size_t)3 * c.S1 * sizeof(double));
        c.acc.ensure((size_t)3 * c.T * sizeof(double));
        c.tmp.ensure((size_t)3 * c.T * sizeof(double));
        c.bvec.ensure((size_t)3 * c.Ctot * sizeof(double));
        c.xsol.ensure((size_t)3 * c.Ctot * sizeof(double));
        HVec<int> &tdrop = c.h_tdrop, &noff = c.h_noff, &ncnt = c.h_ncnt, &unoff = c.h_unoff, &uncnt = c.h_uncnt;
        tdrop.resize(c.T);
        noff.resize(c.nd);
        ncnt.resize(c.nd);
        unoff.resize(c.nd);
        uncnt.resize(c.nd);
        for (int i = 0; i < c.nd; ++i) {
            for (int t = 0; t < npts(ds[i].p); ++t) tdrop[ds[i].toff + t] = i;
            noff[i] = (int)ds[i].toff;
            ncnt[i] = npts(ds[i].p);
            unoff[i] = (int)ds[i].uoff;
            uncnt[i] = npts(ds[i].qu);
        }
        c.sys_h.assign(c.nd, 0);
        c.h_sys.assign(c.nd, 0);
        up(c.sysd, c.h_sys);
        up(c.tdrop, tdrop);
        up(c.noff, noff);
        up(c.ncnt, ncnt);
        c.h_hfac.resize(c.nd);
        for (int i = 0; i < c.nd; ++i) c.h_hfac[i] = kPi / (ds[i].p + 1);
        up(c.hfac, c.h_hfac);
        up(c.unoff, unoff);
        up(c.uncnt, uncnt);
        // Galerkin operator diagonal (lambda_i + 1)
        HVec<double> &scl = c.h_scl;
        scl.resize((size_t)3 * c.Ctot);
        for (int comp = 0; comp < 3; ++comp)
            for (int i = 0; i < c.nd; ++i)
                for (long e = 0; e < 2L * ncoef(ds[i].p); ++e) scl[comp * c.Ctot + ds[i].coff + e] = ds[i].lam + 1.0;
        up(c.scl, scl);
        c.h_gU.assign(c.gradU, c.gradU + 9);
        up(c.gU, c.h_gU);
        invalidate(c);
        // tables for every grid in use
        for (auto &d : ds) {
            grid(c, d.p, d.p);
            grid(c, d.qu, d.p);
            grid(c, d.qg, d.p);
            grid(c, d.qs, d.p);
            rot(c, d.p);
        }
        HIPC(hipStreamSynchronize(c.stream));
        return BIM_OK;
    });
}

int bim_set_systems(bim_ctx h, const int *system_of_drop)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        require_drops(c);
        REQUIRE(system_of_drop, BIM_EINVAL, "null system array");
        for (int i = 0; i < c.nd; ++i) REQUIRE(system_of_drop[i] >= 0, BIM_EINVAL, "negative system id");
        c.sys_h.assign(system_of_drop, system_of_drop + c.nd);
        HIPC(hipMemcpyAsync(c.sysd.ptr, c.sys_h.data(), c.nd * sizeof(int), hipMemcpyHostToDevice, c.stream));
        HIPC(hipStreamSynchronize(c.stream));
        c.regions_ok = false;
        c.regions_exact = false;
        c.fmm_tuned = -1;  // other drop pairs: choose the fast-summation order again
        c.pair_tuned = false;
        c.pair_T_fix = c.pair_ch = 0;
        return BIM_OK;
    });
}

int bim_set_tension(bim_ctx h, const double *gamma_coef, int eos, double E, double xs, double sigma0, int mem_kind)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        require_drops(c);
        REQUIRE(eos >= 0 && eos <= 2, BIM_EINVAL, "bad equation of state");
        REQUIRE(eos == BIM_EOS_UNIFORM || gamma_coef, BIM_EINVAL, "gamma_coef required for this equation of state");
        REQUIRE(std::isfinite(E) && std::isfinite(xs) && std::isfinite(sigma0), BIM_EINVAL, "non-finite parameter");
        c.eos = eos;
        c.E = E;
        c.xs = xs;
        c.sigma0 = sigma0;
        if (gamma_coef) {
            std::vector<double> hg((size_t)c.Ctot);
            if (mem_kind == BIM_MEM_DEVICE) {
                HIPC(hipMemcpyAsync(hg.data(), gamma_coef, hg.size() * sizeof(double), hipMemcpyDeviceToHost,
                                    c.stream));
                HIPC(hipStreamSynchronize(c.stream));
            } else {
                std::memcpy(hg.data(), gamma_coef, hg.size() * sizeof(double));
            }
            for (double v : hg) REQUIRE(std::isfinite(v), BIM_EINVAL, "non-finite surfactant coefficient");
            HIPC(hipMemcpyAsync(c.gc.ptr, hg.data(), hg.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
            HIPC(hipStreamSynchronize(c.stream));
            c.have_gamma = true;
        }
        c.force_ok = false;
        return BIM_OK;
    });
}

int bim_set_farfield(bim_ctx h, const double U0[3], const double gradU[9])
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        for (int i = 0; i < 3; ++i) c.U0[i] = U0 ? U0[i] : 0.0;
        for (int i = 0; i < 9; ++i) c.gradU[i] = gradU ? gradU[i] : 0.0;
        for (int i = 0; i < 3; ++i) REQUIRE(std::isfinite(c.U0[i]), BIM_EINVAL, "non-finite U0");
        for (int i = 0; i < 9; ++i) REQUIRE(std::isfinite(c.gradU[i]), BIM_EINVAL, "non-finite gradU");
        c.gU.ensure(9 * sizeof(double));
        HIPC(hipMemcpyAsync(c.gU.ptr, c.gradU, 9 * sizeof(double), hipMemcpyHostToDevice, c.stream));
        HIPC(hipStreamSynchronize(c.stream));
        return BIM_OK;
    });
}

int bim_force(bim_ctx h, double *f_coef, int mem_kind)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        require_drops(c);
        REQUIRE(f_coef, BIM_EINVAL, "null output");
        build_force(c);
        copy_out(c, f_coef, c.fc.ptr, (size_t)3 * c.Ctot * sizeof(double), mem_kind);
        return BIM_OK;
    });
}

int bim_regions(bim_ctx h, int8_t *regions, double *dist, int mem_kind)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        require_drops(c);
        if (dist && !c.regions_exact) {
            c.regions_exact = true;
            c.regions_ok = false;
        }
        build_regions(c);
        if (regions) copy_out(c, regions, c.reg.ptr, (size_t)c.T * c.nd, mem_kind);
        if (dist) copy_out(c, dist, c.dist.ptr, (size_t)c.T * c.nd * sizeof(double), mem_kind);
        return BIM_OK;
    });
}

int bim_single_layer(bim_ctx h, const double *f_coef, double *out, int mem_kind)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        require_drops(c);
        REQUIRE(out, BIM_EINVAL, "null output");
        const double *dens;
        if (f_coef) {
            c.bvec.ensure((size_t)3 * c.Ctot * sizeof(double));
            copy_in(c, c.bvec.ptr, f_coef, (size_t)3 * c.Ctot * sizeof(double), mem_kind);
            dens = c.bvec.d();
        } else {
            build_force(c);
            dens = c.fc.d();
        }
        single_layer_grid(c, dens);
        launch_scale_add(c.stream, 3 * c.T, -1.0 / (8.0 * kPi), c.acc.d(), 0.0, c.acc.d());
        copy_out(c, out, c.acc.ptr, (size_t)3 * c.T * sizeof(double), mem_kind);
        return BIM_OK;
    });
}

// --------------------------------------------------------------------------
// Drop and surfactant time step (Sec. 3, Algorithm 1): explicit midpoint rule
// for the drops, second-order IMEX for the surfactant, conservation error.
// --------------------------------------------------------------------------
// per-drop offsets into the surface-field buffer (33 fields on the degree
// U_geom p grid) and into the grid outputs (2 fields)
static void surf_layout(Ctx &c, std::vector<long> &so, std::vector<long> &go, long &stot, long &gtot)
{
    so.resize(c.nd);
    go.resize(c.nd);
    stot = gtot = 0;
    for (int i = 0; i < c.nd; ++i) {
        const long np = npts(c.drops[i].qg);
        so[i] = stot;
        go[i] = gtot;
        stot += 33 * np;
        gtot += 2 * np;
    }
}

// synthesis on the degree U_geom p grid of each drop: x (6 derivative fields
// x 3 components), Gamma (6 fields), u (3 fields x 3 components); a null
// argument leaves those fields as they are
static void surf_synth(Ctx &c, const double *x, const double *g, const double *u)
{
    std::vector<long> so, go;
    long stot, gtot;
    surf_layout(c, so, go, stot, gtot);
    c.ts_syn.ensure((size_t)stot * sizeof(double));
    std::vector<SynJob> jobs;
    for (int i = 0; i < c.nd; ++i) {
        const Drop &d = c.drops[i];
        const long np = npts(d.qg);
        double *s = c.ts_syn.d() + so[i];
        if (x) jobs.push_back(syn_job(c, d.p, d.qg, 3, x + d.coff, c.Ctot, 0x3f, s, np, 3 * np));
        if (g) jobs.push_back(syn_job(c, d.p, d.qg, 1, g + d.coff, 0, 0x3f, s + 18 * np, 0, np));
        if (u) jobs.push_back(syn_job(c, d.p, d.qg, 3, u + d.coff, c.Ctot, 0x7, s + 24 * np, np, 3 * np));
    }
    syn_run(c, jobs);
}

// surface terms from the fields in ts_syn: -Gamma div_s u into fEc and the
// Laplace-Beltrami of Gamma into lgc (coefficients to degree p, layout
// [Ctot]); int Gamma dS into mass[nd] and the enclosed volume into vol[nd]
static void surf_terms(Ctx &c, bool gam, double *fEc, double *lgc, double *mass, double *vol)
{
    std::vector<long> so, go;
    long stot, gtot;
    surf_layout(c, so, go, stot, gtot);
    c.ts_grid.ensure((size_t)gtot * sizeof(double));
    if (mass) HIPC(hipMemsetAsync(mass, 0, c.nd * sizeof(double), c.stream));
    if (vol) HIPC(hipMemsetAsync(vol, 0, c.nd * sizeof(double), c.stream));
    std::vector<SurfJob> jobs;
    std::vector<AnaJob> ajobs;
    for (int i = 0; i < c.nd; ++i) {
        const Drop &d = c.drops[i];
        const long np = npts(d.qg);
        SurfJob j{};
        j.syn = c.ts_syn.d() + so[i];
        j.wreg = grid(c, d.qg, d.p).wreg.d();
        j.fE = fEc ? c.ts_grid.d() + go[i] : nullptr;
        j.lg = lgc ? c.ts_grid.d() + go[i] + np : nullptr;
        j.mass = mass ? mass + i : nullptr;
        j.vol = vol ? vol + i : nullptr;
        j.np = np;
        j.q = d.qg;
        j.gam = gam ? 1 : 0;
        jobs.push_back(j);
        if (fEc) ajobs.push_back(ana_job(c, d.qg, d.p, 1, j.fE, 0, fEc + d.coff, 0));
        if (lgc) ajobs.push_back(ana_job(c, d.qg, d.p, 1, j.lg, 0, lgc + d.coff, 0));
    }
    {
        ProfScope ps(c, "surface_terms", 0.0, 0.0);
        launch_surf_terms(c.stream, jobs.data(), (int)jobs.size());
    }
    if (!ajobs.empty()) ana_run(c, ajobs);
}

static void dcopy(Ctx &c, double *dst, const double *src, long n)
{
    HIPC(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
}

static std::vector<double> dget(Ctx &c, const double *src, long n)
{
    std::vector<double> h(n);
    HIPC(hipMemcpyAsync(h.data(), src, n * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    HIPC(hipStreamSynchronize(c.stream));
    return h;
}

static int solve_velocity(Ctx &c, int &iters, double &relres, int &nmv);

// One step from the context's state. On return the context holds the state
// at t + dt when accepted, else the state at t.
static int time_step(Ctx &c, double dt, double Pe, double tol, bim_step_report &r)
{
    const long n3 = 3 * c.Ctot, n1 = c.Ctot;
    const bool surf = c.have_gamma;
    const bool diff = surf && std::isfinite(Pe);
    for (DBuf *b : {&c.ts_x0, &c.ts_u0, &c.ts_uh, &c.ts_xh}) b->ensure((size_t)n3 * sizeof(double));
    for (DBuf *b : {&c.ts_g0, &c.ts_gh, &c.ts_fe, &c.ts_ki, &c.ts_ke, &c.ts_sinv, &c.ts_w, &c.ts_lw, &c.ts_z})
        b->ensure((size_t)n1 * sizeof(double));
    c.ts_acc.ensure((size_t)3 * c.nd * sizeof(double));
    double *m0 = c.ts_acc.d(), *m1 = m0 + c.nd, *vol = m1 + c.nd;
    double *x0 = c.ts_x0.d(), *g0 = c.ts_g0.d(), *u0 = c.ts_u0.d(), *uh = c.ts_uh.d(), *xh = c.ts_xh.d(),
           *gh = c.ts_gh.d(), *fe = c.ts_fe.d(), *ki = c.ts_ki.d(), *ke = c.ts_ke.d();
    dcopy(c, x0, c.xc.d(), n3);
    if (surf) dcopy(c, g0, c.gc.d(), n1);
    auto restore = [&]() {
        dcopy(c, c.xc.d(), x0, n3);
        if (surf) dcopy(c, c.gc.d(), g0, n1);
        invalidate(c);
        HIPC(hipStreamSynchronize(c.stream));
    };
    // velocity at t
    int it = 0, nmv = 0;
    double rr = 0.0;
    int rc = solve_velocity(c, it, rr, nmv);
    r.gmres_velocity[0] = it;
    if (rc != BIM_OK) {
        restore();
        return rc;
    }
    dcopy(c, u0, c.xsol.d(), n3);
    if (surf) {
        surf_synth(c, x0, g0, u0);
        surf_terms(c, true, fe, nullptr, m0, nullptr);
    }
    // half step: x + dt/2 u; (I - dt/(2 Pe) L) Gamma_h = Gamma + dt/2 fE
    launch_axpby(c.stream, n3, 1.0, x0, 0.5 * dt, u0, xh);
    r.gmres_imex = 0;
    if (surf) {
        launch_axpby(c.stream, n1, 1.0, g0, 0.5 * dt, fe, gh);  // right-hand side, then the stage value
        if (diff) {
            const double cf = 0.5 * dt / Pe;
            surf_synth(c, xh, nullptr, nullptr);
            surf_terms(c, false, nullptr, nullptr, nullptr, vol);
            // right preconditioner: the operator's diagonal on the sphere of each
            // drop's volume-equivalent radius, 1 + cf n (n + 1) / R^2 (Sec. 3.2.1)
            const std::vector<double> hv = dget(c, vol, c.nd);
            std::vector<double> sinv(n1);
            for (int i = 0; i < c.nd; ++i) {
                const Drop &d = c.drops[i];
                const double R = std::cbrt(3.0 * hv[i] / (4.0 * kPi));
                for (int n = 0; n <= d.p; ++n)
                    for (int m = 0; m <= n; ++m) {
                        const long e = d.coff + 2L * (n * (n + 1) / 2 + m);
                        sinv[e] = sinv[e + 1] = 1.0 / (1.0 + cf * n * (n + 1) / (R * R));
                    }
            }
            HIPC(hipMemcpyAsync(c.ts_sinv.ptr, sinv.data(), n1 * sizeof(double), hipMemcpyHostToDevice, c.stream));
            HIPC(hipStreamSynchronize(c.stream));
            double *si = c.ts_sinv.d(), *w = c.ts_w.d(), *lw = c.ts_lw.d(), *z = c.ts_z.d();
            auto op = [&](const double *zin, double *y) {  // y = (I - cf L) S^-1 zin
                launch_mul(c.stream, n1, si, zin, w);
                surf_synth(c, nullptr, w, nullptr);
                surf_terms(c, true, nullptr, lw, nullptr, nullptr);
                launch_axpby(c.stream, n1, 1.0, w, -cf, lw, y);
            };
            int nm2 = 0;
            rc = gmres_op(c, n1, op, gh, z, c.opt.gmres_tol, it, rr, nm2);
            r.gmres_imex = it;
            if (rc != BIM_OK) {
                restore();
                return rc;
            }
            launch_mul(c.stream, n1, si, z, gh);
            // L Gamma_h (the implicit stage slope times Pe)
            surf_synth(c, nullptr, gh, nullptr);
            surf_terms(c, true, nullptr, ki, nullptr, nullptr);
        }
    }
    // velocity at t + dt/2
    dcopy(c, c.xc.d(), xh, n3);
    if (surf) dcopy(c, c.gc.d(), gh, n1);
    rc = solve_velocity(c, it, rr, nmv);
    r.gmres_velocity[1] = it;
    if (rc != BIM_OK) {
        restore();
        return rc;
    }
    dcopy(c, uh, c.xsol.d(), n3);
    // full step: x0 + dt u_h; Gamma0 + dt (fE_h + L Gamma_h / Pe)
    launch_axpby(c.stream, n3, 1.0, x0, dt, uh, c.xc.d());
    double mass0 = 0.0, mass1 = 0.0, esurf = 0.0;
    if (surf) {
        surf_synth(c, xh, gh, uh);
        surf_terms(c, true, ke, nullptr, nullptr, nullptr);
        if (diff) launch_axpby(c.stream, n1, 1.0, ke, 1.0 / Pe, ki, ke);
        launch_axpby(c.stream, n1, 1.0, g0, dt, ke, c.gc.d());
        surf_synth(c, c.xc.d(), c.gc.d(), nullptr);
        surf_terms(c, true, nullptr, nullptr, m1, nullptr);
        const std::vector<double> hm = dget(c, m0, 2 * c.nd);
        for (int i = 0; i < c.nd; ++i) {
            mass0 += hm[i];
            mass1 += hm[c.nd + i];
            esurf = std::max(esurf, std::fabs(hm[c.nd + i] - hm[i]) / std::fabs(hm[i]));
        }
    }
    // drop error: midpoint against the explicit Euler row, ||x1 - x_E|| = dt ||u_h - u_0||
    const std::vector<double> hu0 = dget(c, u0, n3), huh = dget(c, uh, n3), hx1 = dget(c, c.xc.d(), n3);
    double sd = 0.0, sx = 0.0;
    for (long e = 0; e < n3; ++e) {
        const double d = dt * (huh[e] - hu0[e]);
        sd += d * d;
        sx += hx1[e] * hx1[e];
    }
    r.err_drop = std::sqrt(sd / sx);
    r.err_surf = esurf;
    r.mass0 = mass0;
    r.mass1 = mass1;
    const double err = std::max(r.err_drop, r.err_surf);
    r.accepted = (tol <= 0.0 || err < tol) ? 1 : 0;
    r.dt_next = (tol > 0.0 && err > 0.0) ? dt * std::sqrt(0.9 * tol / err) : dt;
    if (!r.accepted) restore();
    invalidate(c);
    HIPC(hipStreamSynchronize(c.stream));
    return BIM_OK;
}

int bim_time_step(bim_ctx h, double dt, double Pe, double tol, bim_step_report *rep)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        require_drops(c);
        REQUIRE(std::isfinite(dt) && dt > 0.0, BIM_EINVAL, "dt must be finite and > 0");
        REQUIRE(Pe > 0.0 && !std::isnan(Pe), BIM_EINVAL, "Pe must be > 0 (infinity: no diffusion)");
        REQUIRE(std::isfinite(tol), BIM_EINVAL, "tol must be finite");
        auto t0 = std::chrono::steady_clock::now();
        bim_step_report r{};
        const int rc = time_step(c, dt, Pe, tol, r);
        r.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (rep) *rep = r;
        return rc;
    });
}

int bim_get_state(bim_ctx h, double *xcoef, double *gamma_coef, int mem_kind)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        require_drops(c);
        REQUIRE(mem_kind == BIM_MEM_HOST || mem_kind == BIM_MEM_DEVICE, BIM_EINVAL, "bad mem_kind");
        REQUIRE(!gamma_coef || c.have_gamma, BIM_ESTATE, "no surfactant set (bim_set_tension with gamma_coef)");
        if (xcoef) copy_out(c, xcoef, c.xc.ptr, (size_t)3 * c.Ctot * sizeof(double), mem_kind);
        if (gamma_coef) copy_out(c, gamma_coef, c.gc.ptr, (size_t)c.Ctot * sizeof(double), mem_kind);
        HIPC(hipStreamSynchronize(c.stream));
        return BIM_OK;
    });
}

// --------------------------------------------------------------------------
// Angle reparametrization (Sec. 4, Algorithm 2)
// --------------------------------------------------------------------------
// Recursion coefficients of the orthonormal associated Legendre functions of
// degree <= q at tri(n, m): a_nm = sqrt((2n+1)(2n-1)/((n-m)(n+m))),
// b_nm = sqrt((2n+1)(n+m-1)(n-m-1)/((2n-3)(n-m)(n+m))) (n >= m + 2),
// d_nm = sqrt((2n+1)(n^2-m^2)/(2n-1)); then c_m = (4 pi)^(-1/2) prod_{k<=m} -sqrt((2k+1)/(2k)).
// Recursion records of the degree-q point evaluation, order-major: for
// m = 0..q, n = m..q the 4 doubles {a, b, d, n} of
//   P_n^m = a cos(theta) P_{n-1}^m - b P_{n-2}^m,
//   sin(theta) dP_n^m/dtheta = n cos(theta) P_n^m - d P_{n-1}^m,
// with (a, b) = (0, -1) at n = m (the start value c_m sin^m(theta) enters as
// P_{m-2}) and (sqrt(2m+3), 0) at n = m + 1; then c_m for m = 0..q.
static const double *rep_table(Ctx &c, int q)
{
    auto it = c.rp_tab.find(q);
    if (it != c.rp_tab.end()) return it->second->d();
    const long R = (long)(q + 1) * (q + 2) / 2;
    std::vector<double> t(4 * R + q + 1, 0.0);
    long j = 0;
    for (int m = 0; m <= q; ++m)
        for (int n = m; n <= q; ++n, ++j) {
            double *h = &t[4 * j];
            if (n == m) {
                h[0] = 0.0;
                h[1] = -1.0;
            } else if (n == m + 1) {
                h[0] = std::sqrt(2.0 * m + 3.0);
            } else {
                h[0] = std::sqrt((2.0 * n + 1.0) * (2.0 * n - 1.0) / ((double)(n - m) * (n + m)));
                h[1] = std::sqrt((2.0 * n + 1.0) * (double)(n + m - 1) * (n - m - 1) /
                                 ((2.0 * n - 3.0) * (double)(n - m) * (n + m)));
            }
            if (n > m) h[2] = std::sqrt((2.0 * n + 1.0) * (double)(n - m) * (n + m) / (2.0 * n - 1.0));
            h[3] = n;
        }
    double cm = 1.0 / std::sqrt(4.0 * kPi);
    for (int m = 0; m <= q; ++m) {
        if (m > 0) cm *= -std::sqrt((2.0 * m + 1.0) / (2.0 * m));
        t[4 * R + m] = cm;
    }
    auto buf = std::make_unique<DBuf>();
    buf->ensure(t.size() * sizeof(double));
    HIPC(hipMemcpyAsync(buf->ptr, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
    HIPC(hipStreamSynchronize(c.stream));
    const double *d = buf->d();
    c.rp_tab[q] = std::move(buf);
    return d;
}

struct RepOut {
    int moves = 0, ncut = 0;
    double gnorm = 0.0;
};

// Algorithm 2 on the drops `ids`, all of degree p, as one batch: the
// initial expansions (degree p, zero-padded to q = U p) stay fixed; the
// angles of the degree-q grid nodes move by forward Euler steps of the
// parameter velocity of w = -(I - n n) grad E, grad E the field of the
// coefficients of degree >= n_cut. Each drop keeps its own cutoff, residual
// and stopping test. The drops' position (and surfactant) coefficients are
// replaced by the analysis of the initial expansions at the final angles,
// truncated to degree p.
static RepOut reparam_group(Ctx &c, const std::vector<int> &ids, int U, double P_cut, double eps, int imax,
                            double dtau)
{
    const int nb = (int)ids.size();
    const int p = c.drops[ids[0]].p, q = U * p;
    const long N = npts(q), nq2 = 2L * ncoef(q), np2 = 2L * ncoef(p);
    GridTab &gq = grid(c, q, q);
    const long R = ncoef(q);
    const double *hdr = rep_table(c, q), *cmt = hdr + 4 * R;
    c.rp_rec.ensure((size_t)nb * 10 * R * sizeof(double));
    c.rp_x0.ensure((size_t)nb * 3 * nq2 * sizeof(double));
    c.rp_g0.ensure((size_t)nb * nq2 * sizeof(double));
    c.rp_xt.ensure((size_t)nb * 3 * nq2 * sizeof(double));
    c.rp_hp.ensure((size_t)nb * 3 * nq2 * sizeof(double));
    c.rp_ang.ensure((size_t)nb * 2 * N * sizeof(double));
    c.rp_E.ensure((size_t)nb * 9 * N * sizeof(double));
    c.rp_gE.ensure((size_t)nb * 3 * N * sizeof(double));
    c.rp_g.ensure((size_t)nb * 3 * N * sizeof(double));
    c.rp_gmax.ensure((size_t)nb * 2 * sizeof(double));  // residual bits [nb], then cutoff [nb] and moves [nb]
    double *x0 = c.rp_x0.d(), *g0 = c.rp_g0.d(), *xt = c.rp_xt.d(), *hp = c.rp_hp.d(), *th = c.rp_ang.d(),
           *ph = th + N, *E = c.rp_E.d(), *gE = c.rp_gE.d(), *g = c.rp_g.d();
    auto *gmax = (unsigned long long *)c.rp_gmax.ptr;
    int *dnc = (int *)(gmax + nb), *dmoves = dnc + nb;
    const long A = 2 * N;  // angle stride between drops: th then ph
    HIPC(hipMemsetAsync(x0, 0, (size_t)nb * 3 * nq2 * sizeof(double), c.stream));
    for (int b = 0; b < nb; ++b)
        HIPC(hipMemcpy2DAsync(x0 + 3L * b * nq2, nq2 * sizeof(double), c.xc.d() + c.drops[ids[b]].coff,
                              c.Ctot * sizeof(double), np2 * sizeof(double), 3, hipMemcpyDeviceToDevice, c.stream));
    if (c.have_gamma) {
        HIPC(hipMemsetAsync(g0, 0, (size_t)nb * nq2 * sizeof(double), c.stream));
        for (int b = 0; b < nb; ++b) dcopy(c, g0 + b * nq2, c.gc.d() + c.drops[ids[b]].coff, np2);
    }
    std::vector<double> ang((size_t)nb * A);
    for (int j = 0; j <= q; ++j)
        for (int k = 0; k < 2 * q; ++k) {
            ang[(long)j * 2 * q + k] = gq.th[j];
            ang[N + (long)j * 2 * q + k] = kPi * k / q;
        }
    for (int b = 1; b < nb; ++b) std::copy(ang.begin(), ang.begin() + A, ang.begin() + (long)b * A);
    HIPC(hipMemcpyAsync(th, ang.data(), ang.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
    HIPC(hipMemsetAsync(dmoves, 0, nb * sizeof(int), c.stream));
    double *rec = c.rp_rec.d();
    launch_rep_pack(c.stream, q, 3, nb, x0, nq2, hdr, rec);
    std::vector<AnaJob> ajobs;
    std::vector<SynJob> sjobs;
    for (int b = 0; b < nb; ++b) {
        ajobs.push_back(ana_job(c, q, q, 3, E + 9 * N * b, 3 * N, xt + 3 * nq2 * b, nq2));
        sjobs.push_back(syn_job(c, q, q, 3, hp + 3 * nq2 * b, nq2, 0x1, gE + 3 * N * b, N, 0));
    }
    // x~ at the current angles, the cutoff and filter, grad E, g and its largest norm
    auto evaluate = [&]() {
        launch_rep_eval(c.stream, q, 3, nb, rec, cmt, th, ph, A, N, E);
        ana_run(c, ajobs);
        launch_rep_cut(c.stream, q, nb, xt, nq2, P_cut, hp, dnc, gmax);
        syn_run(c, sjobs);
        launch_rep_grad(c.stream, nb, N, E, gE, g, gmax);
    };
    // all iterations are enqueued at once: once a drop's max |g| < eps its
    // moves are skipped on the device and its evaluations repeat the final state
    evaluate();
    for (int it = 1; it < imax; ++it) {
        launch_rep_move(c.stream, nb, N, E, g, dtau, th, ph, A, gmax, eps, it > 1, dmoves);
        evaluate();
    }
    RepOut r;
    r.ncut = 1 << 30;
    {
        std::vector<char> hs((size_t)nb * 2 * sizeof(double));
        HIPC(hipMemcpyAsync(hs.data(), c.rp_gmax.ptr, hs.size(), hipMemcpyDeviceToHost, c.stream));
        HIPC(hipStreamSynchronize(c.stream));
        for (int b = 0; b < nb; ++b) {
            double gn;
            int nc, mv;
            std::memcpy(&gn, hs.data() + b * sizeof(double), sizeof(double));
            std::memcpy(&nc, hs.data() + nb * sizeof(double) + b * sizeof(int), sizeof(int));
            std::memcpy(&mv, hs.data() + nb * sizeof(double) + (nb + b) * sizeof(int), sizeof(int));
            r.gnorm = std::max(r.gnorm, gn);
            r.ncut = std::min(r.ncut, nc);
            r.moves = std::max(r.moves, mv);
        }
    }
    for (int b = 0; b < nb; ++b)
        HIPC(hipMemcpy2DAsync(c.xc.d() + c.drops[ids[b]].coff, c.Ctot * sizeof(double), xt + 3L * b * nq2,
                              nq2 * sizeof(double), np2 * sizeof(double), 3, hipMemcpyDeviceToDevice, c.stream));
    if (c.have_gamma) {
        launch_rep_pack(c.stream, q, 1, nb, g0, nq2, hdr, rec);
        launch_rep_eval(c.stream, q, 1, nb, rec, cmt, th, ph, A, N, E);
        std::vector<AnaJob> gjobs;
        for (int b = 0; b < nb; ++b) gjobs.push_back(ana_job(c, q, q, 1, E + 3 * N * b, 0, hp + nq2 * b, 0));
        ana_run(c, gjobs);
        for (int b = 0; b < nb; ++b) dcopy(c, c.gc.d() + c.drops[ids[b]].coff, hp + nq2 * b, np2);
    }
    HIPC(hipStreamSynchronize(c.stream));
    return r;
}

int bim_reparametrize(bim_ctx h, int U_rep, double P_cut, double eps, int imax, double dtau, bim_rep_report *rep)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        require_drops(c);
        REQUIRE(U_rep >= 1, BIM_EINVAL, "U_rep must be >= 1");
        for (auto &d : c.drops) REQUIRE(U_rep * d.p <= 64, BIM_EINVAL, "U_rep * p must be <= 64");
        REQUIRE(P_cut > 0.0 && P_cut <= 1.0, BIM_EINVAL, "P_cut must be in (0, 1]");
        REQUIRE(std::isfinite(eps) && eps >= 0.0, BIM_EINVAL, "eps must be finite and >= 0");
        REQUIRE(imax >= 1, BIM_EINVAL, "imax must be >= 1");
        REQUIRE(std::isfinite(dtau) && dtau > 0.0, BIM_EINVAL, "dtau must be finite and > 0");
        auto t0 = std::chrono::steady_clock::now();
        bim_rep_report r{};
        r.ncut_min = 1 << 30;
        std::map<int, std::vector<int>> by_degree;  // one batch per drop degree
        for (int i = 0; i < c.nd; ++i) by_degree[c.drops[i].p].push_back(i);
        for (const auto &grp : by_degree) {
            const RepOut o = reparam_group(c, grp.second, U_rep, P_cut, eps, imax, dtau);
            r.moves = std::max(r.moves, o.moves);
            r.gnorm = std::max(r.gnorm, o.gnorm);
            r.ncut_min = std::min(r.ncut_min, o.ncut);
        }
        invalidate(c);
        r.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (rep) *rep = r;
        return BIM_OK;
    });
}

int bim_apply_double_layer(bim_ctx h, const double *u_coef, double *out, int mode, int mem_kind)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        require_drops(c);
        REQUIRE(u_coef && out, BIM_EINVAL, "null argument");
        REQUIRE(mode == 0 || mode == 1, BIM_EINVAL, "mode must be 0 or 1");
        c.xsol.ensure((size_t)3 * c.Ctot * sizeof(double));
        copy_in(c, c.xsol.ptr, u_coef, (size_t)3 * c.Ctot * sizeof(double), mem_kind);
        if (mode == 0) {
            std::vector<double> wt((size_t)c.nd * c.nd, 1.0 / (4.0 * kPi));
            double_layer_grid(c, c.xsol.d(), wt);
            copy_out(c, out, c.acc.ptr, (size_t)3 * c.T * sizeof(double), mem_kind);
        } else {
            c.bvec.ensure((size_t)3 * c.Ctot * sizeof(double));
            apply_operator(c, c.xsol.d(), c.bvec.d(), dl_weights(c));
            copy_out(c, out, c.bvec.ptr, (size_t)3 * c.Ctot * sizeof(double), mem_kind);
        }
        return BIM_OK;
    });
}

// The same operator with nothing allocated: the pair partial sums go to the
// static scratch of the context's device, every other buffer must exist
// (t_no_alloc turns an allocation into BIM_ESTATE). Device pointers only.
int bim_apply_double_layer_noalloc(bim_ctx h, const double *u_coef, double *out, int mode)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        require_drops(c);
        REQUIRE(u_coef && out, BIM_EINVAL, "null argument");
        REQUIRE(mode == 0 || mode == 1, BIM_EINVAL, "mode must be 0 or 1");
        double *sp = scratch_on(c.device);
        REQUIRE(sp, BIM_EDEVICE, "the device address of the no-allocation scratch is not available");
        REQUIRE(!c.prof_on, BIM_ESTATE, "kernel timing is on (it creates events): bim_profile(ctx, 0) first");
        REQUIRE(c.regions_ok, BIM_ESTATE,
                "the drops' regions and pair work lists are not built: apply bim_apply_double_layer once first");
        const std::vector<double> wt =
            mode == 0 ? std::vector<double>((size_t)c.nd * c.nd, 1.0 / (4.0 * kPi)) : dl_weights(c);
        const Ctx::WList *L = nullptr;
        for (auto &e : c.wlists)
            if (!e->stale && e->wt == wt) L = e.get();
        REQUIRE(L, BIM_ESTATE, "the pair work list of this mode is not built: apply bim_apply_double_layer once first");
        const double need = std::max((double)L->n * 3 * 64 * c.pair_T, (double)c.near_nwork * 3 * 64);
        REQUIRE(need <= (double)kScratchDoubles, BIM_ENOMEM,
                "the pair partial sums need " + std::to_string((long)(need * 8 / (1 << 20))) +
                    " MiB, above the " + std::to_string((long)(kScratchDoubles * 8 >> 20)) + " MiB scratch");
        struct Guard {  // restores the context and the thread flag, also when a step throws
            Ctx &c;
            Guard(Ctx &cc, double *p) : c(cc)
            {
                t_no_alloc = true;
                c.part_override = p;
            }
            ~Guard()
            {
                t_no_alloc = false;
                c.part_override = nullptr;
            }
        } guard(c, sp);
        c.xsol.ensure((size_t)3 * c.Ctot * sizeof(double));
        copy_in(c, c.xsol.ptr, u_coef, (size_t)3 * c.Ctot * sizeof(double), BIM_MEM_DEVICE);
        if (mode == 0) {
            double_layer_grid(c, c.xsol.d(), wt);
            copy_out(c, out, c.acc.ptr, (size_t)3 * c.T * sizeof(double), BIM_MEM_DEVICE);
        } else {
            c.bvec.ensure((size_t)3 * c.Ctot * sizeof(double));
            apply_operator(c, c.xsol.d(), c.bvec.d(), wt);
            copy_out(c, out, c.bvec.ptr, (size_t)3 * c.Ctot * sizeof(double), BIM_MEM_DEVICE);
        }
        return BIM_OK;
    });
}

// (a correction's tolerance relative to its own right-hand side is floored
// like the joint solve's)
constexpr double kTolFloorCorr = 1e-14;

// Per-system check of a joint solve of independent systems: r = b - A x,
// and for every system whose own relative residual ||r_s|| / ||b_s|| is
// above tol, a GMRES solve of A d = r restricted to that system (zero
// elsewhere) to tol ||b_s|| / ||r_s||, then x += d. hb is the host image of
// b. relres becomes the largest per-system residual of the final check.
static int correct_systems(Ctx &c, const std::vector<double> &wt, const std::vector<double> &hb, double tol,
                           int &iters, double &relres, int &nmv)
{
    const long n = 3 * c.Ctot;
    std::vector<double> hax(n), hr(n);
    c.bcorr.ensure((size_t)n * sizeof(double));
    c.xcorr.ensure((size_t)n * sizeof(double));
    auto residuals = [&](std::map<int, std::pair<double, double>> &rs) {
        apply_operator(c, c.xsol.d(), c.bcorr.d(), wt);
        ++nmv;
        HIPC(hipMemcpyAsync(hax.data(), c.bcorr.ptr, n * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        HIPC(hipStreamSynchronize(c.stream));
        rs.clear();
        for (int i = 0; i < c.nd; ++i) {
            auto &e = rs[c.sys_h[i]];
            for (int comp = 0; comp < 3; ++comp)
                for (long k = 0; k < 2L * ncoef(c.drops[i].p); ++k) {
                    const long idx = comp * c.Ctot + c.drops[i].coff + k;
                    hr[idx] = hb[idx] - hax[idx];
                    e.first += hr[idx] * hr[idx];
                    e.second += hb[idx] * hb[idx];
                }
        }
    };
    std::map<int, std::pair<double, double>> rs;
    residuals(rs);
    int rc = BIM_OK;
    bool corrected = false;
    for (auto &kv : rs) {
        const double rn = std::sqrt(kv.second.first), bn = std::sqrt(kv.second.second);
        if (rn <= tol * bn) continue;
        std::vector<double> rsys(n, 0.0);
        for (int i = 0; i < c.nd; ++i) {
            if (c.sys_h[i] != kv.first) continue;
            for (int comp = 0; comp < 3; ++comp)
                for (long k = 0; k < 2L * ncoef(c.drops[i].p); ++k) {
                    const long idx = comp * c.Ctot + c.drops[i].coff + k;
                    rsys[idx] = hr[idx];
                }
        }
        HIPC(hipMemcpyAsync(c.bcorr.ptr, rsys.data(), n * sizeof(double), hipMemcpyHostToDevice, c.stream));
        int it = 0, mv = 0;
        double rr = 0.0;
        const int r1 = gmres(c, c.bcorr.d(), c.xcorr.d(), wt, std::max(tol * bn / rn, kTolFloorCorr), it, rr, mv);
        iters += it;
        nmv += mv;
        if (r1 != BIM_OK) rc = r1;
        launch_scale_add(c.stream, n, 1.0, c.xcorr.d(), 1.0, c.xsol.d());
        corrected = true;
    }
    if (corrected) residuals(rs);
    relres = 0.0;
    for (auto &kv : rs)
        if (kv.second.second > 0.0) relres = std::max(relres, std::sqrt(kv.second.first / kv.second.second));
    return rc;
}

// Velocity solve at the current drop and surfactant state: geometry, force,
// single layer, right-hand side and GMRES on the second-kind operator; the
// velocity coefficients are left in c.xsol [3][Ctot].
static int solve_velocity(Ctx &c, int &iters, double &relres, int &nmv)
{
    // a velocity evaluation always recomputes the geometry, the force and
    // the regions from the drop coefficients
    invalidate(c);
    build_force(c);
    bool all_one = true;
    for (auto &d : c.drops) all_one = all_one && d.lam == 1.0;
    std::vector<char> with_dl(c.nd, 0);
    if (!all_one) {
        const std::vector<double> wt = dl_weights(c);
        for (int i = 0; i < c.nd; ++i) with_dl[i] = wt[(size_t)i * c.nd + i] != 0.0;
    }
    const std::vector<double> wt_dl = all_one ? std::vector<double>() : dl_weights(c);
    single_layer_grid(c, c.fc.d(), &with_dl, all_one ? nullptr : &wt_dl);
    // b = 2 u_inf - S / (4 pi) on the grid, then Galerkin projection
    c.tmp.ensure((size_t)3 * std::max<long>(c.Ctot, c.T) * sizeof(double));
    launch_rhs(c.stream, (int)c.T, c.tx.d(), c.T, c.acc.d(), -1.0 / (4.0 * kPi), c.U0, c.gU.d(), c.tmp.d());
    c.bvec.ensure((size_t)3 * c.Ctot * sizeof(double));
    project(c, c.tmp.d(), c.bvec.d());
    int rc = BIM_OK;
    iters = 0;
    nmv = 0;
    relres = 0.0;
    const long n = 3 * c.Ctot;
    c.xsol.ensure((size_t)n * sizeof(double));
    if (all_one) {
        launch_scale_add(c.stream, n, 0.5, c.bvec.d(), 0.0, c.xsol.d());
    } else {
        // independent systems in one solve: a tolerance scaled by
        // min_s ||b_s|| / ||b|| bounds every system's own relative
        // residual by gmres_tol (||r_s|| <= ||r||). It is floored at
        // kTolFloor, below which rounding stalls GMRES; when the floor
        // applies, every system's residual is checked afterwards and those
        // above gmres_tol are corrected by their own solves (the operator
        // does not couple systems, so a right-hand side that is zero outside
        // one system keeps every Krylov vector there)
        constexpr double kTolFloor = 1e-14;
        const double tol = c.opt.gmres_tol;
        double bound = 1.0;
        std::map<int, double> bs;
        for (int i = 0; i < c.nd; ++i) bs[c.sys_h[i]] = 0.0;
        std::vector<double> hb;
        if (bs.size() > 1) {
            hb.resize(n);
            HIPC(hipMemcpyAsync(hb.data(), c.bvec.ptr, n * sizeof(double), hipMemcpyDeviceToHost, c.stream));
            HIPC(hipStreamSynchronize(c.stream));
            double tot = 0.0;
            for (int i = 0; i < c.nd; ++i)
                for (int comp = 0; comp < 3; ++comp)
                    for (long e = 0; e < 2L * ncoef(c.drops[i].p); ++e) {
                        const double v = hb[comp * c.Ctot + c.drops[i].coff + e];
                        bs[c.sys_h[i]] += v * v;
                        tot += v * v;
                    }
            double bmin = 0.0;
            for (auto &kv : bs)
                if (kv.second > 0.0 && (bmin == 0.0 || kv.second < bmin)) bmin = kv.second;
            if (bmin > 0.0 && tot > 0.0) bound = std::sqrt(tot / bmin);
        }
        const std::vector<double> wt = dl_weights(c);
        const bool floored = tol / bound < kTolFloor;
        rc = gmres(c, c.bvec.d(), c.xsol.d(), wt, floored ? kTolFloor : tol / bound, iters, relres, nmv);
        relres *= bound;
        if (floored && rc == BIM_OK) rc = correct_systems(c, wt, hb, tol, iters, relres, nmv);
    }
    return rc;
}

int bim_eval_velocity(bim_ctx h, double *u_out, int out_kind, bim_report *rep)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        require_drops(c);
        REQUIRE(u_out, BIM_EINVAL, "null output");
        REQUIRE(out_kind >= 0 && out_kind <= 3, BIM_EINVAL, "bad out_kind");
        auto t0 = std::chrono::steady_clock::now();
        int iters = 0, nmv = 0;
        double relres = 0.0;
        const int rc = solve_velocity(c, iters, relres, nmv);
        const long n = 3 * c.Ctot;
        const bool dev = (out_kind & 2) != 0;
        if (out_kind & 1) {
            copy_out(c, u_out, c.xsol.ptr, (size_t)n * sizeof(double), dev ? BIM_MEM_DEVICE : BIM_MEM_HOST);
        } else {
            synth_grid_all(c, c.xsol.d(), c.tmp.d());
            copy_out(c, u_out, c.tmp.ptr, (size_t)3 * c.T * sizeof(double), dev ? BIM_MEM_DEVICE : BIM_MEM_HOST);
        }
        if (rep) {
            if (dev) HIPC(hipStreamSynchronize(c.stream));
            rep->gmres_iterations = iters;
            rep->gmres_residual = relres;
            rep->n_targets = (int)c.T;
            rep->n_omega1 = c.n_om1;
            rep->n_omega2 = c.n_om2;
            rep->n_fmm_pairs = (int)c.fmm.pairs.size();
            rep->fmm_order = c.fmm.P;
            rep->pair_targets_per_lane = c.pair_T;
            rep->pair_sources_per_item = c.pair_ch;
            rep->xform_matrix_cores = (c.xmode[0][c.opt.precision == BIM_PREC_MIXED] == 1 ? 1 : 0) |
                                      (c.xmode[1][c.opt.precision == BIM_PREC_MIXED] == 1 ? 2 : 0);
            rep->n_matvec = nmv;
            rep->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        if (rc == BIM_ENOCONV) c.err = "GMRES stopped at maxit above tolerance";
        return rc;
    });
}

int bim_sh_synthesize(bim_ctx h, int p, int q, int nf, const double *coef, int dt, int dp, double *grid_out,
                      int mem_kind)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        REQUIRE(p >= 0 && q >= p && q >= 1 && q <= 512 && nf >= 1 && coef && grid_out, BIM_EINVAL, "bad arguments");
        REQUIRE(dt >= 0 && dp >= 0 && dt + dp <= 2, BIM_EINVAL, "derivative order > 2");
        const size_t cb = (size_t)nf * 2 * ncoef(p) * sizeof(double), gb = (size_t)nf * npts(q) * sizeof(double);
        DBuf ci, go;
        const double *cin = coef;
        double *gout = grid_out;
        if (mem_kind != BIM_MEM_DEVICE) {
            ci.ensure(cb);
            go.ensure(gb);
            HIPC(hipMemcpyAsync(ci.ptr, coef, cb, hipMemcpyHostToDevice, c.stream));
            cin = ci.d();
            gout = go.d();
        }
        if (dt == 0 && dp == 0 && xform_fits(p, q, false)) {
            Ctx::XPlan &pl = xfield_plan(c, p, q, nf);
            std::vector<XJob> jobs;
            size_t goff = 0;
            const bool f32 = c.opt.precision == BIM_PREC_MIXED;
            jobs.push_back(xjob(c, pl, q, pl.gb0, gout, false, false, f32, goff));
            xsynth_run(c, jobs, goff, cin, f32);
        } else {
            synth(c, p, q, nf, cin, 2L * ncoef(p), dt, dp, gout, npts(q));
        }
        if (mem_kind != BIM_MEM_DEVICE) {
            HIPC(hipMemcpyAsync(grid_out, gout, gb, hipMemcpyDeviceToHost, c.stream));
            HIPC(hipStreamSynchronize(c.stream));
        }
        return BIM_OK;
    });
}

int bim_sh_analyze(bim_ctx h, int q, int p, int nf, const double *grid_in, double *coef, int mem_kind)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        REQUIRE(p >= 0 && q >= p && q >= 1 && q <= 512 && nf >= 1 && coef && grid_in, BIM_EINVAL, "bad arguments");
        const size_t cb = (size_t)nf * 2 * ncoef(p) * sizeof(double), gb = (size_t)nf * npts(q) * sizeof(double);
        DBuf gi, co;
        const double *gin = grid_in;
        double *cout = coef;
        if (mem_kind != BIM_MEM_DEVICE) {
            gi.ensure(gb);
            co.ensure(cb);
            HIPC(hipMemcpyAsync(gi.ptr, grid_in, gb, hipMemcpyHostToDevice, c.stream));
            gin = gi.d();
            cout = co.d();
        }
        if (xform_fits(p, q, true)) {
            Ctx::XPlan &pl = xfield_plan(c, p, q, nf);
            std::vector<XJob> jobs;
            size_t goff = 0;
            const bool f32 = c.opt.precision == BIM_PREC_MIXED;
            jobs.push_back(xjob(c, pl, q, pl.gb0, const_cast<double *>(gin), true, false, f32, goff));
            xanal_run(c, jobs, goff, nullptr, cout, 1.0, f32);
        } else {
            analyze(c, q, p, nf, gin, npts(q), cout, 2L * ncoef(p));
        }
        if (mem_kind != BIM_MEM_DEVICE) {
            HIPC(hipMemcpyAsync(coef, cout, cb, hipMemcpyDeviceToHost, c.stream));
            HIPC(hipStreamSynchronize(c.stream));
        }
        return BIM_OK;
    });
}

int bim_profile(bim_ctx h, int enable)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        prof_drain(c);
        if (enable) c.prof.clear();
        c.prof_on = enable != 0;
        return BIM_OK;
    });
}

int bim_profile_select(bim_ctx h, const char *names)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        c.prof_sel.clear();
        if (names) {
            std::string s(names), cur;
            for (char ch : s + ",") {
                if (ch == ',') {
                    if (!cur.empty()) c.prof_sel.insert(cur);
                    cur.clear();
                } else if (ch != ' ') {
                    cur += ch;
                }
            }
        }
        return BIM_OK;
    });
}

int bim_profile_query(bim_ctx h, const char *name, int *launches, double *ms, double *flops, double *bytes)
{
    return guarded(h ? &h->c : nullptr, [&]() {
        Ctx &c = h->c;
        REQUIRE(name, BIM_EINVAL, "null kernel name");
        prof_drain(c);
        auto it = c.prof.find(name);
        const bool f = it != c.prof.end();
        if (launches) *launches = f ? it->second.launches : 0;
        if (ms) *ms = f ? it->second.ms : 0.0;
        if (flops) *flops = f ? it->second.flops : 0.0;
        if (bytes) *bytes = f ? it->second.bytes : 0.0;
        return BIM_OK;
    });
}

// ---- host-side tables (no device needed) ----
int bim_host_gauss_legendre(int q, double *t, double *w)
{
    if (q < 1 || q > 1024 || !t || !w) return BIM_EINVAL;
    std::vector<double> tv, wv;
    gauss_legendre(q, tv, wv);
    std::copy(tv.begin(), tv.end(), t);
    std::copy(wv.begin(), wv.end(), w);
    return BIM_OK;
}

int bim_host_legendre(int nmax, double t, double *P, double *D1, double *D2)
{
    if (nmax < 0 || nmax > 1024 || !P || !(t > -1.0 && t < 1.0)) return BIM_EINVAL;
    legendre_table(nmax, t, P, D1, D2);
    return BIM_OK;
}

int bim_host_wigner_d(int n, double beta, double *d)
{
    if (n < 0 || n > 256 || !d) return BIM_EINVAL;
    std::vector<double> all;
    wigner_table(n, beta, all);
    const size_t off = (size_t)n * (4 * (size_t)n * n - 1) / 3;
    std::copy(all.begin() + off, all.end(), d);
    return BIM_OK;
}

}  // extern "C"
