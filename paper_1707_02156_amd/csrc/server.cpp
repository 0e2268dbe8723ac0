// Request server over the velocity evaluation: continuous admission of
// independent drop systems into a fixed set of slots, each slot a context
// with its own HIP stream and a host worker thread, so that the device work
// of requests admitted at different times overlaps. A free slot takes the
// head of the queue (first come, first served) when its estimated device
// memory fits in the budget next to the running requests, together with
// further queued requests of the same tension up to the batch limits: a
// batch runs as independent systems of one context (one launch sequence for
// all of them). The per-degree tables of a context stay resident.
#include "../../include/bim.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

inline long ncoef_s(int p) { return (long)(p + 1) * (p + 2) / 2; }
inline long npts_s(int q) { return 2L * q * (q + 1); }

struct Request {
    uint64_t id = 0;
    int nd = 0;
    std::vector<int> p;
    std::vector<double> xc, lam, gamma;
    int eos = 0;
    double E = 0.0, xs = 0.0, sigma0 = 1.0;
    int out_kind = 0;
    std::vector<double> out;
    bim_report rep{};
    int status = BIM_OK;
    std::string err;
    double footprint = 0.0;
    Clock::time_point t_submit, t_start, t_end;
    bool done = false;
};

}  // namespace

struct bim_server_s {
    bim_server_options opt{};
    std::vector<bim_ctx> ctx;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    double inflight = 0.0;  // estimated bytes of running requests
    uint64_t next_id = 1;
    bool stop = false;
};

namespace {

bool admissible(const bim_server_s &s)
{
    if (s.queue.empty()) return false;
    const double budget = s.opt.hbm_budget_gb * 1e9;
    return s.inflight == 0.0 || s.inflight + s.queue.front()->footprint <= budget;
}

void run_request(bim_ctx ctx, Request &r)
{
    int st = bim_set_drops(ctx, r.nd, r.p.data(), r.xc.data(), r.lam.data(), BIM_MEM_HOST);
    if (st == BIM_OK)
        st = bim_set_tension(ctx, r.gamma.empty() ? nullptr : r.gamma.data(), r.eos, r.E, r.xs, r.sigma0,
                             BIM_MEM_HOST);
    if (st == BIM_OK) st = bim_eval_velocity(ctx, r.out.data(), r.out_kind & 1, &r.rep);
    r.status = st;
    if (st != BIM_OK) r.err = bim_last_error(ctx);
}

bool same_tension(const Request &a, const Request &b)
{
    return a.eos == b.eos && a.E == b.E && a.xs == b.xs && a.sigma0 == b.sigma0 && a.out_kind == b.out_kind &&
           a.gamma.empty() == b.gamma.empty();
}

// Several requests as independent systems of one context: one evaluation,
// outputs split back per request.
void run_batch(bim_ctx ctx, std::vector<Request *> &batch)
{
    if (batch.size() == 1) {
        run_request(ctx, *batch[0]);
        return;
    }
    std::vector<int> p, sys;
    std::vector<double> lam, gamma;
    std::vector<long> coff, toff;  // per request: offsets inside one component block
    long ctot = 0, T = 0;
    for (size_t q = 0; q < batch.size(); ++q) {
        const Request &r = *batch[q];
        coff.push_back(ctot);
        toff.push_back(T);
        for (int d = 0; d < r.nd; ++d) {
            p.push_back(r.p[d]);
            sys.push_back((int)q);
            lam.push_back(r.lam[d]);
            ctot += 2 * ncoef_s(r.p[d]);
            T += npts_s(r.p[d]);
        }
        gamma.insert(gamma.end(), r.gamma.begin(), r.gamma.end());
    }
    std::vector<double> xc((size_t)3 * ctot);
    for (size_t q = 0; q < batch.size(); ++q) {
        const Request &r = *batch[q];
        const long n = (long)r.xc.size() / 3;
        for (int c = 0; c < 3; ++c) std::memcpy(&xc[c * ctot + coff[q]], &r.xc[c * n], n * sizeof(double));
    }
    const Request &r0 = *batch[0];
    const bool coef = (r0.out_kind & 1) != 0;
    const long per = coef ? ctot : T;
    std::vector<double> out((size_t)3 * per);
    bim_report rep{};
    int st = bim_set_drops(ctx, (int)p.size(), p.data(), xc.data(), lam.data(), BIM_MEM_HOST);
    if (st == BIM_OK) st = bim_set_systems(ctx, sys.data());
    if (st == BIM_OK)
        st = bim_set_tension(ctx, gamma.empty() ? nullptr : gamma.data(), r0.eos, r0.E, r0.xs, r0.sigma0,
                             BIM_MEM_HOST);
    if (st == BIM_OK) st = bim_eval_velocity(ctx, out.data(), coef ? 1 : 0, &rep);
    const std::string err = st != BIM_OK ? bim_last_error(ctx) : std::string();
    for (size_t q = 0; q < batch.size(); ++q) {
        Request &r = *batch[q];
        const long n = (long)r.out.size() / 3, o = coef ? coff[q] : toff[q];
        for (int c = 0; c < 3; ++c) std::memcpy(&r.out[c * n], &out[c * per + o], n * sizeof(double));
        r.rep = rep;
        long tq = 0;
        for (int d = 0; d < r.nd; ++d) tq += npts_s(r.p[d]);
        r.rep.n_targets = (int)tq;
        r.status = st;
        r.err = err;
    }
}

void worker(bim_server_s *s, int k)
{
    for (;;) {
        std::vector<Request *> batch;
        double fp = 0.0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || admissible(*s); });
            if (s->stop) return;
            // the head, then further queued requests of the same tension while
            // they fit the batch limits and the memory budget
            const double budget = s->opt.hbm_budget_gb * 1e9;
            int drops = 0;
            while (!s->queue.empty() && (int)batch.size() < std::max(1, s->opt.max_batch)) {
                Request *r = s->queue.front();
                if (!batch.empty() && (!same_tension(*r, *batch[0]) || drops + r->nd > s->opt.max_batch_drops ||
                                       s->inflight + fp + r->footprint > budget))
                    break;
                s->queue.pop_front();
                batch.push_back(r);
                fp += r->footprint;
                drops += r->nd;
                r->t_start = Clock::now();
            }
            s->inflight += fp;
        }
        s->cv_work.notify_all();  // the next request may fit too
        run_batch(s->ctx[k], batch);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->inflight -= fp;
            if (s->inflight < 0.5) s->inflight = 0.0;
            const auto t = Clock::now();
            for (Request *r : batch) {
                r->t_end = t;
                r->done = true;
            }
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

}  // namespace

extern "C" {

int bim_server_footprint(const bim_options *opt, int n_drops, const int *p, double *bytes)
{
    if (!opt || !p || !bytes || n_drops < 1) return BIM_EINVAL;
    double b = 0.0;
    long ctot = 0, T = 0;
    int pmax = 0;
    for (int d = 0; d < n_drops; ++d) {
        if (p[d] < 2 || p[d] > 64) return BIM_EINVAL;
        const long nc = ncoef_s(p[d]);
        ctot += 2 * nc;
        T += npts_s(p[d]);
        pmax = p[d] > pmax ? p[d] : pmax;
        b += (double)npts_s(p[d]) * 6 * 2 * nc * 8;                           // stored double-layer rows
        b += (double)npts_s(opt->U_tilde * p[d]) * 10 * 8;                    // upsampled nodes
        b += (double)npts_s(opt->U_geom * p[d]) * 21 * 8;                     // force grid fields
    }
    b += (double)T * 3 * 8 * 12;                                              // grids, accumulators
    b += (double)(opt->gmres_restart + 4) * 3 * ctot * 8;                     // Krylov basis
    // singular pipeline intermediates for the largest degree (capped chunk)
    const double P1 = pmax + 1, Q1 = opt->U_sing * pmax + 1, nc = ncoef_s(pmax), nk = 2.0 * pmax;
    const double per_lat = nk * 8.0 * (nc * 12 + P1 * 3 * Q1 * 6 + P1 * Q1 * 12 + nc * 12 + Q1 * 3 + 3);
    const double pipe = per_lat * P1 * n_drops;
    const double cap = opt->pipe_budget_gb * 1024.0 * 1024 * 1024;
    b += pipe < cap ? pipe : cap;
    *bytes = b;
    return BIM_OK;
}

int bim_server_default_options(bim_server_options *o)
{
    if (!o) return BIM_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->slots = 3;
    o->hbm_budget_gb = 64.0;
    o->max_batch = 1;
    o->max_batch_drops = 128;
    const int rc = bim_default_options(&o->opt);
    // requests are mostly one-off problem shapes: timing the pair work shape
    // or the transform path of each would cost more than it saves and add to
    // the latency tail; the transforms of small systems are latency-bound,
    // where the scalar kernels are the faster; and concurrent slots keep
    // small singular-pipeline chunks (with 8 GB chunks an overloaded stream
    // served half as many requests per second)
    o->opt.pair_tune = 0;
    o->opt.xform_path = 1;
    o->opt.pipe_budget_gb = 0.75;
    return rc;
}

int bim_server_create(const bim_server_options *opt, bim_server *out)
{
    if (!opt || !out) return BIM_EINVAL;
    *out = nullptr;
    if (opt->slots < 1 || opt->slots > 64 || !(opt->hbm_budget_gb > 0.0) || opt->opt.stream || opt->max_batch < 1 ||
        opt->max_batch_drops < 1 || opt->max_queue < 0)
        return BIM_EINVAL;
    std::unique_ptr<bim_server_s> s;
    try {
        s = std::make_unique<bim_server_s>();
    } catch (...) {
        return BIM_ENOMEM;
    }
    s->opt = *opt;
    for (int k = 0; k < opt->slots; ++k) {
        bim_ctx c = nullptr;
        const int st = bim_create(&opt->opt, &c);
        if (st != BIM_OK) {
            for (bim_ctx x : s->ctx) bim_destroy(x);
            return st;
        }
        s->ctx.push_back(c);
    }
    try {
        for (int k = 0; k < opt->slots; ++k) s->workers.emplace_back(worker, s.get(), k);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        for (auto &t : s->workers) t.join();
        for (bim_ctx x : s->ctx) bim_destroy(x);
        return BIM_ENOMEM;
    }
    *out = s.release();
    return BIM_OK;
}

int bim_server_destroy(bim_server s)
{
    if (!s) return BIM_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    for (bim_ctx c : s->ctx) bim_destroy(c);
    delete s;
    return BIM_OK;
}

int bim_server_submit(bim_server s, int n_drops, const int *p, const double *xcoef, const double *lambda,
                      const double *gamma_coef, int eos, double E, double xs, double sigma0, int out_kind,
                      uint64_t *id)
{
    if (!s || !p || !xcoef || !lambda || !id || n_drops < 1 || out_kind < 0 || out_kind > 1) return BIM_EINVAL;
    auto r = std::make_unique<Request>();
    r->nd = n_drops;
    r->p.assign(p, p + n_drops);
    long ctot = 0, T = 0;
    for (int d = 0; d < n_drops; ++d) {
        if (p[d] < 2 || p[d] > 64) return BIM_EINVAL;
        ctot += 2 * ncoef_s(p[d]);
        T += npts_s(p[d]);
    }
    r->xc.assign(xcoef, xcoef + 3 * ctot);
    r->lam.assign(lambda, lambda + n_drops);
    if (gamma_coef) r->gamma.assign(gamma_coef, gamma_coef + ctot);
    r->eos = eos;
    r->E = E;
    r->xs = xs;
    r->sigma0 = sigma0;
    r->out_kind = out_kind;
    r->out.assign(out_kind & 1 ? 3 * ctot : 3 * T, 0.0);
    if (bim_server_footprint(&s->opt.opt, n_drops, p, &r->footprint) != BIM_OK) return BIM_EINVAL;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->opt.max_queue > 0 && (long)s->queue.size() >= s->opt.max_queue) return BIM_EBUSY;
        r->id = s->next_id++;
        *id = r->id;
        s->queue.push_back(r.get());
        s->reqs[r->id] = std::move(r);
    }
    s->cv_work.notify_all();
    return BIM_OK;
}

int bim_server_wait(bim_server s, uint64_t id, double timeout_s, double *out, bim_report *rep, double *times_ms)
{
    if (!s) return BIM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return BIM_EINVAL;
    Request *r = it->second.get();
    auto ready = [&] { return r->done; };
    if (timeout_s < 0.0) {
        s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
        return BIM_EAGAIN;
    }
    if (out) std::memcpy(out, r->out.data(), r->out.size() * sizeof(double));
    if (rep) *rep = r->rep;
    if (times_ms) {
        using ms = std::chrono::duration<double, std::milli>;
        times_ms[0] = ms(r->t_start - r->t_submit).count();
        times_ms[1] = ms(r->t_end - r->t_start).count();
        times_ms[2] = ms(r->t_end - r->t_submit).count();
    }
    const int st = r->status;
    s->reqs.erase(it);
    return st;
}

}  // extern "C"
