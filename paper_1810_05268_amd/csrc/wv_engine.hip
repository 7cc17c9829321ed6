// Serving engine: continuous batching of shot-gradient requests on one GPU.
//
// Shots are independent (the paper's gradients are computed per shot and summed,
// Sec. "Example adjoint problem: Seismic inversion"), so the engine runs several of
// them at once.  Each admitted request gets a slice of a caller-provided device pool
// (its workspace, including its checkpoint arena) and one of max_active worker
// threads, each with its own HIP stream, so the kernels of different shots overlap on
// the device.
//
// Admission is first fit in arrival order: a free worker takes the oldest queued
// request whose workspace fits a contiguous free slice of the pool, so a large request
// that must wait for memory does not hold back smaller ones behind it.  To keep it from
// waiting for ever, once it has been passed over kMaxSkips times nothing behind it is
// admitted until it is.
//
// With batching on (wv_engine_set_batching), 2-D requests go to a batch lane instead:
// one more worker takes every queued 2-D request that shares the oldest one's grid,
// order, steps, time step, receiver count, tolerance and budget (up to max_batch of
// them) and runs them as one batched call (wv_batch_misfit_gradient: one persistent
// kernel advances all of them), while the 3-D requests keep their own workers.  Requests
// that arrive while a batch runs join the next one.
//
// Every request is computed exactly as it would be alone (same kernels and reduction
// orders; a batched shot's arithmetic is the solo call's), so its result does not
// depend on what else is in flight.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "wv_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kMaxSkips = 8;

struct Request {
    int id = 0;
    wv_model model{};
    wv_geom geom{};
    std::vector<double> src, rec;
    const float *d_obs = nullptr;
    size_t mem_budget = 0;
    double tol = 0.0, ratio_hint = 0.0;
    double *grad = nullptr;
    float *d_sim = nullptr;
    size_t ws_bytes = 0, ws_off = 0;
    bool batchable = false;   // a 2-D OT2 request
    int skipped = 0;          // times a later request was admitted before it
    bool done = false;
    wv_result res{};
    Clock::time_point t_submit, t_start, t_end;
};

// requests that can share one batched call
bool same_batch(const Request &a, const Request &b)
{
    const wv_model &x = a.model, &y = b.model;
    return x.n[0] == y.n[0] && x.n[1] == y.n[1] && x.h[0] == y.h[0] && x.h[1] == y.h[1] && x.nbl == y.nbl &&
           x.space_order == y.space_order && x.nt == y.nt && x.dt == y.dt && x.vmax == y.vmax &&
           a.geom.nrec == b.geom.nrec && a.tol == b.tol && a.mem_budget == b.mem_budget &&
           a.ratio_hint == b.ratio_hint;
}

// first-fit allocator over [0, size) with coalescing, 256-byte granularity
struct Pool {
    std::map<size_t, size_t> free_;   // offset -> length
    explicit Pool(size_t size) { free_[0] = size; }
    bool take(size_t len, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= len) {
                *off = it->first;
                const size_t rest = it->second - len;
                const size_t roff = it->first + len;
                free_.erase(it);
                if (rest) free_[roff] = rest;
                return true;
            }
        }
        return false;
    }
    void give(size_t off, size_t len)
    {
        auto it = free_.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

}  // namespace

struct wv_engine {
    uint8_t *pool_base = nullptr;
    size_t pool_bytes = 0;
    int device = 0;
    Pool pool{0};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::map<int, Request *> reqs;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    int next_id = 0;
    int active = 0;
    int max_batch = 0;        // > 1: 2-D requests run in batches of up to this many
    bool batch_started = false;
    std::thread batch_worker;
    hipStream_t batch_stream = nullptr;
    bool stop = false;
    Clock::time_point t0;

    double ms(Clock::time_point t) const { return std::chrono::duration<double, std::milli>(t - t0).count(); }

    // Under mu: the request a solo worker admits now (taking its pool slice), or null.
    Request *admit_solo()
    {
        for (auto it = queue.begin(); it != queue.end(); ++it) {
            Request *r = *it;
            if (max_batch > 1 && r->batchable) continue;   // the batch lane's
            size_t off;
            if (pool.take(r->ws_bytes, &off)) {
                r->ws_off = off;
                // every solo request before it that did not fit is passed over once more
                for (auto jt = queue.begin(); jt != it; ++jt)
                    if (!(max_batch > 1 && (*jt)->batchable)) (*jt)->skipped++;
                queue.erase(it);
                return r;
            }
            if (r->skipped >= kMaxSkips) return nullptr;   // it is next: nothing passes it
        }
        return nullptr;
    }

    void finish(Request *r, int rc, double phi, const wv_stats &st, Clock::time_point t_end)
    {
        r->t_end = t_end;
        r->res.status = rc;
        r->res.misfit = phi;
        r->res.stats = st;
        r->res.t_submit_ms = ms(r->t_submit);
        r->res.t_start_ms = ms(r->t_start);
        r->res.t_end_ms = ms(r->t_end);
        r->done = true;
    }

    void run(int w)
    {
        (void)hipSetDevice(device);
        for (;;) {
            Request *r = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    if (stop && queue.empty()) return true;
                    return (r = admit_solo()) != nullptr || (stop && !has_solo());
                });
                if (!r) return;   // stopping
                ++active;
                r->t_start = Clock::now();
            }
            // the next request may fit as well
            cv_work.notify_all();
            r->geom.src_xyz = r->src.data();
            r->geom.rec_xyz = r->rec.data();
            wv_stats st{};
            double phi = 0.0;
            const int rc = wv_misfit_gradient(&r->model, &r->geom, r->d_obs, r->mem_budget, r->tol, r->ratio_hint,
                                              &phi, r->grad, r->d_sim, &st, pool_base + r->ws_off, r->ws_bytes,
                                              streams[w]);
            {
                std::lock_guard<std::mutex> lk(mu);
                finish(r, rc, phi, st, Clock::now());
                pool.give(r->ws_off, r->ws_bytes);
                --active;
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }

    bool has_solo() const
    {
        for (const Request *r : queue)
            if (!(max_batch > 1 && r->batchable)) return true;
        return false;
    }
    bool has_batchable() const
    {
        for (const Request *r : queue)
            if (r->batchable) return true;
        return false;
    }

    // The batch lane: the oldest queued 2-D request and every later one that can share
    // its call, as many as fit max_batch and the pool.
    void run_batch()
    {
        (void)hipSetDevice(device);
        for (;;) {
            std::vector<Request *> batch;
            size_t off = 0, bytes = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    if (stop && !has_batchable()) return true;
                    Request *head = nullptr;
                    for (Request *r : queue)
                        if (r->batchable) {
                            head = r;
                            break;
                        }
                    if (!head) return false;
                    std::vector<Request *> cand;
                    for (Request *r : queue)
                        if (r->batchable && same_batch(*head, *r) && (int)cand.size() < max_batch) cand.push_back(r);
                    // the largest prefix of the candidates whose batch workspace fits the pool
                    while (!cand.empty()) {
                        std::vector<wv_model> ms;
                        std::vector<wv_geom> gs;
                        for (Request *r : cand) {
                            ms.push_back(r->model);
                            gs.push_back(r->geom);
                            gs.back().src_xyz = r->src.data();
                            gs.back().rec_xyz = r->rec.data();
                        }
                        const size_t need = wv_batch_workspace_bytes((int)cand.size(), ms.data(), gs.data(),
                                                                     head->mem_budget);
                        const size_t need_al = (need + 255) / 256 * 256;
                        if (need == 0) {
                            // not a valid batch (cannot happen for requests that passed submit):
                            // fail the head alone
                            cand.resize(1);
                            bytes = 0;
                            break;
                        }
                        if (pool.take(need_al, &off)) {
                            bytes = need_al;
                            break;
                        }
                        cand.pop_back();
                    }
                    if (cand.empty()) return false;
                    batch = cand;
                    return true;
                });
                if (batch.empty()) return;   // stopping
                const Clock::time_point t0 = Clock::now();   // one start time per batch
                for (Request *r : batch) {
                    queue.erase(std::find(queue.begin(), queue.end(), r));
                    r->t_start = t0;
                }
                active += (int)batch.size();
            }
            const int n = (int)batch.size();
            std::vector<wv_model> ms((size_t)n);
            std::vector<wv_geom> gs((size_t)n);
            std::vector<const float *> dobs((size_t)n);
            std::vector<double *> grads((size_t)n);
            std::vector<float *> dsims((size_t)n);
            std::vector<double> phis((size_t)n, 0.0);
            std::vector<wv_stats> sts((size_t)n);
            for (int i = 0; i < n; ++i) {
                Request *r = batch[i];
                r->geom.src_xyz = r->src.data();
                r->geom.rec_xyz = r->rec.data();
                ms[i] = r->model;
                gs[i] = r->geom;
                dobs[i] = r->d_obs;
                grads[i] = r->grad;
                dsims[i] = r->d_sim;
            }
            // a batch of one runs the solo path (the same bits; the persistent launch pays a
            // device-wide barrier per phase that only several shots amortise)
            int rc = WV_EINVAL;
            if (bytes && n == 1)
                rc = wv_misfit_gradient(&ms[0], &gs[0], dobs[0], batch[0]->mem_budget, batch[0]->tol,
                                        batch[0]->ratio_hint, &phis[0], grads[0], dsims[0], &sts[0], pool_base + off,
                                        bytes, batch_stream);
            else if (bytes)
                rc = wv_batch_misfit_gradient(n, ms.data(), gs.data(), dobs.data(), batch[0]->mem_budget,
                                              batch[0]->tol, batch[0]->ratio_hint, phis.data(), grads.data(),
                                              dsims.data(), sts.data(), pool_base + off, bytes, batch_stream);
            {
                std::lock_guard<std::mutex> lk(mu);
                const Clock::time_point t_end = Clock::now();
                for (int i = 0; i < n; ++i) finish(batch[i], rc, phis[i], sts[i], t_end);
                if (bytes) pool.give(off, bytes);
                active -= n;
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }
};

extern "C" {

int wv_engine_create(void *pool, size_t pool_bytes, int max_active, wv_engine **out)
{
    if (!out || !pool || pool_bytes == 0 || max_active < 1 || max_active > 64 || (((uintptr_t)pool) & 255))
        return WV_EINVAL;
    wv_engine *e = new wv_engine();
    e->pool_base = (uint8_t *)pool;
    e->pool_bytes = pool_bytes / 256 * 256;
    e->pool = Pool(e->pool_bytes);
    e->t0 = Clock::now();
    if (hipGetDevice(&e->device) != hipSuccess) {
        delete e;
        return WV_EHIP;
    }
    for (int w = 0; w < max_active; ++w) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t t : e->streams) (void)hipStreamDestroy(t);
            delete e;
            return WV_EHIP;
        }
        e->streams.push_back(s);
    }
    for (int w = 0; w < max_active; ++w) e->workers.emplace_back([e, w] { e->run(w); });
    *out = e;
    return WV_OK;
}

int wv_engine_set_batching(wv_engine *e, int max_batch)
{
    if (!e || max_batch < 0 || max_batch > 256) return WV_EINVAL;
    std::lock_guard<std::mutex> lk(e->mu);
    if (e->batch_started || !e->queue.empty() || e->active) return WV_EINVAL;   // before the first request only
    e->max_batch = max_batch;
    if (max_batch > 1) {
        if (hipStreamCreateWithFlags(&e->batch_stream, hipStreamNonBlocking) != hipSuccess) return WV_EHIP;
        e->batch_started = true;
        e->batch_worker = std::thread([e] { e->run_batch(); });
    }
    return WV_OK;
}

int wv_engine_submit(wv_engine *e, const wv_model *model, const wv_geom *geom, const float *d_obs,
                     size_t mem_budget, double tol, double ratio_hint, double *grad_m, float *d_sim)
{
    if (!e || !model || !geom || !d_obs || !grad_m || !geom->src_xyz || !geom->rec_xyz) return WV_EINVAL;
    const size_t ws = wv_workspace_bytes(model, geom, WV_OP_GRADIENT, mem_budget);
    if (ws == 0) return WV_EINVAL;
    const size_t need = (ws + 255) / 256 * 256;
    Request *r = new Request();
    r->model = *model;
    r->geom = *geom;
    r->src.assign(geom->src_xyz, geom->src_xyz + (size_t)geom->nsrc * model->ndim);
    r->rec.assign(geom->rec_xyz, geom->rec_xyz + (size_t)geom->nrec * model->ndim);
    r->geom.src_xyz = r->src.data();
    r->geom.rec_xyz = r->rec.data();
    r->d_obs = d_obs;
    r->mem_budget = mem_budget;
    r->tol = tol;
    r->ratio_hint = ratio_hint;
    r->grad = grad_m;
    r->d_sim = d_sim;
    r->ws_bytes = need;
    r->batchable = model->ndim == 2 && (model->time_order == 0 || model->time_order == 2);
    if (r->batchable && e->max_batch > 1) {
        // a batch of one must fit the pool
        const size_t nb = wv_batch_workspace_bytes(1, &r->model, &r->geom, mem_budget);
        if (nb == 0) {
            delete r;
            return WV_EINVAL;
        }
        if ((nb + 255) / 256 * 256 > e->pool_bytes) {
            delete r;
            return WV_EBUDGET;
        }
    } else if (need > e->pool_bytes) {
        delete r;
        return WV_EBUDGET;   // could never be admitted
    }
    {
        std::lock_guard<std::mutex> lk(e->mu);
        if (e->stop) {
            delete r;
            return WV_EINVAL;
        }
        r->id = e->next_id++;
        r->t_submit = Clock::now();
        e->reqs[r->id] = r;
        e->queue.push_back(r);
    }
    e->cv_work.notify_all();
    return r->id;
}

int wv_engine_wait(wv_engine *e, int id, double timeout_ms, wv_result *res)
{
    if (!e || !res) return WV_EINVAL;
    std::unique_lock<std::mutex> lk(e->mu);
    auto it = e->reqs.find(id);
    if (it == e->reqs.end()) return WV_EINVAL;
    Request *r = it->second;
    auto ready = [&] { return r->done; };
    if (timeout_ms < 0) e->cv_done.wait(lk, ready);
    else if (!e->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready))
        return WV_ETIMEOUT;
    *res = r->res;
    e->reqs.erase(it);
    delete r;
    return WV_OK;
}

int wv_engine_pending(wv_engine *e, int *queued, int *active)
{
    if (!e) return WV_EINVAL;
    std::lock_guard<std::mutex> lk(e->mu);
    if (queued) *queued = (int)e->queue.size();
    if (active) *active = e->active;
    return WV_OK;
}

int wv_engine_destroy(wv_engine *e)
{
    if (!e) return WV_EINVAL;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        e->stop = true;
    }
    e->cv_work.notify_all();
    for (std::thread &t : e->workers) t.join();
    if (e->batch_worker.joinable()) e->batch_worker.join();
    for (hipStream_t s : e->streams) (void)hipStreamDestroy(s);
    if (e->batch_stream) (void)hipStreamDestroy(e->batch_stream);
    for (auto &kv : e->reqs) delete kv.second;
    delete e;
    return WV_OK;
}

}  // extern "C"
