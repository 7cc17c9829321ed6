// Serving engine: continuous batching of shot-gradient requests on one GPU.
//
// Shots are independent (the paper's gradients are computed per shot and summed,
// Sec. "Example adjoint problem: Seismic inversion"), so the engine runs several of
// them at once: each admitted request gets a slice of a caller-provided device
// pool (its workspace, including its checkpoint arena) and one of max_active
// worker threads, each with its own HIP stream, so the kernels of different shots
// overlap on the device.  Admission is first come, first served: the head of the
// queue starts as soon as a worker is free and a contiguous slice of the pool that
// holds its workspace is free; a finished request returns its slice and the next
// one is admitted at once.  Every request is computed exactly as it would be alone
// (same kernels, same launch shapes, no shared accumulators), so its result does
// not depend on what else is in flight.
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
    bool done = false;
    wv_result res{};
    Clock::time_point t_submit, t_start, t_end;
};

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
    bool stop = false;
    Clock::time_point t0;

    void run(int w)
    {
        (void)hipSetDevice(device);
        for (;;) {
            Request *r = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    if (stop && queue.empty()) return true;
                    if (queue.empty()) return false;
                    size_t off;
                    if (!pool.take(queue.front()->ws_bytes, &off)) return false;
                    queue.front()->ws_off = off;
                    return true;
                });
                if (queue.empty()) return;   // stopping
                r = queue.front();
                queue.pop_front();
                ++active;
                r->t_start = Clock::now();
            }
            // the next request may fit as well
            cv_work.notify_one();
            r->geom.src_xyz = r->src.data();
            r->geom.rec_xyz = r->rec.data();
            wv_stats st{};
            double phi = 0.0;
            const int rc = wv_misfit_gradient(&r->model, &r->geom, r->d_obs, r->mem_budget, r->tol, r->ratio_hint,
                                              &phi, r->grad, r->d_sim, &st, pool_base + r->ws_off, r->ws_bytes,
                                              streams[w]);
            {
                std::lock_guard<std::mutex> lk(mu);
                r->t_end = Clock::now();
                r->res.status = rc;
                r->res.misfit = phi;
                r->res.stats = st;
                auto ms = [&](Clock::time_point t) {
                    return std::chrono::duration<double, std::milli>(t - t0).count();
                };
                r->res.t_submit_ms = ms(r->t_submit);
                r->res.t_start_ms = ms(r->t_start);
                r->res.t_end_ms = ms(r->t_end);
                r->done = true;
                pool.give(r->ws_off, r->ws_bytes);
                --active;
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

int wv_engine_submit(wv_engine *e, const wv_model *model, const wv_geom *geom, const float *d_obs,
                     size_t mem_budget, double tol, double ratio_hint, double *grad_m, float *d_sim)
{
    if (!e || !model || !geom || !d_obs || !grad_m || !geom->src_xyz || !geom->rec_xyz) return WV_EINVAL;
    const size_t ws = wv_workspace_bytes(model, geom, WV_OP_GRADIENT, mem_budget);
    if (ws == 0) return WV_EINVAL;
    const size_t need = (ws + 255) / 256 * 256;
    if (need > e->pool_bytes) return WV_EBUDGET;   // could never be admitted
    Request *r = new Request();
    r->model = *model;
    r->geom = *geom;
    r->src.assign(geom->src_xyz, geom->src_xyz + (size_t)geom->nsrc * model->ndim);
    r->rec.assign(geom->rec_xyz, geom->rec_xyz + (size_t)geom->nrec * model->ndim);
    r->d_obs = d_obs;
    r->mem_budget = mem_budget;
    r->tol = tol;
    r->ratio_hint = ratio_hint;
    r->grad = grad_m;
    r->d_sim = d_sim;
    r->ws_bytes = need;
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
    e->cv_work.notify_one();
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
    for (hipStream_t s : e->streams) (void)hipStreamDestroy(s);
    for (auto &kv : e->reqs) delete kv.second;
    delete e;
    return WV_OK;
}

}  // extern "C"
