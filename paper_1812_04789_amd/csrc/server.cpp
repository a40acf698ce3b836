// Serving loop: implicit time-step requests (one BDF2 step of Sec. 4 with the
// pMG-FGMRES solver of Sec. 6 each) admitted by device-memory footprint and
// run concurrently on the GPU.
//
// `slots` worker threads each own one request at a time and run it on the
// request's context stream, so up to `slots` requests overlap on the device.
// Admission is first-in first-out: the oldest waiting request starts as soon
// as a slot is free and its footprint (dg_footprint_bytes) fits in the budget
// next to the contexts the server holds; idle cached contexts are freed (least
// recently used first) to make room.  Contexts of straight-box requests are
// kept after completion and reused by later requests of the same mesh,
// degree and gas, so their device state stays resident.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

namespace {

using Clock = std::chrono::steady_clock;

// Requests share a cached context only when mesh, degree, gas and every
// option that decides the context's allocations agree, so a reused context
// never grows beyond the footprint charged for it.
struct Key {
    int nx, ny, nz, p;
    double lo[3], hi[3];
    double gamma, mu, Pr, eta;
    int levels[5], prec_fine, prec_coarse, cmf, cplain, smoother, cycle, nu, cprec, citers, restart;
    bool operator==(const Key& o) const {
        return nx == o.nx && ny == o.ny && nz == o.nz && p == o.p && std::equal(lo, lo + 3, o.lo) &&
               std::equal(hi, hi + 3, o.hi) && gamma == o.gamma && mu == o.mu && Pr == o.Pr && eta == o.eta &&
               std::equal(levels, levels + 5, o.levels) && prec_fine == o.prec_fine && prec_coarse == o.prec_coarse &&
               cmf == o.cmf && cplain == o.cplain && smoother == o.smoother && cycle == o.cycle && nu == o.nu && cprec == o.cprec &&
               citers == o.citers && restart == o.restart;
    }
};

struct Entry {
    Key key{};
    dg_ctx* ctx = nullptr;
    hipStream_t s = nullptr;
    double bytes = 0.0;         // charged against the budget
    bool busy = false;
    bool cacheable = true;
    long long last_used = 0;
};

struct Pending {
    dg_request rq;
    double t_submit = 0.0;
    double fp = 0.0;
};

Key key_of(const dg_request& r) {
    Key k{};
    k.nx = r.mesh.nx;
    k.ny = r.mesh.ny;
    k.nz = r.mesh.nz;
    k.p = r.p;
    std::copy(r.mesh.lo, r.mesh.lo + 3, k.lo);
    std::copy(r.mesh.hi, r.mesh.hi + 3, k.hi);
    k.gamma = r.phys.gamma;
    k.mu = r.phys.mu;
    k.Pr = r.phys.Pr;
    k.eta = r.phys.eta;
    k.levels[0] = r.popts.n_levels;
    for (int i = 0; i < 4; ++i) k.levels[1 + i] = i < r.popts.n_levels ? r.popts.p_level[i] : 0;
    k.prec_fine = r.popts.prec_fine;
    k.prec_coarse = r.popts.prec_coarse;
    k.cmf = r.popts.coarse_matrix_free;
    k.cplain = r.popts.coarsest_plain;
    k.smoother = r.popts.smoother;
    k.cycle = r.popts.cycle;
    k.cprec = r.popts.coarsest_prec;
    k.nu = r.popts.smoother == 1 ? std::max(r.popts.nu_pre, r.popts.nu_post) : 0;
    k.citers = r.popts.coarsest_iters;
    k.restart = r.fopts.restart;
    return k;
}

void destroy_entry(Entry& e) {
    if (e.ctx) (void)dg_destroy(e.ctx);
    if (e.s) (void)hipStreamDestroy(e.s);
    e.ctx = nullptr;
    e.s = nullptr;
}

}  // namespace

struct dg_server {
    int device = 0;
    dg_server_opts o{};
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Pending> pending;
    std::vector<Entry*> entries;
    std::vector<dg_response> done;
    double held = 0.0;               // bytes charged by contexts the server holds
    double peak_held = 0.0;
    int running = 0;
    long long submitted = 0, completed = 0, tick = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    std::string err;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    // Called with the lock held: admit the head request if possible.
    // Returns the entry to run it on (new entries have ctx == nullptr).
    Entry* admit(const Pending& h) {
        const Key k = key_of(h.rq);
        const bool cacheable = (h.rq.mesh.vtx == nullptr) && o.cache;
        if (cacheable)
            for (Entry* e : entries)
                if (!e->busy && e->cacheable && e->key == k) {
                    // a cached context: charge the growth if this request needs more
                    const double extra = std::max(0.0, h.fp - e->bytes);
                    if (held + extra > o.hbm_budget && !evict_until(extra, e)) return nullptr;
                    held += extra;
                    e->bytes += extra;
                    return e;
                }
        if (held + h.fp > o.hbm_budget && !evict_until(h.fp, nullptr)) return nullptr;
        Entry* e = new Entry();
        e->key = k;
        e->bytes = h.fp;
        e->cacheable = cacheable;
        held += h.fp;
        entries.push_back(e);
        return e;
    }

    // Free idle contexts, least recently used first, until `need` bytes fit.
    bool evict_until(double need, const Entry* keep) {
        for (;;) {
            if (held + need <= o.hbm_budget) return true;
            Entry* victim = nullptr;
            for (Entry* e : entries)
                if (!e->busy && e != keep && (!victim || e->last_used < victim->last_used)) victim = e;
            if (!victim) return false;
            held -= victim->bytes;
            destroy_entry(*victim);
            entries.erase(std::find(entries.begin(), entries.end(), victim));
            delete victim;
        }
    }

    void worker() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            Entry* e = nullptr;
            Pending job;
            for (;;) {
                if (stop && pending.empty()) return;
                if (!pending.empty()) {
                    if (pending.front().fp > o.hbm_budget) {      // can never fit: fail it
                        Pending bad = pending.front();
                        pending.pop_front();
                        dg_response r{};
                        r.tag = bad.rq.tag;
                        r.status = DG_ENOMEM;
                        r.t_submit = r.t_admit = bad.t_submit;
                        r.t_done = now();
                        r.footprint = bad.fp;
                        done.push_back(r);
                        ++completed;
                        cv_done.notify_all();
                        continue;
                    }
                    e = admit(pending.front());
                    if (e) {
                        job = pending.front();
                        pending.pop_front();
                        e->busy = true;
                        peak_held = std::max(peak_held, held);
                        ++running;
                        break;
                    }
                }
                cv_work.wait(lk);
            }
            const double t_admit = now();
            const int slot_running = running;
            lk.unlock();
            dg_response r{};
            r.tag = job.rq.tag;
            r.t_submit = job.t_submit;
            r.t_admit = t_admit;
            r.footprint = job.fp;
            r.concurrent = slot_running;
            dg_status st = DG_OK;
            if (!e->ctx) {
                if (hipStreamCreateWithFlags(&e->s, hipStreamNonBlocking) != hipSuccess) st = DG_EHIP;
                if (st == DG_OK) st = dg_create(&job.rq.mesh, &job.rq.phys, job.rq.p, e->s, &e->ctx);
            }
            if (st == DG_OK) {
                r.ndof = dg_ndof(e->ctx);
                st = dg_bdf2_step(e->ctx, job.rq.Wn, job.rq.Wnm1, job.rq.dt, &job.rq.popts, &job.rq.fopts,
                                  job.rq.newton_rtol, job.rq.max_newton, job.rq.Wnp1, &r.stats);
                if (hipStreamSynchronize(e->s) != hipSuccess && st == DG_OK) st = DG_EHIP;
                r.device_bytes = dg_device_bytes(e->ctx);
            }
            r.status = st;
            r.t_done = now();
            lk.lock();
            --running;
            e->busy = false;
            e->last_used = ++tick;
            // charge what the context really holds (bounded below by zero growth)
            if (e->ctx && r.device_bytes > e->bytes) {
                held += r.device_bytes - e->bytes;
                e->bytes = r.device_bytes;
            }
            if (st != DG_OK && st != DG_ENOCONV) {
                std::string m = e->ctx ? dg_last_error(e->ctx) : "context creation failed";
                err = "request " + std::to_string(r.tag) + ": " + m;
            }
            if (!e->cacheable || !e->ctx || (st != DG_OK && st != DG_ENOCONV)) {
                held -= e->bytes;
                destroy_entry(*e);
                entries.erase(std::find(entries.begin(), entries.end(), e));
                delete e;
            }
            done.push_back(r);
            ++completed;
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }
};

extern "C" {

dg_status dg_server_create(const dg_server_opts* opts, dg_server** out) {
    if (!out || !opts) return DG_EINVAL;
    *out = nullptr;
    if (opts->slots < 1 || opts->slots > 64 || opts->hbm_budget < 0.0) return DG_EINVAL;
    dg_server* sv = new (std::nothrow) dg_server();
    if (!sv) return DG_ENOMEM;
    sv->o = *opts;
    if (hipGetDevice(&sv->device) != hipSuccess) {
        delete sv;
        return DG_EHIP;
    }
    if (sv->o.hbm_budget == 0.0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete sv;
            return DG_EHIP;
        }
        sv->o.hbm_budget = 0.85 * (double)fr;
    }
    sv->t0 = Clock::now();
    try {
        for (int i = 0; i < sv->o.slots; ++i) sv->workers.emplace_back([sv] { sv->worker(); });
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stop = true;
        }
        sv->cv_work.notify_all();
        for (auto& t : sv->workers) t.join();
        delete sv;
        return DG_ENOMEM;
    }
    *out = sv;
    return DG_OK;
}

double dg_server_time(const dg_server* sv) { return sv ? sv->now() : 0.0; }

dg_status dg_server_submit(dg_server* sv, const dg_request* rq) {
    if (!sv || !rq || !rq->Wn || !rq->Wnp1 || rq->p < 1 || rq->p > dg::MAXP) return DG_EINVAL;
    if (rq->mesh.vtx) return DG_EINVAL;          // the serving loop takes straight boxes
    const double fp = dg_footprint_bytes(&rq->mesh, rq->p, &rq->popts, &rq->fopts);
    if (!(fp > 0.0)) return DG_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return DG_ESTATE;
    Pending pd;
    pd.rq = *rq;
    pd.t_submit = sv->now();
    pd.fp = fp;
    sv->pending.push_back(pd);
    ++sv->submitted;
    sv->cv_work.notify_one();
    return DG_OK;
}

int dg_server_poll(dg_server* sv, dg_response* out, int max, int wait_ms) {
    if (!sv || !out || max < 1) return -1;
    std::unique_lock<std::mutex> lk(sv->mu);
    if (sv->done.empty() && wait_ms > 0)
        sv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [sv] { return !sv->done.empty(); });
    const int n = (int)std::min<size_t>(sv->done.size(), (size_t)max);
    std::copy(sv->done.begin(), sv->done.begin() + n, out);
    sv->done.erase(sv->done.begin(), sv->done.begin() + n);
    return n;
}

dg_status dg_server_drain(dg_server* sv) {
    if (!sv) return DG_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [sv] { return sv->completed == sv->submitted; });
    return DG_OK;
}

dg_status dg_server_stats(dg_server* sv, dg_server_info* info) {
    if (!sv || !info) return DG_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    info->submitted = sv->submitted;
    info->completed = sv->completed;
    info->pending = (long long)sv->pending.size();
    info->running = sv->running;
    info->contexts = (int)sv->entries.size();
    info->held_bytes = sv->held;
    info->peak_held_bytes = sv->peak_held;
    info->budget_bytes = sv->o.hbm_budget;
    return DG_OK;
}

const char* dg_server_last_error(const dg_server* sv) { return sv ? sv->err.c_str() : "null server"; }

dg_status dg_server_destroy(dg_server* sv) {
    if (!sv) return DG_EINVAL;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    for (auto& t : sv->workers) t.join();
    (void)hipSetDevice(sv->device);
    for (Entry* e : sv->entries) {
        destroy_entry(*e);
        delete e;
    }
    delete sv;
    return DG_OK;
}

}  // extern "C"
