// Batches of independent DG cases (different meshes and degrees) on one GPU.
//
// The DG operator of every case (residual, finite-difference product of
// Sec. 5.1 Eq. DG-mf, exact product) runs in ONE persistent launch over a
// device work list of (case, element tile) items; each item selects the
// compile-time path of its degree.  The tile shape (workgroup size, elements
// per workgroup for each degree, grid) is chosen by an on-device autotuner.
// The finite-difference product (per-case steps + the persistent launch) can
// be replayed as a HIP graph.  Implicit time steps of the whole batch run each
// case's solver (Sec. 4, 6) on its own stream, several cases at a time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace dg;

namespace {

struct BErr {
    dg_status st;
};

template <class T>
struct Dev {
    T* p = nullptr;
    size_t n = 0;
    void ensure(size_t want) {
        if (want <= n) return;
        release();
        if (hipMalloc(&p, want * sizeof(T)) != hipSuccess) {
            p = nullptr;
            n = 0;
            throw BErr{DG_ENOMEM};
        }
        n = want;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

constexpr size_t LDS_MAX = 160 * 1024;      // LDS of one CU (gfx950)
constexpr int NUM_CU = 256;
constexpr int MODES = 3;                     // M_RES, M_JVP_FD, M_TANGENT

struct Tile {
    int threads = 0;
    int epb[MAXP + 1] = {0, 0, 0, 0, 0};
    int grid = 0;
    size_t lds = 0;
    double ms = -1.0;
    int tried = 0;
};

struct GraphSlot {
    const void* key[4] = {nullptr, nullptr, nullptr, nullptr};
    double shift = 0.0;
    hipGraphExec_t exec = nullptr;
};

}  // namespace

struct dg_batch {
    int device = 0;
    hipStream_t s = nullptr;          // caller's stream (NULL = the default stream)
    hipStream_t cap = nullptr;        // private stream for graph capture
    int nc = 0;
    bool ns = false, curved = false;
    std::vector<dg_ctx*> ctx;
    std::vector<hipStream_t> cs;
    std::vector<int> p;
    std::vector<size_t> off, nd;
    size_t N = 0;
    std::vector<BatchCaseDev> host_cases;
    Dev<BatchCaseDev> cases;
    Tile tile[MODES];
    Dev<BatchItem> items[MODES];
    int nitems[MODES] = {0, 0, 0};
    Dev<SegBlock> seg;
    int nseg = 0;
    Dev<int> first, nbk;
    Dev<double> px, py, h, scratch;
    bool use_graphs = true;
    GraphSlot g[MODES];
    std::string err;
};

namespace {

#define BK(expr)                                                                        \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            b->err = std::string(#expr) + ": " + hipGetErrorString(e_);                 \
            throw BErr{DG_EHIP};                                                        \
        }                                                                               \
    } while (0)

void bfail(dg_batch* b, dg_status st, const std::string& msg) {
    b->err = msg;
    throw BErr{st};
}

template <class F>
dg_status bguard(dg_batch* b, F&& f) {
    if (!b) return DG_EINVAL;
    try {
        (void)hipSetDevice(b->device);
        f();
        return DG_OK;
    } catch (const BErr& e) {
        return e.st;
    } catch (const std::bad_alloc&) {
        b->err = "host allocation failed";
        return DG_ENOMEM;
    } catch (...) {
        b->err = "unexpected exception";
        return DG_EHIP;
    }
}

int nq_of(int P) { return (P + 1) * (P + 1) * (P + 1); }

// Items of a tile shape: degrees from high to low (heavy work first), then
// case, then element.
std::vector<BatchItem> make_items(const dg_batch* b, const Tile& t) {
    std::vector<BatchItem> v;
    for (int P = MAXP; P >= 1; --P)
        for (int c = 0; c < b->nc; ++c) {
            if (b->p[c] != P) continue;
            const int ne = b->host_cases[c].m.ne;
            for (int e0 = 0; e0 < ne; e0 += t.epb[P]) v.push_back(BatchItem{c, e0, P, std::min(t.epb[P], ne - e0)});
        }
    return v;
}

// Shape with `threads` per workgroup, at most `cap` bytes of LDS where the
// degree allows more than one element, grid = min(items, gridf * CUs).
bool make_tile(const dg_batch* b, int mode, int threads, size_t cap, int gridf, Tile& t) {
    t = Tile{};
    t.threads = threads;
    bool present[MAXP + 1] = {false, false, false, false, false};
    for (int c = 0; c < b->nc; ++c) present[b->p[c]] = true;
    for (int P = 1; P <= MAXP; ++P) {
        if (!present[P]) continue;
        const int nq = nq_of(P);
        const size_t sb = batch_slot_bytes(P, mode);
        if (nq > threads || sb > LDS_MAX) return false;
        int e = threads / nq;
        const int ecap = (int)(cap / sb);
        if (ecap < e) e = ecap;
        if (e < 1) e = 1;
        t.epb[P] = e;
        t.lds = std::max(t.lds, (size_t)e * sb);
    }
    if (t.lds > LDS_MAX) return false;
    size_t ni = 0;
    for (int c = 0; c < b->nc; ++c) {
        const int ne = b->host_cases[c].m.ne;
        ni += (size_t)((ne + t.epb[b->p[c]] - 1) / t.epb[b->p[c]]);
    }
    t.grid = (int)std::min(ni, (size_t)gridf * NUM_CU);
    if (t.grid < 1) t.grid = 1;
    return true;
}

void install_tile(dg_batch* b, int mode, const Tile& t) {
    const std::vector<BatchItem> v = make_items(b, t);
    b->items[mode].ensure(std::max<size_t>(v.size(), 1));
    BK(hipMemcpy(b->items[mode].p, v.data(), v.size() * sizeof(BatchItem), hipMemcpyHostToDevice));
    b->nitems[mode] = (int)v.size();
    b->tile[mode] = t;
    if (b->g[mode].exec) {
        (void)hipGraphExecDestroy(b->g[mode].exec);
        b->g[mode] = GraphSlot{};
    }
}

int mode_of_kind(int kind) {
    switch (kind) {
        case DG_K_RESIDUAL: return M_RES;
        case DG_K_JVP_FD: return M_JVP_FD;
        case DG_K_JVP_EXACT: return M_TANGENT;
        default: return -1;
    }
}

void launch_mode(dg_batch* b, int mode, const double* W, const double* V, const double* RW, double shift,
                 double* out, hipStream_t s) {
    const Tile& t = b->tile[mode];
    if (mode == M_JVP_FD)
        BK(launch_seg_fd_step(b->seg.p, b->nseg, b->first.p, b->nbk.p, b->nc, W, V, b->px.p, b->py.p, 1e-7, b->h.p,
                              s));
    BK(launch_batch_dg(mode, b->ns, b->curved, b->cases.p, b->items[mode].p, b->nitems[mode], t.threads, t.grid, t.lds,
                       W, V, RW, b->h.p, shift, out, s));
}

// FD product as a graph replay when the same operands come back.
void run_mode(dg_batch* b, int mode, const double* W, const double* V, const double* RW, double shift, double* out) {
    if (!(b->use_graphs && mode == M_JVP_FD)) {
        launch_mode(b, mode, W, V, RW, shift, out, b->s);
        return;
    }
    GraphSlot& g = b->g[mode];
    const void* key[4] = {W, V, RW, out};
    const bool hit = g.exec && g.shift == shift && std::equal(key, key + 4, g.key);
    if (!hit) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = GraphSlot{};
        hipGraph_t graph = nullptr;
        BK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        try {
            launch_mode(b, mode, W, V, RW, shift, out, b->cap);
        } catch (...) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(b->cap, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            throw;
        }
        BK(hipStreamEndCapture(b->cap, &graph));
        hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g.exec = nullptr;
            b->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
            throw BErr{DG_EHIP};
        }
        std::copy(key, key + 4, g.key);
        g.shift = shift;
    }
    BK(hipGraphLaunch(g.exec, b->s));
}

void check_vec(dg_batch* b, const void* p, const char* what) {
    if (!p) bfail(b, DG_EINVAL, std::string(what) + " is null");
}

void release(dg_batch* b) {
    for (auto& g : b->g)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    for (dg_ctx* c : b->ctx)
        if (c) (void)dg_destroy(c);
    for (hipStream_t s : b->cs)
        if (s) (void)hipStreamDestroy(s);
    b->cases.release();
    for (auto& it : b->items) it.release();
    b->seg.release(); b->first.release(); b->nbk.release();
    b->px.release(); b->py.release(); b->h.release(); b->scratch.release();
    if (b->cap) (void)hipStreamDestroy(b->cap);
}

}  // namespace

extern "C" {

dg_status dg_batch_create(const dg_case_desc* cases, int ncases, void* hip_stream, dg_batch** out) {
    if (!out) return DG_EINVAL;
    *out = nullptr;
    if (!cases || ncases < 1 || ncases > 65536) return DG_EINVAL;
    dg_batch* b = new (std::nothrow) dg_batch();
    if (!b) return DG_ENOMEM;
    dg_status st = bguard(b, [&] {
        BK(hipGetDevice(&b->device));
        b->s = (hipStream_t)hip_stream;
        BK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        b->nc = ncases;
        b->ns = cases[0].phys.mu > 0.0;
        b->curved = cases[0].mesh.vtx != nullptr;
        for (int c = 0; c < ncases; ++c) {
            if ((cases[c].phys.mu > 0.0) != b->ns || (cases[c].mesh.vtx != nullptr) != b->curved)
                bfail(b, DG_EINVAL, "every case of a batch must share Euler/Navier-Stokes and straight/curved");
            hipStream_t cst = nullptr;
            BK(hipStreamCreateWithFlags(&cst, hipStreamNonBlocking));
            b->cs.push_back(cst);
            dg_ctx* cx = nullptr;
            const dg_status cs_ = dg_create(&cases[c].mesh, &cases[c].phys, cases[c].p, cst, &cx);
            if (cs_ != DG_OK) bfail(b, cs_, "case " + std::to_string(c) + ": dg_create failed");
            b->ctx.push_back(cx);
            b->p.push_back(cases[c].p);
            b->off.push_back(b->N);
            b->nd.push_back(dg_ndof(cx));
            BatchCaseDev d{};
            d.m = ctx_args(cx).m;
            d.g = ctx_args(cx).g;
            d.off = b->N;
            b->host_cases.push_back(d);
            b->N += dg_ndof(cx);
        }
        b->cases.ensure(ncases);
        BK(hipMemcpy(b->cases.p, b->host_cases.data(), ncases * sizeof(BatchCaseDev), hipMemcpyHostToDevice));
        // per-case reduction blocks, laid out case after case
        std::vector<SegBlock> sb;
        std::vector<int> first(ncases), nbk(ncases);
        for (int c = 0; c < ncases; ++c) {
            first[c] = (int)sb.size();
            nbk[c] = red_blocks_for(b->nd[c]);
            for (int lb = 0; lb < nbk[c]; ++lb) sb.push_back(SegBlock{c, lb, nbk[c], 0, b->off[c], b->nd[c]});
        }
        b->nseg = (int)sb.size();
        b->seg.ensure(sb.size());
        BK(hipMemcpy(b->seg.p, sb.data(), sb.size() * sizeof(SegBlock), hipMemcpyHostToDevice));
        b->first.ensure(ncases);
        b->nbk.ensure(ncases);
        BK(hipMemcpy(b->first.p, first.data(), ncases * sizeof(int), hipMemcpyHostToDevice));
        BK(hipMemcpy(b->nbk.p, nbk.data(), ncases * sizeof(int), hipMemcpyHostToDevice));
        b->px.ensure(sb.size());
        b->py.ensure(sb.size());
        b->h.ensure(ncases);
        // default tiles: 128 threads (64 when every degree fits), 64 KB, 4 workgroups per CU
        int maxnq = 0;
        for (int c = 0; c < ncases; ++c) maxnq = std::max(maxnq, nq_of(b->p[c]));
        for (int m = 0; m < MODES; ++m) {
            Tile t;
            if (!make_tile(b, m, maxnq <= 64 ? 64 : 128, 64 * 1024, 4, t)) bfail(b, DG_EINVAL, "no valid tile");
            install_tile(b, m, t);
        }
    });
    if (st != DG_OK) {
        release(b);
        delete b;
        return st;
    }
    *out = b;
    return DG_OK;
}

dg_status dg_batch_destroy(dg_batch* b) {
    if (!b) return DG_EINVAL;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->s);
    release(b);
    delete b;
    return DG_OK;
}

const char* dg_batch_last_error(const dg_batch* b) { return b ? b->err.c_str() : "null batch"; }

size_t dg_batch_ndof(const dg_batch* b, int c) {
    if (!b) return 0;
    if (c < 0) return b->N;
    return c < b->nc ? b->nd[c] : 0;
}

size_t dg_batch_offset(const dg_batch* b, int c) {
    if (!b || c < 0 || c >= b->nc) return 0;
    return b->off[c];
}

dg_ctx* dg_batch_case(dg_batch* b, int c) {
    if (!b || c < 0 || c >= b->nc) return nullptr;
    return b->ctx[c];
}

dg_status dg_batch_residual(dg_batch* b, const double* W, double* R) {
    return bguard(b, [&] {
        check_vec(b, W, "W");
        check_vec(b, R, "R");
        if (W == R) bfail(b, DG_EINVAL, "R aliases W");
        run_mode(b, M_RES, W, nullptr, nullptr, 0.0, R);
    });
}

dg_status dg_batch_jvp(dg_batch* b, const double* W, const double* RW, const double* v, double shift, double* y) {
    return bguard(b, [&] {
        check_vec(b, W, "W");
        check_vec(b, RW, "RW");
        check_vec(b, v, "v");
        check_vec(b, y, "y");
        if (y == W || y == v || y == RW) bfail(b, DG_EINVAL, "y aliases an input");
        run_mode(b, M_JVP_FD, W, v, RW, shift, y);
    });
}

dg_status dg_batch_jvp_exact(dg_batch* b, const double* W, const double* v, double shift, double* y) {
    return bguard(b, [&] {
        check_vec(b, W, "W");
        check_vec(b, v, "v");
        check_vec(b, y, "y");
        if (y == W || y == v) bfail(b, DG_EINVAL, "y aliases an input");
        run_mode(b, M_TANGENT, W, v, nullptr, shift, y);
    });
}

dg_status dg_batch_use_graphs(dg_batch* b, int enable) {
    return bguard(b, [&] {
        b->use_graphs = enable != 0;
        if (!b->use_graphs)
            for (auto& g : b->g)
                if (g.exec) {
                    (void)hipGraphExecDestroy(g.exec);
                    g = GraphSlot{};
                }
    });
}

dg_status dg_batch_get_tile(dg_batch* b, int kind, dg_batch_tile* t) {
    return bguard(b, [&] {
        const int m = mode_of_kind(kind);
        if (m < 0 || !t) bfail(b, DG_EINVAL, "kind must be DG_K_RESIDUAL, DG_K_JVP_FD or DG_K_JVP_EXACT");
        const Tile& x = b->tile[m];
        t->threads = x.threads;
        for (int P = 0; P <= MAXP; ++P) t->epb[P] = x.epb[P];
        t->grid = x.grid;
        t->lds_bytes = x.lds;
        t->ms = x.ms;
        t->candidates = x.tried;
        t->items = b->nitems[m];
    });
}

dg_status dg_batch_set_tile(dg_batch* b, int kind, int threads, size_t lds_cap, int grid_per_cu) {
    return bguard(b, [&] {
        const int m = mode_of_kind(kind);
        if (m < 0) bfail(b, DG_EINVAL, "kind must be DG_K_RESIDUAL, DG_K_JVP_FD or DG_K_JVP_EXACT");
        if (threads < 64 || threads > BATCH_MAX_THREADS || threads % 64 || grid_per_cu < 1)
            bfail(b, DG_EINVAL, "threads must be 64..256 in steps of 64, grid_per_cu >= 1");
        BK(hipStreamSynchronize(b->s));
        Tile t;
        if (!make_tile(b, m, threads, lds_cap, grid_per_cu, t)) bfail(b, DG_EINVAL, "tile does not fit these degrees");
        install_tile(b, m, t);
    });
}

// Autotuner: time every candidate shape on the given operands and keep the
// fastest.  Candidates: 64..256 threads, LDS caps 32/64/96/160 KB, 1/2/4/8
// workgroups per CU.  The output of the timed launches goes to scratch.
dg_status dg_batch_tune(dg_batch* b, int kind, const double* W, const double* RW, const double* v, int reps,
                        dg_batch_tile* chosen) {
    return bguard(b, [&] {
        const int m = mode_of_kind(kind);
        if (m < 0) bfail(b, DG_EINVAL, "kind must be DG_K_RESIDUAL, DG_K_JVP_FD or DG_K_JVP_EXACT");
        check_vec(b, W, "W");
        if (m == M_JVP_FD) check_vec(b, RW, "RW");
        if (m != M_RES) check_vec(b, v, "v");
        if (reps < 1) reps = 3;
        b->scratch.ensure(b->N);
        hipEvent_t e0, e1;
        BK(hipEventCreate(&e0));
        BK(hipEventCreate(&e1));
        Tile best;
        int tried = 0;
        try {
            const int thr[4] = {64, 128, 192, 256};
            const size_t caps[4] = {32 * 1024, 64 * 1024, 96 * 1024, LDS_MAX};
            const int gf[4] = {1, 2, 4, 8};
            std::vector<std::vector<int>> seen;
            for (int ti = 0; ti < 4; ++ti)
                for (int ci = 0; ci < 4; ++ci)
                    for (int gi = 0; gi < 4; ++gi) {
                        Tile t;
                        if (!make_tile(b, m, thr[ti], caps[ci], gf[gi], t)) continue;
                        std::vector<int> sig = {t.threads, t.grid, t.epb[1], t.epb[2], t.epb[3], t.epb[4]};
                        if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;
                        seen.push_back(sig);
                        install_tile(b, m, t);
                        launch_mode(b, m, W, v, RW, 30.0, b->scratch.p, b->s);     // warm-up
                        BK(hipEventRecord(e0, b->s));
                        for (int r = 0; r < reps; ++r) launch_mode(b, m, W, v, RW, 30.0, b->scratch.p, b->s);
                        BK(hipEventRecord(e1, b->s));
                        BK(hipEventSynchronize(e1));
                        float ms = 0.0f;
                        BK(hipEventElapsedTime(&ms, e0, e1));
                        t.ms = ms / reps;
                        ++tried;
                        if (best.ms < 0.0 || t.ms < best.ms) best = t;
                    }
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (best.ms < 0.0) bfail(b, DG_EINVAL, "no valid tile");
        best.tried = tried;
        install_tile(b, m, best);
        if (chosen) {
            chosen->threads = best.threads;
            for (int P = 0; P <= MAXP; ++P) chosen->epb[P] = best.epb[P];
            chosen->grid = best.grid;
            chosen->lds_bytes = best.lds;
            chosen->ms = best.ms;
            chosen->candidates = tried;
            chosen->items = b->nitems[m];
        }
    });
}

// One BDF2 step of every case (Sec. 4 with the pMG-FGMRES solver of Sec. 6):
// `workers` host threads each take the next case (largest first) and run its
// step on the case's own stream, so up to `workers` cases share the GPU.
dg_status dg_batch_bdf2_step(dg_batch* b, const double* Wn, const double* Wnm1, double dt, const pmg_opts* popts,
                             const fgmres_opts* fopts, double newton_rtol, int max_newton, int workers, double* Wnp1,
                             dg_step_stats* stats) {
    dg_status first_err = DG_OK;
    dg_status st = bguard(b, [&] {
        check_vec(b, Wn, "Wn");
        check_vec(b, Wnp1, "Wnp1");
        if (!popts || !fopts) bfail(b, DG_EINVAL, "popts/fopts are null");
        if (Wnp1 == Wn || Wnp1 == Wnm1) bfail(b, DG_EINVAL, "Wnp1 aliases an input");
        if (workers < 1) workers = 1;
        if (workers > b->nc) workers = b->nc;
        BK(hipStreamSynchronize(b->s));          // inputs written on the batch stream are ready
        std::vector<int> order(b->nc);
        for (int c = 0; c < b->nc; ++c) order[c] = c;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->nd[x] > b->nd[y]; });
        std::vector<dg_status> res(b->nc, DG_OK);
        std::vector<std::string> msg(b->nc);
        std::atomic<int> next{0};
        auto work = [&] {
            (void)hipSetDevice(b->device);
            for (;;) {
                const int k = next.fetch_add(1);
                if (k >= b->nc) break;
                const int c = order[k];
                dg_step_stats local{};
                res[c] = dg_bdf2_step(b->ctx[c], Wn + b->off[c], Wnm1 ? Wnm1 + b->off[c] : nullptr, dt, &popts[c],
                                      fopts, newton_rtol, max_newton, Wnp1 + b->off[c], &local);
                if (stats) stats[c] = local;
                if (res[c] != DG_OK) msg[c] = dg_last_error(b->ctx[c]);
            }
        };
        std::vector<std::thread> pool;
        for (int t = 1; t < workers; ++t) pool.emplace_back(work);
        work();
        for (auto& t : pool) t.join();
        for (int c = 0; c < b->nc; ++c) BK(hipStreamSynchronize(b->cs[c]));
        for (int c = 0; c < b->nc; ++c)
            if (res[c] != DG_OK && res[c] != DG_ENOCONV) {
                b->err = "case " + std::to_string(c) + ": " + msg[c];
                throw BErr{res[c]};
            }
        for (int c = 0; c < b->nc; ++c)
            if (res[c] == DG_ENOCONV) {
                b->err = "case " + std::to_string(c) + ": " + msg[c];
                first_err = DG_ENOCONV;
                break;
            }
    });
    return st != DG_OK ? st : first_err;
}

}  // extern "C"
