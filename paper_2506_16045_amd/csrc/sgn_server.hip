// libsgn request server: HBM-footprint admission, continuous batching of small
// 1D solves into sgn_batch_solve launches, and worker lanes (one context and
// HIP stream each) for 2D and large 1D solves and RK4 time-steps.  A client of
// the C ABI in sgn.h.
#include "sgn.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

constexpr int BATCH_N_MAX = 8192;      // largest 1D size the batched solver takes
constexpr size_t ALIGN = 256;

size_t up(size_t b) { return (b + ALIGN - 1) & ~(ALIGN - 1); }

bool grid_ok(const sgn_grid& g) {
    auto pow2 = [](int v) { return v >= 2 && (v & (v - 1)) == 0; };
    if (g.bc != SGN_BC_PERIODIC) return false;   // served requests: periodic grids
    if (g.dim == 1) return pow2(g.nx) && g.nx <= 16384 && g.Lx > 0.0 && std::isfinite(g.Lx);
    if (g.dim == 2)
        return pow2(g.nx) && pow2(g.ny) && g.nx <= 4096 && g.ny <= 1024 && g.Lx > 0.0 && g.Ly > 0.0 &&
               std::isfinite(g.Lx) && std::isfinite(g.Ly);
    return false;
}

size_t npts(const sgn_grid& g) { return (size_t)g.nx * (g.dim == 2 ? (size_t)g.ny : 1); }

bool batchable(const sgn_request& r) {
    return r.kind == SGN_REQ_SOLVE && r.grid.dim == 1 && r.grid.nx <= BATCH_N_MAX;
}

// Device layout of a lane request: fields, then the Krylov workspace, then the
// stepping state workspace (STEP).  Offsets in bytes.
struct LaneLayout {
    size_t eta, gh, rhs, u, h, U, ws, sws, total;
};

LaneLayout lane_layout(const sgn_request& r) {
    LaneLayout l{};
    const size_t N = npts(r.grid), dN = (size_t)r.grid.dim * N;
    size_t o = 0;
    auto take = [&](size_t doubles) {
        const size_t at = o;
        o += up(doubles * sizeof(double));
        return at;
    };
    l.eta = take(N);
    l.gh = take(dN);
    l.u = take(dN);
    if (r.kind == SGN_REQ_SOLVE) {
        l.rhs = take(dN);
    } else {
        l.h = take(N);
        l.U = take(dN);
    }
    l.ws = o;
    o += up(sgn_workspace_bytes(&r.grid, r.opts.precision));
    if (r.kind == SGN_REQ_STEP_RK4) {
        l.sws = o;
        o += up(sgn_state_workspace_bytes(&r.grid, r.opts.precision));
    }
    l.total = o;
    return l;
}

// Size class of a pooled lane block: the power of two (at least 4 KiB) that
// holds `b` bytes, which is what a lane request really occupies.
size_t pool_class(size_t b) {
    size_t c = 4096;
    while (c < b) c <<= 1;
    return c;
}

// Device bytes charged to an admitted request: its pooled block for a lane
// request; for a batched 1D solve its fields and its share of the batching
// lane's buffer (a group's buffer never exceeds the sum of its members' charges).
size_t footprint(const sgn_request& r) {
    if (batchable(r)) {
        const int32_t n = r.grid.nx;
        return 4 * up((size_t)n * sizeof(double)) + sgn_batch_workspace_bytes(1, &n, r.opts.precision);
    }
    return pool_class(lane_layout(r).total);
}

bool request_ok(const sgn_request& r) {
    if (r.kind != SGN_REQ_SOLVE && r.kind != SGN_REQ_STEP_RK4) return false;
    if (!grid_ok(r.grid)) return false;
    if (r.opts.method != SGN_PCG) return false;
    if (r.opts.precision != SGN_FP64 && r.opts.precision != SGN_MIXED) return false;
    if (!(r.opts.tol > 0.0) || r.opts.max_iter < 1) return false;
    if (!r.h_eta || !r.h_u_out) return false;
    if (r.kind == SGN_REQ_SOLVE) {
        if (!r.h_grad_h || !r.h_rhs) return false;
        if (r.opts.x0_is_guess && !r.h_u0) return false;
    } else {
        if (!r.h_h || !r.h_u0 || r.nsteps < 0 || !std::isfinite(r.dt)) return false;
    }
    return true;
}

struct Req {
    uint64_t id = 0;
    sgn_request r{};
    std::vector<double> in;   // copied inputs: eta | grad_h | rhs | h | u0
    size_t fp = 0;
    bool batch = false;
    sgn_result res{};         // read and written under the server mutex only
};

// What a lane or the batching lane learned about a request; copied into the
// request's result under the server mutex when it finishes.
struct Outcome {
    int64_t iters = 0, solves = 0;
    double relres = 0.0;
    int32_t batched = 0, batch_size = 0;
};

// Device memory kept in power-of-two size classes for reuse (hipFree would
// synchronise the device under running lanes).  Cached free blocks are given
// back (trim) when an allocation would otherwise take the server's device
// memory past its budget.
class Pool {
   public:
    explicit Pool(size_t budget = 0) : budget_(budget) {}
    void set_budget(size_t b) { budget_ = b; }

    // A block of class c: a cached one, else a new allocation; if the new block
    // would take the held bytes past the budget, the cached blocks are freed first.
    void* get(size_t c) {
        std::lock_guard<std::mutex> g(m_);
        auto& v = free_[c];
        if (!v.empty()) {
            void* p = v.back();
            v.pop_back();
            free_bytes_ -= c;
            return p;
        }
        void* p = alloc_locked(c);
        if (p) all_[p] = c;
        return p;
    }
    // Replace the batching lane's buffer (`old`, old_bytes) by one of `need` bytes,
    // under the same accounting.  Returns null (old freed) on failure.
    void* regrow(void* old, size_t old_bytes, size_t need) {
        std::lock_guard<std::mutex> g(m_);
        if (old) {
            (void)hipFree(old);
            held_ -= old_bytes;
        }
        return alloc_locked(need);
    }
    void free_extra(void* p, size_t bytes) {
        std::lock_guard<std::mutex> g(m_);
        if (p) {
            (void)hipFree(p);
            held_ -= bytes;
        }
    }
    void put(void* p, size_t c) {
        std::lock_guard<std::mutex> g(m_);
        free_[c].push_back(p);
        free_bytes_ += c;
    }
    // Device bytes held: pooled blocks (cached or in use) and the batch buffer.
    size_t held() {
        std::lock_guard<std::mutex> g(m_);
        return held_;
    }
    void release() {
        std::lock_guard<std::mutex> g(m_);
        for (auto& kv : all_) (void)hipFree(kv.first);
        all_.clear();
        free_.clear();
        held_ = free_bytes_ = 0;
    }

   private:
    void* alloc_locked(size_t bytes) {
        if (held_ + bytes > budget_) trim_locked();
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            trim_locked();
            if (hipMalloc(&p, bytes) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
        }
        held_ += bytes;
        return p;
    }
    void trim_locked() {
        for (auto& kv : free_) {
            for (void* p : kv.second) {
                (void)hipFree(p);
                all_.erase(p);
                held_ -= kv.first;
            }
            kv.second.clear();
        }
        free_bytes_ = 0;
    }
    std::mutex m_;
    std::map<size_t, std::vector<void*>> free_;
    std::unordered_map<void*, size_t> all_;
    size_t held_ = 0, free_bytes_ = 0, budget_ = 0;
};

struct Lane {
    sgn_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    std::thread th;
};

}  // namespace

struct sgn_server {
    int device = 0;
    size_t budget = 0;
    int max_batch = 1024;
    Clock::time_point t0;
    std::mutex m;
    std::condition_variable cv_work;   // lanes and the batching lane wait here
    std::condition_variable cv_done;   // waiters
    std::deque<Req*> queued;           // submitted, not yet admitted
    std::deque<Req*> lane_q;           // admitted, for the worker lanes
    std::deque<Req*> batch_q;          // admitted, for the batching lane
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    uint64_t next_id = 1;
    // Device memory accounting (under m).  lane_charged: pooled blocks of the
    // admitted lane requests; batch_charged: footprints of the admitted batched
    // solves.  The batching lane's grow-only buffer (d_batch_bytes) stays held
    // after its group finishes, so the commitment is
    //   lane_charged + max(batch_charged, d_batch_bytes) <= budget,
    // and every block the server holds (pool blocks, cached or in use, and the
    // batch buffer) is freed back to that bound before an allocation exceeds it.
    size_t lane_charged = 0, batch_charged = 0;
    int64_t n_admitted = 0, n_completed = 0;
    int running = 0;                   // requests taken by a lane and not yet finished
    bool stopping = false;
    std::vector<Lane> lanes;
    Lane blane;
    Pool pool;
    // batching lane buffers (grow only)
    void* d_batch = nullptr;
    size_t d_batch_bytes = 0;
    double* h_stage = nullptr;
    size_t h_stage_doubles = 0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    // Admit queued requests in arrival order while they fit (caller holds m).
    void admit_locked() {
        bool any = false;
        while (!queued.empty()) {
            Req* q = queued.front();
            const size_t after = q->batch ? lane_charged + std::max(batch_charged + q->fp, d_batch_bytes)
                                          : lane_charged + q->fp + std::max(batch_charged, d_batch_bytes);
            if (after > budget) break;
            queued.pop_front();
            (q->batch ? batch_charged : lane_charged) += q->fp;
            q->res.t_admit = now();
            ++n_admitted;
            (q->batch ? batch_q : lane_q).push_back(q);
            any = true;
        }
        if (any) cv_work.notify_all();
    }

    void finish(Req* q, sgn_status st, const Outcome& oc) {
        std::lock_guard<std::mutex> g(m);
        q->res.iters = oc.iters;
        q->res.solves = oc.solves;
        q->res.relres = oc.relres;
        q->res.batched = oc.batched;
        q->res.batch_size = oc.batch_size;
        q->res.status = st;
        q->res.t_done = now();
        q->res.done = 1;
        (q->batch ? batch_charged : lane_charged) -= q->fp;
        ++n_completed;
        --running;
        admit_locked();
        cv_done.notify_all();
        cv_work.notify_all();
    }



    bool idle_locked() const { return queued.empty() && lane_q.empty() && batch_q.empty() && running == 0; }

    void lane_loop(Lane* L);
    void batch_loop();
    sgn_status run_lane(Lane* L, Req* q, Outcome* oc);
};

sgn_status sgn_server::run_lane(Lane* L, Req* q, Outcome* oc) {
    const sgn_request& r = q->r;
    const LaneLayout lay = lane_layout(r);
    const size_t cls = pool_class(lay.total);
    char* base = static_cast<char*>(pool.get(cls));
    if (!base) return SGN_ENOMEM;
    const size_t N = npts(r.grid), dN = (size_t)r.grid.dim * N;
    auto D = [&](size_t off) { return reinterpret_cast<double*>(base + off); };
    auto h2d = [&](double* dst, const double* src, size_t n) {
        return hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyHostToDevice, L->stream) == hipSuccess;
    };
    auto d2h = [&](double* dst, const double* src, size_t n) {
        return hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToHost, L->stream) == hipSuccess;
    };
    sgn_status st = SGN_OK;
    bool ok = true;
    if (r.kind == SGN_REQ_SOLVE) {
        ok = h2d(D(lay.eta), r.h_eta, N) && h2d(D(lay.gh), r.h_grad_h, dN) && h2d(D(lay.rhs), r.h_rhs, dN);
        if (ok) {
            if (r.opts.x0_is_guess)
                ok = h2d(D(lay.u), r.h_u0, dN);
            else
                ok = hipMemsetAsync(D(lay.u), 0, dN * sizeof(double), L->stream) == hipSuccess;
        }
        if (!ok) st = SGN_EDEVICE;
        sgn_solve_info info{};
        if (st == SGN_OK)
            st = sgn_krylov_solve(L->ctx, &r.grid, D(lay.eta), D(lay.gh), D(lay.rhs), D(lay.u), nullptr, &r.opts,
                                  &info, base + lay.ws);
        oc->iters = info.iters;
        oc->solves = 1;
        oc->relres = info.relres;
        if ((st == SGN_OK || st == SGN_ENOCONV) && !(d2h(r.h_u_out, D(lay.u), dN))) st = SGN_EDEVICE;
    } else {
        ok = h2d(D(lay.h), r.h_h, N) && h2d(D(lay.eta), r.h_eta, N) && h2d(D(lay.u), r.h_u0, dN);
        if (!ok) st = SGN_EDEVICE;
        int32_t flat = 0;
        if (st == SGN_OK) st = sgn_bathy_prepare(L->ctx, &r.grid, D(lay.h), D(lay.gh), &flat, base + lay.ws);
        if (st == SGN_OK)
            st = sgn_apply_constraint(L->ctx, &r.grid, D(lay.eta), D(lay.gh), D(lay.u), D(lay.U), base + lay.ws);
        sgn_state* state = nullptr;
        if (st == SGN_OK)
            st = sgn_state_create(L->ctx, &r.grid, D(lay.h), D(lay.gh), flat, D(lay.eta), D(lay.U), D(lay.u),
                                  base + lay.sws, base + lay.ws, &state);
        sgn_step_info info{};
        if (st == SGN_OK) st = sgn_step_rk4(L->ctx, state, r.dt, r.nsteps, &r.opts, &info);
        if (state) sgn_state_destroy(state);
        oc->iters = info.iters;
        oc->solves = info.solves;
        if (st == SGN_OK || st == SGN_ENOCONV) {
            ok = d2h(r.h_u_out, D(lay.u), dN);
            if (ok && r.h_eta_out) ok = d2h(r.h_eta_out, D(lay.eta), N);
            if (!ok) st = SGN_EDEVICE;
        }
    }
    if (hipStreamSynchronize(L->stream) != hipSuccess && st == SGN_OK) st = SGN_EDEVICE;
    pool.put(base, cls);
    return st;
}

void sgn_server::lane_loop(Lane* L) {
    (void)hipSetDevice(device);
    for (;;) {
        Req* q = nullptr;
        {
            std::unique_lock<std::mutex> g(m);
            cv_work.wait(g, [&] { return !lane_q.empty() || (stopping && idle_locked()); });
            if (lane_q.empty()) return;
            q = lane_q.front();
            lane_q.pop_front();
            ++running;
            q->res.t_start = now();
        }
        Outcome oc;
        const sgn_status st = run_lane(L, q, &oc);
        finish(q, st, oc);
    }
}

namespace {
bool same_batch_opts(const sgn_solve_opts& a, const sgn_solve_opts& b) {
    return a.precision == b.precision && a.tol == b.tol && a.max_iter == b.max_iter &&
           a.x0_is_guess == b.x0_is_guess && a.inner_tol == b.inner_tol && a.max_outer == b.max_outer &&
           a.coeff_kind == b.coeff_kind;
}
}  // namespace

void sgn_server::batch_loop() {
    (void)hipSetDevice(device);
    for (;;) {
        std::vector<Req*> group;
        {
            std::unique_lock<std::mutex> g(m);
            cv_work.wait(g, [&] { return !batch_q.empty() || (stopping && idle_locked()); });
            if (batch_q.empty()) return;
            // every admitted 1D solve with the options of the oldest one joins this launch
            const sgn_solve_opts key = batch_q.front()->r.opts;
            for (auto it = batch_q.begin(); it != batch_q.end() && (int)group.size() < max_batch;) {
                if (same_batch_opts((*it)->r.opts, key)) {
                    group.push_back(*it);
                    it = batch_q.erase(it);
                } else {
                    ++it;
                }
            }
            const double ts = now();
            for (Req* q : group) q->res.t_start = ts;
            running += (int)group.size();
        }
        const int n = (int)group.size();
        std::vector<int32_t> sizes(n);
        std::vector<double> periods(n);
        size_t tot = 0;
        for (int i = 0; i < n; ++i) {
            sizes[i] = group[i]->r.grid.nx;
            periods[i] = group[i]->r.grid.Lx;
            tot += (size_t)sizes[i];
        }
        const sgn_solve_opts opts = group[0]->r.opts;
        const size_t wsb = sgn_batch_workspace_bytes(n, sizes.data(), opts.precision);
        const size_t need = 4 * up(tot * sizeof(double)) + up(wsb);
        sgn_status st = SGN_OK;
        if (need > d_batch_bytes) {
            // the group's charges cover `need` (each member was charged its fields and
            // a one-system workspace, at least its share of the group's)
            void* nb = pool.regrow(d_batch, d_batch_bytes, need);
            std::lock_guard<std::mutex> g(m);
            d_batch = nb;
            d_batch_bytes = nb ? need : 0;
            if (!nb) st = SGN_ENOMEM;
        }
        if (st == SGN_OK && 4 * tot > h_stage_doubles) {
            if (h_stage) (void)hipHostFree(h_stage);
            h_stage = nullptr;
            h_stage_doubles = 0;
            if (hipHostMalloc((void**)&h_stage, 4 * tot * sizeof(double), hipHostMallocDefault) == hipSuccess)
                h_stage_doubles = 4 * tot;
            else
                st = SGN_ENOMEM;
        }
        std::vector<sgn_solve_info> info(n);
        sgn_status bst = SGN_OK;
        if (st == SGN_OK) {
            // pack eta | h_x | rhs | u0 in pinned memory, one copy in, one copy out
            double* he = h_stage;
            double* hg = he + tot;
            double* hb = hg + tot;
            double* hu = hb + tot;
            size_t o = 0;
            for (int i = 0; i < n; ++i) {
                const sgn_request& r = group[i]->r;
                const size_t ni = (size_t)sizes[i];
                std::memcpy(he + o, r.h_eta, ni * sizeof(double));
                std::memcpy(hg + o, r.h_grad_h, ni * sizeof(double));
                std::memcpy(hb + o, r.h_rhs, ni * sizeof(double));
                if (opts.x0_is_guess)
                    std::memcpy(hu + o, r.h_u0, ni * sizeof(double));
                else
                    std::memset(hu + o, 0, ni * sizeof(double));
                o += ni;
            }
            double* d = static_cast<double*>(d_batch);
            const size_t stride = up(tot * sizeof(double)) / sizeof(double);
            double *de = d, *dg = d + stride, *db = d + 2 * stride, *du = d + 3 * stride;
            void* dws = d + 4 * stride;
            bool ok = hipMemcpyAsync(de, he, tot * sizeof(double), hipMemcpyHostToDevice, blane.stream) == hipSuccess &&
                      hipMemcpyAsync(dg, hg, tot * sizeof(double), hipMemcpyHostToDevice, blane.stream) == hipSuccess &&
                      hipMemcpyAsync(db, hb, tot * sizeof(double), hipMemcpyHostToDevice, blane.stream) == hipSuccess &&
                      hipMemcpyAsync(du, hu, tot * sizeof(double), hipMemcpyHostToDevice, blane.stream) == hipSuccess;
            if (!ok) st = SGN_EDEVICE;
            if (st == SGN_OK) {
                bst = sgn_batch_solve(blane.ctx, n, sizes.data(), periods.data(), de, dg, db, du, &opts, info.data(),
                                      dws);
                if (bst != SGN_OK && bst != SGN_ENOCONV && bst != SGN_EDOMAIN) st = bst;
            }
            if (st == SGN_OK) {
                if (hipMemcpyAsync(hu, du, tot * sizeof(double), hipMemcpyDeviceToHost, blane.stream) != hipSuccess ||
                    hipStreamSynchronize(blane.stream) != hipSuccess)
                    st = SGN_EDEVICE;
            }
            if (st == SGN_OK) {
                o = 0;
                for (int i = 0; i < n; ++i) {
                    std::memcpy(group[i]->r.h_u_out, hu + o, (size_t)sizes[i] * sizeof(double));
                    o += (size_t)sizes[i];
                }
            }
        }
        for (int i = 0; i < n; ++i) {
            Outcome oc;
            oc.batched = 1;
            oc.batch_size = n;
            sgn_status qs = st;
            if (st == SGN_OK) {
                oc.iters = info[i].iters;
                oc.solves = 1;
                oc.relres = info[i].relres;
                if (!(info[i].relres == info[i].relres))
                    qs = SGN_EDOMAIN;
                else if (!info[i].converged)
                    qs = SGN_ENOCONV;
            }
            finish(group[i], qs, oc);
        }
    }
}

extern "C" {

size_t sgn_request_footprint(const sgn_request* req) {
    if (!req || !request_ok(*req)) return 0;
    return footprint(*req);
}

sgn_status sgn_server_create(sgn_server** out, int device, const sgn_server_opts* opts) {
    if (!out) return SGN_EINVAL;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return SGN_EDEVICE;
    std::unique_ptr<sgn_server> s(new (std::nothrow) sgn_server());
    if (!s) return SGN_ENOMEM;
    s->device = device;
    s->t0 = Clock::now();
    size_t fr = 0, total = 0;
    if (hipMemGetInfo(&fr, &total) != hipSuccess) return SGN_EDEVICE;
    s->budget = (opts && opts->hbm_budget) ? opts->hbm_budget : (size_t)(0.8 * (double)fr);
    s->pool.set_budget(s->budget);
    const int nl = (opts && opts->lanes > 0) ? opts->lanes : 3;
    s->max_batch = (opts && opts->max_batch > 0) ? opts->max_batch : 1024;
    auto make_lane = [&](Lane& L) -> bool {
        if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess) return false;
        return sgn_create(&L.ctx, device, L.stream) == SGN_OK;
    };
    s->lanes.resize(nl);
    bool ok = make_lane(s->blane);
    for (auto& L : s->lanes) ok = ok && make_lane(L);
    if (!ok) {
        for (auto& L : s->lanes) {
            if (L.ctx) sgn_destroy(L.ctx);
            if (L.stream) (void)hipStreamDestroy(L.stream);
        }
        if (s->blane.ctx) sgn_destroy(s->blane.ctx);
        if (s->blane.stream) (void)hipStreamDestroy(s->blane.stream);
        return SGN_EDEVICE;
    }
    sgn_server* sp = s.get();
    for (auto& L : s->lanes) L.th = std::thread([sp, &L] { sp->lane_loop(&L); });
    s->blane.th = std::thread([sp] { sp->batch_loop(); });
    *out = s.release();
    return SGN_OK;
}

void sgn_server_destroy(sgn_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->m);
        s->stopping = true;
        s->cv_work.notify_all();
    }
    for (auto& L : s->lanes)
        if (L.th.joinable()) L.th.join();
    if (s->blane.th.joinable()) s->blane.th.join();
    for (auto& L : s->lanes) {
        sgn_destroy(L.ctx);
        (void)hipStreamDestroy(L.stream);
    }
    sgn_destroy(s->blane.ctx);
    (void)hipStreamDestroy(s->blane.stream);
    s->pool.free_extra(s->d_batch, s->d_batch_bytes);
    if (s->h_stage) (void)hipHostFree(s->h_stage);
    s->pool.release();
    delete s;
}

sgn_status sgn_server_submit(sgn_server* s, const sgn_request* req, uint64_t* id) {
    if (!s || !req || !id) return SGN_EINVAL;
    if (!request_ok(*req)) return SGN_EINVAL;
    std::unique_ptr<Req> q(new (std::nothrow) Req());
    if (!q) return SGN_ENOMEM;
    q->r = *req;
    q->fp = footprint(*req);
    if (q->fp > s->budget) return SGN_ENOMEM;
    q->batch = batchable(*req);
    // copy the inputs so the caller may reuse its arrays at once
    const sgn_grid& g = req->grid;
    const size_t N = npts(g), dN = (size_t)g.dim * N;
    const bool guess = req->kind == SGN_REQ_STEP_RK4 || req->opts.x0_is_guess;
    const bool solve = req->kind == SGN_REQ_SOLVE;
    q->in.resize(N + (solve ? 2 * dN : N) + (guess ? dN : 0));
    double* p = q->in.data();
    std::memcpy(p, req->h_eta, N * sizeof(double));
    q->r.h_eta = p;
    p += N;
    if (solve) {
        std::memcpy(p, req->h_grad_h, dN * sizeof(double));
        q->r.h_grad_h = p;
        p += dN;
        std::memcpy(p, req->h_rhs, dN * sizeof(double));
        q->r.h_rhs = p;
        p += dN;
    } else {
        std::memcpy(p, req->h_h, N * sizeof(double));
        q->r.h_h = p;
        p += N;
    }
    if (guess) {
        std::memcpy(p, req->h_u0, dN * sizeof(double));
        q->r.h_u0 = p;
    }
    std::lock_guard<std::mutex> lk(s->m);
    if (s->stopping) return SGN_EINVAL;
    q->id = s->next_id++;
    q->res.t_submit = s->now();
    *id = q->id;
    Req* raw = q.get();
    s->reqs.emplace(q->id, std::move(q));
    s->queued.push_back(raw);
    s->admit_locked();
    return SGN_OK;
}

sgn_status sgn_server_poll(sgn_server* s, uint64_t id, sgn_result* res) {
    if (!s || !res) return SGN_EINVAL;
    std::lock_guard<std::mutex> g(s->m);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return SGN_EINVAL;
    *res = it->second->res;
    if (res->done) s->reqs.erase(it);
    return SGN_OK;
}

sgn_status sgn_server_wait(sgn_server* s, uint64_t id, double timeout_s, sgn_result* res) {
    if (!s || !res) return SGN_EINVAL;
    std::unique_lock<std::mutex> g(s->m);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return SGN_EINVAL;
    Req* q = it->second.get();
    auto ready = [&] { return q->res.done != 0; };
    if (timeout_s < 0)
        s->cv_done.wait(g, ready);
    else
        s->cv_done.wait_for(g, std::chrono::duration<double>(timeout_s), ready);
    *res = q->res;
    if (res->done) s->reqs.erase(id);
    return SGN_OK;
}

sgn_status sgn_server_stats(sgn_server* s, int64_t* queued, int64_t* admitted, int64_t* completed,
                            size_t* bytes_in_use, size_t* bytes_held, size_t* budget) {
    if (!s) return SGN_EINVAL;
    const size_t pool_held = s->pool.held();
    std::lock_guard<std::mutex> g(s->m);
    if (queued) *queued = (int64_t)s->queued.size();
    if (admitted) *admitted = s->n_admitted;
    if (completed) *completed = s->n_completed;
    if (bytes_in_use) *bytes_in_use = s->lane_charged + s->batch_charged;
    if (bytes_held) *bytes_held = pool_held;
    if (budget) *budget = s->budget;
    return SGN_OK;
}

}  // extern "C"
