// libsgn request server: HBM-footprint admission, continuous batching of small
// 1D solves into sgn_batch_solve launches and of small 1D RK4 runs into
// sgn_batch_step_rk4 launches (a batching lane for each), and worker lanes (one
// context and HIP stream each) for 2D and large 1D solves and steps.  A client
// of the C ABI in sgn.h.
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

constexpr int BATCH_N_MAX = 8192;      // largest 1D size the batched solver and stepper take
enum { BATCH_SOLVES = 0, BATCH_STEPS = 1, BATCH_LANES = 2 };
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

// Batching lane of a request (BATCH_SOLVES, BATCH_STEPS), or -1: a worker lane.
int batch_lane_of(const sgn_request& r) {
    if (r.grid.dim != 1 || r.grid.nx > BATCH_N_MAX) return -1;
    return r.kind == SGN_REQ_SOLVE ? BATCH_SOLVES : BATCH_STEPS;
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

// Device bytes a batched group of the lane's kind needs for its fields and
// workspace: eta | h_x | rhs | u then the batched solver's workspace, or h |
// eta | u then the batched stepper's.
size_t batch_group_bytes(int lane, size_t tot, int n, const int32_t* sizes, int32_t precision) {
    if (lane == BATCH_SOLVES) return 4 * up(tot * sizeof(double)) + up(sgn_batch_workspace_bytes(n, sizes, precision));
    return 3 * up(tot * sizeof(double)) + up(sgn_batch_step_workspace_bytes(n, sizes, precision));
}

// Device bytes charged to an admitted request: its pooled block for a lane
// request; for a batched 1D solve or run its fields and its share of the
// batching lane's buffer (a group's buffer never exceeds the sum of its
// members' charges: every per-system term of the group's layout is in one
// member's charge, and each member's charge holds the fixed terms once).
size_t footprint(const sgn_request& r) {
    const int bl = batch_lane_of(r);
    if (bl >= 0) {
        const int32_t n = r.grid.nx;
        return batch_group_bytes(bl, (size_t)n, 1, &n, r.opts.precision);
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
    int batch = -1;           // batching lane, or -1: a worker lane
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

// A batching lane: its admitted requests, their charges, and its grow-only
// device buffer and pinned staging (held until the server is destroyed).
struct BatchLane {
    Lane lane;
    std::deque<Req*> q;
    size_t charged = 0;
    void* d_buf = nullptr;
    size_t d_bytes = 0;
    double* h_stage = nullptr;
    size_t h_doubles = 0;
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
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    uint64_t next_id = 1;
    // Device memory accounting (under m).  lane_charged: pooled blocks of the
    // admitted lane requests; a batching lane's `charged`: footprints of its
    // admitted requests.  A batching lane's grow-only buffer (d_bytes) stays held
    // after its group finishes, so the commitment is
    //   lane_charged + sum over batching lanes of max(charged, d_bytes) <= budget,
    // and every block the server holds (pool blocks, cached or in use, and the
    // batch buffers) is freed back to that bound before an allocation exceeds it.
    size_t lane_charged = 0;
    int64_t n_admitted = 0, n_completed = 0;
    int running = 0;                   // requests taken by a lane and not yet finished
    bool stopping = false;
    std::vector<Lane> lanes;
    BatchLane bl[BATCH_LANES];
    Pool pool;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    // Device bytes committed with `add` more charged to lane `to` (-1: worker lanes).
    size_t committed_locked(int to, size_t add) const {
        size_t c = lane_charged + (to < 0 ? add : 0);
        for (int b = 0; b < BATCH_LANES; ++b) c += std::max(bl[b].charged + (to == b ? add : 0), bl[b].d_bytes);
        return c;
    }

    // Admit queued requests in arrival order while they fit (caller holds m).
    void admit_locked() {
        bool any = false;
        while (!queued.empty()) {
            Req* q = queued.front();
            if (committed_locked(q->batch, q->fp) > budget) break;
            queued.pop_front();
            (q->batch >= 0 ? bl[q->batch].charged : lane_charged) += q->fp;
            q->res.t_admit = now();
            ++n_admitted;
            (q->batch >= 0 ? bl[q->batch].q : lane_q).push_back(q);
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
        (q->batch >= 0 ? bl[q->batch].charged : lane_charged) -= q->fp;
        ++n_completed;
        --running;
        admit_locked();
        cv_done.notify_all();
        cv_work.notify_all();
    }



    bool idle_locked() const {
        return queued.empty() && lane_q.empty() && bl[0].q.empty() && bl[1].q.empty() && running == 0;
    }

    void lane_loop(Lane* L);
    void batch_loop(int b);
    sgn_status run_batch(int b, const std::vector<Req*>& group, std::vector<Outcome>& oc,
                         std::vector<sgn_status>& qs);
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
           a.coeff_kind == b.coeff_kind && a.guess == b.guess;
}
}  // namespace

// One batched launch over `group` (all of lane b's kind, with the same options):
// inputs packed in pinned memory and copied in at once, the batched call, the
// outputs copied back at once.  Fills each member's outcome and status; returns
// a status that applies to the whole group (staging or device failures).
sgn_status sgn_server::run_batch(int b, const std::vector<Req*>& group, std::vector<Outcome>& oc,
                                 std::vector<sgn_status>& qs) {
    BatchLane& B = bl[b];
    const int n = (int)group.size();
    const bool steps = b == BATCH_STEPS;
    std::vector<int32_t> sizes(n), nsteps(n);
    std::vector<double> periods(n), dts(n);
    size_t tot = 0;
    for (int i = 0; i < n; ++i) {
        const sgn_request& r = group[i]->r;
        sizes[i] = r.grid.nx;
        periods[i] = r.grid.Lx;
        dts[i] = r.dt;
        nsteps[i] = r.nsteps;
        tot += (size_t)sizes[i];
    }
    const sgn_solve_opts opts = group[0]->r.opts;
    const size_t need = batch_group_bytes(b, tot, n, sizes.data(), opts.precision);
    if (need > B.d_bytes) {
        // the group's charges cover `need` (each member was charged its fields and
        // a one-system workspace, at least its share of the group's)
        void* nb = pool.regrow(B.d_buf, B.d_bytes, need);
        std::lock_guard<std::mutex> g(m);
        B.d_buf = nb;
        B.d_bytes = nb ? need : 0;
        if (!nb) return SGN_ENOMEM;
    }
    const int nf = steps ? 3 : 4;   // staged fields: h | eta | u, or eta | h_x | rhs | u
    if (nf * tot > B.h_doubles) {
        if (B.h_stage) (void)hipHostFree(B.h_stage);
        B.h_stage = nullptr;
        B.h_doubles = 0;
        if (hipHostMalloc((void**)&B.h_stage, nf * tot * sizeof(double), hipHostMallocDefault) != hipSuccess)
            return SGN_ENOMEM;
        B.h_doubles = nf * tot;
    }
    double* hs[4];
    for (int f = 0; f < nf; ++f) hs[f] = B.h_stage + f * tot;
    size_t o = 0;
    for (int i = 0; i < n; ++i) {
        const sgn_request& r = group[i]->r;
        const size_t ni = (size_t)sizes[i], nb = ni * sizeof(double);
        if (steps) {
            std::memcpy(hs[0] + o, r.h_h, nb);
            std::memcpy(hs[1] + o, r.h_eta, nb);
            std::memcpy(hs[2] + o, r.h_u0, nb);
        } else {
            std::memcpy(hs[0] + o, r.h_eta, nb);
            std::memcpy(hs[1] + o, r.h_grad_h, nb);
            std::memcpy(hs[2] + o, r.h_rhs, nb);
            if (opts.x0_is_guess)
                std::memcpy(hs[3] + o, r.h_u0, nb);
            else
                std::memset(hs[3] + o, 0, nb);
        }
        o += ni;
    }
    double* d = static_cast<double*>(B.d_buf);
    const size_t stride = up(tot * sizeof(double)) / sizeof(double);
    double* ds[4];
    for (int f = 0; f < nf; ++f) ds[f] = d + f * stride;
    void* dws = d + nf * stride;
    hipStream_t stream = B.lane.stream;
    bool ok = true;
    for (int f = 0; f < nf && ok; ++f)
        ok = hipMemcpyAsync(ds[f], hs[f], tot * sizeof(double), hipMemcpyHostToDevice, stream) == hipSuccess;
    if (!ok) return SGN_EDEVICE;
    sgn_status bst;
    std::vector<sgn_solve_info> info(steps ? 0 : n);
    std::vector<sgn_step_info> sinfo(steps ? n : 0);
    std::vector<sgn_status> sst(steps ? n : 0);
    if (steps)
        bst = sgn_batch_step_rk4(B.lane.ctx, n, sizes.data(), periods.data(), dts.data(), nsteps.data(), ds[0], ds[1],
                                 ds[2], &opts, sinfo.data(), sst.data(), dws);
    else
        bst = sgn_batch_solve(B.lane.ctx, n, sizes.data(), periods.data(), ds[0], ds[1], ds[2], ds[3], &opts,
                              info.data(), dws);
    if (bst != SGN_OK && bst != SGN_ENOCONV && bst != SGN_EDOMAIN) return bst;
    // outputs: u (solves); eta and u (runs)
    for (int f = steps ? 1 : 3; f < nf && ok; ++f)
        ok = hipMemcpyAsync(hs[f], ds[f], tot * sizeof(double), hipMemcpyDeviceToHost, stream) == hipSuccess;
    if (!ok || hipStreamSynchronize(stream) != hipSuccess) return SGN_EDEVICE;
    o = 0;
    for (int i = 0; i < n; ++i) {
        const sgn_request& r = group[i]->r;
        const size_t nb = (size_t)sizes[i] * sizeof(double);
        oc[i].batched = 1;
        oc[i].batch_size = n;
        if (steps) {
            oc[i].iters = sinfo[i].iters;
            oc[i].solves = sinfo[i].solves;
            qs[i] = sst[i];
            if (sst[i] != SGN_EDOMAIN) {
                std::memcpy(r.h_u_out, hs[2] + o, nb);
                if (r.h_eta_out) std::memcpy(r.h_eta_out, hs[1] + o, nb);
            }
        } else {
            oc[i].iters = info[i].iters;
            oc[i].solves = 1;
            oc[i].relres = info[i].relres;
            qs[i] = !(info[i].relres == info[i].relres) ? SGN_EDOMAIN : !info[i].converged ? SGN_ENOCONV : SGN_OK;
            std::memcpy(r.h_u_out, hs[3] + o, nb);
        }
        o += (size_t)sizes[i];
    }
    return SGN_OK;
}

void sgn_server::batch_loop(int b) {
    (void)hipSetDevice(device);
    BatchLane& B = bl[b];
    for (;;) {
        std::vector<Req*> group;
        {
            std::unique_lock<std::mutex> g(m);
            cv_work.wait(g, [&] { return !B.q.empty() || (stopping && idle_locked()); });
            if (B.q.empty()) return;
            // every admitted request of the lane with the options of the oldest one joins this launch
            const sgn_solve_opts key = B.q.front()->r.opts;
            for (auto it = B.q.begin(); it != B.q.end() && (int)group.size() < max_batch;) {
                if (same_batch_opts((*it)->r.opts, key)) {
                    group.push_back(*it);
                    it = B.q.erase(it);
                } else {
                    ++it;
                }
            }
            const double ts = now();
            for (Req* q : group) q->res.t_start = ts;
            running += (int)group.size();
        }
        std::vector<Outcome> oc(group.size());
        std::vector<sgn_status> qs(group.size(), SGN_OK);
        const sgn_status st = run_batch(b, group, oc, qs);
        for (size_t i = 0; i < group.size(); ++i) finish(group[i], st == SGN_OK ? qs[i] : st, oc[i]);
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
    bool ok = true;
    for (auto& B : s->bl) ok = ok && make_lane(B.lane);
    for (auto& L : s->lanes) ok = ok && make_lane(L);
    if (!ok) {
        auto drop = [](Lane& L) {
            if (L.ctx) sgn_destroy(L.ctx);
            if (L.stream) (void)hipStreamDestroy(L.stream);
        };
        for (auto& L : s->lanes) drop(L);
        for (auto& B : s->bl) drop(B.lane);
        return SGN_EDEVICE;
    }
    sgn_server* sp = s.get();
    for (auto& L : s->lanes) L.th = std::thread([sp, &L] { sp->lane_loop(&L); });
    for (int b = 0; b < BATCH_LANES; ++b) s->bl[b].lane.th = std::thread([sp, b] { sp->batch_loop(b); });
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
    for (auto& B : s->bl)
        if (B.lane.th.joinable()) B.lane.th.join();
    for (auto& L : s->lanes) {
        sgn_destroy(L.ctx);
        (void)hipStreamDestroy(L.stream);
    }
    for (auto& B : s->bl) {
        sgn_destroy(B.lane.ctx);
        (void)hipStreamDestroy(B.lane.stream);
        s->pool.free_extra(B.d_buf, B.d_bytes);
        if (B.h_stage) (void)hipHostFree(B.h_stage);
    }
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
    q->batch = batch_lane_of(*req);
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
    if (bytes_in_use) *bytes_in_use = s->lane_charged + s->bl[0].charged + s->bl[1].charged;
    if (bytes_held) *bytes_held = pool_held;
    if (budget) *budget = s->budget;
    return SGN_OK;
}

}  // extern "C"
