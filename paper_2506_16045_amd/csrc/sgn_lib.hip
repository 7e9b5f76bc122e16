// libsgn: C ABI entry points (include/sgn.h) and their host orchestration.
#include "sgn.h"
#include "sgn_kernels.h"
#include "sgn_batch.h"
#include "sgn_wall.h"
#include "sgn_wave.h"
#include <hip/hip_ext.h>

#include <algorithm>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

using namespace sgn;

// Stepper solves that keep an initial-guess history (sgn_guess).
enum { GUESS_RK2 = 0, GUESS_RK3, GUESS_RK4, GUESS_RK_FINAL, GUESS_AB, GUESS_SLOTS };

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct sgn_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    cpx<double>* tw64 = nullptr;
    cpx<float>* tw32 = nullptr;
    SolveScal* hscal = nullptr;   // pinned readback of solver scalars
    int* hflag = nullptr;         // pinned readback of the done flag
    std::string err;
    // opt-in kernel timing: HIP events around every launch of each kernel family
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_next = 0;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_marks;
    std::vector<std::pair<int, float>> prof_last;   // the last profile's launches (kind, ms)
    // PCG iteration chunks captured as HIP graphs on a private stream and replayed
    // on `stream`; keyed by everything the captured launches depend on
    struct GraphEntry {
        std::vector<const void*> key;
        int chunk;
        hipGraphExec_t exec;  // null: seen once (ran eagerly), capture on the next use
    };
    hipStream_t cap_stream = nullptr;
    std::vector<GraphEntry> graphs;
    bool use_graphs = false;
    // iterations of the previous solve per precision (FP64 / FP32 loop) and
    // stepper slot (last entry: solves outside a stepper)
    int last_iters[2][GUESS_SLOTS + 1] = {};
    int* stage_last = nullptr;    // the running stepper solve's counters (state-owned), if any
    bool stage = false;           // solving inside a stepper: skip the final scalar readback
    bool wall_twin = false;       // solving on the periodic twin of a wall grid
    bool wall_native = false;     // stepping a 2D wall grid on its own points (fields in transform order)
    int cus = 256;                // compute units of the device
    void* hbatch = nullptr;       // pinned staging of batch item tables and results
    size_t hbatch_bytes = 0;
    int slot = GUESS_SLOTS;       // stepper slot of the running solve
    // extrapolated guess of a stepper solve on the FP64 row/column path: the solve
    // reads u (the base) + (gx_c1 gx_a + gx_c2 gx_b) while transforming it, and
    // writes its result's offset from the base to gx_off while storing it
    const double* gx_a = nullptr;
    const double* gx_b = nullptr;
    double gx_c1 = 0.0, gx_c2 = 0.0;
    double* gx_off = nullptr;
    // readbacks in the solve loops wait by polling this event: a blocking stream
    // synchronisation wakes the host tens of microseconds after the GPU is done,
    // and the GPU idles until the next launches arrive
    hipEvent_t ev_sync = nullptr;
    // the loop flags are published by a one-thread kernel straight into this
    // host-coherent pinned buffer (hpub; dpub its device address), tagged with a
    // sequence number; the host polls it (no device-to-host copy in the stream)
    int* hpub = nullptr;
    int* dpub = nullptr;
    int pub_seq = 0;
    // device address of this device's copy of the allocation-free solve's scratch
    void* scratch = nullptr;
};

// Workspace of sgn_krylov_solve_noalloc: a static device array, so that the call
// allocates nothing.  Every device the library runs on holds its own copy of it
// (at its own address) until the process ends.  In host code the array's name is
// only a host-side stand-in: host code uses the address hipGetSymbolAddress
// returns for the current device, looked up once per device at context creation.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)48 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Address of `scratch` on `device` (which must be current); null on failure.
void* scratch_address(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[device] = ptr;
    }
    return g_scratch_ptr[device];
}

}  // namespace

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

sgn_status fail(sgn_ctx* ctx, sgn_status s, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return s;
}

#define HIPCHK(ctx, call)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail((ctx), SGN_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define CHECK_LAUNCH(ctx) HIPCHK(ctx, hipGetLastError())

inline bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
inline int next_pow2(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures, which is how sgn_workspace_bytes is computed.
struct Carve {
    char* base;
    size_t off = 0;
    explicit Carve(void* b) : base(static_cast<char*>(b)) {}
    template <class X>
    X* take(size_t count) {
        off = align_up(off, 256);
        X* p = base ? reinterpret_cast<X*>(base + off) : nullptr;
        off += count * sizeof(X);
        return p;
    }
};

struct Dims {
    int D, nx, ny;
    size_t N;   // physical points
    size_t NS;  // spectral modes (nx/2+1) * ny
    double tpx, tpy, inv_n;
    double Lx;
    int bc = SGN_BC_PERIODIC;
    double Ly = 1.0;
};

sgn_status check_grid(sgn_ctx* ctx, const sgn_grid* g, Dims* d) {
    if (!g) return fail(ctx, SGN_EINVAL, "grid is null");
    if (g->dim != 1 && g->dim != 2) return fail(ctx, SGN_EINVAL, "grid dim must be 1 or 2");
    const int ny = g->dim == 1 ? 1 : g->ny;
    if (g->bc != SGN_BC_PERIODIC && g->bc != SGN_BC_WALLS) return fail(ctx, SGN_EINVAL, "bad boundary condition");
    if (!is_pow2(g->nx) || g->nx < 2 || !is_pow2(ny))
        return fail(ctx, SGN_EUNSUPPORTED, "grid sizes must be powers of two (nx >= 2)");
    // a grid between walls runs on its periodic twin, twice as long per axis
    const int w = g->bc == SGN_BC_WALLS ? 2 : 1;
    if (g->dim == 1 && g->nx * w > 16384) return fail(ctx, SGN_EUNSUPPORTED, "1D nx above 16384 (8192 with walls)");
    if (g->dim == 2 && (g->nx * w > 4096 || ny * w > 1024 || ny < 2))
        return fail(ctx, SGN_EUNSUPPORTED, "2D sizes: nx in [2, 4096], ny in [2, 1024] (half with walls)");
    if (!(g->Lx > 0.0) || (g->dim == 2 && !(g->Ly > 0.0)))
        return fail(ctx, SGN_EINVAL, "domain lengths must be positive");
    d->D = g->dim;
    d->nx = g->nx;
    d->ny = ny;
    d->N = (size_t)g->nx * ny;
    d->NS = (size_t)(g->nx / 2 + 1) * ny;
    d->tpx = kTwoPi / g->Lx;
    d->tpy = g->dim == 2 ? kTwoPi / g->Ly : 0.0;
    d->inv_n = 1.0 / (double)d->N;
    d->Lx = g->Lx;
    d->Ly = g->dim == 2 ? g->Ly : 1.0;
    d->bc = g->bc;
    return SGN_OK;
}

// The periodic grid of twice the length per axis on which a grid between walls runs.
Dims twin_dims(const Dims& d) {
    Dims t = d;
    t.bc = SGN_BC_PERIODIC;
    t.nx = 2 * d.nx;
    t.ny = d.D == 2 ? 2 * d.ny : 1;
    t.N = (size_t)t.nx * t.ny;
    t.NS = (size_t)(t.nx / 2 + 1) * t.ny;
    t.Lx = 2 * d.Lx;
    t.Ly = d.D == 2 ? 2 * d.Ly : 1.0;
    t.tpx = kTwoPi / t.Lx;
    t.tpy = d.D == 2 ? kTwoPi / t.Ly : 0.0;
    t.inv_n = 1.0 / (double)t.N;
    return t;
}

sgn_status require_periodic(sgn_ctx* ctx, const Dims& d) {
    if (d.bc != SGN_BC_PERIODIC)
        return fail(ctx, SGN_EUNSUPPORTED, "grids between walls are taken by the constraint solve calls only");
    return SGN_OK;
}

// ---------------------------------------------------------------------------
// Launch geometry
// ---------------------------------------------------------------------------
struct RowLaunch {
    RowGeom g;
    int threads;
    size_t lds;
    int epc;
};
// wide: on 2D rows of 64 to 1024 points, two entries per thread and up to
// 512-thread blocks, so that more waves are resident to hide the transposed
// accesses' latency (the grid has only ny / R blocks); taken by the Krylov row
// pass and the plain row transforms.
template <typename T>
RowLaunch row_launch(int nx, int ny, bool wide = false) {
    RowLaunch L;
    const int M = nx / 2;
    const bool two = wide && ny > 1 && M >= 32 && M <= 512;
    L.epc = two ? 2 : (M > 4096) ? 8 : 4;
    RowGeom& g = L.g;
    g.nx = nx;
    g.ny = ny;
    g.M = M;
    g.TPR = M / L.epc > 0 ? M / L.epc : 1;
    int R = (two ? 512 : 256) / g.TPR;
    if (R < 1) R = 1;
    const int np = next_pow2(ny);
    if (R > np) R = np;
    // keep a block per compute unit: fewer rows per block (down to 64 threads)
    // while the grid has fewer than 256 R rows (Krylov row pass: 512^2 2 rows
    // per block, 16.8 -> 13.6 us; 256^2 one row of 64 threads, 19.0 -> 10.2 us;
    // 128^2 two rows, 17.4 -> 9.5 us)
    if (two)
        while (R > 1 && ny / R < 256 && (R / 2) * g.TPR >= 64) R >>= 1;
    g.R = R;
    g.nblocks = (ny + R - 1) / R;
    L.threads = R * g.TPR;
    L.lds = (size_t)R * (M + 1) * sizeof(cpx<T>);
    return L;
}

struct ColLaunch {
    ColGeom g;
    int threads;
    size_t lds;
    int epc;
};
// epc: column entries per thread (4; 8 for the columns of 2048 on a padded grid)
template <typename T>
ColLaunch col_launch(int nx, int ny, int epc = 4) {
    ColLaunch L;
    ColGeom& g = L.g;
    g.nx = nx;
    g.ny = ny;
    g.nxh = nx / 2 + 1;
    g.TPC = ny / epc > 0 ? ny / epc : 1;
    g.Cb = 256 / g.TPC > 0 ? 256 / g.TPC : 1;
    g.nblocks = (g.nxh + g.Cb - 1) / g.Cb;
    L.threads = g.Cb * g.TPC;
    L.lds = (size_t)g.Cb * ny * sizeof(cpx<T>);
    if (L.lds < 16) L.lds = 16;
    L.epc = epc;
    return L;
}

// Column geometry of the Krylov passes (the PcgLaunch of every solve): 2D
// columns of up to 512 points take two entries per thread (256^2: C1 10.9 ->
// 8.5 us, C2 10.5 -> 8.8 us; 512^2: C1 12.7 -> 10.2 us), longer ones four.
template <typename T>
ColLaunch pcg_col_launch(const Dims& d) { return col_launch<T>(d.nx, d.ny, (d.D == 2 && d.ny <= 512) ? 2 : 4); }

// Column passes of a wall solve (columns of up to 512): two entries per thread,
// 256-thread blocks as every column pass (the partial sums are reduced over 256
// lanes); 512^2: one column per block, C1 13.8 -> 11.4 us, C2 14.0 -> 11.5 us.
ColLaunch wall_col_launch(int nx, int ny) { return col_launch<double>(nx, ny, 2); }

// Column entries per thread: columns up to 1024 use 4 (the grids the solvers
// take); the padded grid of the de-aliased right-hand side has columns of 2048.
inline int col_epc(int ny) { return ny > 1024 ? 8 : 4; }

// LDS bytes of a row / column kernel transforming NF fields at a time (data,
// then the staged twiddle table when the transform length allows it).
inline int twl_entries(int M) { return (M <= TWL_MAX && M >= 4) ? M : 0; }
template <typename T>
size_t row_lds_bytes(const RowGeom& g, int NF) {
    return (size_t)(row_lds_data(g, NF) + twl_entries(g.M)) * sizeof(cpx<T>);
}
template <typename T>
size_t col_lds_bytes(const ColGeom& g, int NF) {
    return (size_t)(col_lds_data(g, NF) + twl_entries(g.ny)) * sizeof(cpx<T>);
}
constexpr size_t LDS_MULTI_MAX = 96 * 1024;  // above this, row kernels transform fields one by one

inline int flat_blocks(size_t n, int per = 256, int cap = 1024) {
    size_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    if (b > (size_t)cap) b = cap;
    return (int)b;
}


template <typename K>
hipError_t allow_lds(K kernel, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename T> const cpx<T>* twiddles(sgn_ctx* ctx);
template <> const cpx<double>* twiddles<double>(sgn_ctx* ctx) { return ctx->tw64; }
template <> const cpx<float>* twiddles<float>(sgn_ctx* ctx) { return ctx->tw32; }

// ---- kernel timing ---------------------------------------------------------
hipEvent_t prof_event(sgn_ctx* ctx) {
    if (ctx->ev_next == ctx->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ctx->ev_pool.push_back(e);
    }
    return ctx->ev_pool[ctx->ev_next++];
}
// Scoped marker: records an event pair around the launches in its scope.  With
// in_launch, the pair (a, b) is instead handed to the scope's single kernel
// launch (hipExtLaunchKernelGGL records it at the kernel's own start and end, so
// the time excludes the marker packets).
struct ProfScope {
    sgn_ctx* ctx;
    int id;
    hipEvent_t a = nullptr, b = nullptr;
    bool in_launch = false;
    ProfScope(sgn_ctx* c, int kid, bool in_launch_ = false) : ctx(c), id(kid) {
        if (!ctx->prof_on || (a = prof_event(ctx)) == nullptr) return;
        if (in_launch_) {
            b = prof_event(ctx);
            if (!b) {
                a = nullptr;
                return;
            }
            in_launch = true;
        } else {
            (void)hipEventRecord(a, ctx->stream);
        }
    }
    ~ProfScope() {
        if (!a) return;
        if (!in_launch) {
            b = prof_event(ctx);
            if (!b) return;
            (void)hipEventRecord(b, ctx->stream);
        }
        ctx->prof_marks.push_back({id, {a, b}});
    }
};

// ---- generic passes --------------------------------------------------------

// Row passes on 2D rows of 1024 points run as wave-private transforms
// (sgn_wave.h); SGN_WAVE_ROWS=0 selects the block-wide passes.
inline bool wave_rows_enabled() {
    static const bool on = [] {
        const char* e = getenv("SGN_WAVE_ROWS");
        return !(e && e[0] == '0');
    }();
    return on;
}
inline bool wave_rows(const Dims& d) {
    return d.D == 2 && d.nx == WROW_NX && d.ny % WROW_WPB == 0 && wave_rows_enabled();
}

// cmb (optional): fields from cmb->first on are read as src + (c1 a + c2 b)
// (at most MAXF fields in that case).
template <typename T, typename Tin>
sgn_status rows_fwd(sgn_ctx* ctx, const Dims& d, std::vector<const Tin*> src, std::vector<cpx<T>*> dst,
                    T scale = (T)1, const RowCombo<Tin>* cmb = nullptr) {
    ProfScope ps(ctx, SGN_KERNEL_ROWS);
    RowLaunch L = row_launch<T>(d.nx, d.ny, true);
    RowCombo<Tin> none{};
    none.first = -1;
    if (cmb && src.size() > (size_t)MAXF) return fail(ctx, SGN_EINVAL, "rows_fwd: combined sources exceed one pass");
    const RowCombo<Tin>& cm = cmb ? *cmb : none;
    for (size_t f0 = 0; f0 < src.size(); f0 += MAXF) {
        PtrList<const Tin, MAXF> s{};
        PtrList<cpx<T>, MAXF> t{};
        s.n = t.n = (int)std::min<size_t>(MAXF, src.size() - f0);
        for (int i = 0; i < s.n; ++i) {
            s.p[i] = src[f0 + i];
            t.p[i] = dst[f0 + i];
        }
        if (wave_rows(d)) {
            hipLaunchKernelGGL((k_rows_fwd_w<T, Tin>), dim3(s.n * d.ny / WROW_WPB), dim3(64 * WROW_WPB), 0,
                               ctx->stream, d.ny, s, t, twiddles<T>(ctx), scale, cm);
            CHECK_LAUNCH(ctx);
            continue;
        }
        const bool multi = row_lds_bytes<T>(L.g, 3) <= LDS_MULTI_MAX;
        const size_t lds = row_lds_bytes<T>(L.g, multi ? 3 : 1);
        auto launch = [&](auto k) -> sgn_status {
            HIPCHK(ctx, allow_lds(k, lds));
            hipLaunchKernelGGL(k, dim3(L.g.nblocks), dim3(L.threads), lds, ctx->stream, L.g, s, t, twiddles<T>(ctx),
                               scale, cm);
            return SGN_OK;
        };
        sgn_status st;
        if (L.epc == 2)
            st = multi ? launch(k_rows_fwd<T, Tin, 2, 3, 512>) : launch(k_rows_fwd<T, Tin, 2, 1, 512>);
        else if (L.epc == 4)
            st = L.threads <= 256
                     ? (multi ? launch(k_rows_fwd<T, Tin, 4, 3, 256>) : launch(k_rows_fwd<T, Tin, 4, 1, 256>))
                     : (multi ? launch(k_rows_fwd<T, Tin, 4, 3>) : launch(k_rows_fwd<T, Tin, 4, 1>));
        else
            st = multi ? launch(k_rows_fwd<T, Tin, 8, 3>) : launch(k_rows_fwd<T, Tin, 8, 1>);
        if (st != SGN_OK) return st;
        CHECK_LAUNCH(ctx);
    }
    return SGN_OK;
}

// offs (optional, one per field): also write new - old value of each dst field
// (added to offs instead with offs_acc).
template <typename T, typename Tout>
sgn_status rows_inv(sgn_ctx* ctx, const Dims& d, std::vector<const cpx<T>*> src, std::vector<Tout*> dst,
                    T scale = (T)1, T acc = (T)0, const std::vector<Tout*>* offs = nullptr, bool offs_acc = false) {
    ProfScope ps(ctx, SGN_KERNEL_ROWS);
    RowLaunch L = row_launch<T>(d.nx, d.ny, true);
    if (offs && offs->size() != src.size()) return fail(ctx, SGN_EINVAL, "rows_inv: offsets per field");
    for (size_t f0 = 0; f0 < src.size(); f0 += MAXF) {
        PtrList<const cpx<T>, MAXF> s{};
        PtrList<Tout, MAXF> t{};
        PtrList<Tout, MAXF> of{};
        s.n = t.n = (int)std::min<size_t>(MAXF, src.size() - f0);
        of.n = offs ? s.n : 0;
        for (int i = 0; i < s.n; ++i) {
            s.p[i] = src[f0 + i];
            t.p[i] = dst[f0 + i];
            if (offs) of.p[i] = (*offs)[f0 + i];
        }
        if (wave_rows(d)) {
            hipLaunchKernelGGL((k_rows_inv_w<T, Tout>), dim3(s.n * d.ny / WROW_WPB), dim3(64 * WROW_WPB), 0,
                               ctx->stream, d.ny, s, t, twiddles<T>(ctx), scale, acc, of, offs_acc ? 1 : 0);
            CHECK_LAUNCH(ctx);
            continue;
        }
        const bool multi = row_lds_bytes<T>(L.g, 3) <= LDS_MULTI_MAX;
        const size_t lds = row_lds_bytes<T>(L.g, multi ? 3 : 1);
        auto launch = [&](auto k) -> sgn_status {
            HIPCHK(ctx, allow_lds(k, lds));
            hipLaunchKernelGGL(k, dim3(L.g.nblocks), dim3(L.threads), lds, ctx->stream, L.g, s, t, twiddles<T>(ctx),
                               scale, acc, of, offs_acc ? 1 : 0);
            return SGN_OK;
        };
        sgn_status st;
        if (L.epc == 2)
            st = multi ? launch(k_rows_inv<T, Tout, 2, 3, 512>) : launch(k_rows_inv<T, Tout, 2, 1, 512>);
        else if (L.epc == 4)
            st = L.threads <= 256
                     ? (multi ? launch(k_rows_inv<T, Tout, 4, 3, 256>) : launch(k_rows_inv<T, Tout, 4, 1, 256>))
                     : (multi ? launch(k_rows_inv<T, Tout, 4, 3>) : launch(k_rows_inv<T, Tout, 4, 1>));
        else
            st = multi ? launch(k_rows_inv<T, Tout, 8, 3>) : launch(k_rows_inv<T, Tout, 8, 1>);
        if (st != SGN_OK) return st;
        CHECK_LAUNCH(ctx);
    }
    return SGN_OK;
}

template <typename T, int NI>
sgn_status cols_lin_n(sgn_ctx* ctx, const Dims& d, const std::vector<const cpx<T>*>& src,
                      const std::vector<cpx<T>*>& dst, const LinCodes& lc, T scale) {
    ProfScope ps(ctx, SGN_KERNEL_COLS);
    ColLaunch L = col_launch<T>(d.nx, d.ny);
    PtrList<const cpx<T>, MAXF> s{};
    PtrList<cpx<T>, MAXF> t{};
    s.n = NI;
    t.n = lc.no;
    for (int i = 0; i < NI; ++i) s.p[i] = src[i];
    for (int i = 0; i < lc.no; ++i) t.p[i] = dst[i];
    // one field at a time: lockstep groups cost more registers than they save barriers
    auto k = k_cols_lin<T, 4, NI, 1>;
    const size_t lds = col_lds_bytes<T>(L.g, 1);
    HIPCHK(ctx, allow_lds(k, lds));
    hipLaunchKernelGGL(k, dim3(L.g.nblocks), dim3(L.threads), lds, ctx->stream, L.g, s, t, lc, twiddles<T>(ctx),
                       (T)d.tpx, (T)d.tpy, scale);
    CHECK_LAUNCH(ctx);
    return SGN_OK;
}

template <typename T>
sgn_status cols_lin(sgn_ctx* ctx, const Dims& d, const std::vector<const cpx<T>*>& src,
                    const std::vector<cpx<T>*>& dst, const std::vector<std::vector<int>>& codes, T scale) {
    LinCodes lc{};
    lc.no = (int)codes.size();
    if (lc.no > LIN_MAXO || (int)dst.size() != lc.no) return fail(ctx, SGN_EINVAL, "cols_lin: bad outputs");
    for (int o = 0; o < lc.no; ++o)
        for (size_t i = 0; i < codes[o].size(); ++i) lc.code[o][i] = codes[o][i];
    switch (src.size()) {
        case 1: return cols_lin_n<T, 1>(ctx, d, src, dst, lc, scale);
        case 2: return cols_lin_n<T, 2>(ctx, d, src, dst, lc, scale);
        case 3: return cols_lin_n<T, 3>(ctx, d, src, dst, lc, scale);
        case 4: return cols_lin_n<T, 4>(ctx, d, src, dst, lc, scale);
        case 5: return cols_lin_n<T, 5>(ctx, d, src, dst, lc, scale);
        default: return fail(ctx, SGN_EINVAL, "cols_lin: bad input count");
    }
}

// Independent linear column operators side by side in one launch (k_cols_lin_jobs).
struct LinJobSpec {
    std::vector<const cpx<double>*> src;
    std::vector<cpx<double>*> dst;
    std::vector<std::vector<int>> codes;
    std::vector<int> kin, kout;   // wall jobs: series kinds of the inputs and outputs
};
sgn_status cols_lin_jobs(sgn_ctx* ctx, const Dims& d, const std::vector<LinJobSpec>& spec, double scale,
                         int kind = SGN_KERNEL_COLS, bool wall = false) {
    ProfScope ps(ctx, kind);
    if (spec.empty() || spec.size() > (size_t)LINJ_MAXJ) return fail(ctx, SGN_EINVAL, "cols_lin_jobs: job count");
    LinJobs<double> J{};
    J.n = (int)spec.size();
    for (int k = 0; k < J.n; ++k) {
        const LinJobSpec& s = spec[k];
        LinJob<double>& j = J.j[k];
        if (s.src.empty() || s.src.size() > (size_t)LINJ_MAXI || s.dst.empty() || s.dst.size() > (size_t)LINJ_MAXO ||
            s.codes.size() != s.dst.size())
            return fail(ctx, SGN_EINVAL, "cols_lin_jobs: bad job");
        j.ni = (int)s.src.size();
        j.no = (int)s.dst.size();
        for (int i = 0; i < j.ni; ++i) j.src[i] = s.src[i];
        for (int o = 0; o < j.no; ++o) {
            j.dst[o] = s.dst[o];
            if (s.codes[o].size() > (size_t)j.ni) return fail(ctx, SGN_EINVAL, "cols_lin_jobs: bad codes");
            for (size_t i = 0; i < s.codes[o].size(); ++i) j.code[o][i] = s.codes[o][i];
        }
    }
    int maxi = 0;
    for (int k = 0; k < J.n; ++k) maxi = std::max(maxi, J.j[k].ni);
    if (wall) {
        // a 2D wall grid on its own points: the slot coefficients of each job's kinds
        for (int k = 0; k < J.n; ++k) {
            const LinJobSpec& sp = spec[k];
            LinJob<double>& j = J.j[k];
            if (j.ni > 3 || j.no > 3 || sp.kin.size() != (size_t)j.ni || sp.kout.size() != (size_t)j.no)
                return fail(ctx, SGN_EINVAL, "cols_lin_jobs: a wall job takes up to three inputs and outputs, kinds given");
            for (int i = 0; i < j.ni; ++i) j.kin[i] = sp.kin[i];
            for (int o = 0; o < j.no; ++o) j.kout[o] = sp.kout[o];
        }
        const ColLaunch L = wall_col_launch(d.nx, d.ny);
        const size_t lds = col_lds_bytes<double>(L.g, 3);
        auto k = L.epc == 2 ? k_wall_cols_jobs<double, 2> : k_wall_cols_jobs<double, 4>;
        HIPCHK(ctx, allow_lds(k, lds));
        hipLaunchKernelGGL(k, dim3(L.g.nblocks * J.n), dim3(L.threads), lds, ctx->stream, L.g, J, ctx->tw64, d.tpx,
                           d.tpy, scale);
        CHECK_LAUNCH(ctx);
        return SGN_OK;
    }
    const int epc = col_epc(d.ny);
    ColLaunch L = col_launch<double>(d.nx, d.ny, epc);
    // the inputs, then the outputs, are transformed up to three at a time in lockstep
    // (one at a time for columns of 2048)
    const size_t lds = col_lds_bytes<double>(L.g, epc == 8 ? 1 : 3);
    auto launch = [&](auto k) -> sgn_status {
        HIPCHK(ctx, allow_lds(k, lds));
        hipLaunchKernelGGL(k, dim3(L.g.nblocks * J.n), dim3(L.threads), lds, ctx->stream, L.g, J, ctx->tw64, d.tpx,
                           d.tpy, scale);
        CHECK_LAUNCH(ctx);
        return SGN_OK;
    };
    // registers for the inputs are sized by the widest job
    if (epc == 8) {
        if (maxi > 3) return fail(ctx, SGN_EINVAL, "cols_lin_jobs: columns of 2048 take at most 3 inputs");
        return launch(k_cols_lin_jobs<double, 8, 3, 1>);
    }
    return maxi <= 3 ? launch(k_cols_lin_jobs<double, 4, 3, 3>) : launch(k_cols_lin_jobs<double, 4, 4, 3>);
}

// ---------------------------------------------------------------------------
// Coefficients (device) -> SolveScal
// ---------------------------------------------------------------------------
// Initial values of a solve's scalars (see k_init_scal).
struct ScalInit {
    double tol;
    int max_iter;
    double inv_n;
    int init_bb;
};

// With eta32 / gh32 set, the same pass also writes FP32 copies of eta and grad h;
// with init set, the finishing kernel also initialises the solve's scalars.
sgn_status launch_coeffs(sgn_ctx* ctx, const Dims& d, const double* eta, const double* gh, int flat,
                         int kind, SolveScal* sc, double* partials, float* eta32 = nullptr,
                         float* gh32 = nullptr, const ScalInit* init = nullptr) {
    const int nb = flat_blocks(d.N, 256, 1024);
    if (d.D == 1)
        hipLaunchKernelGGL(k_coeffs<1>, dim3(nb), dim3(256), 0, ctx->stream, d.N, eta, gh, partials, eta32, gh32);
    else
        hipLaunchKernelGGL(k_coeffs<2>, dim3(nb), dim3(256), 0, ctx->stream, d.N, eta, gh, partials, eta32, gh32);
    hipLaunchKernelGGL(k_coeffs_finish, dim3(1), dim3(256), 0, ctx->stream, sc, (const double*)partials, nb, flat,
                       kind, init ? 1 : 0, init ? init->tol : 0.0, init ? init->max_iter : 0,
                       init ? init->inv_n : 0.0, init ? init->init_bb : 0);
    CHECK_LAUNCH(ctx);
    return SGN_OK;
}

// ---------------------------------------------------------------------------
// Workspace layouts
// ---------------------------------------------------------------------------
struct Common {
    SolveScal* sc;        // [4]: 0 = FP64 solve / misc, 1 = FP32 inner solve
    double* partials;     // PART_TOTAL doubles (see sgn_kernels.h)
};
Common carve_common(Carve& cv) {
    Common c;
    c.sc = cv.take<SolveScal>(4);
    c.partials = cv.take<double>((size_t)PART_TOTAL);
    return c;
}

template <typename T>
struct PcgBufs {
    cpx<T>*H, *xh, *rh, *ph, *qh, *bh;
};
template <typename T>
PcgBufs<T> carve_pcg(Carve& cv, const Dims& d, bool keep_b) {
    PcgBufs<T> b;
    b.H = cv.take<cpx<T>>((size_t)(d.D + 1) * d.NS);
    b.xh = cv.take<cpx<T>>((size_t)d.D * d.NS);
    b.rh = cv.take<cpx<T>>((size_t)d.D * d.NS);
    b.ph = cv.take<cpx<T>>((size_t)d.D * d.NS);
    b.qh = cv.take<cpx<T>>((size_t)d.D * d.NS);
    b.bh = keep_b ? cv.take<cpx<T>>((size_t)d.D * d.NS) : nullptr;
    return b;
}

struct RhsBufs {
    cpx<double>* H;     // spectral temporaries
    int nH;
};
RhsBufs carve_rhs(Carve& cv, const Dims& d) {
    RhsBufs b;
    const int D = d.D;
    b.nH = (2 * D + 1) + 2 + (2 * D + 2) + (2 * D);
    b.H = cv.take<cpx<double>>((size_t)b.nH * d.NS);
    return b;
}

size_t workspace_bytes(const Dims& d, int precision) {
    size_t best = 0;
    {   // FP64 PCG
        Carve cv(nullptr);
        carve_common(cv);
        carve_pcg<double>(cv, d, true);
        best = std::max(best, cv.off);
    }
    {   // mixed: FP64 outer + FP32 inner + FP32 copies of eta and grad h
        Carve cv(nullptr);
        carve_common(cv);
        carve_pcg<double>(cv, d, true);
        carve_pcg<float>(cv, d, false);
        cv.take<float>((size_t)(1 + d.D) * d.N);
        if (precision == SGN_MIXED) best = std::max(best, cv.off);
    }
    {   // right-hand side
        Carve cv(nullptr);
        carve_common(cv);
        carve_rhs(cv, d);
        best = std::max(best, cv.off);
    }
    if (d.D == 1 && d.nx <= BATCH_NMAX) {   // one-workgroup 1D solve, right-hand side and RK4 run
        best = std::max(best, (size_t)512 + (size_t)batch_item_doubles(d.nx, BATCH_MIXED) * sizeof(double));
        best = std::max(best, (size_t)1024 + (size_t)step_scratch_doubles(d.nx, BATCH_MIXED) * sizeof(double));
        Carve cv(nullptr);
        carve_common(cv);
        cv.take<cpx<double>>((size_t)5 * (d.nx / 2 + 1));
        cv.take<double>((size_t)5 * d.nx);
        best = std::max(best, cv.off);
    }
    return best + 256;
}

// ---------------------------------------------------------------------------
// Krylov solve (PCG), templated on the working precision of the iteration.
// The iteration runs on S-layout state; see sgn_kernels.h.
// ---------------------------------------------------------------------------
template <typename T, int D>
struct PcgLaunch {
    sgn_ctx* ctx;
    Dims d;
    RowLaunch rl;
    ColLaunch cl;
    PcgBufs<T> b;
    SolveScal* sc;
    double* partials;
    const T* eta;
    const T* gh;
    bool wall = false;  // the grid is the periodic twin of a wall grid (residuals projected)
    bool native = false;  // a 2D grid between walls on its own points (the wall column passes)
};

// mode C1_ACCUM (T = double only): x_hat += dx (FP32) and G is applied to the
// corrected x_hat.
template <typename T, int D>
sgn_status pcg_c1(PcgLaunch<T, D>& P, int mode, const cpx<T>* xsrc, const cpx<float>* dx = nullptr) {
    ProfScope ps(P.ctx, SGN_KERNEL_PCG_C1 + (sizeof(T) == 4 ? 6 : 0), true);
    auto& L = P.cl;
    const size_t lds = col_lds_bytes<T>(L.g, D + 1);
    if (P.native) {
        if (D != 2 || mode != C1_UPDATE) return fail(P.ctx, SGN_EINVAL, "pcg_c1: wall column pass takes updates only");
        auto k = L.epc == 2 ? k_wall_c1<T, 2> : k_wall_c1<T, 4>;
        HIPCHK(P.ctx, allow_lds(k, lds));
        hipExtLaunchKernelGGL(k, dim3(L.g.nblocks), dim3(L.threads), lds, P.ctx->stream, ps.a, ps.b, 0, L.g,
                              twiddles<T>(P.ctx), P.sc, (const double*)P.partials, P.cl.g.nblocks,
                              (const cpx<T>*)P.b.rh, P.b.ph, P.b.H, P.d.NS, (T)P.d.tpx, (T)P.d.tpy);
        CHECK_LAUNCH(P.ctx);
        return SGN_OK;
    }
    if (mode == C1_UPDATE && col_wave(P)) {
        hipExtLaunchKernelGGL(k_pcg_c1w<T>, dim3(L.g.nblocks), dim3(WCOL_THREADS), 0, P.ctx->stream, ps.a, ps.b, 0,
                              P.d.nx, twiddles<T>(P.ctx), P.sc, (const double*)P.partials, P.cl.g.nblocks,
                              (const cpx<T>*)P.b.rh, P.b.ph, P.b.H, P.d.NS, (T)P.d.tpx, (T)P.d.tpy);
        CHECK_LAUNCH(P.ctx);
        return SGN_OK;
    }
    auto launch = [&](auto k, cpx<T>* ph) -> sgn_status {
        HIPCHK(P.ctx, allow_lds(k, lds));
        hipExtLaunchKernelGGL(k, dim3(L.g.nblocks), dim3(L.threads), lds, P.ctx->stream, ps.a, ps.b, 0, L.g,
                              twiddles<T>(P.ctx), P.sc, (const double*)P.partials, P.cl.g.nblocks, P.b.rh, ph, xsrc,
                              P.b.H, P.d.NS, (T)P.d.tpx, (T)P.d.tpy, dx);
        return SGN_OK;
    };
    sgn_status s;
    const bool e2 = L.epc == 2;
    if (mode == C1_COPY)
        s = launch(e2 ? k_pcg_c1<T, 2, D, C1_COPY> : k_pcg_c1<T, 4, D, C1_COPY>, P.b.ph);
    else if (mode == C1_ACCUM) {
        if (sizeof(T) != 8 || !dx) return fail(P.ctx, SGN_EINVAL, "pcg_c1: accumulate needs an FP64 solve");
        s = launch(e2 ? k_pcg_c1<T, 2, D, C1_ACCUM> : k_pcg_c1<T, 4, D, C1_ACCUM>, P.b.xh);
    } else
        s = launch(e2 ? k_pcg_c1<T, 2, D, C1_UPDATE> : k_pcg_c1<T, 4, D, C1_UPDATE>, P.b.ph);
    if (s != SGN_OK) return s;
    CHECK_LAUNCH(P.ctx);
    return SGN_OK;
}

// Rows per wave of the wave-private Krylov row pass: two in FP32 (16-byte
// accesses to the transposed layout), one in FP64 (two would not fit the
// registers of three waves per SIMD).
template <typename T>
constexpr int r1_rows() { return sizeof(T) == 4 ? 2 : 1; }
template <typename T, int D>
bool r1_wave(const PcgLaunch<T, D>& P) {
    return D == 2 && P.d.nx == WROW_NX && P.d.ny % r1_rows<T>() == 0 && P.d.ny / r1_rows<T>() <= PARTIALS_MAX &&
           !P.native && wave_rows_enabled();
}
// The FP32 Krylov loop's column passes on columns of 1024 points run as
// wave-private transforms too (k_pcg_c1w, k_pcg_c2w: one column per block, as the
// block kernels).  In FP64 the block kernels are faster (1024^2: C1 16.9 against
// 24.2 us, C2 21.8 against 26.1 us with the wave passes).
template <typename T, int D>
bool col_wave(const PcgLaunch<T, D>& P) {
    return sizeof(T) == 4 && D == 2 && P.d.ny == WCOL_NY && P.cl.g.Cb == 1 && !P.native && !P.wall &&
           wave_rows_enabled();
}
// Blocks of the row pass, i.e. the p.Gp partials the next column pass reduces.
template <typename T, int D>
int r1_blocks(const PcgLaunch<T, D>& P) { return r1_wave(P) ? P.d.ny / r1_rows<T>() : P.rl.g.nblocks; }

template <typename T, int D>
sgn_status pcg_r1(PcgLaunch<T, D>& P, bool curvature = false) {
    ProfScope ps(P.ctx, SGN_KERNEL_PCG_R1 + (sizeof(T) == 4 ? 6 : 0), true);
    double* part = curvature ? P.partials : nullptr;
    if (r1_wave(P)) {
        hipExtLaunchKernelGGL(k_pcg_r1w<T, r1_rows<T>()>, dim3(P.d.ny / r1_rows<T>()), dim3(192), 0,
                              P.ctx->stream, ps.a, ps.b, 0, P.d.ny,
                              twiddles<T>(P.ctx), P.sc, P.b.H, P.d.NS, P.eta, P.gh, part, PART_C2);
        CHECK_LAUNCH(P.ctx);
        return SGN_OK;
    }
    auto& L = P.rl;
    const bool seq = row_lds_bytes<T>(L.g, D + 1) > LDS_MULTI_MAX;
    const size_t lds = row_lds_bytes<T>(L.g, seq ? 1 : D + 1);
    auto launch = [&](auto k) -> sgn_status {
        HIPCHK(P.ctx, allow_lds(k, lds));
        hipExtLaunchKernelGGL(k, dim3(L.g.nblocks), dim3(L.threads), lds, P.ctx->stream, ps.a, ps.b, 0, L.g,
                              twiddles<T>(P.ctx), P.sc, P.b.H, P.d.NS, P.eta, P.gh, part);
        return SGN_OK;
    };
    sgn_status st;
    if (L.epc == 2)
        st = seq ? launch(k_pcg_r1<T, 2, D, true, 512>) : launch(k_pcg_r1<T, 2, D, false, 512>);
    else if (L.epc == 4)
        st = L.threads <= 256
                 ? (seq ? launch(k_pcg_r1<T, 4, D, true, 256>) : launch(k_pcg_r1<T, 4, D, false, 256>))
                 : (seq ? launch(k_pcg_r1<T, 4, D, true>) : launch(k_pcg_r1<T, 4, D, false>));
    else
        st = seq ? launch(k_pcg_r1<T, 8, D, true>) : launch(k_pcg_r1<T, 8, D, false>);
    if (st != SGN_OK) return st;
    CHECK_LAUNCH(P.ctx);
    return SGN_OK;
}

template <typename T, int D, int MODE>
sgn_status pcg_c2_mode(PcgLaunch<T, D>& P, const cpx<T>* bh, cpx<T>* rh_out, const ProfScope& ps) {
    auto& L = P.cl;
    const size_t lds = col_lds_bytes<T>(L.g, D + 1);
    // partials reduced at the start: p.Gp of the row pass, or ||b||^2 of the setup pass
    const int nb_red = MODE == C2_RESID_INIT ? L.g.nblocks : r1_blocks(P);
    auto launch = [&](auto k) -> sgn_status {
        HIPCHK(P.ctx, allow_lds(k, lds));
        hipExtLaunchKernelGGL(k, dim3(L.g.nblocks), dim3(L.threads), lds, P.ctx->stream, ps.a, ps.b, 0, L.g,
                              twiddles<T>(P.ctx), P.sc, (const cpx<T>*)P.b.H, P.d.NS, P.b.qh, (const cpx<T>*)P.b.ph,
                              P.b.xh, bh, rh_out, P.partials, nb_red, (T)P.d.tpx, (T)P.d.tpy);
        CHECK_LAUNCH(P.ctx);
        return SGN_OK;
    };
    if (P.native) {
        if constexpr (D == 2 && (MODE == C2_UPDATE || MODE == C2_RESID_INIT)) {
            auto k = L.epc == 2 ? k_wall_c2<T, 2, MODE> : k_wall_c2<T, 4, MODE>;
            HIPCHK(P.ctx, allow_lds(k, lds));
            hipExtLaunchKernelGGL(k, dim3(L.g.nblocks), dim3(L.threads), lds, P.ctx->stream, ps.a, ps.b, 0, L.g,
                                  twiddles<T>(P.ctx), P.sc, (const cpx<T>*)P.b.H, P.d.NS, (const cpx<T>*)P.b.ph,
                                  P.b.xh, bh, rh_out, P.partials, nb_red, (T)P.d.tpx, (T)P.d.tpy);
            CHECK_LAUNCH(P.ctx);
            return SGN_OK;
        } else {
            return fail(P.ctx, SGN_EINVAL, "pcg_c2: wall column pass takes updates and the initial residual only");
        }
    }
    if constexpr (MODE == C2_UPDATE) {
        if (col_wave(P)) {
            hipExtLaunchKernelGGL(k_pcg_c2w<T>, dim3(L.g.nblocks), dim3(WCOL_THREADS), 0, P.ctx->stream, ps.a, ps.b,
                                  0, P.d.nx, twiddles<T>(P.ctx), P.sc, (const cpx<T>*)P.b.H, P.d.NS,
                                  (const cpx<T>*)P.b.ph, P.b.xh, rh_out, P.partials, nb_red, (T)P.d.tpx,
                                  (T)P.d.tpy);
            CHECK_LAUNCH(P.ctx);
            return SGN_OK;
        }
    }
    if (L.epc == 2) return P.wall ? launch(k_pcg_c2<T, 2, D, MODE, true>) : launch(k_pcg_c2<T, 2, D, MODE>);
    return P.wall ? launch(k_pcg_c2<T, 4, D, MODE, true>) : launch(k_pcg_c2<T, 4, D, MODE>);
}

template <typename T, int D>
sgn_status pcg_c2(PcgLaunch<T, D>& P, int mode, const cpx<T>* bh, cpx<T>* rh_out) {
    ProfScope ps(P.ctx, SGN_KERNEL_PCG_C2 + (sizeof(T) == 4 ? 6 : 0), true);
    if (mode == C2_STORE) return pcg_c2_mode<T, D, C2_STORE>(P, bh, rh_out, ps);
    if (mode == C2_RESID) return pcg_c2_mode<T, D, C2_RESID>(P, bh, rh_out, ps);
    if (mode == C2_RESID_INIT) return pcg_c2_mode<T, D, C2_RESID_INIT>(P, bh, rh_out, ps);
    return pcg_c2_mode<T, D, C2_UPDATE>(P, nullptr, P.b.rh, ps);
}

// First pass of a solve in FP64: b (and the guess u0) to the half spectrum in one
// row launch, then k_pcg_setup; with a guess also G x_0 and r_0 = b - G x_0.
// Afterwards the partials of (r.z, r.r) of r_0 wait for the first C1.
template <int D>
sgn_status pcg_start(PcgLaunch<double, D>& P, const double* rhs, const double* u0, bool guess, cpx<double>* bh) {
    sgn_ctx* ctx = P.ctx;
    const Dims& d = P.d;
    // b's row transforms go to ph (unused until the first iteration) when a guess
    // is transformed too: the setup's two column jobs then read b from ph while
    // the guess job writes the row-pass fields of G x_0 to H
    cpx<double>* Hb = guess ? P.b.ph : P.b.H;
    std::vector<const double*> src;
    std::vector<cpx<double>*> dst;
    for (int c = 0; c < D; ++c) {
        src.push_back(rhs + c * d.N);
        dst.push_back(Hb + c * d.NS);
    }
    RowCombo<double> cmb{};
    cmb.first = -1;
    if (guess) {
        for (int c = 0; c < D; ++c) {
            src.push_back(u0 + c * d.N);
            dst.push_back(P.b.qh + c * d.NS);
        }
        if (ctx->gx_a) {   // stepper guess: base + offsets, formed while loading
            cmb.first = D;
            cmb.c1 = ctx->gx_c1;
            cmb.c2 = ctx->gx_c2;
            for (int c = 0; c < D; ++c) {
                cmb.a[c] = ctx->gx_a + c * d.N;
                cmb.b[c] = ctx->gx_b ? ctx->gx_b + c * d.N : nullptr;
            }
        }
    }
    sgn_status s;
    if ((s = rows_fwd<double, double>(ctx, d, src, dst, 1.0, &cmb)) != SGN_OK) return s;
    {
        ProfScope ps(ctx, SGN_KERNEL_PCG_INIT);
        const size_t lds = col_lds_bytes<double>(P.cl.g, D + 1);
        auto launch = [&](auto k) -> sgn_status {
            HIPCHK(ctx, allow_lds(k, lds));
            hipLaunchKernelGGL(k, dim3(P.cl.g.nblocks * (guess ? 2 : 1)), dim3(P.cl.threads), lds, ctx->stream,
                               P.cl.g, ctx->tw64, (const SolveScal*)P.sc, (const cpx<double>*)Hb,
                               (const cpx<double>*)P.b.qh, d.NS, bh, P.b.rh, P.b.xh, P.b.H, P.partials, d.tpx,
                               d.tpy);
            CHECK_LAUNCH(ctx);
            return SGN_OK;
        };
        if (P.native && P.cl.epc == 2)
            s = guess ? launch(k_wall_setup<double, 2, true>) : launch(k_wall_setup<double, 2, false>);
        else if (P.native)
            s = guess ? launch(k_wall_setup<double, 4, true>) : launch(k_wall_setup<double, 4, false>);
        else if (P.cl.epc == 2)
            s = guess ? launch(k_pcg_setup<double, 2, D, true>) : launch(k_pcg_setup<double, 2, D, false>);
        else
            s = guess ? launch(k_pcg_setup<double, 4, D, true>) : launch(k_pcg_setup<double, 4, D, false>);
        if (s != SGN_OK) return s;
    }
    if (guess) {
        if ((s = pcg_r1<double, D>(P)) != SGN_OK) return s;
        if ((s = pcg_c2<double, D>(P, C2_RESID_INIT, bh ? bh : P.b.rh, P.b.rh)) != SGN_OK) return s;
    }
    return SGN_OK;
}

// Wait until the stream has drained (polling an event when the context has one).
sgn_status wait_stream(sgn_ctx* ctx) {
    if (!ctx->ev_sync) {
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        return SGN_OK;
    }
    HIPCHK(ctx, hipEventRecord(ctx->ev_sync, ctx->stream));
    for (;;) {
        const hipError_t e = hipEventQuery(ctx->ev_sync);
        if (e == hipSuccess) return SGN_OK;
        if (e != hipErrorNotReady) return fail(ctx, SGN_EDEVICE, hipGetErrorString(e));
    }
}

// Read the solve's device scalars into ctx->hscal (synchronises the stream).
sgn_status read_scal(sgn_ctx* ctx, const SolveScal* sc) {
    HIPCHK(ctx, hipMemcpyAsync(ctx->hscal, sc, sizeof(SolveScal), hipMemcpyDeviceToHost, ctx->stream));
    return wait_stream(ctx);
}

// Initialise a SolveScal on the device (stream-ordered, no host round trip).
sgn_status init_scal(sgn_ctx* ctx, SolveScal* sc, double tol, int max_iter, double inv_n,
                     const sgn_coeffs* co, int init_bb = 0) {
    hipLaunchKernelGGL(k_init_scal, dim3(1), dim3(64), 0, ctx->stream, sc, tol, max_iter, inv_n, co ? 1 : 0,
                       co ? co->sigma : 0.0, co ? co->alpha : 0.0, co ? co->kappa_ub : 0.0, co ? co->flat : 0,
                       init_bb);
    CHECK_LAUNCH(ctx);
    return SGN_OK;
}

// Stop test; with pub set it also publishes the loop flags (sequence number seq).
template <typename T, int D>
sgn_status pcg_check(PcgLaunch<T, D>& P, int* pub = nullptr, int seq = 0, const SolveScal* inner = nullptr) {
    hipLaunchKernelGGL(k_pcg_check, dim3(1), dim3(256), 0, P.ctx->stream, P.sc, (const double*)P.partials,
                       P.cl.g.nblocks, pub, seq, inner);
    CHECK_LAUNCH(P.ctx);
    return SGN_OK;
}

// One chunk of `chunk` PCG iterations followed by the stop test (publishing the
// flags with sequence number seq when pub is set; none when check is false, for
// an inner solve whose state is discarded after the chunk).
template <typename T, int D>
sgn_status pcg_chunk_eager(PcgLaunch<T, D>& P, int chunk, int* pub = nullptr, int seq = 0, bool check = true) {
    for (int c = 0; c < chunk; ++c) {
        sgn_status s;
        if ((s = pcg_c1<T, D>(P, C1_UPDATE, nullptr)) != SGN_OK) return s;
        if ((s = pcg_r1<T, D>(P, true)) != SGN_OK) return s;
        if ((s = pcg_c2<T, D>(P, C2_UPDATE, nullptr, nullptr)) != SGN_OK) return s;
    }
    return check ? pcg_check<T, D>(P, pub, seq) : SGN_OK;
}

// The same chunk replayed from a HIP graph (captured on the second use of a
// configuration; the first use runs eagerly so every launch attribute is set).
// *published: whether the chunk's stop test already published the flags with
// the context's current sequence number (eager launches do; graphs do not).
template <typename T, int D>
sgn_status pcg_chunk(PcgLaunch<T, D>& P, int chunk, bool* published) {
    sgn_ctx* ctx = P.ctx;
    *published = false;
    if (!ctx->use_graphs || ctx->prof_on || ctx->cap_stream == nullptr) {
        *published = ctx->dpub != nullptr;
        return pcg_chunk_eager<T, D>(P, chunk, ctx->dpub, ctx->pub_seq);
    }
    std::vector<const void*> key = {(const void*)(uintptr_t)sizeof(T), (const void*)(uintptr_t)D,
                                    (const void*)(uintptr_t)(P.wall ? 1 : 0), (const void*)(uintptr_t)(P.native ? 1 : 0),
                                    (const void*)(uintptr_t)P.d.nx, (const void*)(uintptr_t)P.d.ny,
                                    (const void*)P.sc, (const void*)P.b.H, (const void*)P.b.xh,
                                    (const void*)P.b.rh, (const void*)P.b.ph, (const void*)P.partials,
                                    (const void*)P.eta, (const void*)P.gh, (const void*)twiddles<T>(ctx)};
    for (auto& g : ctx->graphs) {
        if (g.chunk == chunk && g.key == key) {
            if (g.exec) {
                HIPCHK(ctx, hipGraphLaunch(g.exec, ctx->stream));
                return SGN_OK;
            }
            // second use: capture
            hipStream_t user = ctx->stream;
            ctx->stream = ctx->cap_stream;
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
            sgn_status s = SGN_OK;
            if (e == hipSuccess) {
                s = pcg_chunk_eager<T, D>(P, chunk);
                e = hipStreamEndCapture(ctx->cap_stream, &graph);
            }
            ctx->stream = user;
            if (s != SGN_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return s;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                g.exec = nullptr;
                ctx->use_graphs = false;   // fall back to eager launches for the context's life
                *published = ctx->dpub != nullptr;
                return pcg_chunk_eager<T, D>(P, chunk, ctx->dpub, ctx->pub_seq);
            }
            HIPCHK(ctx, hipGraphLaunch(g.exec, ctx->stream));
            return SGN_OK;
        }
    }
    if (ctx->graphs.size() >= 64) {
        if (ctx->graphs.front().exec) (void)hipGraphExecDestroy(ctx->graphs.front().exec);
        ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back({key, chunk, nullptr});
    *published = ctx->dpub != nullptr;
    return pcg_chunk_eager<T, D>(P, chunk, ctx->dpub, ctx->pub_seq);
}

// Integer state of a solve after its last readback.
struct LoopOut {
    int iter = 0, done = 0, converged = 0, status = 0;
    int outer = -1;   // refinement steps taken (published flags only; -1 unknown)
};

// Read iter, max_iter, done, converged, flat, status of a solve (synchronises the stream).
// Next sequence number of the published loop flags.
void next_pub_seq(sgn_ctx* ctx) { ctx->pub_seq = ctx->pub_seq == 0x7fffffff ? 1 : ctx->pub_seq + 1; }

// Enqueue the publication of iter, max_iter, done, converged, flat, status
// (unless the last stop test already published them under the current sequence
// number) and mark it.
sgn_status issue_loop_readback(sgn_ctx* ctx, const SolveScal* sc, bool published = false) {
    if (ctx->dpub) {
        if (!published) {
            next_pub_seq(ctx);
            hipLaunchKernelGGL(k_publish_flags, dim3(1), dim3(64), 0, ctx->stream, sc, ctx->dpub, ctx->pub_seq);
            CHECK_LAUNCH(ctx);
        }
        return SGN_OK;
    }
    HIPCHK(ctx, hipMemcpyAsync(ctx->hflag, &sc->iter, 6 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    if (ctx->ev_sync) HIPCHK(ctx, hipEventRecord(ctx->ev_sync, ctx->stream));
    return SGN_OK;
}
// Wait for the flags enqueued by issue_loop_readback (work enqueued after them
// may still run) and decode them.
sgn_status wait_loop_readback(sgn_ctx* ctx, LoopOut* out) {
    const int* f = ctx->hflag;
    if (ctx->dpub) {
        // poll the published sequence number; a drained stream bounds the wait if
        // the value is somehow not seen
        int* h = ctx->hpub;
        for (long spins = 0;; ++spins) {
            if (__atomic_load_n(&h[6], __ATOMIC_ACQUIRE) == ctx->pub_seq) break;
            if ((spins & 4095) == 4095) {
                const hipError_t e = hipStreamQuery(ctx->stream);
                if (e == hipSuccess) {
                    if (__atomic_load_n(&h[6], __ATOMIC_ACQUIRE) == ctx->pub_seq) break;
                    return fail(ctx, SGN_EDEVICE, "published solver flags not visible to the host");
                }
                if (e != hipErrorNotReady) return fail(ctx, SGN_EDEVICE, hipGetErrorString(e));
            }
        }
        f = h;
    } else if (!ctx->ev_sync) {
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    } else {
        for (;;) {
            const hipError_t e = hipEventQuery(ctx->ev_sync);
            if (e == hipSuccess) break;
            if (e != hipErrorNotReady) return fail(ctx, SGN_EDEVICE, hipGetErrorString(e));
        }
    }
    out->iter = f[0];
    out->done = f[2];
    out->converged = f[3];
    out->status = f[5];
    out->outer = ctx->dpub ? f[7] : -1;
    return SGN_OK;
}

sgn_status read_loop(sgn_ctx* ctx, const SolveScal* sc, LoopOut* out) {
    sgn_status s = issue_loop_readback(ctx, sc);
    return s != SGN_OK ? s : wait_loop_readback(ctx, out);
}

// Run PCG iterations until the device flag says done.  The first chunk is sized
// from the previous solve of the same precision (warm-started stage solves need
// about as many iterations as the one before), later chunks are short, so a
// solve usually needs one host readback and wastes at most a couple of
// iterations (which return at once on the device).
//
// tail (optional): the work that follows the solve on the device (storing the
// result).  It is enqueued right after the first readback, so the GPU runs it
// while the host waits for the flag; if the solve needed more iterations, it is
// enqueued again after them with redo = true.
template <typename T, int D, typename Tail = std::nullptr_t>
sgn_status pcg_loop(PcgLaunch<T, D>& P, int max_iter, int check_every, LoopOut* out, Tail tail = nullptr) {
    if (check_every < 1) check_every = 1;
    const int prec = sizeof(T) == 4 ? 1 : 0;
    int& last = P.ctx->stage_last ? P.ctx->stage_last[prec] : P.ctx->last_iters[prec][P.ctx->slot];
    // as many iterations as the previous solve of the slot took: a solve that
    // needs more continues in short chunks after a readback.  (One iteration of
    // margin, whose launches return at once when the solve has converged, measured
    // slower on the 1024^2 RK4 workload: 2.744 against 2.727 ms per step; the
    // launches are the same work either way, so results do not change.)
    int chunk = last > 0 ? last : check_every;
    int it = 0;
    bool tail_done = false, rounds = false;
    sgn_status s;
    while (it < max_iter) {
        chunk = std::max(1, std::min(chunk, max_iter - it));
        if (P.ctx->dpub) next_pub_seq(P.ctx);
        bool published = false;
        if ((s = pcg_chunk<T, D>(P, chunk, &published)) != SGN_OK) return s;
        it += chunk;
        if ((s = issue_loop_readback(P.ctx, P.sc, published)) != SGN_OK) return s;
        if constexpr (!std::is_same<Tail, std::nullptr_t>::value) {
            if (!rounds) {
                if ((s = tail(false)) != SGN_OK) return s;
                tail_done = true;
            }
        }
        if ((s = wait_loop_readback(P.ctx, out)) != SGN_OK) return s;
        if (out->done) break;
        rounds = true;
        chunk = std::min(2, check_every);
    }
    if constexpr (!std::is_same<Tail, std::nullptr_t>::value) {
        if (!tail_done || rounds)
            if ((s = tail(tail_done)) != SGN_OK) return s;
    }
    if (out->iter > 0) last = out->iter;
    return SGN_OK;
}

template <int D>
sgn_status solve_fp64(sgn_ctx* ctx, const Dims& d, const double* eta, const double* gh, const double* rhs,
                      double* u, const sgn_coeffs* coeffs, int flat, const sgn_solve_opts& o,
                      sgn_solve_info* info, void* ws) {
    Carve cv(ws);
    Common cm = carve_common(cv);
    PcgLaunch<double, D> P;
    P.wall = ctx->wall_twin;
    P.native = D == 2 && ctx->wall_native;
    P.ctx = ctx;
    P.d = d;
    P.rl = row_launch<double>(d.nx, d.ny, true);
    P.cl = P.native ? wall_col_launch(d.nx, d.ny) : pcg_col_launch<double>(d);
    P.b = carve_pcg<double>(cv, d, false);
    P.sc = cm.sc;
    P.partials = cm.partials;
    P.eta = eta;
    P.gh = gh;
    sgn_status s;
    // without a guess r_0 = b, so ||b||^2 is the first r.r (init_bb); computed
    // coefficients initialise the scalars in their finishing kernel
    if (coeffs) {
        if ((s = init_scal(ctx, P.sc, o.tol, o.max_iter, d.inv_n, coeffs, o.x0_is_guess ? 0 : 1)) != SGN_OK) return s;
    } else {
        const ScalInit in{o.tol, o.max_iter, d.inv_n, o.x0_is_guess ? 0 : 1};
        if ((s = launch_coeffs(ctx, d, eta, gh, flat, o.coeff_kind, P.sc, P.partials, nullptr, nullptr, &in)) !=
            SGN_OK)
            return s;
    }
    if ((s = pcg_start<D>(P, rhs, u, o.x0_is_guess != 0, nullptr)) != SGN_OK) return s;
    // u = IFFT(x_hat) (and the stepper's offset record); stored a second time after
    // further iterations, the offset accumulates the difference
    auto store = [&](bool redo) -> sgn_status {
        auto k = P.native ? (P.cl.epc == 2 ? k_wall_from_S<double, 2> : k_wall_from_S<double, 4>)
                          : (P.cl.epc == 2 ? k_cols_from_S<double, 2, D> : k_cols_from_S<double, 4, D>);
        HIPCHK(ctx, allow_lds(k, col_lds_bytes<double>(P.cl.g, D)));
        hipLaunchKernelGGL(k, dim3(P.cl.g.nblocks), dim3(P.cl.threads), col_lds_bytes<double>(P.cl.g, D), ctx->stream,
                           P.cl.g, ctx->tw64, (const cpx<double>*)P.b.xh, d.NS, P.b.H, d.inv_n);
        CHECK_LAUNCH(ctx);
        std::vector<const cpx<double>*> hs;
        std::vector<double*> ud, od;
        for (int c = 0; c < D; ++c) {
            hs.push_back(P.b.H + c * d.NS);
            ud.push_back(u + c * d.N);
            if (ctx->gx_off) od.push_back(ctx->gx_off + c * d.N);
        }
        return rows_inv<double, double>(ctx, d, hs, ud, 1.0, 0.0, ctx->gx_off ? &od : nullptr, redo);
    };
    LoopOut lo;
    if (ctx->stage) {
        // stepper: the store is enqueued behind the first readback, so the GPU does
        // it while the host waits for the convergence flag
        if ((s = pcg_loop<double, D>(P, o.max_iter, o.check_every, &lo, store)) != SGN_OK) return s;
    } else {
        if ((s = pcg_loop<double, D>(P, o.max_iter, o.check_every, &lo)) != SGN_OK) return s;
        if ((s = store(false)) != SGN_OK) return s;
    }
    if (ctx->stage) {
        // stepper: iterations and the outcome are known from the loop's readback
        if (info) {
            info->iters = lo.iter;
            info->converged = lo.converged;
        }
        if (lo.status == -2) return fail(ctx, SGN_EDOMAIN, "non-positive depth or non-finite data in the solve");
        if (!lo.converged) return fail(ctx, SGN_ENOCONV, "Krylov solve did not reach the tolerance");
        return SGN_OK;
    }
    if ((s = read_scal(ctx, P.sc)) != SGN_OK) return s;
    const SolveScal& h = *ctx->hscal;
    if (info) {
        info->iters = h.iter;
        info->outer_iters = 0;
        info->converged = h.converged;
        info->relres = h.relres;
        info->coeffs.sigma = h.sig;
        info->coeffs.alpha = h.alp;
        info->coeffs.kappa_ub = h.kap;
        info->coeffs.flat = h.flat;
    }
    if (h.status == -2) return fail(ctx, SGN_EDOMAIN, "non-positive depth or non-finite data in the solve");
    if (!h.converged) return fail(ctx, SGN_ENOCONV, "Krylov solve did not reach the tolerance");
    return SGN_OK;
}

// ---------------------------------------------------------------------------
// FP64 PCG on a 2D grid between walls on the grid's own points: eta, grad h, b
// (and the guess) are put in transform order (sgn_wall.h), the iteration runs
// the periodic row pass between the wall column passes, and the result goes
// back to grid order.  No periodic twin is formed.
// ---------------------------------------------------------------------------
struct WallOrderBufs {
    double *eta, *gh, *b, *u;
};
void carve_wall_order(Carve& cv, const Dims& d, WallOrderBufs* w) {
    w->eta = cv.take<double>(d.N);
    w->gh = cv.take<double>(2 * d.N);
    w->b = cv.take<double>(2 * d.N);
    w->u = cv.take<double>(2 * d.N);
}

// A scalar or a 2D vector field (u sine along x, v sine along y) between grid
// order and transform order.
sgn_status wall_order(sgn_ctx* ctx, const Dims& d, const double* src, double* dst, bool vector, bool to_order) {
    ProfScope ps(ctx, SGN_KERNEL_WALL_ORDER);
    const int nf = vector ? 2 : 1;
    const unsigned sx = vector ? 1u : 0u, sy = vector ? 2u : 0u;
    hipLaunchKernelGGL(k_wall_order, dim3(flat_blocks(d.N * nf)), dim3(256), 0, ctx->stream, d.nx, d.ny, nf, sx, sy,
                       to_order ? 1 : 0, src, dst);
    CHECK_LAUNCH(ctx);
    return SGN_OK;
}

// Solves between walls that run on the grid's own points; the others (1D,
// mixed precision, GMRES) run on the periodic twin.
bool wall_native(const Dims& d, const sgn_solve_opts& o) {
    return d.D == 2 && d.bc == SGN_BC_WALLS && o.method == SGN_PCG && o.precision == SGN_FP64 &&
           4 * d.nx <= TW_SIZE && 4 * d.ny <= TW_SIZE;
}

sgn_status solve_wall_native(sgn_ctx* ctx, const Dims& dw, const double* eta, const double* gh, const double* rhs,
                             double* u, const sgn_coeffs* coeffs, int flat, const sgn_solve_opts& o,
                             sgn_solve_info* info, void* ws) {
    if (o.method != SGN_PCG || o.precision != SGN_FP64) return fail(ctx, SGN_EINVAL, "wall solve: FP64 PCG only");
    if (!(o.tol > 0.0) || o.max_iter < 1) return fail(ctx, SGN_EINVAL, "tol must be > 0 and max_iter >= 1");
    if (coeffs && !(coeffs->sigma > 0.0 && coeffs->alpha > 0.0))
        return fail(ctx, SGN_EINVAL, "coefficients must be positive");
    // wavenumbers of the slots: s pi / L
    Dims d = dw;
    d.tpx = 0.5 * kTwoPi / d.Lx;
    d.tpy = 0.5 * kTwoPi / d.Ly;
    Carve cv(ws);
    WallOrderBufs w;
    carve_wall_order(cv, d, &w);
    Common cm = carve_common(cv);
    PcgLaunch<double, 2> P;
    P.native = true;
    P.ctx = ctx;
    P.d = d;
    P.rl = row_launch<double>(d.nx, d.ny, true);
    P.cl = wall_col_launch(d.nx, d.ny);
    P.b = carve_pcg<double>(cv, d, false);
    P.sc = cm.sc;
    P.partials = cm.partials;
    P.eta = w.eta;
    P.gh = w.gh;
    const bool guess = o.x0_is_guess != 0;
    sgn_status s;
    if ((s = wall_order(ctx, d, eta, w.eta, false, true)) != SGN_OK) return s;
    if ((s = wall_order(ctx, d, gh, w.gh, true, true)) != SGN_OK) return s;
    if ((s = wall_order(ctx, d, rhs, w.b, true, true)) != SGN_OK) return s;
    if (guess && (s = wall_order(ctx, d, u, w.u, true, true)) != SGN_OK) return s;
    // the coefficients are pointwise extrema: taken on the grid-order fields
    if (coeffs) {
        if ((s = init_scal(ctx, P.sc, o.tol, o.max_iter, d.inv_n, coeffs, guess ? 0 : 1)) != SGN_OK) return s;
    } else {
        const ScalInit in{o.tol, o.max_iter, d.inv_n, guess ? 0 : 1};
        if ((s = launch_coeffs(ctx, d, eta, gh, flat, o.coeff_kind, P.sc, P.partials, nullptr, nullptr, &in)) !=
            SGN_OK)
            return s;
    }
    if ((s = pcg_start<2>(P, w.b, w.u, guess, nullptr)) != SGN_OK) return s;
    LoopOut lo;
    if ((s = pcg_loop<double, 2>(P, o.max_iter, o.check_every, &lo)) != SGN_OK) return s;
    if ((s = read_scal(ctx, P.sc)) != SGN_OK) return s;
    const SolveScal& h = *ctx->hscal;
    if (info) {
        info->iters = h.iter;
        info->outer_iters = 0;
        info->converged = h.converged;
        info->relres = h.relres;
        info->coeffs.sigma = h.sig;
        info->coeffs.alpha = h.alp;
        info->coeffs.kappa_ub = h.kap;
        info->coeffs.flat = h.flat;
    }
    if (h.status == -2) return fail(ctx, SGN_EDOMAIN, "non-positive depth or non-finite data in the solve");
    // the iterate is returned on success and when max_iter stops the solve
    {
        auto k = P.cl.epc == 2 ? k_wall_from_S<double, 2> : k_wall_from_S<double, 4>;
        const size_t lds = col_lds_bytes<double>(P.cl.g, 2);
        HIPCHK(ctx, allow_lds(k, lds));
        hipLaunchKernelGGL(k, dim3(P.cl.g.nblocks), dim3(P.cl.threads), lds, ctx->stream, P.cl.g, ctx->tw64,
                           (const cpx<double>*)P.b.xh, d.NS, P.b.H, d.inv_n);
        CHECK_LAUNCH(ctx);
    }
    if ((s = rows_inv<double, double>(ctx, d, {P.b.H, P.b.H + d.NS}, {w.u, w.u + d.N})) != SGN_OK) return s;
    if ((s = wall_order(ctx, d, w.u, u, true, false)) != SGN_OK) return s;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (!h.converged) return fail(ctx, SGN_ENOCONV, "Krylov solve did not reach the tolerance");
    return SGN_OK;
}

// Inner tolerance of refinement steps relative to the remaining gap to the
// target: the inner solve aims at the outer tolerance itself (c = 1).  The
// outer FP64 stop test decides convergence whatever c is; on the 1024^2 RK4
// workload (40 steps) c = 1/2, 1/sqrt(2), 1 took 6.1, 5.8, 5.35 inner
// iterations per solve and 2.83, 2.78, 2.72 ms per step.
constexpr double INNER_SAFETY2 = 1.0;

// Mixed precision: FP64 iterative refinement around FP32 PCG inner solves.  The
// outer state (x_hat, r_hat = b_hat - G x_hat) and every dot product stay in
// FP64; the inner operator, FFTs and preconditioner run in FP32.
template <int D>
sgn_status solve_mixed(sgn_ctx* ctx, const Dims& d, const double* eta, const double* gh, const double* rhs,
                       double* u, const sgn_coeffs* coeffs, int flat, const sgn_solve_opts& o,
                       sgn_solve_info* info, void* ws) {
    Carve cv(ws);
    Common cm = carve_common(cv);
    PcgLaunch<double, D> P;
    P.wall = ctx->wall_twin;
    P.ctx = ctx;
    P.d = d;
    P.rl = row_launch<double>(d.nx, d.ny, true);
    P.cl = pcg_col_launch<double>(d);
    P.b = carve_pcg<double>(cv, d, true);
    P.sc = cm.sc;
    P.partials = cm.partials;
    P.eta = eta;
    P.gh = gh;
    PcgLaunch<float, D> Q;
    Q.wall = ctx->wall_twin;
    Q.ctx = ctx;
    Q.d = d;
    Q.rl = row_launch<float>(d.nx, d.ny, true);
    Q.cl = pcg_col_launch<float>(d);
    Q.b = carve_pcg<float>(cv, d, false);
    Q.sc = cm.sc + 1;
    Q.partials = cm.partials;
    float* eta32 = cv.take<float>((size_t)(1 + D) * d.N);
    Q.eta = eta32;
    Q.gh = eta32 + d.N;
    sgn_status s;
    if ((s = init_scal(ctx, P.sc, o.tol, 1 << 30, d.inv_n, coeffs, o.x0_is_guess ? 0 : 1)) != SGN_OK) return s;
    if (!coeffs) {
        // the coefficient pass also writes the FP32 copies of eta and grad h
        if ((s = launch_coeffs(ctx, d, eta, gh, flat, o.coeff_kind, P.sc, P.partials, eta32, eta32 + d.N)) !=
            SGN_OK)
            return s;
    } else {
        hipLaunchKernelGGL((k_convert<float, double>), dim3(flat_blocks(d.N)), dim3(256), 0, ctx->stream, d.N, eta,
                           eta32);
        hipLaunchKernelGGL((k_convert<float, double>), dim3(flat_blocks(d.D * d.N)), dim3(256), 0, ctx->stream,
                           (size_t)D * d.N, gh, eta32 + d.N);
        CHECK_LAUNCH(ctx);
    }
    // b_hat (kept) and r_hat = b_hat - G x_hat in FP64, with the partials of r_0
    if ((s = pcg_start<D>(P, rhs, u, o.x0_is_guess != 0, P.b.bh)) != SGN_OK) return s;
    int total_inner = 0, outer = 0;
    const int max_outer = o.max_outer > 0 ? o.max_outer : 20;
    const double inner_tol = o.inner_tol > 0 ? o.inner_tol : 1e-5;
    LoopOut lo;
    // u = IFFT(x_hat) and the stepper's offset record (as in the FP64 solve: the
    // guess was formed from the base while pcg_start loaded it); a store after a
    // further refinement step adds its difference to the offset
    int stores = 0;
    auto store = [&]() -> sgn_status {
        auto k = P.cl.epc == 2 ? k_cols_from_S<double, 2, D> : k_cols_from_S<double, 4, D>;
        HIPCHK(ctx, allow_lds(k, col_lds_bytes<double>(P.cl.g, D)));
        hipLaunchKernelGGL(k, dim3(P.cl.g.nblocks), dim3(P.cl.threads), col_lds_bytes<double>(P.cl.g, D),
                           ctx->stream, P.cl.g, ctx->tw64, (const cpx<double>*)P.b.xh, d.NS, P.b.H, d.inv_n);
        CHECK_LAUNCH(ctx);
        std::vector<const cpx<double>*> hs;
        std::vector<double*> ud, od;
        for (int c = 0; c < D; ++c) {
            hs.push_back(P.b.H + c * d.NS);
            ud.push_back(u + c * d.N);
            if (ctx->gx_off) od.push_back(ctx->gx_off + c * d.N);
        }
        return rows_inv<double, double>(ctx, d, hs, ud, 1.0, 0.0, ctx->gx_off ? &od : nullptr, stores++ > 0);
    };
    // the inner FP32 solve of one refinement step and the FP64 residual after it;
    // the inner solve is marked done at once when the outer stop test has already
    // converged, so that every kernel of the step returns at once
    auto open_inner = [&]() -> sgn_status {
        ProfScope ps(ctx, SGN_KERNEL_PCG_INIT + 6);
        // the inner scalars, r32 = r, x32 = 0 and the inner solve's first partials,
        // in one pass
        hipLaunchKernelGGL((k_inner_start<D>), dim3(Q.cl.g.nblocks), dim3(256), 0, ctx->stream, d.nx, d.ny, d.NS,
                           (const SolveScal*)P.sc, Q.sc, inner_tol, o.max_iter, d.inv_n, INNER_SAFETY2,
                           (const cpx<double>*)P.b.rh, Q.b.rh, Q.b.xh, Q.partials, (float)d.tpx, (float)d.tpy);
        CHECK_LAUNCH(ctx);
        return SGN_OK;
    };
    auto close_inner = [&]() -> sgn_status {
        // x_hat += dx_hat inside the pass that starts G x_hat; r_hat = b_hat - G x_hat
        // (FP64) with its dot products
        sgn_status t;
        if ((t = pcg_c1<double, D>(P, C1_ACCUM, nullptr, Q.b.xh)) != SGN_OK) return t;
        if ((t = pcg_r1<double, D>(P)) != SGN_OK) return t;
        return pcg_c2<double, D>(P, C2_RESID, P.b.bh, P.b.rh);
    };
    // the outer stop test after a refinement step, which first counts the step
    // and its inner iterations
    auto check_outer = [&](int* pub) -> sgn_status {
        return pcg_check<double, D>(P, pub, ctx->pub_seq, (const SolveScal*)Q.sc);
    };
    // stop test of the initial residual (a step after it returns at once if it converged)
    if ((s = pcg_check<double, D>(P)) != SGN_OK) return s;
    if (ctx->stage) {
        // Stepper solves: refinement steps are enqueued without waiting for the
        // host; the inner solve runs a fixed chunk of iterations sized from the
        // stepping state's previous solve (one that has not converged in it still
        // yields a correction: the FP64 residual decides, and the next step's
        // chunk is twice as long).  The host reads the flags once per step, with
        // the store of the result already enqueued behind them; steps and inner
        // iterations are counted on the device.  The chunk depends only on the
        // state's own history, so a run's result does not depend on what else
        // its context solved.
        int& last_in = ctx->stage_last[1];
        int chunk_in = std::max(1, std::min(o.max_iter, last_in > 0 ? last_in + 1 : o.check_every));
        while (outer < max_outer) {
            if ((s = open_inner()) != SGN_OK) return s;
            if ((s = pcg_chunk_eager<float, D>(Q, chunk_in, nullptr, 0, false)) != SGN_OK) return s;
            if ((s = close_inner()) != SGN_OK) return s;
            ++outer;
            // the stop test publishes the flags itself when the context has a
            // host-coherent flag buffer
            if (ctx->dpub) next_pub_seq(ctx);
            if ((s = check_outer(ctx->dpub)) != SGN_OK) return s;
            if ((s = issue_loop_readback(ctx, P.sc, ctx->dpub != nullptr)) != SGN_OK) return s;
            if ((s = store()) != SGN_OK) return s;
            if ((s = wait_loop_readback(ctx, &lo)) != SGN_OK) return s;
            if (lo.done) break;
            chunk_in = std::min(o.max_iter, 2 * chunk_in);
        }
        if (lo.outer > 0) last_in = (lo.iter + lo.outer - 1) / lo.outer;
    } else {
        // Standalone and served solves: every inner solve runs to its own
        // tolerance (host-checked chunks), so the result does not depend on the
        // context's earlier solves.
        if ((s = read_loop(ctx, P.sc, &lo)) != SGN_OK) return s;
        while (!lo.done && outer < max_outer) {
            if ((s = open_inner()) != SGN_OK) return s;
            LoopOut li;
            if ((s = pcg_loop<float, D>(Q, o.max_iter, o.check_every, &li)) != SGN_OK) return s;
            if ((s = close_inner()) != SGN_OK) return s;
            ++outer;
            if ((s = check_outer(nullptr)) != SGN_OK) return s;
            if ((s = read_loop(ctx, P.sc, &lo)) != SGN_OK) return s;
        }
        if ((s = store()) != SGN_OK) return s;
    }
    if (lo.outer >= 0) {   // the device's counts (published with the flags)
        total_inner = lo.iter;
        outer = lo.outer;
    } else {
        if ((s = read_scal(ctx, P.sc)) != SGN_OK) return s;
        total_inner = ctx->hscal->iter;
        outer = ctx->hscal->outer;
    }
    if (ctx->stage && lo.done) {
        if (info) {
            info->iters = total_inner;
            info->outer_iters = outer;
            info->converged = lo.converged;
        }
        if (lo.status == -2) return fail(ctx, SGN_EDOMAIN, "non-positive depth or non-finite data in the solve");
        if (!lo.converged) return fail(ctx, SGN_ENOCONV, "refinement did not reach the tolerance");
        return SGN_OK;
    }
    if ((s = read_scal(ctx, P.sc)) != SGN_OK) return s;
    const SolveScal& h = *ctx->hscal;
    if (info) {
        info->iters = total_inner;
        info->outer_iters = outer;
        info->converged = h.converged;
        info->relres = h.relres;
        info->coeffs.sigma = h.sig;
        info->coeffs.alpha = h.alp;
        info->coeffs.kappa_ub = h.kap;
        info->coeffs.flat = h.flat;
    }
    if (h.status == -2) return fail(ctx, SGN_EDOMAIN, "non-positive depth or non-finite data in the solve");
    if (!h.converged) return fail(ctx, SGN_ENOCONV, "refinement did not reach the tolerance");
    return SGN_OK;
}

// ---------------------------------------------------------------------------
// Right-preconditioned restarted GMRES(m) in FP64 (section 3.2 names GMRES
// beside PCG for the constraint solve).  The Krylov basis lives in the S layout
// (half spectrum, Parseval inner products), so G is applied by the same three
// passes as in PCG and A^{-1} is a pointwise multiply.  Arnoldi uses classical
// Gram-Schmidt with one reorthogonalisation (CGS2: two block dot products and
// two block updates per step, all against the contiguous basis), which equals
// modified Gram-Schmidt in exact arithmetic; the small Hessenberg least-squares
// problem (Givens rotations, back substitution) and the stop tests run in
// one-thread kernels on device-resident state, so the host issues Arnoldi steps
// in chunks and reads the state back once per chunk (check_every steps), not
// once per step; the steps issued after a cycle has ended return at once.
// Only V_0..V_m are stored: the update x += A^{-1} (V y) uses the linearity of
// A^{-1} instead of keeping Z_j.
// ---------------------------------------------------------------------------
sgn_status batch_staging(sgn_ctx* ctx, size_t bytes);
template <int D>
sgn_status to_S_d(sgn_ctx* ctx, const Dims& d, const double* f, cpx<double>* H, cpx<double>* Sd);
template <int D>
sgn_status from_S_d(sgn_ctx* ctx, const Dims& d, const cpx<double>* Ssrc, cpx<double>* H, double* f);

constexpr int GMRES_MAX_RESTART = 256;
static_assert(sizeof(GmresCtl) <= 512, "GMRES state readback");
constexpr int GMRES_DOT_BLOCKS = 512;

struct GmresBufs {
    cpx<double>* bh;     // b in S
    cpx<double>* V;      // (m + 1) basis vectors of D * NS modes
    double* part;        // per-block partial dot products
    double* coef;        // device coefficients: h (m + 1), h2 (m + 1), ||w||^2
    double* hs;          // Hessenberg matrix, rotations, g and y of a cycle (gmres_hess_doubles)
    GmresCtl* ctl;
};
GmresBufs carve_gmres(Carve& cv, const Dims& d, int m) {
    GmresBufs g;
    g.bh = cv.take<cpx<double>>((size_t)d.D * d.NS);
    g.V = cv.take<cpx<double>>((size_t)(m + 1) * d.D * d.NS);
    g.part = cv.take<double>((size_t)GMRES_DOT_BLOCKS * (m + 1));
    g.coef = cv.take<double>((size_t)3 * (m + 2));
    g.hs = cv.take<double>(gmres_hess_doubles(m));
    g.ctl = cv.take<GmresCtl>(1);
    return g;
}

size_t gmres_workspace_bytes(const Dims& d, int m) {
    Carve cv(nullptr);
    carve_common(cv);
    carve_pcg<double>(cv, d, false);
    carve_gmres(cv, d, m);
    return std::max(cv.off + 256, workspace_bytes(d, SGN_FP64));
}

template <int D>
struct Gmres {
    PcgLaunch<double, D> P;
    GmresBufs g;
    int dot_blocks;
    size_t nd;   // doubles per S vector

    cpx<double>* Vi(int i) { return g.V + (size_t)i * D * P.d.NS; }

    // coef[out .. out + nv) = <w, V_i> for i < nv; stop: the gate (null: always run)
    sgn_status dots(const cpx<double>* w, const cpx<double>* V, int nv, double* out, const SolveScal* stop) {
        sgn_ctx* ctx = P.ctx;
        hipLaunchKernelGGL(k_S_multidot<D>, dim3(dot_blocks), dim3(256), 0, ctx->stream, P.d.nx, P.d.ny, P.d.NS, w,
                           V, (size_t)D * P.d.NS, nv, g.part, stop);
        hipLaunchKernelGGL(k_S_multidot_finish, dim3(1), dim3(256), 0, ctx->stream, (const double*)g.part,
                           dot_blocks, nv, P.d.inv_n, out, stop);
        CHECK_LAUNCH(ctx);
        return SGN_OK;
    }
    // w += sign * sum_i coef[i] V_i (i < nv, or i < *nv_dev when set)
    sgn_status axpy(cpx<double>* w, int nv, const double* coef, double sign, const SolveScal* stop,
                    const int* nv_dev = nullptr) {
        hipLaunchKernelGGL(k_S_multiaxpy, dim3(flat_blocks(nd)), dim3(256), 0, P.ctx->stream, nd, (double*)w,
                           (const double*)g.V, nd, nv, coef, sign, stop, nv_dev);
        CHECK_LAUNCH(P.ctx);
        return SGN_OK;
    }
    // y = scale[0] x (scale in device memory)
    sgn_status scale(const double* sc_dev, const cpx<double>* x, cpx<double>* y, const SolveScal* stop) {
        hipLaunchKernelGGL(k_S_scale, dim3(flat_blocks(nd)), dim3(256), 0, P.ctx->stream, nd, sc_dev,
                           (const double*)x, (double*)y, stop);
        CHECK_LAUNCH(P.ctx);
        return SGN_OK;
    }
    // q_hat = G x for x in S (three passes of the PCG operator)
    sgn_status apply(const cpx<double>* x) {
        sgn_status s;
        if ((s = pcg_c1<double, D>(P, C1_COPY, x)) != SGN_OK) return s;
        if ((s = pcg_r1<double, D>(P)) != SGN_OK) return s;
        return pcg_c2<double, D>(P, C2_STORE, nullptr, nullptr);
    }
    sgn_status precond(const cpx<double>* v, cpx<double>* z, double sig, double alp, const SolveScal* stop) {
        hipLaunchKernelGGL(k_S_precond<D>, dim3(flat_blocks(P.d.NS)), dim3(256), 0, P.ctx->stream, P.d.nx, P.d.ny,
                           P.d.NS, P.d.tpx, P.d.tpy, sig, alp, v, z, stop);
        CHECK_LAUNCH(P.ctx);
        return SGN_OK;
    }
    // y = a x + b y over one S vector
    sgn_status axpby(double a, const cpx<double>* x, double b, cpx<double>* y) {
        hipLaunchKernelGGL(k_axpby, dim3(flat_blocks(nd)), dim3(256), 0, P.ctx->stream, nd, a, (const double*)x, b,
                           (double*)y);
        CHECK_LAUNCH(P.ctx);
        return SGN_OK;
    }
    sgn_status read(const double* dsrc, double* hdst, int n) {
        HIPCHK(P.ctx, hipMemcpyAsync(hdst, dsrc, n * sizeof(double), hipMemcpyDeviceToHost, P.ctx->stream));
        return wait_stream(P.ctx);
    }
};

template <int D>
sgn_status solve_gmres(sgn_ctx* ctx, const Dims& d, const double* eta, const double* gh, const double* rhs,
                       double* u, const sgn_coeffs* coeffs, int flat, const sgn_solve_opts& o,
                       sgn_solve_info* info, void* ws) {
    const int m = o.gmres_restart;
    Carve cv(ws);
    Common cm = carve_common(cv);
    Gmres<D> G;
    auto& P = G.P;
    P.ctx = ctx;
    P.d = d;
    P.rl = row_launch<double>(d.nx, d.ny, true);
    P.cl = pcg_col_launch<double>(d);
    P.b = carve_pcg<double>(cv, d, false);
    P.sc = cm.sc;
    P.partials = cm.partials;
    P.eta = eta;
    P.gh = gh;
    G.g = carve_gmres(cv, d, m);
    G.dot_blocks = std::min(GMRES_DOT_BLOCKS, flat_blocks(d.NS));
    G.nd = (size_t)2 * D * d.NS;
    sgn_status s;
    // pinned readback: ||b||^2, then the cycle state and the stop flag (at byte 512)
    if ((s = batch_staging(ctx, 1024)) != SGN_OK) return s;
    double* hc = static_cast<double*>(ctx->hbatch);
    // coefficients of A (given or computed), read once: the basis loop is host driven
    if ((s = init_scal(ctx, P.sc, o.tol, o.max_iter, d.inv_n, coeffs)) != SGN_OK) return s;
    if (!coeffs) {
        if ((s = launch_coeffs(ctx, d, eta, gh, flat, o.coeff_kind, P.sc, P.partials)) != SGN_OK) return s;
    }
    if ((s = read_scal(ctx, P.sc)) != SGN_OK) return s;
    const SolveScal sc0 = *ctx->hscal;
    auto finish_info = [&](int iters, bool conv, double relres) {
        if (!info) return;
        info->iters = iters;
        info->outer_iters = 0;
        info->converged = conv ? 1 : 0;
        info->relres = relres;
        info->coeffs.sigma = sc0.sig;
        info->coeffs.alpha = sc0.alp;
        info->coeffs.kappa_ub = sc0.kap;
        info->coeffs.flat = sc0.flat;
    };
    if (sc0.status != 0 || !(sc0.sig > 0.0) || !(sc0.alp > 0.0)) {
        finish_info(0, false, std::nan(""));
        return fail(ctx, SGN_EDOMAIN, "non-positive depth or non-finite data in the solve");
    }
    const double sig = sc0.sig, alp = sc0.alp;
    cpx<double>* bh = G.g.bh;
    cpx<double>* xh = P.b.xh;
    cpx<double>* zh = P.b.ph;
    cpx<double>* qh = P.b.qh;
    if ((s = to_S_d<D>(ctx, d, rhs, P.b.H, bh)) != SGN_OK) return s;
    if ((s = G.dots(bh, bh, 1, G.g.coef, nullptr)) != SGN_OK) return s;
    if ((s = G.read(G.g.coef, hc, 1)) != SGN_OK) return s;
    const double bnorm = std::sqrt(std::max(hc[0], 0.0));
    if (!std::isfinite(bnorm)) {
        finish_info(0, false, std::nan(""));
        return fail(ctx, SGN_EDOMAIN, "non-finite right-hand side");
    }
    if (bnorm == 0.0) {   // x = 0 solves it exactly, whatever the guess
        hipLaunchKernelGGL(k_zero_c, dim3(flat_blocks((size_t)D * d.N)), dim3(256), 0, ctx->stream,
                           (size_t)D * d.N, (void*)u);
        CHECK_LAUNCH(ctx);
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        finish_info(0, true, 0.0);
        return SGN_OK;
    }
    const bool guess = o.x0_is_guess != 0;
    if (guess) {
        if ((s = to_S_d<D>(ctx, d, u, P.b.H, xh)) != SGN_OK) return s;
    } else {
        hipLaunchKernelGGL(k_zero_c, dim3(flat_blocks(G.nd)), dim3(256), 0, ctx->stream, G.nd, (void*)xh);
        CHECK_LAUNCH(ctx);
    }
    GmresCtl* ctl = G.g.ctl;
    SolveScal* gate = P.sc;   // its done flag gates the Arnoldi kernels and the operator passes
    double* y = G.g.hs + (size_t)(m + 1) * m + 2 * (size_t)m + (m + 1);
    hipLaunchKernelGGL(k_gmres_init, dim3(1), dim3(64), 0, ctx->stream, ctl, o.tol * bnorm, bnorm, o.max_iter);
    CHECK_LAUNCH(ctx);
    const int chunk = std::max(1, o.check_every);
    GmresCtl* hctl = reinterpret_cast<GmresCtl*>(hc);
    for (int cycle = 0;; ++cycle) {
        // true residual r = b - G x into V_0 (x = 0 on the first cycle without a guess)
        hipLaunchKernelGGL(k_gmres_open, dim3(1), dim3(64), 0, ctx->stream, (const GmresCtl*)ctl, gate);
        CHECK_LAUNCH(ctx);
        if (guess || cycle > 0) {
            if ((s = G.apply(xh)) != SGN_OK) return s;
            if ((s = G.axpby(1.0, bh, 0.0, G.Vi(0))) != SGN_OK) return s;
            if ((s = G.axpby(-1.0, qh, 1.0, G.Vi(0))) != SGN_OK) return s;
        } else {
            if ((s = G.axpby(1.0, bh, 0.0, G.Vi(0))) != SGN_OK) return s;
        }
        if ((s = G.dots(G.Vi(0), G.Vi(0), 1, G.g.coef, nullptr)) != SGN_OK) return s;
        hipLaunchKernelGGL(k_gmres_begin, dim3(1), dim3(64), 0, ctx->stream, ctl, gate, (const double*)G.g.coef,
                           G.g.hs, m);
        CHECK_LAUNCH(ctx);
        if ((s = G.scale(&ctl->scale, G.Vi(0), G.Vi(0), gate)) != SGN_OK) return s;
        // Arnoldi steps, issued check_every at a time; the state is read after each chunk
        for (int j0 = 0; j0 < m; j0 += chunk) {
            for (int j = j0; j < std::min(m, j0 + chunk); ++j) {
                if ((s = G.precond(G.Vi(j), zh, sig, alp, gate)) != SGN_OK) return s;
                if ((s = G.apply(zh)) != SGN_OK) return s;
                double* h1 = G.g.coef;
                double* h2 = G.g.coef + (m + 1);
                double* ww = G.g.coef + 2 * (m + 1);
                if ((s = G.dots(qh, G.g.V, j + 1, h1, gate)) != SGN_OK) return s;
                if ((s = G.axpy(qh, j + 1, h1, -1.0, gate)) != SGN_OK) return s;
                if ((s = G.dots(qh, G.g.V, j + 1, h2, gate)) != SGN_OK) return s;
                if ((s = G.axpy(qh, j + 1, h2, -1.0, gate)) != SGN_OK) return s;
                if ((s = G.dots(qh, qh, 1, ww, gate)) != SGN_OK) return s;
                hipLaunchKernelGGL(k_gmres_givens, dim3(1), dim3(64), 0, ctx->stream, j, m,
                                   (const double*)G.g.coef, G.g.hs, ctl, gate);
                CHECK_LAUNCH(ctx);
                if ((s = G.scale(&ctl->scale, qh, G.Vi(j + 1), gate)) != SGN_OK) return s;
            }
            HIPCHK(ctx, hipMemcpyAsync(hctl, ctl, sizeof(GmresCtl), hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(ctx, hipMemcpyAsync(hc + 64, &gate->done, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
            if ((s = wait_stream(ctx)) != SGN_OK) return s;
            if (*reinterpret_cast<const int*>(hc + 64)) break;
        }
        const GmresCtl c = *hctl;
        if (c.status == -2) {
            finish_info(c.iters, false, std::nan(""));
            return fail(ctx, SGN_EDOMAIN, "non-finite data in the residual or the Arnoldi process");
        }
        if (c.final_) break;
        // y = R^{-1} g, then x += A^{-1} (V y), over the cycle's columns
        hipLaunchKernelGGL(k_gmres_backsolve, dim3(1), dim3(64), 0, ctx->stream, m, (const GmresCtl*)ctl, G.g.hs);
        CHECK_LAUNCH(ctx);
        if ((s = G.axpby(0.0, nullptr, 0.0, zh)) != SGN_OK) return s;
        if ((s = G.axpy(zh, m, y, 1.0, nullptr, &ctl->jd)) != SGN_OK) return s;
        if ((s = G.precond(zh, qh, sig, alp, nullptr)) != SGN_OK) return s;
        if ((s = G.axpby(1.0, qh, 1.0, xh)) != SGN_OK) return s;
    }
    const GmresCtl c = *hctl;
    if ((s = from_S_d<D>(ctx, d, xh, P.b.H, u)) != SGN_OK) return s;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    finish_info(c.iters, c.conv != 0, c.relres);
    if (!c.conv) return fail(ctx, SGN_ENOCONV, "Krylov solve did not reach the tolerance");
    return SGN_OK;
}

sgn_solve_opts default_opts() {
    sgn_solve_opts o;
    std::memset(&o, 0, sizeof(o));
    o.method = SGN_PCG;
    o.precision = SGN_FP64;
    o.tol = 1e-12;
    o.max_iter = 1000;
    o.x0_is_guess = 0;
    o.gmres_restart = 30;
    o.inner_tol = 1e-5;
    o.max_outer = 20;
    o.check_every = 8;
    o.coeff_kind = SGN_COEFF_OPTIMAL;
    o.guess = SGN_GUESS_EXTRAPOLATE;
    return o;
}

sgn_status solve_1d_block(sgn_ctx* ctx, const Dims& d, double L, const double* eta, const double* gh,
                          const double* rhs, double* u, const sgn_coeffs* coeffs, int flat, const sgn_solve_opts& o,
                          sgn_solve_info* info, void* ws);

sgn_status solve_dispatch(sgn_ctx* ctx, const Dims& d, const double* eta, const double* gh, const double* rhs,
                          double* u, const sgn_coeffs* coeffs, int flat, const sgn_solve_opts& o,
                          sgn_solve_info* info, void* ws) {
    if (o.method != SGN_PCG && o.method != SGN_GMRES) return fail(ctx, SGN_EINVAL, "unknown method");
    if (!(o.tol > 0.0) || o.max_iter < 1) return fail(ctx, SGN_EINVAL, "tol must be > 0 and max_iter >= 1");
    if (ctx->wall_native && !(d.D == 2 && o.method == SGN_PCG && o.precision == SGN_FP64))
        return fail(ctx, SGN_EUNSUPPORTED, "a wall grid on its own points takes FP64 PCG only");
    if (coeffs && !(coeffs->sigma > 0.0 && coeffs->alpha > 0.0))
        return fail(ctx, SGN_EINVAL, "coefficients must be positive");
    if (o.method == SGN_GMRES) {
        if (ctx->stage) return fail(ctx, SGN_EUNSUPPORTED, "stepper solves use PCG");
        if (o.precision != SGN_FP64) return fail(ctx, SGN_EUNSUPPORTED, "GMRES runs in FP64 only");
        if (o.gmres_restart < 1 || o.gmres_restart > GMRES_MAX_RESTART)
            return fail(ctx, SGN_EINVAL, "gmres_restart must be in [1, 256]");
        return d.D == 1 ? solve_gmres<1>(ctx, d, eta, gh, rhs, u, coeffs, flat, o, info, ws)
                        : solve_gmres<2>(ctx, d, eta, gh, rhs, u, coeffs, flat, o, info, ws);
    }
    // a 1D system that fits one workgroup is solved by it in one launch
    if (d.D == 1 && d.nx <= BATCH_NMAX && (o.precision == SGN_FP64 || o.precision == SGN_MIXED))
        return solve_1d_block(ctx, d, d.Lx, eta, gh, rhs, u, coeffs, flat, o, info, ws);
    if (o.precision == SGN_FP64)
        return d.D == 1 ? solve_fp64<1>(ctx, d, eta, gh, rhs, u, coeffs, flat, o, info, ws)
                        : solve_fp64<2>(ctx, d, eta, gh, rhs, u, coeffs, flat, o, info, ws);
    if (o.precision == SGN_MIXED)
        return d.D == 1 ? solve_mixed<1>(ctx, d, eta, gh, rhs, u, coeffs, flat, o, info, ws)
                        : solve_mixed<2>(ctx, d, eta, gh, rhs, u, coeffs, flat, o, info, ws);
    return fail(ctx, SGN_EINVAL, "unknown precision");
}

// Pinned host staging of batch item tables and results (grows on demand).
sgn_status batch_staging(sgn_ctx* ctx, size_t bytes) {
    if (ctx->hbatch_bytes >= bytes) return SGN_OK;
    if (ctx->hbatch) (void)hipHostFree(ctx->hbatch);
    ctx->hbatch = nullptr;
    ctx->hbatch_bytes = 0;
    if (hipHostMalloc(&ctx->hbatch, bytes, hipHostMallocDefault) != hipSuccess)
        return fail(ctx, SGN_ENOMEM, "pinned staging allocation failed");
    ctx->hbatch_bytes = bytes;
    return SGN_OK;
}

// A 1D system of nx <= BATCH_NMAX points solved by one workgroup in one launch
// (the batched solver with a single system): workspace = item | result | region.
sgn_status solve_1d_block(sgn_ctx* ctx, const Dims& d, double L, const double* eta, const double* gh,
                          const double* rhs, double* u, const sgn_coeffs* coeffs, int flat, const sgn_solve_opts& o,
                          sgn_solve_info* info, void* ws) {
    sgn_status s;
    if ((s = batch_staging(ctx, std::max(sizeof(BatchItem), sizeof(BatchResult)))) != SGN_OK) return s;
    const int mode = o.precision == SGN_MIXED ? BATCH_MIXED : BATCH_FP64;
    BatchItem* hit = static_cast<BatchItem*>(ctx->hbatch);
    hit->n = d.nx;
    hit->index = 0;
    hit->L = L;
    hit->off = 0;
    hit->wso = 0;
    char* base = static_cast<char*>(ws);
    BatchItem* d_item = reinterpret_cast<BatchItem*>(base);
    BatchResult* d_res = reinterpret_cast<BatchResult*>(base + 256);
    double* d_data = reinterpret_cast<double*>(base + 512);
    HIPCHK(ctx, hipMemcpyAsync(d_item, hit, sizeof(BatchItem), hipMemcpyHostToDevice, ctx->stream));
    BatchParams prm{};
    prm.tol = o.tol;
    prm.inner_tol = o.inner_tol > 0 ? o.inner_tol : 1e-5;
    prm.max_iter = o.max_iter;
    prm.max_outer = o.max_outer > 0 ? o.max_outer : 20;
    prm.x0_is_guess = o.x0_is_guess ? 1 : 0;
    prm.coeff_kind = o.coeff_kind;
    prm.nitems = 1;
    prm.flat = flat < 0 ? -1 : (flat ? 1 : 0);
    if (coeffs) {
        prm.have_coeffs = 1;
        prm.sig = coeffs->sigma;
        prm.alp = coeffs->alpha;
        prm.kap = coeffs->kappa_ub;
        prm.flat = coeffs->flat ? 1 : 0;
    }
    const size_t lds = (size_t)(d.nx / 2 + 1) * sizeof(cpx<double>) * (mode == BATCH_FP64 ? 2 : 1);
    {
        ProfScope ps(ctx, SGN_KERNEL_BATCH);
        auto launch = [&](auto k, int nt) -> sgn_status {
            HIPCHK(ctx, allow_lds(k, lds));
            hipLaunchKernelGGL(k, dim3(1), dim3(nt), lds, ctx->stream, (const BatchItem*)d_item, 1, eta, gh, rhs, u,
                               d_data, ctx->tw64, ctx->tw32, prm, d_res, (int*)nullptr);
            CHECK_LAUNCH(ctx);
            return SGN_OK;
        };
        const bool mx = mode == BATCH_MIXED;
        if (d.nx <= 2048)
            s = mx ? launch(k_batch_solve<BATCH_MIXED, 256>, 256) : launch(k_batch_solve<BATCH_FP64, 256>, 256);
        else
            s = mx ? launch(k_batch_solve<BATCH_MIXED, 512>, 512) : launch(k_batch_solve<BATCH_FP64, 512>, 512);
        if (s != SGN_OK) return s;
    }
    BatchResult* hres = static_cast<BatchResult*>(ctx->hbatch);
    HIPCHK(ctx, hipMemcpyAsync(hres, d_res, sizeof(BatchResult), hipMemcpyDeviceToHost, ctx->stream));
    if ((s = wait_stream(ctx)) != SGN_OK) return s;
    const BatchResult r = *hres;
    if (info) {
        info->iters = r.iters;
        info->outer_iters = r.outer;
        info->converged = r.converged;
        info->relres = r.relres;
        info->coeffs.sigma = r.sig;
        info->coeffs.alpha = r.alp;
        info->coeffs.kappa_ub = r.kap;
        info->coeffs.flat = r.flat;
    }
    if (r.status == -2) return fail(ctx, SGN_EDOMAIN, "non-positive depth or non-finite data in the solve");
    if (!r.converged) return fail(ctx, SGN_ENOCONV, "Krylov solve did not reach the tolerance");
    return SGN_OK;
}

// physical D-vector field -> S layout (FP64)
template <int D>
sgn_status to_S_d(sgn_ctx* ctx, const Dims& d, const double* f, cpx<double>* H, cpx<double>* Sd) {
    std::vector<const double*> src;
    std::vector<cpx<double>*> hd;
    for (int c = 0; c < D; ++c) {
        src.push_back(f + c * d.N);
        hd.push_back(H + c * d.NS);
    }
    sgn_status s;
    if ((s = rows_fwd<double, double>(ctx, d, src, hd)) != SGN_OK) return s;
    ColLaunch L = col_launch<double>(d.nx, d.ny);
    auto k = k_cols_to_S<double, 4, D>;
    HIPCHK(ctx, allow_lds(k, col_lds_bytes<double>(L.g, D)));
    hipLaunchKernelGGL(k, dim3(L.g.nblocks), dim3(L.threads), col_lds_bytes<double>(L.g, D), ctx->stream, L.g, ctx->tw64,
                       (const cpx<double>*)H, d.NS, Sd);
    CHECK_LAUNCH(ctx);
    return SGN_OK;
}
// S layout -> physical D-vector field (FP64), with the 1/(nx ny) normalisation
template <int D>
sgn_status from_S_d(sgn_ctx* ctx, const Dims& d, const cpx<double>* Ssrc, cpx<double>* H, double* f) {
    ColLaunch L = col_launch<double>(d.nx, d.ny);
    auto k = k_cols_from_S<double, 4, D>;
    HIPCHK(ctx, allow_lds(k, col_lds_bytes<double>(L.g, D)));
    hipLaunchKernelGGL(k, dim3(L.g.nblocks), dim3(L.threads), col_lds_bytes<double>(L.g, D), ctx->stream, L.g, ctx->tw64, Ssrc, d.NS, H,
                       d.inv_n);
    CHECK_LAUNCH(ctx);
    std::vector<const cpx<double>*> hs;
    std::vector<double*> od;
    for (int c = 0; c < D; ++c) {
        hs.push_back(H + c * d.NS);
        od.push_back(f + c * d.N);
    }
    return rows_inv<double, double>(ctx, d, hs, od);
}

// ---------------------------------------------------------------------------
// G apply (standalone): u -> S (p_hat), C1 copy, R1, C2 store q_hat, -> physical
// ---------------------------------------------------------------------------
template <int D>
sgn_status apply_G(sgn_ctx* ctx, const Dims& d, const double* eta, const double* gh, const double* u,
                   double* out, void* ws) {
    Carve cv(ws);
    Common cm = carve_common(cv);
    PcgLaunch<double, D> P;
    P.ctx = ctx;
    P.d = d;
    P.rl = row_launch<double>(d.nx, d.ny, true);
    P.cl = pcg_col_launch<double>(d);
    P.b = carve_pcg<double>(cv, d, false);
    P.sc = cm.sc;
    P.partials = cm.partials;
    P.eta = eta;
    P.gh = gh;
    sgn_status s;
    if ((s = init_scal(ctx, P.sc, 1.0, 1, d.inv_n, nullptr)) != SGN_OK) return s;
    std::vector<const double*> usrc;
    std::vector<cpx<double>*> hdst;
    for (int c = 0; c < D; ++c) {
        usrc.push_back(u + c * d.N);
        hdst.push_back(P.b.H + c * d.NS);
    }
    if ((s = rows_fwd<double, double>(ctx, d, usrc, hdst)) != SGN_OK) return s;
    {
        auto k = P.cl.epc == 2 ? k_cols_to_S<double, 2, D> : k_cols_to_S<double, 4, D>;
        HIPCHK(ctx, allow_lds(k, col_lds_bytes<double>(P.cl.g, D)));
        hipLaunchKernelGGL(k, dim3(P.cl.g.nblocks), dim3(P.cl.threads), col_lds_bytes<double>(P.cl.g, D), ctx->stream, P.cl.g, ctx->tw64,
                           (const cpx<double>*)P.b.H, d.NS, P.b.xh);
        CHECK_LAUNCH(ctx);
    }
    if ((s = pcg_c1<double, D>(P, C1_COPY, P.b.xh)) != SGN_OK) return s;
    if ((s = pcg_r1<double, D>(P)) != SGN_OK) return s;
    if ((s = pcg_c2<double, D>(P, C2_STORE, nullptr, nullptr)) != SGN_OK) return s;
    return from_S_d<D>(ctx, d, P.b.qh, P.b.H, out);
}

// ---------------------------------------------------------------------------
// Preconditioner solve (standalone)
// ---------------------------------------------------------------------------
template <int D>
sgn_status precond_apply(sgn_ctx* ctx, const Dims& d, double sig, double alp, const double* rhs, double* out,
                         void* ws) {
    Carve cv(ws);
    carve_common(cv);
    cpx<double>* H = cv.take<cpx<double>>((size_t)D * d.NS);
    std::vector<const double*> src;
    std::vector<cpx<double>*> hd;
    std::vector<const cpx<double>*> hs;
    std::vector<double*> od;
    for (int c = 0; c < D; ++c) {
        src.push_back(rhs + c * d.N);
        hd.push_back(H + c * d.NS);
        hs.push_back(H + c * d.NS);
        od.push_back(out + c * d.N);
    }
    sgn_status s;
    if ((s = rows_fwd<double, double>(ctx, d, src, hd)) != SGN_OK) return s;
    ColLaunch L = col_launch<double>(d.nx, d.ny);
    PtrList<const cpx<double>, MAXF> a{};
    PtrList<cpx<double>, MAXF> b{};
    a.n = b.n = D;
    for (int c = 0; c < D; ++c) {
        a.p[c] = H + c * d.NS;
        b.p[c] = H + c * d.NS;
    }
    auto k = k_cols_precond<double, 4, D>;
    HIPCHK(ctx, allow_lds(k, col_lds_bytes<double>(L.g, D)));
    hipLaunchKernelGGL(k, dim3(L.g.nblocks), dim3(L.threads), col_lds_bytes<double>(L.g, D), ctx->stream, L.g, a, b, ctx->tw64, d.tpx, d.tpy,
                       sig, alp, d.inv_n);
    CHECK_LAUNCH(ctx);
    return rows_inv<double, double>(ctx, d, hs, od);
}

// ---------------------------------------------------------------------------
// Right-hand side f(w, p)  (FP64)
// ---------------------------------------------------------------------------
template <int D>
sgn_status rhs_impl(sgn_ctx* ctx, const Dims& d, const double* eta, const double* gh, const double* u,
                    double* eta_t, double* U_t, void* ws) {
    Carve cv(ws);
    carve_common(cv);
    RhsBufs b = carve_rhs(cv, d);
    const size_t N = d.N, NS = d.NS;
    // a 2D grid between walls on its own points: eta, grad h, u (and the results)
    // in transform order; only the column operators differ
    const bool wall = D == 2 && ctx->wall_native;
    cpx<double>* HA = b.H;                    // 2D + 1
    cpx<double>* HB = HA + (2 * D + 1) * NS;  // 2
    cpx<double>* OA = HB + 2 * NS;            // 2D + 2
    cpx<double>* OB = OA + (2 * D + 2) * NS;  // 2D
    sgn_status s;
    // products and forward transforms: group A = [u_c, eta u_c, eta], group B =
    // [-eta u_1 u_D, beta] (the source fields of rhs_source)
    std::vector<cpx<double>*> dA, dB;
    for (int i = 0; i < 2 * D + 1; ++i) dA.push_back(HA + i * NS);
    for (int i = 0; i < 2; ++i) dB.push_back(HB + i * NS);
    // the fused right-hand-side row passes transform their fields one at a time
    // (lockstep groups need more registers than the pointwise state leaves)
    // (the fused right-hand-side row passes keep 256-thread blocks: their pointwise
    // state makes the wide launch slower)
    const RowLaunch RL = row_launch<double>(d.nx, d.ny);
    const size_t rlds = row_lds_bytes<double>(RL.g, 1);
    {
        ProfScope ps(ctx, D == 2 ? SGN_KERNEL_RHS_ROWS_FWD : SGN_KERNEL_ROWS);
        PtrList<cpx<double>, MAXF> t{};
        t.n = 0;
        for (auto p : dA) t.p[t.n++] = p;
        for (auto p : dB) t.p[t.n++] = p;
        auto launch = [&](auto k) -> sgn_status {
            HIPCHK(ctx, allow_lds(k, rlds));
            hipLaunchKernelGGL(k, dim3(RL.g.nblocks), dim3(RL.threads), rlds, ctx->stream, RL.g, eta, u, gh, t,
                               ctx->tw64);
            CHECK_LAUNCH(ctx);
            return SGN_OK;
        };
        // the forward pass holds no pointwise state: its fields go three at a time
        const size_t l3 = row_lds_bytes<double>(RL.g, 3);
        // (wave-private forms measured slower at 1024^2: one wave per field and row
        // 47 -> 58 us, each field's wave re-reading the shared inputs; one wave per
        // row and group of fields sharing inputs 47 -> 65 us, the group's fields
        // transformed one after another in each wave)
        if (RL.epc == 4 && RL.threads <= 256 && l3 <= LDS_MULTI_MAX) {
            HIPCHK(ctx, allow_lds(k_rhs_rows_fwd<D, 4, 3, 256>, l3));
            hipLaunchKernelGGL((k_rhs_rows_fwd<D, 4, 3, 256>), dim3(RL.g.nblocks), dim3(RL.threads), l3,
                               ctx->stream, RL.g, eta, u, gh, t, ctx->tw64);
            CHECK_LAUNCH(ctx);
            s = SGN_OK;
        } else if (RL.epc == 4 && RL.threads <= 256)
            s = launch(k_rhs_rows_fwd<D, 4, 1, 256>);
        else if (RL.epc == 4)
            s = launch(k_rhs_rows_fwd<D, 4, 1, 1024>);
        else
            s = launch(k_rhs_rows_fwd<D, 8, 1, 1024>);
        if (s != SGN_OK) return s;
    }
    std::vector<const cpx<double>*> cA(dA.begin(), dA.end()), cB(dB.begin(), dB.end());
    std::vector<cpx<double>*> oA, oB;
    for (int i = 0; i < 2 * D + 2; ++i) oA.push_back(OA + i * NS);
    for (int i = 0; i < 2 * D; ++i) oB.push_back(OB + i * NS);
    // codes: 1 id, 2 ikx, 3 iky, 4 (ikx)^2, 5 (ikx)(iky), 6 (iky)^2
    // Periodic rows of 1024 points: the inverse row pass (k_rhs_rows_inv_w) forms
    // the x-derivatives of delta, eta and beta itself (i k_x times a row spectrum
    // it loads anyway), so the column pass skips those three outputs.
    const bool dx_rows = D == 2 && !wall && wave_rows(d);
    if (D == 2) {
        // the column operators, split by shared inputs so that each block holds
        // at most three transformed inputs in registers, run side by side in one
        // launch: [u, v] -> [delta, dx delta, dy delta]; [eu, ev, eta] -> [m, dx eta,
        // dy eta]; [beta] -> [dx beta, dy beta]
        // between walls (fields in transform order) the kinds: u sine along x (1),
        // v sine along y (2), scalars cosine (0), u v sine along both (3)
        std::vector<LinJobSpec> jobs = {
            {{cA[0], cA[1]}, {oA[0], oA[1], oA[2]}, {{2, 3}, {4, 5}, {5, 6}}, {1, 2}, {0, 1, 2}},
            {{cA[2], cA[3], cA[4]}, {oA[3], oA[4], oA[5]}, {{2, 3, 0}, {0, 0, 2}, {0, 0, 3}}, {1, 2, 0}, {0, 1, 2}},
            {{cB[1]}, {oB[0], oB[1]}, {{2}, {3}}, {0}, {1, 2}},
        };
        if (dx_rows) {
            // d_x delta, d_x eta and d_x beta are formed by the inverse row pass
            // from delta's output and the row spectra of eta and beta
            jobs = {{{cA[0], cA[1]}, {oA[0], oA[2]}, {{2, 3}, {5, 6}}, {1, 2}, {0, 2}},
                    {{cA[2], cA[3], cA[4]}, {oA[3], oA[5]}, {{2, 3, 0}, {0, 0, 3}}, {1, 2, 0}, {0, 2}},
                    {{cB[1]}, {oB[1]}, {{3}}, {0}, {2}}};
        }
        if ((s = cols_lin_jobs(ctx, d, jobs, d.inv_n, SGN_KERNEL_RHS_COLS, wall)) != SGN_OK) return s;
    } else {
        if ((s = cols_lin<double>(ctx, d, cA, oA, {{2, 0, 0}, {4, 0, 0}, {0, 2, 0}, {0, 0, 2}}, d.inv_n)) != SGN_OK)
            return s;
        if ((s = cols_lin<double>(ctx, d, {cB[1]}, {oB[0]}, {{2}}, d.inv_n)) != SGN_OK) return s;
    }
    // back to physical: Q = [m, delta, d delta (D), d eta (D), d beta (D)], consumed
    // pointwise into eta_t, U_t (without grad S - div(eta u (x) u)) and S, whose row
    // transform goes to HA (slot 0; in 2D S_x = S - eta u_x^2 there and S_y =
    // S - eta u_y^2 in slot 1, the inputs of the column pass in slots 0 and 1
    // having been consumed)
    {
        ProfScope ps(ctx, D == 2 ? SGN_KERNEL_RHS_ROWS_INV : SGN_KERNEL_ROWS);
        PtrList<const cpx<double>, MAXF> q{};
        q.n = 0;
        // OA = [delta, d delta (D), m, d eta (D)], OB = [d beta (D)]
        q.p[q.n++] = OA + (1 + D) * NS;
        for (int i = 0; i <= D; ++i) q.p[q.n++] = OA + i * NS;
        for (int i = 0; i < D; ++i) q.p[q.n++] = OA + (2 + D + i) * NS;
        for (int i = 0; i < D; ++i) q.p[q.n++] = OB + i * NS;
        auto launch = [&](auto k) -> sgn_status {
            HIPCHK(ctx, allow_lds(k, rlds));
            hipLaunchKernelGGL(k, dim3(RL.g.nblocks), dim3(RL.threads), rlds, ctx->stream, RL.g, q, eta, u, gh, eta_t,
                               U_t, HA, D == 2 ? HA + NS : nullptr, ctx->tw64, 1.0);
            CHECK_LAUNCH(ctx);
            return SGN_OK;
        };
        if (D == 2 && wave_rows(d) && q.n == 8) {
            RowDx dx{};
            if (dx_rows) {
                q.p[2] = OA;                       // delta's output: d_x delta = i k_x delta
                q.p[4] = HA + 2 * D * NS;          // eta's row spectrum
                q.p[6] = HB + NS;                  // beta's row spectrum
                dx.f[2] = 1.0;
                dx.f[4] = dx.f[6] = 1.0 / d.nx;
            }
            hipLaunchKernelGGL(k_rhs_rows_inv_w, dim3(d.ny), dim3(512), 0, ctx->stream, d.ny, q, eta, u, gh, eta_t,
                               U_t, HA, HA + NS, ctx->tw64, 1.0, dx, d.tpx);
            CHECK_LAUNCH(ctx);
            s = SGN_OK;
        } else if (RL.epc == 4 && RL.threads <= 256)
            s = launch(k_rhs_rows_inv<D, 4, 1, 256>);
        else if (RL.epc == 4)
            s = launch(k_rhs_rows_inv<D, 4, 1, 1024>);
        else
            s = launch(k_rhs_rows_inv<D, 8, 1, 1024>);
        if (s != SGN_OK) return s;
    }
    // U_t += grad S - div(eta u (x) u), formed in the spectral domain from S and the
    // (negated) row-transformed flux fields in HB, into OA (free again)
    std::vector<cpx<double>*> gS;
    for (int c = 0; c < D; ++c) gS.push_back(OA + c * NS);
    if (D == 2) {
        // (U_t)_x += d_x S_x + d_y (-eta u_x u_y), (U_t)_y += d_x (-eta u_x u_y) +
        // d_y S_y: three transformed inputs, two outputs, one job
        std::vector<LinJobSpec> fj = {
            {{HA, cB[0], HA + NS}, {gS[0], gS[1]}, {{2, 3, 0}, {0, 2, 3}}, {0, 3, 0}, {1, 2}}};
        if ((s = cols_lin_jobs(ctx, d, fj, d.inv_n, SGN_KERNEL_RHS_FLUX, wall)) != SGN_OK) return s;
    } else {
        if ((s = cols_lin<double>(ctx, d, {HA, cB[0]}, gS, {{2, 2}}, d.inv_n)) != SGN_OK) return s;
    }
    std::vector<const cpx<double>*> gs2(gS.begin(), gS.end());
    std::vector<double*> ud;
    for (int c = 0; c < D; ++c) ud.push_back(U_t + c * N);
    return rows_inv<double, double>(ctx, d, gs2, ud, 1.0, 1.0);
}


// A 1D right-hand side of up to BATCH_NMAX points by one workgroup in one launch.
sgn_status rhs_1d_block(sgn_ctx* ctx, const Dims& d, const double* eta, const double* gh, const double* u,
                        double* eta_t, double* U_t, void* ws) {
    Carve cv(ws);
    carve_common(cv);
    const int M1 = d.nx / 2 + 1;
    cpx<double>* spec = cv.take<cpx<double>>((size_t)5 * M1);
    double* st = cv.take<double>((size_t)5 * d.nx);
    const size_t lds = (size_t)M1 * sizeof(cpx<double>);
    ProfScope ps(ctx, SGN_KERNEL_ROWS);
    auto launch = [&](auto k, int nt) -> sgn_status {
        HIPCHK(ctx, allow_lds(k, lds));
        hipLaunchKernelGGL(k, dim3(1), dim3(nt), lds, ctx->stream, d.nx, d.Lx, eta, gh, u, eta_t, U_t, spec, st,
                           ctx->tw64);
        CHECK_LAUNCH(ctx);
        return SGN_OK;
    };
    return d.nx <= 2048 ? launch(k_rhs_1d<256>, 256) : launch(k_rhs_1d<512>, 512);
}

sgn_status rhs_dispatch(sgn_ctx* ctx, const Dims& d, const double* eta, const double* gh, const double* u,
                        double* eta_t, double* U_t, void* ws) {
    if (d.D == 1 && d.nx <= BATCH_NMAX) return rhs_1d_block(ctx, d, eta, gh, u, eta_t, U_t, ws);
    return d.D == 1 ? rhs_impl<1>(ctx, d, eta, gh, u, eta_t, U_t, ws) : rhs_impl<2>(ctx, d, eta, gh, u, eta_t, U_t, ws);
}

// ---------------------------------------------------------------------------
// De-aliased right-hand side (subsec:dswe_1d, remark on aliasing after Test 2):
// eta, u and grad h are interpolated onto the grid twice as fine per axis by
// zero-padding their spectra, f(w, p) is formed there by the same kernels, and
// eta_t, U_t are truncated back to the modes of the original grid.  Both
// transfers keep the modes |m| < n/2 of the original grid (its Nyquist modes,
// to which D gives no wavenumber, are dropped), so padding grad h equals
// differentiating the padded h.
// ---------------------------------------------------------------------------
constexpr int DEALIAS_FACTOR = 2;
constexpr int DEALIAS_MAX_1D = 8192;                       // padded: 16384
constexpr int DEALIAS_MAX_NX = 2048, DEALIAS_MAX_NY = 1024; // padded: 4096 x 2048

bool dealias_supported(const Dims& d) {
    return d.D == 1 ? d.nx <= DEALIAS_MAX_1D : (d.nx <= DEALIAS_MAX_NX && d.ny <= DEALIAS_MAX_NY);
}

Dims fine_dims(const Dims& d) {
    Dims f = d;
    f.nx = d.nx * DEALIAS_FACTOR;
    f.ny = d.D == 2 ? d.ny * DEALIAS_FACTOR : 1;
    f.N = (size_t)f.nx * f.ny;
    f.NS = (size_t)(f.nx / 2 + 1) * f.ny;
    f.inv_n = 1.0 / (double)f.N;
    return f;
}

size_t rhs_workspace_bytes(const Dims& d) {
    Carve cv(nullptr);
    carve_common(cv);
    if (d.D == 1 && d.nx <= BATCH_NMAX) {
        cv.take<cpx<double>>((size_t)5 * (d.nx / 2 + 1));
        cv.take<double>((size_t)5 * d.nx);
    } else {
        carve_rhs(cv, d);
    }
    return cv.off + 256;
}

struct DealiasBufs {
    double *eta_f, *u_f, *gh_f, *et_f, *Ut_f;  // fields on the padded grid
    cpx<double>*Hf, *Sf, *Hc, *Sc;              // transfer spectra (1 + D fields each)
    void* ws_f;                                 // the padded grid's right-hand-side workspace
};
size_t carve_dealias(Carve& cv, const Dims& d, DealiasBufs* b) {
    const Dims f = fine_dims(d);
    const size_t nf = (size_t)(1 + d.D);
    DealiasBufs t;
    t.eta_f = cv.take<double>(nf * f.N);   // eta_f, u_f adjacent (padded as one group)
    t.u_f = t.eta_f ? t.eta_f + f.N : nullptr;
    t.gh_f = cv.take<double>((size_t)d.D * f.N);
    t.et_f = cv.take<double>(nf * f.N);    // et_f, Ut_f adjacent (truncated as one group)
    t.Ut_f = t.et_f ? t.et_f + f.N : nullptr;
    t.Hf = cv.take<cpx<double>>(nf * f.NS);
    t.Sf = cv.take<cpx<double>>(nf * f.NS);
    t.Hc = cv.take<cpx<double>>(nf * d.NS);
    t.Sc = cv.take<cpx<double>>(nf * d.NS);
    t.ws_f = cv.take<unsigned char>(rhs_workspace_bytes(f));
    if (b) *b = t;
    return cv.off;
}

// y-FFT of nf H fields (stride NS) into S fields, columns of the grid d.
template <int NF>
sgn_status cols_to_S_n(sgn_ctx* ctx, const Dims& d, const cpx<double>* H, cpx<double>* S) {
    ProfScope ps(ctx, SGN_KERNEL_COLS);
    const int epc = col_epc(d.ny);
    const ColLaunch L = col_launch<double>(d.nx, d.ny, epc);
    const size_t lds = col_lds_bytes<double>(L.g, NF);
    auto launch = [&](auto k) -> sgn_status {
        HIPCHK(ctx, allow_lds(k, lds));
        hipLaunchKernelGGL(k, dim3(L.g.nblocks), dim3(L.threads), lds, ctx->stream, L.g, ctx->tw64, H, d.NS, S);
        CHECK_LAUNCH(ctx);
        return SGN_OK;
    };
    return epc == 8 ? launch(k_cols_to_S<double, 8, NF>) : launch(k_cols_to_S<double, 4, NF>);
}

template <int NF>
sgn_status cols_resample_n(sgn_ctx* ctx, const Dims& s, const Dims& t, const cpx<double>* S, cpx<double>* Ht) {
    ProfScope ps(ctx, SGN_KERNEL_COLS);
    const int epc = col_epc(t.ny);
    const ColLaunch L = col_launch<double>(t.nx, t.ny, epc);
    const size_t lds = col_lds_bytes<double>(L.g, NF);
    PtrList<const cpx<double>, MAXF> src{};
    PtrList<cpx<double>, MAXF> dst{};
    src.n = dst.n = NF;
    for (int f = 0; f < NF; ++f) {
        src.p[f] = S + f * s.NS;
        dst.p[f] = Ht + f * t.NS;
    }
    const int kx_keep = std::min(s.nx, t.nx) / 2;
    const int m_keep = s.D == 1 ? 1 : std::min(s.ny, t.ny) / 2;
    auto launch = [&](auto k) -> sgn_status {
        HIPCHK(ctx, allow_lds(k, lds));
        hipLaunchKernelGGL(k, dim3(L.g.nblocks), dim3(L.threads), lds, ctx->stream, L.g, ctx->tw64, src, s.ny, dst,
                           kx_keep, m_keep, s.inv_n);
        CHECK_LAUNCH(ctx);
        return SGN_OK;
    };
    return epc == 8 ? launch(k_cols_resample<double, 8, NF>) : launch(k_cols_resample<double, 4, NF>);
}

// Spectral resampling of nf physical fields (stride s.N) from grid s to grid t
// (same domain, same dimension): rows forward on s, y-FFT on s (2D), mode
// transfer with the inverse y-FFT on t, rows inverse on t.
sgn_status resample_fields(sgn_ctx* ctx, const Dims& s, const Dims& t, const double* src, int nf, double* dst,
                           cpx<double>* Hs, cpx<double>* Ss, cpx<double>* Ht) {
    if (nf < 1 || nf > 3) return fail(ctx, SGN_EINVAL, "resample: 1 to 3 fields");
    std::vector<const double*> a;
    std::vector<cpx<double>*> h;
    std::vector<const cpx<double>*> ht;
    std::vector<double*> o;
    for (int f = 0; f < nf; ++f) {
        a.push_back(src + f * s.N);
        h.push_back(Hs + f * s.NS);
        ht.push_back(Ht + f * t.NS);
        o.push_back(dst + f * t.N);
    }
    sgn_status st;
    if ((st = rows_fwd<double, double>(ctx, s, a, h)) != SGN_OK) return st;
    const cpx<double>* S = Hs;   // 1D: the column transform is the identity
    if (s.D == 2) {
        st = nf == 1 ? cols_to_S_n<1>(ctx, s, Hs, Ss) : nf == 2 ? cols_to_S_n<2>(ctx, s, Hs, Ss)
                                                           : cols_to_S_n<3>(ctx, s, Hs, Ss);
        if (st != SGN_OK) return st;
        S = Ss;
    }
    st = nf == 1 ? cols_resample_n<1>(ctx, s, t, S, Ht) : nf == 2 ? cols_resample_n<2>(ctx, s, t, S, Ht)
                                                             : cols_resample_n<3>(ctx, s, t, S, Ht);
    if (st != SGN_OK) return st;
    return rows_inv<double, double>(ctx, t, ht, o);
}

// grad h on the padded grid (once per bathymetry).
sgn_status dealias_pad_gh(sgn_ctx* ctx, const Dims& d, const double* gh, const DealiasBufs& b) {
    return resample_fields(ctx, d, fine_dims(d), gh, d.D, b.gh_f, b.Hc, b.Sc, b.Hf);
}

// (eta_t, U_t) on grid d from eta, u on d and grad h already on the padded grid.
sgn_status rhs_dealiased(sgn_ctx* ctx, const Dims& d, const double* eta, const double* u, double* eta_t,
                         double* U_t, const DealiasBufs& b) {
    const Dims f = fine_dims(d);
    sgn_status s;
    // eta and u are adjacent on the padded grid only: pad them as one group when
    // they are adjacent on the original grid as well
    if (u == eta + d.N) {
        if ((s = resample_fields(ctx, d, f, eta, 1 + d.D, b.eta_f, b.Hc, b.Sc, b.Hf)) != SGN_OK) return s;
    } else {
        if ((s = resample_fields(ctx, d, f, eta, 1, b.eta_f, b.Hc, b.Sc, b.Hf)) != SGN_OK) return s;
        if ((s = resample_fields(ctx, d, f, u, d.D, b.u_f, b.Hc, b.Sc, b.Hf)) != SGN_OK) return s;
    }
    if ((s = rhs_dispatch(ctx, f, b.eta_f, b.gh_f, b.u_f, b.et_f, b.Ut_f, b.ws_f)) != SGN_OK) return s;
    if (U_t == eta_t + d.N) return resample_fields(ctx, f, d, b.et_f, 1 + d.D, eta_t, b.Hf, b.Sf, b.Hc);
    if ((s = resample_fields(ctx, f, d, b.et_f, 1, eta_t, b.Hf, b.Sf, b.Hc)) != SGN_OK) return s;
    return resample_fields(ctx, f, d, b.Ut_f, d.D, U_t, b.Hf, b.Sf, b.Hc);
}


// ---------------------------------------------------------------------------
// Grids between walls (homogeneous Neumann, Subsec:DAEform): the cosine / sine
// series of a cell-centred wall grid are the Fourier series of the fields
// reflected evenly (scalars) or oddly (each velocity component along its own
// axis) onto the periodic grid of twice the length per axis, and G, A^{-1} and
// the Krylov iteration preserve that symmetry.  A call on a wall grid reflects
// its inputs onto the twin, runs the periodic path there, and restricts the
// result to the first quadrant.  Dot products over the twin are twice those
// over the wall grid, so every ratio the iteration forms is unchanged.
// ---------------------------------------------------------------------------
struct WallBufs {
    double *eta, *et, *gh, *f, *u;  // on the twin: eta, eta_t [N], grad h [D N], input [D N], result [D N]
    void* ws;                       // the twin's own workspace
};
size_t carve_walls(Carve& cv, const Dims& t, WallBufs* b) {
    WallBufs w;
    w.eta = cv.take<double>(t.N);
    w.et = cv.take<double>(t.N);
    w.gh = cv.take<double>((size_t)t.D * t.N);
    w.f = cv.take<double>((size_t)t.D * t.N);
    w.u = cv.take<double>((size_t)t.D * t.N);
    cv.off = align_up(cv.off, 256);
    w.ws = cv.base ? cv.base + cv.off : nullptr;
    if (b) *b = w;
    return cv.off;
}

sgn_status wall_reflect(sgn_ctx* ctx, const Dims& d, const double* src, double* dst, bool vector) {
    const Dims t = twin_dims(d);
    const int nf = vector ? d.D : 1;
    const unsigned oddx = vector ? 1u : 0u, oddy = (vector && d.D == 2) ? 2u : 0u;
    hipLaunchKernelGGL(k_reflect, dim3(flat_blocks(t.N * nf)), dim3(256), 0, ctx->stream, d.nx, d.ny, t.ny, src,
                       d.N, dst, t.N, nf, oddx, oddy);
    CHECK_LAUNCH(ctx);
    return SGN_OK;
}

// The symmetric part of a twin field back on the wall grid: a scalar (vector =
// false) or the D components of a vector field.
sgn_status wall_restrict(sgn_ctx* ctx, const Dims& d, const double* src, double* dst, bool vector = true) {
    const Dims t = twin_dims(d);
    const int nf = vector ? d.D : 1;
    const unsigned oddx = vector ? 1u : 0u, oddy = (vector && d.D == 2) ? 2u : 0u;
    hipLaunchKernelGGL(k_restrict, dim3(flat_blocks(d.N * nf)), dim3(256), 0, ctx->stream, d.nx, d.ny, t.ny, src,
                       t.N, dst, d.N, nf, oddx, oddy);
    CHECK_LAUNCH(ctx);
    return SGN_OK;
}

// A stepping state between walls keeps its fields' reflections on the twin, and a
// periodic state over them: h, grad h once; eta, U, u at every stepping call.
struct WallStateBufs {
    double *h, *gh, *eta, *U, *u;
};
size_t carve_wall_state(Carve& cv, const Dims& t, WallStateBufs* b) {
    WallStateBufs w;
    const size_t DN = (size_t)t.D * t.N;
    w.h = cv.take<double>(t.N);
    w.gh = cv.take<double>(DN);
    w.eta = cv.take<double>(t.N);
    w.U = cv.take<double>(DN);
    w.u = cv.take<double>(DN);
    if (b) *b = w;
    return cv.off;
}

// ---------------------------------------------------------------------------
// Time-stepping state (section 5)
// ---------------------------------------------------------------------------
struct StateBufs {
    double* rk_fe[4];   // RK4 stage right-hand sides
    double* rk_fU[4];
    double* ab_fe[4];   // Adams-Bashforth history ring
    double* ab_fU[4];
    double *eta_s, *U_s, *u_s;              // RK4 stage values
    // linearly implicit history: levels n .. n+s-2 (s <= 3) in a ring of two slots
    double *lv_eta[2], *lv_U[2], *lv_fe[2], *lv_fU[2], *tmp_e, *tmp_U;
    cpx<double>*lv_R[2], *lv_uh[2];
    cpx<double>*R_cur, *uh, *Uh, *Hs;   // the current level's R and u (spectral), U and row scratch
    double* gx_off[GUESS_SLOTS][2];  // recorded offsets of each stepper slot (ring of two)
    double* gx_base;                 // base velocity of the running solve
};

size_t carve_state(Carve& cv, const Dims& d, StateBufs* b) {
    const size_t N = d.N, DN = (size_t)d.D * d.N, DS = (size_t)d.D * d.NS;
    StateBufs t;
    for (int k = 0; k < 4; ++k) {
        t.rk_fe[k] = cv.take<double>(N);
        t.rk_fU[k] = cv.take<double>(DN);
        t.ab_fe[k] = cv.take<double>(N);
        t.ab_fU[k] = cv.take<double>(DN);
    }
    t.eta_s = cv.take<double>(N);
    t.U_s = cv.take<double>(DN);
    t.u_s = cv.take<double>(DN);
    for (int k = 0; k < 2; ++k) {
        t.lv_eta[k] = cv.take<double>(N);
        t.lv_U[k] = cv.take<double>(DN);
        t.lv_fe[k] = cv.take<double>(N);
        t.lv_fU[k] = cv.take<double>(DN);
        t.lv_R[k] = cv.take<cpx<double>>(DS);
        t.lv_uh[k] = cv.take<cpx<double>>(DS);
    }
    t.tmp_e = cv.take<double>(N);
    t.tmp_U = cv.take<double>(DN);
    t.R_cur = cv.take<cpx<double>>(DS);
    t.uh = cv.take<cpx<double>>(DS);
    t.Uh = cv.take<cpx<double>>(DS);
    t.Hs = cv.take<cpx<double>>((size_t)(d.D + 1) * d.NS);
    for (int k = 0; k < GUESS_SLOTS; ++k)
        for (int l = 0; l < 2; ++l) t.gx_off[k][l] = cv.take<double>(DN);
    t.gx_base = cv.take<double>(DN);
    if (b) *b = t;
    return cv.off;
}

}  // namespace

struct sgn_state {
    sgn_ctx* ctx;
    sgn_grid grid;
    Dims d;
    const double* h;
    const double* gh;
    int flat;
    double *eta, *U, *u;
    void* ws;
    StateBufs b;
    double t;
    int64_t steps;
    int kind;       // history held: 0 none, 1 Adams-Bashforth, 2 linearly implicit
    int ab_order;
    int ab_count;   // levels of f stored
    int ab_head;    // next ring slot
    double hist_dt;
    // linearly implicit history: the scheme (steps and the parameter r of the
    // third-order family; r < 0 for SBDF2), A = (sb_sig I - sb_alp grad div) with
    // the scale theta already applied, the caller's fixed coefficients (0 if none),
    // levels recorded in the ring and its oldest slot
    int lm_s = 0;
    double lm_r = -1.0, lm_theta = 1.0;
    double sb_sig, sb_alp;
    double lm_fix_sig = 0.0, lm_fix_alp = 0.0;
    int lm_count = 0, lm_head = 0;
    // initial-guess history: offsets recorded per slot, newest in gx_head
    int gx_mode;
    double gx_dt;
    int gx_count[GUESS_SLOTS];
    int gx_head[GUESS_SLOTS];
    // iterations of the previous solve of each slot (FP64 / FP32 loop): the first
    // chunk of the next one, kept with the state so that a run's launches (and with
    // them its results) do not depend on what else its context solved before
    int last_iters[GUESS_SLOTS][2] = {};
    // de-aliased right-hand side (sgn_state_set_dealias): buffers in the caller's workspace
    int dealias = 0;
    DealiasBufs dl{};
    // between walls: the periodic state on the twin, and (2D) the state on the
    // grid's own points with its fields in transform order, which FP64 PCG calls
    // of RK4 and Adams-Bashforth take; path: the sub-state of the last call (0
    // none, 1 twin, 2 own points)
    sgn_state* twin = nullptr;
    WallStateBufs wb{};
    sgn_state* nat = nullptr;
    WallStateBufs nb{};
    int path = 0;
    ~sgn_state() {
        delete twin;
        delete nat;
    }
};

namespace {

// f(w, p) of a state: the plain or the de-aliased form.
sgn_status state_rhs(sgn_state* st, const double* eta, const double* u, double* fe, double* fU) {
    if (st->dealias) return rhs_dealiased(st->ctx, st->d, eta, u, fe, fU, st->dl);
    return rhs_dispatch(st->ctx, st->d, eta, st->gh, u, fe, fU, st->ws);
}

sgn_status copy_d(sgn_ctx* ctx, double* dst, const double* src, size_t n) {
    HIPCHK(ctx, hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    return SGN_OK;
}

// out = (base + dt * sum_k c_k f_k) / div (base may be null)
sgn_status lincomb(sgn_ctx* ctx, size_t n, const double* base, double dt, std::vector<const double*> f,
                   std::vector<double> c, double* out, double div = 1.0) {
    Lincomb4 lc{};
    if (f.size() > (size_t)LINCOMB_MAX || f.size() != c.size()) return fail(ctx, SGN_EINVAL, "lincomb: terms");
    lc.div = div;
    lc.n = (int)f.size();
    for (int k = 0; k < lc.n; ++k) {
        lc.f[k] = f[k];
        lc.c[k] = c[k];
    }
    hipLaunchKernelGGL(k_lincomb, dim3(flat_blocks(n)), dim3(256), 0, ctx->stream, n, base, dt, lc, out);
    CHECK_LAUNCH(ctx);
    return SGN_OK;
}

// Independent linear combinations in one launch (k_lincomb_jobs).
struct LcSpec {
    double* out;
    const double* base;
    double dt;
    std::vector<const double*> f;
    std::vector<double> c;
    size_t n;
    double* save;
};
sgn_status lincomb_jobs(sgn_ctx* ctx, const std::vector<LcSpec>& spec) {
    LcJobs J{};
    J.n = (int)spec.size();
    if (J.n < 1 || J.n > 3) return fail(ctx, SGN_EINVAL, "lincomb_jobs: job count");
    size_t nmax = 0;
    for (int k = 0; k < J.n; ++k) {
        const LcSpec& s = spec[k];
        LcJob& j = J.j[k];
        if (s.f.size() > 4 || s.f.size() != s.c.size()) return fail(ctx, SGN_EINVAL, "lincomb_jobs: terms");
        j.out = s.out;
        j.base = s.base;
        j.save = s.save;
        j.dt = s.dt;
        j.nf = (int)s.f.size();
        j.n = s.n;
        for (int q = 0; q < j.nf; ++q) {
            j.f[q] = s.f[q];
            j.c[q] = s.c[q];
        }
        nmax = std::max(nmax, s.n);
    }
    hipLaunchKernelGGL(k_lincomb_jobs, dim3(flat_blocks(nmax)), dim3(256), 0, ctx->stream, J);
    CHECK_LAUNCH(ctx);
    return SGN_OK;
}

// Start of a stepping call: the guess history holds offsets for this dt and mode.
void guess_prepare(sgn_state* st, const sgn_solve_opts& o, double dt) {
    if (st->gx_mode != o.guess || st->gx_dt != dt) {
        st->gx_mode = o.guess;
        st->gx_dt = dt;
        for (int k = 0; k < GUESS_SLOTS; ++k) st->gx_count[k] = 0;
    }
}

void account(sgn_step_info* acc, const sgn_solve_info& si) {
    acc->solves += 1;
    acc->iters += si.iters;
    if (si.iters > acc->max_iters) acc->max_iters = si.iters;
    if (!si.converged) acc->converged = 0;
}

// G_{eta,h} u = U for stepper slot `slot`; u holds the base velocity on entry.
// With extrapolated guesses the solve starts from base + o_{n-1} or
// base + 2 o_{n-1} - o_{n-2} and records o_n = u - base afterwards.  A is
// built from the current eta.
sgn_status stage_solve(sgn_state* st, int slot, const double* eta, const double* U, double* u,
                       const sgn_solve_opts& o, sgn_step_info* acc) {
    sgn_ctx* ctx = st->ctx;
    StateBufs& b = st->b;
    const size_t DN = (size_t)st->d.D * st->d.N;
    const bool ex = o.guess == SGN_GUESS_EXTRAPOLATE;
    // PCG on the row/column path (FP64 and mixed) forms the guess and records the
    // offset inside its first and last passes; the one-workgroup 1D solve does
    // both with separate passes
    const bool fused = ex && (o.precision == SGN_FP64 || o.precision == SGN_MIXED) && o.method == SGN_PCG &&
                       !(st->d.D == 1 && st->d.nx <= BATCH_NMAX);
    sgn_status s;
    int& cnt = st->gx_count[slot];
    int& head = st->gx_head[slot];
    const int nh = cnt == 0 ? head : head ^ 1;
    if (fused) {
        ctx->gx_a = cnt >= 1 ? b.gx_off[slot][head] : nullptr;
        ctx->gx_b = cnt >= 2 ? b.gx_off[slot][head ^ 1] : nullptr;
        ctx->gx_c1 = cnt >= 2 ? 2.0 : 1.0;
        ctx->gx_c2 = -1.0;
        ctx->gx_off = b.gx_off[slot][nh];
    } else if (ex) {
        // keep the base and form the guess in place, in one pass
        if (cnt == 0) {
            if ((s = copy_d(ctx, b.gx_base, u, DN)) != SGN_OK) return s;
        } else if (cnt == 1) {
            if ((s = lincomb_jobs(ctx, {{u, u, 1.0, {b.gx_off[slot][head]}, {1.0}, DN, b.gx_base}})) != SGN_OK)
                return s;
        } else {
            if ((s = lincomb_jobs(ctx, {{u, u, 1.0, {b.gx_off[slot][head], b.gx_off[slot][head ^ 1]}, {2.0, -1.0},
                                         DN, b.gx_base}})) != SGN_OK)
                return s;
        }
    }
    sgn_solve_opts so = o;
    so.x0_is_guess = 1;
    sgn_solve_info si;
    std::memset(&si, 0, sizeof(si));
    ctx->stage = true;
    ctx->slot = slot;
    ctx->stage_last = st->last_iters[slot];
    s = solve_dispatch(ctx, st->d, eta, st->gh, U, u, nullptr, st->flat, so, &si, st->ws);
    ctx->stage = false;
    ctx->slot = GUESS_SLOTS;
    ctx->stage_last = nullptr;
    ctx->gx_a = ctx->gx_b = nullptr;
    ctx->gx_off = nullptr;
    account(acc, si);
    if (s != SGN_OK) {
        if (fused) cnt = 0;   // the offset ring may hold a partial record
        return s;
    }
    if (ex) {
        if (!fused && (s = lincomb(ctx, DN, u, 1.0, {b.gx_base}, {-1.0}, b.gx_off[slot][nh])) != SGN_OK) return s;
        head = nh;
        if (cnt < 2) cnt += 1;
    }
    return SGN_OK;
}

// One RK4 step (Eq:ERK): stage i uses eta_n + dt a_i f^(i-1), U_n + dt a_i f^(i-1),
// solves G u^(i) = U^(i) from u^(i-1); the final combination advances eta and U
// and u_{n+1} is solved from u^(4).  have_f1: f at the current level is already
// in rk_fe[0], rk_fU[0].
sgn_status rk4_one(sgn_state* st, double dt, const sgn_solve_opts& o, sgn_step_info* acc, bool have_f1) {
    sgn_ctx* ctx = st->ctx;
    const Dims& d = st->d;
    StateBufs& b = st->b;
    const size_t N = d.N, DN = (size_t)d.D * d.N;
    static const double a[3] = {0.5, 0.5, 1.0};
    static const double w[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    sgn_status s;
    if (!have_f1 && (s = state_rhs(st, st->eta, st->u, b.rk_fe[0], b.rk_fU[0])) != SGN_OK)
        return s;
    if ((s = copy_d(ctx, b.u_s, st->u, DN)) != SGN_OK) return s;
    for (int i = 1; i < 4; ++i) {
        if ((s = lincomb_jobs(ctx, {{b.eta_s, st->eta, dt, {b.rk_fe[i - 1]}, {a[i - 1]}, N, nullptr},
                                    {b.U_s, st->U, dt, {b.rk_fU[i - 1]}, {a[i - 1]}, DN, nullptr}})) != SGN_OK)
            return s;
        if ((s = stage_solve(st, GUESS_RK2 + i - 1, b.eta_s, b.U_s, b.u_s, o, acc)) != SGN_OK) return s;
        if ((s = state_rhs(st, b.eta_s, b.u_s, b.rk_fe[i], b.rk_fU[i])) != SGN_OK) return s;
    }
    if ((s = lincomb_jobs(ctx, {{st->eta, st->eta, dt, {b.rk_fe[0], b.rk_fe[1], b.rk_fe[2], b.rk_fe[3]},
                                 {w[0], w[1], w[2], w[3]}, N, nullptr},
                                {st->U, st->U, dt, {b.rk_fU[0], b.rk_fU[1], b.rk_fU[2], b.rk_fU[3]},
                                 {w[0], w[1], w[2], w[3]}, DN, nullptr}})) != SGN_OK)
        return s;
    if ((s = copy_d(ctx, st->u, b.u_s, DN)) != SGN_OK) return s;
    // eta and U now hold level n+1: the step counts even if its final solve fails
    // (u then holds that solve's last iterate), so that t and steps_done always
    // describe eta and U and a retry does not advance them twice
    s = stage_solve(st, GUESS_RK_FINAL, st->eta, st->U, st->u, o, acc);
    if (s == SGN_OK || s == SGN_ENOCONV || s == SGN_EDOMAIN) {
        st->t += dt;
        st->steps += 1;
    }
    return s;
}

// R_hat = A u_hat - G_{eta,h} u_hat + U_hat at the state's level (u_hat in b.uh).
template <int D>
__global__ void k_sbdf2_R(int nx, int ny, size_t NS, double tpx, double tpy, double sig, double alp,
                          const cpx<double>* __restrict__ uh, const cpx<double>* __restrict__ Guh,
                          const cpx<double>* __restrict__ Uh, cpx<double>* __restrict__ R) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < NS; idx += stride) {
        const int kxi = (int)(idx / ny), kyi = (int)(idx - (size_t)kxi * ny);
        const double kx = wavenumber<double>(kxi, nx, tpx);
        const double ky = D == 2 ? wavenumber<double>(kyi, ny, tpy) : 0.0;
        cpx<double> uu[D];
        for (int c = 0; c < D; ++c) uu[c] = uh[c * NS + idx];
        cpx<double> ku = kx * uu[0];
        if (D == 2) ku = ku + ky * uu[1 % D];
        for (int c = 0; c < D; ++c) {
            const double kc = c == 0 ? kx : ky;
            const cpx<double> Au = sig * uu[c] + (alp * kc) * ku;   // (sig I + alp k k^T) u_hat
            R[c * NS + idx] = (Au - Guh[c * NS + idx]) + Uh[c * NS + idx];
        }
    }
}

// Linearly implicit scheme of s <= 3 steps (Eq:IMEX_DAE): coefficients a_j,
// c_j (j = 0..s) and b_j (j < s), lowest index first.
struct LinimpScheme {
    int s;
    double a[4], b[3], c[4];
};

// Inputs of the constraint update: R_j and u_hat_j of the levels j < s.
struct LinimpLevels {
    const cpx<double>* R[3];
    const cpx<double>* uh[3];
    double b[3], c[3];
    int s;
};

// u_hat_new = A^{-1} (sum_j b_j R_j - sum_{j<s} c_j A u_hat_j) / c_s per mode (the
// constraint equation of Eq:IMEX_DAE; Eq:MM for SBDF2, where c_j = 0 for j < s).
// out may alias an input (each mode is read before it is written).
template <int D>
__global__ void k_linimp_solve(int nx, int ny, size_t NS, double tpx, double tpy, double sig, double alp,
                               double inv_cs, LinimpLevels L, cpx<double>* out) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < NS; idx += stride) {
        const int kxi = (int)(idx / ny), kyi = (int)(idx - (size_t)kxi * ny);
        const double kx = wavenumber<double>(kxi, nx, tpx);
        const double ky = D == 2 ? wavenumber<double>(kyi, ny, tpy) : 0.0;
        cpx<double> r[D], z[D];
        for (int c = 0; c < D; ++c) r[c] = C<double>(0.0, 0.0);
        for (int j = 0; j < L.s; ++j) {
            for (int c = 0; c < D; ++c) r[c] = r[c] + L.b[j] * L.R[j][c * NS + idx];
            if (L.c[j] != 0.0) {
                cpx<double> uu[D];
                for (int c = 0; c < D; ++c) uu[c] = L.uh[j][c * NS + idx];
                cpx<double> ku = kx * uu[0];
                if (D == 2) ku = ku + ky * uu[1 % D];
                for (int c = 0; c < D; ++c) {
                    const double kc = c == 0 ? kx : ky;
                    r[c] = r[c] - L.c[j] * (sig * uu[c] + (alp * kc) * ku);
                }
            }
        }
        if (inv_cs != 1.0)
            for (int c = 0; c < D; ++c) r[c] = inv_cs * r[c];
        precond_mode<double, D>(kx, ky, sig, alp, r, z);
        for (int c = 0; c < D; ++c) out[c * NS + idx] = z[c];
    }
}

template <int D>
sgn_status sbdf2_R(sgn_state* st, cpx<double>* Rout) {
    sgn_ctx* ctx = st->ctx;
    const Dims& d = st->d;
    Carve cv(st->ws);
    Common cm = carve_common(cv);
    PcgLaunch<double, D> P;
    P.ctx = ctx;
    P.d = d;
    P.rl = row_launch<double>(d.nx, d.ny, true);
    P.cl = pcg_col_launch<double>(d);
    P.b = carve_pcg<double>(cv, d, false);
    P.sc = cm.sc;
    P.partials = cm.partials;
    P.eta = st->eta;
    P.gh = st->gh;
    sgn_status s;
    if ((s = init_scal(ctx, P.sc, 1.0, 1, d.inv_n, nullptr)) != SGN_OK) return s;
    if ((s = to_S_d<D>(ctx, d, st->U, st->b.Hs, st->b.Uh)) != SGN_OK) return s;
    if ((s = pcg_c1<double, D>(P, C1_COPY, st->b.uh)) != SGN_OK) return s;
    if ((s = pcg_r1<double, D>(P)) != SGN_OK) return s;
    if ((s = pcg_c2<double, D>(P, C2_STORE, nullptr, nullptr)) != SGN_OK) return s;
    hipLaunchKernelGGL(k_sbdf2_R<D>, dim3(flat_blocks(d.NS)), dim3(256), 0, ctx->stream, d.nx, d.ny, d.NS, d.tpx,
                       d.tpy, st->sb_sig, st->sb_alp, (const cpx<double>*)st->b.uh, (const cpx<double>*)P.b.qh,
                       (const cpx<double>*)st->b.Uh, Rout);
    CHECK_LAUNCH(ctx);
    return SGN_OK;
}

// Record the state's level (eta, U, f, R = A u - G u + U, u_hat) in ring slot k.
// b.uh holds the state's u_hat on entry; afterwards b.uh is scratch.
template <int D>
sgn_status linimp_record(sgn_state* st, int k) {
    sgn_ctx* ctx = st->ctx;
    StateBufs& b = st->b;
    const size_t N = st->d.N, DN = (size_t)st->d.D * st->d.N;
    sgn_status s;
    if ((s = state_rhs(st, st->eta, st->u, b.lv_fe[k], b.lv_fU[k])) != SGN_OK) return s;
    if ((s = sbdf2_R<D>(st, b.lv_R[k])) != SGN_OK) return s;
    std::swap(b.lv_uh[k], b.uh);
    if ((s = copy_d(ctx, b.lv_eta[k], st->eta, N)) != SGN_OK) return s;
    return copy_d(ctx, b.lv_U[k], st->U, DN);
}

// nsteps steps of a linearly implicit scheme of s <= 3 steps with A = theta
// (sigma I - alpha grad div): (sigma, alpha) fixed by the caller or taken from
// the state's eta when a history starts (section 6.5), kept for its life.  A new
// history records the current level and takes s-1 RK4 steps (opts), recording
// each level; then every step forms
//   w_{n+s}   = (-sum_{j<s} a_j w_{n+j} + dt sum_j b_j f_{n+j}) / a_s,
//   A u_{n+s} = (sum_j b_j R_{n+j} - sum_{j<s} c_j A u_{n+j}) / c_s,
// R = A u - G_{eta,h} u + U, with one A-solve and no Krylov iteration.
template <int D>
sgn_status linimp_steps(sgn_state* st, const LinimpScheme& sch, double scheme_r, double theta, double dt,
                        int nsteps, const sgn_coeffs* fixed, const sgn_solve_opts& o, sgn_step_info* acc) {
    sgn_ctx* ctx = st->ctx;
    const Dims& d = st->d;
    StateBufs& b = st->b;
    const size_t N = d.N, DN = (size_t)d.D * d.N;
    const int S = sch.s;
    sgn_status s;
    if (nsteps <= 0) return SGN_OK;
    // Eq:IMEX_DAE needs the same A on both sides of every step: another scheme,
    // scale, dt or fixed coefficients start a new history
    const double fs = fixed ? fixed->sigma : 0.0, fa = fixed ? fixed->alpha : 0.0;
    const bool same = st->kind == 2 && st->hist_dt == dt && st->lm_s == S && st->lm_r == scheme_r &&
                      st->lm_theta == theta && st->lm_fix_sig == fs && st->lm_fix_alp == fa;
    if (!same) {
        if (fixed) {
            st->sb_sig = theta * fixed->sigma;
            st->sb_alp = theta * fixed->alpha;
        } else {
            Carve cv(st->ws);
            Common cm = carve_common(cv);
            if ((s = init_scal(ctx, cm.sc, 1.0, 1, d.inv_n, nullptr)) != SGN_OK) return s;
            if ((s = launch_coeffs(ctx, d, st->eta, st->gh, st->flat, o.coeff_kind, cm.sc, cm.partials)) != SGN_OK)
                return s;
            if ((s = read_scal(ctx, cm.sc)) != SGN_OK) return s;
            if (ctx->hscal->status != 0) return fail(ctx, SGN_EDOMAIN, "total depth must be positive and finite");
            st->sb_sig = theta * ctx->hscal->sig;
            st->sb_alp = theta * ctx->hscal->alp;
        }
        st->kind = 2;
        st->hist_dt = dt;
        st->lm_s = S;
        st->lm_r = scheme_r;
        st->lm_theta = theta;
        st->lm_fix_sig = fs;
        st->lm_fix_alp = fa;
        st->lm_count = 0;
        st->lm_head = 0;
    }
    const int slots = S - 1;
    auto slot = [&](int j) { return (st->lm_head + j) % slots; };   // j = 0: the oldest level
    // start-up: record the level, then an RK4 step (its first stage reuses the f just formed)
    while (st->lm_count < slots && nsteps > 0) {
        const int k = slot(st->lm_count);
        if ((s = to_S_d<D>(ctx, d, st->u, b.Hs, b.uh)) != SGN_OK) return s;
        if ((s = linimp_record<D>(st, k)) != SGN_OK) return s;
        if ((s = copy_d(ctx, b.rk_fe[0], b.lv_fe[k], N)) != SGN_OK) return s;
        if ((s = copy_d(ctx, b.rk_fU[0], b.lv_fU[k], DN)) != SGN_OK) return s;
        if ((s = rk4_one(st, dt, o, acc, true)) != SGN_OK) return s;
        st->lm_count += 1;
        nsteps -= 1;
        if (st->lm_count == slots && (s = to_S_d<D>(ctx, d, st->u, b.Hs, b.uh)) != SGN_OK) return s;
    }
    for (int n = 0; n < nsteps; ++n) {
        // the current level n+s-1 is the state: f and R from eta, U and u_hat (b.uh)
        if ((s = state_rhs(st, st->eta, st->u, b.rk_fe[0], b.rk_fU[0])) != SGN_OK) return s;
        if ((s = sbdf2_R<D>(st, b.R_cur)) != SGN_OK) return s;
        std::vector<const double*> te, tU;
        std::vector<double> cw;
        for (int j = 0; j < S; ++j) {
            te.push_back(j < slots ? b.lv_eta[slot(j)] : st->eta);
            tU.push_back(j < slots ? b.lv_U[slot(j)] : st->U);
            cw.push_back(-sch.a[j]);
        }
        for (int j = 0; j < S; ++j) {
            te.push_back(j < slots ? b.lv_fe[slot(j)] : b.rk_fe[0]);
            tU.push_back(j < slots ? b.lv_fU[slot(j)] : b.rk_fU[0]);
            cw.push_back(dt * sch.b[j]);
        }
        if ((s = lincomb(ctx, N, nullptr, 1.0, te, cw, b.tmp_e, sch.a[S])) != SGN_OK) return s;
        if ((s = lincomb(ctx, DN, nullptr, 1.0, tU, cw, b.tmp_U, sch.a[S])) != SGN_OK) return s;
        // u_hat of level n+s into the oldest slot's u_hat buffer (read first per mode)
        LinimpLevels lv{};
        lv.s = S;
        for (int j = 0; j < S; ++j) {
            lv.R[j] = j < slots ? b.lv_R[slot(j)] : b.R_cur;
            lv.uh[j] = j < slots ? b.lv_uh[slot(j)] : b.uh;
            lv.b[j] = sch.b[j];
            lv.c[j] = sch.c[j];
        }
        const int old = slot(0);
        hipLaunchKernelGGL(k_linimp_solve<D>, dim3(flat_blocks(d.NS)), dim3(256), 0, ctx->stream, d.nx, d.ny, d.NS,
                           d.tpx, d.tpy, st->sb_sig, st->sb_alp, 1.0 / sch.c[S], lv, b.lv_uh[old]);
        CHECK_LAUNCH(ctx);
        // ring shift: the oldest slot takes the current level; the new level becomes the state
        if ((s = copy_d(ctx, b.lv_eta[old], st->eta, N)) != SGN_OK) return s;
        if ((s = copy_d(ctx, b.lv_U[old], st->U, DN)) != SGN_OK) return s;
        std::swap(b.lv_fe[old], b.rk_fe[0]);
        std::swap(b.lv_fU[old], b.rk_fU[0]);
        std::swap(b.lv_R[old], b.R_cur);
        std::swap(b.lv_uh[old], b.uh);   // slot: the current u_hat; b.uh: the new one
        st->lm_head = (st->lm_head + 1) % slots;
        if ((s = copy_d(ctx, st->eta, b.tmp_e, N)) != SGN_OK) return s;
        if ((s = copy_d(ctx, st->U, b.tmp_U, DN)) != SGN_OK) return s;
        if ((s = from_S_d<D>(ctx, d, b.uh, b.Hs, st->u)) != SGN_OK) return s;
        st->t += dt;
        st->steps += 1;
    }
    return SGN_OK;
}

// Coefficients of SBDF2 (Table LMMCoeffs).
LinimpScheme scheme_sbdf2() {
    LinimpScheme q{};
    q.s = 2;
    q.a[0] = 0.5;
    q.a[1] = -2.0;
    q.a[2] = 1.5;
    q.b[0] = -1.0;
    q.b[1] = 2.0;
    q.c[2] = 1.0;
    return q;
}

// The third-order family with c(z) = (z - r)^3 and b(z) = c(z) - (z - 1)^3 (so the
// constraint recurrence has defect O(dt^3)); a(z) solves the third-order
// conditions sum_j a_j j^k = k sum_j c_j j^(k-1), k = 0..3 (Gaussian elimination
// of the 4 x 4 Vandermonde system).  r = 0 is SBDF3.
LinimpScheme scheme_sbdf3r(double r) {
    LinimpScheme q{};
    q.s = 3;
    q.c[0] = -r * r * r;
    q.c[1] = 3.0 * r * r;
    q.c[2] = -3.0 * r;
    q.c[3] = 1.0;
    const double cube[4] = {-1.0, 3.0, -3.0, 1.0};   // (z - 1)^3
    for (int j = 0; j < 3; ++j) q.b[j] = q.c[j] - cube[j];
    double M[4][5];
    for (int k = 0; k < 4; ++k) {
        double rhs = 0.0;
        for (int j = 0; j < 4; ++j) {
            M[k][j] = (k == 0) ? 1.0 : std::pow((double)j, k);
            if (k >= 1) rhs += q.c[j] * (k == 1 ? 1.0 : std::pow((double)j, k - 1));
        }
        M[k][4] = k * rhs;
    }
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int r2 = col + 1; r2 < 4; ++r2)
            if (std::fabs(M[r2][col]) > std::fabs(M[piv][col])) piv = r2;
        for (int j = 0; j < 5; ++j) std::swap(M[col][j], M[piv][j]);
        for (int r2 = 0; r2 < 4; ++r2) {
            if (r2 == col) continue;
            const double f = M[r2][col] / M[col][col];
            for (int j = col; j < 5; ++j) M[r2][j] -= f * M[col][j];
        }
    }
    for (int j = 0; j < 4; ++j) q.a[j] = M[j][4] / M[j][j];
    // a(1) = 0 exactly in floating point, in the order k_lincomb sums the terms, so
    // that the update keeps a constant level (and the mass) to rounding
    q.a[3] = -((q.a[0] + q.a[1]) + q.a[2]);
    return q;
}

// Real stable interval of the third-order family (roots of Eq:CharEq in |z| < 1):
// (1 / (1 + (1 + r)^3), 1 / (1 - ((1 + r) / 2)^3)).
void sbdf3r_interval(double r, double* lo, double* hi) {
    *lo = 1.0 / (1.0 + (1.0 + r) * (1.0 + r) * (1.0 + r));
    const double h = 0.5 * (1.0 + r);
    *hi = 1.0 / (1.0 - h * h * h);
}

void info_init(sgn_step_info* acc) {
    std::memset(acc, 0, sizeof(*acc));
    acc->converged = 1;
}
void info_finish(sgn_state* st, sgn_step_info* acc, sgn_step_info* out) {
    acc->t = st->t;
    acc->steps_done = st->steps;
    if (out) *out = *acc;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* sgn_version(void) { return "sgn-mi355x 0.1 (gfx950)"; }

sgn_status sgn_create(sgn_ctx** out, int device, void* hip_stream) {
    if (!out) return SGN_EINVAL;
    *out = nullptr;
    sgn_ctx* ctx = new (std::nothrow) sgn_ctx();
    if (!ctx) return SGN_ENOMEM;
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return SGN_EDEVICE;
    }
    // twiddle tables: for every power of two L <= TW_SIZE the roots W_L^j =
    // exp(-2 pi i j / L), j < L, at offset L - 1, from long double cos/sin
    std::vector<cpx<double>> t64(TW_ALL);
    std::vector<cpx<float>> t32(TW_ALL);
    const long double pi2 = 6.283185307179586476925286766559005768L;
    for (int L = 1; L <= TW_SIZE; L <<= 1) {
        for (int j = 0; j < L; ++j) {
            const long double a = pi2 * (long double)j / (long double)L;
            const long double c = cosl(a), sn = -sinl(a);
            t64[L - 1 + j] = cpx<double>{(double)c, (double)sn};
            t32[L - 1 + j] = cpx<float>{(float)c, (float)sn};
        }
    }
    bool ok = hipMalloc(&ctx->tw64, TW_ALL * sizeof(cpx<double>)) == hipSuccess &&
              hipMalloc(&ctx->tw32, TW_ALL * sizeof(cpx<float>)) == hipSuccess &&
              hipHostMalloc((void**)&ctx->hscal, sizeof(SolveScal), hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void**)&ctx->hflag, 64, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipMemcpy(ctx->tw64, t64.data(), TW_ALL * sizeof(cpx<double>), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(ctx->tw32, t32.data(), TW_ALL * sizeof(cpx<float>), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        sgn_destroy(ctx);
        return SGN_ENOMEM;
    }
    if (hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) ctx->cap_stream = nullptr;
    if (hipEventCreateWithFlags(&ctx->ev_sync, hipEventDisableTiming) != hipSuccess) ctx->ev_sync = nullptr;
    if (ctx->ev_sync &&
        hipHostMalloc((void**)&ctx->hpub, 64, hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess) {
        std::memset(ctx->hpub, 0, 64);
        if (hipHostGetDevicePointer((void**)&ctx->dpub, ctx->hpub, 0) != hipSuccess) ctx->dpub = nullptr;
    } else {
        ctx->hpub = nullptr;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        ctx->cus = cus;
    // pinned staging of one batch item and result and of the GMRES(m <= 256)
    // coefficients, allocated here so that a single solve (sgn_krylov_solve_noalloc
    // included) allocates nothing
    if (batch_staging(ctx, 8192) != SGN_OK) {
        sgn_destroy(ctx);
        return SGN_ENOMEM;
    }
    ctx->scratch = scratch_address(device);
    // HIP graphs for the PCG chunks are opt-in: their host-side launch costs more
    // than the eager launches of a chunk (measured: 1024^2 RK4 step 3.58 ms with
    // graphs, 3.56 ms without)
    const char* ug = getenv("SGN_GRAPHS");
    ctx->use_graphs = ug && ug[0] && ug[0] != '0';
    *out = ctx;
    return SGN_OK;
}

void sgn_destroy(sgn_ctx* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->tw64) (void)hipFree(ctx->tw64);
    if (ctx->tw32) (void)hipFree(ctx->tw32);
    if (ctx->hscal) (void)hipHostFree(ctx->hscal);
    if (ctx->hflag) (void)hipHostFree(ctx->hflag);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->ev_sync) (void)hipEventDestroy(ctx->ev_sync);
    if (ctx->hpub) (void)hipHostFree(ctx->hpub);
    for (auto& g : ctx->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->hbatch) (void)hipHostFree(ctx->hbatch);
    delete ctx;
}

sgn_status sgn_profile_begin(sgn_ctx* ctx) {
    if (!ctx) return SGN_EINVAL;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->prof_marks.clear();
    ctx->ev_next = 0;
    ctx->prof_on = true;
    return SGN_OK;
}

sgn_status sgn_profile_end(sgn_ctx* ctx, int64_t* launches, double* total_ms, int32_t nkinds) {
    if (!ctx || !launches || !total_ms || nkinds < 1) return SGN_EINVAL;
    ctx->prof_on = false;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < nkinds; ++k) {
        launches[k] = 0;
        total_ms[k] = 0.0;
    }
    ctx->prof_last.clear();
    for (auto& m : ctx->prof_marks) {
        float ms = 0.0f;
        HIPCHK(ctx, hipEventElapsedTime(&ms, m.second.first, m.second.second));
        ctx->prof_last.push_back({m.first, ms});
        if (m.first >= 0 && m.first < nkinds) {
            launches[m.first] += 1;
            total_ms[m.first] += ms;
        }
    }
    ctx->prof_marks.clear();
    ctx->ev_next = 0;
    return SGN_OK;
}

sgn_status sgn_profile_launches(const sgn_ctx* ctx, int32_t* kinds, float* ms, int64_t cap, int64_t* count) {
    if (!ctx || !count || cap < 0 || (cap > 0 && (!kinds || !ms))) return SGN_EINVAL;
    const int64_t n = (int64_t)ctx->prof_last.size();
    *count = n;
    for (int64_t i = 0; i < n && i < cap; ++i) {
        kinds[i] = ctx->prof_last[(size_t)i].first;
        ms[i] = ctx->prof_last[(size_t)i].second;
    }
    return SGN_OK;
}

sgn_status sgn_set_stream(sgn_ctx* ctx, void* hip_stream) {
    if (!ctx) return SGN_EINVAL;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return SGN_OK;
}

const char* sgn_last_error(const sgn_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

size_t sgn_workspace_bytes(const sgn_grid* grid, int32_t precision) {
    Dims d;
    if (check_grid(nullptr, grid, &d) != SGN_OK) return 0;
    if (d.bc == SGN_BC_WALLS) {
        const Dims t = twin_dims(d);
        Carve cv(nullptr);
        return carve_walls(cv, t, nullptr) + workspace_bytes(t, precision);
    }
    return workspace_bytes(d, precision);
}

size_t sgn_gmres_workspace_bytes(const sgn_grid* grid, int32_t restart) {
    Dims d;
    if (check_grid(nullptr, grid, &d) != SGN_OK) return 0;
    if (restart < 1 || restart > GMRES_MAX_RESTART) return 0;
    if (d.bc == SGN_BC_WALLS) {
        const Dims t = twin_dims(d);
        Carve cv(nullptr);
        return carve_walls(cv, t, nullptr) + gmres_workspace_bytes(t, restart);
    }
    return gmres_workspace_bytes(d, restart);
}

}  // extern "C"

namespace {
sgn_status bathy_impl(sgn_ctx* ctx, const Dims& d, const double* h, double* grad_h, int32_t* flat, void* ws) {
    sgn_status s;
    Carve cv(ws);
    Common cm = carve_common(cv);
    cpx<double>* H = cv.take<cpx<double>>((size_t)(1 + d.D) * d.NS);
    if ((s = init_scal(ctx, cm.sc, 1.0, 1, d.inv_n, nullptr)) != SGN_OK) return s;
    hipLaunchKernelGGL(k_minmax, dim3(flat_blocks(d.N)), dim3(256), 0, ctx->stream, d.N, h, cm.partials);
    hipLaunchKernelGGL(k_minmax_finish, dim3(1), dim3(256), 0, ctx->stream, cm.sc, (const double*)cm.partials,
                       flat_blocks(d.N));
    CHECK_LAUNCH(ctx);
    if ((s = read_scal(ctx, cm.sc)) != SGN_OK) return s;
    const double hmin = ctx->hscal->red[0], hmax = ctx->hscal->red[1];
    if (!std::isfinite(hmin) || !std::isfinite(hmax)) return fail(ctx, SGN_EDOMAIN, "non-finite bathymetry");
    if (hmin == hmax) {
        hipLaunchKernelGGL(k_zero_c, dim3(flat_blocks((size_t)d.D * d.N)), dim3(256), 0, ctx->stream,
                           (size_t)d.D * d.N, (void*)grad_h);
        CHECK_LAUNCH(ctx);
        *flat = 1;
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        return SGN_OK;
    }
    *flat = 0;
    if ((s = rows_fwd<double, double>(ctx, d, {h}, {H})) != SGN_OK) return s;
    std::vector<cpx<double>*> gd;
    for (int c = 0; c < d.D; ++c) gd.push_back(H + (1 + c) * d.NS);
    if (d.D == 2)
        s = cols_lin<double>(ctx, d, {H}, gd, {{2}, {3}}, d.inv_n);
    else
        s = cols_lin<double>(ctx, d, {H}, gd, {{2}}, d.inv_n);
    if (s != SGN_OK) return s;
    std::vector<const cpx<double>*> gs(gd.begin(), gd.end());
    std::vector<double*> od;
    for (int c = 0; c < d.D; ++c) od.push_back(grad_h + c * d.N);
    if ((s = rows_inv<double, double>(ctx, d, gs, od)) != SGN_OK) return s;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SGN_OK;
}
}  // namespace

extern "C" {

sgn_status sgn_bathy_prepare(sgn_ctx* ctx, const sgn_grid* grid, const double* h, double* grad_h, int32_t* flat,
                             void* ws) {
    if (!ctx) return SGN_EINVAL;
    Dims d;
    sgn_status s = check_grid(ctx, grid, &d);
    if (s != SGN_OK) return s;
    if (!h || !grad_h || !flat || !ws) return fail(ctx, SGN_EINVAL, "null pointer");
    if (d.bc != SGN_BC_WALLS) return bathy_impl(ctx, d, h, grad_h, flat, ws);
    const Dims t = twin_dims(d);
    WallBufs w;
    Carve cv(ws);
    carve_walls(cv, t, &w);
    if ((s = wall_reflect(ctx, d, h, w.eta, false)) != SGN_OK) return s;
    if ((s = bathy_impl(ctx, t, w.eta, w.gh, flat, w.ws)) != SGN_OK) return s;
    if ((s = wall_restrict(ctx, d, w.gh, grad_h)) != SGN_OK) return s;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SGN_OK;
}

sgn_status sgn_precond_coeffs(sgn_ctx* ctx, const sgn_grid* grid, const double* eta, const double* grad_h,
                              int32_t flat, int32_t kind, sgn_coeffs* out, void* ws) {
    if (!ctx) return SGN_EINVAL;
    Dims d;
    sgn_status s = check_grid(ctx, grid, &d);
    if (s != SGN_OK) return s;
    if (!eta || !grad_h || !out || !ws) return fail(ctx, SGN_EINVAL, "null pointer");
    if (kind != SGN_COEFF_OPTIMAL && kind != SGN_COEFF_REPLACEMENT) return fail(ctx, SGN_EINVAL, "bad kind");
    Carve cv(ws);
    Common cm = carve_common(cv);
    if ((s = init_scal(ctx, cm.sc, 1.0, 1, d.inv_n, nullptr)) != SGN_OK) return s;
    if ((s = launch_coeffs(ctx, d, eta, grad_h, flat ? 1 : 0, kind, cm.sc, cm.partials)) != SGN_OK) return s;
    if ((s = read_scal(ctx, cm.sc)) != SGN_OK) return s;
    if (ctx->hscal->status != 0) return fail(ctx, SGN_EDOMAIN, "total depth must be positive and finite");
    out->sigma = ctx->hscal->sig;
    out->alpha = ctx->hscal->alp;
    out->kappa_ub = ctx->hscal->kap;
    out->flat = ctx->hscal->flat;
    return SGN_OK;
}

sgn_status sgn_apply_constraint(sgn_ctx* ctx, const sgn_grid* grid, const double* eta, const double* grad_h,
                                const double* u, double* out, void* ws) {
    if (!ctx) return SGN_EINVAL;
    Dims d;
    sgn_status s = check_grid(ctx, grid, &d);
    if (s != SGN_OK) return s;
    if (!eta || !grad_h || !u || !out || !ws) return fail(ctx, SGN_EINVAL, "null pointer");
    if (out == u) return fail(ctx, SGN_EINVAL, "out may not alias u");
    if (d.bc != SGN_BC_WALLS)
        return d.D == 1 ? apply_G<1>(ctx, d, eta, grad_h, u, out, ws) : apply_G<2>(ctx, d, eta, grad_h, u, out, ws);
    const Dims t = twin_dims(d);
    WallBufs w;
    Carve cv(ws);
    carve_walls(cv, t, &w);
    if ((s = wall_reflect(ctx, d, eta, w.eta, false)) != SGN_OK) return s;
    if ((s = wall_reflect(ctx, d, grad_h, w.gh, true)) != SGN_OK) return s;
    if ((s = wall_reflect(ctx, d, u, w.f, true)) != SGN_OK) return s;
    s = d.D == 1 ? apply_G<1>(ctx, t, w.eta, w.gh, w.f, w.u, w.ws) : apply_G<2>(ctx, t, w.eta, w.gh, w.f, w.u, w.ws);
    if (s != SGN_OK) return s;
    return wall_restrict(ctx, d, w.u, out);
}

sgn_status sgn_precond_solve(sgn_ctx* ctx, const sgn_grid* grid, const sgn_coeffs* co, const double* rhs,
                             double* out, void* ws) {
    if (!ctx) return SGN_EINVAL;
    Dims d;
    sgn_status s = check_grid(ctx, grid, &d);
    if (s != SGN_OK) return s;
    if (!co || !rhs || !out || !ws) return fail(ctx, SGN_EINVAL, "null pointer");
    if (!(co->sigma > 0.0) || !(co->alpha > 0.0)) return fail(ctx, SGN_EINVAL, "sigma and alpha must be > 0");
    if (d.bc != SGN_BC_WALLS)
        return d.D == 1 ? precond_apply<1>(ctx, d, co->sigma, co->alpha, rhs, out, ws)
                        : precond_apply<2>(ctx, d, co->sigma, co->alpha, rhs, out, ws);
    const Dims t = twin_dims(d);
    WallBufs w;
    Carve cv(ws);
    carve_walls(cv, t, &w);
    if ((s = wall_reflect(ctx, d, rhs, w.f, true)) != SGN_OK) return s;
    s = d.D == 1 ? precond_apply<1>(ctx, t, co->sigma, co->alpha, w.f, w.u, w.ws)
                 : precond_apply<2>(ctx, t, co->sigma, co->alpha, w.f, w.u, w.ws);
    if (s != SGN_OK) return s;
    return wall_restrict(ctx, d, w.u, out);
}

sgn_status sgn_krylov_solve(sgn_ctx* ctx, const sgn_grid* grid, const double* eta, const double* grad_h,
                            const double* rhs, double* u, const sgn_coeffs* coeffs, const sgn_solve_opts* opts,
                            sgn_solve_info* info, void* ws) {
    if (!ctx) return SGN_EINVAL;
    Dims d;
    sgn_status s = check_grid(ctx, grid, &d);
    if (s != SGN_OK) return s;
    if (!eta || !grad_h || !rhs || !u || !ws) return fail(ctx, SGN_EINVAL, "null pointer");
    const sgn_solve_opts o = opts ? *opts : default_opts();
    if (o.coeff_kind != SGN_COEFF_OPTIMAL && o.coeff_kind != SGN_COEFF_REPLACEMENT)
        return fail(ctx, SGN_EINVAL, "bad coeff_kind");
    // without given coefficients the flat formulas apply iff |grad h|_max = 0
    if (d.bc != SGN_BC_WALLS)
        return solve_dispatch(ctx, d, eta, grad_h, rhs, u, coeffs, coeffs ? coeffs->flat : -1, o, info, ws);
    if (wall_native(d, o)) {
        return solve_wall_native(ctx, d, eta, grad_h, rhs, u, coeffs, coeffs ? coeffs->flat : -1, o, info, ws);
    }
    const Dims t = twin_dims(d);
    WallBufs w;
    Carve cv(ws);
    carve_walls(cv, t, &w);
    if ((s = wall_reflect(ctx, d, eta, w.eta, false)) != SGN_OK) return s;
    if ((s = wall_reflect(ctx, d, grad_h, w.gh, true)) != SGN_OK) return s;
    if ((s = wall_reflect(ctx, d, rhs, w.f, true)) != SGN_OK) return s;
    if (o.x0_is_guess && (s = wall_reflect(ctx, d, u, w.u, true)) != SGN_OK) return s;
    ctx->wall_twin = true;
    s = solve_dispatch(ctx, t, w.eta, w.gh, w.f, w.u, coeffs, coeffs ? coeffs->flat : -1, o, info, w.ws);
    ctx->wall_twin = false;
    // the iterate is returned as for a periodic grid: on success and when max_iter stops it
    if (s == SGN_OK || s == SGN_ENOCONV) {
        const sgn_status r = wall_restrict(ctx, d, w.u, u);
        if (r != SGN_OK) return r;
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    return s;
}

sgn_status sgn_krylov_solve_noalloc(sgn_ctx* ctx, const sgn_grid* grid, const double* eta, const double* grad_h,
                                    const double* rhs, double* u, const sgn_coeffs* coeffs,
                                    const sgn_solve_opts* opts, sgn_solve_info* info) {
    if (!ctx) return SGN_EINVAL;
    if (!ctx->scratch) return fail(ctx, SGN_EDEVICE, "the no-alloc scratch has no device address");
    Dims d;
    sgn_status s = check_grid(ctx, grid, &d);
    if (s != SGN_OK) return s;
    const sgn_solve_opts o = opts ? *opts : default_opts();
    const size_t need = o.method == SGN_GMRES ? sgn_gmres_workspace_bytes(grid, o.gmres_restart)
                                              : sgn_workspace_bytes(grid, o.precision);
    if (need == 0) return fail(ctx, SGN_EINVAL, "bad solver options for this grid");
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(ctx, SGN_EINVAL, "workspace of " + std::to_string(need) + " bytes exceeds the " +
                                         std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte no-alloc scratch");
    // graph capture allocates: the iteration chunks run eagerly here
    const bool graphs = ctx->use_graphs;
    ctx->use_graphs = false;
    s = sgn_krylov_solve(ctx, grid, eta, grad_h, rhs, u, coeffs, opts, info, ctx->scratch);
    ctx->use_graphs = graphs;
    return s;
}

}  // extern "C"

namespace {

// Layout of a batch workspace: the work-queue counter, the item table, results,
// then each system's region.
struct BatchLayout {
    size_t queue, items, results, data, total;
};
constexpr size_t BATCH_HEAD = 256;   // bytes before the item table (the counter, padded)

BatchLayout batch_layout(int nitems, const int32_t* n, int mode) {
    BatchLayout l;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    l.queue = 0;
    l.items = BATCH_HEAD;
    l.results = l.items + up(sizeof(BatchItem) * (size_t)nitems);
    l.data = l.results + up(sizeof(BatchResult) * (size_t)nitems);
    size_t dbl = 0;
    for (int i = 0; i < nitems; ++i) dbl += (size_t)batch_item_doubles(n[i], mode);
    l.total = l.data + up(dbl * sizeof(double)) + 256;
    return l;
}

bool batch_size_ok(int n) { return n >= 2 && n <= BATCH_NMAX && (n & (n - 1)) == 0; }

// Workgroup size of every system of a batched call (sgn_batch_solve,
// sgn_batch_step_rk4); the one-system paths take the size class of their n.
constexpr int BATCH_CALL_THREADS = 512;

// k_batch_solve over nitems table entries (workgroups of nt threads) on
// `stream`.  LDS: two transform buffers of the largest system's M + 1 modes (FP64
// ones in FP64 mode; in mixed mode the FP32 pair or one FP64 buffer, the
// refinement residual, whichever is larger).  grid = 0: as many workgroups as fit
// the device (at most nitems), sharing the work queue d_queue.
sgn_status launch_batch_solve(sgn_ctx* ctx, hipStream_t stream, int nt, const BatchItem* d_items, int nitems,
                              int nmax, int mode, int grid, const double* eta, const double* gh, const double* rhs,
                              double* u, double* d_data, const BatchParams& prm, BatchResult* d_res, int* d_queue) {
    const size_t lds = (size_t)(nmax / 2 + 1) * sizeof(cpx<double>) * (mode == BATCH_FP64 ? 2 : 1);
    auto launch = [&](auto k) -> sgn_status {
        HIPCHK(ctx, allow_lds(k, lds));
        int g = grid;
        if (g <= 0) {
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, nt, lds) != hipSuccess || per_cu < 1)
                per_cu = 1;
            g = std::min(nitems, per_cu * ctx->cus);
        }
        hipLaunchKernelGGL(k, dim3(g), dim3(nt), lds, stream, d_items, nitems, eta, gh, rhs, u, d_data, ctx->tw64,
                           ctx->tw32, prm, d_res, d_queue);
        CHECK_LAUNCH(ctx);
        return SGN_OK;
    };
    const bool mx = mode == BATCH_MIXED;
    if (nt == 256) return mx ? launch(k_batch_solve<BATCH_MIXED, 256>) : launch(k_batch_solve<BATCH_FP64, 256>);
    return mx ? launch(k_batch_solve<BATCH_MIXED, 512>) : launch(k_batch_solve<BATCH_FP64, 512>);
}

// ---- batched RK4 runs (k_batch_rk4) ----------------------------------------

// One state's arrays in a batched run, each 256-byte aligned: h_x, U, the four
// stage right-hand sides of eta and of U, eta_s, U_s, u_s, the solve base, the
// two recorded offsets of each guess slot; then the scratch.
constexpr int STEP_ARRAYS = 2 + 8 + 4 + 2 * STEP_SLOTS;
long long step_align(long long d) { return (d + 31) & ~31LL; }
long long step_item_doubles(int n, int mode) {
    return STEP_ARRAYS * step_align(n) + step_align(step_scratch_doubles(n, mode));
}

struct StepLayout {
    size_t items, results, data, total;
};
StepLayout step_layout(int nitems, const int32_t* n, int mode) {
    StepLayout l;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    l.items = BATCH_HEAD;
    l.results = l.items + up(sizeof(StepItem) * (size_t)nitems);
    l.data = l.results + up(sizeof(StepResult) * (size_t)nitems);
    size_t dbl = 0;
    for (int i = 0; i < nitems; ++i) dbl += (size_t)step_item_doubles(n[i], mode);
    l.total = l.data + dbl * sizeof(double) + 256;
    return l;
}

// Solve parameters of every stage solve of a run.
BatchParams step_params(const sgn_solve_opts& o, int nitems) {
    BatchParams prm{};
    prm.tol = o.tol;
    prm.inner_tol = o.inner_tol > 0 ? o.inner_tol : 1e-5;
    prm.max_iter = o.max_iter;
    prm.max_outer = o.max_outer > 0 ? o.max_outer : 20;
    prm.x0_is_guess = 1;
    prm.coeff_kind = o.coeff_kind;
    prm.nitems = nitems;
    prm.flat = -1;
    return prm;
}

// Workgroup size of a state's runs: fixed by its own size, so that its
// reductions (and with them its results) do not depend on what shares a launch.
int step_threads(int n) { return batch_threads_for(n); }

// k_batch_rk4 over nitems table entries (workgroups of nt
// threads) on `stream`; grid = 0: as many workgroups as fit the device (at most
// nitems), which then share the work queue d_queue (zero at launch).
sgn_status launch_batch_rk4(sgn_ctx* ctx, hipStream_t stream, int nt, const StepItem* d_items, int nitems, int nmax,
                            int mode, int grid, const BatchParams& prm, bool extrapolate, StepResult* d_res,
                            int* d_queue) {
    const size_t lds = (size_t)(nmax / 2 + 1) * sizeof(cpx<double>) * (mode == BATCH_FP64 ? 2 : 1);
    auto launch = [&](auto k) -> sgn_status {
        HIPCHK(ctx, allow_lds(k, lds));
        int g = grid;
        if (g <= 0) {
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, nt, lds) != hipSuccess || per_cu < 1)
                per_cu = 1;
            g = std::min(nitems, per_cu * ctx->cus);
        }
        hipLaunchKernelGGL(k, dim3(g), dim3(nt), lds, stream, d_items, nitems, ctx->tw64, ctx->tw32, prm,
                           extrapolate ? 1 : 0, d_res, d_queue);
        CHECK_LAUNCH(ctx);
        return SGN_OK;
    };
    const bool mx = mode == BATCH_MIXED;
    if (nt == 256) return mx ? launch(k_batch_rk4<BATCH_MIXED, 256>) : launch(k_batch_rk4<BATCH_FP64, 256>);
    return mx ? launch(k_batch_rk4<BATCH_MIXED, 512>) : launch(k_batch_rk4<BATCH_FP64, 512>);
}

static_assert(sizeof(StepItem) <= 512 && sizeof(StepResult) <= 512, "step table entries");

// RK4 steps of a periodic 1D state of up to BATCH_NMAX points in one launch:
// k_batch_rk4 with the single state, its own buffers and guess history.  The
// table entry, its result and the scratch sit at the start of the state's solve
// workspace (item | result | scratch from byte 1024).
sgn_status rk4_block(sgn_state* st, double dt, int nsteps, const sgn_solve_opts& o, sgn_step_info* acc) {
    sgn_ctx* ctx = st->ctx;
    StateBufs& b = st->b;
    sgn_status s;
    if ((s = batch_staging(ctx, 1024)) != SGN_OK) return s;
    const int mode = o.precision == SGN_MIXED ? BATCH_MIXED : BATCH_FP64;
    StepItem* hit = static_cast<StepItem*>(ctx->hbatch);
    std::memset(hit, 0, sizeof(StepItem));
    hit->eta = st->eta;
    hit->U = st->U;
    hit->u = st->u;
    hit->hx = const_cast<double*>(st->gh);   // read only: h is null
    hit->h = nullptr;
    for (int k = 0; k < 4; ++k) {
        hit->fe[k] = b.rk_fe[k];
        hit->fU[k] = b.rk_fU[k];
    }
    hit->eta_s = b.eta_s;
    hit->U_s = b.U_s;
    hit->u_s = b.u_s;
    hit->base = b.gx_base;
    static_assert(GUESS_RK2 == 0 && GUESS_RK_FINAL == STEP_SLOTS - 1, "stepper slots");
    for (int k = 0; k < STEP_SLOTS; ++k) {
        hit->off[k][0] = b.gx_off[k][0];
        hit->off[k][1] = b.gx_off[k][1];
        hit->cnt[k] = st->gx_count[k];
        hit->head[k] = st->gx_head[k];
    }
    char* base = static_cast<char*>(st->ws);
    hit->scr = reinterpret_cast<double*>(base + 1024);
    hit->L = st->d.Lx;
    hit->dt = dt;
    hit->n = st->d.nx;
    hit->index = 0;
    hit->nsteps = nsteps;
    hit->flat = st->flat ? 1 : 0;
    StepItem* d_item = reinterpret_cast<StepItem*>(base);
    StepResult* d_res = reinterpret_cast<StepResult*>(base + 512);
    HIPCHK(ctx, hipMemcpyAsync(d_item, hit, sizeof(StepItem), hipMemcpyHostToDevice, ctx->stream));
    {
        ProfScope ps(ctx, SGN_KERNEL_BATCH_STEP);
        if ((s = launch_batch_rk4(ctx, ctx->stream, step_threads(st->d.nx), d_item, 1, st->d.nx, mode, 1,
                                  step_params(o, 1), o.guess == SGN_GUESS_EXTRAPOLATE, d_res, nullptr)) != SGN_OK)
            return s;
    }
    StepResult* hres = reinterpret_cast<StepResult*>(static_cast<char*>(ctx->hbatch) + 512);
    HIPCHK(ctx, hipMemcpyAsync(hres, d_res, sizeof(StepResult), hipMemcpyDeviceToHost, ctx->stream));
    if ((s = wait_stream(ctx)) != SGN_OK) return s;
    const StepResult r = *hres;
    acc->solves += r.solves;
    acc->iters += r.iters;
    if (r.max_iters > acc->max_iters) acc->max_iters = r.max_iters;
    if (!r.converged) acc->converged = 0;
    for (int k = 0; k < r.steps; ++k) st->t += dt;
    st->steps += r.steps;
    for (int k = 0; k < STEP_SLOTS; ++k) {
        st->gx_count[k] = r.cnt[k];
        st->gx_head[k] = r.head[k];
    }
    if (r.status == -2) return fail(ctx, SGN_EDOMAIN, "non-positive depth or non-finite data in the solve");
    if (r.status == -3) return fail(ctx, SGN_ENOCONV, "Krylov solve did not reach the tolerance");
    return SGN_OK;
}

// The state's RK4 steps run in one launch: a periodic 1D grid of up to
// BATCH_NMAX points, the plain right-hand side, PCG in FP64 or mixed precision.
bool rk4_block_ok(const sgn_state* st, const sgn_solve_opts& o) {
    return st->d.D == 1 && st->d.nx <= BATCH_NMAX && !st->dealias && o.method == SGN_PCG &&
           (o.precision == SGN_FP64 || o.precision == SGN_MIXED);
}


}  // namespace

extern "C" {

size_t sgn_batch_workspace_bytes(int32_t nitems, const int32_t* n, int32_t precision) {
    if (nitems < 0 || (nitems > 0 && !n)) return 0;
    if (precision != SGN_FP64 && precision != SGN_MIXED) return 0;
    for (int i = 0; i < nitems; ++i)
        if (!batch_size_ok(n[i])) return 0;
    return batch_layout(nitems, n, precision == SGN_MIXED ? BATCH_MIXED : BATCH_FP64).total;
}

sgn_status sgn_batch_solve(sgn_ctx* ctx, int32_t nitems, const int32_t* n, const double* L, const double* eta,
                           const double* grad_h, const double* rhs, double* u, const sgn_solve_opts* opts,
                           sgn_solve_info* info, void* ws) {
    if (!ctx) return SGN_EINVAL;
    if (nitems < 0) return fail(ctx, SGN_EINVAL, "nitems < 0");
    if (nitems == 0) return SGN_OK;
    if (!n || !L || !eta || !grad_h || !rhs || !u || !ws) return fail(ctx, SGN_EINVAL, "null pointer");
    const sgn_solve_opts o = opts ? *opts : default_opts();
    if (o.method != SGN_PCG) return fail(ctx, SGN_EUNSUPPORTED, "only PCG is available");
    if (o.precision != SGN_FP64 && o.precision != SGN_MIXED) return fail(ctx, SGN_EINVAL, "unknown precision");
    if (!(o.tol > 0.0) || o.max_iter < 1) return fail(ctx, SGN_EINVAL, "tol must be > 0 and max_iter >= 1");
    if (o.coeff_kind != SGN_COEFF_OPTIMAL && o.coeff_kind != SGN_COEFF_REPLACEMENT)
        return fail(ctx, SGN_EINVAL, "bad coeff_kind");
    int nmax = 0;
    for (int i = 0; i < nitems; ++i) {
        if (!batch_size_ok(n[i])) return fail(ctx, SGN_EUNSUPPORTED, "batch sizes must be powers of two in [2, 8192]");
        if (!(L[i] > 0.0) || !std::isfinite(L[i])) return fail(ctx, SGN_EINVAL, "periods must be positive");
        nmax = std::max(nmax, (int)n[i]);
    }
    const int mode = o.precision == SGN_MIXED ? BATCH_MIXED : BATCH_FP64;
    const BatchLayout lay = batch_layout(nitems, n, mode);
    sgn_status s;
    if ((s = batch_staging(ctx, BATCH_HEAD + std::max(sizeof(BatchItem), sizeof(BatchResult)) * (size_t)nitems)) !=
        SGN_OK)
        return s;
    // systems in the caller's order for offsets; the table is sorted by size
    // (largest first) so that blocks take the long systems first
    std::vector<long long> off(nitems), wso(nitems);
    long long po = 0, pw = 0;
    for (int i = 0; i < nitems; ++i) {
        off[i] = po;
        wso[i] = pw;
        po += n[i];
        pw += batch_item_doubles(n[i], mode);
    }
    // systems in the caller's order for offsets; the table is sorted by size
    // (largest first) so that workgroups take the long systems first
    std::vector<int> order(nitems);
    for (int i = 0; i < nitems; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n[a] > n[b]; });
    // staging: the queue counter (0), then the item table, copied in one transfer
    std::memset(ctx->hbatch, 0, BATCH_HEAD);
    BatchItem* hit = reinterpret_cast<BatchItem*>(static_cast<char*>(ctx->hbatch) + BATCH_HEAD);
    for (int s2 = 0; s2 < nitems; ++s2) {
        const int i = order[s2];
        hit[s2].n = n[i];
        hit[s2].index = i;
        hit[s2].L = L[i];
        hit[s2].off = off[i];
        hit[s2].wso = wso[i];
    }
    char* base = static_cast<char*>(ws);
    int* d_queue = reinterpret_cast<int*>(base + lay.queue);
    BatchItem* d_items = reinterpret_cast<BatchItem*>(base + lay.items);
    BatchResult* d_res = reinterpret_cast<BatchResult*>(base + lay.results);
    double* d_data = reinterpret_cast<double*>(base + lay.data);
    HIPCHK(ctx, hipMemcpyAsync(base, ctx->hbatch, BATCH_HEAD + sizeof(BatchItem) * (size_t)nitems,
                               hipMemcpyHostToDevice, ctx->stream));
    BatchParams prm{};
    prm.tol = o.tol;
    prm.inner_tol = o.inner_tol > 0 ? o.inner_tol : 1e-5;
    prm.max_iter = o.max_iter;
    prm.max_outer = o.max_outer > 0 ? o.max_outer : 20;
    prm.x0_is_guess = o.x0_is_guess ? 1 : 0;
    prm.coeff_kind = o.coeff_kind;
    prm.nitems = nitems;
    prm.flat = -1;
    {
        ProfScope ps(ctx, SGN_KERNEL_BATCH);
        // every system of a batched call on 512 threads, whatever its size: a
        // system's reductions, and so its result, do not depend on the batch
        if ((s = launch_batch_solve(ctx, ctx->stream, BATCH_CALL_THREADS, d_items, nitems, nmax, mode, 0, eta, grad_h,
                                    rhs, u, d_data, prm, d_res, d_queue)) != SGN_OK)
            return s;
    }
    BatchResult* hres = static_cast<BatchResult*>(ctx->hbatch);
    HIPCHK(ctx, hipMemcpyAsync(hres, d_res, sizeof(BatchResult) * (size_t)nitems, hipMemcpyDeviceToHost, ctx->stream));
    if ((s = wait_stream(ctx)) != SGN_OK) return s;
    bool bad = false, nc = false;
    for (int i = 0; i < nitems; ++i) {
        const BatchResult& r = hres[i];
        if (info) {
            info[i].iters = r.iters;
            info[i].outer_iters = r.outer;
            info[i].converged = r.converged;
            info[i].relres = r.relres;
            info[i].coeffs.sigma = r.sig;
            info[i].coeffs.alpha = r.alp;
            info[i].coeffs.kappa_ub = r.kap;
            info[i].coeffs.flat = r.flat;
        }
        if (r.status == -2) bad = true;
        else if (!r.converged) nc = true;
    }
    if (bad) return fail(ctx, SGN_EDOMAIN, "non-positive depth or non-finite data in a batched system");
    if (nc) return fail(ctx, SGN_ENOCONV, "a batched system did not reach the tolerance");
    return SGN_OK;
}

size_t sgn_batch_step_workspace_bytes(int32_t nitems, const int32_t* n, int32_t precision) {
    if (nitems < 0 || (nitems > 0 && !n)) return 0;
    if (precision != SGN_FP64 && precision != SGN_MIXED) return 0;
    for (int i = 0; i < nitems; ++i)
        if (!batch_size_ok(n[i])) return 0;
    return step_layout(nitems, n, precision == SGN_MIXED ? BATCH_MIXED : BATCH_FP64).total;
}

sgn_status sgn_batch_step_rk4(sgn_ctx* ctx, int32_t nitems, const int32_t* n, const double* L, const double* dt,
                              const int32_t* nsteps, const double* h, double* eta, double* u,
                              const sgn_solve_opts* opts, sgn_step_info* info, sgn_status* status, void* ws) {
    if (!ctx) return SGN_EINVAL;
    if (nitems < 0) return fail(ctx, SGN_EINVAL, "nitems < 0");
    if (nitems == 0) return SGN_OK;
    if (!n || !L || !dt || !nsteps || !h || !eta || !u || !ws) return fail(ctx, SGN_EINVAL, "null pointer");
    const sgn_solve_opts o = opts ? *opts : default_opts();
    if (o.method != SGN_PCG) return fail(ctx, SGN_EUNSUPPORTED, "stepper solves use PCG");
    if (o.precision != SGN_FP64 && o.precision != SGN_MIXED) return fail(ctx, SGN_EINVAL, "unknown precision");
    if (!(o.tol > 0.0) || o.max_iter < 1) return fail(ctx, SGN_EINVAL, "tol must be > 0 and max_iter >= 1");
    if (o.coeff_kind != SGN_COEFF_OPTIMAL && o.coeff_kind != SGN_COEFF_REPLACEMENT)
        return fail(ctx, SGN_EINVAL, "bad coeff_kind");
    if (o.guess != SGN_GUESS_PREVIOUS && o.guess != SGN_GUESS_EXTRAPOLATE) return fail(ctx, SGN_EINVAL, "bad guess");
    int nmax = 0;
    for (int i = 0; i < nitems; ++i) {
        if (!batch_size_ok(n[i])) return fail(ctx, SGN_EUNSUPPORTED, "batch sizes must be powers of two in [2, 8192]");
        if (!(L[i] > 0.0) || !std::isfinite(L[i])) return fail(ctx, SGN_EINVAL, "periods must be positive");
        if (!std::isfinite(dt[i]) || nsteps[i] < 0) return fail(ctx, SGN_EINVAL, "bad step arguments");
        nmax = std::max(nmax, (int)n[i]);
    }
    const int mode = o.precision == SGN_MIXED ? BATCH_MIXED : BATCH_FP64;
    const StepLayout lay = step_layout(nitems, n, mode);
    sgn_status s;
    if ((s = batch_staging(ctx, BATCH_HEAD + std::max(sizeof(StepItem), sizeof(StepResult)) * (size_t)nitems)) !=
        SGN_OK)
        return s;
    char* base = static_cast<char*>(ws);
    double* data = reinterpret_cast<double*>(base + lay.data);
    // states in the caller's order for offsets; the table runs longest first
    // (points times steps) so that workgroups take the long runs first
    std::vector<long long> off(nitems), dso(nitems);
    long long po = 0, pd = 0;
    for (int i = 0; i < nitems; ++i) {
        off[i] = po;
        dso[i] = pd;
        po += n[i];
        pd += step_item_doubles(n[i], mode);
    }
    // the table runs longest first (points times steps) so that workgroups take
    // the long runs first
    std::vector<int> order(nitems);
    for (int i = 0; i < nitems; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (long long)n[a] * nsteps[a] > (long long)n[b] * nsteps[b];
    });
    std::memset(ctx->hbatch, 0, BATCH_HEAD);   // the queue counter
    StepItem* hit = reinterpret_cast<StepItem*>(static_cast<char*>(ctx->hbatch) + BATCH_HEAD);
    for (int q = 0; q < nitems; ++q) {
        const int i = order[q];
        StepItem& it = hit[q];
        std::memset(&it, 0, sizeof(it));
        const long long a = step_align(n[i]);
        double* p = data + dso[i];
        auto take = [&]() {
            double* r = p;
            p += a;
            return r;
        };
        it.eta = eta + off[i];
        it.u = u + off[i];
        it.h = h + off[i];
        it.hx = take();
        it.U = take();
        for (int k = 0; k < 4; ++k) {
            it.fe[k] = take();
            it.fU[k] = take();
        }
        it.eta_s = take();
        it.U_s = take();
        it.u_s = take();
        it.base = take();
        for (int k = 0; k < STEP_SLOTS; ++k) {
            it.off[k][0] = take();
            it.off[k][1] = take();
        }
        it.scr = p;
        it.L = L[i];
        it.dt = dt[i];
        it.n = n[i];
        it.index = i;
        it.nsteps = nsteps[i];
    }
    HIPCHK(ctx, hipMemcpyAsync(base, ctx->hbatch, BATCH_HEAD + sizeof(StepItem) * (size_t)nitems,
                               hipMemcpyHostToDevice, ctx->stream));
    const StepItem* d_items = reinterpret_cast<const StepItem*>(base + lay.items);
    StepResult* d_res = reinterpret_cast<StepResult*>(base + lay.results);
    int* d_queue = reinterpret_cast<int*>(base);   // counters at bytes 0 and 128
    const BatchParams prm = step_params(o, nitems);
    const bool ex = o.guess == SGN_GUESS_EXTRAPOLATE;
    {
        // every run of a batched call on 512 threads, whatever its size: a run's
        // reductions, and so its result, do not depend on the batch
        ProfScope ps(ctx, SGN_KERNEL_BATCH_STEP);
        if ((s = launch_batch_rk4(ctx, ctx->stream, BATCH_CALL_THREADS, d_items, nitems, nmax, mode, 0, prm, ex, d_res,
                                  d_queue)) != SGN_OK)
            return s;
    }
    StepResult* hres = static_cast<StepResult*>(ctx->hbatch);
    HIPCHK(ctx, hipMemcpyAsync(hres, base + lay.results, sizeof(StepResult) * (size_t)nitems, hipMemcpyDeviceToHost,
                               ctx->stream));
    if ((s = wait_stream(ctx)) != SGN_OK) return s;
    bool bad = false, nc = false;
    for (int i = 0; i < nitems; ++i) {
        const StepResult& r = hres[i];
        if (info) {
            sgn_step_info& f = info[i];
            std::memset(&f, 0, sizeof(f));
            f.solves = r.solves;
            f.iters = r.iters;
            f.max_iters = r.max_iters;
            f.converged = r.converged;
            double t = 0.0;
            for (int k = 0; k < r.steps; ++k) t += dt[i];
            f.t = t;
            f.steps_done = r.steps;
        }
        const sgn_status si = r.status == -2 ? SGN_EDOMAIN : r.status == -3 ? SGN_ENOCONV : SGN_OK;
        if (status) status[i] = si;
        bad = bad || si == SGN_EDOMAIN;
        nc = nc || si == SGN_ENOCONV;
    }
    if (bad) return fail(ctx, SGN_EDOMAIN, "non-positive depth or non-finite data in a batched run");
    if (nc) return fail(ctx, SGN_ENOCONV, "a batched run's solve did not reach the tolerance");
    return SGN_OK;
}

sgn_status sgn_rhs(sgn_ctx* ctx, const sgn_grid* grid, const double* eta, const double* h, const double* grad_h,
                   const double* u, double* eta_t, double* U_t, void* ws) {
    if (!ctx) return SGN_EINVAL;
    Dims d;
    sgn_status s = check_grid(ctx, grid, &d);
    if (s != SGN_OK) return s;
    if (!eta || !h || !grad_h || !u || !eta_t || !U_t || !ws) return fail(ctx, SGN_EINVAL, "null pointer");
    if (d.bc != SGN_BC_WALLS) return rhs_dispatch(ctx, d, eta, grad_h, u, eta_t, U_t, ws);
    if (d.D == 2) {
        // a 2D grid between walls on its own points: the fields in transform order
        // through the periodic row passes and the wall column operators
        Dims n = d;
        n.bc = SGN_BC_PERIODIC;
        n.tpx = 0.5 * kTwoPi / d.Lx;
        n.tpy = 0.5 * kTwoPi / d.Ly;
        Carve cv(ws);
        WallStateBufs o;
        carve_wall_state(cv, d, &o);   // h unused; gh, eta, u in order, U (the U_t result)
        double* et = o.h;
        if ((s = wall_order(ctx, d, eta, o.eta, false, true)) != SGN_OK) return s;
        if ((s = wall_order(ctx, d, grad_h, o.gh, true, true)) != SGN_OK) return s;
        if ((s = wall_order(ctx, d, u, o.u, true, true)) != SGN_OK) return s;
        ctx->wall_native = true;
        s = rhs_dispatch(ctx, n, o.eta, o.gh, o.u, et, o.U, static_cast<char*>(ws) + align_up(cv.off, 256));
        ctx->wall_native = false;
        if (s != SGN_OK) return s;
        if ((s = wall_order(ctx, d, et, eta_t, false, false)) != SGN_OK) return s;
        return wall_order(ctx, d, o.U, U_t, true, false);
    }
    // between walls: the periodic right-hand side of the reflected fields, restricted
    const Dims t = twin_dims(d);
    WallBufs w;
    Carve cv(ws);
    carve_walls(cv, t, &w);
    if ((s = wall_reflect(ctx, d, eta, w.eta, false)) != SGN_OK) return s;
    if ((s = wall_reflect(ctx, d, grad_h, w.gh, true)) != SGN_OK) return s;
    if ((s = wall_reflect(ctx, d, u, w.f, true)) != SGN_OK) return s;
    if ((s = rhs_dispatch(ctx, t, w.eta, w.gh, w.f, w.et, w.u, w.ws)) != SGN_OK) return s;
    if ((s = wall_restrict(ctx, d, w.et, eta_t, false)) != SGN_OK) return s;
    return wall_restrict(ctx, d, w.u, U_t);
}

}  // extern "C"

namespace {
// One stepping call of a state between walls: its fields reflected onto the twin,
// the call run on the twin's periodic state, the fields restricted back (also
// after a failed solve, as a periodic state leaves its fields).
template <typename F>
sgn_status wall_steps(sgn_state* st, F call) {
    sgn_ctx* ctx = st->ctx;
    const Dims& d = st->d;
    sgn_state* tw = st->twin;
    sgn_status s;
    if (st->path != 1) {   // the other sub-state ran last: its histories are not this one's
        tw->t = st->t;
        tw->steps = st->steps;
        tw->kind = 0;
        tw->gx_mode = -1;
        st->path = 1;
    }
    if ((s = wall_reflect(ctx, d, st->eta, tw->eta, false)) != SGN_OK) return s;
    if ((s = wall_reflect(ctx, d, st->U, tw->U, true)) != SGN_OK) return s;
    if ((s = wall_reflect(ctx, d, st->u, tw->u, true)) != SGN_OK) return s;
    ctx->wall_twin = true;
    s = call(tw);
    ctx->wall_twin = false;
    sgn_status r = wall_restrict(ctx, d, tw->eta, st->eta, false);
    if (r == SGN_OK) r = wall_restrict(ctx, d, tw->U, st->U);
    if (r == SGN_OK) r = wall_restrict(ctx, d, tw->u, st->u);
    st->t = tw->t;
    st->steps = tw->steps;
    return s != SGN_OK ? s : r;
}

// A stepping call of a 2D wall state on the grid's own points: eta, U, u go to
// transform order, the periodic stepper runs with the wall column passes
// (ctx->wall_native) and the fields come back to grid order.
template <typename F>
sgn_status wall_native_steps(sgn_state* st, F call) {
    sgn_ctx* ctx = st->ctx;
    const Dims& d = st->d;
    sgn_state* nt = st->nat;
    sgn_status s;
    if (st->path != 2) {
        nt->t = st->t;
        nt->steps = st->steps;
        nt->kind = 0;
        nt->gx_mode = -1;
        st->path = 2;
    }
    if ((s = wall_order(ctx, d, st->eta, nt->eta, false, true)) != SGN_OK) return s;
    if ((s = wall_order(ctx, d, st->U, nt->U, true, true)) != SGN_OK) return s;
    if ((s = wall_order(ctx, d, st->u, nt->u, true, true)) != SGN_OK) return s;
    ctx->wall_native = true;
    s = call(nt);
    ctx->wall_native = false;
    sgn_status r = wall_order(ctx, d, nt->eta, st->eta, false, false);
    if (r == SGN_OK) r = wall_order(ctx, d, nt->U, st->U, true, false);
    if (r == SGN_OK) r = wall_order(ctx, d, nt->u, st->u, true, false);
    st->t = nt->t;
    st->steps = nt->steps;
    return s != SGN_OK ? s : r;
}

// Whether a stepping call of a wall state runs on the grid's own points.
bool wall_native_call(const sgn_state* st, const sgn_solve_opts* opts) {
    const sgn_solve_opts o = opts ? *opts : default_opts();
    return st->nat && o.method == SGN_PCG && o.precision == SGN_FP64;
}

}  // namespace

extern "C" {

size_t sgn_dealias_workspace_bytes(const sgn_grid* grid) {
    Dims d;
    if (check_grid(nullptr, grid, &d) != SGN_OK || d.bc != SGN_BC_PERIODIC || !dealias_supported(d)) return 0;
    Carve cv(nullptr);
    return carve_dealias(cv, d, nullptr) + 256;
}

sgn_status sgn_rhs_dealiased(sgn_ctx* ctx, const sgn_grid* grid, const double* eta, const double* h,
                             const double* grad_h, const double* u, double* eta_t, double* U_t, void* dws) {
    if (!ctx) return SGN_EINVAL;
    Dims d;
    sgn_status s = check_grid(ctx, grid, &d);
    if (s != SGN_OK) return s;
    if ((s = require_periodic(ctx, d)) != SGN_OK) return s;
    if (!dealias_supported(d)) return fail(ctx, SGN_EUNSUPPORTED, "de-aliasing: grid too large to pad");
    if (!eta || !h || !grad_h || !u || !eta_t || !U_t || !dws) return fail(ctx, SGN_EINVAL, "null pointer");
    DealiasBufs b;
    Carve cv(dws);
    carve_dealias(cv, d, &b);
    if ((s = dealias_pad_gh(ctx, d, grad_h, b)) != SGN_OK) return s;
    return rhs_dealiased(ctx, d, eta, u, eta_t, U_t, b);
}

sgn_status sgn_state_set_dealias(sgn_ctx* ctx, sgn_state* st, void* dws) {
    if (!ctx || !st || st->ctx != ctx) return SGN_EINVAL;
    if (st->twin) return fail(ctx, SGN_EUNSUPPORTED, "de-aliasing takes periodic grids only");
    if (dws && !dealias_supported(st->d)) return fail(ctx, SGN_EUNSUPPORTED, "de-aliasing: grid too large to pad");
    // a multistep history holds right-hand sides of the form used so far
    st->kind = 0;
    if (!dws) {
        st->dealias = 0;
        return SGN_OK;
    }
    Carve cv(dws);
    carve_dealias(cv, st->d, &st->dl);
    sgn_status s = dealias_pad_gh(ctx, st->d, st->gh, st->dl);
    st->dealias = s == SGN_OK ? 1 : 0;
    return s;
}

size_t sgn_state_workspace_bytes(const sgn_grid* grid, int32_t precision) {
    (void)precision;
    Dims d;
    if (check_grid(nullptr, grid, &d) != SGN_OK) return 0;
    Carve cv(nullptr);
    if (d.bc == SGN_BC_WALLS) {
        // the layout of sgn_state_create: the twin's reflected fields, the twin's
        // state, and in 2D the fields in transform order and their state
        const Dims t = twin_dims(d);
        Carve c1(nullptr), c2(nullptr), c3(nullptr), c4(nullptr);
        size_t n = align_up(carve_wall_state(c1, t, nullptr), 256) + align_up(carve_state(c2, t, nullptr), 256);
        if (d.D == 2) n += align_up(carve_wall_state(c3, d, nullptr), 256) + carve_state(c4, d, nullptr);
        return n + 256;
    }
    return carve_state(cv, d, nullptr) + 256;
}

sgn_status sgn_state_create(sgn_ctx* ctx, const sgn_grid* grid, const double* h, const double* grad_h,
                            int32_t flat, double* eta, double* U, double* u, void* state_ws, void* ws,
                            sgn_state** out) {
    if (!ctx || !out) return SGN_EINVAL;
    *out = nullptr;
    Dims d;
    sgn_status s = check_grid(ctx, grid, &d);
    if (s != SGN_OK) return s;
    if (!h || !grad_h || !eta || !U || !u || !state_ws || !ws) return fail(ctx, SGN_EINVAL, "null pointer");
    if (d.bc == SGN_BC_WALLS) {
        // the twin's periodic state over the reflected fields; the caller's d_ws
        // (sgn_workspace_bytes of the wall grid) is larger than the twin's own
        const Dims t = twin_dims(d);
        sgn_grid tg = *grid;
        tg.bc = SGN_BC_PERIODIC;
        tg.nx = t.nx;
        tg.ny = t.ny;
        tg.Lx = t.Lx;
        tg.Ly = t.Ly;
        Carve cv(state_ws);
        WallStateBufs wb;
        carve_wall_state(cv, t, &wb);
        if ((s = wall_reflect(ctx, d, h, wb.h, false)) != SGN_OK) return s;
        if ((s = wall_reflect(ctx, d, grad_h, wb.gh, true)) != SGN_OK) return s;
        sgn_state* tw = nullptr;
        void* tws = static_cast<char*>(state_ws) + align_up(cv.off, 256);
        if ((s = sgn_state_create(ctx, &tg, wb.h, wb.gh, flat, wb.eta, wb.U, wb.u, tws, ws, &tw)) != SGN_OK)
            return s;
        sgn_state* st = new (std::nothrow) sgn_state();
        if (!st) {
            delete tw;
            return fail(ctx, SGN_ENOMEM, "host allocation failed");
        }
        st->ctx = ctx;
        st->grid = *grid;
        st->d = d;
        st->h = h;
        st->gh = grad_h;
        st->flat = flat ? 1 : 0;
        st->eta = eta;
        st->U = U;
        st->u = u;
        st->ws = ws;
        st->twin = tw;
        st->wb = wb;
        if (d.D == 2) {
            // the state on the grid's own points: h and grad h in transform order
            // once, its own stepping buffers after the twin's
            Carve ct(nullptr);
            const size_t tsz = align_up(carve_state(ct, t, nullptr), 256);
            char* nbase = static_cast<char*>(tws) + tsz;
            Carve cn(nbase);
            WallStateBufs nb;
            carve_wall_state(cn, d, &nb);
            if ((s = wall_order(ctx, d, h, nb.h, false, true)) != SGN_OK || (s = wall_order(ctx, d, grad_h, nb.gh, true, true)) != SGN_OK) {
                delete st;
                return s;
            }
            sgn_grid ng = *grid;
            ng.bc = SGN_BC_PERIODIC;
            sgn_state* nt = nullptr;
            if ((s = sgn_state_create(ctx, &ng, nb.h, nb.gh, flat, nb.eta, nb.U, nb.u, nbase + align_up(cn.off, 256),
                                      ws, &nt)) != SGN_OK) {
                delete st;
                return s;
            }
            // wavenumbers of the slots: s pi / L
            nt->d.tpx = 0.5 * kTwoPi / d.Lx;
            nt->d.tpy = 0.5 * kTwoPi / d.Ly;
            st->nat = nt;
            st->nb = nb;
        }
        *out = st;
        return SGN_OK;
    }
    sgn_state* st = new (std::nothrow) sgn_state();
    if (!st) return fail(ctx, SGN_ENOMEM, "host allocation failed");
    st->ctx = ctx;
    st->grid = *grid;
    st->d = d;
    st->h = h;
    st->gh = grad_h;
    st->flat = flat ? 1 : 0;
    st->eta = eta;
    st->U = U;
    st->u = u;
    st->ws = ws;
    Carve cv(state_ws);
    carve_state(cv, d, &st->b);
    st->t = 0.0;
    st->steps = 0;
    st->kind = 0;
    st->gx_mode = -1;   // the first stepping call sets mode and dt and clears the history
    st->gx_dt = 0.0;
    *out = st;
    return SGN_OK;
}

void sgn_state_destroy(sgn_state* st) { delete st; }

sgn_status sgn_step_rk4(sgn_ctx* ctx, sgn_state* st, double dt, int32_t nsteps, const sgn_solve_opts* opts,
                        sgn_step_info* info) {
    if (!ctx || !st || st->ctx != ctx) return SGN_EINVAL;
    if (st->twin && wall_native_call(st, opts))
        return wall_native_steps(st, [&](sgn_state* nt) { return sgn_step_rk4(ctx, nt, dt, nsteps, opts, info); });
    if (st->twin)
        return wall_steps(st, [&](sgn_state* tw) { return sgn_step_rk4(ctx, tw, dt, nsteps, opts, info); });
    if (nsteps < 0 || !std::isfinite(dt)) return fail(ctx, SGN_EINVAL, "bad step arguments");
    const sgn_solve_opts o = opts ? *opts : default_opts();
    if (o.guess != SGN_GUESS_PREVIOUS && o.guess != SGN_GUESS_EXTRAPOLATE) return fail(ctx, SGN_EINVAL, "bad guess");
    guess_prepare(st, o, dt);
    sgn_step_info acc;
    info_init(&acc);
    st->kind = 0;  // a multistep history does not survive other steps
    sgn_status s = SGN_OK;
    if (rk4_block_ok(st, o)) {
        if (nsteps > 0) s = rk4_block(st, dt, nsteps, o, &acc);
    } else {
        for (int n = 0; n < nsteps && s == SGN_OK; ++n) s = rk4_one(st, dt, o, &acc, false);
    }
    info_finish(st, &acc, info);
    return s;
}

sgn_status sgn_step_ab(sgn_ctx* ctx, sgn_state* st, int32_t order, double dt, int32_t nsteps,
                       const sgn_solve_opts* opts, sgn_step_info* info) {
    if (!ctx || !st || st->ctx != ctx) return SGN_EINVAL;
    if (st->twin && wall_native_call(st, opts))
        return wall_native_steps(st,
                                 [&](sgn_state* nt) { return sgn_step_ab(ctx, nt, order, dt, nsteps, opts, info); });
    if (st->twin)
        return wall_steps(st, [&](sgn_state* tw) { return sgn_step_ab(ctx, tw, order, dt, nsteps, opts, info); });
    if (nsteps < 0 || order < 2 || order > 4 || !std::isfinite(dt)) return fail(ctx, SGN_EINVAL, "bad AB arguments");
    const sgn_solve_opts o = opts ? *opts : default_opts();
    if (o.guess != SGN_GUESS_PREVIOUS && o.guess != SGN_GUESS_EXTRAPOLATE) return fail(ctx, SGN_EINVAL, "bad guess");
    guess_prepare(st, o, dt);
    // b_j, j = 0 .. s-1 (Table LMMCoeffs)
    static const double B[5][4] = {{0, 0, 0, 0},
                                   {0, 0, 0, 0},
                                   {-1.0 / 2.0, 3.0 / 2.0, 0, 0},
                                   {5.0 / 12.0, -16.0 / 12.0, 23.0 / 12.0, 0},
                                   {-9.0 / 24.0, 37.0 / 24.0, -59.0 / 24.0, 55.0 / 24.0}};
    sgn_step_info acc;
    info_init(&acc);
    if (st->kind != 1 || st->ab_order != order || st->hist_dt != dt) {
        st->kind = 1;
        st->ab_order = order;
        st->hist_dt = dt;
        st->ab_count = 0;
        st->ab_head = 0;
        st->gx_count[GUESS_AB] = 0;
    }
    const Dims& d = st->d;
    StateBufs& b = st->b;
    const size_t N = d.N, DN = (size_t)d.D * d.N;
    sgn_status s = SGN_OK;
    for (int n = 0; n < nsteps; ++n) {
        const int slot = st->ab_head & 3;
        if ((s = state_rhs(st, st->eta, st->u, b.ab_fe[slot], b.ab_fU[slot])) != SGN_OK) break;
        st->ab_head += 1;
        if (st->ab_count < order) st->ab_count += 1;
        if (st->ab_count < order) {
            // start-up: an RK4 step with the same dt; f at this level is its first stage
            if ((s = copy_d(ctx, b.rk_fe[0], b.ab_fe[slot], N)) != SGN_OK) break;
            if ((s = copy_d(ctx, b.rk_fU[0], b.ab_fU[slot], DN)) != SGN_OK) break;
            if ((s = rk4_one(st, dt, o, &acc, true)) != SGN_OK) break;
            continue;
        }
        std::vector<const double*> fe, fU;
        std::vector<double> c;
        for (int j = 0; j < order; ++j) {
            const int sl = (st->ab_head - order + j) & 3;
            fe.push_back(b.ab_fe[sl]);
            fU.push_back(b.ab_fU[sl]);
            c.push_back(B[order][j]);
        }
        if ((s = lincomb(ctx, N, st->eta, dt, fe, c, st->eta)) != SGN_OK) break;
        if ((s = lincomb(ctx, DN, st->U, dt, fU, c, st->U)) != SGN_OK) break;
        // as in RK4: the step counts even if its solve fails (u: the last iterate)
        s = stage_solve(st, GUESS_AB, st->eta, st->U, st->u, o, &acc);
        if (s == SGN_OK || s == SGN_ENOCONV || s == SGN_EDOMAIN) {
            st->t += dt;
            st->steps += 1;
        }
        if (s != SGN_OK) break;
    }
    if (s != SGN_OK) st->kind = 0;   // the history no longer holds converged levels
    info_finish(st, &acc, info);
    return s;
}

sgn_status sgn_step_linimp(sgn_ctx* ctx, sgn_state* st, double dt, int32_t nsteps, const sgn_coeffs* fixed,
                           const sgn_solve_opts* opts, sgn_step_info* info) {
    if (!ctx || !st || st->ctx != ctx) return SGN_EINVAL;
    if (st->twin)
        return wall_steps(st, [&](sgn_state* tw) { return sgn_step_linimp(ctx, tw, dt, nsteps, fixed, opts, info); });
    if (nsteps < 0 || !std::isfinite(dt)) return fail(ctx, SGN_EINVAL, "bad step arguments");
    if (fixed && !(fixed->sigma > 0.0 && fixed->alpha > 0.0)) return fail(ctx, SGN_EINVAL, "bad fixed coefficients");
    const sgn_solve_opts o = opts ? *opts : default_opts();
    if (o.guess != SGN_GUESS_PREVIOUS && o.guess != SGN_GUESS_EXTRAPOLATE) return fail(ctx, SGN_EINVAL, "bad guess");
    guess_prepare(st, o, dt);
    sgn_step_info acc;
    info_init(&acc);
    const LinimpScheme q = scheme_sbdf2();
    sgn_status s = st->d.D == 1 ? linimp_steps<1>(st, q, -1.0, 1.0, dt, nsteps, fixed, o, &acc)
                                : linimp_steps<2>(st, q, -1.0, 1.0, dt, nsteps, fixed, o, &acc);
    if (s != SGN_OK) st->kind = 0;
    if (s == SGN_OK) HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    info_finish(st, &acc, info);
    return s;
}

sgn_status sgn_linimp3_choose(double kappa, double margin, double* r, double* theta) {
    if (!r || !theta || !(kappa >= 1.0) || !(margin >= 1.0) || !std::isfinite(kappa) || !std::isfinite(margin))
        return SGN_EINVAL;
    const double need = kappa * margin * margin;
    auto ratio = [](double q) {
        double lo, hi;
        sbdf3r_interval(q, &lo, &hi);
        return hi / lo;
    };
    double rr = 0.0;
    if (ratio(0.0) < need) {
        // the ratio grows monotonically from 16/7 at r = 0 without bound as r -> 1
        double a = 0.0, b = 1.0 - 1e-15;
        for (int it = 0; it < 200; ++it) {
            const double m = 0.5 * (a + b);
            if (ratio(m) >= need)
                b = m;
            else
                a = m;
        }
        rr = b;
    }
    double lo, hi;
    sbdf3r_interval(rr, &lo, &hi);
    *r = rr;
    *theta = 1.0 / std::sqrt(lo * hi * kappa);
    return SGN_OK;
}

sgn_status sgn_step_linimp3(sgn_ctx* ctx, sgn_state* st, double r, double theta, double dt, int32_t nsteps,
                            const sgn_coeffs* fixed, const sgn_solve_opts* opts, sgn_step_info* info) {
    if (!ctx || !st || st->ctx != ctx) return SGN_EINVAL;
    if (st->twin)
        return wall_steps(st, [&](sgn_state* tw) {
            return sgn_step_linimp3(ctx, tw, r, theta, dt, nsteps, fixed, opts, info);
        });
    if (nsteps < 0 || !std::isfinite(dt)) return fail(ctx, SGN_EINVAL, "bad step arguments");
    if (!(r >= 0.0 && r < 1.0) || !(theta > 0.0) || !std::isfinite(theta))
        return fail(ctx, SGN_EINVAL, "r must lie in [0, 1) and theta be > 0");
    if (fixed && !(fixed->sigma > 0.0 && fixed->alpha > 0.0)) return fail(ctx, SGN_EINVAL, "bad fixed coefficients");
    const sgn_solve_opts o = opts ? *opts : default_opts();
    if (o.guess != SGN_GUESS_PREVIOUS && o.guess != SGN_GUESS_EXTRAPOLATE) return fail(ctx, SGN_EINVAL, "bad guess");
    guess_prepare(st, o, dt);
    sgn_step_info acc;
    info_init(&acc);
    const LinimpScheme q = scheme_sbdf3r(r);
    sgn_status s = st->d.D == 1 ? linimp_steps<1>(st, q, r, theta, dt, nsteps, fixed, o, &acc)
                                : linimp_steps<2>(st, q, r, theta, dt, nsteps, fixed, o, &acc);
    if (s != SGN_OK) st->kind = 0;
    if (s == SGN_OK) HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    info_finish(st, &acc, info);
    return s;
}

}  // extern "C"
