// Wave-private row transforms for 2D rows of nx = 1024 points (M = 512
// complex points per real row), and the Krylov row pass built on them.
//
// The block-wide Stockham engine of sgn_device.h spreads one row over several
// waves and pays two block barriers per radix pass.  Here one wave (64 lanes,
// eight complex entries per lane) owns one field of one row: the 512-point
// transform is three radix-8 stages in registers with two exchanges through a
// wave-private LDS region, so no block barrier sits inside a transform and the
// waves of a CU drift apart, overlapping one wave's loads with another's
// arithmetic.  Stage decomposition (n = l + 64 m, k = k1 + 8 j1 + 64 j2,
// l = l1 + 8 l2):
//   X[k1 + 8 j1 + 64 j2] = sum_l1 W8^{l1 j2} W64^{l1 j1}
//                          sum_l2 W8^{l2 j1} W512^{l k1} sum_m W8^{m k1} x[l + 64 m].
// Input and output both sit in the natural layout: lane l holds index l + 64 s
// in slot s.  The real-to-complex split of section 6.1's transforms (a real row
// of nx points as M complex points) pairs index k with M - k, which another lane
// holds; the pair is exchanged through the same LDS region.
#pragma once
#include "sgn_device.h"
#include "sgn_kernels.h"

namespace sgn {

constexpr int WROW_NX = 1024;   // real row length taken by the wave row pass
constexpr int WROW_M = 512;     // complex transform length
constexpr int WROW_BUF = 584;   // LDS entries per field wave (padded exchange layouts)
constexpr int WROW_S1 = 72;     // first exchange: row stride of the (k1, l) layout
constexpr int WROW_S2 = 73;     // second exchange: row stride of the (j1, lambda) layout

// Orders this wave's LDS accesses around a cross-lane exchange: LDS performs
// one wave's accesses in issue order, so only the compiler needs fencing.  The
// fences name LDS only, so global loads in flight are not waited for.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}



// v[k] *= a^k for k = 1..7 from a, a^2, a^4 (the conjugates for the inverse):
// each slot is multiplied by the factors of its binary digits in turn, so no
// table of powers is held in registers.
template <typename T>
__device__ __forceinline__ void wave_twiddle7(cpx<T> (&v)[8], cpx<T> a1, cpx<T> a2, cpx<T> a4, bool inverse) {
    if (inverse) {
        a1 = cj(a1);
        a2 = cj(a2);
        a4 = cj(a4);
    }
#pragma unroll
    for (int k = 1; k < 8; ++k) {
        if (k & 1) v[k] = v[k] * a1;
        if (k & 2) v[k] = v[k] * a2;
        if (k & 4) v[k] = v[k] * a4;
    }
}

// Per-block LDS table of the twiddle bases the wave transforms read, filled once
// at block start from the global table, so no stage waits on an L2 access.
template <typename T>
struct WaveTwl {
    cpx<T> a[3][64];  // W512^{l}, W512^{2l}, W512^{4l}      (first stage, l = lane)
    cpx<T> b[3][8];   // W64^{l1}, W64^{2 l1}, W64^{4 l1}    (second stage, l1 = lane & 7)
    cpx<T> r[64];     // W1024^{l}                          (real-to-complex split)
};
constexpr int WAVE_TWL_ENTRIES = 3 * 64 + 3 * 8 + 64;

// Entry e of the table (flat index over a, b, r), read from the global table.
template <typename T>
__device__ __forceinline__ cpx<T> wave_twl_entry(const cpx<T>* __restrict__ tw_all, int e) {
    const cpx<T>* t512 = tw_size(tw_all, WROW_M);
    if (e < 192) return t512[(1 << (e >> 6)) * (e & 63)];
    if (e < 216) return t512[8 * (1 << ((e - 192) >> 3)) * ((e - 192) & 7)];
    return tw_size(tw_all, WROW_NX)[e - 216];
}

// W16^j, j = 0..7: W1024^{lane + 64 j} = W1024^{lane} W16^j.
template <typename T>
__device__ __forceinline__ cpx<T> w16(int j) {
    const T c = (T)0.92387953251128675613, s = (T)0.38268343236508977173, r = (T)0.70710678118654752440;
    switch (j & 7) {
        case 0: return C<T>(1, 0);
        case 1: return C<T>(c, -s);
        case 2: return C<T>(r, -r);
        case 3: return C<T>(s, -c);
        case 4: return C<T>(0, -1);
        case 5: return C<T>(-s, -c);
        case 6: return C<T>(-r, -r);
        default: return C<T>(-c, -s);
    }
}

// The six twiddle bases of one lane's transform stages.
template <typename T>
struct WaveBases {
    cpx<T> a1, a2, a4;  // W512^{l}, W512^{2l}, W512^{4l}      (l = lane)
    cpx<T> b1, b2, b4;  // W64^{l1}, W64^{2 l1}, W64^{4 l1}    (l1 = lane & 7)
};
template <typename T>
__device__ __forceinline__ WaveBases<T> wave_bases(const WaveTwl<T>& tl, int lane) {
    const int l1 = lane & 7;
    return WaveBases<T>{tl.a[0][lane], tl.a[1][lane], tl.a[2][lane], tl.b[0][l1], tl.b[1][l1], tl.b[2][l1]};
}
// From the global table, for kernels whose waves run without a block barrier.
template <typename T>
__device__ __forceinline__ WaveBases<T> wave_bases(const cpx<T>* __restrict__ tw_all, int lane) {
    const cpx<T>* t512 = tw_size(tw_all, WROW_M);
    const int l1 = lane & 7;
    return WaveBases<T>{t512[lane], t512[2 * lane], t512[4 * lane], t512[8 * l1], t512[16 * l1], t512[32 * l1]};
}

// 512-point FFT of one field held by one wave.  In: v[s] = x[lane + 64 s];
// out: v[s] = X[lane + 64 s] (forward: exp(-i), inverse: exp(+i), unnormalised).
// Twiddles: per stage three bases a, a^2, a^4, the other powers by products.
// NR rows of one field held by one wave go through the stages in lockstep: their
// exchanges share the wave's synchronisations, and entry e of row r sits at
// buf[NR e + r], so the rows' entries of one exchange index are adjacent in LDS
// (one 16-byte access for two FP32 rows).  buf: NR WROW_BUF entries.
template <typename T, int NR>
__device__ __forceinline__ void wave_fft512_rows(cpx<T> (&v)[NR][8], cpx<T>* buf, const WaveBases<T>& wb,
                                                 int lane, bool inverse) {
    // first stage: 8-point DFT over m, twiddle W512^{l k1}; lane l holds k1 = 0..7
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        dft_small<T, 8>(v[r], inverse);
        wave_twiddle7(v[r], wb.a1, wb.a2, wb.a4, inverse);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int r = 0; r < NR; ++r) buf[NR * (k * WROW_S1 + lane) + r] = v[r][k];
    wave_lds_sync();
    // second stage: lane = l1 + 8 k1 takes l2 = 0..7 of l = l1 + 8 l2
    {
        const int l1 = lane & 7, k1 = lane >> 3;
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int r = 0; r < NR; ++r) v[r][q] = buf[NR * (k1 * WROW_S1 + l1 + 8 * q) + r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        dft_small<T, 8>(v[r], inverse);
        wave_twiddle7(v[r], wb.b1, wb.b2, wb.b4, inverse);   // W64^{l1 j1}
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int r = 0; r < NR; ++r) buf[NR * (j * WROW_S2 + lane + (lane >> 3)) + r] = v[r][j];
    wave_lds_sync();
    // third stage: lane = k1 + 8 j1 takes l1 = 0..7 (written by lane l1 + 8 k1)
    {
        const int k1 = lane & 7, j1 = lane >> 3;
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int r = 0; r < NR; ++r) v[r][q] = buf[NR * (j1 * WROW_S2 + q + 9 * k1) + r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < NR; ++r) dft_small<T, 8>(v[r], inverse);
}
template <typename T>
__device__ __forceinline__ void wave_fft512(cpx<T> (&v)[8], cpx<T>* buf, const WaveBases<T>& wb, int lane,
                                            bool inverse) {
    wave_fft512_rows<T, 1>(reinterpret_cast<cpx<T>(&)[1][8]>(v), buf, wb, lane, inverse);
}

// Entry e of NR consecutive rows of a transposed field (rows are its fast
// index, so the entries are adjacent): one 16-byte access for two FP32 rows.
template <typename T, int NR>
__device__ __forceinline__ void rows_load(const cpx<T>* p, cpx<T> (&x)[NR]) {
    if constexpr (NR == 2 && sizeof(T) == 4) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        x[0] = C<T>(q.x, q.y);
        x[1] = C<T>(q.z, q.w);
    } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) x[r] = p[r];
    }
}
template <typename T, int NR>
__device__ __forceinline__ void rows_store(cpx<T>* p, const cpx<T> (&x)[NR]) {
    if constexpr (NR == 2 && sizeof(T) == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(x[0].re, x[0].im, x[1].re, x[1].im);
    } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) p[r] = x[r];
    }
}

// Half spectrum of one real row (H layout: entry kx at Hrow[kx * ny], kx = 0..M)
// to the complex input of the inverse transform, Z_k = (X_k + X*_{M-k}) +
// i (X_k - X*_{M-k}) W1024^{-k}, Z_0 = (X_0 + X_M) + i (X_0 - X_M) on the real
// parts.  X: the loaded entries X[lane + 64 s]; XM: X[M] (lane 0).
// The loaded entries go to LDS and are read back with their mirrors, so they
// do not stay live in registers across the exchange.  NR rows in lockstep, LDS
// layout as in wave_fft512_rows.
template <typename T, int NR>
__device__ __forceinline__ void wave_c2r_split_rows(cpx<T> (&v)[NR][8], const cpx<T> (&X)[NR][8],
                                                    const cpx<T> (&XM)[NR], cpx<T>* buf, cpx<T> r1, int lane) {
    T x0[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
#pragma unroll
        for (int s = 0; s < 8; ++s) buf[NR * (lane + 64 * s) + r] = X[r][s];
        x0[r] = X[r][0].re;
    }
    wave_lds_sync();
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const cpx<T> wk = cj(r1 * w16<T>(s));
        const int m = (WROW_M - lane - 64 * s) & (WROW_M - 1);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const cpx<T> xk = buf[NR * (lane + 64 * s) + r];
            const cpx<T> xm = buf[NR * m + r];
            v[r][s] = (xk + cj(xm)) + mul_i((xk - cj(xm)) * wk);
        }
    }
    wave_lds_sync();
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r][0] = C<T>(x0[r] + XM[r].re, x0[r] - XM[r].re);
    }
}
template <typename T>
__device__ __forceinline__ void wave_c2r_split(cpx<T> (&v)[8], const cpx<T> (&X)[8], cpx<T> XM, cpx<T>* buf,
                                               cpx<T> r1, int lane) {
    const cpx<T> xm[1] = {XM};
    wave_c2r_split_rows<T, 1>(reinterpret_cast<cpx<T>(&)[1][8]>(v), reinterpret_cast<const cpx<T>(&)[1][8]>(X), xm,
                              buf, r1, lane);
}

// Forward transform output Z[lane + 64 s] (v) to the half spectrum,
// X_k = (Z_k + Z*_{M-k})/2 - i W1024^k (Z_k - Z*_{M-k})/2, X_0 and X_M from Z_0,
// each multiplied by scale and stored at Hrow[kx * ny] (NR rows: row r at
// Hrow + r, the rows' entries stored together).
template <typename T, int NR>
__device__ __forceinline__ void wave_r2c_store_rows(const cpx<T> (&v)[NR][8], cpx<T>* buf, cpx<T> r1, int lane,
                                                    cpx<T>* Hrow, int ny, T scale) {
    cpx<T> z0[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
#pragma unroll
        for (int s = 0; s < 8; ++s) buf[NR * (lane + 64 * s) + r] = v[r][s];
        z0[r] = v[r][0];
    }
    wave_lds_sync();
    const T half = (T)0.5;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int k = lane + 64 * s;
        const cpx<T> wk = r1 * w16<T>(s);
        const int m = (WROW_M - lane - 64 * s) & (WROW_M - 1);
        cpx<T> X[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const cpx<T> zk = buf[NR * k + r], zm = buf[NR * m + r];
            X[r] = half * (zk + cj(zm)) - half * mul_i(wk * (zk - cj(zm)));
            if (k == 0) X[r] = C<T>(zk.re + zk.im, 0);
            X[r] = scale * X[r];
        }
        rows_store<T, NR>(Hrow + (size_t)k * ny, X);
    }
    if (lane == 0) {
        cpx<T> X[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) X[r] = scale * C<T>(z0[r].re - z0[r].im, 0);
        rows_store<T, NR>(Hrow + (size_t)WROW_M * ny, X);
    }
}
template <typename T>
__device__ __forceinline__ void wave_r2c_store(const cpx<T> (&v)[8], cpx<T>* buf, cpx<T> r1, int lane,
                                               cpx<T>* Hrow, int ny, T scale) {
    wave_r2c_store_rows<T, 1>(reinterpret_cast<const cpx<T>(&)[1][8]>(v), buf, r1, lane, Hrow, ny, scale);
}

// Krylov row pass (the G apply's x-direction work, Def:G) on rows of 1024
// points: one block per NR consecutive rows, one wave per field (p_x, p_y,
// div p) holding the field's NR rows.  Each wave loads its field's half-spectrum
// rows, splits and inverse-transforms them, and leaves the real rows in its LDS
// region; after a block barrier wave f forms the pointwise products of the slots
// [3f, 3f + 3) of all three fields
//   a = eta p + grad h (eta^2/2 div p + eta beta),  w = eta^3/3 div p + eta^2/2 beta,
// beta = grad h . p, and the B-density eta|p|^2 + div p w + beta (eta^2/2 div p +
// eta beta) of the curvature p.Gp (section 3.1); after a second barrier each wave
// forward-transforms its field of (a, w) and stores it.  Launch: ny / NR blocks
// of 192 threads; part[part_base + block] receives the block's curvature sum.
// Three waves per SIMD: at 1024 rows and NR = 1 the whole grid (12 waves per CU)
// is then resident at once.  NR = 2 (FP32): the transposed H layout holds the
// two rows' entries of one kx side by side, so each lane moves 16 bytes per
// access instead of 8 and a wave's loads, stores and exchanges serve two rows.
template <typename T, int NR>
__global__ void __launch_bounds__(192) __attribute__((amdgpu_waves_per_eu(3))) k_pcg_r1w(int ny, const cpx<T>* __restrict__ tw,
                                                 SolveScal* __restrict__ sc, cpx<T>* H, size_t NS,
                                                 const T* __restrict__ eta, const T* __restrict__ gh,
                                                 double* __restrict__ part, int part_base) {
    static_assert(NR == 1 || (NR == 2 && sizeof(T) == 4), "two rows per wave in FP32 only");
    // eta and grad h of the wave's pointwise slots are loaded before the inverse
    // transform, so their latency hides behind it
    constexpr bool PF = true;
    // the stop flag is read here and tested after the twiddle table is staged,
    // so its latency hides behind the table's loads
    const int done = sc->done;
    __shared__ __align__(16) cpx<T> lds[3][NR * WROW_BUF];
    __shared__ WaveTwl<T> tl;
    __shared__ double red[4];
    const int f = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int y = xcd_remap(blockIdx.x, gridDim.x) * NR;
    cpx<T>* Hrow = H + (size_t)f * NS + y;
    cpx<T>* buf = lds[f];
    // FP64: twiddle table first (L2-resident; one L2 round trip per block instead
    // of one per transform stage), then the row's transposed loads (row loads in
    // flight across a block barrier were spilled to scratch by the compiler, so
    // the table's barrier comes before them).  FP32 has the registers to hold
    // the lane's seven twiddle bases: they are loaded with the row, no table.
    constexpr bool TWREG = sizeof(T) == 4;
    WaveBases<T> wbr;
    cpx<T> r1r;
    if (TWREG) {
        if (done) return;
        wbr = wave_bases<T>(tw, lane);
        r1r = tw_size(tw, WROW_NX)[lane];
    } else {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int e = threadIdx.x + i * blockDim.x;
            if (e < WAVE_TWL_ENTRIES) (&tl.a[0][0])[e] = wave_twl_entry<T>(tw, e);
        }
        block_lds_barrier();
        if (done) return;
    }
    auto bases = [&]() { return TWREG ? wbr : wave_bases<T>(tl, lane); };
    auto r1 = [&]() { return TWREG ? r1r : tl.r[lane]; };
    cpx<T> X[NR][8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        cpx<T> x[NR];
        rows_load<T, NR>(Hrow + (size_t)(lane + 64 * s) * ny, x);
#pragma unroll
        for (int r = 0; r < NR; ++r) X[r][s] = x[r];
    }
    cpx<T> XM[NR];
    if (lane == 0) {
        rows_load<T, NR>(Hrow + (size_t)WROW_M * ny, XM);
    } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) XM[r] = C<T>(0, 0);
    }
    cpx<T> v[NR][8];
    wave_c2r_split_rows<T, NR>(v, X, XM, buf, r1(), lane);
    const size_t npts = (size_t)WROW_NX * ny;
    const int m0 = 3 * f;
    const int ms = f == 2 ? 2 : 3;
    // row r of eta (grad h) as complex pairs: entry n at er[r WROW_M + n]
    const cpx<T>* er = reinterpret_cast<const cpx<T>*>(eta + (size_t)y * WROW_NX);
    const cpx<T>* gxr = reinterpret_cast<const cpx<T>*>(gh + (size_t)y * WROW_NX);
    const cpx<T>* gyr = reinterpret_cast<const cpx<T>*>(gh + npts + (size_t)y * WROW_NX);
    cpx<T> pe[NR][3], px[NR][3], py[NR][3];
    auto load_coeffs = [&]() {
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                if (i < ms) {
                    const int n = r * WROW_M + lane + 64 * (m0 + i);
                    pe[r][i] = er[n];
                    px[r][i] = gxr[n];
                    py[r][i] = gyr[n];
                }
            }
    };
    if (PF) load_coeffs();
    wave_fft512_rows<T, NR>(v, buf, bases(), lane, true);
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int r = 0; r < NR; ++r) buf[NR * (lane + 64 * s) + r] = v[r][s];
    block_lds_barrier();

    if (!PF) load_coeffs();
    double acc = 0.0;
    const T third = (T)1 / (T)3, half = (T)0.5;
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (i < ms) {
                const int n = NR * (lane + 64 * (m0 + i)) + r;
                cpx<T> p0 = lds[0][n], p1 = lds[1][n], dv = lds[2][n];
                const T et2[2] = {pe[r][i].re, pe[r][i].im};
                const T hx2[2] = {px[r][i].re, px[r][i].im};
                const T hy2[2] = {py[r][i].re, py[r][i].im};
                T a0[2], a1[2], ww[2];
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const T et = et2[s];
                    const T pxs = s ? p0.im : p0.re, pys = s ? p1.im : p1.re, dl = s ? dv.im : dv.re;
                    const T bt = hx2[s] * pxs + hy2[s] * pys;
                    const T e2 = et * et;
                    const T w1 = third * e2 * et * dl + half * e2 * bt;
                    const T w2 = half * e2 * dl + et * bt;
                    const double pp = (double)pxs * (double)pxs + (double)pys * (double)pys;
                    acc += (double)et * pp + (double)dl * (double)w1 + (double)bt * (double)w2;
                    a0[s] = et * pxs + hx2[s] * w2;
                    a1[s] = et * pys + hy2[s] * w2;
                    ww[s] = w1;
                }
                lds[0][n] = C<T>(a0[0], a0[1]);
                lds[1][n] = C<T>(a1[0], a1[1]);
                lds[2][n] = C<T>(ww[0], ww[1]);
            }
        }
    // the block's curvature sum: waves in order after the barrier that also
    // publishes the pointwise results
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) red[f] = acc;
    block_lds_barrier();
    if (part && threadIdx.x == 0) part[part_base + blockIdx.x] = red[0] + red[1] + red[2];
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r][s] = buf[NR * (lane + 64 * s) + r];
    wave_lds_sync();
    wave_fft512_rows<T, NR>(v, buf, bases(), lane, false);
    wave_r2c_store_rows<T, NR>(v, buf, r1(), lane, Hrow, ny, (T)1);
}

}  // namespace sgn

namespace sgn {

// ---------------------------------------------------------------------------
// Plain row transforms and the right-hand side's inverse row pass on rows of
// 1024 points, one wave per (field, row).  The plain passes need no exchange
// between waves, so their blocks hold WROW_WPB independent waves and no block
// barrier; the waves of a field take consecutive rows, so the transposed H
// lines of neighbouring rows are touched on one XCD.
// ---------------------------------------------------------------------------
constexpr int WROW_WPB = 4;

struct WaveRow {
    int f, y;
};
__device__ __forceinline__ WaveRow wave_row_of(int ny) {
    const int w = xcd_remap(blockIdx.x, gridDim.x) * WROW_WPB + (int)(threadIdx.x >> 6);
    const int f = w / ny;
    return WaveRow{f, w - f * ny};
}

// Forward transform of one real row held as v[s] = (x_2n, x_2n+1), n = lane + 64 s,
// into the half spectrum at Hrow[kx * ny], each value times scale.
template <typename T>
__device__ __forceinline__ void wave_row_forward(cpx<T> (&v)[8], cpx<T>* buf, const cpx<T>* __restrict__ tw,
                                                 int lane, cpx<T>* Hrow, int ny, T scale) {
    const WaveBases<T> wb = wave_bases<T>(tw, lane);
    const cpx<T> r1 = tw_size(tw, WROW_NX)[lane];
    wave_fft512<T>(v, buf, wb, lane, false);
    wave_r2c_store<T>(v, buf, r1, lane, Hrow, ny, scale);
}

// Inverse transform of the half-spectrum row at Hrow[kx * ny] into
// v[s] = (x_2n, x_2n+1), n = lane + 64 s (nx times the inverse DFT).
template <typename T>
__device__ __forceinline__ void wave_row_inverse(cpx<T> (&v)[8], cpx<T>* buf, const cpx<T>* __restrict__ tw,
                                                 int lane, const cpx<T>* Hrow, int ny) {
    cpx<T> X[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) X[s] = Hrow[(size_t)(lane + 64 * s) * ny];
    const cpx<T> XM = lane == 0 ? Hrow[(size_t)WROW_M * ny] : C<T>(0, 0);
    const WaveBases<T> wb = wave_bases<T>(tw, lane);
    const cpx<T> r1 = tw_size(tw, WROW_NX)[lane];
    wave_c2r_split<T>(v, X, XM, buf, r1, lane);
    wave_fft512<T>(v, buf, wb, lane, true);
}

// Forward row transforms of src.n physical fields (the k_rows_fwd contract:
// fields from cmb.first on are read as src + c1 a + c2 b).  Launch:
// src.n * ny / WROW_WPB blocks of 64 WROW_WPB threads.
template <typename T, typename Tin>
__global__ void __launch_bounds__(64 * WROW_WPB) k_rows_fwd_w(int ny, PtrList<const Tin, MAXF> src,
                                                              PtrList<cpx<T>, MAXF> dst,
                                                              const cpx<T>* __restrict__ tw, T scale,
                                                              RowCombo<Tin> cmb) {
    __shared__ cpx<T> ldsw[WROW_WPB][WROW_BUF];
    const int lane = threadIdx.x & 63;
    const WaveRow wr = wave_row_of(ny);
    if (wr.f >= src.n) return;
    cpx<T>* buf = ldsw[threadIdx.x >> 6];
    const size_t o = (size_t)wr.y * WROW_NX;
    const cpx<Tin>* sf = reinterpret_cast<const cpx<Tin>*>(src.p[wr.f] + o);
    const int k = wr.f - cmb.first;
    const bool comb = cmb.first >= 0 && k >= 0;
    cpx<T> v[8];
    if (comb) {
        const cpx<Tin>* ca = reinterpret_cast<const cpx<Tin>*>(cmb.a[k] + o);
        const cpx<Tin>* cb = cmb.b[k] ? reinterpret_cast<const cpx<Tin>*>(cmb.b[k] + o) : nullptr;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int n = lane + 64 * s;
            const cpx<Tin> x = sf[n], a = ca[n];
            double t0 = cmb.c1 * (double)a.re, t1 = cmb.c1 * (double)a.im;
            if (cb) {
                const cpx<Tin> b = cb[n];
                t0 += cmb.c2 * (double)b.re;
                t1 += cmb.c2 * (double)b.im;
            }
            v[s] = C<T>((T)((double)x.re + t0), (T)((double)x.im + t1));
        }
    } else {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const cpx<Tin> x = sf[lane + 64 * s];
            v[s] = C<T>((T)x.re, (T)x.im);
        }
    }
    wave_row_forward<T>(v, buf, tw, lane, dst.p[wr.f] + wr.y, ny, scale);
}

// Inverse row transforms of src.n H fields (the k_rows_inv contract:
// dst = acc dst + scale value; offs_f = new - old, or += with oacc).  Launch as
// k_rows_fwd_w.
template <typename T, typename Tout>
__global__ void __launch_bounds__(64 * WROW_WPB) k_rows_inv_w(int ny, PtrList<const cpx<T>, MAXF> src,
                                                              PtrList<Tout, MAXF> dst,
                                                              const cpx<T>* __restrict__ tw, T scale, T acc,
                                                              PtrList<Tout, MAXF> offs, int oacc) {
    __shared__ cpx<T> ldsw[WROW_WPB][WROW_BUF];
    const int lane = threadIdx.x & 63;
    const WaveRow wr = wave_row_of(ny);
    if (wr.f >= src.n) return;
    cpx<T>* buf = ldsw[threadIdx.x >> 6];
    cpx<T> v[8];
    wave_row_inverse<T>(v, buf, tw, lane, src.p[wr.f] + wr.y, ny);
    const size_t o = (size_t)wr.y * WROW_NX;
    cpx<Tout>* d = reinterpret_cast<cpx<Tout>*>(dst.p[wr.f] + o);
    cpx<Tout>* od = offs.n > 0 ? reinterpret_cast<cpx<Tout>*>(offs.p[wr.f] + o) : nullptr;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int n = lane + 64 * s;
        T v0 = scale * v[s].re, v1 = scale * v[s].im;
        cpx<Tout> old = C<Tout>(0, 0);
        if (acc != (T)0 || od) old = d[n];
        if (acc != (T)0) {
            v0 += acc * (T)old.re;
            v1 += acc * (T)old.im;
        }
        if (od) {
            const Tout d0 = (Tout)v0 - old.re, d1 = (Tout)v1 - old.im;
            if (oacc) {
                const cpx<Tout> p = od[n];
                od[n] = C<Tout>(p.re + d0, p.im + d1);
            } else {
                od[n] = C<Tout>(d0, d1);
            }
        }
        d[n] = C<Tout>((Tout)v0, (Tout)v1);
    }
}

// Inverse row transforms of the 2D right-hand side's eight derivative fields
// (m = div(eta u), delta = div u, grad delta, grad eta, grad beta) and the
// pointwise right-hand side (the k_rhs_rows_inv contract): one block per row,
// wave q inverse-transforms field q into LDS; after a barrier wave q forms, at
// the points of its slot q, eta_t = -m, U_t = -eta grad(eta - h) - T grad h and
// S of Def:bigF (S, T from P = u.grad(delta) - delta^2 and Q = u.grad(beta)),
// kept as S_x = S - eta u_x^2 and S_y = S - eta u_y^2 (see rhs_source); after a
// second barrier waves 0 and 1 forward-transform S_x into Sdst and S_y into
// Sydst.  Launch: ny blocks of 512 threads.
// An x-derivative field needs no column transform: with dx.f[q] != 0, wave q
// loads the row spectrum src.p[q] of the field it differentiates (a column
// pass output, f = 1, or a forward row transform, f = 1/nx, the column pass's
// scale of 1/(nx ny) times the ny of its y round trip) and multiplies entry kx
// by i k_x f before the inverse transform (the Nyquist entry has no wavenumber).
struct RowDx {
    double f[8];
};
__global__ void __launch_bounds__(512) k_rhs_rows_inv_w(int ny, PtrList<const cpx<double>, MAXF> src,
                                                        const double* __restrict__ eta,
                                                        const double* __restrict__ u,
                                                        const double* __restrict__ gh, double* __restrict__ eta_t,
                                                        double* __restrict__ U_t, cpx<double>* __restrict__ Sdst,
                                                        cpx<double>* __restrict__ Sydst,
                                                        const cpx<double>* __restrict__ tw, double scale, RowDx dx,
                                                        double tpx) {
    __shared__ cpx<double> ldsr[8][WROW_BUF];
    __shared__ WaveTwl<double> tl;
    const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int y = xcd_remap(blockIdx.x, gridDim.x);
    if (threadIdx.x < WAVE_TWL_ENTRIES) (&tl.a[0][0])[threadIdx.x] = wave_twl_entry<double>(tw, threadIdx.x);
    block_lds_barrier();
    cpx<double>* buf = ldsr[q];
    const cpx<double>* Hrow = src.p[q] + y;
    cpx<double> X[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) X[s] = Hrow[(size_t)(lane + 64 * s) * ny];
    cpx<double> XM = lane == 0 ? Hrow[(size_t)WROW_M * ny] : C<double>(0, 0);
    const double fq = dx.f[q];
    // inputs at this wave's pointwise slot (n = lane + 64 q), in flight during the transform
    const size_t npts = (size_t)WROW_NX * ny, o = (size_t)y * WROW_NX;
    const int n = lane + 64 * q;
    const cpx<double> pe = reinterpret_cast<const cpx<double>*>(eta + o)[n];
    const cpx<double> pu0 = reinterpret_cast<const cpx<double>*>(u + o)[n];
    const cpx<double> pu1 = reinterpret_cast<const cpx<double>*>(u + npts + o)[n];
    const cpx<double> ph0 = reinterpret_cast<const cpx<double>*>(gh + o)[n];
    const cpx<double> ph1 = reinterpret_cast<const cpx<double>*>(gh + npts + o)[n];
    if (fq != 0.0) {
#pragma unroll
        for (int s = 0; s < 8; ++s) X[s] = ik(wavenumber<double>(lane + 64 * s, WROW_NX, tpx) * fq, X[s]);
        XM = C<double>(0, 0);
    }
    cpx<double> v[8];
    wave_c2r_split<double>(v, X, XM, buf, tl.r[lane], lane);
    wave_fft512<double>(v, buf, wave_bases<double>(tl, lane), lane, true);
#pragma unroll
    for (int s = 0; s < 8; ++s) buf[lane + 64 * s] = v[s];
    block_lds_barrier();
    double Sx[2], Sy[2], et[2], ut0[2], ut1[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        double qv[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const cpx<double> z = ldsr[i][n];
            qv[i] = scale * (p ? z.im : z.re);
        }
        const double e0 = p ? pe.im : pe.re;
        const double uc[2] = {p ? pu0.im : pu0.re, p ? pu1.im : pu1.re};
        const double hc[2] = {p ? ph0.im : ph0.re, p ? ph1.im : ph1.re};
        double A0 = qv[0];                       // m
        et[p] = -qv[0];
        double A1 = qv[1];                       // delta
        double A2 = -qv[1] * qv[1];
        A2 += uc[0] * qv[2];                     // P = u.grad(delta) - delta^2
        A2 += uc[1] * qv[3];
        {
            double bt = 0.0;
            bt += hc[0] * uc[0];
            bt += hc[1] * uc[1];
            const double e2 = e0 * e0, mm = A0, d0 = A1, pp = A2;
            A0 = e2 * e0 / 3.0 * pp + e2 * mm * d0 + e0 * mm * bt;   // S
            A1 = e2 / 2.0 * pp + e0 * mm * d0 + mm * bt;             // T
        }
        const double U0 = -e0 * (qv[4] - hc[0]);
        const double U1 = -e0 * (qv[5] - hc[1]);
#pragma unroll
        for (int c = 0; c < 2; ++c) {            // Q = u.grad(beta)
            const double t = uc[c] * qv[6 + c];
            A0 += e0 * e0 / 2.0 * t;
            A1 += e0 * t;
        }
        ut0[p] = U0 - hc[0] * A1;
        ut1[p] = U1 - hc[1] * A1;
        Sx[p] = A0 - e0 * uc[0] * uc[0];
        Sy[p] = A0 - e0 * uc[1] * uc[1];
    }
    reinterpret_cast<cpx<double>*>(eta_t + o)[n] = C<double>(et[0], et[1]);
    reinterpret_cast<cpx<double>*>(U_t + o)[n] = C<double>(ut0[0], ut0[1]);
    reinterpret_cast<cpx<double>*>(U_t + npts + o)[n] = C<double>(ut1[0], ut1[1]);
    // slot n of fields 0 and 1 is read by this wave only, so S_x and S_y take
    // their places
    ldsr[0][n] = C<double>(Sx[0], Sx[1]);
    ldsr[1][n] = C<double>(Sy[0], Sy[1]);
    block_lds_barrier();
    if (q > 1) return;
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = buf[lane + 64 * s];
    wave_lds_sync();
    wave_fft512<double>(v, buf, wave_bases<double>(tl, lane), lane, false);
    wave_r2c_store<double>(v, buf, tl.r[lane], lane, (q == 0 ? Sdst : Sydst) + y, ny, 1.0);
}

}  // namespace sgn

namespace sgn {

// ---------------------------------------------------------------------------
// Column transforms of 1024 points (complex, along y) by two waves per column
// and field.  Forward (decimation in frequency): wave h forms
//   h = 0: x[n] + x[n+512],   h = 1: (x[n] - x[n+512]) W1024^n,   n < 512,
// and its 512-point transform gives X[2k + h]; both waves read the whole column
// (the second read is served by the caches), so the forward direction needs
// no exchange between waves.  Inverse (decimation in time): wave h transforms
// X[2k + h] to e_h[n], and x[n] = e_0[n] + W1024^{-n} e_1[n], x[n+512] =
// e_0[n] - W1024^{-n} e_1[n] after one exchange.  A block holds one column of
// three fields (six waves); each wave's LDS region is its exchange buffer and
// then holds its half of the spectrum compactly (X[2k + h] at entry k).
// ---------------------------------------------------------------------------
constexpr int WCOL_NY = 1024;
constexpr int WCOL_THREADS = 384;

// Wave h's forward transform of the column whose entries lo[s] = x[lane + 64 s]
// and hi[s] = x[lane + 64 s + 512] it holds; v[s] = X[2 (lane + 64 s) + h].
template <typename T>
__device__ __forceinline__ void wave_col_forward(cpx<T> (&v)[8], const cpx<T> (&lo)[8], const cpx<T> (&hi)[8],
                                                 int h, cpx<T>* buf, const WaveTwl<T>& tl, int lane) {
    const cpx<T> r1 = tl.r[lane];
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = h == 0 ? lo[s] + hi[s] : (lo[s] - hi[s]) * (r1 * w16<T>(s));
    wave_fft512<T>(v, buf, wave_bases<T>(tl, lane), lane, false);
}

// Krylov update pass (MODE C2_UPDATE of k_pcg_c2) on columns of 1024 points:
// reduce p.Gp -> alpha; y-FFT of the row pass's (a_x, a_y, w); q = a - i k w;
// x += alpha p; r -= alpha q; z = A^{-1} r; partial r.z, r.r per column.  Launch:
// nx/2 + 1 blocks of 384 threads.
template <typename T>
__global__ void __launch_bounds__(WCOL_THREADS) k_pcg_c2w(int nx, const cpx<T>* __restrict__ tw,
                                                          SolveScal* __restrict__ sc, const cpx<T>* __restrict__ H,
                                                          size_t NS, const cpx<T>* __restrict__ ph,
                                                          cpx<T>* __restrict__ xh, cpx<T>* __restrict__ rh,
                                                          double* __restrict__ part, int nb_r1, T tpx, T tpy) {
    if (sc->done) return;
    __shared__ cpx<T> ldsb[6][WROW_BUF];
    __shared__ WaveTwl<T> tl;
    __shared__ double red[32];
    __shared__ double slot[1];
    constexpr int NY = WCOL_NY;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int f = wv >> 1, h = wv & 1;
    const int kx = blockIdx.x;
    if (threadIdx.x < WAVE_TWL_ENTRIES) (&tl.a[0][0])[threadIdx.x] = wave_twl_entry<T>(tw, threadIdx.x);
    // the partials of the reduction, then the columns (in flight across it)
    double pb[PF_K][1];
    partials_fetch<1>(part + PART_C2, nb_r1, pb);
    __builtin_amdgcn_sched_barrier(0);
    const cpx<T>* col = H + (size_t)f * NS + (size_t)kx * NY;
    cpx<T> lo[8], hi[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        lo[s] = col[lane + 64 * s];
        hi[s] = col[lane + 64 * s + 512];
    }
    __builtin_amdgcn_sched_barrier(0);
    double tot[1];
    partials_sum<1, true>(part + PART_C2, nb_r1, pb, tot, red);
    const double pq = bcast<true>(tot[0], slot);
    const double a = sc->rho / pq;
    const T alpha = (T)a;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->pq = pq;
        sc->alpha = a;
        sc->rho_prev = sc->rho;
        sc->iter = sc->iter + 1;
        sc->first = 0;
    }
    cpx<T>* buf = ldsb[wv];
    cpx<T> v[8];
    wave_col_forward<T>(v, lo, hi, h, buf, tl, lane);
#pragma unroll
    for (int s = 0; s < 8; ++s) buf[lane + 64 * s] = v[s];
    block_lds_barrier();
    const T kxw = wavenumber<T>(kx, nx, tpx);
    const T sig = (T)sc->sig, alp = (T)sc->alp;
    const double w = half_weight(kx, nx);
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int j = threadIdx.x + WCOL_THREADS * i;
        if (j < NY) {
            const size_t idx = (size_t)kx * NY + j;
            const T ky = wavenumber<T>(j, NY, tpy);
            const cpx<T> wq = ldsb[4 + (j & 1)][j >> 1];
            cpx<T> r[2], z[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const T kc = (c == 0) ? kxw : ky;
                const cpx<T> q = ldsb[2 * c + (j & 1)][j >> 1] - ik(kc, wq);
                xh[c * NS + idx] = xh[c * NS + idx] + alpha * ph[c * NS + idx];
                r[c] = rh[c * NS + idx] - alpha * q;
                rh[c * NS + idx] = r[c];
            }
            precond_mode<T, 2>(kxw, ky, sig, alp, r, z);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                acc[0] += w * ((double)r[c].re * (double)z[c].re + (double)r[c].im * (double)z[c].im);
                acc[1] += w * ((double)r[c].re * (double)r[c].re + (double)r[c].im * (double)r[c].im);
            }
        }
    }
    block_sum<2>(acc, red);
    if (threadIdx.x == 0) {
        part[PART_C3 + 2 * blockIdx.x] = acc[0];
        part[PART_C3 + 2 * blockIdx.x + 1] = acc[1];
    }
}

// Krylov direction pass (MODE C1_UPDATE of k_pcg_c1) on columns of 1024 points:
// reduce r.z, r.r -> stop test, beta; z = A^{-1} r; p = z + beta p; emit
// (p, div p)/N and y-IFFT it into H.  Launch: nx/2 + 1 blocks of 384 threads.
template <typename T>
__global__ void __launch_bounds__(WCOL_THREADS) k_pcg_c1w(int nx, const cpx<T>* __restrict__ tw,
                                                          SolveScal* __restrict__ sc, const double* __restrict__ part,
                                                          int nb3, const cpx<T>* __restrict__ rh,
                                                          cpx<T>* __restrict__ ph, cpx<T>* __restrict__ H, size_t NS,
                                                          T tpx, T tpy) {
    if (sc->done) return;
    __shared__ cpx<T> ldsb[6][WROW_BUF];
    __shared__ WaveTwl<T> tl;
    __shared__ double red[32];
    __shared__ double slot[2];
    constexpr int NY = WCOL_NY;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int f = wv >> 1, h = wv & 1;
    const int kx = blockIdx.x;
    if (threadIdx.x < WAVE_TWL_ENTRIES) (&tl.a[0][0])[threadIdx.x] = wave_twl_entry<T>(tw, threadIdx.x);
    double beta_d = 0.0;
    if (pcg_iterate_state(sc, part, nb3, red, slot, beta_d)) return;
    const T beta = (T)beta_d, sig = (T)sc->sig, alp = (T)sc->alp, inv_n = (T)sc->inv_n;
    const T kxw = wavenumber<T>(kx, nx, tpx);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int j = threadIdx.x + WCOL_THREADS * i;
        if (j < NY) {
            const size_t idx = (size_t)kx * NY + j;
            const T ky = wavenumber<T>(j, NY, tpy);
            cpx<T> r[2], z[2], p[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) r[c] = rh[c * NS + idx];
            precond_mode<T, 2>(kxw, ky, sig, alp, r, z);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                // beta = 0 on the first iteration: p = z without reading the
                // previous (unset) direction
                p[c] = (beta != (T)0) ? z[c] + beta * ph[c * NS + idx] : z[c];
                ph[c * NS + idx] = p[c];
            }
            const cpx<T> dv = ik(kxw, p[0]) + ik(ky, p[1]);
            ldsb[0 + (j & 1)][j >> 1] = inv_n * p[0];
            ldsb[2 + (j & 1)][j >> 1] = inv_n * p[1];
            ldsb[4 + (j & 1)][j >> 1] = inv_n * dv;
        }
    }
    block_lds_barrier();
    cpx<T>* buf = ldsb[wv];
    cpx<T> v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = buf[lane + 64 * s];
    wave_lds_sync();
    wave_fft512<T>(v, buf, wave_bases<T>(tl, lane), lane, true);
    // e_0 (h = 0) or W1024^{-n} e_1 (h = 1) at entry n = lane + 64 s
    if (h == 1) {
        const cpx<T> r1 = tl.r[lane];
#pragma unroll
        for (int s = 0; s < 8; ++s) v[s] = v[s] * cj(r1 * w16<T>(s));
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) buf[lane + 64 * s] = v[s];
    block_lds_barrier();
    const cpx<T>* other = ldsb[wv ^ 1];
    cpx<T>* out = H + (size_t)f * NS + (size_t)kx * NY + (h ? 512 : 0);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int n = lane + 64 * s;
        const cpx<T> o = other[n];
        out[n] = h == 0 ? v[s] + o : o - v[s];
    }
}

}  // namespace sgn
