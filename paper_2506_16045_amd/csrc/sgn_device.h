// Device building blocks of the spectral engine (gfx950, wave64).
//
// Spectral discretisation of section 6.1: every derivative is D = F^{-1}(iK)F
// with the Nyquist wavenumber of each axis set to zero.  A 2D real field
// f[ny][nx] (x fast) goes through two kinds of passes:
//   row pass    : real-to-complex FFT along x of each row, written transposed to
//                 the "H" layout H[kx][y] (kx = 0..nx/2, y contiguous), and the
//                 inverse complex-to-real pass back;
//   column pass : complex FFT along y of each kx column of H (contiguous), giving
//                 the "S" layout S[kx][ky] used for the Krylov state.
// A 1D field is the ny = 1 case: the column pass is then a plain per-mode loop.
// All transforms are unnormalised; callers apply 1/(nx*ny) once per round trip.
//
// FFTs run in LDS as radix-4 Stockham passes (autosort, decimation in time)
// with a final radix-2 pass when log2 M is odd; the fields a pass needs are
// transformed in lockstep so they share the block barriers.  A real row of
// length nx is transformed as a complex sequence of length M = nx/2
// (z_j = x_2j + i x_2j+1) followed by the usual even/odd split.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sgn {

constexpr int TW_LOG = 14;
constexpr int TW_SIZE = 1 << TW_LOG;          // largest transform length
constexpr int TW_ALL = 2 * TW_SIZE - 1;       // entries of the per-size twiddle table

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T re, im;
};

template <typename T> __device__ __forceinline__ cpx<T> C(T a, T b) { return cpx<T>{a, b}; }
template <typename T> __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return C(a.re + b.re, a.im + b.im); }
template <typename T> __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return C(a.re - b.re, a.im - b.im); }
template <typename T> __device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
    return C(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T> __device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return C(s * a.re, s * a.im); }
template <typename T> __device__ __forceinline__ cpx<T> cj(cpx<T> a) { return C(a.re, -a.im); }
template <typename T> __device__ __forceinline__ cpx<T> mul_i(cpx<T> a) { return C(-a.im, a.re); }   // i a
template <typename T> __device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) { return C(a.im, -a.re); }  // -i a
// i k a for a real wavenumber k
template <typename T> __device__ __forceinline__ cpx<T> ik(T k, cpx<T> a) { return C(-k * a.im, k * a.re); }

__device__ __forceinline__ int ilog2(int x) { return 31 - __clz(x); }

// Signed wavenumber of FFT index j on an axis of n points and length L, with
// the Nyquist index n/2 mapped to zero (section 6.1).
template <typename T>
__device__ __forceinline__ T wavenumber(int j, int n, T two_pi_over_L) {
    int m = (j < n / 2) ? j : j - n;
    if (2 * j == n) m = 0;
    return two_pi_over_L * (T)m;
}

// ---------------------------------------------------------------------------
// Twiddles.  The global table holds, for every power of two L <= TW_SIZE, the
// L-th roots of unity W_L^j = exp(-2 pi i j / L) contiguously at offset L - 1
// (2 TW_SIZE - 1 entries).  An FFT of length M reads W_M^m; kernels copy the M
// entries into LDS once per block when they fit (see twl_setup).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ const cpx<T>* tw_size(const cpx<T>* __restrict__ tw_all, int L) {
    return tw_all + (L - 1);
}

constexpr int TWL_MAX = 0;     // largest FFT length whose twiddles are staged in LDS (0: read from the global table)

// Stage W_M^m (m < M) in LDS when M <= TWL_MAX; returns the table to use (LDS or
// global).  Contains a block barrier; every thread must call it.
template <typename T>
__device__ __forceinline__ const cpx<T>* twl_setup(const cpx<T>* __restrict__ tw_all, int M, cpx<T>* lds_tw) {
    const cpx<T>* g = tw_size(tw_all, M);
    if (M > TWL_MAX || M < 4) return g;
    for (int j = threadIdx.x; j < M; j += blockDim.x) lds_tw[j] = g[j];
    __syncthreads();
    return lds_tw;
}

// ---------------------------------------------------------------------------
// Stockham FFT of length M (power of two) on NF buffers at buf + f * fstride,
// transformed in lockstep by TPX cooperating threads (thread index t): radix-8
// (few fields) or radix-4 (many fields) passes while they fit, then one
// radix-4 or radix-2 pass for the remaining factor (mixed-radix Stockham: a pass of radix R over span Ns reads
// x[j + r M/R], twiddles by W_{R Ns}^{k r} with k = j mod Ns, and writes the
// R-point DFT to y[(j - k) R + k + q Ns]).  Every thread of the block must call
// it (it contains block barriers); M <= EPC * TPX.  twm[m] = W_M^m.
// Forward: exp(-i ...); inverse: exp(+i ...); unnormalised.
// ---------------------------------------------------------------------------

// In-register R-point DFTs (R = 2, 4, 8) of v[0..R).
template <typename T, int R>
__device__ __forceinline__ void dft_small(cpx<T> (&v)[R], bool inverse) {
    if (R == 2) {
        const cpx<T> a = v[0], b = v[1 % R];
        v[0] = a + b;
        v[1 % R] = a - b;
    } else if (R == 4) {
        const cpx<T> a0 = v[0] + v[2 % R], a1 = v[0] - v[2 % R];
        const cpx<T> a2 = v[1 % R] + v[3 % R], d = v[1 % R] - v[3 % R];
        const cpx<T> a3 = inverse ? mul_i(d) : mul_mi(d);
        v[0] = a0 + a2;
        v[1 % R] = a1 + a3;
        v[2 % R] = a0 - a2;
        v[3 % R] = a1 - a3;
    } else {
        // two 4-point DFTs (even and odd inputs), then W_8^q on the odd half
        cpx<T> e[4], o[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            e[q] = v[(2 * q) % R];
            o[q] = v[(2 * q + 1) % R];
        }
        dft_small<T, 4>(e, inverse);
        dft_small<T, 4>(o, inverse);
        const T h = (T)0.70710678118654752440;
        const T sg = inverse ? (T)1 : (T)-1;
        const cpx<T> w1 = C<T>(h, sg * h), w3 = C<T>(-h, sg * h);
        const cpx<T> t0 = o[0];
        const cpx<T> t1 = w1 * o[1];
        const cpx<T> t2 = inverse ? mul_i(o[2]) : mul_mi(o[2]);
        const cpx<T> t3 = w3 * o[3];
        v[0] = e[0] + t0;
        v[4 % R] = e[0] - t0;
        v[1 % R] = e[1] + t1;
        v[5 % R] = e[1] - t1;
        v[2 % R] = e[2] + t2;
        v[6 % R] = e[2] - t2;
        v[3 % R] = e[3] + t3;
        v[7 % R] = e[3] - t3;
    }
}

// LDS index swizzle of the intermediate Stockham layouts: bits 0-2 of an index
// are XORed with a function of bits 3-5, which permutes every aligned group of 8
// entries.  The first passes write at strides R and R^2 entries; swizzled, eight
// consecutive threads then write eight different 16-byte bank groups (radix 4
// and radix 8).
__device__ __forceinline__ int lds_swz(int i) {
    return i ^ (((i >> 3) & 7) ^ (((i >> 4) & 1) << 2));
}

template <typename T, int R, int NB, int NF>
__device__ __forceinline__ void fft_pass(cpx<T>* buf, int fstride, int M, int t, int TPX,
                                         const cpx<T>* __restrict__ twm, bool inverse, int Ns, int sh,
                                         bool swz_in = false, bool swz_out = false) {
    const int MR = M / R;
    cpx<T> v[NB][NF][R];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = t + i * TPX;
        if (j < MR) {
            const int k = j & (Ns - 1);
            cpx<T> w[R];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                w[r] = twm[(k * r) << sh];   // W_{R Ns}^{k r} = W_M^{k r M / (R Ns)}
                if (inverse) w[r].im = -w[r].im;
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const cpx<T>* bf = buf + f * fstride;
                v[i][f][0] = bf[swz_in ? lds_swz(j) : j];
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const int a = j + r * MR;
                    v[i][f][r] = bf[swz_in ? lds_swz(a) : a] * w[r];
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = t + i * TPX;
        if (j < MR) {
            const int k = j & (Ns - 1);
            const int o = (j - k) * R + k;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                dft_small<T, R>(v[i][f], inverse);
                cpx<T>* bf = buf + f * fstride;
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const int a = o + q * Ns;
                    bf[swz_out ? lds_swz(a) : a] = v[i][f][q];
                }
            }
        }
    }
    __syncthreads();
}

// SWZ: the passes between the first and the last keep their data in the
// swizzled layout (lds_swz); input and output are in the natural layout.
template <typename T, int EPC, int NF, bool SWZ = false>
__device__ __forceinline__ void lds_fft(cpx<T>* buf, int fstride, int M, int t, int TPX,
                                        const cpx<T>* __restrict__ twm, bool inverse) {
    constexpr int NB8 = EPC / 8 > 0 ? EPC / 8 : 1;
    constexpr int NB4 = EPC / 4 > 0 ? EPC / 4 : 1;
    constexpr int NB2 = EPC / 2 > 0 ? EPC / 2 : 1;
    // radix-8 passes hold 8 NF values per butterfly in registers: used while that
    // stays within 16 FP64 complex words (more fields in lockstep use radix 4)
    constexpr bool R8 = NF * (int)sizeof(T) <= 16;
    const int logM = ilog2(M);
    int Ns = 1;
    int logNs = 0;
    bool sw = false;   // the layout the next pass reads
    auto last = [&](int R) { return Ns * R == M; };
    if (R8) {
        for (; Ns * 8 <= M; Ns <<= 3, logNs += 3) {
            const bool so = SWZ && !last(8);
            fft_pass<T, 8, NB8, NF>(buf, fstride, M, t, TPX, twm, inverse, Ns, logM - (logNs + 3), sw, so);
            sw = so;
        }
    } else {
        for (; Ns * 16 <= M; Ns <<= 2, logNs += 2) {
            const bool so = SWZ && !last(4);
            fft_pass<T, 4, NB4, NF>(buf, fstride, M, t, TPX, twm, inverse, Ns, logM - (logNs + 2), sw, so);
            sw = so;
        }
    }
    if (Ns * 4 <= M) {
        const bool so = SWZ && !last(4);
        fft_pass<T, 4, NB4, NF>(buf, fstride, M, t, TPX, twm, inverse, Ns, logM - (logNs + 2), sw, so);
        sw = so;
        Ns <<= 2;
        logNs += 2;
    }
    if (Ns * 2 <= M) fft_pass<T, 2, NB2, NF>(buf, fstride, M, t, TPX, twm, inverse, Ns, logM - (logNs + 1), sw, false);
}

// Column transforms take the swizzled intermediate layouts in FP64 (16-byte
// entries, where the first passes' strided writes conflict).
template <typename T>
constexpr bool col_swz() { return sizeof(T) == 8; }

// ---------------------------------------------------------------------------
// Row geometry: a block holds R rows of TPR threads each; row r of the block is
// grid row row0 + r.  Thread t of a row owns complex positions j = t + TPR*e
// (e < EPC), i.e. real positions 2j and 2j+1.  LDS: NF fields x R rows of M+1
// complex entries (field stride R (M+1)), then the twiddle table.
// ---------------------------------------------------------------------------
struct RowGeom {
    int nx, ny, M, TPR, R, nblocks;
};

template <typename T>
struct RowThread {
    int r, t, y, row0;
    bool valid;
    cpx<T>* lds;  // block LDS base
    int fstride;  // R (M+1)
};

// Map a launch block index to a row group so that consecutive row groups land on
// the same XCD (blocks are dealt round-robin over 8 XCDs, each with its own L2):
// neighbouring row groups share the cache lines of the transposed H layout.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

// Row thread of row block `blk` (blockIdx.x, or the block within one part of a
// launch that runs several independent row jobs side by side).
template <typename T>
__device__ __forceinline__ RowThread<T> row_thread_at(const RowGeom& g, cpx<T>* lds, int blk) {
    RowThread<T> rt;
    rt.r = threadIdx.x / g.TPR;
    rt.t = threadIdx.x - rt.r * g.TPR;
    rt.row0 = xcd_remap(blk, g.nblocks) * g.R;
    rt.y = rt.row0 + rt.r;
    rt.valid = rt.y < g.ny;
    rt.lds = lds;
    rt.fstride = g.R * (g.M + 1);
    return rt;
}
template <typename T>
__device__ __forceinline__ RowThread<T> row_thread(const RowGeom& g, cpx<T>* lds) {
    return row_thread_at<T>(g, lds, blockIdx.x);
}

// LDS entries a row kernel with NF fields needs before its twiddle table.
__host__ __device__ inline int row_lds_data(const RowGeom& g, int NF) { return NF * g.R * (g.M + 1); }

// Inverse row transforms of NF fields: H_f[kx][y] (kx = 0..M) -> real pairs
// z[f][e] = (x_2j, x_2j+1), unnormalised (nx times the inverse DFT).  The
// imaginary parts of the kx = 0 and kx = nx/2 entries are ignored (real signal).
// The even/odd recombination Z_k = (X_k + X*_{M-k}) + i (X_k - X*_{M-k}) W_nx^{-k}
// is formed while the mirrored pair (k, M - k) is loaded from H, so it costs no
// LDS pass of its own.
template <typename T, int EPC, int NF>
__device__ __forceinline__ void row_inverse(const RowGeom& g, const RowThread<T>& rt,
                                            const cpx<T>* const (&H)[NF],
                                            const cpx<T>* __restrict__ tw_all, const cpx<T>* twm,
                                            cpx<T> (&z)[NF][EPC]) {
    const int M = g.M, R = g.R, ny = g.ny;
    const int totalp = R * (M / 2 + 1);
    const cpx<T>* tw2 = tw_size(tw_all, 2 * M);  // W_nx^k
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        for (int i = threadIdx.x; i < totalp; i += blockDim.x) {
            const int r = i & (R - 1);
            const int p = i / R;
            const int y = rt.row0 + r;
            const int k = p, m = M - p;
            const cpx<T> Xk = (y < ny) ? H[f][(size_t)k * ny + y] : C<T>(0, 0);
            const cpx<T> Xm = (y < ny) ? H[f][(size_t)m * ny + y] : C<T>(0, 0);
            cpx<T>* b = rt.lds + f * rt.fstride + r * (M + 1);
            if (p == 0) {
                b[0] = C<T>(Xk.re + Xm.re, Xk.re - Xm.re);
            } else {
                cpx<T> wk = tw2[k], wm = tw2[m];
                wk.im = -wk.im;
                wm.im = -wm.im;
                const cpx<T> Zk = (Xk + cj(Xm)) + mul_i((Xk - cj(Xm)) * wk);
                if (m != k) b[m] = (Xm + cj(Xk)) + mul_i((Xm - cj(Xk)) * wm);
                b[k] = Zk;
            }
        }
    }
    __syncthreads();
    cpx<T>* rowb = rt.lds + rt.r * (M + 1);
    lds_fft<T, EPC, NF>(rowb, rt.fstride, M, rt.t, g.TPR, twm, true);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = rt.t + g.TPR * e;
            if (j < M) z[f][e] = rowb[f * rt.fstride + j];
        }
    }
    __syncthreads();
}

// row_inverse with every transposed load of the block issued before the first
// LDS store: each thread keeps its mirrored pairs (k, M - k) of all NF fields in
// registers (EPC/2 + 1 pairs per field), so the loads of all fields are in
// flight together.  For the short rows of the Krylov row pass, whose launch
// leaves few waves per CU to hide the latency of the transposed accesses.
template <typename T, int EPC, int NF>
__device__ __forceinline__ void row_inverse_batched(const RowGeom& g, const RowThread<T>& rt,
                                                    const cpx<T>* const (&H)[NF],
                                                    const cpx<T>* __restrict__ tw_all, const cpx<T>* twm,
                                                    cpx<T> (&z)[NF][EPC]) {
    const int M = g.M, R = g.R, ny = g.ny;
    // R (M/2 + 1) pairs over R M / EPC threads: EPC/2 pairs each, R more for the first threads
    constexpr int Q = EPC / 2 + 1;
    const int totalp = R * (M / 2 + 1);
    const cpx<T>* tw2 = tw_size(tw_all, 2 * M);
    cpx<T> Xk[Q][NF], Xm[Q][NF];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = threadIdx.x + q * blockDim.x;
        const int y = rt.row0 + (i & (R - 1));
        const int p = i / R;
        const bool ok = i < totalp && y < ny;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            Xk[q][f] = ok ? H[f][(size_t)p * ny + y] : C<T>(0, 0);
            Xm[q][f] = ok ? H[f][(size_t)(M - p) * ny + y] : C<T>(0, 0);
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = threadIdx.x + q * blockDim.x;
        if (i >= totalp) continue;
        const int r = i & (R - 1);
        const int k = i / R, m = M - k;
        cpx<T> wk = tw2[k], wm = tw2[m];
        wk.im = -wk.im;
        wm.im = -wm.im;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            cpx<T>* b = rt.lds + f * rt.fstride + r * (M + 1);
            const cpx<T> xk = Xk[q][f], xm = Xm[q][f];
            if (k == 0) {
                b[0] = C<T>(xk.re + xm.re, xk.re - xm.re);
            } else {
                const cpx<T> Zk = (xk + cj(xm)) + mul_i((xk - cj(xm)) * wk);
                if (m != k) b[m] = (xm + cj(xk)) + mul_i((xm - cj(xk)) * wm);
                b[k] = Zk;
            }
        }
    }
    __syncthreads();
    cpx<T>* rowb = rt.lds + rt.r * (M + 1);
    lds_fft<T, EPC, NF>(rowb, rt.fstride, M, rt.t, g.TPR, twm, true);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = rt.t + g.TPR * e;
            if (j < M) z[f][e] = rowb[f * rt.fstride + j];
        }
    }
    __syncthreads();
}

// Forward row transforms of NF fields: real pairs z[f][e] -> H_f[kx][y] for
// kx = 0..M, each value multiplied by `scale`.  The recombination
// X_k = (Z_k + Z*_{M-k})/2 - i W_nx^k (Z_k - Z*_{M-k})/2 is formed as each entry
// is stored (no LDS pass of its own).
template <typename T, int EPC, int NF>
__device__ __forceinline__ void row_forward(const RowGeom& g, const RowThread<T>& rt, const cpx<T> (&z)[NF][EPC],
                                            cpx<T>* const (&H)[NF], const cpx<T>* __restrict__ tw_all,
                                            const cpx<T>* twm, T scale) {
    const int M = g.M, R = g.R, ny = g.ny;
    cpx<T>* rowb = rt.lds + rt.r * (M + 1);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = rt.t + g.TPR * e;
            if (j < M) rowb[f * rt.fstride + j] = z[f][e];
        }
    }
    __syncthreads();
    lds_fft<T, EPC, NF>(rowb, rt.fstride, M, rt.t, g.TPR, twm, false);
    const cpx<T>* tw2 = tw_size(tw_all, 2 * M);
    const T half = (T)0.5;
    const int total = R * (M + 1);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        for (int i = threadIdx.x; i < total; i += blockDim.x) {
            const int r = i & (R - 1);
            const int kx = i / R;
            const int y = rt.row0 + r;
            const cpx<T>* b = rt.lds + f * rt.fstride + r * (M + 1);
            cpx<T> X;
            if (kx == 0 || kx == M) {
                const cpx<T> Z0 = b[0];
                X = C<T>(kx == 0 ? Z0.re + Z0.im : Z0.re - Z0.im, 0);
            } else {
                const cpx<T> wk = tw2[kx];
                const cpx<T> Zk = b[kx], Zm = b[M - kx];
                X = half * (Zk + cj(Zm)) - half * mul_i(wk * (Zk - cj(Zm)));
            }
            if (y < ny) H[f][(size_t)kx * ny + y] = scale * X;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Column geometry: a block holds Cb columns (kx) of TPC threads each; column c
// is kx = blockIdx.x * Cb + c.  Thread t owns modes j = t + TPC*e (e < EPC,
// j < ny).  LDS: NF fields x Cb columns of ny entries (field stride Cb ny), then
// the twiddle table.
// ---------------------------------------------------------------------------
struct ColGeom {
    int nx, ny, nxh, TPC, Cb, nblocks;
};

template <typename T>
struct ColThread {
    int c, t, kx;
    bool valid;
    cpx<T>* buf;  // field 0 of this column
    int fstride;  // Cb ny
};

__host__ __device__ inline int col_lds_data(const ColGeom& g, int NF) { return NF * g.Cb * g.ny; }

// Column thread of column block `blk` (blockIdx.x, or the block within one part
// of a launch that runs several column jobs side by side).
template <typename T>
__device__ __forceinline__ ColThread<T> col_thread_at(const ColGeom& g, cpx<T>* lds, int blk) {
    ColThread<T> ct;
    ct.c = threadIdx.x / g.TPC;
    ct.t = threadIdx.x - ct.c * g.TPC;
    ct.kx = blk * g.Cb + ct.c;
    ct.valid = ct.kx < g.nxh;
    ct.buf = lds + ct.c * g.ny;
    ct.fstride = g.Cb * g.ny;
    return ct;
}
template <typename T>
__device__ __forceinline__ ColThread<T> col_thread(const ColGeom& g, cpx<T>* lds) {
    return col_thread_at<T>(g, lds, blockIdx.x);
}

// Load NF columns of H (or S) into registers (col_fetch), then optionally
// transform them along y (col_fft); col_load does both.
// Entry (column kx, row j) of a column-layout field, clamped in range (entry 0
// of the field where the lane has no entry), and whether it is a real entry.
// The loads through it are unconditional: predicated loads make the compiler
// wait for every load in flight (see partials_fetch).
template <typename T>
__device__ __forceinline__ size_t col_index(const ColGeom& g, const ColThread<T>& ct, int j, bool& ok) {
    ok = ct.valid && j < g.ny;
    return ok ? (size_t)ct.kx * g.ny + j : 0;
}
// A lane without an entry (a column past nx/2 in the last block) holds a copy
// of entry 0: finite, transformed with its column and never stored or summed
// (the callers guard outputs and weights by ct.valid).
template <typename T, int EPC, int NF>
__device__ __forceinline__ void col_fetch(const ColGeom& g, const ColThread<T>& ct, const cpx<T>* const (&H)[NF],
                                          cpx<T> (&v)[NF][EPC]) {
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
        bool ok;
        const size_t idx = col_index(g, ct, ct.t + g.TPC * e, ok);
#pragma unroll
        for (int f = 0; f < NF; ++f) v[f][e] = H[f][idx];
    }
}
template <typename T, int EPC, int NF>
__device__ __forceinline__ void col_fft(const ColGeom& g, const ColThread<T>& ct, const cpx<T>* twm,
                                        cpx<T> (&v)[NF][EPC]) {
    const int ny = g.ny;
    if (ny > 1) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                const int j = ct.t + g.TPC * e;
                if (j < ny) ct.buf[f * ct.fstride + j] = v[f][e];
            }
        }
        __syncthreads();
        lds_fft<T, EPC, NF, col_swz<T>()>(ct.buf, ct.fstride, ny, ct.t, g.TPC, twm, false);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                const int j = ct.t + g.TPC * e;
                if (j < ny) v[f][e] = ct.buf[f * ct.fstride + j];
            }
        }
        __syncthreads();
    }
}
// col_load: lanes without an entry hold zeros.
template <typename T, int EPC, int NF>
__device__ __forceinline__ void col_load(const ColGeom& g, const ColThread<T>& ct, const cpx<T>* const (&H)[NF],
                                         bool fft, const cpx<T>* twm, cpx<T> (&v)[NF][EPC]) {
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
        const int j = ct.t + g.TPC * e;
#pragma unroll
        for (int f = 0; f < NF; ++f)
            if (j < g.ny) v[f][e] = ct.valid ? H[f][(size_t)ct.kx * g.ny + j] : C<T>(0, 0);
    }
    if (fft) col_fft<T, EPC, NF>(g, ct, twm, v);
}

// Optionally inverse-transform NF columns along y, then store them to H (or S).
template <typename T, int EPC, int NF>
__device__ __forceinline__ void col_store(const ColGeom& g, const ColThread<T>& ct, cpx<T> (&v)[NF][EPC],
                                          cpx<T>* const (&H)[NF], bool ifft, const cpx<T>* twm) {
    const int ny = g.ny;
    if (ifft && ny > 1) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                const int j = ct.t + g.TPC * e;
                if (j < ny) ct.buf[f * ct.fstride + j] = v[f][e];
            }
        }
        __syncthreads();
        lds_fft<T, EPC, NF, col_swz<T>()>(ct.buf, ct.fstride, ny, ct.t, g.TPC, twm, true);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                const int j = ct.t + g.TPC * e;
                if (j < ny) v[f][e] = ct.buf[f * ct.fstride + j];
            }
        }
        __syncthreads();
    }
    if (ct.valid) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                const int j = ct.t + g.TPC * e;
                if (j < ny) H[f][(size_t)ct.kx * ny + j] = v[f][e];
            }
        }
    }
}

// Block barrier that orders LDS only.  __syncthreads() fences all memory, which
// makes every wave wait for its global loads in flight (vmcnt(0)) at the
// barrier; kernels that issue their data loads before a reduction or an LDS
// exchange keep them in flight across such barriers.
__device__ __forceinline__ void block_lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Deterministic reductions.  Each block reduces NACC doubles in a fixed tree
// (wave shuffles, then waves in order) and writes them to partials[block];
// the last block to finish sums the partials in block order, so the result
// does not depend on scheduling.
// ---------------------------------------------------------------------------
// LDS_ONLY: the barriers order LDS only (global loads in flight stay in flight);
// the arithmetic, and so the result, is the same.
template <int NACC, bool LDS_ONLY = false>
__device__ __forceinline__ void block_sum(double (&v)[NACC], double* red /*LDS, NACC*16*/) {
#pragma unroll
    for (int a = 0; a < NACC; ++a) {
        double x = v[a];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        v[a] = x;
    }
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int nw = (blockDim.x + 63) >> 6;
    if (lane == 0) {
#pragma unroll
        for (int a = 0; a < NACC; ++a) red[a * 16 + wave] = v[a];
    }
    if (LDS_ONLY)
        block_lds_barrier();
    else
        __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int a = 0; a < NACC; ++a) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += red[a * 16 + w];
            v[a] = s;
        }
    }
    if (LDS_ONLY)
        block_lds_barrier();
    else
        __syncthreads();
}

// Sum of the per-block partials (layout partials[NACC*b + a]) by the whole
// last block: thread t < 256 adds blocks t, t+256, ... in order, then the fixed
// block tree (further threads and waves add zeros); the result is in thread 0.
// The order, and so the value, is the same in every kernel that reduces the same
// partials, whatever its block size (at least 256 threads).  Every thread of the
// block must call it.
template <int NACC, bool LDS_ONLY = false>
__device__ __forceinline__ void final_sum(const double* __restrict__ partials, unsigned nblocks,
                                          double (&v)[NACC], double* red) {
#pragma unroll
    for (int a = 0; a < NACC; ++a) v[a] = 0.0;
    for (unsigned b = threadIdx.x; threadIdx.x < 256 && b < nblocks; b += 256) {
#pragma unroll
        for (int a = 0; a < NACC; ++a) v[a] += partials[(size_t)NACC * b + a];
    }
    block_sum<NACC, LDS_ONLY>(v, red);
}

// final_sum in two steps, so that a kernel can issue the partials' loads ahead
// of its data loads (a wait for a load also waits for every load issued before
// it): partials_fetch loads the partials of up to 256 PF_K blocks (every
// reducing launch: PARTIALS_MAX) into registers, partials_sum adds them in
// final_sum's order, so the result is the same bits.  No loop: a load inside a
// loop makes the compiler wait for every load in flight at the loop entry.
constexpr int PF_K = 16;
template <int NACC>
__device__ __forceinline__ void partials_fetch(const double* __restrict__ partials, unsigned nblocks,
                                               double (&pb)[PF_K][NACC]) {
    // branch-free: every lane loads an in-range entry (predicated loads would
    // make the compiler wait for all loads); partials_sum drops the extra ones
#pragma unroll
    for (int k = 0; k < PF_K; ++k) {
        const unsigned b = threadIdx.x + 256u * k;
        const unsigned bc = (threadIdx.x < 256 && b < nblocks) ? b : 0u;
#pragma unroll
        for (int a = 0; a < NACC; ++a) pb[k][a] = partials[(size_t)NACC * bc + a];
    }
}
template <int NACC, bool LDS_ONLY = false>
__device__ __forceinline__ void partials_sum(const double* __restrict__ partials, unsigned nblocks,
                                             const double (&pb)[PF_K][NACC], double (&v)[NACC], double* red) {
#pragma unroll
    for (int a = 0; a < NACC; ++a) v[a] = 0.0;
#pragma unroll
    for (int k = 0; k < PF_K; ++k) {
        const bool ok = threadIdx.x < 256 && threadIdx.x + 256u * k < nblocks;
#pragma unroll
        for (int a = 0; a < NACC; ++a) v[a] += ok ? pb[k][a] : 0.0;
    }
    block_sum<NACC, LDS_ONLY>(v, red);
}

// Maximum of the per-block partials by the whole last block (order independent);
// the result is in thread 0.
template <int NACC>
__device__ __forceinline__ void final_max(const double* __restrict__ partials, unsigned nblocks,
                                          double (&v)[NACC], double* red) {
#pragma unroll
    for (int a = 0; a < NACC; ++a) v[a] = -1.0e308;
    for (unsigned b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
        for (int a = 0; a < NACC; ++a) v[a] = fmax(v[a], partials[(size_t)NACC * b + a]);
    }
#pragma unroll
    for (int a = 0; a < NACC; ++a) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[a] = fmax(v[a], __shfl_xor(v[a], off, 64));
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
    if (lane == 0) {
#pragma unroll
        for (int a = 0; a < NACC; ++a) red[a * 16 + wave] = v[a];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int a = 0; a < NACC; ++a) {
            double m = red[a * 16];
            for (int w = 1; w < nw; ++w) m = fmax(m, red[a * 16 + w]);
            v[a] = m;
        }
    }
    __syncthreads();
}

}  // namespace sgn
