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
// with a final radix-2 pass when log2 M is odd.  A real row of length nx is
// transformed as a complex sequence of length M = nx/2 (z_j = x_2j + i x_2j+1)
// followed by the usual even/odd split; twiddles come from one table of
// W^k = exp(-2 pi i k / TW), TW = 16384.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sgn {

constexpr int TW_LOG = 14;
constexpr int TW_SIZE = 1 << TW_LOG;

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
// Stockham FFT of length M (power of two) in LDS buffer `buf`, executed by TPX
// cooperating threads (thread index t).  Every thread of the block must call
// it (it contains block barriers); EPC bounds the elements per thread
// (M <= EPC * TPX).  Forward: exp(-i ...); inverse: exp(+i ...), unnormalised.
// ---------------------------------------------------------------------------
template <typename T, int EPC>
__device__ __forceinline__ void lds_fft(cpx<T>* buf, int M, int t, int TPX,
                                        const cpx<T>* __restrict__ tw, bool inverse) {
    constexpr int NB4 = EPC / 4 > 0 ? EPC / 4 : 1;
    constexpr int NB2 = EPC / 2 > 0 ? EPC / 2 : 1;
    const int M4 = M >> 2;
    int Ns = 1;
    int logNs = 0;
    for (; Ns * 4 <= M; Ns <<= 2, logNs += 2) {
        cpx<T> v[NB4][4];
        const int sh = TW_LOG - (logNs + 2);
#pragma unroll
        for (int i = 0; i < NB4; ++i) {
            const int j = t + i * TPX;
            if (j < M4) {
                const int k = j & (Ns - 1);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    cpx<T> a = buf[j + r * M4];
                    if (r > 0) {
                        cpx<T> w = tw[(k * r) << sh];
                        if (inverse) w.im = -w.im;
                        a = a * w;
                    }
                    v[i][r] = a;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NB4; ++i) {
            const int j = t + i * TPX;
            if (j < M4) {
                const int k = j & (Ns - 1);
                const cpx<T> a0 = v[i][0] + v[i][2];
                const cpx<T> a1 = v[i][0] - v[i][2];
                const cpx<T> a2 = v[i][1] + v[i][3];
                const cpx<T> d = v[i][1] - v[i][3];
                const cpx<T> a3 = inverse ? mul_i(d) : mul_mi(d);
                const int o = ((j - k) << 2) + k;
                buf[o] = a0 + a2;
                buf[o + Ns] = a1 + a3;
                buf[o + 2 * Ns] = a0 - a2;
                buf[o + 3 * Ns] = a1 - a3;
            }
        }
        __syncthreads();
    }
    if (Ns < M) {  // one radix-2 pass remains (log2 M odd)
        const int M2 = M >> 1;
        const int sh = TW_LOG - (logNs + 1);
        cpx<T> v[NB2][2];
#pragma unroll
        for (int i = 0; i < NB2; ++i) {
            const int j = t + i * TPX;
            if (j < M2) {
                const int k = j & (Ns - 1);
                cpx<T> w = tw[k << sh];
                if (inverse) w.im = -w.im;
                v[i][0] = buf[j];
                v[i][1] = buf[j + M2] * w;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NB2; ++i) {
            const int j = t + i * TPX;
            if (j < M2) {
                const int k = j & (Ns - 1);
                const int o = ((j - k) << 1) + k;
                buf[o] = v[i][0] + v[i][1];
                buf[o + Ns] = v[i][0] - v[i][1];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Row geometry: a block holds R rows of TPR threads each; row r of the block is
// grid row row0 + r.  Thread t of a row owns complex positions j = t + TPR*e
// (e < EPC), i.e. real positions 2j and 2j+1.
// ---------------------------------------------------------------------------
struct RowGeom {
    int nx, ny, M, TPR, R, nblocks;
};

template <typename T>
struct RowThread {
    int r, t, y, row0;
    bool valid;
    cpx<T>* buf;  // this row's LDS buffer, M+1 entries
    cpx<T>* lds;  // block LDS base (R rows of stride M+1)
};

// Map a launch block index to a row group so that consecutive row groups land on
// the same XCD (blocks are dealt round-robin over 8 XCDs, each with its own L2):
// neighbouring row groups share the cache lines of the transposed H layout.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

template <typename T>
__device__ __forceinline__ RowThread<T> row_thread(const RowGeom& g, cpx<T>* lds) {
    RowThread<T> rt;
    rt.r = threadIdx.x / g.TPR;
    rt.t = threadIdx.x - rt.r * g.TPR;
    rt.row0 = xcd_remap(blockIdx.x, g.nblocks) * g.R;
    rt.y = rt.row0 + rt.r;
    rt.valid = rt.y < g.ny;
    rt.lds = lds;
    rt.buf = lds + rt.r * (g.M + 1);
    return rt;
}

// Inverse row transform: H[kx][y] (kx = 0..M) -> real pairs z[e] = (x_2j, x_2j+1),
// unnormalised (returns nx times the inverse DFT).  The imaginary parts of the
// kx = 0 and kx = nx/2 entries are ignored (real signal).
template <typename T, int EPC>
__device__ __forceinline__ void row_inverse(const RowGeom& g, const RowThread<T>& rt,
                                            const cpx<T>* __restrict__ H,
                                            const cpx<T>* __restrict__ tw, cpx<T> (&z)[EPC]) {
    const int M = g.M, R = g.R, ny = g.ny;
    const int total = R * (M + 1);
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
        const int r = i & (R - 1);
        const int kx = i / R;
        const int y = rt.row0 + r;
        rt.lds[r * (M + 1) + kx] = (y < ny) ? H[(size_t)kx * ny + y] : C<T>(0, 0);
    }
    __syncthreads();
    const int sh = TW_LOG - ilog2(2 * M);  // W_nx^k = tw[k << sh]
    for (int p = rt.t; p <= M / 2; p += g.TPR) {
        cpx<T>* b = rt.buf;
        if (p == 0) {
            const T x0 = b[0].re, xm = b[M].re;
            b[0] = C<T>(x0 + xm, x0 - xm);
        } else {
            const int k = p, m = M - p;
            const cpx<T> Xk = b[k], Xm = b[m];
            cpx<T> wk = tw[k << sh];
            wk.im = -wk.im;
            const cpx<T> Zk = (Xk + cj(Xm)) + mul_i((Xk - cj(Xm)) * wk);
            if (m != k) {
                cpx<T> wm = tw[m << sh];
                wm.im = -wm.im;
                const cpx<T> Zm = (Xm + cj(Xk)) + mul_i((Xm - cj(Xk)) * wm);
                b[m] = Zm;
            }
            b[k] = Zk;
        }
    }
    __syncthreads();
    lds_fft<T, EPC>(rt.buf, M, rt.t, g.TPR, tw, true);
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
        const int j = rt.t + g.TPR * e;
        if (j < M) z[e] = rt.buf[j];
    }
    __syncthreads();
}

// Forward row transform: real pairs z[e] -> H[kx][y] for kx = 0..M, each value
// multiplied by `scale`.
template <typename T, int EPC>
__device__ __forceinline__ void row_forward(const RowGeom& g, const RowThread<T>& rt,
                                            const cpx<T> (&z)[EPC], cpx<T>* __restrict__ H,
                                            const cpx<T>* __restrict__ tw, T scale) {
    const int M = g.M, R = g.R, ny = g.ny;
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
        const int j = rt.t + g.TPR * e;
        if (j < M) rt.buf[j] = z[e];
    }
    __syncthreads();
    lds_fft<T, EPC>(rt.buf, M, rt.t, g.TPR, tw, false);
    const int sh = TW_LOG - ilog2(2 * M);
    const T half = (T)0.5;
    for (int p = rt.t; p <= M / 2; p += g.TPR) {
        cpx<T>* b = rt.buf;
        if (p == 0) {
            const cpx<T> Z0 = b[0];
            b[0] = C<T>(Z0.re + Z0.im, 0);
            b[M] = C<T>(Z0.re - Z0.im, 0);
        } else {
            const int k = p, m = M - p;
            const cpx<T> Zk = b[k], Zm = b[m];
            const cpx<T> wk = tw[k << sh];
            const cpx<T> Xk = half * (Zk + cj(Zm)) - half * mul_i(wk * (Zk - cj(Zm)));
            if (m != k) {
                const cpx<T> wm = tw[m << sh];
                const cpx<T> Xm = half * (Zm + cj(Zk)) - half * mul_i(wm * (Zm - cj(Zk)));
                b[m] = Xm;
            }
            b[k] = Xk;
        }
    }
    __syncthreads();
    const int total = R * (M + 1);
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
        const int r = i & (R - 1);
        const int kx = i / R;
        const int y = rt.row0 + r;
        if (y < ny) H[(size_t)kx * ny + y] = scale * rt.lds[r * (M + 1) + kx];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Column geometry: a block holds Cb columns (kx) of TPC threads each; column c
// is kx = blockIdx.x * Cb + c.  Thread t owns modes j = t + TPC*e (e < EPC, j < ny).
// ---------------------------------------------------------------------------
struct ColGeom {
    int nx, ny, nxh, TPC, Cb, nblocks;
};

template <typename T>
struct ColThread {
    int c, t, kx;
    bool valid;
    cpx<T>* buf;
};

template <typename T>
__device__ __forceinline__ ColThread<T> col_thread(const ColGeom& g, cpx<T>* lds) {
    ColThread<T> ct;
    ct.c = threadIdx.x / g.TPC;
    ct.t = threadIdx.x - ct.c * g.TPC;
    ct.kx = blockIdx.x * g.Cb + ct.c;
    ct.valid = ct.kx < g.nxh;
    ct.buf = lds + ct.c * g.ny;
    return ct;
}

// Load a column of H (or S) and optionally transform it along y.
template <typename T, int EPC>
__device__ __forceinline__ void col_load(const ColGeom& g, const ColThread<T>& ct,
                                         const cpx<T>* __restrict__ H, bool fft,
                                         const cpx<T>* __restrict__ tw, cpx<T> (&v)[EPC]) {
    const int ny = g.ny;
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
        const int j = ct.t + g.TPC * e;
        if (j < ny) v[e] = ct.valid ? H[(size_t)ct.kx * ny + j] : C<T>(0, 0);
    }
    if (fft && ny > 1) {
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = ct.t + g.TPC * e;
            if (j < ny) ct.buf[j] = v[e];
        }
        __syncthreads();
        lds_fft<T, EPC>(ct.buf, ny, ct.t, g.TPC, tw, false);
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = ct.t + g.TPC * e;
            if (j < ny) v[e] = ct.buf[j];
        }
        __syncthreads();
    }
}

// Optionally inverse-transform along y, then store a column of H (or S).
template <typename T, int EPC>
__device__ __forceinline__ void col_store(const ColGeom& g, const ColThread<T>& ct,
                                          cpx<T> (&v)[EPC], cpx<T>* __restrict__ H, bool ifft,
                                          const cpx<T>* __restrict__ tw) {
    const int ny = g.ny;
    if (ifft && ny > 1) {
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = ct.t + g.TPC * e;
            if (j < ny) ct.buf[j] = v[e];
        }
        __syncthreads();
        lds_fft<T, EPC>(ct.buf, ny, ct.t, g.TPC, tw, true);
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = ct.t + g.TPC * e;
            if (j < ny) v[e] = ct.buf[j];
        }
        __syncthreads();
    }
    if (ct.valid) {
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = ct.t + g.TPC * e;
            if (j < ny) H[(size_t)ct.kx * ny + j] = v[e];
        }
    }
}

// ---------------------------------------------------------------------------
// Deterministic reductions.  Each block reduces NACC doubles in a fixed tree
// (wave shuffles, then waves in order) and writes them to partials[block];
// the last block to finish sums the partials in block order, so the result
// does not depend on scheduling.
// ---------------------------------------------------------------------------
template <int NACC>
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
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int a = 0; a < NACC; ++a) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += red[a * 16 + w];
            v[a] = s;
        }
    }
    __syncthreads();
}

// Sum of the per-block partials (layout partials[NACC*b + a]) by the whole
// last block: thread t adds blocks t, t+blockDim, ... in order, then the fixed
// block tree; the result is in thread 0.  Every thread of the block must call it.
template <int NACC>
__device__ __forceinline__ void final_sum(const double* __restrict__ partials, unsigned nblocks,
                                          double (&v)[NACC], double* red) {
#pragma unroll
    for (int a = 0; a < NACC; ++a) v[a] = 0.0;
    for (unsigned b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
        for (int a = 0; a < NACC; ++a) v[a] += partials[(size_t)NACC * b + a];
    }
    block_sum<NACC>(v, red);
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
