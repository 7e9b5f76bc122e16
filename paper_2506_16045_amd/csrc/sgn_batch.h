// Batched independent 1D constraint solves in one launch: each workgroup takes
// whole systems G_{eta,h} u = b (Def:G in 1D) of its own size and runs the
// preconditioned CG of section 3.2 on them to completion, every vector in the
// half spectrum (modes 0..N/2) and every transform in LDS.  MODE_FP64 iterates
// in FP64; MODE_MIXED runs FP32 inner PCG solves of G d = r inside an FP64
// iterative refinement (outer residual r = b - G x, the stop test and x in
// FP64).  Per-system convergence: a workgroup moves to its next system as soon
// as the current one is done.
#pragma once

#include "sgn_kernels.h"

namespace sgn {

constexpr int BATCH_MMAX = 4096;                 // largest half length M = N/2
constexpr int BATCH_NMAX = 2 * BATCH_MMAX;       // 8192 points
// Size classes: a system of n <= 2048 points runs on 256 threads whose
// per-mode registers and transform tiling cover M <= 1024; a larger one on 512
// threads covering M <= 4096.  The class is a function of n alone, so a
// system's reductions, and its results, do not depend on what shares a launch.
__host__ __device__ constexpr int batch_threads_for(int n) { return n <= 2048 ? 256 : 512; }
template <int NT>
constexpr int batch_mmax() { return NT <= 256 ? 1024 : BATCH_MMAX; }
// Complex points per thread of one transform pass for a workgroup of NT threads.
template <int NT>
constexpr int batch_epc() { return batch_mmax<NT>() / NT; }
#ifndef SGN_BATCH_WAVES_SMALL
#define SGN_BATCH_WAVES_SMALL 2
#endif
// Waves per SIMD the compiler must leave room for (register budget): the small
// class keeps several workgroups resident per CU.
template <int NT>
constexpr int batch_waves() { return NT <= 256 ? SGN_BATCH_WAVES_SMALL : 1; }

enum { BATCH_FP64 = 0, BATCH_MIXED = 1 };

struct BatchItem {
    int n;           // grid points, a power of two in [2, BATCH_NMAX]
    int index;       // position of the system in the caller's order
    double L;        // period
    long long off;   // first point of the system in the packed field arrays
    long long wso;   // first double of the system's workspace
};

struct BatchResult {
    int iters;       // Krylov iterations (inner iterations in mixed mode)
    int outer;       // refinement steps (mixed mode)
    int converged;
    int status;      // 0, or -2: non-positive depth or non-finite data
    int flat;
    int pad;
    double relres, sig, alp, kap;
};

struct BatchParams {
    double tol, inner_tol;
    int max_iter, max_outer, x0_is_guess, coeff_kind, nitems;
    int flat;             // -1: flat formulas iff h_x == 0; 0 / 1: forced
    int have_coeffs;      // 1: use sig, alp, kap (and flat) as given
    int pad;
    double sig, alp, kap;
};

// Doubles of workspace one system of n points uses in the given mode.
__host__ __device__ inline long long batch_item_doubles(int n, int mode) {
    const long long M1 = n / 2 + 1;
    long long w = 5 * 2 * M1 + n;            // FP64: b, x, r, p, a_hat (spectral) + physical scratch
    if (mode == BATCH_MIXED) w += n;         // FP32 eta and h_x
    return (w + 1) & ~1LL;
}

// A value every lane of the wave holds alike, moved to scalar registers (the
// block-wide results below are read from LDS, which the compiler cannot see
// as uniform; in vector registers they would crowd the per-mode state).
__device__ __forceinline__ double uniform_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Workgroup scratch for block reductions: blk_allsum<NACC> and blk_allmax<NACC>
// use the first 17 NACC doubles; RED_PQ..RED_PQ+15 holds the wave partials of
// the PCG curvature between the pointwise pass and the forward transform.
constexpr int RED_PQ = 96;
constexpr int RED_DOUBLES = RED_PQ + 16;

// Block-wide sums of NACC doubles, the result in every thread (fixed order).
template <int NACC>
__device__ __forceinline__ void blk_allsum(double (&v)[NACC], double* red) {
    block_sum<NACC>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int a = 0; a < NACC; ++a) red[16 * NACC + a] = v[a];
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < NACC; ++a) v[a] = uniform_d(red[16 * NACC + a]);
    __syncthreads();
}

// Block-wide maxima of NACC doubles, the result in every thread.
template <int NACC>
__device__ __forceinline__ void blk_allmax(double (&v)[NACC], double* red) {
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
#pragma unroll
    for (int a = 0; a < NACC; ++a) {
        double m = red[a * 16];
        for (int w = 1; w < nw; ++w) m = fmax(m, red[a * 16 + w]);
        v[a] = uniform_d(m);
    }
    __syncthreads();
}

// Forward real transforms of N = 2M points, NF fields at buf + f fstride held
// as pairs buf[j] = (x_2j, x_2j+1), j < M: on return buf[k] = X_k =
// sum_n x_n W_N^{kn} for k = 0..M.  Whole block; the fields in lockstep.
template <typename T, int NT, int NF>
__device__ __forceinline__ void blk_rfft_fwd_n(cpx<T>* buf, int fstride, int M, const cpx<T>* __restrict__ tw_all) {
    __syncthreads();
    lds_fft<T, batch_epc<NT>(), NF>(buf, fstride, M, threadIdx.x, blockDim.x, tw_size(tw_all, M), false);
    const cpx<T>* tw2 = tw_size(tw_all, 2 * M);
    const T half = (T)0.5;
    for (int p = threadIdx.x; p <= M / 2; p += blockDim.x) {
        const int k = p, m = M - p;
        const cpx<T> wk = tw2[k], wm = tw2[m];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            cpx<T>* b = buf + f * fstride;
            if (p == 0) {
                const cpx<T> Z0 = b[0];
                b[0] = C<T>(Z0.re + Z0.im, 0);
                b[M] = C<T>(Z0.re - Z0.im, 0);
            } else {
                const cpx<T> Zk = b[k], Zm = b[m];
                const cpx<T> Xk = half * (Zk + cj(Zm)) - half * mul_i(wk * (Zk - cj(Zm)));
                if (m != k) b[m] = half * (Zm + cj(Zk)) - half * mul_i(wm * (Zm - cj(Zk)));
                b[k] = Xk;
            }
        }
    }
    __syncthreads();
}

// Inverse of blk_rfft_fwd_n up to the factor N: buf[k] = X_k (k = 0..M; the
// imaginary parts of X_0 and X_M are ignored) -> buf[j] = N (x_2j, x_2j+1).
template <typename T, int NT, int NF>
__device__ __forceinline__ void blk_rfft_inv_n(cpx<T>* buf, int fstride, int M, const cpx<T>* __restrict__ tw_all) {
    __syncthreads();
    const cpx<T>* tw2 = tw_size(tw_all, 2 * M);
    for (int p = threadIdx.x; p <= M / 2; p += blockDim.x) {
        const int k = p, m = M - p;
        cpx<T> wk = tw2[k], wm = tw2[m];
        wk.im = -wk.im;
        wm.im = -wm.im;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            cpx<T>* b = buf + f * fstride;
            if (p == 0) {
                const T x0 = b[0].re, xm = b[M].re;
                b[0] = C<T>(x0 + xm, x0 - xm);
            } else {
                const cpx<T> Xk = b[k], Xm = b[m];
                const cpx<T> Zk = (Xk + cj(Xm)) + mul_i((Xk - cj(Xm)) * wk);
                if (m != k) b[m] = (Xm + cj(Xk)) + mul_i((Xm - cj(Xk)) * wm);
                b[k] = Zk;
            }
        }
    }
    __syncthreads();
    lds_fft<T, batch_epc<NT>(), NF>(buf, fstride, M, threadIdx.x, blockDim.x, tw_size(tw_all, M), true);
}

template <typename T, int NT>
__device__ __forceinline__ void blk_rfft_fwd(cpx<T>* buf, int M, const cpx<T>* __restrict__ tw_all) {
    blk_rfft_fwd_n<T, NT, 1>(buf, 0, M, tw_all);
}

template <typename T, int NT>
__device__ __forceinline__ void blk_rfft_inv(cpx<T>* buf, int M, const cpx<T>* __restrict__ tw_all) {
    blk_rfft_inv_n<T, NT, 1>(buf, 0, M, tw_all);
}

// One system's view for G applies in precision T.
template <typename T>
struct BatchOp {
    int N, M;
    T tp;                        // 2 pi / L
    const T* eta;                // total depth, N points
    const T* hx;                 // bathymetry slope, N points
    T* scr;                      // N-point physical scratch
    cpx<T>* ah;                  // M+1 spectral scratch
    const cpx<T>* tw;
};

// q_hat = G v_hat (modes 0..M of the half spectrum).  The weak form of Def:G in
// 1D: a = eta (1 + h_x^2) v + eta^2/2 h_x Dv, w = eta^3/3 Dv + eta^2/2 h_x v,
// G v = a - D w.  The pointwise pass also sums v.Gv = sum (v a + Dv w), so the
// curvature is known (pq, every thread) before q_hat is formed; `fin(k, kk,
// q_k, pq)` then consumes q_hat mode by mode (kk the wavenumber) with the same
// thread mapping as every other mode loop of the system.
template <typename T, int NT, typename Fin>
__device__ __forceinline__ void blk_apply(const BatchOp<T>& A, const cpx<T>* vh, cpx<T>* lds, double* red,
                                          Fin&& fin) {
    const int M = A.M, N = A.N;
    const T invN = (T)1 / (T)N;
    // D v into the physical scratch
    for (int k = threadIdx.x; k <= M; k += blockDim.x) lds[k] = invN * ik(wavenumber<T>(k, N, A.tp), vh[k]);
    blk_rfft_inv<T, NT>(lds, M, A.tw);
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        A.scr[2 * j] = lds[j].re;
        A.scr[2 * j + 1] = lds[j].im;
    }
    __syncthreads();
    // v, then the pointwise products (a into LDS, w into the scratch)
    for (int k = threadIdx.x; k <= M; k += blockDim.x) lds[k] = invN * vh[k];
    blk_rfft_inv<T, NT>(lds, M, A.tw);
    const T third = (T)1 / (T)3, half = (T)0.5;
    double acc[1] = {0.0};
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        cpx<T> pv = lds[j];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int i = 2 * j + s;
            const T p = s ? pv.im : pv.re;
            const T dl = A.scr[i], et = A.eta[i], h = A.hx[i];
            const T bt = h * p, e2 = et * et;
            const T w1 = third * e2 * et * dl + half * e2 * bt;
            const T w2 = half * e2 * dl + et * bt;
            const T a = et * p + h * w2;
            acc[0] += (double)et * (double)p * (double)p + (double)dl * (double)w1 + (double)bt * (double)w2;
            A.scr[i] = w1;
            if (s) pv.im = a; else pv.re = a;
        }
        lds[j] = pv;
    }
    blk_allsum<1>(acc, red);
    const double pq = acc[0];
    // a_hat to the spectral scratch, then w_hat; q = a_hat - i k w_hat
    blk_rfft_fwd<T, NT>(lds, M, A.tw);
    for (int k = threadIdx.x; k <= M; k += blockDim.x) A.ah[k] = lds[k];
    __syncthreads();
    for (int j = threadIdx.x; j < M; j += blockDim.x) lds[j] = C<T>(A.scr[2 * j], A.scr[2 * j + 1]);
    blk_rfft_fwd<T, NT>(lds, M, A.tw);
    for (int k = threadIdx.x; k <= M; k += blockDim.x) {
        const T kk = wavenumber<T>(k, N, A.tp);
        fin(k, kk, A.ah[k] - ik(kk, lds[k]), pq);
    }
    __syncthreads();
}

// z = A^{-1} r for one mode (Def:A in 1D).
template <typename T>
__device__ __forceinline__ cpx<T> batch_precond(T kk, T sig, T alp, cpx<T> r) {
    return ((T)1 / (sig + alp * kk * kk)) * r;
}

template <typename T, typename U>
__device__ __forceinline__ cpx<T> cvt(cpx<U> v) {
    return C<T>((T)v.re, (T)v.im);
}

// PCG of section 3.2 on G d = r0 in precision T from d = 0, with the Krylov
// vectors d, r, p in the registers of the workgroup (mode k of the half
// spectrum in thread k mod NT, slot k / NT) and the transforms in two LDS
// buffers (lds and lds + M + 1: p and D p inverse-transformed in lockstep, a and
// w forward-transformed in lockstep), so the loop touches global memory for the
// coefficient fields at most (REGCOEF: eta and h_x held in registers too).
// r0 is read from r0h; on return xh += d (xh may hold a wider type).  Stops
// when r.r <= tol2 * bbref or after max_iter iterations; returns the
// iterations, rr the last r.r.
template <typename T, int NT, bool REGCOEF, typename TX>
__device__ int blk_pcg_reg(const BatchOp<T>& A, cpx<TX>* xh, const cpx<TX>* r0h, T sig, T alp, double tol2,
                           double bbref, int max_iter, double& rr, cpx<T>* lds, double* red) {
    constexpr int KPT = batch_mmax<NT>() / NT + 1;
    constexpr int JPT = batch_mmax<NT>() / NT;
    constexpr int JC = REGCOEF ? JPT : 1;
    const int M = A.M, N = A.N, t = threadIdx.x;
    const int fs = M + 1;
    cpx<T>* la = lds;
    cpx<T>* lb = lds + fs;
    const T invN = (T)1 / (T)N;
    const double dinvN = 1.0 / (double)N;
    // FP32 inner solves accumulate their correction in registers; the FP64 solve,
    // whose registers are fuller, adds each step to xh directly
    constexpr bool XREG = sizeof(T) == 4;
    cpx<T> x[XREG ? KPT : 1], r[KPT], p[KPT];
    T er[JC][2], hr[JC][2];
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int e = 0; e < KPT; ++e) {
        const int k = t + NT * e;
        if (XREG) x[XREG ? e : 0] = C<T>(0, 0);
        p[e] = C<T>(0, 0);
        r[e] = C<T>(0, 0);
        if (k <= M) {
            r[e] = cvt<T>(r0h[k]);
            const cpx<T> z = batch_precond<T>(wavenumber<T>(k, N, A.tp), sig, alp, r[e]);
            const double w = half_weight(k, N) * dinvN;
            acc[0] += w * ((double)r[e].re * (double)z.re + (double)r[e].im * (double)z.im);
            acc[1] += w * ((double)r[e].re * (double)r[e].re + (double)r[e].im * (double)r[e].im);
        }
    }
    if (REGCOEF) {
#pragma unroll
        for (int e = 0; e < JC; ++e) {
            const int j = t + NT * e;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                er[e][s] = j < M ? A.eta[2 * j + s] : (T)0;
                hr[e][s] = j < M ? A.hx[2 * j + s] : (T)0;
            }
        }
    }
    blk_allsum<2>(acc, red);
    double rz = acc[0];
    rr = acc[1];
    double rho_prev = 1.0;
    int it = 0;
    const T third = (T)1 / (T)3, half = (T)0.5;
    while (!(rr <= tol2 * bbref) && it < max_iter && rr == rr) {
        // FP64: the thread index, opaque to the compiler inside the loop, so that
        // per-mode indices, wavenumbers and weights are recomputed each iteration
        // instead of being hoisted into registers that the Krylov vectors need
        int t = threadIdx.x;
        if (!XREG) asm volatile("" : "+v"(t));
        const T beta = it == 0 ? (T)0 : (T)(rz / rho_prev);
        // p = z + beta p; p / N and i k p / N into the two buffers
#pragma unroll
        for (int e = 0; e < KPT; ++e) {
            const int k = t + NT * e;
            const T kk = wavenumber<T>(k, N, A.tp);
            const cpx<T> z = batch_precond<T>(kk, sig, alp, r[e]);
            p[e] = it == 0 ? z : z + beta * p[e];
            if (k <= M) {
                la[k] = invN * p[e];
                lb[k] = invN * ik(kk, p[e]);
            }
        }
        blk_rfft_inv_n<T, NT, 2>(lds, fs, M, A.tw);
        // pointwise: a into buffer a, w into buffer b; curvature p.Gp
        double pqa[1] = {0.0};
        constexpr int PU = REGCOEF ? JPT : 1;   // the FP64 loop reads eta, h_x from memory
#pragma unroll PU
        for (int e = 0; e < JPT; ++e) {
            const int j = t + NT * e;
            if (j < M) {
                cpx<T> pv = la[j], dv = lb[j];
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const T pp = s ? pv.im : pv.re;
                    const T dl = s ? dv.im : dv.re;
                    const T et = REGCOEF ? er[REGCOEF ? e : 0][s] : A.eta[2 * j + s];
                    const T h = REGCOEF ? hr[REGCOEF ? e : 0][s] : A.hx[2 * j + s];
                    const T bt = h * pp, e2 = et * et;
                    const T w1 = third * e2 * et * dl + half * e2 * bt;
                    const T w2 = half * e2 * dl + et * bt;
                    const T a = et * pp + h * w2;
                    pqa[0] += (double)et * (double)pp * (double)pp + (double)dl * (double)w1 + (double)bt * (double)w2;
                    if (s) {
                        pv.im = a;
                        dv.im = w1;
                    } else {
                        pv.re = a;
                        dv.re = w1;
                    }
                }
                la[j] = pv;
                lb[j] = dv;
            }
        }
        // p.Gp: wave sums now, the block sum (waves in order, as blk_allsum) after
        // the forward transform, whose barriers publish the wave partials
        {
            double x = pqa[0];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
            if ((threadIdx.x & 63) == 0) red[RED_PQ + (threadIdx.x >> 6)] = x;
        }
        blk_rfft_fwd_n<T, NT, 2>(lds, fs, M, A.tw);
        double pq = 0.0;
        for (int w = 0; w < NT / 64; ++w) pq += red[RED_PQ + w];
        pq = uniform_d(pq);
        const double rho = rz;
        const T alpha = (T)(rho / pq);
        acc[0] = acc[1] = 0.0;
#pragma unroll
        for (int e = 0; e < KPT; ++e) {
            const int k = t + NT * e;
            if (k <= M) {
                const T kk = wavenumber<T>(k, N, A.tp);
                const cpx<T> q = la[k] - ik(kk, lb[k]);
                if (XREG)
                    x[XREG ? e : 0] = x[XREG ? e : 0] + alpha * p[e];
                else
                    xh[k] = xh[k] + cvt<TX>(alpha * p[e]);
                r[e] = r[e] - alpha * q;
                const cpx<T> z = batch_precond<T>(kk, sig, alp, r[e]);
                const double w = half_weight(k, N) * dinvN;
                acc[0] += w * ((double)r[e].re * (double)z.re + (double)r[e].im * (double)z.im);
                acc[1] += w * ((double)r[e].re * (double)r[e].re + (double)r[e].im * (double)r[e].im);
            }
        }
        blk_allsum<2>(acc, red);
        rho_prev = rho;
        rz = acc[0];
        rr = acc[1];
        ++it;
    }
    if (XREG) {
#pragma unroll
        for (int e = 0; e < KPT; ++e) {
            const int k = t + NT * e;
            if (k <= M) xh[k] = xh[k] + cvt<TX>(x[XREG ? e : 0]);
        }
    }
    __syncthreads();
    return it;
}

// r_hat = b_hat - G x_hat in FP64, with its (r.z, r.r).
template <int NT>
__device__ __forceinline__ void blk_residual(const BatchOp<double>& A, const cpx<double>* bh, const cpx<double>* xh,
                                             cpx<double>* rh, double sig, double alp, double& rz, double& rr,
                                             cpx<double>* lds, double* red) {
    const double invN = 1.0 / (double)A.N;
    double acc[2] = {0.0, 0.0};
    blk_apply<double, NT>(A, xh, lds, red, [&](int k, double kk, cpx<double> q, double) {
        const cpx<double> r = bh[k] - q;
        rh[k] = r;
        const cpx<double> z = batch_precond<double>(kk, sig, alp, r);
        const double w = half_weight(k, A.N) * invN;
        acc[0] += w * (r.re * z.re + r.im * z.im);
        acc[1] += w * (r.re * r.re + r.im * r.im);
    });
    blk_allsum<2>(acc, red);
    rz = acc[0];
    rr = acc[1];
}

// Transform N physical FP64 points into modes 0..M (dst), returning sum x^2.
template <int NT>
__device__ __forceinline__ void blk_to_spectral(const double* x, int N, cpx<double>* dst,
                                                const cpx<double>* tw, cpx<double>* lds) {
    const int M = N / 2;
    for (int j = threadIdx.x; j < M; j += blockDim.x) lds[j] = C<double>(x[2 * j], x[2 * j + 1]);
    blk_rfft_fwd<double, NT>(lds, M, tw);
    for (int k = threadIdx.x; k <= M; k += blockDim.x) dst[k] = lds[k];
    __syncthreads();
}

// Next system of a block.  queue = null: a static stride over the table.
// Otherwise a work queue: the first round takes the block's own index, later
// systems come from a global counter (zero at launch) in table order, so a block
// that finishes early takes the next largest system.  Every thread of the block
// calls it; the result is the same in all of them.
__device__ __forceinline__ int batch_next(int* queue, int cur, int* slot) {
    if (!queue) return cur + gridDim.x;
    __syncthreads();
    if (threadIdx.x == 0) *slot = (int)gridDim.x + atomicAdd(queue, 1);
    __syncthreads();
    return *slot;
}

// One system's solve G u = b (section 3.2, Def:G in 1D) by the whole block:
// coefficients of section 4 from eta and h_x, b_hat, the initial residual
// (from u when `guess`, else from 0), PCG (FP64) or FP32 inner PCG inside FP64
// refinement (MIXED), and u (physical) on return; w is the system's workspace
// (batch_item_doubles).  Every thread of the block calls it.
template <int MODE, int NT>
__device__ __forceinline__ BatchResult blk_solve_system(const BatchItem& it, const double* __restrict__ eta,
                                        const double* __restrict__ hx, const double* __restrict__ b, double* u,
                                        bool guess, double* w, const cpx<double>* __restrict__ tw64,
                                        const cpx<float>* __restrict__ tw32, const BatchParams& prm,
                                        cpx<double>* lds64, cpx<float>* lds32, double* red) {
    const int N = it.n, M = N / 2;
    cpx<double>* bh = reinterpret_cast<cpx<double>*>(w);
    cpx<double>* xh = bh + (M + 1);
    cpx<double>* rh = xh + (M + 1);
    cpx<double>* ph = rh + (M + 1);
    BatchOp<double> A64;
    A64.N = N;
    A64.M = M;
    A64.tp = 6.283185307179586476925286766559 / it.L;
    A64.eta = eta;
    A64.hx = hx;
    A64.ah = ph + (M + 1);
    A64.scr = reinterpret_cast<double*>(A64.ah + (M + 1));
    A64.tw = tw64;
    BatchResult out{};
    // coefficients of section 4 from the extremes of eta and h_x
    const double lp = (4.0 + sqrt(13.0)) / 6.0;
    double ex[5] = {-1.0e308, -1.0e308, -1.0e308, 0.0, 0.0};
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double e = eta[i], h = hx[i], g2 = h * h;
        if (!isfinite(e) || !isfinite(g2) || !isfinite(b[i]) ||
            (guess && !isfinite(u[i])))
            ex[4] = 1.0;
        ex[0] = fmax(ex[0], -e);
        ex[1] = fmax(ex[1], e);
        ex[2] = fmax(ex[2], e + lp * e * g2);
        ex[3] = fmax(ex[3], g2);
    }
    blk_allmax<5>(ex, red);
    const double emin = -ex[0];
    if (ex[4] != 0.0 || !(emin > 0.0)) {
        out.status = -2;
        out.relres = __builtin_nan("");
        return out;
    }
    double sig, alp, kap;
    int fl;
    if (prm.have_coeffs) {
        sig = prm.sig;
        alp = prm.alp;
        kap = prm.kap;
        fl = prm.flat;
    } else {
        coeffs_formula(emin, ex[1], ex[2], ex[3], prm.flat, prm.coeff_kind, sig, alp, kap, fl);
    }
    out.sig = sig;
    out.alp = alp;
    out.kap = kap;
    out.flat = fl;
    // b_hat, ||b||^2, and the initial x_hat, r_hat
    blk_to_spectral<NT>(b, N, bh, tw64, lds64);
    double bb = 0.0, rz = 0.0, rr = 0.0;
    {
        double acc[2] = {0.0, 0.0};
        for (int k = threadIdx.x; k <= M; k += blockDim.x) {
            const cpx<double> b = bh[k];
            const double kk = wavenumber<double>(k, N, A64.tp);
            const cpx<double> z = batch_precond<double>(kk, sig, alp, b);
            const double wt = half_weight(k, N) / (double)N;
            acc[0] += wt * (b.re * z.re + b.im * z.im);
            acc[1] += wt * (b.re * b.re + b.im * b.im);
        }
        blk_allsum<2>(acc, red);
        bb = acc[1];
        rz = acc[0];
        rr = acc[1];
    }
    const double tol2 = prm.tol * prm.tol;
    if (guess && bb > 0.0) {
        blk_to_spectral<NT>(u, N, xh, tw64, lds64);
        blk_residual<NT>(A64, bh, xh, rh, sig, alp, rz, rr, lds64, red);
    } else {
        for (int k = threadIdx.x; k <= M; k += blockDim.x) {
            xh[k] = C<double>(0, 0);
            rh[k] = bh[k];
        }
        __syncthreads();
    }
    if (MODE == BATCH_FP64) {
        out.iters = blk_pcg_reg<double, NT, false>(A64, xh, rh, sig, alp, tol2, bb, prm.max_iter, rr, lds64, red);
    } else {
        // FP32 view of the same system: coefficient fields rounded once
        float* e32 = reinterpret_cast<float*>(A64.scr + N);
        float* h32 = e32 + N;
        BatchOp<float> A32;
        A32.N = N;
        A32.M = M;
        A32.tp = (float)A64.tp;
        A32.eta = e32;
        A32.hx = h32;
        A32.scr = nullptr;
        A32.ah = nullptr;
        A32.tw = tw32;
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            e32[i] = (float)eta[i];
            h32[i] = (float)hx[i];
        }
        __syncthreads();
        const float sig32 = (float)sig, alp32 = (float)alp;
        const double itol2 = prm.inner_tol * prm.inner_tol;
        while (!(rr <= tol2 * bb) && rr == rr && out.outer < prm.max_outer && bb > 0.0) {
            // inner FP32 solve of G d = r to t ||r||, then x += d and the FP64
            // residual r = b - G x; t = max(inner_tol, tol ||b|| / (2 ||r||)),
            // capped at 1/2: no tighter than the outer target needs
            double t2 = 0.25 * tol2 * (bb / rr);
            t2 = t2 < itol2 ? itol2 : (t2 > 0.25 ? 0.25 : t2);
            double irr = 0.0;
            out.iters += blk_pcg_reg<float, NT, true>(A32, xh, rh, sig32, alp32, t2, rr, prm.max_iter, irr,
                                                      lds32, red);
            blk_residual<NT>(A64, bh, xh, rh, sig, alp, rz, rr, lds64, red);
            out.outer += 1;
        }
    }
    out.converged = (bb == 0.0 || rr <= tol2 * bb) ? 1 : 0;
    out.relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    if (!(rr == rr)) out.status = -2;
    // u = x (physical)
    const double invN = 1.0 / (double)N;
    for (int k = threadIdx.x; k <= M; k += blockDim.x) lds64[k] = invN * xh[k];
    blk_rfft_inv<double, NT>(lds64, M, tw64);
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        u[2 * j] = lds64[j].re;
        u[2 * j + 1] = lds64[j].im;
    }
    __syncthreads();
    return out;
}

template <int MODE, int NT>
__global__ void __launch_bounds__(NT, batch_waves<NT>()) k_batch_solve(const BatchItem* __restrict__ items, int nitems,
                                                               const double* __restrict__ eta_all,
                                                               const double* __restrict__ hx_all,
                                                               const double* __restrict__ b_all,
                                                               double* __restrict__ u_all, double* __restrict__ ws,
                                                               const cpx<double>* __restrict__ tw64,
                                                               const cpx<float>* __restrict__ tw32, BatchParams prm,
                                                               BatchResult* __restrict__ res, int* queue) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<double>* lds64 = reinterpret_cast<cpx<double>*>(smem_raw);
    cpx<float>* lds32 = reinterpret_cast<cpx<float>*>(smem_raw);
    __shared__ double red[RED_DOUBLES];
    __shared__ int next_slot;
    for (int s = blockIdx.x; s < nitems; s = batch_next(queue, s, &next_slot)) {
        const BatchItem it = items[s];
        const BatchResult out =
            blk_solve_system<MODE, NT>(it, eta_all + it.off, hx_all + it.off, b_all + it.off, u_all + it.off,
                                       prm.x0_is_guess != 0, ws + it.wso, tw64, tw32, prm, lds64, lds32, red);
        if (threadIdx.x == 0) res[it.index] = out;
        __syncthreads();
    }
}

}  // namespace sgn

namespace sgn {

// Right-hand side f(w, p) of a 1D system (Eq:DSWEcf, Def:bigF, Eq:DAE_DSWE) by
// the whole workgroup: eta_t = -(eta u)_x, U_t = -eta (eta - h)_x - (eta u u)_x + F
// with F = S_x - T h_x, S and T of Def:bigF, (u.grad)^2 h read as u (u h_x)_x.
// All thirteen real transforms run in LDS; spec (5 (N/2+1) modes) and st (5 N
// points) are global scratch the workgroup owns.  Each thread always handles the
// same points and modes, so the scratch needs no barriers of its own.
template <int NT>
__device__ void blk_rhs_1d(int N, double L, const double* __restrict__ eta, const double* __restrict__ hx,
                           const double* __restrict__ u, double* __restrict__ eta_t, double* __restrict__ U_t,
                           cpx<double>* __restrict__ spec, double* __restrict__ st,
                           const cpx<double>* __restrict__ tw, cpx<double>* lds) {
    const int M = N / 2, M1 = M + 1;
    const double tp = 6.283185307179586476925286766559 / L;
    const double invN = 1.0 / (double)N;
    double* s_dl = st;
    double* s_P = st + N;
    double* s_m = st + 2 * N;
    double* s_Ut = st + 3 * N;
    double* s_Q = st + 4 * N;
    // forward transforms of u, eta u, eta, eta u u, beta = h_x u
    for (int f = 0; f < 5; ++f) {
        for (int j = threadIdx.x; j < M; j += NT) {
            double v[2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int i = 2 * j + s;
                const double e = eta[i], uu = u[i], h = hx[i];
                v[s] = f == 0 ? uu : f == 1 ? e * uu : f == 2 ? e : f == 3 ? e * uu * uu : h * uu;
            }
            lds[j] = C<double>(v[0], v[1]);
        }
        blk_rfft_fwd<double, NT>(lds, M, tw);
        for (int k = threadIdx.x; k <= M; k += NT) spec[f * M1 + k] = lds[k];
        __syncthreads();
    }
    // the derivative fields, consumed pointwise as they arrive:
    // delta = u_x, delta_x = u_xx, m = (eta u)_x, eta_x, (eta u u)_x, beta_x
    for (int q = 0; q < 6; ++q) {
        const int src = q <= 1 ? 0 : q - 1;
        for (int k = threadIdx.x; k <= M; k += NT) {
            const double kk = wavenumber<double>(k, N, tp);
            const cpx<double> X = spec[src * M1 + k];
            lds[k] = invN * (q == 1 ? (-kk * kk) * X : ik(kk, X));
        }
        blk_rfft_inv<double, NT>(lds, M, tw);
        for (int j = threadIdx.x; j < M; j += NT) {
            const cpx<double> z = lds[j];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int i = 2 * j + s;
                const double v = s ? z.im : z.re;
                if (q == 0) {
                    s_dl[i] = v;
                    s_P[i] = -v * v;
                } else if (q == 1) {
                    s_P[i] += u[i] * v;
                } else if (q == 2) {
                    s_m[i] = v;
                } else if (q == 3) {
                    s_Ut[i] = -eta[i] * (v - hx[i]);
                } else if (q == 4) {
                    s_Ut[i] = s_Ut[i] - v;
                } else {
                    s_Q[i] = u[i] * v;
                }
            }
        }
        __syncthreads();
    }
    // S, T, eta_t and U_t without S_x; then U_t += S_x
    for (int j = threadIdx.x; j < M; j += NT) {
        double sv[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int i = 2 * j + s;
            const double e = eta[i], h = hx[i], uu = u[i];
            const double bt = h * uu, e2 = e * e;
            const double mm = s_m[i], d0 = s_dl[i], pp = s_P[i], qq = s_Q[i];
            sv[s] = e2 * e / 3.0 * pp + e2 * mm * d0 + e2 / 2.0 * qq + e * mm * bt;
            const double Tv = e2 / 2.0 * pp + e * mm * d0 + e * qq + mm * bt;
            eta_t[i] = -mm;
            U_t[i] = s_Ut[i] - h * Tv;
        }
        lds[j] = C<double>(sv[0], sv[1]);
    }
    blk_rfft_fwd<double, NT>(lds, M, tw);
    for (int k = threadIdx.x; k <= M; k += NT) lds[k] = invN * ik(wavenumber<double>(k, N, tp), lds[k]);
    blk_rfft_inv<double, NT>(lds, M, tw);
    for (int j = threadIdx.x; j < M; j += NT) {
        const cpx<double> z = lds[j];
        U_t[2 * j] = z.re + U_t[2 * j];
        U_t[2 * j + 1] = z.im + U_t[2 * j + 1];
    }
}

template <int NT>
__global__ void __launch_bounds__(NT) k_rhs_1d(int N, double L, const double* __restrict__ eta,
                                               const double* __restrict__ hx, const double* __restrict__ u,
                                               double* __restrict__ eta_t, double* __restrict__ U_t,
                                               cpx<double>* __restrict__ spec, double* __restrict__ st,
                                               const cpx<double>* __restrict__ tw) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    blk_rhs_1d<NT>(N, L, eta, hx, u, eta_t, U_t, spec, st, tw, reinterpret_cast<cpx<double>*>(smem_raw));
}

// ---- batched RK4 stepping --------------------------------------------------
// Whole RK4 runs (Eq:ERK) of independent 1D states of up to BATCH_NMAX points,
// one workgroup per state: every right-hand side (blk_rhs_1d), stage
// combination and constraint solve (blk_solve_system) of every step runs inside
// the workgroup, so a run of any length is one launch.  The arithmetic of each
// step is that of the library's one-state stepper: the same stage values, the
// same initial guesses (the previous stage's velocity, or that plus the
// extrapolated offsets of the slot's last two solves) and the same sums.

constexpr int STEP_SLOTS = 4;   // solves of stages 2, 3, 4 and of the new level

struct StepItem {
    double *eta, *U, *u;           // state (in / out): total depth, U = G u, velocity
    double* hx;                    // bathymetry slope (written from h when h is set)
    const double* h;               // bathymetry, or null when hx and U are given
    double *fe[4], *fU[4];         // stage right-hand sides
    double *eta_s, *U_s, *u_s;     // stage values
    double* base;                  // velocity a solve started from
    double* off[STEP_SLOTS][2];    // offsets recorded by each slot's solves (ring of two)
    double* scr;                   // step_scratch_doubles(n, mode) doubles
    double L, dt;
    int n, index, nsteps, flat;    // flat: 0 / 1 (ignored when h is set)
    int cnt[STEP_SLOTS], head[STEP_SLOTS];
};

struct StepResult {
    long long iters, solves;
    int max_iters, converged, steps, status;   // status 0, -2 (domain) or -3 (a solve missed tol)
    int flat, pad;
    int cnt[STEP_SLOTS], head[STEP_SLOTS];
};

// Doubles of per-state scratch: the right-hand side's (5 (N/2+1) modes and 5 N
// points) or one solve's workspace, whichever is larger.
__host__ __device__ inline long long step_scratch_doubles(int n, int mode) {
    const long long rhs = 10LL * (n / 2 + 1) + 5LL * n;
    const long long sol = batch_item_doubles(n, mode);
    return rhs > sol ? rhs : sol;
}

// h_x = D h (zero when h is constant: the flat formulas apply) and U = G_{eta,h} u
// for a state given by eta, h and u.  False for non-finite h.
template <int NT>
__device__ bool blk_step_prepare(const StepItem& it, int& flat, const cpx<double>* __restrict__ tw,
                                 cpx<double>* lds, double* red) {
    const int N = it.n, M = N / 2;
    const double invN = 1.0 / (double)N, tp = 6.283185307179586476925286766559 / it.L;
    double ex[3] = {-1.0e308, -1.0e308, 0.0};
    for (int i = threadIdx.x; i < N; i += NT) {
        const double v = it.h[i];
        if (!isfinite(v)) ex[2] = 1.0;
        ex[0] = fmax(ex[0], -v);
        ex[1] = fmax(ex[1], v);
    }
    blk_allmax<3>(ex, red);
    if (ex[2] != 0.0) return false;
    flat = (-ex[0] == ex[1]) ? 1 : 0;
    if (flat) {
        for (int i = threadIdx.x; i < N; i += NT) it.hx[i] = 0.0;
    } else {
        for (int j = threadIdx.x; j < M; j += NT) lds[j] = C<double>(it.h[2 * j], it.h[2 * j + 1]);
        blk_rfft_fwd<double, NT>(lds, M, tw);
        for (int k = threadIdx.x; k <= M; k += NT) lds[k] = invN * ik(wavenumber<double>(k, N, tp), lds[k]);
        blk_rfft_inv<double, NT>(lds, M, tw);
        for (int j = threadIdx.x; j < M; j += NT) {
            it.hx[2 * j] = lds[j].re;
            it.hx[2 * j + 1] = lds[j].im;
        }
    }
    __syncthreads();
    // U = G u: u_hat, then q_hat = G u_hat (blk_apply) back to physical space
    cpx<double>* uh = reinterpret_cast<cpx<double>*>(it.scr);
    BatchOp<double> A;
    A.N = N;
    A.M = M;
    A.tp = tp;
    A.eta = it.eta;
    A.hx = it.hx;
    A.ah = uh + (M + 1);
    A.scr = reinterpret_cast<double*>(A.ah + (M + 1));
    A.tw = tw;
    blk_to_spectral<NT>(it.u, N, uh, tw, lds);
    blk_apply<double, NT>(A, uh, lds, red, [&](int k, double, cpx<double> q, double) { uh[k] = invN * q; });
    for (int k = threadIdx.x; k <= M; k += NT) lds[k] = uh[k];
    blk_rfft_inv<double, NT>(lds, M, tw);
    for (int j = threadIdx.x; j < M; j += NT) {
        it.U[2 * j] = lds[j].re;
        it.U[2 * j + 1] = lds[j].im;
    }
    __syncthreads();
    return true;
}

// G_{eta,h} u = U for stepper slot `slot`, u holding the base velocity on entry.
// With extrapolation the solve starts from base + o_1 (one recorded offset) or
// base + (2 o_1 - o_2) (two), and records u - base afterwards.  0, -2 or -3.
template <int MODE, int NT>
__device__ int blk_step_solve(const StepItem& it, StepResult& out, int slot, bool extrapolate, const double* eta,
                              const double* U, double* u, const cpx<double>* __restrict__ tw64,
                              const cpx<float>* __restrict__ tw32, const BatchParams& prm, cpx<double>* lds64,
                              cpx<float>* lds32, double* red) {
    const int N = it.n;
    int& cnt = out.cnt[slot];
    int& head = out.head[slot];
    const int nh = cnt == 0 ? head : head ^ 1;
    if (extrapolate) {
        const double* o1 = it.off[slot][head];
        const double* o2 = it.off[slot][head ^ 1];
        for (int i = threadIdx.x; i < N; i += NT) {
            const double b = u[i];
            it.base[i] = b;
            if (cnt == 1) {
                double s = 0.0;
                s += 1.0 * o1[i];
                u[i] = b + 1.0 * s;
            } else if (cnt >= 2) {
                double s = 0.0;
                s += 2.0 * o1[i];
                s += -1.0 * o2[i];
                u[i] = b + 1.0 * s;
            }
        }
        __syncthreads();
    }
    BatchItem bi;
    bi.n = N;
    bi.index = it.index;
    bi.L = it.L;
    bi.off = 0;
    bi.wso = 0;
    const BatchResult r = blk_solve_system<MODE, NT>(bi, eta, it.hx, U, u, true, it.scr, tw64, tw32, prm, lds64,
                                                     lds32, red);
    out.solves += 1;
    out.iters += r.iters;
    if (r.iters > out.max_iters) out.max_iters = r.iters;
    if (!r.converged) out.converged = 0;
    if (r.status != 0) return -2;
    if (!r.converged) return -3;
    if (extrapolate) {
        double* o = it.off[slot][nh];
        for (int i = threadIdx.x; i < N; i += NT) {
            double s = 0.0;
            s += -1.0 * it.base[i];
            o[i] = u[i] + 1.0 * s;
        }
        __syncthreads();
        head = nh;
        if (cnt < 2) cnt += 1;
    }
    return 0;
}

// RK4 steps of one state by the whole workgroup (Eq:ERK): stage i takes
// eta_n + dt a_i f^(i-1) and U_n + dt a_i f^(i-1) and solves G u^(i) = U^(i) from
// u^(i-1); the weighted sum advances eta and U, and u_{n+1} is solved from u^(4).
// A step counts once eta and U have advanced, even if its last solve fails.
template <int MODE, int NT>
__device__ StepResult blk_rk4_run(const StepItem& it, bool extrapolate, const cpx<double>* __restrict__ tw64,
                                  const cpx<float>* __restrict__ tw32, BatchParams prm, cpx<double>* lds64,
                                  cpx<float>* lds32, double* red) {
    StepResult out{};
    out.converged = 1;
#pragma unroll
    for (int k = 0; k < STEP_SLOTS; ++k) {
        out.cnt[k] = it.cnt[k];
        out.head[k] = it.head[k];
    }
    const int N = it.n;
    int flat = it.flat;
    if (it.h && !blk_step_prepare<NT>(it, flat, tw64, lds64, red)) {
        out.status = -2;
        return out;
    }
    out.flat = flat;
    prm.flat = flat ? 1 : 0;
    prm.have_coeffs = 0;
    prm.x0_is_guess = 1;
    cpx<double>* spec = reinterpret_cast<cpx<double>*>(it.scr);
    double* st = it.scr + 10LL * (N / 2 + 1);
    const double a[3] = {0.5, 0.5, 1.0};
    const double w[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    const double dt = it.dt;
    // phase k of a step: k > 0 forms stage k + 1's values (the new level for
    // k = 4) and solves for its velocity; k < 4 then evaluates f^(k) there.  One
    // call site for the solve and one for the right-hand side keep the kernel's
    // code (and register allocation) to a single copy of each.
    for (int n = 0; n < it.nsteps; ++n) {
        for (int k = 0; k <= 4; ++k) {
            if (k > 0) {
                const bool last = k == 4;
                for (int i = threadIdx.x; i < N; i += NT) {
                    if (!last) {
                        double s = 0.0;
                        s += a[k - 1] * it.fe[k - 1][i];
                        it.eta_s[i] = it.eta[i] + dt * s;
                        double q = 0.0;
                        q += a[k - 1] * it.fU[k - 1][i];
                        it.U_s[i] = it.U[i] + dt * q;
                    } else {
                        double s = 0.0, q = 0.0;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            s += w[j] * it.fe[j][i];
                            q += w[j] * it.fU[j][i];
                        }
                        it.eta[i] = it.eta[i] + dt * s;
                        it.U[i] = it.U[i] + dt * q;
                        it.u[i] = it.u_s[i];
                    }
                }
                __syncthreads();
                const int rc = blk_step_solve<MODE, NT>(it, out, k - 1, extrapolate, last ? it.eta : it.eta_s,
                                                        last ? it.U : it.U_s, last ? it.u : it.u_s, tw64, tw32, prm,
                                                        lds64, lds32, red);
                if (last) out.steps += 1;
                if (rc != 0) {
                    out.status = rc;
                    return out;
                }
            }
            if (k < 4) {
                blk_rhs_1d<NT>(N, it.L, k ? it.eta_s : it.eta, it.hx, k ? it.u_s : it.u, it.fe[k], it.fU[k], spec,
                               st, tw64, lds64);
                __syncthreads();
                if (k == 0) {
                    for (int i = threadIdx.x; i < N; i += NT) it.u_s[i] = it.u[i];
                    __syncthreads();
                }
            }
        }
    }
    return out;
}

// Batched RK4 runs: workgroups take states from the table (a work queue when
// queue is set, its counter zero at launch) until none is left.  LDS: two FP64
// transform buffers of the largest state's N/2 + 1 modes.
template <int MODE, int NT>
__global__ void __launch_bounds__(NT, batch_waves<NT>()) k_batch_rk4(const StepItem* __restrict__ items, int nitems,
                                                  const cpx<double>* __restrict__ tw64,
                                                  const cpx<float>* __restrict__ tw32, BatchParams prm,
                                                  int extrapolate, StepResult* __restrict__ res, int* queue) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<double>* lds64 = reinterpret_cast<cpx<double>*>(smem_raw);
    cpx<float>* lds32 = reinterpret_cast<cpx<float>*>(smem_raw);
    __shared__ double red[RED_DOUBLES];
    __shared__ int next_slot;
    for (int s = blockIdx.x; s < nitems; s = batch_next(queue, s, &next_slot)) {
        // the table entry stays in memory and is read where used (uniform loads)
        const StepItem& it = items[__builtin_amdgcn_readfirstlane(s)];
        const StepResult out = blk_rk4_run<MODE, NT>(it, extrapolate != 0, tw64, tw32, prm, lds64, lds32, red);
        if (threadIdx.x == 0) res[it.index] = out;
        __syncthreads();
    }
}

}  // namespace sgn
