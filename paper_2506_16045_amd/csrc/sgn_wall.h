// Krylov passes of a 2D grid between walls on its own points (homogeneous
// Neumann boundaries, Subsec:DAEform and Subsec:linop; the cosine / sine series
// reading: scalars are cosine series on both axes, the velocity component u is a
// sine series along x and a cosine series along y, v the transpose).
//
// Transform order.  Read a real line f_0 .. f_{n-1} as v_i = f_{2i} for i < n/2
// and v_i = f_{2(n-1-i)+1} for i >= n/2, and let V be the DFT of v and
// w_k = exp(-i pi k / 2n).  Then w_k V_k = C_k - i C_{n-k} for the cosine sums
// C_k = sum_j f_j cos(pi k (2j+1) / 2n) (C_n = 0).  A sine line read with the sign
// (-1)^j, which is -1 exactly on the second half of the order, has as its cosine
// sums C_{n-m} the sine sums sum_j f_j sin(pi m (2j+1) / 2n) of mode m.  Fields put
// in this order (k_wall_order) therefore go through the periodic row transforms
// and column FFTs unchanged; only the column passes turn FFT values into series
// amplitudes and back.  The row pass of the iteration is the periodic one: its
// pointwise operator sees eta and grad h in the same order, grad h signed like
// the velocity (sign^2 = 1 keeps grad h . p and the B-density unchanged).
//
// Slots.  The amplitude of mode m on an axis of n points sits at slot m mod n:
// the sine Nyquist mode n, whose wavenumber is zero (section 6.1), shares slot 0
// with the cosine mode 0.  With kappa_s = s pi / L every operator of the
// iteration is diagonal in slots: d/dx takes a cosine amplitude to the sine one
// times -kappa and a sine amplitude to the cosine one times +kappa, and A^{-1}
// (Def:A) is the periodic split along and across k with real wavenumbers.
// S layout: column k = 0 .. nx/2 holds (slot k, slot nx - k) as (re, im) at every
// y slot; column 0 has no second slot (im = 0), and at k = nx/2 both parts hold
// the same amplitude.  The amplitudes are the unnormalised sums, so that
// sum_points f g = sum_slots c_x c_y F G / (nx ny) with c = 1 at slot 0 and 2
// elsewhere (Parseval for the cosine / sine sums).
#pragma once
#include "sgn_kernels.h"

namespace sgn {

// Grid index of transform-order position i on an axis of n points, and back.
__device__ __forceinline__ int wall_from_order(int i, int n) { return i < n / 2 ? 2 * i : 2 * (n - 1 - i) + 1; }
__device__ __forceinline__ int wall_to_order(int j, int n) { return (j & 1) ? n - 1 - (j >> 1) : j >> 1; }

// nf fields of nx x ny points between grid order and transform order: to_order
// writes dst[order] = sign * src[grid], otherwise dst[grid] = sign * src[order].
// Field f is a sine series along x when bit f of sx is set, along y for sy.
__global__ void __launch_bounds__(256) k_wall_order(int nx, int ny, int nf, unsigned sx, unsigned sy, int to_order,
                                                     const double* __restrict__ src, double* __restrict__ dst) {
    const size_t N = (size_t)nx * ny, total = N * nf;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int f = (int)(i / N);
        const size_t r = i - (size_t)f * N;
        const int y = (int)(r / nx), x = (int)(r - (size_t)y * nx);
        int oy, ox, gy, gx;
        if (to_order) {
            oy = y;
            ox = x;
            gy = wall_from_order(y, ny);
            gx = wall_from_order(x, nx);
        } else {
            gy = y;
            gx = x;
            oy = wall_to_order(y, ny);
            ox = wall_to_order(x, nx);
        }
        double s = 1.0;
        if (((sx >> f) & 1u) && 2 * ox >= nx) s = -s;
        if (((sy >> f) & 1u) && 2 * oy >= ny) s = -s;
        const size_t from = to_order ? (size_t)gy * nx + gx : (size_t)oy * nx + ox;
        dst[i] = s * src[(size_t)f * N + from];
    }
}

// Column FFT values F1 = F[q], F2 = F[ny - q] of column k -> the field's
// amplitudes at y slots q and ny - q.  wx = w_k of the
// x axis (4 nx roots), wy = w_q of the y axis; xs / ys: sine series along x / y.
// The column holds the x-line sums C_k - i C_{nx-k} of every row, so
// P_a = (F1 + conj F2) / 2 and P_b = i (F1 - conj F2) / 2 are the y-DFTs of the
// real columns C_k and C_{nx-k}; w_q P = E_q - i E_{ny-q} gives their y sums.
template <typename T>
__device__ __forceinline__ void wall_to_slots(cpx<T> F1, cpx<T> F2, cpx<T> wx, cpx<T> wy, bool k0, bool q0, bool xs,
                                              bool ys, cpx<T>& Sq, cpx<T>& Sm) {
    F1 = wx * F1;
    F2 = wx * F2;
    const T h = (T)0.5;
    const cpx<T> ua = wy * (h * (F1 + cj(F2)));
    const cpx<T> ub = wy * (h * mul_i(F1 - cj(F2)));
    T aq = ua.re, am = -ua.im, bq = ub.re, bm = -ub.im;
    if (k0) {
        bq = (T)0;
        bm = (T)0;
    } else if (xs) {   // x-line sums C_k, C_{nx-k} are the sine modes nx-k, k
        const T t0 = aq, t1 = am;
        aq = bq;
        am = bm;
        bq = t0;
        bm = t1;
    }
    const cpx<T> vq = C<T>(aq, bq), vm = C<T>(am, bm);
    if (ys && !q0) {
        Sq = vm;
        Sm = vq;
    } else {
        Sq = vq;
        Sm = vm;
    }
}

// The inverse of wall_to_slots: amplitudes at y slots q and ny - q (the same
// value twice for q = 0 and q = ny/2) -> the column values F[q], F[ny - q] whose
// inverse y-FFT and inverse row transform give the field in transform order
// (times nx ny).
template <typename T>
__device__ __forceinline__ void wall_from_slots(cpx<T> Sq, cpx<T> Sm, cpx<T> wx, cpx<T> wy, bool k0, bool q0, bool xs,
                                                bool ys, cpx<T>& F1, cpx<T>& F2) {
    cpx<T> eq, em;
    if (q0) {
        eq = Sq;
        em = C<T>(0, 0);
    } else if (ys) {
        eq = Sm;
        em = Sq;
    } else {
        eq = Sq;
        em = Sm;
    }
    T aq, am, bq, bm;
    if (k0) {
        aq = eq.re;
        am = em.re;
        bq = (T)0;
        bm = (T)0;
    } else if (xs) {
        aq = eq.im;
        am = em.im;
        bq = eq.re;
        bm = em.re;
    } else {
        aq = eq.re;
        am = em.re;
        bq = eq.im;
        bm = em.im;
    }
    const cpx<T> wyc = cj(wy), wxc = cj(wx);
    const cpx<T> pa = wyc * C<T>(aq, -am), pb = wyc * C<T>(bq, -bm);
    F1 = wxc * (pa - mul_i(pb));
    F2 = wxc * (cj(pa) - mul_i(cj(pb)));
}

// z = A^{-1} r for one real amplitude pair (r0 of u, r1 of v) of wavenumber
// (kx, ky): the split of precond_mode with real values.
template <typename T>
__device__ __forceinline__ void wall_precond(T kx, T ky, T sig, T alp, T r0, T r1, T& z0, T& z1) {
    const T k2 = kx * kx + ky * ky;
    const T is = (T)1 / sig;
    if (k2 == (T)0) {
        z0 = is * r0;
        z1 = is * r1;
        return;
    }
    const T kr = ((T)1 / k2) * (kx * r0 + ky * r1);
    const T px = kx * kr, py = ky * kr;
    const T ip = (T)1 / (sig + alp * k2);
    z0 = is * (r0 - px) + ip * px;
    z1 = is * (r1 - py) + ip * py;
}

// Per-column constants: x twiddle, the two x wavenumbers (re: slot k, im: slot
// nx - k) and their Parseval factors.
template <typename T>
struct WallColumn {
    cpx<T> wx;
    T kre, kim;
    double cre, cim;
    bool k0;
};
template <typename T>
__device__ __forceinline__ WallColumn<T> wall_column(const ColGeom& g, const ColThread<T>& ct,
                                                     const cpx<T>* __restrict__ tw, T pix) {
    WallColumn<T> w;
    const int k = ct.valid ? ct.kx : 0;
    w.k0 = k == 0;
    const bool kh = 2 * k == g.nx;
    w.wx = tw_size(tw, 4 * g.nx)[k];
    w.kre = (T)k * pix;
    w.kim = w.k0 ? (T)0 : (T)(g.nx - k) * pix;
    w.cre = (w.k0 || kh) ? 1.0 : 2.0;
    w.cim = w.k0 ? 0.0 : (kh ? 1.0 : 2.0);
    return w;
}

// Load NF H columns into LDS and y-FFT them there (the values stay in LDS; the
// FFT ends with a block barrier).
template <typename T, int EPC, int NF>
__device__ __forceinline__ void wall_col_fft(const ColGeom& g, const ColThread<T>& ct, const cpx<T>* const (&H)[NF],
                                             const cpx<T>* twm) {
    const int ny = g.ny;
    cpx<T> v[NF][EPC];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = ct.t + g.TPC * e;
            v[f][e] = (ct.valid && j < ny) ? H[f][(size_t)ct.kx * ny + j] : C<T>(0, 0);
        }
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = ct.t + g.TPC * e;
            if (j < ny) ct.buf[f * ct.fstride + j] = v[f][e];
        }
    __syncthreads();
    lds_fft<T, EPC, NF>(ct.buf, ct.fstride, ny, ct.t, g.TPC, twm, false);
}

// Inverse y-FFT of the NF columns the threads wrote to LDS, then store to H.
template <typename T, int EPC, int NF>
__device__ __forceinline__ void wall_col_emit(const ColGeom& g, const ColThread<T>& ct, cpx<T>* const (&H)[NF],
                                              const cpx<T>* twm) {
    const int ny = g.ny;
    __syncthreads();
    lds_fft<T, EPC, NF>(ct.buf, ct.fstride, ny, ct.t, g.TPC, twm, true);
    if (ct.valid) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                const int j = ct.t + g.TPC * e;
                if (j < ny) H[f][(size_t)ct.kx * ny + j] = ct.buf[f * ct.fstride + j];
            }
    }
}

// Kinds of the three fields of a pass: u (sine x), v (sine y), the scalar.
__device__ __forceinline__ bool wall_xs(int f) { return f == 0; }
__device__ __forceinline__ bool wall_ys(int f) { return f == 1; }

// Each kernel walks the pairs of y slots (q, ny - q), q = 0 .. ny/2, of its
// column: thread t takes q = t + TPC e for e = 0 .. EPC/2 (the last only for
// t = 0); q = 0 and q = ny/2 pair with themselves.

// First column pass of a wall solve (the k_pcg_setup of the periodic grid): Hb
// holds the row transforms of b in transform order, Hu those of the guess.  b's
// amplitudes -> rh (and bh); GUESS: partial ||b||^2, and on the second half of
// the blocks the guess's amplitudes -> xh with (x, div x) / (nx ny) inverse
// transformed into H for the row pass of G x_0; otherwise xh = 0 and the
// partials r.z, r.r of r_0 = b.
template <typename T, int EPC, bool GUESS>
__global__ void __launch_bounds__(256) k_wall_setup(ColGeom g, const cpx<T>* __restrict__ tw,
                                                     const SolveScal* __restrict__ sc, const cpx<T>* Hb,
                                                     const cpx<T>* __restrict__ Hu, size_t NS, cpx<T>* __restrict__ bh,
                                                     cpx<T>* __restrict__ rh, cpx<T>* __restrict__ xh, cpx<T>* H,
                                                     double* __restrict__ part, T pix, T piy) {
    if (sc->done) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    __shared__ double red[32];
    const cpx<T>* twm = twl_setup<T>(tw, g.ny, lds + col_lds_data(g, 3));
    const int job = GUESS ? (int)blockIdx.x / g.nblocks : 0;
    const ColThread<T> ct = col_thread_at<T>(g, lds, (int)blockIdx.x - job * g.nblocks);
    const WallColumn<T> wc = wall_column<T>(g, ct, tw, pix);
    const cpx<T>* twy = tw_size(tw, 4 * g.ny);
    const T sig = (T)sc->sig, alp = (T)sc->alp, inv_n = (T)sc->inv_n;
    const size_t col = (size_t)ct.kx * g.ny;
    if (GUESS && job == 1) {
        {
            const cpx<T>* srcs[2] = {Hu, Hu + NS};
            wall_col_fft<T, EPC, 2>(g, ct, srcs, twm);
        }
#pragma unroll
        for (int e_ = 0; e_ <= EPC / 2; ++e_) {
            const int q = ct.t + g.TPC * e_;
            if (q > g.ny / 2) continue;
            const int m = (g.ny - q) & (g.ny - 1);
            const bool self = q == m;
            const cpx<T> wy = twy[q];
            cpx<T> a[2][2];
#pragma unroll
            for (int f = 0; f < 2; ++f)
                wall_to_slots<T>(ct.buf[f * ct.fstride + q], ct.buf[f * ct.fstride + m], wc.wx, wy, wc.k0, q == 0,
                                 wall_xs(f), wall_ys(f), a[f][0], a[f][1]);
            cpx<T> o[3][2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int ysl = s ? m : q;
                const T ky = (T)ysl * piy;
                if (ct.valid && (s == 0 || !self)) {
                    xh[col + ysl] = a[0][s];
                    xh[NS + col + ysl] = a[1][s];
                }
                o[0][s] = inv_n * a[0][s];
                o[1][s] = inv_n * a[1][s];
                o[2][s] = inv_n * C<T>(wc.kre * a[0][s].re + ky * a[1][s].re, wc.kim * a[0][s].im + ky * a[1][s].im);
            }
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                cpx<T> F1, F2;
                wall_from_slots<T>(o[f][0], self ? o[f][0] : o[f][1], wc.wx, wy, wc.k0, q == 0, wall_xs(f),
                                   wall_ys(f), F1, F2);
                ct.buf[f * ct.fstride + q] = F1;
                if (!self) ct.buf[f * ct.fstride + m] = F2;
            }
        }
        cpx<T>* dsts[3] = {H, H + NS, H + 2 * NS};
        wall_col_emit<T, EPC, 3>(g, ct, dsts, twm);
        return;
    }
    {
        const cpx<T>* srcs[2] = {Hb, Hb + NS};
        wall_col_fft<T, EPC, 2>(g, ct, srcs, twm);
    }
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int e_ = 0; e_ <= EPC / 2; ++e_) {
        const int q = ct.t + g.TPC * e_;
        if (q > g.ny / 2) continue;
        const int m = (g.ny - q) & (g.ny - 1);
        const bool self = q == m;
        const cpx<T> wy = twy[q];
        cpx<T> a[2][2];
#pragma unroll
        for (int f = 0; f < 2; ++f)
            wall_to_slots<T>(ct.buf[f * ct.fstride + q], ct.buf[f * ct.fstride + m], wc.wx, wy, wc.k0, q == 0,
                             wall_xs(f), wall_ys(f), a[f][0], a[f][1]);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (!ct.valid || (s == 1 && self)) continue;
            const int ysl = s ? m : q;
            const double cy = ysl == 0 ? 1.0 : 2.0;
            const T ky = (T)ysl * piy;
            const cpx<T> r0 = a[0][s], r1 = a[1][s];
            if (bh) {
                bh[col + ysl] = r0;
                bh[NS + col + ysl] = r1;
            }
            rh[col + ysl] = r0;
            rh[NS + col + ysl] = r1;
            if (!GUESS) {
                xh[col + ysl] = C<T>(0, 0);
                xh[NS + col + ysl] = C<T>(0, 0);
            }
            const double wre = wc.cre * cy, wim = wc.cim * cy;
            const double rr = wre * ((double)r0.re * r0.re + (double)r1.re * r1.re) +
                              wim * ((double)r0.im * r0.im + (double)r1.im * r1.im);
            if (GUESS) {
                acc[0] += rr;
            } else {
                T z0r, z1r, z0i, z1i;
                wall_precond<T>(wc.kre, ky, sig, alp, r0.re, r1.re, z0r, z1r);
                wall_precond<T>(wc.kim, ky, sig, alp, r0.im, r1.im, z0i, z1i);
                acc[0] += wre * ((double)r0.re * z0r + (double)r1.re * z1r) +
                          wim * ((double)r0.im * z0i + (double)r1.im * z1i);
                acc[1] += rr;
            }
        }
    }
    if (GUESS) {
        double bsum[1] = {acc[0]};
        block_sum<1>(bsum, red);
        if (threadIdx.x == 0) part[PART_GEN + blockIdx.x] = bsum[0];
    } else {
        block_sum<2>(acc, red);
        if (threadIdx.x == 0) {
            part[PART_C3 + 2 * blockIdx.x] = acc[0];
            part[PART_C3 + 2 * blockIdx.x + 1] = acc[1];
        }
    }
}

// Column pass C1 of a wall solve (k_pcg_c1, mode C1_UPDATE): stop test and beta
// from the last update's partials; z = A^{-1} r, p = z + beta p on the slots;
// (p, div p) / (nx ny) -> column values -> inverse y-FFT into H.
template <typename T, int EPC>
__global__ void __launch_bounds__(256) k_wall_c1(ColGeom g, const cpx<T>* __restrict__ tw, SolveScal* __restrict__ sc,
                                                  const double* __restrict__ part, int nb3,
                                                  const cpx<T>* __restrict__ rh, cpx<T>* __restrict__ ph,
                                                  cpx<T>* __restrict__ H, size_t NS, T pix, T piy) {
    if (sc->done) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    __shared__ double red[32];
    __shared__ double slot[2];
    double beta_d = 0.0;
    if (pcg_iterate_state(sc, part, nb3, red, slot, beta_d)) return;
    const cpx<T>* twm = twl_setup<T>(tw, g.ny, lds + col_lds_data(g, 3));
    const ColThread<T> ct = col_thread<T>(g, lds);
    const WallColumn<T> wc = wall_column<T>(g, ct, tw, pix);
    const cpx<T>* twy = tw_size(tw, 4 * g.ny);
    const T beta = (T)beta_d, sig = (T)sc->sig, alp = (T)sc->alp, inv_n = (T)sc->inv_n;
    const size_t col = (size_t)ct.kx * g.ny;
#pragma unroll
    for (int e_ = 0; e_ <= EPC / 2; ++e_) {
        const int q = ct.t + g.TPC * e_;
        if (q > g.ny / 2) continue;
        const int m = (g.ny - q) & (g.ny - 1);
        const bool self = q == m;
        const cpx<T> wy = twy[q];
        cpx<T> o[3][2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int ysl = s ? m : q;
            const T ky = (T)ysl * piy;
            cpx<T> p0 = C<T>(0, 0), p1 = C<T>(0, 0);
            if (ct.valid && (s == 0 || !self)) {
                const cpx<T> r0 = rh[col + ysl], r1 = rh[NS + col + ysl];
                T z0r, z1r, z0i, z1i;
                wall_precond<T>(wc.kre, ky, sig, alp, r0.re, r1.re, z0r, z1r);
                wall_precond<T>(wc.kim, ky, sig, alp, r0.im, r1.im, z0i, z1i);
                p0 = C<T>(z0r, z0i);
                p1 = C<T>(z1r, z1i);
                // beta = 0 on the first iteration: p = z without reading the unset direction
                if (beta != (T)0) {
                    p0 = p0 + beta * ph[col + ysl];
                    p1 = p1 + beta * ph[NS + col + ysl];
                }
                ph[col + ysl] = p0;
                ph[NS + col + ysl] = p1;
            }
            o[0][s] = inv_n * p0;
            o[1][s] = inv_n * p1;
            o[2][s] = inv_n * C<T>(wc.kre * p0.re + ky * p1.re, wc.kim * p0.im + ky * p1.im);
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            cpx<T> F1, F2;
            wall_from_slots<T>(o[f][0], self ? o[f][0] : o[f][1], wc.wx, wy, wc.k0, q == 0, wall_xs(f), wall_ys(f),
                               F1, F2);
            ct.buf[f * ct.fstride + q] = F1;
            if (!self) ct.buf[f * ct.fstride + m] = F2;
        }
    }
    cpx<T>* dsts[3] = {H, H + NS, H + 2 * NS};
    wall_col_emit<T, EPC, 3>(g, ct, dsts, twm);
}

// Column pass C2 of a wall solve (k_pcg_c2): y-FFT of the row pass's (a_u, a_v, w)
// -> slots; q = a - grad w, i.e. a + kappa w on every slot (= G p, Def:G).
// MODE C2_UPDATE: alpha from p.Gp; x += alpha p, r -= alpha q, z = A^{-1} r,
// partial r.z, r.r.  MODE C2_RESID_INIT: bb from the setup partials;
// r = b - G x_0 (zero for a zero b), partial r.z, r.r.
template <typename T, int EPC, int MODE>
__global__ void __launch_bounds__(256) k_wall_c2(ColGeom g, const cpx<T>* __restrict__ tw, SolveScal* __restrict__ sc,
                                                  const cpx<T>* __restrict__ H, size_t NS,
                                                  const cpx<T>* __restrict__ ph, cpx<T>* __restrict__ xh,
                                                  const cpx<T>* bh, cpx<T>* rh, double* __restrict__ part,
                                                  int nb_red, T pix, T piy) {
    static_assert(MODE == C2_UPDATE || MODE == C2_RESID_INIT, "wall column pass mode");
    if (sc->done) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    __shared__ double red[32];
    __shared__ double slot[1];
    T alpha = (T)0;
    bool zero_x = false;
    if (MODE == C2_RESID_INIT) {
        double tot[1];
        final_sum<1>(part + PART_GEN, nb_red, tot, red);
        const double bb = bcast(tot[0], slot) * sc->inv_n;
        const bool bad = !(bb == bb) || bb > 1.0e300;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->bb = bb;
            if (bad) {
                sc->status = -2;
                sc->done = 1;
            }
        }
        if (bad) return;
        zero_x = !sc->init_bb && bb == 0.0;
    } else {
        double tot[1];
        final_sum<1>(part + PART_C2, nb_red, tot, red);
        const double pq = bcast(tot[0], slot);
        const double a = sc->rho / pq;
        alpha = (T)a;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->pq = pq;
            sc->alpha = a;
            sc->rho_prev = sc->rho;
            sc->iter = sc->iter + 1;
            sc->first = 0;
        }
    }
    const cpx<T>* twm = twl_setup<T>(tw, g.ny, lds + col_lds_data(g, 3));
    const ColThread<T> ct = col_thread<T>(g, lds);
    const WallColumn<T> wc = wall_column<T>(g, ct, tw, pix);
    const cpx<T>* twy = tw_size(tw, 4 * g.ny);
    const T sig = (T)sc->sig, alp = (T)sc->alp;
    const size_t col = (size_t)ct.kx * g.ny;
    {
        const cpx<T>* srcs[3] = {H, H + NS, H + 2 * NS};
        wall_col_fft<T, EPC, 3>(g, ct, srcs, twm);
    }
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int e_ = 0; e_ <= EPC / 2; ++e_) {
        const int q = ct.t + g.TPC * e_;
        if (q > g.ny / 2) continue;
        const int m = (g.ny - q) & (g.ny - 1);
        const bool self = q == m;
        const cpx<T> wy = twy[q];
        cpx<T> a[3][2];
#pragma unroll
        for (int f = 0; f < 3; ++f)
            wall_to_slots<T>(ct.buf[f * ct.fstride + q], ct.buf[f * ct.fstride + m], wc.wx, wy, wc.k0, q == 0,
                             wall_xs(f), wall_ys(f), a[f][0], a[f][1]);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (!ct.valid || (s == 1 && self)) continue;
            const int ysl = s ? m : q;
            const double cy = ysl == 0 ? 1.0 : 2.0;
            const T ky = (T)ysl * piy;
            const cpx<T> wv = a[2][s];
            const cpx<T> q0 = C<T>(a[0][s].re + wc.kre * wv.re, a[0][s].im + wc.kim * wv.im);
            const cpx<T> q1 = C<T>(a[1][s].re + ky * wv.re, a[1][s].im + ky * wv.im);
            cpx<T> r0, r1;
            if (MODE == C2_RESID_INIT) {
                r0 = zero_x ? C<T>(0, 0) : bh[col + ysl] - q0;
                r1 = zero_x ? C<T>(0, 0) : bh[NS + col + ysl] - q1;
                if (zero_x) {
                    xh[col + ysl] = C<T>(0, 0);
                    xh[NS + col + ysl] = C<T>(0, 0);
                }
            } else {
                xh[col + ysl] = xh[col + ysl] + alpha * ph[col + ysl];
                xh[NS + col + ysl] = xh[NS + col + ysl] + alpha * ph[NS + col + ysl];
                r0 = rh[col + ysl] - alpha * q0;
                r1 = rh[NS + col + ysl] - alpha * q1;
            }
            rh[col + ysl] = r0;
            rh[NS + col + ysl] = r1;
            T z0r, z1r, z0i, z1i;
            wall_precond<T>(wc.kre, ky, sig, alp, r0.re, r1.re, z0r, z1r);
            wall_precond<T>(wc.kim, ky, sig, alp, r0.im, r1.im, z0i, z1i);
            const double wre = wc.cre * cy, wim = wc.cim * cy;
            acc[0] += wre * ((double)r0.re * z0r + (double)r1.re * z1r) +
                      wim * ((double)r0.im * z0i + (double)r1.im * z1i);
            acc[1] += wre * ((double)r0.re * r0.re + (double)r1.re * r1.re) +
                      wim * ((double)r0.im * r0.im + (double)r1.im * r1.im);
        }
    }
    block_sum<2>(acc, red);
    if (threadIdx.x == 0) {
        part[PART_C3 + 2 * blockIdx.x] = acc[0];
        part[PART_C3 + 2 * blockIdx.x + 1] = acc[1];
    }
}

// The two velocity fields' slots S (times scale) -> column values -> inverse
// y-FFT into H (the last column pass of a wall solve, before the inverse row
// transforms and the return to grid order).
template <typename T, int EPC>
__global__ void __launch_bounds__(256) k_wall_from_S(ColGeom g, const cpx<T>* __restrict__ tw,
                                                      const cpx<T>* __restrict__ S, size_t NS, cpx<T>* __restrict__ H,
                                                      T scale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    const cpx<T>* twm = twl_setup<T>(tw, g.ny, lds + col_lds_data(g, 2));
    const ColThread<T> ct = col_thread<T>(g, lds);
    const WallColumn<T> wc = wall_column<T>(g, ct, tw, (T)0);
    const cpx<T>* twy = tw_size(tw, 4 * g.ny);
    const size_t col = (size_t)ct.kx * g.ny;
#pragma unroll
    for (int e_ = 0; e_ <= EPC / 2; ++e_) {
        const int q = ct.t + g.TPC * e_;
        if (q > g.ny / 2) continue;
        const int m = (g.ny - q) & (g.ny - 1);
        const bool self = q == m;
        const cpx<T> wy = twy[q];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            cpx<T> sq = C<T>(0, 0), sm = C<T>(0, 0);
            if (ct.valid) {
                sq = scale * S[f * NS + col + q];
                sm = self ? sq : scale * S[f * NS + col + m];
            }
            cpx<T> F1, F2;
            wall_from_slots<T>(sq, sm, wc.wx, wy, wc.k0, q == 0, wall_xs(f), wall_ys(f), F1, F2);
            ct.buf[f * ct.fstride + q] = F1;
            if (!self) ct.buf[f * ct.fstride + m] = F2;
        }
    }
    cpx<T>* dsts[2] = {H, H + NS};
    wall_col_emit<T, EPC, 2>(g, ct, dsts, twm);
}

// Coefficient of derivative code c (1 identity, 2 d/dx, 3 d/dy, 4 d2/dx2,
// 5 d2/dxdy, 6 d2/dy2) on the slot of wavenumbers (kx, ky), for an input of
// series kind `kind` (bit 0: sine along x, bit 1: sine along y): d/dx takes a
// cosine amplitude to the sine one times -kx and a sine amplitude to the cosine
// one times +kx; a second derivative along one axis is -k^2 either way.
template <typename T>
__device__ __forceinline__ T wall_coef(int code, T kx, T ky, int kind) {
    const T dx = (kind & 1) ? kx : -kx;
    const T dy = (kind & 2) ? ky : -ky;
    switch (code) {
        case 1: return (T)1;
        case 2: return dx;
        case 3: return dy;
        case 4: return -kx * kx;
        case 5: return dx * dy;
        case 6: return -ky * ky;
        default: return (T)0;
    }
}

// Linear column operators of a 2D wall grid (the k_cols_lin_jobs of the
// right-hand side): job jb of the launch takes blocks [jb nblocks, (jb + 1)
// nblocks); its ni inputs (H columns of fields in transform order, kinds kin)
// are y-transformed together in LDS, turned into slot amplitudes pair by pair,
// combined into the no outputs (kinds kout) with the slot coefficients, turned
// back and inverse-transformed together.  At most three inputs and three
// outputs per job (the LDS holds three columns per block column).
template <typename T, int EPC>
__global__ void __launch_bounds__(256) k_wall_cols_jobs(ColGeom g, LinJobs<T> jobs, const cpx<T>* __restrict__ tw,
                                                         T pix, T piy, T scale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    const int jb = blockIdx.x / g.nblocks;
    if (jb >= jobs.n) return;
    const LinJob<T>& J = jobs.j[jb];
    const cpx<T>* twm = twl_setup<T>(tw, g.ny, lds + col_lds_data(g, 3));
    const ColThread<T> ct = col_thread_at<T>(g, lds, (int)blockIdx.x - jb * g.nblocks);
    const WallColumn<T> wc = wall_column<T>(g, ct, tw, pix);
    const cpx<T>* twy = tw_size(tw, 4 * g.ny);
    const int ny = g.ny;
    {
        cpx<T> v[3][EPC];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                const int j = ct.t + g.TPC * e;
                v[i][e] = (i < J.ni && ct.valid && j < ny) ? J.src[i][(size_t)ct.kx * ny + j] : C<T>(0, 0);
            }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                const int j = ct.t + g.TPC * e;
                if (j < ny) ct.buf[i * ct.fstride + j] = v[i][e];
            }
    }
    __syncthreads();
    if (J.ni == 1)
        lds_fft<T, EPC, 1>(ct.buf, ct.fstride, ny, ct.t, g.TPC, twm, false);
    else if (J.ni == 2)
        lds_fft<T, EPC, 2>(ct.buf, ct.fstride, ny, ct.t, g.TPC, twm, false);
    else
        lds_fft<T, EPC, 3>(ct.buf, ct.fstride, ny, ct.t, g.TPC, twm, false);
#pragma unroll
    for (int e_ = 0; e_ <= EPC / 2; ++e_) {
        const int q = ct.t + g.TPC * e_;
        if (q > ny / 2) continue;
        const int m = (ny - q) & (ny - 1);
        const bool self = q == m;
        const cpx<T> wy = twy[q];
        cpx<T> a[3][2];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            a[i][0] = a[i][1] = C<T>(0, 0);
            if (i < J.ni)
                wall_to_slots<T>(ct.buf[i * ct.fstride + q], ct.buf[i * ct.fstride + m], wc.wx, wy, wc.k0, q == 0,
                                 (J.kin[i] & 1) != 0, (J.kin[i] & 2) != 0, a[i][0], a[i][1]);
        }
        cpx<T> o[3][2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const T ky = (T)(s ? m : q) * piy;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                T re = (T)0, im = (T)0;
                if (k < J.no) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        if (i >= J.ni) continue;
                        re += wall_coef<T>(J.code[k][i], wc.kre, ky, J.kin[i]) * a[i][s].re;
                        im += wall_coef<T>(J.code[k][i], wc.kim, ky, J.kin[i]) * a[i][s].im;
                    }
                }
                o[k][s] = C<T>(scale * re, scale * im);
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (k >= J.no) continue;
            cpx<T> F1, F2;
            wall_from_slots<T>(o[k][0], self ? o[k][0] : o[k][1], wc.wx, wy, wc.k0, q == 0, (J.kout[k] & 1) != 0,
                               (J.kout[k] & 2) != 0, F1, F2);
            ct.buf[k * ct.fstride + q] = F1;
            if (!self) ct.buf[k * ct.fstride + m] = F2;
        }
    }
    __syncthreads();
    if (J.no == 1)
        lds_fft<T, EPC, 1>(ct.buf, ct.fstride, ny, ct.t, g.TPC, twm, true);
    else if (J.no == 2)
        lds_fft<T, EPC, 2>(ct.buf, ct.fstride, ny, ct.t, g.TPC, twm, true);
    else
        lds_fft<T, EPC, 3>(ct.buf, ct.fstride, ny, ct.t, g.TPC, twm, true);
    if (ct.valid) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (k >= J.no) break;
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                const int j = ct.t + g.TPC * e;
                if (j < ny) J.dst[k][(size_t)ct.kx * ny + j] = ct.buf[k * ct.fstride + j];
            }
        }
    }
}

}  // namespace sgn
