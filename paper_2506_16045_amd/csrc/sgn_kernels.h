// Kernels of the SGN hot path.  Templated on the working precision T (double
// or float) and on the dimension D (1 or 2); reductions always accumulate in
// double.  Layouts: physical fields [ny][nx]; "H" and "S" spectral fields
// [kx][y] / [kx][ky] with kx = 0..nx/2 (see sgn_device.h).
#pragma once
#include "sgn_device.h"

namespace sgn {

// Device-side scalars of one Krylov solve (one instance per solve in flight).
// Protocol (no device-scope fences or atomics): a reducing kernel writes one
// partial sum per block; the next kernel in the stream reduces those partials
// in every block, in a fixed order, and block 0 publishes the scalars.
struct SolveScal {
    double rho;        // r.z of the current search direction
    double rho_prev;   // r.z used by the last x, r update
    double alpha, beta, bb, rr, pq, tol2, relres;
    double sig, alp, kap;     // preconditioner A = sig I - alp grad div, bound kappa_ub
    double inv_n;             // 1 / (nx ny)
    double red[8];            // results of the last generic reduction
    int iter, max_iter, done, converged, flat, status;
    int first;                // 1 until the first update (beta = 0)
    int init_bb;              // 1: ||b|| is the norm of the initial residual
    int outer;                // refinement steps taken (mixed precision)
};

constexpr int PARTIALS_MAX = 4096;  // blocks of a reducing launch (256 PF_K)
static_assert(PARTIALS_MAX <= 256 * PF_K, "prefetched partials cover every reducing launch");
// regions of the partials buffer (doubles)
constexpr int PART_C2 = 0;                       // p.Gp of the row pass (one per row block)
constexpr int PART_C3 = 4096;                    // (r.z, r.r) of the update pass (two per column block)
constexpr int PART_GEN = 4096 + 2 * 4096;        // one-off reductions (up to 5 per block)
constexpr int PART_TOTAL = PART_GEN + 5 * PARTIALS_MAX;

template <typename T, int N>
struct PtrList {
    T* p[N];
    int n;
};
constexpr int MAXF = 12;

// Mode weight of the half spectrum for Parseval sums: kx = 0 and kx = nx/2 appear
// once in the full spectrum, every other kx twice (with its conjugate).
__device__ __forceinline__ double half_weight(int kx, int nx) {
    return (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
}

// z = A^{-1} r in Fourier space (Def:A, section 6.1): the symbol of A is
//   1D: sig + alp k^2;   2D: sig I + alp k k^T.
// In 2D the inverse splits r into its parts along k and across k,
//   z = r_perp / sig + r_par / (sig + alp |k|^2),  r_par = k (k.r) / |k|^2,
// which keeps full relative accuracy in both parts (the equivalent
// Sherman-Morrison form r/sig - alp k (k.r)/(sig (sig + alp |k|^2)) cancels
// digits along k when alp |k|^2 >> sig).
template <typename T, int D>
__device__ __forceinline__ void precond_mode(T kx, T ky, T sig, T alp, const cpx<T> (&r)[D],
                                             cpx<T> (&z)[D]) {
    if (D == 1) {
        const T s = (T)1 / (sig + alp * kx * kx);
        z[0] = s * r[0];
    } else {
        const T k2 = kx * kx + ky * ky;
        const T is = (T)1 / sig;
        if (k2 == (T)0) {
            z[0] = is * r[0];
            z[1 % D] = is * r[1 % D];
        } else {
            const cpx<T> kr = ((T)1 / k2) * (kx * r[0] + ky * r[1 % D]);   // (k.r) / |k|^2
            const cpx<T> px = kx * kr, py = ky * kr;                       // r_par
            const T ip = (T)1 / (sig + alp * k2);
            z[0] = is * (r[0] - px) + ip * px;
            z[1 % D] = is * (r[1 % D] - py) + ip * py;
        }
    }
}

// ---------------------------------------------------------------------------
// Generic FFT passes
// ---------------------------------------------------------------------------

// Fields f >= first of a forward row pass are read as src + (c1 a + c2 b): an
// extrapolated initial guess formed from its base and two recorded offsets as
// it is loaded (b may be null; first < 0: no field is combined).
template <typename Tin>
struct RowCombo {
    const Tin* a[4];
    const Tin* b[4];
    double c1, c2;
    int first;
};

// Forward row transforms of n physical fields (Tin = double or T) into H fields,
// NFG fields at a time in lockstep (the remainder one by one).
template <typename T, typename Tin, int EPC, int NFG>
__device__ __forceinline__ void rows_fwd_group(const RowGeom& g, const RowThread<T>& rt,
                                               const PtrList<const Tin, MAXF>& src, const PtrList<cpx<T>, MAXF>& dst,
                                               int f0, const cpx<T>* __restrict__ tw, const cpx<T>* twm, T scale,
                                               const RowCombo<Tin>& cmb) {
    cpx<T> z[NFG][EPC];
    cpx<T>* H[NFG];
#pragma unroll
    for (int f = 0; f < NFG; ++f) {
        H[f] = dst.p[f0 + f];
        const int k = f0 + f - cmb.first;
        const bool comb = cmb.first >= 0 && k >= 0;
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = rt.t + g.TPR * e;
            z[f][e] = C<T>(0, 0);
            if (j < g.M && rt.valid) {
                const size_t o = (size_t)rt.y * g.nx + 2 * j;
                if (comb) {
                    double v[2];
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        double t = cmb.c1 * (double)cmb.a[k][o + s];
                        if (cmb.b[k]) t += cmb.c2 * (double)cmb.b[k][o + s];
                        v[s] = (double)src.p[f0 + f][o + s] + t;
                    }
                    z[f][e] = C<T>((T)v[0], (T)v[1]);
                } else {
                    z[f][e] = C<T>((T)src.p[f0 + f][o], (T)src.p[f0 + f][o + 1]);
                }
            }
        }
    }
    row_forward<T, EPC, NFG>(g, rt, z, H, tw, twm, scale);
}

template <typename T, typename Tin, int EPC, int NFG, int MAXT = 1024>
__global__ void __launch_bounds__(MAXT) k_rows_fwd(RowGeom g, PtrList<const Tin, MAXF> src,
                                                   PtrList<cpx<T>, MAXF> dst,
                                                   const cpx<T>* __restrict__ tw, T scale, RowCombo<Tin> cmb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    const cpx<T>* twm = twl_setup<T>(tw, g.M, lds + row_lds_data(g, NFG));
    const RowThread<T> rt = row_thread<T>(g, lds);
    int f = 0;
    for (; f + NFG <= src.n; f += NFG) rows_fwd_group<T, Tin, EPC, NFG>(g, rt, src, dst, f, tw, twm, scale, cmb);
    for (; f < src.n; ++f) rows_fwd_group<T, Tin, EPC, 1>(g, rt, src, dst, f, tw, twm, scale, cmb);
}

// Inverse row transforms of n H fields into physical fields (Tout):
// dst = acc * dst + scale * value  (acc = 0 overwrites).  With offs.n > 0,
// offs_f = new - old value of dst_f is written too (the offset of a solve's
// result from its base, recorded for the next extrapolated guess); with
// oacc != 0 it is added to offs_f instead (a result stored a second time).
template <typename T, typename Tout, int EPC, int NFG>
__device__ __forceinline__ void rows_inv_group(const RowGeom& g, const RowThread<T>& rt,
                                               const PtrList<const cpx<T>, MAXF>& src, const PtrList<Tout, MAXF>& dst,
                                               int f0, const cpx<T>* __restrict__ tw, const cpx<T>* twm, T scale,
                                               T acc, const PtrList<Tout, MAXF>& offs, int oacc) {
    cpx<T> z[NFG][EPC];
    const cpx<T>* H[NFG];
#pragma unroll
    for (int f = 0; f < NFG; ++f) H[f] = src.p[f0 + f];
    row_inverse<T, EPC, NFG>(g, rt, H, tw, twm, z);
#pragma unroll
    for (int f = 0; f < NFG; ++f) {
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = rt.t + g.TPR * e;
            if (j < g.M && rt.valid) {
                const size_t o = (size_t)rt.y * g.nx + 2 * j;
                Tout* d = dst.p[f0 + f];
                T v0 = scale * z[f][e].re, v1 = scale * z[f][e].im;
                if (acc != (T)0) {
                    v0 += acc * (T)d[o];
                    v1 += acc * (T)d[o + 1];
                }
                if (offs.n > 0) {
                    Tout* od = offs.p[f0 + f];
                    const Tout d0 = (Tout)v0 - d[o], d1 = (Tout)v1 - d[o + 1];
                    od[o] = oacc ? od[o] + d0 : d0;
                    od[o + 1] = oacc ? od[o + 1] + d1 : d1;
                }
                d[o] = (Tout)v0;
                d[o + 1] = (Tout)v1;
            }
        }
    }
}

template <typename T, typename Tout, int EPC, int NFG, int MAXT = 1024>
__global__ void __launch_bounds__(MAXT) k_rows_inv(RowGeom g, PtrList<const cpx<T>, MAXF> src,
                                                   PtrList<Tout, MAXF> dst,
                                                   const cpx<T>* __restrict__ tw, T scale, T acc,
                                                   PtrList<Tout, MAXF> offs, int oacc) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    const cpx<T>* twm = twl_setup<T>(tw, g.M, lds + row_lds_data(g, NFG));
    const RowThread<T> rt = row_thread<T>(g, lds);
    int f = 0;
    for (; f + NFG <= src.n; f += NFG)
        rows_inv_group<T, Tout, EPC, NFG>(g, rt, src, dst, f, tw, twm, scale, acc, offs, oacc);
    for (; f < src.n; ++f) rows_inv_group<T, Tout, EPC, 1>(g, rt, src, dst, f, tw, twm, scale, acc, offs, oacc);
}

// ---------------------------------------------------------------------------
// Right-hand side row passes (Eq:DSWEcf, Def:bigF, Eq:DAE_DSWE), fused with
// their pointwise stages.
// ---------------------------------------------------------------------------

// Source field i of the right-hand side's forward transforms at one point:
// [u_c (D), eta u_c (D), eta, -eta u_1 u_D, beta = grad h . u].  The momentum
// flux enters negated: its divergence is later summed with grad S in the
// spectral domain, so both reach U_t through one pair of inverse transforms.
// In 2D only the mixed flux -eta u_x u_y is transformed here: the diagonal
// terms reach U_t only through d_x (eta u_x^2) and d_y (eta u_y^2), so the
// inverse pass folds them into S_x = S - eta u_x^2 and S_y = S - eta u_y^2, and
// (U_t)_x gains d_x S_x - d_y (eta u_x u_y), (U_t)_y gains d_y S_y - d_x (eta u_x u_y).
template <int D>
__device__ __forceinline__ double rhs_source(int i, double e, const double (&uc)[D], const double (&hc)[D]) {
    if (i < D) return uc[i];
    if (i < 2 * D) return e * uc[i - D];
    if (i == 2 * D) return e;
    if (i == 2 * D + 1) return -(e * uc[0] * uc[D - 1]);
    double b = hc[0] * uc[0];
    if (D == 2) b += hc[1 % D] * uc[1 % D];
    return b;
}

// Products and forward row transforms of the right-hand side's source fields
// (rhs_source order) in groups of NFG fields; dst.p[i] receives field i.  Each
// block does every group in turn (running the groups side by side in separate
// blocks was measured slower: every group then reloads its inputs).  With
// 256-thread blocks eta, u and beta = grad h . u are read once per point into
// registers before the first group, so each input crosses HBM once; larger
// blocks, whose register budget is smaller, read them again for every group.
// MAXT bounds the workgroup size (256 lets the compiler use more registers).
template <int D, int EPC, int NFG, int MAXT>
__global__ void __launch_bounds__(MAXT) k_rhs_rows_fwd(RowGeom g, const double* __restrict__ eta,
                                                       const double* __restrict__ u, const double* __restrict__ gh,
                                                       PtrList<cpx<double>, MAXF> dst,
                                                       const cpx<double>* __restrict__ tw) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<double>* lds = reinterpret_cast<cpx<double>*>(smem_raw);
    const cpx<double>* twm = twl_setup<double>(tw, g.M, lds + row_lds_data(g, NFG));
    const RowThread<double> rt = row_thread<double>(g, lds);
    const size_t npts = (size_t)g.nx * g.ny;
    constexpr int NFLD = 2 * D + 3;
    // the inputs of this thread's points: eta, u_c and beta (the last field)
    constexpr bool KEEP = MAXT <= 256;
    constexpr int EK = KEEP ? EPC : 1;
    double ie[EK][2], iu[D][EK][2], ib[EK][2];
    auto load = [&](int e, int s, double& et, double (&uc)[D], double (&hc)[D]) {
        const int j = rt.t + g.TPR * e;
        const bool ok = j < g.M && rt.valid;
        const size_t o = ok ? (size_t)rt.y * g.nx + 2 * j : 0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            uc[c] = ok ? u[c * npts + o + s] : 0.0;
            hc[c] = ok ? gh[c * npts + o + s] : 0.0;
        }
        et = ok ? eta[o + s] : 0.0;
    };
    if (KEEP) {
#pragma unroll
        for (int e = 0; e < EK; ++e) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                double uc[D], hc[D];
                load(e, s, ie[e][s], uc, hc);
#pragma unroll
                for (int c = 0; c < D; ++c) iu[c][e][s] = uc[c];
                ib[e][s] = rhs_source<D>(NFLD - 1, ie[e][s], uc, hc);
            }
        }
    }
#pragma unroll
    for (int f0 = 0; f0 < NFLD; f0 += NFG) {
        cpx<double> z[NFG][EPC];
        cpx<double>* H[NFG];
#pragma unroll
        for (int k = 0; k < NFG; ++k) H[k] = (f0 + k < NFLD) ? dst.p[f0 + k] : dst.p[f0];
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = rt.t + g.TPR * e;
#pragma unroll
            for (int k = 0; k < NFG; ++k) z[k][e] = C<double>(0, 0);
            if (j < g.M && rt.valid) {
                double v[NFG][2];
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    double et, uc[D], hc[D];
                    if (KEEP) {
                        const int ek = KEEP ? e : 0;
                        et = ie[ek][s];
#pragma unroll
                        for (int c = 0; c < D; ++c) {
                            uc[c] = iu[c][ek][s];
                            hc[c] = 0.0;
                        }
                    } else {
                        load(e, s, et, uc, hc);
                    }
#pragma unroll
                    for (int k = 0; k < NFG; ++k)
                        v[k][s] = KEEP && f0 + k == NFLD - 1 ? ib[KEEP ? e : 0][s] : rhs_source<D>(f0 + k, et, uc, hc);
                }
#pragma unroll
                for (int k = 0; k < NFG; ++k) z[k][e] = C<double>(v[k][0], v[k][1]);
            }
        }
        if (f0 + NFG <= NFLD) {
            row_forward<double, EPC, NFG>(g, rt, z, H, tw, twm, 1.0);
        } else {
            // the last group holds fewer fields: transform them one by one
            for (int k = 0; f0 + k < NFLD; ++k) {
                cpx<double> z1[1][EPC];
                cpx<double>* H1[1] = {H[k]};
#pragma unroll
                for (int e = 0; e < EPC; ++e) z1[0][e] = z[k][e];
                row_forward<double, EPC, 1>(g, rt, z1, H1, tw, twm, 1.0);
            }
        }
    }
}

// Inverse row transforms of the derivative fields Q, in the order m =
// div(eta u), delta = div u, d_c delta, d_c eta, d_c beta, in groups of NFG,
// consumed into the pointwise right-hand side as they arrive: eta_t = -m,
// U_t = -eta grad(eta - h) - T grad h (grad S - div(eta u (x) u) is added later),
// and S, T of Def:bigF accumulated as S = e^3/3 P + e^2 m delta + e m beta +
// e^2/2 Q, T = e^2/2 P + e m delta + m beta + e Q with P = u.grad(delta) -
// delta^2 and Q = u.grad(beta) (the reading u.grad(u.grad h)), so that at most
// four values per point are live.  S's forward row transform goes to Sdst
// (grad S is added to U_t later); in 2D S_x = S - eta u_x^2 goes to Sdst and
// S_y = S - eta u_y^2 to Sydst (see rhs_source).
template <int D, int EPC, int NFG, int MAXT>
__global__ void __launch_bounds__(MAXT) k_rhs_rows_inv(RowGeom g, PtrList<const cpx<double>, MAXF> src,
                                                       const double* __restrict__ eta, const double* __restrict__ u,
                                                       const double* __restrict__ gh, double* __restrict__ eta_t,
                                                       double* __restrict__ U_t, cpx<double>* __restrict__ Sdst,
                                                       cpx<double>* __restrict__ Sydst,
                                                       const cpx<double>* __restrict__ tw, double scale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<double>* lds = reinterpret_cast<cpx<double>*>(smem_raw);
    const cpx<double>* twm = twl_setup<double>(tw, g.M, lds + row_lds_data(g, NFG));
    const RowThread<double> rt = row_thread<double>(g, lds);
    const size_t npts = (size_t)g.nx * g.ny;
    constexpr int NQ = 3 * D + 2;
    // live state per point: (m, delta, P) while the first 2 + D fields arrive,
    // then (S, T) and U_t (D)
    double A0[EPC][2], A1[EPC][2], A2[EPC][2], Ut[D][EPC][2];
    for (int f0 = 0; f0 < NQ; f0 += NFG) {
        const int nf = NQ - f0 < NFG ? NQ - f0 : NFG;
        cpx<double> z[NFG][EPC];
        if (nf == NFG) {
            const cpx<double>* Hs[NFG];
#pragma unroll
            for (int k = 0; k < NFG; ++k) Hs[k] = src.p[f0 + k];
            row_inverse<double, EPC, NFG>(g, rt, Hs, tw, twm, z);
        } else {
            for (int k = 0; k < nf; ++k) {
                const cpx<double>* H1[1] = {src.p[f0 + k]};
                cpx<double> z1[1][EPC];
                row_inverse<double, EPC, 1>(g, rt, H1, tw, twm, z1);
#pragma unroll
                for (int e = 0; e < EPC; ++e) z[k][e] = z1[0][e];
            }
        }
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = rt.t + g.TPR * e;
            if (j < g.M && rt.valid) {
                const size_t o = (size_t)rt.y * g.nx + 2 * j;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
#pragma unroll
                    for (int k = 0; k < NFG; ++k) {
                        const int i = f0 + k;
                        if (k >= nf) continue;
                        const double q = scale * (s ? z[k][e].im : z[k][e].re);
                        if (i == 0) {                       // m
                            A0[e][s] = q;
                            eta_t[o + s] = -q;
                        } else if (i == 1) {                // delta
                            A1[e][s] = q;
                            A2[e][s] = -q * q;
                        } else if (i <= 1 + D) {            // d_c delta: P += u_c d_c delta
                            const int c = i - 2;
                            A2[e][s] += u[c * npts + o + s] * q;
                            if (c == D - 1) {               // P complete: fold into S, T
                                const double e0 = eta[o + s];
                                double bt = 0.0;
#pragma unroll
                                for (int cc = 0; cc < D; ++cc) bt += gh[cc * npts + o + s] * u[cc * npts + o + s];
                                const double e2 = e0 * e0, mm = A0[e][s], d0 = A1[e][s], pp = A2[e][s];
                                A0[e][s] = e2 * e0 / 3.0 * pp + e2 * mm * d0 + e0 * mm * bt;   // S
                                A1[e][s] = e2 / 2.0 * pp + e0 * mm * d0 + mm * bt;            // T
                            }
                        } else if (i <= 1 + 2 * D) {        // d_c eta
                            const int c = i - 2 - D;
                            Ut[c][e][s] = -eta[o + s] * (q - gh[c * npts + o + s]);
                        } else {                            // d_c beta: Q += u_c d_c beta
                            const int c = i - 2 - 2 * D;
                            const double e0 = eta[o + s];
                            const double t = u[c * npts + o + s] * q;
                            A0[e][s] += e0 * e0 / 2.0 * t;
                            A1[e][s] += e0 * t;
                        }
                    }
                }
            }
        }
    }
    // U_t = U_t - T grad h; S (2D: S_x, S_y) forward-transformed
    cpx<double> zs[D][EPC];
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
        const int j = rt.t + g.TPR * e;
#pragma unroll
        for (int c = 0; c < D; ++c) zs[c][e] = C<double>(0, 0);
        if (j < g.M && rt.valid) {
            const size_t o = (size_t)rt.y * g.nx + 2 * j;
            double sc[D][2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    U_t[c * npts + o + s] = Ut[c][e][s] - gh[c * npts + o + s] * A1[e][s];
                    if (D == 2) {
                        const double uc = u[c * npts + o + s];
                        sc[c][s] = A0[e][s] - eta[o + s] * uc * uc;
                    } else {
                        sc[c][s] = A0[e][s];
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < D; ++c) zs[c][e] = C<double>(sc[c][0], sc[c][1]);
        }
    }
    // one field at a time: the launch's LDS holds NFG fields
#pragma unroll
    for (int c = 0; c < D; ++c) {
        cpx<double> z1[1][EPC];
#pragma unroll
        for (int e = 0; e < EPC; ++e) z1[0][e] = zs[c][e];
        cpx<double>* H1[1] = {c == 0 ? Sdst : Sydst};
        row_forward<double, EPC, 1>(g, rt, z1, H1, tw, twm, 1.0);
    }
}

// Linear spectral operators on columns: out_o = sum_i c(code[o][i], k) in_i, with
// y-FFT of the inputs and y-IFFT of the outputs.  Codes: 0 none, 1 identity,
// 2 i kx, 3 i ky, 4 (i kx)^2, 5 (i kx)(i ky), 6 (i ky)^2; every value is also
// multiplied by `scale`.
constexpr int LIN_MAXO = 6;
constexpr int LIN_MAXI = 5;
struct LinCodes {
    int code[LIN_MAXO][LIN_MAXI];
    int no;
};

template <typename T>
__device__ __forceinline__ cpx<T> lin_coef(int code, T kx, T ky) {
    switch (code) {
        case 1: return C<T>(1, 0);
        case 2: return C<T>(0, kx);
        case 3: return C<T>(0, ky);
        case 4: return C<T>(-kx * kx, 0);
        case 5: return C<T>(-kx * ky, 0);
        case 6: return C<T>(-ky * ky, 0);
        default: return C<T>(0, 0);
    }
}

// Inputs loaded (and y-transformed) G fields at a time in lockstep; outputs
// formed and inverse-transformed G at a time.
template <typename T, int EPC, int G>
__device__ __forceinline__ void cols_lin_load(const ColGeom& g, const ColThread<T>& ct,
                                              const PtrList<const cpx<T>, MAXF>& src, int i0,
                                              const cpx<T>* twm, cpx<T> (&vi)[G][EPC]) {
    const cpx<T>* srcs[G];
#pragma unroll
    for (int k = 0; k < G; ++k) srcs[k] = src.p[i0 + k];
    col_load<T, EPC, G>(g, ct, srcs, true, twm, vi);
}

template <typename T, int EPC, int G, int NI>
__device__ __forceinline__ void cols_lin_store(const ColGeom& g, const ColThread<T>& ct,
                                               const PtrList<cpx<T>, MAXF>& dst, const LinCodes& lc, int o0,
                                               const cpx<T> (&in)[NI][EPC], T kx, T tpy, T scale,
                                               const cpx<T>* twm) {
    cpx<T> v[G][EPC];
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
        const int j = ct.t + g.TPC * e;
        const T ky = (g.ny > 1) ? wavenumber<T>(j, g.ny, tpy) : (T)0;
#pragma unroll
        for (int k = 0; k < G; ++k) {
            cpx<T> s = C<T>(0, 0);
#pragma unroll
            for (int i = 0; i < NI; ++i) s = s + lin_coef<T>(lc.code[o0 + k][i], kx, ky) * in[i][e];
            v[k][e] = scale * s;
        }
    }
    cpx<T>* dsts[G];
#pragma unroll
    for (int k = 0; k < G; ++k) dsts[k] = dst.p[o0 + k];
    col_store<T, EPC, G>(g, ct, v, dsts, true, twm);
}

template <typename T, int EPC, int NI, int G>
__global__ void __launch_bounds__(256) k_cols_lin(ColGeom g, PtrList<const cpx<T>, MAXF> src,
                                                   PtrList<cpx<T>, MAXF> dst, LinCodes lc,
                                                   const cpx<T>* __restrict__ tw, T tpx, T tpy,
                                                   T scale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    const cpx<T>* twm = twl_setup<T>(tw, g.ny, lds + col_lds_data(g, G));
    const ColThread<T> ct = col_thread<T>(g, lds);
    cpx<T> in[NI][EPC];
#pragma unroll
    for (int i0 = 0; i0 < NI; i0 += G) {
        if (i0 + G <= NI) {
            cpx<T> vi[G][EPC];
            cols_lin_load<T, EPC, G>(g, ct, src, i0, twm, vi);
#pragma unroll
            for (int k = 0; k < G; ++k)
#pragma unroll
                for (int e = 0; e < EPC; ++e) in[(i0 + k) % NI][e] = vi[k][e];
        } else {
#pragma unroll
            for (int i = i0; i < NI; ++i) {
                cpx<T> vi[1][EPC];
                cols_lin_load<T, EPC, 1>(g, ct, src, i, twm, vi);
#pragma unroll
                for (int e = 0; e < EPC; ++e) in[i][e] = vi[0][e];
            }
        }
    }
    const T kx = wavenumber<T>(ct.kx, g.nx, tpx);
    int o0 = 0;
    for (; o0 + G <= lc.no; o0 += G) cols_lin_store<T, EPC, G, NI>(g, ct, dst, lc, o0, in, kx, tpy, scale, twm);
    for (; o0 < lc.no; ++o0) cols_lin_store<T, EPC, 1, NI>(g, ct, dst, lc, o0, in, kx, tpy, scale, twm);
}

// Several independent linear column operators in one launch: job k takes
// blocks [k nblocks, (k+1) nblocks).  Each block first issues the loads of all
// its inputs (so their latencies overlap), then transforms them along y one by
// one, forms each output and inverse-transforms and stores it.  The jobs of the
// 2D right-hand side run side by side this way instead of in four launches,
// which keeps four times as many columns in flight.
constexpr int LINJ_MAXI = 4;
constexpr int LINJ_MAXO = 3;
constexpr int LINJ_MAXJ = 4;
template <typename T>
struct LinJob {
    const cpx<T>* src[LINJ_MAXI];
    cpx<T>* dst[LINJ_MAXO];
    int ni, no;
    int code[LINJ_MAXO][LINJ_MAXI];
    int kin[LINJ_MAXI], kout[LINJ_MAXO];   // series kinds of a wall job (bit 0: sine along x, bit 1: along y)
};
template <typename T>
struct LinJobs {
    LinJob<T> j[LINJ_MAXJ];
    int n;
};

template <typename T, int EPC>
__device__ __forceinline__ void col_fft_regs(const ColGeom& g, const ColThread<T>& ct, const cpx<T>* twm,
                                             cpx<T> (&v)[EPC], bool inverse) {
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
        const int j = ct.t + g.TPC * e;
        if (j < g.ny) ct.buf[j] = v[e];
    }
    __syncthreads();
    lds_fft<T, EPC, 1, col_swz<T>()>(ct.buf, ct.fstride, g.ny, ct.t, g.TPC, twm, inverse);
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
        const int j = ct.t + g.TPC * e;
        if (j < g.ny) v[e] = ct.buf[j];
    }
    __syncthreads();
}

// NF register columns of a block through one y-FFT in lockstep (shared barriers):
// fields f < nf of v go to LDS (field stride ct.fstride), are transformed and
// read back.
template <typename T, int EPC, int NF>
__device__ __forceinline__ void col_fft_group(const ColGeom& g, const ColThread<T>& ct, const cpx<T>* twm,
                                              cpx<T> (*v)[EPC], bool inverse) {
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = ct.t + g.TPC * e;
            if (j < g.ny) ct.buf[f * ct.fstride + j] = v[f][e];
        }
    __syncthreads();
    lds_fft<T, EPC, NF, col_swz<T>()>(ct.buf, ct.fstride, g.ny, ct.t, g.TPC, twm, inverse);
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = ct.t + g.TPC * e;
            if (j < g.ny) v[f][e] = ct.buf[f * ct.fstride + j];
        }
    __syncthreads();
}

// The first nf (1..3) register columns of v through one lockstep y-FFT.
template <typename T, int EPC, int NMAX>
__device__ __forceinline__ void col_fft_first(const ColGeom& g, const ColThread<T>& ct, const cpx<T>* twm,
                                              cpx<T> (&v)[NMAX][EPC], int nf, bool inverse) {
    if (nf == 1) col_fft_group<T, EPC, 1>(g, ct, twm, v, inverse);
    else if (nf == 2 || NMAX < 3) col_fft_group<T, EPC, (NMAX < 2 ? NMAX : 2)>(g, ct, twm, v, inverse);
    else col_fft_group<T, EPC, (NMAX < 3 ? NMAX : 3)>(g, ct, twm, v, inverse);
}

// LK: columns per lockstep transform, 3 (LDS holds three columns per block) or 1
// (one at a time, for columns of 2048 where three would leave one block per CU).
template <typename T, int EPC, int NI, int LK>
__global__ void __launch_bounds__(256) k_cols_lin_jobs(ColGeom g, LinJobs<T> jobs, const cpx<T>* __restrict__ tw,
                                                        T tpx, T tpy, T scale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    const int jb = blockIdx.x / g.nblocks;
    if (jb >= jobs.n) return;
    const LinJob<T>& J = jobs.j[jb];
    constexpr int NL = LK == 1 ? 1 : (NI < 3 ? NI : 3);
    const cpx<T>* twm = twl_setup<T>(tw, g.ny, lds + col_lds_data(g, NL));
    ColThread<T> ct;
    ct.c = threadIdx.x / g.TPC;
    ct.t = threadIdx.x - ct.c * g.TPC;
    ct.kx = (blockIdx.x - jb * g.nblocks) * g.Cb + ct.c;
    ct.valid = ct.kx < g.nxh;
    ct.buf = lds + ct.c * g.ny;
    ct.fstride = g.Cb * g.ny;
    const int ny = g.ny;
    cpx<T> in[NI][EPC];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = ct.t + g.TPC * e;
            in[i][e] = (i < J.ni && ct.valid && j < ny) ? J.src[i][(size_t)ct.kx * ny + j] : C<T>(0, 0);
        }
    }
    if (ny > 1 && LK == 1) {
#pragma unroll
        for (int i = 0; i < NI; ++i)
            if (i < J.ni) col_fft_group<T, EPC, 1>(g, ct, twm, in + i, false);
    } else if (ny > 1) {
        // the inputs in groups of up to three sharing their transform's barriers
        if (NI <= 3 || J.ni <= 3) {
            col_fft_first<T, EPC, NI>(g, ct, twm, in, J.ni, false);
        } else {
            col_fft_first<T, EPC, NI>(g, ct, twm, in, 3, false);
            col_fft_group<T, EPC, 1>(g, ct, twm, in + 3, false);
        }
    }
    const T kx = wavenumber<T>(ct.kx, g.nx, tpx);
    cpx<T> out[LINJ_MAXO][EPC];
#pragma unroll
    for (int o = 0; o < LINJ_MAXO; ++o) {
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = ct.t + g.TPC * e;
            const T ky = (ny > 1) ? wavenumber<T>(j, ny, tpy) : (T)0;
            cpx<T> s = C<T>(0, 0);
            if (o < J.no) {
#pragma unroll
                for (int i = 0; i < NI; ++i) s = s + lin_coef<T>(J.code[o][i], kx, ky) * in[i][e];
            }
            out[o][e] = scale * s;
        }
    }
    if (ny > 1 && LK == 1) {
#pragma unroll
        for (int o = 0; o < LINJ_MAXO; ++o)
            if (o < J.no) col_fft_group<T, EPC, 1>(g, ct, twm, out + o, true);
    } else if (ny > 1) {
        col_fft_first<T, EPC, LINJ_MAXO>(g, ct, twm, out, J.no, true);
    }
    if (ct.valid) {
#pragma unroll
        for (int o = 0; o < LINJ_MAXO; ++o) {
            if (o >= J.no) break;
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                const int j = ct.t + g.TPC * e;
                if (j < ny) J.dst[o][(size_t)ct.kx * ny + j] = out[o][e];
            }
        }
    }
}

// A^{-1} on D spectral columns: y-FFT, per-mode A^{-1} (times scale), y-IFFT.
template <typename T, int EPC, int D>
__global__ void __launch_bounds__(256) k_cols_precond(ColGeom g, PtrList<const cpx<T>, MAXF> src,
                                                       PtrList<cpx<T>, MAXF> dst,
                                                       const cpx<T>* __restrict__ tw, T tpx, T tpy,
                                                       T sig, T alp, T scale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    const cpx<T>* twm = twl_setup<T>(tw, g.ny, lds + col_lds_data(g, D));
    const ColThread<T> ct = col_thread<T>(g, lds);
    cpx<T> in[D][EPC];
    const cpx<T>* srcs[D];
    cpx<T>* dsts[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
        srcs[c] = src.p[c];
        dsts[c] = dst.p[c];
    }
    col_load<T, EPC, D>(g, ct, srcs, true, twm, in);
    const T kx = wavenumber<T>(ct.kx, g.nx, tpx);
    cpx<T> out[D][EPC];
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
        const int j = ct.t + g.TPC * e;
        const T ky = (D == 2) ? wavenumber<T>(j, g.ny, tpy) : (T)0;
        cpx<T> r[D], z[D];
#pragma unroll
        for (int c = 0; c < D; ++c) r[c] = in[c][e];
        precond_mode<T, D>(kx, ky, sig, alp, r, z);
#pragma unroll
        for (int c = 0; c < D; ++c) out[c][e] = scale * z[c];
    }
    col_store<T, EPC, D>(g, ct, out, dsts, true, twm);
}

// ---------------------------------------------------------------------------
// Krylov solve kernels (PCG of section 3.2 with the state x, r, p, q kept in
// the S layout; dot products by Parseval over the half spectrum, in FP64).
// One iteration is C1 -> R1 -> C2:
//   C1: reduce the previous update's (r.z, r.r) -> stop test, beta;
//       z = A^{-1} r, p = z + beta p; emits (p, div p) / (nx ny) and the y-IFFT
//   R1: x-IFFT -> pointwise  a = eta p + grad h (eta^2/2 div p + eta grad h.p),
//                            w = eta^3/3 div p + eta^2/2 grad h.p  -> x-FFT;
//       partial p.Gp as the grid sum of the weak form B[p, p] (section 3.1),
//       sum_x (p, div p)^T M(x) (p, div p) with M of Appendix A
//   C2: reduce p.Gp -> alpha; y-FFT; q = a - i k w (= G p, Def:G);
//       x += alpha p, r -= alpha q, z = A^{-1} r; partial r.z, r.r
// p.Gp equals B[p, p] exactly for the spectral D (real antisymmetric), so the
// curvature is known before q is formed and the update needs no extra pass.
// Every kernel returns at once when the solve is done.
// ---------------------------------------------------------------------------

// Broadcast thread 0's value to the block.
template <bool LDS_ONLY = false>
__device__ __forceinline__ double bcast(double v, double* slot) {
    if (threadIdx.x == 0) *slot = v;
    if (LDS_ONLY)
        block_lds_barrier();
    else
        __syncthreads();
    const double r = *slot;
    if (LDS_ONLY)
        block_lds_barrier();
    else
        __syncthreads();
    return r;
}

// Stop test and beta from the partials of the last update pass (or of the
// initial residual).  Identical in every block; block 0 publishes.  Returns done.
__device__ __forceinline__ bool pcg_iterate_state(SolveScal* __restrict__ sc, const double* __restrict__ part,
                                                  int nb3, double* red, double* slot, double& beta_out) {
    double tot[2];
    final_sum<2>(part + PART_C3, nb3, tot, red);
    const double rz = bcast(tot[0], slot) * sc->inv_n;
    const double rr = bcast(tot[1], slot + 1) * sc->inv_n;
    const int first = sc->first;
    // init_bb: ||b||^2 is the first r.r seen (r_0 = b); taken once, while bb is unset
    const double bb = (sc->init_bb && first && sc->iter == 0 && sc->bb == 0.0) ? rr : sc->bb;
    const bool bad = !(rr == rr) || !(rz == rz) || !(rr <= 1.0e300);
    const bool conv = !bad && (bb == 0.0 || rr <= sc->tol2 * bb);
    const bool done = bad || conv || sc->iter >= sc->max_iter;
    const double beta = first ? 0.0 : rz / sc->rho_prev;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rr = rr;
        sc->bb = bb;
        sc->relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
        sc->rho = rz;
        sc->beta = beta;
        sc->converged = conv ? 1 : 0;
        if (bad) sc->status = -2;
        sc->done = done ? 1 : 0;
    }
    beta_out = beta;
    return done;
}

// C1_UPDATE: the PCG step (p = z + beta p); C1_COPY: p = xsrc (apply G to a
// given field); C1_ACCUM: x += dx (FP32 correction of a refinement step,
// x in ph) and p = x, so the pass that starts the FP64 residual also applies
// the correction.
enum { C1_UPDATE = 0, C1_COPY = 1, C1_ACCUM = 2 };

template <typename T, int EPC, int D, int MODE>
__global__ void __launch_bounds__(256) k_pcg_c1(ColGeom g, const cpx<T>* __restrict__ tw,
                                                 SolveScal* __restrict__ sc, const double* __restrict__ part,
                                                 int nb3, const cpx<T>* __restrict__ rh, cpx<T>* __restrict__ ph,
                                                 const cpx<T>* __restrict__ xsrc, cpx<T>* __restrict__ H,
                                                 size_t NS, T tpx, T tpy, const cpx<float>* __restrict__ dx) {
    if (sc->done) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    __shared__ double red[32];
    __shared__ double slot[2];
    double beta_d = 0.0;
    if (MODE == C1_UPDATE) {
        if (pcg_iterate_state(sc, part, nb3, red, slot, beta_d)) return;
    }
    // (loading r and p ahead of this reduction, in flight across it, measured
    // slower: 17.0 -> 18.5 us at 1024^2 FP64)
    const cpx<T>* twm = twl_setup<T>(tw, g.ny, lds + col_lds_data(g, D + 1));
    const ColThread<T> ct = col_thread<T>(g, lds);
    const T beta = (T)beta_d, sig = (T)sc->sig, alp = (T)sc->alp, inv_n = (T)sc->inv_n;
    const T kx = wavenumber<T>(ct.kx, g.nx, tpx);
    cpx<T> o[D + 1][EPC];
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
        const int j = ct.t + g.TPC * e;
#pragma unroll
        for (int c = 0; c <= D; ++c) o[c][e] = C<T>(0, 0);
        if (ct.valid && j < g.ny) {
            const size_t idx = (size_t)ct.kx * g.ny + j;
            const T ky = (D == 2) ? wavenumber<T>(j, g.ny, tpy) : (T)0;
            cpx<T> p[D];
            if (MODE == C1_COPY) {
#pragma unroll
                for (int c = 0; c < D; ++c) p[c] = xsrc[c * NS + idx];
            } else if (MODE == C1_ACCUM) {
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    const cpx<T> x = ph[c * NS + idx];
                    const cpx<float> e = dx[c * NS + idx];
                    p[c] = cpx<T>{x.re + (T)e.re, x.im + (T)e.im};
                    ph[c * NS + idx] = p[c];
                }
            } else {
                cpx<T> r[D], z[D];
#pragma unroll
                for (int c = 0; c < D; ++c) r[c] = rh[c * NS + idx];
                precond_mode<T, D>(kx, ky, sig, alp, r, z);
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    // beta = 0 on the first iteration: p = z without reading the
                    // previous (unset) direction
                    p[c] = (beta != (T)0) ? z[c] + beta * ph[c * NS + idx] : z[c];
                    ph[c * NS + idx] = p[c];
                }
            }
            cpx<T> dv = ik(kx, p[0]);
            if (D == 2) dv = dv + ik(ky, p[1 % D]);
#pragma unroll
            for (int c = 0; c < D; ++c) o[c][e] = inv_n * p[c];
            o[D][e] = inv_n * dv;
        }
    }
    cpx<T>* dsts[D + 1];
#pragma unroll
    for (int c = 0; c <= D; ++c) dsts[c] = H + c * NS;
    col_store<T, EPC, D + 1>(g, ct, o, dsts, true, twm);
}

// Stop test only (one block): closes a chunk of iterations so the host can
// read the done flag.  Idempotent with the C1 that follows.  With pub set,
// thread 0 then publishes the loop flags as k_publish_flags does.
__device__ __forceinline__ void publish_flags(const SolveScal* sc, int* d, int seq) {
    volatile int* v = d;
    v[0] = sc->iter;
    v[1] = sc->max_iter;
    v[2] = sc->done;
    v[3] = sc->converged;
    v[4] = sc->flat;
    v[5] = sc->status;
    v[7] = sc->outer;
    v[6] = seq;
}
__device__ __forceinline__ void inner_close(SolveScal* s, const SolveScal* d);
// With inner set (the FP32 inner solve of a refinement step that has just
// ended), thread 0 first adds that step to the counters (see inner_close).
__global__ void __launch_bounds__(256) k_pcg_check(SolveScal* __restrict__ sc, const double* __restrict__ part,
                                                   int nb3, int* pub, int seq, const SolveScal* __restrict__ inner) {
    if (inner) {
        if (threadIdx.x == 0) inner_close(sc, inner);
        __syncthreads();
    }
    if (!sc->done) {
        __shared__ double red[32];
        __shared__ double slot[2];
        double beta;
        pcg_iterate_state(sc, part, nb3, red, slot, beta);
    }
    // block 0 thread 0 wrote the scalars above and reads them back here
    if (pub && blockIdx.x == 0 && threadIdx.x == 0) publish_flags(sc, pub, seq);
}

// Publish iter, max_iter, done, converged, flat, status of a solve into host
// memory (d: device address of a host-coherent pinned buffer), then the
// sequence number seq in d[6].  The stores are volatile and system-coherent:
// each completes before the next is issued, so a host that sees seq also sees
// the values (no cache-wide fence needed for one thread's ordered stores).
__global__ void k_publish_flags(const SolveScal* __restrict__ sc, int* d, int seq) {
    if (threadIdx.x == 0 && blockIdx.x == 0) publish_flags(sc, d, seq);
}

template <typename T, int EPC, int D, bool SEQ, int MAXT = 1024>
__global__ void __launch_bounds__(MAXT) k_pcg_r1(RowGeom g, const cpx<T>* __restrict__ tw,
                                                 SolveScal* __restrict__ sc, cpx<T>* H, size_t NS,
                                                 const T* __restrict__ eta, const T* __restrict__ gh,
                                                 double* __restrict__ part) {
    if (sc->done) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    __shared__ double red[16];
    constexpr int NF = SEQ ? 1 : D + 1;
    const cpx<T>* twm = twl_setup<T>(tw, g.M, lds + row_lds_data(g, NF));
    const RowThread<T> rt = row_thread<T>(g, lds);
    double acc[1] = {0.0};
    cpx<T> v[D + 1][EPC];
    if (SEQ) {
#pragma unroll
        for (int c = 0; c <= D; ++c) {
            const cpx<T>* Hc[1] = {H + c * NS};
            cpx<T> vc[1][EPC];
            row_inverse<T, EPC, 1>(g, rt, Hc, tw, twm, vc);
#pragma unroll
            for (int e = 0; e < EPC; ++e) v[c][e] = vc[0][e];
        }
    } else {
        const cpx<T>* Hs[D + 1];
#pragma unroll
        for (int c = 0; c <= D; ++c) Hs[c] = H + c * NS;
        if (EPC <= 2)
            row_inverse_batched<T, EPC, D + 1>(g, rt, Hs, tw, twm, v);
        else
            row_inverse<T, EPC, D + 1>(g, rt, Hs, tw, twm, v);
    }
    const size_t npts = (size_t)g.nx * g.ny;
    const T third = (T)1 / (T)3, half = (T)0.5;
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
        const int j = rt.t + g.TPR * e;
        if (j < g.M && rt.valid) {
            const size_t o = (size_t)rt.y * g.nx + 2 * j;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const T et = eta[o + s];
                T hc[D], pc[D];
                T bt = 0;
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    hc[c] = gh[c * npts + o + s];
                    pc[c] = s ? v[c][e].im : v[c][e].re;
                    bt += hc[c] * pc[c];
                }
                const T dl = s ? v[D][e].im : v[D][e].re;
                const T e2 = et * et;
                const T w1 = third * e2 * et * dl + half * e2 * bt;
                const T w2 = half * e2 * dl + et * bt;
                // B-density: eta |p|^2 + eta^3/3 dl^2 + eta^2 dl bt + eta bt^2 = p.a + dl w1
                double pp = 0.0;
#pragma unroll
                for (int c = 0; c < D; ++c) pp += (double)pc[c] * (double)pc[c];
                acc[0] += (double)et * pp + (double)dl * (double)w1 + (double)bt * (double)w2;
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    const T a = et * pc[c] + hc[c] * w2;
                    if (s) v[c][e].im = a; else v[c][e].re = a;
                }
                if (s) v[D][e].im = w1; else v[D][e].re = w1;
            }
        }
    }
    if (SEQ) {
#pragma unroll
        for (int c = 0; c <= D; ++c) {
            cpx<T>* Hc[1] = {H + c * NS};
            cpx<T> vc[1][EPC];
#pragma unroll
            for (int e = 0; e < EPC; ++e) vc[0][e] = v[c][e];
            row_forward<T, EPC, 1>(g, rt, vc, Hc, tw, twm, (T)1);
        }
    } else {
        cpx<T>* Hs[D + 1];
#pragma unroll
        for (int c = 0; c <= D; ++c) Hs[c] = H + c * NS;
        row_forward<T, EPC, D + 1>(g, rt, v, Hs, tw, twm, (T)1);
    }
    if (part) {
        block_sum<1>(acc, red);
        if (threadIdx.x == 0) part[PART_C2 + blockIdx.x] = acc[0];
    }
}

enum { C2_RESID = 1, C2_STORE = 2, C2_UPDATE = 3, C2_RESID_INIT = 4 };

// MODE C2_UPDATE: reduce p.Gp (row-pass partials, nb_r1 blocks) -> alpha;
//   q = G p; x += alpha p; r -= alpha q; z = A^{-1} r; partial r.z, r.r.
// MODE C2_RESID: r = b - G x -> rh; partial r.z, r.r.
// MODE C2_RESID_INIT: reduce ||b||^2 (setup partials, nb_r1 blocks) -> bb;
//   r = b - G x -> rh (x = r = 0 for a zero b); partial r.z, r.r of r_0.
// MODE C2_STORE: q = G p -> qh.
// Projection of a residual mode onto the reflection-symmetric modes of a wall
// grid's periodic twin (Nx x Ny points): velocity component c is odd along its
// own axis and even along the other.  A field with E[N-1-X] = s E[X] along an
// axis has E^[k] = s e^{2 pi i k / N} E^[-k]; in the half spectrum E^[ky][-kx] is
// conj(E^[-ky][kx]), so both reflections pair the mode (kx, ky) with (kx, -ky) of
// the same column.  a: the mode, b: its partner (kx, -ky).
template <typename T, int D>
__device__ __forceinline__ cpx<T> wall_project(int c, cpx<T> a, cpx<T> b, int kx, int nx, int ky, int ny) {
    const T half = (T)0.5;
    if (D == 2) {
        const T sy = c == 1 ? (T)-1 : (T)1;
        T sn, cs;
        if (sizeof(T) == 8) {
            double s2, c2;
            sincospi(2.0 * (double)ky / (double)ny, &s2, &c2);
            sn = (T)s2;
            cs = (T)c2;
        } else {
            float s2, c2;
            sincospif(2.0f * (float)ky / (float)ny, &s2, &c2);
            sn = (T)s2;
            cs = (T)c2;
        }
        const cpx<T> om = C<T>(sy * cs, sy * sn), omc = C<T>(sy * cs, -sy * sn);
        const cpx<T> a2 = half * (a + om * b);
        const cpx<T> b2 = half * (b + omc * a);
        a = a2;
        b = b2;
    }
    const T sx = c == 0 ? (T)-1 : (T)1;
    T sn, cs;
    if (sizeof(T) == 8) {
        double s2, c2;
        sincospi(2.0 * (double)kx / (double)nx, &s2, &c2);
        sn = (T)s2;
        cs = (T)c2;
    } else {
        float s2, c2;
        sincospif(2.0f * (float)kx / (float)nx, &s2, &c2);
        sn = (T)s2;
        cs = (T)c2;
    }
    const cpx<T> ph = C<T>(sx * cs, sx * sn);
    return half * (a + ph * cj(b));
}

// WALL: the solve runs on the periodic twin of a wall grid; the new residual is
// projected onto the symmetric modes before it is used (rounding would otherwise
// seed the other parity, which the iteration amplifies at low wavenumbers).
template <typename T, int EPC, int D, int MODE, bool WALL = false>
__global__ void __launch_bounds__(256) k_pcg_c2(ColGeom g, const cpx<T>* __restrict__ tw,
                                                 SolveScal* __restrict__ sc, const cpx<T>* __restrict__ H,
                                                 size_t NS, cpx<T>* __restrict__ qh, const cpx<T>* __restrict__ ph,
                                                 cpx<T>* __restrict__ xh, const cpx<T>* __restrict__ bh,
                                                 cpx<T>* __restrict__ rh, double* __restrict__ part, int nb_r1,
                                                 T tpx, T tpy) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    __shared__ double red[32];
    __shared__ double slot[1];
    const cpx<T>* twm = twl_setup<T>(tw, g.ny, lds + col_lds_data(g, D + 1));
    const ColThread<T> ct = col_thread<T>(g, lds);
    // the row pass's columns do not depend on alpha: loaded right after the
    // partials of the reduction, in flight across it (LDS-only barriers)
    if (sc->done) return;
    double pb[PF_K][1];
    if (MODE == C2_UPDATE) partials_fetch<1>(part + PART_C2, nb_r1, pb);
    if (MODE == C2_RESID_INIT) partials_fetch<1>(part + PART_GEN, nb_r1, pb);
    __builtin_amdgcn_sched_barrier(0);   // the partials' loads first
    cpx<T> in[D + 1][EPC];
    {
        const cpx<T>* srcs[D + 1];
#pragma unroll
        for (int c = 0; c <= D; ++c) srcs[c] = H + c * NS;
        col_fetch<T, EPC, D + 1>(g, ct, srcs, in);
    }
    __builtin_amdgcn_sched_barrier(0);   // keep the data loads ahead of the reduction
    T alpha = (T)0;
    bool zero_x = false;
    if (MODE == C2_RESID_INIT) {
        double tot[1];
        partials_sum<1, true>(part + PART_GEN, nb_r1, pb, tot, red);
        const double bb = bcast<true>(tot[0], slot) * sc->inv_n;
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
    }
    if (MODE == C2_UPDATE) {
        double tot[1];
        partials_sum<1, true>(part + PART_C2, nb_r1, pb, tot, red);
        const double pq = bcast<true>(tot[0], slot);
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
    col_fft<T, EPC, D + 1>(g, ct, twm, in);
    const T kx = wavenumber<T>(ct.kx, g.nx, tpx);
    const T sig = (T)sc->sig, alp = (T)sc->alp;
    const double w = ct.valid ? half_weight(ct.kx, g.nx) : 0.0;
    double acc[2] = {0.0, 0.0};
    if (WALL && MODE != C2_STORE) {
        // the new residual of the whole column first, then its projection
        cpx<T> rn[D][EPC];
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = ct.t + g.TPC * e;
#pragma unroll
            for (int c = 0; c < D; ++c) rn[c][e] = C<T>(0, 0);
            if (ct.valid && j < g.ny) {
                const size_t idx = (size_t)ct.kx * g.ny + j;
                const T ky = (D == 2) ? wavenumber<T>(j, g.ny, tpy) : (T)0;
                const cpx<T> wv = in[D][e];
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    const T kc = (c == 0) ? kx : ky;
                    const cpx<T> q = in[c][e] - ik(kc, wv);
                    if (MODE == C2_RESID) {
                        rn[c][e] = bh[c * NS + idx] - q;
                    } else if (MODE == C2_RESID_INIT) {
                        rn[c][e] = zero_x ? C<T>(0, 0) : bh[c * NS + idx] - q;
                        if (zero_x) xh[c * NS + idx] = C<T>(0, 0);
                    } else {
                        xh[c * NS + idx] = xh[c * NS + idx] + alpha * ph[c * NS + idx];
                        rn[c][e] = rh[c * NS + idx] - alpha * q;
                    }
                    ct.buf[c * ct.fstride + j] = rn[c][e];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = ct.t + g.TPC * e;
            if (ct.valid && j < g.ny) {
                const size_t idx = (size_t)ct.kx * g.ny + j;
                const int jm = (g.ny - j) & (g.ny - 1);
                const T ky = (D == 2) ? wavenumber<T>(j, g.ny, tpy) : (T)0;
                cpx<T> r[D], z[D];
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    r[c] = wall_project<T, D>(c, rn[c][e], ct.buf[c * ct.fstride + jm], ct.kx, g.nx, j, g.ny);
                    rh[c * NS + idx] = r[c];
                }
                precond_mode<T, D>(kx, ky, sig, alp, r, z);
#pragma unroll
                for (int c = 0; c < D; ++c) {
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
        return;
    }
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
        const int j = ct.t + g.TPC * e;
        if (ct.valid && j < g.ny) {
            const size_t idx = (size_t)ct.kx * g.ny + j;
            const T ky = (D == 2) ? wavenumber<T>(j, g.ny, tpy) : (T)0;
            const cpx<T> wv = in[D][e];
            cpx<T> r[D], z[D];
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const T kc = (c == 0) ? kx : ky;
                const cpx<T> q = in[c][e] - ik(kc, wv);
                if (MODE == C2_STORE) {
                    qh[c * NS + idx] = q;
                } else if (MODE == C2_RESID) {
                    r[c] = bh[c * NS + idx] - q;
                    rh[c * NS + idx] = r[c];
                } else if (MODE == C2_RESID_INIT) {
                    r[c] = zero_x ? C<T>(0, 0) : bh[c * NS + idx] - q;
                    rh[c * NS + idx] = r[c];
                    if (zero_x) xh[c * NS + idx] = C<T>(0, 0);
                } else {
                    xh[c * NS + idx] = xh[c * NS + idx] + alpha * ph[c * NS + idx];
                    r[c] = rh[c * NS + idx] - alpha * q;
                    rh[c * NS + idx] = r[c];
                }
            }
            if (MODE != C2_STORE) {
                precond_mode<T, D>(kx, ky, sig, alp, r, z);
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    acc[0] += w * ((double)r[c].re * (double)z[c].re + (double)r[c].im * (double)z[c].im);
                    acc[1] += w * ((double)r[c].re * (double)r[c].re + (double)r[c].im * (double)r[c].im);
                }
            }
        }
    }
    if (MODE != C2_STORE) {
        block_sum<2>(acc, red);
        if (threadIdx.x == 0) {
            part[PART_C3 + 2 * blockIdx.x] = acc[0];
            part[PART_C3 + 2 * blockIdx.x + 1] = acc[1];
        }
    }
}

// First column pass of a solve.  Hb holds the row transforms of b (D fields),
// Hu those of the initial guess u0 (GUESS).  y-FFT of b -> b_hat into rh (and
// bh).  GUESS: partial ||b||^2; y-FFT of u0 -> x_hat, and (x_hat, div x_hat)/N
// y-inverse-transformed into H for the row pass of G x_0 (C2_RESID_INIT then
// forms r_0).  Otherwise x_hat = 0, r_0 = b_hat and the partials r.z, r.r.
// GUESS: the b part runs on blocks [0, nblocks) and the u0 part on blocks
// [nblocks, 2 nblocks), side by side (H must not alias Hb then).
template <typename T, int EPC, int D, bool GUESS>
__global__ void __launch_bounds__(256) k_pcg_setup(ColGeom g, const cpx<T>* __restrict__ tw,
                                                    const SolveScal* __restrict__ sc, const cpx<T>* Hb,
                                                    const cpx<T>* __restrict__ Hu, size_t NS, cpx<T>* __restrict__ bh,
                                                    cpx<T>* __restrict__ rh, cpx<T>* __restrict__ xh, cpx<T>* H,
                                                    double* __restrict__ part, T tpx, T tpy) {
    if (sc->done) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    __shared__ double red[32];
    const cpx<T>* twm = twl_setup<T>(tw, g.ny, lds + col_lds_data(g, D + 1));
    const int job = GUESS ? (int)blockIdx.x / g.nblocks : 0;
    const ColThread<T> ct = col_thread_at<T>(g, lds, (int)blockIdx.x - job * g.nblocks);
    const double w = ct.valid ? half_weight(ct.kx, g.nx) : 0.0;
    const T kx = wavenumber<T>(ct.kx, g.nx, tpx);
    const T sig = (T)sc->sig, alp = (T)sc->alp, inv_n = (T)sc->inv_n;
    if (GUESS && job == 1) {
        cpx<T> vu[D][EPC];
        {
            const cpx<T>* srcs[D];
#pragma unroll
            for (int c = 0; c < D; ++c) srcs[c] = Hu + c * NS;
            col_load<T, EPC, D>(g, ct, srcs, false, twm, vu);
        }
        // the row pass's u0 columns need no y round trip: IFFT_y(x_hat / N) of
        // x_hat = FFT_y(u0 rows) is the u0 rows times ny / N, stored as loaded;
        // only div x_hat is formed in the spectral domain and inverse-transformed
        const T sraw = inv_n * (T)g.ny;
        if (ct.valid) {
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                const int j = ct.t + g.TPC * e;
                if (j < g.ny) {
#pragma unroll
                    for (int c = 0; c < D; ++c) H[c * NS + (size_t)ct.kx * g.ny + j] = sraw * vu[c][e];
                }
            }
        }
        col_fft<T, EPC, D>(g, ct, twm, vu);
        cpx<T> o[1][EPC];
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = ct.t + g.TPC * e;
            o[0][e] = C<T>(0, 0);
            if (ct.valid && j < g.ny) {
                const size_t idx = (size_t)ct.kx * g.ny + j;
                const T ky = (D == 2) ? wavenumber<T>(j, g.ny, tpy) : (T)0;
#pragma unroll
                for (int c = 0; c < D; ++c) xh[c * NS + idx] = vu[c][e];
                cpx<T> dv = ik(kx, vu[0][e]);
                if (D == 2) dv = dv + ik(ky, vu[1 % D][e]);
                o[0][e] = inv_n * dv;
            }
        }
        cpx<T>* dsts[1] = {H + D * NS};
        col_store<T, EPC, 1>(g, ct, o, dsts, true, twm);
        return;
    }
    cpx<T> vb[D][EPC];
    {
        const cpx<T>* srcs[D];
#pragma unroll
        for (int c = 0; c < D; ++c) srcs[c] = Hb + c * NS;
        col_load<T, EPC, D>(g, ct, srcs, true, twm, vb);
    }
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
        const int j = ct.t + g.TPC * e;
        if (ct.valid && j < g.ny) {
            const size_t idx = (size_t)ct.kx * g.ny + j;
            cpx<T> r[D], z[D];
#pragma unroll
            for (int c = 0; c < D; ++c) {
                r[c] = vb[c][e];
                if (bh) bh[c * NS + idx] = r[c];
                rh[c * NS + idx] = r[c];
                if (!GUESS) xh[c * NS + idx] = C<T>(0, 0);
            }
            if (GUESS) {
#pragma unroll
                for (int c = 0; c < D; ++c)
                    acc[0] += w * ((double)r[c].re * (double)r[c].re + (double)r[c].im * (double)r[c].im);
            } else {
                const T ky = (D == 2) ? wavenumber<T>(j, g.ny, tpy) : (T)0;
                precond_mode<T, D>(kx, ky, sig, alp, r, z);
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    acc[0] += w * ((double)r[c].re * (double)z[c].re + (double)r[c].im * (double)z[c].im);
                    acc[1] += w * ((double)r[c].re * (double)r[c].re + (double)r[c].im * (double)r[c].im);
                }
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


// Forward y-FFT of D H fields into S fields (no reduction).
template <typename T, int EPC, int D>
__global__ void __launch_bounds__(256) k_cols_to_S(ColGeom g, const cpx<T>* __restrict__ tw,
                                                    const cpx<T>* __restrict__ H, size_t NS,
                                                    cpx<T>* __restrict__ Sdst) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    const cpx<T>* twm = twl_setup<T>(tw, g.ny, lds + col_lds_data(g, D));
    const ColThread<T> ct = col_thread<T>(g, lds);
    cpx<T> v[D][EPC];
    const cpx<T>* srcs[D];
    cpx<T>* dsts[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
        srcs[c] = H + c * NS;
        dsts[c] = Sdst + c * NS;
    }
    col_load<T, EPC, D>(g, ct, srcs, true, twm, v);
    col_store<T, EPC, D>(g, ct, v, dsts, false, twm);
}

// Inverse y-FFT of D S fields (times scale) into H fields.
template <typename T, int EPC, int D>
__global__ void __launch_bounds__(256) k_cols_from_S(ColGeom g, const cpx<T>* __restrict__ tw,
                                                      const cpx<T>* __restrict__ Ssrc, size_t NS,
                                                      cpx<T>* __restrict__ H, T scale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    const cpx<T>* twm = twl_setup<T>(tw, g.ny, lds + col_lds_data(g, D));
    const ColThread<T> ct = col_thread<T>(g, lds);
    cpx<T> v[D][EPC];
    const cpx<T>* srcs[D];
    cpx<T>* dsts[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
        srcs[c] = Ssrc + c * NS;
        dsts[c] = H + c * NS;
    }
    col_load<T, EPC, D>(g, ct, srcs, false, twm, v);
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
        for (int e = 0; e < EPC; ++e) v[c][e] = scale * v[c][e];
    col_store<T, EPC, D>(g, ct, v, dsts, true, twm);
}

// Spectral resampling between two grids of one domain, column part (the
// de-aliased right-hand side, subsec:dswe_1d): column kx of the destination
// takes the source's S-layout modes (source column length ny_src) for
// kx < kx_keep and signed ky mode |m| < m_keep, zero elsewhere, times scale,
// then runs the inverse y-FFT of the destination length; the result is the
// destination's H layout.  kx_keep and m_keep are half the smaller grid's
// lengths (m_keep = 1 in 1D), so the smaller grid's Nyquist modes are dropped.
template <typename T, int EPC, int NF>
__global__ void __launch_bounds__(256) k_cols_resample(ColGeom g, const cpx<T>* __restrict__ tw,
                                                        PtrList<const cpx<T>, MAXF> src, int ny_src,
                                                        PtrList<cpx<T>, MAXF> dst, int kx_keep, int m_keep,
                                                        T scale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    const cpx<T>* twm = twl_setup<T>(tw, g.ny, lds + col_lds_data(g, NF));
    const ColThread<T> ct = col_thread<T>(g, lds);
    const bool col_kept = ct.valid && ct.kx < kx_keep;
    cpx<T> v[NF][EPC];
    cpx<T>* dsts[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        dsts[f] = dst.p[f];
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const int j = ct.t + g.TPC * e;
            const int m = (g.ny == 1) ? 0 : (j < g.ny / 2 ? j : j - g.ny);
            const bool keep = col_kept && j < g.ny && m < m_keep && -m < m_keep;
            const int js = m < 0 ? m + ny_src : m;
            v[f][e] = keep ? scale * src.p[f][(size_t)ct.kx * ny_src + js] : C<T>(0, 0);
        }
    }
    col_store<T, EPC, NF>(g, ct, v, dsts, true, twm);
}

// Grids between walls run on their periodic twin (twice the length per axis):
// k_reflect writes the even / odd reflection of nf fields of the nx x ny wall
// grid (field stride sstride) onto the twin (field stride dstride):
// dst[Y][X] = sx sy src[ry][rx], r(X) = X below n and 2n - 1 - X above, with the
// sign -1 on the reflected half of an axis along which field f is odd (bit f of
// oddx / oddy).
__global__ void __launch_bounds__(256) k_reflect(int nx, int ny, int nye, const double* __restrict__ src,
                                                  size_t sstride, double* __restrict__ dst, size_t dstride, int nf,
                                                  unsigned oddx, unsigned oddy) {
    const int nxe = 2 * nx;
    const size_t ne = (size_t)nxe * nye;
    const size_t total = ne * (size_t)nf;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int f = (int)(i / ne);
        const size_t p = i - (size_t)f * ne;
        const int Y = (int)(p / nxe), X = (int)(p - (size_t)Y * nxe);
        const bool fx = X >= nx, fy = Y >= ny;
        const int x = fx ? nxe - 1 - X : X;
        const int y = fy ? 2 * ny - 1 - Y : Y;
        double v = src[(size_t)f * sstride + (size_t)y * nx + x];
        if (fx && ((oddx >> f) & 1u)) v = -v;
        if (fy && ((oddy >> f) & 1u)) v = -v;
        dst[(size_t)f * dstride + p] = v;
    }
}

// k_restrict returns the symmetric part: the mean of a point's images on the twin
// (2 in 1D, 4 in 2D, signed as in k_reflect), which is the point itself for a
// symmetric field and drops what rounding put into the other parities.
__global__ void __launch_bounds__(256) k_restrict(int nx, int ny, int nye, const double* __restrict__ src,
                                                   size_t sstride, double* __restrict__ dst, size_t dstride, int nf,
                                                   unsigned oddx, unsigned oddy) {
    const size_t n = (size_t)nx * ny;
    const size_t total = n * (size_t)nf;
    const int nxe = 2 * nx;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int f = (int)(i / n);
        const size_t p = i - (size_t)f * n;
        const int y = (int)(p / nx), x = (int)(p - (size_t)y * nx);
        const double* sf = src + (size_t)f * sstride;
        const double sx = ((oddx >> f) & 1u) ? -1.0 : 1.0;
        const int xm = nxe - 1 - x;
        double v = sf[(size_t)y * nxe + x] + sx * sf[(size_t)y * nxe + xm];
        if (nye > 1) {
            const double sy = ((oddy >> f) & 1u) ? -1.0 : 1.0;
            const int ym = nye - 1 - y;
            v += sy * (sf[(size_t)ym * nxe + x] + sx * sf[(size_t)ym * nxe + xm]);
            v *= 0.25;
        } else {
            v *= 0.5;
        }
        dst[(size_t)f * dstride + p] = v;
    }
}

// Initialise the scalars of a solve on the device (no host round trip).  With
// have_coeffs the preconditioner coefficients are given; otherwise they are
// filled later by k_coeffs_finish or copied from another solve.
__global__ void k_init_scal(SolveScal* __restrict__ sc, double tol, int max_iter, double inv_n, int have_coeffs,
                            double sig, double alp, double kap, int flat, int init_bb) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    sc->rho = sc->rho_prev = sc->alpha = sc->beta = sc->bb = sc->rr = sc->pq = sc->relres = 0.0;
    sc->tol2 = tol * tol;
    sc->inv_n = inv_n;
    sc->iter = 0;
    sc->max_iter = max_iter;
    sc->done = 0;
    sc->converged = 0;
    sc->status = 0;
    sc->first = 1;
    sc->init_bb = init_bb;
    sc->outer = 0;
    if (have_coeffs) {
        sc->sig = sig;
        sc->alp = alp;
        sc->kap = kap;
        sc->flat = flat;
    }
}

// One refinement step enqueued without a host round trip: inner_open (run by
// the first thread of k_inner_start) starts the inner FP32 solve d of the step
// (the scalars of k_init_scal, the outer solve's coefficients), or, when the
// outer solve s has already converged, marks the inner solve done so that every
// kernel of the step returns at once.  The inner tolerance is no tighter than
// the outer target needs: with outer residual r, target tol ||b|| and inner stop
// ||r_in|| <= t ||r||, t = max(t_min, c tol ||b|| / ||r||) (c2 = c^2), so once r
// is within a few orders of the target the inner solve stops as soon as the
// corrected outer residual will meet it.  inner_close (run by k_pcg_check's
// first thread after the step's FP64 residual) adds the step's inner iterations
// and the step itself to the outer solve's counters (s->iter, s->outer) unless
// it was skipped.
__device__ __forceinline__ void inner_open(const SolveScal* __restrict__ s, SolveScal* __restrict__ d, double tol,
                                           int max_iter, double inv_n, double c2) {
    if (s->done) {
        d->done = 1;
        return;
    }
    d->rho = d->rho_prev = d->alpha = d->beta = d->bb = d->rr = d->pq = d->relres = 0.0;
    d->tol2 = tol * tol;
    d->inv_n = inv_n;
    d->iter = 0;
    d->max_iter = max_iter;
    d->done = 0;
    d->converged = 0;
    d->status = 0;
    d->first = 1;
    d->init_bb = 1;
    d->outer = 0;
    d->sig = s->sig;
    d->alp = s->alp;
    d->kap = s->kap;
    d->flat = s->flat;
    if (s->rr > 0.0 && s->bb > 0.0) {
        const double t2 = c2 * s->tol2 * (s->bb / s->rr);
        if (t2 > d->tol2) d->tol2 = t2 < 0.25 ? t2 : 0.25;
    }
}
__device__ __forceinline__ void inner_close(SolveScal* s, const SolveScal* d) {
    if (s->done) return;
    s->iter += d->iter;
    s->outer += 1;
}

// ---------------------------------------------------------------------------
// Reductions over physical fields (FP64)
// ---------------------------------------------------------------------------

// Per-block extremes for the coefficients of section 4: min eta, max eta,
// max(eta + lambda_+ eta |grad h|^2), max |grad h|^2 and a non-finite flag.
template <int D>
__global__ void __launch_bounds__(256) k_coeffs(size_t npts, const double* __restrict__ eta,
                                                const double* __restrict__ gh, double* __restrict__ part,
                                                float* __restrict__ eta32, float* __restrict__ gh32) {
    __shared__ double red[5 * 16];
    const double lp = (4.0 + sqrt(13.0)) / 6.0;
    double mn = 1.0e308, mx = -1.0e308, smax = -1.0e308, g2max = 0.0, bad = 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += stride) {
        const double e = eta[i];
        double g2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const double h = gh[c * npts + i];
            g2 += h * h;
            if (gh32) gh32[c * npts + i] = (float)h;
        }
        if (eta32) eta32[i] = (float)e;
        if (!isfinite(e) || !isfinite(g2)) bad = 1.0;
        mn = fmin(mn, e);
        mx = fmax(mx, e);
        smax = fmax(smax, e + lp * e * g2);
        g2max = fmax(g2max, g2);
    }
    double v[5] = {-mn, mx, smax, g2max, bad};
#pragma unroll
    for (int a = 0; a < 5; ++a) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[a] = fmax(v[a], __shfl_xor(v[a], off, 64));
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
    if (lane == 0)
        for (int a = 0; a < 5; ++a) red[a * 16 + wave] = v[a];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int a = 0; a < 5; ++a) {
            double s = red[a * 16];
            for (int w = 1; w < nw; ++w) s = fmax(s, red[a * 16 + w]);
            part[PART_GEN + 5 * blockIdx.x + a] = s;
        }
    }
}

// (sigma*, alpha*, kappa_ub) of Eq:FlatbathCoeff (flat), Eq:Optcoeff and
// Eq:Optcoeffb (kind 0) or Remark 4.2 (kind 1) from min eta, max eta,
// max(eta + lambda_+ eta |grad h|^2) and max |grad h|^2.  flat < 0 selects the
// flat formulas iff |grad h|_max = 0; the choice is returned in fl.
__host__ __device__ inline void coeffs_formula(double emin, double emax, double smx, double g2m, int flat, int kind,
                                               double& sig, double& alp, double& kap, int& fl) {
    const double lp = (4.0 + sqrt(13.0)) / 6.0;
    const double lm = (4.0 - sqrt(13.0)) / 6.0;
    const double ratio3 = (emax / emin) * (emax / emin) * (emax / emin);
    fl = flat < 0 ? (g2m == 0.0 ? 1 : 0) : (flat != 0 ? 1 : 0);
    if (fl) {
        sig = emax;
        alp = emax * emax * emax / 3.0;
        kap = ratio3;
    } else if (kind == 0) {
        sig = smx;
        alp = lp * emax * emax * emax;
        kap = fmax(smx / emin, (lp / lm) * ratio3);
    } else {
        sig = emax * (1.0 + lp * g2m);
        alp = lp * emax * emax * emax;
        kap = fmax((emax / emin) * (1.0 + lp * g2m), (lp / lm) * ratio3);
    }
}

// One block: the coefficients from the per-block extremes of k_coeffs.
// With init set, the solve's scalars are initialised here too (as k_init_scal
// with the given tol, max_iter, inv_n, init_bb), saving a launch per solve.
__global__ void __launch_bounds__(256) k_coeffs_finish(SolveScal* __restrict__ sc, const double* __restrict__ part,
                                                       int nb, int flat, int kind, int init, double tol,
                                                       int max_iter, double inv_n, int init_bb) {
    __shared__ double red[5 * 16];
    double r[5];
    final_max<5>(part + PART_GEN, nb, r, red);
    if (threadIdx.x != 0) return;
    if (init) {
        sc->rho = sc->rho_prev = sc->alpha = sc->beta = sc->bb = sc->rr = sc->pq = sc->relres = 0.0;
        sc->tol2 = tol * tol;
        sc->inv_n = inv_n;
        sc->iter = 0;
        sc->max_iter = max_iter;
        sc->done = 0;
        sc->converged = 0;
        sc->status = 0;
        sc->first = 1;
        sc->init_bb = init_bb;
    }
    const double emin = -r[0], emax = r[1], smx = r[2], g2m = r[3];
    sc->red[0] = emin;
    sc->red[1] = emax;
    sc->red[2] = smx;
    sc->red[3] = g2m;
    if (r[4] != 0.0 || !(emin > 0.0)) {
        sc->status = -2;
        sc->done = 1;
        return;
    }
    double sig, alp, kap;
    int fl;
    coeffs_formula(emin, emax, smx, g2m, flat, kind, sig, alp, kap, fl);
    sc->flat = fl;
    sc->sig = sig;
    sc->alp = alp;
    sc->kap = kap;
}

// Per-block min and max of a physical field (the flat-bottom test).
__global__ void __launch_bounds__(256) k_minmax(size_t n, const double* __restrict__ f, double* __restrict__ part) {
    __shared__ double red[2 * 16];
    double mn = 1.0e308, mx = -1.0e308;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        mn = fmin(mn, f[i]);
        mx = fmax(mx, f[i]);
    }
    double v[2] = {-mn, mx};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[a] = fmax(v[a], __shfl_xor(v[a], off, 64));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
    if (lane == 0) {
        red[wave] = v[0];
        red[16 + wave] = v[1];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = red[0], b = red[16];
        for (int w = 1; w < nw; ++w) {
            a = fmax(a, red[w]);
            b = fmax(b, red[16 + w]);
        }
        part[PART_GEN + 2 * blockIdx.x] = a;
        part[PART_GEN + 2 * blockIdx.x + 1] = b;
    }
}
__global__ void __launch_bounds__(256) k_minmax_finish(SolveScal* __restrict__ sc, const double* __restrict__ part,
                                                       int nb) {
    __shared__ double red[2 * 16];
    double r[2];
    final_max<2>(part + PART_GEN, nb, r, red);
    if (threadIdx.x == 0) {
        sc->red[0] = -r[0];
        sc->red[1] = r[1];
    }
}

// ---------------------------------------------------------------------------
// Small elementwise kernels
// ---------------------------------------------------------------------------
template <typename Td, typename Ts>
__global__ void k_convert(size_t n, const Ts* __restrict__ s, Td* __restrict__ d) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) d[i] = (Td)s[i];
}

// y = a*x + b*y  (b = 0 overwrites, x may be null for a pure scale)
__global__ void k_axpby(size_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double xv = x ? x[i] : 0.0;
        y[i] = (b == 0.0) ? a * xv : a * xv + b * y[i];
    }
}

// out = (base + dt * sum_k c_k f_k) / div  (up to 6 terms, in the order given;
// base may be null; div = 1 skips the division).  A multistep update divides by
// its leading coefficient rather than multiplying by a rounded reciprocal, so
// that coefficients summing to zero keep a constant field (and the mass) exact.
constexpr int LINCOMB_MAX = 6;
struct Lincomb4 {
    const double* f[LINCOMB_MAX];
    double c[LINCOMB_MAX];
    int n;
    double div;
};
__global__ void k_lincomb(size_t n, const double* __restrict__ base, double dt, Lincomb4 lc,
                          double* __restrict__ out) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double s = 0.0;
        for (int k = 0; k < lc.n; ++k) s += lc.c[k] * lc.f[k][i];
        const double v = (base ? base[i] : 0.0) + dt * s;
        out[i] = lc.div == 1.0 ? v : v / lc.div;
    }
}

// Up to three independent linear combinations in one launch, each
// out = base + dt * sum_k c_k f_k as in k_lincomb (same order of operations);
// with `save` set, base is also copied there (out may alias base).
struct LcJob {
    double* out;
    const double* base;
    double* save;
    const double* f[4];
    double c[4];
    double dt;
    int nf;
    size_t n;
};
struct LcJobs {
    LcJob j[3];
    int n;
};
__global__ void k_lincomb_jobs(LcJobs J) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (int k = 0; k < J.n; ++k) {
        const LcJob& a = J.j[k];
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
            double s = 0.0;
            for (int q = 0; q < a.nf; ++q) s += a.c[q] * a.f[q][i];
            const double b = a.base ? a.base[i] : 0.0;
            if (a.save) a.save[i] = b;
            a.out[i] = b + a.dt * s;
        }
    }
}

__global__ void k_zero_c(size_t n, void* __restrict__ p) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    double* d = reinterpret_cast<double*>(p);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) d[i] = 0.0;
}

// Start of an FP32 inner solve from the FP64 outer residual: the inner solve's
// scalars (inner_open, first thread), r32 = (float) r, x32 = 0, and the
// partials of r32.z, r32.r32, in one pass.  The other blocks read only the
// outer scalars s, so the first thread's writes to sc race with nothing.
template <int D>
__global__ void __launch_bounds__(256) k_inner_start(int nx, int ny, size_t NS, const SolveScal* __restrict__ s,
                                                     SolveScal* __restrict__ sc, double tol, int max_iter,
                                                     double inv_n, double c2, const cpx<double>* __restrict__ r64,
                                                     cpx<float>* __restrict__ r32, cpx<float>* __restrict__ x32,
                                                     double* __restrict__ part, float tpx, float tpy) {
    __shared__ double red[32];
    if (blockIdx.x == 0 && threadIdx.x == 0) inner_open(s, sc, tol, max_iter, inv_n, c2);
    if (s->done) return;   // the refinement had already converged
    const float sig = (float)s->sig, alp = (float)s->alp;
    double acc[2] = {0.0, 0.0};
    const int nsi = (int)NS;
    const int lny = ilog2(ny);
    const int stride = gridDim.x * blockDim.x;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nsi; idx += stride) {
        const int kxi = idx >> lny;
        const int kyi = idx & (ny - 1);
        const float kx = wavenumber<float>(kxi, nx, tpx);
        const float ky = (D == 2) ? wavenumber<float>(kyi, ny, tpy) : 0.0f;
        cpx<float> r[D], z[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const cpx<double> v = r64[c * NS + idx];
            r[c] = cpx<float>{(float)v.re, (float)v.im};
            r32[c * NS + idx] = r[c];
            x32[c * NS + idx] = C<float>(0, 0);
        }
        precond_mode<float, D>(kx, ky, sig, alp, r, z);
        const double w = half_weight(kxi, nx);
#pragma unroll
        for (int c = 0; c < D; ++c) {
            acc[0] += w * ((double)r[c].re * (double)z[c].re + (double)r[c].im * (double)z[c].im);
            acc[1] += w * ((double)r[c].re * (double)r[c].re + (double)r[c].im * (double)r[c].im);
        }
    }
    block_sum<2>(acc, red);
    if (threadIdx.x == 0) {
        part[PART_C3 + 2 * blockIdx.x] = acc[0];
        part[PART_C3 + 2 * blockIdx.x + 1] = acc[1];
    }
}


}  // namespace sgn

namespace sgn {

// ---------------------------------------------------------------------------
// GMRES building blocks on D-vector fields in the S layout (modes [kx][ky],
// kx = 0..nx/2), FP64.  Dot products are Parseval sums over the half spectrum
// (weight 1 at kx = 0 and nx/2, 2 elsewhere) divided by nx ny.
// ---------------------------------------------------------------------------

// The kernels below take an optional stop flag (the done flag of the solve's
// scalars): when it is set they return at once, so a host that issues several
// Arnoldi steps ahead pays little for the steps after the cycle has ended.
__device__ __forceinline__ bool gmres_stopped(const SolveScal* stop) { return stop && stop->done; }

// Per-block partials of <w, V_i> for i < nv (V_i = V + i * vstride):
// part[block * nv + i].
template <int D>
__global__ void __launch_bounds__(256) k_S_multidot(int nx, int ny, size_t NS, const cpx<double>* __restrict__ w,
                                                    const cpx<double>* __restrict__ V, size_t vstride, int nv,
                                                    double* __restrict__ part, const SolveScal* stop) {
    if (gmres_stopped(stop)) return;
    __shared__ double red[16 * 8];
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (int i0 = 0; i0 < nv; i0 += 8) {
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const int nb = nv - i0 < 8 ? nv - i0 : 8;
        for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < NS; idx += stride) {
            const int kx = (int)(idx / ny);
            const double wt = half_weight(kx, nx);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const cpx<double> a = w[c * NS + idx];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    if (k < nb) {
                        const cpx<double> v = V[(size_t)(i0 + k) * vstride + c * NS + idx];
                        acc[k] += wt * (a.re * v.re + a.im * v.im);
                    }
                }
            }
        }
        block_sum<8>(acc, red);
        if (threadIdx.x == 0)
            for (int k = 0; k < nb; ++k) part[(size_t)blockIdx.x * nv + i0 + k] = acc[k];
    }
}

// out[i] = scale * sum over blocks of part[b * nv + i] (fixed order), one block.
__global__ void __launch_bounds__(256) k_S_multidot_finish(const double* __restrict__ part, int nblocks, int nv,
                                                           double scale, double* __restrict__ out,
                                                           const SolveScal* stop) {
    if (gmres_stopped(stop)) return;
    __shared__ double red[16];
    for (int i = 0; i < nv; ++i) {
        double v[1] = {0.0};
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v[0] += part[(size_t)b * nv + i];
        block_sum<1>(v, red);
        if (threadIdx.x == 0) out[i] = scale * v[0];
    }
}

// w += sign sum_i coef[i] V_i (coef in device memory), over n doubles; nv_dev,
// when set, gives the count in device memory instead of nv.
__global__ void k_S_multiaxpy(size_t n, double* __restrict__ w, const double* __restrict__ V, size_t vstride_d,
                              int nv, const double* __restrict__ coef, double sign, const SolveScal* stop,
                              const int* nv_dev) {
    if (gmres_stopped(stop)) return;
    if (nv_dev) nv = *nv_dev;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double s = 0.0;
        for (int k = 0; k < nv; ++k) s += coef[k] * V[(size_t)k * vstride_d + i];
        w[i] += sign * s;
    }
}

// z = A^{-1} v on S fields (Def:A, section 6.1).
template <int D>
__global__ void k_S_precond(int nx, int ny, size_t NS, double tpx, double tpy, double sig, double alp,
                            const cpx<double>* __restrict__ v, cpx<double>* __restrict__ z, const SolveScal* stop) {
    if (gmres_stopped(stop)) return;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < NS; idx += stride) {
        const int kxi = (int)(idx / ny), kyi = (int)(idx - (size_t)kxi * ny);
        const double kx = wavenumber<double>(kxi, nx, tpx);
        const double ky = D == 2 ? wavenumber<double>(kyi, ny, tpy) : 0.0;
        cpx<double> r[D], zz[D];
#pragma unroll
        for (int c = 0; c < D; ++c) r[c] = v[c * NS + idx];
        precond_mode<double, D>(kx, ky, sig, alp, r, zz);
#pragma unroll
        for (int c = 0; c < D; ++c) z[c * NS + idx] = zz[c];
    }
}

// y = scale[0] x over n doubles (the scale in device memory).
__global__ void k_S_scale(size_t n, const double* __restrict__ scale, const double* __restrict__ x,
                          double* __restrict__ y, const SolveScal* stop) {
    if (gmres_stopped(stop)) return;
    const double a = *scale;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = a * x[i];
}

// State of a restarted GMRES(m) solve kept on the device: the Hessenberg
// matrix of the running cycle reduced by Givens rotations, and the stop logic,
// so that the host reads it back once per few Arnoldi steps.
struct GmresCtl {
    double thr;       // tol ||b||
    double bnorm;
    double beta;      // ||r|| at the start of the running cycle
    double relres;    // beta / ||b||
    double scale;     // normalisation of the next basis vector (1 / beta, then 1 / h_{j+1,j})
    int jd;           // columns of the running cycle
    int iters, max_iter;
    int final_;       // 1: no further cycle (converged, max_iter reached or bad data)
    int conv, status; // status -2: non-finite data
};

// Hessenberg storage of a cycle of m steps: H (m + 1) x m by rows, cs, sn (m),
// g (m + 1), y (m) in one array.
__host__ __device__ inline size_t gmres_hess_doubles(int m) {
    return (size_t)(m + 1) * m + 2 * (size_t)m + (size_t)(m + 1) + (size_t)m;
}

__global__ void k_gmres_init(GmresCtl* ctl, double thr, double bnorm, int max_iter) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    ctl->thr = thr;
    ctl->bnorm = bnorm;
    ctl->beta = 0.0;
    ctl->relres = 0.0;
    ctl->scale = 1.0;
    ctl->jd = 0;
    ctl->iters = 0;
    ctl->max_iter = max_iter;
    ctl->final_ = 0;
    ctl->conv = 0;
    ctl->status = 0;
}

// Open a cycle: the operator passes run again (done = 0) unless the solve is over.
__global__ void k_gmres_open(const GmresCtl* ctl, SolveScal* sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) sc->done = ctl->final_ ? 1 : 0;
}

// Start of a cycle from rr = ||r||^2 of the true residual (in V_0): the stop
// tests of the restart (||r|| <= thr: converged; max_iter reached; non-finite),
// else g = (beta, 0, ...) and V_0 is scaled by 1 / beta.
__global__ void k_gmres_begin(GmresCtl* ctl, SolveScal* sc, const double* __restrict__ rr, double* __restrict__ hs,
                              int m) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double beta = sqrt(fmax(*rr, 0.0));
    ctl->beta = beta;
    ctl->relres = beta / ctl->bnorm;
    ctl->jd = 0;
    bool stop = false;
    if (!isfinite(beta)) {
        ctl->status = -2;
        stop = true;
    } else if (beta <= ctl->thr) {
        ctl->conv = 1;
        stop = true;
    } else if (ctl->iters >= ctl->max_iter) {
        stop = true;
    }
    if (stop) {
        ctl->final_ = 1;
        sc->done = 1;
        return;
    }
    double* g = hs + (size_t)(m + 1) * m + 2 * (size_t)m;
    for (int i = 0; i <= m; ++i) g[i] = 0.0;
    g[0] = beta;
    ctl->scale = 1.0 / beta;
    sc->done = 0;
}

// Arnoldi step j: column j of H from the two Gram-Schmidt passes (h1 + h2) and
// h_{j+1,j} = ||w||, the earlier rotations applied to it, the new rotation
// that zeroes h_{j+1,j}, and the residual estimate |g_{j+1}|; the cycle ends
// (done) when that estimate reaches thr, at max_iter, or after step m - 1.
__global__ void k_gmres_givens(int j, int m, const double* __restrict__ coef, double* __restrict__ hs,
                               GmresCtl* ctl, SolveScal* sc) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || sc->done) return;
    double* H = hs;
    double* cs = hs + (size_t)(m + 1) * m;
    double* sn = cs + m;
    double* g = sn + m;
    const double* h1 = coef;
    const double* h2 = coef + (m + 1);
    for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h1[i] + h2[i];
    const double hn = sqrt(fmax(coef[2 * (m + 1)], 0.0));
    ctl->iters += 1;
    if (!isfinite(hn)) {
        ctl->status = -2;
        ctl->final_ = 1;
        sc->done = 1;
        return;
    }
    H[(size_t)(j + 1) * m + j] = hn;
    ctl->scale = hn != 0.0 ? 1.0 / hn : 1.0;
    for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
    }
    const double hjj = H[(size_t)j * m + j];
    const double den = hypot(hjj, hn);
    cs[j] = hjj / den;
    sn[j] = hn / den;
    H[(size_t)j * m + j] = den;
    H[(size_t)(j + 1) * m + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    ctl->jd = j + 1;
    if (fabs(g[j + 1]) <= ctl->thr || ctl->iters >= ctl->max_iter || j + 1 >= m) sc->done = 1;
}

// y = R^{-1} g over the cycle's jd columns (back substitution).
__global__ void k_gmres_backsolve(int m, const GmresCtl* ctl, double* __restrict__ hs) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double* H = hs;
    const double* g = hs + (size_t)(m + 1) * m + 2 * (size_t)m;
    double* y = hs + (size_t)(m + 1) * m + 2 * (size_t)m + (m + 1);
    const int jd = ctl->status == 0 ? ctl->jd : 0;
    for (int i = jd - 1; i >= 0; --i) {
        double t = g[i];
        for (int k = i + 1; k < jd; ++k) t -= H[(size_t)i * m + k] * y[k];
        y[i] = t / H[(size_t)i * m + i];
    }
}

}  // namespace sgn
