// Device code of the p-multigrid CGKS cycle for gfx950.  Included once, by
// cgks_api.hip.
//
// Layout: every per-cell array is structure-of-arrays over the batch's
// concatenated library cell order, [component][NC]; per-face arrays are
// [component][NF]; per-Gauss-point arrays [component][NG].  Indices are
// int32.  One thread per cell, face or Gauss point; all gathers follow a
// fixed slot order, so every result is bitwise reproducible run to run (no
// floating-point atomics anywhere).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <type_traits>

namespace cgks {

constexpr int kBlock = 256;

struct DevParams {
    double gamma;
    int32_t active;    // 0: the case is frozen (finished), kernels leave it untouched
    int32_t scheme;    // 0 S2O4, 1 S1O2
    // (gamma and active share the first 16 bytes: a gather kernel reads them
    // with one load, so the flag arrives with the value its arithmetic needs)
    double mu, Pr, T_wall;
    double W_inf[5];
    double cfl_high, cfl_low, dt_fixed;
    double K;          // internal degrees of freedom of the gas
    int32_t explicit_only;
    int32_t low_flux;  // 0 KFVS, 1 Lax-Friedrichs (low-order level)
    int32_t flux_full; // 1: full time-dependent gas-kinetic solution (discontinuities)
    int32_t pad_;
    double weno_eps;   // > 0: nonlinear reconstruction weights with this epsilon
    // per-case constants of the flux, set on the host: 1 / (K + D) and the
    // Prandtl correction's factor (1/Pr - 1) (-mu gamma / (gamma - 1)) of the
    // normal temperature derivative (0 when Pr = 1 or mu = 0)
    double invN, qcoef;
};
static_assert(offsetof(DevParams, active) == 8, "gamma and active in the first 16 bytes");

// gamma and the active flag of a case with one 16-byte load
__device__ __forceinline__ void gamma_active(const DevParams &P, double &gamma, bool &active) {
    const int4 g = *reinterpret_cast<const int4 *>(&P);
    gamma = __longlong_as_double((long long)(unsigned(g.x)) | ((long long)g.y << 32));
    active = g.z != 0;
}

struct Dev {
    int32_t NC, NF, NG, NB;   // NB >= 1 (array extent); NB_real boundary faces
    int32_t NB_real;
    // cells: cell-major records (Rec<D>) for everything gathered from
    // neighbours, SoA [component][NC] for what only the cell itself reads
    double *st;               // [NC][sr]: W (nv), grad W [axis][v]
    const double *geo;        // [NC][gr]: centroid (D), central second moments (nq), h
    double *ev;               // [NC][er]: centroid, 1/h, <phi_quad>, W, coefficients [k][v]
    float *ev32;              // the same records in FP32 (mixed-precision batches)
    double *Wn, *L0, *Lt0, *G0;
    const double *vol, *h, *minv;
    const float *minv32;      // FP32 copy of minv (mixed-precision batches)
    const int2 *slot;         // [ns][NC]: (x) face code +-(f + 1), 0 = none; (y) neighbour cell or -1
    const int32_t *cell_case;
    // faces
    const int32_t *fL, *fR, *fbc, *fcase, *bslot;
    const int2 *gp_rng;       // [NF] Gauss points [x, y) of each face
    const double *avec, *S, *shift, *gavg;
    const int32_t *bface;     // [NB] face of each boundary slot
    double *gdat;             // [NB][nv + D nv] ghost cell average and gradient
    // gauss points
    const double *gx, *gn, *gw;
    double *fsum;      // per face [NF][Dim<D>::fs]: sum_g wJ of (F0, Ft), then the Gauss-Green groups (Dim<D>)
    float *fsum32;     // the same in FP32 (mixed-precision batches)
    // low level: U and dU in one cell-major record per cell (LowRec: U in
    // FP64, then dU in the sweep precision; a neighbour gather reads one
    // record), Sf, RHS, R1 [nv][NC]
    double *U, *Sf, *RHS, *D, *R1;
    double *lowf;      // [NF][nv]: S_f F_kfvs
    double *swp;       // [NF][4]: area vector S_f n_f (D values, set at upload), S_f lam_f (each low-level step)
    // per case
    const DevParams *prm;
    double *dt, *res;
    double *force;     // per case [3]: wall force (reduced from wallf on request)
    double *wallf;     // per boundary slot [3]: sum_g wJ F0 momentum of the latest stage-0 pass (wall faces)
    const int2 *case_b;          // per case: first boundary slot, count
    int32_t *flag;     // per case: bit 0 non-physical state met
    // reductions
    const int32_t *rb_start, *rb_count, *rb_case, *case_rb_off;
    double *part0, *part1;
};

template <int D> struct Dim;

// Single-use streams (a cell's own operator and stage arrays, whole-line
// record writes): non-temporal loads and stores, which leave L2 to the
// records that neighbours read again.  Not for scattered partial-line
// writes (the face sums), where they cost far more than they save.
template <typename T> __device__ __forceinline__ T ld_nt(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T> __device__ __forceinline__ void st_nt(T v, T *p) { __builtin_nontemporal_store(v, p); }

// precision-dependent arrays of the high-order pass
template <typename R> struct HoArrays;
template <> struct HoArrays<double> {
    static __device__ __forceinline__ double *ev(const Dev &d) { return d.ev; }
    static __device__ __forceinline__ double *fsum(const Dev &d) { return d.fsum; }
    static __device__ __forceinline__ const double *minv(const Dev &d) { return d.minv; }
};
template <> struct HoArrays<float> {
    static __device__ __forceinline__ float *ev(const Dev &d) { return d.ev32; }
    static __device__ __forceinline__ float *fsum(const Dev &d) { return d.fsum32; }
    static __device__ __forceinline__ const float *minv(const Dev &d) { return d.minv32; }
};

// record layouts of the cell-major arrays
template <int D> struct Rec {
    static constexpr int nv = D + 2, nk = D == 2 ? 5 : 9, nq = D == 2 ? 3 : 6;
    static constexpr int sr = nv + D * nv;            // W, grad W
    static constexpr int gr = D + nq + 1;             // centroid, second moments, h
    static constexpr int OW = D + 1 + nq;             // offset of W in the evaluation record
    static constexpr int OC = OW + nv;                // offset of the coefficients
    static constexpr int er = OC + nk * nv;
};

template <int D> struct Dim {
    static constexpr int nv = D + 2;
    static constexpr int nk = D == 2 ? 5 : 9;
    static constexpr int nq = D == 2 ? 3 : 6;
    static constexpr int ns = D == 2 ? 4 : 8;   // slots per cell
    static constexpr int nsym = nk * (nk + 1) / 2;
    static constexpr int lanes = D == 2 ? 2 : 4;   // threads per face (one per Gauss point)
    static constexpr int sl = 4;                   // threads per cell in the slot gathers
    // face record: F0, Ft (2 nv), then the Gauss-Green sums.  Any face: one
    // group per axis (sum w W n_a, sum w W_t n_a).  A planar face (every
    // Gauss point has the same normal): one plain group (sum w W, sum w W_t)
    // in the first group's place and the face normal after it, where the
    // second group would be; the cell kernel multiplies by the normal
    static constexpr int fg = 2 * nv;                // Gauss-Green groups offset
    static constexpr int fh = 4 * nv;                // normal offset (planar faces)
    static constexpr int fs = fg + 2 * D * nv;       // record size (a planar face uses 4 nv + D)
};
// planar faces are marked on the host in the face tag (the boundary tag is
// in the low three bits) and in the slot codes (bit 30 of |code|, below the
// sign that gives the face's orientation seen from the cell)
constexpr int kFacePlanar = 8;
constexpr int kSlotPlanar = 1 << 30;
__device__ __forceinline__ int slot_face(int code) { return ((code > 0 ? code : -code) & (kSlotPlanar - 1)) - 1; }
__device__ __forceinline__ bool slot_planar(int code) { return ((code > 0 ? code : -code) & kSlotPlanar) != 0; }

// quadratic basis (a, b) pairs: 2-D (00, 01, 11); 3-D (00, 11, 22, 01, 02, 12)
template <int D> __device__ __forceinline__ int qa(int q) {
    if (D == 2) return q == 2 ? 1 : 0;
    return q < 3 ? q : (q == 5 ? 1 : 0);
}
template <int D> __device__ __forceinline__ int qb(int q) {
    if (D == 2) return q == 0 ? 0 : 1;
    return q < 3 ? q : (q == 3 ? 1 : 2);
}
// packed index of the symmetric pair (a, b) in the second-moment arrays
template <int D> __device__ __forceinline__ int sidx(int a, int b) {
    if (a > b) { int t = a; a = b; b = t; }
    if (D == 2) return a + b;
    return a == 0 ? b : (a == 1 ? 2 + b : 5);
}
// packed upper-triangle index of (j, k) in an nk x nk symmetric matrix
template <int D> __device__ __forceinline__ int midx(int j, int k) {
    if (j > k) { int t = j; j = k; k = t; }
    return j * Dim<D>::nk - (j * (j - 1)) / 2 + (k - j);
}

// ---------------------------------------------------------------------
// Local face frame (n, t1, t2): an orthonormal basis built without
// branches on the normal (Duff et al., "Building an orthonormal basis,
// revisited", 2017).  The flux is frame invariant.
// ---------------------------------------------------------------------
template <int D, typename R> struct Frame {
    R e[D][D];
    __device__ __forceinline__ void build(const R *n) {
        if constexpr (D == 2) {
            e[0][0] = n[0]; e[0][1] = n[1];
            e[1][0] = -n[1]; e[1][1] = n[0];
        } else {
            const R s = copysign(R(1.0), n[2]);
            const R a = -R(1.0) / (s + n[2]);
            const R b = n[0] * n[1] * a;
            e[0][0] = n[0]; e[0][1] = n[1]; e[0][2] = n[2];
            e[1][0] = R(1.0) + s * n[0] * n[0] * a; e[1][1] = s * b; e[1][2] = -s * n[0];
            e[2][0] = b; e[2][1] = s + n[1] * n[1] * a; e[2][2] = -n[1];
        }
    }
    // vector components of a state (momentum) global -> local
    __device__ __forceinline__ void to_local(const R *W, R *Wl) const {
        constexpr int nv = D + 2;
        Wl[0] = W[0];
        Wl[nv - 1] = W[nv - 1];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            R s = 0;
#pragma unroll
            for (int b = 0; b < D; ++b) s += e[a][b] * W[1 + b];
            Wl[1 + a] = s;
        }
    }
    __device__ __forceinline__ void to_global(const R *Wl, R *W) const {
        constexpr int nv = D + 2;
        W[0] = Wl[0];
        W[nv - 1] = Wl[nv - 1];
#pragma unroll
        for (int b = 0; b < D; ++b) {
            R s = 0;
#pragma unroll
            for (int a = 0; a < D; ++a) s += e[a][b] * Wl[1 + a];
            W[1 + b] = s;
        }
    }
    // gradient G[axis][v] global -> derivatives along local axes of local components
    __device__ __forceinline__ void grad_to_local(const R G[D][D + 2], R Gl[D][D + 2]) const {
        constexpr int nv = D + 2;
        R T[D][nv];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int v = 0; v < nv; ++v) {
                R s = 0;
#pragma unroll
                for (int b = 0; b < D; ++b) s += e[a][b] * G[b][v];
                T[a][v] = s;
            }
#pragma unroll
        for (int a = 0; a < D; ++a) to_local(T[a], Gl[a]);
    }
};

// ---------------------------------------------------------------------
// Moments of the Maxwellian in central form.  With c = u - U (local
// frame) and s = (|c|^2 + xi^2) / 2 the moment vectors psi = (1, u, E-term)
// and psi_c = (1, c, s) are related by psi = M psi_c:
//   psi_0 = 1,  psi_k = U_k + c_k,  psi_E = |U|^2/2 + U.c + s.
// Under the Maxwellian c is Gaussian with variance theta = 1/(2 lam) per
// component, so odd central moments vanish and the even ones needed here
// are closed forms in theta and N = K + D (Isserlis' theorem):
//   E[c_j c_k] = theta d_jk,  E[s] = N theta/2,  E[c_j c_k s] = d_jk theta^2 (N+2)/2,
//   E[s^2] = N (N+2) theta^2/4,  E[c_j c_k s^2] = d_jk theta^3 (N+2)(N+4)/4.
// A micro-slope a.psi whose moments <a psi> = g are given is, in central
// form, alpha_0 + alpha.c + a_E s with
//   g_c = M^-1 g,  alpha_k theta = g_ck,
//   a_E = 2 g_cs / (N theta^2) - g_c0 / theta,  alpha_0 = g_c0 - a_E N theta/2,
// and every product moment the flux needs reduces to g_c (below), so the
// slopes never have to be formed explicitly.
// ---------------------------------------------------------------------

// x_c = M^-1 x (u2h = |U|^2 / 2)
template <int D, typename R> __device__ __forceinline__ void to_central(const R *x, const R *U, R u2h, R *xc) {
    R ux = 0;
    xc[0] = x[0];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        xc[1 + k] = x[1 + k] - U[k] * x[0];
        ux += U[k] * x[1 + k];
    }
    xc[D + 1] = x[D + 1] - ux + u2h * x[0];
}

// x = M x_c, scaled by rho
template <int D, typename R> __device__ __forceinline__ void from_central(const R *xc, const R *U, R u2h, R rho, R *x) {
    R ux = 0;
    x[0] = rho * xc[0];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        x[1 + k] = rho * (xc[1 + k] + U[k] * xc[0]);
        ux += U[k] * xc[1 + k];
    }
    x[D + 1] = rho * (xc[D + 1] + ux + u2h * xc[0]);
}

// primitive variables of a local-frame state
// 1/x from the hardware reciprocal estimate refined by Newton's iteration
// for the reciprocal, r <- r + r (1 - x r) with a fused multiply-add (each
// step doubles the correct bits; two steps in double, one in single).  For
// the positive normal-range quantities of a state (density, pressure,
// temperature); a non-physical state is discarded by its caller anyway.
template <typename R> __device__ __forceinline__ R recip(R x);
template <> __device__ __forceinline__ double recip<double>(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
template <> __device__ __forceinline__ float recip<float>(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

template <int D, typename R> struct Prim {
    R rho, U[D], p, lam, ir, th;   // ir = 1 / rho, th = p / rho = 1 / (2 lam)
    __device__ __forceinline__ void from(const R *W, R gamma) {
        rho = W[0];
        ir = recip<R>(rho);
        R ke = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            U[a] = W[1 + a] * ir;
            ke += U[a] * U[a];
        }
        p = (gamma - R(1.0)) * (W[D + 1] - R(0.5) * rho * ke);
        th = p * ir;
        lam = R(0.5) * recip<R>(th);
    }
};

// Smooth-flow gas-kinetic flux (local frame, axis 0 = normal):
//   f = g^c [1 - tau (a.u + A) + A t]
// F0 = flux at t = 0, Ft = its time derivative, Wt = rho <A psi>.
// With the micro-slope a^(j) of direction j (its central moments
// g^(j)_c = M^-1 (grad_j W / rho)) and n = 0 the normal axis:
//   <A psi_c> = b_c = -sum_j E[u_j a^(j) psi_c]
//   sum_j E[u_n u_j a^(j) psi_c] = sum_j (U_n U_j g_c + U_n E[c_j a psi_c]
//                                  + U_j E[c_n a psi_c] + E[c_n c_j a psi_c])
//   E[c_n c_j a psi_c] = (d_nj c1 g_cs,
//                         theta (d_nj g_ck + d_nk g_cj + d_jk g_cn),
//                         d_nj c2 (2 c1 g_cs - theta g_c0))
// F0 = rho M (E[u_n psi_c] - tau (sum_j E[u_n u_j a psi_c] + E[u_n A psi_c])),
// Ft = rho M E[u_n A psi_c], Wt = rho M b_c.
// Returns false for a non-physical interface state.
template <int D, typename R> __device__ bool gks_flux(const R *Wc, const R Gc[D][D + 2], const DevParams &P, R *F0,
                                          R *Ft, R *Wt) {
    constexpr int nv = D + 2, S = D + 1;
    Prim<D, R> q;
    q.from(Wc, R(P.gamma));
    if (!(q.rho > R(0.0)) || !(q.p > R(0.0))) return false;
    const R N = R(P.K) + D;
    // Fourier heat flux of the interface state along the normal (R = 1,
    // T = p / rho), used for the Prandtl-number correction
    R qcorr = R(0.0);
    if (P.qcoef != 0.0) {
        R ke = 0, ked = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            ke += q.U[k] * q.U[k];
            ked += q.U[k] * Gc[0][1 + k];
        }
        const R pn = (R(P.gamma) - R(1.0)) * (Gc[0][nv - 1] - ked + R(0.5) * ke * Gc[0][0]);
        const R Tn = (pn * q.rho - q.p * Gc[0][0]) * (q.ir * q.ir);
        qcorr = R(P.qcoef) * Tn;
    }
    const R ir = q.ir;
    const R th = q.th;                          // theta = 1 / (2 lam)
    const R tau = R(P.mu) * (R(2.0) * q.lam * ir);   // mu / p
    const R c1 = R(2.0) * R(P.invN), c2 = R(0.5) * th * (N + R(2.0));
    R u2h = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) u2h += q.U[k] * q.U[k];
    u2h *= R(0.5);
    const R Un = q.U[0];
    R bc[nv], tc[nv];
#pragma unroll
    for (int v = 0; v < nv; ++v) bc[v] = tc[v] = R(0.0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
        R g[nv], gc[nv];
#pragma unroll
        for (int v = 0; v < nv; ++v) g[v] = Gc[j][v] * ir;
        to_central<D, R>(g, q.U, u2h, gc);
        const R Uj = q.U[j];
        // E[c_j a psi_c] = (g_cj, d_jk c1 g_cs, c2 g_cj), c1 = 2/N,
        // c2 = theta (N+2)/2; the same with j = n; E[u_j a psi_c] = U_j g_c + rj
        R rj[nv], rn[nv];
#pragma unroll
        for (int v = 0; v < nv; ++v) rj[v] = rn[v] = R(0.0);
        rj[0] = gc[1 + j];
        rj[1 + j] = c1 * gc[S];
        rj[S] = c2 * gc[1 + j];
        rn[0] = gc[1];
        rn[1] = c1 * gc[S];
        rn[S] = c2 * gc[1];
        // E[c_n c_j a psi_c]
        R sj[nv];
#pragma unroll
        for (int v = 0; v < nv; ++v) sj[v] = R(0.0);
        if (j == 0) {
            sj[0] = c1 * gc[S];
            sj[S] = c2 * (R(2.0) * c1 * gc[S] - th * gc[0]);
#pragma unroll
            for (int k = 0; k < D; ++k) sj[1 + k] = th * gc[1 + k];
            sj[1] += th * R(2.0) * gc[1];
        } else {
            sj[1] = th * gc[1 + j];
            sj[1 + j] = th * gc[1];
        }
        const R UnUj = Un * Uj;
#pragma unroll
        for (int v = 0; v < nv; ++v) {
            bc[v] -= Uj * gc[v] + rj[v];
            tc[v] += UnUj * gc[v] + Un * rj[v] + Uj * rn[v] + sj[v];
        }
    }
    // E[u_n A psi_c] for the slope A with central moments b_c
    R ea[nv], fc[nv];
#pragma unroll
    for (int v = 0; v < nv; ++v) ea[v] = Un * bc[v];
    ea[0] += bc[1];
    ea[1] += c1 * bc[S];
    ea[S] += c2 * bc[1];
    // E[u_n psi_c] = (U_n, theta d_nk, U_n N theta / 2)
#pragma unroll
    for (int v = 0; v < nv; ++v) fc[v] = -tau * (tc[v] + ea[v]);
    fc[0] += Un;
    fc[1] += th;
    fc[S] += R(0.5) * Un * N * th;
    from_central<D, R>(fc, q.U, u2h, q.rho, F0);
    from_central<D, R>(ea, q.U, u2h, q.rho, Ft);
    from_central<D, R>(bc, q.U, u2h, q.rho, Wt);
    F0[nv - 1] += qcorr;
    return true;
}

// Maclaurin coefficients of erf, (-1)^n / (n! (2n + 1)) (Abramowitz and
// Stegun 7.1.5), folded to constants at compile time
__host__ __device__ constexpr double erf_series_coef(int n) {
    double f = 1.0;
    for (int k = 2; k <= n; ++k) f *= k;
    return (n % 2 ? -1.0 : 1.0) / (f * (2 * n + 1));
}

// 1 + erf(y) = erfc(-y).  For |y| <= 1/2 the first term left out of twelve
// is below 1e-17 of the leading one (double rounding), the first left out
// of seven below 1e-9 (single); larger |y| take the library erfc.
template <typename R> __device__ __forceinline__ R one_plus_erf(R y) {
    constexpr int nt = sizeof(R) == 8 ? 12 : 7;
    if (fabs(y) <= R(0.5)) {
        const R y2 = y * y;
        R s = R(erf_series_coef(nt - 1));
#pragma unroll
        for (int n = nt - 2; n >= 0; --n) s = s * y2 + R(erf_series_coef(n));
        return R(1.0) + R(1.1283791670955126) * y * s;   // 2 / sqrt(pi)
    }
    return erfc(-y);
}

// half-range moments <u^k>_{u >< 0}, k = 0..3
template <typename R> __device__ __forceinline__ void half_moments(R U, R lam, R th, R sgn, R *m) {
    const R hl = th;   // 1/(2 lam)
    m[0] = R(0.5) * one_plus_erf<R>(sgn * sqrt(lam) * U);
    m[1] = U * m[0] + sgn * R(0.5) * exp(-lam * U * U) * rsqrt(R(M_PI) * lam);
    m[2] = U * m[1] + hl * m[0];
    m[3] = U * m[2] + R(2.0) * hl * m[1];
}

// accumulate rho <psi>_{half} (state) and rho <u psi>_{half} (flux) of one side
template <int D, typename R> __device__ __forceinline__ bool half_side(const R *W, const DevParams &P, R sgn,
                                                           R *Wacc, R *Facc) {
    constexpr int nv = D + 2;
    Prim<D, R> q;
    q.from(W, R(P.gamma));
    if (!(q.rho > R(0.0)) || !(q.p > R(0.0))) return false;
    R m[4];
    half_moments<R>(q.U[0], q.lam, q.th, sgn, m);
    R ut2 = 0;
#pragma unroll
    for (int a = 1; a < D; ++a) ut2 += q.U[a] * q.U[a];
    const R rest = ut2 + (R(P.K) + D - 1) * q.th;   // <v^2> + <w^2> + <xi^2>
    if (Wacc) {
        Wacc[0] += q.rho * m[0];
        Wacc[1] += q.rho * m[1];
#pragma unroll
        for (int a = 1; a < D; ++a) Wacc[1 + a] += q.rho * m[0] * q.U[a];
        Wacc[nv - 1] += R(0.5) * q.rho * (m[2] + m[0] * rest);
    }
    if (Facc) {
        Facc[0] += q.rho * m[1];
        Facc[1] += q.rho * m[2];
#pragma unroll
        for (int a = 1; a < D; ++a) Facc[1 + a] += q.rho * m[1] * q.U[a];
        Facc[nv - 1] += R(0.5) * q.rho * (m[3] + m[1] * rest);
    }
    return true;
}

// ---------------------------------------------------------------------
// Full time-dependent gas-kinetic solution (the 2nd-flux equation of
// Sec. 2.2, for flows with discontinuities):
//   f(t) = (1 - e) g^c + [(t + tau) e - tau] (a^c.u) g^c + (t - tau + tau e) A^c g^c
//        + e g^l [1 - (tau + t) a^l.u - tau A^l] H(u) + e g^r [...] (1 - H(u)),
// e = exp(-t / tau_n), tau_n = tau + |p_l - p_r| / (p_l + p_r) dt.  The
// equilibrium part reuses the central-moment algebra of gks_flux.  The
// left and right parts need half-range moments in the normal velocity u,
// where odd central moments no longer vanish, so their micro-slopes are
// formed explicitly in the raw basis psi = (1, u, v, w, (|u|^2 + Z)/2)
// (Z = xi^2) and every expectation is expanded over monomials
// u^a v^b w^c Z^e: the normal part uses the half-range moments of u, the
// tangential velocities and Z their full Gaussian moments.
// ---------------------------------------------------------------------

// monomials u^a v^b w^c Z^e of psi_p, with their coefficients
template <int D> struct PsiTerms;
template <> struct PsiTerms<3> {
    static constexpr int n[5] = {1, 1, 1, 1, 4};
    static constexpr int m[5][4][4] = {{{0, 0, 0, 0}}, {{1, 0, 0, 0}}, {{0, 1, 0, 0}}, {{0, 0, 1, 0}},
                                       {{2, 0, 0, 0}, {0, 2, 0, 0}, {0, 0, 2, 0}, {0, 0, 0, 1}}};
    static constexpr double k[5][4] = {{1.0}, {1.0}, {1.0}, {1.0}, {0.5, 0.5, 0.5, 0.5}};
};
template <> struct PsiTerms<2> {
    static constexpr int n[4] = {1, 1, 1, 3};
    static constexpr int m[4][4][4] = {{{0, 0, 0, 0}}, {{1, 0, 0, 0}}, {{0, 1, 0, 0}},
                                       {{2, 0, 0, 0}, {0, 2, 0, 0}, {0, 0, 0, 1}}};
    static constexpr double k[4][4] = {{1.0}, {1.0}, {1.0}, {0.5, 0.5, 0.5}};
};

// the central-moment coefficients (alpha_0, alpha, a_E) of a slope whose
// central moments are gc, turned into raw psi coefficients
template <int D, typename R>
__device__ __forceinline__ void central_to_raw(const R *gc, const R *U, R u2h, R th, R N, R *raw) {
    constexpr int S = D + 1;
    const R it = R(1.0) / th;
    const R aE = R(2.0) * gc[S] * it * it / N - gc[0] * it;
    R a0 = gc[0] - aE * N * th * R(0.5), aU = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const R al = gc[1 + k] * it;
        aU += al * U[k];
        raw[1 + k] = al - aE * U[k];
    }
    raw[0] = a0 - aU + aE * u2h;
    raw[S] = aE;
}

// One side (sgn = +1: u > 0, left; -1: u < 0, right) of the full
// solution's free-transport part: accumulates rho <w psi>, rho <w psi a.u>
// and rho <w psi A> over the half space for w = u (flux: Fg, Fa, FA) and
// w = 1 (state: Wg, Wa, WA).  W, G: state and gradient [axis][v] in the
// face frame.  Returns false for a non-physical state.
template <int D, typename R>
__device__ bool half_side_full(const R *W, const R G[D][D + 2], const DevParams &P, R sgn, R *Fg, R *Fa, R *FA,
                               R *Wg, R *Wa, R *WA) {
    constexpr int nv = D + 2, S = D + 1;
    using PT = PsiTerms<D>;
    Prim<D, R> q;
    q.from(W, R(P.gamma));
    if (!(q.rho > R(0.0)) || !(q.p > R(0.0))) return false;
    const R N = R(P.K) + D, ir = q.ir, th = q.th;
    const R c1 = R(2.0) * R(P.invN), c2 = R(0.5) * th * (N + R(2.0));
    R u2h = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) u2h += q.U[k] * q.U[k];
    u2h *= R(0.5);
    // raw micro-slopes a^(j) of the three axes and A (compatibility over
    // the whole velocity space, as on the smooth path)
    R a[D][nv], bc[nv], A[nv];
#pragma unroll
    for (int v = 0; v < nv; ++v) bc[v] = R(0.0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
        R g[nv], gc[nv];
#pragma unroll
        for (int v = 0; v < nv; ++v) g[v] = G[j][v] * ir;
        to_central<D, R>(g, q.U, u2h, gc);
        central_to_raw<D, R>(gc, q.U, u2h, th, N, a[j]);
        R rj[nv];
#pragma unroll
        for (int v = 0; v < nv; ++v) rj[v] = R(0.0);
        rj[0] = gc[1 + j];
        rj[1 + j] = c1 * gc[S];
        rj[S] = c2 * gc[1 + j];
#pragma unroll
        for (int v = 0; v < nv; ++v) bc[v] -= q.U[j] * gc[v] + rj[v];
    }
    central_to_raw<D, R>(bc, q.U, u2h, th, N, A);
    // moments: u over the half space, v, w over the whole line, Z
    R Hu[7], Mv[6], Mw[6], MZ[3];
    const R var = q.th;   // variance of each velocity component: 1 / (2 lam)
    Hu[0] = R(0.5) * one_plus_erf<R>(sgn * sqrt(q.lam) * q.U[0]);
    Hu[1] = q.U[0] * Hu[0] + sgn * R(0.5) * exp(-q.lam * q.U[0] * q.U[0]) * rsqrt(R(M_PI) * q.lam);
#pragma unroll
    for (int k = 0; k + 2 < 7; ++k) Hu[k + 2] = q.U[0] * Hu[k + 1] + R(k + 1) * var * Hu[k];
    Mv[0] = R(1.0);
    Mv[1] = D > 1 ? q.U[1] : R(0.0);
#pragma unroll
    for (int k = 0; k + 2 < 6; ++k) Mv[k + 2] = Mv[1] * Mv[k + 1] + R(k + 1) * var * Mv[k];
    Mw[0] = R(1.0);
    Mw[1] = D > 2 ? q.U[D - 1] : R(0.0);
#pragma unroll
    for (int k = 0; k + 2 < 6; ++k) Mw[k + 2] = Mw[1] * Mw[k + 1] + R(k + 1) * var * Mw[k];
    MZ[0] = R(1.0);
    MZ[1] = R(P.K) * var;
    MZ[2] = R(P.K) * (R(P.K) + R(2.0)) * var * var;
#define CGKS_EXP(ua, vb, wc, ze) (Hu[ua] * Mv[vb] * Mw[wc] * MZ[ze])
#pragma unroll
    for (int p = 0; p < nv; ++p) {
        R eg[2] = {0, 0}, ea[2] = {0, 0}, eA[2] = {0, 0};   // [w = 1, w = u]
#pragma unroll
        for (int i1 = 0; i1 < PT::n[p]; ++i1) {
            const int pa = PT::m[p][i1][0], pb = PT::m[p][i1][1], pc = PT::m[p][i1][2], pe = PT::m[p][i1][3];
            const R k1 = R(PT::k[p][i1]);
            eg[0] += k1 * CGKS_EXP(pa, pb, pc, pe);
            eg[1] += k1 * CGKS_EXP(pa + 1, pb, pc, pe);
#pragma unroll
            for (int qq = 0; qq < nv; ++qq)
#pragma unroll
                for (int i2 = 0; i2 < PT::n[qq]; ++i2) {
                    const int ua = pa + PT::m[qq][i2][0], vb = pb + PT::m[qq][i2][1];
                    const int wc = pc + PT::m[qq][i2][2], ze = pe + PT::m[qq][i2][3];
                    const R kk = k1 * R(PT::k[qq][i2]);
                    // A psi_q
                    eA[0] += A[qq] * kk * CGKS_EXP(ua, vb, wc, ze);
                    eA[1] += A[qq] * kk * CGKS_EXP(ua + 1, vb, wc, ze);
                    // sum_j a^(j)_q psi_q u_j
                    R s0 = a[0][qq] * CGKS_EXP(ua + 1, vb, wc, ze);
                    R s1 = a[0][qq] * CGKS_EXP(ua + 2, vb, wc, ze);
                    if (D > 1) {
                        s0 += a[1][qq] * CGKS_EXP(ua, vb + 1, wc, ze);
                        s1 += a[1][qq] * CGKS_EXP(ua + 1, vb + 1, wc, ze);
                    }
                    if (D > 2) {
                        s0 += a[D - 1][qq] * CGKS_EXP(ua, vb, wc + 1, ze);
                        s1 += a[D - 1][qq] * CGKS_EXP(ua + 1, vb, wc + 1, ze);
                    }
                    ea[0] += kk * s0;
                    ea[1] += kk * s1;
                }
        }
        Wg[p] += q.rho * eg[0];
        Fg[p] += q.rho * eg[1];
        Wa[p] += q.rho * ea[0];
        Fa[p] += q.rho * ea[1];
        WA[p] += q.rho * eA[0];
        FA[p] += q.rho * eA[1];
    }
#undef CGKS_EXP
    return true;
}

// Equilibrium part of the full solution: rho <w psi>, rho <w psi a.u>,
// rho <w psi A> of g^c for w = u (Fcg, Fca, FcA) and the state slope
// rho <psi A> (WcA; rho <psi a.u> = -WcA by compatibility), from the same
// central-moment algebra as gks_flux.  Returns false for a non-physical
// interface state.
template <int D, typename R>
__device__ bool equilibrium_terms(const R *Wc, const R Gc[D][D + 2], const DevParams &P, R *Fcg, R *Fca, R *FcA,
                                  R *WcA) {
    constexpr int nv = D + 2, S = D + 1;
    Prim<D, R> q;
    q.from(Wc, R(P.gamma));
    if (!(q.rho > R(0.0)) || !(q.p > R(0.0))) return false;
    const R N = R(P.K) + D, ir = q.ir, th = q.th;
    const R c1 = R(2.0) * R(P.invN), c2 = R(0.5) * th * (N + R(2.0));
    R u2h = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) u2h += q.U[k] * q.U[k];
    u2h *= R(0.5);
    const R Un = q.U[0];
    R bc[nv], tc[nv];
#pragma unroll
    for (int v = 0; v < nv; ++v) bc[v] = tc[v] = R(0.0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
        R g[nv], gc[nv];
#pragma unroll
        for (int v = 0; v < nv; ++v) g[v] = Gc[j][v] * ir;
        to_central<D, R>(g, q.U, u2h, gc);
        const R Uj = q.U[j];
        R rj[nv], rn[nv], sj[nv];
#pragma unroll
        for (int v = 0; v < nv; ++v) rj[v] = rn[v] = sj[v] = R(0.0);
        rj[0] = gc[1 + j];
        rj[1 + j] = c1 * gc[S];
        rj[S] = c2 * gc[1 + j];
        rn[0] = gc[1];
        rn[1] = c1 * gc[S];
        rn[S] = c2 * gc[1];
        if (j == 0) {
            sj[0] = c1 * gc[S];
            sj[S] = c2 * (R(2.0) * c1 * gc[S] - th * gc[0]);
#pragma unroll
            for (int k = 0; k < D; ++k) sj[1 + k] = th * gc[1 + k];
            sj[1] += th * R(2.0) * gc[1];
        } else {
            sj[1] = th * gc[1 + j];
            sj[1 + j] = th * gc[1];
        }
#pragma unroll
        for (int v = 0; v < nv; ++v) {
            bc[v] -= Uj * gc[v] + rj[v];
            tc[v] += Un * Uj * gc[v] + Un * rj[v] + Uj * rn[v] + sj[v];
        }
    }
    R ea[nv], eu[nv];
#pragma unroll
    for (int v = 0; v < nv; ++v) {
        ea[v] = Un * bc[v];
        eu[v] = R(0.0);
    }
    ea[0] += bc[1];
    ea[1] += c1 * bc[S];
    ea[S] += c2 * bc[1];
    eu[0] = Un;
    eu[1] = th;
    eu[S] = R(0.5) * Un * N * th;
    from_central<D, R>(eu, q.U, u2h, q.rho, Fcg);
    from_central<D, R>(tc, q.U, u2h, q.rho, Fca);
    from_central<D, R>(ea, q.U, u2h, q.rho, FcA);
    from_central<D, R>(bc, q.U, u2h, q.rho, WcA);
    return true;
}

// the five time functions of the full solution -- 1 - e, (t + tau) e - tau,
// t - tau + tau e, e, (tau + t) e -- at t = T, or integrated over [0, T]
template <typename R> __device__ __forceinline__ void full_time_weights(R T, R tau, R taun, bool integral, R *w) {
    const R E = taun > R(0.0) ? exp(-T / taun) : R(0.0);
    if (!integral) {
        w[0] = R(1.0) - E;
        w[1] = (T + tau) * E - tau;
        w[2] = T - tau + tau * E;
        w[3] = E;
        w[4] = (tau + T) * E;
        return;
    }
    const R omE = R(1.0) - E;
    w[0] = T - taun * omE;
    w[1] = taun * taun * omE - taun * T * E + tau * taun * omE - tau * T;
    w[2] = R(0.5) * T * T - tau * T + tau * taun * omE;
    w[3] = taun * omE;
    w[4] = tau * taun * omE + taun * taun * omE - taun * T * E;
}

// Full solution at a Gauss point (face frame): flux F0 + t Ft with the
// solution's integrals over [0, dt/2] and [0, dt], interface state W0 + t
// Wt through its values at dt/2 and dt.  WL, GL, WR, GR: left and right
// states and gradients; Wc, Gc: the half-space equilibrium state and the
// mean gradient.  Returns false for a non-physical state.
template <int D, typename R>
__device__ bool gks_flux_full(const R *WL, const R GL[D][D + 2], const R *WR, const R GR[D][D + 2], const R *Wc,
                              const R Gc[D][D + 2], const DevParams &P, R dt, R *F0, R *Ft, R *W0, R *Wt) {
    constexpr int nv = D + 2;
    R Fcg[nv], Fca[nv], FcA[nv], WcA[nv];
    if (!equilibrium_terms<D, R>(Wc, Gc, P, Fcg, Fca, FcA, WcA)) return false;
    R SFg[nv], SFa[nv], SFA[nv], SWg[nv], SWa[nv], SWA[nv];
#pragma unroll
    for (int v = 0; v < nv; ++v) SFg[v] = SFa[v] = SFA[v] = SWg[v] = SWa[v] = SWA[v] = R(0.0);
    __builtin_amdgcn_sched_barrier(0);
    bool ok = half_side_full<D, R>(WL, GL, P, R(1.0), SFg, SFa, SFA, SWg, SWa, SWA);
    __builtin_amdgcn_sched_barrier(0);
    ok = half_side_full<D, R>(WR, GR, P, -R(1.0), SFg, SFa, SFA, SWg, SWa, SWA) && ok;
    if (!ok) return false;
    Prim<D, R> qc, ql, qr;
    qc.from(Wc, R(P.gamma));
    ql.from(WL, R(P.gamma));
    qr.from(WR, R(P.gamma));
    const R tau = R(P.mu) / qc.p;
    const R taun = tau + fabs(ql.p - qr.p) / (ql.p + qr.p) * dt;
    R w[5];
    R I1[nv], I2[nv], V1[nv], V2[nv];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const R T = (k & 1) ? R(0.5) * dt : dt;
        const bool integral = k < 2;
        full_time_weights<R>(T, tau, taun, integral, w);
#pragma unroll
        for (int v = 0; v < nv; ++v) {
            const R out = integral
                ? w[0] * Fcg[v] + w[1] * Fca[v] + w[2] * FcA[v] + w[3] * (SFg[v] - tau * SFA[v]) - w[4] * SFa[v]
                : w[0] * Wc[v] - w[1] * WcA[v] + w[2] * WcA[v] + w[3] * (SWg[v] - tau * SWA[v]) - w[4] * SWa[v];
            if (k == 0) I1[v] = out;
            else if (k == 1) I2[v] = out;
            else if (k == 2) V1[v] = out;
            else V2[v] = out;
        }
    }
    const R idt = R(1.0) / dt;
#pragma unroll
    for (int v = 0; v < nv; ++v) {
        F0[v] = (R(4.0) * I2[v] - I1[v]) * idt;
        Ft[v] = R(4.0) * (I1[v] - R(2.0) * I2[v]) * idt * idt;
        W0[v] = R(2.0) * V2[v] - V1[v];
        Wt[v] = R(2.0) * (V1[v] - V2[v]) * idt;
    }
    if (R(P.Pr) != R(1.0) && R(P.mu) != R(0.0)) {
        R ke = 0, ked = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            ke += qc.U[k] * qc.U[k];
            ked += qc.U[k] * Gc[0][1 + k];
        }
        const R pn = (R(P.gamma) - R(1.0)) * (Gc[0][nv - 1] - ked + R(0.5) * ke * Gc[0][0]);
        const R Tn = (pn * qc.rho - qc.p * Gc[0][0]) / (qc.rho * qc.rho);
        F0[nv - 1] += (R(1.0) / R(P.Pr) - R(1.0)) * (-R(P.mu) * R(P.gamma) / (R(P.gamma) - R(1.0)) * Tn);
    }
    return true;
}

// characteristic far-field state (local frame, axis 0 outward)
template <int D, typename R> __device__ void farfield_state(const R *Wl, const R *Wo, R gamma, R *Wb) {
    constexpr int nv = D + 2;
    Prim<D, R> I, O;
    I.from(Wl, gamma);
    O.from(Wo, gamma);
    const R cI = sqrt(gamma * I.p / I.rho), cO = sqrt(gamma * O.p / O.rho);
    if (O.U[0] <= -cO) {
#pragma unroll
        for (int v = 0; v < nv; ++v) Wb[v] = Wo[v];
        return;
    }
    if (I.U[0] >= cI) {
#pragma unroll
        for (int v = 0; v < nv; ++v) Wb[v] = Wl[v];
        return;
    }
    const R Rp = I.U[0] + R(2.0) * cI / (gamma - R(1.0));
    const R Rm = O.U[0] - R(2.0) * cO / (gamma - R(1.0));
    const R Un = R(0.5) * (Rp + Rm);
    const R c = R(0.25) * (gamma - R(1.0)) * (Rp - Rm);
    const Prim<D, R> &up = Un > 0 ? I : O;
    const R s = up.p / pow(up.rho, gamma);
    const R rho = pow(c * c / (gamma * s), R(1.0) / (gamma - R(1.0)));
    const R p = rho * c * c / gamma;
    R ke = Un * Un;
    Wb[0] = rho;
    Wb[1] = rho * Un;
#pragma unroll
    for (int a = 1; a < D; ++a) {
        Wb[1 + a] = rho * up.U[a];
        ke += up.U[a] * up.U[a];
    }
    Wb[nv - 1] = p / (gamma - R(1.0)) + R(0.5) * rho * ke;
}

// normal Euler flux of U along unit n (global frame)
template <int D> __device__ __forceinline__ void euler_flux(const double *U, const double *n, double gamma, double *F) {
    constexpr int nv = D + 2;
    const double rho = U[0];
    double ke = 0, un = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        ke += U[1 + a] * U[1 + a];
        un += U[1 + a] * n[a];
    }
    const double ir = recip<double>(rho);
    un *= ir;
    const double p = (gamma - 1.0) * (U[nv - 1] - 0.5 * ke * ir);
    F[0] = rho * un;
#pragma unroll
    for (int a = 0; a < D; ++a) F[1 + a] = U[1 + a] * un + p * n[a];
    F[nv - 1] = (U[nv - 1] + p) * un;
}

// The same flux's change F_A(U + dU) - F_A(U), written so that no two large
// terms are subtracted: with u' = (m + dm)/(rho + drho), du = u' - u,
//   d(rho u.A) = dm.A,   d(m u.A) = dm (u'.A) + m (du.A) + dp A,
//   d((E + p) u.A) = (dE + dp)(u'.A) + (E + p)(du.A),
//   dp = (gamma - 1)(dE - (dm.u' + m.du)/2).
// Accurate relative to |dU| in any precision (used by FP32 sweeps).
template <int D, typename S>
__device__ __forceinline__ void euler_dflux(const S *U, const S *dU, const S *A, S gamma, S *dF) {
    constexpr int nv = D + 2;
    const S ir = recip<S>(U[0]), ir1 = recip<S>(U[0] + dU[0]);
    S u[D], du[D], un1 = S(0), dun = S(0), mu = S(0), dmu = S(0), dmA = S(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        u[a] = U[1 + a] * ir;
        du[a] = (dU[1 + a] - u[a] * dU[0]) * ir1;
        un1 += (u[a] + du[a]) * A[a];
        dun += du[a] * A[a];
        mu += U[1 + a] * u[a];
        dmu += dU[1 + a] * (u[a] + du[a]) + U[1 + a] * du[a];
        dmA += dU[1 + a] * A[a];
    }
    const S p = (gamma - S(1)) * (U[nv - 1] - S(0.5) * mu);
    const S dp = (gamma - S(1)) * (dU[nv - 1] - S(0.5) * dmu);
    dF[0] = dmA;
#pragma unroll
    for (int a = 0; a < D; ++a) dF[1 + a] = dU[1 + a] * un1 + U[1 + a] * dun + dp * A[a];
    dF[nv - 1] = (dU[nv - 1] + dp) * un1 + (U[nv - 1] + p) * dun;
}

// Low-level state records, one per cell, [cell][stride] doubles: U (nv
// FP64 values), then dU (nv values in the sweep precision S).  FP64 sweeps:
// stride 2 nv.  FP32 sweeps: nv doubles + nv floats padded to 16 bytes
// (3-D: 64 bytes, one memory sector per neighbour gather).
template <int D, typename S> struct LowRec;
template <int D> struct LowRec<D, double> {
    static constexpr int nv = D + 2, stride = 2 * nv;
    static __device__ __forceinline__ double *U(const Dev &d, size_t i) { return d.U + i * stride; }
    static __device__ __forceinline__ double *dU(const Dev &d, size_t i) { return d.U + i * stride + nv; }
};
template <int D> struct LowRec<D, float> {
    static constexpr int nv = D + 2, stride = (nv + (nv + 1) / 2 + 1) / 2 * 2;
    static __device__ __forceinline__ double *U(const Dev &d, size_t i) { return d.U + i * stride; }
    static __device__ __forceinline__ float *dU(const Dev &d, size_t i) {
        return reinterpret_cast<float *>(d.U + i * stride + nv);
    }
};

// cell i's low-level record set to U = u, dU = 0 by the cell's SL lanes:
// the record's 16-byte pieces go to lane k % SL (U below nv doubles; dU and
// the padding after it are zero bits in either precision)
template <int D, typename S, int SL>
__device__ __forceinline__ void low_rec_reset(const Dev &d, int i, const double *u, int q) {
    constexpr int nv = D + 2, np = LowRec<D, S>::stride / 2;
    double2 *rec = reinterpret_cast<double2 *>(LowRec<D, S>::U(d, i));
#pragma unroll
    for (int r = 0; r < np; r += SL) {
        double2 v = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = r; j < r + SL && j < np; ++j)
            if (q == j - r) v = make_double2(2 * j < nv ? u[2 * j] : 0.0, 2 * j + 1 < nv ? u[2 * j + 1] : 0.0);
        if (r + q < np) rec[r + q] = v;
    }
}

// ---------------------------------------------------------------------
// Global time step: per-block minimum over a case's cells, then per case.
// ---------------------------------------------------------------------
template <int D> __device__ __forceinline__ double state_dt(const double *U, double h, double cfl, const DevParams &P) {
    constexpr int nv = D + 2;
    const double rho = U[0], ir = recip<double>(rho);
    double ke = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double u = U[1 + a] * ir;
        ke += u * u;
    }
    const double p = (P.gamma - 1.0) * (U[nv - 1] - 0.5 * rho * ke);
    const double c = sqrt(P.gamma * p * ir);
    return cfl * h * recip<double>(sqrt(ke) + c + 2.0 * P.mu * ir * recip<double>(h));
}

// The face, cell and sweep kernels take their block size from the launch
// (a multiple of 4 lanes, at most kBlock) so that it can be tuned per batch;
// a thread's work never depends on it.
//
// Workgroups are handed to the 8 XCDs round-robin (block b runs on XCD
// b mod 8), each XCD with its own L2.  xcd_block renumbers the launch so
// that every XCD works through one contiguous range of logical blocks:
// neighbouring cells and faces, which share gathered records, then meet
// in the same L2.  A bijection of [0, nb).
constexpr int kXcd = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b % kXcd, k = b / kXcd, per = nb / kXcd, rem = nb % kXcd;
    return x * per + min(x, rem) + k;
}

__device__ __forceinline__ double block_reduce_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}
__device__ __forceinline__ double block_reduce_min(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] = fmin(sh[t], sh[t + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

template <int D> __global__ __launch_bounds__(kBlock) void k_dt_partial(Dev d) {
    __shared__ double sh[kBlock];
    const int b = blockIdx.x;
    const int c = d.rb_case[b];
    const DevParams &P = d.prm[c];
    const int n = d.rb_count[b];
    double v = INFINITY;
    for (int k = threadIdx.x; k < n; k += kBlock) {
        const int i = d.rb_start[b] + k;
        v = fmin(v, state_dt<D>(d.st + size_t(i) * Rec<D>::sr, d.h[i], P.cfl_high, P));
    }
    v = block_reduce_min(v, sh);
    if (threadIdx.x == 0) d.part0[b] = v;
}

// one block per case: thread t folds the case's block partials t, t + kBlock,
// ... in order, then a block tree; the shape depends only on the case
__global__ __launch_bounds__(kBlock) void k_dt_final(Dev d, int n_case) {
    __shared__ double sh[kBlock];
    const int c = blockIdx.x;
    const DevParams &P = d.prm[c];
    if (!P.active) return;
    double v = INFINITY;
    for (int b = d.case_rb_off[c] + threadIdx.x; b < d.case_rb_off[c + 1]; b += kBlock) v = fmin(v, d.part0[b]);
    v = block_reduce_min(v, sh);
    if (threadIdx.x == 0) d.dt[c] = P.dt_fixed > 0 ? P.dt_fixed : v;
}

// ---------------------------------------------------------------------
// Compact reconstruction: c = (M^T M)^-1 M^T b per cell, with the rows of
// M generated here from the cell geometry (face neighbours, mirror ghosts
// of boundary faces, own gradient) and (M^T M)^-1 precomputed on the host.
// ---------------------------------------------------------------------
template <int D> __device__ __forceinline__ void ghost_data(int bc, const double *n, const double *Wi,
                                                            const double Gi[D][D + 2], const DevParams &P, double *Wg,
                                                            double Gg[D][D + 2]) {
    constexpr int nv = D + 2;
    if (bc == 4) {  // far field
        Frame<D, double> fr;
        fr.build(n);
        double Wl[nv], Wo[nv], Wo_g[nv], Wb[nv];
#pragma unroll
        for (int v = 0; v < nv; ++v) Wo_g[v] = P.W_inf[v];
        fr.to_local(Wi, Wl);
        fr.to_local(Wo_g, Wo);
        farfield_state<D, double>(Wl, Wo, P.gamma, Wb);
        fr.to_global(Wb, Wg);
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int v = 0; v < nv; ++v) Gg[a][v] = 0.0;
        return;
    }
    // slip (M = R on momentum) or no-slip (M = -I on momentum); R = I - 2 n n^T
    const bool slip = bc == 1;
    double R[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) R[a][b] = (a == b ? 1.0 : 0.0) - 2.0 * n[a] * n[b];
    Wg[0] = Wi[0];
    Wg[nv - 1] = Wi[nv - 1];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double s = 0;
#pragma unroll
        for (int b = 0; b < D; ++b) s += (slip ? R[a][b] : (a == b ? -1.0 : 0.0)) * Wi[1 + b];
        Wg[1 + a] = s;
    }
    // MG[b][v] = (M G_i[b])_v, then Gg[a][v] = sum_b R[a][b] MG[b][v]
    double MG[D][nv];
#pragma unroll
    for (int b = 0; b < D; ++b) {
        MG[b][0] = Gi[b][0];
        MG[b][nv - 1] = Gi[b][nv - 1];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double s = 0;
#pragma unroll
            for (int c = 0; c < D; ++c) s += (slip ? R[a][c] : (a == c ? -1.0 : 0.0)) * Gi[b][1 + c];
            MG[b][1 + a] = s;
        }
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int v = 0; v < nv; ++v) {
            double s = 0;
#pragma unroll
            for (int b = 0; b < D; ++b) s += R[a][b] * MG[b][v];
            Gg[a][v] = s;
        }
}

// ghost cell data of every boundary face, from its owner's current state
template <int D> __global__ __launch_bounds__(kBlock) void k_ghost(Dev d) {
    constexpr int nv = D + 2;
    const int B = blockIdx.x * kBlock + threadIdx.x;
    if (B >= d.NB_real) return;
    const int f = d.bface[B];
    if (f < 0 || !d.prm[d.fcase[f]].active) return;
    const int i = d.fL[f];
    const int NC = d.NC;
    const DevParams &P = d.prm[d.fcase[f]];
    double Wi[nv], Gi[D][nv], Wg[nv], Gg[D][nv], n[D];
    const double *si = d.st + size_t(i) * Rec<D>::sr;
#pragma unroll
    for (int v = 0; v < nv; ++v) Wi[v] = si[v];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int v = 0; v < nv; ++v) Gi[a][v] = si[nv + a * nv + v];
    (void)NC;
    const double iS = 1.0 / d.S[f];
#pragma unroll
    for (int a = 0; a < D; ++a) n[a] = d.avec[size_t(a) * d.NF + f] * iS;
    ghost_data<D>(d.fbc[f] & 7, n, Wi, Gi, P, Wg, Gg);
    double *o = d.gdat + size_t(B) * (nv + D * nv);
#pragma unroll
    for (int v = 0; v < nv; ++v) o[v] = Wg[v];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int v = 0; v < nv; ++v) o[nv + a * nv + v] = Gg[a][v];
}

// Nonlinear (WENO-type) weights of the compact reconstruction, for flows
// with discontinuities (Sec. 4 applies them with a small epsilon; their
// form is taken from other work).  Candidates: the quadratic P0 just
// fitted (coefficients c, [k][v]) and, for each face neighbour or ghost m,
// the linear polynomial fitting m's average and h-scaled averaged gradient
// in the least-squares sense, in closed form c_m = g + r (dW - r.g) /
// (1 + |r|^2) with r the scaled centroid offset and g = h grad W_m.  Linear
// weights 0.95 and 0.05 / M; indicators in xi = (x - x_i)/h:
// beta = sum_a <(dP/dxi_a)^2> + sum_{a<=b} (d2P/dxi_a dxi_b)^2; weights
// proportional to gamma / (eps + beta)^2; the result
// omega_0/gamma_0 (P0 - sum gamma_m P_m) + sum omega_m P_m replaces c.
constexpr double kWenoGamma0 = 0.95;
template <int D, typename R>
__device__ void weno_weights(const Dev &d, int i, int NC, const double *xc, double ih, double h, const double *own,
                             const double *Wi, R eps, R *c) {
    using T = Dim<D>;
    using RC = Rec<D>;
    constexpr int nv = T::nv, nq = T::nq;
    // cell second moments in xi and the indicator of P0
    R M[D][D];
#pragma unroll
    for (int q = 0; q < nq; ++q) M[qa<D>(q)][qb<D>(q)] = M[qb<D>(q)][qa<D>(q)] = R(own[q]);
    R beta0[nv];
#pragma unroll
    for (int v = 0; v < nv; ++v) {
        R H[D][D];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = 0; b < D; ++b) H[a][b] = R(0.0);
#pragma unroll
        for (int q = 0; q < nq; ++q) {
            const int a = qa<D>(q), b = qb<D>(q);
            const R cq = c[(D + q) * nv + v];
            if (a == b) H[a][a] += R(2.0) * cq;
            else {
                H[a][b] += cq;
                H[b][a] += cq;
            }
        }
        R bt = R(0.0);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const R ca = c[a * nv + v];
            R quad = R(0.0);
#pragma unroll
            for (int b = 0; b < D; ++b)
#pragma unroll
                for (int b2 = 0; b2 < D; ++b2) quad += H[a][b] * H[a][b2] * M[b][b2];
            bt += ca * ca + quad;
#pragma unroll
            for (int b = a; b < D; ++b) bt += H[a][b] * H[a][b];
        }
        beta0[v] = bt;
    }
    // the linear candidates, one per slot
    R Sw[nv], Sc[D][nv], Sg[D][nv];
#pragma unroll
    for (int v = 0; v < nv; ++v) {
        Sw[v] = R(0.0);
#pragma unroll
        for (int a = 0; a < D; ++a) Sc[a][v] = Sg[a][v] = R(0.0);
    }
    int M_cand = 0;
#pragma unroll 1
    for (int s = 0; s < T::ns; ++s) {
        const int2 sl = d.slot[size_t(s) * NC + i];
        const int code = sl.x;
        if (code == 0) break;
        const int f = slot_face(code);
        const int nb = sl.y;
        R r[D];
        const double *gd;
        if (nb >= 0) {
            const double sg = code > 0 ? 1.0 : -1.0;
            const double *gm = d.geo + size_t(nb) * RC::gr;
#pragma unroll
            for (int a = 0; a < D; ++a) r[a] = R((gm[a] + sg * d.shift[size_t(a) * d.NF + f] - xc[a]) * ih);
            gd = d.st + size_t(nb) * RC::sr;
        } else {
            const int bs = d.bslot[f];
#pragma unroll
            for (int a = 0; a < D; ++a) r[a] = R(d.gavg[size_t(a) * d.NB + bs]);
            gd = d.gdat + size_t(bs) * (nv + D * nv);
        }
        ++M_cand;
        R rr = R(1.0);
#pragma unroll
        for (int a = 0; a < D; ++a) rr += r[a] * r[a];
        const R irr = R(1.0) / rr;
#pragma unroll
        for (int v = 0; v < nv; ++v) {
            R g[D], rg = R(0.0);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                g[a] = R(h * gd[nv + a * nv + v]);
                rg += r[a] * g[a];
            }
            const R t = (R(gd[v] - Wi[v]) - rg) * irr;
            R beta = R(0.0), cm[D];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                cm[a] = g[a] + r[a] * t;
                beta += cm[a] * cm[a];
            }
            const R wk = R(1.0) / ((eps + beta) * (eps + beta));
            Sw[v] += wk;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                Sc[a][v] += wk * cm[a];
                Sg[a][v] += cm[a];
            }
        }
    }
    const R g0 = R(kWenoGamma0), gk = (R(1.0) - R(kWenoGamma0)) / R(M_cand);
#pragma unroll
    for (int v = 0; v < nv; ++v) {
        const R w0 = g0 / ((eps + beta0[v]) * (eps + beta0[v]));
        const R itot = R(1.0) / (w0 + gk * Sw[v]);
        const R s0 = w0 * itot / g0;   // omega_0 / gamma_0
#pragma unroll
        for (int a = 0; a < D; ++a) c[a * nv + v] = s0 * (c[a * nv + v] - gk * Sg[a][v]) + gk * Sc[a][v] * itot;
#pragma unroll
        for (int q = 0; q < nq; ++q) c[(D + q) * nv + v] *= s0;
    }
}

// One thread per cell, all conservative variables: c = Minv M^T b.  The
// evaluation records of the block's cells are assembled in LDS and written
// out as one contiguous, coalesced range.
constexpr int kReconBlock = 64;
// WENO: the launch also serves cases with nonlinear weights (weno_eps > 0),
// applied after the linear-weight fit; other cases are untouched by it.
template <int D, typename R, bool WENO> __global__ __launch_bounds__(kReconBlock) void k_recon(Dev d) {
    using T = Dim<D>;
    constexpr int nv = T::nv, nk = T::nk, nq = T::nq;
    constexpr int ERP = Rec<D>::er + 1;   // padded LDS row
    __shared__ R rec_lds[kReconBlock * ERP];
    const int i0 = xcd_block(blockIdx.x, gridDim.x) * kReconBlock;
    const int i = i0 + threadIdx.x;
    const int NC = d.NC;
    const int ncell = min(kReconBlock, NC - i0);
    if (i < NC && d.prm[d.cell_case[i]].active) {
    using RC = Rec<D>;
    const double *gi = d.geo + size_t(i) * RC::gr;
    const double *si = d.st + size_t(i) * RC::sr;
    const double h = gi[D + nq], ih = 1.0 / h;
    double xc[D], own[nq], Wi[nv];
    R rhs[nk][nv];
    // own-gradient rows first: they only touch the linear coefficients
#pragma unroll
    for (int v = 0; v < nv; ++v) {
        Wi[v] = si[v];
#pragma unroll
        for (int a = 0; a < D; ++a) rhs[a][v] = R(h * si[nv + a * nv + v]);
#pragma unroll
        for (int q = 0; q < nq; ++q) rhs[D + q][v] = R(0.0);
    }
#pragma unroll
    for (int a = 0; a < D; ++a) xc[a] = gi[a];
#pragma unroll
    for (int q = 0; q < nq; ++q) own[q] = gi[D + sidx<D>(qa<D>(q), qb<D>(q))] * ih * ih;
#pragma unroll 1
    for (int s = 0; s < T::ns; ++s) {
        const int2 sl = d.slot[size_t(s) * NC + i];
        const int code = sl.x;
        if (code == 0) break;
        const int f = slot_face(code);
        const int nb = sl.y;
        R avg[nk];
        const double *gd;
        if (nb >= 0) {
            const double sg = code > 0 ? 1.0 : -1.0;
            const double *gm = d.geo + size_t(nb) * RC::gr;
            double dx[D];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                dx[a] = gm[a] + sg * d.shift[size_t(a) * d.NF + f] - xc[a];
                avg[a] = R(dx[a] * ih);
            }
#pragma unroll
            for (int q = 0; q < nq; ++q) {
                const int a = qa<D>(q), b = qb<D>(q);
                avg[D + q] = R((gm[D + sidx<D>(a, b)] + dx[a] * dx[b]) * ih * ih);
            }
            gd = d.st + size_t(nb) * RC::sr;
        } else {
            const int bs = d.bslot[f];
#pragma unroll
            for (int k = 0; k < nk; ++k) avg[k] = R(d.gavg[size_t(k) * d.NB + bs]);
            gd = d.gdat + size_t(bs) * (nv + D * nv);
        }
#pragma unroll
        for (int v = 0; v < nv; ++v) {
            // average row
            const R bv = R(gd[v] - Wi[v]);
#pragma unroll
            for (int a = 0; a < D; ++a) rhs[a][v] += avg[a] * bv;
#pragma unroll
            for (int q = 0; q < nq; ++q) rhs[D + q][v] += (avg[D + q] - R(own[q])) * bv;
            // gradient rows
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const R bg = R(h * gd[nv + a * nv + v]);
                rhs[a][v] += bg;
#pragma unroll
                for (int q = 0; q < nq; ++q) {
                    const int p = qa<D>(q), r = qb<D>(q);
                    const R row = (p == a ? avg[r] : R(0.0)) + (r == a ? avg[p] : R(0.0));
                    rhs[D + q][v] += row * bg;
                }
            }
        }
    }
    // evaluation record: centroid, 1/h, <phi_quad>_i, W, c = Minv rhs
    R *e = rec_lds + threadIdx.x * ERP;
#pragma unroll
    for (int a = 0; a < D; ++a) e[a] = R(xc[a]);
    e[D] = R(ih);
#pragma unroll
    for (int q = 0; q < nq; ++q) e[D + 1 + q] = R(own[q]);
#pragma unroll
    for (int v = 0; v < nv; ++v) e[RC::OW + v] = R(Wi[v]);
    const R *minv = HoArrays<R>::minv(d);
#pragma unroll
    for (int k = 0; k < nk; ++k) {
        R c[nv];
#pragma unroll
        for (int v = 0; v < nv; ++v) c[v] = R(0.0);
#pragma unroll
        for (int j = 0; j < nk; ++j) {
            const R mkj = ld_nt(minv + size_t(midx<D>(k, j)) * NC + i);
#pragma unroll
            for (int v = 0; v < nv; ++v) c[v] += mkj * rhs[j][v];
        }
#pragma unroll
        for (int v = 0; v < nv; ++v) e[RC::OC + k * nv + v] = c[v];
    }
    if constexpr (WENO) {
        const double eps_d = d.prm[d.cell_case[i]].weno_eps;
        if (eps_d > 0.0) weno_weights<D, R>(d, i, NC, xc, ih, h, own, Wi, R(eps_d), e + RC::OC);
    }
    }
    __syncthreads();
    R *dst = HoArrays<R>::ev(d) + size_t(i0) * Rec<D>::er;
    const int total = ncell * Rec<D>::er;
    for (int k = threadIdx.x; k < total; k += kReconBlock) {
        const int c = k / Rec<D>::er, j = k - c * Rec<D>::er;
        st_nt(rec_lds[c * ERP + j], dst + k);
    }
}

// lane p of each group of G lanes (G = 2 or 4, all active) to the whole group
template <int G, int P> __device__ __forceinline__ int bcast_i32(int x) {
    constexpr int ctrl = G == 4 ? (P | P << 2 | P << 4 | P << 6) : (P | P << 2 | (P + 2) << 4 | (P + 2) << 6);
    return __builtin_amdgcn_mov_dpp(x, ctrl, 0xF, 0xF, false);
}
template <int G, int P> __device__ __forceinline__ double bcast(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = bcast_i32<G, P>(int(u & 0xffffffffll)), hi = bcast_i32<G, P>(int(u >> 32));
    return __longlong_as_double((long long)(unsigned(lo)) | ((long long)hi << 32));
}
template <int G, int P> __device__ __forceinline__ float bcast(float v) {
    return __int_as_float(bcast_i32<G, P>(__float_as_int(v)));
}
template <int G, typename R> __device__ __forceinline__ R bcast_from(R v, int p) {
    switch (p) {
        case 0: return bcast<G, 0>(v);
        case 1: return bcast<G, 1>(v);
        case 2: return G == 4 ? bcast<G, 2>(v) : v;
        default: return G == 4 ? bcast<G, 3>(v) : v;
    }
}

// Reconstruction of cell i evaluated at x: W(x) into Wx, and its gradient
// added into G (global frame).  The G lanes of a face group share the
// record: lane q loads values [q er/G, (q+1) er/G) and every value reaches
// the group by a quad-permute broadcast, so the record crosses the memory
// pipeline once per face instead of once per Gauss point.
template <int D> constexpr int rec_share() {
    static_assert(Rec<D>::er % Dim<D>::lanes == 0, "record splits evenly over the face lanes");
    return Rec<D>::er / Dim<D>::lanes;
}

template <int D, typename R> __device__ __forceinline__ void recon_eval_share(const R *mine, const R *x, R *Wx,
                                                                              R G[D][D + 2]);

template <int D, typename R> __device__ __forceinline__ void recon_eval(const Dev &d, int i, int q, const R *x, R *Wx,
                                                                        R G[D][D + 2]) {
    constexpr int PL = rec_share<D>();
    const R *base = HoArrays<R>::ev(d) + size_t(i) * Rec<D>::er + q * PL;
    R mine[PL];
#pragma unroll
    for (int m = 0; m < PL; ++m) mine[m] = base[m];
    recon_eval_share<D, R>(mine, x, Wx, G);
}

// the evaluation itself, value j of the record taken by rec(j)
template <int D, typename R, typename Get> __device__ __forceinline__ void recon_eval_from(const Get &rec, const R *x,
                                                                                          R *Wx, R G[D][D + 2]) {
    using T = Dim<D>;
    using RC = Rec<D>;
    constexpr int nv = T::nv, nq = T::nq, KG = 3;
#define CGKS_REC(j) rec(j)
    R r[RC::OC];
#pragma unroll
    for (int k = 0; k < RC::OC; ++k) r[k] = CGKS_REC(k);
    const R ih = r[D];
    R y[D], yh[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        y[a] = (x[a] - r[a]) * ih;
        yh[a] = y[a] * ih;
    }
#pragma unroll
    for (int v = 0; v < nv; ++v) Wx[v] = r[RC::OW + v];
#pragma unroll
    for (int k = 0; k < D + nq; ++k) {
        if (k % KG == 0 && k > 0) __builtin_amdgcn_sched_barrier(0);
        if (k < D) {
#pragma unroll
            for (int v = 0; v < nv; ++v) {
                const R ck = CGKS_REC(RC::OC + k * nv + v);
                Wx[v] += ck * y[k];
                G[k][v] += ck * ih;
            }
        } else {
            const int qq = k - D, a = qa<D>(qq), b = qb<D>(qq);
            const R phi = y[a] * y[b] - r[D + 1 + qq];
#pragma unroll
            for (int v = 0; v < nv; ++v) {
                const R ck = CGKS_REC(RC::OC + k * nv + v);
                Wx[v] += ck * phi;
                G[a][v] += ck * yh[b];
                G[b][v] += ck * yh[a];
            }
        }
    }
#undef CGKS_REC
}

// the same from a share already in registers: value j comes from lane
// j / PL of the group by a quad-permute broadcast
template <int D, typename R> __device__ __forceinline__ void recon_eval_share(const R *mine, const R *x, R *Wx,
                                                                              R G[D][D + 2]) {
    constexpr int GL = Dim<D>::lanes, PL = Rec<D>::er / GL;
    recon_eval_from<D, R>([&](int j) { return bcast_from<GL, R>(mine[j % PL], j / PL); }, x, Wx, G);
}

// ---------------------------------------------------------------------
// Face flux at every Gauss point: interface states, boundary states,
// kinetic interface equilibrium, smooth gas-kinetic flux.  Outputs are
// weighted by wJ and in the global frame.
// ---------------------------------------------------------------------
// Sets bit 0 of flag[c] for the case c of every lane whose state is not
// physical: one atomic per (wave, case), not one per lane, so a case that
// has gone bad does not stall the launch on a single contended address.
// Called by every active lane of the wave.
__device__ inline void flag_nonphysical(int32_t *flag, bool bad, int c) {
    unsigned long long m = __ballot(bad);
    while (m) {
        const int l = __ffsll(m) - 1;
        const int cl = __shfl(c, l);
        if (int(__lane_id()) == l) atomicOr(flag + cl, 1);
        m &= ~__ballot(bad && c == cl);
    }
}

// sum of v over the G consecutive lanes of a face group (every lane gets it)
// DPP quad permutation (lane l of each group of four takes lane l ^ m,
// m = 1 or 2) of a 32- or 64-bit value, without the LDS crossbar
template <int M> __device__ __forceinline__ int dpp_xor_i32(int x) {
    constexpr int ctrl = M == 1 ? 0xB1 : 0x4E;   // quad_perm [1,0,3,2] / [2,3,0,1]
    return __builtin_amdgcn_mov_dpp(x, ctrl, 0xF, 0xF, false);
}
template <int M> __device__ __forceinline__ double dpp_xor(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = dpp_xor_i32<M>(int(u & 0xffffffffll)), hi = dpp_xor_i32<M>(int(u >> 32));
    return __longlong_as_double((long long)(unsigned(lo)) | ((long long)hi << 32));
}
template <int M> __device__ __forceinline__ float dpp_xor(float v) {
    return __int_as_float(dpp_xor_i32<M>(__float_as_int(v)));
}

// sum of v over the G (2 or 4) consecutive lanes of a group, every lane
// of the group gets it: butterfly of quad permutations (all lanes of a
// group active)
template <int G, typename T> __device__ __forceinline__ T group_sum(T v) {
    static_assert(G == 2 || G == 4, "lane groups of 2 or 4");
    v += dpp_xor<1>(v);
    if constexpr (G == 4) v += dpp_xor<2>(v);
    return v;
}

// N consecutive values of a face record that every lane of the face's
// group holds (after group_sum), spread over the group: lane q stores the
// values q, q + G, ..., so one store instruction writes G adjacent values
// of each face instead of one value from one lane
// (val(j) gives value j; it is called for a row of G values at a time so
// that only one row of sums is live)
template <int G, int N, typename R, typename Val>
__device__ __forceinline__ void group_store(R *dst, int q, bool on, Val val) {
#pragma unroll
    for (int r = 0; r < N; r += G) {
        R v = val(r);
#pragma unroll
        for (int k = 1; k < G; ++k)
            if (r + k < N) {
                const R u = val(r + k);
                v = q == k ? u : v;
            }
        if (on && r + q < N) dst[r + q] = v;
    }
}

// One group of Dim<D>::lanes threads per face, one thread per Gauss point;
// a lane without a Gauss point (triangles in 3-D) repeats the first point
// with weight 0, so every lane runs the same code.  The face sums
//   sum_g wJ (F0, Ft, W_c n, W_t n)   (global frame)
// are reduced across the group and stored face-major, spread over the
// group's lanes (group_store).
// want_grad: 0 = flux sums only (the residual pass); 2 = the flux sums,
// both Gauss-Green groups and the wall faces' momentum sums in wallf (stage
// 0); 1 = the second S2O4 stage, whose update takes only the time
// derivatives: the F_t sums and the Gauss-Green sums of W_t (the record's
// F0 and W groups keep the first stage's values, which the cell kernel
// reads along but does not use)
// FULL: the launch also serves cases with the full time-dependent solution
// (flux_full); smooth cases of such a launch take exactly the smooth path.
template <int D, typename R, bool FULL> __global__ __launch_bounds__(kBlock) void k_flux(Dev d, int want_grad) {
    using T = Dim<D>;
    constexpr int nv = T::nv, G = T::lanes, FS = T::fs;
    constexpr int PL = rec_share<D>();
    const int t = xcd_block(blockIdx.x, gridDim.x) * int(blockDim.x) + threadIdx.x;
    const int fr_raw = t / G, q = t % G;
    const bool face_ok = fr_raw < d.NF;
    const int f = face_ok ? fr_raw : d.NF - 1;
    // Two rounds to memory before any arithmetic: everything indexed by the
    // face, then everything indexed by what that holds (the Gauss points,
    // both cells' record shares, the case), and only then the case's active
    // flag, so no load waits on a branch.  A boundary face reads its own
    // cell's share twice and drops the second.
    const int cs = d.fcase[f];
    const int2 gr_ = d.gp_rng[f];
    const int cL = d.fL[f], cR = d.fR[f];
    const int fcode = d.fbc[f];
    R sft[D];
#pragma unroll
    for (int a = 0; a < D; ++a) sft[a] = R(d.shift[size_t(a) * d.NF + f]);
    const int g0 = gr_.x, g1 = gr_.y;
    const bool gp_ok = face_ok && g0 + q < g1;
    const int g = gp_ok ? g0 + q : g0;
    R x[D], n[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        x[a] = R(d.gx[size_t(a) * d.NG + g]);
        n[a] = R(d.gn[size_t(a) * d.NG + g]);
    }
    const R wJ = gp_ok ? R(d.gw[g]) : R(0.0);
    const int case_on = d.prm[cs].active;
    R shareL[PL], shareR[PL];
    {
        const R *ev = HoArrays<R>::ev(d);
        const R *bl = ev + size_t(cL) * Rec<D>::er + q * PL;
        const R *br = ev + size_t(cR >= 0 ? cR : cL) * Rec<D>::er + q * PL;
#pragma unroll
        for (int m = 0; m < PL; ++m) {
            shareL[m] = bl[m];
            shareR[m] = br[m];
        }
        // the shares and the flag are taken here, so the compiler cannot
        // sink the shares' loads below the branch on the flag
        asm volatile("" ::"v"(case_on));
#pragma unroll
        for (int m = 0; m < PL; ++m) asm volatile("" ::"v"(shareL[m]), "v"(shareR[m]));
    }
    if (!case_on) return;   // the face group leaves together
    const DevParams &P = d.prm[cs];
    Frame<D, R> fr;
    fr.build(n);
    R Wc[nv], Gc[D][nv];
    bool ok = true;
    const int bc = fcode & 7;
    const bool planar = (fcode & kFacePlanar) != 0;
    const bool full = FULL && P.flux_full != 0;
    bool did_full = false;
    R F0f[nv], Ftf[nv], Wtf[nv];
    {
        // gradients summed in the global frame, rotated once
        R Gs[D][nv], WL[nv];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int v = 0; v < nv; ++v) Gs[a][v] = R(0.0);
        {
            R Wg[nv];
            recon_eval_share<D, R>(shareL, x, Wg, Gs);
            fr.to_local(Wg, WL);
        }
        // the left gradient alone, for the full solution
        R GLg[FULL ? D : 1][nv];
        if constexpr (FULL) {
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int v = 0; v < nv; ++v) GLg[a][v] = Gs[a][v];
        }
        if (cR >= 0 || bc != 2) {
            R WR[nv];
            if (cR >= 0) {
                R xr[D], WRg[nv];
#pragma unroll
                for (int a = 0; a < D; ++a) xr[a] = x[a] - sft[a];
                recon_eval_share<D, R>(shareR, xr, WRg, Gs);
                fr.to_local(WRg, WR);
            } else if (bc == 1 || bc == 3) {
                // mirror: normal momentum reversed (slip), every momentum
                // component reversed (no-slip adiabatic)
#pragma unroll
                for (int v = 0; v < nv; ++v) WR[v] = WL[v];
                WR[1] = -WL[1];
                if (bc == 3) {
#pragma unroll
                    for (int a = 1; a < D; ++a) WR[1 + a] = -WL[1 + a];
                }
            } else {
                R Wo_g[nv], Wo[nv];
#pragma unroll
                for (int v = 0; v < nv; ++v) Wo_g[v] = R(P.W_inf[v]);
                fr.to_local(Wo_g, Wo);
                farfield_state<D, R>(WL, Wo, R(P.gamma), WR);
            }
#pragma unroll
            for (int v = 0; v < nv; ++v) Wc[v] = R(0.0);
            // FP32: one side at a time (the erfc and exp of both sides
            // interleaved set the register peak; measured 2.7 % faster).
            // FP64 is left to the scheduler (measured 1.8 % faster).
            constexpr bool sides_apart = sizeof(R) == 4;
            if (sides_apart) __builtin_amdgcn_sched_barrier(0);
            ok = half_side<D, R>(WL, P, R(1.0), Wc, nullptr);
            if (sides_apart) __builtin_amdgcn_sched_barrier(0);
            ok = half_side<D, R>(WR, P, -R(1.0), Wc, nullptr) && ok;
            if (sides_apart) __builtin_amdgcn_sched_barrier(0);
            fr.grad_to_local(Gs, Gc);
            if (cR < 0 && (bc == 1 || bc == 3)) {
                // mirror ghost: a derivative flips sign when exactly one of
                // (normal direction, reversed momentum component) applies to
                // it; flipped ones cancel in the average, the others are kept
                // whole.  No-slip adiabatic: zero normal derivative of rho and
                // E at zero velocity, hence no heat flux.
                const bool all_mom = bc == 3;
#pragma unroll
                for (int a = 0; a < D; ++a)
#pragma unroll
                    for (int v = 0; v < nv; ++v) {
                        const bool rev = all_mom ? (v >= 1 && v <= D) : (v == 1);
                        if ((a == 0) != rev) Gc[a][v] = R(0.0);
                    }
            } else {
                // interior: average of both sides; far field: the exterior
                // state has zero gradient
#pragma unroll
                for (int a = 0; a < D; ++a)
#pragma unroll
                    for (int v = 0; v < nv; ++v) Gc[a][v] *= R(0.5);
            }
            if constexpr (FULL) {
                if (full && ok) {
                    // the two one-sided gradients in the face frame: the right
                    // cell's reconstruction once more, the mirror of the left
                    // one at a slip or adiabatic wall, zero at the far field
                    R GL[D][nv], GR[D][nv];
                    fr.grad_to_local(GLg, GL);
                    if (cR >= 0) {
                        R GRg[D][nv], xr[D], WRg[nv];
#pragma unroll
                        for (int a = 0; a < D; ++a)
#pragma unroll
                            for (int v = 0; v < nv; ++v) GRg[a][v] = R(0.0);
#pragma unroll
                        for (int a = 0; a < D; ++a) xr[a] = x[a] - sft[a];
                        recon_eval<D, R>(d, cR, q, xr, WRg, GRg);
                        fr.grad_to_local(GRg, GR);
                    } else if (bc == 1 || bc == 3) {
                        const bool all_mom = bc == 3;
#pragma unroll
                        for (int a = 0; a < D; ++a)
#pragma unroll
                            for (int v = 0; v < nv; ++v) {
                                const bool rev = all_mom ? (v >= 1 && v <= D) : (v == 1);
                                GR[a][v] = (a == 0) != rev ? -GL[a][v] : GL[a][v];
                            }
                    } else {
#pragma unroll
                        for (int a = 0; a < D; ++a)
#pragma unroll
                            for (int v = 0; v < nv; ++v) GR[a][v] = R(0.0);
                    }
                    R W0[nv];
                    ok = gks_flux_full<D, R>(WL, GL, WR, GR, Wc, Gc, P, R(d.dt[cs]), F0f, Ftf, W0, Wtf);
                    did_full = true;
                    // the Gauss-Green sums take the interface state's time fit
#pragma unroll
                    for (int v = 0; v < nv; ++v) Wc[v] = W0[v];
                }
            }
        } else {
            // no-slip isothermal wall: (p_L / T_w, 0, p_L), interior gradient
            Prim<D, R> pq;
            pq.from(WL, R(P.gamma));
#pragma unroll
            for (int v = 0; v < nv; ++v) Wc[v] = R(0.0);
            Wc[0] = pq.p / R(P.T_wall);
            Wc[nv - 1] = pq.p / (R(P.gamma) - R(1.0));
            fr.grad_to_local(Gs, Gc);
        }
    }
    R *dst = HoArrays<R>::fsum(d) + size_t(f) * FS;
    const bool writer = face_ok && q == 0;
    // a wave whose faces are all planar reduces one Gauss-Green group per
    // quantity instead of D (uniform branch)
    const bool wave_planar = __all(planar);
    R o[nv];
    // Gauss-Green sums of the interface state (at t = 0, then its time
    // derivative): a planar face has the plain sum in the first group and
    // the normal after it; in a wave with any warped face every face runs
    // the same D reductions, a planar one with weights (1, 0, 0)
    auto gauss_green = [&](const R *Wl, int off) {
        fr.to_global(Wl, o);
        R w[nv];
#pragma unroll
        for (int v = 0; v < nv; ++v) w[v] = wJ * o[v];
        if (wave_planar) {
            group_store<G, nv>(dst + T::fg + off, q, face_ok, [&](int v) { return group_sum<G, R>(w[v]); });
        } else {
#pragma unroll
            for (int a = 0; a < D; ++a)
                group_store<G, nv>(dst + T::fg + a * 2 * nv + off, q, face_ok && (!planar || a == 0), [&](int v) {
                    return group_sum<G, R>(planar ? (a == 0 ? w[v] : R(0.0)) : w[v] * n[a]);
                });
        }
    };
    const bool t_only = want_grad == 1;
    if (want_grad) {
        group_store<G, D>(dst + T::fh, q, face_ok && planar, [&](int a) { return n[a]; });
        if (!t_only) {
            R Wz[nv];
#pragma unroll
            for (int v = 0; v < nv; ++v) Wz[v] = ok ? Wc[v] : R(0.0);
            gauss_green(Wz, 0);
        }
    }
    R F0[nv], Ft[nv], Wt[nv];
    if (FULL && did_full) {
#pragma unroll
        for (int v = 0; v < nv; ++v) {
            F0[v] = F0f[v];
            Ft[v] = Ftf[v];
            Wt[v] = Wtf[v];
        }
    } else if (ok) {
        ok = gks_flux<D, R>(Wc, Gc, P, F0, Ft, Wt);
    }
    flag_nonphysical(d.flag, !ok && gp_ok, cs);
    if (!ok) {
#pragma unroll
        for (int v = 0; v < nv; ++v) F0[v] = Ft[v] = Wt[v] = R(0.0);
    }
    if (cR < 0 && bc == 2) {
        F0[0] = R(0.0);
        Ft[0] = R(0.0);
#pragma unroll
        for (int v = 0; v < nv; ++v) Wt[v] = R(0.0);
    }
    {
        R of[2 * nv];
        fr.to_global(F0, of);
        fr.to_global(Ft, of + nv);
        const bool wall_out = want_grad == 2 && writer && cR < 0 && (bc == 1 || bc == 2 || bc == 3);
        if (t_only) {
            group_store<G, nv>(dst + nv, q, face_ok, [&](int v) { return group_sum<G, R>(wJ * of[nv + v]); });
        } else {
            group_store<G, 2 * nv>(dst, q, face_ok, [&](int v) {
                const R sum = group_sum<G, R>(wJ * of[v]);
                if (v >= 1 && v <= D && wall_out) d.wallf[size_t(d.bslot[f]) * 3 + (v - 1)] = double(sum);
                return sum;
            });
        }
    }
    if (want_grad) gauss_green(Wt, nv);
}

// ---------------------------------------------------------------------
// Per-cell gather of the face Gauss-point results and the stage update.
// ---------------------------------------------------------------------
enum { MODE_STAGE0 = 0, MODE_STAGE1 = 1, MODE_R1 = 2 };

// Dim<D>::sl lanes per cell: lane q gathers slots q, q + sl, ...; the sums
// are reduced across the group and lane q then owns variables q, q + sl.
template <int D, typename R> __global__ __launch_bounds__(kBlock) void k_cell(Dev d, int mode) {
    using T = Dim<D>;
    constexpr int nv = T::nv, SL = T::sl, GW = 2 * nv, SR = Rec<D>::sr;
    // stage passes: the block's new state records pass through LDS so that
    // its stores are consecutive (the lanes of a cell would store 5 doubles
    // apart, 16 cells at once)
    __shared__ __align__(16) double stage[kBlock / SL * SR];
    __shared__ int live_s[kBlock / SL];
    const int nbc = int(blockDim.x) / SL;
    const int c0 = xcd_block(blockIdx.x, gridDim.x) * nbc;
    if (c0 >= d.NC) return;   // the whole block
    const int ir = c0 + int(threadIdx.x) / SL, q = int(threadIdx.x) % SL, lc = ir - c0;
    const bool ok = ir < d.NC;
    const int i = ok ? ir : d.NC - 1;
    const int NC = d.NC;
    const int cs = d.cell_case[i];
    const DevParams &P = d.prm[cs];
    const bool act = P.active;
    if (mode == MODE_R1) {
        // the residual needs only the flux groups (F0, Ft): lane q takes the
        // cell's slot q (every cell has at least SL faces in 3-D; a missing
        // one in 2-D reads with weight 0 the cell's first face, written in
        // the same pass), and slot q + SL only where the cell has it; the
        // lanes' partial sums meet in a lane-group sum
        constexpr int NS = T::ns / SL;
        const int code0 = d.slot[size_t(q) * NC + i].x;
        const int f_first = slot_face(bcast_i32<SL, 0>(code0));
        double a[GW];
        {
            const bool has = code0 != 0;
            const int f = has ? slot_face(code0) : f_first;
            const double sg = has ? (code0 > 0 ? 1.0 : -1.0) : 0.0;
            const R *rec = HoArrays<R>::fsum(d) + size_t(f) * T::fs;
#pragma unroll
            for (int j = 0; j < GW; ++j) a[j] = sg * double(rec[j]);
        }
#pragma unroll
        for (int k = 1; k < NS; ++k) {
            const int code = d.slot[size_t(q + k * SL) * NC + i].x;
            if (code != 0) {
                const double sg = code > 0 ? 1.0 : -1.0;
                const R *rec = HoArrays<R>::fsum(d) + size_t(slot_face(code)) * T::fs;
#pragma unroll
                for (int j = 0; j < GW; ++j) a[j] += sg * double(rec[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < GW; ++j) a[j] = group_sum<SL, double>(a[j]);
        if (!ok || !act || q != 0) return;
        const double dt = d.dt[cs];
#pragma unroll
        for (int v = 0; v < nv; ++v) st_nt(-(a[v] + 0.5 * dt * a[nv + v]), d.R1 + size_t(v) * NC + i);
        return;
    }
    // stage passes: lane 0 sums the flux group (F0, Ft) of the cell's face
    // records, lane 1 + a the Gauss-Green group of axis a (W_c n_a, W_t n_a):
    // each lane reads 2 nv values of every face and needs no other lane's
    // sums.  For a planar face (marked in its slot code) lane 1 + a reads the
    // one plain group and scales it by n_a.
    const bool mine = q <= D;
    const int ax = q - 1;
    double acc[GW];
#pragma unroll
    for (int k = 0; k < GW; ++k) acc[k] = 0.0;
    if (act && mine) {
        if constexpr (std::is_same<R, float>::value) {
            // FP32 face records: every slot code first, then all face
            // groups at once; an empty slot reads face 0 with weight 0 (face
            // sums are always finite: a non-physical Gauss point contributes
            // zeros).  -6 % on the sphere; with FP64 records the loads in
            // flight cost the kernel its occupancy (+7 %), so FP64 gathers
            // slot by slot.
            int code[T::ns];
#pragma unroll
            for (int s = 0; s < T::ns; ++s) code[s] = d.slot[size_t(s) * NC + i].x;
#pragma unroll
            for (int s = 0; s < T::ns; ++s) {
                const bool has = code[s] != 0;
                const int f = has ? slot_face(code[s]) : 0;
                const double sg = has ? (code[s] > 0 ? 1.0 : -1.0) : 0.0;
                const R *rec = HoArrays<R>::fsum(d) + size_t(f) * T::fs;
                // one instruction stream for the whole lane group: lane 0
                // takes (F0, Ft) with weight 1, the others their group
                const bool pl = q > 0 && slot_planar(code[s]);
                const R na = rec[T::fh + (q > 0 ? ax : 0)];
                const R *g = rec + (q == 0 ? 0 : T::fg + (pl ? 0 : ax * GW));
                const double w = sg * (pl ? double(na) : 1.0);
#pragma unroll
                for (int k = 0; k < GW; ++k) acc[k] += w * double(g[k]);
            }
        } else {
#pragma unroll 1
            for (int s = 0; s < T::ns; ++s) {
                const int code = d.slot[size_t(s) * NC + i].x;
                if (code == 0) break;
                const int f = slot_face(code);
                const double sg = code > 0 ? 1.0 : -1.0;
                const R *rec = HoArrays<R>::fsum(d) + size_t(f) * T::fs;
                const bool pl = q > 0 && slot_planar(code);
                const R na = rec[T::fh + (q > 0 ? ax : 0)];
                const R *g = rec + (q == 0 ? 0 : T::fg + (pl ? 0 : ax * GW));
                const double w = sg * (pl ? double(na) : 1.0);
#pragma unroll
                for (int k = 0; k < GW; ++k) acc[k] += w * double(g[k]);
            }
        }
    }
    const bool live = ok && act;
    const double dt = d.dt[cs];
    // lane 0: the new W (record positions 0 .. nv-1); lane 1 + a: the new
    // gradient along axis a (positions nv (1 + a) ...)
    double *o = stage + lc * SR + q * nv;
    if (live && mine) {
        const double iV = recip<double>(d.vol[i]);
        const double *si = d.st + size_t(i) * SR;
        if (q == 0) {
#pragma unroll
            for (int v = 0; v < nv; ++v) {
                const double L = -acc[v] * iV, Lt = -acc[nv + v] * iV;
                if (mode == MODE_STAGE0) {
                    const double w = si[v];
                    st_nt(w, d.Wn + size_t(v) * NC + i);
                    st_nt(L, d.L0 + size_t(v) * NC + i);
                    st_nt(Lt, d.Lt0 + size_t(v) * NC + i);
                    o[v] = P.scheme == 0 ? w + 0.5 * dt * L + 0.125 * dt * dt * Lt : w + dt * L + 0.5 * dt * dt * Lt;
                } else {
                    o[v] = ld_nt(d.Wn + size_t(v) * NC + i) + dt * ld_nt(d.L0 + size_t(v) * NC + i) +
                           dt * dt / 6.0 * (ld_nt(d.Lt0 + size_t(v) * NC + i) + 2.0 * Lt);
                }
            }
        } else {
            const int a = q - 1;
#pragma unroll
            for (int v = 0; v < nv; ++v) {
                const size_t k = size_t(a * nv + v) * NC + i;
                const double G = acc[v] * iV, Gt = acc[nv + v] * iV;
                if (mode == MODE_STAGE0) {
                    st_nt(G, d.G0 + k);
                    o[v] = P.scheme == 0 ? G + 0.5 * dt * Gt : G + dt * Gt;
                } else {
                    o[v] = ld_nt(d.G0 + k) + dt * Gt;
                }
            }
        }
    }
    if (q == 0) live_s[lc] = live;
    __syncthreads();
    // the block's records are consecutive: 16-byte stores, a cell's only
    // where it is live
    const int ncell = min(nbc, NC - c0);
    double2 *dst = reinterpret_cast<double2 *>(d.st + size_t(c0) * SR);
    const double2 *src = reinterpret_cast<const double2 *>(stage);
    for (int e = int(threadIdx.x); e < ncell * (SR / 2); e += int(blockDim.x))
        if (live_s[e / (SR / 2)]) dst[e] = src[e];
}

// ---------------------------------------------------------------------
// Low level: first-order KFVS face flux, spectral radius, cell setup,
// multicolour point relaxation, prolongation and the residual norm.
// ---------------------------------------------------------------------
template <int D> __device__ __forceinline__ double side_radius(const double *U, const double *n, double Sf, double V,
                                                               const DevParams &P) {
    constexpr int nv = D + 2;
    const double rho = U[0], ir = recip<double>(rho);
    double un = 0, ke = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double u = U[1 + a] * ir;
        un += u * n[a];
        ke += u * u;
    }
    const double p = (P.gamma - 1.0) * (U[nv - 1] - 0.5 * rho * ke);
    return fabs(un) + sqrt(P.gamma * p * ir) + 2.0 * P.mu * ir * Sf * recip<double>(V);
}

enum { LOW_SRC_W = 0, LOW_SRC_U_DU = 2 };

// state of cell i: W from the state records, or the low-level U + dU
template <int D, typename S, int src> __device__ __forceinline__ void low_state(const Dev &d, int i, double *out) {
    constexpr int nv = D + 2;
    if constexpr (src == LOW_SRC_W) {
#pragma unroll
        for (int v = 0; v < nv; ++v) out[v] = d.st[size_t(i) * Rec<D>::sr + v];
    } else {
        const double *U = LowRec<D, S>::U(d, i);
        const S *dU = LowRec<D, S>::dU(d, i);
#pragma unroll
        for (int v = 0; v < nv; ++v) out[v] = src == LOW_SRC_U_DU ? U[v] + double(dU[v]) : U[v];
    }
}

// lowf[f] = S_f F(U_L, U_R; n_f), F the case's first-order flux (KFVS or
// Lax-Friedrichs); swp[f][D] = S_f lam_f (the area vector S_f n_f in
// swp[f][0..D) is written at upload).
template <int D, typename S, int SRC> __global__ __launch_bounds__(kBlock) void k_low_face(Dev d) {
    constexpr int nv = D + 2, src = SRC;
    // the block's flux records pass through LDS so that its stores to lowf
    // are consecutive (one face per thread would store 2 nv doubles apart)
    __shared__ double stage[kBlock * nv];
    __shared__ int live_s[kBlock];
    const int nb = int(blockDim.x);
    const int f0 = xcd_block(blockIdx.x, gridDim.x) * nb;
    if (f0 >= d.NF) return;   // the whole block
    const int fr_raw = f0 + int(threadIdx.x);
    const bool in = fr_raw < d.NF;
    const int f = in ? fr_raw : d.NF - 1;
    // Two rounds to memory before any arithmetic (as in the flux): the
    // face's own data, then both cells' states and volumes with the case's
    // active flag, and only then the branch on the flag.  A boundary face
    // reads its own cell twice and drops the second.
    const int cs = d.fcase[f];
    const int L = d.fL[f], R = d.fR[f];
    const double Sf = d.S[f];
    double av[D];
#pragma unroll
    for (int a = 0; a < D; ++a) av[a] = d.avec[size_t(a) * d.NF + f];
    const int case_on = d.prm[cs].active;
    double UL[nv], UR[nv];
    low_state<D, S, src>(d, L, UL);
    low_state<D, S, src>(d, R >= 0 ? R : L, UR);
    const double VL = d.vol[L], VR = d.vol[R >= 0 ? R : L];
    asm volatile("" ::"v"(case_on), "v"(VL), "v"(VR));
#pragma unroll
    for (int v = 0; v < nv; ++v) asm volatile("" ::"v"(UL[v]), "v"(UR[v]));
    const bool live = in && case_on;
    if (live) {
        const DevParams &P = d.prm[cs];
        const double iS = recip<double>(Sf);
        double n[D];
#pragma unroll
        for (int a = 0; a < D; ++a) n[a] = av[a] * iS;
        Frame<D, double> fr;
        fr.build(n);
        double Ul[nv], Ur[nv];
        fr.to_local(UL, Ul);
        double lam = side_radius<D>(UL, n, Sf, VL, P);
        if (R >= 0) {
            fr.to_local(UR, Ur);
            lam = fmax(lam, side_radius<D>(UR, n, Sf, VR, P));
        } else {
            const int bc = d.fbc[f] & 7;
#pragma unroll
            for (int v = 0; v < nv; ++v) Ur[v] = Ul[v];
            if (bc == 1) {
                Ur[1] = -Ul[1];
            } else if (bc == 2 || bc == 3) {
#pragma unroll
                for (int a = 0; a < D; ++a) Ur[1 + a] = -Ul[1 + a];
            } else {
                double Wo_g[nv], Wo[nv];
#pragma unroll
                for (int v = 0; v < nv; ++v) Wo_g[v] = P.W_inf[v];
                fr.to_local(Wo_g, Wo);
                farfield_state<D, double>(Ul, Wo, P.gamma, Ur);
            }
        }
        double Fl[nv], F[nv];
        bool ok;
        if (P.low_flux == 1) {
            // Lax-Friedrichs with the face's spectral radius
            Prim<D, double> a, c;
            a.from(Ul, P.gamma);
            c.from(Ur, P.gamma);
            ok = a.rho > 0.0 && a.p > 0.0 && c.rho > 0.0 && c.p > 0.0;
            const double e0[D] = {1.0};
            double Fa[nv], Fb[nv];
            euler_flux<D>(Ul, e0, P.gamma, Fa);
            euler_flux<D>(Ur, e0, P.gamma, Fb);
#pragma unroll
            for (int v = 0; v < nv; ++v) Fl[v] = 0.5 * (Fa[v] + Fb[v]) - 0.5 * lam * (Ur[v] - Ul[v]);
        } else {
#pragma unroll
            for (int v = 0; v < nv; ++v) Fl[v] = 0.0;
            ok = half_side<D, double>(Ul, P, 1.0, nullptr, Fl) && half_side<D, double>(Ur, P, -1.0, nullptr, Fl);
        }
        flag_nonphysical(d.flag, !ok, cs);
        fr.to_global(Fl, F);
#pragma unroll
        for (int v = 0; v < nv; ++v) stage[threadIdx.x * nv + v] = ok ? Sf * F[v] : 0.0;
        d.swp[size_t(f) * 4 + D] = Sf * lam;   // the area vector part is written at upload
    }
    live_s[threadIdx.x] = live;
    __syncthreads();
    const int nrow = min(nb, d.NF - f0);
    double *dst = d.lowf + size_t(f0) * nv;
    for (int e = int(threadIdx.x); e < nrow * nv; e += nb)
        if (live_s[e / nv]) dst[e] = stage[e];
}

// LOW_FORCE: forcing S = R1 - R0(W), U = W, and the first implicit step's
// set-up at U = W (its KFVS fluxes are the ones R0(W) was gathered from);
// LOW_STEP: U += dU and the next step's set-up; LOW_R0_OUT: R0 only.
enum { LOW_FORCE = 0, LOW_STEP = 2, LOW_R0_OUT = 3 };

template <int D, typename S, int MODE> __global__ __launch_bounds__(kBlock) void k_low_cell(Dev d, double *out) {
    constexpr int mode = MODE;
    using T = Dim<D>;
    constexpr int nv = T::nv, SL = T::sl, NS = T::ns / SL;   // slots per lane
    const int t = xcd_block(blockIdx.x, gridDim.x) * int(blockDim.x) + threadIdx.x;
    const int ir = t / SL, q = t % SL;
    const bool ok = ir < d.NC;
    const int i = ok ? ir : d.NC - 1;
    const int NC = d.NC;
    // all slot codes first, then every face record at once, the case flag
    // with gamma, and the cell's own inputs of the mode.  An empty slot reads
    // face 0: its KFVS flux enters with weight 0 (lowf is always finite: a
    // non-physical face stores zeros), its S lam through a select (that one
    // may not be finite).  A select of the flux itself would become a branch
    // around each load.
    int code[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) code[k] = d.slot[size_t(q + k * SL) * NC + i].x;
    const DevParams &P = d.prm[d.cell_case[i]];
    const bool active = P.active;
    double *Ui = LowRec<D, S>::U(d, i);
    S *dUi = LowRec<D, S>::dU(d, i);
    double u[nv], own[nv];   // state of the step; Sf (steps) or R1 (forcing) of this lane's variables
    if constexpr (mode == LOW_FORCE) {
#pragma unroll
        for (int v = 0; v < nv; ++v) u[v] = d.st[size_t(i) * Rec<D>::sr + v];
#pragma unroll
        for (int v = 0; v < nv; ++v) own[v] = v % SL == q ? d.R1[size_t(v) * NC + i] : 0.0;
    } else if constexpr (mode == LOW_STEP) {
#pragma unroll
        for (int v = 0; v < nv; ++v) u[v] = Ui[v] + double(dUi[v]);
#pragma unroll
        for (int v = 0; v < nv; ++v) own[v] = v % SL == q ? d.Sf[size_t(v) * NC + i] : 0.0;
    }
    const double Vi = d.vol[i], hi = d.h[i];
    double R0[nv], lS = 0.0;
#pragma unroll
    for (int v = 0; v < nv; ++v) R0[v] = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const bool has = code[k] != 0;
        const int f = has ? slot_face(code[k]) : 0;
        const double sg = has ? (code[k] > 0 ? 1.0 : -1.0) : 0.0;
        const double *lf = d.lowf + size_t(f) * nv;
        const double sl_lam = d.swp[size_t(f) * 4 + D];
#pragma unroll
        for (int v = 0; v < nv; ++v) R0[v] -= sg * lf[v];
        lS += has ? sl_lam : 0.0;
    }
#pragma unroll
    for (int v = 0; v < nv; ++v) R0[v] = group_sum<SL, double>(R0[v]);
    lS = group_sum<SL, double>(lS);
    if (!ok || !active) return;   // the cell's lane group leaves together
    if constexpr (mode == LOW_R0_OUT) {
#pragma unroll
        for (int v = 0; v < nv; ++v)
            if (v % SL == q) out[size_t(v) * NC + i] = R0[v];
        return;
    }
    if constexpr (mode == LOW_FORCE) {
#pragma unroll
        for (int v = 0; v < nv; ++v)
            if (v % SL == q) {
                const double sf = own[v] - R0[v];
                d.Sf[size_t(v) * NC + i] = sf;
                d.RHS[size_t(v) * NC + i] = R0[v] + sf;
            }
    } else {
#pragma unroll
        for (int v = 0; v < nv; ++v)
            if (v % SL == q) d.RHS[size_t(v) * NC + i] = R0[v] + own[v];
    }
    low_rec_reset<D, S, SL>(d, i, u, q);
    if (q == 0) d.D[i] = Vi * recip<double>(state_dt<D>(u, hi, P.cfl_low, P)) + 0.5 * lS;
}

// one colour class: blocks listed in (start, count) tables.  With A = s S_f n_f
// (outward from i) the delta flux of a neighbour is
//   S_f [F-(U_m + dU_m) - F-(U_m)] = 1/2 (F_A(U_m + dU_m) - F_A(U_m)) - 1/2 S_f lam_f dU_m.
// FP64 sweeps difference the two fluxes as written; FP32 sweeps (S = float)
// evaluate the flux change in the cancellation-free form euler_dflux.
template <int D, typename S>
__global__ __launch_bounds__(kBlock) void k_sweep(Dev d, const int32_t *blk_start, const int32_t *blk_count) {
    using T = Dim<D>;
    constexpr int nv = T::nv, SL = T::sl, NS = T::ns / SL;   // slots per lane
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int lc = threadIdx.x / SL, q = threadIdx.x % SL;
    const bool ok = lc < blk_count[b];
    const int i = blk_start[b] + (ok ? lc : 0);
    const int NC = d.NC;
    S acc[nv];
#pragma unroll
    for (int v = 0; v < nv; ++v) acc[v] = S(0);
    if constexpr (std::is_same<S, double>::value) {
        // FP64: everything this lane reads is addressed up front, so both
        // slots, both neighbour records and the cell's own RHS and D are in
        // flight together.  A slot without a neighbour reads the cell's own
        // record and face 0, and a select (not a product: those records may
        // hold anything) drops it.  The lane's RHS values are loaded without
        // a select (a select of a load becomes a branch around it): its own
        // variable q and the last one, which lane 0 owns when nv > SL.
        int2 sl[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) sl[k] = d.slot[size_t(q + k * SL) * NC + i];
        double gamma;
        bool active;
        gamma_active(d.prm[d.cell_case[i]], gamma, active);
        const double Di = d.D[i];
        const double rhs_q = d.RHS[size_t(q) * NC + i], rhs_last = d.RHS[size_t(nv - 1) * NC + i];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const bool has = (sl[k].x != 0) & (sl[k].y >= 0);
            const int nb = has ? sl[k].y : i;
            const int f = has ? slot_face(sl[k].x) : 0;
            const double sg = sl[k].x > 0 ? 1.0 : -1.0;
            const double *w = d.swp + size_t(f) * 4;
            const double *Unb = LowRec<D, S>::U(d, nb);
            const double *dUnb = LowRec<D, S>::dU(d, nb);
            double A[D], Um[nv], dUm[nv], Up[nv], Fa[nv], Fb[nv];
#pragma unroll
            for (int a = 0; a < D; ++a) A[a] = sg * w[a];
            const double sl_lam = w[D];
#pragma unroll
            for (int v = 0; v < nv; ++v) {
                Um[v] = Unb[v];
                dUm[v] = dUnb[v];
                Up[v] = Um[v] + dUm[v];
            }
            euler_flux<D>(Up, A, gamma, Fa);
            euler_flux<D>(Um, A, gamma, Fb);
#pragma unroll
            for (int v = 0; v < nv; ++v) acc[v] += has ? 0.5 * (Fa[v] - Fb[v]) - 0.5 * sl_lam * dUm[v] : 0.0;
        }
#pragma unroll
        for (int v = 0; v < nv; ++v) acc[v] = group_sum<SL, S>(acc[v]);
        if (!ok || !active) return;
        double *dUi = LowRec<D, S>::dU(d, i);
        const double iD = recip<double>(Di);
#pragma unroll
        for (int v = 0; v < nv; ++v)
            if (v % SL == q) dUi[v] = ((v < SL ? rhs_q : rhs_last) - acc[v]) * iD;
    } else {
        // FP32 (lighter records): slot by slot, the loads guarded by the
        // slot's test, faster here than addressing everything up front
        const DevParams &P = d.prm[d.cell_case[i]];
#pragma unroll
        for (int s = q; s < T::ns; s += SL) {
            const int2 sl = d.slot[size_t(s) * NC + i];
            if (sl.x != 0 && sl.y >= 0) {
                const int nb = sl.y;
                const int f = slot_face(sl.x);
                const double sg = sl.x > 0 ? 1.0 : -1.0;
                const double *w = d.swp + size_t(f) * 4;
                const double *Unb = LowRec<D, S>::U(d, nb);
                const S *dUnb = LowRec<D, S>::dU(d, nb);
                float A[D], Um[nv], dUm[nv], dF[nv];
#pragma unroll
                for (int a = 0; a < D; ++a) A[a] = float(sg * w[a]);
                const float sl_lam = float(w[D]);
#pragma unroll
                for (int v = 0; v < nv; ++v) {
                    Um[v] = float(Unb[v]);
                    dUm[v] = dUnb[v];
                }
                euler_dflux<D, float>(Um, dUm, A, float(P.gamma), dF);
#pragma unroll
                for (int v = 0; v < nv; ++v) acc[v] += 0.5f * dF[v] - 0.5f * sl_lam * dUm[v];
            }
        }
#pragma unroll
        for (int v = 0; v < nv; ++v) acc[v] = group_sum<SL, S>(acc[v]);
        if (!ok || !P.active) return;
        const double iD = recip<double>(d.D[i]);
        S *dUi = LowRec<D, S>::dU(d, i);
#pragma unroll
        for (int v = 0; v < nv; ++v)
            if (v % SL == q) dUi[v] = S((d.RHS[size_t(v) * NC + i] - double(acc[v])) * iD);
    }
}

// W += (U + dU) - W_p0 (W_p0 = W); partial sums of |rho - rho^n| and rho^n.
// prolong = 0: sums only (explicit cycle).
template <int D, typename S> __global__ __launch_bounds__(kBlock) void k_prolong_res(Dev d, int prolong) {
    constexpr int nv = D + 2;
    __shared__ double sh[kBlock];
    const int b = blockIdx.x;
    const int cs = d.rb_case[b];
    const DevParams &P = d.prm[cs];
    const int n = d.rb_count[b];
    const int NC = d.NC;
    const int i0 = d.rb_start[b];
    const bool pro = prolong && P.active;
    // NB cells per thread at a time: every load of the batch first, then the
    // updates and sums in the cells' order (the stores would otherwise keep
    // each cell's loads behind the previous cell's stores)
    constexpr int NB = 4;
    double s0 = 0, s1 = 0;
    for (int k0 = int(threadIdx.x); k0 < n; k0 += NB * kBlock) {
        double up[NB][nv], w[NB][nv], wn[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int k = k0 + j * kBlock;
            const int i = i0 + (k < n ? k : 0);
            const double *U = LowRec<D, S>::U(d, i);
            const S *dU = LowRec<D, S>::dU(d, i);
#pragma unroll
            for (int v = 0; v < nv; ++v) {
                up[j][v] = U[v] + double(dU[v]);
                w[j][v] = d.st[size_t(i) * Rec<D>::sr + v];
            }
            wn[j] = d.Wn[i];
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int k = k0 + j * kBlock;
            if (k >= n) break;
            const int i = i0 + k;
            double r0 = w[j][0];
            if (pro) {
#pragma unroll
                for (int v = 0; v < nv; ++v) {
                    const double nw = w[j][v] + (up[j][v] - w[j][v]);
                    d.st[size_t(i) * Rec<D>::sr + v] = nw;
                    if (v == 0) r0 = nw;
                }
            }
            s0 += fabs(r0 - wn[j]);
            s1 += wn[j];
        }
    }
    s0 = block_reduce_sum(s0, sh);
    s1 = block_reduce_sum(s1, sh);
    if (threadIdx.x == 0) {
        d.part0[b] = s0;
        d.part1[b] = s1;
    }
}

// copy the per-case Res of the last cycle into slot k of a device history
__global__ void k_res_store(const double *res, double *hist, int n_case) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n_case) hist[c] = res[c];
}

// Force of the gas on the walls (slip and no-slip boundary faces) of each
// case: the momentum sums sum_g wJ F0 the latest stage-0 flux pass kept per
// boundary slot, one block per case over its boundary slots in order.
// Reduced on request only (not part of the cycle).
template <int D> __global__ __launch_bounds__(kBlock) void k_wall_force(Dev d) {
    __shared__ double sh[kBlock];
    const int c = blockIdx.x;
    double f[D];
#pragma unroll
    for (int a = 0; a < D; ++a) f[a] = 0.0;
    const int2 cb = d.case_b[c];
    for (int B = cb.x + threadIdx.x; B < cb.x + cb.y; B += kBlock) {
        const int F = d.bface[B];
        if (F < 0) continue;
        const int bc = d.fbc[F] & 7;
        if (bc != 1 && bc != 2 && bc != 3) continue;
#pragma unroll
        for (int a = 0; a < D; ++a) f[a] += d.wallf[size_t(B) * 3 + a];
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double t = block_reduce_sum(f[a], sh);
        if (threadIdx.x == 0) d.force[3 * c + a] = t;
    }
    if (D == 2 && threadIdx.x == 0) d.force[3 * c + 2] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_res_final(Dev d, int n_case) {
    __shared__ double sh[kBlock];
    const int c = blockIdx.x;
    if (!d.prm[c].active) return;
    double a = 0, b = 0;
    for (int k = d.case_rb_off[c] + threadIdx.x; k < d.case_rb_off[c + 1]; k += kBlock) {
        a += d.part0[k];
        b += d.part1[k];
    }
    a = block_reduce_sum(a, sh);
    b = block_reduce_sum(b, sh);
    if (threadIdx.x == 0) d.res[c] = a / b;
}

}  // namespace cgks
