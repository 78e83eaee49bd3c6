// qtm_body.h -- device code shared by the trajectory kernels (layouts, tableau,
// Philox, per-column controller); included by qtm_dense.hip and qtm_sparse.hip.
#pragma once
// HIP kernels for gfx950 (MI355X) of the quantum
// trajectories method: many independent state vectors evolved under
// M = -i H_eff with Dormand-Prince 5(4), norm-threshold jumps (the paper's
// Algorithm 1, Sec. 2.2), jump-time root finding on the dense output,
// channel selection, renormalisation and FP64 averaging on the device.
//
// Structure.  A workgroup owns NB "columns" (trajectory slots).  All columns
// of a workgroup share every product K = M W: with a dense M the product is a
// real-embedded GEMM on the matrix cores (16x16x4 MFMA, FP64 or FP32) with the
// column block W staged through LDS; with a sparse M it is a sliced-ELL SpMM,
// one thread per row, W in LDS.  Per-column control (step size, accept/reject,
// jumps, outputs) is scalar work of one thread per column on LDS state; the
// vector work is uniform across columns (per-column coefficients), so columns
// in different phases (segment start, stepping, idle) share the same passes.
// Reductions over the state dimension are done per column in a fixed order,
// so results do not depend on scheduling.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <climits>
#include <cfloat>
#include "qtm_internal.h"
#include <type_traits>
#include <algorithm>

namespace qtm {

#define QTM_DI __device__ __attribute__((always_inline)) inline

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ tableau
// Dormand & Prince (1980) 5(4) pair, FSAL; stage s (0-based) uses k_0..k_{s-1}.
__device__ __forceinline__ constexpr double dp_a(int s, int j) {
    return s == 1 ? (j == 0 ? 1.0 / 5 : 0.0)
         : s == 2 ? (j == 0 ? 3.0 / 40 : j == 1 ? 9.0 / 40 : 0.0)
         : s == 3 ? (j == 0 ? 44.0 / 45 : j == 1 ? -56.0 / 15 : j == 2 ? 32.0 / 9 : 0.0)
         : s == 4 ? (j == 0 ? 19372.0 / 6561 : j == 1 ? -25360.0 / 2187 : j == 2 ? 64448.0 / 6561
                   : j == 3 ? -212.0 / 729 : 0.0)
         : s == 5 ? (j == 0 ? 9017.0 / 3168 : j == 1 ? -355.0 / 33 : j == 2 ? 46732.0 / 5247
                   : j == 3 ? 49.0 / 176 : j == 4 ? -5103.0 / 18656 : 0.0)
         : s == 6 ? (j == 0 ? 35.0 / 384 : j == 1 ? 0.0 : j == 2 ? 500.0 / 1113 : j == 3 ? 125.0 / 192
                   : j == 4 ? -2187.0 / 6784 : j == 5 ? 11.0 / 84 : 0.0)
         : 0.0;
}
// nodes c_s: stage s evaluates the right-hand side at t + c_s h
__device__ __forceinline__ constexpr double dp_c(int s) {
    return s == 1 ? 1.0 / 5 : s == 2 ? 3.0 / 10 : s == 3 ? 4.0 / 5 : s == 4 ? 8.0 / 9 : s >= 5 ? 1.0 : 0.0;
}
// error weights e_j = b_j - b*_j (7 stages)
__device__ __forceinline__ constexpr double dp_e(int j) {
    return j == 0 ? 35.0 / 384 - 5179.0 / 57600 : j == 1 ? 0.0 : j == 2 ? 500.0 / 1113 - 7571.0 / 16695
         : j == 3 ? 125.0 / 192 - 393.0 / 640 : j == 4 ? -2187.0 / 6784 + 92097.0 / 339200
         : j == 5 ? 11.0 / 84 - 187.0 / 2100 : -1.0 / 40;
}
// dense-output weights (Hairer, Norsett & Wanner, Sec. II.6)
__device__ __forceinline__ constexpr double dp_d(int j) {
    return j == 0 ? -12715105075.0 / 11282082432.0 : j == 1 ? 0.0 : j == 2 ? 87487479700.0 / 32700410799.0
         : j == 3 ? -10690763975.0 / 1880347072.0 : j == 4 ? 701980252875.0 / 199316789632.0
         : j == 5 ? -1453857185.0 / 822651844.0 : 69997945.0 / 29380423.0;
}

// ------------------------------------------------------------------ Philox
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11).
__device__ __forceinline__ void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = 0xD2E7470EE14C6C93ULL, m1 = 0xCA5A826395121157ULL;
        uint64_t lo0 = m0 * c[0], hi0 = __umul64hi(m0, c[0]);
        uint64_t lo1 = m1 * c[2], hi1 = __umul64hi(m1, c[2]);
        uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
}
__device__ __forceinline__ double u53(uint64_t x) { return ((double)(x >> 11) + 0.5) * 0x1.0p-53; }

// x^(-1/5) for x > 0: FP32 seed, then two Newton steps on g^5 x = 1 in FP64
// (relative error ~1e-16; far cheaper in registers than the double-double pow).
__device__ __forceinline__ double inv_fifth_root(double x) {
    double g = (double)exp2f(-0.2f * log2f((float)x));
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        double g2 = g * g;
        double e = 1.0 - x * (g2 * g2 * g);        // residual of g^5 x = 1
        g = fma(g, 0.2 * e, g);                      // g (1 + e/5)
    }
    return g;
}
// 2^(k/4) for integer k, exactly: 2^floor(k/4) times a correctly rounded 2^(m/4)
__device__ __forceinline__ double exp2_quarter(int k) {
    const double f[4] = {1.0, 1.18920711500272106672, 1.41421356237309504880, 1.68179283050742908606};
    int q = k >> 2;                                   // floor division
    return ldexp(f[k & 3], q);
}
// The learned form's first step from the network's log-step lh: h = 2^(k/4) with
// k = round(4 log2 h), log2 h first limited to [-40, 10] (a non-finite output takes the
// lower end) so that the step is positive and finite whatever the network returns
__device__ __forceinline__ double snap_proposal(float lh) {
    double l2 = (double)lh / 0.69314718055994530942;
    if (!(l2 >= -40.0)) l2 = -40.0;
    if (l2 > 10.0) l2 = 10.0;
    return exp2_quarter((int)rint(4.0 * l2));
}

// ------------------------------------------------------------------ complex
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 cfma(double s, double2 a, double2 acc) {
    return make_double2(fma(s, a.x, acc.x), fma(s, a.y, acc.y));
}
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double2 to_d2(double2 a) { return a; }
__device__ __forceinline__ double2 to_d2(float2 a) { return make_double2((double)a.x, (double)a.y); }
template <class V> __device__ __forceinline__ V from_d2(double2 a);
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 a) { return a; }
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }

// ------------------------------------------------------------------ column state (LDS)
struct Col {
    double t, h, h0, d1, r, u;   // time, step, probe step, starting-step norm, threshold, channel uniform
    double tb, fac, th;          // step end (or jump time), step factor, jump theta
    double err, n2;              // error norm, norm^2 of the step result
    double oth;                  // theta of the current output evaluation
    double pch;                  // probability of the chosen channel
    double tseg;                 // start time of the current segment
    long long traj;              // relative trajectory index, -1 when empty
    int state, action, seg, kk;
    int nacc, nrej, njump, natt;
    int last, rejected, omode, ch;
    int seg_rec;                 // segment records written
    int first_acc;
};

// ------------------------------------------------------------------ layouts
// Real embedding of a complex d-vector for the MFMA path: each 16-row tile
// holds 8 complex components.  The FP64 16x16x4 MFMA returns rows
// lg + 4 i (i = 0..3) to lane group lg, the FP32 one rows 4 lg + i; the row
// order is chosen per precision so that a lane always holds (re, im) of two
// whole components: acc = (Re q0, Im q0, Re q1, Im q1).
// Loads through pointers known to address global memory.  Pointers read from the
// LDS copy of the system descriptor are otherwise generic, and a generic (flat)
// load waits on the LDS counter as well.
typedef double gd2_t __attribute__((ext_vector_type(2)));
typedef float gf2_t __attribute__((ext_vector_type(2)));
QTM_DI int gload(const int* p, int i) { return ((const __attribute__((address_space(1))) int*)p)[i]; }
QTM_DI double gload(const double* p, int i) { return ((const __attribute__((address_space(1))) double*)p)[i]; }
QTM_DI double2 gload(const double2* p, int i) {
    const gd2_t v = ((const __attribute__((address_space(1))) gd2_t*)p)[i];
    return make_double2(v.x, v.y);
}
QTM_DI float2 gload(const float2* p, int i) {
    const gf2_t v = ((const __attribute__((address_space(1))) gf2_t*)p)[i];
    return make_float2(v.x, v.y);
}

template <int PREC> struct RowMap;
template <> struct RowMap<0> {
    __device__ static int comp(int rt, int lg, int m) { return 8 * rt + lg + 4 * m; }
    __device__ static int row(int q, int p) { return 16 * (q >> 3) + 4 * (2 * ((q & 7) >> 2) + p) + (q & 3); }
};
template <> struct RowMap<1> {
    __device__ static int comp(int rt, int lg, int m) { return 8 * rt + 2 * lg + m; }
    __device__ static int row(int q, int p) { return 2 * q + p; }
};

template <int PREC> struct MfmaT;
template <> struct MfmaT<0> {
    typedef double in_t; typedef d4 acc_t;
    __device__ static acc_t op(in_t a, in_t b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static const in_t* frag(const DevSystem& s) { return s.Mfrag; }
    __device__ static const in_t* team(const DevSystem& s) { return s.Mteam; }
    __device__ static const in_t* td(const DevSystem& s) { return s.Mtd; }
};
template <> struct MfmaT<1> {
    typedef float in_t; typedef f4 acc_t;
    __device__ static acc_t op(in_t a, in_t b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static const in_t* frag(const DevSystem& s) { return s.Mfrag32; }
    __device__ static const in_t* team(const DevSystem& s) { return s.Mteam32; }
    __device__ static const in_t* td(const DevSystem& s) { return s.Mtd32; }
};

// Dense layout: wave w handles column tile ct = w / wpc (16 columns, one per
// lane & 15) and row tiles rg*T .. rg*T+T-1 of the real-embedded operator.
template <int T, int PREC> struct DenseLayout {
    static constexpr int NE = 2 * T;    // complex elements per lane
    static constexpr int CPT = 1;       // columns per lane
    static constexpr int GMAX = 7;      // observables per output reduction
    typedef typename std::conditional<PREC == 0, double2, float2>::type kv_t;   // stage vectors
    typedef typename MfmaT<PREC>::in_t in_t;
    int lane, w, lg, c16, ct, rg, wpc, nct, NB, RT, KB, dp, d;
    bool active;
    const DevSystem* S;
    in_t* Wb;                           // LDS: [nct][2dp][16] operand staging
    double2* Stage;                     // LDS alias: [dp][NB] complex staging
    const in_t* Mf;                     // A fragments (LDS copy or global)
    double* red;                        // LDS: [NW][16][kNVMax]

    QTM_DI int qraw(int e) const {
        int rt = rg * T + (e >> 1);
        return (active && rt < RT) ? RowMap<PREC>::comp(rt, lg, e & 1) : -1;
    }
    QTM_DI int comp(int e) const { int q = qraw(e); return q < d ? q : -1; }
    QTM_DI int slot(int) const { return 0; }
    // distinct rows of a lane (each element its own row)
    static constexpr int NRW = NE;
    QTM_DI int row_q(int r) const { return comp(r); }
    static constexpr int erow(int e) { return e; }
    QTM_DI int gcol(int) const { return active ? ct * 16 + c16 : -1; }

    // K = M W for every column of the block.
    QTM_DI void rhs(const double2 (&W)[NE], kv_t (&K)[NE]) {
        if (active) {
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                int q = qraw(e);
                if (q >= 0) {   // padded components (d <= q < dp) are staged as zeros
                    in_t* base = Wb + (size_t)ct * 2 * dp * 16 + c16;
                    base[RowMap<PREC>::row(q, 0) * 16] = q < d ? (in_t)W[e].x : (in_t)0;
                    base[RowMap<PREC>::row(q, 1) * 16] = q < d ? (in_t)W[e].y : (in_t)0;
                }
            }
        }
        __syncthreads();
        if (active) {
            typename MfmaT<PREC>::acc_t acc[T][2];
#pragma unroll
            for (int t = 0; t < T; ++t) { acc[t][0] = 0; acc[t][1] = 0; }
            const in_t* bb = Wb + (size_t)ct * 2 * dp * 16 + lg * 16 + c16;
            for (int kb = 0; kb < KB; kb += 2) {
                in_t b0 = bb[(4 * kb) * 16];
                in_t b1 = (kb + 1 < KB) ? bb[(4 * kb + 4) * 16] : (in_t)0;
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    int rt = rg * T + t;
                    if (rt < RT) {
                        const in_t* af = Mf + ((size_t)rt * KB + kb) * 64 + lane;
                        acc[t][0] = MfmaT<PREC>::op(af[0], b0, acc[t][0]);
                        if (kb + 1 < KB) acc[t][1] = MfmaT<PREC>::op(af[64], b1, acc[t][1]);
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < T; ++t) {
                K[2 * t + 0] = from_d2<kv_t>(make_double2((double)acc[t][0][0] + (double)acc[t][1][0], (double)acc[t][0][1] + (double)acc[t][1][1]));
                K[2 * t + 1] = from_d2<kv_t>(make_double2((double)acc[t][0][2] + (double)acc[t][1][2], (double)acc[t][0][3] + (double)acc[t][1][3]));
            }
        }
        __syncthreads();
    }

    // Per-column sums of NV partial values: result for column c, value v is
    // red_sum(c, v) after the call (fixed order over waves).
    template <int NV> QTM_DI void reduce(double (&p)[CPT][NV]) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double x = p[0][v];
            x += __shfl_xor(x, 16);
            x += __shfl_xor(x, 32);
            p[0][v] = x;
        }
        if (active && lg == 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v) red[(w * 16 + c16) * kNVMax + v] = p[0][v];
        }
        __syncthreads();
    }
    QTM_DI double red_sum(int c, int v) const {
        int cct = c >> 4, cc = c & 15;
        double s = 0.0;
        for (int g = 0; g < wpc; ++g) s += red[((cct * wpc + g) * 16 + cc) * kNVMax + v];
        return s;
    }
};

// Sparse layout: thread tid owns rows tid + r*blockDim (r < RPT) for all NB columns.
template <int RPT, int NBC, int PREC> struct SparseLayout {
    static constexpr int NE = RPT * NBC;
    static constexpr int CPT = NBC;
    static constexpr int GMAX = NBC == 1 ? 7 : 2;
    typedef typename std::conditional<PREC == 0, double2, float2>::type kv_t;
    int tid, nthr, lane, w, NW, d, NB, dp;
    const DevSystem* S;
    double2* Stage;                     // LDS: [d][NB] complex (FP64) staging
    float2* Stage32;                    // LDS alias for FP32 products
    double* red;                        // LDS: [NW][NB][kNVMax]
    // LDS-resident sliced ELL (when ell_lds): values, 16-bit columns, slice offsets and widths
    int ell_lds;
    const double2* lval;
    const float2* lval32;
    const unsigned short* lcol;
    const int* lsoff;
    const int* lsw;
    typedef typename std::conditional<PREC == 0, double2, float2>::type vt_t;   // product arithmetic

    QTM_DI const vt_t* lvals() const { return PREC == 0 ? (const vt_t*)lval : (const vt_t*)lval32; }
    QTM_DI vt_t stage_at(int i) const { return PREC == 0 ? ((const vt_t*)Stage)[i] : ((const vt_t*)Stage32)[i]; }

    QTM_DI int comp(int e) const { int q = tid + (e / NBC) * nthr; return q < d ? q : -1; }
    QTM_DI int slot(int e) const { return e % NBC; }
    // distinct rows of a thread: element e is row e / NBC of column e % NBC
    static constexpr int NRW = RPT;
    QTM_DI int row_q(int r) const { return comp(r * NBC); }
    static constexpr int erow(int e) { return e / NBC; }
    QTM_DI int gcol(int s) const { return s; }

    // NR rows (r0 .. r0+NR-1 of this thread) of K = M W over the block's NBC columns.
    // LDSM: the sliced ELL is resident in LDS; otherwise it is read from global
    // memory.  Slice widths are multiples of four (zero-valued padding).  The 64 rows
    // of a wavefront share one slice (blocks are a multiple of 64 threads), so offsets
    // and widths are wave-uniform.  Entries go in groups of four per row, the NR rows'
    // groups side by side: all their column and value loads are issued together, then
    // all staged-vector reads, then the arithmetic.  A row whose slice is narrower than
    // the widest re-reads its first group with the values zeroed.
    template <bool LDSM, int NR> QTM_DI void rows(int r0, vt_t (&acc)[NR][NBC]) const {
        int off[NR], wd[NR], wmax = 0;
        const int ln = tid & 63;
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int sl = (tid + (r0 + i) * nthr) >> 6;
            const bool in = sl * 64 < d;            // wave-uniform: the slice exists
            off[i] = __builtin_amdgcn_readfirstlane(in ? (LDSM ? lsoff[sl] : gload(S->sl_off, sl)) : 0);
            wd[i] = __builtin_amdgcn_readfirstlane(in ? (LDSM ? lsw[sl] : gload(S->sl_w, sl)) : 0);
            wmax = wd[i] > wmax ? wd[i] : wmax;
#pragma unroll
            for (int b = 0; b < NBC; ++b) { acc[i][b].x = 0; acc[i][b].y = 0; }
        }
        const vt_t* gval = PREC == 0 ? (const vt_t*)S->sl_val : (const vt_t*)S->sl_val32;
        const int* gcol = S->sl_col;
        for (int p = 0; p < wmax; p += 4) {
            int c[NR][4];
            vt_t v[NR][4];
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                const bool live = p < wd[i];
                const int base = off[i] + (live ? p : 0) * 64 + ln;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int idx = base + j * 64;
                    c[i][j] = LDSM ? (int)lcol[idx] : gload(gcol, idx);
                    v[i][j] = LDSM ? lvals()[idx] : gload(gval, idx);
                    if (!live) { v[i][j].x = 0; v[i][j].y = 0; }
                }
            }
            vt_t x[NR][4][NBC];
#pragma unroll
            for (int i = 0; i < NR; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int b = 0; b < NBC; ++b) x[i][j][b] = stage_at(c[i][j] * NBC + b);
#pragma unroll
            for (int i = 0; i < NR; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int b = 0; b < NBC; ++b) {
                        acc[i][b].x = fma(v[i][j].x, x[i][j][b].x, fma(-v[i][j].y, x[i][j][b].y, acc[i][b].x));
                        acc[i][b].y = fma(v[i][j].x, x[i][j][b].y, fma(v[i][j].y, x[i][j][b].x, acc[i][b].y));
                    }
        }
    }

    QTM_DI void rhs(const double2 (&W)[NE], kv_t (&K)[NE]) {
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            int q = comp(e);
            if (q >= 0) {
                if (PREC == 0) Stage[q * NBC + slot(e)] = W[e];
                else Stage32[q * NBC + slot(e)] = make_float2((float)W[e].x, (float)W[e].y);
            }
        }
        __syncthreads();
        // FP32 products: up to four of a thread's rows side by side; FP64: one (register room)
        constexpr int NR = (PREC == 1 && RPT >= 2) ? (RPT >= 4 ? 4 : RPT) : 1;
#pragma unroll
        for (int r = 0; r < RPT; r += NR) {
            vt_t acc[NR][NBC];
            if (ell_lds) rows<true, NR>(r, acc);
            else rows<false, NR>(r, acc);
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                const bool in = tid + (r + i) * nthr < d;
#pragma unroll
                for (int b = 0; b < NBC; ++b)
                    K[(r + i) * NBC + b] = in ? from_d2<kv_t>(make_double2(acc[i][b].x, acc[i][b].y)) : from_d2<kv_t>(make_double2(0.0, 0.0));
            }
        }
        __syncthreads();
    }

    template <int NV> QTM_DI void reduce(double (&p)[CPT][NV]) {
#pragma unroll
        for (int b = 0; b < NBC; ++b)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double x = p[b][v];
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) x += __shfl_xor(x, o);
                p[b][v] = x;
            }
        if (lane == 0) {
#pragma unroll
            for (int b = 0; b < NBC; ++b)
#pragma unroll
                for (int v = 0; v < NV; ++v) red[(w * NBC + b) * kNVMax + v] = p[b][v];
        }
        __syncthreads();
    }
    QTM_DI double red_sum(int c, int v) const {
        double s = 0.0;
        for (int g = 0; g < NW; ++g) s += red[(g * NBC + c) * kNVMax + v];
        return s;
    }
};

// ------------------------------------------------------------------ proposal MLP (inference)
__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

// FP32 accumulation on BF16-valued weights; one thread.
static __device__ __noinline__ float mlp_logh(const float* P, const float* f) {
    const float* W1 = P;
    const float* b1 = W1 + kNH * kNF;
    const float* W2 = b1 + kNH;
    const float* b2 = W2 + kNH * kNH;
    const float* W3 = b2 + kNH;
    const float* b3 = W3 + kNO * kNH;
    const float* mu = b3 + kNO;
    const float* sd = mu + kNF;
    float x[kNF], a1[kNH];
    for (int i = 0; i < kNF; ++i) x[i] = (f[i] - mu[i]) / sd[i];
    for (int h = 0; h < kNH; ++h) {
        float s = b1[h];
        for (int i = 0; i < kNF; ++i) s = fmaf(W1[h * kNF + i], x[i], s);
        a1[h] = gelu_f(s);
    }
    float o = b3[0];
    for (int h = 0; h < kNH; ++h) {
        float s = b2[h];
        for (int i = 0; i < kNH; ++i) s = fmaf(W2[h * kNH + i], a1[i], s);
        o = fmaf(W3[h], gelu_f(s), o);
    }
    return o;
}

// ------------------------------------------------------------------ the trajectory kernel body
// Values reduced per column in the different phases.
// dense output u(th) = y + th (D + (1-th)(B + th (R4 + (1-th) R5)))
//   D = yn - y, B = h k1 - D, R4 = D - h k7 - B, R5 = h sum_j d_j k_j
template <class L>
struct Body {
    L& Ly;
    const DevSystem& S;
    const RunArgs& A;
    Col* cs;
    int* flags;

    unsigned long long passes = 0;   // product passes of this block (thread 0), added once at exit
    unsigned long long roots = 0;    // norm-polynomial evaluations of the jump-time root finds of
                                     // this thread's columns, added once at exit
    // vectors (registers): state and step result in FP64, stage derivatives in the product precision
    typedef typename L::kv_t kv_t;
    double2 y[L::NE], yn[L::NE];
    kv_t k[7][L::NE];

    QTM_DI Body(L& l, const DevSystem& s, const RunArgs& a, Col* c, int* f) : Ly(l), S(s), A(a), cs(c), flags(f) {}

    QTM_DI double2 dense_at(int e, double th, const Col& c) const {
        double2 D = csub(yn[e], y[e]);
        if constexpr (sizeof(kv_t) == 8) {
            // FP32 products: B, R4, R5 and the two inner levels in FP32 (the stage
            // vectors are FP32); the outer two levels, with y and D, in FP64
            const float hf = (float)c.h, thf = (float)th, t1f = 1.f - thf;
            const float Dx = (float)D.x, Dy = (float)D.y;
            const float2 k1 = (const float2&)k[0][e], k7 = (const float2&)k[6][e];
            const float Bx = fmaf(hf, k1.x, -Dx), By = fmaf(hf, k1.y, -Dy);
            const float R4x = Dx - fmaf(hf, k7.x, Bx), R4y = Dy - fmaf(hf, k7.y, By);
            float R5x = 0.f, R5y = 0.f;
#pragma unroll
            for (int j = 0; j < 7; ++j)
                if (dp_d(j) != 0.0) {
                    const float2 kj = (const float2&)k[j][e];
                    R5x = fmaf((float)dp_d(j), kj.x, R5x);
                    R5y = fmaf((float)dp_d(j), kj.y, R5y);
                }
            R5x *= hf;
            R5y *= hf;
            const float ix = fmaf(thf, fmaf(t1f, R5x, R4x), Bx), iy = fmaf(thf, fmaf(t1f, R5y, R4y), By);
            const double t1 = 1.0 - th;
            return make_double2(fma(th, fma(t1, (double)ix, D.x), y[e].x), fma(th, fma(t1, (double)iy, D.y), y[e].y));
        }
        double2 B = csub(cscale(c.h, to_d2(k[0][e])), D);
        double2 R4 = csub(csub(D, cscale(c.h, to_d2(k[6][e]))), B);
        double2 R5 = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < 7; ++j)
            if (dp_d(j) != 0.0) R5 = cfma(c.h * dp_d(j), to_d2(k[j][e]), R5);
        double t1 = 1.0 - th;
        double2 in = cadd(R4, cscale(t1, R5));
        in = cadd(B, cscale(th, in));
        in = cadd(D, cscale(t1, in));
        return cadd(y[e], cscale(th, in));
    }

    // vector for output mode: 1 current y, 2 yn, 3 dense output at theta
    QTM_DI double2 vec_mode(int e, const Col& c) const {
        return c.omode == 1 ? y[e] : c.omode == 2 ? yn[e] : dense_at(e, c.oth, c);
    }

    // Products with CSR operators (collapse or observable) on a staged vector.
    QTM_DI double2 csr_row(const int* rp, const int* ci, const double2* val, int q, int gc) const {
        double2 s = make_double2(0.0, 0.0);
        const int p1 = gload(rp, q + 1);
        for (int p = gload(rp, q); p < p1; ++p) s = cadd(s, cmul(gload(val, p), Ly.Stage[gload(ci, p) * Ly.NB + gc]));
        return s;
    }

    // Stage per-column vectors selected by omode into the complex staging buffer.
    QTM_DI void stage_mode() {
#pragma unroll
        for (int e = 0; e < L::NE; ++e) {
            int q = Ly.comp(e), gc = Ly.gcol(Ly.slot(e));
            if (q >= 0 && gc >= 0) {
                const Col& c = cs[gc];
                Ly.Stage[q * Ly.NB + gc] = c.omode ? vec_mode(e, c) : make_double2(0.0, 0.0);
            }
        }
        __syncthreads();
    }

    // One round of output evaluation for all columns with omode != 0:
    // values per column: <u|u>, then (re, im) of <u|O_e|u> for G observables.
    template <int G> QTM_DI void output_group(int e0) {
        constexpr int NV = 1 + 2 * G;
        double p[L::CPT][NV];
#pragma unroll
        for (int b = 0; b < L::CPT; ++b)
#pragma unroll
            for (int v = 0; v < NV; ++v) p[b][v] = 0.0;
#pragma unroll
        for (int e = 0; e < L::NE; ++e) {
            int q = Ly.comp(e), gc = Ly.gcol(Ly.slot(e));
            if (q < 0 || gc < 0) continue;
            const Col& c = cs[gc];
            if (!c.omode) continue;
            double2 u = vec_mode(e, c);
            double a2 = cabs2(u);
            p[Ly.slot(e)][0] += a2;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                int o = e0 + g;
                if (o >= S.n_e) break;
                if (S.e_fmt[o] == 2) {
                    double2 dv = gload(S.e_val, S.e_doff[o] + q);
                    p[Ly.slot(e)][1 + 2 * g] += dv.x * a2;
                    p[Ly.slot(e)][2 + 2 * g] += dv.y * a2;
                } else {
                    double2 Ou = csr_row(S.e_rp + (size_t)o * (S.d + 1), S.e_ci, S.e_val, q, gc);
                    p[Ly.slot(e)][1 + 2 * g] += u.x * Ou.x + u.y * Ou.y;     // Re conj(u) Ou
                    p[Ly.slot(e)][2 + 2 * g] += u.x * Ou.y - u.y * Ou.x;     // Im conj(u) Ou
                }
            }
        }
        Ly.template reduce<NV>(p);
        int tid = threadIdx.x;
        if (tid < Ly.NB) {
            Col& c = cs[tid];
            if (c.omode) {
                double nn = Ly.red_sum(tid, 0);
                for (int g = 0; g < G && e0 + g < S.n_e; ++g) {
                    double re = Ly.red_sum(tid, 1 + 2 * g) / nn;
                    double im = Ly.red_sum(tid, 2 + 2 * g) / nn;
                    S.X[((size_t)c.traj * S.n_e + e0 + g) * S.n_t + c.kk] = make_double2(re, im);
                }
            }
        }
        __syncthreads();
    }

    // All observables diagonal: |u_q|^2 of every element is formed once per round
    // (a2, zero for columns without an output) and feeds the norm and each of the
    // group's G observables.  The group's diagonal values are loaded once per distinct
    // row of the thread, all before any is used; REAL (every observable real): the
    // real parts only.  One block reduction of 1 + G (REAL) or 1 + 2G values.
    template <int G, bool REAL> QTM_DI void output_group_diag(int e0, const double (&a2)[L::NE]) {
        constexpr int NV = REAL ? 1 + G : 1 + 2 * G;
        double p[L::CPT][NV];
#pragma unroll
        for (int b = 0; b < L::CPT; ++b)
#pragma unroll
            for (int v = 0; v < NV; ++v) p[b][v] = 0.0;
#pragma unroll
        for (int e = 0; e < L::NE; ++e) p[Ly.slot(e)][0] += a2[e];
        const int last = S.n_e - 1;
        typedef typename std::conditional<REAL, double, double2>::type ov_t;
        ov_t v[G][L::NRW];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int o = e0 + g < last ? e0 + g : last;        // clamped: every load in range
            const double2* dv = S.e_val + S.e_doff[o];
#pragma unroll
            for (int r = 0; r < L::NRW; ++r) {
                const int q = Ly.row_q(r);
                if constexpr (REAL) v[g][r] = gload((const double*)dv, 2 * (q >= 0 ? q : 0));
                else v[g][r] = gload(dv, q >= 0 ? q : 0);
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (e0 + g > last) break;
#pragma unroll
            for (int e = 0; e < L::NE; ++e) {
                const ov_t x = v[g][L::erow(e)];
                if constexpr (REAL) p[Ly.slot(e)][1 + g] += x * a2[e];
                else {
                    p[Ly.slot(e)][1 + 2 * g] += x.x * a2[e];
                    p[Ly.slot(e)][2 + 2 * g] += x.y * a2[e];
                }
            }
        }
        Ly.template reduce<NV>(p);
        const int tid = threadIdx.x;
        if (tid < Ly.NB) {
            Col& c = cs[tid];
            if (c.omode) {
                const double nn = Ly.red_sum(tid, 0);
                for (int g = 0; g < G && e0 + g < S.n_e; ++g) {
                    const double re = Ly.red_sum(tid, REAL ? 1 + g : 1 + 2 * g) / nn;
                    const double im = REAL ? 0.0 : Ly.red_sum(tid, 2 + 2 * g) / nn;
                    S.X[((size_t)c.traj * S.n_e + e0 + g) * S.n_t + c.kk] = make_double2(re, im);
                }
            }
        }
        __syncthreads();
    }

    QTM_DI void output_round() {
        // the single-pass diagonal path for FP32 products; with FP64 stage vectors its
        // extra live registers cost more in the stage code than it saves here
        if (sizeof(kv_t) == 8 && !S.any_csr_e) {
            double a2[L::NE];
#pragma unroll
            for (int e = 0; e < L::NE; ++e) {
                const int q = Ly.comp(e), gc = Ly.gcol(Ly.slot(e));
                a2[e] = 0.0;
                if (q >= 0 && gc >= 0) {
                    const Col& c = cs[gc];
                    if (c.omode) a2[e] = cabs2(vec_mode(e, c));
                }
            }
            bool real = true;
            for (int o = 0; o < S.n_e; ++o) real = real && S.e_nv[o] == 1;
            for (int e0 = 0; e0 < S.n_e;) {
                if (real) {
                    if (S.n_e - e0 <= 3) { output_group_diag<3, true>(e0, a2); e0 += 3; }
                    else { output_group_diag<7, true>(e0, a2); e0 += 7; }
                } else {
                    output_group_diag<3, false>(e0, a2); e0 += 3;
                }
            }
            return;
        }
        if (S.any_csr_e) stage_mode();
        for (int e0 = 0; e0 < S.n_e;) {
            if (S.n_e - e0 <= 2 || L::GMAX == 2) { output_group<2>(e0); e0 += 2; }
            else { output_group<(L::GMAX > 2 ? L::GMAX : 2)>(e0); e0 += L::GMAX; }
        }
    }

    // Controller helper: set omode for the next pending output; returns 1 if any.
    // phase 0: new trajectory (t_k == t), 1: accepted step (t < t_k <= tb),
    // 2: before a jump (t < t_k < tb), 3: after a jump (t_k == tb, current y)
    QTM_DI void next_output(Col& c) {
        c.omode = 0;
        if (c.kk >= S.n_t) return;
        double tk = S.tlist[c.kk];
        if (c.action == ACT_NONE && c.state == ST_NEW) {
            if (tk == c.t) c.omode = 1;
        } else if (c.action == ACT_ACCEPT) {
            if (tk <= c.tb) {
                if (tk == c.tb) c.omode = 2;
                else { c.omode = 3; c.oth = (tk - c.t) / c.h; }
            }
        } else if (c.action == ACT_JUMP) {
            if (tk < c.tb) { c.omode = 3; c.oth = (tk - c.t) / c.h; }
        } else if (c.action == ACT_POSTJUMP) {   // post-jump outputs at the jump time
            if (tk == c.t) c.omode = 1;
        }
    }

    QTM_DI void outputs_loop(int phase) {
        for (;;) {
            int tid = threadIdx.x;
            if (tid == 0) flags[1] = 0;
            __syncthreads();
            if (tid < Ly.NB) {
                Col& c = cs[tid];
                c.omode = 0;
                bool want = (phase == 0 && c.state == ST_NEW) ||
                            (phase == 1 && (c.action == ACT_ACCEPT || c.action == ACT_JUMP)) ||
                            (phase == 3 && c.action == ACT_POSTJUMP);
                if (want) next_output(c);
                if (c.omode) atomicOr(&flags[1], 1);
            }
            __syncthreads();
            if (!flags[1]) break;
            output_round();
            if (tid < Ly.NB) {
                Col& c = cs[tid];
                if (c.omode) c.kk++;
            }
            __syncthreads();
        }
    }

    // Finish a trajectory (done or failed): per-trajectory counters.
    QTM_DI void retire(Col& c, bool failed) {
        int* st = S.tstat + (size_t)c.traj * 4;
        st[0] = c.nacc; st[1] = c.nrej; st[2] = c.seg + 1; st[3] = c.njump;
        S.jn[c.traj] = c.njump;
        if (failed) atomicMin((unsigned long long*)A.fail, (unsigned long long)(S.traj_begin + c.traj));
        c.state = ST_EMPTY;
        c.traj = -1;
    }

    // ---------------------------------------------------------------- main loop
    QTM_DI void run() {
        const int tid = threadIdx.x;
        const int NB = Ly.NB;
        const double tend = S.tend;
        bool exhausted = false;
        if (tid < NB) { cs[tid].state = ST_EMPTY; cs[tid].traj = -1; cs[tid].action = ACT_NONE; cs[tid].omode = 0; }
#pragma unroll
        for (int e = 0; e < L::NE; ++e) {
            y[e] = yn[e] = make_double2(0.0, 0.0);
#pragma unroll
            for (int j = 0; j < 7; ++j) k[j][e] = from_d2<kv_t>(make_double2(0.0, 0.0));
        }
        __syncthreads();
        long long cycles = 0;
        for (;;) {
            // ---- refill and segment starts (one thread per column)
            if (tid == 0) { flags[0] = 0; flags[2] = 0; flags[3] = 0; }
            __syncthreads();
            if (tid < NB) {
                Col& c = cs[tid];
                c.action = ACT_NONE;
                if (c.state == ST_EMPTY && !exhausted && (A.persistent || cycles == 0)) {
                    unsigned long long idx = atomicAdd(S.queue, 1ULL);
                    if ((long long)idx < S.count) {
                        c.traj = (long long)idx;
                        c.t = S.t0; c.seg = 0; c.kk = 0; c.nacc = c.nrej = c.njump = c.natt = 0;
                        c.rejected = 0; c.seg_rec = 0;
                        c.state = ST_NEW;
                    } else {
                        exhausted = true;
                    }
                }
                if (c.state != ST_EMPTY) atomicOr(&flags[0], 1);
                if (c.state == ST_NEW) atomicOr(&flags[2], 1);
            }
            __syncthreads();
            if (!flags[0]) break;
            if (++cycles > A.max_cycles) {      // failsafe: retire everything as failed
                if (tid < NB && cs[tid].state != ST_EMPTY) retire(cs[tid], true);
                __syncthreads();
                break;
            }
            if (flags[2]) {
                // load psi0 into new columns, outputs at t0
#pragma unroll
                for (int e = 0; e < L::NE; ++e) {
                    int q = Ly.comp(e), gc = Ly.gcol(Ly.slot(e));
                    if (gc >= 0 && cs[gc].state == ST_NEW) y[e] = q >= 0 ? S.psi0[q] : make_double2(0.0, 0.0);
                }
                outputs_loop(0);
                if (tid < NB && cs[tid].state == ST_NEW) cs[tid].state = ST_NEEDK1;
                __syncthreads();
            }
            // segment start: thresholds (Philox), flag for the k1 pass
            if (tid < NB) {
                Col& c = cs[tid];
                if (c.state == ST_NEEDK1) {
                    if (!(c.t < tend)) { retire(c, false); }
                    else if (c.natt >= A.max_steps) { retire(c, true); }
                    else {
                        c.tseg = c.t;
                        c.rejected = 0;         // the step controller restarts with the segment
                        uint64_t ctr[4] = {(uint64_t)(S.traj_begin + c.traj), (uint64_t)c.seg, 0, 0};
                        philox4x64(ctr, S.key0, S.key1);
                        c.r = u53(ctr[0]);
                        c.u = u53(ctr[1]);
                        c.first_acc = 1;
                        atomicOr(&flags[3], 1);
                    }
                }
            }
            __syncthreads();
            if (flags[3]) segment_start();
            // the last step of the span is clamped to end exactly at t_end
            if (tid < NB) {
                Col& c = cs[tid];
                if (c.state == ST_STEP) {
                    c.last = (c.t + c.h >= tend);
                    if (c.last) c.h = tend - c.t;
                }
            }
            __syncthreads();
            // ---- the six stage passes of the DOPRI5 step
            stages();
            // ---- error, norm, accept/reject, jumps, outputs
            post_step();
        }
    }

    // k1 = M y for new segments, then the starting step (or the proposal).
    QTM_DI void segment_start() {
        const int tid = threadIdx.x;
        kv_t K[L::NE];
        Ly.rhs(y, K);
        if (tid == 0) ++passes;
#pragma unroll
        for (int e = 0; e < L::NE; ++e) {
            int gc = Ly.gcol(Ly.slot(e));
            if (gc >= 0 && cs[gc].state == ST_NEEDK1) k[0][e] = K[e];
        }
        // segment-start features (learned form, or records for its training data):
        // 12 diagonal expectations, <C0^dag C0>, <C1^dag C1> (normalised), log r, elapsed fraction
        if (A.learned || A.seg_cap > 0) {
            double p[L::CPT][15];
#pragma unroll
            for (int b = 0; b < L::CPT; ++b)
#pragma unroll
                for (int v = 0; v < 15; ++v) p[b][v] = 0.0;
            if (tid < Ly.NB) cs[tid].omode = (cs[tid].state == ST_NEEDK1) ? 1 : 0;
            __syncthreads();
            stage_mode();
#pragma unroll
            for (int e = 0; e < L::NE; ++e) {
                int q = Ly.comp(e), gc = Ly.gcol(Ly.slot(e));
                if (q < 0 || gc < 0 || cs[gc].state != ST_NEEDK1) continue;
                double a2 = cabs2(y[e]);
                p[Ly.slot(e)][14] += a2;
#pragma unroll
                for (int f = 0; f < 12; ++f)
                    if (f < S.n_f) p[Ly.slot(e)][f] += S.f_diag[(size_t)f * S.d + q] * a2;
#pragma unroll
                for (int n = 0; n < 2; ++n)
                    if (n < S.n_c)
                        p[Ly.slot(e)][12 + n] += cabs2(csr_row(S.c_rp + (size_t)n * (S.d + 1), S.c_ci, S.c_val, q, gc));
            }
            Ly.template reduce<15>(p);
            if (tid < Ly.NB) {
                Col& c = cs[tid];
                c.omode = 0;
                if (c.state == ST_NEEDK1) {
                    float f[kNF];
                    double nn = Ly.red_sum(tid, 14);
#pragma unroll
                    for (int v = 0; v < 14; ++v) f[v] = (float)(Ly.red_sum(tid, v) / nn);
                    f[14] = logf((float)c.r);
                    f[15] = (float)((c.t - S.t0) / (S.tend - S.t0));
                    if (A.learned) {
                        float lh = mlp_logh(A.mlp, f);
                        double h = snap_proposal(lh);
                        c.h = fmin(h, S.tend - c.t);
                        c.state = ST_STEP;
                    }
                    if (A.seg_cap > 0 && c.seg_rec < A.seg_cap) {
                        float* rec = S.segs + ((size_t)c.traj * A.seg_cap + c.seg_rec) * kSegRec;
#pragma unroll
                        for (int v = 0; v < kNF; ++v) rec[v] = f[v];
                        rec[16] = 0.f; rec[17] = -1.f; rec[18] = 1.f; rec[19] = 1.f;
                    }
                }
            }
            __syncthreads();
        }
        if (!A.learned) {
            // starting step: d0 = ||y/sc||, d1 = ||f0/sc||, sc = atol + rtol |y|
            double p[L::CPT][2];
#pragma unroll
            for (int b = 0; b < L::CPT; ++b) p[b][0] = p[b][1] = 0.0;
#pragma unroll
            for (int e = 0; e < L::NE; ++e) {
                int q = Ly.comp(e), gc = Ly.gcol(Ly.slot(e));
                if (q < 0 || gc < 0) continue;
                double sc = A.atol + A.rtol * sqrt(cabs2(y[e]));
                double isc2 = 1.0 / (sc * sc);
                p[Ly.slot(e)][0] += cabs2(y[e]) * isc2;
                p[Ly.slot(e)][1] += cabs2(to_d2(k[0][e])) * isc2;
            }
            Ly.template reduce<2>(p);
            if (tid < Ly.NB) {
                Col& c = cs[tid];
                if (c.state == ST_NEEDK1) {
                    double d0 = sqrt(Ly.red_sum(tid, 0) / S.d), d1 = sqrt(Ly.red_sum(tid, 1) / S.d);
                    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
                    h0 = fmin(h0, S.tend - c.t);
                    c.h0 = h0; c.d1 = d1;
                    c.state = ST_NEEDF1;
                }
            }
            __syncthreads();
        }
    }

    // Stage passes: w_s = y + sum_j c_sj k_j with per-column coefficients, k_s = M w_s.
    template <int s> QTM_DI void one_stage() {
        double cf[6];
        double2 W[L::NE];
#pragma unroll
        for (int e = 0; e < L::NE; ++e) {
            int gc = Ly.gcol(Ly.slot(e));
            // per-column coefficients (columns owned by this element)
            int st = gc >= 0 ? cs[gc].state : ST_EMPTY;
            double h = gc >= 0 ? cs[gc].h : 0.0;
#pragma unroll
            for (int j = 0; j < 6; ++j) cf[j] = (st == ST_STEP) ? h * dp_a(s, j) : 0.0;
            if (s == 1 && st == ST_NEEDF1) cf[0] = cs[gc].h0;
            if constexpr (std::is_same<kv_t, float2>::value && s != 6) {
                // FP32 products: a stage input only feeds them, so it is y rounded to FP32
                // plus the FP32 increment (y_new, the last stage input, is formed in FP64)
                float ix = 0.f, iy = 0.f;
#pragma unroll
                for (int j = 0; j < s; ++j)
                    if (dp_a(s, j) != 0.0 || (s == 1 && j == 0)) {
                        const float2 kj = (const float2&)k[j][e];
                        ix = fmaf((float)cf[j], kj.x, ix);
                        iy = fmaf((float)cf[j], kj.y, iy);
                    }
                W[e] = make_double2((double)((float)y[e].x + ix), (double)((float)y[e].y + iy));
                continue;
            }
            double2 acc = y[e];
#pragma unroll
            for (int j = 0; j < s; ++j)
                if (dp_a(s, j) != 0.0 || (s == 1 && j == 0)) acc = cfma(cf[j], to_d2(k[j][e]), acc);
            W[e] = acc;
            if (s == 6) yn[e] = acc;
        }
        Ly.rhs(W, k[s]);
        if (threadIdx.x == 0) ++passes;
    }

    QTM_DI void stages() {
        const int tid = threadIdx.x;
        one_stage<1>();
        // starting-step probe finished for NEEDF1 columns: d2 = ||(f1 - f0)/sc|| / h0
        if (tid == 0) flags[4] = 0;
        __syncthreads();
        if (tid < Ly.NB && cs[tid].state == ST_NEEDF1) atomicOr(&flags[4], 1);
        __syncthreads();
        if (flags[4]) {
            double p[L::CPT][1];
#pragma unroll
            for (int b = 0; b < L::CPT; ++b) p[b][0] = 0.0;
#pragma unroll
            for (int e = 0; e < L::NE; ++e) {
                int q = Ly.comp(e), gc = Ly.gcol(Ly.slot(e));
                if (q < 0 || gc < 0) continue;
                double sc = A.atol + A.rtol * sqrt(cabs2(y[e]));
                p[Ly.slot(e)][0] += cabs2(csub(to_d2(k[1][e]), to_d2(k[0][e]))) / (sc * sc);
            }
            Ly.template reduce<1>(p);
            if (tid < Ly.NB) {
                Col& c = cs[tid];
                if (c.state == ST_NEEDF1) {
                    double d2 = sqrt(Ly.red_sum(tid, 0) / S.d) / c.h0;
                    double h1 = (c.d1 <= 1e-15 && d2 <= 1e-15) ? fmax(1e-6, c.h0 * 1e-3)
                                                               : 1.0 / inv_fifth_root(0.01 / fmax(c.d1, d2));
                    c.h = fmin(fmin(100.0 * c.h0, h1), S.tend - c.t);
                    c.state = ST_PROBED;
                }
            }
            __syncthreads();
        }
        one_stage<2>();
        one_stage<3>();
        one_stage<4>();
        one_stage<5>();
        one_stage<6>();
    }

    QTM_DI void post_step() {
        const int tid = threadIdx.x;
        const double tend = S.tend;
        // err^2 sum and ||yn||^2
        {
            double p[L::CPT][2];
#pragma unroll
            for (int b = 0; b < L::CPT; ++b) p[b][0] = p[b][1] = 0.0;
#pragma unroll
            for (int e = 0; e < L::NE; ++e) {
                int q = Ly.comp(e), gc = Ly.gcol(Ly.slot(e));
                if (q < 0 || gc < 0 || cs[gc].state != ST_STEP) continue;
                double h = cs[gc].h;
                double2 er = make_double2(0.0, 0.0);
#pragma unroll
                for (int j = 0; j < 7; ++j)
                    if (dp_e(j) != 0.0) er = cfma(h * dp_e(j), to_d2(k[j][e]), er);
                double sc = A.atol + A.rtol * sqrt(fmax(cabs2(y[e]), cabs2(yn[e])));   // = max(|y|, |y_new|): one root
                p[Ly.slot(e)][0] += cabs2(er) / (sc * sc);
                p[Ly.slot(e)][1] += cabs2(yn[e]);
            }
            Ly.template reduce<2>(p);
        }
        if (tid == 0) { flags[5] = 0; flags[6] = 0; }
        __syncthreads();
        if (tid < Ly.NB) {
            Col& c = cs[tid];
            c.action = ACT_NONE;
            if (c.state == ST_PROBED) c.state = ST_STEP;   // starting step known, step next cycle
            else if (c.state == ST_STEP) {
                c.natt++;
                double err = sqrt(Ly.red_sum(tid, 0) / S.d);
                c.n2 = Ly.red_sum(tid, 1);
                if (!(err <= 1.0)) {
                    double f = isfinite(err) ? fmax(0.2, 0.9 * inv_fifth_root(err)) : 0.2;
                    c.h *= f;
                    c.rejected = 1;
                    c.nrej++;
                    c.action = ACT_REJECT;
                    if (!(c.h > 16.0 * DBL_EPSILON * fabs(c.t)) || c.natt >= A.max_steps) c.action = ACT_FAIL;
                } else {
                    c.nacc++;
                    double fac = (err == 0.0) ? 10.0 : fmin(10.0, 0.9 * inv_fifth_root(err));
                    if (c.rejected) fac = fmin(1.0, fac);
                    c.fac = fac;
                    if (A.seg_cap > 0 && c.first_acc && c.seg_rec < A.seg_cap) {
                        float* rec = S.segs + ((size_t)c.traj * A.seg_cap + c.seg_rec) * kSegRec;
                        rec[17] = (float)(c.h * fac);
                    }
                    c.first_acc = 0;
                    c.tb = c.last ? tend : c.t + c.h;
                    if (S.n_c > 0 && c.n2 < c.r) { c.action = ACT_JUMP; atomicOr(&flags[5], 1); }
                    else {
                        c.action = ACT_ACCEPT;
                        if (!c.last && c.natt >= A.max_steps) c.action = ACT_FAIL;
                    }
                }
                if (c.action == ACT_ACCEPT) atomicOr(&flags[6], 1);
            }
        }
        __syncthreads();
        if (flags[5]) jump_time();
        if (flags[6] || flags[5]) outputs_loop(1);
        if (flags[5]) do_jump();
        // accepted steps: y <- yn, k1 <- k7 (FSAL), t <- tb
#pragma unroll
        for (int e = 0; e < L::NE; ++e) {
            int gc = Ly.gcol(Ly.slot(e));
            if (gc >= 0 && cs[gc].action == ACT_ACCEPT) { y[e] = yn[e]; k[0][e] = k[6][e]; }
        }
        __syncthreads();
        if (tid < Ly.NB) {
            Col& c = cs[tid];
            if (c.action == ACT_ACCEPT) {
                c.t = c.tb;
                c.h *= c.fac;
                c.rejected = 0;
                if (!(c.t < tend)) retire(c, false);
            } else if (c.action == ACT_FAIL) {
                retire(c, true);
            }
        }
        __syncthreads();
    }

    // Root of ||u(theta)||^2 = r on [0, 1] from the Gram matrix of
    // v = {y, D, B, R4, R5}: u = sum_p c_p(theta) v_p with
    // c = (1, th, th(1-th), th^2(1-th), th^2(1-th)^2).
    QTM_DI void jump_time() {
        const int tid = threadIdx.x;
        double p[L::CPT][15];
#pragma unroll
        for (int b = 0; b < L::CPT; ++b)
#pragma unroll
            for (int v = 0; v < 15; ++v) p[b][v] = 0.0;
#pragma unroll
        for (int e = 0; e < L::NE; ++e) {
            int q = Ly.comp(e), gc = Ly.gcol(Ly.slot(e));
            if (q < 0 || gc < 0 || cs[gc].action != ACT_JUMP) continue;
            const Col& c = cs[gc];
            double2 v[5];
            v[0] = y[e];
            v[1] = csub(yn[e], y[e]);
            v[2] = csub(cscale(c.h, to_d2(k[0][e])), v[1]);
            v[3] = csub(csub(v[1], cscale(c.h, to_d2(k[6][e]))), v[2]);
            double2 R5 = make_double2(0.0, 0.0);
#pragma unroll
            for (int j = 0; j < 7; ++j)
                if (dp_d(j) != 0.0) R5 = cfma(c.h * dp_d(j), to_d2(k[j][e]), R5);
            v[4] = R5;
            int n = 0;
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int b = a; b < 5; ++b) p[Ly.slot(e)][n++] += v[a].x * v[b].x + v[a].y * v[b].y;
        }
        Ly.template reduce<15>(p);
        if (tid < Ly.NB) {
            Col& c = cs[tid];
            if (c.action == ACT_JUMP) {
                double G[5][5];
#pragma unroll
                for (int a = 0; a < 5; ++a)
#pragma unroll
                    for (int b = a; b < 5; ++b) {
                        constexpr int dummy = 0; (void)dummy;
                        int n = a * 5 - a * (a - 1) / 2 + (b - a);
                        G[a][b] = G[b][a] = Ly.red_sum(tid, n);
                    }
                auto f = [&](double th) {
                    double t1 = 1.0 - th;
                    double cc[5] = {1.0, th, th * t1, th * th * t1, th * th * t1 * t1};
                    double s = 0.0;
#pragma unroll
                    for (int a = 0; a < 5; ++a)
#pragma unroll
                        for (int b = 0; b < 5; ++b) s += cc[a] * cc[b] * G[a][b];
                    return s - c.r;
                };
                double lo = 0.0, hi = 1.0;
                for (int m = 1; m <= 32; ++m) {
                    double th = (double)m / 32.0;
                    ++roots;
                    if (f(th) < 0.0) { hi = th; lo = (double)(m - 1) / 32.0; break; }
                }
                while (hi - lo > 1e-13) {
                    double mid = 0.5 * (lo + hi);
                    ++roots;
                    if (f(mid) < 0.0) hi = mid; else lo = mid;
                }
                c.th = 0.5 * (lo + hi);
                c.tb = c.t + c.th * c.h;       // jump time (outputs strictly before it)
            }
        }
        __syncthreads();
    }

    QTM_DI void do_jump() {
        const int tid = threadIdx.x;
        // psi* = u(theta*) staged; channel probabilities p_n = ||C_n psi*||^2
        if (tid < Ly.NB) {
            Col& c = cs[tid];
            if (c.action == ACT_JUMP) { c.omode = 3; c.oth = c.th; } else c.omode = 0;
        }
        __syncthreads();
        stage_mode();
        double pn[L::CPT][kMaxC];
#pragma unroll
        for (int b = 0; b < L::CPT; ++b)
#pragma unroll
            for (int n = 0; n < kMaxC; ++n) pn[b][n] = 0.0;
#pragma unroll
        for (int e = 0; e < L::NE; ++e) {
            int q = Ly.comp(e), gc = Ly.gcol(Ly.slot(e));
            if (q < 0 || gc < 0 || cs[gc].action != ACT_JUMP) continue;
#pragma unroll
            for (int n = 0; n < kMaxC; ++n)
                if (n < S.n_c)
                    pn[Ly.slot(e)][n] += cabs2(csr_row(S.c_rp + (size_t)n * (S.d + 1), S.c_ci, S.c_val, q, gc));
        }
        Ly.template reduce<kMaxC>(pn);
        if (tid < Ly.NB) {
            Col& c = cs[tid];
            if (c.action == ACT_JUMP) {
                double tot = 0.0;
                for (int n = 0; n < S.n_c; ++n) tot += Ly.red_sum(tid, n);
                int ch = -1;
                double pch = 0.0;
                if (tot > 0.0) {
                    double thr = c.u * tot, cum = 0.0;
                    for (int n = 0; n < S.n_c; ++n) {
                        double pv = Ly.red_sum(tid, n);
                        cum += pv;
                        if (pv > 0.0 && cum >= thr) { ch = n; pch = pv; break; }
                    }
                    if (ch < 0)
                        for (int n = S.n_c - 1; n >= 0; --n) {
                            double pv = Ly.red_sum(tid, n);
                            if (pv > 0.0) { ch = n; pch = pv; break; }
                        }
                }
                c.ch = ch;
                c.pch = pch;
            }
        }
        __syncthreads();
        // y <- C_ch psi* / sqrt(p_ch)  (ch < 0: renormalised psi*)
        double nrm[L::CPT][1];
#pragma unroll
        for (int b = 0; b < L::CPT; ++b) nrm[b][0] = 0.0;
#pragma unroll
        for (int e = 0; e < L::NE; ++e) {
            int q = Ly.comp(e), gc = Ly.gcol(Ly.slot(e));
            if (q < 0 || gc < 0 || cs[gc].action != ACT_JUMP) continue;
            const Col& c = cs[gc];
            if (c.ch >= 0) {
                double2 v = csr_row(S.c_rp + (size_t)c.ch * (S.d + 1), S.c_ci, S.c_val, q, gc);
                y[e] = cscale(1.0 / sqrt(c.pch), v);
            } else {
                y[e] = Ly.Stage[q * Ly.NB + gc];
                nrm[Ly.slot(e)][0] += cabs2(y[e]);
            }
        }
        Ly.template reduce<1>(nrm);
#pragma unroll
        for (int e = 0; e < L::NE; ++e) {
            int gc = Ly.gcol(Ly.slot(e));
            if (gc >= 0 && cs[gc].action == ACT_JUMP && cs[gc].ch < 0) y[e] = cscale(1.0 / sqrt(Ly.red_sum(gc, 0)), y[e]);
        }
        __syncthreads();
        if (tid < Ly.NB) {
            Col& c = cs[tid];
            if (c.action == ACT_JUMP) {
                if (c.njump < A.jcap) {
                    S.jt[(size_t)c.traj * A.jcap + c.njump] = c.tb;
                    S.jc[(size_t)c.traj * A.jcap + c.njump] = c.ch;
                }
                if (A.seg_cap > 0 && c.seg_rec < A.seg_cap) {
                    float* rec = S.segs + ((size_t)c.traj * A.seg_cap + c.seg_rec) * kSegRec;
                    rec[16] = (float)(c.tb - c.tseg); rec[18] = 0.f;
                }
                c.njump++;
                c.t = c.tb;
                c.action = ACT_POSTJUMP;   // marks "post-jump outputs pending"
            }
        }
        __syncthreads();
        outputs_loop(3);
        if (tid < Ly.NB) {
            Col& c = cs[tid];
            if (c.action == ACT_POSTJUMP) {
                c.action = ACT_NONE;
                c.seg++;
                c.seg_rec++;
                c.state = ST_NEEDK1;
            }
        }
        __syncthreads();
    }
};


}  // namespace qtm
