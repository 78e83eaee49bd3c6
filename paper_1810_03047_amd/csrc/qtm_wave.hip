// qtm_wave.hip -- trajectory kernel for small dense H_eff (d <= 64): a "team"
// of NWT wavefronts owns 16 trajectories (lane & 15); the team's waves split
// the row tiles of the real-embedded operator (T tiles each), so every lane
// holds 2*T complex state components of its trajectory and the whole DOPRI5
// state stays in registers.  A block holds one team, or up to four single-wave
// teams that share the operator in LDS.
//
// The product K = M W runs on the matrix cores (16x16x4 MFMA, FP64 or FP32).
// The operator's A-fragments (real embedding, in LDS) have their columns
// permuted so that K-block (source tile s, slot i) is exactly the value each
// lane keeps in accumulator slot i of its tile s: a single-wave team feeds W
// to the matrix cores from registers, and larger teams exchange their tiles
// through LDS in plain lane order.
//
// Per-trajectory scalars (t, h, threshold, ...) are replicated on the four lane
// groups and on the team's waves, which all take identical decisions from
// identical reductions: within a wave two xor-shuffles, across the team one LDS
// exchange summed in wave order.  Only the team's own waves meet at barriers,
// and every barrier sits in control flow that is uniform across the team.
#include "qtm_body.h"

namespace qtm {

// Sum over the four lanes of a column (lane & 15) with the gfx950 VALU lane swaps:
// permlane32_swap pairs lanes l and l ^ 32, permlane16_swap then lanes l and l ^ 16.
// Each addition is commutative, so every lane of a column ends with identical bits.
__device__ __forceinline__ double swap_add32(double v) {
    auto a = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
    auto b = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
    return __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
}
__device__ __forceinline__ double swap_add16(double v) {
    auto a = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
    auto b = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
    return __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
}
__device__ __forceinline__ double csum(double x) { return swap_add16(swap_add32(x)); }
__device__ __forceinline__ float csumf(float v) {
    auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    auto b = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}
__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ULL; }
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kXV = 8;       // values per column in one team reduction

// LEARN = false compiles out the segment-start features and the proposal network
// (kernels that never run the learned form or record segments).  TD = true adds the
// time-dependent terms of the Hamiltonian: every product is M W + sum_k M_k (f_k(t_s) W)
// with each lane's own stage time t_s.
template <int T, int NWT, int PREC, bool LEARN = true, int BAND = 0, bool TD = false>
struct Team {
    typedef typename MfmaT<PREC>::in_t in_t;
    typedef typename std::conditional<PREC == 0, double2, float2>::type kv_t;   // stage vectors
    static constexpr int NE = 2 * T;

    const DevSystem& S;
    const RunArgs& A;
    const in_t* Mf;          // LDS: A-fragments [RT][RT][64][4] (output tile, source tile, lane, slot)
    const in_t* Mt;          // TD: A-fragments of the time-dependent terms [n_td][RT][RT][64][4]
                             // (LDS, or global memory when they do not fit)
    in_t* Wb;                // LDS: operand tiles [RT][64][4] (teams of several waves)
    double2* St;             // alias of Wb: complex staging [dp][16]
    double* Xb;              // LDS: team reduction exchange [NWT][16][kXV]
    unsigned long long* Ib;  // LDS: trajectory hand-out [16]
    int* Fb;                 // LDS: team flags, one per wave
    const double2* Od;       // LDS copy of the diagonal observables [n_e][d] (when od_lds;
                             // od_lds == 2: every one real)
    const float* Ft;         // LDS: FP32 feature table [d][16] (rows 12, 13: C_n^dag C_n when diagonal)
    const int* Cjc = nullptr;      // LDS jump table (one entry per row of each C_n): column, -1 for none
    const double2* Cjv = nullptr;  // and value, [n_c][d]; nullptr: the CSR arrays in global memory
    int od_lds;
    int lane, lg, c16, wv, RT, d, dp, q0;

    // per-lane trajectory state (identical on every lane of a column, on every wave)
    double t, h, h0, d1, r, u, tseg, tb, fac, th, oth, tnext, tnext2;   // output times k, k + 1
    double tstage;           // TD: time at which the next product evaluates the right-hand side
    long long traj;
    int state, action, seg, kk, nacc, nrej, njump, natt, last, rejected, omode, ch, seg_rec, first_acc;
    bool exhausted;
    unsigned long long passes;

    double2 y[NE], yn[NE];
    kv_t k[7][NE];
    kv_t es[NE], ds[NE];     // sum_j e_j k_j and sum_j d_j k_j over stages 1..6 (product precision)

    QTM_DI Team(const DevSystem& s, const RunArgs& a) : S(s), A(a) {}

    // acc + c k in the product precision
    QTM_DI static double2 kfma(double c, const double2& k, const double2& acc) { return cfma(c, k, acc); }
    QTM_DI static float2 kfma(double c, const float2& k, const float2& acc) {
        return make_float2(fmaf((float)c, k.x, acc.x), fmaf((float)c, k.y, acc.y));
    }

    QTM_DI void team_sync() const {
        if (NWT > 1) __syncthreads();
        else wave_sync();
    }
    // Component held in element e of a lane: q0 + cst(e), q0 = 8 T wv + lg (FP64,
    // output rows lg + 4 i) or 8 T wv + 2 lg (FP32, rows 4 lg + i); elements
    // 2 tt and 2 tt + 1 are accumulator slots (0, 1) and (2, 3) of tile tt.
    // Components at or past d (padding, or tiles past RT) are invalid.
    static constexpr int cst(int e) { return PREC == 0 ? 8 * (e >> 1) + 4 * (e & 1) : 8 * (e >> 1) + (e & 1); }
    // q0 passed through an empty asm statement: addresses built from it are recomputed
    // where they are used (two VALU ops) instead of being hoisted out of the main loop,
    // where they would live for the whole kernel and end up in scratch
    QTM_DI int qbase() const { int x = q0; asm volatile("" : "+v"(x)); return x; }
    QTM_DI int comp(int e) const { int q = qbase() + cst(e); return q < d ? q : -1; }

    // team-wide per-column sums of NV values (NV <= kXV), identical on every lane
    template <int NV> QTM_DI void tsum(double (&p)[NV]) {
#pragma unroll
        for (int v = 0; v < NV; ++v) p[v] = csum(p[v]);
        if (NWT == 1) return;
        if (lg == 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v) Xb[(wv * 16 + c16) * kXV + v] = p[v];
        }
        __syncthreads();
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double s = 0.0;
#pragma unroll
            for (int g = 0; g < NWT; ++g) s += Xb[(g * 16 + c16) * kXV + v];
            p[v] = s;
        }
        __syncthreads();
    }
    template <int NV> QTM_DI void tsumf(float (&p)[NV]) {
#pragma unroll
        for (int v = 0; v < NV; ++v) p[v] = csumf(p[v]);
        if (NWT == 1) return;
        if (lg == 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v) Xb[(wv * 16 + c16) * kXV + v] = p[v];
        }
        __syncthreads();
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double sv = 0.0;
#pragma unroll
            for (int g = 0; g < NWT; ++g) sv += Xb[(g * 16 + c16) * kXV + v];
            p[v] = (float)sv;
        }
        __syncthreads();
    }
    QTM_DI double tsum1(double x) { double p[1] = {x}; tsum<1>(p); return p[0]; }
    QTM_DI bool team_any(bool pred) {
        bool w = wave_any(pred);
        if (NWT == 1) return w;
        if (lane == 0) Fb[wv] = w ? 1 : 0;
        __syncthreads();
        bool any = false;
#pragma unroll
        for (int g = 0; g < NWT; ++g) any |= Fb[g] != 0;
        __syncthreads();
        return any;
    }

    // ------------------------------------------------------------ product
    struct alignas(16) In4 { in_t v[4]; };
    template <class V> QTM_DI static In4 slots(const V& a, const V& b) {
        In4 r;
        r.v[0] = (in_t)a.x; r.v[1] = (in_t)a.y; r.v[2] = (in_t)b.x; r.v[3] = (in_t)b.y;
        return r;
    }
    // K = M W for the team's 16 columns; W in the lane layout of the state.
    // Every lane of the team must take part (uniform call).
    static constexpr bool in_band(int tt, int s) { return BAND == 0 || (tt - s <= 1 && s - tt <= 1); }
    template <class V> QTM_DI void product(const V (&W)[NE], kv_t (&K)[NE]) {
        typename MfmaT<PREC>::acc_t acc[T];
#pragma unroll
        for (int tt = 0; tt < T; ++tt) acc[tt] = 0;
        if constexpr (NWT == 1) {
            // the lane's own tiles are all source tiles (T == RT).  BAND: the operator's
            // nonzero tiles lie within one tile of the diagonal, and only those are
            // multiplied (the others would add exact zeros); the tile pattern is fixed at
            // compile time, so no branch separates the matrix-core instructions
#pragma unroll
            for (int s = 0; s < T; ++s) {
                const In4 b = slots(W[2 * s], W[2 * s + 1]);
                In4 av[T];
#pragma unroll
                for (int tt = 0; tt < T; ++tt)
                    if (in_band(tt, s)) av[tt] = *(const In4*)(Mf + ((size_t)(tt * T + s) * 64 + lane) * 4);
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int tt = 0; tt < T; ++tt)
                        if (in_band(tt, s)) acc[tt] = MfmaT<PREC>::op(av[tt].v[i], b.v[i], acc[tt]);
                __builtin_amdgcn_sched_barrier(0);     // one source tile of fragments in flight at a time
            }
            if constexpr (TD) {
                // + M_k (f_k(t_s) W): the scale is the lane's own (its trajectory's) coefficient
                for (int q = 0; q < S.n_td; ++q) {
                    const in_t f = (in_t)td_coef(q);
                    const in_t* Mq = Mt + (size_t)q * RT * RT * 256;
#pragma unroll
                    for (int s = 0; s < T; ++s) {
                        In4 b = slots(W[2 * s], W[2 * s + 1]);
#pragma unroll
                        for (int i = 0; i < 4; ++i) b.v[i] *= f;
                        In4 av[T];
#pragma unroll
                        for (int tt = 0; tt < T; ++tt) av[tt] = *(const In4*)(Mq + ((size_t)(tt * T + s) * 64 + lane) * 4);
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (int tt = 0; tt < T; ++tt) acc[tt] = MfmaT<PREC>::op(av[tt].v[i], b.v[i], acc[tt]);
                    }
                }
            }
        } else {
            team_sync();                // earlier readers of the operand tiles are done
#pragma unroll
            for (int tt = 0; tt < T; ++tt) {
                const int rt = wv * T + tt;
                if (rt < RT) *(In4*)(Wb + ((size_t)rt * 64 + lane) * 4) = slots(W[2 * tt], W[2 * tt + 1]);
            }
            team_sync();
            // padded tiles (rt >= RT) multiply a valid tile; their results are never used
            const in_t* ap[T];
#pragma unroll
            for (int tt = 0; tt < T; ++tt) {
                const int rt = wv * T + tt < RT ? wv * T + tt : RT - 1;
                ap[tt] = Mf + ((size_t)rt * RT * 64 + lane) * 4;
            }
            for (int s = 0; s < RT; ++s) {
                const In4 b = *(const In4*)(Wb + ((size_t)s * 64 + lane) * 4);
                In4 av[T];
#pragma unroll
                for (int tt = 0; tt < T; ++tt) av[tt] = *(const In4*)(ap[tt] + (size_t)s * 256);
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int tt = 0; tt < T; ++tt) acc[tt] = MfmaT<PREC>::op(av[tt].v[i], b.v[i], acc[tt]);
            }
            if constexpr (TD) {
                // + M_k (f_k(t_s) W); the staged tile a lane reads holds its own trajectory
                for (int q = 0; q < S.n_td; ++q) {
                    const in_t f = (in_t)td_coef(q);
                    const size_t qo = (size_t)q * RT * RT * 256;
                    for (int s = 0; s < RT; ++s) {
                        In4 b = *(const In4*)(Wb + ((size_t)s * 64 + lane) * 4);
#pragma unroll
                        for (int i = 0; i < 4; ++i) b.v[i] *= f;
                        In4 av[T];
#pragma unroll
                        for (int tt = 0; tt < T; ++tt) av[tt] = *(const In4*)(Mt + qo + (ap[tt] - Mf) + (size_t)s * 256);
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (int tt = 0; tt < T; ++tt) acc[tt] = MfmaT<PREC>::op(av[tt].v[i], b.v[i], acc[tt]);
                    }
                }
            }
        }
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            K[2 * tt + 0] = from_d2<kv_t>(make_double2((double)acc[tt][0], (double)acc[tt][1]));
            K[2 * tt + 1] = from_d2<kv_t>(make_double2((double)acc[tt][2], (double)acc[tt][3]));
        }
        ++passes;       // summed into the run counters once, when the team exits
    }

    // f_q(tstage) = c + a cos(w t) + b sin(w t) of time-dependent term q (FP64, this lane's time)
    QTM_DI double td_coef(int q) const {
        const double* c = S.td + 4 * q;
        double sn, cs;
        sincos(c[3] * tstage, &sn, &cs);
        return c[0] + c[1] * cs + c[2] * sn;
    }

    // ------------------------------------------------------------ dense output
    // u(th) = y + th (D + (1-th)(B + th (R4 + (1-th) R5))),
    // D = yn - y, B = h k1 - D, R4 = D - h k7 - B, R5 = h sum_j d_j k_j
    QTM_DI double2 dense_at(int e, double tht) const {
        double2 D = csub(yn[e], y[e]);
        if constexpr (PREC == 1) {
            // FP32 products: B, R4, R5 and the two inner levels in FP32 (the stage
            // vectors are FP32); the outer two levels, with y and D, in FP64
            const float2 k1 = (const float2&)k[0][e], k7 = (const float2&)k[6][e], sd = (const float2&)ds[e];
            const float hf = (float)h, th = (float)tht, t1 = 1.f - th, d7 = (float)dp_d(6);
            const float Dx = (float)D.x, Dy = (float)D.y;
            const float Bx = fmaf(hf, k1.x, -Dx), By = fmaf(hf, k1.y, -Dy);
            const float R4x = Dx - fmaf(hf, k7.x, Bx), R4y = Dy - fmaf(hf, k7.y, By);
            const float R5x = hf * fmaf(d7, k7.x, sd.x), R5y = hf * fmaf(d7, k7.y, sd.y);
            const float ix = fmaf(th, fmaf(t1, R5x, R4x), Bx), iy = fmaf(th, fmaf(t1, R5y, R4y), By);
            const double t1d = 1.0 - tht;
            return make_double2(fma(tht, fma(t1d, (double)ix, D.x), y[e].x), fma(tht, fma(t1d, (double)iy, D.y), y[e].y));
        }
        double2 B = csub(cscale(h, to_d2(k[0][e])), D);
        double2 R4 = csub(csub(D, cscale(h, to_d2(k[6][e]))), B);
        double2 R5 = cscale(h, cfma(dp_d(6), to_d2(k[6][e]), to_d2(ds[e])));
        double t1 = 1.0 - tht;
        double2 in = cadd(R4, cscale(t1, R5));
        in = cadd(B, cscale(tht, in));
        in = cadd(D, cscale(t1, in));
        return cadd(y[e], cscale(tht, in));
    }
    QTM_DI double2 vec_mode(int e) const { return omode == 1 ? y[e] : omode == 2 ? yn[e] : dense_at(e, oth); }

    QTM_DI double2 csr_row(const int* rp, const int* ci, const double2* val, int q) const {
        double2 s = make_double2(0.0, 0.0);
        for (int p = rp[q]; p < rp[q + 1]; ++p) s = cadd(s, cmul(val[p], St[ci[p] * 16 + c16]));
        return s;
    }
    QTM_DI void stage_vec(const double2 (&v)[NE]) {
        team_sync();   // earlier readers of the staging tile are done
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            int q = comp(e);
            if (q >= 0) St[q * 16 + c16] = v[e];
        }
        team_sync();
    }

    // ------------------------------------------------------------ outputs
    // <u|O_o|u>/<u|u> for every lane with omode != 0 (one team reduction per observable)
    // real diagonal observables (od_lds == 2): G observables and the norm per team
    // reduction, real parts only (the imaginary parts are zero)
    template <int G> QTM_DI void output_round_real(bool on, int o0) {
        const int qb = qbase();
        const int no = S.n_e - o0 < G ? S.n_e - o0 : G;
        const double2* dv0 = Od + (size_t)o0 * d;
        double p[G + 1];
#pragma unroll
        for (int v = 0; v <= G; ++v) p[v] = 0.0;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const int q = qb + cst(e);
            const double2 u = (on && q < d) ? vec_mode(e) : make_double2(0.0, 0.0);
            const double a2 = cabs2(u);
            const int qi = q < d ? q : 0;
            p[G] += a2;
#pragma unroll
            for (int j = 0; j < G; ++j)
                if (j < no) p[j] = fma(dv0[(size_t)j * d + qi].x, a2, p[j]);
        }
        tsum<G + 1>(p);
        if (on && lg == 0 && wv == 0) {
#pragma unroll
            for (int j = 0; j < G; ++j)
                if (j < no) S.X[((size_t)traj * S.n_e + o0 + j) * S.n_t + kk] = make_double2(p[j] / p[G], 0.0);
        }
    }

    QTM_DI void output_round(bool on) {
        if (S.any_csr_e || !od_lds) { output_round_staged(on); return; }   // observables not all in LDS
        if (od_lds == 2) {
            for (int o0 = 0; o0 < S.n_e; o0 += 3) output_round_real<3>(on, o0);
            return;
        }
        // diagonal observables only: each component of u is evaluated once and goes
        // straight into the norm and the observable sums (no vector kept)
        const int qb = qbase();
        for (int o0 = 0; o0 < S.n_e; o0 += 3) {
            const int no = S.n_e - o0 < 3 ? S.n_e - o0 : 3;
            const double2* dv0 = Od + (size_t)o0 * d;
            double p[7];
#pragma unroll
            for (int v = 0; v < 7; ++v) p[v] = 0.0;
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const int q = qb + cst(e);
                const double2 u = (on && q < d) ? vec_mode(e) : make_double2(0.0, 0.0);
                const double a2 = cabs2(u);
                const int qi = q < d ? q : 0;
                p[6] += a2;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    if (j < no) {
                        const double2 v = dv0[(size_t)j * d + qi];
                        p[2 * j] = fma(v.x, a2, p[2 * j]);
                        p[2 * j + 1] = fma(v.y, a2, p[2 * j + 1]);
                    }
                }
            }
            tsum<7>(p);
            if (on && lg == 0 && wv == 0) {
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    if (j < no) S.X[((size_t)traj * S.n_e + o0 + j) * S.n_t + kk] = make_double2(p[2 * j] / p[6], p[2 * j + 1] / p[6]);
            }
        }
    }

    // general observables (some CSR): u is written to the LDS staging tile as it is
    // evaluated (no vector kept in registers) and read back for every observable
    QTM_DI void output_round_staged(bool on) {
        double nn = 0.0;
        const int qb = qbase();
        team_sync();                        // earlier readers of the staging tile are done
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const int q = qb + cst(e);
            if (q < d) {
                const double2 u = on ? vec_mode(e) : make_double2(0.0, 0.0);
                St[q * 16 + c16] = u;
                nn += cabs2(u);
            }
        }
        team_sync();
        // up to three observables and the norm per team reduction
        for (int o0 = 0; o0 < S.n_e; o0 += 3) {
            double p[7];
#pragma unroll
            for (int v = 0; v < 6; ++v) p[v] = 0.0;
            p[6] = o0 == 0 ? nn : 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int o = o0 + j;
                if (o >= S.n_e) break;
                const bool diag = S.e_fmt[o] == 2;
                const double2* dv = S.e_val + S.e_doff[o];
                const int* rp = S.e_rp + (size_t)o * (S.d + 1);
#pragma unroll
                for (int e = 0; e < NE; ++e) {
                    const int q = qb + cst(e);
                    if (q >= d || !on) continue;
                    const double2 u = St[q * 16 + c16];
                    if (diag) {
                        const double a2 = cabs2(u);
                        const double2 v = dv[q];
                        p[2 * j] = fma(v.x, a2, p[2 * j]);
                        p[2 * j + 1] = fma(v.y, a2, p[2 * j + 1]);
                    } else {
                        const double2 Ou = csr_row(rp, S.e_ci, S.e_val, q);
                        p[2 * j] += u.x * Ou.x + u.y * Ou.y;     // Re conj(u) O u
                        p[2 * j + 1] += u.x * Ou.y - u.y * Ou.x; // Im conj(u) O u
                    }
                }
            }
            tsum<7>(p);
            if (o0 == 0) nn = p[6];
            if (on && lg == 0 && wv == 0) {
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const int o = o0 + j;
                    if (o < S.n_e) S.X[((size_t)traj * S.n_e + o) * S.n_t + kk] = make_double2(p[2 * j] / nn, p[2 * j + 1] / nn);
                }
            }
        }
    }

    // phase 0: new trajectory or segment start after a jump (t_k == t, current y);
    // 1: accepted step (t < t_k <= tb) or jump step (t < t_k < tb)
    QTM_DI void next_output(int phase) {
        omode = 0;
        if (kk >= S.n_t) return;
        const double tk = tnext;
        if (phase == 0 && (state == ST_NEW || state == ST_NEEDK1)) {
            if (tk == t) omode = 1;
        } else if (phase == 1 && action == ACT_ACCEPT) {
            if (tk <= tb) {
                if (tk == tb) omode = 2;
                else { omode = 3; oth = (tk - t) / h; }
            }
        } else if (phase == 1 && action == ACT_JUMP) {
            if (tk < tb) { omode = 3; oth = (tk - t) / h; }
        }
    }
    QTM_DI void outputs_loop(int phase) {
        for (;;) {
            next_output(phase);
            bool on = omode != 0;
            if (!team_any(on)) break;
            output_round(on);
            if (on) {
                kk++;
                // the time after next is requested now and first needed a round later
                tnext = tnext2;
                tnext2 = kk + 1 < S.n_t ? S.tlist[kk + 1] : 0.0;
            }
        }
        omode = 0;
    }

    QTM_DI void retire(bool failed) {
        if (lg == 0 && wv == 0) {
            int* st = S.tstat + (size_t)traj * 4;
            st[0] = nacc; st[1] = nrej; st[2] = seg + 1; st[3] = njump;
            S.jn[traj] = njump;
            if (failed) atomicMin((unsigned long long*)A.fail, (unsigned long long)(S.traj_begin + traj));
        }
        state = ST_EMPTY;
        traj = -1;
    }

    // ------------------------------------------------------------ main loop
    QTM_DI void run() {
        const double tend = S.tend;
        state = ST_EMPTY; traj = -1; action = ACT_NONE; omode = 0; exhausted = false;
        t = h = h0 = d1 = r = u = tseg = tb = fac = th = oth = tnext = tnext2 = 0.0;
        seg = kk = nacc = nrej = njump = natt = last = rejected = ch = seg_rec = first_acc = 0;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            y[e] = yn[e] = make_double2(0.0, 0.0);
            es[e] = ds[e] = from_d2<kv_t>(make_double2(0.0, 0.0));
#pragma unroll
            for (int j = 0; j < 7; ++j) k[j][e] = from_d2<kv_t>(make_double2(0.0, 0.0));
        }
        long long cycles = 0;
        bool first = true;
        passes = 0;
        for (;;) {
            // ---- refill empty slots (wave 0 takes the indices, the team reads them)
            action = ACT_NONE;
            bool want = state == ST_EMPTY && !exhausted && (A.persistent || first);
            first = false;
            if (wv == 0 && lg == 0) Ib[c16] = want ? atomicAdd(S.queue, 1ULL) : 0ULL;
            team_sync();
            unsigned long long idx = Ib[c16];
            team_sync();
            if (want) {
                if ((long long)idx < S.count) {
                    traj = (long long)idx;
                    t = S.t0; seg = 0; kk = 0; nacc = nrej = njump = natt = 0;
                    rejected = 0; seg_rec = 0;
                    tnext = S.tlist[0];
                    tnext2 = S.n_t > 1 ? S.tlist[1] : 0.0;
                    state = ST_NEW;
                } else {
                    exhausted = true;
                }
            }
            if (!team_any(state != ST_EMPTY)) break;
            if (++cycles > A.max_cycles) {      // failsafe: retire everything as failed
                if (state != ST_EMPTY) retire(true);
                break;
            }
            // outputs at t_k == t: a new trajectory's first ones, and those at the jump
            // time of a trajectory that jumped in the previous pass (now at its segment start)
            if (team_any(state == ST_NEW || state == ST_NEEDK1)) {
#pragma unroll
                for (int e = 0; e < NE; ++e) {
                    int q = comp(e);
                    if (state == ST_NEW) y[e] = q >= 0 ? S.psi0[q] : make_double2(0.0, 0.0);
                }
                outputs_loop(0);
                if (state == ST_NEW) state = ST_NEEDK1;
            }
            // ---- segment start: threshold r and channel uniform (Philox)
            if (state == ST_NEEDK1) {
                if (!(t < tend)) retire(false);
                else if (natt >= A.max_steps) retire(true);
                else {
                    uint64_t ctr[4] = {(uint64_t)(S.traj_begin + traj), (uint64_t)seg, 0, 0};
                    philox4x64(ctr, S.key0, S.key1);
                    r = u53(ctr[0]);
                    u = u53(ctr[1]);
                    first_acc = 1;
                    tseg = t;
                    rejected = 0;
                }
            }
            if (team_any(state == ST_NEEDK1)) segment_start();
            // the last step of the span ends exactly at t_end
            if (state == ST_STEP) {
                last = (t + h >= tend);
                if (last) h = tend - t;
            }
            stages();
            post_step();
        }
    }

    // k1 = M y, then the starting step (or the learned proposal)
    QTM_DI void segment_start() {
        kv_t K[NE];
        if constexpr (TD) tstage = t;
        product(y, K);
#pragma unroll
        for (int e = 0; e < NE; ++e)
            if (state == ST_NEEDK1) k[0][e] = K[e];
        if (LEARN && (A.learned || A.seg_cap > 0)) features();
        if (!LEARN || !A.learned) {
            // Hairer-Norsett-Wanner starting step, first part: d0 = ||y/sc||, d1 = ||f0/sc||
            double p[2] = {0.0, 0.0};
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                int q = comp(e);
                if (q < 0) continue;
                double sc = A.atol + A.rtol * sqrt(cabs2(y[e]));
                double isc2 = 1.0 / (sc * sc);
                p[0] += cabs2(y[e]) * isc2;
                p[1] += cabs2(to_d2(k[0][e])) * isc2;
            }
            tsum<2>(p);
            if (state == ST_NEEDK1) {
                double dd0 = sqrt(p[0] / S.d), dd1 = sqrt(p[1] / S.d);
                double hh = (dd0 < 1e-5 || dd1 < 1e-5) ? 1e-6 : 0.01 * dd0 / dd1;
                h0 = fmin(hh, S.tend - t);
                d1 = dd1;
                state = ST_NEEDF1;
            }
        }
    }

    // 16 segment-start features; the learned form turns them into the first step
    QTM_DI void features() {
        const bool on = state == ST_NEEDK1;
        const bool cd = S.c_isdiag != 0;
        if (!cd && S.n_c > 0) {
            double2 v[NE];
#pragma unroll
            for (int e = 0; e < NE; ++e) v[e] = on ? y[e] : make_double2(0.0, 0.0);
            stage_vec(v);
        }
        // populations |y_q|^2 (zero off the trajectory's valid components) against the
        // FP32 table [q][16] (rows: 12 feature populations, <C_n^dag C_n> for n < 2 when
        // diagonal), four 16-byte LDS reads per component, FP32 sums; norm in FP64
        float f[kNF];
        double nn = 0.0;
        float acc[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.f;
        const int qb = qbase();
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const int q = qb + cst(e);
            const bool ok = on && q < d;
            const double a2 = ok ? cabs2(y[e]) : 0.0;
            nn += a2;
            const float af = (float)a2;
            const float4* row = (const float4*)(Ft + (q < d ? q : 0) * 16);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const float4 v = row[g];
                acc[4 * g + 0] = fmaf(v.x, af, acc[4 * g + 0]);
                acc[4 * g + 1] = fmaf(v.y, af, acc[4 * g + 1]);
                acc[4 * g + 2] = fmaf(v.z, af, acc[4 * g + 2]);
                acc[4 * g + 3] = fmaf(v.w, af, acc[4 * g + 3]);
            }
        }
        nn = tsum1(nn);
        {
            float h0f[8], h1f[8];
#pragma unroll
            for (int r = 0; r < 7; ++r) { h0f[r] = acc[r]; h1f[r] = acc[7 + r]; }
            h0f[7] = h1f[7] = 0.f;
            tsumf<8>(h0f);
            tsumf<8>(h1f);
            const float inv = (float)(1.0 / nn);
#pragma unroll
            for (int r = 0; r < 7; ++r) { f[r] = h0f[r] * inv; f[7 + r] = h1f[r] * inv; }
        }
        double pv0 = nn;
        if (!cd) {
            // general collapse operators: ||C_n y||^2 from the staged state
            for (int n = 0; n < 2; ++n) {
                double acc = 0.0;
                if (n < S.n_c) {
                    const int* rp = S.c_rp + (size_t)n * (S.d + 1);
#pragma unroll
                    for (int e = 0; e < NE; ++e) {
                        int q = comp(e);
                        if (on && q >= 0) acc += cabs2(csr_row(rp, S.c_ci, S.c_val, q));
                    }
                    acc = tsum1(acc);
                }
                f[12 + n] = (float)(acc / pv0);
            }
        }
        if (!on) {
#pragma unroll
            for (int v = 0; v < 14; ++v) f[v] = 0.f;
        }
        f[14] = on ? logf((float)r) : 0.f;
        f[15] = on ? (float)((t - S.t0) / (S.tend - S.t0)) : 0.f;
        if (A.learned) {
            const float lh = team_mlp(f);
            if (on) {
                double hh = snap_proposal(lh);
                h = fmin(hh, S.tend - t);
                state = ST_STEP;
            }
        }
        if (on && A.seg_cap > 0 && seg_rec < A.seg_cap && lg == 0 && wv == 0) {
            float* rec = S.segs + ((size_t)traj * A.seg_cap + seg_rec) * kSegRec;
#pragma unroll
            for (int v = 0; v < kNF; ++v) rec[v] = f[v];
            rec[16] = 0.f; rec[17] = -1.f; rec[18] = 1.f; rec[19] = 1.f;
        }
    }

    // Proposal network 16 -> 64 -> 64 -> 3 (GELU) for the team's 16 trajectories
    // at once on the matrix cores: FP32 16x16x4 MFMA on BF16-valued weights, FP32
    // activations.  Trajectory = MFMA column.  A layer's hidden units come back in
    // the accumulator layout (unit 16 s + 4 lg + i in slot i of tile s) and feed
    // the next layer in place: the weight fragments' columns are permuted to
    // match.  Layer 1 takes standardised features 4 lg .. 4 lg + 3 from each lane
    // group.  Returns output 0 (log of the proposed first step) on every lane.
    // Uniform call: every lane of the wave takes part.
    QTM_DI float team_mlp(const float (&f)[kNF]) {
        const float* b1 = A.mlp + kNH * kNF;
        const float* b2 = b1 + kNH + kNH * kNH;
        const float* b3 = b2 + kNH + kNO * kNH;
        const float* mu = b3 + kNO;
        const float* sd = mu + kNF;
        const uint2* F = (const uint2*)A.mlpf;          // 4 BF16 values per lane and group
        auto bf = [](unsigned int w, int hi) { return __uint_as_float(hi ? (w & 0xFFFF0000u) : (w << 16)); };
        // every operand of the three layers is requested at once (one memory latency per
        // call); the biases b1, b2 sit at multiples of 4 floats from the 256-byte aligned start
        uint2 w1[4], w2[16], w3[4];
        float4 c1[4], c2[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) w1[g] = F[(size_t)g * 64 + lane];
#pragma unroll
        for (int g = 0; g < 16; ++g) w2[g] = F[(size_t)(4 + g) * 64 + lane];
#pragma unroll
        for (int g = 0; g < 4; ++g) w3[g] = F[(size_t)(20 + g) * 64 + lane];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            c1[rt] = *(const float4*)(b1 + 16 * rt + 4 * lg);
            c2[rt] = *(const float4*)(b2 + 16 * rt + 4 * lg);
        }
        // mean and scale start at an odd offset: plain scalar loads
        float m4[4], s4[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) { m4[j] = mu[4 * lg + j]; s4[j] = sd[4 * lg + j]; }
        const float ob = b3[0];
        float x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float v = lg == 0 ? f[j] : lg == 1 ? f[4 + j] : lg == 2 ? f[8 + j] : f[12 + j];
            x[j] = (v - m4[j]) / s4[j];
        }
        float h1[4][4], h2[4][4];
        f4 z1[4], z2[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) z1[rt] = 0;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
                z1[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(bf(kb < 2 ? w1[rt].x : w1[rt].y, kb & 1), x[kb], z1[rt], 0, 0, 0);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            h1[rt][0] = gelu_f(z1[rt][0] + c1[rt].x); h1[rt][1] = gelu_f(z1[rt][1] + c1[rt].y);
            h1[rt][2] = gelu_f(z1[rt][2] + c1[rt].z); h1[rt][3] = gelu_f(z1[rt][3] + c1[rt].w);
            z2[rt] = 0;
        }
        // four independent accumulation chains (output tiles) interleaved
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) {
                    const uint2 wq = w2[4 * rt + s2];
                    z2[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(bf(i < 2 ? wq.x : wq.y, i & 1), h1[s2][i], z2[rt], 0, 0, 0);
                }
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            h2[rt][0] = gelu_f(z2[rt][0] + c2[rt].x); h2[rt][1] = gelu_f(z2[rt][1] + c2[rt].y);
            h2[rt][2] = gelu_f(z2[rt][2] + c2[rt].z); h2[rt][3] = gelu_f(z2[rt][3] + c2[rt].w);
        }
        f4 o = 0;
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
            const uint2 wq = w3[s2];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                o = __builtin_amdgcn_mfma_f32_16x16x4f32(bf(i < 2 ? wq.x : wq.y, i & 1), h2[s2][i], o, 0, 0, 0);
        }
        // output 0 is row 0: slot 0 of lane group 0
        return __shfl(o[0] + ob, c16);
    }

    // stage s (0-based): w = y + sum_j c_j k_j, k_s = M w
    template <int s> QTM_DI void one_stage() {
        double cf[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) cf[j] = (state == ST_STEP) ? h * dp_a(s, j) : 0.0;
        if (s == 1 && state == ST_NEEDF1) cf[0] = h0;
        kv_t w[NE];              // the stage input, rounded to the product precision
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            double2 acc;
            if constexpr (PREC == 0) {
                acc = y[e];
#pragma unroll
                for (int j = 0; j < s; ++j)
                    if (dp_a(s, j) != 0.0 || (s == 1 && j == 0)) acc = cfma(cf[j], to_d2(k[j][e]), acc);
            } else {
                // FP32 form: the increment sum_j c_j k_j of FP32 products is formed in FP32
                // and added to the FP64 state
                float2 inc = make_float2(0.f, 0.f);
#pragma unroll
                for (int j = 0; j < s; ++j)
                    if (dp_a(s, j) != 0.0 || (s == 1 && j == 0)) {
                        float2 kj = (float2&)k[j][e];
                        inc.x = fmaf((float)cf[j], kj.x, inc.x);
                        inc.y = fmaf((float)cf[j], kj.y, inc.y);
                    }
                if constexpr (s != 6) {
                    // a stage input only feeds the FP32 products: y rounded to FP32 plus the
                    // FP32 increment (y_new, the last stage input, is formed in FP64 below)
                    w[e] = from_d2<kv_t>(make_double2(0.0, 0.0));
                    float2& wf = (float2&)w[e];
                    wf.x = (float)y[e].x + inc.x;
                    wf.y = (float)y[e].y + inc.y;
                    continue;
                }
                acc = make_double2(y[e].x + (double)inc.x, y[e].y + (double)inc.y);
            }
            if constexpr (s == 6) {
                // y_new is the last stage input; fold k1..k6 into the error and
                // dense-output sums now so that k2..k6 need not live longer
                yn[e] = acc;
                kv_t se = from_d2<kv_t>(make_double2(0.0, 0.0)), sd = se;
#pragma unroll
                for (int j = 0; j < 6; ++j) {
                    if (dp_e(j) != 0.0) se = kfma(dp_e(j), k[j][e], se);
                    if (dp_d(j) != 0.0) sd = kfma(dp_d(j), k[j][e], sd);
                }
                es[e] = se;
                ds[e] = sd;
            } else {
                w[e] = from_d2<kv_t>(acc);
            }
        }
        if constexpr (TD) {
            // stage s of a step at t + c_s h; the starting step's probe (stage 1 of a
            // segment start) at t + h0
            tstage = state == ST_STEP ? t + dp_c(s) * h : (s == 1 && state == ST_NEEDF1) ? t + h0 : t;
        }
        if constexpr (s == 6) product(yn, k[s]);
        else product(w, k[s]);
    }

    QTM_DI void stages() {
        one_stage<1>();
        if (team_any(state == ST_NEEDF1)) {
            // starting step, second part: d2 = ||(f1 - f0)/sc|| / h0
            double p0 = 0.0;
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                int q = comp(e);
                if (q < 0) continue;
                double sc = A.atol + A.rtol * sqrt(cabs2(y[e]));
                p0 += cabs2(csub(to_d2(k[1][e]), to_d2(k[0][e]))) / (sc * sc);
            }
            p0 = tsum1(p0);
            if (state == ST_NEEDF1) {
                double d2 = sqrt(p0 / S.d) / h0;
                double h1 = (d1 <= 1e-15 && d2 <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : 1.0 / inv_fifth_root(0.01 / fmax(d1, d2));
                h = fmin(fmin(100.0 * h0, h1), S.tend - t);
                state = ST_PROBED;
            }
        }
        one_stage<2>();
        one_stage<3>();
        one_stage<4>();
        one_stage<5>();
        one_stage<6>();
    }

    QTM_DI void post_step() {
        const double tend = S.tend;
        double p[2] = {0.0, 0.0};
        if (state == ST_STEP) {
            // FP32 products: the error terms in FP32 too (hardware square root and
            // reciprocal); the error ratio only steers the step size
            const float hf = (float)h, atf = (float)A.atol, rtf = (float)A.rtol;
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                int q = comp(e);
                if (q < 0) continue;
                if constexpr (PREC == 1) {
                    const float2 k6 = (const float2&)k[6][e], s6 = (const float2&)es[e];
                    const float erx = hf * fmaf((float)dp_e(6), k6.x, s6.x);
                    const float ery = hf * fmaf((float)dp_e(6), k6.y, s6.y);
                    const float scf = fmaf(rtf, __builtin_amdgcn_sqrtf((float)fmax(cabs2(y[e]), cabs2(yn[e]))), atf);
                    p[0] += (double)((erx * erx + ery * ery) * __builtin_amdgcn_rcpf(fmaxf(scf * scf, 1.17549435e-38f)));
                } else {
                    double2 er = cscale(h, cfma(dp_e(6), to_d2(k[6][e]), to_d2(es[e])));
                    double sc = A.atol + A.rtol * sqrt(fmax(cabs2(y[e]), cabs2(yn[e])));   // = max(|y|, |y_new|): one root
                    p[0] += cabs2(er) / (sc * sc);
                }
                p[1] += cabs2(yn[e]);
            }
        }
        tsum<2>(p);
        action = ACT_NONE;
        if (state == ST_PROBED) state = ST_STEP;
        else if (state == ST_STEP) {
            natt++;
            double err = sqrt(p[0] / S.d);
            if (!(err <= 1.0)) {
                double f = isfinite(err) ? fmax(0.2, 0.9 * inv_fifth_root(err)) : 0.2;
                h *= f;
                rejected = 1;
                nrej++;
                action = ACT_REJECT;
                if (!(h > 16.0 * DBL_EPSILON * fabs(t)) || natt >= A.max_steps) action = ACT_FAIL;
            } else {
                nacc++;
                double fc = (err == 0.0) ? 10.0 : fmin(10.0, 0.9 * inv_fifth_root(err));
                if (rejected) fc = fmin(1.0, fc);
                fac = fc;
                if (A.seg_cap > 0 && first_acc && seg_rec < A.seg_cap && lg == 0 && wv == 0)
                    S.segs[((size_t)traj * A.seg_cap + seg_rec) * kSegRec + 17] = (float)(h * fc);
                first_acc = 0;
                tb = last ? tend : t + h;
                if (S.n_c > 0 && p[1] < r) action = ACT_JUMP;
                else {
                    action = ACT_ACCEPT;
                    if (!last && natt >= A.max_steps) action = ACT_FAIL;
                }
            }
        }
        const bool anyj = team_any(action == ACT_JUMP);
        if (NWT == 1 && od_lds == 2 && S.n_e <= 2) {
            // real diagonal observables: one pass of norm polynomials per step serves the
            // jump time and every output time of every lane (each lane's own polynomials: a
            // trajectory's results do not depend on its wave neighbours)
            const bool need = action == ACT_JUMP || (action == ACT_ACCEPT && kk < S.n_t && tnext <= tb);
            if (team_any(need)) {
                if (S.n_e == 1) gram_outputs<1>(need);
                else gram_outputs<2>(need);
            }
        } else {
            if (anyj) jump_time();
            if (team_any(action == ACT_ACCEPT || action == ACT_JUMP)) outputs_loop(1);
        }
        if (anyj) do_jump();
        if (action == ACT_ACCEPT) {
#pragma unroll
            for (int e = 0; e < NE; ++e) { y[e] = yn[e]; k[0][e] = k[6][e]; }
            t = tb;
            h *= fac;
            rejected = 0;
            if (!(t < tend)) retire(false);
        } else if (action == ACT_FAIL) {
            retire(true);
        }
    }

    // The dense output of element e as a polynomial in th, in FP64: u(th) = sum_k th^k w_k.
    // From u = y + th D + th(1-th) B + th^2(1-th) R4 + th^2(1-th)^2 R5 (D = yn - y,
    // B = h k1 - D, R4 = D - h k7 - B, R5 = h sum_j d_j k_j):
    // w = {y, D + B, R4 + R5 - B, -(R4 + 2 R5), R5}
    QTM_DI void dense_monomials(int e, double2 (&w)[5]) const {
        const double2 D = csub(yn[e], y[e]);
        const double2 B = csub(cscale(h, to_d2(k[0][e])), D);
        const double2 R4 = csub(csub(D, cscale(h, to_d2(k[6][e]))), B);
        const double2 R5 = cscale(h, cfma(dp_d(6), to_d2(k[6][e]), to_d2(ds[e])));
        w[0] = y[e];
        w[1] = cadd(D, B);
        w[2] = csub(cadd(R4, R5), B);
        w[3] = make_double2(-(R4.x + 2.0 * R5.x), -(R4.y + 2.0 * R5.y));
        w[4] = R5;
    }

    // Coefficients of the degree-8 polynomials <u(th)|u(th)> (P[0]) and <u(th)|O_j|u(th)>
    // (P[1 + j], the NO real diagonal observables O_j), reduced over the team, for the lanes
    // with on set: P[o][m] = sum over k + l = m of Re <w_k, O w_l> (both orders).  Every
    // output time of the step and the jump time's norm come from these 9 (NO + 1) sums.
    template <int NO> QTM_DI void poly_sums(bool on, double (&P)[NO + 1][9]) {
#pragma unroll
        for (int o = 0; o <= NO; ++o)
#pragma unroll
            for (int m = 0; m < 9; ++m) P[o][m] = 0.0;
        if (on) {
            const int qb = qbase();
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const int q = qb + cst(e);
                if (q >= d) continue;
                double2 w[5];
                dense_monomials(e, w);
                double o1[NO > 0 ? NO : 1], o2[NO > 0 ? NO : 1];
#pragma unroll
                for (int jo = 0; jo < NO; ++jo) { o1[jo] = Od[(size_t)jo * d + q].x; o2[jo] = 2.0 * o1[jo]; }
#pragma unroll
                for (int a = 0; a < 5; ++a)
#pragma unroll
                    for (int b = a; b < 5; ++b) {
                        const double pab = w[a].x * w[b].x + w[a].y * w[b].y;
                        if (a == b) P[0][a + b] += pab;
                        else P[0][a + b] = fma(2.0, pab, P[0][a + b]);
#pragma unroll
                        for (int jo = 0; jo < NO; ++jo) P[1 + jo][a + b] = fma(a == b ? o1[jo] : o2[jo], pab, P[1 + jo][a + b]);
                    }
            }
        }
        // team reductions of kXV values at a time
        constexpr int NV = (NO + 1) * 9;
#pragma unroll
        for (int c0 = 0; c0 < NV; c0 += kXV) {
            double tmp[kXV];
#pragma unroll
            for (int i = 0; i < kXV; ++i) tmp[i] = c0 + i < NV ? P[(c0 + i) / 9][(c0 + i) % 9] : 0.0;
            tsum<kXV>(tmp);
#pragma unroll
            for (int i = 0; i < kXV; ++i)
                if (c0 + i < NV) P[(c0 + i) / 9][(c0 + i) % 9] = tmp[i];
        }
    }

    QTM_DI static double horner8(const double (&p)[9], double x) {
        double v = p[8];
#pragma unroll
        for (int m = 7; m >= 0; --m) v = fma(v, x, p[m]);
        return v;
    }

    // Outputs inside the step from the polynomials: each lane evaluates its own output
    // times, t < t_k <= t + h (accepted step; t_k = t + h from th = 1) or t < t_k < t*
    // (jump step); no team reduction per output time
    template <int NO> QTM_DI void outputs_poly(bool on, const double (&P)[NO + 1][9]) {
        const bool acc = action == ACT_ACCEPT, jmp = action == ACT_JUMP;
        while (on) {
            const double tk = tnext;
            const bool out = kk < S.n_t && ((acc && tk <= tb) || (jmp && tk < tb));
            if (!out) break;
            const double th = (acc && tk == tb) ? 1.0 : (tk - t) / h;
            const double inn = 1.0 / horner8(P[0], th);
            if (lg == 0 && wv == 0) {
#pragma unroll
                for (int jo = 0; jo < NO; ++jo)
                    S.X[((size_t)traj * S.n_e + jo) * S.n_t + kk] = make_double2(horner8(P[1 + jo], th) * inn, 0.0);
            }
            kk++;
            tnext = tnext2;
            tnext2 = kk + 1 < S.n_t ? S.tlist[kk + 1] : 0.0;
        }
    }

    // Jump time of the lanes with action ACT_JUMP: the first th in [0, 1] where the
    // degree-8 norm polynomial p reaches r -- a 32-point scan for the first sign change,
    // then bisection to 1e-13
    QTM_DI void jump_root(const double (&p)[9]) {
        if (action == ACT_JUMP) {
            auto f = [&](double x) { return horner8(p, x) - r; };
            double lo = 0.0, hi = 1.0;
            int nev = 0;
            for (int m = 1; m <= 32; ++m) {
                double x = (double)m / 32.0;
                ++nev;
                if (f(x) < 0.0) { hi = x; lo = (double)(m - 1) / 32.0; break; }
            }
            while (hi - lo > 1e-13) {
                double mid = 0.5 * (lo + hi);
                ++nev;
                if (f(mid) < 0.0) hi = mid; else lo = mid;
            }
            // norm-polynomial evaluations into the run counters (jumps are rare: no register kept)
            if (lg == 0 && wv == 0) atomicAdd(&A.counters[1], (unsigned long long)nev);
            th = 0.5 * (lo + hi);
            tb = t + th * h;
        }
    }

    // Jump time for the other output paths: the norm polynomial alone
    QTM_DI void jump_time() {
        double P[1][9];
        poly_sums<0>(action == ACT_JUMP, P);
        jump_root(P[0]);
    }

    template <int NO> QTM_DI void gram_outputs(bool need) {
        double P[NO + 1][9];
        poly_sums<NO>(need, P);
        jump_root(P[0]);
        outputs_poly<NO>(need, P);
    }

    // this lane's part of ||C_n psi*||^2 (psi* staged), before the team reduction
    QTM_DI double chan_part(int n, bool on) const {
        double acc = 0.0;
        if (S.c_isdiag) {
            const double* g = S.f_diag + (size_t)(12 + n) * S.d;
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const int q = comp(e);
                if (on && q >= 0) acc += g[q] * cabs2(St[q * 16 + c16]);
            }
        } else {
            const int* rp = S.c_rp + (size_t)n * (S.d + 1);
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const int q = comp(e);
                if (on && q >= 0) acc += cabs2(csr_row(rp, S.c_ci, S.c_val, q));
            }
        }
        return acc;
    }

    // ||C_n psi*||^2 for this lane's trajectory (psi* staged); uniform call
    QTM_DI double chan_prob(int n, bool on) { return tsum1(chan_part(n, on)); }

    QTM_DI void do_jump() {
        const bool on = action == ACT_JUMP;
        {
            // psi* = u(theta*), written to the staging tile component by component
            const int qb = qbase();
            team_sync();                        // earlier readers of the staging tile are done
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const int q = qb + cst(e);
                if (q < d) St[q * 16 + c16] = on ? dense_at(e, th) : make_double2(0.0, 0.0);
            }
            team_sync();
        }
        // channel: smallest n with sum_{m<=n} p_m >= u * sum p; the probabilities of
        // kXV channels at a time in one team reduction
        double tot = 0.0, pn[kMaxC];
        for (int n0 = 0; n0 < S.n_c; n0 += kXV) {
            double pc[kXV];
#pragma unroll
            for (int i = 0; i < kXV; ++i) pc[i] = n0 + i < S.n_c ? chan_part(n0 + i, on) : 0.0;
            tsum<kXV>(pc);
#pragma unroll
            for (int i = 0; i < kXV; ++i)
                if (n0 + i < S.n_c) pn[n0 + i] = pc[i];
        }
        for (int n = 0; n < S.n_c; ++n) tot += pn[n];
        const double thr = u * tot;
        double cum = 0.0, plast = 0.0, pch = 0.0;
        int lastpos = -1, chosen = -1;
        for (int n = 0; n < S.n_c; ++n) {
            const double pv = pn[n];
            cum += pv;
            if (pv > 0.0) { lastpos = n; plast = pv; }
            if (chosen < 0 && pv > 0.0 && cum >= thr) { chosen = n; pch = pv; }
        }
        if (tot > 0.0 && chosen < 0) { chosen = lastpos; pch = plast; }   // rounding left none: last with p > 0
        if (!(tot > 0.0)) chosen = -1;
        if (on) ch = chosen;
        // y <- C_ch psi* / sqrt(p_ch)  (no channel: renormalised psi*)
        double nrm = 0.0;
        if (on) {
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                int q = comp(e);
                if (q < 0) { y[e] = make_double2(0.0, 0.0); continue; }
                if (ch >= 0) {
                    double2 cv;
                    if (Cjc) {
                        const int j = ch * S.d + q, c = Cjc[j];
                        cv = c >= 0 ? cmul(Cjv[j], St[c * 16 + c16]) : make_double2(0.0, 0.0);
                    } else {
                        cv = csr_row(S.c_rp + (size_t)ch * (S.d + 1), S.c_ci, S.c_val, q);
                    }
                    y[e] = cscale(1.0 / sqrt(pch), cv);
                }
                else { y[e] = St[q * 16 + c16]; nrm += cabs2(y[e]); }
            }
        }
        nrm = tsum1(nrm);
        if (on && ch < 0) {
#pragma unroll
            for (int e = 0; e < NE; ++e) y[e] = cscale(1.0 / sqrt(nrm), y[e]);
        }
        if (on) {
            if (lg == 0 && wv == 0) {
                if (njump < A.jcap) {
                    S.jt[(size_t)traj * A.jcap + njump] = tb;
                    S.jc[(size_t)traj * A.jcap + njump] = ch;
                }
                if (A.seg_cap > 0 && seg_rec < A.seg_cap) {
                    float* rec = S.segs + ((size_t)traj * A.seg_cap + seg_rec) * kSegRec;
                    rec[16] = (float)(tb - tseg);
                    rec[18] = 0.f;
                }
            }
            njump++;
            t = tb;
            // a new segment; an output time equal to the jump time is recorded from the
            // post-jump state at the start of the next pass (with the new trajectories'
            // first outputs), which keeps a single copy of the output code per phase
            action = ACT_NONE;
            seg++;
            seg_rec++;
            state = ST_NEEDK1;
        }
    }
};

// LDS of a block: [A-fragments of M][A-fragments of the ntd time-dependent terms kept in
// LDS][per team: operand tile, team exchange, hand-out, flags][diagonal observables][FP32
// feature table].  Blocks of single-wave teams hold TPB teams that share M and never meet
// at a barrier after the set-up.
struct TeamLds { size_t m, team, w, x, ib, fb, od, ft, cj, total; };
// ncj: channels of the LDS jump table (one entry per row: column, value), 0 for none
static __host__ __device__ TeamLds team_lds(int dp, int d, int n_e, int prec, int nwt, int tpb, int od_lds,
                                            int ntd = 0, int ncj = 0) {
    TeamLds L;
    size_t es = prec == 0 ? 8 : 4;
    L.m = 0;
    L.w = (((size_t)(1 + ntd) * (2 * dp) * (2 * dp) * es) + 15) & ~(size_t)15;   // first team's tile
    L.x = (size_t)2 * dp * 16 * sizeof(double);                             // offsets inside a team
    L.ib = L.x + (size_t)nwt * 16 * kXV * sizeof(double);
    L.fb = L.ib + 16 * sizeof(unsigned long long);
    L.team = (L.fb + 4 * (size_t)(nwt > 4 ? nwt : 4) + 15) & ~(size_t)15;  // bytes per team (one flag per wave)
    L.od = L.w + (size_t)tpb * L.team;
    L.ft = L.od + (od_lds ? (size_t)n_e * d * sizeof(double2) : 0);
    L.cj = (L.ft + (size_t)16 * d * sizeof(float) + 15) & ~(size_t)15;   // after the FP32 feature table [d][16]
    L.total = L.cj + (size_t)ncj * d * (sizeof(double2) + sizeof(int));
    return L;
}

// td_lds (TD instances): the time-dependent terms' fragments are copied into LDS after M
// (otherwise read from global memory).  cj_lds: every C_n has at most one entry per row,
// and the (column, value) of each row's entry is tabulated in LDS for the jumps (otherwise
// the rows are read from the CSR arrays in global memory, a chain of dependent loads).
template <int T, int NWT, int PREC, int BAND = 0, bool TD = false>
__global__ void __launch_bounds__(NWT == 1 ? 256 : 64 * NWT) traj_team_kernel(RunArgs a, int od_lds, int tpb, int td_lds,
                                                                              int cj_lds) {
    typedef typename MfmaT<PREC>::in_t in_t;
    extern __shared__ double smem[];
    const DevSystem& S = a.sys[0];
    const int ntd_lds = (TD && td_lds) ? S.n_td : 0;
    const int ncj = cj_lds ? S.n_c : 0;
    const TeamLds L = team_lds(S.dp, S.d, S.n_e, PREC, NWT, tpb, od_lds, ntd_lds, ncj);
    char* base = (char*)smem;
    const in_t* Mg = MfmaT<PREC>::frag(S);
    in_t* Ml = (in_t*)(base + L.m);
    const size_t nm = (size_t)(2 * S.dp) * (2 * S.dp);
    for (size_t i = threadIdx.x; i < nm; i += blockDim.x) Ml[i] = Mg[i];
    if constexpr (TD) {
        const in_t* Tg = MfmaT<PREC>::td(S);
        for (size_t i = threadIdx.x; i < (size_t)ntd_lds * nm; i += blockDim.x) Ml[nm + i] = Tg[i];
    }
    double2* Odl = (double2*)(base + L.od);
    if (od_lds)
        for (int o = 0; o < S.n_e; ++o)
            for (int i = threadIdx.x; i < S.d; i += blockDim.x) Odl[(size_t)o * S.d + i] = S.e_val[S.e_doff[o] + i];
    // segment-start features: rows 0..11 of the diagonal table and, when C^dag C is
    // diagonal, rows 12..13 (first two channels), in FP32
    float* Ftl = (float*)(base + L.ft);
    for (int i = threadIdx.x; i < 16 * S.d; i += blockDim.x) {
        const int q = i >> 4, row = i & 15;
        const bool have = row < 12 || (row < 14 && S.c_isdiag && row - 12 < S.n_c);
        Ftl[i] = have ? (float)S.f_diag[(size_t)row * S.d + q] : 0.f;
    }
    double2* Cjv = (double2*)(base + L.cj);
    int* Cjc = (int*)(Cjv + (size_t)ncj * S.d);
    for (int i = threadIdx.x; i < ncj * S.d; i += blockDim.x) {
        const int n = i / S.d, q = i - n * S.d;
        const int* rp = S.c_rp + (size_t)n * (S.d + 1);
        const int p0 = rp[q];
        const bool has = rp[q + 1] > p0;
        Cjc[i] = has ? S.c_ci[p0] : -1;
        Cjv[i] = has ? S.c_val[p0] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int team = (threadIdx.x >> 6) / NWT;
    char* tb = base + L.w + (size_t)team * L.team;
    Team<T, NWT, PREC, true, BAND, TD> W(S, a);
    W.Mf = Ml;
    W.Mt = ntd_lds ? (const in_t*)(Ml + nm) : MfmaT<PREC>::td(S);
    W.Wb = (in_t*)tb;
    W.St = (double2*)tb;
    W.Xb = (double*)(tb + L.x);
    W.Ib = (unsigned long long*)(tb + L.ib);
    W.Fb = (int*)(tb + L.fb);
    W.Od = Odl;
    W.od_lds = od_lds;
    W.Ft = Ftl;
    W.Cjc = ncj ? Cjc : nullptr;
    W.Cjv = Cjv;
    W.lane = threadIdx.x & 63;
    W.wv = (threadIdx.x >> 6) % NWT;
    W.lg = W.lane >> 4;
    W.c16 = W.lane & 15;
    W.d = S.d;
    W.dp = S.dp;
    W.RT = 2 * S.dp / 16;
    W.q0 = 8 * T * W.wv + (PREC == 0 ? W.lg : 2 * W.lg);
    W.run();
    if ((threadIdx.x & 63) == 0 && W.wv == 0) {
        atomicAdd(&a.counters[0], W.passes);
        atomicMax(&a.counters[2], W.passes);
    }
}

// LDS of a batch block: one team whose operator stays in global memory; tables sized
// for the largest system of its tile class.
static __host__ __device__ TeamLds team_lds_batch(int dpmax, int dmax, int nemax, int nwt) {
    TeamLds L;
    L.m = 0;
    L.w = 0;
    L.x = (size_t)2 * dpmax * 16 * sizeof(double);
    L.ib = L.x + (size_t)nwt * 16 * kXV * sizeof(double);
    L.fb = L.ib + 16 * sizeof(unsigned long long);
    L.team = (L.fb + 4 * (size_t)(nwt > 4 ? nwt : 4) + 15) & ~(size_t)15;  // one flag per wave
    L.od = L.team;
    L.ft = L.od + (size_t)nemax * dmax * sizeof(double2);
    L.total = L.ft + (size_t)16 * dmax * sizeof(float);
    return L;
}

// A batch's dense systems of one tile class in one persistent launch: the block (one
// team) takes the first system whose trajectory queue is not exhausted, runs it with
// slot refill until the queue runs dry, then moves on; a.sys_cursor skips finished
// systems.  A-fragments of each system's operator are read from global memory (L2).
template <int T, int NWT, int PREC>
__global__ void __launch_bounds__(64 * NWT) traj_team_batch_kernel(RunArgs a, int dpmax, int dmax, int nemax) {
    typedef typename MfmaT<PREC>::in_t in_t;
    extern __shared__ double smem[];
    __shared__ int cur;
    const TeamLds L = team_lds_batch(dpmax, dmax, nemax, NWT);
    char* base = (char*)smem;
    unsigned long long passes = 0, pmax = 0;
    // XCD-aware hand-out: with a.xcd_off the class's systems are split into eight lists,
    // one per XCD (blocks are dispatched to the XCDs round-robin), so that the blocks of
    // an XCD share the operators held in that XCD's L2; a block that has emptied its own
    // list takes work from the others in turn
    const int nseg = a.xcd_off ? 8 : 1;
    const int home = a.xcd_off ? (int)(blockIdx.x % 8) : 0;
    for (int g = 0; g < nseg; ++g) {
    const int seg = (home + g) % nseg;
    const int lo = a.xcd_off ? a.xcd_off[seg] : 0, hi = a.xcd_off ? a.xcd_off[seg + 1] : a.n_sys;
    unsigned int* cursor = a.sys_cursor + seg;
    int si = lo;
    for (;;) {
        if (threadIdx.x == 0) {
            int s2 = max(si, (int)__atomic_load_n(cursor, __ATOMIC_RELAXED));
            while (s2 < hi &&
                   __atomic_load_n(a.sys[s2].queue, __ATOMIC_RELAXED) >= (unsigned long long)a.sys[s2].count) {
                atomicMax(cursor, (unsigned int)(s2 + 1));
                ++s2;
            }
            cur = s2;
        }
        __syncthreads();
        si = cur;
        // every wave has read cur before thread 0 may write it again: on the break path
        // the next write (the next list's hand-out) follows with no other barrier between
        __syncthreads();
        if (si >= hi) break;
        const DevSystem& S = a.sys[si];
        int od_lds = S.any_csr_e ? 0 : 2;
        for (int o = 0; o < S.n_e && od_lds; ++o) if (S.e_nv[o] != 1) od_lds = 1;
        double2* Odl = (double2*)(base + L.od);
        if (od_lds)
            for (int o = 0; o < S.n_e; ++o)
                for (int i = threadIdx.x; i < S.d; i += blockDim.x) Odl[(size_t)o * S.d + i] = S.e_val[S.e_doff[o] + i];
        float* Ftl = (float*)(base + L.ft);
        for (int i = threadIdx.x; i < 16 * S.d; i += blockDim.x) {
            const int q = i >> 4, row = i & 15;
            const bool have = row < 12 || (row < 14 && S.c_isdiag && row - 12 < S.n_c);
            Ftl[i] = have ? (float)S.f_diag[(size_t)row * S.d + q] : 0.f;
        }
        __syncthreads();
        Team<T, NWT, PREC, false> W(S, a);
        W.Mf = MfmaT<PREC>::team(S);
        W.Mt = nullptr;
        W.Wb = (in_t*)(base + L.w);
        W.St = (double2*)(base + L.w);
        W.Xb = (double*)(base + L.x);
        W.Ib = (unsigned long long*)(base + L.ib);
        W.Fb = (int*)(base + L.fb);
        W.Od = Odl;
        W.od_lds = od_lds;
        W.Ft = Ftl;
        W.lane = threadIdx.x & 63;
        W.wv = threadIdx.x >> 6;
        W.lg = W.lane >> 4;
        W.c16 = W.lane & 15;
        W.d = S.d;
        W.dp = S.dp;
        W.RT = 2 * S.dp / 16;
        W.q0 = 8 * T * W.wv + (PREC == 0 ? W.lg : 2 * W.lg);
        W.run();
        passes += W.passes;
        pmax = W.passes > pmax ? W.passes : pmax;
        __syncthreads();                 // the block leaves the system together
        ++si;
    }
    }
    if (threadIdx.x == 0) {
        atomicAdd(&a.counters[0], passes);
        atomicMax(&a.counters[2], pmax);
    }
}

#ifndef QTM_WAVE_INSTANCES
// Instances live in per-shape translation units (qtm_wave_t*.hip) so that they
// compile in parallel; each defines QTM_WAVE_INSTANCES.
template <int T, int NWT, int PREC> const void* team_fn_inst();
template <int T, int PREC> const void* team_fn_band_inst();   // single-wave teams, banded operator
template <int T, int NWT, int PREC> const void* team_fn_td_inst();   // default shapes, time-dependent terms

// Team shapes (T row tiles per wave, NWT waves per team) compiled for each number
// of 16-row tiles RT = 2 dp / 16; the first entry of a row is the default.
static const int kShapes[9][3][2] = {
    {{0, 0}, {0, 0}, {0, 0}},
    {{1, 1}, {0, 0}, {0, 0}},
    {{2, 1}, {1, 2}, {0, 0}},
    {{3, 1}, {2, 2}, {1, 3}},
    {{4, 1}, {2, 2}, {1, 4}},
    {{5, 1}, {3, 2}, {1, 5}},
    {{3, 2}, {2, 3}, {1, 6}},
    {{4, 2}, {1, 7}, {0, 0}},
    {{2, 4}, {4, 2}, {1, 8}},
};

// waves_per_team: 0 = default shape, else the listed shape with that many waves
static int team_shape(int rt, int waves_per_team, int* T, int* nwt) {
    if (rt < 1 || rt > 8) return -1;
    for (int i = 0; i < 3; ++i) {
        int tt = kShapes[rt][i][0], nn = kShapes[rt][i][1];
        if (!tt) break;
        if (waves_per_team == 0 || waves_per_team == nn) { *T = tt; *nwt = nn; return 0; }
    }
    return -1;
}

static const void* team_fn(int T, int nwt, int prec) {
#define QTM_TEAM_CASE(TT, NN) \
    if (T == TT && nwt == NN) return prec == 0 ? team_fn_inst<TT, NN, 0>() : team_fn_inst<TT, NN, 1>();
    QTM_TEAM_CASE(1, 1) QTM_TEAM_CASE(2, 1) QTM_TEAM_CASE(1, 2) QTM_TEAM_CASE(1, 3) QTM_TEAM_CASE(1, 4)
    QTM_TEAM_CASE(2, 2) QTM_TEAM_CASE(1, 5) QTM_TEAM_CASE(3, 2) QTM_TEAM_CASE(5, 1) QTM_TEAM_CASE(1, 6)
    QTM_TEAM_CASE(2, 3) QTM_TEAM_CASE(1, 7) QTM_TEAM_CASE(4, 2) QTM_TEAM_CASE(1, 8) QTM_TEAM_CASE(2, 4)
    QTM_TEAM_CASE(3, 1) QTM_TEAM_CASE(4, 1)
#undef QTM_TEAM_CASE
    return nullptr;
}

// Team sizes available for dimension d (waves per team), for the autotuner.
int team_candidates(int d, int* waves, int cap) {
    int dp = (d + 7) / 8 * 8, rt = 2 * dp / 16, n = 0;
    if (rt < 1 || rt > 8) return 0;
    for (int i = 0; i < 3 && n < cap; ++i)
        if (kShapes[rt][i][0]) waves[n++] = kShapes[rt][i][1];
    return n;
}

int wave_supported(int d) {
    int dp = (d + 7) / 8 * 8, rt = 2 * dp / 16, T, nwt;
    return team_shape(rt, 0, &T, &nwt) == 0;
}

// LDS of a team-kernel block for one shape; tpb reduced until it fits (0 if it never does)
static size_t team_block_lds(int dp, const DevSystem& s0, int prec, int nwt, int od_lds, int* tpb, int ntd = 0) {
    *tpb = nwt == 1 ? 4 : 1;
    TeamLds L = team_lds(dp, s0.d, s0.n_e, prec, nwt, *tpb, od_lds, ntd);
    while (*tpb > 1 && L.total > 160 * 1024) L = team_lds(dp, s0.d, s0.n_e, prec, nwt, --*tpb, od_lds, ntd);
    return L.total > 160 * 1024 ? 0 : L.total;
}

// The time-dependent instance of the default shape for RT tiles (see kShapes)
static const void* team_fn_td(int T, int nwt, int prec) {
#define QTM_TD_CASE(TT, NN) \
    if (T == TT && nwt == NN) return prec == 0 ? team_fn_td_inst<TT, NN, 0>() : team_fn_td_inst<TT, NN, 1>();
    QTM_TD_CASE(1, 1) QTM_TD_CASE(2, 1) QTM_TD_CASE(3, 1) QTM_TD_CASE(4, 1) QTM_TD_CASE(5, 1)
    QTM_TD_CASE(3, 2) QTM_TD_CASE(4, 2) QTM_TD_CASE(2, 4)
#undef QTM_TD_CASE
    return nullptr;
}

int launch_wave(const RunArgs& a, const DevSystem& s0, int prec, int waves_per_team, hipStream_t st, LaunchInfo* info) {
    int dp = s0.dp, rt = 2 * dp / 16, T, nwt;
    if (team_shape(rt, waves_per_team, &T, &nwt)) return -1;
    // diagonal observables are copied to LDS when every observable is diagonal
    int od_lds = 2;                              // 2: every observable real as well
    for (int o = 0; o < s0.n_e; ++o) if (s0.e_nv[o] != 1) od_lds = 1;
    for (int o = 0; o < s0.n_e; ++o) if (s0.e_fmt[o] != 2) od_lds = 0;
    // single-wave teams: up to 4 per block, sharing the operator in LDS; a shape whose
    // block does not fit the 160 KB of LDS gives way to the next shape of the same tile count
    int tpb = 1;
    if (s0.n_td > 0) {
        // time-dependent terms: the default shape only; their fragments in LDS when they fit
        int T0, n0;
        team_shape(rt, 0, &T0, &n0);
        if (waves_per_team != 0 && waves_per_team != n0) return -1;
        T = T0; nwt = n0;
        int td_lds = 1;
        size_t ltd = team_block_lds(dp, s0, prec, nwt, od_lds, &tpb, s0.n_td);
        if (ltd == 0) { td_lds = 0; ltd = team_block_lds(dp, s0, prec, nwt, od_lds, &tpb); }
        if (ltd == 0 && od_lds) { od_lds = 0; ltd = team_block_lds(dp, s0, prec, nwt, od_lds, &tpb); }
        if (ltd == 0) return -2;
        int cj_lds = 0;
        if (s0.c_isdiag && s0.n_c > 0) {
            const size_t l2 = team_lds(dp, s0.d, s0.n_e, prec, nwt, tpb, od_lds, td_lds ? s0.n_td : 0, s0.n_c).total;
            if (l2 <= 160 * 1024) { ltd = l2; cj_lds = 1; }
        }
        const void* fn = team_fn_td(T, nwt, prec);
        if (!fn) return -1;
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ltd) != hipSuccess) return -3;
        int dev = 0, ncu = 0, nb = 1;
        const int threads = nwt * tpb * 64;
        if (hipGetDevice(&dev) != hipSuccess) return -3;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -3;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, ltd) != hipSuccess || nb < 1) nb = 1;
        const int cols = 16 * tpb;
        long long need = (s0.count + cols - 1) / cols;
        long long blocks = a.persistent ? (long long)ncu * nb : need;
        if (blocks > need) blocks = need;
        if (blocks < 1) blocks = 1;
        void* args[] = {(void*)&a, (void*)&od_lds, (void*)&tpb, (void*)&td_lds, (void*)&cj_lds};
        if (hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(threads), args, ltd, st) != hipSuccess) return -3;
        if (info) {
            info->blocks = (int)blocks; info->threads = threads; info->lds = (int)ltd; info->cols = cols;
            info->shape = T * 100 + nwt;
        }
        return hipGetLastError() == hipSuccess ? 0 : -3;
    }
    size_t lds = team_block_lds(dp, s0, prec, nwt, od_lds, &tpb);
    for (int i = 0; i < 3 && lds == 0 && waves_per_team == 0; ++i) {
        T = kShapes[rt][i][0]; nwt = kShapes[rt][i][1];
        if (T) lds = team_block_lds(dp, s0, prec, nwt, od_lds, &tpb);
    }
    if (lds == 0 && od_lds) {                    // observables stay in global memory
        od_lds = 0;
        team_shape(rt, waves_per_team, &T, &nwt);
        lds = team_block_lds(dp, s0, prec, nwt, od_lds, &tpb);
        for (int i = 0; i < 3 && lds == 0 && waves_per_team == 0; ++i) {
            T = kShapes[rt][i][0]; nwt = kShapes[rt][i][1];
            if (T) lds = team_block_lds(dp, s0, prec, nwt, od_lds, &tpb);
        }
    }
    if (lds == 0) return -2;
    if (nwt == 1 && T != rt) return -1;          // a single-wave team holds every source tile
    const void* fn = team_fn(T, nwt, prec);
    if (nwt == 1 && s0.tile_band && T == 4) fn = prec == 0 ? team_fn_band_inst<4, 0>() : team_fn_band_inst<4, 1>();
    if (nwt == 1 && s0.tile_band && T == 5) fn = prec == 0 ? team_fn_band_inst<5, 0>() : team_fn_band_inst<5, 1>();
    if (!fn) return -1;
    // the jump table joins the LDS when it fits without fewer teams per block
    int cj_lds = 0;
    if (s0.c_isdiag && s0.n_c > 0) {
        const size_t l2 = team_lds(dp, s0.d, s0.n_e, prec, nwt, tpb, od_lds, 0, s0.n_c).total;
        if (l2 <= 160 * 1024) { lds = l2; cj_lds = 1; }
    }
    TeamLds L;
    L.total = lds;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total) != hipSuccess) return -3;
    int dev = 0, ncu = 0, nb = 1;
    const int threads = nwt * tpb * 64;
    if (hipGetDevice(&dev) != hipSuccess) return -3;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -3;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, L.total) != hipSuccess || nb < 1) nb = 1;
    const int cols = 16 * tpb;
    long long need = (s0.count + cols - 1) / cols;
    long long blocks = a.persistent ? (long long)ncu * nb : need;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    int td_lds = 0;
    void* args[] = {(void*)&a, (void*)&od_lds, (void*)&tpb, (void*)&td_lds, (void*)&cj_lds};
    if (hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(threads), args, L.total, st) != hipSuccess) return -3;
    const bool band = nwt == 1 && s0.tile_band && (T == 4 || T == 5);
    if (info) {
        info->blocks = (int)blocks; info->threads = threads; info->lds = (int)L.total; info->cols = cols;
        info->shape = T * 100 + nwt + (band ? 1000 : 0);
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
#endif  // QTM_WAVE_INSTANCES

}  // namespace qtm
