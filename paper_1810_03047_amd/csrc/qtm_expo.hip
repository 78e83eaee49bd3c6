// qtm_expo.hip -- the exact-propagator (stiff) form of the trajectory kernel.
//
// For a time-independent effective Hamiltonian the no-jump evolution between two
// times is psi(t + tau) = exp(tau M) psi(t).  With the output times on a uniform grid
// of spacing m h, a single-wave team of 16 trajectories advances every trajectory by
// one product with P_0 = exp(h M) per interval, whatever the stiffness of M (the
// reason the paper offers BDF, Sec. 2.1).  The squared norm is non-increasing, so a
// jump lies in the first interval whose end norm is below the threshold r; it is
// located by a binary search over positions p / 2^J of the interval with the exact
// sub-propagators P_j = exp(h 2^-j M): from the last position known to be above r,
// the candidate P_j psi is kept when its norm is still at least r.  After the jump
// the new state is carried to the end of the interval by the P_j of the binary digits
// of 2^J - p.  Search and carry share one pass over j = 1..J (the operand of each
// MFMA column, a trajectory, is that trajectory's own vector), so a team pays J
// products for every pass in which any of its trajectories jumps.
//
// FP64 products only (no step-size control absorbs rounding here), d <= 40
// (single-wave teams, T = RT <= 5).  Outputs, channel choice, jump and random
// streams are those of the DOPRI5 team kernel.
#define QTM_WAVE_INSTANCES
#include "qtm_wave.hip"

namespace qtm {

enum : int { EX_ADV = 10, EX_SEARCH = 11 };

template <int T>
struct ExpTeam : Team<T, 1, 0, false, 0, false> {
    typedef Team<T, 1, 0, false, 0, false> B;
    using B::NE; using B::S; using B::A; using B::y; using B::yn; using B::k;
    using B::lane; using B::lg; using B::wv; using B::c16; using B::d; using B::state; using B::traj;
    using B::kk; using B::seg; using B::njump; using B::nacc; using B::nrej; using B::omode; using B::r; using B::u;
    using B::exhausted; using B::Ib; using B::St; using B::Mf; using B::passes;

    const double* P0;        // LDS: exp(h M) fragments
    const double* Pg;        // global: [J][RT][RT][64][4] fragments of exp(h 2^-j M), j = 1..J
    int J, m;
    long long NS;            // intervals from t0 to t_end
    double h;
    unsigned long long pos;  // position in the current interval, units h 2^-J
    long long nint;          // intervals completed

    QTM_DI ExpTeam(const DevSystem& s, const RunArgs& a) : B(s, a) {}

    QTM_DI void draw() {
        uint64_t ctr[4] = {(uint64_t)(S.traj_begin + traj), (uint64_t)seg, 0, 0};
        philox4x64(ctr, S.key0, S.key1);
        r = u53(ctr[0]);
        u = u53(ctr[1]);
    }
    QTM_DI double norm2(const double2 (&v)[B::NE]) {
        double s = 0.0;
#pragma unroll
        for (int e = 0; e < NE; ++e)
            if (this->comp(e) >= 0) s += cabs2(v[e]);
        return this->tsum1(s);
    }

    QTM_DI void run() {
        state = ST_EMPTY; traj = -1; omode = 0; exhausted = false;
        kk = seg = njump = nacc = nrej = 0;
        r = u = 0.0;
        pos = 0; nint = 0;
#pragma unroll
        for (int e = 0; e < NE; ++e) { y[e] = yn[e] = k[0][e] = make_double2(0.0, 0.0); }
        long long cycles = 0;
        bool first = true;
        passes = 0;
        const unsigned long long full = 1ULL << J;
        for (;;) {
            // ---- refill empty slots
            bool want = state == ST_EMPTY && !exhausted && (A.persistent || first);
            first = false;
            if (wv == 0 && lg == 0) Ib[c16] = want ? atomicAdd(S.queue, 1ULL) : 0ULL;
            this->team_sync();
            unsigned long long idx = Ib[c16];
            this->team_sync();
            if (want) {
                if ((long long)idx < S.count) {
                    traj = (long long)idx;
                    seg = 0; kk = 0; njump = 0; nacc = 0; nrej = 0;
                    pos = 0; nint = 0;
                    state = ST_NEW;
                } else {
                    exhausted = true;
                }
            }
            if (!this->team_any(state != ST_EMPTY)) break;
            if (++cycles > A.max_cycles) {
                if (state != ST_EMPTY) this->retire(true);
                break;
            }
            // ---- new trajectories: psi0, the output at t0, the first threshold
            if (this->team_any(state == ST_NEW)) {
#pragma unroll
                for (int e = 0; e < NE; ++e) {
                    const int q = this->comp(e);
                    if (state == ST_NEW) y[e] = q >= 0 ? S.psi0[q] : make_double2(0.0, 0.0);
                }
                omode = state == ST_NEW ? 1 : 0;
                this->output_round(omode != 0);
                if (state == ST_NEW) {
                    kk = 1;
                    draw();
                    state = EX_ADV;
                }
                omode = 0;
            }
            // ---- 1. trajectories at the start of an interval: one product with P_0
            const bool adv0 = state == EX_ADV && pos == 0;
            if (this->team_any(adv0)) {
                Mf = P0;
                this->product(y, k[0]);
                if (adv0) {
#pragma unroll
                    for (int e = 0; e < NE; ++e) yn[e] = k[0][e];
                }
            }
            // ---- 2. carry (after a jump inside the interval) and search, j = 1..J
            const bool rs = state == EX_ADV && pos > 0;
            const bool sr = state == EX_SEARCH;
            if (this->team_any(rs || sr)) {
                const unsigned long long rem = full - pos;
                if (rs) {
#pragma unroll
                    for (int e = 0; e < NE; ++e) yn[e] = y[e];
                }
                for (int j = 1; j <= J; ++j) {
                    const unsigned long long stepj = 1ULL << (J - j);
                    double2 w[B::NE];
#pragma unroll
                    for (int e = 0; e < NE; ++e) w[e] = rs ? yn[e] : y[e];
                    Mf = Pg + (size_t)(j - 1) * (size_t)(T * T * 256);
                    this->product(w, k[0]);
                    const bool test = sr && pos + stepj < full;
                    double nn = 0.0;
#pragma unroll
                    for (int e = 0; e < NE; ++e)
                        if (test && this->comp(e) >= 0) nn += cabs2(k[0][e]);
                    nn = this->tsum1(nn);
                    if (test && nn >= r) {
#pragma unroll
                        for (int e = 0; e < NE; ++e) y[e] = k[0][e];
                        pos += stepj;
                    }
                    if (rs && (rem & stepj)) {
#pragma unroll
                        for (int e = 0; e < NE; ++e) yn[e] = k[0][e];
                    }
                }
            }
            // ---- 3. end of the interval: accept, or search the interval in the next pass
            const bool ended = adv0 || rs;
            if (this->team_any(ended)) {
                const double nn = norm2(yn);
                bool out = false;
                if (ended) {
                    if (nn >= r) {
#pragma unroll
                        for (int e = 0; e < NE; ++e) y[e] = yn[e];
                        pos = 0;
                        ++nint;
                        ++nacc;
                        out = nint % m == 0;
                    } else {
                        state = EX_SEARCH;
                    }
                }
                omode = out ? 1 : 0;
                if (this->team_any(out)) this->output_round(out);
                omode = 0;
                if (out) ++kk;
                if (ended && state == EX_ADV && nint >= NS) this->retire(false);
            }
            // ---- 4. jumps at the positions the searches found
            if (this->team_any(sr)) jump(sr);
        }
    }

    // psi* = y at position pos of interval nint: channel, jump, new threshold
    QTM_DI void jump(bool on) {
        double2 v[B::NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) v[e] = on ? y[e] : make_double2(0.0, 0.0);
        this->stage_vec(v);
        double tot = 0.0;
        for (int n = 0; n < S.n_c; ++n) tot += this->chan_prob(n, on);
        const double thr = u * tot;
        double cum = 0.0, plast = 0.0, pch = 0.0;
        int lastpos = -1, chosen = -1;
        for (int n = 0; n < S.n_c; ++n) {
            const double pv = this->chan_prob(n, on);
            cum += pv;
            if (pv > 0.0) { lastpos = n; plast = pv; }
            if (chosen < 0 && pv > 0.0 && cum >= thr) { chosen = n; pch = pv; }
        }
        if (tot > 0.0 && chosen < 0) { chosen = lastpos; pch = plast; }
        if (!(tot > 0.0)) chosen = -1;
        double nrm = 0.0;
        if (on) {
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const int q = this->comp(e);
                if (q < 0) { y[e] = make_double2(0.0, 0.0); continue; }
                if (chosen >= 0) y[e] = cscale(1.0 / sqrt(pch), this->csr_row(S.c_rp + (size_t)chosen * (S.d + 1), S.c_ci, S.c_val, q));
                else { y[e] = St[q * 16 + c16]; nrm += cabs2(y[e]); }
            }
        }
        nrm = this->tsum1(nrm);
        if (on && chosen < 0) {
#pragma unroll
            for (int e = 0; e < NE; ++e) y[e] = cscale(1.0 / sqrt(nrm), y[e]);
        }
        if (on) {
            if (lg == 0 && wv == 0 && njump < A.jcap) {
                S.jt[(size_t)traj * A.jcap + njump] = S.t0 + ((double)nint + ldexp((double)pos, -J)) * h;
                S.jc[(size_t)traj * A.jcap + njump] = chosen;
            }
            ++njump;
            ++seg;
            draw();
            state = EX_ADV;
        }
    }
};

// LDS of a block: [P_0 fragments][per team: staging tile, exchange, hand-out, flags]
// [diagonal observables][FP32 feature table] (the team kernel's layout with one operator)
template <int T>
__global__ void __launch_bounds__(256) traj_expo_kernel(RunArgs a, int od_lds, int tpb, const double* Pg, int J,
                                                        int m, double h, long long NS) {
    extern __shared__ double smem[];
    const DevSystem& S = a.sys[0];
    const TeamLds L = team_lds(S.dp, S.d, S.n_e, 0, 1, tpb, od_lds);
    char* base = (char*)smem;
    double* Pl = (double*)(base + L.m);
    const size_t nm = (size_t)(2 * S.dp) * (2 * S.dp);
    for (size_t i = threadIdx.x; i < nm; i += blockDim.x) Pl[i] = Pg[i];
    double2* Odl = (double2*)(base + L.od);
    if (od_lds)
        for (int o = 0; o < S.n_e; ++o)
            for (int i = threadIdx.x; i < S.d; i += blockDim.x) Odl[(size_t)o * S.d + i] = S.e_val[S.e_doff[o] + i];
    __syncthreads();
    const int team = threadIdx.x >> 6;
    char* tb = base + L.w + (size_t)team * L.team;
    ExpTeam<T> W(S, a);
    W.Mf = Pl;
    W.Mt = nullptr;
    W.P0 = Pl;
    W.Pg = Pg + nm;
    W.J = J; W.m = m; W.h = h; W.NS = NS;
    W.Wb = (double*)tb;
    W.St = (double2*)tb;
    W.Xb = (double*)(tb + L.x);
    W.Ib = (unsigned long long*)(tb + L.ib);
    W.Fb = (int*)(tb + L.fb);
    W.Od = Odl;
    W.od_lds = od_lds;
    W.Ft = nullptr;
    W.lane = threadIdx.x & 63;
    W.wv = 0;
    W.lg = W.lane >> 4;
    W.c16 = W.lane & 15;
    W.d = S.d;
    W.dp = S.dp;
    W.RT = 2 * S.dp / 16;
    W.q0 = W.lg;
    W.run();
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&a.counters[0], W.passes);
        atomicMax(&a.counters[2], W.passes);
    }
}

template <int T> static const void* expo_fn() { return (const void*)&traj_expo_kernel<T>; }

// One launch of the exact-propagator kernel for system s0 (d <= 40, FP64): Pg holds J + 1
// propagator fragment sets, exp(h 2^-j M) for j = 0..J.
int launch_expo(const RunArgs& a, const DevSystem& s0, const double* Pg, int J, int m, double h, long long NS,
                hipStream_t st, LaunchInfo* info) {
    const int rt = 2 * s0.dp / 16;
    if (rt < 1 || rt > 5) return -1;
    int od_lds = 2;
    for (int o = 0; o < s0.n_e; ++o) if (s0.e_nv[o] != 1) od_lds = 1;
    for (int o = 0; o < s0.n_e; ++o) if (s0.e_fmt[o] != 2) od_lds = 0;
    int tpb = 4;
    TeamLds L = team_lds(s0.dp, s0.d, s0.n_e, 0, 1, tpb, od_lds);
    while (tpb > 1 && L.total > 160 * 1024) L = team_lds(s0.dp, s0.d, s0.n_e, 0, 1, --tpb, od_lds);
    if (L.total > 160 * 1024 && od_lds) { od_lds = 0; tpb = 4; L = team_lds(s0.dp, s0.d, s0.n_e, 0, 1, tpb, od_lds);
        while (tpb > 1 && L.total > 160 * 1024) L = team_lds(s0.dp, s0.d, s0.n_e, 0, 1, --tpb, od_lds); }
    if (L.total > 160 * 1024) return -2;
    const void* fn = rt == 1 ? expo_fn<1>() : rt == 2 ? expo_fn<2>() : rt == 3 ? expo_fn<3>() : rt == 4 ? expo_fn<4>() : expo_fn<5>();
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total) != hipSuccess) return -3;
    int dev = 0, ncu = 0, nb = 1;
    const int threads = 64 * tpb;
    if (hipGetDevice(&dev) != hipSuccess) return -3;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -3;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, L.total) != hipSuccess || nb < 1) nb = 1;
    const int cols = 16 * tpb;
    long long need = (s0.count + cols - 1) / cols;
    long long blocks = a.persistent ? (long long)ncu * nb : need;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    void* args[] = {(void*)&a, (void*)&od_lds, (void*)&tpb, (void*)&Pg, (void*)&J, (void*)&m, (void*)&h, (void*)&NS};
    if (hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(threads), args, L.total, st) != hipSuccess) return -3;
    if (info) { info->blocks = (int)blocks; info->threads = threads; info->lds = (int)L.total; info->cols = cols; info->shape = rt * 100 + 1; }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace qtm
