// qtm_capi.cpp -- host runtime and C ABI of libqtm (declared in include/qtm.h).
//
// qtm_create validates the problem, assembles the right-hand-side operator
// M = -i H - 1/2 sum_n C_n^dag C_n (= -i H_eff, the paper's effective
// Hamiltonian with hbar = 1) in FP64 on the host, lays it out for the chosen
// kernel (MFMA A-fragments for dense M, 64-row sliced ELL for sparse M) and
// uploads everything once.  qtm_run launches the trajectory kernel on the
// context's stream, then the index-ordered averaging kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qtm.h"
#include "qtm_internal.h"

using cd = std::complex<double>;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHECK(x)                                                                        \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return fail(QTM_E_DEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

// Host CSR with complex values.
struct HCsr {
    int d = 0;
    std::vector<int> rp, ci;
    std::vector<cd> v;
};

int validate_op(const qtm_op* o, int d, const char* what, int idx) {
    if (!o) return fail(QTM_E_INVAL, "%s[%d]: null operator", what, idx);
    if (o->dim != d) return fail(QTM_E_INVAL, "%s[%d]: dimension %d, expected %d", what, idx, o->dim, d);
    if (!o->val) return fail(QTM_E_INVAL, "%s[%d]: null values", what, idx);
    size_t n = 0;
    if (o->fmt == QTM_FMT_DENSE) n = (size_t)d * d;
    else if (o->fmt == QTM_FMT_DIAG) n = (size_t)d;
    else if (o->fmt == QTM_FMT_CSR) {
        if (!o->row_ptr || !o->col_ind) return fail(QTM_E_INVAL, "%s[%d]: CSR without row_ptr/col_ind", what, idx);
        if (o->row_ptr[0] != 0 || o->row_ptr[d] != o->nnz || o->nnz < 0)
            return fail(QTM_E_INVAL, "%s[%d]: CSR row_ptr[0] must be 0 and row_ptr[d] == nnz", what, idx);
        for (int i = 0; i < d; ++i)
            if (o->row_ptr[i + 1] < o->row_ptr[i]) return fail(QTM_E_INVAL, "%s[%d]: CSR row_ptr not non-decreasing", what, idx);
        for (int64_t p = 0; p < o->nnz; ++p)
            if (o->col_ind[p] < 0 || o->col_ind[p] >= d)
                return fail(QTM_E_INVAL, "%s[%d]: CSR column index %d out of range", what, idx, o->col_ind[p]);
        n = (size_t)o->nnz;
    } else {
        return fail(QTM_E_INVAL, "%s[%d]: unknown format %d", what, idx, o->fmt);
    }
    for (size_t i = 0; i < 2 * n; ++i)
        if (!std::isfinite(o->val[i])) return fail(QTM_E_INVAL, "%s[%d]: non-finite entry", what, idx);
    return QTM_OK;
}

HCsr to_csr(const qtm_op* o, bool drop_zeros) {
    HCsr c;
    int d = o->dim;
    c.d = d;
    c.rp.assign(d + 1, 0);
    if (o->fmt == QTM_FMT_CSR) {
        c.rp.assign(o->row_ptr, o->row_ptr + d + 1);
        c.ci.assign(o->col_ind, o->col_ind + o->nnz);
        for (int64_t p = 0; p < o->nnz; ++p) c.v.push_back(cd(o->val[2 * p], o->val[2 * p + 1]));
        return c;
    }
    for (int i = 0; i < d; ++i) {
        if (o->fmt == QTM_FMT_DIAG) {
            cd z(o->val[2 * i], o->val[2 * i + 1]);
            if (!drop_zeros || z != 0.0) { c.ci.push_back(i); c.v.push_back(z); }
        } else {
            for (int j = 0; j < d; ++j) {
                cd z(o->val[2 * ((size_t)i * d + j)], o->val[2 * ((size_t)i * d + j) + 1]);
                if (!drop_zeros || z != 0.0) { c.ci.push_back(j); c.v.push_back(z); }
            }
        }
        c.rp[i + 1] = (int)c.ci.size();
    }
    return c;
}

// M = -i H - 1/2 sum_n C_n^dag C_n as CSR (rows accumulated in a dense buffer).
HCsr build_M(const qtm_op* H, const qtm_op* c, int n_c) {
    const int d = H->dim;
    HCsr h = to_csr(H, false);
    std::vector<HCsr> C;
    for (int n = 0; n < n_c; ++n) C.push_back(to_csr(&c[n], true));
    // (C^dag C)_{pq} = sum_k conj(C_kp) C_kq: contributions per row p
    std::vector<std::vector<std::pair<int, cd>>> extra(d);
    for (const HCsr& m : C)
        for (int k = 0; k < d; ++k)
            for (int a = m.rp[k]; a < m.rp[k + 1]; ++a)
                for (int b = m.rp[k]; b < m.rp[k + 1]; ++b)
                    extra[m.ci[a]].push_back({m.ci[b], -0.5 * std::conj(m.v[a]) * m.v[b]});
    HCsr M;
    M.d = d;
    M.rp.assign(d + 1, 0);
    std::vector<cd> acc(d, 0.0);
    std::vector<char> used(d, 0);
    std::vector<int> cols;
    for (int i = 0; i < d; ++i) {
        cols.clear();
        for (int p = h.rp[i]; p < h.rp[i + 1]; ++p) {
            int j = h.ci[p];
            if (!used[j]) { used[j] = 1; cols.push_back(j); }
            acc[j] += cd(0.0, -1.0) * h.v[p];
        }
        for (auto& e : extra[i]) {
            if (!used[e.first]) { used[e.first] = 1; cols.push_back(e.first); }
            acc[e.first] += e.second;
        }
        std::sort(cols.begin(), cols.end());
        for (int j : cols) { M.ci.push_back(j); M.v.push_back(acc[j]); acc[j] = 0.0; used[j] = 0; }
        M.rp[i + 1] = (int)M.ci.size();
    }
    return M;
}

// MFMA A-fragments of the real-embedded operator (see the row maps in the kernels):
// frag[(rt*KB + kb)*64 + lane] = Mreal[16 rt + (lane & 15)][4 kb + (lane >> 4)].
int row_of(int q, int p, int prec) {
    if (prec == 0) return 16 * (q >> 3) + 4 * (2 * ((q & 7) >> 2) + p) + (q & 3);
    return 2 * q + p;
}

template <class T>
std::vector<T> build_frag(const HCsr& M, int dp, int prec) {
    const int n = 2 * dp, KB = n / 4, RT = n / 16;
    std::vector<double> real((size_t)n * n, 0.0);
    for (int i = 0; i < M.d; ++i)
        for (int p = M.rp[i]; p < M.rp[i + 1]; ++p) {
            int j = M.ci[p];
            double re = M.v[p].real(), im = M.v[p].imag();
            real[(size_t)row_of(i, 0, prec) * n + row_of(j, 0, prec)] += re;
            real[(size_t)row_of(i, 0, prec) * n + row_of(j, 1, prec)] += -im;
            real[(size_t)row_of(i, 1, prec) * n + row_of(j, 0, prec)] += im;
            real[(size_t)row_of(i, 1, prec) * n + row_of(j, 1, prec)] += re;
        }
    std::vector<T> f((size_t)n * n);
    for (int rt = 0; rt < RT; ++rt)
        for (int kb = 0; kb < KB; ++kb)
            for (int l = 0; l < 64; ++l)
                f[((size_t)rt * KB + kb) * 64 + l] = (T)real[(size_t)(16 * rt + (l & 15)) * n + 4 * kb + (l >> 4)];
    return f;
}

// Team-kernel fragments [RT][RT][64][4]: A-fragment of output tile rt and K-block
// (source tile s, slot i), whose K index at lane group g is the real-embedded row
// that lane group g holds in accumulator slot i of tile s (FP64: 16 s + g + 4 i,
// FP32: 16 s + 4 g + i), so the state feeds the matrix cores in place.
template <class T>
std::vector<T> build_frag_team(const HCsr& M, int dp, int prec) {
    const int n = 2 * dp, RT = n / 16;
    std::vector<double> real((size_t)n * n, 0.0);
    for (int i = 0; i < M.d; ++i)
        for (int p = M.rp[i]; p < M.rp[i + 1]; ++p) {
            int j = M.ci[p];
            double re = M.v[p].real(), im = M.v[p].imag();
            real[(size_t)row_of(i, 0, prec) * n + row_of(j, 0, prec)] += re;
            real[(size_t)row_of(i, 0, prec) * n + row_of(j, 1, prec)] += -im;
            real[(size_t)row_of(i, 1, prec) * n + row_of(j, 0, prec)] += im;
            real[(size_t)row_of(i, 1, prec) * n + row_of(j, 1, prec)] += re;
        }
    std::vector<T> f((size_t)n * n);
    for (int rt = 0; rt < RT; ++rt)
        for (int s = 0; s < RT; ++s)
            for (int l = 0; l < 64; ++l)
                for (int i = 0; i < 4; ++i) {
                    const int g = l >> 4;
                    const int col = prec == 0 ? 16 * s + g + 4 * i : 16 * s + 4 * g + i;
                    f[(((size_t)rt * RT + s) * 64 + l) * 4 + i] = (T)real[(size_t)(16 * rt + (l & 15)) * n + col];
                }
    return f;
}

// 1 when every tile (rt, s) of the team layout holding a nonzero lies within one tile
// of the diagonal (a banded operator: the kernel then skips the other tiles' products)
int team_tile_band(const std::vector<double>& f, int RT) {
    for (int rt = 0; rt < RT; ++rt)
        for (int s = 0; s < RT; ++s) {
            if (rt - s <= 1 && s - rt <= 1) continue;
            for (int k = 0; k < 256; ++k)
                if (f[((size_t)rt * RT + s) * 256 + k] != 0.0) return 0;
        }
    return 1;
}

struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
};

struct SysHost {
    int d = 0, n_c = 0, n_e = 0, n_t = 0, n_f = 0;
    double cost = 0.0;         // estimated work of one trajectory: d^2 ||M||_inf (t_end - t0)
    // exact-propagator integrator: fragments of exp(h 2^-j M), j = 0..expo_J (device)
    bool expo = false;
    const double* expo_P = nullptr;
    int expo_J = 0, expo_m = 1;
    double expo_h = 0.0;
    long long expo_NS = 0;
    bool sparse = false;       // sliced-ELL kernel (CSR H, or dense H with d > 128)
    bool team = false;         // team kernel (dense, d <= 64); otherwise the block dense kernel
    qtm::DevSystem dev{};
    std::vector<double> tlist;
    std::vector<double> cdiag;         // [n_c][d] diagonal of C_n^dag C_n (valid when dev.c_isdiag)
    std::vector<DevBuf> bufs;          // device allocations owned by the system
    // run outputs
    DevBuf X, tstat, jt, jc, jn, segs, queue, sum, sumsq, avg_part;
    long long cap_count = 0;
    std::vector<double> h_sum, h_sumsq;
    long long sum_count = 0;
};

}  // namespace

struct qtm_ctx {
    qtm_opts o{};
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<SysHost> sys;
    qtm::DevSystem* d_sys = nullptr;   // device copy of the DevSystem array
    long long* d_fail = nullptr;
    unsigned long long* d_counters = nullptr;
    unsigned int* d_cursor = nullptr;
    int* d_cls_off = nullptr;                // [3][9] offsets of the per-XCD system lists of each tile class
    unsigned int* d_cls_cur = nullptr;       // [3][8] cursors of those lists
    float* d_mlp = nullptr;            // BF16-rounded weights for inference
    unsigned short* d_mlpf = nullptr;  // the same weights as BF16 matrix-core fragments
    std::vector<float> mlp_master;     // FP32 master weights
    bool have_mlp = false;
    bool ran = false;
    qtm_stats_t st{};
    long long last_begin = 0, last_count = 0;
    int ncu = 0;
    bool batch = false;                // created by qtm_create_batch
    // per-system launches of a batch fan out over these streams (default priority)
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_ev;
    hipEvent_t fork = nullptr;
    // the batched form's captured run (valid for graph_count trajectories)
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    long long graph_count = -1;
    qtm::LaunchInfo graph_li{};
    unsigned long long* d_stamp = nullptr;   // [2] wall-clock stamps around the trajectory kernels
    // batches of dense systems (d <= 256): systems ordered by tile class, one launch per class
    bool tile_classes = false;
    qtm::DevSystem* d_sys_cls = nullptr;
    std::vector<int> cls_sys;                // system index of each entry of d_sys_cls
    int cls_off[3] = {0, 0, 0}, cls_n[3] = {0, 0, 0}, cls_maxd[3] = {0, 0, 0}, cls_maxne[3] = {0, 0, 0};
    int cls_xoff[3][9] = {};                 // per-XCD list offsets inside each class (host copy)
    int wall_khz = 100000;                   // rate of the device wall clock
    // pinned host staging of a run's read-back (stamps, failure, counters, per-trajectory
    // statistics, sums): every copy is queued on the run's stream, then one synchronization
    void* pin = nullptr;
    size_t pin_bytes = 0;
};

namespace {

int dalloc(SysHost& s, void** p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return fail(QTM_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    s.bufs.push_back({*p, bytes});
    return QTM_OK;
}

template <class T>
int upload(SysHost& s, const T** out, const std::vector<T>& v) {
    void* p = nullptr;
    int rc = dalloc(s, &p, v.size() * sizeof(T));
    if (rc) return rc;
    if (!v.empty()) HIPCHECK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    *out = (const T*)p;
    return QTM_OK;
}

void free_buf(DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.n = 0;
}

int ensure_buf(DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.n >= bytes) return QTM_OK;
    free_buf(b);
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) { b.p = nullptr; return fail(QTM_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e)); }
    b.n = bytes;
    return QTM_OK;
}

// exp(A) of a dense complex d x d matrix (row-major) by scaling and squaring: A / 2^s has
// infinity norm at most 1/4, where the degree-18 Taylor polynomial leaves a truncation
// error below (1/4)^19 / 19! (about 2e-29 relative), then s squarings.
std::vector<cd> expm_dense(const std::vector<cd>& A, int d) {
    double nrm = 0.0;
    for (int i = 0; i < d; ++i) {
        double rs = 0.0;
        for (int j = 0; j < d; ++j) rs += std::abs(A[(size_t)i * d + j]);
        nrm = std::max(nrm, rs);
    }
    int sq = 0;
    while (nrm > 0.25 && sq < 1000) { nrm *= 0.5; ++sq; }
    const double sc = std::ldexp(1.0, -sq);
    std::vector<cd> B(A.size()), E((size_t)d * d, 0.0), term((size_t)d * d, 0.0), tmp((size_t)d * d);
    for (size_t i = 0; i < A.size(); ++i) B[i] = A[i] * sc;
    for (int i = 0; i < d; ++i) { E[(size_t)i * d + i] = 1.0; term[(size_t)i * d + i] = 1.0; }
    auto mul = [&](const std::vector<cd>& X, const std::vector<cd>& Y, std::vector<cd>& Z) {
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                cd acc = 0.0;
                for (int l = 0; l < d; ++l) acc += X[(size_t)i * d + l] * Y[(size_t)l * d + j];
                Z[(size_t)i * d + j] = acc;
            }
    };
    for (int kx = 1; kx <= 18; ++kx) {
        mul(term, B, tmp);
        for (size_t i = 0; i < tmp.size(); ++i) term[i] = tmp[i] / (double)kx;
        for (size_t i = 0; i < E.size(); ++i) E[i] += term[i];
    }
    for (int q = 0; q < sq; ++q) {
        mul(E, E, tmp);
        E.swap(tmp);
    }
    return E;
}

// Time-dependent terms of one system (qtm_create_td).
struct TdSpec {
    const qtm_op* H = nullptr;
    const qtm_drive* f = nullptr;
    int n = 0;
};

int setup_system(SysHost& S, const qtm_system& in, int idx, const qtm_opts& o, bool want_ell,
                 const TdSpec* td = nullptr) {
    const qtm_op* H = in.H;
    if (!H) return fail(QTM_E_INVAL, "system %d: null H", idx);
    const int d = H->dim;
    if (d < 1) return fail(QTM_E_INVAL, "system %d: dimension %d < 1", idx, d);
    int rc = validate_op(H, d, "H", 0);
    if (rc) return rc;
    if (in.n_c < 0 || in.n_c > qtm::kMaxC) return fail(QTM_E_INVAL, "system %d: n_c = %d outside [0, %d]", idx, in.n_c, qtm::kMaxC);
    if (in.n_c > 0 && !in.c_ops) return fail(QTM_E_INVAL, "system %d: null c_ops", idx);
    for (int n = 0; n < in.n_c; ++n) if ((rc = validate_op(&in.c_ops[n], d, "c_ops", n))) return rc;
    if (in.n_e < 1 || in.n_e > qtm::kMaxE) return fail(QTM_E_INVAL, "system %d: n_e = %d outside [1, %d]", idx, in.n_e, qtm::kMaxE);
    if (!in.e_ops) return fail(QTM_E_INVAL, "system %d: null e_ops", idx);
    for (int n = 0; n < in.n_e; ++n) if ((rc = validate_op(&in.e_ops[n], d, "e_ops", n))) return rc;
    if (!in.psi0) return fail(QTM_E_INVAL, "system %d: null psi0", idx);
    double nn = 0.0;
    for (int i = 0; i < 2 * d; ++i) {
        if (!std::isfinite(in.psi0[i])) return fail(QTM_E_INVAL, "system %d: non-finite psi0", idx);
        nn += in.psi0[i] * in.psi0[i];
    }
    if (std::fabs(std::sqrt(nn) - 1.0) > 1e-10) return fail(QTM_E_INVAL, "system %d: ||psi0|| = %.17g, not 1", idx, std::sqrt(nn));
    if (in.n_t < 2 || !in.tlist) return fail(QTM_E_INVAL, "system %d: need n_t >= 2 output times", idx);
    for (int k = 0; k < in.n_t; ++k) {
        if (!std::isfinite(in.tlist[k])) return fail(QTM_E_INVAL, "system %d: non-finite tlist", idx);
        if (k > 0 && !(in.tlist[k] > in.tlist[k - 1])) return fail(QTM_E_INVAL, "system %d: tlist not strictly increasing at %d", idx, k);
    }
    // kernel choice: CSR H -> sliced-ELL SpMM; dense H -> MFMA team kernel (d <= 64),
    // MFMA block kernel (d <= 128), or the SpMM kernel on full rows (d <= 2048)
    S.sparse = H->fmt == QTM_FMT_CSR || d > 128;
    S.team = !S.sparse && qtm::wave_supported(d);
    if (o.integrator == QTM_INT_EXPO && d <= 40) {
        S.sparse = false;                   // the exact-propagator kernel uses the team layout
        S.team = true;
    }
    const int n_td = td ? td->n : 0;
    if (n_td) {
        if (n_td < 0 || n_td > QTM_MAX_TD) return fail(QTM_E_INVAL, "n_td = %d outside [1, %d]", n_td, QTM_MAX_TD);
        if (!td->H || !td->f) return fail(QTM_E_INVAL, "null time-dependent terms");
        if (!qtm::wave_supported(d))
            return fail(QTM_E_INVAL, "time-dependent terms need d <= 64 (the small dense kernel); d = %d", d);
        for (int k = 0; k < n_td; ++k) {
            if ((rc = validate_op(&td->H[k], d, "H_td", k))) return rc;
            const qtm_drive& f = td->f[k];
            if (!std::isfinite(f.c) || !std::isfinite(f.a) || !std::isfinite(f.b) || !std::isfinite(f.omega))
                return fail(QTM_E_INVAL, "f_td[%d]: non-finite coefficient", k);
        }
        S.sparse = false;                   // every format goes to the small dense kernel
        S.team = true;
    }
    if (d > 2048) return fail(QTM_E_INVAL, "system %d: dimension %d above the supported 2048", idx, d);
    S.d = d; S.n_c = in.n_c; S.n_e = in.n_e; S.n_t = in.n_t;
    S.tlist.assign(in.tlist, in.tlist + in.n_t);
    qtm::DevSystem& D = S.dev;
    std::memset(&D, 0, sizeof(D));
    D.d = d; D.n_c = in.n_c; D.n_e = in.n_e; D.n_t = in.n_t; D.n_f = 0;
    D.t0 = in.tlist[0]; D.tend = in.tlist[in.n_t - 1];
    D.key1 = (unsigned long long)idx;
    HCsr M = build_M(H, in.c_ops, in.n_c);
    {
        double mn = 0.0;
        for (int i = 0; i < d; ++i) {
            double rs = 0.0;
            for (int p = M.rp[i]; p < M.rp[i + 1]; ++p) rs += std::abs(M.v[p]);
            mn = std::max(mn, rs);
        }
        S.cost = (double)d * d * std::max(mn, 1e-3) * (in.tlist[in.n_t - 1] - in.tlist[0]);
    }
    if (!S.sparse) {
        int dp = (d + 7) / 8 * 8;
        D.dp = dp;
        D.rt = 2 * dp / 16;
        if (S.team) {
            const std::vector<double> f64 = build_frag_team<double>(M, dp, 0);
            D.tile_band = team_tile_band(f64, 2 * dp / 16);
            if ((rc = upload(S, &D.Mfrag, f64))) return rc;
            if ((rc = upload(S, &D.Mfrag32, build_frag_team<float>(M, dp, 1)))) return rc;
            D.Mteam = D.Mfrag;
            D.Mteam32 = D.Mfrag32;
            if (n_td) {
                // fragments of the right-hand-side matrices -i H_k, one after the other, and
                // the coefficients (c, a, b, omega) of f_k
                std::vector<double> t64;
                std::vector<float> t32;
                std::vector<double> coef;
                for (int k = 0; k < n_td; ++k) {
                    HCsr hk = to_csr(&td->H[k], true);
                    for (auto& z : hk.v) z *= cd(0.0, -1.0);
                    const std::vector<double> a = build_frag_team<double>(hk, dp, 0);
                    const std::vector<float> b = build_frag_team<float>(hk, dp, 1);
                    t64.insert(t64.end(), a.begin(), a.end());
                    t32.insert(t32.end(), b.begin(), b.end());
                    const qtm_drive& f = td->f[k];
                    coef.insert(coef.end(), {f.c, f.a, f.b, f.omega});
                }
                if ((rc = upload(S, &D.Mtd, t64))) return rc;
                if ((rc = upload(S, &D.Mtd32, t32))) return rc;
                if ((rc = upload(S, &D.td, coef))) return rc;
                D.n_td = n_td;
            }
        } else {
            if ((rc = upload(S, &D.Mfrag, build_frag<double>(M, dp, 0)))) return rc;
            if ((rc = upload(S, &D.Mfrag32, build_frag<float>(M, dp, 1)))) return rc;
            if (want_ell && d <= 256) {        // batches: the tile-class launch reads the team layout
                if ((rc = upload(S, &D.Mteam, build_frag_team<double>(M, dp, 0)))) return rc;
                if ((rc = upload(S, &D.Mteam32, build_frag_team<float>(M, dp, 1)))) return rc;
            }
        }
    } else {
        D.dp = d;
        if (want_ell && H->fmt != QTM_FMT_CSR && d <= 256) {
            // dense system of a batch above the block kernel's range: team layout for the
            // tile-class launch
            const int dp = (d + 7) / 8 * 8;
            D.dp = dp;
            D.rt = 2 * dp / 16;
            if ((rc = upload(S, &D.Mteam, build_frag_team<double>(M, dp, 0)))) return rc;
            if ((rc = upload(S, &D.Mteam32, build_frag_team<float>(M, dp, 1)))) return rc;
        }
    }
    if (o.integrator == QTM_INT_EXPO) {
        // exact propagator: uniform output grid, h = spacing / substeps, fragments of
        // exp(h 2^-j M) for j = 0..J with h 2^-J of about 1e-12
        if (n_td) return fail(QTM_E_INVAL, "the exact-propagator integrator needs a time-independent H");
        if (d > 40) return fail(QTM_E_INVAL, "the exact-propagator integrator supports d <= 40; d = %d", d);
        const double span = in.tlist[in.n_t - 1] - in.tlist[0], dt = span / (in.n_t - 1);
        for (int k = 0; k + 1 < in.n_t; ++k)
            if (std::fabs((in.tlist[k + 1] - in.tlist[k]) - dt) > 1e-9 * dt)
                return fail(QTM_E_INVAL, "the exact-propagator integrator needs uniformly spaced output times");
        const int m = std::max(1, (int)o.expo_substeps);
        const double h = dt / m;
        int J = (int)std::ceil(std::log2(h / 1e-12));
        J = std::min(52, std::max(8, J));
        const int dp = S.dev.dp, n = 2 * dp;
        std::vector<cd> Md((size_t)d * d, 0.0);
        for (int i = 0; i < d; ++i)
            for (int p = M.rp[i]; p < M.rp[i + 1]; ++p) Md[(size_t)i * d + M.ci[p]] += M.v[p];
        std::vector<double> frags;
        frags.reserve((size_t)(J + 1) * n * n);
        for (int j = 0; j <= J; ++j) {
            std::vector<cd> A(Md.size());
            const double tau = std::ldexp(h, -j);
            for (size_t i = 0; i < Md.size(); ++i) A[i] = tau * Md[i];
            const std::vector<cd> P = expm_dense(A, d);
            HCsr Pc;
            Pc.d = d;
            Pc.rp.assign(d + 1, 0);
            for (int i = 0; i < d; ++i) {
                for (int c = 0; c < d; ++c) { Pc.ci.push_back(c); Pc.v.push_back(P[(size_t)i * d + c]); }
                Pc.rp[i + 1] = (int)Pc.ci.size();
            }
            const std::vector<double> f = build_frag_team<double>(Pc, dp, 0);
            frags.insert(frags.end(), f.begin(), f.end());
        }
        if ((rc = upload(S, &S.expo_P, frags))) return rc;
        S.expo = true;
        S.expo_J = J;
        S.expo_m = m;
        S.expo_h = h;
        S.expo_NS = (long long)(in.n_t - 1) * m;
    }
    // sliced ELL: for the SpMM kernel, and for every system of a batch (the single
    // launch over all systems runs on it)
    if (S.sparse || want_ell) {
        int nsl = (d + 63) / 64;
        std::vector<int> off(nsl + 1, 0), wd(nsl, 0);
        for (int s = 0; s < nsl; ++s) {
            int w = 0;
            for (int i = 64 * s; i < std::min(d, 64 * s + 64); ++i) w = std::max(w, M.rp[i + 1] - M.rp[i]);
            // the kernel takes entries in groups of four, and may read the first group of
            // any slice (with zeroed values): every slice holds at least one group
            wd[s] = std::max(4, (w + 3) & ~3);
            off[s + 1] = off[s] + 64 * wd[s];
        }
        std::vector<int> col(off[nsl], 0);
        std::vector<double2> val(off[nsl], make_double2(0.0, 0.0));
        std::vector<float2> val32(off[nsl], make_float2(0.f, 0.f));
        for (int s = 0; s < nsl; ++s)
            for (int i = 64 * s; i < std::min(d, 64 * s + 64); ++i) {
                int ln = i - 64 * s;
                for (int p = M.rp[i], k = 0; p < M.rp[i + 1]; ++p, ++k) {
                    int idx2 = off[s] + k * 64 + ln;
                    col[idx2] = M.ci[p];
                    val[idx2] = make_double2(M.v[p].real(), M.v[p].imag());
                    val32[idx2] = make_float2((float)M.v[p].real(), (float)M.v[p].imag());
                }
                // padding entries: column of the row itself with value 0 (in range, harmless)
                for (int k = M.rp[i + 1] - M.rp[i]; k < wd[s]; ++k) col[off[s] + k * 64 + ln] = i;
            }
        // rows past d in the last slice point at row 0 with zero values
        D.ell_n = off[nsl];
        if ((rc = upload(S, &D.sl_off, off))) return rc;
        if ((rc = upload(S, &D.sl_w, wd))) return rc;
        if ((rc = upload(S, &D.sl_col, col))) return rc;
        if ((rc = upload(S, &D.sl_val, val))) return rc;
        if ((rc = upload(S, &D.sl_val32, val32))) return rc;
    }
    // collapse operators: CSR with absolute row pointers
    {
        std::vector<int> rp, ci;
        std::vector<double2> v;
        for (int n = 0; n < in.n_c; ++n) {
            HCsr c = to_csr(&in.c_ops[n], true);
            int base = (int)ci.size();
            for (int i = 0; i <= d; ++i) rp.push_back(base + c.rp[i]);
            for (size_t p = 0; p < c.ci.size(); ++p) { ci.push_back(c.ci[p]); v.push_back(make_double2(c.v[p].real(), c.v[p].imag())); }
        }
        if (rp.empty()) rp.push_back(0);
        // C_n^dag C_n is diagonal when no row of C_n has two entries; its diagonal is
        // sum_k |C_kp|^2 (rows 12 + n of the diagonal table)
        D.c_isdiag = 1;
        S.cdiag.assign((size_t)in.n_c * d, 0.0);
        for (int n = 0; n < in.n_c; ++n)
            for (int k = 0; k < d; ++k) {
                const int a = rp[(size_t)n * (d + 1) + k], b = rp[(size_t)n * (d + 1) + k + 1];
                if (b - a > 1) D.c_isdiag = 0;
                for (int q = a; q < b; ++q) S.cdiag[(size_t)n * d + ci[q]] += v[q].x * v[q].x + v[q].y * v[q].y;
            }
        if ((rc = upload(S, &D.c_rp, rp))) return rc;
        if ((rc = upload(S, &D.c_ci, ci))) return rc;
        if ((rc = upload(S, &D.c_val, v))) return rc;
    }
    // observables: diagonal ones keep their diagonal, others become CSR
    {
        std::vector<int> rp, ci;
        std::vector<double2> v;
        for (int e = 0; e < in.n_e; ++e) {
            const qtm_op* O = &in.e_ops[e];
            if (O->fmt == QTM_FMT_DIAG) {
                D.e_fmt[e] = 2;
                D.e_doff[e] = (int)v.size();
                bool real = true;
                for (int i = 0; i < d; ++i) {
                    v.push_back(make_double2(O->val[2 * i], O->val[2 * i + 1]));
                    if (O->val[2 * i + 1] != 0.0) real = false;
                }
                D.e_nv[e] = real ? 1 : 2;
                for (int i = 0; i <= d; ++i) rp.push_back(0);
            } else {
                D.e_fmt[e] = 1;
                D.e_nv[e] = 2;
                D.any_csr_e = 1;
                HCsr c = to_csr(O, true);
                int base = (int)v.size();
                // CSR values appended after any diagonal block; column indices parallel to values
                ci.resize(v.size(), 0);
                for (int i = 0; i <= d; ++i) rp.push_back(base + c.rp[i]);
                for (size_t p = 0; p < c.ci.size(); ++p) { v.push_back(make_double2(c.v[p].real(), c.v[p].imag())); ci.push_back(c.ci[p]); }
            }
        }
        ci.resize(v.size(), 0);
        if ((rc = upload(S, &D.e_rp, rp))) return rc;
        if ((rc = upload(S, &D.e_ci, ci))) return rc;
        if ((rc = upload(S, &D.e_val, v))) return rc;
    }
    {
        std::vector<double2> p0(d);
        for (int i = 0; i < d; ++i) p0[i] = make_double2(in.psi0[2 * i], in.psi0[2 * i + 1]);
        if ((rc = upload(S, &D.psi0, p0))) return rc;
        if ((rc = upload(S, &D.tlist, S.tlist))) return rc;
        std::vector<double> fd((size_t)(12 + in.n_c) * d, 0.0);
        std::copy(S.cdiag.begin(), S.cdiag.end(), fd.begin() + (size_t)12 * d);
        if ((rc = upload(S, &D.f_diag, fd))) return rc;
    }
    (void)o;
    return QTM_OK;
}

float bf16_round(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;          // round to nearest even
    u &= 0xFFFF0000u;
    float r;
    std::memcpy(&r, &u, 4);
    return r;
}

int check_ctx(const qtm_ctx* c) {
    if (!c) return fail(QTM_E_INVAL, "null context");
    return QTM_OK;
}


// Host-side standardisation and initial weights for training from scratch.
void init_proposal(std::vector<float>& P, const float* feat, const float* tgt, int64_t n, uint64_t seed) {
    P.assign(qtm::kNTotal, 0.f);
    const int NF = qtm::kNF, NH = qtm::kNH, NO = qtm::kNO;
    const int oW1 = 0, ob1 = NH * NF, oW2 = ob1 + NH, ob2 = oW2 + NH * NH, oW3 = ob2 + NH, ob3 = oW3 + NO * NH;
    const int omu = ob3 + NO, osd = omu + NF;
    for (int i = 0; i < NF; ++i) {
        double s = 0.0, s2 = 0.0;
        for (int64_t q = 0; q < n; ++q) { double x = feat[q * NF + i]; s += x; s2 += x * x; }
        double mu = s / (double)n, var = s2 / (double)n - mu * mu;
        P[omu + i] = (float)mu;
        P[osd + i] = (float)std::max(1e-3, std::sqrt(std::max(0.0, var)));
    }
    // splitmix64 stream for the initial weights (uniform, fan-in scaled)
    uint64_t x = seed ^ 0x5DEECE66DULL;
    auto uni = [&]() {
        x += 0x9E3779B97F4A7C15ULL;
        uint64_t z = x;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        z ^= z >> 31;
        return ((double)(z >> 11) + 0.5) * 0x1.0p-53;
    };
    auto fill = [&](int off, int cnt, int fan_in) {
        double a = std::sqrt(3.0 / fan_in);
        for (int i = 0; i < cnt; ++i) P[off + i] = (float)((2.0 * uni() - 1.0) * a);
    };
    fill(oW1, NH * NF, NF);
    fill(oW2, NH * NH, NH);
    fill(oW3, NO * NH, NH);
    // output biases start at the target means
    double m0 = 0.0, m1 = 0.0;
    int64_t n1 = 0;
    for (int64_t q = 0; q < n; ++q) {
        m0 += tgt[q * 3];
        if (tgt[q * 3 + 2] == 0.f) { m1 += tgt[q * 3 + 1]; ++n1; }
    }
    P[ob3 + 0] = (float)(m0 / (double)n);
    P[ob3 + 1] = P[ob3 + 2] = (float)(n1 ? m1 / (double)n1 : 0.0);
}

void working_copy(const std::vector<float>& master, std::vector<float>& q) {
    q = master;
    const int nW1 = qtm::kNH * qtm::kNF, nW2 = qtm::kNH * qtm::kNH, nW3 = qtm::kNO * qtm::kNH;
    const int oW1 = 0, oW2 = nW1 + qtm::kNH, oW3 = oW2 + nW2 + qtm::kNH;
    for (int i = 0; i < nW1; ++i) q[oW1 + i] = bf16_round(q[oW1 + i]);
    for (int i = 0; i < nW2; ++i) q[oW2 + i] = bf16_round(q[oW2 + i]);
    for (int i = 0; i < nW3; ++i) q[oW3 + i] = bf16_round(q[oW3 + i]);
}

// Matrix-core fragments of the BF16 working copy (FP32 16x16x4 A-operands, 4 per
// lane and group, stored as BF16): groups 0..3 layer 1 (output tile rt, K-block
// kb = feature 4 g + kb at lane group g), 4..19 layer 2 (rt, source tile s: slot i
// = hidden unit 16 s + 4 g + i, the accumulator layout), 20..23 layer 3 (rows
// past the 3 outputs are zero).
std::vector<uint16_t> mlp_fragments(const std::vector<float>& q) {
    const int NF = qtm::kNF, NH = qtm::kNH, NO = qtm::kNO;
    const float* W1 = q.data();
    const float* W2 = W1 + NH * NF + NH;
    const float* W3 = W2 + NH * NH + NH;
    auto bits = [](float x) { uint32_t u; std::memcpy(&u, &x, 4); return (uint16_t)(u >> 16); };
    std::vector<uint16_t> f(qtm::kMlpFrag, 0);
    for (int l = 0; l < 64; ++l) {
        const int m = l & 15, g = l >> 4;
        for (int i = 0; i < 4; ++i) {
            for (int rt = 0; rt < 4; ++rt) {
                f[((size_t)rt * 64 + l) * 4 + i] = bits(W1[(16 * rt + m) * NF + 4 * g + i]);
                for (int s2 = 0; s2 < 4; ++s2)
                    f[((size_t)(4 + 4 * rt + s2) * 64 + l) * 4 + i] = bits(W2[(16 * rt + m) * NH + 16 * s2 + 4 * g + i]);
            }
            for (int s2 = 0; s2 < 4; ++s2)
                f[((size_t)(20 + s2) * 64 + l) * 4 + i] = m < NO ? bits(W3[m * NH + 16 * s2 + 4 * g + i]) : 0;
        }
    }
    return f;
}

struct DevScratch {
    std::vector<void*> ptrs;
    ~DevScratch() { for (void* p : ptrs) if (p) (void)hipFree(p); }
    template <class T> int get(T** p, size_t n) {
        if (hipMalloc((void**)p, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess) return -2;
        ptrs.push_back(*p);
        return 0;
    }
};

}  // namespace

// ------------------------------------------------------------------ no-allocation runs
// Per-run device memory of qtm_run_range_noalloc: a fixed array in the library's code
// object (one copy per device, alive until the process ends), so that the call never
// allocates.  Host code must not pass the array's name to a kernel or copy: it stands
// for a host-side shadow, not the device address; the device address comes from
// hipGetSymbolAddress, taken once per device.
constexpr size_t kNoallocScratchBytes = (size_t)QTM_NOALLOC_SCRATCH_MB << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of this device's scratch array (the device must be current).
int scratch_address(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(QTM_E_DEVICE, "device ordinal %d above %d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(QTM_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = (unsigned char*)g_scratch_dev[dev];
    return QTM_OK;
}

// tot += part, element by element (part: one chunk's sums, added in chunk order)
__global__ void accumulate_kernel(double* tot, const double* part, int n, int first) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) tot[i] = first ? part[i] : tot[i] + part[i];
}

// out[j] += sum over q of st[q][j] (j < 4), integer sums (order-independent)
__global__ void tstat_sum_kernel(const int* st, long long count, unsigned long long* out) {
    unsigned long long s[4] = {0, 0, 0, 0};
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (long long)gridDim.x * blockDim.x)
        for (int j = 0; j < 4; ++j) s[j] += (unsigned long long)(unsigned int)st[4 * q + j];
    for (int j = 0; j < 4; ++j)
        if (s[j]) atomicAdd(&out[j], s[j]);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

void qtm_opts_default(qtm_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->rtol = 1e-6;
    o->atol = 1e-8;
    o->precision = QTM_PREC_FP64;
    o->form = 0;
    o->max_steps = 1000000;
    o->device = 0;
    o->record_jumps = 0;
    o->stream = nullptr;
}

const char* qtm_last_error(void) { return g_err.c_str(); }

int qtm_batch_tile_candidates(int32_t cls, int32_t* waves, int32_t cap) {
    if (!waves || cap < 1) return 0;
    int tmp[8];
    int n = std::min(qtm::team_batch_candidates(cls, tmp, 8), (int)cap);
    for (int i = 0; i < n; ++i) waves[i] = tmp[i];
    return n;
}

int qtm_tile_candidates(int32_t d, int32_t* waves, int32_t cap) {
    if (!waves || cap < 1) return 0;
    int tmp[8];
    int n = qtm::team_candidates(d, tmp, 8);
    n = std::min(n, (int)cap);
    for (int i = 0; i < n; ++i) waves[i] = tmp[i];
    return n;
}

static int create_common(qtm_ctx** out, int32_t n_sys, const qtm_system* sys, const qtm_opts* o, bool batch,
                         const TdSpec* td = nullptr) {
    if (!out) return fail(QTM_E_INVAL, "null output pointer");
    *out = nullptr;
    qtm_opts opt;
    if (o) opt = *o; else qtm_opts_default(&opt);
    if (!(opt.rtol > 0.0) || !(opt.atol >= 0.0) || !std::isfinite(opt.rtol) || !std::isfinite(opt.atol))
        return fail(QTM_E_INVAL, "rtol must be > 0 and atol >= 0");
    if (opt.precision != QTM_PREC_FP64 && opt.precision != QTM_PREC_FP32) return fail(QTM_E_INVAL, "unknown precision %d", opt.precision);
    if (opt.max_steps < 1) return fail(QTM_E_INVAL, "max_steps must be >= 1");
    if (opt.record_jumps < 0 || opt.seg_cap < 0) return fail(QTM_E_INVAL, "negative capacity");
    if (opt.team_waves < 0 || opt.tile_cols < 0) return fail(QTM_E_INVAL, "negative tile option");
    if (opt.chunk_traj < 0) return fail(QTM_E_INVAL, "negative chunk_traj");
    for (int k = 0; k < 3; ++k) {
        if (opt.class_waves[k] == 0 || opt.class_waves[k] == -1) continue;
        int w[8];
        const int n = qtm::team_batch_candidates(k, w, 8);
        bool ok = false;
        for (int i = 0; i < n; ++i) ok |= w[i] == opt.class_waves[k];
        if (!ok) return fail(QTM_E_INVAL, "class_waves[%d] = %d is not offered for that tile class", k, opt.class_waves[k]);
    }
    if (opt.integrator != QTM_INT_DOPRI5 && opt.integrator != QTM_INT_EXPO) return fail(QTM_E_INVAL, "unknown integrator %d", opt.integrator);
    if (opt.integrator == QTM_INT_EXPO) {
        if (opt.precision != QTM_PREC_FP64) return fail(QTM_E_INVAL, "the exact-propagator integrator uses FP64 products");
        if ((opt.form & QTM_FORM_LEARNED) || opt.seg_cap > 0)
            return fail(QTM_E_INVAL, "the exact-propagator integrator has no step proposal");
        if (batch) return fail(QTM_E_INVAL, "the exact-propagator integrator takes one system (qtm_create)");
        if (opt.expo_substeps < 0) return fail(QTM_E_INVAL, "negative expo_substeps");
    }
    int ndev = 0;
    hipError_t de = hipGetDeviceCount(&ndev);
    if (de != hipSuccess || ndev < 1) return fail(QTM_E_DEVICE, "no HIP device (%s, count %d)", hipGetErrorString(de), ndev);
    if (opt.device < 0 || opt.device >= ndev) return fail(QTM_E_INVAL, "device %d not present", opt.device);
    HIPCHECK(hipSetDevice(opt.device));
    hipDeviceProp_t prop;
    HIPCHECK(hipGetDeviceProperties(&prop, opt.device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(QTM_E_DEVICE, "device %d is %s; this library is built for gfx950", opt.device, prop.gcnArchName);
    qtm_ctx* c = new qtm_ctx();
    c->o = opt;
    c->device = opt.device;
    c->stream = (hipStream_t)opt.stream;
    c->ncu = prop.multiProcessorCount;
    c->batch = batch;
    {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, opt.device) == hipSuccess && khz > 0) c->wall_khz = khz;
    }
    c->sys.resize(n_sys);
    for (int s = 0; s < n_sys; ++s) {
        int rc = setup_system(c->sys[s], sys[s], s, opt, batch, td);
        if (rc) { qtm_destroy(c); return rc; }
    }
    if (batch && n_sys > 1) {
        bool all = true;
        for (int s = 0; s < n_sys; ++s)
            if (sys[s].H->fmt == QTM_FMT_CSR || c->sys[s].d > 256) all = false;
        if (all) {
            c->tile_classes = true;
            for (int k = 0; k < 3; ++k) {
                c->cls_off[k] = (int)c->cls_sys.size();
                for (int s = 0; s < n_sys; ++s)
                    if (qtm::team_batch_class(c->sys[s].d) == k) {
                        c->cls_sys.push_back(s);
                        c->cls_maxd[k] = std::max(c->cls_maxd[k], c->sys[s].d);
                        c->cls_maxne[k] = std::max(c->cls_maxne[k], c->sys[s].n_e);
                    }
                c->cls_n[k] = (int)c->cls_sys.size() - c->cls_off[k];
                // eight lists, one per XCD, balanced by estimated cost (largest first to the
                // list with the least cost so far); each list most expensive first
                std::vector<int> cl(c->cls_sys.begin() + c->cls_off[k], c->cls_sys.end());
                std::stable_sort(cl.begin(), cl.end(), [&](int x, int y) { return c->sys[x].cost > c->sys[y].cost; });
                std::vector<std::vector<int>> bins(8);
                double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                for (int s2 : cl) {
                    int b = (int)(std::min_element(load, load + 8) - load);
                    bins[b].push_back(s2);
                    load[b] += c->sys[s2].cost;
                }
                c->cls_sys.resize(c->cls_off[k]);
                c->cls_xoff[k][0] = 0;
                for (int b = 0; b < 8; ++b) {
                    c->cls_sys.insert(c->cls_sys.end(), bins[b].begin(), bins[b].end());
                    c->cls_xoff[k][b + 1] = c->cls_xoff[k][b] + (int)bins[b].size();
                }
            }
            if (hipMalloc(&c->d_sys_cls, sizeof(qtm::DevSystem) * n_sys) != hipSuccess ||
                hipMalloc(&c->d_cls_off, sizeof(int) * 27) != hipSuccess ||
                hipMalloc(&c->d_cls_cur, sizeof(unsigned int) * 24) != hipSuccess) {
                qtm_destroy(c);
                return fail(QTM_E_NOMEM, "device allocation failed");
            }
            if (hipMemcpy(c->d_cls_off, c->cls_xoff, sizeof(int) * 27, hipMemcpyHostToDevice) != hipSuccess) {
                qtm_destroy(c);
                return fail(QTM_E_DEVICE, "upload of the tile-class lists failed");
            }
        }
    }
    if (hipMalloc(&c->d_sys, sizeof(qtm::DevSystem) * n_sys) != hipSuccess ||
        hipMalloc(&c->d_fail, sizeof(long long)) != hipSuccess ||
        hipMalloc(&c->d_counters, 4 * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&c->d_cursor, 4 * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&c->d_stamp, 2 * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&c->d_mlp, sizeof(float) * qtm::kNTotal) != hipSuccess ||
        hipMalloc(&c->d_mlpf, sizeof(unsigned short) * qtm::kMlpFrag) != hipSuccess) {
        qtm_destroy(c);
        return fail(QTM_E_NOMEM, "device allocation failed");
    }
    *out = c;
    return QTM_OK;
}

int qtm_create(qtm_ctx** out, const qtm_op* H, const qtm_op* c_ops, int32_t n_c, const double* psi0,
               const double* tlist, int32_t n_t, const qtm_op* e_ops, int32_t n_e, const qtm_opts* o) {
    qtm_system s{H, c_ops, n_c, psi0, tlist, n_t, e_ops, n_e};
    return create_common(out, 1, &s, o, false);
}

int qtm_create_td(qtm_ctx** out, const qtm_op* H0, const qtm_op* H_td, const qtm_drive* f_td, int32_t n_td,
                  const qtm_op* c_ops, int32_t n_c, const double* psi0, const double* tlist, int32_t n_t,
                  const qtm_op* e_ops, int32_t n_e, const qtm_opts* o) {
    if (n_td < 1 || n_td > QTM_MAX_TD) return fail(QTM_E_INVAL, "n_td = %d outside [1, %d]", n_td, QTM_MAX_TD);
    qtm_system s{H0, c_ops, n_c, psi0, tlist, n_t, e_ops, n_e};
    TdSpec td;
    td.H = H_td; td.f = f_td; td.n = n_td;
    return create_common(out, 1, &s, o, false, &td);
}

int qtm_create_batch(qtm_ctx** out, int32_t n_sys, const qtm_system* sys, const qtm_opts* o) {
    if (n_sys < 1 || !sys) return fail(QTM_E_INVAL, "need n_sys >= 1 systems");
    return create_common(out, n_sys, sys, o, true);
}

int qtm_run(qtm_ctx* ctx, int64_t ntraj, uint64_t seed) { return qtm_run_range(ctx, 0, ntraj, seed); }

// Everything one run puts on the device after the system table is uploaded:
// clearing the outputs and counters (fill kernels, so that the sequence can be
// captured into a graph), the trajectory kernel(s) between two device timestamps, and the
// fixed-order averages.
// The outputs are the ones the host copies of the system descriptors name (X, counters,
// segment records, queue); avg, when given, replaces system 0's averaging buffers
// (partial sums, sums, sums of squares).
static int enqueue_run(qtm_ctx* c, const qtm::RunArgs& a, long long count, hipStream_t st, qtm::LaunchInfo* li,
                       double* const* avg = nullptr) {
    const int segc = a.seg_cap;
    // the clearing of outputs and counters, up to qtm::kFillSet buffers per fill launch
    qtm::FillSet fs{};
    auto flush = [&]() {
        const int r = fs.count ? qtm::launch_fills(fs, st) : 0;
        fs.count = 0;
        return r ? fail(QTM_E_DEVICE, "fill kernel launch failed") : QTM_OK;
    };
    auto fill = [&](void* p, size_t bytes, unsigned long long v) {
        if (bytes % 8 != 0) return fail(QTM_E_DEVICE, "fill of %zu bytes", bytes);
        if (bytes == 0) return QTM_OK;
        if (fs.count == qtm::kFillSet) { const int r = flush(); if (r) return r; }
        fs.p[fs.count] = (unsigned long long*)p;
        fs.n[fs.count] = (long long)(bytes / 8);
        fs.v[fs.count] = v;
        ++fs.count;
        return QTM_OK;
    };
    int rc;
    for (auto& S : c->sys) {
        size_t m = (size_t)S.n_e * S.n_t;
        if ((rc = fill(S.dev.queue, sizeof(unsigned long long), 0))) return rc;
        if ((rc = fill(S.dev.X, sizeof(double2) * m * count, 0))) return rc;
        if ((rc = fill(S.dev.tstat, sizeof(int) * 4 * count, 0))) return rc;
        if (segc && (rc = fill(S.dev.segs, sizeof(float) * qtm::kSegRec * segc * count, 0))) return rc;
    }
    if ((rc = fill(c->d_fail, sizeof(long long), (unsigned long long)LLONG_MAX))) return rc;
    if ((rc = fill(c->d_counters, 4 * sizeof(unsigned long long), 0))) return rc;
    if ((rc = fill(c->d_cursor, 4 * sizeof(unsigned long long), 0))) return rc;
    if (c->d_cls_cur && (rc = fill(c->d_cls_cur, 24 * sizeof(unsigned int), 0))) return rc;
    if ((rc = flush())) return rc;

    if (qtm::launch_stamp(c->d_stamp, st)) return fail(QTM_E_DEVICE, "timestamp kernel launch failed");
    const bool one_launch = c->batch && c->sys.size() > 1 && (c->o.form & QTM_FORM_BATCHED);
    auto ensure_side = [&](size_t want) -> int {
        if (c->side.size() >= want) return QTM_OK;
        const size_t old_n = c->side.size();
        c->side.resize(want, nullptr);
        c->side_ev.resize(want, nullptr);
        for (size_t i = old_n; i < want; ++i) {
            HIPCHECK(hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking));
            HIPCHECK(hipEventCreateWithFlags(&c->side_ev[i], hipEventDisableTiming));
        }
        if (!c->fork) HIPCHECK(hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
        return QTM_OK;
    };
    if (one_launch && c->tile_classes && !(c->o.form & QTM_FORM_LEARNED) && c->o.seg_cap == 0) {
        // one persistent launch per tile class (team kernel, operator in L2; d <= 64, 128,
        // 256), the classes side by side
        if ((rc = ensure_side(3))) return rc;
        HIPCHECK(hipEventRecord(c->fork, st));
        for (int k = 0; k < 3; ++k) HIPCHECK(hipStreamWaitEvent(c->side[k], c->fork, 0));
        bool first = true;
        for (int k = 0; k < 3; ++k) {
            if (!c->cls_n[k]) continue;
            qtm::RunArgs ak = a;
            ak.sys = c->d_sys_cls + c->cls_off[k];
            ak.n_sys = c->cls_n[k];
            ak.sys_cursor = c->d_cls_cur + 8 * k;
            ak.xcd_off = c->d_cls_off + 9 * k;
            qtm::LaunchInfo lx{};
            int lr;
            if (c->o.class_waves[k] < 0) {
                // the class on the SpMM kernel (every system of a batch has its sliced ELL)
                long long max_ell = 0;
                for (int q = 0; q < c->cls_n[k]; ++q)
                    max_ell = std::max(max_ell, c->sys[c->cls_sys[c->cls_off[k] + q]].dev.ell_n);
                ak.xcd_off = nullptr;
                const int cols = c->o.tile_cols > 0 ? c->o.tile_cols : (c->o.precision == QTM_PREC_FP32 ? 4 : 2);
                lr = qtm::launch_sparse(ak, c->sys[c->cls_sys[c->cls_off[k]]].dev, c->cls_maxd[k], max_ell, c->o.precision,
                                        cols, c->side[k], &lx);
            } else {
                lr = qtm::launch_team_batch(ak, c->cls_maxd[k], c->cls_maxne[k], c->o.precision, c->o.class_waves[k],
                                            c->side[k], &lx);
            }
            if (lr) return fail(QTM_E_DEVICE, "tile-class launch %d failed (%d): %s", k, lr, hipGetErrorString(hipGetLastError()));
            if (first) { *li = lx; first = false; }
        }
        for (int k = 0; k < 3; ++k) {
            HIPCHECK(hipEventRecord(c->side_ev[k], c->side[k]));
            HIPCHECK(hipStreamWaitEvent(st, c->side_ev[k], 0));
        }
    } else if (one_launch) {
        // every system in one persistent launch of the SpMM kernel: blocks move from
        // system to system as the trajectory queues run dry
        int max_d = 0;
        long long max_ell = 0;
        for (auto& Sx : c->sys) { max_d = std::max(max_d, Sx.d); max_ell = std::max(max_ell, Sx.dev.ell_n); }
        const int cols = c->o.tile_cols > 0 ? c->o.tile_cols : (c->o.precision == QTM_PREC_FP32 ? 4 : 2);
        int lr = qtm::launch_sparse(a, c->sys[0].dev, max_d, max_ell, c->o.precision, cols, st, li);
        if (lr) return fail(QTM_E_DEVICE, "batch launch failed (%d): %s", lr, hipGetErrorString(hipGetLastError()));
    } else {
        // one launch per system; a batch spreads them over side streams so that they overlap
        const bool fan = c->sys.size() > 1;
        if (fan && (rc = ensure_side(std::min<size_t>(8, c->sys.size())))) return rc;
        if (fan) {
            HIPCHECK(hipEventRecord(c->fork, st));
            for (auto ss : c->side) HIPCHECK(hipStreamWaitEvent(ss, c->fork, 0));
        }
        for (size_t si = 0; si < c->sys.size(); ++si) {
            const SysHost& Sx = c->sys[si];
            hipStream_t ss = fan ? c->side[si % c->side.size()] : st;
            qtm::RunArgs as = a;
            as.sys = c->d_sys + si;
            as.n_sys = 1;
            int lr;
            qtm::LaunchInfo lx{};
            if (Sx.expo) {
                lr = qtm::launch_expo(as, Sx.dev, Sx.expo_P, Sx.expo_J, Sx.expo_m, Sx.expo_h, Sx.expo_NS, ss, &lx);
            } else if (Sx.sparse) {
                int cols = c->o.tile_cols > 0 ? c->o.tile_cols : (c->o.precision == QTM_PREC_FP32 ? 4 : 2);
                lr = qtm::launch_sparse(as, Sx.dev, Sx.d, Sx.dev.ell_n, c->o.precision, cols, ss, &lx);
            } else if (Sx.team) {
                lr = qtm::launch_wave(as, Sx.dev, c->o.precision, c->o.team_waves, ss, &lx);
            } else {
                int bpc = 0, lds = 0;
                if (qtm::dense_occupancy(Sx.d, c->o.precision, c->o.tile_cols, &bpc, &lds)) bpc = 1;
                lr = qtm::launch_dense(as, Sx.dev, Sx.d, c->o.precision, bpc, ss, &lx);
            }
            if (Sx.team && lr == -1) return fail(QTM_E_INVAL, "system %zu: no team shape with %d waves for dimension %d", si, c->o.team_waves, Sx.d);
            if (Sx.team && lr == -2) return fail(QTM_E_INVAL, "system %zu: the team shape does not fit in LDS (dimension %d)", si, Sx.d);
            if (lr) return fail(QTM_E_DEVICE, "kernel launch failed for system %zu (%d): %s", si, lr, hipGetErrorString(hipGetLastError()));
            if (si == 0) *li = lx;
        }
        if (fan) {
            for (size_t i = 0; i < c->side.size(); ++i) {
                HIPCHECK(hipEventRecord(c->side_ev[i], c->side[i]));
                HIPCHECK(hipStreamWaitEvent(st, c->side_ev[i], 0));
            }
        }
    }
    if (qtm::launch_stamp(c->d_stamp + 1, st)) return fail(QTM_E_DEVICE, "timestamp kernel launch failed");
    for (size_t si = 0; si < c->sys.size(); ++si) {
        auto& S = c->sys[si];
        double* part = (avg && si == 0) ? avg[0] : (double*)S.avg_part.p;
        double* sum = (avg && si == 0) ? avg[1] : (double*)S.sum.p;
        double* sumsq = (avg && si == 0) ? avg[2] : (double*)S.sumsq.p;
        if (qtm::launch_average(S.dev, part, sum, sumsq, st)) return fail(QTM_E_DEVICE, "average kernel launch failed");
    }
    return QTM_OK;
}

// Launch arguments of one run of count trajectories.
static qtm::RunArgs run_args(const qtm_ctx* c, long long count, int jcap, int segc) {
    qtm::RunArgs a{};
    a.sys = c->d_sys;
    a.n_sys = (int)c->sys.size();
    a.sys_cursor = c->d_cursor;
    a.rtol = c->o.rtol;
    a.atol = c->o.atol;
    a.max_steps = c->o.max_steps;
    a.jcap = jcap;
    a.seg_cap = segc;
    a.learned = (c->o.form & QTM_FORM_LEARNED) ? 1 : 0;
    a.mlp = c->d_mlp;
    a.mlpf = c->d_mlpf;
    a.fail = c->d_fail;
    a.counters = c->d_counters;
    a.tile_cols = c->o.tile_cols;
    a.persistent = (c->o.form & QTM_FORM_BATCHED) ? 1 : 0;
    // failsafe bound on block cycles: every slot may run all its trajectories at max_steps
    long long per_slot = count;   // worst case (one slot)
    long long mc = (c->o.max_steps + 4) * 3;
    a.max_cycles = (per_slot > 0 && mc < LLONG_MAX / (per_slot + 1)) ? mc * (per_slot + 1) : LLONG_MAX;
    return a;
}

static int run_range_one(qtm_ctx* c, int64_t traj_begin, int64_t count, uint64_t seed);

// A run of more trajectories than one chunk holds: chunks of consecutive indices, each a
// complete run, their FP64 sums added on the host in chunk order and their statistics summed.
static int run_chunked(qtm_ctx* c, int64_t traj_begin, int64_t count, uint64_t seed, long long chunk) {
    auto t0 = std::chrono::steady_clock::now();
    std::vector<std::vector<double>> ts(c->sys.size()), tq(c->sys.size());
    qtm_stats_t acc{};
    for (long long done = 0; done < count; done += chunk) {
        const long long n = std::min<long long>(chunk, count - done);
        const int rc = run_range_one(c, traj_begin + done, n, seed);
        if (rc) return rc;
        const qtm_stats_t& s = c->st;
        acc.accepted += s.accepted; acc.rejected += s.rejected; acc.segments += s.segments; acc.jumps += s.jumps;
        acc.rhs_evals += s.rhs_evals; acc.passes += s.passes; acc.root_evals += s.root_evals;
        acc.kernel_ms += s.kernel_ms;
        acc.max_team_passes = std::max(acc.max_team_passes, s.max_team_passes);
        acc.blocks = s.blocks; acc.threads = s.threads; acc.tile_cols = s.tile_cols; acc.lds_bytes = s.lds_bytes;
        acc.team_shape = s.team_shape;
        for (size_t i = 0; i < c->sys.size(); ++i) {
            const SysHost& S = c->sys[i];
            if (done == 0) { ts[i] = S.h_sum; tq[i] = S.h_sumsq; continue; }
            for (size_t j = 0; j < ts[i].size(); ++j) ts[i][j] += S.h_sum[j];
            for (size_t j = 0; j < tq[i].size(); ++j) tq[i][j] += S.h_sumsq[j];
        }
    }
    for (size_t i = 0; i < c->sys.size(); ++i) {
        c->sys[i].h_sum = ts[i];
        c->sys[i].h_sumsq = tq[i];
        c->sys[i].sum_count = count;
    }
    acc.ntraj = count;
    acc.failed_traj = -1;
    acc.elapsed_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    c->st = acc;
    c->last_begin = traj_begin;
    c->last_count = count;
    return QTM_OK;
}

int qtm_run_range(qtm_ctx* c, int64_t traj_begin, int64_t count, uint64_t seed) {
    if (check_ctx(c)) return QTM_E_INVAL;
    if (count < 1 || traj_begin < 0) return fail(QTM_E_INVAL, "need count >= 1 and traj_begin >= 0");
    if ((c->o.form & QTM_FORM_LEARNED) && !c->have_mlp) return fail(QTM_E_STATE, "learned form requested before qtm_set_proposal");
    if (!c->o.keep_traj && c->o.record_jumps == 0 && c->o.seg_cap == 0) {
        // no per-trajectory data is kept: the samples of one chunk bound the device memory
        size_t per_traj = 0;
        for (auto& S : c->sys) per_traj += sizeof(double2) * (size_t)S.n_e * S.n_t;
        long long chunk = (long long)(((size_t)QTM_RUN_CHUNK_MB << 20) / std::max<size_t>(per_traj, 1));
        if (c->o.chunk_traj > 0) chunk = std::min<long long>(chunk, c->o.chunk_traj);
        chunk = std::max(chunk, 1LL);
        if (count > chunk) return run_chunked(c, traj_begin, count, seed, chunk);
    }
    return run_range_one(c, traj_begin, count, seed);
}

// One run of count trajectories (every per-trajectory buffer sized for count).
static int run_range_one(qtm_ctx* c, int64_t traj_begin, int64_t count, uint64_t seed) {
    HIPCHECK(hipSetDevice(c->device));
    auto t0 = std::chrono::steady_clock::now();
    c->ran = false;
    const int jcap = c->o.record_jumps, segc = c->o.seg_cap;
    bool realloc = false;
    for (auto& S : c->sys) {
        size_t m = (size_t)S.n_e * S.n_t;
        int rc;
        void* before[10] = {S.X.p, S.tstat.p, S.jn.p, S.jt.p, S.jc.p, S.segs.p, S.queue.p, S.sum.p, S.sumsq.p, S.avg_part.p};
        if ((rc = ensure_buf(S.X, sizeof(double2) * m * count))) return rc;
        if ((rc = ensure_buf(S.tstat, sizeof(int) * 4 * count))) return rc;
        if ((rc = ensure_buf(S.jn, sizeof(int) * count))) return rc;
        if ((rc = ensure_buf(S.jt, sizeof(double) * (size_t)std::max(1, jcap) * (jcap ? count : 1)))) return rc;
        if ((rc = ensure_buf(S.jc, sizeof(int) * (size_t)std::max(1, jcap) * (jcap ? count : 1)))) return rc;
        if ((rc = ensure_buf(S.segs, sizeof(float) * qtm::kSegRec * (size_t)std::max(1, segc) * (segc ? count : 1)))) return rc;
        if ((rc = ensure_buf(S.queue, sizeof(unsigned long long)))) return rc;
        if ((rc = ensure_buf(S.sum, sizeof(double) * 2 * m))) return rc;
        if ((rc = ensure_buf(S.sumsq, sizeof(double) * m))) return rc;
        if ((rc = ensure_buf(S.avg_part, sizeof(double) * qtm::average_part_size((int)m, count)))) return rc;
        void* after[10] = {S.X.p, S.tstat.p, S.jn.p, S.jt.p, S.jc.p, S.segs.p, S.queue.p, S.sum.p, S.sumsq.p, S.avg_part.p};
        for (int i = 0; i < 10; ++i) realloc |= before[i] != after[i];
        S.dev.X = (double2*)S.X.p;
        S.dev.tstat = (int*)S.tstat.p;
        S.dev.jt = (double*)S.jt.p;
        S.dev.jc = (int*)S.jc.p;
        S.dev.jn = (int*)S.jn.p;
        S.dev.segs = (float*)S.segs.p;
        S.dev.queue = (unsigned long long*)S.queue.p;
        S.dev.count = count;
        S.dev.traj_begin = traj_begin;
        S.dev.key0 = seed;
    }
    // the system table carries everything that changes from run to run (seed,
    // trajectory range, output buffers); a captured graph reads it from the device
    std::vector<qtm::DevSystem> ds;
    for (auto& S : c->sys) ds.push_back(S.dev);
    HIPCHECK(hipMemcpyAsync(c->d_sys, ds.data(), sizeof(qtm::DevSystem) * ds.size(), hipMemcpyHostToDevice, c->stream));
    std::vector<qtm::DevSystem> dsc;
    if (c->tile_classes) {
        for (int s2 : c->cls_sys) dsc.push_back(c->sys[s2].dev);
        HIPCHECK(hipMemcpyAsync(c->d_sys_cls, dsc.data(), sizeof(qtm::DevSystem) * dsc.size(), hipMemcpyHostToDevice, c->stream));
    }

    qtm::RunArgs a = run_args(c, count, jcap, segc);

    qtm::LaunchInfo li{};
    if (c->o.form & QTM_FORM_BATCHED) {
        // the batched form replays one captured graph per trajectory count
        if (realloc || c->graph_count != count) {
            if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
            if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
            c->graph_count = -1;
            if (!c->cap) HIPCHECK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
            HIPCHECK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
            int rc = enqueue_run(c, a, count, c->cap, &li);
            hipGraph_t g = nullptr;
            hipError_t ee = hipStreamEndCapture(c->cap, &g);
            if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
            if (ee != hipSuccess) return fail(QTM_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ee));
            c->graph = g;
            HIPCHECK(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
            c->graph_count = count;
            c->graph_li = li;
        }
        li = c->graph_li;
        HIPCHECK(hipGraphLaunch(c->gexec, c->stream));
    } else {
        int rc = enqueue_run(c, a, count, c->stream, &li);
        if (rc) return rc;
    }
    // read-back: every copy queued on the run's stream into pinned staging, one wait
    size_t rb = 64;                                   // stamps [2], failure, counters [4]
    for (auto& S : c->sys) rb += sizeof(int) * 4 * (size_t)count + sizeof(double) * 3 * (size_t)S.n_e * S.n_t;
    if (rb > c->pin_bytes) {
        if (c->pin) { (void)hipHostFree(c->pin); c->pin = nullptr; c->pin_bytes = 0; }
        HIPCHECK(hipHostMalloc(&c->pin, rb, hipHostMallocDefault));
        c->pin_bytes = rb;
    }
    char* hp = (char*)c->pin;
    HIPCHECK(hipMemcpyAsync(hp, c->d_stamp, 16, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(hipMemcpyAsync(hp + 16, c->d_fail, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(hipMemcpyAsync(hp + 32, c->d_counters, 32, hipMemcpyDeviceToHost, c->stream));
    {
        char* q = hp + 64;
        for (auto& S : c->sys) {
            const size_t m = (size_t)S.n_e * S.n_t;
            HIPCHECK(hipMemcpyAsync(q, S.tstat.p, sizeof(int) * 4 * count, hipMemcpyDeviceToHost, c->stream));
            q += sizeof(int) * 4 * count;
            HIPCHECK(hipMemcpyAsync(q, S.sum.p, sizeof(double) * 2 * m, hipMemcpyDeviceToHost, c->stream));
            q += sizeof(double) * 2 * m;
            HIPCHECK(hipMemcpyAsync(q, S.sumsq.p, sizeof(double) * m, hipMemcpyDeviceToHost, c->stream));
            q += sizeof(double) * m;
        }
    }
    HIPCHECK(hipStreamSynchronize(c->stream));
    // trajectory kernel(s) time from the two device timestamps around them
    unsigned long long stamps[2];
    std::memcpy(stamps, hp, 16);
    const double ms = (double)(stamps[1] - stamps[0]) / (double)c->wall_khz;
    long long failv = 0;
    unsigned long long ctrs[4];
    std::memcpy(&failv, hp + 16, 8);
    std::memcpy(ctrs, hp + 32, 32);
    // statistics
    qtm_stats_t st{};
    st.ntraj = count;
    {
        const char* q = hp + 64;
        for (auto& S : c->sys) {
            const int* ts = (const int*)q;
            for (long long i = 0; i < count; ++i) {
                st.accepted += ts[4 * i]; st.rejected += ts[4 * i + 1]; st.segments += ts[4 * i + 2]; st.jumps += ts[4 * i + 3];
            }
            q += sizeof(int) * 4 * count;
            const size_t m = (size_t)S.n_e * S.n_t;
            S.h_sum.resize(2 * m);
            S.h_sumsq.resize(m);
            std::memcpy(S.h_sum.data(), q, sizeof(double) * 2 * m);
            q += sizeof(double) * 2 * m;
            std::memcpy(S.h_sumsq.data(), q, sizeof(double) * m);
            q += sizeof(double) * m;
            S.sum_count = count;
        }
    }
    st.passes = (int64_t)ctrs[0];
    st.max_team_passes = (int64_t)ctrs[2];
    st.root_evals = (int64_t)ctrs[1];
    st.team_shape = li.shape;
    st.rhs_evals = (int64_t)ctrs[0] * li.cols;
    st.failed_traj = failv == LLONG_MAX ? -1 : failv;
    st.kernel_ms = ms;
    st.elapsed_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    st.blocks = li.blocks; st.threads = li.threads; st.tile_cols = li.cols; st.lds_bytes = li.lds;
    c->st = st;
    c->last_begin = traj_begin;
    c->last_count = count;
    if (failv != LLONG_MAX) return fail(QTM_E_STEP, "trajectory %lld failed (max_steps or step-size underflow)", failv);
    c->ran = true;
    return QTM_OK;
}

int qtm_sums(const qtm_ctx* c, int32_t s, double* sum, double* sumsq, int64_t* count) {
    if (check_ctx(c)) return QTM_E_INVAL;
    if (s < 0 || s >= (int)c->sys.size()) return fail(QTM_E_INVAL, "system index %d out of range", s);
    if (!c->ran) return fail(QTM_E_STATE, "no successful run");
    const SysHost& S = c->sys[s];
    if (sum) std::memcpy(sum, S.h_sum.data(), sizeof(double) * S.h_sum.size());
    if (sumsq) std::memcpy(sumsq, S.h_sumsq.data(), sizeof(double) * S.h_sumsq.size());
    if (count) *count = S.sum_count;
    return QTM_OK;
}

int qtm_expect_system(const qtm_ctx* c, int32_t s, double* mean, double* var) {
    if (check_ctx(c)) return QTM_E_INVAL;
    if (s < 0 || s >= (int)c->sys.size()) return fail(QTM_E_INVAL, "system index %d out of range", s);
    if (!c->ran) return fail(QTM_E_STATE, "qtm_expect before a successful qtm_run");
    if (!mean) return fail(QTM_E_INVAL, "null mean buffer");
    const SysHost& S = c->sys[s];
    size_t m = (size_t)S.n_e * S.n_t;
    double n = (double)S.sum_count;
    for (size_t i = 0; i < m; ++i) {
        double mr = S.h_sum[2 * i] / n, mi = S.h_sum[2 * i + 1] / n;
        mean[2 * i] = mr;
        mean[2 * i + 1] = mi;
        if (var) var[i] = std::max(0.0, S.h_sumsq[i] / n - mr * mr);
    }
    return QTM_OK;
}

int qtm_expect(const qtm_ctx* c, double* mean, double* var) { return qtm_expect_system(c, 0, mean, var); }

int qtm_traj_expect(const qtm_ctx* c, int32_t s, double* X) {
    if (check_ctx(c)) return QTM_E_INVAL;
    if (s < 0 || s >= (int)c->sys.size()) return fail(QTM_E_INVAL, "system index %d out of range", s);
    if (!c->ran) return fail(QTM_E_STATE, "no successful run");
    if (!c->o.keep_traj) return fail(QTM_E_STATE, "context created without keep_traj");
    const SysHost& S = c->sys[s];
    HIPCHECK(hipMemcpy(X, S.X.p, sizeof(double2) * (size_t)S.n_e * S.n_t * c->last_count, hipMemcpyDeviceToHost));
    return QTM_OK;
}

int qtm_jumps(const qtm_ctx* c, int32_t s, int64_t traj, int32_t cap, double* times, int32_t* channels, int32_t* count) {
    if (check_ctx(c)) return QTM_E_INVAL;
    if (s < 0 || s >= (int)c->sys.size()) return fail(QTM_E_INVAL, "system index %d out of range", s);
    if (c->o.record_jumps <= 0) return fail(QTM_E_STATE, "context created without record_jumps");
    if (!c->ran) return fail(QTM_E_STATE, "no successful run");
    if (traj < 0 || traj >= c->last_count) return fail(QTM_E_INVAL, "trajectory %lld outside the last run", (long long)traj);
    const SysHost& S = c->sys[s];
    int n = 0;
    HIPCHECK(hipMemcpy(&n, (int*)S.jn.p + traj, sizeof(int), hipMemcpyDeviceToHost));
    if (count) *count = n;
    int m = std::min(std::min(n, cap), c->o.record_jumps);
    if (m > 0 && times) HIPCHECK(hipMemcpy(times, (double*)S.jt.p + (size_t)traj * c->o.record_jumps, sizeof(double) * m, hipMemcpyDeviceToHost));
    if (m > 0 && channels) HIPCHECK(hipMemcpy(channels, (int*)S.jc.p + (size_t)traj * c->o.record_jumps, sizeof(int) * m, hipMemcpyDeviceToHost));
    return QTM_OK;
}

int qtm_traj_stats(const qtm_ctx* c, int32_t s, int32_t* stats) {
    if (check_ctx(c)) return QTM_E_INVAL;
    if (s < 0 || s >= (int)c->sys.size()) return fail(QTM_E_INVAL, "system index %d out of range", s);
    if (c->last_count == 0) return fail(QTM_E_STATE, "no run");
    HIPCHECK(hipMemcpy(stats, c->sys[s].tstat.p, sizeof(int) * 4 * c->last_count, hipMemcpyDeviceToHost));
    return QTM_OK;
}

int qtm_stats(const qtm_ctx* c, qtm_stats_t* st) {
    if (check_ctx(c)) return QTM_E_INVAL;
    if (!st) return fail(QTM_E_INVAL, "null stats");
    *st = c->st;
    return QTM_OK;
}

int qtm_segments(const qtm_ctx* c, float* out) {
    if (check_ctx(c)) return QTM_E_INVAL;
    if (c->o.seg_cap <= 0) return fail(QTM_E_STATE, "context created without seg_cap");
    if (c->last_count == 0) return fail(QTM_E_STATE, "no run");
    HIPCHECK(hipMemcpy(out, c->sys[0].segs.p, sizeof(float) * qtm::kSegRec * c->o.seg_cap * c->last_count, hipMemcpyDeviceToHost));
    return QTM_OK;
}

int qtm_set_proposal(qtm_ctx* c, const float* params, int32_t n_params, const qtm_op* f_ops, int32_t n_f) {
    if (check_ctx(c)) return QTM_E_INVAL;
    if (!params || n_params != qtm::kNTotal) return fail(QTM_E_INVAL, "expected %d parameters", qtm::kNTotal);
    if (n_f < 0 || n_f > 12) return fail(QTM_E_INVAL, "n_f must be in [0, 12]");
    for (int i = 0; i < n_params; ++i) if (!std::isfinite(params[i])) return fail(QTM_E_INVAL, "non-finite parameter");
    for (int i = qtm::kNParam + qtm::kNF; i < qtm::kNTotal; ++i)
        if (!(params[i] > 0.f)) return fail(QTM_E_INVAL, "input scales must be positive");
    HIPCHECK(hipSetDevice(c->device));
    c->mlp_master.assign(params, params + n_params);
    // weights (not biases, not the standardisation) rounded to BF16 for inference
    std::vector<float> q;
    working_copy(c->mlp_master, q);
    HIPCHECK(hipMemcpy(c->d_mlp, q.data(), sizeof(float) * qtm::kNTotal, hipMemcpyHostToDevice));
    {
        std::vector<uint16_t> fr = mlp_fragments(q);
        HIPCHECK(hipMemcpy(c->d_mlpf, fr.data(), sizeof(uint16_t) * fr.size(), hipMemcpyHostToDevice));
    }
    for (auto& S : c->sys) {
        const int d = S.d;
        std::vector<double> fd((size_t)(12 + S.n_c) * d, 0.0);
        std::copy(S.cdiag.begin(), S.cdiag.end(), fd.begin() + (size_t)12 * d);
        for (int f = 0; f < n_f; ++f) {
            if (f_ops[f].fmt != QTM_FMT_DIAG || f_ops[f].dim != d || !f_ops[f].val)
                return fail(QTM_E_INVAL, "feature operator %d must be diagonal of dimension %d", f, d);
            for (int i = 0; i < d; ++i) fd[(size_t)f * d + i] = f_ops[f].val[2 * i];
        }
        HIPCHECK(hipMemcpy((void*)S.dev.f_diag, fd.data(), sizeof(double) * fd.size(), hipMemcpyHostToDevice));
        S.dev.n_f = n_f;
    }
    c->have_mlp = true;
    return QTM_OK;
}

int qtm_get_proposal(const qtm_ctx* c, float* params, int32_t n_params) {
    if (check_ctx(c)) return QTM_E_INVAL;
    if (!c->have_mlp) return fail(QTM_E_STATE, "no proposal installed");
    if (!params || n_params != qtm::kNTotal) return fail(QTM_E_INVAL, "expected %d parameters", qtm::kNTotal);
    std::memcpy(params, c->mlp_master.data(), sizeof(float) * qtm::kNTotal);
    return QTM_OK;
}

int qtm_proposal_grad(qtm_ctx* c, const float* feat, const float* tgt, int64_t n, float* loss, float* grad) {
    if (check_ctx(c)) return QTM_E_INVAL;
    if (!c->have_mlp) return fail(QTM_E_STATE, "no proposal installed");
    if (!feat || !tgt || n < 1 || n > (1 << 24) || !grad) return fail(QTM_E_INVAL, "bad batch");
    HIPCHECK(hipSetDevice(c->device));
    DevScratch sc;
    float *dF, *dT, *dP, *dPart, *dLp, *dG, *dL;
    int nblk = qtm::mlp_partial_rows((int)n);
    if (sc.get(&dF, n * qtm::kNF) || sc.get(&dT, n * 3) || sc.get(&dP, qtm::kNTotal) ||
        sc.get(&dPart, (size_t)nblk * qtm::kNParam) || sc.get(&dLp, nblk) || sc.get(&dG, qtm::kNParam) || sc.get(&dL, 1))
        return fail(QTM_E_NOMEM, "device allocation failed");
    std::vector<float> q;
    working_copy(c->mlp_master, q);
    HIPCHECK(hipMemcpy(dF, feat, sizeof(float) * n * qtm::kNF, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(dT, tgt, sizeof(float) * n * 3, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(dP, q.data(), sizeof(float) * qtm::kNTotal, hipMemcpyHostToDevice));
    if (qtm::launch_mlp_grad(dP, dF, dT, nullptr, 0, (int)n, dPart, dLp, dG, dL, c->stream))
        return fail(QTM_E_DEVICE, "gradient kernel launch failed");
    HIPCHECK(hipStreamSynchronize(c->stream));
    HIPCHECK(hipMemcpy(grad, dG, sizeof(float) * qtm::kNParam, hipMemcpyDeviceToHost));
    float l = 0.f;
    HIPCHECK(hipMemcpy(&l, dL, sizeof(float), hipMemcpyDeviceToHost));
    if (loss) *loss = l;
    return QTM_OK;
}

int qtm_train_proposal(qtm_ctx* c, const float* feat, const float* tgt, int64_t n, int32_t n_epochs, int32_t batch,
                       float lr, uint64_t shuffle_seed, float* loss_out) {
    if (check_ctx(c)) return QTM_E_INVAL;
    if (!feat || !tgt || n < 1 || n > (1LL << 30)) return fail(QTM_E_INVAL, "bad training set");
    if (n_epochs < 1 || batch < 1 || !(lr > 0.f)) return fail(QTM_E_INVAL, "bad training options");
    for (int64_t i = 0; i < n * qtm::kNF; ++i) if (!std::isfinite(feat[i])) return fail(QTM_E_INVAL, "non-finite feature");
    for (int64_t i = 0; i < n * 3; ++i) if (!std::isfinite(tgt[i])) return fail(QTM_E_INVAL, "non-finite target");
    HIPCHECK(hipSetDevice(c->device));
    if (!c->have_mlp) {
        init_proposal(c->mlp_master, feat, tgt, n, shuffle_seed);
        c->have_mlp = true;
    }
    DevScratch sc;
    float *dF, *dT, *dMaster, *dWork, *dM, *dV, *dPart, *dLp, *dL;
    int* dPerm;
    int nblk = qtm::mlp_partial_rows(batch);
    // one loss per step of an epoch, read back once per epoch (no wait between steps)
    const int64_t steps_ep = n < batch ? 1 : n / batch;
    if (sc.get(&dF, (size_t)n * qtm::kNF) || sc.get(&dT, (size_t)n * 3) || sc.get(&dMaster, qtm::kNTotal) ||
        sc.get(&dWork, qtm::kNTotal) || sc.get(&dM, qtm::kNParam) || sc.get(&dV, qtm::kNParam) ||
        sc.get(&dPart, (size_t)nblk * qtm::kNParam) || sc.get(&dLp, nblk) ||
        sc.get(&dL, (size_t)steps_ep) || sc.get(&dPerm, (size_t)n))
        return fail(QTM_E_NOMEM, "device allocation failed");
    std::vector<float> hl((size_t)steps_ep);
    std::vector<float> q;
    working_copy(c->mlp_master, q);
    HIPCHECK(hipMemcpy(dF, feat, sizeof(float) * n * qtm::kNF, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(dT, tgt, sizeof(float) * n * 3, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(dMaster, c->mlp_master.data(), sizeof(float) * qtm::kNTotal, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(dWork, q.data(), sizeof(float) * qtm::kNTotal, hipMemcpyHostToDevice));
    HIPCHECK(hipMemset(dM, 0, sizeof(float) * qtm::kNParam));
    HIPCHECK(hipMemset(dV, 0, sizeof(float) * qtm::kNParam));
    std::vector<int> perm(n);
    uint64_t x = shuffle_seed * 0x9E3779B97F4A7C15ULL + 1;
    auto next = [&]() { x ^= x << 13; x ^= x >> 7; x ^= x << 17; return x; };
    int step = 0;
    for (int ep = 0; ep < n_epochs; ++ep) {
        for (int64_t i = 0; i < n; ++i) perm[i] = (int)i;
        for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[next() % (uint64_t)(i + 1)]);
        HIPCHECK(hipMemcpy(dPerm, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice));
        double esum = 0.0;
        int64_t eseen = 0, k = 0;
        std::vector<int> nbs;
        for (int64_t b0 = 0; b0 + batch <= n || (b0 == 0 && n < batch); b0 += batch) {
            int nb = (int)std::min<int64_t>(batch, n - b0);
            if (qtm::launch_mlp_train_step(dMaster, dWork, dM, dV, dF, dT, dPerm, b0, nb, dPart, dLp, dL + k, lr, ++step,
                                           c->stream))
                return fail(QTM_E_DEVICE, "training step launch failed");
            nbs.push_back(nb);
            ++k;
            if (n < batch) break;
        }
        HIPCHECK(hipMemcpyAsync(hl.data(), dL, sizeof(float) * k, hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(hipStreamSynchronize(c->stream));
        for (int64_t i = 0; i < k; ++i) { esum += (double)hl[i] * nbs[i]; eseen += nbs[i]; }
        if (loss_out) loss_out[ep] = (float)(esum / (double)std::max<int64_t>(1, eseen));
    }
    HIPCHECK(hipMemcpy(c->mlp_master.data(), dMaster, sizeof(float) * qtm::kNTotal, hipMemcpyDeviceToHost));
    working_copy(c->mlp_master, q);
    HIPCHECK(hipMemcpy(c->d_mlp, q.data(), sizeof(float) * qtm::kNTotal, hipMemcpyHostToDevice));
    {
        std::vector<uint16_t> fr = mlp_fragments(q);
        HIPCHECK(hipMemcpy(c->d_mlpf, fr.data(), sizeof(uint16_t) * fr.size(), hipMemcpyHostToDevice));
    }
    return QTM_OK;
}

int qtm_run_range_noalloc(qtm_ctx* c, int64_t traj_begin, int64_t count, uint64_t seed, double* sum, double* sumsq) {
    if (check_ctx(c)) return QTM_E_INVAL;
    if (c->sys.size() != 1) return fail(QTM_E_INVAL, "qtm_run_range_noalloc takes a context of one system");
    if (count < 1 || traj_begin < 0) return fail(QTM_E_INVAL, "need count >= 1 and traj_begin >= 0");
    if (!sum || !sumsq) return fail(QTM_E_INVAL, "null output buffer");
    if ((c->o.form & QTM_FORM_LEARNED) && !c->have_mlp) return fail(QTM_E_STATE, "learned form requested before qtm_set_proposal");
    HIPCHECK(hipSetDevice(c->device));
    unsigned char* base = nullptr;
    int rc = scratch_address(c->device, &base);
    if (rc) return rc;
    auto t0 = std::chrono::steady_clock::now();
    // the context's per-run read-back calls refer to qtm_run only
    c->ran = false;
    c->last_count = 0;
    SysHost& S = c->sys[0];
    const size_t m = (size_t)S.n_e * S.n_t;
    // scratch layout: [total sums 2m][total sums of squares m][chunk sums 2m][chunk squares m]
    // [averaging partials][queue][run counters 4][X chunk][counters chunk][jump counts chunk]
    const int nchunk_max = 256;
    const size_t o_tsum = 0, o_tsq = o_tsum + align256(16 * m), o_csum = o_tsq + align256(8 * m),
                 o_csq = o_csum + align256(16 * m), o_part = o_csq + align256(8 * m),
                 o_queue = o_part + align256(sizeof(double) * std::max(qtm::average_part_size((int)m, nchunk_max),
                                                                      qtm::average_part_size((int)m, 1))),
                 o_cnt = o_queue + 256, o_traj = o_cnt + 256;
    const size_t per_traj = 16 * m + 16 + 4;
    if (o_traj + align256(per_traj) + 1024 > kNoallocScratchBytes)
        return fail(QTM_E_INVAL, "one trajectory's outputs (%zu values) do not fit the %d MiB scratch", m, QTM_NOALLOC_SCRATCH_MB);
    const long long cap = (long long)((kNoallocScratchBytes - o_traj - 1024) / per_traj);   // 1024: alignment of 3 regions
    const long long chunk = std::min<long long>(cap, count);
    const size_t o_X = o_traj, o_ts = o_X + align256(16 * m * chunk), o_jn = o_ts + align256(16 * chunk);
    if (o_jn + align256(4 * chunk) > kNoallocScratchBytes) return fail(QTM_E_INVAL, "scratch layout overflow");
    hipStream_t st = c->stream;
    double* tsum = (double*)(base + o_tsum);
    double* tsq = (double*)(base + o_tsq);
    double* avg[3] = {(double*)(base + o_part), (double*)(base + o_csum), (double*)(base + o_csq)};
    unsigned long long* cnt = (unsigned long long*)(base + o_cnt);
    if (qtm::launch_fill(cnt, 4 * sizeof(unsigned long long), 0, st)) return fail(QTM_E_DEVICE, "fill kernel launch failed");
    qtm_stats_t stt{};
    stt.ntraj = count;
    stt.failed_traj = -1;
    qtm::LaunchInfo li{};
    for (long long done = 0; done < count; done += chunk) {
        const long long n = std::min(chunk, count - done);
        qtm::DevSystem ds = S.dev;
        ds.X = (double2*)(base + o_X);
        ds.tstat = (int*)(base + o_ts);
        ds.jn = (int*)(base + o_jn);
        ds.jt = (double*)(base + o_X);      // no jump log or segment records (capacities 0)
        ds.jc = (int*)(base + o_X);
        ds.segs = (float*)(base + o_X);
        ds.queue = (unsigned long long*)(base + o_queue);
        ds.count = n;
        ds.traj_begin = traj_begin + done;
        ds.key0 = seed;
        S.dev = ds;                       // enqueue_run reads the host copy (qtm_run resets it)
        HIPCHECK(hipMemcpyAsync(c->d_sys, &ds, sizeof(ds), hipMemcpyHostToDevice, st));
        qtm::RunArgs a = run_args(c, n, 0, 0);
        if ((rc = enqueue_run(c, a, n, st, &li, avg))) return rc;
        const int blk = 256, g = (int)((2 * m + blk - 1) / blk);
        hipLaunchKernelGGL(accumulate_kernel, dim3(g), dim3(blk), 0, st, tsum, (const double*)avg[1], (int)(2 * m), done == 0 ? 1 : 0);
        hipLaunchKernelGGL(accumulate_kernel, dim3(g), dim3(blk), 0, st, tsq, (const double*)avg[2], (int)m, done == 0 ? 1 : 0);
        hipLaunchKernelGGL(tstat_sum_kernel, dim3(64), dim3(256), 0, st, (const int*)ds.tstat, n, cnt);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(st));
        unsigned long long stamps[2] = {0, 0}, ctrs[4] = {0, 0, 0, 0};
        long long failv = 0;
        HIPCHECK(hipMemcpy(stamps, c->d_stamp, sizeof(stamps), hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(&failv, c->d_fail, sizeof(long long), hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(ctrs, c->d_counters, sizeof(ctrs), hipMemcpyDeviceToHost));
        stt.kernel_ms += (double)(stamps[1] - stamps[0]) / (double)c->wall_khz;
        stt.passes += (int64_t)ctrs[0];
        stt.root_evals += (int64_t)ctrs[1];
        stt.max_team_passes = std::max<int64_t>(stt.max_team_passes, (int64_t)ctrs[2]);
        stt.rhs_evals += (int64_t)ctrs[0] * li.cols;
        if (failv != LLONG_MAX) {
            stt.failed_traj = failv;
            c->st = stt;
            return fail(QTM_E_STEP, "trajectory %lld failed (max_steps or step-size underflow)", failv);
        }
    }
    unsigned long long tot[4] = {0, 0, 0, 0};
    HIPCHECK(hipMemcpy(tot, cnt, sizeof(tot), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(sum, tsum, sizeof(double) * 2 * m, hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(sumsq, tsq, sizeof(double) * m, hipMemcpyDeviceToHost));
    stt.accepted = (int64_t)tot[0]; stt.rejected = (int64_t)tot[1]; stt.segments = (int64_t)tot[2]; stt.jumps = (int64_t)tot[3];
    stt.blocks = li.blocks; stt.threads = li.threads; stt.tile_cols = li.cols; stt.lds_bytes = li.lds; stt.team_shape = li.shape;
    stt.elapsed_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    c->st = stt;
    return QTM_OK;
}

void qtm_destroy(qtm_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    for (auto& S : c->sys) {
        for (auto& b : S.bufs) if (b.p) (void)hipFree(b.p);
        free_buf(S.X); free_buf(S.tstat); free_buf(S.jt); free_buf(S.jc); free_buf(S.jn);
        free_buf(S.segs); free_buf(S.queue); free_buf(S.sum); free_buf(S.sumsq); free_buf(S.avg_part);
    }
    if (c->d_sys) (void)hipFree(c->d_sys);
    if (c->d_fail) (void)hipFree(c->d_fail);
    if (c->d_counters) (void)hipFree(c->d_counters);
    if (c->d_cursor) (void)hipFree(c->d_cursor);
    if (c->d_cls_off) (void)hipFree(c->d_cls_off);
    if (c->d_cls_cur) (void)hipFree(c->d_cls_cur);
    if (c->d_stamp) (void)hipFree(c->d_stamp);
    if (c->d_sys_cls) (void)hipFree(c->d_sys_cls);
    if (c->d_mlp) (void)hipFree(c->d_mlp);
    if (c->d_mlpf) (void)hipFree(c->d_mlpf);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    for (auto e : c->side_ev) if (e) (void)hipEventDestroy(e);
    for (auto st : c->side) if (st) (void)hipStreamDestroy(st);
    if (c->fork) (void)hipEventDestroy(c->fork);
    if (c->pin) (void)hipHostFree(c->pin);
    delete c;
}

}  // extern "C"
