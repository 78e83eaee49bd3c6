/*
 * qtm_oracle.cpp -- plain FP64 CPU oracle for the quantum trajectories method.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table
 * or helper with the HIP library; everything here is written out in the most
 * direct form so that it can be checked against the paper by eye.
 *
 * What it computes (one trajectory, the paper's Algorithm 1 of Sec. 2.2):
 *   * effective Hamiltonian H_eff = H - (i/2) sum_n C_n^dag C_n (Eq. for
 *     H_eff, hbar = 1), stored as the right-hand-side matrix M = -i H_eff so
 *     that d psi/dt = M psi;
 *   * (A) a uniform threshold r drawn for every segment;
 *   * (B) integration of d psi/dt = M psi while <psi|psi> >= r, here with the
 *     Dormand-Prince 5(4) pair and its 4th-order continuous extension
 *     (Dormand & Prince 1980; Hairer, Norsett & Wanner, Solving ODEs I,
 *     Sec. II.4-II.6), standard step-size controller and starting step;
 *   * the jump time: the first theta in [0,1] where the dense-output norm
 *     ||u(theta)||^2 crosses r, by a uniform scan plus bisection;
 *   * (C) channel choice: the smallest n with sum_{m<=n} P_m >= u, where
 *     P_m = <psi|C_m^dag C_m|psi> / sum (Eq. for P_i), with u an independent
 *     uniform; the jump psi <- C_n psi / sqrt(<psi|C_n^dag C_n|psi>)
 *     (Eq. for the post-jump state);
 *   * (D) a new threshold and a restart at the jump time;
 *   * expectation values <psi|O|psi>/<psi|psi> at the output times, averaged
 *     over trajectories in FP64 (Sec. 3: the per-node and final averages).
 * Random numbers: Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11), key
 * (seed, system id), counter (trajectory, segment, 0, 0); word 0 gives r and
 * word 1 gives u through U(x) = ((x >> 11) + 0.5) 2^-53.
 *
 * The learned form replaces only the starting step of each segment by the
 * MLP proposal (16 -> 64 -> 64 -> 3, GELU), evaluated here in FP64 on the
 * same (BF16-rounded) weights, snapped to the grid 2^(k/4).
 *
 * Time-dependent Hamiltonians (the right-hand-side function of Sec. 3 receives
 * the time): H(t) = H0 + sum_k f_k(t) H_k with f_k(t) = c + a cos(w t) + b sin(w t);
 * the collapse operators stay constant, so M(t) = M0 - i sum_k f_k(t) H_k with
 * M0 = -i H0 - 1/2 sum_n C_n^dag C_n, and every evaluation of the right-hand side
 * (DOPRI5 stages at t + c_s h, the starting step's probe at t + h0) takes its time.
 */
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cd = std::complex<double>;

/* ------------------------------------------------------------ operators */
struct Op {
    int fmt = 0;            // 0 dense row-major, 1 CSR, 2 diagonal
    int dim = 0;
    std::vector<cd> v;
    std::vector<int> rp, ci;
};

// y = A x
void apply(const Op& A, const cd* x, cd* y) {
    const int d = A.dim;
    if (A.fmt == 0) {
        for (int i = 0; i < d; ++i) {
            cd s = 0.0;
            for (int j = 0; j < d; ++j) s += A.v[(size_t)i * d + j] * x[j];
            y[i] = s;
        }
    } else if (A.fmt == 1) {
        for (int i = 0; i < d; ++i) {
            cd s = 0.0;
            for (int p = A.rp[i]; p < A.rp[i + 1]; ++p) s += A.v[p] * x[A.ci[p]];
            y[i] = s;
        }
    } else {
        for (int i = 0; i < d; ++i) y[i] = A.v[i] * x[i];
    }
}

// f(t) = c + a cos(w t) + b sin(w t), the coefficient of one time-dependent term
struct Drive {
    double c = 0.0, a = 0.0, b = 0.0, w = 0.0;
    double at(double t) const { return c + a * std::cos(w * t) + b * std::sin(w * t); }
};

double norm2(const cd* x, int d) {
    double s = 0.0;
    for (int i = 0; i < d; ++i) s += std::norm(x[i]);
    return s;
}

// Dense row-major copy of any operator (used only to build M).
std::vector<cd> to_dense(const Op& A) {
    const int d = A.dim;
    std::vector<cd> out((size_t)d * d, 0.0);
    if (A.fmt == 0) return A.v;
    if (A.fmt == 1) {
        for (int i = 0; i < d; ++i)
            for (int p = A.rp[i]; p < A.rp[i + 1]; ++p) out[(size_t)i * d + A.ci[p]] += A.v[p];
    } else {
        for (int i = 0; i < d; ++i) out[(size_t)i * d + i] = A.v[i];
    }
    return out;
}

/* Right-hand-side matrix M = -i H - 1/2 sum_n C_n^dag C_n  (= -i H_eff).
 * Kept dense when H is dense, else CSR with the union pattern of the terms. */
Op build_M(const Op& H, const std::vector<Op>& C) {
    const int d = H.dim;
    const cd mi(0.0, -1.0);
    if (H.fmt != 1) {
        std::vector<cd> M = to_dense(H);
        for (auto& z : M) z *= mi;
        for (const Op& c : C) {
            std::vector<cd> Cd = to_dense(c);
            // (C^dag C)_{pq} = sum_k conj(C_kp) C_kq
            for (int p = 0; p < d; ++p)
                for (int q = 0; q < d; ++q) {
                    cd s = 0.0;
                    for (int k = 0; k < d; ++k) s += std::conj(Cd[(size_t)k * d + p]) * Cd[(size_t)k * d + q];
                    M[(size_t)p * d + q] -= 0.5 * s;
                }
        }
        Op out;
        out.fmt = 0; out.dim = d; out.v = std::move(M);
        return out;
    }
    // Sparse: accumulate each row into a dense row buffer, keep touched columns.
    std::vector<std::vector<std::pair<int, cd>>> rows(d);
    for (int i = 0; i < d; ++i)
        for (int p = H.rp[i]; p < H.rp[i + 1]; ++p) rows[i].push_back({H.ci[p], mi * H.v[p]});
    for (const Op& c : C) {
        // rows of C as (col, val) lists
        std::vector<std::vector<std::pair<int, cd>>> crow(d);
        if (c.fmt == 1) {
            for (int k = 0; k < d; ++k)
                for (int p = c.rp[k]; p < c.rp[k + 1]; ++p) crow[k].push_back({c.ci[p], c.v[p]});
        } else if (c.fmt == 2) {
            for (int k = 0; k < d; ++k) crow[k].push_back({k, c.v[k]});
        } else {
            for (int k = 0; k < d; ++k)
                for (int j = 0; j < d; ++j)
                    if (c.v[(size_t)k * d + j] != 0.0) crow[k].push_back({j, c.v[(size_t)k * d + j]});
        }
        for (int k = 0; k < d; ++k)
            for (auto& a : crow[k])
                for (auto& b : crow[k]) rows[a.first].push_back({b.first, -0.5 * std::conj(a.second) * b.second});
    }
    Op out;
    out.fmt = 1; out.dim = d; out.rp.assign(d + 1, 0);
    std::vector<cd> acc(d, 0.0);
    std::vector<char> touched(d, 0);
    for (int i = 0; i < d; ++i) {
        std::vector<int> cols;
        for (auto& e : rows[i]) {
            if (!touched[e.first]) { touched[e.first] = 1; cols.push_back(e.first); }
            acc[e.first] += e.second;
        }
        std::sort(cols.begin(), cols.end());
        for (int j : cols) { out.ci.push_back(j); out.v.push_back(acc[j]); acc[j] = 0.0; touched[j] = 0; }
        out.rp[i + 1] = (int)out.ci.size();
    }
    return out;
}

/* ------------------------------------------------------ Philox4x64-10 */
void philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ULL * x0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ULL * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ x1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ x3 ^ k1;
        uint64_t n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

double uniform53(uint64_t x) { return ((double)(x >> 11) + 0.5) * 0x1.0p-53; }

/* ------------------------------------------------ Dormand-Prince 5(4) */
struct Dopri {
    double c[7];
    double a[7][6];   // a[s][j], stage s (0-based) uses k_0..k_{s-1}
    double b[7];      // 5th-order weights (= a[6][*], FSAL)
    double bs[7];     // 4th-order weights
    double dd[7];     // dense-output weights
    Dopri() {
        std::memset(this, 0, sizeof(*this));
        c[0] = 0.0; c[1] = 1.0 / 5; c[2] = 3.0 / 10; c[3] = 4.0 / 5; c[4] = 8.0 / 9; c[5] = 1.0; c[6] = 1.0;
        a[1][0] = 1.0 / 5;
        a[2][0] = 3.0 / 40;        a[2][1] = 9.0 / 40;
        a[3][0] = 44.0 / 45;       a[3][1] = -56.0 / 15;       a[3][2] = 32.0 / 9;
        a[4][0] = 19372.0 / 6561;  a[4][1] = -25360.0 / 2187;  a[4][2] = 64448.0 / 6561;  a[4][3] = -212.0 / 729;
        a[5][0] = 9017.0 / 3168;   a[5][1] = -355.0 / 33;      a[5][2] = 46732.0 / 5247;  a[5][3] = 49.0 / 176;
        a[5][4] = -5103.0 / 18656;
        b[0] = 35.0 / 384; b[1] = 0.0; b[2] = 500.0 / 1113; b[3] = 125.0 / 192; b[4] = -2187.0 / 6784;
        b[5] = 11.0 / 84; b[6] = 0.0;
        for (int j = 0; j < 6; ++j) a[6][j] = b[j];
        bs[0] = 5179.0 / 57600; bs[1] = 0.0; bs[2] = 7571.0 / 16695; bs[3] = 393.0 / 640;
        bs[4] = -92097.0 / 339200; bs[5] = 187.0 / 2100; bs[6] = 1.0 / 40;
        dd[0] = -12715105075.0 / 11282082432.0; dd[1] = 0.0; dd[2] = 87487479700.0 / 32700410799.0;
        dd[3] = -10690763975.0 / 1880347072.0; dd[4] = 701980252875.0 / 199316789632.0;
        dd[5] = -1453857185.0 / 822651844.0; dd[6] = 69997945.0 / 29380423.0;
    }
};
const Dopri& dopri() { static const Dopri t; return t; }

/* One attempted DOPRI5 step from (t, y, k[0] = f(t, y)) with step h; f(t, x, out)
 * evaluates the right-hand side, stage s at time t + c_s h.
 * Fills k[1..6], y_new (the stage-7 input) and the error vector e. */
template <class F>
void dopri_step(const F& f, double t, int d, const cd* y, double h, std::vector<std::vector<cd>>& k,
                std::vector<cd>& ynew, std::vector<cd>& e, std::vector<cd>& w) {
    const Dopri& T = dopri();
    for (int s = 1; s < 7; ++s) {
        for (int i = 0; i < d; ++i) {
            cd acc = 0.0;
            for (int j = 0; j < s; ++j) acc += T.a[s][j] * k[j][i];
            w[i] = y[i] + h * acc;
        }
        if (s == 6) ynew.assign(w.begin(), w.begin() + d);
        f(t + T.c[s] * h, w.data(), k[s].data());
    }
    for (int i = 0; i < d; ++i) {
        cd acc = 0.0;
        for (int j = 0; j < 7; ++j) acc += (T.b[j] - T.bs[j]) * k[j][i];
        e[i] = h * acc;
    }
}

// err = sqrt( (1/d) sum_i |e_i|^2 / sc_i^2 ),  sc_i = atol + rtol * max(|y_i|, |ynew_i|)
double error_norm(const cd* e, const cd* y, const cd* ynew, int d, double rtol, double atol) {
    double s = 0.0;
    for (int i = 0; i < d; ++i) {
        double sc = atol + rtol * std::max(std::abs(y[i]), std::abs(ynew[i]));
        s += std::norm(e[i]) / (sc * sc);
    }
    return std::sqrt(s / d);
}

// Continuous extension u(theta) = y + th (D + (1-th)(B + th (R4 + (1-th) R5)))
struct Dense {
    std::vector<cd> y, D, B, R4, R5;
    void build(const cd* y0, const cd* y1, const std::vector<std::vector<cd>>& k, double h, int d) {
        const Dopri& T = dopri();
        y.assign(y0, y0 + d); D.resize(d); B.resize(d); R4.resize(d); R5.resize(d);
        for (int i = 0; i < d; ++i) {
            D[i] = y1[i] - y0[i];
            B[i] = h * k[0][i] - D[i];
            R4[i] = D[i] - h * k[6][i] - B[i];
            cd acc = 0.0;
            for (int j = 0; j < 7; ++j) acc += T.dd[j] * k[j][i];
            R5[i] = h * acc;
        }
    }
    void eval(double th, cd* u, int d) const {
        const double t1 = 1.0 - th;
        for (int i = 0; i < d; ++i) u[i] = y[i] + th * (D[i] + t1 * (B[i] + th * (R4[i] + t1 * R5[i])));
    }
};

/* Starting step (Hairer-Norsett-Wanner Sec. II.4, with the step limited to
 * the remaining interval).  f0 = f(t0, y0) is given; costs one more evaluation,
 * f(t0 + h0, y0 + h0 f0). */
template <class F>
double initial_step(const F& f, double t0, int d, const cd* y0, const cd* f0, double span, double rtol, double atol,
                    std::vector<cd>& tmp, std::vector<cd>& f1, int64_t& rhs) {
    double s0 = 0.0, s1 = 0.0;
    for (int i = 0; i < d; ++i) {
        double sc = atol + rtol * std::abs(y0[i]);
        s0 += std::norm(y0[i]) / (sc * sc);
        s1 += std::norm(f0[i]) / (sc * sc);
    }
    double d0 = std::sqrt(s0 / d), d1 = std::sqrt(s1 / d);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    h0 = std::min(h0, span);
    for (int i = 0; i < d; ++i) tmp[i] = y0[i] + h0 * f0[i];
    f(t0 + h0, tmp.data(), f1.data());
    ++rhs;
    double s2 = 0.0;
    for (int i = 0; i < d; ++i) {
        double sc = atol + rtol * std::abs(y0[i]);
        s2 += std::norm(f1[i] - f0[i]) / (sc * sc);
    }
    double d2 = std::sqrt(s2 / d) / h0;
    double h1;
    if (d1 <= 1e-15 && d2 <= 1e-15) h1 = std::max(1e-6, h0 * 1e-3);
    else h1 = std::pow(0.01 / std::max(d1, d2), 1.0 / 5.0);
    return std::min(std::min(100.0 * h0, h1), span);
}

/* ----------------------------------------------------------------- MLP */
constexpr int NF = 16, NH = 64, NO = 3;
struct Mlp {
    // layout: W1[NH][NF], b1[NH], W2[NH][NH], b2[NH], W3[NO][NH], b3[NO], mu[NF], sd[NF]
    const double* p;
    const double* W1() const { return p; }
    const double* b1() const { return p + NH * NF; }
    const double* W2() const { return b1() + NH; }
    const double* b2() const { return W2() + NH * NH; }
    const double* W3() const { return b2() + NH; }
    const double* b3() const { return W3() + NO * NH; }
    const double* mu() const { return b3() + NO; }
    const double* sd() const { return mu() + NF; }
};
constexpr int MLP_NPARAM = NH * NF + NH + NH * NH + NH + NO * NH + NO;   // trainable
constexpr int MLP_NTOTAL = MLP_NPARAM + 2 * NF;                          // + input standardisation

double gelu(double x) { return 0.5 * x * (1.0 + std::erf(x / std::sqrt(2.0))); }
double gelu_d(double x) {
    return 0.5 * (1.0 + std::erf(x / std::sqrt(2.0))) + x * std::exp(-0.5 * x * x) / std::sqrt(2.0 * M_PI);
}

struct MlpTape { double x[NF], z1[NH], a1[NH], z2[NH], a2[NH], o[NO]; };

void mlp_forward(const Mlp& m, const double* feat, MlpTape& t) {
    for (int i = 0; i < NF; ++i) t.x[i] = (feat[i] - m.mu()[i]) / m.sd()[i];
    for (int h = 0; h < NH; ++h) {
        double s = m.b1()[h];
        for (int i = 0; i < NF; ++i) s += m.W1()[h * NF + i] * t.x[i];
        t.z1[h] = s; t.a1[h] = gelu(s);
    }
    for (int h = 0; h < NH; ++h) {
        double s = m.b2()[h];
        for (int i = 0; i < NH; ++i) s += m.W2()[h * NH + i] * t.a1[i];
        t.z2[h] = s; t.a2[h] = gelu(s);
    }
    for (int o = 0; o < NO; ++o) {
        double s = m.b3()[o];
        for (int i = 0; i < NH; ++i) s += m.W3()[o * NH + i] * t.a2[i];
        t.o[o] = s;
    }
}

/* Per-sample loss: (o0 - log h*)^2 + [uncensored] (pin_0.05(log tau - o1) + pin_0.95(log tau - o2)),
 * pinball pin_q(z) = z (q - [z < 0]).  Returns loss; adds dL/dparam * scale to g. */
double mlp_loss_grad(const Mlp& m, const double* feat, double log_h, double log_tau, int censored,
                     double scale, double* g) {
    MlpTape t;
    mlp_forward(m, feat, t);
    double L = 0.0, dO[NO] = {0, 0, 0};
    double r0 = t.o[0] - log_h;
    L += r0 * r0;
    dO[0] = 2.0 * r0;
    if (!censored) {
        const double q[2] = {0.05, 0.95};
        for (int k = 0; k < 2; ++k) {
            double z = log_tau - t.o[1 + k];
            double ind = z < 0 ? 1.0 : 0.0;
            L += z * (q[k] - ind);
            dO[1 + k] = -(q[k] - ind);
        }
    }
    if (!g) return L;
    double* gW1 = g;
    double* gb1 = gW1 + NH * NF;
    double* gW2 = gb1 + NH;
    double* gb2 = gW2 + NH * NH;
    double* gW3 = gb2 + NH;
    double* gb3 = gW3 + NO * NH;
    double da2[NH], dz2[NH], da1[NH], dz1[NH];
    for (int o = 0; o < NO; ++o) {
        gb3[o] += scale * dO[o];
        for (int i = 0; i < NH; ++i) gW3[o * NH + i] += scale * dO[o] * t.a2[i];
    }
    for (int i = 0; i < NH; ++i) {
        double s = 0.0;
        for (int o = 0; o < NO; ++o) s += m.W3()[o * NH + i] * dO[o];
        da2[i] = s;
        dz2[i] = s * gelu_d(t.z2[i]);
    }
    for (int h = 0; h < NH; ++h) {
        gb2[h] += scale * dz2[h];
        for (int i = 0; i < NH; ++i) gW2[h * NH + i] += scale * dz2[h] * t.a1[i];
    }
    for (int i = 0; i < NH; ++i) {
        double s = 0.0;
        for (int h = 0; h < NH; ++h) s += m.W2()[h * NH + i] * dz2[h];
        da1[i] = s;
        dz1[i] = s * gelu_d(t.z1[i]);
    }
    for (int h = 0; h < NH; ++h) {
        gb1[h] += scale * dz1[h];
        for (int i = 0; i < NF; ++i) gW1[h * NF + i] += scale * dz1[h] * t.x[i];
    }
    (void)da1; (void)da2;
    return L;
}

/* --------------------------------------------------------- trajectories */
struct Problem {
    int d = 0, n_c = 0, n_e = 0, n_t = 0;
    Op M;
    std::vector<Op> Htd;         // time-dependent terms H_k and their coefficients f_k
    std::vector<Drive> ftd;
    std::vector<Op> C, O, F;     // collapse, expectation, feature (diagonal) operators
    std::vector<cd> psi0;
    std::vector<double> tl;
    double rtol = 1e-6, atol = 1e-8;
    int64_t max_steps = 1000000;
    uint64_t seed = 0, sys_id = 0;
    const double* mlp = nullptr;   // learned form when non-null
};

/* out = M(t) x = M0 x - i sum_k f_k(t) H_k x  (tmp: scratch of length d) */
void rhs_at(const Problem& P, double t, const cd* x, cd* out, cd* tmp) {
    apply(P.M, x, out);
    for (size_t k = 0; k < P.Htd.size(); ++k) {
        apply(P.Htd[k], x, tmp);
        const cd c(0.0, -P.ftd[k].at(t));
        for (int i = 0; i < P.d; ++i) out[i] += c * tmp[i];
    }
}

struct TrajResult {
    int64_t accepted = 0, rejected = 0, rhs = 0, segments = 0, jumps = 0;
    int failed = 0;
};

// Value of <u|O|u>/<u|u> (complex) written to X[(e*n_t + kk)*2 + {0,1}].
void record(const Problem& P, const cd* u, int kk, double* X, std::vector<cd>& tmp) {
    const int d = P.d;
    double nn = norm2(u, d);
    for (int e = 0; e < P.n_e; ++e) {
        apply(P.O[e], u, tmp.data());
        cd s = 0.0;
        for (int i = 0; i < d; ++i) s += std::conj(u[i]) * tmp[i];
        X[((size_t)e * P.n_t + kk) * 2 + 0] = s.real() / nn;
        X[((size_t)e * P.n_t + kk) * 2 + 1] = s.imag() / nn;
    }
}

// Segment-start features of the learned proposal (16 values).
void features(const Problem& P, const cd* y, double r, double t, double* f, std::vector<cd>& tmp) {
    const int d = P.d;
    double nn = norm2(y, d);
    for (int q = 0; q < 12; ++q) {
        double s = 0.0;
        if (q < (int)P.F.size())
            for (int i = 0; i < d; ++i) s += P.F[q].v[i].real() * std::norm(y[i]);
        f[q] = s / nn;
    }
    for (int n = 0; n < 2; ++n) {
        double s = 0.0;
        if (n < P.n_c) { apply(P.C[n], y, tmp.data()); s = norm2(tmp.data(), d); }
        f[12 + n] = s / nn;
    }
    f[14] = std::log(r);
    f[15] = (t - P.tl[0]) / (P.tl[P.n_t - 1] - P.tl[0]);
}

double snap_step(double log_h) {
    // h = 2^(k/4) with k = round(4 log2 h), evaluated exactly as 2^floor(k/4) * 2^((k mod 4)/4).
    // log2 h is first limited to [-40, 10], a non-finite proposal taking the lower end, so
    // that the proposed step is positive and finite whatever the network returns (the
    // controller then corrects it like any other first step).
    const double quarter[4] = {1.0, 1.18920711500272106672, 1.41421356237309504880, 1.68179283050742908606};
    double l2 = log_h / std::log(2.0);
    if (!(l2 >= -40.0)) l2 = -40.0;
    if (l2 > 10.0) l2 = 10.0;
    long k = std::lrint(4.0 * l2);
    long q = k >= 0 ? k / 4 : -((-k + 3) / 4);
    return std::ldexp(quarter[k - 4 * q], (int)q);
}

/* Segment record for training data: features, realised jump delay (or censored),
 * and the controller's proposal after the segment's first accepted step. */
struct SegRec { double f[NF]; double tau; double h_next; int censored; int valid; };

int run_trajectory(const Problem& P, int64_t traj, double* X, int jcap, double* jt, int* jc, int* jn,
                   TrajResult& R, int seg_cap, SegRec* segs) {
    const int d = P.d;
    const double t0 = P.tl[0], tend = P.tl[P.n_t - 1];
    std::vector<std::vector<cd>> k(7, std::vector<cd>(d));
    std::vector<cd> y(P.psi0), ynew(d), e(d), w(d), tmp(d), f1(d), u(d), scr(d);
    auto f = [&](double tt, const cd* x, cd* out) { rhs_at(P, tt, x, out, scr.data()); };
    Dense D;
    double t = t0;
    int kk = 0;                       // next output index
    while (kk < P.n_t && P.tl[kk] == t0) { record(P, y.data(), kk, X, tmp); ++kk; }
    int64_t seg = 0, jumps = 0, attempts = 0;
    int nrec = 0;
    for (;;) {
        if (!(t < tend)) break;
        /* (A)/(D): new threshold r and channel uniform u for this segment */
        uint64_t ctr[4] = {(uint64_t)traj, (uint64_t)seg, 0, 0}, key[2] = {P.seed, P.sys_id}, rnd[4];
        philox4x64_10(ctr, key, rnd);
        const double r = uniform53(rnd[0]), uch = uniform53(rnd[1]);
        R.segments++;
        f(t, y.data(), k[0].data());
        R.rhs++;
        double h;
        SegRec* rec = (segs && nrec < seg_cap) ? &segs[nrec] : nullptr;
        double feat[NF];
        if (P.mlp || rec) features(P, y.data(), r, t, feat, tmp);
        if (P.mlp) {
            Mlp m{P.mlp};
            MlpTape tp;
            mlp_forward(m, feat, tp);
            h = std::min(snap_step(tp.o[0]), tend - t);
        } else {
            h = initial_step(f, t, d, y.data(), k[0].data(), tend - t, P.rtol, P.atol, tmp, f1, R.rhs);
        }
        if (rec) { std::memcpy(rec->f, feat, sizeof(feat)); rec->valid = 1; rec->h_next = -1; rec->censored = 1; rec->tau = 0; nrec++; }
        const double tseg = t;
        bool first_accept = true;
        bool rejected = false;
        bool jumped = false;
        while (t < tend) {
            if (attempts >= P.max_steps) { R.failed = 1; goto done; }
            bool last = false;
            if (t + h >= tend) { h = tend - t; last = true; }
            dopri_step(f, t, d, y.data(), h, k, ynew, e, w);
            R.rhs += 6;
            ++attempts;
            double err = error_norm(e.data(), y.data(), ynew.data(), d, P.rtol, P.atol);
            if (!(err <= 1.0)) {
                double f = std::isfinite(err) ? std::max(0.2, 0.9 * std::pow(err, -0.2)) : 0.2;
                h *= f;
                rejected = true;
                R.rejected++;
                if (!(h > 16.0 * DBL_EPSILON * std::fabs(t))) { R.failed = 1; goto done; }
                continue;
            }
            R.accepted++;
            const double tb = last ? tend : t + h;
            double fac = (err == 0.0) ? 10.0 : std::min(10.0, 0.9 * std::pow(err, -0.2));
            if (rejected) fac = std::min(1.0, fac);
            if (rec && first_accept) rec->h_next = h * fac;
            first_accept = false;
            const double n2 = norm2(ynew.data(), d);
            D.build(y.data(), ynew.data(), k, h, d);
            if (P.n_c > 0 && n2 < r) {
                /* jump inside this step: first theta with ||u(theta)||^2 = r */
                const int NS = 32;
                double lo = 0.0, hi = 1.0;
                for (int m = 1; m <= NS; ++m) {
                    double th = (double)m / NS;
                    D.eval(th, u.data(), d);
                    if (norm2(u.data(), d) < r) { hi = th; lo = (double)(m - 1) / NS; break; }
                }
                while (hi - lo > 1e-13) {
                    double mid = 0.5 * (lo + hi);
                    D.eval(mid, u.data(), d);
                    if (norm2(u.data(), d) < r) hi = mid; else lo = mid;
                }
                const double th = 0.5 * (lo + hi);
                const double tj = t + th * h;
                while (kk < P.n_t && P.tl[kk] < tj) {
                    D.eval((P.tl[kk] - t) / h, u.data(), d);
                    record(P, u.data(), kk, X, tmp);
                    ++kk;
                }
                D.eval(th, u.data(), d);            // psi* = u(theta*)
                std::vector<double> p(P.n_c);
                double tot = 0.0;
                for (int n = 0; n < P.n_c; ++n) {
                    apply(P.C[n], u.data(), tmp.data());
                    p[n] = norm2(tmp.data(), d);
                    tot += p[n];
                }
                int ch = -1;
                if (tot > 0.0) {
                    double thr = uch * tot, cum = 0.0;
                    for (int n = 0; n < P.n_c; ++n) {
                        cum += p[n];
                        if (p[n] > 0.0 && cum >= thr) { ch = n; break; }
                    }
                    if (ch < 0)
                        for (int n = P.n_c - 1; n >= 0; --n) if (p[n] > 0.0) { ch = n; break; }
                }
                if (ch >= 0) {
                    apply(P.C[ch], u.data(), tmp.data());
                    double s = 1.0 / std::sqrt(p[ch]);
                    for (int i = 0; i < d; ++i) y[i] = tmp[i] * s;
                } else {
                    double s = 1.0 / std::sqrt(norm2(u.data(), d));
                    for (int i = 0; i < d; ++i) y[i] = u[i] * s;
                }
                if (jumps < jcap) { jt[jumps] = tj; jc[jumps] = ch; }
                ++jumps;
                if (rec) { rec->tau = tj - tseg; rec->censored = 0; }
                t = tj;
                while (kk < P.n_t && P.tl[kk] == tj) { record(P, y.data(), kk, X, tmp); ++kk; }
                ++seg;
                jumped = true;
                break;
            }
            while (kk < P.n_t && P.tl[kk] <= tb) {
                if (P.tl[kk] == tb) record(P, ynew.data(), kk, X, tmp);
                else { D.eval((P.tl[kk] - t) / h, u.data(), d); record(P, u.data(), kk, X, tmp); }
                ++kk;
            }
            t = tb;
            y.swap(ynew);
            k[0].swap(k[6]);
            h *= fac;
            rejected = false;
        }
        if (!jumped) break;
    }
done:
    R.jumps = jumps;
    *jn = (int)jumps;
    return R.failed ? -4 : 0;
}

Op op_from_c(int fmt, int dim, int64_t nnz, const double* val, const int32_t* rp, const int32_t* ci) {
    Op o;
    o.fmt = fmt; o.dim = dim;
    size_t n = fmt == 0 ? (size_t)dim * dim : fmt == 2 ? (size_t)dim : (size_t)nnz;
    o.v.resize(n);
    for (size_t i = 0; i < n; ++i) o.v[i] = cd(val[2 * i], val[2 * i + 1]);
    if (fmt == 1) { o.rp.assign(rp, rp + dim + 1); o.ci.assign(ci, ci + nnz); }
    return o;
}

}  // namespace

extern "C" {

typedef struct {
    int32_t fmt;            // 0 dense row-major, 1 CSR, 2 diagonal
    int32_t dim;
    int64_t nnz;            // CSR only
    const double* val;      // interleaved (re, im)
    const int32_t* row_ptr; // CSR only
    const int32_t* col_ind; // CSR only
} qtmref_op;

void qtmref_philox4x64_10(const uint64_t* ctr, const uint64_t* key, uint64_t* out) { philox4x64_10(ctr, key, out); }
double qtmref_uniform53(uint64_t x) { return uniform53(x); }

// Dense copy of M = -i H_eff (row-major, interleaved) for inspection by tests.
int qtmref_build_M(const qtmref_op* H, const qtmref_op* c, int n_c, double* out) {
    Op h = op_from_c(H->fmt, H->dim, H->nnz, H->val, H->row_ptr, H->col_ind);
    std::vector<Op> C;
    for (int n = 0; n < n_c; ++n) C.push_back(op_from_c(c[n].fmt, c[n].dim, c[n].nnz, c[n].val, c[n].row_ptr, c[n].col_ind));
    Op M = build_M(h, C);
    std::vector<cd> Md = to_dense(M);
    for (size_t i = 0; i < Md.size(); ++i) { out[2 * i] = Md[i].real(); out[2 * i + 1] = Md[i].imag(); }
    return 0;
}

/* One DOPRI5 step of d psi/dt = M psi (M dense, interleaved) for tests:
 * outputs y_new, the error vector, the error norm and the dense output at n_th thetas. */
int qtmref_dopri_step(int d, const double* Mri, const double* yri, double h, double rtol, double atol,
                      double* ynew_out, double* err_vec, double* err_norm, int n_th, const double* th,
                      double* u_out) {
    Op M;
    M.fmt = 0; M.dim = d; M.v.resize((size_t)d * d);
    for (size_t i = 0; i < M.v.size(); ++i) M.v[i] = cd(Mri[2 * i], Mri[2 * i + 1]);
    std::vector<cd> y(d), ynew(d), e(d), w(d), u(d);
    for (int i = 0; i < d; ++i) y[i] = cd(yri[2 * i], yri[2 * i + 1]);
    std::vector<std::vector<cd>> k(7, std::vector<cd>(d));
    apply(M, y.data(), k[0].data());
    auto f = [&](double, const cd* x, cd* out) { apply(M, x, out); };
    dopri_step(f, 0.0, d, y.data(), h, k, ynew, e, w);
    for (int i = 0; i < d; ++i) {
        ynew_out[2 * i] = ynew[i].real(); ynew_out[2 * i + 1] = ynew[i].imag();
        err_vec[2 * i] = e[i].real(); err_vec[2 * i + 1] = e[i].imag();
    }
    *err_norm = error_norm(e.data(), y.data(), ynew.data(), d, rtol, atol);
    Dense D;
    D.build(y.data(), ynew.data(), k, h, d);
    for (int q = 0; q < n_th; ++q) {
        D.eval(th[q], u.data(), d);
        for (int i = 0; i < d; ++i) { u_out[(size_t)q * 2 * d + 2 * i] = u[i].real(); u_out[(size_t)q * 2 * d + 2 * i + 1] = u[i].imag(); }
    }
    return 0;
}

/* Integrates d psi/dt = M psi from t0 to tend without jumps and logs the
 * accepted times (for the cross-check of the stepper and controller).
 * first_step > 0 replaces the starting-step rule (so that a test can force
 * rejected attempts); *n_rej receives the number of rejected attempts. */
int qtmref_integrate_nojump(int d, const double* Mri, const double* yri, double t0, double tend,
                            double rtol, double atol, int cap, double* t_out, int* n_out, double* y_end,
                            double* h_first, double first_step, int* n_rej) {
    Op M;
    M.fmt = 0; M.dim = d; M.v.resize((size_t)d * d);
    for (size_t i = 0; i < M.v.size(); ++i) M.v[i] = cd(Mri[2 * i], Mri[2 * i + 1]);
    std::vector<cd> y(d), ynew(d), e(d), w(d), tmp(d), f1(d);
    for (int i = 0; i < d; ++i) y[i] = cd(yri[2 * i], yri[2 * i + 1]);
    std::vector<std::vector<cd>> k(7, std::vector<cd>(d));
    apply(M, y.data(), k[0].data());
    auto f = [&](double, const cd* x, cd* out) { apply(M, x, out); };
    int64_t rhs = 0;
    double h = first_step > 0.0 ? first_step : initial_step(f, t0, d, y.data(), k[0].data(), tend - t0, rtol, atol, tmp, f1, rhs);
    *h_first = h;
    double t = t0;
    int n = 0, nrej = 0;
    bool rejected = false;
    int64_t guard = 0;
    while (t < tend && guard++ < 10000000) {
        bool last = false;
        if (t + h >= tend) { h = tend - t; last = true; }
        dopri_step(f, t, d, y.data(), h, k, ynew, e, w);
        double err = error_norm(e.data(), y.data(), ynew.data(), d, rtol, atol);
        if (!(err <= 1.0)) {
            h *= std::isfinite(err) ? std::max(0.2, 0.9 * std::pow(err, -0.2)) : 0.2;
            rejected = true;
            ++nrej;
            continue;
        }
        double fac = (err == 0.0) ? 10.0 : std::min(10.0, 0.9 * std::pow(err, -0.2));
        if (rejected) fac = std::min(1.0, fac);
        t = last ? tend : t + h;
        if (n < cap) t_out[n] = t;
        ++n;
        y.swap(ynew);
        k[0].swap(k[6]);
        h *= fac;
        rejected = false;
    }
    *n_out = n;
    if (n_rej) *n_rej = nrej;
    for (int i = 0; i < d; ++i) { y_end[2 * i] = y[i].real(); y_end[2 * i + 1] = y[i].imag(); }
    return 0;
}

/* Runs trajectories [traj_begin, traj_begin + ntraj).
 *   X      [ntraj][n_e][n_t][2]   per-trajectory <O_e>(t_k) (required)
 *   jt/jc  [ntraj][jcap], jn [ntraj]   jump log (nullable when jcap == 0)
 *   stats  [ntraj][5]: accepted, rejected, rhs evaluations, segments, jumps (nullable)
 *   mlp    learned-form weights (nullable); f_ops: up to 12 diagonal feature operators
 *   segs   [ntraj][seg_cap][NF + 4] segment records (nullable)
 *   h_td   n_td time-dependent terms H_k, td_coef [n_td][4] = (c, a, b, w) of
 *          f_k(t) = c + a cos(w t) + b sin(w t) (nullable when n_td == 0)
 * Returns 0, or -4 when a trajectory failed (smallest failing index in *fail_traj). */
int qtmref_run(const qtmref_op* H, const qtmref_op* c_ops, int n_c, const double* psi0, const double* tlist,
               int n_t, const qtmref_op* e_ops, int n_e, double rtol, double atol, int64_t max_steps,
               uint64_t seed, uint64_t sys_id, int64_t traj_begin, int64_t ntraj, int nthreads,
               const double* mlp, const qtmref_op* f_ops, int n_f,
               double* X, int jcap, double* jt, int* jc, int* jn, int64_t* stats,
               int seg_cap, double* segs, int64_t* fail_traj,
               const qtmref_op* h_td, const double* td_coef, int n_td) {
    Problem P;
    P.d = H->dim; P.n_c = n_c; P.n_e = n_e; P.n_t = n_t;
    Op h = op_from_c(H->fmt, H->dim, H->nnz, H->val, H->row_ptr, H->col_ind);
    for (int n = 0; n < n_c; ++n) P.C.push_back(op_from_c(c_ops[n].fmt, c_ops[n].dim, c_ops[n].nnz, c_ops[n].val, c_ops[n].row_ptr, c_ops[n].col_ind));
    for (int n = 0; n < n_e; ++n) P.O.push_back(op_from_c(e_ops[n].fmt, e_ops[n].dim, e_ops[n].nnz, e_ops[n].val, e_ops[n].row_ptr, e_ops[n].col_ind));
    for (int n = 0; n < n_f; ++n) P.F.push_back(op_from_c(f_ops[n].fmt, f_ops[n].dim, f_ops[n].nnz, f_ops[n].val, f_ops[n].row_ptr, f_ops[n].col_ind));
    P.M = build_M(h, P.C);
    for (int n = 0; n < n_td; ++n) {
        P.Htd.push_back(op_from_c(h_td[n].fmt, h_td[n].dim, h_td[n].nnz, h_td[n].val, h_td[n].row_ptr, h_td[n].col_ind));
        Drive dv;
        dv.c = td_coef[4 * n]; dv.a = td_coef[4 * n + 1]; dv.b = td_coef[4 * n + 2]; dv.w = td_coef[4 * n + 3];
        P.ftd.push_back(dv);
    }
    P.psi0.resize(P.d);
    for (int i = 0; i < P.d; ++i) P.psi0[i] = cd(psi0[2 * i], psi0[2 * i + 1]);
    P.tl.assign(tlist, tlist + n_t);
    P.rtol = rtol; P.atol = atol; P.max_steps = max_steps; P.seed = seed; P.sys_id = sys_id; P.mlp = mlp;
    int64_t first_fail = -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    std::vector<int> failed(ntraj, 0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < ntraj; ++q) {
        TrajResult R;
        int jn_local = 0;
        std::vector<SegRec> srec(seg_cap > 0 ? seg_cap : 0);
        for (auto& s : srec) s.valid = 0;
        run_trajectory(P, traj_begin + q, X + (size_t)q * n_e * n_t * 2, jcap,
                       jcap ? jt + (size_t)q * jcap : nullptr, jcap ? jc + (size_t)q * jcap : nullptr, &jn_local, R,
                       seg_cap, seg_cap > 0 ? srec.data() : nullptr);
        if (jn) jn[q] = jn_local;
        if (stats) {
            int64_t* s = stats + q * 5;
            s[0] = R.accepted; s[1] = R.rejected; s[2] = R.rhs; s[3] = R.segments; s[4] = R.jumps;
        }
        if (segs) {
            for (int z = 0; z < seg_cap; ++z) {
                double* o = segs + ((size_t)q * seg_cap + z) * (NF + 4);
                std::memcpy(o, srec[z].f, sizeof(double) * NF);
                o[NF] = srec[z].tau; o[NF + 1] = srec[z].h_next; o[NF + 2] = srec[z].censored; o[NF + 3] = srec[z].valid;
            }
        }
        failed[q] = R.failed;
    }
    for (int64_t q = 0; q < ntraj; ++q) if (failed[q]) { first_fail = traj_begin + q; break; }
    if (fail_traj) *fail_traj = first_fail;
    return first_fail >= 0 ? -4 : 0;
}

/* Trajectory average in index order: mean [n_e][n_t][2], var of the real part [n_e][n_t]. */
void qtmref_average(const double* X, int64_t ntraj, int n_e, int n_t, double* mean, double* var) {
    const size_t m = (size_t)n_e * n_t;
    std::vector<double> s(2 * m, 0.0), s2(m, 0.0);
    for (int64_t q = 0; q < ntraj; ++q)
        for (size_t i = 0; i < m; ++i) {
            double re = X[(q * m + i) * 2], im = X[(q * m + i) * 2 + 1];
            s[2 * i] += re; s[2 * i + 1] += im; s2[i] += re * re;
        }
    for (size_t i = 0; i < m; ++i) {
        mean[2 * i] = s[2 * i] / ntraj; mean[2 * i + 1] = s[2 * i + 1] / ntraj;
        if (var) var[i] = std::max(0.0, s2[i] / ntraj - mean[2 * i] * mean[2 * i]);
    }
}

int qtmref_mlp_nparam(void) { return MLP_NPARAM; }
int qtmref_mlp_ntotal(void) { return MLP_NTOTAL; }

// Forward pass for n samples: feat [n][16] -> out [n][3].
void qtmref_mlp_forward(const double* params, const double* feat, int64_t n, double* out) {
    Mlp m{params};
    for (int64_t s = 0; s < n; ++s) {
        MlpTape t;
        mlp_forward(m, feat + s * NF, t);
        for (int o = 0; o < NO; ++o) out[s * NO + o] = t.o[o];
    }
}

/* Mean loss over n samples and its gradient w.r.t. the MLP_NPARAM trainable parameters.
 * tgt [n][3]: log h*, log tau, censored flag. */
double qtmref_mlp_loss_grad(const double* params, const double* feat, const double* tgt, int64_t n, double* grad) {
    Mlp m{params};
    if (grad) std::memset(grad, 0, sizeof(double) * MLP_NPARAM);
    double L = 0.0;
    for (int64_t s = 0; s < n; ++s)
        L += mlp_loss_grad(m, feat + s * NF, tgt[s * 3], tgt[s * 3 + 1], tgt[s * 3 + 2] != 0.0, 1.0 / n, grad);
    return L / n;
}

double qtmref_snap_step(double log_h) { return snap_step(log_h); }

/* The tableau as the oracle uses it: c[7], a[7][6], b[7], b*[7], dense-output d[7]. */
void qtmref_tableau(double* c, double* a, double* b, double* bs, double* dd) {
    const Dopri& T = dopri();
    for (int s = 0; s < 7; ++s) {
        c[s] = T.c[s]; b[s] = T.b[s]; bs[s] = T.bs[s]; dd[s] = T.dd[s];
        for (int j = 0; j < 6; ++j) a[s * 6 + j] = T.a[s][j];
    }
}

}  // extern "C"
