/*
 * sanitize_check.cpp -- TEST INFRASTRUCTURE: a stand-alone driver that runs the
 * oracle's C interface on small problems, built together with qtm_oracle.cpp in
 * one translation unit under AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitize.py).  Every path of the trajectory solver is taken:
 * dense and CSR right-hand sides, one and several channels, the learned proposal
 * (including a proposal far outside the step range), segment records, a jump log
 * shorter than the jump count, the max_steps failure and the step-size underflow
 * failure, plus the single-step and jump-free entry points.
 */
#include "qtm_oracle.cpp"

#include <cstdio>
#include <cstdlib>

namespace {

int g_fail = 0;
void check(bool ok, const char* what) {
    if (!ok) { std::fprintf(stderr, "FAILED: %s\n", what); g_fail = 1; }
}

struct DenseOp {
    std::vector<double> v;   // interleaved complex, row-major
    qtmref_op op{};
    DenseOp(int d, std::initializer_list<double> vals) : v(vals) {
        op.fmt = 0; op.dim = d; op.nnz = 0; op.val = v.data(); op.row_ptr = nullptr; op.col_ind = nullptr;
    }
};

struct DiagOp {
    std::vector<double> v;
    qtmref_op op{};
    explicit DiagOp(std::vector<double> re) {
        for (double x : re) { v.push_back(x); v.push_back(0.0); }
        op.fmt = 2; op.dim = (int)re.size(); op.nnz = 0; op.val = v.data(); op.row_ptr = nullptr; op.col_ind = nullptr;
    }
};

struct CsrOp {
    std::vector<double> v;
    std::vector<int32_t> rp, ci;
    qtmref_op op{};
    void finish(int d) {
        op.fmt = 1; op.dim = d; op.nnz = (int64_t)ci.size(); op.val = v.data(); op.row_ptr = rp.data(); op.col_ind = ci.data();
    }
};

// open transverse-field Ising chain of L sites in CSR, decay sqrt(g) sigma_- per site
void ising(int L, double J, double hx, double g, CsrOp& H, std::vector<CsrOp>& C) {
    const int d = 1 << L;
    H.rp.assign(1, 0);
    for (int i = 0; i < d; ++i) {
        double zz = 0.0;
        for (int s = 0; s + 1 < L; ++s) {
            int a = (i >> (L - 1 - s)) & 1, b = (i >> (L - 2 - s)) & 1;
            zz += (1 - 2 * a) * (1 - 2 * b);
        }
        std::vector<std::pair<int, double>> row = {{i, -J * zz}};
        for (int s = 0; s < L; ++s) row.push_back({i ^ (1 << (L - 1 - s)), -hx});
        std::sort(row.begin(), row.end());
        for (auto& e : row) { H.ci.push_back(e.first); H.v.push_back(e.second); H.v.push_back(0.0); }
        H.rp.push_back((int32_t)H.ci.size());
    }
    H.finish(d);
    C.resize(L);
    for (int s = 0; s < L; ++s) {
        CsrOp& c = C[s];
        c.rp.assign(1, 0);
        for (int i = 0; i < d; ++i) {
            // row i holds <i|sigma_-^s|j> with j = i without the down bit of site s
            const int bit = 1 << (L - 1 - s);
            if (i & bit) { c.ci.push_back(i ^ bit); c.v.push_back(std::sqrt(g)); c.v.push_back(0.0); }
            c.rp.push_back((int32_t)c.ci.size());
        }
        c.finish(d);
    }
}

}  // namespace

int main() {
    // driven two-level atom: H = sigma_x / 2, C = sqrt(0.5) sigma_-, psi0 = |g>
    DenseOp H(2, {0, 0, 0.5, 0, 0.5, 0, 0, 0});
    DenseOp Cm(2, {0, 0, 0, 0, std::sqrt(0.5), 0, 0, 0});
    DiagOp Z({1.0, -1.0});
    std::vector<double> psi0 = {0, 0, 1, 0};
    std::vector<double> tl(101);
    for (int k = 0; k < 101; ++k) tl[k] = 0.1 * k;
    const int n = 24, jcap = 2;
    std::vector<double> X((size_t)n * 101 * 2), jt((size_t)n * jcap);
    std::vector<int> jc((size_t)n * jcap), jn(n);
    std::vector<int64_t> st((size_t)n * 5);
    int64_t fail = 0;
    int rc = qtmref_run(&H.op, &Cm.op, 1, psi0.data(), tl.data(), 101, &Z.op, 1, 1e-6, 1e-8, 1000000, 0, 0, 0, n, 2,
                        nullptr, nullptr, 0, X.data(), jcap, jt.data(), jc.data(), jn.data(), st.data(), 0, nullptr, &fail, nullptr, nullptr, 0);
    check(rc == 0 && fail == -1, "two-level run");
    int total = 0;
    for (int q = 0; q < n; ++q) total += jn[q];
    check(total > n, "two-level jumps (more than the log capacity)");

    // learned proposal with segment records: a random network, then one whose output is
    // far below the step range (the snap limits it)
    std::vector<double> mlp(MLP_NTOTAL, 0.0);
    uint64_t x = 12345;
    for (int i = 0; i < MLP_NPARAM; ++i) {
        x = x * 6364136223846793005ULL + 1442695040888963407ULL;
        mlp[i] = 0.1 * (((double)(x >> 11) * 0x1.0p-53) - 0.5);
    }
    for (int i = MLP_NPARAM + NF; i < MLP_NTOTAL; ++i) mlp[i] = 1.0;
    DiagOp F0({1.0, 0.0});
    const int seg_cap = 3;
    std::vector<double> segs((size_t)n * seg_cap * (NF + 4));
    rc = qtmref_run(&H.op, &Cm.op, 1, psi0.data(), tl.data(), 101, &Z.op, 1, 1e-6, 1e-8, 1000000, 3, 0, 0, n, 2,
                    mlp.data(), &F0.op, 1, X.data(), jcap, jt.data(), jc.data(), jn.data(), st.data(), seg_cap,
                    segs.data(), &fail, nullptr, nullptr, 0);
    check(rc == 0, "learned run");
    mlp[MLP_NPARAM - 3] = -1e4;          // b3[0]: log h0 = -1e4
    rc = qtmref_run(&H.op, &Cm.op, 1, psi0.data(), tl.data(), 101, &Z.op, 1, 1e-6, 1e-8, 1000000, 3, 0, 0, n, 2,
                    mlp.data(), &F0.op, 1, X.data(), jcap, jt.data(), jc.data(), jn.data(), st.data(), 0, nullptr, &fail, nullptr, nullptr, 0);
    check(rc == 0, "learned run with a proposal below the step range");

    // CSR right-hand side with several channels and a CSR observable (Ising chain, L = 4)
    CsrOp Hs;
    std::vector<CsrOp> Cs;
    ising(4, 1.0, 0.8, 0.2, Hs, Cs);
    std::vector<qtmref_op> cops;
    for (auto& c : Cs) cops.push_back(c.op);
    std::vector<double> p16(32, 0.0);
    p16[0] = 1.0;
    std::vector<double> tl2(21);
    for (int k = 0; k < 21; ++k) tl2[k] = 0.25 * k;
    DiagOp Z16(std::vector<double>(16, 0.5));
    const qtmref_op eops2[2] = {Hs.op, Z16.op};
    std::vector<double> X2((size_t)n * 2 * 21 * 2);
    rc = qtmref_run(&Hs.op, cops.data(), (int)cops.size(), p16.data(), tl2.data(), 21, eops2, 2, 1e-6, 1e-8, 1000000, 1,
                    0, 0, n, 2, nullptr, nullptr, 0, X2.data(), jcap, jt.data(), jc.data(), jn.data(), st.data(), 0,
                    nullptr, &fail, nullptr, nullptr, 0);
    check(rc == 0, "CSR run");

    // time-dependent Hamiltonian: H0 + (0.3 + 0.5 cos(2 t) + 0.1 sin(2 t)) sigma_x
    DenseOp Hx(2, {0, 0, 1, 0, 1, 0, 0, 0});
    const double coef[4] = {0.3, 0.5, 0.1, 2.0};
    rc = qtmref_run(&H.op, &Cm.op, 1, psi0.data(), tl.data(), 101, &Z.op, 1, 1e-6, 1e-8, 1000000, 5, 0, 0, n, 2,
                    nullptr, nullptr, 0, X.data(), jcap, jt.data(), jc.data(), jn.data(), st.data(), 0, nullptr, &fail,
                    &Hx.op, coef, 1);
    check(rc == 0, "time-dependent run");

    // failure paths: max_steps, then a step-size underflow (huge H at t0 = 1e6)
    rc = qtmref_run(&H.op, &Cm.op, 1, psi0.data(), tl.data(), 101, &Z.op, 1, 1e-6, 1e-8, 3, 0, 0, 7, 4, 1,
                    nullptr, nullptr, 0, X.data(), 0, nullptr, nullptr, jn.data(), st.data(), 0, nullptr, &fail, nullptr, nullptr, 0);
    check(rc == -4 && fail == 7, "max_steps failure");
    DenseOp Hbig(2, {0, 0, 1e12, 0, 1e12, 0, 0, 0});
    std::vector<double> tl3 = {1e6, 1e6 + 1.0};
    rc = qtmref_run(&Hbig.op, &Cm.op, 1, psi0.data(), tl3.data(), 2, &Z.op, 1, 1e-6, 1e-8, 1000000, 0, 0, 0, 2, 1,
                    nullptr, nullptr, 0, X.data(), 0, nullptr, nullptr, jn.data(), st.data(), 0, nullptr, &fail, nullptr, nullptr, 0);
    check(rc == -4 && fail == 0, "step-size underflow failure");

    // single step with dense output, the jump-free integrator with a forced rejection
    std::vector<double> M(8);
    qtmref_build_M(&H.op, &Cm.op, 1, M.data());
    std::vector<double> yn(4), ev(4), u(3 * 4);
    double en = 0.0, th[3] = {0.0, 0.5, 1.0};
    qtmref_dopri_step(2, M.data(), psi0.data(), 0.1, 1e-6, 1e-8, yn.data(), ev.data(), &en, 3, th, u.data());
    check(std::isfinite(en), "dopri step");
    std::vector<double> ts(1000), ye(4);
    int nacc = 0, nrej = 0;
    double h0 = 0.0;
    qtmref_integrate_nojump(2, M.data(), psi0.data(), 0.0, 10.0, 1e-6, 1e-8, 1000, ts.data(), &nacc, ye.data(), &h0,
                            5.0, &nrej);
    check(nacc > 0 && nrej > 0, "jump-free integration with a rejected first step");
    std::vector<double> mean(202), var(101);
    qtmref_average(X.data(), 4, 1, 101, mean.data(), var.data());
    if (g_fail) return 1;
    std::printf("sanitize check ok\n");
    return 0;
}
