// qtm_internal.h -- device-side data structures shared by the host runtime and
// the HIP kernels of libqtm (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qtm {

constexpr int kMaxE = 16;        // expectation operators per system
constexpr int kMaxC = 16;        // collapse operators per system
constexpr int kMaxTD = 4;        // time-dependent Hamiltonian terms per system
constexpr int kNVMax = 16;       // values per column in one block reduction
constexpr int kNF = 16, kNH = 64, kNO = 3;   // proposal network 16 -> 64 -> 64 -> 3
constexpr int kNParam = kNH * kNF + kNH + kNH * kNH + kNH + kNO * kNH + kNO;  // 5443
constexpr int kNTotal = kNParam + 2 * kNF;                                      // + mean, scale
constexpr int kSegRec = 20;      // floats per segment record
constexpr int kMlpFrag = 24 * 64 * 4;   // BF16 A-fragments of the proposal: 24 groups x 64 lanes x 4

// Column (trajectory slot) states.
enum : int { ST_EMPTY = 0, ST_NEW = 1, ST_NEEDK1 = 2, ST_NEEDF1 = 3, ST_PROBED = 4, ST_STEP = 5 };
// Post-step actions.
enum : int { ACT_NONE = 0, ACT_REJECT = 1, ACT_ACCEPT = 2, ACT_JUMP = 3, ACT_FAIL = 4, ACT_POSTJUMP = 5 };

// One system as the kernels see it.
struct DevSystem {
    int d, dp;                 // dimension; dense kernels pad it to a multiple of 8
    int n_c, n_e, n_t, n_f;
    int rt;                    // dense: 16-row tiles of the real-embedded operator (2dp/16)
    int any_csr_e;             // some observable needs the staged-vector product
    int e_nv[kMaxE];           // values per observable (1: real diagonal, 2: complex)
    int e_fmt[kMaxE];          // 1 CSR, 2 diagonal
    int e_doff[kMaxE];         // diagonal values offset into e_val
    // right-hand-side operator M = -i H_eff
    const double* Mfrag;       // dense: (2dp)^2 doubles in MFMA A-fragment order (block kernel:
                               // [RT][KB][64]; team kernel: [RT][RT][64][4], permuted columns)
    const float* Mfrag32;      // same, rounded to FP32
    const double* Mteam;       // team-kernel layout [RT][RT][64][4] (every dense system of a batch)
    const float* Mteam32;
    const int* sl_off;         // sparse: sliced ELL, 64-row slices; entry offset of each slice
    const int* sl_w;           // width of each slice
    const int* sl_col;         // [slice entries], column-major inside a slice
    const double2* sl_val;
    const float2* sl_val32;
    long long ell_n;           // entries of the sliced ELL (sum over slices of 64 x width)
    // collapse operators (CSR, concatenated; row pointers absolute)
    const int* c_rp;           // [n_c][d+1]
    const int* c_ci;
    const double2* c_val;
    // observables (CSR part: absolute row pointers [n_e][d+1]; diagonal part in e_val)
    const int* e_rp;
    const int* e_ci;
    const double2* e_val;
    const double* f_diag;      // [12 + n_c][d]: rows 0..11 diagonal feature operators (learned form),
                               // rows 12 + n: diagonal of C_n^dag C_n when c_isdiag
    // time-dependent terms (small dense kernel): M(t) = M + sum_k f_k(t) (-i H_k) with
    // f_k(t) = td[4k] + td[4k+1] cos(td[4k+3] t) + td[4k+2] sin(td[4k+3] t)
    int n_td;
    const double* td;          // [n_td][4] coefficients (c, a, b, w)
    const double* Mtd;         // [n_td][(2dp)^2] team-layout A-fragments of -i H_k
    const float* Mtd32;        // same, rounded to FP32
    int c_isdiag;              // every C_n has at most one entry per row, so C_n^dag C_n is diagonal
    int tile_band;             // team layout: every 16-row tile (rt, s) holding a nonzero has |rt - s| <= 1
    const double2* psi0;       // [d]
    const double* tlist;       // [n_t]
    double t0, tend;
    // per-run outputs (indices relative to traj_begin)
    double2* X;                // [count][n_e][n_t]
    int* tstat;                // [count][4] accepted, rejected, segments, jumps
    double* jt;                // [count][jcap]
    int* jc;                   // [count][jcap]
    int* jn;                   // [count]
    float* segs;               // [count][seg_cap][kSegRec]
    unsigned long long* queue; // next relative trajectory index to hand out
    long long count;
    long long traj_begin;
    unsigned long long key0;   // Philox key word 0 (the run's seed)
    unsigned long long key1;   // Philox key word 1 (system index)
};

struct RunArgs {
    const DevSystem* sys;      // device array of systems handled by this launch
    int n_sys;
    unsigned int* sys_cursor;  // first system that may still have trajectories (tile classes with
                               // xcd_off: one cursor per XCD list, absolute system indices)
    const int* xcd_off;        // tile classes: [9] offsets of the eight per-XCD system lists in sys
                               // (nullptr: one list)
    double rtol, atol;
    long long max_steps;
    int jcap, seg_cap;
    int learned;
    const float* mlp;          // [kNTotal] weights (BF16-rounded values), biases, mean, scale
    const unsigned short* mlpf;  // [kMlpFrag] BF16 weight fragments for the matrix-core evaluation
    long long* fail;           // smallest failing global trajectory index (LLONG_MAX: none)
    unsigned long long* counters;  // [4]: product passes (sum over teams), norm-polynomial evaluations of
                                   // the jump-time root finds, most passes of one team, unused
    long long max_cycles;      // failsafe bound on block cycles
    int tile_cols;             // requested columns per block (0: as many as the waves allow)
    int persistent;            // refill free slots from the queue
    int ell_lds;               // sparse kernel: the sliced ELL of each system is copied into LDS
};

// Host-side launchers (defined in qtm_kernels.hip).
struct LaunchInfo { int blocks, threads, lds, cols, shape; };
int launch_dense(const RunArgs& a, const DevSystem& s0, int max_d, int prec, int blocks_per_cu,
                 hipStream_t st, LaunchInfo* info);
// one launch for the systems a.sys[0 .. a.n_sys) of dimension at most max_d
// (max_ell: most sliced-ELL entries of one of them; the ELL goes into LDS when it fits
// there without lowering the occupancy)
int launch_sparse(const RunArgs& a, const DevSystem& s0, int max_d, long long max_ell, int prec, int cols,
                  hipStream_t st, LaunchInfo* info);
// fixed-order trajectory average: partial sums over chunks of trajectories, then
// the chunks in order; part holds average_part_size(m) doubles
size_t average_part_size(int m, long long count);
int launch_average(const DevSystem& s, double* part, double* sum, double* sumsq, hipStream_t st);
// fills bytes (a multiple of 8) with the 8-byte pattern v (graph-capturable clearing)
int launch_fill(void* p, size_t bytes, unsigned long long v, hipStream_t st);
// several fills in one launch (buffer i: n[i] 8-byte words set to v[i])
constexpr int kFillSet = 8;
struct FillSet {
    unsigned long long* p[kFillSet];
    long long n[kFillSet];
    unsigned long long v[kFillSet];
    int count;
};
int launch_fills(const FillSet& f, hipStream_t st);
// writes the device wall clock (hipDeviceAttributeWallClockRate kHz) to *t
int launch_stamp(unsigned long long* t, hipStream_t st);
int dense_occupancy(int max_d, int prec, int tile_cols, int* blocks_per_cu, int* lds);
// proposal network (qtm_mlp.hip)
int launch_mlp_grad(const float* P, const float* feat, const float* tgt, const int* perm, long long base, int n,
                    float* partial, float* loss_part, float* grad, float* loss, hipStream_t st);
// one training step: gradient of the batch, then Adam on the masters and the BF16-valued copy
int launch_mlp_train_step(float* master, float* work, float* m, float* v, const float* feat, const float* tgt,
                          const int* perm, long long base, int n, float* partial, float* loss_part, float* loss, float lr,
                          int step, hipStream_t st);
int mlp_partial_rows(int n);
// wave-per-tile dense kernel (qtm_wave.hip), d <= 64
int wave_supported(int d);
int launch_wave(const RunArgs& a, const DevSystem& s0, int prec, int waves_per_team, hipStream_t st, LaunchInfo* info);
int team_candidates(int d, int* waves, int cap);
// a batch's dense systems in one persistent launch per tile class (d <= 64, 128, 256),
// operator A-fragments read from L2; a.sys holds the class's systems in the order blocks
// take them; returns -1 when max_d > 256
// waves: waves per team, one of team_batch_candidates(class) (0: the class's default shape)
int launch_team_batch(const RunArgs& a, int max_d, int max_ne, int prec, int waves, hipStream_t st, LaunchInfo* info);
int team_batch_class(int d);      // 0, 1, 2 for d <= 64, 128, 256; -1 above
int team_batch_candidates(int cls, int* waves, int cap);
// exact-propagator kernel (qtm_expo.hip), d <= 40, FP64: Pg = fragments of exp(h 2^-j M),
// j = 0..J; m steps per output interval, NS steps from t0 to t_end
int launch_expo(const RunArgs& a, const DevSystem& s0, const double* Pg, int J, int m, double h, long long NS,
                hipStream_t st, LaunchInfo* info);

}  // namespace qtm
