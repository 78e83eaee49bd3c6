/*
 * qtm.h -- C ABI of libqtm.so, a quantum-trajectories (Monte-Carlo wave
 * function) engine for AMD Instinct MI355X (gfx950).
 *
 * The method (the paper's Sec. 2.2): every trajectory evolves a state vector
 * under the non-Hermitian effective Hamiltonian
 *     H_eff = H - (i/2) sum_n C_n^dag C_n                (Eq. for H_eff, hbar = 1)
 * while its squared norm stays at or above a uniform random threshold r;
 * when the norm falls below r a quantum jump psi <- C_n psi / ||C_n psi||
 * (Eq. for the post-jump state) takes place, with channel n chosen with
 * probability P_n proportional to <psi|C_n^dag C_n|psi> (Eq. for P_i), and a
 * new threshold is drawn (Algorithm 1, steps A-D).  Expectation values
 * <psi|O|psi>/<psi|psi> are averaged over trajectories (Sec. 3).
 *
 * This library integrates d psi/dt = M psi, M = -i H_eff, with the adaptive
 * Dormand-Prince 5(4) pair and its 4th-order dense output, finds the jump time
 * as the root of the dense-output norm, draws its random numbers from
 * counter-based Philox4x64-10 streams (key = (seed, system index), counter =
 * (trajectory index, segment index, 0, 0); word 0 -> r, word 1 -> channel
 * uniform, U(x) = ((x >> 11) + 0.5) 2^-53) and averages on the device in FP64.
 *
 * Conventions for every entry point:
 *  - all functions return an int status (QTM_OK or a negative QTM_E_* code)
 *    unless stated otherwise; on error, qtm_last_error() returns a message
 *    (thread-local) and no output buffer is written;
 *  - pointers named in the arguments are HOST pointers unless the name says
 *    device; the library copies every input it needs, so callers keep
 *    ownership of their arrays and may free them right after the call;
 *  - complex numbers are interleaved (re, im) pairs of doubles;
 *  - no C++ exception crosses this boundary.
 */
#ifndef QTM_H
#define QTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- status codes */
#define QTM_OK        0
#define QTM_E_INVAL  (-1)   /* invalid argument (shape, value, NaN, ordering) */
#define QTM_E_NOMEM  (-2)   /* device or host allocation failed */
#define QTM_E_DEVICE (-3)   /* HIP runtime error, or no gfx950 device */
#define QTM_E_STEP   (-4)   /* a trajectory hit max_steps or a step-size underflow
                               (the integrator failure the paper reports as an
                               error level, Sec. 3 solver wrapper) */
#define QTM_E_STATE  (-5)   /* call order violated, e.g. qtm_expect before qtm_run */

/* ------------------------------------------------------------- operators */
#define QTM_FMT_DENSE 0     /* val: dim*dim complex, row-major */
#define QTM_FMT_CSR   1     /* compressed sparse rows: row_ptr[dim+1], col_ind[nnz], val[nnz] */
#define QTM_FMT_DIAG  2     /* val: dim complex diagonal entries */

/* An operator on the d-dimensional state space (the paper's dense uMatrix and
 * sparse uCSRMatrix types, Sec. 3).  Host pointers, FP64 values always; the
 * storage and precision used on the device are the library's choice. */
typedef struct {
    int32_t fmt;              /* QTM_FMT_* */
    int32_t dim;              /* d */
    int64_t nnz;              /* CSR only: number of stored entries */
    const double* val;        /* interleaved complex values */
    const int32_t* row_ptr;   /* CSR only */
    const int32_t* col_ind;   /* CSR only, column indices in [0, d) */
} qtm_op;

/* ------------------------------------------------------------- options */
#define QTM_PREC_FP64   0     /* every product in FP64 (the plain form) */
#define QTM_PREC_FP32   1     /* H_eff products in FP32 with FP32 accumulation; state,
                                 stage sums, norms, root finding and averages in FP64 */

#define QTM_FORM_LEARNED 1u   /* segment start step from the trained MLP proposal */
#define QTM_FORM_BATCHED 2u   /* persistent kernel with per-slot trajectory refill and
                                 autotuned tiles (otherwise: one workgroup per block of
                                 trajectories, no refill) */

typedef struct {
    double rtol;              /* relative tolerance (default 1e-6) */
    double atol;              /* absolute tolerance (default 1e-8) */
    int32_t precision;        /* QTM_PREC_* (default FP64) */
    uint32_t form;            /* OR of QTM_FORM_* (default 0: plain) */
    int64_t max_steps;        /* attempted steps per trajectory before QTM_E_STEP (default 1e6) */
    int32_t device;           /* HIP device ordinal (default 0) */
    int32_t record_jumps;     /* jump-log capacity per trajectory (0: off) */
    void* stream;             /* hipStream_t to run on, NULL: the null stream */
    int32_t keep_traj;        /* keep per-trajectory expectation values (qtm_traj_expect) */
    int32_t seg_cap;          /* segment records per trajectory for proposal training (0: off) */
    int32_t tile_cols;        /* sparse and large dense kernels: trajectories per workgroup (0: default) */
    int32_t team_waves;       /* small dense kernel (d <= 64): wavefronts per 16-trajectory team,
                                 one of qtm_tile_candidates() (0: default shape) */
    int32_t integrator;       /* QTM_INT_DOPRI5 (default) or QTM_INT_EXPO */
    int32_t expo_substeps;    /* QTM_INT_EXPO: propagator steps per output interval (0: 1) */
    int32_t class_waves[3];   /* batches of dense systems, batched form: waves per 16-trajectory team
                                 of the tile classes d <= 64, 128, 256, one of
                                 qtm_batch_tile_candidates(class) (0: the class's default shape;
                                 -1: the class runs on the sliced-ELL SpMM kernel instead) */
    int32_t chunk_traj;       /* runs that keep no per-trajectory data (keep_traj, record_jumps and
                                 seg_cap all 0): at most this many trajectories per chunk (0: as many
                                 as QTM_RUN_CHUNK_MB of expectation samples hold) */
} qtm_opts;

/* Device memory for the per-trajectory expectation samples of one chunk of a run that
 * keeps no per-trajectory data: a run of more trajectories than that processes them in
 * chunks of consecutive indices and adds the chunks' FP64 sums in chunk order. */
#define QTM_RUN_CHUNK_MB 2048

/* Integrators.  QTM_INT_DOPRI5: adaptive Dormand-Prince 5(4) with dense output (the
 * default; every form).  QTM_INT_EXPO: the exact propagator for stiff problems --
 * between jumps psi(t + h) = exp(h M) psi(t) with exp(h M) computed once on the host,
 * one product per step whatever the stiffness of M (the role the paper gives its
 * BDF option, Sec. 2.1 and Sec. 3); the jump time is found by a binary search with
 * the exact propagators exp(h 2^-j M) to h 2^-J <= about 1e-12.  Requirements:
 * time-independent H (qtm_create), FP64 products, the plain or batched form, d <= 40,
 * output times uniformly spaced (steps of h = spacing / expo_substeps). */
#define QTM_INT_DOPRI5 0
#define QTM_INT_EXPO   1

/* Per-run statistics (summed over trajectories of the last qtm_run). */
typedef struct {
    int64_t ntraj;
    int64_t accepted;         /* accepted DOPRI5 steps */
    int64_t rejected;         /* rejected DOPRI5 steps */
    int64_t segments;         /* segments (= jumps + trajectories, unless failed) */
    int64_t jumps;
    int64_t rhs_evals;        /* products M w evaluated (per trajectory-column) */
    int64_t passes;           /* block-wide product passes executed by the kernel */
    int64_t failed_traj;      /* smallest failing trajectory index, -1 if none */
    double kernel_ms;         /* device time of the trajectory kernel(s): device wall-clock stamps
                                 taken on the launch stream just before and after them */
    double elapsed_ms;        /* host wall time of qtm_run */
    int32_t blocks, threads, tile_cols, lds_bytes;   /* launch configuration used */
    int64_t max_team_passes;  /* most product passes of one trajectory team (the launch's critical
                                 path; team kernel only, 0 for the others) */
    int64_t root_evals;       /* evaluations of the dense-output norm polynomial by the jump-time
                                 root finds (32-point scan plus bisection to 1e-13 in theta) */
    int32_t team_shape;       /* small dense kernel: 100 x row tiles per wave + waves per team,
                                 plus 1000 when the banded-operator instance ran; 0 otherwise */
    int32_t reserved_stats;
} qtm_stats_t;

/* A system for qtm_create_batch (same meaning as the qtm_create arguments). */
typedef struct {
    const qtm_op* H;
    const qtm_op* c_ops;
    int32_t n_c;
    const double* psi0;
    const double* tlist;
    int32_t n_t;
    const qtm_op* e_ops;
    int32_t n_e;
} qtm_system;

typedef struct qtm_ctx qtm_ctx;

/* Fills *o with the defaults listed above. */
void qtm_opts_default(qtm_opts* o);

/* Creates a context for one system (the problem statement of the paper's
 * examples, Sec. 4: Hamiltonian, collapse operators, initial state, output
 * times, expectation operators).
 *   H       d x d Hermitian operator (any format).  A CSR H selects the sparse
 *           kernel; a dense H (d <= 256) the MFMA kernel.
 *   c_ops   n_c collapse operators C_n (0 <= n_c <= 16), d x d, any format.
 *   psi0    d complex amplitudes with | ||psi0|| - 1 | <= 1e-10.
 *   tlist   n_t >= 2 strictly increasing output times; tlist[0] is the start
 *           time t0 and tlist[n_t-1] the end time.
 *   e_ops   n_e (1..16) expectation operators O_k (any format).
 *   o       options (NULL: defaults).
 * Builds M = -i H - 1/2 sum C_n^dag C_n on the host in FP64 and uploads it.
 * Errors: QTM_E_INVAL (shape, non-finite entry, bad norm, bad tlist, index
 * out of range), QTM_E_NOMEM, QTM_E_DEVICE. */
int qtm_create(qtm_ctx** out, const qtm_op* H, const qtm_op* c_ops, int32_t n_c, const double* psi0,
               const double* tlist, int32_t n_t, const qtm_op* e_ops, int32_t n_e, const qtm_opts* o);

/* Coefficient of a time-dependent Hamiltonian term: f(t) = c + a cos(omega t) +
 * b sin(omega t). */
typedef struct {
    double c, a, b, omega;
} qtm_drive;
#define QTM_MAX_TD 4

/* Creates a context for one system with a time-dependent Hamiltonian
 *     H(t) = H0 + sum_k f_k(t) H_k,   k < n_td <= QTM_MAX_TD,
 * the case the paper's right-hand-side function supports by receiving the time
 * (Sec. 3, and the remark on the time argument after the trilinear example of
 * Sec. 4.2); the collapse operators stay constant, so H_eff(t) = H(t) - (i/2)
 * sum_n C_n^dag C_n.  Every evaluation of the right-hand side uses its own time
 * (Runge-Kutta stage s at t + c_s h).
 *   H0, c_ops, psi0, tlist, e_ops, o  as for qtm_create;
 *   H_td   n_td Hermitian d x d operators H_k (any format);
 *   f_td   n_td coefficient functions (host array).
 * Supported on the small dense kernel only: d <= 64 (any operator format).
 * Errors: as qtm_create; QTM_E_INVAL also for n_td outside [1, QTM_MAX_TD], d > 64,
 * a non-finite coefficient. */
int qtm_create_td(qtm_ctx** out, const qtm_op* H0, const qtm_op* H_td, const qtm_drive* f_td, int32_t n_td,
                  const qtm_op* c_ops, int32_t n_c, const double* psi0, const double* tlist, int32_t n_t,
                  const qtm_op* e_ops, int32_t n_e, const qtm_opts* o);

/* Creates a context holding n_sys systems of mixed dimension (each dense,
 * d <= 256, n_e <= 16) that qtm_run integrates in one persistent launch per
 * tile class (batched form).  Inside a class the systems are handed to the
 * persistent blocks in decreasing order of an estimated cost d^2 x ||M||_inf x
 * (t_end - t0) (work per step times the steps the norm of M asks for), so that the
 * largest start first.  System s uses Philox key (seed, s).  Errors as qtm_create;
 * the message names the offending system index. */
int qtm_create_batch(qtm_ctx** out, int32_t n_sys, const qtm_system* sys, const qtm_opts* o);

/* Runs trajectories 0..ntraj-1 (of every system of a batch) on the context's
 * stream and waits for them: every trajectory follows Algorithm 1 (steps A-D:
 * threshold draw, no-jump evolution under H_eff until the norm falls below the
 * threshold, channel choice by the probabilities P_n, jump and renormalisation)
 * from t0 to the end time, and its expectation values are averaged over the
 * trajectories on the device (the final averaging of Sec. 3).  Equivalent to
 * qtm_run_range(ctx, 0, ntraj, seed).  Outputs stay in device memory owned by
 * the context until the next run or qtm_destroy.
 * Errors: QTM_E_INVAL (ntraj < 1), QTM_E_NOMEM, QTM_E_DEVICE, QTM_E_STEP (one
 * or more trajectories failed -- the analogue of the negative solver status the
 * paper's solver wrapper reports, Sec. 3; qtm_stats names the smallest index;
 * averages are then not available).  A context with keep_traj, record_jumps and
 * seg_cap all 0 runs more trajectories than one chunk holds (chunk_traj, else
 * QTM_RUN_CHUNK_MB of samples) chunk after chunk, so device memory stays bounded
 * whatever ntraj is; the averages then add the chunks' sums in chunk order. */
int qtm_run(qtm_ctx* ctx, int64_t ntraj, uint64_t seed);

/* Runs trajectories traj_begin .. traj_begin+count-1 (traj_begin >= 0,
 * count >= 1).  This is the work unit of the paper's master/worker split of
 * independent trajectories over computing nodes (Sec. 3): because the random
 * stream of trajectory i depends only on (seed, system, i), the sums of
 * disjoint ranges combine into the sums of their union.  Errors as qtm_run. */
int qtm_run_range(qtm_ctx* ctx, int64_t traj_begin, int64_t count, uint64_t seed);

/* Trajectory averages of the last run (of system 0 for a batch): the final
 * trajectory of Sec. 3, i.e. the mean over trajectories of <psi|O_k|psi>/<psi|psi>
 * at every output time (Sec. 2.2, expectation values of the unnormalised state).
 *   mean [n_e][n_t] complex (interleaved), var [n_e][n_t] variance of the real
 *   part over trajectories (nullable).  Host buffers, caller-allocated; summed in
 *   FP64 in trajectory-index order, so independent of scheduling.
 * Errors: QTM_E_STATE before a successful qtm_run. */
int qtm_expect(const qtm_ctx* ctx, double* mean, double* var);

/* Same for system s of a batch context. */
int qtm_expect_system(const qtm_ctx* ctx, int32_t s, double* mean, double* var);

/* The running sums behind the averages: sum [n_e][n_t] complex, sumsq
 * [n_e][n_t] (of the real part) and the trajectory count, in FP64; sums of
 * disjoint trajectory ranges add. */
int qtm_sums(const qtm_ctx* ctx, int32_t s, double* sum, double* sumsq, int64_t* count);

/* Per-trajectory expectation values of the last run (requires keep_traj):
 * X [count][n_e][n_t] complex for system s. */
int qtm_traj_expect(const qtm_ctx* ctx, int32_t s, double* X);

/* Jump log of trajectory traj (index within the last run's range) of system s
 * (requires record_jumps > 0): the jump times (roots of ||psi(t)||^2 = r,
 * Algorithm 1 step B) and channels n (step C, Eq. for P_i) in order, up to cap
 * (time, channel) pairs written to the host buffers times[cap], channels[cap]
 * (channel -1: every P_n was zero and the state was only renormalised); *count
 * receives the total number of jumps (which may exceed the log capacity).
 * Errors: QTM_E_STATE without record_jumps or before a run, QTM_E_INVAL. */
int qtm_jumps(const qtm_ctx* ctx, int32_t s, int64_t traj, int32_t cap, double* times, int32_t* channels,
              int32_t* count);

/* Per-trajectory counters of the last run: [count][4] = accepted steps,
 * rejected steps, segments, jumps (int32), for system s. */
int qtm_traj_stats(const qtm_ctx* ctx, int32_t s, int32_t* stats);

/* Statistics of the last run (the integrator's work per Sec. 2.1's adaptive
 * step control, and the launch configuration), copied to the host struct *st.
 * Filled also after a run that failed with QTM_E_STEP. */
int qtm_stats(const qtm_ctx* ctx, qtm_stats_t* st);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same computation as
 * qtm_run_range on a context of ONE system, with every per-run device buffer
 * (per-trajectory outputs and counters, queue, averaging partial sums) taken from
 * a fixed array of QTM_NOALLOC_SCRATCH_MB MiB inside the library, one per device,
 * held until the process ends.  The call allocates nothing (no hipMalloc, hipFree
 * or graph capture); trajectories are processed in chunks that fit the array, and
 * the chunk sums are added in chunk order, so the result does not depend on
 * scheduling.
 *   sum    [n_e][n_t] complex (interleaved) sums over the trajectories of
 *          <psi|O_k|psi>/<psi|psi>, caller-allocated host buffer;
 *   sumsq  [n_e][n_t] sums of the squared real parts, caller-allocated host buffer.
 * The mean is sum / count, as qtm_expect forms it from qtm_sums.  Jump logs and
 * segment records are not kept; qtm_stats describes the call.  Afterwards the
 * context's per-run read-back calls (qtm_expect, qtm_sums, qtm_traj_expect,
 * qtm_jumps, qtm_traj_stats, qtm_segments) return QTM_E_STATE until the next
 * qtm_run.  Every call on one device shares that device's array and leaves the
 * last call's contents in it: calls that overlap on one device (several host
 * threads, or several streams in flight) race and must not be made.
 * Errors: QTM_E_INVAL (batch context of several systems, count < 1, null
 * buffer, one trajectory's outputs n_e x n_t larger than the array allows),
 * QTM_E_STATE, QTM_E_DEVICE, QTM_E_STEP as qtm_run. */
#define QTM_NOALLOC_SCRATCH_MB 32
int qtm_run_range_noalloc(qtm_ctx* ctx, int64_t traj_begin, int64_t count, uint64_t seed, double* sum,
                          double* sumsq);

/* ---------------------------------------------------- learned proposal */
/* The proposal network maps 16 segment-start features to (log h0, log tau_lo,
 * log tau_hi): features are 12 diagonal-observable expectations (the f_ops
 * given to qtm_set_proposal), <C_0^dag C_0>, <C_1^dag C_1>, log r and the
 * elapsed fraction of the time span; architecture 16 -> 64 -> 64 -> 3 with
 * GELU, BF16 weights and FP32 accumulation.  The proposed h0 is snapped to the
 * grid 2^(k/4) and replaces the starting-step rule; the exact root finding of
 * the jump time is unchanged. */
#define QTM_MLP_NPARAM 5443   /* trainable parameters (W1,b1,W2,b2,W3,b3) */
#define QTM_MLP_NTOTAL 5475   /* + input mean[16] and scale[16] */

/* Installs proposal weights (FP32 masters, QTM_MLP_NTOTAL values, host) and
 * the feature operators (n_f <= 12 diagonal operators). */
int qtm_set_proposal(qtm_ctx* ctx, const float* params, int32_t n_params, const qtm_op* f_ops, int32_t n_f);

/* Copies the current proposal weights (FP32 masters) to params (host). */
int qtm_get_proposal(const qtm_ctx* ctx, float* params, int32_t n_params);

/* Segment records of the last run (requires seg_cap > 0): [count][seg_cap][20]
 * floats = 16 features, realised jump delay tau, the controller's step after the
 * first accepted step, censored flag, valid flag. */
int qtm_segments(const qtm_ctx* ctx, float* out);

/* Trains the proposal on the device with the library's forward/backward/Adam
 * kernels.  feat [n][16], tgt [n][3] (log h*, log tau, censored flag) are host
 * FP32 arrays; the loss is the mean of (o0 - log h*)^2 plus, for uncensored
 * samples, the pinball losses at quantiles 0.05 and 0.95 of log tau.  Writes the
 * mean loss of each epoch to loss_out (nullable, n_epochs values). */
int qtm_train_proposal(qtm_ctx* ctx, const float* feat, const float* tgt, int64_t n, int32_t n_epochs,
                       int32_t batch, float lr, uint64_t shuffle_seed, float* loss_out);

/* Loss and gradient of the proposal on one batch with the current weights,
 * computed by the device forward and backward kernels (BF16 weights, FP32
 * activations): grad receives QTM_MLP_NPARAM floats (host). */
int qtm_proposal_grad(qtm_ctx* ctx, const float* feat, const float* tgt, int64_t n, float* loss, float* grad);

/* Team sizes (wavefronts per 16-trajectory team) the small dense kernel offers
 * for dimension d, written to waves[0..return-1] (at most cap); the first one
 * is the default.  Used by autotuners; returns 0 when d > 64.  Not a status. */
int qtm_tile_candidates(int32_t d, int32_t* waves, int32_t cap);

/* Team sizes (wavefronts per 16-trajectory team) the batched tile-class launch offers for
 * class cls (0, 1, 2: dense systems with d <= 64, 128, 256), written to waves[0..return-1]
 * (at most cap); the first is the default.  For autotuners; not a status. */
int qtm_batch_tile_candidates(int32_t cls, int32_t* waves, int32_t cap);

/* ----------------------------------------------------------- misc */
/* Message of the last failing call in this thread ("" if none).  Not an int. */
const char* qtm_last_error(void);

/* Frees every device and host resource of the context.  Not an int; NULL is a no-op. */
void qtm_destroy(qtm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* QTM_H */
