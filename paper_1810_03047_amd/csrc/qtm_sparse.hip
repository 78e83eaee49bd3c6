// qtm_sparse.hip -- trajectory kernel for sparse H_eff: sliced-ELL SpMM, each thread
// owns RPT state components (rows) of the block's NBC trajectories, the column block
// staged in LDS.  Blocks of 256 threads: the register file then holds the state
// without spilling (a 1024-thread block would cap every lane at 128 registers).  Wide
// blocks of 512 threads with half the rows per thread: two waves per SIMD, which hide
// each other's LDS latency in the SpMM, for the same trajectories per block.
#include "qtm_body.h"

namespace qtm {

constexpr int kSparseThreads = 256;
static_assert(sizeof(DevSystem) % 8 == 0, "the descriptor is copied to LDS in 8-byte words");

// One launch can serve several systems (a batch of mixed dimension): a block
// takes the first system whose trajectory queue is not exhausted, runs it with
// slot refill until its queue runs dry, then moves on.  a.sys_cursor records the
// first system that may still have work, so finished systems are skipped.
template <int RPT, int NBC, int PREC, int NT = kSparseThreads>
__global__ void __launch_bounds__(NT) traj_sparse_kernel(RunArgs a) {
    extern __shared__ __attribute__((aligned(16))) double smem[];   // 16-byte base: double2 staging
    __shared__ int flags[8];
    __shared__ int cur;
    __shared__ DevSystem sys_lds;
    unsigned long long passes = 0;
    unsigned long long roots = 0;
    int si = 0;
    for (;;) {
        if (a.n_sys > 1) {
            if (threadIdx.x == 0) {
                int s2 = max(si, (int)__atomic_load_n(a.sys_cursor, __ATOMIC_RELAXED));
                while (s2 < a.n_sys &&
                       __atomic_load_n(a.sys[s2].queue, __ATOMIC_RELAXED) >= (unsigned long long)a.sys[s2].count) {
                    atomicMax(a.sys_cursor, (unsigned int)(s2 + 1));
                    ++s2;
                }
                cur = s2;
            }
            __syncthreads();
            si = cur;
            if (si >= a.n_sys) break;
        }
        // the system descriptor is read all through the run: a copy in LDS turns every
        // field access into an LDS read instead of a dependent global load
        {
            const unsigned long long* src = (const unsigned long long*)(a.sys + si);
            unsigned long long* dst = (unsigned long long*)&sys_lds;
            for (int i = threadIdx.x; i < (int)(sizeof(DevSystem) / 8); i += blockDim.x) dst[i] = src[i];
        }
        __syncthreads();
        const DevSystem& S = sys_lds;
        SparseLayout<RPT, NBC, PREC> L;
        L.S = &S;
        L.tid = threadIdx.x; L.nthr = blockDim.x; L.lane = threadIdx.x & 63; L.w = threadIdx.x >> 6;
        L.NW = blockDim.x >> 6; L.d = S.d; L.NB = NBC; L.dp = S.d;
        char* p = (char*)smem;
        Col* cs = (Col*)p;
        p += ((size_t)NBC * sizeof(Col) + 15) & ~(size_t)15;
        size_t ssz = (size_t)S.d * NBC * sizeof(double2);
        L.Stage = (double2*)p;
        L.Stage32 = (float2*)p;
        p += ssz;
        L.red = (double*)p;
        p += (size_t)L.NW * NBC * kNVMax * sizeof(double);
        L.ell_lds = a.ell_lds;
        if (a.ell_lds) {
            // the operator's sliced ELL, resident for the whole system: values, then
            // 16-bit columns, then slice offsets and widths (sized per system; the launch
            // reserves room for the largest)
            const int nsl = (S.d + 63) >> 6;
            const int n = (int)S.ell_n;
            typedef typename std::conditional<PREC == 0, double2, float2>::type v_t;
            v_t* lv = (v_t*)p;
            p += ((size_t)n * sizeof(v_t) + 15) & ~(size_t)15;
            unsigned short* lc = (unsigned short*)p;
            p += ((size_t)n * 2 + 15) & ~(size_t)15;
            int* lo = (int*)p;
            int* lw = lo + nsl + 1;
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                if (PREC == 0) ((double2*)lv)[i] = S.sl_val[i];
                else ((float2*)lv)[i] = S.sl_val32[i];
                lc[i] = (unsigned short)S.sl_col[i];
            }
            for (int i = threadIdx.x; i <= nsl; i += blockDim.x) lo[i] = S.sl_off[i];
            for (int i = threadIdx.x; i < nsl; i += blockDim.x) lw[i] = S.sl_w[i];
            L.lval = (const double2*)lv;
            L.lval32 = (const float2*)lv;
            L.lcol = lc;
            L.lsoff = lo;
            L.lsw = lw;
            __syncthreads();
        }
        Body<SparseLayout<RPT, NBC, PREC>> B(L, S, a, cs, flags);
        B.run();
        passes += B.passes;
        roots += B.roots;
        __syncthreads();                 // the block leaves the system together
        if (a.n_sys <= 1) break;
        ++si;
    }
    if (threadIdx.x == 0) atomicAdd(&a.counters[0], passes);
    if (roots) atomicAdd(&a.counters[1], roots);
}

#ifndef QTM_SPARSE_INSTANCES
// instances (rows per thread x trajectories per block, rows x trajectories <= 8) live in
// qtm_sparse_r*.hip so that they compile in parallel
template <int R, int C, int P> const void* sparse_fn_inst();
template <int R, int C, int P> const void* sparse_fn_wide();

int launch_sparse(const RunArgs& a0, const DevSystem& s0, int max_d, long long max_ell, int prec, int cols,
                  hipStream_t st, LaunchInfo* info) {
    RunArgs a = a0;
    // Block size.  The registers allow one wave per SIMD (four per CU) at up to four rows
    // per thread, so for d <= 512 the block is as small as four rows per thread allow: the
    // same waves per CU in more, smaller blocks, whose barriers and reductions span fewer
    // waves (trilinear d = 512: 38 ms against 54 with 256-thread blocks; Ising d = 256:
    // 40 against 72; dense d = 200: 52 against 72, FP32).  512 < d <= 1024: wide blocks,
    // two rows per thread and at most two trajectories per block, two waves per SIMD
    // (Ising d = 1024, where the ELL in LDS leaves one block per CU: 691 ms against 748
    // in FP32, 1,202 against 1,293 in FP64).  Beyond: 256 threads, up to eight rows.
    // A launch with too few trajectories to occupy the small blocks (about four single-wave
    // blocks per CU) is latency bound: the block grows back towards 256 threads, more
    // threads per trajectory (the per-system launches of a batch's plain form, 500 each).
    const bool wide = max_d > 2 * kSparseThreads && max_d <= 4 * kSparseThreads;
    if (wide && cols > 2) cols = 2;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -3;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -3;
    int threads = wide ? 2 * kSparseThreads
                       : max_d > 2 * kSparseThreads ? kSparseThreads
                                                    : std::max(64, ((max_d + 3) / 4 + 63) / 64 * 64);
    if (!wide && threads < kSparseThreads) {
        const long long total = s0.count * (long long)std::max(1, a.n_sys);
        while (threads < kSparseThreads && total < (long long)ncu * (kSparseThreads / threads) * cols) threads *= 2;
    }
    int rpt = (max_d + threads - 1) / threads;
    if (rpt == 3) rpt = 4;
    if (rpt > 4 && rpt <= 8) rpt = 8;
    if (rpt > 8) return -1;
    if (cols != 1 && cols != 2 && cols != 4) cols = 2;
    while (rpt * cols > 8) cols >>= 1;
    size_t lds = (((size_t)cols * sizeof(Col) + 15) & ~(size_t)15) + (size_t)max_d * cols * sizeof(double2) +
                 (size_t)(threads / 64) * cols * kNVMax * sizeof(double);
    const void* fn = nullptr;
#define QTM_SPARSE_CASE(R, C) \
    if (rpt == R && cols == C) fn = prec == 0 ? sparse_fn_inst<R, C, 0>() : sparse_fn_inst<R, C, 1>();
    QTM_SPARSE_CASE(1, 1) QTM_SPARSE_CASE(1, 2) QTM_SPARSE_CASE(1, 4)
    QTM_SPARSE_CASE(2, 1) QTM_SPARSE_CASE(2, 2) QTM_SPARSE_CASE(2, 4)
    QTM_SPARSE_CASE(4, 1) QTM_SPARSE_CASE(4, 2) QTM_SPARSE_CASE(8, 1)
#undef QTM_SPARSE_CASE
    if (wide) {
        fn = nullptr;
#define QTM_SPARSE_WIDE(R, C) \
    if (rpt == R && cols == C) fn = prec == 0 ? sparse_fn_wide<R, C, 0>() : sparse_fn_wide<R, C, 1>();
        QTM_SPARSE_WIDE(2, 1) QTM_SPARSE_WIDE(2, 2)
#undef QTM_SPARSE_WIDE
    }
    if (!fn) return -1;
    // the sliced ELL joins the LDS when it fits there (16-bit columns) and the block
    // count per CU stays what the registers and the staging allow
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return -3;
    const int nsl = (max_d + 63) / 64;
    const size_t ell = (((size_t)max_ell * (prec == 0 ? 16 : 8) + 15) & ~(size_t)15) + (((size_t)max_ell * 2 + 15) & ~(size_t)15) +
                       (size_t)(2 * nsl + 1) * sizeof(int);
    int nb = 1;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return -3;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, lds) != hipSuccess) nb = 1;
    if (nb < 1) nb = 1;
    a.ell_lds = 0;
    if (max_d <= 65536 && max_ell > 0 && lds + ell <= (size_t)lds_max) {
        int nb2 = 0;
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(lds + ell)) != hipSuccess) return -3;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb2, fn, threads, lds + ell) != hipSuccess) nb2 = 0;
        if (nb2 >= nb) { a.ell_lds = 1; lds += ell; }
    }
    long long need = ((s0.count + cols - 1) / cols) * (a.n_sys > 0 ? a.n_sys : 1);
    long long blocks = a.persistent ? (long long)ncu * nb : need;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    void* args[] = {(void*)&a};
    if (hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(threads), args, lds, st) != hipSuccess) return -3;
    if (info) { info->blocks = (int)blocks; info->threads = threads; info->lds = (int)lds; info->cols = cols; }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
#endif  // QTM_SPARSE_INSTANCES

}  // namespace qtm
