// qtm_sparse.hip -- trajectory kernel for sparse H_eff: sliced-ELL SpMM, each thread
// owns RPT state components (rows) of the block's NBC trajectories, the column block
// staged in LDS.  Blocks of 256 threads: the register file then holds the state
// without spilling (a 1024-thread block would cap every lane at 128 registers).
#include "qtm_body.h"

namespace qtm {

constexpr int kSparseThreads = 256;

// One launch can serve several systems (a batch of mixed dimension): a block
// takes the first system whose trajectory queue is not exhausted, runs it with
// slot refill until its queue runs dry, then moves on.  a.sys_cursor records the
// first system that may still have work, so finished systems are skipped.
template <int RPT, int NBC, int PREC>
__global__ void __launch_bounds__(kSparseThreads) traj_sparse_kernel(RunArgs a) {
    extern __shared__ double smem[];
    __shared__ int flags[8];
    __shared__ int cur;
    unsigned long long passes = 0;
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
        const DevSystem& S = a.sys[si];
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
        Body<SparseLayout<RPT, NBC, PREC>> B(L, S, a, cs, flags);
        B.run();
        passes += B.passes;
        __syncthreads();                 // the block leaves the system together
        if (a.n_sys <= 1) break;
        ++si;
    }
    if (threadIdx.x == 0) atomicAdd(&a.counters[0], passes);
}

#ifndef QTM_SPARSE_INSTANCES
// instances (rows per thread x trajectories per block, rows x trajectories <= 8) live in
// qtm_sparse_r*.hip so that they compile in parallel
template <int R, int C, int P> const void* sparse_fn_inst();

int launch_sparse(const RunArgs& a, const DevSystem& s0, int max_d, int prec, int cols, hipStream_t st, LaunchInfo* info) {
    const int threads = max_d >= kSparseThreads ? kSparseThreads : ((max_d + 63) / 64) * 64;
    int rpt = (max_d + threads - 1) / threads;
    if (rpt == 3) rpt = 4;
    if (rpt > 4 && rpt <= 8) rpt = 8;
    if (rpt > 8) return -1;
    if (cols != 1 && cols != 2 && cols != 4) cols = 2;
    while (rpt * cols > 8) cols >>= 1;
    size_t lds = (((size_t)cols * sizeof(Col) + 15) & ~(size_t)15) + (size_t)max_d * cols * sizeof(double2) +
                 (size_t)(threads / 64) * cols * kNVMax * sizeof(double);
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -3;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -3;
    const void* fn = nullptr;
#define QTM_SPARSE_CASE(R, C) \
    if (rpt == R && cols == C) fn = prec == 0 ? sparse_fn_inst<R, C, 0>() : sparse_fn_inst<R, C, 1>();
    QTM_SPARSE_CASE(1, 1) QTM_SPARSE_CASE(1, 2) QTM_SPARSE_CASE(1, 4)
    QTM_SPARSE_CASE(2, 1) QTM_SPARSE_CASE(2, 2) QTM_SPARSE_CASE(2, 4)
    QTM_SPARSE_CASE(4, 1) QTM_SPARSE_CASE(4, 2) QTM_SPARSE_CASE(8, 1)
#undef QTM_SPARSE_CASE
    if (!fn) return -1;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return -3;
    int nb = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, lds) != hipSuccess) nb = 1;
    if (nb < 1) nb = 1;
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
