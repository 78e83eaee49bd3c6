// qtm_dense.hip -- trajectory kernel for dense H_eff: the product K = M W of a
// 16-column block is a real-embedded GEMM on the FP64 or FP32 matrix cores with
// the operand block staged in LDS; plus the index-ordered averaging kernel.
#include "qtm_body.h"

namespace qtm {

template <int T, int PREC>
__global__ void __launch_bounds__(512) traj_dense_kernel(RunArgs a, int lds_m) {
    extern __shared__ __attribute__((aligned(16))) double smem[];   // 16-byte base: double2 staging
    __shared__ int flags[8];
    typedef typename MfmaT<PREC>::in_t in_t;
    const DevSystem& S = a.sys[0];
    DenseLayout<T, PREC> L;
    L.S = &S;
    L.lane = threadIdx.x & 63; L.w = threadIdx.x >> 6; L.lg = L.lane >> 4; L.c16 = L.lane & 15;
    const int NW = blockDim.x >> 6;
    L.RT = S.rt; L.dp = S.dp; L.d = S.d; L.KB = 2 * S.dp / 4;
    L.wpc = (L.RT + T - 1) / T;
    L.nct = a.tile_cols / 16;                 // set by the launcher; NW == wpc * nct
    L.NB = 16 * L.nct;
    L.ct = L.w / L.wpc; L.rg = L.w % L.wpc;
    L.active = L.ct < L.nct;
    // LDS carve-up: [column states][M fragments if lds_m][W staging][reduction]
    char* p = (char*)smem;
    Col* cs = (Col*)p;
    p += ((size_t)L.NB * sizeof(Col) + 15) & ~(size_t)15;
    size_t msz = (size_t)(2 * S.dp) * (2 * S.dp) * sizeof(in_t);
    if (lds_m) {
        in_t* Ml = (in_t*)p;
        const in_t* Mg = MfmaT<PREC>::frag(S);
        for (size_t i = threadIdx.x; i < msz / sizeof(in_t); i += blockDim.x) Ml[i] = Mg[i];
        L.Mf = Ml;
        p += (msz + 15) & ~(size_t)15;
    } else {
        L.Mf = MfmaT<PREC>::frag(S);
    }
    size_t wsz = (size_t)L.nct * 2 * S.dp * 16 * sizeof(double);   // also holds [dp][NB] double2
    L.Wb = (in_t*)p;
    L.Stage = (double2*)p;
    p += wsz;
    L.red = (double*)p;
    __syncthreads();
    Body<DenseLayout<T, PREC>> B(L, S, a, cs, flags);
    B.run();
    if (threadIdx.x == 0) atomicAdd(&a.counters[0], B.passes);
    if (B.roots) atomicAdd(&a.counters[1], B.roots);
}

// Trajectory average in a fixed order (independent of scheduling): chunk c of
// the trajectories is summed in index order by one thread per (observable,
// time) point, then the chunks are summed in chunk order.  part = [3][nchunk][m].
__global__ void average_partial_kernel(const double2* X, long long count, int m, int nchunk, long long per,
                                       double* part) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= m) return;
    const long long q0 = (long long)c * per;
    const long long q1 = q0 + per < count ? q0 + per : count;
    double sr = 0.0, si = 0.0, s2 = 0.0;
    // unrolled: the loads of eight trajectories are issued ahead of their additions, which
    // keep trajectory order
#pragma unroll 8
    for (long long q = q0; q < q1; ++q) {
        const double2 x = X[q * m + i];
        sr += x.x; si += x.y; s2 += x.x * x.x;
    }
    part[((size_t)0 * nchunk + c) * m + i] = sr;
    part[((size_t)1 * nchunk + c) * m + i] = si;
    part[((size_t)2 * nchunk + c) * m + i] = s2;
}

__global__ void average_final_kernel(const double* part, int nchunk, int m, double* sum, double* sumsq) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double sr = 0.0, si = 0.0, s2 = 0.0;
#pragma unroll 8
    for (int c = 0; c < nchunk; ++c) {
        sr += part[((size_t)0 * nchunk + c) * m + i];
        si += part[((size_t)1 * nchunk + c) * m + i];
        s2 += part[((size_t)2 * nchunk + c) * m + i];
    }
    sum[2 * i] = sr; sum[2 * i + 1] = si; sumsq[i] = s2;
}

static int average_chunks(int m, long long count) {
    long long n = (65536 + m - 1) / m;           // about 64k threads in the first pass
    if (n > 256) n = 256;
    if (n > count) n = count;
    return n < 1 ? 1 : (int)n;
}

// ------------------------------------------------------------------ host launchers
static size_t dense_lds(int max_dp, int prec, int waves, int lds_m, int nct) {
    size_t es = prec == 0 ? 8 : 4;
    size_t cols = (((size_t)16 * nct * sizeof(Col)) + 15) & ~(size_t)15;
    size_t m = lds_m ? (((size_t)(2 * max_dp) * (2 * max_dp) * es + 15) & ~(size_t)15) : 0;
    size_t wsz = (size_t)nct * 2 * max_dp * 16 * sizeof(double);
    size_t red = (size_t)waves * 16 * kNVMax * sizeof(double);
    return cols + m + wsz + red;
}

template <int T, int PREC> static const void* dense_fn() { return (const void*)&traj_dense_kernel<T, PREC>; }

// Block geometry of the dense kernel for dimension d: T row tiles per wave,
// wpc waves per 16-column tile, nct column tiles (at most 8 waves per block).
static int dense_geometry(int d, int tile_cols, int* T, int* wpc, int* nct, int* dp) {
    *dp = (d + 7) / 8 * 8;
    int rt = 2 * *dp / 16;
    if (rt > 16) return -1;
    *T = rt <= 8 ? 1 : 2;
    *wpc = (rt + *T - 1) / *T;
    int maxct = 8 / *wpc;
    int want = tile_cols > 0 ? tile_cols / 16 : 1;
    *nct = std::max(1, std::min(maxct, want));
    return 0;
}

static const void* dense_kernel_fn(int T, int prec) {
    return T == 1 ? (prec == 0 ? dense_fn<1, 0>() : dense_fn<1, 1>()) : (prec == 0 ? dense_fn<2, 0>() : dense_fn<2, 1>());
}

int dense_occupancy(int max_d, int prec, int tile_cols, int* blocks_per_cu, int* lds) {
    int T, wpc, nct, dp;
    if (dense_geometry(max_d, tile_cols, &T, &wpc, &nct, &dp)) return -1;
    size_t es = prec == 0 ? 8 : 4;
    int lds_m = (size_t)(2 * dp) * (2 * dp) * es <= 56 * 1024;
    int waves = wpc * nct;
    size_t l = dense_lds(dp, prec, waves, lds_m, nct);
    const void* fn = dense_kernel_fn(T, prec);
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l) != hipSuccess) return -2;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, waves * 64, l) != hipSuccess) return -2;
    *blocks_per_cu = nb;
    *lds = (int)l;
    return 0;
}

int launch_dense(const RunArgs& a, const DevSystem& s0, int max_d, int prec, int blocks_per_cu,
                 hipStream_t st, LaunchInfo* info) {
    int T, wpc, nct, dp;
    if (dense_geometry(max_d, a.tile_cols, &T, &wpc, &nct, &dp)) return -1;
    int waves = wpc * nct;
    size_t es = prec == 0 ? 8 : 4;
    int lds_m = (size_t)(2 * dp) * (2 * dp) * es <= 56 * 1024;
    size_t lds = dense_lds(dp, prec, waves, lds_m, nct);
    int cols = 16 * nct;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -3;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -3;
    long long need = (s0.count + cols - 1) / cols;
    long long blocks = a.persistent ? (long long)ncu * (blocks_per_cu > 0 ? blocks_per_cu : 1) : need;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    const void* fn = dense_kernel_fn(T, prec);
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return -3;
    RunArgs aa = a;
    aa.tile_cols = cols;
    int lm = lds_m;
    void* args[] = {(void*)&aa, (void*)&lm};
    if (hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(waves * 64), args, lds, st) != hipSuccess) return -3;
    if (info) { info->blocks = (int)blocks; info->threads = waves * 64; info->lds = (int)lds; info->cols = cols; }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// Fills n 8-byte words with v.  Used instead of hipMemsetAsync so that a run can be
// captured into a graph.
__global__ void fill_words_kernel(unsigned long long* p, long long n, unsigned long long v) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// The fills of a FillSet in one launch: the grid strides over each buffer in turn.
__global__ void fill_set_kernel(FillSet f) {
    const long long stride = (long long)gridDim.x * blockDim.x, t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (int j = 0; j < f.count; ++j) {
        unsigned long long* p = f.p[j];
        const unsigned long long v = f.v[j];
        for (long long i = t; i < f.n[j]; i += stride) p[i] = v;
    }
}

// Device timestamp (constant-rate wall clock) for timing a stretch of a stream; a
// kernel, unlike an event, can be captured into a graph.
__global__ void stamp_kernel(unsigned long long* t) { t[0] = wall_clock64(); }

int launch_stamp(unsigned long long* t, hipStream_t st) {
    hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(1), 0, st, t);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_fill(void* p, size_t bytes, unsigned long long v, hipStream_t st) {
    if (bytes % 8 != 0) return -1;
    const long long n = (long long)(bytes / 8);
    if (n == 0) return 0;
    long long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_words_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (unsigned long long*)p, n, v);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_fills(const FillSet& f, hipStream_t st) {
    long long nmax = 0;
    for (int j = 0; j < f.count; ++j) nmax = f.n[j] > nmax ? f.n[j] : nmax;
    if (f.count < 1 || f.count > kFillSet || nmax == 0) return f.count == 0 || nmax == 0 ? 0 : -1;
    long long blocks = (nmax + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_set_kernel, dim3((unsigned)blocks), dim3(256), 0, st, f);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

size_t average_part_size(int m, long long count) { return (size_t)3 * average_chunks(m, count) * m; }

int launch_average(const DevSystem& s, double* part, double* sum, double* sumsq, hipStream_t st) {
    const int m = s.n_e * s.n_t;
    const int nchunk = average_chunks(m, s.count);
    const long long per = (s.count + nchunk - 1) / nchunk;
    hipLaunchKernelGGL(average_partial_kernel, dim3((m + 255) / 256, nchunk), dim3(256), 0, st, (const double2*)s.X,
                       s.count, m, nchunk, per, part);
    hipLaunchKernelGGL(average_final_kernel, dim3((m + 255) / 256), dim3(256), 0, st, (const double*)part, nchunk, m,
                       sum, sumsq);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace qtm
