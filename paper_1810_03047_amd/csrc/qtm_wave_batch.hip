// Tile-class launches of the team kernel for a batch of dense systems (operator
// A-fragments in global memory): one persistent launch per class of d (<= 64, 128,
// 256 -- 8, 16 or 32 row tiles of the real embedding), each with a team shape the
// autotuner picks among those offered for the class, FP64 and FP32 products.
#define QTM_WAVE_INSTANCES
#include "qtm_wave.hip"

namespace qtm {

int team_batch_class(int d) {
    const int dp = (d + 7) / 8 * 8, rt = 2 * dp / 16;
    return rt <= 8 ? 0 : rt <= 16 ? 1 : rt <= 32 ? 2 : -1;
}

// Team shapes offered per tile class (row tiles per wave x waves per team, covering 8, 16
// or 32 row tiles); the first is the default.  Eight row tiles per wave (class 2's first
// shape in earlier versions) spill part of the state; four tiles per wave do not.
static const int kBatchShapes[3][3][2] = {
    {{2, 4}, {1, 8}, {0, 0}},
    {{4, 4}, {2, 8}, {0, 0}},
    {{4, 8}, {8, 4}, {2, 16}},
};

int team_batch_candidates(int cls, int* waves, int cap) {
    if (cls < 0 || cls > 2) return 0;
    int n = 0;
    for (int i = 0; i < 3 && n < cap; ++i)
        if (kBatchShapes[cls][i][0]) waves[n++] = kBatchShapes[cls][i][1];
    return n;
}

template <int T, int NWT> static const void* batch_fn(int prec) {
    return prec == 0 ? (const void*)&traj_team_batch_kernel<T, NWT, 0> : (const void*)&traj_team_batch_kernel<T, NWT, 1>;
}

int launch_team_batch(const RunArgs& a, int max_d, int max_ne, int prec, int waves, hipStream_t st, LaunchInfo* info) {
    const int cls = team_batch_class(max_d);
    if (cls < 0 || a.n_sys < 1) return -1;
    int T = 0, nwt = 0;
    for (int i = 0; i < 3; ++i) {
        const int tt = kBatchShapes[cls][i][0], nn = kBatchShapes[cls][i][1];
        if (tt && (waves == 0 || waves == nn)) { T = tt; nwt = nn; break; }
    }
    if (!T) return -1;
    const int dpmax = (max_d + 7) / 8 * 8;
    const void* fn = nullptr;
    if (T == 2 && nwt == 4) fn = batch_fn<2, 4>(prec);
    if (T == 1 && nwt == 8) fn = batch_fn<1, 8>(prec);
    if (T == 4 && nwt == 4) fn = batch_fn<4, 4>(prec);
    if (T == 2 && nwt == 8) fn = batch_fn<2, 8>(prec);
    if (T == 4 && nwt == 8) fn = batch_fn<4, 8>(prec);
    if (T == 8 && nwt == 4) fn = batch_fn<8, 4>(prec);
    if (T == 2 && nwt == 16) fn = batch_fn<2, 16>(prec);
    if (!fn) return -1;
    const TeamLds L = team_lds_batch(dpmax, max_d, max_ne, nwt);
    if (L.total > 160 * 1024) return -2;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total) != hipSuccess) return -3;
    int dev = 0, ncu = 0, nb = 1;
    const int threads = 64 * nwt;
    if (hipGetDevice(&dev) != hipSuccess) return -3;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -3;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, L.total) != hipSuccess || nb < 1) nb = 1;
    long long blocks = (long long)ncu * nb;
    int dpm = dpmax, dm = max_d, nem = max_ne;
    RunArgs aa = a;
    void* args[] = {(void*)&aa, (void*)&dpm, (void*)&dm, (void*)&nem};
    if (hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(threads), args, L.total, st) != hipSuccess) return -3;
    if (info) { info->blocks = (int)blocks; info->threads = threads; info->lds = (int)L.total; info->cols = 16; info->shape = T * 100 + nwt; }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace qtm
