// Tile-class launches of the team kernel for a batch of dense systems (operator
// A-fragments in global memory), teams of 4 waves with 2, 4 or 8 row tiles per wave
// (d <= 64, 128, 256), FP64 and FP32 products.
#define QTM_WAVE_INSTANCES
#include "qtm_wave.hip"

namespace qtm {

int team_batch_class(int d) {
    const int dp = (d + 7) / 8 * 8, rt = 2 * dp / 16;
    return rt <= 8 ? 0 : rt <= 16 ? 1 : rt <= 32 ? 2 : -1;
}
// class 2 (eight row tiles per wave) spills part of its state, and still runs the
// d <= 256 systems faster than the SpMM kernel (C4 with FP32 products: 0.49 s against 0.62 s)

int launch_team_batch(const RunArgs& a, int max_d, int max_ne, int prec, hipStream_t st, LaunchInfo* info) {
    const int cls = team_batch_class(max_d);
    if (cls < 0 || a.n_sys < 1) return -1;
    const int T = cls == 0 ? 2 : cls == 1 ? 4 : 8, nwt = 4;
    const int dpmax = (max_d + 7) / 8 * 8;
    const void* fn = nullptr;
    if (cls == 0) fn = prec == 0 ? (const void*)&traj_team_batch_kernel<2, 4, 0> : (const void*)&traj_team_batch_kernel<2, 4, 1>;
    if (cls == 1) fn = prec == 0 ? (const void*)&traj_team_batch_kernel<4, 4, 0> : (const void*)&traj_team_batch_kernel<4, 4, 1>;
    if (cls == 2) fn = prec == 0 ? (const void*)&traj_team_batch_kernel<8, 4, 0> : (const void*)&traj_team_batch_kernel<8, 4, 1>;
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
