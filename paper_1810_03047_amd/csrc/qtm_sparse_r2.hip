// Instances of the sparse trajectory kernel (rows per thread, trajectories per block): 2x1, 2x2, 2x4, and the wide (512-thread) 2x1, 2x2.
#define QTM_SPARSE_INSTANCES
#include "qtm_sparse.hip"

namespace qtm {
template <int R, int C, int P> const void* sparse_fn_inst();
template <> const void* sparse_fn_inst<2, 1, 0>() { return (const void*)&traj_sparse_kernel<2, 1, 0>; }
template <> const void* sparse_fn_inst<2, 1, 1>() { return (const void*)&traj_sparse_kernel<2, 1, 1>; }
template <> const void* sparse_fn_inst<2, 2, 0>() { return (const void*)&traj_sparse_kernel<2, 2, 0>; }
template <> const void* sparse_fn_inst<2, 2, 1>() { return (const void*)&traj_sparse_kernel<2, 2, 1>; }
template <> const void* sparse_fn_inst<2, 4, 0>() { return (const void*)&traj_sparse_kernel<2, 4, 0>; }
template <> const void* sparse_fn_inst<2, 4, 1>() { return (const void*)&traj_sparse_kernel<2, 4, 1>; }
// wide blocks (512 threads)
template <int R, int C, int P> const void* sparse_fn_wide();
template <> const void* sparse_fn_wide<2, 1, 0>() { return (const void*)&traj_sparse_kernel<2, 1, 0, 512>; }
template <> const void* sparse_fn_wide<2, 1, 1>() { return (const void*)&traj_sparse_kernel<2, 1, 1, 512>; }
template <> const void* sparse_fn_wide<2, 2, 0>() { return (const void*)&traj_sparse_kernel<2, 2, 0, 512>; }
template <> const void* sparse_fn_wide<2, 2, 1>() { return (const void*)&traj_sparse_kernel<2, 2, 1, 512>; }
}  // namespace qtm
