// Instances of the sparse trajectory kernel (rows per thread, trajectories per block): 4x1, 4x2, 8x1.
#define QTM_SPARSE_INSTANCES
#include "qtm_sparse.hip"

namespace qtm {
template <int R, int C, int P> const void* sparse_fn_inst();
template <> const void* sparse_fn_inst<4, 1, 0>() { return (const void*)&traj_sparse_kernel<4, 1, 0>; }
template <> const void* sparse_fn_inst<4, 1, 1>() { return (const void*)&traj_sparse_kernel<4, 1, 1>; }
template <> const void* sparse_fn_inst<4, 2, 0>() { return (const void*)&traj_sparse_kernel<4, 2, 0>; }
template <> const void* sparse_fn_inst<4, 2, 1>() { return (const void*)&traj_sparse_kernel<4, 2, 1>; }
template <> const void* sparse_fn_inst<8, 1, 0>() { return (const void*)&traj_sparse_kernel<8, 1, 0>; }
template <> const void* sparse_fn_inst<8, 1, 1>() { return (const void*)&traj_sparse_kernel<8, 1, 1>; }
}  // namespace qtm
