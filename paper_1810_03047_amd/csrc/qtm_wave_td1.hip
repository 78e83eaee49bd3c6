// Instances of the team trajectory kernel with time-dependent Hamiltonian terms, default
// team shape of every tile count, FP32 products.
#define QTM_WAVE_INSTANCES
#include "qtm_wave.hip"

namespace qtm {
template <int T, int NWT, int PREC> const void* team_fn_td_inst();
template <> const void* team_fn_td_inst<1, 1, 1>() { return (const void*)&traj_team_kernel<1, 1, 1, 0, true>; }
template <> const void* team_fn_td_inst<2, 1, 1>() { return (const void*)&traj_team_kernel<2, 1, 1, 0, true>; }
template <> const void* team_fn_td_inst<3, 1, 1>() { return (const void*)&traj_team_kernel<3, 1, 1, 0, true>; }
template <> const void* team_fn_td_inst<4, 1, 1>() { return (const void*)&traj_team_kernel<4, 1, 1, 0, true>; }
template <> const void* team_fn_td_inst<5, 1, 1>() { return (const void*)&traj_team_kernel<5, 1, 1, 0, true>; }
template <> const void* team_fn_td_inst<3, 2, 1>() { return (const void*)&traj_team_kernel<3, 2, 1, 0, true>; }
template <> const void* team_fn_td_inst<4, 2, 1>() { return (const void*)&traj_team_kernel<4, 2, 1, 0, true>; }
template <> const void* team_fn_td_inst<2, 4, 1>() { return (const void*)&traj_team_kernel<2, 4, 1, 0, true>; }
}  // namespace qtm
