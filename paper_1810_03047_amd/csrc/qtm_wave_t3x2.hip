// Instances of the team trajectory kernel: 3 row tile(s) per wave, 2 wave(s) per team.
#define QTM_WAVE_INSTANCES
#include "qtm_wave.hip"

namespace qtm {
template <int T, int NWT, int PREC> const void* team_fn_inst();
template <> const void* team_fn_inst<3, 2, 0>() { return (const void*)&traj_team_kernel<3, 2, 0>; }
template <> const void* team_fn_inst<3, 2, 1>() { return (const void*)&traj_team_kernel<3, 2, 1>; }
}  // namespace qtm
