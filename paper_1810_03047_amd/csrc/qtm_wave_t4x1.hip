// Instances of the team trajectory kernel: 4 row tile(s) per wave, 1 wave(s) per team.
#define QTM_WAVE_INSTANCES
#include "qtm_wave.hip"

namespace qtm {
template <int T, int NWT, int PREC> const void* team_fn_inst();
template <> const void* team_fn_inst<4, 1, 0>() { return (const void*)&traj_team_kernel<4, 1, 0>; }
template <> const void* team_fn_inst<4, 1, 1>() { return (const void*)&traj_team_kernel<4, 1, 1>; }
// banded operators (nonzero tiles within one tile of the diagonal)
template <int T, int PREC> const void* team_fn_band_inst();
template <> const void* team_fn_band_inst<4, 0>() { return (const void*)&traj_team_kernel<4, 1, 0, 1>; }
template <> const void* team_fn_band_inst<4, 1>() { return (const void*)&traj_team_kernel<4, 1, 1, 1>; }
}  // namespace qtm
