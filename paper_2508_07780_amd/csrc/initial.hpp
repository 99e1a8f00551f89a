// General initial data of the forward problem (eq. forward_initial_cond: E(0) = f_0,
// dE/dt(0) = f_1): launches that write the starting levels and the level-0 gradient rows.
#pragma once

#include "dd_common.hpp"

namespace dd {

// Starting levels on the FD grid from f_0, f_1 ([N][3] node-major, float32): E^0 = f_0 into
// E0 and E^{-1} = f_0 - dt f_1 into Em1 (both [3][N]); the layer-0 values of E^0 into
// iface0 ([3][n_l0], face order of the FEM box's surface).  blo = grid index of the FEM
// box's lower corner node, fs = FEM nodes per axis.
void launch_init_grid(const float* f0, const float* f1, double dt, int nx, int ny, int nz, const int blo[3],
                      const int fs[3], int64_t n_l0, float* E0, float* Em1, float* iface0, hipStream_t s);
// Starting FEM state on the owned nodes: E^0 = f_0 into E0 and V^0 = dt f_1 into V0 (both
// [3][n_own]); the same pair into each non-null ck ([2][3][n_own]: E, then V).
void launch_init_own(const float* f0, const float* f1, double dt, const int* own_api, int64_t n_own, int nx, int ny,
                     const int blo[3], const int fs[3], float* E0, float* V0, float* ck_a, float* ck_b, hipStream_t s);
// The boundary row of the summed-by-parts mass term: g_eps[id] -= m_id lambda^0 . V^0 / dt^2
// on free owned nodes (own_grid < 0); lam0, V0 [3][n_own].
void launch_init_mass_row(const float* lam0, const float* V0, const int* own_grid, const double* mass_d,
                          int64_t n_own, double inv_dt2, double* g_eps, hipStream_t s);

}  // namespace dd
