// General initial data of the forward problem (eq. forward_initial_cond).  The scheme takes
// the two starting levels E^0 = f_0 and E^{-1} = f_0 - dt f_1 (one-sided difference of
// dE/dt at t = 0); the FD grid holds the two levels, the FEM region its level and the
// increment V^0 = E^0 - E^{-1} = dt f_1, and the layer-0 interface history starts with the
// surface values of E^0.  Both levels are independent of eps and sigma, so the exact
// gradient differs from the start from rest only by level-0 rows: the adjoint steps
// accumulate the mass term summed by parts, sum_n (lambda^n - lambda^{n+1}) . V^{n+1}, whose
// boundary row -lambda^0 . V^0 (the discrete -lambda(x, 0) f_1 of eq. gradeps) is added here.
#include <algorithm>

#include "initial.hpp"

namespace dd {

namespace {

int blocks_of(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

__global__ void init_grid_kernel(const float* __restrict__ f0, const float* __restrict__ f1, double dt, int nx,
                                 int ny, int nz, int b0, int b1, int b2, int s0, int s1, int s2, int64_t n_l0,
                                 float* __restrict__ E0, float* __restrict__ Em1, float* __restrict__ iface0) {
  const int64_t N = (int64_t)nx * ny * nz;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < N; g += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(g % nx), y = (int)((g / nx) % ny), z = (int)(g / ((int64_t)nx * ny));
    const int lx = x - b0, ly = y - b1, lz = z - b2;
    int64_t q = -1;
    if (lx >= 0 && lx < s0 && ly >= 0 && ly < s1 && lz >= 0 && lz < s2)
      q = face_lex_index(lx, ly, lz, s0, s1, s2, 63u);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float e = f0[3 * g + c];
      E0[c * N + g] = e;
      Em1[c * N + g] = (float)((double)e - dt * (double)f1[3 * g + c]);
      if (q >= 0) iface0[c * n_l0 + q] = e;
    }
  }
}

__global__ void init_own_kernel(const float* __restrict__ f0, const float* __restrict__ f1, double dt,
                                const int* __restrict__ own_api, int64_t n_own, int nx, int ny, int b0, int b1,
                                int b2, int s0, int s1, float* __restrict__ E0, float* __restrict__ V0,
                                float* __restrict__ ck_a, float* __restrict__ ck_b) {
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < n_own;
       id += (int64_t)gridDim.x * blockDim.x) {
    const int64_t api = own_api[id];
    const int lx = (int)(api % s0), ly = (int)((api / s0) % s1), lz = (int)(api / ((int64_t)s0 * s1));
    const int64_t g = (int64_t)(b0 + lx) + (int64_t)nx * ((int64_t)(b1 + ly) + (int64_t)ny * (b2 + lz));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float e = f0[3 * g + c];
      const float v = (float)(dt * (double)f1[3 * g + c]);
      E0[c * n_own + id] = e;
      V0[c * n_own + id] = v;
      if (ck_a) {
        ck_a[c * n_own + id] = e;
        ck_a[(3 + c) * n_own + id] = v;
      }
      if (ck_b) {
        ck_b[c * n_own + id] = e;
        ck_b[(3 + c) * n_own + id] = v;
      }
    }
  }
}

__global__ void init_mass_row_kernel(const float* __restrict__ lam0, const float* __restrict__ V0,
                                     const int* __restrict__ own_grid, const double* __restrict__ mass_d,
                                     int64_t n_own, double inv_dt2, double* __restrict__ g_eps) {
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < n_own;
       id += (int64_t)gridDim.x * blockDim.x) {
    if (own_grid[id] >= 0) continue;   // layer-1 nodes carry no gradient
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) s += (double)lam0[c * n_own + id] * (double)V0[c * n_own + id];
    g_eps[id] -= mass_d[id] * inv_dt2 * s;
  }
}

}  // namespace

void launch_init_grid(const float* f0, const float* f1, double dt, int nx, int ny, int nz, const int blo[3],
                      const int fs[3], int64_t n_l0, float* E0, float* Em1, float* iface0, hipStream_t s) {
  const int64_t N = (int64_t)nx * ny * nz;
  hipLaunchKernelGGL(init_grid_kernel, dim3(blocks_of(N)), dim3(256), 0, s, f0, f1, dt, nx, ny, nz, blo[0], blo[1],
                     blo[2], fs[0], fs[1], fs[2], n_l0, E0, Em1, iface0);
}

void launch_init_own(const float* f0, const float* f1, double dt, const int* own_api, int64_t n_own, int nx, int ny,
                     const int blo[3], const int fs[3], float* E0, float* V0, float* ck_a, float* ck_b,
                     hipStream_t s) {
  if (n_own <= 0) return;
  hipLaunchKernelGGL(init_own_kernel, dim3(blocks_of(n_own)), dim3(256), 0, s, f0, f1, dt, own_api, n_own, nx, ny,
                     blo[0], blo[1], blo[2], fs[0], fs[1], E0, V0, ck_a, ck_b);
}

void launch_init_mass_row(const float* lam0, const float* V0, const int* own_grid, const double* mass_d,
                          int64_t n_own, double inv_dt2, double* g_eps, hipStream_t s) {
  if (n_own <= 0) return;
  hipLaunchKernelGGL(init_mass_row_kernel, dim3(blocks_of(n_own)), dim3(256), 0, s, lam0, V0, own_grid, mass_d, n_own,
                     inv_dt2, g_eps);
}

}  // namespace dd
