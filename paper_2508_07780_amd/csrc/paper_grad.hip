// Paper-formula gradient variant.  eq. gradeps writes the div-div part of g_eps as the time
// integral of div(lambda) div(E), having replaced div(eps~ E) by eps~ div(E).  On the
// discrete scheme, with lumped P1 weights (the integral of phi_i over K is |K|/4), that is
//     P_i = sum_k sum_{K ∋ i} (|K| / 4) div_K(lambda^k) div_K(E^k),
// while the exact derivative of the scheme (the nodal product (eps - 1) E inside the
// divergence) has
//     Q_i = sum_k sum_{K ∋ i} |K| div_K(lambda^k) (grad phi_i|_K . E^k_i).
// The solver's adjoint accumulates the exact gradient; with the variant on, these kernels
// add P_i - Q_i per adjoint step, so that the variant is the exact gradient plus that sum.
// The kernel adds any weighted pair wp P_i - wx Q_i of one level's terms: (1, 1) for the
// variant, (1, 0) for the paper term alone, (0, -1) for the exact term alone (the level-0
// row of a solve that starts from initial data, which the adjoint steps do not visit).
//
// The per-tile arithmetic (geometry of the Kuhn split, the tile and its staging) is
// pg_tile in pg_tile.hpp, shared with the fused adjoint step of the form R2.
#include "paper_grad.hpp"
#include "pg_tile.hpp"

namespace dd {

namespace {

__global__ void invert_own_kernel(const int* __restrict__ own_api, int64_t n_own, int* __restrict__ api_own) {
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < n_own; id += (int64_t)gridDim.x * blockDim.x)
    api_own[own_api[id]] = (int)id;
}

__global__ void fill_i32_kernel(int* p, int64_t n, int v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ __launch_bounds__(256) void pg_step_kernel(PgArgs g) { pg_tile(g, blockIdx.x); }

__global__ void add_free_kernel(const double* __restrict__ acc, int fsx, int fsy, int fsz, double* __restrict__ out) {
  const int64_t n = (int64_t)fsx * fsy * fsz;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int lx = (int)(i % fsx), ly = (int)((i / fsx) % fsy), lz = (int)(i / ((int64_t)fsx * fsy));
    const int lay = min(min(min(lx, fsx - 1 - lx), min(ly, fsy - 1 - ly)), min(lz, fsz - 1 - lz));
    if (lay >= 2) out[i] += acc[i];
  }
}

int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

}  // namespace

void launch_invert_own(const int* own_api, int64_t n_own, int64_t n_fem, int* api_own, hipStream_t s) {
  hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks_for(n_fem)), dim3(256), 0, s, api_own, n_fem, -1);
  if (n_own > 0) hipLaunchKernelGGL(invert_own_kernel, dim3(blocks_for(n_own)), dim3(256), 0, s, own_api, n_own, api_own);
}

void launch_divdiv_grad_terms(const float* lam, const float* E, int64_t n_own, const int* api_own, const int fs[3],
                              double h, double wp, double wx, double* acc, hipStream_t s) {
  const int tiles = pg_tiles(fs);
  if (!tiles) return;   // no free node
  PgArgs g;
  g.lam = lam; g.E = E; g.n_own = n_own; g.api_own = api_own;
  for (int c = 0; c < 3; ++c) g.fs[c] = fs[c];
  g.h = h; g.wp = wp; g.wx = wx; g.acc = acc;
  hipLaunchKernelGGL(pg_step_kernel, dim3(tiles), dim3(256), PG_LDS_BYTES, s, g);
}

void launch_paper_grad_step(const float* lam, const float* E, int64_t n_own, const int* api_own, const int fs[3],
                            double h, bool sub_exact, double* acc, hipStream_t s) {
  launch_divdiv_grad_terms(lam, E, n_own, api_own, fs, h, 1.0, sub_exact ? 1.0 : 0.0, acc, s);
}

void launch_add_free(const double* acc, const int fs[3], double* out_eps, hipStream_t s) {
  const int64_t n = (int64_t)fs[0] * fs[1] * fs[2];
  hipLaunchKernelGGL(add_free_kernel, dim3(blocks_for(n)), dim3(256), 0, s, acc, fs[0], fs[1], fs[2], out_eps);
}

}  // namespace dd
