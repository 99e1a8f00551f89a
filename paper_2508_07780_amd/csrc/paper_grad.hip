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
// Geometry of the Kuhn split: the cell with lower corner c (spacing h) holds one
// tetrahedron per axis permutation (a, b, c): v0 = c, v1 = v0 + e_a, v2 = v1 + e_b,
// v3 = v2 + e_c.  Its barycentric functions are 1 - x_a, x_a - x_b, x_b - x_c, x_c (local
// coordinates in units of h), so h grad phi = -e_a, e_a - e_b, e_b - e_c, e_c, |K| = h^3/6 and
//     h div_K(u) = (u1 - u0)_a + (u2 - u1)_b + (u3 - u2)_c.
// With dl = h div_K(lambda), de = h div_K(E), g = h grad phi_i:
//     (|K|/4) div lambda div E - |K| div lambda (grad phi_i . E_i) = (h / 24) dl (de - 4 g.E_i).
// A free node (layer >= 2) only touches cells whose corners are all FEM-owned, so lambda
// needs no restriction and only those interior cells are visited.
//
// One launch per adjoint step: a block takes an 8 x 8 x 4 tile of free nodes, stages
// lambda^k and E^k of the 10 x 10 x 6 nodes around it in LDS, computes (dl, de) of the six
// tetrahedra of the 9 x 9 x 5 cells the tile touches into LDS, and each thread then gathers
// its node's 24 tetrahedra over the 8 cells around it and adds to an FP64 accumulator: no
// atomics, a fixed order.
#include "paper_grad.hpp"

namespace dd {

namespace {

// axis permutations (a, b, c) of the six tetrahedra
__constant__ int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

__global__ void invert_own_kernel(const int* __restrict__ own_api, int64_t n_own, int* __restrict__ api_own) {
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < n_own; id += (int64_t)gridDim.x * blockDim.x)
    api_own[own_api[id]] = (int)id;
}

__global__ void fill_i32_kernel(int* p, int64_t n, int v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

constexpr int PG_TX = 8, PG_TY = 8, PG_TZ = 4;                 // free nodes per block
constexpr int PG_NX = PG_TX + 2, PG_NY = PG_TY + 2, PG_NZ = PG_TZ + 2;  // staged nodes
constexpr int PG_CX = PG_TX + 1, PG_CY = PG_TY + 1, PG_CZ = PG_TZ + 1;  // cells touched

__global__ __launch_bounds__(256) void pg_step_kernel(const float* __restrict__ lam, const float* __restrict__ E,
                                                      int64_t n_own, const int* __restrict__ api_own, int fsx,
                                                      int fsy, int fsz, double h, double wp, double wx,
                                                      double* __restrict__ acc) {
  __shared__ float sl[3][PG_NZ][PG_NY][PG_NX];
  __shared__ float se[3][PG_NZ][PG_NY][PG_NX];
  __shared__ float2 sc[6][PG_CZ][PG_CY][PG_CX];
  // free nodes: lattice coordinates 2 .. fs - 3 per axis
  const int nfx = fsx - 4, nfy = fsy - 4, nfz = fsz - 4;
  const int tbx = (nfx + PG_TX - 1) / PG_TX, tby = (nfy + PG_TY - 1) / PG_TY;
  const int b = blockIdx.x;
  const int x0 = 2 + (b % tbx) * PG_TX, y0 = 2 + ((b / tbx) % tby) * PG_TY, z0 = 2 + (b / (tbx * tby)) * PG_TZ;
  const int t = threadIdx.x;
  // stage nodes x0-1 .. x0+TX (clamped to the last owned node; values past it are unused)
  for (int i = t; i < PG_NX * PG_NY * PG_NZ; i += 256) {
    const int ix = i % PG_NX, iy = (i / PG_NX) % PG_NY, iz = i / (PG_NX * PG_NY);
    const int gx = min(x0 - 1 + ix, fsx - 2), gy = min(y0 - 1 + iy, fsy - 2), gz = min(z0 - 1 + iz, fsz - 2);
    const int64_t id = api_own[(int64_t)gx + fsx * ((int64_t)gy + (int64_t)fsy * gz)];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sl[c][iz][iy][ix] = lam[c * n_own + id];
      se[c][iz][iy][ix] = E[c * n_own + id];
    }
  }
  __syncthreads();
  // cells with lower corner x0-1+cx ...: corner (cx + ox) in the staged box
  for (int i = t; i < PG_CX * PG_CY * PG_CZ; i += 256) {
    const int cx = i % PG_CX, cy = (i / PG_CX) % PG_CY, cz = i / (PG_CX * PG_CY);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int a = kPerm[k][0], bb = kPerm[k][1], c = kPerm[k][2];
      const int v1 = 1 << a, v2 = v1 | (1 << bb);
#define PG_AT(arr, comp, o) arr[comp][cz + ((o) >> 2)][cy + (((o) >> 1) & 1)][cx + ((o) & 1)]
      const float dl = (PG_AT(sl, a, v1) - PG_AT(sl, a, 0)) + (PG_AT(sl, bb, v2) - PG_AT(sl, bb, v1)) +
                       (PG_AT(sl, c, 7) - PG_AT(sl, c, v2));
      const float de = (PG_AT(se, a, v1) - PG_AT(se, a, 0)) + (PG_AT(se, bb, v2) - PG_AT(se, bb, v1)) +
                       (PG_AT(se, c, 7) - PG_AT(se, c, v2));
#undef PG_AT
      sc[k][cz][cy][cx] = make_float2(dl, de);
    }
  }
  __syncthreads();
  const int tx = t % PG_TX, ty = (t / PG_TX) % PG_TY, tz = t / (PG_TX * PG_TY);
  const int lx = x0 + tx, ly = y0 + ty, lz = z0 + tz;
  if (lx > fsx - 3 || ly > fsy - 3 || lz > fsz - 3) return;
  const float Ei[3] = {se[0][tz + 1][ty + 1][tx + 1], se[1][tz + 1][ty + 1][tx + 1], se[2][tz + 1][ty + 1][tx + 1]};
  double s = 0.0;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    // the cell whose corner o is this node: staged cell (tx + 1 - ox, ...)
    const int cx = tx + 1 - (o & 1), cy = ty + 1 - ((o >> 1) & 1), cz = tz + 1 - (o >> 2);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int a = kPerm[k][0], bb = kPerm[k][1], c = kPerm[k][2];
      const int v1 = 1 << a, v2 = v1 | (1 << bb);
      float gE;   // h grad phi . E_i for the vertex this node is
      if (o == 0) gE = -Ei[a];
      else if (o == v1) gE = Ei[a] - Ei[bb];
      else if (o == v2) gE = Ei[bb] - Ei[c];
      else if (o == 7) gE = Ei[c];
      else continue;
      const float2 v = sc[k][cz][cy][cx];
      s += (double)v.x * (wp * (double)v.y - wx * 4.0 * (double)gE);
    }
  }
  acc[(int64_t)lx + fsx * ((int64_t)ly + (int64_t)fsy * lz)] += s * (h / 24.0);
}

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
  if (fs[0] < 5 || fs[1] < 5 || fs[2] < 5) return;   // no free node
  const int tbx = (fs[0] - 4 + PG_TX - 1) / PG_TX, tby = (fs[1] - 4 + PG_TY - 1) / PG_TY;
  const int tbz = (fs[2] - 4 + PG_TZ - 1) / PG_TZ;
  hipLaunchKernelGGL(pg_step_kernel, dim3(tbx * tby * tbz), dim3(256), 0, s, lam, E, n_own, api_own, fs[0], fs[1],
                     fs[2], h, wp, wx, acc);
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
