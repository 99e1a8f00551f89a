// Paper-formula gradient variant.  eq. gradeps writes the div-div part of g_eps as the time
// integral of div(lambda) div(E), having replaced div(eps~ E) by eps~ div(E).  On the
// discrete scheme, with lumped P1 weights (the integral of phi_i over K is |K|/4), that is
//     P_i = sum_k sum_{K ∋ i} (|K| / 4) div_K(lambda^k) div_K(E^k),
// while the exact derivative of the scheme (the nodal product (eps - 1) E inside the
// divergence) has
//     Q_i = sum_k sum_{K ∋ i} |K| div_K(lambda^k) (grad phi_i|_K . E^k_i).
// The solver's adjoint accumulates the exact gradient; with the variant on, these kernels
// add P_i - Q_i per adjoint step, so that the variant is the exact gradient plus that sum.
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
// Pass 1 (one thread per interior cell) stores (dl, de) of its six tetrahedra; pass 2 (one
// thread per free node) gathers its 24 tetrahedra over the 8 cells around it and adds to an
// FP64 accumulator: no atomics, a fixed order.
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

__global__ __launch_bounds__(256) void pg_cell_kernel(const float* __restrict__ lam, const float* __restrict__ E,
                                                      int64_t n_own, const int* __restrict__ api_own, int fsx,
                                                      int fsy, int fsz, float2* __restrict__ cellbuf) {
  const int ncx = fsx - 3, ncy = fsy - 3, ncz = fsz - 3;
  const int64_t n_cells = (int64_t)ncx * ncy * ncz;
  for (int64_t ci = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ci < n_cells;
       ci += (int64_t)gridDim.x * blockDim.x) {
    const int cx = 1 + (int)(ci % ncx);
    const int cy = 1 + (int)((ci / ncx) % ncy);
    const int cz = 1 + (int)(ci / ((int64_t)ncx * ncy));
    float L[8][3], X[8][3];
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const int64_t api = (int64_t)(cx + (o & 1)) + fsx * ((int64_t)(cy + ((o >> 1) & 1)) + (int64_t)fsy * (cz + (o >> 2)));
      const int64_t id = api_own[api];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        L[o][c] = lam[c * n_own + id];
        X[o][c] = E[c * n_own + id];
      }
    }
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      const int a = kPerm[t][0], b = kPerm[t][1], c = kPerm[t][2];
      const int v1 = 1 << a, v2 = v1 | (1 << b);
      const float dl = (L[v1][a] - L[0][a]) + (L[v2][b] - L[v1][b]) + (L[7][c] - L[v2][c]);
      const float de = (X[v1][a] - X[0][a]) + (X[v2][b] - X[v1][b]) + (X[7][c] - X[v2][c]);
      cellbuf[ci * 6 + t] = make_float2(dl, de);
    }
  }
}

__global__ __launch_bounds__(256) void pg_node_kernel(const float* __restrict__ E, int64_t n_own,
                                                      const int* __restrict__ api_own, int fsx, int fsy, int fsz,
                                                      double h, const float2* __restrict__ cellbuf,
                                                      double* __restrict__ acc) {
  // free nodes: lattice coordinates in [2, fs - 3] per axis
  const int nx = fsx - 4, ny = fsy - 4, nz = fsz - 4;
  const int ncx = fsx - 3, ncy = fsy - 3;
  const int64_t n_free = (int64_t)nx * ny * nz;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_free; q += (int64_t)gridDim.x * blockDim.x) {
    const int lx = 2 + (int)(q % nx);
    const int ly = 2 + (int)((q / nx) % ny);
    const int lz = 2 + (int)(q / ((int64_t)nx * ny));
    const int64_t api = (int64_t)lx + fsx * ((int64_t)ly + (int64_t)fsy * lz);
    const int64_t id = api_own[api];
    const float Ei[3] = {E[id], E[n_own + id], E[2 * n_own + id]};
    double s = 0.0;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      // the cell whose corner o is this node; its interior index
      const int cx = lx - (o & 1), cy = ly - ((o >> 1) & 1), cz = lz - (o >> 2);
      const int64_t ci = (int64_t)(cx - 1) + ncx * ((int64_t)(cy - 1) + (int64_t)ncy * (cz - 1));
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const int a = kPerm[t][0], b = kPerm[t][1], c = kPerm[t][2];
        const int v1 = 1 << a, v2 = v1 | (1 << b);
        float gE;   // h grad phi . E_i for the vertex this node is
        if (o == 0) gE = -Ei[a];
        else if (o == v1) gE = Ei[a] - Ei[b];
        else if (o == v2) gE = Ei[b] - Ei[c];
        else if (o == 7) gE = Ei[c];
        else continue;
        const float2 v = cellbuf[ci * 6 + t];
        s += (double)v.x * ((double)v.y - 4.0 * (double)gE);
      }
    }
    acc[api] += s * (h / 24.0);
  }
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

void launch_paper_grad_step(const float* lam, const float* E, int64_t n_own, const int* api_own, const int fs[3],
                            double h, float2* cellbuf, double* acc, hipStream_t s) {
  if (fs[0] < 5 || fs[1] < 5 || fs[2] < 5) return;   // no free node
  const int64_t n_cells = (int64_t)(fs[0] - 3) * (fs[1] - 3) * (fs[2] - 3);
  const int64_t n_free = (int64_t)(fs[0] - 4) * (fs[1] - 4) * (fs[2] - 4);
  hipLaunchKernelGGL(pg_cell_kernel, dim3(blocks_for(n_cells)), dim3(256), 0, s, lam, E, n_own, api_own, fs[0], fs[1],
                     fs[2], cellbuf);
  hipLaunchKernelGGL(pg_node_kernel, dim3(blocks_for(n_free)), dim3(256), 0, s, E, n_own, api_own, fs[0], fs[1], fs[2],
                     h, cellbuf, acc);
}

void launch_add_free(const double* acc, const int fs[3], double* out_eps, hipStream_t s) {
  const int64_t n = (int64_t)fs[0] * fs[1] * fs[2];
  hipLaunchKernelGGL(add_free_kernel, dim3(blocks_for(n)), dim3(256), 0, s, acc, fs[0], fs[1], fs[2], out_eps);
}

}  // namespace dd
