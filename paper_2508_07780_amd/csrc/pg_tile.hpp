// The paper-formula div-div gradient terms of one tile of free nodes (eq. gradeps with
// div(eps~ E) replaced by eps~ div(E)), as a device function shared by the standalone
// kernel and the fused adjoint step of the form R2.
//
// Geometry of the Kuhn split: the cell with lower corner c (spacing h) holds one
// tetrahedron per axis permutation (a, b, c): v0 = c, v1 = v0 + e_a, v2 = v1 + e_b,
// v3 = v2 + e_c.  Its barycentric functions are 1 - x_a, x_a - x_b, x_b - x_c, x_c (local
// coordinates in units of h), so h grad phi = -e_a, e_a - e_b, e_b - e_c, e_c, |K| = h^3/6 and
//     h div_K(u) = (u1 - u0)_a + (u2 - u1)_b + (u3 - u2)_c.
// With dl = h div_K(lambda), de = h div_K(E), g = h grad phi_i, the paper term P_i and the
// exact R1 term Q_i of one tetrahedron K containing node i are
//     (|K|/4) div lambda div E = (h / 24) dl de,   |K| div lambda (grad phi_i . E_i) = (h / 24) dl 4 g.E_i,
// and acc_i += sum_K (h / 24) dl (wp de - wx 4 g.E_i).  A free node (layer >= 2) only touches
// cells whose corners are all FEM-owned, so lambda needs no restriction.
//
// A block of 256 threads takes an 8 x 8 x 4 tile of free nodes, stages lambda and E of the
// 10 x 10 x 6 nodes around it in LDS (14.4 KB of the dynamic LDS), and each thread forms the
// 24 tetrahedra of its node from the staged values (one barrier; no atomics, a fixed order).
#pragma once

#include "dd_common.hpp"

namespace dd {

constexpr int PG_TX = 8, PG_TY = 8, PG_TZ = 4;                          // free nodes per block
constexpr int PG_NX = PG_TX + 2, PG_NY = PG_TY + 2, PG_NZ = PG_TZ + 2;  // staged nodes
constexpr size_t PG_LDS_BYTES = 2 * 3 * PG_NX * PG_NY * PG_NZ * sizeof(float);

// Tiles of one launch over the free nodes (lattice 2 .. fs - 3 per axis); 0 without free nodes.
__host__ __device__ inline int pg_tiles(const int fs[3]) {
  if (fs[0] < 5 || fs[1] < 5 || fs[2] < 5) return 0;
  return ((fs[0] - 4 + PG_TX - 1) / PG_TX) * ((fs[1] - 4 + PG_TY - 1) / PG_TY) * ((fs[2] - 4 + PG_TZ - 1) / PG_TZ);
}

// Tile b (< pg_tiles(g.fs)) by a block of 256 threads; the whole block calls it.
__device__ __forceinline__ void pg_tile(const PgArgs& g, int b) {
  extern __shared__ __align__(16) unsigned char lds[];
  float (*sl)[PG_NZ][PG_NY][PG_NX] = reinterpret_cast<float (*)[PG_NZ][PG_NY][PG_NX]>(lds);
  float (*se)[PG_NZ][PG_NY][PG_NX] = reinterpret_cast<float (*)[PG_NZ][PG_NY][PG_NX]>(lds) + 3;
  // axis permutations (a, b, c) of the six tetrahedra
  constexpr int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  const int fsx = g.fs[0], fsy = g.fs[1], fsz = g.fs[2];
  const int tbx = (fsx - 4 + PG_TX - 1) / PG_TX, tby = (fsy - 4 + PG_TY - 1) / PG_TY;
  const int x0 = 2 + (b % tbx) * PG_TX, y0 = 2 + ((b / tbx) % tby) * PG_TY, z0 = 2 + (b / (tbx * tby)) * PG_TZ;
  const int t = threadIdx.x;
  // stage nodes x0-1 .. x0+TX (clamped to the last owned node; values past it are unused)
  for (int i = t; i < PG_NX * PG_NY * PG_NZ; i += 256) {
    const int ix = i % PG_NX, iy = (i / PG_NX) % PG_NY, iz = i / (PG_NX * PG_NY);
    const int gx = min(x0 - 1 + ix, fsx - 2), gy = min(y0 - 1 + iy, fsy - 2), gz = min(z0 - 1 + iz, fsz - 2);
    const int64_t id = g.api_own[(int64_t)gx + fsx * ((int64_t)gy + (int64_t)fsy * gz)];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sl[c][iz][iy][ix] = g.lam[c * g.n_own + id];
      se[c][iz][iy][ix] = g.E[c * g.n_own + id];
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
    // the cell whose corner o is this node: lower corner at staged (tx + 1 - ox, ...)
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
#define PG_AT(arr, comp, q) arr[comp][cz + ((q) >> 2)][cy + (((q) >> 1) & 1)][cx + ((q) & 1)]
      const float dl = (PG_AT(sl, a, v1) - PG_AT(sl, a, 0)) + (PG_AT(sl, bb, v2) - PG_AT(sl, bb, v1)) +
                       (PG_AT(sl, c, 7) - PG_AT(sl, c, v2));
      const float de = (PG_AT(se, a, v1) - PG_AT(se, a, 0)) + (PG_AT(se, bb, v2) - PG_AT(se, bb, v1)) +
                       (PG_AT(se, c, 7) - PG_AT(se, c, v2));
#undef PG_AT
      s += (double)dl * (g.wp * (double)de - g.wx * 4.0 * (double)gE);
    }
  }
  g.acc[(int64_t)lx + fsx * ((int64_t)ly + (int64_t)fsy * lz)] += s * (g.h / 24.0);
}

}  // namespace dd
