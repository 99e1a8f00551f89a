// HIP kernels (gfx950) of the hybrid FE/FD leapfrog: finite-difference region,
// FEM region, and the small helpers around them.
//
// Both regions advance the same explicit scheme (the central-difference leapfrog for
// eq. forward_prob / eq. model1), the FEM region in increment form
//     V^{n+1} = [ (M/dt^2 - C/(2dt)) V^n - A E^n + F^n ] / (M/dt^2 + C/(2dt)),
//     E^{n+1} = E^n + V^{n+1},
// the finite-difference region (vacuum) in three-level form, V^n = E^n - E^{n-1} formed
// from the two stored levels, so that only E is stored there (36 B per node and step),
// and its exact transpose for the adjoint (eq. adjoint_prob) run backward:
//     Lambda^k = [ (M/dt^2 - C^{k+1}/(2dt)) Lambda^{k+1} - A^T lambda^k - r^k
//                  - (C^{k-1} - C^{k+1}) lambda^k / (2dt) ] / (M/dt^2 + C^{k-1}/(2dt)),
//     lambda^{k-1} = lambda^k + Lambda^k.
// Field state is FP32; the energy and gradient sums are FP64.
#include "dd_common.hpp"
#include "pg_tile.hpp"

namespace dd {

// ---------------------------------------------------------------------------------------
// Finite-difference region.  eps = 1, sigma = 0 here (eq. epsilon_sigma_constraint), so
// the update is the 7-point wave stencil with mirror (Neumann) weights on the outer box,
// lumped absorbing damping on absorbing faces and the plane-wave / dipole forcing.
// Tile = 32 x 8 nodes in (x, y), marching a chunk of fd_zc(NT) planes in z: the current plane sits in LDS
// (with a one-node halo, double-buffered), the z-1 / z+1 values of each column stay in a
// register queue that is prefetched three planes ahead; the previous level and the halo
// two ahead.
// The march is fully unrolled, so the queues rotate by renaming registers, and every
// access is a 32-bit byte offset from a uniform base pointer (one offset register serves
// the three components).  Loads never branch on a lane's position: lanes outside the grid
// read a valid clamped address and their values are discarded.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ float ld_at(const char* base, uint32_t off) {
  return *reinterpret_cast<const float*>(base + off);
}
// The node's own previous level and its new level are each touched once per step.  When
// the grid's two levels of E do not fit in the last-level cache (NT), these two streams
// use non-temporal accesses, which keeps the caches for the E planes that neighbouring
// tiles re-read; when they fit, ordinary accesses let the next step find them there.
template <bool NT>
__device__ __forceinline__ float ld_own(const char* base, uint32_t off) {
  if (NT) return __builtin_nontemporal_load(reinterpret_cast<const float*>(base + off));
  return *reinterpret_cast<const float*>(base + off);
}
template <bool NT>
__device__ __forceinline__ void st_own(char* base, uint32_t off, float v) {
  if (NT) __builtin_nontemporal_store(v, reinterpret_cast<float*>(base + off));
  else *reinterpret_cast<float*>(base + off) = v;
}

// The time function of an obliquely incident plane wave at top-face node (x, y): the pulse of
// the source kind delayed by tau = pw_kx (x - pw_x0) + pw_ky (y - pw_y0).  Inside the pulse's
// support the sine's argument stays within 3 pi (the Gaussian-modulated sine: |omega u| <=
// omega t0 = 3 pi; one sine period: < 2 pi), where the hardware sine and exponential are
// accurate to about 1e-6, well inside the trace tolerance, and need no argument reduction.
// kind, tn: the step's source kind and time (t_n, or t_n - t0 for the Gaussian-modulated sine).
__device__ __forceinline__ float oblique_pulse_at(const FdArgs& a, int kind, float tn, int x, int y) {
  const float tau = a.pw_kx * (float)(x - a.pw_x0) + a.pw_ky * (float)(y - a.pw_y0);
  const float u = tn - tau;
  if (kind == DD_SRC_GAUSS_SINE) {
    if (!(fabsf(u) <= a.pw_sup)) return 0.f;
    const float v = u * a.pw_iw;
    return __sinf(a.pw_omega * u) * __expf(-0.5f * v * v);
  }
  if (!(u > 0.f && u < a.pw_sup)) return 0.f;
  return __sinf(a.pw_omega * u);
}
__device__ __forceinline__ float oblique_pulse(const FdArgs& a, int x, int y) {
  return oblique_pulse_at(a, a.pw_kind, a.pw_t, x, y);
}

// b: block index within the finite-difference part of the launch; b % N_XCD must equal
// blockIdx.x % N_XCD so that the remap below keeps consecutive tiles on one XCD.
// OBL: the top face may carry an obliquely incident plane wave (a separate instantiation, so
// that the kernels of normal incidence keep their register allocation).
// The node update, here and in the two-step tiles, is written with explicit fused multiply-adds
// and no other contraction, so every path rounds alike: S = wz sz + (wy sy + wx sx) (mirror
// weights 1 inside), E^{n+1} = E^n + [(E^n - E^{n-1}) - nu^2 S + F] (damped faces: the divided
// form).  With unit weights and no forcing it is the interior update of the two-step tiles.
// DYN: the two planes live at the start of the launch's dynamic LDS instead of a static array
// (a launch whose other blocks need more dynamic LDS then holds one buffer, not both).
template <bool ENERGY, bool NT, bool OBL = false, bool DYN = false>
__device__ __forceinline__ void fd_tile(const FdArgs& a, const int b) {
#pragma clang fp contract(off)
  constexpr int ZC = fd_zc(NT);
  // two LDS planes: plane z is written while plane z-1 may still be read by slower waves,
  // so one barrier per plane suffices
  constexpr int SW = FD_TX + 2, SC = (FD_TY + 2) * SW;   // row and component strides
  __shared__ float s_static[DYN ? 1 : 2][DYN ? 1 : 3 * SC];
  extern __shared__ __align__(16) unsigned char fd_dyn[];
  float (*s)[3 * SC] = DYN ? reinterpret_cast<float (*)[3 * SC]>(fd_dyn)
                           : reinterpret_cast<float (*)[3 * SC]>(&s_static[0][0]);
  __shared__ double red[ENERGY ? FD_THREADS : 1];
  // consecutive tiles share an XCD's L2; on alternate steps each XCD sweeps its tiles in
  // reverse, starting where the previous step ended, whose fields are still in the caches
  const int kx = a.rev ? a.per_xcd - 1 - b / N_XCD : b / N_XCD;
  const int t = (b % N_XCD) * a.per_xcd + kx;
  if (t >= a.ntiles) return;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  constexpr int ZG = fd_zgroup(NT);
  const int bx = t % a.nbx;
  int by, bz;
  if (ZG > 1) {
    const int r = t / a.nbx;
    by = (r / ZG) % a.nby;
    bz = (r / (ZG * a.nby)) * ZG + r % ZG;
  } else {
    by = (t / a.nbx) % a.nby;
    bz = t / (a.nbx * a.nby);
  }
  const int x0 = bx * FD_TX, y0 = by * FD_TY, z0 = bz * ZC;
  if (z0 >= nz) {
    // past the grid (a group's padding, or a tile grid built for another z-chunk)
    if (ENERGY && threadIdx.x == 0) a.epart[t] = 0.0;
    return;
  }
  const int z1 = min(z0 + ZC, nz);
  const int tid = threadIdx.x;
  if (x0 > a.blo[0] && x0 + FD_TX - 1 < a.bhi[0] && y0 > a.blo[1] && y0 + FD_TY - 1 < a.bhi[1] &&
      z0 > a.blo[2] && z1 - 1 < a.bhi[2]) {
    // every node of the tile is FEM-owned
    if (ENERGY && tid == 0) a.epart[t] = 0.0;
    return;
  }
  const int tx = tid % FD_TX, ty = tid / FD_TX;
  const int x = x0 + tx, y = y0 + ty;
  const bool col_ok = (x < nx) && (y < ny);
  // byte offsets within one component (the grid has fewer than 2^30 nodes)
  const uint32_t plane4 = 4u * (uint32_t)(nx * ny);
  const uint32_t col4 = col_ok ? 4u * (uint32_t)(y * nx + x) : 0u;
  const size_t comp = (size_t)a.N * 4;
  const char* X0 = reinterpret_cast<const char*>(a.X_in);
  const char* X1 = X0 + comp;
  const char* X2 = X1 + comp;
  // level n-1 on entry, overwritten with level n+1 node by node (only the node's own lane
  // reads or writes its value in this array); or level n-1 read from X_prev when it is set
  char* P0 = reinterpret_cast<char*>(a.X_out);
  char* P1 = P0 + comp;
  char* P2 = P1 + comp;
  const char* V0 = a.X_prev ? reinterpret_cast<const char*>(a.X_prev) : P0;
  const char* V1 = V0 + comp;
  const char* V2 = V1 + comp;

  // halo cell of this thread (80 ring cells of the 32 x 8 tile, corners unused)
  int hx = 0, hy = 0, hs = 0;
  if (tid < FD_TX) { hx = x0 + tid; hy = y0 - 1; hs = tid + 1; }
  else if (tid < 2 * FD_TX) { hx = x0 + tid - FD_TX; hy = y0 + FD_TY; hs = (FD_TY + 1) * SW + tid - FD_TX + 1; }
  else if (tid < 2 * FD_TX + FD_TY) { hx = x0 - 1; hy = y0 + tid - 2 * FD_TX; hs = (tid - 2 * FD_TX + 1) * SW; }
  else { hx = x0 + FD_TX; hy = y0 + tid - 2 * FD_TX - FD_TY; hs = (tid - 2 * FD_TX - FD_TY + 1) * SW + FD_TX + 1; }
  const bool h_role = tid < 2 * FD_TX + 2 * FD_TY;
  const bool h_ok = hx >= 0 && hx < nx && hy >= 0 && hy < ny;
  const uint32_t hcol4 = (h_role && h_ok) ? 4u * (uint32_t)(hy * nx + hx) : 0u;

  const bool bxl = x == 0, bxh = x == nx - 1, byl = y == 0, byh = y == ny - 1;
  const bool in_box_xy = x > a.blo[0] && x < a.bhi[0] && y > a.blo[1] && y < a.bhi[1];
  const bool in_box_xy_closed = x >= a.blo[0] && x <= a.bhi[0] && y >= a.blo[1] && y <= a.bhi[1];

  // Register queues along z.  Column: q0 = z-1, q1 = z, q2 = z+1, q3 = z+2, q4 = z+3 (in
  // flight); previous level pv = z, pn = z+1, pn2 = z+2 (in flight); halo cell hv = z, hn = z+1,
  // hn2 = z+2 (in flight).  Planes outside the grid or past the chunk read as 0.
  float q0[3] = {0.f, 0.f, 0.f}, q1[3], q2[3] = {0.f, 0.f, 0.f}, q3[3] = {0.f, 0.f, 0.f}, q4[3];
  float hv[3] = {0.f, 0.f, 0.f}, hn[3] = {0.f, 0.f, 0.f}, hn2[3];
  float pv[3], pn[3] = {0.f, 0.f, 0.f}, pn2[3];
  {
    const uint32_t o = (uint32_t)z0 * plane4 + col4;
    q1[0] = ld_at(X0, o); q1[1] = ld_at(X1, o); q1[2] = ld_at(X2, o);
    if (z0 > 0) { q0[0] = ld_at(X0, o - plane4); q0[1] = ld_at(X1, o - plane4); q0[2] = ld_at(X2, o - plane4); }
    if (z0 + 1 < nz) { q2[0] = ld_at(X0, o + plane4); q2[1] = ld_at(X1, o + plane4); q2[2] = ld_at(X2, o + plane4); }
    if (z0 + 2 < nz && z0 + 2 <= z1) {
      const uint32_t o2 = o + 2 * plane4;
      q3[0] = ld_at(X0, o2); q3[1] = ld_at(X1, o2); q3[2] = ld_at(X2, o2);
    }
    pv[0] = ld_own<NT>(V0, o); pv[1] = ld_own<NT>(V1, o); pv[2] = ld_own<NT>(V2, o);
    if (z0 + 1 < z1) { pn[0] = ld_own<NT>(V0, o + plane4); pn[1] = ld_own<NT>(V1, o + plane4); pn[2] = ld_own<NT>(V2, o + plane4); }
  }
  if (h_role) {
    const uint32_t o = (uint32_t)z0 * plane4 + hcol4;
    hv[0] = ld_at(X0, o); hv[1] = ld_at(X1, o); hv[2] = ld_at(X2, o);
    if (z0 + 1 < z1) { hn[0] = ld_at(X0, o + plane4); hn[1] = ld_at(X1, o + plane4); hn[2] = ld_at(X2, o + plane4); }
  }
  double eacc = 0.0;
#pragma unroll
  for (int k = 0; k < ZC; ++k) {
    const int z = z0 + k;
    if (z >= z1) break;
    const uint32_t zo = (uint32_t)z * plane4;
    float* sb = s[k & 1];
    const int sc = (ty + 1) * SW + tx + 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) sb[c * SC + sc] = q1[c];
    if (h_role) {
#pragma unroll
      for (int c = 0; c < 3; ++c) sb[c * SC + hs] = hv[c];
    }
    // prefetch: column three planes ahead (up to the plane just past the chunk), halo and
    // increment two planes ahead (within the chunk)
    q4[0] = q4[1] = q4[2] = 0.f;
    hn2[0] = hn2[1] = hn2[2] = 0.f;
    pn2[0] = pn2[1] = pn2[2] = 0.f;
    if (z + 3 < nz && z + 3 <= z1) {
      const uint32_t o = zo + 3 * plane4 + col4;
      q4[0] = ld_at(X0, o); q4[1] = ld_at(X1, o); q4[2] = ld_at(X2, o);
    }
    if (z + 2 < z1) {
      const uint32_t o = zo + 2 * plane4 + col4;
      pn2[0] = ld_own<NT>(V0, o); pn2[1] = ld_own<NT>(V1, o); pn2[2] = ld_own<NT>(V2, o);
      if (h_role) {
        const uint32_t oh = zo + 2 * plane4 + hcol4;
        hn2[0] = ld_at(X0, oh); hn2[1] = ld_at(X1, oh); hn2[2] = ld_at(X2, oh);
      }
    }
    // Adjoint: when the top face is the last plane of a full chunk, its trace cotangent is
    // loaded here, before the barrier, rather than after the stencil where its latency
    // would add to the march.  In this last unrolled iteration nothing is prefetched for
    // later planes, so these registers come free.
    float cr[3] = {0.f, 0.f, 0.f};
    const bool top_pref = k == ZC - 1 && a.cot_in && (a.det_mask & DD_FACE_TOP) && z == nz - 1;
    if (top_pref) {
      const uint32_t o3 = 12u * (uint32_t)face_lex_index(0, 0, nz - 1, nx, ny, nz, a.det_mask) + 3u * col4;
      const char* cot = reinterpret_cast<const char*>(a.cot_in);
      cr[0] = ld_at(cot, o3); cr[1] = ld_at(cot, o3 + 4); cr[2] = ld_at(cot, o3 + 8);
      if (a.obs_in) {
        const char* obs = reinterpret_cast<const char*>(a.obs_in);
        cr[0] -= ld_at(obs, o3); cr[1] -= ld_at(obs, o3 + 4); cr[2] -= ld_at(obs, o3 + 8);
      }
    }
    __syncthreads();
    const bool fem_owned = in_box_xy && z > a.blo[2] && z < a.bhi[2];
    if (col_ok && !fem_owned) {
      const bool bzl = z == 0, bzh = z == nz - 1;
      const float wx = (bxl || bxh) ? 2.f : 1.f;   // 2 / (neighbours along x): mirror weights
      const float wy = (byl || byh) ? 2.f : 1.f;
      const float wz = (bzl || bzh) ? 2.f : 1.f;
      const uint32_t idx4 = zo + col4;
      float S[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float xc = q1[c];
        const float* p = sb + c * SC + sc;
        const float sx = (bxl ? 0.f : xc - p[-1]) + (bxh ? 0.f : xc - p[1]);
        const float sy = (byl ? 0.f : xc - p[-SW]) + (byh ? 0.f : xc - p[SW]);
        const float sz = (bzl ? 0.f : xc - q0[c]) + (bzh ? 0.f : xc - q2[c]);
        S[c] = __builtin_fmaf(wz, sz, __builtin_fmaf(wy, sy, wx * sx));
      }
      const bool on_bnd = bxl || bxh || byl || byh || bzl || bzh;
      float src[3] = {0.f, 0.f, 0.f};
      int na = 0, nb = 0, bcount = 0;
      int64_t det = -1;
      if (on_bnd) {
        bcount = (int)(bxl || bxh) + (int)(byl || byh) + (int)(bzl || bzh);
        const unsigned am = a.abs_mask;
        const int fixed = ((am & DD_FACE_BOTTOM) && bzl) + ((am & DD_FACE_XMIN) && bxl) +
                          ((am & DD_FACE_XMAX) && bxh) + ((am & DD_FACE_YMIN) && byl) + ((am & DD_FACE_YMAX) && byh);
        const int top = (am & DD_FACE_TOP) && bzh;
        na = fixed + top * a.top_a;
        nb = fixed + top * a.top_b;
        if (bzh) {
          src[0] += a.pw[0];
          src[1] += a.pw[1];
          src[2] += a.pw[2];
          if (OBL && a.pw_kind) {
            const float pv = oblique_pulse(a, x, y);
            src[0] += a.pw_amp[0] * pv;
            src[1] += a.pw_amp[1] * pv;
            src[2] += a.pw_amp[2] * pv;
          }
        }
        if (a.det_mask) det = face_lex_index(x, y, z, nx, ny, nz, a.det_mask);
        if (det >= 0 && a.cot_in) {
          const float sc2 = a.dt2_h3 * (float)(1 << bcount);   // dt^2 / m_i
          // r = dJ/dT: the cotangent itself, or T - E_obs when the observations are given
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float r = (top_pref && bzh) ? cr[c]
                          : a.obs_in ? a.cot_in[det * 3 + c] - a.obs_in[det * 3 + c] : a.cot_in[det * 3 + c];
            src[c] -= r * sc2;
          }
        }
      }
      if ((int64_t)(idx4 >> 2) == a.dip_idx) {
#pragma unroll
        for (int c = 0; c < 3; ++c) src[c] += a.dip[c];
      }
      int64_t l0 = -1;
      if (a.iface_out && in_box_xy_closed && z >= a.blo[2] && z <= a.bhi[2])
        l0 = face_lex_index(x - a.blo[0], y - a.blo[1], z - a.blo[2], a.fs[0], a.fs[1], a.fs[2], 63u);
      // three-level form: the increment of this level is the difference of the two stored
      // levels, out = increment of the next level, xn = next level
      float out[3], xn[3];
      if (na == 0 && nb == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] = __builtin_fmaf(-a.nu2, S[c], q1[c] - pv[c]) + src[c];
      } else {
        const float ba = a.nu * (float)na, bb = a.nu * (float)nb;
#pragma unroll
        for (int c = 0; c < 3; ++c)
          out[c] = ((1.f - bb) * (q1[c] - pv[c]) - a.nu2 * S[c] + src[c] - (ba - bb) * q1[c]) / (1.f + ba);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) xn[c] = q1[c] + out[c];
      st_own<NT>(P0, idx4, xn[0]); st_own<NT>(P1, idx4, xn[1]); st_own<NT>(P2, idx4, xn[2]);
      if (det >= 0 && a.tr_out) {
#pragma unroll
        for (int c = 0; c < 3; ++c) a.tr_out[det * 3 + c] = xn[c];
      }
      if (l0 >= 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) a.iface_out[c * a.n_l0 + l0] = xn[c];
      }
      if (ENERGY) {
        double e_node = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) e_node += (double)out[c] * (double)out[c] + (double)xn[c] * (double)(a.nu2 * S[c]);
        eacc += a.e_coef * ldexp(1.0, -bcount) * e_node;
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      q0[c] = q1[c];
      q1[c] = q2[c];
      q2[c] = q3[c];
      q3[c] = q4[c];
      hv[c] = hn[c];
      hn[c] = hn2[c];
      pv[c] = pn[c];
      pn[c] = pn2[c];
    }
  }
  if (ENERGY) {
    red[tid] = eacc;
    __syncthreads();
    for (int w = FD_THREADS / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) a.epart[t] = red[0];
  }
}

template <bool ENERGY, bool NT, bool OBL>
__global__ __launch_bounds__(FD_THREADS) void fd_step_kernel(FdArgs a) {
  fd_tile<ENERGY, NT, OBL>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------------------
// FEM region: lumped-mass P1 on tetrahedra (stiffness + div-div stabiliser of eq.
// lagrangian_weak).  One workgroup per partition: the partition's owned and halo node
// values are staged in LDS, the element terms are summed per owned node, then owned nodes
// are advanced.  Two forms of the sums: colour by colour, each element scattered into LDS
// accumulators of its owned nodes with a barrier between colours, or gathered per owned node
// over its incident elements in the same colour order, in registers and with no barrier (the
// same sums up to rounding; faster on the measured meshes, the default).
//   forward:  (A E)_i = sum_K |K| [grad phi_i . grad(E_c)|_K + d_c phi_i div_K((eps-1) E)]
//   adjoint:  (A^T l)_i = sum_K |K| grad phi_i . grad(l_c)|_K + (eps_i - 1) q_i,
//             q_i = sum_K |K| grad phi_i div_K(l)
// and the adjoint also accumulates, on free nodes, the gradient of eq. gradeps:
//   g_eps += q_i . E^k_i + (m_i / dt^2) Lambda^k_i . V^k_i,
//   g_sig += (m_i / (2 dt)) lambda^{k-1}_i . (V^k_i + V^{k-1}_i).
// Layer-0 values come from the interface buffer written by the finite-difference kernel;
// layer-1 results are also written into the finite-difference grid (the two-node overlap).
// ---------------------------------------------------------------------------------------
// Row of owned node l (local id) of a partition's element sums in the gather form: the terms of
// the elements incident to the node, in the partition's colour order (the scatter's order; each
// term is formed through the element's stiffness entries of the node's row instead of the
// element's full gradient, so the two forms agree to rounding).  Forward: acc = the node's
// row of K E + the div-div row of (eps - 1) E; adjoint: acc = the row of K^T lambda without
// the div-div part, acd = sum over K of |K| grad phi_l div_K lambda (scaled by eps_l - 1 later).
template <bool ADJ>
__device__ __forceinline__ void fem_gather_row(const uint16_t* __restrict__ inc, const int ni, const int no,
                                               const int l, const uint64_t* __restrict__ gE,
                                               const float* __restrict__ G, const float4* sX, float4& acc,
                                               float4& acd) {
  acc = make_float4(0.f, 0.f, 0.f, 0.f);
  acd = acc;
  // GB entries and their element words are loaded before the arithmetic of any of them, so
  // that one batch waits for two memory latencies, not two per element
  constexpr int GB = DD_FEM_GB;
  for (int i0 = 0; i0 < ni; i0 += GB) {
    unsigned ub[GB];
#pragma unroll
    for (int b = 0; b < GB; ++b) ub[b] = i0 + b < ni ? (unsigned)inc[(i0 + b) * no + l] : 0xFFFFu;
    uint64_t wb[GB];
#pragma unroll
    for (int b = 0; b < GB; ++b) wb[b] = ub[b] != 0xFFFFu ? gE[ub[b] >> 2] : 0ull;
#pragma unroll
    for (int b = 0; b < GB; ++b) {
      const unsigned u = ub[b];
      if (u == 0xFFFFu) break;   // a node's list is padded at its end
      const uint64_t w = wb[b];
      const int k = (int)(u & 3u);
      const float* g = G + (int)(w >> 44) * GEOM_STRIDE;
      const float4* g4 = reinterpret_cast<const float4*>(g);
      float gr[12];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const float4 a4 = g4[q];
        gr[4 * q] = a4.x; gr[4 * q + 1] = a4.y; gr[4 * q + 2] = a4.z; gr[4 * q + 3] = a4.w;
      }
      // |K| grad phi_k of the node's slot
      const float a0 = g[12 + 3 * k], a1 = g[13 + 3 * k], a2 = g[14 + 3 * k];
      // the node's row through the element's stiffness entries s_j = |K| grad phi_k . grad phi_j:
      // sum_j s_j E_j (+ |K| grad phi_k div_K((eps - 1) E) forward); dv = div_K of (eps-1)E or lambda
      float c0 = 0.f, c1 = 0.f, c2 = 0.f, dv = 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float4 x = sX[(int)((w >> (11 * j)) & 0x7FFu)];
        const float sj = a0 * gr[3 * j] + a1 * gr[3 * j + 1] + a2 * gr[3 * j + 2];
        c0 += sj * x.x;
        c1 += sj * x.y;
        c2 += sj * x.z;
        const float dj = x.x * gr[3 * j] + x.y * gr[3 * j + 1] + x.z * gr[3 * j + 2];
        dv += ADJ ? dj : x.w * dj;
      }
      if (!ADJ) {
        c0 += a0 * dv;
        c1 += a1 * dv;
        c2 += a2 * dv;
      }
      acc.x += c0;
      acc.y += c1;
      acc.z += c2;
      if (ADJ) {
        acd.x += a0 * dv;
        acd.y += a1 * dv;
        acd.z += a2 * dv;
      }
    }
    if (ub[GB - 1] == 0xFFFFu) break;
  }
}

// One FEM partition p of the element-coloured step, by a block of FEM_THREADS threads
// (GATHER: the gather form of the element sums).
template <bool ADJ, bool ENERGY, bool GEOM_LDS, bool STAGE, bool GATHER = false>
__device__ __forceinline__ void fem_el_part(const FemArgs& a, const int p) {
  static_assert(!(GATHER && STAGE), "the gather form reads the elements from global memory");
  constexpr int NPT = FEM_OWN_MAX / FEM_THREADS;   // owned nodes per thread in the update
  constexpr int NA4 = ADJ ? 2 : 1;                 // float4 accumulators per owned node
  // Dynamic LDS sized from the mesh.  One float4 per node (E_x, E_y, E_z, eps - 1) and per
  // accumulator, so a node is gathered or scattered with a single 16-byte access; each
  // accumulator row has 32 trash slots that absorb the contributions to halo nodes.  STAGE:
  // the packed elements are staged in LDS too (8 B each); otherwise each colour reads them
  // from global memory, and a block needs less LDS, so that more blocks share a CU.
  extern __shared__ __align__(16) unsigned char lds[];
  // GATHER: the sums stay in registers, no accumulator rows
  const int LOC = a.lds_loc, ROW = GATHER ? 0 : a.lds_own + 32;
  float4* sX = reinterpret_cast<float4*>(lds);                // [LOC]
  float4* sA = sX + LOC;                                      // [NA4][ROW]
  uint64_t* sE = reinterpret_cast<uint64_t*>(sA + NA4 * ROW);  // [lds_elem] (even), if STAGE
  float* sG = reinterpret_cast<float*>(sE + (STAGE ? a.lds_elem : 0));   // [n_geom][GEOM_STRIDE]
  int* sC = reinterpret_cast<int*>(sG + (GEOM_LDS ? a.n_geom * GEOM_STRIDE : 0));   // [ncl + 1]
  __shared__ double red[ENERGY ? FEM_THREADS : 1];
  const int tid = threadIdx.x;
  const int o0 = a.own_off[p], no = a.own_off[p + 1] - o0;
  const int h0 = a.halo_off[p], nh = a.halo_off[p + 1] - h0;
  const int nl = no + nh;
  const int ncl = a.ncol[p], cb = a.col_base[p];
  const int e_beg = a.col_off[cb], ne = a.col_off[cb + ncl] - e_beg;
  const int64_t n_own = a.n_own, n_l0 = a.n_l0;

  // ---- stage: colour offsets, geometry, node values.  Loads are issued in unrolled
  // batches so that one batch costs one memory latency, not one per iteration.
  if (tid <= ncl) sC[tid] = a.col_off[cb + tid] - e_beg;
  if (STAGE) {
    constexpr int EB = 8;
    for (int base = 0; base < ne; base += EB * FEM_THREADS) {
      uint64_t tmp[EB];
#pragma unroll
      for (int k = 0; k < EB; ++k) {
        const int i = base + k * FEM_THREADS + tid;
        tmp[k] = i < ne ? a.elems[e_beg + i] : 0ull;
      }
#pragma unroll
      for (int k = 0; k < EB; ++k) {
        const int i = base + k * FEM_THREADS + tid;
        if (i < ne) sE[i] = tmp[k];
      }
    }
  }
  const uint64_t* __restrict__ gE = STAGE ? sE : a.elems + e_beg;
  if (GEOM_LDS)
    for (int i = tid; i < a.n_geom * GEOM_STRIDE; i += FEM_THREADS) sG[i] = a.geom[i];
  constexpr int NB = 4;
  for (int base = 0; base < nl; base += NB * FEM_THREADS) {
    int code[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int l = base + k * FEM_THREADS + tid;
      code[k] = l < no ? o0 + l : (l < nl ? a.halo[h0 + l - no] : 0);
    }
    float4 xv[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int l = base + k * FEM_THREADS + tid;
      xv[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (l < nl && code[k] >= 0) {
        const int id = code[k];
        xv[k].x = a.X_in[id];
        xv[k].y = a.X_in[n_own + id];
        xv[k].z = a.X_in[2 * n_own + id];
        if (!ADJ) xv[k].w = a.em1[id];
      } else if (l < nl) {
        const int64_t q = -1 - (int64_t)code[k];
        xv[k].x = a.iface_in[q];
        xv[k].y = a.iface_in[n_l0 + q];
        xv[k].z = a.iface_in[2 * n_l0 + q];
      }
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int l = base + k * FEM_THREADS + tid;
      if (l < nl) sX[l] = xv[k];
    }
  }
  for (int l = tid; l < ROW; l += FEM_THREADS) {   // (no rows in the gather form)
#pragma unroll
    for (int c = 0; c < NA4; ++c) sA[c * ROW + l] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  // per-node data of the update, prefetched into registers while the elements run
  float pI[NPT][3], pc1[NPT], pc2[NPT], pem[NPT];
  float pwE[NPT][3], pwV[NPT][3], pwVm[NPT][3];
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int l = tid + j * FEM_THREADS;
    if (l < no) {
      const int id = o0 + l;
#pragma unroll
      for (int c = 0; c < 3; ++c) pI[j][c] = a.I_in[c * n_own + id];
      pc1[j] = a.c1[id];
      pc2[j] = a.c2[id];
      pem[j] = a.em1[id];
      if (ADJ) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          pwE[j][c] = __builtin_nontemporal_load(a.wE + c * n_own + id);
          pwV[j][c] = __builtin_nontemporal_load(a.wV + c * n_own + id);
          pwVm[j][c] = __builtin_nontemporal_load(a.wVm + c * n_own + id);
        }
      }
    }
  }
  __syncthreads();

  // ---- elements, colour by colour (no two elements of a colour share an owned node)
  const float* __restrict__ G = GEOM_LDS ? sG : a.geom;
  const int trash = a.lds_own + (tid & 31);
  for (int c = 0; c < (GATHER ? 0 : ncl); ++c) {
    const int e0 = sC[c], e1 = sC[c + 1];
    for (int e = e0 + tid; e < e1; e += FEM_THREADS) {
      const uint64_t w = gE[e];
      int v[4], t[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        v[k] = (int)((w >> (11 * k)) & 0x7FFu);
        t[k] = v[k] < no ? v[k] : trash;
      }
      // accumulator reads first: their latency overlaps the element arithmetic
      float4 acc[4], acd[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        acc[k] = sA[t[k]];
        if (ADJ) acd[k] = sA[ROW + t[k]];
      }
      const float4* g4 = reinterpret_cast<const float4*>(G + (int)(w >> 44) * GEOM_STRIDE);
      // g4[0..2]: grad phi_0..3 (12 floats), g4[3..5]: |K| grad phi_0..3
      float gr[12], vg[12];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const float4 a4 = g4[i], b4 = g4[3 + i];
        gr[4 * i] = a4.x; gr[4 * i + 1] = a4.y; gr[4 * i + 2] = a4.z; gr[4 * i + 3] = a4.w;
        vg[4 * i] = b4.x; vg[4 * i + 1] = b4.y; vg[4 * i + 2] = b4.z; vg[4 * i + 3] = b4.w;
      }
      // Gm[q] = gradient of component q on the element; dv = div of (eps-1)E (forward) or lambda
      float Gm[3][3];
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int d = 0; d < 3; ++d) Gm[q][d] = 0.f;
      float dv = 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float4 x = sX[v[j]];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          Gm[0][d] += x.x * gr[3 * j + d];
          Gm[1][d] += x.y * gr[3 * j + d];
          Gm[2][d] += x.z * gr[3 * j + d];
        }
        const float dj = x.x * gr[3 * j] + x.y * gr[3 * j + 1] + x.z * gr[3 * j + 2];
        dv += ADJ ? dj : x.w * dj;
      }
      if (!ADJ) {
        // contribution to slot k, component q: |K| grad phi_k . (Gm[q] + dv e_q)
#pragma unroll
        for (int q = 0; q < 3; ++q) Gm[q][q] += dv;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float a0 = vg[3 * k], a1 = vg[3 * k + 1], a2 = vg[3 * k + 2];
          acc[k].x += a0 * Gm[0][0] + a1 * Gm[0][1] + a2 * Gm[0][2];
          acc[k].y += a0 * Gm[1][0] + a1 * Gm[1][1] + a2 * Gm[1][2];
          acc[k].z += a0 * Gm[2][0] + a1 * Gm[2][1] + a2 * Gm[2][2];
          sA[t[k]] = acc[k];
        }
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float a0 = vg[3 * k], a1 = vg[3 * k + 1], a2 = vg[3 * k + 2];
          acc[k].x += a0 * Gm[0][0] + a1 * Gm[0][1] + a2 * Gm[0][2];
          acc[k].y += a0 * Gm[1][0] + a1 * Gm[1][1] + a2 * Gm[1][2];
          acc[k].z += a0 * Gm[2][0] + a1 * Gm[2][1] + a2 * Gm[2][2];
          acd[k].x += a0 * dv;
          acd[k].y += a1 * dv;
          acd[k].z += a2 * dv;
          sA[t[k]] = acc[k];
          sA[ROW + t[k]] = acd[k];
        }
      }
    }
    __syncthreads();
  }

  // ---- owned-node update
  double eacc = 0.0;
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int l = tid + j * FEM_THREADS;
    if (l >= no) continue;
    const int id = o0 + l;
    const float4 x4 = sX[l];
    float4 s4, d4;
    if (GATHER) {
      fem_gather_row<ADJ>(a.inc + a.inc_off[p], a.inc_n[p], no, l, a.elems + e_beg, G, sX, s4, d4);
    } else {
      s4 = sA[l];
      d4 = ADJ ? sA[ROW + l] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const float xo[3] = {x4.x, x4.y, x4.z};
    const float q[3] = {d4.x, d4.y, d4.z};
    float r[3] = {s4.x, s4.y, s4.z};
    if (ADJ) {
#pragma unroll
      for (int c = 0; c < 3; ++c) r[c] += pem[j] * q[c];
    }
    float xn[3], inc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      inc[c] = pc1[j] * pI[j][c] - pc2[j] * r[c];
      xn[c] = xo[c] + inc[c];
      a.I_out[c * n_own + id] = inc[c];
      a.X_out[c * n_own + id] = xn[c];
    }
    if (a.fd_out) {
      const int gi = a.own_grid[id];
      if (gi >= 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) a.fd_out[c * a.N + gi] = xn[c];
      }
    }
    // the saved forward state is read back only by the adjoint, much later: streamed past
    // the caches (non-temporal), as are the adjoint's reads of it
    if (!ADJ && a.ck_X) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        __builtin_nontemporal_store(xn[c], a.ck_X + c * n_own + id);
        __builtin_nontemporal_store(inc[c], a.ck_I + c * n_own + id);
      }
    }
    if (ENERGY) {
      const double me = a.mass_d[id] * (1.0 + (double)pem[j]);
      double vv = 0.0, er = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        vv += (double)inc[c] * (double)inc[c];
        er += (double)xn[c] * (double)r[c];
      }
      eacc += me * a.inv_2dt2 * vv + 0.5 * er;
    }
    if (ADJ && a.own_grid[id] < 0) {
      const double m = a.mass_d[id];
      double ge = 0.0, gm = 0.0, gs = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double wv = (double)pwV[j][c];
        ge += (double)q[c] * (double)pwE[j][c];
        gm += (double)inc[c] * wv;
        gs += (double)xn[c] * (wv + (double)pwVm[j][c]);
      }
      a.g_eps[id] += ge + m * a.inv_dt2 * gm;
      a.g_sig[id] += m * a.inv_2dt * gs;
    }
  }
  if (ENERGY) {
    red[tid] = eacc;
    __syncthreads();
    for (int w = FEM_THREADS / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) a.epart[a.epart_off + p] = red[0];
  }
}

template <bool ADJ, bool ENERGY, bool GEOM_LDS, bool STAGE, bool GATHER>
__global__ __launch_bounds__(FEM_THREADS) void fem_step_kernel(FemArgs a) {
  fem_el_part<ADJ, ENERGY, GEOM_LDS, STAGE, GATHER>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------------------
// FEM region, assembled-stencil form.  When every FEM-owned node has the same assembled
// element star (the Kuhn split of a uniform box: each owned node is surrounded by the same
// 24 tetrahedra), the lumped-mass P1 operator of the element kernel above is one nodal
// stencil of 3x3 blocks, assembled once on the host in FP64 from the same element
// geometry:
//     (A E)_i = sum_s [ K_s E_{i+o_s} + B_s ((eps - 1) E)_{i+o_s} ],
//     K_s = sum_K |K| grad phi_i . grad phi_j,  B_s = sum_K |K| grad phi_i (grad phi_j)^T,
// and for the adjoint (A^T l)_i = sum_s K_s l_{i+o_s} + (eps_i - 1) q_i with
// q_i = sum_s B_s l_{i+o_s} (B_s^T is the block of the mirrored slot, so the same stencil
// applies).  Results equal the element form up to floating-point rounding; there is no
// scatter, hence no colouring and no barrier after the staging.
// ---------------------------------------------------------------------------------------
// The div-div form R2, sum_K |K| (mean_K eps - 1) grad phi_i div_K(u), is symmetric and has
// no fixed stencil (its coefficient varies by element), so it is evaluated element by
// element from the staged box: a Kuhn cell holds one tetrahedron per axis permutation
// (a, b, c) with v1 = e_a, v2 = e_a + e_b, v3 = (1,1,1); h grad phi of its vertices is -e_a,
// e_a - e_b, e_b - e_c, e_c, |K| = h^3 / 6, and h div_K(u) = (u_v1 - u_v0)_a + (u_v2 - u_v1)_b
// + (u_v3 - u_v2)_c.  Cells touching layer 0 have mean eps - 1 = 0, so the same form serves
// the forward and (restricted to the FEM rows) the adjoint.
__device__ __forceinline__ float f4c(const float4& v, int c) { return c == 0 ? v.x : (c == 1 ? v.y : v.z); }

// (h / 6) sum over the 24 tetrahedra around box node (bx, by, bz) of mean(w) (h grad phi_i) (h div u)
__device__ __forceinline__ void r2_term(const float4* sX, int BX, int BY, int bx, int by, int bz, float h, float r[3]) {
  // axis permutations (a, b, c); a compile-time table, so that the unrolled loops index
  // registers, not memory
  constexpr int kKuhnPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  float d[3] = {0.f, 0.f, 0.f};
  // four cells at a time: fully unrolled, the compiler hoists the 64 staged loads of all
  // eight cells (117 VGPRs, 4 waves per SIMD for the launch); four at a time keeps the
  // launch at 6 waves with no spill (73 VGPRs; the R2 solve 158.9 -> 148.8 ms, one cell at
  // a time 155.8 ms)
#pragma unroll 4
  for (int o = 0; o < 8; ++o) {
    const int cb = (bx - (o & 1)) + BX * ((by - ((o >> 1) & 1)) + BY * (bz - (o >> 2)));
    float4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = sX[cb + (u & 1) + BX * (((u >> 1) & 1) + BY * (u >> 2))];
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      const int ax = kKuhnPerm[t][0], bx2 = kKuhnPerm[t][1], cx = kKuhnPerm[t][2];
      const int v1 = 1 << ax, v2 = v1 | (1 << bx2);
      if (o != 0 && o != v1 && o != v2 && o != 7) continue;
      const float eb = 0.25f * (v[0].w + v[v1].w + v[v2].w + v[7].w);
      const float dl = (f4c(v[v1], ax) - f4c(v[0], ax)) + (f4c(v[v2], bx2) - f4c(v[v1], bx2)) +
                       (f4c(v[7], cx) - f4c(v[v2], cx));
      const float f = eb * dl;
      if (o == 0) d[ax] -= f;
      else if (o == v1) { d[ax] += f; d[bx2] -= f; }
      else if (o == v2) { d[bx2] += f; d[cx] -= f; }
      else d[cx] += f;
    }
  }
  const float k = h * (1.f / 6.f);
#pragma unroll
  for (int c = 0; c < 3; ++c) r[c] += k * d[c];
}

template <bool ADJ, bool ENERGY, bool R2 = false>
__device__ __forceinline__ void fem_stencil_part(const FemArgs& a, const int p) {
  constexpr int NPT = FEM_OWN_MAX / STENCIL_THREADS;
  extern __shared__ __align__(16) unsigned char lds[];
  float4* sX = reinterpret_cast<float4*>(lds);                   // [box]: E_x, E_y, E_z, eps - 1
  float* sKB = reinterpret_cast<float*>(sX + a.lds_box);          // [n_slots][12]: K, B (9), pad
  int* sOff = reinterpret_cast<int*>(sKB + 12 * STENCIL_SLOTS_MAX);  // [n_slots] box offsets
  __shared__ double red[ENERGY ? STENCIL_THREADS : 1];
  const int tid = threadIdx.x;
  const int ox = a.part_dims[4 * p], oy = a.part_dims[4 * p + 1], oz = a.part_dims[4 * p + 2];
  const int bbase = a.part_dims[4 * p + 3];
  const int BX = ox + 2, BY = oy + 2;
  const int nbox = BX * BY * (oz + 2);
  const int o0 = a.own_off[p], no = ox * oy * oz;
  const int ns = a.n_slots;
  const int64_t n_own = a.n_own, n_l0 = a.n_l0;

  if (tid < ns) {
    const int dx = a.slot_off[4 * tid], dy = a.slot_off[4 * tid + 1], dz = a.slot_off[4 * tid + 2];
    sOff[tid] = dx + BX * (dy + BY * dz);
    sKB[12 * tid] = a.slot_k[tid];
#pragma unroll
    for (int q = 0; q < 9; ++q) sKB[12 * tid + 1 + q] = a.slot_b[9 * tid + q];
  }
  // stage the box of node values in batches (one memory latency per batch)
  constexpr int NB = 4;
  for (int base = 0; base < nbox; base += NB * STENCIL_THREADS) {
    int code[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int l = base + k * STENCIL_THREADS + tid;
      code[k] = l < nbox ? a.box_codes[bbase + l] : 0;
    }
    float4 xv[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int l = base + k * STENCIL_THREADS + tid;
      xv[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (l < nbox && code[k] >= 0) {
        const int id = code[k];
        xv[k].x = a.X_in[id];
        xv[k].y = a.X_in[n_own + id];
        xv[k].z = a.X_in[2 * n_own + id];
        if (!ADJ || R2) xv[k].w = a.em1[id];
      } else if (l < nbox) {
        const int64_t q = -1 - (int64_t)code[k];
        xv[k].x = a.iface_in[q];
        xv[k].y = a.iface_in[n_l0 + q];
        xv[k].z = a.iface_in[2 * n_l0 + q];
      }
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int l = base + k * STENCIL_THREADS + tid;
      if (l < nbox) sX[l] = xv[k];
    }
  }
  // per-node data of the update, prefetched before the barrier (the adjoint's forward
  // window is read after the stencil sum to keep register pressure low)
  float pI[NPT][3], pc1[NPT], pc2[NPT], pem[NPT];
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int l = tid + j * STENCIL_THREADS;
    if (l < no) {
      const int id = o0 + l;
#pragma unroll
      for (int c = 0; c < 3; ++c) pI[j][c] = a.I_in[c * n_own + id];
      pc1[j] = a.c1[id];
      pc2[j] = a.c2[id];
      pem[j] = a.em1[id];
    }
  }
  __syncthreads();

  double eacc = 0.0;
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int l = tid + j * STENCIL_THREADS;
    if (l >= no) continue;
    const int id = o0 + l;
    const int ix = l % ox, iy = (l / ox) % oy, iz = l / (ox * oy);
    const int li = (ix + 1) + BX * ((iy + 1) + BY * (iz + 1));
    float r[3] = {0.f, 0.f, 0.f}, q[3] = {0.f, 0.f, 0.f};
    for (int s = 0; s < ns; ++s) {
      const float4 x = sX[li + sOff[s]];
      const float* kb = sKB + 12 * s;
      const float K = kb[0];
      r[0] += K * x.x;
      r[1] += K * x.y;
      r[2] += K * x.z;
      if (R2) {
        // the div-div term follows below, element by element
      } else if (ADJ) {
        q[0] += kb[1] * x.x + kb[2] * x.y + kb[3] * x.z;
        q[1] += kb[4] * x.x + kb[5] * x.y + kb[6] * x.z;
        q[2] += kb[7] * x.x + kb[8] * x.y + kb[9] * x.z;
      } else {
        const float w0 = x.w * x.x, w1 = x.w * x.y, w2 = x.w * x.z;
        r[0] += kb[1] * w0 + kb[2] * w1 + kb[3] * w2;
        r[1] += kb[4] * w0 + kb[5] * w1 + kb[6] * w2;
        r[2] += kb[7] * w0 + kb[8] * w1 + kb[9] * w2;
      }
    }
    if (R2) r2_term(sX, BX, BY, ix + 1, iy + 1, iz + 1, a.h, r);
    else if (ADJ) {
#pragma unroll
      for (int c = 0; c < 3; ++c) r[c] += pem[j] * q[c];
    }
    const float4 x4 = sX[li];
    const float xo[3] = {x4.x, x4.y, x4.z};
    float xn[3], inc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      inc[c] = pc1[j] * pI[j][c] - pc2[j] * r[c];
      xn[c] = xo[c] + inc[c];
      a.I_out[c * n_own + id] = inc[c];
      a.X_out[c * n_own + id] = xn[c];
    }
    if (a.fd_out) {
      const int gi = a.own_grid[id];
      if (gi >= 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) a.fd_out[c * a.N + gi] = xn[c];
      }
    }
    // the saved forward state is read back only by the adjoint, much later: streamed past
    // the caches (non-temporal), as are the adjoint's reads of it
    if (!ADJ && a.ck_X) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        __builtin_nontemporal_store(xn[c], a.ck_X + c * n_own + id);
        __builtin_nontemporal_store(inc[c], a.ck_I + c * n_own + id);
      }
    }
    if (ENERGY) {
      const double me = a.mass_d[id] * (1.0 + (double)pem[j]);
      double vv = 0.0, er = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        vv += (double)inc[c] * (double)inc[c];
        er += (double)xn[c] * (double)r[c];
      }
      eacc += me * a.inv_2dt2 * vv + 0.5 * er;
    }
    if (ADJ && a.own_grid[id] < 0) {
      const double m = a.mass_d[id];
      double ge = 0.0, gm = 0.0, gs = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double wv = (double)__builtin_nontemporal_load(a.wV + c * n_own + id);
        // R2: the div-div part of the eps gradient is added by the paper-formula kernel
        if (!R2) ge += (double)q[c] * (double)__builtin_nontemporal_load(a.wE + c * n_own + id);
        gm += (double)inc[c] * wv;
        gs += (double)xn[c] * (wv + (double)__builtin_nontemporal_load(a.wVm + c * n_own + id));
      }
      // one contribution per node and launch: the device-side FP64 add (no value returned,
      // so nothing waits for it) rounds once, exactly like a load-add-store
      unsafeAtomicAdd(a.g_eps + id, ge + m * a.inv_dt2 * gm);
      unsafeAtomicAdd(a.g_sig + id, m * a.inv_2dt * gs);
    }
  }
  if (ENERGY) {
    red[tid] = eacc;
    __syncthreads();
    for (int w = STENCIL_THREADS / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) a.epart[a.epart_off + p] = red[0];
  }
}

// Partition of FEM block b of a range of `blocks` (a multiple of N_XCD) blocks: blocks are
// dealt to the XCDs round-robin, so consecutive partitions, whose staging boxes overlap,
// are given to one XCD and share its L2 (in reverse order on alternate steps).
__device__ __forceinline__ int fem_part_of_block(int b, int blocks, int rev) {
  const int per = blocks / N_XCD;
  return (b % N_XCD) * per + (rev ? per - 1 - b / N_XCD : b / N_XCD);
}

template <bool ADJ, bool ENERGY, bool R2>
__global__ __launch_bounds__(STENCIL_THREADS) void fem_stencil_kernel(FemArgs a) {
  const int p = fem_part_of_block(blockIdx.x, gridDim.x, a.rev);
  if (p < a.n_part) fem_stencil_part<ADJ, ENERGY, R2>(a, p);
}

// One launch per time step: blocks [0, fem_blocks) advance the FEM partitions (scheduled
// first: their staging is latency-bound), the remaining blocks the finite-difference
// tiles.  Both read level n and write level n+1 only, so they need no ordering.
template <bool ADJ, bool ENERGY, bool NT, bool OBL = false>
__global__ __launch_bounds__(FD_THREADS) void step_kernel(FdArgs fa, FemArgs ea, int fem_blocks) {
  const int b = blockIdx.x;
  if (b < fem_blocks) {
    const int p = fem_part_of_block(b, fem_blocks, ea.rev);
    if (p < ea.n_part) fem_stencil_part<ADJ, ENERGY>(ea, p);
    return;
  }
  fd_tile<ENERGY, NT, OBL>(fa, b - fem_blocks);
}

// The same fused step on a general mesh: the FEM partitions run the element-coloured code
// (elements read from global memory, so that a block's LDS stays small enough for the
// finite-difference tiles of the same launch to share the CUs; GATHER: the gather form).
// Held to 5 waves per SIMD (at most 96 VGPRs): the adjoint's element sums would otherwise take
// about 105 and leave the FD tiles of the same launch 4 waves.
template <bool ADJ, bool ENERGY, bool NT, bool OBL, bool GEOM_LDS, bool GATHER>
__global__ __launch_bounds__(FD_THREADS, 5) void step_kernel_el(FdArgs fa, FemArgs ea, int fem_blocks) {
  static_assert(FD_THREADS == FEM_THREADS, "one block size for both parts");
  const int b = blockIdx.x;
  if (b < fem_blocks) {
    const int p = fem_part_of_block(b, fem_blocks, ea.rev);
    if (p < ea.n_part) fem_el_part<ADJ, ENERGY, GEOM_LDS, false, GATHER>(ea, p);
    return;
  }
  fd_tile<ENERGY, NT, OBL, true>(fa, b - fem_blocks);
}

// ---------------------------------------------------------------------------------------
// Temporal blocking of the finite-difference region: two steps per launch.
// A far tile (no node of the closed FEM box among its own) advances its 32 x 8 columns over a
// z-chunk of tb_zc planes from level n to n+2.  Per plane it recomputes level n+1 on the tile
// plus a one-node ring, from level n on the tile plus two rings; one plane behind, it forms
// level n+2 on the tile from those values.  A level-n+1 value on the ring is the FD update
// of a node outside the open FEM box (at most a layer-0 node, whose stencil reads the
// layer-1 value of level n that the FEM wrote into the grid), so nothing it needs comes from
// this launch's FEM partitions.  Levels n-1 and n are read, n+1 and n+2 written, in four
// distinct buffers, so no tile reads a value another tile writes in the same launch.  The
// FD fields then move 24 B per node and step instead of 36.  Near tiles, and the second
// launch of a pair, take one step with the same code (ONE).
// Lanes: the tile node (tid % 32, tid / 32); lanes [0, TB_RING1) also a ring-1 node (rows y0-1
// and y0+8, then columns x0-1 and x0+32).  The level-n planes z-1 .. z+2 (tile plus two rings,
// loaded by all lanes, one plane ahead) and the level-n+1 planes z-2 .. z (tile plus one ring)
// sit in LDS; two barriers per plane (after the level-n plane is in, after level n+1 is).
// Measured on MI355X the one-step launches are faster (the grids whose fields the last-level
// cache holds are not bandwidth-bound, and the recomputed ring and end planes cost a third
// more node updates), so the two-step launches are an option (DD_TB=1 at dd_create).
// ---------------------------------------------------------------------------------------

// Per-column data of a node: its (x, y), the outer-face flags of x and y, and whether the
// column holds the dipole node.
struct FdCol {
  int x, y;
  bool bxl, bxh, byl, byh, dip;
};
__device__ __forceinline__ FdCol fd_col(const FdArgs& a, int x, int y, int dip_x, int dip_y) {
  FdCol c;
  c.x = x; c.y = y;
  c.bxl = x == 0; c.bxh = x == a.nx - 1; c.byl = y == 0; c.byh = y == a.ny - 1;
  c.dip = x == dip_x && y == dip_y;
  return c;
}

// One node's three-level update (the arithmetic of fd_tile, in the same order, so that both
// paths round alike): xc its level-n value, xm / xp, ym / yp, zm / zp the neighbours (ignored
// across the outer box's faces), pv the previous level; the next level in xn and the node's
// detector index (or -1) in det.  INT: a node with no outer face and no dipole, where the
// mirror weights are 1 and there is no forcing, damping or detector.
template <bool OBL, bool INT>
__device__ __forceinline__ void fd_point(const FdArgs& a, const FdStepData& sd, const FdCol& cl, int z, int dip_z,
                                         const float xc[3], const float xm[3], const float xp[3], const float ym[3],
                                         const float yp[3], const float zm[3], const float zp[3], const float pv[3],
                                         float xn[3], int64_t& det) {
#pragma clang fp contract(off)
  det = -1;
  if (INT) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float v = xc[c];
      const float sx = (v - xm[c]) + (v - xp[c]);
      const float sy = (v - ym[c]) + (v - yp[c]);
      const float sz = (v - zm[c]) + (v - zp[c]);
      const float S = (sx + sy) + sz;
      xn[c] = v + __builtin_fmaf(-a.nu2, S, v - pv[c]);
    }
    return;
  }
  const int nz = a.nz;
  const bool bxl = cl.bxl, bxh = cl.bxh, byl = cl.byl, byh = cl.byh, bzl = z == 0, bzh = z == nz - 1;
  const float wx = (bxl || bxh) ? 2.f : 1.f;
  const float wy = (byl || byh) ? 2.f : 1.f;
  const float wz = (bzl || bzh) ? 2.f : 1.f;
  float S[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float v = xc[c];
    const float sx = (bxl ? 0.f : v - xm[c]) + (bxh ? 0.f : v - xp[c]);
    const float sy = (byl ? 0.f : v - ym[c]) + (byh ? 0.f : v - yp[c]);
    const float sz = (bzl ? 0.f : v - zm[c]) + (bzh ? 0.f : v - zp[c]);
    S[c] = __builtin_fmaf(wz, sz, __builtin_fmaf(wy, sy, wx * sx));
  }
  float src[3] = {0.f, 0.f, 0.f};
  int na = 0, nb = 0;
  if (bxl || bxh || byl || byh || bzl || bzh) {
    const int bcount = (int)(bxl || bxh) + (int)(byl || byh) + (int)(bzl || bzh);
    const unsigned am = a.abs_mask;
    const int fixed = ((am & DD_FACE_BOTTOM) && bzl) + ((am & DD_FACE_XMIN) && bxl) + ((am & DD_FACE_XMAX) && bxh) +
                      ((am & DD_FACE_YMIN) && byl) + ((am & DD_FACE_YMAX) && byh);
    const int top = (am & DD_FACE_TOP) && bzh;
    na = fixed + top * sd.top_a;
    nb = fixed + top * sd.top_b;
    if (bzh) {
      src[0] += sd.pw[0];
      src[1] += sd.pw[1];
      src[2] += sd.pw[2];
      if (OBL && sd.pw_kind) {
        const float pvl = oblique_pulse_at(a, sd.pw_kind, sd.pw_t, cl.x, cl.y);
        src[0] += a.pw_amp[0] * pvl;
        src[1] += a.pw_amp[1] * pvl;
        src[2] += a.pw_amp[2] * pvl;
      }
    }
    if (a.det_mask) det = face_lex_index(cl.x, cl.y, z, a.nx, a.ny, nz, a.det_mask);
    if (det >= 0 && sd.cot_in) {
      const float sc2 = a.dt2_h3 * (float)(1 << bcount);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float r = sd.obs_in ? sd.cot_in[det * 3 + c] - sd.obs_in[det * 3 + c] : sd.cot_in[det * 3 + c];
        src[c] -= r * sc2;
      }
    }
  }
  if (cl.dip && z == dip_z) {
#pragma unroll
    for (int c = 0; c < 3; ++c) src[c] += sd.dip[c];
  }
  float out[3];
  if (na == 0 && nb == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = __builtin_fmaf(-a.nu2, S[c], xc[c] - pv[c]) + src[c];
  } else {
    const float ba = a.nu * (float)na, bb = a.nu * (float)nb;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      out[c] = ((1.f - bb) * (xc[c] - pv[c]) - a.nu2 * S[c] + src[c] - (ba - bb) * xc[c]) / (1.f + ba);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) xn[c] = xc[c] + out[c];
}

__device__ __forceinline__ bool fd_fem_owned(const FdArgs& a, int x, int y, int z) {
  return x > a.blo[0] && x < a.bhi[0] && y > a.blo[1] && y < a.bhi[1] && z > a.blo[2] && z < a.bhi[2];
}

// LDS of a one-step tile (ONE): the level-n planes only
constexpr size_t TB_LDS_ONE_BYTES = (size_t)4 * 3 * TB_LX * TB_LY * 4;

// The march of one tile (see above); INT (two steps only): the level-n+1 region touches no
// outer face and holds no dipole node, so every node takes the interior update.
template <bool ONE, bool NT, bool OBL, bool INT>
__device__ __forceinline__ void fd_tile2_march(const FdArgs& a, const int t) {
#pragma clang fp contract(off)
  constexpr int ZC = tb_zc(NT);
  constexpr int CN = TB_LX * TB_LY, CU = TB_EX * TB_EY;   // component strides of the LDS planes
  constexpr int NL = (CN + FD_THREADS - 1) / FD_THREADS;  // level-n plane nodes per lane (2)
  extern __shared__ __align__(16) unsigned char lds[];
  float* sN = reinterpret_cast<float*>(lds);            // [4][3][TB_LY][TB_LX]: level n, planes z-1..z+2
  float* sU = sN + 4 * 3 * CN;                          // [3][3][TB_EY][TB_EX]: level n+1, planes z-2..z
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int bx = t % a.nbx, by = (t / a.nbx) % a.nby, bz = t / (a.nbx * a.nby);
  const int x0 = bx * FD_TX, y0 = by * FD_TY, z0 = bz * ZC;
  const int z1 = min(z0 + ZC, nz);
  const int tid = threadIdx.x;
  const int tx = tid % FD_TX, ty = tid / FD_TX;
  const int ox = x0 + tx, oy = y0 + ty;                 // the lane's tile node
  const bool o_col = ox < nx && oy < ny;
  // the lane's ring-1 node (lanes [0, TB_RING1)), in level-n plane coordinates
  int alx = 1, aly = 1;
  const bool ring1 = !ONE && tid < TB_RING1;
  if (ring1) {
    const int r = tid;
    if (r < TB_EX) { alx = r + 1; aly = 1; }
    else if (r < 2 * TB_EX) { alx = r - TB_EX + 1; aly = TB_EY; }
    else if (r < 2 * TB_EX + FD_TY) { alx = 1; aly = 2 + r - 2 * TB_EX; }
    else { alx = TB_EX; aly = 2 + r - 2 * TB_EX - FD_TY; }
  }
  const int ax = x0 - 2 + alx, ay = y0 - 2 + aly;
  const bool a_col = ring1 && ax >= 0 && ax < nx && ay >= 0 && ay < ny;
  int dip_x = -1, dip_y = -1, dip_z = -1;
  if (!INT && a.dip_idx >= 0) {
    dip_x = (int)(a.dip_idx % nx);
    dip_y = (int)((a.dip_idx / nx) % ny);
    dip_z = (int)(a.dip_idx / ((int64_t)nx * ny));
  }
  const FdCol co = fd_col(a, ox, oy, dip_x, dip_y), ca = fd_col(a, ax, ay, dip_x, dip_y);
  const bool o_box = ox > a.blo[0] && ox < a.bhi[0] && oy > a.blo[1] && oy < a.bhi[1];
  const uint32_t plane4 = 4u * (uint32_t)(nx * ny);
  const uint32_t oc4 = o_col ? 4u * (uint32_t)(oy * nx + ox) : 0u;
  const uint32_t ac4 = a_col ? 4u * (uint32_t)(ay * nx + ax) : 0u;
  // the level-n plane nodes this lane loads: plane positions tid and tid + FD_THREADS
  uint32_t lc4[NL];
  bool l_ok[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int i = tid + q * FD_THREADS;
    const int gx = x0 - 2 + i % TB_LX, gy = y0 - 2 + i / TB_LX;
    l_ok[q] = i < CN && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    lc4[q] = l_ok[q] ? 4u * (uint32_t)(gy * nx + gx) : 0u;
  }
  const size_t comp = (size_t)a.N * 4;
  const char* X0 = reinterpret_cast<const char*>(a.X_in);
  const char* Q0 = reinterpret_cast<const char*>(a.X_prev ? a.X_prev : a.X_out);
  char* P0 = reinterpret_cast<char*>(a.X_out);
  char* R0 = reinterpret_cast<char*>(a.X_out2);
  FdStepData s1;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s1.pw[c] = a.pw[c];
    s1.dip[c] = a.dip[c];
  }
  s1.top_a = a.top_a; s1.top_b = a.top_b; s1.pw_kind = a.pw_kind; s1.pw_t = a.pw_t;
  s1.tr_out = a.tr_out; s1.cot_in = a.cot_in; s1.obs_in = a.obs_in;

  // level n+1 is formed on planes [zs, ze); level n is read on [zs - 1, ze]
  const int zs = ONE ? z0 : z0 - 1, ze = ONE ? z1 : z1 + 1;
  float ln[NL][3], lp[3], la[3];   // loads in flight: level n (plane z+3), level n-1 (plane z+1)
  auto load_n = [&](int z) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const bool ok = l_ok[q] && z >= 0 && z < nz && z <= ze;
      const uint32_t o = (uint32_t)z * plane4 + lc4[q];
#pragma unroll
      for (int c = 0; c < 3; ++c) ln[q][c] = ok ? ld_at(X0 + c * comp, o) : 0.f;
    }
  };
  auto store_n = [&](int z) {
    float* sn = sN + (z & 3) * 3 * CN;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int i = tid + q * FD_THREADS;
      if (i < CN) {
#pragma unroll
        for (int c = 0; c < 3; ++c) sn[c * CN + i] = ln[q][c];
      }
    }
  };
  auto load_p = [&](int z) {
    const bool ok = o_col && z >= 0 && z < nz && z < ze;
    const bool oka = a_col && z >= 0 && z < nz && z < ze;
    const uint32_t o = (uint32_t)z * plane4;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lp[c] = ok ? ld_own<NT>(Q0 + c * comp, o + oc4) : 0.f;
      la[c] = oka ? ld_at(Q0 + c * comp, o + ac4) : 0.f;
    }
  };
  const int oq = (ty + 2) * TB_LX + tx + 2, aq = aly * TB_LX + alx;
  const int ou = (ty + 1) * TB_EX + tx + 1, au = (aly - 1) * TB_EX + (alx - 1);
  load_n(zs - 1);
  store_n(zs - 1);
  load_n(zs);
  store_n(zs);
  load_n(zs + 1);
  store_n(zs + 1);
  load_n(zs + 2);   // in flight for a whole iteration: stored at the end of the first one
  load_p(zs);
#pragma unroll 1
  for (int z = zs; z < ze; ++z) {
    float pv[3], pa[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) { pv[c] = lp[c]; pa[c] = la[c]; }
    load_p(z + 1);
    __syncthreads();
    // level n+1 at the tile node, then (two steps) at the ring-1 node; one node at a time, which
    // keeps a single node's operands live.  A two-step tile holds no FEM-owned node.
    float* su = sU + ((z + 3) % 3) * 3 * CU;   // z >= -1: a non-negative slot
    const float* sm = sN + ((z - 1) & 3) * 3 * CN;
    const float* sc = sN + (z & 3) * 3 * CN;
    const float* sp = sN + ((z + 1) & 3) * 3 * CN;
#pragma unroll 1
    for (int r = 0; r < (ONE ? 1 : 2); ++r) {
      const bool tile = r == 0;
      if (!tile && !ring1) break;
      float xn[3] = {0.f, 0.f, 0.f};
      const bool ok = (tile ? o_col : a_col) && z >= 0 && z < nz && (!ONE || !(o_box && z > a.blo[2] && z < a.bhi[2]));
      if (ok) {
        const int q = tile ? oq : aq;
        float xc[3], xm[3], xp[3], ym[3], yp[3], zm[3], zp[3], pp[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float* cc = sc + c * CN + q;
          xc[c] = cc[0]; xm[c] = cc[-1]; xp[c] = cc[1]; ym[c] = cc[-TB_LX]; yp[c] = cc[TB_LX];
          zm[c] = sm[c * CN + q]; zp[c] = sp[c * CN + q];
          pp[c] = tile ? pv[c] : pa[c];
        }
        int64_t det;
        fd_point<OBL, INT>(a, s1, tile ? co : ca, z, dip_z, xc, xm, xp, ym, yp, zm, zp, pp, xn, det);
        if (tile && z >= z0 && z < z1) {
          const uint32_t o = (uint32_t)z * plane4 + oc4;
#pragma unroll
          for (int c = 0; c < 3; ++c) st_own<NT>(P0 + c * comp, o, xn[c]);
          if (!INT && det >= 0 && s1.tr_out) {
#pragma unroll
            for (int c = 0; c < 3; ++c) s1.tr_out[det * 3 + c] = xn[c];
          }
          if (ONE && a.iface_out && ox >= a.blo[0] && ox <= a.bhi[0] && oy >= a.blo[1] && oy <= a.bhi[1] &&
              z >= a.blo[2] && z <= a.bhi[2]) {
            const int64_t l0 = face_lex_index(ox - a.blo[0], oy - a.blo[1], z - a.blo[2], a.fs[0], a.fs[1], a.fs[2], 63u);
            if (l0 >= 0) {
#pragma unroll
              for (int c = 0; c < 3; ++c) a.iface_out[c * a.n_l0 + l0] = xn[c];
            }
          }
        }
      }
      if (!ONE) {
        const int u = tile ? ou : au;
#pragma unroll
        for (int c = 0; c < 3; ++c) su[c * CU + u] = xn[c];
      }
    }
    // the level-n plane z + 2 (loaded one iteration ago) for the next iterations (its slot, that
    // of plane z - 2, was last read before this iteration's first barrier), then plane z + 3
    store_n(z + 2);
    load_n(z + 3);
    if (!ONE) {
      __syncthreads();
      // level n+2 at the tile node, one plane behind
      const int zb = z - 1;
      if (zb >= z0 && zb < z1 && o_col) {
        const float* um = sU + ((zb + 2) % 3) * 3 * CU + ou;   // plane zb - 1 (zb >= 0)
        const float* uc = sU + (zb % 3) * 3 * CU + ou;
        const float* up = sU + ((z + 3) % 3) * 3 * CU + ou;
        float xc[3], xm[3], xp[3], ym[3], yp[3], zm[3], zp[3], pv2[3], x2[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float* cc = uc + c * CU;
          xc[c] = cc[0]; xm[c] = cc[-1]; xp[c] = cc[1]; ym[c] = cc[-TB_EX]; yp[c] = cc[TB_EX];
          zm[c] = um[c * CU]; zp[c] = up[c * CU];
          pv2[c] = sm[c * CN + oq];   // level n at plane zb
        }
        int64_t det;
        fd_point<OBL, INT>(a, a.s2, co, zb, dip_z, xc, xm, xp, ym, yp, zm, zp, pv2, x2, det);
        const uint32_t o = (uint32_t)zb * plane4 + oc4;
#pragma unroll
        for (int c = 0; c < 3; ++c) st_own<NT>(R0 + c * comp, o, x2[c]);
        if (!INT && det >= 0 && a.s2.tr_out) {
#pragma unroll
          for (int c = 0; c < 3; ++c) a.s2.tr_out[det * 3 + c] = x2[c];
        }
      }
    }
  }
}

// A tile of a two-step launch: ONE, one step (near tiles); else two, by the interior update
// where the tile's level-n+1 region (the tile, a one-node ring and one plane beyond each end
// of its chunk) touches no outer face and holds no dipole node.
template <bool ONE, bool NT, bool OBL>
__device__ __forceinline__ void fd_tile2(const FdArgs& a, const int t) {
  if (ONE) {
    fd_tile2_march<true, NT, OBL, false>(a, t);
    return;
  }
  constexpr int ZC = tb_zc(NT);
  const int bx = t % a.nbx, by = (t / a.nbx) % a.nby, bz = t / (a.nbx * a.nby);
  const int x0 = bx * FD_TX, y0 = by * FD_TY, z0 = bz * ZC;
  const int z1 = min(z0 + ZC, a.nz);
  bool in = x0 - 1 >= 1 && x0 + FD_TX <= a.nx - 2 && y0 - 1 >= 1 && y0 + FD_TY <= a.ny - 2 && z0 - 1 >= 1 &&
            z1 <= a.nz - 2;
  if (in && a.dip_idx >= 0) {
    const int dx = (int)(a.dip_idx % a.nx), dy = (int)((a.dip_idx / a.nx) % a.ny);
    const int dz = (int)(a.dip_idx / ((int64_t)a.nx * a.ny));
    in = !(dx >= x0 - 1 && dx <= x0 + FD_TX && dy >= y0 - 1 && dy <= y0 + FD_TY && dz >= z0 - 1 && dz <= z1);
  }
  if (in)
    fd_tile2_march<false, NT, OBL, true>(a, t);
  else
    fd_tile2_march<false, NT, OBL, false>(a, t);
}

// Two-step launches (temporal blocking).  pair_a = 1: blocks [0, fem_blocks) the FEM
// partitions' step n, then the two-step tile grid: far tiles steps n and n+1, near tiles step
// n.  pair_a = 0: the FEM partitions' step n+1 and the near tiles (fa.tb_list) step n+1.
template <bool ADJ, bool NT, bool OBL>
__global__ __launch_bounds__(FD_THREADS) void step_pair_kernel(FdArgs fa, FemArgs ea, int fem_blocks, int pair_a) {
  const int b = blockIdx.x;
  if (b < fem_blocks) {
    const int p = fem_part_of_block(b, fem_blocks, ea.rev);
    if (p < ea.n_part) fem_stencil_part<ADJ, false>(ea, p);
    return;
  }
  const int f = b - fem_blocks;
  if (pair_a) {
    const int kx = fa.rev ? fa.tb_per_xcd - 1 - f / N_XCD : f / N_XCD;
    const int t = (f % N_XCD) * fa.tb_per_xcd + kx;
    if (t >= fa.tb_ntiles) return;
    const int c = tb_tile_class(t, fa.nbx, fa.nby, fa.nx, fa.ny, fa.nz, tb_zc(NT), fa.blo, fa.bhi);
    if (c == 2) fd_tile2<false, NT, OBL>(fa, t);
    else if (c == 1) fd_tile2<true, NT, OBL>(fa, t);
  } else if (f < fa.tb_nlist) {
    fd_tile2<true, NT, OBL>(fa, fa.tb_list[f]);
  }
}

// The adjoint step of the form R1 with the paper-formula variant on: it also carries the
// variant's div-div gradient terms of its input level (blocks [fem_blocks, fem_blocks +
// pg_blocks), pg_tile), which read lambda^k and the saved E^k that the step does not write.
template <bool NT>
__global__ __launch_bounds__(FD_THREADS) void step_kernel_pg(FdArgs fa, FemArgs ea, int fem_blocks, PgArgs pg,
                                                             int pg_blocks) {
  const int b = blockIdx.x;
  if (b < fem_blocks) {
    const int p = fem_part_of_block(b, fem_blocks, ea.rev);
    if (p < ea.n_part) fem_stencil_part<true, false>(ea, p);
    return;
  }
  if (b < fem_blocks + pg_blocks) {
    if (b - fem_blocks < pg_tiles(pg.fs)) pg_tile(pg, b - fem_blocks);
    return;
  }
  fd_tile<false, NT>(fa, b - fem_blocks - pg_blocks);
}

// The same step with the FEM rows in the div-div form R2 (about 73 VGPRs, 6 waves per SIMD,
// with r2_term's cell loop unrolled four at a time).  An adjoint step also carries the
// div-div gradient terms of its input level (blocks [fem_blocks, fem_blocks + pg_blocks),
// pg_tile): they read lambda^k and the saved E^k, which the step does not write.
template <bool ADJ, bool ENERGY, bool NT, bool OBL = false>
__global__ __launch_bounds__(FD_THREADS) void step_kernel_r2(FdArgs fa, FemArgs ea, int fem_blocks, PgArgs pg,
                                                                  int pg_blocks) {
  const int b = blockIdx.x;
  if (b < fem_blocks) {
    const int p = fem_part_of_block(b, fem_blocks, ea.rev);
    if (p < ea.n_part) fem_stencil_part<ADJ, ENERGY, true>(ea, p);
    return;
  }
  if (ADJ && b < fem_blocks + pg_blocks) {
    if (b - fem_blocks < pg_tiles(pg.fs)) pg_tile(pg, b - fem_blocks);
    return;
  }
  fd_tile<ENERGY, NT, OBL>(fa, b - fem_blocks - pg_blocks);
}

// One job's adjoint step together with the next FEM-only recompute step of the segment before
// it (which writes the other window), arguments by value: blocks [0, fem_blocks) the adjoint
// FEM partitions, [fem_blocks, fem_blocks + rec_blocks) the recompute partitions, the rest the
// FD tiles.  The same device code as the batched launch of these two items, without the item
// lookup; held to 6 waves per SIMD like the batched kernel (the union of the forward and
// adjoint FEM variants).
template <bool NT>
__global__ __launch_bounds__(FD_THREADS, 6) void step_rec_kernel(FdArgs fa, FemArgs ea, int fem_blocks, FemArgs er,
                                                                   int rec_blocks) {
  const int b = blockIdx.x;
  if (b < fem_blocks) {
    const int p = fem_part_of_block(b, fem_blocks, ea.rev);
    if (p < ea.n_part) fem_stencil_part<true, false>(ea, p);
    return;
  }
  if (b < fem_blocks + rec_blocks) {
    const int p = fem_part_of_block(b - fem_blocks, rec_blocks, er.rev);
    if (p < er.n_part) fem_stencil_part<false, false>(er, p);
    return;
  }
  fd_tile<false, NT>(fa, b - fem_blocks - rec_blocks);
}

void launch_step_rec(const FdArgs& fa, const FemArgs& ea, const FemArgs& er, hipStream_t s, bool nt) {
  const int fem_blocks = (ea.n_part + N_XCD - 1) / N_XCD * N_XCD;
  const int rec_blocks = (er.n_part + N_XCD - 1) / N_XCD * N_XCD;
  const dim3 grid(fem_blocks + rec_blocks + fa.per_xcd * N_XCD);
  const size_t lds = std::max(stencil_lds(ea), stencil_lds(er));   // the items may be of two problems
  if (nt)
    hipLaunchKernelGGL((step_rec_kernel<true>), grid, dim3(FD_THREADS), lds, s, fa, ea, fem_blocks, er, rec_blocks);
  else
    hipLaunchKernelGGL((step_rec_kernel<false>), grid, dim3(FD_THREADS), lds, s, fa, ea, fem_blocks, er, rec_blocks);
}

// ---------------------------------------------------------------------------------------
// Batched step: one launch advances every active job of a batch by one time step.  Item i
// covers blocks [base_i, base_{i+1}): its FEM partitions first, then its FD tiles
// (fem_blocks_i and base_i are multiples of N_XCD, keeping each item's tile-to-XCD
// mapping).  kind: 0 forward step, 1 adjoint step, 2 forward FEM-only recompute step.
// Items live in device memory (uniform per block: scalar loads); their first blocks are
// kernel arguments.  (Measured: putting the FEM blocks of all items ahead of all FD tiles
// is slower than this per-item order.)  The forward and adjoint FEM variants share this
// kernel; without the occupancy bound the compiler allocates registers for their union
// (93 VGPRs, 5 waves per SIMD instead of 6).
// ---------------------------------------------------------------------------------------
template <bool NT, bool OBL>
__global__ __launch_bounds__(FD_THREADS, 6) void batch_step_kernel(const BatchItem* __restrict__ items, BatchBases bb) {
  const int b = blockIdx.x;
  // the item whose block range holds b: binary search over the bases in the arguments
  int lo = 0, hi = bb.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bb.base[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const BatchItem& it = items[lo];
  const int local = b - bb.base[lo];
  if (local < it.fem_blocks) {
    const int p = fem_part_of_block(local, it.fem_blocks, it.ea.rev);
    if (p < it.ea.n_part) {
      if (it.kind == 1)
        fem_stencil_part<true, false>(it.ea, p);
      else
        fem_stencil_part<false, false>(it.ea, p);
    }
    return;
  }
  if (local - it.fem_blocks < it.fd_blocks) fd_tile<false, NT, OBL>(it.fa, local - it.fem_blocks);
}

void launch_batch(const BatchItem* items_dev, const BatchBases& bases, size_t lds, hipStream_t s, bool nt, bool obl) {
  const dim3 grid(bases.base[bases.n]);
  if (nt && obl)
    hipLaunchKernelGGL((batch_step_kernel<true, true>), grid, dim3(FD_THREADS), lds, s, items_dev, bases);
  else if (nt)
    hipLaunchKernelGGL((batch_step_kernel<true, false>), grid, dim3(FD_THREADS), lds, s, items_dev, bases);
  else if (obl)
    hipLaunchKernelGGL((batch_step_kernel<false, true>), grid, dim3(FD_THREADS), lds, s, items_dev, bases);
  else
    hipLaunchKernelGGL((batch_step_kernel<false, false>), grid, dim3(FD_THREADS), lds, s, items_dev, bases);
}

size_t stencil_lds(const FemArgs& a) {
  return (size_t)a.lds_box * 16 + 12 * 4 * STENCIL_SLOTS_MAX + 4 * STENCIL_SLOTS_MAX;
}

// ---------------------------------------------------------------------------------------
// Helpers
// ---------------------------------------------------------------------------------------
__global__ void energy_reduce_kernel(const double* __restrict__ part, int n, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void fill_f32_kernel(float* p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void copy_f32_kernel(float* __restrict__ d, const float* __restrict__ s, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) d[i] = s[i];
}

// eq. epsilon_sigma_constraint on the FEM nodes: eps = 1, sigma = 0 on lattice layers 0-1,
// eps >= 1, sigma >= 0 and finite everywhere.  The n_extra nodes after the lattice (a caller
// mesh) lie strictly inside layer 1's shell and are free.
__global__ void validate_kernel(const float* eps, const float* sig, int fsx, int fsy, int fsz, int64_t n_extra,
                                int* err) {
  const int64_t n_lat = (int64_t)fsx * fsy * fsz, n = n_lat + n_extra;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int lay = 2;
    if (i < n_lat) {
      const int x = (int)(i % fsx), y = (int)((i / fsx) % fsy), z = (int)(i / ((int64_t)fsx * fsy));
      lay = min(x, fsx - 1 - x);
      lay = min(lay, min(y, fsy - 1 - y));
      lay = min(lay, min(z, fsz - 1 - z));
    }
    const float e = eps[i], s = sig[i];
    bool bad = !(isfinite(e) && isfinite(s)) || e < 1.f || s < 0.f;
    if (lay <= 1 && (e != 1.f || s != 0.f)) bad = true;
    if (bad) atomicAdd(err, 1);
  }
}

// guard (nullable): the validation count of these coefficients; nothing is written when it is
// nonzero (the previous coefficients stay)
__global__ void coefficients_kernel(const float* eps, const float* sig, const int* own_api, const double* mass,
                                    int64_t n_own, double dt, float* em1, float* c1, float* c2, float* sig_own,
                                    const int* guard) {
  if (guard && *guard) return;
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < n_own; id += (int64_t)gridDim.x * blockDim.x) {
    const int api = own_api[id];
    const double e = (double)eps[api], s = (double)sig[api], m = mass[id];
    const double aa = m * e / (dt * dt), bb = m * s / (2.0 * dt);
    em1[id] = (float)(e - 1.0);   // exact: eps >= 1 is a float32 value
    c1[id] = (float)((aa - bb) / (aa + bb));
    c2[id] = (float)(1.0 / (aa + bb));
    sig_own[id] = sig[api];
  }
}

// Derivative of the Tikhonov term gamma/2 sum_i m_i (c_i - c0_i)^2 on the free nodes,
// added to the gradient arrays (FEM-node order).  eps = 1 + (eps - 1) exactly.
__global__ void tikhonov_add_kernel(const float* em1, const float* sig_own, const int* own_api, const int* own_grid,
                                    const double* mass, int64_t n_own, double ge, double gs, const float* eps0,
                                    const float* sig0, double* g_eps, double* g_sig) {
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < n_own; id += (int64_t)gridDim.x * blockDim.x) {
    if (own_grid[id] >= 0) continue;   // layer 1: not free
    const int api = own_api[id];
    const double m = mass[id];
    g_eps[api] += ge * m * ((1.0 + (double)em1[id]) - (double)eps0[api]);
    g_sig[api] += gs * m * ((double)sig_own[id] - (double)sig0[api]);
  }
}

__global__ void gradient_out_kernel(const double* g_eps, const double* g_sig, const int* own_api, const int* own_grid,
                                    int64_t n_own, double* out_eps, double* out_sig) {
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < n_own; id += (int64_t)gridDim.x * blockDim.x) {
    if (own_grid[id] < 0) {
      out_eps[own_api[id]] = g_eps[id];
      out_sig[own_api[id]] = g_sig[id];
    }
  }
}

__global__ void count_nonfinite_kernel(const float* x, int64_t n, int* err) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad += !isfinite(x[i]);
  if (bad) atomicAdd(err, bad);
}

static int grid_for(int64_t n, int block = 256, int cap = 4096) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

template <bool NT>
static void launch_fd_t(const FdArgs& a, hipStream_t s, bool energy) {
  const int grid = a.per_xcd * N_XCD;
  const bool obl = a.pw_kind != 0;
  if (energy && obl)
    hipLaunchKernelGGL((fd_step_kernel<true, NT, true>), dim3(grid), dim3(FD_THREADS), 0, s, a);
  else if (energy)
    hipLaunchKernelGGL((fd_step_kernel<true, NT, false>), dim3(grid), dim3(FD_THREADS), 0, s, a);
  else if (obl)
    hipLaunchKernelGGL((fd_step_kernel<false, NT, true>), dim3(grid), dim3(FD_THREADS), 0, s, a);
  else
    hipLaunchKernelGGL((fd_step_kernel<false, NT, false>), dim3(grid), dim3(FD_THREADS), 0, s, a);
}

void launch_fd(const FdArgs& a, hipStream_t s, bool energy, bool nt) {
  if (nt)
    launch_fd_t<true>(a, s, energy);
  else
    launch_fd_t<false>(a, s, energy);
}

size_t fem_lds_bytes(const FemArgs& a, bool adj, bool stage) {
  const bool geom_lds = a.n_geom <= FEM_GEOM_LDS;
  // node values; the scatter form's accumulator rows (the gather form sums in registers)
  size_t f = (size_t)a.lds_loc * 4 + (a.gather ? 0 : (size_t)(adj ? 8 : 4) * (a.lds_own + 32));
  f += (stage ? (size_t)a.lds_elem * 2 : 0) + (geom_lds ? (size_t)a.n_geom * GEOM_STRIDE : 0);
  f += FEM_COLORS_MAX + 1;   // colour offsets
  return f * 4;
}

namespace {
int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || cus <= 0)
      cus = 256;
  }
  return cus;
}

template <bool ADJ, bool ENERGY, bool GEOM, bool STAGE, bool GATHER = false>
void launch_fem_v(const FemArgs& a, int n_part, size_t lds, hipStream_t s) {
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)fem_step_kernel<ADJ, ENERGY, GEOM, STAGE, GATHER>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((fem_step_kernel<ADJ, ENERGY, GEOM, STAGE, GATHER>), dim3(n_part), dim3(FEM_THREADS), lds, s,
                     a);
}
}  // namespace

// The elements are staged in LDS when the partitions then still run in one round of blocks
// (160 KB of LDS per CU); otherwise they are read from global memory and more blocks share a CU.
// The gather form reads the elements from global memory.
template <bool ADJ, bool ENERGY>
static void launch_fem_t(const FemArgs& a, int n_part, hipStream_t s) {
  if (a.gather) {
    const size_t lds = fem_lds_bytes(a, ADJ, false);
    if (a.n_geom <= FEM_GEOM_LDS) launch_fem_v<ADJ, ENERGY, true, false, true>(a, n_part, lds, s);
    else launch_fem_v<ADJ, ENERGY, false, false, true>(a, n_part, lds, s);
    return;
  }
  constexpr size_t LDS_CU = 160 * 1024;
  const size_t staged = fem_lds_bytes(a, ADJ, true);
  const bool stage = (int64_t)n_part <= (int64_t)(LDS_CU / staged) * device_cus();
  const size_t lds = stage ? staged : fem_lds_bytes(a, ADJ, false);
  const bool geom = a.n_geom <= FEM_GEOM_LDS;
  if (geom && stage) launch_fem_v<ADJ, ENERGY, true, true>(a, n_part, lds, s);
  else if (geom) launch_fem_v<ADJ, ENERGY, true, false>(a, n_part, lds, s);
  else if (stage) launch_fem_v<ADJ, ENERGY, false, true>(a, n_part, lds, s);
  else launch_fem_v<ADJ, ENERGY, false, false>(a, n_part, lds, s);
}

void launch_fem_fwd(const FemArgs& a, int n_part, hipStream_t s, bool energy) {
  if (energy)
    launch_fem_t<false, true>(a, n_part, s);
  else
    launch_fem_t<false, false>(a, n_part, s);
}

void launch_fem_adj(const FemArgs& a, int n_part, hipStream_t s) { launch_fem_t<true, false>(a, n_part, s); }

static int xcd_round(int n) { return (n + N_XCD - 1) / N_XCD * N_XCD; }

static size_t stencil_lds_bytes(const FemArgs& a) {
  return (size_t)a.lds_box * 16 + 12 * 4 * STENCIL_SLOTS_MAX + 4 * STENCIL_SLOTS_MAX;
}

template <bool R2>
static void launch_fem_stencil_fwd_t(const FemArgs& a, int n_part, hipStream_t s, bool energy) {
  const size_t lds = stencil_lds_bytes(a);
  if (energy)
    hipLaunchKernelGGL((fem_stencil_kernel<false, true, R2>), dim3(xcd_round(n_part)), dim3(STENCIL_THREADS), lds, s, a);
  else
    hipLaunchKernelGGL((fem_stencil_kernel<false, false, R2>), dim3(xcd_round(n_part)), dim3(STENCIL_THREADS), lds, s, a);
}

void launch_fem_stencil_fwd(const FemArgs& a, int n_part, hipStream_t s, bool energy) {
  if (a.r2) launch_fem_stencil_fwd_t<true>(a, n_part, s, energy);
  else launch_fem_stencil_fwd_t<false>(a, n_part, s, energy);
}

void launch_fem_stencil_adj(const FemArgs& a, int n_part, hipStream_t s) {
  if (a.r2)
    hipLaunchKernelGGL((fem_stencil_kernel<true, false, true>), dim3(xcd_round(n_part)), dim3(STENCIL_THREADS),
                       stencil_lds_bytes(a), s, a);
  else
    hipLaunchKernelGGL((fem_stencil_kernel<true, false, false>), dim3(xcd_round(n_part)), dim3(STENCIL_THREADS),
                       stencil_lds_bytes(a), s, a);
}

template <bool NT>
static void launch_step_t(const FdArgs& fa, const FemArgs& ea, hipStream_t s, bool adj, bool energy,
                          const PgArgs* pg) {
  const int fem_blocks = (ea.n_part + N_XCD - 1) / N_XCD * N_XCD;   // keeps FD blocks XCD-aligned
  const dim3 grid(fem_blocks + fa.per_xcd * N_XCD);
  const size_t lds = stencil_lds_bytes(ea);
  if (ea.r2) {
    PgArgs g{};
    int pg_blocks = 0;
    if (adj && pg) {
      g = *pg;
      pg_blocks = (pg_tiles(g.fs) + N_XCD - 1) / N_XCD * N_XCD;
    }
    const dim3 grid_r2(fem_blocks + pg_blocks + fa.per_xcd * N_XCD);
    const size_t lds_r2 = pg_blocks ? std::max(lds, PG_LDS_BYTES) : lds;
    if (adj)
      hipLaunchKernelGGL((step_kernel_r2<true, false, NT>), grid_r2, dim3(FD_THREADS), lds_r2, s, fa, ea, fem_blocks, g,
                         pg_blocks);
    else if (fa.pw_kind && energy)
      hipLaunchKernelGGL((step_kernel_r2<false, true, NT, true>), grid_r2, dim3(FD_THREADS), lds_r2, s, fa, ea,
                         fem_blocks, g, 0);
    else if (fa.pw_kind)
      hipLaunchKernelGGL((step_kernel_r2<false, false, NT, true>), grid_r2, dim3(FD_THREADS), lds_r2, s, fa, ea,
                         fem_blocks, g, 0);
    else if (energy)
      hipLaunchKernelGGL((step_kernel_r2<false, true, NT>), grid_r2, dim3(FD_THREADS), lds_r2, s, fa, ea, fem_blocks,
                         g, 0);
    else
      hipLaunchKernelGGL((step_kernel_r2<false, false, NT>), grid_r2, dim3(FD_THREADS), lds_r2, s, fa, ea, fem_blocks,
                         g, 0);
  } else if (adj && pg) {
    const int pg_blocks = (pg_tiles(pg->fs) + N_XCD - 1) / N_XCD * N_XCD;
    hipLaunchKernelGGL((step_kernel_pg<NT>), dim3(fem_blocks + pg_blocks + fa.per_xcd * N_XCD), dim3(FD_THREADS),
                       std::max(lds, PG_LDS_BYTES), s, fa, ea, fem_blocks, *pg, pg_blocks);
  } else if (adj)
    hipLaunchKernelGGL((step_kernel<true, false, NT>), grid, dim3(FD_THREADS), lds, s, fa, ea, fem_blocks);
  else if (fa.pw_kind && energy)
    hipLaunchKernelGGL((step_kernel<false, true, NT, true>), grid, dim3(FD_THREADS), lds, s, fa, ea, fem_blocks);
  else if (fa.pw_kind)
    hipLaunchKernelGGL((step_kernel<false, false, NT, true>), grid, dim3(FD_THREADS), lds, s, fa, ea, fem_blocks);
  else if (energy)
    hipLaunchKernelGGL((step_kernel<false, true, NT>), grid, dim3(FD_THREADS), lds, s, fa, ea, fem_blocks);
  else
    hipLaunchKernelGGL((step_kernel<false, false, NT>), grid, dim3(FD_THREADS), lds, s, fa, ea, fem_blocks);
}

template <bool NT>
static void launch_pair_t(const FdArgs& fa, const FemArgs& ea, hipStream_t s, bool adj, int pair_a) {
  const int fem_blocks = (ea.n_part + N_XCD - 1) / N_XCD * N_XCD;
  const int fd_blocks = pair_a ? fa.tb_per_xcd * N_XCD : fa.tb_nlist;
  if (fem_blocks + fd_blocks == 0) return;
  const dim3 grid(fem_blocks + fd_blocks);
  const size_t lds = std::max(stencil_lds_bytes(ea), pair_a ? TB_LDS_BYTES : TB_LDS_ONE_BYTES);
  if (adj)
    hipLaunchKernelGGL((step_pair_kernel<true, NT, false>), grid, dim3(FD_THREADS), lds, s, fa, ea, fem_blocks, pair_a);
  else if (fa.pw_kind || fa.s2.pw_kind)
    hipLaunchKernelGGL((step_pair_kernel<false, NT, true>), grid, dim3(FD_THREADS), lds, s, fa, ea, fem_blocks, pair_a);
  else
    hipLaunchKernelGGL((step_pair_kernel<false, NT, false>), grid, dim3(FD_THREADS), lds, s, fa, ea, fem_blocks,
                       pair_a);
}

void launch_step_pair(const FdArgs& fa, const FemArgs& ea, hipStream_t s, bool adj, bool nt, int pair_a) {
  if (nt)
    launch_pair_t<true>(fa, ea, s, adj, pair_a);
  else
    launch_pair_t<false>(fa, ea, s, adj, pair_a);
}

void launch_step(const FdArgs& fa, const FemArgs& ea, hipStream_t s, bool adj, bool energy, bool nt,
                 const PgArgs* pg) {
  if (nt)
    launch_step_t<true>(fa, ea, s, adj, energy, pg);
  else
    launch_step_t<false>(fa, ea, s, adj, energy, pg);
}

template <bool NT, bool GEOM, bool GATHER>
static void launch_step_el_t(const FdArgs& fa, const FemArgs& ea, hipStream_t s, bool adj, bool energy) {
  const int fem_blocks = (ea.n_part + N_XCD - 1) / N_XCD * N_XCD;   // keeps FD blocks XCD-aligned
  const dim3 grid(fem_blocks + fa.per_xcd * N_XCD);
  const size_t lds = std::max(fem_lds_bytes(ea, adj, false), FD_DYN_LDS_BYTES);
  if (adj)
    hipLaunchKernelGGL((step_kernel_el<true, false, NT, false, GEOM, GATHER>), grid, dim3(FD_THREADS), lds, s, fa, ea,
                       fem_blocks);
  else if (fa.pw_kind && energy)
    hipLaunchKernelGGL((step_kernel_el<false, true, NT, true, GEOM, GATHER>), grid, dim3(FD_THREADS), lds, s, fa, ea,
                       fem_blocks);
  else if (fa.pw_kind)
    hipLaunchKernelGGL((step_kernel_el<false, false, NT, true, GEOM, GATHER>), grid, dim3(FD_THREADS), lds, s, fa, ea,
                       fem_blocks);
  else if (energy)
    hipLaunchKernelGGL((step_kernel_el<false, true, NT, false, GEOM, GATHER>), grid, dim3(FD_THREADS), lds, s, fa, ea,
                       fem_blocks);
  else
    hipLaunchKernelGGL((step_kernel_el<false, false, NT, false, GEOM, GATHER>), grid, dim3(FD_THREADS), lds, s, fa, ea,
                       fem_blocks);
}

template <bool GATHER>
static void launch_step_el_g(const FdArgs& fa, const FemArgs& ea, hipStream_t s, bool adj, bool energy, bool nt) {
  const bool geom = ea.n_geom <= FEM_GEOM_LDS;
  if (nt && geom) launch_step_el_t<true, true, GATHER>(fa, ea, s, adj, energy);
  else if (nt) launch_step_el_t<true, false, GATHER>(fa, ea, s, adj, energy);
  else if (geom) launch_step_el_t<false, true, GATHER>(fa, ea, s, adj, energy);
  else launch_step_el_t<false, false, GATHER>(fa, ea, s, adj, energy);
}

void launch_step_el(const FdArgs& fa, const FemArgs& ea, hipStream_t s, bool adj, bool energy, bool nt) {
  if (ea.gather)
    launch_step_el_g<true>(fa, ea, s, adj, energy, nt);
  else
    launch_step_el_g<false>(fa, ea, s, adj, energy, nt);
}

void launch_energy_reduce(const double* part, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(energy_reduce_kernel, dim3(1), dim3(256), 0, s, part, n, out);
}

void launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
}

void launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
}

void launch_copy_f32(float* dst, const float* src, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(copy_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, dst, src, n);
}

void launch_validate(const float* eps, const float* sig, int fsx, int fsy, int fsz, int64_t n_extra, int* err,
                     hipStream_t s) {
  hipLaunchKernelGGL(validate_kernel, dim3(grid_for((int64_t)fsx * fsy * fsz + n_extra)), dim3(256), 0, s, eps, sig,
                     fsx, fsy, fsz, n_extra, err);
}

void launch_coefficients(const float* eps, const float* sig, const int* own_api, const double* mass_d, int64_t n_own,
                         double dt, float* em1, float* c1, float* c2, float* sig_own, const int* guard, hipStream_t s) {
  hipLaunchKernelGGL(coefficients_kernel, dim3(grid_for(n_own)), dim3(256), 0, s, eps, sig, own_api, mass_d, n_own, dt,
                     em1, c1, c2, sig_own, guard);
}

__global__ void fill_i32_kernel(int* p, int n, int v) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

void launch_fill_i32(int* p, int n, int v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, p, n, v);
}

void launch_tikhonov_add(const float* em1, const float* sig_own, const int* own_api, const int* own_grid,
                         const double* mass_d, int64_t n_own, double gamma_eps, double gamma_sig, const float* eps0,
                         const float* sig0, double* g_eps, double* g_sig, hipStream_t s) {
  hipLaunchKernelGGL(tikhonov_add_kernel, dim3(grid_for(n_own)), dim3(256), 0, s, em1, sig_own, own_api, own_grid,
                     mass_d, n_own, gamma_eps, gamma_sig, eps0, sig0, g_eps, g_sig);
}

void launch_gradient_out(const double* g_eps, const double* g_sig, const int* own_api, const int* own_grid,
                         int64_t n_own, double* out_eps, double* out_sig, hipStream_t s) {
  hipLaunchKernelGGL(gradient_out_kernel, dim3(grid_for(n_own)), dim3(256), 0, s, g_eps, g_sig, own_api, own_grid,
                     n_own, out_eps, out_sig);
}

void launch_count_nonfinite(const float* x, int64_t n, int* err, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(count_nonfinite_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, err);
}

}  // namespace dd
