// HIP kernels (gfx950) of the hybrid FE/FD leapfrog: finite-difference region,
// FEM region, and the small helpers around them.
//
// Both regions advance the same explicit scheme (increment form of the
// central-difference leapfrog for eq. forward_prob / eq. model1):
//     V^{n+1} = [ (M/dt^2 - C/(2dt)) V^n - A E^n + F^n ] / (M/dt^2 + C/(2dt)),
//     E^{n+1} = E^n + V^{n+1},
// and its exact transpose for the adjoint (eq. adjoint_prob) run backward:
//     Lambda^k = [ (M/dt^2 - C^{k+1}/(2dt)) Lambda^{k+1} - A^T lambda^k - r^k
//                  - (C^{k-1} - C^{k+1}) lambda^k / (2dt) ] / (M/dt^2 + C^{k-1}/(2dt)),
//     lambda^{k-1} = lambda^k + Lambda^k.
// Field state is FP32; the energy and gradient sums are FP64.
#include "dd_common.hpp"

namespace dd {

// ---------------------------------------------------------------------------------------
// Finite-difference region.  eps = 1, sigma = 0 here (eq. epsilon_sigma_constraint), so
// the update is the 7-point wave stencil with mirror (Neumann) weights on the outer box,
// lumped absorbing damping on absorbing faces and the plane-wave / dipole forcing.
// Tile = 32 x 8 nodes in (x, y), marching FD_ZC planes in z: the current plane sits in LDS
// (with a one-node halo), the z-1 and z+1 values of each column stay in registers.
// ---------------------------------------------------------------------------------------
template <bool ENERGY>
__global__ __launch_bounds__(FD_THREADS) void fd_step_kernel(FdArgs a) {
  __shared__ float s[3][FD_TY + 2][FD_TX + 2];
  __shared__ double red[ENERGY ? FD_THREADS : 1];
  const int b = blockIdx.x;
  const int t = (b % N_XCD) * a.per_xcd + b / N_XCD;  // consecutive tiles share an XCD's L2
  if (t >= a.ntiles) return;
  const int bx = t % a.nbx;
  const int by = (t / a.nbx) % a.nby;
  const int bz = t / (a.nbx * a.nby);
  const int x0 = bx * FD_TX, y0 = by * FD_TY, z0 = bz * FD_ZC;
  const int z1 = min(z0 + FD_ZC, a.nz);
  const int tid = threadIdx.x;
  if (x0 > a.blo[0] && x0 + FD_TX - 1 < a.bhi[0] && y0 > a.blo[1] && y0 + FD_TY - 1 < a.bhi[1] &&
      z0 > a.blo[2] && z1 - 1 < a.bhi[2]) {
    // every node of the tile is FEM-owned
    if (ENERGY && tid == 0) a.epart[t] = 0.0;
    return;
  }
  const int tx = tid % FD_TX, ty = tid / FD_TX;
  const int x = x0 + tx, y = y0 + ty;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const bool col_ok = (x < nx) && (y < ny);
  const int64_t N = a.N;
  const int64_t plane = (int64_t)nx * ny;
  const int64_t col = (int64_t)y * nx + x;
  const float* __restrict__ X = a.X_in;

  const bool bxl = x == 0, bxh = x == nx - 1, byl = y == 0, byh = y == ny - 1;
  const float wx = (bxl || bxh) ? 2.f : 1.f;   // 2 / (neighbours along x)
  const float wy = (byl || byh) ? 2.f : 1.f;
  const bool in_box_xy = x > a.blo[0] && x < a.bhi[0] && y > a.blo[1] && y < a.bhi[1];
  const bool in_box_xy_closed = x >= a.blo[0] && x <= a.bhi[0] && y >= a.blo[1] && y <= a.bhi[1];

  float cur[3] = {0.f, 0.f, 0.f}, prv[3] = {0.f, 0.f, 0.f}, nxt[3] = {0.f, 0.f, 0.f};
  if (col_ok) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cur[c] = X[c * N + z0 * plane + col];
      prv[c] = z0 > 0 ? X[c * N + (z0 - 1) * plane + col] : 0.f;
    }
  }
  double eacc = 0.0;
  for (int z = z0; z < z1; ++z) {
    const int64_t zoff = (int64_t)z * plane;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float* Xc = X + c * N + zoff;
      if (col_ok) s[c][ty + 1][tx + 1] = cur[c];
      if (tx == 0 && x0 > 0 && y < ny) s[c][ty + 1][0] = Xc[(int64_t)y * nx + x0 - 1];
      if (tx == FD_TX - 1 && x0 + FD_TX < nx && y < ny) s[c][ty + 1][FD_TX + 1] = Xc[(int64_t)y * nx + x0 + FD_TX];
      if (ty == 0 && y0 > 0 && x < nx) s[c][0][tx + 1] = Xc[(int64_t)(y0 - 1) * nx + x];
      if (ty == FD_TY - 1 && y0 + FD_TY < ny && x < nx) s[c][FD_TY + 1][tx + 1] = Xc[(int64_t)(y0 + FD_TY) * nx + x];
      nxt[c] = (col_ok && z + 1 < nz) ? X[c * N + zoff + plane + col] : 0.f;
    }
    __syncthreads();
    const bool fem_owned = in_box_xy && z > a.blo[2] && z < a.bhi[2];
    if (col_ok && !fem_owned) {
      const bool bzl = z == 0, bzh = z == nz - 1;
      const float wz = (bzl || bzh) ? 2.f : 1.f;
      const int64_t idx = zoff + col;
      float L[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float xc = cur[c];
        float sx = 0.f, sy = 0.f, sz = 0.f;
        if (!bxl) sx += xc - s[c][ty + 1][tx];
        if (!bxh) sx += xc - s[c][ty + 1][tx + 2];
        if (!byl) sy += xc - s[c][ty][tx + 1];
        if (!byh) sy += xc - s[c][ty + 2][tx + 1];
        if (!bzl) sz += xc - prv[c];
        if (!bzh) sz += xc - nxt[c];
        L[c] = a.nu2 * (wx * sx + wy * sy + wz * sz);
      }
      const bool on_bnd = bxl || bxh || byl || byh || bzl || bzh;
      const int bcount = (int)(bxl || bxh) + (int)(byl || byh) + (int)(bzl || bzh);
      float src[3] = {0.f, 0.f, 0.f};
      int na = 0, nb = 0;
      int64_t det = -1;
      if (on_bnd) {
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
        }
        if (a.det_mask) det = face_lex_index(x, y, z, nx, ny, nz, a.det_mask);
        if (det >= 0 && a.cot_in) {
          const float sc = a.dt2_h3 * (float)(1 << bcount);   // dt^2 / m_i
#pragma unroll
          for (int c = 0; c < 3; ++c) src[c] -= a.cot_in[det * 3 + c] * sc;
        }
      }
      if (idx == a.dip_idx) {
#pragma unroll
        for (int c = 0; c < 3; ++c) src[c] += a.dip[c];
      }
      int64_t l0 = -1;
      if (a.iface_out && in_box_xy_closed && z >= a.blo[2] && z <= a.bhi[2])
        l0 = face_lex_index(x - a.blo[0], y - a.blo[1], z - a.blo[2], a.fs[0], a.fs[1], a.fs[2], 63u);
      const float ba = a.nu * (float)na, bb = a.nu * (float)nb;
      double e_node = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float inc = a.I[c * N + idx];
        float out;
        if (na == 0 && nb == 0)
          out = inc - L[c] + src[c];
        else
          out = ((1.f - bb) * inc - L[c] + src[c] - (ba - bb) * cur[c]) / (1.f + ba);
        const float xn = cur[c] + out;
        a.I[c * N + idx] = out;
        a.X_out[c * N + idx] = xn;
        if (det >= 0 && a.tr_out) a.tr_out[det * 3 + c] = xn;
        if (l0 >= 0) a.iface_out[c * a.n_l0 + l0] = xn;
        if (ENERGY) e_node += (double)out * (double)out + (double)xn * (double)L[c];
      }
      if (ENERGY) eacc += a.e_coef * ldexp(1.0, -bcount) * e_node;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      prv[c] = cur[c];
      cur[c] = nxt[c];
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

// ---------------------------------------------------------------------------------------
// FEM region: lumped-mass P1 on tetrahedra (stiffness + div-div stabiliser of eq.
// lagrangian_weak).  One workgroup per partition: the partition's owned and halo node
// values are staged in LDS, elements are evaluated colour by colour and scattered into
// LDS accumulators of the owned nodes, then owned nodes are advanced.
//   forward:  (A E)_i = sum_K |K| [grad phi_i . grad(E_c)|_K + d_c phi_i div_K((eps-1) E)]
//   adjoint:  (A^T l)_i = sum_K |K| grad phi_i . grad(l_c)|_K + (eps_i - 1) q_i,
//             q_i = sum_K |K| grad phi_i div_K(l)
// and the adjoint also accumulates, on free nodes, the gradient of eq. gradeps:
//   g_eps += q_i . E^k_i + (m_i / dt^2) Lambda^k_i . V^k_i,
//   g_sig += (m_i / (2 dt)) lambda^{k-1}_i . (V^k_i + V^{k-1}_i).
// Layer-0 values come from the interface buffer written by the finite-difference kernel;
// layer-1 results are also written into the finite-difference grid (the two-node overlap).
// ---------------------------------------------------------------------------------------
template <bool ADJ, bool ENERGY>
__global__ __launch_bounds__(FEM_THREADS) void fem_step_kernel(FemArgs a) {
  __shared__ float sX[3][FEM_LOC_MAX];
  __shared__ float sM[ADJ ? 1 : FEM_LOC_MAX];
  __shared__ float sA[ADJ ? 6 : 3][FEM_OWN_MAX];
  __shared__ double red[ENERGY ? FEM_THREADS : 1];
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const int o0 = a.own_off[p], no = a.own_off[p + 1] - o0;
  const int h0 = a.halo_off[p], nh = a.halo_off[p + 1] - h0;
  const int nl = no + nh;
  const int64_t n_own = a.n_own, n_l0 = a.n_l0;

  for (int l = tid; l < nl; l += FEM_THREADS) {
    float v0, v1, v2, m = 0.f;
    if (l < no) {
      const int id = o0 + l;
      v0 = a.X_in[id];
      v1 = a.X_in[n_own + id];
      v2 = a.X_in[2 * n_own + id];
      if (!ADJ) m = a.em1[id];
    } else {
      const int hc = a.halo[h0 + l - no];
      if (hc >= 0) {
        v0 = a.X_in[hc];
        v1 = a.X_in[n_own + hc];
        v2 = a.X_in[2 * n_own + hc];
        if (!ADJ) m = a.em1[hc];
      } else {
        const int64_t q = -1 - (int64_t)hc;
        v0 = a.iface_in[q];
        v1 = a.iface_in[n_l0 + q];
        v2 = a.iface_in[2 * n_l0 + q];
      }
    }
    sX[0][l] = v0;
    sX[1][l] = v1;
    sX[2][l] = v2;
    if (!ADJ) sM[l] = m;
  }
  for (int l = tid; l < no; l += FEM_THREADS) {
#pragma unroll
    for (int c = 0; c < (ADJ ? 6 : 3); ++c) sA[c][l] = 0.f;
  }
  __syncthreads();

  const int ncl = a.ncol[p], cb = a.col_base[p];
  for (int c = 0; c < ncl; ++c) {
    const int e0 = a.col_off[cb + c], e1 = a.col_off[cb + c + 1];
    for (int e = e0 + tid; e < e1; e += FEM_THREADS) {
      const uint64_t w = a.elems[e];
      int v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = (int)((w >> (11 * k)) & 0x7FFu);
      const float* g = a.geom + ((w >> 44) << 4);
      float gr[4][3];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int d = 0; d < 3; ++d) gr[j][d] = g[3 * j + d];
      const float vol = g[12];
      float G[3][3];
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int d = 0; d < 3; ++d) G[q][d] = 0.f;
      float dv = 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float e0v = sX[0][v[j]], e1v = sX[1][v[j]], e2v = sX[2][v[j]];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          G[0][d] += e0v * gr[j][d];
          G[1][d] += e1v * gr[j][d];
          G[2][d] += e2v * gr[j][d];
        }
        const float mj = ADJ ? 1.f : sM[v[j]];
        dv += mj * (e0v * gr[j][0] + e1v * gr[j][1] + e2v * gr[j][2]);
      }
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int d = 0; d < 3; ++d) G[q][d] *= vol;
      dv *= vol;
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) {
        const int li = v[sl];
        if (li < no) {
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const float kc = gr[sl][0] * G[q][0] + gr[sl][1] * G[q][1] + gr[sl][2] * G[q][2];
            const float dc = gr[sl][q] * dv;
            if (ADJ) {
              sA[q][li] += kc;
              sA[3 + q][li] += dc;
            } else {
              sA[q][li] += kc + dc;
            }
          }
        }
      }
    }
    __syncthreads();
  }

  double eacc = 0.0;
  for (int l = tid; l < no; l += FEM_THREADS) {
    const int id = o0 + l;
    const float k1 = a.c1[id], k2 = a.c2[id];
    float xn[3], inc[3], r[3];
    if (!ADJ) {
#pragma unroll
      for (int c = 0; c < 3; ++c) r[c] = sA[c][l];
    } else {
      const float em = a.em1[id];
#pragma unroll
      for (int c = 0; c < 3; ++c) r[c] = sA[c][l] + em * sA[3 + c][l];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      inc[c] = k1 * a.I_in[c * n_own + id] - k2 * r[c];
      xn[c] = sX[c][l] + inc[c];
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
    if (!ADJ && a.ck_X) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a.ck_X[c * n_own + id] = xn[c];
        a.ck_I[c * n_own + id] = inc[c];
      }
    }
    if (ENERGY) {
      const double me = a.mass_d[id] * (1.0 + (double)a.em1[id]);
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
        const double wv = (double)a.wV[c * n_own + id];
        ge += (double)sA[3 + c][l] * (double)a.wE[c * n_own + id];
        gm += (double)inc[c] * wv;
        gs += (double)xn[c] * (wv + (double)a.wVm[c * n_own + id]);
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

// eq. epsilon_sigma_constraint on the FEM lattice: eps = 1, sigma = 0 on layers 0-1,
// eps >= 1, sigma >= 0 and finite everywhere.
__global__ void validate_kernel(const float* eps, const float* sig, int fsx, int fsy, int fsz, int* err) {
  const int64_t n = (int64_t)fsx * fsy * fsz;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % fsx), y = (int)((i / fsx) % fsy), z = (int)(i / ((int64_t)fsx * fsy));
    int lay = min(x, fsx - 1 - x);
    lay = min(lay, min(y, fsy - 1 - y));
    lay = min(lay, min(z, fsz - 1 - z));
    const float e = eps[i], s = sig[i];
    bool bad = !(isfinite(e) && isfinite(s)) || e < 1.f || s < 0.f;
    if (lay <= 1 && (e != 1.f || s != 0.f)) bad = true;
    if (bad) atomicAdd(err, 1);
  }
}

__global__ void coefficients_kernel(const float* eps, const float* sig, const int* own_api, const double* mass,
                                    int64_t n_own, double dt, float* em1, float* c1, float* c2) {
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < n_own; id += (int64_t)gridDim.x * blockDim.x) {
    const int api = own_api[id];
    const double e = (double)eps[api], s = (double)sig[api], m = mass[id];
    const double aa = m * e / (dt * dt), bb = m * s / (2.0 * dt);
    em1[id] = (float)(e - 1.0);
    c1[id] = (float)((aa - bb) / (aa + bb));
    c2[id] = (float)(1.0 / (aa + bb));
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

void launch_fd(const FdArgs& a, hipStream_t s, bool energy) {
  const int grid = a.per_xcd * N_XCD;
  if (energy)
    hipLaunchKernelGGL(fd_step_kernel<true>, dim3(grid), dim3(FD_THREADS), 0, s, a);
  else
    hipLaunchKernelGGL(fd_step_kernel<false>, dim3(grid), dim3(FD_THREADS), 0, s, a);
}

void launch_fem_fwd(const FemArgs& a, int n_part, hipStream_t s, bool energy) {
  if (energy)
    hipLaunchKernelGGL((fem_step_kernel<false, true>), dim3(n_part), dim3(FEM_THREADS), 0, s, a);
  else
    hipLaunchKernelGGL((fem_step_kernel<false, false>), dim3(n_part), dim3(FEM_THREADS), 0, s, a);
}

void launch_fem_adj(const FemArgs& a, int n_part, hipStream_t s) {
  hipLaunchKernelGGL((fem_step_kernel<true, false>), dim3(n_part), dim3(FEM_THREADS), 0, s, a);
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

void launch_validate(const float* eps, const float* sig, int fsx, int fsy, int fsz, int* err, hipStream_t s) {
  hipLaunchKernelGGL(validate_kernel, dim3(grid_for((int64_t)fsx * fsy * fsz)), dim3(256), 0, s, eps, sig, fsx, fsy,
                     fsz, err);
}

void launch_coefficients(const float* eps, const float* sig, const int* own_api, const double* mass_d, int64_t n_own,
                         double dt, float* em1, float* c1, float* c2, hipStream_t s) {
  hipLaunchKernelGGL(coefficients_kernel, dim3(grid_for(n_own)), dim3(256), 0, s, eps, sig, own_api, mass_d, n_own, dt,
                     em1, c1, c2);
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
