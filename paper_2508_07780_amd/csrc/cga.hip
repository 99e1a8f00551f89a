// Conjugate gradient update of the coefficients eps and sigma (box "CGA", steps 2-6) on
// the FEM lattice, after the forward / adjoint / gradient solves of step 1.
//
// With the lumped-mass L2 inner product (u, v) = sum_i m_i u_i v_i (m_i = h^3 on every free
// node of the Kuhn split, i.e. layer >= 2; on a general mesh each free node's lumped mass, and
// its extra nodes are free) the gradient function of eq. gradeps at a free node is
//     g_i = (dJ/dc_i) / m_i + gamma^m (c_i - c^0_i),
// the nodal derivative of the trace misfit turned into a function, plus the Tikhonov term
// of eq. tikhonov_functional (centre = the initial guess).  One update then takes
//     beta^m  = |g^m|^2 / |g^{m-1}|^2               (0 at m = 0 or when |g^{m-1}| = 0)
//     d^m     = -g^m + beta^m d^{m-1}
//     c^{m+1} = clamp(c^m + alpha^m d^m, lo, hi)     (the box of eq. epsilon_sigma_constraint)
//     alpha^{m+1} = -(g^m, d^m) / (gamma^m (d^m, d^m))   (alpha^m kept when d^m = 0)
//     gamma^{m+1} = gamma^0 / (m + 1)^p
// and the stop test (|c^{m+1} - c^m| < eta1 for eps or sigma) and (|g^m| < eta2 for eps or
// sigma).  Nodes of layers 0 and 1 are never touched (eps = 1, sigma = 0 there).
//
// The work is a few streaming passes over FEM-node arrays (HBM-bound, a few microseconds
// at the paper's sizes).  Every sum is FP64 and deterministic: each block reduces its
// grid-stride share in a fixed order, one block then adds the block partials in order.
#include <mutex>

#include "cga.hpp"

namespace dd {

// Scratch of the no-allocation misfit (dd_misfit_noalloc): the FP64 block partials of J,
// then the time weights z.  One copy per GPU, held until the process ends.  In host code this
// name is a stand-in, not a device address: kernels and copies take the address from
// misfit_scratch.
static __device__ __align__(256) double scratch[CGA_MAX_BLOCKS + DD_MISFIT_NOALLOC_MAX_STEPS];

namespace {

constexpr int CGA_THREADS = 256;

// Free FEM node: lattice layer >= 2, or one of a general mesh's extra nodes (after the lattice).
__device__ inline bool cga_free(int64_t i, int fsx, int fsy, int fsz) {
  if (i >= (int64_t)fsx * fsy * fsz) return true;
  const int lx = (int)(i % fsx);
  const int64_t r = i / fsx;
  const int ly = (int)(r % fsy);
  const int lz = (int)(r / fsy);
  const int lay = min(min(min(lx, fsx - 1 - lx), min(ly, fsy - 1 - ly)), min(lz, fsz - 1 - lz));
  return lay >= 2;
}

__device__ inline double cga_g(double dJ, double w, float c, float c0, double gamma) {
  return dJ / w + gamma * ((double)c - (double)c0);
}

// Block-wide sums of NQ values per thread, in a fixed order; thread 0 writes them to out.
template <int NQ>
__device__ inline void block_sums(const double (&v)[NQ], double* out) {
  __shared__ double red[NQ][CGA_THREADS];
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < NQ; ++q) red[q][t] = v[q];
  __syncthreads();
  for (int s = CGA_THREADS / 2; s > 0; s >>= 1) {
    if (t < s) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) red[q][t] += red[q][t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) out[q] = red[q][0];
  }
}

// Sums of NQ partials over nb blocks (partials laid out [nb][NQ]).
template <int NQ>
__device__ inline void sum_partials(const double* part, int nb, double* out) {
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  for (int b = threadIdx.x; b < nb; b += CGA_THREADS) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] += part[(int64_t)b * NQ + q];
  }
  block_sums<NQ>(v, out);
}

// |g^m|^2 partials of eps and sigma.
__global__ __launch_bounds__(CGA_THREADS) void cga_norm_kernel(
    const double* __restrict__ gJe, const double* __restrict__ gJs, const float* __restrict__ eps,
    const float* __restrict__ sig, const float* __restrict__ eps0, const float* __restrict__ sig0, int fsx, int fsy,
    int fsz, int64_t n_extra, const double* __restrict__ wn, const CgaDev* __restrict__ st,
    double* __restrict__ part) {
  const int64_t n = (int64_t)fsx * fsy * fsz + n_extra;
  const double gam_e = st->gamma[0], gam_s = st->gamma[1];
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * CGA_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * CGA_THREADS) {
    if (!cga_free(i, fsx, fsy, fsz)) continue;
    const double w = wn ? wn[i] : st->w;
    const double ge = cga_g(gJe[i], w, eps[i], eps0[i], gam_e);
    const double gs = cga_g(gJs[i], w, sig[i], sig0[i], gam_s);
    acc[0] += w * ge * ge;
    acc[1] += w * gs * gs;
  }
  block_sums<2>(acc, part + (int64_t)blockIdx.x * 2);
}

// |g^m|^2 and beta^m (one block).
__global__ __launch_bounds__(CGA_THREADS) void cga_beta_kernel(const double* __restrict__ part, int nb,
                                                               CgaDev* __restrict__ st) {
  __shared__ double tot[2];
  sum_partials<2>(part, nb, tot);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int f = 0; f < 2; ++f) {
      const double gn2 = tot[f];
      st->gn2[f] = gn2;
      st->beta[f] = (st->m > 0 && st->gn2_prev[f] > 0.0) ? gn2 / st->gn2_prev[f] : 0.0;
    }
  }
}

// d^m, c^{m+1} (in place) and the partials of (g, d), (d, d), |c^{m+1} - c^m|^2.
__global__ __launch_bounds__(CGA_THREADS) void cga_step_kernel(
    const double* __restrict__ gJe, const double* __restrict__ gJs, float* __restrict__ eps, float* __restrict__ sig,
    const float* __restrict__ eps0, const float* __restrict__ sig0, double* __restrict__ d_eps,
    double* __restrict__ d_sig, int fsx, int fsy, int fsz, int64_t n_extra, const double* __restrict__ wn,
    const CgaDev* __restrict__ st, double* __restrict__ part) {
  const int64_t n = (int64_t)fsx * fsy * fsz + n_extra;
  const double gam[2] = {st->gamma[0], st->gamma[1]};
  const double beta[2] = {st->beta[0], st->beta[1]};
  const double alpha[2] = {st->alpha[0], st->alpha[1]};
  const double lo[2] = {st->lo[0], st->lo[1]}, hi[2] = {st->hi[0], st->hi[1]};
  double acc[CGA_SUMS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * CGA_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * CGA_THREADS) {
    if (!cga_free(i, fsx, fsy, fsz)) continue;
    const double w = wn ? wn[i] : st->w;
    {
      const float c = eps[i];
      const double g = cga_g(gJe[i], w, c, eps0[i], gam[0]);
      const double d = -g + beta[0] * d_eps[i];
      const float cn = (float)fmin(fmax((double)c + alpha[0] * d, lo[0]), hi[0]);
      d_eps[i] = d;
      eps[i] = cn;
      const double dc = (double)cn - (double)c, dc0 = (double)cn - (double)eps0[i];
      acc[0] += w * g * d;
      acc[1] += w * d * d;
      acc[2] += w * dc * dc;
      acc[6] += w * dc0 * dc0;
    }
    {
      const float c = sig[i];
      const double g = cga_g(gJs[i], w, c, sig0[i], gam[1]);
      const double d = -g + beta[1] * d_sig[i];
      const float cn = (float)fmin(fmax((double)c + alpha[1] * d, lo[1]), hi[1]);
      d_sig[i] = d;
      sig[i] = cn;
      const double dc = (double)cn - (double)c, dc0 = (double)cn - (double)sig0[i];
      acc[3] += w * g * d;
      acc[4] += w * d * d;
      acc[5] += w * dc * dc;
      acc[7] += w * dc0 * dc0;
    }
  }
  block_sums<CGA_SUMS>(acc, part + (int64_t)blockIdx.x * CGA_SUMS);
}

// alpha^{m+1}, gamma^{m+1}, the stop test, m -> m + 1 (one block).
__global__ __launch_bounds__(CGA_THREADS) void cga_finish_kernel(const double* __restrict__ part, int nb,
                                                                 CgaDev* __restrict__ st) {
  __shared__ double tot[CGA_SUMS];
  sum_partials<CGA_SUMS>(part, nb, tot);
  __syncthreads();
  if (threadIdx.x == 0) {
    bool small_step = false, small_grad = false;
    for (int f = 0; f < 2; ++f) {
      const double gd = tot[3 * f], dd = tot[3 * f + 1], step2 = tot[3 * f + 2];
      st->gd[f] = gd;
      st->dd[f] = dd;
      st->step2[f] = step2;
      st->change2[f] = tot[6 + f];
      st->alpha_used[f] = st->alpha[f];
      st->gamma_used[f] = st->gamma[f];
      if (dd > 0.0) st->alpha[f] = -gd / (st->gamma[f] * dd);
      st->gamma[f] = st->gamma0[f] / pow((double)(st->m + 1), st->p);
      st->gn2_prev[f] = st->gn2[f];
      small_step = small_step || sqrt(step2) < st->eta1[f];
      small_grad = small_grad || sqrt(st->gn2[f]) < st->eta2[f];
    }
    st->converged = (small_step && small_grad) ? 1 : 0;
    st->m += 1;
  }
}

// One pass over traces and observations: the weighted cotangent and the FP64 partials of J.
// The difference of two float32 values is exact in FP64, so cot is that difference times z,
// rounded once.  VEC: 16-byte accesses, four values of one row each (row_len a multiple of 4).
template <bool VEC>
__global__ __launch_bounds__(CGA_THREADS) void misfit_kernel(const float* __restrict__ traces,
                                                             const float* __restrict__ obs, int64_t n,
                                                             int64_t row_len, int64_t n_rows,
                                                             const double* __restrict__ z, float* cot,
                                                             double* __restrict__ part) {
  double acc[1] = {0.0};
  const int64_t stride = (int64_t)gridDim.x * CGA_THREADS;
  if (VEC) {
    const int64_t n4 = n / 4;
    const float4* t4 = reinterpret_cast<const float4*>(traces);
    const float4* o4 = reinterpret_cast<const float4*>(obs);
    for (int64_t i = (int64_t)blockIdx.x * CGA_THREADS + threadIdx.x; i < n4; i += stride) {
      const float4 tv = t4[i], ov = o4[i];
      const double w = z ? z[(4 * i / row_len) % n_rows] : 1.0;
      const double r0 = (double)tv.x - (double)ov.x, r1 = (double)tv.y - (double)ov.y;
      const double r2 = (double)tv.z - (double)ov.z, r3 = (double)tv.w - (double)ov.w;
      if (cot) reinterpret_cast<float4*>(cot)[i] = make_float4((float)(w * r0), (float)(w * r1), (float)(w * r2),
                                                               (float)(w * r3));
      acc[0] += w * (r0 * r0 + r1 * r1 + r2 * r2 + r3 * r3);
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * CGA_THREADS + threadIdx.x; i < n; i += stride) {
      const double r = (double)traces[i] - (double)obs[i];
      const double w = z ? z[(i / row_len) % n_rows] : 1.0;
      if (cot) cot[i] = (float)(w * r);
      acc[0] += w * r * r;
    }
  }
  block_sums<1>(acc, part + blockIdx.x);
}

__global__ __launch_bounds__(CGA_THREADS) void misfit_finish_kernel(const double* __restrict__ part, int nb,
                                                                    double* __restrict__ j) {
  __shared__ double tot[1];
  sum_partials<1>(part, nb, tot);
  __syncthreads();
  if (threadIdx.x == 0) *j = 0.5 * tot[0];
}

__global__ void cga_upper_check_kernel(const float* __restrict__ eps, const float* __restrict__ sig, int64_t n,
                                       double eps_max, double sig_max, int* err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!((double)eps[i] <= eps_max) || !((double)sig[i] <= sig_max)) atomicAdd(err, 1);
}

// Step sizes from the gradient of J at the initial guess: per block, the largest |dJ/dc| over
// the free nodes of eps and of sigma.
__global__ __launch_bounds__(CGA_THREADS) void cga_gmax_kernel(const double* __restrict__ gJe,
                                                               const double* __restrict__ gJs, int fsx, int fsy,
                                                               int fsz, int64_t n_extra, const double* __restrict__ wn,
                                                               const CgaDev* __restrict__ st, double* __restrict__ part) {
  __shared__ double red[2][CGA_THREADS];
  const int64_t n = (int64_t)fsx * fsy * fsz + n_extra;
  double m[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * CGA_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * CGA_THREADS) {
    if (!cga_free(i, fsx, fsy, fsz)) continue;
    const double w = wn ? wn[i] : st->w;
    m[0] = fmax(m[0], fabs(gJe[i]) / w);
    m[1] = fmax(m[1], fabs(gJs[i]) / w);
  }
  const int t = threadIdx.x;
  red[0][t] = m[0];
  red[1][t] = m[1];
  __syncthreads();
  for (int w = CGA_THREADS / 2; w > 0; w >>= 1) {
    if (t < w) {
      red[0][t] = fmax(red[0][t], red[0][t + w]);
      red[1][t] = fmax(red[1][t], red[1][t + w]);
    }
    __syncthreads();
  }
  if (t == 0) {
    part[2 * (int64_t)blockIdx.x] = red[0][0];
    part[2 * (int64_t)blockIdx.x + 1] = red[1][0];
  }
}

// gamma^0 = gamma^m = G / step and alpha^m = step / G per field, G = max(max |dJ/dc_i| / w_i, 1e-30)
// (w_i: the lumped mass of free node i): the first update then moves the field by at most `step`.
__global__ __launch_bounds__(CGA_THREADS) void cga_steps_finish_kernel(const double* __restrict__ part, int nb,
                                                                       double step_e, double step_s,
                                                                       CgaDev* __restrict__ st) {
  __shared__ double red[2][CGA_THREADS];
  const int t = threadIdx.x;
  double m[2] = {0.0, 0.0};
  for (int b = t; b < nb; b += CGA_THREADS) {
    m[0] = fmax(m[0], part[2 * (int64_t)b]);
    m[1] = fmax(m[1], part[2 * (int64_t)b + 1]);
  }
  red[0][t] = m[0];
  red[1][t] = m[1];
  __syncthreads();
  for (int w = CGA_THREADS / 2; w > 0; w >>= 1) {
    if (t < w) {
      red[0][t] = fmax(red[0][t], red[0][t + w]);
      red[1][t] = fmax(red[1][t], red[1][t + w]);
    }
    __syncthreads();
  }
  if (t == 0) {
    const double step[2] = {step_e, step_s};
    for (int f = 0; f < 2; ++f) {
      const double g = fmax(red[f][0], 1e-30);
      st->gamma0[f] = st->gamma[f] = g / step[f];
      st->alpha[f] = step[f] / g;
    }
  }
}

}  // namespace

void launch_cga_steps(const double* gJe, const double* gJs, const CgaMesh& g, double step_eps, double step_sig,
                      CgaDev* st, double* part, hipStream_t s) {
  const int nb = cga_blocks((int64_t)g.fs[0] * g.fs[1] * g.fs[2] + g.n_extra);
  hipLaunchKernelGGL(cga_gmax_kernel, dim3(nb), dim3(CGA_THREADS), 0, s, gJe, gJs, g.fs[0], g.fs[1], g.fs[2], g.n_extra,
                     g.w, st, part);
  hipLaunchKernelGGL(cga_steps_finish_kernel, dim3(1), dim3(CGA_THREADS), 0, s, part, nb, step_eps, step_sig, st);
}

int cga_blocks(int64_t n_fem) {
  const int64_t b = (n_fem + CGA_THREADS - 1) / CGA_THREADS;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, CGA_MAX_BLOCKS));
}

void launch_cga_update(const double* gJe, const double* gJs, float* eps, float* sig, const float* eps0,
                       const float* sig0, double* d_eps, double* d_sig, const CgaMesh& g, CgaDev* st,
                       double* part, hipStream_t s) {
  const int nb = cga_blocks((int64_t)g.fs[0] * g.fs[1] * g.fs[2] + g.n_extra);
  hipLaunchKernelGGL(cga_norm_kernel, dim3(nb), dim3(CGA_THREADS), 0, s, gJe, gJs, eps, sig, eps0, sig0, g.fs[0],
                     g.fs[1], g.fs[2], g.n_extra, g.w, st, part);
  hipLaunchKernelGGL(cga_beta_kernel, dim3(1), dim3(CGA_THREADS), 0, s, part, nb, st);
  hipLaunchKernelGGL(cga_step_kernel, dim3(nb), dim3(CGA_THREADS), 0, s, gJe, gJs, eps, sig, eps0, sig0, d_eps,
                     d_sig, g.fs[0], g.fs[1], g.fs[2], g.n_extra, g.w, st, part);
  hipLaunchKernelGGL(cga_finish_kernel, dim3(1), dim3(CGA_THREADS), 0, s, part, nb, st);
}

void launch_misfit(const float* traces, const float* obs, int64_t n, int64_t row_len, int64_t n_rows,
                   const double* z, float* cot, double* part, double* j, hipStream_t s) {
  const int nb = cga_blocks(n);
  const bool vec = row_len % 4 == 0 && ((uintptr_t)traces | (uintptr_t)obs | (uintptr_t)cot) % 16 == 0;
  if (vec)
    hipLaunchKernelGGL((misfit_kernel<true>), dim3(nb), dim3(CGA_THREADS), 0, s, traces, obs, n, row_len, n_rows, z,
                       cot, part);
  else
    hipLaunchKernelGGL((misfit_kernel<false>), dim3(nb), dim3(CGA_THREADS), 0, s, traces, obs, n, row_len, n_rows, z,
                       cot, part);
  if (j) hipLaunchKernelGGL(misfit_finish_kernel, dim3(1), dim3(CGA_THREADS), 0, s, part, nb, j);
}

hipError_t misfit_scratch(double** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    // with device `dev` current: that GPU's copy of the array
    void* q = nullptr;
    e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double*>(q);
  }
  *out = addr[dev];
  return hipSuccess;
}

void launch_cga_upper_check(const float* eps, const float* sig, int64_t n, double eps_max, double sig_max, int* err,
                            hipStream_t s) {
  const int nb = cga_blocks(n);
  hipLaunchKernelGGL(cga_upper_check_kernel, dim3(nb), dim3(CGA_THREADS), 0, s, eps, sig, n, eps_max, sig_max, err);
}

}  // namespace dd
