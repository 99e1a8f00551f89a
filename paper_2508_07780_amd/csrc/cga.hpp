// Conjugate gradient update of eps and sigma (box "CGA", steps 2-6): device state and launch.
#pragma once

#include "dd_common.hpp"

namespace dd {

// ---- conjugate gradient update of eps and sigma (box "CGA", steps 2-6) ----------------
// Index 0 = eps, 1 = sigma.  Lives in device memory; written by one thread of the
// single-block kernels, read by all.
struct CgaDev {
  // parameters
  double gamma0[2], p, lo[2], hi[2], eta1[2], eta2[2];
  double w;                  // lumped mass of a free lattice node (h^3): the L2 weight when the
                             // FEM nodes carry no mass array (the Kuhn split)
  // iteration state: gamma^m, alpha^m, |g^{m-1}|^2, m
  double gamma[2], alpha[2], gn2_prev[2];
  int m, converged;
  // results of the last update
  double gn2[2], beta[2], gd[2], dd[2], step2[2], alpha_used[2], gamma_used[2];
  double change2[2];         // |c^{m+1} - c^0|^2: the distance from the initial guess
};
// The FEM nodes of a run: the (fs[0] x fs[1] x fs[2]) lattice, then n_extra nodes of a general
// mesh (free); w: FP64 lumped mass per FEM node (API order) or null for h^3 on every free node.
struct CgaMesh {
  int fs[3];
  int64_t n_extra;
  const double* w;
};
constexpr int CGA_MAX_BLOCKS = 1024;
// FP64 sums per block of an update: (g, d), (d, d), |step|^2 per field, then |c - c^0|^2 per field
constexpr int CGA_SUMS = 8;
int cga_blocks(int64_t n_fem);
// Four launches: gradient-function norms, beta, direction / update / projection, step sizes.
// part holds CGA_MAX_BLOCKS x CGA_SUMS doubles.
void launch_cga_update(const double* gJe, const double* gJs, float* eps, float* sig, const float* eps0,
                       const float* sig0, double* d_eps, double* d_sig, const CgaMesh& g, CgaDev* st,
                       double* part, hipStream_t s);
// gamma^0 = gamma^m = G / step and alpha^m = step / G for eps and sigma, G = max |dJ/dc_i| / w_i over
// the free nodes (two launches; part holds CGA_MAX_BLOCKS x 2 doubles).
void launch_cga_steps(const double* gJe, const double* gJs, const CgaMesh& g, double step_eps, double step_sig,
                      CgaDev* st, double* part, hipStream_t s);
// Counts FEM nodes with eps > eps_max or sigma > sig_max into *err.
void launch_cga_upper_check(const float* eps, const float* sig, int64_t n, double eps_max, double sig_max, int* err,
                            hipStream_t s);

// Trace misfit of eq. tikhonov_functional with time weights z (null: z = 1) at the trace rows:
// cot (nullable) = z_row (traces - obs) in float32; j (nullable) = 1/2 sum z_row |traces - obs|^2
// in FP64 (block partials in part[CGA_MAX_BLOCKS], summed in order by one block).
void launch_misfit(const float* traces, const float* obs, int64_t n, int64_t row_len, int64_t n_rows,
                   const double* z, float* cot, double* part, double* j, hipStream_t s);

// Device address of the current GPU's copy of the static scratch array of the no-allocation
// misfit: CGA_MAX_BLOCKS block partials, then DD_MISFIT_NOALLOC_MAX_STEPS time weights.  The
// symbol is resolved once per device (hipGetSymbolAddress); returns hipSuccess or its error.
hipError_t misfit_scratch(double** out);

}  // namespace dd
