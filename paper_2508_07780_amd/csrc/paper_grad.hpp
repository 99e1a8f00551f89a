// Paper-formula gradient variant (eq. gradeps with div(eps~ E) ~ eps~ div E): launches.
#pragma once

#include "dd_common.hpp"

namespace dd {

// api_own[i] = owned internal id of FEM node i, or -1 (built from own_api).
void launch_invert_own(const int* own_api, int64_t n_own, int64_t n_fem, int* api_own, hipStream_t s);
// One adjoint step's contribution: lam = lambda^k, E = forward E^k (both [3][n_own], owned
// internal order).  acc[i] (FEM-node index, free nodes) += the paper term of node i, minus
// the exact R1 div-div term when sub_exact (the variant of an R1 solve; an R2 solve's exact
// div-div term is the paper term itself).
void launch_paper_grad_step(const float* lam, const float* E, int64_t n_own, const int* api_own, const int fs[3],
                            double h, bool sub_exact, double* acc, hipStream_t s);
// One level's div-div terms with weights: acc[i] += wp P_i - wx Q_i, P the paper term and Q
// the exact R1 term of node i for lam = lambda^n and E = E^n ([3][n_own], owned order).
void launch_divdiv_grad_terms(const float* lam, const float* E, int64_t n_own, const int* api_own, const int fs[3],
                              double h, double wp, double wx, double* acc, hipStream_t s);
// out_eps[i] += acc[i] on free nodes.
void launch_add_free(const double* acc, const int fs[3], double* out_eps, hipStream_t s);

}  // namespace dd
