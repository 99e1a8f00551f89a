// Internal declarations shared by the host setup, the kernels and the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "dd.h"

namespace dd {

// Finite-difference tile: 32 x 8 nodes in (x, y), marching a chunk of planes in z.
#ifndef DD_FD_TY
#define DD_FD_TY 8
#endif
constexpr int FD_TX = 32;
constexpr int FD_TY = DD_FD_TY;
// z-chunk length.  Where the grid's fields fit the last-level cache, short chunks: more and
// smaller blocks fill the GPU more evenly, and the extra reads of the planes that
// neighbouring chunks share hit the cache.  Where the fields stream from HBM (the
// non-temporal variant), long chunks, which read those shared planes less often.
#ifndef DD_FD_ZC_CACHED
#define DD_FD_ZC_CACHED 2
#endif
constexpr int FD_ZC_CACHED = DD_FD_ZC_CACHED;
#ifndef DD_FD_ZC_STREAM
#define DD_FD_ZC_STREAM 8
#endif
constexpr int FD_ZC_STREAM = DD_FD_ZC_STREAM;
__host__ __device__ constexpr int fd_zc(bool nt) { return nt ? FD_ZC_STREAM : FD_ZC_CACHED; }
// Streaming variant: the tile order takes FD_ZGROUP consecutive z-chunks of each row of tiles
// in turn (x fastest, then the chunks of the group, then y), so that the plane two chunks
// share is read again while it is still in the XCD's L2.
#ifndef DD_FD_ZGROUP
#define DD_FD_ZGROUP 2
#endif
constexpr int FD_ZGROUP = DD_FD_ZGROUP;
__host__ __device__ constexpr int fd_zgroup(bool nt) { return nt ? FD_ZGROUP : 1; }
constexpr int FD_THREADS = FD_TX * FD_TY;
// the FD tile's two LDS planes of three components (when they sit in the dynamic LDS)
constexpr size_t FD_DYN_LDS_BYTES = sizeof(float) * 2 * 3 * (FD_TY + 2) * (FD_TX + 2);
// Last-level cache (MI355X Infinity Cache).  A grid whose two levels of E exceed it streams
// each node's own previous and new level with non-temporal accesses.
constexpr double LLC_BYTES = 256.0 * 1024 * 1024;

// FEM partition: a block of at most FEM_PB^3 owned nodes plus its halo.
constexpr int FEM_PB = 8;          // default block edge; DD_FEM_PB="x,y,z" overrides
constexpr int FEM_THREADS = 256;
// gather form of the element kernel: list entries (and their element words) loaded per batch
#ifndef DD_FEM_GB
#define DD_FEM_GB 8
#endif
// the assembled-stencil FEM part shares launches with the FD tiles: same block size
constexpr int STENCIL_THREADS = FD_THREADS;
constexpr int FEM_LOC_MAX = 1024;  // owned + halo nodes per partition (11-bit local ids)
constexpr int FEM_OWN_MAX = 512;
constexpr int FEM_COLORS_MAX = 64;
constexpr int FEM_ELEM_MAX = 4608;  // elements per partition (staged in LDS)
constexpr int FEM_GEOM_LDS = 64;    // geometry tables up to this size are staged in LDS
// Geometry entry: grad phi_0..3 (12 floats), |K| grad phi_0..3 (12), |K|, padding.  The
// stride of 36 floats puts consecutive entries on different LDS banks for 16-byte reads.
constexpr int GEOM_STRIDE = 36;

constexpr int N_XCD = 8;  // MI355X: workgroups are dispatched round-robin over 8 XCDs

// Index of node (x, y, z) among the nodes of an nx*ny*nz box that lie on the
// faces in `mask`, counted in lexicographic order (x fastest); -1 if the node
// is on none of them.  Requires nx, ny, nz >= 2.
__host__ __device__ inline int64_t face_lex_index(int x, int y, int z, int nx, int ny, int nz, unsigned mask) {
  const bool zlo = (mask & DD_FACE_BOTTOM) && z == 0;
  const bool zhi = (mask & DD_FACE_TOP) && z == nz - 1;
  const bool xlo = (mask & DD_FACE_XMIN) && x == 0;
  const bool xhi = (mask & DD_FACE_XMAX) && x == nx - 1;
  const bool ylo = (mask & DD_FACE_YMIN) && y == 0;
  const bool yhi = (mask & DD_FACE_YMAX) && y == ny - 1;
  if (!(zlo || zhi || xlo || xhi || ylo || yhi)) return -1;
  const int64_t cm = ((mask & DD_FACE_XMIN) ? 1 : 0) + ((mask & DD_FACE_XMAX) ? 1 : 0);
  const int64_t ny_mid = ny - ((mask & DD_FACE_YMIN) ? 1 : 0) - ((mask & DD_FACE_YMAX) ? 1 : 0);
  const int64_t p_mid = (int64_t)(ny - ny_mid) * nx + ny_mid * cm;
  const int64_t p_full = (int64_t)nx * ny;
  int64_t before = 0;
  if (z > 0) before = ((mask & DD_FACE_BOTTOM) ? p_full : p_mid) + (int64_t)(z - 1) * p_mid;
  if (zlo || zhi) return before + (int64_t)y * nx + x;
  int64_t rows = 0;
  if (y > 0) rows = ((mask & DD_FACE_YMIN) ? (int64_t)nx : cm) + (int64_t)(y - 1) * cm;
  if (ylo || yhi) return before + rows + x;
  return before + rows + (xlo ? 0 : ((mask & DD_FACE_XMIN) ? 1 : 0));
}

inline int64_t face_lex_count(int nx, int ny, int nz, unsigned mask) {
  const int64_t cm = ((mask & DD_FACE_XMIN) ? 1 : 0) + ((mask & DD_FACE_XMAX) ? 1 : 0);
  const int64_t ny_mid = ny - ((mask & DD_FACE_YMIN) ? 1 : 0) - ((mask & DD_FACE_YMAX) ? 1 : 0);
  const int64_t p_mid = (int64_t)(ny - ny_mid) * nx + ny_mid * cm;
  const int64_t p_full = (int64_t)nx * ny;
  const int64_t nzf = ((mask & DD_FACE_BOTTOM) ? 1 : 0) + ((mask & DD_FACE_TOP) ? 1 : 0);
  return nzf * p_full + (nz - nzf) * p_mid;
}

// Tile grid of an nx * ny * nz grid for the z-chunk of the streaming (nt) or cached variant;
// per_xcd = tiles each XCD takes.
inline void fd_tile_grid(int nx, int ny, int nz, bool nt, int& nbx, int& nby, int& nbz, int& ntiles, int& per_xcd) {
  const int zc = fd_zc(nt), zg = fd_zgroup(nt);
  nbx = (nx + FD_TX - 1) / FD_TX;
  nby = (ny + FD_TY - 1) / FD_TY;
  nbz = (nz + zc - 1) / zc;
  ntiles = nbx * nby * ((nbz + zg - 1) / zg * zg);   // whole groups of z-chunks
  per_xcd = (ntiles + N_XCD - 1) / N_XCD;
}

// ---- kernel arguments -------------------------------------------------------------------

// The data of one finite-difference step that change from step to step.
struct FdStepData {
  float pw[3];
  int top_a, top_b;
  float dip[3];
  int pw_kind;
  float pw_t;
  float* tr_out;
  const float* cot_in;
  const float* obs_in;
};

// Temporal blocking: two-step tiles march z-chunks of tb_zc planes (the level n+1 is
// recomputed on one extra plane at each end of the chunk, so longer chunks waste less).
__host__ __device__ constexpr int tb_zc(bool nt) { return nt ? 16 : 8; }
// LDS of a two-step tile: four planes of level n on the tile plus two rings (36 x 12), three
// planes of level n+1 on the tile plus one ring (34 x 10), three components each
constexpr int TB_LX = FD_TX + 4, TB_LY = FD_TY + 4, TB_EX = FD_TX + 2, TB_EY = FD_TY + 2;
constexpr int TB_RING1 = TB_EX * TB_EY - FD_TX * FD_TY;   // lanes with a ring-1 node
constexpr int TB_RING2 = TB_LX * TB_LY - TB_EX * TB_EY;   // lanes with a ring-2 node, after those
constexpr size_t TB_LDS_BYTES = (size_t)(4 * 3 * TB_LX * TB_LY + 3 * 3 * TB_EX * TB_EY) * 4;
// Class of two-step tile t: 0 nothing to do (past the grid, or every node FEM-owned), 1 near
// (the tile holds a node of the closed FEM box: one step per launch, the FEM's level n+1 is
// needed), 2 far (two steps per launch).
__host__ __device__ inline int tb_tile_class(int t, int nbx, int nby, int nx, int ny, int nz, int zc, const int blo[3],
                                             const int bhi[3]) {
  const int bx = t % nbx, by = (t / nbx) % nby, bz = t / (nbx * nby);
  const int x0 = bx * FD_TX, y0 = by * FD_TY, z0 = bz * zc;
  if (z0 >= nz) return 0;
  const int x1 = x0 + FD_TX - 1 < nx - 1 ? x0 + FD_TX - 1 : nx - 1;
  const int y1 = y0 + FD_TY - 1 < ny - 1 ? y0 + FD_TY - 1 : ny - 1;
  const int z1 = z0 + zc - 1 < nz - 1 ? z0 + zc - 1 : nz - 1;
  if (x0 > blo[0] && x1 < bhi[0] && y0 > blo[1] && y1 < bhi[1] && z0 > blo[2] && z1 < bhi[2]) return 0;
  if (x1 >= blo[0] && x0 <= bhi[0] && y1 >= blo[1] && y0 <= bhi[1] && z1 >= blo[2] && z0 <= bhi[2]) return 1;
  return 2;
}

struct FdArgs {
  const float* X_in;   // field at level n (forward E^n, adjoint lambda^k), [3][N]
  float* X_out;        // field at the previous level on entry (forward E^{n-1}, adjoint
                       // lambda^{k+1}), overwritten with the next level, [3][N]
  int64_t N;
  int nx, ny, nz;
  int blo[3], bhi[3];  // FEM box node range [fem_lo, fem_lo + fem_cells] per axis
  int nbx, nby, nbz, ntiles, per_xcd;
  float nu2, nu;       // (dt/h)^2, dt/h
  unsigned abs_mask;
  int top_a, top_b;    // top face absorbing at the levels of D+ (a) and D- (b)
  float pw[3];         // plane-wave forcing F dt^2 / m on the top face (0 when off)
  // obliquely incident plane wave, while on (pw_kind != 0; pw is 0 then): top-face node (x, y)
  // takes pw_amp * P(t_n - tau), tau = pw_kx (x - pw_x0) + pw_ky (y - pw_y0)
  int pw_kind;         // 0, DD_SRC_SINE1 or DD_SRC_GAUSS_SINE
  float pw_amp[3];     // 2 dt^2 / h * amp * pol
  float pw_t;          // t_n (SINE1) or t_n - t0 (GAUSS_SINE)
  float pw_kx, pw_ky;  // delay per node step along x and y (k_x h, k_y h)
  int pw_x0, pw_y0;    // top-face node of delay 0
  float pw_omega;      // omega
  float pw_iw;         // 1 / width (GAUSS_SINE)
  float pw_sup;        // support: |t - tau - t0| <= pw_sup (GAUSS_SINE: t0), 0 < t - tau < pw_sup (SINE1: period)
  int64_t dip_idx;     // dipole grid node or -1
  float dip[3];        // dipole forcing F dt^2 / m at that node
  unsigned det_mask;
  float* tr_out;       // forward: traces of this step [n_det][3] or null
  const float* cot_in; // adjoint: cotangent of this step [n_det][3] or null
  const float* obs_in; // adjoint: observations of this step; the cotangent is then cot_in - obs_in
  float dt2_h3;        // dt^2 / h^3
  float* iface_out;    // layer-0 values of the next level [3][n_l0] or null
  int64_t n_l0;
  int fs[3];           // FEM lattice shape (fem_cells + 1)
  double* epart;       // energy partial per tile or null
  double e_coef;       // h^3 / (2 dt^2)
  int rev;             // 1: each XCD takes its tiles in reverse order (alternate steps: a
                       // step starts where the previous one ended, whose data the caches hold)
  const float* X_prev; // the previous level when it is not X_out (two-step launches: four
                       // rotating buffers, none read and written in one launch); null: X_out
  // Two-step launches (temporal blocking): the second step's level and per-step data, the
  // two-step tile grid (z-chunks of tb_zc(NT) planes) and the list of near tiles (those with
  // a FEM box node) that a one-step launch covers
  float* X_out2;
  FdStepData s2;
  int tb_nbz, tb_ntiles, tb_per_xcd;
  const int* tb_list;
  int tb_nlist;
};

constexpr int STENCIL_SLOTS_MAX = 27;

struct FemArgs {
  const int* own_off;   // [n_part + 1]
  const int* halo_off;  // [n_part + 1]
  const int* halo;      // owned internal id, or -1 - layer0 index
  const int* col_base;  // [n_part] start of the partition's colour offsets in col_off
  const int* ncol;      // [n_part]
  const int* col_off;   // absolute element offsets per colour
  const uint64_t* elems;
  const float* geom;    // [n_geom][GEOM_STRIDE]
  int n_geom;
  int lds_loc, lds_own, lds_elem;  // LDS sizing: max local nodes, owned nodes, elements (even)
  // node-gather form of the element loop: per partition, the elements incident to each owned
  // node in colour order, entry i of owned node l at inc[inc_off[p] + i * no + l] (element
  // index within the partition << 2 | the node's slot in it), lists padded with 0xFFFF to
  // inc_n[p] entries; gather = 1 selects this form, 0 the colour-by-colour scatter
  const uint16_t* inc; const int* inc_off; const int* inc_n;
  int gather;
  const int* own_grid;  // grid index for layer-1 owned nodes, -1 otherwise (free)
  const float* em1;     // eps - 1
  const float* c1;      // (a - b) / (a + b)
  const float* c2;      // 1 / (a + b);  a = m eps / dt^2, b = m sigma / (2 dt)
  const double* mass_d; // lumped mass (FP64)
  const float* X_in; float* X_out;
  const float* I_in; float* I_out;
  const float* iface_in;  // layer-0 values at the current level [3][n_l0]
  float* fd_out;          // grid field of the next level for the layer-1 dual write, or null
  float* ck_X; float* ck_I;  // checkpoint dual write or null
  int64_t n_own, n_l0, N;
  double* epart; int epart_off; double inv_2dt2;
  // assembled-stencil path
  const int* part_dims; const int* box_codes; const int* slot_off; const float* slot_k; const float* slot_b;
  int n_slots, lds_box;
  int n_part;
  int rev;             // 1: each XCD takes its partitions in reverse order (alternate steps)
  int r2;              // div-div form R2 (element mean of eps - 1 outside the divergence)
  float h;             // grid spacing (the R2 term is evaluated element by element)
  // adjoint
  const float* wE; const float* wV; const float* wVm;  // forward E^k, V^k, V^{k-1} [3][n_own]
  double* g_eps; double* g_sig;
  double inv_dt2, inv_2dt;
};

void launch_fd(const FdArgs& a, hipStream_t s, bool energy, bool nt);
size_t fem_lds_bytes(const FemArgs& a, bool adj, bool stage);
// One fused step on a general mesh: element-coloured FEM partitions and the FD tiles.
void launch_step_el(const FdArgs& fa, const FemArgs& ea, hipStream_t s, bool adj, bool energy, bool nt);
void launch_fem_fwd(const FemArgs& a, int n_part, hipStream_t s, bool energy);
void launch_fem_adj(const FemArgs& a, int n_part, hipStream_t s);
void launch_fem_stencil_fwd(const FemArgs& a, int n_part, hipStream_t s, bool energy);
void launch_fem_stencil_adj(const FemArgs& a, int n_part, hipStream_t s);
// fused FD + FEM (assembled-stencil) step, one launch
// Arguments of the paper-formula div-div gradient terms of one level (pg_tile.hpp).
struct PgArgs {
  const float* lam;     // lambda^k, [3][n_own] (owned order)
  const float* E;       // forward E^k, [3][n_own]
  int64_t n_own;
  const int* api_own;   // FEM-node -> owned id
  int fs[3];            // FEM nodes per axis
  double h, wp, wx;
  double* acc;          // [n_fem] FP64, free nodes
};
// pg: the div-div gradient terms of the step's input level, fused into an adjoint step of
// the form R2 (nullable).
// Two-step launches: pair_a = 1 the first launch of a pair (far tiles two steps, near tiles
// and the FEM partitions one), 0 the second (near tiles from fa.tb_list and the FEM, one step).
void launch_step_pair(const FdArgs& fa, const FemArgs& ea, hipStream_t s, bool adj, bool nt, int pair_a);
void launch_step(const FdArgs& fa, const FemArgs& ea, hipStream_t s, bool adj, bool energy, bool nt,
                 const PgArgs* pg = nullptr);

// adjoint step and FEM-only recompute step of one problem in one launch (arguments by value)
void launch_step_rec(const FdArgs& fa, const FemArgs& ea, const FemArgs& er, hipStream_t s, bool nt);
// one item of a batched step launch
struct BatchItem {
  FdArgs fa;
  FemArgs ea;
  int kind;         // 0 forward, 1 adjoint, 2 forward FEM-only recompute
  int fem_blocks;   // multiple of N_XCD (extra blocks exit)
  int fd_blocks;    // per_xcd * N_XCD, or 0 for a recompute step
};
// First block of each item of a batched launch (base[n] = total blocks), passed by value
// so that a block finds its item among the kernel arguments.
constexpr int BATCH_MAX = 64;
struct BatchBases {
  int n;
  int base[BATCH_MAX + 1];
};
// obl: some item carries an obliquely incident plane wave (pw_kind != 0)
void launch_batch(const BatchItem* items_dev, const BatchBases& bases, size_t lds, hipStream_t s, bool nt, bool obl);
size_t stencil_lds(const FemArgs& a);
void launch_energy_reduce(const double* part, int n, double* out, hipStream_t s);
void launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
void launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);
void launch_copy_f32(float* dst, const float* src, int64_t n, hipStream_t s);
void launch_validate(const float* eps, const float* sig, int fsx, int fsy, int fsz, int64_t n_extra, int* err,
                     hipStream_t s);
void launch_coefficients(const float* eps, const float* sig, const int* own_api, const double* mass_d,
                         int64_t n_own, double dt, float* em1, float* c1, float* c2, float* sig_own,
                         const int* guard, hipStream_t s);
void launch_fill_i32(int* p, int n, int v, hipStream_t s);
void launch_tikhonov_add(const float* em1, const float* sig_own, const int* own_api, const int* own_grid,
                         const double* mass_d, int64_t n_own, double gamma_eps, double gamma_sig, const float* eps0,
                         const float* sig0, double* g_eps, double* g_sig, hipStream_t s);
void launch_gradient_out(const double* g_eps, const double* g_sig, const int* own_api, const int* own_grid,
                         int64_t n_own, double* out_eps, double* out_sig, hipStream_t s);
void launch_count_nonfinite(const float* x, int64_t n, int* err, hipStream_t s);

// ---- host-side mesh and partitions ----------------------------------------------------

struct HostMesh {
  int64_t n_fem = 0, n_own = 0, n_l0 = 0;
  int n_part = 0, n_geom = 0;
  std::vector<int> own_off, halo_off, halo, col_base, ncol, col_off;
  std::vector<uint64_t> elems;
  std::vector<float> geom;
  std::vector<int> own_grid, own_api;
  std::vector<double> mass;
  int max_colors = 0, max_loc = 0, max_own = 0, max_elem = 0;
  // Assembled-stencil form (used when every owned node has the same assembled stencil,
  // as on the Kuhn lattice): per partition the owned block dims and a (dims+2)^3 box of
  // node codes in lattice order; per stencil slot the lattice offset, K_ij and B_ij.
  bool stencil_ok = false;
  int n_slots = 0, max_box = 0;
  std::vector<int> part_dims;   // [n_part][4]: owned dims x, y, z, box base
  std::vector<int> box_codes;   // owned internal id or -1 - layer0 index
  std::vector<int> slot_off;    // [n_slots][4]: dx, dy, dz, 0
  std::vector<float> slot_k;    // [n_slots]
  std::vector<float> slot_b;    // [n_slots][9], row-major 3x3
};

// Builds the Kuhn split of the FEM box: node partitions, the assembled stencil, masses and
// the staging boxes of the stencil kernel, and with `elements` the element kernel's data
// (per-partition elements, halos and colouring).  Returns an empty string on success, else
// the error text.
std::string build_mesh(const dd_problem_desc& d, HostMesh& m, const int pb[3], bool elements);
// General tetrahedral mesh of the FEM box (lattice nodes, then n_extra nodes at xyz strictly
// inside the box; n_tets tetrahedra in those indices), for the element kernel, its owned nodes
// grouped by lattice blocks of pb[0] x pb[1] x pb[2] cells.  Empty string on success, else the
// error text.
std::string build_mesh_general(const dd_problem_desc& d, int64_t n_extra, const double* xyz, int64_t n_tets,
                               const int32_t* tets, HostMesh& m, const int pb[3]);

}  // namespace dd
