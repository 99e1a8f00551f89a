// C-ABI of the hybrid FE/FD solver: problem setup, forward / adjoint / gradient drivers.
//
// Time loops run on the host and queue one launch per step on the caller's stream: the
// fused step kernel (FEM partitions and FD tiles together), or one FD and one FEM launch.
// Within a step the FD tiles read level n and write level n+1 over level n-1 node by node
// (each node's own lane only), the FEM reads level n and writes level n+1 (ping-pong, with
// the increment updated in place), so neither depends on the other's writes of the step.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "cga.hpp"
#include "initial.hpp"
#include "paper_grad.hpp"
#include "dd_common.hpp"

using namespace dd;

// One replayable graph of a problem's launches (the forward's or the adjoint's): the executable
// graph, the key of the call it was captured for, the key of the last call, the number of
// captures and replays, and an event marking the end of the last replay.
struct GraphCache {
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  std::vector<unsigned char> key, last;
  int64_t captures = 0, replays = 0;
};

struct dd_problem {
  dd_problem_desc d{};
  int nx = 0, ny = 0, nz = 0;
  int64_t N = 0;
  int fs[3] = {0, 0, 0};
  int64_t n_fem = 0, n_own = 0, n_l0 = 0, n_det = 0;
  bool general = false;   // a caller mesh (dd_create_mesh): n_extra nodes beyond the lattice
  int64_t n_extra = 0;
  double* mass_api = nullptr;   // a caller mesh's lumped masses per FEM node (API order; 0 off the owned set)
  int n_part = 0, n_geom = 0;
  int lds_loc = 0, lds_own = 0, lds_elem = 0, lds_box = 0;
  bool use_stencil = false;             // assembled-stencil FEM kernel instead of the element kernel
  int n_slots = 0;
  int *part_dims = nullptr, *box_codes = nullptr, *slot_off = nullptr;
  float *slot_k = nullptr, *slot_b = nullptr;
  int nbx = 0, nby = 0, nbz = 0, n_tiles = 0, per_xcd = 0;
  bool fd_nt = false;     // non-temporal own-node streams in the FD tiles (grid exceeds the LLC)
  // topology (device)
  int *own_off = nullptr, *halo_off = nullptr, *halo = nullptr, *col_base = nullptr, *ncol = nullptr,
      *col_off = nullptr, *own_grid = nullptr, *own_api = nullptr;
  uint64_t* elems = nullptr;
  // incidence lists of the element kernel's gather form (FemArgs::inc); fem_gather selects it
  uint16_t* inc = nullptr;
  int *inc_off = nullptr, *inc_n = nullptr;
  bool fem_gather = true;
  float* geom = nullptr;
  double* mass_d = nullptr;
  float *em1 = nullptr, *c1 = nullptr, *c2 = nullptr;
  float* sig_own = nullptr;   // sigma of the last dd_set_coefficients (owned order; the Tikhonov term)
  // device allocator of every buffer the problem owns (null: hipMalloc / hipFree)
  dd_alloc_fn alloc_fn = nullptr;
  dd_free_fn free_fn = nullptr;
  void* actx = nullptr;
  size_t alloc_bytes = 0;     // bytes currently allocated
  // state (device)
  // FD grid: two levels of E (three-level form); FEM: two levels of E and the increment V
  float *Efd[4] = {nullptr, nullptr, nullptr, nullptr}, *Efem[2] = {nullptr, nullptr}, *Vfem = nullptr;
  // temporal blocking (two FD steps per launch for the tiles away from the FEM box): level n
  // of the FD grid in Efd[n & 3]; the two-step tile grid, its near-tile list and node counts
  bool tb = false, tb_nt = false;
  int tb_nbz = 0, tb_ntiles = 0, tb_per_xcd = 0, tb_nlist = 0;
  int* tb_list = nullptr;
  int64_t tb_far = 0, tb_near = 0;   // FD-updated nodes of far / near tiles
  float* iring = nullptr;  // [2][3][n_l0]
  double* epart = nullptr;
  int* d_err = nullptr;
  // saved forward for the adjoint, per source: layer-0 history, segment-start checkpoints
  // and the last segment's full FEM state (written by the forward, never recomputed)
  std::vector<float*> ihist, ckpt, tail;
  int n_ck = 0;
  float* win = nullptr;             // recompute windows [(K+1)][2][3][n_own], for even and
  float* win_b = nullptr;           // odd segments (one segment is recomputed while another runs)
  // FD and FEM launches of one step run concurrently on the caller's stream and `aux`
  hipStream_t aux = nullptr;
  hipEvent_t ev_fd = nullptr, ev_fem = nullptr;
  // adjoint segment pipeline: a segment's recompute (on `aux`) is done; a segment's adjoint
  // steps (on the caller's stream) are done
  hipEvent_t ev_rec[2] = {nullptr, nullptr}, ev_adj = nullptr;
  bool overlap = false;   // measured slower than one stream (cross-stream waits per step)
  // graphs: the launches of a dd_forward / dd_adjoint call captured once into a HIP graph (on
  // the capture stream `cap`) and replayed while the call's arguments and the problem's launch
  // options stay the same (DD_GRAPH_AUTO: on grids of at most kGraphAutoNodes nodes, from the
  // second call in a row with the same key)
  int graph = DD_GRAPH_AUTO;
  hipStream_t cap = nullptr;
  GraphCache gfwd, gadj;
  bool fused = true;      // one launch per step (FD tiles + stencil FEM partitions)
  bool saved = false;
  int saved_n_src = 0;
  double *g_eps = nullptr, *g_sig = nullptr;
  bool have_grad = false;
  bool adj_obs = false;   // the last adjoint formed its cotangent as traces - observations
  // dd_misfit: time weights (n_steps; a host copy of the last upload) and FP64 block partials
  double *mis_z = nullptr, *mis_part = nullptr;
  std::vector<double> mis_z_host;
  // paper-formula gradient variant: FEM-node -> owned id map, FP64 sum
  bool pg_on = false, have_pg = false;
  bool r2 = false;        // div-div form R2 (its own step kernel instantiations)
  int* api_own = nullptr;
  double* pg_acc = nullptr;
  // general initial data (dd_set_initial_data): f_0, f_1 [N][3]; the level-0 div-div rows of
  // the exact R1 gradient (FEM-node index), added by dd_gradient when the last adjoint set them
  bool init_on = false, ic_used = false;
  float *init_f0 = nullptr, *init_f1 = nullptr;
  double* ic_acc = nullptr;
  std::string err;
  std::vector<void*> allocs;
  // kernel timing: event pairs around each step launch, per launch kind
  int prof_stride = 0;      // 0: off; k: time every k-th launch of each kind
  std::vector<hipEvent_t> ev[DD_PROF_KINDS];
  size_t ev_used[DD_PROF_KINDS] = {};
  uint64_t ev_seen[DD_PROF_KINDS] = {};
};

namespace {

constexpr size_t kProfMaxPairs = 16384;

// Kernel timing: a window of `prof_window(kind)` consecutive launches of one kind is
// bracketed by one event pair every `prof_stride` launches.  Windows of several launches
// amortise the event markers; they are used only for kinds that are launched back to back
// (the fused one-step kernels), single launches otherwise (the two launches of a pair alternate).
int prof_window(int kind) { return (kind == DD_PROF_STEP_FWD || kind == DD_PROF_STEP_ADJ) ? 8 : 1; }

long prof_begin(dd_problem* p, int kind, hipStream_t st) {
  if (p->prof_stride <= 0) return -1;
  const uint64_t seen = p->ev_seen[kind]++;
  const int w = prof_window(kind);
  const uint64_t period = (uint64_t)std::max(p->prof_stride, w);
  const uint64_t pos = seen % period;
  if (pos >= (uint64_t)w) return -1;
  const size_t i = p->ev_used[kind];
  if (i >= kProfMaxPairs) return -1;
  auto& v = p->ev[kind];
  while (v.size() < 2 * (i + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    v.push_back(e);
  }
  if (pos == 0 && hipEventRecord(v[2 * i], st) != hipSuccess) return -1;
  return (long)(pos == (uint64_t)(w - 1) ? i : -2);   // -2: inside a window, no closing event yet
}

void prof_end(dd_problem* p, int kind, long slot, hipStream_t st) {
  if (slot < 0) return;
  if (hipEventRecord(p->ev[kind][2 * slot + 1], st) == hipSuccess) p->ev_used[kind] = (size_t)slot + 1;
}

int fail(dd_problem* p, int code, const std::string& msg) {
  if (p) p->err = msg;
  return code;
}

// One device buffer through the problem's allocator (the caller's, else hipMalloc).
void* raw_alloc(dd_alloc_fn fn, void* ctx, size_t bytes) {
  void* q = nullptr;
  if (fn) return fn(bytes, ctx);
  if (hipMalloc(&q, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return q;
}

void raw_free(dd_free_fn fn, void* ctx, void* q) {
  if (!q) return;
  if (fn) fn(q, ctx);
  else (void)hipFree(q);
}

template <class T>
int dalloc(dd_problem* p, T** ptr, size_t count) {
  const size_t bytes = count ? count * sizeof(T) : sizeof(T);
  void* q = raw_alloc(p->alloc_fn, p->actx, bytes);
  if (!q) return fail(p, DD_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  p->allocs.push_back(q);
  p->alloc_bytes += bytes;
  *ptr = static_cast<T*>(q);
  return DD_OK;
}

template <class T>
int upload(dd_problem* p, T** ptr, const std::vector<T>& v) {
  int rc = dalloc(p, ptr, v.size());
  if (rc) return rc;
  if (!v.empty() && hipMemcpy(*ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return fail(p, DD_ERR_HIP, "hipMemcpy upload failed");
  return DD_OK;
}

int check_launch(dd_problem* p) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(p, DD_ERR_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return DD_OK;
}

std::string check_desc(const dd_problem_desc* d) {
  if (!d) return "null descriptor";
  for (int a = 0; a < 3; ++a) {
    if (d->n_outer[a] < 4) return "n_outer must be >= 4 per axis";
    if (d->fem_cells[a] < 2) return "fem_cells must be >= 2 per axis";
    if (d->fem_lo[a] < 1 || (int64_t)d->fem_lo[a] + d->fem_cells[a] > (int64_t)d->n_outer[a] - 2)
      return "the FEM box must lie strictly inside the outer grid";
  }
  const double n = (double)d->n_outer[0] * d->n_outer[1] * d->n_outer[2];
  // the FD kernels address one field component with 32-bit byte offsets
  if (n >= 1073741824.0) return "outer grid must have fewer than 2^30 nodes";
  if (!(d->h > 0.0) || !std::isfinite(d->h)) return "h must be positive";
  if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return "dt must be positive";
  if (d->dt * std::sqrt(3.0) > d->h * (1.0 + 1e-12)) return "dt exceeds the explicit stability bound h/sqrt(3)";
  if (d->n_steps < 1) return "n_steps must be >= 1";
  if (d->ckpt_every < 1) return "ckpt_every must be >= 1";
  if (d->detector_faces == 0 || d->detector_faces > 63u) return "detector_faces must be a non-empty face mask";
  if (d->absorbing_faces > 63u) return "absorbing_faces must be a face mask";
  if (!std::isfinite(d->s_stab)) return "s_stab must be finite";
  if (d->ckpt_mode < 0) return "ckpt_mode must be a DD_CKPT_* value";
  return std::string();
}

// Valid descriptor values this build does not run (DD_ERR_UNSUPPORTED).
std::string check_desc_supported(const dd_problem_desc* d) {
  if (d->overlap != 0 && d->overlap != 2) return "only a two-node overlap is built (overlap 2)";
  if (d->s_stab != 0.0 && d->s_stab != 1.0)
    return "only s = 1 is built: other s would break the plain wave equation of the finite-difference region";
  if (d->ckpt_mode != DD_CKPT_FEM_IFACE && d->ckpt_mode != DD_CKPT_STORE_ALL)
    return "ckpt_mode: full-state checkpoints are not built";
  return std::string();
}

// Checkpoint interval the problem runs with: every level kept under DD_CKPT_STORE_ALL.
int32_t effective_ckpt_every(const dd_problem_desc* d) {
  return d->ckpt_mode == DD_CKPT_STORE_ALL ? std::max<int32_t>(d->n_steps, 1) : d->ckpt_every;
}

double source_time(const dd_source& s, double t) {
  if (s.kind == DD_SRC_SINE1) {
    const double T = 2.0 * M_PI / s.omega;
    return (t > 0.0 && t < T) ? s.amp * std::sin(s.omega * t) : 0.0;
  }
  if (t < 0.0 || t > 2.0 * s.t0) return 0.0;
  const double u = (t - s.t0) / s.width;
  return s.amp * std::sin(s.omega * (t - s.t0)) * std::exp(-0.5 * u * u);
}

std::string check_source(const dd_problem* p, const dd_source& s) {
  if (s.kind != DD_SRC_SINE1 && s.kind != DD_SRC_GAUSS_SINE && s.kind != DD_SRC_DIPOLE) return "unknown source kind";
  if (!(s.omega > 0.0) || !std::isfinite(s.omega)) return "source omega must be positive";
  if (s.kind != DD_SRC_SINE1 && !(s.width > 0.0)) return "source width must be positive";
  if (s.kind != DD_SRC_DIPOLE) {
    const double n2 = s.dir[0] * s.dir[0] + s.dir[1] * s.dir[1] + s.dir[2] * s.dir[2];
    if (!std::isfinite(n2)) return "plane-wave direction must be finite";
    if (n2 > 0.0 && !(s.dir[2] < 0.0)) return "a plane wave enters through the top face: dir must have dir_z < 0";
  }
  if (s.kind == DD_SRC_DIPOLE) {
    for (int a = 0; a < 3; ++a)
      if (s.pos[a] < 0 || s.pos[a] >= p->d.n_outer[a]) return "dipole position outside the grid";
    bool inside = true;
    for (int a = 0; a < 3; ++a) inside &= s.pos[a] > p->d.fem_lo[a] && s.pos[a] < p->d.fem_lo[a] + p->d.fem_cells[a];
    if (inside) return "dipole must sit on a finite-difference node";
  }
  return std::string();
}

bool top_absorbs(const dd_problem* p, int64_t level) {
  return (p->d.absorbing_faces & DD_FACE_TOP) && (double)level * p->d.dt > p->d.t_switch;
}

FdArgs fd_base(const dd_problem* p) {
  FdArgs a;
  std::memset(&a, 0, sizeof(a));
  a.N = p->N;
  a.nx = p->nx; a.ny = p->ny; a.nz = p->nz;
  for (int c = 0; c < 3; ++c) {
    a.blo[c] = p->d.fem_lo[c];
    a.bhi[c] = p->d.fem_lo[c] + p->d.fem_cells[c];
    a.fs[c] = p->fs[c];
  }
  a.nbx = p->nbx; a.nby = p->nby; a.nbz = p->nbz; a.ntiles = p->n_tiles; a.per_xcd = p->per_xcd;
  const double nu = p->d.dt / p->d.h;
  a.nu = (float)nu;
  a.nu2 = (float)(nu * nu);
  a.abs_mask = p->d.absorbing_faces;
  a.dip_idx = -1;
  a.det_mask = p->d.detector_faces;
  a.dt2_h3 = (float)(p->d.dt * p->d.dt / (p->d.h * p->d.h * p->d.h));
  a.n_l0 = p->n_l0;
  a.e_coef = p->d.h * p->d.h * p->d.h / (2.0 * p->d.dt * p->d.dt);
  a.tb_nbz = p->tb_nbz; a.tb_ntiles = p->tb_ntiles; a.tb_per_xcd = p->tb_per_xcd;
  a.tb_list = p->tb_list; a.tb_nlist = p->tb_nlist;
  return a;
}

FemArgs fem_base(const dd_problem* p) {
  FemArgs a;
  std::memset(&a, 0, sizeof(a));
  a.own_off = p->own_off; a.halo_off = p->halo_off; a.halo = p->halo;
  a.col_base = p->col_base; a.ncol = p->ncol; a.col_off = p->col_off;
  a.elems = p->elems; a.geom = p->geom; a.n_geom = p->n_geom; a.own_grid = p->own_grid;
  a.lds_loc = p->lds_loc; a.lds_own = p->lds_own; a.lds_elem = p->lds_elem;
  a.inc = p->inc; a.inc_off = p->inc_off; a.inc_n = p->inc_n;
  a.gather = p->fem_gather && p->inc ? 1 : 0;
  a.part_dims = p->part_dims; a.box_codes = p->box_codes; a.slot_off = p->slot_off;
  a.slot_k = p->slot_k; a.slot_b = p->slot_b; a.n_slots = p->n_slots; a.lds_box = p->lds_box;
  a.n_part = p->n_part;
  a.em1 = p->em1; a.c1 = p->c1; a.c2 = p->c2; a.mass_d = p->mass_d;
  a.n_own = p->n_own; a.n_l0 = p->n_l0; a.N = p->N;
  a.epart_off = p->n_tiles;
  a.r2 = p->r2 ? 1 : 0;
  a.h = (float)p->d.h;
  const double dt = p->d.dt;
  a.inv_2dt2 = 1.0 / (2.0 * dt * dt);
  a.inv_dt2 = 1.0 / (dt * dt);
  a.inv_2dt = 1.0 / (2.0 * dt);
  return a;
}

void fem_fwd(const dd_problem* p, const FemArgs& a, hipStream_t st, bool energy) {
  if (p->use_stencil)
    launch_fem_stencil_fwd(a, p->n_part, st, energy);
  else
    launch_fem_fwd(a, p->n_part, st, energy);
}

void fem_adj(const dd_problem* p, const FemArgs& a, hipStream_t st) {
  if (p->use_stencil)
    launch_fem_stencil_adj(a, p->n_part, st);
  else
    launch_fem_adj(a, p->n_part, st);
}

void zero_state(dd_problem* p, hipStream_t st) {
  for (int b = 0; b < 4; ++b)
    if (p->Efd[b]) launch_fill_f32(p->Efd[b], 3 * p->N, 0.f, st);
  for (int b = 0; b < 2; ++b) launch_fill_f32(p->Efem[b], 3 * p->n_own, 0.f, st);
  launch_fill_f32(p->Vfem, 3 * p->n_own, 0.f, st);
  launch_fill_f32(p->iring, 6 * p->n_l0, 0.f, st);
}

// Bytes of the two levels of E on the FD grid, the set every step streams through.
double fd_field_bytes(const dd_problem* p) { return 24.0 * (double)p->N; }

// Segments of the adjoint: [k0, k1) per segment, K steps each, the last one shorter.
int64_t n_segments(const dd_problem* p) {
  const int64_t nt = p->d.n_steps, K = p->d.ckpt_every;
  return (nt + K - 1) / K;
}
int64_t last_segment_start(const dd_problem* p) { return (n_segments(p) - 1) * (int64_t)p->d.ckpt_every; }

int ensure_saved_storage(dd_problem* p, int n_src) {
  const int64_t nt = p->d.n_steps;
  const int64_t tail_levels = nt - last_segment_start(p) + 1;
  while ((int)p->ihist.size() < n_src) {
    float *h = nullptr, *c = nullptr, *t = nullptr;
    int rc = dalloc(p, &h, (size_t)(nt + 1) * 3 * p->n_l0);
    if (rc) return rc;
    rc = dalloc(p, &c, (size_t)p->n_ck * 6 * p->n_own);
    if (rc) return rc;
    rc = dalloc(p, &t, (size_t)tail_levels * 6 * p->n_own);
    if (rc) return rc;
    p->ihist.push_back(h);
    p->ckpt.push_back(c);
    p->tail.push_back(t);
  }
  const int64_t K = p->d.ckpt_every;
  if (!p->win && n_segments(p) > 1) {
    int rc = dalloc(p, &p->win, (size_t)(K + 1) * 6 * p->n_own);
    if (rc) return rc;
  }
  if (!p->win_b && n_segments(p) > 2) {
    int rc = dalloc(p, &p->win_b, (size_t)(K + 1) * 6 * p->n_own);
    if (rc) return rc;
  }
  return DD_OK;
}

// Two-stream step pipeline: within a step the FD launch (main stream) and the FEM launch
// (aux stream) are independent; across steps each waits for both of the previous step.
void fork_streams(dd_problem* p, hipStream_t st) {
  if (!p->overlap) return;
  (void)hipEventRecord(p->ev_fd, st);
  (void)hipStreamWaitEvent(p->aux, p->ev_fd, 0);
}
void step_barrier(dd_problem* p, hipStream_t st) {
  if (!p->overlap) return;
  (void)hipEventRecord(p->ev_fd, st);
  (void)hipEventRecord(p->ev_fem, p->aux);
  (void)hipStreamWaitEvent(st, p->ev_fem, 0);
  (void)hipStreamWaitEvent(p->aux, p->ev_fd, 0);
}
void join_streams(dd_problem* p, hipStream_t st) {
  if (!p->overlap) return;
  (void)hipEventRecord(p->ev_fem, p->aux);
  (void)hipStreamWaitEvent(st, p->ev_fem, 0);
}

// ---- per-step argument builders (shared by the single-problem driver and the batch engine)

struct SrcPlan {
  int64_t dip_idx = -1;
  double dip_scale = 0.0;   // dt^2 / m at the dipole node
  // obliquely incident plane wave: unit direction's in-face components (time per unit length,
  // the wave speed being 1) and the top-face node of delay 0
  bool oblique = false;
  double kx = 0.0, ky = 0.0;
  int x0 = 0, y0 = 0;
};

SrcPlan source_plan(const dd_problem* p, const dd_source& src) {
  SrcPlan sp;
  if (src.kind != DD_SRC_DIPOLE) {
    const double n = std::sqrt(src.dir[0] * src.dir[0] + src.dir[1] * src.dir[1] + src.dir[2] * src.dir[2]);
    if (n > 0.0 && (src.dir[0] != 0.0 || src.dir[1] != 0.0)) {
      sp.oblique = true;
      sp.kx = src.dir[0] / n;
      sp.ky = src.dir[1] / n;
      // the node the wave front reaches first: the smallest k . x over the top face
      sp.x0 = sp.kx < 0.0 ? p->nx - 1 : 0;
      sp.y0 = sp.ky < 0.0 ? p->ny - 1 : 0;
    }
  }
  if (src.kind == DD_SRC_DIPOLE) {
    sp.dip_idx = src.pos[0] + (int64_t)p->nx * (src.pos[1] + (int64_t)p->ny * src.pos[2]);
    int b = 0;
    b += (src.pos[0] == 0 || src.pos[0] == p->nx - 1);
    b += (src.pos[1] == 0 || src.pos[1] == p->ny - 1);
    b += (src.pos[2] == 0 || src.pos[2] == p->nz - 1);
    const double h = p->d.h;
    sp.dip_scale = p->d.dt * p->d.dt / (h * h * h * std::ldexp(1.0, -b));
  }
  return sp;
}

// Starting state (rest, or the levels of the initial data when `initial`) and the level-0
// entries of the saved forward of source s.
void forward_prologue(dd_problem* p, int s, bool save, bool initial, hipStream_t st) {
  zero_state(p, st);
  if (save) {
    launch_fill_f32(p->ihist[s], 3 * p->n_l0, 0.f, st);   // layer-0 values of level 0
    launch_fill_f32(p->ckpt[s], 6 * p->n_own, 0.f, st);   // checkpoint of level 0
    if (last_segment_start(p) == 0) launch_fill_f32(p->tail[s], 6 * p->n_own, 0.f, st);
  }
  if (initial && p->init_on) {
    // level 0 in Efd[0] / Efem[0], level -1 in Efd[1], the increment V^0 in Vfem
    const int blo[3] = {p->d.fem_lo[0], p->d.fem_lo[1], p->d.fem_lo[2]};
    launch_init_grid(p->init_f0, p->init_f1, p->d.dt, p->nx, p->ny, p->nz, blo, p->fs, p->n_l0, p->Efd[0], p->Efd[1],
                     save ? p->ihist[s] : p->iring, st);
    launch_init_own(p->init_f0, p->init_f1, p->d.dt, p->own_api, p->n_own, p->nx, p->ny, blo, p->fs, p->Efem[0],
                    p->Vfem, save ? p->ckpt[s] : nullptr,
                    (save && last_segment_start(p) == 0) ? p->tail[s] : nullptr, st);
  }
}

// Arguments of forward step n (level n -> n+1) of source s.
void fwd_step_args(const dd_problem* p, const dd_source& src, const SrcPlan& sp, int s, int64_t n, float* traces,
                   bool save, FdArgs& fa, FemArgs& ea) {
  const int64_t nt = p->d.n_steps, K = p->d.ckpt_every;
  const int64_t n_l0 = p->n_l0, n_own = p->n_own;
  const double dt = p->d.dt, h = p->d.h;
  const double t = (double)n * dt;
  const double P = source_time(src, t);
  const int cur = (int)(n & 1), nxt = (int)((n + 1) & 1);
  fa.X_in = p->Efd[cur];
  fa.X_out = p->Efd[nxt];
  // grids larger than the last-level cache: alternate steps sweep in reverse, starting where
  // the previous step ended (whose fields the cache still holds)
  fa.rev = ea.rev = (int)(n & 1);
  fa.top_a = fa.top_b = top_absorbs(p, n) ? 1 : 0;
  const bool plane_on = src.kind != DD_SRC_DIPOLE && t <= p->d.t_switch;
  for (int c = 0; c < 3; ++c) {
    fa.pw[c] = (plane_on && !sp.oblique) ? (float)(2.0 * dt * dt / h * P * src.pol[c]) : 0.f;
    fa.dip[c] = (float)(P * src.pol[c] * sp.dip_scale);
  }
  fa.dip_idx = sp.dip_idx;
  // oblique incidence: the kernel evaluates the delayed pulse per top-face node
  fa.pw_kind = (plane_on && sp.oblique) ? src.kind : 0;
  if (fa.pw_kind) {
    for (int c = 0; c < 3; ++c) fa.pw_amp[c] = (float)(2.0 * dt * dt / h * src.amp * src.pol[c]);
    fa.pw_kx = (float)(sp.kx * h);
    fa.pw_ky = (float)(sp.ky * h);
    fa.pw_x0 = sp.x0;
    fa.pw_y0 = sp.y0;
    fa.pw_omega = (float)src.omega;
    if (src.kind == DD_SRC_GAUSS_SINE) {
      fa.pw_t = (float)(t - src.t0);
      fa.pw_iw = (float)(1.0 / src.width);
      fa.pw_sup = (float)src.t0;
    } else {
      fa.pw_t = (float)t;
      fa.pw_iw = 0.f;
      fa.pw_sup = (float)(2.0 * M_PI / src.omega);
    }
  }
  fa.tr_out = traces + ((int64_t)s * nt + n) * p->n_det * 3;
  fa.cot_in = nullptr;
  fa.obs_in = nullptr;
  fa.iface_out = save ? p->ihist[s] + (n + 1) * 3 * n_l0 : p->iring + nxt * 3 * n_l0;
  ea.X_in = p->Efem[cur];
  ea.X_out = p->Efem[nxt];
  ea.I_in = ea.I_out = p->Vfem;
  ea.iface_in = save ? p->ihist[s] + n * 3 * n_l0 : p->iring + cur * 3 * n_l0;
  ea.fd_out = p->Efd[nxt];
  // dual write of the new FEM state: the last segment entirely, else segment-start checkpoints
  const int64_t k_tail = last_segment_start(p);
  ea.ck_X = nullptr;
  if (save && n + 1 >= k_tail)
    ea.ck_X = p->tail[s] + (n + 1 - k_tail) * 6 * n_own;
  else if (save && (n + 1) % K == 0 && (n + 1) / K < p->n_ck)
    ea.ck_X = p->ckpt[s] + ((n + 1) / K) * 6 * n_own;
  ea.ck_I = ea.ck_X ? ea.ck_X + 3 * n_own : nullptr;
}

// Forward FEM state of the levels of segment seg: stored by the forward for the last
// segment, recomputed into the shared window otherwise.
float* segment_window(const dd_problem* p, int s, int64_t seg) {
  if (seg == n_segments(p) - 1) return p->tail[s];
  return (seg & 1) ? p->win_b : p->win;
}

void segment_prologue(dd_problem* p, int s, int64_t seg, hipStream_t st) {
  if (seg != n_segments(p) - 1)
    launch_copy_f32(segment_window(p, s, seg), p->ckpt[s] + seg * 6 * p->n_own, 6 * p->n_own, st);
}

// Arguments of the FEM-only forward recompute of level k -> k+1 inside segment [k0, k1).
void recompute_args(const dd_problem* p, int s, int64_t k, int64_t k0, float* win, FemArgs& fw) {
  const int64_t n_own = p->n_own;
  fw.X_in = win + (k - k0) * 6 * n_own;
  fw.X_out = win + (k - k0 + 1) * 6 * n_own;
  fw.I_in = fw.X_in + 3 * n_own;
  fw.I_out = fw.X_out + 3 * n_own;
  fw.iface_in = p->ihist[s] + k * 3 * p->n_l0;
  fw.rev = (int)(k & 1);
  fw.fd_out = nullptr;
  fw.ck_X = fw.ck_I = nullptr;
}

// Arguments of adjoint step k (lambda^k -> lambda^{k-1}) of source s inside segment k0.
void adj_step_args(const dd_problem* p, int s, int64_t k, int64_t k0, const float* win, const float* cot,
                   const float* obs, FdArgs& fa, FemArgs& ea) {
  const int64_t nt = p->d.n_steps, n_l0 = p->n_l0, n_own = p->n_own;
  const int cur = (int)(k & 1), prv = (int)((k - 1) & 1);
  fa.X_in = p->Efd[cur];
  fa.X_out = p->Efd[prv];
  fa.rev = ea.rev = (int)(k & 1);
  fa.top_a = top_absorbs(p, k - 1) ? 1 : 0;
  fa.top_b = top_absorbs(p, k + 1) ? 1 : 0;
  for (int c = 0; c < 3; ++c) fa.pw[c] = fa.dip[c] = 0.f;
  fa.dip_idx = -1;
  fa.tr_out = nullptr;
  const int64_t row = ((int64_t)s * nt + (k - 1)) * p->n_det * 3;
  fa.cot_in = cot + row;
  fa.obs_in = obs ? obs + row : nullptr;
  fa.iface_out = p->iring + prv * 3 * n_l0;
  ea.X_in = p->Efem[cur];
  ea.X_out = p->Efem[prv];
  ea.I_in = ea.I_out = p->Vfem;
  ea.iface_in = p->iring + cur * 3 * n_l0;
  ea.fd_out = p->Efd[prv];
  ea.ck_X = ea.ck_I = nullptr;
  ea.wE = win + (k - k0) * 6 * n_own;
  ea.wV = ea.wE + 3 * n_own;
  ea.wVm = win + (k - 1 - k0) * 6 * n_own + 3 * n_own;
  ea.g_eps = p->g_eps;
  ea.g_sig = p->g_sig;
}

// The per-step data of a step's FD arguments (the second step of a two-step launch).
FdStepData step_data(const FdArgs& f) {
  FdStepData d;
  for (int c = 0; c < 3; ++c) {
    d.pw[c] = f.pw[c];
    d.dip[c] = f.dip[c];
  }
  d.top_a = f.top_a; d.top_b = f.top_b; d.pw_kind = f.pw_kind; d.pw_t = f.pw_t;
  d.tr_out = f.tr_out; d.cot_in = f.cot_in; d.obs_in = f.obs_in;
  return d;
}

// Temporal blocking: FD levels in four rotating buffers, level m in Efd[m & 3].  A step from
// level `from` to level `to` (= from + 1 forward, from - 1 adjoint) reads `from` and the level
// on the other side of it, and writes `to`; the FEM dual-writes layer 1 of `to`.
void tb_levels(const dd_problem* p, int64_t from, int64_t to, FdArgs& fa, FemArgs& ea) {
  const int64_t other = 2 * from - to;
  fa.X_in = p->Efd[from & 3];
  fa.X_prev = p->Efd[other & 3];
  fa.X_out = p->Efd[to & 3];
  ea.fd_out = p->Efd[to & 3];
}

// Whether the forward / adjoint of this problem takes two-step launches: the fused one-stream
// path with the div-div form R1, no energy, no initial data (and, for the adjoint, without the
// paper-formula variant's extra terms).
bool tb_forward(const dd_problem* p, bool energy) {
  return p->tb && p->use_stencil && p->fused && !p->overlap && !p->r2 && !p->init_on && !energy;
}
bool tb_adjoint(const dd_problem* p) {
  return p->tb && p->use_stencil && p->fused && !p->overlap && !p->r2 && !p->pg_on && !p->init_on;
}

int run_forward(dd_problem* p, const dd_source& src, int s, float* traces, bool save, double* energy, hipStream_t st) {
  const int64_t nt = p->d.n_steps;
  forward_prologue(p, s, save, true, st);
  hipStream_t sf = p->overlap ? p->aux : st;           // stream of the FEM launches
  fork_streams(p, st);
  FdArgs fa = fd_base(p);
  FemArgs ea = fem_base(p);
  const SrcPlan sp = source_plan(p, src);
  fa.epart = energy ? p->epart : nullptr;
  ea.epart = energy ? p->epart : nullptr;
  const bool fused = p->use_stencil && p->fused;
  // the element-coloured FEM path (general meshes) fuses its forward step too
  const bool el_fused = !p->use_stencil && p->fused && !p->overlap;
  const bool tb = tb_forward(p, energy != nullptr);
  for (int64_t n = 0; n < nt; ++n) {
    fwd_step_args(p, src, sp, s, n, traces, save, fa, ea);
    long ps = -1;
    if (tb) {
      tb_levels(p, n, n + 1, fa, ea);
      if ((n & 1) == 0 && n + 1 < nt) {
        // first launch of a pair: far tiles also take step n + 1
        FdArgs f2 = fa;
        FemArgs e2 = ea;
        fwd_step_args(p, src, sp, s, n + 1, traces, save, f2, e2);
        fa.s2 = step_data(f2);
        fa.X_out2 = p->Efd[(n + 2) & 3];
        ps = prof_begin(p, DD_PROF_PAIR_FWD, st);
        launch_step_pair(fa, ea, st, false, p->tb_nt, 1);
        prof_end(p, DD_PROF_PAIR_FWD, ps, st);
      } else if (n & 1) {
        ps = prof_begin(p, DD_PROF_PAIR2_FWD, st);
        launch_step_pair(fa, ea, st, false, p->tb_nt, 0);
        prof_end(p, DD_PROF_PAIR2_FWD, ps, st);
      } else {
        // the last step of an odd count: one whole step
        ps = prof_begin(p, DD_PROF_STEP_FWD, st);
        launch_step(fa, ea, st, false, false, p->fd_nt);
        prof_end(p, DD_PROF_STEP_FWD, ps, st);
      }
    } else if (fused) {
      ps = prof_begin(p, DD_PROF_STEP_FWD, st);
      launch_step(fa, ea, st, false, energy != nullptr, p->fd_nt);
      prof_end(p, DD_PROF_STEP_FWD, ps, st);
    } else if (el_fused) {
      ps = prof_begin(p, DD_PROF_STEP_FWD, st);
      launch_step_el(fa, ea, st, false, energy != nullptr, p->fd_nt);
      prof_end(p, DD_PROF_STEP_FWD, ps, st);
    } else {
      ps = prof_begin(p, DD_PROF_FD_FWD, st);
      launch_fd(fa, st, energy != nullptr, p->fd_nt);
      prof_end(p, DD_PROF_FD_FWD, ps, st);
      ps = prof_begin(p, DD_PROF_FEM_FWD, sf);
      fem_fwd(p, ea, sf, energy != nullptr);
      prof_end(p, DD_PROF_FEM_FWD, ps, sf);
      step_barrier(p, st);
    }
    if (energy) launch_energy_reduce(p->epart, p->n_tiles + p->n_part, energy + (int64_t)s * nt + n, st);
  }
  join_streams(p, st);
  return check_launch(p);
}

int run_adjoint(dd_problem* p, int s, const float* cot, const float* obs, hipStream_t st) {
  const int64_t nt = p->d.n_steps, K = p->d.ckpt_every;
  zero_state(p, st);
  FdArgs fa = fd_base(p);
  FemArgs fw = fem_base(p);   // recompute (forward, FEM only)
  FemArgs ea = fem_base(p);   // adjoint
  const int64_t nseg = n_segments(p);
  hipStream_t sf = p->overlap ? p->aux : st;
  const bool fused = p->use_stencil && p->fused;
  const bool tb = tb_adjoint(p);
  // Segment pipeline (single-stream steps): the FEM recompute of a segment runs on `aux`,
  // into its own window, while the adjoint steps of the segment after it run on st.  A
  // segment's steps wait for its recompute; a recompute reuses the window of the segment
  // two later, after that segment's steps.
  const bool pipe = !p->overlap;
  auto recompute = [&](int64_t seg, hipStream_t rs) {
    const int64_t k0 = seg * K, k1 = std::min(k0 + K, nt);
    float* win = segment_window(p, s, seg);
    segment_prologue(p, s, seg, rs);
    for (int64_t k = k0; k < k1; ++k) {
      recompute_args(p, s, k, k0, win, fw);
      const long ps = prof_begin(p, DD_PROF_FEM_RECOMPUTE, rs);
      fem_fwd(p, fw, rs, false);
      prof_end(p, DD_PROF_FEM_RECOMPUTE, ps, rs);
    }
    if (pipe) (void)hipEventRecord(p->ev_rec[seg & 1], rs);
  };
  if (pipe) {
    // aux starts after the work already queued on st (the forward's checkpoints)
    (void)hipEventRecord(p->ev_adj, st);
    (void)hipStreamWaitEvent(p->aux, p->ev_adj, 0);
    if (nseg >= 2) recompute(nseg - 2, p->aux);
  } else {
    fork_streams(p, st);
  }
  for (int64_t seg = nseg - 1; seg >= 0; --seg) {
    const int64_t k0 = seg * K, k1 = std::min(k0 + K, nt);
    float* win = segment_window(p, s, seg);
    if (seg != nseg - 1) {
      if (pipe) (void)hipStreamWaitEvent(st, p->ev_rec[seg & 1], 0);
      else recompute(seg, sf);
    }
    for (int64_t k = k1; k > k0; --k) {
      adj_step_args(p, s, k, k0, win, cot, obs, fa, ea);
      long ps = -1;
      if (tb) {
        // pairs (k, k - 1) from the last step down; a launch-B step may open the next segment
        tb_levels(p, k, k - 1, fa, ea);
        const bool first = ((nt - k) & 1) == 0;
        if (first && k > 1) {
          FdArgs f2 = fa;
          FemArgs e2 = ea;
          adj_step_args(p, s, k - 1, k0, win, cot, obs, f2, e2);
          fa.s2 = step_data(f2);
          fa.X_out2 = p->Efd[(k - 2) & 3];
          ps = prof_begin(p, DD_PROF_PAIR_ADJ, st);
          launch_step_pair(fa, ea, st, true, p->tb_nt, 1);
          prof_end(p, DD_PROF_PAIR_ADJ, ps, st);
        } else if (!first) {
          ps = prof_begin(p, DD_PROF_PAIR2_ADJ, st);
          launch_step_pair(fa, ea, st, true, p->tb_nt, 0);
          prof_end(p, DD_PROF_PAIR2_ADJ, ps, st);
        } else {
          ps = prof_begin(p, DD_PROF_STEP_ADJ, st);
          launch_step(fa, ea, st, true, false, p->fd_nt, nullptr);
          prof_end(p, DD_PROF_STEP_ADJ, ps, st);
        }
        continue;
      }
      // the div-div gradient terms of lambda^k (the R2 div-div gradient, or the R1 variant's
      // difference): inside the fused step, which reads but does not write lambda^k and E^k,
      // else a launch of their own after the step (lambda^k, ea.X_in, is overwritten two
      // steps later, on the same stream)
      const bool pg_fused = fused && (p->r2 || p->pg_on);
      if (fused) {
        PgArgs pga{};
        if (pg_fused) {
          pga.lam = ea.X_in; pga.E = ea.wE; pga.n_own = p->n_own; pga.api_own = p->api_own;
          for (int c = 0; c < 3; ++c) pga.fs[c] = p->fs[c];
          pga.h = p->d.h; pga.wp = 1.0; pga.wx = p->r2 ? 0.0 : 1.0; pga.acc = p->pg_acc;
        }
        ps = prof_begin(p, DD_PROF_STEP_ADJ, st);
        launch_step(fa, ea, st, true, false, p->fd_nt, pg_fused ? &pga : nullptr);
        prof_end(p, DD_PROF_STEP_ADJ, ps, st);
      } else if (!p->use_stencil && p->fused && !p->overlap && !p->r2 && !p->pg_on) {
        // a general mesh: element-coloured FEM partitions and FD tiles in one launch
        ps = prof_begin(p, DD_PROF_STEP_ADJ, st);
        launch_step_el(fa, ea, st, true, false, p->fd_nt);
        prof_end(p, DD_PROF_STEP_ADJ, ps, st);
      } else {
        ps = prof_begin(p, DD_PROF_FD_ADJ, st);
        launch_fd(fa, st, false, p->fd_nt);
        prof_end(p, DD_PROF_FD_ADJ, ps, st);
        ps = prof_begin(p, DD_PROF_FEM_ADJ, sf);
        fem_adj(p, ea, sf);
        prof_end(p, DD_PROF_FEM_ADJ, ps, sf);
        step_barrier(p, st);
      }
      if ((p->pg_on || p->r2) && !pg_fused)
        launch_paper_grad_step(ea.X_in, ea.wE, p->n_own, p->api_own, p->fs, p->d.h, !p->r2, p->pg_acc, st);
    }
    if (pipe && seg >= 2) {
      (void)hipEventRecord(p->ev_adj, st);
      (void)hipStreamWaitEvent(p->aux, p->ev_adj, 0);
      recompute(seg - 2, p->aux);
    }
  }
  // pipelined: every recompute queued on aux has been waited for by a segment on st
  if (!pipe) join_streams(p, st);
  if (p->init_on) {
    // level-0 rows of the gradient: lambda^0 (the last step's output, Efem[0]) against the
    // stored level 0 (E^0, V^0) of this source
    const float* lam0 = p->Efem[0];
    const float* lvl0 = (nseg == 1) ? p->tail[s] : p->ckpt[s];
    launch_init_mass_row(lam0, lvl0 + 3 * p->n_own, p->own_grid, p->mass_d, p->n_own, 1.0 / (p->d.dt * p->d.dt),
                         p->g_eps, st);
    if (p->r2) {
      launch_divdiv_grad_terms(lam0, lvl0, p->n_own, p->api_own, p->fs, p->d.h, 1.0, 0.0, p->pg_acc, st);
    } else {
      launch_divdiv_grad_terms(lam0, lvl0, p->n_own, p->api_own, p->fs, p->d.h, 0.0, -1.0, p->ic_acc, st);
      if (p->pg_on)
        launch_divdiv_grad_terms(lam0, lvl0, p->n_own, p->api_own, p->fs, p->d.h, 1.0, 1.0, p->pg_acc, st);
    }
  }
  return check_launch(p);
}

template <class T>
void key_put(std::vector<unsigned char>& k, const T& v) {
  const unsigned char* b = reinterpret_cast<const unsigned char*>(&v);
  k.insert(k.end(), b, b + sizeof(T));
}

// Grids up to this many nodes replay a repeated forward as a graph under DD_GRAPH_AUTO: their
// steps take a few microseconds, of which the graph saves 0.5-0.9 (none on larger grids).
constexpr int64_t kGraphAutoNodes = int64_t(1) << 19;

// What the launches of a dd_forward call depend on besides device memory the problem owns
// (coefficients, initial data, saved forward): the sources, the caller's buffers, the flags
// and the problem's launch options.
std::vector<unsigned char> forward_key(const dd_problem* p, const dd_source* src, int32_t n_src, const float* traces,
                                       bool save, const double* energy) {
  std::vector<unsigned char> key;
  for (int s = 0; s < n_src; ++s) {
    const dd_source& q = src[s];
    key_put(key, q.kind); key_put(key, q.amp); key_put(key, q.omega); key_put(key, q.t0); key_put(key, q.width);
    for (int c = 0; c < 3; ++c) { key_put(key, q.pol[c]); key_put(key, q.dir[c]); key_put(key, q.pos[c]); }
  }
  key_put(key, n_src); key_put(key, traces); key_put(key, save); key_put(key, energy);
  key_put(key, p->init_on); key_put(key, p->r2); key_put(key, p->tb); key_put(key, p->fd_nt); key_put(key, p->fused);
  return key;
}

// Whether a call with this key replays the graph of `g` (and records the call for
// DD_GRAPH_AUTO).
bool graph_wanted(dd_problem* p, GraphCache& g, const std::vector<unsigned char>& key) {
  if (p->graph == DD_GRAPH_OFF || p->overlap || p->prof_stride > 0) return false;
  if (p->graph == DD_GRAPH_ON) return true;
  if (p->N > kGraphAutoNodes) return false;
  const bool repeat = (g.exec && key == g.key) || key == g.last;
  g.last = key;
  return repeat;
}

// The launches `queue` issues on a stream, as one HIP graph: captured on the problem's capture
// stream (whose captured work never runs there; streams that join the capture through events
// rejoin it before its end), instantiated, and launched on the caller's stream.  The graph is
// kept and replayed while the key stays the same; a new key captures anew.
template <class Queue>
int graph_run(dd_problem* p, GraphCache& g, const std::vector<unsigned char>& key, hipStream_t st, Queue&& queue) {
  if (!g.exec || key != g.key) {
    if (g.exec) {
      // the last replay may still run
      if (hipEventSynchronize(g.done) != hipSuccess) return fail(p, DD_ERR_HIP, "graph wait failed");
      (void)hipGraphExecDestroy(g.exec);
      g.exec = nullptr;
    }
    if (!p->cap && hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess)
      return fail(p, DD_ERR_HIP, "capture stream creation failed");
    if (!g.done && hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess)
      return fail(p, DD_ERR_HIP, "event creation failed");
    if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return fail(p, DD_ERR_HIP, "stream capture failed to start");
    int rc = queue(p->cap);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap, &graph);
    if (!rc && (e != hipSuccess || !graph)) rc = fail(p, DD_ERR_HIP, "stream capture failed");
    if (!rc && hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      g.exec = nullptr;
      rc = fail(p, DD_ERR_HIP, "graph instantiation failed");
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) return rc;
    g.key = key;
    ++g.captures;
  }
  if (hipGraphLaunch(g.exec, st) != hipSuccess || hipEventRecord(g.done, st) != hipSuccess)
    return fail(p, DD_ERR_HIP, "graph launch failed");
  ++g.replays;
  return DD_OK;
}

void graph_free(GraphCache& g) {
  // the last replay may still run
  if (g.exec && g.done) (void)hipEventSynchronize(g.done);
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.done) (void)hipEventDestroy(g.done);
  g = GraphCache();
}
}  // namespace

extern "C" {

const char* dd_error_string(int code) {
  switch (code) {
    case DD_OK: return "ok";
    case DD_ERR_INVALID_ARG: return "invalid argument";
    case DD_ERR_CONSTRAINT: return "eps/sigma violate the coefficient constraint";
    case DD_ERR_UNSTABLE: return "non-finite field values";
    case DD_ERR_OOM: return "device out of memory";
    case DD_ERR_HIP: return "HIP runtime error";
    case DD_ERR_STATE: return "call out of order";
    case DD_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown error";
  }
}

const char* dd_last_error(const dd_problem* p) { return p ? p->err.c_str() : "null problem"; }

int dd_detector_nodes(const dd_problem_desc* desc, int64_t* out, int64_t capacity, int64_t* n_written) {
  const std::string e = check_desc(desc);
  if (!e.empty()) return DD_ERR_INVALID_ARG;
  const int nx = desc->n_outer[0], ny = desc->n_outer[1], nz = desc->n_outer[2];
  const int64_t n = face_lex_count(nx, ny, nz, desc->detector_faces);
  if (n_written) *n_written = n;
  if (!out) return DD_OK;
  if (capacity < n) return DD_ERR_INVALID_ARG;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int64_t i = face_lex_index(x, y, z, nx, ny, nz, desc->detector_faces);
        if (i >= 0) out[i] = x + (int64_t)nx * (y + (int64_t)ny * z);
      }
  return DD_OK;
}

}  // extern "C"

namespace {
// FEM partition block of the Kuhn split: 8^3 owned nodes, or 8 x 4 x 4 when an 8^3 split leaves
// fewer than 128 partitions (small boxes: the FEM partitions are the longest blocks of a step,
// and more, shorter ones finish sooner; measured on a 32^3-hex box: 10.1 -> 7.5 us per step,
// while from 48^3 hexes up the 8^3 blocks are faster).
void fem_block(const dd_problem_desc* d, int pb[3]) {
  int64_t n8 = 1;
  for (int a = 0; a < 3; ++a) n8 *= (d->fem_cells[a] - 1 + FEM_PB - 1) / FEM_PB;
  pb[0] = FEM_PB;
  pb[1] = pb[2] = n8 < 128 ? FEM_PB / 2 : FEM_PB;
}

// Incidence lists of the element kernel's gather form: per partition, the elements incident to
// each owned node in the partition's colour order (its element order), entry i of owned node l
// at off[p] + i * no + l (element index within the partition << 2 | the node's slot), each list
// padded with 0xFFFF to cnt[p] entries.
std::string build_incidence(const HostMesh& m, std::vector<uint16_t>& inc, std::vector<int>& off,
                            std::vector<int>& cnt) {
  off.assign(m.n_part + 1, 0);
  cnt.assign(m.n_part, 0);
  inc.clear();
  std::vector<std::vector<uint16_t>> lists;
  for (int p = 0; p < m.n_part; ++p) {
    const int o0 = m.own_off[p], no = m.own_off[p + 1] - o0;
    const int cb = m.col_base[p];
    const int e_beg = m.col_off[cb], e_end = m.col_off[cb + m.ncol[p]];
    if (e_end - e_beg > (0xFFFF >> 2)) return "too many elements in a partition for the gather form";
    lists.assign(no, {});
    size_t mx = 0;
    for (int e = e_beg; e < e_end; ++e) {
      const uint64_t w = m.elems[e];
      for (int k = 0; k < 4; ++k) {
        const int loc = (int)((w >> (11 * k)) & 0x7FFu);
        if (loc < no) {
          lists[loc].push_back((uint16_t)(((e - e_beg) << 2) | k));
          mx = std::max(mx, lists[loc].size());
        }
      }
    }
    if (inc.size() + mx * no > (size_t)INT32_MAX) return "incidence lists exceed 2^31 entries";
    off[p] = (int)inc.size();
    cnt[p] = (int)mx;
    inc.resize(inc.size() + mx * no, 0xFFFF);
    for (int l = 0; l < no; ++l)
      for (size_t i = 0; i < lists[l].size(); ++i) inc[off[p] + i * no + l] = lists[l][i];
  }
  off[m.n_part] = (int)inc.size();
  return std::string();
}

}  // namespace

extern "C" {

size_t dd_footprint_bytes(const dd_problem_desc* desc, int32_t n_src) {
  if (!check_desc(desc).empty() || n_src < 0) return 0;
  const int64_t N = (int64_t)desc->n_outer[0] * desc->n_outer[1] * desc->n_outer[2];
  const int64_t fs[3] = {desc->fem_cells[0] + 1, desc->fem_cells[1] + 1, desc->fem_cells[2] + 1};
  const int64_t n_fem = fs[0] * fs[1] * fs[2];
  int pb[3];
  fem_block(desc, pb);
  int64_t n_own = 1, n_part = 1;
  for (int a = 0; a < 3; ++a) {
    n_own *= desc->fem_cells[a] - 1;
    n_part *= (desc->fem_cells[a] - 1 + pb[a] - 1) / pb[a];
  }
  const int64_t n_l0 = face_lex_count((int)fs[0], (int)fs[1], (int)fs[2], 63u);
  const int64_t nt = desc->n_steps, K = effective_ckpt_every(desc);
  const int64_t nseg = (nt + K - 1) / K;
  const int64_t n_ck = nseg, tail_levels = nt - (nseg - 1) * K + 1;
  // tile count of the variant with the most tiles (short z-chunks)
  int nbx, nby, nbz, ntiles, per_xcd;
  fd_tile_grid(desc->n_outer[0], desc->n_outer[1], desc->n_outer[2], false, nbx, nby, nbz, ntiles, per_xcd);
  // per partition of at most pb0 x pb1 x pb2 owned nodes: a staging box / halo list of at
  // most (pb + 2)^3 codes, at most 6 (pb + 1)^3 elements, at most FEM_COLORS_MAX colours
  const int64_t box = (int64_t)(pb[0] + 2) * (pb[1] + 2) * (pb[2] + 2);
  const int64_t elem = 6ll * (pb[0] + 1) * (pb[1] + 1) * (pb[2] + 1);
  int64_t b = 0;
  // topology: partition offsets, colours, halo lists, elements, geometry, index maps, masses,
  // stencil boxes and slots
  b += 4 * (5 * n_part + 2 + n_part * (FEM_COLORS_MAX + 1) + n_part * box) + 8 * n_part * elem;
  b += 4 * 64 * GEOM_STRIDE + 4 * 2 * n_own + 8 * n_own;
  // the element kernel's incidence lists, on the element path only (DD_FEM_PATH=element, as
  // dd_create reads it): an owned node of the Kuhn split lies in at most 24 tetrahedra (2-byte
  // entries, padded per partition), offsets and counts
  if (const char* e = std::getenv("DD_FEM_PATH"))
    if (std::strcmp(e, "element") == 0) b += 2 * 24 * n_part * (int64_t)pb[0] * pb[1] * pb[2] + 4 * (2 * n_part + 1);
  b += 4 * (4 * n_part + n_part * box) + 4 * STENCIL_SLOTS_MAX * 14;
  b += 4 * 4 * n_own;                     // eps - 1, c1, c2, sigma
  b += 4 * 6 * N;                         // E (2 levels) on the grid
  b += 4 * 6 * N + 4 * (int64_t)ntiles;   // two more levels and the near-tile list (two-step launches)
  b += 4 * 9 * n_own;                     // E (2 levels) + V on the FEM nodes
  b += 4 * 6 * n_l0;                      // interface ring
  b += 8 * ((int64_t)ntiles + n_part) + 8 + 8 * 2 * n_own;   // energy partials, error flags, gradients
  b += (int64_t)n_src * ((nt + 1) * 3 * n_l0 * 4 + (n_ck + tail_levels) * 6 * n_own * 4);  // saved forward
  if (nseg > 1) b += (K + 1) * 6 * n_own * 4;  // recompute window
  if (nseg > 2) b += (K + 1) * 6 * n_own * 4;  // the second one (two segments in flight)
  // optional buffers: misfit partials and weights; FEM-node map and sum of the div-div
  // gradient terms (R2 / paper-formula gradient); initial data and its level-0 rows; a CGA run
  b += 8 * 1024 + 8 * nt;
  b += (4 + 8) * n_fem;
  b += 2 * 4 * 3 * N + 8 * n_fem;
  b += (2 * 4 + 2 * 8) * n_fem + 8 * 6 * 1024 + 1024;
  return (size_t)b;
}

namespace {
// A general mesh of the FEM box (dd_create_mesh); null for the Kuhn split.
struct MeshInput {
  int64_t n_extra, n_tets;
  const double* xyz;
  const int32_t* tets;
};

int create_problem(const dd_problem_desc* desc, const MeshInput* gm, dd_alloc_fn alloc_fn, dd_free_fn free_fn,
                   void* ctx, dd_problem** out) {
  if (!out) return DD_ERR_INVALID_ARG;
  *out = nullptr;
  const std::string e = check_desc(desc);
  if (!e.empty()) return DD_ERR_INVALID_ARG;
  if (!check_desc_supported(desc).empty()) return DD_ERR_UNSUPPORTED;
  if ((alloc_fn == nullptr) != (free_fn == nullptr)) return DD_ERR_INVALID_ARG;
  dd_problem* p = new (std::nothrow) dd_problem();
  if (!p) return DD_ERR_OOM;
  p->d = *desc;
  p->d.ckpt_every = effective_ckpt_every(desc);
  p->alloc_fn = alloc_fn;
  p->free_fn = free_fn;
  p->actx = ctx;
  p->nx = desc->n_outer[0];
  p->ny = desc->n_outer[1];
  p->nz = desc->n_outer[2];
  p->N = (int64_t)p->nx * p->ny * p->nz;
  for (int a = 0; a < 3; ++a) p->fs[a] = desc->fem_cells[a] + 1;
  p->n_det = face_lex_count(p->nx, p->ny, p->nz, desc->detector_faces);
  HostMesh m;
  int pb[3];
  fem_block(desc, pb);
  if (gm) pb[0] = pb[1] = pb[2] = FEM_PB;   // a caller mesh: lattice blocks of 8^3 cells by default
  if (const char* e = std::getenv("DD_FEM_PB")) {
    int x = 0, y = 0, z = 0;
    if (std::sscanf(e, "%d,%d,%d", &x, &y, &z) == 3) { pb[0] = x; pb[1] = y; pb[2] = z; }
  }
  bool element_path = gm != nullptr;   // the element-coloured FEM kernel instead of the assembled stencil
  if (const char* e = std::getenv("DD_FEM_PATH"))
    if (std::strcmp(e, "element") == 0) element_path = true;
  const std::string me = gm ? build_mesh_general(*desc, gm->n_extra, gm->xyz, gm->n_tets, gm->tets, m, pb)
                            : build_mesh(*desc, m, pb, element_path);
  if (!me.empty()) {
    delete p;
    // a caller mesh that is malformed is an argument error; one the kernel cannot partition is not
    return gm && me.find("too dense") == std::string::npos && me.find("exceeds") == std::string::npos
               ? DD_ERR_INVALID_ARG : DD_ERR_UNSUPPORTED;
  }
  p->general = gm != nullptr;
  p->n_extra = gm ? gm->n_extra : 0;
  p->n_fem = m.n_fem;
  p->n_own = m.n_own;
  p->n_l0 = m.n_l0;
  p->n_part = m.n_part;
  p->n_geom = m.n_geom;
  p->lds_loc = (m.max_loc + 3) & ~3;     // multiples of 4 floats keep the LDS sub-arrays 16-byte aligned
  p->lds_own = (m.max_own + 3) & ~3;
  p->lds_elem = (m.max_elem + 1) & ~1;
  p->lds_box = m.max_box;
  p->n_slots = m.n_slots;
  p->use_stencil = m.stencil_ok && m.n_slots <= STENCIL_SLOTS_MAX && !element_path;
  if (!p->use_stencil && !element_path) {
    delete p;
    return DD_ERR_UNSUPPORTED;
  }
  p->fd_nt = fd_field_bytes(p) > LLC_BYTES;
  if (const char* e = std::getenv("DD_FD_NT")) p->fd_nt = std::atoi(e) != 0;
  fd_tile_grid(p->nx, p->ny, p->nz, p->fd_nt, p->nbx, p->nby, p->nbz, p->n_tiles, p->per_xcd);
  // temporal blocking (two-step launches), an option of the fused single-stream stencil path:
  // DD_TB=1 switches it on
  p->tb = false;
  if (const char* e = std::getenv("DD_TB")) p->tb = p->use_stencil && std::atoi(e) != 0;
  std::vector<int> tb_list;
  if (p->tb) {
    // four levels stream through a two-step launch
    p->tb_nt = 2.0 * fd_field_bytes(p) > LLC_BYTES;
    if (const char* e = std::getenv("DD_FD_NT")) p->tb_nt = std::atoi(e) != 0;
    const int zc = tb_zc(p->tb_nt);
    p->tb_nbz = (p->nz + zc - 1) / zc;
    p->tb_ntiles = p->nbx * p->nby * p->tb_nbz;
    p->tb_per_xcd = (p->tb_ntiles + N_XCD - 1) / N_XCD;
    int blo[3], bhi[3];
    for (int a = 0; a < 3; ++a) {
      blo[a] = desc->fem_lo[a];
      bhi[a] = desc->fem_lo[a] + desc->fem_cells[a];
    }
    for (int t = 0; t < p->tb_ntiles; ++t) {
      const int c = tb_tile_class(t, p->nbx, p->nby, p->nx, p->ny, p->nz, zc, blo, bhi);
      if (c == 0) continue;
      // FD-updated nodes of the tile: its nodes in the grid minus those of the open box
      const int bx = t % p->nbx, by = (t / p->nbx) % p->nby, bz = t / (p->nbx * p->nby);
      const int lo[3] = {bx * FD_TX, by * FD_TY, bz * zc};
      const int hi[3] = {std::min(lo[0] + FD_TX, p->nx), std::min(lo[1] + FD_TY, p->ny), std::min(lo[2] + zc, p->nz)};
      int64_t all = 1, inner = 1;
      for (int a = 0; a < 3; ++a) {
        all *= hi[a] - lo[a];
        inner *= std::max(0, std::min(hi[a], bhi[a]) - std::max(lo[a], blo[a] + 1));
      }
      if (c == 1) {
        tb_list.push_back(t);
        p->tb_near += all - inner;
      } else {
        p->tb_far += all - inner;
      }
    }
    p->tb_nlist = (int)tb_list.size();
  }
  p->n_ck = (int)((desc->n_steps + desc->ckpt_every - 1) / desc->ckpt_every);
  if (const char* ov = std::getenv("DD_OVERLAP")) p->overlap = std::atoi(ov) != 0;
  if (const char* fu = std::getenv("DD_FUSED")) p->fused = std::atoi(fu) != 0;
  if (const char* e = std::getenv("DD_GRAPH")) p->graph = std::atoi(e);
  int rc = DD_OK;
  auto chk = [&](int r) { if (r && !rc) rc = r; };
  chk(upload(p, &p->own_off, m.own_off));
  chk(upload(p, &p->halo_off, m.halo_off));
  chk(upload(p, &p->halo, m.halo));
  chk(upload(p, &p->col_base, m.col_base));
  chk(upload(p, &p->ncol, m.ncol));
  chk(upload(p, &p->col_off, m.col_off));
  chk(upload(p, &p->own_grid, m.own_grid));
  chk(upload(p, &p->own_api, m.own_api));
  chk(upload(p, &p->elems, m.elems));
  if (!p->use_stencil) {
    // the element kernel's gather form (DD_FEM_GATHER=0: the colour-by-colour scatter)
    if (const char* e = std::getenv("DD_FEM_GATHER")) p->fem_gather = std::atoi(e) != 0;
    std::vector<uint16_t> inc;
    std::vector<int> inc_off, inc_n;
    if (p->fem_gather && build_incidence(m, inc, inc_off, inc_n).empty()) {
      chk(upload(p, &p->inc, inc));
      chk(upload(p, &p->inc_off, inc_off));
      chk(upload(p, &p->inc_n, inc_n));
    }
  }
  chk(upload(p, &p->geom, m.geom));
  chk(upload(p, &p->mass_d, m.mass));
  if (gm) {
    std::vector<double> wa((size_t)m.n_fem, 0.0);
    for (int64_t id = 0; id < m.n_own; ++id) wa[m.own_api[id]] = m.mass[id];
    chk(upload(p, &p->mass_api, wa));
  }
  if (m.stencil_ok) {
    chk(upload(p, &p->part_dims, m.part_dims));
    chk(upload(p, &p->box_codes, m.box_codes));
    chk(upload(p, &p->slot_off, m.slot_off));
    chk(upload(p, &p->slot_k, m.slot_k));
    chk(upload(p, &p->slot_b, m.slot_b));
  }
  chk(dalloc(p, &p->em1, p->n_own));
  chk(dalloc(p, &p->c1, p->n_own));
  chk(dalloc(p, &p->c2, p->n_own));
  chk(dalloc(p, &p->sig_own, p->n_own));
  for (int b = 0; b < 2; ++b) {
    chk(dalloc(p, &p->Efd[b], 3 * p->N));
    chk(dalloc(p, &p->Efem[b], 3 * p->n_own));
  }
  if (p->tb) {
    chk(dalloc(p, &p->Efd[2], 3 * p->N));
    chk(dalloc(p, &p->Efd[3], 3 * p->N));
    if (!tb_list.empty()) chk(upload(p, &p->tb_list, tb_list));
  }
  chk(dalloc(p, &p->Vfem, 3 * p->n_own));
  chk(dalloc(p, &p->iring, 6 * p->n_l0));
  chk(dalloc(p, &p->epart, p->n_tiles + p->n_part));
  chk(dalloc(p, &p->d_err, 2));   // [0]: synchronous checks, [1]: the last dd_set_coefficients_async
  chk(dalloc(p, &p->g_eps, p->n_own));
  chk(dalloc(p, &p->g_sig, p->n_own));
  if (!rc && (hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking) != hipSuccess ||
              hipEventCreateWithFlags(&p->ev_fd, hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&p->ev_fem, hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&p->ev_rec[0], hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&p->ev_rec[1], hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&p->ev_adj, hipEventDisableTiming) != hipSuccess))
    rc = DD_ERR_HIP;
  if (rc) {
    dd_destroy(p);
    return rc;
  }
  // eps = 1, sigma = 0 until dd_set_coefficients
  std::vector<float> em1(p->n_own, 0.f), c1(p->n_own, 1.f), c2(p->n_own);
  for (int64_t i = 0; i < p->n_own; ++i) c2[i] = (float)(desc->dt * desc->dt / m.mass[i]);
  const int zeros[2] = {0, 0};
  if (hipMemcpy(p->em1, em1.data(), 4 * p->n_own, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->sig_own, em1.data(), 4 * p->n_own, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_err, zeros, sizeof(zeros), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->c1, c1.data(), 4 * p->n_own, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->c2, c2.data(), 4 * p->n_own, hipMemcpyHostToDevice) != hipSuccess) {
    dd_destroy(p);
    return DD_ERR_HIP;
  }
  *out = p;
  return DD_OK;
}
}  // namespace

int dd_create(const dd_problem_desc* desc, dd_alloc_fn alloc_fn, dd_free_fn free_fn, void* ctx, dd_problem** out) {
  return create_problem(desc, nullptr, alloc_fn, free_fn, ctx, out);
}

int dd_create_mesh(const dd_problem_desc* desc, int64_t n_extra, const double* extra_xyz, int64_t n_tets,
                   const int32_t* tets, dd_alloc_fn alloc_fn, dd_free_fn free_fn, void* ctx, dd_problem** out) {
  if (n_extra < 0 || n_tets < 1 || !tets || (n_extra > 0 && !extra_xyz)) {
    if (out) *out = nullptr;
    return DD_ERR_INVALID_ARG;
  }
  const MeshInput gm{n_extra, n_tets, extra_xyz, tets};
  return create_problem(desc, &gm, alloc_fn, free_fn, ctx, out);
}

int dd_destroy(dd_problem* p) {
  if (!p) return DD_ERR_INVALID_ARG;
  // hipMalloc memory: nothing may still read it.  A caller allocator orders reuse after the
  // work queued on the caller's stream; the library's own second stream is waited for here.
  if (!p->free_fn) (void)hipDeviceSynchronize();
  else if (p->aux) (void)hipStreamSynchronize(p->aux);
  for (auto& v : p->ev)
    for (hipEvent_t e : v) (void)hipEventDestroy(e);
  if (p->ev_fd) (void)hipEventDestroy(p->ev_fd);
  if (p->ev_fem) (void)hipEventDestroy(p->ev_fem);
  for (hipEvent_t e : {p->ev_rec[0], p->ev_rec[1], p->ev_adj})
    if (e) (void)hipEventDestroy(e);
  if (p->aux) (void)hipStreamDestroy(p->aux);
  graph_free(p->gfwd);
  graph_free(p->gadj);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  for (void* q : p->allocs) raw_free(p->free_fn, p->actx, q);
  delete p;
  return DD_OK;
}

int dd_sizes(const dd_problem* p, int64_t* n_fem_nodes, int64_t* n_detectors, int64_t* n_grid) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (n_fem_nodes) *n_fem_nodes = p->n_fem;
  if (n_detectors) *n_detectors = p->n_det;
  if (n_grid) *n_grid = p->N;
  return DD_OK;
}

int dd_set_coefficients(dd_problem* p, const float* eps_dev, const float* sigma_dev, void* stream) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (!eps_dev || !sigma_dev) return fail(p, DD_ERR_INVALID_ARG, "null coefficient pointer");
  hipStream_t st = (hipStream_t)stream;
  int h_err = 0;
  if (hipMemsetAsync(p->d_err, 0, sizeof(int), st) != hipSuccess) return fail(p, DD_ERR_HIP, "hipMemsetAsync failed");
  launch_validate(eps_dev, sigma_dev, p->fs[0], p->fs[1], p->fs[2], p->n_extra, p->d_err, st);
  if (int rc = check_launch(p)) return rc;
  if (hipMemcpyAsync(&h_err, p->d_err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(p, DD_ERR_HIP, "error readback failed");
  if (h_err) return fail(p, DD_ERR_CONSTRAINT, std::to_string(h_err) + " FEM nodes violate the coefficient constraint");
  launch_coefficients(eps_dev, sigma_dev, p->own_api, p->mass_d, p->n_own, p->d.dt, p->em1, p->c1, p->c2, p->sig_own,
                      nullptr, st);
  if (int rc = check_launch(p)) return rc;
  if (hipStreamSynchronize(st) != hipSuccess) return fail(p, DD_ERR_HIP, "stream synchronize failed");
  p->saved = false;
  p->have_grad = false;
  p->have_pg = false;
  return DD_OK;
}

int dd_set_coefficients_async(dd_problem* p, const float* eps_dev, const float* sigma_dev, void* stream) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (!eps_dev || !sigma_dev) return fail(p, DD_ERR_INVALID_ARG, "null coefficient pointer");
  hipStream_t st = (hipStream_t)stream;
  int* flag = p->d_err + 1;
  launch_fill_i32(flag, 1, 0, st);
  launch_validate(eps_dev, sigma_dev, p->fs[0], p->fs[1], p->fs[2], p->n_extra, flag, st);
  launch_coefficients(eps_dev, sigma_dev, p->own_api, p->mass_d, p->n_own, p->d.dt, p->em1, p->c1, p->c2, p->sig_own,
                      flag, st);
  if (int rc = check_launch(p)) return rc;
  p->saved = false;
  p->have_grad = false;
  p->have_pg = false;
  return DD_OK;
}

int dd_coefficients_status(dd_problem* p, void* stream) {
  if (!p) return DD_ERR_INVALID_ARG;
  int h = 0;
  if (hipMemcpyAsync(&h, p->d_err + 1, sizeof(int), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess ||
      hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return fail(p, DD_ERR_HIP, "status readback failed");
  if (h) return fail(p, DD_ERR_CONSTRAINT, std::to_string(h) + " FEM nodes violated the coefficient constraint");
  return DD_OK;
}

int dd_forward(dd_problem* p, const dd_source* src, int32_t n_src, float* traces_dev, int32_t save, double* energy_dev,
               void* stream) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (!src || n_src < 1 || !traces_dev) return fail(p, DD_ERR_INVALID_ARG, "need sources and a trace buffer");
  for (int s = 0; s < n_src; ++s) {
    const std::string e = check_source(p, src[s]);
    if (!e.empty()) return fail(p, DD_ERR_INVALID_ARG, e);
  }
  hipStream_t st = (hipStream_t)stream;
  p->saved = false;
  p->have_grad = false;
  p->have_pg = false;
  if (save) {
    int rc = ensure_saved_storage(p, n_src);
    if (rc) return rc;
  }
  const std::vector<unsigned char> key = forward_key(p, src, n_src, traces_dev, save != 0, energy_dev);
  if (graph_wanted(p, p->gfwd, key)) {
    int rc = graph_run(p, p->gfwd, key, st, [&](hipStream_t cs) {
      int r = DD_OK;
      for (int s = 0; s < n_src && !r; ++s) r = run_forward(p, src[s], s, traces_dev, save != 0, energy_dev, cs);
      return r;
    });
    if (rc) return rc;
  } else {
    for (int s = 0; s < n_src; ++s) {
      int rc = run_forward(p, src[s], s, traces_dev, save != 0, energy_dev, st);
      if (rc) return rc;
    }
  }
  if (save) {
    p->saved = true;
    p->saved_n_src = n_src;
  }
  return DD_OK;
}

namespace {
// The adjoint sweeps of every saved source with their gradient sums cleared first.
int adjoint_launches(dd_problem* p, const float* cot, const float* obs, hipStream_t st) {
  launch_fill_f64(p->g_eps, p->n_own, 0.0, st);
  launch_fill_f64(p->g_sig, p->n_own, 0.0, st);
  if (p->pg_on || p->r2) launch_fill_f64(p->pg_acc, p->n_fem, 0.0, st);
  if (p->ic_used) launch_fill_f64(p->ic_acc, p->n_fem, 0.0, st);
  for (int s = 0; s < p->saved_n_src; ++s) {
    int rc = run_adjoint(p, s, cot, obs, st);
    if (rc) return rc;
  }
  return DD_OK;
}

int adjoint_all(dd_problem* p, const float* cot, const float* obs, hipStream_t st) {
  p->ic_used = p->init_on && !p->r2;
  p->adj_obs = obs != nullptr;
  std::vector<unsigned char> key;
  key_put(key, cot); key_put(key, obs); key_put(key, p->saved_n_src);
  key_put(key, p->pg_on); key_put(key, p->r2); key_put(key, p->init_on); key_put(key, p->tb); key_put(key, p->fd_nt);
  key_put(key, p->fused);
  // one checkpoint segment only: with several, the recompute runs on a second stream, and a
  // graph with that parallel branch gained nothing and its launch held the host until the
  // stream had drained
  if (n_segments(p) == 1 && graph_wanted(p, p->gadj, key)) {
    int rc = graph_run(p, p->gadj, key, st, [&](hipStream_t cs) {
      int r = adjoint_launches(p, cot, obs, cs);
      // the segment recompute stream joined the capture through the sweep's first event
      // wait, with nothing to do in one segment: it rejoins here
      if (!r && (hipEventRecord(p->ev_fem, p->aux) != hipSuccess || hipStreamWaitEvent(cs, p->ev_fem, 0) != hipSuccess))
        r = fail(p, DD_ERR_HIP, "stream join failed");
      return r;
    });
    if (rc) return rc;
  } else {
    int rc = adjoint_launches(p, cot, obs, st);
    if (rc) return rc;
  }
  p->have_grad = true;
  p->have_pg = p->pg_on || p->r2;
  return DD_OK;
}
}  // namespace

int dd_adjoint(dd_problem* p, const float* cot_dev, void* stream) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (!cot_dev) return fail(p, DD_ERR_INVALID_ARG, "null cotangent");
  if (!p->saved) return fail(p, DD_ERR_STATE, "dd_adjoint needs a preceding dd_forward with save");
  return adjoint_all(p, cot_dev, nullptr, (hipStream_t)stream);
}

int dd_adjoint_misfit(dd_problem* p, const float* traces_dev, const float* obs_dev, void* stream) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (!traces_dev || !obs_dev) return fail(p, DD_ERR_INVALID_ARG, "null traces or observations");
  if (!p->saved) return fail(p, DD_ERR_STATE, "dd_adjoint_misfit needs a preceding dd_forward with save");
  return adjoint_all(p, traces_dev, obs_dev, (hipStream_t)stream);
}

int dd_gradient(dd_problem* p, double* g_eps_dev, double* g_sigma_dev, const dd_tikhonov* reg, void* stream) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (!g_eps_dev || !g_sigma_dev) return fail(p, DD_ERR_INVALID_ARG, "null gradient buffer");
  if (reg && (!reg->eps0_dev || !reg->sigma0_dev || !(reg->gamma_eps >= 0.0) || !(reg->gamma_sig >= 0.0) ||
              !std::isfinite(reg->gamma_eps) || !std::isfinite(reg->gamma_sig)))
    return fail(p, DD_ERR_INVALID_ARG, "Tikhonov term needs finite gammas >= 0 and both centres");
  if (!p->have_grad) return fail(p, DD_ERR_STATE, "dd_gradient needs a preceding dd_adjoint");
  hipStream_t st = (hipStream_t)stream;
  launch_fill_f64(g_eps_dev, p->n_fem, 0.0, st);
  launch_fill_f64(g_sigma_dev, p->n_fem, 0.0, st);
  launch_gradient_out(p->g_eps, p->g_sig, p->own_api, p->own_grid, p->n_own, g_eps_dev, g_sigma_dev, st);
  if (p->r2) launch_add_free(p->pg_acc, p->fs, g_eps_dev, st);   // R2: the div-div part is the paper term
  if (p->ic_used) launch_add_free(p->ic_acc, p->fs, g_eps_dev, st);   // level-0 div-div rows (initial data)
  if (reg)
    launch_tikhonov_add(p->em1, p->sig_own, p->own_api, p->own_grid, p->mass_d, p->n_own, reg->gamma_eps,
                        reg->gamma_sig, reg->eps0_dev, reg->sigma0_dev, g_eps_dev, g_sigma_dev, st);
  return check_launch(p);
}

int dd_misfit(dd_problem* p, const float* traces_dev, const float* obs_dev, int32_t n_src, const double* z_host,
              float* cot_dev, double* j_dev, void* stream) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (!traces_dev || !obs_dev || n_src < 1) return fail(p, DD_ERR_INVALID_ARG, "need traces, observations, n_src >= 1");
  hipStream_t st = (hipStream_t)stream;
  const int64_t nt = p->d.n_steps;
  if (!p->mis_part) {
    int rc = dalloc(p, &p->mis_part, (size_t)CGA_MAX_BLOCKS);
    if (!rc) rc = dalloc(p, &p->mis_z, (size_t)nt);
    if (rc) return rc;
  }
  if (z_host) {
    for (int64_t n = 0; n < nt; ++n)
      if (!std::isfinite(z_host[n]) || z_host[n] < 0.0) return fail(p, DD_ERR_INVALID_ARG, "weights must be finite, >= 0");
    // upload only new weights; the copy completes before the call returns, and it is ordered
    // after the work already queued on the stream that reads the previous weights
    if (p->mis_z_host.size() != (size_t)nt || !std::equal(p->mis_z_host.begin(), p->mis_z_host.end(), z_host)) {
      if (hipMemcpyAsync(p->mis_z, z_host, (size_t)nt * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return fail(p, DD_ERR_HIP, "weight upload failed");
      p->mis_z_host.assign(z_host, z_host + nt);
    }
  }
  const int64_t row = p->n_det * 3;
  launch_misfit(traces_dev, obs_dev, (int64_t)n_src * nt * row, row, nt, z_host ? p->mis_z : nullptr, cot_dev,
                p->mis_part, j_dev, st);
  return check_launch(p);
}

int dd_misfit_taper(int32_t n_steps, double dt, double delta, double* z_host) {
  if (n_steps < 1 || !z_host || !(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(delta)) return DD_ERR_INVALID_ARG;
  const double t_end = (double)n_steps * dt;
  for (int32_t n = 0; n < n_steps; ++n) {
    z_host[n] = 1.0;
    if (delta > 0.0) {
      // s runs from 0 at t = T - delta to 1 at the end time T (trace row n is time level n + 1)
      const double s = ((double)(n + 1) * dt - (t_end - delta)) / delta;
      if (s > 0.0) z_host[n] = 0.5 * (1.0 + std::cos(M_PI * std::min(s, 1.0)));
    }
  }
  return DD_OK;
}

int dd_misfit_noalloc(dd_problem* p, const float* traces_dev, const float* obs_dev, int32_t n_src, const double* z_host,
                      float* cot_dev, double* j_dev, void* stream) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (!traces_dev || !obs_dev || n_src < 1) return fail(p, DD_ERR_INVALID_ARG, "need traces, observations, n_src >= 1");
  const int64_t nt = p->d.n_steps;
  if (nt > DD_MISFIT_NOALLOC_MAX_STEPS)
    return fail(p, DD_ERR_INVALID_ARG, "n_steps " + std::to_string(nt) + " exceeds the no-allocation misfit's maximum of " +
                                           std::to_string((int)DD_MISFIT_NOALLOC_MAX_STEPS) + " steps");
  if (z_host)
    for (int64_t n = 0; n < nt; ++n)
      if (!std::isfinite(z_host[n]) || z_host[n] < 0.0) return fail(p, DD_ERR_INVALID_ARG, "weights must be finite, >= 0");
  hipStream_t st = (hipStream_t)stream;
  double* scr = nullptr;   // [CGA_MAX_BLOCKS] block partials, then [n_steps] weights
  if (hipError_t e = misfit_scratch(&scr); e != hipSuccess)
    return fail(p, DD_ERR_HIP, std::string("scratch symbol lookup failed: ") + hipGetErrorString(e));
  double* zd = scr + CGA_MAX_BLOCKS;
  if (z_host) {
    // every call uploads its weights (the array is shared by all calls on this GPU); the copy
    // follows the work already queued on the stream, and completes before the call returns
    if (hipMemcpyAsync(zd, z_host, (size_t)nt * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(p, DD_ERR_HIP, "weight upload failed");
  }
  // every block writes its partial before the one-block sum reads it: nothing to clear
  const int64_t row = p->n_det * 3;
  launch_misfit(traces_dev, obs_dev, (int64_t)n_src * nt * row, row, nt, z_host ? zd : nullptr, cot_dev, scr, j_dev, st);
  return check_launch(p);
}

namespace {
int pg_setup(dd_problem* p) {
  if (p->overlap) return fail(p, DD_ERR_UNSUPPORTED, "the paper-formula gradient needs the single-stream step order");
  if (!p->api_own) {
    int rc = dalloc(p, &p->api_own, (size_t)p->n_fem);
    if (!rc) rc = dalloc(p, &p->pg_acc, (size_t)p->n_fem);
    if (rc) return rc;
    launch_invert_own(p->own_api, p->n_own, p->n_fem, p->api_own, nullptr);
    if (int rc2 = check_launch(p)) return rc2;
    if (hipStreamSynchronize(nullptr) != hipSuccess) return fail(p, DD_ERR_HIP, "stream synchronize failed");
  }
  return DD_OK;
}
}  // namespace

int dd_paper_gradient_enable(dd_problem* p, int32_t on) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (!on) {
    p->pg_on = false;
    return DD_OK;
  }
  if (p->general) return fail(p, DD_ERR_UNSUPPORTED, "the paper-formula gradient needs the Kuhn split of the FEM box");
  if (int rc = pg_setup(p)) return rc;
  p->pg_on = true;
  return DD_OK;
}

int dd_set_graph(dd_problem* p, int32_t mode) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (mode != DD_GRAPH_OFF && mode != DD_GRAPH_ON && mode != DD_GRAPH_AUTO)
    return fail(p, DD_ERR_INVALID_ARG, "unknown graph mode");
  p->graph = mode;
  p->gfwd.last.clear();
  p->gadj.last.clear();
  return DD_OK;
}

int dd_graph_stats(const dd_problem* p, int32_t which, int64_t* captures, int64_t* replays) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (which != DD_GRAPH_FORWARD && which != DD_GRAPH_ADJOINT) return DD_ERR_INVALID_ARG;
  const GraphCache& g = which == DD_GRAPH_FORWARD ? p->gfwd : p->gadj;
  if (captures) *captures = g.captures;
  if (replays) *replays = g.replays;
  return DD_OK;
}

int dd_set_divdiv_form(dd_problem* p, int32_t form) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (form != DD_DIVDIV_R1 && form != DD_DIVDIV_R2) return fail(p, DD_ERR_INVALID_ARG, "unknown div-div form");
  const bool r2 = form == DD_DIVDIV_R2;
  if (r2 == p->r2) return DD_OK;
  if (r2) {
    if (!p->use_stencil) return fail(p, DD_ERR_UNSUPPORTED, "the R2 form needs the assembled-stencil FEM path");
    if (int rc = pg_setup(p)) return rc;
  }
  p->r2 = r2;
  p->saved = false;        // a saved forward of the other form no longer matches
  p->have_grad = false;
  p->have_pg = false;
  return DD_OK;
}

int dd_gradient_paper(dd_problem* p, double* g_eps_dev, double* g_sigma_dev, void* stream) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (!g_eps_dev || !g_sigma_dev) return fail(p, DD_ERR_INVALID_ARG, "null gradient buffer");
  if (!p->have_grad || !p->have_pg)
    return fail(p, DD_ERR_STATE, "dd_gradient_paper needs a preceding dd_adjoint with the variant enabled");
  hipStream_t st = (hipStream_t)stream;
  launch_fill_f64(g_eps_dev, p->n_fem, 0.0, st);
  launch_fill_f64(g_sigma_dev, p->n_fem, 0.0, st);
  launch_gradient_out(p->g_eps, p->g_sig, p->own_api, p->own_grid, p->n_own, g_eps_dev, g_sigma_dev, st);
  launch_add_free(p->pg_acc, p->fs, g_eps_dev, st);
  if (p->ic_used) launch_add_free(p->ic_acc, p->fs, g_eps_dev, st);
  return check_launch(p);
}

int dd_check_finite(dd_problem* p, void* stream) {
  if (!p) return DD_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  int h_err = 0;
  if (hipMemsetAsync(p->d_err, 0, sizeof(int), st) != hipSuccess) return fail(p, DD_ERR_HIP, "hipMemsetAsync failed");
  for (int b = 0; b < 4; ++b)
    if (p->Efd[b]) launch_count_nonfinite(p->Efd[b], 3 * p->N, p->d_err, st);
  for (int b = 0; b < 2; ++b) launch_count_nonfinite(p->Efem[b], 3 * p->n_own, p->d_err, st);
  launch_count_nonfinite(p->Vfem, 3 * p->n_own, p->d_err, st);
  if (int rc = check_launch(p)) return rc;
  if (hipMemcpyAsync(&h_err, p->d_err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(p, DD_ERR_HIP, "error readback failed");
  if (h_err) return fail(p, DD_ERR_UNSTABLE, std::to_string(h_err) + " non-finite field values");
  return DD_OK;
}

int dd_set_initial_data(dd_problem* p, const float* f0_dev, const float* f1_dev, void* stream) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (!f0_dev && !f1_dev) {
    if (p->init_on) {
      p->init_on = false;
      p->saved = false;
      p->have_grad = false;
      p->have_pg = false;
    }
    return DD_OK;
  }
  if (!f0_dev || !f1_dev) return fail(p, DD_ERR_INVALID_ARG, "initial data needs both f_0 and f_1 (or neither)");
  if (p->general) return fail(p, DD_ERR_UNSUPPORTED, "initial data needs the Kuhn split of the FEM box");
  hipStream_t st = (hipStream_t)stream;
  int h_err = 0;
  if (hipMemsetAsync(p->d_err, 0, sizeof(int), st) != hipSuccess) return fail(p, DD_ERR_HIP, "hipMemsetAsync failed");
  launch_count_nonfinite(f0_dev, 3 * p->N, p->d_err, st);
  launch_count_nonfinite(f1_dev, 3 * p->N, p->d_err, st);
  if (int rc = check_launch(p)) return rc;
  if (hipMemcpyAsync(&h_err, p->d_err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(p, DD_ERR_HIP, "error readback failed");
  if (h_err) return fail(p, DD_ERR_CONSTRAINT, std::to_string(h_err) + " non-finite initial data values");
  if (int rc = pg_setup(p)) return rc;   // FEM-node -> owned map of the level-0 div-div rows
  if (!p->init_f0) {
    int rc = dalloc(p, &p->init_f0, (size_t)3 * p->N);
    if (!rc) rc = dalloc(p, &p->init_f1, (size_t)3 * p->N);
    if (!rc) rc = dalloc(p, &p->ic_acc, (size_t)p->n_fem);
    if (rc) return rc;
  }
  const size_t bytes = (size_t)3 * p->N * sizeof(float);
  if (hipMemcpyAsync(p->init_f0, f0_dev, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(p->init_f1, f1_dev, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return fail(p, DD_ERR_HIP, "initial data copy failed");
  p->init_on = true;
  p->saved = false;
  p->have_grad = false;
  p->have_pg = false;
  return DD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Conjugate gradient reconstruction (box "CGA"): device state of one run.
// ---------------------------------------------------------------------------------------
struct dd_cga {
  CgaMesh mesh{};
  int64_t n = 0;
  dd_free_fn free_fn = nullptr;   // the allocator of the problem the run started on
  void* actx = nullptr;
  float* c0 = nullptr;      // [2][n]: eps^0, sigma^0 (Tikhonov centres)
  double* d = nullptr;      // [2][n]: previous directions d^{m-1}
  double* part = nullptr;   // [CGA_MAX_BLOCKS][6] block partials
  CgaDev* st = nullptr;
  double* w = nullptr;      // [n]: a general mesh's lumped masses (own copy; null on the Kuhn split)
};

namespace {
bool cga_params_ok(const dd_cga_params& q, std::string& why) {
  const double v[] = {q.gamma_eps, q.gamma_sig, q.p, q.alpha_eps, q.alpha_sig, q.eps_max, q.sig_max,
                      q.eta1_eps, q.eta1_sig, q.eta2_eps, q.eta2_sig};
  for (double x : v)
    if (!std::isfinite(x)) { why = "CGA parameters must be finite"; return false; }
  if (!(q.gamma_eps > 0.0 && q.gamma_sig > 0.0)) { why = "gamma^0 must be > 0"; return false; }
  if (!(q.p > 0.0 && q.p < 1.0)) { why = "p must lie in (0, 1)"; return false; }
  if (!(q.alpha_eps >= 0.0 && q.alpha_sig >= 0.0)) { why = "alpha^0 must be >= 0"; return false; }
  if (!(q.eps_max > 1.0 && q.sig_max > 0.0)) { why = "need eps_max > 1 and sig_max > 0"; return false; }
  if (!(q.eta1_eps >= 0.0 && q.eta1_sig >= 0.0 && q.eta2_eps >= 0.0 && q.eta2_sig >= 0.0)) {
    why = "tolerances must be >= 0";
    return false;
  }
  return true;
}

void cga_free(dd_cga* c) {
  if (!c) return;
  raw_free(c->free_fn, c->actx, c->c0);
  raw_free(c->free_fn, c->actx, c->d);
  raw_free(c->free_fn, c->actx, c->part);
  raw_free(c->free_fn, c->actx, c->st);
  raw_free(c->free_fn, c->actx, c->w);
  delete c;
}
}  // namespace

extern "C" {

int dd_cga_create(dd_problem* p, const dd_cga_params* prm, const float* eps0_dev, const float* sig0_dev, void* stream,
                  dd_cga** out) {
  if (!p) return DD_ERR_INVALID_ARG;
  if (!prm || !eps0_dev || !sig0_dev || !out) return fail(p, DD_ERR_INVALID_ARG, "null CGA argument");
  *out = nullptr;
  std::string why;
  if (!cga_params_ok(*prm, why)) return fail(p, DD_ERR_INVALID_ARG, why);
  hipStream_t st = (hipStream_t)stream;
  // the initial guess must satisfy eq. epsilon_sigma_constraint, upper bounds included
  int h_err[2] = {0, 0};
  if (hipMemsetAsync(p->d_err, 0, sizeof(int), st) != hipSuccess) return fail(p, DD_ERR_HIP, "hipMemsetAsync failed");
  launch_validate(eps0_dev, sig0_dev, p->fs[0], p->fs[1], p->fs[2], p->n_extra, p->d_err, st);
  if (hipMemcpyAsync(&h_err[0], p->d_err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(p, DD_ERR_HIP, "error readback failed");
  if (hipMemsetAsync(p->d_err, 0, sizeof(int), st) != hipSuccess) return fail(p, DD_ERR_HIP, "hipMemsetAsync failed");
  launch_cga_upper_check(eps0_dev, sig0_dev, p->n_fem, prm->eps_max, prm->sig_max, p->d_err, st);
  if (int rc = check_launch(p)) return rc;
  if (hipMemcpyAsync(&h_err[1], p->d_err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(p, DD_ERR_HIP, "error readback failed");
  if (h_err[0] || h_err[1])
    return fail(p, DD_ERR_CONSTRAINT, std::to_string(h_err[0] + h_err[1]) +
                                          " FEM nodes of the initial guess violate the coefficient box");
  dd_cga* c = new dd_cga();
  for (int a = 0; a < 3; ++a) c->mesh.fs[a] = p->fs[a];
  c->mesh.n_extra = p->n_extra;
  c->n = p->n_fem;
  c->free_fn = p->free_fn;
  c->actx = p->actx;
  c->c0 = static_cast<float*>(raw_alloc(p->alloc_fn, p->actx, 2 * c->n * sizeof(float)));
  c->d = static_cast<double*>(raw_alloc(p->alloc_fn, p->actx, 2 * c->n * sizeof(double)));
  c->part = static_cast<double*>(raw_alloc(p->alloc_fn, p->actx, (size_t)CGA_MAX_BLOCKS * CGA_SUMS * sizeof(double)));
  c->st = static_cast<CgaDev*>(raw_alloc(p->alloc_fn, p->actx, sizeof(CgaDev)));
  if (p->mass_api) c->w = static_cast<double*>(raw_alloc(p->alloc_fn, p->actx, c->n * sizeof(double)));
  if (!c->c0 || !c->d || !c->part || !c->st || (p->mass_api && !c->w)) {
    cga_free(c);
    return fail(p, DD_ERR_OOM, "CGA state allocation failed");
  }
  // a general mesh's masses are copied so that the run keeps nothing of p; on the Kuhn split
  // every free node weighs h^3
  if (c->w && hipMemcpyAsync(c->w, p->mass_api, c->n * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess) {
    cga_free(c);
    return fail(p, DD_ERR_HIP, "copy of the lumped masses failed");
  }
  c->mesh.w = c->w;
  CgaDev h{};
  h.gamma0[0] = h.gamma[0] = prm->gamma_eps;
  h.gamma0[1] = h.gamma[1] = prm->gamma_sig;
  h.p = prm->p;
  h.alpha[0] = prm->alpha_eps;
  h.alpha[1] = prm->alpha_sig;
  h.lo[0] = 1.0;
  h.lo[1] = 0.0;
  h.hi[0] = prm->eps_max;
  h.hi[1] = prm->sig_max;
  h.eta1[0] = prm->eta1_eps;
  h.eta1[1] = prm->eta1_sig;
  h.eta2[0] = prm->eta2_eps;
  h.eta2[1] = prm->eta2_sig;
  h.w = p->d.h * p->d.h * p->d.h;
  launch_copy_f32(c->c0, eps0_dev, c->n, st);
  launch_copy_f32(c->c0 + c->n, sig0_dev, c->n, st);
  launch_fill_f64(c->d, 2 * c->n, 0.0, st);
  if (int rc = check_launch(p)) {
    cga_free(c);
    return rc;
  }
  if (hipStreamSynchronize(st) != hipSuccess || hipMemcpy(c->st, &h, sizeof(CgaDev), hipMemcpyHostToDevice) != hipSuccess) {
    cga_free(c);
    return fail(p, DD_ERR_HIP, "CGA state upload failed");
  }
  *out = c;
  return DD_OK;
}

int dd_cga_steps_from_gradient(dd_cga* c, const double* g_eps_dev, const double* g_sigma_dev, double step_eps,
                               double step_sig, void* stream) {
  if (!c || !g_eps_dev || !g_sigma_dev || !(step_eps > 0.0) || !(step_sig > 0.0) || !std::isfinite(step_eps) ||
      !std::isfinite(step_sig))
    return DD_ERR_INVALID_ARG;
  launch_cga_steps(g_eps_dev, g_sigma_dev, c->mesh, step_eps, step_sig, c->st, c->part, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? DD_OK : DD_ERR_HIP;
}

int dd_cga_destroy(dd_cga* c) {
  if (!c) return DD_ERR_INVALID_ARG;
  cga_free(c);
  return DD_OK;
}

int dd_cga_update(dd_cga* c, const double* g_eps_dev, const double* g_sigma_dev, float* eps_dev, float* sigma_dev,
                  void* stream) {
  if (!c || !g_eps_dev || !g_sigma_dev || !eps_dev || !sigma_dev) return DD_ERR_INVALID_ARG;
  launch_cga_update(g_eps_dev, g_sigma_dev, eps_dev, sigma_dev, c->c0, c->c0 + c->n, c->d, c->d + c->n, c->mesh,
                    c->st, c->part, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? DD_OK : DD_ERR_HIP;
}

int dd_cga_get_info(dd_cga* c, dd_cga_info* out, void* stream) {
  if (!c || !out) return DD_ERR_INVALID_ARG;
  CgaDev h{};
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess ||
      hipMemcpy(&h, c->st, sizeof(CgaDev), hipMemcpyDeviceToHost) != hipSuccess)
    return DD_ERR_HIP;
  out->iterations = h.m;
  out->converged = h.converged;
  for (int f = 0; f < 2; ++f) {
    out->grad_norm[f] = std::sqrt(h.gn2[f]);
    out->step_norm[f] = std::sqrt(h.step2[f]);
    out->beta[f] = h.beta[f];
    out->alpha_used[f] = h.alpha_used[f];
    out->alpha_next[f] = h.alpha[f];
    out->gamma_used[f] = h.gamma_used[f];
    out->gamma_next[f] = h.gamma[f];
    out->change_norm[f] = std::sqrt(h.change2[f]);
  }
  return DD_OK;
}

int dd_profile_enable(dd_problem* p, int32_t stride) {
  if (!p || stride < 0) return DD_ERR_INVALID_ARG;
  p->prof_stride = stride;
  for (auto& u : p->ev_used) u = 0;
  for (auto& u : p->ev_seen) u = 0;
  return DD_OK;
}

int dd_profile_read(dd_problem* p, int32_t kind, double* total_ms, int64_t* launches, int32_t reset) {
  if (!p || kind < 0 || kind >= DD_PROF_KINDS) return DD_ERR_INVALID_ARG;
  double tot = 0.0;
  const size_t n = p->ev_used[kind];   // closed windows
  if (n) {
    if (hipEventSynchronize(p->ev[kind][2 * n - 1]) != hipSuccess) return fail(p, DD_ERR_HIP, "event synchronize failed");
    for (size_t i = 0; i < n; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p->ev[kind][2 * i], p->ev[kind][2 * i + 1]) != hipSuccess)
        return fail(p, DD_ERR_HIP, "hipEventElapsedTime failed");
      tot += ms;
    }
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = (int64_t)n * prof_window(kind);
  if (reset) {
    p->ev_used[kind] = 0;
    p->ev_seen[kind] = 0;
  }
  return DD_OK;
}

int dd_algorithmic_bytes(const dd_problem* p, int32_t kind, double* bytes_per_launch) {
  if (!p || !bytes_per_launch || kind < 0 || kind >= DD_PROF_KINDS) return DD_ERR_INVALID_ARG;
  const double n_fd = (double)(p->N - p->n_own);
  const double n_own = (double)p->n_own, n_l0 = (double)p->n_l0, n_det = (double)p->n_det;
  int64_t n_free_i = 1;
  for (int a = 0; a < 3; ++a) n_free_i *= std::max(p->d.fem_cells[a] - 3, 0);
  const double n_free = (double)n_free_i, n_l1 = n_own - n_free;
  // a saving forward also writes the FEM state (E, V) of the levels the adjoint reads back:
  // every level of the last segment and the segment-start checkpoints before it
  const int64_t nt = p->d.n_steps, K = p->d.ckpt_every, k_tail = last_segment_start(p);
  int64_t saved = 0;
  for (int64_t n = 0; n < nt; ++n)
    if (n + 1 >= k_tail || ((n + 1) % K == 0 && (n + 1) / K < p->n_ck)) ++saved;
  const double save_fem = 24.0 * n_own * (double)saved / (double)std::max<int64_t>(nt, 1);
  // FD (three-level form): E^n and E^{n-1} read, E^{n+1} written; traces (forward)
  // written or cotangent (adjoint) read; layer-0 values written
  const double fd = 36.0 * n_fd + 12.0 * n_det + 12.0 * n_l0;
  const double fd_adj = fd + (p->adj_obs ? 12.0 * n_det : 0.0);   // observations read as well
  // FEM: state read and written, coefficients (eps - 1, c1, c2), layer-0 values read,
  // layer-1 values dual-written into the FD grid
  const double fem = 48.0 * n_own + 12.0 * n_own + 12.0 * n_l0 + 12.0 * n_l1;
  // adjoint FEM, free nodes: forward window E^k, V^k, V^{k-1} read, FP64 gradients updated
  const double grad = 36.0 * n_free + 32.0 * n_free;
  double b = 0.0;
  switch (kind) {
    case DD_PROF_FD_FWD: b = fd; break;
    case DD_PROF_FD_ADJ: b = fd_adj; break;
    case DD_PROF_FEM_FWD: b = fem + save_fem; break;
    case DD_PROF_FEM_RECOMPUTE: b = 48.0 * n_own + 12.0 * n_own + 12.0 * n_l0; break;   // window to window
    case DD_PROF_FEM_ADJ: b = fem + grad; break;
    case DD_PROF_STEP_FWD: b = fd + fem + save_fem; break;
    case DD_PROF_STEP_ADJ: b = fd_adj + fem + grad; break;
    // two-step launches: far-tile nodes read levels n-1, n and write n+1, n+2 (48 B), near-tile
    // nodes take one step (36 B); traces / cotangents of both steps, layer-0 values of one
    case DD_PROF_PAIR_FWD:
    case DD_PROF_PAIR_ADJ: {
      const double fdp = 48.0 * (double)p->tb_far + 36.0 * (double)p->tb_near + 24.0 * n_det + 12.0 * n_l0 +
                         (kind == DD_PROF_PAIR_ADJ && p->adj_obs ? 24.0 * n_det : 0.0);
      b = fdp + fem + (kind == DD_PROF_PAIR_FWD ? save_fem : grad);
      break;
    }
    case DD_PROF_PAIR2_FWD:
    case DD_PROF_PAIR2_ADJ:
      b = 36.0 * (double)p->tb_near + 12.0 * n_l0 + fem + (kind == DD_PROF_PAIR2_FWD ? save_fem : grad);
      break;
  }
  *bytes_per_launch = b;
  return DD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Batch engine: several problems (jobs) advance together, one launch per iteration, each
// active job contributing its next time step (forward, adjoint, or FEM-only recompute).
// ---------------------------------------------------------------------------------------
namespace {

struct BatchJob {
  dd_problem* p = nullptr;
  std::vector<dd_source> src;
  std::vector<SrcPlan> plans;
  float* traces = nullptr;
  const float* obs = nullptr;
  double *g_eps = nullptr, *g_sig = nullptr;
  int id = 0;
  size_t bytes = 0;           // the problem's footprint counted against the batch's budget
  int phase = 0;              // 0 forward, 1 adjoint, 2 finished
  int s = 0;                  // current source
  int64_t n = 0;              // forward step
  int64_t seg = 0, k = 0;     // adjoint segment and step
  int64_t rseg = -1, rk = 0;  // segment whose FEM states are being recomputed, its next step
  bool started = false;       // prologue of the current source queued
  bool seg_started = false;   // current adjoint segment started (and the recompute of the one before it)
};

// Adjoint segment [k0, k1) of segment seg.
int64_t seg_k0(const dd_problem* p, int64_t seg) { return seg * (int64_t)p->d.ckpt_every; }
int64_t seg_k1(const dd_problem* p, int64_t seg) {
  return std::min(seg_k0(p, seg) + (int64_t)p->d.ckpt_every, (int64_t)p->d.n_steps);
}

// The job's adjoint segment can start: the last segment (stored by the forward), or one whose
// recompute has taken all its steps.
bool seg_ready(const BatchJob& j) {
  return j.seg == n_segments(j.p) - 1 || (j.rseg == j.seg && j.rk == seg_k1(j.p, j.seg));
}

// Queues the prologue work due before the job's next launch and writes the items the job
// contributes to it into `it` (returns how many: 0 when the job has no step left).  In the
// adjoint, a launch carries the adjoint step of segment seg and, as a second item, the next
// FEM recompute step of segment seg - 1 (into the other window), as the single-problem
// path overlaps them on two streams; a segment whose recompute is still short of its last
// step (after a shorter last segment) first takes recompute-only launches.
int job_items(BatchJob& j, hipStream_t st, BatchItem* it) {
  dd_problem* p = j.p;
  const int64_t nt = p->d.n_steps;
  const int nsrc = (int)j.src.size();
  if (j.phase == 0) {
    if (!j.started) {
      forward_prologue(p, j.s, true, false, st);   // batched jobs start from rest
      j.started = true;
    }
    it[0].fa = fd_base(p);
    it[0].ea = fem_base(p);
    fwd_step_args(p, j.src[j.s], j.plans[j.s], j.s, j.n, j.traces, true, it[0].fa, it[0].ea);
    it[0].kind = 0;
    if (++j.n == nt) {
      j.n = 0;
      j.started = false;
      if (++j.s == nsrc) {
        j.s = 0;
        j.phase = j.obs ? 1 : 2;
      }
    }
    return 1;
  }
  if (j.phase != 1) return 0;
  const int64_t nseg = n_segments(p);
  if (!j.started) {
    if (j.s == 0) {
      launch_fill_f64(p->g_eps, p->n_own, 0.0, st);
      launch_fill_f64(p->g_sig, p->n_own, 0.0, st);
    }
    zero_state(p, st);
    j.seg = nseg - 1;
    j.seg_started = false;
    j.rseg = -1;
    j.started = true;
  }
  int n = 0;
  auto recompute_item = [&]() {
    it[n].fa = fd_base(p);
    it[n].ea = fem_base(p);
    recompute_args(p, j.s, j.rk, seg_k0(p, j.rseg), segment_window(p, j.s, j.rseg), it[n].ea);
    it[n].kind = 2;
    ++j.rk;
    ++n;
  };
  if (!j.seg_started) {
    if (!seg_ready(j)) {
      recompute_item();          // the rest of this segment's recompute, alone
      return n;
    }
    j.k = seg_k1(p, j.seg);
    j.seg_started = true;
    if (j.seg >= 1) {
      // the recompute of the segment before starts now, into the window whose last readers
      // (the adjoint steps of segment seg + 1) are already queued
      j.rseg = j.seg - 1;
      j.rk = seg_k0(p, j.rseg);
      segment_prologue(p, j.s, j.rseg, st);
    }
  }
  const int64_t k0 = seg_k0(p, j.seg);
  it[n].fa = fd_base(p);
  it[n].ea = fem_base(p);
  adj_step_args(p, j.s, j.k, k0, segment_window(p, j.s, j.seg), j.traces, j.obs, it[n].fa, it[n].ea);
  it[n].kind = 1;
  ++n;
  if (j.rseg == j.seg - 1 && j.rseg >= 0 && j.rk < seg_k1(p, j.rseg)) recompute_item();
  if (--j.k == k0) {
    j.seg_started = false;
    if (--j.seg < 0) {
      j.started = false;
      if (++j.s == nsrc) j.phase = 2;
    }
  }
  return n;
}

// True when the job's next job_items call queues prologue work (a source's forward or
// adjoint start, or an adjoint segment start with the next segment's recompute prologue)
// ahead of its items.
bool job_needs_prologue(const BatchJob& j) {
  if (j.phase == 0) return !j.started;
  if (j.phase == 1) return !j.started || (!j.seg_started && seg_ready(j));
  return false;
}

}  // namespace

struct dd_batch {
  int max_slots = 0;
  int width = 0;                // items per launch: two per job (an adjoint step and a recompute step)
  std::vector<BatchJob> jobs;
  std::vector<int> done;
  int next_id = 1;
  BatchItem* host = nullptr;    // pinned [ring][width]
  BatchItem* dev = nullptr;     // device [ring][width]
  // Items go up on a copy stream of their own, so that an upload runs while the kernels before
  // it are still running instead of waiting its turn between them on the launch stream.
  hipStream_t copy = nullptr;
  std::vector<hipEvent_t> ev;       // per ring segment: its upload is done (host and launches wait)
  std::vector<hipEvent_t> ev_used;  // per ring segment: the launches that read it are done
  // The ring holds the items of `ring` launches in segments of `seg` launches; the items of
  // the launches of one segment are uploaded with one copy.
  static constexpr int seg = 16;
  int ring = 64, pos = 0;
  bool return_on_done = true;   // dd_batch_step returns after the launch in which a job finishes
  // a launch takes the oldest active job and then the following ones while their cells per
  // step together stay within this (0: every active job in every launch).  Measured with the
  // single-job launches by value (against one problem at a time; 16-problem mix of 1-11 M
  // cells per step / small-job serving burst): 2M 0.984 / 0.90, 6M 0.985 / 1.09, 9M 0.985 /
  // 1.12; the earlier rule that added jobs until the target was passed: 6M 0.944 / 1.12.
  // Jobs that fill the GPU alone run alone; small, launch-bound jobs share launches.
  int64_t fill_cells = 9000000;
  // FD tile variant of the launches: -1 by the launch's combined FD fields against the
  // last-level cache, 0 / 1 forced cached / streaming (DD_FD_NT at dd_batch_create)
  int nt_mode = -1;
  size_t hbm_budget = 0;        // 0: no limit
  size_t in_use = 0;            // footprint of the problems with an active job
  std::string err;
};

extern "C" {

int dd_batch_create(int32_t max_slots, size_t hbm_budget, dd_batch** out) {
  if (!out || max_slots < 1 || 2 * max_slots > BATCH_MAX) return DD_ERR_INVALID_ARG;
  *out = nullptr;
  dd_batch* b = new (std::nothrow) dd_batch();
  if (!b) return DD_ERR_OOM;
  b->max_slots = max_slots;
  b->hbm_budget = hbm_budget;
  b->width = 2 * max_slots;
  if (const char* e = std::getenv("DD_FD_NT")) b->nt_mode = std::atoi(e) != 0 ? 1 : 0;
  const size_t bytes = sizeof(BatchItem) * (size_t)b->ring * b->width;
  if (hipHostMalloc((void**)&b->host, bytes, hipHostMallocDefault) != hipSuccess) {
    delete b;
    return DD_ERR_OOM;
  }
  if (hipMalloc((void**)&b->dev, bytes) != hipSuccess) {
    (void)hipHostFree(b->host);
    delete b;
    return DD_ERR_OOM;
  }
  b->ev.resize(b->ring / b->seg, nullptr);
  b->ev_used.resize(b->ring / b->seg, nullptr);
  for (auto* v : {&b->ev, &b->ev_used})
    for (auto& e : *v)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        dd_batch_destroy(b);
        return DD_ERR_HIP;
      }
  if (hipStreamCreateWithFlags(&b->copy, hipStreamNonBlocking) != hipSuccess) {
    b->copy = nullptr;
    dd_batch_destroy(b);
    return DD_ERR_HIP;
  }
  *out = b;
  return DD_OK;
}

int dd_batch_destroy(dd_batch* b) {
  if (!b) return DD_ERR_INVALID_ARG;
  (void)hipDeviceSynchronize();
  for (auto* v : {&b->ev, &b->ev_used})
    for (auto e : *v)
      if (e) (void)hipEventDestroy(e);
  if (b->copy) (void)hipStreamDestroy(b->copy);
  if (b->dev) (void)hipFree(b->dev);
  if (b->host) (void)hipHostFree(b->host);
  delete b;
  return DD_OK;
}

int dd_batch_submit(dd_batch* b, dd_problem* p, const dd_source* src, int32_t n_src, float* traces_dev,
                    const float* obs_dev, double* g_eps_dev, double* g_sigma_dev, int32_t* job_out) {
  if (!b || !p) return DD_ERR_INVALID_ARG;
  if (!src || n_src < 1 || !traces_dev) return fail(p, DD_ERR_INVALID_ARG, "need sources and a trace buffer");
  if ((g_eps_dev || g_sigma_dev) && !obs_dev) return fail(p, DD_ERR_INVALID_ARG, "a gradient needs observations");
  if ((int)b->jobs.size() >= b->max_slots) return fail(p, DD_ERR_STATE, "no free batch slot");
  for (const auto& j : b->jobs)
    if (j.p == p) return fail(p, DD_ERR_STATE, "problem already has an active batch job");
  if (!p->use_stencil || !p->fused)
    return fail(p, DD_ERR_UNSUPPORTED, "batched steps need the assembled-stencil FEM path");
  if (p->r2) return fail(p, DD_ERR_UNSUPPORTED, "batched steps run the div-div form R1 only");
  if (p->init_on) return fail(p, DD_ERR_UNSUPPORTED, "batched jobs start from rest (the problem has initial data)");
  for (int s = 0; s < n_src; ++s) {
    const std::string e = check_source(p, src[s]);
    if (!e.empty()) return fail(p, DD_ERR_INVALID_ARG, e);
  }
  const size_t bytes = dd_footprint_bytes(&p->d, n_src);
  if (b->hbm_budget && b->in_use + bytes > b->hbm_budget)
    return fail(p, DD_ERR_STATE, "the job does not fit the batch's HBM budget (" + std::to_string(bytes) + " bytes, " +
                                     std::to_string(b->hbm_budget - std::min(b->in_use, b->hbm_budget)) + " free)");
  int rc = ensure_saved_storage(p, n_src);
  if (rc) return rc;
  BatchJob j;
  j.bytes = bytes;
  j.p = p;
  j.src.assign(src, src + n_src);
  for (int s = 0; s < n_src; ++s) j.plans.push_back(source_plan(p, src[s]));
  j.traces = traces_dev;
  j.obs = obs_dev;
  p->adj_obs = obs_dev != nullptr;
  p->have_pg = false;
  j.g_eps = g_eps_dev;
  j.g_sig = g_sigma_dev;
  j.id = b->next_id++;
  p->saved = false;
  p->have_grad = false;
  p->have_pg = false;
  p->ic_used = false;
  b->jobs.push_back(j);
  b->in_use += bytes;
  if (job_out) *job_out = j.id;
  return DD_OK;
}

namespace {
// Number of jobs (a prefix of b->jobs, oldest first) that take part in the next launch.
size_t launch_jobs(const dd_batch* b) {
  if (b->fill_cells <= 0) return b->jobs.size();
  int64_t cells = 0;
  size_t n = 0;
  for (const auto& j : b->jobs) {
    const int64_t c = j.phase != 2 ? j.p->N + j.p->n_own : 0;
    if (n > 0 && cells + c > b->fill_cells) break;
    cells += c;
    ++n;
  }
  return n;
}
}  // namespace

int dd_batch_set_fill(dd_batch* b, int64_t cells) {
  if (!b || cells < 0) return DD_ERR_INVALID_ARG;
  b->fill_cells = cells;
  return DD_OK;
}

int dd_batch_step(dd_batch* b, int32_t max_steps, void* stream) {
  if (!b || max_steps < 0) return DD_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const size_t done0 = b->done.size();
  int iter = 0;
  while (iter < max_steps && !b->jobs.empty()) {
    // Fill one ring segment with the items of up to `seg` launches, upload them with one
    // copy and launch them.  The segment ends early before a job's prologue work (which
    // must follow the launches before it in stream order) and after a launch in which a
    // job takes its last step.
    const int g = b->pos / b->seg;
    if (hipEventSynchronize(b->ev[g]) != hipSuccess) {
      b->err = "event synchronize failed";
      return DD_ERR_HIP;
    }
    BatchBases bases[dd_batch::seg];
    size_t lds[dd_batch::seg];
    bool nt[dd_batch::seg], obl[dd_batch::seg];
    int m = 0;
    bool finished = false;
    while (m < b->seg && iter < max_steps && !b->jobs.empty()) {
      const size_t nj = launch_jobs(b);
      if (m > 0 && std::any_of(b->jobs.begin(), b->jobs.begin() + nj, job_needs_prologue)) break;
      BatchItem* h = b->host + (size_t)(b->pos + m) * b->width;
      int n = 0, base = 0;
      size_t l = 0;
      double fd_bytes = 0.0;   // the FD field sets this launch streams through
      const dd_problem* owner[BATCH_MAX];
      for (size_t q = 0; q < nj; ++q) {
        BatchJob& j = b->jobs[q];
        const int c = job_items(j, st, h + n);
        for (int i = 0; i < c; ++i) {
          if (h[n].kind != 2) fd_bytes += fd_field_bytes(j.p);
          owner[n++] = j.p;
        }
      }
      // the launch's variant (and with it the z-chunk) follows the FD fields it streams;
      // each item's tile grid is laid out for that chunk
      const bool use_nt = b->nt_mode < 0 ? fd_bytes > LLC_BYTES : b->nt_mode != 0;
      bool use_obl = false;
      for (int i = 0; i < n; ++i) use_obl |= h[i].fa.pw_kind != 0;
      for (int i = 0; i < n; ++i) {
        BatchItem& it = h[i];
        const dd_problem* q = owner[i];
        it.fem_blocks = (q->n_part + N_XCD - 1) / N_XCD * N_XCD;
        it.fd_blocks = 0;
        if (it.kind != 2) {
          fd_tile_grid(q->nx, q->ny, q->nz, use_nt, it.fa.nbx, it.fa.nby, it.fa.nbz, it.fa.ntiles, it.fa.per_xcd);
          it.fd_blocks = it.fa.per_xcd * N_XCD;
        }
        l = std::max(l, stencil_lds(it.ea));
        bases[m].base[i] = base;   // each item's FEM partitions, then its FD tiles
        base += it.fem_blocks + it.fd_blocks;
      }
      bases[m].n = n;
      bases[m].base[n] = base;
      lds[m] = l;
      nt[m] = use_nt;
      obl[m] = use_obl;
      ++m;
      ++iter;
      if (std::any_of(b->jobs.begin(), b->jobs.end(), [](const BatchJob& j) { return j.phase == 2; })) {
        finished = true;
        break;
      }
    }
    if (m) {
      const size_t off = (size_t)b->pos * b->width;
      // a launch of a single forward or adjoint step, or of one job's adjoint step with its
      // recompute step, passes its arguments by value; only the others read the uploaded items
      auto by_value = [&](int k) {
        const BatchItem& one = b->host[off + (size_t)k * b->width];
        const BatchItem& two = b->host[off + (size_t)k * b->width + 1];
        return (bases[k].n == 1 && one.kind != 2) || (bases[k].n == 2 && one.kind == 1 && two.kind == 2 && !obl[k]);
      };
      bool upload = false;
      for (int k = 0; k < m; ++k) upload = upload || (bases[k].n && !by_value(k));
      // the copy overwrites the device segment once the launches that read it last are done,
      // and the launches below read it once the copy is done
      if (upload && (hipStreamWaitEvent(b->copy, b->ev_used[g], 0) != hipSuccess ||
                     hipMemcpyAsync(b->dev + off, b->host + off, sizeof(BatchItem) * b->width * m,
                                    hipMemcpyHostToDevice, b->copy) != hipSuccess ||
                     hipEventRecord(b->ev[g], b->copy) != hipSuccess ||
                     hipStreamWaitEvent(st, b->ev[g], 0) != hipSuccess)) {
        b->err = "batch upload failed";
        return DD_ERR_HIP;
      }
      for (int k = 0; k < m; ++k) {
        if (!bases[k].n) continue;
        const BatchItem& one = b->host[off + (size_t)k * b->width];
        const BatchItem& two = b->host[off + (size_t)k * b->width + 1];
        if (bases[k].n == 1 && one.kind != 2)
          // a single forward or adjoint step: the fused step kernel, arguments by value (the
          // same device code on the same arguments, without the item lookup)
          launch_step(one.fa, one.ea, st, one.kind == 1, false, nt[k], nullptr);
        else if (bases[k].n == 2 && one.kind == 1 && two.kind == 2 && !obl[k])
          // one job's adjoint step and its recompute step: likewise by value
          launch_step_rec(one.fa, one.ea, two.ea, st, nt[k]);
        else
          launch_batch(b->dev + off + (size_t)k * b->width, bases[k], lds[k], st, nt[k], obl[k]);
      }
      if (upload && hipEventRecord(b->ev_used[g], st) != hipSuccess) {
        b->err = "batch event record failed";
        return DD_ERR_HIP;
      }
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) {
        b->err = std::string("batch launch failed: ") + hipGetErrorString(e);
        return DD_ERR_HIP;
      }
    }
    b->pos = ((g + 1) * b->seg) % b->ring;
    if (finished) {
      for (auto it = b->jobs.begin(); it != b->jobs.end();) {
        if (it->phase == 2) {
          dd_problem* p = it->p;
          p->saved = true;
          p->saved_n_src = (int)it->src.size();
          if (it->obs) {
            p->have_grad = true;
            if (it->g_eps && it->g_sig) {
              launch_fill_f64(it->g_eps, p->n_fem, 0.0, st);
              launch_fill_f64(it->g_sig, p->n_fem, 0.0, st);
              launch_gradient_out(p->g_eps, p->g_sig, p->own_api, p->own_grid, p->n_own, it->g_eps, it->g_sig, st);
            }
          }
          b->done.push_back(it->id);
          b->in_use -= std::min(b->in_use, it->bytes);
          it = b->jobs.erase(it);
        } else {
          ++it;
        }
      }
      // a job finished: return so that the caller can collect it (and admit new work)
      // without waiting for the rest of the requested steps
      if (b->return_on_done && b->done.size() > done0) break;
    }
  }
  return DD_OK;
}

int dd_batch_poll(dd_batch* b, int32_t* done_jobs, int32_t capacity, int32_t* n_done, int32_t* n_active) {
  if (!b) return DD_ERR_INVALID_ARG;
  const int n = std::min<int>((int)b->done.size(), done_jobs ? capacity : 0);
  for (int i = 0; i < n; ++i) done_jobs[i] = b->done[i];
  b->done.erase(b->done.begin(), b->done.begin() + n);
  if (n_done) *n_done = n;
  if (n_active) *n_active = (int)b->jobs.size();
  return DD_OK;
}

}  // extern "C"
