/*
 * dd.h -- C-ABI of the hybrid FE/FD time-domain Maxwell solver (MI355X / gfx950).
 *
 * The solver advances the stabilised Maxwell system of the paper's box
 * "Forward problem" (eq. forward_prob; model problem eq. model1 with the
 * plane-wave source eq. f):
 *     eps E_tt + sigma E_t - Laplace E - grad div((eps - 1) E) = 0,
 * explicitly in time on a structured outer grid (7-point finite differences)
 * coupled, through a two-node overlap, to lumped-mass P1 finite elements on
 * the Kuhn tetrahedra of an inner box (section "The mathematical model",
 * domain decomposition paragraph; eq. epsilon_sigma_constraint).  It then runs
 * the adjoint problem of the box "Adjoint problem" (eq. adjoint_prob) backward
 * in time and forms the eps / sigma gradient of eq. gradeps as time integrals
 * of forward x adjoint products, exactly on the discrete scheme.
 *
 * Conventions
 *   - Outer-grid node (i,j,k) is at origin + h*(i,j,k); grid arrays are
 *     lexicographic, x fastest.
 *   - FEM box = outer hex cells [fem_lo, fem_lo + fem_cells); its nodes have
 *     local indices l in [0, fem_cells] per axis, and "FEM-node arrays" (eps,
 *     sigma, gradients) are lexicographic over them, x fastest.  A node's layer
 *     is min over axes of min(l, fem_cells - l): layer 0 belongs to the
 *     finite-difference region, layer 1 is FEM-owned, layers >= 2 are free.
 *   - Detectors: outer-grid nodes on the faces selected by detector_faces, in
 *     lexicographic grid order.  Trace arrays are [n_src][n_steps][n_det][3]
 *     float32; row n holds E at time level n+1.
 *   - Face bits: DD_FACE_TOP (z max; the paper's backscatter boundary d_1),
 *     DD_FACE_BOTTOM (z min; d_2), DD_FACE_XMIN/XMAX/YMIN/YMAX (the sides d_3).
 *
 * Memory and streams
 *   - Every pointer argument named *_dev is device memory owned by the caller
 *     and must stay valid until the work queued on `stream` has finished.
 *   - The library owns its internal state (fields, checkpoints, interface
 *     history, FP64 accumulators).  It allocates that device memory through the
 *     allocator given to dd_create (e.g. a framework's caching allocator), or with
 *     hipMalloc when none is given, in dd_create, dd_forward / dd_batch_submit (the
 *     saved forward) and on the first use of an optional form; dd_destroy releases it.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All device work is
 *     queued asynchronously on it; calls return once the work is queued, except
 *     dd_set_coefficients, which synchronises the stream to report violations.
 *   - A dd_problem is not thread-safe; use it from one host thread and one
 *     stream at a time.
 *
 * Errors: every call returns DD_OK (0) or a negative DD_ERR_* code; no C++
 * exception crosses the ABI.  dd_error_string(code) gives a static text and
 * dd_last_error(problem) the message of the problem's last failure.
 */
#ifndef DD_H
#define DD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DD_OK = 0,
  DD_ERR_INVALID_ARG = -1,  /* bad descriptor, null pointer, size mismatch */
  DD_ERR_CONSTRAINT = -2,   /* eps / sigma violate eq. epsilon_sigma_constraint */
  DD_ERR_UNSTABLE = -3,     /* non-finite field values after a solve (dd_check_finite) */
  DD_ERR_OOM = -4,          /* device allocation failed */
  DD_ERR_HIP = -5,          /* a HIP runtime call or kernel launch failed */
  DD_ERR_STATE = -6,        /* call out of order (e.g. adjoint without a saved forward) */
  DD_ERR_UNSUPPORTED = -7   /* valid request this build does not handle */
};

enum {
  DD_FACE_TOP = 1, DD_FACE_BOTTOM = 2, DD_FACE_XMIN = 4,
  DD_FACE_XMAX = 8, DD_FACE_YMIN = 16, DD_FACE_YMAX = 32
};

enum {
  DD_SRC_SINE1 = 1,       /* P(t) = amp sin(omega t) on (0, 2 pi / omega), eq. f */
  DD_SRC_GAUSS_SINE = 2,  /* P(t) = amp sin(omega (t - t0)) exp(-((t - t0)/width)^2 / 2) on [0, 2 t0] */
  DD_SRC_DIPOLE = 3       /* Gaussian-sine time function, point force pol * P(t) at grid node pos */
};

typedef struct dd_problem dd_problem;

/* Checkpoint schemes of the forward saved for the adjoint (dd_problem_desc.ckpt_mode). */
enum {
  DD_CKPT_FEM_IFACE = 0,  /* FEM state (E, V) every ckpt_every steps plus the layer-0 interface
                             values of every step; the adjoint recomputes the FEM region of a
                             segment from its checkpoint (the FD region needs no recompute) */
  DD_CKPT_STORE_ALL = 1,  /* every FEM level kept (ckpt_every is taken as n_steps) */
  DD_CKPT_FULL = 2        /* full-state checkpoints: not built (DD_ERR_UNSUPPORTED) */
};

typedef struct {
  int32_t n_outer[3];       /* outer grid nodes per axis, each >= 4; product < 2^30 */
  double h;                 /* grid spacing > 0 */
  double origin[3];         /* coordinates of grid node (0,0,0) */
  int32_t fem_lo[3];        /* grid index of the FEM box's lower corner; >= 1 */
  int32_t fem_cells[3];     /* FEM hex cells per axis; >= 2, fem_lo + fem_cells <= n_outer - 2 */
  int32_t overlap;          /* node layers shared by the FD and FEM regions (section "The
                               mathematical model", domain decomposition): 2 (0 = 2); any other
                               value DD_ERR_UNSUPPORTED */
  double dt;                /* time step > 0, fixed (never derived from eps) */
  int32_t n_steps;          /* N_t >= 1 */
  int32_t ckpt_every;       /* forward checkpoint interval K >= 1 for the adjoint */
  double s_stab;            /* weight s of the div-div stabiliser s grad div(eps E) of the target
                               system: 1 (0 = 1), the only value for which the FD region carries the
                               plain wave equation of the paper; other values DD_ERR_UNSUPPORTED */
  uint32_t detector_faces;  /* face bits of the detector set (non-empty) */
  uint32_t absorbing_faces; /* face bits with first-order absorbing BC (eq. model1) */
  double t_switch;          /* top face: plane-wave source for t_n <= t_switch, absorbing
                               (if DD_FACE_TOP is in absorbing_faces) for t_n > t_switch */
  int32_t ckpt_mode;        /* DD_CKPT_* (0 = DD_CKPT_FEM_IFACE) */
} dd_problem_desc;

typedef struct {
  int32_t kind;             /* DD_SRC_* */
  double omega, t0, width, amp;
  double dir[3];            /* plane waves: direction of travel k (normalised by the library);
                               all zero = normal incidence (k = -e_z, the model problem of
                               eq. model1).  Otherwise k_z < 0 is required: the wave enters
                               through the top face, reaching top-face node i at the delay
                               tau_i = k . (x_i - x_ref) (x_ref: the top-face node it reaches
                               first), where the forcing is P(t - tau_i) instead of P(t); the
                               source stays on while t_n <= t_switch, which should cover
                               max tau_i plus the pulse.  Ignored for DD_SRC_DIPOLE. */
  double pol[3];            /* polarisation / dipole moment direction */
  int32_t pos[3];           /* DD_SRC_DIPOLE: grid node; must be finite-difference owned */
} dd_source;

/* Device allocator of a problem's state: alloc returns `bytes` of device memory (NULL on
 * failure, reported as DD_ERR_OOM), free releases a pointer alloc returned; ctx is passed
 * through.  Calls happen on the thread that calls into the library. */
typedef void* (*dd_alloc_fn)(size_t bytes, void* ctx);
typedef void (*dd_free_fn)(void* ptr, void* ctx);

/* Build the mesh, partitions, element colouring and device state of one problem
 * (paper: domain decomposition of section "The mathematical model"; Kuhn split of
 * the FEM box).  eps = 1, sigma = 0 until dd_set_coefficients is called.
 * alloc_fn, free_fn, ctx: the allocator of every device buffer the problem owns (its
 * fields, saved forward, recompute windows, optional buffers and a dd_cga run started on
 * it); both NULL: hipMalloc / hipFree; only one NULL: DD_ERR_INVALID_ARG.  They must stay
 * usable until dd_destroy (and the last dd_cga_destroy of a run on the problem).
 * out: receives the handle (owned by the caller, release with dd_destroy).
 * Errors: DD_ERR_INVALID_ARG (descriptor), DD_ERR_UNSUPPORTED (overlap, s_stab, ckpt_mode),
 * DD_ERR_OOM, DD_ERR_HIP. */
int dd_create(const dd_problem_desc* desc, dd_alloc_fn alloc_fn, dd_free_fn free_fn, void* ctx, dd_problem** out);
/* dd_create on a general tetrahedral mesh of the FEM box (the locally refined meshes of
 * eq. meshref: the FEM region of section "Numerical results" on a mesh refined where the
 * reconstructed |eps| is large).  The FEM nodes are the box's (fem_cells + 1)^3 lattice nodes,
 * lexicographic (x fastest), followed by n_extra nodes at extra_xyz (host, [n_extra][3] physical
 * coordinates, each strictly inside the box); tets (host, [n_tets][4]) lists the tetrahedra by
 * FEM-node index.  The tetrahedra must fill the box (volume sum within 1e-9), none degenerate,
 * every node of lattice layer >= 1 and every extra node on at least one of them.  The lattice
 * nodes of layers 0 and 1 keep their roles (finite-difference data; the dual-written layer) and
 * the extra nodes are free.  FEM-node arrays (coefficients, gradients) then hold n_fem_nodes =
 * (fem_cells + 1)^3 + n_extra entries.  The FEM rows run on the element-coloured kernel with
 * the div-div form R1 (and a dd_cga run weighs each free node by its lumped mass); the form R2,
 * the paper-formula gradient, initial data and batched jobs report DD_ERR_UNSUPPORTED for such
 * a problem.  The arrays are read during the
 * call only.  The explicit step is stable for dt up to 2 / sqrt(lambda_max(M_eps^-1 A)),
 * which a refined mesh lowers: the caller chooses dt accordingly.
 * Errors: DD_ERR_INVALID_ARG (descriptor, or a mesh that breaks the rules above),
 * DD_ERR_UNSUPPORTED (as dd_create, or a mesh too dense for the kernel's partitions of
 * at most 512 owned / 1024 local nodes, 4608 elements and 64 element colours: lattice blocks
 * of 8^3 owned nodes are cut at their median until they fit, so only a node with more than
 * 64 elements around it, or a single node over the limits, is refused), DD_ERR_OOM, DD_ERR_HIP. */
int dd_create_mesh(const dd_problem_desc* desc, int64_t n_extra, const double* extra_xyz, int64_t n_tets,
                   const int32_t* tets, dd_alloc_fn alloc_fn, dd_free_fn free_fn, void* ctx, dd_problem** out);

/* ---- Local mesh refinement (box "ACGA", steps 2 and 3; eq. meshref, eq. meshfunction) ----
 * Host only; no device work.  dd_meshref_create marks the elements of a mesh of the FEM box and
 * refines them.  The mesh: n_tets = 0 (tets and extra_xyz NULL, n_extra = 0) for the uniform
 * Kuhn split (per cell, lexicographic with x fastest, its six tetrahedra from the lowest corner
 * one axis step at a time along x y z, x z y, y x z, y z x, z x y, z y x), or extra nodes and
 * tetrahedra as dd_create_mesh takes them (host arrays, read during the call only).
 * eps, sigma: host float32 values at the mesh's FEM nodes (lattice nodes, then extra nodes).
 * Marking: with h_K the diameter (longest edge) of element K, K is marked when at one of its
 * vertices v both h_K |eps(v)| >= beta_eps M_eps and h_K |sigma(v)| >= beta_sig M_sig hold
 * (M: the largest such product over all elements and their vertices; beta in [0, 1]).
 * Refining: longest-edge bisection with propagation.  A marked element is bisected at its
 * longest edge (ties within 1e-9 relative: the edge with the smaller (low, high) pair of node
 * ids), together with every element around that edge, at the edge's midpoint, after every
 * element around the edge whose own longest edge is another one has been bisected the same
 * way (recursively, in increasing element id; an element split at (a, b), a < b, becomes
 * its half with b replaced by the midpoint and then its half with a replaced by it, with ids
 * after all existing ones).  So every element is split at its longest edge and the mesh stays
 * conforming.  An edge is bisected only when every element around it has all its vertices
 * FEM-owned (lattice layer >= 1): the elements touching layer 0 are never split, and a marked
 * element whose propagation reaches such an edge stays as it is.  Marked elements are taken in
 * element order, skipping those already split; the k-th bisection's midpoint becomes FEM node
 * n_old + k.  On the Kuhn split this inserts the centre of every cell one of whose corners meets
 * the rule (and whose corners are all FEM-owned) and bisects its six tetrahedra across its
 * main diagonal.
 * out: a host handle (release with dd_meshref_destroy).
 * Errors: DD_ERR_INVALID_ARG (null arguments, beta outside [0, 1], an index out of range, an
 * extra node outside the box's interior, a descriptor with fewer than 2 FEM cells per axis). */
typedef struct dd_refinement dd_refinement;
int dd_meshref_create(const dd_problem_desc* desc, int64_t n_extra, const double* extra_xyz, int64_t n_tets,
                      const int32_t* tets, const float* eps, const float* sigma, double beta_eps, double beta_sig,
                      dd_refinement** out);
/* Sizes of the result: marked input elements, bisected edges (= new nodes), extra nodes of the
 * refined mesh (the input's extra nodes, then the midpoints) and its elements.  Any pointer may
 * be NULL. */
int dd_meshref_sizes(const dd_refinement* r, int64_t* n_marked, int64_t* n_bisected, int64_t* n_extra,
                     int64_t* n_tets);
/* Copies the result into host arrays: marks [input elements] (1 = marked; may be NULL),
 * extra_xyz [n_extra][3] (physical coordinates; may be NULL when n_extra = 0), tets
 * [n_tets][4] (FEM-node ids; elements in the order of the input's, each replaced in place by
 * its pieces), ready for dd_create_mesh. */
int dd_meshref_result(const dd_refinement* r, uint8_t* marks, double* extra_xyz, int32_t* tets);
/* A nodal function of the input mesh (host, n_old entries) on the refined mesh's nodes (host,
 * n_old + n_bisected entries): old nodes keep their values, each midpoint in bisection order
 * takes the mean of its edge's endpoints (the refined mesh carries the same piecewise-linear
 * function); computed in FP64 and rounded once. */
int dd_meshref_interpolate(const dd_refinement* r, const float* in, float* out);
int dd_meshref_destroy(dd_refinement* r);
/* Releases the problem.  With hipMalloc memory the device is synchronised first; with a
 * caller allocator only the library's own second stream is, and each buffer goes back
 * through free_fn while the caller's stream may still hold queued work that reads it: the
 * allocator must order reuse after that work (a stream-ordered caching allocator on the
 * stream of the calls does). */
int dd_destroy(dd_problem* p);

/* Sizes: FEM nodes (lattice, plus a general mesh's extra nodes), detectors, outer grid
 * nodes (any pointer may be NULL). */
int dd_sizes(const dd_problem* p, int64_t* n_fem_nodes, int64_t* n_detectors, int64_t* n_grid);

/* Host-only: grid indices of the detector nodes in trace order (n_detectors entries). */
int dd_detector_nodes(const dd_problem_desc* desc, int64_t* out, int64_t capacity, int64_t* n_written);

/* Upper bound of the device bytes a problem of this descriptor allocates through its
 * allocator: dd_create, a saving dd_forward (or dd_batch_submit) with n_src sources and every
 * optional buffer (initial data, the div-div form R2 / paper-formula gradient, the misfit's
 * weights and partials, a dd_cga run), for admission control.  0 for an invalid descriptor. */
size_t dd_footprint_bytes(const dd_problem_desc* desc, int32_t n_src);

/* eps, sigma: FEM-node arrays (float32, n_fem_nodes each) on the device.
 * Enforces eq. epsilon_sigma_constraint: eps = 1, sigma = 0 on layers 0 and 1,
 * eps >= 1 and sigma >= 0 everywhere, all finite; else DD_ERR_CONSTRAINT and the
 * previous coefficients stay.  Synchronises `stream`. */
int dd_set_coefficients(dd_problem* p, const float* eps_dev, const float* sigma_dev, void* stream);

/* dd_set_coefficients without the wait: the check of eq. epsilon_sigma_constraint runs on the
 * device, and the coefficients are applied only if it passes (else the previous ones stay);
 * nothing is read back, so the call only queues work on `stream`.  dd_coefficients_status
 * (synchronises `stream`) gives DD_ERR_CONSTRAINT if the last dd_set_coefficients_async was
 * refused, else DD_OK.  For callers whose coefficients are valid by construction (e.g. the
 * iterate of dd_cga_update, kept in the coefficient box) and who must not wait. */
int dd_set_coefficients_async(dd_problem* p, const float* eps_dev, const float* sigma_dev, void* stream);
int dd_coefficients_status(dd_problem* p, void* stream);

/* Forward solve of each source from rest (E = E_t = 0 at t = 0), or from the initial data
 * set by dd_set_initial_data.
 * traces_dev: [n_src][n_steps][n_det][3] float32 output.
 * save: nonzero keeps what dd_adjoint needs (FEM checkpoints every ckpt_every steps
 *       and the per-step layer-0 interface values), per source.
 * energy_dev: NULL or [n_src][n_steps] float64 output of the discrete energy
 *       W^{n+1/2} = |V^{n+1}|^2_{M_eps} / (2 dt^2) + E^{n+1} . A E^n / 2. */
int dd_forward(dd_problem* p, const dd_source* src, int32_t n_src, float* traces_dev,
               int32_t save, double* energy_dev, void* stream);

/* Scans the current field state (both FD levels, the FEM levels and increment: after
 * dd_forward the last forward state, after dd_adjoint the adjoint's) for non-finite values:
 * DD_ERR_UNSTABLE when there are any, else DD_OK.  Synchronises `stream`.  The solve calls
 * do not check by themselves (they stay asynchronous): with a time step within the CFL
 * bound and coefficients that pass dd_set_coefficients the scheme is stable, so non-finite
 * fields come from non-finite inputs that are not checked (cotangents, observations). */
int dd_check_finite(dd_problem* p, void* stream);

/* General initial data of the forward problem (eq. forward_initial_cond): E(x, 0) = f_0,
 * dE/dt(x, 0) = f_1.  f0_dev, f1_dev: [n_grid][3] float32 on the device, node index
 * x + Nx (y + Ny z), checked (any non-finite value: DD_ERR_CONSTRAINT, and the data set
 * before stay) and copied into library-owned buffers; synchronises `stream`, so the caller's
 * arrays may be freed when the call returns.  The scheme starts from the levels
 * E^0 = f_0 and E^{-1} = f_0 - dt f_1 (the one-sided difference of dE/dt at t = 0), for every
 * source of the following dd_forward calls.  The gradient of the
 * following adjoints is the exact derivative with both levels held fixed: its level-0 rows
 * hold the -lambda(x, 0) f_1 term of eq. gradeps (as -m_i lambda^0 . dt f_1 / dt^2) and the
 * level-0 div-div term, for either div-div form and for dd_gradient_paper.
 * Both NULL: start from rest again.  One NULL: DD_ERR_INVALID_ARG.  Setting or clearing the
 * data discards a saved forward.  The first call allocates up to 24 n_grid + 20 n_fem_nodes
 * bytes (not counted by dd_footprint_bytes) and synchronises the device; DD_ERR_UNSUPPORTED
 * when FD and FEM run on two streams.
 * Batched jobs (dd_batch_submit) always start from rest and are refused (DD_ERR_UNSUPPORTED)
 * while initial data is set. */
int dd_set_initial_data(dd_problem* p, const float* f0_dev, const float* f1_dev, void* stream);

/* Adjoint solve (eq. adjoint_prob, exact transpose of the discrete forward scheme)
 * for each source of the last saved dd_forward, with the trace cotangent
 * cot_dev = dJ/dtraces ([n_src][n_steps][n_det][3] float32; E - E_obs for the
 * loss J = 1/2 sum |E - E_obs|^2).  Recomputes the FEM forward state segment by
 * segment from the checkpoints and accumulates the eps / sigma gradient of
 * eq. gradeps in FP64, summed over sources.  DD_ERR_STATE without a saved forward. */
int dd_adjoint(dd_problem* p, const float* cot_dev, void* stream);

/* Tikhonov term of eq. tikhonov_functional, gamma_eps/2 |eps - eps0|^2 + gamma_sig/2 |sigma - sigma0|^2
 * in L2 of the FEM box with the lumped-mass quadrature (|u|^2 = sum_i m_i u_i^2 over the free
 * nodes, m_i = h^3), at the coefficients of the last dd_set_coefficients. */
typedef struct {
  double gamma_eps, gamma_sig;    /* >= 0, finite */
  const float* eps0_dev;          /* Tikhonov centres: FEM-node arrays (float32, n_fem_nodes) */
  const float* sigma0_dev;
} dd_tikhonov;

/* Gradient of the last dd_adjoint: g_eps_dev, g_sigma_dev are FEM-node arrays
 * (float64, n_fem_nodes each), dJ/deps_i and dJ/dsigma_i on the free nodes, zero on nodes of
 * layer 0 and 1.  reg (nullable): adds the derivative of the Tikhonov term,
 * gamma m_i (c_i - c0_i), on the free nodes.  DD_ERR_STATE without a preceding adjoint,
 * DD_ERR_INVALID_ARG for null buffers or a reg with negative / non-finite gammas or null centres. */
int dd_gradient(dd_problem* p, double* g_eps_dev, double* g_sigma_dev, const dd_tikhonov* reg, void* stream);

/* dd_adjoint for the trace misfit of eq. tikhonov_functional, J = 1/2 sum |E - E_obs|^2:
 * the cotangent traces - obs is formed inside the adjoint kernels as they read it (no
 * cotangent array is written).  traces_dev: the traces of the last saved dd_forward;
 * obs_dev: observations, same layout ([n_src][n_steps][n_det][3] float32).  Same
 * requirements and results as dd_adjoint. */
int dd_adjoint_misfit(dd_problem* p, const float* traces_dev, const float* obs_dev, void* stream);

/* Trace misfit of eq. tikhonov_functional with its smoothing function z, on the device:
 * traces_dev, obs_dev: [n_src][n_steps][n_det][3] float32; z_host: NULL (z = 1) or n_steps
 * float64 weights >= 0 on the host, entry n for trace row n (time level n + 1).
 *   cot_dev (nullable): z_n (traces - obs), float32, same layout (may be traces_dev itself);
 *     dd_adjoint(p, cot_dev) then gives the gradient of the weighted misfit;
 *   j_dev (nullable): J = 1/2 sum_n z_n sum |traces - obs|^2, one float64 (a deterministic
 *     FP64 sum).
 * Queued on `stream`; z_host is read before the call returns (weights that differ from the
 * last call's are uploaded, synchronising `stream`).  Calls on different streams must not
 * overlap. */
int dd_misfit(dd_problem* p, const float* traces_dev, const float* obs_dev, int32_t n_src, const double* z_host,
              float* cot_dev, double* j_dev, void* stream);

/* Host-only: a smoothing function z of eq. tikhonov_functional as time weights for dd_misfit
 * (the paper names it without a formula): z_out[n] (trace row n, time level n + 1,
 * t = (n + 1) dt) is 1 up to T - delta and (1 + cos(pi s)) / 2 with s = (t - (T - delta)) / delta
 * over the last delta, so the misfit fades out smoothly to 0 at the end time T = n_steps dt;
 * delta <= 0 gives z = 1.  z_out: n_steps doubles (caller-owned host memory).
 * DD_ERR_INVALID_ARG for n_steps < 1, a null z_out, dt <= 0 or non-finite dt, delta. */
int dd_misfit_taper(int32_t n_steps, double dt, double delta, double* z_out);

/* dd_misfit without any device allocation, for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * results and error behaviour as dd_misfit (the same kernels: results are bit-identical).
 * Its scratch (the FP64 block partials of J and the time weights) is a static device array of
 * 8 * (1024 + DD_MISFIT_NOALLOC_MAX_STEPS) bytes (about 520 KB), one copy per GPU, held until
 * the process ends; n_steps above DD_MISFIT_NOALLOC_MAX_STEPS gives DD_ERR_INVALID_ARG.  All
 * calls on one GPU share that array: calls that overlap on one GPU (different streams, or host
 * threads) race.  With z_host the weights are uploaded on every call, which synchronises
 * `stream`; with z_host = NULL the call only queues kernels. */
enum { DD_MISFIT_NOALLOC_MAX_STEPS = 65536 };
int dd_misfit_noalloc(dd_problem* p, const float* traces_dev, const float* obs_dev, int32_t n_src, const double* z_host,
                      float* cot_dev, double* j_dev, void* stream);

/* Solves as HIP graphs.  A step of a small grid takes a few microseconds, a good part of it the
 * dispatch of its launch; replaying a call's launches as one graph (hipGraphLaunch on the
 * caller's stream) cuts that part.  The forward (dd_forward) and the adjoint (dd_adjoint,
 * dd_adjoint_misfit; only for problems whose adjoint has one checkpoint segment, i.e.
 * ckpt_every >= n_steps or DD_CKPT_STORE_ALL) each keep one graph.  DD_GRAPH_ON: every such call replays its graph,
 * captured on the first call and again whenever the call's arguments (forward: sources,
 * trace / energy buffers, save flag; adjoint: cotangent / observation buffers, saved source
 * count) or the problem's options (div-div form, initial data, paper-formula variant) differ
 * from the captured ones; a capture takes about as long as queuing the launches one by one.
 * The graphs read the coefficients, initial data and saved-forward buffers the problem owns,
 * so they follow dd_set_coefficients.  DD_GRAPH_AUTO (default): as ON on grids of at most
 * 2^19 nodes, from the second call in a row with the same arguments; the first of them runs
 * launch by launch.  DD_GRAPH_OFF: launch by launch.  Results are bitwise those of the
 * launch-by-launch calls.  Not while kernel timing (dd_profile_enable) is on, nor with the
 * two-stream step order.  A re-capture waits for the previous replay of that graph to
 * finish, and dd_destroy for the last replays of the problem's graphs.  The environment variable DD_GRAPH (0, 1, 2) sets the mode of problems created
 * after it. */
enum { DD_GRAPH_OFF = 0, DD_GRAPH_ON = 1, DD_GRAPH_AUTO = 2 };
int dd_set_graph(dd_problem* p, int32_t mode);
/* Graphs captured and calls replayed as a graph so far, for which = DD_GRAPH_FORWARD or
 * DD_GRAPH_ADJOINT (either pointer may be NULL). */
enum { DD_GRAPH_FORWARD = 0, DD_GRAPH_ADJOINT = 1 };
int dd_graph_stats(const dd_problem* p, int32_t which, int64_t* captures, int64_t* replays);

/* Div-div form of the FEM rows.  DD_DIVDIV_R1 (default): the nodal product (eps - 1) E inside
 * the element divergence, as eq. forward_prob writes it.  DD_DIVDIV_R2: the element mean of
 * eps - 1 outside it, sum_K |K| (mean_K eps - 1) grad phi_i div_K(E) (symmetric); for this form
 * the paper's gradient formula (eq. gradeps with grad(eps~).E dropped) is the exact gradient,
 * and dd_gradient returns it.  R2 needs the assembled-stencil path (uniform Kuhn box;
 * DD_ERR_UNSUPPORTED otherwise); its steps are fused launches of their own, the adjoint
 * ones carrying the div-div gradient terms; batched jobs run R1 only and report
 * DD_ERR_UNSUPPORTED for an R2 problem.  Switching the form discards a saved forward.
 * The first switch to R2 allocates FEM-node sized buffers and synchronises the device. */
enum { DD_DIVDIV_R1 = 1, DD_DIVDIV_R2 = 2 };
int dd_set_divdiv_form(dd_problem* p, int32_t form);

/* Paper-formula gradient variant.  eq. gradeps writes the div-div part of g_eps as the
 * time integral of div(lambda) div(E), having replaced div(eps~ E) by eps~ div(E); on the
 * discrete scheme that term is sum_k sum_{K containing i} (|K|/4) div_K(lambda^k) div_K(E^k)
 * in place of the exact sum_k sum_K |K| div_K(lambda^k) (grad phi_i . E^k_i).  (It is the
 * exact derivative of a scheme whose div-div term carries the element mean of eps - 1
 * outside the divergence, not of this one.)
 * dd_paper_gradient_enable(p, 1): the following dd_adjoint / dd_adjoint_misfit calls also
 * accumulate the difference of the two terms (inside the fused adjoint step launches, a
 * launch of its own after each step otherwise; FEM-node sized buffers allocated on the
 * first call, which synchronises the device);
 * 0 switches it off.  DD_ERR_UNSUPPORTED when FD and FEM run on two streams.  Batched jobs
 * never accumulate it.
 * dd_gradient_paper: after such an adjoint, the variant's g_eps and the (unchanged) g_sigma,
 * same layout as dd_gradient; DD_ERR_STATE if the last adjoint did not accumulate it. */
int dd_paper_gradient_enable(dd_problem* p, int32_t on);
int dd_gradient_paper(dd_problem* p, double* g_eps_dev, double* g_sigma_dev, void* stream);

/* ---- Conjugate gradient reconstruction (box "CGA") -----------------------------------
 * One CGA iteration m is: dd_set_coefficients(eps^m, sigma^m), dd_forward(save),
 * dd_adjoint_misfit, dd_gradient (step 1), then dd_cga_update (steps 2-6), which turns
 * the gradient of J into the gradient functions of eq. gradeps,
 *     g_i = (dJ/dc_i) / m_i + gamma^m (c_i - c^0_i)   on free nodes (layer >= 2),
 * with m_i the lumped mass of node i and c^0 the initial guess (the Tikhonov centre of
 * eq. tikhonov_functional), and updates the coefficients in place:
 *     beta^m = |g^m|^2 / |g^{m-1}|^2 (0 at m = 0 or when |g^{m-1}| = 0),
 *     d^m = -g^m + beta^m d^{m-1},
 *     c^{m+1} = c^m + alpha^m d^m, kept in the box 1 <= eps <= eps_max, 0 <= sigma <= sig_max
 *               of eq. epsilon_sigma_constraint,
 *     alpha^{m+1} = -(g^m, d^m) / (gamma^m (d^m, d^m)) (alpha^m kept when d^m = 0),
 *     gamma^{m+1} = gamma^0 / (m + 1)^p,
 * where (u, v) = sum over free nodes of m_i u_i v_i (lumped-mass L2 inner product: m_i = h^3
 * on the Kuhn split; on a mesh of dd_create_mesh each node's own mass, and its extra nodes are
 * free) and |u| = (u, u)^{1/2}; eps and sigma are updated independently with their own scalars.
 * The stop test of step 6 holds when (|eps^{m+1} - eps^m| < eta1_eps or
 * |sigma^{m+1} - sigma^m| < eta1_sig) and (|g_eps^m| < eta2_eps or |g_sig^m| < eta2_sig).
 * All of it runs on the device, with deterministic FP64 sums. */
typedef struct dd_cga dd_cga;
typedef struct {
  double gamma_eps, gamma_sig;   /* gamma^0 > 0 */
  double p;                      /* exponent of the gamma rule, 0 < p < 1 */
  double alpha_eps, alpha_sig;   /* alpha^0 >= 0 */
  double eps_max, sig_max;       /* coefficient box: eps_max > 1, sig_max > 0 */
  double eta1_eps, eta1_sig, eta2_eps, eta2_sig;   /* tolerances of the stop test, >= 0 */
} dd_cga_params;
typedef struct {
  int32_t iterations;            /* updates done (m after the last update) */
  int32_t converged;             /* the stop test held at the last update */
  /* of the last update, [0] = eps, [1] = sigma: */
  double grad_norm[2];           /* |g^m| */
  double step_norm[2];           /* |c^{m+1} - c^m| */
  double beta[2];                /* beta^m */
  double alpha_used[2];          /* alpha^m */
  double alpha_next[2];          /* alpha^{m+1} */
  double gamma_used[2];          /* gamma^m */
  double gamma_next[2];          /* gamma^{m+1} */
  double change_norm[2];         /* |c^{m+1} - c^0|: distance from the initial guess */
} dd_cga_info;

/* Start a run on problem p from the initial guess eps0_dev, sig0_dev (FEM-node arrays,
 * float32, copied: they are the Tikhonov centres).  The initial guess must satisfy the
 * coefficient constraint and the box (else DD_ERR_CONSTRAINT); parameters out of range
 * give DD_ERR_INVALID_ARG.  Synchronises `stream`.  The run keeps only the lattice sizes
 * of p (and, on a mesh of dd_create_mesh, its own copy of the lumped masses) and may outlive
 * it; release it with dd_cga_destroy. */
int dd_cga_create(dd_problem* p, const dd_cga_params* prm, const float* eps0_dev, const float* sig0_dev, void* stream,
                  dd_cga** out);
int dd_cga_destroy(dd_cga* c);
/* Step sizes of a run from the gradient of J at the initial guess, on the device (no host
 * read): with G = max over the free nodes of |dJ/dc_i| / m_i (at least 1e-30), per field,
 * gamma^0 = gamma^m = G / step and alpha^m = step / G, so that the first update moves eps by at
 * most step_eps and sigma by at most step_sig.  Call before the first dd_cga_update; replaces
 * those values of the parameters given to dd_cga_create.  Asynchronous. */
int dd_cga_steps_from_gradient(dd_cga* c, const double* g_eps_dev, const double* g_sigma_dev, double step_eps,
                               double step_sig, void* stream);
/* Steps 2-6: g_eps_dev, g_sigma_dev are dd_gradient's output at (eps^m, sigma^m);
 * eps_dev, sigma_dev hold eps^m, sigma^m on entry and eps^{m+1}, sigma^{m+1} when the
 * queued work is done (nodes of layers 0 and 1 are not written).  Asynchronous. */
int dd_cga_update(dd_cga* c, const double* g_eps_dev, const double* g_sigma_dev, float* eps_dev, float* sigma_dev,
                  void* stream);
/* Scalars of the last update (synchronises `stream`). */
int dd_cga_get_info(dd_cga* c, dd_cga_info* out, void* stream);

const char* dd_error_string(int code);
const char* dd_last_error(const dd_problem* p);

/* ---- Batched solves (several problems in one launch per step) ----------------------
 * A batch holds up to max_slots (1..32) jobs.  A job is the solve of one problem: the forward of
 * each source with saving, then -- when obs_dev is given -- the adjoint for the misfit
 * cotangent traces - obs (read inside the adjoint kernel; obs_dev has the traces' layout)
 * and the gradient summed over sources, written to g_eps_dev / g_sigma_dev (FEM-node
 * arrays, float64) when those are given.  dd_batch_step issues up to max_steps kernel
 * launches.  A launch takes the oldest active job and then the following ones while their
 * cells per step (outer nodes + FEM-owned nodes) together stay within the batch's fill target
 * (dd_batch_set_fill),
 * and each job it takes contributes its next step (a forward step, or an adjoint step
 * together with the next checkpoint recompute step of the segment before it, which uses
 * the other window).  So jobs of uneven grid sizes, step counts and source counts share
 * the GPU while they are small, a job that fills the GPU alone runs alone, and new jobs
 * can join while others run.  dd_batch_step returns early, after the launch in which a job completed, so
 * that a caller can collect results and admit new jobs without waiting for the remaining
 * steps it asked for.  A finished job's results are complete once `stream` reaches the work
 * queued by the dd_batch_step call that reported it through dd_batch_poll; afterwards the
 * problem behaves as after dd_forward(save) + dd_adjoint.
 * Requirements: the problem uses the assembled-stencil FEM path (uniform Kuhn box) and the
 * fused step (else DD_ERR_UNSUPPORTED); it has no other active job and is not used
 * outside the batch until its job is done; all buffers stay valid until then.  A batch is
 * driven from one host thread and one stream.  Storage for the saved forward is allocated
 * in dd_batch_submit (see dd_footprint_bytes); dd_batch_step allocates nothing. */
typedef struct dd_batch dd_batch;
/* hbm_budget: bytes (0 = no limit) that the problems with an active job may hold together,
 * each counted at dd_footprint_bytes(its descriptor, its job's sources); dd_batch_submit of a
 * job that does not fit gives DD_ERR_STATE and changes nothing (like a full batch), and a
 * job's bytes are returned when it completes. */
int dd_batch_create(int32_t max_slots, size_t hbm_budget, dd_batch** out);
/* Fill target of a launch in cells per step (default 9,000,000); 0 lets every active job
 * take part in every launch.  Negative: DD_ERR_INVALID_ARG. */
int dd_batch_set_fill(dd_batch* b, int64_t cells);
int dd_batch_destroy(dd_batch* b);
int dd_batch_submit(dd_batch* b, dd_problem* p, const dd_source* src, int32_t n_src, float* traces_dev,
                    const float* obs_dev, double* g_eps_dev, double* g_sigma_dev, int32_t* job_out);
int dd_batch_step(dd_batch* b, int32_t max_steps, void* stream);
/* Ids of jobs finished since the last poll (up to capacity), and the number still active. */
int dd_batch_poll(dd_batch* b, int32_t* done_jobs, int32_t capacity, int32_t* n_done, int32_t* n_active);

/* Kernel timing.  dd_profile_enable(p, stride): with stride k > 0, HIP events on the
 * stream of the launch bracket, every k launches of each kind below, a window of
 * consecutive launches (8 for the fused step kinds, which run back to back; 1 otherwise;
 * up to 16384 windows per kind).  A window's elapsed time covers its kernels and the
 * dispatch gaps between them; 0 switches timing off.  dd_profile_read synchronises on the
 * last event of `kind` and returns the summed time and the number of timed launches;
 * reset != 0 clears that kind.  dd_algorithmic_bytes
 * gives the minimum HBM bytes one launch of `kind` must move (each field value read or
 * written once); for the forward kinds it is the average over the launches of a forward
 * that saves its state for dd_adjoint (store-every-level: each launch writes the FEM
 * state once more). */
enum {
  DD_PROF_FD_FWD = 0, DD_PROF_FEM_FWD = 1, DD_PROF_FD_ADJ = 2, DD_PROF_FEM_ADJ = 3,
  DD_PROF_FEM_RECOMPUTE = 4,
  DD_PROF_STEP_FWD = 5, DD_PROF_STEP_ADJ = 6,  /* fused FD + FEM step launches */
  /* two-step launches (temporal blocking of the FD region, switched on by the environment
   * variable DD_TB=1 at dd_create; forwards without energy and adjoints of the form R1 without
   * the paper-formula variant or initial data take them): the first launch of a pair (FD
   * tiles away from the FEM box two steps, the rest one) and the second (near tiles and FEM) */
  DD_PROF_PAIR_FWD = 7, DD_PROF_PAIR_ADJ = 8, DD_PROF_PAIR2_FWD = 9, DD_PROF_PAIR2_ADJ = 10,
  DD_PROF_KINDS = 11
};
int dd_profile_enable(dd_problem* p, int32_t stride);
int dd_profile_read(dd_problem* p, int32_t kind, double* total_ms, int64_t* launches, int32_t reset);
int dd_algorithmic_bytes(const dd_problem* p, int32_t kind, double* bytes_per_launch);

/* Diagnostic (host only, no GPU): applies the FEM rows of the operator -- forward
 * (K + A_dd) E, or with flags bit 0 set the transpose K E + (eps - 1) q(E) -- in FP64 by
 * walking exactly the data a FEM kernel reads, checking every index bound: with flags
 * bit 1 clear the element kernel's partition / halo / colour / geometry data (and that no
 * colour touches an owned node twice), with bit 1 set the assembled-stencil kernel's
 * partition boxes and stencil table (DD_ERR_UNSUPPORTED if the mesh has no shared stencil).
 * eps: FEM-node array; E, out: [n_fem_nodes][3] (out is written on FEM-owned nodes,
 * zero elsewhere).  stats (nullable, 8 entries): partitions, max colours, max local
 * nodes, geometry entries, element evaluations, owned nodes, layer-0 nodes, stencil slots.
 * Returns DD_ERR_UNSUPPORTED if any check fails. */
int dd_debug_fem_apply(const dd_problem_desc* desc, const double* eps, const double* E, int32_t flags,
                       double* out, int64_t* stats);
/* dd_debug_fem_apply on the element data that dd_create_mesh builds from a general mesh (same
 * arguments as there; flags bit 1 must be clear: a general mesh has no assembled stencil).
 * eps, E, out: over the n_fem_nodes = (fem_cells + 1)^3 + n_extra FEM nodes. */
int dd_debug_fem_apply_mesh(const dd_problem_desc* desc, int64_t n_extra, const double* extra_xyz, int64_t n_tets,
                            const int32_t* tets, const double* eps, const double* E, int32_t flags, double* out,
                            int64_t* stats);

#ifdef __cplusplus
}
#endif

#endif /* DD_H */
