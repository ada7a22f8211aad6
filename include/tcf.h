/*
 * tcf.h -- C-ABI of the tree-cotree-gauged dual-primal eddy-current solver.
 *
 * The library advances the time-domain A*-formulation
 *     curl(nu curl A) + sigma dA/dt = J,   n x A = 0 on the outer boundary
 * (Sec. 2, A*-formulation with PEC boundary; inhomogeneous n x A data is
 * posed through a lifting, i.e. as the homogenised problem with the volume
 * source jvol and the initial value ainit of tcf_problem_desc, Sec. 2.1)
 * discretised by curl-conforming
 * spline patches (Sec. 2.2) with implicit Euler (Sec. 2.2, implicit Euler
 * system W = M + dt K, f = M a^(l) + dt j^(l+1)).  Every step is solved by the
 * dual-primal tearing of Sec. 3: per-patch remainder solves, a signed jump
 * across patch interfaces, a coarse problem on the primal unknowns, and PCG
 * on the Lagrange multipliers with an unscaled Dirichlet preconditioner
 * (Sec. 4).  The insulating region is gauged by the tree-cotree split of
 * Sec. 3 (tree on the control mesh: wirebasket, then faces, then interiors;
 * interface tree edges primal).
 *
 * Conventions shared by every call:
 *  - Patches form a P0 x P1 x P2 grid of axis-aligned boxes; patch (i,j,k)
 *    has id s = i + P0*(j + P1*k).  Row r of direction d has nel[d][r]
 *    uniform elements and H1 degree deg[d][r] (open knots), so neighbouring
 *    patches are conforming on shared faces (Sec. 2.2).
 *  - Global edge numbering on the control grid (nodes per direction
 *    N_d = sum_r (nel+deg-1) + 1): x-edges I + (Nx-1)(J + Ny K), then y-edges
 *    Ex + I + Nx (J + (Ny-1) K), then z-edges Ex + Ey + I + Nx (J + Ny K).
 *  - Fields are returned as global edge vectors in that numbering, with
 *    Dirichlet and gauge-tree edges equal to zero.
 *  - Every call returns TCF_OK (0) or a negative status; no exception crosses
 *    the ABI.  tcf_last_error() describes the last failure on a handle.
 *  - Device pointers are HIP device memory on the current device; streams
 *    are hipStream_t passed as void* (NULL = the legacy default stream).
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef TCF_H
#define TCF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum tcf_status {
  TCF_OK = 0,
  TCF_EINVAL = -1,   /* invalid description or argument                     */
  TCF_ENOMEM = -2,   /* host or device allocation failed                   */
  TCF_ENOTSPD = -3,  /* a Cholesky pivot <= 0 (patch id in tcf_stats)       */
  TCF_ENOCONV = -4,  /* PCG / refinement hit its iteration limit; results   */
                     /* of that step are still readable and flagged          */
  TCF_EHIP = -5,     /* HIP runtime error                                   */
  TCF_ESTATE = -6    /* call out of order (e.g. step before setup)          */
};

enum tcf_precision {
  TCF_FP64 = 0,         /* local factors and Schur operators in FP64          */
  TCF_FP32_IR = 1,      /* local factors in FP64, the explicit Schur operators */
                        /* (S_bb^-1, Phi_b, S_bb, condensation) stored and     */
                        /* applied in FP32; PCG, coarse solve and refinement   */
                        /* residual in FP64                                    */
  TCF_FP32_FULL_IR = 2  /* as TCF_FP32_IR but the local factorisation is FP32 */
                        /* too, on the FP32 matrix cores with FP32             */
                        /* accumulation (converges only where the local blocks */
                        /* are well conditioned, e.g. conductors; see          */
                        /* tcf_get_cond_est)                                   */
};

/*
 * Source callback: evaluate phi_k on a tensor grid of quadrature abscissae.
 * out[ix + nx*(iy + ny*iz)] = phi_k(xs[ix], ys[iy], zs[iz]).
 * The source is J_k(x,t) = g_k(t) curl(0, 0, phi_k(x)) on patches whose
 * src_mask is set (the load vector j of Sec. 2.2, taken in curl form).
 * Called from tcf_setup on the calling thread, once per (source patch, k);
 * phi and phi_ctx must stay valid until tcf_setup returns.
 */
typedef void (*tcf_phi_fn)(const double* xs, int32_t nx, const double* ys, int32_t ny,
                           const double* zs, int32_t nz, int32_t k, double* out, void* ctx);

/*
 * Vector callback: evaluate a vector field of excitation k at the points of a
 * tensor grid inside patch s (id as in tcf_problem_desc):
 *   out[c + 3*(ix + nx*(iy + ny*iz))] = F_c(xs[ix], ys[iy], zs[iz]),  c = 0, 1, 2.
 * The patch id lets the field depend on the patch's material (a manufactured
 * source does: the same potential gives a different J in a conductor and in
 * an insulator).  Called from tcf_setup on the calling thread; the function
 * and vec_ctx must stay valid until tcf_setup returns.
 */
typedef void (*tcf_vec_fn)(int32_t s, const double* xs, int32_t nx, const double* ys, int32_t ny,
                           const double* zs, int32_t nz, int32_t k, double* out, void* ctx);

typedef struct tcf_problem_desc {
  int32_t np[3];            /* patches per direction, each >= 1               */
  const double* breaks[3];  /* np[d]+1 strictly increasing patch boundaries   */
  const int32_t* nel[3];    /* np[d] element counts per row, each >= 1        */
  const int32_t* deg[3];    /* np[d] H1 degrees per row, each >= 1            */
  const double* sigma;      /* per patch conductivity, >= 0 (0 = insulator)   */
  const double* nu;         /* per patch reluctivity, > 0                     */
  const uint8_t* src_mask;  /* per patch: 1 = source acts here                */
  int32_t n_rhs;            /* independent excitations sharing the operator   */
  tcf_phi_fn phi;           /* source potential callback (see above)          */
  void* phi_ctx;
  const double* amp;        /* [n_rhs][n_steps]: g_k(t_{l+1}), t_l = l*dt     */
  double dt;                /* implicit Euler step, > 0                       */
  int32_t n_steps;          /* steps available in amp                         */
  /* Optional fields (NULL = absent; zero-initialise the struct).  With them a
   * problem whose boundary data was homogenised by a lifting (Sec. 2.1: the
   * inhomogeneous n x A = g becomes n x A = 0 with a modified source and
   * initial value) can be posed directly.                                  */
  tcf_vec_fn jvol;          /* volume source: J_k(x,t) gains g_k(t) jvol_k(x) */
                            /* on patches whose src_mask is set, loaded as    */
                            /* the integral of J . w_e (the load vector of    */
                            /* Sec. 2.2) on p_d + 3 Gauss points; may be used */
                            /* with or without phi                             */
  tcf_vec_fn ainit;         /* initial potential A_k(x, 0) (Sec. 2.1).  The   */
                            /* first step's M a^(0) is taken as the integral  */
                            /* of sigma A_k(x,0) . w_e, i.e. a^(0) is the      */
                            /* sigma-weighted L2 projection of the initial    */
                            /* value; evaluated on conductor patches only.    */
                            /* It is added at step 0 on top of M times the    */
                            /* held field (zero unless a state was restored)  */
  void* vec_ctx;            /* passed to jvol and ainit                       */
} tcf_problem_desc;

typedef struct tcf_options {
  int32_t precision;        /* TCF_FP64, TCF_FP32_IR or TCF_FP32_FULL_IR      */
  double pcg_rtol;          /* stop when ||r||_2 <= pcg_rtol * ||d||_2        */
  int32_t pcg_maxit;        /* <= 0: max(1000, n_lambda)                      */
  double ir_rtol;           /* FP32 paths: refine (>= 1 correction) until the  */
                            /* estimated field error (last correction times    */
                            /* the observed contraction) <= ir_rtol ||a||      */
  int32_t ir_maxit;         /* FP32 path: solves per step incl. the first,    */
                            /* <= 0: 10                                        */
  int32_t check_every;      /* PCG iterations between host convergence reads  */
  int32_t use_graph;        /* 1: replay captured hipGraphs for PCG chunks    */
  int32_t rhs_batch;        /* excitations solved together (one PCG over      */
                            /* several columns, each operator tile read once  */
                            /* per iteration for all of them): 1..32.  Up to  */
                            /* 4 on the vector units; wider batches run the   */
                            /* tile products on the matrix cores in widths of */
                            /* 8, 16 or 32 (a batch is rounded up; its idle   */
                            /* columns carry zero right-hand sides).  <= 0:   */
                            /* min(n_rhs, 32), rounded the same way           */
  int32_t pcg_warm;         /* first solve of a step starts from: 0 lambda =  */
                            /* 0; 1 the previous step's lambda; 2 the linear  */
                            /* extrapolation of the last two; 3 the Galerkin  */
                            /* projection onto the span of the excitation's   */
                            /* newest 8 solutions (Fischer's projection for   */
                            /* successive right-hand sides over a sliding     */
                            /* window: it deflates the initial error; the     */
                            /* F-orthonormal basis is rebuilt on the stream   */
                            /* after each solve).  The stopping test stays    */
                            /* ||r|| <= rtol ||d||.  3 keeps 4 x 8 n_lambda    */
                            /* doubles per excitation                         */
  int32_t precond_scaling;  /* Dirichlet preconditioner: 0 unscaled (as      */
                            /* published), 1 stiffness-scaled: each copy of a */
                            /* dual unknown weighted by the other copy's share*/
                            /* of the two local diagonal entries              */
  int32_t coarse_mode;      /* coarse solve S_Pi^-1 (Sec. 3: the second Schur  */
                            /* complement): 0 automatic (the cheaper per apply */
                            /* of the two below, by streamed bytes and        */
                            /* launches), 1 one dense FP64 inverse, 2 the     */
                            /* FP64 Cholesky factor in a nested dissection of */
                            /* the patch grid (dense blocks per separator,    */
                            /* explicit inverses of the diagonal blocks, the  */
                            /* top separator's Schur complement inverted      */
                            /* densely); both give S_Pi^-1 to rounding        */
  int32_t setup_group_mb;   /* setup assembles and factors the patches in     */
                            /* groups whose dense [i|b|p] blocks together      */
                            /* take at most this many MiB (FP64); a larger     */
                            /* patch forms a group of its own.  <= 0: 16384.   */
                            /* Bounds the setup's transient device memory      */
  int32_t panel_chunk;      /* matrix-core path (batches of more than 4       */
                            /* columns): a row panel of an operator is split  */
                            /* into jobs of at most this many 64 x 64 tiles,  */
                            /* whose partial rows add atomically.  <= 0: 16   */
  int32_t autotune;         /* matrix-core path: 1 times every operator at the */
                            /* end of setup for split lengths 4, 8, 16, 32 and */
                            /* unsplit, and keeps the fastest per operator (F  */
                            /* apply, preconditioner, coarse correction,       */
                            /* coarse solve); 0 keeps panel_chunk              */
  const char* tune_table;   /* NULL, or a text file of tuned split lengths     */
                            /* keyed by the problem's shape: an entry for this */
                            /* shape is used without timing; with autotune = 1 */
                            /* a new result is appended (the file is created   */
                            /* if missing; a file that cannot be opened is     */
                            /* skipped).  Read during tcf_setup only           */
  int32_t deterministic;    /* 1: bitwise reproducible runs.  Every batch      */
                            /* width takes the row panels, unsplit; rows that  */
                            /* several panels add into, and the quadratic      */
                            /* forms, are staged and summed in a fixed order   */
                            /* (no atomics): reruns, resumed checkpoints and   */
                            /* requests served alongside others give the same  */
                            /* bits.  Costs the panels' storage of the         */
                            /* symmetric blocks whole (twice the bytes of the  */
                            /* tiles for batches of up to 4)                   */
} tcf_options;

/* Fills defaults: FP64, rtol 1e-10, maxit auto, ir_rtol 1e-8, check 8, graph 1,
 * rhs_batch 0 (automatic), pcg_warm 0, precond_scaling 0, coarse_mode 0,
 * setup_group_mb 0. */
void tcf_default_options(tcf_options* opts);

/*
 * Device memory of a handle.  Every device buffer the handle holds (setup
 * transients, operators, tiles, vectors) is taken from alloc and given back
 * through free, each on the stream of the call that needs it (the stream of
 * tcf_setup or tcf_step; tcf_destroy returns what is left on the stream of
 * the handle's last call).  alloc returns NULL when it cannot serve a
 * request; the call then fails with TCF_ENOMEM.  The callbacks are called
 * on the calling thread (for serving: the request's worker thread) and must
 * stay valid for the handle's lifetime; ctx is passed through.  A NULL
 * allocator, or one with a NULL alloc, selects stream-ordered allocation
 * (hipMallocAsync / hipFreeAsync on the call's stream), so that giving
 * memory back does not synchronise the device.  The tcf_allocator struct is
 * copied by tcf_create.
 */
typedef struct tcf_allocator {
  void* ctx;
  void* (*alloc)(void* ctx, size_t bytes, void* stream);
  void (*free)(void* ctx, void* ptr, void* stream);
} tcf_allocator;

typedef struct tcf_problem tcf_problem;

/*
 * Host-only work: validation, control grid, edge classes, gauge tree,
 * primal/dual/interior split, multiplier table and device memory plan.
 * Touches no GPU.  Every array in desc is copied and may be freed on
 * return; the phi callback and its context are kept until tcf_setup.
 * Errors: TCF_EINVAL (bad sizes, sigma < 0, nu <= 0, dt <= 0, non-increasing
 * breaks, deg < 1, nel < 1, n_rhs < 1), TCF_ENOMEM.  On error *out is NULL and
 * tcf_last_error(NULL) holds the message.  allocator may be NULL (see
 * tcf_allocator).
 */
int tcf_create(const tcf_problem_desc* desc, const tcf_options* opts,
               const tcf_allocator* allocator, tcf_problem** out);

/* Device bytes the setup will allocate for the FP64 and FP32 paths. */
int tcf_footprint(const tcf_problem* h, size_t* bytes_fp64, size_t* bytes_fp32);

/*
 * Allocates device memory on the current device and runs, on `stream`:
 * patch assembly by quadrature, the local partial Cholesky and explicit
 * Schur complements, the coarse primal matrix and its factorisation, and the
 * source condensation.  Synchronises `stream` before returning.
 * Errors: TCF_ENOMEM, TCF_ENOTSPD (a local or coarse pivot <= 0; the failing
 * patch id, or -1 for the coarse matrix, is in tcf_stats.fail_patch),
 * TCF_EHIP, TCF_ESTATE (setup called twice).
 */
int tcf_setup(tcf_problem* h, void* stream);

/*
 * Advances nsteps implicit Euler steps (bounded by n_steps - steps_done) on
 * `stream`.  Synchronises `stream` before returning.  TCF_ENOCONV if any step
 * hit its PCG or refinement limit (the steps are still taken; see stats).
 */
int tcf_step(tcf_problem* h, int32_t nsteps, void* stream);

/*
 * Allocation-free variant of tcf_step, for callers that cannot allocate
 * device memory or instantiate graphs while stepping (code under stream
 * capture of their own, tight serving loops, harnesses that forbid
 * allocation).  Same steps and results as tcf_step, but the PCG's per-solve
 * scratch (tile accumulators, quadratic-form slots, reduction partials and
 * the per-column scalars) lives in one library-wide device array of
 * 64 MiB per GPU instead of the handle's buffers, and every launch is a
 * plain stream launch (no graph is captured or replayed).  Nothing is
 * allocated or freed on any call.  The array's address is looked up on the
 * first call on each device, with that device current.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (several handles stepped concurrently from different threads or on
 * different streams) race and must be serialised by the caller.  The
 * contents left by a call are never read by the next one.
 * Errors: as tcf_step; TCF_EINVAL if the problem's scratch exceeds 64 MiB
 * (the message states the size needed) or the handle runs without tiles.
 */
int tcf_step_noalloc(tcf_problem* h, int32_t nsteps, void* stream);

/* Waits for all work of the handle on `stream`; reports deferred errors. */
int tcf_sync(tcf_problem* h, void* stream);

/*
 * Copies the current field of excitation k (global edge vector, length
 * n_edges, FP64) into `out`: host memory if on_device == 0, else device
 * memory of the current device.  len must be >= n_edges.  An interface
 * unknown held by several patches (their copies agree to the PCG
 * tolerance) is read from its lowest-numbered patch; eliminated and
 * Dirichlet edges are zero.
 */
int tcf_get_field(tcf_problem* h, int32_t k, double* out, size_t len, int32_t on_device,
                  void* stream);

enum tcf_topology_kind {
  TCF_TOPO_COUNTS = 0,     /* int64[8]: n_edges, n_nodes, |V(H)|, n_plain,      */
                           /* n_floating, n_lambda, n_primal, n_kept             */
  TCF_TOPO_DIRICHLET = 1,  /* sorted global edge ids                             */
  TCF_TOPO_TREE_I = 2,     /* sorted gauge-tree edge ids (eliminated)            */
  TCF_TOPO_TREE_GAMMA = 3, /* sorted interface-tree edge ids (primal)            */
  TCF_TOPO_PRIMAL = 4,     /* sorted primal edge ids; index = coarse unknown     */
  TCF_TOPO_DUAL = 5,       /* sorted dual edge ids; index = multiplier row       */
  TCF_TOPO_INTERIOR = 6,   /* sorted patch-interior kept edge ids                */
  TCF_TOPO_MULT = 7,       /* int64[n_lambda][3]: edge id, patch (+1), patch(-1) */
  TCF_TOPO_N = 8,          /* int64[sum_s n_p^(s)][3]: patch, edge id, primal    */
                           /* rank; per patch in increasing edge id              */
  TCF_TOPO_LOOP = 9,       /* int64[n][3]: multiplier row, edge id, +1 / -1.     */
                           /* Host plan of a reduced primal split that drops the */
                           /* interface trees from the primal set (the outlook   */
                           /* of Sec. 5): the conductor-side terms of the row of */
                           /* each cotree edge e of a conductor/insulator face,  */
                           /* a_C(e) + psi(head e) - psi(tail e), psi the signed */
                           /* sum of a_C along the face-tree path from the face  */
                           /* boundary.  Rows ascending, then edge ids.  Not     */
                           /* used by the solver.                                */
  TCF_TOPO_LOOP_PSI = 10,  /* int64[n][3]: node id, edge id, +1 / -1.  psi of   */
                           /* the same split as a function of a_C on the face-  */
                           /* tree edges, at every node where it can be nonzero: */
                           /* face-interior nodes, then continued as a constant  */
                           /* along the gauge tree into the insulator (so the    */
                           /* gauge is kept), stopping at grounded nodes.  The   */
                           /* load correction of a face-tree edge t is           */
                           /* -sum_n (G^T f_I)(n) c(n, t).  Nodes ascending,     */
                           /* then edge ids.  TCF_EINVAL if a gauge subtree hangs */
                           /* from two face nodes.  Not used by the solver.      */
  TCF_TOPO_LOOP_PLAN = 11, /* int64[n][5]: per-patch plan of the same split,    */
                           /* patches in order.  The interface-tree edges leave  */
                           /* the primal set: a conductor appends its own to its */
                           /* b block (by edge id), an insulator eliminates them;*/
                           /* the i block is unchanged; coarse ranks renumber    */
                           /* the primal edges left.  Records:                   */
                           /*  (s, 0, b index, edge id, 0): b block, in order;   */
                           /*  (s, 1, p index, edge id, coarse rank): p block;   */
                           /*  (s, 2, row, b index, +1 / -1): entries of B_s, by */
                           /*  row then b index.  On a loop row the insulator's  */
                           /*  entry is -1 and the conductor's are the row's     */
                           /*  TCF_TOPO_LOOP terms; other rows keep the          */
                           /*  multiplier table's signs.  Not used by the solver.*/
  TCF_TOPO_COARSE = 12     /* The coarse solver's plan: n_Pi values, the index  */
                           /* of each coarse unknown (TCF_TOPO_PRIMAL order) in  */
                           /* the factor's elimination order; then per node of   */
                           /* its elimination tree, in postorder: j0, n_J,       */
                           /* parent (-1 for a root), height, n_S, then the n_S  */
                           /* ascending indices of its structure S (ancestor     */
                           /* unknowns its factor columns reach).  The node owns */
                           /* indices [j0, j0 + n_J); the last node is inverted  */
                           /* densely.  One node: the dense inverse of S_Pi.     */
};

/*
 * Topology of the split, for bit-exact checks.  With out == NULL, *len
 * receives the number of int64 values; otherwise *len is the capacity on
 * entry and the count written on return (TCF_EINVAL if too small).  The
 * loop-split kinds are built on each call and can fail with TCF_ENOMEM.
 */
int tcf_get_topology(const tcf_problem* h, int32_t kind, int64_t* out, size_t* len);

/*
 * Per-patch condition estimate of the local factorisation (after setup):
 * (max_k L_kk / min_k L_kk)^2 over the factor's interior and dual rows, the
 * ratio of the largest to the smallest Cholesky pivot of W_rr restricted to
 * them.  It is a lower bound on that block's condition number and shows which
 * patches can take FP32 factors (TCF_FP32_FULL_IR).  out == NULL returns the
 * count (the number of patches) in *len; otherwise *len is the capacity on
 * entry and the count on return.  Host memory.  TCF_ESTATE before
 * tcf_setup, TCF_EINVAL for a small buffer.
 */
int tcf_get_cond_est(const tcf_problem* h, double* out, size_t* len);

typedef struct tcf_stats {
  int64_t n_patches, n_edges, n_kept, n_lambda, n_primal, n_tree_I;
  int32_t steps_done;
  int32_t last_pcg_iters;      /* of the last PCG solve (last IR sweep)         */
  int64_t total_pcg_iters;     /* summed over all steps and IR sweeps            */
  int32_t max_pcg_iters;
  int32_t last_ir_sweeps;      /* FP32 path; 0 on the FP64 path                  */
  int32_t nonconverged_steps;
  int32_t fail_patch;          /* non-SPD patch, -1 coarse, -2 none              */
  double last_rel_residual;    /* ||r||/||d|| of the last PCG solve              */
  double last_ir_residual;     /* assembled ||f - W a||/||f|| after the last     */
                               /* step (FP32 path; FP64 operator, matrix-free)   */
  double setup_ms;
  double step_ms_total;
  size_t device_bytes;
  double setup_flops;          /* algorithmic flops of the setup factorisations: */
                               /* per patch n_i^3/3 + n_i^2 (n_b + n_p) +        */
                               /* n_i (n_b + n_p)^2 (interior elimination),      */
                               /* n_b^3/3 + n_b^2 n_p + n_b n_p^2 (dual block),  */
                               /* n_b^3/3 + n_b^2 (n_b + n_p) (S_bb^-1, Phi_b),  */
                               /* n_i^3/3 + n_i^2 (n_b + n_p) (Q^T); coarse: per */
                               /* node of its factor below the top block         */
                               /* 2 n_J^3/3 + 2 n_J^2 n_S + n_J n_S^2 (partial    */
                               /* Cholesky, L_JJ^-1, L_JJ^-T L_SJ^T), the top    */
                               /* block 5 n^3/3 (Cholesky, triangular inverse,   */
                               /* one full triangular solve); triangular         */
                               /* right-hand sides counted by their nonzeros     */
  double cond_est_max;         /* largest per-patch pivot ratio (see            */
  int32_t cond_est_patch;      /* tcf_get_cond_est) and its patch; -1 before    */
                               /* setup                                         */
  int32_t coarse_nodes;        /* nodes of the coarse factor (1: dense inverse)  */
  int32_t coarse_launches;     /* tile launches per coarse solve (the kernel    */
                               /* group TCF_KG_COARSE; with the factor, one     */
                               /* more small reduction for p.Fp)                */
  int32_t coarse_root;         /* unknowns of the densely inverted top block    */
  int32_t setup_chunks;        /* patch groups the setup factorised in turn     */
  double coarse_bytes;         /* algorithmic bytes of one coarse solve         */
  size_t device_bytes_peak;    /* high-water mark of the handle's device memory */
  int32_t rhs_batch;           /* excitations per batched PCG after rounding    */
                               /* (more than 4: the matrix-core row panels)     */
  int32_t panel_jobs;          /* row-panel jobs of the F apply (0: the vector  */
                               /* tile path)                                    */
  int32_t panel_chunk[4];      /* split lengths in use: F apply, preconditioner,*/
                               /* coarse correction, coarse solve (0: tiles)    */
  int32_t panel_chunk_src;     /* 0 default or panel_chunk, 1 tune table, 2     */
                               /* timed at setup                                */
  double panel_tune_us[20];    /* when timed: microseconds per launch of each   */
                               /* operator (4, in the order above) at split     */
                               /* lengths 4, 8, 16, 32 and unsplit              */
} tcf_stats;

int tcf_get_stats(const tcf_problem* h, tcf_stats* st);

/*
 * Per-step log of the last `n` steps: PCG iterations (summed over
 * refinement sweeps), refinement sweeps and wall milliseconds.  Any pointer
 * may be NULL.  n is clamped to steps_done.
 */
int tcf_get_step_log(const tcf_problem* h, int32_t n, int32_t* pcg_iters, int32_t* ir_sweeps,
                     double* step_ms);

/*
 * Checkpoint: the state is the step counter and the current field of every
 * excitation.  tcf_get_state with buf == NULL returns the size in *bytes.
 * tcf_set_state restores a state taken from a handle of the same problem.
 */
int tcf_get_state(tcf_problem* h, void* buf, size_t* bytes, void* stream);
int tcf_set_state(tcf_problem* h, const void* buf, size_t bytes, void* stream);

/*
 * Kernel timing for measurement.  While enabled, every launch of the
 * per-step kernel groups below is bracketed by HIP events on its launch
 * stream; launches issued after the PCG converged (which exit at once) are
 * not counted.  tcf_profile_get returns, for group g, the summed event time
 * in milliseconds, the number of launches and the algorithmic bytes one
 * launch must move (each matrix entry read once, symmetric matrices as one
 * triangle, plus its vectors).  Enabling resets the counters.
 */
enum tcf_kernel_group {
  TCF_KG_APPLY = 0,    /* [S_bb^-1 | Phi_b]^T x over all patches (F apply)   */
  TCF_KG_PRECOND = 1,  /* S_bb x over all patches (Dirichlet preconditioner) */
  TCF_KG_PHI = 2,      /* Phi_b N q over all patches                         */
  TCF_KG_COARSE = 3,   /* S_Pi^-1 c in the PCG: tcf_stats.coarse_launches    */
                       /* launches per solve (1 for the dense inverse); its  */
                       /* bytes are those of one whole solve                 */
  TCF_KG_CONDENSE = 4, /* per-step condensation of conductor patches         */
  TCF_KG_RECOVER = 5,  /* interior recovery of all patches                   */
  TCF_KG_COUNT = 6
};
int tcf_profile_enable(tcf_problem* h, int32_t on);
int tcf_profile_get(const tcf_problem* h, int32_t group, double* total_ms, int64_t* launches,
                    double* alg_bytes_per_launch);
/*
 * Algorithmic flops of one launch of group g (per coarse solve for
 * TCF_KG_COARSE): 2 per matrix entry and column of the batch (rhs_batch
 * after rounding), symmetric matrices counted whole, triangular ones as
 * triangles; the matrix-core fraction of a batched product is these flops
 * over its time.  0 for the condensation and recovery groups.  Host only;
 * TCF_EINVAL for a bad group or a NULL output.
 */
int tcf_profile_get_flops(const tcf_problem* h, int32_t group, double* alg_flops_per_launch);

/*
 * Measurement reference: one launch of a plain streaming copy that reads and
 * writes `bytes` (rounded down to 32) through device buffers it allocates
 * and frees.  Traffic counters of the library's kernels are scaled by what
 * the same counters report for this launch.
 */
int tcf_copy_probe(size_t bytes, void* stream);

/*
 * Practical HBM ceilings of the device: a streaming read of `bytes` (16-byte
 * non-temporal loads, 8 in flight per thread) and a copy of `bytes`, each
 * the best of 3 event-timed launches after a warm one, in GB/s (bytes moved:
 * read, and read + written).  Allocates and frees its buffers; synchronises
 * the stream.  TCF_EINVAL for bytes < 32 or NULL outputs, TCF_ENOMEM when the
 * buffers do not fit.
 */
int tcf_bandwidth_probe(size_t bytes, void* stream, double* read_gbs, double* copy_gbs);

/*
 * Releases the handle.  Its device memory goes back to its allocator on the
 * stream of the handle's last stream call, which must still exist (or be
 * the null stream); work already queued there finishes first.
 */
void tcf_destroy(tcf_problem* h);

/*
 * Serving: a stream of independent simulations admitted by device memory.
 *
 * tcf_server_submit does the host work of tcf_create on the calling thread
 * and queues the request with its device footprint (tcf_footprint for the
 * requested precision).  A dispatcher admits queued requests in arrival
 * order whenever a slot is free and the footprint fits in max_bytes next to
 * the running ones; each admitted request runs setup and all n_steps steps
 * on its own worker thread and HIP stream (default priority) on the device
 * that was current at tcf_server_create, so the work of running requests
 * overlaps on the GPU.  When a request finishes, its fields are copied to
 * host memory and its device memory is released, which may admit the next.
 * The phi callback of a request must stay valid until the request is DONE
 * or FAILED (it is called from the worker thread during setup).
 * A request whose footprint exceeds max_bytes fails with TCF_ENOMEM.
 */
typedef struct tcf_server tcf_server;

enum tcf_request_state {
  TCF_REQ_QUEUED = 0,
  TCF_REQ_RUNNING = 1,
  TCF_REQ_DONE = 2,
  TCF_REQ_FAILED = 3
};

typedef struct tcf_server_report {
  int32_t submitted, admitted, completed, failed, running, queued;
  int64_t steps;             /* steps completed over all requests              */
  double p50_step_ms;        /* over all steps of all completed requests       */
  double p99_step_ms;
  double p50_queue_ms;       /* submit -> admission                            */
  double p99_queue_ms;
  double busy_ms;            /* first admission -> last completion             */
  size_t peak_bytes;         /* peak admitted footprint                        */
} tcf_server_report;

int tcf_server_create(size_t max_bytes, int32_t max_slots, tcf_server** out);
int tcf_server_submit(tcf_server* srv, const tcf_problem_desc* desc, const tcf_options* opts,
                      int32_t* req_id);
int tcf_server_poll(tcf_server* srv, int32_t req_id, int32_t* state);
/* Blocks until the request is DONE or FAILED; returns its final status. */
int tcf_server_wait(tcf_server* srv, int32_t req_id);
/* Final field of excitation k (host copy), length n_edges; stats may be NULL. */
int tcf_server_fetch(tcf_server* srv, int32_t req_id, int32_t k, double* out, size_t len,
                     tcf_stats* stats);
int tcf_server_stats(tcf_server* srv, tcf_server_report* st);
/* Failure message of a FAILED request (empty otherwise); owned by the server. */
const char* tcf_server_error(tcf_server* srv, int32_t req_id);
/* Waits for every request, joins the threads and frees everything. */
void tcf_server_destroy(tcf_server* srv);

/* Message of the last failure on h (h may be NULL for create failures). */
const char* tcf_last_error(const tcf_problem* h);

#ifdef __cplusplus
}
#endif

#endif /* TCF_H */
