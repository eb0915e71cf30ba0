/*
 * dgfas.h - C ABI of the MI355X (gfx950) FAS multigrid / weighted-Schwarz
 * library for SIPG discontinuous Galerkin spectral elements.
 *
 * Problem (Sec. 2.1, eq. helmholtz): kappa u - div(nu grad u) = f on a mesh of
 * conforming hexahedra with Dirichlet or Neumann faces; constant kappa >= 0
 * and nu > 0.  Discretisation (Sec. 2.2, eq. helmholtz:dgm): nodal GLL basis of
 * degree p per element, isoparametric geometry in the same basis, GLL
 * quadrature, symmetric interior penalty with mu = mu_star avg(p(p+1)/(2 h_perp)).
 *
 * Conventions
 *  - Vectors are device pointers to FP64 data in element-major layout: element
 *    e owns [e*(p+1)^3, (e+1)*(p+1)^3); inside an element nodes are
 *    lexicographic with i (xi_1) fastest, then j (xi_2), then k (xi_3).  The
 *    caller owns every pointer it passes; the library never frees them.
 *  - Faces are numbered 0:-xi_1 1:+xi_1 2:-xi_2 3:+xi_2 4:-xi_3 5:+xi_3.
 *    Neighbours must be aligned (face node (a,b) of one side is face node
 *    (a,b) of the other).
 *  - Levels count from 1 (root, p = 1) to L (finest), as in Sec. 3.1; each
 *    coarser level halves the degree: p_{l-1} = max(1, floor(p_l / 2)).
 *  - All device work is enqueued on the stream given at creation (NULL = the
 *    null stream) and is asynchronous unless stated otherwise.
 *  - Errors: every call returns a dgfas_status; on failure nothing has been
 *    enqueued and dgfas_last_error() gives a message.  Nothing is thrown.
 *  - One solver object must not be used by two threads at the same time.
 */
#ifndef DGFAS_H
#define DGFAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DGFAS_OK = 0,
  DGFAS_ENOTCONV = 1,      /* warning: tolerance not reached; outputs are valid */
  DGFAS_EFALLBACK = 2,     /* warning: converged after the learned correction was switched off */
  DGFAS_EINVAL = -1,       /* bad argument (null pointer, bad size, bad level) */
  DGFAS_ENOMEM = -2,       /* device allocation failed */
  DGFAS_EHIP = -3,         /* HIP runtime error (message in dgfas_last_error) */
  DGFAS_EUNSUPPORTED = -4, /* valid input outside what the library implements */
  DGFAS_EBREAKDOWN = -5    /* non-finite value or p^T A p <= 0 inside SCG */
} dgfas_status;

enum { DGFAS_INTERIOR = 0, DGFAS_DIRICHLET = 1, DGFAS_NEUMANN = 2,
       /* Schwarz side code only: an interior face toward an element of another degree,
          where the subdomain has no overlap (own half of the interior face terms) */
       DGFAS_INTERIOR_NO_OVERLAP = 3 };
enum { DGFAS_WAS = 0, DGFAS_SCG = 1 };
enum { DGFAS_FP64 = 0, DGFAS_FP32 = 1, DGFAS_BF16 = 2, DGFAS_FP32_MFMA = 3 };
enum { DGFAS_BATCH_PER_DEGREE = 0, DGFAS_BATCH_ONE_LAUNCH = 1, DGFAS_BATCH_TUNED = 2, DGFAS_BATCH_PERSISTENT = 3 };
enum { DGFAS_ORDER_NATURAL = 0, DGFAS_ORDER_MORTON = 1 };
enum { DGFAS_START_NONE = 0, DGFAS_START_CMG = 1, DGFAS_START_FMG = 2 };
enum { DGFAS_WEIGHT_QUINTIC = 0, DGFAS_WEIGHT_PLAIN = 1 };
enum { DGFAS_PROJECT_INTERP = 0, DGFAS_PROJECT_L2 = 1 };

typedef struct dgfas_solver_s* dgfas_solver;

/* Mesh (Sec. 2.2): host arrays, read during dgfas_create only.
 * Degrees may differ between elements (an extension: the paper keeps one degree per level,
 * Sec. 3.1).  A face between degrees p and p' is integrated with the GLL rule of the finer
 * side, the penalty uses both degrees, the Schwarz subdomains do not overlap into an
 * element of another degree, and p-coarsening p -> max(1, p / 2) is applied per element.
 * Every vector is element-major: element e owns the (p_e+1)^3 entries after those of
 * elements 0..e-1, its nodes lexicographic with xi_1 fastest. */
typedef struct {
  int32_t n_elem;
  const int32_t* degree;    /* [n_elem] polynomial degree per element, 1..8 */
  const double* coords;     /* per element, in element order, [3][(p_e+1)^3] nodal x, y, z at
                               the element's GLL nodes (the GLL nodes of dgfas_gll); the map
                               must keep det J > 0 */
  const int32_t* face_nbr;  /* [n_elem][6] neighbour element, or -1 on the boundary */
  const int8_t* face_bc;    /* [n_elem][6] DGFAS_DIRICHLET / DGFAS_NEUMANN on boundary faces */
  int32_t box[3];           /* h-coarsening only (options.h_levels > 0): the mesh is a box of
                               nx x ny x nz elements numbered e = ex + nx (ey + ny ez), its face
                               neighbours those of the box or its periodic wraps; else ignored */
  const double* nu_nodal;   /* spatially varying diffusivity nu(x) of eq. helmholtz:pde at the GLL
                               nodes, laid out like a solution vector, or NULL: options.nu
                               everywhere.  One degree only.  Values >= 0 with positive element
                               averages.  The bilinear form (eq. helmholtz:dgm) weights the volume
                               term and each side's normal flux with its own nodal values and the
                               interior penalty with max(nu-, nu+); the Schwarz surrogate takes the
                               element average (Sec. 4.3.1); coarser levels evaluate the field at
                               their own nodes, as they do the geometry */
  const int32_t* refine_count;  /* local refinement (options.local_steps > 0, Sec. 3.1): elements of
                               the base mesh, then of each refined level in turn, marked for regular
                               refinement; refine_count[k] entries of refine_list per step k */
  const int32_t* refine_list;   /* element ids of the level being refined.  A marked element must be
                               active, and so must every element of its 3 x 3 x 3 block inside the
                               domain (the block's other elements are refined irregularly: their
                               children are frozen).  The refined level lists, parent by parent in
                               id order, the 8 children c = bx + 2 by + 4 bz of every regularly or
                               irregularly refined parent (b = 1: the upper half of the parent's
                               reference interval along that axis); a child's geometry is its
                               parent's map at the child's nodes */
  const int8_t* face_nbr_face;  /* unstructured meshes (Sec. 5.1 keeps, per face, the neighbour, its related
                               face and the relative orientation): [n_elem][6] the face (0..5) of the
                               neighbour that meets each interior face, or NULL: aligned neighbours
                               (face phi ^ 1, orientation 0; the structured grids).  With it the
                               Schwarz subdomains of Sec. 4.3.1 are found by walking across oriented
                               faces: edge and vertex neighbours without a counterpart are zero-filled,
                               the nodes of surplus ones on the shared edge or vertex are averaged into
                               one slot, and the corrections are normalised by the weight sum per node.
                               One degree; no h_levels, local_steps, matrix-core precisions or learned
                               correction */
  const int8_t* face_orient;    /* [n_elem][6] relative orientation code 0..7 of each interior face, or
                               NULL (all 0).  Face nodes are laid out (first, second) = (xi_3, xi_2) on
                               faces 0/1, (xi_3, xi_1) on 2/3, (xi_2, xi_1) on 4/5; the own face node
                               (a, b) is the neighbour's face node (a', b') with (x, y) = (b, a) if bit 0
                               is set, else (a, b), then a' = n-1-x if bit 1, else x, and b' = n-1-y if
                               bit 2, else y.  Both sides must list each other with inverse codes */
} dgfas_mesh_desc;

/* Solver options.  Defaults come from dgfas_default_options. */
typedef struct {
  double kappa;             /* >= 0 */
  double nu;                /* > 0 */
  double mu_star;           /* penalty scale of eq. helmholtz:dgm, > 0 */
  int32_t overlap;          /* Schwarz overlap m in node layers (Sec. 4.3.1 item 3), or < 0: m per
                               degree from delta (the neighbour's GLL nodes with (1 + xi)/2 <= delta,
                               its face node included).  Kernels exist for m in {0, 1} at every
                               degree, m = 2 at p = 4 and 8, and m = 3 at p = 8; other pairs on any
                               level give DGFAS_EUNSUPPORTED */
  int32_t smoother;         /* DGFAS_WAS (Alg. 5) or DGFAS_SCG (Alg. 6) on levels > 1 */
  int32_t ns1, ns2;         /* pre- and post-smoothing steps (Alg. 2) */
  int32_t root_max_iter;    /* SCG iteration cap of the root solve */
  double root_rtol;         /* root SCG stops when ||r|| <= root_rtol * ||r_0||; 0: exactly
                               root_max_iter iterations with no convergence test (no host
                               synchronisation: with graph = 1 the whole cycle is one graph) */
  int32_t precision;        /* DGFAS_FP64, or DGFAS_FP32: smoothing of the correction system
                               (eq. smoothers:system:correction) in FP32 on levels > 1 with the
                               FAS residual, tau-correction and root solve in FP64, or DGFAS_BF16:
                               as DGFAS_FP32 with the subdomain solves' tensor contractions on
                               BF16 matrix cores (operands rounded to BF16, FP32 accumulation),
                               or DGFAS_FP32_MFMA: the same contractions on FP32 matrix cores */
  int32_t n_rhs;            /* right-hand sides solved together, 1..64: every vector argument is then
                               [n_rhs][n_dof] (each right-hand side contiguous) and every SCG scalar is
                               kept per right-hand side; the geometry is shared */
  int32_t batch;            /* mixed-degree levels: DGFAS_BATCH_PER_DEGREE (one launch per degree
                               bucket and stage), DGFAS_BATCH_ONE_LAUNCH (one launch per sweep
                               stage over all buckets, a workgroup per tile),
                               DGFAS_BATCH_PERSISTENT (one launch per stage whose workgroups, about
                               24 waves per compute unit, stride through the tile list) or
                               DGFAS_BATCH_TUNED (the choice per level and stage made by
                               dgfas_autotune; per-degree until it has run).
                               Levels with one degree always take one launch per stage */
  int32_t graph;            /* 1: dgfas_solve replays each V-cycle's smoothing and transfer legs
                               as two captured HIP graphs (the root solve between them runs
                               eagerly), or the whole cycle as one graph when root_rtol = 0;
                               results are bitwise those of the eager cycle.  Not with the
                               learned correction */
  int32_t order;            /* element processing order of the sweep kernels: DGFAS_ORDER_NATURAL
                               (element index) or DGFAS_ORDER_MORTON (Morton order of the element
                               centroids, so that concurrently running workgroups of one XCD take
                               a compact 3D block and share their neighbours' data in L2).
                               Operator and Schwarz results are bitwise the same; dot products
                               fused into the kernels sum their partials in another order */
  int32_t start;            /* start-up of dgfas_solve (Sec. 3.3): DGFAS_START_NONE, DGFAS_START_CMG
                               (Alg. 3, cascadic) or DGFAS_START_FMG (Alg. 4, full multigrid); the
                               coarser levels' right-hand sides are f_{l-1} = R f_l */
  int32_t ns0;              /* CMG smoothing steps per level; <= 0: ns1 + ns2 */
  int32_t nsc;              /* crossover smoothing (Sec. 6.1 method names): top-level steps between
                               the residual checks of two consecutive cycles, i.e. every cycle after
                               the first starts with nsc - ns2 pre-smoothing steps on the finest
                               level; <= 0: ns1 + ns2 (no crossover); must be >= ns2 */
  int32_t weighting;        /* DGFAS_WEIGHT_QUINTIC (the partition of unity of Sec. 4.3.1) or
                               DGFAS_WEIGHT_PLAIN (W = I: plain additive Schwarz) */
  double delta;             /* overlap width in the standard element when overlap < 0, 0 <= delta < 1 */
  int32_t projection;       /* FAS solution projection P (Sec. 3.2): DGFAS_PROJECT_INTERP (embedded
                               interpolation: evaluation at the coarse GLL nodes) or DGFAS_PROJECT_L2
                               (reference-element L2 projection (I^T W I)^-1 I^T W per direction) */
  int32_t h_levels;         /* h-coarsening (Sec. 3.1): the finest box mesh is coarsened h_levels
                               times into parents of 2 x 2 x 2 children at the same degree, with the
                               transfers of Sec. 3.2 (I embedded, R = I^T, P the children's fields at
                               the parent's nodes averaged where they meet); needs one degree and
                               mesh.box.  0: none */
  int32_t h_only;           /* with h_levels > 0: 1 makes the coarsest h-level the root (pure h-MG,
                               root SCG at the fine degree); 0 p-coarsens it down to p = 1 */
  int32_t local_steps;      /* local h-refinement (Sec. 3.1, 3.3): levels above the given base mesh
                               built from mesh.refine_count / refine_list, with twig, leaf and
                               frozen elements; the base is p-coarsened down to p = 1 below it.
                               One degree, FP64, one right-hand side, no h_levels, CMG start-up,
                               crossover, graph, nodal nu or learned correction.  0: none */
  int32_t null_space;       /* 1: the operator is semidefinite (kappa = 0 and no Dirichlet face: periodic
                               or pure Neumann), with the constants as its null space; the root SCG
                               projects its residual and every preconditioned residual onto the
                               range of A (the zero-mean vectors; remark on IPCG for semidefinite
                               systems, Sec. 4.3.2).  The right-hand side must have zero mean in every
                               right-hand side; the solution is fixed up to a constant.  0: off */
} dgfas_options;

void dgfas_default_options(dgfas_options* opt);

/* GLL nodes and weights of degree p (1..16), host arrays of p+1 doubles
 * (Remark on basis functions).  Usable without a GPU. */
dgfas_status dgfas_gll(int32_t p, double* x, double* w);

/* Host-only: 1D subdomain tables of the Schwarz method (Sec. 4.3.1) for degree p,
 * overlap m and face conditions (left, right) in {DGFAS_INTERIOR, DGFAS_DIRICHLET,
 * DGFAS_NEUMANN, DGFAS_INTERIOR_NO_OVERLAP}.  Outputs (host, caller-sized): ns = number of subdomain nodes,
 * S [ns*ns] row-major with S^T M S = I and S^T L S = diag(lam), lam [ns], weights [ns].
 * ns <= p + 1 + 2m.  Usable without a GPU. */
dgfas_status dgfas_schwarz_tables_1d(int32_t p, int32_t m, int32_t left, int32_t right,
                                     double mu_star, int32_t* ns, double* S, double* lam,
                                     double* weights);

/* Build the level hierarchy, the geometry on every level and the Schwarz data.
 * stream: a hipStream_t (NULL = null stream).  Synchronous. */
dgfas_status dgfas_create(const dgfas_mesh_desc* mesh, const dgfas_options* opt, void* stream,
                          dgfas_solver* out);
void dgfas_destroy(dgfas_solver s);

/* Number of levels L, and degree / DOF count of one level (the largest degree of the
 * level when degrees differ; n_dof is the sum of (p_e+1)^3 over the elements). */
dgfas_status dgfas_levels(dgfas_solver s, int32_t* n_levels);
dgfas_status dgfas_level_info(dgfas_solver s, int32_t level, int32_t* degree, int64_t* n_dof);
/* Schwarz overlap m (node layers) of a level's largest degree, as set by overlap or delta; the
 * subdomain tile of that degree has ns = degree + 1 + 2m nodes per direction. */
dgfas_status dgfas_level_overlap(dgfas_solver s, int32_t level, int32_t* m);
/* Subdomain blocks of an unstructured level (mesh.face_nbr_face given; Sec. 4.3.1 design
 * principles 4-6): counts[5] = the element blocks, face blocks, edge and vertex blocks mapped
 * one-to-one, zero-filled ones and merged ones, summed over the level's subdomains (host array,
 * written; all zero on a structured level). */
dgfas_status dgfas_level_blocks(dgfas_solver s, int32_t level, int64_t* counts);

/* Workspace: the per-call scratch of the configured cycle (the work vectors of every level,
 * the overlap inboxes, reduction partials and SCG scalars; no state is kept in it between
 * calls).  After dgfas_create it is one library-owned device block of workspace_size bytes.
 * dgfas_set_workspace hands in a caller-owned device buffer instead (for example a torch
 * tensor): at least that many bytes, 256-byte aligned, kept alive by the caller until the
 * solver is destroyed or another workspace is set; the library then frees its block, so the
 * configured cycle runs in caller-owned memory only (the geometry and tables stay the
 * library's).  dptr = NULL returns to a library-owned block.  The call synchronises the stream
 * first, clears what must start at zero, and drops captured graphs.  Work that the configured
 * cycle does not do (dgfas_root_solve on a level without SCG vectors, the learned correction)
 * may still allocate its buffers on first use. */
dgfas_status dgfas_workspace_size(dgfas_solver s, size_t* bytes);
dgfas_status dgfas_set_workspace(dgfas_solver s, void* dptr, size_t bytes);

/* Right-hand side of eq. helmholtz:system on the finest level from nodal values
 * (device): f [n_dof], uD [n_dof] (values at Dirichlet face nodes are used; may be
 * NULL for u_D = 0), qN [n_dof] (Neumann flux at Neumann face nodes; may be NULL).
 * b [n_dof] is written. */
dgfas_status dgfas_rhs(dgfas_solver s, const double* f, const double* uD, const double* qN, double* b);

/* Local refinement (options.local_steps > 0).  Every level keeps its own solution; the leaves
 * of every level carry the original right-hand side and the twigs the FAS one (eq.
 * helmholtz:fas).  dgfas_solve then runs Alg. 2 with the frozen update and measures the
 * composite residual: the 2-norm of f^l - A u over the leaf rows of every level (eq.
 * helmholtz:fas:converged:leaves), relative to its value at the start; the top level's u and f
 * are the call's, the other levels start from zero in every call.
 *
 * Element classes of a level into cls (host, [n_elem] of that level): 0 twig, 1 leaf, 2 frozen. */
dgfas_status dgfas_level_classes(dgfas_solver s, int32_t level, int8_t* cls);
/* Nodal coordinates of a level (host, per element [3][(p+1)^3]), e.g. to evaluate f there. */
dgfas_status dgfas_level_coords(dgfas_solver s, int32_t level, double* coords);
/* b = the discrete right-hand side of eq. helmholtz:system on level l (device vectors of that
 * level; uD, qN may be NULL), over all its elements. */
dgfas_status dgfas_level_rhs(dgfas_solver s, int32_t level, const double* f, const double* uD, const double* qN,
                             double* b);
/* b (device, n_dof of the level): the discrete right-hand side of a level below the top, copied
 * into library memory.  Its leaf rows enter every cycle (the twig rows are set by the cycle);
 * with the FMG start-up (options.start, Alg. 4) each level's active rows serve the stage whose
 * top it is, its twigs acting as leaves there, so every level below the top needs one. */
dgfas_status dgfas_set_level_rhs(dgfas_solver s, int32_t level, const double* b);
/* u = the current solution of a level below the top (device, n_dof of the level). */
dgfas_status dgfas_level_solution(dgfas_solver s, int32_t level, double* u);

/* Au = A_l u (eq. helmholtz:system on level l).  On a locally refined level only the rows of
 * active elements are written. */
dgfas_status dgfas_apply(dgfas_solver s, int32_t level, const double* u, double* Au);

/* r = g - A_l u (Alg. 2 residual computation). */
dgfas_status dgfas_residual(dgfas_solver s, int32_t level, const double* u, const double* g, double* r);

/* z = sum_e R_s^T W^e (A~_s^e)^-1 R_s r: one weighted Schwarz application
 * (eq. schwarz:correction) with fast-diagonalisation subdomain solves. */
dgfas_status dgfas_schwarz(dgfas_solver s, int32_t level, const double* r, double* z);

/* The same z = B r as dgfas_schwarz, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The call allocates
 * nothing: its overlap inbox is a static device array of 8 Mi doubles (64 MiB), one per device,
 * which every call on that device shares and which keeps the last call's contents; the call clears
 * what it needs with a fill kernel first.  Calls that overlap on one device race on it.
 * Levels whose inbox (n_rhs times the overlap slots of every element) exceeds the array are
 * refused with DGFAS_EINVAL; with the learned correction attached, the finest level is refused
 * with DGFAS_EUNSUPPORTED (its network may allocate). */
dgfas_status dgfas_schwarz_noalloc(dgfas_solver s, int32_t level, const double* r, double* z);

/* n_steps smoothing steps of the configured smoother on A_l u = g, in place
 * (Alg. 5 WAS, or Alg. 6 SCG with r_max = 0). */
dgfas_status dgfas_smooth(dgfas_solver s, int32_t level, double* u, const double* g, int32_t n_steps);

/* Transfers between level l (fine) and l-1 (coarse), Sec. 3.2:
 *   restrict:    r_c = R r_f = I^T r_f
 *   project:     u_c = P u_f (embedded interpolation at the coarse GLL nodes)
 *   prolong_add: u_f += I (u_c - ubar_c)   (ubar_c may be NULL for u_f += I u_c) */
dgfas_status dgfas_restrict(dgfas_solver s, int32_t level, const double* r_fine, double* r_coarse);
dgfas_status dgfas_project(dgfas_solver s, int32_t level, const double* u_fine, double* u_coarse);
dgfas_status dgfas_prolong_add(dgfas_solver s, int32_t level, const double* u_coarse,
                               const double* ubar_coarse, double* u_fine);

/* Root solve on level 1: SCG (Alg. 6) from u until ||r|| <= root_rtol ||r_0|| or
 * root_max_iter iterations (root_rtol = 0: exactly root_max_iter, asynchronous); iters
 * (host, may be NULL) receives the count.  Synchronous when root_rtol > 0. */
dgfas_status dgfas_root_solve(dgfas_solver s, double* u, const double* g, int32_t* iters);

/* The configured start-up alone (DGFAS_START_CMG: Alg. 3, DGFAS_START_FMG: Alg. 4) from the
 * finest-level start value u (projected to the coarser levels); u receives the interpolated
 * start value I u_{L-1}.  DGFAS_START_NONE leaves u unchanged.  Synchronous (root solves). */
dgfas_status dgfas_startup(dgfas_solver s, double* u, const double* f);

/* One FAS V-cycle (Alg. 2, global p-coarsening) on the finest-level u for rhs f. */
dgfas_status dgfas_vcycle(dgfas_solver s, double* u, const double* f);

/* The configured start-up (start), then FAS V-cycles with crossover smoothing (nsc) until
 * ||f - A u|| <= rtol ||f - A u_0|| for every right-hand side, or max_cycles.
 * hist (host, may be NULL) receives max_cycles+1 relative residuals, the largest over the
 * right-hand sides (entry 0 = 1);
 * n_done (host, may be NULL) the number of cycles run.  Synchronises once per cycle.
 * Returns DGFAS_ENOTCONV (a warning) if the tolerance was not reached. */
dgfas_status dgfas_solve(dgfas_solver s, double* u, const double* f, int32_t max_cycles, double rtol,
                         double* hist, int32_t* n_done);

/* Autotuner of the mixed-degree launch shape: for every level with more than one degree and
 * each sweep stage (operator, subdomain solves, overlap add) it times the per-degree launches,
 * the one-launch batch and the persistent one-launch batch with HIP events (median of `reps`
 * runs on the solver's stream, on scratch vectors) and keeps the fastest; it then sets
 * opt.batch = DGFAS_BATCH_TUNED.
 * cache_path (may be NULL): a JSON file of earlier choices keyed by device architecture,
 * level degree histogram, precision and n_rhs; entries found there are used without timing
 * and new ones are appended.  report (host, may be NULL): [n_levels][3][3] times in ms,
 * per-degree, one-launch, persistent, 0 where a level has one degree.  Synchronous. */
dgfas_status dgfas_autotune(dgfas_solver s, const char* cache_path, int32_t reps, double* report);

/* Euclidean norm of a level-l vector per right-hand side, written to out (host, n_rhs doubles).
 * Synchronous. */
dgfas_status dgfas_norm(dgfas_solver s, int32_t level, const double* v, double* out);

/* ---- Learned subdomain correction (addition to the paper's method) -------------------
 * A 3-layer MLP in -> hidden -> hidden -> out, ReLU after the first two layers, BF16
 * weights with FP32 accumulation on the matrix cores, FP32 master weights.  Parameters
 * (FP32, one array): W1[in][hidden] b1[hidden] W2[hidden][hidden] b2[hidden]
 * W3[hidden][out] b3[out].  Device arrays X [rows][in], Y/T [rows][out] are FP32, row-major. */
typedef struct dgfas_mlp_s* dgfas_mlp;

/* Create with He-normal weights drawn from `seed` and zero biases; stream as in dgfas_create. */
dgfas_status dgfas_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, uint64_t seed, void* stream,
                              dgfas_mlp* out);
void dgfas_mlp_destroy(dgfas_mlp m);
dgfas_status dgfas_mlp_num_params(dgfas_mlp m, int64_t* n);
/* Host copies of the FP32 master parameters (n_params floats).  set resets Adam. Synchronous. */
dgfas_status dgfas_mlp_get_params(dgfas_mlp m, float* host);
dgfas_status dgfas_mlp_set_params(dgfas_mlp m, const float* host);
/* Y = MLP(X) for `rows` rows. */
dgfas_status dgfas_mlp_forward(dgfas_mlp m, const float* X, int32_t rows, float* Y);
/* loss = mean((MLP(X) - T)^2) over rows*out values and its gradient with respect to the
 * parameters (device, n_params floats; may be NULL).  Synchronous. */
dgfas_status dgfas_mlp_gradient(dgfas_mlp m, const float* X, const float* T, int32_t rows, float* grad,
                                double* loss);
/* `steps` Adam steps (beta 0.9/0.999, eps 1e-8) on consecutive mini-batches of `batch` rows of
 * (X, T) [n rows], learning rate lr_min + (lr0 - lr_min)(1 + cos(pi t / total_steps))/2 at
 * global step t; losses (host, may be NULL) receives the loss of every step.  Synchronous. */
dgfas_status dgfas_mlp_train(dgfas_mlp m, const float* X, const float* T, int64_t n, int32_t batch,
                             int32_t steps, float lr0, float lr_min, int32_t total_steps, double* losses);

/* Attach (enabled = 1; 2 = attach without the fallback rule, for diagnostics) or detach
 * (enabled = 0) the network as a correction of the finest-level FD subdomain
 * solves: du_s <- du_s + |r_s| MLP(r_s / |r_s|, J9) with r_s the subdomain residual tile
 * (ns^3 values, ns = p + 1 + 2m) and J9 the element's linear map Jacobian / det^(1/3).
 * Needs n_rhs = 1 and DGFAS_FP64; the network must map ns^3 + 9 -> ns^3.  The network must
 * outlive the attachment.  dgfas_solve then judges it against the plain smoother: the first two
 * cycles of the first solve after attaching run plain and the second one's reduction factor is
 * the reference; a learned cycle that reduces less (or goes non-finite) is undone, the rest of
 * the solve runs plain and the call returns DGFAS_EFALLBACK. */
dgfas_status dgfas_set_learned(dgfas_solver s, dgfas_mlp m, int32_t enabled);

/* Training pairs from the method itself: for the n finest-level elements `centers` (host; any
 * two at least 4 elements apart so that their 3x3x3 patches neither overlap nor touch), the
 * subdomain residual r_s = R_s r, the FD solve and the exact local solve (R_s A R_s^T)^-1 r_s
 * (masked PCG with the FD preconditioner to 1e-11).  Writes X [n][ns^3 + 9] =
 * [r_s / |r_s|, J9] and T [n][ns^3] = (exact - FD) / |r_s| (device, FP32, tile order of the
 * FD solve).  pcg_iters (host, may be NULL) gets the PCG iteration count.  Synchronous. */
dgfas_status dgfas_learned_pairs(dgfas_solver s, const double* r, const int32_t* centers, int32_t n,
                                 float* X, float* T, int32_t* pcg_iters);

/* Message of the last failed call on this thread. */
const char* dgfas_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DGFAS_H */
