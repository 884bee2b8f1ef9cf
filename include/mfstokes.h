/*
 * mfstokes: matrix-free Taylor-Hood Stokes / stabilised Navier-Stokes
 * operators and multigrid solvers on structured hexahedral meshes, for AMD
 * MI355X (gfx950).
 *
 * Methods follow Munch et al., "Solving the (Navier-)Stokes equations with
 * space and time adaptivity using deal.II":
 *   - Stokes weak form, Sec. 1 eq. (stokes); block system and
 *     Silvester-Wathen preconditioner, Sec. 3 eq. (stokes_block);
 *   - matrix-free operator evaluation in smoothing and transfer, Sec. 1/2;
 *   - cell-wise transfer x_f = sum_e S_e W_e P_e C_e G_e x_c, restriction its
 *     transpose, Sec. 2 eq. (transfer);
 *   - Chebyshev smoothing around point Jacobi, Sec. 2 and 3;
 *   - p-multigrid then global-coarsening h-multigrid, Sec. 3;
 *   - SUPG/PSPG stabilised Navier-Stokes Jacobian with BDF2, Sec. 5.
 *
 * Conventions shared by every call
 * --------------------------------
 * Mesh: structured grid of n[0] x n[1] (x n[2]) cells, vertices numbered
 *   lexicographically with x fastest; each cell is the Q1 (bi/trilinear) image
 *   of the reference cell [0,1]^dim.
 * Bases: nodal Lagrange on Gauss-Lobatto-Legendre points; quadrature: tensor
 *   Gauss-Legendre with k+1 points per direction (k = velocity degree).
 * Vectors: blocked [u_0 | u_1 | (u_2) | p].  Scalar node (i,j,l) of degree d
 *   has index i + (d n0 + 1) (j + (d n1 + 1) l).  Pressure degree is k-1
 *   (Taylor-Hood) or k (equal order, Navier-Stokes).
 * Constraints: every velocity node on the boundary is a Dirichlet node.  The
 *   operators act as the identity on Dirichlet rows and ignore the source
 *   values there in every other row (homogeneous operator; inhomogeneous data
 *   enters the right-hand side by lifting, see mfs_rhs).
 * Sign: the pressure rows carry B^T u with B_ij = -(psi_j, div phi_i), making
 *   the Stokes matrix [[A, B], [B^T, 0]] symmetric (eq. (stokes_block)).
 * Memory: every vector argument is a device pointer (hipMalloc / torch CUDA
 *   tensor) of exactly the documented length, in the precision named by the
 *   call, not aliasing any other argument unless stated.  Device memory the
 *   library needs internally is allocated in mfs_setup and freed by
 *   mfs_destroy, or carved from a caller-owned arena (mfs_setup_arena).  Streams are hipStream_t passed as void* (NULL = default).
 * Errors: every call returns MFS_OK (0) or a negative code; mfs_last_error()
 *   returns a thread-local message for the last failure.  No C++ exception
 *   crosses this interface.
 * Threads: a problem handle may be used by one host thread at a time;
 *   different handles are independent.
 */
#ifndef MFSTOKES_H
#define MFSTOKES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MFS_OK 0
#define MFS_EINVAL (-1)
#define MFS_ENOMEM (-2)
#define MFS_EUNSUPPORTED (-3)
#define MFS_EHIP (-4)
#define MFS_ENOCONV (-5)

/* precision of an operation */
#define MFS_FP64 0
#define MFS_FP32 1

/* relaxation of the monolithic Navier-Stokes multigrid (mfs_options.relax_type) */
#define MFS_RELAX_JACOBI 0 /* damped point Jacobi x += omega D^-1 (b - J x) */
#define MFS_RELAX_ASM 1    /* additive Schwarz: x += omega sum_P R_P^T W A_P^-1 R_P (b - J x), one patch
                              per vertex (the unknowns within one cell of it), W = 1/multiplicity */

/* operators for mfs_vmult */
#define MFS_OP_STOKES 0      /* [u;p] -> [A u + B p ; B^T u], full vectors            */
#define MFS_OP_A 1           /* velocity block: u -> A u (vector Laplacian, nu-scaled) */
#define MFS_OP_B 2           /* p -> B p (velocity-sized output, 0 on Dirichlet rows)  */
#define MFS_OP_BT 3          /* u -> B^T u (pressure-sized output)                     */
#define MFS_OP_MASS_P 4      /* p -> M_p p (pressure mass)                             */
#define MFS_OP_NS_JACOBIAN 5 /* [du;dp] -> J [du;dp], SUPG/PSPG Jacobian (Sec. 5)      */
#define MFS_OP_MASS_U 6      /* u -> M_u u, velocity mass per component (Sec. 4)        */

typedef struct mfs_problem mfs_problem;

typedef struct mfs_mesh {
  int dim;                /* 2 or 3 */
  int n[3];               /* cells per direction (n[2] ignored in 2D) */
  const double *vertices; /* host, [(n0+1)(n1+1)(n2+1)][dim], x fastest */
} mfs_mesh;

typedef struct mfs_options {
  int pressure_offset;   /* 1: Taylor-Hood Q_k/Q_{k-1}; 0: equal order Q_k/Q_k */
  int mg_levels;         /* 1: multigrid hierarchy built at setup; 0: operators only */
  int cheb_degree;       /* Chebyshev degree of the smoother (Sec. 3: 5) */
  double cheb_range;     /* smoothing range: interval [lambda/range, lambda] */
  double cheb_safety;    /* lambda = safety * estimated lambda_max(D^-1 A) */
  int lanczos_steps;     /* steps of the lambda_max estimate */
  int p_min;             /* lowest degree of the p-levels (1 by Sec. 3) */
  int coarse_min_cells;  /* stop h-coarsening when a direction has <= this many cells */
  int schur_iterations;  /* PCG iterations for S~^{-1} = nu M_p^{-1} */
  int restart;           /* FGMRES restart length */
  int maxit;             /* FGMRES iteration limit */
  double rtol;           /* FGMRES relative residual target */
  int precond_precision; /* MFS_FP32 or MFS_FP64 for the block preconditioner */
  uint64_t seed;         /* seed of the Lanczos start vector */
  /* monolithic Navier-Stokes multigrid (Sec. 5) */
  int relax_steps;       /* damped point-Jacobi sweeps before and after the coarse correction (5) */
  double relax_omega;    /* Jacobi damping omega (0.5) */
  /* solve loop */
  int graphs;            /* 1: the FP32 preconditioner of a solve is recorded once per problem as a
                            HIP graph and replayed each FGMRES iteration; 0: launched kernel by kernel */
  int relax_type;        /* Navier-Stokes relaxation: MFS_RELAX_JACOBI (point Jacobi) or MFS_RELAX_ASM
                            (additive Schwarz on vertex patches, Sec. 2 and Sec. 5 Exp. 4; structured
                            meshes, degrees 1 and 2; the paper's Exp. 4 uses 2 steps, omega = 1) */
} mfs_options;

typedef struct mfs_solve_info {
  int iterations;        /* outer FGMRES iterations performed */
  int status;            /* MFS_OK or MFS_ENOCONV */
  double rel_residual;   /* ||b - K x||_2 / ||b||_2 recomputed in FP64 at exit */
  double seconds;        /* wall time of the solve on the host clock */
} mfs_solve_info;

/* Fill *opts with the defaults listed in the implementation. */
void mfs_default_options(mfs_options *opts);

/* Thread-local text of the last error. */
const char *mfs_last_error(void);

/*
 * Device bytes mfs_setup will allocate for this mesh / degree / options
 * (the footprint used for memory-based admission of requests).
 * Host only; validates like mfs_setup.  MFS_EINVAL on bad sizes or degree.
 */
int mfs_footprint(const mfs_mesh *mesh, int k, const mfs_options *opts, size_t *bytes);

/*
 * setup(mesh, degrees, nu): copies the mesh to the device, checks det J > 0
 * at every quadrature point (MFS_EINVAL with the cell id in mfs_last_error),
 * builds the multigrid hierarchy (p-levels k -> p_min, then h-levels by
 * halving n while every n is even and > coarse_min_cells; Sec. 3), the
 * inverse diagonals, the Chebyshev bounds (Lanczos estimate, host readback),
 * and the FP64 coarse-level inverse.  k in [1, 6] (Taylor-Hood: k >= 2).
 * With pressure_offset = 0 the problem is the equal-order SUPG/PSPG
 * Navier-Stokes system of Sec. 5 instead: the hierarchy coarsens the mesh
 * first and the degree afterwards (h-levels, then p-levels down to p_min),
 * every level is equal order, k <= 2 with mg_levels = 1 and k <= 3 without,
 * and the operator data is computed by mfs_set_linearization.
 * Returns a handle owned by the caller, released by mfs_destroy.  Runs on
 * `stream` and synchronises it before returning.
 */
int mfs_setup(const mfs_mesh *mesh, int k, double nu, const mfs_options *opts, void *stream,
              mfs_problem **out);
int mfs_destroy(mfs_problem *p);

/*
 * mfs_setup into a caller-owned device arena (for example a torch uint8
 * CUDA tensor) instead of a library allocation: every device array of the
 * problem (levels, Krylov space, work vectors) is carved from `arena`, which
 * must be 256-byte aligned, hold at least mfs_footprint() bytes (MFS_ENOMEM
 * otherwise) and outlive the problem; mfs_destroy does not free it.  The
 * library still keeps a small pinned readback block and, with graphs, a
 * capture stream per problem, taken from process-wide free lists and
 * returned to them by mfs_destroy (neither frees device memory, so neither
 * waits for other work on the device).  Structured meshes only (mfs_setup's
 * problems); hp and refined-mesh problems allocate their own.
 */
int mfs_setup_arena(const mfs_mesh *mesh, int k, double nu, const mfs_options *opts, void *arena, size_t bytes,
                    void *stream, mfs_problem **out);

/*
 * setup for the hp variant of Sec. 3: velocity degree cell_degree[c] in [2, 6]
 * per cell (host array, n0*n1*n2 entries, lexicographic cells), pressure degree
 * cell_degree[c] - 1, 3D only, Taylor-Hood (pressure_offset = 1).  The space
 * is the continuous one: on a face or edge shared by cells of different degree
 * the trace has the lowest of their degrees (minimum rule), realised by the
 * cell-local maps C_e of eq. (transfer).  Unknowns are numbered by mesh entity:
 * vertices (lexicographic), edges along x, y, z (lexicographic over their index
 * boxes; m-1 unknowns at the interior degree-m GLL points, m = lowest degree of
 * the cells around the edge), faces normal to x, y, z ((m-1)^2 unknowns, lower
 * free axis fastest), cell interiors ((k-1)^3, x fastest); vectors are blocked
 * [u_0 | u_1 | u_2 | p].  Multigrid: hp p-levels with k <- max(k-1, 2) until
 * every degree is 2 (levels 0 .. nhp-1), then the structured degree-2 levels
 * of mfs_setup with the mesh halved (levels nhp ..).  mfs_vmult offers every
 * operator on level 0 and MFS_OP_A on the others; mfs_rhs and the support
 * point queries are not provided (MFS_EUNSUPPORTED).  Jacobi diagonals are
 * computed by applying A to colour indicators (no two unknowns of a colour
 * share a cell).  Returns MFS_EINVAL on a degree outside [2, 6].
 */
int mfs_setup_hp(const mfs_mesh *mesh, const int *cell_degree, double nu, const mfs_options *opts, void *stream,
                 mfs_problem **out);

/* Locally refined mesh of the unit cube: the leaves of octrees over n^3
 * Cartesian base cells.  Leaf c has refinement level level[c] in [0, levels]
 * and index (idx[3c], idx[3c+1], idx[3c+2]) on its level's grid of
 * (n 2^level)^3 cells, i.e. it spans [i, i+1] x [j, j+1] x [m, m+1] / (n 2^level).
 * Host arrays, read during the call only.  The leaves must partition the cube. */
typedef struct mfs_refined_mesh {
  int n;             /* base cells per direction */
  int levels;        /* finest refinement level present, in [0, 4] */
  int64_t ncells;    /* number of leaves */
  const int *level;  /* [ncells] */
  const int *idx;    /* [ncells][3] */
} mfs_refined_mesh;

/*
 * setup on a locally refined mesh (Sec. 5: the stabilised Navier-Stokes
 * problem on meshes with hanging nodes): equal-order Q_k/Q_k, k in {1, 2}
 * (opts->pressure_offset must be 0).  The space is the continuous one: a node
 * of a finer cell that lies on a face or edge of a coarser neighbour without
 * being one of its nodes (a hanging node) takes the neighbour's interpolant
 * there, realised by the cell-local constraint maps C_e of eq. (transfer).
 * Unknowns: every other node position, numbered in lexicographic order of
 * position (x fastest); vectors blocked [u_0 | u_1 | u_2 | p] with
 * n_u = n_p = number of unknowns; velocity unknowns on the boundary of the
 * cube are Dirichlet unknowns.
 *
 * opts->mg_levels = 0: level 0 only.  opts->mg_levels = 1: the monolithic
 * multigrid of Sec. 5 with global coarsening: level j + 1 is level j with
 * every family of eight leaves replaced by its parent, down to the uniform
 * base mesh; the levels above the base (0 .. G-1, G = finest refinement level
 * present, which must be >= 1) have their own Jacobian and Jacobi diagonal
 * (by colour probes), and the base mesh and its coarsenings are the levels
 * G .. of the structured Navier-Stokes hierarchy of mfs_setup (Cartesian
 * base cube).  Transfers between GC levels: the coarse field at the fine
 * unknowns (Dirichlet velocity rows and columns zero, pressure
 * unconstrained); restriction is the transpose.
 *
 * Offers mfs_set_linearization (u0: 3 n_u values at the level-0 unknowns,
 * copied at the coarse unknowns level by level), mfs_vmult with
 * MFS_OP_NS_JACOBIAN on every level, mfs_n_dofs, mfs_n_levels,
 * mfs_level_info, mfs_support_points (deg = k: the level-0 unknowns'
 * coordinates), and with multigrid mfs_diagonal, mfs_prolongate_add,
 * mfs_restrict, mfs_vcycle, mfs_precondition (one V-cycle) and the solve
 * calls; mfs_rhs, the quadrature-point queries and the lambda calls return
 * MFS_EUNSUPPORTED.  MFS_EINVAL when the leaves are out of range, overlap or
 * leave a gap, or for multigrid on an unrefined mesh; MFS_EUNSUPPORTED for
 * other degrees or options.  The hanging-node maps are built on the host
 * (sort of all cell-node positions) and copied to the device; `stream` is
 * synchronised before returning.
 */
int mfs_setup_refined(const mfs_refined_mesh *mesh, int k, double nu, const mfs_options *opts, void *stream,
                      mfs_problem **out);

/* Host only (no device call): sizes of the refined-mesh space that
 * mfs_setup_refined would build, without building it on the device.
 * n_unknowns = unknowns per component (n_u = n_p), n_hanging = hanging node
 * positions.  Validates the leaves like mfs_setup_refined (MFS_EINVAL,
 * MFS_EUNSUPPORTED). */
int mfs_refined_count(const mfs_refined_mesh *mesh, int k, int64_t *n_unknowns, int64_t *n_hanging);

/*
 * Host only: the parallel efficiency metrics of Sec. 2 (Tables tab:tc and
 * tab:fpc) for the two multigrid level hierarchies of a refined mesh, global
 * coarsening (the library's levels) and local smoothing (all cells of each
 * refinement level), when every level is spread over `nprocs` processes:
 *   eta[0], eta[1]: eta_w, eta_v of global coarsening;
 *   eta[2], eta[3]: eta_w, eta_v of local smoothing.
 * eta_w = sum_l n_l / (P sum_l max_p n_{l,p}) (work against the busiest
 * process per level), eta_v = the fraction of fine cells owned by the
 * process that owns the coarse cell they transfer to.  Partitions: the
 * leaves and every global-coarsening level are cut into P contiguous chunks
 * of the Morton curve; a local-smoothing parent belongs to the owner of its
 * first child.  MFS_EINVAL on bad cells.
 */
int mfs_refined_mg_metrics(const mfs_refined_mesh *mesh, int nprocs, double *eta);

/* Sizes at level `level` (0 = finest): scalar velocity nodes per component and
 * pressure nodes (0 on levels without pressure; n_u on every level of a
 * Navier-Stokes problem). */
int mfs_n_dofs(const mfs_problem *p, int level, int64_t *n_u, int64_t *n_p);
int mfs_n_levels(const mfs_problem *p, int *n_levels);
/* degree and cells per direction of a level */
int mfs_level_info(const mfs_problem *p, int level, int *k, int *n);

/* Physical coordinates of the scalar nodes of degree `deg` (host buffer of
 * (deg n0 + 1)(deg n1 + 1)(..) x dim doubles). */
int mfs_support_points(const mfs_problem *p, int deg, double *host_xyz);
/* Physical coordinates of the Gauss points of every cell, [n_cells][(k+1)^dim][dim]
 * in cell order and lexicographic point order (host buffer). */
int mfs_quadrature_points(const mfs_problem *p, double *host_xyz);

/* Same coordinates written to a device buffer (FP64, same layout), enqueued on
 * `stream`. */
int mfs_quadrature_points_device(const mfs_problem *p, double *dev_xyz, void *stream);

/*
 * dst = op(src) on level `level` (0 = finest) in precision `prec`.
 * Lengths: STOKES and NS_JACOBIAN: dim*n_u + n_p -> same; A, MASS_U: dim*n_u -> dim*n_u;
 * B: n_p -> dim*n_u; BT: dim*n_u -> n_p; MASS_P: n_p -> n_p.
 * STOKES, B, BT, MASS_P need a level with pressure (level 0).  NS_JACOBIAN
 * works on every level of a Navier-Stokes problem after
 * mfs_set_linearization (the level's own rediscretised Jacobian).  Enqueue
 * only.
 */
int mfs_vmult(mfs_problem *p, int op, int prec, int level, void *dst, const void *src, void *stream);

/* dst = diag(A) on `level` for one velocity component (n_u entries; 1 on
 * Dirichlet rows), FP64.  Navier-Stokes problem: the diagonal of the
 * level's Jacobian, (dim+1)*n_u entries (after mfs_set_linearization). */
int mfs_diagonal(mfs_problem *p, int level, double *dst, void *stream);

/* Chebyshev bound used by the smoother on `level` (after setup). */
int mfs_get_lambda(const mfs_problem *p, int level, double *lambda_max);
/* Override the Chebyshev bound on `level` (for parity checks with a fixed value). */
int mfs_set_lambda(mfs_problem *p, int level, double lambda_max);

/*
 * dst = one multigrid V-cycle on the velocity block A applied to src
 * (approximates A^{-1} src, Sec. 3), initial guess 0 on free rows and src on
 * Dirichlet rows.  Vectors dim*n_u long in precision `prec`.  Navier-Stokes
 * problem: one monolithic V-cycle on J (Sec. 5; damped Jacobi relaxation,
 * pinned direct coarse solve, see mfs_set_linearization) on full vectors.
 * Enqueue only.
 */
int mfs_vcycle(mfs_problem *p, int prec, void *dst, const void *src, void *stream);

/* Multigrid transfer between level `fine` and level fine+1 (Sec. 2
 * eq. (transfer)): dst_fine += P src_coarse (prolongate) or
 * dst_coarse = P^T src_fine (restrict).  Velocity vectors of the two levels;
 * full vectors of a Navier-Stokes problem, whose pressure component is
 * transferred without constraints. */
int mfs_prolongate_add(mfs_problem *p, int prec, int fine, void *dst_fine, const void *src_coarse, void *stream);
int mfs_restrict(mfs_problem *p, int prec, int fine, void *dst_coarse, const void *src_fine, void *stream);

/*
 * dst = P^{-1} src, the block-triangular preconditioner of eq. (stokes_block):
 * y_p = -(nu^{-1} M_p)^{-1} r_p by `schur_iterations` Jacobi-PCG steps,
 * y_u = Vcycle(r_u - B y_p).  Full-length vectors in precision `prec`.
 * Navier-Stokes problem: one monolithic V-cycle (as mfs_vcycle).
 */
int mfs_precondition(mfs_problem *p, int prec, void *dst, const void *src, void *stream);

/*
 * Right-hand side of the constrained Stokes system: b_i = (f, phi_i) minus the
 * unconstrained operator applied to the lifting on free rows, b_i = u_D on
 * Dirichlet rows, pressure rows minus B^T of the lifting.
 *   f_qp: device FP64 [n_cells][(k+1)^dim][dim] forcing at the Gauss points
 *         (mfs_quadrature_points order);
 *   u_dirichlet: device FP64 dim*n_u blocked velocity values at the support
 *         points (only Dirichlet entries are read);
 *   b: device FP64, full length.
 */
int mfs_rhs(mfs_problem *p, const double *f_qp, const double *u_dirichlet, double *b, void *stream);

/*
 * Solve K x = b by FGMRES(restart) with the block preconditioner in
 * opts->precond_precision (FP32 preconditioner inside FP64 FGMRES, or all
 * FP64), x0 = lifting of b's Dirichlet rows.  b, x: device FP64 full length.
 * Host-synchronous (one readback per iteration).  The pressure is returned
 * with zero mass-weighted mean.  MFS_ENOCONV if rtol is not reached within
 * maxit (x holds the last iterate, info filled).  Navier-Stokes problem:
 * K = the Jacobian J at the linearisation point, preconditioner = one
 * monolithic V-cycle; J is singular (constant pressures), so b must have
 * pressure rows summing to zero (true for b = J y); the pressure is returned
 * with zero nodal mean.
 * Of `opts` (NULL: the setup options) a solve reads rtol, maxit,
 * precond_precision and graphs; the restart length, the smoother (Chebyshev
 * degree and range, relaxation), the Schur iterations and the hierarchy are
 * those given to mfs_setup, whatever the other fields hold.
 */
int mfs_solve(mfs_problem *p, const double *b, double *x, const mfs_options *opts, mfs_solve_info *info,
              void *stream);

/*
 * Resumable form of mfs_solve for a request loop that interleaves many
 * problems: mfs_solve_begin enqueues the start of a solve on `stream`;
 * mfs_solve_advance checks without blocking whether the last enqueued
 * iteration has finished and, if so, reads its residual and enqueues the next
 * one.  *done becomes 1 when the solve has converged or hit maxit (then
 * info is filled and x holds the result).  Returns MFS_OK while progressing.
 */
int mfs_solve_begin(mfs_problem *p, const double *b, double *x, const mfs_options *opts, void *stream);
int mfs_solve_advance(mfs_problem *p, int *done, mfs_solve_info *info);

/*
 * Serving step over many resumable solves (each begun with mfs_solve_begin
 * on its own stream): for every listed problem whose last enqueued iteration
 * has finished, read its residual and enqueue its next FGMRES iteration, as
 * mfs_solve_advance does, without blocking on the others.  The system
 * operator applications (w = K z_j, FP64) of all Taylor-Hood Q2/Q1 problems
 * on structured 3D meshes that step in this call are one grouped launch pair
 * (brick kernel and face combine over all their cells, up to 16 problems per
 * pair) on `stream`, ordered after each problem's preconditioner and before
 * its Gram-Schmidt by events; the preconditioners (the recorded FP32 graph)
 * and Gram-Schmidt run on the problems' own streams, as do all the steps of
 * other problems.  Results are the same as with mfs_solve_advance.
 * done[i] = 1 (and infos[i] filled, when infos is not NULL) once problem i
 * has converged or reached maxit.  The problems must be distinct and used by
 * no other host thread meanwhile.
 */
int mfs_batch_step(mfs_problem **ps, int n, void *stream, int *done, mfs_solve_info *infos);

/*
 * Navier-Stokes linearisation point (Sec. 5) of a problem set up with
 * pressure_offset = 0.  u0: device FP64 dim*n_u nodal velocity (every node,
 * boundary included; the pressure of the point is 0).  dt > 0: BDF2 step,
 * mass shift alpha = 3/(2 dt).  newton = 1: full Gateaux derivative;
 * 0: Oseen (drops du.grad u0 and (R(u0), du.grad v)).
 * Computes, on every level, u0 at the level's nodes (copied from the fine
 * nodes they coincide with), the per-Gauss-point data u0, grad u0,
 * R(u0) = u0.grad u0 - nu Lap u0 and the frozen SUPG/PSPG parameter
 * delta_1 = [(2/dt)^2 + (2|u0|/h_K)^2 + 9 (4 nu/h_K^2)^2]^(-1/2),
 * h_K = |K|^(1/dim)/k (FP64 and FP32 copies); with mg_levels also the
 * diagonals of J (by applying J to node colourings) and the FP64 inverse of
 * the coarsest J with pressure node 0 pinned (its row and column replaced by
 * the identity and its right-hand side entry ignored).  Host-synchronous on
 * `stream`.  MFS_EINVAL for a Taylor-Hood problem or dt <= 0.
 */
int mfs_set_linearization(mfs_problem *p, const double *u0, double dt, int newton, void *stream);

/*
 * Space-time Kronecker operator of the transient Stokes equations on one time
 * slab (Sec. 4 eq. (proceedings-kronecker)):
 *   dst = (G (x) M + tau I_Q (x) A) src
 * on stage-major vectors [x_1 | .. | x_Q], each x_q a full Stokes vector of
 * dim n_u + n_p entries (level 0), M the Stokes block mass (velocity mass,
 * zero pressure block), A the Stokes operator of mfs_vmult(MFS_OP_STOKES).
 * Every stage carries the spatial constraints: dst_q = src_q on the velocity
 * Dirichlet rows, Dirichlet source values ignored elsewhere.
 *   G: host Q x Q row-major (G_Q = M_Q^{-1} A_Q^tau of the time
 *      discretisation), 1 <= Q <= 8;  tau > 0: the slab length;
 *   work: device scratch of Q dim n_u entries in the precision `prec`.
 * Structured Taylor-Hood problems.  Enqueue only.
 */
int mfs_st_vmult(mfs_problem *p, int Q, const double *G, double tau, int prec, void *dst, const void *src, void *work,
                 void *stream);

/*
 * Stage mixing on stage-major level-0 vectors: dst_i = sum_j C[i][j] src_j
 * (i < q_out, j < q_in, C host row-major q_out x q_in, q_out, q_in <= 8),
 * entry by entry over the full Stokes vector: the temporal transfers of
 * Sec. 4 (P_tau for prolongation, P_tau^T for restriction) applied per
 * spatial unknown.  dst and src must not overlap.  Enqueue only.
 */
int mfs_st_stage_transfer(mfs_problem *p, int q_out, int q_in, const double *C, int prec, void *dst, const void *src,
                          void *stream);

/*
 * hp space-time multigrid (hp-STMG) of Sec. 4 for the Kronecker stage system
 * K x = (G (x) M + tau I_Q (x) A) x = b on one slab with DG(kt) in time
 * (Q = kt + 1 stages on the Gauss points of the slab) and Taylor-Hood
 * Q_k / Q_{k-1} in space: FGMRES preconditioned by one V-cycle.
 * Levels (the paper's two coarsening rules, no geometric coarsening in time):
 * spatial degree k -> 2, then h-coarsening while every n is even and larger
 * than 2, then the temporal degree kt -> 0 on the coarsest mesh.  Transfers: per stage the
 * constrained velocity and unconstrained pressure Lagrange transfers
 * (restriction: their transpose); in time the coarse DG polynomial at the
 * fine nodes, restricted by M_c^{-1} P^T M_f.  Smoother: relax_steps
 * additive Schwarz steps x <- x + relax_omega B (b - K x) before and after
 * the coarse correction, B the sum of the exact inverses of the vertex-star
 * space-time patches (every velocity component at the velocity nodes
 * |i - k v| < k and the pressure at the nodes |j - (k-1) v| < k-1 of
 * vertex v, all Q stages, Dirichlet rows left out) weighted by the inverse
 * number of patches holding each unknown.  Coarsest level: the dense inverse
 * with the first pressure node of every stage pinned to zero.
 *
 * mfs_stmg_setup: structured meshes (mfs_mesh, host vertices); k = 2, 3 in
 * 2D and k = 2 in 3D, with kt <= 2 (patches of at most 177 unknowns in 2D,
 * 246 in 3D); nu, tau > 0, relax_steps in [0, 16].  Builds every level on the device (library-owned memory;
 * MFS_EUNSUPPORTED outside these cases); synchronous.
 * mfs_stmg_levels: number of levels, and for `level` its cells n[dim],
 * velocity degree k, stages Q and vector length Q (dim n_u + n_p) (any
 * output may be NULL).
 * mfs_stmg_vmult: dst = K_level src (stage-major device FP64 vectors of that
 * length; every stage carries the Dirichlet rows as identity).  Enqueue
 * only.
 * mfs_stmg_vcycle: dst = one V-cycle applied to src on level 0, in precision
 * prec (MFS_FP64 or MFS_FP32: device vectors of that type; the FP32 V-cycle
 * runs every level in FP32 with FP32 copies of the patch inverses and the
 * FP64 coarse inverse); x starts from b on the Dirichlet rows and 0
 * elsewhere.  Enqueue only; calls on one handle must not overlap.
 * mfs_stmg_solve: x = FGMRES(30) in FP64 with one V-cycle in precision prec
 * per iteration, from x = 0 to ||b - K x|| <= rtol ||b|| (device FP64 b and
 * x of the level-0 length; the constant pressure of each stage is in the
 * kernel of K: b must be consistent).  Synchronous on the setup stream;
 * MFS_ENOCONV with `info` filled when maxit iterations do not reach rtol.
 */
typedef struct mfs_stmg mfs_stmg;
int mfs_stmg_setup(const mfs_mesh *mesh, int k, int kt, double nu, double tau, int relax_steps, double relax_omega,
                   void *stream, mfs_stmg **out);
int mfs_stmg_levels(const mfs_stmg *m, int level, int *n_levels, int *n, int *k, int *Q, int64_t *length);
int mfs_stmg_vmult(mfs_stmg *m, int level, double *dst, const double *src, void *stream);
int mfs_stmg_vcycle(mfs_stmg *m, int prec, void *dst, const void *src, void *stream);
int mfs_stmg_solve(mfs_stmg *m, const double *b, double *x, double rtol, int maxit, int prec, mfs_solve_info *info);
int mfs_stmg_destroy(mfs_stmg *m);

/*
 * General Navier-Stokes state (Sec. 5, BDF2): the linearisation at
 * x0 = [u0 | p0] (device FP64, full length (dim+1) n_u; velocity with its
 * boundary values) with the BDF2 history u_hist = (4 u^n - u^{n-1}) / 3
 * (device FP64, dim n_u; NULL: u_hist = u0), so that the time derivative is
 * alpha (u - u_hist), alpha = 3/(2 dt), and the strong residual at the state
 * is R(u0, p0) = alpha (u0 - u_hist) + u0.grad u0 + grad p0 - nu Lap u0
 * (mfs_set_linearization is the case p0 = 0, u_hist = u0).  The Jacobian of
 * mfs_vmult(MFS_OP_NS_JACOBIAN) is then the Gateaux derivative of the
 * residual below at x0 (newton = 1) or its Oseen part (newton = 0).
 * keep_delta = 1 keeps the SUPG/PSPG parameter delta_1 of the previous
 * linearisation on every level (frozen during a time step), 0 recomputes it
 * from u0 as mfs_set_linearization does.  Computes the multigrid data too
 * (with mg_levels).  Host-synchronous; drops the recorded preconditioner.
 */
int mfs_set_linearization_point(mfs_problem *p, const double *x0, const double *u_hist, double dt, int newton,
                                int keep_delta, void *stream);

/*
 * F = the residual F_NS + F_SUPG + F_PSPG of Sec. 5 at the state of the last
 * linearisation, tested with every basis function:
 *   (alpha (u - u_hist) + u.grad u, v) + (nu grad u, grad v) - (p, div v)
 *   + (div u, q) + sum_K delta_1 (R(u, p), u.grad v + grad q)_K,
 * f = 0, delta_1 as stored.  Velocity Dirichlet rows of F are 0 (the state
 * carries the boundary values).  F: device FP64, (dim+1) n_u.  Enqueue only.
 */
int mfs_ns_residual(mfs_problem *p, double *F, void *stream);

typedef struct mfs_newton_options {
  int max_newton;        /* Newton iterations per step (20) */
  double rtol;           /* stop when ||F(x_k)||_2 <= max(rtol ||F(x_0)||_2, atol) (1e-8) */
  double atol;           /* (0) */
  double linear_rtol;    /* FGMRES relative tolerance of each correction J dx = -F (1e-6); a
                            correction is never solved below a tenth of the Newton target:
                            the tolerance used is max(linear_rtol, 0.1 target / ||F(x_k)||) */
  int linear_maxit;      /* FGMRES iterations per correction (200) */
  int precond_precision; /* MFS_FP32 (default) or MFS_FP64 multigrid preconditioner */
} mfs_newton_options;

typedef struct mfs_newton_info {
  int newton_iterations; /* corrections applied */
  int linear_iterations; /* FGMRES iterations over all corrections */
  int linear_failures;   /* corrections whose FGMRES stopped at linear_maxit */
  int status;            /* MFS_OK or MFS_ENOCONV */
  double res0, res;      /* ||F||_2 at the initial guess and at the result */
  double seconds;
} mfs_newton_info;

void mfs_default_newton_options(mfs_newton_options *opts);

/*
 * One BDF2 time step of the stabilised Navier-Stokes equations (Sec. 5) by
 * Newton's method, each correction solved by FGMRES with one monolithic
 * multigrid V-cycle as preconditioner (the Newton-Krylov method of Sec. 5).
 *   u_n, u_nm1: device FP64 velocities (dim n_u) of the last two steps (the
 *     first step passes the initial velocity twice);
 *   x: device FP64 (dim+1) n_u; on entry the initial guess, whose velocity
 *     Dirichlet rows are the boundary values of the new time level (kept);
 *     on exit the new state, pressure with zero nodal mean.
 * delta_1 is frozen at u_n for the whole step, so each Jacobian is the exact
 * derivative of the residual the step solves.  The boundary data must have
 * zero net flux (the pressure rows of F then sum to zero, as the singular
 * Jacobian needs).  Needs mg_levels = 1.  Host-synchronous.  MFS_ENOCONV
 * when Newton does not reach its tolerance (x holds the last iterate, info
 * filled).
 */
int mfs_ns_bdf2_step(mfs_problem *p, const double *u_n, const double *u_nm1, double *x, double dt,
                     const mfs_newton_options *opts, mfs_newton_info *info, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the 3D
 * Taylor-Hood Q2/Q1 Stokes operator, dst = K src, on a structured mesh of
 * n[0] x n[1] x n[2] cells, without a problem handle and without any
 * allocation.  It is the operator mfs_vmult(MFS_OP_STOKES, level 0) applies
 * for a problem set up by mfs_setup with dim = 3, k = 2, Taylor-Hood and the
 * same vertices and nu, computed by the same kernels (results are identical).
 *   n:        host array of 3 cell counts, each >= 1;
 *   vertices: device, [(n0+1)(n1+1)(n2+1)][3] coordinates, x fastest, in
 *             the precision `prec` (FP64: double, FP32: float); every cell
 *             must have det J > 0 (not checked here: mfs_setup checks it);
 *   nu > 0;  prec: MFS_FP64 or MFS_FP32;
 *   src, dst: device, 3 Nv + Np entries, Nv = (2n0+1)(2n1+1)(2n2+1),
 *             Np = (n0+1)(n1+1)(n2+1), blocked [u_0 | u_1 | u_2 | p] as
 *             everywhere; non-aliasing; Dirichlet rows dst = src.
 * Scratch: a library-owned static device array of MFS_NOALLOC_SCRATCH_BYTES
 * per GPU (held until the process ends), which bounds the mesh: one brick of
 * 8 x 4 x 2 cells needs 19,440 bytes in FP64 and 9,720 in FP32, so at most
 * 1,726 bricks (FP64) or 3,452 (FP32), e.g. 32^3 cells (512 bricks).  Larger
 * meshes return MFS_EINVAL before anything is enqueued.  Calls on one GPU
 * share its array: calls that overlap (other streams, other host threads)
 * race on it; calls ordered on one stream do not.  Enqueue only.
 */
#define MFS_NOALLOC_SCRATCH_BYTES (32u << 20)
int mfs_stokes_vmult_noalloc(const int n[3], const void *vertices, double nu, int prec, void *dst, const void *src,
                             void *stream);

#ifdef __cplusplus
}
#endif
#endif
