/*
 * mfsem.h -- C ABI of the matrix-free spectral-element monodomain operator for
 * AMD Instinct MI355X (gfx950).
 *
 * What it computes (arXiv 2205.05136):
 *   A = alpha*M + K(sigma), the implicit operator of the monodomain linear
 *   system (Section 3, the linear system; the paper has alpha = 3/(2 dt) with
 *   chi = Cm = 1), on conforming hexahedral meshes of degree p, with the
 *   diffusion tensor sigma = sigma_l f f^T + sigma_t s s^T + sigma_n n n^T
 *   (Section 2), applied matrix-free with sum factorisation (Section 4.1),
 *   either with GLL quadrature collocated with the nodes (SEM-NI, diagonal mass)
 *   or with Legendre-Gauss quadrature (SEM) (Section 3); a preconditioned CG
 *   (Section 4) with a matrix-free geometric multigrid V-cycle whose smoother
 *   is Chebyshev-Jacobi with a CG/Lanczos estimate of lambda_max, and whose
 *   levels are linked by p- and octree h-interpolation and its transpose
 *   (Section 4.3; parameters from Section 5).
 *
 * Conventions for every entry point:
 *   - Array arguments marked [device] are HIP device pointers owned by the
 *     caller; [host] marks host memory.  Scalars are passed by value.
 *   - The library never allocates device memory.  Objects that need device
 *     storage take a caller-provided workspace `ws` of at least the size the
 *     matching *_workspace_bytes query returns, aligned to 256 bytes; the
 *     object keeps pointers into it, so `ws` must outlive the object.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call is enqueued on `stream` and returns without synchronising,
 *     except those marked [sync], which wait for `stream` before returning.
 *   - Return value: MFSEM_OK or a negative mfsem_status.  On failure
 *     mfsem_last_error() returns a message (thread-local, valid until the next
 *     failing call on the same thread).  Arguments are validated on the host
 *     before any launch; a failed call leaves outputs untouched unless stated.
 *   - Vectors with a batch dimension are laid out [batch][n_dof], contiguous.
 *     An operator may have no elements (A is then the zero matrix on its
 *     nodes) and no DOFs; the vectors of an operator with n_dof == 0 have no
 *     entries and may be NULL in mfsem_op_apply*, mfsem_op_diagonal and
 *     mfsem_pcg*.
 *   - Local node numbering inside an element is i = a + P*(b + P*c), P = p+1,
 *     a along the first reference axis (fastest).
 */
#ifndef MFSEM_H
#define MFSEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MFSEM_ABI_VERSION 9
#define MFSEM_MAX_P 8

typedef enum {
  MFSEM_OK = 0,
  MFSEM_EINVAL = -1,        /* invalid argument (null pointer, size, range, alignment) */
  MFSEM_EUNSUPPORTED = -2,  /* valid but not implemented (e.g. a degree above MFSEM_MAX_P) */
  MFSEM_EGEOMETRY = -3,     /* det J <= 0 at some quadrature point (message names it) */
  MFSEM_EDEVICE = -4,       /* a HIP runtime or launch error */
  MFSEM_ENOCONV = -5,       /* iteration limit reached before the tolerance */
  MFSEM_EBREAKDOWN = -6,    /* p^T A p <= 0 or (r, z) <= 0 in (P)CG */
  MFSEM_ENONFINITE = -7     /* NaN or Inf met in a residual norm */
} mfsem_status;

typedef enum { MFSEM_GLL = 0, /* SEM-NI */ MFSEM_GAUSS = 1 /* SEM */ } mfsem_quad;
typedef enum { MFSEM_F64 = 0, MFSEM_F32 = 1 } mfsem_dtype;
typedef enum { MFSEM_TRANSFER_P = 0, MFSEM_TRANSFER_H = 1 } mfsem_transfer_kind;
/* Where the FP64 stiffness apply takes W|J| J^{-1} sigma J^{-T} from (Section 4:
 * the Jacobian may be cached or evaluated in the cell loop).  On MI355X the
 * stored values are faster at every degree (the on-the-fly kernel moves about
 * 40% fewer bytes but is bound by its FP64 arithmetic and LDS reads), so AUTO
 * selects them. */
typedef enum {
  MFSEM_GEOM_AUTO = 0,      /* the library's choice: stored */
  MFSEM_GEOM_STORED = 1,    /* the values stored at create */
  MFSEM_GEOM_ONTHEFLY = 2   /* on the fly; EINVAL if the operator is not eligible */
} mfsem_geometry;

typedef struct mfsem_op mfsem_op;
typedef struct mfsem_mg mfsem_mg;

/* ABI version (MFSEM_ABI_VERSION of the built library). */
int mfsem_abi_version(void);

/* Message of the last failing call on this thread ("" if none). [host] */
const char* mfsem_last_error(void);

/* ------------------------------------------------------------------------ */
/* Mesh setup: structured boxes (Section 3: conforming hexahedral meshes and
 * the Q_p space with nodes at the GLL points of each element).
 *
 * The (p*n[0]+1) x (p*n[1]+1) x (p*n[2]+1) node lattice has global index
 * g = I + NX*(J + NY*K); element (ex,ey,ez) has index ex + n0*(ey + n1*ez).
 * Nodes inside an element sit at the GLL points of the element's edges.
 * If shear_amp != 0 every node (x,y,z) moves to (x+d, y+d, z+d) with
 * d = shear_amp * (length[0]/n[0]) * sin(2*pi*(x - origin[0])/length[0]).
 * If fiber != 0 the fiber at a node is (cos t, sin t, 0) with t going linearly
 * from theta0 at z = origin[2] to theta1 at z = origin[2] + length[2]
 * (undeformed z).                                                            */
typedef struct {
  int32_t p;            /* 1..MFSEM_MAX_P */
  int32_t n[3];         /* elements per axis, >= 1 */
  double origin[3];
  double length[3];     /* > 0 */
  double shear_amp;
  int32_t fiber;        /* 0 or 1 */
  double theta0, theta1;/* radians */
} mfsem_box_desc;

/* Element and node counts of a box. [host] */
mfsem_status mfsem_box_counts(const mfsem_box_desc* box, int64_t* n_elem, int64_t* n_dof);

/* Fill elem_dof [n_elem][(p+1)^3] (int32), xyz [n_dof][3] and, if box->fiber,
 * fiber [n_dof][3] (may be NULL otherwise).  All [device], caller-sized from
 * mfsem_box_counts.  EINVAL if n_dof exceeds INT32_MAX.                     */
mfsem_status mfsem_box_generate(const mfsem_box_desc* box, int32_t* elem_dof, double* xyz,
                                double* fiber, void* stream);

/* Octree parents for a box of n_fine[3] elements (all even) coarsened to
 * n_fine/2: parent[e] = coarse element containing fine element e, child[e] =
 * cx | cy<<1 | cz<<2 with c* the fine element's offset (0/1) inside its parent
 * along each axis.  [device] int32 parent[n_elem_fine], int8 child[n_elem_fine]. */
mfsem_status mfsem_box_parents(const int32_t n_fine[3], int32_t* parent, int8_t* child,
                               void* stream);

/* Nodes of derived meshes on arbitrary conforming meshes (Section 4.3: the
 * octree hierarchy refined from a coarse mesh T0, whose children keep their
 * parent's geometry, and the lower-degree levels of the same elements).  The
 * parent mesh has degree p (1..MFSEM_MAX_P): elem_dof [n_elem][(p+1)^3] int32
 * (local index a + (p+1)(b + (p+1)c)), xyz and fiber [n_nodes][3] FP64 (fiber
 * may be NULL).  Each element carries an M^3 lattice of reference points:
 *   refine: M = 2p + 1, the GLL points of degree p of the two halves of
 *           [-1, 1] along each axis (the nodes of the element's 8 children);
 *   degree: M = pc + 1, the GLL points of degree pc (1..MFSEM_MAX_P).
 * New node g lies at lattice point loc[g] = I + M (J + M K) of element
 * elem[g] (any element holding it; the numbering of the new nodes, i.e. which
 * lattice points of which elements coincide, is the caller's).  Its position
 * is the parent's isoparametric map there,
 *   xyz_new[g] = sum_{a,b,c} l_a(xi_I) l_b(xi_J) l_c(xi_K) xyz[elem_dof[e][a,b,c]],
 * with l the degree-p Lagrange basis on the GLL nodes, and fiber_new[g] the
 * same interpolation of the fiber (not normalised; the operator normalises it
 * at its quadrature points).  fiber_new is written when fiber is given.
 * elem, loc [device] int32 [n_new]; xyz_new, fiber_new [device] [n_new][3].
 * EINVAL for p or pc out of range or a NULL array with n_new > 0; an element,
 * lattice point or node index out of range gives NaN for that node (nothing
 * is read out of bounds).                                                     */
mfsem_status mfsem_mesh_refine_nodes(int32_t p, int64_t n_elem, const int32_t* elem_dof,
                                     int64_t n_nodes, const double* xyz, const double* fiber,
                                     int64_t n_new, const int32_t* elem, const int32_t* loc,
                                     double* xyz_new, double* fiber_new, void* stream);
mfsem_status mfsem_mesh_degree_nodes(int32_t p, int64_t n_elem, const int32_t* elem_dof,
                                     int64_t n_nodes, const double* xyz, const double* fiber,
                                     int32_t pc, int64_t n_new, const int32_t* elem,
                                     const int32_t* loc, double* xyz_new, double* fiber_new,
                                     void* stream);

/* ------------------------------------------------------------------------ */
/* Operator A = alpha*M + K(sigma).
 *
 * DOF space: degree p, numbering elem_dof.  Geometry: the isoparametric map of
 * degree map_p through map_xyz at the nodes map_elem_dof (a p-coarsened
 * multigrid level keeps the fine map with a coarser DOF space).  At each
 * quadrature point the fiber (and sheet) are interpolated with the map basis
 * and normalised (the sheet is made orthogonal to the fiber, n = f x s); sigma
 * is sigma_t I + (sigma_l - sigma_t) f f^T without a sheet, the full
 * orthotropic tensor with one, and sigma_t I without a fiber.
 * Set-up computes and stores, in FP64 (and/or FP32), per element and
 * quadrature point, G = W |J| J^{-1} sigma J^{-T} (6 values) and W |J|.      */
typedef struct {
  int32_t p;                   /* DOF degree, 1..MFSEM_MAX_P */
  int32_t quad;                /* mfsem_quad */
  int32_t nq1d;                /* points per axis: GLL needs p+1; GAUSS p+1..p+3; 0 = p+1 */
  int64_t n_elem;
  int64_t n_dof;               /* number of global DOFs (<= INT32_MAX) */
  const int32_t* elem_dof;     /* [device] [n_elem][(p+1)^3]; referenced until destroy */
  int32_t map_p;               /* geometry degree, 1..MFSEM_MAX_P (0 = p) */
  const int32_t* map_elem_dof; /* [device] [n_elem][(map_p+1)^3]; NULL = elem_dof (map_p == p) */
  int64_t n_map_nodes;         /* rows of map_xyz / fiber / sheet */
  const double* map_xyz;       /* [device] [n_map_nodes][3]; referenced until destroy */
  const double* fiber;         /* [device] [n_map_nodes][3] or NULL; referenced until destroy */
  const double* sheet;         /* [device] [n_map_nodes][3] or NULL (needs fiber) */
  const double* sigma;         /* [device] [batch][n_elem][3] (sigma_l, sigma_t, sigma_n) or NULL */
  double sigma_const[3];       /* used when sigma == NULL */
  int32_t batch;               /* >= 1 parameter sets; vectors become [batch][n_dof] */
  double alpha;                /* mass coefficient, >= 0 */
  int32_t store_f64;           /* build FP64 geometry (needed by FP64 calls) */
  int32_t store_f32;           /* build FP32 geometry (needed by FP32 calls) */
  int32_t lattice[3];          /* elements per axis when elem_dof is the structured box
                                  numbering of mfsem_box_generate (checked at create;
                                  EINVAL if it is not), enabling the brick kernels;
                                  {0,0,0} for any other mesh                           */
  int32_t geometry;            /* mfsem_geometry.  On the fly, the FP64 apply recomputes
                                  J from the lattice's map_xyz and G from the fiber and
                                  sigma at every point instead of reading the stored G
                                  (48 bytes per point -> 48 bytes per node); eligible:
                                  structured lattice, GLL, p <= 6, map = DOF nodes
                                  (map_p == p, map_elem_dof NULL or elem_dof,
                                  n_map_nodes == n_dof), no sheet, store_f64.  FP32 calls,
                                  the diagonal, the mass and the gradient always use the
                                  stored values.                                       */
} mfsem_op_desc;

/* Workspace an operator needs. [host] */
mfsem_status mfsem_op_workspace_bytes(const mfsem_op_desc* d, size_t* bytes);

/* Create an operator: validates `d`, runs the geometry kernel and checks
 * det J > 0 everywhere (EGEOMETRY names the first bad element and point).
 * sigma is read during this call only.  [sync]                               */
mfsem_status mfsem_op_create(const mfsem_op_desc* d, void* ws, size_t ws_bytes, void* stream,
                             mfsem_op** out);

/* Release the host handle (NULL-safe); the workspace belongs to the caller. */
mfsem_status mfsem_op_destroy(mfsem_op* op);

/* Change alpha (host-side, takes effect for later calls). */
mfsem_status mfsem_op_set_alpha(mfsem_op* op, double alpha);

/* Replace the per-element conductivities [device][batch][n_elem][3] and
 * recompute the stored geometry. [sync]                                      */
mfsem_status mfsem_op_set_sigma(mfsem_op* op, const double* sigma, void* stream);

/* y = A x for every batch member; x, y [device][batch][n_dof] of `dtype`.
 * x and y must not overlap.  (Section 4: the matrix-vector product inside
 * CG; Alg. 1's cell loop, with the sum factorisation of Section 4.1.)        */
mfsem_status mfsem_op_apply(const mfsem_op* op, int32_t dtype, const void* x, void* y,
                            void* stream);

/* y += A x: the same operator kernel without clearing y first (one launch;
 * the global sum is an atomic add, so y may be any vector to add to).       */
mfsem_status mfsem_op_apply_add(const mfsem_op* op, int32_t dtype, const void* x, void* y,
                                void* stream);

/* y = M x (the mass matrix alone, same quadrature). */
mfsem_status mfsem_op_apply_mass(const mfsem_op* op, int32_t dtype, const void* x, void* y,
                                 void* stream);

/* d = diag(A) [device][batch][n_dof] (the point-Jacobi part of the
 * Chebyshev smoother, Section 4.3).                                          */
mfsem_status mfsem_op_diagonal(const mfsem_op* op, int32_t dtype, void* d, void* stream);

/* g[b][e][c] = scale * w_b^T (dA/dsigma_{e,c}) u_b for c = (l, t, n): the
 * derivative of A with respect to each element's conductivities contracted
 * with two vectors (FP64).  Without a sheet, c = t covers the whole plane
 * normal to the fiber and g[..][2] = 0; without a fiber only c = t is
 * non-zero.  scale = 1 gives the apply's adjoint (dL/dsigma of y = A u with
 * w = dL/dy); scale = -1 the solve's (dL/dsigma of u = A^{-1} f with w the
 * adjoint solution of A w = dL/du).  EINVAL for a non-finite scale.
 * u, w [device][batch][n_dof]; g [device][batch][n_elem][3].                  */
mfsem_status mfsem_op_grad_sigma(const mfsem_op* op, const double* u, const double* w,
                                 double scale, double* g, void* stream);

/* ------------------------------------------------------------------------ */
/* Matrix-based path: A assembled as a sparse matrix (the paper's matrix-based
 * comparison: the global matrix from the element matrices, Alg. 2, and sparse
 * matrix-vector products, Section 4), for operators on a structured lattice
 * with GLL quadrature, batch 1 and FP64 geometry (EUNSUPPORTED otherwise).
 * CSR, row g in increasing column order, in one of two patterns:
 *   MFSEM_CSR_ELEMENT  every node of every element containing node g (up to
 *                      (2p+1)^3 per row), the explicit zeros of collocation
 *                      included, as a standard assembly of full element
 *                      matrices stores them;
 *   MFSEM_CSR_COUPLED  only the nodes of that set sharing at least one
 *                      lattice coordinate with node g: the pairs GLL
 *                      collocation can make non-zero (about 0.43 of the
 *                      element pattern's entries at p = 4).
 * Both give the same products; alpha is the operator's at assembly.  An
 * unknown pattern is EINVAL.                                                 */
typedef enum { MFSEM_CSR_ELEMENT = 0, MFSEM_CSR_COUPLED = 1 } mfsem_csr_pattern;

/* Number of stored entries in the pattern. [host] */
mfsem_status mfsem_csr_nnz(const mfsem_op* op, int pattern, int64_t* nnz);

/* Fill row_ptr [n_dof+1] (int64), col [nnz] (int32) and val [nnz] (FP64),
 * all [device] and caller-sized from mfsem_csr_nnz with the same pattern.   */
mfsem_status mfsem_csr_assemble(const mfsem_op* op, int pattern, int64_t* row_ptr, int32_t* col,
                                double* val, void* stream);

/* y = A x with a CSR matrix; x, y [device][n_rows] FP64, not aliased.  nnz
 * [host] is the number of stored entries (row_ptr[n_rows], from
 * mfsem_csr_nnz); its mean per row picks 16 or 32 lanes per row.  A wrong
 * nnz only changes that choice, never the result.                           */
mfsem_status mfsem_csr_spmv(int64_t n_rows, int64_t nnz, const int64_t* row_ptr,
                            const int32_t* col, const double* val, const double* x, double* y,
                            void* stream);

/* ------------------------------------------------------------------------ */
/* Geometric multigrid V-cycle (Section 4.3).  Levels are operators created by
 * the caller, finest first; transfers[l] links level l (fine) and l+1.
 * P-transfers keep the elements and lower the degree; H-transfers map each
 * fine element to its octree parent.  Prolongation interpolates the coarse
 * function at the fine nodes; restriction is its exact transpose.  Smoothing
 * is Chebyshev-Jacobi of `degree` on [lo_frac, hi_frac] * lambda_max, with
 * lambda_max from `eig_iters` Jacobi-CG steps on a seeded start vector
 * (Section 5: 10 steps, [0.08, 1.2]); the coarsest level is a Chebyshev
 * smoothing of `coarse_degree` from zero.  The polynomial is applied in its
 * factored form, `degree` damped-Jacobi steps weighted by the inverse roots
 * (largest root first), which ends on the same iterate as the three-term
 * recurrence.  The cycle is symmetric, so it is a valid CG preconditioner.
 * Every level must hold geometry in `precision`.                            */
typedef struct {
  int32_t kind;             /* mfsem_transfer_kind */
  const int32_t* parent;    /* H: [device] [n_elem_fine], coarse element of each fine
                               element (0 <= parent < n_elem_coarse); P: NULL */
  const int8_t* child;      /* H: [device] [n_elem_fine], octant cx + 2 cy + 4 cz of the
                               fine element in its parent's local axes; P: NULL.
                               mfsem_mg_create checks both ranges on the device
                               (EINVAL naming the level).                        */
} mfsem_transfer_desc;

typedef struct {
  int32_t n_levels;                      /* 1..16 */
  const mfsem_op* const* ops;            /* [host] [n_levels] */
  const mfsem_transfer_desc* transfers;  /* [host] [n_levels-1] */
  int32_t degree;                        /* >= 1 */
  int32_t coarse_degree;                 /* >= 1 */
  double lo_frac, hi_frac;               /* 0 < lo < hi */
  int32_t eig_iters;                     /* >= 1 */
  uint64_t eig_seed;
  const double* lambda_max;              /* [host] [n_levels][batch] or NULL = estimate */
  int32_t precision;                     /* mfsem_dtype of the whole cycle */
  int32_t graphs;                        /* 1: the first cycle with a given (r, z) pair (and
                                            levels' alpha) is captured into a HIP graph on a
                                            private stream, later ones replay it with one
                                            graph launch on `stream` (up to 4 pairs kept);
                                            0: plain launches                              */
} mfsem_mg_desc;

mfsem_status mfsem_mg_workspace_bytes(const mfsem_mg_desc* d, size_t* bytes);

/* Build the hierarchy: diagonals, lambda_max estimates, transfer data. [sync] */
mfsem_status mfsem_mg_create(const mfsem_mg_desc* d, void* ws, size_t ws_bytes, void* stream,
                             mfsem_mg** out);
mfsem_status mfsem_mg_destroy(mfsem_mg* mg);

/* z = V(r): one V-cycle from a zero guess.  r, z [device][batch][n_dof] in
 * the cycle's precision.  Uses buffers inside the workspace, which hold
 * zeros between cycles (each kernel clears what it read last): calls on the
 * same mg must not overlap, and r and z must not alias.                     */
mfsem_status mfsem_mg_vcycle(const mfsem_mg* mg, const void* r, void* z, void* stream);

/* lambda_max per level and batch member, [host] [n_levels][batch]. */
mfsem_status mfsem_mg_lambdas(const mfsem_mg* mg, double* lam);

/* One transfer between levels `level` (fine) and `level`+1 (coarse), in the
 * cycle's precision, [device] [batch][n_dof of the level]:
 *   direction 0 (prolongation): out_fine = P in_coarse (every fine DOF written);
 *   direction 1 (restriction):  out_coarse = P^T in_fine (out is overwritten). */
mfsem_status mfsem_mg_transfer(const mfsem_mg* mg, int32_t level, int32_t direction,
                               const void* in, void* out, void* stream);

/* ------------------------------------------------------------------------ */
/* Preconditioned CG in FP64 (Section 4).  mg == NULL: plain CG.  An FP32 mg
 * is applied to an FP32 copy of r and its result widened; use flexible = 1
 * then (Polak-Ribiere beta).  Stops each batch member when
 * ||r||_2 <= max(rtol*||b||_2, atol) (true recurrence residual, l2 norm).   */
typedef struct {
  double rtol, atol;
  int32_t max_it;     /* >= 1 */
  int32_t flexible;   /* 0/1 */
} mfsem_solve_opts;

typedef struct {
  int32_t iters;
  int32_t status;     /* mfsem_status of this batch member */
  double r0_norm, r_norm, b_norm;
} mfsem_solve_info;

mfsem_status mfsem_pcg_workspace_bytes(const mfsem_op* op, const mfsem_mg* mg, size_t* bytes);

/* Solve A x = b.  b, x [device][batch][n_dof] FP64; x holds the initial
 * guess on entry and the last iterate on exit.  info [host][batch].
 * Returns the worst member status (ENOCONV, EBREAKDOWN, ENONFINITE). [sync] */
mfsem_status mfsem_pcg(const mfsem_op* op, const mfsem_mg* mg, const double* b, double* x,
                       const mfsem_solve_opts* opts, mfsem_solve_info* info, void* ws,
                       size_t ws_bytes, void* stream);

/* The same solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * instead of a caller workspace, the CG work vectors, scalars and reduction
 * partials live in a fixed array of MFSEM_NOALLOC_SCRATCH_MB MiB that the
 * library holds on every GPU it runs on until the process ends.  Nothing is
 * allocated or freed by this call (no hipMalloc, hipFree or allocating
 * library routine).  The scratch serves n_dof * batch up to about 1.3M DOFs
 * (the size mfsem_pcg_workspace_bytes reports must not exceed it): larger
 * solves fail with EINVAL before any launch, and the message says so.
 * The array of the calling thread's current device is used (it must be the
 * device of op, mg and stream).  Every call on one GPU shares that GPU's
 * array, which keeps the last call's contents (each call writes every value
 * before reading it, so nothing needs to start at zero): calls that overlap
 * on one GPU (from several host threads or streams) race and must be
 * serialised by the caller.  Arguments and results as mfsem_pcg.  [sync]    */
#define MFSEM_NOALLOC_SCRATCH_MB 64
mfsem_status mfsem_pcg_noalloc(const mfsem_op* op, const mfsem_mg* mg, const double* b,
                               double* x, const mfsem_solve_opts* opts, mfsem_solve_info* info,
                               void* stream);

/* ------------------------------------------------------------------------ */
/* Pointwise ionic step for the full monodomain time loop (the DOF-wise ionic
 * loop and right-hand side of Alg. 1, first-order IMEX in place of BDF2, with
 * the two-variable Aliev-Panfilov model in place of the paper's ionic
 * models).  With u = (V - v_rest)/v_amp:
 *   F = k u (1-u)(u-a) - u w,   G = (eps0 + mu1 w/(u+mu2)) (-w - k u (u-a-1))
 *   b = mass_diag * (chi*cm/dt * V + chi*cm*(v_amp/t_scale)*F + i_stim)
 *   w <- w + (dt/t_scale) G
 * All arrays [device][n] FP64; i_stim may be NULL (zero).                    */
typedef struct {
  double k, a, eps0, mu1, mu2, v_rest, v_amp, t_scale;
} mfsem_ap_params;

mfsem_status mfsem_ap_imex_rhs(int64_t n, double dt, double chi, double cm,
                               const mfsem_ap_params* prm, const double* V, double* w,
                               const double* i_stim, const double* mass_diag, double* b,
                               void* stream);

/* The paper's BDF2 step of the partitioned scheme (Section 3, the ionic and
 * monodomain discretization, with the extrapolation V* = 2 V^n - V^{n-1} and
 * ionic current interpolation, lumped for SEM-NI), for the same model:
 *   gating, implicit in w^{n+1}:
 *     3 w^{n+1} - 4 w^n + w^{n-1} = (2 dt/t_scale) G(u*, w^{n+1}),
 *     u* = (V* - v_rest)/v_amp  (solved in closed form: G is quadratic in w);
 *   b = mass_diag * (chi*cm/dt * (4 V^n - V^{n-1})/2
 *                    + chi*cm*(v_amp/t_scale) * F(u*, w^{n+1}) + i_stim),
 * the right-hand side of (3/2 chi*cm/dt M + K) V^{n+1} = b; then
 * w_old <- w^n and w <- w^{n+1}.  V = V^n, V_old = V^{n-1}.
 * All arrays [device][n] FP64; i_stim may be NULL (zero).  A first step from
 * rest may take V_old = V and w_old = w.                                     */
mfsem_status mfsem_ap_bdf2_rhs(int64_t n, double dt, double chi, double cm,
                               const mfsem_ap_params* prm, const double* V, const double* V_old,
                               double* w, double* w_old, const double* i_stim,
                               const double* mass_diag, double* b, void* stream);

/* Activation times (Section 5.1: at each node, the time at which the
 * transmembrane potential changes fastest, tau = argmax_t |du/dt|), kept as a
 * running maximum over a time loop.  Call once after every step with
 * V = V^{n+1} (at time t) and V_old = V^n (at t - dt):
 *   q = |V - V_old| / dt;   where q > rate:  rate = q,  act = t - dt/2
 * (the step's midpoint, where the difference quotient estimates du/dt to
 * second order; the comparison is strict, so of equally steep steps the
 * earliest is kept).  Start from act = -1 and rate = 0: nodes whose potential
 * never changes keep -1.  act and rate must both be given or both be NULL.
 * cross (may be NULL): where cross < 0 and V_old < v_cross <= V, cross is set
 * to the crossing time interpolated linearly in [t - dt, t] (a level
 * crossing, which precedes the steepest point of an upstroke; not the
 * activation time).  At least one of act and cross is given.
 * All arrays [device][n] FP64; V, V_old are read only.  EINVAL for dt <= 0,
 * non-finite t or v_cross, or a NULL array with n > 0.                      */
mfsem_status mfsem_activation_update(int64_t n, double t, double dt, const double* V,
                                     const double* V_old, double* act, double* rate,
                                     double v_cross, double* cross, void* stream);

/* out = 2 v - v_old: the linear extrapolation of a time series (the V* of
 * the BDF2 scheme, Section 3), used as the initial guess of the next implicit
 * solve in place of v.  [device] arrays of n FP64 values; out may be v or
 * v_old (elementwise).                                                       */
mfsem_status mfsem_extrapolate(int64_t n, const double* v, const double* v_old, double* out,
                               void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MFSEM_H */
