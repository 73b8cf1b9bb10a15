/*
 * ufem.h -- C ABI of the MI355X (gfx950) matrix-free unfitted DG operator.
 *
 * Operator: v = A u for the SIPG discretisation of the Poisson problem on a
 * Cartesian background mesh cut by a level set (union of balls), with Nitsche
 * terms on the embedded boundary and a face ghost penalty on the faces of cut
 * cells (Bergbauer, Munch, Wall, Kronbichler, arXiv 2404.07911, Section 2.1
 * bilinear forms of the CG and DG methods, Section 2.2 ghost penalty).
 *
 * Conventions shared by every entry point
 *  - Return value: UFEM_OK (0) or a negative error code; ufem_last_error()
 *    returns a message for the calling thread.  No C++ exception crosses the
 *    ABI.
 *  - "host" pointers are ordinary CPU memory, "device" pointers are HIP device
 *    memory of the device the operator was set up on.  The caller owns every
 *    pointer it passes; the library owns what it allocates (released by the
 *    matching destroy call).
 *  - Vectors are cell-contiguous: active cells in background order
 *    (b = ix + n iy + n^2 iz), (p+1)^dim values per cell, local index
 *    l = i + k j + k^2 m with k = p + 1 (x fastest; Section 3.2, tensor-product
 *    index of the sum-factorised evaluation).  The nodal basis is the Lagrange
 *    basis on the Gauss-Lobatto points of each cell.
 *  - Quadrature-point (kappa) vectors follow the layout of ufem_info.seg:
 *    [inside-cell volume | cut-cell volume | structured SIPG faces |
 *     cut SIPG faces | interface], each segment in active-cell resp. face
 *    order (faces ordered by lower cell, then axis).
 *  - Stream arguments are hipStream_t values passed as void* (NULL = the
 *    default stream).  Calls that take a stream are asynchronous.
 */
#ifndef UFEM_H
#define UFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  UFEM_OK = 0,
  UFEM_EINVAL = -1,      /* bad argument (null, size, aliasing, range) */
  UFEM_ENOMEM = -2,      /* host or device allocation failed */
  UFEM_EHIP = -3,        /* HIP runtime error (message has the HIP string) */
  UFEM_EUNSUPPORTED = -4,/* valid but unsupported configuration */
  UFEM_ESTATE = -5       /* call out of order (e.g. kappa missing) */
};

/* Term mask bits: volume (Poisson) term, SIPG interior-face terms, Nitsche
 * interface terms, face ghost penalty. */
enum {
  UFEM_TERM_VOLUME = 1,
  UFEM_TERM_SIPG = 2,
  UFEM_TERM_NITSCHE = 4,
  UFEM_TERM_GHOST = 8,
  UFEM_TERM_ALL = 15
};

/* Arithmetic of an apply: every input, table, quadrature datum and
 * accumulation is in this precision, with one exception: the last sum of a
 * cut cell's volume and interface line contributions into the cell's row
 * (the rows are kept in float64 in shared memory for both precisions, where
 * float64 atomic adds are the cheap ones). */
enum { UFEM_F64 = 0, UFEM_F32 = 1 };

/* Kernel stages of one apply (ufem_apply_part).  Stage 1 writes the rows of
 * inside cells.  Stage 2 writes the rows of cut cells with their
 * structured-face and ghost-penalty terms (sum factorisation with kappa = 1,
 * per-point face quadrature with a kappa field).  Stages 4 and 8 add the
 * dimension-reduction volume and interface lines and the cut-face lines to
 * the rows stage 2 wrote. */
enum {
  UFEM_PART_INSIDE = 1,
  UFEM_PART_CUT_STRUCTURED = 2,
  UFEM_PART_CUT_LINES = 4,
  UFEM_PART_CUT_FACE_LINES = 8,
  UFEM_PART_CUT = 14,
  UFEM_PART_ALL = 15
};

typedef struct ufem_plan ufem_plan; /* host-side plan (no GPU) */
typedef struct ufem_op ufem_op;     /* device-side operator */

/* Level-set kinds of ufem_problem.levelset.  BALLS: a union of balls,
 * phi = min_i (|x - c_i| - r_i) (the sphere geometries of Section 6).  PLANE:
 * phi = (n . x - offset) / |n| (the plane benchmark of Section 5.2). */
enum { UFEM_LEVELSET_BALLS = 0, UFEM_LEVELSET_PLANE = 1 };

/* Ghost-penalty kinds of ufem_problem.gp_kind.  FACE: the face ghost
 * penalty sum_j gamma_j h^(2j-1) ([d_n^j v], [d_n^j u])_F on every face of
 * a cut cell.  VOLUME: the volume ghost penalty of Section 2.2 (eq.
 * volume_based_gp), (tau_v / h^2) (J_P v, J_P u)_P over patches P of two
 * face neighbours, J_P u the difference of the two cells' polynomials
 * extended over the patch, tau_v = gp_gamma; patches by the stable-neighbour
 * strategy (each cut cell with its neighbour of largest volume fraction,
 * fractions within 1e-10 equal, the lower slot 2 axis + side first).
 * VOLUME_ALL: the same term on every face of a cut cell. */
enum { UFEM_GP_FACE = 0, UFEM_GP_VOLUME = 1, UFEM_GP_VOLUME_ALL = 2 };

/* Function spaces of ufem_problem.space.  DG: the discontinuous Q_p space
 * with the SIPG interior-face terms (eq. bilinear_dg).  CG: the continuous
 * Q_p space (FE_Q, eq. bilinear_cg: Poisson and Nitsche terms, no SIPG)
 * with the same ghost penalty; its DoFs are the Gauss-Lobatto nodes of the
 * active cells on the global node lattice ((n p + 1)^dim nodes, node
 * (I_0, I_1, I_2) at lo + h (I / p)), numbered in lattice order (I_0
 * fastest).  The operator is evaluated as P^T A_cell P with P the copy of
 * node values into the cells' DoFs and P^T the sum of the cells'
 * contributions per node (the read and distribute operators R, D of Section
 * 3.1, eq. matrixfreeopcompact). */
enum { UFEM_SPACE_DG = 0, UFEM_SPACE_CG = 1 };

/* Problem description.  All pointers are host pointers read during
 * ufem_plan_create only.  The physical domain is {phi < 0}. */
typedef struct {
  int32_t dim;           /* 2 or 3 */
  int32_t n;             /* background cells per direction, >= 2 */
  double lo, hi;         /* background box [lo, hi]^dim */
  int32_t degree;        /* polynomial degree p, 1..7 (3D), 1..7 (2D) */
  int32_t q_cut;         /* Gauss points per 1D piece of the cut-cell, cut-face
                            and interface rules; 0 selects p + 1 */
  int32_t max_depth;     /* subdivision limit of the cut rules; < 0 selects 4 */
  int32_t n_balls;       /* BALLS: number of balls, >= 1 (PLANE: ignored) */
  const double* centers; /* BALLS: host, n_balls * dim, row-major */
  const double* radii;   /* BALLS: host, n_balls, > 0 */
  double nitsche_factor; /* tau_D = nitsche_factor * p^2 (Section 2.1) */
  double sipg_factor;    /* gamma = sipg_factor * p^2, SIPG penalty gamma/h */
  double gp_gamma;       /* ghost penalty weight (tau_v of the volume kinds) */
  int32_t gp_jmin;       /* face kind: lowest derivative order penalised, 0..p */
  int32_t gp_flat;       /* face kind: 0: gamma_j = gp_gamma/(j!)^2, 1: gp_gamma */
  int32_t levelset;      /* UFEM_LEVELSET_BALLS (0, the zero-initialised
                            default) or UFEM_LEVELSET_PLANE */
  double plane_normal[3];/* PLANE: normal n (first dim entries, nonzero) */
  double plane_offset;   /* PLANE: offset; phi = (n . x - offset) / |n| */
  int32_t gp_kind;       /* UFEM_GP_FACE (0, default), UFEM_GP_VOLUME or
                            UFEM_GP_VOLUME_ALL */
  int32_t space;         /* UFEM_SPACE_DG (0, default) or UFEM_SPACE_CG */
} ufem_problem;

typedef struct {
  int64_t n_background; /* n^dim */
  int64_t n_active;     /* cells with DoFs: inside + cut */
  int64_t n_inside;
  int64_t n_cut;
  int64_t n_dofs;       /* DoFs of the space: n_active * (p+1)^dim (DG), the
                           nodes of the active cells (CG) */
  int64_t n_faces;      /* interior faces between active cells */
  int64_t n_faces_str;  /* with structured SIPG quadrature */
  int64_t n_faces_cut;  /* with dimension-reduction SIPG quadrature */
  int64_t n_faces_gp;   /* with ghost penalty */
  int64_t n_qp;         /* length of a kappa vector */
  int64_t seg[6];       /* kappa segment offsets (see header comment) */
  int64_t max_qp_cut_cell; /* largest cut-cell volume rule */
  int64_t n_fallback;   /* sub-boxes that hit the subdivision limit */
  double h;             /* background cell size */
  int64_t n_cell_dofs;  /* n_active * (p+1)^dim (equal to n_dofs for DG) */
} ufem_info;

/* Build the host plan: cell classes (inside / cut / outside by exact
 * ball-versus-box distances), the face lists, the dimension-reduction
 * quadrature of every cut cell, cut face and interface piece (Saye 2015, as
 * cited in Sections 1 and 2.3), and the quadrature-point layout.  No GPU is
 * touched.  Faces on the boundary of the background box carry no term.
 * Errors: EINVAL for out-of-range fields or a level set that leaves no active
 * cell, EUNSUPPORTED beyond 2e9 DoFs, ENOMEM on host allocation failure. */
int ufem_plan_create(const ufem_problem* prob, ufem_plan** out);
int ufem_plan_destroy(ufem_plan* plan);
int ufem_plan_info(const ufem_plan* plan, ufem_info* info);

/* Plan export (host buffers sized from ufem_info).
 *  cls:   int8[n_background], 0 inside, 1 cut, 2 outside.
 *  faces: int32[n_faces * 5], rows (lower cell, upper cell, axis, kind, gp)
 *         with background cell indices and kind 0 structured, 1 cut,
 *         2 no SIPG term. */
int ufem_plan_cells(const ufem_plan* plan, int8_t* cls);
int ufem_plan_faces(const ufem_plan* plan, int32_t* faces);
/* Quadrature-point data in kappa order: xyz = physical coordinates
 * (double[n_qp * dim]), ref = reference coordinates in the owning cell
 * (double[n_qp * dim]; faces use the lower cell, on its upper face), w =
 * reference weights (double[n_qp]; physical weight = w * h^dim for volume
 * points, w * h^(dim-1) for face and interface points), nrm = unit normals of
 * interface points (double[n_qp * dim], zero elsewhere).  Any pointer may be
 * NULL. */
int ufem_plan_qp(const ufem_plan* plan, double* xyz, double* ref, double* w, double* nrm);

/* Replace the plan's dimension-reduction rules by explicit ones: the
 * "quadrature" input of setup, for rules from another generator (Section 2.3
 * only requires some quadrature of the cut cells, cut faces and interface).
 * The cells, faces and their classes stay; the counts, the point lines and
 * the kappa layout (ufem_plan_info) are rebuilt.  Host arrays:
 *   vol_count[n_cut], face_count[n_faces_cut], surf_count[n_cut]: points of
 *     each cut cell's volume rule, each cut face's rule and each cut cell's
 *     interface rule (cut cells in active order, cut faces in face order);
 *   ref[dim * N], w[N], nrm[dim * N] with N the sum of all counts: the
 *     points of the three rules in kappa order (every cut cell's volume
 *     rule, then every cut face's rule, then every interface rule), as
 *     ufem_plan_qp exports them for the segments seg[1]..seg[2],
 *     seg[3]..seg[4] and seg[4]..seg[5]: reference coordinates in [0, 1]
 *     (face points in the lower cell; their face-axis coordinate is not
 *     read), reference weights >= 0, unit normals (read for interface points
 *     only).
 * Errors: EINVAL for a null array where points exist, a negative count,
 * coordinates outside [0, 1] (1e-12 slack), non-finite values or negative
 * weights (the plan is then unchanged); EUNSUPPORTED beyond 2^31 points of
 * a kind.  Operators set up before the call keep their rules. */
int ufem_plan_import_quadrature(ufem_plan* plan, const int64_t* vol_count, const int64_t* face_count,
                                const int64_t* surf_count, const double* ref, const double* w, const double* nrm);

/* Upload the plan to `device` and build the operator.  The plan may be
 * destroyed afterwards.  Allocates all device memory the operator needs
 * (max_device_bytes > 0 caps it; ENOMEM beyond).  Tables are stored for both
 * precisions. */
int ufem_setup(const ufem_plan* plan, int device, void* stream, int64_t max_device_bytes, ufem_op** out);
int ufem_destroy(ufem_op* op);
int ufem_info_op(const ufem_op* op, ufem_info* info);

/* Mixed evaluation (Section 3.2, eq. additive_decomp, the "mixed" option):
 * enable != 0 precomputes the cut cells' unstructured cell terms (volume and
 * interface quadrature) as one dense nd x nd element matrix per cut cell
 * (nd = (p+1)^dim; built on `stream` from the matrix-free line kernels
 * applied to unit vectors, float64, rounded once for the float32 operator),
 * and later applies, adjoint passes and CG iterations apply them as a
 * batched matrix-vector product; structured terms and cut faces stay
 * matrix-free.  Device memory: n_cut nd^2 (8 + 4) bytes, allocated at the
 * first enable and counted against max_device_bytes (ENOMEM beyond), plus
 * two temporary vectors during the build.  The matrices follow
 * ufem_set_terms and ufem_set_kappa (float64 kappa; rebuilt there, which
 * synchronises the stream).  enable == 0 returns to the matrix-free
 * evaluation (the memory stays until ufem_destroy).  Synchronous. */
int ufem_set_mixed(ufem_op* op, int32_t enable, void* stream);

/* Select the terms of subsequent applies and adjoint passes (default
 * UFEM_TERM_ALL). */
int ufem_set_terms(ufem_op* op, int32_t term_mask);

/* Cap on the workgroups of every kernel launch of subsequent calls (0, the
 * default: each launch is sized by its work, the persistent cut-cell kernels
 * by occupancy times compute units).  Every kernel loops over its cell
 * groups or batches, so any cap gives the same result bit for bit; a small
 * cap makes each workgroup take many groups in turn (used by the tests to
 * run the multi-batch paths on small problems).  EINVAL for a negative cap. */
int ufem_set_max_blocks(ufem_op* op, int32_t max_blocks);

/* Per-quadrature-point coefficient kappa (the variable coefficient of the
 * volume, SIPG and Nitsche terms; the ghost penalty carries none).  kappa is a
 * device pointer to n_qp values of the given precision, copied into the
 * operator on `stream`; kappa == NULL returns to kappa = 1. */
int ufem_set_kappa(ufem_op* op, int32_t precision, const void* kappa, void* stream);

/* v := A u (overwrite): the operator action of Section 3.1 (eq.
 * operatorevaluation), the sum over cells and faces of read, evaluate,
 * quadrature-point operator, integrate and distribute (eq.
 * matrixfreeopcompact) for the DG form of Section 2.1 (eq. bilinear_dg with
 * the Nitsche terms of eq. bilinear_cg) plus the face ghost penalty; uncut
 * cells and faces with tensor-product (structured) quadrature, cut cells,
 * cut faces and the interface with the dimension-reduction (unstructured)
 * quadrature of Section 3.2 (eq. unstructured_cell, unstructured_face).
 * u, v: device pointers to n_dofs values of `precision`, cell-contiguous
 * (layout above); u must not overlap v (EINVAL).  Every entry of v is
 * written.  Asynchronous on `stream`; allocates nothing. */
int ufem_apply(ufem_op* op, int32_t precision, const void* u, void* v, void* stream);

/* The kernel stages of ufem_apply (UFEM_PART_* bits, any non-empty mask),
 * for per-kernel timing; UFEM_PART_ALL is ufem_apply.  Stages run in the
 * order 1, 2, 4, 8 on `stream` (with kappa = 1, stages 1 and 2 requested
 * together are one kernel); rows of the cells a mask does not cover are left
 * untouched, and stages 4 and 8 add to v, so the rows of cut cells are A u
 * only when stages 2, 4 and 8 run after one another (in one call or in
 * consecutive calls with the same u and v).  EINVAL for an empty or unknown
 * mask. */
int ufem_apply_part(ufem_op* op, int32_t precision, int32_t part, const void* u, void* v, void* stream);

/* Adjoint pass for L(kappa, u) with residual weight w:
 *   ATw := A^T w  (the transposed operator of eq. matrixfreeopcompact, each
 *                  cell and face term with evaluation and integration
 *                  swapped, R^T E^T B^T I^T D^T; for the self-adjoint Poisson
 *                  form of Section 2.1 I = E^T, so this equals A w),
 *   dkappa[q] := a_q(w, u), the contribution of quadrature point q to
 *                w^T A(kappa) u divided by kappa_q (dL/dkappa_q for
 *                L = 0.5 |A u - b|^2 with w = A u - b).
 * The term mask (ufem_set_terms) selects the terms of both outputs: points
 * of a switched-off term get dkappa = 0 (the ghost penalty carries no kappa).
 * w, u, ATw: device, n_dofs; dkappa: device, n_qp, or NULL to skip.  ATw must
 * not overlap w or u, dkappa none of the three (EINVAL).  Asynchronous on
 * `stream`; allocates nothing. */
int ufem_apply_adjoint(ufem_op* op, int32_t precision, const void* w, const void* u, void* ATw,
                       void* dkappa, void* stream);

/* Device BLAS-1 of the solvers (float64 unless noted), asynchronous on
 * `stream`.  Result scalars are written to device memory.
 *   dot:    out[0] = sum x_i y_i (float64 accumulation for both precisions)
 *   axpby:  y = a x + b y
 *   cast:   y (precision_out) = x (precision_in) element-wise */
int ufem_dot(int32_t precision, int64_t n, const void* x, const void* y, double* out, void* stream);
int ufem_axpby(int32_t precision, int64_t n, double a, const void* x, double b, void* y, void* stream);
int ufem_cast(int32_t precision_in, int32_t precision_out, int64_t n, const void* x, void* y, void* stream);

/* n_iter iterations of unpreconditioned conjugate gradients for A x = b
 * (the paper solves with CG, Section 3.6), entirely on the device: each
 * iteration is one apply (Ap) and three vector kernels, with no host
 * synchronisation.  x, r, p, ap: device, n_dofs values of `precision`, no
 * two overlapping; scal: device, 4 float64 values.  On entry r = b - A x,
 * p = r, scal = [r.r, 0, 0, 0] (the caller sets them up, e.g. with
 * ufem_apply / ufem_axpby / ufem_dot); on return x, r, p are advanced by
 * n_iter iterations, scal[0] = r.r of the new residual, and scal[3] != 0 if
 * p.Ap <= 0 occurred (breakdown: x, r, p were left as they were before that
 * iteration and further iterations do nothing).  The dot products
 * accumulate in float64 for both precisions, so their rounding order (one
 * atomic add per block) varies between runs.  Asynchronous on `stream`;
 * allocates nothing. */
int ufem_cg_iterate(ufem_op* op, int32_t precision, int32_t n_iter, void* x, void* r, void* p, void* ap,
                    double* scal, void* stream);

/* ufem_cg_iterate without a workspace argument and without any allocation,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  The CG
 * scalars and the vector A p live in a fixed device array of the library,
 * one per device, held until the process ends: 64 MiB for A p (n_dofs up to
 * 8,388,608 float64 or 16,777,216 float32 values; EINVAL beyond) after 256
 * bytes of scalars.  Its device address is taken once per device by
 * ufem_setup.  Every call clears the scalars and computes r.r itself, so
 * only x, r, p carry state between calls: on entry r = b - A x and p = r
 * (or the r, p a previous call returned); on return x, r, p are advanced by
 * n_iter iterations as by ufem_cg_iterate, result[0] = r.r of the new
 * residual and result[1] != 0 if p.Ap <= 0 occurred (breakdown; the
 * remaining iterations did nothing).  x, r, p: device, n_dofs values of
 * `precision`, not overlapping; result: device, 2 float64.  All calls on
 * one device share the array: calls that overlap in time on one device
 * (two streams, or two host threads) race and give wrong results.
 * Asynchronous on `stream`; allocates nothing. */
int ufem_cg_iterate_static(ufem_op* op, int32_t precision, int32_t n_iter, void* x, void* r, void* p,
                           double* result, void* stream);

/* Thread-local message of the last failing call (never NULL). */
const char* ufem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* UFEM_H */
