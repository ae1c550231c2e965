/*
 * dgpoly -- SIPG matrix assembly on polytopic meshes for AMD MI355X (gfx950).
 *
 * C ABI of libdgpoly.so.  Plain C99: no C++ types and no exceptions cross this
 * boundary; every call returns a dgp_status.  On any status other than DGP_OK
 * no output has been written and dgp_last_error() describes the failure.
 *
 * What is computed (Dong, Georgoulis, Kappas, "GPU-accelerated discontinuous
 * Galerkin methods on polytopic meshes"):
 *   find u_h in S^p with B(u_h, v_h) = l(v_h) for all v_h       (Section 2.2)
 *   B = the symmetric interior penalty bilinear form   (equation dg-bilinear)
 *   l = the linear functional                          (equation dg-linear)
 *   sigma_F = C_sigma * max_{kappa in F} abar_kappa p_kappa^2 / h_kappa, or the
 *             covering form of Appendix A (dgp_problem.penalty; h = diameter,
 *             abar = max of a over the element's volume quadrature points)
 * with physical-frame orthonormal Legendre bases of total degree p on each
 * element's bounding box (Section 3.1), quadrature on the fan sub-triangles of
 * each polygon and Gauss-Legendre points on each edge (Section 3), written into
 * a precomputed block sparsity pattern (Section 3.4, Approach 2).
 *
 * Matrix layout (block CSR, rows = elements):
 *   row_ptr[n_rows+1]  (int64)  blocks of row r are k = row_ptr[r] .. row_ptr[r+1]-1
 *   col_idx[nnzb]      (int32)  ascending within a row; the diagonal is present
 *   val_ptr[nnzb+1]    (int64)  block k occupies vals[val_ptr[k] .. val_ptr[k+1])
 *   dof_ptr[n_rows+1]  (int64)  rhs entries of row r: rhs[dof_ptr[r] ..]
 * Block (r, c) is row-major n_b(p_r) x n_b(p_c); entry (i, j) = B(phi_j^c, phi_i^r)
 * (row = test function, column = trial function).  n_b(p) = (p+1)(p+2)/2 in 2D.
 * Basis order: total degree k = 0..p, x-exponent descending within k.
 *
 * Threading: a context is bound to one device and one HIP stream; it is not
 * thread-safe.  All device work is asynchronous on that stream unless stated.
 */
#ifndef DGPOLY_H
#define DGPOLY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dgp_status;
#define DGP_OK 0
#define DGP_EINVAL (-1)       /* null pointer, size mismatch, bad enum */
#define DGP_EMESH (-2)        /* malformed mesh: face not adjacent to its cells, bad ids, < 3 vertices,
                                 clockwise or zero-area polygon, zero-volume tetrahedron */
#define DGP_EUNSUPPORTED (-3) /* degree or dimension outside what the kernels are built for */
#define DGP_ENOMEM (-4)       /* device allocation failed */
#define DGP_EDEVICE (-5)      /* any HIP runtime error */
#define DGP_ESTATE (-6)       /* call order: e.g. assemble before pattern */

#define DGP_F64 0 /* contraction and output in double precision */
#define DGP_F32 1 /* geometry, penalty and weights in FP64; contraction and output in FP32 */

#define DGP_RULE_PLAIN 0   /* volume terms on the fan sub-triangles (Section 3) */
#define DGP_RULE_REDUCED 1 /* volume matrix with each element's accepted 16-node rule (dgp_qrule_build) */

#define DGP_INIT_NETWORK 0  /* reduced rules start from the network's prediction */
#define DGP_INIT_TEMPLATE 1 /* reduced rules start from the 4 x 4 Gauss tensor rule on the box */

#define DGP_MLP_PARAMS 43952 /* FP32 parameters of the rule network */

#define DGP_U_SIN 0  /* manufactured u = sin(pi x) sin(pi y) (times sin(pi z) in 3D) */
#define DGP_U_POLY 1 /* u = c0 + c1 x + c2 y + c3 z + c4 x^2 + c5 y^2 + c6 z^2 + c7 xy + c8 xz + c9 yz */

typedef struct dgp_ctx dgp_ctx;

/* Polytopic mesh, host memory; dgp_mesh_upload copies every array (the
 * caller keeps ownership).
 *
 * dim = 2: polygons.  cell_vtx holds each cell's counter-clockwise vertex loop
 *   (the first vertex is the apex of the fan of sub-triangles, Section 3);
 *   face k of a cell is the edge (v_k, v_{k+1}) of its loop, cell_face_ptr
 *   equals cell_ptr; face_vtx holds 2 ids per edge, lower id first; degrees
 *   1..4; at most 24 edges per cell.
 * dim = 3: polyhedra, each the union of the tetrahedra whose 4 vertex ids it
 *   lists in cell_vtx (cell_ptr in multiples of 4).  Its faces are the
 *   triangles of that union's boundary (3 ids each in face_vtx), listed in
 *   cell_face / cell_face_ptr in any order; face_opp names the vertex of the
 *   left cell's tetrahedron opposite the triangle (it fixes the outward
 *   normal); degrees 1..2 (the degree-4 tetrahedron and triangle rules);
 *   at most 1024 faces per cell, fewer than 2^27 faces.  dgp_pattern fails
 *   with DGP_EUNSUPPORTED if a cell's boundary has more than 384 distinct
 *   vertices or the cell has more than 64 neighbours and boundary codes. */
typedef struct {
    int32_t dim;                  /* 2 or 3 */
    int64_t n_vertices;
    const double *x, *y, *z;      /* [n_vertices]; z may be NULL in 2D */
    int64_t n_cells;
    const int64_t *cell_ptr;      /* [n_cells+1] offsets into cell_vtx */
    const int32_t *cell_vtx;      /* 2D: vertex loop; 3D: 4 ids per tetrahedron */
    const int8_t *cell_p;         /* [n_cells] degree */
    const int64_t *cell_face_ptr; /* [n_cells+1] offsets into cell_face */
    const int32_t *cell_face;     /* faces of each cell */
    int64_t n_faces;
    const int32_t *face_vtx;      /* [dim n_faces] face vertex ids, in the order the face rule uses */
    const int32_t *face_cell;     /* [2 n_faces] left, right cell; right = -1 on the boundary */
    const int8_t *face_bc;        /* [n_faces] 0 interior, 1 Dirichlet, 2 Neumann */
    const int32_t *face_opp;      /* [n_faces] 3D only (may be NULL in 2D) */
} dgp_mesh_desc;

/* Penalty sigma_F on a face F shared by elements kappa_1, kappa_2 (Appendix A;
 * on a boundary face kappa_1 only), abar_kappa = max of a over the element's
 * volume quadrature points:
 *   DGP_PEN_DIAMETER  C_sigma max_kappa abar p^2 / h_kappa (h = diameter)
 *   DGP_PEN_COVERING  C_sigma max_kappa abar p^2 |F| min(1 / |K^F|, C_cov / |kappa|)
 *                     with the element's fan sub-triangles as its covering, K^F
 *                     the sub-triangle having F as a side (v0 v1 v2 for the
 *                     first edge, v0 v_{n-2} v_{n-1} for the last, v0 v_k v_k+1
 *                     for edge k otherwise) and C_cov = p^2, every element taken
 *                     as p-coverable; 2D meshes only (DGP_EUNSUPPORTED in 3D) */
#define DGP_PEN_DIAMETER 0
#define DGP_PEN_COVERING 1

/* -div(a grad u) + b . grad u + c u = f, a(x) = a0 + a1 sin(2 pi x) cos(2 pi y)
 * (3D meshes: a1 must be 0, DGP_EUNSUPPORTED otherwise), b and c constant;
 * f, Dirichlet data g_D = u and Neumann data g_N = n . (a grad u) come from the
 * manufactured u and are evaluated on the device at quadrature points. */
typedef struct {
    double a0, a1;
    double b[3];
    double c;
    double c_sigma;    /* penalty constant C_sigma (10 in every workload) */
    int32_t u_kind;    /* DGP_U_SIN or DGP_U_POLY */
    double u_poly[10];
    int32_t penalty;   /* DGP_PEN_DIAMETER or DGP_PEN_COVERING */
} dgp_problem;

typedef struct {
    int64_t n_rows, nnzb, n_vals, n_dofs;
    /* device pointers owned by the context, valid until the next upload or destroy */
    const int64_t *row_ptr;
    const int32_t *col_idx;
    const int64_t *val_ptr;
    const int64_t *dof_ptr;
} dgp_pattern_info;

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t (NULL
 * = the null stream).  Allocates nothing on the device yet. */
dgp_status dgp_create(dgp_ctx **out, int device, void *hip_stream);
dgp_status dgp_destroy(dgp_ctx *ctx);
dgp_status dgp_set_stream(dgp_ctx *ctx, void *hip_stream);
/* Text of the last failure on this context (static storage inside ctx). */
const char *dgp_last_error(const dgp_ctx *ctx);

/* The host checks of dgp_mesh_upload, without a context or a device: ids in
 * range, every face listed by the cells it bounds (2D: as the edge between
 * consecutive loop vertices), loops of >= 3 vertices running counter-clockwise
 * around a positive area (twice the signed area > 1e-13 times the squared
 * diagonal of the cell's box), 3D tetrahedra of nonzero volume, supported
 * degrees and sizes.  Returns DGP_EMESH, DGP_EINVAL or DGP_EUNSUPPORTED with
 * the reason in msg[0 .. msg_len) (msg may be NULL).  No HIP call. */
dgp_status dgp_mesh_check(const dgp_mesh_desc *mesh, char *msg, size_t msg_len);

/* Validate the mesh on the host (as dgp_mesh_check; nothing reaches the device
 * on failure) and copy it to the device.  Synchronous.  Invalidates any
 * previous pattern. */
dgp_status dgp_mesh_upload(dgp_ctx *ctx, const dgp_mesh_desc *mesh);

/* Block sparsity pattern on the device (Section 3.4): row r = sorted unique
 * {r} U {elements sharing a face with r}.  Synchronous (the sizes are read
 * back once to allocate); fills *out. */
dgp_status dgp_pattern(dgp_ctx *ctx, dgp_pattern_info *out);

/* Copy the context's pattern arrays into caller-owned device buffers of the
 * sizes reported by dgp_pattern (any pointer may be NULL to skip it).
 * Asynchronous on the context stream. */
dgp_status dgp_pattern_copy(dgp_ctx *ctx, int64_t *row_ptr, int32_t *col_idx, int64_t *val_ptr, int64_t *dof_ptr);

/* Assemble values and right-hand side into caller-owned device buffers of the
 * chosen precision: vals[n_vals], rhs[n_dofs] (float or double).  Requires
 * dgp_pattern.  Asynchronous on the context stream; runs the preparation
 * kernel (bounding boxes, diameters, abar) and the assembly kernel, which
 * leaves the pattern arrays untouched.
 * rule_mode DGP_RULE_REDUCED integrates the volume matrix of every element
 * whose reduced rule was accepted by dgp_qrule_build with that rule, and the
 * rest as DGP_RULE_PLAIN; the load vector and the faces always use the plain
 * rules.  It needs p <= 3 (DGP_EUNSUPPORTED otherwise), so that with constant
 * coefficients every volume integrand has degree <= 6 and both rules give it
 * to rounding; with a variable a (a1 != 0) neither rule is exact and the two
 * differ by their quadrature errors, O(h^(7 - 2 (p - 1))) relative to the
 * block as the mesh is refined (a's Taylor terms of degree <= 6 - 2 (p - 1)
 * are integrated exactly).  Needs a prior dgp_qrule_build (DGP_ESTATE). */
dgp_status dgp_assemble(dgp_ctx *ctx, const dgp_problem *prob, int precision, int rule_mode, void *vals, void *rhs);

/* The whole path on the device: pattern (recomputed into the context's
 * arrays, bit-identical), geometry, assembly.  Requires a prior dgp_pattern
 * (sizes known).  Asynchronous; no host synchronisation. */
dgp_status dgp_run(dgp_ctx *ctx, const dgp_problem *prob, int precision, int rule_mode, void *vals, void *rhs);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): dgp_run with the
 * step's scratch (the preparation outputs: element records, edge or face
 * records, row counts, tile sums) in a static device array of
 * DGP_STATIC_SCRATCH_BYTES that the library holds on every device it runs on,
 * instead of the buffer the context allocates at upload.  Same arguments,
 * results bit-identical to dgp_run; the call itself allocates and frees
 * nothing.  Fails with DGP_EUNSUPPORTED if the mesh needs more scratch than
 * the array holds (2D: 128 B per element of geometry and 16 B of row counts,
 * 36 B per loop edge, 16 B per face, 40 B per tile of 32 elements).  All calls on one device share
 * that device's array: calls that overlap on one device (several streams or
 * contexts, host threads) race and must be serialised by the caller.
 * Asynchronous.  Afterwards dgp_time_kernels and dgp_autotune report
 * DGP_ESTATE until the next dgp_run or dgp_assemble. */
#define DGP_STATIC_SCRATCH_BYTES (64u << 20)
dgp_status dgp_run_static(dgp_ctx *ctx, const dgp_problem *prob, int precision, int rule_mode, void *vals,
                          void *rhs);

/* Capture dgp_run (what = 0) or dgp_assemble (what = 1) with these arguments
 * into a HIP graph held by the context, and replay it. */
dgp_status dgp_graph_capture(dgp_ctx *ctx, int what, const dgp_problem *prob, int precision, int rule_mode,
                             void *vals, void *rhs);
dgp_status dgp_graph_launch(dgp_ctx *ctx);

/* Per-kernel timing of the last dgp_run / dgp_assemble (device milliseconds,
 * from HIP events recorded on the context stream around each kernel when
 * timing is enabled).  names: "prep" (geometry, and the pattern in dgp_run),
 * "assemble". */
dgp_status dgp_set_timing(dgp_ctx *ctx, int enable);
dgp_status dgp_kernel_ms(dgp_ctx *ctx, const char *name, float *ms);

/* Device time per launch of the preparation kernels and of the assembly
 * kernel(s) of the last dgp_run / dgp_assemble, from `reps` back-to-back
 * re-launches with the same arguments between two HIP events on the context
 * stream (values rewritten, pattern untouched; that call's output buffers
 * must still be allocated).  Synchronous. */
dgp_status dgp_time_kernels(dgp_ctx *ctx, int reps, float *prep_ms, float *assemble_ms);

/* Launch tuning per degree bin (Section 3.1 groups the elements by p; the
 * upload also orders each degree's rows a second way: the id order cut into
 * the eight ranges the launch gives the XCDs, each range sorted by the number
 * of fan sub-triangles, largest first).  A 2D launch configuration is
 * cfg = r + 2 s with r = 1 for the row kernel's larger occupancy (one more
 * wave per SIMD, fewer registers) and s = 1 for the rows in that second order
 * instead of id order.
 * For the last dgp_run / dgp_assemble on a 2D mesh with plain rules, times the
 * four configurations of each degree bin within about budget_ms milliseconds of
 * device time and keeps the fastest for later launches of that precision and
 * degree.  Results do not depend on the configuration.  Values of the last
 * call's output buffers are rewritten (they must still be allocated).  3D
 * meshes and reduced rules have a single configuration (nothing changes).
 * Configurations whose larger occupancy makes the kernel spill more than 32
 * bytes per lane beyond the default are not tried.  On a mesh of mixed degrees the tuned
 * per-degree launches are then timed against one persistent launch over all
 * bins and the faster is kept.  choice: NULL or int32[2][5], per [FP64, FP32]:
 * entry 0 = 1 if mixed degrees take the single launch, entries 1..4 = the cfg
 * of each degree.  Synchronous.  DGP_EINVAL if budget_ms < 1, DGP_ESTATE
 * before an assembly. */
dgp_status dgp_autotune(dgp_ctx *ctx, int budget_ms, int32_t *choice);

/* Set the 2D launch configuration cfg (0..3, as for dgp_autotune) of one
 * precision and degree without timing, for reproducible launches (a new
 * context starts every degree at cfg 2: the default register budget, rows in
 * the second order); p = 0 sets
 * how meshes of mixed degree are launched: cfg 0 one launch per degree, cfg 1
 * one persistent launch over every (degree, sub-triangle count) bin, the
 * costliest bins first (the same per-row arithmetic: bit-identical results).
 * DGP_EINVAL for a bad precision or cfg, DGP_EUNSUPPORTED for p outside 0..4. */
dgp_status dgp_set_launch(dgp_ctx *ctx, int precision, int p, int cfg);

/* Approach 1 of Section 3.3, as an ablation of the pattern-first assembly:
 * every element and every face computes its local blocks on its own and emits
 * them as COO records with duplicates (element: its block and load; interior
 * face: four blocks; boundary face: one block and its load); a stable radix
 * sort of the records by (row, column) and a segmented reduction (each block
 * summed over its records in sorted order) then produce the block pattern and
 * the values.  Outputs are caller-owned device buffers of the sizes dgp_pattern
 * reports (required first; its arrays are not used): row_ptr[n_rows+1],
 * col_idx[nnzb], val_ptr[nnzb+1], dof_ptr[n_rows+1], vals[n_vals], rhs[n_dofs].
 * 2D meshes of one degree (DGP_EUNSUPPORTED otherwise); either penalty.  The
 * first call allocates the record and sort workspace (about (n_cells + 4 n_faces)
 * (n_b^2 + n_b) doubles), kept by the context.  Asynchronous. */
dgp_status dgp_assemble_coo(dgp_ctx *ctx, const dgp_problem *prob, int precision, void *vals, void *rhs,
                            int64_t *row_ptr, int32_t *col_idx, int64_t *val_ptr, int64_t *dof_ptr);

/* One time slab I_n = (t0, t1] of the space-time method of Section 2.3
 * (equation spacetime_dg) on prisms I_n x kappa over the uploaded 2D mesh. */
typedef struct {
    double t0, t1;       /* the slab, t1 > t0 */
    double tp0;          /* start of the previous slab (its box in time is [tp0, t0]); used with prev */
    double tau1, tau2;   /* manufactured u(x, y, t) = u_s(x, y) (1 + tau1 t + tau2 t^2), u_s from dgp_problem */
    const double *prev;  /* device: the previous slab's coefficients [n_cells][n_b] (FP64), or NULL to take
                            U_{n-1}^- = u(., t0) */
} dgp_slab;

/* Matrix and load of one slab: the basis of total degree p in (x, y, t) on each
 * prism's box [lo, hi] x [t0, t1] (n_b = (p+1)(p+2)(p+3)/6, same order as the
 * 3D basis with t as the third coordinate); volume terms with the time
 * derivative, the time jump (U^+, W^+) on the prism's bottom and
 * (U_{n-1}^-, W^+) in the load, the SIPG face terms on I_n x F (penalty
 * C_sigma max abar p^2 / h with h the prism's diameter), the load with
 * f = u_s T' + T f_s.  Quadrature: the fan rule x (p + 1) Gauss points in time;
 * edge Gauss points x time Gauss points on the faces.  Block pattern: that of
 * dgp_pattern (required first), blocks n_b x n_b: vals[nnzb n_b^2],
 * rhs[n_cells n_b].  2D meshes of one degree p = 1..3, diameter penalty
 * (DGP_EUNSUPPORTED otherwise).  Asynchronous. */
dgp_status dgp_assemble_st(dgp_ctx *ctx, const dgp_problem *prob, int precision, const dgp_slab *slab, void *vals,
                           void *rhs);

/* ---------------------------------------------------------------------
 * Reduced volume rules for polygons (an extension of Section 3: the paper
 * integrates on the fan sub-triangles only).  Every element with at most 12
 * vertices is mapped to [-1, 1]^2 by its bounding box; a network predicts a
 * 16-node rule (nodes in [-1, 1]^2, weights summing to the mapped area |P|),
 * FP64 damped minimum-norm Gauss-Newton steps (Levenberg-Marquardt: a step
 * du = -J^T (J J^T + mu g I)^{-1} r, g = max diag(J J^T), is taken only if it
 * lowers ||r||_2, mu starting at 1e-6) fit it to the element's 28 Legendre
 * moments int_P P_a(xi) P_b(eta), a + b <= 6, and the rule is accepted iff
 * max_ab |Q_ab - M_ab| / |P| <= tol.  Network: 36 inputs (the loop's 12
 * vertices from the one of smallest xi, then eta, zero padded, and 12 validity
 * flags), three SiLU layers of 128, 48 outputs (nodes tanh(z_0..31) as
 * (xi, eta) pairs, weights |P| softmax(z_32..47)).  Parameter blob (FP32,
 * weights [in][out] row-major): W1[36][128] b1[128] W2[128][128] b2 W3[128][128]
 * b3 W4[128][48] b4[48]. */
typedef struct {
    int64_t n_cells, n_eligible, n_accepted;
    int64_t iters_hist[16];      /* accepted elements by refinement steps taken (15 = 15 or more) */
    double max_residual_accepted;
    float ms_features, ms_network, ms_refine; /* device time of the three stages */
    /* DGP_INIT_NETWORK: eligible elements that started from the network's rule
     * (the others from the template, whose initial residual was smaller), and
     * elements refined again from the template after the first attempt,
     * with how many of those were accepted */
    int64_t n_start_network, n_retried, n_retry_accepted;
} dgp_qrule_stats;

typedef struct {
    int64_t n_polygons;          /* training polygons, indices 0 .. n-1 of the seeded stream */
    uint64_t data_seed;          /* key of the polygon stream (dgp_train_polygons) */
    uint64_t init_seed;          /* initial weights N(0, 1/fan_in) (output layer x 1/10), hidden biases 0,
                                    output biases at the template rule's pre-activations */
    int32_t epochs, batch;
    float lr, beta1, beta2, eps; /* Adam */
} dgp_train_cfg;

typedef struct {
    float loss_first, loss_last; /* mean loss over the first and the last epoch */
    double ms;                   /* wall time of data generation and training */
    int64_t steps;
} dgp_train_stats;

/* Load network parameters from host memory (n_params = DGP_MLP_PARAMS). Synchronous. */
dgp_status dgp_mlp_load(dgp_ctx *ctx, const float *params, int64_t n_params);

/* Build a rule for every element of the uploaded mesh (requires dgp_pattern):
 * element data, initial rule (init = DGP_INIT_NETWORK needs loaded or trained
 * parameters), at most max_iters damped Gauss-Newton steps (stopping at tol), the
 * acceptance flags.  With DGP_INIT_NETWORK each element starts from the
 * network's rule or the template's, whichever has the smaller moment residual,
 * for at most 3/4 of max_iters steps; an element not accepted then is refined
 * again from the template for max_iters steps (its steps count both
 * attempts).  Synchronous; fills *out if non-NULL. */
dgp_status dgp_qrule_build(dgp_ctx *ctx, int init, int max_iters, double tol, dgp_qrule_stats *out);

/* Copy the rules into caller-owned device buffers (any may be NULL):
 * nodes[n_cells][16][2] (xi, eta), weights[n_cells][16], accepted[n_cells],
 * residual[n_cells] (infinite for elements with more than 12 vertices),
 * iters[n_cells].  Asynchronous. */
dgp_status dgp_qrule_get(dgp_ctx *ctx, double *nodes, double *weights, uint8_t *accepted, double *residual,
                         int32_t *iters);

/* The element data behind the rules: features[n_cells][36] (float),
 * moments[n_cells][28], area[n_cells] (|P| in box coordinates).  Asynchronous. */
dgp_status dgp_qrule_cell_data(dgp_ctx *ctx, float *features, double *moments, double *area);

/* Training polygons first .. first+n-1 (device buffers): features[n][36]
 * (float), features64[n][36] (double, may be NULL), moments[n][28], area[n].
 * Polygon i: Philox-4x32-10 keyed by (seed low word, seed high word), counter
 * (i, j, 0, 0) for draw j; draw 0 fixes the vertex count 3 + floor(10 u0), the
 * kind (convex if u1 < 1/2, else star-shaped), the aspect 0.3 + 0.7 u2 and the
 * rotation 2 pi u3; draw j >= 1 places vertex j-1 at the angle
 * 2 pi (j-1 + 0.1 + 0.8 u0) / m + rotation, on the ellipse (cos, aspect sin)
 * or at radius 0.35 + 0.65 u1; u = (word >> 8) / 2^24.  The polygon is then
 * normalised to its bounding box and rotated as for the elements.
 * Asynchronous. */
dgp_status dgp_train_polygons(dgp_ctx *ctx, uint64_t seed, int64_t first, int64_t n, float *features,
                              double *features64, double *moments, double *area);

/* Network output out[n][48] for rows x[n][36]; params, x, out are device
 * pointers.  Synchronous (scratch is allocated and freed inside). */
dgp_status dgp_mlp_forward(dgp_ctx *ctx, const float *params, const float *x, int64_t n, float *out);

/* Gradient of the training loss, mean over the n rows of
 * sum_ab (Q_ab - M_ab)^2 / |P|^2, with respect to every parameter
 * (grad[DGP_MLP_PARAMS], blob layout), and the sum of the per-row losses into
 * loss_sum[0].  Device pointers.  Synchronous. */
dgp_status dgp_mlp_loss_grad(dgp_ctx *ctx, const float *params, const float *x, const double *moments,
                             const double *area, int64_t n, float *grad, float *loss_sum);

/* One Adam step (Kingma and Ba) on device arrays of n parameters, step t >= 1. */
dgp_status dgp_adam_step(dgp_ctx *ctx, float *params, const float *grad, float *m, float *v, int64_t n, int32_t t,
                         float lr, float beta1, float beta2, float eps);

/* Generate cfg->n_polygons training polygons on the device and train the
 * network with Adam on mini-batches in index order; the result becomes the
 * context's network and is copied to params_out (host, DGP_MLP_PARAMS floats,
 * may be NULL); epoch_loss[epochs] (host, may be NULL) receives the mean loss
 * of each epoch.  Synchronous. */
dgp_status dgp_mlp_train(dgp_ctx *ctx, const dgp_train_cfg *cfg, float *params_out, float *epoch_loss,
                         dgp_train_stats *stats);

#ifdef __cplusplus
}
#endif
#endif
