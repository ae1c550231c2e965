/*
 * FP64 CPU oracle for SIPG assembly on polytopic meshes -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
 * library.  It shares no code with the GPU path.  Everything here is plain,
 * single-threaded double-precision C written to be checked against the paper
 * by eye:
 *
 *   bilinear form B(w, v)   -- Section 2.2, equation (dg-bilinear)
 *   linear functional l(v)  -- Section 2.2, equation (dg-linear)
 *   penalty sigma           -- Appendix A, read as sigma_F =
 *                              C_sigma * max_{kappa in F} abar_kappa p_kappa^2 / h_kappa,
 *                              or (2D) with the covering factor of Appendix A
 *                              (fan sub-triangles as the covering)
 *   basis                   -- Section 3.1: orthonormal tensor Legendre
 *                              polynomials of total degree p on the element's
 *                              bounding box, physical frame, hierarchical order
 *   quadrature              -- Section 3: standard rules on the simplices of a
 *                              subdivision (2D: fan from the first vertex;
 *                              3D: the given sub-tetrahedra) and on every face
 *   sparsity pattern        -- Section 3.4 (Approach 2): one block per element
 *                              and per pair of elements sharing at least one face
 *
 * Matrix convention: row = test function (element r, index i), column = trial
 * function (element c, index j); block (r, c) is row-major
 * n_b(p_r) x n_b(p_c) at vals[val_ptr[k]] where col_idx[k] == c.
 */
#ifndef DGP_ORACLE_H
#define DGP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t dim;
    int64_t n_vertices;
    const double *x, *y, *z;
    int64_t n_cells;
    const int64_t *cell_ptr;   /* 2D: CCW loop; 3D: 4 ids per sub-tetrahedron */
    const int32_t *cell_vtx;
    const int8_t *cell_p;
    const int64_t *cell_face_ptr;
    const int32_t *cell_face;
    int64_t n_faces;
    const int32_t *face_vtx;   /* dim ids per face */
    const int32_t *face_cell;  /* left, right (-1 = boundary) */
    const int8_t *face_bc;     /* 0 interior, 1 Dirichlet, 2 Neumann */
    const int32_t *face_opp;   /* 3D: left-cell tetrahedron vertex opposite the face */
} orc_mesh;

enum { ORC_U_SIN = 0, ORC_U_POLY = 1 };
enum { ORC_T_VOLUME = 1, ORC_T_INTERIOR = 2, ORC_T_BOUNDARY = 4, ORC_T_RHS = 8, ORC_T_ALL = 15 };

typedef struct {
    double a0, a1;          /* a(x) = a0 + a1 sin(2 pi x) cos(2 pi y), A = a I */
    double b[3];            /* constant advection field */
    double c;               /* constant reaction */
    double c_sigma;         /* penalty constant C_sigma */
    int32_t u_kind;         /* manufactured solution: product of sines or polynomial */
    double u_poly[10];      /* 1, x, y, z, x^2, y^2, z^2, xy, xz, yz */
    int32_t term_mask;      /* ORC_T_* bits: which terms to assemble */
    double sigma_override;  /* < 0: penalty formula; >= 0: this constant */
    int32_t penalty;        /* ORC_PEN_DIAMETER or ORC_PEN_COVERING */
} orc_problem;

/* Penalty formulas (Appendix A):
 *   ORC_PEN_DIAMETER  sigma_F = C_sigma max_kappa abar p^2 / h_kappa
 *   ORC_PEN_COVERING  sigma_F = C_sigma max_kappa abar p^2 |F| min(1 / |K^F|, C_cov / |kappa|)
 *                     with the fan sub-triangles as the covering, K^F the one
 *                     having F as a side, C_cov = p^2 (2D; every element taken
 *                     as p-coverable) */
enum { ORC_PEN_DIAMETER = 0, ORC_PEN_COVERING = 1 };

typedef struct {
    int32_t n;
    const double *pts;      /* [n*(d+1)] barycentric, or [n] on [0,1] */
    const double *w;        /* [n], summing to 1 */
} orc_rule;

typedef struct {
    orc_rule tri[3];        /* triangle rules of degree 4, 6, 8 */
    orc_rule seg[16];       /* seg[n]: n-point Gauss-Legendre on [0,1] (n >= 1) */
    orc_rule tet;           /* tetrahedron rule of degree 4 */
} orc_rules;

/* Number of basis functions of total degree p in dimension dim. */
int orc_nb(int dim, int p);

/* Basis values and physical gradients at a point x for a box [lo, hi];
 * phi[nb], grad[nb*dim]. Returns nb. */
int orc_basis(int dim, int p, const double *lo, const double *hi, const double *x, double *phi, double *grad);

/* Per-cell geometry: bbox lo/hi [n_cells*3 each], measure, diameter, abar. */
int orc_geometry(const orc_mesh *m, const orc_problem *pr, const orc_rules *ru,
                 double *lo, double *hi, double *meas, double *diam, double *abar);

int orc_pattern_sizes(const orc_mesh *m, int64_t *nnzb, int64_t *n_vals, int64_t *n_dofs);
int orc_pattern(const orc_mesh *m, int64_t *row_ptr, int32_t *col_idx, int64_t *val_ptr, int64_t *dof_ptr);

/* Assemble the block rows listed in rows[0..n_rows) (all rows if rows == NULL)
 * into vals / rhs (full-size arrays; other rows are left untouched).
 * Returns 0, or a negative code on malformed input. */
int orc_assemble(const orc_mesh *m, const orc_problem *pr, const orc_rules *ru,
                 const int64_t *row_ptr, const int32_t *col_idx, const int64_t *val_ptr,
                 const int64_t *dof_ptr, const int64_t *rows, int64_t n_rows,
                 double *vals, double *rhs);

/* Space-time slab I_n = (t0, t1] over a 2D mesh (Section 2.3, equation
 * spacetime_dg): prisms I_n x kappa with the total-degree-p space-time basis on
 * the box [lo_x, hi_x] x [lo_y, hi_y] x [t0, t1] (the 3D basis with t as the
 * third coordinate, n_b = (p+1)(p+2)(p+3)/6; blocks laid out as for a 3D
 * mesh).  The manufactured solution is u(x, y, t) = u_s(x, y) T(t), u_s as in
 * orc_problem, T = 1 + tau1 t + tau2 t^2, so f = u_s T' + T f_s.  The time jump
 * takes U_{n-1}^- from prev (the previous slab's coefficients on the box in
 * time [tp0, t0], same degrees and dof layout) or, if prev is NULL, the exact
 * u(., t0). */
typedef struct {
    double t0, t1, tp0;
    double tau1, tau2;
    const double *prev;
} orc_slab;

/* Rows of the slab system (diameter penalty with h = the prism's diameter;
 * the covering penalty is not defined here: -3). */
int orc_assemble_st(const orc_mesh *m, const orc_problem *pr, const orc_rules *ru, const orc_slab *sl,
                    const int64_t *row_ptr, const int32_t *col_idx, const int64_t *val_ptr,
                    const int64_t *dof_ptr, const int64_t *rows, int64_t n_rows, double *vals, double *rhs);

/* Threads used by orc_assemble: 1 in the plain build; the OpenMP build
 * (compiled with -fopenmp) assembles rows in parallel. */
int orc_threads(void);

/* Manufactured data at a point: u, f = -div(a grad u) + b.grad u + c u. */
void orc_exact(const orc_problem *pr, int dim, const double *x, double *u, double *f);

#ifdef __cplusplus
}
#endif
#endif
