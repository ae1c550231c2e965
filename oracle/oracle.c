/*
 * FP64 CPU oracle for SIPG assembly on polytopic meshes -- TEST INFRASTRUCTURE.
 * Used only by the tests, the smoke check and the CPU-baseline leg of the
 * benchmark.  Shares no code with the GPU path.  See oracle.h for the
 * conventions and the passages of the paper each part follows.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846
#define MAXP 6
#define MAXNB 84 /* (6+1)(6+2)(6+3)/6 */

/* ---------------------------------------------------------------- Legendre */
/* Power-form coefficients of the Legendre polynomials,
 *   P_n(x) = 2^-n sum_k (-1)^k C(n,k) C(2n-2k,n) x^(n-2k),
 * evaluated by Horner's scheme (independent of any recurrence). */
static double leg[MAXP + 1][MAXP + 1];
static int leg_ready = 0;

static double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

static void leg_init(void) {
    if (leg_ready) return;
    memset(leg, 0, sizeof(leg));
    for (int n = 0; n <= MAXP; ++n) {
        for (int k = 0; 2 * k <= n; ++k) {
            double c = binom(n, k) * binom(2 * n - 2 * k, n) / pow(2.0, n);
            leg[n][n - 2 * k] = (k % 2 ? -c : c);
        }
    }
    leg_ready = 1;
}

static void legendre(int n, double x, double *P, double *dP) {
    for (int m = 0; m <= n; ++m) {
        double v = 0.0, d = 0.0;
        for (int e = m; e >= 0; --e) v = v * x + leg[m][e];
        for (int e = m; e >= 1; --e) d = d * x + e * leg[m][e];
        P[m] = v;
        dP[m] = d;
    }
}

int orc_nb(int dim, int p) {
    if (p < 0) return 0;
    return dim == 2 ? (p + 1) * (p + 2) / 2 : (p + 1) * (p + 2) * (p + 3) / 6;
}

/* hierarchical ordering: total degree k = 0..p; a descending, then b descending */
static int exponents(int dim, int p, int *ea, int *eb, int *ec) {
    int n = 0;
    for (int k = 0; k <= p; ++k) {
        for (int a = k; a >= 0; --a) {
            if (dim == 2) {
                ea[n] = a; eb[n] = k - a; ec[n] = 0; ++n;
            } else {
                for (int b = k - a; b >= 0; --b) {
                    ea[n] = a; eb[n] = b; ec[n] = k - a - b; ++n;
                }
            }
        }
    }
    return n;
}

/* The basis at the point ref + d, where ref lies in the box (a vertex of the
 * element or of its face) and d is the point's offset from it: the box
 * coordinate ((ref - lo) - (hi - ref) + 2 d) / (hi - lo) keeps the point's
 * position relative to the box to the rounding of d, whatever the size of the
 * absolute coordinates (a point stored as a double near 1 is known only to
 * 1e-16 absolutely, i.e. 1e-13 relative to a cell of size 1e-3). */
static int basis_rel(int dim, int p, const double *lo, const double *hi, const double *ref, const double *dx,
                     double *phi, double *grad) {
    if (p < 0 || p > MAXP || (dim != 2 && dim != 3)) return -3;
    leg_init();
    double P[3][MAXP + 1], dP[3][MAXP + 1], chain[3], box = 1.0;
    for (int d = 0; d < dim; ++d) {
        double h = hi[d] - lo[d];
        box *= h;
        chain[d] = 2.0 / h;
        legendre(p, ((ref[d] - lo[d]) - (hi[d] - ref[d]) + 2.0 * dx[d]) / h, P[d], dP[d]);
    }
    int ea[MAXNB], eb[MAXNB], ec[MAXNB];
    int nb = exponents(dim, p, ea, eb, ec);
    for (int i = 0; i < nb; ++i) {
        int a = ea[i], b = eb[i], c = ec[i];
        if (dim == 2) {
            double s = sqrt((2.0 * a + 1) * (2.0 * b + 1) / box);
            phi[i] = s * P[0][a] * P[1][b];
            grad[2 * i + 0] = s * dP[0][a] * chain[0] * P[1][b];
            grad[2 * i + 1] = s * P[0][a] * dP[1][b] * chain[1];
        } else {
            double s = sqrt((2.0 * a + 1) * (2.0 * b + 1) * (2.0 * c + 1) / box);
            phi[i] = s * P[0][a] * P[1][b] * P[2][c];
            grad[3 * i + 0] = s * dP[0][a] * chain[0] * P[1][b] * P[2][c];
            grad[3 * i + 1] = s * P[0][a] * dP[1][b] * chain[1] * P[2][c];
            grad[3 * i + 2] = s * P[0][a] * P[1][b] * dP[2][c] * chain[2];
        }
    }
    return nb;
}

int orc_basis(int dim, int p, const double *lo, const double *hi, const double *x, double *phi, double *grad) {
    const double zero[3] = {0.0, 0.0, 0.0};
    return basis_rel(dim, p, lo, hi, x, zero, phi, grad);
}

/* ------------------------------------------------- coefficients and data */
/* sin(pi x) and cos(pi x) with the argument reduced exactly (shifts by whole
 * periods are exact in binary floating point), so that sin(pi k) = 0 and
 * cos(pi (k + 1/2)) = 0 hold exactly at integer and half-integer points. */
static double sinpi_(double x) {
    double r = x - 2.0 * floor(0.5 * x); /* [0, 2) */
    if (r > 1.5) return sin(PI * (r - 2.0));
    if (r > 0.5) return sin(PI * (1.0 - r));
    return sin(PI * r);
}

static double cospi_(double x) { return sinpi_(x + 0.5); }

static double coef_a(const orc_problem *pr, const double *x) {
    return pr->a0 + pr->a1 * sinpi_(2 * x[0]) * cospi_(2 * x[1]);
}

static void coef_grad_a(const orc_problem *pr, const double *x, double *g) {
    g[0] = pr->a1 * 2 * PI * cospi_(2 * x[0]) * cospi_(2 * x[1]);
    g[1] = -pr->a1 * 2 * PI * sinpi_(2 * x[0]) * sinpi_(2 * x[1]);
    g[2] = 0.0;
}

static void exact_u(const orc_problem *pr, int dim, const double *x, double *u, double *gu, double *lap) {
    double X = x[0], Y = x[1], Z = dim == 3 ? x[2] : 0.0;
    if (pr->u_kind == ORC_U_SIN) {
        double sx = sinpi_(X), cx = cospi_(X), sy = sinpi_(Y), cy = cospi_(Y);
        double sz = dim == 3 ? sinpi_(Z) : 1.0, cz = dim == 3 ? cospi_(Z) : 0.0;
        *u = sx * sy * sz;
        gu[0] = PI * cx * sy * sz;
        gu[1] = PI * sx * cy * sz;
        gu[2] = dim == 3 ? PI * sx * sy * cz : 0.0;
        *lap = -dim * PI * PI * (*u);
    } else {
        const double *c = pr->u_poly;
        *u = c[0] + c[1] * X + c[2] * Y + c[3] * Z + c[4] * X * X + c[5] * Y * Y + c[6] * Z * Z
             + c[7] * X * Y + c[8] * X * Z + c[9] * Y * Z;
        gu[0] = c[1] + 2 * c[4] * X + c[7] * Y + c[8] * Z;
        gu[1] = c[2] + 2 * c[5] * Y + c[7] * X + c[9] * Z;
        gu[2] = dim == 3 ? c[3] + 2 * c[6] * Z + c[8] * X + c[9] * Y : 0.0;
        *lap = 2 * c[4] + 2 * c[5] + (dim == 3 ? 2 * c[6] : 0.0);
    }
}

/* equation (CDR) with A = a I:  f = -(grad a . grad u + a lap u) + b . grad u + c u */
void orc_exact(const orc_problem *pr, int dim, const double *x, double *u, double *f) {
    double gu[3], ga[3], lap;
    exact_u(pr, dim, x, u, gu, &lap);
    coef_grad_a(pr, x, ga);
    double a = coef_a(pr, x);
    double s = 0.0;
    for (int d = 0; d < dim; ++d) s += -ga[d] * gu[d] + pr->b[d] * gu[d];
    *f = s - a * lap + pr->c * (*u);
}

/* ------------------------------------------------------------- quadrature */
static const orc_rule *tri_rule_for(const orc_rules *ru, int p) {
    int deg = p * 2 > 4 ? p * 2 : 4;
    if (deg == 4) return &ru->tri[0];
    if (deg == 6) return &ru->tri[1];
    if (deg == 8) return &ru->tri[2];
    return NULL;
}

static void vtx(const orc_mesh *m, int v, double *out) {
    out[0] = m->x[v];
    out[1] = m->y[v];
    out[2] = m->dim == 3 ? m->z[v] : 0.0;
}

/* Volume quadrature points of cell c for degree p: simplices of the
 * subdivision times the reference rule.  Returns the count (malloc'ed X, W). */
/* 2D: also the offsets D[3 q ..] of the points from the fan apex v0 (ref, 3
 * doubles), D = l1 (v1 - v0) + l2 (v2 - v0), and X = v0 + D; the basis is
 * evaluated from (ref, D) (basis_rel), the coefficients at X.  3D: D = 0 and
 * ref unused (the basis takes X). */
static int64_t vol_points(const orc_mesh *m, const orc_rules *ru, int64_t c, int p, double **X, double **W,
                          double **D, double *ref) {
    int64_t s = m->cell_ptr[c], e = m->cell_ptr[c + 1];
    if (m->dim == 2) {
        const orc_rule *r = tri_rule_for(ru, p);
        if (!r) return -3;
        int64_t nv = e - s, nt = nv - 2;
        if (nt < 1) return -2;
        *X = (double *)malloc(sizeof(double) * 3 * nt * r->n);
        *W = (double *)malloc(sizeof(double) * nt * r->n);
        double *Dq = (double *)malloc(sizeof(double) * 3 * nt * r->n);
        int64_t q = 0;
        double v0[3], v1[3], v2[3];
        vtx(m, m->cell_vtx[s], v0);
        for (int d = 0; d < 3; ++d) ref[d] = v0[d];
        for (int64_t t = 0; t < nt; ++t) {
            vtx(m, m->cell_vtx[s + 1 + t], v1);
            vtx(m, m->cell_vtx[s + 2 + t], v2);
            double area = 0.5 * ((v1[0] - v0[0]) * (v2[1] - v0[1]) - (v2[0] - v0[0]) * (v1[1] - v0[1]));
            for (int k = 0; k < r->n; ++k, ++q) {
                const double *l = r->pts + 3 * k;
                for (int d = 0; d < 3; ++d) {
                    Dq[3 * q + d] = l[1] * (v1[d] - v0[d]) + l[2] * (v2[d] - v0[d]);
                    (*X)[3 * q + d] = v0[d] + Dq[3 * q + d];
                }
                (*W)[q] = r->w[k] * area;
            }
        }
        if (D)
            *D = Dq;
        else
            free(Dq);
        return q;
    } else {
        const orc_rule *r = &ru->tet;
        int64_t nt = (e - s) / 4;
        if (nt < 1 || (e - s) % 4) return -2;
        *X = (double *)malloc(sizeof(double) * 3 * nt * r->n);
        *W = (double *)malloc(sizeof(double) * nt * r->n);
        if (D) *D = (double *)calloc((size_t)(3 * nt * r->n), sizeof(double));
        if (ref) ref[0] = ref[1] = ref[2] = 0.0;
        int64_t q = 0;
        for (int64_t t = 0; t < nt; ++t) {
            double v[4][3];
            for (int j = 0; j < 4; ++j) vtx(m, m->cell_vtx[s + 4 * t + j], v[j]);
            double a[3], b[3], cc[3];
            for (int d = 0; d < 3; ++d) {
                a[d] = v[1][d] - v[0][d];
                b[d] = v[2][d] - v[0][d];
                cc[d] = v[3][d] - v[0][d];
            }
            double det = a[0] * (b[1] * cc[2] - b[2] * cc[1]) - a[1] * (b[0] * cc[2] - b[2] * cc[0])
                         + a[2] * (b[0] * cc[1] - b[1] * cc[0]);
            double vol = fabs(det) / 6.0;
            for (int k = 0; k < r->n; ++k, ++q) {
                const double *l = r->pts + 4 * k;
                for (int d = 0; d < 3; ++d)
                    (*X)[3 * q + d] = l[0] * v[0][d] + l[1] * v[1][d] + l[2] * v[2][d] + l[3] * v[3][d];
                (*W)[q] = r->w[k] * vol;
            }
        }
        return q;
    }
}

/* ---------------------------------------------------------------- geometry */
typedef struct {
    double lo[3], hi[3], meas, diam, abar;
} cellgeo;

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int cell_geometry(const orc_mesh *m, const orc_problem *pr, const orc_rules *ru, int64_t c, cellgeo *g) {
    int64_t s = m->cell_ptr[c], e = m->cell_ptr[c + 1];
    int dim = m->dim;
    int64_t n = e - s;
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    memcpy(ids, m->cell_vtx + s, sizeof(int32_t) * n);
    qsort(ids, n, sizeof(int32_t), cmp_i32);
    int64_t u = 0;
    for (int64_t i = 0; i < n; ++i)
        if (i == 0 || ids[i] != ids[i - 1]) ids[u++] = ids[i];
    for (int d = 0; d < 3; ++d) {
        g->lo[d] = INFINITY;
        g->hi[d] = -INFINITY;
    }
    for (int64_t i = 0; i < u; ++i) {
        double v[3];
        vtx(m, ids[i], v);
        for (int d = 0; d < dim; ++d) {
            if (v[d] < g->lo[d]) g->lo[d] = v[d];
            if (v[d] > g->hi[d]) g->hi[d] = v[d];
        }
    }
    /* h_kappa = diam(kappa): largest distance between two vertices */
    double diam2 = 0.0;
    for (int64_t i = 0; i < u; ++i) {
        double vi[3];
        vtx(m, ids[i], vi);
        for (int64_t j = i + 1; j < u; ++j) {
            double vj[3], d2 = 0.0;
            vtx(m, ids[j], vj);
            for (int d = 0; d < dim; ++d) d2 += (vi[d] - vj[d]) * (vi[d] - vj[d]);
            if (d2 > diam2) diam2 = d2;
        }
    }
    free(ids);
    g->diam = sqrt(diam2);
    /* |kappa|: shoelace (2D) or sum of sub-tetrahedron volumes (3D) */
    double *X = NULL, *W = NULL, ref[3];
    int64_t nq = vol_points(m, ru, c, m->cell_p[c], &X, &W, NULL, ref);
    if (nq < 0) return (int)nq;
    if (dim == 2) {
        /* shoelace about the first vertex: the terms are products of coordinate
         * differences (exact), so the area keeps its relative precision on
         * small cells far from the origin */
        double a2 = 0.0, o[3];
        vtx(m, m->cell_vtx[s], o);
        for (int64_t i = 0; i < n; ++i) {
            double p0[3], p1[3];
            vtx(m, m->cell_vtx[s + i], p0);
            vtx(m, m->cell_vtx[s + (i + 1) % n], p1);
            a2 += (p0[0] - o[0]) * (p1[1] - o[1]) - (p1[0] - o[0]) * (p0[1] - o[1]);
        }
        g->meas = 0.5 * a2;
    } else {
        double v = 0.0;
        for (int64_t q = 0; q < nq; ++q) v += W[q];
        g->meas = v;
    }
    /* abar_kappa = ||a||_{L_inf(kappa)}, taken over the volume quadrature points */
    double amax = -INFINITY;
    for (int64_t q = 0; q < nq; ++q) {
        double a = coef_a(pr, X + 3 * q);
        if (a > amax) amax = a;
    }
    g->abar = amax;
    free(X);
    free(W);
    return 0;
}

int orc_geometry(const orc_mesh *m, const orc_problem *pr, const orc_rules *ru,
                 double *lo, double *hi, double *meas, double *diam, double *abar) {
    leg_init();
    for (int64_t c = 0; c < m->n_cells; ++c) {
        cellgeo g;
        int rc = cell_geometry(m, pr, ru, c, &g);
        if (rc) return rc;
        for (int d = 0; d < 3; ++d) {
            lo[3 * c + d] = g.lo[d];
            hi[3 * c + d] = g.hi[d];
        }
        meas[c] = g.meas;
        diam[c] = g.diam;
        abar[c] = g.abar;
    }
    return 0;
}

/* ----------------------------------------------------------------- pattern */
/* sorted unique {c} U {elements sharing a face with c}; returns count */
static int64_t row_cols(const orc_mesh *m, int64_t c, int32_t *out) {
    int64_t n = 0;
    out[n++] = (int32_t)c;
    for (int64_t k = m->cell_face_ptr[c]; k < m->cell_face_ptr[c + 1]; ++k) {
        int32_t f = m->cell_face[k];
        int32_t l = m->face_cell[2 * f], r = m->face_cell[2 * f + 1];
        int32_t o = (l == c) ? r : l;
        if (o >= 0 && o != c) out[n++] = o;
    }
    qsort(out, n, sizeof(int32_t), cmp_i32);
    int64_t u = 0;
    for (int64_t i = 0; i < n; ++i)
        if (i == 0 || out[i] != out[i - 1]) out[u++] = out[i];
    return u;
}

static int64_t max_faces(const orc_mesh *m) {
    int64_t mx = 0;
    for (int64_t c = 0; c < m->n_cells; ++c) {
        int64_t k = m->cell_face_ptr[c + 1] - m->cell_face_ptr[c];
        if (k > mx) mx = k;
    }
    return mx;
}

int orc_pattern_sizes(const orc_mesh *m, int64_t *nnzb, int64_t *n_vals, int64_t *n_dofs) {
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (max_faces(m) + 1));
    int64_t nz = 0, nv = 0, nd = 0;
    for (int64_t c = 0; c < m->n_cells; ++c) {
        int64_t k = row_cols(m, c, buf);
        int nbr = orc_nb(m->dim, m->cell_p[c]);
        nz += k;
        nd += nbr;
        for (int64_t j = 0; j < k; ++j) nv += (int64_t)nbr * orc_nb(m->dim, m->cell_p[buf[j]]);
    }
    free(buf);
    *nnzb = nz;
    *n_vals = nv;
    *n_dofs = nd;
    return 0;
}

int orc_pattern(const orc_mesh *m, int64_t *row_ptr, int32_t *col_idx, int64_t *val_ptr, int64_t *dof_ptr) {
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (max_faces(m) + 1));
    row_ptr[0] = 0;
    val_ptr[0] = 0;
    dof_ptr[0] = 0;
    for (int64_t c = 0; c < m->n_cells; ++c) {
        int64_t k = row_cols(m, c, buf);
        int nbr = orc_nb(m->dim, m->cell_p[c]);
        for (int64_t j = 0; j < k; ++j) {
            int64_t idx = row_ptr[c] + j;
            col_idx[idx] = buf[j];
            val_ptr[idx + 1] = val_ptr[idx] + (int64_t)nbr * orc_nb(m->dim, m->cell_p[buf[j]]);
        }
        row_ptr[c + 1] = row_ptr[c] + k;
        dof_ptr[c + 1] = dof_ptr[c] + nbr;
    }
    free(buf);
    return 0;
}

/* ------------------------------------------------------------- face data */
typedef struct {
    double n[3];      /* unit normal, outward from the row's element */
    double meas;      /* |F| */
    int npts;
    double X[64 * 3]; /* quadrature points */
    double W[64];
    double ref[3];    /* 2D: the face's first vertex; points X = ref + D */
    double D[64 * 3];
} facepts;

/* basis at a quadrature point: in 2D from its offset D to a mesh vertex ref
 * (basis_rel), in 3D from its coordinates */
static void eval_basis(int dim, int p, const double *lo, const double *hi, const double *x, const double *ref,
                       const double *d, double *phi, double *grad) {
    if (dim == 2)
        basis_rel(dim, p, lo, hi, ref, d, phi, grad);
    else
        orc_basis(dim, p, lo, hi, x, phi, grad);
}

static int face_points(const orc_mesh *m, const orc_rules *ru, int32_t f, int64_t row, int pmax,
                       const cellgeo *grow, facepts *fp) {
    int dim = m->dim;
    const int32_t *fv = m->face_vtx + (int64_t)dim * f;
    if (dim == 2) {
        double a[3], b[3];
        vtx(m, fv[0], a);
        vtx(m, fv[1], b);
        double t[2] = {b[0] - a[0], b[1] - a[1]};
        double len = sqrt(t[0] * t[0] + t[1] * t[1]);
        double n0[3] = {t[1] / len, -t[0] / len, 0.0};
        /* orient away from the row element: vertex average is interior for convex cells */
        double cen[2] = {0.0, 0.0};
        int64_t s = m->cell_ptr[row], e = m->cell_ptr[row + 1];
        for (int64_t i = s; i < e; ++i) {
            cen[0] += m->x[m->cell_vtx[i]];
            cen[1] += m->y[m->cell_vtx[i]];
        }
        cen[0] /= (double)(e - s);
        cen[1] /= (double)(e - s);
        double mid[2] = {0.5 * (a[0] + b[0]), 0.5 * (a[1] + b[1])};
        double sgn = ((mid[0] - cen[0]) * n0[0] + (mid[1] - cen[1]) * n0[1]) < 0 ? -1.0 : 1.0;
        for (int d = 0; d < 3; ++d) fp->n[d] = sgn * n0[d];
        fp->meas = len;
        int ng = pmax + 1 > 3 ? pmax + 1 : 3;
        if (ng >= 16) return -3;
        const orc_rule *r = &ru->seg[ng];
        fp->npts = r->n;
        for (int d = 0; d < 3; ++d) fp->ref[d] = a[d];
        for (int q = 0; q < r->n; ++q) {
            for (int d = 0; d < 3; ++d) {
                fp->D[3 * q + d] = r->pts[q] * (b[d] - a[d]);
                fp->X[3 * q + d] = a[d] + fp->D[3 * q + d];
            }
            fp->W[q] = r->w[q] * len;
        }
    } else {
        double v0[3], v1[3], v2[3], o[3];
        vtx(m, fv[0], v0);
        vtx(m, fv[1], v1);
        vtx(m, fv[2], v2);
        vtx(m, m->face_opp[f], o);
        double a[3], b[3];
        for (int d = 0; d < 3; ++d) {
            a[d] = v1[d] - v0[d];
            b[d] = v2[d] - v0[d];
        }
        double cr[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
        double len = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        double sgn = ((o[0] - v0[0]) * cr[0] + (o[1] - v0[1]) * cr[1] + (o[2] - v0[2]) * cr[2]) > 0 ? -1.0 : 1.0;
        if (m->face_cell[2 * f] != row) sgn = -sgn;
        for (int d = 0; d < 3; ++d) fp->n[d] = sgn * cr[d] / len;
        fp->meas = 0.5 * len;
        const orc_rule *r = &ru->tri[0];
        fp->npts = r->n;
        for (int q = 0; q < r->n; ++q) {
            const double *l = r->pts + 3 * q;
            for (int d = 0; d < 3; ++d) fp->X[3 * q + d] = l[0] * v0[d] + l[1] * v1[d] + l[2] * v2[d];
            fp->W[q] = r->w[q] * fp->meas;
        }
    }
    (void)grow;
    return 0;
}

/* ---------------------------------------------------------------- penalty */
/* Appendix A, one side of face f in 2D: the covering is the fan of cell c
 * (triangles (v0, v_t, v_t+1), t = 1..n-2); the sub-triangle having the edge
 * (v_k, v_k+1) as a side is t = k, except t = 1 for k = 0 and t = n - 2 for
 * k = n - 1.  Returns abar p^2 |F| min(1 / |K^F|, C_cov / |kappa|), C_cov = p^2,
 * or -1 if f is not an edge of c. */
static double covering_side(const orc_mesh *m, const cellgeo *g, int64_t c, int32_t f, double flen) {
    int64_t s = m->cell_ptr[c], n = m->cell_ptr[c + 1] - s;
    int64_t k = -1;
    for (int64_t i = 0; i < n; ++i)
        if (m->cell_face[s + i] == f) k = i;
    if (k < 0) return -1.0;
    int64_t t = k == 0 ? 1 : (k == n - 1 ? n - 2 : k);
    double v0[3], v1[3], v2[3];
    vtx(m, m->cell_vtx[s], v0);
    vtx(m, m->cell_vtx[s + t], v1);
    vtx(m, m->cell_vtx[s + t + 1], v2);
    double kf = 0.5 * fabs((v1[0] - v0[0]) * (v2[1] - v0[1]) - (v2[0] - v0[0]) * (v1[1] - v0[1]));
    int p = m->cell_p[c];
    double inv_k = 1.0 / kf; /* a degenerate sub-triangle leaves the C_cov bound */
    double cov = (double)(p * p) / g->meas;
    return g->abar * p * p * flen * (inv_k < cov ? inv_k : cov);
}

/* sigma_F (Appendix A) for face f of row r; o = the other element or -1 */
static double face_sigma(const orc_mesh *m, const orc_problem *pr, const cellgeo *geo, int64_t r, int32_t o,
                         int32_t f, double flen) {
    if (pr->sigma_override >= 0) return pr->sigma_override;
    int p_r = m->cell_p[r];
    if (pr->penalty == ORC_PEN_COVERING) {
        double s1 = covering_side(m, &geo[r], r, f, flen);
        double s2 = o >= 0 ? covering_side(m, &geo[o], o, f, flen) : 0.0;
        return pr->c_sigma * (s1 > s2 ? s1 : s2);
    }
    double s1 = geo[r].abar * p_r * p_r / geo[r].diam;
    double s2 = 0.0;
    if (o >= 0) {
        int p_o = m->cell_p[o];
        s2 = geo[o].abar * p_o * p_o / geo[o].diam;
    }
    return pr->c_sigma * (s1 > s2 ? s1 : s2);
}

static double dotn(const double *g, const double *n, int dim) {
    double s = 0.0;
    for (int d = 0; d < dim; ++d) s += g[d] * n[d];
    return s;
}

/* ---------------------------------------------------------------- assembly */
static int assemble_row(const orc_mesh *m, const orc_problem *pr, const orc_rules *ru, const cellgeo *geo,
                        const int64_t *row_ptr, const int32_t *col_idx, const int64_t *val_ptr,
                        const int64_t *dof_ptr, int64_t r, double *vals, double *rhs) {
    const int dim = m->dim;
    const int pr_ = m->cell_p[r];
    const int nbr = orc_nb(dim, pr_);
    const cellgeo *gr = &geo[r];
    int64_t k0 = row_ptr[r], k1 = row_ptr[r + 1];
    int64_t kd = -1;
    for (int64_t k = k0; k < k1; ++k)
        if (col_idx[k] == r) kd = k;
    if (kd < 0) return -2;
    for (int64_t v = val_ptr[k0]; v < val_ptr[k1]; ++v) vals[v] = 0.0;
    double *F = rhs + dof_ptr[r];
    for (int i = 0; i < nbr; ++i) F[i] = 0.0;
    double *D = vals + val_ptr[kd];

    double phi[MAXNB], grad[MAXNB * 3], phio[MAXNB], grado[MAXNB * 3];

    /* element term: first line of (dg-bilinear) and the f-term of (dg-linear) */
    if (pr->term_mask & (ORC_T_VOLUME | ORC_T_RHS)) {
        double *X = NULL, *W = NULL, *Dv = NULL, ref[3];
        int64_t nq = vol_points(m, ru, r, pr_, &X, &W, &Dv, ref);
        if (nq < 0) return (int)nq;
        for (int64_t q = 0; q < nq; ++q) {
            const double *x = X + 3 * q;
            eval_basis(dim, pr_, gr->lo, gr->hi, x, ref, Dv + 3 * q, phi, grad);
            double a = coef_a(pr, x), u, f;
            orc_exact(pr, dim, x, &u, &f);
            if (pr->term_mask & ORC_T_VOLUME) {
                for (int i = 0; i < nbr; ++i) {
                    for (int j = 0; j < nbr; ++j) {
                        double gg = 0.0, bg = 0.0;
                        for (int d = 0; d < dim; ++d) {
                            gg += grad[dim * j + d] * grad[dim * i + d];
                            bg += pr->b[d] * grad[dim * j + d];
                        }
                        D[i * nbr + j] += W[q] * (a * gg + bg * phi[i] + pr->c * phi[j] * phi[i]);
                    }
                }
            }
            if (pr->term_mask & ORC_T_RHS)
                for (int i = 0; i < nbr; ++i) F[i] += W[q] * f * phi[i];
        }
        free(X);
        free(W);
        free(Dv);
    }

    /* face terms: upwind, inflow-boundary and interior-penalty lines of
     * (dg-bilinear) and the boundary lines of (dg-linear), written for the
     * test functions of element r (row owner) */
    facepts fp;
    for (int64_t k = m->cell_face_ptr[r]; k < m->cell_face_ptr[r + 1]; ++k) {
        int32_t f = m->cell_face[k];
        int32_t lft = m->face_cell[2 * f], rgt = m->face_cell[2 * f + 1];
        if (lft != r && rgt != r) return -2;
        int32_t o = (lft == r) ? rgt : lft;
        int po = o >= 0 ? m->cell_p[o] : -1;
        int pmax = po > pr_ ? po : pr_;
        int rc = face_points(m, ru, f, r, pmax, gr, &fp);
        if (rc) return rc;
        const double *n = fp.n;
        double bn = dotn(pr->b, n, dim);
        if (o >= 0) {
            if (!(pr->term_mask & ORC_T_INTERIOR)) continue;
            const cellgeo *go = &geo[o];
            int nbo = orc_nb(dim, po);
            double sigma = face_sigma(m, pr, geo, r, o, f, fp.meas);
            int64_t kc = -1;
            for (int64_t kk = k0; kk < k1; ++kk)
                if (col_idx[kk] == o) kc = kk;
            if (kc < 0) return -2;
            double *C = vals + val_ptr[kc];
            for (int q = 0; q < fp.npts; ++q) {
                const double *x = fp.X + 3 * q;
                double w = fp.W[q];
                eval_basis(dim, pr_, gr->lo, gr->hi, x, fp.ref, fp.D + 3 * q, phi, grad);
                eval_basis(dim, po, go->lo, go->hi, x, fp.ref, fp.D + 3 * q, phio, grado);
                double a = coef_a(pr, x);
                int up = bn < 0.0; /* x in the inflow part of the boundary of r */
                for (int i = 0; i < nbr; ++i) {
                    double dni = dotn(grad + dim * i, n, dim);
                    for (int j = 0; j < nbr; ++j) {
                        double dnj = dotn(grad + dim * j, n, dim);
                        double s = -0.5 * a * dnj * phi[i] - 0.5 * a * dni * phi[j] + sigma * phi[j] * phi[i];
                        if (up) s -= bn * phi[j] * phi[i];
                        D[i * nbr + j] += w * s;
                    }
                    for (int j = 0; j < nbo; ++j) {
                        double dnj = dotn(grado + dim * j, n, dim);
                        double s = -0.5 * a * dnj * phi[i] + 0.5 * a * dni * phio[j] - sigma * phio[j] * phi[i];
                        if (up) s += bn * phio[j] * phi[i];
                        C[i * nbo + j] += w * s;
                    }
                }
            }
        } else if (m->face_bc[f] == 1) {
            double sigma = face_sigma(m, pr, geo, r, -1, f, fp.meas);
            for (int q = 0; q < fp.npts; ++q) {
                const double *x = fp.X + 3 * q;
                double w = fp.W[q];
                eval_basis(dim, pr_, gr->lo, gr->hi, x, fp.ref, fp.D + 3 * q, phi, grad);
                double a = coef_a(pr, x), g, fdummy;
                orc_exact(pr, dim, x, &g, &fdummy);
                int up = bn < 0.0;
                for (int i = 0; i < nbr; ++i) {
                    double dni = dotn(grad + dim * i, n, dim);
                    if (pr->term_mask & ORC_T_BOUNDARY) {
                        for (int j = 0; j < nbr; ++j) {
                            double dnj = dotn(grad + dim * j, n, dim);
                            double s = -a * dnj * phi[i] - a * dni * phi[j] + sigma * phi[j] * phi[i];
                            if (up) s -= bn * phi[j] * phi[i];
                            D[i * nbr + j] += w * s;
                        }
                    }
                    if (pr->term_mask & ORC_T_RHS) {
                        double s = -g * a * dni + sigma * g * phi[i];
                        if (up) s -= bn * g * phi[i];
                        F[i] += w * s;
                    }
                }
            }
        } else if (m->face_bc[f] == 2) {
            if (!(pr->term_mask & ORC_T_RHS)) continue;
            for (int q = 0; q < fp.npts; ++q) {
                const double *x = fp.X + 3 * q;
                double u, gu[3], lap;
                eval_basis(dim, pr_, gr->lo, gr->hi, x, fp.ref, fp.D + 3 * q, phi, grad);
                exact_u(pr, dim, x, &u, gu, &lap);
                double gN = coef_a(pr, x) * dotn(gu, n, dim); /* n . (A grad u) */
                for (int i = 0; i < nbr; ++i) F[i] += fp.W[q] * gN * phi[i];
            }
        } else {
            return -2;
        }
    }
    return 0;
}

/* Threads the OpenMP build uses (1 in the plain build). */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_assemble(const orc_mesh *m, const orc_problem *pr, const orc_rules *ru,
                 const int64_t *row_ptr, const int32_t *col_idx, const int64_t *val_ptr,
                 const int64_t *dof_ptr, const int64_t *rows, int64_t n_rows,
                 double *vals, double *rhs) {
    if (!m || !pr || !ru || (m->dim != 2 && m->dim != 3)) return -1;
    if (pr->penalty != ORC_PEN_DIAMETER && pr->penalty != ORC_PEN_COVERING) return -1;
    if (pr->penalty == ORC_PEN_COVERING && m->dim != 2) return -3;
    leg_init();
    for (int64_t c = 0; c < m->n_cells; ++c)
        if (m->cell_p[c] < 0 || m->cell_p[c] > MAXP || (m->dim == 2 && m->cell_p[c] > 4)) return -3;
    /* geometry of the requested rows and their neighbours */
    cellgeo *geo = (cellgeo *)calloc((size_t)m->n_cells, sizeof(cellgeo));
    char *need = (char *)calloc((size_t)m->n_cells, 1);
    int64_t nr = rows ? n_rows : m->n_cells;
    for (int64_t t = 0; t < nr; ++t) {
        int64_t r = rows ? rows[t] : t;
        if (r < 0 || r >= m->n_cells) {
            free(geo);
            free(need);
            return -1;
        }
        need[r] = 1;
        for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) need[col_idx[k]] = 1;
    }
    int rc = 0;
    /* Rows are independent (each writes only its own blocks and load), so the
     * OpenMP build (liboracle_omp.so, the CPU baseline on all host cores)
     * splits them over threads; the plain build runs them in order.  Both
     * compute every row with the same arithmetic in the same order. */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) reduction(| : rc)
#endif
    for (int64_t c = 0; c < m->n_cells; ++c)
        if (need[c]) rc |= cell_geometry(m, pr, ru, c, &geo[c]) != 0;
    int err = 0; /* the most negative row status (0 if every row assembled) */
    if (!rc) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) reduction(min : err)
#endif
        for (int64_t t = 0; t < nr; ++t) {
            int64_t r = rows ? rows[t] : t;
            int e = assemble_row(m, pr, ru, geo, row_ptr, col_idx, val_ptr, dof_ptr, r, vals, rhs);
            if (e < err) err = e;
        }
    }
    rc = rc ? -2 : err;
    free(geo);
    free(need);
    return rc;
}

/* ------------------------------------------------------------ space-time */
/* u = u_s T, T(t) = 1 + tau1 t + tau2 t^2; grad u = T grad u_s; f = u_s T' + T f_s */
static void st_exact(const orc_problem *pr, const orc_slab *sl, const double *x, double t, double *u, double *gu,
                     double *f) {
    double us, gus[3], lap, fs;
    exact_u(pr, 2, x, &us, gus, &lap);
    orc_exact(pr, 2, x, &us, &fs);
    double T = 1.0 + sl->tau1 * t + sl->tau2 * t * t, dT = sl->tau1 + 2.0 * sl->tau2 * t;
    *u = us * T;
    if (gu) {
        gu[0] = T * gus[0];
        gu[1] = T * gus[1];
    }
    if (f) *f = us * dT + T * fs;
}

/* Row r of the slab: the volume terms (time derivative, diffusion, advection,
 * reaction) on the prism, the time-jump term on its bottom, the face terms on
 * the space-time faces I_n x F, and the load. */
static int assemble_row_st(const orc_mesh *m, const orc_problem *pr, const orc_rules *ru, const orc_slab *sl,
                           const cellgeo *geo, const int64_t *row_ptr, const int32_t *col_idx,
                           const int64_t *val_ptr, const int64_t *dof_ptr, int64_t r, double *vals, double *rhs) {
    const int pr_ = m->cell_p[r];
    const int nbr = orc_nb(3, pr_);
    const cellgeo *gr = &geo[r];
    const double tau = sl->t1 - sl->t0;
    int64_t k0 = row_ptr[r], k1 = row_ptr[r + 1], kd = -1;
    for (int64_t k = k0; k < k1; ++k)
        if (col_idx[k] == r) kd = k;
    if (kd < 0) return -2;
    for (int64_t v = val_ptr[k0]; v < val_ptr[k1]; ++v) vals[v] = 0.0;
    double *F = rhs + dof_ptr[r];
    for (int i = 0; i < nbr; ++i) F[i] = 0.0;
    double *D = vals + val_ptr[kd];
    double lo[3] = {gr->lo[0], gr->lo[1], sl->t0}, hi[3] = {gr->hi[0], gr->hi[1], sl->t1};
    double phi[MAXNB], grad[MAXNB * 3], phio[MAXNB], grado[MAXNB * 3];
    /* Gauss in time with p + 1 points: exact for the degree-2p products */
    const orc_rule *gt = &ru->seg[pr_ + 1];

    double *X = NULL, *W = NULL, *Dv = NULL, ref[3];
    int64_t nq = vol_points(m, ru, r, pr_, &X, &W, &Dv, ref);
    if (nq < 0) return (int)nq;
    /* points as offsets from (fan apex, t0), as in 2D */
    const double ref3[3] = {ref[0], ref[1], sl->t0};
    for (int64_t q = 0; q < nq; ++q) {
        for (int k = 0; k < gt->n; ++k) {
            double t = sl->t0 + gt->pts[k] * tau;
            double w = W[q] * gt->w[k] * tau;
            double d3[3] = {Dv[3 * q], Dv[3 * q + 1], gt->pts[k] * tau};
            basis_rel(3, pr_, lo, hi, ref3, d3, phi, grad);
            double a = coef_a(pr, X + 3 * q), u, f;
            st_exact(pr, sl, X + 3 * q, t, &u, NULL, &f);
            for (int i = 0; i < nbr; ++i) {
                for (int j = 0; j < nbr; ++j) {
                    double gg = grad[3 * j] * grad[3 * i] + grad[3 * j + 1] * grad[3 * i + 1];
                    double bg = pr->b[0] * grad[3 * j] + pr->b[1] * grad[3 * j + 1];
                    D[i * nbr + j] += w * (grad[3 * j + 2] * phi[i] + a * gg + bg * phi[i] + pr->c * phi[j] * phi[i]);
                }
                F[i] += w * f * phi[i];
            }
        }
    }
    /* time jump at t0: (U^+, W^+) on the matrix side, (U^-_{n-1}, W^+) on the load side */
    for (int64_t q = 0; q < nq; ++q) {
        double d3[3] = {Dv[3 * q], Dv[3 * q + 1], 0.0};
        basis_rel(3, pr_, lo, hi, ref3, d3, phi, grad);
        double uprev;
        if (sl->prev) {
            double plo[3] = {gr->lo[0], gr->lo[1], sl->tp0}, phi_[3] = {gr->hi[0], gr->hi[1], sl->t0};
            basis_rel(3, pr_, plo, phi_, ref3, d3, phio, grado);
            uprev = 0.0;
            for (int j = 0; j < nbr; ++j) uprev += sl->prev[dof_ptr[r] + j] * phio[j];
        } else {
            st_exact(pr, sl, X + 3 * q, sl->t0, &uprev, NULL, NULL);
        }
        for (int i = 0; i < nbr; ++i) {
            for (int j = 0; j < nbr; ++j) D[i * nbr + j] += W[q] * phi[j] * phi[i];
            F[i] += W[q] * uprev * phi[i];
        }
    }
    free(X);
    free(W);
    free(Dv);

    const double hst_r = sqrt(gr->diam * gr->diam + tau * tau);
    facepts fp;
    for (int64_t kf = m->cell_face_ptr[r]; kf < m->cell_face_ptr[r + 1]; ++kf) {
        int32_t f = m->cell_face[kf];
        int32_t lft = m->face_cell[2 * f], rgt = m->face_cell[2 * f + 1];
        if (lft != r && rgt != r) return -2;
        int32_t o = (lft == r) ? rgt : lft;
        int po = o >= 0 ? m->cell_p[o] : -1;
        int pmax = po > pr_ ? po : pr_;
        int rc = face_points(m, ru, f, r, pmax, gr, &fp);
        if (rc) return rc;
        const double *n = fp.n;
        double bn = pr->b[0] * n[0] + pr->b[1] * n[1];
        double sigma;
        if (pr->sigma_override >= 0) {
            sigma = pr->sigma_override;
        } else {
            double s1 = gr->abar * pr_ * pr_ / hst_r, s2 = 0.0;
            if (o >= 0) {
                double hso = sqrt(geo[o].diam * geo[o].diam + tau * tau);
                s2 = geo[o].abar * po * po / hso;
            }
            sigma = pr->c_sigma * (s1 > s2 ? s1 : s2);
        }
        int nbo = o >= 0 ? orc_nb(3, po) : 0;
        double *C = NULL;
        double olo[3] = {0, 0, 0}, ohi[3] = {0, 0, 0};
        if (o >= 0) {
            for (int64_t kk = k0; kk < k1; ++kk)
                if (col_idx[kk] == o) C = vals + val_ptr[kk];
            if (!C) return -2;
            olo[0] = geo[o].lo[0], olo[1] = geo[o].lo[1], olo[2] = sl->t0;
            ohi[0] = geo[o].hi[0], ohi[1] = geo[o].hi[1], ohi[2] = sl->t1;
        }
        for (int q = 0; q < fp.npts; ++q) {
            for (int k = 0; k < gt->n; ++k) {
                double t = sl->t0 + gt->pts[k] * tau;
                double w = fp.W[q] * gt->w[k] * tau;
                const double fref[3] = {fp.ref[0], fp.ref[1], sl->t0};
                double d3[3] = {fp.D[3 * q], fp.D[3 * q + 1], gt->pts[k] * tau};
                basis_rel(3, pr_, lo, hi, fref, d3, phi, grad);
                double a = coef_a(pr, fp.X + 3 * q);
                int up = bn < 0.0;
                if (o >= 0) {
                    basis_rel(3, po, olo, ohi, fref, d3, phio, grado);
                    for (int i = 0; i < nbr; ++i) {
                        double dni = grad[3 * i] * n[0] + grad[3 * i + 1] * n[1];
                        for (int j = 0; j < nbr; ++j) {
                            double dnj = grad[3 * j] * n[0] + grad[3 * j + 1] * n[1];
                            double s = -0.5 * a * dnj * phi[i] - 0.5 * a * dni * phi[j] + sigma * phi[j] * phi[i];
                            if (up) s -= bn * phi[j] * phi[i];
                            D[i * nbr + j] += w * s;
                        }
                        for (int j = 0; j < nbo; ++j) {
                            double dnj = grado[3 * j] * n[0] + grado[3 * j + 1] * n[1];
                            double s = -0.5 * a * dnj * phi[i] + 0.5 * a * dni * phio[j] - sigma * phio[j] * phi[i];
                            if (up) s += bn * phio[j] * phi[i];
                            C[i * nbo + j] += w * s;
                        }
                    }
                } else if (m->face_bc[f] == 1) {
                    double g, gu[2];
                    st_exact(pr, sl, fp.X + 3 * q, t, &g, gu, NULL);
                    for (int i = 0; i < nbr; ++i) {
                        double dni = grad[3 * i] * n[0] + grad[3 * i + 1] * n[1];
                        for (int j = 0; j < nbr; ++j) {
                            double dnj = grad[3 * j] * n[0] + grad[3 * j + 1] * n[1];
                            double s = -a * dnj * phi[i] - a * dni * phi[j] + sigma * phi[j] * phi[i];
                            if (up) s -= bn * phi[j] * phi[i];
                            D[i * nbr + j] += w * s;
                        }
                        double s = -g * a * dni + sigma * g * phi[i];
                        if (up) s -= bn * g * phi[i];
                        F[i] += w * s;
                    }
                } else if (m->face_bc[f] == 2) {
                    double g, gu[2];
                    st_exact(pr, sl, fp.X + 3 * q, t, &g, gu, NULL);
                    double gN = a * (gu[0] * n[0] + gu[1] * n[1]);
                    for (int i = 0; i < nbr; ++i) F[i] += w * gN * phi[i];
                } else {
                    return -2;
                }
            }
        }
    }
    return 0;
}

int orc_assemble_st(const orc_mesh *m, const orc_problem *pr, const orc_rules *ru, const orc_slab *sl,
                    const int64_t *row_ptr, const int32_t *col_idx, const int64_t *val_ptr,
                    const int64_t *dof_ptr, const int64_t *rows, int64_t n_rows, double *vals, double *rhs) {
    if (!m || !pr || !ru || !sl || m->dim != 2 || m->n_cells <= 0 || !(sl->t1 > sl->t0)) return -1;
    if (pr->penalty != ORC_PEN_DIAMETER) return -3;
    if (sl->prev && !(sl->t0 > sl->tp0)) return -1;
    leg_init();
    for (int64_t c = 0; c < m->n_cells; ++c)
        if (m->cell_p[c] < 1 || m->cell_p[c] > 4) return -3;
    const int64_t ncell = m->n_cells;
    if (ncell > ((int64_t)1 << 31)) return -1;
    cellgeo *geo = (cellgeo *)calloc((size_t)ncell, sizeof(cellgeo));
    if (!geo) return -1;
    int rc = 0;
    for (int64_t c = 0; c < ncell && !rc; ++c) rc = cell_geometry(m, pr, ru, c, &geo[c]);
    int64_t nr = rows ? n_rows : ncell;
    int err = 0;
    if (!rc) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) reduction(min : err)
#endif
        for (int64_t t = 0; t < nr; ++t) {
            int64_t r = rows ? rows[t] : t;
            int e = (r < 0 || r >= m->n_cells) ? -1
                                                : assemble_row_st(m, pr, ru, sl, geo, row_ptr, col_idx, val_ptr,
                                                                  dof_ptr, r, vals, rhs);
            if (e < err) err = e;
        }
    }
    free(geo);
    return rc ? rc : err;
}
