/*
 * dg_oracle.c -- TEST INFRASTRUCTURE, not product code.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of the discontinuous
 * Galerkin discretisation of Uzunca & Karasozen, "A Matlab Tutorial for
 * Diffusion-Convection-Reaction Equations using DGFEM" (arXiv:1502.02941):
 *
 *     alpha u - eps Lap u + b . grad u = f   in Omega          (section 1, eq. 1)
 *     u = g^D on Gamma^D,  eps grad u . n = g^N on Gamma^N
 *
 * discretised by the interior penalty bilinear form a_h and load functional
 * l_h of section 1, eq. (ds), split into diffusion / convection / reaction
 * parts D_h, C_h, R_h as in section 2.3, eq. (dgscheme), and the linear system
 * of eq. (system) (row = test function phi_i, column = trial function phi_j).
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file's library.  It shares no code with the GPU library.
 *
 * Every integral is evaluated point by point, exactly as it is written in the
 * paper: basis functions are re-evaluated at every quadrature point from
 * their monomial coefficients, and edge traces are found by mapping the
 * physical point back into each neighbouring element.
 *
 * Readings of points the paper leaves open (each one is listed in the
 * project's design notes):
 *   - h_e is the edge length |e| (raised to the superpenalty exponent b0, =1
 *     in the paper's standard setting).
 *   - the boundary penalty is sigma_D (the caller passes 2*sigma, section 1:
 *     "twice the penalty on boundary edges"); Neumann edges get no penalty
 *     and no jump terms (the sums of a_h run over Gamma_0 u Gamma_D).
 *   - the Dirichlet symmetry term of l_h is  +kappa eps grad v . n g^D , which
 *     is the paper's  -eps grad v . n g^D  for SIPG (kappa=-1) and keeps the
 *     scheme consistent for NIPG and IIPG.
 *   - the inflow terms  -b.n u v  (a_h) and  -b.n g^D v  (l_h) act on the
 *     Dirichlet part of the inflow boundary only; on Neumann edges there is
 *     no convective boundary term.
 *   - upwinding is decided pointwise (per quadrature point), b.n < 0 strictly.
 *   - basis = orthonormal Dubiner basis on the reference triangle, vertex 1
 *     of an element row -> (0,0), vertex 2 -> (1,0), vertex 3 -> (0,1).
 *   - the alternative basis the paper's set_parameter names ("1: monomials",
 *     no formula) is xi^p eta^q on the same reference triangle, in the same
 *     order (total degree d = p+q, then q = 0..d); its mass matrix is full.
 *   - quadrature: Stroud conical product with q=k+2 points per direction on
 *     triangles, Gauss-Legendre with k+2 points on edges.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXK 6
#define ORC_MAXN (((ORC_MAXK) + 1) * ((ORC_MAXK) + 2) / 2)
#define ORC_MAXQ 24
#define ORC_NP ((ORC_MAXK) + 1) /* monomial table side */

enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_ORIENTATION = -2, ORC_ERR_BOUNDARY = -3,
       ORC_ERR_NONMANIFOLD = -4, ORC_ERR_DEGREE = -5, ORC_ERR_NOMEM = -9 };

enum { ORC_CONST = 0, ORC_AFFINE = 1, ORC_GAUSS_SUM = 2, ORC_POINTS = 3 };
enum { ORC_PART_D = 1, ORC_PART_C = 2, ORC_PART_R = 4 };

/* ------------------------------------------------------------------------ */
/* Jacobi polynomials P_n^{(a,b)}(x) by the standard three-term recurrence.  */
/* ------------------------------------------------------------------------ */
static double jacobi(int n, double a, double b, double x)
{
    if (n == 0) return 1.0;
    double p0 = 1.0;
    double p1 = 0.5 * (a - b + (a + b + 2.0) * x);
    for (int m = 2; m <= n; ++m) {
        double c = 2.0 * m + a + b;
        double a1 = 2.0 * m * (m + a + b) * (c - 2.0);
        double a2 = (c - 1.0) * (a * a - b * b);
        double a3 = (c - 2.0) * (c - 1.0) * c;
        double a4 = 2.0 * (m + a - 1.0) * (m + b - 1.0) * c;
        double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

static double jacobi_deriv(int n, double a, double b, double x)
{
    if (n == 0) return 0.0;
    return 0.5 * (n + a + b + 1.0) * jacobi(n - 1, a + 1.0, b + 1.0, x);
}

/* Gauss-Jacobi rule with n points for the weight (1-x)^a (1+x)^b on [-1,1]:
 * nodes = zeros of P_n^{(a,b)} found by Newton's method with deflation from
 * Chebyshev starting values; weights from the classical closed form
 *   w_i = 2^{a+b+1} G(n+a+1) G(n+b+1) / (G(n+a+b+1) n!) / ((1-x_i^2) P_n'(x_i)^2). */
static void gauss_jacobi(int n, double a, double b, double* x, double* w)
{
    for (int k = 0; k < n; ++k) {
        double r = -cos((2.0 * k + 1.0) * M_PI / (2.0 * n));
        if (k > 0) r = 0.5 * (r + x[k - 1]);
        for (int it = 0; it < 200; ++it) {
            double s = 0.0;
            for (int i = 0; i < k; ++i) s += 1.0 / (r - x[i]);
            double p = jacobi(n, a, b, r);
            double dp = jacobi_deriv(n, a, b, r);
            double delta = -p / (dp - s * p);
            r += delta;
            if (fabs(delta) < 1e-16) break;
        }
        x[k] = r;
    }
    /* sort ascending (Newton from Chebyshev guesses already is, keep it safe) */
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            if (x[j] < x[i]) { double t = x[i]; x[i] = x[j]; x[j] = t; }
    double c = pow(2.0, a + b + 1.0) * tgamma(n + a + 1.0) * tgamma(n + b + 1.0) /
               (tgamma(n + a + b + 1.0) * tgamma(n + 1.0));
    for (int i = 0; i < n; ++i) {
        double dp = jacobi_deriv(n, a, b, x[i]);
        w[i] = c / ((1.0 - x[i] * x[i]) * dp * dp);
    }
}

/* Volume rule on the reference triangle {xi,eta >= 0, xi+eta <= 1}: Stroud
 * conical product, Gauss-Legendre in a, Gauss-Jacobi(1,0) in b, with
 *   xi = (1+a)(1-b)/4,  eta = (1+b)/2,  weight = wa*wb/8.
 * Exact for total degree 2q-1.  Returns the number of points q*q. */
int orc_volume_rule(int q, double* xi, double* eta, double* w)
{
    if (q < 1 || q > ORC_MAXQ) return ORC_ERR_ARG;
    double a[ORC_MAXQ], wa[ORC_MAXQ], bb[ORC_MAXQ], wb[ORC_MAXQ];
    gauss_jacobi(q, 0.0, 0.0, a, wa);
    gauss_jacobi(q, 1.0, 0.0, bb, wb);
    int m = 0;
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) {
            xi[m] = 0.25 * (1.0 + a[i]) * (1.0 - bb[j]);
            eta[m] = 0.5 * (1.0 + bb[j]);
            w[m] = 0.125 * wa[i] * wb[j];
            ++m;
        }
    return m;
}

/* Gauss-Legendre rule with q points on [0,1]. */
int orc_edge_rule(int q, double* t, double* w)
{
    if (q < 1 || q > ORC_MAXQ) return ORC_ERR_ARG;
    double a[ORC_MAXQ], wa[ORC_MAXQ];
    gauss_jacobi(q, 0.0, 0.0, a, wa);
    for (int i = 0; i < q; ++i) {
        t[i] = 0.5 * (1.0 + a[i]);
        w[i] = 0.5 * wa[i];
    }
    return q;
}

/* ------------------------------------------------------------------------ */
/* Orthonormal Dubiner basis, built as monomial coefficients c[i][j] of      */
/* xi^i eta^j.  phi_{pq} = sqrt(2(2p+1)(p+q+1)) P_p(a) (1-eta)^p             */
/*                         P_q^{(2p+1,0)}(2 eta - 1),  a = 2 xi/(1-eta) - 1, */
/* ordered d = p+q = 0..k, then q = 0..d (p = d-q).                          */
/* ------------------------------------------------------------------------ */
typedef struct { double c[ORC_NP][ORC_NP]; } poly2;

static void poly_zero(poly2* p) { memset(p, 0, sizeof(*p)); }

/* r = p * (c0 + cx xi + ce eta) */
static void poly_mul_lin(const poly2* p, double c0, double cx, double ce, poly2* r)
{
    poly2 t;
    poly_zero(&t);
    for (int i = 0; i < ORC_NP; ++i)
        for (int j = 0; j < ORC_NP; ++j) {
            double v = p->c[i][j];
            if (v == 0.0) continue;
            t.c[i][j] += c0 * v;
            if (i + 1 < ORC_NP) t.c[i + 1][j] += cx * v;
            if (j + 1 < ORC_NP) t.c[i][j + 1] += ce * v;
        }
    *r = t;
}

static void poly_axpy(double s, const poly2* x, poly2* y)
{
    for (int i = 0; i < ORC_NP; ++i)
        for (int j = 0; j < ORC_NP; ++j) y->c[i][j] += s * x->c[i][j];
}

static void poly_mul(const poly2* p, const poly2* q, poly2* r)
{
    poly2 t;
    poly_zero(&t);
    for (int i = 0; i < ORC_NP; ++i)
        for (int j = 0; j < ORC_NP; ++j) {
            if (p->c[i][j] == 0.0) continue;
            for (int k = 0; i + k < ORC_NP; ++k)
                for (int l = 0; j + l < ORC_NP; ++l) t.c[i + k][j + l] += p->c[i][j] * q->c[k][l];
        }
    *r = t;
}

typedef struct {
    int k, n;
    poly2 phi[ORC_MAXN];
} basis_t;

enum { ORC_BASIS_DUBINER = 0, ORC_BASIS_MONOMIAL = 1 };

static void build_basis(int k, int basis, basis_t* B)
{
    B->k = k;
    B->n = (k + 1) * (k + 2) / 2;
    if (basis == ORC_BASIS_MONOMIAL) {
        int m = 0;
        for (int d = 0; d <= k; ++d)
            for (int q = 0; q <= d; ++q) {
                poly_zero(&B->phi[m]);
                B->phi[m].c[d - q][q] = 1.0;  /* xi^p eta^q, p = d - q */
                ++m;
            }
        return;
    }
    /* Q_p = P_p(a) (1-eta)^p :  Q_0 = 1, Q_1 = 2xi + eta - 1,
     * (p+1) Q_{p+1} = (2p+1)(2xi + eta - 1) Q_p - p (1-eta)^2 Q_{p-1}
     * (Legendre's recurrence multiplied through by (1-eta)^{p+1}). */
    poly2 Q[ORC_NP];
    poly_zero(&Q[0]);
    Q[0].c[0][0] = 1.0;
    if (k >= 1) { poly_zero(&Q[1]); Q[1].c[0][0] = -1.0; Q[1].c[1][0] = 2.0; Q[1].c[0][1] = 1.0; }
    for (int p = 1; p < k; ++p) {
        poly2 t1, t2;
        poly_mul_lin(&Q[p], -1.0, 2.0, 1.0, &t1);
        poly_mul_lin(&Q[p - 1], 1.0, 0.0, -1.0, &t2);
        poly_mul_lin(&t2, 1.0, 0.0, -1.0, &t2);
        poly_zero(&Q[p + 1]);
        poly_axpy((2.0 * p + 1.0) / (p + 1.0), &t1, &Q[p + 1]);
        poly_axpy(-(double)p / (p + 1.0), &t2, &Q[p + 1]);
    }
    int m = 0;
    for (int d = 0; d <= k; ++d)
        for (int q = 0; q <= d; ++q) {
            int p = d - q;
            double al = 2.0 * p + 1.0;
            /* R_q(eta) = P_q^{(al,0)}(x), x = 2 eta - 1, by the Jacobi recurrence
             * in polynomial arithmetic (only the eta column is used). */
            poly2 R[ORC_NP];
            poly_zero(&R[0]);
            R[0].c[0][0] = 1.0;
            if (q >= 1) {
                poly_zero(&R[1]);
                /* 0.5 (al + (al+2) x) with x = 2 eta - 1 */
                R[1].c[0][0] = 0.5 * (al - (al + 2.0));
                R[1].c[0][1] = (al + 2.0);
            }
            for (int mm = 2; mm <= q; ++mm) {
                double c = 2.0 * mm + al;
                double a1 = 2.0 * mm * (mm + al) * (c - 2.0);
                double a2 = (c - 1.0) * (al * al);
                double a3 = (c - 2.0) * (c - 1.0) * c;
                double a4 = 2.0 * (mm + al - 1.0) * (mm - 1.0) * c;
                poly2 t1;
                /* (a2 + a3 x) R_{m-1} = (a2 - a3 + 2 a3 eta) R_{m-1} */
                poly_mul_lin(&R[mm - 1], a2 - a3, 0.0, 2.0 * a3, &t1);
                poly_zero(&R[mm]);
                poly_axpy(1.0 / a1, &t1, &R[mm]);
                poly_axpy(-a4 / a1, &R[mm - 2], &R[mm]);
            }
            poly2 ph;
            poly_mul(&Q[p], &R[q], &ph);
            double s = sqrt(2.0 * (2.0 * p + 1.0) * (p + q + 1.0));
            poly_zero(&B->phi[m]);
            poly_axpy(s, &ph, &B->phi[m]);
            ++m;
        }
}

/* value and reference gradient of every basis function at (xi, eta) */
static void eval_basis(const basis_t* B, double xi, double eta, double* v, double* dxi, double* deta)
{
    double px[ORC_NP], py[ORC_NP];
    px[0] = py[0] = 1.0;
    for (int i = 1; i < ORC_NP; ++i) { px[i] = px[i - 1] * xi; py[i] = py[i - 1] * eta; }
    for (int m = 0; m < B->n; ++m) {
        double s = 0.0, sx = 0.0, sy = 0.0;
        for (int i = 0; i <= B->k; ++i)
            for (int j = 0; i + j <= B->k; ++j) {
                double c = B->phi[m].c[i][j];
                s += c * px[i] * py[j];
                if (i > 0) sx += c * i * px[i - 1] * py[j];
                if (j > 0) sy += c * j * px[i] * py[j - 1];
            }
        v[m] = s;
        if (dxi) dxi[m] = sx;
        if (deta) deta[m] = sy;
    }
}

static int basis_ok(int basis) { return basis == ORC_BASIS_DUBINER || basis == ORC_BASIS_MONOMIAL; }

/* exported for the basis pins: values and reference gradients at points */
int orc_basis_eval(int k, int basis, int npts, const double* xi, const double* eta, double* v, double* dxi,
                   double* deta)
{
    if (k < 0 || k > ORC_MAXK) return ORC_ERR_DEGREE;
    if (!basis_ok(basis)) return ORC_ERR_ARG;
    basis_t B;
    build_basis(k, basis, &B);
    for (int p = 0; p < npts; ++p)
        eval_basis(&B, xi[p], eta[p], v + (size_t)p * B.n, dxi ? dxi + (size_t)p * B.n : NULL,
                   deta ? deta + (size_t)p * B.n : NULL);
    return B.n;
}

/* ------------------------------------------------------------------------ */
/* Mesh: elements (counter-clockwise vertex triples), edge classification.   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n_nodes, T;
    double* xy;    /* [n_nodes][2] */
    int32_t* el;   /* [T][3] */
    /* interior edges: K_i < K_j; (va, vb) in K_i's counter-clockwise order */
    int64_t n_int;
    int32_t* int_el;  /* [n_int][2] */
    int32_t* int_v;   /* [n_int][2] */
    /* boundary edges, (va, vb) in the element's counter-clockwise order */
    int64_t n_bnd;
    int32_t* bnd_el;  /* [n_bnd] */
    int32_t* bnd_v;   /* [n_bnd][2] */
    int32_t* bnd_type; /* 0 = Dirichlet, 1 = Neumann */
    double hmax;
} orc_mesh;

typedef struct { int32_t lo, hi, el, a, b; } half_edge;

static int cmp_half(const void* x, const void* y)
{
    const half_edge* p = (const half_edge*)x;
    const half_edge* q = (const half_edge*)y;
    if (p->lo != q->lo) return p->lo < q->lo ? -1 : 1;
    if (p->hi != q->hi) return p->hi < q->hi ? -1 : 1;
    if (p->el != q->el) return p->el < q->el ? -1 : 1;
    return 0;
}

typedef struct { int32_t lo, hi, type; } bc_key;

static int cmp_bc(const void* x, const void* y)
{
    const bc_key* p = (const bc_key*)x;
    const bc_key* q = (const bc_key*)y;
    if (p->lo != q->lo) return p->lo < q->lo ? -1 : 1;
    if (p->hi != q->hi) return p->hi < q->hi ? -1 : 1;
    return 0;
}

void orc_mesh_free(orc_mesh* M)
{
    if (!M) return;
    free(M->xy); free(M->el); free(M->int_el); free(M->int_v);
    free(M->bnd_el); free(M->bnd_v); free(M->bnd_type);
    free(M);
}

/* Builds the mesh from the four arrays of section 2.1 (0-based here):
 * nodes (x, y), elements (3 node ids, counter-clockwise), Dirichlet and
 * Neumann boundary edges (start, end node).  A boundary edge must be listed in
 * exactly one of the two; every listed edge must be a boundary edge. */
int orc_mesh_create(const double* xy, int64_t n_nodes, const int32_t* el, int64_t T,
                    const int32_t* dir, int64_t n_dir, const int32_t* neu, int64_t n_neu, orc_mesh** out)
{
    *out = NULL;
    if (n_nodes <= 0 || T <= 0 || !xy || !el) return ORC_ERR_ARG;
    orc_mesh* M = (orc_mesh*)calloc(1, sizeof(orc_mesh));
    if (!M) return ORC_ERR_NOMEM;
    M->n_nodes = n_nodes;
    M->T = T;
    M->xy = (double*)malloc(sizeof(double) * 2 * n_nodes);
    M->el = (int32_t*)malloc(sizeof(int32_t) * 3 * T);
    memcpy(M->xy, xy, sizeof(double) * 2 * n_nodes);
    memcpy(M->el, el, sizeof(int32_t) * 3 * T);
    for (int64_t K = 0; K < T; ++K) {
        for (int l = 0; l < 3; ++l)
            if (el[3 * K + l] < 0 || el[3 * K + l] >= n_nodes) { orc_mesh_free(M); return ORC_ERR_ARG; }
        const double* p1 = xy + 2 * el[3 * K];
        const double* p2 = xy + 2 * el[3 * K + 1];
        const double* p3 = xy + 2 * el[3 * K + 2];
        double det = (p2[0] - p1[0]) * (p3[1] - p1[1]) - (p3[0] - p1[0]) * (p2[1] - p1[1]);
        if (!(det > 0.0)) { orc_mesh_free(M); return ORC_ERR_ORIENTATION; }
    }
    half_edge* H = (half_edge*)malloc(sizeof(half_edge) * 3 * T);
    for (int64_t K = 0; K < T; ++K)
        for (int l = 0; l < 3; ++l) {
            int32_t a = el[3 * K + l], b = el[3 * K + (l + 1) % 3];
            half_edge h = { a < b ? a : b, a < b ? b : a, (int32_t)K, a, b };
            H[3 * K + l] = h;
        }
    qsort(H, 3 * T, sizeof(half_edge), cmp_half);
    bc_key* BC = (bc_key*)malloc(sizeof(bc_key) * (n_dir + n_neu + 1));
    for (int64_t i = 0; i < n_dir; ++i) {
        int32_t a = dir[2 * i], b = dir[2 * i + 1];
        bc_key k = { a < b ? a : b, a < b ? b : a, 0 };
        BC[i] = k;
    }
    for (int64_t i = 0; i < n_neu; ++i) {
        int32_t a = neu[2 * i], b = neu[2 * i + 1];
        bc_key k = { a < b ? a : b, a < b ? b : a, 1 };
        BC[n_dir + i] = k;
    }
    int64_t nbc = n_dir + n_neu;
    qsort(BC, nbc, sizeof(bc_key), cmp_bc);
    for (int64_t i = 1; i < nbc; ++i)
        if (cmp_bc(&BC[i - 1], &BC[i]) == 0) { free(H); free(BC); orc_mesh_free(M); return ORC_ERR_BOUNDARY; }
    M->int_el = (int32_t*)malloc(sizeof(int32_t) * 3 * T);
    M->int_v = (int32_t*)malloc(sizeof(int32_t) * 3 * T);
    M->bnd_el = (int32_t*)malloc(sizeof(int32_t) * 3 * T);
    M->bnd_v = (int32_t*)malloc(sizeof(int32_t) * 6 * T);
    M->bnd_type = (int32_t*)malloc(sizeof(int32_t) * 3 * T);
    int64_t used_bc = 0;
    int64_t i = 0;
    int err = ORC_OK;
    double hmax = 0.0;
    while (i < 3 * T) {
        int64_t j = i;
        while (j < 3 * T && H[j].lo == H[i].lo && H[j].hi == H[i].hi) ++j;
        int64_t cnt = j - i;
        double dx = xy[2 * H[i].b] - xy[2 * H[i].a], dy = xy[2 * H[i].b + 1] - xy[2 * H[i].a + 1];
        double len = sqrt(dx * dx + dy * dy);
        if (len > hmax) hmax = len;
        if (cnt == 2) {
            /* H is sorted by element id within a key, so H[i] is K_i (the lower index). */
            M->int_el[2 * M->n_int] = H[i].el;
            M->int_el[2 * M->n_int + 1] = H[i + 1].el;
            M->int_v[2 * M->n_int] = H[i].a;
            M->int_v[2 * M->n_int + 1] = H[i].b;
            if (H[i].el == H[i + 1].el || H[i + 1].a != H[i].b || H[i + 1].b != H[i].a) {
                err = ORC_ERR_NONMANIFOLD; break;
            }
            M->n_int++;
        } else if (cnt == 1) {
            bc_key key = { H[i].lo, H[i].hi, 0 };
            bc_key* f = nbc ? (bc_key*)bsearch(&key, BC, nbc, sizeof(bc_key), cmp_bc) : NULL;
            if (!f) { err = ORC_ERR_BOUNDARY; break; }
            ++used_bc;
            M->bnd_el[M->n_bnd] = H[i].el;
            M->bnd_v[2 * M->n_bnd] = H[i].a;
            M->bnd_v[2 * M->n_bnd + 1] = H[i].b;
            M->bnd_type[M->n_bnd] = f->type;
            M->n_bnd++;
        } else {
            err = ORC_ERR_NONMANIFOLD; break;
        }
        i = j;
    }
    free(H);
    free(BC);
    if (err == ORC_OK && used_bc != nbc) err = ORC_ERR_BOUNDARY; /* a listed edge is not on the boundary */
    if (err != ORC_OK) { orc_mesh_free(M); return err; }
    M->hmax = hmax;
    *out = M;
    return ORC_OK;
}

int64_t orc_mesh_counts(const orc_mesh* M, int64_t* out6)
{
    int64_t nd = 0, nn = 0;
    for (int64_t b = 0; b < M->n_bnd; ++b) {
        if (M->bnd_type[b] == 0) ++nd; else ++nn;
    }
    out6[0] = M->T; out6[1] = M->n_int; out6[2] = M->n_bnd; out6[3] = nd; out6[4] = nn; out6[5] = 0;
    return M->T;
}

double orc_mesh_hmax(const orc_mesh* M) { return M->hmax; }

void orc_mesh_edges(const orc_mesh* M, int32_t* int_el, int32_t* int_v, int32_t* bnd_el, int32_t* bnd_v, int32_t* bnd_type)
{
    memcpy(int_el, M->int_el, sizeof(int32_t) * 2 * M->n_int);
    memcpy(int_v, M->int_v, sizeof(int32_t) * 2 * M->n_int);
    memcpy(bnd_el, M->bnd_el, sizeof(int32_t) * M->n_bnd);
    memcpy(bnd_v, M->bnd_v, sizeof(int32_t) * 2 * M->n_bnd);
    memcpy(bnd_type, M->bnd_type, sizeof(int32_t) * M->n_bnd);
}

/* ------------------------------------------------------------------------ */
/* Geometry of the affine map F_K(xi,eta) = P1 + (P2-P1) xi + (P3-P1) eta.   */
/* ------------------------------------------------------------------------ */
typedef struct { double x1, y1, j11, j12, j21, j22, det, g11, g12, g21, g22; } affine_t;

static void element_map(const orc_mesh* M, int64_t K, affine_t* A)
{
    const double* p1 = M->xy + 2 * M->el[3 * K];
    const double* p2 = M->xy + 2 * M->el[3 * K + 1];
    const double* p3 = M->xy + 2 * M->el[3 * K + 2];
    A->x1 = p1[0]; A->y1 = p1[1];
    A->j11 = p2[0] - p1[0]; A->j12 = p3[0] - p1[0];
    A->j21 = p2[1] - p1[1]; A->j22 = p3[1] - p1[1];
    A->det = A->j11 * A->j22 - A->j12 * A->j21;
    /* G = J^{-T}: grad_x phi = G grad_ref phi */
    A->g11 = A->j22 / A->det;  A->g12 = -A->j21 / A->det;
    A->g21 = -A->j12 / A->det; A->g22 = A->j11 / A->det;
}

static void to_physical(const affine_t* A, double xi, double eta, double* x, double* y)
{
    *x = A->x1 + A->j11 * xi + A->j12 * eta;
    *y = A->y1 + A->j21 * xi + A->j22 * eta;
}

static void to_reference(const affine_t* A, double x, double y, double* xi, double* eta)
{
    double dx = x - A->x1, dy = y - A->y1;
    *xi = (A->j22 * dx - A->j12 * dy) / A->det;
    *eta = (-A->j21 * dx + A->j11 * dy) / A->det;
}

/* basis values and physical gradients of element K at physical point (x,y) */
static void eval_phys(const basis_t* B, const affine_t* A, double x, double y, double* v, double* gx, double* gy)
{
    double xi, eta, dxi[ORC_MAXN], deta[ORC_MAXN];
    to_reference(A, x, y, &xi, &eta);
    eval_basis(B, xi, eta, v, dxi, deta);
    for (int m = 0; m < B->n; ++m) {
        gx[m] = A->g11 * dxi[m] + A->g12 * deta[m];
        gy[m] = A->g21 * dxi[m] + A->g22 * deta[m];
    }
}

/* ------------------------------------------------------------------------ */
/* Coefficient fields                                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t kind;      /* ORC_CONST, ORC_AFFINE, ORC_GAUSS_SUM, ORC_POINTS */
    int32_t m;         /* number of Gaussians (GAUSS_SUM) */
    double c[16];      /* CONST: c0; AFFINE: c0 + c1 x + c2 y; GAUSS_SUM: (cx, cy, w, A) per term */
    const double* vals; /* POINTS: one value per point of the array the field is used on */
} orc_field;

static double field_at(const orc_field* F, double x, double y, int64_t pidx)
{
    switch (F->kind) {
    case ORC_CONST: return F->c[0];
    case ORC_AFFINE: return F->c[0] + F->c[1] * x + F->c[2] * y;
    case ORC_GAUSS_SUM: {
        double s = 0.0;
        for (int i = 0; i < F->m; ++i) {
            double dx = x - F->c[4 * i], dy = y - F->c[4 * i + 1], w = F->c[4 * i + 2];
            s += F->c[4 * i + 3] * exp(-(dx * dx + dy * dy) / (2.0 * w * w));
        }
        return s;
    }
    case ORC_POINTS: return F->vals[pidx];
    }
    return NAN;
}

typedef struct {
    int32_t degree;
    int32_t basis;   /* ORC_BASIS_DUBINER or ORC_BASIS_MONOMIAL */
    double sigma;    /* penalty on interior edges */
    double sigma_D;  /* penalty on Dirichlet edges (the paper: twice sigma) */
    double kappa;    /* -1 SIPG, +1 NIPG, 0 IIPG */
    double b0;       /* superpenalty exponent, 1 in the standard setting */
    orc_field eps, bx, by, alpha, f, gD, gN;
} orc_problem;

/* quadrature sizes used by the assembly: q = k+2 per direction / on edges */
int orc_nq(int k) { return (k + 2) * (k + 2); }
int orc_nqe(int k) { return k + 2; }

/* coordinates of the volume quadrature points, [T][nq][2] (f as POINTS uses this order) */
int orc_volume_points(const orc_mesh* M, int k, int q, double* out)
{
    double xi[ORC_MAXQ * ORC_MAXQ], eta[ORC_MAXQ * ORC_MAXQ], w[ORC_MAXQ * ORC_MAXQ];
    int nq = orc_volume_rule(q, xi, eta, w);
    if (nq < 0) return nq;
    (void)k;
    for (int64_t K = 0; K < M->T; ++K) {
        affine_t A;
        element_map(M, K, &A);
        for (int g = 0; g < nq; ++g)
            to_physical(&A, xi[g], eta[g], out + 2 * (K * nq + g), out + 2 * (K * nq + g) + 1);
    }
    return nq;
}

/* coordinates of the boundary-edge quadrature points, [n_bnd][nqe][2], and the
 * outward unit normal of each boundary edge [n_bnd][2] (gD / gN as POINTS). */
int orc_boundary_points(const orc_mesh* M, int q, double* out, double* normals)
{
    double t[ORC_MAXQ], w[ORC_MAXQ];
    int nqe = orc_edge_rule(q, t, w);
    if (nqe < 0) return nqe;
    for (int64_t b = 0; b < M->n_bnd; ++b) {
        const double* pa = M->xy + 2 * M->bnd_v[2 * b];
        const double* pb = M->xy + 2 * M->bnd_v[2 * b + 1];
        double dx = pb[0] - pa[0], dy = pb[1] - pa[1], len = sqrt(dx * dx + dy * dy);
        for (int g = 0; g < nqe; ++g) {
            out[2 * (b * nqe + g)] = pa[0] + t[g] * dx;
            out[2 * (b * nqe + g) + 1] = pa[1] + t[g] * dy;
        }
        if (normals) { normals[2 * b] = dy / len; normals[2 * b + 1] = -dx / len; }
    }
    return nqe;
}

/* ------------------------------------------------------------------------ */
/* Assembly of D + C + R (selected by `parts`) and F, section 1 eq. (ds),    */
/* section 2.3 eq. (dgscheme) and (system).                                  */
/* Output: diag[T][n][n] (block (K,K)), off_ij[n_int][n][n] (row K_i, column */
/* K_j), off_ji[n_int][n][n] (row K_j, column K_i), rhs[T][n].  Block entry  */
/* [a][c] = form(phi_c trial, phi_a test).                                   */
/* ------------------------------------------------------------------------ */
int orc_assemble(const orc_mesh* M, const orc_problem* P, uint32_t parts,
                 double* diag, double* off_ij, double* off_ji, double* rhs)
{
    const int k = P->degree;
    if (k < 0 || k > ORC_MAXK) return ORC_ERR_DEGREE;
    if (!basis_ok(P->basis)) return ORC_ERR_ARG;
    basis_t B;
    build_basis(k, P->basis, &B);
    const int n = B.n;
    const int q = k + 2;
    double xi[ORC_MAXQ * ORC_MAXQ], eta[ORC_MAXQ * ORC_MAXQ], wv[ORC_MAXQ * ORC_MAXQ];
    const int nq = orc_volume_rule(q, xi, eta, wv);
    double te[ORC_MAXQ], we[ORC_MAXQ];
    const int nqe = orc_edge_rule(q, te, we);
    const int useD = (parts & ORC_PART_D) != 0, useC = (parts & ORC_PART_C) != 0, useR = (parts & ORC_PART_R) != 0;
    /* eps, b and alpha are functions of (x, y) (section 2.2): no POINTS kind */
    if (P->eps.kind == ORC_POINTS || P->bx.kind == ORC_POINTS || P->by.kind == ORC_POINTS ||
        P->alpha.kind == ORC_POINTS)
        return ORC_ERR_ARG;

    memset(diag, 0, sizeof(double) * M->T * n * n);
    memset(off_ij, 0, sizeof(double) * M->n_int * n * n);
    memset(off_ji, 0, sizeof(double) * M->n_int * n * n);
    memset(rhs, 0, sizeof(double) * M->T * n);

    double v[ORC_MAXN], gx[ORC_MAXN], gy[ORC_MAXN];

    /* --- volume integrals: eps grad u . grad v + (b . grad u) v + alpha u v, and f v --- */
    for (int64_t K = 0; K < M->T; ++K) {
        affine_t A;
        element_map(M, K, &A);
        double* DK = diag + K * n * n;
        for (int g = 0; g < nq; ++g) {
            double x, y;
            to_physical(&A, xi[g], eta[g], &x, &y);
            eval_phys(&B, &A, x, y, v, gx, gy);
            const double dx = wv[g] * A.det; /* |det J| = det J > 0 */
            const double e = field_at(&P->eps, x, y, -1);
            const double b1 = field_at(&P->bx, x, y, -1), b2 = field_at(&P->by, x, y, -1);
            const double al = field_at(&P->alpha, x, y, -1);
            const double fv = field_at(&P->f, x, y, K * nq + g);
            for (int a = 0; a < n; ++a) {          /* test  phi_a */
                for (int c = 0; c < n; ++c) {      /* trial phi_c */
                    double s = 0.0;
                    if (useD) s += e * (gx[c] * gx[a] + gy[c] * gy[a]);
                    if (useC) s += (b1 * gx[c] + b2 * gy[c]) * v[a];
                    if (useR) s += al * v[c] * v[a];
                    DK[a * n + c] += dx * s;
                }
                rhs[K * n + a] += dx * fv * v[a];
            }
        }
    }

    /* --- interior edges e = K_i cap K_j, n_e pointing from K_i to K_j --- */
    double vs[2][ORC_MAXN], gxs[2][ORC_MAXN], gys[2][ORC_MAXN];
    for (int64_t e = 0; e < M->n_int; ++e) {
        int64_t Ks[2] = { M->int_el[2 * e], M->int_el[2 * e + 1] };
        affine_t As[2];
        element_map(M, Ks[0], &As[0]);
        element_map(M, Ks[1], &As[1]);
        const double* pa = M->xy + 2 * M->int_v[2 * e];
        const double* pb = M->xy + 2 * M->int_v[2 * e + 1];
        const double ex = pb[0] - pa[0], ey = pb[1] - pa[1];
        const double len = sqrt(ex * ex + ey * ey);
        const double nx = ey / len, ny = -ex / len; /* outward normal of K_i */
        const double he = pow(len, P->b0);
        for (int g = 0; g < nqe; ++g) {
            const double x = pa[0] + te[g] * ex, y = pa[1] + te[g] * ey;
            const double ds = we[g] * len;
            for (int s = 0; s < 2; ++s) eval_phys(&B, &As[s], x, y, vs[s], gxs[s], gys[s]);
            const double eps = field_at(&P->eps, x, y, -1);
            const double beta = field_at(&P->bx, x, y, -1) * nx + field_at(&P->by, x, y, -1) * ny;
            const double pen = P->sigma * eps / he;
            for (int T = 0; T < 2; ++T)            /* side of the test function */
                for (int a = 0; a < n; ++a)
                    for (int S = 0; S < 2; ++S)    /* side of the trial function */
                        for (int c = 0; c < n; ++c) {
                            const double sT = T == 0 ? 1.0 : -1.0, sS = S == 0 ? 1.0 : -1.0;
                            /* [v] = s_T v n_e, [u] = s_S u n_e; {eps grad w} = eps grad w / 2 */
                            const double jvx = sT * vs[T][a] * nx, jvy = sT * vs[T][a] * ny;
                            const double jux = sS * vs[S][c] * nx, juy = sS * vs[S][c] * ny;
                            const double avux = 0.5 * eps * gxs[S][c], avuy = 0.5 * eps * gys[S][c];
                            const double avvx = 0.5 * eps * gxs[T][a], avvy = 0.5 * eps * gys[T][a];
                            double val = 0.0;
                            if (useD) {
                                val += -(avux * jvx + avuy * jvy);
                                val += P->kappa * (avvx * jux + avvy * juy);
                                val += pen * (jux * jvx + juy * jvy);
                            }
                            if (useC) {
                                /* sum over K in {K_i, K_j} with b.n_K < 0 of b.n_K (u_out - u_in) v|_K */
                                for (int Kk = 0; Kk < 2; ++Kk) {
                                    const double bnK = Kk == 0 ? beta : -beta;
                                    if (!(bnK < 0.0)) continue;
                                    const double vK = (T == Kk) ? vs[T][a] : 0.0;
                                    const double uin = (S == Kk) ? vs[S][c] : 0.0;
                                    const double uout = (S != Kk) ? vs[S][c] : 0.0;
                                    val += bnK * (uout - uin) * vK;
                                }
                            }
                            double* blk;
                            if (T == S) blk = diag + Ks[T] * n * n;
                            else if (T == 0) blk = off_ij + e * n * n;
                            else blk = off_ji + e * n * n;
                            blk[a * n + c] += ds * val;
                        }
        }
    }

    /* --- boundary edges --- */
    for (int64_t bi = 0; bi < M->n_bnd; ++bi) {
        const int64_t K = M->bnd_el[bi];
        affine_t A;
        element_map(M, K, &A);
        const double* pa = M->xy + 2 * M->bnd_v[2 * bi];
        const double* pb = M->xy + 2 * M->bnd_v[2 * bi + 1];
        const double ex = pb[0] - pa[0], ey = pb[1] - pa[1];
        const double len = sqrt(ex * ex + ey * ey);
        const double nx = ey / len, ny = -ex / len;
        const double he = pow(len, P->b0);
        double* DK = diag + K * n * n;
        for (int g = 0; g < nqe; ++g) {
            const double x = pa[0] + te[g] * ex, y = pa[1] + te[g] * ey;
            const double ds = we[g] * len;
            eval_phys(&B, &A, x, y, v, gx, gy);
            const int64_t pidx = bi * nqe + g;
            if (M->bnd_type[bi] == 1) { /* Neumann: l_h gets g^N v; no bilinear terms */
                const double gn = field_at(&P->gN, x, y, pidx);
                for (int a = 0; a < n; ++a) rhs[K * n + a] += ds * gn * v[a];
                continue;
            }
            /* Dirichlet: [v] = v n, {eps grad v} = eps grad v, penalty sigma_D */
            const double eps = field_at(&P->eps, x, y, -1);
            const double beta = field_at(&P->bx, x, y, -1) * nx + field_at(&P->by, x, y, -1) * ny;
            const double pen = P->sigma_D * eps / he;
            const double gd = field_at(&P->gD, x, y, pidx);
            for (int a = 0; a < n; ++a) {
                const double dnv = gx[a] * nx + gy[a] * ny;
                for (int c = 0; c < n; ++c) {
                    const double dnu = gx[c] * nx + gy[c] * ny;
                    double val = 0.0;
                    if (useD) val += -eps * dnu * v[a] + P->kappa * eps * dnv * v[c] + pen * v[c] * v[a];
                    if (useC && beta < 0.0) val += -beta * v[c] * v[a];
                    DK[a * n + c] += ds * val;
                }
                double r = gd * (pen * v[a] + P->kappa * eps * dnv);
                if (beta < 0.0) r += -beta * gd * v[a];
                rhs[K * n + a] += ds * r;
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Block operator y = A x over the assembled blocks.                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_mesh* M;
    int n;
    const double *diag, *off_ij, *off_ji;
} blockop;

static void op_apply(const blockop* O, const double* x, double* y)
{
    const int n = O->n;
    for (int64_t K = 0; K < O->M->T; ++K)
        for (int a = 0; a < n; ++a) {
            double s = 0.0;
            for (int c = 0; c < n; ++c) s += O->diag[K * n * n + a * n + c] * x[K * n + c];
            y[K * n + a] = s;
        }
    for (int64_t e = 0; e < O->M->n_int; ++e) {
        int64_t Ki = O->M->int_el[2 * e], Kj = O->M->int_el[2 * e + 1];
        for (int a = 0; a < n; ++a) {
            double s1 = 0.0, s2 = 0.0;
            for (int c = 0; c < n; ++c) {
                s1 += O->off_ij[e * n * n + a * n + c] * x[Kj * n + c];
                s2 += O->off_ji[e * n * n + a * n + c] * x[Ki * n + c];
            }
            y[Ki * n + a] += s1;
            y[Kj * n + a] += s2;
        }
    }
}

/* block-Jacobi preconditioner: LU with partial pivoting of every diagonal block */
typedef struct { int n; int64_t T; double* lu; int32_t* piv; } bjac;

static int bjac_setup(bjac* P, const orc_mesh* M, int n, const double* diag)
{
    P->n = n; P->T = M->T;
    P->lu = (double*)malloc(sizeof(double) * M->T * n * n);
    P->piv = (int32_t*)malloc(sizeof(int32_t) * M->T * n);
    if (!P->lu || !P->piv) return ORC_ERR_NOMEM;
    memcpy(P->lu, diag, sizeof(double) * M->T * n * n);
    for (int64_t K = 0; K < M->T; ++K) {
        double* L = P->lu + K * n * n;
        int32_t* pv = P->piv + K * n;
        for (int j = 0; j < n; ++j) {
            int p = j;
            for (int i = j + 1; i < n; ++i) if (fabs(L[i * n + j]) > fabs(L[p * n + j])) p = i;
            pv[j] = p;
            if (p != j) for (int c = 0; c < n; ++c) { double t = L[j * n + c]; L[j * n + c] = L[p * n + c]; L[p * n + c] = t; }
            if (L[j * n + j] == 0.0) return ORC_ERR_ARG;
            for (int i = j + 1; i < n; ++i) {
                L[i * n + j] /= L[j * n + j];
                for (int c = j + 1; c < n; ++c) L[i * n + c] -= L[i * n + j] * L[j * n + c];
            }
        }
    }
    return ORC_OK;
}

static void bjac_apply(const bjac* P, const double* v, double* z)
{
    const int n = P->n;
    for (int64_t K = 0; K < P->T; ++K) {
        const double* L = P->lu + K * n * n;
        const int32_t* pv = P->piv + K * n;
        double t[ORC_MAXN];
        for (int i = 0; i < n; ++i) t[i] = v[K * n + i];
        for (int j = 0; j < n; ++j) if (pv[j] != j) { double s = t[j]; t[j] = t[pv[j]]; t[pv[j]] = s; }
        for (int i = 0; i < n; ++i) for (int c = 0; c < i; ++c) t[i] -= L[i * n + c] * t[c];
        for (int i = n - 1; i >= 0; --i) {
            for (int c = i + 1; c < n; ++c) t[i] -= L[i * n + c] * t[c];
            t[i] /= L[i * n + i];
        }
        for (int i = 0; i < n; ++i) z[K * n + i] = t[i];
    }
}

static void bjac_free(bjac* P) { free(P->lu); free(P->piv); }

static double dot(int64_t N, const double* a, const double* b)
{
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) s += a[i] * b[i];
    return s;
}

/* y = A x for the caller (tests) */
int orc_matvec(const orc_mesh* M, int k, const double* diag, const double* off_ij, const double* off_ji,
               const double* x, double* y)
{
    blockop O = { M, (k + 1) * (k + 2) / 2, diag, off_ij, off_ji };
    op_apply(&O, x, y);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Restarted GMRES(m), right block-Jacobi preconditioner M = blockdiag(A):   */
/* Arnoldi on A M^{-1} with modified Gram-Schmidt, Givens rotations, x =     */
/* x0 + M^{-1} V y.  Stops when the true relative residual                   */
/* ||F - A x||_2 / ||F||_2 <= tol (checked at every restart and whenever the */
/* Arnoldi estimate reaches tol) or after max_iters Arnoldi steps.           */
/* x holds the initial guess on entry.  Returns 0 if converged, 1 if not.    */
/* ------------------------------------------------------------------------ */
int orc_gmres(const orc_mesh* M, int k, const double* diag, const double* off_ij, const double* off_ji,
              const double* F, double* x, int m, double tol, int max_iters, int* iters_out, double* relres_out)
{
    const int n = (k + 1) * (k + 2) / 2;
    const int64_t N = M->T * n;
    blockop O = { M, n, diag, off_ij, off_ji };
    bjac P;
    int st = bjac_setup(&P, M, n, diag);
    if (st != ORC_OK) { bjac_free(&P); return st; }
    double* V = (double*)malloc(sizeof(double) * (m + 1) * N);
    double* z = (double*)malloc(sizeof(double) * N);
    double* w = (double*)malloc(sizeof(double) * N);
    double* r = (double*)malloc(sizeof(double) * N);
    double* H = (double*)calloc((size_t)(m + 1) * m, sizeof(double));
    double* cs = (double*)malloc(sizeof(double) * m);
    double* sn = (double*)malloc(sizeof(double) * m);
    double* gvec = (double*)malloc(sizeof(double) * (m + 1));
    double* yv = (double*)malloc(sizeof(double) * m);
    const double nF = sqrt(dot(N, F, F));
    int its = 0, conv = 0;
    double rel = 0.0;
    if (nF == 0.0) {
        for (int64_t i = 0; i < N; ++i) x[i] = 0.0;
        conv = 1;
    }
    while (!conv) {
        op_apply(&O, x, r);
        for (int64_t i = 0; i < N; ++i) r[i] = F[i] - r[i];
        const double beta = sqrt(dot(N, r, r));
        rel = beta / nF;
        if (rel <= tol) { conv = 1; break; }
        if (its >= max_iters) break;
        for (int64_t i = 0; i < N; ++i) V[i] = r[i] / beta;
        for (int i = 0; i <= m; ++i) gvec[i] = 0.0;
        gvec[0] = beta;
        int j = 0;
        for (; j < m && its < max_iters; ++j) {
            ++its;
            bjac_apply(&P, V + j * N, z);
            op_apply(&O, z, w);
            for (int i = 0; i <= j; ++i) {   /* modified Gram-Schmidt */
                double h = dot(N, w, V + i * N);
                H[i * m + j] = h;
                for (int64_t t = 0; t < N; ++t) w[t] -= h * V[i * N + t];
            }
            double hn = sqrt(dot(N, w, w));
            H[(j + 1) * m + j] = hn;
            if (hn != 0.0) for (int64_t t = 0; t < N; ++t) V[(j + 1) * N + t] = w[t] / hn;
            for (int i = 0; i < j; ++i) {    /* apply previous rotations to column j */
                double a = H[i * m + j], b = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * b;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            double a = H[j * m + j], b = H[(j + 1) * m + j];
            double d = sqrt(a * a + b * b);
            cs[j] = d == 0.0 ? 1.0 : a / d;
            sn[j] = d == 0.0 ? 0.0 : b / d;
            H[j * m + j] = d;
            H[(j + 1) * m + j] = 0.0;
            gvec[j + 1] = -sn[j] * gvec[j];
            gvec[j] = cs[j] * gvec[j];
            if (fabs(gvec[j + 1]) / nF <= tol || hn == 0.0) { ++j; break; }
        }
        /* least squares: upper-triangular H(0:j,0:j) y = g(0:j) */
        for (int i = j - 1; i >= 0; --i) {
            double s = gvec[i];
            for (int c = i + 1; c < j; ++c) s -= H[i * m + c] * yv[c];
            yv[i] = s / H[i * m + i];
        }
        for (int64_t t = 0; t < N; ++t) w[t] = 0.0;
        for (int i = 0; i < j; ++i) for (int64_t t = 0; t < N; ++t) w[t] += yv[i] * V[i * N + t];
        bjac_apply(&P, w, z);
        for (int64_t t = 0; t < N; ++t) x[t] += z[t];
    }
    if (!conv && nF != 0.0) {
        op_apply(&O, x, r);
        for (int64_t i = 0; i < N; ++i) r[i] = F[i] - r[i];
        rel = sqrt(dot(N, r, r)) / nF;
        conv = rel <= tol;
    }
    free(V); free(z); free(w); free(r); free(H); free(cs); free(sn); free(gvec); free(yv);
    bjac_free(&P);
    *iters_out = its;
    *relres_out = rel;
    return conv ? 0 : 1;
}

/* ------------------------------------------------------------------------ */
/* Post-processing (section 2.4): u_h at points and the L2 error.            */
/* ------------------------------------------------------------------------ */

/* u_h(x_p) for points p lying in elements elem[p] */
int orc_eval_solution(const orc_mesh* M, int k, int basis, const double* coef, int64_t np, const int32_t* elem,
                      const double* xy, double* out)
{
    if (k < 0 || k > ORC_MAXK || !basis_ok(basis)) return ORC_ERR_ARG;
    basis_t B;
    build_basis(k, basis, &B);
    double v[ORC_MAXN], gx[ORC_MAXN], gy[ORC_MAXN];
    for (int64_t p = 0; p < np; ++p) {
        affine_t A;
        element_map(M, elem[p], &A);
        eval_phys(&B, &A, xy[2 * p], xy[2 * p + 1], v, gx, gy);
        double s = 0.0;
        for (int m = 0; m < B.n; ++m) s += coef[(int64_t)elem[p] * B.n + m] * v[m];
        out[p] = s;
    }
    return ORC_OK;
}

/* ||u_h - u||_{L2} with the q x q Stroud rule; exact = u at orc_volume_points(M,k,q) */
double orc_l2_error(const orc_mesh* M, int k, int basis, const double* coef, int q, const double* exact)
{
    if (k < 0 || k > ORC_MAXK || !basis_ok(basis)) return NAN;
    basis_t B;
    build_basis(k, basis, &B);
    double xi[ORC_MAXQ * ORC_MAXQ], eta[ORC_MAXQ * ORC_MAXQ], w[ORC_MAXQ * ORC_MAXQ];
    int nq = orc_volume_rule(q, xi, eta, w);
    double v[ORC_MAXN];
    double s = 0.0;
    for (int64_t K = 0; K < M->T; ++K) {
        affine_t A;
        element_map(M, K, &A);
        for (int g = 0; g < nq; ++g) {
            eval_basis(&B, xi[g], eta[g], v, NULL, NULL);
            double uh = 0.0;
            for (int m = 0; m < B.n; ++m) uh += coef[K * B.n + m] * v[m];
            double d = uh - exact[K * nq + g];
            s += w[g] * A.det * d * d;
        }
    }
    return sqrt(s);
}

/* ------------------------------------------------------------------------ */
/* Non-linear reaction (section 3): H_i(v) = int r(u_h) phi_i and its        */
/* Jacobian HJ_ij = int r'(u_h) phi_j phi_i, with r(u) = sum_p c_p u^p        */
/* (p = 1..np) and the volume rule of the assembly (q = k + 2).  HJ is       */
/* element-local: hj[K][i][j] is the diagonal block of element K (row = test */
/* i, column = trial j).  Either output may be NULL.                          */
/* ------------------------------------------------------------------------ */
int orc_reaction_terms(const orc_mesh* M, int k, int basis, int np, const double* c, const double* coef, double* h,
                       double* hj)
{
    if (k < 0 || k > ORC_MAXK || np < 0 || np > 8 || !basis_ok(basis)) return ORC_ERR_ARG;
    basis_t B;
    build_basis(k, basis, &B);
    const int n = B.n, q = k + 2;
    double xi[ORC_MAXQ * ORC_MAXQ], eta[ORC_MAXQ * ORC_MAXQ], w[ORC_MAXQ * ORC_MAXQ];
    const int nq = orc_volume_rule(q, xi, eta, w);
    double v[ORC_MAXN];
    for (int64_t K = 0; K < M->T; ++K) {
        affine_t A;
        element_map(M, K, &A);
        if (h)
            for (int i = 0; i < n; ++i) h[K * n + i] = 0.0;
        if (hj)
            for (int i = 0; i < n * n; ++i) hj[K * n * n + i] = 0.0;
        for (int g = 0; g < nq; ++g) {
            eval_basis(&B, xi[g], eta[g], v, NULL, NULL);
            double u = 0.0;
            for (int m = 0; m < n; ++m) u += coef[K * n + m] * v[m];
            /* r(u) and r'(u) term by term */
            double r = 0.0, dr = 0.0, up = 1.0; /* up = u^(p-1) */
            for (int p = 1; p <= np; ++p) {
                dr += p * c[p - 1] * up;
                up *= u;
                r += c[p - 1] * up;
            }
            const double dx = w[g] * A.det;
            if (h)
                for (int i = 0; i < n; ++i) h[K * n + i] += dx * r * v[i];
            if (hj)
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) hj[(K * n + i) * n + j] += dx * dr * v[j] * v[i];
        }
    }
    return ORC_OK;
}
