/*
 * mfcg_oracle.c -- plain, slow, obviously correct FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only tests/, __graft_entry__.smoke() and the cpu_baseline
 * leg of bench.py use it.  It shares no code, header, table or constant with
 * the HIP path.
 *
 * What it computes (Kronbichler, Sashko, Munch, "Enhancing data locality of
 * the conjugate gradient method for high-order matrix-free finite-element
 * implementations"):
 *   - the scalar Poisson problem -div(a grad u) = f on a mapped hexahedral
 *     mesh (Sec. 2, Eq. 1 in its scalar form, Eq. 2 ansatz with tensor-product
 *     Lagrange polynomials of degree k),
 *   - the global matrix A of Eq. 3, assembled as the sum of element matrices
 *     of Eq. 4/5 integrated by tensor Gauss quadrature, into CSR,
 *     with Dirichlet nodes kept as identity rows and columns (Sec. 5.3,
 *     the fourth class of unknowns: constrained entries kept in the system),
 *   - the point-Jacobi diagonal d = diag(A) (Sec. 3, preconditioner),
 *   - textbook preconditioned CG, Algorithm 1, terminating on the
 *     unpreconditioned residual norm (Sec. 3.1).
 * Everything is a direct transcription of these definitions: element
 * matrices are built by brute force over all (i, j, q) triples, no sum
 * factorization, no fusion.
 *
 *   - optionally, the map replaced by its per-cell quadratic interpolant
 *     (quadratic geometry, Sec. 2.2; map kind bit OR_MAP_QUADRATIC).
 * Readings where the paper is silent:
 *   - nodal points of the 1D basis: Gauss-Lobatto-Legendre points,
 *   - quadrature: Gauss-Legendre with nq1 points per direction (nq1 = k+1
 *     by default), or Gauss-Lobatto-Legendre with -nq1 points (nq1 < 0),
 *   - per-cell constant coefficient a_e multiplies the cell integral,
 *   - Dirichlet rows/columns replaced by the identity, b_C as given,
 *   - stopping rule: ||r_j||_2 < tol * ||b||_2.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC -o liboracle.so mfcg_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* 1D polynomials                                                       */
/* ------------------------------------------------------------------ */

/* Legendre polynomial P_n(t) on [-1,1] and its derivative, three-term
 * recurrence (textbook). */
static void legendre(int n, double t, double *p, double *dp)
{
    double p0 = 1.0, p1 = t;
    if (n == 0) { *p = 1.0; *dp = 0.0; return; }
    for (int m = 2; m <= n; ++m) {
        double p2 = ((2.0 * m - 1.0) * t * p1 - (m - 1.0) * p0) / m;
        p0 = p1; p1 = p2;
    }
    *p = p1;
    /* P_n'(t) = n (t P_n - P_{n-1}) / (t^2 - 1) for |t| < 1 */
    *dp = n * (t * p1 - p0) / (t * t - 1.0);
}

/* Gauss-Legendre rule with n points mapped to [0,1]; Newton on P_n. */
int oracle_gauss(int n, double *x, double *w)
{
    if (n < 1 || n > 64) return -1;
    for (int i = 0; i < n; ++i) {
        double t = cos(OR_PI * (i + 0.75) / (n + 0.5));
        double p = 0, dp = 1;
        for (int it = 0; it < 100; ++it) {
            legendre(n, t, &p, &dp);
            double dt = p / dp;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        legendre(n, t, &p, &dp);
        /* ascending order on [0,1] */
        x[n - 1 - i] = 0.5 * (1.0 + t);
        w[n - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp); /* 2/((1-t^2)P'^2) * 1/2 */
    }
    return 0;
}

/* Gauss-Lobatto-Legendre points (k+1 of them) on [0,1]: the end points and
 * the roots of P_k'.  Newton on P_k' using P_k'' from the Legendre ODE:
 * (1-t^2) P'' = 2 t P' - k(k+1) P. */
int oracle_gll(int k, double *x)
{
    if (k < 1 || k > 32) return -1;
    x[0] = 0.0;
    x[k] = 1.0;
    for (int i = 1; i < k; ++i) {
        double t = -cos(OR_PI * i / k); /* Chebyshev-Lobatto initial guess */
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(k, t, &p, &dp);
            double ddp = (2.0 * t * dp - k * (k + 1.0) * p) / (1.0 - t * t);
            double dt = dp / ddp;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        x[i] = 0.5 * (1.0 + t);
    }
    return 0;
}

/* Gauss-Lobatto-Legendre quadrature weights on [0,1] for the k+1 points x
 * of oracle_gll: w_i = 2 / (k (k+1) P_k(t_i)^2) on [-1,1], t = 2x - 1,
 * halved for the unit interval (textbook). */
int oracle_gll_weights(int k, const double *x, double *w)
{
    if (k < 1 || k > 32) return -1;
    for (int i = 0; i <= k; ++i) {
        double p, dp;
        double t = 2.0 * x[i] - 1.0;
        if (i == 0 || i == k) {
            p = (i == 0 && (k & 1)) ? -1.0 : 1.0; /* P_k(+-1) = (+-1)^k */
        } else {
            legendre(k, t, &p, &dp);
        }
        w[i] = 1.0 / (k * (k + 1.0) * p * p);
    }
    return 0;
}

/* Lagrange basis polynomial i over nodes[0..np-1], value at x. */
double oracle_lagrange(int np, const double *nodes, int i, double x)
{
    double v = 1.0;
    for (int j = 0; j < np; ++j)
        if (j != i) v *= (x - nodes[j]) / (nodes[i] - nodes[j]);
    return v;
}

/* Derivative of the Lagrange basis polynomial i at x (product rule). */
double oracle_lagrange_deriv(int np, const double *nodes, int i, double x)
{
    double s = 0.0;
    for (int m = 0; m < np; ++m) {
        if (m == i) continue;
        double term = 1.0 / (nodes[i] - nodes[m]);
        for (int j = 0; j < np; ++j)
            if (j != i && j != m) term *= (x - nodes[j]) / (nodes[i] - nodes[j]);
        s += term;
    }
    return s;
}

/* ------------------------------------------------------------------ */
/* Geometry                                                             */
/* ------------------------------------------------------------------ */

/* Map kinds: 0 identity (Cartesian), 1 cyclic sine shear
 *   x_i + A sin(2 pi x_{i+1}) sin(2 pi x_{i+2}),
 * 2 sine product  x_i + A prod_j sin(2 pi x_j)  (keeps the unit cube). */
static void map_point(int kind, double A, const double X[3], double x[3],
                      double DF[3][3])
{
    double s[3], c[3];
    for (int d = 0; d < 3; ++d) {
        s[d] = sin(2.0 * OR_PI * X[d]);
        c[d] = cos(2.0 * OR_PI * X[d]);
    }
    for (int i = 0; i < 3; ++i) {
        x[i] = X[i];
        for (int j = 0; j < 3; ++j) DF[i][j] = (i == j) ? 1.0 : 0.0;
    }
    if (kind == 1) {
        for (int i = 0; i < 3; ++i) {
            int a = (i + 1) % 3, b = (i + 2) % 3;
            x[i] += A * s[a] * s[b];
            DF[i][a] += A * 2.0 * OR_PI * c[a] * s[b];
            DF[i][b] += A * 2.0 * OR_PI * s[a] * c[b];
        }
    } else if (kind == 2) {
        double prod = s[0] * s[1] * s[2];
        for (int i = 0; i < 3; ++i) {
            x[i] += A * prod;
            for (int j = 0; j < 3; ++j) {
                double dj = 2.0 * OR_PI * c[j];
                for (int l = 0; l < 3; ++l)
                    if (l != j) dj *= s[l];
                DF[i][j] += A * dj;
            }
        }
    }
}

/* Map kinds with this bit set: in every cell the map is replaced by its
 * tensor-product quadratic interpolant through the 27 points
 * (c + (a, b, d) / 2) / n, a, b, d in {0, 1, 2} -- the quadratic geometry
 * of Sec. 2.2 whose Jacobians are evaluated at the quadrature points
 * instead of being stored. */
#define OR_MAP_QUADRATIC 16

/* Point of cell (cx,cy,cz) at reference coordinate xi in [0,1]^3: the
 * Cartesian position X, the mapped position x and the Jacobian
 * J = dx/dxi = DF(X) * diag(1/n) (of the interpolant for quadratic
 * geometry: x = sum_node x_node N_node(xi), J = sum_node x_node grad N_node). */
static void cell_point(const int n[3], int kind, double A, const int c[3],
                       const double xi[3], double x[3], double J[3][3])
{
    double X[3], DF[3][3];
    if (kind & OR_MAP_QUADRATIC) {
        static const double q2nodes[3] = {0.0, 0.5, 1.0};
        double N[3][3], dN[3][3]; /* [direction][node] */
        for (int d = 0; d < 3; ++d)
            for (int a = 0; a < 3; ++a) {
                N[d][a] = oracle_lagrange(3, q2nodes, a, xi[d]);
                dN[d][a] = oracle_lagrange_deriv(3, q2nodes, a, xi[d]);
            }
        for (int i = 0; i < 3; ++i) {
            x[i] = 0.0;
            for (int j = 0; j < 3; ++j) J[i][j] = 0.0;
        }
        for (int cz = 0; cz < 3; ++cz)
            for (int cy = 0; cy < 3; ++cy)
                for (int cx = 0; cx < 3; ++cx) {
                    double xn[3];
                    const int a[3] = {cx, cy, cz};
                    for (int d = 0; d < 3; ++d) X[d] = (c[d] + q2nodes[a[d]]) / n[d];
                    map_point(kind & ~OR_MAP_QUADRATIC, A, X, xn, DF);
                    const double v = N[0][cx] * N[1][cy] * N[2][cz];
                    const double g[3] = {dN[0][cx] * N[1][cy] * N[2][cz], N[0][cx] * dN[1][cy] * N[2][cz],
                                         N[0][cx] * N[1][cy] * dN[2][cz]};
                    for (int i = 0; i < 3; ++i) {
                        x[i] += xn[i] * v;
                        for (int j = 0; j < 3; ++j) J[i][j] += xn[i] * g[j];
                    }
                }
        return;
    }
    for (int d = 0; d < 3; ++d) X[d] = (c[d] + xi[d]) / n[d];
    map_point(kind, A, X, x, DF);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) J[i][j] = DF[i][j] / n[j];
}

static double det3(double J[3][3])
{
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
         - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
         + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/* inverse by the adjugate */
static void inv3(double J[3][3], double det, double Ji[3][3])
{
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
}

/* Mapped position of a lattice point (used by tests to evaluate exact
 * solutions at nodes). */
void oracle_map(int kind, double A, const double *X, double *x)
{
    double DF[3][3];
    map_point(kind, A, X, x, DF);
}

/* Jacobian determinant of the global map at X (tests use it to check
 * that the maps stay invertible). */
double oracle_map_det(int kind, double A, const double *X)
{
    double x[3], DF[3][3];
    map_point(kind, A, X, x, DF);
    return det3(DF);
}

/* ------------------------------------------------------------------ */
/* Mesh description shared by the entry points below                    */
/* ------------------------------------------------------------------ */

typedef struct {
    int n[3];       /* cells per direction */
    int k;          /* polynomial degree */
    int nq1;        /* Gauss points per direction */
    int map_kind;
    double amp;
    int bc;         /* 0: Dirichlet on the whole boundary, 1: none */
    const double *coeff; /* per cell, index cx + nx*(cy + ny*cz); NULL -> 1 */
    int op;         /* 0: Laplacian (Eq. 5), 1: mass matrix */
} om_mesh;

static int64_t lat(const om_mesh *m, int d) { return (int64_t)m->n[d] * m->k + 1; }

static int64_t n_nodes(const om_mesh *m)
{
    return lat(m, 0) * lat(m, 1) * lat(m, 2);
}

static int is_constrained(const om_mesh *m, const int64_t g[3])
{
    if (m->bc != 0) return 0;
    for (int d = 0; d < 3; ++d)
        if (g[d] == 0 || g[d] == lat(m, d) - 1) return 1;
    return 0;
}

static void node_coords(const om_mesh *m, int64_t idx, int64_t g[3])
{
    g[0] = idx % lat(m, 0);
    idx /= lat(m, 0);
    g[1] = idx % lat(m, 1);
    g[2] = idx / lat(m, 1);
}

static int64_t node_index(const om_mesh *m, const int64_t g[3])
{
    return g[0] + lat(m, 0) * (g[1] + lat(m, 1) * g[2]);
}

/* 1D tables: nodes, Gauss rule, basis values and derivatives at the Gauss
 * points.  phi[q*np + i] = phi_i(x_q). */
typedef struct {
    int np, nq;
    double nodes[33];
    double xq[64], wq[64];
    double *phi, *dphi;
} om_tab;

/* nq1 > 0: Gauss-Legendre with nq1 points per direction; nq1 < 0:
 * Gauss-Lobatto-Legendre with -nq1 points (for -nq1 = k+1 the points are
 * the nodes: collocation). */
static int tab_init(om_tab *t, int k, int nq1)
{
    t->np = k + 1;
    t->nq = nq1 > 0 ? nq1 : -nq1;
    if (oracle_gll(k, t->nodes) != 0) return -1;
    if (nq1 > 0) {
        if (oracle_gauss(nq1, t->xq, t->wq) != 0) return -1;
    } else {
        if (oracle_gll(t->nq - 1, t->xq) != 0) return -1;
        if (oracle_gll_weights(t->nq - 1, t->xq, t->wq) != 0) return -1;
    }
    t->phi = malloc(sizeof(double) * t->np * t->nq);
    t->dphi = malloc(sizeof(double) * t->np * t->nq);
    if (!t->phi || !t->dphi) return -2;
    for (int q = 0; q < t->nq; ++q)
        for (int i = 0; i < t->np; ++i) {
            t->phi[q * t->np + i] = oracle_lagrange(t->np, t->nodes, i, t->xq[q]);
            t->dphi[q * t->np + i] = oracle_lagrange_deriv(t->np, t->nodes, i, t->xq[q]);
        }
    return 0;
}

static void tab_free(om_tab *t)
{
    free(t->phi);
    free(t->dphi);
}

/* Element matrix of Eq. 5 by brute force:
 *   (A_e)_ij = a_e sum_q w_q det J_q (J_q^{-T} grad phi_i) . (J_q^{-T} grad phi_j)
 * or, for the mass operator, a_e sum_q w_q det J_q phi_i phi_j.
 * Local index i = ix + np*(iy + np*iz).  Ae has nb*nb entries. */
static int element_matrix(const om_mesh *m, const om_tab *t, const int c[3],
                          double *Ae, double *grad /* 3*nb scratch */)
{
    int np = t->np, nq = t->nq, nb = np * np * np;
    double ae = 1.0;
    if (m->coeff)
        ae = m->coeff[c[0] + (int64_t)m->n[0] * (c[1] + (int64_t)m->n[1] * c[2])];
    memset(Ae, 0, sizeof(double) * nb * nb);
    for (int qz = 0; qz < nq; ++qz)
        for (int qy = 0; qy < nq; ++qy)
            for (int qx = 0; qx < nq; ++qx) {
                double xi[3] = {t->xq[qx], t->xq[qy], t->xq[qz]};
                double x[3], J[3][3], Ji[3][3];
                cell_point(m->n, m->map_kind, m->amp, c, xi, x, J);
                double det = det3(J);
                if (!(det > 0.0)) return -5;
                inv3(J, det, Ji);
                double wdet = ae * t->wq[qx] * t->wq[qy] * t->wq[qz] * det;
                if (m->op == 1) {
                    for (int i = 0; i < nb; ++i) {
                        const int ix = i % np, iy = (i / np) % np, iz = i / (np * np);
                        grad[i] = t->phi[qx * np + ix] * t->phi[qy * np + iy] * t->phi[qz * np + iz];
                    }
                    for (int i = 0; i < nb; ++i)
                        for (int j = 0; j < nb; ++j) Ae[i * nb + j] += wdet * grad[i] * grad[j];
                    continue;
                }
                for (int iz = 0; iz < np; ++iz)
                    for (int iy = 0; iy < np; ++iy)
                        for (int ix = 0; ix < np; ++ix) {
                            int i = ix + np * (iy + np * iz);
                            /* reference gradient of phi_i at the point */
                            double gr[3] = {
                                t->dphi[qx * np + ix] * t->phi[qy * np + iy] * t->phi[qz * np + iz],
                                t->phi[qx * np + ix] * t->dphi[qy * np + iy] * t->phi[qz * np + iz],
                                t->phi[qx * np + ix] * t->phi[qy * np + iy] * t->dphi[qz * np + iz]};
                            /* real gradient J^{-T} gr */
                            for (int a = 0; a < 3; ++a)
                                grad[3 * i + a] = Ji[0][a] * gr[0] + Ji[1][a] * gr[1] + Ji[2][a] * gr[2];
                        }
                for (int i = 0; i < nb; ++i)
                    for (int j = 0; j < nb; ++j)
                        Ae[i * nb + j] += wdet * (grad[3 * i] * grad[3 * j] + grad[3 * i + 1] * grad[3 * j + 1]
                                                  + grad[3 * i + 2] * grad[3 * j + 2]);
            }
    return 0;
}

static void local_to_global(const om_mesh *m, const int c[3], int np, int i, int64_t g[3])
{
    int ix = i % np, iy = (i / np) % np, iz = i / (np * np);
    g[0] = (int64_t)c[0] * m->k + ix;
    g[1] = (int64_t)c[1] * m->k + iy;
    g[2] = (int64_t)c[2] * m->k + iz;
}

static int mesh_check(const om_mesh *m)
{
    const int nq = m->nq1 > 0 ? m->nq1 : -m->nq1;
    if (m->k < 1 || m->k > 16 || nq < 1 || nq > 32 || (m->nq1 < 0 && nq < 2)) return -1;
    if (m->op != 0 && m->op != 1) return -1;
    for (int d = 0; d < 3; ++d)
        if (m->n[d] < 1) return -1;
    return 0;
}

#define OM_MESH_ARGS const int *ncells, int k, int nq1, int map_kind, double amp, int bc, const double *coeff, int op
#define OM_MESH_INIT {{ncells[0], ncells[1], ncells[2]}, k, nq1, map_kind, amp, bc, coeff, op}

int64_t oracle_n_nodes(const int *ncells, int k)
{
    return ((int64_t)ncells[0] * k + 1) * ((int64_t)ncells[1] * k + 1) * ((int64_t)ncells[2] * k + 1);
}

/* Dense element matrix of one cell (for tests on tiny meshes). */
int oracle_element_matrix(OM_MESH_ARGS, const int *cell, double *Ae)
{
    om_mesh m = OM_MESH_INIT;
    if (mesh_check(&m)) return -1;
    om_tab t;
    if (tab_init(&t, k, nq1)) return -2;
    int nb = (k + 1) * (k + 1) * (k + 1);
    double *grad = malloc(sizeof(double) * 3 * nb);
    int rc = element_matrix(&m, &t, cell, Ae, grad);
    free(grad);
    tab_free(&t);
    return rc;
}

/* ------------------------------------------------------------------ */
/* CSR assembly (Eq. 4: A = sum_e P_e^T A_e P_e)                        */
/* ------------------------------------------------------------------ */

/* 1D column range of node coordinate g: all lattice points of the cells
 * that contain g. */
static void col_range(const om_mesh *m, int d, int64_t g, int64_t *lo, int64_t *hi)
{
    int k = m->k;
    if (g % k == 0) {
        *lo = g - k < 0 ? 0 : g - k;
        *hi = g + k > lat(m, d) - 1 ? lat(m, d) - 1 : g + k;
    } else {
        *lo = (g / k) * k;
        *hi = *lo + k;
    }
}

/* Row lengths: free rows couple to the free nodes of the adjacent cells,
 * constrained rows hold only their diagonal. */
int oracle_csr_rowptr(OM_MESH_ARGS, int64_t *rowptr)
{
    om_mesh m = OM_MESH_INIT;
    if (mesh_check(&m)) return -1;
    int64_t n = n_nodes(&m);
    rowptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t g[3];
        node_coords(&m, i, g);
        int64_t cnt = 0;
        if (is_constrained(&m, g)) {
            cnt = 1;
        } else {
            int64_t lo[3], hi[3];
            for (int d = 0; d < 3; ++d) col_range(&m, d, g[d], &lo[d], &hi[d]);
            for (int64_t z = lo[2]; z <= hi[2]; ++z)
                for (int64_t y = lo[1]; y <= hi[1]; ++y)
                    for (int64_t x = lo[0]; x <= hi[0]; ++x) {
                        int64_t h[3] = {x, y, z};
                        if (!is_constrained(&m, h)) ++cnt;
                    }
        }
        rowptr[i + 1] = rowptr[i] + cnt;
    }
    return 0;
}

static int64_t find_col(const int64_t *rowptr, const int32_t *col, int64_t row, int64_t j)
{
    int64_t a = rowptr[row], b = rowptr[row + 1] - 1;
    while (a <= b) {
        int64_t mid = (a + b) / 2;
        if (col[mid] == j) return mid;
        if (col[mid] < j) a = mid + 1; else b = mid - 1;
    }
    return -1;
}

/* Column indices and values.  Cells are visited in 8 colour classes (parity
 * of the cell index per direction) so that cells handled concurrently never
 * share a node; the summation order per entry is then fixed. */
int oracle_csr_fill(OM_MESH_ARGS, const int64_t *rowptr, int32_t *col, double *val)
{
    om_mesh m = OM_MESH_INIT;
    if (mesh_check(&m)) return -1;
    int64_t n = n_nodes(&m);
    if (n > 2147483647LL) return -1;
    /* columns, ascending */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t g[3];
        node_coords(&m, i, g);
        int64_t p = rowptr[i];
        if (is_constrained(&m, g)) {
            col[p] = (int32_t)i;
            val[p] = 1.0;
            continue;
        }
        int64_t lo[3], hi[3];
        for (int d = 0; d < 3; ++d) col_range(&m, d, g[d], &lo[d], &hi[d]);
        for (int64_t z = lo[2]; z <= hi[2]; ++z)
            for (int64_t y = lo[1]; y <= hi[1]; ++y)
                for (int64_t x = lo[0]; x <= hi[0]; ++x) {
                    int64_t h[3] = {x, y, z};
                    if (is_constrained(&m, h)) continue;
                    col[p] = (int32_t)node_index(&m, h);
                    val[p] = 0.0;
                    ++p;
                }
    }
    om_tab t;
    if (tab_init(&t, k, nq1)) return -2;
    int np = k + 1, nb = np * np * np;
    int rc = 0;
    for (int colour = 0; colour < 8; ++colour) {
        int64_t ncol[3];
        for (int d = 0; d < 3; ++d) ncol[d] = (m.n[d] - ((colour >> d) & 1) + 1) / 2;
        int64_t ncells_col = ncol[0] * ncol[1] * ncol[2];
#pragma omp parallel
        {
            double *Ae = malloc(sizeof(double) * nb * nb);
            double *grad = malloc(sizeof(double) * 3 * nb);
            int64_t *gidx = malloc(sizeof(int64_t) * nb);
            int *cons = malloc(sizeof(int) * nb);
#pragma omp for schedule(dynamic, 4)
            for (int64_t e = 0; e < ncells_col; ++e) {
                int c[3];
                int64_t r = e;
                for (int d = 0; d < 3; ++d) {
                    c[d] = (int)(2 * (r % ncol[d]) + ((colour >> d) & 1));
                    r /= ncol[d];
                }
                if (element_matrix(&m, &t, c, Ae, grad)) {
#pragma omp atomic write
                    rc = -5;
                    continue;
                }
                for (int i = 0; i < nb; ++i) {
                    int64_t g[3];
                    local_to_global(&m, c, np, i, g);
                    gidx[i] = node_index(&m, g);
                    cons[i] = is_constrained(&m, g);
                }
                for (int i = 0; i < nb; ++i) {
                    if (cons[i]) continue;
                    for (int j = 0; j < nb; ++j) {
                        if (cons[j]) continue;
                        int64_t p = find_col(rowptr, col, gidx[i], gidx[j]);
                        val[p] += Ae[i * nb + j];
                    }
                }
            }
            free(Ae);
            free(grad);
            free(gidx);
            free(cons);
        }
    }
    tab_free(&t);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Right-hand side and L2 error                                         */
/* ------------------------------------------------------------------ */

/* Forcing terms: kind 0: 3 pi^2 prod sin(pi x_j) (manufactured solution
 * u = prod sin(pi x_j) on the unit cube); kind 1: sum of Gaussian bumps,
 * params = [nb, (A, cx, cy, cz, s) * nb]. */
static double forcing(int kind, const double *params, const double x[3])
{
    if (kind == 0)
        return 3.0 * OR_PI * OR_PI * sin(OR_PI * x[0]) * sin(OR_PI * x[1]) * sin(OR_PI * x[2]);
    double f = 0.0;
    int nbump = (int)params[0];
    for (int b = 0; b < nbump; ++b) {
        const double *p = params + 1 + 5 * b;
        double r2 = (x[0] - p[1]) * (x[0] - p[1]) + (x[1] - p[2]) * (x[1] - p[2]) + (x[2] - p[3]) * (x[2] - p[3]);
        f += p[0] * exp(-r2 / (2.0 * p[4] * p[4]));
    }
    return f;
}

/* b_i = sum_e sum_q f(x_q) phi_i(xi_q) w_q det J_q for free i, 0 on
 * constrained nodes.  Cells in 8 colour classes as in the assembly. */
int oracle_rhs(OM_MESH_ARGS, int fkind, const double *fparams, double *b)
{
    om_mesh m = OM_MESH_INIT;
    if (mesh_check(&m)) return -1;
    int64_t n = n_nodes(&m);
    memset(b, 0, sizeof(double) * n);
    om_tab t;
    if (tab_init(&t, k, nq1)) return -2;
    int np = k + 1, nb = np * np * np, nq = t.nq;
    for (int colour = 0; colour < 8; ++colour) {
        int64_t ncol[3];
        for (int d = 0; d < 3; ++d) ncol[d] = (m.n[d] - ((colour >> d) & 1) + 1) / 2;
        int64_t ncells_col = ncol[0] * ncol[1] * ncol[2];
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t e = 0; e < ncells_col; ++e) {
            int c[3];
            int64_t r = e;
            for (int d = 0; d < 3; ++d) {
                c[d] = (int)(2 * (r % ncol[d]) + ((colour >> d) & 1));
                r /= ncol[d];
            }
            for (int qz = 0; qz < nq; ++qz)
                for (int qy = 0; qy < nq; ++qy)
                    for (int qx = 0; qx < nq; ++qx) {
                        double xi[3] = {t.xq[qx], t.xq[qy], t.xq[qz]};
                        double x[3], J[3][3];
                        cell_point(m.n, m.map_kind, m.amp, c, xi, x, J);
                        double fw = forcing(fkind, fparams, x) * t.wq[qx] * t.wq[qy] * t.wq[qz] * det3(J);
                        for (int i = 0; i < nb; ++i) {
                            int ix = i % np, iy = (i / np) % np, iz = i / (np * np);
                            int64_t g[3];
                            local_to_global(&m, c, np, i, g);
                            if (is_constrained(&m, g)) continue;
                            b[node_index(&m, g)] += fw * t.phi[qx * np + ix] * t.phi[qy * np + iy] * t.phi[qz * np + iz];
                        }
                    }
        }
    }
    tab_free(&t);
    return 0;
}

/* || u - u_h ||_{L2} with u = prod sin(pi x_j), Gauss rule with nqe points
 * per direction. */
double oracle_l2_error(OM_MESH_ARGS, int nqe, const double *uh)
{
    om_mesh m = OM_MESH_INIT;
    if (mesh_check(&m)) return -1.0;
    om_tab t;
    if (tab_init(&t, k, nqe)) return -1.0;
    int np = k + 1, nb = np * np * np;
    int64_t ncell_tot = (int64_t)m.n[0] * m.n[1] * m.n[2];
    double err2 = 0.0;
#pragma omp parallel for reduction(+ : err2) schedule(static)
    for (int64_t e = 0; e < ncell_tot; ++e) {
        int c[3] = {(int)(e % m.n[0]), (int)((e / m.n[0]) % m.n[1]), (int)(e / ((int64_t)m.n[0] * m.n[1]))};
        for (int qz = 0; qz < nqe; ++qz)
            for (int qy = 0; qy < nqe; ++qy)
                for (int qx = 0; qx < nqe; ++qx) {
                    double xi[3] = {t.xq[qx], t.xq[qy], t.xq[qz]};
                    double x[3], J[3][3];
                    cell_point(m.n, m.map_kind, m.amp, c, xi, x, J);
                    double uhq = 0.0;
                    for (int i = 0; i < nb; ++i) {
                        int ix = i % np, iy = (i / np) % np, iz = i / (np * np);
                        int64_t g[3];
                        local_to_global(&m, c, np, i, g);
                        uhq += uh[node_index(&m, g)] * t.phi[qx * np + ix] * t.phi[qy * np + iy] * t.phi[qz * np + iz];
                    }
                    double u = sin(OR_PI * x[0]) * sin(OR_PI * x[1]) * sin(OR_PI * x[2]);
                    err2 += (u - uhq) * (u - uhq) * t.wq[qx] * t.wq[qy] * t.wq[qz] * det3(J);
                }
    }
    tab_free(&t);
    return sqrt(err2);
}

/* ------------------------------------------------------------------ */
/* Operator rows evaluated one by one (sampled parity at large sizes)   */
/* ------------------------------------------------------------------ */

/* out[s] = (A u)_{rows[s]}: each row is the sum of the matching rows of
 * the element matrices of the cells around the node (Eq. 4), evaluated
 * without a global matrix. */
int oracle_apply_rows(OM_MESH_ARGS, const double *u, int64_t nrows, const int64_t *rows, double *out)
{
    om_mesh m = OM_MESH_INIT;
    if (mesh_check(&m)) return -1;
    if (m.op != 0) return -3; /* Laplacian rows only */
    om_tab t;
    if (tab_init(&t, k, nq1)) return -2;
    int np = k + 1, nb = np * np * np, nq = t.nq;
    int rc = 0;
#pragma omp parallel
    {
        double *grad = malloc(sizeof(double) * 3 * nb);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < nrows; ++s) {
            int64_t g[3];
            node_coords(&m, rows[s], g);
            if (is_constrained(&m, g)) { out[s] = u[rows[s]]; continue; }
            double acc = 0.0;
            /* cells containing the node */
            int clo[3], chi[3];
            for (int d = 0; d < 3; ++d) {
                if (g[d] % k == 0) {
                    clo[d] = (int)(g[d] / k) - 1;
                    chi[d] = (int)(g[d] / k);
                } else {
                    clo[d] = chi[d] = (int)(g[d] / k);
                }
                if (clo[d] < 0) clo[d] = 0;
                if (chi[d] > m.n[d] - 1) chi[d] = m.n[d] - 1;
            }
            for (int cz = clo[2]; cz <= chi[2]; ++cz)
                for (int cy = clo[1]; cy <= chi[1]; ++cy)
                    for (int cx = clo[0]; cx <= chi[0]; ++cx) {
                        int c[3] = {cx, cy, cz};
                        int il[3];
                        for (int d = 0; d < 3; ++d) il[d] = (int)(g[d] - (int64_t)c[d] * k);
                        double ae = m.coeff ? m.coeff[cx + (int64_t)m.n[0] * (cy + (int64_t)m.n[1] * cz)] : 1.0;
                        for (int qz = 0; qz < nq; ++qz)
                            for (int qy = 0; qy < nq; ++qy)
                                for (int qx = 0; qx < nq; ++qx) {
                                    double xi[3] = {t.xq[qx], t.xq[qy], t.xq[qz]};
                                    double x[3], J[3][3], Ji[3][3];
                                    cell_point(m.n, m.map_kind, m.amp, c, xi, x, J);
                                    double det = det3(J);
                                    inv3(J, det, Ji);
                                    double wdet = ae * t.wq[qx] * t.wq[qy] * t.wq[qz] * det;
                                    /* gradient of u_h restricted to free nodes */
                                    double gu[3] = {0, 0, 0};
                                    for (int j = 0; j < nb; ++j) {
                                        int jx = j % np, jy = (j / np) % np, jz = j / (np * np);
                                        int64_t h[3];
                                        local_to_global(&m, c, np, j, h);
                                        if (is_constrained(&m, h)) continue;
                                        double uj = u[node_index(&m, h)];
                                        double gr[3] = {
                                            t.dphi[qx * np + jx] * t.phi[qy * np + jy] * t.phi[qz * np + jz],
                                            t.phi[qx * np + jx] * t.dphi[qy * np + jy] * t.phi[qz * np + jz],
                                            t.phi[qx * np + jx] * t.phi[qy * np + jy] * t.dphi[qz * np + jz]};
                                        for (int a = 0; a < 3; ++a)
                                            gu[a] += uj * (Ji[0][a] * gr[0] + Ji[1][a] * gr[1] + Ji[2][a] * gr[2]);
                                    }
                                    double gi[3] = {
                                        t.dphi[qx * np + il[0]] * t.phi[qy * np + il[1]] * t.phi[qz * np + il[2]],
                                        t.phi[qx * np + il[0]] * t.dphi[qy * np + il[1]] * t.phi[qz * np + il[2]],
                                        t.phi[qx * np + il[0]] * t.phi[qy * np + il[1]] * t.dphi[qz * np + il[2]]};
                                    for (int a = 0; a < 3; ++a) {
                                        double gia = Ji[0][a] * gi[0] + Ji[1][a] * gi[1] + Ji[2][a] * gi[2];
                                        acc += wdet * gia * gu[a];
                                    }
                                }
                    }
            out[s] = acc;
        }
        free(grad);
    }
    tab_free(&t);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Sparse kernels and Algorithm 1                                       */
/* ------------------------------------------------------------------ */

void oracle_spmv(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                 const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) s += val[p] * x[col[p]];
        y[i] = s;
    }
}

/* Dot product with a summation order that does not depend on the thread
 * count: fixed chunks, chunk sums added in order. */
#define OR_CHUNK 4096
static double dot(int64_t n, const double *a, const double *b, double *scratch)
{
    int64_t nch = (n + OR_CHUNK - 1) / OR_CHUNK;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nch; ++c) {
        double s = 0.0;
        int64_t e = (c + 1) * OR_CHUNK < n ? (c + 1) * OR_CHUNK : n;
        for (int64_t i = c * OR_CHUNK; i < e; ++i) s += a[i] * b[i];
        scratch[c] = s;
    }
    double s = 0.0;
    for (int64_t c = 0; c < nch; ++c) s += scratch[c];
    return s;
}

/* Algorithm 1 (preconditioned CG) with M = diag(A).  x holds x_0 on entry
 * and the last iterate on return.  hist[j] = ||r_j||_2 for j = 0..iters.
 * Returns 0 (converged), -4 (maxit reached), -5 (breakdown p^T A p <= 0). */
int oracle_pcg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
               const double *diag, const double *b, double *x, double tol, int maxit,
               int *iters, double *hist)
{
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *v = malloc(sizeof(double) * n);
    double *scr = malloc(sizeof(double) * ((n + OR_CHUNK - 1) / OR_CHUNK + 1));
    int rc = -4;
    *iters = 0;
    double eps = tol * sqrt(dot(n, b, b, scr));
    oracle_spmv(n, rowptr, col, val, x, v);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        r[i] = b[i] - v[i];
        z[i] = r[i] / diag[i];
        p[i] = z[i];
    }
    double e = dot(n, r, z, scr);
    double rn = sqrt(dot(n, r, r, scr));
    if (hist) hist[0] = rn;
    if (rn < eps || rn == 0.0) { rc = 0; goto done; }
    for (int j = 0; j < maxit; ++j) {
        oracle_spmv(n, rowptr, col, val, p, v);
        double pv = dot(n, p, v, scr);
        if (!(pv > 0.0)) { rc = -5; break; }
        double alpha = e / pv;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * v[i];
        }
        rn = sqrt(dot(n, r, r, scr));
        *iters = j + 1;
        if (hist) hist[j + 1] = rn;
        if (rn < eps) { rc = 0; break; }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) z[i] = r[i] / diag[i];
        double enew = dot(n, r, z, scr);
        double beta = enew / e;
        e = enew;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
done:
    free(r); free(z); free(p); free(v); free(scr);
    return rc;
}

/* The diagonal of a CSR matrix. */
void oracle_csr_diag(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, double *d)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        d[i] = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            if (col[p] == i) d[i] = val[p];
    }
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
