/*
 * kernels_setup.hip -- once-per-handle and once-per-solve kernels:
 *   geometry tensor G_q = a_e w_q det(J_q) J_q^{-1} J_q^{-T} per quadrature
 *   point (the "final tensor load" data of Sec. 2.2, Eq. 5), the Jacobi
 *   diagonal (Sec. 3), the load vector, the lexicographic <-> internal
 *   permutations, the solver initialisation (Algorithm 5, first line) and
 *   the delayed x reconstruction at exit (Algorithm 5, exit branch).
 * Node-centric kernels gather over the cells around a node in a fixed
 * order, so no atomics are used and results are reproducible.
 */
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace mfcg {

constexpr int SETUP_WG = 256;

/* ------------------------------------------------------------------ */
/* Geometry                                                            */
/* ------------------------------------------------------------------ */

/* Global map x = F(X) of [0,1]^3 and its Jacobian DF. */
__device__ inline void map_eval(int kind, double A, const double X[3], double x[3], double DF[3][3])
{
    const double twopi = 6.283185307179586476925286766559;
    double s[3], c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) sincos(twopi * X[d], &s[d], &c[d]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        x[i] = X[i];
#pragma unroll
        for (int j = 0; j < 3; ++j) DF[i][j] = i == j ? 1.0 : 0.0;
    }
    if (kind == 1) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int p = (i + 1) % 3, q = (i + 2) % 3;
            x[i] += A * s[p] * s[q];
            DF[i][p] += A * twopi * c[p] * s[q];
            DF[i][q] += A * twopi * s[p] * c[q];
        }
    } else if (kind == 2) {
        const double pr = s[0] * s[1] * s[2];
        const double g[3] = {twopi * c[0] * s[1] * s[2], twopi * s[0] * c[1] * s[2], twopi * s[0] * s[1] * c[2]};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            x[i] += A * pr;
#pragma unroll
            for (int j = 0; j < 3; ++j) DF[i][j] += A * g[j];
        }
    }
}

__device__ inline int64_t x_offset(const LayoutView &L, int nq, const int c[3]);

/* Reference point xi of cell c -> mapped point x, J = dx/dxi, det J (of
 * the quadratic interpolant when g.X holds the quadratic geometry). */
__device__ inline double cell_jacobian(const GeomArgs &g, const int c[3], const double xi[3], double x[3],
                                       double J[3][3])
{
    double X[3], DF[3][3];
    if (g.X) {
        const double *Xc = g.X + x_offset(g.L, g.nq, c);
        double N[3][3], dN[3][3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double t = xi[d];
            N[d][0] = (2.0 * t - 1.0) * (t - 1.0);
            N[d][1] = 4.0 * t * (1.0 - t);
            N[d][2] = t * (2.0 * t - 1.0);
            dN[d][0] = 4.0 * t - 3.0;
            dN[d][1] = 4.0 - 8.0 * t;
            dN[d][2] = 4.0 * t - 1.0;
        }
        for (int i = 0; i < 3; ++i) {
            x[i] = 0.0;
            for (int j = 0; j < 3; ++j) J[i][j] = 0.0;
        }
        for (int p = 0; p < 27; ++p) {
            const int a = p % 3, b = (p / 3) % 3, d = p / 9;
            const double v = N[0][a] * N[1][b] * N[2][d];
            const double gx = dN[0][a] * N[1][b] * N[2][d], gy = N[0][a] * dN[1][b] * N[2][d],
                         gz = N[0][a] * N[1][b] * dN[2][d];
            for (int i = 0; i < 3; ++i) {
                const double xn = Xc[i * 27 + p];
                x[i] += xn * v;
                J[i][0] += xn * gx;
                J[i][1] += xn * gy;
                J[i][2] += xn * gz;
            }
        }
        return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
               J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) X[d] = (c[d] + xi[d]) / g.L.d[d].ncells;
    map_eval(g.map_kind, g.amp, X, x, DF);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) J[i][j] = DF[i][j] / g.L.d[j].ncells;
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/* Offset of component 0 of G at (cell, q) in the tile-blocked layout read
 * by the fused kernel (nq points per direction), and the component stride. */
__device__ inline int64_t g_offset(const LayoutView &L, int nq, const int c[3], int qx, int qy, int qz,
                                   int64_t &cstride)
{
    const int n = nq, n2 = n * n, n3 = n2 * n;
    int t[3], cl[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        t[d] = c[d] / L.d[d].T;
    }
    const int64_t tid = t[0] + (int64_t)L.d[0].ntiles * (t[1] + (int64_t)L.d[1].ntiles * t[2]);
    const TileDesc td = L.tiles[tid];
#pragma unroll
    for (int d = 0; d < 3; ++d) cl[d] = c[d] - td.c0[d];
    const int nlc = td.nc[0] * td.nc[1];
    const int line = (cl[0] + td.nc[0] * cl[1]) * n2 + qx + n * qz;
    cstride = (int64_t)nlc * n3;
    return td.gbase + (int64_t)cl[2] * 6 * nlc * n3 + (int64_t)qy * nlc * n2 + line;
}

/* Offset of cell c's block in the quadratic geometry array: the cells in
 * the order of the geometry tensor (tile, then layer, then x fastest). */
__device__ inline int64_t x_offset(const LayoutView &L, int nq, const int c[3])
{
    const int n3 = nq * nq * nq; /* quadratic geometry of the geometry tensor's nq^3-point layout */
    int t[3], cl[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) t[d] = c[d] / L.d[d].T;
    const int64_t tid = t[0] + (int64_t)L.d[0].ntiles * (t[1] + (int64_t)L.d[1].ntiles * t[2]);
    const TileDesc td = L.tiles[tid];
#pragma unroll
    for (int d = 0; d < 3; ++d) cl[d] = c[d] - td.c0[d];
    const int64_t first = td.gbase / (6 * n3); /* cells of the earlier tiles */
    return (first + cl[0] + (int64_t)td.nc[0] * (cl[1] + (int64_t)td.nc[1] * cl[2])) * QGEOM_STRIDE;
}

__global__ __launch_bounds__(SETUP_WG) void qgeom_nodes_kernel(const GeomArgs g, double *X)
{
    const int64_t ncell = (int64_t)g.L.d[0].ncells * g.L.d[1].ncells * g.L.d[2].ncells;
    const int64_t t = (int64_t)blockIdx.x * SETUP_WG + threadIdx.x;
    if (t >= ncell * 27) return;
    const int64_t cell = t / 27;
    const int p = (int)(t % 27), a = p % 3, b = (p / 3) % 3, d = p / 9;
    const int c[3] = {(int)(cell % g.L.d[0].ncells), (int)((cell / g.L.d[0].ncells) % g.L.d[1].ncells),
                      (int)(cell / ((int64_t)g.L.d[0].ncells * g.L.d[1].ncells))};
    const int ab[3] = {a, b, d};
    double Xp[3], x[3], DF[3][3];
#pragma unroll
    for (int e = 0; e < 3; ++e) Xp[e] = (c[e] + 0.5 * ab[e]) / g.L.d[e].ncells;
    map_eval(g.map_kind, g.amp, Xp, x, DF);
    const int64_t o = x_offset(g.L, g.nq, c);
#pragma unroll
    for (int i = 0; i < 3; ++i) X[o + i * 27 + p] = x[i];
    if (p == 0) X[o + 81] = g.coeff ? g.coeff[cell] : 1.0;
}

hipError_t launch_qgeom_nodes(const GeomArgs &g, double *X, hipStream_t s)
{
    const int64_t tot = (int64_t)g.L.d[0].ncells * g.L.d[1].ncells * g.L.d[2].ncells * 27;
    const int64_t nb = (tot + SETUP_WG - 1) / SETUP_WG;
    hipLaunchKernelGGL(qgeom_nodes_kernel, dim3((unsigned)nb), dim3(SETUP_WG), 0, s, g, X);
    return hipGetLastError();
}

__global__ __launch_bounds__(SETUP_WG) void geometry_kernel(const GeomArgs g, double *G)
{
    const int n = g.nq, n3 = n * n * n;
    const int64_t ncell = (int64_t)g.L.d[0].ncells * g.L.d[1].ncells * g.L.d[2].ncells;
    const int64_t t = (int64_t)blockIdx.x * SETUP_WG + threadIdx.x;
    if (t >= ncell * n3) return;
    const int64_t cell = t / n3;
    const int q = (int)(t % n3), qx = q % n, qy = (q / n) % n, qz = q / (n * n);
    const int c[3] = {(int)(cell % g.L.d[0].ncells), (int)((cell / g.L.d[0].ncells) % g.L.d[1].ncells),
                      (int)(cell / ((int64_t)g.L.d[0].ncells * g.L.d[1].ncells))};
    const double xi[3] = {g.tab.xq[qx], g.tab.xq[qy], g.tab.xq[qz]};
    double x[3], J[3][3];
    const double det = cell_jacobian(g, c, xi, x, J);
    double Ji[3][3];
    const double id = 1.0 / det;
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    const double ae = g.coeff ? g.coeff[cell] : 1.0;
    const double w = ae * g.tab.wq[qx] * g.tab.wq[qy] * g.tab.wq[qz] * det;
    auto m = [&](int p, int r) { return w * (Ji[p][0] * Ji[r][0] + Ji[p][1] * Ji[r][1] + Ji[p][2] * Ji[r][2]); };
    int64_t cs;
    const int64_t o = g_offset(g.L, n, c, qx, qy, qz, cs);
    if (g.op == 1) { /* mass operator: a_e w_q det J_q */
        G[o] = w;
        for (int comp = 1; comp < 6; ++comp) G[o + comp * cs] = 0.0;
        return;
    }
    G[o] = m(0, 0);
    G[o + cs] = m(1, 1);
    G[o + 2 * cs] = m(2, 2);
    G[o + 3 * cs] = m(0, 1);
    G[o + 4 * cs] = m(0, 2);
    G[o + 5 * cs] = m(1, 2);
}

hipError_t launch_geometry(const GeomArgs &g, double *G, hipStream_t s)
{
    const int n = g.nq;
    const int64_t tot = (int64_t)g.L.d[0].ncells * g.L.d[1].ncells * g.L.d[2].ncells * n * n * n;
    const int64_t nb = (tot + SETUP_WG - 1) / SETUP_WG;
    hipLaunchKernelGGL(geometry_kernel, dim3((unsigned)nb), dim3(SETUP_WG), 0, s, g, G);
    return hipGetLastError();
}

/* ------------------------------------------------------------------ */
/* Node helpers                                                        */
/* ------------------------------------------------------------------ */

__device__ inline void dim_locate(const Dim1 &d, int64_t g, int64_t &e, int64_t &l, int64_t &len)
{
    const int64_t Ek = (int64_t)d.T * d.K;
    const int64_t last = (int64_t)d.ncells * d.K;
    if (g == last) {
        e = 2 * (int64_t)d.ntiles;
        l = 0;
        len = 1;
        return;
    }
    const int64_t j = g / Ek, r = g - j * Ek;
    if (r == 0) {
        e = 2 * j;
        l = 0;
        len = 1;
    } else {
        e = 2 * j + 1;
        l = r - 1;
        const int64_t rem = d.ncells - j * d.T;
        len = (rem < d.T ? rem : d.T) * d.K - 1;
    }
}

__device__ inline int64_t internal_index(const LayoutView &L, const int64_t g[3])
{
    int64_t e[3], l[3], len[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) dim_locate(L.d[d], g[d], e[d], l[d], len[d]);
    const int64_t ne0 = 2 * (int64_t)L.d[0].ntiles + 1, ne1 = 2 * (int64_t)L.d[1].ntiles + 1;
    return L.ent_base[e[0] + ne0 * (e[1] + ne1 * e[2])] + l[0] + len[0] * (l[1] + len[1] * l[2]);
}

__device__ inline void lex_coords(const LayoutView &L, int64_t t, int64_t g[3])
{
    const int64_t l0 = (int64_t)L.d[0].ncells * L.d[0].K + 1, l1 = (int64_t)L.d[1].ncells * L.d[1].K + 1;
    g[0] = t % l0;
    g[1] = (t / l0) % l1;
    g[2] = t / (l0 * l1);
}

__device__ inline bool on_boundary(const LayoutView &L, const int64_t g[3])
{
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (g[d] == 0 || g[d] == (int64_t)L.d[d].ncells * L.d[d].K) return true;
    return false;
}

/* cells containing lattice coordinate gd in one direction */
__device__ inline void cell_range(const Dim1 &d, int64_t gd, int &lo, int &hi)
{
    if (gd % d.K == 0) {
        lo = (int)(gd / d.K) - 1;
        hi = (int)(gd / d.K);
    } else {
        lo = hi = (int)(gd / d.K);
    }
    if (lo < 0) lo = 0;
    if (hi > d.ncells - 1) hi = d.ncells - 1;
}

/* ------------------------------------------------------------------ */
/* Cell-by-cell assembly of node vectors                               */
/* ------------------------------------------------------------------ */

/* The cells whose coordinates have the parities of `colour` (bit d: odd in
 * direction d) share no node, so the cells of one colour class add their
 * element contributions into a node vector without atomics; the 8 classes
 * run one after another, so every node's sum has a fixed order. */
constexpr int CELL_WG = 256;
constexpr int MAXQ3 = 9 * 9 * 9; /* up to 9 quadrature points per direction */

__device__ inline bool colour_cell(const LayoutView &L, int colour, int64_t b, int c[3])
{
    int64_t nc[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) nc[d] = (L.d[d].ncells - ((colour >> d) & 1) + 1) / 2;
    if (b >= nc[0] * nc[1] * nc[2]) return false;
    c[0] = (int)(2 * (b % nc[0]) + (colour & 1));
    c[1] = (int)(2 * ((b / nc[0]) % nc[1]) + ((colour >> 1) & 1));
    c[2] = (int)(2 * (b / (nc[0] * nc[1])) + ((colour >> 2) & 1));
    return true;
}

/* v[0..n) = 0 (a kernel rather than a memset node, so that a caller may
 * capture the assembly in a graph) */
__global__ __launch_bounds__(SETUP_WG) void zero_kernel(int64_t n, double *v)
{
    const int64_t t = (int64_t)blockIdx.x * SETUP_WG + threadIdx.x;
    if (t < n) v[t] = 0.0;
}

static void launch_zero(int64_t n, double *v, hipStream_t s)
{
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + SETUP_WG - 1) / SETUP_WG)), dim3(SETUP_WG), 0, s, n, v);
}

/* lexicographic index of local node (ix, iy, iz) of cell c */
__device__ inline int64_t cell_node_lex(const LayoutView &L, int K, const int c[3], int ix, int iy, int iz)
{
    const int64_t l0 = (int64_t)L.d[0].ncells * K + 1, l1 = (int64_t)L.d[1].ncells * K + 1;
    return ((int64_t)c[0] * K + ix) + l0 * (((int64_t)c[1] * K + iy) + l1 * ((int64_t)c[2] * K + iz));
}

/* ------------------------------------------------------------------ */
/* Diagonal (Sec. 3: point Jacobi)                                     */
/* ------------------------------------------------------------------ */

/* One cell of colour class `colour` per workgroup: the cell's tensor G_q
 * staged in LDS, then every local node i adds
 * sum_q (grad phi_i)^T G_q grad phi_i (Laplacian) or sum_q G_q phi_i^2
 * (mass: component 0 holds a_e w_q det J_q) into diag_lex. */
__global__ __launch_bounds__(CELL_WG) void diagonal_cells_kernel(const GeomArgs g, const double *G, int colour,
                                                                 double *diag_lex)
{
    __shared__ double gs[6 * MAXQ3];
    const LayoutView &L = g.L;
    const int K = g.K, n = K + 1, nq = g.nq, nq3 = nq * nq * nq;
    int c[3];
    if (!colour_cell(L, colour, blockIdx.x, c)) return;
    const int ncomp = g.op == 1 ? 1 : 6;
    for (int q = threadIdx.x; q < nq3; q += CELL_WG) {
        const int qx = q % nq, qy = (q / nq) % nq, qz = q / (nq * nq);
        int64_t cs;
        const int64_t o = g_offset(L, nq, c, qx, qy, qz, cs);
        for (int comp = 0; comp < ncomp; ++comp) gs[comp * nq3 + q] = G[o + comp * cs];
    }
    __syncthreads();
    for (int li = threadIdx.x; li < n * n * n; li += CELL_WG) {
        const int ix = li % n, iy = (li / n) % n, iz = li / (n * n);
        double dsum = 0.0;
        for (int qz = 0; qz < nq; ++qz)
            for (int qy = 0; qy < nq; ++qy)
                for (int qx = 0; qx < nq; ++qx) {
                    const int q = qx + nq * (qy + nq * qz);
                    const double sx = g.tab.S[qx * n + ix], sy = g.tab.S[qy * n + iy], sz = g.tab.S[qz * n + iz];
                    if (g.op == 1) {
                        const double phi = sx * sy * sz;
                        dsum += gs[q] * phi * phi;
                        continue;
                    }
                    const double gx = g.tab.Sd[qx * n + ix] * sy * sz;
                    const double gy = sx * g.tab.Sd[qy * n + iy] * sz;
                    const double gz = sx * sy * g.tab.Sd[qz * n + iz];
                    dsum += gs[q] * gx * gx + gs[nq3 + q] * gy * gy + gs[2 * nq3 + q] * gz * gz +
                            2.0 * (gs[3 * nq3 + q] * gx * gy + gs[4 * nq3 + q] * gx * gz + gs[5 * nq3 + q] * gy * gz);
                }
        diag_lex[cell_node_lex(L, K, c, ix, iy, iz)] += dsum;
    }
}

/* Dirichlet rows (identity: diagonal 1) and the inverse in internal order. */
__global__ __launch_bounds__(SETUP_WG) void diagonal_finish_kernel(const GeomArgs g, double *diag_lex,
                                                                   double *dinv_int)
{
    const LayoutView &L = g.L;
    const int64_t t = (int64_t)blockIdx.x * SETUP_WG + threadIdx.x;
    if (t >= L.n) return;
    int64_t gc[3];
    lex_coords(L, t, gc);
    double d = diag_lex[t];
    if (g.bc == 0 && on_boundary(L, gc)) {
        d = 1.0;
        diag_lex[t] = d;
    }
    if (dinv_int) dinv_int[internal_index(L, gc)] = 1.0 / d;
}

hipError_t launch_diagonal(const GeomArgs &g, const double *G, double *diag_lex, double *dinv_int, hipStream_t s)
{
    if (g.nq * g.nq * g.nq > MAXQ3) return hipErrorInvalidValue;
    launch_zero(g.L.n, diag_lex, s);
    for (int colour = 0; colour < 8; ++colour) {
        int64_t m = 1;
        for (int d = 0; d < 3; ++d) m *= (g.L.d[d].ncells - ((colour >> d) & 1) + 1) / 2;
        if (m == 0) continue;
        hipLaunchKernelGGL(diagonal_cells_kernel, dim3((unsigned)m), dim3(CELL_WG), 0, s, g, G, colour, diag_lex);
    }
    const int64_t nb = (g.L.n + SETUP_WG - 1) / SETUP_WG;
    hipLaunchKernelGGL(diagonal_finish_kernel, dim3((unsigned)nb), dim3(SETUP_WG), 0, s, g, diag_lex, dinv_int);
    return hipGetLastError();
}

/* ------------------------------------------------------------------ */
/* Load vector                                                         */
/* ------------------------------------------------------------------ */

struct RhsParams {
    int32_t kind, nbumps;
    double p[5 * 16];
};

__device__ inline double forcing(const RhsParams &f, const double x[3])
{
    const double pi = 3.141592653589793238462643383279;
    if (f.kind == 0) return 3.0 * pi * pi * sin(pi * x[0]) * sin(pi * x[1]) * sin(pi * x[2]);
    double s = 0.0;
    for (int b = 0; b < f.nbumps; ++b) {
        const double *q = f.p + 5 * b;
        const double dx = x[0] - q[1], dy = x[1] - q[2], dz = x[2] - q[3];
        s += q[0] * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * q[4] * q[4]));
    }
    return s;
}

/* One cell of colour class `colour` per workgroup: f(x_q) w_q det J_q at
 * the cell's quadrature points, staged in LDS, then every local node i
 * that is not a Dirichlet node adds sum_q phi_i(x_q) f(x_q) w_q det J_q
 * into b. */
__global__ __launch_bounds__(CELL_WG) void rhs_cells_kernel(const GeomArgs g, const RhsParams f, int colour, double *b)
{
    __shared__ double fq[MAXQ3];
    const LayoutView &L = g.L;
    const int K = g.K, n = K + 1, nq = g.nq, nq3 = nq * nq * nq;
    int c[3];
    if (!colour_cell(L, colour, blockIdx.x, c)) return;
    for (int q = threadIdx.x; q < nq3; q += CELL_WG) {
        const int qx = q % nq, qy = (q / nq) % nq, qz = q / (nq * nq);
        const double xi[3] = {g.tab.xq[qx], g.tab.xq[qy], g.tab.xq[qz]};
        double x[3], J[3][3];
        const double det = cell_jacobian(g, c, xi, x, J);
        fq[q] = forcing(f, x) * g.tab.wq[qx] * g.tab.wq[qy] * g.tab.wq[qz] * det;
    }
    __syncthreads();
    for (int li = threadIdx.x; li < n * n * n; li += CELL_WG) {
        const int ix = li % n, iy = (li / n) % n, iz = li / (n * n);
        const int64_t gc[3] = {(int64_t)c[0] * K + ix, (int64_t)c[1] * K + iy, (int64_t)c[2] * K + iz};
        if (g.bc == 0 && on_boundary(L, gc)) continue;
        double acc = 0.0;
        for (int qz = 0; qz < nq; ++qz)
            for (int qy = 0; qy < nq; ++qy) {
                const double syz = g.tab.S[qy * n + iy] * g.tab.S[qz * n + iz];
                for (int qx = 0; qx < nq; ++qx) acc += fq[qx + nq * (qy + nq * qz)] * g.tab.S[qx * n + ix] * syz;
            }
        b[cell_node_lex(L, K, c, ix, iy, iz)] += acc;
    }
}

hipError_t launch_rhs(const GeomArgs &g, int kind, const double *params, int nparams, double *b_lex, hipStream_t s)
{
    RhsParams f;
    f.kind = kind;
    f.nbumps = 0;
    if (kind == 1) {
        f.nbumps = (int)params[0];
        if (f.nbumps < 0 || f.nbumps > 16 || nparams < 1 + 5 * f.nbumps) return hipErrorInvalidValue;
        for (int i = 0; i < 5 * f.nbumps; ++i) f.p[i] = params[1 + i];
    }
    if (g.nq * g.nq * g.nq > MAXQ3) return hipErrorInvalidValue;
    launch_zero(g.L.n, b_lex, s);
    for (int colour = 0; colour < 8; ++colour) {
        int64_t m = 1;
        for (int d = 0; d < 3; ++d) m *= (g.L.d[d].ncells - ((colour >> d) & 1) + 1) / 2;
        if (m == 0) continue;
        hipLaunchKernelGGL(rhs_cells_kernel, dim3((unsigned)m), dim3(CELL_WG), 0, s, g, f, colour, b_lex);
    }
    return hipGetLastError();
}

/* ------------------------------------------------------------------ */
/* Permutations and vector kernels                                     */
/* ------------------------------------------------------------------ */

template <typename T>
__global__ __launch_bounds__(SETUP_WG) void lex_to_int_kernel(const LayoutView L, const double *in, T *out)
{
    const int64_t t = (int64_t)blockIdx.x * SETUP_WG + threadIdx.x;
    if (t >= L.n) return;
    int64_t g[3];
    lex_coords(L, t, g);
    out[internal_index(L, g)] = (T)in[t];
}

template <typename T>
__global__ __launch_bounds__(SETUP_WG) void int_to_lex_kernel(const LayoutView L, const T *in, double *out)
{
    const int64_t t = (int64_t)blockIdx.x * SETUP_WG + threadIdx.x;
    if (t >= L.n) return;
    int64_t g[3];
    lex_coords(L, t, g);
    out[t] = (double)in[internal_index(L, g)];
}

template <typename T>
hipError_t launch_lex_to_int(const LayoutView &L, const double *in_lex, T *out_int, hipStream_t s)
{
    const int64_t nb = (L.n + SETUP_WG - 1) / SETUP_WG;
    hipLaunchKernelGGL((lex_to_int_kernel<T>), dim3((unsigned)nb), dim3(SETUP_WG), 0, s, L, in_lex, out_int);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_int_to_lex(const LayoutView &L, const T *in_int, double *out_lex, hipStream_t s)
{
    const int64_t nb = (L.n + SETUP_WG - 1) / SETUP_WG;
    hipLaunchKernelGGL((int_to_lex_kernel<T>), dim3((unsigned)nb), dim3(SETUP_WG), 0, s, L, in_int, out_lex);
    return hipGetLastError();
}

template hipError_t launch_lex_to_int<double>(const LayoutView &, const double *, double *, hipStream_t);
template hipError_t launch_lex_to_int<float>(const LayoutView &, const double *, float *, hipStream_t);
template hipError_t launch_int_to_lex<double>(const LayoutView &, const double *, double *, hipStream_t);
template hipError_t launch_int_to_lex<float>(const LayoutView &, const float *, double *, hipStream_t);

/* r = r - v (when use_v), p = 0, v = 0: Algorithm 5, first line. */
__global__ __launch_bounds__(SETUP_WG) void init_cg_kernel(int64_t n, double *r, double *p, double *v, int use_v)
{
    const int64_t i = (int64_t)blockIdx.x * SETUP_WG + threadIdx.x;
    if (i >= n) return;
    if (use_v) r[i] = r[i] - v[i];
    p[i] = 0.0;
    v[i] = 0.0;
}

hipError_t launch_init_cg(int64_t n, double *r, double *p, double *v, int use_v, hipStream_t s)
{
    const int64_t nb = (n + SETUP_WG - 1) / SETUP_WG;
    hipLaunchKernelGGL(init_cg_kernel, dim3((unsigned)nb), dim3(SETUP_WG), 0, s, n, r, p, v, use_v);
    return hipGetLastError();
}

/* part[b] = sum over block b's grid-stride range of (a_i - c_i)^2 (c may be
 * NULL); partial sums in a fixed order, finished on the host. */
__global__ __launch_bounds__(SETUP_WG) void sumsq_kernel(int64_t n, const double *a, const double *c, double *part)
{
    __shared__ double red[SETUP_WG / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * SETUP_WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * SETUP_WG) {
        const double d = c ? a[i] - c[i] : a[i];
        s += d * d;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < SETUP_WG / 64; ++w) t += red[w];
        part[blockIdx.x] = t;
    }
}

hipError_t launch_sumsq(int64_t n, const double *b, const double *ax, double *part, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(sumsq_kernel, dim3((unsigned)nb), dim3(SETUP_WG), 0, s, n, b, ax, part);
    return hipGetLastError();
}

/* part[block] = partial sums of a_i b_i (mode 0) or (a_i - s b_i)^2 (mode 1) */
__global__ __launch_bounds__(SETUP_WG) void pair_sum_kernel(int64_t n, int mode, const double *a, const double *b,
                                                            double sc, double *part)
{
    __shared__ double red[SETUP_WG / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * SETUP_WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * SETUP_WG) {
        if (mode == 0) {
            s += a[i] * b[i];
        } else {
            const double d = fma(-sc, b[i], a[i]);
            s += d * d;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < SETUP_WG / 64; ++w) t += red[w];
        part[blockIdx.x] = t;
    }
}

hipError_t launch_pair_sum(int64_t n, int mode, const double *a, const double *b, double sc, double *part, int nb,
                           hipStream_t s)
{
    hipLaunchKernelGGL(pair_sum_kernel, dim3((unsigned)nb), dim3(SETUP_WG), 0, s, n, mode, a, b, sc, part);
    return hipGetLastError();
}

__global__ __launch_bounds__(SETUP_WG) void scale_kernel(int64_t n, const double *a, double sc, double *out)
{
    const int64_t i = (int64_t)blockIdx.x * SETUP_WG + threadIdx.x;
    if (i < n) out[i] = sc * a[i];
}

hipError_t launch_scale(int64_t n, const double *a, double sc, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((n + SETUP_WG - 1) / SETUP_WG)), dim3(SETUP_WG), 0, s, n, a, sc,
                       out);
    return hipGetLastError();
}

/* Interpolation of a continuous Q_kf function (lexicographic nodal values
 * on the GLL nodes of every cell) at the nodes of the Q_kt space on the
 * same cells: each destination node lies in cell e = min(g / kt, N - 1)
 * of every axis at local index i = g - kt e, and its value is the tensor
 * product of the 1D weights W[i][j] = L_j(xi_i) over the (kf + 1)^3 source
 * nodes of that cell.  One thread per destination node. */
__global__ __launch_bounds__(SETUP_WG) void interpolate_kernel(const InterpArgs a)
{
    const int64_t nx = (int64_t)a.ncells[0] * a.kt + 1, ny = (int64_t)a.ncells[1] * a.kt + 1;
    const int64_t nz = (int64_t)a.ncells[2] * a.kt + 1;
    const int64_t g = (int64_t)blockIdx.x * SETUP_WG + threadIdx.x;
    if (g >= nx * ny * nz) return;
    const int64_t gz = g / (nx * ny), rem = g - gz * nx * ny, gy = rem / nx, gx = rem - gy * nx;
    const int64_t gg[3] = {gx, gy, gz};
    int64_t base[3];
    int li[3];
    for (int d = 0; d < 3; ++d) {
        const int64_t e = min(gg[d] / a.kt, (int64_t)a.ncells[d] - 1);
        li[d] = (int)(gg[d] - e * a.kt);
        base[d] = e * a.kf;
    }
    const int64_t sx = (int64_t)a.ncells[0] * a.kf + 1, sy = (int64_t)a.ncells[1] * a.kf + 1;
    const int nf = a.kf + 1;
    double acc = 0.0;
    for (int jz = 0; jz < nf; ++jz) {
        const double wz = a.W[li[2] * nf + jz];
        if (wz == 0.0) continue;
        for (int jy = 0; jy < nf; ++jy) {
            const double wyz = wz * a.W[li[1] * nf + jy];
            if (wyz == 0.0) continue;
            const double *row = a.src + ((base[2] + jz) * sy + base[1] + jy) * sx + base[0];
            double t = 0.0;
            for (int jx = 0; jx < nf; ++jx) t += a.W[li[0] * nf + jx] * row[jx];
            acc += wyz * t;
        }
    }
    a.dst[g] = acc;
}

hipError_t launch_interpolate(const InterpArgs &a, hipStream_t s)
{
    const int64_t n = ((int64_t)a.ncells[0] * a.kt + 1) * ((int64_t)a.ncells[1] * a.kt + 1) *
                      ((int64_t)a.ncells[2] * a.kt + 1);
    hipLaunchKernelGGL(interpolate_kernel, dim3((unsigned)((n + SETUP_WG - 1) / SETUP_WG)), dim3(SETUP_WG), 0, s, a);
    return hipGetLastError();
}

/* out = sum_i c_i U_i over m <= LINCOMB_MAX vectors U_i = U + i n */
__global__ __launch_bounds__(SETUP_WG) void lincomb_kernel(int64_t n, int m, const double *__restrict__ U,
                                                           const LinComb c, double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * SETUP_WG + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int j = 0; j < m; ++j) acc += c.c[j] * U[j * n + i];
    out[i] = acc;
}

hipError_t launch_lincomb(int64_t n, int m, const double *U, const LinComb &c, double *out, hipStream_t s)
{
    if (m < 1 || m > LINCOMB_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(lincomb_kernel, dim3((unsigned)((n + SETUP_WG - 1) / SETUP_WG)), dim3(SETUP_WG), 0, s, n, m, U,
                       c, out);
    return hipGetLastError();
}

/* Algorithm 5 exit: x_{k+1} = x_k + alpha_k p_k (k odd) or
 * x_{k-1} + alpha_k p_k + alpha_{k-1}/beta_{k-1} (p_k - D^{-1} r_k) (k even);
 * x_k on breakdown (xa = 0). */
template <typename T>
__global__ __launch_bounds__(SETUP_WG) void reconstruct_kernel(int64_t n, T *x, const T *p, const T *r,
                                                               const T *dinv, const CGState *st)
{
    const int64_t i = (int64_t)blockIdx.x * SETUP_WG + threadIdx.x;
    if (i >= n) return;
    const int k = st->k;
    if (k == 0) return;
    const T xa = (T)st->xa, xr = (T)st->xratio;
    T xi = fma(xa, p[i], x[i]);
    if ((k & 1) == 0) xi = fma(xr, fma(dinv ? -dinv[i] : (T)-1, r[i], p[i]), xi);
    x[i] = xi;
}

template <typename T>
hipError_t launch_reconstruct(int64_t n, T *x, const T *p, const T *r, const T *dinv, const CGState *st,
                              hipStream_t s)
{
    const int64_t nb = (n + SETUP_WG - 1) / SETUP_WG;
    hipLaunchKernelGGL((reconstruct_kernel<T>), dim3((unsigned)nb), dim3(SETUP_WG), 0, s, n, x, p, r, dinv, st);
    return hipGetLastError();
}
template hipError_t launch_reconstruct<double>(int64_t, double *, const double *, const double *, const double *,
                                               const CGState *, hipStream_t);
template hipError_t launch_reconstruct<float>(int64_t, float *, const float *, const float *, const float *,
                                              const CGState *, hipStream_t);

__global__ __launch_bounds__(SETUP_WG) void convert_kernel(int64_t n, const double *in, float *out)
{
    const int64_t i = (int64_t)blockIdx.x * SETUP_WG + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

hipError_t launch_convert(int64_t n, const double *in, float *out, hipStream_t s)
{
    const int64_t nb = (n + SETUP_WG - 1) / SETUP_WG;
    hipLaunchKernelGGL(convert_kernel, dim3((unsigned)nb), dim3(SETUP_WG), 0, s, n, in, out);
    return hipGetLastError();
}

}  // namespace mfcg

namespace mfcg {

/* ------------------------------------------------------------------ */
/* Streaming reference kernels: the measured bandwidth ceiling of the    */
/* device (copy: 1 read + 1 write per element; read: 1 read, reduced)    */
/* ------------------------------------------------------------------ */

/* U independent 16-byte loads in flight per thread (grid-stride blocks of
 * U strides), optionally with the non-temporal hint. */
typedef double dbl2 __attribute__((ext_vector_type(2)));

template <int U, bool NT>
__device__ __forceinline__ dbl2 sload(const dbl2 *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <int U, bool NT>
__global__ __launch_bounds__(256) void stream_copy_kernel(int64_t n2, const dbl2 *__restrict__ src,
                                                          dbl2 *__restrict__ dst)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + (U - 1) * stride < n2; i += U * stride) {
        dbl2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = sload<U, NT>(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (NT)
                __builtin_nontemporal_store(v[u], dst + i + u * stride);
            else
                dst[i + u * stride] = v[u];
        }
    }
    for (; i < n2; i += stride) dst[i] = src[i];
}

template <int U, bool NT>
__global__ __launch_bounds__(256) void stream_read_kernel(int64_t n2, const dbl2 *__restrict__ src, double *out)
{
    __shared__ double red[4];
    const int64_t stride = (int64_t)gridDim.x * 256;
    double s = 0.0;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + (U - 1) * stride < n2; i += U * stride) {
        dbl2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = sload<U, NT>(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u].x + v[u].y;
    }
    for (; i < n2; i += stride) {
        const dbl2 v = src[i];
        s += v.x + v.y;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

template <int U, bool NT>
static void launch_stream_t(bool read, int64_t n2, const double *src, double *dst, int nblocks, hipStream_t s)
{
    if (read)
        hipLaunchKernelGGL((stream_read_kernel<U, NT>), dim3(nblocks), dim3(256), 0, s, n2, (const dbl2 *)src, dst);
    else
        hipLaunchKernelGGL((stream_copy_kernel<U, NT>), dim3(nblocks), dim3(256), 0, s, n2, (const dbl2 *)src,
                           (dbl2 *)dst);
}

/* kind: bit 0 read (1) or copy (0); bits 1-2: log2 of the loads in flight
 * per thread (1, 2 or 4); bit 3: non-temporal hint */
hipError_t launch_stream(int kind, int64_t n, const double *src, double *dst, int nblocks, hipStream_t s)
{
    const int64_t n2 = n / 2;
    const bool read = kind & 1, nt = kind & 8;
    const int lu = (kind >> 1) & 3;
    if (lu == 0) nt ? launch_stream_t<1, true>(read, n2, src, dst, nblocks, s) : launch_stream_t<1, false>(read, n2, src, dst, nblocks, s);
    else if (lu == 1) nt ? launch_stream_t<2, true>(read, n2, src, dst, nblocks, s) : launch_stream_t<2, false>(read, n2, src, dst, nblocks, s);
    else nt ? launch_stream_t<4, true>(read, n2, src, dst, nblocks, s) : launch_stream_t<4, false>(read, n2, src, dst, nblocks, s);
    return hipGetLastError();
}

}  // namespace mfcg

namespace mfcg {

/* r = b - v (FP64, internal order) */
__global__ __launch_bounds__(256) void residual_kernel(int64_t n, const double *b, const double *v, double *r)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) r[i] = b[i] - v[i];
}

/* x += (double) d */
__global__ __launch_bounds__(256) void add_correction_kernel(int64_t n, double *x, const float *d)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] += (double)d[i];
}

hipError_t launch_residual(int64_t n, const double *b, const double *v, double *r, hipStream_t s)
{
    hipLaunchKernelGGL(residual_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, b, v, r);
    return hipGetLastError();
}

hipError_t launch_add_correction(int64_t n, double *x, const float *d, hipStream_t s)
{
    hipLaunchKernelGGL(add_correction_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, x, d);
    return hipGetLastError();
}

}  // namespace mfcg
