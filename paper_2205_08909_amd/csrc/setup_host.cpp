/*
 * setup_host.cpp -- host-side setup of the fused CG library:
 *   - 1D tables of the sum factorisation (Sec. 2: tensor-product Lagrange
 *     basis of degree k on Gauss-Lobatto points, Gauss quadrature with k+1
 *     points per direction),
 *   - the tile partition and the enumeration of unknowns (the GPU form of
 *     Sec. 5.3: tile-interior unknowns first, then unknowns shared between
 *     tiles grouped by face/edge/vertex, Dirichlet unknowns last).
 * Integer work only, O(n) once per handle.
 */
#include "setup_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace mfcg {

/* ---------------------------------------------------------------- */
/* 1D tables, computed in long double                                 */
/* ---------------------------------------------------------------- */

/* Legendre P_n(t) and P_n'(t) on [-1,1] by the Bonnet recurrence. */
static void legendre_ld(int n, long double t, long double &p, long double &dp)
{
    long double a = 1.0L, b = t;
    if (n == 0) {
        p = 1.0L;
        dp = 0.0L;
        return;
    }
    for (int m = 2; m <= n; ++m) {
        long double c = ((2 * m - 1) * t * b - (m - 1) * a) / m;
        a = b;
        b = c;
    }
    p = b;
    dp = n * (a - t * b) / (1.0L - t * t);
}

static void gauss_points(int n, long double *x, long double *w)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        long double t = -cosl(pi * (i + 0.75L) / (n + 0.5L));
        long double p, dp;
        for (int it = 0; it < 200; ++it) {
            legendre_ld(n, t, p, dp);
            long double dt = p / dp;
            t -= dt;
            if (fabsl(dt) < 1e-19L) break;
        }
        legendre_ld(n, t, p, dp);
        x[i] = 0.5L * (1.0L + t);
        w[i] = 1.0L / ((1.0L - t * t) * dp * dp);
    }
}

static void lobatto_points(int k, long double *x)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    x[0] = 0.0L;
    x[k] = 1.0L;
    for (int i = 1; i < k; ++i) {
        long double t = -cosl(pi * i / k);
        for (int it = 0; it < 200; ++it) {
            long double p, dp;
            legendre_ld(k, t, p, dp);
            long double ddp = (2.0L * t * dp - k * (k + 1.0L) * p) / (1.0L - t * t);
            long double dt = dp / ddp;
            t -= dt;
            if (fabsl(dt) < 1e-19L) break;
        }
        x[i] = 0.5L * (1.0L + t);
    }
}

static void bary_weights(int n, const long double *x, long double *w)
{
    for (int i = 0; i < n; ++i) {
        w[i] = 1.0L;
        for (int j = 0; j < n; ++j)
            if (j != i) w[i] /= (x[i] - x[j]);
    }
}

/* value of the i-th Lagrange polynomial over nodes x at point t */
static long double lagrange_value(int n, const long double *x, int i, long double t)
{
    long double v = 1.0L;
    for (int j = 0; j < n; ++j)
        if (j != i) v *= (t - x[j]) / (x[i] - x[j]);
    return v;
}

void interp_weights(int kf, int kt, double *W)
{
    long double xf[MAXN], xt[MAXN];
    lobatto_points(kf, xf);
    lobatto_points(kt, xt);
    for (int i = 0; i <= kt; ++i)
        for (int j = 0; j <= kf; ++j) W[i * (kf + 1) + j] = (double)lagrange_value(kf + 1, xf, j, xt[i]);
}

int build_tables(int K, Tables<double> &tab, bool gll_quadrature, int nq)
{
    if (nq == 0) nq = K + 1;
    if (K < 1 || K + 1 > MAXN || nq > MAXN || nq < K + 1 || nq > K + 2 || (gll_quadrature && nq != K + 1)) return -1;
    const int n = K + 1;
    long double xg[MAXN], wg[MAXN], xl[MAXN], bw[MAXN];
    gauss_points(nq, xg, wg);
    lobatto_points(K, xl);
    if (gll_quadrature) {
        /* quadrature on the nodes: weights 2 / (k (k+1) P_k(t_i)^2) on
         * [-1,1], halved for [0,1]; P_k(+-1) = (+-1)^k */
        for (int i = 0; i <= K; ++i) {
            long double p = 1.0L, dp = 0.0L;
            if (i == 0)
                p = (K & 1) ? -1.0L : 1.0L;
            else if (i < K)
                legendre_ld(K, 2.0L * xl[i] - 1.0L, p, dp);
            xg[i] = xl[i];
            wg[i] = 1.0L / ((long double)K * (K + 1) * p * p);
        }
    }
    /* S: nq x n (basis at the points), D: nq x nq (collocation derivative
     * on the points), Sd = D S: nq x n (basis derivatives at the points) */
    bary_weights(nq, xg, bw);
    long double S[MAXN * MAXN], D[MAXN * MAXN];
    for (int q = 0; q < nq; ++q)
        for (int i = 0; i < n; ++i) S[q * n + i] = lagrange_value(n, xl, i, xg[q]);
    for (int q = 0; q < nq; ++q) {
        long double diag = 0.0L;
        for (int m = 0; m < nq; ++m) {
            if (m == q) continue;
            D[q * nq + m] = (bw[m] / bw[q]) / (xg[q] - xg[m]);
            diag -= D[q * nq + m];
        }
        D[q * nq + q] = diag;
    }
    std::memset(&tab, 0, sizeof(tab));
    for (int i = 0; i < n; ++i) tab.gll[i] = (double)xl[i];
    for (int q = 0; q < nq; ++q) {
        tab.xq[q] = (double)xg[q];
        tab.wq[q] = (double)wg[q];
        for (int m = 0; m < nq; ++m) tab.D[q * nq + m] = (double)D[q * nq + m];
        for (int i = 0; i < n; ++i) {
            tab.S[q * n + i] = (double)S[q * n + i];
            long double sd = 0.0L;
            for (int m = 0; m < nq; ++m) sd += D[q * nq + m] * S[m * n + i];
            tab.Sd[q * n + i] = (double)sd;
        }
    }
    return 0;
}

/* ---------------------------------------------------------------- */
/* Tile partition and enumeration                                     */
/* ---------------------------------------------------------------- */

void default_tile(int K, int tile[3])
{
    /* xy extent of about 16 nodes per tile (the fused kernel's compiled
     * maximum), z streamed in layers */
    static const int tx[9] = {0, 8, 8, 8, 4, 4, 2, 2, 2}, ty[9] = {0, 8, 8, 4, 4, 3, 2, 2, 1};
    tile[0] = tx[K];
    tile[1] = ty[K];
    tile[2] = 16;
}

/* 1D piece of lattice coordinate g: entity index e (even: plane, odd:
 * segment), local offset l within it, piece length. */
void dim_locate_host(const Dim1 &d, int64_t g, int64_t &e, int64_t &l, int64_t &len)
{
    const int64_t Ek = (int64_t)d.T * d.K;
    const int64_t last = (int64_t)d.ncells * d.K;
    if (g == last) {
        e = 2 * d.ntiles;
        l = 0;
        len = 1;
        return;
    }
    int64_t j = g / Ek, r = g - j * Ek;
    if (r == 0) {
        e = 2 * j;
        l = 0;
        len = 1;
    } else {
        e = 2 * j + 1;
        l = r - 1;
        int64_t cells = std::min<int64_t>(d.T, d.ncells - j * d.T);
        len = cells * d.K - 1;
    }
}

static int64_t piece_len(const Dim1 &d, int64_t e)
{
    if ((e & 1) == 0) return 1;
    int64_t j = e / 2;
    int64_t cells = std::min<int64_t>(d.T, d.ncells - j * d.T);
    return cells * d.K - 1;
}

int build_layout(const int ncells[3], int K, const int tile_in[3], int bc, HostLayout &L, int nq)
{
    L = HostLayout();
    L.K = K;
    int tile[3];
    default_tile(K, tile);
    for (int d = 0; d < 3; ++d) {
        if (tile_in && tile_in[d] > 0) tile[d] = tile_in[d];
        if (tile[d] > ncells[d]) tile[d] = ncells[d];
        L.d[d].ncells = ncells[d];
        L.d[d].T = tile[d];
        L.d[d].ntiles = (ncells[d] + tile[d] - 1) / tile[d];
        L.d[d].K = K;
    }
    int64_t ne[3];
    for (int d = 0; d < 3; ++d) ne[d] = 2 * (int64_t)L.d[d].ntiles + 1;
    L.ne[0] = ne[0];
    L.ne[1] = ne[1];
    L.ne[2] = ne[2];
    const int64_t nent = ne[0] * ne[1] * ne[2];
    L.ent_base.assign(nent, -1);
    L.ent_kind.assign(nent, KIND_I);
    L.ent_class_off.assign(nent, 0);
    L.ntiles = (int64_t)L.d[0].ntiles * L.d[1].ntiles * L.d[2].ntiles;

    auto ent_id = [&](int64_t ex, int64_t ey, int64_t ez) { return ex + ne[0] * (ey + ne[1] * ez); };
    auto is_boundary_plane = [&](int d, int64_t e) {
        return bc == 0 && (e == 0 || e == ne[d] - 1);
    };

    /* classify */
    for (int64_t ez = 0; ez < ne[2]; ++ez)
        for (int64_t ey = 0; ey < ne[1]; ++ey)
            for (int64_t ex = 0; ex < ne[0]; ++ex) {
                int64_t id = ent_id(ex, ey, ez);
                int nplanes = ((ex & 1) == 0) + ((ey & 1) == 0) + ((ez & 1) == 0);
                bool cons = is_boundary_plane(0, ex) || is_boundary_plane(1, ey) || is_boundary_plane(2, ez);
                L.ent_kind[id] = cons ? KIND_C : (nplanes == 0 ? KIND_I : KIND_S);
            }

    /* class I: tile interiors in tile order (tx fastest) */
    int64_t pos = 0;
    L.tiles.resize(L.ntiles);
    int64_t gpos = 0;
    const int n = nq > 0 ? nq : K + 1; /* quadrature points per direction */
    for (int64_t tz = 0; tz < L.d[2].ntiles; ++tz)
        for (int64_t ty = 0; ty < L.d[1].ntiles; ++ty)
            for (int64_t tx = 0; tx < L.d[0].ntiles; ++tx) {
                int64_t t = tx + L.d[0].ntiles * (ty + L.d[1].ntiles * tz);
                int64_t id = ent_id(2 * tx + 1, 2 * ty + 1, 2 * tz + 1);
                L.ent_base[id] = pos;
                pos += piece_len(L.d[0], 2 * tx + 1) * piece_len(L.d[1], 2 * ty + 1) * piece_len(L.d[2], 2 * tz + 1);
                TileDesc &td = L.tiles[t];
                int64_t tt[3] = {tx, ty, tz};
                for (int d = 0; d < 3; ++d) {
                    td.c0[d] = (int32_t)(tt[d] * L.d[d].T);
                    td.nc[d] = (int32_t)std::min<int64_t>(L.d[d].T, L.d[d].ncells - td.c0[d]);
                }
                td.gbase = gpos;
                gpos += 6LL * td.nc[0] * td.nc[1] * td.nc[2] * n * n * n;
            }
    L.nI = pos;
    L.g_elems = gpos;
    /* class S by number of planes, lexicographic entity order; then C */
    int64_t counts[4] = {0, 0, 0, 0};
    int64_t offs[4];
    for (int np_want = 1; np_want <= 3; ++np_want) {
        offs[np_want] = pos;
        for (int64_t ez = 0; ez < ne[2]; ++ez)
            for (int64_t ey = 0; ey < ne[1]; ++ey)
                for (int64_t ex = 0; ex < ne[0]; ++ex) {
                    int64_t id = ent_id(ex, ey, ez);
                    if (L.ent_kind[id] != KIND_S) continue;
                    int nplanes = ((ex & 1) == 0) + ((ey & 1) == 0) + ((ez & 1) == 0);
                    if (nplanes != np_want) continue;
                    L.ent_base[id] = pos;
                    L.ent_class_off[id] = pos - offs[np_want];
                    int64_t sz = piece_len(L.d[0], ex) * piece_len(L.d[1], ey) * piece_len(L.d[2], ez);
                    pos += sz;
                    counts[np_want] += sz;
                }
    }
    L.nF = counts[1];
    L.nE = counts[2];
    L.nV = counts[3];
    L.offF = offs[1];
    L.offE = offs[2];
    L.offV = offs[3];
    L.offC = pos;
    for (int64_t ez = 0; ez < ne[2]; ++ez)
        for (int64_t ey = 0; ey < ne[1]; ++ey)
            for (int64_t ex = 0; ex < ne[0]; ++ex) {
                int64_t id = ent_id(ex, ey, ez);
                if (L.ent_kind[id] != KIND_C) continue;
                L.ent_base[id] = pos;
                pos += piece_len(L.d[0], ex) * piece_len(L.d[1], ey) * piece_len(L.d[2], ez);
            }
    L.nC = pos - L.offC;
    L.n = pos;
    L.partF = 0;
    L.partE = 2 * L.nF;
    L.partV = 2 * L.nF + 4 * L.nE;
    L.npart = 2 * L.nF + 4 * L.nE + 8 * L.nV;

    /* per-tile entity table */
    L.tile_ent.resize(L.ntiles * 27);
    for (int64_t tz = 0; tz < L.d[2].ntiles; ++tz)
        for (int64_t ty = 0; ty < L.d[1].ntiles; ++ty)
            for (int64_t tx = 0; tx < L.d[0].ntiles; ++tx) {
                int64_t t = tx + L.d[0].ntiles * (ty + L.d[1].ntiles * tz);
                for (int dz = 0; dz < 3; ++dz)
                    for (int dy = 0; dy < 3; ++dy)
                        for (int dx = 0; dx < 3; ++dx) {
                            int64_t e[3] = {2 * tx + dx, 2 * ty + dy, 2 * tz + dz};
                            int dd[3] = {dx, dy, dz};
                            int64_t id = ent_id(e[0], e[1], e[2]);
                            EntityRef &r = L.tile_ent[t * 27 + dx + 3 * dy + 9 * dz];
                            r.vbase = L.ent_base[id];
                            r.kind = L.ent_kind[id];
                            r.pad = 0;
                            r.pbase = -1;
                            if (r.kind == KIND_S) {
                                int slot = 0, rank = 0, nplanes = 0;
                                for (int d = 0; d < 3; ++d) {
                                    if ((e[d] & 1) == 0) {
                                        /* the tile sits above the plane when it is its lower plane */
                                        if (dd[d] == 0) slot |= 1 << rank;
                                        ++rank;
                                        ++nplanes;
                                    }
                                }
                                int64_t cls_n = nplanes == 1 ? L.nF : (nplanes == 2 ? L.nE : L.nV);
                                int64_t cls_p = nplanes == 1 ? L.partF : (nplanes == 2 ? L.partE : L.partV);
                                r.pbase = cls_p + slot * cls_n + L.ent_class_off[id];
                            }
                        }
            }
    return 0;
}

/* lexicographic index -> internal index, host version */
void host_permutation(const HostLayout &L, int64_t *perm)
{
    const int64_t lat[3] = {(int64_t)L.d[0].ncells * L.K + 1, (int64_t)L.d[1].ncells * L.K + 1,
                            (int64_t)L.d[2].ncells * L.K + 1};
    for (int64_t gz = 0; gz < lat[2]; ++gz)
        for (int64_t gy = 0; gy < lat[1]; ++gy)
            for (int64_t gx = 0; gx < lat[0]; ++gx) {
                int64_t g[3] = {gx, gy, gz}, e[3], l[3], len[3];
                for (int d = 0; d < 3; ++d) dim_locate_host(L.d[d], g[d], e[d], l[d], len[d]);
                int64_t id = e[0] + L.ne[0] * (e[1] + L.ne[1] * e[2]);
                perm[gx + lat[0] * (gy + lat[1] * gz)] = L.ent_base[id] + l[0] + len[0] * (l[1] + len[1] * l[2]);
            }
}

}  // namespace mfcg
