/* setup_host.h -- host setup routines of the fused CG library. */
#pragma once
#include <stdint.h>

#include <vector>

#include "mfcg_internal.h"

namespace mfcg {

struct HostLayout {
    int K = 0;
    Dim1 d[3] = {};
    int64_t ne[3] = {0, 0, 0};
    int64_t n = 0, nI = 0, nF = 0, nE = 0, nV = 0, nC = 0;
    int64_t offF = 0, offE = 0, offV = 0, offC = 0;
    int64_t partF = 0, partE = 0, partV = 0, npart = 0;
    int64_t ntiles = 0;
    int64_t g_elems = 0; /* elements of the geometry tensor (6 per q-point) */
    std::vector<int64_t> ent_base;
    std::vector<int32_t> ent_kind;
    std::vector<int64_t> ent_class_off;
    std::vector<EntityRef> tile_ent;
    std::vector<TileDesc> tiles;
};

/* nq Gauss points per direction (default k + 1; k + 2 allowed) or, with
 * gll_quadrature, the k + 1 GLL nodes themselves as quadrature points
 * (S = identity).  S and Sd are nq x (k+1), D is nq x nq, row-major. */
int build_tables(int K, Tables<double> &tab, bool gll_quadrature = false, int nq = 0);
void default_tile(int K, int tile[3]);
/* W[i (kf+1) + j] = the j-th degree-kf Lagrange polynomial on the GLL nodes
 * of [0, 1], evaluated at the i-th degree-kt GLL node (kf, kt in 1..8) */
void interp_weights(int kf, int kt, double *W);
/* nq: quadrature points per direction of the geometry tensor (0: k + 1) */
int build_layout(const int ncells[3], int K, const int tile[3], int bc, HostLayout &L, int nq = 0);
void dim_locate_host(const Dim1 &d, int64_t g, int64_t &e, int64_t &l, int64_t &len);
void host_permutation(const HostLayout &L, int64_t *perm);

}  // namespace mfcg
