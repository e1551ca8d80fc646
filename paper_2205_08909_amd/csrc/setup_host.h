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

/* Gauss points (default) or, with gll_quadrature, the GLL nodes themselves
 * as quadrature points (S = identity). */
int build_tables(int K, Tables<double> &tab, bool gll_quadrature = false);
void default_tile(int K, int tile[3]);
int build_layout(const int ncells[3], int K, const int tile[3], int bc, HostLayout &L);
void dim_locate_host(const Dim1 &d, int64_t g, int64_t &e, int64_t &l, int64_t &len);
void host_permutation(const HostLayout &L, int64_t *perm);

}  // namespace mfcg
