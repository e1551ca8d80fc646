/* fused_k2.hip -- the fused tile kernels of degree 2 (all operator
 * variants, modes and precisions; see fused_tile.h). */
#include "fused_tile.h"

namespace mfcg {
MFCG_FUSED_DEGREE(2)
}  // namespace mfcg
