/* fused_k1.hip -- the fused tile kernels of degree 1 (all operator
 * variants, modes and precisions; see fused_tile.h). */
#include "fused_tile.h"

namespace mfcg {
MFCG_FUSED_DEGREE(1)
}  // namespace mfcg
