/* fused_k6.hip -- the fused tile kernels of degree 6 (all operator
 * variants, modes and precisions; see fused_tile.h). */
#include "fused_tile.h"

namespace mfcg {
MFCG_FUSED_DEGREE(6)
}  // namespace mfcg
