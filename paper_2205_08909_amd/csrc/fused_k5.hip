/* fused_k5.hip -- the fused tile kernels of degree 5 (all operator
 * variants, modes and precisions; see fused_tile.h). */
#include "fused_tile.h"

namespace mfcg {
MFCG_FUSED_DEGREE(5)
}  // namespace mfcg
