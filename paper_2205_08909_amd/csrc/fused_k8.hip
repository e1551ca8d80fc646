/* fused_k8.hip -- the fused tile kernels of degree 8 (all operator
 * variants, modes and precisions; see fused_tile.h). */
#include "fused_tile.h"

namespace mfcg {
MFCG_FUSED_DEGREE(8)
}  // namespace mfcg
