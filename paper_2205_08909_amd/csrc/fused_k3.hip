/* fused_k3.hip -- the fused tile kernels of degree 3 (all operator
 * variants, modes and precisions; see fused_tile.h). */
#include "fused_tile.h"

namespace mfcg {
MFCG_FUSED_DEGREE(3)
}  // namespace mfcg
