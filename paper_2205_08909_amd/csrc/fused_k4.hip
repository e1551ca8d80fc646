/* fused_k4.hip -- the fused tile kernels of degree 4 (all operator
 * variants, modes and precisions; see fused_tile.h). */
#include "fused_tile.h"

namespace mfcg {
MFCG_FUSED_DEGREE(4)
}  // namespace mfcg
