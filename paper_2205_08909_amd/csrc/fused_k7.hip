/* fused_k7.hip -- the fused tile kernels of degree 7 (all operator
 * variants, modes and precisions; see fused_tile.h). */
#include "fused_tile.h"

namespace mfcg {
MFCG_FUSED_DEGREE(7)
}  // namespace mfcg
