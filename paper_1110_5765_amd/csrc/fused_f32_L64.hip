// Fused kernel instantiation: float inputs, float packing, L = 64.
#include "fused.h"

namespace tdg {
TDG_FUSED_INSTANCE(float, float, 64)
}  // namespace tdg
