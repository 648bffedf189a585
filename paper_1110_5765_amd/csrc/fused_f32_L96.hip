// Fused kernel instantiation: float inputs, float packing, L = 96.
#include "fused.h"

namespace tdg {
TDG_FUSED_INSTANCE(float, float, 96)
}  // namespace tdg
