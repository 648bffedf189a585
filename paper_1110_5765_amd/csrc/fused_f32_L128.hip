// Fused kernel instantiation: float inputs, float packing, L = 128.
#include "fused.h"

namespace tdg {
TDG_FUSED_INSTANCE(float, float, 128)
}  // namespace tdg
