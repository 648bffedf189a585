// Fused kernel instantiation: float inputs, double packing, L = 64.
#include "fused.h"

namespace tdg {
TDG_FUSED_INSTANCE(float, double, 64)
}  // namespace tdg
