// Fused kernel instantiation: float inputs, double packing, L = 96.
#include "fused.h"

namespace tdg {
TDG_FUSED_INSTANCE(float, double, 96)
}  // namespace tdg
