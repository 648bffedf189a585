// Fused kernel instantiation: float inputs, double packing, L = 128.
#include "fused.h"

namespace tdg {
TDG_FUSED_INSTANCE(float, double, 128)
}  // namespace tdg
