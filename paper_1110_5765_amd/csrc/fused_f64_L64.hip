// Fused kernel instantiation: double inputs, double packing, L = 64.
#include "fused.h"

namespace tdg {
TDG_FUSED_INSTANCE(double, double, 64)
}  // namespace tdg
