// Fused kernel instantiation: double inputs, double packing, L = 96.
#include "fused.h"

namespace tdg {
TDG_FUSED_INSTANCE(double, double, 96)
}  // namespace tdg
