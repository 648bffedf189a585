// Fused kernel instantiation: double inputs, double packing, L = 128.
#include "fused.h"

namespace tdg {
TDG_FUSED_INSTANCE(double, double, 128)
}  // namespace tdg
