// Dispatch of the fused kernel over input type, packing type and L. The kernel
// itself is in fused.h; each combination is compiled in its own fused_*.hip.
#include "fused.h"

namespace tdg {

TDG_FUSED_EXTERN(double, double, 64)
TDG_FUSED_EXTERN(double, double, 96)
TDG_FUSED_EXTERN(double, double, 128)
TDG_FUSED_EXTERN(float, double, 64)
TDG_FUSED_EXTERN(float, double, 96)
TDG_FUSED_EXTERN(float, double, 128)
TDG_FUSED_EXTERN(float, float, 64)
TDG_FUSED_EXTERN(float, float, 96)
TDG_FUSED_EXTERN(float, float, 128)

template <typename IT, typename PT>
static hipError_t launch_fused_l(const GemmOperands &g, const void *A, const void *B, void *C,
                                 void *part, hipStream_t st) {
  if (g.pb.L == 64) return launch_fused_il<IT, PT, 64>(g, A, B, C, part, st);
  if (g.pb.L == 96) return launch_fused_il<IT, PT, 96>(g, A, B, C, part, st);
  return launch_fused_il<IT, PT, 128>(g, A, B, C, part, st);
}

hipError_t launch_fused(const GemmOperands &g, const void *A, const void *B, void *C, void *part,
                        hipStream_t st) {
  if (g.in_dtype == TDGEMM_F64 && g.prec == TDGEMM_F64) return launch_fused_l<double, double>(g, A, B, C, part, st);
  if (g.in_dtype == TDGEMM_F32 && g.prec == TDGEMM_F64) return launch_fused_l<float, double>(g, A, B, C, part, st);
  return launch_fused_l<float, float>(g, A, B, C, part, st);
}

}  // namespace tdg
