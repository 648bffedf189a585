// Host-side internals of the tdgemm C-ABI shared by its source files: the plan
// object and the steps of tdgemm_plan / tdgemm_gemm that other entry points reuse.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

struct tdgemm_plan_s {
  tdgemm_desc desc;
  tdg::Layout ly;
  char *ws;
  hipStream_t stream;
  bool tile_map;        // per-inner-kernel targets were given (copied to ws + off_target)
};

namespace tdg {

// Descriptor checks of every entry point (tdgemm.h: argument and shape errors).
tdgemm_status validate_desc(const tdgemm_desc *d);

// Workspace layout of a valid descriptor.
Layout layout_of(const tdgemm_desc &d);

bool is_block_scaled(int prec);

// Checks of tdgemm_plan's inputs other than the workspace: A and B present when
// there is work, a calibration table where the control mode reads one.
tdgemm_status check_plan_inputs(const tdgemm_desc &d, const void *A, const void *B,
                                const tdgemm_calib *calib);

// Enqueue the statistics and plan kernels of p (desc, ly, ws and stream set) on
// p.stream. tile_target: the caller's host map of per-inner-kernel targets, or
// nullptr; when given it is copied next to the plan and the stream synchronised.
hipError_t enqueue_plan(const tdgemm_plan_s &p, const void *A, const void *B,
                        const tdgemm_calib *calib, const double *tile_target);

// Enqueue the fused product of the plan: C = A B (zeros when K = 0). Packed
// forms only (prec F64 or F32).
hipError_t enqueue_fused(const tdgemm_plan_s &p, const void *A, const void *B, void *C);

}  // namespace tdg
