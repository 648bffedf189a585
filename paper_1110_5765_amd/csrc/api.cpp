// C-ABI of the tdgemm library: argument validation on the host, workspace
// layout, plan lifecycle and launches. Declarations and contracts: tdgemm.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "api_internal.h"

namespace {

using tdg::Layout;
using tdg::Problem;
using tdg::layout_of;

bool is_finite(double x) { return std::isfinite(x); }

constexpr int64_t kMaxTileBytes = int64_t(1) << 30;  // L * lda and L * ldb, in bytes, must stay below

bool valid_l(int L) { return L == 64 || L == 96 || L == 128; }

// Packings a block size supports: W divides L (eq. 1): {1, 2, 4} at L = 64 and
// 128, {1, 2, 3, 4} at L = 96. E_ARG for a W outside {1, ..., 4} or one that
// does not divide L.
tdgemm_status check_w(int w, int L) {
  if (w < 1 || w > 4 || L % w != 0) return TDGEMM_E_ARG;
  return TDGEMM_OK;
}

bool block_scaled(int prec) { return prec == TDGEMM_I8 || prec == TDGEMM_E4M3; }

}  // namespace

namespace tdg {

bool is_block_scaled(int prec) { return block_scaled(prec); }

tdgemm_status validate_desc(const tdgemm_desc *d) {
  if (!d) return TDGEMM_E_ARG;
  if (d->M < 0 || d->N < 0 || d->K < 0) return TDGEMM_E_ARG;
  if (d->trans_a != 0 && d->trans_a != 1) return TDGEMM_E_ARG;
  if (d->trans_b != 0 && d->trans_b != 1) return TDGEMM_E_ARG;
  if (d->in_dtype != TDGEMM_F64 && d->in_dtype != TDGEMM_F32) return TDGEMM_E_ARG;
  if (d->prec != TDGEMM_F64 && d->prec != TDGEMM_F32 && !block_scaled(d->prec)) return TDGEMM_E_ARG;
  if (d->prec == TDGEMM_F32 && d->in_dtype == TDGEMM_F64) return TDGEMM_E_UNSUPPORTED;
  if (d->k_split < 0) return TDGEMM_E_ARG;
  if (block_scaled(d->prec)) {                                   // INT8 / FP8 form
    if (d->k_split > 1) return TDGEMM_E_UNSUPPORTED;
    if (d->ctrl != TDGEMM_CTRL_SEPARABLE || d->fixed_w != 1) return TDGEMM_E_ARG;
    if (!(d->sep_q >= 1.0) || !(d->sep_q <= (d->prec == TDGEMM_I8 ? 127.0 : 448.0)))
      return TDGEMM_E_ARG;
    if (d->L != 128) return valid_l(d->L) ? TDGEMM_E_UNSUPPORTED : TDGEMM_E_ARG;
  }
  if (!valid_l(d->L)) return (d->L > 0) ? TDGEMM_E_UNSUPPORTED : TDGEMM_E_ARG;
  if (d->form != TDGEMM_SYM && d->form != TDGEMM_ASYM) return TDGEMM_E_ARG;
  const int64_t need_a = d->trans_a ? d->M : d->K;
  const int64_t need_b = d->trans_b ? d->K : d->N;
  if (d->lda < (need_a > 0 ? need_a : 1) || d->ldb < (need_b > 0 ? need_b : 1) ||
      d->ldc < (d->N > 0 ? d->N : 1))
    return TDGEMM_E_ARG;
  // the fused kernel reads L rows (or columns) of an operand as one buffer
  // resource, by 32-bit byte offsets below L * ld * element size
  const int64_t esz = d->in_dtype == TDGEMM_F64 ? 8 : 4;
  if ((int64_t)d->L * d->lda * esz >= kMaxTileBytes || (int64_t)d->L * d->ldb * esz >= kMaxTileBytes)
    return TDGEMM_E_UNSUPPORTED;
  if (!(d->u_safe > 0.0) || !is_finite(d->u_safe)) return TDGEMM_E_ARG;
  switch (d->ctrl) {
    case TDGEMM_CTRL_ACCEL:
      if (!(d->accel >= 0.0 && d->accel <= 1.0)) return TDGEMM_E_ARG;
      if (d->accel_units[0] != 0 || d->accel_units[1] != 0) return TDGEMM_E_ARG;
      for (int w = 2; w <= 4; ++w)
        if (d->accel_units[w] < 0 || d->accel_units[w] > (1 << 20)) return TDGEMM_E_ARG;
      [[fallthrough]];
    case TDGEMM_CTRL_SNR: {
      if (d->ctrl == TDGEMM_CTRL_SNR && std::isnan(d->snr_db)) return TDGEMM_E_ARG;
      if (!(d->w_allowed & 2u)) return TDGEMM_E_ARG;
      if (d->w_allowed & ~(2u | 4u | 8u | 16u)) return TDGEMM_E_ARG;
      for (int w = 2; w <= 4; ++w) {
        if (!(d->w_allowed & (1u << w))) continue;
        const tdgemm_status sw = check_w(w, d->L);
        if (sw != TDGEMM_OK) return sw;
      }
      break;
    }
    case TDGEMM_CTRL_FIXED: {
      const tdgemm_status sw = check_w(d->fixed_w, d->L);
      if (sw != TDGEMM_OK) return sw;
      if (!(d->fixed_rmax > 0.0) || !is_finite(d->fixed_rmax)) return TDGEMM_E_ARG;
      break;
    }
    case TDGEMM_CTRL_TARGET: {
      const tdgemm_status sw = check_w(d->fixed_w, d->L);
      if (sw != TDGEMM_OK) return sw;
      if (!(d->fixed_rmax > 0.0) || !is_finite(d->fixed_rmax)) return TDGEMM_E_ARG;
      if (std::isnan(d->snr_db) || d->snr_db == -INFINITY) return TDGEMM_E_ARG;
      break;
    }
    case TDGEMM_CTRL_SEPARABLE: {
      const tdgemm_status sw = check_w(d->fixed_w, d->L);
      if (sw != TDGEMM_OK) return sw;
      if (!(d->sep_q >= 1.0) || !is_finite(d->sep_q)) return TDGEMM_E_ARG;
      break;
    }
    default:
      return TDGEMM_E_ARG;
  }
  if (d->tile_target) {                                          // per-inner-kernel targets
    if (d->ctrl != TDGEMM_CTRL_SNR && d->ctrl != TDGEMM_CTRL_ACCEL && d->ctrl != TDGEMM_CTRL_TARGET)
      return TDGEMM_E_ARG;
    const int64_t nt = ((d->M + d->L - 1) / d->L) * ((d->N + d->L - 1) / d->L);
    for (int64_t t = 0; t < nt; ++t) {
      const double v = d->tile_target[t];
      const bool ok = d->ctrl == TDGEMM_CTRL_ACCEL ? (v >= 0.0 && v <= 1.0)
                    : d->ctrl == TDGEMM_CTRL_SNR   ? !std::isnan(v)
                                                   : !std::isnan(v) && v != -INFINITY;
      if (!ok) return TDGEMM_E_ARG;
    }
  }
  const int64_t nL = (d->K + d->L - 1) / d->L;
  if (nL > 512) return TDGEMM_E_UNSUPPORTED;                     // plan kernel keeps 512 per wave
  return TDGEMM_OK;
}

Layout layout_of(const tdgemm_desc &d) {
  const size_t elem = d.prec == TDGEMM_F32 ? sizeof(float) : sizeof(double);
  return tdg::make_layout(d.M, d.N, d.K, d.L, d.k_split, elem);
}

}  // namespace tdg

namespace {

tdgemm_status validate(const tdgemm_desc *d) { return tdg::validate_desc(d); }

Problem problem_of(const tdgemm_desc &d, const Layout &ly) {
  Problem p;
  p.M = d.M; p.N = d.N; p.K = d.K;
  p.lda = d.lda; p.ldb = d.ldb; p.ldc = d.ldc;
  p.nI = ly.nI; p.nL = ly.nL; p.nJ = ly.nJ;
  p.L = d.L;
  return p;
}

tdg::GemmOperands operands_of(const tdgemm_plan_s *p) {
  tdg::GemmOperands g;
  g.pb = problem_of(p->desc, p->ly);
  g.in_dtype = p->desc.in_dtype;
  g.prec = p->desc.prec;
  g.form = p->desc.form;
  g.ta = p->desc.trans_a != 0;
  g.tb = p->desc.trans_b != 0;
  g.pairs = reinterpret_cast<const tdgemm_pair *>(p->ws + p->ly.off_pairs);
  g.gsize = p->ly.gsize;
  return g;
}

tdg::Gemm8Args gemm8_args(const tdgemm_plan_s *p) {
  tdg::Gemm8Args q;
  q.qA = nullptr; q.qB = nullptr; q.in = nullptr; q.out = nullptr;
  q.Kp = p->ly.nL * p->desc.L;
  q.nI = p->ly.nI; q.nL = p->ly.nL; q.nJ = p->ly.nJ;
  q.M = p->desc.M; q.N = p->desc.N; q.ldc = p->desc.ldc;
  q.pairs = reinterpret_cast<const tdgemm_pair *>(p->ws + p->ly.off_pairs);
  return q;
}

tdgemm_status hip_status(hipError_t e) { return e == hipSuccess ? TDGEMM_OK : TDGEMM_E_HIP; }

bool empty_output(const tdgemm_desc &d) { return d.M == 0 || d.N == 0; }

int packing_exponent_host(double r_safe, double u_safe) {
  int e;
  double m = std::frexp(2.0 * r_safe + u_safe, &e);
  return (m == 0.5) ? e - 1 : e;
}

}  // namespace

namespace tdg {

tdgemm_status check_plan_inputs(const tdgemm_desc &d, const void *A, const void *B,
                                const tdgemm_calib *calib) {
  if (!empty_output(d) && d.K > 0 && (!A || !B)) return TDGEMM_E_ARG;
  const bool tables = d.ctrl == TDGEMM_CTRL_SNR || d.ctrl == TDGEMM_CTRL_ACCEL ||
                      d.ctrl == TDGEMM_CTRL_TARGET;
  if (tables && (!calib || calib->n_r < 1 || calib->n_r > 512 || !calib->r || !calib->s))
    return TDGEMM_E_CALIB;
  return TDGEMM_OK;
}

hipError_t enqueue_plan(const tdgemm_plan_s &p, const void *A, const void *B,
                        const tdgemm_calib *calib, const double *tile_target) {
  const tdgemm_desc &d = p.desc;
  const Layout &ly = p.ly;
  if (empty_output(d) || d.K == 0) return hipSuccess;      // no pairs
  const bool with_options = d.ctrl == TDGEMM_CTRL_SNR || d.ctrl == TDGEMM_CTRL_ACCEL;
  auto *sa = reinterpret_cast<tdgemm_block_stats *>(p.ws + ly.off_stats_a);
  auto *sb = reinterpret_cast<tdgemm_block_stats *>(p.ws + ly.off_stats_b);
  auto *tab = reinterpret_cast<PlanTable *>(p.ws + ly.off_table);
  StatsArgs sargs;
  sargs.A = A; sargs.B = B;
  sargs.M = d.M; sargs.N = d.N; sargs.K = d.K;
  sargs.lda = d.lda; sargs.ldb = d.ldb;
  sargs.ta = d.trans_a != 0; sargs.tb = d.trans_b != 0;
  sargs.nI = ly.nI; sargs.nL = ly.nL; sargs.nJ = ly.nJ;
  sargs.stats_a = sa; sargs.stats_b = sb;
  sargs.calib_r = with_options ? calib->r : nullptr;
  sargs.calib_s = with_options ? calib->s : nullptr;
  sargs.n_r = with_options ? calib->n_r : 0;
  sargs.table = with_options ? tab : nullptr;
  hipError_t e = launch_stats(sargs, d.in_dtype, d.L, p.stream);
  if (e != hipSuccess) return e;
  PlanLaunch pl;
  pl.pb = problem_of(d, ly);
  pl.stats_a = sa;
  pl.stats_b = sb;
  pl.pairs = reinterpret_cast<tdgemm_pair *>(p.ws + ly.off_pairs);
  pl.budget = reinterpret_cast<double *>(p.ws + ly.off_budget);
  pl.calib_r = calib ? calib->r : nullptr;
  pl.calib_s = calib ? calib->s : nullptr;
  pl.table = tab;
  pl.n_r = calib ? calib->n_r : 0;
  pl.ctrl = d.ctrl;
  pl.n_opt = 0;
  for (int w : {4, 3, 2, 1})
    if (!with_options || (d.w_allowed & (1u << w))) pl.w_desc[pl.n_opt++] = w;
  if (!with_options) { pl.n_opt = 1; pl.w_desc[0] = d.fixed_w; }
  pl.accel = d.accel;
  // saved work per pair and packing: measured units when given, else twelfths of
  // the W = 1 MFMA work
  const bool measured = d.accel_units[2] || d.accel_units[3] || d.accel_units[4];
  for (int w = 0; w < 5; ++w)
    pl.units[w] = w < 2 ? 0 : (measured ? d.accel_units[w] : 12 - 12 / w);
  pl.fixed_w = d.fixed_w;
  pl.block_scaled = block_scaled(d.prec) ? 1 : 0;
  pl.fixed_rmax = d.fixed_rmax;
  pl.sep_q = d.sep_q;
  pl.u_safe = d.u_safe;
  pl.snr_lin = std::pow(10.0, -d.snr_db / 10.0);
  pl.tgt_pow = std::pow(10.0, 0.1 * d.snr_db);
  pl.tile = nullptr;
  if (tile_target) {
    // per inner kernel: 10^(-S/10) (SNR), 10^(S/10) (TARGET) or F_kernel (ACCEL),
    // copied next to the plan
    const int64_t nt = ly.nI * ly.nJ;
    std::vector<double> h(nt);
    for (int64_t t = 0; t < nt; ++t)
      h[t] = d.ctrl == TDGEMM_CTRL_SNR    ? std::pow(10.0, -tile_target[t] / 10.0)
           : d.ctrl == TDGEMM_CTRL_TARGET ? std::pow(10.0, 0.1 * tile_target[t])
                                          : tile_target[t];
    double *dt = reinterpret_cast<double *>(p.ws + ly.off_target);
    e = hipMemcpyAsync(dt, h.data(), sizeof(double) * nt, hipMemcpyHostToDevice, p.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p.stream);   // h is released below
    if (e != hipSuccess) return e;
    pl.tile = dt;
  }
  return launch_plan(pl, p.stream);
}

hipError_t enqueue_fused(const tdgemm_plan_s &p, const void *A, const void *B, void *C) {
  const tdgemm_desc &d = p.desc;
  if (empty_output(d)) return hipSuccess;
  if (d.K == 0) return launch_fill_zero(C, d.prec, d.M, d.N, d.ldc, p.stream);
  return launch_fused(operands_of(&p), A, B, C, p.ws + p.ly.off_part, p.stream);
}

}  // namespace tdg

extern "C" {

const char *tdgemm_status_string(tdgemm_status s) {
  switch (s) {
    case TDGEMM_OK: return "TDGEMM_OK";
    case TDGEMM_E_ARG: return "TDGEMM_E_ARG: invalid argument or shape";
    case TDGEMM_E_UNSUPPORTED: return "TDGEMM_E_UNSUPPORTED: valid but not implemented";
    case TDGEMM_E_WORKSPACE: return "TDGEMM_E_WORKSPACE: workspace missing or too small";
    case TDGEMM_E_CALIB: return "TDGEMM_E_CALIB: calibration table missing or malformed";
    case TDGEMM_E_HIP: return "TDGEMM_E_HIP: HIP runtime error";
  }
  return "unknown tdgemm status";
}

size_t tdgemm_workspace_size(const tdgemm_desc *desc) {
  if (validate(desc) != TDGEMM_OK) return 0;
  return layout_of(*desc).total;
}

tdgemm_status tdgemm_plan(const tdgemm_desc *desc, const void *A, const void *B,
                          const tdgemm_calib *calib, void *ws, size_t ws_bytes, void *stream,
                          tdgemm_plan_t *out) {
  if (!out) return TDGEMM_E_ARG;
  *out = nullptr;
  tdgemm_status s = validate(desc);
  if (s != TDGEMM_OK) return s;
  const Layout ly = layout_of(*desc);
  if (!empty_output(*desc) && desc->K > 0 && (!A || !B)) return TDGEMM_E_ARG;
  if (!ws || ws_bytes < ly.total) return TDGEMM_E_WORKSPACE;
  s = tdg::check_plan_inputs(*desc, A, B, calib);
  if (s != TDGEMM_OK) return s;
  tdgemm_plan_s *p = new (std::nothrow) tdgemm_plan_s;
  if (!p) return TDGEMM_E_ARG;
  p->desc = *desc;
  p->tile_map = desc->tile_target != nullptr;
  p->desc.tile_target = nullptr;          // read here only; not kept
  p->ly = ly;
  p->ws = static_cast<char *>(ws);
  p->stream = static_cast<hipStream_t>(stream);
  if (tdg::enqueue_plan(*p, A, B, calib, desc->tile_target) != hipSuccess) {
    delete p;
    return TDGEMM_E_HIP;
  }
  *out = p;
  return TDGEMM_OK;
}

tdgemm_status tdgemm_plan_dims(tdgemm_plan_t plan, int64_t *nI, int64_t *nL, int64_t *nJ,
                               int64_t *n_pairs) {
  if (!plan) return TDGEMM_E_ARG;
  if (nI) *nI = plan->ly.nI;
  if (nL) *nL = plan->ly.nL;
  if (nJ) *nJ = plan->ly.nJ;
  if (n_pairs) *n_pairs = plan->ly.n_pairs;
  return TDGEMM_OK;
}

tdgemm_status tdgemm_plan_destroy(tdgemm_plan_t plan) {
  if (!plan) return TDGEMM_E_ARG;
  delete plan;
  return TDGEMM_OK;
}

tdgemm_status tdgemm_plan_export(tdgemm_plan_t plan, tdgemm_block_stats *stats_a,
                                 tdgemm_block_stats *stats_b, tdgemm_pair *pairs,
                                 double *budgets) {
  if (!plan) return TDGEMM_E_ARG;
  if (hipStreamSynchronize(plan->stream) != hipSuccess) return TDGEMM_E_HIP;
  const Layout &ly = plan->ly;
  const bool has_work = !empty_output(plan->desc) && plan->desc.K > 0;
  if (!has_work) return TDGEMM_OK;
  struct Item { void *dst; size_t off, bytes; } items[] = {
      {stats_a, ly.off_stats_a, sizeof(tdgemm_block_stats) * ly.nI * ly.nL},
      {stats_b, ly.off_stats_b, sizeof(tdgemm_block_stats) * ly.nL * ly.nJ},
      {pairs, ly.off_pairs, sizeof(tdgemm_pair) * ly.n_pairs},
      {budgets, ly.off_budget, sizeof(double) * ly.nI * ly.nJ}};
  for (const Item &it : items) {
    if (!it.dst) continue;
    if (hipMemcpy(it.dst, plan->ws + it.off, it.bytes, hipMemcpyDeviceToHost) != hipSuccess)
      return TDGEMM_E_HIP;
  }
  return TDGEMM_OK;
}

tdgemm_status tdgemm_plan_query(tdgemm_plan_t plan, double *pred_snr_db, int64_t *w_hist,
                                int64_t *n_short) {
  if (!plan) return TDGEMM_E_ARG;
  if (hipStreamSynchronize(plan->stream) != hipSuccess) return TDGEMM_E_HIP;
  if (pred_snr_db) *pred_snr_db = INFINITY;
  if (w_hist)
    for (int w = 0; w < 5; ++w) w_hist[w] = 0;
  if (n_short) *n_short = 0;
  const Layout &ly = plan->ly;
  const tdgemm_desc &d = plan->desc;
  if (empty_output(d) || d.K == 0 || ly.n_pairs == 0) return TDGEMM_OK;
  std::vector<tdgemm_block_stats> sa(ly.nI * ly.nL), sb(ly.nL * ly.nJ);
  std::vector<tdgemm_pair> pr(ly.n_pairs);
  const bool target = d.ctrl == TDGEMM_CTRL_TARGET;
  std::vector<double> tgt(target && plan->tile_map ? ly.nI * ly.nJ : 0);
  struct Item { void *dst; size_t off, bytes; } items[] = {
      {sa.data(), ly.off_stats_a, sizeof(tdgemm_block_stats) * sa.size()},
      {sb.data(), ly.off_stats_b, sizeof(tdgemm_block_stats) * sb.size()},
      {pr.data(), ly.off_pairs, sizeof(tdgemm_pair) * pr.size()},
      {tgt.data(), ly.off_target, sizeof(double) * tgt.size()}};
  for (const Item &it : items) {
    if (it.bytes == 0) continue;
    if (hipMemcpy(it.dst, plan->ws + it.off, it.bytes, hipMemcpyDeviceToHost) != hipSuccess)
      return TDGEMM_E_HIP;
  }
  const double tgt_all = std::pow(10.0, 0.1 * d.snr_db);
  double signal = 0.0, noise = 0.0;
  int64_t short_pairs = 0;
  for (int64_t i = 0; i < ly.nI; ++i)
    for (int64_t j = 0; j < ly.nJ; ++j)
      for (int64_t l = 0; l < ly.nL; ++l) {
        const tdgemm_block_stats &a = sa[i * ly.nL + l], &b = sb[l * ly.nJ + j];
        const tdgemm_pair &o = pr[(i * ly.nJ + j) * ly.nL + l];
        const double va = a.n > 0 ? a.sumsq / (double)a.n : 0.0;
        const double vb = b.n > 0 ? b.sumsq / (double)b.n : 0.0;
        const double l_eff = (double)std::min<int64_t>(d.L, d.K - l * d.L);
        const double sig = (l_eff * va) * vb;        // expected signal power of the pair
        signal += sig;
        noise += o.d;
        if (w_hist && o.w >= 1 && o.w <= 4) ++w_hist[o.w];
        if (target && o.w > 1 && o.d > 0.0) {
          const double want = plan->tile_map ? tgt[i * ly.nJ + j] : tgt_all;
          if (sig < want * o.d * (1.0 - 1e-9)) ++short_pairs;
        }
      }
  if (pred_snr_db && noise > 0.0) *pred_snr_db = 10.0 * std::log10(signal / noise);
  if (n_short) *n_short = short_pairs;
  return TDGEMM_OK;
}

tdgemm_status tdgemm_compand(tdgemm_plan_t plan, const void *A, const void *B, void *qA, void *qB,
                             void *stream) {
  if (!plan) return TDGEMM_E_ARG;
  if (plan->ly.n_pairs == 0 || empty_output(plan->desc)) return TDGEMM_OK;
  if (!A || !B || !qA || !qB) return TDGEMM_E_ARG;
  const tdgemm_desc &d = plan->desc;
  if (block_scaled(d.prec)) {
    const Layout &ly = plan->ly;
    tdg::Quant8Args q;
    q.A = A; q.B = B;
    q.M = d.M; q.N = d.N; q.K = d.K; q.lda = d.lda; q.ldb = d.ldb;
    q.ta = d.trans_a; q.tb = d.trans_b;
    q.nI = ly.nI; q.nL = ly.nL; q.nJ = ly.nJ;
    q.Kp = ly.nL * d.L;
    q.stats_a = reinterpret_cast<const tdgemm_block_stats *>(plan->ws + ly.off_stats_a);
    q.stats_b = reinterpret_cast<const tdgemm_block_stats *>(plan->ws + ly.off_stats_b);
    q.q = d.sep_q;
    q.qA = static_cast<uint8_t *>(qA);
    q.qB = static_cast<uint8_t *>(qB);
    return hip_status(tdg::launch_quant8(q, d.in_dtype, d.prec, (hipStream_t)stream));
  }
  return hip_status(tdg::launch_compand(operands_of(plan), A, B, qA, qB, (hipStream_t)stream));
}

tdgemm_status tdgemm_pack(tdgemm_plan_t plan, const void *qA, const void *qB, void *pA, void *pB,
                          void *stream) {
  if (!plan) return TDGEMM_E_ARG;
  if (plan->ly.n_pairs == 0 || empty_output(plan->desc)) return TDGEMM_OK;
  if (block_scaled(plan->desc.prec)) return TDGEMM_E_UNSUPPORTED;   // nothing is packed
  if (!qA || !qB || !pA || !pB) return TDGEMM_E_ARG;
  return hip_status(tdg::launch_pack(operands_of(plan), qA, qB, pA, pB, (hipStream_t)stream));
}

tdgemm_status tdgemm_gemm(tdgemm_plan_t plan, const void *a, const void *b, void *out, int fused,
                          void *stream) {
  if (!plan) return TDGEMM_E_ARG;
  if (fused != 0 && fused != 1) return TDGEMM_E_ARG;
  const tdgemm_desc &d = plan->desc;
  if (empty_output(d)) return TDGEMM_OK;
  if (!out) return TDGEMM_E_ARG;
  tdg::GemmOperands g = operands_of(plan);
  if (d.K == 0) {
    if (!fused) return TDGEMM_OK;     // no pairs: nothing to multiply
    return hip_status(tdg::launch_fill_zero(out, d.prec, d.M, d.N, d.ldc, (hipStream_t)stream));
  }
  if (!a || !b) return TDGEMM_E_ARG;
  if (block_scaled(d.prec)) {
    tdg::Gemm8Args q = gemm8_args(plan);
    q.qA = static_cast<const uint8_t *>(a);
    q.qB = static_cast<const uint8_t *>(b);
    q.out = out;
    return hip_status(tdg::launch_gemm8(q, d.prec, !fused, (hipStream_t)stream));
  }
  if (fused)
    return hip_status(tdg::launch_fused(g, a, b, out, plan->ws + plan->ly.off_part, (hipStream_t)stream));
  return hip_status(tdg::launch_packed_product(g, a, b, out, (hipStream_t)stream));
}

tdgemm_status tdgemm_unpack(tdgemm_plan_t plan, const void *Rbar, void *r_int, void *C,
                            void *stream) {
  if (!plan) return TDGEMM_E_ARG;
  const tdgemm_desc &d = plan->desc;
  if (empty_output(d)) return TDGEMM_OK;
  if (!C && !r_int) return TDGEMM_E_ARG;
  if (d.K == 0)
    return C ? hip_status(tdg::launch_fill_zero(C, d.prec, d.M, d.N, d.ldc, (hipStream_t)stream))
             : TDGEMM_OK;
  if (!Rbar) return TDGEMM_E_ARG;
  if (block_scaled(d.prec)) {
    if (r_int || !C) return TDGEMM_E_ARG;        // the staged products are already integers
    tdg::Gemm8Args q = gemm8_args(plan);
    q.in = Rbar;
    q.out = C;
    return hip_status(tdg::launch_scale_sum8(q, d.prec, (hipStream_t)stream));
  }
  return hip_status(tdg::launch_unpack(operands_of(plan), Rbar, r_int, C, (hipStream_t)stream));
}

size_t tdgemm_calibrate_workspace_size(int32_t L, int32_t n_inst) {
  if (!valid_l(L) || n_inst < 1) return 0;
  const size_t slot = tdg::align256(sizeof(double) * (size_t)n_inst * L * L);
  // qA qB pA pB Rbar r_int refA refB refR, records x2, moments
  return 9 * slot + 2 * tdg::align256(sizeof(tdgemm_pair) * (size_t)n_inst) + 256;
}

tdgemm_status tdgemm_calibrate(int32_t L, int32_t W, int32_t form, int32_t prec, const double *q,
                               int32_t n_q, const double *u_a, const double *u_b, int32_t n_inst,
                               double u_safe, double *r_out, double *m_out, double *s_out, void *ws,
                               size_t ws_bytes, void *stream) {
  if (!valid_l(L)) return L > 0 ? TDGEMM_E_UNSUPPORTED : TDGEMM_E_ARG;
  if (W < 2) return TDGEMM_E_ARG;
  const tdgemm_status sw = check_w(W, L);
  if (sw != TDGEMM_OK) return sw;
  if (form != TDGEMM_SYM && form != TDGEMM_ASYM) return TDGEMM_E_ARG;
  if (prec != TDGEMM_F64 && prec != TDGEMM_F32) return TDGEMM_E_ARG;
  if (!q || n_q < 1 || !u_a || !u_b || n_inst < 1 || !r_out || !m_out || !s_out) return TDGEMM_E_ARG;
  if (!(u_safe > 0.0) || !is_finite(u_safe)) return TDGEMM_E_ARG;
  for (int t = 0; t < n_q; ++t)
    if (!(q[t] >= 1.0) || !is_finite(q[t]) || q[t] != std::floor(q[t])) return TDGEMM_E_ARG;
  const size_t need = tdgemm_calibrate_workspace_size(L, n_inst);
  if (!ws || ws_bytes < need) return TDGEMM_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char *w = static_cast<char *>(ws);
  const size_t slot = tdg::align256(sizeof(double) * (size_t)n_inst * L * L);
  void *qA = w, *qB = w + slot, *pA = w + 2 * slot, *pB = w + 3 * slot, *Rb = w + 4 * slot,
       *rint_ = w + 5 * slot;
  double *refA = reinterpret_cast<double *>(w + 6 * slot);
  double *refB = reinterpret_cast<double *>(w + 7 * slot);
  double *refR = reinterpret_cast<double *>(w + 8 * slot);
  const size_t rec = tdg::align256(sizeof(tdgemm_pair) * (size_t)n_inst);
  auto *pairs_w = reinterpret_cast<tdgemm_pair *>(w + 9 * slot);
  auto *pairs_1 = reinterpret_cast<tdgemm_pair *>(w + 9 * slot + rec);
  double *mom = reinterpret_cast<double *>(w + 9 * slot + 2 * rec);
  const int64_t n = (int64_t)n_inst * L * L;

  tdg::GemmOperands g;
  g.pb.M = g.pb.N = g.pb.K = L;
  g.pb.lda = g.pb.ldb = g.pb.ldc = L;
  g.pb.nI = n_inst; g.pb.nJ = 1; g.pb.nL = 1;
  g.gsize = 1;
  g.pb.L = L;
  g.in_dtype = prec; g.prec = prec; g.form = form; g.ta = g.tb = false;
  g.pairs = pairs_w;
  tdg::GemmOperands gref = g;
  gref.in_dtype = TDGEMM_F64; gref.prec = TDGEMM_F64; gref.form = TDGEMM_SYM;
  gref.pairs = pairs_1;

  std::vector<tdgemm_pair> hp(n_inst), h1(n_inst);
  tdgemm_pair one;
  std::memset(&one, 0, sizeof(one));
  one.c_a = one.c_b = one.inv = 1.0;
  one.w = 1;
  for (auto &x : h1) x = one;
  if (hipStreamSynchronize(st) != hipSuccess) return TDGEMM_E_HIP;
  if (hipMemcpy(pairs_1, h1.data(), sizeof(tdgemm_pair) * n_inst, hipMemcpyHostToDevice) != hipSuccess)
    return TDGEMM_E_HIP;
  for (int t = 0; t < n_q; ++t) {
    const double qq = q[t];
    const double r_max = ((double)L * qq) * qq;
    tdgemm_pair o = one;
    o.w = W;
    o.p = packing_exponent_host(r_max, u_safe);
    o.r_max = r_max;
    for (auto &x : hp) x = o;
    hipError_t e = hipMemcpy(pairs_w, hp.data(), sizeof(tdgemm_pair) * n_inst, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = tdg::launch_int_inputs(u_a, n, qq, prec, qA, st);
    if (e == hipSuccess) e = tdg::launch_int_inputs(u_b, n, qq, prec, qB, st);
    if (e == hipSuccess) e = tdg::launch_pack(g, qA, qB, pA, pB, st);
    if (e == hipSuccess) e = tdg::launch_packed_product(g, pA, pB, Rb, st);
    if (e == hipSuccess) e = tdg::launch_unpack(g, Rb, rint_, nullptr, st);
    if (e == hipSuccess) e = tdg::launch_int_inputs(u_a, n, qq, TDGEMM_F64, refA, st);
    if (e == hipSuccess) e = tdg::launch_int_inputs(u_b, n, qq, TDGEMM_F64, refB, st);
    if (e == hipSuccess) e = tdg::launch_packed_product(gref, refA, refB, refR, st);
    if (e == hipSuccess) e = tdg::launch_error_moments(rint_, refR, prec, n, mom, st);
    double hm[3];
    if (e == hipSuccess) e = hipMemcpyAsync(hm, mom, sizeof(hm), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return TDGEMM_E_HIP;
    r_out[t] = r_max;
    if (hm[2] > 0.0) {
      m_out[t] = NAN;
      s_out[t] = INFINITY;
    } else {
      m_out[t] = hm[0] / (double)n;
      s_out[t] = std::sqrt(hm[1] / (double)n);
    }
  }
  return TDGEMM_OK;
}

}  // extern "C"
