// Analytic runtime model of a stem plan and the step features of the
// learned model (host only).
//
// Paper §A.1: a pairwise contraction of tensors A and B costs 2^|E_AB|
// multiply-adds (here M K N complex ones, 8 real flops each) and the stem
// is read and written once per step; a group of g slices repeats every step
// g times in one launch.  Each launch is bounded by the larger of its HBM
// time and its matrix-core time (a roofline), plus a fixed launch cost.

#include <algorithm>
#include <cmath>

#include "stem_internal.h"

namespace {

stem_hw default_hw() {
  stem_hw hw;
  hw.hbm_bytes_per_s = 8.0e12;
  hw.fp32_flops_per_s = 157.3e12;
  hw.fp16_flops_per_s = 2.5e15;
  hw.launch_s = 4.0e-6;
  return hw;
}

// Seconds of one product launch over g slices.
double product_seconds(const stem_step_info& s, int precision, double g, const stem_hw& hw) {
  const double bytes = g * s.bytes;
  const double flops = g * s.flops;
  const double rate = precision == STEM_FP32 ? hw.fp32_flops_per_s : hw.fp16_flops_per_s / 3.0;
  return std::max(bytes / hw.hbm_bytes_per_s, flops / rate) + hw.launch_s;
}

}  // namespace

extern "C" {

stem_status stem_cost_analytic(const stem_step_info* steps, int32_t n_steps, int32_t precision,
                               uint32_t slices_in_flight, uint64_t n_slices, const stem_hw* hw_in,
                               double* seconds) {
  if ((!steps && n_steps) || !seconds || n_steps < 0) {
    stem::set_error("null argument");
    return STEM_EINVAL;
  }
  if (slices_in_flight < 1) {
    stem::set_error("slices_in_flight must be positive");
    return STEM_ERANGE;
  }
  const stem_hw hw = hw_in ? *hw_in : default_hw();
  const double g = (double)std::min<uint64_t>(slices_in_flight, std::max<uint64_t>(n_slices, 1));
  const double groups = std::ceil((double)std::max<uint64_t>(n_slices, 1) / g);
  double per_group = hw.launch_s;  // the FP64 accumulation
  for (int32_t i = 0; i < n_steps; ++i) {
    per_group += product_seconds(steps[i], precision, g, hw);
    if (steps[i].permuted) per_group += g * steps[i].perm_bytes / hw.hbm_bytes_per_s + hw.launch_s;
  }
  *seconds = groups * per_group;
  return STEM_OK;
}

stem_status stem_step_features(const stem_step_info* s, int32_t precision,
                               uint32_t slices_in_flight, float* f) {
  if (!s || !f) {
    stem::set_error("null argument");
    return STEM_EINVAL;
  }
  const double g = std::max<uint32_t>(slices_in_flight, 1);
  const stem_hw hw = default_hw();
  f[0] = (float)std::log2((double)s->M);
  f[1] = (float)std::log2((double)s->K);
  f[2] = (float)std::log2((double)s->N);
  f[3] = (float)std::log2(g);
  f[4] = (float)s->amode;
  f[5] = (float)s->cmode;
  f[6] = precision == STEM_FP32 ? 1.f : 0.f;
  f[7] = precision == STEM_SPLIT_FP16 ? 1.f : 0.f;
  f[8] = precision == STEM_SPLIT_BF16 ? 1.f : 0.f;
  f[9] = (float)std::log2(g * s->bytes);
  f[10] = (float)std::log2(g * s->flops);
  f[11] = (float)std::log2(product_seconds(*s, precision, g, hw));
  return STEM_OK;
}

}  // extern "C"
