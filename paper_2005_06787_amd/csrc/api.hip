// C-ABI of libstemgpu: plan creation, the slice loop of the sliced stem
// contraction, and utilities.  Paper §A.1 (slicing), §A.2 (stem and
// branches), §A.3 (branches computed once and shared by every slice).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "device_common.h"
#include "kernels.h"
#include "stem_internal.h"

namespace stem {

static thread_local std::string g_error;

void set_error(const std::string& msg) { g_error = msg; }

}  // namespace stem

using namespace stem;

struct StepDev {
  size_t boff = 0;          // offset of variant 0 in the plan's branch buffer (bytes)
  size_t bstride = 0;       // bytes per variant block (header + fragments)
};

struct stem_plan_s {
  PlanLayout L;
  int precision = STEM_FP32;
  int device = 0;
  float* d_stem = nullptr;          // initial stem, fixed labels most significant
  uint64_t stem_var_elems = 0;      // complex entries per stem variant
  unsigned char* d_branch = nullptr;
  std::vector<StepDev> sd;
  std::vector<hipEvent_t> ev;       // 4 per step when timing: perm start/end, gemm start/end
  std::vector<float> gemm_us, perm_us;
  std::vector<float> tuned_us;      // per step, from stem_tune
  std::vector<int> tuned_nz;
  int timed_slices = 0;
  bool timed_pending = false;
};

#define HIPCHK(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));               \
      return STEM_EHIP;                                                           \
    }                                                                             \
  } while (0)

static stem_status fail(stem_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

// An operand without per-slice variants: batch item z at ptr + z * zstride.
static Operand plain_operand(const void* ptr, int64_t zstride) {
  Operand o;
  std::memset(&o, 0, sizeof(o));
  o.ptr = ptr;
  o.zstride = zstride;
  return o;
}

// The product operands of a step with h batch labels: launch item z is
// slice z >> h, batch index z & (2^h - 1), whose bits sit at the address
// positions pos (stem and output; none for the branch, whose variant
// selects them).
static Operand batched(Operand o, int h, const int32_t* pos) {
  o.hbits = h;
  o.nhpos = pos ? h : 0;
  for (int q = 0; q < h && pos; ++q) o.hpos[q] = (int8_t)pos[q];
  return o;
}

static void out_batch_pos(const StepLayout& S, int32_t* pos) {
  const int h = (int)S.batch.size();
  for (int q = 0; q < h; ++q) pos[q] = S.rank_out - h + q;
}

// Variant selection of a tensor's fixed labels (MSB first) for one
// projected assignment pa: projected bits go into vbase, sliced ones are
// read from the slice id on the device.
static SliceSel make_sel(const std::vector<FixedSrc>& src, uint64_t pa, int n_sliced, int n_proj) {
  SliceSel s;
  std::memset(&s, 0, sizeof(s));
  const int nf = (int)src.size();
  int h = 0;  // the step's batch labels: batch index bit h-1-index
  for (const FixedSrc& f : src) h += f.is_proj == 2 ? 1 : 0;
  for (int j = 0; j < nf; ++j) {
    const int vpos = nf - 1 - j;
    if (src[j].is_proj == 2) {
      s.hshift[s.nh] = (int8_t)(h - 1 - src[j].index);
      s.hvpos[s.nh] = (int8_t)vpos;
      s.nh++;
    } else if (src[j].is_proj) {
      s.vbase |= (uint64_t)fixed_bit(src[j], 0, pa, n_sliced, n_proj) << vpos;
    } else {
      s.vshift[s.nv] = (int8_t)(n_sliced - 1 - src[j].index);
      s.vpos[s.nv] = (int8_t)vpos;
      s.nv++;
    }
  }
  return s;
}

static void free_plan(stem_plan_s* p) {
  if (!p) return;
  if (p->d_stem) (void)hipFree(p->d_stem);
  if (p->d_branch) (void)hipFree(p->d_branch);
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  delete p;
}

extern "C" {

const char* stem_status_str(stem_status s) {
  switch (s) {
    case STEM_OK: return "ok";
    case STEM_EINVAL: return "invalid argument";
    case STEM_ELABEL: return "label error";
    case STEM_ESHAPE: return "shape error";
    case STEM_EUNSUPPORTED: return "unsupported network";
    case STEM_ENOMEM: return "out of memory or workspace too small";
    case STEM_ERANGE: return "range error";
    case STEM_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* stem_last_error(void) { return g_error.c_str(); }

stem_status stem_plan_validate(const stem_plan_desc* desc, stem_plan_summary* summary) {
  try {
    PlanLayout L;
    std::string err;
    stem_status s = build_layout(desc, &L, &err);
    if (s != STEM_OK) return fail(s, err);
    if (summary) *summary = L.summary;
    return STEM_OK;
  } catch (const std::bad_alloc&) {
    return fail(STEM_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(STEM_EINVAL, "unexpected host exception");
  }
}

static stem_status plan_create_impl(const stem_plan_desc* d, hipStream_t st, stem_plan_s* p) {
  std::string err;
  stem_status s = build_layout(d, &p->L, &err);
  if (s != STEM_OK) return fail(s, err);
  PlanLayout& L = p->L;
  p->precision = d->precision;
  HIPCHK(hipGetDevice(&p->device));

  // ---- initial stem: fixed labels moved to the most significant bits ----
  const int r0 = d->stem_rank;
  const uint64_t n0 = 1ull << r0;
  HIPCHK(hipMalloc(&p->d_stem, n0 * 8));
  p->stem_var_elems = 1ull << L.stem_rest.size();
  std::vector<int32_t> stem_order = L.stem_fixed;
  stem_order.insert(stem_order.end(), L.stem_rest.begin(), L.stem_rest.end());
  const bool stem_perm = !same_order(L.stem_labels_in, stem_order);
  if (!stem_perm) {
    HIPCHK(hipMemcpyAsync(p->d_stem, d->stem_data, n0 * 8,
                          d->stem_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          st));
  } else {
    const float* src = d->stem_data;
    float* tmp = nullptr;
    if (!d->stem_on_device) {
      HIPCHK(hipMalloc(&tmp, n0 * 8));
      HIPCHK(hipMemcpyAsync(tmp, d->stem_data, n0 * 8, hipMemcpyHostToDevice, st));
      src = tmp;
    }
    const PermArgs pa = make_perm(L.stem_labels_in, stem_order);
    hipError_t e = launch_permute(plain_operand(src, 0), plain_operand(p->d_stem, 0), pa, 0, 1, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return fail(STEM_EHIP, std::string("stem relayout: ") + hipGetErrorString(e));
  }

  // ---- branches: host relayout to (fixed, sigma, free), then MFMA layout ----
  size_t total = 0;
  p->sd.resize(L.steps.size());
  std::vector<size_t> data_off(d->n_branches + 1, 0);
  for (int i = 0; i < d->n_branches; ++i)
    data_off[i + 1] = data_off[i] + (size_t(1) << d->branch_ranks[i]) * 2;
  std::vector<size_t> label_off(d->n_branches + 1, 0);
  for (int i = 0; i < d->n_branches; ++i) label_off[i + 1] = label_off[i] + d->branch_ranks[i];
  for (size_t i = 0; i < L.steps.size(); ++i) {
    const StepLayout& S = L.steps[i];
    const uint64_t nvar = 1ull << S.fixed.size();
    const size_t per = branch_block_bytes(p->precision, S.K, S.N);
    p->sd[i].boff = total;
    p->sd[i].bstride = per;
    total += per * nvar;
  }
  std::vector<unsigned char> hb(std::max<size_t>(total, 256), 0);
  for (size_t i = 0; i < L.steps.size(); ++i) {
    const StepLayout& S = L.steps[i];
    const int bi = S.branch_index;
    const int r = d->branch_ranks[bi];
    std::vector<int32_t> from(d->branch_labels + label_off[bi], d->branch_labels + label_off[bi + 1]);
    std::vector<int32_t> to = S.fixed;
    to.insert(to.end(), S.sigma.begin(), S.sigma.end());
    to.insert(to.end(), S.free_labels.begin(), S.free_labels.end());
    std::vector<float> re((size_t(1) << r) * 2);
    host_relayout(d->branch_data + data_off[bi], re.data(), from, to);
    const uint64_t nvar = 1ull << S.fixed.size();
    const size_t sub = (size_t)(S.K * S.N) * 2;  // floats per variant
    for (uint64_t v = 0; v < nvar; ++v) {
      unsigned char* blk = hb.data() + p->sd[i].boff + v * p->sd[i].bstride;
      unsigned char* dst = blk + kBranchHeader;
      float inv_b = 1.f;
      if (p->precision == STEM_FP32) {
        build_bfrag_f32(re.data() + v * sub, S.K, S.N, (float*)dst);
        if (bfrag_gauss_floats(S.K, S.N))
          build_bfrag_gauss(re.data() + v * sub, S.K, S.N,
                            (float*)dst + bfrag_f32_floats(S.K, S.N));
      } else {
        const int eb = build_bfrag_split(re.data() + v * sub, S.K, S.N,
                                         p->precision == STEM_SPLIT_BF16, (uint16_t*)dst);
        inv_b = std::ldexp(1.f, -eb);
      }
      std::memcpy(blk, &inv_b, sizeof(inv_b));
    }
  }
  HIPCHK(hipMalloc(&p->d_branch, hb.size()));
  HIPCHK(hipMemcpyAsync(p->d_branch, hb.data(), hb.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  p->gemm_us.assign(L.steps.size(), -1.f);
  p->perm_us.assign(L.steps.size(), -1.f);
  p->tuned_us.assign(L.steps.size(), -1.f);
  p->tuned_nz.assign(L.steps.size(), 0);
  return STEM_OK;
}

stem_status stem_plan_create(const stem_plan_desc* desc, void* stream, stem_plan_t* plan) {
  if (!plan) return fail(STEM_EINVAL, "null plan output");
  *plan = nullptr;
  stem_plan_s* p = nullptr;
  try {
    p = new stem_plan_s();
    stem_status s = plan_create_impl(desc, (hipStream_t)stream, p);
    if (s != STEM_OK) {
      free_plan(p);
      return s;
    }
  } catch (const std::bad_alloc&) {
    free_plan(p);
    return fail(STEM_ENOMEM, "host allocation failed");
  } catch (...) {
    free_plan(p);
    return fail(STEM_EINVAL, "unexpected host exception");
  }
  *plan = p;
  return STEM_OK;
}

stem_status stem_plan_destroy(stem_plan_t plan) {
  free_plan(plan);
  return STEM_OK;
}

stem_status stem_plan_summary_get(stem_plan_t plan, stem_plan_summary* summary) {
  if (!plan || !summary) return fail(STEM_EINVAL, "null argument");
  *summary = plan->L.summary;
  return STEM_OK;
}

static uint64_t slice_ws_bytes(const stem_plan_s* p) {
  if (p->L.steps.empty()) return 0;
  return 2 * (((8ull << p->L.max_ws_rank) + 255) & ~255ull);
}

stem_status stem_plan_workspace_bytes(stem_plan_t plan, uint32_t slices_in_flight,
                                      uint64_t* bytes) {
  if (!plan || !bytes) return fail(STEM_EINVAL, "null argument");
  if (slices_in_flight < 1 || slices_in_flight > (uint32_t)kMaxSlicesInFlight)
    return fail(STEM_ERANGE, "slices_in_flight outside [1, 4096]");
  *bytes = std::max<uint64_t>(slice_ws_bytes(plan) * slices_in_flight, 256);
  return STEM_OK;
}

}  // extern "C"

// Shape, cost and layout fields of a step (timing fields -1).
static void fill_info(const StepLayout& S, stem_step_info* info) {
  std::memset(info, 0, sizeof(*info));
  info->rank_in = S.rank_in;
  info->rank_out = S.rank_out;
  info->n_shared = S.s;
  info->n_free = S.f;
  info->permuted = S.permuted ? 1 : 0;
  info->M = S.M;
  info->K = S.K;
  info->N = S.N;
  const double M = (double)S.M, K = (double)S.K, N = (double)S.N;
  const double H = (double)(1 << S.batch.size());
  info->n_batch = (int32_t)S.batch.size();
  info->flops = 8.0 * H * M * K * N;
  info->bytes = 8.0 * H * (M * K + M * N + K * N);
  info->perm_bytes = S.permuted ? 16.0 * (double)(1ull << S.rank_in) : 0.0;
  info->last_gemm_us = -1.f;
  info->last_perm_us = -1.f;
  info->amode = S.gemm.amode;
  info->cmode = S.gemm.cmode;
  info->sched_tm = S.sched.tm;
  info->sched_ntw = S.sched.ntw;
  info->sched_blocks = S.sched.blocks;
  info->sched_lds = S.sched.lds;
  info->sched_algo = S.sched.algo;
  info->tuned_us = -1.f;
}

extern "C" {

stem_status stem_plan_steps(const stem_plan_desc* desc, stem_step_info* steps, int32_t capacity,
                            int32_t* n_steps) {
  if (!n_steps || capacity < 0 || (capacity && !steps)) return fail(STEM_EINVAL, "null argument");
  try {
    PlanLayout L;
    std::string err;
    stem_status s = build_layout(desc, &L, &err);
    if (s != STEM_OK) return fail(s, err);
    *n_steps = (int32_t)L.steps.size();
    for (int32_t i = 0; i < std::min(capacity, *n_steps); ++i) fill_info(L.steps[i], &steps[i]);
    return STEM_OK;
  } catch (const std::bad_alloc&) {
    return fail(STEM_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(STEM_EINVAL, "unexpected host exception");
  }
}

stem_status stem_step_info_get(stem_plan_t plan, int32_t step, stem_step_info* info) {
  if (!plan || !info) return fail(STEM_EINVAL, "null argument");
  if (step < 0 || step >= (int32_t)plan->L.steps.size())
    return fail(STEM_ERANGE, "step index out of range");
  const StepLayout& S = plan->L.steps[step];
  fill_info(S, info);
  if (plan->timed_pending) {
    // resolve the events of the last timed call (the caller synchronised)
    for (size_t i = 0; i < plan->L.steps.size(); ++i) {
      float ms = -1.f;
      if (hipEventElapsedTime(&ms, plan->ev[4 * i + 2], plan->ev[4 * i + 3]) == hipSuccess)
        plan->gemm_us[i] = ms * 1000.f;
      if (plan->L.steps[i].permuted &&
          hipEventElapsedTime(&ms, plan->ev[4 * i], plan->ev[4 * i + 1]) == hipSuccess)
        plan->perm_us[i] = ms * 1000.f;
    }
    plan->timed_pending = false;
  }
  info->last_slices = plan->timed_slices;
  info->last_gemm_us = plan->gemm_us[step];
  info->last_perm_us = plan->perm_us[step];
  info->tuned_us = plan->tuned_us[step];
  info->tuned_slices = plan->tuned_nz[step];
  return STEM_OK;
}

}  // extern "C"

// ---- autotuner -------------------------------------------------------------

namespace {

struct TuneKey {
  int prec, amode, cmode, lm, lk, ln, nz;
  bool operator<(const TuneKey& o) const {
    return std::tie(prec, amode, cmode, lm, lk, ln, nz) <
           std::tie(o.prec, o.amode, o.cmode, o.lm, o.lk, o.ln, o.nz);
  }
};

struct TuneBest {
  GemmSched sched;
  float us = 1e30f;
};

int ilog2(int64_t v) {
  int r = 0;
  while ((1ll << r) < v) ++r;
  return r;
}

void load_cache(const char* path, std::map<TuneKey, TuneBest>* best) {
  if (!path) return;
  std::ifstream f(path);
  std::string tag;
  while (f >> tag) {
    TuneKey k;
    GemmSched s;
    float us;
    const bool v2 = tag == "stem-tune-v2";
    if ((tag != "stem-tune-v1" && !v2) ||
        !(f >> k.prec >> k.amode >> k.cmode >> k.lm >> k.lk >> k.ln >> k.nz >> s.tm >> s.ntw >>
          s.blocks >> s.lds) ||
        (v2 && !(f >> s.algo)) || !(f >> us)) {
      if (!f.eof()) f.clear();
      std::string rest;
      std::getline(f, rest);
      continue;
    }
    TuneBest& b = (*best)[k];
    if (us < b.us) {
      b.us = us;
      b.sched = s;
    }
  }
}

// Candidate schedules of one step (distinct after the kernel's own clamping).
std::vector<GemmSched> candidates(const StepLayout& S, int precision) {
  const int nr = (int)(2 * S.N);
  const int nt = std::max(16, nr) / 16;
  int nt2 = 1;
  while (nt2 < nt) nt2 <<= 1;
  std::vector<int> ntws;
  for (int w : {8, 4, 2, 1})
    if (w <= nt2 && (w == std::min(8, nt2) || w * 2 == std::min(8, nt2))) ntws.push_back(w);
  const int kq = precision == STEM_FP32 ? 16 : 32;
  const int kc = std::max<int>(kq, (int)(2 * S.K)) / kq;
  std::vector<GemmSched> out;
  // the 3M FP32 product where its whole-tile shape holds
  if (precision == STEM_FP32 && S.gemm.cmode == 1 && S.K % 8 == 0 && S.N % 16 == 0 &&
      S.M % 64 == 0) {
    const int ntc_all = (int)(S.N / 16);
    const int top = std::min(4, ntc_all);
    for (int tm : {1, 2, 4}) {
      if (S.M % (64 * tm) != 0) continue;
      for (int w : {top, top / 2, top / 4}) {
        if (w < 1 || tm * w > 4) continue;
        for (int blocks : {1024, 4096, 16384}) {
          // -1: LDS (up to 64 KB) with prefetch, else global with prefetch;
          // 0: global with prefetch; 1: LDS up to the device limit, no
          // prefetch; 2: as 1 with 8-wave workgroups, 3: LDS with prefetch
          // and 8-wave workgroups (2 and 3 above 64 KB)
          const size_t lds = (size_t)kc * w * 1536;
          for (int l : {-1, 0, 1, 2, 3}) {
            if (l == 0 && lds > (size_t)kLdsBudget) continue;
            if (l >= 1 && lds > lds_limit()) continue;
            if (l >= 2 && (lds <= (size_t)kLdsBudget || S.M % (128 * tm) != 0)) continue;
            GemmSched s;
            s.tm = tm;
            s.ntw = w;
            s.blocks = blocks;
            s.lds = l;
            s.algo = 1;
            out.push_back(s);
          }
        }
      }
    }
  }
  for (int tm : {1, 2, 4})
    for (int w : ntws)
      for (int blocks : {1024, 4096, 16384}) {
        const size_t lds = precision == STEM_FP32 ? (size_t)kc * w * 1024 : (size_t)kc * w * 2048;
        for (int l : {-1, 0, 1, 2}) {
          if (l == 0 && lds > (size_t)kLdsBudget) continue;  // -1 is already global
          if (l >= 1 && (lds <= (size_t)kLdsBudget || lds > lds_limit())) continue;
          // 2: split products with 8-wave workgroups sharing the LDS copy
          if (l == 2 && (precision == STEM_FP32 || S.gemm.cmode != 1 || S.M % (128 * tm) != 0))
            continue;
          GemmSched s;
          s.tm = tm;
          s.ntw = w;
          s.blocks = blocks;
          s.lds = l;
          out.push_back(s);
        }
      }
  return out;
}

}  // namespace

extern "C" {

stem_status stem_step_sched_set(stem_plan_t p, int32_t step, int32_t tm, int32_t ntw,
                                int32_t blocks, int32_t lds, int32_t algo) {
  if (!p) return fail(STEM_EINVAL, "null plan");
  if (step < 0 || step >= (int32_t)p->L.steps.size()) return fail(STEM_ERANGE, "step index");
  if ((tm != 1 && tm != 2 && tm != 4) || (ntw != 1 && ntw != 2 && ntw != 4 && ntw != 8) ||
      blocks < 256 || blocks > 65536 || lds < -1 || lds > 3 || algo < 0 || algo > 1 ||
      (algo == 1 && ntw > 4) || (algo == 0 && lds >= 2 && p->precision == STEM_FP32) ||
      (algo == 0 && lds == 3))
    return fail(STEM_ERANGE, "schedule value outside its set");
  StepLayout& S = p->L.steps[step];
  if (algo == 1 && (p->precision != STEM_FP32 || S.gemm.cmode != 1 || S.K % 8 != 0 ||
                    S.N % 16 != 0 || S.M % 64 != 0))
    return fail(STEM_EUNSUPPORTED, "the 3M product needs FP32 and whole tiles");
  GemmSched s;
  s.tm = tm;
  s.ntw = ntw;
  s.blocks = blocks;
  s.lds = lds;
  s.algo = algo;
  const GemmGeom g = make_geom(S.gemm, S.M, S.K, S.N, p->precision == STEM_FP32 ? 16 : 32);
  S.sched = resolve_sched(g, s);
  return STEM_OK;
}

stem_status stem_tune(stem_plan_t p, uint32_t nz, void* ws, uint64_t ws_bytes, int32_t reps,
                      const char* cache_path, void* stream) {
  if (!p) return fail(STEM_EINVAL, "null plan");
  hipStream_t st = (hipStream_t)stream;
  const PlanLayout& L = p->L;
  if (L.steps.empty()) return STEM_OK;
  if (nz < 1 || nz > (uint32_t)kMaxSlicesInFlight) return fail(STEM_ERANGE, "slices_in_flight");
  for (const StepLayout& S : L.steps)
    if (((uint64_t)nz << S.batch.size()) > 65535u)
      return fail(STEM_ERANGE, "slices_in_flight x 2^(batch labels of a step) above 65535");
  const uint64_t per = slice_ws_bytes(p);
  if (!ws || ws_bytes < per * nz)
    return fail(STEM_ENOMEM, "workspace smaller than stem_plan_workspace_bytes(plan, slices)");
  const bool force = reps < 0;
  const int nrep = std::max(1, reps < 0 ? -reps : reps);
  std::map<TuneKey, TuneBest> best;
  load_cache(cache_path, &best);
  std::ofstream log;
  if (cache_path) log.open(cache_path, std::ios::app);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int64_t half = (int64_t)(per / 2);
  const Operand in = plain_operand(ws, half);
  const Operand out = plain_operand((unsigned char*)ws + half * (int64_t)nz, half);
  stem_status rs = STEM_OK;
  for (size_t i = 0; i < L.steps.size() && rs == STEM_OK; ++i) {
    StepLayout& S = p->L.steps[i];
    const int h = (int)S.batch.size();
    const int nzh = (int)(nz << h);
    const TuneKey key{p->precision, S.gemm.amode, S.gemm.cmode, ilog2(S.M), ilog2(S.K),
                      ilog2(S.N), nzh};
    auto it = best.find(key);
    if (!force && it != best.end()) {
      S.sched = it->second.sched;
      p->tuned_us[i] = it->second.us;
      p->tuned_nz[i] = (int)nz;
      continue;
    }
    int32_t cpos[kMaxBatchLabels];
    out_batch_pos(S, cpos);
    const Operand bop = batched(plain_operand(p->d_branch + p->sd[i].boff, 0), h, nullptr);
    // successive launches swap the two stem buffers, so that every launch
    // reads what the one before it wrote, as the steps of a contraction do
    // (values are irrelevant to the timing)
    // the first step reads the initial stem, which can be larger than the
    // workspace buffers (they hold the tensors the steps write); its timing
    // launches read the stem's first variant, as slice 0 does
    const bool from_stem = i == 0 && !S.permuted;
    const Operand stem0 = plain_operand(p->d_stem, 0);
    if (!from_stem && (8ull << S.rank_in) > (uint64_t)half) {
      rs = fail(STEM_EINVAL, "tuning: step input larger than its workspace buffer");
      break;
    }
    const Operand a_in[2] = {batched(from_stem ? stem0 : in, h, S.hpos_a),
                             batched(from_stem ? stem0 : out, h, S.hpos_a)};
    const Operand c_out[2] = {batched(out, h, cpos), batched(in, h, cpos)};
    TuneBest win;
    for (const GemmSched& c : candidates(S, p->precision)) {
      hipError_t e = launch_cgemm(p->precision, a_in[0], bop, c_out[0], 0, nzh, S.M, S.K, S.N,
                                  S.gemm, c, st);
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      for (int r = 0; r < nrep && e == hipSuccess; ++r)
        e = launch_cgemm(p->precision, a_in[(r + 1) & 1], bop, c_out[(r + 1) & 1], 0, nzh, S.M,
                         S.K, S.N, S.gemm, c, st);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        rs = fail(STEM_EHIP, std::string("tuning launch: ") + hipGetErrorString(e));
        break;
      }
      const float us = ms * 1000.f / (float)nrep;
      if (log.is_open())
        log << "stem-tune-v2 " << key.prec << ' ' << key.amode << ' ' << key.cmode << ' '
            << key.lm << ' ' << key.lk << ' ' << key.ln << ' ' << key.nz << ' ' << c.tm << ' '
            << c.ntw << ' ' << c.blocks << ' ' << c.lds << ' ' << c.algo << ' ' << us << '\n';
      if (us < win.us) {
        win.us = us;
        win.sched = c;
      }
    }
    if (rs != STEM_OK) break;
    if (it == best.end() || win.us < it->second.us) best[key] = win;
    S.sched = best[key].sched;
    p->tuned_us[i] = best[key].us;
    p->tuned_nz[i] = (int)nz;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rs;
}

}  // extern "C"

// The slice loop of stem_contract; also recorded into graphs by stem_batch_create.
// The steps of a plan for slices [c0, c0 + nz) of one projected assignment
// (stem_op and bsel carry its variant selections): the final stems end in
// *cur (the initial stem itself when the plan has no steps), in workspace
// buffer *cur_buf (0 = X, 1 = Y, -1 = none).
static stem_status run_chain(stem_plan_t p, const Operand& stem_op,
                             const std::vector<SliceSel>& bsel, uint64_t c0, int nz,
                             unsigned char* wsb, int64_t half, int64_t ybase, bool time_this,
                             hipStream_t st, Operand* cur_out, int* buf_out) {
  const PlanLayout& L = p->L;
  Operand cur = stem_op;
  int cur_buf = -1;
  for (size_t i = 0; i < L.steps.size(); ++i) {
    const StepLayout& S = L.steps[i];
    if (S.permuted) {
      const int dst = cur_buf == 0 ? 1 : 0;
      const Operand o = plain_operand(wsb + (dst ? ybase : 0), half);
      if (time_this) HIPCHK(hipEventRecord(p->ev[4 * i], st));
      hipError_t e = launch_permute(cur, o, S.perm, c0, nz, st);
      if (e != hipSuccess) return fail(STEM_EHIP, std::string("permute: ") + hipGetErrorString(e));
      if (time_this) HIPCHK(hipEventRecord(p->ev[4 * i + 1], st));
      cur = o;
      cur_buf = dst;
    }
    const int dst = cur_buf == 0 ? 1 : 0;
    const Operand o = plain_operand(wsb + (dst ? ybase : 0), half);
    Operand bop = plain_operand(p->d_branch + p->sd[i].boff, 0);
    bop.vstride = (int64_t)p->sd[i].bstride;
    bop.sel = bsel[i];
    const int h = (int)S.batch.size();
    int32_t cpos[kMaxBatchLabels];
    out_batch_pos(S, cpos);
    if (time_this) HIPCHK(hipEventRecord(p->ev[4 * i + 2], st));
    hipError_t e = launch_cgemm(p->precision, batched(cur, h, S.hpos_a), batched(bop, h, nullptr),
                                batched(o, h, cpos), c0, nz << h, S.M, S.K, S.N, S.gemm,
                                S.sched, st);
    if (e != hipSuccess) return fail(STEM_EHIP, std::string("product: ") + hipGetErrorString(e));
    if (time_this) HIPCHK(hipEventRecord(p->ev[4 * i + 3], st));
    cur = o;
    cur_buf = dst;
  }
  *cur_out = cur;
  *buf_out = cur_buf;
  return STEM_OK;
}

static stem_status contract_impl(stem_plan_t p, uint64_t s0, uint64_t s1,
                                 const uint64_t* proj_assign, uint32_t n_batch, void* ws,
                                 uint64_t ws_bytes, double* out, uint32_t flags, hipStream_t st) {
  if (!p || !out) return fail(STEM_EINVAL, "null plan or output");
  const PlanLayout& L = p->L;
  const int n_sl = (int)L.sliced.size(), n_pr = (int)L.proj.size();
  const uint64_t n_slices = 1ull << n_sl;
  if (s0 > s1 || s1 > n_slices) return fail(STEM_ERANGE, "slice range outside [0, 2^n_sliced)");
  if (n_batch == 0) return STEM_OK;
  if (proj_assign)
    for (uint32_t b = 0; b < n_batch; ++b)
      if (proj_assign[b] >= (1ull << n_pr))
        return fail(STEM_ERANGE, "projected assignment out of range");
  const uint64_t per = slice_ws_bytes(p);
  uint64_t group = kMaxSlicesInFlight;
  if (per) {
    if (!ws || ws_bytes < per)
      return fail(STEM_ENOMEM, "workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                                   std::to_string(per) + " per slice in flight");
    group = std::min<uint64_t>(ws_bytes / per, kMaxSlicesInFlight);
  }
  // a batched step launches 2^h items per slice; the grid's z extent is
  // at most 65535
  size_t hmax = 0;
  for (const StepLayout& S : L.steps) hmax = std::max(hmax, S.batch.size());
  group = std::min<uint64_t>(group, 65535u >> hmax);
  const uint64_t n_out = 1ull << L.open.size();
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev != p->device) return fail(STEM_EINVAL, "plan was created on another device");
  // without STEM_ACCUMULATE the first group of each batch entry overwrites
  // its output, so out is only zeroed for an empty range
  const bool fresh = !(flags & STEM_ACCUMULATE);
  if (fresh && s0 == s1) {
    hipError_t e = launch_zero_f64(out, 2 * n_out * n_batch, st);
    if (e != hipSuccess) return fail(STEM_EHIP, std::string("zero: ") + hipGetErrorString(e));
  }
  if (s0 == s1) return STEM_OK;
  const bool timing = (flags & STEM_TIME_STEPS) != 0;
  if (timing && p->ev.empty()) {
    p->ev.resize(4 * L.steps.size());
    for (auto& e : p->ev) HIPCHK(hipEventCreate(&e));
  }
  // the two stem buffers of every slice in flight: [X: group][Y: group]
  const int64_t half = (int64_t)(per / 2);
  const int64_t ybase = half * (int64_t)group;
  unsigned char* wsb = (unsigned char*)ws;
  std::vector<SliceSel> bsel(L.steps.size());
  for (uint32_t b = 0; b < n_batch; ++b) {
    const uint64_t pa = proj_assign ? proj_assign[b] : 0;
    Operand stem_op = plain_operand(p->d_stem, 0);
    stem_op.vstride = (int64_t)(8 * p->stem_var_elems);
    stem_op.sel = make_sel(L.stem_fixed_src, pa, n_sl, n_pr);
    for (size_t i = 0; i < L.steps.size(); ++i)
      bsel[i] = make_sel(L.steps[i].fixed_src, pa, n_sl, n_pr);
    for (uint64_t c0 = s0; c0 < s1; c0 += group) {
      const int nz = (int)std::min<uint64_t>(group, s1 - c0);
      const bool time_this = timing && b + 1 == n_batch && c0 + group >= s1;
      if (time_this) p->timed_slices = nz;
      Operand cur;
      int cur_buf = -1;
      stem_status rs = run_chain(p, stem_op, bsel, c0, nz, wsb, half, ybase, time_this, st, &cur,
                                 &cur_buf);
      if (rs != STEM_OK) return rs;
      // large results take the tiled sum (contiguous reads and writes)
      hipError_t e =
          L.final_labels.size() >= (size_t)kAccTileMaxBits
              ? launch_acc_tiled(cur, c0, nz, out + 2 * n_out * b, L.final_perm, st,
                                 fresh && c0 == s0)
              : launch_acc_f64(cur, c0, nz, out + 2 * n_out * b, L.final_map, st,
                               fresh && c0 == s0);
      if (e != hipSuccess) return fail(STEM_EHIP, std::string("accumulate: ") + hipGetErrorString(e));
    }
  }
  if (timing) p->timed_pending = true;
  return STEM_OK;
}

// ---------------------------------------------------------------------------
// Two-sided stems (paper §A.2): two plans over the same sliced and projected
// labels, each run slice by slice, then joined at the root by contracting
// their final tensors over the labels they share.
// ---------------------------------------------------------------------------
constexpr int kJoinMaxOpenLog = 12;   // the join kernel keeps 16 outputs per thread

struct stem_join_s {
  stem_plan_t left = nullptr, right = nullptr;
  std::vector<int32_t> open;
  std::vector<int32_t> left_order, right_order;  // [shared..., left-only...], [shared..., right-only...]
  bool perm_left = false, perm_right = false;
  PermArgs pl{}, pr{};
  int a_log = 0, b_log = 0, k_log = 0, chunk_log = 0;
  BitMap out_map{};
  int device = 0;
};

static uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// Bytes per slice in flight, in the order the workspace holds them: the
// two chains' stem buffers, the two re-ordered final tensors, the partial
// sums of the k chunks.
struct JoinParts {
  uint64_t chain_l, chain_r, tl, tr, part;
  uint64_t total() const { return chain_l + chain_r + tl + tr + part; }
};

static JoinParts join_parts(const stem_join_s* j) {
  JoinParts q;
  q.chain_l = slice_ws_bytes(j->left);
  q.chain_r = slice_ws_bytes(j->right);
  q.tl = j->perm_left ? align256(8ull << j->left->L.final_labels.size()) : 0;
  q.tr = j->perm_right ? align256(8ull << j->right->L.final_labels.size()) : 0;
  const uint64_t n_out = 1ull << (j->a_log + j->b_log);
  q.part = align256((16ull * n_out) << (j->k_log - j->chunk_log));
  return q;
}

static stem_status join_contract_impl(stem_join_s* j, uint64_t s0, uint64_t s1,
                                      const uint64_t* proj_assign, uint32_t n_batch, void* ws,
                                      uint64_t ws_bytes, double* out, uint32_t flags,
                                      hipStream_t st) {
  if (!j || !out) return fail(STEM_EINVAL, "null join or output");
  if (flags & STEM_TIME_STEPS) return fail(STEM_EINVAL, "STEM_TIME_STEPS is not allowed on a join");
  stem_plan_t pl = j->left, pr = j->right;
  const int n_sl = (int)pl->L.sliced.size(), n_pr = (int)pl->L.proj.size();
  if (s0 > s1 || s1 > (1ull << n_sl)) return fail(STEM_ERANGE, "slice range outside [0, 2^n_sliced)");
  if (n_batch == 0) return STEM_OK;
  if (proj_assign)
    for (uint32_t b = 0; b < n_batch; ++b)
      if (proj_assign[b] >= (1ull << n_pr))
        return fail(STEM_ERANGE, "projected assignment out of range");
  const JoinParts q = join_parts(j);
  const uint64_t per = q.total();
  if (!ws || ws_bytes < per)
    return fail(STEM_ENOMEM, "workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                                 std::to_string(per) + " per slice in flight");
  uint64_t group = std::min<uint64_t>(ws_bytes / per, kMaxSlicesInFlight);
  size_t hmax = 0;
  for (const StepLayout& S : pl->L.steps) hmax = std::max(hmax, S.batch.size());
  for (const StepLayout& S : pr->L.steps) hmax = std::max(hmax, S.batch.size());
  group = std::min<uint64_t>(group, 65535u >> hmax);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev != j->device) return fail(STEM_EINVAL, "join was created on another device");
  const int out_log = j->a_log + j->b_log;
  const uint64_t n_out = 1ull << out_log;
  if (!(flags & STEM_ACCUMULATE)) {
    hipError_t e = launch_zero_f64(out, 2 * n_out * n_batch, st);
    if (e != hipSuccess) return fail(STEM_EHIP, std::string("zero: ") + hipGetErrorString(e));
  }
  if (s0 == s1) return STEM_OK;
  unsigned char* base = (unsigned char*)ws;
  unsigned char* ws_l = base;
  unsigned char* ws_r = ws_l + q.chain_l * group;
  unsigned char* t_l = ws_r + q.chain_r * group;
  unsigned char* t_r = t_l + q.tl * group;
  double* part = (double*)(t_r + q.tr * group);
  const int nchunks = 1 << (j->k_log - j->chunk_log);
  std::vector<SliceSel> sel_l(pl->L.steps.size()), sel_r(pr->L.steps.size());
  for (uint32_t b = 0; b < n_batch; ++b) {
    const uint64_t pa = proj_assign ? proj_assign[b] : 0;
    Operand stem_l = plain_operand(pl->d_stem, 0);
    stem_l.vstride = (int64_t)(8 * pl->stem_var_elems);
    stem_l.sel = make_sel(pl->L.stem_fixed_src, pa, n_sl, n_pr);
    for (size_t i = 0; i < pl->L.steps.size(); ++i)
      sel_l[i] = make_sel(pl->L.steps[i].fixed_src, pa, n_sl, n_pr);
    Operand stem_r = plain_operand(pr->d_stem, 0);
    stem_r.vstride = (int64_t)(8 * pr->stem_var_elems);
    stem_r.sel = make_sel(pr->L.stem_fixed_src, pa, n_sl, n_pr);
    for (size_t i = 0; i < pr->L.steps.size(); ++i)
      sel_r[i] = make_sel(pr->L.steps[i].fixed_src, pa, n_sl, n_pr);
    for (uint64_t c0 = s0; c0 < s1; c0 += group) {
      const int nz = (int)std::min<uint64_t>(group, s1 - c0);
      Operand fl, fr;
      int buf = -1;
      stem_status rs = run_chain(pl, stem_l, sel_l, c0, nz, ws_l, (int64_t)(q.chain_l / 2),
                                 (int64_t)(q.chain_l / 2 * group), false, st, &fl, &buf);
      if (rs != STEM_OK) return rs;
      rs = run_chain(pr, stem_r, sel_r, c0, nz, ws_r, (int64_t)(q.chain_r / 2),
                     (int64_t)(q.chain_r / 2 * group), false, st, &fr, &buf);
      if (rs != STEM_OK) return rs;
      if (j->perm_left) {
        const Operand o = plain_operand(t_l, (int64_t)q.tl);
        hipError_t e = launch_permute(fl, o, j->pl, c0, nz, st);
        if (e != hipSuccess) return fail(STEM_EHIP, std::string("permute: ") + hipGetErrorString(e));
        fl = o;
      }
      if (j->perm_right) {
        const Operand o = plain_operand(t_r, (int64_t)q.tr);
        hipError_t e = launch_permute(fr, o, j->pr, c0, nz, st);
        if (e != hipSuccess) return fail(STEM_EHIP, std::string("permute: ") + hipGetErrorString(e));
        fr = o;
      }
      hipError_t e = launch_join_partial(fl, fr, c0, nz, j->a_log, j->b_log, j->k_log,
                                         j->chunk_log, part, st);
      if (e != hipSuccess) return fail(STEM_EHIP, std::string("join: ") + hipGetErrorString(e));
      e = launch_join_acc(part, nz, nchunks, out_log, out + 2 * n_out * b, j->out_map, st);
      if (e != hipSuccess) return fail(STEM_EHIP, std::string("join sum: ") + hipGetErrorString(e));
    }
  }
  return STEM_OK;
}

struct stem_batch_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> events;  // fork, then one join per plan
  int device = 0;
};

static void free_batch(stem_batch_s* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (hipStream_t s : b->side) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
  delete b;
}

// Record every plan's range on its own stream, forked from and joined to st.
static stem_status batch_record(stem_batch_s* b, int32_t n, const stem_plan_t* plans,
                                const uint64_t* s0, const uint64_t* s1, const uint64_t* proj,
                                double* const* out, unsigned char* ws, uint64_t part,
                                uint32_t flags, hipStream_t st) {
  HIPCHK(hipEventRecord(b->events[0], st));
  for (int32_t j = 0; j < n; ++j) {
    HIPCHK(hipStreamWaitEvent(b->side[j], b->events[0], 0));
    const uint64_t pa = proj ? proj[j] : 0;
    stem_status s = contract_impl(plans[j], s0[j], s1[j], &pa, 1, ws + part * j, part, out[j],
                                  flags, b->side[j]);
    if (s != STEM_OK) return s;
    HIPCHK(hipEventRecord(b->events[1 + j], b->side[j]));
    HIPCHK(hipStreamWaitEvent(st, b->events[1 + j], 0));
  }
  return STEM_OK;
}

extern "C" {

stem_status stem_contract(stem_plan_t p, uint64_t s0, uint64_t s1, const uint64_t* proj_assign,
                          uint32_t n_batch, void* ws, uint64_t ws_bytes, double* out,
                          uint32_t flags, void* stream) {
  return contract_impl(p, s0, s1, proj_assign, n_batch, ws, ws_bytes, out, flags,
                       (hipStream_t)stream);
}

stem_status stem_join_create(stem_plan_t left, stem_plan_t right, int32_t n_open,
                             const int32_t* open_labels, stem_join_t* join) {
  if (!join) return fail(STEM_EINVAL, "null join output");
  *join = nullptr;
  if (!left || !right) return fail(STEM_EINVAL, "null plan");
  if (n_open < 0 || (n_open && !open_labels)) return fail(STEM_EINVAL, "bad open label list");
  if (left->device != right->device) return fail(STEM_EINVAL, "plans on different devices");
  const PlanLayout &A = left->L, &B = right->L;
  if (A.sliced != B.sliced || A.proj != B.proj)
    return fail(STEM_ELABEL, "the two plans must list the same sliced and projected labels");
  std::set<int32_t> la(A.open.begin(), A.open.end()), lb(B.open.begin(), B.open.end());
  std::vector<int32_t> shared, only_a, only_b;
  for (int32_t x : A.final_labels) (lb.count(x) ? shared : only_a).push_back(x);
  for (int32_t x : B.final_labels)
    if (!la.count(x)) only_b.push_back(x);
  std::vector<int32_t> open(open_labels, open_labels + n_open);
  std::set<int32_t> want(open.begin(), open.end());
  std::set<int32_t> sym(only_a.begin(), only_a.end());
  sym.insert(only_b.begin(), only_b.end());
  if (want.size() != open.size() || want != sym)
    return fail(STEM_ELABEL, "the join's open labels must be the labels open in exactly one plan");
  if (n_open > kJoinMaxOpenLog)
    return fail(STEM_EUNSUPPORTED, "a join has at most 12 open labels");
  stem_join_s* j = nullptr;
  try {
    j = new stem_join_s();
  } catch (const std::bad_alloc&) {
    return fail(STEM_ENOMEM, "host allocation failed");
  }
  j->left = left;
  j->right = right;
  j->device = left->device;
  j->open = open;
  j->left_order = shared;
  j->left_order.insert(j->left_order.end(), only_a.begin(), only_a.end());
  j->right_order = shared;
  j->right_order.insert(j->right_order.end(), only_b.begin(), only_b.end());
  j->perm_left = !same_order(A.final_labels, j->left_order);
  j->perm_right = !same_order(B.final_labels, j->right_order);
  if (j->perm_left) j->pl = make_perm(A.final_labels, j->left_order);
  if (j->perm_right) j->pr = make_perm(B.final_labels, j->right_order);
  j->a_log = (int)only_a.size();
  j->b_log = (int)only_b.size();
  j->k_log = (int)shared.size();
  // at most 256 chunks of at least 256 k values (all of k when shorter)
  j->chunk_log = j->k_log <= 8 ? j->k_log : std::max(8, j->k_log - 8);
  // output index a 2^b_log + b -> position of each label in the join's order
  const int r = n_open;
  j->out_map.rank = r;
  auto pos_of = [&](int32_t x) {
    int k = 0;
    while (open[k] != x) ++k;
    return r - 1 - k;
  };
  for (int t = 0; t < j->b_log; ++t) j->out_map.dst[j->b_log - 1 - t] = pos_of(only_b[t]);
  for (int t = 0; t < j->a_log; ++t)
    j->out_map.dst[j->b_log + j->a_log - 1 - t] = pos_of(only_a[t]);
  *join = j;
  return STEM_OK;
}

stem_status stem_join_workspace_bytes(stem_join_t join, uint32_t slices_in_flight,
                                      uint64_t* bytes) {
  if (!join || !bytes) return fail(STEM_EINVAL, "null argument");
  if (slices_in_flight < 1 || slices_in_flight > (uint32_t)kMaxSlicesInFlight)
    return fail(STEM_ERANGE, "slices_in_flight outside [1, 4096]");
  *bytes = join_parts(join).total() * slices_in_flight;
  return STEM_OK;
}

stem_status stem_join_contract(stem_join_t join, uint64_t s0, uint64_t s1,
                               const uint64_t* proj_assign, uint32_t n_batch, void* ws,
                               uint64_t ws_bytes, double* out, uint32_t flags, void* stream) {
  return join_contract_impl(join, s0, s1, proj_assign, n_batch, ws, ws_bytes, out, flags,
                            (hipStream_t)stream);
}

stem_status stem_join_destroy(stem_join_t join) {
  delete join;
  return STEM_OK;
}

stem_status stem_batch_create(int32_t n, const stem_plan_t* plans, const uint64_t* s0,
                              const uint64_t* s1, const uint64_t* proj, double* const* out,
                              void* ws, uint64_t ws_bytes, uint32_t flags, void* stream,
                              stem_batch_t* batch) {
  if (!batch) return fail(STEM_EINVAL, "null batch output");
  *batch = nullptr;
  if (n < 1 || !plans || !s0 || !s1 || !out) return fail(STEM_EINVAL, "empty or null batch");
  if (flags & STEM_TIME_STEPS) return fail(STEM_EINVAL, "STEM_TIME_STEPS is not allowed in a batch");
  hipStream_t st = (hipStream_t)stream;
  const uint64_t part = (ws_bytes / (uint64_t)n) & ~255ull;
  for (int32_t j = 0; j < n; ++j) {
    if (!plans[j] || !out[j]) return fail(STEM_EINVAL, "null plan or output in batch");
    if (s0[j] > s1[j] || s1[j] > (1ull << plans[j]->L.sliced.size()))
      return fail(STEM_ERANGE, "slice range of plan " + std::to_string(j) + " out of range");
    const uint64_t per = slice_ws_bytes(plans[j]);
    if (per && (!ws || part < per))
      return fail(STEM_ENOMEM, "workspace part of " + std::to_string(part) + " bytes for plan " +
                                   std::to_string(j) + ", need " + std::to_string(per));
  }
  stem_batch_s* b = nullptr;
  try {
    b = new stem_batch_s();
  } catch (const std::bad_alloc&) {
    return fail(STEM_ENOMEM, "host allocation failed");
  }
  auto bail = [&](stem_status s) {
    free_batch(b);
    return s;
  };
  if (hipGetDevice(&b->device) != hipSuccess) return bail(fail(STEM_EHIP, "hipGetDevice failed"));
  // Recording happens on a private stream (the caller's may be the null
  // stream, which cannot be captured); side[n] is that stream.
  b->side.resize(n + 1, nullptr);
  b->events.resize(n + 1, nullptr);
  for (auto& s : b->side)
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(STEM_EHIP, "hipStreamCreateWithFlags failed"));
  for (auto& e : b->events)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
      return bail(fail(STEM_EHIP, "hipEventCreate failed"));
  (void)stream;
  st = b->side[n];
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return bail(fail(STEM_EHIP, std::string("begin capture: ") + hipGetErrorString(e)));
  stem_status rs = batch_record(b, n, plans, s0, s1, proj, out, (unsigned char*)ws, part, flags, st);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(st, &g);
  b->graph = g;
  if (rs != STEM_OK) return bail(rs);
  if (e != hipSuccess) return bail(fail(STEM_EHIP, std::string("end capture: ") + hipGetErrorString(e)));
  e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return bail(fail(STEM_EHIP, std::string("instantiate: ") + hipGetErrorString(e)));
  *batch = b;
  return STEM_OK;
}

stem_status stem_batch_launch(stem_batch_t batch, void* stream) {
  if (!batch) return fail(STEM_EINVAL, "null batch");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev != batch->device) return fail(STEM_EINVAL, "batch was created on another device");
  HIPCHK(hipGraphLaunch(batch->exec, (hipStream_t)stream));
  return STEM_OK;
}

stem_status stem_batch_destroy(stem_batch_t batch) {
  free_batch(batch);
  return STEM_OK;
}

stem_status stem_fill_counter(float* dst, uint64_t n, uint64_t seed, int32_t scale_log2,
                              void* stream) {
  if (!dst && n) return fail(STEM_EINVAL, "null destination");
  hipError_t e = launch_fill_counter(dst, n, seed, scale_log2, (hipStream_t)stream);
  if (e != hipSuccess) return fail(STEM_EHIP, std::string("fill: ") + hipGetErrorString(e));
  return STEM_OK;
}

stem_status stem_xeb_f64(const double* amps, uint64_t n, int32_t n_qubits, double* out,
                         void* stream) {
  if ((!amps && n) || !out) return fail(STEM_EINVAL, "null argument");
  if (n_qubits < 0 || n_qubits > 1000) return fail(STEM_EINVAL, "bad qubit count");
  hipError_t e = launch_xeb_f64(amps, n, n_qubits, out, (hipStream_t)stream);
  if (e != hipSuccess) return fail(STEM_EHIP, std::string("xeb: ") + hipGetErrorString(e));
  return STEM_OK;
}

}  // extern "C"
