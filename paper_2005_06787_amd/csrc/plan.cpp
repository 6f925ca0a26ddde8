// Host planner of libstemgpu: validation of a sliced stem network and the
// label order of the stem before and after every step.  Pure C++; it needs
// no GPU, so stem_plan_validate works on any host.
//
// Paper §A.1: each step is a pairwise contraction of the stem with one
// branch over the labels they share; the result keeps the other labels.
// Fixing the sliced labels (slicing) and the projected labels (a batch of
// amplitudes, §3) removes them from every tensor before the steps run.

#include <algorithm>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "stem_internal.h"

namespace stem {

namespace {

bool has_dup(const std::vector<int32_t>& v) {
  std::set<int32_t> s(v.begin(), v.end());
  return s.size() != v.size();
}

std::string join(const std::vector<int32_t>& v) {
  std::string out = "[";
  for (size_t i = 0; i < v.size(); ++i) {
    if (i) out += ",";
    out += std::to_string(v[i]);
  }
  return out + "]";
}

}  // namespace

bool same_order(const std::vector<int32_t>& from, const std::vector<int32_t>& to) {
  return from == to;
}

PermArgs make_perm(const std::vector<int32_t>& from, const std::vector<int32_t>& to, int low_bits,
                   int max_bits) {
  PermArgs p;
  std::memset(&p, 0, sizeof(p));
  const int r = (int)from.size();
  p.rank = r;
  std::map<int32_t, int> pos_out;
  for (int j = 0; j < r; ++j) pos_out[to[j]] = r - 1 - j;
  std::vector<int> dst(r);
  for (int j = 0; j < r; ++j) dst[r - 1 - j] = pos_out[from[j]];
  // tile: the fastest input bits and the input bits that become the fastest
  // output bits, then more fast input bits up to the tile size
  const int low = std::min(low_bits, r);
  std::vector<bool> in_tile(r, false);
  for (int q = 0; q < low; ++q) in_tile[q] = true;
  for (int q = 0; q < r; ++q)
    if (dst[q] < low) in_tile[q] = true;
  int t = 0;
  for (int q = 0; q < r; ++q) t += in_tile[q] ? 1 : 0;
  const int target = std::min(r, max_bits);
  for (int q = 0; q < r && t < target; ++q)
    if (!in_tile[q]) {
      in_tile[q] = true;
      ++t;
    }
  std::vector<int> tin, nin;
  for (int q = 0; q < r; ++q) (in_tile[q] ? tin : nin).push_back(q);
  std::vector<int> tout;
  for (int q : tin) tout.push_back(dst[q]);
  std::sort(tout.begin(), tout.end());
  p.t = (int)tin.size();
  p.nn = (int)nin.size();
  for (int i = 0; i < p.t; ++i) {
    p.tin[i] = tin[i];
    p.tout[i] = tout[i];
    // input-order index of the tile bit whose output position is tout[i]
    for (int k = 0; k < p.t; ++k)
      if (dst[tin[k]] == tout[i]) p.f2e[i] = k;
  }
  for (int i = 0; i < p.nn; ++i) {
    p.nin[i] = nin[i];
    p.nout[i] = dst[nin[i]];
  }
  return p;
}

void host_relayout(const float* src, float* dst, const std::vector<int32_t>& from,
                   const std::vector<int32_t>& to) {
  const int r = (int)from.size();
  std::map<int32_t, int> pos_out;
  for (int j = 0; j < r; ++j) pos_out[to[j]] = r - 1 - j;
  std::vector<int> d(r);
  for (int j = 0; j < r; ++j) d[r - 1 - j] = pos_out[from[j]];
  const uint64_t n = 1ull << r;
  for (uint64_t a = 0; a < n; ++a) {
    uint64_t b = 0;
    for (int q = 0; q < r; ++q) b |= ((a >> q) & 1ull) << d[q];
    dst[2 * b] = src[2 * a];
    dst[2 * b + 1] = src[2 * a + 1];
  }
}

stem_status build_layout(const stem_plan_desc* d, PlanLayout* L, std::string* err) {
  if (!d || !L) {
    *err = "null descriptor";
    return STEM_EINVAL;
  }
  if (d->n_open < 0 || d->n_sliced < 0 || d->n_proj < 0 || d->stem_rank < 0 ||
      d->n_branches < 0) {
    *err = "negative count in descriptor";
    return STEM_EINVAL;
  }
  if ((d->n_open && !d->open_labels) || (d->n_sliced && !d->sliced_labels) ||
      (d->n_proj && !d->proj_labels) || (d->stem_rank && !d->stem_labels) ||
      !d->stem_data || (d->n_branches && (!d->branch_ranks || !d->branch_data))) {
    *err = "null array in descriptor";
    return STEM_EINVAL;
  }
  if (d->precision < STEM_FP32 || d->precision > STEM_SPLIT_BF16) {
    *err = "unknown precision " + std::to_string(d->precision);
    return STEM_EINVAL;
  }
  L->max_rank = d->max_rank > 0 ? d->max_rank : kDefaultMaxRank;
  if (L->max_rank > 40) {
    *err = "max_rank above 40";
    return STEM_EINVAL;
  }
  if (d->n_sliced > 62 || d->n_proj > 62 || d->n_open > 40) {
    *err = "too many sliced, projected or open labels";
    return STEM_EINVAL;
  }
  L->open.assign(d->open_labels, d->open_labels + d->n_open);
  L->sliced.assign(d->sliced_labels, d->sliced_labels + d->n_sliced);
  L->proj.assign(d->proj_labels, d->proj_labels + d->n_proj);
  if (has_dup(L->open) || has_dup(L->sliced) || has_dup(L->proj)) {
    *err = "repeated label in open, sliced or projected list";
    return STEM_ELABEL;
  }
  std::map<int32_t, FixedSrc> fixed;
  std::set<int32_t> open_set(L->open.begin(), L->open.end());
  for (int j = 0; j < d->n_sliced; ++j) fixed[L->sliced[j]] = FixedSrc{0, j};
  for (int j = 0; j < d->n_proj; ++j) {
    if (fixed.count(L->proj[j])) {
      *err = "label " + std::to_string(L->proj[j]) + " is both sliced and projected";
      return STEM_ELABEL;
    }
    fixed[L->proj[j]] = FixedSrc{1, j};
  }
  for (int32_t x : L->open)
    if (fixed.count(x)) {
      *err = "label " + std::to_string(x) + " is open and sliced or projected";
      return STEM_ELABEL;
    }

  // tensors and label counts
  std::vector<std::vector<int32_t>> br(d->n_branches);
  std::map<int32_t, int> count;
  L->stem_labels_in.assign(d->stem_labels, d->stem_labels + d->stem_rank);
  if (has_dup(L->stem_labels_in)) {
    *err = "repeated label in the stem";
    return STEM_ELABEL;
  }
  for (int32_t x : L->stem_labels_in) {
    if (x < 0) {
      *err = "negative label";
      return STEM_ELABEL;
    }
    count[x]++;
  }
  int64_t off = 0;
  for (int i = 0; i < d->n_branches; ++i) {
    const int r = d->branch_ranks[i];
    if (r < 0 || r > 24) {
      *err = "branch " + std::to_string(i) + " has rank " + std::to_string(r) + " (0..24)";
      return STEM_ESHAPE;
    }
    if (r && !d->branch_labels) {
      *err = "null branch_labels";
      return STEM_EINVAL;
    }
    br[i].assign(d->branch_labels + off, d->branch_labels + off + r);
    off += r;
    if (has_dup(br[i])) {
      *err = "repeated label in branch " + std::to_string(i);
      return STEM_ELABEL;
    }
    for (int32_t x : br[i]) {
      if (x < 0) {
        *err = "negative label";
        return STEM_ELABEL;
      }
      count[x]++;
    }
  }
  for (int32_t x : L->open)
    if (count[x] < 1) {
      *err = "open label " + std::to_string(x) + " occurs in no tensor";
      return STEM_ELABEL;
    }
  for (auto& kv : count) {
    if (open_set.count(kv.first) || fixed.count(kv.first)) continue;
    if (kv.second < 2) {
      *err = "label " + std::to_string(kv.first) + " occurs in " + std::to_string(kv.second) +
             " tensor (a summed label must join two or more)";
      return STEM_ELABEL;
    }
  }

  // initial stem: fixed labels first (in stem order), then the rest
  L->stem_fixed.clear();
  L->stem_fixed_src.clear();
  L->stem_rest.clear();
  for (int32_t x : L->stem_labels_in) {
    auto it = fixed.find(x);
    if (it != fixed.end()) {
      L->stem_fixed.push_back(x);
      L->stem_fixed_src.push_back(it->second);
    } else {
      L->stem_rest.push_back(x);
    }
  }
  std::vector<int32_t> cur = L->stem_rest;
  auto too_many_fixed = [](const std::vector<FixedSrc>& src) {
    int n_sl = 0;
    for (const FixedSrc& f : src) n_sl += f.is_proj == 0 ? 1 : 0;
    return n_sl > kMaxSlicedPerTensor || src.size() > 62;
  };
  if (too_many_fixed(L->stem_fixed_src)) {
    *err = "the initial stem carries more than 32 sliced or 62 fixed labels";
    return STEM_EUNSUPPORTED;
  }
  if ((int)cur.size() > L->max_rank) {
    *err = "initial stem rank " + std::to_string(cur.size()) + " above max_rank " +
           std::to_string(L->max_rank);
    return STEM_ESHAPE;
  }
  L->peak_rank = (int)cur.size();
  L->max_ws_rank = 0;

  // labels carried by branches after branch i
  std::vector<std::set<int32_t>> later(d->n_branches);
  {
    std::set<int32_t> acc;
    for (int i = d->n_branches - 1; i >= 0; --i) {
      later[i] = acc;
      acc.insert(br[i].begin(), br[i].end());
    }
  }

  // steps whose branch carries each (unfixed) label, for the layout choice
  std::map<int32_t, std::vector<int>> uses;
  for (int j = 0; j < d->n_branches; ++j)
    for (int32_t x : br[j])
      if (!fixed.count(x)) uses[x].push_back(j);
  auto next_use = [&](int32_t x, int i) -> int {
    auto it = uses.find(x);
    if (it == uses.end()) return 1 << 30;
    for (int j : it->second)
      if (j > i) return j;
    return 1 << 30;
  };

  L->steps.clear();
  stem_plan_summary& S = L->summary;
  std::memset(&S, 0, sizeof(S));
  for (int i = 0; i < d->n_branches; ++i) {
    StepLayout st;
    st.branch_index = i;
    st.labels_before = cur;
    std::vector<int32_t> rest_b;
    for (int32_t x : br[i]) {
      auto it = fixed.find(x);
      if (it != fixed.end()) {
        st.fixed.push_back(x);
        st.fixed_src.push_back(it->second);
      } else {
        rest_b.push_back(x);
      }
    }
    std::set<int32_t> rest_set(rest_b.begin(), rest_b.end());
    std::set<int32_t> cur_set(cur.begin(), cur.end());
    // labels the stem and the branch share: summed, or kept when a later
    // branch or the result still carries them (batch labels: the product
    // runs once per assignment of them, a batched product)
    std::vector<int32_t> shared, keep;
    for (int32_t x : cur) {
      if (!rest_set.count(x))
        keep.push_back(x);
      else if (later[i].count(x) || open_set.count(x))
        st.batch.push_back(x);
      else
        shared.push_back(x);
    }
    for (int32_t x : rest_b)
      if (!cur_set.count(x)) st.free_labels.push_back(x);
    const int h = (int)st.batch.size();
    if (h > kMaxBatchLabels) {
      *err = "step " + std::to_string(i) + " keeps " + std::to_string(h) +
             " labels shared by the stem and the branch (at most 4)";
      return STEM_EUNSUPPORTED;
    }
    // the branch's batch labels select its variant like fixed labels do
    for (int j = 0; j < h; ++j) {
      st.fixed.push_back(st.batch[j]);
      st.fixed_src.push_back(FixedSrc{2, j});
    }
    if (too_many_fixed(st.fixed_src)) {
      *err = "branch " + std::to_string(i) + " carries more than 32 sliced labels";
      return STEM_EUNSUPPORTED;
    }
    std::set<int32_t> batch_set(st.batch.begin(), st.batch.end());
    const int R = (int)cur.size();
    const int s = (int)shared.size();
    st.rank_in = R;
    st.s = s;
    st.f = (int)st.free_labels.size();
    if (s > kMaxShared || st.f > kMaxFree) {
      *err = "step " + std::to_string(i) + " sums " + std::to_string(s) + " labels and adds " +
             std::to_string(st.f) + " (at most 16 each)";
      return STEM_ESHAPE;
    }
    // Operand addressing: the product reads the stem in place when its 4
    // fastest labels are all kept (M-fast) or its min(s, 3) fastest labels
    // are all summed (K-low); otherwise one permute re-stores it.  The 4
    // labels that become the output's fastest are the input's 4 fastest in
    // M-fast mode and otherwise the 4 kept labels whose next use is latest.
    std::set<int32_t> shared_set(shared.begin(), shared.end());
    const int m_bits = R - s - h;
    const int n_lo = std::min(4, m_bits);
    // Labels for the output's `count` fastest bits (bit 0 first).  Best: 3 or
    // more kept labels that a later step sums together (the latest such
    // step), so that step finds its 3 fastest bits summed and runs K-low,
    // with a 4th label needed no earlier; else the labels needed latest.
    auto latest = [&](const std::vector<int32_t>& kept, int count) {
      std::vector<std::pair<int, int>> by_use;  // (next use, position in kept)
      for (int j = 0; j < (int)kept.size(); ++j) by_use.push_back({next_use(kept[j], i), j});
      std::stable_sort(by_use.begin(), by_use.end(),
                       [](const std::pair<int, int>& a, const std::pair<int, int>& b) {
                         return a.first > b.first;
                       });
      std::vector<int32_t> out;
      if (count == 4) {
        for (size_t a = 0; a < by_use.size(); ) {
          size_t b = a;
          while (b < by_use.size() && by_use[b].first == by_use[a].first) ++b;
          if (b - a >= 3) {
            for (size_t j = a; j < b && out.size() < 4; ++j) out.push_back(kept[by_use[j].second]);
            // a 4th label needed no earlier than the group: the latest one left
            for (size_t j = 0; j < a && out.size() < 4; ++j) out.push_back(kept[by_use[j].second]);
            if (out.size() == 4) return out;
            out.clear();
          }
          a = b;
        }
      }
      // the labels needed latest; the earliest-needed one at bit 0
      for (int j = count - 1; j >= 0; --j) out.push_back(kept[by_use[j].second]);
      return out;
    };
    bool bottom_kept = m_bits >= 4;
    for (int q = 0; q < 4 && bottom_kept; ++q)
      if (shared_set.count(cur[R - 1 - q]) || batch_set.count(cur[R - 1 - q])) bottom_kept = false;
    bool low_summed = true;
    for (int q = 0; q < std::min(s, 3); ++q)
      if (!shared_set.count(cur[R - 1 - q])) low_summed = false;
    GemmLayout& G = st.gemm;
    std::memset(&G, 0, sizeof(G));
    std::vector<int32_t> mlo_labels;  // m bit 0 first
    if (bottom_kept) {
      st.permuted = false;
      st.labels_gemm = cur;
      G.amode = 1;
      for (int q = 0; q < 4; ++q) mlo_labels.push_back(cur[R - 1 - q]);
    } else if (low_summed) {
      st.permuted = false;
      st.labels_gemm = cur;
      G.amode = 0;
      mlo_labels = latest(keep, n_lo);
    } else {
      st.permuted = true;
      if (m_bits >= 4) {
        const std::vector<int32_t> b4 = latest(keep, 4);
        const std::set<int32_t> b4s(b4.begin(), b4.end());
        for (int32_t x : keep)
          if (!b4s.count(x)) st.labels_gemm.push_back(x);
        st.labels_gemm.insert(st.labels_gemm.end(), st.batch.begin(), st.batch.end());
        st.labels_gemm.insert(st.labels_gemm.end(), shared.begin(), shared.end());
        for (int q = 3; q >= 0; --q) st.labels_gemm.push_back(b4[q]);
        mlo_labels = b4;
        G.amode = 1;
      } else {
        st.labels_gemm = keep;
        st.labels_gemm.insert(st.labels_gemm.end(), st.batch.begin(), st.batch.end());
        st.labels_gemm.insert(st.labels_gemm.end(), shared.begin(), shared.end());
        mlo_labels = latest(keep, n_lo);
        G.amode = 0;
      }
      st.perm = make_perm(cur, st.labels_gemm);
      L->max_ws_rank = std::max(L->max_ws_rank, R);
    }
    auto pos_of = [&](int32_t x) {
      return R - 1 - (int)(std::find(st.labels_gemm.begin(), st.labels_gemm.end(), x) -
                           st.labels_gemm.begin());
    };
    // k index: summed labels in the order of the stem read by the product,
    // so k's low bits are its fastest summed labels
    std::vector<int32_t> kept_g;
    st.sigma.clear();
    for (int32_t x : st.labels_gemm) {
      if (shared_set.count(x))
        st.sigma.push_back(x);
      else if (!batch_set.count(x))
        kept_g.push_back(x);
    }
    // batch index bit q (q = 0 least significant) is batch label h-1-q
    for (int q = 0; q < h; ++q) st.hpos_a[q] = pos_of(st.batch[h - 1 - q]);
    G.s = s;
    G.f = st.f;
    for (int j = 0; j < s; ++j) G.spos[s - 1 - j] = pos_of(st.sigma[j]);
    // m index: bits 0..3 at the chosen labels, the rest in address order
    std::vector<int32_t> ins;
    for (int j = 0; j < s; ++j) ins.push_back(G.spos[j]);
    for (int q = 0; q < h; ++q) ins.push_back(st.hpos_a[q]);
    const std::set<int32_t> mlo_set(mlo_labels.begin(), mlo_labels.end());
    for (int b = 0; b < (int)mlo_labels.size(); ++b) {
      G.mlo[b] = pos_of(mlo_labels[b]);
      ins.push_back(G.mlo[b]);
    }
    std::sort(ins.begin(), ins.end());
    G.nins = (int)ins.size();
    for (int j = 0; j < G.nins; ++j) G.ins[j] = ins[j];
    std::vector<int32_t> m_hi;  // most significant first
    for (int32_t x : kept_g)
      if (!mlo_set.count(x)) m_hi.push_back(x);
    G.cmode = m_bits >= 4 ? 1 : 0;
    // the output: batch labels most significant, then the product's rows
    // and columns
    st.labels_after = st.batch;
    st.labels_after.insert(st.labels_after.end(), m_hi.begin(), m_hi.end());
    if (G.cmode == 1)
      st.labels_after.insert(st.labels_after.end(), st.free_labels.begin(), st.free_labels.end());
    for (int b = (int)mlo_labels.size() - 1; b >= 0; --b) st.labels_after.push_back(mlo_labels[b]);
    if (G.cmode == 0)
      st.labels_after.insert(st.labels_after.end(), st.free_labels.begin(), st.free_labels.end());
    st.rank_out = (int)st.labels_after.size();
    if (st.rank_out > L->max_rank) {
      *err = "stem rank " + std::to_string(st.rank_out) + " after step " + std::to_string(i) +
             " above max_rank " + std::to_string(L->max_rank);
      return STEM_ESHAPE;
    }
    st.M = 1ll << (R - s - h);
    st.K = 1ll << s;
    st.N = 1ll << st.f;
    L->peak_rank = std::max(L->peak_rank, st.rank_out);
    L->max_ws_rank = std::max(L->max_ws_rank, st.rank_out);
    const double M = (double)st.M, K = (double)st.K, N = (double)st.N, H = (double)(1 << h);
    S.flops_per_slice += 8.0 * H * M * K * N;
    S.bytes_per_slice += 8.0 * H * (M * K + M * N + K * N);
    if (st.permuted) {
      S.perm_bytes_per_slice += 16.0 * (double)(1ull << R);
      S.n_permutes++;
    }
    cur = st.labels_after;
    L->steps.push_back(st);
  }
  std::set<int32_t> fin(cur.begin(), cur.end());
  if (fin != open_set || cur.size() != L->open.size()) {
    *err = "the final stem carries " + join(cur) + ", not the open labels " + join(L->open);
    return STEM_ELABEL;
  }
  L->final_labels = cur;
  const int r = (int)cur.size();
  L->final_map.rank = r;
  for (int j = 0; j < r; ++j) {
    const int pos_in = r - 1 - j;
    int k = 0;
    while (L->open[k] != cur[j]) ++k;
    L->final_map.dst[pos_in] = r - 1 - k;
  }
  L->final_perm = make_perm(cur, L->open, kAccTileLowBits, kAccTileMaxBits);
  S.n_steps = d->n_branches;
  S.peak_rank = L->peak_rank;
  S.n_open = d->n_open;
  S.n_slices = 1ull << d->n_sliced;
  return STEM_OK;
}

}  // namespace stem
