// Internal declarations shared by the host planner, the kernels and the
// C-ABI layer of libstemgpu.  Nothing here is part of the public interface.
#pragma once

#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/stemgpu.h"

namespace stem {

constexpr int kDefaultMaxRank = 33;
constexpr int kPermTileLowBits = 5;   // permute: output and input runs of 32 entries (256 B)
constexpr int kPermTileMaxBits = 11;  // permute: at most 2048 entries per tile (measured
                                      // faster than 1024 or 4096 on 2^17-2^30-entry stems)
constexpr int kAccTileLowBits = 5;    // result sum: the same runs, FP64 tile entries
constexpr int kAccTileMaxBits = 10;   // result sum: at most 1024 entries per tile

// Bit permutation of a rank-r tensor, in the form the permute kernel takes.
// Input address bit p (0 = least significant) moves to output bit dst[p].
// Tile bits (tin, ascending) are staged through LDS; the others index the
// workgroup.
struct PermArgs {
  int32_t rank;
  int32_t t;            // tile bits
  int32_t nn;           // non-tile bits = rank - t
  int32_t pad;
  int32_t tin[16];      // input positions of the tile bits, ascending
  int32_t tout[16];     // output positions of the tile bits, ascending
  int32_t f2e[16];      // output-order tile bit i is input-order tile bit f2e[i]
  int32_t nin[64];      // input positions of the non-tile bits, ascending
  int32_t nout[64];     // their output positions
};

// Destination bit of every source bit, for the final reorder into the
// open-label order (rank <= 63).
struct BitMap {
  int32_t rank;
  int32_t dst[63];
};

// Operand addressing of one product (see the kernels).  Row m of the stem
// starts at lo(m & 15) | spread(m >> 4): the 4 low bits of m go to the
// address positions mlo[], the others fill the positions not taken by the
// summed labels or mlo[], in ascending order.  Entry k of a row is at
// kpos(k): k bit i at position spos[i].
//   amode 0 = K-low: k bits 0..2 are address bits 0..2 (or K < 8 and the
//             summed labels are exactly the fastest ones), so a lane reads
//             2 adjacent complex entries as one 16-byte vector;
//   amode 1 = M-fast: mlo[] = 0..3, so the 16 rows of a block are 16
//             consecutive entries for every k.
//   cmode 0 = N-fast output: address m N + n (used when M < 16);
//   cmode 1 = output order (rows by m >> 4), new labels, (rows by m & 15):
//             address (m >> 4) 2^(4+f) | n 2^4 | (m & 15).
struct GemmLayout {
  int32_t amode, cmode, s, f;
  int32_t spos[16];     // stem address position of k bit i (i = 0 least significant)
  int32_t mlo[4];       // address positions of m bits 0..3
  int32_t nins;         // positions to skip when spreading m >> 4 (summed, mlo, batch)
  int32_t ins[24];      // ascending
};

// Launch schedule of one product (chosen by the autotuner; 0 = default):
// tm 16-row blocks per wave, at most ntw 16-column tiles per workgroup,
// about `blocks` workgroups per launch, branch fragments in LDS or not.
struct GemmSched {
  int32_t tm = 0;       // 1, 2 or 4
  int32_t ntw = 0;      // 1, 2, 4 or 8 (algo 1: 16-complex-column tiles, 1, 2 or 4)
  int32_t blocks = 0;   // 256 .. 65536
  int32_t lds = -1;     // branch in LDS: 1 up to the device's 160 KB, 0 never, -1 up to 64 KB
  int32_t algo = 0;     // FP32 only: 0 real embedding, 1 three real products (3M)
};

struct GemmGeom {
  int64_t M;
  int32_t K, N, Kr, Nr, KC, NT, s, f;
  int32_t spos[16];
  int32_t mlo[4];
  int32_t nins;
  int32_t ins[24];
};

constexpr int kMaxShared = 16;  // K <= 2^16
constexpr int kMaxBatchLabels = 4;  // labels shared by stem and branch and kept, per step
constexpr int kMaxFree = 16;    // N <= 2^16
constexpr int kMaxSlicedPerTensor = 32;
constexpr int kMaxSlicesInFlight = 4096;
constexpr int kBranchHeader = 256;  // bytes before each branch variant's fragments

// Selection of one slice's sub-tensor: the variant index (the values of the
// tensor's fixed labels, most significant first) is vbase (bits fixed by
// the projected assignment) plus, for each sliced label j, bit vshift[j] of
// the slice id placed at variant bit vpos[j], plus, for each batch label i
// of the step, bit hshift[i] of the batch index placed at variant bit
// hvpos[i].
struct SliceSel {
  uint64_t vbase;
  int32_t nv;
  int32_t nh;
  int8_t vshift[kMaxSlicedPerTensor];
  int8_t vpos[kMaxSlicedPerTensor];
  int8_t hshift[kMaxBatchLabels];
  int8_t hvpos[kMaxBatchLabels];
};

// A kernel operand for a batch of slices.  A launch's batch item z is
// slice s0 + (z >> hbits) of the group and batch index hb = z & (2^hbits -
// 1) over the step's batch labels (labels the stem and the branch share
// and keep, a batched product); it starts at ptr + (z >> hbits) * zstride
// + variant * vstride + 8 * (sum_i bit i of hb << hpos[i]) bytes.
struct Operand {
  const void* ptr;
  int64_t zstride;
  int64_t vstride;
  SliceSel sel;
  int32_t hbits;
  int32_t nhpos;
  int8_t hpos[kMaxBatchLabels];
  int32_t pad;
};

// Where the value of a fixed (sliced or projected) label comes from.
struct FixedSrc {
  int32_t is_proj;      // 0: sliced label, 1: projected label, 2: batch label of the step
  int32_t index;        // position in sliced_labels / proj_labels / the step's batch labels
};

struct StepLayout {
  int32_t rank_in = 0, rank_out = 0, s = 0, f = 0;
  bool permuted = false;
  std::vector<int32_t> labels_before;  // stem order entering the step
  std::vector<int32_t> labels_gemm;    // stem order read by the product
  std::vector<int32_t> labels_after;   // stem order written by the product
  std::vector<int32_t> sigma;          // summed labels, K index order (first = MSB)
  std::vector<int32_t> free_labels;    // new labels, N index order (first = MSB)
  std::vector<int32_t> fixed;          // branch labels fixed per slice/batch, MSB first
  std::vector<FixedSrc> fixed_src;
  std::vector<int32_t> batch;          // labels shared and kept (batched product), MSB first
  int32_t hpos_a[kMaxBatchLabels] = {0, 0, 0, 0};  // stem address bit of batch-index bit i
  int32_t branch_index = 0;
  int64_t M = 0, K = 0, N = 0;
  GemmLayout gemm{};
  GemmSched sched{};                   // autotuned launch schedule (0 = default)
  PermArgs perm{};                     // valid when permuted
};

struct PlanLayout {
  std::vector<int32_t> open, sliced, proj;
  std::vector<int32_t> stem_labels_in;   // as given
  std::vector<int32_t> stem_fixed;       // stem's fixed labels, MSB first
  std::vector<FixedSrc> stem_fixed_src;
  std::vector<int32_t> stem_rest;        // stem's other labels, original order
  std::vector<StepLayout> steps;
  std::vector<int32_t> final_labels;
  BitMap final_map{};
  PermArgs final_perm{};                 // the same reorder as tiles (large results)
  int32_t peak_rank = 0;       // over every stem the steps read or write
  int32_t max_ws_rank = 0;     // largest tensor written to the workspace
  int32_t max_rank = kDefaultMaxRank;
  stem_plan_summary summary{};
};

// Build the layout of a descriptor on the host.  Returns a status and sets
// *err on failure.
stem_status build_layout(const stem_plan_desc* d, PlanLayout* out, std::string* err);

// Bit permutation that re-stores a tensor from C order over `from` to C
// order over `to` (both permutations of one label set).  The LDS tile holds
// the `low_bits` fastest input and output bits, padded with the next
// fastest input bits up to `max_bits`.
PermArgs make_perm(const std::vector<int32_t>& from, const std::vector<int32_t>& to,
                   int low_bits = kPermTileLowBits, int max_bits = kPermTileMaxBits);

// True when `from` and `to` are the same order.
bool same_order(const std::vector<int32_t>& from, const std::vector<int32_t>& to);

// Host reorder of a complex64 tensor (2 floats per entry) from C order over
// `from` to C order over `to`.
void host_relayout(const float* src, float* dst, const std::vector<int32_t>& from,
                   const std::vector<int32_t>& to);

// Value (0/1) of a fixed label for slice id s and projected assignment p.
inline int fixed_bit(const FixedSrc& fs, uint64_t s, uint64_t p, int n_sliced, int n_proj) {
  if (fs.is_proj == 2) return 0;  // batch labels vary within a launch (SliceSel::hshift)
  if (fs.is_proj) return (int)((p >> (n_proj - 1 - fs.index)) & 1ull);
  return (int)((s >> (n_sliced - 1 - fs.index)) & 1ull);
}

inline uint64_t variant_index(const std::vector<FixedSrc>& src, uint64_t s, uint64_t p,
                              int n_sliced, int n_proj) {
  uint64_t v = 0;
  for (const FixedSrc& fs : src) v = (v << 1) | (uint64_t)fixed_bit(fs, s, p, n_sliced, n_proj);
  return v;
}

// Thread-local error message of the C-ABI.
void set_error(const std::string& msg);

}  // namespace stem
