// Device helpers shared by the libstemgpu kernels (gfx950): operand
// selection per slice, the product's operand addressing, launch geometry.
// Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>

#include "kernels.h"

namespace stem {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kLdsBudget = 64 * 1024;  // LDS staging by default: two workgroups still fit a CU
constexpr int kLdsMax = 160 * 1024;    // gfx950's LDS per workgroup (schedule lds = 1)

// The LDS one workgroup may use on the current device (cached per device).
static inline size_t lds_limit() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return kLdsBudget;
  if (!cache[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = kLdsBudget;
    cache[dev] = std::max(kLdsBudget, std::min(v, kLdsMax));
  }
  return (size_t)cache[dev];
}

// Whether a product stages its branch fragments (lds bytes) in LDS: the
// schedule's choice (1 = up to the device limit, 0 = never, -1 = up to the
// default budget).
static inline bool use_lds(int sched_lds, size_t lds) {
  if (sched_lds == 0) return false;
  return lds <= (sched_lds == 1 ? lds_limit() : (size_t)kLdsBudget);
}

// Raise a kernel's dynamic LDS limit above the default when a launch needs
// it (once per kernel and size).
template <typename F>
static inline hipError_t allow_lds(F* kernel, size_t lds, size_t* allowed) {
  if (lds <= (size_t)kLdsBudget || lds <= *allowed) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) *allowed = lds;
  return e;
}
constexpr int kTargetBlocks = 4096;    // workgroups per launch before row loops kick in

// Loops over the small per-launch tables below are fully unrolled with a
// predicate, so every table index is a constant and the tables stay in
// scalar registers instead of being copied into per-lane arrays.
__device__ __forceinline__ const char* op_base(const Operand& o, int z, uint64_t s0) {
  const uint32_t j = (uint32_t)z >> o.hbits;
  const uint32_t hb = (uint32_t)z & ((1u << o.hbits) - 1u);
  uint64_t v = o.sel.vbase;
  const uint64_t s = s0 + (uint64_t)j;
#pragma unroll
  for (int q = 0; q < kMaxSlicedPerTensor; ++q)
    if (q < o.sel.nv) v |= ((s >> o.sel.vshift[q]) & 1ull) << o.sel.vpos[q];
  int64_t off = 0;
#pragma unroll
  for (int q = 0; q < kMaxBatchLabels; ++q) {
    if (q < o.sel.nh) v |= (uint64_t)((hb >> o.sel.hshift[q]) & 1u) << o.sel.hvpos[q];
    if (q < o.nhpos) off |= (int64_t)((hb >> q) & 1u) << o.hpos[q];
  }
  return (const char*)o.ptr + (int64_t)j * o.zstride + (int64_t)v * o.vstride + 8 * off;
}

// ---------------------------------------------------------------------------
// Complex product C[M x N] = A[M x K] . B[K x N] of one stem step.
//
// Operand addressing (GemmLayout).  A is the stem: row m starts at
// lo(m & 15) | spread(m >> 4) and entry k sits kpos(k) further, so any
// order of the stem's labels is read in place:
//   K-low (AM = 0): k bits 0..2 are the 3 fastest address bits; lane group
//                   g reads k = 2g, 2g+1 of its row as one 16-byte vector
//                   and the 4 groups cover 64 contiguous bytes of the row;
//   M-fast (AM = 1): the 4 low bits of m are the 4 fastest address bits, so
//                   the 16 rows of a block are 128 contiguous bytes per k.
// C is the next stem: entry (m, n) goes to
//   N-fast (CM = 0): m N + n                           (when M < 16)
//   CM = 1:          (m>>4) 2^(4+f) | n 2^4 | (m&15)   (the 4 labels of m's
//                   low bits become the output's fastest, new labels above)
// so the next step can read the output M-fast, and the host chooses which
// 4 labels sit at the bottom without a separate permute pass.
// ---------------------------------------------------------------------------

// The row start splits into a per-lane part (m & 15 = the lane's row in its
// 16-row block, fixed for the whole kernel) and a wave-uniform part
// (m >> 4, the block), so the expensive bit spreading of the block index
// runs on the scalar unit; likewise a k offset splits into the lane's low
// k bits and the chunk's uniform high bits (kpos of disjoint bit sets ORs).
__device__ __forceinline__ int64_t row_lo(int r16, const GemmGeom& g) {
  int64_t lo = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) lo |= (int64_t)((r16 >> b) & 1) << g.mlo[b];
  return lo;
}

__device__ __forceinline__ int64_t row_hi(int64_t mh, const GemmGeom& g) {
  int64_t a = mh;
#pragma unroll
  for (int i = 0; i < kMaxShared + 4 + kMaxBatchLabels; ++i) {
    if (i < g.nins) {
      const int p = g.ins[i];
      a = ((a >> p) << (p + 1)) | (a & ((1ll << p) - 1));
    }
  }
  return a;
}

__device__ __forceinline__ int64_t k_offset(int k, const GemmGeom& g) {
  int64_t a = 0;
#pragma unroll
  for (int i = 0; i < kMaxShared; ++i)
    if (i < g.s) a |= (int64_t)((k >> i) & 1) << g.spos[i];
  return a;
}

// Index of the calling wave in its workgroup, as a scalar.
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// 4 consecutive reals A[m][kr0 .. kr0+3] (= complex k0 = kr0/2 and k0+1);
// ko0/ko1 are the offsets of those two k values (adjacent in K-low mode).
// FULL: the caller guarantees a valid row (rb >= 0) and kr0 + 4 <= 2K.
template <int AM, int FULL>
__device__ __forceinline__ f32x4 load_kr4(const float* __restrict__ A, int64_t rb, int kr0,
                                          int64_t ko0, int64_t ko1, const GemmGeom& g) {
  f32x4 v = f32x4{0.f, 0.f, 0.f, 0.f};
  if (FULL) {
    if (AM == 0) return *(const f32x4*)(A + 2 * (rb + ko0));
    const float2 t0 = *(const float2*)(A + 2 * (rb + ko0));
    const float2 t1 = *(const float2*)(A + 2 * (rb + ko1));
    return f32x4{t0.x, t0.y, t1.x, t1.y};
  }
  if (rb < 0) return v;
  if (AM == 0) {
    if (kr0 < g.Kr) {
      const float* src = A + 2 * (rb + ko0);
      if (g.Kr >= 4) {
        v = *(const f32x4*)src;
      } else {
        const float2 t = *(const float2*)src;
        v.x = t.x;
        v.y = t.y;
      }
    }
  } else {
    const int k0 = kr0 >> 1;
    if (k0 < g.K) {
      const float2 t = *(const float2*)(A + 2 * (rb + ko0));
      v.x = t.x;
      v.y = t.y;
    }
    if (k0 + 1 < g.K) {
      const float2 t = *(const float2*)(A + 2 * (rb + ko1));
      v.z = t.x;
      v.w = t.y;
    }
  }
  return v;
}

// Store the 4 consecutive reals C[m][nr0 .. nr0+3]; FULL: nr0 + 4 <= 2N.
// The product's output is written once and read by the next step only after
// the whole launch, far beyond what the caches hold: the stores are
// non-temporal (streamed past the caches), which measured about 3 % faster
// on the HBM-bound steps with identical bits.
template <int CM, int FULL>
__device__ __forceinline__ void store_nr4(float* __restrict__ C, int64_t m, int nr0, f32x4 v,
                                          const GemmGeom& g) {
  if (CM == 0) {
    if (!FULL && nr0 >= g.Nr) return;
    float* dst = C + m * (int64_t)g.Nr + nr0;
    if (FULL || g.Nr >= 4)
      __builtin_nontemporal_store(v, (f32x4*)dst);
    else
      __builtin_nontemporal_store(f32x2{v.x, v.y}, (f32x2*)dst);
  } else {
    const int n0 = nr0 >> 1;
    const int64_t base = ((m >> 4) << (4 + g.f)) | (m & 15);
    if (FULL || n0 < g.N)
      __builtin_nontemporal_store(f32x2{v.x, v.y}, (f32x2*)(C + 2 * (base | ((int64_t)n0 << 4))));
    if (FULL || n0 + 1 < g.N)
      __builtin_nontemporal_store(f32x2{v.z, v.w},
                                  (f32x2*)(C + 2 * (base | ((int64_t)(n0 + 1) << 4))));
  }
}

// The next value of a bit-spread counter: positions `mask` hold the
// counter's bits, all other positions are ignored.
__device__ __forceinline__ int64_t spread_next(int64_t x, int64_t mask) {
  return ((x | ~mask) + 1) & mask;
}

static inline GemmGeom make_geom(const GemmLayout& lay, int64_t M, int64_t K, int64_t N, int kq) {
  GemmGeom g;
  std::memset(&g, 0, sizeof(g));
  g.M = M;
  g.K = (int)K;
  g.N = (int)N;
  g.Kr = (int)(2 * K);
  g.Nr = (int)(2 * N);
  g.KC = std::max(kq, g.Kr) / kq;
  g.NT = std::max(16, g.Nr) / 16;
  g.s = lay.s;
  g.f = lay.f;
  for (int i = 0; i < 16; ++i) g.spos[i] = lay.spos[i];
  for (int i = 0; i < 4; ++i) g.mlo[i] = lay.mlo[i];
  g.nins = lay.nins;
  for (int i = 0; i < 24; ++i) g.ins[i] = lay.ins[i];
  return g;
}

// True when the 3M FP32 product applies: whole 16-complex-column tiles,
// whole 8-complex k chunks, output in block order, whole row blocks.
static inline bool gauss_ok(const GemmGeom& g, int cmode) {
  return cmode == 1 && g.K % 8 == 0 && g.N % 16 == 0 && g.M % 64 == 0;
}

// Schedule with the defaults filled in (see GemmSched).
static inline GemmSched resolve_sched(const GemmGeom& g, GemmSched s) {
  if (s.algo == 1) {
    const int ntc_all = g.NT >> 1;
    if (s.ntw <= 0) s.ntw = std::min(4, ntc_all);
    s.ntw = std::min(s.ntw, std::min(4, ntc_all));
    while (s.ntw & (s.ntw - 1)) s.ntw &= s.ntw - 1;
    if (s.tm <= 0) s.tm = 1;
    s.tm = s.tm >= 4 ? 4 : s.tm >= 2 ? 2 : 1;
    while (s.tm > 1 && g.M % (64 * s.tm) != 0) s.tm >>= 1;
    while (s.tm * s.ntw > 4) s.ntw >>= 1;  // register budget: 3 accumulators per pair
    if (s.blocks <= 0) s.blocks = kTargetBlocks;
    return s;
  }
  s.algo = 0;
  int nt2 = 1;
  while (nt2 < g.NT) nt2 <<= 1;
  if (s.ntw <= 0) s.ntw = std::min(8, nt2);
  s.ntw = std::min(s.ntw, std::min(8, nt2));
  while (s.ntw & (s.ntw - 1)) s.ntw &= s.ntw - 1;  // a power of two: NT % ntw == 0
  if (s.tm <= 0) s.tm = s.ntw <= 2 ? 4 : 2;
  s.tm = s.tm >= 4 ? 4 : s.tm >= 2 ? 2 : 1;
  if (s.blocks <= 0) s.blocks = kTargetBlocks;
  return s;
}

// Grid of a product launch: x row-block groups (each workgroup loops over
// row blocks when there are more than the target), y column chunks, z slices.
static inline dim3 gemm_grid(const GemmGeom& g, int TM, int NTW, int nz, int target) {
  const int64_t rows_per_wg = 4 * 16 * TM;
  const int64_t nblk = (g.M + rows_per_wg - 1) / rows_per_wg;
  const int gy = (g.NT + NTW - 1) / NTW;
  const int64_t want = std::max<int64_t>(1, target / ((int64_t)gy * nz));
  const int64_t gx = std::min<int64_t>(nblk, want);
  return dim3((unsigned)gx, (unsigned)gy, (unsigned)nz);
}

// True when every row block, k chunk and column tile of the launch is
// whole, so the kernel runs without bounds predicates: M a multiple of the
// rows per workgroup, 2K of the k chunk (kq reals), 2N of the tile width,
// output in block order (CM = 1).
static inline bool gemm_full(const GemmGeom& g, int TM, int NTW, int CM, int kq) {
  return CM == 1 && g.M % (64 * TM) == 0 && g.Kr % kq == 0 && g.Nr % 16 == 0 &&
         g.NT % NTW == 0;
}

struct LaunchCtx {
  const Operand* A;
  const Operand* B;
  const Operand* C;
  uint64_t s0;
  int nz;
  GemmGeom g;
  GemmSched sch;
  hipStream_t st;
};

#define STEM_TM_NTW_DISPATCH(FN, ...)                                        \
  switch (c.sch.tm * 16 + c.sch.ntw) {                                       \
    case 16 + 1: FN<1, 1, __VA_ARGS__>(c); break;                            \
    case 16 + 2: FN<1, 2, __VA_ARGS__>(c); break;                            \
    case 16 + 4: FN<1, 4, __VA_ARGS__>(c); break;                            \
    case 16 + 8: FN<1, 8, __VA_ARGS__>(c); break;                            \
    case 32 + 1: FN<2, 1, __VA_ARGS__>(c); break;                            \
    case 32 + 2: FN<2, 2, __VA_ARGS__>(c); break;                            \
    case 32 + 4: FN<2, 4, __VA_ARGS__>(c); break;                            \
    case 32 + 8: FN<2, 8, __VA_ARGS__>(c); break;                            \
    case 64 + 1: FN<4, 1, __VA_ARGS__>(c); break;                            \
    case 64 + 2: FN<4, 2, __VA_ARGS__>(c); break;                            \
    case 64 + 4: FN<4, 4, __VA_ARGS__>(c); break;                            \
    default: FN<4, 8, __VA_ARGS__>(c); break;                                \
  }


// Product launchers, one translation unit per arithmetic.
void launch_gemm_f32(const LaunchCtx& c, const GemmLayout& lay);
void launch_gemm_f32g(const LaunchCtx& c, const GemmLayout& lay);
void launch_gemm_split(const LaunchCtx& c, const GemmLayout& lay, int bf16);

}  // namespace stem
