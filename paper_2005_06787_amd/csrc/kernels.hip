// Device kernels of libstemgpu for gfx950 (CDNA4, wave64).
//
// One stem step (paper §A.1, pairwise contraction; §A.2, the stem absorbs a
// branch) is an optional bit permutation of the stem's address followed by
// a complex matrix product [M x K] . [K x N] on the matrix cores.  The sum
// over slices (§A.1, slicing) is accumulated in FP64.  Every step kernel
// handles a batch of slices at once: blockIdx.z is the batch item, and each
// operand finds its slice's sub-tensor from the slice id (Operand).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "kernels.h"

namespace stem {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kLdsBudget = 64 * 1024;  // branch fragments staged in LDS up to this size
constexpr int kTargetBlocks = 4096;    // workgroups per launch before row loops kick in

// Loops over the small per-launch tables below are fully unrolled with a
// predicate, so every table index is a constant and the tables stay in
// scalar registers instead of being copied into per-lane arrays.
__device__ __forceinline__ const char* op_base(const Operand& o, int z, uint64_t s0) {
  uint64_t v = o.sel.vbase;
  const uint64_t s = s0 + (uint64_t)z;
#pragma unroll
  for (int j = 0; j < kMaxSlicedPerTensor; ++j)
    if (j < o.sel.nv) v |= ((s >> o.sel.vshift[j]) & 1ull) << o.sel.vpos[j];
  return (const char*)o.ptr + (int64_t)z * o.zstride + (int64_t)v * o.vstride;
}

// ---------------------------------------------------------------------------
// Bit-permutation transpose, staged through LDS.
//
// A workgroup owns one assignment of the non-tile bits (its block index).
// It reads the 2^t tile entries in input order -- the tile holds the 5
// fastest input bits, so each run of 32 entries (256 B) is contiguous --
// into LDS, then writes them in output order, where the 5 fastest output
// bits are also tile bits, so the writes are contiguous runs too.  One
// padding entry per 32 keeps the strided LDS reads off a single bank.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void stem_permute_kernel(Operand in_op, Operand out_op,
                                                           uint64_t s0, PermArgs p) {
  __shared__ float2 tile[(1 << kPermTileMaxBits) + (1 << kPermTileMaxBits) / 32];
  const int z = blockIdx.z;
  const float2* __restrict__ in = (const float2*)op_base(in_op, z, s0);
  float2* __restrict__ out = (float2*)op_base(out_op, z, s0);
  const uint64_t w = (uint64_t)blockIdx.x + (uint64_t)blockIdx.y * gridDim.x;
  uint64_t ib = 0, ob = 0;
  for (int i = 0; i < p.nn; ++i) {
    const uint64_t bit = (w >> i) & 1ull;
    ib |= bit << p.nin[i];
    ob |= bit << p.nout[i];
  }
  const int T = 1 << p.t;
  for (int e = threadIdx.x; e < T; e += blockDim.x) {
    uint64_t a = ib;
    for (int i = 0; i < p.t; ++i) a |= (uint64_t)((e >> i) & 1) << p.tin[i];
    tile[e + (e >> 5)] = in[a];
  }
  __syncthreads();
  for (int f = threadIdx.x; f < T; f += blockDim.x) {
    uint64_t a = ob;
    int e = 0;
    for (int i = 0; i < p.t; ++i) {
      const int bit = (f >> i) & 1;
      a |= (uint64_t)bit << p.tout[i];
      e |= bit << p.f2e[i];
    }
    out[a] = tile[e + (e >> 5)];
  }
}

hipError_t launch_permute(const Operand& in, const Operand& out, const PermArgs& p, uint64_t s0,
                          int nz, hipStream_t st) {
  const uint64_t blocks = 1ull << p.nn;
  const uint64_t gx = std::min<uint64_t>(blocks, 1ull << 20);
  const uint64_t gy = blocks / gx;
  hipLaunchKernelGGL(stem_permute_kernel, dim3((unsigned)gx, (unsigned)gy, (unsigned)nz),
                     dim3(256), 0, st, in, out, s0, p);
  return hipGetLastError();
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

__device__ __forceinline__ int64_t row_base(int64_t m, const GemmGeom& g) {
  int64_t lo = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) lo |= ((m >> b) & 1ll) << g.mlo[b];
  int64_t a = m >> 4;
#pragma unroll
  for (int i = 0; i < kMaxShared + 4; ++i) {
    if (i < g.nins) {
      const int p = g.ins[i];
      a = ((a >> p) << (p + 1)) | (a & ((1ll << p) - 1));
    }
  }
  return a | lo;
}

__device__ __forceinline__ int64_t k_offset(int k, const GemmGeom& g) {
  int64_t a = 0;
#pragma unroll
  for (int i = 0; i < kMaxShared; ++i)
    if (i < g.s) a |= (int64_t)((k >> i) & 1) << g.spos[i];
  return a;
}

// 4 consecutive reals A[m][kr0 .. kr0+3] (= complex k0 = kr0/2 and k0+1);
// ko0/ko1 are the offsets of those two k values (adjacent in K-low mode).
template <int AM>
__device__ __forceinline__ f32x4 load_kr4(const float* __restrict__ A, int64_t rb, int kr0,
                                          int64_t ko0, int64_t ko1, const GemmGeom& g) {
  f32x4 v = f32x4{0.f, 0.f, 0.f, 0.f};
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

// Store the 4 consecutive reals C[m][nr0 .. nr0+3].
template <int CM>
__device__ __forceinline__ void store_nr4(float* __restrict__ C, int64_t m, int nr0, f32x4 v,
                                          const GemmGeom& g) {
  if (CM == 0) {
    if (nr0 >= g.Nr) return;
    float* dst = C + m * (int64_t)g.Nr + nr0;
    if (g.Nr >= 4)
      *(f32x4*)dst = v;
    else
      *(float2*)dst = float2{v.x, v.y};
  } else {
    const int n0 = nr0 >> 1;
    const int64_t base = ((m >> 4) << (4 + g.f)) | (m & 15);
    if (n0 < g.N) *(float2*)(C + 2 * (base | ((int64_t)n0 << 4))) = float2{v.x, v.y};
    if (n0 + 1 < g.N) *(float2*)(C + 2 * (base | ((int64_t)(n0 + 1) << 4))) = float2{v.z, v.w};
  }
}

// ---------------------------------------------------------------------------
// FP32 product on the 16x16x4 f32 MFMA.
//
// The kernel computes the transposed product C^T = B'^T A^T so that the
// (possibly narrow) 2N real output columns sit on the MFMA's row side and
// the long M side on its column side: lane l owns stem row m = l%16 of a
// 16-row block, and its accumulator holds the 4 consecutive real outputs
// C[m][16 nt + 4 (l/16) + r], r = 0..3.  Summation order inside a 16-wide
// real k chunk is free, so lane group g = l/16 holds the 4 consecutive reals
// A[m][16 kc + 4 g .. +3] and feeds element j to MFMA number j; the branch
// fragments were laid out on the host in the same k order.
//
// Each wave handles TM 16-row blocks (every branch fragment is reused TM
// times) and NTW 16-column tiles; blockIdx.y splits wide outputs.  With
// BLDS the workgroup first copies its branch fragments into LDS; the
// workgroups then loop over the row blocks.
// ---------------------------------------------------------------------------
template <int TM, int NTW, int AM, int CM, int BLDS>
__global__ __launch_bounds__(256) void stem_cgemm_f32_kernel(Operand Ao, Operand Bo, Operand Co,
                                                             uint64_t s0, GemmGeom g) {
  extern __shared__ __align__(16) float sB[];
  const int z = blockIdx.z;
  const float* __restrict__ A = (const float*)op_base(Ao, z, s0);
  const float* __restrict__ Bf = (const float*)(op_base(Bo, z, s0) + kBranchHeader);
  float* __restrict__ C = (float*)op_base(Co, z, s0);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int grp = lane >> 4;
  const int r16 = lane & 15;
  const int nt0 = blockIdx.y * NTW;
  const int ntw = min(NTW, g.NT - nt0);

  if (BLDS) {
    const int per_kc = ntw * 256;
    for (int i = threadIdx.x * 4; i < g.KC * per_kc; i += 1024) {
      const int kc = i / per_kc, r = i - kc * per_kc;
      *(f32x4*)(sB + kc * NTW * 256 + r) = *(const f32x4*)(Bf + (size_t)(kc * g.NT + nt0) * 256 + r);
    }
    __syncthreads();
  }

  const int64_t rows_per_wg = 4 * 16 * TM;
  const int64_t nblk = (g.M + rows_per_wg - 1) / rows_per_wg;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t row0 = (blk * 4 + wave) * (16 * TM);
    if (row0 >= g.M) continue;
    f32x4 acc[TM][NTW];
    int64_t rb[TM];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int64_t row = row0 + t * 16 + r16;
      rb[t] = row < g.M ? row_base(row, g) : -1;
#pragma unroll
      for (int n = 0; n < NTW; ++n) acc[t][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    f32x4 a[TM];
    {
      const int kr0 = grp * 4;
      const int64_t ko0 = k_offset(kr0 >> 1, g);
      const int64_t ko1 = AM == 1 ? k_offset((kr0 >> 1) + 1, g) : 0;
#pragma unroll
      for (int t = 0; t < TM; ++t) a[t] = load_kr4<AM>(A, rb[t], kr0, ko0, ko1, g);
    }
    for (int kc = 0; kc < g.KC; ++kc) {
      // prefetch the next k chunk of A while this one is multiplied
      f32x4 an[TM];
      if (kc + 1 < g.KC) {
        const int kr1 = (kc + 1) * 16 + grp * 4;
        const int64_t ko0 = k_offset(kr1 >> 1, g);
        const int64_t ko1 = AM == 1 ? k_offset((kr1 >> 1) + 1, g) : 0;
#pragma unroll
        for (int t = 0; t < TM; ++t) an[t] = load_kr4<AM>(A, rb[t], kr1, ko0, ko1, g);
      }
#pragma unroll
      for (int n = 0; n < NTW; ++n) {
        if (n < ntw) {
          float b[4];
          if (BLDS) {
            const float* bp = sB + (kc * NTW + n) * 256 + lane;
            b[0] = bp[0]; b[1] = bp[64]; b[2] = bp[128]; b[3] = bp[192];
          } else {
            const float* bp = Bf + ((size_t)(kc * g.NT + nt0 + n) * 4) * 64 + lane;
            b[0] = bp[0]; b[1] = bp[64]; b[2] = bp[128]; b[3] = bp[192];
          }
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int t = 0; t < TM; ++t)
              acc[t][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[j], a[t][j], acc[t][n], 0, 0, 0);
        }
      }
      if (kc + 1 < g.KC) {
#pragma unroll
        for (int t = 0; t < TM; ++t) a[t] = an[t];
      }
    }
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int64_t row = row0 + t * 16 + r16;
      if (row >= g.M) continue;
#pragma unroll
      for (int n = 0; n < NTW; ++n)
        if (n < ntw) store_nr4<CM>(C, row, (nt0 + n) * 16 + grp * 4, acc[t][n], g);
    }
  }
}

size_t bfrag_f32_floats(int64_t K, int64_t N) {
  const int64_t Kp = std::max<int64_t>(16, 2 * K), Np = std::max<int64_t>(16, 2 * N);
  return (size_t)(Kp * Np);
}

size_t bfrag_split_halves(int64_t K, int64_t N) {
  const int64_t Kq = std::max<int64_t>(32, 2 * K), Np = std::max<int64_t>(16, 2 * N);
  return (size_t)(Kq * Np);
}

size_t branch_block_bytes(int precision, int64_t K, int64_t N) {
  size_t body = precision == STEM_FP32 ? bfrag_f32_floats(K, N) * 4 : bfrag_split_halves(K, N) * 4;
  return (kBranchHeader + body + 255) & ~size_t(255);
}

// Expanded real entry B'[kr][nr] of a complex [K x N] matrix b (interleaved).
static inline float expanded(const float* b, int64_t K, int64_t N, int64_t kr, int64_t nr) {
  if (kr >= 2 * K || nr >= 2 * N) return 0.f;
  const int64_t k = kr >> 1, n = nr >> 1;
  const float br = b[2 * (k * N + n)], bi = b[2 * (k * N + n) + 1];
  const int p = (int)(kr & 1), q = (int)(nr & 1);
  if (p == 0) return q == 0 ? br : bi;
  return q == 0 ? -bi : br;
}

void build_bfrag_f32(const float* b, int64_t K, int64_t N, float* out) {
  const int64_t Kp = std::max<int64_t>(16, 2 * K), Np = std::max<int64_t>(16, 2 * N);
  const int64_t KC = Kp / 16, NT = Np / 16;
  for (int64_t kc = 0; kc < KC; ++kc)
    for (int64_t nt = 0; nt < NT; ++nt)
      for (int j = 0; j < 4; ++j)
        for (int lane = 0; lane < 64; ++lane) {
          const int64_t kr = 16 * kc + 4 * (lane >> 4) + j;
          const int64_t nr = 16 * nt + (lane & 15);
          out[((kc * NT + nt) * 4 + j) * 64 + lane] = expanded(b, K, N, kr, nr);
        }
}

static GemmGeom make_geom(const GemmLayout& lay, int64_t M, int64_t K, int64_t N, int kq) {
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
  for (int i = 0; i < 20; ++i) g.ins[i] = lay.ins[i];
  return g;
}

// Schedule with the defaults filled in (see GemmSched).
static GemmSched resolve_sched(const GemmGeom& g, GemmSched s) {
  int nt2 = 1;
  while (nt2 < g.NT) nt2 <<= 1;
  if (s.ntw <= 0) s.ntw = std::min(8, nt2);
  s.ntw = std::min(s.ntw, std::min(8, nt2));
  if (s.tm <= 0) s.tm = s.ntw <= 2 ? 4 : 2;
  if (s.blocks <= 0) s.blocks = kTargetBlocks;
  return s;
}

// Grid of a product launch: x row-block groups (each workgroup loops over
// row blocks when there are more than the target), y column chunks, z slices.
static dim3 gemm_grid(const GemmGeom& g, int TM, int NTW, int nz, int target) {
  const int64_t rows_per_wg = 4 * 16 * TM;
  const int64_t nblk = (g.M + rows_per_wg - 1) / rows_per_wg;
  const int gy = (g.NT + NTW - 1) / NTW;
  const int64_t want = std::max<int64_t>(1, target / ((int64_t)gy * nz));
  const int64_t gx = std::min<int64_t>(nblk, want);
  return dim3((unsigned)gx, (unsigned)gy, (unsigned)nz);
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

template <int TM, int NTW, int AM, int CM>
static void launch_f32_t(const LaunchCtx& c) {
  const dim3 grid = gemm_grid(c.g, TM, NTW, c.nz, c.sch.blocks);
  const size_t lds = (size_t)c.g.KC * NTW * 256 * 4;
  if (lds <= (size_t)kLdsBudget && c.sch.lds != 0)
    hipLaunchKernelGGL((stem_cgemm_f32_kernel<TM, NTW, AM, CM, 1>), grid, dim3(256), lds, c.st,
                       *c.A, *c.B, *c.C, c.s0, c.g);
  else
    hipLaunchKernelGGL((stem_cgemm_f32_kernel<TM, NTW, AM, CM, 0>), grid, dim3(256), 0, c.st,
                       *c.A, *c.B, *c.C, c.s0, c.g);
}

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

template <int AM, int CM>
static void launch_f32_m(const LaunchCtx& c) {
  STEM_TM_NTW_DISPATCH(launch_f32_t, AM, CM)
}

// ---------------------------------------------------------------------------
// Three-term split product on the 16x16x32 f16 / bf16 MFMA, FP32 accumulate.
//
// x = hi + lo with hi = round(x 2^e), lo = round(x 2^e - hi); the product
// keeps hi*hi + hi*lo + lo*hi and drops lo*lo (Markidis et al. 2018, the
// mixed-precision refinement the paper points to for tensor cores).  For
// FP16 every stem row gets its own power-of-two scale 2^e per 32-wide real
// k chunk, from the row's largest magnitude in the chunk, so that the row's
// largest entry lands in [2^13, 2^14); the chunk's partial product is then
// scaled back by 2^-e before it joins the FP32 accumulator.  BF16 has
// FP32's range and uses e = 0.  The branch was split and scaled (2^eb) on
// the host; 2^-eb sits in the variant's header.  Lane layout as in the FP32
// kernel with 8 consecutive reals of k per lane group.
// ---------------------------------------------------------------------------
template <int BF16>
struct SplitT;
template <>
struct SplitT<0> {
  typedef f16x8 vec;
  static __device__ inline uint16_t cvt(float x, float* back) {
    const _Float16 h = (_Float16)x;
    *back = (float)h;
    uint16_t u;
    __builtin_memcpy(&u, &h, 2);
    return u;
  }
  static __device__ inline f32x4 mfma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct SplitT<1> {
  typedef bf16x8 vec;
  static __device__ inline uint16_t cvt(float x, float* back) {
    const __bf16 h = (__bf16)x;
    *back = (float)h;
    uint16_t u;
    __builtin_memcpy(&u, &h, 2);
    return u;
  }
  static __device__ inline f32x4 mfma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <int TM, int NTW, int BF16, int AM, int CM, int BLDS>
__global__ __launch_bounds__(256) void stem_cgemm_split_kernel(Operand Ao, Operand Bo,
                                                               Operand Co, uint64_t s0,
                                                               GemmGeom g) {
  typedef SplitT<BF16> S;
  typedef typename S::vec vec;
  extern __shared__ __align__(16) uint16_t sBh[];
  const int z = blockIdx.z;
  const float* __restrict__ A = (const float*)op_base(Ao, z, s0);
  const char* bblock = op_base(Bo, z, s0);
  const float inv_b = *(const float*)bblock;
  const uint16_t* __restrict__ Bh = (const uint16_t*)(bblock + kBranchHeader);
  const size_t part = (size_t)g.KC * g.NT * 512;  // halves per part (hi or lo)
  const uint16_t* __restrict__ Bl = Bh + part;
  float* __restrict__ C = (float*)op_base(Co, z, s0);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int grp = lane >> 4;
  const int r16 = lane & 15;
  const int nt0 = blockIdx.y * NTW;
  const int ntw = min(NTW, g.NT - nt0);
  uint16_t* sBl = sBh + (size_t)g.KC * NTW * 512;

  if (BLDS) {
    const int per_kc = ntw * 512;  // halves of one part per k chunk
    for (int i = threadIdx.x * 8; i < g.KC * per_kc; i += 2048) {
      const int kc = i / per_kc, r = i - kc * per_kc;
      const size_t src = (size_t)(kc * g.NT + nt0) * 512 + r;
      *(u16x8*)(sBh + kc * NTW * 512 + r) = *(const u16x8*)(Bh + src);
      *(u16x8*)(sBl + kc * NTW * 512 + r) = *(const u16x8*)(Bl + src);
    }
    __syncthreads();
  }

  const int64_t rows_per_wg = 4 * 16 * TM;
  const int64_t nblk = (g.M + rows_per_wg - 1) / rows_per_wg;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t row0 = (blk * 4 + wave) * (16 * TM);
    if (row0 >= g.M) continue;
    f32x4 acc[TM][NTW];
    int64_t rb[TM];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int64_t row = row0 + t * 16 + r16;
      rb[t] = row < g.M ? row_base(row, g) : -1;
#pragma unroll
      for (int n = 0; n < NTW; ++n) acc[t][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    for (int kc = 0; kc < g.KC; ++kc) {
      const int kr0 = kc * 32 + grp * 8;
      int64_t ko[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) ko[i] = k_offset((kr0 >> 1) + i, g);
      vec ahi[TM], alo[TM];
      float inv_a[TM];
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        const f32x4 x0 = load_kr4<AM>(A, rb[t], kr0, ko[0], ko[1], g);
        const f32x4 x1 = load_kr4<AM>(A, rb[t], kr0 + 4, ko[2], ko[3], g);
        const float x[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
        float scale = 1.f;
        inv_a[t] = 1.f;
        if (!BF16) {
          float mx = 0.f;
#pragma unroll
          for (int i = 0; i < 8; ++i) mx = fmaxf(mx, fabsf(x[i]));
          mx = fmaxf(mx, __shfl_xor(mx, 16));
          mx = fmaxf(mx, __shfl_xor(mx, 32));
          if (mx > 0.f) {
            int ex;
            frexpf(mx, &ex);  // mx in [2^(ex-1), 2^ex)
            scale = ldexpf(1.f, 14 - ex);
            inv_a[t] = ldexpf(1.f, ex - 14);
          }
        }
        u16x8 h, l;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float xs = x[i] * scale;
          float back, dummy;
          h[i] = S::cvt(xs, &back);
          l[i] = S::cvt(xs - back, &dummy);
        }
        __builtin_memcpy(&ahi[t], &h, 16);
        __builtin_memcpy(&alo[t], &l, 16);
      }
#pragma unroll
      for (int n = 0; n < NTW; ++n) {
        if (n < ntw) {
          u16x8 bh, bl;
          if (BLDS) {
            const size_t fo = ((size_t)(kc * NTW + n) * 64 + lane) * 8;
            bh = *(const u16x8*)(sBh + fo);
            bl = *(const u16x8*)(sBl + fo);
          } else {
            const size_t fo = ((size_t)(kc * g.NT + nt0 + n) * 64 + lane) * 8;
            bh = *(const u16x8*)(Bh + fo);
            bl = *(const u16x8*)(Bl + fo);
          }
          vec vbh, vbl;
          __builtin_memcpy(&vbh, &bh, 16);
          __builtin_memcpy(&vbl, &bl, 16);
          f32x4 part3[TM];
#pragma unroll
          for (int t = 0; t < TM; ++t) part3[t] = S::mfma(vbh, ahi[t], f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
          for (int t = 0; t < TM; ++t) part3[t] = S::mfma(vbl, ahi[t], part3[t]);
#pragma unroll
          for (int t = 0; t < TM; ++t) part3[t] = S::mfma(vbh, alo[t], part3[t]);
#pragma unroll
          for (int t = 0; t < TM; ++t) acc[t][n] += part3[t] * inv_a[t];
        }
      }
    }
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int64_t row = row0 + t * 16 + r16;
      if (row >= g.M) continue;
#pragma unroll
      for (int n = 0; n < NTW; ++n)
        if (n < ntw) store_nr4<CM>(C, row, (nt0 + n) * 16 + grp * 4, acc[t][n] * inv_b, g);
    }
  }
}

static uint16_t host_f16(float x, float* back) {
  const _Float16 h = (_Float16)x;
  *back = (float)h;
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}

static uint16_t host_bf16(float x, float* back) {
  // round to nearest, ties to even, on the FP32 bit pattern
  uint32_t u;
  std::memcpy(&u, &x, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  const uint32_t r = (u + 0x7FFFu + lsb) >> 16;
  const uint32_t b32 = r << 16;
  std::memcpy(back, &b32, 4);
  return (uint16_t)r;
}

int build_bfrag_split(const float* b, int64_t K, int64_t N, int bf16, uint16_t* out) {
  const int64_t Kq = std::max<int64_t>(32, 2 * K), Np = std::max<int64_t>(16, 2 * N);
  const int64_t KC = Kq / 32, NT = Np / 16;
  const size_t part = (size_t)(Kq * Np);
  int eb = 0;
  if (!bf16) {
    float mx = 0.f;
    for (int64_t i = 0; i < 2 * K * N; ++i) mx = std::max(mx, std::fabs(b[i]));
    if (mx > 0.f) {
      int ex;
      std::frexp(mx, &ex);
      eb = 14 - ex;
    }
  }
  for (int64_t kc = 0; kc < KC; ++kc)
    for (int64_t nt = 0; nt < NT; ++nt)
      for (int lane = 0; lane < 64; ++lane)
        for (int i = 0; i < 8; ++i) {
          const int64_t kr = 32 * kc + 8 * (lane >> 4) + i;
          const int64_t nr = 16 * nt + (lane & 15);
          const float x = std::ldexp(expanded(b, K, N, kr, nr), eb);
          float back, dummy;
          const size_t o = ((size_t)(kc * NT + nt) * 64 + lane) * 8 + i;
          if (bf16) {
            out[o] = host_bf16(x, &back);
            out[part + o] = host_bf16(x - back, &dummy);
          } else {
            out[o] = host_f16(x, &back);
            out[part + o] = host_f16(x - back, &dummy);
          }
        }
  return eb;
}

template <int TM, int NTW, int BF16, int AM, int CM>
static void launch_split_t(const LaunchCtx& c) {
  const dim3 grid = gemm_grid(c.g, TM, NTW, c.nz, c.sch.blocks);
  const size_t lds = (size_t)c.g.KC * NTW * 512 * 2 * 2;
  if (lds <= (size_t)kLdsBudget && c.sch.lds != 0)
    hipLaunchKernelGGL((stem_cgemm_split_kernel<TM, NTW, BF16, AM, CM, 1>), grid, dim3(256), lds,
                       c.st, *c.A, *c.B, *c.C, c.s0, c.g);
  else
    hipLaunchKernelGGL((stem_cgemm_split_kernel<TM, NTW, BF16, AM, CM, 0>), grid, dim3(256), 0,
                       c.st, *c.A, *c.B, *c.C, c.s0, c.g);
}

template <int BF16, int AM, int CM>
static void launch_split_n(const LaunchCtx& c) {
  STEM_TM_NTW_DISPATCH(launch_split_t, BF16, AM, CM)
}

template <int BF16>
static void launch_split_b(const LaunchCtx& c, const GemmLayout& lay) {
  if (lay.amode == 0 && lay.cmode == 0)
    launch_split_n<BF16, 0, 0>(c);
  else if (lay.amode == 0)
    launch_split_n<BF16, 0, 1>(c);
  else if (lay.cmode == 0)
    launch_split_n<BF16, 1, 0>(c);
  else
    launch_split_n<BF16, 1, 1>(c);
}

hipError_t launch_cgemm(int precision, const Operand& A, const Operand& B, const Operand& C,
                        uint64_t s0, int nz, int64_t M, int64_t K, int64_t N,
                        const GemmLayout& lay, const GemmSched& sched, hipStream_t st) {
  LaunchCtx c;
  c.A = &A;
  c.B = &B;
  c.C = &C;
  c.s0 = s0;
  c.nz = nz;
  c.st = st;
  if (precision == STEM_FP32) {
    c.g = make_geom(lay, M, K, N, 16);
    c.sch = resolve_sched(c.g, sched);
    if (lay.amode == 0 && lay.cmode == 0)
      launch_f32_m<0, 0>(c);
    else if (lay.amode == 0)
      launch_f32_m<0, 1>(c);
    else if (lay.cmode == 0)
      launch_f32_m<1, 0>(c);
    else
      launch_f32_m<1, 1>(c);
  } else {
    c.g = make_geom(lay, M, K, N, 32);
    c.sch = resolve_sched(c.g, sched);
    if (precision == STEM_SPLIT_BF16)
      launch_split_b<1>(c, lay);
    else
      launch_split_b<0>(c, lay);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 accumulation of a batch of slices' final stems into the result
// (paper §A.1: the value is the sum of the sliced sub-network values),
// reordered from the stem's final label order into the open-label order.
// One thread per entry adds the batch items in increasing slice order, so
// the sum is deterministic.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void stem_acc_f64_kernel(Operand in_op, uint64_t s0, int nz,
                                                           double2* __restrict__ out, BitMap m,
                                                           uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t o = 0;
  for (int q = 0; q < m.rank; ++q) o |= ((i >> q) & 1ull) << m.dst[q];
  double2 r = out[o];
  for (int z = 0; z < nz; ++z) {
    const float2 v = ((const float2*)op_base(in_op, z, s0))[i];
    r.x += (double)v.x;
    r.y += (double)v.y;
  }
  out[o] = r;
}

hipError_t launch_acc_f64(const Operand& in, uint64_t s0, int nz, double* out, const BitMap& m,
                          hipStream_t st) {
  const uint64_t n = 1ull << m.rank;
  const uint64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(stem_acc_f64_kernel, dim3((unsigned)blocks), dim3(256), 0, st, in, s0, nz,
                     (double2*)out, m, n);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void stem_zero_f64_kernel(double* __restrict__ p, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

hipError_t launch_zero_f64(double* p, uint64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(stem_zero_f64_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Counter-based test tensor: SplitMix64 (Steele, Lea, Flood 2014).  State
// after k+1 steps is seed + (k+1) * golden-gamma; the output is the
// published mixing function of that state.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ int64_t two_fields(uint64_t w) {
  return (int64_t)(w >> 42) + (int64_t)((w >> 10) & 0x3FFFFFull);
}

__global__ __launch_bounds__(256) void stem_fill_counter_kernel(float2* __restrict__ dst,
                                                                uint64_t n, uint64_t seed,
                                                                float scale) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t re = two_fields(splitmix64(seed, 4 * i)) + two_fields(splitmix64(seed, 4 * i + 1)) -
                     (1ll << 23);
  const int64_t im = two_fields(splitmix64(seed, 4 * i + 2)) +
                     two_fields(splitmix64(seed, 4 * i + 3)) - (1ll << 23);
  dst[i] = float2{(float)re * scale, (float)im * scale};
}

hipError_t launch_fill_counter(float* dst, uint64_t n, uint64_t seed, int scale_log2,
                               hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = (n + 255) / 256;
  const unsigned gx = (unsigned)std::min<uint64_t>(blocks, 0x7FFFFFFFull);
  if (blocks > gx) return hipErrorInvalidValue;
  hipLaunchKernelGGL(stem_fill_counter_kernel, dim3(gx), dim3(256), 0, st, (float2*)dst, n, seed,
                     std::ldexp(1.f, -scale_log2));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// XEB in FP64 (paper §2): F = 2^n <|a|^2> - 1.  One workgroup; thread t adds
// entries t, t + 1024, ... in order, then a fixed-shape tree in LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void stem_xeb_f64_kernel(const double2* __restrict__ a,
                                                            uint64_t n, int n_qubits,
                                                            double* __restrict__ out) {
  __shared__ double part[1024];
  double s = 0.0;
  for (uint64_t i = threadIdx.x; i < n; i += 1024) {
    const double2 v = a[i];
    s += v.x * v.x + v.y * v.y;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double tot = part[0];
    out[0] = n ? ldexp(tot / (double)n, n_qubits) - 1.0 : 0.0;
    out[1] = tot;
  }
}

hipError_t launch_xeb_f64(const double* amps, uint64_t n, int n_qubits, double* out,
                          hipStream_t st) {
  hipLaunchKernelGGL(stem_xeb_f64_kernel, dim3(1), dim3(1024), 0, st, (const double2*)amps, n,
                     n_qubits, out);
  return hipGetLastError();
}

}  // namespace stem
