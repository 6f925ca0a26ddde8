// Three-term split FP16 / BF16 complex product of a stem step on the
// gfx950 matrix cores.

#include "device_common.h"

namespace stem {

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
  const int wave = wave_id();
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

  // lane constants: row bits 0..3 and k bits 0..3 (k = 16 kc + 4 grp + i)
  const int64_t rlo = row_lo(r16, g);
  int64_t kl[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) kl[i] = k_offset(4 * grp + i, g);

  // The wave's row blocks are blk = blockIdx.x, + gridDim.x, ...; the raw
  // A values of the chunk after the current one are always in flight, also
  // across the boundary from one row block to the next.
  const int64_t rows_per_wg = 4 * 16 * TM;
  const int64_t nblk = (g.M + rows_per_wg - 1) / rows_per_wg;
  int64_t blk = blockIdx.x;
  if ((blk * 4 + wave) * (16 * TM) >= g.M) return;  // no barrier follows
  int64_t rb[TM];
  f32x4 x0[TM], x1[TM];
#pragma unroll
  for (int t = 0; t < TM; ++t) {
    const int64_t row0 = (blk * 4 + wave) * (16 * TM);
    const int64_t hi = row_hi((row0 >> 4) + t, g);  // wave-uniform
    rb[t] = row0 + t * 16 + r16 < g.M ? (hi | rlo) : -1;
    x0[t] = load_kr4<AM>(A, rb[t], grp * 8, kl[0], kl[1], g);
    x1[t] = load_kr4<AM>(A, rb[t], grp * 8 + 4, kl[2], kl[3], g);
  }
  while (true) {
    const int64_t row0 = (blk * 4 + wave) * (16 * TM);
    const int64_t nxt = blk + gridDim.x;
    const int64_t row0n = (nxt * 4 + wave) * (16 * TM);
    const bool has_next = nxt < nblk && row0n < g.M;
    f32x4 acc[TM][NTW];
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
      for (int n = 0; n < NTW; ++n) acc[t][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    int64_t rbn[TM];
    for (int kc = 0; kc < g.KC; ++kc) {
      f32x4 y0[TM], y1[TM];
      if (kc + 1 < g.KC) {
        const int kr0 = (kc + 1) * 32 + grp * 8;
        const int64_t kh = k_offset(16 * (kc + 1), g);  // wave-uniform
#pragma unroll
        for (int t = 0; t < TM; ++t) {
          y0[t] = load_kr4<AM>(A, rb[t], kr0, kh | kl[0], kh | kl[1], g);
          y1[t] = load_kr4<AM>(A, rb[t], kr0 + 4, kh | kl[2], kh | kl[3], g);
        }
      } else if (has_next) {
#pragma unroll
        for (int t = 0; t < TM; ++t) {
          const int64_t hi = row_hi((row0n >> 4) + t, g);
          rbn[t] = row0n + t * 16 + r16 < g.M ? (hi | rlo) : -1;
          y0[t] = load_kr4<AM>(A, rbn[t], grp * 8, kl[0], kl[1], g);
          y1[t] = load_kr4<AM>(A, rbn[t], grp * 8 + 4, kl[2], kl[3], g);
        }
      }
      vec ahi[TM], alo[TM];
      float inv_a[TM];
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        const float x[8] = {x0[t].x, x0[t].y, x0[t].z, x0[t].w,
                            x1[t].x, x1[t].y, x1[t].z, x1[t].w};
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
          if (BF16) {
            // no scale: the three products accumulate in place
#pragma unroll
            for (int t = 0; t < TM; ++t) acc[t][n] = S::mfma(vbh, ahi[t], acc[t][n]);
#pragma unroll
            for (int t = 0; t < TM; ++t) acc[t][n] = S::mfma(vbl, ahi[t], acc[t][n]);
#pragma unroll
            for (int t = 0; t < TM; ++t) acc[t][n] = S::mfma(vbh, alo[t], acc[t][n]);
          } else {
            f32x4 part3[TM];
#pragma unroll
            for (int t = 0; t < TM; ++t)
              part3[t] = S::mfma(vbh, ahi[t], f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int t = 0; t < TM; ++t) part3[t] = S::mfma(vbl, ahi[t], part3[t]);
#pragma unroll
            for (int t = 0; t < TM; ++t) part3[t] = S::mfma(vbh, alo[t], part3[t]);
#pragma unroll
            for (int t = 0; t < TM; ++t) acc[t][n] += part3[t] * inv_a[t];
          }
        }
      }
      if (kc + 1 < g.KC || has_next) {
#pragma unroll
        for (int t = 0; t < TM; ++t) {
          x0[t] = y0[t];
          x1[t] = y1[t];
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
    if (!has_next) break;
    blk = nxt;
#pragma unroll
    for (int t = 0; t < TM; ++t) rb[t] = rbn[t];
  }
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

void launch_gemm_split(const LaunchCtx& c, const GemmLayout& lay, int bf16) {
  if (bf16)
    launch_split_b<1>(c, lay);
  else
    launch_split_b<0>(c, lay);
}

}  // namespace stem
