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

// A streams through a ring of R register buffers of raw FP32 chunks, in one
// flat sequence over the wave's row blocks, as in the FP32 kernel: after a
// chunk's MFMAs its buffer is refilled with the chunk R places later (from
// the next row block at the end of the current one; the last row block
// re-reads its own rows), so R - 1 chunks are in flight.
template <int R, int TM, int NTW, int BF16, int AM, int CM, int BLDS, int FULL, int WAVES>
__device__ __forceinline__ void split_rows(const float* __restrict__ A,
                                           const uint16_t* __restrict__ Bh,
                                           const uint16_t* __restrict__ Bl, float inv_b,
                                           float* __restrict__ C, const GemmGeom& g, int wave,
                                           int lane, int nt0, int ntw) {
  typedef SplitT<BF16> S;
  typedef typename S::vec vec;
  const int grp = lane >> 4;
  const int r16 = lane & 15;
  // lane constants: row bits 0..3 and k bits 0..3 (k = 16 kc + 4 grp + i);
  // the chunk's k bits 4.. advance as a bit-spread counter over khmask
  const int64_t rlo = row_lo(r16, g);
  int64_t kl[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) kl[i] = k_offset(4 * grp + i, g);
  const int64_t khmask = k_offset(g.K - 1, g) & ~k_offset(15, g);
  const int64_t rows_per_wg = WAVES * 16 * TM;
  const int64_t nblk = (g.M + rows_per_wg - 1) / rows_per_wg;

  auto block_rows = [&](int64_t blk, int64_t (&rb)[TM]) {
    const int64_t row0 = (blk * WAVES + wave) * (16 * TM);
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int64_t hi = row_hi((row0 >> 4) + t, g);  // wave-uniform
      rb[t] = FULL || row0 + t * 16 + r16 < g.M ? (hi | rlo) : -1;
    }
  };
  auto load_chunk = [&](f32x4 (&dst)[TM][2], const int64_t (&rb)[TM], int kc, int64_t kh) {
    const int kr0 = kc * 32 + grp * 8;
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      dst[t][0] = load_kr4<AM, FULL>(A, rb[t], kr0, kh | kl[0], kh | kl[1], g);
      dst[t][1] = load_kr4<AM, FULL>(A, rb[t], kr0 + 4, kh | kl[2], kh | kl[3], g);
    }
  };

  int64_t blk = blockIdx.x;
  if ((blk * WAVES + wave) * (16 * TM) >= g.M) return;  // no barrier follows
  int64_t rb[TM];
  block_rows(blk, rb);
  f32x4 buf[R][TM][2];
  int64_t kh = 0;  // k offset of the chunk loaded last
#pragma unroll
  for (int i = 0; i < R; ++i) {
    if (i > 0) kh = spread_next(kh, khmask);
    load_chunk(buf[i], rb, i, kh);
  }
  while (true) {
    const int64_t row0 = (blk * WAVES + wave) * (16 * TM);
    const int64_t nxt = blk + gridDim.x;
    const bool has_next = nxt < nblk && (FULL || (nxt * WAVES + wave) * (16 * TM) < g.M);
    int64_t rbn[TM];
    if (has_next)
      block_rows(nxt, rbn);
    else
#pragma unroll
      for (int t = 0; t < TM; ++t) rbn[t] = rb[t];
    f32x4 acc[TM][NTW];
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
      for (int n = 0; n < NTW; ++n) acc[t][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < g.KC; kc += R) {
      const bool tail = kc + R >= g.KC;  // refills come from the next row block
#pragma unroll
      for (int i = 0; i < R; ++i) {
        vec ahi[TM], alo[TM];
        float inv_a[TM];
#pragma unroll
        for (int t = 0; t < TM; ++t) {
          const f32x4 x0 = buf[i][t][0], x1 = buf[i][t][1];
          const float x[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
          float scale = 1.f;
          inv_a[t] = 1.f;
          if (!BF16) {
            float mx = 0.f;
#pragma unroll
            for (int e = 0; e < 8; ++e) mx = fmaxf(mx, fabsf(x[e]));
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
          for (int e = 0; e < 8; ++e) {
            const float xs = x[e] * scale;
            float back, dummy;
            h[e] = S::cvt(xs, &back);
            l[e] = S::cvt(xs - back, &dummy);
          }
          __builtin_memcpy(&ahi[t], &h, 16);
          __builtin_memcpy(&alo[t], &l, 16);
        }
        // the raw chunk is converted: refill its buffer now
        kh = spread_next(kh, khmask);
        {
          int64_t rl[TM];
#pragma unroll
          for (int t = 0; t < TM; ++t) rl[t] = tail ? rbn[t] : rb[t];
          load_chunk(buf[i], rl, (kc + i + R) & (g.KC - 1), kh);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int n = 0; n < NTW; ++n) {
          if (n < ntw) {
            const size_t fo = BLDS ? ((size_t)((kc + i) * NTW + n) * 64 + lane) * 8
                                   : ((size_t)((kc + i) * g.NT + nt0 + n) * 64 + lane) * 8;
            const u16x8 bh = *(const u16x8*)(Bh + fo);
            const u16x8 bl = *(const u16x8*)(Bl + fo);
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
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int64_t row = row0 + t * 16 + r16;
      if (!FULL && row >= g.M) continue;
#pragma unroll
      for (int n = 0; n < NTW; ++n)
        if (n < ntw)
          store_nr4<CM, FULL>(C, row, (nt0 + n) * 16 + grp * 4, acc[t][n] * inv_b, g);
    }
    if (!has_next) break;
    blk = nxt;
#pragma unroll
    for (int t = 0; t < TM; ++t) rb[t] = rbn[t];
  }
}

template <int TM, int NTW, int BF16, int AM, int CM, int BLDS, int FULL, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void stem_cgemm_split_kernel(Operand Ao, Operand Bo,
                                                               Operand Co, uint64_t s0,
                                                               GemmGeom g) {
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
  const int nt0 = blockIdx.y * NTW;
  // FULL: every tile of the launch is whole (gemm_full), no predicates
  const int ntw = FULL ? NTW : min(NTW, g.NT - nt0);
  uint16_t* sBl = sBh + (size_t)g.KC * NTW * 512;

  if (BLDS) {
    const int per_kc = ntw * 512;  // halves of one part per k chunk
    for (int i = threadIdx.x * 8; i < g.KC * per_kc; i += 512 * WAVES) {
      const int kc = i / per_kc, r = i - kc * per_kc;
      const size_t src = (size_t)(kc * g.NT + nt0) * 512 + r;
      *(u16x8*)(sBh + kc * NTW * 512 + r) = *(const u16x8*)(Bh + src);
      *(u16x8*)(sBl + kc * NTW * 512 + r) = *(const u16x8*)(Bl + src);
    }
    __syncthreads();
  }
  const uint16_t* Bhs = BLDS ? (const uint16_t*)sBh : Bh;
  const uint16_t* Bls = BLDS ? (const uint16_t*)sBl : Bl;
  // KC is a power of two; the ring holds min(2, KC) chunks of 32 reals per
  // row (one for the small partial shapes that run without FULL)
  if constexpr (FULL) {
    if (g.KC >= 2)
      split_rows<2, TM, NTW, BF16, AM, CM, BLDS, FULL, WAVES>(A, Bhs, Bls, inv_b, C, g, wave,
                                                              lane, nt0, ntw);
    else
      split_rows<1, TM, NTW, BF16, AM, CM, BLDS, FULL, WAVES>(A, Bhs, Bls, inv_b, C, g, wave,
                                                              lane, nt0, ntw);
  } else {
    split_rows<1, TM, NTW, BF16, AM, CM, BLDS, FULL, WAVES>(A, Bhs, Bls, inv_b, C, g, wave, lane,
                                                            nt0, ntw);
  }
}

template <int TM, int NTW, int BF16, int AM, int CM, int FULL>
static void launch_split_f(const LaunchCtx& c, const dim3& grid) {
  const size_t lds = (size_t)c.g.KC * NTW * 512 * 2 * 2;
  static size_t allowed = 0, allowed_w8 = 0;
  if constexpr (FULL) {
    // lds 2: fragments in LDS shared by 8-wave workgroups (two waves per SIMD)
    if (c.sch.lds == 2 && c.g.M % (128 * TM) == 0 && use_lds(1, lds) &&
        allow_lds(stem_cgemm_split_kernel<TM, NTW, BF16, AM, CM, 1, FULL, 8>, lds, &allowed_w8) ==
            hipSuccess) {
      const int64_t nblk = c.g.M / (128 * TM);
      const dim3 g8((unsigned)std::max<int64_t>(1, std::min<int64_t>(nblk, (grid.x + 1) / 2)),
                    grid.y, grid.z);
      hipLaunchKernelGGL((stem_cgemm_split_kernel<TM, NTW, BF16, AM, CM, 1, FULL, 8>), g8,
                         dim3(512), lds, c.st, *c.A, *c.B, *c.C, c.s0, c.g);
      return;
    }
  }
  if (use_lds(c.sch.lds == 2 ? 1 : c.sch.lds, lds) &&
      allow_lds(stem_cgemm_split_kernel<TM, NTW, BF16, AM, CM, 1, FULL, 4>, lds, &allowed) ==
          hipSuccess)
    hipLaunchKernelGGL((stem_cgemm_split_kernel<TM, NTW, BF16, AM, CM, 1, FULL, 4>), grid,
                       dim3(256), lds, c.st, *c.A, *c.B, *c.C, c.s0, c.g);
  else
    hipLaunchKernelGGL((stem_cgemm_split_kernel<TM, NTW, BF16, AM, CM, 0, FULL, 4>), grid,
                       dim3(256), 0, c.st, *c.A, *c.B, *c.C, c.s0, c.g);
}

// Whole shapes run the requested schedule without predicates; partial ones
// run one generic predicated kernel with one row block per wave.
template <int TM, int NTW, int BF16, int AM, int CM>
static void launch_split_t(const LaunchCtx& c) {
  if constexpr (CM == 1) {
    if (gemm_full(c.g, TM, NTW, CM, 32)) {
      launch_split_f<TM, NTW, BF16, AM, CM, 1>(c, gemm_grid(c.g, TM, NTW, c.nz, c.sch.blocks));
      return;
    }
  }
  launch_split_f<1, NTW, BF16, AM, CM, 0>(c, gemm_grid(c.g, 1, NTW, c.nz, c.sch.blocks));
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
