// FP32 complex product of a stem step on the gfx950 matrix cores.

#include "device_common.h"

namespace stem {

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
//
// A streams through a ring of R register buffers, one k chunk each, in one
// flat sequence over the wave's row blocks: right after the MFMAs of a
// chunk, its buffer is refilled with the chunk R places later (in the next
// row block once the current one runs out), so R - 1 chunks are always in
// flight.  The refill is issued unconditionally (the last row block
// re-reads its own rows) so that every path issues the loads in the same
// order and the memory-counter waits stay exact.
// ---------------------------------------------------------------------------
template <int R, int TM, int NTW, int AM, int CM, int BLDS, int FULL>
__device__ __forceinline__ void f32_rows(const float* __restrict__ A,
                                         const float* __restrict__ Bsrc, float* __restrict__ C,
                                         const GemmGeom& g, int wave, int lane, int nt0, int ntw) {
  const int grp = lane >> 4;
  const int r16 = lane & 15;
  // lane constants: row bits 0..3 and k bits 0..2 (k = 8 kc + 2 grp + i);
  // the chunk's k bits 3.. advance as a bit-spread counter over khmask,
  // which wraps to chunk 0 after the last one
  const int64_t rlo = row_lo(r16, g);
  const int64_t kl0 = k_offset(2 * grp, g);
  const int64_t kl1 = k_offset(2 * grp + 1, g);
  const int64_t khmask = k_offset(g.K - 1, g) & ~k_offset(7, g);
  const int64_t rows_per_wg = 4 * 16 * TM;
  const int64_t nblk = (g.M + rows_per_wg - 1) / rows_per_wg;

  auto block_rows = [&](int64_t blk, int64_t (&rb)[TM]) {
    const int64_t row0 = (blk * 4 + wave) * (16 * TM);
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int64_t hi = row_hi((row0 >> 4) + t, g);  // wave-uniform
      rb[t] = FULL || row0 + t * 16 + r16 < g.M ? (hi | rlo) : -1;
    }
  };
  auto load_chunk = [&](f32x4 (&dst)[TM], const int64_t (&rb)[TM], int kc, int64_t kh) {
#pragma unroll
    for (int t = 0; t < TM; ++t)
      dst[t] = load_kr4<AM, FULL>(A, rb[t], kc * 16 + grp * 4, kh | kl0, kh | kl1, g);
  };

  auto load_b = [&](float (&dst)[NTW][4], int kc) {
#pragma unroll
    for (int n = 0; n < NTW; ++n) {
      if (n < ntw) {
        const float* bp = BLDS ? Bsrc + (kc * NTW + n) * 256 + lane
                               : Bsrc + ((size_t)(kc * g.NT + nt0 + n) * 4) * 64 + lane;
        dst[n][0] = bp[0];
        dst[n][1] = bp[64];
        dst[n][2] = bp[128];
        dst[n][3] = bp[192];
      }
    }
  };

  int64_t blk = blockIdx.x;
  if ((blk * 4 + wave) * (16 * TM) >= g.M) return;  // no barrier follows
  int64_t rb[TM];
  block_rows(blk, rb);
  float bq[2][NTW][4];
  if (R >= 2) load_b(bq[0], 0);
  f32x4 buf[R][TM];
  int64_t kh = 0;  // k offset of the chunk loaded last
#pragma unroll
  for (int i = 0; i < R; ++i) {
    if (i > 0) kh = spread_next(kh, khmask);
    load_chunk(buf[i], rb, i, kh);
  }
  while (true) {
    const int64_t row0 = (blk * 4 + wave) * (16 * TM);
    const int64_t nxt = blk + gridDim.x;
    const bool has_next = nxt < nblk && (FULL || (nxt * 4 + wave) * (16 * TM) < g.M);
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
        // the branch fragments of the chunk: prefetched one chunk ahead into
        // the other half of bq when the ring holds an even number of chunks
        // (chunk parity = i parity), else loaded here
        float b[NTW][4];
        if (R >= 2) {
          const int nk = (kc + i + 1) & (g.KC - 1);
#pragma unroll
          for (int n = 0; n < NTW; ++n)
#pragma unroll
            for (int q = 0; q < 4; ++q) b[n][q] = bq[i & 1][n][q];
          load_b(bq[(i + 1) & 1], nk);
        } else {
          load_b(b, kc + i);
        }
        // the MFMAs ordered so that TM * NTW independent accumulators
        // separate two dependent ones
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int n = 0; n < NTW; ++n)
            if (n < ntw) {
#pragma unroll
              for (int t = 0; t < TM; ++t)
                acc[t][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[n][j], buf[i][t][j], acc[t][n],
                                                                 0, 0, 0);
            }
        kh = spread_next(kh, khmask);
        int64_t rl[TM];
#pragma unroll
        for (int t = 0; t < TM; ++t) rl[t] = tail ? rbn[t] : rb[t];
        load_chunk(buf[i], rl, (kc + i + R) & (g.KC - 1), kh);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int64_t row = row0 + t * 16 + r16;
      if (!FULL && row >= g.M) continue;
#pragma unroll
      for (int n = 0; n < NTW; ++n)
        if (n < ntw) store_nr4<CM, FULL>(C, row, (nt0 + n) * 16 + grp * 4, acc[t][n], g);
    }
    if (!has_next) break;
    blk = nxt;
#pragma unroll
    for (int t = 0; t < TM; ++t) rb[t] = rbn[t];
  }
}

template <int TM, int NTW, int AM, int CM, int BLDS, int FULL>
__global__ __launch_bounds__(256) void stem_cgemm_f32_kernel(Operand Ao, Operand Bo, Operand Co,
                                                             uint64_t s0, GemmGeom g) {
  extern __shared__ __align__(16) float sB[];
  const int z = blockIdx.z;
  const float* __restrict__ A = (const float*)op_base(Ao, z, s0);
  const float* __restrict__ Bf = (const float*)(op_base(Bo, z, s0) + kBranchHeader);
  float* __restrict__ C = (float*)op_base(Co, z, s0);
  const int lane = threadIdx.x & 63;
  const int wave = wave_id();
  const int nt0 = blockIdx.y * NTW;
  // FULL: every tile of the launch is whole (gemm_full), no predicates
  const int ntw = FULL ? NTW : min(NTW, g.NT - nt0);

  if (BLDS) {
    const int per_kc = ntw * 256;
    for (int i = threadIdx.x * 4; i < g.KC * per_kc; i += 1024) {
      const int kc = i / per_kc, r = i - kc * per_kc;
      *(f32x4*)(sB + kc * NTW * 256 + r) = *(const f32x4*)(Bf + (size_t)(kc * g.NT + nt0) * 256 + r);
    }
    __syncthreads();
  }
  const float* Bsrc = BLDS ? (const float*)sB : Bf;
  // KC is a power of two; the ring holds min(4, KC) chunks (one for the
  // small partial shapes that run without FULL)
  if constexpr (FULL) {
    if (g.KC >= 4)
      f32_rows<4, TM, NTW, AM, CM, BLDS, FULL>(A, Bsrc, C, g, wave, lane, nt0, ntw);
    else if (g.KC == 2)
      f32_rows<2, TM, NTW, AM, CM, BLDS, FULL>(A, Bsrc, C, g, wave, lane, nt0, ntw);
    else
      f32_rows<1, TM, NTW, AM, CM, BLDS, FULL>(A, Bsrc, C, g, wave, lane, nt0, ntw);
  } else {
    f32_rows<1, TM, NTW, AM, CM, BLDS, FULL>(A, Bsrc, C, g, wave, lane, nt0, ntw);
  }
}

template <int TM, int NTW, int AM, int CM, int FULL>
static void launch_f32_f(const LaunchCtx& c, const dim3& grid) {
  const size_t lds = (size_t)c.g.KC * NTW * 256 * 4;
  static size_t allowed = 0;
  if (use_lds(c.sch.lds, lds) &&
      allow_lds(stem_cgemm_f32_kernel<TM, NTW, AM, CM, 1, FULL>, lds, &allowed) == hipSuccess)
    hipLaunchKernelGGL((stem_cgemm_f32_kernel<TM, NTW, AM, CM, 1, FULL>), grid, dim3(256), lds,
                       c.st, *c.A, *c.B, *c.C, c.s0, c.g);
  else
    hipLaunchKernelGGL((stem_cgemm_f32_kernel<TM, NTW, AM, CM, 0, FULL>), grid, dim3(256), 0,
                       c.st, *c.A, *c.B, *c.C, c.s0, c.g);
}

// Whole shapes run the requested schedule without predicates; partial ones
// (small M, K or N) run one generic predicated kernel with one row block
// per wave.
template <int TM, int NTW, int AM, int CM>
static void launch_f32_t(const LaunchCtx& c) {
  if constexpr (CM == 1) {
    if (gemm_full(c.g, TM, NTW, CM, 16)) {
      launch_f32_f<TM, NTW, AM, CM, 1>(c, gemm_grid(c.g, TM, NTW, c.nz, c.sch.blocks));
      return;
    }
  }
  launch_f32_f<1, NTW, AM, CM, 0>(c, gemm_grid(c.g, 1, NTW, c.nz, c.sch.blocks));
}

template <int AM, int CM>
static void launch_f32_m(const LaunchCtx& c) {
  STEM_TM_NTW_DISPATCH(launch_f32_t, AM, CM)
}
// ---------------------------------------------------------------------------
// FP32 product with three real products per complex one (the 3M method,
// Higham 1992): with a = x + iy and b = c + id,
//   Re(ab) = xc - yd,  Im(ab) = (x + y)(c + d) - xc - yd,
// so P1 = X C, P2 = Y D and P3 = (X + Y)(C + D) give the complex product
// with 3/4 of the real embedding's MFMA work.  Lane (r16, grp) loads the
// same 4 reals as above (complex k = 8 kc + 2 grp + j, j = 0, 1) and feeds
// x_j, y_j and x_j + y_j to the three products; the branch fragments hold
// C, D and C + D for 16 complex output columns per tile, 6 per k chunk
// ([kc][tile][j][C, D, C + D][64 lanes], after the real-embedding
// fragments).  Lane (r16, grp) accumulates complex columns 4 grp + r of its
// tile for row r16 and writes them as 8 consecutive reals.  Whole shapes
// only: M a multiple of 64 TM, K of 8, N of 16, output in block order.
// PF: the next chunk's fragments are loaded into registers one chunk ahead
// (without PF they are read where they are used, which saves 6 NTC
// registers and suits fragments in LDS).  WAVES: waves per workgroup (4, or
// 8 so that two waves per SIMD share one LDS copy of large fragments).
// ---------------------------------------------------------------------------
template <int R, int TM, int NTC, int AM, int BLDS, int PF, int WAVES>
__device__ __forceinline__ void f32g_rows(const float* __restrict__ A,
                                          const float* __restrict__ Bsrc, float* __restrict__ C,
                                          const GemmGeom& g, int wave, int lane, int ct0) {
  const int grp = lane >> 4;
  const int r16 = lane & 15;
  const int64_t rlo = row_lo(r16, g);
  const int64_t kl0 = k_offset(2 * grp, g);
  const int64_t kl1 = k_offset(2 * grp + 1, g);
  const int64_t khmask = k_offset(g.K - 1, g) & ~k_offset(7, g);
  const int64_t nblk = g.M / (16 * WAVES * TM);
  const int ntc_all = g.NT >> 1;

  auto block_rows = [&](int64_t blk, int64_t (&rb)[TM]) {
    const int64_t row0 = (blk * WAVES + wave) * (16 * TM);
#pragma unroll
    for (int t = 0; t < TM; ++t) rb[t] = row_hi((row0 >> 4) + t, g) | rlo;
  };
  auto load_chunk = [&](f32x4 (&dst)[TM], const int64_t (&rb)[TM], int kc, int64_t kh) {
#pragma unroll
    for (int t = 0; t < TM; ++t)
      dst[t] = load_kr4<AM, 1>(A, rb[t], kc * 16 + grp * 4, kh | kl0, kh | kl1, g);
  };
  auto load_b = [&](float (&dst)[NTC][6], int kc) {
#pragma unroll
    for (int n = 0; n < NTC; ++n) {
      const float* bp = BLDS ? Bsrc + (kc * NTC + n) * 384 + lane
                             : Bsrc + (size_t)(kc * ntc_all + ct0 + n) * 384 + lane;
#pragma unroll
      for (int q = 0; q < 6; ++q) dst[n][q] = bp[64 * q];
    }
  };

  int64_t blk = blockIdx.x;
  if (blk >= nblk) return;  // no barrier follows
  int64_t rb[TM];
  block_rows(blk, rb);
  constexpr bool kPre = PF && R >= 2;
  float bq[kPre ? 2 : 1][NTC][6];
  if (kPre) load_b(bq[0], 0);
  f32x4 buf[R][TM];
  int64_t kh = 0;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    if (i > 0) kh = spread_next(kh, khmask);
    load_chunk(buf[i], rb, i, kh);
  }
  while (true) {
    const int64_t row0 = (blk * WAVES + wave) * (16 * TM);
    const int64_t nxt = blk + gridDim.x;
    const bool has_next = nxt < nblk;
    int64_t rbn[TM];
    if (has_next)
      block_rows(nxt, rbn);
    else
#pragma unroll
      for (int t = 0; t < TM; ++t) rbn[t] = rb[t];
    f32x4 p1[TM][NTC], p2[TM][NTC], p3[TM][NTC];
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
      for (int n = 0; n < NTC; ++n) {
        p1[t][n] = f32x4{0.f, 0.f, 0.f, 0.f};
        p2[t][n] = p1[t][n];
        p3[t][n] = p1[t][n];
      }
    for (int kc = 0; kc < g.KC; kc += R) {
      const bool tail = kc + R >= g.KC;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        float b[NTC][6];
        if constexpr (kPre) {
          const int nk = (kc + i + 1) & (g.KC - 1);
#pragma unroll
          for (int n = 0; n < NTC; ++n)
#pragma unroll
            for (int q = 0; q < 6; ++q) b[n][q] = bq[i & 1][n][q];
          load_b(bq[(i + 1) & 1], nk);
        } else {
          load_b(b, kc + i);
        }
        float xs[TM][2], ys[TM][2], ss[TM][2];
#pragma unroll
        for (int t = 0; t < TM; ++t) {
          xs[t][0] = buf[i][t][0];
          ys[t][0] = buf[i][t][1];
          xs[t][1] = buf[i][t][2];
          ys[t][1] = buf[i][t][3];
          ss[t][0] = xs[t][0] + ys[t][0];
          ss[t][1] = xs[t][1] + ys[t][1];
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int n = 0; n < NTC; ++n)
#pragma unroll
            for (int t = 0; t < TM; ++t) {
              p1[t][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[n][3 * j], xs[t][j], p1[t][n],
                                                              0, 0, 0);
              p2[t][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[n][3 * j + 1], ys[t][j],
                                                              p2[t][n], 0, 0, 0);
              p3[t][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[n][3 * j + 2], ss[t][j],
                                                              p3[t][n], 0, 0, 0);
            }
        kh = spread_next(kh, khmask);
        int64_t rl[TM];
#pragma unroll
        for (int t = 0; t < TM; ++t) rl[t] = tail ? rbn[t] : rb[t];
        load_chunk(buf[i], rl, (kc + i + R) & (g.KC - 1), kh);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int64_t row = row0 + t * 16 + r16;
#pragma unroll
      for (int n = 0; n < NTC; ++n) {
        f32x4 re, im;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          re[r] = p1[t][n][r] - p2[t][n][r];
          im[r] = p3[t][n][r] - p1[t][n][r] - p2[t][n][r];
        }
        const int col = (ct0 + n) * 32 + grp * 8;
        store_nr4<1, 1>(C, row, col, f32x4{re[0], im[0], re[1], im[1]}, g);
        store_nr4<1, 1>(C, row, col + 4, f32x4{re[2], im[2], re[3], im[3]}, g);
      }
    }
    if (!has_next) break;
    blk = nxt;
#pragma unroll
    for (int t = 0; t < TM; ++t) rb[t] = rbn[t];
  }
}

template <int TM, int NTC, int AM, int BLDS, int PF, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void stem_cgemm_f32g_kernel(Operand Ao, Operand Bo, Operand Co,
                                                              uint64_t s0, GemmGeom g) {
  extern __shared__ __align__(16) float sB[];
  const int z = blockIdx.z;
  const float* __restrict__ A = (const float*)op_base(Ao, z, s0);
  // the 3M fragments follow the real-embedding ones (2K x 2N reals)
  const float* __restrict__ Bf = (const float*)(op_base(Bo, z, s0) + kBranchHeader) +
                                 (size_t)g.Kr * g.Nr;
  float* __restrict__ C = (float*)op_base(Co, z, s0);
  const int lane = threadIdx.x & 63;
  const int wave = wave_id();
  const int ct0 = blockIdx.y * NTC;
  const int ntc_all = g.NT >> 1;
  if (BLDS) {
    const int per_kc = NTC * 384;
    for (int i = threadIdx.x * 4; i < g.KC * per_kc; i += 256 * WAVES) {
      const int kc = i / per_kc, r = i - kc * per_kc;
      *(f32x4*)(sB + kc * per_kc + r) = *(const f32x4*)(Bf + (size_t)(kc * ntc_all + ct0) * 384 + r);
    }
    __syncthreads();
  }
  const float* Bsrc = BLDS ? (const float*)sB : Bf;
  if (g.KC >= 4)
    f32g_rows<4, TM, NTC, AM, BLDS, PF, WAVES>(A, Bsrc, C, g, wave, lane, ct0);
  else if (g.KC == 2)
    f32g_rows<2, TM, NTC, AM, BLDS, PF, WAVES>(A, Bsrc, C, g, wave, lane, ct0);
  else
    f32g_rows<1, TM, NTC, AM, BLDS, PF, WAVES>(A, Bsrc, C, g, wave, lane, ct0);
}

template <int TM, int NTC, int AM>
static void launch_f32g_t(const LaunchCtx& c) {
  const int ntc_all = c.g.NT >> 1;
  const int gy = ntc_all / NTC;
  const int64_t want = std::max<int64_t>(1, c.sch.blocks / ((int64_t)gy * c.nz));
  auto grid = [&](int waves) {
    const int64_t nblk = c.g.M / (16 * waves * TM);
    return dim3((unsigned)std::min<int64_t>(nblk, want), (unsigned)gy, (unsigned)c.nz);
  };
  // lds -1: fragments in LDS up to 64 KB, prefetched into registers;
  // lds 1: in LDS up to the device limit, read where used; lds 2: as 1
  // with 8-wave workgroups; lds 3: in LDS up to the device limit,
  // prefetched, 8-wave workgroups; else global, prefetched
  const size_t lds = (size_t)c.g.KC * NTC * 384 * 4;
  static size_t allowed_pf = 0, allowed_np = 0, allowed_w8 = 0, allowed_w8pf = 0;
  const bool w8 = c.g.M % (128 * TM) == 0 && use_lds(1, lds);
  if (c.sch.lds == 3 && w8 &&
      allow_lds(stem_cgemm_f32g_kernel<TM, NTC, AM, 1, 1, 8>, lds, &allowed_w8pf) == hipSuccess)
    hipLaunchKernelGGL((stem_cgemm_f32g_kernel<TM, NTC, AM, 1, 1, 8>), grid(8), dim3(512), lds,
                       c.st, *c.A, *c.B, *c.C, c.s0, c.g);
  else if (c.sch.lds == 2 && w8 &&
           allow_lds(stem_cgemm_f32g_kernel<TM, NTC, AM, 1, 0, 8>, lds, &allowed_w8) == hipSuccess)
    hipLaunchKernelGGL((stem_cgemm_f32g_kernel<TM, NTC, AM, 1, 0, 8>), grid(8), dim3(512), lds,
                       c.st, *c.A, *c.B, *c.C, c.s0, c.g);
  else if (c.sch.lds >= 1 && use_lds(1, lds) &&
           allow_lds(stem_cgemm_f32g_kernel<TM, NTC, AM, 1, 0, 4>, lds, &allowed_np) == hipSuccess)
    hipLaunchKernelGGL((stem_cgemm_f32g_kernel<TM, NTC, AM, 1, 0, 4>), grid(4), dim3(256), lds,
                       c.st, *c.A, *c.B, *c.C, c.s0, c.g);
  else if (c.sch.lds == -1 && use_lds(-1, lds) &&
           allow_lds(stem_cgemm_f32g_kernel<TM, NTC, AM, 1, 1, 4>, lds, &allowed_pf) == hipSuccess)
    hipLaunchKernelGGL((stem_cgemm_f32g_kernel<TM, NTC, AM, 1, 1, 4>), grid(4), dim3(256), lds,
                       c.st, *c.A, *c.B, *c.C, c.s0, c.g);
  else
    hipLaunchKernelGGL((stem_cgemm_f32g_kernel<TM, NTC, AM, 0, 1, 4>), grid(4), dim3(256), 0,
                       c.st, *c.A, *c.B, *c.C, c.s0, c.g);
}

template <int AM>
static void launch_f32g_m(const LaunchCtx& c) {
  // at most 4 (row block, tile) pairs per wave: three accumulators each
  switch (c.sch.tm * 16 + c.sch.ntw) {
    case 16 + 1: launch_f32g_t<1, 1, AM>(c); break;
    case 16 + 2: launch_f32g_t<1, 2, AM>(c); break;
    case 16 + 4: launch_f32g_t<1, 4, AM>(c); break;
    case 32 + 1: launch_f32g_t<2, 1, AM>(c); break;
    case 32 + 2: launch_f32g_t<2, 2, AM>(c); break;
    default: launch_f32g_t<4, 1, AM>(c); break;
  }
}

void launch_gemm_f32g(const LaunchCtx& c, const GemmLayout& lay) {
  if (lay.amode == 0)
    launch_f32g_m<0>(c);
  else
    launch_f32g_m<1>(c);
}

void launch_gemm_f32(const LaunchCtx& c, const GemmLayout& lay) {
  if (lay.amode == 0 && lay.cmode == 0)
    launch_f32_m<0, 0>(c);
  else if (lay.amode == 0)
    launch_f32_m<0, 1>(c);
  else if (lay.cmode == 0)
    launch_f32_m<1, 0>(c);
  else
    launch_f32_m<1, 1>(c);
}

}  // namespace stem
