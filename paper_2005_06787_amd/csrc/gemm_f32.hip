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
  const int wave = wave_id();
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

  // lane constants: row bits 0..3 and k bits 0..2 (k = 8 kc + 2 grp + i)
  const int64_t rlo = row_lo(r16, g);
  const int64_t kl0 = k_offset(2 * grp, g);
  const int64_t kl1 = k_offset(2 * grp + 1, g);

  const int64_t rows_per_wg = 4 * 16 * TM;
  const int64_t nblk = (g.M + rows_per_wg - 1) / rows_per_wg;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t row0 = (blk * 4 + wave) * (16 * TM);
    if (row0 >= g.M) continue;
    f32x4 acc[TM][NTW];
    int64_t rb[TM];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int64_t hi = row_hi((row0 >> 4) + t, g);  // wave-uniform
      rb[t] = row0 + t * 16 + r16 < g.M ? (hi | rlo) : -1;
#pragma unroll
      for (int n = 0; n < NTW; ++n) acc[t][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    f32x4 a[TM];
#pragma unroll
    for (int t = 0; t < TM; ++t) a[t] = load_kr4<AM>(A, rb[t], grp * 4, kl0, kl1, g);
    for (int kc = 0; kc < g.KC; ++kc) {
      // prefetch the next k chunk of A while this one is multiplied
      f32x4 an[TM];
      if (kc + 1 < g.KC) {
        const int64_t kh = k_offset(8 * (kc + 1), g);  // wave-uniform
#pragma unroll
        for (int t = 0; t < TM; ++t)
          an[t] = load_kr4<AM>(A, rb[t], (kc + 1) * 16 + grp * 4, kh | kl0, kh | kl1, g);
      }
      // all branch fragments of this k chunk first, then the MFMAs ordered
      // so that TM * NTW independent accumulators separate two dependent
      // ones
      float b[NTW][4];
#pragma unroll
      for (int n = 0; n < NTW; ++n) {
        if (n < ntw) {
          const float* bp = BLDS ? sB + (kc * NTW + n) * 256 + lane
                                 : Bf + ((size_t)(kc * g.NT + nt0 + n) * 4) * 64 + lane;
          b[n][0] = bp[0];
          b[n][1] = bp[64];
          b[n][2] = bp[128];
          b[n][3] = bp[192];
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int n = 0; n < NTW; ++n)
          if (n < ntw) {
#pragma unroll
            for (int t = 0; t < TM; ++t)
              acc[t][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[n][j], a[t][j], acc[t][n], 0, 0, 0);
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

template <int AM, int CM>
static void launch_f32_m(const LaunchCtx& c) {
  STEM_TM_NTW_DISPATCH(launch_f32_t, AM, CM)
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
