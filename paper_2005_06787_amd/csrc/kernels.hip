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

#include "device_common.h"

namespace stem {

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
  if (p.t == 0) {  // rank 0: one entry
    if (threadIdx.x == 0) out[ob] = in[ib];
    return;
  }
  // address bit 0 is tile bit 0 on both sides (the fastest bits are tile
  // bits), so each thread moves two adjacent entries as one 16-byte access.
  // Thread x takes tile entries 2x + 512 j: tile bits 1..8 are fixed per
  // thread (their address parts are computed once), bits 9.. follow j.
  const int e0 = 2 * (int)threadIdx.x;
  const int lb = p.t < 9 ? p.t : 9;
  uint64_t in_lo = 0, out_lo = 0;
  int e_lo = 0;
  for (int i = 1; i < lb; ++i) {
    const int bit = (e0 >> i) & 1;
    in_lo |= (uint64_t)bit << p.tin[i];
    out_lo |= (uint64_t)bit << p.tout[i];
    e_lo |= bit << p.f2e[i];
  }
  for (int e = e0; e < T; e += 512) {
    uint64_t a = ib | in_lo;
    for (int i = 9; i < p.t; ++i) a |= (uint64_t)((e >> i) & 1) << p.tin[i];
    const float4 v = *(const float4*)(in + a);
    tile[e + (e >> 5)] = make_float2(v.x, v.y);
    tile[e + 1 + (e >> 5)] = make_float2(v.z, v.w);
  }
  __syncthreads();
  for (int f = e0; f < T; f += 512) {
    uint64_t a = ob | out_lo;
    int e = e_lo;
    for (int i = 9; i < p.t; ++i) {
      const int bit = (f >> i) & 1;
      a |= (uint64_t)bit << p.tout[i];
      e |= bit << p.f2e[i];
    }
    const int e1 = e | (1 << p.f2e[0]);
    const float2 u = tile[e + (e >> 5)], w = tile[e1 + (e1 >> 5)];
    *(float4*)(out + a) = make_float4(u.x, u.y, w.x, w.y);
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

size_t bfrag_f32_floats(int64_t K, int64_t N) {
  const int64_t Kp = std::max<int64_t>(16, 2 * K), Np = std::max<int64_t>(16, 2 * N);
  return (size_t)(Kp * Np);
}

size_t bfrag_split_halves(int64_t K, int64_t N) {
  const int64_t Kq = std::max<int64_t>(32, 2 * K), Np = std::max<int64_t>(16, 2 * N);
  return (size_t)(Kq * Np);
}

size_t bfrag_gauss_floats(int64_t K, int64_t N) {
  return (K % 8 == 0 && N % 16 == 0) ? (size_t)(3 * K * N) : 0;
}

size_t branch_block_bytes(int precision, int64_t K, int64_t N) {
  size_t body = precision == STEM_FP32 ? (bfrag_f32_floats(K, N) + bfrag_gauss_floats(K, N)) * 4
                                       : bfrag_split_halves(K, N) * 4;
  return (kBranchHeader + body + 255) & ~size_t(255);
}

void build_bfrag_gauss(const float* b, int64_t K, int64_t N, float* out) {
  const int64_t KC = K / 8, NTC = N / 16;
  for (int64_t kc = 0; kc < KC; ++kc)
    for (int64_t ct = 0; ct < NTC; ++ct)
      for (int j = 0; j < 2; ++j)
        for (int lane = 0; lane < 64; ++lane) {
          const int64_t k = 8 * kc + 2 * (lane >> 4) + j;
          const int64_t n = 16 * ct + (lane & 15);
          const float br = b[2 * (k * N + n)], bi = b[2 * (k * N + n) + 1];
          float* o = out + ((kc * NTC + ct) * 6 + 3 * j) * 64 + lane;
          o[0] = br;
          o[64] = bi;
          o[128] = br + bi;
        }
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
  c.g = make_geom(lay, M, K, N, precision == STEM_FP32 ? 16 : 32);
  GemmSched want = sched;
  if (want.algo == 1 && (precision != STEM_FP32 || !gauss_ok(c.g, lay.cmode))) want.algo = 0;
  c.sch = resolve_sched(c.g, want);
  if (precision == STEM_FP32 && c.sch.algo == 1)
    launch_gemm_f32g(c, lay);
  else if (precision == STEM_FP32)
    launch_gemm_f32(c, lay);
  else
    launch_gemm_split(c, lay, precision == STEM_SPLIT_BF16);
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
                                                           uint64_t n, int overwrite) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t o = 0;
  for (int q = 0; q < m.rank; ++q) o |= ((i >> q) & 1ull) << m.dst[q];
  // overwrite: start from 0 instead of reading out (0 + x is exact, so the
  // bits equal zeroing out first)
  double2 r = overwrite ? make_double2(0.0, 0.0) : out[o];
  // the loads of 16 slices are issued before they are added (in slice
  // order), so that a short result is not one memory latency per slice
  constexpr int kBatch = 16;
  int z = 0;
  for (; z + kBatch <= nz; z += kBatch) {
    float2 v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) v[u] = ((const float2*)op_base(in_op, z + u, s0))[i];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      r.x += (double)v[u].x;
      r.y += (double)v[u].y;
    }
  }
  for (; z < nz; ++z) {
    const float2 v = ((const float2*)op_base(in_op, z, s0))[i];
    r.x += (double)v.x;
    r.y += (double)v.y;
  }
  out[o] = r;
}

hipError_t launch_acc_f64(const Operand& in, uint64_t s0, int nz, double* out, const BitMap& m,
                          hipStream_t st, bool overwrite) {
  const uint64_t n = 1ull << m.rank;
  const uint64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(stem_acc_f64_kernel, dim3((unsigned)blocks), dim3(256), 0, st, in, s0, nz,
                     (double2*)out, m, n, overwrite ? 1 : 0);
  return hipGetLastError();
}

// The same sum for large results, staged through LDS like the permute so
// that the slices' reads and the result's reads and writes are contiguous
// runs: a workgroup loads its tile of the result (output order) into LDS,
// adds every slice's entries (input order) in slice order, and writes the
// tile back.  Per entry the additions are those of stem_acc_f64_kernel, in
// the same order, so the bits are the same.
__global__ __launch_bounds__(256) void stem_acc_tiled_kernel(Operand in_op, uint64_t s0, int nz,
                                                             double2* __restrict__ out,
                                                             PermArgs p, int overwrite) {
  __shared__ double2 tile[(1 << kAccTileMaxBits) + (1 << kAccTileMaxBits) / 32];
  const uint64_t w = (uint64_t)blockIdx.x + (uint64_t)blockIdx.y * gridDim.x;
  uint64_t ib = 0, ob = 0;
  for (int i = 0; i < p.nn; ++i) {
    const uint64_t bit = (w >> i) & 1ull;
    ib |= bit << p.nin[i];
    ob |= bit << p.nout[i];
  }
  const int T = 1 << p.t;
  // thread x takes tile entries x + 256 j: tile bits 0..7 are fixed per
  // thread (their address parts are computed once), bits 8.. follow j
  const int x0 = (int)threadIdx.x;
  const int lb = p.t < 8 ? p.t : 8;
  uint64_t out_lo = 0;
  int e_lo = 0;
  for (int i = 0; i < lb; ++i) {
    const int bit = (x0 >> i) & 1;
    out_lo |= (uint64_t)bit << p.tout[i];
    e_lo |= bit << p.f2e[i];
  }
  auto out_entry = [&](int f, uint64_t* a_out, int* e_out) {
    uint64_t a = ob | out_lo;
    int e = e_lo;
    for (int i = 8; i < p.t; ++i) {
      const int bit = (f >> i) & 1;
      a |= (uint64_t)bit << p.tout[i];
      e |= bit << p.f2e[i];
    }
    *a_out = a;
    *e_out = e;
  };
  for (int f = x0; f < T; f += 256) {
    uint64_t a;
    int e;
    out_entry(f, &a, &e);
    tile[e + (e >> 5)] = overwrite ? make_double2(0.0, 0.0) : out[a];
  }
  __syncthreads();
  // the slices' entries in pairs: tile bit 0 is input address bit 0, so
  // thread x reads tile entries 2x + 512 j and 2x + 1 + 512 j as one
  // 16-byte load (tile bits 1..8 fixed per thread, bits 9.. follow j); the
  // host runs this kernel on tiles of 2^10 entries only
  const int lb2 = p.t < 9 ? p.t : 9;
  uint64_t in_lo2 = 0;
  for (int i = 1; i < lb2; ++i) in_lo2 |= (uint64_t)(((2 * x0) >> i) & 1) << p.tin[i];
  for (int e = 2 * x0; e < T; e += 512) {
    uint64_t a = ib | in_lo2;
    for (int i = 9; i < p.t; ++i) a |= (uint64_t)((e >> i) & 1) << p.tin[i];
    const int s = e + (e >> 5);  // e is even: entry e + 1 sits at s + 1
    double2 r0 = tile[s], r1 = tile[s + 1];
    for (int z = 0; z < nz; ++z) {
      const float4 v = *(const float4*)((const float2*)op_base(in_op, z, s0) + a);
      r0.x += (double)v.x;
      r0.y += (double)v.y;
      r1.x += (double)v.z;
      r1.y += (double)v.w;
    }
    tile[s] = r0;
    tile[s + 1] = r1;
  }
  __syncthreads();
  for (int f = x0; f < T; f += 256) {
    uint64_t a;
    int e;
    out_entry(f, &a, &e);
    out[a] = tile[e + (e >> 5)];
  }
}

hipError_t launch_acc_tiled(const Operand& in, uint64_t s0, int nz, double* out,
                            const PermArgs& p, hipStream_t st, bool overwrite) {
  // the kernel reads entry pairs and owns 4 tile entries per thread
  if (p.t < 1 || p.t > kAccTileMaxBits) return hipErrorInvalidValue;
  const uint64_t blocks = 1ull << p.nn;
  const uint64_t gx = std::min<uint64_t>(blocks, 1ull << 20);
  const uint64_t gy = blocks / gx;
  hipLaunchKernelGGL(stem_acc_tiled_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st,
                     in, s0, nz, (double2*)out, p, overwrite ? 1 : 0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Root join of two stem halves (the contraction of the two final tensors
// over the labels they share).  The output is small (the open labels) and
// the shared index long, so the work is split over k: every workgroup
// takes one slice and one chunk of k, stages the chunk's rows of L and R
// in LDS (both k-major, so every stage is one contiguous run of each), and
// every thread sums the products of its outputs in FP64.
// ---------------------------------------------------------------------------
constexpr int kJoinStageLog = 8;       // k values per LDS stage, at most
constexpr int kJoinLds = 64 * 1024;     // LDS of one stage, at most

__global__ __launch_bounds__(256) void stem_join_partial_kernel(Operand Lop, Operand Rop,
                                                                uint64_t s0, int a_log, int b_log,
                                                                int k_log, int chunk_log,
                                                                int stage_log,
                                                                double2* __restrict__ part) {
  extern __shared__ float2 sj[];
  const int z = blockIdx.y;
  const int chunk = blockIdx.x;
  const float2* __restrict__ L = (const float2*)op_base(Lop, z, s0);
  const float2* __restrict__ R = (const float2*)op_base(Rop, z, s0);
  const int na = 1 << a_log, nb = 1 << b_log;
  const int n_out = na * nb;
  const int64_t k0 = (int64_t)chunk << chunk_log;
  const int kn = 1 << chunk_log;
  const int stage = 1 << stage_log;       // <= kn
  float2* sL = sj;                       // [stage][na]
  float2* sR = sj + (size_t)stage * na;  // [stage][nb]
  double2 acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = make_double2(0.0, 0.0);
  for (int kk = 0; kk < kn; kk += stage) {
    __syncthreads();
    for (int i = threadIdx.x; i < stage * na; i += blockDim.x) sL[i] = L[(k0 + kk) * na + i];
    for (int i = threadIdx.x; i < stage * nb; i += blockDim.x) sR[i] = R[(k0 + kk) * nb + i];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int o = threadIdx.x + q * 256;
      if (o < n_out) {
        const int a = o >> b_log, b = o & (nb - 1);
        double re = acc[q].x, im = acc[q].y;
        for (int k = 0; k < stage; ++k) {
          const float2 l = sL[k * na + a];
          const float2 r = sR[k * nb + b];
          re += (double)l.x * r.x - (double)l.y * r.y;
          im += (double)l.x * r.y + (double)l.y * r.x;
        }
        acc[q] = make_double2(re, im);
      }
    }
  }
  const int nchunks = 1 << (k_log - chunk_log);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int o = threadIdx.x + q * 256;
    if (o < n_out) part[((int64_t)z * nchunks + chunk) * n_out + o] = acc[q];
  }
}

hipError_t launch_join_partial(const Operand& L, const Operand& R, uint64_t s0, int nz, int a_log,
                               int b_log, int k_log, int chunk_log, double* part,
                               hipStream_t st) {
  const int na = 1 << a_log, nb = 1 << b_log;
  int stage_log = std::min(chunk_log, kJoinStageLog);
  while (stage_log > 0 && (size_t)(na + nb) * ((size_t)8 << stage_log) > (size_t)kJoinLds)
    --stage_log;
  const size_t lds = (size_t)(na + nb) * ((size_t)8 << stage_log);
  const int nchunks = 1 << (k_log - chunk_log);
  hipLaunchKernelGGL(stem_join_partial_kernel, dim3((unsigned)nchunks, (unsigned)nz), dim3(256),
                     lds, st, L, R, s0, a_log, b_log, k_log, chunk_log, stage_log,
                     (double2*)part);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void stem_join_acc_kernel(const double2* __restrict__ part,
                                                            int nz, int nchunks, int n_out,
                                                            double2* __restrict__ out, BitMap m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_out) return;
  uint64_t o = 0;
  for (int q = 0; q < m.rank; ++q) o |= ((uint64_t)(i >> q) & 1ull) << m.dst[q];
  double2 r = out[o];
  for (int z = 0; z < nz; ++z) {
    double re = 0.0, im = 0.0;
    for (int c = 0; c < nchunks; ++c) {
      const double2 v = part[((int64_t)z * nchunks + c) * n_out + i];
      re += v.x;
      im += v.y;
    }
    r.x += re;
    r.y += im;
  }
  out[o] = r;
}

hipError_t launch_join_acc(const double* part, int nz, int nchunks, int out_log, double* out,
                           const BitMap& m, hipStream_t st) {
  const int n_out = 1 << out_log;
  hipLaunchKernelGGL(stem_join_acc_kernel, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0,
                     st, (const double2*)part, nz, nchunks, n_out, (double2*)out, m);
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
