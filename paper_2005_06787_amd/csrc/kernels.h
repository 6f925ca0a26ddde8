// Launchers of the libstemgpu kernels (gfx950) and the host-side layout of
// branch operands they read.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stem_internal.h"

namespace stem {

// ---- branch operand layouts (host) -------------------------------------
//
// A complex product C[M x N] = A[M x K] . B[K x N] is run as the real
// product [M x 2K] . [2K x 2N] on interleaved (re, im) data, with every
// complex branch entry b = br + i bi expanded to the 2x2 block
//     [[ br, bi],
//      [-bi, br]]   (rows: re/im part of A; columns: re/im part of C),
// so that C's interleaved (re, im) columns come out directly.

// FP32 path: fragment order for the 16x16x4 f32 MFMA.  Kp = max(16, 2K),
// Np = max(16, 2N); element ((kc*NT + nt)*4 + j)*64 + lane holds the
// expanded B'[16 kc + 4 (lane/16) + j][16 nt + lane%16] (zero padded).
size_t bfrag_f32_floats(int64_t K, int64_t N);
void build_bfrag_f32(const float* b, int64_t K, int64_t N, float* out);
// 3M fragments (C, D, C + D per k chunk and 16-column tile) of a [K x N]
// complex branch, stored after the real-embedding ones; zero floats unless
// K % 8 == 0 and N % 16 == 0.
size_t bfrag_gauss_floats(int64_t K, int64_t N);
void build_bfrag_gauss(const float* b, int64_t K, int64_t N, float* out);

// Split paths: fragment order for the 16x16x32 f16/bf16 MFMA.  Kq =
// max(32, 2K), Np = max(16, 2N); 8 consecutive halves per lane:
// element (((kc*NT + nt)*64 + lane)*8 + i) holds B'[32 kc + 8 (lane/16) + i]
// [16 nt + lane%16].  hi and lo parts are stored one after the other; the
// FP16 variant scales B by 2^eb first (eb chosen so that max |B'| 2^eb lies
// in [2^13, 2^14)), the BF16 variant uses eb = 0.
size_t bfrag_split_halves(int64_t K, int64_t N);  // per part (hi or lo)
// Writes hi then lo (2 * bfrag_split_halves uint16 values); returns eb.
int build_bfrag_split(const float* b, int64_t K, int64_t N, int bf16, uint16_t* out);

// Bytes of one branch variant block: a kBranchHeader header (the split
// paths keep 2^-eb there as a float) and the fragments.
size_t branch_block_bytes(int precision, int64_t K, int64_t N);

// ---- launchers ---------------------------------------------------------
// Every step kernel runs nz slices at once (batch item z = slice s0 + z).
hipError_t launch_permute(const Operand& in, const Operand& out, const PermArgs& p, uint64_t s0,
                          int nz, hipStream_t st);
hipError_t launch_cgemm(int precision, const Operand& A, const Operand& B, const Operand& C,
                        uint64_t s0, int nz, int64_t M, int64_t K, int64_t N,
                        const GemmLayout& lay, const GemmSched& sched, hipStream_t st);
// out[o] += sum over z < nz (in order) of in_z[i], o = i re-ordered by m
// (overwrite: out[o] = that sum, out is not read).
hipError_t launch_acc_f64(const Operand& in, uint64_t s0, int nz, double* out, const BitMap& m,
                          hipStream_t st, bool overwrite = false);
// The same sum with the reorder p (from the stem's final order to the
// result's), staged through LDS in tiles; same bits as launch_acc_f64.
hipError_t launch_acc_tiled(const Operand& in, uint64_t s0, int nz, double* out,
                            const PermArgs& p, hipStream_t st, bool overwrite);
hipError_t launch_zero_f64(double* p, uint64_t n, hipStream_t st);
// Root join of two stem halves, split over K: for every slice z < nz and
// chunk c of 2^chunk_log k values, part[(z * nchunks + c) * 2^(a+b) + o]
// = sum over k in the chunk of L_z[k][a] R_z[k][b] (o = a 2^b_log + b),
// complex, accumulated in FP64; L_z is [2^k_log][2^a_log] and R_z is
// [2^k_log][2^b_log] complex64, row-major; a_log + b_log <= 12.
hipError_t launch_join_partial(const Operand& L, const Operand& R, uint64_t s0, int nz, int a_log,
                               int b_log, int k_log, int chunk_log, double* part,
                               hipStream_t st);
// out[m(o)] += sum over z < nz (in order) of (sum over chunks, in order, of
// part[z][c][o]).
hipError_t launch_join_acc(const double* part, int nz, int nchunks, int out_log, double* out,
                           const BitMap& m, hipStream_t st);
hipError_t launch_fill_counter(float* dst, uint64_t n, uint64_t seed, int scale_log2,
                               hipStream_t st);
hipError_t launch_xeb_f64(const double* amps, uint64_t n, int n_qubits, double* out,
                          hipStream_t st);

}  // namespace stem
