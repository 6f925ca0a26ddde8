// Learned runtime model of the stem steps: a 3-layer FP32 MLP trained and
// evaluated entirely in HIP kernels (forward, back-propagation, Adam).
//
// y = W3^T relu(W2^T relu(W1^T x' + b1) + b2) + b3,  x' = (x - mean) inv_std,
// loss = mean over rows of (y - t')^2,  t' = (t - t_mean) / t_std.
// Every reduction runs in a fixed order (one thread per output, rows in
// order), so results are deterministic.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "stem_internal.h"

using namespace stem;

namespace {

constexpr int kMaxHidden = 256;
constexpr int kMaxFeatures = 64;

struct Layout {
  int F, H;
  int64_t w1, b1, w2, b2, w3, b3, n;
};

Layout layout(int F, int H) {
  Layout l;
  l.F = F;
  l.H = H;
  l.w1 = 0;
  l.b1 = l.w1 + (int64_t)F * H;
  l.w2 = l.b1 + H;
  l.b2 = l.w2 + (int64_t)H * H;
  l.w3 = l.b2 + H;
  l.b3 = l.w3 + H;
  l.n = l.b3 + 1;
  return l;
}

// One workgroup per row (grid-stride), one thread per hidden unit.
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ P, Layout L,
                                                          const float* __restrict__ X, int n,
                                                          const float* __restrict__ xm,
                                                          const float* __restrict__ xs,
                                                          float* __restrict__ Z1,
                                                          float* __restrict__ Z2,
                                                          float* __restrict__ Y) {
  __shared__ float sx[kMaxFeatures];
  __shared__ float sh[kMaxHidden];
  __shared__ float sr[kMaxHidden];
  const int tid = threadIdx.x;
  for (int r = blockIdx.x; r < n; r += gridDim.x) {
    if (tid < L.F) sx[tid] = (X[(int64_t)r * L.F + tid] - xm[tid]) * xs[tid];
    __syncthreads();
    if (tid < L.H) {
      float z = P[L.b1 + tid];
      for (int f = 0; f < L.F; ++f) z += sx[f] * P[L.w1 + (int64_t)f * L.H + tid];
      Z1[(int64_t)r * L.H + tid] = z;
      sh[tid] = fmaxf(z, 0.f);
    }
    __syncthreads();
    if (tid < L.H) {
      float z = P[L.b2 + tid];
      for (int j = 0; j < L.H; ++j) z += sh[j] * P[L.w2 + (int64_t)j * L.H + tid];
      Z2[(int64_t)r * L.H + tid] = z;
      sr[tid] = fmaxf(z, 0.f) * P[L.w3 + tid];
    }
    __syncthreads();
    if (tid == 0) {
      float y = P[L.b3];
      for (int h = 0; h < L.H; ++h) y += sr[h];
      Y[r] = y;
    }
    __syncthreads();
  }
}

// Per row: dy = 2/n (y - t'), dz2 = dy W3 [z2 > 0], dz1 = (W2 dz2) [z1 > 0].
__global__ __launch_bounds__(256) void mlp_backward_rows_kernel(
    const float* __restrict__ P, Layout L, const float* __restrict__ Y,
    const float* __restrict__ T, int n, float t_mean, float t_inv_std,
    const float* __restrict__ Z1, const float* __restrict__ Z2, float* __restrict__ DZ1,
    float* __restrict__ DZ2, float* __restrict__ DY) {
  __shared__ float sd[kMaxHidden];
  const int tid = threadIdx.x;
  for (int r = blockIdx.x; r < n; r += gridDim.x) {
    const float dy = 2.f / (float)n * (Y[r] - (T[r] - t_mean) * t_inv_std);
    if (tid == 0) DY[r] = dy;
    if (tid < L.H) {
      const float dz2 = Z2[(int64_t)r * L.H + tid] > 0.f ? dy * P[L.w3 + tid] : 0.f;
      DZ2[(int64_t)r * L.H + tid] = dz2;
      sd[tid] = dz2;
    }
    __syncthreads();
    if (tid < L.H) {
      float dh = 0.f;
      for (int h = 0; h < L.H; ++h) dh += sd[h] * P[L.w2 + (int64_t)tid * L.H + h];
      DZ1[(int64_t)r * L.H + tid] = Z1[(int64_t)r * L.H + tid] > 0.f ? dh : 0.f;
    }
    __syncthreads();
  }
}

// One thread per parameter: its gradient summed over the rows in order.
__global__ __launch_bounds__(256) void mlp_backward_params_kernel(
    Layout L, const float* __restrict__ X, int n, const float* __restrict__ xm,
    const float* __restrict__ xs, const float* __restrict__ Z1, const float* __restrict__ Z2,
    const float* __restrict__ DZ1, const float* __restrict__ DZ2, const float* __restrict__ DY,
    float* __restrict__ G) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= L.n) return;
  const int H = L.H;
  float g = 0.f;
  if (p < L.b1) {
    const int f = (int)(p / H), h = (int)(p % H);
    for (int r = 0; r < n; ++r)
      g += (X[(int64_t)r * L.F + f] - xm[f]) * xs[f] * DZ1[(int64_t)r * H + h];
  } else if (p < L.w2) {
    const int h = (int)(p - L.b1);
    for (int r = 0; r < n; ++r) g += DZ1[(int64_t)r * H + h];
  } else if (p < L.b2) {
    const int j = (int)((p - L.w2) / H), h = (int)((p - L.w2) % H);
    for (int r = 0; r < n; ++r) g += fmaxf(Z1[(int64_t)r * H + j], 0.f) * DZ2[(int64_t)r * H + h];
  } else if (p < L.w3) {
    const int h = (int)(p - L.b2);
    for (int r = 0; r < n; ++r) g += DZ2[(int64_t)r * H + h];
  } else if (p < L.b3) {
    const int h = (int)(p - L.w3);
    for (int r = 0; r < n; ++r) g += fmaxf(Z2[(int64_t)r * H + h], 0.f) * DY[r];
  } else {
    for (int r = 0; r < n; ++r) g += DY[r];
  }
  G[p] = g;
}

__global__ __launch_bounds__(256) void mlp_loss_kernel(const float* __restrict__ Y,
                                                       const float* __restrict__ T, int n,
                                                       float t_mean, float t_inv_std,
                                                       float* __restrict__ loss) {
  __shared__ float part[256];
  float s = 0.f;
  for (int r = threadIdx.x; r < n; r += 256) {
    const float d = Y[r] - (T[r] - t_mean) * t_inv_std;
    s += d * d;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = part[0] / (float)n;
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ P,
                                                       const float* __restrict__ G,
                                                       float* __restrict__ M,
                                                       float* __restrict__ V, int64_t np,
                                                       float lr, float c1, float c2) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const float g = G[p];
  const float m = 0.9f * M[p] + 0.1f * g;
  const float v = 0.999f * V[p] + 0.001f * g * g;
  M[p] = m;
  V[p] = v;
  const float mh = m / c1, vh = v / c2;
  P[p] -= lr * mh / (sqrtf(vh) + 1e-8f);
}

__global__ void mlp_unscale_kernel(float* __restrict__ Y, int n, float t_mean, float t_std) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) Y[r] = Y[r] * t_std + t_mean;
}

}  // namespace

struct stem_mlp_s {
  Layout L{};
  float* d_params = nullptr;
  float* d_grad = nullptr;
  float* d_m = nullptr;
  float* d_v = nullptr;
  float* d_xm = nullptr;
  float* d_xs = nullptr;
  float t_mean = 0.f, t_std = 1.f;
  int64_t adam_t = 0;
  int cap = 0;  // rows the work buffers hold
  float* d_z1 = nullptr;
  float* d_z2 = nullptr;
  float* d_dz1 = nullptr;
  float* d_dz2 = nullptr;
  float* d_y = nullptr;
  float* d_dy = nullptr;
  float* d_loss = nullptr;
};

static stem_status mfail(stem_status s, const std::string& m) {
  set_error(m);
  return s;
}

#define MHIP(call)                                                                  \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) return mfail(STEM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

static void mlp_free_work(stem_mlp_s* m) {
  for (float** p : {&m->d_z1, &m->d_z2, &m->d_dz1, &m->d_dz2, &m->d_y, &m->d_dy}) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  m->cap = 0;
}

static stem_status mlp_reserve(stem_mlp_s* m, int n) {
  if (n <= m->cap) return STEM_OK;
  mlp_free_work(m);
  const size_t rh = (size_t)n * m->L.H * sizeof(float);
  MHIP(hipMalloc(&m->d_z1, rh));
  MHIP(hipMalloc(&m->d_z2, rh));
  MHIP(hipMalloc(&m->d_dz1, rh));
  MHIP(hipMalloc(&m->d_dz2, rh));
  MHIP(hipMalloc(&m->d_y, (size_t)n * sizeof(float)));
  MHIP(hipMalloc(&m->d_dy, (size_t)n * sizeof(float)));
  m->cap = n;
  return STEM_OK;
}

static int row_grid(int n) { return std::max(1, std::min(n, 4096)); }

static void run_forward(stem_mlp_s* m, const float* x, int n, hipStream_t st) {
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(row_grid(n)), dim3(std::max(64, m->L.H)), 0, st,
                     m->d_params, m->L, x, n, m->d_xm, m->d_xs, m->d_z1, m->d_z2, m->d_y);
}

static void run_loss_grad(stem_mlp_s* m, const float* x, const float* t, int n, float* loss,
                          float* grad, hipStream_t st) {
  run_forward(m, x, n, st);
  const float tis = 1.f / m->t_std;
  hipLaunchKernelGGL(mlp_backward_rows_kernel, dim3(row_grid(n)), dim3(std::max(64, m->L.H)), 0,
                     st, m->d_params, m->L, m->d_y, t, n, m->t_mean, tis, m->d_z1, m->d_z2,
                     m->d_dz1, m->d_dz2, m->d_dy);
  hipLaunchKernelGGL(mlp_backward_params_kernel, dim3((unsigned)((m->L.n + 255) / 256)), dim3(256),
                     0, st, m->L, x, n, m->d_xm, m->d_xs, m->d_z1, m->d_z2, m->d_dz1, m->d_dz2,
                     m->d_dy, grad);
  if (loss)
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(256), 0, st, m->d_y, t, n, m->t_mean, tis,
                       loss);
}

static void mlp_destroy_impl(stem_mlp_s* m) {
  if (!m) return;
  mlp_free_work(m);
  for (float* p : {m->d_params, m->d_grad, m->d_m, m->d_v, m->d_xm, m->d_xs, m->d_loss})
    if (p) (void)hipFree(p);
  delete m;
}

extern "C" {

int64_t stem_mlp_n_params(int32_t n_features, int32_t hidden) {
  if (n_features < 1 || hidden < 1) return 0;
  return layout(n_features, hidden).n;
}

stem_status stem_mlp_create(int32_t F, int32_t H, const float* init, stem_mlp_t* out) {
  if (!out || !init) return mfail(STEM_EINVAL, "null argument");
  *out = nullptr;
  if (F < 1 || F > kMaxFeatures || H < 1 || H > kMaxHidden)
    return mfail(STEM_ESHAPE, "features must be 1..64 and hidden units 1..256");
  stem_mlp_s* m = new (std::nothrow) stem_mlp_s();
  if (!m) return mfail(STEM_ENOMEM, "host allocation failed");
  m->L = layout(F, H);
  const size_t pb = (size_t)m->L.n * sizeof(float);
  auto bail = [&](const char* what, hipError_t e) {
    mlp_destroy_impl(m);
    return mfail(STEM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e;
  for (float** p : {&m->d_params, &m->d_grad, &m->d_m, &m->d_v})
    if ((e = hipMalloc(p, pb)) != hipSuccess) return bail("hipMalloc", e);
  if ((e = hipMalloc(&m->d_xm, F * sizeof(float))) != hipSuccess) return bail("hipMalloc", e);
  if ((e = hipMalloc(&m->d_xs, F * sizeof(float))) != hipSuccess) return bail("hipMalloc", e);
  if ((e = hipMalloc(&m->d_loss, sizeof(float))) != hipSuccess) return bail("hipMalloc", e);
  std::vector<float> zeros(m->L.n, 0.f), ones(F, 1.f);
  if ((e = hipMemcpy(m->d_params, init, pb, hipMemcpyHostToDevice)) != hipSuccess) return bail("copy", e);
  if ((e = hipMemcpy(m->d_m, zeros.data(), pb, hipMemcpyHostToDevice)) != hipSuccess) return bail("copy", e);
  if ((e = hipMemcpy(m->d_v, zeros.data(), pb, hipMemcpyHostToDevice)) != hipSuccess) return bail("copy", e);
  if ((e = hipMemcpy(m->d_xm, zeros.data(), F * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
    return bail("copy", e);
  if ((e = hipMemcpy(m->d_xs, ones.data(), F * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
    return bail("copy", e);
  *out = m;
  return STEM_OK;
}

stem_status stem_mlp_set_scaling(stem_mlp_t m, const float* xm, const float* xs, float t_mean,
                                 float t_std) {
  if (!m || !xm || !xs) return mfail(STEM_EINVAL, "null argument");
  if (!(t_std > 0.f)) return mfail(STEM_EINVAL, "t_std must be positive");
  MHIP(hipMemcpy(m->d_xm, xm, m->L.F * sizeof(float), hipMemcpyHostToDevice));
  MHIP(hipMemcpy(m->d_xs, xs, m->L.F * sizeof(float), hipMemcpyHostToDevice));
  m->t_mean = t_mean;
  m->t_std = t_std;
  return STEM_OK;
}

stem_status stem_mlp_get_params(stem_mlp_t m, float* host) {
  if (!m || !host) return mfail(STEM_EINVAL, "null argument");
  MHIP(hipMemcpy(host, m->d_params, (size_t)m->L.n * sizeof(float), hipMemcpyDeviceToHost));
  return STEM_OK;
}

stem_status stem_mlp_loss_grad(stem_mlp_t m, const float* x, const float* t, int32_t n,
                               float* loss, float* grad, void* stream) {
  if (!m || !x || !t || !grad || n < 1) return mfail(STEM_EINVAL, "bad argument");
  stem_status s = mlp_reserve(m, n);
  if (s != STEM_OK) return s;
  run_loss_grad(m, x, t, n, loss, grad, (hipStream_t)stream);
  MHIP(hipGetLastError());
  return STEM_OK;
}

stem_status stem_mlp_train(stem_mlp_t m, const float* x, const float* t, int32_t n, int32_t steps,
                           float lr, float* loss, void* stream) {
  if (!m || !x || !t || n < 1 || steps < 0) return mfail(STEM_EINVAL, "bad argument");
  stem_status s = mlp_reserve(m, n);
  if (s != STEM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const unsigned pg = (unsigned)((m->L.n + 255) / 256);
  for (int i = 0; i < steps; ++i) {
    run_loss_grad(m, x, t, n, nullptr, m->d_grad, st);
    m->adam_t += 1;
    const float c1 = 1.f - std::pow(0.9f, (float)m->adam_t);
    const float c2 = 1.f - std::pow(0.999f, (float)m->adam_t);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3(pg), dim3(256), 0, st, m->d_params, m->d_grad, m->d_m,
                       m->d_v, m->L.n, lr, c1, c2);
  }
  if (loss) {
    run_forward(m, x, n, st);
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(256), 0, st, m->d_y, t, n, m->t_mean,
                       1.f / m->t_std, loss);
  }
  MHIP(hipGetLastError());
  return STEM_OK;
}

stem_status stem_mlp_predict(stem_mlp_t m, const float* x, int32_t n, float* y, void* stream) {
  if (!m || !x || !y || n < 1) return mfail(STEM_EINVAL, "bad argument");
  stem_status s = mlp_reserve(m, n);
  if (s != STEM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(row_grid(n)), dim3(std::max(64, m->L.H)), 0, st,
                     m->d_params, m->L, x, n, m->d_xm, m->d_xs, m->d_z1, m->d_z2, y);
  hipLaunchKernelGGL(mlp_unscale_kernel, dim3((n + 255) / 256), dim3(256), 0, st, y, n, m->t_mean,
                     m->t_std);
  MHIP(hipGetLastError());
  return STEM_OK;
}

stem_status stem_mlp_destroy(stem_mlp_t m) {
  mlp_destroy_impl(m);
  return STEM_OK;
}

}  // extern "C"
