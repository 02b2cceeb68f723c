// Check entry points (generator words and normals, MFMA lane layout) and the
// sizing network (32-64-64-2 ReLU MLP in FP32: forward, backward, Adam).
#include "common.hpp"
#include "philox.hpp"
#include "../../include/rgsvd.h"

using namespace rg;

namespace {

__global__ void k_gauss_fill(uint64_t seed, uint32_t sid, int64_t rows, int64_t col0, int64_t ncols,
                             int dtype, void* out, int64_t ld, int words) {
  int64_t r = blockIdx.y;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // column group
  int64_t j = (col0 >> 2) + g;
  if (r >= rows || 4 * j >= col0 + ncols) return;
  if (words) {
    U4 w = philox4x32_10((uint32_t)r, (uint32_t)j, sid, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
    for (int e = 0; e < 4; ++e) {
      int64_t c = 4 * j + e - col0;
      if (c >= 0 && c < ncols) ((uint32_t*)out)[r * ld + c] = w.x[e];
    }
    return;
  }
  if (dtype == 0) {
    double z[4];
    gauss4_f64(seed, sid, (uint32_t)r, (uint32_t)j, z);
    for (int e = 0; e < 4; ++e) {
      int64_t c = 4 * j + e - col0;
      if (c >= 0 && c < ncols) ((double*)out)[r * ld + c] = z[e];
    }
  } else {
    float z[4];
    gauss4_f32(seed, sid, (uint32_t)r, (uint32_t)j, z);
    for (int e = 0; e < 4; ++e) {
      int64_t c = 4 * j + e - col0;
      if (c >= 0 && c < ncols) ((float*)out)[r * ld + c] = z[e];
    }
  }
}

// One 16 x 16 output tile; lane ln supplies A row ln%16 and B column ln%16,
// k = (ln/16)*KPI + e, and receives column ln%16 at rows out_row(ln/16, i).
// which >= 8: raw dump, D[ln*4 + i] = value i of lane ln (layout discovery).
__global__ void k_selftest(int which, const void* A, const void* B, void* D) {
  const int ln = threadIdx.x, g = ln >> 4, li = ln & 15;
  const bool raw = which >= 8;
  const int w = which & 7;
  if (w == 0) {
    const double* a = (const double*)A; const double* b = (const double*)B;
    d4 c = {0, 0, 0, 0};
    c = mma64(a[li * 4 + g], b[g * 16 + li], c);
    for (int i = 0; i < 4; ++i)
      ((double*)D)[raw ? ln * 4 + i : out_row<0>(g, i) * 16 + li] = c[i];
  } else if (w == 1) {
    const float* a = (const float*)A; const float* b = (const float*)B;
    f4 c = {0, 0, 0, 0};
    c = mma32(a[li * 4 + g], b[g * 16 + li], c);
    for (int i = 0; i < 4; ++i)
      ((float*)D)[raw ? ln * 4 + i : out_row<1>(g, i) * 16 + li] = c[i];
  } else {
    const float* a = (const float*)A; const float* b = (const float*)B;   // K = 32
    bf8 va, vb;
    for (int e = 0; e < 8; ++e) {
      va[e] = f2bf(a[li * 32 + 8 * g + e]);
      vb[e] = f2bf(b[(8 * g + e) * 16 + li]);
    }
    f4 c = {0, 0, 0, 0};
    c = mmabf(va, vb, c);
    for (int i = 0; i < 4; ++i)
      ((float*)D)[raw ? ln * 4 + i : out_row<2>(g, i) * 16 + li] = c[i];
  }
}

// ------------------------------------------------------------------ MLP --
constexpr int H = 64, IN = 32, OUT = 2;
constexpr int OW1 = 0, OB1 = OW1 + H * IN, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H,
              OB3 = OW3 + OUT * H, NP = OB3 + OUT;
static_assert(NP == RGSVD_MLP_PARAMS, "parameter count");

// one thread per sample; parameters staged in LDS
__global__ __launch_bounds__(64) void k_mlp_fwd(const float* __restrict__ th, const float* __restrict__ X,
                                                int batch, float* __restrict__ Y, float* __restrict__ act) {
  __shared__ float w[NP];
  for (int i = threadIdx.x; i < NP; i += 64) w[i] = th[i];
  __syncthreads();
  int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= batch) return;
  float x[IN], h1[H], h2[H];
  for (int i = 0; i < IN; ++i) x[i] = X[(int64_t)b * IN + i];
  for (int o = 0; o < H; ++o) {
    float s = w[OB1 + o];
    for (int i = 0; i < IN; ++i) s = fmaf(w[OW1 + o * IN + i], x[i], s);
    h1[o] = fmaxf(s, 0.0f);
  }
  for (int o = 0; o < H; ++o) {
    float s = w[OB2 + o];
    for (int i = 0; i < H; ++i) s = fmaf(w[OW2 + o * H + i], h1[i], s);
    h2[o] = fmaxf(s, 0.0f);
  }
  for (int o = 0; o < OUT; ++o) {
    float s = w[OB3 + o];
    for (int i = 0; i < H; ++i) s = fmaf(w[OW3 + o * H + i], h2[i], s);
    Y[(int64_t)b * OUT + o] = s;
  }
  if (act) {
    for (int i = 0; i < H; ++i) act[(int64_t)b * 2 * H + i] = h1[i];
    for (int i = 0; i < H; ++i) act[(int64_t)b * 2 * H + H + i] = h2[i];
  }
}

// per-sample pre-activation gradients dz1 (64), dz2 (64), dz3 (2) -> dz (batch x 130)
__global__ __launch_bounds__(64) void k_mlp_delta(const float* __restrict__ th, const float* __restrict__ T,
                                                  int batch, const float* __restrict__ act,
                                                  float* __restrict__ dz) {
  __shared__ float w[NP];
  for (int i = threadIdx.x; i < NP; i += 64) w[i] = th[i];
  __syncthreads();
  int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= batch) return;
  const float* h1 = act + (int64_t)b * 2 * H;
  const float* h2 = h1 + H;
  float d3[OUT];
  for (int o = 0; o < OUT; ++o) {
    float s = w[OB3 + o];
    for (int i = 0; i < H; ++i) s = fmaf(w[OW3 + o * H + i], h2[i], s);
    d3[o] = (s - T[(int64_t)b * OUT + o]) / (float)batch;
  }
  float d2[H];
  for (int i = 0; i < H; ++i) {
    float s = 0.0f;
    for (int o = 0; o < OUT; ++o) s = fmaf(w[OW3 + o * H + i], d3[o], s);
    d2[i] = h2[i] > 0.0f ? s : 0.0f;
  }
  float* out = dz + (int64_t)b * (2 * H + OUT);
  for (int i = 0; i < H; ++i) {
    float s = 0.0f;
    for (int o = 0; o < H; ++o) s = fmaf(w[OW2 + o * H + i], d2[o], s);
    out[i] = h1[i] > 0.0f ? s : 0.0f;
  }
  for (int i = 0; i < H; ++i) out[H + i] = d2[i];
  for (int o = 0; o < OUT; ++o) out[2 * H + o] = d3[o];
}

// one thread per parameter: sum over the batch in fixed order
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ X, const float* __restrict__ act,
                                                  const float* __restrict__ dz, int batch,
                                                  float* __restrict__ grad) {
  int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= NP) return;
  const int DZ = 2 * H + OUT;
  float s = 0.0f;
  if (p < OB1) {
    int o = (p - OW1) / IN, i = (p - OW1) % IN;
    for (int b = 0; b < batch; ++b) s = fmaf(dz[(int64_t)b * DZ + o], X[(int64_t)b * IN + i], s);
  } else if (p < OW2) {
    int o = p - OB1;
    for (int b = 0; b < batch; ++b) s += dz[(int64_t)b * DZ + o];
  } else if (p < OB2) {
    int o = (p - OW2) / H, i = (p - OW2) % H;
    for (int b = 0; b < batch; ++b) s = fmaf(dz[(int64_t)b * DZ + H + o], act[(int64_t)b * 2 * H + i], s);
  } else if (p < OW3) {
    int o = p - OB2;
    for (int b = 0; b < batch; ++b) s += dz[(int64_t)b * DZ + H + o];
  } else if (p < OB3) {
    int o = (p - OW3) / H, i = (p - OW3) % H;
    for (int b = 0; b < batch; ++b) s = fmaf(dz[(int64_t)b * DZ + 2 * H + o], act[(int64_t)b * 2 * H + H + i], s);
  } else {
    int o = p - OB3;
    for (int b = 0; b < batch; ++b) s += dz[(int64_t)b * DZ + 2 * H + o];
  }
  grad[p] = s;
}

// loss = 0.5 sum (y - T)^2 / batch, single workgroup, fixed order
__global__ __launch_bounds__(256) void k_mlp_loss(const float* __restrict__ dz, int batch,
                                                  float* __restrict__ loss) {
  const int DZ = 2 * H + OUT;
  double s = 0.0;
  for (int b = threadIdx.x; b < batch; b += 256)
    for (int o = 0; o < OUT; ++o) {
      double d = (double)dz[(int64_t)b * DZ + 2 * H + o] * batch;
      s += 0.5 * d * d;
    }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(red[0] / batch);
}

__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.0f - b1) * gi;
  float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi; v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

extern "C" {

int rgsvd_gaussian(uint64_t seed, uint32_t stream_id, int64_t rows, int64_t col0, int64_t ncols,
                   int32_t dtype, void* out, int64_t ld, void* stream) {
  if (!out || rows < 0 || col0 < 0 || ncols < 0 || ld < ncols || (dtype != 0 && dtype != 1) ||
      rows > 65535)
    return RGSVD_EINVAL;
  if (rows == 0 || ncols == 0) return RGSVD_OK;
  int64_t groups = ((col0 + ncols - 1) >> 2) - (col0 >> 2) + 1;
  dim3 grid((unsigned)((groups + 63) / 64), (unsigned)rows);
  hipLaunchKernelGGL(k_gauss_fill, grid, dim3(64), 0, (hipStream_t)stream, seed, stream_id, rows,
                     col0, ncols, dtype, out, ld, 0);
  return hipGetLastError() == hipSuccess ? RGSVD_OK : RGSVD_EHIP;
}

int rgsvd_philox_words(uint64_t seed, uint32_t stream_id, int64_t rows, int64_t col0, int64_t ncols,
                       uint32_t* out, int64_t ld, void* stream) {
  if (!out || rows < 0 || col0 < 0 || ncols < 0 || ld < ncols || rows > 65535) return RGSVD_EINVAL;
  if (rows == 0 || ncols == 0) return RGSVD_OK;
  int64_t groups = ((col0 + ncols - 1) >> 2) - (col0 >> 2) + 1;
  dim3 grid((unsigned)((groups + 63) / 64), (unsigned)rows);
  hipLaunchKernelGGL(k_gauss_fill, grid, dim3(64), 0, (hipStream_t)stream, seed, stream_id, rows,
                     col0, ncols, 0, (void*)out, ld, 1);
  return hipGetLastError() == hipSuccess ? RGSVD_OK : RGSVD_EHIP;
}

int rgsvd_selftest_mfma(int32_t which, const void* A, const void* B, void* D, void* stream) {
  if (!A || !B || !D || (which & 7) > 2 || which < 0 || which > 10) return RGSVD_EINVAL;
  hipLaunchKernelGGL(k_selftest, dim3(1), dim3(64), 0, (hipStream_t)stream, which, A, B, D);
  return hipGetLastError() == hipSuccess ? RGSVD_OK : RGSVD_EHIP;
}

int rgsvd_mlp_forward(const float* params, const float* X, int32_t batch, float* Y, float* act,
                      void* stream) {
  if (!params || !X || !Y || batch < 0) return RGSVD_EINVAL;
  if (batch == 0) return RGSVD_OK;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((batch + 63) / 64), dim3(64), 0, (hipStream_t)stream, params, X,
                     batch, Y, act);
  return hipGetLastError() == hipSuccess ? RGSVD_OK : RGSVD_EHIP;
}

int rgsvd_mlp_backward(const float* params, const float* X, const float* T, int32_t batch,
                       const float* act, float* grad, float* loss, void* stream) {
  if (!params || !X || !T || !act || !grad || batch < 1) return RGSVD_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  float* dz = nullptr;
  // per-sample deltas: (2H + OUT) floats per sample, stream-ordered allocation
  if (hipMallocAsync((void**)&dz, (size_t)batch * (2 * H + OUT) * sizeof(float), st) != hipSuccess)
    return RGSVD_EHIP;
  hipLaunchKernelGGL(k_mlp_delta, dim3((batch + 63) / 64), dim3(64), 0, st, params, T, batch, act, dz);
  hipLaunchKernelGGL(k_mlp_grad, dim3((NP + 255) / 256), dim3(256), 0, st, X, act, dz, batch, grad);
  if (loss) hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, st, dz, batch, loss);
  hipFreeAsync(dz, st);
  return hipGetLastError() == hipSuccess ? RGSVD_OK : RGSVD_EHIP;
}

int rgsvd_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                   float beta1, float beta2, float eps, void* stream) {
  if (!params || !grad || !m || !v || step < 1) return RGSVD_EINVAL;
  float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, grad, m,
                     v, NP, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? RGSVD_OK : RGSVD_EHIP;
}

}  // extern "C"
