// Tall-skinny MFMA products of the basis extraction (Algorithm 1's G Omega_i,
// the subspace iterations G^T Q and G W, and the projection B = Q^T G of
// Algorithm 2).  The cost section of the paper attributes the method's time
// to exactly these matrix-matrix products.
//
// k-assignment used by every kernel here: inside a chunk of KC consecutive
// k indices, lane group g = lane/16 owns the contiguous run
// [g*KC/4, (g+1)*KC/4); MFMA instruction s consumes elements
// [s*KPI, (s+1)*KPI) of that run.  Both operands use the same assignment, so
// each lane's operand loads are contiguous vectors and no operand needs an
// LDS transpose.
#pragma once
#include "common.hpp"

namespace rg {

template <int P> struct Tr;
template <> struct Tr<P64> {
  using cT = double; using acc = d4; using wT = double;
  static constexpr int KPI = 1, KC = 32, PAD = 2;
};
template <> struct Tr<P32> {
  using cT = float; using acc = f4; using wT = float;
  static constexpr int KPI = 1, KC = 64, PAD = 4;
};
template <> struct Tr<PBF> {
  using cT = __bf16; using acc = f4; using wT = float;
  static constexpr int KPI = 8, KC = 128, PAD = 8;
};

template <int P> __device__ inline typename Tr<P>::cT cvt(double x);
template <> __device__ inline double cvt<P64>(double x) { return x; }
template <> __device__ inline float cvt<P32>(double x) { return (float)x; }
template <> __device__ inline __bf16 cvt<PBF>(double x) { return f2bf((float)x); }
template <int P> __device__ inline typename Tr<P>::cT cvtf(float x);
template <> __device__ inline double cvtf<P64>(float x) { return (double)x; }
template <> __device__ inline float cvtf<P32>(float x) { return x; }
template <> __device__ inline __bf16 cvtf<PBF>(float x) { return f2bf(x); }

template <int P>
__device__ inline void mma_step(typename Tr<P>::acc& c, const typename Tr<P>::cT* a,
                                const typename Tr<P>::cT* b);
template <> __device__ inline void mma_step<P64>(d4& c, const double* a, const double* b) {
  c = mma64(a[0], b[0], c);
}
template <> __device__ inline void mma_step<P32>(f4& c, const float* a, const float* b) {
  c = mma32(a[0], b[0], c);
}
template <> __device__ inline void mma_step<PBF>(f4& c, const __bf16* a, const __bf16* b) {
  bf8 va, vb;
#pragma unroll
  for (int e = 0; e < 8; ++e) { va[e] = a[e]; vb[e] = b[e]; }
  c = mmabf(va, vb, c);
}

// Load N contiguous elements x[k .. k+N) of one row (length n) into float or
// double registers; entries beyond n, or of an invalid row, are zero.
template <typename TS, typename TD, int N>
__device__ inline void load_run(TD* out, const TS* __restrict__ row, int k, int n, bool ok) {
  if (ok && k + N <= n) {
    if constexpr (sizeof(TS) == 4 && N % 4 == 0) {
      if ((((uintptr_t)(row + k)) & 15) == 0) {
#pragma unroll
        for (int v = 0; v < N / 4; ++v) {
          f4 t = *(const f4*)(row + k + 4 * v);
          out[4 * v] = t[0]; out[4 * v + 1] = t[1]; out[4 * v + 2] = t[2]; out[4 * v + 3] = t[3];
        }
        return;
      }
    }
    if constexpr (sizeof(TS) == 8 && N % 2 == 0) {
      if ((((uintptr_t)(row + k)) & 15) == 0) {
#pragma unroll
        for (int v = 0; v < N / 2; ++v) {
          d2 t = *(const d2*)(row + k + 2 * v);
          out[2 * v] = (TD)t[0]; out[2 * v + 1] = (TD)t[1];
        }
        return;
      }
    }
#pragma unroll
    for (int e = 0; e < N; ++e) out[e] = (TD)row[k + e];
    return;
  }
#pragma unroll
  for (int e = 0; e < N; ++e) out[e] = (ok && k + e < n) ? (TD)row[k + e] : (TD)0;
}

}  // namespace rg
