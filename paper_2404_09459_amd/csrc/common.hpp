// Shared device/host definitions of the gfx950 randomized-GSVD library.
//
// Layout conventions (all device memory, row-major unless stated):
//  * G_i      : m_i x n, leading dimension ldg >= n, fp64 or fp32 storage.
//  * tall-skinny matrices (sketch Y, basis Q: m x l; W, Z: n x l) are kept
//    *transposed*, as L x len row-major ("Xt" layout), L = l rounded up to a
//    multiple of 16.  A column of Q is then one contiguous row, which is what
//    the MFMA operand loads, the Gram reduction and the triangular update read.
//  * rows l..L-1 of every Xt buffer are kept at zero.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// working precision of a run
enum Prec : int { P64 = 0, P32 = 1, PBF = 2 };
enum GType : int { G_F64 = 0, G_F32 = 1 };

constexpr int MAXL = 256;          // largest padded sketch width handled

// Per-matrix state of one run.  One entry per matrix (2 per pair); kernels
// are grouped over an array of these and find their entry from a tile
// prefix table.
struct Side {
  const void* G;       // input matrix
  int64_t ldg;
  int32_t m, n;        // rows, columns
  int32_t l, L;        // sketch width and its 16-padded size
  int32_t gdt;         // GType
  int32_t stream_id;   // Philox stream of this matrix's Omega
  uint64_t seed;
  int32_t ldy, ldw;    // leading dims of Yt (>= m) and Wt (>= n)
  void* Yt;            // L x ldy   sketch / basis Q (transposed)
  void* Wt;            // L x ldw   W / Z / projected block B (transposed)
  void* part;          // partial products of split reductions
  double* gram;        // L x L Gram matrix
  double* sinv;        // L x L  R^{-T} (lower triangular) of the last CholQR
  double* work;        // per-side scalars: [0]=||G||_F^2, [1]=||B||_F^2 ...
  int32_t* info;       // per-pair device status words
  int32_t mchunk;      // rows per split-reduction chunk of G^T Q
  int32_t nchunk;      // number of such chunks
  int32_t gchunk;      // columns per chunk of the Gram reduction
  int32_t pair;        // pair index (batched runs)
  int32_t which;       // 0 = G1, 1 = G2
  int32_t lcur;        // active width for adaptive runs (<= l)
};

// XCD-aware tile order.  Workgroups are handed to the 8 XCDs round-robin
// (block b to XCD b % 8), each XCD with its own L2.  Launching
// xcd_grid(tiles) blocks and running logical tile xcd_tile(b) gives every
// XCD one contiguous eighth of the tiles, so neighbouring tiles that read
// the same operand slice share an L2.  Blocks with xcd_tile(b) >= tiles exit.
constexpr int NXCD = 8;
__host__ __device__ inline int xcd_grid(int tiles) { return (tiles + NXCD - 1) / NXCD * NXCD; }
__device__ inline int xcd_tile(int b, int grid) { return (b % NXCD) * (grid / NXCD) + b / NXCD; }

// find the side that owns flat tile index `tile` in a prefix table pre[0..ns]
__device__ inline int find_side(const int* __restrict__ pre, int ns, int tile) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ----------------------------------------------------------- MFMA wrappers --
// Lane `ln` supplies row ln%16 of A and column ln%16 of B; the k index a lane
// supplies is any fixed assignment as long as A and B use the same one.
// Output: lane `ln` holds 4 values of column ln%16; value i sits in row
// out_row<P>(ln/16, i) (checked by the library's self-test).
template <int P> __device__ __host__ inline int out_row(int g, int i);
template <> __device__ __host__ inline int out_row<0>(int g, int i) { return 4 * i + g; }   // fp64
template <> __device__ __host__ inline int out_row<1>(int g, int i) { return 4 * g + i; }   // fp32
template <> __device__ __host__ inline int out_row<2>(int g, int i) { return 4 * g + i; }   // bf16
__device__ inline d4 mma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f4 mmabf(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// round-to-nearest-even fp32 -> bf16 (NaN kept quiet)
__device__ inline __bf16 f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) u |= 0x00400000u;
  else u += 0x7fffu + ((u >> 16) & 1u);
  uint16_t h = (uint16_t)(u >> 16);
  return __builtin_bit_cast(__bf16, h);
}

template <typename T> __device__ inline double to_d(T x) { return (double)x; }

// wave-wide sum (64 lanes)
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// A double moved across lanes by a DPP control (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// A double from lane ^ 16 (ds_swizzle bit-mask mode, within 32 lanes).
__device__ __forceinline__ double swz16_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)b, 0x401F);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x401F);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over each aligned group of G lanes (G a power of two <= 64), left in
// every lane of the group.  Each step adds a partner holding the same
// partial (quad xor 1, xor 2; 8-lane mirror; 16-lane mirror; lane ^ 16;
// lane ^ 32), so both sides of every step form the same two-term sum and
// all G lanes end with bit-identical results.  The whole wave must be
// active.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if (G > 1) v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  if (G > 2) v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  if (G > 4) v += dpp_f64<0x141>(v);   // row_half_mirror
  if (G > 8) v += dpp_f64<0x140>(v);   // row_mirror
  if (G > 16) v += swz16_f64(v);
  if (G > 32) v += __shfl_xor(v, 32, 64);
  return v;
}

}  // namespace rg
