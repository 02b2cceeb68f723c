// Streaming kernels of the basis extraction: every pass over G.
//
//  k_gw  : Y = G W          (the sketch G Omega and the power step G W)
//  k_gtq : partial Q^T G    (the power step G^T Q and the projection B = Q^T G
//                            of Algorithm 2, one row chunk of G per job)
//  k_pack: the small operand (W^T or Q^T, FP32) in MFMA fragment order, in
//          the compute type of the pass (BF16 or FP32)
//
// Design: one wave per workgroup, no LDS and no barriers.  G is streamed from
// HBM straight into registers (each lane a contiguous run of k values); the
// small operand (W^T or Q^T, a few MB, L2-resident) is read as MFMA fragments
// directly from L2.  Both operands use the same k assignment (lane group
// g = lane/16 owns k = g*KL .. g*KL+KL-1 of each KS-wide step), so no operand
// is ever transposed.  In the BF16 and FP32 passes the small operand is
// packed in fragment order (k_pack): the fragment of one k-step and one
// 16-row tile is 64 x KL contiguous elements, one 1 KB load per wave.
#include "common.hpp"
#include "gemm.hpp"
#include "jobs.hpp"
#include "launch.hpp"

namespace rg {

template <int P> struct St;
template <> struct St<P64> { using cT = double; using acc = d4; static constexpr int KL = 4, KPI = 1; };
template <> struct St<P32> { using cT = float;  using acc = f4; static constexpr int KL = 4, KPI = 1; };
template <> struct St<PBF> { using cT = __bf16; using acc = f4; static constexpr int KL = 8, KPI = 8; };

template <int P>
__device__ inline void mma_run(typename St<P>::acc& c, const typename St<P>::cT* a,
                               const typename St<P>::cT* b) {
  if constexpr (P == PBF) {
    bf8 va, vb;
    __builtin_memcpy(&va, a, 16);
    __builtin_memcpy(&vb, b, 16);
    c = mmabf(va, vb, c);
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) mma_step<P>(c, a + s, b + s);
  }
}

template <int P, typename TS>
__device__ inline typename St<P>::cT to_c(TS x) {
  if constexpr (P == PBF) return (__bf16)(float)x;
  else return (typename St<P>::cT)x;
}

// ------------------------------------------------------ memory helpers --
// G is read through a raw buffer resource: offsets past num_records return
// zero (no guards in the loops, no alignment requirement beyond the element
// size).  Small operands are read through global-address-space pointers.
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef unsigned int u2v __attribute__((ext_vector_type(2)));
template <typename T> using gptr = const T __attribute__((address_space(1)))*;

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes) {
  if (bytes > 0x7ffffff0LL) bytes = 0x7ffffff0LL;
  if (bytes < 0) bytes = 0;
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)bytes, 0x00020000);
}
__device__ inline u4v bload16(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
}
__device__ inline u2v bload8(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
}

// N contiguous elements of G (type TS) at byte offset off, as float/double
template <typename TS, typename TD, int N>
__device__ inline void gload(TD* out, __amdgpu_buffer_rsrc_t r, int off) {
  if constexpr (sizeof(TS) == 4) {
    static_assert(N % 2 == 0, "");
    if constexpr (N % 4 == 0) {
#pragma unroll
      for (int v = 0; v < N / 4; ++v) {
        f4 t = __builtin_bit_cast(f4, bload16(r, off + 16 * v));
        out[4 * v] = (TD)t[0]; out[4 * v + 1] = (TD)t[1]; out[4 * v + 2] = (TD)t[2]; out[4 * v + 3] = (TD)t[3];
      }
    } else {
#pragma unroll
      for (int v = 0; v < N / 2; ++v) {
        f2 t = __builtin_bit_cast(f2, bload8(r, off + 8 * v));
        out[2 * v] = (TD)t[0]; out[2 * v + 1] = (TD)t[1];
      }
    }
  } else {
    static_assert(N % 2 == 0, "");
#pragma unroll
    for (int v = 0; v < N / 2; ++v) {
      d2 t = __builtin_bit_cast(d2, bload16(r, off + 16 * v));
      out[2 * v] = (TD)t[0]; out[2 * v + 1] = (TD)t[1];
    }
  }
}

// KL contiguous elements of a small operand (compute type), in bounds
template <int P>
__device__ inline void sload(typename St<P>::cT* out, const typename St<P>::cT* p) {
  if constexpr (P == P64) {
    d2 a = *(gptr<d2>)p, b = *(gptr<d2>)(p + 2);
    out[0] = a[0]; out[1] = a[1]; out[2] = b[0]; out[3] = b[1];
  } else if constexpr (P == P32) {
    f4 a = *(gptr<f4>)p;
    out[0] = a[0]; out[1] = a[1]; out[2] = a[2]; out[3] = a[3];
  } else {
    u4v v = *(gptr<u4v>)p;
    __builtin_memcpy(out, &v, 16);
  }
}

// Fragment order of a packed small operand with ctn 16-row tiles: element
// (row c, column k) sits at frag_off(k / KS, c / 16, lane, ctn) * KL + k % KL,
// lane = ((k % KS) / KL) * 16 + c % 16.
__device__ __host__ inline int64_t frag_off(int64_t st, int b, int ln, int ctn) {
  return (st * ctn + b) * 64 + ln;
}

// ------------------------------------------------------------------ k_gw --
// Job: Yt (L x ldy) = (G W)^T with W given as Wt (L x ldw, compute type,
// zero beyond column n).  Wave tile: RT*16 rows of G, all CT column tiles.
// NB-deep register pipeline (loads issued NB-1 steps ahead).
template <int P, typename TG, int RT, int CT, int NB = 3>
__global__ __launch_bounds__(64) void k_gw(const NnJob* __restrict__ jobs, const int* __restrict__ pre,
                                           int nj) {
  using cT = typename St<P>::cT;
  using acc_t = typename St<P>::acc;
  using aT = typename std::conditional<P == P64, double, float>::type;
  constexpr int KL = St<P>::KL, KS = 4 * KL;
  const int jb = find_side(pre, nj, blockIdx.x);
  const NnJob J = jobs[jb];
  const int tile = blockIdx.x - pre[jb];
  const int ln = threadIdx.x, g = ln >> 4, li = ln & 15;
  const int row0 = tile * 16 * RT;
  const int ctn = J.L >> 4;
  const int esz = (int)sizeof(TG);
  const __amdgpu_buffer_rsrc_t rs =
      make_rsrc((const char*)J.G + (int64_t)row0 * J.ldg * esz, (int64_t)(J.m - row0) * J.ldg * esz);
  int roff[RT];
#pragma unroll
  for (int a = 0; a < RT; ++a) roff[a] = (a * 16 + li) * (int)J.ldg * esz;
  constexpr bool PK = P != P64;     // packed W (fragment order)
  const cT* wrow[CT];
#pragma unroll
  for (int b = 0; b < CT; ++b) wrow[b] = (const cT*)J.Wt + (PK ? 0 : (int64_t)(b * 16 + li) * J.ldw);

  acc_t acc[RT][CT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  aT ga[NB][RT][KL];
  cT wb[NB][CT][KL];
  const int nsteps = (J.n + KS - 1) / KS;
  auto load = [&](int buf, int st) {
    const int k = st * KS + g * KL;
#pragma unroll
    for (int a = 0; a < RT; ++a) gload<TG, aT, KL>(ga[buf][a], rs, roff[a] + k * esz);
#pragma unroll
    for (int b = 0; b < CT; ++b)
      if (b < ctn) sload<P>(wb[buf][b], PK ? wrow[b] + frag_off(st, b, ln, ctn) * KL : wrow[b] + k);
  };
#pragma unroll
  for (int b = 0; b < NB - 1; ++b)
    if (b < nsteps) load(b, b);
  for (int st0 = 0; st0 < nsteps; st0 += NB) {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int st = st0 + u;
      if (st >= nsteps) break;
      if (st + NB - 1 < nsteps) load((u + NB - 1) % NB, st + NB - 1);
      cT av[RT][KL];
      const int k = st * KS + g * KL;
      const bool last = (st + 1) * KS > J.n;      // wave-uniform
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int e = 0; e < KL; ++e) {
          aT v = ga[u][a][e];
          if (last && k + e >= J.n) v = (aT)0;     // user padding between rows
          av[a][e] = to_c<P>(v);
        }
#pragma unroll
      for (int b = 0; b < CT; ++b)
        if (b < ctn)
#pragma unroll
          for (int a = 0; a < RT; ++a) mma_run<P>(acc[a][b], av[a], wb[u][b]);
    }
  }
  // lane holds Y[row0 + a*16 + out_row(g, ii)][b*16 + li]
  typedef typename std::conditional<P == P64, double, float>::type yT;
  yT* Yt = (yT*)J.Yt;
#pragma unroll
  for (int b = 0; b < CT; ++b) {
    if (b < ctn) {
      yT* dst = Yt + (int64_t)(b * 16 + li) * J.ldy;
#pragma unroll
      for (int a = 0; a < RT; ++a) {
        const int rb = row0 + a * 16;
        if constexpr (P != P64) {
          const int r = rb + 4 * g;     // out_row = 4g + ii: four consecutive rows
          if (r + 3 < J.m) {
            *(f4*)(dst + r) = f4{acc[a][b][0], acc[a][b][1], acc[a][b][2], acc[a][b][3]};
          } else {
#pragma unroll
            for (int ii = 0; ii < 4; ++ii) if (r + ii < J.m) dst[r + ii] = acc[a][b][ii];
          }
        } else {
#pragma unroll
          for (int ii = 0; ii < 4; ++ii) {
            const int r = rb + out_row<P>(g, ii);
            if (r < J.m) dst[r] = acc[a][b][ii];
          }
        }
      }
    }
  }
}

// ----------------------------------------------------------------- k_gw4 --
// The same product for FP32 G with the packed W shared by a workgroup: 4
// waves, wave w streams the 16 rows row0 + 16 w .. row0 + 16 w + 15 of G
// through an NB-deep register pipeline, and the packed W of a k-step
// (ctn x 64 x KL contiguous elements) is staged once per workgroup into LDS
// (two buffers, one barrier per step), where the four waves read their
// fragments.  16-row waves keep every SIMD busy in the MFMA-bound FP32 pass
// while W's L2 traffic stays that of 64-row tiles.  Used for the FP32
// passes; the HBM-bound BF16 passes measured faster with k_gw's single-wave
// 64-row tiles.
template <int P, int CT, int NB>
__global__ __launch_bounds__(256) void k_gw4(const NnJob* __restrict__ jobs, const int* __restrict__ pre,
                                             int nj) {
  using cT = typename St<P>::cT;
  using acc_t = typename St<P>::acc;
  constexpr int KL = St<P>::KL, KS = 4 * KL;
  constexpr int CH = (CT * 64 + 255) / 256;       // 16-byte chunks of a W step per thread
  static_assert(KL * sizeof(cT) == 16, "a lane's fragment is 16 bytes");
  __shared__ u4v wl[2][CT * 64];
  const int jb = find_side(pre, nj, blockIdx.x);
  const NnJob J = jobs[jb];
  const int tile = blockIdx.x - pre[jb];
  const int tid = threadIdx.x, wave = tid >> 6, ln = tid & 63, g = ln >> 4, li = ln & 15;
  const int row0 = tile * 64 + wave * 16;
  const int ctn = J.L >> 4;
  const int nch = ctn * 64;                        // 16-byte chunks per W step
  const __amdgpu_buffer_rsrc_t rs =
      make_rsrc((const char*)J.G + (int64_t)row0 * J.ldg * 4, (int64_t)(J.m - row0) * J.ldg * 4);
  const int roff = li * (int)J.ldg * 4;
  const u4v* wsrc = (const u4v*)J.Wt;             // packed, nch chunks per step

  acc_t acc[CT];
#pragma unroll
  for (int b = 0; b < CT; ++b) acc[b] = acc_t{0, 0, 0, 0};
  // W of a step is fetched into a register ring WR steps ahead and stored
  // into the LDS buffer of its step one step ahead
  constexpr int WR = 4;
  static_assert(NB % WR == 0, "ring indices stay compile-time");
  float ga[NB][KL];
  u4v wt[WR][CH];
  const int nsteps = (J.n + KS - 1) / KS;
  auto gl = [&](int buf, int st) { gload<float, float, KL>(ga[buf], rs, roff + (st * KS + g * KL) * 4); };
  auto wfetch = [&](int slot, int st) {
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int c = tid + 256 * i;
      if (c < nch) wt[slot][i] = *(gptr<u4v>)(wsrc + (int64_t)st * nch + c);
    }
  };
  auto wstore = [&](int slot, int buf) {
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int c = tid + 256 * i;
      if (c < nch) wl[buf][c] = wt[slot][i];
    }
  };
#pragma unroll
  for (int b = 0; b < NB - 1; ++b)
    if (b < nsteps) gl(b, b);
  // tiles past ctn stay zero, so the MFMAs below run unconditionally
  for (int c = nch + tid; c < CT * 64; c += 256) { wl[0][c] = u4v{0, 0, 0, 0}; wl[1][c] = u4v{0, 0, 0, 0}; }
#pragma unroll
  for (int b = 0; b < WR; ++b)
    if (b < nsteps) wfetch(b, b);
  wstore(0, 0);
  __syncthreads();
  for (int st0 = 0; st0 < nsteps; st0 += NB) {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int st = st0 + u;
      if (st >= nsteps) break;
      if (st + NB - 1 < nsteps) gl((u + NB - 1) % NB, st + NB - 1);
      const bool more = st + 1 < nsteps;
      cT av[KL];
      const int k = st * KS + g * KL;
      const bool last = (st + 1) * KS > J.n;      // wave-uniform
#pragma unroll
      for (int e = 0; e < KL; ++e) {
        float v = ga[u][e];
        if (last && k + e >= J.n) v = 0.0f;      // user padding between rows
        av[e] = to_c<P>(v);
      }
      const u4v* wb = wl[st & 1];
#pragma unroll
      for (int b = 0; b < CT; ++b) {
        const u4v wv = wb[b * 64 + ln];
        cT wf[KL];
        __builtin_memcpy(wf, &wv, 16);
        mma_run<P>(acc[b], av, wf);
      }
      if (more) wstore((u + 1) % WR, (st + 1) & 1);
      if (st + WR < nsteps) wfetch(u % WR, st + WR);   // its slot held W(st), already in LDS
      __syncthreads();
    }
  }
  // lane holds Y[row0 + out_row(g, ii)][b*16 + li]: four consecutive rows
  float* Yt = (float*)J.Yt;
#pragma unroll
  for (int b = 0; b < CT; ++b) {
    if (b < ctn) {
      float* dst = Yt + (int64_t)(b * 16 + li) * J.ldy;
      const int r = row0 + 4 * g;
      if (r + 3 < J.m) {
        *(f4*)(dst + r) = f4{acc[b][0], acc[b][1], acc[b][2], acc[b][3]};
      } else {
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) if (r + ii < J.m) dst[r + ii] = acc[b][ii];
      }
    }
  }
}

// ------------------------------------------------------------------ k_nn --
// Y = G W for FP32 G on BF16 MFMA, with the packed W shared by a workgroup
// through LDS.  NW waves; wave w streams the 16 RT rows row0 + 16 RT w ...
// of G through an NB-deep register pipeline, and the packed W of a k-step
// (NPW pieces x ctn tiles x 64 lanes x 16 bytes) is staged once per
// workgroup into LDS (two buffers, one barrier per step), where every wave
// reads the fragments of its RT row tiles.  W then crosses L2 once per
// 16 RT NW rows of G instead of once per wave tile.
//
// SPLIT = false: G is rounded to BF16 (RNE) and W is one BF16 piece.
// SPLIT = true: an FP32-accurate product.  G and W are each split into three
// BF16 pieces, x = x1 + x2 + x3 with x1 = bf16(x), x2 = bf16(x - x1),
// x3 = bf16(x - x1 - x2) (both differences exact in FP32), and the six
// products g_i w_j with i + j <= 4 are accumulated in FP32; the three
// dropped ones are below 2^-24 of the product.
constexpr int NN_NW = 8;

template <bool SPLIT> __device__ __forceinline__ void split_bf16(const float (&x)[8], bf8 (&p)[SPLIT ? 3 : 1]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)x[e];
    p[0][e] = h;
    if constexpr (SPLIT) {
      const float r1 = x[e] - (float)h;
      const __bf16 m = (__bf16)r1;
      p[1][e] = m;
      p[2][e] = (__bf16)(r1 - (float)m);
    }
  }
}

template <bool SPLIT, int CT, int RT>
__global__ __launch_bounds__(64 * NN_NW) void k_nn(const NnJob* __restrict__ jobs, const int* __restrict__ pre,
                                                   int nj) {
  constexpr int NPW = SPLIT ? 3 : 1;         // BF16 pieces of W (and of G)
  constexpr int KL = 8, KS = 32, NB = 3;
  constexpr int STR = NPW * CT * 64;          // 16-byte chunks per LDS buffer
  constexpr int NT = 64 * NN_NW;
  constexpr int CH = (STR + NT - 1) / NT;     // chunks a thread stages per step
  extern __shared__ u4v wl[];                 // 2 x STR
  const int jb = find_side(pre, nj, blockIdx.x);
  const NnJob J = jobs[jb];
  const int tile = blockIdx.x - pre[jb];
  const int tid = threadIdx.x, wave = tid >> 6, ln = tid & 63, g = ln >> 4, li = ln & 15;
  const int row0 = tile * (16 * RT * NN_NW) + wave * 16 * RT;
  const int ctn = J.L >> 4;
  const int nchw = ctn * 64;                  // chunks of one piece per step
  const int nsteps = (J.n + KS - 1) / KS;
  const __amdgpu_buffer_rsrc_t rs =
      make_rsrc((const char*)J.G + (int64_t)row0 * J.ldg * 4, (int64_t)(J.m - row0) * J.ldg * 4);
  int roff[RT];
#pragma unroll
  for (int a = 0; a < RT; ++a) roff[a] = (a * 16 + li) * (int)J.ldg * 4;
  const u4v* wsrc = (const u4v*)J.Wt;         // piece p, step st: chunks (p nsteps + st) nchw ...

  f4 acc[RT][CT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) acc[a][b] = f4{0.0f, 0.0f, 0.0f, 0.0f};

  float ga[NB][RT][KL];
  u4v wt[CH];
  auto gl = [&](int buf, int st) {
#pragma unroll
    for (int a = 0; a < RT; ++a) gload<float, float, KL>(ga[buf][a], rs, roff[a] + (st * KS + g * KL) * 4);
  };
  auto wfetch = [&](int st) {
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int c = tid + NT * i;
      if (c < NPW * nchw) {
        const int pc = c / nchw, w = c - pc * nchw;
        wt[i] = *(gptr<u4v>)(wsrc + ((int64_t)pc * nsteps + st) * nchw + w);
      }
    }
  };
  auto wstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int c = tid + NT * i;
      if (c < NPW * nchw) {
        const int pc = c / nchw, w = c - pc * nchw;
        wl[buf * STR + pc * CT * 64 + w] = wt[i];
      }
    }
  };
#pragma unroll
  for (int b = 0; b < NB - 1; ++b)
    if (b < nsteps) gl(b, b);
  // column tiles past ctn read zeros, so the MFMAs below need no branch and
  // independent tiles interleave
  for (int c = tid; c < 2 * STR; c += NT)
    if ((c % (CT * 64)) >= nchw) wl[c] = u4v{0, 0, 0, 0};
  if (nsteps > 0) { wfetch(0); wstore(0); }
  if (nsteps > 1) wfetch(1);
  __syncthreads();
#pragma unroll 1
  for (int st0 = 0; st0 < nsteps; st0 += NB) {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int st = st0 + u;
      if (st >= nsteps) break;
      if (st + NB - 1 < nsteps) gl((u + NB - 1) % NB, st + NB - 1);
      const int k = st * KS + g * KL;
      const bool last = (st + 1) * KS > J.n;      // wave-uniform
      bf8 gp[RT][NPW];
#pragma unroll
      for (int a = 0; a < RT; ++a) {
        float v[KL];
#pragma unroll
        for (int e = 0; e < KL; ++e) v[e] = (last && k + e >= J.n) ? 0.0f : ga[u][a][e];   // padding between rows
        split_bf16<SPLIT>(v, gp[a]);
      }
      const u4v* wb = wl + (st & 1) * STR;
      // no branch over the tiles (those past ctn read zeros); the column
      // tiles go in groups, product-major within a group, so that four
      // independent accumulators sit between dependent MFMAs
      constexpr int TG = RT == 1 ? (CT < 4 ? CT : 4) : (CT < 2 ? CT : 2);
      constexpr int PG[6] = {2, 1, 0, 1, 0, 0}, PW[6] = {0, 1, 2, 0, 1, 0};   // smallest terms first
#pragma unroll
      for (int b0 = 0; b0 < CT; b0 += TG) {
        bf8 wp[TG][NPW];
#pragma unroll
        for (int bb = 0; bb < TG; ++bb)
#pragma unroll
          for (int pc = 0; pc < NPW; ++pc)
            wp[bb][pc] = __builtin_bit_cast(bf8, wb[pc * CT * 64 + (b0 + bb) * 64 + ln]);
#pragma unroll
        for (int t = SPLIT ? 0 : 5; t < 6; ++t)
#pragma unroll
          for (int bb = 0; bb < TG; ++bb)
#pragma unroll
            for (int a = 0; a < RT; ++a)
              acc[a][b0 + bb] = mmabf(gp[a][PG[t]], wp[bb][PW[t]], acc[a][b0 + bb]);
      }
      if (st + 1 < nsteps) wstore((st + 1) & 1);   // W(st + 1), fetched one step ago
      if (st + 2 < nsteps) wfetch(st + 2);
      __syncthreads();
    }
  }
  // lane holds Y[row0 + 16 a + 4 g + ii][16 b + li]: four consecutive rows
  float* Yt = (float*)J.Yt;
#pragma unroll
  for (int b = 0; b < CT; ++b) {
    if (b >= ctn) continue;
    float* dst = Yt + (int64_t)(b * 16 + li) * J.ldy;
#pragma unroll
    for (int a = 0; a < RT; ++a) {
      const int r = row0 + a * 16 + 4 * g;
      if (r + 3 < J.m) {
        *(f4*)(dst + r) = acc[a][b];
      } else {
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) if (r + ii < J.m) dst[r + ii] = acc[a][b][ii];
      }
    }
  }
}

// ----------------------------------------------------------------- k_gtq --
// Job (AbJob): D (rows x J, partial, ldd) = A (rows x K) B (K x J): A = Q^T
// columns of this row chunk in the compute type (lda, zero beyond m), B = the
// row chunk of G (ldb, K rows; rows past K read as zero through the buffer
// resource).  Wave tile: 16*JS columns of G (lane li owns JS consecutive
// columns, one per MFMA sub-tile), all CT row tiles of D.  Tiles run in XCD
// order: the column tiles of one row chunk read the same Q^T slice, which
// then stays in one XCD's L2.
template <int P, typename TG, int CT, int JS, int NB = 3>
__global__ __launch_bounds__(64) void k_gtq(const AbJob* __restrict__ jobs, const int* __restrict__ pre,
                                            int nj, int ntiles) {
  using cT = typename St<P>::cT;
  using acc_t = typename St<P>::acc;
  using bT = typename std::conditional<P == P64, double, float>::type;
  constexpr int KL = St<P>::KL, KS = 4 * KL;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  if (t >= ntiles) return;
  const int jb = find_side(pre, nj, t);
  const AbJob J = jobs[jb];
  const int tile = t - pre[jb];
  const int ln = threadIdx.x, g = ln >> 4, li = ln & 15;
  const int col0 = tile * 16 * JS + JS * li;
  const int ctn = (J.rows + 15) >> 4;
  const int esz = (int)sizeof(TG);
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(J.B, (int64_t)J.K * J.ldb * esz);
  const int coff = (col0 < J.J ? col0 : 0) * esz;
  bool cok[JS];
#pragma unroll
  for (int q = 0; q < JS; ++q) cok[q] = col0 + q < J.J;
  constexpr bool PK = P != P64;     // packed Q^T (fragment order, from the chunk's first step)
  const cT* arow[CT];
#pragma unroll
  for (int b = 0; b < CT; ++b) arow[b] = (const cT*)J.A + (PK ? 0 : (int64_t)(b * 16 + li) * J.lda);

  acc_t acc[CT][JS];
#pragma unroll
  for (int a = 0; a < CT; ++a)
#pragma unroll
    for (int q = 0; q < JS; ++q) acc[a][q] = acc_t{0, 0, 0, 0};

  bT gb[NB][KL][JS];
  cT af[NB][CT][KL];
  const int nsteps = (J.K + KS - 1) / KS;
  auto load = [&](int buf, int st) {
    const int k = st * KS + g * KL;
#pragma unroll
    for (int e = 0; e < KL; ++e) gload<TG, bT, JS>(gb[buf][e], rs, (k + e) * (int)J.ldb * esz + coff);
#pragma unroll
    for (int b = 0; b < CT; ++b)
      if (b < ctn) sload<P>(af[buf][b], PK ? arow[b] + frag_off(st, b, ln, ctn) * KL : arow[b] + k);
  };
#pragma unroll
  for (int b = 0; b < NB - 1; ++b)
    if (b < nsteps) load(b, b);
  for (int st0 = 0; st0 < nsteps; st0 += NB) {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int st = st0 + u;
      if (st >= nsteps) break;
      if (st + NB - 1 < nsteps) load((u + NB - 1) % NB, st + NB - 1);
      cT bv[JS][KL];
#pragma unroll
      for (int e = 0; e < KL; ++e)
#pragma unroll
        for (int q = 0; q < JS; ++q) bv[q][e] = to_c<P>(cok[q] ? gb[u][e][q] : (bT)0);
#pragma unroll
      for (int b = 0; b < CT; ++b)
        if (b < ctn)
#pragma unroll
          for (int q = 0; q < JS; ++q) mma_run<P>(acc[b][q], af[u][b], bv[q]);
    }
  }
  typedef typename std::conditional<P == P64, double, float>::type dT;
  dT* D = (dT*)J.D;
#pragma unroll
  for (int b = 0; b < CT; ++b) {
    if (b < ctn) {
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int c = b * 16 + out_row<P>(g, ii);
        if (c < J.rows) {
          dT* dst = D + (int64_t)c * J.ldd;
          if constexpr (JS == 4 && sizeof(dT) == 4) {
            if (col0 + 4 <= J.J) {
              *(f4*)(dst + col0) = f4{(float)acc[b][0][ii], (float)acc[b][1][ii], (float)acc[b][2][ii],
                                      (float)acc[b][3][ii]};
              continue;
            }
          }
#pragma unroll
          for (int q = 0; q < JS; ++q)
            if (col0 + q < J.J) dst[col0 + q] = (dT)acc[b][q][ii];
        }
      }
    }
  }
}

// ------------------------------------------------------------------ k_tn --
// The mixed path's G^T Q passes over FP32 G.  Job (AbJob) as for k_gtq:
// D (rows x J, partial, ldd) = A (rows x K) B (K x J), A = Q^T of the row
// chunk packed in BF16 fragment order (piece p at lda elements after piece
// 0, the chunk's first k-step first), B = the chunk of G (K rows, ldb).
// Workgroup: TN_NW waves over TN_NW / RH consecutive 32-column tiles of one
// chunk (lane li owns two adjacent columns, one per MFMA sub-tile); the RH
// waves of a column tile share its CT = RH CTW row tiles of D, CTW each (RH
// = 2 halves the accumulators of the split pass over many row tiles; the
// second wave's loads of the same G rows hit the cache).  The packed A of a k-step is staged in LDS once for all the
// waves (double-buffered, written one step ahead, one barrier per step);
// G streams from HBM into registers NB - 1 steps ahead.
// SPLIT = false: G rounded to BF16, A one BF16 piece.  SPLIT = true: the
// FP32-accurate product of k_nn's split: three BF16 pieces of both operands,
// the six products g_i q_j with i + j <= 4, smallest first.
constexpr int TN_NW = TN_WAVES;

template <bool SPLIT, int CTW, int RH>
__global__ __launch_bounds__(64 * TN_NW) void k_tn(const AbJob* __restrict__ jobs, const int* __restrict__ pre,
                                                   int nj, int ntiles) {
  constexpr int NP = SPLIT ? 3 : 1;
  constexpr int CT = CTW * RH;                // row tiles staged
  constexpr int CG = TN_NW / RH;              // column tiles per workgroup
  // G pipeline depth: three steps, two for a split wave over 6 or more row
  // tiles (its accumulators and pieces fill the registers)
  constexpr int KL = 8, KS = 32, NB = (SPLIT && CTW >= 6) ? 2 : 3, JS = 2;
  constexpr int STR = NP * CT * 64;           // 16-byte chunks per LDS buffer
  constexpr int NT = 64 * TN_NW;
  constexpr int CH = (STR + NT - 1) / NT;     // chunks a thread stages per step
  extern __shared__ u4v al[];                 // 2 x STR
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  if (t >= ntiles) return;                    // whole workgroups only
  const int jb = find_side(pre, nj, t);
  const AbJob J = jobs[jb];
  const int wg = t - pre[jb];
  const int tid = threadIdx.x, wave = tid >> 6, ln = tid & 63, g = ln >> 4, li = ln & 15;
  const int cw = wave % CG, rh = wave / CG;   // column tile in the workgroup, row half
  const int col0 = (wg * CG + cw) * 16 * JS + JS * li;
  const int ctn = (J.rows + 15) >> 4;
  const int nchw = ctn * 64;                  // chunks of one piece per step
  const int nsteps = (J.K + KS - 1) / KS;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(J.B, (int64_t)J.K * J.ldb * 4);
  const bool cok0 = col0 < J.J, cok1 = col0 + 1 < J.J;
  const int coff = (cok0 ? col0 : 0) * 4;
  const u4v* asrc = (const u4v*)J.A;          // piece pc, step st: chunks pc lda / 8 + st nchw ...
  const int64_t pst = J.lda / 8;

  f4 acc[CTW][JS];
#pragma unroll
  for (int b = 0; b < CTW; ++b)
#pragma unroll
    for (int q = 0; q < JS; ++q) acc[b][q] = f4{0.0f, 0.0f, 0.0f, 0.0f};

  float gb[NB][KL][JS];
  u4v at[CH];
  // the lane's part of the address in a VGPR, the step's and the row's in
  // the scalar offset
  const int voff = g * KL * (int)J.ldb * 4 + coff;
  const int rstr = (int)J.ldb * 4;
  auto gl = [&](int buf, int st) {
#pragma unroll
    for (int e = 0; e < KL; ++e) {
      const f2 t = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, (st * KS + e) * rstr, 0));
      gb[buf][e][0] = t[0];
      gb[buf][e][1] = t[1];
    }
  };
  auto afetch = [&](int st) {
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int c = tid + NT * i;
      if (c < NP * nchw) {
        const int pc = c / nchw, w = c - pc * nchw;
        at[i] = *(gptr<u4v>)(asrc + pc * pst + (int64_t)st * nchw + w);
      }
    }
  };
  auto astore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int c = tid + NT * i;
      if (c < NP * nchw) {
        const int pc = c / nchw, w = c - pc * nchw;
        al[buf * STR + pc * CT * 64 + w] = at[i];
      }
    }
  };
  // row tiles past ctn read zeros, so the MFMAs below need no branch
  for (int c = tid; c < 2 * STR; c += NT)
    if ((c % (CT * 64)) >= nchw) al[c] = u4v{0, 0, 0, 0};
  if (nsteps > 0) { afetch(0); astore(0); }
#pragma unroll
  for (int b = 0; b < NB - 1; ++b)
    if (b < nsteps) gl(b, b);
  __syncthreads();
#pragma unroll 1
  for (int st0 = 0; st0 < nsteps; st0 += NB) {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int st = st0 + u;
      if (st >= nsteps) break;
      // A of the next step (L2-resident) is loaded before this step's G
      // prefetch and stored once it arrives, so its registers are free
      // again before the MFMAs; the buffer it fills was last read in the
      // step before the last barrier
      if (st + 1 < nsteps) afetch(st + 1);
      if (st + NB - 1 < nsteps) gl((u + NB - 1) % NB, st + NB - 1);
      if (st + 1 < nsteps) astore((st + 1) & 1);
      bf8 bp[JS][NP];
      {
        float v0[KL], v1[KL];
#pragma unroll
        for (int e = 0; e < KL; ++e) {
          v0[e] = cok0 ? gb[u][e][0] : 0.0f;
          v1[e] = cok1 ? gb[u][e][1] : 0.0f;
        }
        split_bf16<SPLIT>(v0, bp[0]);
        split_bf16<SPLIT>(v1, bp[1]);
      }
      const u4v* ab = al + (st & 1) * STR + rh * CTW * 64;
      // row tiles in pairs, product-major within a pair: four independent
      // accumulators between dependent MFMAs
#pragma unroll
      for (int b0 = 0; b0 < CTW; b0 += 2) {
        constexpr int PA[6] = {0, 1, 2, 0, 1, 0}, PB[6] = {2, 1, 0, 1, 0, 0};   // smallest terms first
        bf8 ap[2][NP];
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
          if (b0 + bb < CTW)
#pragma unroll
            for (int pc = 0; pc < NP; ++pc)
              ap[bb][pc] = __builtin_bit_cast(bf8, ab[pc * CT * 64 + (b0 + bb) * 64 + ln]);
#pragma unroll
        for (int t = SPLIT ? 0 : 5; t < 6; ++t)
#pragma unroll
          for (int bb = 0; bb < 2; ++bb)
            if (b0 + bb < CTW)
#pragma unroll
              for (int q = 0; q < JS; ++q)
                acc[b0 + bb][q] = mmabf(ap[bb][PA[t]], bp[q][PB[t]], acc[b0 + bb][q]);
      }
      __syncthreads();
    }
  }
  // lane holds D[16 (rh CTW + b) + 4 g + ii][col0 + q]
  float* D = (float*)J.D;
#pragma unroll
  for (int b = 0; b < CTW; ++b) {
    if (rh * CTW + b >= ctn) continue;
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int c = (rh * CTW + b) * 16 + 4 * g + ii;
      if (c >= J.rows) continue;
      float* dst = D + (int64_t)c * J.ldd + col0;
      if (cok1) *(f2*)dst = f2{acc[b][0][ii], acc[b][1][ii]};
      else if (cok0) dst[0] = acc[b][0][ii];
    }
  }
}

// ---------------------------------------------------------------- k_pack --
// FP32 operand (L x ld, Xt layout; FP64 with f64src, BF16 output only) ->
// fragment order in BF16 (KL = 8) or FP32 (KL = 4) for nst k-steps of
// KS = 4 KL columns; nst * KS <= ld.  One
// thread per fragment piece (KL elements); consecutive threads write
// consecutive pieces.
struct PackJob { const void* src; void* dst; int64_t ld; int32_t L, nst, bf16, pieces, f64src; };

__global__ __launch_bounds__(256) void k_pack(const PackJob* __restrict__ jobs, const int* __restrict__ pre,
                                              int nj) {
  const int jb = find_side(pre, nj, blockIdx.x);
  const PackJob J = jobs[jb];
  const int ctn = J.L >> 4, KL = J.bf16 ? 8 : 4;
  const int64_t piece = (int64_t)(blockIdx.x - pre[jb]) * 256 + threadIdx.x;
  if (piece >= (int64_t)J.nst * ctn * 64) return;
  const int ln = (int)(piece & 63);
  const int64_t q = piece >> 6;
  const int b = (int)(q % ctn);
  const int64_t st = q / ctn;
  const int c = b * 16 + (ln & 15);
  const int64_t k = st * 4 * KL + (ln >> 4) * KL;
  const int64_t so = (int64_t)c * J.ld + k;
  if (J.bf16) {
    float x[8];
    if (J.f64src) {
      // an FP64 source (the CholeskyQR inverse), rounded to FP32 first
      const double* sd = (const double*)J.src + so;
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = (float)sd[e];
    } else {
      const float* src = (const float*)J.src + so;
      const f4 v0 = *(const f4*)src, v1 = *(const f4*)(src + 4);
#pragma unroll
      for (int e = 0; e < 4; ++e) { x[e] = v0[e]; x[4 + e] = v1[e]; }
    }
    // BF16 pieces x1, x2 = bf16(x - x1), x3 = bf16(x - x1 - x2); piece p of
    // the operand follows piece p - 1 (nst ctn 64 fragments apart)
    const int64_t pstride = (int64_t)J.nst * ctn * 64 * 8;
    for (int p = 0; p < (J.pieces > 1 ? J.pieces : 1); ++p) {
      __bf16 o[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) { o[e] = (__bf16)x[e]; x[e] -= (float)o[e]; }
      __builtin_memcpy((__bf16*)J.dst + p * pstride + piece * 8, o, 16);
    }
  } else {
    *(f4*)((float*)J.dst + piece * 4) = *(const f4*)((const float*)J.src + so);
  }
}

// ---------------------------------------------------------------- launch --
template <int P, typename TG, int RT>
static void gw_ct(int ct, const NnJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  switch (ct) {
    case 1: hipLaunchKernelGGL((k_gw<P, TG, RT, 1>), dim3(tiles), dim3(64), 0, st, j, pre, nj); break;
    case 2: hipLaunchKernelGGL((k_gw<P, TG, RT, 2>), dim3(tiles), dim3(64), 0, st, j, pre, nj); break;
    case 4: hipLaunchKernelGGL((k_gw<P, TG, RT, 4>), dim3(tiles), dim3(64), 0, st, j, pre, nj); break;
    case 8: hipLaunchKernelGGL((k_gw<P, TG, RT, 8>), dim3(tiles), dim3(64), 0, st, j, pre, nj); break;
    default: hipLaunchKernelGGL((k_gw<P, TG, RT, 16>), dim3(tiles), dim3(64), 0, st, j, pre, nj); break;
  }
}

template <int P, int NB>
static void gw4_ct(int ct, const NnJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  switch (ct) {
    case 1: hipLaunchKernelGGL((k_gw4<P, 1, NB>), dim3(tiles), dim3(256), 0, st, j, pre, nj); break;
    case 2: hipLaunchKernelGGL((k_gw4<P, 2, NB>), dim3(tiles), dim3(256), 0, st, j, pre, nj); break;
    case 4: hipLaunchKernelGGL((k_gw4<P, 4, NB>), dim3(tiles), dim3(256), 0, st, j, pre, nj); break;
    case 8: hipLaunchKernelGGL((k_gw4<P, 8, NB>), dim3(tiles), dim3(256), 0, st, j, pre, nj); break;
    default: hipLaunchKernelGGL((k_gw4<P, 16, NB>), dim3(tiles), dim3(256), 0, st, j, pre, nj); break;
  }
}

template <bool SPLIT, int RT>
static void nn_ct(int ct, const NnJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  const size_t lds = (size_t)2 * (SPLIT ? 3 : 1) * (ct <= 8 ? ct : 16) * 64 * 16;
  auto go = [&](auto kern) {
    static bool attr_set = false;   // one flag per instantiation
    if (!attr_set) {
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      attr_set = true;
    }
    hipLaunchKernelGGL(kern, dim3(tiles), dim3(64 * NN_NW), lds, st, j, pre, nj);
  };
  switch (ct) {
    case 1: go(k_nn<SPLIT, 1, RT>); break;
    case 2: go(k_nn<SPLIT, 2, RT>); break;
    case 4: go(k_nn<SPLIT, 4, RT>); break;
    case 8: go(k_nn<SPLIT, 8, RT>); break;
    default: go(k_nn<SPLIT, 16, RT>); break;
  }
}

// rt: 16-row tiles per wave, 2 except for the split pass over 16 column
// tiles (1: its registers are full)
void launch_nn(bool split, int rt, int ct, const NnJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  if (split) {
    if (rt == 2) nn_ct<true, 2>(ct, j, pre, nj, tiles, st);
    else nn_ct<true, 1>(ct, j, pre, nj, tiles, st);
  } else {
    nn_ct<false, 2>(ct, j, pre, nj, tiles, st);
  }
}

void launch_gw4(int prec, int ct, const NnJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  (void)prec;   // FP32 passes only
  gw4_ct<P32, 8>(ct, j, pre, nj, tiles, st);
}

void launch_gw(int prec, int gdt, int rt, int ct, const NnJob* j, const int* pre, int nj, int tiles,
               hipStream_t st) {
  if (prec == P64) {
    if (gdt == G_F64) gw_ct<P64, double, 1>(ct, j, pre, nj, tiles, st);
    else gw_ct<P64, float, 1>(ct, j, pre, nj, tiles, st);
  } else if (prec == P32) {
    if (gdt == G_F64) gw_ct<P32, double, 1>(ct, j, pre, nj, tiles, st);
    else if (rt == 4) gw_ct<P32, float, 4>(ct, j, pre, nj, tiles, st);
    else gw_ct<P32, float, 1>(ct, j, pre, nj, tiles, st);
  } else {
    if (gdt == G_F64) gw_ct<PBF, double, 1>(ct, j, pre, nj, tiles, st);
    else if (rt == 4) gw_ct<PBF, float, 4>(ct, j, pre, nj, tiles, st);
    else gw_ct<PBF, float, 1>(ct, j, pre, nj, tiles, st);
  }
}

template <int P, typename TG, int JS>
static void gtq_ct(int ct, const AbJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  const dim3 grid(xcd_grid(tiles));
  switch (ct) {
    case 1: hipLaunchKernelGGL((k_gtq<P, TG, 1, JS>), grid, dim3(64), 0, st, j, pre, nj, tiles); break;
    case 2: hipLaunchKernelGGL((k_gtq<P, TG, 2, JS>), grid, dim3(64), 0, st, j, pre, nj, tiles); break;
    case 4: hipLaunchKernelGGL((k_gtq<P, TG, 4, JS>), grid, dim3(64), 0, st, j, pre, nj, tiles); break;
    case 8: hipLaunchKernelGGL((k_gtq<P, TG, 8, JS>), grid, dim3(64), 0, st, j, pre, nj, tiles); break;
    default: hipLaunchKernelGGL((k_gtq<P, TG, 16, JS>), grid, dim3(64), 0, st, j, pre, nj, tiles); break;
  }
}

void launch_gtq(int prec, int gdt, int ct, int js, const AbJob* j, const int* pre, int nj, int tiles,
                hipStream_t st) {
  if (prec == P64) {
    if (gdt == G_F64) gtq_ct<P64, double, 2>(ct, j, pre, nj, tiles, st);
    else gtq_ct<P64, float, 2>(ct, j, pre, nj, tiles, st);
  } else if (prec == P32) {
    if (gdt == G_F64) gtq_ct<P32, double, 2>(ct, j, pre, nj, tiles, st);
    else if (js == 4) gtq_ct<P32, float, 4>(ct, j, pre, nj, tiles, st);
    else gtq_ct<P32, float, 2>(ct, j, pre, nj, tiles, st);
  } else {
    if (gdt == G_F64) gtq_ct<PBF, double, 2>(ct, j, pre, nj, tiles, st);
    else if (js == 4) gtq_ct<PBF, float, 4>(ct, j, pre, nj, tiles, st);
    else gtq_ct<PBF, float, 2>(ct, j, pre, nj, tiles, st);
  }
}

// ct: row tiles of D (1, or an even count up to 16); the split pass over 10
// or more runs two waves per column tile, ct / 2 row tiles each
template <bool SPLIT>
static void tn_ct(int ct, const AbJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  const size_t lds = (size_t)2 * (SPLIT ? 3 : 1) * ct * 64 * 16;
  const dim3 grid(xcd_grid(tiles));
  auto go = [&](auto kern) {
    static bool attr_set = false;   // one flag per instantiation
    if (!attr_set) {
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      attr_set = true;
    }
    hipLaunchKernelGGL(kern, grid, dim3(64 * TN_NW), lds, st, j, pre, nj, tiles);
  };
  switch (ct) {
    case 1: go(k_tn<SPLIT, 1, 1>); break;
    case 2: go(k_tn<SPLIT, 2, 1>); break;
    case 4: go(k_tn<SPLIT, 4, 1>); break;
    case 6: go(k_tn<SPLIT, 6, 1>); break;
    case 8: go(k_tn<SPLIT, 8, 1>); break;
    default:
      if constexpr (SPLIT) {
        switch (ct) {
          case 10: go(k_tn<true, 5, 2>); break;
          case 12: go(k_tn<true, 6, 2>); break;
          case 14: go(k_tn<true, 7, 2>); break;
          default: go(k_tn<true, 8, 2>); break;
        }
      } else {
        switch (ct) {
          case 10: go(k_tn<false, 10, 1>); break;
          case 12: go(k_tn<false, 12, 1>); break;
          case 14: go(k_tn<false, 14, 1>); break;
          default: go(k_tn<false, 16, 1>); break;
        }
      }
  }
}

// workgroups per row chunk of k_tn over n columns
int tn_tiles_per_chunk(bool split, int ct, int n) {
  const int cg = (split && ct >= 10) ? TN_NW / 2 : TN_NW;
  return ((n + 31) / 32 + cg - 1) / cg;
}

void launch_tn(bool split, int ct, const AbJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  if (split) tn_ct<true>(ct, j, pre, nj, tiles, st);
  else tn_ct<false>(ct, j, pre, nj, tiles, st);
}

void launch_pack(const void* j, const int* pre, int nj, int tiles, hipStream_t st) {
  hipLaunchKernelGGL(k_pack, dim3(tiles), dim3(256), 0, st, (const PackJob*)j, pre, nj);
}

}  // namespace rg
