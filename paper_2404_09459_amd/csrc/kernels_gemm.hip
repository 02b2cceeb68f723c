// Grouped tall-skinny kernels of the basis extraction and projection.
//
//  k_gen     : Omega^T from the counter-based generator (sketch operand)
//  k_ab      : D = A B, A small, B tall   (G^T Q and the projection Q^T G of
//                                          Algorithm 2, split over row chunks;
//                                          the triangular solve Q = Y R^{-1};
//                                          the recovery products of U, V, R)
//  k_gram    : partial X X^T in fp64      (CholeskyQR Gram; B B^T of the pair)
//  k_reduce  : fixed-order sum of partials
//  k_zero    : zero fill (kept as a kernel so runs stay graph-capturable)
#include "common.hpp"
#include "gemm.hpp"
#include "jobs.hpp"
#include "philox.hpp"
#include "launch.hpp"

namespace rg {

// --------------------------------------------------------------- k_zero --
__global__ void k_zero(uint32_t* __restrict__ p, int64_t nwords) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < nwords; i += stride) p[i] = 0u;
}

// Grouped zero fill: a tile clears 4096 consecutive words of its job's buffer.
__global__ __launch_bounds__(256) void k_zerog(const ZeroJob* __restrict__ jobs, const int* __restrict__ pre,
                                               int nj) {
  const int jb = find_side(pre, nj, blockIdx.x);
  const ZeroJob J = jobs[jb];
  const int64_t base = (int64_t)(blockIdx.x - pre[jb]) * 4096;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t i = base + k * 256 + threadIdx.x;
    if (i < J.nwords) J.p[i] = 0u;
  }
}

// ---------------------------------------------------------------- k_gen --
template <typename TW, bool F64>
__global__ __launch_bounds__(256) void k_gen(const GenJob* __restrict__ jobs,
                                             const int* __restrict__ pre, int nj) {
  const int jb = find_side(pre, nj, blockIdx.x);
  const GenJob J = jobs[jb];
  const int tile = blockIdx.x - pre[jb];
  const int nrt = (J.n + 255) / 256;
  const int rt = tile % nrt, grp = tile / nrt;
  const int r = rt * 256 + threadIdx.x;
  if (r >= J.n) return;
  const int j = (J.col0 >> 2) + grp;
  TW* Wt = (TW*)J.Wt;
  if constexpr (F64) {
    double z[4];
    gauss4_f64(J.seed, (uint32_t)J.stream, (uint32_t)r, (uint32_t)j, z);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int c = 4 * j + e - J.col0;
      if (c >= 0 && c < J.ncols) Wt[(int64_t)c * J.ldw + r] = (TW)z[e];
    }
  } else {
    float z[4];
    gauss4_f32(J.seed, (uint32_t)J.stream, (uint32_t)r, (uint32_t)j, z);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int c = 4 * j + e - J.col0;
      if (c >= 0 && c < J.ncols) Wt[(int64_t)c * J.ldw + r] = (TW)z[e];
    }
  }
}

// ----------------------------------------------------------------- k_ab --
// D (rows x J) (+)= A (rows x K) B (K x J).  WG = 4 waves along J; each wave
// covers 16*JS columns (lane li owns columns JS*li .. JS*li+JS-1 of them, one
// per MFMA sub-tile) and all CT row tiles.  A chunks are staged in LDS; B is
// streamed per lane.
template <int P> struct AbK;
template <> struct AbK<P64> { static constexpr int KC = 16; };
template <> struct AbK<P32> { static constexpr int KC = 32; };
template <> struct AbK<PBF> { static constexpr int KC = 64; };

template <int P, typename TA, typename TB, typename TD, int CT, int JS>
__global__ __launch_bounds__(256) void k_ab(const AbJob* __restrict__ jobs,
                                            const int* __restrict__ pre, int nj) {
  using TR = Tr<P>;
  using cT = typename TR::cT;
  using acc_t = typename TR::acc;
  using bT = typename std::conditional<P == P64, double, float>::type;
  constexpr int KC = AbK<P>::KC, KL = KC / 4, KPI = TR::KPI, NI = KL / KPI;
  constexpr int RL = KC + TR::PAD;
  constexpr int NAE = CT * 16 * KC;
  constexpr int APT = (NAE + 255) / 256;
  __shared__ cT As[CT * 16 * RL];

  const int jb = find_side(pre, nj, blockIdx.x);
  const AbJob J = jobs[jb];
  const int tile = blockIdx.x - pre[jb];
  const int wave = threadIdx.x >> 6, ln = threadIdx.x & 63, g = ln >> 4, li = ln & 15;
  const int col0 = tile * 64 * JS + wave * 16 * JS + JS * li;
  const int ctn = (J.rows + 15) >> 4;
  const TA* __restrict__ A = (const TA*)J.A;
  const TB* __restrict__ B = (const TB*)J.B;

  acc_t acc[CT][JS];
#pragma unroll
  for (int a = 0; a < CT; ++a)
#pragma unroll
    for (int q = 0; q < JS; ++q) acc[a][q] = acc_t{0, 0, 0, 0};

  bT bn[KL][JS];
  TA an[APT];
  const int nk = (J.K + KC - 1) / KC;

  auto load_b = [&](int kc) {
#pragma unroll
    for (int e = 0; e < KL; ++e) {
      int k = kc * KC + g * KL + e;
      bool ok = k < J.K;
      const TB* rowp = B + (int64_t)(ok ? k : 0) * J.ldb;
      load_run<TB, bT, JS>(bn[e], rowp, col0, J.J, ok);
    }
  };
  auto load_a = [&](int kc) {
#pragma unroll
    for (int i = 0; i < APT; ++i) {
      int e = threadIdx.x + 256 * i;
      int c = e / KC, kk = e - c * KC;
      int k = kc * KC + kk;
      an[i] = (e < NAE && c < J.rows && k < J.K) ? A[(int64_t)c * J.lda + k] : (TA)0;
    }
  };

  load_b(0);
  load_a(0);
  for (int kc = 0; kc < nk; ++kc) {
    cT b[JS][KL];
#pragma unroll
    for (int e = 0; e < KL; ++e)
#pragma unroll
      for (int q = 0; q < JS; ++q) b[q][e] = cvt<P>((double)bn[e][q]);
    TA a_[APT];
#pragma unroll
    for (int i = 0; i < APT; ++i) a_[i] = an[i];
    if (kc + 1 < nk) { load_b(kc + 1); load_a(kc + 1); }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < APT; ++i) {
      int e = threadIdx.x + 256 * i;
      if (e < NAE) {
        int c = e / KC, kk = e - c * KC;
        As[c * RL + kk] = cvt<P>((double)a_[i]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      if (ct < ctn) {
        cT a[KL];
        const cT* src = As + (ct * 16 + li) * RL + g * KL;
#pragma unroll
        for (int e = 0; e < KL; ++e) a[e] = src[e];
#pragma unroll
        for (int q = 0; q < JS; ++q)
#pragma unroll
          for (int s = 0; s < NI; ++s) mma_step<P>(acc[ct][q], &a[s * KPI], &b[q][s * KPI]);
      }
    }
  }
  // all loads of B (possibly aliasing D) are done by every wave of this WG
  __syncthreads();
  TD* D = (TD*)J.D;
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    if (ct < ctn) {
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        int c = ct * 16 + out_row<P>(g, ii);
        if (c < J.rows) {
          double sc = J.colscale ? J.colscale[c] : 1.0;
          TD* dst = D + (int64_t)c * J.ldd;
#pragma unroll
          for (int q = 0; q < JS; ++q) {
            int j = col0 + q;
            if (j < J.J) {
              double v = (double)acc[ct][q][ii] * sc;
              if (J.accumulate) v += (double)dst[j];
              dst[j] = (TD)v;
            }
          }
        }
      }
    }
  }
}

// --------------------------------------------------------------- k_gram --
// Partial Gram X[:, k0:k1] X[:, k0:k1]^T in fp64 MFMA over the R = r1 + r2
// rows of X (X1's rows, then X2's).  One single-wave workgroup per strip: RG
// (1 or 2) groups of 16 rows against the NQ (1..4) groups of 16 columns of
// one 64-column block that start at or after the first row group's diagonal
// group and below R (with RG = 2 each B fragment serves both row groups).
// The groups on or above the diagonal are the Gram's; the one group of the
// second row group that falls below it is written to the lower triangle,
// which the reduction does not read (it mirrors the upper groups and zeroes
// rows and columns at and past R).
// No LDS: lane (g, li) reads 4 consecutive k of its A rows and of its NQ B
// rows straight from L2 (16 or 32 bytes per row), NB steps of 16 k ahead.
// The 4-wide loads need k0, clen, ld1 and ld2 to be multiples of 4 (the
// plans pad leading dimensions to 64 and chunk lengths to 32).
template <typename TX, int NB, int NQ, int RG>
__device__ __forceinline__ void gram_strip(const GramJob& J, int chunk, int rp, int cb, int q0) {
  const int ln = threadIdx.x & 63, g = ln >> 4, li = ln & 15;
  const int kb = J.k0 + chunk * J.clen;
  const int ke = min(J.k1, kb + J.clen);
  const TX* X1 = (const TX*)J.X1;
  const TX* X2 = (const TX*)J.X2;
  auto rowptr = [&](int c) -> const TX* {
    if (c < J.r1) return X1 + (int64_t)c * J.ld1;
    if (c < J.r1 + J.r2) return X2 + (int64_t)(c - J.r1) * J.ld2;
    return nullptr;
  };
  // rows past R read row 0 of X1 scaled by zero (loads stay unconditional)
  const TX* pa[RG];
  double wa[RG];
#pragma unroll
  for (int r = 0; r < RG; ++r) {
    pa[r] = rowptr((RG * rp + r) * 16 + li);
    wa[r] = pa[r] ? 1.0 : 0.0;
    if (!pa[r]) pa[r] = X1;
  }
  const TX* pb[NQ];
  double wb[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    pb[q] = rowptr(cb * 64 + (q0 + q) * 16 + li);
    wb[q] = pb[q] ? 1.0 : 0.0;
    if (!pb[q]) pb[q] = X1;
  }
  d4 acc[RG][NQ];
#pragma unroll
  for (int r = 0; r < RG; ++r)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[r][q] = d4{0, 0, 0, 0};
  double ra[NB][RG][4], rbv[NB][NQ][4];
  // 4 consecutive k from kx (kx % 4 == 0, kx < ke <= ld), zero at and past ke
  auto ld4 = [&](double* o, const TX* p, int kx, double w) {
    if constexpr (sizeof(TX) == 4) {
      const f4 v = *(const f4*)(p + kx);
#pragma unroll
      for (int e = 0; e < 4; ++e) o[e] = (kx + e < ke) ? (double)v[e] * w : 0.0;
    } else {
      const d2 v0 = *(const d2*)(p + kx), v1 = *(const d2*)(p + kx + 2);
      o[0] = (kx < ke) ? v0[0] * w : 0.0;
      o[1] = (kx + 1 < ke) ? v0[1] * w : 0.0;
      o[2] = (kx + 2 < ke) ? v1[0] * w : 0.0;
      o[3] = (kx + 3 < ke) ? v1[1] * w : 0.0;
    }
  };
  const int nsteps = (ke - kb + 15) / 16;
  auto load = [&](int buf, int st) {
    const int kx = kb + st * 16 + g * 4;
    if (kx < ke) {
#pragma unroll
      for (int r = 0; r < RG; ++r) ld4(ra[buf][r], pa[r], kx, wa[r]);
#pragma unroll
      for (int q = 0; q < NQ; ++q) ld4(rbv[buf][q], pb[q], kx, wb[q]);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int r = 0; r < RG; ++r) ra[buf][r][e] = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) rbv[buf][q][e] = 0.0;
      }
    }
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
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int r = 0; r < RG; ++r)
#pragma unroll
          for (int q = 0; q < NQ; ++q) acc[r][q] = mma64(ra[u][r][e], rbv[u][q][e], acc[r][q]);
    }
  }
  // lane holds D[out_row(g, ii)][li] of row group RG rp + r, column group
  // q0 + q (rows below 16 RG npr <= npad: npad is a multiple of 64)
  double* out = J.out + (int64_t)chunk * J.npad * J.npad;
#pragma unroll
  for (int r = 0; r < RG; ++r)
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int row = (RG * rp + r) * 16 + out_row<P64>(g, ii);
        const int c = cb * 64 + (q0 + q) * 16 + li;
        out[(int64_t)row * J.npad + c] = acc[r][q][ii];
      }
}

template <typename TX, int RG>
__device__ __forceinline__ void gram_tile(const GramJob& J, int R, int tile) {
  constexpr int NB = RG == 1 ? 4 : 2;   // loads in flight: two waves per SIMD either way
  const int chunk = tile / gram_strips(R, RG);
  int s = tile - chunk * gram_strips(R, RG);
  // strip s -> (strip row rp, column block cb), in the order gram_strips counts
  const int ncb = (R + 63) / 64;
  int rp = 0;
  while (s >= ncb - rp * RG / 4) { s -= ncb - rp * RG / 4; ++rp; }
  const int cb = rp * RG / 4 + s;
  const int q0 = (cb == rp * RG / 4) ? ((rp * RG) & 3) : 0;
  const int q1 = min(4, (R - cb * 64 + 15) / 16);
  switch (q1 - q0) {
    case 1: gram_strip<TX, NB, 1, RG>(J, chunk, rp, cb, q0); break;
    case 2: gram_strip<TX, NB, 2, RG>(J, chunk, rp, cb, q0); break;
    case 3: gram_strip<TX, NB, 3, RG>(J, chunk, rp, cb, q0); break;
    default: gram_strip<TX, NB, 4, RG>(J, chunk, rp, cb, q0); break;
  }
}

// Strips run in XCD order, so the strips of one chunk (which share its rows)
// run on one XCD and share its L2.
// One strip height per kernel (the host gives every job of a launch the
// same rgs), so each keeps its own register budget.
template <typename TX, int RG>
__global__ __launch_bounds__(64) void k_gram(const GramJob* __restrict__ jobs,
                                             const int* __restrict__ pre, int nj, int ntiles) {
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  if (t >= ntiles) return;
  const int jb = find_side(pre, nj, t);
  const GramJob J = jobs[jb];
  gram_tile<TX, RG>(J, J.r1 + J.r2, t - pre[jb]);
}

// ------------------------------------------------------------- k_reduce --
// Fixed-order sum over partials.  SYM: the input holds only the 16 x 16
// groups with (row group <= column group) below nz (k_gram's strips); entries
// below them are mirrored, rows and columns at and past nz are zero.
template <typename TI, typename TO, bool SYM>
__global__ __launch_bounds__(256) void k_reduce(const RedJob* __restrict__ jobs,
                                                const int* __restrict__ pre, int nj) {
  const int jb = find_side(pre, nj, blockIdx.x);
  const RedJob J = jobs[jb];
  const int64_t i = (int64_t)(blockIdx.x - pre[jb]) * 256 + threadIdx.x;
  const int64_t cnt = (int64_t)J.rows * J.cols;
  if (i < cnt) {
    int r = (int)(i / J.cols), c = (int)(i - (int64_t)r * J.cols);
    int64_t src;
    if (SYM && (r >> 4) > (c >> 4)) src = (int64_t)c * J.ldi + r;
    else src = (int64_t)r * J.ldi + c;
    const TI* in = (const TI*)J.in;
    double s = 0.0;
    if (!SYM || (r < J.nz && c < J.nz)) {
      // eight loads in flight, then their sum in the same fixed order
      int p = 0;
      for (; p + 8 <= J.nparts; p += 8) {
        TI v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = in[(int64_t)(p + u) * J.stride + src];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += (double)v[u];
      }
      for (; p < J.nparts; ++p) s += (double)in[(int64_t)p * J.stride + src];
    }
    ((TO*)J.out)[(int64_t)r * J.ldo + c] = (TO)s;
  }
}

// ---------------------------------------------------------------- launch --
template <int P, typename TA, typename TB, typename TD, int JS>
static void launch_ab_js(int ct, const AbJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  switch (ct) {
    case 1: hipLaunchKernelGGL((k_ab<P, TA, TB, TD, 1, JS>), dim3(tiles), dim3(256), 0, st, j, pre, nj); break;
    case 2: hipLaunchKernelGGL((k_ab<P, TA, TB, TD, 2, JS>), dim3(tiles), dim3(256), 0, st, j, pre, nj); break;
    case 4: hipLaunchKernelGGL((k_ab<P, TA, TB, TD, 4, JS>), dim3(tiles), dim3(256), 0, st, j, pre, nj); break;
    case 8: hipLaunchKernelGGL((k_ab<P, TA, TB, TD, 8, JS>), dim3(tiles), dim3(256), 0, st, j, pre, nj); break;
    default: hipLaunchKernelGGL((k_ab<P, TA, TB, TD, 16, JS>), dim3(tiles), dim3(256), 0, st, j, pre, nj); break;
  }
}

// kinds: A/B/D element types given as 0 = double, 1 = float
void launch_ab(int prec, int ta, int tb, int td, int ct, int js, const AbJob* j, const int* pre,
               int nj, int tiles, hipStream_t st) {
#define AB_CASE(PP, A_, B_, D_)                                                        \
  if (js == 4) launch_ab_js<PP, A_, B_, D_, 4>(ct, j, pre, nj, tiles, st);              \
  else if (js == 2) launch_ab_js<PP, A_, B_, D_, 2>(ct, j, pre, nj, tiles, st);         \
  else launch_ab_js<PP, A_, B_, D_, 1>(ct, j, pre, nj, tiles, st);
  if (prec == P64) {
    // fp64 path: A, D double; B double or float (fp32-stored G)
    if (tb == 0) { AB_CASE(P64, double, double, double) }
    else { AB_CASE(P64, double, float, double) }
  } else if (prec == P32) {
    if (ta == 0 && tb == 1 && td == 1) { AB_CASE(P32, double, float, float) }
    else if (ta == 1 && tb == 1 && td == 1) { AB_CASE(P32, float, float, float) }
    else if (ta == 1 && tb == 1 && td == 0) { AB_CASE(P32, float, float, double) }
    else if (ta == 0 && tb == 1 && td == 0) { AB_CASE(P32, double, float, double) }
    else { AB_CASE(P32, float, double, float) }
  } else {
    if (tb == 1) { AB_CASE(PBF, float, float, float) }
    else { AB_CASE(PBF, float, double, float) }
  }
#undef AB_CASE
}

void launch_gen(bool f64, const GenJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  if (f64) hipLaunchKernelGGL((k_gen<double, true>), dim3(tiles), dim3(256), 0, st, j, pre, nj);
  else hipLaunchKernelGGL((k_gen<float, false>), dim3(tiles), dim3(256), 0, st, j, pre, nj);
}

void launch_gram(int tx, int rgs, const GramJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  const dim3 grid(xcd_grid(tiles));
  if (tx == 0 && rgs == 2) hipLaunchKernelGGL((k_gram<double, 2>), grid, dim3(64), 0, st, j, pre, nj, tiles);
  else if (tx == 0) hipLaunchKernelGGL((k_gram<double, 1>), grid, dim3(64), 0, st, j, pre, nj, tiles);
  else if (rgs == 2) hipLaunchKernelGGL((k_gram<float, 2>), grid, dim3(64), 0, st, j, pre, nj, tiles);
  else hipLaunchKernelGGL((k_gram<float, 1>), grid, dim3(64), 0, st, j, pre, nj, tiles);
}

void launch_reduce(int ti, int to, bool sym, const RedJob* j, const int* pre, int nj, int tiles,
                   hipStream_t st) {
  if (sym) hipLaunchKernelGGL((k_reduce<double, double, true>), dim3(tiles), dim3(256), 0, st, j, pre, nj);
  else if (ti == 0 && to == 0) hipLaunchKernelGGL((k_reduce<double, double, false>), dim3(tiles), dim3(256), 0, st, j, pre, nj);
  else if (ti == 1 && to == 1) hipLaunchKernelGGL((k_reduce<float, float, false>), dim3(tiles), dim3(256), 0, st, j, pre, nj);
  else if (ti == 1 && to == 0) hipLaunchKernelGGL((k_reduce<float, double, false>), dim3(tiles), dim3(256), 0, st, j, pre, nj);
  else hipLaunchKernelGGL((k_reduce<double, float, false>), dim3(tiles), dim3(256), 0, st, j, pre, nj);
}

void launch_zerog(const ZeroJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  hipLaunchKernelGGL(k_zerog, dim3(tiles), dim3(256), 0, st, j, pre, nj);
}

void launch_zero(void* p, int64_t bytes, hipStream_t st) {
  int64_t nw = bytes / 4;
  if (nw <= 0) return;
  int64_t blocks = (nw + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t*)p, nw);
}

}  // namespace rg
