// Small dense FP64 steps, one workgroup (1024 threads) per matrix or pair.
//
//  k_chol     : Cholesky of the CholeskyQR Gram and the inverse of its lower
//               factor (the orthonormalisation replacing Algorithm 1's QR),
//               blocked, the Gram in registers
//  k_small    : the compressed-pair GSVD of Algorithm 2 with the truncation
//               reading: eigen-decomposition of M = B B^T (one-sided Jacobi),
//               the rank-t joint basis L = [L1; L2], the SVD of L1 (one-sided
//               Jacobi with accumulated Y), beta from L2 Y, and the
//               comparative quantities theta, P1, P2, D1, D2 of Sec. 1
//  k_rowsign  : sign convention (largest-magnitude entry of each row of R > 0)
#include "common.hpp"
#include "jobs.hpp"
#include "small.hpp"
#include "launch.hpp"

namespace rg {

// ---------------------------------------------------------------- k_chol --
// Largest entry and sum of the Gram's diagonal (N entries, ld np) into
// *md_s and *tr_s: wave 0 strides the diagonal and reduces by shuffles.  A
// NaN or infinity anywhere in the Gram shows in the sum of its diagonal (a
// Gram's diagonal holds the squared norms its entries are formed from).
__device__ __forceinline__ void gram_diag_stats(const CholJob& J, int N, int np, double* md_s, double* tr_s) {
  if (threadIdx.x < 64) {
    const int ln = threadIdx.x;
    double md = 0.0, tr = 0.0;
    for (int i = ln; i < N; i += 64) { const double d = J.gram[(int64_t)i * np + i]; md = fmax(md, d); tr += d; }
    for (int o = 32; o > 0; o >>= 1) { md = fmax(md, __shfl_xor(md, o, 64)); tr += __shfl_xor(tr, o, 64); }
    if (ln == 0) { *md_s = md; *tr_s = tr; }
  }
}

// Lane ln's part of the sum of squares of a column of n <= SMALL_MAXN entries
// in global memory (rows ln, ln + 64, ...), for a wave to reduce: all of the
// lane's loads are issued before the first add (a loop over a runtime count
// waits for each load in turn); the adds keep row order (the zeros past n add
// nothing).  Rows below `split` go to *lo, the rest to *hi.
static_assert(SMALL_MAXN <= 8 * 64, "a lane holds at most eight rows of a column");
__device__ __forceinline__ void col_sumsq2(const double* col, int n, int split, int ln, double* lo, double* hi) {
  double v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int r = ln + 64 * u;
    v[u] = r < n ? col[r] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    if (ln + 64 * u < split) *lo += v[u] * v[u];
    else *hi += v[u] * v[u];
  }
}
__device__ __forceinline__ double col_sumsq(const double* col, int n, int ln) {
  double s = 0.0, none = 0.0;
  col_sumsq2(col, n, n, ln, &s, &none);
  return s;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Factor of one 16 x 16 diagonal block A = R^T R by one wave, with X = R^{-T}
// (the inverse of the lower factor L = R^T): elimination on the rows of
// [A | I].  Lane (i, h) = (lane / 4, lane % 4) holds entries 4h .. 4h + 3 of
// row i of both halves.  Step k scales row k by 1 / sqrt(pivot) (the hardware
// estimate and two Newton steps), publishes it in `row` (32 doubles of LDS,
// read by the same wave in order, so no barrier), and every row below
// subtracts R_ki times it: the left half becomes R, the right half the
// forward substitution L^{-1}.  On exit a[e] = R[i][4h + e] (4h + e >= i) and
// b[e] = X[i][4h + e] (4h + e <= i).  blk(i, c) gives A[i][c] for c >= i;
// d0(r) is the original diagonal entry of row r, for the pivot tests.
// trunc: a pivot below CHOL_TRUNC_REL of it gives a zero row k of R and zero
// row and column k of X (the row eliminates nothing).  Returns whether a
// pivot failed (not finite, or not above both rel d0(k) and floor), which
// cannot happen for a dropped row.
template <typename BLK, typename D0>
__device__ __forceinline__ bool factor_diag16(BLK blk, D0 d0, double* row, double (&a)[4], double (&b)[4],
                                              bool trunc, double rel, double floor) {
  const int ln = threadIdx.x & 63, i = ln >> 2, h = ln & 3;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int c = 4 * h + e;
    a[e] = c >= i ? blk(i, c) : blk(c, i);
    b[e] = c == i ? 1.0 : 0.0;
  }
  const double d0l = d0(ln & 15);
  bool bad = false;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const double piv = readlane_f64(a[k & 3], 4 * k + (k >> 2));
    const double dk0 = readlane_f64(d0l, k);
    if (trunc && isfinite(piv) && !(piv > CHOL_TRUNC_REL * dk0 && piv > 0.0)) {
      if (i == k) {
#pragma unroll
        for (int e = 0; e < 4; ++e) { a[e] = 0.0; b[e] = 0.0; }
      }
      continue;
    }
    if (!(piv > rel * dk0) || !(piv > floor) || !(piv > 0.0) || !isfinite(piv)) bad = true;
    const double hp = 0.5 * piv;
    double y = __builtin_amdgcn_rsq(piv);
    y = y * fma(-hp * y, y, 1.5);
    y = y * fma(-hp * y, y, 1.5);
    if (i == k) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        a[e] *= y;
        b[e] *= y;
        row[4 * h + e] = a[e];
        row[16 + 4 * h + e] = b[e];
      }
    }
    // the row is written before any lane reads it, and read before the next
    // step writes it (LDS serves a wave in program order; the wave barrier
    // keeps the compiler from moving the accesses across)
    __builtin_amdgcn_wave_barrier();
    if (i > k) {
      const double rki = row[i];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        a[e] = fma(-rki, row[4 * h + e], a[e]);
        b[e] = fma(-rki, row[16 + 4 * h + e], b[e]);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  return bad;
}

// Cholesky A = R^T R of an N x N Gram (N <= CB_MAXN) and X = R^{-T}, the
// inverse of the lower factor L = R^T, right-looking in 16 x 16 blocks.
//
// The upper triangle's nb (nb + 1) / 2 blocks (nb = ceil(N / 16); the order
// is padded to 16 nb with the identity) are numbered column by column; block
// f lives in registers, in slot f / CB_W of wave f % CB_W, as one FP64 MFMA
// accumulator (lane (g, c) holds rows 4q + g, q < 4, of column c).  The same
// slots carry the inverse: block (i, j) holds A[i][j] until step i turns it
// into R[i][j], and from then on T[j][i], the right-hand side of the block
// forward substitution L X = I, until step j finishes X[j][i].  Step kb:
//   1. the owner of A[kb][kb] publishes it; wave 0 factors it, R_kk^T R_kk,
//      one column per lane with scalar broadcasts, and forms X_kk = R_kk^{-T};
//   2. the panel R[kb][j] = X_kk A[kb][j] (j > kb) and the finished row of
//      the inverse X[kb][i] = X_kk T[kb][i] (i < kb) go to LDS (X also to
//      sinv);
//   3. trailing updates on FP64 MFMA: A[i][j] -= R[kb][i]^T R[kb][j]
//      (kb < i <= j) and T[j][i] -= R[kb][j]^T X[kb][i] (i <= kb < j).
// Pivot test and recovery: a pivot that is not positive and above 1e-15 of
// its original diagonal restarts the factorisation with a diagonal shift
// (1e-14 N max diag, growing 100-fold, at most 8 times; the run's flag bit
// records it), unless `trunc` is set, where a pivot below CHOL_TRUNC_REL of
// its original diagonal marks a row numerically inside the span of the rows
// before it: that row of R and of X becomes zero and it eliminates nothing.
// A non-finite Gram leaves X = 0 and raises FLAG_NONFINITE.
constexpr int CB_MAXN = 256, CB_MAXNB = CB_MAXN / 16, CB_W = 8;
constexpr int CB_NBLK = CB_MAXNB * (CB_MAXNB + 1) / 2;
constexpr int CB_SLOTS = (CB_NBLK + CB_W - 1) / CB_W;
constexpr int CB_LD = CB_MAXN + 4;   // panel row stride (doubles): rows of a k-step fall on different banks
constexpr size_t CB_LDS_BYTES = (size_t)(2 * 16 * CB_LD + 2 * 256 + CB_MAXN) * sizeof(double);

__global__ __launch_bounds__(64 * CB_W) void k_chol(const CholJob* __restrict__ jobs, int nj) {
  extern __shared__ double lds[];
  __shared__ unsigned char bi_s[CB_NBLK], bj_s[CB_NBLK];
  __shared__ int bad_s;
  __shared__ double trace_s, maxd_s;
  const CholJob J = jobs[blockIdx.x];
  const int N = J.N, np = J.npad;
  const int nb = (N + 15) >> 4, nblk = nb * (nb + 1) / 2;
  const int tid = threadIdx.x, wave = tid >> 6, ln = tid & 63, g = ln >> 4, c16 = ln & 15;
  double* panel = lds;                 // 16 x CB_LD: R[kb][j] in columns 16 j .. 16 j + 15
  double* xrow = panel + 16 * CB_LD;   // 16 x CB_LD: X[kb][i] in columns 16 i .. 16 i + 15
  double* Dk = xrow + 16 * CB_LD;      // A[kb][kb], row-major 16 x 16
  double* Xk = Dk + 256;               // X_kk, row-major 16 x 16 (lower)
  double* d0 = Xk + 256;               // the Gram's diagonal (pivot tests)
  if (tid < nblk) {
    int f = tid, j = 0;
    while (f > j) { f -= j + 1; ++j; }   // column j of the upper triangle holds j + 1 blocks
    bi_s[tid] = (unsigned char)f;
    bj_s[tid] = (unsigned char)j;
  }
  gram_diag_stats(J, N, np, &maxd_s, &trace_s);
  for (int i = tid; i < 16 * nb; i += 64 * CB_W) d0[i] = i < N ? J.gram[(int64_t)i * np + i] : 1.0;
  for (int e = tid; e < np * np; e += 64 * CB_W) J.sinv[e] = 0.0;
  __syncthreads();
  if (!isfinite(trace_s)) {
    if (tid == 0 && J.info) atomicOr(J.info + 4, FLAG_NONFINITE);
    return;
  }
  const double maxdiag = maxd_s;
  double shift = J.shift0 > 0.0 ? J.shift0 * trace_s : 0.0;
  bool shifted = false;
  d4 S[CB_SLOTS];
  for (int attempt = 0;; ++attempt) {
    // the Gram's upper blocks (+ shift on the diagonal; identity past N)
#pragma unroll
    for (int s = 0; s < CB_SLOTS; ++s) {
      const int f = CB_W * s + wave;
      d4 v = {0.0, 0.0, 0.0, 0.0};
      if (f < nblk) {
        const int col = 16 * bj_s[f] + c16;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = 16 * bi_s[f] + 4 * q + g;
          v[q] = (row < N && col < N) ? J.gram[(int64_t)row * np + col] + (row == col ? shift : 0.0)
                                      : (row == col ? 1.0 : 0.0);
        }
      }
      S[s] = v;
    }
    if (tid == 0) bad_s = 0;
    __syncthreads();
    for (int kb = 0; kb < nb; ++kb) {
      const int o = 16 * kb;
      // 1. the diagonal block, factored by wave 0
      const int fd = kb * (kb + 1) / 2 + kb;
      if (wave == fd % CB_W) {
#pragma unroll
        for (int s = 0; s < CB_SLOTS; ++s)
          if (s == fd / CB_W)
#pragma unroll
            for (int q = 0; q < 4; ++q) Dk[(4 * q + g) * 16 + c16] = S[s][q];
      }
      __syncthreads();
      if (wave == 0) {
        // Dk serves as the factor's row buffer once read
        double a[4], b[4];
        const bool bad = factor_diag16([&](int r, int c) { return Dk[r * 16 + c]; },
                                       [&](int r) { return d0[o + r]; }, Dk, a, b, J.trunc != 0, 1e-15, 0.0);
        const int i = ln >> 2, h = ln & 3;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = 4 * h + e;
          const double v = c <= i ? b[e] : 0.0;
          Xk[i * 16 + c] = v;
          xrow[i * CB_LD + o + c] = v;
          if (c <= i && o + i < N) J.sinv[(int64_t)(o + i) * np + o + c] = v;
        }
        if (bad && ln == 0) bad_s = 1;
      }
      __syncthreads();
      if (bad_s) break;
      // 2. panel row kb of R and row kb of the inverse
#pragma unroll
      for (int s = 0; s < CB_SLOTS; ++s) {
        const int f = CB_W * s + wave;
        if (f >= nblk) continue;
        const int bi = bi_s[f], bj = bj_s[f];
        if (bi == bj || (bi != kb && bj != kb)) continue;
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc = mma64(Xk[c16 * 16 + 4 * kk + g], S[s][kk], acc);
        if (bi == kb) {
          // R[kb][bj]; the slot now holds T[bj][kb], which starts at zero
#pragma unroll
          for (int q = 0; q < 4; ++q) panel[(4 * q + g) * CB_LD + 16 * bj + c16] = acc[q];
          S[s] = d4{0.0, 0.0, 0.0, 0.0};
        } else {
          // X[kb][bi] (bj == kb > bi), final
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int row = o + 4 * q + g;
            xrow[(4 * q + g) * CB_LD + 16 * bi + c16] = acc[q];
            if (row < N) J.sinv[(int64_t)row * np + 16 * bi + c16] = acc[q];
          }
        }
      }
      __syncthreads();
      // 3. trailing updates
#pragma unroll
      for (int s = 0; s < CB_SLOTS; ++s) {
        const int f = CB_W * s + wave;
        if (f >= nblk) continue;
        const int bi = bi_s[f], bj = bj_s[f];
        if (bj <= kb) continue;
        // A[bi][bj] -= R[kb][bi]^T R[kb][bj]  or  T[bj][bi] -= R[kb][bj]^T X[kb][bi]
        const double* pa = panel + 16 * (bi > kb ? bi : bj) + c16;
        const double* pb = (bi > kb ? panel + 16 * bj : xrow + 16 * bi) + c16;
        d4 acc = S[s];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int m = 4 * kk + g;
          acc = mma64(-pa[m * CB_LD], pb[m * CB_LD], acc);
        }
        S[s] = acc;
      }
      __syncthreads();
    }
    if (!bad_s) break;
    if (attempt >= 8 || !(maxdiag > 0.0)) {
      for (int e = tid; e < np * np; e += 64 * CB_W) J.sinv[e] = 0.0;
      if (tid == 0 && J.info) atomicOr(J.info + 4, (1 << J.flagbit) | FLAG_CHOL_FAIL);
      return;
    }
    shift = (shift == 0.0) ? 1e-14 * maxdiag * (double)N : shift * 100.0;
    shifted = true;
    __syncthreads();
  }
  if (tid == 0 && shifted && J.info) atomicOr(J.info + 4, 1 << J.flagbit);
}

// ------------------------------------------------------ one-sided Jacobi --
// Orthogonalises the nc columns of A (column-major, ld lda) by plane
// rotations (Hestenes) over rows [0, nr).  Parallel round-robin ordering:
// each round pairs every column once.
//
// G lanes hold one column pair, EM >= nr / G entries of each column per
// lane, so a pair's three inner products reduce in log2(G)
// shuffle steps and 1024 / G pairs rotate at once.  When A fits in the
// LDS buffer it is copied there for all sweeps; otherwise the rounds work
// on A in global memory.
//
// topk > 0: a pair is skipped when both columns have squared norm below a
// quarter of the topk-th largest (norms refreshed every sweep); at
// convergence the topk dominant columns are orthogonal to every other
// column, so they span the dominant invariant subspace.  Returns the number
// of sweeps used (maxsweep + 1 when not converged).
// One column pair (p, q) held by G consecutive lanes: lane j owns rows
// j + G e (e < EM) of both columns.  Inner products over rows [0, nd), the
// rotation over rows [0, nr).  The pair turns unless
// |gamma| <= tol sqrt(alpha beta) (tested on squares); when thr >= 0 and
// one column is below thr (a dominant column against a sub-threshold one)
// it also needs |gamma| > tol max(alpha, beta): such a rotation turns the
// dominant column by about gamma / max(alpha, beta), and the dominant
// subspace is settled below that.  Returns whether the pair turned.
// Rotation of a column pair from its inner products alpha = ||x||^2,
// beta = ||y||^2, gamma = x^T y.  The pair turns unless
// |gamma| <= tol sqrt(alpha beta) (tested on squares); when thr >= 0 and
// one column is below thr (a dominant column against a sub-threshold one)
// it also needs |gamma| > tol max(alpha, beta): such a rotation turns the
// dominant column by about gamma / max(alpha, beta), and the dominant
// subspace is settled below that.  On a turn, (c, s) with
// x' = c x - s y, y' = s x + c y orthogonal.
__device__ __forceinline__ bool jacobi_turn(double al, double be, double ga, bool live, double tol, double thr,
                                            double& c, double& s) {
  const double g2 = ga * ga, tol2 = tol * tol;
  bool turn = live && al > 0.0 && be > 0.0 && g2 > tol2 * (al * be);
  if (turn && thr >= 0.0 && fmin(al, be) < thr) {
    const double mx = fmax(al, be);
    turn = g2 > tol2 * (mx * mx);
  }
  if (turn) {
    // t = tan of the angle that zeroes gamma, the root of
    // t^2 + 2 zeta t - 1 = 0 (zeta = (beta - alpha) / (2 gamma)) of smaller
    // magnitude, written without zeta: 2 gamma sign(d) / (|d| + sqrt(d^2 + 4 gamma^2))
    const double d = be - al;
    const double t = (d >= 0.0 ? 2.0 * ga : -2.0 * ga) / (fabs(d) + sqrt(fma(d, d, 4.0 * g2)));
    c = rsqrt(fma(t, t, 1.0));
    s = c * t;
  }
  return turn;
}

// One column pair (p, q) of nr rows held by G consecutive lanes: lane j
// owns rows j + G e (e < EM) of both columns.  Rows past nr read the last
// row (in bounds) scaled by zero, so every load is unconditional.  Returns
// whether the pair turned.
template <int G, int EM>
__device__ __attribute__((always_inline)) inline bool
pair_step(double* Lp, double* Lq, int j, int nr, bool live, double tol, double thr, double& rel2) {
  double x[EM], y[EM];
  double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
  for (int e = 0; e < EM; ++e) {
    const int r = j + G * e;
    const int rr = r < nr ? r : nr - 1;
    const double w = (live && r < nr) ? 1.0 : 0.0;
    x[e] = Lp[rr] * w;
    y[e] = Lq[rr] * w;
    al = fma(x[e], x[e], al);
    be = fma(y[e], y[e], be);
    ga = fma(x[e], y[e], ga);
  }
  al = group_sum<G>(al);
  be = group_sum<G>(be);
  ga = group_sum<G>(ga);
  double c, s;
  const bool turn = jacobi_turn(al, be, ga, live, tol, thr, c, s);
  if (turn) {
    rel2 = fmax(rel2, ga * ga / (al * be));
#pragma unroll
    for (int e = 0; e < EM; ++e) {
      const int r = j + G * e;
      if (r < nr) {
        Lp[r] = c * x[e] - s * y[e];
        Lq[r] = s * x[e] + c * y[e];
      }
    }
  }
  return turn;
}

// The same on LDS columns padded to G * EM rows whose rows past the order
// hold zeros (they stay zero under rotations): no bounds tests.
template <int G, int EM>
__device__ __attribute__((always_inline)) inline bool
pair_step_padded(double* Lp, double* Lq, int j, bool live, double tol, double thr, double& rel2) {
  double x[EM], y[EM];
  double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
  for (int e = 0; e < EM; ++e) {
    x[e] = Lp[j + G * e];
    y[e] = Lq[j + G * e];
    al = fma(x[e], x[e], al);
    be = fma(y[e], y[e], be);
    ga = fma(x[e], y[e], ga);
  }
  al = group_sum<G>(al);
  be = group_sum<G>(be);
  ga = group_sum<G>(ga);
  double c, s;
  const bool turn = jacobi_turn(al, be, ga, live, tol, thr, c, s);
  if (turn) {
    rel2 = fmax(rel2, ga * ga / (al * be));
#pragma unroll
    for (int e = 0; e < EM; ++e) {
      Lp[j + G * e] = c * x[e] - s * y[e];
      Lq[j + G * e] = s * x[e] + c * y[e];
    }
  }
  return turn;
}

// The same with column p held in registers (x, EM rows per lane) across
// steps: only column q passes through LDS.
template <int G, int EM>
__device__ __attribute__((always_inline)) inline bool
pair_step_reg(double (&x)[EM], double* Lq, int j, bool live, double tol, double thr, double& rel2) {
  double y[EM];
  double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
  for (int e = 0; e < EM; ++e) {
    y[e] = Lq[j + G * e];
    al = fma(x[e], x[e], al);
    be = fma(y[e], y[e], be);
    ga = fma(x[e], y[e], ga);
  }
  al = group_sum<G>(al);
  be = group_sum<G>(be);
  ga = group_sum<G>(ga);
  double c, s;
  const bool turn = jacobi_turn(al, be, ga, live, tol, thr, c, s);
  if (turn) {
    rel2 = fmax(rel2, ga * ga / (al * be));
#pragma unroll
    for (int e = 0; e < EM; ++e) {
      const double xn = c * x[e] - s * y[e];
      Lq[j + G * e] = s * x[e] + c * y[e];
      x[e] = xn;
    }
  }
  return turn;
}

// Round-robin tournament on m1 + 1 players (m1 odd): in round `round`,
// slot pi (0 <= pi <= m1 / 2) pairs players u and v; slot 0 keeps player 0
// and the others rotate, so every pair meets once in m1 rounds.
__device__ inline void tournament(int pi, int round, int m1, int& u, int& v) {
  u = 0;
  if (pi > 0) { u = pi - 1 + round; if (u >= m1) u -= m1; u += 1; }
  v = m1 - pi - 1 + round;          // m1 - pi >= 1
  if (v >= m1) v -= m1;
  v += 1;
}

template <int G, int EM>
__device__ __attribute__((always_inline)) inline void
jacobi_round(double* L, int ldl, int nr, int nc, int round, double thr, const double* nrm2,
             double tol, int* rotated, double& rel2) {
  constexpr int SLOTS = 1024 / G;
  const int tid = threadIdx.x, grp = tid / G, j = tid % G;
  const int nc2 = nc + (nc & 1), npairs = nc2 / 2, m1 = nc2 - 1;
  bool any = false;
  for (int p0 = 0; p0 < npairs; p0 += SLOTS) {
    const int pi = p0 + grp;
    int p = -1, q = -1;
    if (pi < npairs) {
      int u, v;
      tournament(pi, round, m1, u, v);
      if (u < nc && v < nc && !(thr >= 0.0 && nrm2[u] < thr && nrm2[v] < thr)) { p = u; q = v; }
    }
    const bool live = p >= 0;
    any |= pair_step<G, EM>(L + (live ? p : 0) * ldl, L + (live ? q : 0) * ldl, j, nr, live, tol, thr, rel2);
  }
  if (any) *rotated = 1;
}

// All sweeps on W (ld ldw): LDS copy or A itself.
template <int G, int EM>
__device__ __attribute__((always_inline)) inline int
jacobi_sweeps(double* W, int ldw, int nr, int nc, double tol, int maxsweep, int topk, double* nrm2,
              int* scratch, double* kth_slot) {
  const int tid = threadIdx.x, wave = tid >> 6, ln = tid & 63;
  const int nc2 = nc + (nc & 1);
  for (int sweep = 0; sweep < maxsweep; ++sweep) {
    for (int c = wave; c < nc; c += 16) {
      double s = 0.0;
      for (int i = ln; i < nr; i += 64) { const double v = W[(int64_t)c * ldw + i]; s += v * v; }
      s = wave_sum(s);
      if (ln == 0) nrm2[c] = s;
    }
    if (tid == 0) { scratch[0] = 0; scratch[1] = 0; }
    __syncthreads();
    double thr = -1.0;
    if (topk > 0 && topk < nc) {
      if (tid < nc) {
        const double v = nrm2[tid];
        int r = 0;
        for (int j2 = 0; j2 < nc; ++j2) { const double w = nrm2[j2]; r += (w > v) || (w == v && j2 < tid); }
        if (r == topk - 1) *kth_slot = v;
      }
      __syncthreads();
      thr = 0.25 * *kth_slot;
    }
    double rel2 = 0.0;   // largest gamma^2 / (alpha beta) this thread turned
    for (int round = 0; round < nc2 - 1; ++round) {
      jacobi_round<G, EM>(W, ldw, nr, nc, round, thr, nrm2, tol, scratch, rel2);
      __syncthreads();
    }
    // Jacobi converges quadratically: a sweep whose turns all had
    // |gamma| < sqrt(tol) sqrt(alpha beta) leaves the next sweep only turns
    // below tol, so it ends the sweeps without that checking sweep
    for (int o = 32; o > 0; o >>= 1) rel2 = fmax(rel2, __shfl_xor(rel2, o, 64));
    if (ln == 0 && rel2 > 0.0) atomicMax(scratch + 1, __float_as_int((float)fmin(rel2, 1.0)));
    __syncthreads();
    const int any = scratch[0];
    const float rmax = __int_as_float(scratch[1]);
    __syncthreads();
    if (!any || rmax < (float)tol) return sweep + 1;
  }
  return maxsweep + 1;
}

template <int G, int EM>
__device__ __attribute__((always_inline)) inline int
jacobi_os(double* A, int lda, int nr, int nc, double tol, int maxsweep, int topk, double* nrm2,
          int* scratch, double* kth_slot, double* lds, int cap) {
  const int tid = threadIdx.x;
  if (nc < 2) return 0;
  if ((int64_t)nc * nr > cap)
    return jacobi_sweeps<G, EM>(A, lda, nr, nc, tol, maxsweep, topk, nrm2, scratch, kth_slot);
  for (int e = tid; e < nc * nr; e += 1024) {
    const int c = e / nr, r = e - c * nr;
    lds[e] = A[(int64_t)c * lda + r];
  }
  __syncthreads();
  const int sw = jacobi_sweeps<G, EM>(lds, nr, nr, nc, tol, maxsweep, topk, nrm2, scratch, kth_slot);
  for (int e = tid; e < nc * nr; e += 1024) {
    const int c = e / nr, r = e - c * nr;
    A[(int64_t)c * lda + r] = lds[e];
  }
  __syncthreads();
  return sw;
}

// rank of key[i] among n keys, descending, ties by index (for sorting).  A
// NaN key ranks below every number, so the ranks stay a permutation and
// every index formed from them stays in range.
__device__ inline int rank_desc(const double* key, int n, int i) {
  const double v = isnan(key[i]) ? -INFINITY : key[i];
  int r = 0;
  for (int j = 0; j < n; ++j) {
    const double w = isnan(key[j]) ? -INFINITY : key[j];
    r += (w > v) || (w == v && j < i);
  }
  return r;
}

// --------------------------------------------------------------- k_small --
// C = A B in one workgroup on FP64 MFMA: element (i, k) of A at
// A[i sai + k sak], element (k, j) of B at B[k sbk + j sbj]; I x J output,
// inner order K.  A wave takes a strip of TW 16 x 16 output tiles along j
// at a time: per step of 4 in k it loads one A fragment and TW B fragments
// and runs TW independent MFMA chains (a single tile's chain waits on its
// loads at every step).  store(i, j, v) receives every output element once;
// with SYM (A B symmetric, I == J) only strips reaching the diagonal are
// formed and store(i, j, v) is called for i <= j.
template <bool SYM, typename Store>
__device__ __attribute__((always_inline)) inline void
wg_gemm64(const double* A, int64_t sai, int64_t sak, const double* B, int64_t sbk, int64_t sbj, int I, int J,
          int K, Store store) {
  constexpr int TW = 4;
  const int wave = threadIdx.x >> 6, ln = threadIdx.x & 63, r16 = ln & 15, g = ln >> 4;
  const int ti = (I + 15) / 16, tj = (J + 15) / 16, ts = (tj + TW - 1) / TW;
  for (int strip = wave; strip < ti * ts; strip += 16) {
    const int bi = strip / ts, bs = strip - bi * ts;
    if (SYM && TW * bs + TW - 1 < bi) continue;
    const int ia = bi * 16 + r16;
    const bool oka = ia < I;
    const double* pa = A + (oka ? ia : 0) * sai;
    const double* pb[TW];
    bool okb[TW];
#pragma unroll
    for (int u = 0; u < TW; ++u) {
      const int jb = (TW * bs + u) * 16 + r16;
      okb[u] = jb < J;
      pb[u] = B + (okb[u] ? jb : 0) * sbj;
    }
    d4 acc[TW];
#pragma unroll
    for (int u = 0; u < TW; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + g;
      const double a = (oka && k < K) ? pa[k * sak] : 0.0;
#pragma unroll
      for (int u = 0; u < TW; ++u) {
        const double b = (okb[u] && k < K) ? pb[u][k * sbk] : 0.0;
        acc[u] = mma64(a, b, acc[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < TW; ++u) {
      const int jb = (TW * bs + u) * 16 + r16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = bi * 16 + out_row<0>(g, q);
        if (i < I && jb < J && (!SYM || i <= jb)) store(i, jb, acc[u][q]);
      }
    }
  }
}

// Diagonally pivoted Cholesky of a K x K PSD matrix S (row-major, ld ld,
// both triangles; overwritten): P^T (S + shift I) P = R^T R.  Column k of F
// (K x K, column-major, ld K) is row k of R scattered back to S's row order,
// so F F^T = S + shift I and the columns of F are graded (large first).
// Stops at the numerical rank (pivot <= 1e-15 of the largest diagonal) and
// returns it; *trace receives the trace of S + shift I.
//
// Right-looking in panels of PC_B columns: a step reads the pivot's row of
// the trailing matrix (contiguous, by symmetry its column), subtracts the
// panel's earlier columns (held in LDS, Fb: PC_B x K), and scales; after a
// panel the trailing matrix takes the panel's rank-PC_B update on MFMA.
// diag/act: shared scratch of K entries; one thread per row.
constexpr int PC_B = 16;

// (value, index) maximum over the 64 lanes of a wave, ties to the smaller
// index (negative index: no candidate); every lane ends with the result.
__device__ __forceinline__ void wave_argmax(double& v, int& j) {
  auto take = [&](double v2, int j2) {
    if (v2 > v || (v2 == v && j2 >= 0 && (j < 0 || j2 < j))) { v = v2; j = j2; }
  };
  take(dpp_f64<0xB1>(v), __builtin_amdgcn_update_dpp(0, j, 0xB1, 0xF, 0xF, false));
  take(dpp_f64<0x4E>(v), __builtin_amdgcn_update_dpp(0, j, 0x4E, 0xF, 0xF, false));
  take(dpp_f64<0x141>(v), __builtin_amdgcn_update_dpp(0, j, 0x141, 0xF, 0xF, false));
  take(dpp_f64<0x140>(v), __builtin_amdgcn_update_dpp(0, j, 0x140, 0xF, 0xF, false));
  take(swz16_f64(v), __builtin_amdgcn_ds_swizzle(j, 0x401F));
  take(__shfl_xor(v, 32, 64), __shfl_xor(j, 32, 64));
}
__device__ int pivoted_cholesky(double* S, int64_t ld, int K, double* F, double* diag, int* act, double* Fb,
                                int* piv_j, double* piv_d, double shift, double* trace) {
  const int tid = threadIdx.x;
  for (int e = tid; e < K * K; e += 1024) F[e] = 0.0;
  for (int i = tid; i < K; i += 1024) { diag[i] = S[(int64_t)i * ld + i] + shift; act[i] = 1; }
  __syncthreads();
  double dmax0 = 0.0;
  for (int i = 0; i < K; ++i) dmax0 = fmax(dmax0, diag[i]);
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < K; ++i) tr += diag[i];
    *trace = tr;
  }
  int rank = 0;
  for (int k0 = 0; k0 < K; k0 += PC_B) {
    const int kend = k0 + PC_B < K ? k0 + PC_B : K;
    int k = k0;
    for (; k < kend; ++k) {
      if (tid < 64) {
        double best = -1.0; int bj = -1;
        for (int j = tid; j < K; j += 64)
          if (act[j] && diag[j] > best) { best = diag[j]; bj = j; }
        wave_argmax(best, bj);
        if (tid == 0) { *piv_j = bj; *piv_d = best; }
      }
      __syncthreads();
      const int js = *piv_j;
      const double d = *piv_d;
      if (js < 0 || !(d > 1e-15 * dmax0) || !(d > 0.0)) break;
      const double sd = sqrt(d), rd = 1.0 / sd;
      if (tid < K) {
        double v = 0.0;
        const bool on = act[tid];
        if (tid == js) {
          v = sd;
          act[tid] = 0;
        } else if (on) {
          double a = S[(int64_t)js * ld + tid];
          for (int c = 0; c < k - k0; ++c) a -= Fb[c * K + tid] * Fb[c * K + js];
          v = a * rd;
          diag[tid] -= v * v;
        }
        Fb[(k - k0) * K + tid] = v;
        F[(int64_t)k * K + tid] = v;
      }
      __syncthreads();
      rank = k + 1;
    }
    if (k < kend) break;
    if (kend < K) {
      wg_gemm64<true>(Fb, 1, K, Fb, K, 1, K, K, kend - k0, [&](int i, int j, double v) {
        S[(int64_t)i * ld + j] -= v;
        if (i != j) S[(int64_t)j * ld + i] -= v;
      });
      __syncthreads();
    }
  }
  __syncthreads();
  return rank;
}

// Unpivoted Cholesky S = R^T R of a K x K SPD matrix in one workgroup,
// right-looking in 16 x 16 blocks on FP64 MFMA with the matrix left in
// global memory (L2): S is row-major (ld), both triangles present; the blocks
// on and above the diagonal are overwritten.  Column k of F (K x K,
// column-major, ld K) receives row k of R, so F F^T = S.  The order is padded
// to a multiple of 16 with the identity (virtually: the padding is never
// stored).  A pivot must exceed CHOL_TRUNC_REL (1e-10) of its row's original
// diagonal and 1e-12 of the largest diagonal, far above the rounding errors
// of the Schur complements (a few u max diag): then the multipliers are
// accurate and no entry of R can grow.  Otherwise (S singular or nearly so,
// where rounding can leave small positive pivots that amplify errors) it
// restores S from its lower triangle and d0 and returns false, and the
// caller falls back to the pivoted form, which stops at the numerical rank.  *trace gets
// the trace of S.  Scratch: d0 (16 ceil(K/16) doubles), panel (16 x ldp,
// ldp >= 16 ceil(K/16)), Xk (256 doubles), all shared; bad_s shared.
__device__ __noinline__ bool chol_unpivoted(double* S, int64_t ld, int K, double* F, double* d0, double* panel, int ldp,
                               double* Xk, int* bad_s, double* trace) {
  const int tid = threadIdx.x, wave = tid >> 6, ln = tid & 63, g = ln >> 4, c16 = ln & 15;
  constexpr int NW = 16;
  const int nb = (K + 15) >> 4;
  auto at = [&](int r, int c) -> double {   // S with the identity padding
    return (r < K && c < K) ? S[(int64_t)r * ld + c] : (r == c ? 1.0 : 0.0);
  };
  for (int e = tid; e < K * K; e += 64 * NW) F[e] = 0.0;
  for (int i = tid; i < 16 * nb; i += 64 * NW) d0[i] = at(i, i);
  if (tid == 0) *bad_s = 0;
  __syncthreads();
  __shared__ double dmax_s;
  if (tid < 64) {
    double tr = 0.0, mx = 0.0;
    for (int i = tid; i < K; i += 64) { tr += d0[i]; mx = fmax(mx, d0[i]); }
    tr = wave_sum(tr);
    for (int o2 = 32; o2 > 0; o2 >>= 1) mx = fmax(mx, __shfl_xor(mx, o2, 64));
    if (tid == 0) { *trace = tr; dmax_s = mx; }
  }
  __syncthreads();
  const double floor = 1e-12 * dmax_s;
  for (int kb = 0; kb < nb; ++kb) {
    const int o = 16 * kb;
    if (wave == 0) {
      // Xk serves as the factor's row buffer until it is written
      double a[4], b[4];
      const bool bad = factor_diag16([&](int r, int c) { return at(o + r, o + c); },
                                     [&](int r) { return d0[o + r]; }, Xk, a, b, false, CHOL_TRUNC_REL, floor);
      const int i = ln >> 2, h = ln & 3;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = 4 * h + e;
        Xk[i * 16 + c] = c <= i ? b[e] : 0.0;            // X_kk = R_kk^{-T}, row i
        if (c >= i) {
          panel[i * ldp + o + c] = a[e];                   // R[o + i][o + c]
          if (o + c < K) F[(int64_t)(o + i) * K + o + c] = a[e];
        }
      }
      if (bad && ln == 0) *bad_s = 1;
    }
    __syncthreads();
    if (*bad_s) {
      for (int e = tid; e < K * K; e += 64 * NW) {
        const int r = e / K, c = e - r * K;
        if (c > r) S[(int64_t)r * ld + c] = S[(int64_t)c * ld + r];
        else if (c == r) S[(int64_t)r * ld + c] = d0[r];
      }
      __syncthreads();
      return false;
    }
    // panel row kb of R: R[kb][jb] = X_kk A[kb][jb]
    for (int jb = kb + 1 + wave; jb < nb; jb += NW) {
      d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) acc = mma64(Xk[c16 * 16 + 4 * kk + g], at(o + 4 * kk + g, 16 * jb + c16), acc);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 4 * q + g, c = 16 * jb + c16;
        panel[r * ldp + c] = acc[q];
        if (o + r < K && c < K) F[(int64_t)(o + r) * K + c] = acc[q];
      }
    }
    __syncthreads();
    // trailing update A[ib][jb] -= R[kb][ib]^T R[kb][jb], kb < ib <= jb
    const int rem = nb - kb - 1;
    for (int tb = wave; tb < rem * (rem + 1) / 2; tb += NW) {
      int ib = 0, tt = tb;
      while (tt >= rem - ib) { tt -= rem - ib; ++ib; }
      const int jb = kb + 1 + ib + tt;
      ib += kb + 1;
      d4 acc;
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = at(16 * ib + 4 * q + g, 16 * jb + c16);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int m = 4 * kk + g;
        acc = mma64(-panel[m * ldp + 16 * ib + c16], panel[m * ldp + 16 * jb + c16], acc);
      }
      // (the strictly lower triangle, diagonal blocks included, keeps the
      // original S for the restore)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * ib + 4 * q + g, c = 16 * jb + c16;
        if (r < K && c < K && r <= c) S[(int64_t)r * ld + c] = acc[q];
      }
    }
    __syncthreads();
  }
  return true;
}

struct SmallShared {
  double keys[SMALL_MAXN];
  double diag[SMALL_MAXN];
  double frow[SMALL_MAXN];
  int perm[SMALL_MAXN];
  int act[SMALL_MAXN];
  int scratch[8];
  int piv_j;
  double piv_d;
  double kth;
  double trace;
};

// G lanes per column pair and EM entries per lane (G * EM >= nr): 16 x 8
// for small factors in LDS, 32 x 16 otherwise (the global-memory sweeps
// only finish factors that the block Jacobi left unconverged)
__device__ __attribute__((always_inline)) inline int
jacobi_any(double* A, int lda, int nr, int nc, double tol, int maxsweep, int topk, SmallShared& sh,
           double* lds, int cap) {
  double* k = sh.keys;
  int* sc = sh.scratch;
  double* kt = &sh.kth;
  if (nr <= 128 && (int64_t)nc * nr <= cap)
    return jacobi_os<16, 8>(A, lda, nr, nc, tol, maxsweep, topk, k, sc, kt, lds, cap);
  return jacobi_os<32, 16>(A, lda, nr, nc, tol, maxsweep, topk, k, sc, kt, lds, cap);
}

// Block Jacobi hand-over: the state for a factor of nc columns and nr rows
// (thread 0).
__device__ inline void bj_start(BJState* S, int nc, int nr, int topk) {
  S->nc = nc; S->nr = nr; S->topk = topk; S->done = 0;
  S->sweeps = 0; S->thr = -1.0;
  for (int i = 0; i < 3; ++i) { S->rot[i] = 1; S->rel[i] = 0; }
  S->bar = 0; S->fail = 0;
}

// Whether the sweep of parity `par` ended the Jacobi: no turns, or only
// turns below sqrt(tol) relative, which leave the next sweep none above tol
// (quadratic convergence).
__device__ inline bool bj_converged(const BJState* S, int par, double tol) {
  return S->rot[par] == 0 || __longlong_as_double((long long)S->rel[par]) < tol;
}

// Sweeps already run by the block Jacobi, and whether single-workgroup
// sweeps must continue (the last launched sweep still rotated).
__device__ inline int bj_sweeps(const BJState* S, double tol, bool& more) {
  if (S->fail) { more = false; return BJ_TIMEOUT_SWEEPS; }
  const int nsw = S->sweeps;
  more = !(S->done || nsw < 1 || bj_converged(S, (nsw - 1) % 3, tol));
  return nsw;
}

// Per pair (one workgroup):
//  1. a Cholesky factor F of M (diagonally pivoted up to order PIVOT_MAX)
//     and one-sided Jacobi on it: the t dominant eigenvectors Z of M, i.e.
//     left singular vectors of B, and sigma_B;
//  2. L = Z (N x t), the joint basis [L1; L2] of Algorithm 2's CS step;
//  3. Y = eigenvectors of H = L1^T L1 (+ a tiny shift, which leaves them
//     unchanged), again by a Cholesky factor + Jacobi;
//  4. L Y: alpha_i = ||L1 y_i||, beta_i = ||L2 y_i|| (beta from L2 as the
//     column norms, never sqrt(1 - alpha^2)), X1, X2, (L Y)^T, quantities.
// Stages (SmallJob::stage) split the step around the block Jacobi launches
// on the factors of M and H and around the multi-workgroup products H and
// L Y of the larger pairs: 1 | block Jacobi on M | 2 | H Gram | 5 | block
// Jacobi on H | 3 | L Y | 4.
// largest order factored by the diagonally pivoted Cholesky in every case
constexpr int PIVOT_MAX = 128;

__device__ __attribute__((always_inline)) inline void small_pair(const SmallJob& J, double* lds, int cap,
                                                             SmallShared& sh) {
  const int l1 = J.l1, N = J.l1 + J.l2, t = J.t;
  const int tid = threadIdx.x;
  double* keys = sh.keys;
  int* perm = sh.perm;
  double* Lg = J.work;                            // N x t column-major
  double* Hg = Lg + (int64_t)N * t;               // t x t
  double* F = Hg + (int64_t)t * t;                // N x N Jacobi factor
  BJState* S = J.st;
  const int stage = J.stage;
  int rh, sw1, sw2;
  double* FH = F;
  // A NaN or infinity in G reaches B and the diagonal of M = B B^T (the
  // squared row norms of B).  Such a pair gets NaN GSVs and quantities, zero
  // recovery coefficients and FLAG_NONFINITE; its later stages and block
  // Jacobi launches return at once (rank -1 and done in its state).
  if (stage <= 1) {
    if (tid == 0) sh.scratch[4] = 0;
    __syncthreads();
    for (int i = tid; i < N; i += 1024)
      if (!isfinite(J.M[(int64_t)i * J.ldm + i])) sh.scratch[4] = 1;
    __syncthreads();
    if (sh.scratch[4]) {
      const double qnan = __longlong_as_double(0x7ff8000000000000ll);
      for (int i = tid; i < t; i += 1024) { J.alpha[i] = J.beta[i] = J.theta[i] = J.P1[i] = J.P2[i] = qnan; }
      for (int i = tid; i < N; i += 1024) J.sigma[i] = qnan;
      for (int e = tid; e < t * l1; e += 1024) J.X1t[(int64_t)(e / l1) * J.ldx1 + e % l1] = 0.0;
      for (int e = tid; e < t * J.l2; e += 1024) J.X2t[(int64_t)(e / J.l2) * J.ldx2 + e % J.l2] = 0.0;
      for (int e = tid; e < t * N; e += 1024) J.Rcoef[(int64_t)(e / N) * J.ldr + e % N] = 0.0;
      if (tid == 0) {
        J.D[0] = J.D[1] = qnan;
        S->rank = -1; S->nc = 0; S->done = 1;
        if (J.info) { J.info[5] = 0; J.info[6] = 0; atomicOr(J.info + 4, FLAG_NONFINITE); }
      }
      return;
    }
  } else if (S->rank < 0) {
    // stage 4 clears Rcoef again: the multi-workgroup L Y launch before it
    // does not read the state
    if (stage == 4)
      for (int e = tid; e < t * N; e += 1024) J.Rcoef[(int64_t)(e / N) * J.ldr + e % N] = 0.0;
    return;
  }
  if (stage <= 2 || stage == 5) {
    if (stage != 5) {
      // ---- 1. eigen-decomposition of M
      int rank, base = 0;
      double trM;
      bool more = true;
      if (stage <= 1) {
        // up to order PIVOT_MAX the diagonally pivoted Cholesky: where B has
        // fewer dominant directions than rows (noise columns in the sketch)
        // its graded factor settles in up to half the Jacobi sweeps of the
        // unpivoted one.  Above it the blocked unpivoted form, whose factor
        // needed as many sweeps on the wide sketches measured, and whose cost
        // does not grow with one barrier per column; the pivoted form, which
        // stops at the numerical rank, when a pivot fails
        const int ldp = 16 * ((N + 15) / 16) + 4;
        if (N > PIVOT_MAX &&
            chol_unpivoted(J.M, J.ldm, N, F, sh.diag, lds, ldp, lds + 16 * ldp, &sh.scratch[5], &sh.trace))
          rank = N;
        else
          rank = pivoted_cholesky(J.M, J.ldm, N, F, sh.diag, sh.act, lds, &sh.piv_j, &sh.piv_d, 0.0, &sh.trace);
        trM = sh.trace;
        if (stage == 1) {
          if (tid == 0) { S->rank = rank; S->trM = trM; bj_start(S, rank, N, t < rank ? t : rank); }
          return;
        }
      } else {
        rank = S->rank;
        trM = S->trM;
        base = bj_sweeps(S, J.tol, more);
      }
      const int tt = t < rank ? t : rank;
      // above order 256 the block sweeps are the whole budget of the factor:
      // one that has not settled after them keeps FLAG_JACOBI_M rather than
      // running single-workgroup sweeps of tens of ms each (20 ms at order
      // 440); smaller factors finish on the single workgroup
      if (stage == 2 && more && N > 256) {
        sw1 = J.maxsweep + 1;
      } else {
        sw1 = base + (more ? jacobi_any(F, N, N, rank, J.tol, J.maxsweep - base, tt, sh, lds, cap) : 0);
      }
      // column norms of F: one wave per column, lanes striding its rows (one
      // thread walking a whole column serialises its loads)
      for (int c = tid >> 6; c < N; c += 16) {
        double s = 0.0;
        if (c < rank) s = col_sumsq(F + (int64_t)c * N, N, tid & 63);
        s = wave_sum(s);
        if ((tid & 63) == 0) keys[c] = sqrt(s);
      }
      __syncthreads();
      for (int c = tid; c < N; c += 1024) perm[rank_desc(keys, N, c)] = c;
      __syncthreads();
      // sigma_B: t dominant singular values of B, then the tail's Frobenius norm
      if (tid < 64) {
        double top = 0.0;
        for (int i = tid; i < t; i += 64) { const double v = keys[perm[i]]; top += v * v; }
        top = wave_sum(top);
        if (tid == 0) sh.kth = sqrt(fmax(0.0, trM - top));
      }
      __syncthreads();
      for (int i = tid; i < N; i += 1024)
        J.sigma[i] = (i < t) ? keys[perm[i]] : (i == t ? sh.kth : 0.0);
      // ---- 2. L = normalised dominant columns of F (N x t)
      for (int e = tid; e < N * t; e += 1024) {
        const int c = e / N, r = e - c * N;
        const int src = perm[c];
        const double nv = keys[src];
        Lg[e] = (c < tt && nv > 0.0) ? F[(int64_t)src * N + r] / nv : 0.0;
      }
      __syncthreads();
      // with hgram set, H comes from the multi-workgroup Gram launches
      // after this stage, and stage 5 factors it
      if (J.hgram) {
        if (tid == 0) S->sw1 = sw1;
        return;
      }
      // ---- 3. H = L1^T L1 + eps I, its eigenvectors Y (F is free again)
      wg_gemm64<true>(Lg, N, 1, Lg, 1, N, t, t, l1, [&](int i, int j, double v) {
        Hg[(int64_t)i * t + j] = v;
        Hg[(int64_t)j * t + i] = v;
      });
      __syncthreads();
    } else {
      sw1 = S->sw1;
    }
    // H + 1e-12 I (the shift leaves the eigenvectors and keeps the factor
    // positive definite when L1 has fewer rows than t or some alpha is 0)
    for (int i = tid; i < t; i += 1024) Hg[(int64_t)i * t + i] += 1e-12;
    __syncthreads();
    {
      const int ldp = 16 * ((t + 15) / 16) + 4;
      if (t > PIVOT_MAX &&
          chol_unpivoted(Hg, t, t, FH, sh.diag, lds, ldp, lds + 16 * ldp, &sh.scratch[5], &sh.trace))
        rh = t;
      else
        rh = pivoted_cholesky(Hg, t, t, FH, sh.diag, sh.act, lds, &sh.piv_j, &sh.piv_d, 0.0, &sh.trace);
    }
    if (J.bjh) {
      if (tid == 0) { S->sw1 = sw1; bj_start(S, rh, t, 0); }
      return;
    }
  }
  if (stage == 4) {
    sw1 = S->sw1;
    sw2 = S->sw2;
  } else {
    {
      // Jacobi on the factor of H (after the block sweeps in stage 3)
      int base = 0;
      bool more = true;
      if (stage == 3) {
        sw1 = S->sw1;
        rh = S->nc;
        base = bj_sweeps(S, J.tol, more);
      }
      sw2 = base + (more ? jacobi_any(FH, t, t, rh, J.tol, J.maxsweep - base, 0, sh, lds, cap) : 0);
    }
    for (int c = tid >> 6; c < t; c += 16) {
      double s = 0.0;
      if (c < rh) s = col_sumsq(FH + (int64_t)c * t, t, tid & 63);
      s = wave_sum(s);
      if ((tid & 63) == 0) keys[c] = sqrt(s);
    }
    __syncthreads();
    if (stage == 3) {
      // L Y runs on many workgroups between this launch and stage 4
      for (int c = tid; c < t; c += 1024) {
        const double nv = keys[c];
        J.ycs[c] = (c < rh && nv > 0.0) ? 1.0 / nv : 0.0;
      }
      if (tid == 0) S->sw2 = sw2;
      return;
    }
    // ---- 4. L Y (rows of Rcoef), alpha, beta (sorted by alpha)
    // row r, column c of L Y (column c of Y = column c of FH / its norm)
    wg_gemm64<false>(Lg, 1, N, FH, 1, t, N, t, t, [&](int r, int c, double v) {
      const double nv = keys[c];
      J.Rcoef[(int64_t)c * J.ldr + r] = (c < rh && nv > 0.0) ? v / nv : 0.0;    // unsorted for now
    });
    __syncthreads();
  }
  for (int c = tid >> 6; c < t; c += 16) {
    double a = 0.0, b = 0.0;
    col_sumsq2(J.Rcoef + (int64_t)c * J.ldr, N, l1, tid & 63, &a, &b);
    a = wave_sum(a);
    b = wave_sum(b);
    if ((tid & 63) == 0) { keys[c] = sqrt(a); sh.frow[c] = sqrt(b); }
  }
  __syncthreads();
  for (int c = tid; c < t; c += 1024) perm[rank_desc(keys, t, c)] = c;
  __syncthreads();
  for (int i = tid; i < t; i += 1024) { J.alpha[i] = keys[perm[i]]; J.beta[i] = sh.frow[perm[i]]; }
  // reorder Rcoef rows in place through Lg (no longer needed) and build X1t, X2t
  for (int e = tid; e < t * N; e += 1024) Lg[e] = J.Rcoef[(int64_t)(e / N) * J.ldr + (e % N)];
  __syncthreads();
  for (int e = tid; e < t * N; e += 1024) {
    const int i = e / N, r = e - i * N;
    const int src = perm[i];
    const double v = Lg[(int64_t)src * N + r];
    J.Rcoef[(int64_t)i * J.ldr + r] = v;
    if (r < l1) {
      const double a = keys[src];
      J.X1t[(int64_t)i * J.ldx1 + r] = a > 0.0 ? v / a : 0.0;
    } else {
      const double b = sh.frow[src];
      J.X2t[(int64_t)i * J.ldx2 + (r - l1)] = b > BETA_ZERO ? v / b : 0.0;
    }
  }
  __syncthreads();
  // ---- 5. comparative quantities over the t pairs
  if (tid < 64) {
    double sa = 0.0, sb = 0.0;
    for (int i = tid; i < t; i += 64) {
      double a = J.alpha[i], b = J.beta[i];
      sa += a * a; sb += b * b;
    }
    sa = wave_sum(sa); sb = wave_sum(sb);
    double h1 = 0.0, h2 = 0.0;
    for (int i = tid; i < t; i += 64) {
      double a = J.alpha[i], b = J.beta[i];
      J.theta[i] = atan2(a, b) - 0.78539816339744831;
      double p1 = sa > 0.0 ? a * a / sa : 0.0;
      double p2 = sb > 0.0 ? b * b / sb : 0.0;
      J.P1[i] = p1; J.P2[i] = p2;
      if (p1 > 0.0) h1 -= p1 * log(p1);
      if (p2 > 0.0) h2 -= p2 * log(p2);
    }
    h1 = wave_sum(h1); h2 = wave_sum(h2);
    bool bz = false;
    for (int i = tid; i < t; i += 64) bz |= !(J.beta[i] > BETA_ZERO);
    bz = __ballot(bz) != 0;
    if (tid == 0) {
      double lt = t > 1 ? log((double)t) : 1.0;
      J.D[0] = t > 1 ? h1 / lt : 0.0;
      J.D[1] = t > 1 ? h2 / lt : 0.0;
      if (J.info) {
        J.info[5] = sw1; J.info[6] = sw2;
        int fl2 = 0;
        if (sw1 > J.maxsweep) fl2 |= FLAG_JACOBI_M;
        if (sw2 > J.maxsweep) fl2 |= FLAG_JACOBI_L1;
        if (!(sa > 0.0)) fl2 |= FLAG_ALPHA_ZERO;
        if (bz) fl2 |= FLAG_BETA_ZERO;
        if (fl2) atomicOr(J.info + 4, fl2);
      }
    }
  }
}

__global__ __launch_bounds__(1024) void k_small(const SmallJob* __restrict__ jobs, int nj, int cap) {
  extern __shared__ double lds[];
  __shared__ SmallShared sh;
  small_pair(jobs[blockIdx.x], lds, cap, sh);
}

// ------------------------------------------------------------ block Jacobi --
// One-sided Jacobi on a factor too large for one workgroup's LDS: the
// columns are split into nblk blocks of B; a round-robin tournament over the
// blocks gives each of nblk / 2 workgroups a block pair per round (one
// launch per round, so the launch boundary orders the rounds).  The
// workgroup stages its 2 B columns in LDS and turns the B^2 cross pairs (B
// inner rounds of B disjoint pairs); in the first round of a sweep, where
// every block meets exactly one other, it also turns the pairs inside both
// blocks.  Each pair of columns is therefore visited once per sweep, as in
// the single-workgroup sweeps, with the same rotation and skip rules.

// Sweep start (launched for the first sweep; later sweeps start inside
// their first round, bj_sweep_start): a sweep without rotations ends the
// run; otherwise the skip threshold (a quarter of the topk-th largest squared
// column norm; the norms come from the previous sweep's last round, or from
// A at sweep 0).
__global__ __launch_bounds__(1024) void k_bjinit(const BJJob* __restrict__ jobs, int nj, int sweep) {
  __shared__ double n2[SMALL_MAXN];
  __shared__ double kth;
  const BJJob J = jobs[blockIdx.x];
  BJState* S = J.st;
  const int tid = threadIdx.x, wave = tid >> 6, ln = tid & 63;
  if (S->done) return;
  if (sweep > 0 && bj_converged(S, (sweep - 1) % 3, J.tol)) {
    if (tid == 0) { S->done = 1; S->sweeps = sweep; }
    return;
  }
  const int nc = S->nc, nr = J.nr, topk = S->topk;
  if (sweep == 0) {
    for (int c = wave; c < nc; c += 16) {
      double v2 = 0.0;
      v2 = col_sumsq(J.A + (int64_t)c * nr, nr, ln);
      v2 = wave_sum(v2);
      if (ln == 0) n2[c] = v2;
    }
    __syncthreads();
    for (int c = tid; c < nc; c += 1024) J.nrm2[c] = n2[c];
  } else {
    // left by the last round of the previous sweep
    for (int c = tid; c < nc; c += 1024) n2[c] = J.nrm2[c];
  }
  __syncthreads();
  double thr = -1.0;
  if (topk > 0 && topk < nc) {
    if (tid < nc) {
      const double v = n2[tid];
      int r = 0;
      for (int j2 = 0; j2 < nc; ++j2) { const double w = n2[j2]; r += (w > v) || (w == v && j2 < tid); }
      if (r == topk - 1) kth = v;
    }
    __syncthreads();
    thr = 0.25 * kth;
  }
  if (tid == 0) {
    S->rot[sweep % 3] = 0; S->rel[sweep % 3] = 0;
    S->rot[(sweep + 1) % 3] = 0; S->rel[(sweep + 1) % 3] = 0;
    S->sweeps = sweep + 1; S->thr = thr;
  }
}

// The start of sweep s > 0 inside its first round (every workgroup of the
// round, so no launch of its own): whether sweep s - 1 ended the Jacobi, and
// otherwise the skip threshold from the squared norms its last round left.
// Workgroup 0 of the job records the outcome and clears the slot of sweep
// s + 1.  Returns false when the Jacobi has ended.
__device__ bool bj_sweep_start(const BJJob& J, BJState* S, int w, int sweep, double& thr, double* n2s,
                               double* kth_s) {
  const int tid = threadIdx.x;
  if (bj_converged(S, (sweep - 1) % 3, J.tol)) {
    if (w == 0 && tid == 0) { S->done = 1; S->sweeps = sweep; }
    return false;
  }
  const int nc = S->nc, topk = S->topk;
  thr = -1.0;
  if (topk > 0 && topk < nc) {
    for (int c = tid; c < nc; c += BJ_THREADS) n2s[c] = J.nrm2[c];
    __syncthreads();
    for (int i = tid; i < nc; i += BJ_THREADS) {
      const double v = n2s[i];
      int r = 0;
      for (int j2 = 0; j2 < nc; ++j2) { const double x = n2s[j2]; r += (x > v) || (x == v && j2 < i); }
      if (r == topk - 1) *kth_s = v;
    }
    __syncthreads();
    thr = 0.25 * *kth_s;
  }
  if (w == 0 && tid == 0) {
    S->thr = thr; S->sweeps = sweep + 1;
    S->rot[(sweep + 1) % 3] = 0; S->rel[(sweep + 1) % 3] = 0;
  }
  return true;
}

template <int B, int G, int EM>
__device__ __attribute__((always_inline)) inline void
bj_visit(const BJJob& J, BJState* S, int w, int sweep, int round, double* lds, double* n0, double thr) {
  const int nr = J.nr, nc = S->nc, tid = threadIdx.x;
  int bu, bv;
  tournament(w, round, J.nblk - 1, bu, bv);
  const int c0u = bu * B, c0v = bv * B;
  const int cu = min(max(nc - c0u, 0), B), cv = min(max(nc - c0v, 0), B);
  if (cu + cv < 2 && round != J.nblk - 2) return;   // the last round still refreshes norms
  // local column c < B is column c0u + c, c >= B is column c0v + c - B
  auto gcol = [&](int c) { return c < B ? c0u + c : c0v + c - B; };
  auto valid = [&](int c) { return c < B ? c < cu : c - B < cv; };
  // staging: TPC threads per column, rows sc_j + TPC i, all loads in flight;
  // LDS columns padded to LD = G EM rows, zero past nr
  constexpr int TPC = BJ_THREADS / (2 * B), RPT = 16, LD = G * EM;   // nr <= TPC * RPT = LD
  static_assert(TPC * RPT == LD, "staging covers the padded column");
  typedef __attribute__((address_space(1))) double gdouble;
  gdouble* gA = (gdouble*)J.A;
  const int sc_c = tid / TPC, sc_j = tid % TPC;
  const bool sc_ok = valid(sc_c);
  const gdouble* src = gA + (int64_t)(sc_ok ? gcol(sc_c) : 0) * nr;
  double* col = lds + sc_c * LD;
  {
    double v[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = sc_j + TPC * i;
      const double w = src[r < nr ? r : nr - 1];
      v[i] = (sc_ok && r < nr) ? w : 0.0;
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) col[sc_j + TPC * i] = v[i];
  }
  if (tid < 2 * B) n0[tid] = valid(tid) ? J.nrm2[gcol(tid)] : 0.0;
  __syncthreads();
  const int g = tid / G, j = tid % G;
  auto live = [&](int a, int b) {
    return valid(a) && valid(b) && !(thr >= 0.0 && n0[a] < thr && n0[b] < thr);
  };
  bool any = false;
  double rel2 = 0.0;
  if (round == 0) {
    // pairs inside each block: slots [0, B/2) in block u, [B/2, B) in block v
    const int side = g / (B / 2), pi = g % (B / 2);
    for (int s2 = 0; s2 < B - 1; ++s2) {
      int u, v;
      tournament(pi, s2, B - 1, u, v);
      const int a = side * B + u, b = side * B + v;
      any |= pair_step_padded<G, EM>(lds + a * LD, lds + b * LD, j, live(a, b), J.tol, thr, rel2);
      __syncthreads();
    }
  }
  // cross pairs: group g keeps column g for the B steps (in registers, one
  // LDS read and write of it per round) and meets the columns of block v in
  // turn, which pass from group to group through LDS
  {
    const int a = g;
    double x[EM];
#pragma unroll
    for (int e = 0; e < EM; ++e) x[e] = lds[a * LD + j + G * e];
    for (int s2 = 0; s2 < B; ++s2) {
      const int b = B + ((g + s2) & (B - 1));
      any |= pair_step_reg<G, EM>(x, lds + b * LD, j, live(a, b), J.tol, thr, rel2);
      __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < EM; ++e) lds[a * LD + j + G * e] = x[e];
    __syncthreads();
  }
  for (int o = 32; o > 0; o >>= 1) rel2 = fmax(rel2, __shfl_xor(rel2, o, 64));
  if ((tid & 63) == 0 && rel2 > 0.0)
    atomicMax((unsigned long long*)&S->rel[sweep % 3], (unsigned long long)__double_as_longlong(rel2));
  // rotations seen: one flag per wave, before the write-back (no barrier
  // after the last step's)
  if (__any(any) && (tid & 63) == 0) atomicOr(&S->rot[sweep % 3], 1);
  // write back; in the last round of the sweep every column passes through
  // exactly one workgroup, which leaves its squared norm for the next sweep
  double n2 = 0.0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = sc_j + TPC * i;
    if (r < nr) {
      const double v = col[r];
      n2 += v * v;
      if (sc_ok) gA[(int64_t)gcol(sc_c) * nr + r] = v;
    }
  }
  if (round == J.nblk - 2) {
    n2 = group_sum<TPC>(n2);
    if (sc_ok && sc_j == 0) J.nrm2[gcol(sc_c)] = n2;
  }
}

// One round of one sweep for every job (nblk / 2 workgroups each).
__global__ __launch_bounds__(BJ_THREADS) void k_bjround(const BJJob* __restrict__ jobs,
                                                        const int* __restrict__ pre, int nj, int sweep,
                                                        int round) {
  extern __shared__ double lds[];
  __shared__ double n0[2 * BJ_B];
  const int jb = find_side(pre, nj, blockIdx.x);
  const BJJob J = jobs[jb];
  BJState* S = J.st;
  if (S->done || round >= J.nblk - 1) return;
  const int w = blockIdx.x - pre[jb];
  double thr;
  if (sweep > 0 && round == 0) {
    __shared__ double n2s[SMALL_MAXN];
    __shared__ double kth_s;
    if (!bj_sweep_start(J, S, w, sweep, thr, n2s, &kth_s)) return;
  } else {
    thr = S->thr;
  }
  if (J.nr <= 256) bj_visit<BJ_B, BJ_THREADS / BJ_B, 8>(J, S, w, sweep, round, lds, n0, thr);
  else bj_visit<BJ_B / 2, 2 * BJ_THREADS / BJ_B, 8>(J, S, w, sweep, round, lds, n0, thr);
}

// Device-wide visibility of a round's columns.  The XCDs' L2 caches are not
// coherent with each other for ordinary device memory: the writer's L2 must
// write its dirty lines back, and the reader's L1 and L2 must drop theirs,
// each finished (vmcnt) before the next step.  Written out here because the
// compiler's fence may drop the wait after the write-back when the issuing
// wave has no store outstanding of its own.
__device__ __forceinline__ void l2_writeback() { asm volatile("buffer_wbl2 sc1\n\ts_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void l2_invalidate() { asm volatile("buffer_inv sc1\n\ts_waitcnt vmcnt(0)" ::: "memory"); }

// Barrier of the workgroups of one job between two rounds of a one-launch
// sweep: every workgroup adds one arrival to the job's counter and waits
// until `target` arrivals are in (the counter only grows during a Jacobi, so
// no reset between rounds).  Every wave's stores of the round reach L2 before
// the workgroup barrier; thread 0 then writes L2 back before the arrival and
// invalidates the caches after the wait.  The wait is bounded: after `spin`
// polls, or when another workgroup of the job has given up, the job is
// marked failed and ended, and the caller returns.
__device__ bool bj_barrier(BJState* S, uint32_t target, int spin, int* ok_s) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    l2_writeback();
    atomicAdd(&S->bar, 1u);
    int ok = 1;
    for (int n = 0; __hip_atomic_load(&S->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; ++n) {
      if (n >= spin || __hip_atomic_load(&S->fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (!ok) {
      atomicOr(&S->fail, 1);
      atomicOr(&S->done, 1);
    }
    l2_invalidate();
    *ok_s = ok;
  }
  __syncthreads();
  return *ok_s != 0;
}

// All rounds of one sweep for every job in one launch (nblk / 2 workgroups
// per job, all resident at once: the host takes this kernel only when the
// launch fits the device).  The visits, their order and the sweep start are
// those of the per-round launches; the launch boundary between rounds is
// replaced by the job's barrier.  Sweeps sw0, sw0 + 1, ... are launched this
// way (earlier ones one launch per round, which do not count arrivals).
__global__ __launch_bounds__(BJ_THREADS) void k_bjsweep(const BJJob* __restrict__ jobs,
                                                        const int* __restrict__ pre, int nj, int sweep,
                                                        int sw0, int spin) {
  extern __shared__ double lds[];
  __shared__ double n0[2 * BJ_B];
  __shared__ double n2s[SMALL_MAXN];
  __shared__ double kth_s;
  __shared__ int ok_s;
  const int jb = find_side(pre, nj, blockIdx.x);
  const BJJob J = jobs[jb];
  BJState* S = J.st;
  if (S->done) return;
  const int w = blockIdx.x - pre[jb];
  double thr;
  if (sweep > 0) {
    if (!bj_sweep_start(J, S, w, sweep, thr, n2s, &kth_s)) return;
  } else {
    thr = S->thr;
  }
  const int nround = J.nblk - 1, nwg = J.nblk / 2;
  for (int round = 0; round < nround; ++round) {
    if (round > 0) {
      const uint32_t target = (uint32_t)(((sweep - sw0) * (nround - 1) + round) * nwg);
      if (!bj_barrier(S, target, spin, &ok_s)) return;
    }
    if (J.nr <= 256) bj_visit<BJ_B, BJ_THREADS / BJ_B, 8>(J, S, w, sweep, round, lds, n0, thr);
    else bj_visit<BJ_B / 2, 2 * BJ_THREADS / BJ_B, 8>(J, S, w, sweep, round, lds, n0, thr);
  }
}

// ------------------------------------------------------------- k_rowsign --
// s_i = sign of the largest-magnitude entry of row i of R (first on ties)
__global__ __launch_bounds__(256) void k_rowsign(const SignJob* __restrict__ jobs,
                                                 const int* __restrict__ pre, int nj) {
  const int jb = find_side(pre, nj, blockIdx.x);
  const SignJob J = jobs[jb];
  const int i = blockIdx.x - pre[jb];
  double best = -1.0, val = 0.0;
  int bj = 0x7fffffff;
  for (int j = threadIdx.x; j < J.n; j += 256) {
    double v = J.R[(int64_t)i * J.ldr + j], a = fabs(v);
    if (a > best || (a == best && j < bj)) { best = a; val = v; bj = j; }
  }
  __shared__ double sb[256], sv[256];
  __shared__ int sj[256];
  sb[threadIdx.x] = best; sv[threadIdx.x] = val; sj[threadIdx.x] = bj;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      double b2 = sb[threadIdx.x + o];
      int j2 = sj[threadIdx.x + o];
      if (b2 > sb[threadIdx.x] || (b2 == sb[threadIdx.x] && j2 < sj[threadIdx.x])) {
        sb[threadIdx.x] = b2; sv[threadIdx.x] = sv[threadIdx.x + o]; sj[threadIdx.x] = j2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) J.sgn[i] = sv[0] < 0.0 ? -1.0 : 1.0;
}

__global__ __launch_bounds__(256) void k_scale_rows(const SignJob* __restrict__ jobs,
                                                    const int* __restrict__ pre, int nj) {
  const int jb = find_side(pre, nj, blockIdx.x);
  const SignJob J = jobs[jb];
  int64_t e = (int64_t)(blockIdx.x - pre[jb]) * 256 + threadIdx.x;
  if (e >= (int64_t)J.t * J.n) return;
  int i = (int)(e / J.n), j = (int)(e - (int64_t)i * J.n);
  J.R[(int64_t)i * J.ldr + j] *= J.sgn[i];
}

// ---------------------------------------------------------------- launch --
void launch_chol(const CholJob* j, int nj, hipStream_t st) {
  static bool attr_set = false;
  if (!attr_set) {
    hipFuncSetAttribute((const void*)k_chol, hipFuncAttributeMaxDynamicSharedMemorySize, (int)CB_LDS_BYTES);
    attr_set = true;
  }
  hipLaunchKernelGGL(k_chol, dim3(nj), dim3(64 * CB_W), CB_LDS_BYTES, st, j, nj);
}

void launch_small(const SmallJob* j, int nj, hipStream_t st) {
  static bool attr_set = false;
  const size_t bytes = SMALL_LDS_BYTES;
  if (!attr_set) {
    hipFuncSetAttribute((const void*)k_small, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    attr_set = true;
  }
  hipLaunchKernelGGL(k_small, dim3(nj), dim3(1024), bytes, st, j, nj, (int)(bytes / sizeof(double)));
}

void launch_bjinit(const BJJob* j, int nj, int sweep, hipStream_t st) {
  hipLaunchKernelGGL(k_bjinit, dim3(nj), dim3(1024), 0, st, j, nj, sweep);
}

void launch_bjround(const BJJob* j, const int* pre, int nj, int tiles, int sweep, int round, hipStream_t st) {
  static bool attr_set = false;
  const size_t bytes = (size_t)2 * BJ_B * 256 * sizeof(double);   // 2 B columns of <= 256 rows
  if (!attr_set) {
    hipFuncSetAttribute((const void*)k_bjround, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    attr_set = true;
  }
  hipLaunchKernelGGL(k_bjround, dim3(tiles), dim3(BJ_THREADS), bytes, st, j, pre, nj, sweep, round);
}

void launch_bjsweep(const BJJob* j, const int* pre, int nj, int tiles, int sweep, int sw0, int spin,
                    hipStream_t st) {
  static bool attr_set = false;
  const size_t bytes = (size_t)2 * BJ_B * 256 * sizeof(double);
  if (!attr_set) {
    hipFuncSetAttribute((const void*)k_bjsweep, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    attr_set = true;
  }
  hipLaunchKernelGGL(k_bjsweep, dim3(tiles), dim3(BJ_THREADS), bytes, st, j, pre, nj, sweep, sw0, spin);
}

void launch_sign(const SignJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  hipLaunchKernelGGL(k_rowsign, dim3(tiles), dim3(256), 0, st, j, pre, nj);
}

void launch_scale(const SignJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_rows, dim3(tiles), dim3(256), 0, st, j, pre, nj);
}

}  // namespace rg
