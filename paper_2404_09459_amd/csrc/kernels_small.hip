// Small dense FP64 steps, one workgroup (1024 threads) per matrix or pair.
//
//  k_chol     : Cholesky of the CholeskyQR Gram and the inverse of its lower
//               factor (the orthonormalisation replacing Algorithm 1's QR)
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
// Row elimination on [A | I]: after N steps the left block is R (A = R^T R)
// and the right block is R^{-T}.  The working array keeps R's upper triangle
// and R^{-T}'s strict lower triangle in one npad x npad array; R^{-T}'s
// diagonal is kept separately.  On a non-positive (or tiny relative) pivot
// the Gram is shifted by s I and the factorisation restarted.
__global__ __launch_bounds__(1024) void k_chol(const CholJob* __restrict__ jobs, int nj,
                                               double* __restrict__ gscratch) {
  extern __shared__ double lds[];
  const CholJob J = jobs[blockIdx.x];
  const int N = J.N, np = J.npad;
  const bool in_lds = (np <= CHOL_LDS_MAX);
  double* W = in_lds ? lds : gscratch + (int64_t)blockIdx.x * (CHOL_MAX * CHOL_MAX + 2 * CHOL_MAX);
  double* xd = in_lds ? lds + np * np : W + (int64_t)np * np;
  double* d0 = xd + np;
  __shared__ int bad;
  __shared__ double shift;
  __shared__ int shifted;
  const int tid = threadIdx.x;
  if (tid == 0) { shift = 0.0; shifted = 0; }
  __syncthreads();
  double maxdiag = 0.0;
  for (int i = 0; i < N; ++i) maxdiag = fmax(maxdiag, J.gram[(int64_t)i * np + i]);
  int attempt = 0;
  for (;;) {
    for (int e = tid; e < np * np; e += 1024) {
      int i = e / np, j = e - i * np;
      double v = 0.0;
      if (i < N && j < N) {
        if (j >= i) v = J.gram[(int64_t)i * np + j] + (i == j ? shift : 0.0);
      }
      W[e] = v;
    }
    for (int i = tid; i < np; i += 1024) {
      xd[i] = 1.0;
      d0[i] = (i < N) ? J.gram[(int64_t)i * np + i] : 0.0;
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    const int tx = tid & 31, ty = tid >> 5;   // 32 x 32 thread grid
    for (int k = 0; k < N; ++k) {
      double piv = W[k * np + k];
      // uniform decision
      bool brk = !(piv > 1e-15 * d0[k]) || !(piv > 0.0) || !isfinite(piv);
      if (brk) { if (tid == 0) bad = 1; break; }
      double d = sqrt(piv), rd = 1.0 / d;
      // scale row k (R's row k and R^{-T}'s row k)
      for (int j = tid; j < N; j += 1024) {
        if (j != k) W[k * np + j] *= rd;
        else { W[k * np + k] = d; xd[k] *= rd; }
      }
      __syncthreads();
      const double xk = xd[k];
      for (int i = k + 1 + ty; i < N; i += 32) {
        const double f = W[k * np + i];
        double* Wi = W + i * np;
        const double* Wk = W + k * np;
        for (int j = tx; j < N; j += 32) {
          if (j >= i) Wi[j] -= f * Wk[j];
          else if (j < k) Wi[j] -= f * Wk[j];
          else if (j == k) Wi[j] -= f * xk;
        }
      }
      __syncthreads();
    }
    __syncthreads();
    if (!bad) break;
    ++attempt;
    if (attempt > 8 || !(maxdiag > 0.0) || !isfinite(maxdiag)) {
      // give up: zero inverse, flag
      for (int e = tid; e < np * np; e += 1024) J.sinv[e] = 0.0;
      if (tid == 0 && J.info) {
        atomicOr(J.info + 4, isfinite(maxdiag) ? (1 << J.flagbit) | FLAG_CHOL_FAIL : FLAG_NONFINITE);
      }
      return;
    }
    if (tid == 0) {
      shift = (shift == 0.0) ? 1e-14 * maxdiag * (double)N : shift * 100.0;
      shifted = 1;
    }
    __syncthreads();
  }
  for (int e = tid; e < np * np; e += 1024) {
    int i = e / np, j = e - i * np;
    double v = 0.0;
    if (i < N && j < N) {
      if (j < i) v = W[e];
      else if (j == i) v = xd[i];
    }
    J.sinv[e] = v;
    if (J.r) J.r[e] = (i < N && j < N && j >= i) ? W[e] : 0.0;
  }
  if (tid == 0 && shifted && J.info) atomicOr(J.info + 4, 1 << J.flagbit);
}

// ------------------------------------------------------ one-sided Jacobi --
// Orthogonalises the columns of A (column-major, lda; nc columns) by plane
// rotations (Hestenes).  Inner products use rows [0, nd); rotations are
// applied to rows [0, nr) (nr >= nd), so rows nd..nr-1 just follow along.
// Parallel round-robin ordering: each round pairs every column once and the
// 16 waves share the round's pairs; a wave loads all of its pairs' columns
// before rotating so that global-memory latency is paid once per round.
// topk > 0: a pair is skipped when both columns have squared norm below
// (0.5 * topk-th largest norm)^2 (norms refreshed every sweep); at
// convergence the topk dominant columns are orthogonal to every other
// column, so they span the dominant invariant subspace.
// Returns the number of sweeps used (maxsweep + 1 when not converged).
template <int EPL>  // elements per lane per column (nr <= 64*EPL)
__device__ int jacobi_os(double* A, int lda, int nr, int nd, int nc, double tol, int maxsweep,
                         int topk, double* nrm2, int* scratch, double* kth_slot) {
  const int tid = threadIdx.x, wave = tid >> 6, ln = tid & 63;
  const int nc2 = nc + (nc & 1);
  if (nc < 2) return 0;
  constexpr int PB = 4;   // pairs per batch per wave (with 16 waves: 64 pairs per pass)
  for (int sweep = 0; sweep < maxsweep; ++sweep) {
    // column norms over the dot rows, and the skip threshold
    for (int c0 = wave * 4; c0 < nc; c0 += 64) {
      double sq[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        double s = 0.0;
        int c = c0 + b;
        if (c < nc)
          for (int i = ln; i < nd; i += 64) { double v = A[(int64_t)c * lda + i]; s += v * v; }
        sq[b] = s;
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int b = 0; b < 4; ++b) sq[b] += __shfl_xor(sq[b], o, 64);
      if (ln == 0)
        for (int b = 0; b < 4; ++b) if (c0 + b < nc) nrm2[c0 + b] = sq[b];
    }
    if (tid == 0) scratch[0] = 0;
    __syncthreads();
    double& kth = *kth_slot;
    double thr = -1.0;
    if (topk > 0 && topk < nc) {
      // topk-th largest squared norm: rank count (nc <= 512)
      if (tid < nc) {
        double v = nrm2[tid];
        int r = 0;
        for (int j = 0; j < nc; ++j) { double w = nrm2[j]; r += (w > v) || (w == v && j < tid); }
        if (r == topk - 1) kth = v;
      }
      __syncthreads();
      thr = 0.25 * kth;
    }
    for (int round = 0; round < nc2 - 1; ++round) {
      const int npairs = nc2 / 2;
      for (int pb = wave * PB; pb < npairs; pb += 16 * PB) {
        double ap[PB][EPL], aq[PB][EPL];
        int P_[PB], Q_[PB];
#pragma unroll
        for (int b = 0; b < PB; ++b) {
          int pi = pb + b;
          int p = -1, q = -1;
          if (pi < npairs) {
            int x0 = pi, x1 = nc2 - 1 - pi;
            p = (x0 == 0) ? 0 : 1 + (x0 - 1 + round) % (nc2 - 1);
            q = (x1 == 0) ? 0 : 1 + (x1 - 1 + round) % (nc2 - 1);
            if (p >= nc || q >= nc) { p = -1; q = -1; }
            else if (thr >= 0.0 && nrm2[p] < thr && nrm2[q] < thr) { p = -1; q = -1; }
          }
          P_[b] = p; Q_[b] = q;
#pragma unroll
          for (int e = 0; e < EPL; ++e) {
            int i = ln + 64 * e;
            bool ok = p >= 0 && i < nr;
            ap[b][e] = ok ? A[(int64_t)p * lda + i] : 0.0;
            aq[b][e] = ok ? A[(int64_t)q * lda + i] : 0.0;
          }
        }
        // the 3*PB inner products of the batch, reduced together so that the
        // shuffle latencies overlap
        double red[3 * PB];
#pragma unroll
        for (int b = 0; b < PB; ++b) {
          double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
          for (int e = 0; e < EPL; ++e) {
            int i = ln + 64 * e;
            if (i < nd) {
              al += ap[b][e] * ap[b][e]; be += aq[b][e] * aq[b][e]; ga += ap[b][e] * aq[b][e];
            }
          }
          red[3 * b] = al; red[3 * b + 1] = be; red[3 * b + 2] = ga;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
#pragma unroll
          for (int x = 0; x < 3 * PB; ++x) red[x] += __shfl_xor(red[x], o, 64);
#pragma unroll
        for (int b = 0; b < PB; ++b) {
          if (P_[b] < 0) continue;
          const double al = red[3 * b], be = red[3 * b + 1], ga = red[3 * b + 2];
          if (!(al > 0.0) || !(be > 0.0)) continue;
          if (!(fabs(ga) > tol * sqrt(al) * sqrt(be))) continue;
          double zeta = (be - al) / (2.0 * ga);
          double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
          const int p = P_[b], q = Q_[b];
#pragma unroll
          for (int e = 0; e < EPL; ++e) {
            int i = ln + 64 * e;
            if (i < nr) {
              double u = ap[b][e], v = aq[b][e];
              A[(int64_t)p * lda + i] = c * u - sn * v;
              A[(int64_t)q * lda + i] = sn * u + c * v;
            }
          }
          if (ln == 0) scratch[0] = 1;
        }
      }
      __syncthreads();
    }
    int any = scratch[0];
    __syncthreads();
    if (!any) return sweep + 1;
  }
  return maxsweep + 1;
}

// rank of key[i] among n keys, descending, ties by index (for sorting)
__device__ inline int rank_desc(const double* key, int n, int i) {
  double v = key[i];
  int r = 0;
  for (int j = 0; j < n; ++j) {
    double w = key[j];
    r += (w > v) || (w == v && j < i);
  }
  return r;
}

// --------------------------------------------------------------- k_small --
// Per pair (one workgroup):
//  1. diagonally pivoted Cholesky of M = B B^T: P^T M P = R^T R; the columns
//     of F = P R^T (rows of R scattered back to M's row order) satisfy
//     F F^T = M, and they are graded, which makes step 2 converge in few
//     sweeps (the QR-preconditioned Jacobi of Drmac and Veselic);
//  2. one-sided Jacobi on F: normalised columns are M's eigenvectors, their
//     norms the singular values of B; L = the t dominant ones (N x t);
//  3. one-sided Jacobi driven by the rows of L1 = L[:l1] and applied to whole
//     columns of L: the result is L Y with L1 Y = X1 diag(alpha) and
//     L2 Y = X2 diag(beta)  (the SVD of L1 in Algorithm 2 and beta from L2);
//  4. sort by alpha, write alpha, beta, X1^T, X2^T, (L Y)^T and the
//     comparative quantities.
struct SmallShared {
  double keys[SMALL_MAXN];
  double diag[SMALL_MAXN];
  double frow[SMALL_MAXN];
  int perm[SMALL_MAXN];
  int act[SMALL_MAXN];
  int scratch[8];
  int piv_j;
  double piv_d;
};

template <int EPL>
__device__ void small_pair(const SmallJob& J, double* lds, size_t lds_doubles, SmallShared& sh) {
  const int N = J.l1 + J.l2, t = J.t, l1 = J.l1;
  const int tid = threadIdx.x;
  int* scratch = sh.scratch;
  double* keys = sh.keys;
  double* diag = sh.diag;
  int* perm = sh.perm;
  int* act = sh.act;
  int& piv_j = sh.piv_j;
  double& piv_d = sh.piv_d;
  // storage: F (N x N) then L (N x t); LDS when they fit, else global work
  const bool fl = (size_t)N * N <= lds_doubles;
  double* F = fl ? lds : J.work;                    // N x N, column k = k-th pivot column
  double* frow = sh.frow;
  // ---- 1. left-looking diagonally pivoted Cholesky of M (read in place)
  for (int e = tid; e < N * N; e += 1024) F[e] = 0.0;
  for (int i = tid; i < N; i += 1024) { diag[i] = J.M[(int64_t)i * J.ldm + i]; act[i] = 1; }
  __syncthreads();
  double dmax0 = 0.0;
  for (int i = 0; i < N; ++i) dmax0 = fmax(dmax0, diag[i]);
  // rows handled by groups of TPR threads
  int TPR = 1;
  while (TPR * 2 * N <= 1024 && TPR < 16) TPR *= 2;
  const int row = tid / TPR, part = tid % TPR;
  int rank = 0;
  for (int k = 0; k < N; ++k) {
    if (tid < 64) {
      double best = -1.0; int bj = -1;
      for (int j = tid; j < N; j += 64)
        if (act[j] && diag[j] > best) { best = diag[j]; bj = j; }
      for (int o = 32; o > 0; o >>= 1) {
        double b2 = __shfl_xor(best, o, 64);
        int j2 = __shfl_xor(bj, o, 64);
        if (b2 > best || (b2 == best && j2 >= 0 && (bj < 0 || j2 < bj))) { best = b2; bj = j2; }
      }
      if (tid == 0) { piv_j = bj; piv_d = best; }
    }
    __syncthreads();
    const int js = piv_j;
    const double d = piv_d;
    if (js < 0 || !(d > 1e-15 * dmax0) || !(d > 0.0)) break;   // numerical rank reached
    for (int kk = tid; kk < k; kk += 1024) frow[kk] = F[(int64_t)kk * N + js];
    __syncthreads();
    const double sd = sqrt(d), rd = 1.0 / sd;
    // column k: (M[:, js] - F[:, :k] F[js, :k]^T) / sqrt(d) on the active rows
    double acc = 0.0;
    if (row < N && act[row])
      for (int kk = part; kk < k; kk += TPR) acc += F[(int64_t)kk * N + row] * frow[kk];
    for (int o = TPR / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    __syncthreads();
    if (row < N && part == 0) {
      double v = 0.0;
      if (row == js) v = sd;
      else if (act[row]) v = (J.M[(int64_t)row * J.ldm + js] - acc) * rd;
      F[(int64_t)k * N + row] = v;
      if (act[row] && row != js) diag[row] -= v * v;
    }
    if (tid == 0) act[js] = 0;
    __syncthreads();
    rank = k + 1;
  }
  __syncthreads();
  // ---- 2. Jacobi on the rank columns of F (only pairs touching the t dominant)
  int sw1 = jacobi_os<EPL>(F, N, N, N, rank, J.tol, J.maxsweep, t, keys, scratch, &sh.piv_d);
  for (int c = tid; c < N; c += 1024) {
    double s = 0.0;
    if (c < rank)
      for (int r = 0; r < N; ++r) { double v = F[(int64_t)c * N + r]; s += v * v; }
    keys[c] = sqrt(s);
  }
  __syncthreads();
  for (int c = tid; c < N; c += 1024) perm[rank_desc(keys, N, c)] = c;
  __syncthreads();
  for (int i = tid; i < N; i += 1024) J.sigma[i] = keys[perm[i]];   // singular values of B
  // L (N x t, column-major) = normalised dominant columns, stored where it fits
  const bool ll = (size_t)N * t <= lds_doubles;
  double* L = ll ? (fl ? J.work : lds) : J.work + (int64_t)N * N;
  // (when F lives in LDS, L goes to global work first, then moved below)
  for (int e = tid; e < N * t; e += 1024) {
    int c = e / N, r = e - c * N;
    int src = perm[c];
    double nv = keys[src];
    L[e] = (c < rank && nv > 0.0) ? F[(int64_t)src * N + r] / nv : 0.0;
  }
  __syncthreads();
  if (ll && fl) {   // move L into LDS (F no longer needed)
    for (int e = tid; e < N * t; e += 1024) lds[e] = L[e];
    __syncthreads();
    L = lds;
  }
  // ---- 3. SVD of L1 driven rotations on whole columns of L
  int sw2 = jacobi_os<EPL>(L, N, N, l1, t, J.tol, J.maxsweep, 0, keys, scratch, &sh.piv_d);
  for (int c = tid; c < t; c += 1024) {
    double s = 0.0;
    for (int r = 0; r < l1; ++r) { double v = L[(int64_t)c * N + r]; s += v * v; }
    keys[c] = sqrt(s);
  }
  __syncthreads();
  for (int c = tid; c < t; c += 1024) perm[rank_desc(keys, t, c)] = c;
  __syncthreads();
  for (int i = tid; i < t; i += 1024) J.alpha[i] = keys[perm[i]];
  for (int i = tid; i < t; i += 1024) {
    int src = perm[i];
    double s = 0.0;
    for (int r = l1; r < N; ++r) { double v = L[(int64_t)src * N + r]; s += v * v; }
    J.beta[i] = sqrt(s);
  }
  __syncthreads();
  for (int e = tid; e < t * N; e += 1024) {
    int i = e / N, r = e - i * N;
    int src = perm[i];
    double v = L[(int64_t)src * N + r];
    J.Rcoef[(int64_t)i * J.ldr + r] = v;
    if (r < l1) {
      double a = keys[src];
      J.X1t[(int64_t)i * J.ldx1 + r] = a > 0.0 ? v / a : 0.0;
    } else {
      double b = J.beta[i];
      J.X2t[(int64_t)i * J.ldx2 + (r - l1)] = b > BETA_ZERO ? v / b : 0.0;
    }
  }
  __syncthreads();
  // ---- 4. comparative quantities over the t pairs
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
        for (int i = 0; i < t; ++i) if (!(J.beta[i] > BETA_ZERO)) fl2 |= FLAG_BETA_ZERO;
        if (fl2) atomicOr(J.info + 4, fl2);
      }
    }
  }
}

__global__ __launch_bounds__(1024) void k_small(const SmallJob* __restrict__ jobs, int nj,
                                                size_t lds_doubles) {
  extern __shared__ double lds[];
  __shared__ SmallShared sh;
  const SmallJob J = jobs[blockIdx.x];
  const int N = J.l1 + J.l2;
  if (N <= 256) small_pair<4>(J, lds, lds_doubles, sh);
  else small_pair<8>(J, lds, lds_doubles, sh);
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
void launch_chol(const CholJob* j, int nj, int npad_max, double* gscratch, hipStream_t st) {
  static bool attr_set = false;
  if (!attr_set) {
    size_t maxlds = (size_t)(CHOL_LDS_MAX * CHOL_LDS_MAX + 2 * CHOL_LDS_MAX) * sizeof(double);
    hipFuncSetAttribute((const void*)k_chol, hipFuncAttributeMaxDynamicSharedMemorySize, (int)maxlds);
    attr_set = true;
  }
  size_t lds = 0;
  if (npad_max <= CHOL_LDS_MAX) lds = (size_t)(npad_max * npad_max + 2 * npad_max) * sizeof(double);
  hipLaunchKernelGGL(k_chol, dim3(nj), dim3(1024), lds, st, j, nj, gscratch);
}

void launch_small(const SmallJob* j, int nj, hipStream_t st) {
  static bool attr_set = false;
  const size_t bytes = SMALL_LDS_BYTES;
  if (!attr_set) {
    hipFuncSetAttribute((const void*)k_small, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    attr_set = true;
  }
  hipLaunchKernelGGL(k_small, dim3(nj), dim3(1024), bytes, st, j, nj, bytes / sizeof(double));
}

void launch_sign(const SignJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  hipLaunchKernelGGL(k_rowsign, dim3(tiles), dim3(256), 0, st, j, pre, nj);
}

void launch_scale(const SignJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_rows, dim3(tiles), dim3(256), 0, st, j, pre, nj);
}

}  // namespace rg
