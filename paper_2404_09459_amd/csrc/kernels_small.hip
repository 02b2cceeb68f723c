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
      const int rows = N - k - 1;
      const int cnt = rows * N;
      for (int e = tid; e < cnt; e += 1024) {
        int i = k + 1 + e / N, j = e % N;
        double f = W[k * np + i];
        if (j >= i) W[i * np + j] -= f * W[k * np + j];
        else if (j < k) W[i * np + j] -= f * W[k * np + j];
        else if (j == k) W[i * np + j] -= f * xd[k];
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
// Orthogonalises the columns of A (nr x nc, column-major, lda) by plane
// rotations (Hestenes); the same rotations are applied to V (nv x nc,
// column-major, ldv) when given.  Parallel round-robin ordering: every round
// pairs each column once; 16 waves share a round's pairs.  Columns stay in
// the memory given (LDS or global).  Returns the number of sweeps used
// (maxsweep + 1 when not converged).
__device__ int jacobi_os(double* A, int lda, int nr, int nc, double* V, int ldv, int nv,
                         double tol, int maxsweep, int* scratch_flag) {
  const int tid = threadIdx.x, wave = tid >> 6, ln = tid & 63;
  const int nc2 = nc + (nc & 1);
  if (nc < 2) return 0;
  int sweep = 0;
  for (; sweep < maxsweep; ++sweep) {
    if (tid == 0) *scratch_flag = 0;
    __syncthreads();
    for (int round = 0; round < nc2 - 1; ++round) {
      for (int pi = wave; pi < nc2 / 2; pi += 16) {
        int x0 = pi, x1 = nc2 - 1 - pi;
        int p = (x0 == 0) ? 0 : 1 + (x0 - 1 + round) % (nc2 - 1);
        int q = (x1 == 0) ? 0 : 1 + (x1 - 1 + round) % (nc2 - 1);
        if (p >= nc || q >= nc) continue;
        double* ap = A + (int64_t)p * lda;
        double* aq = A + (int64_t)q * lda;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = ln; i < nr; i += 64) {
          double u = ap[i], v = aq[i];
          al += u * u; be += v * v; ga += u * v;
        }
        al = wave_sum(al); be = wave_sum(be); ga = wave_sum(ga);
        if (!(al > 0.0) || !(be > 0.0)) continue;
        if (!(fabs(ga) > tol * sqrt(al) * sqrt(be))) continue;
        double zeta = (be - al) / (2.0 * ga);
        double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int i = ln; i < nr; i += 64) {
          double u = ap[i], v = aq[i];
          ap[i] = c * u - s * v;
          aq[i] = s * u + c * v;
        }
        if (V) {
          double* vp = V + (int64_t)p * ldv;
          double* vq = V + (int64_t)q * ldv;
          for (int i = ln; i < nv; i += 64) {
            double u = vp[i], v = vq[i];
            vp[i] = c * u - s * v;
            vq[i] = s * u + c * v;
          }
        }
        if (ln == 0) *scratch_flag = 1;
      }
      __syncthreads();
    }
    __syncthreads();
    int any = *scratch_flag;
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
__global__ __launch_bounds__(1024) void k_small(const SmallJob* __restrict__ jobs, int nj) {
  const SmallJob J = jobs[blockIdx.x];
  const int N = J.l1 + J.l2, t = J.t, l1 = J.l1, l2 = J.l2;
  const int tid = threadIdx.x;
  __shared__ int flag;
  __shared__ double keys[SMALL_MAXN];
  __shared__ int perm[SMALL_MAXN];
  double* Aw = J.work;                       // N x N column-major (copy of M)
  double* Lw = Aw + (int64_t)N * N;          // N x t column-major: L then L Y
  double* Yw = Lw + (int64_t)N * t;          // t x t column-major
  double* Cw = Yw + (int64_t)t * t;          // l1 x t column-major: L1 (rotated)
  // ---- eigen-decomposition of M = B B^T by one-sided Jacobi on M itself
  for (int e = tid; e < N * N; e += 1024) {
    int c = e / N, r = e - c * N;
    Aw[e] = J.M[(int64_t)r * J.ldm + c];
  }
  __syncthreads();
  int sw1 = jacobi_os(Aw, N, N, N, nullptr, 0, 0, J.tol, J.maxsweep, &flag);
  // column norms = eigenvalues (M is positive semidefinite)
  for (int c = tid; c < N; c += 1024) {
    double s = 0.0;
    for (int r = 0; r < N; ++r) { double v = Aw[(int64_t)c * N + r]; s += v * v; }
    keys[c] = sqrt(s);
  }
  __syncthreads();
  for (int c = tid; c < N; c += 1024) perm[rank_desc(keys, N, c)] = c;
  __syncthreads();
  for (int i = tid; i < N; i += 1024) J.sigma[i] = sqrt(keys[perm[i]]);   // singular values of B
  // L = normalised top-t eigenvectors
  for (int e = tid; e < N * t; e += 1024) {
    int c = e / N, r = e - c * N;
    int src = perm[c];
    double nrm = keys[src];
    Lw[e] = nrm > 0.0 ? Aw[(int64_t)src * N + r] / nrm : 0.0;
  }
  __syncthreads();
  // ---- SVD of L1 (l1 x t) by one-sided Jacobi, accumulating Y (t x t)
  for (int e = tid; e < l1 * t; e += 1024) {
    int c = e / l1, r = e - c * l1;
    Cw[e] = Lw[(int64_t)c * N + r];
  }
  for (int e = tid; e < t * t; e += 1024) {
    int c = e / t, r = e - c * t;
    Yw[e] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  int sw2 = jacobi_os(Cw, l1, l1, t, Yw, t, t, J.tol, J.maxsweep, &flag);
  for (int c = tid; c < t; c += 1024) {
    double s = 0.0;
    for (int r = 0; r < l1; ++r) { double v = Cw[(int64_t)c * l1 + r]; s += v * v; }
    keys[c] = sqrt(s);
  }
  __syncthreads();
  for (int c = tid; c < t; c += 1024) perm[rank_desc(keys, t, c)] = c;
  __syncthreads();
  // alpha and X1^T (t x l1 row-major); zero-alpha columns of X1 left at 0
  for (int i = tid; i < t; i += 1024) J.alpha[i] = keys[perm[i]];
  for (int e = tid; e < t * l1; e += 1024) {
    int i = e / l1, r = e - i * l1;
    int src = perm[i];
    double a = keys[src];
    J.X1t[(int64_t)i * J.ldx1 + r] = a > 0.0 ? Cw[(int64_t)src * l1 + r] / a : 0.0;
  }
  // LY (N x t) = L * Y(:, perm): stored as Rcoef (t x N row-major)
  for (int e = tid; e < t * N; e += 1024) {
    int i = e / N, r = e - i * N;
    int src = perm[i];
    double s = 0.0;
    for (int c = 0; c < t; ++c) s += Lw[(int64_t)c * N + r] * Yw[(int64_t)src * t + c];
    J.Rcoef[(int64_t)i * J.ldr + r] = s;
  }
  __syncthreads();
  // beta_i = || L2 y_i ||,  X2 = L2 Y / beta   (rows l1..N-1 of LY)
  for (int i = tid; i < t; i += 1024) {
    double s = 0.0;
    for (int r = l1; r < N; ++r) { double v = J.Rcoef[(int64_t)i * J.ldr + r]; s += v * v; }
    J.beta[i] = sqrt(s);
  }
  __syncthreads();
  for (int e = tid; e < t * l2; e += 1024) {
    int i = e / l2, r = e - i * l2;
    double b = J.beta[i];
    J.X2t[(int64_t)i * J.ldx2 + r] = b > BETA_ZERO ? J.Rcoef[(int64_t)i * J.ldr + l1 + r] / b : 0.0;
  }
  __syncthreads();
  // ---- comparative quantities over the t pairs
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
        int fl = 0;
        if (sw1 > J.maxsweep) fl |= FLAG_JACOBI_M;
        if (sw2 > J.maxsweep) fl |= FLAG_JACOBI_L1;
        if (!(sa > 0.0)) fl |= FLAG_ALPHA_ZERO;
        for (int i = 0; i < t; ++i) if (!(J.beta[i] > BETA_ZERO)) fl |= FLAG_BETA_ZERO;
        if (fl) atomicOr(J.info + 4, fl);
      }
    }
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
  hipLaunchKernelGGL(k_small, dim3(nj), dim3(1024), 0, st, j, nj);
}

void launch_sign(const SignJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  hipLaunchKernelGGL(k_rowsign, dim3(tiles), dim3(256), 0, st, j, pre, nj);
}

void launch_scale(const SignJob* j, const int* pre, int nj, int tiles, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_rows, dim3(tiles), dim3(256), 0, st, j, pre, nj);
}

}  // namespace rg
