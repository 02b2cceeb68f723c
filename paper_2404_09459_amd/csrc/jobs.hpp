// Job descriptors shared by the host orchestration and the kernels.  Every
// kernel launch processes a table of jobs; a prefix table of per-job tile
// counts maps blockIdx.x to (job, tile).  One launch thus serves both
// matrices of a pair, or every matrix of a batch.
#pragma once
#include <vector>
#include <stdint.h>

namespace rg {

// Yt = (G W)^T :  G m x n (row-major, ldg), Wt L x n (ldw), Yt L x m (ldy)
struct NnJob {
  const void* G; const void* Wt; void* Yt;
  int64_t ldg, ldw, ldy;
  int32_t m, n, L, pad;
};

// D[c][j] (+)= sum_{k<K} A[c][k] B[k][j] for c < rows, j < J.
// A small (rows x K, lda), B big (K x J, ldb), D (rows x J, ldd).
struct AbJob {
  const void* A; const void* B; void* D;
  int64_t lda, ldb, ldd;
  int32_t rows, K, J, accumulate;
  const double* colscale;   // optional: D[c][j] *= colscale[c] (sign fixes), or null
};

// Partial Grams of a row-stacked matrix X = [X1 (r1 rows); X2 (r2 rows)]
// over column chunks [k0 + c*clen, k0 + (c+1)*clen) of [k0, k1):
//   out[c] = X[:, chunk c] X[:, chunk c]^T   (npad x npad, double)
// Only the 16 x 16 groups on or above the diagonal with both indices below
// r1 + r2 are written; one tile per strip (gram_strips per chunk).
struct GramJob {
  const void* X1; const void* X2; double* out;
  int64_t ld1, ld2;
  int32_t r1, r2, k0, k1, npad, clen;
  int32_t rgs, pad;   // row groups per strip (1 or 2, gram_rgs)
};

// Strips of a Gram over R rows: strip row rp (row groups rgs rp ...
// rgs rp + rgs - 1, 16 rows each) meets the 64-column blocks from
// rgs rp / 4 to the last one that starts below R.
__host__ __device__ inline int gram_strips(int R, int rgs) {
  const int npr = (R + 16 * rgs - 1) / (16 * rgs), ncb = (R + 63) / 64;
  int s = 0;
  for (int rp = 0; rp < npr; ++rp) s += ncb - rp * rgs / 4;
  return s;
}

// Row groups per strip for a Gram over R rows in `chunks` row chunks: two
// (each column fragment serves both, half the column reads) while that
// still leaves 1024 single-wave strips to fill the device, else one.
inline int gram_rgs(int R, int chunks) { return gram_strips(R, 2) * chunks >= 1024 ? 2 : 1; }

// One strip height per launch (the two heights are separate kernels): two
// row groups only when every job of the launch takes them; the tile counts
// follow.  Returns the launch's rgs.
inline int gram_uniform(std::vector<GramJob>& gj, std::vector<int>& gtl) {
  int rgs = 2;
  for (auto& g : gj) rgs = g.rgs < rgs ? g.rgs : rgs;
  for (size_t i = 0; i < gj.size(); ++i) {
    const int R = gj[i].r1 + gj[i].r2;
    const int chunks = gtl[i] / gram_strips(R, gj[i].rgs);
    gj[i].rgs = rgs;
    gtl[i] = gram_strips(R, rgs) * chunks;
  }
  return rgs;
}

// out[r][c] = sum_{p < nparts} in[p*stride + r*ldi + c] in fixed order,
// converted to the output type.  Symmetric (Gram) reductions read the upper
// 16 x 16 groups for the lower ones and write zero at and past row or
// column nz.
struct RedJob {
  const void* in; void* out; double* sq;
  int64_t stride; int64_t count;
  int32_t nparts, rows, cols, ldo;   // output viewed as rows x cols with ld ldo
  int64_t ldi;                       // input row stride (cols <= ldi)
  int32_t nz, pad;                   // symmetric reductions: rows / columns kept
};

// Omega^T generation: Wt[c][r] = Omega[r][col0 + c] for c < ncols, r < n.
// Rows ncols..L-1 are not written: the caller clears them beforehand.
struct GenJob {
  void* Wt; int64_t ldw;
  uint64_t seed;
  int32_t n, col0, ncols, L, stream, pad;
};

// Cholesky of an N x N SPD Gram (N <= 256; sum of partials already formed)
// and the inverse of its lower factor: sinv = L^{-1} (lower, npad x npad,
// zero past N).  shift0 > 0 adds shift0 * trace(Gram) to the diagonal from
// the start.  trunc != 0: a row whose pivot is below CHOL_TRUNC_REL times
// its original diagonal (numerically inside the span of the rows before it)
// gets a zero row in L^{-1} instead of a restart.
struct CholJob {
  const double* gram; double* sinv; int32_t* info;
  int32_t N, npad, flagbit, trunc;
  double shift0;
};

// Zero fill of nwords 32-bit words (one grouped launch for many buffers).
struct ZeroJob {
  uint32_t* p; int64_t nwords;
};

// Sum of squares of a rows x cols block (row stride ld, FP64 or FP32
// elements): tile t of the job writes the partial of rows
// [t*rpt, (t+1)*rpt) to part[t]; the finishing job adds the ntiles partials
// in order into out[0].
struct SumsqJob {
  const void* X; int64_t ld;
  int32_t rows, cols, f64, rpt;
  double* part;
};
struct SumsqFin {
  const double* part; double* out;
  int32_t ntiles, pad;
};

// Probe features of one matrix: eigenvalues of its 16 x 16 probe Gram
// (ld ldg) -> log10(sigma_j / sigma_1), floored, into out[0..15].
struct FeatJob {
  const double* gram; float* out;
  int32_t ldg, pad;
};

// Sketch profile: the diagonal of X = R^{-T} from the CholeskyQR Cholesky of
// the widest sketch (ld x ld, order L); k the target rank.
struct ProfJob {
  const double* sinv; float* out;
  int32_t ld, L, k, pad;
};

}  // namespace rg
