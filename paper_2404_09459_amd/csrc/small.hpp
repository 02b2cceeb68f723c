// Job descriptor and limits of the small FP64 steps.
#pragma once
#include <stdint.h>

namespace rg {

constexpr int SMALL_MAXN = 512;     // largest l1 + l2 of the compressed pair
constexpr double BETA_ZERO = 1e-14;
constexpr double CHOL_TRUNC_REL = 1e-10;   // truncated Cholesky: pivot / original diagonal
constexpr size_t SMALL_LDS_BYTES = 80000;   // dynamic LDS of k_small: Jacobi factors up to 10000 entries

// flag bits of info[4] (same values as the public header)
constexpr int FLAG_CHOL_FAIL = 0x4;
constexpr int FLAG_JACOBI_M = 0x8;
constexpr int FLAG_JACOBI_L1 = 0x10;
constexpr int FLAG_BETA_ZERO = 0x20;
constexpr int FLAG_ALPHA_ZERO = 0x40;
constexpr int FLAG_NONFINITE = 0x80;

// Block one-sided Jacobi for factors too large for k_small's LDS (order^2 >
// SMALL_LDS_BYTES / 8): columns in blocks of BJ_B (order <= 256) or BJ_B / 2
// (order <= 512); one workgroup per block pair and one launch per round
// (sweeps from BJ_SWEEP_WHOLE on: one launch per sweep with a barrier between
// rounds, when every workgroup of the launch fits on the device at once); at
// most BJ_SWEEPS sweeps are launched, the single-workgroup sweeps finish a
// factor that has not converged by then.
constexpr int BJ_B = 16;
constexpr int BJ_SWEEPS = 10;
constexpr int BJ_SWEEP_WHOLE = 7;   // default: sweeps from this one on take one launch each
constexpr int BJ_THREADS = 512;

// State of a block Jacobi run, shared by the staged small kernel and the
// sweep and round kernels (device memory, one per pair).
struct BJState {
  int32_t nc, nr, topk, done;       // columns, rows, dominant count, converged flag
  int32_t sweeps, rank, sw1, sw2;   // sweeps started; rank of M; sweeps on M and on H
  int32_t rot[3], pad;              // rotations seen in sweep s (slot s % 3)
  double thr;                       // skip threshold of the sweep (-1: none)
  double trM;                       // trace of M (M is overwritten by its factorisation)
  uint64_t rel[3];                  // largest gamma^2 / (alpha beta) turned in sweep s (slot
                                    // s % 3; bits of a non-negative double).  Three slots: the
                                    // first round of sweep s reads slot s - 1, clears slot s + 1
                                    // and the rounds of sweep s raise slot s
  uint32_t bar;                     // one-launch sweeps: workgroup arrivals at the barriers
                                    // between rounds since the start of the Jacobi
  int32_t fail;                     // a barrier wait ran out (the Jacobi ended unconverged)
};

// Sweeps reported for a block Jacobi whose barrier wait ran out: above any
// sweep limit, so the pair carries the sweep-limit flag.
constexpr int BJ_TIMEOUT_SWEEPS = 1 << 20;
// Polls of the barrier counter before a one-launch sweep gives up (each poll
// is a device-scope load and a short sleep, about a microsecond or more).
constexpr int BJ_SPIN = 1 << 20;

// One compressed pair: M = B B^T (N x N, ldm), the Gram of the stacked
// compressed pair B = [Q1^T G1; Q2^T G2], N = l1 + l2.
//
// stage 0 runs the whole step.  With the block Jacobi the step runs in
// stages: 1 factors M and stops before its Jacobi; 2 finishes that Jacobi,
// forms H, factors it and stops before its Jacobi when bjh is set (else
// runs to the end); 3 finishes the Jacobi on H and leaves the reciprocal
// norms of its factor's columns in ycs, for the product L Y that a
// multi-workgroup launch (k_ab) writes into Rcoef; 4 runs from there to the
// end.  With hgram set, stage 2 stops once L is formed, multi-workgroup
// launches (k_gram, k_reduce) form H = L1^T L1, and stage 5 factors H and
// stops before its Jacobi.
struct SmallJob {
  double* M; int64_t ldm;           // overwritten by the pivoted Cholesky
  int32_t l1, l2, t, maxsweep;
  double tol;
  int32_t stage, bjh;
  BJState* st;
  double* work;                     // N*t (L) + t*t (H) + N*N (Jacobi factor) doubles
  double* sigma;                    // N
  double *alpha, *beta, *theta, *P1, *P2, *D;
  double* X1t; int64_t ldx1;        // t x l1
  double* X2t; int64_t ldx2;        // t x l2
  double* Rcoef; int64_t ldr;       // t x N  ((L Y)^T)
  int32_t* info;
  double* ycs;                      // t: 1 / ||column c of H's factor|| (0 past its rank), stage 3
  int32_t hgram, pad2;
};

// sign convention of one pair: sgn[i] from row i of R (t x n)
// One block Jacobi factor: A (nr x nc, column-major, ld nr), nc read from
// the state; nblk = 2 P blocks, P workgroups per round; nrm2: squared column
// norms at the start of the sweep (nr entries).
struct BJJob {
  double* A; BJState* st; double* nrm2;
  double tol;
  int32_t nr, nblk;
};

struct SignJob {
  double* R; int64_t ldr; double* sgn; int32_t t, n;
};

}  // namespace rg
