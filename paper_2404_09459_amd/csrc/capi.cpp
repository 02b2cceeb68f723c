// C-ABI of the randomized GSVD: plan, workspace layout, job tables and the
// enqueue sequence of one run.  Host code only; the arithmetic is in the
// kernels.
//
// Sequence of one run (per pair; every launch is grouped over all matrices):
//   Omega_i^T <- generator                      (Algorithm 1's Gaussian block)
//   Y_i = G_i Omega_i ; Q_i = orth(Y_i)         (Algorithm 1's product and QR)
//   q times: W_i = orth(G_i^T Q_i); Q_i = orth(G_i W_i)   (subspace iteration)
//   B_i = Q_i^T G_i                             (Algorithm 2's compressed pair)
//   M = [B1; B2][B1; B2]^T ; small FP64 step    (Algorithm 2 with truncation)
//   R = (L Y)^T [B1; B2];  U = Q1 X1;  V = Q2 X2 (recovery after Algorithm 2)
// orth() is CholeskyQR with an FP64 Gram and Cholesky: one pass for the
// intermediate bases (their span is what the next product uses), two passes
// (CholeskyQR2) for the final Q_i.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rgsvd.h"
#include "common.hpp"
#include "jobs.hpp"
#include "launch.hpp"
#include "small.hpp"

using namespace rg;

namespace {

constexpr size_t ALIGN = 256;
inline size_t up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int64_t upi(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
inline int ct_of(int L) {
  int c = (L + 15) / 16;
  if (c <= 1) return 1;
  if (c <= 2) return 2;
  if (c <= 4) return 4;
  if (c <= 8) return 8;
  return 16;
}

enum Kind { K_ZERO, K_COPY, K_GEN, K_AB, K_GRAM, K_RED, K_CHOL, K_SMALL, K_SIGN, K_SCALE, K_GW, K_GTQ,
            K_PACK, K_SUMSQ, K_SUMFIN, K_FEAT, K_MLP, K_BJINIT, K_BJROUND, K_GW4, K_ZEROG, K_NN, K_PROF, K_TN,
            K_BJSWEEP };

enum Tag { T_ZERO, T_COPY, T_GEN, T_NN, T_TN, T_RED, T_GRAM, T_CHOL, T_SX, T_SMALL, T_RECOVER, T_SIGN,
           T_MGRAM, T_BJAC, T_NTAGS };

struct Stage {
  Kind kind;
  int tag = 0;
  size_t joff = 0, poff = 0;  // byte offsets of job array and prefix table in the job area
  int nj = 0, tiles = 0;
  int prec = 0, gdt = 0, rt = 1, ct = 1, js = 1;   // rt: rows per tile (K_GRAM: row groups per strip)
  int ta = 0, tb = 0, td = 0;
  bool sym = false, f64 = false, split = false;
  size_t zoff = 0, zbytes = 0;  // K_ZERO: workspace range
  int sweep = 0, round = 0;     // K_BJINIT, K_BJROUND, K_BJSWEEP (round: its first whole sweep)
  int spin = 0;                 // K_BJSWEEP: polls of its barrier before it gives up
};

struct CopyJob { const uint32_t* src; uint32_t* dst; int64_t nwords; };
struct PackJobH { const void* src; void* dst; int64_t ld; int32_t L, nst, bf16, pieces, f64src; };

struct SideLay {
  int m = 0, n = 0, l = 0, L = 0, which = 0, pair = 0;
  int ldy = 0, ldw = 0;
  int nchunk = 1, mchunk = 0;
  int gch_m = 1, gcl_m = 0, gch_n = 1, gcl_n = 0;
  size_t Yt = 0, Wt = 0, part = 0, gpart = 0, gram = 0, sinv = 0;
  size_t Yt16 = 0, Wt16 = 0, Yp32 = 0, Wp32 = 0;   // packed BF16 / FP32 operands (fragment order)
  size_t Xp16 = 0;                                  // R^-T of the CholeskyQR in three BF16 pieces (mixed)
  const void* G = nullptr; int64_t ldg = 0;
  uint64_t seed = 0; int stream = 1;
  // adaptive basis (Algorithm 1): Omega block buffer, rows formed so far,
  // current block width, per-side scalars (||G||_F^2, block energy) and the
  // partial sums behind them
  size_t Ot = 0, scal = 0, spart = 0;
  int cap = 0, lcur = 0, bcur = 0, gtiles = 0;
  bool active = false;
  int nchunk0 = 1, nchunk_max = 1;   // heuristic and largest row-chunk counts of G^T Q
  int tn_nchunk = 1, tn_mchunk = 0;  // row chunks of the mixed path's 8-wave G^T Q (k_tn)
};

struct PairLay {
  int64_t m = 0, p = 0, n = 0, k = 0, o = 0;
  int q = 0, l1 = 0, l2 = 0, t = 0, N = 0, Npad = 0;
  uint64_t seed = 0;
  int gch = 1, gcl = 0;
  size_t mpart = 0, M = 0, work = 0, sigma = 0, X1t = 0, X2t = 0, Rcoef = 0, sgn = 0, info = 0;
  size_t bjn = 0, bjs = 0;   // block Jacobi: column norms, state
  size_t alpha = 0;  // internal outputs when the caller passes null
  int l1cap = 0, l2cap = 0;
  rgsvd_out out{};
};

}  // namespace

struct rgsvd_plan_s {
  rgsvd_desc d{};
  uint64_t id = 0;    // unique per plan (the static scratch remembers which plan's tables it holds)
  uint64_t gen = 0;   // bumped whenever the job tables are rebuilt
  bool batched = false;
  int prec = 0, gdt = 0, mode = 0;
  int Lmax = 16, npadG = 64;
  std::vector<PairLay> pairs;
  std::vector<SideLay> sides;
  size_t off_jobs = 0, jobs_cap = 0, ws = 0;
  // adaptive sizing: which part build() emits, and the block size
  // FIXED: a whole fixed-size run.  A_INIT, A_BLOCK, TAIL: the steps of
  // Algorithm 1 (adaptive runs).  L_HEAD: the sketch of a learned run at its
  // widest grid width, whose first 16 columns give the probe features, and
  // the network on them (with `probe_only`, the features alone).  L_TAIL: the
  // rest of a learned run at one grid point (l, q).
  enum Part { FIXED, A_INIT, A_BLOCK, TAIL, L_HEAD, L_TAIL } part = FIXED;
  bool adaptive = false, learned = false;
  bool judge = false;        // learned run with tol > 0: residual test, adaptive fallback
  bool probe_only = false;
  bool append = false;       // build() adds to the job tables already in `host`
  int extra_flags = 0;       // ORed into the info template's flag word
  // learned runs: the head and one tail per grid point, built and uploaded
  // once per binding
  std::vector<Stage> lhead;
  std::vector<std::vector<Stage>> ltails;
  std::vector<std::pair<int, int>> lgrid;   // (l, q) of each tail
  int lmaxw = 16;                           // widest grid width
  bool lbound = false;
  hipGraphExec_t lhead_exec = nullptr;      // graphs of the head and of the tails
  std::vector<hipGraphExec_t> ltail_exec;   // (captured when first run)
  size_t off_feat = 0;      // probe features (32 floats), network output (2), activations (128)
  int block = 100;
  double* hscal = nullptr;   // pinned host copy of the per-side scalars
  // tile-shape knobs of the streaming kernels (0: heuristic); set by the
  // autotuner or taken from its per-shape cache.  tune_wg picks the mixed
  // path's streaming kernels over FP32 storage: 1 the 8-wave k_nn and k_tn,
  // 2 the per-wave k_gw, k_gw4 and k_gtq
  int tune_rt = 0, tune_js = 0, tune_chunk = 0, tune_wg = 0;
  int wave_slots = 2048;   // concurrently resident single-wave workgroups
  // job tables
  std::vector<unsigned char> host;   // serialized job tables
  std::vector<Stage> stages;
  void* pinned = nullptr;
  hipEvent_t ev = nullptr;
  bool ev_pending = false;
  // cache of the last bound pointers
  const void* lastG1 = nullptr; const void* lastG2 = nullptr; void* lastws = nullptr;
  int64_t lastld1 = 0, lastld2 = 0;
  rgsvd_out lastout{};
  bool bound = false;
  // batched graph
  hipGraphExec_t gexec = nullptr;
  void* bws = nullptr;
  // sizing network
  float* mlp = nullptr;
  // per-stage event profiling
  bool prof = false;
  std::vector<hipEvent_t> pev;
  int prof_count = 0;
  const std::vector<Stage>* prof_list = nullptr;   // the stage list the events bracket
};

namespace {

bool out_eq(const rgsvd_out& a, const rgsvd_out& b) { return std::memcmp(&a, &b, sizeof(a)) == 0; }

// --------------------------------------------------------------- layout --
int layout(rgsvd_plan_s* P) {
  const int prec = P->prec;
  // a learned run with a judge may fall back to Algorithm 1 in FP64 on the
  // same buffers: they are laid out for FP64 and the adaptive steps
  const bool fb = P->adaptive || P->judge;
  const size_t wsz = (prec == P64 || fb) ? 8 : 4;   // working element size
  const size_t psz = wsz;                            // partial element size
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = up(off + bytes, ALIGN); return o; };
  // adaptive runs grow Q by blocks written 16-row aligned at offset l: one
  // spare 16-row group past the capacity
  const int spare = fb ? 16 : 0;
  P->Lmax = 16;
  for (auto& pr : P->pairs) P->Lmax = std::max(P->Lmax, (int)upi(std::max(pr.l1, pr.l2), 16) + spare);
  P->npadG = (int)upi(P->Lmax, 64);
  const int nsides = 2 * (int)P->pairs.size();
  P->sides.clear();
  for (size_t pi = 0; pi < P->pairs.size(); ++pi) {
    PairLay& pr = P->pairs[pi];
    for (int w = 0; w < 2; ++w) {
      SideLay s;
      s.pair = (int)pi; s.which = w;
      s.m = (int)(w ? pr.p : pr.m); s.n = (int)pr.n;
      s.l = w ? pr.l2 : pr.l1;
      s.cap = s.l;
      s.L = (int)upi(s.l, 16) + spare;
      s.ldy = (int)upi(s.m, 64); s.ldw = (int)upi(s.n, 64);
      s.seed = pr.seed; s.stream = w ? 2 : 1;
      // G^T Q row chunks.  One pair: enough single-wave tiles to fill the
      // wave slots once, all waves of equal length.  A batch of uneven pairs:
      // sides shorter than a slot's share would leave the long sides' waves
      // running alone at the end, so waves get a quarter of the share (at
      // least 8 L rows, so that a chunk's L x n partial adds at most an
      // eighth to the pass's traffic) and the wave slots balance them.
      int js = (prec == P64 || P->gdt == RGSVD_F64 || s.L > 128) ? 2 : 4;
      int jt = (int)((s.n + 16 * js - 1) / (16 * js));
      int nch;
      if (P->pairs.size() == 1) {
        int64_t rows_all = 0;
        for (auto& q : P->pairs) rows_all += q.m + q.p;
        nch = (int)std::max<int64_t>(1, (int64_t)P->wave_slots * s.m / std::max<int64_t>(1, rows_all * jt));
      } else {
        int64_t work = 0;   // sum over sides of rows x column tiles
        for (auto& q : P->pairs) {
          const int qjs = (prec == P64 || P->gdt == RGSVD_F64 || (int)upi(std::max(q.l1, q.l2), 16) > 128) ? 2 : 4;
          work += (q.m + q.p) * ((q.n + 16 * qjs - 1) / (16 * qjs));
        }
        const int64_t share = work / std::max(1, P->wave_slots);
        const int64_t rows = std::max<int64_t>({share / 4, 8 * (int64_t)s.L, 256});
        nch = (int)((s.m + rows - 1) / rows);
      }
      nch = std::max(1, std::min(nch, (s.m + 255) / 256));
      int mch = (int)upi((s.m + nch - 1) / nch, 32);
      nch = (s.m + mch - 1) / mch;
      s.nchunk = nch; s.mchunk = mch;
      s.nchunk0 = nch;
      s.nchunk_max = std::max(1, std::min(2 * nch, (s.m + 31) / 32));
      if (prec == PBF && P->gdt != RGSVD_F64) {
        // k_tn: about two 8-wave workgroups per CU over all sides, chunks
        // in proportion to the rows, at least 256 rows each
        int64_t rows_all = 0;
        for (auto& q : P->pairs) rows_all += q.m + q.p;
        const int64_t wpc = ((s.n + 31) / 32 + TN_WAVES - 1) / TN_WAVES;
        int64_t tn = 2 * (int64_t)(P->wave_slots / 4) * s.m / std::max<int64_t>(1, rows_all * wpc);
        tn = std::max<int64_t>(1, std::min<int64_t>(tn, (s.m + 255) / 256));
        s.tn_mchunk = (int)upi((s.m + tn - 1) / tn, 32);
        s.tn_nchunk = (s.m + s.tn_mchunk - 1) / s.tn_mchunk;
        s.nchunk_max = std::max(s.nchunk_max, s.tn_nchunk);
      }
      // Gram chunks over m and over n
      int nb = P->npadG / 64, nblk = nb * (nb + 1) / 2;
      // (about 512 tiles in all, but no chunk longer than 1024 rows: a batch of
      // many sides would otherwise leave one long chunk per side)
      int gt = std::max(1, 512 / std::max(1, nblk * nsides));
      s.gch_m = std::max(1, std::min((s.m + 255) / 256, std::max(gt, (s.m + 1023) / 1024)));
      s.gcl_m = (int)upi((s.m + s.gch_m - 1) / s.gch_m, 32);
      s.gch_m = (s.m + s.gcl_m - 1) / s.gcl_m;
      s.gch_n = std::max(1, std::min((s.n + 255) / 256, std::max(gt, (s.n + 1023) / 1024)));
      s.gcl_n = (int)upi((s.n + s.gch_n - 1) / s.gch_n, 32);
      s.gch_n = (s.n + s.gcl_n - 1) / s.gcl_n;
      s.Yt = take((size_t)s.L * s.ldy * wsz);
      s.Wt = take((size_t)s.L * s.ldw * wsz);
      if (prec == PBF) {
        // three BF16 pieces each: the FP32-accurate split passes use them all
        s.Yt16 = take((size_t)3 * s.L * s.ldy * 2);
        s.Wt16 = take((size_t)3 * s.L * s.ldw * 2);
        s.Xp16 = take((size_t)3 * P->npadG * P->npadG * 2);
      }
      if (prec != P64) {
        s.Yp32 = take((size_t)s.L * s.ldy * 4);
        s.Wp32 = take((size_t)s.L * s.ldw * 4);
      }
      s.part = take((size_t)s.nchunk_max * s.L * s.ldw * psz);
      int gch = std::max(s.gch_m, s.gch_n);
      s.gpart = take((size_t)gch * P->npadG * P->npadG * 8);
      s.gram = take((size_t)P->npadG * P->npadG * 8);
      s.sinv = take((size_t)P->npadG * P->npadG * 8);
      if (fb) {
        const int lb = (int)upi(std::min(P->block, s.cap), 16);
        s.Ot = take((size_t)lb * s.ldw * wsz);
        s.scal = take(8 * 8);
        s.gtiles = (s.m + 63) / 64;
        s.spart = take((size_t)std::max(s.gtiles, 64) * 8);
      }
      P->sides.push_back(s);
    }
  }
  for (auto& pr : P->pairs) {
    pr.N = pr.l1 + pr.l2;
    pr.Npad = (int)upi(pr.N, 64);
    int nb = pr.Npad / 64, nblk = nb * (nb + 1) / 2;
    int gt = std::max(1, 512 / std::max(1, nblk * (int)P->pairs.size()));
    pr.gch = std::max(1, std::min((int)((pr.n + 255) / 256), std::max(gt, (int)((pr.n + 1023) / 1024))));
    pr.gcl = (int)upi((pr.n + pr.gch - 1) / pr.gch, 32);
    pr.gch = (int)((pr.n + pr.gcl - 1) / pr.gcl);
    pr.mpart = take((size_t)pr.gch * pr.Npad * pr.Npad * 8);
    pr.M = take((size_t)pr.Npad * pr.Npad * 8);
    size_t N = pr.N, t = pr.t;
    pr.work = take((N * t + t * t + N * N) * 8);
    pr.bjn = take(N * 8);
    pr.bjs = take(sizeof(BJState));
    pr.sigma = take(N * 8);
    pr.X1t = take(t * pr.l1 * 8);
    pr.X2t = take(t * pr.l2 * 8);
    pr.Rcoef = take(t * N * 8);
    pr.sgn = take(t * 8);
    pr.info = take(RGSVD_INFO_WORDS * 4);
    pr.alpha = take(t * 8 * 5 + 16);   // alpha, beta, theta, P1, P2, D when not given
  }
  P->off_feat = take((RGSVD_MLP_IN + RGSVD_MLP_OUT + 2 * 64 + 2) * sizeof(float));
  // job area: generous bound
  size_t per_side = 64 * 1024 + (size_t)(P->sides.empty() ? 0 : P->sides[0].nchunk_max) * 256;
  P->jobs_cap = up(per_side * nsides + 256 * 1024, ALIGN);
  if (P->learned) P->jobs_cap *= 24;   // the head and up to 20 tails (one per grid point)
  P->off_jobs = take(P->jobs_cap);
  P->ws = off;
  return RGSVD_OK;
}

// ------------------------------------------------------------ job tables --
struct Builder {
  rgsvd_plan_s* P;
  std::vector<unsigned char>& h;
  explicit Builder(rgsvd_plan_s* p) : P(p), h(p->host) {}
  template <typename T>
  size_t put(const std::vector<T>& v) {
    size_t o = up(h.size(), 64);
    h.resize(o + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(h.data() + o, v.data(), v.size() * sizeof(T));
    return o;
  }
  // add a stage from jobs and per-job tile counts
  template <typename T>
  Stage& add(Kind k, const std::vector<T>& jobs, const std::vector<int>& tiles) {
    Stage s;
    s.kind = k;
    s.joff = put(jobs);
    std::vector<int> pre(jobs.size() + 1, 0);
    for (size_t i = 0; i < jobs.size(); ++i) pre[i + 1] = pre[i] + tiles[i];
    s.poff = put(pre);
    s.nj = (int)jobs.size();
    s.tiles = pre.back();
    P->stages.push_back(s);
    return P->stages.back();
  }
};

inline char* WS(void* ws, size_t off) { return (char*)ws + off; }

int build(rgsvd_plan_s* P, void* ws) {
  if (!P->append) P->host.clear();
  P->stages.clear();
  Builder B(P);
  const int prec = P->prec;
  const int wt = (prec == P64) ? 0 : 1;            // working type code
  const int gt = (P->gdt == RGSVD_F64) ? 0 : 1;
  const bool mixed = (prec == PBF);
  const int ctL = ct_of([&] { int L = 16; for (auto& s : P->sides) L = std::max(L, s.L); return L; }());
  // k_nn and k_tn share each k-step's W or Q^T across 8 waves behind one
  // barrier; with up to 4 row tiles (L <= 64) a step holds too few MFMAs to
  // pay for it, and the per-wave kernels are faster (a batch of narrow pairs)
  const bool wg8 = mixed && gt == 1 && (P->tune_wg ? P->tune_wg == 1 : ctL >= 8);
  std::vector<SideLay>& S = P->sides;
  const int ns = (int)S.size();
  // row chunks of the G^T Q reductions: heuristic, half or twice as many
  for (auto& s : S) {
    int nch = s.nchunk0;
    if (P->tune_chunk == 1) nch = std::max(1, nch / 2);
    if (P->tune_chunk == 2) nch = std::min(s.nchunk_max, 2 * nch);
    s.mchunk = (int)upi((s.m + nch - 1) / nch, 32);
    s.nchunk = (s.m + s.mchunk - 1) / s.mchunk;
  }

  const auto part = P->part;
  const bool head = (part == rgsvd_plan_s::FIXED || part == rgsvd_plan_s::A_INIT ||
                     part == rgsvd_plan_s::L_HEAD);
  const bool tail = (part == rgsvd_plan_s::FIXED || part == rgsvd_plan_s::TAIL ||
                     part == rgsvd_plan_s::L_TAIL);
  // 0. zero the W buffers (their padding rows must read as zero) and copy
  //    the info templates
  if (head) {
    // one grouped launch for every side's W and Y buffers
    std::vector<ZeroJob> zj; std::vector<int> zt;
    const size_t esz = prec == P64 ? 8 : 4;
    for (auto& s : S) {
      for (int y = 0; y < 2; ++y) {
        const size_t bytes = (size_t)s.L * (y ? s.ldy : s.ldw) * esz;
        zj.push_back(ZeroJob{(uint32_t*)WS(ws, y ? s.Yt : s.Wt), (int64_t)(bytes / 4)});
        zt.push_back((int)((bytes / 4 + 4095) / 4096));
      }
    }
    B.add(K_ZEROG, zj, zt).tag = T_ZERO;
  }
  if ((head && !P->probe_only) || part == rgsvd_plan_s::TAIL || part == rgsvd_plan_s::L_TAIL) {
    // the tails of adaptive and learned runs rewrite the words with the
    // final sizes (flags raised before are kept)
    const int nw = head ? RGSVD_INFO_WORDS : 4;
    std::vector<uint32_t> tmpl;
    std::vector<CopyJob> cj;
    std::vector<int> tl;
    for (auto& pr : P->pairs) {
      uint32_t w[RGSVD_INFO_WORDS] = {0};
      w[1] = pr.l1; w[2] = pr.l2; w[3] = P->adaptive ? 0 : pr.q;
      w[RGSVD_INFO_FLAGS] = (uint32_t)P->extra_flags;
      for (int i = 0; i < RGSVD_INFO_WORDS; ++i) tmpl.push_back(w[i]);
    }
    size_t toff = B.put(tmpl);
    for (size_t i = 0; i < P->pairs.size(); ++i) {
      auto& pr = P->pairs[i];
      int32_t* info = pr.out.info ? pr.out.info : (int32_t*)WS(ws, pr.info);
      cj.push_back(CopyJob{(const uint32_t*)WS(ws, P->off_jobs + toff) + i * RGSVD_INFO_WORDS,
                           (uint32_t*)info, nw});
      tl.push_back(1);
    }
    B.add(K_COPY, cj, tl).tag = T_COPY;
  }
  auto info_of = [&](int pair) -> int32_t* {
    auto& pr = P->pairs[pair];
    return pr.out.info ? pr.out.info : (int32_t*)WS(ws, pr.info);
  };

  // 1. Omega
  if (part == rgsvd_plan_s::FIXED || part == rgsvd_plan_s::L_HEAD) {
    std::vector<GenJob> j; std::vector<int> tl;
    for (auto& s : S) {
      GenJob g{};
      g.Wt = WS(ws, s.Wt); g.ldw = s.ldw; g.seed = s.seed; g.n = s.n; g.col0 = 0;
      g.ncols = s.l; g.L = s.L; g.stream = s.stream;
      j.push_back(g);
      int ngr = ((s.l - 1) >> 2) + 1;
      tl.push_back(((s.n + 255) / 256) * ngr);
    }
    Stage& st = B.add(K_GEN, j, tl);
    st.f64 = (prec == P64); st.tag = T_GEN;
  }

  // the W (ymat = false) or Q (ymat = true) buffers packed in MFMA fragment
  // order for a BF16 or FP32 pass (k-steps of 32 or 16 columns)
  auto pack_dst = [&](const SideLay& s, bool ymat, int p) -> size_t {
    return p == PBF ? (ymat ? s.Yt16 : s.Wt16) : (ymat ? s.Yp32 : s.Wp32);
  };
  auto add_pack = [&](bool ymat, int p, int pieces = 1) {
    std::vector<PackJobH> j; std::vector<int> tl;
    const int ks = p == PBF ? 32 : 16;
    for (auto& s : S) {
      PackJobH c{};
      const int len = ymat ? s.m : s.n;
      c.src = (const float*)WS(ws, ymat ? s.Yt : s.Wt);
      c.dst = WS(ws, pack_dst(s, ymat, p));
      c.ld = ymat ? s.ldy : s.ldw; c.L = s.L; c.nst = (len + ks - 1) / ks; c.bf16 = p == PBF;
      c.pieces = pieces;
      j.push_back(c);
      tl.push_back((int)(((int64_t)c.nst * (s.L / 16) * 64 + 255) / 256));
    }
    B.add(K_PACK, j, tl).tag = T_ZERO;
  };

  auto add_nn = [&](int p) {
    if (wg8) {
      // mixed path over FP32 G: 8-wave workgroups sharing the packed W in
      // LDS; the BF16 passes round G and W to BF16, the last power pass
      // (FP32 in the method) runs the FP32-accurate three-piece split
      const bool split = p == P32;
      add_pack(false, PBF, split ? 3 : 1);
      // two 16-row tiles per wave reuse each W fragment twice; the split
      // pass with 16 column tiles keeps one (its registers are full)
      const int rt = (split && ctL >= 16) ? 1 : 2;
      const int wrows = 16 * rt * 8;
      std::vector<NnJob> j; std::vector<int> tl;
      for (auto& s : S) {
        NnJob x{};
        x.G = s.G; x.Wt = WS(ws, s.Wt16); x.Yt = WS(ws, s.Yt);
        x.ldg = s.ldg; x.ldw = s.ldw; x.ldy = s.ldy; x.m = s.m; x.n = s.n; x.L = s.L;
        j.push_back(x);
        tl.push_back((s.m + wrows - 1) / wrows);
      }
      Stage& st = B.add(K_NN, j, tl);
      st.split = split; st.rt = rt; st.ct = ctL; st.tag = T_NN;
      return;
    }
    if (p != P64) add_pack(false, p);
    if (p == P32 && gt == 1) {
      // FP32 pass over FP32 G (MFMA-bound): 4-wave workgroups of 64 rows
      // sharing the packed W through LDS.  The HBM-bound BF16 passes keep the
      // single-wave 64-row tiles, measured faster.
      std::vector<NnJob> j; std::vector<int> tl;
      for (auto& s : S) {
        NnJob x{};
        x.G = s.G; x.Wt = WS(ws, pack_dst(s, false, p)); x.Yt = WS(ws, s.Yt);
        x.ldg = s.ldg; x.ldw = s.ldw; x.ldy = s.ldy; x.m = s.m; x.n = s.n; x.L = s.L;
        j.push_back(x);
        tl.push_back((s.m + 63) / 64);
      }
      Stage& st = B.add(K_GW4, j, tl);
      st.prec = p; st.gdt = gt; st.ct = ctL; st.tag = T_NN;
      return;
    }
    std::vector<NnJob> j; std::vector<int> tl;
    const bool rt4_ok = !(p == P64 || gt == 0 || ctL > 8);
    int rt = P->tune_rt ? (P->tune_rt == 4 && rt4_ok ? 4 : 1) : (rt4_ok ? 4 : 1);
    // FP64 over more than 8 column tiles: two jobs per side, the first 128
    // columns of Y and the rest (8 tiles' accumulators and operands fill a
    // wave's registers; G is read twice)
    const bool halves = p == P64 && ctL > 8;
    for (auto& s : S) {
      for (int h = 0; h < (halves ? 2 : 1); ++h) {
        const int r0 = h * 128;
        if (r0 >= s.L) break;
        NnJob x{};
        const size_t wsz8 = p == P64 ? 8 : 0;
        x.G = s.G;
        x.Wt = p == P64 ? (const void*)(WS(ws, s.Wt) + (size_t)r0 * s.ldw * wsz8) : WS(ws, pack_dst(s, false, p));
        x.Yt = WS(ws, s.Yt) + (size_t)r0 * s.ldy * (p == P64 ? 8 : 4);
        x.ldg = s.ldg; x.ldw = s.ldw; x.ldy = s.ldy; x.m = s.m; x.n = s.n;
        x.L = halves ? std::min(128, s.L - r0) : s.L;
        j.push_back(x);
        tl.push_back((s.m + 16 * rt - 1) / (16 * rt));
      }
    }
    Stage& st = B.add(K_GW, j, tl);
    st.prec = p; st.gdt = gt; st.rt = rt; st.ct = halves ? 8 : ctL; st.tag = T_NN;
  };

  // CholeskyQR passes on the Yt (ymat = true) or Wt buffers
  auto add_orth = [&](bool ymat, int passes) {
    const int sxp = (prec == P64) ? P64 : P32;
    for (int ps = 0; ps < passes; ++ps) {
      std::vector<GramJob> gj; std::vector<int> gtl;
      std::vector<RedJob> rj; std::vector<int> rtl;
      std::vector<CholJob> cj; std::vector<int> ctl;
      std::vector<AbJob> aj; std::vector<int> atl;
      const int nb = P->npadG / 64, nblk = nb * (nb + 1) / 2;
      for (auto& s : S) {
        int len = ymat ? s.m : s.n;
        int ld = ymat ? s.ldy : s.ldw;
        void* X = WS(ws, ymat ? s.Yt : s.Wt);
        int gch = ymat ? s.gch_m : s.gch_n, gcl = ymat ? s.gcl_m : s.gcl_n;
        GramJob g{};
        g.X1 = X; g.X2 = nullptr; g.out = (double*)WS(ws, s.gpart);
        g.ld1 = ld; g.ld2 = 0; g.r1 = s.L; g.r2 = 0; g.k0 = 0; g.k1 = len;
        g.npad = P->npadG; g.clen = gcl;
        g.rgs = gram_rgs(s.L, gch);
        gj.push_back(g); gtl.push_back(gram_strips(s.L, g.rgs) * gch);
        RedJob r{};
        r.in = WS(ws, s.gpart); r.out = WS(ws, s.gram); r.sq = nullptr;
        r.stride = (int64_t)P->npadG * P->npadG; r.count = r.stride;
        r.nparts = gch; r.rows = P->npadG; r.cols = P->npadG; r.ldo = P->npadG; r.ldi = P->npadG;
        r.nz = s.L;
        rj.push_back(r); rtl.push_back((int)((r.count + 255) / 256));
        CholJob c{};
        c.gram = (const double*)WS(ws, s.gram); c.sinv = (double*)WS(ws, s.sinv);
        c.info = info_of(s.pair); c.N = s.l; c.npad = P->npadG; c.flagbit = ymat ? 0 : 1;
        cj.push_back(c); ctl.push_back(1);
        AbJob a{};
        a.A = WS(ws, s.sinv); a.lda = P->npadG; a.B = X; a.ldb = ld; a.D = X; a.ldd = ld;
        a.rows = s.L; a.K = s.L; a.J = len; a.accumulate = 0; a.colscale = nullptr;
        aj.push_back(a);
        // one column per lane in the FP32 update Q = Y R^{-1}: twice the
        // workgroups of two, measured faster at l = 110 (the update is latency-bound)
        int js = (sxp == P64) ? 2 : 1;
        atl.push_back((len + 64 * js - 1) / (64 * js));
      }
      const int rgs = gram_uniform(gj, gtl);
      Stage& gs = B.add(K_GRAM, gj, gtl); gs.ta = wt; gs.rt = rgs; gs.tag = T_GRAM;
      Stage& r = B.add(K_RED, rj, rtl); r.sym = true; r.ta = 0; r.td = 0; r.tag = T_RED;
      Stage& c = B.add(K_CHOL, cj, ctl); c.tag = T_CHOL;
      if (mixed) {
        // the mixed path: R^-T packed in three BF16 pieces, then Q^T = R^-T Y^T
        // in place on k_tn's three-piece products (one row chunk: K = L)
        std::vector<PackJobH> pj; std::vector<int> ptl;
        std::vector<AbJob> tj; std::vector<int> ttl;
        const int ctn = [&] { int t = 1; for (auto& s : S) t = std::max(t, s.L / 16); return t; }();
        const int tct = ctn == 1 ? 1 : std::min(16, (ctn + 1) & ~1);
        for (auto& s : S) {
          const int len = ymat ? s.m : s.n;
          const int ld = ymat ? s.ldy : s.ldw;
          const int nst = (s.L + 31) / 32;
          PackJobH pk{};
          pk.src = WS(ws, s.sinv); pk.dst = WS(ws, s.Xp16); pk.ld = P->npadG; pk.L = s.L; pk.nst = nst;
          pk.bf16 = 1; pk.pieces = 3; pk.f64src = 1;
          pj.push_back(pk);
          ptl.push_back((int)(((int64_t)nst * (s.L / 16) * 64 + 255) / 256));
          AbJob a{};
          a.A = WS(ws, s.Xp16); a.lda = (int64_t)nst * s.L * 32;   // elements between pieces
          a.B = WS(ws, ymat ? s.Yt : s.Wt); a.ldb = ld;
          a.D = WS(ws, ymat ? s.Yt : s.Wt); a.ldd = ld;
          a.rows = s.L; a.K = s.L; a.J = len; a.accumulate = 0; a.colscale = nullptr;
          tj.push_back(a);
          ttl.push_back(tn_tiles_per_chunk(true, tct, len));
        }
        B.add(K_PACK, pj, ptl).tag = T_SX;
        Stage& a = B.add(K_TN, tj, ttl);
        a.split = true; a.ct = tct; a.tag = T_SX;
        continue;
      }
      Stage& a = B.add(K_AB, aj, atl);
      a.prec = sxp; a.ta = 0; a.tb = wt; a.td = wt; a.ct = ctL; a.tag = T_SX;
      a.js = (sxp == P64) ? 2 : 1;
    }
  };

  // G^T Q (or Q^T G) into the Wt buffers: split over row chunks then reduced
  auto add_tn = [&](int p) {
    if (wg8) {
      // mixed path over FP32 G: 8-wave workgroups sharing the packed Q^T in
      // LDS; the BF16 pass rounds both operands, the FP32 passes of the
      // method run the three-piece split
      const bool split = p == P32;
      add_pack(true, PBF, split ? 3 : 1);
      // row tiles: the largest side's count, rounded up to even
      const int ctn = [&] { int t = 1; for (auto& s : S) t = std::max(t, s.L / 16); return t; }();
      const int tct = ctn == 1 ? 1 : std::min(16, (ctn + 1) & ~1);
      std::vector<AbJob> aj; std::vector<int> atl;
      std::vector<RedJob> rj; std::vector<int> rtl;
      for (auto& s : S) {
        const int64_t pstride = (int64_t)((s.m + 31) / 32) * s.L * 32;   // elements between BF16 pieces
        for (int c = 0; c < s.tn_nchunk; ++c) {
          const int r0 = c * s.tn_mchunk;
          AbJob a{};
          a.A = (const char*)WS(ws, s.Yt16) + (size_t)r0 * s.L * 2; a.lda = pstride;
          a.B = (const char*)s.G + (size_t)r0 * s.ldg * 4; a.ldb = s.ldg;
          a.D = WS(ws, s.part) + (size_t)c * s.L * s.ldw * 4; a.ldd = s.ldw;
          a.rows = s.L; a.K = std::min(s.tn_mchunk, s.m - r0); a.J = s.n; a.accumulate = 0; a.colscale = nullptr;
          aj.push_back(a);
          atl.push_back(tn_tiles_per_chunk(split, tct, s.n));
        }
        RedJob r{};
        r.in = WS(ws, s.part); r.out = WS(ws, s.Wt); r.sq = nullptr;
        r.stride = (int64_t)s.L * s.ldw; r.count = (int64_t)s.L * s.n;
        r.nparts = s.tn_nchunk; r.rows = s.L; r.cols = s.n; r.ldo = s.ldw; r.ldi = s.ldw;
        rj.push_back(r); rtl.push_back((int)((r.count + 255) / 256));
      }
      Stage& a = B.add(K_TN, aj, atl);
      a.split = split; a.ct = tct; a.tag = T_TN;
      Stage& r = B.add(K_RED, rj, rtl);
      r.sym = false; r.ta = wt; r.td = wt; r.tag = T_RED;
      return;
    }
    if (p != P64) add_pack(true, p);
    std::vector<AbJob> aj; std::vector<int> atl;
    std::vector<RedJob> rj; std::vector<int> rtl;
    // FP64 over more than 8 row tiles: two jobs per chunk, rows [0, 128) of
    // D and the rest (as in the G W pass)
    const bool halves = p == P64 && ctL > 8;
    const bool js4_ok = !(p == P64 || gt == 0 || ctL > 8);
    const int js = P->tune_js ? (P->tune_js == 4 && js4_ok ? 4 : 2) : (js4_ok ? 4 : 2);
    const size_t psz = (prec == P64) ? 8 : 4;
    const size_t asz = (p == P64) ? 8 : (p == P32 ? 4 : 2);
    for (auto& s : S) {
      for (int c = 0; c < s.nchunk; ++c) {
        int r0 = c * s.mchunk;
        int rows = std::min(s.mchunk, s.m - r0);
        AbJob a{};
        // packed operands start at the chunk's first k-step (r0 is a multiple of 32)
        a.A = p == P64 ? (const char*)WS(ws, s.Yt) + (size_t)r0 * asz
                       : (const char*)WS(ws, pack_dst(s, true, p)) + (size_t)r0 * s.L * asz;
        a.lda = s.ldy;
        a.B = (const char*)s.G + (size_t)r0 * s.ldg * (gt == 0 ? 8 : 4); a.ldb = s.ldg;
        a.D = WS(ws, s.part) + (size_t)c * s.L * s.ldw * psz; a.ldd = s.ldw;
        a.rows = s.L; a.K = rows; a.J = s.n; a.accumulate = 0; a.colscale = nullptr;
        if (halves) {
          // P64 reads Q^T unpacked (row c at c lda): the second job starts at row 128
          for (int h = 0; h < 2 && h * 128 < s.L; ++h) {
            AbJob b = a;
            b.A = (const char*)a.A + (size_t)h * 128 * s.ldy * 8;
            b.D = (char*)a.D + (size_t)h * 128 * s.ldw * psz;
            b.rows = std::min(128, s.L - h * 128);
            aj.push_back(b);
            atl.push_back((s.n + 16 * js - 1) / (16 * js));
          }
          continue;
        }
        aj.push_back(a);
        atl.push_back((s.n + 16 * js - 1) / (16 * js));
      }
      RedJob r{};
      r.in = WS(ws, s.part); r.out = WS(ws, s.Wt); r.sq = nullptr;
      r.stride = (int64_t)s.L * s.ldw; r.count = (int64_t)s.L * s.n;
      r.nparts = s.nchunk; r.rows = s.L; r.cols = s.n; r.ldo = s.ldw; r.ldi = s.ldw;
      rj.push_back(r); rtl.push_back((int)((r.count + 255) / 256));
    }
    Stage& a = B.add(K_GTQ, aj, atl);
    a.prec = p; a.gdt = gt; a.ct = halves ? 8 : ctL; a.js = js; a.tag = T_TN;
    Stage& r = B.add(K_RED, rj, rtl);
    r.sym = false; r.ta = wt; r.td = wt; r.tag = T_RED;
  };

  // sums of squares (adaptive runs and the residual judge of learned runs):
  // jobs and their finishing sums
  auto add_sumsq = [&](std::vector<SumsqJob>& j, std::vector<int>& tl, std::vector<SumsqFin>& f) {
    Stage& a = B.add(K_SUMSQ, j, tl); a.tag = T_RED;
    std::vector<int> ftl(f.size(), 1);
    B.add(K_SUMFIN, f, ftl).tag = T_RED;
  };
  // ||G_i||_F^2 into scal[0] (FP64 partials over 64-row slabs, summed in order)
  auto add_gnorm = [&]() {
    std::vector<SumsqJob> j; std::vector<int> tl; std::vector<SumsqFin> f;
    for (auto& s : S) {
      j.push_back(SumsqJob{s.G, s.ldg, s.m, s.n, gt == 0 ? 1 : 0, 64, (double*)WS(ws, s.spart)});
      tl.push_back(s.gtiles);
      f.push_back(SumsqFin{(const double*)WS(ws, s.spart), (double*)WS(ws, s.scal), s.gtiles, 0});
    }
    add_sumsq(j, tl, f);
  };

  if (part == rgsvd_plan_s::FIXED || part == rgsvd_plan_s::L_HEAD)
    add_nn(mixed ? PBF : prec);   // sketch
  if (part == rgsvd_plan_s::L_HEAD) {
    // features: the probe (the sketch's first 16 columns, which Omega's
    // global columns make the 16-column sketch): their FP64 Gram, its
    // eigenvalues, log10 of the normalised singular values; then the first
    // CholeskyQR pass over the whole sketch, whose factor's diagonal is the
    // profile (its Q stays in Yt: every tail starts from its prefix); then
    // the network
    std::vector<GramJob> gj; std::vector<int> gtl;
    std::vector<RedJob> rj; std::vector<int> rtl;
    std::vector<FeatJob> fj; std::vector<int> ftl;
    for (size_t i = 0; i < S.size(); ++i) {
      auto& s = S[i];
      GramJob g{};
      g.X1 = WS(ws, s.Yt); g.X2 = nullptr; g.out = (double*)WS(ws, s.gpart);
      g.ld1 = s.ldy; g.ld2 = 0; g.r1 = 16; g.r2 = 0; g.k0 = 0; g.k1 = s.m; g.npad = 64; g.clen = s.gcl_m;
      g.rgs = gram_rgs(16, s.gch_m);
      gj.push_back(g); gtl.push_back(gram_strips(16, g.rgs) * s.gch_m);
      RedJob r{};
      r.in = WS(ws, s.gpart); r.out = WS(ws, s.gram); r.sq = nullptr;
      r.stride = 64 * 64; r.count = r.stride;
      r.nparts = s.gch_m; r.rows = 64; r.cols = 64; r.ldo = 64; r.ldi = 64; r.nz = 16;
      rj.push_back(r); rtl.push_back((int)((r.count + 255) / 256));
      fj.push_back(FeatJob{(const double*)WS(ws, s.gram), (float*)WS(ws, P->off_feat) + 16 * i, 64, 0});
      ftl.push_back(1);
    }
    const int rgs = gram_uniform(gj, gtl);
      Stage& gs = B.add(K_GRAM, gj, gtl); gs.ta = wt; gs.rt = rgs; gs.tag = T_GRAM;
    Stage& r = B.add(K_RED, rj, rtl); r.sym = true; r.ta = 0; r.td = 0; r.tag = T_RED;
    B.add(K_FEAT, fj, ftl).tag = T_SMALL;
    add_orth(true, 1);
    std::vector<ProfJob> pj; std::vector<int> ptl;
    for (size_t i = 0; i < S.size(); ++i)
      pj.push_back(ProfJob{(const double*)WS(ws, S[i].sinv), (float*)WS(ws, P->off_feat) + 16 * i + 8, P->npadG,
                           S[i].l, (int)P->pairs[S[i].pair].k, 0});
    ptl.assign(pj.size(), 1);
    B.add(K_PROF, pj, ptl).tag = T_SMALL;
    if (!P->probe_only) {
      if (P->mlp) { Stage m; m.kind = K_MLP; m.tag = T_SMALL; P->stages.push_back(m); }
      if (P->judge) add_gnorm();
    }
    if (P->host.size() > P->jobs_cap) return RGSVD_ENOMEM;
    return RGSVD_OK;
  }
  if (part == rgsvd_plan_s::L_TAIL) {
    // the chosen width l <= the head's: the sketch rows [l, L) are cleared
    std::vector<ZeroJob> zj; std::vector<int> zt;
    const size_t esz = prec == P64 ? 8 : 4;
    for (auto& s : S) {
      const size_t bytes = (size_t)(upi(P->lmaxw, 16) - s.l) * s.ldy * esz;
      if (bytes == 0) continue;
      zj.push_back(ZeroJob{(uint32_t*)(WS(ws, s.Yt) + (size_t)s.l * s.ldy * esz), (int64_t)(bytes / 4)});
      zt.push_back((int)((bytes / 4 + 4095) / 4096));
    }
    if (!zj.empty()) B.add(K_ZEROG, zj, zt).tag = T_ZERO;
  }
  if (part == rgsvd_plan_s::FIXED || part == rgsvd_plan_s::L_TAIL) {
    const int qmax = [&] { int q = 0; for (auto& pr : P->pairs) q = std::max(q, pr.q); return q; }();
    // a learned tail starts after the head's first pass at the widest width
    // (the prefix of its Q is the first pass at width l)
    const int first = (qmax == 0 ? 2 : 1) - (part == rgsvd_plan_s::L_TAIL ? 1 : 0);
    if (first > 0) add_orth(true, first);
    for (int it = 1; it <= qmax; ++it) {
      int p = mixed ? (it < qmax ? PBF : P32) : prec;
      add_tn(p);
      add_orth(false, 1);
      add_nn(p);
      add_orth(true, it == qmax ? 2 : 1);
    }
    // projection B_i = Q_i^T G_i
    add_tn(mixed ? P32 : prec);
    if (part == rgsvd_plan_s::L_TAIL && P->judge) {
      // ||B_i||_F^2 into scal[1]: with ||G_i||_F^2 the residual
      // ||(I - Q_i Q_i^T) G_i||_F^2 = ||G_i||_F^2 - ||B_i||_F^2 of the judge
      std::vector<SumsqJob> j; std::vector<int> tl; std::vector<SumsqFin> f;
      for (auto& s : S) {
        const int nt = (s.l + 15) / 16;
        j.push_back(SumsqJob{WS(ws, s.Wt), s.ldw, s.l, s.n, prec == P64 ? 1 : 0, 16, (double*)WS(ws, s.spart)});
        tl.push_back(nt);
        f.push_back(SumsqFin{(const double*)WS(ws, s.spart), (double*)WS(ws, s.scal) + 1, nt, 0});
      }
      add_sumsq(j, tl, f);
    }
  }
  if (part == rgsvd_plan_s::A_INIT) add_gnorm();
  if (part == rgsvd_plan_s::A_BLOCK) {
    // one block of Algorithm 1 on every active side: Omega columns
    // [l, l + b) of the side's stream, Y = G Omega into Q's rows [l, l + b),
    // then Y projected against the earlier rows and orthonormalised by three
    // truncated CholeskyQR passes over the stacked [Q; Y] (only Y's rows are
    // rewritten), B rows [l, l + b) = Q_new^T G and the block's energy
    // ||B_new||_F^2.
    std::vector<SideLay*> A;
    for (auto& s : S) if (s.active) A.push_back(&s);
    const size_t wsz = 8;
    {
      // the generator writes the block's bcur rows of Omega^T; the product
      // below reads them rounded up to 16, so the rows past bcur are cleared
      std::vector<ZeroJob> zj; std::vector<int> zt;
      for (auto* s : A) {
        const size_t bytes = (size_t)upi(s->bcur, 16) * s->ldw * wsz;
        zj.push_back(ZeroJob{(uint32_t*)WS(ws, s->Ot), (int64_t)(bytes / 4)});
        zt.push_back((int)((bytes / 4 + 4095) / 4096));
      }
      B.add(K_ZEROG, zj, zt).tag = T_ZERO;
    }
    {
      std::vector<GenJob> j; std::vector<int> tl;
      for (auto* s : A) {
        GenJob g{};
        g.Wt = WS(ws, s->Ot); g.ldw = s->ldw; g.seed = s->seed; g.n = s->n; g.col0 = s->lcur;
        g.ncols = s->bcur; g.L = (int)upi(s->bcur, 16); g.stream = s->stream;
        j.push_back(g);
        tl.push_back(((s->n + 255) / 256) * (((s->bcur - 1) >> 2) + 1));
      }
      Stage& st = B.add(K_GEN, j, tl); st.f64 = true; st.tag = T_GEN;
    }
    {
      std::vector<NnJob> j; std::vector<int> tl;
      for (auto* s : A) {
        NnJob x{};
        x.G = s->G; x.Wt = WS(ws, s->Ot); x.Yt = WS(ws, s->Yt) + (size_t)s->lcur * s->ldy * wsz;
        x.ldg = s->ldg; x.ldw = s->ldw; x.ldy = s->ldy; x.m = s->m; x.n = s->n; x.L = (int)upi(s->bcur, 16);
        j.push_back(x);
        tl.push_back((s->m + 15) / 16);
      }
      Stage& st = B.add(K_GW, j, tl);
      st.prec = P64; st.gdt = gt; st.rt = 1; st.ct = ctL; st.tag = T_NN;
    }
    for (int ps = 0; ps < 3; ++ps) {
      std::vector<GramJob> gj; std::vector<int> gtl;
      std::vector<RedJob> rj; std::vector<int> rtl;
      std::vector<CholJob> cj; std::vector<int> ctl;
      std::vector<AbJob> aj; std::vector<int> atl;
      const int nb = P->npadG / 64, nblk = nb * (nb + 1) / 2;
      for (auto* s : A) {
        const int N = s->lcur + s->bcur;
        GramJob g{};
        g.X1 = WS(ws, s->Yt); g.X2 = nullptr; g.out = (double*)WS(ws, s->gpart);
        g.ld1 = s->ldy; g.ld2 = 0; g.r1 = N; g.r2 = 0; g.k0 = 0; g.k1 = s->m;
        g.npad = P->npadG; g.clen = s->gcl_m;
        g.rgs = gram_rgs(N, s->gch_m);
        gj.push_back(g); gtl.push_back(gram_strips(N, g.rgs) * s->gch_m);
        RedJob r{};
        r.in = WS(ws, s->gpart); r.out = WS(ws, s->gram); r.sq = nullptr;
        r.stride = (int64_t)P->npadG * P->npadG; r.count = r.stride;
        r.nparts = s->gch_m; r.rows = P->npadG; r.cols = P->npadG; r.ldo = P->npadG; r.ldi = P->npadG;
        r.nz = N;
        rj.push_back(r); rtl.push_back((int)((r.count + 255) / 256));
        CholJob c{};
        c.gram = (const double*)WS(ws, s->gram); c.sinv = (double*)WS(ws, s->sinv);
        c.info = info_of(s->pair); c.N = N; c.npad = P->npadG; c.flagbit = 0;
        // rows of the block that lie (numerically) in the span of Q and of
        // the block's earlier rows become zero rows of the basis
        c.trunc = 1; c.shift0 = 0.0;
        cj.push_back(c); ctl.push_back(1);
        AbJob a{};
        a.A = (const double*)WS(ws, s->sinv) + (size_t)s->lcur * P->npadG; a.lda = P->npadG;
        a.B = WS(ws, s->Yt); a.ldb = s->ldy;
        a.D = WS(ws, s->Yt) + (size_t)s->lcur * s->ldy * wsz; a.ldd = s->ldy;
        a.rows = s->bcur; a.K = N; a.J = s->m; a.accumulate = 0; a.colscale = nullptr;
        aj.push_back(a);
        atl.push_back((s->m + 64 * 2 - 1) / (64 * 2));
      }
      const int rgs = gram_uniform(gj, gtl);
      Stage& gs = B.add(K_GRAM, gj, gtl); gs.ta = 0; gs.rt = rgs; gs.tag = T_GRAM;
      Stage& r = B.add(K_RED, rj, rtl); r.sym = true; r.ta = 0; r.td = 0; r.tag = T_RED;
      Stage& c = B.add(K_CHOL, cj, ctl); c.tag = T_CHOL;
      Stage& a = B.add(K_AB, aj, atl);
      a.prec = P64; a.ta = 0; a.tb = 0; a.td = 0; a.ct = ctL; a.js = 2; a.tag = T_SX;
    }
    {
      std::vector<AbJob> aj; std::vector<int> atl;
      std::vector<RedJob> rj; std::vector<int> rtl;
      for (auto* s : A) {
        const int lb = (int)upi(s->bcur, 16);
        for (int c = 0; c < s->nchunk; ++c) {
          int r0 = c * s->mchunk;
          int rows = std::min(s->mchunk, s->m - r0);
          AbJob a{};
          a.A = WS(ws, s->Yt) + ((size_t)s->lcur * s->ldy + r0) * wsz; a.lda = s->ldy;
          a.B = (const char*)s->G + (size_t)r0 * s->ldg * (gt == 0 ? 8 : 4); a.ldb = s->ldg;
          a.D = WS(ws, s->part) + (size_t)c * lb * s->ldw * wsz; a.ldd = s->ldw;
          a.rows = lb; a.K = rows; a.J = s->n; a.accumulate = 0; a.colscale = nullptr;
          aj.push_back(a);
          atl.push_back((s->n + 31) / 32);
        }
        RedJob r{};
        r.in = WS(ws, s->part); r.out = WS(ws, s->Wt) + (size_t)s->lcur * s->ldw * wsz; r.sq = nullptr;
        r.stride = (int64_t)lb * s->ldw; r.count = (int64_t)lb * s->n;
        r.nparts = s->nchunk; r.rows = lb; r.cols = s->n; r.ldo = s->ldw; r.ldi = s->ldw;
        rj.push_back(r); rtl.push_back((int)((r.count + 255) / 256));
      }
      Stage& a = B.add(K_GTQ, aj, atl);
      a.prec = P64; a.gdt = gt; a.ct = ctL; a.js = 2; a.tag = T_TN;
      Stage& r = B.add(K_RED, rj, rtl);
      r.sym = false; r.ta = 0; r.td = 0; r.tag = T_RED;
    }
    {
      std::vector<SumsqJob> j; std::vector<int> tl; std::vector<SumsqFin> f;
      for (auto* s : A) {
        const int nt = (s->bcur + 15) / 16;
        j.push_back(SumsqJob{WS(ws, s->Wt) + (size_t)s->lcur * s->ldw * wsz, s->ldw, s->bcur, s->n, 1, 16,
                             (double*)WS(ws, s->spart)});
        tl.push_back(nt);
        f.push_back(SumsqFin{(const double*)WS(ws, s->spart), (double*)WS(ws, s->scal) + 1, nt, 0});
      }
      add_sumsq(j, tl, f);
    }
  }
  if (!tail) {
    if (P->host.size() > P->jobs_cap) return RGSVD_ENOMEM;
    return RGSVD_OK;
  }

  // M = B B^T per pair
  {
    std::vector<GramJob> gj; std::vector<int> gtl;
    std::vector<RedJob> rj; std::vector<int> rtl;
    std::vector<GramJob> dummy;
    for (size_t pi = 0; pi < P->pairs.size(); ++pi) {
      auto& pr = P->pairs[pi];
      auto& s1 = S[2 * pi];
      auto& s2 = S[2 * pi + 1];
      int nb = pr.Npad / 64, nblk = nb * (nb + 1) / 2;
      GramJob g{};
      g.X1 = WS(ws, s1.Wt); g.X2 = WS(ws, s2.Wt); g.out = (double*)WS(ws, pr.mpart);
      g.ld1 = s1.ldw; g.ld2 = s2.ldw; g.r1 = pr.l1; g.r2 = pr.l2; g.k0 = 0; g.k1 = (int)pr.n;
      g.npad = pr.Npad; g.clen = pr.gcl;
      g.rgs = gram_rgs(pr.l1 + pr.l2, pr.gch);
      gj.push_back(g); gtl.push_back(gram_strips(pr.l1 + pr.l2, g.rgs) * pr.gch);
      RedJob r{};
      r.in = WS(ws, pr.mpart); r.out = WS(ws, pr.M); r.sq = nullptr;
      r.stride = (int64_t)pr.Npad * pr.Npad; r.count = r.stride;
      r.nparts = pr.gch; r.rows = pr.Npad; r.cols = pr.Npad; r.ldo = pr.Npad; r.ldi = pr.Npad;
      r.nz = pr.l1 + pr.l2;
      rj.push_back(r); rtl.push_back((int)((r.count + 255) / 256));
    }
    const int rgs = gram_uniform(gj, gtl);
      Stage& gs = B.add(K_GRAM, gj, gtl); gs.ta = wt; gs.rt = rgs; gs.tag = T_MGRAM;
    Stage& r = B.add(K_RED, rj, rtl); r.sym = true; r.tag = T_RED;
  }
  // small step: one launch, or stages around the block Jacobi sweeps on the
  // factors of M (order N) and H (order t) that do not fit k_small's LDS
  {
    // (l1 + l2 is the order the run uses: below the laid-out capacity N
    // after adaptive or learned sizing; t <= l1 + l2)
    auto big = [](int64_t order) { return order * order * 8 > (int64_t)SMALL_LDS_BYTES; };
    auto bjm = [&](const PairLay& pr) { return big(pr.l1 + pr.l2); };
    auto bjh = [&](const PairLay& pr) { return big(pr.t); };
    auto small_job = [&](size_t pi, int stage) {
      auto& pr = P->pairs[pi];
      SmallJob x{};
      x.stage = stage; x.bjh = bjh(pr) ? 1 : 0;
      x.st = (BJState*)WS(ws, pr.bjs);
      x.M = (double*)WS(ws, pr.M); x.ldm = pr.Npad;
      x.l1 = pr.l1; x.l2 = pr.l2; x.t = pr.t; x.maxsweep = 40; x.tol = 1e-15;
      x.work = (double*)WS(ws, pr.work);
      x.sigma = pr.out.sigma_B ? pr.out.sigma_B : (double*)WS(ws, pr.sigma);
      double* ia = (double*)WS(ws, pr.alpha);
      x.alpha = pr.out.alpha ? pr.out.alpha : ia;
      x.beta = pr.out.beta ? pr.out.beta : ia + pr.t;
      x.theta = pr.out.theta ? pr.out.theta : ia + 2 * pr.t;
      x.P1 = pr.out.P1 ? pr.out.P1 : ia + 3 * pr.t;
      x.P2 = pr.out.P2 ? pr.out.P2 : ia + 4 * pr.t;
      x.D = pr.out.D ? pr.out.D : ia + 5 * pr.t;
      x.X1t = (double*)WS(ws, pr.X1t); x.ldx1 = pr.l1;
      x.X2t = (double*)WS(ws, pr.X2t); x.ldx2 = pr.l2;
      x.Rcoef = (double*)WS(ws, pr.Rcoef); x.ldr = pr.N;
      x.info = info_of((int)pi);
      x.ycs = (double*)WS(ws, pr.bjn);   // free once H's block Jacobi is done
      x.hgram = bjh(pr) ? 1 : 0;
      return x;
    };
    auto add_small = [&](int stage) {
      std::vector<SmallJob> sj; std::vector<int> tl;
      for (size_t pi = 0; pi < P->pairs.size(); ++pi) {
        const auto& pr = P->pairs[pi];
        const int st = stage == 1 ? (bjm(pr) ? 1 : 0) : stage;
        if ((stage == 2 && !bjm(pr)) || (stage >= 3 && !bjh(pr))) continue;   // 3, 4, 5: H on the block Jacobi
        sj.push_back(small_job(pi, st)); tl.push_back(1);
      }
      if (!sj.empty()) B.add(K_SMALL, sj, tl).tag = T_SMALL;
      return !sj.empty();
    };
    // sweeps of the block Jacobi: one launch per round (jobs with fewer
    // rounds skip the extra ones); the first sweep starts with a launch of
    // its own (the factor's column norms), later sweeps start inside their
    // first round
    auto add_bj = [&](bool onH) {
      std::vector<BJJob> bj; std::vector<int> tl, one;
      int rmax = 0, wgs = 0;
      for (auto& pr : P->pairs) {
        if (!(onH ? bjh(pr) : bjm(pr))) continue;
        const int N = pr.l1 + pr.l2, t = pr.t;
        const int nr = onH ? t : N;
        const int b = nr <= 256 ? BJ_B : BJ_B / 2;
        const int nblk = 2 * ((nr + 2 * b - 1) / (2 * b));
        double* F = (double*)WS(ws, pr.work) + (size_t)N * t + (size_t)t * t;
        bj.push_back(BJJob{F, (BJState*)WS(ws, pr.bjs), (double*)WS(ws, pr.bjn), 1e-15, nr, nblk});
        tl.push_back(nblk / 2); one.push_back(1);
        rmax = std::max(rmax, nblk - 1);
        wgs += nblk / 2;
      }
      Stage si = B.add(K_BJINIT, bj, one);
      si.tag = T_BJAC;
      P->stages.pop_back();
      // sweeps from sw0 on take one launch each when the sweep's workgroups
      // can all be resident at once (one per CU: the sweep kernel's
      // registers leave room for one workgroup of 8 waves); earlier ones, or
      // all when it does not fit, one launch per round.  An active round
      // costs more behind the barrier than behind a launch, a converged
      // sweep far less in one launch than in nblk - 1.
      int sw0 = BJ_SWEEP_WHOLE;
      if (P->d.options & RGSVD_OPT_JACOBI_SWEEPS) sw0 = 0;
      if ((P->d.options & RGSVD_OPT_JACOBI_ROUNDS) || wgs > P->wave_slots / 4) sw0 = BJ_SWEEPS;
      Stage sr = B.add(K_BJROUND, bj, tl);
      sr.tag = T_BJAC;
      P->stages.pop_back();
      P->stages.push_back(si);
      for (int sw = 0; sw < BJ_SWEEPS; ++sw) {
        if (sw >= sw0) {
          Stage ss = sr;
          ss.kind = K_BJSWEEP; ss.sweep = sw; ss.round = sw0;
          ss.spin = (P->d.options & RGSVD_OPT_JACOBI_NOWAIT) ? 0 : BJ_SPIN;
          P->stages.push_back(ss);
          continue;
        }
        for (int r = 0; r < rmax; ++r) {
          sr.sweep = sw; sr.round = r;
          P->stages.push_back(sr);
        }
      }
    };
    bool any_m = false, any_h = false;
    for (auto& pr : P->pairs) { any_m |= bjm(pr); any_h |= bjh(pr); }
    add_small(1);
    if (any_m) { add_bj(false); add_small(2); }
    if (any_h) {
      // H = L1^T L1 on FP64 MFMA across workgroups: the Gram of the rows of
      // L^T (columns of L, l1 entries each) in up to four chunks of l1, whose
      // partials go to mpart (free since M's reduction), then their
      // fixed-order sum into H (t x t)
      std::vector<GramJob> gj; std::vector<int> gtl;
      std::vector<RedJob> rj; std::vector<int> rtl;
      for (size_t pi = 0; pi < P->pairs.size(); ++pi) {
        auto& pr = P->pairs[pi];
        if (!bjh(pr)) continue;
        const int N = pr.l1 + pr.l2, t = pr.t;
        const int hpad = 64 * ((t + 63) / 64);
        const int64_t room = (int64_t)pr.gch * pr.Npad * pr.Npad / ((int64_t)hpad * hpad);
        const int hch = (int)std::max<int64_t>(1, std::min<int64_t>({4, room, (pr.l1 + 31) / 32}));
        const int hcl = (int)upi((pr.l1 + hch - 1) / hch, 32);
        double* Lg = (double*)WS(ws, pr.work);
        GramJob g{};
        g.X1 = Lg; g.X2 = Lg; g.out = (double*)WS(ws, pr.mpart);
        g.ld1 = N; g.ld2 = N; g.r1 = t; g.r2 = 0; g.k0 = 0; g.k1 = pr.l1;
        g.npad = hpad; g.clen = hcl;
        const int hparts = (pr.l1 + hcl - 1) / hcl;
        g.rgs = gram_rgs(t, hparts);
        gj.push_back(g);
        gtl.push_back(gram_strips(t, g.rgs) * hparts);
        RedJob r{};
        r.in = WS(ws, pr.mpart); r.out = Lg + (size_t)N * t; r.sq = nullptr;
        r.stride = (int64_t)hpad * hpad; r.count = (int64_t)t * t;
        r.nparts = (pr.l1 + hcl - 1) / hcl; r.rows = t; r.cols = t; r.ldo = t; r.ldi = hpad;
        r.nz = t;
        rj.push_back(r); rtl.push_back((int)((r.count + 255) / 256));
      }
      const int rgs = gram_uniform(gj, gtl);
      Stage& gs = B.add(K_GRAM, gj, gtl); gs.ta = 0; gs.rt = rgs; gs.tag = T_SMALL;
      Stage& rs = B.add(K_RED, rj, rtl); rs.sym = true; rs.tag = T_SMALL;
      add_small(5);
      add_bj(true);
      add_small(3);
      // Rcoef = (L Y)^T = diag(ycs) (H's factor)^T L^T on FP64 MFMA over 64-column
      // tiles of L^T (one workgroup held it as 16 waves before), then stage 4
      std::vector<AbJob> aj; std::vector<int> atl;
      int tmax = 1;
      for (size_t pi = 0; pi < P->pairs.size(); ++pi) {
        auto& pr = P->pairs[pi];
        if (!bjh(pr)) continue;
        const int N = pr.l1 + pr.l2, t = pr.t;
        double* Lg = (double*)WS(ws, pr.work);
        AbJob a{};
        a.A = Lg + (size_t)N * t + (size_t)t * t; a.lda = t;   // factor of H, column-major: its transpose
        a.B = Lg; a.ldb = N;                                    // L (N x t, column-major): L^T
        a.D = WS(ws, pr.Rcoef); a.ldd = pr.N;
        a.rows = t; a.K = t; a.J = N; a.accumulate = 0;
        a.colscale = (const double*)WS(ws, pr.bjn);
        aj.push_back(a);
        atl.push_back((N + 63) / 64);
        tmax = std::max(tmax, t);
      }
      Stage& a = B.add(K_AB, aj, atl);
      a.prec = P64; a.ta = 0; a.tb = 0; a.td = 0; a.ct = ct_of(tmax); a.js = 1;
      a.tag = T_SMALL;
      add_small(4);
    }
  }
  // recovery: R (needed for the sign convention), then U, V
  const int ctT = ct_of([&] { int t = 1; for (auto& pr : P->pairs) t = std::max(t, pr.t); return t; }());
  bool anyR = false, anyUV = false;
  for (auto& pr : P->pairs) { anyR |= pr.out.R != nullptr; anyUV |= (pr.out.U || pr.out.V); }
  if (anyR || anyUV) {
    for (int seg = 0; seg < 2; ++seg) {
      std::vector<AbJob> aj; std::vector<int> atl;
      for (size_t pi = 0; pi < P->pairs.size(); ++pi) {
        auto& pr = P->pairs[pi];
        if (!pr.out.R) continue;
        auto& s = S[2 * pi + seg];
        AbJob a{};
        a.A = (const double*)WS(ws, pr.Rcoef) + (seg ? pr.l1 : 0); a.lda = pr.N;
        a.B = WS(ws, s.Wt); a.ldb = s.ldw;
        a.D = pr.out.R; a.ldd = pr.out.ldr;
        a.rows = pr.t; a.K = seg ? pr.l2 : pr.l1; a.J = (int)pr.n; a.accumulate = seg;
        a.colscale = nullptr;
        aj.push_back(a);
        atl.push_back((int)((pr.n + 63) / 64));
      }
      if (!aj.empty()) {
        Stage& a = B.add(K_AB, aj, atl);
        a.prec = (prec == P64) ? P64 : P32; a.ta = 0; a.tb = wt; a.td = 0; a.ct = ctT; a.js = 1;
        a.tag = T_RECOVER;
      }
    }
    std::vector<SignJob> sj; std::vector<int> stl, ctl;
    for (size_t pi = 0; pi < P->pairs.size(); ++pi) {
      auto& pr = P->pairs[pi];
      if (!pr.out.R) continue;
      SignJob x{};
      x.R = pr.out.R; x.ldr = pr.out.ldr; x.sgn = (double*)WS(ws, pr.sgn); x.t = pr.t; x.n = (int)pr.n;
      sj.push_back(x); stl.push_back(pr.t);
      ctl.push_back((int)(((int64_t)pr.t * pr.n + 255) / 256));
    }
    if (!sj.empty()) {
      B.add(K_SIGN, sj, stl).tag = T_SIGN;
      B.add(K_SCALE, sj, ctl).tag = T_SIGN;
    }
    std::vector<AbJob> aj; std::vector<int> atl;
    for (size_t pi = 0; pi < P->pairs.size(); ++pi) {
      auto& pr = P->pairs[pi];
      for (int w = 0; w < 2; ++w) {
        double* dst = w ? pr.out.V : pr.out.U;
        if (!dst) continue;
        auto& s = S[2 * pi + w];
        AbJob a{};
        a.A = WS(ws, w ? pr.X2t : pr.X1t); a.lda = w ? pr.l2 : pr.l1;
        a.B = WS(ws, s.Yt); a.ldb = s.ldy;
        a.D = dst; a.ldd = w ? pr.out.ldv : pr.out.ldu;
        // the widths the run used (adaptive and learned runs end below the
        // side's capacity s.l; X1t, X2t have leading dimension l1, l2)
        a.rows = pr.t; a.K = w ? pr.l2 : pr.l1; a.J = s.m; a.accumulate = 0;
        a.colscale = pr.out.R ? (const double*)WS(ws, pr.sgn) : nullptr;
        aj.push_back(a);
        atl.push_back((s.m + 63) / 64);
      }
    }
    if (!aj.empty()) {
      Stage& a = B.add(K_AB, aj, atl);
      a.prec = (prec == P64) ? P64 : P32; a.ta = 0; a.tb = wt; a.td = 0; a.ct = ctT; a.js = 1;
      a.tag = T_RECOVER;
    }
  }
  if (P->host.size() > P->jobs_cap) return RGSVD_ENOMEM;
  return RGSVD_OK;
}

__global__ void k_copy(const CopyJob* j, const int* pre, int nj) {
  const int jb = find_side(pre, nj, blockIdx.x);
  const CopyJob J = j[jb];
  for (int64_t i = threadIdx.x; i < J.nwords; i += blockDim.x) J.dst[i] = J.src[i];
}

// sum of squares of a row slab per tile (256 threads), in FP64
__global__ __launch_bounds__(256) void k_sumsq(const SumsqJob* j, const int* pre, int nj) {
  const int jb = find_side(pre, nj, blockIdx.x);
  const SumsqJob J = j[jb];
  const int t = blockIdx.x - pre[jb];
  const int r0 = t * J.rpt, r1 = min(J.rows, r0 + J.rpt);
  double acc = 0.0;
  for (int r = r0; r < r1; ++r) {
    if (J.f64) {
      const double* x = (const double*)J.X + (int64_t)r * J.ld;
      for (int c = threadIdx.x; c < J.cols; c += 256) acc += x[c] * x[c];
    } else {
      const float* x = (const float*)J.X + (int64_t)r * J.ld;
      for (int c = threadIdx.x; c < J.cols; c += 256) { const double v = x[c]; acc += v * v; }
    }
  }
  acc = wave_sum(acc);
  __shared__ double ws4[4];
  if ((threadIdx.x & 63) == 0) ws4[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) J.part[t] = ws4[0] + ws4[1] + ws4[2] + ws4[3];
}

__global__ void k_sumfin(const SumsqFin* j, int nj) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nj) return;
  const SumsqFin J = j[i];
  double s = 0.0;
  for (int t = 0; t < J.ntiles; ++t) s += J.part[t];
  J.out[0] = s;
}

// Probe features: eigenvalues of the 16 x 16 probe Gram by two-sided
// Jacobi in one wave, sigma_j = sqrt(lambda_j) in descending order, then
// log10(sigma_j / sigma_1) for j = 2, 4, ..., 16, floored at -8 (the Gram
// resolves sigma_j / sigma_1 down to about sqrt(eps)).  Parallel ordering: each of the 15 rounds of a
// sweep turns 8 disjoint pairs (round-robin over the 16 indices), lanes 0..7
// forming the rotations, then all 64 lanes applying them to the columns and
// then to the rows of the matrix (held in LDS).  Sweeps end when the
// off-diagonal mass is below 1e-32 of the diagonal's, at most 40.
__global__ __launch_bounds__(64) void k_feat(const FeatJob* j, int nj) {
  const FeatJob J = j[blockIdx.x];
  __shared__ double a[16][17];
  __shared__ double cs[8][2];
  __shared__ int pq[8][2];
  const int ln = threadIdx.x;
  for (int e = ln; e < 256; e += 64) {
    const int r = e >> 4, c = e & 15;
    // the reduction filled the upper triangle
    a[r][c] = (c >= r) ? J.gram[(int64_t)r * J.ldg + c] : J.gram[(int64_t)c * J.ldg + r];
  }
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = ln; e < 256; e += 64) {
      const int r = e >> 4, c = e & 15;
      const double v = a[r][c];
      if (r != c) off += v * v; else dia += v * v;
    }
    off = wave_sum(off);
    dia = wave_sum(dia);
    if (!(off > 1e-32 * dia)) break;
    for (int round = 0; round < 15; ++round) {
      if (ln < 8) {
        int u = 0, v;
        if (ln > 0) { u = ln - 1 + round; if (u >= 15) u -= 15; u += 1; }
        v = 15 - ln - 1 + round; if (v >= 15) v -= 15; v += 1;
        const int p = u < v ? u : v, q = u < v ? v : u;
        const double apq = a[p][q];
        double c = 1.0, sn = 0.0;
        if (apq != 0.0) {
          const double th = (a[q][q] - a[p][p]) / (2.0 * apq);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
          c = 1.0 / sqrt(1.0 + t * t);
          sn = t * c;
        }
        cs[ln][0] = c; cs[ln][1] = sn; pq[ln][0] = p; pq[ln][1] = q;
      }
      __syncthreads();
      // columns p, q of every row: 8 pairs x 16 rows, two per lane
      for (int e = ln; e < 128; e += 64) {
        const int pi = e >> 4, r = e & 15;
        const int p = pq[pi][0], q = pq[pi][1];
        const double c = cs[pi][0], sn = cs[pi][1];
        const double x = a[r][p], y = a[r][q];
        a[r][p] = c * x - sn * y; a[r][q] = sn * x + c * y;
      }
      __syncthreads();
      // rows p, q
      for (int e = ln; e < 128; e += 64) {
        const int pi = e >> 4, r = e & 15;
        const int p = pq[pi][0], q = pq[pi][1];
        const double c = cs[pi][0], sn = cs[pi][1];
        const double x = a[p][r], y = a[q][r];
        a[p][r] = c * x - sn * y; a[q][r] = sn * x + c * y;
      }
      __syncthreads();
    }
  }
  if (ln != 0) return;
  double sv[16];
  for (int i = 0; i < 16; ++i) sv[i] = sqrt(fmax(a[i][i], 0.0));
  for (int i = 1; i < 16; ++i)
    for (int k = i; k > 0 && sv[k] > sv[k - 1]; --k) { const double t = sv[k]; sv[k] = sv[k - 1]; sv[k - 1] = t; }
  // s_2, s_4, ..., s_16 over s_1
  for (int i = 0; i < 8; ++i) {
    const double v = sv[2 * i + 1];
    J.out[i] = (float)((sv[0] > 0.0 && v > 0.0) ? fmax(log10(v / sv[0]), -8.0) : -8.0);
  }
}

// Sketch profile: rho_j = R_jj of the Cholesky factor of the widest
// sketch's Gram (the distance of sketch column j from the span of the ones
// before it) is 1 / X_jj of X = R^{-T}; log10(rho_j / rho_1) floored at -8
// at the columns ceil(k/4), ceil(k/2), ceil(3k/4), k, k+4, k+8, k+16, L
// (1-based, clamped to [1, L]).  A dropped or failed pivot (X_jj not a
// positive finite number) reads as the floor.
__global__ __launch_bounds__(64) void k_prof(const ProfJob* j, int nj) {
  const ProfJob J = j[blockIdx.x];
  const int i = threadIdx.x;
  if (i >= 8) return;
  const int k = J.k, L = J.L;
  const int raw[8] = {(k + 3) / 4, (k + 1) / 2, (3 * k + 3) / 4, k, k + 4, k + 8, k + 16, L};
  const int pos = min(max(raw[i], 1), L);
  const double x1 = J.sinv[0], xj = J.sinv[(int64_t)(pos - 1) * (J.ld + 1)];
  const bool ok = isfinite(x1) && isfinite(xj) && x1 > 0.0 && xj > 0.0;
  J.out[i] = (float)(ok ? fmax(log10(x1 / xj), -8.0) : -8.0);
}

int enqueue_list(rgsvd_plan_s* P, void* ws, hipStream_t st, const std::vector<Stage>& list) {
  char* jb = (char*)ws + P->off_jobs;
  if (P->prof) {
    while (P->pev.size() < list.size() + 1) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return RGSVD_EHIP;
      P->pev.push_back(e);
    }
    P->prof_count = (int)list.size();
    P->prof_list = &list;
  }
  int si = 0;
  for (const Stage& s : list) {
    if (P->prof) hipEventRecord(P->pev[si], st);
    ++si;
    const int* pre = (const int*)(jb + s.poff);
    const void* j = jb + s.joff;
    switch (s.kind) {
      case K_ZERO: launch_zero((char*)ws + s.zoff, (int64_t)s.zbytes, st); break;
      case K_ZEROG: launch_zerog((const ZeroJob*)j, pre, s.nj, s.tiles, st); break;
      case K_COPY: hipLaunchKernelGGL(k_copy, dim3(s.tiles), dim3(64), 0, st, (const CopyJob*)j, pre, s.nj); break;
      case K_GEN: launch_gen(s.f64, (const GenJob*)j, pre, s.nj, s.tiles, st); break;
      case K_AB: launch_ab(s.prec, s.ta, s.tb, s.td, s.ct, s.js, (const AbJob*)j, pre, s.nj, s.tiles, st); break;
      case K_GRAM: launch_gram(s.ta, s.rt, (const GramJob*)j, pre, s.nj, s.tiles, st); break;
      case K_RED: launch_reduce(s.ta, s.td, s.sym, (const RedJob*)j, pre, s.nj, s.tiles, st); break;
      case K_CHOL: launch_chol((const CholJob*)j, s.nj, st); break;
      case K_SMALL: launch_small((const SmallJob*)j, s.nj, st); break;
      case K_BJINIT: launch_bjinit((const BJJob*)j, s.nj, s.sweep, st); break;
      case K_BJROUND: launch_bjround((const BJJob*)j, pre, s.nj, s.tiles, s.sweep, s.round, st); break;
      case K_BJSWEEP: launch_bjsweep((const BJJob*)j, pre, s.nj, s.tiles, s.sweep, s.round, s.spin, st); break;
      case K_SIGN: launch_sign((const SignJob*)j, pre, s.nj, s.tiles, st); break;
      case K_SCALE: launch_scale((const SignJob*)j, pre, s.nj, s.tiles, st); break;
      case K_GW: launch_gw(s.prec, s.gdt, s.rt, s.ct, (const NnJob*)j, pre, s.nj, s.tiles, st); break;
      case K_GW4: launch_gw4(s.prec, s.ct, (const NnJob*)j, pre, s.nj, s.tiles, st); break;
      case K_NN: launch_nn(s.split, s.rt, s.ct, (const NnJob*)j, pre, s.nj, s.tiles, st); break;
      case K_GTQ: launch_gtq(s.prec, s.gdt, s.ct, s.js, (const AbJob*)j, pre, s.nj, s.tiles, st); break;
      case K_TN: launch_tn(s.split, s.ct, (const AbJob*)j, pre, s.nj, s.tiles, st); break;
      case K_PACK: launch_pack(j, pre, s.nj, s.tiles, st); break;
      case K_SUMSQ: hipLaunchKernelGGL(k_sumsq, dim3(s.tiles), dim3(256), 0, st, (const SumsqJob*)j, pre, s.nj); break;
      case K_SUMFIN:
        hipLaunchKernelGGL(k_sumfin, dim3((s.nj + 63) / 64), dim3(64), 0, st, (const SumsqFin*)j, s.nj);
        break;
      case K_FEAT: hipLaunchKernelGGL(k_feat, dim3(s.nj), dim3(64), 0, st, (const FeatJob*)j, s.nj); break;
      case K_PROF: hipLaunchKernelGGL(k_prof, dim3(s.nj), dim3(64), 0, st, (const ProfJob*)j, s.nj); break;
      case K_MLP: {
        float* f = (float*)((char*)ws + P->off_feat);
        rgsvd_mlp_forward(P->mlp, f, 1, f + RGSVD_MLP_IN, f + RGSVD_MLP_IN + RGSVD_MLP_OUT, st);
        break;
      }
    }
  }
  if (P->prof) hipEventRecord(P->pev[si], st);
  return hipGetLastError() == hipSuccess ? RGSVD_OK : RGSVD_EHIP;
}

int enqueue(rgsvd_plan_s* P, void* ws, hipStream_t st) { return enqueue_list(P, ws, st, P->stages); }

int upload(rgsvd_plan_s* P, void* ws, hipStream_t st) {
  if (!P->pinned) {
    if (hipHostMalloc(&P->pinned, P->jobs_cap, hipHostMallocDefault) != hipSuccess) return RGSVD_EHIP;
    if (hipEventCreateWithFlags(&P->ev, hipEventDisableTiming) != hipSuccess) return RGSVD_EHIP;
  }
  if (P->ev_pending) { hipEventSynchronize(P->ev); P->ev_pending = false; }
  std::memcpy(P->pinned, P->host.data(), P->host.size());
  if (hipMemcpyAsync((char*)ws + P->off_jobs, P->pinned, P->host.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    return RGSVD_EHIP;
  if (hipEventRecord(P->ev, st) != hipSuccess) return RGSVD_EHIP;
  P->ev_pending = true;
  return RGSVD_OK;
}

// Single-pair runs replay their launch sequence as a HIP graph once a
// binding has run eagerly (a few hundred short launches, mostly the block
// Jacobi rounds, otherwise wait on the host's launch rate).  The graph holds
// the bound pointers, so every rebuild of the job tables drops it.
void drop_graph(rgsvd_plan_s* P) {
  if (P->gexec) { hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
}

int enqueue_list(rgsvd_plan_s* P, void* ws, hipStream_t st, const std::vector<Stage>& list);

// Capture a stage list into an executable graph (on a stream of its own).
int capture_list(rgsvd_plan_s* P, void* ws, const std::vector<Stage>& list, hipGraphExec_t* exec) {
  *exec = nullptr;
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return RGSVD_EHIP;
  hipGraph_t g = nullptr;
  const bool prof = P->prof;
  P->prof = false;
  bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    const int rc = enqueue_list(P, ws, cs, list);
    ok = hipStreamEndCapture(cs, &g) == hipSuccess && g && rc == RGSVD_OK;
  }
  P->prof = prof;
  if (ok) ok = hipGraphInstantiate(exec, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) hipGraphDestroy(g);
  hipStreamDestroy(cs);
  if (!ok) { *exec = nullptr; return RGSVD_EHIP; }
  return RGSVD_OK;
}

int capture_graph(rgsvd_plan_s* P, void* ws) {
  drop_graph(P);
  return capture_list(P, ws, P->stages, &P->gexec);
}

// Drop the learned run's graphs (they hold the bound pointers).
void drop_learned_graphs(rgsvd_plan_s* P) {
  if (P->lhead_exec) { hipGraphExecDestroy(P->lhead_exec); P->lhead_exec = nullptr; }
  for (auto& e : P->ltail_exec)
    if (e) { hipGraphExecDestroy(e); e = nullptr; }
  P->ltail_exec.clear();
}

// Launch a stage list: eagerly when profiling (events between stages),
// otherwise as its graph, captured on first use.
int run_list(rgsvd_plan_s* P, void* ws, hipStream_t st, const std::vector<Stage>& list, hipGraphExec_t* exec) {
  if (P->prof) return enqueue_list(P, ws, st, list);
  if (!*exec) {
    const int rc = capture_list(P, ws, list, exec);
    if (rc) return rc;
  }
  return hipGraphLaunch(*exec, st) == hipSuccess ? RGSVD_OK : RGSVD_EHIP;
}

// capacity of an adaptive basis: lmax (0: no cap) clamped to min(rows, n)
// and to the largest supported width
int64_t adaptive_cap(int64_t lmax, int64_t rows, int64_t n) {
  int64_t c = std::min<int64_t>(rows, n);
  if (lmax > 0) c = std::min(c, lmax);
  return std::min<int64_t>(c, MAXL - 32);
}

int check_desc(const rgsvd_desc* d) {
  if (!d) return RGSVD_EINVAL;
  if (d->m < 1 || d->p < 1 || d->n < 1 || d->k < 1 || d->oversample < 0 || d->power_iters < 0)
    return RGSVD_EINVAL;
  if (d->in_dtype != RGSVD_F64 && d->in_dtype != RGSVD_F32) return RGSVD_EINVAL;
  if (d->precision < RGSVD_PREC_FP64 || d->precision > RGSVD_PREC_MIXED) return RGSVD_EINVAL;
  if (d->mode != RGSVD_TRUNCATED && d->mode != RGSVD_FULL) return RGSVD_EINVAL;
  if ((d->options & ~(RGSVD_OPT_JACOBI_ROUNDS | RGSVD_OPT_JACOBI_SWEEPS | RGSVD_OPT_JACOBI_NOWAIT)) ||
      (d->options & RGSVD_OPT_JACOBI_ROUNDS && d->options & RGSVD_OPT_JACOBI_SWEEPS))
    return RGSVD_EINVAL;
  if (d->m > (1 << 30) || d->p > (1 << 30) || d->n > (1 << 30)) return RGSVD_EINVAL;
  const int64_t l = d->k + d->oversample;
  // Theorem "projector": k + p <= min(m, n) (and <= min(p, n) for G2)
  if (d->sizing == RGSVD_SIZE_FIXED) {
    if (l > std::min(d->m, d->n) || l > std::min(d->p, d->n)) return RGSVD_EINVAL;
    if (l > MAXL - 32) return RGSVD_EUNSUPPORTED;
    if (d->mode == RGSVD_FULL && 2 * l < d->n) return RGSVD_ENOTGMP;
    if (d->mode == RGSVD_TRUNCATED && d->k > l) return RGSVD_EINVAL;
    if (2 * l > SMALL_MAXN) return RGSVD_EUNSUPPORTED;
  } else if (d->sizing == RGSVD_SIZE_ADAPTIVE) {
    // Algorithm 1 with an absolute tolerance; FP64 arithmetic.  Full mode
    // needs capacities that can reach l1 + l2 >= n (checked again on the
    // widths the run reaches)
    if (!(d->tol > 0.0) || !std::isfinite(d->tol) || d->block < 0 || d->lmax < 0) return RGSVD_EINVAL;
    if (d->precision != RGSVD_PREC_FP64) return RGSVD_EUNSUPPORTED;
    if (d->mode == RGSVD_FULL &&
        adaptive_cap(d->lmax, d->m, d->n) + adaptive_cap(d->lmax, d->p, d->n) < d->n)
      return RGSVD_ENOTGMP;
    if (d->k > adaptive_cap(d->lmax, d->m, d->n) || d->k > adaptive_cap(d->lmax, d->p, d->n))
      return RGSVD_EINVAL;
  } else if (d->sizing == RGSVD_SIZE_LEARNED) {
    // the network picks l on a grid up to min(2k, capacity) and q <= 3; tol
    // > 0 turns on the residual judge (fallback: Algorithm 1 with b = block)
    if (d->lmax < 0 || d->block < 0 || !(d->tol >= 0.0) || !std::isfinite(d->tol)) return RGSVD_EINVAL;
    if (d->mode != RGSVD_TRUNCATED) return RGSVD_EUNSUPPORTED;
    if (d->k > adaptive_cap(d->lmax, d->m, d->n) || d->k > adaptive_cap(d->lmax, d->p, d->n))
      return RGSVD_EINVAL;
  } else {
    return RGSVD_EUNSUPPORTED;
  }
  return RGSVD_OK;
}

// single-wave workgroups resident at once: compute units x 4 SIMDs x 1 wave
int device_wave_slots() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  return cus * 4;
}

PairLay pair_from(const rgsvd_desc* d) {
  PairLay pr;
  pr.m = d->m; pr.p = d->p; pr.n = d->n; pr.k = d->k; pr.o = d->oversample; pr.q = d->power_iters;
  pr.seed = d->seed;
  pr.l1 = pr.l2 = (int)(d->k + d->oversample);
  if (d->sizing == RGSVD_SIZE_ADAPTIVE || d->sizing == RGSVD_SIZE_LEARNED) {
    pr.l1 = (int)adaptive_cap(d->lmax, d->m, d->n);
    pr.l2 = (int)adaptive_cap(d->lmax, d->p, d->n);
    pr.q = 0;
  }
  pr.l1cap = pr.l1; pr.l2cap = pr.l2;
  pr.t = (d->mode == RGSVD_FULL) ? (int)d->n : (int)d->k;
  return pr;
}

}  // namespace

// Algorithm 1 on both matrices, block by block, then the shared tail.  The
// stopping test needs the residual on the host, so the stream is
// synchronised once after the norms and once per block.
int run_adaptive(rgsvd_plan_s* P, void* ws, hipStream_t st) {
  PairLay& pr = P->pairs[0];
  std::vector<SideLay>& S = P->sides;
  if (!P->hscal && hipHostMalloc((void**)&P->hscal, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return RGSVD_EHIP;
  pr.l1 = pr.l1cap; pr.l2 = pr.l2cap;
  for (auto& s : S) { s.lcur = 0; s.bcur = 0; s.active = true; }
  auto stage_list = [&](rgsvd_plan_s::Part part) {
    P->part = part;
    int rc = build(P, ws);
    P->part = rgsvd_plan_s::FIXED;
    if (!rc) rc = upload(P, ws, st);
    if (!rc) rc = enqueue(P, ws, st);
    return rc;
  };
  auto fetch = [&](int word) {   // scal[word] of every side into hscal[side]
    for (size_t i = 0; i < S.size(); ++i)
      if (hipMemcpyAsync(P->hscal + i, (char*)ws + S[i].scal + 8 * word, 8, hipMemcpyDeviceToHost, st) != hipSuccess)
        return RGSVD_EHIP;
    return hipStreamSynchronize(st) == hipSuccess ? RGSVD_OK : RGSVD_EHIP;
  };
  int rc = stage_list(rgsvd_plan_s::A_INIT);
  if (!rc) rc = fetch(0);
  if (rc) return rc;
  std::vector<double> g2(S.size()), esum(S.size(), 0.0);
  for (size_t i = 0; i < S.size(); ++i) g2[i] = P->hscal[i];
  const double eps = P->d.tol;
  for (;;) {
    bool any = false;
    for (auto& s : S) {
      if (!s.active) continue;
      s.bcur = std::min(P->block, s.cap - s.lcur);
      if (s.bcur <= 0) s.active = false; else any = true;
    }
    if (!any) break;
    rc = stage_list(rgsvd_plan_s::A_BLOCK);
    if (!rc) rc = fetch(1);
    if (rc) return rc;
    for (size_t i = 0; i < S.size(); ++i) {
      auto& s = S[i];
      if (!s.active) continue;
      esum[i] += P->hscal[i];
      s.lcur += s.bcur;
      const double res = std::sqrt(std::max(0.0, g2[i] - esum[i]));
      if (!(res >= eps) || s.lcur >= s.cap) s.active = false;
    }
  }
  pr.l1 = S[0].lcur;
  pr.l2 = S[1].lcur;
  // full mode (t = n) is Algorithm 2 on a GMP: the bases must span n together
  if (pr.t > pr.l1 + pr.l2) return RGSVD_ENOTGMP;
  return stage_list(rgsvd_plan_s::TAIL);
}

// Every side at sketch width l (its buffers hold the capacity).
void set_width(rgsvd_plan_s* P, int l, int q) {
  for (auto& s : P->sides) { s.l = l; s.L = (int)upi(l, 16); }
  for (auto& pr : P->pairs) { pr.l1 = pr.l2 = l; pr.q = q; }
}

// The sketch widths a sizing network can pick: {k+4, k+8, k+16, k+32, 2k},
// capped at cap, ascending and distinct.
std::vector<int> l_grid(int k, int cap) {
  std::vector<int> grid;
  for (int v : {k + 4, k + 8, k + 16, k + 32, 2 * k}) { v = std::min(v, cap); if (v >= k) grid.push_back(v); }
  std::sort(grid.begin(), grid.end());
  grid.erase(std::unique(grid.begin(), grid.end()), grid.end());
  return grid;
}

// The features alone (rgsvd_probe_features): the head of a learned run
// (the sketch at the widest grid width of the plan's k and capacity, the
// probe, the first CholeskyQR pass and the profile) in the plan's sketch
// precision, so the features equal those a learned run computes from its
// own sketch.
int run_probe(rgsvd_plan_s* P, void* ws, hipStream_t st) {
  const int keep = P->lmaxw;
  const PairLay& pr = P->pairs[0];
  P->lmaxw = l_grid((int)pr.k, std::min(pr.l1cap, pr.l2cap)).back();
  set_width(P, P->lmaxw, 0);
  P->part = rgsvd_plan_s::L_HEAD;
  P->probe_only = true;
  int rc = build(P, ws);
  P->probe_only = false;
  P->part = rgsvd_plan_s::FIXED;
  P->lmaxw = keep;
  P->lbound = false;
  drop_learned_graphs(P);
  if (!rc) rc = upload(P, ws, st);
  if (!rc) rc = enqueue(P, ws, st);
  return rc;
}

// Sketch sizes from the network output (log2(l / k), q): the smallest l of
// the grid at or above k 2^y0, and q rounded with a bias of 0.4 towards more
// passes (q >= 1 from y1 = 0.1 on), clamped to [0, 3].
void decide_sizes(double y0, double y1, int k, int cap, int* l, int* q) {
  const std::vector<int> grid = l_grid(k, cap);
  const double want = k * std::exp2(std::isfinite(y0) ? std::min(y0, 8.0) : 8.0);
  *l = grid.back();
  for (int v : grid) if (v >= want) { *l = v; break; }
  const double qq = std::floor((std::isfinite(y1) ? y1 : 3.0) + 0.9);
  *q = (int)std::min(3.0, std::max(0.0, qq));
}

// Job tables of a learned run for the bound pointers: the head (sketch at
// the widest grid width, probe features, network) and one tail per grid
// point, serialised once into the job area.
int bind_learned(rgsvd_plan_s* P, void* ws, hipStream_t st) {
  PairLay& pr = P->pairs[0];
  const int cap = std::min(pr.l1cap, pr.l2cap);
  const std::vector<int> grid = l_grid((int)pr.k, cap);
  P->lmaxw = grid.back();
  drop_learned_graphs(P);
  P->host.clear();
  P->append = true;
  P->ltails.clear();
  P->lgrid.clear();
  set_width(P, P->lmaxw, 0);
  P->part = rgsvd_plan_s::L_HEAD;
  int rc = build(P, ws);
  P->lhead = std::move(P->stages);
  for (int q = 0; q <= 3 && !rc; ++q)
    for (int l : grid) {
      set_width(P, l, q);
      P->part = rgsvd_plan_s::L_TAIL;
      rc = build(P, ws);
      if (rc) break;
      P->ltails.push_back(std::move(P->stages));
      P->lgrid.push_back({l, q});
    }
  P->append = false;
  P->part = rgsvd_plan_s::FIXED;
  P->stages.clear();
  P->ltail_exec.assign(P->ltails.size(), nullptr);
  if (!rc) rc = upload(P, ws, st);
  P->lbound = !rc;
  return rc;
}

// Learned sizing: the head (sketch, features, network), one read of the
// network's two outputs, then the tail at the chosen (l, q).  With a
// tolerance (the judge), the residual ||G_i||_F^2 - ||Q_i^T G_i||_F^2 of
// either side above tol^2 sends the pair to Algorithm 1 (adaptive blocks,
// FP64) instead, and FLAG_FALLBACK marks it.
int run_learned(rgsvd_plan_s* P, const void* G1, int64_t ld1, const void* G2, int64_t ld2, void* ws,
                hipStream_t st, const rgsvd_out* out) {
  PairLay& pr = P->pairs[0];
  if (!P->mlp) return RGSVD_ENOMODEL;
  if (!P->hscal && hipHostMalloc((void**)&P->hscal, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return RGSVD_EHIP;
  const bool same = P->lbound && P->lastG1 == G1 && P->lastG2 == G2 && P->lastws == ws && P->lastld1 == ld1 &&
                    P->lastld2 == ld2 && out_eq(P->lastout, *out);
  if (!same) {
    pr.out = *out;
    P->sides[0].G = G1; P->sides[0].ldg = ld1;
    P->sides[1].G = G2; P->sides[1].ldg = ld2;
    const int rc = bind_learned(P, ws, st);
    if (rc) return rc;
    P->lastG1 = G1; P->lastG2 = G2; P->lastws = ws; P->lastld1 = ld1; P->lastld2 = ld2;
    P->lastout = *out;
  }
  int rc = run_list(P, ws, st, P->lhead, &P->lhead_exec);
  if (rc) return rc;
  const float* yd = (const float*)((char*)ws + P->off_feat) + RGSVD_MLP_IN;
  if (hipMemcpyAsync(P->hscal, yd, 2 * sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return RGSVD_EHIP;
  const float* y = (const float*)P->hscal;
  int l = 0, q = 0;
  decide_sizes(y[0], y[1], (int)pr.k, std::min(pr.l1cap, pr.l2cap), &l, &q);
  size_t idx = 0;
  while (idx < P->lgrid.size() && P->lgrid[idx] != std::make_pair(l, q)) ++idx;
  if (idx == P->lgrid.size()) return RGSVD_EHIP;
  set_width(P, l, q);
  rc = run_list(P, ws, st, P->ltails[idx], &P->ltail_exec[idx]);
  if (rc || !P->judge) return rc;
  // the judge: a posteriori residual of each side's basis
  std::vector<SideLay>& S = P->sides;
  for (size_t i = 0; i < S.size(); ++i)
    if (hipMemcpyAsync(P->hscal + 2 * i, (char*)ws + S[i].scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st) !=
        hipSuccess)
      return RGSVD_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return RGSVD_EHIP;
  bool accept = true;
  for (size_t i = 0; i < S.size(); ++i) {
    const double res = std::sqrt(std::max(0.0, P->hscal[2 * i] - P->hscal[2 * i + 1]));
    accept &= !(res >= P->d.tol);
  }
  if (accept) return RGSVD_OK;
  // fallback: Algorithm 1 at the plan's capacity, in FP64 (the plan's
  // working buffers are laid out for it)
  const int prec = P->prec;
  P->prec = P64;
  P->adaptive = true;
  P->extra_flags = RGSVD_FLAG_FALLBACK;
  for (auto& s : S) { s.l = s.cap; s.L = (int)upi(s.cap, 16) + 16; }
  rc = run_adaptive(P, ws, st);
  P->prec = prec;
  P->adaptive = false;
  P->extra_flags = 0;
  P->lbound = false;   // the adaptive steps replaced the job tables
  drop_learned_graphs(P);
  return rc;
}

// --------------------------------------------------------------- autotune --
// Tile shapes of the streaming kernels, chosen by timing: rows per tile of
// the G W kernel (1 or 4), columns per lane of the G^T Q kernel (2 or 4) and
// the number of row chunks its reduction is split over (the heuristic count,
// half of it or twice it).  Every valid combination runs `reps` times after
// one warm-up with HIP events around the enqueued stages; the fastest total
// wins and is remembered for the plan's shape key.
struct TuneChoice { int rt, js, chunk, wg; float ms; };
std::map<std::string, TuneChoice>& tune_cache() {
  static std::map<std::string, TuneChoice> c;
  return c;
}

std::string shape_key(const rgsvd_plan_s* P) {
  std::string k = std::to_string(P->prec) + "/" + std::to_string(P->gdt) + "/" + std::to_string(P->batched);
  for (auto& pr : P->pairs)
    k += ":" + std::to_string(pr.m) + "," + std::to_string(pr.p) + "," + std::to_string(pr.n) + "," +
         std::to_string(pr.l1) + "," + std::to_string(pr.l2) + "," + std::to_string(pr.q);
  return k;
}

void apply_cached_tune(rgsvd_plan_s* P) {
  auto it = tune_cache().find(shape_key(P));
  if (it == tune_cache().end()) return;
  P->tune_rt = it->second.rt; P->tune_js = it->second.js; P->tune_chunk = it->second.chunk;
  P->tune_wg = it->second.wg;
}

int autotune_plan(rgsvd_plan_s* P, void* ws, hipStream_t st, int reps, int32_t* choice, float* best_ms) {
  const bool streamy = P->prec != P64 && P->gdt == RGSVD_F32;
  const bool mixed = P->prec == PBF && P->gdt == RGSVD_F32;
  // the mixed path's 8-wave kernels (k_nn, k_tn) have none of the three
  // knobs; its per-wave kernels have all of them
  std::vector<int> rts = streamy ? std::vector<int>{1, 4} : std::vector<int>{1};
  std::vector<int> jss = streamy ? std::vector<int>{2, 4} : std::vector<int>{2};
  std::vector<int> wgs = mixed ? std::vector<int>{1, 2} : std::vector<int>{0};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return RGSVD_EHIP;
  TuneChoice best{0, 0, 0, 0, 1e30f};
  int rc = RGSVD_OK;
  for (int wg : wgs)
  for (int rt : rts)
    for (int js : jss)
      for (int ch = 0; ch < 3 && !rc; ++ch) {
        if (wg == 1 && (rt != rts[0] || js != jss[0] || ch != 0)) continue;
        P->tune_rt = rt; P->tune_js = js; P->tune_chunk = ch; P->tune_wg = wg;
        P->part = rgsvd_plan_s::FIXED;
        rc = build(P, ws);
        if (!rc) rc = upload(P, ws, st);
        if (!rc) rc = enqueue(P, ws, st);   // warm-up
        if (rc) break;
        hipEventRecord(e0, st);
        for (int r = 0; r < reps && !rc; ++r) rc = enqueue(P, ws, st);
        hipEventRecord(e1, st);
        if (rc || hipEventSynchronize(e1) != hipSuccess) { rc = rc ? rc : RGSVD_EHIP; break; }
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        ms /= (float)std::max(1, reps);
        if (ms < best.ms) best = TuneChoice{rt, js, ch, wg, ms};
      }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  P->tune_rt = best.rt; P->tune_js = best.js; P->tune_chunk = best.chunk; P->tune_wg = best.wg;
  tune_cache()[shape_key(P)] = best;
  P->bound = false;
  if (!P->batched) drop_graph(P);
  if (choice) { choice[0] = best.rt; choice[1] = best.js; choice[2] = best.chunk; choice[3] = best.wg; }
  if (best_ms) *best_ms = best.ms;
  return RGSVD_OK;
}

static uint64_t next_plan_id() {
  static std::atomic<uint64_t> n{0};
  return ++n;
}

// ------------------------------------------------- allocation-free runs --
// Workspace of rgsvd_run_static: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never passes the array's name
// to a kernel or copy (on the host it is only a stand-in symbol): the first
// static run on a device looks up that device's address once, with the
// device current, and every later use goes through it.
static __device__ __align__(256) unsigned char scratch[RGSVD_STATIC_SCRATCH_BYTES];

struct StaticSlot {
  void* ptr = nullptr;   // device address of `scratch` on this GPU
  uint64_t owner = 0;    // plan whose job tables the scratch holds
  uint64_t gen = 0;      // and their generation
};
constexpr int MAX_DEVICES = 64;
static std::mutex& static_mutex() {
  static std::mutex m;
  return m;
}
static StaticSlot g_static[MAX_DEVICES];

// ===================================================================== ABI ==
extern "C" {

const char* rgsvd_strerror(int code) {
  switch (code) {
    case RGSVD_OK: return "ok";
    case RGSVD_EINVAL: return "invalid argument";
    case RGSVD_ENOTGMP: return "full mode needs l1 + l2 >= n";
    case RGSVD_EHIP: return "HIP runtime error";
    case RGSVD_ENOMEM: return "host allocation failed";
    case RGSVD_EWORKSPACE: return "workspace null or not 256-byte aligned";
    case RGSVD_ENOMODEL: return "learned sizing needs a sizing model";
    case RGSVD_EUNSUPPORTED: return "unsupported combination";
    case RGSVD_ETOOBIG: return "workspace larger than the static scratch (RGSVD_STATIC_SCRATCH_BYTES)";
    default: return "unknown error";
  }
}

int rgsvd_plan(const rgsvd_desc* desc, rgsvd_plan_t* plan, size_t* workspace_bytes) {
  if (!plan || !workspace_bytes) return RGSVD_EINVAL;
  *plan = nullptr;
  int rc = check_desc(desc);
  if (rc) return rc;
  rgsvd_plan_s* P = new (std::nothrow) rgsvd_plan_s();
  if (!P) return RGSVD_ENOMEM;
  P->d = *desc;
  P->id = next_plan_id();
  P->prec = desc->precision == RGSVD_PREC_FP64 ? P64 : (desc->precision == RGSVD_PREC_FP32 ? P32 : PBF);
  P->gdt = desc->in_dtype;
  P->mode = desc->mode;
  P->adaptive = desc->sizing == RGSVD_SIZE_ADAPTIVE;
  P->learned = desc->sizing == RGSVD_SIZE_LEARNED;
  P->judge = P->learned && desc->tol > 0.0;
  P->block = desc->block > 0 ? (int)desc->block : 100;
  P->pairs.push_back(pair_from(desc));
  P->wave_slots = device_wave_slots();
  rc = layout(P);
  if (rc) { delete P; return rc; }
  apply_cached_tune(P);
  *plan = P;
  *workspace_bytes = P->ws;
  return RGSVD_OK;
}

int rgsvd_plan_sizes(rgsvd_plan_t P, int64_t* t, int64_t* l1, int64_t* l2) {
  if (!P || P->pairs.empty()) return RGSVD_EINVAL;
  if (t) *t = P->pairs[0].t;
  if (l1) *l1 = P->pairs[0].l1cap;
  if (l2) *l2 = P->pairs[0].l2cap;
  return RGSVD_OK;
}

int rgsvd_run(rgsvd_plan_t P, const void* G1, int64_t ld1, const void* G2, int64_t ld2,
              void* workspace, void* stream, const rgsvd_out* out) {
  if (!P || P->batched || !G1 || !G2 || !out) return RGSVD_EINVAL;
  if (!workspace || ((uintptr_t)workspace & (ALIGN - 1))) return RGSVD_EWORKSPACE;
  PairLay& pr = P->pairs[0];
  if (ld1 < pr.n || ld2 < pr.n) return RGSVD_EINVAL;
  if ((out->U && out->ldu < pr.m) || (out->V && out->ldv < pr.p) || (out->R && out->ldr < pr.n))
    return RGSVD_EINVAL;
  if (P->d.sizing == RGSVD_SIZE_LEARNED && !P->mlp) return RGSVD_ENOMODEL;
  hipStream_t st = (hipStream_t)stream;
  if (P->adaptive) {
    pr.out = *out;
    P->sides[0].G = G1; P->sides[0].ldg = ld1;
    P->sides[1].G = G2; P->sides[1].ldg = ld2;
    P->bound = false;
    return run_adaptive(P, workspace, st);
  }
  if (P->learned) return run_learned(P, G1, ld1, G2, ld2, workspace, st, out);
  bool same = P->bound && P->lastG1 == G1 && P->lastG2 == G2 && P->lastws == workspace &&
              P->lastld1 == ld1 && P->lastld2 == ld2 && out_eq(P->lastout, *out);
  if (!same) {
    drop_graph(P);
    pr.out = *out;
    P->sides[0].G = G1; P->sides[0].ldg = ld1;
    P->sides[1].G = G2; P->sides[1].ldg = ld2;
    int rc = build(P, workspace);
    if (rc) return rc;
    rc = upload(P, workspace, st);
    if (rc) return rc;
    P->bound = true;
    P->lastG1 = G1; P->lastG2 = G2; P->lastws = workspace; P->lastld1 = ld1; P->lastld2 = ld2;
    P->lastout = *out;
    return enqueue(P, workspace, st);   // the first run of a binding is eager
  }
  // per-stage profiling needs its events between launches: eager
  if (P->prof) return enqueue(P, workspace, st);
  if (!P->gexec) {
    const int rc = capture_graph(P, workspace);
    if (rc) return rc;
  }
  return hipGraphLaunch(P->gexec, st) == hipSuccess ? RGSVD_OK : RGSVD_EHIP;
}

int rgsvd_run_static(rgsvd_plan_t P, const void* G1, int64_t ld1, const void* G2, int64_t ld2, void* stream,
                     const rgsvd_out* out) {
  if (!P || P->batched || !G1 || !G2 || !out) return RGSVD_EINVAL;
  if (P->adaptive || P->learned) return RGSVD_EUNSUPPORTED;
  if (P->ws > RGSVD_STATIC_SCRATCH_BYTES) return RGSVD_ETOOBIG;
  PairLay& pr = P->pairs[0];
  if (ld1 < pr.n || ld2 < pr.n) return RGSVD_EINVAL;
  if ((out->U && out->ldu < pr.m) || (out->V && out->ldv < pr.p) || (out->R && out->ldr < pr.n))
    return RGSVD_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return RGSVD_EHIP;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(static_mutex());
  StaticSlot& sl = g_static[dev];
  if (!sl.ptr) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return RGSVD_EHIP;
    sl.ptr = ptr;
  }
  void* ws = sl.ptr;
  const bool same = P->bound && P->lastG1 == G1 && P->lastG2 == G2 && P->lastws == ws && P->lastld1 == ld1 &&
                    P->lastld2 == ld2 && out_eq(P->lastout, *out);
  if (!same) {
    drop_graph(P);
    pr.out = *out;
    P->sides[0].G = G1; P->sides[0].ldg = ld1;
    P->sides[1].G = G2; P->sides[1].ldg = ld2;
    P->bound = false;
    const int rc = build(P, ws);
    if (rc) return rc;
    ++P->gen;
    P->bound = true;
    P->lastG1 = G1; P->lastG2 = G2; P->lastws = ws; P->lastld1 = ld1; P->lastld2 = ld2;
    P->lastout = *out;
  }
  // the job tables live in the scratch too: copied in again whenever another
  // plan or another binding of this one ran there last (ordered on `stream`)
  if (sl.owner != P->id || sl.gen != P->gen) {
    if (hipMemcpyAsync((char*)ws + P->off_jobs, P->host.data(), P->host.size(), hipMemcpyHostToDevice, st) !=
        hipSuccess)
      return RGSVD_EHIP;
    sl.owner = P->id;
    sl.gen = P->gen;
  }
  const bool prof = P->prof;
  P->prof = false;   // per-stage events are not created here
  const int rc = enqueue(P, ws, st);
  P->prof = prof;
  return rc;
}

void rgsvd_destroy(rgsvd_plan_t P) {
  if (!P) return;
  if (P->ev_pending) hipEventSynchronize(P->ev);
  if (P->ev) hipEventDestroy(P->ev);
  if (P->pinned) hipHostFree(P->pinned);
  if (P->gexec) hipGraphExecDestroy(P->gexec);
  drop_learned_graphs(P);
  if (P->mlp) hipFree(P->mlp);
  if (P->hscal) hipHostFree(P->hscal);
  for (auto e : P->pev) hipEventDestroy(e);
  delete P;
}

int rgsvd_profile(rgsvd_plan_t P, int32_t enable) {
  if (!P || P->batched) return RGSVD_EINVAL;
  P->prof = enable != 0;
  return RGSVD_OK;
}

int rgsvd_profile_read(rgsvd_plan_t P, int32_t max, float* ms, int32_t* tag, int32_t* count) {
  if (!P || !count || max < 0) return RGSVD_EINVAL;
  int n = P->prof ? P->prof_count : 0;
  *count = n;
  for (int i = 0; i < n && i < max; ++i) {
    float t = 0.0f;
    if (hipEventSynchronize(P->pev[i + 1]) != hipSuccess) return RGSVD_EHIP;
    if (hipEventElapsedTime(&t, P->pev[i], P->pev[i + 1]) != hipSuccess) return RGSVD_EHIP;
    if (ms) ms[i] = t;
    if (tag) tag[i] = (*P->prof_list)[i].tag;
  }
  return RGSVD_OK;
}

// ------------------------------------------------------------- batched --
int rgsvd_batch_plan(const rgsvd_desc* shapes, int32_t npairs, rgsvd_plan_t* plan,
                     size_t* workspace_bytes) {
  if (!shapes || npairs < 1 || !plan || !workspace_bytes) return RGSVD_EINVAL;
  *plan = nullptr;
  for (int i = 0; i < npairs; ++i) {
    int rc = check_desc(&shapes[i]);
    if (rc) return rc;
    if (shapes[i].in_dtype != shapes[0].in_dtype || shapes[i].precision != shapes[0].precision ||
        shapes[i].mode != shapes[0].mode || shapes[i].options != shapes[0].options)
      return RGSVD_EINVAL;
    // every grouped launch serves all pairs at one step of the subspace
    // iteration, so the pairs of a batch share the power count
    if (shapes[i].power_iters != shapes[0].power_iters || shapes[i].sizing != RGSVD_SIZE_FIXED)
      return RGSVD_EUNSUPPORTED;
  }
  rgsvd_plan_s* P = new (std::nothrow) rgsvd_plan_s();
  if (!P) return RGSVD_ENOMEM;
  P->d = shapes[0];
  P->id = next_plan_id();
  P->batched = true;
  P->prec = shapes[0].precision == RGSVD_PREC_FP64 ? P64 : (shapes[0].precision == RGSVD_PREC_FP32 ? P32 : PBF);
  P->gdt = shapes[0].in_dtype;
  P->mode = shapes[0].mode;
  for (int i = 0; i < npairs; ++i) P->pairs.push_back(pair_from(&shapes[i]));
  P->wave_slots = device_wave_slots();
  int rc = layout(P);
  if (rc) { delete P; return rc; }
  apply_cached_tune(P);
  *plan = P;
  *workspace_bytes = P->ws;
  return RGSVD_OK;
}

int rgsvd_batch_bind(rgsvd_plan_t P, const rgsvd_pair_io* io, void* workspace, void* stream) {
  if (!P || !P->batched || !io) return RGSVD_EINVAL;
  if (!workspace || ((uintptr_t)workspace & (ALIGN - 1))) return RGSVD_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  for (size_t i = 0; i < P->pairs.size(); ++i) {
    auto& pr = P->pairs[i];
    if (!io[i].G1 || !io[i].G2 || io[i].ld1 < pr.n || io[i].ld2 < pr.n) return RGSVD_EINVAL;
    pr.out = io[i].out;
    P->sides[2 * i].G = io[i].G1; P->sides[2 * i].ldg = io[i].ld1;
    P->sides[2 * i + 1].G = io[i].G2; P->sides[2 * i + 1].ldg = io[i].ld2;
  }
  int rc = build(P, workspace);
  if (rc) return rc;
  rc = upload(P, workspace, st);
  if (rc) return rc;
  if (hipStreamSynchronize(st) != hipSuccess) return RGSVD_EHIP;
  if (P->gexec) { hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
  // capture the whole enqueue sequence once
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return RGSVD_EHIP;
  hipGraph_t g = nullptr;
  bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    enqueue(P, workspace, cs);
    ok = hipStreamEndCapture(cs, &g) == hipSuccess && g;
  }
  if (ok) ok = hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) hipGraphDestroy(g);
  hipStreamDestroy(cs);
  if (!ok) { P->gexec = nullptr; return RGSVD_EHIP; }
  P->bws = workspace;
  P->bound = true;
  return RGSVD_OK;
}

int rgsvd_batch_run(rgsvd_plan_t P, void* stream) {
  if (!P || !P->batched || !P->bound || !P->gexec) return RGSVD_EINVAL;
  return hipGraphLaunch(P->gexec, (hipStream_t)stream) == hipSuccess ? RGSVD_OK : RGSVD_EHIP;
}

int rgsvd_autotune(rgsvd_plan_t P, const void* G1, int64_t ld1, const void* G2, int64_t ld2, void* workspace,
                   void* stream, const rgsvd_out* out, int32_t reps, int32_t* choice, float* best_ms) {
  if (!P || P->batched || P->adaptive || P->learned || !G1 || !G2 || !out || reps < 1) return RGSVD_EINVAL;
  if (!workspace || ((uintptr_t)workspace & (ALIGN - 1))) return RGSVD_EWORKSPACE;
  PairLay& pr = P->pairs[0];
  if (ld1 < pr.n || ld2 < pr.n) return RGSVD_EINVAL;
  pr.out = *out;
  P->sides[0].G = G1; P->sides[0].ldg = ld1;
  P->sides[1].G = G2; P->sides[1].ldg = ld2;
  const bool prof = P->prof;
  P->prof = false;
  int rc = autotune_plan(P, workspace, (hipStream_t)stream, reps, choice, best_ms);
  P->prof = prof;
  return rc;
}

int rgsvd_batch_autotune(rgsvd_plan_t P, const rgsvd_pair_io* io, void* workspace, void* stream, int32_t reps,
                         int32_t* choice, float* best_ms) {
  if (!P || !P->batched || !io || reps < 1) return RGSVD_EINVAL;
  if (!workspace || ((uintptr_t)workspace & (ALIGN - 1))) return RGSVD_EWORKSPACE;
  for (size_t i = 0; i < P->pairs.size(); ++i) {
    auto& pr = P->pairs[i];
    if (!io[i].G1 || !io[i].G2 || io[i].ld1 < pr.n || io[i].ld2 < pr.n) return RGSVD_EINVAL;
    pr.out = io[i].out;
    P->sides[2 * i].G = io[i].G1; P->sides[2 * i].ldg = io[i].ld1;
    P->sides[2 * i + 1].G = io[i].G2; P->sides[2 * i + 1].ldg = io[i].ld2;
  }
  if (P->gexec) { hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
  P->bound = false;
  return autotune_plan(P, workspace, (hipStream_t)stream, reps, choice, best_ms);
}

}  // extern "C"

// ------------------------------------------------- sizing-model entry points --
extern "C" int rgsvd_set_sizing_model(rgsvd_plan_t P, const float* params, void* stream) {
  if (!P || !params) return RGSVD_EINVAL;
  if (!P->mlp && hipMalloc((void**)&P->mlp, RGSVD_MLP_PARAMS * sizeof(float)) != hipSuccess)
    return RGSVD_EHIP;
  return hipMemcpyAsync(P->mlp, params, RGSVD_MLP_PARAMS * sizeof(float), hipMemcpyDeviceToDevice,
                        (hipStream_t)stream) == hipSuccess ? RGSVD_OK : RGSVD_EHIP;
}

extern "C" int rgsvd_probe_features(rgsvd_plan_t P, const void* G1, int64_t ld1, const void* G2, int64_t ld2,
                                    void* workspace, float* feat, void* stream) {
  if (!P || P->batched || !G1 || !G2 || !feat) return RGSVD_EINVAL;
  if (!workspace || ((uintptr_t)workspace & (ALIGN - 1))) return RGSVD_EWORKSPACE;
  PairLay& pr = P->pairs[0];
  if (ld1 < pr.n || ld2 < pr.n) return RGSVD_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  P->sides[0].G = G1; P->sides[0].ldg = ld1;
  P->sides[1].G = G2; P->sides[1].ldg = ld2;
  P->bound = false;
  // restore the plan's own widths afterwards (the probe runs at the widest grid width)
  std::vector<std::pair<int, int>> keep;
  for (auto& s : P->sides) keep.push_back({s.l, s.L});
  const int l1 = pr.l1, l2 = pr.l2, q = pr.q;
  int rc = run_probe(P, workspace, st);
  for (size_t i = 0; i < P->sides.size(); ++i) { P->sides[i].l = keep[i].first; P->sides[i].L = keep[i].second; }
  pr.l1 = l1; pr.l2 = l2; pr.q = q;
  if (rc) return rc;
  return hipMemcpyAsync(feat, (char*)workspace + P->off_feat, RGSVD_MLP_IN * sizeof(float),
                        hipMemcpyDeviceToDevice, st) == hipSuccess ? RGSVD_OK : RGSVD_EHIP;
}
