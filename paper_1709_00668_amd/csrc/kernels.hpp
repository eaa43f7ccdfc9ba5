// Host-side launchers of the gfx950 kernels of the SamBaTen update.
// Every launcher enqueues on `stream` and returns the launch status.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace sbt {

// Timing of one kernel by events the launch itself records at the kernel's
// start and end (hipExtLaunchKernel), instead of events around its dispatch:
// when set, the next timed_launch on this host thread takes the pair.
struct LaunchTiming {
  hipEvent_t start = nullptr, stop = nullptr;
};
inline LaunchTiming& launch_timing() {
  static thread_local LaunchTiming lt;
  return lt;
}
template <typename... KArgs, typename... Args>
inline void timed_launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t sh,
                         hipStream_t s, Args&&... args) {
  LaunchTiming& lt = launch_timing();
  if (lt.start) {
    hipEvent_t a = lt.start, b = lt.stop;
    lt.start = lt.stop = nullptr;
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)sh, s, a, b, 0u,
                          std::forward<Args>(args)...);
  } else {
    kernel<<<grid, block, sh, s>>>(std::forward<Args>(args)...);
  }
}

// Summary / MTTKRP element types.
enum Prec : int { kF64 = 0, kF32 = 1, kBF16 = 2 };

inline size_t prec_bytes(int p) { return p == kF64 ? 8 : (p == kF32 ? 4 : 2); }
// Accumulation type of the MTTKRP kernels: double for FP64, float otherwise.
inline size_t acc_bytes(int p) { return p == kF64 ? 8 : 4; }

constexpr int kMaxRank = 32;

// Shapes of the r summaries of one update (identical for every repetition)
// and the per-repetition strides of every workspace array (in elements).
struct RepSet {
  int n1, n2, n3;   // summary dims; n3 = K' = sampled old slices + new slices
  int R;
  int rep0, nrep;   // repetitions [rep0, rep0 + nrep) of this launch
  int64_t sZ;       // summary elements
  int64_t sA, sB, sC;  // factor rows * R
  int64_t sW;       // W workspace per repetition: R * n1*n2 (acc type)
  int nsplit;       // partial sums per row of W (1: pass W writes complete rows)
  int64_t sM;       // max rows * R (double)
  int64_t sG;       // R*R
  int64_t ldz = 0;  // stride between the slices c of a dense summary (0: n1*n2)
};
// elements from one slice of a dense summary to the next
__host__ __device__ inline int64_t zslice(const RepSet& rs) {
  return rs.ldz > 0 ? rs.ldz : (int64_t)rs.n1 * rs.n2;
}

// ---- importance (Eq. 1), integer form ------------------------------------
hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);
// max over x*x of a dense block, as the bit pattern of a non-negative double
hipError_t launch_maxsq_dense(int prec, const void* X, int64_t n, uint64_t* out_bits,
                              hipStream_t s);
hipError_t launch_maxsq_coo(const float* v, int64_t n, uint64_t* out_bits, hipStream_t s);
// per-index sums of q(x) = floor(x*x*scale) of a dense I x J x K block;
// w3 receives one entry per slice.  err |= 1 on a non-finite x or q > qmax.
hipError_t launch_moi_dense(int prec, const void* Y, int64_t I, int64_t J, int64_t K,
                            double scale, uint64_t qmax, uint64_t* w1, uint64_t* w2,
                            uint64_t* w3, uint32_t* err, hipStream_t s);
// Same for COO entries (k relative to w3).  err |= 2 on a coordinate outside
// I x J x K.
hipError_t launch_moi_coo(const int32_t* ii, const int32_t* jj, const int32_t* kk,
                          const float* v, int64_t nnz, int64_t I, int64_t J, int64_t K,
                          double scale, uint64_t qmax, uint64_t* w1, uint64_t* w2,
                          uint64_t* w3, uint32_t* err, hipStream_t s);

// ---- weighted sampling without replacement --------------------------------
struct SampleArgs {
  const uint64_t* w[3];  // importance per mode
  int64_t N[3];          // population per mode
  int n[3];              // sample size per mode
  int64_t key_off[3];    // offsets into the per-repetition key scratch
  int64_t key_stride;    // per repetition
  int64_t idx_off[3];    // offsets into the per-repetition index output
  int64_t idx_stride;
  uint64_t seed;
  uint32_t tensor_id;
  uint32_t t;
  int nrep;
  int nmodes;  // modes in this launch (0 = 3)
  int mode0;   // index of the first one (its Philox tag carries mode0 + 1)
};
hipError_t launch_sample(const SampleArgs& a, uint64_t* keys, int32_t* idx, hipStream_t s);

// ---- summaries -----------------------------------------------------------
// Z[rep](a,b,c) = X(Is[a], Js[b], K'[c]) with K'[c] = Ks[c] for c < n3old and
// Kold + c - n3old after; converted to the summary precision.  Slices c < c0
// are left as they are (a kept summary's old part).
hipError_t launch_gather_dense(int store_prec, int sum_prec, const void* X, int64_t I,
                               int64_t J, const int32_t* idx, int64_t idx_stride,
                               int64_t offJ, int64_t offK, int n3old, int64_t Kold, int c0,
                               const RepSet& rs, void* Z, hipStream_t s);

// ---- BF16 summaries on the matrix cores ----------------------------------
// Zk[rep][c][a + ld1 b] (slice stride sk) and Zc[rep][a + n1 b][c] (row
// stride ldc); padding entries are zero.
struct MfmaLayout {
  int ld1;      // n1 rounded up to 8
  int64_t sk;   // Zk slice stride: ld1 * n2 rounded up to 32
  int ldc;      // Zc row stride: largest K' rounded up to 32
  int64_t sZk;  // per repetition
  int64_t sZc;
};
MfmaLayout mfma_layout(int n1, int n2, int kpmax);
// whether the MFMA kernels' LDS staging fits these summary shapes
bool mfma_supported(int n1, int n2, int R);
// number of K ranges of the mode-3 kernel
int mfma_mode3_splits(const RepSet& rs, const MfmaLayout& L);
// Launch shapes of the gather and of the two matrix-core passes that give
// identical results: `choice` in [0, SBT_TUNE_SHAPES) picks one (0 is the
// default shape; the tuner in autotune.h picks the others by their time).
// both BF16 layouts; the groups of 8 slices from the one holding c0 on are
// gathered (earlier slices are a kept summary's old part)
hipError_t launch_gather_mfma(int store_prec, const void* X, int64_t I, int64_t J,
                              const int32_t* idx, int64_t idx_stride, int64_t offJ, int64_t offK,
                              int n3old, int64_t Kold, int c0, const RepSet& rs,
                              const MfmaLayout& L, uint16_t* Zk, uint16_t* Zc, hipStream_t s,
                              int choice = 0);
// one repetition from a column-major BF16 tensor (no sampling)
hipError_t launch_relayout_bf16(const uint16_t* Z, const RepSet& rs, const MfmaLayout& L,
                                uint16_t* Zk, uint16_t* Zc, hipStream_t s);
// staged operands of the two passes, floats per repetition (the `ops` buffer
// holds this times the repetitions)
size_t mfma_operand_floats(const MfmaLayout& L, int n2, int R);
// W(e, f) = sum_c Zc(e, c) C~(c, f), C~ = C diag(invlamC) (invlamC may be null)
hipError_t launch_pw_mfma(const RepSet& rs, const MfmaLayout& L, const uint16_t* Zc,
                          const double* Cf, const double* invlamC, float* W, float* ops,
                          hipStream_t s, int choice = 0);
// partial rows of Zk (B~ kr A~) over nsplit K ranges into P[rep][split] (stride sP,
// row stride 16 or 32)
hipError_t launch_p3_mfma(const RepSet& rs, const MfmaLayout& L, int nsplit, const uint16_t* Zk,
                          const double* Af, const double* invlamA, const double* Bf,
                          const double* invlamB, float* P, int64_t sP, float* ops,
                          hipStream_t s, int choice = 0);
// U(c, :) = (sum_split P) V^-1 [/ lam_div]
// gpart: also the Gram matrix of each block's rows, as launch_cw writes them
hipError_t launch_mode3_finish(const RepSet& rs, int nsplit, const float* P, int64_t sP,
                               const double* Vinv, const double* lam_div, double* U, int64_t sU,
                               hipStream_t s, double* gpart = nullptr, int64_t sGpart = 0);

// ---- CP-ALS on the summaries --------------------------------------------
// B', C' <- U[0,1) from Philox counters (row, col0 + col, tag(stream, mode, rep), t)
hipError_t launch_als_init(const RepSet& rs, uint64_t seed, uint32_t tensor_id, uint32_t stream,
                           uint32_t t, double* Bp, double* Cp, hipStream_t s, uint32_t col0 = 0);
// warm start: B' <- Bw, C' rows < n3keep <- Cw, the other C' rows as launch_als_init
hipError_t launch_als_warm(const RepSet& rs, uint64_t seed, uint32_t tensor_id, uint32_t stream,
                           uint32_t t, const double* Bw, const double* Cw, int n3keep,
                           double* Bp, double* Cp, hipStream_t s);
// G = U^T U for rows x R factors of each repetition
hipError_t launch_gram(const RepSet& rs, const double* U, int64_t sU, int rows, double* G,
                       hipStream_t s);
// W(ab, f) = sum_c Z(ab, c) Cf(c, f)
hipError_t launch_p1(int prec, const RepSet& rs, const void* Z, const double* Cf, void* W,
                     hipStream_t s);
// mode 0 from W: M(a, f) = sum_b W(a,b,f) Bf(b,f)
hipError_t launch_cw1(int prec, const RepSet& rs, const void* W, const double* Bf, double* M,
                      hipStream_t s);
// mode 1 from W: M(b, f) = sum_a W(a,b,f) Af(a,f)
hipError_t launch_cw2(int prec, const RepSet& rs, const void* W, const double* Af, double* M,
                      hipStream_t s);
// mode 2: M(c, f) = sum_ab Z(a,b,c) Af(a,f) Bf(b,f)
hipError_t launch_p2(int prec, const RepSet& rs, const void* Z, const double* Af,
                     const double* Bf, double* M, hipStream_t s);
// U = M (G1 .* G2)^-1 (Cholesky, pseudo-inverse fallback).
//  normalize=1: lam_out = column norms, U normalised, Gout = U^T U.
//  normalize=0: U(:, f) /= lam_div[f] (0 when lam_div[f] == 0).
hipError_t launch_solve(const RepSet& rs, int rows, const double* M, const double* G1,
                        int64_t sG1, const double* G2, int64_t sG2, double* U, int64_t sU,
                        double* Gout,
                        double* lam_out, const double* lam_div, int normalize,
                        uint32_t* pinv_count, hipStream_t s);

// ---- batched CP-ALS (latency-oriented) ----------------------------------
// Outputs of one mode update: raw rows U of the new factor, its normalised
// Gram matrix, 1/lambda, optionally lambda, and V_next^-1 = (Gx .* Gy)^-1 for
// the next step, all per repetition.
struct AlsTail {
  const double* Gin = nullptr;  // raw Gram of U per repetition (stride sG), or computed here
  double* U;
  int64_t sU;
  int rows;
  double* Gout;
  double* invlam_out;
  double* lam_out;
  const double* Gx;
  const double* Gy;
  double* Vinv_out;
  int64_t sG;
  uint32_t* pinv_count;
};
// V^-1 = (Gx .* Gy)^-1 per repetition (pseudo-inverse when singular)
hipError_t launch_inverse(const RepSet& rs, const double* Gx, int64_t sGx, const double* Gy,
                          int64_t sGy, double* Vinv, uint32_t* pinv_count, hipStream_t s);
// raw factors -> unit columns (multiplies by the stored 1/lambda of A, B, C)
hipError_t launch_normalize(const RepSet& rs, double* Ap, double* Bp, double* Cp,
                            const double* invlam, hipStream_t s);
// W[rep][split][ab][f] = sum_{c in split} Z(ab, c) C(c, f) / lambda_C(f)
hipError_t launch_pw(int prec, const RepSet& rs, const void* Z, const double* Cf,
                     const double* invlamC, void* W, hipStream_t s);
// mode 0: A rows = (W x_b B~) V^-1; mode 1: B rows = (W x_a A~) V^-1.
// before: the tail of the step that produced F (its rows must fit the tail's
// staging, Gin unused), folded into this launch: every block computes it,
// the first block of each repetition stores its outputs, and this step's
// V^-1 and F's 1/lambda come from it instead of Vinv and invlamF.
// gpart: also the Gram matrix of each block's rows, [rep][block][R x R] at
// stride sGpart per repetition (gram_parts(rows) blocks), for launch_tail_parts.
hipError_t launch_cw(int prec, const RepSet& rs, int mode, const void* W, const double* F,
                     const double* invlamF, const double* Vinv, double* U, int64_t sU,
                     hipStream_t s, const AlsTail* before = nullptr, double* gpart = nullptr,
                     int64_t sGpart = 0);
// whether launch_p3 can stage both factors of an n1 x n2 slice in LDS
bool p3_fits(int prec, int n1, int n2, int R);
// C rows = (Z_(3) (B~ kr A~)) V^-1, or with row_solve those rows / lam_div
hipError_t launch_p3(int prec, const RepSet& rs, bool row_solve, const void* Z, const double* Af,
                     const double* invlamA, const double* Bf, const double* invlamB,
                     const double* Vinv, const double* lam_div, double* U, int64_t sU,
                     hipStream_t s);
// tail of a mode update: Gram, lambda, normalised Gram, next V^-1
hipError_t launch_tail(const RepSet& rs, const AlsTail& t, hipStream_t s);
// the same with the Gram matrix summed from the partial ones of the kernel
// that wrote the rows (nparts of them, in block order, t.Gin null)
hipError_t launch_tail_parts(const RepSet& rs, const AlsTail& t, const double* parts,
                             int64_t sParts, int nparts, hipStream_t s);
// row blocks of the kernels that write partial Gram matrices
int gram_parts(int rows);

// ---- cross products X^T Y (R x R) over many rows ------------------------------
struct XJob {
  const double* X;    // rows of X: X + rep * sX + (ix ? ix[rep * six + i] : i) * R
  int64_t sX;
  const int32_t* ix;
  int64_t six;
  const double* Y;    // likewise
  int64_t sY;
  const int32_t* iy;
  int64_t siy;
  int rows;
};
constexpr int kXJobs = 9;
struct XProd {
  XJob job[kXJobs];
  int njobs, R, rep0, nrep;
  int nblk;       // chunks the partial buffer holds per (rep, job)
  double* part;   // [rep][job][nblk][R * R]
  double* out;    // [rep][job][R * R], or with sOut > 0 at (rep * njobs + job) * sOut
  int64_t sOut;
};
// chunks needed for `max_rows` rows
int xprod_blocks(int max_rows);
hipError_t launch_xprod(XProd xp, hipStream_t s);
// whether the tail stages all rows at once (else pass the Gram matrix in)
bool tail_rows_fit(int rows, int R);

// ---- matching, row solve inputs ------------------------------------------
struct MatchArgs {
  const double* xo;             // per repetition: A(Is)^T A', B(Js)^T B', C(Ks)^T C',
                                // A(Is)^T A(Is), B(Js)^T B(Js), C(Ks)^T C(Ks), A'^T A',
                                // B'^T B', C'^T C' (anchor rows), each R x R
  double* scl;                  // per repetition 2R: column scales of At, Bt
  const double *A, *B, *C;      // current model (row-major)
  const int32_t* idx;           // per-repetition sampled indices
  int64_t idx_stride, offJ, offK;
  int n3old;                    // anchor rows of C' (sampled old slices)
  const double *Ap, *Bp, *Cp;   // summary factors
  double *At, *Bt;              // matched, rescaled
  double* Gt;                   // (At^T At) .* (Bt^T Bt)
  int32_t *pi, *valid;
  const int32_t* rnew;          // per repetition rank of the summary factors, or null (R)
};
hipError_t launch_match(const RepSet& rs, const MatchArgs& m, hipStream_t s);

// ---- commit ----------------------------------------------------------------
struct CommitArgs {
  const uint32_t* err;
  double *A, *B, *C;  // model, updated in place
  int64_t I, J, Kold, Knew;
  int R, nrep, n1, n2, n3old, Kp;
  const int32_t* idx;
  int64_t idx_stride, offJ, offK;
  const double *At, *Bt, *Ct;
  int64_t sA, sB, sC;
  const int32_t* valid;
  uint64_t *w1, *w2, *w3;            // state importance
  const uint64_t *dw1, *dw2, *dw3;   // batch importance
};
hipError_t launch_commit(const CommitArgs& c, hipStream_t s);
// per repetition and component, the matched summary weight in the current
// model's units (-1: none), from the matching's cross products xo
hipError_t launch_lambda_hat(const RepSet& rs, const double* xo, const double* lamp,
                             const int32_t* pi, const int32_t* valid, double* lhat,
                             hipStream_t s);
// lambda <- (lambda + mean of the valid lhat) / 2, unless *err
hipError_t launch_lambda_avg(const uint32_t* err, double* lam, const double* lhat, int nrep,
                             int R, hipStream_t s);

// ---- sparse (COO) path ------------------------------------------------------
struct CooScratch {   // ingest of one batch
  uint32_t *key_in, *key_out;
  int32_t *val_in, *val_out;
  uint32_t* hist;
  void* tmp;
  size_t tmp_bytes;
  int64_t cap;        // entries
};
struct CooSummary {   // the r summaries of one update, concatenated by repetition
  int32_t *a, *b, *c;       // sorted by c
  float* v;
  int32_t *a_x, *a_y;       // sorted by a: (b, c)
  float* a_v;
  int32_t *b_x, *b_y;       // sorted by b: (a, c)
  float* b_v;
  int64_t *offA, *offB, *offC;  // per repetition row offsets (absolute)
  int64_t sOffA, sOffB, sOffC;
  int64_t* rep_off;         // device copy of rep_off_h (nrep + 1)
  int64_t rep_off_h[65];
  uint32_t *key_a, *key_b, *key_out;
  int32_t *val, *perm;
  void* tmp;
  size_t tmp_bytes;
  int64_t cap;              // entries allocated
};
// Work units of the sparse MTTKRP of one mode: every row's entry segment cut
// into pieces of at most kCooUnit entries (heavy rows of skewed data are
// spread over many wavefronts; the pieces are added back in order).
constexpr int kCooUnit = 512;
struct CooUnits {
  uint32_t* cnt;     // units per (rep, row)                     [nrep * rows]
  int64_t* uoff;     // exclusive scan of cnt, total at the end   [nrep * rows + 1]
  int32_t* urow;     // rep * rows + row of each unit
  int64_t* ustart;   // first entry of each unit
  int32_t* ulen;     // entries of each unit
  int64_t cap;       // units allocated
};
hipError_t coo_sort_tmp_bytes(int64_t n, size_t* bytes);
int64_t coo_scan_blocks(int64_t nnz);
// append a batch (k batch-relative) sorted by k at store position `base`;
// koff[Kold .. Kold + Knew] receives the slice offsets
hipError_t launch_coo_ingest(const int32_t* bi, const int32_t* bj, const int32_t* bk,
                             const float* bv, int64_t n, int64_t Knew, int64_t Kold,
                             int32_t* si, int32_t* sj, int32_t* sk, float* sv, int64_t base,
                             int64_t* koff, CooScratch& w, hipStream_t s);
hipError_t launch_coo_maps(const int32_t* idx, int64_t idx_stride, int64_t offJ, int64_t offK,
                           int n1, int n2, int n3old, int nrep, int32_t* posI, int32_t* posJ,
                           int32_t* posK, int64_t I, int64_t J, int64_t Kcap, uint64_t* bitI,
                           uint64_t* bitJ, uint64_t* bitK, hipStream_t s);
// per block and repetition counts of kept entries, and per repetition
// exclusive scans bbase[rep][0..nblk] (relative to the repetition's start)
// per repetition q: cnt[q] entries of (a, b, c, v) from src[q] to dst[q] of
// (oa, ob, oc, ov); max_cnt >= every cnt[q] (device arrays src, cnt, dst)
hipError_t launch_summary_move(const int32_t* a, const int32_t* b, const int32_t* c,
                               const float* v, const int64_t* src, const int64_t* cnt,
                               const int64_t* dst, int nrep, int64_t max_cnt, int32_t* oa,
                               int32_t* ob, int32_t* oc, float* ov, hipStream_t s);
hipError_t launch_coo_count(const int32_t* si, const int32_t* sj, const int32_t* sk, int64_t nnz,
                            const uint64_t* bitI, const uint64_t* bitJ, const uint64_t* bitK,
                            int64_t Kold, int nrep, uint32_t* bcount, int64_t* bbase,
                            hipStream_t s);
hipError_t launch_coo_emit(const int32_t* si, const int32_t* sj, const int32_t* sk,
                           const float* sv, int64_t nnz, const uint64_t* bitI,
                           const uint64_t* bitJ, const uint64_t* bitK, int64_t Kold, int n3old,
                           int nrep, const int32_t* posI, const int32_t* posJ,
                           const int32_t* posK, int64_t I, int64_t J, int64_t Kcap,
                           const int64_t* bbase, CooSummary& z, hipStream_t s);
// the copies sorted by a and by b, and the row offsets of all three modes
// (n1, n2, n3 rows per repetition) from the sorted keys
hipError_t launch_coo_sorts(CooSummary& z, int nrep, int64_t total, int n1, int n2, int n3,
                            hipStream_t s);
// one COO tensor (a, b, c, v) of extents n1 x n2 x n3 as the single summary
// of z: entries ordered by c (stable), the a- and b-ordered copies and the
// row offsets of all three modes (z.rep_off must hold {0, nnz} on the device)
hipError_t launch_coo_single_summary(const int32_t* a, const int32_t* b, const int32_t* c,
                                     const float* v, int64_t nnz, int n1, int n2, int n3,
                                     CooSummary& z, hipStream_t s);
// rows of mode `mode` (0: A from B, C; 1: B from A, C; 2: C from A, B):
// U = (COO MTTKRP) V^-1, or divided by lam_div (row solve)
// unit table of one mode from the row offsets of the summaries
hipError_t launch_coo_units_build(const RepSet& rs, int mode, const CooSummary& z, CooUnits& u,
                                  hipStream_t s);
// FP32 scaled copies of factor rows for the sparse MTTKRP: Xf[rep][row][RX],
// RX = 16 for R <= 16, else 32 (zero beyond R)
hipError_t launch_coo_prep(const RepSet& rs, int rows, const double* X, int64_t sX,
                           const double* invlam, float* Xf, hipStream_t s);
// partial rows (RP floats per unit) of the MTTKRP of one mode from the FP32
// copies of the two other factors (rowsX, rowsY rows per repetition); the
// launch covers u.cap units, the ones past the device-side total return.
// avg_row_nnz (summary entries per row, a host estimate) picks the lanes per
// unit; the result does not depend on it beyond the order of additions.
hipError_t launch_coo_units(const RepSet& rs, int mode, const CooSummary& z, const CooUnits& u,
                            const float* Xf, int rowsX, const float* Yf, int rowsY, float* part,
                            double avg_row_nnz, hipStream_t s);
// rows U(row, :) = (sum of the row's unit partials, in order) V^-1 [/ lam_div]
hipError_t launch_coo_units_finish(const RepSet& rs, int mode, const CooUnits& u,
                                   const float* part, const double* Vinv, const double* lam_div,
                                   double* U, int64_t sU, hipStream_t s);
hipError_t launch_coo_rows(const RepSet& rs, int mode, const CooSummary& z, const double* X,
                           int64_t sX, const double* invlamX, const double* Y, int64_t sY,
                           const double* invlamY, const double* Vinv, const double* lam_div,
                           double* U, int64_t sU, hipStream_t s);

// ---- fit -------------------------------------------------------------------
// M3(k, f) = sum_ij X(i,j,k) A(i,f) B(j,f) and nrm(k) = sum_ij X(i,j,k)^2, FP64
hipError_t launch_fit_slices(int prec, const void* X, int64_t I, int64_t J, int64_t K, int R,
                             const double* A, const double* B, double* M3, double* nrm,
                             hipStream_t s);
hipError_t launch_fit_coo(const int32_t* ii, const int32_t* jj, const float* v,
                          const int64_t* koff, int64_t K, int R, const double* A,
                          const double* B, double* M3, double* nrm, hipStream_t s);
// fit = 1 - sqrt(max(0, sum nrm - 2 <X,Xhat> + ||Xhat||^2)) / sqrt(sum nrm)
// G3: the Gram matrices of A, B, C (3 x R x R)
// ---- GetRank (Sec. 3.2) --------------------------------------------------------
// projected core P = Z x1 A^T x2 B^T x3 C^T of every repetition (rank rs.R)
// from W = Z x3 C^T in the [f][e] layout of launch_p1; P is [rep][a][b][c]
hipError_t launch_core(int prec, const RepSet& rs, const void* W, const double* Ap,
                       const double* Bp, double* P, int64_t sP, hipStream_t s);
// the same projected core from COO summaries (entries stored slice by slice
// of the third mode, slice z of repetition rep at offC[rep sOffC + z ..
// + 1]): the slice partials go to Wz ([rep][z][a][b], stride sWz >= n3 R^2)
hipError_t launch_core_coo(const RepSet& rs, const int32_t* za, const int32_t* zb,
                           const float* zv, const int64_t* offC, int64_t sOffC, const double* Ap,
                           const double* Bp, const double* Cp, double* Wz, int64_t sWz,
                           double* P, int64_t sP, hipStream_t s);
// core consistency (percent) of every repetition from P, the inverse Grams
// (GA^-1, GB^-1, GC^-1 at Gi, Gi + sGi, Gi + 2 sGi) and the run's lambda
hipError_t launch_corcondia(const RepSet& rs, const double* P, double* X1, double* X2, int64_t sP,
                            const double* Gi, int64_t sGi, const double* lam, double* cc,
                            hipStream_t s);
// keep run j at rank rs.R where it is the best at that rank and the rank
// counts; kept factors padded to Rf columns, rnew = rs.R
hipError_t launch_rank_select(const RepSet& rs, int Rf, int runs, int j, bool force, double tau,
                              const double* cc, double* bestcc, double* cctab, int32_t* rnew,
                              const double* Ap, const double* Bp, const double* Cp,
                              const double* lamp, double* Ak, double* Bk, double* Ck,
                              double* lamk, hipStream_t s);
// factor match score of two models from their nine cross products
// (A1^T A2, B1^T B2, C1^T C2, the Grams of model 1, the Grams of model 2)
hipError_t launch_fms(const double* xo, const double* lam1, const double* lam2, int R,
                      double* out, hipStream_t s);
hipError_t launch_fit_final(const double* G3, const double* C, const double* lam,
                            const double* M3, const double* nrm, int64_t K, int R, double* fit,
                            hipStream_t s);

// ---- initial model ordering ----------------------------------------------
// Order components by lam descending (ties: lower index first) in place.
hipError_t launch_sort_components(double* A, double* B, double* C, double* lam, int64_t I,
                                  int64_t J, int64_t K, int R, hipStream_t s);

// ---- tensors of order N (last mode growing) ----------------------------------
constexpr int kMaxOrder = 8;

// importance of a dense block of order N (extents D, column-major): w[m][i]
// += sum of q(x) over the entries whose m-th index is i, for every mode.
struct MoiNd {
  const void* X;
  int N;
  int64_t D[kMaxOrder];
  uint64_t* w[kMaxOrder];
  double scale;
  uint64_t qmax;
  uint32_t* err;
};
hipError_t launch_moi_nd(int prec, const MoiNd& a, hipStream_t s);

// Rows of several factors per repetition (row-major, R columns):
// U[m] + rep * sU[m], n[m] rows.
struct NdFactors {
  double* U[kMaxOrder];
  int64_t sU[kMaxOrder];
  int n[kMaxOrder];
};

// Khatri-Rao rows of modes [lo, hi): out(p, f) = prod_l U_l(a_l, f) with
// p = a_lo + n_lo * (a_lo+1 + ...), per repetition at out + rep * sOut.
hipError_t launch_krp_nd(const NdFactors& F, int lo, int hi, int R, int rep0, int nrep,
                         double* out, int64_t sOut, hipStream_t s);
// out = Hadamard product of the Gram matrices G + m * sMode (per repetition
// stride sG) of the modes in `mask` (all ones when empty).
hipError_t launch_hadamard_nd(const double* G, int64_t sMode, int64_t sG, uint32_t mask, int N,
                              int R, int rep0, int nrep, double* out, hipStream_t s);
// U[0,1) initial factors of modes 1..N-1: entry (row, col) of mode m from
// Philox counter (row, col, tag(stream, m + 1, rep), t).
hipError_t launch_als_init_nd(const NdFactors& F, int N, int R, int rep0, int nrep,
                              uint64_t seed, uint32_t tensor_id, uint32_t stream, uint32_t t,
                              hipStream_t s);

// Summary of order N: Z[rep](a_0, ..., a_N-1) = X(S_0[a_0], ..., K'[a_N-1]),
// S_m at idx + rep * idx_stride + off[m]; K'[c] = S_N-1[c] for c < n3old,
// Kold + c - n3old after.
struct GatherNd {
  const void* X;
  int N;
  int64_t D[kMaxOrder];  // store extents (last one unused)
  int n[kMaxOrder];      // summary extents
  const int32_t* idx;
  int64_t idx_stride;
  int64_t off[kMaxOrder];
  int n3old;
  int64_t Kold;
  int rep0, nrep;
  void* Z;
  int64_t sZ;
};
hipError_t launch_gather_nd(int prec, const GatherNd& g, hipStream_t s);

// R x R cross products X^T Y over `rows` rows, one block per (job, repetition):
// X rows X + rep * sX + (ix ? ix[rep * six + i] : i) * R, Y likewise; result
// at out + (rep * njobs + job) * R * R.
constexpr int kCrossJobs = 3 * kMaxOrder;
struct CrossNd {
  XJob job[kCrossJobs];
  int njobs, R, rep0, nrep;
  double* out;
};
hipError_t launch_cross_nd(const CrossNd& c, hipStream_t s);

// Matching over N modes from the cross products of CrossNd laid out per mode
// as (anchor^T sample, anchor^T anchor, sample^T sample): similarity = product
// of |cosine| over the modes, assignment, signs and scales of the fixed modes
// (scl[rep][m][f]), validity and Gt = prod over fixed modes of the matched
// Gram matrices.
struct MatchNd {
  const double* xo;
  int N, R, rep0, nrep;
  double* scl;      // [rep][kMaxOrder][R]
  int32_t *pi, *valid;
  double* Gt;       // [rep][R * R]
};
hipError_t launch_match_nd(const MatchNd& m, hipStream_t s);
// Ut_m(a, f) = scl_m(f) Up_m(a, pi(f)) for the fixed modes
hipError_t launch_match_rows_nd(const NdFactors& Up, const NdFactors& Ut, int N, int R,
                                int rep0, int nrep, const double* scl, const int32_t* pi,
                                hipStream_t s);

// Zero fill of the fixed-mode factors and of the last factor's sampled rows,
// the new rows of the last factor (average over the valid repetitions) and
// the importance commit; nothing is written when *err != 0.
struct CommitNd {
  const uint32_t* err;
  int N, R, nrep;
  double* U[kMaxOrder];      // model (last factor: Kcap rows)
  int64_t D[kMaxOrder];      // fixed extents; D[N-1] = Kold
  int64_t Knew;
  const int32_t* idx;
  int64_t idx_stride;
  int64_t off[kMaxOrder];
  int n[kMaxOrder];          // sample sizes (last: n3old)
  const double* Ut[kMaxOrder];
  int64_t sUt[kMaxOrder];
  const double* Ct;          // per repetition Kp x R
  int64_t sCt;
  const int32_t* valid;
  uint64_t* w[kMaxOrder];    // importance (last: Kcap entries)
  const uint64_t* dw[kMaxOrder];
};
hipError_t launch_commit_nd(const CommitNd& c, hipStream_t s);
// W = Z x3 C on a view with few rows and a long third index (p1's [f][e]
// layout of W): S ranges of the third index per row tile, partial W in Wp
// (stride sWp per repetition, S * n1 * n2 * R) summed in range order; S = 1
// writes W directly.  p1s_splits: the S used for a view.
int p1s_splits(int64_t n12, int Q, int nrep);
// krp: instead of reading Cf, form the Khatri-Rao rows of the modes c0..N-1
// of these factors while staging them (the view's third index runs over
// those modes, c0 fastest).
hipError_t launch_p1s(int prec, const RepSet& rs, const void* Z, const double* Cf, int S,
                      void* Wp, int64_t sWp, void* W, hipStream_t s,
                      const NdFactors* krp = nullptr, int c0 = -1, int N = 0);
// launch_solve (normalising) with V = the Hadamard product, in mode order, of
// the Gram matrices Gm + m * sGmode (per repetition stride R*R) of the modes
// in `mask`
hipError_t launch_solve_prod(const RepSet& rs, int rows, const double* M, const double* Gm,
                             int64_t sGmode, uint32_t mask, double* U, int64_t sU, double* Gout,
                             double* lam_out, uint32_t* pinv_count, hipStream_t s);
// components ordered by lam descending (ties: lower index first), every factor
hipError_t launch_sort_nd(const NdFactors& F, int N, int R, double* lam, hipStream_t s);

// ---------------------------------------------------------------------------
// Sparse (COO) tensors of order N
// ---------------------------------------------------------------------------
// A batch (or the initial entries): coordinates per mode, values; D the
// extents the coordinates must lie in (the last: the batch's slices).
struct CooNd {
  int N;
  const int32_t* idx[kMaxOrder];
  const float* v;
  int64_t nnz;
  int64_t D[kMaxOrder];
};
struct NdWeights {
  uint64_t* w[kMaxOrder];
};
struct CooStoreNd {
  int32_t* idx[kMaxOrder];
  float* v;
};
// concatenated summaries: coordinates (positions in the samples), values and
// the repetition of every entry (null: all repetition 0)
struct CooSumNd {
  int32_t* idx[kMaxOrder];
  float* v;
  uint8_t* rep;
};
// position maps per repetition: mode m's part at posoff[m], stride entries
struct PosViewNd {
  int N;
  int64_t posoff[kMaxOrder];
  int64_t stride;
};
struct PosMapsNd {
  int N;
  const int32_t* idx;  // samples (per repetition at rep * idx_stride, mode m at off[m])
  int64_t idx_stride;
  int64_t off[kMaxOrder];
  int n[kMaxOrder];    // sample sizes (the last: old slices)
  int64_t posoff[kMaxOrder];
  int64_t stride;
  int64_t Kold, Knew;
};
// M(rep, row, f) over the entries [off[rep (rows + 1) + row], ... + 1) in the
// order perm (null: positions themselves) of mode `mode`
struct MttkrpCooNd {
  int N, mode, R, rows, rep0, nrep;
  const int32_t* idx[kMaxOrder];
  const float* v;
  const int32_t* perm;
  const int64_t* off;
  NdFactors F;
  double* M;
  int64_t sM;
};
// importance of a batch for every mode (integer atomics); err bit 1:
// non-finite or overflow, bit 2: coordinate out of range
hipError_t launch_moi_coo_nd(const CooNd& b, double scale, uint64_t qmax, const NdWeights& w,
                             uint32_t* err, hipStream_t s);
// scratch of launch_coo_ingest_nd for a batch of n entries
size_t coo_nd_sort_bytes(int64_t n);
// the batch stably sorted by its last coordinate, placed at base.. of the
// store with the last coordinate shifted by k0 (nbits: bits of the largest
// batch-relative last coordinate)
hipError_t launch_coo_ingest_nd(const CooNd& b, int64_t base, int64_t k0, int nbits,
                                const CooStoreNd& st, void* tmp, size_t tmp_bytes,
                                hipStream_t s);
// off[x] = lower bound of x in the ascending key[0..n), x in [x0, x1]
hipError_t launch_lower_bounds(const int32_t* key, int64_t n, int64_t x0, int64_t x1,
                               int64_t* off, hipStream_t s);
hipError_t launch_pos_maps_nd(const PosMapsNd& a, int nrep, int32_t* pos, hipStream_t s);
// keep flags of the stored entries per repetition (nrep * nnz + 1 entries)
// and their exclusive scan `at` (at[nrep * nnz] = total kept)
size_t coo_nd_scan_bytes(int64_t n);
hipError_t launch_keep_flags_nd(const CooStoreNd& st, int64_t nnz, const PosViewNd& pv,
                                const int32_t* pos, int nrep, uint32_t* flag, uint32_t* at,
                                void* tmp, size_t tmp_bytes, hipStream_t s);
hipError_t launch_summary_emit_nd(const CooStoreNd& st, int64_t nnz, const PosViewNd& pv,
                                  const int32_t* pos, int nrep, const uint32_t* flag,
                                  const uint32_t* at, const CooSumNd& z, hipStream_t s);
// the summary positions sorted by (repetition, coordinate of mode m) and the
// row offsets off[rep * (rows + 1) + x]
size_t coo_nd_mode_sort_bytes(int64_t n);
hipError_t launch_mode_sort_nd(const CooSumNd& z, int64_t total, int m, int rows, int nrep,
                               uint32_t* key, uint32_t* key_sorted, int32_t* iota,
                               int32_t* perm, int64_t* off, void* tmp, size_t tmp_bytes,
                               hipStream_t s);
// part: room for mttkrp_coo_nd_parts(R) doubles, where the ranges of long
// rows leave their partial rows (null: one wavefront per row)
hipError_t launch_mttkrp_coo_nd(const MttkrpCooNd& a, double* part, hipStream_t s);
// out.idx[l][p] = z.idx[l][perm[p]] for every mode l < N but m,
// out.v[p] = z.v[perm[p]], p < total
hipError_t launch_gather_sorted_nd(const CooSumNd& z, int N, int64_t total, int m,
                                  const int32_t* perm, const CooSumNd& out, hipStream_t s);
int64_t mttkrp_coo_nd_parts(int R);
// nrm[k] = sum of v^2 over the entries [koff[k], koff[k + 1])
hipError_t launch_slice_norms(const float* v, const int64_t* koff, int64_t K, double* nrm,
                              hipStream_t s);

}  // namespace sbt
