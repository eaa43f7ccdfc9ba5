// Tensor state, workspace and the C ABI of the SamBaTen update library.
//
// The library keeps, per tensor, on one GPU:
//   X     the stored tensor (dense column-major, or COO structure of arrays),
//         sized for k_capacity slices so that appending a batch is one copy;
//   A,B,C the CP model (row-major FP64) and lambda;
//   w1..3 the importance of every index of the three modes (exact uint64 sums
//         of floor(x^2 2^S)), kept incrementally across batches;
//   t     the batch counter that keys the sampler's random numbers.
// An update runs entirely on the GPU; the host only enqueues kernels and reads
// back one status word at the end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/sambaten.h"
#include "autotune.h"
#include "device_common.hpp"
#include "kernels.hpp"

using namespace sbt;

// launch shapes whose CP-ALS sweep graphs a tensor keeps
constexpr size_t kGraphCache = 8;

struct NdState;  // tensors of order N (the N-mode part of this file)
struct NdWork;

struct sbt_tensor {
  sbt_config cfg{};
  int64_t I = 0, J = 0, K = 0, Kcap = 0;
  int R = 0;
  int fmt = SBT_DENSE;
  int store_prec = kF32;  // kF64 or kF32
  int sum_prec = kF32;    // kF64, kF32 or kBF16
  // stored tensor
  void* X = nullptr;
  int32_t *ci = nullptr, *cj = nullptr, *ck = nullptr;
  float* cv = nullptr;
  int64_t nnz = 0, nnz_cap = 0;
  // model and importance
  double *A = nullptr, *B = nullptr, *C = nullptr, *lam = nullptr;
  uint64_t *w1 = nullptr, *w2 = nullptr, *w3 = nullptr;
  int S = 0;
  double scale = 1.0;
  uint64_t qmax = 0, nmax = 1;
  uint32_t t = 0;
  // update workspace
  int n1 = 0, n2 = 0, n3max = 0, Kpmax = 0;
  int64_t idx_stride = 0, key_stride = 0;
  uint64_t *dw1 = nullptr, *dw2 = nullptr, *dw3 = nullptr, *keys = nullptr, *bits = nullptr;
  uint32_t *err = nullptr, *pinv = nullptr, *cnt = nullptr;
  int32_t *idx = nullptr, *pi = nullptr, *valid = nullptr;
  void *Z = nullptr, *W = nullptr;
  // BF16 summaries on the matrix cores (batched schedule)
  bool mfma = false;
  MfmaLayout ml{};
  uint16_t *Zk = nullptr, *Zc = nullptr;
  float* P3 = nullptr;  // mode-3 partial rows
  int64_t sP3 = 0;
  float* mops = nullptr;  // staged MFMA operands
  double *Ap = nullptr, *Bp = nullptr, *Cp = nullptr, *GA = nullptr, *GB = nullptr, *GC = nullptr,
         *Gt = nullptr, *ones = nullptr, *lamp = nullptr, *M = nullptr, *At = nullptr,
         *Bt = nullptr, *Ct = nullptr, *M3 = nullptr, *nrm = nullptr, *fitv = nullptr,
         *Vinv = nullptr, *invlam = nullptr;
  uint32_t* h_err = nullptr;  // pinned
  std::vector<void*> allocs;
  // COO path
  int64_t* koff = nullptr;        // slice offsets of the k-sorted store (Kcap + 1)
  int64_t pending_nnz = 0;        // batch entries appended but not yet committed
  int32_t *posI = nullptr, *posJ = nullptr, *posK = nullptr;
  uint64_t *bitI = nullptr, *bitJ = nullptr, *bitK = nullptr;
  uint32_t* bcount = nullptr;
  int64_t* bbase = nullptr;
  CooScratch ing{};               // ingest scratch (grown on demand)
  CooSummary z{};                 // summaries (grown on demand)
  CooUnits cu[3]{};               // MTTKRP work units per mode (grown with the summaries)
  float* upart = nullptr;         // unit partial rows (RP floats per unit)
  float *fA = nullptr, *fB = nullptr, *fC = nullptr;  // FP32 scaled factor copies
  // cross products over many rows (Gram matrices, matching), all repetitions
  double *xpart = nullptr, *xout = nullptr, *scl = nullptr;
  int xnblk = 1;
  int64_t xpart_mats = 0;  // R x R matrices the partial buffer holds
  // GetRank: kept factors (rows padded to R), scores, chosen ranks, cores
  double *gAk = nullptr, *gBk = nullptr, *gCk = nullptr, *glamk = nullptr;
  double *gcc = nullptr, *gbest = nullptr, *gtab = nullptr, *gP = nullptr, *gX1 = nullptr,
         *gX2 = nullptr, *gGi = nullptr;
  double* gWz = nullptr;  // COO: per-slice partial cores [rep][z][R x R]
  int32_t* grnew = nullptr;
  // captured CP-ALS sweep sequences by launch shape (null: seen once)
  std::map<uint64_t, hipGraphExec_t> graphs;
  hipStream_t capst = nullptr;
  // persistent summaries: kept summary factors for the warm start
  double *Bw = nullptr, *Cw = nullptr;
  // SBT_FLAG_LAMBDA_AVG: per repetition the matched summary weights
  double* lhat = nullptr;
  bool have_kept = false;  // I_s, J_s, K_s in idx are the kept ones
  bool z_kept = false;     // the summaries' K_s slices were gathered with those indices
  bool coo_kept = false;   // COO summaries hold the old part of the kept indices
  int64_t* keep_d = nullptr;  // device: old-part starts, counts, new starts (3 x 64)
  int64_t keep_h[4 * 64] = {};  // host: the same, and where each batch part begins
  int n3kept = 0;
  bool warm_now = false;   // this update's summary CP-ALS starts from Bw, Cw
  int warm_n3 = 0;
  std::vector<std::pair<void*, size_t>> grow_allocs; // freed when regrown or destroyed
  int64_t last_summary_nnz = 0;
  // kernel timing (sbt_profile_*)
  bool prof_on = false;
  int prof_stride = 1;   // time every prof_stride-th kernel launch
  uint64_t prof_seq = 0; // kernel launches offered for timing so far
  std::vector<hipEvent_t> prof_ev;     // pairs
  std::vector<int> prof_kind;          // per recorded pair
  std::vector<char> prof_launch;       // pair recorded by a kernel launch itself
  std::vector<double> prof_bytes;      // per recorded pair
  int64_t prof_n[SBT_K_COUNT] = {};
  double prof_ms[SBT_K_COUNT] = {};
  double prof_b[SBT_K_COUNT] = {};
  // tensors of order N created by sbt_nd_init_dense (null otherwise)
  NdState* nd = nullptr;
  NdWork* nd_work = nullptr;
  // last update, for the inspection calls
  bool has_last = false;
  int last_n3old = 0, last_Kp = 0;
  std::string errmsg;
  // device bytes held: fixed allocations, of which the store and the model
  // (store + A, B, C, lambda, importance); grown buffers are in grow_allocs
  size_t bytes_fixed = 0, bytes_resident = 0;
  // one call at a time (SBT_E_BUSY otherwise); server requests queued or running
  std::atomic<bool> busy{false};
  std::atomic<int> leases{0};
};

namespace {

struct Fail {
  sbt_status st;
};

void set_err(sbt_tensor* t, const std::string& m) {
  if (t) t->errmsg = m;
}

#define SBT_CK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      set_err(t, std::string(#expr) + ": " + hipGetErrorString(e_));                    \
      return e_ == hipErrorOutOfMemory ? SBT_E_NOMEM : SBT_E_DEVICE;                    \
    }                                                                                   \
  } while (0)

template <typename T>
sbt_status dalloc(sbt_tensor* t, T** p, size_t count) {
  if (count == 0) count = 1;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) {
    set_err(t, std::string("hipMalloc: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? SBT_E_NOMEM : SBT_E_DEVICE;
  }
  t->allocs.push_back(q);
  t->bytes_fixed += count * sizeof(T);
  *p = (T*)q;
  return SBT_OK;
}

sbt_status dalloc_bytes(sbt_tensor* t, void** p, size_t bytes) {
  return dalloc<char>(t, (char**)p, bytes);
}

#define SBT_TRY(expr)                   \
  do {                                  \
    sbt_status s_ = (expr);             \
    if (s_ != SBT_OK) return s_;        \
  } while (0)

// Pass 1 splits the third mode into at most this many ranges (partial W).

// Kernel timing: an event pair per timed launch, resolved after the update's
// final synchronisation.
constexpr size_t kProfPairs = 8192;

// a free event pair, or -1
int prof_pair(sbt_tensor* t) {
  if (!t->prof_on) return -1;
  const size_t q = t->prof_kind.size();
  if (q >= kProfPairs) return -1;
  if (t->prof_ev.size() < 2 * (q + 1)) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return -1;
    }
    t->prof_ev.push_back(a);
    t->prof_ev.push_back(b);
  }
  t->prof_kind.push_back(-1);
  t->prof_bytes.push_back(0.0);
  t->prof_launch.push_back(0);
  return (int)q;
}

// events on the stream around what follows (the whole update)
int prof_begin(sbt_tensor* t, hipStream_t st) {
  const int q = prof_pair(t);
  if (q >= 0 && hipEventRecord(t->prof_ev[2 * (size_t)q], st) != hipSuccess) {
    t->prof_kind.pop_back();
    t->prof_bytes.pop_back();
    t->prof_launch.pop_back();
    return -1;
  }
  return q;
}

// events the next timed kernel launch records at its own start and end
int prof_kernel(sbt_tensor* t) {
  if (!t->prof_on || (t->prof_seq++ % (uint64_t)t->prof_stride) != 0) return -1;
  const int q = prof_pair(t);
  if (q >= 0) {
    t->prof_launch[(size_t)q] = 1;
    launch_timing() = LaunchTiming{t->prof_ev[2 * (size_t)q], t->prof_ev[2 * (size_t)q + 1]};
  }
  return q;
}

void prof_end(sbt_tensor* t, int q, int kind, double bytes, hipStream_t st) {
  if (q < 0) return;
  if (t->prof_launch[(size_t)q]) {
    LaunchTiming& lt = launch_timing();
    if (lt.start == t->prof_ev[2 * (size_t)q]) {  // no timed launch took the pair
      lt = LaunchTiming{};
      return;
    }
  } else if (hipEventRecord(t->prof_ev[2 * (size_t)q + 1], st) != hipSuccess) {
    return;
  }
  t->prof_kind[(size_t)q] = kind;
  t->prof_bytes[(size_t)q] = bytes;
}

// after the stream has been synchronised
void prof_collect(sbt_tensor* t) {
  for (size_t q = 0; q < t->prof_kind.size(); ++q) {
    const int kind = t->prof_kind[q];
    if (kind < 0) continue;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, t->prof_ev[2 * q], t->prof_ev[2 * q + 1]) != hipSuccess) continue;
    t->prof_n[kind] += 1;
    t->prof_ms[kind] += ms;
    t->prof_b[kind] += t->prof_bytes[q];
  }
  t->prof_kind.clear();
  t->prof_bytes.clear();
  t->prof_launch.clear();
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

int64_t sample_size(int64_t N, int64_t s) {
  int64_t n = ceil_div(N, s);
  if (n < 1) n = 1;
  if (n > N) n = N;
  return n;
}

int bit_length(uint64_t v) {
  int n = 0;
  while (v) {
    ++n;
    v >>= 1;
  }
  return n;
}

sbt_status validate_config(const sbt_config* c, std::string& why) {
  if (!c) {
    why = "null config";
    return SBT_E_INVALID;
  }
  bool sf_ok = true;
  for (int m = 0; m < 3; ++m) sf_ok = sf_ok && c->sample_factor[m] >= 1;
  const bool gr = c->getrank_runs > 0;
  const struct {
    bool bad;
    const char* why;
  } checks[] = {
      {c->rank < 1 || c->rank > kMaxRank, "rank must be in 1..32"},
      {c->repetitions < 1 || c->repetitions > 4096, "repetitions must be in 1..4096"},
      {c->als_iters < 1 || c->init_iters < 0, "bad iteration counts"},
      {!sf_ok, "sample factors must be >= 1"},
      {c->format != SBT_DENSE && c->format != SBT_COO, "bad format"},
      {c->precision < SBT_P_F64 || c->precision > SBT_P_BF16, "bad precision"},
      {c->schedule != SBT_SCHED_BATCHED && c->schedule != SBT_SCHED_PLAIN, "bad schedule"},
      {(c->flags & ~(uint32_t)SBT_FLAG_LAMBDA_AVG) != 0 || c->reserved != 0,
       "unknown flags, or reserved not 0"},
      {c->getrank_runs < 0 || c->getrank_runs > 64, "getrank_runs must be in 0..64"},
      {gr && c->precision == SBT_P_BF16, "GetRank needs FP64 or FP32 summaries"},
      {gr && !(c->getrank_threshold == c->getrank_threshold), "bad GetRank threshold"},
      {c->persist_summaries != 0 && c->persist_summaries != 1, "persist_summaries must be 0 or 1"},
      {c->summary_refresh < 0, "summary_refresh must be >= 0"},
      {c->persist_summaries && gr, "persistent summaries and GetRank do not combine"},
      {c->max_batch < 1, "max_batch must be >= 1"},
  };
  for (const auto& k : checks) {
    if (k.bad) {
      why = k.why;
      return SBT_E_INVALID;
    }
  }
  return SBT_OK;
}

RepSet make_repset(const sbt_tensor* t, int n3, int rep0, int nrep) {
  RepSet rs;
  rs.n1 = t->n1;
  rs.n2 = t->n2;
  rs.n3 = n3;
  rs.R = t->R;
  rs.rep0 = rep0;
  rs.nrep = nrep;
  // dense summary slices start on 128-byte lines: the streaming passes read
  // each slice's rows in 256-byte pieces, which then never straddle a line
  // shared with a piece another block reads
  const int64_t al = 128 / (int64_t)prec_bytes(t->sum_prec);
  rs.ldz = ((int64_t)t->n1 * t->n2 + al - 1) / al * al;
  rs.sZ = rs.ldz * t->Kpmax;
  rs.sA = (int64_t)t->n1 * t->R;
  rs.sB = (int64_t)t->n2 * t->R;
  rs.sC = (int64_t)t->Kpmax * t->R;
  rs.sW = (int64_t)t->n1 * t->n2 * t->R;
  rs.nsplit = 1;
  int64_t mx = t->n1 > t->n2 ? t->n1 : t->n2;
  if (t->Kpmax > mx) mx = t->Kpmax;
  rs.sM = mx * t->R;
  rs.sG = (int64_t)t->R * t->R;
  return rs;
}

// Common part of init: state buffers, workspace, scale of the importance.
sbt_status alloc_state(sbt_tensor* t) {
  const sbt_config& c = t->cfg;
  const int R = t->R;
  SBT_TRY(dalloc(t, &t->A, (size_t)t->I * R));
  SBT_TRY(dalloc(t, &t->B, (size_t)t->J * R));
  SBT_TRY(dalloc(t, &t->C, (size_t)t->Kcap * R));
  SBT_TRY(dalloc(t, &t->lam, (size_t)R));
  SBT_TRY(dalloc(t, &t->w1, (size_t)t->I));
  SBT_TRY(dalloc(t, &t->w2, (size_t)t->J));
  SBT_TRY(dalloc(t, &t->w3, (size_t)t->Kcap));
  t->n1 = (int)sample_size(t->I, c.sample_factor[0]);
  t->n2 = (int)sample_size(t->J, c.sample_factor[1]);
  t->n3max = (int)sample_size(t->Kcap, c.sample_factor[2]);
  t->Kpmax = t->n3max + (int)c.max_batch;
  const int r = c.repetitions;
  t->idx_stride = (int64_t)t->n1 + t->n2 + t->n3max;
  t->key_stride = t->I + t->J + t->Kcap;
  SBT_TRY(dalloc(t, &t->dw1, (size_t)t->I));
  SBT_TRY(dalloc(t, &t->dw2, (size_t)t->J));
  SBT_TRY(dalloc(t, &t->dw3, (size_t)c.max_batch));
  SBT_TRY(dalloc(t, &t->keys, (size_t)r * t->key_stride));
  SBT_TRY(dalloc(t, &t->bits, 1));
  SBT_TRY(dalloc(t, &t->err, 1));
  SBT_TRY(dalloc(t, &t->pinv, 1));
  SBT_TRY(dalloc(t, &t->cnt, (size_t)2 * r));
  SBT_TRY(dalloc(t, &t->idx, (size_t)r * t->idx_stride));
  SBT_TRY(dalloc(t, &t->pi, (size_t)r * R));
  SBT_TRY(dalloc(t, &t->valid, (size_t)r * R));
  RepSet rs = make_repset(t, t->Kpmax, 0, r);
  t->mfma = t->fmt == SBT_DENSE && t->sum_prec == kBF16 &&
            c.schedule == SBT_SCHED_BATCHED && mfma_supported(t->n1, t->n2, R);
  if (t->mfma) {
    t->ml = mfma_layout(t->n1, t->n2, t->Kpmax);
    RepSet r1 = rs;
    r1.n3 = 1;
    const int nsmax = mfma_mode3_splits(r1, t->ml);
    t->sP3 = (int64_t)t->Kpmax * (R <= 16 ? 16 : 32);
    SBT_TRY(dalloc(t, &t->Zk, (size_t)r * t->ml.sZk));
    SBT_TRY(dalloc(t, &t->Zc, (size_t)r * t->ml.sZc));
    SBT_TRY(dalloc(t, &t->P3, (size_t)r * nsmax * t->sP3));
    SBT_TRY(dalloc(t, &t->mops, (size_t)r * mfma_operand_floats(t->ml, t->n2, R)));
    SBT_TRY(dalloc_bytes(t, &t->W, (size_t)r * rs.sW * sizeof(float)));
    // padding of Zk is never written by the gather: zero it once
    hipError_t e = hipMemset(t->Zk, 0, sizeof(uint16_t) * (size_t)r * t->ml.sZk);
    if (e != hipSuccess) {
      set_err(t, hipGetErrorString(e));
      return SBT_E_DEVICE;
    }
  } else if (t->fmt == SBT_DENSE) {
    SBT_TRY(dalloc_bytes(t, &t->Z, (size_t)r * rs.sZ * prec_bytes(t->sum_prec)));
    SBT_TRY(dalloc_bytes(t, &t->W, (size_t)r * rs.sW * acc_bytes(t->sum_prec)));
  }
  SBT_TRY(dalloc(t, &t->Ap, (size_t)r * rs.sA));
  SBT_TRY(dalloc(t, &t->Bp, (size_t)r * rs.sB));
  SBT_TRY(dalloc(t, &t->Cp, (size_t)r * rs.sC));
  SBT_TRY(dalloc(t, &t->At, (size_t)r * rs.sA));
  SBT_TRY(dalloc(t, &t->Bt, (size_t)r * rs.sB));
  SBT_TRY(dalloc(t, &t->Ct, (size_t)r * rs.sC));
  SBT_TRY(dalloc(t, &t->M, (size_t)r * rs.sM));
  SBT_TRY(dalloc(t, &t->GA, (size_t)r * rs.sG));
  SBT_TRY(dalloc(t, &t->GB, (size_t)r * rs.sG));
  SBT_TRY(dalloc(t, &t->GC, (size_t)r * rs.sG));
  SBT_TRY(dalloc(t, &t->Gt, (size_t)r * rs.sG));
  SBT_TRY(dalloc(t, &t->ones, (size_t)rs.sG));
  SBT_TRY(dalloc(t, &t->lamp, (size_t)r * R));
  SBT_TRY(dalloc(t, &t->Vinv, (size_t)r * rs.sG));
  SBT_TRY(dalloc(t, &t->invlam, (size_t)r * 3 * R));
  {
    int mr = t->n1 > t->n2 ? t->n1 : t->n2;
    if (t->Kpmax > mr) mr = t->Kpmax;
    int64_t mf = t->I > t->J ? t->I : t->J;
    if (t->Kcap > mf) mf = t->Kcap;
    t->xnblk = xprod_blocks(mr);
    const int64_t fit_nblk = xprod_blocks((int)mf);
    int64_t np = (int64_t)r * 9 * t->xnblk;
    if (9 * fit_nblk > np) np = 9 * fit_nblk;  // fit: 3 products, FMS: 9
    SBT_TRY(dalloc(t, &t->xpart, (size_t)np * R * R));
    t->xpart_mats = np;
    SBT_TRY(dalloc(t, &t->xout, (size_t)r * 9 * R * R));
    SBT_TRY(dalloc(t, &t->scl, (size_t)r * 2 * R));
  }
  if (c.persist_summaries) {
    SBT_TRY(dalloc(t, &t->Bw, (size_t)r * rs.sB));
    SBT_TRY(dalloc(t, &t->Cw, (size_t)r * rs.sC));
  }
  if (c.flags & SBT_FLAG_LAMBDA_AVG) SBT_TRY(dalloc(t, &t->lhat, (size_t)r * R));
  if (c.getrank_runs > 0) {
    const size_t R3 = (size_t)R * R * R;
    SBT_TRY(dalloc(t, &t->gAk, (size_t)r * rs.sA));
    SBT_TRY(dalloc(t, &t->gBk, (size_t)r * rs.sB));
    SBT_TRY(dalloc(t, &t->gCk, (size_t)r * rs.sC));
    SBT_TRY(dalloc(t, &t->glamk, (size_t)r * R));
    SBT_TRY(dalloc(t, &t->gcc, (size_t)r));
    SBT_TRY(dalloc(t, &t->gbest, (size_t)r));
    SBT_TRY(dalloc(t, &t->gtab, (size_t)r * R * c.getrank_runs));
    SBT_TRY(dalloc(t, &t->gP, (size_t)r * R3));
    SBT_TRY(dalloc(t, &t->gX1, (size_t)r * R3));
    SBT_TRY(dalloc(t, &t->gX2, (size_t)r * R3));
    SBT_TRY(dalloc(t, &t->gGi, (size_t)3 * r * rs.sG));
    SBT_TRY(dalloc(t, &t->grnew, (size_t)r));
    if (t->fmt == SBT_COO) SBT_TRY(dalloc(t, &t->gWz, (size_t)r * t->Kpmax * R * R));
  }
  SBT_TRY(dalloc(t, &t->M3, (size_t)t->Kcap * R));
  SBT_TRY(dalloc(t, &t->nrm, (size_t)t->Kcap));
  SBT_TRY(dalloc(t, &t->fitv, 1));
  if (t->fmt == SBT_COO) {
    const int64_t nblk = coo_scan_blocks(t->nnz_cap);
    SBT_TRY(dalloc(t, &t->koff, (size_t)t->Kcap + 1));
    SBT_TRY(dalloc(t, &t->posI, (size_t)r * t->I));
    SBT_TRY(dalloc(t, &t->posJ, (size_t)r * t->J));
    SBT_TRY(dalloc(t, &t->posK, (size_t)r * t->Kcap));
    SBT_TRY(dalloc(t, &t->bitI, (size_t)t->I));
    SBT_TRY(dalloc(t, &t->bitJ, (size_t)t->J));
    SBT_TRY(dalloc(t, &t->bitK, (size_t)t->Kcap));
    SBT_TRY(dalloc(t, &t->bcount, (size_t)r * nblk));
    SBT_TRY(dalloc(t, &t->bbase, (size_t)r * (nblk + 1)));
    SBT_TRY(dalloc(t, &t->ing.hist, (size_t)t->Kcap));
    CooSummary& z = t->z;
    z.sOffA = t->n1 + 1;
    z.sOffB = t->n2 + 1;
    z.sOffC = t->Kpmax + 1;
    SBT_TRY(dalloc(t, &z.offA, (size_t)r * z.sOffA));
    SBT_TRY(dalloc(t, &z.offB, (size_t)r * z.sOffB));
    SBT_TRY(dalloc(t, &z.offC, (size_t)r * z.sOffC));
    SBT_TRY(dalloc(t, &z.rep_off, 65));
    SBT_TRY(dalloc(t, &t->keep_d, (size_t)3 * 64));
    const int64_t mrows[3] = {t->n1, t->n2, t->Kpmax};
    for (int m = 0; m < 3; ++m) {
      SBT_TRY(dalloc(t, &t->cu[m].cnt, (size_t)r * mrows[m]));
      SBT_TRY(dalloc(t, &t->cu[m].uoff, (size_t)r * mrows[m] + 1));
    }
    SBT_TRY(dalloc(t, &t->fA, (size_t)r * t->n1 * kMaxRank));
    SBT_TRY(dalloc(t, &t->fB, (size_t)r * t->n2 * kMaxRank));
    SBT_TRY(dalloc(t, &t->fC, (size_t)r * t->Kpmax * kMaxRank));
  }
  void* h = nullptr;
  hipError_t e = hipHostMalloc(&h, 64, hipHostMallocDefault);
  if (e != hipSuccess) {
    set_err(t, "hipHostMalloc failed");
    return SBT_E_NOMEM;
  }
  t->h_err = (uint32_t*)h;
  return SBT_OK;
}

// Grown-on-demand buffers (ingest scratch, summaries).
template <typename T>
sbt_status galloc(sbt_tensor* t, T** p, size_t count) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, (count ? count : 1) * sizeof(T));
  if (e != hipSuccess) {
    set_err(t, std::string("hipMalloc: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? SBT_E_NOMEM : SBT_E_DEVICE;
  }
  t->grow_allocs.emplace_back(q, (count ? count : 1) * sizeof(T));
  *p = (T*)q;
  return SBT_OK;
}

void gfree(sbt_tensor* t, void* p) {
  for (size_t q = 0; q < t->grow_allocs.size(); ++q)
    if (t->grow_allocs[q].first == p) {
      (void)hipFree(p);
      t->grow_allocs.erase(t->grow_allocs.begin() + (long)q);
      return;
    }
}

sbt_status ensure_ingest(sbt_tensor* t, int64_t n, hipStream_t st) {
  CooScratch& w = t->ing;
  if (n <= w.cap) return SBT_OK;
  SBT_CK(hipStreamSynchronize(st));
  gfree(t, w.key_in);
  gfree(t, w.key_out);
  gfree(t, w.val_in);
  gfree(t, w.val_out);
  gfree(t, w.tmp);
  const int64_t cap = n + n / 4 + 1024;
  SBT_TRY(galloc(t, &w.key_in, (size_t)cap));
  SBT_TRY(galloc(t, &w.key_out, (size_t)cap));
  SBT_TRY(galloc(t, &w.val_in, (size_t)cap));
  SBT_TRY(galloc(t, &w.val_out, (size_t)cap));
  SBT_CK(coo_sort_tmp_bytes(cap, &w.tmp_bytes));
  SBT_TRY(galloc(t, (char**)&w.tmp, w.tmp_bytes));
  w.cap = cap;
  return SBT_OK;
}

sbt_status ensure_summary(sbt_tensor* t, int64_t n, hipStream_t st) {
  CooSummary& z = t->z;
  if (n <= z.cap) return SBT_OK;
  SBT_CK(hipStreamSynchronize(st));
  void* olds[] = {z.a, z.b, z.c, z.v, z.a_x, z.a_y, z.a_v, z.b_x, z.b_y, z.b_v,
                  z.key_a, z.key_b, z.key_out, z.val, z.perm, z.tmp};
  for (void* p : olds) gfree(t, p);
  const int64_t cap = n + n / 4 + 4096;
  SBT_TRY(galloc(t, &z.a, (size_t)cap));
  SBT_TRY(galloc(t, &z.b, (size_t)cap));
  SBT_TRY(galloc(t, &z.c, (size_t)cap));
  SBT_TRY(galloc(t, &z.v, (size_t)cap));
  SBT_TRY(galloc(t, &z.a_x, (size_t)cap));
  SBT_TRY(galloc(t, &z.a_y, (size_t)cap));
  SBT_TRY(galloc(t, &z.a_v, (size_t)cap));
  SBT_TRY(galloc(t, &z.b_x, (size_t)cap));
  SBT_TRY(galloc(t, &z.b_y, (size_t)cap));
  SBT_TRY(galloc(t, &z.b_v, (size_t)cap));
  SBT_TRY(galloc(t, &z.key_a, (size_t)cap));
  SBT_TRY(galloc(t, &z.key_b, (size_t)cap));
  SBT_TRY(galloc(t, &z.key_out, (size_t)cap));
  SBT_TRY(galloc(t, &z.val, (size_t)cap));
  SBT_TRY(galloc(t, &z.perm, (size_t)cap));
  SBT_CK(coo_sort_tmp_bytes(cap, &z.tmp_bytes));
  SBT_TRY(galloc(t, (char**)&z.tmp, z.tmp_bytes));
  z.cap = cap;
  // work units: at most entries / unit + one per row, per mode
  const int r = t->cfg.repetitions;
  const int64_t mrows[3] = {t->n1, t->n2, t->Kpmax};
  int64_t pmax = 0;
  for (int m = 0; m < 3; ++m) {
    CooUnits& u = t->cu[m];
    gfree(t, u.urow);
    gfree(t, u.ustart);
    gfree(t, u.ulen);
    u.cap = cap / kCooUnit + (int64_t)r * mrows[m] + 1;
    SBT_TRY(galloc(t, &u.urow, (size_t)u.cap));
    SBT_TRY(galloc(t, &u.ustart, (size_t)u.cap));
    SBT_TRY(galloc(t, &u.ulen, (size_t)u.cap));
    if (u.cap > pmax) pmax = u.cap;
  }
  gfree(t, t->upart);
  SBT_TRY(galloc(t, &t->upart, (size_t)pmax * kMaxRank));
  return SBT_OK;
}

// Build the r COO summaries of an update: position maps and masks, count,
// per repetition offsets, emit (sorted by c), row offsets, sorted copies.
// Persistent COO summaries: the old part of each summary (its rows c < n3old,
// a prefix in c order) is what the last build left for the same indices, so
// only the batch's entries are scanned.  The old parts move to their places
// in the new layout (through the a-sorted copy's arrays, rebuilt afterwards),
// the batch's entries are emitted behind them, and the arrays come out
// exactly as a scan of the whole store would leave them.  false: the
// summaries do not fit the allocation; nothing has been changed.
sbt_status coo_keep_old(sbt_tensor* t, int64_t Kold, int n3old, int Kp, bool* done,
                        hipStream_t st) {
  *done = false;
  const int r = t->cfg.repetitions;
  CooSummary& z = t->z;
  if (r > 64) return SBT_OK;
  std::vector<int64_t> oe((size_t)r), tot((size_t)r);
  for (int q = 0; q < r; ++q)
    SBT_CK(hipMemcpyAsync(&oe[(size_t)q], z.offC + (int64_t)q * z.sOffC + n3old, 8,
                          hipMemcpyDeviceToHost, st));
  const int32_t* bi = t->ci + t->nnz;
  const int32_t* bj = t->cj + t->nnz;
  const int32_t* bk = t->ck + t->nnz;
  const float* bv = t->cv + t->nnz;
  const int64_t nb = t->pending_nnz;
  SBT_CK(launch_coo_count(bi, bj, bk, nb, t->bitI, t->bitJ, t->bitK, Kold, r, t->bcount,
                          t->bbase, st));
  const int64_t nblk = coo_scan_blocks(nb);
  for (int q = 0; q < r; ++q)
    SBT_CK(hipMemcpyAsync(&tot[(size_t)q], t->bbase + (int64_t)q * (nblk + 1) + nblk, 8,
                          hipMemcpyDeviceToHost, st));
  SBT_CK(hipStreamSynchronize(st));
  int64_t* src = t->keep_h;
  int64_t* cnt = t->keep_h + 64;
  int64_t* dst = t->keep_h + 128;
  int64_t total = 0, most = 0;
  for (int q = 0; q < r; ++q) {
    src[q] = z.rep_off_h[q];
    cnt[q] = oe[(size_t)q] - src[q];
    dst[q] = total;
    total += cnt[q] + tot[(size_t)q];
    most = std::max(most, cnt[q]);
  }
  if (total > z.cap) return SBT_OK;
  SBT_CK(hipMemcpyAsync(t->keep_d, t->keep_h, sizeof(int64_t) * 3 * 64, hipMemcpyHostToDevice,
                        st));
  const int64_t* src_d = t->keep_d;
  const int64_t* cnt_d = t->keep_d + 64;
  const int64_t* dst_d = t->keep_d + 128;
  const int gq = prof_kernel(t);
  SBT_CK(launch_summary_move(z.a, z.b, z.c, z.v, src_d, cnt_d, dst_d, r, most, z.a_x, z.a_y,
                             z.b_x, z.a_v, st));
  SBT_CK(launch_summary_move(z.a_x, z.a_y, z.b_x, z.a_v, dst_d, cnt_d, dst_d, r, most, z.a, z.b,
                             z.c, z.v, st));
  prof_end(t, gq, SBT_K_GATHER, 32.0 * (double)(total - nb), st);
  // the batch's entries behind each old part: the emit writes repetition q
  // from z.rep_off[q] on
  int64_t* starts = t->keep_h + 192;
  for (int q = 0; q < r; ++q) starts[q] = dst[q] + cnt[q];
  SBT_CK(hipMemcpyAsync(z.rep_off, starts, sizeof(int64_t) * r, hipMemcpyHostToDevice, st));
  SBT_CK(launch_coo_emit(bi, bj, bk, bv, nb, t->bitI, t->bitJ, t->bitK, Kold, n3old, r, t->posI,
                         t->posJ, t->posK, t->I, t->J, t->Kcap, t->bbase, z, st));
  for (int q = 0; q < r; ++q) z.rep_off_h[q] = dst[q];
  z.rep_off_h[r] = total;
  SBT_CK(hipMemcpyAsync(z.rep_off, z.rep_off_h, sizeof(int64_t) * (r + 1), hipMemcpyHostToDevice,
                        st));
  // the pinned host copies above are read by the stream before they change
  SBT_CK(hipStreamSynchronize(st));
  t->last_summary_nnz = total;
  SBT_CK(launch_coo_sorts(z, r, total, t->n1, t->n2, Kp, st));
  RepSet rs = make_repset(t, Kp, 0, r);
  for (int m = 0; m < 3; ++m) SBT_CK(launch_coo_units_build(rs, m, z, t->cu[m], st));
  *done = true;
  return SBT_OK;
}

sbt_status coo_build_summaries(sbt_tensor* t, int64_t Kold, int n3old, int Kp, bool keep_old,
                               hipStream_t st) {
  const int r = t->cfg.repetitions;
  const int64_t offJ = t->n1, offK = (int64_t)t->n1 + t->n2;
  const int64_t nnz_all = t->nnz + t->pending_nnz;
  SBT_CK(launch_coo_maps(t->idx, t->idx_stride, offJ, offK, t->n1, t->n2, n3old, r, t->posI,
                         t->posJ, t->posK, t->I, t->J, t->Kcap, t->bitI, t->bitJ, t->bitK, st));
  if (keep_old) {
    bool done = false;
    SBT_TRY(coo_keep_old(t, Kold, n3old, Kp, &done, st));
    if (done) return SBT_OK;
  }
  SBT_CK(launch_coo_count(t->ci, t->cj, t->ck, nnz_all, t->bitI, t->bitJ, t->bitK, Kold, r,
                          t->bcount, t->bbase, st));
  const int64_t nblk = coo_scan_blocks(nnz_all);
  std::vector<int64_t> tot((size_t)r);
  for (int q = 0; q < r; ++q)
    SBT_CK(hipMemcpyAsync(&tot[(size_t)q], t->bbase + (int64_t)q * (nblk + 1) + nblk, 8,
                          hipMemcpyDeviceToHost, st));
  SBT_CK(hipStreamSynchronize(st));
  CooSummary& z = t->z;
  z.rep_off_h[0] = 0;
  for (int q = 0; q < r; ++q) z.rep_off_h[q + 1] = z.rep_off_h[q] + tot[(size_t)q];
  const int64_t total = z.rep_off_h[r];
  t->last_summary_nnz = total;
  SBT_TRY(ensure_summary(t, total, st));
  SBT_CK(hipMemcpyAsync(z.rep_off, z.rep_off_h, sizeof(int64_t) * (r + 1), hipMemcpyHostToDevice,
                        st));
  const int gq = prof_kernel(t);
  SBT_CK(launch_coo_emit(t->ci, t->cj, t->ck, t->cv, nnz_all, t->bitI, t->bitJ, t->bitK, Kold,
                         n3old, r, t->posI, t->posJ, t->posK, t->I, t->J, t->Kcap, t->bbase, z,
                         st));
  prof_end(t, gq, SBT_K_GATHER, (double)nnz_all * 16.0 + (double)total * 16.0, st);
  SBT_CK(launch_coo_sorts(z, r, total, t->n1, t->n2, Kp, st));
  RepSet rs = make_repset(t, Kp, 0, r);
  for (int m = 0; m < 3; ++m) SBT_CK(launch_coo_units_build(rs, m, z, t->cu[m], st));
  return SBT_OK;
}

// Gram matrices U^T U of `rows` rows for every repetition of rs into G (stride sG):
// one block per repetition for short factors, the chunked cross-product
// kernels for long ones.
sbt_status gram_rows(sbt_tensor* t, const RepSet& rs, const double* U, int64_t sU, int rows,
                     double* G, hipStream_t st) {
  if (rows <= 256) {
    SBT_CK(launch_gram(rs, U, sU, rows, G, st));
    return SBT_OK;
  }
  XProd xp{};
  xp.job[0] = XJob{U, sU, nullptr, 0, U, sU, nullptr, 0, rows};
  xp.njobs = 1;
  xp.R = rs.R;
  xp.rep0 = rs.rep0;
  xp.nrep = rs.nrep;
  xp.nblk = xprod_blocks(rows);  // also the whole-tensor factors of the initial CP-ALS
  if ((int64_t)(rs.rep0 + rs.nrep) * xp.nblk > t->xpart_mats) {
    set_err(t, "cross-product workspace too small for these rows");
    return SBT_E_SHAPE;
  }
  xp.part = t->xpart;
  xp.out = G;  // [rep][1][rs.R^2] at stride sG (also below the full rank)
  xp.sOut = rs.sG;
  SBT_CK(launch_xprod(xp, st));
  return SBT_OK;
}

// Partial Gram matrices of a row kernel (one per block of rows) go to the
// cross-product workspace, one slab of this many elements per repetition.
int64_t gram_part_stride(const sbt_tensor* t) { return (int64_t)9 * t->xnblk * t->R * t->R; }

// The buffer for the partial Gram matrices of `rows` rows, when the tail
// would otherwise take the chunked cross products and they fit the workspace.
double* gram_parts_buf(sbt_tensor* t, const RepSet& rs, int rows) {
  if (tail_rows_fit(rows / 2, rs.R)) return nullptr;
  const int64_t mats = gram_part_stride(t) / ((int64_t)t->R * t->R);
  const int64_t need = (int64_t)(rs.rep0 + rs.nrep - 1) * mats + gram_parts(rows);
  return need <= t->xpart_mats ? t->xpart : nullptr;
}

// the tail of a mode update; the tail kernel takes the factor's rows in
// chunks of its staging buffer (one block per repetition), and factors longer
// than two chunks get their Gram matrix from the partial ones the row kernel
// wrote (parts), or else from the chunked cross products (many blocks)
sbt_status tail(sbt_tensor* t, const RepSet& rs, AlsTail ta, hipStream_t st,
                const double* parts = nullptr) {
  if (parts) {
    SBT_CK(launch_tail_parts(rs, ta, parts, gram_part_stride(t), gram_parts(ta.rows), st));
    return SBT_OK;
  }
  if (!tail_rows_fit(ta.rows / 2, rs.R)) {
    SBT_TRY(gram_rows(t, rs, ta.U, ta.sU, ta.rows, t->xout, st));
    ta.Gin = t->xout;
  }
  SBT_CK(launch_tail(rs, ta, st));
  return SBT_OK;
}

// Buffers of a CP-ALS run on COO summaries (the r summaries of an update, or
// the whole tensor as one summary for the initial decomposition).
struct CooAlsBufs {
  const CooSummary* z;
  CooUnits* cu;                       // work units of the three modes
  float *fA, *fB, *fC, *upart;        // staged FP32 factor rows, unit partial rows
  double *Ap, *Bp, *Cp;               // factors (raw during the sweeps, unit at the end)
  double *GA, *GB, *GC, *Vinv, *invlam, *lamp;
  double avg[3];                      // summary entries per row, per mode
  double ebytes;                      // algorithmic bytes of one MTTKRP launch
  int iters;
  uint32_t stream;                    // Philox stream of the initial factors
  uint32_t t_ctr;
  uint32_t col0;                      // first counter column of the initial factors
  bool warm;                          // start from the kept summary factors
};

// CP-ALS on COO summaries: one row-producing MTTKRP launch and one tail per
// mode update.
sbt_status als_coo_core(sbt_tensor* t, RepSet rs, const CooAlsBufs& b, hipStream_t st) {
  const int R = rs.R;
  double* ilA = b.invlam;
  double* ilB = b.invlam + R;
  double* ilC = b.invlam + 2 * R;
  if (b.warm)
    SBT_CK(launch_als_warm(rs, t->cfg.seed, t->cfg.tensor_id, b.stream, b.t_ctr, t->Bw, t->Cw,
                           t->warm_n3, b.Bp, b.Cp, st));
  else
    SBT_CK(launch_als_init(rs, t->cfg.seed, t->cfg.tensor_id, b.stream, b.t_ctr, b.Bp, b.Cp,
                           st, b.col0));
  SBT_TRY(gram_rows(t, rs, b.Bp, rs.sB, rs.n2, b.GB, st));
  SBT_TRY(gram_rows(t, rs, b.Cp, rs.sC, rs.n3, b.GC, st));
  SBT_CK(launch_fill_f64(b.invlam + (int64_t)rs.rep0 * 3 * R, (int64_t)rs.nrep * 3 * R, 1.0,
                         st));
  SBT_CK(launch_inverse(rs, b.GB, rs.sG, b.GC, rs.sG, b.Vinv, t->pinv, st));
  SBT_CK(launch_coo_prep(rs, rs.n2, b.Bp, rs.sB, nullptr, b.fB, st));
  SBT_CK(launch_coo_prep(rs, rs.n3, b.Cp, rs.sC, nullptr, b.fC, st));
  AlsTail ta;
  ta.sG = rs.sG;
  ta.pinv_count = t->pinv;
  for (int it = 0; it < b.iters; ++it) {
    int pq = prof_kernel(t);
    SBT_CK(launch_coo_units(rs, 0, *b.z, b.cu[0], b.fB, rs.n2, b.fC, rs.n3, b.upart, b.avg[0],
                            st));
    prof_end(t, pq, SBT_K_COO_MTTKRP, b.ebytes, st);
    SBT_CK(launch_coo_units_finish(rs, 0, b.cu[0], b.upart, b.Vinv, nullptr, b.Ap, rs.sA, st));
    ta.U = b.Ap; ta.sU = rs.sA; ta.rows = rs.n1; ta.Gout = b.GA; ta.invlam_out = ilA;
    ta.lam_out = nullptr; ta.Gx = b.GA; ta.Gy = b.GC; ta.Vinv_out = b.Vinv;
    SBT_TRY(tail(t, rs, ta, st));
    SBT_CK(launch_coo_prep(rs, rs.n1, b.Ap, rs.sA, ilA, b.fA, st));
    pq = prof_kernel(t);
    SBT_CK(launch_coo_units(rs, 1, *b.z, b.cu[1], b.fA, rs.n1, b.fC, rs.n3, b.upart, b.avg[1],
                            st));
    prof_end(t, pq, SBT_K_COO_MTTKRP, b.ebytes, st);
    SBT_CK(launch_coo_units_finish(rs, 1, b.cu[1], b.upart, b.Vinv, nullptr, b.Bp, rs.sB, st));
    ta.U = b.Bp; ta.sU = rs.sB; ta.rows = rs.n2; ta.Gout = b.GB; ta.invlam_out = ilB;
    ta.lam_out = nullptr; ta.Gx = b.GA; ta.Gy = b.GB; ta.Vinv_out = b.Vinv;
    SBT_TRY(tail(t, rs, ta, st));
    SBT_CK(launch_coo_prep(rs, rs.n2, b.Bp, rs.sB, ilB, b.fB, st));
    pq = prof_kernel(t);
    SBT_CK(launch_coo_units(rs, 2, *b.z, b.cu[2], b.fA, rs.n1, b.fB, rs.n2, b.upart, b.avg[2],
                            st));
    prof_end(t, pq, SBT_K_COO_MTTKRP, b.ebytes, st);
    SBT_CK(launch_coo_units_finish(rs, 2, b.cu[2], b.upart, b.Vinv, nullptr, b.Cp, rs.sC, st));
    ta.U = b.Cp; ta.sU = rs.sC; ta.rows = rs.n3; ta.Gout = b.GC; ta.invlam_out = ilC;
    ta.lam_out = b.lamp; ta.Gx = b.GB; ta.Gy = b.GC; ta.Vinv_out = b.Vinv;
    SBT_TRY(tail(t, rs, ta, st));
    SBT_CK(launch_coo_prep(rs, rs.n3, b.Cp, rs.sC, ilC, b.fC, st));
  }
  SBT_CK(launch_normalize(rs, b.Ap, b.Bp, b.Cp, b.invlam, st));
  return SBT_OK;
}

// CP-ALS on the r COO summaries of an update (at rank rs.R, initial factors
// from the given stream at counter columns col0 + f).
sbt_status run_als_coo(sbt_tensor* t, RepSet rs, uint32_t t_ctr, hipStream_t st,
                       uint32_t stream = kStreamAlsInit, uint32_t col0 = 0) {
  CooAlsBufs b;
  b.z = &t->z;
  b.cu = t->cu;
  b.fA = t->fA;
  b.fB = t->fB;
  b.fC = t->fC;
  b.upart = t->upart;
  b.Ap = t->Ap;
  b.Bp = t->Bp;
  b.Cp = t->Cp;
  b.GA = t->GA;
  b.GB = t->GB;
  b.GC = t->GC;
  b.Vinv = t->Vinv;
  b.invlam = t->invlam;
  b.lamp = t->lamp;
  const double nrow_all = (double)t->cfg.repetitions;
  b.avg[0] = (double)t->last_summary_nnz / (nrow_all * rs.n1);
  b.avg[1] = (double)t->last_summary_nnz / (nrow_all * rs.n2);
  b.avg[2] = (double)t->last_summary_nnz / (nrow_all * rs.n3);
  b.ebytes = (double)t->last_summary_nnz * 12.0;
  b.iters = t->cfg.als_iters;
  b.stream = stream;
  b.t_ctr = t_ctr;
  b.col0 = col0;
  b.warm = t->warm_now && stream == kStreamAlsInit;
  return als_coo_core(t, rs, b, st);
}

// The initial decomposition of a COO tensor: CP-ALS (init_iters sweeps from
// U[0,1) factors of the init stream) on the whole stored tensor, taken as one
// summary with every index kept, then components ordered by lambda.  The
// summary's sorted copies and work units live in temporary buffers.
sbt_status init_cp_als_coo(sbt_tensor* t, hipStream_t st) {
  const int R = t->R;
  const int64_t nnz = t->nnz, I = t->I, J = t->J, K = t->K;
  if (I >= (1 << 24) || J >= (1 << 24) || K >= (1 << 24) || nnz > INT32_MAX) {
    set_err(t, "the initial CP-ALS of a COO tensor needs extents below 2^24");
    return SBT_E_SHAPE;
  }
  RepSet rs;
  rs.n1 = (int)I;
  rs.n2 = (int)J;
  rs.n3 = (int)K;
  rs.R = R;
  rs.rep0 = 0;
  rs.nrep = 1;
  rs.sZ = 0;
  rs.sA = I * R;
  rs.sB = J * R;
  rs.sC = K * R;
  rs.sW = 0;
  rs.sM = 0;
  rs.sG = (int64_t)R * R;
  rs.nsplit = 1;
  std::vector<void*> bufs;
  auto get = [&](void** p, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(p, bytes ? bytes : 1);
    if (e == hipSuccess) bufs.push_back(*p);
    return e;
  };
  auto body = [&]() -> sbt_status {
    const int64_t cap = nnz + 1;
    CooSummary z{};
    int32_t** i32s[] = {&z.a, &z.b, &z.c, &z.a_x, &z.a_y, &z.b_x, &z.b_y, &z.val, &z.perm};
    for (int32_t** q : i32s) SBT_CK(get((void**)q, sizeof(int32_t) * cap));
    float** f32s[] = {&z.v, &z.a_v, &z.b_v};
    for (float** q : f32s) SBT_CK(get((void**)q, sizeof(float) * cap));
    uint32_t** u32s[] = {&z.key_a, &z.key_b, &z.key_out};
    for (uint32_t** q : u32s) SBT_CK(get((void**)q, sizeof(uint32_t) * cap));
    SBT_CK(coo_sort_tmp_bytes(cap, &z.tmp_bytes));
    SBT_CK(get(&z.tmp, z.tmp_bytes));
    z.sOffA = I + 1;
    z.sOffB = J + 1;
    z.sOffC = K + 1;
    SBT_CK(get((void**)&z.offA, sizeof(int64_t) * z.sOffA));
    SBT_CK(get((void**)&z.offB, sizeof(int64_t) * z.sOffB));
    SBT_CK(get((void**)&z.offC, sizeof(int64_t) * z.sOffC));
    SBT_CK(get((void**)&z.rep_off, sizeof(int64_t) * 2));
    z.rep_off_h[0] = 0;
    z.rep_off_h[1] = nnz;
    z.cap = cap;
    SBT_CK(hipMemcpyAsync(z.rep_off, z.rep_off_h, sizeof(int64_t) * 2, hipMemcpyHostToDevice,
                          st));
    SBT_CK(launch_coo_single_summary(t->ci, t->cj, t->ck, t->cv, nnz, rs.n1, rs.n2, rs.n3, z,
                                     st));
    CooUnits cu[3]{};
    const int64_t rows[3] = {I, J, K};
    int64_t pmax = 0;
    for (int m = 0; m < 3; ++m) {
      CooUnits& u = cu[m];
      u.cap = cap / kCooUnit + rows[m] + 1;
      SBT_CK(get((void**)&u.cnt, sizeof(uint32_t) * rows[m]));
      SBT_CK(get((void**)&u.uoff, sizeof(int64_t) * (rows[m] + 1)));
      SBT_CK(get((void**)&u.urow, sizeof(int32_t) * u.cap));
      SBT_CK(get((void**)&u.ustart, sizeof(int64_t) * u.cap));
      SBT_CK(get((void**)&u.ulen, sizeof(int32_t) * u.cap));
      SBT_CK(launch_coo_units_build(rs, m, z, u, st));
      if (u.cap > pmax) pmax = u.cap;
    }
    CooAlsBufs b;
    b.z = &z;
    b.cu = cu;
    SBT_CK(get((void**)&b.fA, sizeof(float) * I * kMaxRank));
    SBT_CK(get((void**)&b.fB, sizeof(float) * J * kMaxRank));
    SBT_CK(get((void**)&b.fC, sizeof(float) * K * kMaxRank));
    SBT_CK(get((void**)&b.upart, sizeof(float) * pmax * kMaxRank));
    double* G = nullptr;
    SBT_CK(get((void**)&G, sizeof(double) * (4 * rs.sG + 3 * R)));
    b.GA = G;
    b.GB = G + rs.sG;
    b.GC = G + 2 * rs.sG;
    b.Vinv = G + 3 * rs.sG;
    b.invlam = G + 4 * rs.sG;
    b.Ap = t->A;
    b.Bp = t->B;
    b.Cp = t->C;
    b.lamp = t->lam;
    b.avg[0] = (double)nnz / (double)I;
    b.avg[1] = (double)nnz / (double)J;
    b.avg[2] = (double)nnz / (double)K;
    b.ebytes = 0.0;
    b.iters = t->cfg.init_iters;
    b.stream = kStreamInit;
    b.t_ctr = 0;
    b.col0 = 0;
    b.warm = false;
    SBT_TRY(als_coo_core(t, rs, b, st));
    SBT_CK(launch_sort_components(t->A, t->B, t->C, t->lam, I, J, K, R, st));
    SBT_CK(hipStreamSynchronize(st));
    return SBT_OK;
  };
  const sbt_status r = body();
  (void)hipStreamSynchronize(st);
  for (void* q : bufs) (void)hipFree(q);
  return r;
}

// Scale S of the importance from max x^2 of the initial tensor (device bits).
sbt_status set_scale(sbt_tensor* t, hipStream_t st) {
  uint64_t b = 0;
  SBT_CK(hipMemcpyAsync(&b, t->bits, 8, hipMemcpyDeviceToHost, st));
  SBT_CK(hipStreamSynchronize(st));
  double mx;
  std::memcpy(&mx, &b, 8);
  if (!std::isfinite(mx)) {
    set_err(t, "initial tensor holds a non-finite value");
    return SBT_E_NUMERIC;
  }
  if (mx > 0.0) {
    int e2 = 0;
    std::frexp(mx, &e2);
    t->S = 58 - e2 - bit_length(t->nmax);
  } else {
    t->S = 32;
  }
  if (t->S < -1000 || t->S > 1000) {
    set_err(t, "importance scale out of range");
    return SBT_E_NUMERIC;
  }
  t->scale = std::ldexp(1.0, t->S);
  t->qmax = (uint64_t)((((unsigned __int128)1) << 63) / t->nmax);
  return SBT_OK;
}

// CP-ALS on a set of summaries (or on the whole tensor with nrep = 1).
sbt_status run_als(sbt_tensor* t, const void* Zp, RepSet rs, double* Ap, double* Bp, double* Cp,
                   double* GA, double* GB, double* GC, double* lam_out, void* W, double* M,
                   double* Vinv, double* invlam, uint32_t stream, uint32_t t_ctr, int iters,
                   bool plain, hipStream_t st, uint32_t col0 = 0) {
  const int prec = t->sum_prec;
  if (t->warm_now && stream == kStreamAlsInit)
    SBT_CK(launch_als_warm(rs, t->cfg.seed, t->cfg.tensor_id, stream, t_ctr, t->Bw, t->Cw,
                           t->warm_n3, Bp, Cp, st));
  else
    SBT_CK(launch_als_init(rs, t->cfg.seed, t->cfg.tensor_id, stream, t_ctr, Bp, Cp, st, col0));
  SBT_TRY(gram_rows(t, rs, Bp, rs.sB, rs.n2, GB, st));
  SBT_TRY(gram_rows(t, rs, Cp, rs.sC, rs.n3, GC, st));
  const double zb = (double)rs.nrep * rs.n1 * rs.n2 * rs.n3 * prec_bytes(prec);
  const double p1_bytes = zb + (double)rs.nrep * rs.R *
                                   ((double)rs.n3 * 8 + (double)rs.n1 * rs.n2 * acc_bytes(prec));
  const double p2_bytes =
      zb + (double)rs.nrep * rs.R * 8.0 * ((double)rs.n1 + rs.n2 + rs.n3);
  if (plain) {
    // one launch per step, three passes over the summary per sweep
    for (int it = 0; it < iters; ++it) {
      int pq = prof_kernel(t);
      SBT_CK(launch_p1(prec, rs, Zp, Cp, W, st));
      prof_end(t, pq, SBT_K_MTTKRP_C, p1_bytes, st);
      SBT_CK(launch_cw1(prec, rs, W, Bp, M, st));
      SBT_CK(launch_solve(rs, rs.n1, M, GB, rs.sG, GC, rs.sG, Ap, rs.sA, GA, lam_out, nullptr, 1,
                          t->pinv, st));
      pq = prof_kernel(t);
      SBT_CK(launch_p1(prec, rs, Zp, Cp, W, st));
      prof_end(t, pq, SBT_K_MTTKRP_C, p1_bytes, st);
      SBT_CK(launch_cw2(prec, rs, W, Ap, M, st));
      SBT_CK(launch_solve(rs, rs.n2, M, GA, rs.sG, GC, rs.sG, Bp, rs.sB, GB, lam_out, nullptr, 1,
                          t->pinv, st));
      pq = prof_kernel(t);
      SBT_CK(launch_p2(prec, rs, Zp, Ap, Bp, M, st));
      prof_end(t, pq, SBT_K_MTTKRP_AB, p2_bytes, st);
      SBT_CK(launch_solve(rs, rs.n3, M, GA, rs.sG, GB, rs.sG, Cp, rs.sC, GC, lam_out, nullptr, 1,
                          t->pinv, st));
    }
    return SBT_OK;
  }
  // batched: three launches per sweep over all repetitions.  Factors stay
  // unnormalised during the sweeps (1/lambda per column in invlam: A | B | C),
  // V^-1 for each step is prepared by the tail of the step before.
  const int R = rs.R;
  double* ilA = invlam;
  double* ilB = invlam + R;
  double* ilC = invlam + 2 * R;
  SBT_CK(launch_fill_f64(invlam + (int64_t)rs.rep0 * 3 * R, (int64_t)rs.nrep * 3 * R, 1.0, st));
  SBT_CK(launch_inverse(rs, GB, rs.sG, GC, rs.sG, Vinv, t->pinv, st));
  rs.nsplit = 1;  // pass W sums the whole third mode inside each block
  const double pw_bytes =
      zb + (double)rs.nrep * rs.R *
               ((double)rs.n3 * 8 + (double)rs.nsplit * rs.n1 * rs.n2 * acc_bytes(prec));
  // invlam is laid out per repetition as [A | B | C]: strides 3R, offset by mode
  AlsTail ta;
  ta.sG = rs.sG;
  ta.pinv_count = t->pinv;
  const bool mf = t->mfma && prec == kBF16;
  const int kp32 = (rs.n3 + 31) / 32 * 32;
  const int ns3 = mf ? mfma_mode3_splits(rs, t->ml) : 1;
  const double pwm_bytes = (double)rs.nrep * rs.n1 * rs.n2 * (kp32 * 2.0 + rs.R * 4.0) +
                           (double)rs.nrep * rs.n3 * rs.R * 8.0;
  // launch-shape keys of the two matrix-core passes (rank, summary rows,
  // repetitions: K' grows with every update and only scales the work) and
  // their units of work (summary elements read)
  const int64_t pw_key[4] = {rs.R, (int64_t)rs.n1 * rs.n2, rs.nrep, 0};
  const int64_t p3_key[4] = {rs.R, (int64_t)rs.n1 * rs.n2, rs.nrep, 0};
  const double mf_work = (double)rs.nrep * rs.n1 * rs.n2 * rs.n3;
  const double p3m_bytes = (double)rs.nrep * rs.n3 * t->ml.sk * 2.0 +
                           (double)rs.nrep * rs.R * 8.0 * ((double)rs.n1 + rs.n2) +
                           (double)rs.nrep * ns3 * rs.n3 * (rs.R <= 16 ? 16 : 32) * 4.0;
  // The sweep sequence of a summary CP-ALS depends only on the launch shape
  // (K', the repetition range, the sweep count): the second time a shape
  // comes round (persistent summaries with equal batches keep K' fixed) it
  // is captured into a HIP graph on the tensor's capture stream, and replayed
  // from then on.  Replays record no per-launch profiling events.
  const bool graphable = stream == kStreamAlsInit;
  const uint64_t gkey = ((uint64_t)(uint32_t)rs.n3 << 32) ^ ((uint64_t)rs.rep0 << 20) ^
                        ((uint64_t)rs.nrep << 8) ^ (uint64_t)iters;
  bool capture = false;
  if (graphable) {
    auto g = t->graphs.find(gkey);
    if (g != t->graphs.end() && g->second) {
      SBT_CK(hipGraphLaunch(g->second, st));
      SBT_CK(launch_normalize(rs, Ap, Bp, Cp, invlam, st));
      return SBT_OK;
    }
    if (g != t->graphs.end()) {
      capture = true;  // seen once before: capture this time
    } else {
      if (t->graphs.size() >= kGraphCache) {
        SBT_CK(hipStreamSynchronize(st));  // no replay of these graphs still running
        for (auto& kv : t->graphs)
          if (kv.second) (void)hipGraphExecDestroy(kv.second);
        t->graphs.clear();
      }
      t->graphs[gkey] = nullptr;
    }
  }
  hipStream_t lst = st;
  const bool prof_keep = t->prof_on;
  if (capture) {
    if (!t->capst) SBT_CK(hipStreamCreateWithFlags(&t->capst, hipStreamNonBlocking));
    SBT_CK(hipStreamBeginCapture(t->capst, hipStreamCaptureModeThreadLocal));
    lst = t->capst;
    t->prof_on = false;  // no event records inside the graph
  }
  auto sweeps = [&]() -> sbt_status {
    const hipStream_t st = lst;
  for (int it = 0; it < iters; ++it) {
    int pq = prof_kernel(t);
    if (mf) {
      const TuneSlot ts = tune_begin(kTunePw, SBT_TUNE_SHAPES, pw_key, mf_work, !capture, st);
      const hipError_t pw_mfma_launch =
          launch_pw_mfma(rs, t->ml, t->Zc, Cp, ilC, (float*)W, t->mops, st, ts.choice);
      if (pw_mfma_launch == hipSuccess) tune_end(ts, st); else tune_cancel(ts);
      SBT_CK(pw_mfma_launch);
      prof_end(t, pq, SBT_K_MTTKRP_C, pwm_bytes, st);
    } else {
      SBT_CK(launch_pw(prec, rs, Zp, Cp, ilC, W, st));
      prof_end(t, pq, SBT_K_MTTKRP_C, pw_bytes, st);
    }
    // mode 1: A (long factors: with the partial Gram matrices of its row blocks)
    const int64_t sgp = gram_part_stride(t);
    double* gpa = gram_parts_buf(t, rs, rs.n1);
    SBT_CK(launch_cw(prec, rs, 0, W, Bp, ilB, Vinv, Ap, rs.sA, st, nullptr, gpa, sgp));
    ta.U = Ap; ta.sU = rs.sA; ta.rows = rs.n1; ta.Gout = GA; ta.invlam_out = ilA;
    ta.lam_out = nullptr; ta.Gx = GA; ta.Gy = GC; ta.Vinv_out = Vinv;
    // mode 2: B, with the tail of mode 1 folded into its launch when A's rows
    // fit the tail's staging
    const bool fold = tail_rows_fit(rs.n1, R);
    if (!fold) SBT_TRY(tail(t, rs, ta, st, gpa));
    double* gpb = gram_parts_buf(t, rs, rs.n2);
    SBT_CK(launch_cw(prec, rs, 1, W, Ap, ilA, Vinv, Bp, rs.sB, st, fold ? &ta : nullptr, gpb,
                     sgp));
    ta.U = Bp; ta.sU = rs.sB; ta.rows = rs.n2; ta.Gout = GB; ta.invlam_out = ilB;
    ta.lam_out = nullptr; ta.Gx = GA; ta.Gy = GB; ta.Vinv_out = Vinv;
    SBT_TRY(tail(t, rs, ta, st, gpb));
    // mode 3: C (lambda' = its column norms)
    pq = prof_kernel(t);
    double* gpc = nullptr;
    if (mf) {
      const TuneSlot ts = tune_begin(kTuneP3, SBT_TUNE_SHAPES, p3_key, mf_work, !capture, st);
      const hipError_t p3_mfma_launch = launch_p3_mfma(
          rs, t->ml, ns3, t->Zk, Ap, ilA, Bp, ilB, t->P3, t->sP3, t->mops, st, ts.choice);
      if (p3_mfma_launch == hipSuccess) tune_end(ts, st); else tune_cancel(ts);
      SBT_CK(p3_mfma_launch);
      prof_end(t, pq, SBT_K_MTTKRP_AB, p3m_bytes, st);
      gpc = gram_parts_buf(t, rs, rs.n3);
      SBT_CK(launch_mode3_finish(rs, ns3, t->P3, t->sP3, Vinv, nullptr, Cp, rs.sC, st, gpc,
                                 sgp));
    } else {
      SBT_CK(launch_p3(prec, rs, false, Zp, Ap, ilA, Bp, ilB, Vinv, nullptr, Cp, rs.sC, st));
      prof_end(t, pq, SBT_K_MTTKRP_AB, p2_bytes, st);
    }
    ta.U = Cp; ta.sU = rs.sC; ta.rows = rs.n3; ta.Gout = GC; ta.invlam_out = ilC;
    ta.lam_out = lam_out; ta.Gx = GB; ta.Gy = GC; ta.Vinv_out = Vinv;
    SBT_TRY(tail(t, rs, ta, st, gpc));
  }
    return SBT_OK;
  };
  const sbt_status sw = sweeps();
  t->prof_on = prof_keep;
  if (capture) {
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(t->capst, &g);
    hipGraphExec_t ex = nullptr;
    hipError_t e2 = hipErrorUnknown;
    if (e == hipSuccess && sw == SBT_OK) e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (sw != SBT_OK) return sw;
    SBT_CK(e);
    SBT_CK(e2);
    t->graphs[gkey] = ex;
    SBT_CK(hipGraphLaunch(ex, st));
  } else if (sw != SBT_OK) {
    return sw;
  }
  SBT_CK(launch_normalize(rs, Ap, Bp, Cp, invlam, st));
  return SBT_OK;
}

sbt_status init_common(sbt_tensor* t, const double* A0, const double* B0, const double* C0,
                       const double* lam0, hipStream_t st) {
  const int R = t->R;
  SBT_CK(launch_fill_f64(t->ones, (int64_t)R * R, 1.0, st));
  SBT_CK(launch_fill_u32(t->pinv, 1, 0, st));
  SBT_CK(launch_fill_u32(t->cnt, 2 * (int64_t)t->cfg.repetitions, 0, st));
  if (A0) {
    SBT_CK(hipMemcpyAsync(t->A, A0, sizeof(double) * t->I * R, hipMemcpyHostToDevice, st));
    SBT_CK(hipMemcpyAsync(t->B, B0, sizeof(double) * t->J * R, hipMemcpyHostToDevice, st));
    SBT_CK(hipMemcpyAsync(t->C, C0, sizeof(double) * t->K * R, hipMemcpyHostToDevice, st));
    SBT_CK(hipMemcpyAsync(t->lam, lam0, sizeof(double) * R, hipMemcpyHostToDevice, st));
    SBT_CK(hipStreamSynchronize(st));
    return SBT_OK;
  }
  if (t->fmt != SBT_DENSE) {
    if (t->cfg.init_iters < 1) {
      set_err(t, "the initial CP-ALS needs init_iters >= 1");
      return SBT_E_INVALID;
    }
    return init_cp_als_coo(t, st);
  }
  // CP-ALS on the whole initial tensor, then components ordered by lambda.
  RepSet rs;
  rs.n1 = (int)t->I;
  rs.n2 = (int)t->J;
  rs.n3 = (int)t->K;
  rs.R = R;
  rs.rep0 = 0;
  rs.nrep = 1;
  rs.sZ = 0;
  rs.sA = t->I * R;
  rs.sB = t->J * R;
  rs.sC = t->K * R;
  rs.nsplit = 1;
  rs.sW = t->I * t->J * R;
  int64_t mx = t->I > t->J ? t->I : t->J;
  if (t->K > mx) mx = t->K;
  rs.sM = mx * R;
  rs.sG = (int64_t)R * R;
  void* W = nullptr;
  double *M = nullptr, *G = nullptr;
  const size_t wbytes = (size_t)rs.sW * acc_bytes(t->store_prec);
  SBT_CK(hipMalloc(&W, wbytes));
  hipError_t e1 = hipMalloc((void**)&M, sizeof(double) * rs.sM);
  hipError_t e2 = hipMalloc((void**)&G, sizeof(double) * 3 * rs.sG);
  sbt_status s = SBT_OK;
  if (e1 != hipSuccess || e2 != hipSuccess) {
    set_err(t, "hipMalloc failed for the initial CP-ALS workspace");
    s = SBT_E_NOMEM;
  } else {
    const int keep = t->sum_prec;
    t->sum_prec = t->store_prec;  // the whole tensor is read in its stored precision
    // the batched mode-3 kernel stages both whole factors in LDS; wider
    // tensors take the one-launch-per-step schedule (the same ALS sweeps)
    const bool plain = !p3_fits(t->sum_prec, rs.n1, rs.n2, R);
    s = run_als(t, t->X, rs, t->A, t->B, t->C, G, G + rs.sG, G + 2 * rs.sG, t->lam, W, M,
                t->Vinv, t->invlam, kStreamInit, 0u, t->cfg.init_iters, plain, st);
    t->sum_prec = keep;
    if (s == SBT_OK && t->cfg.init_iters == 0) s = SBT_E_INVALID;
    if (s == SBT_OK) {
      hipError_t e = launch_sort_components(t->A, t->B, t->C, t->lam, t->I, t->J, t->K, R, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        set_err(t, std::string("initial CP-ALS: ") + hipGetErrorString(e));
        s = SBT_E_DEVICE;
      }
    }
  }
  (void)hipStreamSynchronize(st);
  (void)hipFree(W);
  if (M) (void)hipFree(M);
  if (G) (void)hipFree(G);
  return s;
}

void free_all(sbt_tensor* t) {
  if (!t->graphs.empty()) (void)hipDeviceSynchronize();
  for (auto& kv : t->graphs)
    if (kv.second) (void)hipGraphExecDestroy(kv.second);
  t->graphs.clear();
  if (t->capst) (void)hipStreamDestroy(t->capst);
  t->capst = nullptr;
  for (auto& g : t->grow_allocs) (void)hipFree(g.first);
  t->grow_allocs.clear();
  for (hipEvent_t e : t->prof_ev) (void)hipEventDestroy(e);
  t->prof_ev.clear();
  for (void* p : t->allocs) (void)hipFree(p);
  t->allocs.clear();
  if (t->h_err) (void)hipHostFree(t->h_err);
  t->h_err = nullptr;
}

sbt_status check_factor_args(const double* A0, const double* B0, const double* C0,
                             const double* lam0, std::string& why) {
  const int n = (A0 != nullptr) + (B0 != nullptr) + (C0 != nullptr) + (lam0 != nullptr);
  if (n != 0 && n != 4) {
    why = "pass all of A0, B0, C0, lambda0 or none";
    return SBT_E_INVALID;
  }
  return SBT_OK;
}

// The update after the batch is in the store and its importance is in dw*.
// GetRank (Sec. 3.2) on the summaries of rs: every candidate rank i = 1..R
// gets getrank_runs CP-ALS runs (initial factors from the GetRank stream, run
// q = (i - 1) runs + j at columns 32 q of the counter), each scored by its
// core consistency; the kept run per repetition ends in Ap, Bp, Cp, lamp (rows
// padded to R columns) and its rank in grnew.  Dense summaries get the
// projected core through Z x3 C^T, COO summaries through their third-mode
// slices (the sparse form of the diagnostic the paper uses).
sbt_status getrank_search(sbt_tensor* t, const RepSet& rs, bool plain, hipStream_t st) {
  const sbt_config& c = t->cfg;
  const int R = t->R, runs = c.getrank_runs;
  const int64_t R3 = (int64_t)R * R * R;
  const int64_t sGi = (int64_t)c.repetitions * rs.sG;
  const bool coo = t->fmt == SBT_COO;
  for (int i = 1; i <= R; ++i) {
    RepSet ri = rs;
    ri.R = i;  // strides stay those of rank R
    SBT_CK(launch_fill_f64(t->gbest + rs.rep0, rs.nrep, -1.0e308, st));
    for (int j = 0; j < runs; ++j) {
      const uint32_t q = (uint32_t)((i - 1) * runs + j);
      if (coo)
        SBT_TRY(run_als_coo(t, ri, t->t, st, kStreamGetRank, 32u * q));
      else
        SBT_TRY(run_als(t, t->Z, ri, t->Ap, t->Bp, t->Cp, t->GA, t->GB, t->GC, t->lamp, t->W,
                        t->M, t->Vinv, t->invlam, kStreamGetRank, t->t, c.als_iters, plain, st,
                        32u * q));
      // Grams of the unit-column factors and their inverses
      SBT_TRY(gram_rows(t, ri, t->Ap, ri.sA, ri.n1, t->GA, st));
      SBT_TRY(gram_rows(t, ri, t->Bp, ri.sB, ri.n2, t->GB, st));
      SBT_TRY(gram_rows(t, ri, t->Cp, ri.sC, ri.n3, t->GC, st));
      SBT_CK(launch_inverse(ri, t->GA, ri.sG, t->ones, 0, t->gGi, t->pinv, st));
      SBT_CK(launch_inverse(ri, t->GB, ri.sG, t->ones, 0, t->gGi + sGi, t->pinv, st));
      SBT_CK(launch_inverse(ri, t->GC, ri.sG, t->ones, 0, t->gGi + 2 * sGi, t->pinv, st));
      // the projected core (dense: W = Z x3 C^T first), the core consistency
      if (coo) {
        SBT_CK(launch_core_coo(ri, t->z.a, t->z.b, t->z.v, t->z.offC, t->z.sOffC, t->Ap, t->Bp,
                               t->Cp, t->gWz, (int64_t)t->Kpmax * R * R, t->gP, R3, st));
      } else {
        SBT_CK(launch_p1(t->sum_prec, ri, t->Z, t->Cp, t->W, st));
        SBT_CK(launch_core(t->sum_prec, ri, t->W, t->Ap, t->Bp, t->gP, R3, st));
      }
      SBT_CK(launch_corcondia(ri, t->gP, t->gX1, t->gX2, R3, t->gGi, sGi, t->lamp, t->gcc, st));
      SBT_CK(launch_rank_select(ri, R, runs, j, i == 1 && j == 0, c.getrank_threshold, t->gcc,
                                t->gbest, t->gtab, t->grnew, t->Ap, t->Bp, t->Cp, t->lamp,
                                t->gAk, t->gBk, t->gCk, t->glamk, st));
    }
  }
  const size_t d = sizeof(double);
  SBT_CK(hipMemcpyAsync(t->Ap + rs.rep0 * rs.sA, t->gAk + rs.rep0 * rs.sA, d * rs.nrep * rs.sA,
                        hipMemcpyDeviceToDevice, st));
  SBT_CK(hipMemcpyAsync(t->Bp + rs.rep0 * rs.sB, t->gBk + rs.rep0 * rs.sB, d * rs.nrep * rs.sB,
                        hipMemcpyDeviceToDevice, st));
  SBT_CK(hipMemcpyAsync(t->Cp + rs.rep0 * rs.sC, t->gCk + rs.rep0 * rs.sC, d * rs.nrep * rs.sC,
                        hipMemcpyDeviceToDevice, st));
  SBT_CK(hipMemcpyAsync(t->lamp + (int64_t)rs.rep0 * R, t->glamk + (int64_t)rs.rep0 * R,
                        d * rs.nrep * R, hipMemcpyDeviceToDevice, st));
  return SBT_OK;
}

sbt_status update_body(sbt_tensor* t, int64_t Kn, int uq, hipStream_t st) {
  const sbt_config& c = t->cfg;
  const int R = t->R, r = c.repetitions;
  const int64_t Kold = t->K;
  // persistent summaries keep the sampled indices (and so K_s and its size)
  const bool reuse = c.persist_summaries && t->have_kept &&
                     !(c.summary_refresh > 0 && t->t % (uint32_t)c.summary_refresh == 0);
  const int n3old = reuse ? t->n3kept : (int)sample_size(Kold, c.sample_factor[2]);
  const int Kp = n3old + (int)Kn;
  // sampling (from the tensor before the update)
  SampleArgs sa{};
  sa.w[0] = t->w1;
  sa.w[1] = t->w2;
  sa.w[2] = t->w3;
  sa.N[0] = t->I;
  sa.N[1] = t->J;
  sa.N[2] = Kold;
  sa.n[0] = t->n1;
  sa.n[1] = t->n2;
  sa.n[2] = n3old;
  sa.key_off[0] = 0;
  sa.key_off[1] = t->I;
  sa.key_off[2] = t->I + t->J;
  sa.key_stride = t->key_stride;
  sa.idx_off[0] = 0;
  sa.idx_off[1] = t->n1;
  sa.idx_off[2] = (int64_t)t->n1 + t->n2;
  sa.idx_stride = t->idx_stride;
  sa.seed = c.seed;
  sa.tensor_id = c.tensor_id;
  sa.t = t->t;
  sa.nrep = r;
  if (!reuse) SBT_CK(launch_sample(sa, t->keys, t->idx, st));
  const int64_t offJ = t->n1, offK = (int64_t)t->n1 + t->n2;
  RepSet all = make_repset(t, Kp, 0, r);
  const bool plain = c.schedule == SBT_SCHED_PLAIN;
  // a kept summary's old part (the K_s slices) is still in place from the
  // update before, which used the same indices: only the new slices are gathered
  const int c0 = (reuse && t->z_kept) ? n3old : 0;
  if (t->mfma) {
    const int gq = prof_kernel(t);
    // (a kept summary's gather reads only the new slices: a key of its own)
    const int64_t gkey[4] = {t->store_prec, (int64_t)t->n1 * t->n2, r, c0 > 0 ? 1 : 0};
    const TuneSlot ts = tune_begin(kTuneGather, SBT_TUNE_SHAPES, gkey,
                                   (double)r * t->n1 * t->n2 * (Kp - c0), true, st);
    const hipError_t gather_mfma_launch =
        launch_gather_mfma(t->store_prec, t->X, t->I, t->J, t->idx, t->idx_stride, offJ, offK,
                           n3old, Kold, c0, all, t->ml, t->Zk, t->Zc, st, ts.choice);
    if (gather_mfma_launch == hipSuccess) tune_end(ts, st); else tune_cancel(ts);
    SBT_CK(gather_mfma_launch);
    prof_end(t, gq, SBT_K_GATHER,
             (double)r * t->n1 * t->n2 * (Kp - c0) * (prec_bytes(t->store_prec) + 4.0), st);
  } else if (t->fmt == SBT_DENSE) {
    const int gq = prof_kernel(t);
    SBT_CK(launch_gather_dense(t->store_prec, t->sum_prec, t->X, t->I, t->J, t->idx,
                               t->idx_stride, offJ, offK, n3old, Kold, c0, all, t->Z, st));
    prof_end(t, gq, SBT_K_GATHER,
             (double)r * t->n1 * t->n2 * (Kp - c0) *
                 (prec_bytes(t->store_prec) + prec_bytes(t->sum_prec)),
             st);
  } else {
    if (!reuse) t->coo_kept = false;
    SBT_TRY(coo_build_summaries(t, Kold, n3old, Kp, reuse && t->coo_kept, st));
  }
  // the summaries now hold X(I_s, J_s, K_s) for the indices in idx
  t->z_kept = t->fmt == SBT_DENSE;
  const bool coo = t->fmt == SBT_COO;
  const int nchunks = (plain && !coo) ? r : 1;
  t->warm_now = reuse;  // read by the summary CP-ALS initialisation
  t->warm_n3 = n3old;
  for (int q = 0; q < nchunks; ++q) {
    RepSet rs = (plain && !coo) ? make_repset(t, Kp, q, 1) : all;
    if (c.getrank_runs > 0) {
      SBT_TRY(getrank_search(t, rs, plain, st));
    } else if (coo) {
      SBT_TRY(run_als_coo(t, rs, t->t, st));
    } else {
      SBT_TRY(run_als(t, t->Z, rs, t->Ap, t->Bp, t->Cp, t->GA, t->GB, t->GC, t->lamp, t->W,
                      t->M, t->Vinv, t->invlam, kStreamAlsInit, t->t, c.als_iters, plain, st));
    }
    MatchArgs ma;
    ma.A = t->A;
    ma.B = t->B;
    ma.C = t->C;
    ma.idx = t->idx;
    ma.idx_stride = t->idx_stride;
    ma.offJ = offJ;
    ma.offK = offK;
    ma.n3old = n3old;
    ma.Ap = t->Ap;
    ma.Bp = t->Bp;
    ma.Cp = t->Cp;
    ma.At = t->At;
    ma.Bt = t->Bt;
    ma.Gt = t->Gt;
    ma.pi = t->pi;
    ma.valid = t->valid;
    ma.xo = t->xout;
    ma.scl = t->scl;
    ma.rnew = c.getrank_runs > 0 ? t->grnew : nullptr;
    {
      // anchor and sample cross products over the sampled rows
      const int32_t* Is = t->idx;
      const int32_t* Js = t->idx + offJ;
      const int32_t* Ks = t->idx + offK;
      const int64_t is = t->idx_stride;
      XProd xp{};
      xp.job[0] = XJob{t->A, 0, Is, is, t->Ap, rs.sA, nullptr, 0, rs.n1};
      xp.job[1] = XJob{t->B, 0, Js, is, t->Bp, rs.sB, nullptr, 0, rs.n2};
      xp.job[2] = XJob{t->C, 0, Ks, is, t->Cp, rs.sC, nullptr, 0, n3old};
      xp.job[3] = XJob{t->A, 0, Is, is, t->A, 0, Is, is, rs.n1};
      xp.job[4] = XJob{t->B, 0, Js, is, t->B, 0, Js, is, rs.n2};
      xp.job[5] = XJob{t->C, 0, Ks, is, t->C, 0, Ks, is, n3old};
      xp.job[6] = XJob{t->Ap, rs.sA, nullptr, 0, t->Ap, rs.sA, nullptr, 0, rs.n1};
      xp.job[7] = XJob{t->Bp, rs.sB, nullptr, 0, t->Bp, rs.sB, nullptr, 0, rs.n2};
      xp.job[8] = XJob{t->Cp, rs.sC, nullptr, 0, t->Cp, rs.sC, nullptr, 0, n3old};
      xp.njobs = 9;
      xp.R = R;
      xp.rep0 = rs.rep0;
      xp.nrep = rs.nrep;
      xp.nblk = t->xnblk;
      xp.part = t->xpart;
      xp.out = t->xout;
      SBT_CK(launch_xprod(xp, st));
    }
    SBT_CK(launch_match(rs, ma, st));
    if (t->lhat)
      SBT_CK(launch_lambda_hat(rs, t->xout, t->lamp, t->pi, t->valid, t->lhat, st));
    // row least squares: D = Z_(3) (Bt kr At) Gt^-1, C~ = D / lambda
    // Gt is already the Hadamard product; the second factor is all ones
    const double rbytes = (double)rs.nrep * rs.n1 * rs.n2 * rs.n3 * prec_bytes(t->sum_prec) +
                          (double)rs.nrep * rs.R * 8.0 * ((double)rs.n1 + rs.n2 + rs.n3);
    const int rq = prof_kernel(t);
    if (coo) {
      SBT_CK(launch_inverse(rs, t->Gt, rs.sG, t->ones, 0, t->Vinv, t->pinv, st));
      SBT_CK(launch_coo_prep(rs, rs.n1, t->At, rs.sA, nullptr, t->fA, st));
      SBT_CK(launch_coo_prep(rs, rs.n2, t->Bt, rs.sB, nullptr, t->fB, st));
      SBT_CK(launch_coo_units(rs, 2, t->z, t->cu[2], t->fA, rs.n1, t->fB, rs.n2, t->upart,
                              (double)t->last_summary_nnz / ((double)t->cfg.repetitions * rs.n3),
                              st));
      prof_end(t, rq, SBT_K_COO_MTTKRP, (double)t->last_summary_nnz * 12.0, st);
      SBT_CK(launch_coo_units_finish(rs, 2, t->cu[2], t->upart, t->Vinv, t->lam, t->Ct, rs.sC,
                                     st));
    } else if (plain) {
      SBT_CK(launch_p2(t->sum_prec, rs, t->Z, t->At, t->Bt, t->M, st));
      prof_end(t, rq, SBT_K_ROW_SOLVE, rbytes, st);
      SBT_CK(launch_solve(rs, Kp, t->M, t->Gt, rs.sG, t->ones, 0, t->Ct, rs.sC, nullptr, nullptr,
                          t->lam, 0, t->pinv, st));
    } else if (t->mfma) {
      SBT_CK(launch_inverse(rs, t->Gt, rs.sG, t->ones, 0, t->Vinv, t->pinv, st));
      const int ns3 = mfma_mode3_splits(rs, t->ml);
      SBT_CK(launch_p3_mfma(rs, t->ml, ns3, t->Zk, t->At, nullptr, t->Bt, nullptr, t->P3, t->sP3,
                            t->mops, st));
      SBT_CK(launch_mode3_finish(rs, ns3, t->P3, t->sP3, t->Vinv, t->lam, t->Ct, rs.sC, st));
      prof_end(t, rq, SBT_K_ROW_SOLVE, rbytes, st);
    } else {
      // V^-1 = Gt^-1, then one launch: rows of C~ = (Z_(3) (Bt kr At)) Gt^-1 / lambda
      SBT_CK(launch_inverse(rs, t->Gt, rs.sG, t->ones, 0, t->Vinv, t->pinv, st));
      SBT_CK(launch_p3(t->sum_prec, rs, true, t->Z, t->At, nullptr, t->Bt, nullptr, t->Vinv,
                       t->lam, t->Ct, rs.sC, st));
      prof_end(t, rq, SBT_K_ROW_SOLVE, rbytes, st);
    }
  }
  t->warm_now = false;
  CommitArgs ca;
  ca.err = t->err;
  ca.A = t->A;
  ca.B = t->B;
  ca.C = t->C;
  ca.I = t->I;
  ca.J = t->J;
  ca.Kold = Kold;
  ca.Knew = Kn;
  ca.R = R;
  ca.nrep = r;
  ca.n1 = t->n1;
  ca.n2 = t->n2;
  ca.n3old = n3old;
  ca.Kp = Kp;
  ca.idx = t->idx;
  ca.idx_stride = t->idx_stride;
  ca.offJ = offJ;
  ca.offK = offK;
  ca.At = t->At;
  ca.Bt = t->Bt;
  ca.Ct = t->Ct;
  ca.sA = all.sA;
  ca.sB = all.sB;
  ca.sC = all.sC;
  ca.valid = t->valid;
  ca.w1 = t->w1;
  ca.w2 = t->w2;
  ca.w3 = t->w3;
  ca.dw1 = t->dw1;
  ca.dw2 = t->dw2;
  ca.dw3 = t->dw3;
  SBT_CK(launch_commit(ca, st));
  if (t->lhat) SBT_CK(launch_lambda_avg(t->err, t->lam, t->lhat, r, R, st));
  prof_end(t, uq, SBT_K_UPDATE, 0.0, st);
  SBT_CK(hipMemcpyAsync(t->h_err, t->err, 4, hipMemcpyDeviceToHost, st));
  SBT_CK(hipStreamSynchronize(st));
  prof_collect(t);
  if (*t->h_err) {
    t->pending_nnz = 0;
    set_err(t, (*t->h_err & 2u)
                   ? "batch coordinate outside the tensor"
                   : "batch holds a non-finite value or overflows the importance sums");
    return (*t->h_err & 2u) ? SBT_E_SHAPE : SBT_E_NUMERIC;
  }
  if (c.persist_summaries) {
    // keep this update's summary factors for the next warm start
    const RepSet ks = make_repset(t, Kp, 0, r);
    SBT_CK(hipMemcpyAsync(t->Bw, t->Bp, sizeof(double) * r * ks.sB, hipMemcpyDeviceToDevice, st));
    SBT_CK(hipMemcpyAsync(t->Cw, t->Cp, sizeof(double) * r * ks.sC, hipMemcpyDeviceToDevice, st));
    SBT_CK(hipStreamSynchronize(st));
    t->have_kept = true;
    t->n3kept = n3old;
    t->coo_kept = t->fmt == SBT_COO;
  }
  t->K = Kold + Kn;
  t->t += 1;
  t->nnz += t->pending_nnz;
  t->pending_nnz = 0;
  t->has_last = true;
  t->last_n3old = n3old;
  t->last_Kp = Kp;
  return SBT_OK;
}

// tensors of order N: the N-mode part at the end of this file
sbt_status nd_update(sbt_tensor* t, const void* Y_dev, int64_t Kn, hipStream_t st);
sbt_status nd_fit(sbt_tensor* t, double* fit, hipStream_t st);
void nd_release(sbt_tensor* t);
bool nd_sample_span(const sbt_tensor* t, int mode, int64_t* off, int64_t* cnt);

// One call at a time on a tensor: a second concurrent call, or a direct call
// on a tensor a server holds requests of, gets SBT_E_BUSY (the first keeps
// running; the tensor's error message is left alone).
struct CallGuard {
  sbt_tensor* t;
  bool ok = false;
  CallGuard(sbt_tensor* tt, bool from_server) : t(tt) {
    if (!from_server && t->leases.load() > 0) return;
    ok = !t->busy.exchange(true);
  }
  ~CallGuard() {
    if (ok) t->busy.store(false);
  }
  CallGuard(const CallGuard&) = delete;
  CallGuard& operator=(const CallGuard&) = delete;
};

// Message of the last failure of a call that has no tensor to record it on
// (sbt_load, the stand-alone kernels), per host thread.
thread_local std::string g_errmsg;

// device bytes of the store, the model and the importance vectors
size_t resident_bytes(const sbt_tensor* t) {
  const size_t R = (size_t)t->R;
  size_t b = ((size_t)t->I + t->J + t->Kcap) * (R + 1) * 8 + R * 8;
  if (t->fmt == SBT_DENSE) b += (size_t)t->I * t->J * t->Kcap * prec_bytes(t->store_prec);
  else b += (size_t)t->nnz_cap * 16;
  return b;
}

// ---- checkpoint files ---------------------------------------------------
// Little-endian binary: the header below, then the arrays in the order of
// ckpt_arrays(), each as raw bytes (device layout).
constexpr char kCkptMagic[8] = {'S', 'B', 'T', 'C', 'K', 'P', 'T', '1'};
constexpr uint32_t kCkptVersion = 1;

struct CkptHeader {
  char magic[8];
  uint32_t version, header_bytes;
  sbt_config cfg;
  int64_t I, J, K, Kcap, nnz;
  int32_t R, fmt, store_prec, sum_prec, S;
  uint32_t t;
  uint64_t nmax;
  int32_t have_kept, n3kept;
  uint64_t payload_bytes;
};

struct CkptArray {
  void* dev;
  size_t bytes;
};

// The state a checkpoint holds: the stored tensor, the model, the importance
// and, for persistent summaries, the kept indices and warm-start factors.
std::vector<CkptArray> ckpt_arrays(sbt_tensor* t, bool have_kept) {
  const size_t R = (size_t)t->R, K = (size_t)t->K;
  std::vector<CkptArray> a;
  if (t->fmt == SBT_DENSE) {
    a.push_back({t->X, (size_t)t->I * t->J * K * prec_bytes(t->store_prec)});
  } else {
    const size_t n = (size_t)t->nnz;
    a.push_back({t->ci, n * 4});
    a.push_back({t->cj, n * 4});
    a.push_back({t->ck, n * 4});
    a.push_back({t->cv, n * 4});
    a.push_back({t->koff, (K + 1) * 8});
  }
  a.push_back({t->A, (size_t)t->I * R * 8});
  a.push_back({t->B, (size_t)t->J * R * 8});
  a.push_back({t->C, K * R * 8});
  a.push_back({t->lam, R * 8});
  a.push_back({t->w1, (size_t)t->I * 8});
  a.push_back({t->w2, (size_t)t->J * 8});
  a.push_back({t->w3, K * 8});
  if (have_kept) {
    const int r = t->cfg.repetitions;
    const RepSet rs = make_repset(t, t->Kpmax, 0, r);
    a.push_back({t->idx, (size_t)r * t->idx_stride * 4});
    a.push_back({t->Bw, (size_t)r * rs.sB * 8});
    a.push_back({t->Cw, (size_t)r * rs.sC * 8});
  }
  return a;
}

// Copies between device arrays and a file through a pinned staging buffer.
struct CkptIO {
  FILE* f = nullptr;
  void* stage = nullptr;
  size_t cap = size_t(64) << 20;
  hipStream_t st = nullptr;
  ~CkptIO() {
    if (stage) (void)hipHostFree(stage);
    if (f) fclose(f);
  }
  bool open(const char* path, const char* mode) {
    f = fopen(path, mode);
    return f && hipHostMalloc(&stage, cap, hipHostMallocDefault) == hipSuccess;
  }
  bool put(const void* dev, size_t n) {
    for (size_t off = 0; off < n; off += cap) {
      const size_t m = n - off < cap ? n - off : cap;
      if (hipMemcpyAsync(stage, (const char*)dev + off, m, hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess || fwrite(stage, 1, m, f) != m)
        return false;
    }
    return true;
  }
  bool get(void* dev, size_t n) {
    for (size_t off = 0; off < n; off += cap) {
      const size_t m = n - off < cap ? n - off : cap;
      if (fread(stage, 1, m, f) != m ||
          hipMemcpyAsync((char*)dev + off, stage, m, hipMemcpyHostToDevice, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return false;
    }
    return true;
  }
};

sbt_status not_for_nd(sbt_tensor* t) {
  set_err(t, "tensor of order N: use the sbt_nd_* calls");
  return SBT_E_STATE;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* sbt_status_str(sbt_status s) {
  switch (s) {
    case SBT_OK: return "ok";
    case SBT_E_INVALID: return "invalid argument";
    case SBT_E_SHAPE: return "shape mismatch or capacity exceeded";
    case SBT_E_NOMEM: return "out of device memory";
    case SBT_E_DEVICE: return "HIP runtime error";
    case SBT_E_NUMERIC: return "non-finite input or importance overflow";
    case SBT_E_STATE: return "invalid state";
    case SBT_E_BUSY: return "another call on this tensor is in flight";
  }
  return "unknown status";
}

const char* sbt_last_error(const sbt_tensor* t) {
  return t ? t->errmsg.c_str() : g_errmsg.c_str();
}

sbt_status sbt_init_dense(const sbt_config* cfg, const void* X0_dev, int64_t I, int64_t J,
                          int64_t K0, const double* A0, const double* B0, const double* C0,
                          const double* lambda0, void* stream, sbt_tensor** out) {
  g_errmsg.clear();
  if (!out) return SBT_E_INVALID;
  *out = nullptr;
  std::string why;
  if (validate_config(cfg, why) != SBT_OK) return SBT_E_INVALID;
  if (cfg->format != SBT_DENSE || !X0_dev) return SBT_E_INVALID;
  if (check_factor_args(A0, B0, C0, lambda0, why) != SBT_OK) return SBT_E_INVALID;
  if (I < 1 || J < 1 || K0 < 1 || I > INT32_MAX || J > INT32_MAX) return SBT_E_SHAPE;
  if (cfg->k_capacity < K0 + 1) return SBT_E_SHAPE;
  sbt_tensor* t = new (std::nothrow) sbt_tensor();
  if (!t) return SBT_E_NOMEM;
  t->cfg = *cfg;
  t->I = I;
  t->J = J;
  t->K = K0;
  t->Kcap = cfg->k_capacity;
  t->R = cfg->rank;
  t->fmt = SBT_DENSE;
  t->store_prec = cfg->precision == SBT_P_F64 ? kF64 : kF32;
  t->sum_prec = cfg->precision == SBT_P_F64 ? kF64 : (cfg->precision == SBT_P_F32 ? kF32 : kBF16);
  int64_t nm = J * t->Kcap;
  if (I * t->Kcap > nm) nm = I * t->Kcap;
  if (I * J > nm) nm = I * J;
  t->nmax = (uint64_t)nm;
  hipStream_t st = (hipStream_t)stream;
  const size_t esz = prec_bytes(t->store_prec);
  sbt_status s = dalloc_bytes(t, &t->X, (size_t)I * J * t->Kcap * esz);
  if (s == SBT_OK) s = alloc_state(t);
  if (s == SBT_OK) {
    hipError_t e = hipMemcpyAsync(t->X, X0_dev, (size_t)I * J * K0 * esz,
                                  hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = launch_maxsq_dense(t->store_prec, t->X, I * J * K0, t->bits, st);
    if (e != hipSuccess) {
      set_err(t, hipGetErrorString(e));
      s = SBT_E_DEVICE;
    }
  }
  if (s == SBT_OK) s = set_scale(t, st);
  if (s == SBT_OK) {
    hipError_t e = launch_fill_u64(t->w1, I, 0, st);
    if (e == hipSuccess) e = launch_fill_u64(t->w2, J, 0, st);
    if (e == hipSuccess) e = launch_fill_u64(t->w3, K0, 0, st);
    if (e == hipSuccess) e = launch_fill_u32(t->err, 1, 0, st);
    if (e == hipSuccess)
      e = launch_moi_dense(t->store_prec, t->X, I, J, K0, t->scale, t->qmax, t->w1, t->w2, t->w3,
                           t->err, st);
    if (e == hipSuccess) e = hipMemcpyAsync(t->h_err, t->err, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      set_err(t, hipGetErrorString(e));
      s = SBT_E_DEVICE;
    } else if (*t->h_err) {
      set_err(t, "initial tensor holds a non-finite value or overflows the importance sums");
      s = SBT_E_NUMERIC;
    }
  }
  if (s == SBT_OK) s = init_common(t, A0, B0, C0, lambda0, st);
  if (s != SBT_OK) {
    g_errmsg = t->errmsg;  // the tensor is gone: sbt_last_error(NULL) keeps it
    free_all(t);
    delete t;
    return s;
  }
  *out = t;
  return SBT_OK;
}

sbt_status sbt_init_coo(const sbt_config* cfg, const int32_t* i_dev, const int32_t* j_dev,
                        const int32_t* k_dev, const float* v_dev, int64_t nnz, int64_t I,
                        int64_t J, int64_t K0, const double* A0, const double* B0,
                        const double* C0, const double* lambda0, void* stream,
                        sbt_tensor** out) {
  g_errmsg.clear();
  if (!out) return SBT_E_INVALID;
  *out = nullptr;
  std::string why;
  if (validate_config(cfg, why) != SBT_OK) return SBT_E_INVALID;
  if (cfg->format != SBT_COO) return SBT_E_INVALID;
  if (cfg->repetitions > 64) return SBT_E_INVALID;  // per index repetition bitmasks
  if (check_factor_args(A0, B0, C0, lambda0, why) != SBT_OK) return SBT_E_INVALID;
  if (nnz < 0 || (nnz > 0 && (!i_dev || !j_dev || !k_dev || !v_dev))) return SBT_E_INVALID;
  if (I < 1 || J < 1 || K0 < 1 || I > INT32_MAX || J > INT32_MAX) return SBT_E_SHAPE;
  if (cfg->k_capacity < K0 + 1 || cfg->k_capacity > INT32_MAX) return SBT_E_SHAPE;
  if (cfg->nnz_capacity < nnz || cfg->nnz_capacity > INT32_MAX) return SBT_E_SHAPE;
  sbt_tensor* t = new (std::nothrow) sbt_tensor();
  if (!t) return SBT_E_NOMEM;
  t->cfg = *cfg;
  t->I = I;
  t->J = J;
  t->K = K0;
  t->Kcap = cfg->k_capacity;
  t->R = cfg->rank;
  t->fmt = SBT_COO;
  t->store_prec = kF32;
  t->sum_prec = kF32;
  t->nnz_cap = cfg->nnz_capacity;
  int64_t nm = J * t->Kcap;
  if (I * t->Kcap > nm) nm = I * t->Kcap;
  if (I * J > nm) nm = I * J;
  if (t->nnz_cap < nm) nm = t->nnz_cap;
  t->nmax = (uint64_t)(nm < 1 ? 1 : nm);
  hipStream_t st = (hipStream_t)stream;
  sbt_status s = dalloc(t, &t->ci, (size_t)t->nnz_cap);
  if (s == SBT_OK) s = dalloc(t, &t->cj, (size_t)t->nnz_cap);
  if (s == SBT_OK) s = dalloc(t, &t->ck, (size_t)t->nnz_cap);
  if (s == SBT_OK) s = dalloc(t, &t->cv, (size_t)t->nnz_cap);
  if (s == SBT_OK) s = alloc_state(t);
  // summary rows are sorted under 24-bit keys (repetition in the high bits)
  if (s == SBT_OK && (t->n1 >= (1 << 24) || t->n2 >= (1 << 24))) {
    set_err(t, "sampled rows per mode must stay below 2^24");
    s = SBT_E_SHAPE;
  }
  if (s == SBT_OK) {
    hipError_t e = launch_maxsq_coo(v_dev, nnz, t->bits, st);
    if (e != hipSuccess) {
      set_err(t, hipGetErrorString(e));
      s = SBT_E_DEVICE;
    }
  }
  if (s == SBT_OK) s = set_scale(t, st);
  if (s == SBT_OK) {
    hipError_t e = launch_fill_u64(t->w1, I, 0, st);
    if (e == hipSuccess) e = launch_fill_u64(t->w2, J, 0, st);
    if (e == hipSuccess) e = launch_fill_u64(t->w3, K0, 0, st);
    if (e == hipSuccess) e = launch_fill_u32(t->err, 1, 0, st);
    if (e == hipSuccess)
      e = launch_moi_coo(i_dev, j_dev, k_dev, v_dev, nnz, I, J, K0, t->scale, t->qmax, t->w1,
                         t->w2, t->w3, t->err, st);
    if (e == hipSuccess) e = hipMemcpyAsync(t->h_err, t->err, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      set_err(t, hipGetErrorString(e));
      s = SBT_E_DEVICE;
    } else if (*t->h_err) {
      set_err(t, (*t->h_err & 2u) ? "coordinate outside the tensor"
                                  : "non-finite value or importance overflow");
      s = (*t->h_err & 2u) ? SBT_E_SHAPE : SBT_E_NUMERIC;
    }
  }
  if (s == SBT_OK) s = ensure_ingest(t, nnz, st);
  if (s == SBT_OK) {
    hipError_t e = launch_fill_u64((uint64_t*)t->koff, 1, 0, st);
    if (e == hipSuccess)
      e = launch_coo_ingest(i_dev, j_dev, k_dev, v_dev, nnz, K0, 0, t->ci, t->cj, t->ck, t->cv, 0,
                            t->koff, t->ing, st);
    if (e != hipSuccess) {
      set_err(t, hipGetErrorString(e));
      s = SBT_E_DEVICE;
    }
    t->nnz = nnz;
  }
  if (s == SBT_OK) s = init_common(t, A0, B0, C0, lambda0, st);
  if (s != SBT_OK) {
    g_errmsg = t->errmsg;  // the tensor is gone: sbt_last_error(NULL) keeps it
    free_all(t);
    delete t;
    return s;
  }
  *out = t;
  return SBT_OK;
}

void sbt_destroy(sbt_tensor* t) {
  if (!t) return;
  (void)hipDeviceSynchronize();
  free_all(t);
  nd_release(t);
  delete t;
}

}  // extern "C"

namespace {

sbt_status update_dense_body(sbt_tensor* t, const void* Y_dev, int64_t K_new, void* stream) {
  if (t->nd) return nd_update(t, Y_dev, K_new, (hipStream_t)stream);
  if (t->fmt != SBT_DENSE) {
    set_err(t, "tensor is not dense");
    return SBT_E_STATE;
  }
  if (K_new < 1 || K_new > t->cfg.max_batch || t->K + K_new > t->Kcap) {
    set_err(t, "batch size outside 1..max_batch or capacity exceeded");
    return SBT_E_SHAPE;
  }
  hipStream_t st = (hipStream_t)stream;
  const size_t esz = prec_bytes(t->store_prec);
  const size_t slice = (size_t)t->I * t->J;
  void* dst = (char*)t->X + (size_t)t->K * slice * esz;
  const int uq = prof_begin(t, st);
  // ingest: append the batch behind the stored slices (not yet part of the tensor)
  SBT_CK(hipMemcpyAsync(dst, Y_dev, slice * K_new * esz, hipMemcpyDeviceToDevice, st));
  SBT_CK(launch_fill_u64(t->dw1, t->I, 0, st));
  SBT_CK(launch_fill_u64(t->dw2, t->J, 0, st));
  SBT_CK(launch_fill_u64(t->dw3, K_new, 0, st));
  SBT_CK(launch_fill_u32(t->err, 1, 0, st));
  SBT_CK(launch_moi_dense(t->store_prec, dst, t->I, t->J, K_new, t->scale, t->qmax, t->dw1,
                          t->dw2, t->dw3, t->err, st));
  return update_body(t, K_new, uq, st);
}

sbt_status update_coo_body(sbt_tensor* t, const int32_t* i_dev, const int32_t* j_dev,
                           const int32_t* k_dev, const float* v_dev, int64_t nnz, int64_t K_new,
                           void* stream) {
  if (t->nd) return not_for_nd(t);
  if (t->fmt != SBT_COO) {
    set_err(t, "tensor is not COO");
    return SBT_E_STATE;
  }
  if (nnz < 0 || (nnz > 0 && (!i_dev || !j_dev || !k_dev || !v_dev))) return SBT_E_INVALID;
  if (K_new < 1 || K_new > t->cfg.max_batch || t->K + K_new > t->Kcap ||
      t->nnz + nnz > t->nnz_cap) {
    set_err(t, "batch size outside 1..max_batch or capacity exceeded");
    return SBT_E_SHAPE;
  }
  hipStream_t st = (hipStream_t)stream;
  const int uq = prof_begin(t, st);
  SBT_CK(launch_fill_u64(t->dw1, t->I, 0, st));
  SBT_CK(launch_fill_u64(t->dw2, t->J, 0, st));
  SBT_CK(launch_fill_u64(t->dw3, K_new, 0, st));
  SBT_CK(launch_fill_u32(t->err, 1, 0, st));
  SBT_CK(launch_moi_coo(i_dev, j_dev, k_dev, v_dev, nnz, t->I, t->J, K_new, t->scale, t->qmax,
                        t->dw1, t->dw2, t->dw3, t->err, st));
  // coordinates are checked before the batch enters the store
  SBT_CK(hipMemcpyAsync(t->h_err, t->err, 4, hipMemcpyDeviceToHost, st));
  SBT_CK(hipStreamSynchronize(st));
  if (*t->h_err) {
    prof_collect(t);
    set_err(t, (*t->h_err & 2u)
                   ? "batch coordinate outside the tensor"
                   : "batch holds a non-finite value or overflows the importance sums");
    return (*t->h_err & 2u) ? SBT_E_SHAPE : SBT_E_NUMERIC;
  }
  SBT_TRY(ensure_ingest(t, nnz, st));
  SBT_CK(launch_coo_ingest(i_dev, j_dev, k_dev, v_dev, nnz, K_new, t->K, t->ci, t->cj, t->ck,
                           t->cv, t->nnz, t->koff, t->ing, st));
  t->pending_nnz = nnz;
  return update_body(t, K_new, uq, st);
}

}  // namespace

namespace sbt {
sbt_status server_update_dense(sbt_tensor* t, const void* Y_dev, int64_t K_new,
                               hipStream_t st) {
  if (!t || !Y_dev) return SBT_E_INVALID;
  CallGuard g(t, true);
  if (!g.ok) return SBT_E_BUSY;
  return update_dense_body(t, Y_dev, K_new, st);
}
sbt_status server_update_coo(sbt_tensor* t, const int32_t* i_dev, const int32_t* j_dev,
                             const int32_t* k_dev, const float* v_dev, int64_t nnz,
                             int64_t K_new, hipStream_t st) {
  if (!t) return SBT_E_INVALID;
  CallGuard g(t, true);
  if (!g.ok) return SBT_E_BUSY;
  return update_coo_body(t, i_dev, j_dev, k_dev, v_dev, nnz, K_new, st);
}
void server_lease(sbt_tensor* t, int delta) { t->leases.fetch_add(delta); }
size_t update_workspace_bytes(const sbt_tensor* t) {
  size_t b = t->bytes_fixed;
  for (const auto& g : t->grow_allocs) b += g.second;
  const size_t res = resident_bytes(t);
  return b > res ? b - res : 0;
}
bool is_coo(const sbt_tensor* t) { return t && !t->nd && t->fmt == SBT_COO; }
}  // namespace sbt

extern "C" {

sbt_status sbt_update_batch_dense(sbt_tensor* t, const void* Y_dev, int64_t K_new, void* stream) {
  if (!t || !Y_dev) return SBT_E_INVALID;
  CallGuard g(t, false);
  if (!g.ok) return SBT_E_BUSY;
  return update_dense_body(t, Y_dev, K_new, stream);
}

sbt_status sbt_update_batch_coo(sbt_tensor* t, const int32_t* i_dev, const int32_t* j_dev,
                                const int32_t* k_dev, const float* v_dev, int64_t nnz,
                                int64_t K_new, void* stream) {
  if (!t) return SBT_E_INVALID;
  CallGuard g(t, false);
  if (!g.ok) return SBT_E_BUSY;
  return update_coo_body(t, i_dev, j_dev, k_dev, v_dev, nnz, K_new, stream);
}

sbt_status sbt_get_shape(const sbt_tensor* t, int64_t* I, int64_t* J, int64_t* K, int32_t* R) {
  if (!t) return SBT_E_INVALID;
  if (t->nd) return SBT_E_STATE;
  if (I) *I = t->I;
  if (J) *J = t->J;
  if (K) *K = t->K;
  if (R) *R = t->R;
  return SBT_OK;
}

sbt_status sbt_memory_bytes(const sbt_tensor* t, int64_t* resident, int64_t* workspace) {
  if (!t) return SBT_E_INVALID;
  if (t->nd) return SBT_E_STATE;
  if (resident) *resident = (int64_t)resident_bytes(t);
  if (workspace) *workspace = (int64_t)sbt::update_workspace_bytes(t);
  return SBT_OK;
}

sbt_status sbt_get_batch_counter(const sbt_tensor* t, uint32_t* counter) {
  if (!t || !counter) return SBT_E_INVALID;
  *counter = t->t;
  return SBT_OK;
}

sbt_status sbt_save(sbt_tensor* t, const char* path, void* stream) {
  if (!t || !path) return SBT_E_INVALID;
  if (t->nd) return not_for_nd(t);
  CallGuard g(t, false);
  if (!g.ok) return SBT_E_BUSY;
  CkptHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kCkptMagic, 8);
  h.version = kCkptVersion;
  h.header_bytes = (uint32_t)sizeof(CkptHeader);
  h.cfg = t->cfg;
  h.I = t->I;
  h.J = t->J;
  h.K = t->K;
  h.Kcap = t->Kcap;
  h.nnz = t->nnz;
  h.R = t->R;
  h.fmt = t->fmt;
  h.store_prec = t->store_prec;
  h.sum_prec = t->sum_prec;
  h.S = t->S;
  h.t = t->t;
  h.nmax = t->nmax;
  h.have_kept = t->have_kept ? 1 : 0;
  h.n3kept = t->n3kept;
  const std::vector<CkptArray> arrs = ckpt_arrays(t, t->have_kept);
  for (const auto& a : arrs) h.payload_bytes += a.bytes;
  CkptIO io;
  io.st = (hipStream_t)stream;
  if (!io.open(path, "wb")) {
    set_err(t, std::string("cannot open ") + path + " for writing");
    return SBT_E_INVALID;
  }
  if (fwrite(&h, sizeof(h), 1, io.f) != 1) {
    set_err(t, std::string("write failed: ") + path);
    return SBT_E_DEVICE;
  }
  for (const auto& a : arrs)
    if (!io.put(a.dev, a.bytes)) {
      set_err(t, std::string("write failed: ") + path);
      return SBT_E_DEVICE;
    }
  if (fflush(io.f) != 0) {
    set_err(t, std::string("write failed: ") + path);
    return SBT_E_DEVICE;
  }
  return SBT_OK;
}

sbt_status sbt_load(const char* path, void* stream, sbt_tensor** out) {
  if (!path || !out) return SBT_E_INVALID;
  *out = nullptr;
  auto fail = [](const std::string& m, sbt_status s) {
    g_errmsg = m;
    return s;
  };
  CkptIO io;
  io.st = (hipStream_t)stream;
  if (!io.open(path, "rb")) return fail(std::string("cannot open ") + path, SBT_E_INVALID);
  CkptHeader h;
  if (fread(&h, sizeof(h), 1, io.f) != 1 || std::memcmp(h.magic, kCkptMagic, 8) != 0 ||
      h.version != kCkptVersion || h.header_bytes != sizeof(CkptHeader))
    return fail(std::string(path) + " is not a checkpoint of this library version",
                SBT_E_INVALID);
  std::string why;
  if (validate_config(&h.cfg, why) != SBT_OK) return fail("checkpoint config: " + why,
                                                          SBT_E_INVALID);
  const bool dense = h.fmt == SBT_DENSE;
  if (h.fmt != h.cfg.format || h.R != h.cfg.rank || h.Kcap != h.cfg.k_capacity || h.I < 1 ||
      h.J < 1 || h.K < 1 || h.K > h.Kcap || h.I > INT32_MAX || h.J > INT32_MAX ||
      (!dense && (h.nnz < 0 || h.nnz > h.cfg.nnz_capacity)) ||
      (h.have_kept && !h.cfg.persist_summaries))
    return fail(std::string(path) + ": inconsistent checkpoint header", SBT_E_INVALID);
  sbt_tensor* t = new (std::nothrow) sbt_tensor();
  if (!t) return SBT_E_NOMEM;
  t->cfg = h.cfg;
  t->I = h.I;
  t->J = h.J;
  t->K = h.K;
  t->Kcap = h.Kcap;
  t->R = h.R;
  t->fmt = h.fmt;
  t->store_prec = h.store_prec;
  t->sum_prec = h.sum_prec;
  t->nmax = h.nmax ? h.nmax : 1;
  t->nnz_cap = dense ? 0 : h.cfg.nnz_capacity;
  sbt_status s = SBT_OK;
  if (dense) {
    s = dalloc_bytes(t, &t->X, (size_t)t->I * t->J * t->Kcap * prec_bytes(t->store_prec));
  } else {
    s = dalloc(t, &t->ci, (size_t)t->nnz_cap);
    if (s == SBT_OK) s = dalloc(t, &t->cj, (size_t)t->nnz_cap);
    if (s == SBT_OK) s = dalloc(t, &t->ck, (size_t)t->nnz_cap);
    if (s == SBT_OK) s = dalloc(t, &t->cv, (size_t)t->nnz_cap);
  }
  if (s == SBT_OK) s = alloc_state(t);
  if (s == SBT_OK) {
    t->nnz = dense ? 0 : h.nnz;
    uint64_t payload = 0;
    const std::vector<CkptArray> arrs = ckpt_arrays(t, h.have_kept != 0);
    for (const auto& a : arrs) payload += a.bytes;
    if (payload != h.payload_bytes) {
      set_err(t, "checkpoint payload size does not match its header");
      s = SBT_E_INVALID;
    }
    for (size_t q = 0; s == SBT_OK && q < arrs.size(); ++q)
      if (!io.get(arrs[q].dev, arrs[q].bytes)) {
        set_err(t, std::string("read failed or file truncated: ") + path);
        s = SBT_E_INVALID;
      }
  }
  if (s == SBT_OK) {
    const int R = t->R;
    hipError_t e = launch_fill_f64(t->ones, (int64_t)R * R, 1.0, io.st);
    if (e == hipSuccess) e = launch_fill_u32(t->pinv, 1, 0, io.st);
    if (e == hipSuccess) e = launch_fill_u32(t->cnt, 2 * (int64_t)t->cfg.repetitions, 0, io.st);
    if (e == hipSuccess) e = hipStreamSynchronize(io.st);
    if (e != hipSuccess) {
      set_err(t, hipGetErrorString(e));
      s = SBT_E_DEVICE;
    }
    t->S = h.S;
    t->scale = std::ldexp(1.0, t->S);
    t->qmax = (uint64_t)((((unsigned __int128)1) << 63) / t->nmax);
    t->t = h.t;
    // the kept summaries themselves are rebuilt from the kept indices at the
    // next update (the same values a kept copy would hold)
    t->have_kept = h.have_kept != 0;
    t->n3kept = h.n3kept;
    t->z_kept = false;
    t->coo_kept = false;
  }
  if (s != SBT_OK) {
    g_errmsg = t->errmsg;
    free_all(t);
    delete t;
    return s;
  }
  *out = t;
  return SBT_OK;
}

sbt_status sbt_get_factors(sbt_tensor* t, double* A, double* B, double* C, double* lambda,
                           void* stream) {
  if (!t) return SBT_E_INVALID;
  CallGuard g(t, false);
  if (!g.ok) return SBT_E_BUSY;
  if (t->nd) return not_for_nd(t);
  hipStream_t st = (hipStream_t)stream;
  const int R = t->R;
  if (A) SBT_CK(hipMemcpyAsync(A, t->A, sizeof(double) * t->I * R, hipMemcpyDeviceToHost, st));
  if (B) SBT_CK(hipMemcpyAsync(B, t->B, sizeof(double) * t->J * R, hipMemcpyDeviceToHost, st));
  if (C) SBT_CK(hipMemcpyAsync(C, t->C, sizeof(double) * t->K * R, hipMemcpyDeviceToHost, st));
  if (lambda) SBT_CK(hipMemcpyAsync(lambda, t->lam, sizeof(double) * R, hipMemcpyDeviceToHost, st));
  SBT_CK(hipStreamSynchronize(st));
  return SBT_OK;
}

sbt_status sbt_fit(sbt_tensor* t, double* fit, void* stream) {
  if (!t || !fit) return SBT_E_INVALID;
  CallGuard g(t, false);
  if (!g.ok) return SBT_E_BUSY;
  hipStream_t st = (hipStream_t)stream;
  if (t->nd) return nd_fit(t, fit, st);
  if (t->fmt == SBT_DENSE) {
    SBT_CK(launch_fit_slices(t->store_prec, t->X, t->I, t->J, t->K, t->R, t->A, t->B, t->M3,
                             t->nrm, st));
  } else {
    SBT_CK(launch_fit_coo(t->ci, t->cj, t->cv, t->koff, t->K, t->R, t->A, t->B, t->M3, t->nrm,
                          st));
  }
  {
    XProd xp{};
    xp.job[0] = XJob{t->A, 0, nullptr, 0, t->A, 0, nullptr, 0, (int)t->I};
    xp.job[1] = XJob{t->B, 0, nullptr, 0, t->B, 0, nullptr, 0, (int)t->J};
    xp.job[2] = XJob{t->C, 0, nullptr, 0, t->C, 0, nullptr, 0, (int)t->K};
    xp.njobs = 3;
    xp.R = t->R;
    xp.rep0 = 0;
    xp.nrep = 1;
    int64_t mf = t->I > t->J ? t->I : t->J;
    if (t->Kcap > mf) mf = t->Kcap;
    xp.nblk = xprod_blocks((int)mf);
    xp.part = t->xpart;
    xp.out = t->xout;
    SBT_CK(launch_xprod(xp, st));
  }
  SBT_CK(launch_fit_final(t->xout, t->C, t->lam, t->M3, t->nrm, t->K, t->R, t->fitv, st));
  SBT_CK(hipMemcpyAsync(fit, t->fitv, sizeof(double), hipMemcpyDeviceToHost, st));
  SBT_CK(hipStreamSynchronize(st));
  return SBT_OK;
}

sbt_status sbt_fms(sbt_tensor* t, const double* A_ref, const double* B_ref, const double* C_ref,
                   const double* lambda_ref, double* score, void* stream) {
  if (!t || !A_ref || !B_ref || !C_ref || !lambda_ref || !score) return SBT_E_INVALID;
  if (t->nd) return not_for_nd(t);
  CallGuard g(t, false);
  if (!g.ok) return SBT_E_BUSY;
  hipStream_t st = (hipStream_t)stream;
  XProd xp{};
  const int I = (int)t->I, J = (int)t->J, K = (int)t->K;
  xp.job[0] = XJob{t->A, 0, nullptr, 0, A_ref, 0, nullptr, 0, I};
  xp.job[1] = XJob{t->B, 0, nullptr, 0, B_ref, 0, nullptr, 0, J};
  xp.job[2] = XJob{t->C, 0, nullptr, 0, C_ref, 0, nullptr, 0, K};
  xp.job[3] = XJob{t->A, 0, nullptr, 0, t->A, 0, nullptr, 0, I};
  xp.job[4] = XJob{t->B, 0, nullptr, 0, t->B, 0, nullptr, 0, J};
  xp.job[5] = XJob{t->C, 0, nullptr, 0, t->C, 0, nullptr, 0, K};
  xp.job[6] = XJob{A_ref, 0, nullptr, 0, A_ref, 0, nullptr, 0, I};
  xp.job[7] = XJob{B_ref, 0, nullptr, 0, B_ref, 0, nullptr, 0, J};
  xp.job[8] = XJob{C_ref, 0, nullptr, 0, C_ref, 0, nullptr, 0, K};
  xp.njobs = 9;
  xp.R = t->R;
  xp.rep0 = 0;
  xp.nrep = 1;
  int mr = I > J ? I : J;
  if (K > mr) mr = K;
  xp.nblk = xprod_blocks(mr);
  if (9 * (int64_t)xp.nblk > t->xpart_mats) {
    set_err(t, "cross-product workspace too small for the factor match score");
    return SBT_E_SHAPE;
  }
  xp.part = t->xpart;
  xp.out = t->xout;
  SBT_CK(launch_xprod(xp, st));
  SBT_CK(launch_fms(t->xout, t->lam, lambda_ref, t->R, t->fitv, st));
  SBT_CK(hipMemcpyAsync(score, t->fitv, sizeof(double), hipMemcpyDeviceToHost, st));
  SBT_CK(hipStreamSynchronize(st));
  return SBT_OK;
}

sbt_status sbt_last_sample(const sbt_tensor* tc, int32_t rep, int32_t mode, int32_t* idx,
                           int64_t* n) {
  sbt_tensor* t = const_cast<sbt_tensor*>(tc);
  if (!t || !idx || !n || mode < 0 || (mode > 2 && !t->nd)) return SBT_E_INVALID;
  if (!t->has_last) return SBT_E_STATE;
  if (rep < 0 || rep >= t->cfg.repetitions) return SBT_E_INVALID;
  int64_t cnt = mode == 0 ? t->n1 : (mode == 1 ? t->n2 : t->last_n3old);
  int64_t off = mode == 0 ? 0 : (mode == 1 ? t->n1 : (int64_t)t->n1 + t->n2);
  if (t->nd && !nd_sample_span(t, mode, &off, &cnt)) return SBT_E_INVALID;
  SBT_CK(hipMemcpy(idx, t->idx + rep * t->idx_stride + off, sizeof(int32_t) * cnt,
                   hipMemcpyDeviceToHost));
  *n = cnt;
  return SBT_OK;
}

sbt_status sbt_last_rep(const sbt_tensor* tc, int32_t rep, int32_t item, double* out,
                        int64_t cap, int64_t* rows) {
  sbt_tensor* t = const_cast<sbt_tensor*>(tc);
  if (!t || !out || !rows) return SBT_E_INVALID;
  if (t->nd) return not_for_nd(t);
  if (!t->has_last) return SBT_E_STATE;
  if (rep < 0 || rep >= t->cfg.repetitions) return SBT_E_INVALID;
  const int R = t->R;
  RepSet rs = make_repset(t, t->last_Kp, 0, t->cfg.repetitions);
  const double* src = nullptr;
  int64_t nr = 0, ncol = R;
  const int32_t* isrc = nullptr;
  switch (item) {
    case SBT_REP_AP: src = t->Ap + rep * rs.sA; nr = t->n1; break;
    case SBT_REP_BP: src = t->Bp + rep * rs.sB; nr = t->n2; break;
    case SBT_REP_CP: src = t->Cp + rep * rs.sC; nr = t->last_Kp; break;
    case SBT_REP_LAMP: src = t->lamp + rep * R; nr = 1; break;
    case SBT_REP_PI: isrc = t->pi + rep * R; nr = 1; break;
    case SBT_REP_VALID: isrc = t->valid + rep * R; nr = 1; break;
    case SBT_REP_AT: src = t->At + rep * rs.sA; nr = t->n1; break;
    case SBT_REP_BT: src = t->Bt + rep * rs.sB; nr = t->n2; break;
    case SBT_REP_CT: src = t->Ct + rep * rs.sC; nr = t->last_Kp; break;
    case SBT_REP_RNEW:
      if (cap < 1) return SBT_E_INVALID;
      if (t->grnew) {
        int32_t v = 0;
        SBT_CK(hipMemcpy(&v, t->grnew + rep, sizeof(int32_t), hipMemcpyDeviceToHost));
        out[0] = (double)v;
      } else {
        out[0] = (double)R;
      }
      *rows = 1;
      return SBT_OK;
    case SBT_REP_CC:
      if (!t->gtab) return SBT_E_STATE;
      src = t->gtab + (int64_t)rep * R * t->cfg.getrank_runs;
      nr = R;
      ncol = t->cfg.getrank_runs;
      break;
    default: return SBT_E_INVALID;
  }
  if (cap < nr * ncol) return SBT_E_INVALID;
  if (src) {
    SBT_CK(hipMemcpy(out, src, sizeof(double) * nr * ncol, hipMemcpyDeviceToHost));
  } else {
    std::vector<int32_t> tmp((size_t)ncol);
    SBT_CK(hipMemcpy(tmp.data(), isrc, sizeof(int32_t) * ncol, hipMemcpyDeviceToHost));
    for (int64_t q = 0; q < ncol; ++q) out[q] = (double)tmp[(size_t)q];
  }
  *rows = nr;
  return SBT_OK;
}

sbt_status sbt_profile_enable(sbt_tensor* t, int32_t on) {
  if (!t || on < 0) return SBT_E_INVALID;
  t->prof_on = on != 0;
  t->prof_stride = on > 1 ? on : 1;
  t->prof_seq = 0;
  for (int k = 0; k < SBT_K_COUNT; ++k) {
    t->prof_n[k] = 0;
    t->prof_ms[k] = 0.0;
    t->prof_b[k] = 0.0;
  }
  t->prof_kind.clear();
  t->prof_bytes.clear();
  return SBT_OK;
}

sbt_status sbt_profile_read(const sbt_tensor* t, int32_t kind, int64_t* launches,
                            double* total_ms, double* alg_bytes) {
  if (!t || kind < 0 || kind >= SBT_K_COUNT) return SBT_E_INVALID;
  if (launches) *launches = t->prof_n[kind];
  if (total_ms) *total_ms = t->prof_ms[kind];
  if (alg_bytes) *alg_bytes = t->prof_b[kind];
  return SBT_OK;
}

sbt_status sbt_mttkrp_dense(int32_t precision, int32_t schedule, const void* Z_dev, int64_t n1,
                            int64_t n2, int64_t n3, int32_t R, const double* U0_dev,
                            const double* U1_dev, const double* U2_dev, int32_t mode,
                            double* out_dev, void* stream) {
  sbt_tensor* t = nullptr;  // for SBT_CK: no tensor to record the message on
  if (!Z_dev || !out_dev || R < 1 || R > kMaxRank || n1 < 1 || n2 < 1 || n3 < 1 || mode < 0 ||
      mode > 2 || precision < SBT_P_F64 || precision > SBT_P_BF16 ||
      (schedule != SBT_SCHED_BATCHED && schedule != SBT_SCHED_PLAIN))
    return SBT_E_INVALID;
  if (n1 > INT32_MAX || n2 > INT32_MAX || n3 > INT32_MAX) return SBT_E_SHAPE;
  const int prec = precision == SBT_P_F64 ? kF64 : (precision == SBT_P_F32 ? kF32 : kBF16);
  hipStream_t st = (hipStream_t)stream;
  RepSet rs;
  rs.n1 = (int)n1;
  rs.n2 = (int)n2;
  rs.n3 = (int)n3;
  rs.R = R;
  rs.rep0 = 0;
  rs.nrep = 1;
  rs.sZ = n1 * n2 * n3;
  rs.sA = n1 * R;
  rs.sB = n2 * R;
  rs.sC = n3 * R;
  rs.sW = n1 * n2 * R;
  rs.sM = 0;
  rs.sG = (int64_t)R * R;
  rs.nsplit = 1;
  if (prec == kBF16 && mfma_supported(rs.n1, rs.n2, R)) {
    // the kernels of the batched BF16 update: relayout, then pass W and the
    // mode-1/2 contraction, or the mode-3 kernel and its finish, with V = I
    if ((mode != 0 && !U0_dev) || (mode != 1 && !U1_dev) || (mode != 2 && !U2_dev))
      return SBT_E_INVALID;
    const MfmaLayout L = mfma_layout(rs.n1, rs.n2, rs.n3);
    rs.sZ = 0;
    std::vector<double> eye((size_t)R * R, 0.0), one((size_t)3 * R, 1.0);
    for (int f = 0; f < R; ++f) eye[(size_t)f * R + f] = 1.0;
    uint16_t *Zk = nullptr, *Zc = nullptr;
    double *I_dev = nullptr, *one_dev = nullptr;
    void* W = nullptr;
    float* P = nullptr;
    const int ns = mfma_mode3_splits(rs, L);
    const int64_t sP = (int64_t)rs.n3 * (R <= 16 ? 16 : 32);
    SBT_CK(hipMallocAsync((void**)&Zk, sizeof(uint16_t) * L.sZk, st));
    SBT_CK(hipMallocAsync((void**)&Zc, sizeof(uint16_t) * L.sZc, st));
    SBT_CK(hipMallocAsync((void**)&I_dev, sizeof(double) * eye.size(), st));
    SBT_CK(hipMallocAsync((void**)&one_dev, sizeof(double) * one.size(), st));
    SBT_CK(hipMallocAsync(&W, sizeof(float) * rs.sW, st));
    SBT_CK(hipMallocAsync((void**)&P, sizeof(float) * ns * sP, st));
    float* ops = nullptr;
    SBT_CK(hipMallocAsync((void**)&ops, sizeof(float) * mfma_operand_floats(L, rs.n2, R), st));
    SBT_CK(hipMemsetAsync(Zk, 0, sizeof(uint16_t) * L.sZk, st));
    SBT_CK(hipMemcpyAsync(I_dev, eye.data(), sizeof(double) * eye.size(), hipMemcpyHostToDevice,
                          st));
    SBT_CK(hipMemcpyAsync(one_dev, one.data(), sizeof(double) * one.size(),
                          hipMemcpyHostToDevice, st));
    SBT_CK(launch_relayout_bf16((const uint16_t*)Z_dev, rs, L, Zk, Zc, st));
    if (mode == 2) {
      SBT_CK(launch_p3_mfma(rs, L, ns, Zk, U0_dev, nullptr, U1_dev, nullptr, P, sP, ops, st));
      SBT_CK(launch_mode3_finish(rs, ns, P, sP, I_dev, nullptr, out_dev, 0, st));
    } else {
      SBT_CK(launch_pw_mfma(rs, L, Zc, U2_dev, nullptr, (float*)W, ops, st));
      SBT_CK(launch_cw(kF32, rs, mode, W, mode == 0 ? U1_dev : U0_dev, one_dev, I_dev, out_dev,
                       0, st));
    }
    SBT_CK(hipStreamSynchronize(st));  // the host vectors above are read by the copies
    void* frees[] = {Zk, Zc, I_dev, one_dev, W, P, ops};
    for (void* q : frees) SBT_CK(hipFreeAsync(q, st));
    return SBT_OK;
  }
  if ((mode != 0 && !U0_dev) || (mode != 1 && !U1_dev) || (mode != 2 && !U2_dev))
    return SBT_E_INVALID;
  if (prec != kBF16 && schedule == SBT_SCHED_BATCHED) {
    // the kernels of the batched update with V = I and unit column scales:
    // pass W and the mode-1/2 contraction, or the fused mode-3 pass
    if (mode == 2 && !p3_fits(prec, rs.n1, rs.n2, R)) return SBT_E_SHAPE;
    std::vector<double> eye((size_t)R * R, 0.0), one((size_t)3 * R, 1.0);
    for (int f = 0; f < R; ++f) eye[(size_t)f * R + f] = 1.0;
    double *I_dev = nullptr, *one_dev = nullptr;
    void* W = nullptr;
    SBT_CK(hipMallocAsync((void**)&I_dev, sizeof(double) * eye.size(), st));
    SBT_CK(hipMallocAsync((void**)&one_dev, sizeof(double) * one.size(), st));
    SBT_CK(hipMemcpyAsync(I_dev, eye.data(), sizeof(double) * eye.size(), hipMemcpyHostToDevice,
                          st));
    SBT_CK(hipMemcpyAsync(one_dev, one.data(), sizeof(double) * one.size(),
                          hipMemcpyHostToDevice, st));
    if (mode == 2) {
      SBT_CK(launch_p3(prec, rs, false, Z_dev, U0_dev, one_dev, U1_dev, one_dev, I_dev, nullptr,
                       out_dev, 0, st));
    } else {
      SBT_CK(hipMallocAsync(&W, (size_t)rs.sW * acc_bytes(prec), st));
      SBT_CK(launch_pw(prec, rs, Z_dev, U2_dev, one_dev, W, st));
      SBT_CK(launch_cw(prec, rs, mode, W, mode == 0 ? U1_dev : U0_dev, one_dev, I_dev, out_dev,
                       0, st));
    }
    SBT_CK(hipStreamSynchronize(st));  // the host vectors above are read by the copies
    void* frees[] = {I_dev, one_dev, W};
    for (void* q : frees)
      if (q) SBT_CK(hipFreeAsync(q, st));
    return SBT_OK;
  }
  if (mode == 2) {
    SBT_CK(launch_p2(prec, rs, Z_dev, U0_dev, U1_dev, out_dev, st));
    return SBT_OK;
  }
  void* W = nullptr;
  SBT_CK(hipMallocAsync(&W, (size_t)rs.sW * acc_bytes(prec), st));
  SBT_CK(launch_p1(prec, rs, Z_dev, U2_dev, W, st));
  if (mode == 0)
    SBT_CK(launch_cw1(prec, rs, W, U1_dev, out_dev, st));
  else
    SBT_CK(launch_cw2(prec, rs, W, U0_dev, out_dev, st));
  SBT_CK(hipFreeAsync(W, st));
  return SBT_OK;
}

sbt_status sbt_mttkrp_coo(const int32_t* a_dev, const int32_t* b_dev, const int32_t* c_dev,
                          const float* v_dev, int64_t nnz, int64_t n1, int64_t n2, int64_t n3,
                          int32_t R, const double* U0_dev, const double* U1_dev,
                          const double* U2_dev, int32_t mode, int32_t lanes, double* out_dev,
                          void* stream) {
  sbt_tensor* t = nullptr;  // for SBT_CK: no tensor to record the message on
  if (!out_dev || R < 1 || R > kMaxRank || n1 < 1 || n2 < 1 || n3 < 1 || mode < 0 || mode > 2 ||
      nnz < 0 || (nnz > 0 && (!a_dev || !b_dev || !c_dev || !v_dev)) ||
      (lanes != 0 && lanes != 32 && lanes != 64))
    return SBT_E_INVALID;
  if ((mode != 0 && !U0_dev) || (mode != 1 && !U1_dev) || (mode != 2 && !U2_dev))
    return SBT_E_INVALID;
  // the a- and b-ordered copies sort on 24-bit row keys; entry positions are int
  if (n1 >= (1 << 24) || n2 >= (1 << 24) || n3 >= (1 << 24) || nnz > INT32_MAX)
    return SBT_E_SHAPE;
  hipStream_t st = (hipStream_t)stream;
  RepSet rs;
  rs.n1 = (int)n1;
  rs.n2 = (int)n2;
  rs.n3 = (int)n3;
  rs.R = R;
  rs.rep0 = 0;
  rs.nrep = 1;
  rs.sZ = 0;
  rs.sA = n1 * R;
  rs.sB = n2 * R;
  rs.sC = n3 * R;
  rs.sW = 0;
  rs.sM = 0;
  rs.sG = (int64_t)R * R;
  rs.nsplit = 1;
  const int rows = mode == 0 ? rs.n1 : (mode == 1 ? rs.n2 : rs.n3);
  const int rowsX = mode == 0 ? rs.n2 : rs.n1;
  const int rowsY = mode == 2 ? rs.n2 : rs.n3;
  const double* X = mode == 0 ? U1_dev : U0_dev;
  const double* Y = mode == 2 ? U1_dev : U2_dev;
  const int RX = R <= 16 ? 16 : 32;
  const int64_t cap = nnz + 1;
  std::vector<void*> bufs;
  auto get = [&](void** p, size_t bytes) -> hipError_t {
    hipError_t e = hipMallocAsync(p, bytes ? bytes : 1, st);
    if (e == hipSuccess) bufs.push_back(*p);
    return e;
  };
  auto release = [&]() {
    for (void* q : bufs) (void)hipFreeAsync(q, st);
    bufs.clear();
  };
  auto body = [&]() -> sbt_status {
    CooSummary z{};
    int32_t** i32s[] = {&z.a, &z.b, &z.c, &z.a_x, &z.a_y, &z.b_x, &z.b_y, &z.val, &z.perm};
    for (int32_t** p : i32s) SBT_CK(get((void**)p, sizeof(int32_t) * cap));
    float** f32s[] = {&z.v, &z.a_v, &z.b_v};
    for (float** p : f32s) SBT_CK(get((void**)p, sizeof(float) * cap));
    uint32_t** u32s[] = {&z.key_a, &z.key_b, &z.key_out};
    for (uint32_t** p : u32s) SBT_CK(get((void**)p, sizeof(uint32_t) * cap));
    SBT_CK(coo_sort_tmp_bytes(cap, &z.tmp_bytes));
    SBT_CK(get(&z.tmp, z.tmp_bytes));
    z.sOffA = n1 + 1;
    z.sOffB = n2 + 1;
    z.sOffC = n3 + 1;
    SBT_CK(get((void**)&z.offA, sizeof(int64_t) * z.sOffA));
    SBT_CK(get((void**)&z.offB, sizeof(int64_t) * z.sOffB));
    SBT_CK(get((void**)&z.offC, sizeof(int64_t) * z.sOffC));
    SBT_CK(get((void**)&z.rep_off, sizeof(int64_t) * 2));
    z.rep_off_h[0] = 0;
    z.rep_off_h[1] = nnz;
    z.cap = cap;
    CooUnits u{};
    u.cap = cap / kCooUnit + rows + 1;
    SBT_CK(get((void**)&u.cnt, sizeof(uint32_t) * rows));
    SBT_CK(get((void**)&u.uoff, sizeof(int64_t) * (rows + 1)));
    SBT_CK(get((void**)&u.urow, sizeof(int32_t) * u.cap));
    SBT_CK(get((void**)&u.ustart, sizeof(int64_t) * u.cap));
    SBT_CK(get((void**)&u.ulen, sizeof(int32_t) * u.cap));
    float *Xf = nullptr, *Yf = nullptr, *part = nullptr;
    SBT_CK(get((void**)&Xf, sizeof(float) * rowsX * RX));
    SBT_CK(get((void**)&Yf, sizeof(float) * rowsY * RX));
    SBT_CK(get((void**)&part, sizeof(float) * u.cap * kMaxRank));
    double* I_dev = nullptr;
    SBT_CK(get((void**)&I_dev, sizeof(double) * R * R));
    std::vector<double> eye((size_t)R * R, 0.0);
    for (int f = 0; f < R; ++f) eye[(size_t)f * R + f] = 1.0;
    SBT_CK(hipMemcpyAsync(I_dev, eye.data(), sizeof(double) * eye.size(), hipMemcpyHostToDevice,
                          st));
    SBT_CK(hipMemcpyAsync(z.rep_off, z.rep_off_h, sizeof(int64_t) * 2, hipMemcpyHostToDevice,
                          st));
    SBT_CK(launch_coo_single_summary(a_dev, b_dev, c_dev, v_dev, nnz, rs.n1, rs.n2, rs.n3, z,
                                     st));
    SBT_CK(launch_coo_units_build(rs, mode, z, u, st));
    SBT_CK(launch_coo_prep(rs, rowsX, X, (int64_t)rowsX * R, nullptr, Xf, st));
    SBT_CK(launch_coo_prep(rs, rowsY, Y, (int64_t)rowsY * R, nullptr, Yf, st));
    // the lane count of the unit kernel follows the summary entries per row
    // (64 lanes from 128 on); `lanes` forces either variant
    const double avg = lanes == 64 ? 1e300 : (lanes == 32 ? 0.0 : (double)nnz / rows);
    SBT_CK(launch_coo_units(rs, mode, z, u, Xf, rowsX, Yf, rowsY, part, avg, st));
    SBT_CK(launch_coo_units_finish(rs, mode, u, part, I_dev, nullptr, out_dev, 0, st));
    SBT_CK(hipStreamSynchronize(st));  // the host arrays above are read by the copies
    return SBT_OK;
  };
  const sbt_status r = body();
  release();
  if (r != SBT_OK) (void)hipStreamSynchronize(st);
  return r;
}

}  // extern "C"

#include "engine_nd.inc"
#include "engine_nd_coo.inc"

namespace sbt {
size_t store_elem_bytes(const sbt_tensor* t) {
  if (!t || t->fmt != SBT_DENSE || t->nd) return 0;
  return prec_bytes(t->store_prec);
}
}  // namespace sbt
