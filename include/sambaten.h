/*
 * sambaten.h - C ABI of the MI355X (gfx950) SamBaTen update library.
 *
 * SamBaTen: Sampling-based Batch Incremental Tensor Decomposition (Gujral,
 * Pasricha, Papalexakis).  The library keeps a 3-mode tensor that grows along
 * its third mode, its rank-R CP model (A, B, C, lambda) and the sampling
 * state on one GPU, and applies the batch update of Algorithm 1 to each new
 * batch of frontal slices.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Indices are 0-based.
 * - A dense tensor is column-major: element (i, j, k) of an I x J x K tensor
 *   sits at i + I*(j + J*k), so a batch of frontal slices is one contiguous
 *   block.  Element type: double for SBT_P_F64, float otherwise.
 * - A COO tensor is structure-of-arrays: int32 i, j, k and float values.
 * - Factor matrices crossing the ABI are row-major double arrays
 *   (A: I x R, B: J x R, C: K x R), lambda is R doubles.
 * - Pointers named *_dev are device pointers; every other pointer is host
 *   memory.  The caller owns all buffers it passes and keeps them valid until
 *   the call returns (calls that take a stream are finished when they return
 *   unless stated otherwise).  The library owns every buffer it allocates and
 *   releases them in sbt_destroy.
 * - `stream` is a hipStream_t (NULL = the default stream).
 * - No C++ exception or abort crosses the ABI.  Every call returns an
 *   sbt_status; sbt_last_error() gives a message for the last failure on a
 *   tensor.  A failed sbt_update_* leaves the tensor exactly as it was.
 * - One call at a time per tensor: a call made while another call on the
 *   same tensor is in flight (another host thread), or while a server holds
 *   queued or running requests of the tensor, returns SBT_E_BUSY and changes
 *   nothing (the first call is unaffected).  sbt_destroy must not overlap
 *   any other call on the tensor.
 * - sbt_last_error(NULL) gives the message of the last failed call of the
 *   calling host thread that had no tensor to record it on (sbt_load, and
 *   the sbt_init_* and sbt_nd_init_* calls, whose tensor is released).
 */
#ifndef SAMBATEN_H
#define SAMBATEN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbt_tensor sbt_tensor;

typedef enum {
  SBT_OK = 0,
  SBT_E_INVALID = 1,  /* bad argument (null pointer, rank out of range ...) */
  SBT_E_SHAPE = 2,    /* I/J mismatch, empty batch, capacity exceeded */
  SBT_E_NOMEM = 3,    /* device allocation failed */
  SBT_E_DEVICE = 4,   /* a HIP runtime call failed */
  SBT_E_NUMERIC = 5,  /* non-finite input, or the integer importance sums would overflow */
  SBT_E_STATE = 6,    /* call not valid in the tensor's current state */
  SBT_E_BUSY = 7      /* another call on the tensor is in flight, or a server
                         holds requests of it; nothing was done */
} sbt_status;

typedef enum { SBT_DENSE = 0, SBT_COO = 1 } sbt_format;

/* Arithmetic of the summaries and of MTTKRP.  Gram matrices, Cholesky
 * solves, normalisation, matching and the row solve are FP64 in all cases.
 *   SBT_P_F64  : FP64 store, FP64 summaries and MTTKRP
 *   SBT_P_F32  : FP32 store, FP32 summaries, FP32 MTTKRP accumulation
 *   SBT_P_BF16 : FP32 store, BF16 summaries (round to nearest even),
 *                MTTKRP on BF16 MFMA with FP32 accumulation            */
typedef enum { SBT_P_F64 = 0, SBT_P_F32 = 1, SBT_P_BF16 = 2 } sbt_precision;

/* How the r repetitions are launched.
 *   SBT_SCHED_BATCHED: every launch covers all r repetitions; the three
 *     MTTKRPs of an ALS sweep take two passes over each summary (the mode-1
 *     and mode-2 products share the contraction with C).
 *   SBT_SCHED_PLAIN:   one launch sequence per repetition, three passes per
 *     sweep (one per mode).  Same arithmetic, used as the baseline.        */
typedef enum { SBT_SCHED_BATCHED = 0, SBT_SCHED_PLAIN = 1 } sbt_schedule;

/* Reading switches (sbt_config.flags).
 *   SBT_FLAG_LAMBDA_AVG: the last step of Algorithm 1 taken literally:
 *     lambda becomes the average of its previous value and the new one, the
 *     new one being, per component f, the mean over the repetitions valid for
 *     f (whose anchor column C(K_s, f) is not zero) of the summary's matched
 *     weight in the current model's units,
 *       lambda'_pi(f) ||C'(anchor rows, pi(f))|| /
 *         (||A(I_s, f)|| ||B(J_s, f)|| ||C(K_s, f)||),
 *     which equals lambda_f when the summary recovers the restriction of the
 *     model.  The new rows of C are still divided by the previous lambda, and
 *     the change of lambda rescales the old slices' reconstruction too.
 *     Default (flag off): lambda is kept, the new rows carry the scale.
 *     Third-order tensors only. */
enum { SBT_FLAG_LAMBDA_AVG = 1 };

typedef struct {
  int32_t rank;              /* R, 1..32 */
  int32_t repetitions;       /* r >= 1 (Algorithm 1) */
  int32_t als_iters;         /* CP-ALS sweeps on each summary (fixed count) */
  int32_t init_iters;        /* CP-ALS sweeps of the initial decomposition */
  int32_t sample_factor[3];  /* s per mode: n_m = ceil(N_m / s_m) (Sec. 3.1) */
  int32_t format;            /* sbt_format */
  int32_t precision;         /* sbt_precision */
  int32_t schedule;          /* sbt_schedule */
  uint64_t seed;             /* Philox key, low word */
  uint32_t tensor_id;        /* xored into the high key word */
  uint32_t flags;            /* readings of the paper, SBT_FLAG_* (0: defaults) */
  int64_t k_capacity;        /* largest third-mode size the tensor may reach */
  int64_t max_batch;         /* largest K_new of one update */
  int64_t nnz_capacity;      /* COO only: largest number of stored nonzeros */
  /* GetRank (Sec. 3.2, Alg. 2), third-order tensors with FP64 or FP32
   * summaries (dense, or COO, whose core consistency is computed from the
   * summary's entries slice by slice, the sparse form the paper uses).  With
   * getrank_runs > 0 every summary is decomposed at each candidate rank
   * i = 1..R, getrank_runs times (CP-ALS, als_iters sweeps, own initial
   * factors per run), each run is scored by its core consistency (percent),
   * and the summary's rank R_new is the largest i whose best run reaches
   * getrank_threshold (rank 1 always counts); that run's factors are the
   * summary's decomposition, and only R_new of the R current components are
   * matched to it.  0 turns GetRank off. */
  int32_t getrank_runs;
  int32_t reserved;          /* must be 0 */
  double getrank_threshold;  /* core consistency a candidate rank must reach */
  /* Persistent summaries (Sec. 3.1 assumes summaries of the tensor exist
   * before an update): with persist_summaries = 1 the indices I_s, J_s, K_s drawn at
   * an update are kept for the following updates (drawn afresh at every
   * update whose batch counter is a multiple of summary_refresh; never again
   * when it is 0), so each summary is X(I_s, J_s, K_s u new) with the same
   * anchors, and its CP-ALS starts from the previous summary factors (B',
   * and C' on the K_s rows; rows of the new slices drawn U[0,1) as usual).
   * Not combined with GetRank. */
  int32_t persist_summaries;
  int32_t summary_refresh;
} sbt_config;

/* --------------------------------------------------------------------------
 * Lifecycle (problem statement of Sec. 2.2: the existing tensor and its
 * R-component decomposition are the starting point).
 * ------------------------------------------------------------------------ */

/* Create a tensor from an existing dense I x J x K0 block X0_dev (device,
 * column-major, element type per cfg->precision).  The library copies X0
 * into its own storage sized for cfg->k_capacity.
 * If A0, B0, C0, lambda0 (host, row-major) are all non-NULL they become the
 * model as given; if all are NULL the library runs cfg->init_iters CP-ALS
 * sweeps on X0 (random U[0,1) start) and orders the components by lambda,
 * largest first.  Any other combination is SBT_E_INVALID. */
sbt_status sbt_init_dense(const sbt_config* cfg, const void* X0_dev, int64_t I, int64_t J,
                          int64_t K0, const double* A0, const double* B0, const double* C0,
                          const double* lambda0, void* stream, sbt_tensor** out);

/* Same for a COO tensor: nnz entries (i_dev[e], j_dev[e], k_dev[e], v_dev[e]),
 * device arrays; coordinates must lie inside I x J x K0, no coordinate
 * twice.  With the factors NULL the initial decomposition is CP-ALS on the
 * whole tensor (cfg->init_iters >= 1 sweeps from U[0,1) factors, the sparse
 * MTTKRP kernels of the update on the tensor taken as one summary with
 * every index; I, J and K0 must stay below 2^24), components ordered by
 * lambda, largest first. */
sbt_status sbt_init_coo(const sbt_config* cfg, const int32_t* i_dev, const int32_t* j_dev,
                        const int32_t* k_dev, const float* v_dev, int64_t nnz, int64_t I,
                        int64_t J, int64_t K0, const double* A0, const double* B0,
                        const double* C0, const double* lambda0, void* stream,
                        sbt_tensor** out);

void sbt_destroy(sbt_tensor* t);

/* --------------------------------------------------------------------------
 * The update (Algorithm 1): append K_new frontal slices and update the model.
 * Steps, all on the GPU: importance of the batch (Eq. 1) and input check;
 * per repetition and mode, weighted sampling without replacement of
 * ceil(N/s) indices from the tensor before the update; gather of the
 * summaries X(I_s, J_s, K_s u new); CP-ALS on every summary; normalisation
 * and optimal matching against A(I_s), B(J_s), C(K_s); least-squares rows of
 * C for the summary's slices; zero-entry fill; average of the new rows over
 * the repetitions; append.  lambda is left unchanged.
 * Returns when the update is complete.  SBT_E_NUMERIC for a non-finite value
 * or an importance overflow (tensor unchanged); SBT_E_SHAPE when K_new < 1,
 * K_new > max_batch or K + K_new > k_capacity.
 * ------------------------------------------------------------------------ */

/* Y_dev: I x J x K_new dense batch, column-major, device. */
sbt_status sbt_update_batch_dense(sbt_tensor* t, const void* Y_dev, int64_t K_new, void* stream);

/* COO batch; k_dev holds batch-relative third-mode indices 0..K_new-1. */
sbt_status sbt_update_batch_coo(sbt_tensor* t, const int32_t* i_dev, const int32_t* j_dev,
                                const int32_t* k_dev, const float* v_dev, int64_t nnz,
                                int64_t K_new, void* stream);

/* --------------------------------------------------------------------------
 * Queries.
 * ------------------------------------------------------------------------ */

sbt_status sbt_get_shape(const sbt_tensor* t, int64_t* I, int64_t* J, int64_t* K, int32_t* R);

/* Copy the model to caller-owned host buffers (row-major A I x R, B J x R,
 * C K x R, lambda R).  Any of the pointers may be NULL to skip it. */
sbt_status sbt_get_factors(sbt_tensor* t, double* A, double* B, double* C, double* lambda,
                           void* stream);

/* fit = 1 - ||X - Xhat||_F / ||X||_F over every stored slice (the relative
 * error of Sec. 4.2, as 1 - RE).  Computed on the GPU in FP64 from one pass
 * over the tensor and the factor Gram matrices. */
sbt_status sbt_fit(sbt_tensor* t, double* fit, void* stream);

/* Factor match score (Sec. 4.4) of the tensor's current model against a
 * reference model of the same shape and rank, given in device memory in the
 * layout of sbt_get_factors (row-major A_ref I x R, B_ref J x R, C_ref K x R,
 * lambda_ref R; K the tensor's current slice count).  Columns of both models
 * are scaled to unit norm with the norms moved into the weights; components
 * are paired by the maximum-weight assignment on the product over the modes
 * of |cosine|; each pair scores that product times the weight penalty
 * 1 - |l1 - l2| / max(l1, l2); *score (host) is the mean over the R pairs,
 * in [0, 1] (1: the same components).  Computed on the GPU in FP64 on
 * `stream`; returns when *score is written.  The reference buffers stay the
 * caller's.  Errors: SBT_E_INVALID for NULL pointers, SBT_E_DEVICE. */
sbt_status sbt_fms(sbt_tensor* t, const double* A_ref, const double* B_ref, const double* C_ref,
                   const double* lambda_ref, double* score, void* stream);

/* --------------------------------------------------------------------------
 * Checkpoint and resume.  A checkpoint holds what the next updates depend
 * on: the stored tensor (its K slices, or its nonzeros with their slice
 * offsets), the model (A, B, C, lambda), the importance vectors of the three
 * modes with their fixed-point scale, the batch counter that keys the
 * sampler, the configuration, and with persistent summaries the kept sample
 * indices and warm-start summary factors.  Updates applied to a loaded
 * tensor give exactly the results they give on the tensor that was saved
 * (the kept summaries are gathered again from the kept indices).  Third-order
 * tensors only (an order-N tensor gives SBT_E_STATE).
 * ------------------------------------------------------------------------ */

/* Write the tensor's state to the file `path` (created or truncated; a
 * little-endian binary of this library version).  Device data is copied out
 * on `stream` through a pinned host buffer; returns when the file is
 * written.  Errors: SBT_E_INVALID (NULL arguments, the file cannot be
 * opened), SBT_E_DEVICE (a copy or a write failed: the file is incomplete),
 * SBT_E_BUSY, SBT_E_STATE.  The tensor is not changed. */
sbt_status sbt_save(sbt_tensor* t, const char* path, void* stream);

/* Create a tensor from a file written by sbt_save, on the current device,
 * allocating the capacity its configuration names.  *out receives the
 * handle (NULL on error).  Errors: SBT_E_INVALID (cannot open, not a
 * checkpoint of this version, inconsistent header, truncated file; message
 * in sbt_last_error(NULL)), SBT_E_NOMEM, SBT_E_DEVICE. */
sbt_status sbt_load(const char* path, void* stream, sbt_tensor** out);

/* Device memory of a third-order tensor: *resident = its store at capacity,
 * model and importance vectors; *workspace = everything else it holds (the
 * r summaries and their factors, sampling, ALS and matching buffers, COO
 * buffers grown so far), which is what an update works in and what a server
 * charges a request against its HBM budget.  Either pointer may be NULL.
 * SBT_E_STATE for an order-N tensor. */
sbt_status sbt_memory_bytes(const sbt_tensor* t, int64_t* resident, int64_t* workspace);

/* Number of completed updates (the batch counter that keys the sampler). */
sbt_status sbt_get_batch_counter(const sbt_tensor* t, uint32_t* counter);

/* --------------------------------------------------------------------------
 * Inspection of the last update, for testing (host outputs).
 * ------------------------------------------------------------------------ */

/* Sampled indices of repetition `rep`, mode 0/1/2 (I_s, J_s, K_s), ascending.
 * idx must hold at least the mode's sample size; *n receives it. */
sbt_status sbt_last_sample(const sbt_tensor* t, int32_t rep, int32_t mode, int32_t* idx,
                           int64_t* n);

typedef enum {
  SBT_REP_AP = 0,     /* summary factor A' (n1 x R), unit columns          */
  SBT_REP_BP = 1,     /* summary factor B' (n2 x R)                        */
  SBT_REP_CP = 2,     /* summary factor C' (K' x R)                        */
  SBT_REP_LAMP = 3,   /* summary weights lambda' (R)                       */
  SBT_REP_PI = 4,     /* matching: sample column matched to column f (R);
                         R_new or more: no partner (GetRank)               */
  SBT_REP_VALID = 5,  /* 1 where the repetition is valid for column f (R)  */
  SBT_REP_AT = 6,     /* matched, rescaled A rows (n1 x R)                 */
  SBT_REP_BT = 7,     /* matched, rescaled B rows (n2 x R)                 */
  SBT_REP_CT = 8,     /* least-squares C rows of the summary (K' x R)      */
  SBT_REP_RNEW = 9,   /* rank of the summary's decomposition (1 value; R
                         without GetRank)                                   */
  SBT_REP_CC = 10     /* GetRank: core consistency of run j at rank i, row
                         i - 1, column j (R x getrank_runs)                 */
} sbt_rep_item;

/* Copy one per-repetition intermediate of the last update as doubles into
 * `out` (host, capacity `cap` doubles); *rows receives the row count. */
sbt_status sbt_last_rep(const sbt_tensor* t, int32_t rep, int32_t item, double* out,
                        int64_t cap, int64_t* rows);

/* --------------------------------------------------------------------------
 * Stand-alone kernels (the same code the update runs), for parity tests and
 * measurement.  All pointers are device pointers.
 * ------------------------------------------------------------------------ */

/* MTTKRP (Sec. 2.1: the matricised tensor times the Khatri-Rao product of
 * the other factors) of a dense n1 x n2 x n3 tensor Z (column-major; element
 * type per `precision`: double, float, or bfloat16 bits as uint16) with
 * row-major double factors U0 (n1 x R), U1 (n2 x R), U2 (n3 x R):
 *   mode 0: out(a,f) = sum_bc Z(a,b,c) U1(b,f) U2(c,f)     (n1 x R)
 *   mode 1: out(b,f) = sum_ac Z(a,b,c) U0(a,f) U2(c,f)     (n2 x R)
 *   mode 2: out(c,f) = sum_ab Z(a,b,c) U0(a,f) U1(b,f)     (n3 x R)
 * out is row-major double.  The factor for `mode` itself is not read (may be
 * NULL).  `schedule` picks the kernels of that update schedule:
 * SBT_SCHED_BATCHED the contraction with U2 followed by the contraction with
 * the other factor (modes 0, 1) and the fused third-mode pass (mode 2);
 * SBT_SCHED_PLAIN the per-step kernels.  BF16 always takes the matrix-core
 * kernels when their staging fits the shape.  Temporary device buffers are
 * allocated and freed on `stream`; returns when the result is written.
 * Errors: SBT_E_INVALID (NULL pointers, bad mode, precision or schedule),
 * SBT_E_SHAPE (extent above 2^31 - 1, or a batched mode-2 pass whose factors
 * do not fit its LDS staging), SBT_E_NOMEM / SBT_E_DEVICE. */
sbt_status sbt_mttkrp_dense(int32_t precision, int32_t schedule, const void* Z_dev, int64_t n1,
                            int64_t n2, int64_t n3, int32_t R, const double* U0_dev,
                            const double* U1_dev, const double* U2_dev, int32_t mode,
                            double* out_dev, void* stream);

/* sbt_mttkrp_dense for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, same kernels and the same result as sbt_mttkrp_dense, but
 * no hipMalloc/hipFree and no host-to-device copy: the temporary buffers
 * (the contraction W, the BF16 relayouts and partial rows, the identity
 * V^-1 and unit scales, which a kernel writes) are carved from one fixed
 * device array of 64 MiB per GPU, held until the process ends.  The call
 * only enqueues kernels on `stream` and returns; the result is written when
 * the stream reaches them.  The first call on a device resolves that
 * device's array address (hipGetSymbolAddress); make it outside graph
 * capture.  Every call on one GPU uses the same array: calls that overlap on
 * one GPU (two streams, two threads, or a second call enqueued before the
 * first has run on a different stream) race and give undefined results;
 * calls on one stream are ordered and safe.  Size limit: the bytes needed,
 * each piece rounded up to 256, must fit 64 MiB:
 *   FP64/FP32 modes 0, 1:  n1 n2 R x (8 for FP64, 4 for FP32) (+ 8 R^2 + 24 R
 *                          in the batched schedule);
 *   FP64/FP32 mode 2:      8 R^2 + 24 R (batched), nothing (plain);
 *   BF16 (matrix cores):   both BF16 relayouts of Z (about 4 n1 n2 n3 bytes
 *                          with padding) + 4 n1 n2 R + partial rows + staged
 *                          operands.
 * Errors: as sbt_mttkrp_dense; SBT_E_SHAPE also when the bytes needed exceed
 * the 64 MiB array (nothing is enqueued then); SBT_E_DEVICE when the array's
 * address cannot be resolved or a launch fails. */
sbt_status sbt_mttkrp_dense_noalloc(int32_t precision, int32_t schedule, const void* Z_dev,
                                    int64_t n1, int64_t n2, int64_t n3, int32_t R,
                                    const double* U0_dev, const double* U1_dev,
                                    const double* U2_dev, int32_t mode, double* out_dev,
                                    void* stream);

/* The same product for a COO tensor of extents n1 x n2 x n3 (the sparse
 * MTTKRP of the update's COO summaries, FP32 products and sums): entries
 * (a_dev[e], b_dev[e], c_dev[e], v_dev[e]), e < nnz, device arrays in any
 * order, coordinates inside the extents and no coordinate twice (not
 * checked: an entry outside gives undefined output).  The entries are
 * ordered, split into work units and contracted by the kernels of the
 * update; `lanes` = 32 or 64 forces the lanes per work unit, 0 lets the
 * entries per row decide as in the update.  Factors, out and the result
 * layout as for sbt_mttkrp_dense.  Returns when the result is written.
 * Errors: SBT_E_INVALID, SBT_E_SHAPE (an extent of 2^24 or more),
 * SBT_E_NOMEM / SBT_E_DEVICE. */
sbt_status sbt_mttkrp_coo(const int32_t* a_dev, const int32_t* b_dev, const int32_t* c_dev,
                          const float* v_dev, int64_t nnz, int64_t n1, int64_t n2, int64_t n3,
                          int32_t R, const double* U0_dev, const double* U1_dev,
                          const double* U2_dev, int32_t mode, int32_t lanes, double* out_dev,
                          void* stream);

/* --------------------------------------------------------------------------
 * Kernel timing.  While enabled, every update records a HIP event pair on its
 * stream around each launch of the kinds below and accumulates, per kind, the
 * launch count, the summed device time and the algorithmic bytes the launches
 * must move (summary elements read once plus factor rows read and outputs
 * written).  Timing adds two event records per timed launch.
 * sbt_profile_enable: on = 0 off; on = 1 every launch of these kinds; on = n > 1
 * every n-th of them (counted over all kinds in launch order), which keeps the
 * cost of the event records small while the per-kind averages stay those of
 * the launches; the whole-update pair (SBT_K_UPDATE) is recorded every time.
 * Enabling resets the accumulated figures.
 * ------------------------------------------------------------------------ */
typedef enum {
  SBT_K_MTTKRP_C = 0,   /* MTTKRP pass contracting the third mode with C'       */
  SBT_K_MTTKRP_AB = 1,  /* MTTKRP pass producing third-mode rows inside CP-ALS   */
  SBT_K_GATHER = 2,     /* summary gather                                        */
  SBT_K_UPDATE = 3,     /* whole update, first to last kernel                   */
  SBT_K_COO_MTTKRP = 4, /* sparse MTTKRP rows of one mode (ALS + row solve)      */
  SBT_K_ROW_SOLVE = 5,  /* dense third-mode row least squares (one per update)   */
  SBT_K_COUNT = 6
} sbt_kernel_kind;

sbt_status sbt_profile_enable(sbt_tensor* t, int32_t on);
sbt_status sbt_profile_read(const sbt_tensor* t, int32_t kind, int64_t* launches,
                            double* total_ms, double* alg_bytes);

/* --------------------------------------------------------------------------
 * Launch-shape tuner (process-wide; not part of the method).
 *
 * The BF16 matrix-core path of the update (the summary gather and the two
 * MTTKRP passes of each CP-ALS sweep, Algorithm 1's inner decompositions)
 * can launch its kernels in SBT_TUNE_SHAPES shapes (rows per block, operand
 * loads in flight, slices per gathering thread) whose results are identical
 * bit for bit: every output sums the same terms in the same order.  The
 * tuner keys each launch by the kernel, the device architecture and the
 * summary shape (R, n1 n2 and the repetitions; K' only scales the work) and, for a
 * key it has not decided, times the hot path's own launches in the shapes in
 * turn (two each, event pairs read back without waiting); from then on the
 * shape with the least time per unit of work is used for that key.  A
 * launch whose key is still undecided uses shape 0 unless it is a trial (a
 * launch captured into a graph never is).  The choice never changes a
 * result, only the time.
 *
 * sbt_autotune_set: mode SBT_TUNE_OFF (shape 0 always), SBT_TUNE_ON (the
 *   default: decide unseen keys online), SBT_TUNE_CACHED (decided keys only,
 *   no trials), SBT_TUNE_FIXED (every launch in `shape`, 0 <= shape < 8; a
 *   kernel with fewer shapes takes shape 0).  SBT_E_INVALID otherwise.
 * sbt_autotune_clear: forget every key (trials in flight are dropped).
 * sbt_autotune_count: keys decided and keys with trials running.
 * sbt_autotune_save: write the decided keys to the text file `path` (written
 *   to path.tmp, then renamed); SBT_E_INVALID if it cannot be written.
 * sbt_autotune_load: merge the keys of a file written by sbt_autotune_save
 *   into the table (a key present in both takes the file's shape); a file
 *   that cannot be read or has a malformed line changes nothing and gives
 *   SBT_E_INVALID.
 * Thread safety: every sbt_autotune_* call may come from any host thread.
 * ------------------------------------------------------------------------ */
typedef enum {
  SBT_TUNE_OFF = 0,
  SBT_TUNE_ON = 1,
  SBT_TUNE_CACHED = 2,
  SBT_TUNE_FIXED = 3
} sbt_tune_mode;
#define SBT_TUNE_SHAPES 3

sbt_status sbt_autotune_set(int32_t mode, int32_t shape);
sbt_status sbt_autotune_clear(void);
sbt_status sbt_autotune_count(int64_t* decided, int64_t* tuning);
sbt_status sbt_autotune_save(const char* path);
sbt_status sbt_autotune_load(const char* path);

/* --------------------------------------------------------------------------
 * Serving loop (many resident tensors, update requests arriving over time).
 *
 * A server owns `slots` worker threads, each driving its own HIP stream, a
 * device staging pool of `staging_bytes`, and an HBM budget for the working
 * sets of the updates it runs at once.  A request's working set is its
 * tensor's update workspace (everything the tensor holds besides its store,
 * model and importance vectors: the r summaries, their factors, the sampling
 * and ALS buffers and grown COO buffers, as they stand when the request is
 * admitted; a COO tensor's summary buffers grow to fit its first updates)
 * plus the request's staged batch.  Requests are admitted in arrival order
 * when a slot is free, the request's tensor has no update in flight (updates
 * of one tensor apply in arrival order), its batch fits the free staging
 * memory and its working set fits what the running requests leave of the
 * budget; a request that cannot start yet lets later requests of other
 * tensors start first.  A request whose working set exceeds the whole budget
 * fails with SBT_E_NOMEM when it comes up (reported by sbt_server_poll).  On
 * admission the batch is copied into the staging pool on the slot's stream
 * and the update runs there; updates of different tensors overlap on the
 * GPU.  Results equal those of the same updates applied one by one with
 * sbt_update_batch_dense / sbt_update_batch_coo.
 *
 * Thread safety: every sbt_server_* call may come from any host thread.
 * While a server holds queued or running requests of a tensor, direct calls
 * on it (update, get_factors, fit, fms, save) return SBT_E_BUSY; it must not
 * be destroyed then.
 * ------------------------------------------------------------------------ */
typedef struct sbt_server sbt_server;

/* slots in 1..32; staging_bytes >= 256; hbm_budget_bytes >= 0 (0: no
 * budget, admission by slots and staging memory only).  SBT_E_NOMEM if the
 * pool cannot be allocated. */
sbt_status sbt_server_create(int32_t slots, int64_t staging_bytes, int64_t hbm_budget_bytes,
                             sbt_server** out);

/* Queue an update of the dense tensor `t` by Y_dev (device, column-major
 * I x J x K_new in the tensor's store type).  Y_dev must hold its values
 * when submitted (the work that writes it complete: the server's streams do
 * not wait on the caller's), and stays valid until sbt_server_poll reports
 * the request running or done.  *ticket identifies the request.
 * SBT_E_NOMEM if the batch is larger than the whole staging pool or the
 * budget, SBT_E_STATE for a COO or order-N tensor, SBT_E_SHAPE for
 * K_new < 1; errors of the update itself are reported by sbt_server_poll. */
sbt_status sbt_server_submit_dense(sbt_server* s, sbt_tensor* t, const void* Y_dev,
                                   int64_t K_new, uint64_t* ticket);

/* Queue an update of the COO tensor `t` by nnz entries (i_dev, j_dev, k_dev,
 * v_dev: device arrays as for sbt_update_batch_coo, k batch-relative); the
 * four arrays are staged (16 bytes per entry, each array 256-byte aligned).
 * Buffer lifetime, ticket and errors as for sbt_server_submit_dense
 * (SBT_E_STATE for a dense tensor). */
sbt_status sbt_server_submit_coo(sbt_server* s, sbt_tensor* t, const int32_t* i_dev,
                                 const int32_t* j_dev, const int32_t* k_dev, const float* v_dev,
                                 int64_t nnz, int64_t K_new, uint64_t* ticket);

/* State of a request: *state 0 queued, 1 running, 2 done; *result the status
 * of the update once done; times in seconds since the server was created
 * (submission, start, completion).  Any output pointer may be null. */
sbt_status sbt_server_poll(sbt_server* s, uint64_t ticket, int32_t* state, sbt_status* result,
                           double* t_submit, double* t_start, double* t_done);

/* Block until every submitted request is done. */
sbt_status sbt_server_drain(sbt_server* s);

/* Drain, stop the workers and release the staging pool. */
void sbt_server_destroy(sbt_server* s);

/* --------------------------------------------------------------------------
 * Tensors of order N, 3 <= N <= 8, whose last mode grows (Sec. 2: the
 * problem and the method carry over to any number of modes).
 *
 * A dense order-N tensor is column-major: element (i_0, ..., i_N-1) of a
 * D_0 x ... x D_N-1 tensor sits at i_0 + D_0*(i_1 + D_1*(...)), so a batch of
 * last-mode slices is one contiguous block.  Factor m crossing the ABI is a
 * row-major D_m x R double array.  The handle is an sbt_tensor: it takes
 * sbt_update_batch_dense (a batch of K_new last-mode slices, element type
 * per cfg->precision), sbt_fit, sbt_last_sample (mode 0..N-1),
 * sbt_get_batch_counter, sbt_profile_* and sbt_destroy; the third-order
 * calls sbt_get_shape, sbt_get_factors, sbt_update_batch_coo, sbt_fms and
 * sbt_last_rep return SBT_E_STATE on it, and a server refuses it.
 *
 * An update follows Algorithm 1 with N - 1 fixed modes: the importance of
 * every mode (Eq. 1, exact integer sums); per repetition and mode,
 * n_m = ceil(D_m / s_m) indices drawn by the same sampler as for three modes
 * (Philox tag mode field m + 1; the last mode among the existing slices);
 * summaries X(S_0, ..., S_N-2, K_s u new); CP-ALS over modes 0..N-1 with U_1
 * ... U_N-1 drawn U[0,1) (tag mode field m + 1); similarity = product over
 * all N modes of |cosine| with the anchors, maximum-weight assignment, signs
 * and scales from the fixed modes; the summary's last-mode rows by least
 * squares against the Khatri-Rao product of the matched fixed-mode factors,
 * divided by lambda; zero fill of every fixed-mode factor and of the last
 * factor's anchor rows; new rows averaged over the valid repetitions.  At
 * N = 3 it computes what the third-order update computes (plain schedule).
 *
 * Supported (dense; the COO form below): cfg->format SBT_DENSE; cfg->precision
 * SBT_P_F64 or SBT_P_F32
 * (store, summaries and MTTKRP in that type; everything else FP64) or
 * SBT_P_BF16 (FP32 store, summaries rounded to BF16 to nearest even, MTTKRP
 * on the vector units with FP32 accumulation; everything else FP64);
 * getrank_runs 0, persist_summaries 0.  cfg->schedule is not read and
 * cfg->sample_factor is replaced by the per-mode factors below (its entries
 * must still be >= 1).
 * ------------------------------------------------------------------------ */

/* Create an order-N tensor from the dense block X0_dev (device, extents
 * dims[0..N-1], dims[N-1] = K0 existing slices).  sample_factor: N host
 * int32 values >= 1.  factors: NULL, or N host pointers to the row-major
 * factors (last one K0 x R) with lambda0 (R host doubles); both NULL runs
 * cfg->init_iters CP-ALS sweeps on X0 (U_1 ... U_N-1 drawn U[0,1)) and orders
 * the components by lambda.  SBT_E_SHAPE when the product of the fixed
 * extents, or a summary, exceeds 2^31 - 1 entries, or cfg->k_capacity <= K0. */
sbt_status sbt_nd_init_dense(const sbt_config* cfg, int32_t order, const int64_t* dims,
                             const int32_t* sample_factor, const void* X0_dev,
                             const double* const* factors, const double* lambda0, void* stream,
                             sbt_tensor** out);

/* The same for a sparse tensor in COO form (cfg->format SBT_COO, cfg->precision
 * SBT_P_F32: FP32 values, every product and sum FP64): nnz entries with
 * coordinates idx_dev[m][e] (N host pointers to device int32 arrays; the
 * last coordinate in 0..dims[N-1]-1) and values v_dev[e] (device FP32), no
 * coordinate twice; the entries are copied.  cfg->nnz_capacity bounds the
 * entries the tensor can hold; cfg->repetitions <= 255; every extent and
 * cfg->k_capacity below 2^24.  With factors NULL the initial decomposition is
 * CP-ALS on the whole tensor (the sparse MTTKRP of the update on the tensor
 * taken as one summary).  SBT_E_SHAPE for a coordinate outside the extents or
 * more entries than the capacity; SBT_E_NUMERIC for a non-finite value.
 * The update (sbt_nd_update_batch_coo) follows the dense order-N update with
 * the summaries kept sparse: the stored entries whose every coordinate is
 * sampled, re-indexed to the sample positions (Sec. 3.1). */
sbt_status sbt_nd_init_coo(const sbt_config* cfg, int32_t order, const int64_t* dims,
                           const int32_t* sample_factor, const int32_t* const* idx_dev,
                           const float* v_dev, int64_t nnz, const double* const* factors,
                           const double* lambda0, void* stream, sbt_tensor** out);

/* A batch of K_new last-mode slices of a COO order-N tensor: nnz entries
 * (idx_dev: N host pointers to device int32 arrays, the last coordinate
 * batch-relative 0..K_new-1; v_dev device FP32).  Returns when the update is
 * complete.  SBT_E_SHAPE for a coordinate outside the extents, K_new outside
 * 1..max_batch, or capacity (slices or entries) exceeded; SBT_E_NUMERIC for a
 * non-finite value; the tensor is unchanged in both cases.  SBT_E_STATE on a
 * dense tensor. */
sbt_status sbt_nd_update_batch_coo(sbt_tensor* t, const int32_t* const* idx_dev,
                                   const float* v_dev, int64_t nnz, int64_t K_new,
                                   void* stream);

/* Order, extents (N int64 written; the last is the current slice count) and rank. */
sbt_status sbt_nd_get_shape(const sbt_tensor* t, int32_t* order, int64_t* dims, int32_t* R);

/* Copy factor `mode` (D_mode x R, row-major) or lambda (R) to host memory. */
sbt_status sbt_nd_get_factor(sbt_tensor* t, int32_t mode, double* U, void* stream);
sbt_status sbt_nd_get_lambda(sbt_tensor* t, double* lambda, void* stream);

/* Intermediates of repetition `rep` of the last update, as doubles:
 *   SBT_ND_REP_UP    summary factor of `mode` (rows: n_mode, the last mode K')
 *   SBT_ND_REP_UT    matched, sign-fixed, rescaled factor of a fixed mode
 *   SBT_ND_REP_CT    the summary's last-mode rows from the row solve (K' x R)
 *   SBT_ND_REP_LAMP  lambda of the summary's decomposition (R)
 *   SBT_ND_REP_PI    summary column matched to each model column (R)
 *   SBT_ND_REP_VALID 1 where the component counts in the averages (R)
 * *n_out = values written; SBT_E_SHAPE when max_values is too small. */
enum {
  SBT_ND_REP_UP = 0,
  SBT_ND_REP_UT = 1,
  SBT_ND_REP_CT = 2,
  SBT_ND_REP_LAMP = 3,
  SBT_ND_REP_PI = 4,
  SBT_ND_REP_VALID = 5
};
sbt_status sbt_nd_last_rep(const sbt_tensor* t, int32_t rep, int32_t item, int32_t mode,
                           double* out, int64_t max_values, int64_t* n_out);

/* Human-readable text for a status, and the last error message of a tensor. */
const char* sbt_status_str(sbt_status s);
const char* sbt_last_error(const sbt_tensor* t);

#ifdef __cplusplus
}
#endif

#endif /* SAMBATEN_H */
