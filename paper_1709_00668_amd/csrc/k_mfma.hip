// BF16 summaries on the matrix cores (MFMA) for the batched CP-ALS sweeps.
//
// The summaries are rounded to BF16 (nearest even) once per update and kept
// in two layouts, so that the contracted index of each pass is contiguous
// for the K-packed MFMA operands:
//
//   Zk[rep][c][e']   e' = a + ld1 * b  (ld1 = n1 rounded up to 8, rows of a
//                    slice padded to sk, a multiple of 32, with zeros)
//                    -> mode 3: rows c of C' = Zk (B~ kr A~), K = e'
//   Zc[rep][e][c]    e = a + n1 * b, c padded to ldc (multiple of 32)
//                    -> pass W: W(e, :) = Zc(e, :) C~, K = c
//
// Both passes run v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  The
// second operand (C~ for pass W, the Khatri-Rao rows A~(a, f) B~(b, f) for
// mode 3) is formed in FP32 and split into BF16 parts, each contracted with
// the summary into one accumulator: three parts for C~ (hi = bf16(x), mid =
// bf16(x - hi), lo = bf16(x - hi - mid): about 24 bits, as in FP32), two for
// the Khatri-Rao rows (hi and lo: about 16 bits; they are formed per lane in
// every K step, where a third part would cost VALU work the pass cannot
// hide).  Only the data are BF16.  Rounding the factor operand itself to
// BF16 makes the MTTKRP inconsistent with the FP64 Gram matrices of the
// normal equations, and with the nearly collinear factors of non-negative
// data that inconsistency is amplified by the conditioning of the solve (the
// fit of an update drops by several 1e-3).  The split costs MFMA issue slots
// the memory-bound passes have to spare.  Modes 1 and 2 then contract W
// (FP32) as in the other precisions; Gram matrices, solves and normalisation
// stay in FP64.
//
// Lane layout of the 16 x 16 x 32 operation (wave of 64): operand A row
// i = lane % 16 holds 8 consecutive K entries of group lane / 16; operand B
// column j = lane % 16 likewise; result lane holds rows 4 (lane / 16) + v,
// v = 0..3, of column lane % 16.  A and B use the same K grouping, so the
// hardware's internal order of K does not matter.
#include "../../include/sambaten.h"
#include "device_common.hpp"
#include "kernels.hpp"

namespace sbt {

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ inline f32x4_t mfma16x16x32(const bf16x8_t& a, const bf16x8_t& b,
                                       const f32x4_t& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__device__ inline bf16x8_t ld_bf16x8(const uint16_t* p) {
  return *reinterpret_cast<const bf16x8_t*>(p);
}

// x = hi + lo with hi = bf16(x) (nearest even) and lo = bf16(x - hi), for
// 8 values at once
__device__ inline void split_bf16x8(const float (&x)[8], bf16x8_t& hi, bf16x8_t& lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const __bf16 h = (__bf16)x[j];
    hi[j] = h;
    lo[j] = (__bf16)(x[j] - (float)h);
  }
}

// ---------------------------------------------------------------------------
// gather: both layouts from the resident store in one pass
// ---------------------------------------------------------------------------
// thread = (e, run of G groups of 8 third-mode positions): with G = 8 the
// thread writes whole 128-byte lines of its Zc row (the groups of a run are
// consecutive), gathering one group of 8 slices at a time; c >= K' are
// written as zeros in Zc (the K range of pass W is K' rounded up to 32).
// G only shapes the launch: every choice writes the same bytes.
constexpr int kGatherChoices[3] = {8, 4, 16};

template <typename TIn, int G>
__global__ __launch_bounds__(256) void gather_mfma_kernel(const TIn* X, int64_t I, int64_t J,
                                                         const int32_t* idx, int64_t idx_stride,
                                                         int64_t offJ, int64_t offK, int n3old,
                                                         int64_t Kold, int cg0, int ncg,
                                                         RepSet rs, MfmaLayout L, uint16_t* Zk,
                                                         uint16_t* Zc) {
  const int rep = rs.rep0 + blockIdx.z;
  const int g0 = cg0 + (int)blockIdx.y * G;
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int32_t* Is = idx + rep * idx_stride;
  // the slices of the block's positions, read once into LDS (-1: c >= K')
  __shared__ int64_t ksl[G * 8];
  if (threadIdx.x < G * 8) {
    const int c = g0 * 8 + (int)threadIdx.x;
    int64_t k = -1;
    if (c < rs.n3) k = c < n3old ? (int64_t)Is[offK + c] : Kold + (c - n3old);
    ksl[threadIdx.x] = k;
  }
  __syncthreads();
  if (e >= n12) return;
  const int a = (int)(e % rs.n1), b = (int)(e / rs.n1);
  const int64_t base = (int64_t)Is[a] + I * (int64_t)Is[offJ + b];
  uint16_t* zk = Zk + rep * L.sZk + a + (int64_t)L.ld1 * b;
  uint16_t* zc = Zc + rep * L.sZc + e * L.ldc;
  for (int cg = g0; cg < g0 + G && cg < cg0 + ncg; ++cg) {
    // the group's eight loads in flight together (positions c >= K' read
    // slice 0 of the store and are dropped)
    TIn x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t kk = ksl[(cg - g0) * 8 + j];
      x[j] = X[base + I * J * (kk >= 0 ? kk : 0)];
    }
    uint16_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = cg * 8 + j;
      v[j] = 0;
      if (c < rs.n3) {
        v[j] = f32_to_bf16_rne((float)x[j]);
        zk[L.sk * c] = v[j];
      }
    }
    uint4 pk;
    pk.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
    pk.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
    pk.z = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
    pk.w = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
    *reinterpret_cast<uint4*>(zc + cg * 8) = pk;
  }
}

// BF16 tensor (column-major bits) -> both layouts, for the stand-alone MTTKRP.
__global__ __launch_bounds__(256) void relayout_bf16_kernel(const uint16_t* Z, RepSet rs,
                                                           MfmaLayout L, uint16_t* Zk,
                                                           uint16_t* Zc) {
  const int cg = blockIdx.y;
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n12) return;
  const int a = (int)(e % rs.n1), b = (int)(e / rs.n1);
  uint16_t v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int c = cg * 8 + j;
    v[j] = 0;
    if (c < rs.n3) {
      v[j] = Z[e + n12 * c];
      Zk[L.sk * c + a + (int64_t)L.ld1 * b] = v[j];
    }
  }
  uint4 pk;
  pk.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
  pk.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
  pk.z = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
  pk.w = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
  *reinterpret_cast<uint4*>(Zc + e * L.ldc + cg * 8) = pk;
}

// ---------------------------------------------------------------------------
// operands staged once per launch
// ---------------------------------------------------------------------------
// C~^T as three BF16 parts: Ct[rep][part][f][kp32 + 8] (rows f >= R and
// columns c >= K' zero)
__global__ void ct_split_kernel(RepSet rs, int kp32, int nf, const double* Cf,
                                const double* invlamC, uint16_t* Ct) {
  const int rep = rs.rep0 + blockIdx.y;
  const int R = rs.R, ldt = kp32 + 8;
  const int64_t n = (int64_t)nf * ldt;
  const double* C = Cf + rep * rs.sC;
  uint16_t* hi = Ct + (int64_t)rep * 3 * n;
  uint16_t* mid = hi + n;
  uint16_t* lo = mid + n;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int f = (int)(q / ldt), c = (int)(q % ldt);
    float x = 0.0f;
    if (f < R && c < rs.n3)
      x = (float)(C[(int64_t)c * R + f] * (invlamC ? invlamC[rep * 3 * R + f] : 1.0));
    const uint16_t h = f32_to_bf16_rne(x);
    const float r1 = x - bf16_to_f32(h);  // exact
    const uint16_t m = f32_to_bf16_rne(r1);
    hi[q] = h;
    mid[q] = m;
    lo[q] = f32_to_bf16_rne(r1 - bf16_to_f32(m));
  }
}

// A~^T and B~^T in FP32: Ft[rep][f][ld] (rows f >= R and columns >= rows zero)
__global__ void ft_kernel(RepSet rs, int rows, int ld, int nf, const double* F, int64_t sF,
                          const double* invlam, float* Ft) {
  const int rep = rs.rep0 + blockIdx.y;
  const int R = rs.R;
  const int64_t n = (int64_t)nf * ld;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int f = (int)(q / ld), a = (int)(q % ld);
    float x = 0.0f;
    if (f < R && a < rows)
      x = (float)(F[rep * sF + (int64_t)a * R + f] * (invlam ? invlam[rep * 3 * R + f] : 1.0));
    Ft[(int64_t)rep * n + q] = x;
  }
}

// ---------------------------------------------------------------------------
// pass W on the matrix cores
// ---------------------------------------------------------------------------
// Block = 4 wavefronts x WT tiles of 16 rows e (64 WT rows) of one repetition;
// every wave runs the whole K range (K' rounded up to 32) against the three
// parts of C~^T, whose R live rows are copied into LDS by the block in chunks
// of at most pw_mfma_chunk(R) columns (one chunk, staged once, whenever K'
// fits; a barrier between chunks otherwise); lanes of the column tiles
// beyond R take zero operands.  One accumulator per tile takes the three
// products: the four tiles' hi products go first, then mid, then lo, so each
// accumulation has three independent MFMAs between it and the one it
// depends on.
constexpr int kStageBatch = 4;  // staging loads a thread issues before its stores
// row tiles per wavefront (WT): 4, 2 or 1; each output row's sums run over
// the same K steps in the same order whatever WT, so it only shapes the launch
constexpr int kWTileChoices[3] = {4, 2, 1};
constexpr int kWSteps = 2;   // K steps whose operand loads are in flight at once

// columns of C~ staged per chunk: three parts' rows [R][chunk + 8] of BF16
// within 52 KB (three blocks per compute unit), a multiple of 32
constexpr int kPwLds = 52 * 1024;
constexpr int pw_mfma_chunk(int R) { return (kPwLds / (3 * R * 2) - 8) / 32 * 32; }

template <int NT, int WT>
__global__ __launch_bounds__(256) void pw_mfma_kernel(RepSet rs, MfmaLayout L, int kp32,
                                                     int chunk, const uint16_t* Zc,
                                                     const uint16_t* Ctg, float* W) {
  extern __shared__ __align__(16) unsigned char pwm_smem[];
  const int R = rs.R;
  const int ldg = kp32 + 8;                            // row stride of the global C~ rows
  const int ldt = chunk + 8;                           // row stride in LDS
  uint16_t* Ct = reinterpret_cast<uint16_t*>(pwm_smem);  // hi part [R][ldt], then mid, lo
  const uint16_t* Cm = Ct + R * ldt;
  const uint16_t* Cl = Cm + R * ldt;
  const int rep = rs.rep0 + blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform (scalar)
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  const int64_t e0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * WT);
  const int kq = lane >> 4;
  const uint16_t* zrow[WT];
#pragma unroll
  for (int t = 0; t < WT; ++t) {
    const int64_t e = e0 + 16 * t + (lane & 15);
    zrow[t] = Zc + rep * L.sZc + (e < n12 ? e : n12 - 1) * L.ldc + 8 * kq;
  }
  f32x4_t acc[WT][NT];
#pragma unroll
  for (int t = 0; t < WT; ++t)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[t][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  const u32x4_t* src = reinterpret_cast<const u32x4_t*>(Ctg + (int64_t)rep * 3 * 16 * NT * ldg);
  u32x4_t* dst = reinterpret_cast<u32x4_t*>(Ct);
  bf16x8_t af[kWSteps][WT];
  for (int c0 = 0; c0 < kp32; c0 += chunk) {
    const int cw = kp32 - c0 < chunk ? kp32 - c0 : chunk;  // a multiple of 32
    const int ksteps = cw / 32;
    const uint16_t* zc[WT];
#pragma unroll
    for (int t = 0; t < WT; ++t) zc[t] = zrow[t] + c0;
    // first operand loads of the chunk before its staging
#pragma unroll
    for (int u = 0; u < kWSteps; ++u)
#pragma unroll
      for (int t = 0; t < WT; ++t)
        if (u < ksteps) af[u][t] = ld_bf16x8(zc[t] + 32 * u);
    if (c0 > 0) __syncthreads();  // every wave is done with the previous chunk
    {
      // 16-byte words: the R live rows of hi, then of mid and lo, cw / 8 words
      // each; a thread issues a batch of loads before its stores
      const int wpr = cw / 8, nw = 3 * R * wpr;
      for (int q0 = tid; q0 < nw; q0 += kStageBatch * 256) {
        // (loads past the end read word 0 again, so the batch has no branch)
        u32x4_t v[kStageBatch];
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
          const int q = q0 + u * 256 < nw ? q0 + u * 256 : 0;
          const int row = q / wpr, w = q - row * wpr;
          const int grow = (row / R) * 16 * NT + row % R;  // row in the global layout
          v[u] = src[grow * (ldg / 8) + c0 / 8 + w];
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the whole batch of loads ahead of the stores
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
          const int q = q0 + u * 256;
          if (q < nw) {
            const int row = q / wpr, w = q - row * wpr;
            dst[row * (ldt / 8) + w] = v[u];
          }
        }
      }
    }
    __syncthreads();
    for (int k0 = 0; k0 < ksteps; k0 += kWSteps) {
      if (k0 > 0) {
#pragma unroll
        for (int u = 0; u < kWSteps; ++u)
#pragma unroll
          for (int t = 0; t < WT; ++t)
            if (k0 + u < ksteps) af[u][t] = ld_bf16x8(zc[t] + 32 * (k0 + u));
      }
#pragma unroll
      for (int u = 0; u < kWSteps; ++u) {
        if (k0 + u < ksteps) {
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            const int f = 16 * j + (lane & 15);
            const int o = f * ldt + 32 * (k0 + u) + 8 * kq;
            bf16x8_t bh = {}, bm = {}, bl = {};
            if (f < R) {
              bh = ld_bf16x8(Ct + o);
              bm = ld_bf16x8(Cm + o);
              bl = ld_bf16x8(Cl + o);
            }
#pragma unroll
            for (int t = 0; t < WT; ++t) acc[t][j] = mfma16x16x32(af[u][t], bh, acc[t][j]);
#pragma unroll
            for (int t = 0; t < WT; ++t) acc[t][j] = mfma16x16x32(af[u][t], bm, acc[t][j]);
#pragma unroll
            for (int t = 0; t < WT; ++t) acc[t][j] = mfma16x16x32(af[u][t], bl, acc[t][j]);
          }
        }
      }
    }
  }
  float* Wr = W + rep * rs.sW;
#pragma unroll
  for (int t = 0; t < WT; ++t)
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int f = 16 * j + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t e = e0 + 16 * t + 4 * kq + v;
        if (e < n12 && f < R) Wr[e * R + f] = acc[t][j][v];
      }
    }
}

// ---------------------------------------------------------------------------
// mode 3 on the matrix cores
// ---------------------------------------------------------------------------
// Block = 64 consecutive rows c of one repetition over one of nsplit ranges
// of the K steps; each of its four wavefronts takes all 64 rows (four row
// tiles) over a quarter of the block's K range, so the Khatri-Rao operand a
// wave forms per lane (from A~^T, all of it, and the B~^T rows the block's
// range touches, both copied into LDS from their FP32 transposes) serves four
// MFMA row tiles.  The four quarters' partial rows are added through LDS in
// wave order; the block's partial rows go to P[rep][split][c][16 NT], and
// mode3_finish adds the ranges in order and applies V^-1.
constexpr int kPTiles = 4;  // row tiles of 16 per wavefront (the block's 64 rows)
// K steps whose operand loads are in flight at once (PS): 2, 1 or 4; the
// steps are taken in the same order whatever PS, so it only shapes the launch
constexpr int kPStepChoices[3] = {2, 1, 4};
static_assert(SBT_TUNE_SHAPES == 3, "one entry per launch shape in each choice table");

template <int NT, int PS>
__global__ __launch_bounds__(256) void p3_mfma_kernel(RepSet rs, MfmaLayout L, int nsplit,
                                                     const uint16_t* Zk, const float* Atg,
                                                     const float* Btg, float* P, int64_t sP) {
  extern __shared__ __align__(16) unsigned char p3m_smem[];
  float* At = reinterpret_cast<float*>(p3m_smem);  // [16 NT][ld1]
  const int rep = rs.rep0 + blockIdx.z;
  const int split = blockIdx.y;
  const int n2 = rs.n2, n3 = rs.n3, ld1 = L.ld1;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int ksteps = (int)(L.sk / 32);
  const int ks_lo = (int)((int64_t)split * ksteps / nsplit);
  const int ks_hi = (int)((int64_t)(split + 1) * ksteps / nsplit);
  const int b_lo = (ks_lo * 32) / ld1;
  int b_hi = ks_hi > ks_lo ? (ks_hi * 32 - 1) / ld1 : b_lo;
  if (b_hi > n2 - 1) b_hi = n2 - 1;
  const int nb = b_hi >= b_lo ? b_hi - b_lo + 1 : 0;
  const int nbp = (nb + 3) / 4 * 4;  // row stride of the staged B~^T rows
  float* Bt = At + 16 * NT * ld1;     // [16 NT][nbp]
  // this wave's quarter of the block's K range
  const int kw_lo = ks_lo + (int)((int64_t)wave * (ks_hi - ks_lo) / 4);
  const int kw_hi = ks_lo + (int)((int64_t)(wave + 1) * (ks_hi - ks_lo) / 4);
  const int c0 = blockIdx.x * 64;
  const int kq = lane >> 4;
  const uint16_t* zrow[kPTiles];
#pragma unroll
  for (int t = 0; t < kPTiles; ++t) {
    const int c = c0 + 16 * t + (lane & 15);
    zrow[t] = Zk + rep * L.sZk + (int64_t)(c < n3 ? c : n3 - 1) * L.sk + 8 * kq;
  }
  bf16x8_t af[PS][kPTiles];
#pragma unroll
  for (int u = 0; u < PS; ++u)
#pragma unroll
    for (int t = 0; t < kPTiles; ++t)
      if (kw_lo + u < kw_hi) af[u][t] = ld_bf16x8(zrow[t] + 32 * (kw_lo + u));
  {
    // a thread issues a batch of loads before its stores
    const int n4 = 16 * NT * ld1 / 4;
    const u32x4_t* src = reinterpret_cast<const u32x4_t*>(Atg + (int64_t)rep * 16 * NT * ld1);
    u32x4_t* dst = reinterpret_cast<u32x4_t*>(At);
    for (int q0 = tid; q0 < n4; q0 += kStageBatch * 256) {
      // (loads past the end read word 0 again, so the batch has no branch)
      u32x4_t v[kStageBatch];
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) v[u] = src[q0 + u * 256 < n4 ? q0 + u * 256 : 0];
      __builtin_amdgcn_sched_barrier(0);  // keep the whole batch of loads ahead of the stores
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u)
        if (q0 + u * 256 < n4) dst[q0 + u * 256] = v[u];
    }
    const int ldb = (n2 + 3) / 4 * 4;
    const float* bsrc = Btg + (int64_t)rep * 16 * NT * ldb;
    const int nbt = 16 * NT * nbp;
    for (int q0 = tid; q0 < nbt; q0 += kStageBatch * 256) {
      float v[kStageBatch];
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int q = q0 + u * 256;
        const int f = q / nbp, bb = q % nbp;
        const bool in = q < nbt && bb < nb;
        const float x = bsrc[in ? (int64_t)f * ldb + b_lo + bb : 0];
        v[u] = in ? x : 0.0f;
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u)
        if (q0 + u * 256 < nbt) Bt[q0 + u * 256] = v[u];
    }
  }
  __syncthreads();
  // one accumulator per tile takes both the hi and the lo product: the four
  // tiles' hi products go first, then their lo products, so each accumulation
  // has three independent MFMAs between it and the one it depends on
  f32x4_t acc[kPTiles][NT];
#pragma unroll
  for (int t = 0; t < kPTiles; ++t)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[t][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kw_lo; k0 < kw_hi; k0 += PS) {
    if (k0 > kw_lo) {
#pragma unroll
      for (int u = 0; u < PS; ++u)
#pragma unroll
        for (int t = 0; t < kPTiles; ++t)
          if (k0 + u < kw_hi) af[u][t] = ld_bf16x8(zrow[t] + 32 * (k0 + u));
    }
#pragma unroll
    for (int u = 0; u < PS; ++u) {
      if (k0 + u < kw_hi) {
        // this lane's 8 consecutive e' share one b (ld1 is a multiple of 8)
        const int ep = 32 * (k0 + u) + 8 * kq;
        const int a0 = ep % ld1, b = ep / ld1;
        const bool bin = b <= b_hi;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const int f = 16 * j + (lane & 15);
          const float4 x0 = *reinterpret_cast<const float4*>(At + f * ld1 + a0);
          const float4 x1 = *reinterpret_cast<const float4*>(At + f * ld1 + a0 + 4);
          const float bv = bin ? Bt[f * nbp + (b - b_lo)] : 0.0f;
          const float x[8] = {x0.x * bv, x0.y * bv, x0.z * bv, x0.w * bv,
                              x1.x * bv, x1.y * bv, x1.z * bv, x1.w * bv};
          bf16x8_t kh, kl;
          split_bf16x8(x, kh, kl);
#pragma unroll
          for (int t = 0; t < kPTiles; ++t) acc[t][j] = mfma16x16x32(af[u][t], kh, acc[t][j]);
#pragma unroll
          for (int t = 0; t < kPTiles; ++t) acc[t][j] = mfma16x16x32(af[u][t], kl, acc[t][j]);
        }
      }
    }
  }
  // the quarters' partial rows, added in wave order (the staging is no longer read)
  __syncthreads();
  float* red = reinterpret_cast<float*>(p3m_smem);  // [wave][64 rows][16 NT]
  constexpr int kRow = 16 * NT;
#pragma unroll
  for (int t = 0; t < kPTiles; ++t)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        red[(wave * 64 + 16 * t + 4 * kq + v) * kRow + 16 * j + (lane & 15)] = acc[t][j][v];
  __syncthreads();
  float* Pr = P + (rep * (int64_t)nsplit + split) * sP;
  for (int q = tid; q < 64 * kRow; q += 256) {
    const int c = c0 + q / kRow;
    if (c < n3)
      Pr[(int64_t)c0 * kRow + q] = ((red[q] + red[64 * kRow + q]) + red[2 * 64 * kRow + q]) +
                                   red[3 * 64 * kRow + q];
  }
}

// rows of C: sum of the split partials (in split order), times V^-1, divided
// by lam_div for the row solve.  Block = 8 rows of one repetition.
__global__ __launch_bounds__(256) void mode3_finish_kernel(RepSet rs, int nsplit, int ldp,
                                                          const float* P, int64_t sP,
                                                          const double* Vinv,
                                                          const double* lam_div, double* Uout,
                                                          int64_t sU, double* gpart,
                                                          int64_t sGpart) {
  __shared__ double M[8][kMaxRank];
  __shared__ double Ub[8][kMaxRank];
  __shared__ double Vi[kMaxRank][kMaxRank + 1];
  const int rep = rs.rep0 + blockIdx.y;
  const int R = rs.R;
  const int tid = threadIdx.x;
  for (int q = tid; q < R * R; q += 256) Vi[q / R][q % R] = Vinv[rep * rs.sG + q];
  const int r = tid / kMaxRank, f = tid % kMaxRank;
  const int c = blockIdx.x * 8 + r;
  if (c < rs.n3 && f < R) {
    double m = 0.0;
    for (int sp = 0; sp < nsplit; ++sp)
      m += (double)P[(rep * (int64_t)nsplit + sp) * sP + (int64_t)c * ldp + f];
    M[r][f] = m;
  }
  __syncthreads();
  double u = 0.0;
  if (c < rs.n3 && f < R) {
    for (int k = 0; k < R; ++k) u += M[r][k] * Vi[k][f];
    if (lam_div) {
      const double l = lam_div[f];
      u = l > 0.0 ? u / l : 0.0;
    }
    Uout[rep * sU + (int64_t)c * R + f] = u;
  }
  if (gpart) {
    // the Gram matrix of the block's eight rows (rows past n3 are zero), in
    // row order, both triangles
    Ub[r][f] = u;
    __syncthreads();
    double* out = gpart + rep * sGpart + (int64_t)blockIdx.x * R * R;
    for (int q = tid; q < R * R; q += 256) {
      const int a = q / R, b = q % R;
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < 8; ++i) acc += Ub[i][a] * Ub[i][b];
      out[q] = acc;
    }
  }
}

inline int ntiles(int R) { return R <= 16 ? 1 : 2; }

}  // namespace

MfmaLayout mfma_layout(int n1, int n2, int kpmax) {
  MfmaLayout L;
  L.ld1 = (n1 + 7) / 8 * 8;
  L.sk = ((int64_t)L.ld1 * n2 + 31) / 32 * 32;
  L.ldc = (kpmax + 31) / 32 * 32;
  L.sZk = (int64_t)kpmax * L.sk;
  L.sZc = (int64_t)n1 * n2 * L.ldc;
  return L;
}

// B~ rows one K range of the mode-3 kernel may touch (LDS bound)
constexpr int kMaxBRows = 64;

inline int brows_cap(int n2) { return n2 < kMaxBRows ? n2 : kMaxBRows; }

bool mfma_supported(int n1, int n2, int R) {
  if (R > 32 || n1 < 1 || n2 < 1) return false;
  // LDS of the mode-3 kernel: A~^T plus the B~^T rows of one K range
  const size_t lds =
      (size_t)16 * ntiles(R) * 4 * ((size_t)(n1 + 7) / 8 * 8 + (brows_cap(n2) + 3) / 4 * 4);
  return lds <= 65536;
}

// rows of B~ the K range [ks_lo, ks_hi) of a split touches, at most
inline int brows_of(int ksteps, int nsplit, int ld1) {
  const int per = (ksteps + nsplit - 1) / nsplit;  // K steps of the longest range
  return (per * 32 + ld1 - 1) / ld1 + 1;
}

int mfma_mode3_splits(const RepSet& rs, const MfmaLayout& L) {
  const int cblocks = (rs.n3 + 63) / 64;
  const int ksteps = (int)(L.sk / 32);
  int ns = (2048 + cblocks * rs.nrep - 1) / (cblocks * rs.nrep);
  const int cap = ksteps / 8 > 0 ? ksteps / 8 : 1;
  if (ns > cap) ns = cap;
  if (ns < 1) ns = 1;
  // enough ranges that each touches at most brows_cap(n2) rows of B~
  while (ns < ksteps && brows_of(ksteps, ns, L.ld1) > brows_cap(rs.n2)) ++ns;
  return ns;
}

hipError_t launch_gather_mfma(int store_prec, const void* X, int64_t I, int64_t J,
                              const int32_t* idx, int64_t idx_stride, int64_t offJ, int64_t offK,
                              int n3old, int64_t Kold, int c0, const RepSet& rs,
                              const MfmaLayout& L, uint16_t* Zk, uint16_t* Zc, hipStream_t s,
                              int choice) {
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  const int kp32 = (rs.n3 + 31) / 32 * 32;
  if (c0 < 0 || c0 >= rs.n3 || choice < 0 || choice >= SBT_TUNE_SHAPES) return hipErrorInvalidValue;
  const int cg0 = c0 / 8;  // groups of 8 slices, the first one gathered whole
  const int ncg = kp32 / 8 - cg0;
  const int G = kGatherChoices[choice];
  dim3 grid((unsigned)((n12 + 255) / 256), (unsigned)((ncg + G - 1) / G), (unsigned)rs.nrep);
#define SBT_GATHER(T, GG)                                                                    \
  timed_launch(gather_mfma_kernel<T, GG>, grid, dim3(256), 0, s, (const T*)X, I, J, idx,      \
               idx_stride, offJ, offK, n3old, Kold, cg0, ncg, rs, L, Zk, Zc)
  if (store_prec == kF64) {
    if (G == 8) SBT_GATHER(double, 8);
    else if (G == 4) SBT_GATHER(double, 4);
    else SBT_GATHER(double, 16);
  } else {
    if (G == 8) SBT_GATHER(float, 8);
    else if (G == 4) SBT_GATHER(float, 4);
    else SBT_GATHER(float, 16);
  }
#undef SBT_GATHER
  return hipGetLastError();
}

hipError_t launch_relayout_bf16(const uint16_t* Z, const RepSet& rs, const MfmaLayout& L,
                                uint16_t* Zk, uint16_t* Zc, hipStream_t s) {
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  const int kp32 = (rs.n3 + 31) / 32 * 32;
  dim3 grid((unsigned)((n12 + 255) / 256), (unsigned)(kp32 / 8));
  relayout_bf16_kernel<<<grid, 256, 0, s>>>(Z, rs, L, Zk, Zc);
  return hipGetLastError();
}

size_t mfma_operand_floats(const MfmaLayout& L, int n2, int R) {
  const size_t nf = 16 * ntiles(R);
  const size_t ct = nf * ((size_t)L.ldc + 8) * 3 / 2;      // three parts' BF16 rows
  const size_t ab = nf * ((size_t)L.ld1 + (n2 + 3) / 4 * 4);  // A~^T and B~^T in FP32
  return ct > ab ? ct : ab;
}

hipError_t launch_pw_mfma(const RepSet& rs, const MfmaLayout& L, const uint16_t* Zc,
                          const double* Cf, const double* invlamC, float* W, float* ops,
                          hipStream_t s, int choice) {
  if (choice < 0 || choice >= SBT_TUNE_SHAPES) return hipErrorInvalidValue;
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  const int kp32 = (rs.n3 + 31) / 32 * 32;
  if (kp32 > L.ldc) return hipErrorInvalidValue;
  const int nt = ntiles(rs.R), nf = 16 * nt;
  uint16_t* Ct = reinterpret_cast<uint16_t*>(ops);
  {
    const int64_t n = (int64_t)nf * (kp32 + 8);
    int blocks = (int)((n + 255) / 256);
    if (blocks > 256) blocks = 256;
    ct_split_kernel<<<dim3((unsigned)blocks, (unsigned)rs.nrep), 256, 0, s>>>(rs, kp32, nf, Cf,
                                                                            invlamC, Ct);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int WT = kWTileChoices[choice];
  const int64_t rows_per_block = 4 * 16 * WT;
  dim3 grid((unsigned)((n12 + rows_per_block - 1) / rows_per_block), (unsigned)rs.nrep);
  const int chunk = kp32 < pw_mfma_chunk(rs.R) ? kp32 : pw_mfma_chunk(rs.R);
  const size_t sh = (size_t)3 * rs.R * (chunk + 8) * 2;
  if (sh > 65536) return hipErrorInvalidValue;
#define SBT_PW(NTT, WTT)                                                                      \
  timed_launch(pw_mfma_kernel<NTT, WTT>, grid, dim3(256), sh, s, rs, L, kp32, chunk, Zc, Ct, W)
  if (nt == 1) {
    if (WT == 4) SBT_PW(1, 4);
    else if (WT == 2) SBT_PW(1, 2);
    else SBT_PW(1, 1);
  } else {
    if (WT == 4) SBT_PW(2, 4);
    else if (WT == 2) SBT_PW(2, 2);
    else SBT_PW(2, 1);
  }
#undef SBT_PW
  return hipGetLastError();
}

hipError_t launch_p3_mfma(const RepSet& rs, const MfmaLayout& L, int nsplit, const uint16_t* Zk,
                          const double* Af, const double* invlamA, const double* Bf,
                          const double* invlamB, float* P, int64_t sP, float* ops,
                          hipStream_t s, int choice) {
  if (choice < 0 || choice >= SBT_TUNE_SHAPES) return hipErrorInvalidValue;
  const int nt = ntiles(rs.R), nf = 16 * nt;
  const int ldb = (rs.n2 + 3) / 4 * 4;
  float* Atg = ops;
  float* Btg = ops + (size_t)(rs.rep0 + rs.nrep) * nf * L.ld1;
  {
    // transposes for repetitions [rep0, rep0 + nrep) at their absolute offsets
    const int64_t na = (int64_t)nf * L.ld1, nb = (int64_t)nf * ldb;
    int ba = (int)((na + 255) / 256), bb = (int)((nb + 255) / 256);
    if (ba > 256) ba = 256;
    if (bb > 256) bb = 256;
    ft_kernel<<<dim3((unsigned)ba, (unsigned)rs.nrep), 256, 0, s>>>(rs, rs.n1, L.ld1, nf, Af,
                                                                   rs.sA, invlamA, Atg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ft_kernel<<<dim3((unsigned)bb, (unsigned)rs.nrep), 256, 0, s>>>(rs, rs.n2, ldb, nf, Bf,
                                                                   rs.sB, invlamB, Btg);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  dim3 grid((unsigned)((rs.n3 + 63) / 64), (unsigned)nsplit, (unsigned)rs.nrep);
  const int ksteps = (int)(L.sk / 32);
  int nbmax = brows_of(ksteps, nsplit, L.ld1);
  if (nbmax > rs.n2) nbmax = rs.n2;
  size_t sh = (size_t)nf * 4 * ((size_t)L.ld1 + (nbmax + 3) / 4 * 4);
  const size_t red = (size_t)4 * 64 * nf * 4;  // the four quarters' partial rows
  if (sh < red) sh = red;
  if (sh > 65536 || sP < (int64_t)rs.n3 * nf) return hipErrorInvalidValue;
  const int PS = kPStepChoices[choice];
#define SBT_P3(NTT, PSS)                                                                      \
  timed_launch(p3_mfma_kernel<NTT, PSS>, grid, dim3(256), sh, s, rs, L, nsplit, Zk, Atg, Btg, \
               P, sP)
  if (nt == 1) {
    if (PS == 2) SBT_P3(1, 2);
    else if (PS == 1) SBT_P3(1, 1);
    else SBT_P3(1, 4);
  } else {
    if (PS == 2) SBT_P3(2, 2);
    else if (PS == 1) SBT_P3(2, 1);
    else SBT_P3(2, 4);
  }
#undef SBT_P3
  return hipGetLastError();
}

hipError_t launch_mode3_finish(const RepSet& rs, int nsplit, const float* P, int64_t sP,
                               const double* Vinv, const double* lam_div, double* U, int64_t sU,
                               hipStream_t s, double* gpart, int64_t sGpart) {
  // eight rows per block: gram_parts(rows) blocks when gpart is given
  if (gpart && gram_parts(8) != 1) return hipErrorInvalidValue;
  dim3 grid((unsigned)((rs.n3 + 7) / 8), (unsigned)rs.nrep);
  mode3_finish_kernel<<<grid, 256, 0, s>>>(rs, nsplit, 16 * ntiles(rs.R), P, sP, Vinv, lam_div,
                                           U, sU, gpart, sGpart);
  return hipGetLastError();
}

}  // namespace sbt
