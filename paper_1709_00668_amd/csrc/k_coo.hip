// Sparse (COO) path of the SamBaTen update: ingest, summary gather, CP-ALS
// MTTKRP on the summaries, fit.  Everything is deterministic: no floating
// point atomics; integer counts only.
//
// Store: structure of arrays (i, j, k, v), kept sorted by the slice index k
// (each batch is stably sorted by k on ingest; batches arrive in slice
// order), with per-slice offsets koff.
//
// Summary of repetition rho = the stored entries with i in I_s, j in J_s and
// k in K_s u new (Sec. 3.1), re-indexed to (a, b, c).  Emitted in store order,
// it is sorted by c.  Modes 1 and 2 need the entries grouped by a and by b:
// one stable radix sort of the keys (rho, a) and (rho, b) per update gives
// those orders (the summaries stay fixed over all ALS sweeps).  Each mode's
// MTTKRP is then one wavefront per output row over a contiguous segment.
#include <hipcub/hipcub.hpp>

#include "device_common.hpp"
#include "kernels.hpp"

namespace sbt {

namespace {

constexpr int kCooBlock = 256;
constexpr int kCooPerThread = 16;                       // entries per thread in scans
constexpr int kCooChunk = kCooBlock * kCooPerThread;    // entries per block in scans

inline int grid_for(int64_t n, int per_block) {
  int64_t b = (n + per_block - 1) / per_block;
  return (int)(b < 1 ? 1 : b);
}

// --------------------------------------------------------------------------
// ingest
// --------------------------------------------------------------------------
__global__ void iota_kernel(int32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int32_t)i;
}

__global__ void copy_u32_kernel(const int32_t* src, uint32_t* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (uint32_t)src[i];
}

// store[base + p] = batch[perm[p]] with k shifted by koff0; slice histogram
__global__ void coo_place_kernel(const int32_t* bi, const int32_t* bj, const int32_t* bk,
                                 const float* bv, const int32_t* perm, int64_t n, int64_t knew,
                                 int64_t kshift,
                                 int32_t* si, int32_t* sj, int32_t* sk, float* sv, int64_t base,
                                 uint32_t* khist) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t e = perm[p];
    const int32_t k = bk[e];
    si[base + p] = bi[e];
    sj[base + p] = bj[e];
    sk[base + p] = (int32_t)(k + kshift);
    sv[base + p] = bv[e];
    if (k >= 0 && k < knew) atomicAdd(&khist[k], 1u);
  }
}

// Exclusive scans of several count arrays at once, one block per array:
// out_b[0..n] = base_b + exclusive prefix sums of cnt_b[0..n), out_b[n] the
// total (cnt_b = cnt + b * scnt, out_b = out + b * sout, base_b = base0 plus
// bases[b] when given).  Each thread adds up kScanItems consecutive counts before the wave and
// block scans, so a block covers 8192 counts per round.
constexpr int kScanItems = 8;

__global__ __launch_bounds__(1024) void scan_to_offsets_kernel(const uint32_t* cnt, int64_t scnt,
                                                              int64_t n, int64_t base0,
                                                              const int64_t* bases, int64_t* out,
                                                              int64_t sout) {
  __shared__ int64_t wsum[16];
  __shared__ int64_t carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t* c = cnt + (int64_t)blockIdx.x * scnt;
  int64_t* o = out + (int64_t)blockIdx.x * sout;
  if (tid == 0) carry = base0 + (bases ? bases[blockIdx.x] : 0);
  __syncthreads();
  for (int64_t c0 = 0; c0 < n; c0 += 1024 * kScanItems) {
    const int64_t i0 = c0 + (int64_t)tid * kScanItems;
    int64_t v[kScanItems];
    int64_t t = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {  // branch-free: all loads in flight
      const bool in = i0 + q < n;
      const int64_t x = (int64_t)c[in ? i0 + q : 0];
      v[q] = in ? x : 0;
      t += v[q];
    }
    // inclusive wave scan of the thread totals
    int64_t x = t;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int64_t pre = carry;
    for (int w = 0; w < wave; ++w) pre += wsum[w];
    pre += x - t;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
      if (i0 + q < n) o[i0 + q] = pre;
      pre += v[q];
    }
    __syncthreads();
    if (tid == 0) {
      int64_t s = 0;
      for (int w = 0; w < 16; ++w) s += wsum[w];
      carry += s;
    }
    __syncthreads();
  }
  if (tid == 0) o[n] = carry;
}

// --------------------------------------------------------------------------
// summaries
// --------------------------------------------------------------------------
// Per repetition position maps (-1 = not sampled) and per index bitmasks of
// the repetitions that sample it (bit rho).
__global__ void sample_maps_kernel(const int32_t* idx, int64_t idx_stride, int64_t offJ,
                                   int64_t offK, int n1, int n2, int n3old, int nrep,
                                   int32_t* posI, int32_t* posJ, int32_t* posK, int64_t I,
                                   int64_t J, int64_t Kcap, uint64_t* bitI, uint64_t* bitJ,
                                   uint64_t* bitK) {
  const int rep = blockIdx.y;
  const int32_t* s = idx + rep * idx_stride;
  const int tot = n1 + n2 + n3old;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += gridDim.x * blockDim.x) {
    const uint64_t bit = 1ull << rep;
    if (q < n1) {
      const int32_t i = s[q];
      posI[rep * I + i] = q;
      atomicOr((unsigned long long*)&bitI[i], (unsigned long long)bit);
    } else if (q < n1 + n2) {
      const int32_t j = s[offJ + (q - n1)];
      posJ[rep * J + j] = q - n1;
      atomicOr((unsigned long long*)&bitJ[j], (unsigned long long)bit);
    } else {
      const int32_t k = s[offK + (q - n1 - n2)];
      posK[rep * Kcap + k] = q - n1 - n2;
      atomicOr((unsigned long long*)&bitK[k], (unsigned long long)bit);
    }
  }
}

__device__ inline uint64_t entry_mask(int32_t i, int32_t j, int32_t k, const uint64_t* bitI,
                                      const uint64_t* bitJ, const uint64_t* bitK, int64_t Kold,
                                      uint64_t all) {
  const uint64_t mk = k < Kold ? bitK[k] : all;
  return bitI[i] & bitJ[j] & mk;
}

// Count, per block of kCooChunk stored entries, how many each repetition keeps.
__global__ __launch_bounds__(kCooBlock) void summary_count_kernel(
    const int32_t* si, const int32_t* sj, const int32_t* sk, int64_t nnz, const uint64_t* bitI,
    const uint64_t* bitJ, const uint64_t* bitK, int64_t Kold, int nrep, uint32_t* bcount,
    int64_t nblk) {
  __shared__ uint32_t cnt[64];
  const int tid = threadIdx.x;
  if (tid < 64) cnt[tid] = 0;
  __syncthreads();
  const uint64_t all = nrep >= 64 ? ~0ull : ((1ull << nrep) - 1);
  const int64_t e0 = (int64_t)blockIdx.x * kCooChunk;
  for (int u = 0; u < kCooPerThread; ++u) {
    const int64_t e = e0 + u * kCooBlock + tid;
    uint64_t m = 0;
    if (e < nnz) m = entry_mask(si[e], sj[e], sk[e], bitI, bitJ, bitK, Kold, all);
    while (m) {
      const int rep = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      atomicAdd(&cnt[rep], 1u);
    }
  }
  __syncthreads();
  if (tid < nrep) bcount[(int64_t)tid * nblk + blockIdx.x] = cnt[tid];
}

__device__ inline uint64_t lmask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ inline uint64_t wave_or(uint64_t m) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1)
    m |= (uint64_t)__shfl_xor((unsigned long long)m, off, 64);
  return m;
}

// Emit the kept entries of every repetition in store order (hence sorted by
// c) at bbase[rep][block] + the rank within the block.  Each wavefront owns a
// contiguous run of kCooPerThread * 64 of the block's entries.  A first pass
// counts, per wavefront and repetition, the kept entries (masks stay in
// registers); after one block barrier every wavefront
// knows where its entries of each repetition start and writes them in store
// order with ballots alone.
__global__ __launch_bounds__(kCooBlock) void summary_emit_kernel(
    const int32_t* si, const int32_t* sj, const int32_t* sk, const float* sv, int64_t nnz,
    const uint64_t* bitI, const uint64_t* bitJ, const uint64_t* bitK, int64_t Kold, int n3old,
    int nrep, const int32_t* posI, const int32_t* posJ, const int32_t* posK, int64_t I,
    int64_t J, int64_t Kcap, const int64_t* bbase, const int64_t* rep_off, int64_t nblk,
    int32_t* za, int32_t* zb, int32_t* zc, float* zv) {
  constexpr int W = kCooBlock / 64;
  __shared__ uint32_t wc[W][64];  // kept entries per wavefront and repetition
  __shared__ int64_t wb[W][64];   // next output position per wavefront and repetition
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const uint64_t all = nrep >= 64 ? ~0ull : ((1ull << nrep) - 1);
  wc[wave][lane] = 0;
  __syncthreads();
  const int64_t e0 = (int64_t)blockIdx.x * kCooChunk + (int64_t)wave * 64 * kCooPerThread;
  uint64_t mk[kCooPerThread];
#pragma unroll
  for (int u = 0; u < kCooPerThread; ++u) {
    const int64_t e = e0 + u * 64 + lane;
    const uint64_t m = e < nnz ? entry_mask(si[e], sj[e], sk[e], bitI, bitJ, bitK, Kold, all) : 0;
    mk[u] = m;
    uint64_t un = wave_or(m);
    while (un) {
      const int rep = __ffsll((unsigned long long)un) - 1;
      un &= un - 1;
      const uint64_t bal = __ballot((m >> rep) & 1ull);
      if (lane == 0) wc[wave][rep] += (uint32_t)__popcll(bal);
    }
  }
  __syncthreads();
  if (tid < nrep) {
    int64_t p = rep_off[tid] + bbase[(int64_t)tid * (nblk + 1) + blockIdx.x];
    for (int w = 0; w < W; ++w) {
      wb[w][tid] = p;
      p += wc[w][tid];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kCooPerThread; ++u) {
    const uint64_t m = mk[u];
    uint64_t un = wave_or(m);
    if (!un) continue;
    const int64_t e = e0 + u * 64 + lane;
    int32_t i = 0, j = 0, k = 0;
    float v = 0.0f;
    if (m) {
      i = si[e];
      j = sj[e];
      k = sk[e];
      v = sv[e];
    }
    while (un) {
      const int rep = __ffsll((unsigned long long)un) - 1;
      un &= un - 1;
      const bool keep = (m >> rep) & 1ull;
      const uint64_t bal = __ballot(keep);
      const int64_t base = wb[wave][rep];
      if (keep) {
        const int64_t pos = base + __popcll(bal & lmask_lt());
        const int a = posI[rep * I + i];
        const int b = posJ[rep * J + j];
        const int c = k < Kold ? posK[rep * Kcap + k] : n3old + (int)(k - Kold);
        za[pos] = a;
        zb[pos] = b;
        zc[pos] = c;
        zv[pos] = v;
      }
      if (lane == 0) wb[wave][rep] = base + __popcll(bal);
    }
  }
}

// keys (rep << 24 | row) for the stable sorts by a and by b
// Row offsets of every repetition from the concatenated summaries sorted by
// (repetition, row): off[rep * sOff + x] = position of the first entry of
// (rep, x) or of the first later key, for x in [0, rows].  Thread p looks at
// the keys on both sides of position p (p in [0, total]) and writes the
// offsets of all (rep, x) pairs falling between them, so each offset is
// written once.  Keys come from `key` ((rep << 24) | row) or, with key null,
// from `row` and the repetition ranges rep_off.
__device__ inline int rep_at(const int64_t* rep_off, int nrep, int64_t p) {
  int r = 0;
  while (r + 1 < nrep && rep_off[r + 1] <= p) ++r;
  return r;
}

__global__ void summary_offsets_kernel(const uint32_t* key, const int32_t* row,
                                       const int64_t* rep_off, int nrep, int64_t total, int rows,
                                       int64_t* off, int64_t sOff) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p > total) return;
  // (rep, x) before position p and at position p, as linear indices rep * (rows + 1) + x
  const int64_t W = (int64_t)rows + 1;
  int64_t lo, hi;
  if (p == 0) {
    lo = -1;
  } else if (key) {
    const uint32_t k = key[p - 1];
    lo = (int64_t)(k >> 24) * W + (k & 0xFFFFFFu);
  } else {
    lo = (int64_t)rep_at(rep_off, nrep, p - 1) * W + row[p - 1];
  }
  if (p == total) {
    hi = (int64_t)nrep * W - 1;  // through x = rows of the last repetition
  } else if (key) {
    const uint32_t k = key[p];
    hi = (int64_t)(k >> 24) * W + (k & 0xFFFFFFu);
  } else {
    hi = (int64_t)rep_at(rep_off, nrep, p) * W + row[p];
  }
  for (int64_t q = lo + 1; q <= hi; ++q) {
    const int64_t r = q / W, x = q % W;
    off[r * sOff + x] = p;
  }
}

__global__ void summary_keys_kernel(const int32_t* za, const int32_t* zb, const int64_t* rep_off,
                                    int nrep, int64_t total, uint32_t* key_a, uint32_t* key_b,
                                    int32_t* val) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int rep = 0;
    while (rep + 1 < nrep && rep_off[rep + 1] <= e) ++rep;
    key_a[e] = ((uint32_t)rep << 24) | (uint32_t)za[e];
    key_b[e] = ((uint32_t)rep << 24) | (uint32_t)zb[e];
    val[e] = (int32_t)e;
  }
}

// mode copies: entry p of the a-sorted copy holds (b, c, v) of perm[p]
__global__ void summary_permute_kernel(const int32_t* perm, int64_t total, const int32_t* x0,
                                       const int32_t* x1, const float* zv, int32_t* y0,
                                       int32_t* y1, float* yv) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t e = perm[p];
    y0[p] = x0[e];
    y1[p] = x1[e];
    yv[p] = zv[e];
  }
}

// --------------------------------------------------------------------------
// MTTKRP on a summary, one wavefront per output row, fused with V^-1
// --------------------------------------------------------------------------
// rows of mode `mode` of every repetition: entries [off[row], off[row+1]) of
// the mode's copy hold (x, y, v) with x, y the indices of the two other modes
// (ascending mode order).  M(row, f) = sum v * X~(x, f) * Y~(y, f);
// U(row, :) = M(row, :) V^-1 (or divided by lam_div for the row solve).
template <int RP>
__global__ __launch_bounds__(256) void coo_rows_kernel(
    RepSet rs, int mode, const int64_t* off, int64_t sOff, const int32_t* cx, const int32_t* cy,
    const float* cv, const double* X, int64_t sX, const double* invlamX, const double* Y,
    int64_t sY, const double* invlamY, const double* Vinv, const double* lam_div, double* U,
    int64_t sU, int rows) {
  __shared__ double Vi[4][kMaxRank][kMaxRank + 1];
  const int R = rs.R;
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t gw = (int64_t)blockIdx.x * 4 + wave;  // global wave index
  const int rep = rs.rep0 + (int)(gw / rows);
  const int row = (int)(gw % rows);
  const bool active = rep < rs.rep0 + rs.nrep;
  if (active)
    for (int q = lane; q < R * R; q += 64) Vi[wave][q / R][q % R] = Vinv[rep * rs.sG + q];
  __syncthreads();
  if (!active) return;
  const int64_t* o = off + rep * sOff;
  const int64_t b0 = o[row], b1 = o[row + 1];
  const double* Xr = X + rep * sX;
  const double* Yr = Y + rep * sY;
  double sx[RP], sy[RP];
#pragma unroll
  for (int f = 0; f < RP; ++f) {
    sx[f] = (f < R && invlamX) ? invlamX[rep * 3 * R + f] : 1.0;
    sy[f] = (f < R && invlamY) ? invlamY[rep * 3 * R + f] : 1.0;
  }
  float acc[RP];
#pragma unroll
  for (int f = 0; f < RP; ++f) acc[f] = 0.0f;
  for (int64_t e = b0 + lane; e < b1; e += 64) {
    const int32_t x = cx[e], y = cy[e];
    const float v = cv[e];
    const double* xr = Xr + (int64_t)x * R;
    const double* yr = Yr + (int64_t)y * R;
#pragma unroll
    for (int f = 0; f < RP; ++f)
      if (f < R) acc[f] += v * (float)(xr[f] * sx[f]) * (float)(yr[f] * sy[f]);
  }
  double m[RP];
#pragma unroll
  for (int f = 0; f < RP; ++f) m[f] = (double)wave_sum(acc[f]);
  // lane f < R finishes column f of the row
  double u = 0.0;
#pragma unroll
  for (int k = 0; k < RP; ++k)
    if (k < R && lane < R) u += m[k] * Vi[wave][k][lane];
  if (lane < R) {
    if (lam_div) {
      const double l = lam_div[lane];
      u = l > 0.0 ? u / l : 0.0;
    }
    U[rep * sU + (int64_t)row * R + lane] = u;
  }
}

// ---------------------------------------------------------------------------
// MTTKRP over work units (pieces of at most kCooUnit entries of one row)
// ---------------------------------------------------------------------------
__global__ void coo_unit_count_kernel(const int64_t* off, int64_t sOff, int rows, int nrep,
                                      uint32_t* cnt) {
  const int64_t n = (int64_t)rows * nrep;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int rep = (int)(q / rows), row = (int)(q % rows);
    const int64_t len = off[rep * sOff + row + 1] - off[rep * sOff + row];
    cnt[q] = (uint32_t)((len + kCooUnit - 1) / kCooUnit);
  }
}

__global__ void coo_unit_fill_kernel(const int64_t* off, int64_t sOff, int rows, int nrep,
                                     const int64_t* uoff, int64_t cap, int32_t* urow,
                                     int64_t* ustart, int32_t* ulen) {
  const int64_t n = (int64_t)rows * nrep;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int rep = (int)(q / rows), row = (int)(q % rows);
    const int64_t start = off[rep * sOff + row];
    const int64_t len = off[rep * sOff + row + 1] - start;
    const int64_t base = uoff[q], nu = uoff[q + 1] - base;
    for (int64_t u = 0; u < nu && base + u < cap; ++u) {
      urow[base + u] = (int32_t)q;
      ustart[base + u] = start + u * kCooUnit;
      const int64_t rem = len - u * kCooUnit;
      ulen[base + u] = (int32_t)(rem < kCooUnit ? rem : kCooUnit);
    }
  }
}

// FP32 copies of the scaled factor rows the sparse MTTKRP gathers:
// Xf[rep][row][RX] = X(row, :) diag(invlam) (zero beyond R), RX = 16 or 32
__global__ void coo_prep_kernel(RepSet rs, int rows, int RX, const double* X, int64_t sX,
                                const double* invlam, float* Xf) {
  const int rep = rs.rep0 + blockIdx.y;
  const int R = rs.R;
  const int64_t n = (int64_t)rows * RX;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = q / RX;
    const int f = (int)(q % RX);
    float v = 0.0f;
    if (f < R) v = (float)(X[rep * sX + row * R + f] * (invlam ? invlam[rep * 3 * R + f] : 1.0));
    Xf[(int64_t)rep * rows * RX + q] = v;
  }
}

// UL lanes per unit (32 or 64; 64 / UL units per wavefront): partial row
// sum_e v * Xf(x_e, :) * Yf(y_e, :).  Units are dealt to the eight XCDs in
// contiguous ranges (workgroup b runs on XCD b mod 8), so each XCD's L2 holds
// the factor rows of about one and a quarter repetitions.  The scaled factor
// copies have rows of 16 (R <= 16) or 32 floats, whole cache-line halves or
// lines; LE = RX / 4 lanes split a row into float4 columns, so one load
// instruction fetches whole rows of UL / LE entries.  The unit's lanes read
// the coordinates of UL entries at once (one per lane) and pass them round
// with cross-lane moves; then LE steps of UL / LE entries issue all their row
// loads before the products.
constexpr int kXcds = 8;

template <int RP, int UL>
__global__ __launch_bounds__(256) void coo_units_kernel(
    RepSet rs, int rows, int rowsX, int rowsY, const int32_t* urow, const int64_t* ustart,
    const int32_t* ulen, const int64_t* ntot, int64_t cap, const int32_t* cx, const int32_t* cy,
    const float* cv, const float* Xf, const float* Yf, float* part) {
  constexpr int G = 256 / UL;             // units per block
  constexpr int RX = RP <= 16 ? 16 : 32;  // floats per staged factor row
  constexpr int LE = RX / 4;              // lanes per entry (float4 columns)
  constexpr int EPS = UL / LE;            // entries per step
  const int64_t T = *ntot < cap ? *ntot : cap;
  const int64_t per = (T + kXcds - 1) / kXcds;
  const int xcd = blockIdx.x % kXcds;
  const int64_t lb = blockIdx.x / kXcds;
  const int grp = threadIdx.x / UL, l = threadIdx.x % UL;
  const int sub = l / LE, c = l % LE;
  const int base = (threadIdx.x % kWave) - l;  // first lane of the unit in the wavefront
  const int64_t k = lb * G + grp;
  const int64_t gu = xcd * per + k;
  const bool ok = k < per && gu < T;
  int64_t b0 = 0, b1 = 0;
  const float4* Xr = nullptr;
  const float4* Yr = nullptr;
  if (ok) {
    const int rep = rs.rep0 + urow[gu] / rows;
    Xr = reinterpret_cast<const float4*>(Xf + (int64_t)rep * rowsX * RX);
    Yr = reinterpret_cast<const float4*>(Yf + (int64_t)rep * rowsY * RX);
    b0 = ustart[gu];
    b1 = b0 + ulen[gu];
  }
  // the wavefront runs the longest of its units (cross-lane moves need all lanes)
  int64_t mlen = b1 - b0;
#pragma unroll
  for (int m = UL; m < kWave; m *= 2) {
    const int64_t o = (int64_t)__shfl_xor((long long)mlen, m, kWave);
    mlen = o > mlen ? o : mlen;
  }
  float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  for (int64_t o = 0; o < mlen; o += UL) {
    const int64_t e = b0 + o + l;
    float vv = 0.0f;  // past the end: row 0 times a zero value
    int32_t xx = 0, yy = 0;
    if (e < b1) {
      vv = cv[e];
      xx = cx[e];
      yy = cy[e];
    }
    float v[LE];
    int32_t ix[LE], iy[LE];
#pragma unroll
    for (int d = 0; d < LE; ++d) {
      const int src = base + d * EPS + sub;
      v[d] = __shfl(vv, src, kWave);
      ix[d] = __shfl(xx, src, kWave);
      iy[d] = __shfl(yy, src, kWave);
    }
    if (Xr) {
      float4 a[LE], b[LE];
#pragma unroll
      for (int d = 0; d < LE; ++d) {
        a[d] = Xr[(int64_t)ix[d] * LE + c];
        b[d] = Yr[(int64_t)iy[d] * LE + c];
      }
#pragma unroll
      for (int d = 0; d < LE; ++d) {
        acc.x += v[d] * a[d].x * b[d].x;
        acc.y += v[d] * a[d].y * b[d].y;
        acc.z += v[d] * a[d].z * b[d].z;
        acc.w += v[d] * a[d].w * b[d].w;
      }
    }
  }
  // add the entry slots of each column (all lanes take part)
#pragma unroll
  for (int m = LE; m < UL; m *= 2) {
    acc.x += __shfl_xor(acc.x, m, kWave);
    acc.y += __shfl_xor(acc.y, m, kWave);
    acc.z += __shfl_xor(acc.z, m, kWave);
    acc.w += __shfl_xor(acc.w, m, kWave);
  }
  if (ok && sub == 0) {
    const int f = 4 * c;
    float* out = part + gu * RP;
    if (f + 0 < RP) out[f + 0] = acc.x;
    if (f + 1 < RP) out[f + 1] = acc.y;
    if (f + 2 < RP) out[f + 2] = acc.z;
    if (f + 3 < RP) out[f + 3] = acc.w;
  }
}

// rows of all repetitions: sum the unit partials of the row in order, times
// V^-1 of the repetition, divided by lam_div for the row solve.  64 rows per
// block, four lanes per row (components f = lane, lane + 4, ...).
constexpr int kFinRows = 64;

template <int RP>
__global__ __launch_bounds__(256) void coo_units_finish_kernel(RepSet rs, int rows,
                                                              const int64_t* uoff, int64_t cap,
                                                              const float* part,
                                                              const double* Vinv,
                                                              const double* lam_div,
                                                              double* Uout, int64_t sU) {
  constexpr int FL = RP / 4;  // components per lane
  __shared__ double M[kFinRows][RP + 1];
  const int R = rs.R;
  const int tid = threadIdx.x;
  const int r = tid / 4, fl = tid % 4;
  const int64_t q = (int64_t)blockIdx.x * kFinRows + r;
  const bool ok = q < (int64_t)rows * rs.nrep;
  if (ok) {
    double m[FL];
#pragma unroll
    for (int t = 0; t < FL; ++t) m[t] = 0.0;
    const int64_t u1 = uoff[q + 1] < cap ? uoff[q + 1] : cap;
    for (int64_t u = uoff[q]; u < u1; ++u) {
#pragma unroll
      for (int t = 0; t < FL; ++t) m[t] += (double)part[u * RP + fl + 4 * t];
    }
#pragma unroll
    for (int t = 0; t < FL; ++t) M[r][fl + 4 * t] = m[t];
  }
  __syncthreads();
  if (ok) {
    const int rep = rs.rep0 + (int)(q / rows), row = (int)(q % rows);
    const double* Vi = Vinv + rep * rs.sG;
#pragma unroll
    for (int t = 0; t < FL; ++t) {
      const int f = fl + 4 * t;
      if (f >= R) continue;
      double u = 0.0;
      for (int k = 0; k < R; ++k) u += M[r][k] * Vi[k * R + f];
      if (lam_div) {
        const double l = lam_div[f];
        u = l > 0.0 ? u / l : 0.0;
      }
      Uout[rep * sU + (int64_t)row * R + f] = u;
    }
  }
}

// fit over a k-sorted COO store: one wavefront per slice
template <int RP>
__global__ __launch_bounds__(256) void coo_fit_kernel(const int32_t* si, const int32_t* sj,
                                                     const float* sv, const int64_t* koff,
                                                     int64_t K, int R, const double* A,
                                                     const double* B, double* M3, double* nrm) {
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t k = (int64_t)blockIdx.x * 4 + wave;
  if (k >= K) return;
  double acc[RP];
#pragma unroll
  for (int f = 0; f < RP; ++f) acc[f] = 0.0;
  double n2 = 0.0;
  for (int64_t e = koff[k] + lane; e < koff[k + 1]; e += 64) {
    const double v = sv[e];
    const double* ar = A + (int64_t)si[e] * R;
    const double* br = B + (int64_t)sj[e] * R;
    n2 += v * v;
#pragma unroll
    for (int f = 0; f < RP; ++f)
      if (f < R) acc[f] += v * ar[f] * br[f];
  }
#pragma unroll
  for (int f = 0; f < RP; ++f) {
    const double s = wave_sum(acc[f]);
    if (lane == 0 && f < R) M3[k * R + f] = s;
  }
  n2 = wave_sum(n2);
  if (lane == 0) nrm[k] = n2;
}

inline int rp_of4(int R) { return ((R + 3) / 4) * 4; }

#define SBT_COO_RP(Rv, ...)                                 \
  switch (rp_of4(Rv)) {                                     \
    case 4: { constexpr int RP = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int RP = 8; __VA_ARGS__; } break;   \
    case 12: { constexpr int RP = 12; __VA_ARGS__; } break; \
    case 16: { constexpr int RP = 16; __VA_ARGS__; } break; \
    case 20: { constexpr int RP = 20; __VA_ARGS__; } break; \
    case 24: { constexpr int RP = 24; __VA_ARGS__; } break; \
    case 28: { constexpr int RP = 28; __VA_ARGS__; } break; \
    default: { constexpr int RP = 32; __VA_ARGS__; } break; \
  }

// Copy per repetition q the entries [src[q], src[q] + cnt[q]) of the four
// summary arrays to [dst[q], dst[q] + cnt[q]) of four others (a persistent
// summary's old part moved to its place in the next update's layout).
__global__ __launch_bounds__(256) void summary_move_kernel(const int32_t* a, const int32_t* b,
                                                          const int32_t* c, const float* v,
                                                          const int64_t* src, const int64_t* cnt,
                                                          const int64_t* dst, int32_t* oa,
                                                          int32_t* ob, int32_t* oc, float* ov) {
  const int q = blockIdx.y;
  const int64_t n = cnt[q], s0 = src[q], d0 = dst[q];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    oa[d0 + e] = a[s0 + e];
    ob[d0 + e] = b[s0 + e];
    oc[d0 + e] = c[s0 + e];
    ov[d0 + e] = v[s0 + e];
  }
}

}  // namespace

// ==========================================================================
// launchers
// ==========================================================================
hipError_t coo_sort_tmp_bytes(int64_t n, size_t* bytes) {
  size_t b = 0;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const uint32_t*)nullptr,
                                                    (uint32_t*)nullptr, (const int32_t*)nullptr,
                                                    (int32_t*)nullptr, (int)n, 0, 32, 0);
  *bytes = b;
  return e;
}

hipError_t launch_coo_ingest(const int32_t* bi, const int32_t* bj, const int32_t* bk,
                             const float* bv, int64_t n, int64_t Knew, int64_t Kold,
                             int32_t* si, int32_t* sj, int32_t* sk, float* sv, int64_t base,
                             int64_t* koff, CooScratch& w, hipStream_t s) {
  if (n <= 0) {
    // no entries: every new slice is empty
    hipError_t e = launch_fill_u32(w.hist, Knew, 0, s);
    if (e != hipSuccess) return e;
    scan_to_offsets_kernel<<<1, 1024, 0, s>>>(w.hist, 0, Knew, base, nullptr, koff + Kold, 0);
    return hipGetLastError();
  }
  hipError_t e;
  int bits = 1;
  while ((1ll << bits) < Knew) ++bits;
  copy_u32_kernel<<<grid_for(n, 256 * 16), 256, 0, s>>>(bk, w.key_in, n);
  iota_kernel<<<grid_for(n, 256 * 16), 256, 0, s>>>(w.val_in, n);
  size_t tb = w.tmp_bytes;
  e = hipcub::DeviceRadixSort::SortPairs(w.tmp, tb, w.key_in, w.key_out, w.val_in, w.val_out,
                                         (int)n, 0, bits, s);
  if (e != hipSuccess) return e;
  e = launch_fill_u32(w.hist, Knew, 0, s);
  if (e != hipSuccess) return e;
  coo_place_kernel<<<grid_for(n, 256 * 16), 256, 0, s>>>(bi, bj, bk, bv, w.val_out, n, Knew,
                                                          Kold, si, sj, sk, sv, base, w.hist);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  scan_to_offsets_kernel<<<1, 1024, 0, s>>>(w.hist, 0, Knew, base, nullptr, koff + Kold, 0);
  return hipGetLastError();
}

hipError_t launch_coo_maps(const int32_t* idx, int64_t idx_stride, int64_t offJ, int64_t offK,
                           int n1, int n2, int n3old, int nrep, int32_t* posI, int32_t* posJ,
                           int32_t* posK, int64_t I, int64_t J, int64_t Kcap, uint64_t* bitI,
                           uint64_t* bitJ, uint64_t* bitK, hipStream_t s) {
  hipError_t e = launch_fill_u32((uint32_t*)posI, (int64_t)nrep * I, 0xFFFFFFFFu, s);
  if (e == hipSuccess) e = launch_fill_u32((uint32_t*)posJ, (int64_t)nrep * J, 0xFFFFFFFFu, s);
  if (e == hipSuccess) e = launch_fill_u32((uint32_t*)posK, (int64_t)nrep * Kcap, 0xFFFFFFFFu, s);
  if (e == hipSuccess) e = launch_fill_u64(bitI, I, 0, s);
  if (e == hipSuccess) e = launch_fill_u64(bitJ, J, 0, s);
  if (e == hipSuccess) e = launch_fill_u64(bitK, Kcap, 0, s);
  if (e != hipSuccess) return e;
  const int tot = n1 + n2 + n3old;
  sample_maps_kernel<<<dim3((unsigned)grid_for(tot, 256), (unsigned)nrep), 256, 0, s>>>(
      idx, idx_stride, offJ, offK, n1, n2, n3old, nrep, posI, posJ, posK, I, J, Kcap, bitI, bitJ,
      bitK);
  return hipGetLastError();
}

int64_t coo_scan_blocks(int64_t nnz) { return (nnz + kCooChunk - 1) / kCooChunk; }

hipError_t launch_coo_count(const int32_t* si, const int32_t* sj, const int32_t* sk, int64_t nnz,
                            const uint64_t* bitI, const uint64_t* bitJ, const uint64_t* bitK,
                            int64_t Kold, int nrep, uint32_t* bcount, int64_t* bbase,
                            hipStream_t s) {
  const int64_t nblk = coo_scan_blocks(nnz);
  summary_count_kernel<<<(unsigned)nblk, kCooBlock, 0, s>>>(si, sj, sk, nnz, bitI, bitJ, bitK,
                                                            Kold, nrep, bcount, nblk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // per repetition exclusive scan over blocks; repetition rho starts where
  // rho - 1 ends, so bbase[rho][0] is the offset of rho's summary
  scan_to_offsets_kernel<<<(unsigned)nrep, 1024, 0, s>>>(bcount, nblk, nblk, 0, nullptr, bbase,
                                                         nblk + 1);
  return hipGetLastError();
}

hipError_t launch_coo_emit(const int32_t* si, const int32_t* sj, const int32_t* sk,
                           const float* sv, int64_t nnz, const uint64_t* bitI,
                           const uint64_t* bitJ, const uint64_t* bitK, int64_t Kold, int n3old,
                           int nrep, const int32_t* posI, const int32_t* posJ,
                           const int32_t* posK, int64_t I, int64_t J, int64_t Kcap,
                           const int64_t* bbase, CooSummary& z, hipStream_t s) {
  const int64_t nblk = coo_scan_blocks(nnz);
  timed_launch(summary_emit_kernel, (unsigned)nblk, dim3(kCooBlock), 0, s, 
      si, sj, sk, sv, nnz, bitI, bitJ, bitK, Kold, n3old, nrep, posI, posJ, posK, I, J, Kcap,
      bbase, z.rep_off, nblk, z.a, z.b, z.c, z.v);
  return hipGetLastError();
}


hipError_t launch_summary_move(const int32_t* a, const int32_t* b, const int32_t* c,
                               const float* v, const int64_t* src, const int64_t* cnt,
                               const int64_t* dst, int nrep, int64_t max_cnt, int32_t* oa,
                               int32_t* ob, int32_t* oc, float* ov, hipStream_t s) {
  if (nrep <= 0 || max_cnt <= 0) return hipSuccess;
  const int blocks = grid_for(max_cnt, 256);
  dim3 grid((unsigned)(blocks < 2048 ? blocks : 2048), (unsigned)nrep);
  summary_move_kernel<<<grid, 256, 0, s>>>(a, b, c, v, src, cnt, dst, oa, ob, oc, ov);
  return hipGetLastError();
}

hipError_t launch_coo_sorts(CooSummary& z, int nrep, int64_t total, int n1, int n2, int n3,
                            hipStream_t s) {
  const unsigned go = (unsigned)grid_for(total + 1, 256);
  // c: the summaries are in store order, sorted by c within each repetition
  summary_offsets_kernel<<<go, 256, 0, s>>>(nullptr, z.c, z.rep_off, nrep, total, n3, z.offC,
                                            z.sOffC);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || total <= 0) {
    if (e == hipSuccess) {  // no entries: every row of every repetition is empty
      summary_offsets_kernel<<<go, 256, 0, s>>>(nullptr, z.a, z.rep_off, nrep, 0, n1, z.offA,
                                                z.sOffA);
      summary_offsets_kernel<<<go, 256, 0, s>>>(nullptr, z.b, z.rep_off, nrep, 0, n2, z.offB,
                                                z.sOffB);
      e = hipGetLastError();
    }
    return e;
  }
  summary_keys_kernel<<<grid_for(total, 256 * 16), 256, 0, s>>>(z.a, z.b, z.rep_off, nrep, total,
                                                                 z.key_a, z.key_b, z.val);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  int bits = 24;
  while ((1ll << (bits - 24)) < nrep) ++bits;
  size_t tb = z.tmp_bytes;
  e = hipcub::DeviceRadixSort::SortPairs(z.tmp, tb, z.key_a, z.key_out, z.val, z.perm, (int)total,
                                         0, bits, s);
  if (e != hipSuccess) return e;
  summary_permute_kernel<<<grid_for(total, 256 * 16), 256, 0, s>>>(z.perm, total, z.b, z.c, z.v,
                                                                    z.a_x, z.a_y, z.a_v);
  summary_offsets_kernel<<<go, 256, 0, s>>>(z.key_out, nullptr, z.rep_off, nrep, total, n1,
                                            z.offA, z.sOffA);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  tb = z.tmp_bytes;
  e = hipcub::DeviceRadixSort::SortPairs(z.tmp, tb, z.key_b, z.key_out, z.val, z.perm, (int)total,
                                         0, bits, s);
  if (e != hipSuccess) return e;
  summary_permute_kernel<<<grid_for(total, 256 * 16), 256, 0, s>>>(z.perm, total, z.a, z.c, z.v,
                                                                    z.b_x, z.b_y, z.b_v);
  summary_offsets_kernel<<<go, 256, 0, s>>>(z.key_out, nullptr, z.rep_off, nrep, total, n2,
                                            z.offB, z.sOffB);
  return hipGetLastError();
}

hipError_t launch_coo_single_summary(const int32_t* a, const int32_t* b, const int32_t* c,
                                     const float* v, int64_t nnz, int n1, int n2, int n3,
                                     CooSummary& z, hipStream_t s) {
  if (nnz > 0) {
    int bits = 1;
    while ((1ll << bits) < n3) ++bits;
    copy_u32_kernel<<<grid_for(nnz, 256 * 16), 256, 0, s>>>(c, z.key_a, nnz);
    iota_kernel<<<grid_for(nnz, 256 * 16), 256, 0, s>>>(z.val, nnz);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t tb = z.tmp_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(z.tmp, tb, z.key_a, z.key_out, z.val, z.perm,
                                           (int)nnz, 0, bits, s);
    if (e != hipSuccess) return e;
    summary_permute_kernel<<<grid_for(nnz, 256 * 16), 256, 0, s>>>(z.perm, nnz, a, b, v, z.a,
                                                                    z.b, z.v);
    copy_u32_kernel<<<grid_for(nnz, 256 * 16), 256, 0, s>>>((const int32_t*)z.key_out,
                                                             (uint32_t*)z.c, nnz);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return launch_coo_sorts(z, 1, nnz, n1, n2, n3, s);
}

namespace {
struct ModeView {
  int rows;
  const int64_t* off;
  int64_t sOff;
  const int32_t *cx, *cy;
  const float* cv;
};
ModeView mode_view(const RepSet& rs, int mode, const CooSummary& z) {
  ModeView m;
  m.rows = mode == 0 ? rs.n1 : (mode == 1 ? rs.n2 : rs.n3);
  m.off = mode == 0 ? z.offA : (mode == 1 ? z.offB : z.offC);
  m.sOff = mode == 0 ? z.sOffA : (mode == 1 ? z.sOffB : z.sOffC);
  m.cx = mode == 0 ? z.a_x : (mode == 1 ? z.b_x : z.a);
  m.cy = mode == 0 ? z.a_y : (mode == 1 ? z.b_y : z.b);
  m.cv = mode == 0 ? z.a_v : (mode == 1 ? z.b_v : z.v);
  return m;
}

}  // namespace

hipError_t launch_coo_units_build(const RepSet& rs, int mode, const CooSummary& z, CooUnits& u,
                                  hipStream_t s) {
  const ModeView m = mode_view(rs, mode, z);
  const int64_t n = (int64_t)m.rows * rs.nrep;
  const int blocks = grid_for(n, 256);
  coo_unit_count_kernel<<<blocks, 256, 0, s>>>(m.off, m.sOff, m.rows, rs.nrep, u.cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  scan_to_offsets_kernel<<<1, 1024, 0, s>>>(u.cnt, 0, n, 0, nullptr, u.uoff, 0);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  coo_unit_fill_kernel<<<blocks, 256, 0, s>>>(m.off, m.sOff, m.rows, rs.nrep, u.uoff, u.cap,
                                              u.urow, u.ustart, u.ulen);
  return hipGetLastError();
}

hipError_t launch_coo_prep(const RepSet& rs, int rows, const double* X, int64_t sX,
                           const double* invlam, float* Xf, hipStream_t s) {
  const int RX = rs.R <= 16 ? 16 : 32;  // row length of the staged copies
  const int64_t n = (int64_t)rows * RX;
  int blocks = grid_for(n, 256);
  if (blocks > 1024) blocks = 1024;
  coo_prep_kernel<<<dim3((unsigned)blocks, (unsigned)rs.nrep), 256, 0, s>>>(rs, rows, RX, X, sX,
                                                                          invlam, Xf);
  return hipGetLastError();
}

hipError_t launch_coo_units(const RepSet& rs, int mode, const CooSummary& z, const CooUnits& u,
                            const float* Xf, int rowsX, const float* Yf, int rowsY, float* part,
                            double avg_row_nnz, hipStream_t s) {
  const ModeView m = mode_view(rs, mode, z);
  const int64_t n = (int64_t)m.rows * rs.nrep;
  if (u.cap <= 0) return hipSuccess;
  // a wavefront per unit when rows hold many entries on average, else two
  const bool wide = avg_row_nnz >= 128.0;
  const int G = wide ? 4 : 8;
  const int64_t per = (u.cap + kXcds - 1) / kXcds;
  const unsigned blocks = (unsigned)(kXcds * ((per + G - 1) / G));
  SBT_COO_RP(rs.R, {
    if (wide)
      timed_launch(coo_units_kernel<RP, 64>, blocks, dim3(256), 0, s, rs, m.rows, rowsX, rowsY,
                   u.urow, u.ustart, u.ulen, u.uoff + n, u.cap, m.cx, m.cy, m.cv, Xf, Yf, part);
    else
      timed_launch(coo_units_kernel<RP, 32>, blocks, dim3(256), 0, s, rs, m.rows, rowsX, rowsY,
                   u.urow, u.ustart, u.ulen, u.uoff + n, u.cap, m.cx, m.cy, m.cv, Xf, Yf, part);
  });
  return hipGetLastError();
}

hipError_t launch_coo_units_finish(const RepSet& rs, int mode, const CooUnits& u,
                                   const float* part, const double* Vinv, const double* lam_div,
                                   double* U, int64_t sU, hipStream_t s) {
  const int rows = mode == 0 ? rs.n1 : (mode == 1 ? rs.n2 : rs.n3);
  const int64_t n = (int64_t)rows * rs.nrep;
  const unsigned blocks = (unsigned)((n + kFinRows - 1) / kFinRows);
  SBT_COO_RP(rs.R, {
    coo_units_finish_kernel<RP><<<blocks, 256, 0, s>>>(rs, rows, u.uoff, u.cap, part, Vinv,
                                                       lam_div, U, sU);
  });
  return hipGetLastError();
}

hipError_t launch_coo_rows(const RepSet& rs, int mode, const CooSummary& z, const double* X,
                           int64_t sX, const double* invlamX, const double* Y, int64_t sY,
                           const double* invlamY, const double* Vinv, const double* lam_div,
                           double* U, int64_t sU, hipStream_t s) {
  const int rows = mode == 0 ? rs.n1 : (mode == 1 ? rs.n2 : rs.n3);
  const int64_t* off = mode == 0 ? z.offA : (mode == 1 ? z.offB : z.offC);
  const int64_t sOff = mode == 0 ? z.sOffA : (mode == 1 ? z.sOffB : z.sOffC);
  const int32_t* cx = mode == 0 ? z.a_x : (mode == 1 ? z.b_x : z.a);
  const int32_t* cy = mode == 0 ? z.a_y : (mode == 1 ? z.b_y : z.b);
  const float* cv = mode == 0 ? z.a_v : (mode == 1 ? z.b_v : z.v);
  const int64_t waves = (int64_t)rows * rs.nrep;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  SBT_COO_RP(rs.R, {
    coo_rows_kernel<RP><<<blocks, 256, 0, s>>>(rs, mode, off, sOff, cx, cy, cv, X, sX, invlamX, Y,
                                              sY, invlamY, Vinv, lam_div, U, sU, rows);
  });
  return hipGetLastError();
}

hipError_t launch_fit_coo(const int32_t* ii, const int32_t* jj, const float* v,
                          const int64_t* koff, int64_t K, int R, const double* A,
                          const double* B, double* M3, double* nrm, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  SBT_COO_RP(R, {
    coo_fit_kernel<RP><<<(unsigned)((K + 3) / 4), 256, 0, s>>>(ii, jj, v, koff, K, R, A, B, M3,
                                                              nrm);
  });
  return hipGetLastError();
}

}  // namespace sbt
