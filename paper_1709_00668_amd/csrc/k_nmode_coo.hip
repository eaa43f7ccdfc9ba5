// Sparse (COO) tensors of order N >= 3 whose last mode grows: importance,
// ingest, summaries and the sparse MTTKRP of their CP-ALS.  Deterministic: no
// floating-point atomics (integer importance sums only), summaries emitted in
// store order, rows summed in a fixed order.
//
// Store: N coordinate arrays and the values, sorted by the last coordinate
// (each batch is stably sorted by it on ingest and batches arrive in slice
// order), with per-slice offsets.
//
// Summary of repetition rho: the stored entries whose every coordinate is
// sampled by rho (the last mode: K_s u new), re-indexed to the positions in
// the samples (Sec. 3.1).  The summaries of all repetitions are concatenated
// in repetition order.  The MTTKRP of mode m reads them grouped by (rho,
// coordinate m): one stable radix sort per mode and update gives that order.
#include <hipcub/hipcub.hpp>

#include "device_common.hpp"
#include "kernels.hpp"

namespace sbt {

namespace {

__global__ void iota_nd_kernel(int32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int32_t)i;
}

// key = last coordinate (batch-relative), for the stable sort of a batch
__global__ void last_key_kernel(const int32_t* k, int64_t n, uint32_t* key) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    key[i] = (uint32_t)k[i];
}

// store[base + p] = batch[perm[p]], last coordinate shifted by k0
__global__ void coo_place_nd_kernel(CooNd b, const int32_t* perm, int64_t base, int64_t k0,
                                    CooStoreNd st) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < b.nnz;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = perm[p];
    for (int m = 0; m < b.N; ++m)
      st.idx[m][base + p] = b.idx[m][e] + (m == b.N - 1 ? (int32_t)k0 : 0);
    st.v[base + p] = b.v[e];
  }
}

// off[x] = first position p in [0, n) with key[p] >= x (n if none), for x in
// [x0, x1]; the keys ascend
__global__ void lower_bounds_kernel(const int32_t* key, int64_t n, int64_t x0, int64_t x1,
                                    int64_t* off) {
  for (int64_t x = x0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x <= x1;
       x += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (key[mid] < x) lo = mid + 1; else hi = mid;
    }
    off[x] = lo;
  }
}

// same for the packed keys (rep << 24 | row) of the sorted summaries:
// off[rep * (rows + 1) + x] for x in [0, rows]
__global__ void row_offsets_kernel(const uint32_t* key, int64_t n, int rows, int nrep,
                                   int64_t* off) {
  const int64_t total = (int64_t)nrep * (rows + 1);
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int rep = (int)(q / (rows + 1)), x = (int)(q % (rows + 1));
    const uint32_t target = ((uint32_t)rep << 24) | (uint32_t)x;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (key[mid] < target) lo = mid + 1; else hi = mid;
    }
    off[q] = lo;
  }
}

// position maps: pos[rep][posoff[m] + index] = position of index in the
// sample of mode m, -1 when not sampled; the last mode's new slices follow
// its n3old sampled old ones
__global__ void pos_maps_kernel(PosMapsNd a, int32_t* pos) {
  const int rep = blockIdx.y;
  int32_t* P = pos + (int64_t)rep * a.stride;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < a.stride;
       q += (int64_t)gridDim.x * blockDim.x)
    P[q] = -1;
  __syncthreads();
  // (a grid-stride fill then scatter needs all fills first: one block per rep
  // in y and a single block in x, so the barrier orders them)
  const int32_t* S = a.idx + rep * a.idx_stride;
  for (int m = 0; m < a.N; ++m) {
    const int n = a.n[m];
    for (int p = threadIdx.x; p < n; p += blockDim.x) P[a.posoff[m] + S[a.off[m] + p]] = p;
  }
  const int64_t last = a.posoff[a.N - 1];
  for (int64_t j = threadIdx.x; j < a.Knew; j += blockDim.x)
    P[last + a.Kold + j] = a.n[a.N - 1] + (int32_t)j;
}

// flag[rep * nnz + e] = 1 when every coordinate of stored entry e is sampled
__global__ void keep_flags_kernel(CooStoreNd st, int64_t nnz, PosViewNd pv, const int32_t* pos,
                                  uint32_t* flag) {
  const int rep = blockIdx.y;
  const int32_t* P = pos + rep * pv.stride;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    bool keep = true;
    for (int m = 0; m < pv.N && keep; ++m) keep = P[pv.posoff[m] + st.idx[m][e]] >= 0;
    flag[rep * nnz + e] = keep ? 1u : 0u;
  }
}

// kept entries to their places in the concatenated summaries (store order)
__global__ void summary_emit_nd_kernel(CooStoreNd st, int64_t nnz, PosViewNd pv,
                                       const int32_t* pos, const uint32_t* flag,
                                       const uint32_t* at, CooSumNd z) {
  const int rep = blockIdx.y;
  const int32_t* P = pos + rep * pv.stride;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = rep * nnz + e;
    if (!flag[f]) continue;
    const int64_t p = at[f];
    for (int m = 0; m < pv.N; ++m) z.idx[m][p] = P[pv.posoff[m] + st.idx[m][e]];
    z.v[p] = st.v[e];
    z.rep[p] = (uint8_t)rep;
  }
}

// keys (rep << 24 | coordinate of mode m) of the summary entries (rep 0
// when the entries carry no repetition)
__global__ void mode_keys_kernel(CooSumNd z, int64_t total, int m, uint32_t* key) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total;
       p += (int64_t)gridDim.x * blockDim.x)
    key[p] = ((uint32_t)(z.rep ? z.rep[p] : 0) << 24) | (uint32_t)z.idx[m][p];
}

// M(rep, row, f) = sum over the row's entries of v * prod over the other
// modes l of U_l(coordinate l, f).  A row's entries are cut into S equal
// ranges (S from the launch shape alone, so that few long rows of skewed
// data still spread over many wavefronts); one wavefront per (rep, row,
// range), a lane per entry: lane i takes entries i, i + 64, ... of the range
// (two per step, so that the gathers of both are in flight together) and
// keeps the RP sums of its entries in registers; the lanes' sums are added
// by a fixed butterfly.  With S = 1 the wavefront writes M's row, else its
// partial row, and the ranges' partial rows are added in range order.
template <int RP>
__global__ __launch_bounds__(256) void mttkrp_coo_nd_kernel(MttkrpCooNd a, int S,
                                                           double* part) {
  const int lane = threadIdx.x & 63;
  const int64_t wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int rep = a.rep0 + blockIdx.y;
  if (wv >= (int64_t)a.rows * S) return;  // a whole wavefront; no block barrier follows
  const int row = (int)(wv / S), sl = (int)(wv % S);
  const int R = a.R;
  const int64_t* off = a.off + (int64_t)rep * (a.rows + 1);
  const int64_t r0 = off[row], len = off[row + 1] - r0;
  const int64_t cs = (len + S - 1) / S;
  const int64_t p0 = r0 + sl * cs;
  const int64_t p1 = r0 + ((sl + 1) * cs < len ? (sl + 1) * cs : len);
  double acc[RP];
#pragma unroll
  for (int f = 0; f < RP; ++f) acc[f] = 0.0;
  for (int64_t p = p0 + lane; p < p1; p += 128) {
    const bool two = p + 64 < p1;
    const int64_t e0 = a.perm ? a.perm[p] : p;
    const int64_t e1 = two ? (a.perm ? a.perm[p + 64] : p + 64) : e0;
    double q0[RP], q1[RP];
    const double v0 = (double)a.v[e0], v1 = two ? (double)a.v[e1] : 0.0;
#pragma unroll
    for (int f = 0; f < RP; ++f) {
      q0[f] = v0;
      q1[f] = v1;
    }
    for (int l = 0; l < a.N; ++l) {
      if (l == a.mode) continue;
      const double* U = a.F.U[l] + rep * a.F.sU[l];
      const double* u0 = U + (int64_t)a.idx[l][e0] * R;
      const double* u1 = U + (int64_t)a.idx[l][e1] * R;
#pragma unroll
      for (int f = 0; f < RP; ++f) {
        if (f < R) {
          q0[f] *= u0[f];
          q1[f] *= u1[f];
        }
      }
    }
#pragma unroll
    for (int f = 0; f < RP; ++f) acc[f] += q0[f] + q1[f];
  }
#pragma unroll
  for (int f = 0; f < RP; ++f) acc[f] = wave_sum(acc[f]);
  if (lane == 0) {
    double* out = S == 1 ? a.M + rep * a.sM + (int64_t)row * R
                         : part + (((int64_t)blockIdx.y * a.rows + row) * S + sl) * R;
#pragma unroll
    for (int f = 0; f < RP; ++f)
      if (f < R) out[f] = acc[f];
  }
}

// M(rep, row, f) = the S partial rows added in range order
__global__ void mttkrp_coo_nd_sum_kernel(MttkrpCooNd a, int S, const double* part) {
  const int64_t n = (int64_t)a.nrep * a.rows * a.R;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int f = (int)(q % a.R);
    const int64_t rr = q / a.R;  // local repetition * rows + row
    const int rl = (int)(rr / a.rows), row = (int)(rr % a.rows);
    const double* p = part + rr * S * a.R + f;
    double s = 0.0;
    for (int k = 0; k < S; ++k) s += p[(int64_t)k * a.R];
    a.M[(a.rep0 + rl) * a.sM + (int64_t)row * a.R + f] = s;
  }
}

// out = the entries of z in the order perm (every coordinate but mode m's,
// and the value): out.idx[l][p] = z.idx[l][perm[p]]
__global__ void gather_sorted_nd_kernel(CooSumNd z, int64_t total, int m, int N,
                                        const int32_t* perm, CooSumNd out) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = perm[p];
    for (int l = 0; l < N; ++l)
      if (l != m) out.idx[l][p] = z.idx[l][e];
    out.v[p] = z.v[e];
  }
}

// nrm[k] = sum of v^2 over slice k of the store (entries [koff[k], koff[k+1]))
__global__ __launch_bounds__(256) void slice_norms_kernel(const float* v, const int64_t* koff,
                                                         int64_t K, double* nrm) {
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= K) return;
  double s = 0.0;
  for (int64_t p = koff[k] + lane; p < koff[k + 1]; p += 64) {
    const double x = v[p];
    s += x * x;
  }
  s = wave_sum(s);
  if (lane == 0) nrm[k] = s;
}

// wavefronts the order-N COO MTTKRP aims at (rows x ranges); its partial rows
// take at most this many R-vectors
constexpr int64_t kNdCooWaves = 16384;

int blocks_for(int64_t n, int cap) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  return (int)(b > cap ? cap : b);
}

}  // namespace

// Stable sort of a batch by its last coordinate and placement behind the
// stored entries (last coordinate + k0); tmp: caller's scratch of
// coo_nd_sort_bytes(nnz) bytes.
size_t coo_nd_sort_bytes(int64_t n) {
  size_t b = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const uint32_t*)nullptr,
                                           (uint32_t*)nullptr, (const int32_t*)nullptr,
                                           (int32_t*)nullptr, (int)(n > 0 ? n : 1));
  size_t c = 0;
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, c, (const uint32_t*)nullptr,
                                         (uint32_t*)nullptr, (int)(n > 0 ? n : 1));
  const size_t words = (size_t)(n > 0 ? n : 1) * 4;  // keys in, keys out, values in, out
  return (b > c ? b : c) + 4 * words + 1024;
}

hipError_t launch_coo_ingest_nd(const CooNd& b, int64_t base, int64_t k0, int nbits,
                                const CooStoreNd& st, void* tmp, size_t tmp_bytes,
                                hipStream_t s) {
  if (b.nnz <= 0) return hipSuccess;
  if (b.nnz > 0x7FFFFFFF) return hipErrorInvalidValue;
  const int64_t n = b.nnz;
  char* t = (char*)tmp;
  uint32_t* kin = (uint32_t*)t;
  uint32_t* kout = kin + n;
  int32_t* vin = (int32_t*)(kout + n);
  int32_t* vout = vin + n;
  void* ctmp = (void*)(((uintptr_t)(vout + n) + 255) & ~(uintptr_t)255);
  const size_t used = (size_t)((char*)ctmp - t);
  if (used > tmp_bytes) return hipErrorInvalidValue;
  size_t cb = tmp_bytes - used;
  last_key_kernel<<<blocks_for(n, 4096), 256, 0, s>>>(b.idx[b.N - 1], n, kin);
  iota_nd_kernel<<<blocks_for(n, 4096), 256, 0, s>>>(vin, n);
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(ctmp, cb, kin, kout, vin, vout, (int)n, 0,
                                                    nbits, s);
  if (e != hipSuccess) return e;
  coo_place_nd_kernel<<<blocks_for(n, 4096), 256, 0, s>>>(b, vout, base, k0, st);
  return hipGetLastError();
}

hipError_t launch_lower_bounds(const int32_t* key, int64_t n, int64_t x0, int64_t x1,
                               int64_t* off, hipStream_t s) {
  if (x1 < x0) return hipSuccess;
  lower_bounds_kernel<<<blocks_for(x1 - x0 + 1, 4096), 256, 0, s>>>(key, n, x0, x1, off);
  return hipGetLastError();
}

hipError_t launch_pos_maps_nd(const PosMapsNd& a, int nrep, int32_t* pos, hipStream_t s) {
  if (nrep <= 0) return hipSuccess;
  pos_maps_kernel<<<dim3(1, (unsigned)nrep), 1024, 0, s>>>(a, pos);
  return hipGetLastError();
}

// flags, their exclusive scan (positions in the concatenated summaries) and
// the emit; at[nrep * nnz] (one past the last) receives the total
size_t coo_nd_scan_bytes(int64_t n) {
  size_t c = 0;
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, c, (const uint32_t*)nullptr,
                                         (uint32_t*)nullptr, (int)(n > 0 ? n : 1));
  return c + 256;
}

hipError_t launch_keep_flags_nd(const CooStoreNd& st, int64_t nnz, const PosViewNd& pv,
                                const int32_t* pos, int nrep, uint32_t* flag, uint32_t* at,
                                void* tmp, size_t tmp_bytes, hipStream_t s) {
  if (nnz <= 0 || nrep <= 0) return hipErrorInvalidValue;
  const int64_t n = (int64_t)nrep * nnz + 1;  // one more: the total lands at at[n - 1]
  if (n > 0x7FFFFFFF) return hipErrorInvalidValue;
  dim3 g((unsigned)blocks_for(nnz, 2048), (unsigned)nrep);
  keep_flags_kernel<<<g, 256, 0, s>>>(st, nnz, pv, pos, flag);
  hipError_t e = launch_fill_u32(flag + (n - 1), 1, 0u, s);
  if (e != hipSuccess) return e;
  size_t cb = tmp_bytes;
  return hipcub::DeviceScan::ExclusiveSum(tmp, cb, flag, at, (int)n, s);
}

hipError_t launch_summary_emit_nd(const CooStoreNd& st, int64_t nnz, const PosViewNd& pv,
                                  const int32_t* pos, int nrep, const uint32_t* flag,
                                  const uint32_t* at, const CooSumNd& z, hipStream_t s) {
  if (nnz <= 0 || nrep <= 0) return hipSuccess;
  dim3 g((unsigned)blocks_for(nnz, 2048), (unsigned)nrep);
  summary_emit_nd_kernel<<<g, 256, 0, s>>>(st, nnz, pv, pos, flag, at, z);
  return hipGetLastError();
}

// per mode m: perm = summary positions sorted by (rep, coordinate m), stably;
// off[rep * (rows + 1) + x] the first sorted position of (rep, x)
size_t coo_nd_mode_sort_bytes(int64_t n) {
  size_t b = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const uint32_t*)nullptr,
                                           (uint32_t*)nullptr, (const int32_t*)nullptr,
                                           (int32_t*)nullptr, (int)(n > 0 ? n : 1));
  return b + 256;
}

hipError_t launch_mode_sort_nd(const CooSumNd& z, int64_t total, int m, int rows, int nrep,
                               uint32_t* key, uint32_t* key_sorted, int32_t* iota,
                               int32_t* perm, int64_t* off, void* tmp, size_t tmp_bytes,
                               hipStream_t s) {
  if (total > 0x7FFFFFFF || nrep > 255 || rows >= (1 << 24)) return hipErrorInvalidValue;
  if (total > 0) {
    mode_keys_kernel<<<blocks_for(total, 4096), 256, 0, s>>>(z, total, m, key);
    iota_nd_kernel<<<blocks_for(total, 4096), 256, 0, s>>>(iota, total);
    size_t b = tmp_bytes;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(tmp, b, key, key_sorted, iota, perm,
                                                      (int)total, 0, 32, s);
    if (e != hipSuccess) return e;
  }
  const int64_t q = (int64_t)nrep * (rows + 1);
  row_offsets_kernel<<<blocks_for(q, 4096), 256, 0, s>>>(key_sorted, total, rows, nrep, off);
  return hipGetLastError();
}

hipError_t launch_gather_sorted_nd(const CooSumNd& z, int N, int64_t total, int m,
                                  const int32_t* perm, const CooSumNd& out, hipStream_t s) {
  if (N < 3 || N > kMaxOrder || m < 0 || m >= N) return hipErrorInvalidValue;
  if (total <= 0) return hipSuccess;
  gather_sorted_nd_kernel<<<blocks_for(total, 4096), 256, 0, s>>>(z, total, m, N, perm, out);
  return hipGetLastError();
}

int64_t mttkrp_coo_nd_parts(int R) { return kNdCooWaves * R; }

int mttkrp_coo_nd_ranges(int rows, int nrep) {
  const int64_t rr = (int64_t)rows * nrep;
  int64_t S = rr > 0 ? kNdCooWaves / rr : 1;
  if (S > 64) S = 64;
  return S < 1 ? 1 : (int)S;
}

hipError_t launch_mttkrp_coo_nd(const MttkrpCooNd& a, double* part, hipStream_t s) {
  if (a.R < 1 || a.R > 32 || a.N < 3 || a.N > kMaxOrder || a.nrep <= 0) return hipErrorInvalidValue;
  if (a.rows <= 0) return hipSuccess;
  const int S = part ? mttkrp_coo_nd_ranges(a.rows, a.nrep) : 1;
  dim3 g((unsigned)(((int64_t)a.rows * S + 3) / 4), (unsigned)a.nrep);
  switch ((a.R + 3) / 4 * 4) {
#define SBT_MCN(RPV) \
  case RPV: timed_launch(mttkrp_coo_nd_kernel<RPV>, g, dim3(256), 0, s, a, S, part); break;
    SBT_MCN(4) SBT_MCN(8) SBT_MCN(12) SBT_MCN(16) SBT_MCN(20) SBT_MCN(24) SBT_MCN(28)
    default: timed_launch(mttkrp_coo_nd_kernel<32>, g, dim3(256), 0, s, a, S, part); break;
#undef SBT_MCN
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || S == 1) return e;
  mttkrp_coo_nd_sum_kernel<<<blocks_for((int64_t)a.nrep * a.rows * a.R, 1024), 256, 0, s>>>(
      a, S, part);
  return hipGetLastError();
}

hipError_t launch_slice_norms(const float* v, const int64_t* koff, int64_t K, double* nrm,
                              hipStream_t s) {
  if (K <= 0) return hipSuccess;
  slice_norms_kernel<<<(unsigned)((K + 3) / 4), 256, 0, s>>>(v, koff, K, nrm);
  return hipGetLastError();
}

}  // namespace sbt
