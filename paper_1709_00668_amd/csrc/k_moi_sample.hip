// Measure of importance (Eq. 1) in exact integer form, and weighted sampling
// without replacement of the indices of every mode (Sec. 3.1, Algorithm 1).
//
// Importance: q(x) = floor(x*x * 2^S) summed in uint64 per index of each mode.
// Integer sums are associative, so the per-index totals do not depend on the
// order the atomics land in: every run and every launch shape gives the same
// weights, which the sampler needs to be reproducible bit for bit.
//
// Sampling: successive sampling proportional to the weights, realised with
// exponential keys kappa_i = E_i / w_i (E_i = -ln U_i, U_i from Philox); the
// n smallest keys win, ties to the smaller index.  One workgroup per
// (repetition, mode) computes the keys, finds the n-th smallest by an 8-bit
// radix select over the 64-bit key patterns (non-negative doubles order like
// their bit patterns), then writes the winners in index order, which leaves
// them sorted ascending.
#include "device_common.hpp"
#include "kernels.hpp"

namespace sbt {

namespace {

__global__ void fill_u64_kernel(uint64_t* p, int64_t n, uint64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

inline int fill_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

__device__ inline double as_f64(double x) { return x; }
__device__ inline double as_f64(float x) { return (double)x; }

template <typename T>
__global__ __launch_bounds__(256) void maxsq_kernel(const T* X, int64_t n, uint64_t* out) {
  uint64_t best = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double x = as_f64(X[i]);
    const double x2 = x * x;
    const uint64_t b = (uint64_t)__double_as_longlong(x2) & 0x7FFFFFFFFFFFFFFFull;
    best = b > best ? b : best;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(best, off, kWave);
    best = o > best ? o : best;
  }
  if (lane_id() == 0) atomicMax((unsigned long long*)out, (unsigned long long)best);
}

// q(x) = floor(x*x * scale); flags a non-finite x or q > qmax.
__device__ inline uint64_t quantize_sq(double x, double scale, uint64_t qmax, bool& bad) {
  const double x2s = (x * x) * scale;
  if (!(x2s < 0x1p63)) {
    bad = true;
    return 0;
  }
  const uint64_t q = (uint64_t)x2s;
  if (q > qmax) bad = true;
  return q;
}

constexpr int kMoiJPerWave = 8;                   // j's per wavefront
constexpr int kMoiJTile = 4 * kMoiJPerWave;       // j's per block
constexpr int kMoiKTile = 8;                      // slices per block

// Block: 64 consecutive i (one per lane) x kMoiJTile j's (wavefront w takes
// j0 + w + 4 jj) x kMoiKTile slices.  Sums stay in registers over the tile:
// per i (lane) over all its j and k, per j over i and k, per k over the
// block (64-bit LDS atomics), and each lands with one 64-bit global atomic
// per block.  Integer sums: the order of the atomics does not matter.
template <typename T>
__global__ __launch_bounds__(256) void moi_dense_kernel(const T* Y, int64_t I, int64_t J,
                                                       int64_t K, double scale, uint64_t qmax,
                                                       uint64_t* w1, uint64_t* w2,
                                                       uint64_t* w3, uint32_t* err) {
  const int lane = lane_id();
  const int wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * kWave + lane;
  const int64_t j0 = (int64_t)blockIdx.y * kMoiJTile;
  const int64_t k0 = (int64_t)blockIdx.z * kMoiKTile;
  __shared__ unsigned long long sk[kMoiKTile];
  __shared__ uint64_t part_i[4][kWave];
  if (threadIdx.x < kMoiKTile) sk[threadIdx.x] = 0ull;
  __syncthreads();
  uint64_t acc_i = 0, acc_j[kMoiJPerWave];
#pragma unroll
  for (int jj = 0; jj < kMoiJPerWave; ++jj) acc_j[jj] = 0;
  bool bad = false;
  for (int kk = 0; kk < kMoiKTile && k0 + kk < K; ++kk) {
    const int64_t k = k0 + kk;
    // branch-free loads (an element outside the tile reads element (0, 0, k)
    // and counts as zero), so that all of them are in flight at once
    T y[kMoiJPerWave];
#pragma unroll
    for (int jj = 0; jj < kMoiJPerWave; ++jj) {
      const int64_t j = j0 + wave + 4 * jj;
      const bool in = i < I && j < J;
      const T v = Y[(in ? i : 0) + I * ((in ? j : 0) + J * k)];
      y[jj] = in ? v : (T)0;
    }
    uint64_t tk = 0;
#pragma unroll
    for (int jj = 0; jj < kMoiJPerWave; ++jj) {
      const uint64_t q = quantize_sq(as_f64(y[jj]), scale, qmax, bad);
      acc_j[jj] += q;
      tk += q;
    }
    acc_i += tk;
    tk = wave_sum_u64(tk);
    if (lane == 0 && tk) atomicAdd(&sk[kk], (unsigned long long)tk);
  }
#pragma unroll
  for (int jj = 0; jj < kMoiJPerWave; ++jj) {
    const int64_t j = j0 + wave + 4 * jj;
    const uint64_t qj = wave_sum_u64(acc_j[jj]);
    if (lane == 0 && j < J && qj) atomicAdd((unsigned long long*)&w2[j], (unsigned long long)qj);
  }
  part_i[wave][lane] = acc_i;
  if (bad) atomicOr(err, 1u);
  __syncthreads();
  if (wave == 0) {
    const uint64_t s = part_i[0][lane] + part_i[1][lane] + part_i[2][lane] + part_i[3][lane];
    if (i < I && s) atomicAdd((unsigned long long*)&w1[i], (unsigned long long)s);
  }
  if (threadIdx.x < kMoiKTile && k0 + threadIdx.x < K && sk[threadIdx.x])
    atomicAdd((unsigned long long*)&w3[k0 + threadIdx.x], sk[threadIdx.x]);
}

// q(v) = floor(v*v*scale) added to the importance of every mode's coordinate;
// err bit 1: non-finite value or overflow, bit 2: coordinate out of range
__global__ void moi_coo_nd_kernel(CooNd b, double scale, uint64_t qmax, NdWeights w,
                                  uint32_t* err) {
  bool bad = false, oob = false;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < b.nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    bool in = true;
    for (int m = 0; m < b.N; ++m) {
      const int32_t x = b.idx[m][e];
      in = in && x >= 0 && x < b.D[m];
    }
    if (!in) {
      oob = true;
      continue;
    }
    const uint64_t q = quantize_sq((double)b.v[e], scale, qmax, bad);
    if (q == 0) continue;
    for (int m = 0; m < b.N; ++m)
      atomicAdd((unsigned long long*)&w.w[m][b.idx[m][e]], (unsigned long long)q);
  }
  if (bad) atomicOr(err, 1u);
  if (oob) atomicOr(err, 2u);
}

__global__ __launch_bounds__(256) void moi_coo_kernel(const int32_t* ii, const int32_t* jj,
                                                     const int32_t* kk, const float* v,
                                                     int64_t nnz, int64_t I, int64_t J,
                                                     int64_t K, double scale, uint64_t qmax,
                                                     uint64_t* w1, uint64_t* w2, uint64_t* w3,
                                                     uint32_t* err) {
  bool bad = false, oob = false;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = ii[e], j = jj[e], k = kk[e];
    if (i < 0 || i >= I || j < 0 || j >= J || k < 0 || k >= K) {
      oob = true;
      continue;
    }
    const uint64_t q = quantize_sq((double)v[e], scale, qmax, bad);
    if (q) {
      atomicAdd((unsigned long long*)&w1[i], (unsigned long long)q);
      atomicAdd((unsigned long long*)&w2[j], (unsigned long long)q);
      atomicAdd((unsigned long long*)&w3[k], (unsigned long long)q);
    }
  }
  if (bad) atomicOr(err, 1u);
  if (oob) atomicOr(err, 2u);
}

// ---------------------------------------------------------------------------
// Importance of a dense block of order N.  The block is read as D_0 rows x
// (D_1 ... D_N-1) columns; a wavefront takes 64 consecutive rows (one per
// lane) of kMoiNdCols consecutive columns, kMoiNdLoads column loads in
// flight.  Row sums stay in the lanes.  Each column's sum goes to every
// higher mode: mode 1 (whose index changes with every column) into per-block
// sums in LDS, flushed with one atomic per index at the end; higher modes,
// whose indices change rarely, into register runs of equal index, one atomic
// per run.  Integer sums, so the order of the atomics does not matter.
// ---------------------------------------------------------------------------
constexpr int kMoiNdCols = 128;
constexpr int kMoiNdLoads = 8;
constexpr int kMoiNdLds1 = 2048;  // mode-1 extents summed in LDS

template <typename T>
__global__ __launch_bounds__(256) void moi_nd_kernel(MoiNd a) {
  __shared__ unsigned long long s1[kMoiNdLds1];
  const T* X = (const T*)a.X;
  const int N = a.N;
  const int64_t D0 = a.D[0], D1 = a.D[1];
  const bool priv = D1 <= kMoiNdLds1;
  int64_t ncols = 1;
  for (int m = 1; m < N; ++m) ncols *= a.D[m];
  const int lane = lane_id();
  const int wave = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)blockIdx.y * kWave + lane;
  const bool in = i0 < D0;
  if (priv)
    for (int64_t i = threadIdx.x; i < D1; i += 256) s1[i] = 0ull;
  __syncthreads();
  const int64_t cb = ((int64_t)blockIdx.x * 4 + wave) * kMoiNdCols;
  const int64_t ce = cb + kMoiNdCols < ncols ? cb + kMoiNdCols : ncols;
  int64_t idx[kMaxOrder], cur[kMaxOrder];
  unsigned long long run[kMaxOrder];
  int64_t rem = cb < ncols ? cb : 0;
#pragma unroll
  for (int m = 1; m < kMaxOrder; ++m) {
    if (m < N) {
      idx[m] = rem % a.D[m];
      rem /= a.D[m];
    } else {
      idx[m] = 0;
    }
    cur[m] = idx[m];
    run[m] = 0ull;
  }
  unsigned long long acc0 = 0ull;
  bool bad = false;
  for (int64_t c0 = cb; c0 < ce; c0 += kMoiNdLoads) {
    // branch-free loads (outside the tile: element (0, column c0), dropped)
    double x[kMoiNdLoads];
#pragma unroll
    for (int u = 0; u < kMoiNdLoads; ++u) {
      const bool v = in && c0 + u < ce;
      const double y = (double)X[(v ? i0 : 0) + D0 * (v ? c0 + u : c0)];
      x[u] = v ? y : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kMoiNdLoads; ++u) {
      if (c0 + u >= ce) break;  // uniform over the wavefront
      const uint64_t q = quantize_sq(x[u], a.scale, a.qmax, bad);
      acc0 += q;
      const unsigned long long col = wave_sum_u64(q);
      if (lane == 0 && col) {
        if (priv)
          atomicAdd(&s1[idx[1]], col);
        else
          atomicAdd((unsigned long long*)&a.w[1][idx[1]], col);
      }
#pragma unroll
      for (int m = 2; m < kMaxOrder; ++m) {
        if (m < N) {
          if (idx[m] != cur[m]) {
            if (lane == 0 && run[m]) atomicAdd((unsigned long long*)&a.w[m][cur[m]], run[m]);
            cur[m] = idx[m];
            run[m] = 0ull;
          }
          run[m] += col;
        }
      }
      // next column's indices (mode 1 fastest)
      for (int m = 1; m < N; ++m) {
        if (++idx[m] < a.D[m]) break;
        idx[m] = 0;
      }
    }
  }
#pragma unroll
  for (int m = 2; m < kMaxOrder; ++m)
    if (m < N && lane == 0 && run[m]) atomicAdd((unsigned long long*)&a.w[m][cur[m]], run[m]);
  if (in && acc0) atomicAdd((unsigned long long*)&a.w[0][i0], acc0);
  if (bad) atomicOr(a.err, 1u);
  __syncthreads();
  if (priv)
    for (int64_t i = threadIdx.x; i < D1; i += 256)
      if (s1[i]) atomicAdd((unsigned long long*)&a.w[1][i], s1[i]);
}

// ---------------------------------------------------------------------------
// Sampler
// ---------------------------------------------------------------------------
constexpr int kSampleThreads = 1024;

__device__ inline uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__global__ __launch_bounds__(kSampleThreads) void sample_kernel(SampleArgs a, uint64_t* keys_all,
                                                               int32_t* idx_all) {
  const int rep = blockIdx.x;
  const int m = blockIdx.y;
  const int tid = threadIdx.x;
  const int64_t N = a.N[m];
  const int64_t n = a.n[m] < N ? a.n[m] : N;
  const uint64_t* w = a.w[m];
  uint64_t* keys = keys_all + rep * a.key_stride + a.key_off[m];
  int32_t* out = idx_all + rep * a.idx_stride + a.idx_off[m];
  const RngKey key = rng_key(a.seed, a.tensor_id);
  const uint32_t tag = rng_tag(kStreamSample, (uint32_t)(a.mode0 + m + 1), (uint32_t)rep);

  // 1. keys kappa_i = -ln(U_i) / double(w_i), +inf for w_i == 0
  for (int64_t i = tid; i < N; i += kSampleThreads) {
    const uint64_t u = rng_bits(key, (uint32_t)i, 0u, tag, a.t);
    const double E = -ln_basic(uniform_open(u));
    const uint64_t wi = w[i];
    uint64_t bits = 0x7FF0000000000000ull;  // +inf
    if (wi) {
#pragma clang fp contract(off)
      const double kap = E / (double)wi;
      bits = (uint64_t)__double_as_longlong(kap);
    }
    keys[i] = bits;
  }
  __syncthreads();

  // 2. radix select: the n-th smallest key T and how many keys equal to T to take
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_prefix;
  __shared__ int64_t s_want;
  uint64_t prefix = 0, mask = 0;
  int64_t want = n;
  if (n > 0) {
    for (int shift = 56; shift >= 0; shift -= 8) {
      for (int d = tid; d < 256; d += kSampleThreads) hist[d] = 0;
      __syncthreads();
      for (int64_t i = tid; i < N; i += kSampleThreads) {
        const uint64_t kv = keys[i];
        if ((kv & mask) == prefix) atomicAdd(&hist[(kv >> shift) & 0xFF], 1u);
      }
      if (tid == 0) {
        s_prefix = prefix;
        s_want = want;
      }
      __syncthreads();
      // the digit where the running count reaches `want`: wavefront 0, four
      // digits per lane, prefix sums across the lanes
      if (tid < kWave) {
        const int d0 = 4 * tid;
        const int64_t h0 = hist[d0], h1 = hist[d0 + 1], h2 = hist[d0 + 2], h3 = hist[d0 + 3];
        const int64_t tot = h0 + h1 + h2 + h3;
        int64_t incl = tot;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
          const int64_t o = __shfl_up(incl, off, kWave);
          if (tid >= off) incl += o;
        }
        int64_t cum = incl - tot;
        if (cum < want && incl >= want) {
          const int64_t hh[4] = {h0, h1, h2, h3};
          for (int k = 0; k < 4; ++k) {
            if (cum + hh[k] >= want) {
              s_prefix = prefix | ((uint64_t)(d0 + k) << shift);
              s_want = want - cum;
              break;
            }
            cum += hh[k];
          }
        }
      }
      __syncthreads();
      prefix = s_prefix;
      want = s_want;
      mask |= 0xFFull << shift;
    }
  }
  const uint64_t T = prefix;
  const int64_t ties_needed = n > 0 ? want : 0;

  // 3. stable compaction in index order
  __shared__ uint32_t wcnt_eq[kSampleThreads / kWave], wcnt_sel[kSampleThreads / kWave];
  __shared__ int64_t run_eq, run_sel;
  if (tid == 0) {
    run_eq = 0;
    run_sel = 0;
  }
  __syncthreads();
  const int wave = tid >> 6;
  for (int64_t base = 0; base < N; base += kSampleThreads) {
    const int64_t i = base + tid;
    const uint64_t kv = i < N ? keys[i] : ~0ull;
    const bool in = i < N && n > 0;
    const bool lt = in && kv < T;
    const bool eq = in && kv == T;
    const uint64_t beq = __ballot(eq);
    if (lane_id() == 0) wcnt_eq[wave] = (uint32_t)__popcll(beq);
    __syncthreads();
    int64_t pre_eq = run_eq;
    for (int q = 0; q < wave; ++q) pre_eq += wcnt_eq[q];
    const int64_t tie_rank = pre_eq + __popcll(beq & lanemask_lt());
    const bool sel = lt || (eq && tie_rank < ties_needed);
    const uint64_t bsel = __ballot(sel);
    if (lane_id() == 0) wcnt_sel[wave] = (uint32_t)__popcll(bsel);
    __syncthreads();
    int64_t pre_sel = run_sel;
    for (int q = 0; q < wave; ++q) pre_sel += wcnt_sel[q];
    const int64_t pos = pre_sel + __popcll(bsel & lanemask_lt());
    if (sel && pos < n) out[pos] = (int32_t)i;
    __syncthreads();
    if (tid == 0) {
      int64_t te = 0, ts = 0;
      for (int q = 0; q < kSampleThreads / kWave; ++q) {
        te += wcnt_eq[q];
        ts += wcnt_sel[q];
      }
      run_eq += te;
      run_sel += ts;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_u64_kernel<<<fill_blocks(n), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_u32_kernel<<<fill_blocks(n), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_f64_kernel<<<fill_blocks(n), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_maxsq_dense(int prec, const void* X, int64_t n, uint64_t* out_bits,
                              hipStream_t s) {
  hipError_t e = launch_fill_u64(out_bits, 1, 0, s);
  if (e != hipSuccess || n <= 0) return e;
  if (prec == kF64)
    maxsq_kernel<double><<<fill_blocks(n), 256, 0, s>>>((const double*)X, n, out_bits);
  else
    maxsq_kernel<float><<<fill_blocks(n), 256, 0, s>>>((const float*)X, n, out_bits);
  return hipGetLastError();
}

hipError_t launch_maxsq_coo(const float* v, int64_t n, uint64_t* out_bits, hipStream_t s) {
  hipError_t e = launch_fill_u64(out_bits, 1, 0, s);
  if (e != hipSuccess || n <= 0) return e;
  maxsq_kernel<float><<<fill_blocks(n), 256, 0, s>>>(v, n, out_bits);
  return hipGetLastError();
}

hipError_t launch_moi_dense(int prec, const void* Y, int64_t I, int64_t J, int64_t K,
                            double scale, uint64_t qmax, uint64_t* w1, uint64_t* w2,
                            uint64_t* w3, uint32_t* err, hipStream_t s) {
  if (I <= 0 || J <= 0 || K <= 0) return hipSuccess;
  dim3 grid((unsigned)((I + kWave - 1) / kWave), (unsigned)((J + kMoiJTile - 1) / kMoiJTile),
            (unsigned)((K + kMoiKTile - 1) / kMoiKTile));
  if (prec == kF64)
    moi_dense_kernel<double><<<grid, 256, 0, s>>>((const double*)Y, I, J, K, scale, qmax, w1, w2,
                                                  w3, err);
  else
    moi_dense_kernel<float><<<grid, 256, 0, s>>>((const float*)Y, I, J, K, scale, qmax, w1, w2,
                                                 w3, err);
  return hipGetLastError();
}

hipError_t launch_moi_coo(const int32_t* ii, const int32_t* jj, const int32_t* kk,
                          const float* v, int64_t nnz, int64_t I, int64_t J, int64_t K,
                          double scale, uint64_t qmax, uint64_t* w1, uint64_t* w2,
                          uint64_t* w3, uint32_t* err, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  moi_coo_kernel<<<fill_blocks(nnz), 256, 0, s>>>(ii, jj, kk, v, nnz, I, J, K, scale, qmax, w1,
                                                  w2, w3, err);
  return hipGetLastError();
}

hipError_t launch_moi_coo_nd(const CooNd& b, double scale, uint64_t qmax, const NdWeights& w,
                             uint32_t* err, hipStream_t s) {
  if (b.nnz <= 0) return hipSuccess;
  moi_coo_nd_kernel<<<fill_blocks(b.nnz), 256, 0, s>>>(b, scale, qmax, w, err);
  return hipGetLastError();
}

hipError_t launch_moi_nd(int prec, const MoiNd& a, hipStream_t s) {
  if (a.N < 2 || a.N > kMaxOrder) return hipErrorInvalidValue;
  int64_t ncols = 1;
  for (int m = 0; m < a.N; ++m) {
    if (a.D[m] <= 0) return hipSuccess;
    if (m > 0) ncols *= a.D[m];
  }
  const int64_t chunks = (ncols + 4 * kMoiNdCols - 1) / (4 * kMoiNdCols);
  const int64_t tiles = (a.D[0] + kWave - 1) / kWave;
  if (chunks > 0x7FFFFFFF || tiles > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)chunks, (unsigned)tiles);
  if (prec == kF64)
    moi_nd_kernel<double><<<grid, 256, 0, s>>>(a);
  else
    moi_nd_kernel<float><<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_sample(const SampleArgs& a, uint64_t* keys, int32_t* idx, hipStream_t s) {
  if (a.nrep <= 0) return hipSuccess;
  const int modes = a.nmodes > 0 ? a.nmodes : 3;
  if (modes > 3 || a.mode0 < 0) return hipErrorInvalidValue;
  sample_kernel<<<dim3((unsigned)a.nrep, (unsigned)modes), kSampleThreads, 0, s>>>(a, keys, idx);
  return hipGetLastError();
}

}  // namespace sbt
