// The update on tensors of order N >= 3 whose last mode grows (Sec. 2 notes
// that the problem and the method carry over to any number of modes): the
// kernels with no third-order counterpart.  The MTTKRPs reuse the
// third-order passes on a three-way view of the summary (leading modes
// merged, trailing modes merged), with the Khatri-Rao rows of the merged
// modes built here.
#include "assign_device.hpp"
#include "device_common.hpp"
#include "kernels.hpp"

namespace sbt {

namespace {

__global__ void krp_nd_kernel(NdFactors F, int lo, int hi, int R, int rep0, int64_t rows,
                              double* out, int64_t sOut) {
  const int rep = rep0 + blockIdx.y;
  const int64_t n = rows * R;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    int64_t p = q / R;
    const int f = (int)(q % R);
    double v = 1.0;
    for (int l = lo; l < hi; ++l) {
      const int64_t a = p % F.n[l];
      p /= F.n[l];
      v *= F.U[l][rep * F.sU[l] + a * R + f];
    }
    out[rep * sOut + q] = v;
  }
}

__global__ void hadamard_nd_kernel(const double* G, int64_t sMode, int64_t sG, uint32_t mask,
                                   int N, int R, int rep0, double* out) {
  const int rep = rep0 + blockIdx.x;
  for (int q = threadIdx.x; q < R * R; q += blockDim.x) {
    double v = 1.0;
    for (int m = 0; m < N; ++m)
      if (mask & (1u << m)) v *= G[m * sMode + rep * sG + q];
    out[rep * sG + q] = v;
  }
}

__global__ void als_init_nd_kernel(NdFactors F, int N, int R, int rep0, uint64_t seed,
                                   uint32_t tensor_id, uint32_t stream, uint32_t t) {
  const int rep = rep0 + blockIdx.y;
  const RngKey key = rng_key(seed, tensor_id);
  int64_t total = 0;
  for (int m = 1; m < N; ++m) total += (int64_t)F.n[m] * R;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    int m = 1;
    int64_t qq = q;
    while (qq >= (int64_t)F.n[m] * R) {
      qq -= (int64_t)F.n[m] * R;
      ++m;
    }
    const uint32_t row = (uint32_t)(qq / R), col = (uint32_t)(qq % R);
    const uint32_t tag = rng_tag(stream, (uint32_t)(m + 1), (uint32_t)rep);
    F.U[m][rep * F.sU[m] + qq] = uniform_closed0(rng_bits(key, row, col, tag, t));
  }
}

// summary element from a store element: the same type, or BF16 (nearest even)
// from FP32
__device__ inline double to_summary(double x, double*) { return x; }
__device__ inline float to_summary(float x, float*) { return x; }
__device__ inline uint16_t to_summary(float x, uint16_t*) { return f32_to_bf16_rne(x); }

// one thread per summary element, the first summary index fastest
template <typename TIn, typename TZ>
__global__ __launch_bounds__(256) void gather_nd_kernel(GatherNd g) {
  const int rep = g.rep0 + blockIdx.y;
  int64_t total = 1;
  for (int m = 0; m < g.N; ++m) total *= g.n[m];
  const int32_t* S = g.idx + rep * g.idx_stride;
  const TIn* X = (const TIn*)g.X;
  TZ* Z = (TZ*)g.Z + rep * g.sZ;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = e, src = 0, stride = 1;
    for (int m = 0; m < g.N - 1; ++m) {
      const int64_t a = rem % g.n[m];
      rem /= g.n[m];
      src += (int64_t)S[g.off[m] + a] * stride;
      stride *= g.D[m];
    }
    const int c = (int)rem;
    const int64_t kk = c < g.n3old ? (int64_t)S[g.off[g.N - 1] + c] : g.Kold + (c - g.n3old);
    src += kk * stride;
    Z[e] = to_summary(X[src], Z);
  }
}

// R x R products over rows, thread per entry (f, g) with a fixed row order
__global__ __launch_bounds__(256) void cross_nd_kernel(CrossNd c) {
  const int job = blockIdx.x, rep = c.rep0 + blockIdx.y;
  const XJob& j = c.job[job];
  const int R = c.R;
  const double* X = j.X + rep * j.sX;
  const double* Y = j.Y + rep * j.sY;
  const int32_t* ix = j.ix ? j.ix + rep * j.six : nullptr;
  const int32_t* iy = j.iy ? j.iy + rep * j.siy : nullptr;
  double* out = c.out + ((int64_t)rep * c.njobs + job) * R * R;
  for (int q = threadIdx.x; q < R * R; q += blockDim.x) {
    const int f = q / R, g = q % R;
    double acc = 0.0;
    for (int i = 0; i < j.rows; ++i) {
      const int64_t rx = ix ? ix[i] : i, ry = iy ? iy[i] : i;
      acc += X[rx * R + f] * Y[ry * R + g];
    }
    out[q] = acc;
  }
}

__global__ __launch_bounds__(256) void match_nd_kernel(MatchNd mt) {
  const int rep = mt.rep0 + blockIdx.x;
  const int N = mt.N, R = mt.R, RR = R * R;
  const int tid = threadIdx.x;
  const double* xo = mt.xo + (int64_t)rep * 3 * N * RR;  // per mode: cross, anchor Gram, sample Gram
  __shared__ double S[kMaxRank][kMaxRank + 1];
  __shared__ double na[kMaxOrder][kMaxRank], ns[kMaxOrder][kMaxRank];
  __shared__ double scl[kMaxOrder][kMaxRank];
  __shared__ int pi_s[kMaxRank];
  for (int q = tid; q < N * R; q += 256) {
    const int m = q / R, f = q % R;
    const double da = xo[(3 * m + 1) * RR + f * R + f];
    const double ds = xo[(3 * m + 2) * RR + f * R + f];
    na[m][f] = sqrt(da > 0.0 ? da : 0.0);
    ns[m][f] = sqrt(ds > 0.0 ? ds : 0.0);
  }
  __syncthreads();
  for (int q = tid; q < RR; q += 256) {
    const int f = q / R, g = q % R;
    double sv = 1.0;
    for (int m = 0; m < N; ++m) {
      const double d = na[m][f] * ns[m][g];
      const double cs = d > 0.0 ? xo[3 * m * RR + q] / d : 0.0;
      sv *= fabs(cs);
    }
    S[f][g] = sv >= 0.0 ? sv : 0.0;  // a non-finite similarity counts as none
  }
  __syncthreads();
  if (tid < R) pi_s[tid] = tid;
  __syncthreads();
  if (tid < kWave) hungarian_wave(S, R, pi_s);
  __syncthreads();
  for (int q = tid; q < (N - 1) * R; q += 256) {
    const int m = q / R, f = q % R, g = pi_s[f];
    const double sg = xo[3 * m * RR + f * R + g] < 0.0 ? -1.0 : 1.0;
    const double v = ns[m][g] > 0.0 ? sg * na[m][f] / ns[m][g] : 0.0;
    scl[m][f] = v;
    mt.scl[((int64_t)rep * kMaxOrder + m) * R + f] = v;
  }
  if (tid < R) {
    bool ok = true;
    for (int m = 0; m < N - 1; ++m) ok = ok && na[m][tid] > 0.0;
    mt.pi[rep * R + tid] = pi_s[tid];
    mt.valid[rep * R + tid] = ok ? 1 : 0;
  }
  __syncthreads();
  for (int q = tid; q < RR; q += 256) {
    const int f = q / R, g = q % R, pf = pi_s[f], pg = pi_s[g];
    double v = 1.0;
    for (int m = 0; m < N - 1; ++m) v *= scl[m][f] * scl[m][g] * xo[(3 * m + 2) * RR + pf * R + pg];
    mt.Gt[(int64_t)rep * RR + q] = v;
  }
}

__global__ void match_rows_nd_kernel(NdFactors Up, NdFactors Ut, int N, int R, int rep0,
                                     const double* scl, const int32_t* pi) {
  const int rep = rep0 + blockIdx.y;
  int64_t total = 0;
  for (int m = 0; m < N - 1; ++m) total += (int64_t)Up.n[m] * R;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    int m = 0;
    int64_t qq = q;
    while (qq >= (int64_t)Up.n[m] * R) {
      qq -= (int64_t)Up.n[m] * R;
      ++m;
    }
    const int64_t a = qq / R;
    const int f = (int)(qq % R);
    Ut.U[m][rep * Ut.sU[m] + qq] = scl[((int64_t)rep * kMaxOrder + m) * R + f] *
                                   Up.U[m][rep * Up.sU[m] + a * R + pi[rep * R + f]];
  }
}

// position of v in the ascending list s[0..n), or -1
__device__ inline int find_sorted_nd(const int32_t* s, int n, int64_t v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)s[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < n && (int64_t)s[lo] == v) ? lo : -1;
}

// One thread per model entry of every part; each entry is read and written by
// its own thread only, so the model is updated in place.
__global__ __launch_bounds__(256) void commit_nd_kernel(CommitNd c) {
  if (*c.err) return;
  const int N = c.N, R = c.R;
  const int64_t Kold = c.D[N - 1];
  int64_t part[2 * kMaxOrder + 2];
  int np = 0;
  for (int m = 0; m < N; ++m) part[np++] = c.D[m] * R;  // zero fill (last: old rows)
  part[np++] = c.Knew * R;                              // new rows of the last factor
  for (int m = 0; m < N - 1; ++m) part[np++] = c.D[m];  // importance of the fixed modes
  part[np++] = c.Knew;                                  // importance of the new slices
  int64_t total = 0;
  for (int p = 0; p < np; ++p) total += part[p];
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    int p = 0;
    int64_t qq = q;
    while (qq >= part[p]) {
      qq -= part[p];
      ++p;
    }
    if (p < N) {  // zero fill of factor p
      const int m = p;
      const int64_t i = qq / R;
      const int f = (int)(qq % R);
      double* u = c.U[m] + qq;
      if (*u != 0.0) continue;
      double acc = 0.0;
      int cnt = 0;
      for (int rep = 0; rep < c.nrep; ++rep) {
        if (!c.valid[rep * R + f]) continue;
        const int pos = find_sorted_nd(c.idx + rep * c.idx_stride + c.off[m], c.n[m], i);
        if (pos < 0) continue;
        const double v = m < N - 1 ? c.Ut[m][rep * c.sUt[m] + (int64_t)pos * R + f]
                                   : c.Ct[rep * c.sCt + (int64_t)pos * R + f];
        acc += v;
        ++cnt;
      }
      if (cnt) *u = acc / cnt;
    } else if (p == N) {  // new rows: average over the valid repetitions, ascending
      const int64_t k = qq / R;
      const int f = (int)(qq % R);
      double acc = 0.0;
      int cnt = 0;
      for (int rep = 0; rep < c.nrep; ++rep) {
        if (!c.valid[rep * R + f]) continue;
        acc += c.Ct[rep * c.sCt + (int64_t)(c.n[N - 1] + k) * R + f];
        ++cnt;
      }
      c.U[N - 1][(Kold + k) * R + f] = cnt ? acc / cnt : 0.0;
    } else if (p < 2 * N) {
      const int m = p - N - 1;
      c.w[m][qq] += c.dw[m][qq];
    } else {
      c.w[N - 1][Kold + qq] = c.dw[N - 1][qq];
    }
  }
}

__global__ __launch_bounds__(256) void sort_nd_kernel(NdFactors F, int N, int R, double* lam) {
  __shared__ int perm[kMaxRank];
  __shared__ double lam_s[kMaxRank];
  if (threadIdx.x == 0) {
    for (int f = 0; f < R; ++f) {
      perm[f] = f;
      lam_s[f] = lam[f];
    }
    // stable insertion sort, largest lambda first
    for (int a = 1; a < R; ++a) {
      const int pa = perm[a];
      int b = a;
      while (b > 0 && lam_s[perm[b - 1]] < lam_s[pa]) {
        perm[b] = perm[b - 1];
        --b;
      }
      perm[b] = pa;
    }
  }
  __syncthreads();
  int64_t rows = 0;
  for (int m = 0; m < N; ++m) rows += F.n[m];
  double row[kMaxRank];
  for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) {
    int m = 0;
    int64_t rr = r;
    while (rr >= F.n[m]) {
      rr -= F.n[m];
      ++m;
    }
    double* u = F.U[m] + rr * R;
    for (int f = 0; f < R; ++f) row[f] = u[f];
    for (int f = 0; f < R; ++f) u[f] = row[perm[f]];
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int f = 0; f < R; ++f) lam[f] = lam_s[perm[f]];
}

// W(e, f) = sum_q Z(e, q) C(q, f) on a three-way view (e = a + n1 b, q = c)
// whose rows are few and whose contraction is long, as the leading-mode
// views of an order-N summary are.  A block takes 64 V consecutive rows (V
// per lane: BF16 summaries take two, so that a lane reads 4 bytes per load)
// and one of S ranges of q; its four wavefronts split the range again, each
// with kP1sLoads summary loads in flight, over C rows staged in LDS.  The
// wavefronts' rows add up in LDS in wavefront order; with S > 1 each range
// writes a partial W that a second kernel sums in range order.
// The row tiles of one (range, repetition) go to one XCD: workgroup b runs
// on XCD b mod 8, and the (tile, range, repetition) triples are dealt to the
// XCDs in contiguous runs.  A view's rows of one q start wherever n12 q puts
// them, so two neighbouring tiles share a 128-byte line at their boundary;
// with both tiles on one XCD that line comes from HBM once, into one L2.
constexpr int kP1sLoads = 4;
constexpr int kP1sXcds = 8;
constexpr int kP1sMaxRows = 128;  // C rows one block stages

template <typename TZ> struct AccNd { using type = float; };
template <> struct AccNd<double> { using type = double; };

// V consecutive summary elements in the accumulation type (BF16 summaries
// widen to FP32; two BF16 elements come from one 4-byte load)
template <int V> __device__ inline void acc_of(const double* p, double (&z)[V]) { z[0] = *p; }
template <int V> __device__ inline void acc_of(const float* p, float (&z)[V]) { z[0] = *p; }
template <int V> __device__ inline void acc_of(const uint16_t* p, float (&z)[V]) {
  if constexpr (V == 2) {
    const uint32_t w = *reinterpret_cast<const uint32_t*>(p);
    z[0] = bf16_to_f32((uint16_t)(w & 0xFFFFu));
    z[1] = bf16_to_f32((uint16_t)(w >> 16));
  } else {
    z[0] = bf16_to_f32(*p);
  }
}

template <typename TZ, int RP, int V>
__global__ __launch_bounds__(256) void p1s_kernel(RepSet rs, const TZ* Z, const double* Cf, int S,
                                                 typename AccNd<TZ>::type* Wp, int64_t sWp,
                                                 NdFactors F, int c0, int N, int tiles) {
  using TA = typename AccNd<TZ>::type;
  __shared__ TA Cs[kP1sMaxRows][RP];
  __shared__ TA red[64 * V][RP + 1];
  const int64_t total = (int64_t)tiles * S * rs.nrep;
  const int64_t per = (total + kP1sXcds - 1) / kP1sXcds;
  const int64_t lin = (int64_t)(blockIdx.x % kP1sXcds) * per + blockIdx.x / kP1sXcds;
  if (lin >= total) return;  // the whole block: no barrier has been reached
  const int tile = (int)(lin % tiles);
  const int sp = (int)((lin / tiles) % S);
  const int rep = rs.rep0 + (int)(lin / ((int64_t)tiles * S));
  const int R = rs.R, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  const int Q = rs.n3;
  const int qs = (int)((int64_t)sp * Q / S), qe = (int)((int64_t)(sp + 1) * Q / S);
  const int L = qe - qs;  // <= kP1sMaxRows (host-chosen S)
  const int64_t e = ((int64_t)tile * 64 + lane) * V;  // first of the lane's V rows
  const bool ok = e < n12;  // (V = 2 only when n12 is even)
  if (c0 < 0) {
    const double* C = Cf + rep * rs.sC + (int64_t)qs * R;
    for (int q = threadIdx.x; q < L * RP; q += 256) {
      const int r = q / RP, f = q % RP;
      Cs[r][f] = f < R ? (TA)C[(int64_t)r * R + f] : (TA)0;
    }
  } else {
    // Khatri-Rao rows of the factors of modes c0..N-1 formed while staging
    // (the same products, in the same order, as krp_nd_kernel)
    for (int q = threadIdx.x; q < L * RP; q += 256) {
      const int r = q / RP, f = q % RP;
      double v = 0.0;
      if (f < R) {
        int64_t p = qs + r;
        v = 1.0;
        for (int l = c0; l < N; ++l) {
          const int64_t a = p % F.n[l];
          p /= F.n[l];
          v *= F.U[l][rep * F.sU[l] + a * R + f];
        }
      }
      Cs[r][f] = (TA)v;
    }
  }
  __syncthreads();
  const int w0 = (wave * L) / 4, w1 = ((wave + 1) * L) / 4;
  const TZ* zp = Z + rep * rs.sZ + (ok ? e : 0) + n12 * qs;
  TA acc[V][RP];
#pragma unroll
  for (int v = 0; v < V; ++v)
#pragma unroll
    for (int f = 0; f < RP; ++f) acc[v][f] = 0;
  int q = w0;
  for (; q + kP1sLoads <= w1; q += kP1sLoads) {
    // branch-free loads (zp is a valid row when !ok; its values are dropped)
    TA z[kP1sLoads][V];
#pragma unroll
    for (int u = 0; u < kP1sLoads; ++u) {
      acc_of<V>(zp + n12 * (q + u), z[u]);
#pragma unroll
      for (int v = 0; v < V; ++v) z[u][v] = ok ? z[u][v] : (TA)0;
    }
#pragma unroll
    for (int u = 0; u < kP1sLoads; ++u)
#pragma unroll
      for (int f = 0; f < RP; ++f) {
        const TA c = Cs[q + u][f];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v][f] += z[u][v] * c;
      }
  }
  for (; q < w1; ++q) {
    TA z[V];
    acc_of<V>(zp + n12 * q, z);
#pragma unroll
    for (int v = 0; v < V; ++v) z[v] = ok ? z[v] : (TA)0;
#pragma unroll
    for (int f = 0; f < RP; ++f) {
      const TA c = Cs[q][f];
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v][f] += z[v] * c;
    }
  }
  // the four wavefronts' rows, added in wavefront order
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int f = 0; f < RP; ++f)
          red[lane * V + v][f] = w == 0 ? acc[v][f] : red[lane * V + v][f] + acc[v][f];
    }
    __syncthreads();
  }
  if (ok) {
    TA* out = Wp + rep * sWp + (int64_t)sp * R * n12;
    for (int f = 0; f < R; ++f)
#pragma unroll
      for (int v = 0; v < V; ++v) out[f * n12 + e + v] = red[lane * V + v][f];
  }
}

// W(f, e) = sum over the S ranges of the partials, in range order
template <typename TA>
__global__ __launch_bounds__(256) void p1s_sum_kernel(RepSet rs, int S, const TA* Wp,
                                                     int64_t sWp, TA* W) {
  const int rep = rs.rep0 + blockIdx.y;
  const int64_t n = (int64_t)rs.n1 * rs.n2 * rs.R;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const TA* p = Wp + rep * sWp + i;
    TA v = p[0];
    for (int sp = 1; sp < S; ++sp) v += p[sp * n];
    W[rep * rs.sW + i] = v;
  }
}

int grid_blocks(int64_t n, int cap) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  return (int)(b > cap ? cap : b);
}

}  // namespace

int p1s_splits(int64_t n12, int Q, int nrep) {
  const int64_t tiles = (n12 + 63) / 64;
  int64_t S = (2048 + tiles * nrep - 1) / (tiles * nrep);  // about 2048 blocks
  const int64_t most = Q / 32 > 1 ? Q / 32 : 1;             // at least 8 rows per wavefront
  if (S > most) S = most;
  const int64_t least = (Q + kP1sMaxRows - 1) / kP1sMaxRows;  // staged rows fit LDS
  if (S < least) S = least;
  if (S < 1) S = 1;
  return (int)S;
}

hipError_t launch_p1s(int prec, const RepSet& rs, const void* Z, const double* Cf, int S,
                      void* Wp, int64_t sWp, void* W, hipStream_t s, const NdFactors* krp, int c0,
                      int N) {
  const NdFactors F = krp ? *krp : NdFactors{};
  if (krp && (c0 < 0 || c0 >= N || N > kMaxOrder)) return hipErrorInvalidValue;
  const int kc0 = krp ? c0 : -1;
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  if (S < 1 || (rs.n3 + S - 1) / S > kP1sMaxRows) return hipErrorInvalidValue;
  void* out = S == 1 ? W : Wp;
  const int64_t so = S == 1 ? rs.sW : sWp;
  if (S > 1 && sWp < (int64_t)S * n12 * rs.R) return hipErrorInvalidValue;
  // BF16 summaries: two rows per lane when every lane's pair is 4-byte aligned
  const bool pair = prec != kF64 && prec != kF32 && n12 % 2 == 0 && rs.sZ % 2 == 0;
  const int tiles = (int)((n12 + (pair ? 127 : 63)) / (pair ? 128 : 64));
  const int64_t total = (int64_t)tiles * S * rs.nrep;
  const int64_t nblk = kP1sXcds * ((total + kP1sXcds - 1) / kP1sXcds);
  if (nblk > INT32_MAX) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nblk);
  switch ((rs.R + 3) / 4 * 4) {
#define SBT_P1S(RPV)                                                                          \
  case RPV:                                                                                   \
    if (prec == kF64)                                                                         \
      timed_launch(p1s_kernel<double, RPV, 1>, grid, dim3(256), 0, s, rs, (const double*)Z,  \
                   Cf, S, (double*)out, so, F, kc0, N, tiles);                                \
    else if (prec == kF32)                                                                    \
      timed_launch(p1s_kernel<float, RPV, 1>, grid, dim3(256), 0, s, rs, (const float*)Z, Cf,\
                   S, (float*)out, so, F, kc0, N, tiles);                                     \
    else if (pair)                                                                            \
      timed_launch(p1s_kernel<uint16_t, RPV, 2>, grid, dim3(256), 0, s, rs,                   \
                   (const uint16_t*)Z, Cf, S, (float*)out, so, F, kc0, N, tiles);             \
    else                                                                                      \
      timed_launch(p1s_kernel<uint16_t, RPV, 1>, grid, dim3(256), 0, s, rs,                   \
                   (const uint16_t*)Z, Cf, S, (float*)out, so, F, kc0, N, tiles);             \
    break;
    SBT_P1S(4) SBT_P1S(8) SBT_P1S(12) SBT_P1S(16) SBT_P1S(20) SBT_P1S(24) SBT_P1S(28)
    SBT_P1S(32)
#undef SBT_P1S
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || S == 1) return e;
  dim3 g2((unsigned)grid_blocks(n12 * rs.R, 1024), (unsigned)rs.nrep);
  if (prec == kF64)
    p1s_sum_kernel<double><<<g2, 256, 0, s>>>(rs, S, (const double*)Wp, sWp, (double*)W);
  else
    p1s_sum_kernel<float><<<g2, 256, 0, s>>>(rs, S, (const float*)Wp, sWp, (float*)W);
  return hipGetLastError();
}

hipError_t launch_krp_nd(const NdFactors& F, int lo, int hi, int R, int rep0, int nrep,
                         double* out, int64_t sOut, hipStream_t s) {
  if (lo < 0 || hi > kMaxOrder || lo >= hi || nrep <= 0) return hipErrorInvalidValue;
  int64_t rows = 1;
  for (int l = lo; l < hi; ++l) rows *= F.n[l];
  if (rows * R > sOut && nrep > 1) return hipErrorInvalidValue;
  dim3 grid((unsigned)grid_blocks(rows * R, 2048), (unsigned)nrep);
  krp_nd_kernel<<<grid, 256, 0, s>>>(F, lo, hi, R, rep0, rows, out, sOut);
  return hipGetLastError();
}

hipError_t launch_hadamard_nd(const double* G, int64_t sMode, int64_t sG, uint32_t mask, int N,
                              int R, int rep0, int nrep, double* out, hipStream_t s) {
  if (nrep <= 0) return hipSuccess;
  hadamard_nd_kernel<<<nrep, 256, 0, s>>>(G, sMode, sG, mask, N, R, rep0, out);
  return hipGetLastError();
}

hipError_t launch_als_init_nd(const NdFactors& F, int N, int R, int rep0, int nrep,
                              uint64_t seed, uint32_t tensor_id, uint32_t stream, uint32_t t,
                              hipStream_t s) {
  if (nrep <= 0) return hipSuccess;
  int64_t total = 0;
  for (int m = 1; m < N; ++m) total += (int64_t)F.n[m] * R;
  dim3 grid((unsigned)grid_blocks(total, 1024), (unsigned)nrep);
  als_init_nd_kernel<<<grid, 256, 0, s>>>(F, N, R, rep0, seed, tensor_id, stream, t);
  return hipGetLastError();
}

hipError_t launch_gather_nd(int prec, const GatherNd& g, hipStream_t s) {
  if (g.nrep <= 0) return hipSuccess;
  int64_t total = 1;
  for (int m = 0; m < g.N; ++m) total *= g.n[m];
  if (total > g.sZ && g.nrep > 1) return hipErrorInvalidValue;
  dim3 grid((unsigned)grid_blocks(total, 8192), (unsigned)g.nrep);
  // (a BF16 summary is gathered from an FP32 store)
  if (prec == kF64)
    timed_launch(gather_nd_kernel<double, double>, grid, dim3(256), 0, s, g);
  else if (prec == kF32)
    timed_launch(gather_nd_kernel<float, float>, grid, dim3(256), 0, s, g);
  else
    timed_launch(gather_nd_kernel<float, uint16_t>, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_cross_nd(const CrossNd& c, hipStream_t s) {
  if (c.njobs <= 0 || c.njobs > kCrossJobs || c.nrep <= 0) return hipErrorInvalidValue;
  cross_nd_kernel<<<dim3((unsigned)c.njobs, (unsigned)c.nrep), 256, 0, s>>>(c);
  return hipGetLastError();
}

hipError_t launch_match_nd(const MatchNd& m, hipStream_t s) {
  if (m.N < 2 || m.N > kMaxOrder || m.R < 1 || m.R > kMaxRank) return hipErrorInvalidValue;
  match_nd_kernel<<<m.nrep, 256, 0, s>>>(m);
  return hipGetLastError();
}

hipError_t launch_match_rows_nd(const NdFactors& Up, const NdFactors& Ut, int N, int R,
                                int rep0, int nrep, const double* scl, const int32_t* pi,
                                hipStream_t s) {
  if (nrep <= 0) return hipSuccess;
  int64_t total = 0;
  for (int m = 0; m < N - 1; ++m) total += (int64_t)Up.n[m] * R;
  dim3 grid((unsigned)grid_blocks(total, 1024), (unsigned)nrep);
  match_rows_nd_kernel<<<grid, 256, 0, s>>>(Up, Ut, N, R, rep0, scl, pi);
  return hipGetLastError();
}

hipError_t launch_commit_nd(const CommitNd& c, hipStream_t s) {
  int64_t total = c.Knew * c.R + c.Knew;
  for (int m = 0; m < c.N; ++m) total += c.D[m] * c.R + (m < c.N - 1 ? c.D[m] : 0);
  commit_nd_kernel<<<grid_blocks(total, 4096), 256, 0, s>>>(c);
  return hipGetLastError();
}

hipError_t launch_sort_nd(const NdFactors& F, int N, int R, double* lam, hipStream_t s) {
  sort_nd_kernel<<<1, 256, 0, s>>>(F, N, R, lam);
  return hipGetLastError();
}

}  // namespace sbt
