// Summary gather and CP-ALS on the r summaries of one update (Sec. 3.1
// "Decompose"; Algorithm 1), all repetitions in one launch per step.
//
// One ALS sweep on a summary Z (n1 x n2 x n3, column-major, i.e. Z viewed as
// the n1*n2 x n3 matrix Z_(3)^T) takes two streaming passes over Z:
//   pass 1  W(ab, f) = sum_c Z(ab, c) C'(c, f)      (contraction with C')
//           M1(a, f) = sum_b W(a,b,f) B'(b,f)        -> A' update
//           M2(b, f) = sum_a W(a,b,f) A'(a,f)        -> B' update (new A')
//   pass 2  M3(c, f) = sum_ab Z(a,b,c) A'(a,f) B'(b,f) -> C' update
// Modes 1 and 2 share W because C' does not change between them.  Each
// update solves U = M (G1 .* G2)^-1 with an FP64 Cholesky of the R x R
// Hadamard product of the other two Gram matrices (pseudo-inverse if a pivot
// is not positive), then normalises the columns (lambda' = their norms) and
// forms the new Gram matrix.
#include "device_common.hpp"
#include "kernels.hpp"
#include "solve_device.hpp"

namespace sbt {

namespace {

// Element loads in accumulation precision.
__device__ inline double ldz(const double* p) { return *p; }
__device__ inline float ldz(const float* p) { return *p; }
__device__ inline float ldz(const uint16_t* p) { return bf16_to_f32(*p); }

template <typename T> struct AccOf { using type = float; };
template <> struct AccOf<double> { using type = double; };

__device__ inline double cvt_out(double x, double*) { return x; }
__device__ inline float cvt_out(double x, float*) { return (float)x; }
__device__ inline float cvt_out(float x, float*) { return x; }
__device__ inline uint16_t cvt_out(float x, uint16_t*) { return f32_to_bf16_rne(x); }
__device__ inline uint16_t cvt_out(double x, uint16_t*) { return f32_to_bf16_rne((float)x); }

inline int rp_of(int R) { return ((R + 3) / 4) * 4; }

#define SBT_DISPATCH_RP(Rv, ...)                 \
  switch (rp_of(Rv)) {                           \
    case 4: { constexpr int RP = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int RP = 8; __VA_ARGS__; } break;   \
    case 12: { constexpr int RP = 12; __VA_ARGS__; } break; \
    case 16: { constexpr int RP = 16; __VA_ARGS__; } break; \
    case 20: { constexpr int RP = 20; __VA_ARGS__; } break; \
    case 24: { constexpr int RP = 24; __VA_ARGS__; } break; \
    case 28: { constexpr int RP = 28; __VA_ARGS__; } break; \
    default: { constexpr int RP = 32; __VA_ARGS__; } break; \
  }

// ---------------------------------------------------------------------------
// Gather
// ---------------------------------------------------------------------------
template <typename TIn, typename TOut>
__global__ __launch_bounds__(256) void gather_dense_kernel(const TIn* X, int64_t I, int64_t J,
                                                          const int32_t* idx, int64_t idx_stride,
                                                          int64_t offJ, int64_t offK, int n3old,
                                                          int64_t Kold, int c0, RepSet rs,
                                                          TOut* Z) {
  const int rep = rs.rep0 + blockIdx.z;
  const int c = c0 + (int)blockIdx.y;
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n12) return;
  const int a = (int)(e % rs.n1), b = (int)(e / rs.n1);
  const int32_t* Is = idx + rep * idx_stride;
  const int64_t kk = c < n3old ? (int64_t)Is[offK + c] : Kold + (c - n3old);
  const int64_t src = (int64_t)Is[a] + I * ((int64_t)Is[offJ + b] + J * kk);
  Z[rep * rs.sZ + e + zslice(rs) * c] = cvt_out(X[src], (TOut*)nullptr);
}

// ---------------------------------------------------------------------------
// Random initial factors B', C' ~ U[0,1)
// ---------------------------------------------------------------------------
__global__ void als_init_kernel(RepSet rs, uint64_t seed, uint32_t tensor_id, uint32_t stream,
                                uint32_t t, uint32_t col0, double* Bp, double* Cp) {
  const int rep = rs.rep0 + blockIdx.y;
  const RngKey key = rng_key(seed, tensor_id);
  const int64_t nb = (int64_t)rs.n2 * rs.R, nc = (int64_t)rs.n3 * rs.R;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nb + nc;
       q += (int64_t)gridDim.x * blockDim.x) {
    const bool isB = q < nb;
    const int64_t qq = isB ? q : q - nb;
    const uint32_t row = (uint32_t)(qq / rs.R), col = (uint32_t)(qq % rs.R);
    const uint32_t tag = rng_tag(stream, isB ? 2u : 3u, (uint32_t)rep);
    const double u = uniform_closed0(rng_bits(key, row, col0 + col, tag, t));
    if (isB)
      Bp[rep * rs.sB + qq] = u;
    else
      Cp[rep * rs.sC + qq] = u;
  }
}

// Warm start from kept summary factors: B' = Bw, C' rows below n3keep = Cw,
// the other C' rows U[0,1) from the same counters as als_init_kernel.
__global__ void als_warm_kernel(RepSet rs, uint64_t seed, uint32_t tensor_id, uint32_t stream,
                                uint32_t t, const double* Bw, const double* Cw, int n3keep,
                                double* Bp, double* Cp) {
  const int rep = rs.rep0 + blockIdx.y;
  const RngKey key = rng_key(seed, tensor_id);
  const int64_t nb = (int64_t)rs.n2 * rs.R, nc = (int64_t)rs.n3 * rs.R;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nb + nc;
       q += (int64_t)gridDim.x * blockDim.x) {
    if (q < nb) {
      Bp[rep * rs.sB + q] = Bw[rep * rs.sB + q];
      continue;
    }
    const int64_t qq = q - nb;
    const uint32_t row = (uint32_t)(qq / rs.R), col = (uint32_t)(qq % rs.R);
    if ((int)row < n3keep) {
      Cp[rep * rs.sC + qq] = Cw[rep * rs.sC + qq];
    } else {
      const uint32_t tag = rng_tag(stream, 3u, (uint32_t)rep);
      Cp[rep * rs.sC + qq] = uniform_closed0(rng_bits(key, row, col, tag, t));
    }
  }
}

// ---------------------------------------------------------------------------
// Gram matrix G = U^T U of a rows x R factor (one block per repetition).
// Thread -> (pair f <= g, row slice); slices combined in LDS.
// ---------------------------------------------------------------------------
__device__ inline void pair_fg(int p, int R, int& f, int& g) {
  f = 0;
  while (p >= R - f) {
    p -= R - f;
    ++f;
  }
  g = f + p;
}

__device__ void block_gram(const double* U, int rows, int R, double* G, double* red) {
  const int P = R * (R + 1) / 2;
  const int tid = threadIdx.x;
  if (P >= 256) {
    for (int p = tid; p < P; p += 256) {
      int f, g;
      pair_fg(p, R, f, g);
      double acc = 0.0;
      for (int i = 0; i < rows; ++i) acc += U[(int64_t)i * R + f] * U[(int64_t)i * R + g];
      G[f * R + g] = acc;
      G[g * R + f] = acc;
    }
    return;
  }
  const int nsl = 256 / P;
  const int pl = tid % P, sl = tid / P;
  double acc = 0.0;
  if (sl < nsl) {
    int f, g;
    pair_fg(pl, R, f, g);
    for (int i = sl; i < rows; i += nsl) acc += U[(int64_t)i * R + f] * U[(int64_t)i * R + g];
  }
  red[tid] = acc;
  __syncthreads();
  if (tid < P) {
    double s = 0.0;
    for (int q = 0; q < nsl; ++q) s += red[q * P + tid];
    int f, g;
    pair_fg(tid, R, f, g);
    G[f * R + g] = s;
    G[g * R + f] = s;
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void gram_kernel(RepSet rs, const double* U, int64_t sU,
                                                  int rows, double* G) {
  const int rep = rs.rep0 + blockIdx.x;
  __shared__ double red[256];
  block_gram(U + rep * sU, rows, rs.R, G + rep * rs.sG, red);
}

// ---------------------------------------------------------------------------
// Pass 1: W(ab, f) = sum_c Z(ab, c) C'(c, f).  Thread per ab (coalesced along
// the fastest summary index), C' rows staged in LDS chunk by chunk.
// ---------------------------------------------------------------------------
constexpr int kP1Chunk = 64;

template <typename TZ, int RP>
__global__ __launch_bounds__(256) void p1_kernel(RepSet rs, const TZ* Z, const double* Cf,
                                                typename AccOf<TZ>::type* W) {
  using TA = typename AccOf<TZ>::type;
  const int rep = rs.rep0 + blockIdx.y;
  const int R = rs.R;
  const int64_t n12 = (int64_t)rs.n1 * rs.n2, ldzc = zslice(rs);
  const int n3 = rs.n3;
  Z += rep * rs.sZ;
  Cf += rep * rs.sC;
  W += rep * rs.sW;
  __shared__ TA Cs[kP1Chunk][RP];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  TA acc[RP];
#pragma unroll
  for (int f = 0; f < RP; ++f) acc[f] = 0;
  for (int c0 = 0; c0 < n3; c0 += kP1Chunk) {
    const int cn = n3 - c0 < kP1Chunk ? n3 - c0 : kP1Chunk;
    __syncthreads();
    for (int q = threadIdx.x; q < kP1Chunk * RP; q += 256) {
      const int cc = q / RP, f = q % RP;
      Cs[cc][f] = (cc < cn && f < R) ? (TA)Cf[(int64_t)(c0 + cc) * R + f] : (TA)0;
    }
    __syncthreads();
    if (e < n12) {
      const TZ* zp = Z + e + ldzc * c0;
#pragma unroll 4
      for (int cc = 0; cc < cn; ++cc) {
        const TA z = ldz(zp + ldzc * cc);
#pragma unroll
        for (int f = 0; f < RP; ++f) acc[f] += z * Cs[cc][f];
      }
    }
  }
  if (e < n12) {
#pragma unroll
    for (int f = 0; f < RP; ++f)
      if (f < R) W[f * n12 + e] = acc[f];
  }
}

// M1(a, f) = sum_b W(a,b,f) B'(b,f): thread per (a, f).
template <typename TA>
__global__ __launch_bounds__(256) void cw1_kernel(RepSet rs, const TA* W, const double* Bf,
                                                 double* M) {
  const int rep = rs.rep0 + blockIdx.z;
  const int f = blockIdx.y;
  const int a = blockIdx.x * 256 + threadIdx.x;
  const int R = rs.R, n1 = rs.n1, n2 = rs.n2;
  if (a >= n1) return;
  const int64_t n12 = (int64_t)n1 * n2;
  W += rep * rs.sW + f * n12;
  Bf += rep * rs.sB;
  TA acc = 0;
  for (int b = 0; b < n2; ++b) acc += W[a + (int64_t)n1 * b] * (TA)Bf[(int64_t)b * R + f];
  M[rep * rs.sM + (int64_t)a * R + f] = (double)acc;
}

// M2(b, f) = sum_a W(a,b,f) A'(a,f): one wavefront per (b, f).
template <typename TA>
__global__ __launch_bounds__(256) void cw2_kernel(RepSet rs, const TA* W, const double* Af,
                                                 double* M) {
  const int rep = rs.rep0 + blockIdx.y;
  const int R = rs.R, n1 = rs.n1, n2 = rs.n2;
  const int64_t wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wv >= (int64_t)n2 * R) return;
  const int b = (int)(wv / R), f = (int)(wv % R);
  const int64_t n12 = (int64_t)n1 * n2;
  const TA* w = W + rep * rs.sW + f * n12 + (int64_t)n1 * b;
  const double* A = Af + rep * rs.sA;
  TA acc = 0;
  for (int a = lane_id(); a < n1; a += kWave) acc += w[a] * (TA)A[(int64_t)a * R + f];
  acc = wave_sum(acc);
  if (lane_id() == 0) M[rep * rs.sM + (int64_t)b * R + f] = (double)acc;
}

// ---------------------------------------------------------------------------
// Pass 2: M3(c, f) = sum_ab Z(a,b,c) A'(a,f) B'(b,f); one block per (c, rep).
// Thread (a, b-slot): acc_f = sum_b Z(a,b,c) B'(b,f) (coalesced along a,
// B' rows broadcast from LDS), then times A'(a,f), reduced over the block.
// ---------------------------------------------------------------------------
constexpr int kP2BChunk = 64;

template <typename TZ, typename TA, int RP, bool kNorm>
__device__ void p2_body(const TZ* Zc, int n1, int n2, int R, const double* Af, const double* Bf,
                        double* out_row, double* nrm_out, TA* Bs, TA (*red)[kMaxRank + 1]) {
  const int tid = threadIdx.x;
  const int nsub = n1 >= 256 ? 1 : 256 / n1;
  const int span = n1 >= 256 ? 256 : n1;  // a values covered per chunk
  const int sub = tid / span;
  const int al = tid % span;
  const bool act = sub < nsub;
  TA tot[RP];
  TA nacc = 0;
#pragma unroll
  for (int f = 0; f < RP; ++f) tot[f] = 0;
  for (int a0 = 0; a0 < n1; a0 += span) {
    const int a = a0 + al;
    const bool ok = act && a < n1;
    TA acc[RP];
#pragma unroll
    for (int f = 0; f < RP; ++f) acc[f] = 0;
    for (int b0 = 0; b0 < n2; b0 += kP2BChunk) {
      const int bn = n2 - b0 < kP2BChunk ? n2 - b0 : kP2BChunk;
      __syncthreads();
      for (int q = tid; q < kP2BChunk * RP; q += 256) {
        const int bb = q / RP, f = q % RP;
        Bs[bb * RP + f] = (bb < bn && f < R) ? (TA)Bf[(int64_t)(b0 + bb) * R + f] : (TA)0;
      }
      __syncthreads();
      if (ok) {
        const TZ* zp = Zc + a + (int64_t)n1 * b0;
#pragma unroll 2
        for (int bb = sub; bb < bn; bb += nsub) {
          const TA z = ldz(zp + (int64_t)n1 * bb);
          if (kNorm) nacc += z * z;
#pragma unroll
          for (int f = 0; f < RP; ++f) acc[f] += z * Bs[bb * RP + f];
        }
      }
    }
    if (ok) {
#pragma unroll
      for (int f = 0; f < RP; ++f)
        if (f < R) tot[f] += acc[f] * (TA)Af[(int64_t)a * R + f];
    }
  }
  const int wave = tid >> 6;
#pragma unroll
  for (int f = 0; f < RP; ++f) {
    const TA v = wave_sum(tot[f]);
    if (lane_id() == 0) red[wave][f] = v;
  }
  if (kNorm) {
    const TA v = wave_sum(nacc);
    if (lane_id() == 0) red[wave][kMaxRank] = v;
  }
  __syncthreads();
  if (tid < R) out_row[tid] = (double)(red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid]);
  if (kNorm && tid == 0)
    *nrm_out = (double)(red[0][kMaxRank] + red[1][kMaxRank] + red[2][kMaxRank] + red[3][kMaxRank]);
}

struct P2Smem {
  double Bs[kP2BChunk * kMaxRank];
  double red[4][kMaxRank + 1];
};

template <typename TZ, int RP>
__global__ __launch_bounds__(256) void p2_kernel(RepSet rs, const TZ* Z, const double* Af,
                                                const double* Bf, double* M) {
  using TA = typename AccOf<TZ>::type;
  __shared__ P2Smem sm;
  const int rep = rs.rep0 + blockIdx.y;
  const int c = blockIdx.x;
  p2_body<TZ, TA, RP, false>(Z + rep * rs.sZ + zslice(rs) * c, rs.n1, rs.n2, rs.R,
                             Af + rep * rs.sA, Bf + rep * rs.sB,
                             M + rep * rs.sM + (int64_t)c * rs.R, nullptr, (TA*)sm.Bs,
                             (TA(*)[kMaxRank + 1])sm.red);
}

// Full-tensor pass for the fit: FP64 accumulation whatever the storage type.
template <typename TZ, int RP>
__global__ __launch_bounds__(256) void fit_slices_kernel(const TZ* X, int64_t I, int64_t J,
                                                        int R, const double* A, const double* B,
                                                        double* M3, double* nrm) {
  __shared__ P2Smem sm;
  const int64_t k = blockIdx.x;
  p2_body<TZ, double, RP, true>(X + I * J * k, (int)I, (int)J, R, A, B, M3 + k * R, nrm + k,
                                sm.Bs, sm.red);
}

// Stand-alone solve (one block per repetition).
template <int RP>
__global__ __launch_bounds__(256) void solve_kernel(RepSet rs, int rows, SolveArgs sa) {
  __shared__ SolveSmem sm;
  block_solve<RP>(sa, rs.rep0 + blockIdx.x, rows, rs.R, sm);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_gather_dense(int store_prec, int sum_prec, const void* X, int64_t I,
                               int64_t J, const int32_t* idx, int64_t idx_stride,
                               int64_t offJ, int64_t offK, int n3old, int64_t Kold, int c0,
                               const RepSet& rs, void* Z, hipStream_t s) {
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  if (c0 < 0 || c0 >= rs.n3) return hipErrorInvalidValue;
  dim3 grid((unsigned)((n12 + 255) / 256), (unsigned)(rs.n3 - c0), (unsigned)rs.nrep);
  if (store_prec == kF64) {
    timed_launch(gather_dense_kernel<double, double>, grid, dim3(256), 0, s, 
        (const double*)X, I, J, idx, idx_stride, offJ, offK, n3old, Kold, c0, rs, (double*)Z);
  } else if (sum_prec == kF32) {
    timed_launch(gather_dense_kernel<float, float>, grid, dim3(256), 0, s, 
        (const float*)X, I, J, idx, idx_stride, offJ, offK, n3old, Kold, c0, rs, (float*)Z);
  } else {
    timed_launch(gather_dense_kernel<float, uint16_t>, grid, dim3(256), 0, s, 
        (const float*)X, I, J, idx, idx_stride, offJ, offK, n3old, Kold, c0, rs, (uint16_t*)Z);
  }
  return hipGetLastError();
}

hipError_t launch_als_init(const RepSet& rs, uint64_t seed, uint32_t tensor_id, uint32_t stream,
                           uint32_t t, double* Bp, double* Cp, hipStream_t s, uint32_t col0) {
  const int64_t n = (int64_t)(rs.n2 + rs.n3) * rs.R;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  als_init_kernel<<<dim3((unsigned)blocks, (unsigned)rs.nrep), 256, 0, s>>>(rs, seed, tensor_id,
                                                                          stream, t, col0, Bp,
                                                                          Cp);
  return hipGetLastError();
}

hipError_t launch_als_warm(const RepSet& rs, uint64_t seed, uint32_t tensor_id, uint32_t stream,
                           uint32_t t, const double* Bw, const double* Cw, int n3keep,
                           double* Bp, double* Cp, hipStream_t s) {
  const int64_t n = (int64_t)(rs.n2 + rs.n3) * rs.R;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  als_warm_kernel<<<dim3((unsigned)blocks, (unsigned)rs.nrep), 256, 0, s>>>(
      rs, seed, tensor_id, stream, t, Bw, Cw, n3keep, Bp, Cp);
  return hipGetLastError();
}

hipError_t launch_gram(const RepSet& rs, const double* U, int64_t sU, int rows, double* G,
                       hipStream_t s) {
  gram_kernel<<<rs.nrep, 256, 0, s>>>(rs, U, sU, rows, G);
  return hipGetLastError();
}

hipError_t launch_p1(int prec, const RepSet& rs, const void* Z, const double* Cf, void* W,
                     hipStream_t s) {
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  dim3 grid((unsigned)((n12 + 255) / 256), (unsigned)rs.nrep);
  SBT_DISPATCH_RP(rs.R, {
    if (prec == kF64)
      timed_launch(p1_kernel<double, RP>, grid, dim3(256), 0, s, rs, (const double*)Z, Cf,
                   (double*)W);
    else if (prec == kF32)
      timed_launch(p1_kernel<float, RP>, grid, dim3(256), 0, s, rs, (const float*)Z, Cf,
                   (float*)W);
    else
      timed_launch(p1_kernel<uint16_t, RP>, grid, dim3(256), 0, s, rs, (const uint16_t*)Z, Cf,
                   (float*)W);
  });
  return hipGetLastError();
}

hipError_t launch_cw1(int prec, const RepSet& rs, const void* W, const double* Bf, double* M,
                      hipStream_t s) {
  dim3 grid((unsigned)((rs.n1 + 255) / 256), (unsigned)rs.R, (unsigned)rs.nrep);
  if (prec == kF64)
    cw1_kernel<double><<<grid, 256, 0, s>>>(rs, (const double*)W, Bf, M);
  else
    cw1_kernel<float><<<grid, 256, 0, s>>>(rs, (const float*)W, Bf, M);
  return hipGetLastError();
}

hipError_t launch_cw2(int prec, const RepSet& rs, const void* W, const double* Af, double* M,
                      hipStream_t s) {
  const int64_t waves = (int64_t)rs.n2 * rs.R;
  dim3 grid((unsigned)((waves + 3) / 4), (unsigned)rs.nrep);
  if (prec == kF64)
    cw2_kernel<double><<<grid, 256, 0, s>>>(rs, (const double*)W, Af, M);
  else
    cw2_kernel<float><<<grid, 256, 0, s>>>(rs, (const float*)W, Af, M);
  return hipGetLastError();
}

hipError_t launch_p2(int prec, const RepSet& rs, const void* Z, const double* Af,
                     const double* Bf, double* M, hipStream_t s) {
  dim3 grid((unsigned)rs.n3, (unsigned)rs.nrep);
  SBT_DISPATCH_RP(rs.R, {
    if (prec == kF64)
      timed_launch(p2_kernel<double, RP>, grid, dim3(256), 0, s, rs, (const double*)Z, Af, Bf, M);
    else if (prec == kF32)
      timed_launch(p2_kernel<float, RP>, grid, dim3(256), 0, s, rs, (const float*)Z, Af, Bf, M);
    else
      timed_launch(p2_kernel<uint16_t, RP>, grid, dim3(256), 0, s, rs, (const uint16_t*)Z, Af,
                   Bf, M);
  });
  return hipGetLastError();
}

static SolveArgs make_solve_args(const RepSet& rs, const double* M, const double* G1,
                                 int64_t sG1, const double* G2, int64_t sG2, double* U,
                                 int64_t sU, double* Gout, double* lam_out,
                                 const double* lam_div, int normalize, uint32_t* pinv_count) {
  SolveArgs a;
  a.M = M;
  a.sM = rs.sM;
  a.G1 = G1;
  a.sG1 = sG1;
  a.G2 = G2;
  a.sG2 = sG2;
  a.U = U;
  a.sU = sU;
  a.Gout = Gout;
  a.sGout = rs.sG;
  a.lam_out = lam_out;
  a.lam_div = lam_div;
  a.normalize = normalize;
  a.pinv_count = pinv_count;
  a.gmask = 0;
  a.Gm = nullptr;
  a.sGmode = 0;
  return a;
}

hipError_t launch_solve(const RepSet& rs, int rows, const double* M, const double* G1,
                        int64_t sG1, const double* G2, int64_t sG2, double* U, int64_t sU,
                        double* Gout, double* lam_out, const double* lam_div, int normalize,
                        uint32_t* pinv_count, hipStream_t s) {
  const SolveArgs a = make_solve_args(rs, M, G1, sG1, G2, sG2, U, sU, Gout, lam_out, lam_div,
                                      normalize, pinv_count);
  SBT_DISPATCH_RP(rs.R, { solve_kernel<RP><<<rs.nrep, 256, 0, s>>>(rs, rows, a); });
  return hipGetLastError();
}

hipError_t launch_solve_prod(const RepSet& rs, int rows, const double* M, const double* Gm,
                             int64_t sGmode, uint32_t mask, double* U, int64_t sU, double* Gout,
                             double* lam_out, uint32_t* pinv_count, hipStream_t s) {
  if (mask == 0 || (mask >> kMaxOrder) != 0) return hipErrorInvalidValue;
  SolveArgs a = make_solve_args(rs, M, nullptr, rs.sG, nullptr, 0, U, sU, Gout, lam_out, nullptr,
                                1, pinv_count);
  a.gmask = mask;
  a.Gm = Gm;
  a.sGmode = sGmode;
  SBT_DISPATCH_RP(rs.R, { solve_kernel<RP><<<rs.nrep, 256, 0, s>>>(rs, rows, a); });
  return hipGetLastError();
}

hipError_t launch_fit_slices(int prec, const void* X, int64_t I, int64_t J, int64_t K, int R,
                             const double* A, const double* B, double* M3, double* nrm,
                             hipStream_t s) {
  if (K <= 0) return hipSuccess;
  SBT_DISPATCH_RP(R, {
    if (prec == kF64)
      fit_slices_kernel<double, RP><<<(unsigned)K, 256, 0, s>>>((const double*)X, I, J, R, A,
                                                                 B, M3, nrm);
    else
      fit_slices_kernel<float, RP><<<(unsigned)K, 256, 0, s>>>((const float*)X, I, J, R, A, B,
                                                                M3, nrm);
  });
  return hipGetLastError();
}

}  // namespace sbt
