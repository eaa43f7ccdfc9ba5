// Batched CP-ALS on the r summaries of one update (Sec. 3.1 "Decompose"),
// organised for latency: three streaming kernels per sweep, each of which
// produces complete rows of the updated factor.
//
//   pass W   W(ab, f) = sum_c Z(ab, c) C~(c, f)                (modes 1 and 2 share)
//   mode 1   A(a, :)  = [sum_b W(a, b, :) * B~(b, :)] V1^-1     rows of A per block
//   mode 2   B(b, :)  = [sum_a W(a, b, :) * A~(a, :)] V2^-1     rows of B per block
//   mode 3   C(c, :)  = [sum_ab Z(a,b,c) A~(a,:) * B~(b,:)] V3^-1   two slices per block
//
// V_n^-1 = (Hadamard product of the other two Gram matrices)^-1 is computed
// ahead of time, by the tail of the previous step, so the streaming blocks
// multiply their rows by it directly.  Factors are stored unnormalised with
// 1/lambda per column beside them; every consumer scales the rows it stages
// (X~ = X diag(1/lambda)), which is the column normalisation of ALS without a
// separate pass.  The tail of each step (one small block per repetition, its
// own launch) forms the Gram matrix of the new factor, its column norms
// lambda, the normalised Gram matrix and the inverse needed by the next step.
// The tail is a separate launch rather than the last block of the streaming
// kernel: on this multi-XCD GPU a device-scope fence writes back and
// invalidates the L2 of the issuing XCD, which costs far more per block than
// one extra launch.  All reductions use a fixed assignment and order.
#include "device_common.hpp"
#include "kernels.hpp"
#include "solve_device.hpp"

namespace sbt {

namespace {

template <typename T> struct AccT { using type = float; };
template <> struct AccT<double> { using type = double; };

__device__ inline double ld1(const double* p) { return *p; }
__device__ inline float ld1(const float* p) { return *p; }
__device__ inline float ld1(const uint16_t* p) { return bf16_to_f32(*p); }

__device__ inline void ldv(const float* p, float (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ inline void ldv(const float* p, float (&o)[2]) {
  const float2 v = *reinterpret_cast<const float2*>(p);
  o[0] = v.x; o[1] = v.y;
}
__device__ inline void ldv(const float* p, float (&o)[1]) { o[0] = *p; }
__device__ inline void ldv(const double* p, double (&o)[2]) {
  const double2 v = *reinterpret_cast<const double2*>(p);
  o[0] = v.x; o[1] = v.y;
}
__device__ inline void ldv(const double* p, double (&o)[1]) { o[0] = *p; }
__device__ inline void ldv(const uint16_t* p, float (&o)[4]) {
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  o[0] = bf16_to_f32((uint16_t)(v.x & 0xFFFFu)); o[1] = bf16_to_f32((uint16_t)(v.x >> 16));
  o[2] = bf16_to_f32((uint16_t)(v.y & 0xFFFFu)); o[3] = bf16_to_f32((uint16_t)(v.y >> 16));
}
__device__ inline void ldv(const uint16_t* p, float (&o)[2]) {
  const uint32_t v = *reinterpret_cast<const uint32_t*>(p);
  o[0] = bf16_to_f32((uint16_t)(v & 0xFFFFu)); o[1] = bf16_to_f32((uint16_t)(v >> 16));
}
__device__ inline void ldv(const uint16_t* p, float (&o)[1]) { o[0] = bf16_to_f32(*p); }

constexpr int ku_of(int V) { return 32 / V; }  // summary elements in flight per thread
constexpr int kTailParts = 16;                 // partial Gram loads in flight per thread
constexpr int kTailBuf = 2304;                  // doubles; >= 2 x 32 x 33 (Jacobi scratch)
constexpr int kLd = kMaxRank + 1;

// Stage rows [0, rows) of a row-major FP64 factor (R columns) into LDS as
// dst[row * RP + f], columns f >= R zero, each column scaled by sc[f] when sc
// is given; blockDim.x == 256.  A thread issues all loads of a batch before
// its first store, so their latencies overlap.
template <typename TA, int RP>
__device__ inline void stage_rows(TA* dst, int rows, const double* src, int R,
                                  const double* sc) {
  constexpr int U = 8;
  const int n = rows * RP;
  for (int q0 = threadIdx.x; q0 < n; q0 += U * 256) {
    double v[U], m[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + u * 256;
      const int r = q / RP, f = q % RP;
      const bool in = q < n && f < R;
      v[u] = in ? src[(int64_t)r * R + f] : 0.0;
      m[u] = (in && sc) ? sc[f] : 1.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + u * 256;
      if (q < n) dst[q] = (TA)(v[u] * m[u]);
    }
  }
}

struct TailSmem {
  double V[kMaxRank][kLd];           // Gram of the new factor, then V_next, then V_next^-1
  double Vin[kMaxRank * kMaxRank];   // V_next as given (input of the fallback)
  double Gold[kMaxRank * kMaxRank];  // the other Gram matrix of V_next
  double buf[kTailBuf];              // factor rows, or Jacobi scratch
  double red[256];
  double lam[kMaxRank];
  int fail;
};

// Step outputs of one mode update (per repetition strides in elements).
struct TailArgs {
  const double* Gin;    // raw Gram of U given (stride sG), or null: computed here
  const double* Gparts; // or the partial Gram matrices of U's row blocks, summed here in
  int64_t sGparts;      // block order ([rep][part][R x R], stride sGparts per repetition)
  int nparts;
  double* U;            // raw rows of the new factor
  int64_t sU;
  int rows;
  double* Gout;         // normalised Gram of the new factor (R*R)
  double* invlam_out;   // 1/lambda (1 where lambda == 0)
  double* lam_out;      // lambda (may be null)
  const double* Gx;     // next step: V_next = Gx .* Gy (normalised Gram matrices)
  const double* Gy;
  double* Vinv_out;     // V_next^-1 (R*R)
  int64_t sG;           // R*R
  uint32_t* pinv_count;
};

__device__ inline void pair_of(int p, int R, int& f, int& g) {
  f = 0;
  while (p >= R - f) {
    p -= R - f;
    ++f;
  }
  g = f + p;
}

// Cyclic Jacobi on the symmetric A (destroyed) -> pseudo-inverse P with
// cut-off R eps max|eig|.  One thread.
__device__ void jacobi_pinv(double* A, double* Q, double* P, int R) {
  for (int i = 0; i < R; ++i)
    for (int j = 0; j < R; ++j) Q[i * kLd + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < R; ++i) {
      dia += A[i * kLd + i] * A[i * kLd + i];
      for (int j = i + 1; j < R; ++j) off += A[i * kLd + j] * A[i * kLd + j];
    }
    if (off <= 1e-32 * dia || off == 0.0) break;
    for (int p = 0; p < R; ++p)
      for (int q = p + 1; q < R; ++q) {
        const double apq = A[p * kLd + q];
        if (apq == 0.0) continue;
        const double theta = (A[q * kLd + q] - A[p * kLd + p]) / (2.0 * apq);
        const double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
        for (int k = 0; k < R; ++k) {
          const double akp = A[k * kLd + p], akq = A[k * kLd + q];
          A[k * kLd + p] = c * akp - s * akq;
          A[k * kLd + q] = s * akp + c * akq;
        }
        for (int k = 0; k < R; ++k) {
          const double apk = A[p * kLd + k], aqk = A[q * kLd + k];
          A[p * kLd + k] = c * apk - s * aqk;
          A[q * kLd + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < R; ++k) {
          const double qkp = Q[k * kLd + p], qkq = Q[k * kLd + q];
          Q[k * kLd + p] = c * qkp - s * qkq;
          Q[k * kLd + q] = s * qkp + c * qkq;
        }
      }
  }
  double emax = 0.0;
  for (int i = 0; i < R; ++i) emax = fmax(emax, fabs(A[i * kLd + i]));
  const double cut = (double)R * 2.220446049250313e-16 * emax;
  for (int i = 0; i < R; ++i)
    for (int j = 0; j < R; ++j) {
      double s = 0.0;
      for (int k = 0; k < R; ++k)
        if (fabs(A[k * kLd + k]) > cut) s += Q[i * kLd + k] * Q[j * kLd + k] / A[k * kLd + k];
      P[i * kLd + j] = s;
    }
}

// The tail runs one 256-thread block per repetition.  Its cost is latency:
// the rows it reads were just written by another kernel, so all loads are
// issued before any is used; the Gram matrix is shared out over the threads;
// the R x R inversion runs in the registers of one wavefront (lane i holds
// row i of [V | I]; the pivot row is broadcast with readlane), so it needs no
// barriers.
constexpr int kTailThreads = 256;
constexpr int kTailUnroll = 8;  // row loads in flight per thread

// Gauss-Jordan inverse of s.V in one wavefront (wave_gj_inverse_v).
template <int RP>
__device__ bool wave_gj_inverse(TailSmem& s, int R) {
  return wave_gj_inverse_v<RP>(s.V, R);
}

// s.V (R x R, already in LDS) -> its inverse in s.V; pseudo-inverse fallback.
template <int RP>
__device__ void block_inverse_lds(TailSmem& s, int R, uint32_t* pinv_count, bool count) {
  const int tid = threadIdx.x;
  __syncthreads();
  if (tid < 64) {
    const bool ok = wave_gj_inverse<RP>(s, R);
    if (tid == 0) s.fail = ok ? 0 : 1;
  }
  __syncthreads();
  if (s.fail) {
    double* A0 = s.buf;
    double* Q = s.buf + kMaxRank * kLd;
    for (int q = tid; q < R * R; q += kTailThreads) A0[(q / R) * kLd + q % R] = s.Vin[q];
    __syncthreads();
    if (tid == 0) {
      jacobi_pinv(A0, Q, &s.V[0][0], R);
      if (pinv_count && count) atomicAdd(pinv_count, 1u);
    }
  }
  __syncthreads();
}

// Vout = (Gx .* Gy)^-1 (start of the sweeps, row solve).
template <int RP>
__device__ void block_inverse(const double* Gx, const double* Gy, int R, double* Vout,
                              TailSmem& s, uint32_t* pinv_count) {
  const int tid = threadIdx.x;
  for (int q = tid; q < R * R; q += kTailThreads) {
    const double v = Gx[q] * Gy[q];
    s.V[q / R][q % R] = v;
    s.Vin[q] = v;
  }
  block_inverse_lds<RP>(s, R, pinv_count, true);
  for (int q = tid; q < R * R; q += kTailThreads) Vout[q] = s.V[q / R][q % R];
}

// Tail of a mode update for one repetition: Gram of the new raw factor,
// lambda, normalised Gram, inverse for the next step.  The results stay in
// LDS (s.V = the next V^-1, s.lam); `write` also stores them to memory.
template <int RP>
__device__ void als_tail(const TailArgs& t, int rep, int R, TailSmem& s, bool write = true) {
  const int tid = threadIdx.x;
  const double* U = t.U + rep * t.sU;
  const int rows = t.rows;
  const int P = R * (R + 1) / 2;
  const int S = P >= kTailThreads ? 1 : kTailThreads / P;
  const int crows = kTailBuf / R;
  // the Gram matrix of the step before, the other factor of V_next
  const bool fresh_x = t.Gx == t.Gout;
  const double* Gold = (fresh_x ? t.Gy : t.Gx) + rep * t.sG;
  for (int q = tid; q < R * R; q += kTailThreads) s.Gold[q] = Gold[q];
  double gacc[3][4];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int u = 0; u < 4; ++u) gacc[j][u] = 0.0;
  for (int r0 = 0; r0 < ((t.Gin || t.Gparts) ? 0 : rows); r0 += crows) {
    const int cn = rows - r0 < crows ? rows - r0 : crows;
    const int n = cn * R;
    const double* src = U + (int64_t)r0 * R;
    __syncthreads();
    int q = tid;
    for (; q + (kTailUnroll - 1) * kTailThreads < n; q += kTailUnroll * kTailThreads) {
      double v[kTailUnroll];
#pragma unroll
      for (int u = 0; u < kTailUnroll; ++u) v[u] = src[q + u * kTailThreads];
#pragma unroll
      for (int u = 0; u < kTailUnroll; ++u) s.buf[q + u * kTailThreads] = v[u];
    }
    for (; q < n; q += kTailThreads) s.buf[q] = src[q];
    __syncthreads();
    for (int j = 0; j < 3; ++j) {
      const int p = P <= kTailThreads ? tid % P : tid + kTailThreads * j;
      const int sl = P <= kTailThreads ? tid / P : 0;
      if ((P <= kTailThreads && (j > 0 || sl >= S)) || p >= P) continue;
      int f, g;
      pair_of(p, R, f, g);
      int i = sl;
      for (; i + 3 * S < cn; i += 4 * S) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          gacc[j][u] += s.buf[(i + u * S) * R + f] * s.buf[(i + u * S) * R + g];
      }
      for (; i < cn; i += S) gacc[j][0] += s.buf[i * R + f] * s.buf[i * R + g];
    }
  }
  __syncthreads();
  // combine -> Gram of the raw factor in s.V
  if (t.Gin) {
    for (int q = tid; q < R * R; q += kTailThreads) s.V[q / R][q % R] = t.Gin[rep * t.sG + q];
  } else if (t.Gparts) {
    // kTailParts loads in flight per thread: part b goes to partial sum
    // b mod kTailParts, and the partial sums are added in a fixed tree
    // (the parts are symmetric: the upper triangle is summed and mirrored)
    const double* gp = t.Gparts + rep * t.sGparts;
    const int RR = R * R;
    for (int p = tid; p < P; p += kTailThreads) {
      int f, g;
      pair_of(p, R, f, g);
      const int q = f * R + g;
      double a[kTailParts];
#pragma unroll
      for (int u = 0; u < kTailParts; ++u) a[u] = 0.0;
      int b = 0;
      for (; b + kTailParts <= t.nparts; b += kTailParts) {
        double v[kTailParts];
#pragma unroll
        for (int u = 0; u < kTailParts; ++u) v[u] = gp[(int64_t)(b + u) * RR + q];
#pragma unroll
        for (int u = 0; u < kTailParts; ++u) a[u] += v[u];
      }
      {  // the last parts, branch-free (past the end: part 0, dropped)
        double v[kTailParts];
#pragma unroll
        for (int u = 0; u < kTailParts; ++u)
          v[u] = gp[(int64_t)(b + u < t.nparts ? b + u : 0) * RR + q];
#pragma unroll
        for (int u = 0; u < kTailParts; ++u)
          if (b + u < t.nparts) a[u] += v[u];
      }
#pragma unroll
      for (int w = kTailParts / 2; w > 0; w /= 2)
#pragma unroll
        for (int u = 0; u < w; ++u) a[u] += a[u + w];
      s.V[f][g] = a[0];
      s.V[g][f] = a[0];
    }
  } else if (P <= kTailThreads) {
    s.red[tid] = (gacc[0][0] + gacc[0][1]) + (gacc[0][2] + gacc[0][3]);
    __syncthreads();
    if (tid < P) {
      double acc = 0.0;
      for (int sl = 0; sl < S; ++sl) acc += s.red[sl * P + tid];
      int f, g;
      pair_of(tid, R, f, g);
      s.V[f][g] = acc;
      s.V[g][f] = acc;
    }
  } else {
    for (int j = 0; j < 3; ++j) {
      const int p = tid + kTailThreads * j;
      if (p < P) {
        int f, g;
        pair_of(p, R, f, g);
        const double acc = (gacc[j][0] + gacc[j][1]) + (gacc[j][2] + gacc[j][3]);
        s.V[f][g] = acc;
        s.V[g][f] = acc;
      }
    }
  }
  __syncthreads();
  if (tid < R) {
    const double l = sqrt(s.V[tid][tid]);
    s.lam[tid] = l;
    if (write) {
      t.invlam_out[rep * 3 * R + tid] = l > 0.0 ? 1.0 / l : 1.0;  // [A | B | C] per repetition
      if (t.lam_out) t.lam_out[rep * R + tid] = l;
    }
  }
  __syncthreads();
  double* G = t.Gout + rep * t.sG;
  for (int q = tid; q < R * R; q += kTailThreads) {
    const int f = q / R, g = q % R;
    const double lf = s.lam[f], lg = s.lam[g];
    double v = s.V[f][g];
    if (lf > 0.0) v = v / lf;
    if (lg > 0.0) v = v / lg;
    if (write) G[q] = v;
    // V_next = Gx .* Gy with the fresh Gram in its place
    const double vn = fresh_x ? v * s.Gold[q] : s.Gold[q] * v;
    s.Vin[q] = vn;
  }
  __syncthreads();
  for (int q = tid; q < R * R; q += kTailThreads) s.V[q / R][q % R] = s.Vin[q];
  block_inverse_lds<RP>(s, R, t.pinv_count, write);
  if (!write) return;
  double* Vout = t.Vinv_out + rep * t.sG;
  for (int q = tid; q < R * R; q += kTailThreads) Vout[q] = s.V[q / R][q % R];
}

// ---------------------------------------------------------------------------
// pass W
// ---------------------------------------------------------------------------
// One block = 64 consecutive (a, b) of one repetition; its four wavefronts
// take equal shares of the third-mode index and add their partial rows in a
// fixed order, so W holds complete sums (one partial per row).
template <typename TZ, int RP>
__global__ __launch_bounds__(256) void pw_kernel(RepSet rs, const TZ* Z, const double* Cf,
                                                const double* invlamC,
                                                typename AccT<TZ>::type* W) {
  using TA = typename AccT<TZ>::type;
  constexpr int KU = 16;                              // loads in flight per thread
  constexpr int CH = sizeof(TA) == 8 ? 128 : 256;     // C~ rows staged at once
  __shared__ TA Cs[CH][RP];
  __shared__ TA red[64][RP];
  const int rep = rs.rep0 + blockIdx.y;
  const int R = rs.R;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t n12 = (int64_t)rs.n1 * rs.n2, ldzc = zslice(rs);
  const int n3 = rs.n3;
  Z += rep * rs.sZ;
  Cf += rep * rs.sC;
  const double* il = invlamC + rep * 3 * R;
  const int64_t e = (int64_t)blockIdx.x * 64 + lane;
  const bool ok = e < n12;
  TA acc[RP];
#pragma unroll
  for (int f = 0; f < RP; ++f) acc[f] = 0;
  for (int cc0 = 0; cc0 < n3; cc0 += CH) {
    const int cn = n3 - cc0 < CH ? n3 - cc0 : CH;
    const int lo = (wave * cn) / 4, hi = ((wave + 1) * cn) / 4;
    const TZ* zp = Z + e + ldzc * cc0;
    // the first KU summary loads go out before C~ is staged
    TA z[KU];
    const bool pre = ok && lo + KU <= hi;
    if (pre) {
#pragma unroll
      for (int u = 0; u < KU; ++u) z[u] = ld1(zp + ldzc * (lo + u));
    }
    __syncthreads();
    stage_rows<TA, RP>(&Cs[0][0], cn, Cf + (int64_t)cc0 * R, R, il);
    __syncthreads();
    if (ok) {
      int c = lo;
      if (pre) {
#pragma unroll
        for (int u = 0; u < KU; ++u)
#pragma unroll
          for (int f = 0; f < RP; ++f) acc[f] += z[u] * Cs[c + u][f];
        c += KU;
      }
      for (; c + KU <= hi; c += KU) {
#pragma unroll
        for (int u = 0; u < KU; ++u) z[u] = ld1(zp + ldzc * (c + u));
#pragma unroll
        for (int u = 0; u < KU; ++u)
#pragma unroll
          for (int f = 0; f < RP; ++f) acc[f] += z[u] * Cs[c + u][f];
      }
      for (; c < hi; ++c) {
        const TA zc = ld1(zp + ldzc * c);
#pragma unroll
        for (int f = 0; f < RP; ++f) acc[f] += zc * Cs[c][f];
      }
    }
  }
  for (int w = 1; w < 4; ++w) {
    __syncthreads();
    if (wave == w) {
#pragma unroll
      for (int f = 0; f < RP; ++f) red[lane][f] = acc[f];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int f = 0; f < RP; ++f) acc[f] += red[lane][f];
    }
  }
  if (wave == 0 && ok) {
    TA* w = W + rep * rs.sW + e * R;
#pragma unroll
    for (int f = 0; f < RP; ++f)
      if (f < R) w[f] = acc[f];
  }
}

// ---------------------------------------------------------------------------
// modes 1 and 2 from W
// ---------------------------------------------------------------------------
// W of one repetition is stored [b][a][f] (row e = a + n1 b of R entries), and
// both contractions read all of it:
//   mode 0: rows a of A, M(a, f) = sum_b W(a, b, f) B~(b, f);
//   mode 1: rows b of B, M(b, f) = sum_a W(a, b, f) A~(a, f).
// Every W element is read by a vector load of V consecutive entries (V the
// widest of 16 bytes, 8, one element that divides R), and the threads of a
// block are laid out so that their loads form contiguous runs in memory:
//   mode 0: the block's 8 rows a form one run of 8 R entries per b; G = 8 R / V
//           threads cover the run and 256 / G slots of G threads step through b;
//   mode 1: row b is one run of n1 R entries; 32 threads per row, of which
//           T = (32 / (R / V)) (R / V) step through it by T vectors, so each
//           keeps the same V columns f throughout.
// The partials of a row are added through LDS in a fixed order, the row is
// multiplied by V^-1 (raw rows U = M V^-1 are written; the tail follows).
// The contracted factor is staged in LDS in chunks of chr rows (one chunk when
// it fits); each thread's first W loads of a chunk go out before its staging.
constexpr int kRowsPerBlock = 8;   // factor rows produced by one block

// out(f, g) = sum over the kRowsPerBlock rows r of U(r, f) U(r, g), rows in
// order (rows past the factor's end hold zeros); both triangles are written
// and are equal, since each product is formed the same way either side.
__device__ inline void block_gram_part(const double (*U)[kMaxRank], int R, double* out) {
  for (int q = threadIdx.x; q < R * R; q += blockDim.x) {
    const int f = q / R, g = q % R;
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < kRowsPerBlock; ++r) acc += U[r][f] * U[r][g];
    out[q] = acc;
  }
}
constexpr int kSlots = 32;         // chunk rows are a multiple of this
constexpr int kCwPre = 8;          // W vector loads in flight per thread

template <typename TA, int V>
__device__ inline void ldw(const TA* p, TA (&o)[V]) {
  if constexpr (V == 4) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  } else if constexpr (V == 2 && sizeof(TA) == 4) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    o[0] = v.x; o[1] = v.y;
  } else if constexpr (V == 2) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    o[0] = v.x; o[1] = v.y;
  } else {
    o[0] = *p;
  }
}

template <typename TA, int RP, int V>
__global__ __launch_bounds__(256) void cw_kernel(RepSet rs, int mode, int chr, const TA* W,
                                                const double* F, const double* invlamF,
                                                const double* Vinv, double* Uout, int64_t sU,
                                                TailArgs pro, double* gpart, int64_t sGpart) {
  extern __shared__ __align__(16) unsigned char cw_smem[];
  __shared__ TA red[256 * V];
  __shared__ double Mrow[kRowsPerBlock][kMaxRank];
  __shared__ double Urow[kRowsPerBlock][kMaxRank];
  __shared__ double Vi[kMaxRank][kLd];
  __shared__ double ilp[kMaxRank];
  TA* Fs = reinterpret_cast<TA*>(cw_smem);  // [chr][RP]
  const int rep = rs.rep0 + blockIdx.y;
  const int R = rs.R, n1 = rs.n1, n2 = rs.n2;
  const int tid = threadIdx.x;
  const int gpr = R / V;  // vectors per row of W
  const int nrows = mode == 0 ? n1 : n2;
  const int ncon = mode == 0 ? n2 : n1;  // contracted extent
  // mode 0: G threads per run, S slots;  mode 1: 32 threads per row, T active
  const int G = kRowsPerBlock * gpr, S = 256 / G;
  const int T = (32 / gpr) * gpr;
  int rl, slot, f0, step;
  if (mode == 0) {
    const int grp = tid % G;
    slot = tid / G;
    rl = grp / gpr;
    f0 = (grp % gpr) * V;
    step = S;  // contracted rows b per step of a slot
  } else {
    rl = tid / 32;
    slot = tid % 32;
    f0 = (slot % gpr) * V;
    step = T;  // vectors per step along the row
  }
  const int row = blockIdx.x * kRowsPerBlock + rl;
  const bool act = (mode == 0 ? slot < S : slot < T) && row < nrows;
  const TA* Wr = W + rep * rs.sW;
  // mode 0: vector of contracted row x is at (x n1 + row) R + f0
  // mode 1: vector q of the row is at row n1 R + q V, contracted row q / gpr
  const TA* wbase = mode == 0 ? Wr + (int64_t)row * R + f0 : Wr + (int64_t)row * n1 * R;
  const int64_t wstep = mode == 0 ? (int64_t)n1 * R : (int64_t)V;
  const double* Fr = F + (mode == 0 ? rep * rs.sB : rep * rs.sA);
  const double* il = invlamF + rep * 3 * R;
  TA acc[V];
#pragma unroll
  for (int v = 0; v < V; ++v) acc[v] = 0;
  for (int x0 = 0; x0 < ncon; x0 += chr) {
    const int xn = ncon - x0 < chr ? ncon - x0 : chr;
    // positions of this thread in the chunk: contracted rows (mode 0) or
    // vectors of the row (mode 1), from p0 by step, below pn
    const int p0 = mode == 0 ? x0 + slot : x0 * gpr + slot;
    const int pn = mode == 0 ? x0 + xn : (x0 + xn) * gpr;
    TA w[kCwPre][V];
#pragma unroll
    for (int u = 0; u < kCwPre; ++u) {
      const int p = p0 + u * step;
      if (act && p < pn) ldw<TA, V>(wbase + wstep * p, w[u]);
    }
    __syncthreads();
    if (x0 == 0) {
      if (pro.U) {
        // the tail of the step before (contracted factor's Gram, lambda, this
        // step's V^-1) folded in: every block computes it the same way, block
        // 0 also stores it; the dynamic LDS is free until the staging below
        TailSmem& ts = *reinterpret_cast<TailSmem*>(cw_smem);
        als_tail<RP>(pro, rep, R, ts, blockIdx.x == 0);
        for (int q = tid; q < R * R; q += 256) Vi[q / R][q % R] = ts.V[q / R][q % R];
        if (tid < R) ilp[tid] = ts.lam[tid] > 0.0 ? 1.0 / ts.lam[tid] : 1.0;
        __syncthreads();
      } else {
        for (int q = tid; q < R * R; q += 256) Vi[q / R][q % R] = Vinv[rep * rs.sG + q];
      }
    }
    stage_rows<TA, RP>(Fs, xn, Fr + (int64_t)x0 * R, R, pro.U ? ilp : il);
    __syncthreads();
    if (act) {
      int p = p0;
      for (bool first = true; p < pn; first = false) {
        if (!first) {
#pragma unroll
          for (int u = 0; u < kCwPre; ++u)
            if (p + u * step < pn) ldw<TA, V>(wbase + wstep * (p + u * step), w[u]);
        }
#pragma unroll
        for (int u = 0; u < kCwPre; ++u) {
          const int q = p + u * step;
          if (q < pn) {
            const int x = (mode == 0 ? q : q / gpr) - x0;
            const TA* fs = Fs + x * RP + f0;
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] += w[u][v] * fs[v];
          }
        }
        p += kCwPre * step;
      }
    }
  }
  // partials of the threads, then each output added in a fixed order
#pragma unroll
  for (int v = 0; v < V; ++v) red[tid * V + v] = act ? acc[v] : (TA)0;
  __syncthreads();
  for (int q = tid; q < kRowsPerBlock * R; q += 256) {
    const int r = q / R, f = q % R, fg = f / V, v = f % V;
    TA s = 0;
    if (mode == 0) {
      for (int sl = 0; sl < S; ++sl) s += red[(sl * G + r * gpr + fg) * V + v];
    } else {
      for (int sl = fg; sl < T; sl += gpr) s += red[(r * 32 + sl) * V + v];
    }
    Mrow[r][f] = (double)s;
  }
  __syncthreads();
  double* U = Uout + rep * sU;
  for (int q = tid; q < kRowsPerBlock * R; q += 256) {
    const int r = q / R, f = q % R;
    const int gr = blockIdx.x * kRowsPerBlock + r;
    double u = 0.0;
    if (gr < nrows) {
      for (int k = 0; k < R; ++k) u += Mrow[r][k] * Vi[k][f];
      U[(int64_t)gr * R + f] = u;
    }
    Urow[r][f] = u;
  }
  if (gpart) {
    // the Gram matrix of this block's rows, summed over the blocks by the tail
    __syncthreads();
    block_gram_part(Urow, R, gpart + rep * sGpart + (int64_t)blockIdx.x * R * R);
  }
}

// ---------------------------------------------------------------------------
// mode 3: a team of two wavefronts per slice, two slices per block
// ---------------------------------------------------------------------------
// The rows of A~ and B~ (scaled by 1/lambda) are staged in LDS once per block
// in the accumulation precision; each thread streams V consecutive a of its
// slice for a strided subset of b, contracts b against B~ then a against A~,
// and the team reduces across its lanes before one wavefront multiplies the
// row by V^-1.
constexpr int kP3Team = 128;               // threads per slice
constexpr int kP3Slices = 256 / kP3Team;   // slices per block

template <typename TA>
size_t p3_smem_bytes(int n1, int n2, int RP) {
  return sizeof(double) * kMaxRank * kLd + sizeof(TA) * 4 * kMaxRank +
         sizeof(TA) * (size_t)(n1 + n2) * RP;
}

// kRow = false: ALS update of C' (raw rows).  kRow = true: the row solve
// (rows divided by lam_div).
template <typename TZ, int RP, int V, bool kRow>
__global__ __launch_bounds__(256) void p3_kernel(RepSet rs, const TZ* Z, const double* Af,
                                                const double* invlamA, const double* Bf,
                                                const double* invlamB, const double* Vinv,
                                                const double* lam_div, double* Uout,
                                                int64_t sU) {
  using TA = typename AccT<TZ>::type;
  constexpr int KU = V == 4 ? 4 : (V == 2 ? 8 : 16);  // loads in flight per thread
  extern __shared__ __align__(16) unsigned char p3_smem[];
  double(*Vi)[kLd] = reinterpret_cast<double(*)[kLd]>(p3_smem);
  TA(*red)[kMaxRank] =
      reinterpret_cast<TA(*)[kMaxRank]>(p3_smem + sizeof(double) * kMaxRank * kLd);
  TA* As = reinterpret_cast<TA*>(p3_smem + sizeof(double) * kMaxRank * kLd +
                                 sizeof(TA) * 4 * kMaxRank);
  const int rep = rs.rep0 + blockIdx.y;
  const int R = rs.R, n1 = rs.n1, n2 = rs.n2;
  const int tid = threadIdx.x;
  TA* Bs = As + (size_t)n1 * RP;
  const int team = tid / kP3Team, tt = tid % kP3Team;
  const int wave = tid >> 6;
  const int c = blockIdx.x * kP3Slices + team;
  const int ng = n1 / V;
  const int span = ng >= kP3Team ? kP3Team : ng;
  const int nsub = kP3Team / span;
  const int sub = tt / span, gl = tt % span;
  const bool act = sub < nsub && c < rs.n3;
  const TZ* Zc = Z + rep * rs.sZ + zslice(rs) * (c < rs.n3 ? c : 0);
  // the first KU summary loads go out before A~ and B~ are staged
  TA z[KU][V];
  const bool pre = act && gl < ng && sub + (KU - 1) * nsub < n2;
  if (pre) {
#pragma unroll
    for (int u = 0; u < KU; ++u) ldv(Zc + (int64_t)gl * V + (int64_t)n1 * (sub + u * nsub), z[u]);
  }
  for (int q = tid; q < R * R; q += 256) Vi[q / R][q % R] = Vinv[rep * rs.sG + q];
  stage_rows<TA, RP>(As, n1, Af + rep * rs.sA, R, invlamA ? invlamA + rep * 3 * R : nullptr);
  stage_rows<TA, RP>(Bs, n2, Bf + rep * rs.sB, R, invlamB ? invlamB + rep * 3 * R : nullptr);
  __syncthreads();
  TA tot[RP];
#pragma unroll
  for (int f = 0; f < RP; ++f) tot[f] = 0;
  if (act) {
    for (int g0 = 0; g0 < ng; g0 += span) {
      const int g = g0 + gl;
      if (g < ng) {
        TA acc[V][RP];
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
          for (int f = 0; f < RP; ++f) acc[v][f] = 0;
        const TZ* zp = Zc + (int64_t)g * V;
        int b = sub;
        bool have = g0 == 0 && pre;
        for (; b + (KU - 1) * nsub < n2; b += KU * nsub) {
          if (!have) {
#pragma unroll
            for (int u = 0; u < KU; ++u) ldv(zp + (int64_t)n1 * (b + u * nsub), z[u]);
          }
          have = false;
#pragma unroll
          for (int u = 0; u < KU; ++u) {
            const TA* bp = Bs + (size_t)(b + u * nsub) * RP;
#pragma unroll
            for (int f = 0; f < RP; ++f) {
              const TA bv = bp[f];
#pragma unroll
              for (int v = 0; v < V; ++v) acc[v][f] += z[u][v] * bv;
            }
          }
        }
        for (; b < n2; b += nsub) {
          TA zz[V];
          ldv(zp + (int64_t)n1 * b, zz);
          const TA* bp = Bs + (size_t)b * RP;
#pragma unroll
          for (int f = 0; f < RP; ++f) {
            const TA bv = bp[f];
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v][f] += zz[v] * bv;
          }
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const TA* ap = As + (size_t)(g * V + v) * RP;
#pragma unroll
          for (int f = 0; f < RP; ++f) tot[f] += acc[v][f] * ap[f];
        }
      }
    }
  }
#pragma unroll
  for (int f = 0; f < RP; ++f) {
    const TA v = wave_sum(tot[f]);
    if (lane_id() == 0 && f < kMaxRank) red[wave][f] = v;
  }
  __syncthreads();
  if (c < rs.n3 && tt < R) {
    const int w0 = team * (kP3Team / 64);
    double u = 0.0;
    for (int k = 0; k < R; ++k) u += (double)(red[w0][k] + red[w0 + 1][k]) * Vi[k][tt];
    if (kRow) {
      const double l = lam_div[tt];
      u = l > 0.0 ? u / l : 0.0;
    }
    Uout[rep * sU + (int64_t)c * R + tt] = u;
  }
}

// Tail of a mode update, one block per repetition.
template <int RP>
__global__ __launch_bounds__(kTailThreads) void tail_kernel(RepSet rs, TailArgs ta) {
  __shared__ TailSmem sm;
  als_tail<RP>(ta, rs.rep0 + blockIdx.x, rs.R, sm);
}

// V^-1 = (Gx .* Gy)^-1 per repetition (start of the sweeps, row solve).
template <int RP>
__global__ __launch_bounds__(kTailThreads) void inverse_kernel(RepSet rs, const double* Gx,
                                                              int64_t sGx, const double* Gy,
                                                              int64_t sGy, double* Vinv,
                                                              uint32_t* pinv_count) {
  __shared__ TailSmem sm;
  const int rep = rs.rep0 + blockIdx.x;
  block_inverse<RP>(Gx + rep * sGx, Gy + rep * sGy, rs.R, Vinv + rep * rs.sG, sm, pinv_count);
}

// Scale raw factor rows to unit columns (end of the sweeps).
__global__ void normalize_kernel(RepSet rs, double* Ap, double* Bp, double* Cp,
                                 const double* invlam) {
  const int rep = rs.rep0 + blockIdx.y;
  const int R = rs.R;
  const int64_t na = (int64_t)rs.n1 * R, nb = (int64_t)rs.n2 * R, nc = (int64_t)rs.n3 * R;
  const double* il = invlam + (int64_t)rep * 3 * R;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < na + nb + nc;
       q += (int64_t)gridDim.x * blockDim.x) {
    if (q < na)
      Ap[rep * rs.sA + q] *= il[q % R];
    else if (q < na + nb)
      Bp[rep * rs.sB + (q - na)] *= il[R + (q - na) % R];
    else
      Cp[rep * rs.sC + (q - na - nb)] *= il[2 * R + (q - na - nb) % R];
  }
}

inline int rp4(int R) { return ((R + 3) / 4) * 4; }

#define SBT_RP_SWITCH(Rv, ...)                              \
  switch (rp4(Rv)) {                                        \
    case 4: { constexpr int RP = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int RP = 8; __VA_ARGS__; } break;   \
    case 12: { constexpr int RP = 12; __VA_ARGS__; } break; \
    case 16: { constexpr int RP = 16; __VA_ARGS__; } break; \
    case 20: { constexpr int RP = 20; __VA_ARGS__; } break; \
    case 24: { constexpr int RP = 24; __VA_ARGS__; } break; \
    case 28: { constexpr int RP = 28; __VA_ARGS__; } break; \
    default: { constexpr int RP = 32; __VA_ARGS__; } break; \
  }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_inverse(const RepSet& rs, const double* Gx, int64_t sGx, const double* Gy,
                          int64_t sGy, double* Vinv, uint32_t* pinv_count, hipStream_t s) {
  SBT_RP_SWITCH(rs.R, {
    inverse_kernel<RP><<<rs.nrep, kTailThreads, 0, s>>>(rs, Gx, sGx, Gy, sGy, Vinv, pinv_count);
  });
  return hipGetLastError();
}

hipError_t launch_normalize(const RepSet& rs, double* Ap, double* Bp, double* Cp,
                            const double* invlam, hipStream_t s) {
  const int64_t n = (int64_t)(rs.n1 + rs.n2 + rs.n3) * rs.R;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 256) blocks = 256;
  normalize_kernel<<<dim3((unsigned)blocks, (unsigned)rs.nrep), 256, 0, s>>>(rs, Ap, Bp, Cp,
                                                                           invlam);
  return hipGetLastError();
}

bool tail_rows_fit(int rows, int R) { return (int64_t)rows * R <= kTailBuf; }

hipError_t launch_tail(const RepSet& rs, const AlsTail& t, hipStream_t s) {
  return launch_tail_parts(rs, t, nullptr, 0, 0, s);
}

int gram_parts(int rows) { return (rows + kRowsPerBlock - 1) / kRowsPerBlock; }

hipError_t launch_tail_parts(const RepSet& rs, const AlsTail& t, const double* parts,
                             int64_t sParts, int nparts, hipStream_t s) {
  if (parts && (t.Gin || nparts < 1)) return hipErrorInvalidValue;
  TailArgs ta{t.Gin, parts, sParts, nparts, t.U, t.sU, t.rows, t.Gout, t.invlam_out,
              t.lam_out, t.Gx, t.Gy, t.Vinv_out, t.sG, t.pinv_count};
  SBT_RP_SWITCH(rs.R, { tail_kernel<RP><<<rs.nrep, kTailThreads, 0, s>>>(rs, ta); });
  return hipGetLastError();
}

hipError_t launch_pw(int prec, const RepSet& rs, const void* Z, const double* Cf,
                     const double* invlamC, void* W, hipStream_t s) {
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  dim3 grid((unsigned)((n12 + 63) / 64), (unsigned)rs.nrep);
  SBT_RP_SWITCH(rs.R, {
    if (prec == kF64)
      timed_launch(pw_kernel<double, RP>, grid, dim3(256), 0, s, rs, (const double*)Z, Cf,
                   invlamC, (double*)W);
    else if (prec == kF32)
      timed_launch(pw_kernel<float, RP>, grid, dim3(256), 0, s, rs, (const float*)Z, Cf, invlamC,
                   (float*)W);
    else
      timed_launch(pw_kernel<uint16_t, RP>, grid, dim3(256), 0, s, rs, (const uint16_t*)Z, Cf,
                   invlamC, (float*)W);
  });
  return hipGetLastError();
}

hipError_t launch_cw(int prec, const RepSet& rs, int mode, const void* W, const double* F,
                     const double* invlamF, const double* Vinv, double* U, int64_t sU,
                     hipStream_t s, const AlsTail* before, double* gpart, int64_t sGpart) {
  TailArgs pro{};
  if (before) {
    if (before->Gin || !tail_rows_fit(before->rows, rs.R)) return hipErrorInvalidValue;
    pro = TailArgs{nullptr, nullptr, 0, 0, before->U, before->sU, before->rows,
                   before->Gout, before->invlam_out, before->lam_out, before->Gx,
                   before->Gy, before->Vinv_out, before->sG, before->pinv_count};
  }
  const int nrows = mode == 0 ? rs.n1 : rs.n2;
  const int ncon = mode == 0 ? rs.n2 : rs.n1;
  dim3 grid((unsigned)((nrows + kRowsPerBlock - 1) / kRowsPerBlock), (unsigned)rs.nrep);
  // staged rows per chunk: all of them when they fit 32 KB
  const size_t row_bytes = (size_t)rp4(rs.R) * (prec == kF64 ? 8 : 4);
  int chr = (int)((32768 / row_bytes) / kSlots * kSlots);
  if (chr > ncon) chr = ncon;
  if (chr < kSlots) chr = kSlots;
  size_t sh = (size_t)chr * row_bytes;
  if (before && sh < sizeof(TailSmem)) sh = sizeof(TailSmem);
  // widest vector of W entries that divides R (16 bytes at most)
  const int vw = prec == kF64 ? (rs.R % 2 == 0 ? 2 : 1)
                              : (rs.R % 4 == 0 ? 4 : (rs.R % 2 == 0 ? 2 : 1));
#define SBT_CW(TA_, RPV, VV)                                                                    \
  cw_kernel<TA_, RPV, VV><<<grid, 256, sh, s>>>(rs, mode, chr, (const TA_*)W, F, invlamF, Vinv, \
                                                U, sU, pro, gpart, sGpart)
  SBT_RP_SWITCH(rs.R, {
    if (prec == kF64) {
      if (vw == 2) SBT_CW(double, RP, 2); else SBT_CW(double, RP, 1);
    } else {
      if (vw == 4) SBT_CW(float, RP, 4);
      else if (vw == 2) SBT_CW(float, RP, 2);
      else SBT_CW(float, RP, 1);
    }
  });
#undef SBT_CW
  return hipGetLastError();
}

bool p3_fits(int prec, int n1, int n2, int R) {
  const int RP = rp4(R);
  const size_t sh = prec == kF64 ? p3_smem_bytes<double>(n1, n2, RP)
                                 : p3_smem_bytes<float>(n1, n2, RP);
  return sh <= 160 * 1024;
}

hipError_t launch_p3(int prec, const RepSet& rs, bool row_solve, const void* Z, const double* Af,
                     const double* invlamA, const double* Bf, const double* invlamB,
                     const double* Vinv, const double* lam_div, double* U, int64_t sU,
                     hipStream_t s) {
  dim3 grid((unsigned)((rs.n3 + kP3Slices - 1) / kP3Slices), (unsigned)rs.nrep);
  const int vw = prec == kF64 ? (rs.n1 % 2 == 0 ? 2 : 1)
                              : (rs.n1 % 4 == 0 ? 4 : (rs.n1 % 2 == 0 ? 2 : 1));
  hipError_t err = hipSuccess;
#define SBT_P3(TZ, RPV, VV)                                                                    \
  do {                                                                                         \
    using TA_ = typename AccT<TZ>::type;                                                       \
    const size_t sh = p3_smem_bytes<TA_>(rs.n1, rs.n2, RPV);                                   \
    const void* fn = row_solve ? (const void*)p3_kernel<TZ, RPV, VV, true>                     \
                               : (const void*)p3_kernel<TZ, RPV, VV, false>;                   \
    if (sh > 65536)                                                                            \
      err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);      \
    if (err != hipSuccess) break;                                                              \
    if (row_solve)                                                                             \
      timed_launch(p3_kernel<TZ, RPV, VV, true>, grid, dim3(256), sh, s, rs, (const TZ*)Z, Af, \
                   invlamA, Bf, invlamB, Vinv, lam_div, U, sU);                                \
    else                                                                                       \
      timed_launch(p3_kernel<TZ, RPV, VV, false>, grid, dim3(256), sh, s, rs, (const TZ*)Z, Af,\
                   invlamA, Bf, invlamB, Vinv, lam_div, U, sU);                                \
  } while (0)
  SBT_RP_SWITCH(rs.R, {
    if (prec == kF64) {
      if (vw == 2) SBT_P3(double, RP, 2); else SBT_P3(double, RP, 1);
    } else if (prec == kF32) {
      if (vw == 4 && RP <= 16) SBT_P3(float, RP, 4);
      else if (vw >= 2) SBT_P3(float, RP, 2);
      else SBT_P3(float, RP, 1);
    } else {
      if (vw == 4 && RP <= 16) SBT_P3(uint16_t, RP, 4);
      else if (vw >= 2) SBT_P3(uint16_t, RP, 2);
      else SBT_P3(uint16_t, RP, 1);
    }
  });
#undef SBT_P3
  if (err != hipSuccess) return err;
  return hipGetLastError();
}

}  // namespace sbt
