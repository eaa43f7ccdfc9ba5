// Batched CP-ALS on the r summaries of one update (Sec. 3.1 "Decompose"),
// organised for latency: three streaming kernels per sweep, each of which
// produces complete rows of the updated factor.
//
//   pass W   W(ab, f) = sum_c Z(ab, c) C~(c, f)                (all modes share)
//   mode 1   A(a, :)  = [sum_b W(a, b, :) * B~(b, :)] V1^-1     rows of A per block
//   mode 2   B(b, :)  = [sum_a W(a, b, :) * A~(a, :)] V2^-1     rows of B per block
//   mode 3   C(c, :)  = [sum_ab Z(a,b,c) A~(a,:) * B~(b,:)] V3^-1   one slice per block
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
constexpr int kChunk = 64;                      // factor rows staged per LDS chunk
constexpr int kTailBuf = 2304;                  // doubles; >= 2 x 32 x 33 (Jacobi scratch)
constexpr int kLd = kMaxRank + 1;

struct TailSmem {
  double V[kMaxRank][kLd];  // Gram of the new factor, then V_next, then V_next^-1
  double buf[kTailBuf];     // factor rows, or Jacobi scratch
  double red[256];
  double lam[kMaxRank];
  int fail;
};

// Step outputs of one mode update (per repetition strides in elements).
struct TailArgs {
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

// Vout = (Gx .* Gy)^-1 by Gauss-Jordan in LDS (symmetric positive definite: no
// pivoting); a pivot that is not positive switches to the pseudo-inverse.
__device__ void block_inverse(const double* Gx, const double* Gy, int R, double* Vout,
                              TailSmem& s, uint32_t* pinv_count) {
  const int tid = threadIdx.x;
  __syncthreads();
  for (int q = tid; q < R * R; q += 256) s.V[q / R][q % R] = Gx[q] * Gy[q];
  if (tid == 0) s.fail = 0;
  __syncthreads();
  for (int k = 0; k < R; ++k) {
    const double piv = s.V[k][k];
    if (!(piv > 0.0)) {  // uniform
      if (tid == 0) s.fail = 1;
      break;
    }
    double nv[4];
    int nq = 0;
    for (int q = tid; q < R * R; q += 256, ++nq) {
      const int i = q / R, j = q % R;
      const double vik = s.V[i][k], vkj = s.V[k][j];
      double v;
      if (i == k)
        v = (j == k) ? 1.0 / piv : vkj / piv;
      else
        v = (j == k) ? -vik / piv : s.V[i][j] - vik * (vkj / piv);
      nv[nq] = v;
    }
    __syncthreads();
    nq = 0;
    for (int q = tid; q < R * R; q += 256, ++nq) s.V[q / R][q % R] = nv[nq];
    __syncthreads();
  }
  __syncthreads();
  if (s.fail) {
    double* A0 = s.buf;
    double* Q = s.buf + kMaxRank * kLd;
    for (int q = tid; q < R * R; q += 256) A0[(q / R) * kLd + q % R] = Gx[q] * Gy[q];
    __syncthreads();
    if (tid == 0) {
      jacobi_pinv(A0, Q, &s.V[0][0], R);
      if (pinv_count) atomicAdd(pinv_count, 1u);
    }
    __syncthreads();
  }
  for (int q = tid; q < R * R; q += 256) Vout[q] = s.V[q / R][q % R];
}

// Last block of a repetition: Gram of the new raw factor, lambda, normalised
// Gram, inverse for the next step.
__device__ void als_tail(const TailArgs& t, int rep, int R, TailSmem& s) {
  const int tid = threadIdx.x;
  const double* U = t.U + rep * t.sU;
  const int rows = t.rows;
  const int P = R * (R + 1) / 2;
  const int S = P >= 256 ? 1 : 256 / P;
  const int crows = kTailBuf / R;
  double gacc[3][4];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int u = 0; u < 4; ++u) gacc[j][u] = 0.0;
  for (int r0 = 0; r0 < rows; r0 += crows) {
    const int cn = rows - r0 < crows ? rows - r0 : crows;
    __syncthreads();
    for (int q = tid; q < cn * R; q += 256) s.buf[q] = U[(int64_t)r0 * R + q];
    __syncthreads();
    for (int j = 0; j < 3; ++j) {
      const int p = P <= 256 ? tid % P : tid + 256 * j;
      const int sl = P <= 256 ? tid / P : 0;
      if ((P <= 256 && (j > 0 || sl >= S)) || p >= P) continue;
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
  if (P <= 256) {
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
      const int p = tid + 256 * j;
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
    t.invlam_out[rep * 3 * R + tid] = l > 0.0 ? 1.0 / l : 1.0;  // [A | B | C] per repetition
    if (t.lam_out) t.lam_out[rep * R + tid] = l;
  }
  __syncthreads();
  double* G = t.Gout + rep * t.sG;
  for (int q = tid; q < R * R; q += 256) {
    const int f = q / R, g = q % R;
    const double lf = s.lam[f], lg = s.lam[g];
    double v = s.V[f][g];
    if (lf > 0.0) v = v / lf;
    if (lg > 0.0) v = v / lg;
    G[q] = v;
  }
  __syncthreads();  // G visible to the block before it is read back below
  block_inverse(t.Gx + rep * t.sG, t.Gy + rep * t.sG, R, t.Vinv_out + rep * t.sG, s,
                t.pinv_count);
}

// ---------------------------------------------------------------------------
// pass W
// ---------------------------------------------------------------------------
template <typename TZ, int RP, int V>
__global__ __launch_bounds__(256) void pw_kernel(RepSet rs, int csz, const TZ* Z,
                                                const double* Cf, const double* invlamC,
                                                typename AccT<TZ>::type* W) {
  using TA = typename AccT<TZ>::type;
  constexpr int KU = ku_of(V);
  const int rep = rs.rep0 + blockIdx.z;
  const int split = blockIdx.y;
  const int R = rs.R;
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  const int c0 = split * csz;
  const int c1 = c0 + csz < rs.n3 ? c0 + csz : rs.n3;
  Z += rep * rs.sZ;
  Cf += rep * rs.sC;
  const double* il = invlamC + rep * 3 * R;
  __shared__ TA Cs[kChunk][RP];
  const int64_t e0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * V;
  const bool ok = e0 < n12;
  TA acc[V][RP];
#pragma unroll
  for (int v = 0; v < V; ++v)
#pragma unroll
    for (int f = 0; f < RP; ++f) acc[v][f] = 0;
  for (int cc0 = c0; cc0 < c1; cc0 += kChunk) {
    const int cn = c1 - cc0 < kChunk ? c1 - cc0 : kChunk;
    __syncthreads();
    for (int q = threadIdx.x; q < kChunk * RP; q += 256) {
      const int cc = q / RP, f = q % RP;
      Cs[cc][f] = (cc < cn && f < R) ? (TA)(Cf[(int64_t)(cc0 + cc) * R + f] * il[f]) : (TA)0;
    }
    __syncthreads();
    if (ok) {
      const TZ* zp = Z + e0 + n12 * cc0;
      int cc = 0;
      for (; cc + KU <= cn; cc += KU) {
        TA z[KU][V];
#pragma unroll
        for (int u = 0; u < KU; ++u) ldv(zp + n12 * (cc + u), z[u]);
#pragma unroll
        for (int u = 0; u < KU; ++u)
#pragma unroll
          for (int f = 0; f < RP; ++f) {
            const TA cv = Cs[cc + u][f];
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v][f] += z[u][v] * cv;
          }
      }
      for (; cc < cn; ++cc) {
        TA z[V];
        ldv(zp + n12 * cc, z);
#pragma unroll
        for (int f = 0; f < RP; ++f)
#pragma unroll
          for (int v = 0; v < V; ++v) acc[v][f] += z[v] * Cs[cc][f];
      }
    }
  }
  if (ok) {
    TA* w = W + rep * rs.sW + ((int64_t)split * n12 + e0) * R;
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int f = 0; f < RP; ++f)
        if (f < R) w[v * R + f] = acc[v][f];
  }
}

// ---------------------------------------------------------------------------
// modes 1 and 2 from W
// ---------------------------------------------------------------------------
constexpr int kRowsPerBlock = 8;   // factor rows produced by one block
constexpr int kSlots = 32;         // threads sharing one row (the contracted index)

template <typename TA, int RP>
struct CwSmem {
  TA Fs[kChunk][RP];                     // staged rows of the contracted factor
  TA red[4][kRowsPerBlock][RP];          // per-wave partial rows
  double Mrow[kRowsPerBlock][kMaxRank];  // contracted rows
  double Vi[kMaxRank][kLd];              // V^-1
};

// mode = 0: rows a of A from B~;  mode = 1: rows b of B from A~.  Raw rows
// U = M V^-1 are written; the tail kernel follows.
template <typename TA, int RP>
__global__ __launch_bounds__(256) void cw_kernel(RepSet rs, int mode, const TA* W,
                                                const double* F, const double* invlamF,
                                                const double* Vinv, double* Uout, int64_t sU) {
  __shared__ CwSmem<TA, RP> sm;
  const int rep = rs.rep0 + blockIdx.y;
  const int R = rs.R, n1 = rs.n1, n2 = rs.n2, ns = rs.nsplit;
  const int tid = threadIdx.x;
  const int64_t n12 = (int64_t)n1 * n2;
  // mode 0: row = low 3 bits of tid (consecutive a, coalesced), slot = high 5
  // mode 1: slot = low 5 bits (consecutive a, coalesced), row = high 3
  const int rl = mode == 0 ? (tid & (kRowsPerBlock - 1)) : (tid >> 5);  // row within block
  const int sl = mode == 0 ? (tid >> 3) : (tid & (kSlots - 1));         // slot
  const int row = blockIdx.x * kRowsPerBlock + rl;
  const int nrows = mode == 0 ? n1 : n2;
  const int ncon = mode == 0 ? n2 : n1;  // contracted extent
  const bool ok = row < nrows;
  const TA* Wr = W + rep * rs.sW;
  const double* Fr = F + (mode == 0 ? rep * rs.sB : rep * rs.sA);
  const double* il = invlamF + rep * 3 * R;
  for (int q = tid; q < R * R; q += 256) sm.Vi[q / R][q % R] = Vinv[rep * rs.sG + q];
  TA acc[RP];
#pragma unroll
  for (int f = 0; f < RP; ++f) acc[f] = 0;
  for (int x0 = 0; x0 < ncon; x0 += kChunk) {
    const int xn = ncon - x0 < kChunk ? ncon - x0 : kChunk;
    __syncthreads();
    for (int q = tid; q < kChunk * RP; q += 256) {
      const int xx = q / RP, f = q % RP;
      sm.Fs[xx][f] = (xx < xn && f < R) ? (TA)(Fr[(int64_t)(x0 + xx) * R + f] * il[f]) : (TA)0;
    }
    __syncthreads();
    if (ok) {
      for (int sp = 0; sp < ns; ++sp) {
        const TA* Ws = Wr + (int64_t)sp * n12 * R;
        int xx = sl;
        for (; xx + kSlots < xn; xx += 2 * kSlots) {
          const int64_t e0 = mode == 0 ? (int64_t)row + (int64_t)n1 * (x0 + xx)
                                       : (int64_t)(x0 + xx) + (int64_t)n1 * row;
          const int64_t e1 = mode == 0 ? e0 + (int64_t)n1 * kSlots : e0 + kSlots;
          TA w0[RP], w1[RP];
#pragma unroll
          for (int f = 0; f < RP; ++f) {
            w0[f] = f < R ? Ws[e0 * R + f] : (TA)0;
            w1[f] = f < R ? Ws[e1 * R + f] : (TA)0;
          }
#pragma unroll
          for (int f = 0; f < RP; ++f)
            acc[f] += w0[f] * sm.Fs[xx][f] + w1[f] * sm.Fs[xx + kSlots][f];
        }
        for (; xx < xn; xx += kSlots) {
          const int64_t e0 = mode == 0 ? (int64_t)row + (int64_t)n1 * (x0 + xx)
                                       : (int64_t)(x0 + xx) + (int64_t)n1 * row;
#pragma unroll
          for (int f = 0; f < RP; ++f)
            if (f < R) acc[f] += Ws[e0 * R + f] * sm.Fs[xx][f];
        }
      }
    }
  }
  // reduce over the 16 slots: within the wave first, then across waves
  const int wave = tid >> 6;
#pragma unroll
  for (int f = 0; f < RP; ++f) {
    TA v = acc[f];
    if (mode == 0) {  // slots differ in tid bits 3..5 within a wave
      v += __shfl_xor(v, 8, kWave);
      v += __shfl_xor(v, 16, kWave);
      v += __shfl_xor(v, 32, kWave);
    } else {          // slots are tid bits 0..4
      v += __shfl_xor(v, 1, kWave);
      v += __shfl_xor(v, 2, kWave);
      v += __shfl_xor(v, 4, kWave);
      v += __shfl_xor(v, 8, kWave);
      v += __shfl_xor(v, 16, kWave);
    }
    acc[f] = v;
  }
  __syncthreads();
  if (mode == 0) {  // each wave holds 8 of the 32 slots
    if ((tid & 63) < kRowsPerBlock)
#pragma unroll
      for (int f = 0; f < RP; ++f) sm.red[wave][rl][f] = acc[f];
  } else {          // each wave holds two rows, all 32 slots
    if (sl == 0)
#pragma unroll
      for (int f = 0; f < RP; ++f) sm.red[0][rl][f] = acc[f];
  }
  __syncthreads();
  for (int q = tid; q < kRowsPerBlock * R; q += 256) {
    const int r = q / R, f = q % R;
    sm.Mrow[r][f] = mode == 0 ? (double)((sm.red[0][r][f] + sm.red[1][r][f]) +
                                         (sm.red[2][r][f] + sm.red[3][r][f]))
                              : (double)sm.red[0][r][f];
  }
  __syncthreads();
  double* U = Uout + rep * sU;
  for (int q = tid; q < kRowsPerBlock * R; q += 256) {
    const int r = q / R, f = q % R;
    const int gr = blockIdx.x * kRowsPerBlock + r;
    if (gr < nrows) {
      double u = 0.0;
      for (int k = 0; k < R; ++k) u += sm.Mrow[r][k] * sm.Vi[k][f];
      U[(int64_t)gr * R + f] = u;
    }
  }
}

// ---------------------------------------------------------------------------
// mode 3: kSpb slices per block
// ---------------------------------------------------------------------------
constexpr int kSpb = 1;

constexpr int kP3Chunk = 128;  // B~ rows staged at once by the mode-3 kernel

template <typename TA, int RP>
struct P3Smem {
  TA Bs[kP3Chunk][RP];
  TA red[4][kMaxRank];
  double Mrow[kMaxRank];
  double Vi[kMaxRank][kLd];
};

// kRow = false: ALS update of C' (raw rows).  kRow = true: the row solve
// (rows divided by lam_div).
template <typename TZ, int RP, int V, bool kRow>
__global__ __launch_bounds__(256) void p3_kernel(RepSet rs, const TZ* Z, const double* Af,
                                                const double* invlamA, const double* Bf,
                                                const double* invlamB, const double* Vinv,
                                                const double* lam_div, double* Uout,
                                                int64_t sU) {
  using TA = typename AccT<TZ>::type;
  constexpr int KU = V >= 4 ? 4 : (V == 2 ? 8 : 16);  // 16 elements in flight per thread
  __shared__ P3Smem<TA, RP> sm;
  const int rep = rs.rep0 + blockIdx.y;
  const int R = rs.R, n1 = rs.n1, n2 = rs.n2;
  const int tid = threadIdx.x;
  const int64_t n12 = (int64_t)n1 * n2;
  const double* Ar = Af + rep * rs.sA;
  const double* Br = Bf + rep * rs.sB;
  const double* ilA = invlamA ? invlamA + rep * 3 * R : nullptr;
  const double* ilB = invlamB ? invlamB + rep * 3 * R : nullptr;
  for (int q = tid; q < R * R; q += 256) sm.Vi[q / R][q % R] = Vinv[rep * rs.sG + q];
  const int ng = n1 / V;
  const int span = ng >= 256 ? 256 : ng;
  const int nsub = 256 / span;
  const int sub = tid / span, gl = tid % span;
  const bool act = sub < nsub;
  const int wave = tid >> 6;
  const int cfirst = blockIdx.x * kSpb;
  for (int c = cfirst; c < cfirst + kSpb && c < rs.n3; ++c) {
    const TZ* Zc = Z + rep * rs.sZ + n12 * c;
    TA tot[RP];
#pragma unroll
    for (int f = 0; f < RP; ++f) tot[f] = 0;
    for (int g0 = 0; g0 < ng; g0 += span) {
      const int g = g0 + gl;
      const bool ok = act && g < ng;
      TA acc[V][RP];
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int f = 0; f < RP; ++f) acc[v][f] = 0;
      for (int b0 = 0; b0 < n2; b0 += kP3Chunk) {
        const int bn = n2 - b0 < kP3Chunk ? n2 - b0 : kP3Chunk;
        // B~ rows are staged once per block when they fit one chunk
        if (c == cfirst || n2 > kP3Chunk || ng > span) {
          __syncthreads();
          for (int q = tid; q < kP3Chunk * RP; q += 256) {
            const int bb = q / RP, f = q % RP;
            double bv = 0.0;
            if (bb < bn && f < R) {
              bv = Br[(int64_t)(b0 + bb) * R + f];
              if (ilB) bv *= ilB[f];
            }
            sm.Bs[bb][f] = (TA)bv;
          }
          __syncthreads();
        }
        if (ok) {
          const TZ* zp = Zc + (int64_t)g * V + (int64_t)n1 * b0;
          int bb = sub;
          for (; bb + (KU - 1) * nsub < bn; bb += KU * nsub) {
            TA z[KU][V];
#pragma unroll
            for (int u = 0; u < KU; ++u) ldv(zp + (int64_t)n1 * (bb + u * nsub), z[u]);
#pragma unroll
            for (int u = 0; u < KU; ++u)
#pragma unroll
              for (int f = 0; f < RP; ++f) {
                const TA bv = sm.Bs[bb + u * nsub][f];
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v][f] += z[u][v] * bv;
              }
          }
          for (; bb < bn; bb += nsub) {
            TA z[V];
            ldv(zp + (int64_t)n1 * bb, z);
#pragma unroll
            for (int f = 0; f < RP; ++f) {
              const TA bv = sm.Bs[bb][f];
#pragma unroll
              for (int v = 0; v < V; ++v) acc[v][f] += z[v] * bv;
            }
          }
        }
      }
      if (ok) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const double* arow = Ar + (int64_t)(g * V + v) * R;
#pragma unroll
          for (int f = 0; f < RP; ++f)
            if (f < R) {
              double av = arow[f];
              if (ilA) av *= ilA[f];
              tot[f] += acc[v][f] * (TA)av;
            }
        }
      }
    }
#pragma unroll
    for (int f = 0; f < RP; ++f) {
      const TA v = wave_sum(tot[f]);
      if (lane_id() == 0) sm.red[wave][f] = v;
    }
    __syncthreads();
    if (tid < R)
      sm.Mrow[tid] = (double)((sm.red[0][tid] + sm.red[1][tid]) + (sm.red[2][tid] + sm.red[3][tid]));
    __syncthreads();
    if (tid < R) {
      double u = 0.0;
      for (int k = 0; k < R; ++k) u += sm.Mrow[k] * sm.Vi[k][tid];
      if (kRow) {
        const double l = lam_div[tid];
        u = l > 0.0 ? u / l : 0.0;
      }
      Uout[rep * sU + (int64_t)c * R + tid] = u;
    }
  }
}

// Tail of a mode update, one block per repetition.
__global__ __launch_bounds__(256) void tail_kernel(RepSet rs, TailArgs ta) {
  __shared__ TailSmem sm;
  als_tail(ta, rs.rep0 + blockIdx.x, rs.R, sm);
}

// V^-1 = (Gx .* Gy)^-1 per repetition (start of the sweeps, row solve).
__global__ __launch_bounds__(256) void inverse_kernel(RepSet rs, const double* Gx,
                                                     int64_t sGx, const double* Gy,
                                                     int64_t sGy, double* Vinv,
                                                     uint32_t* pinv_count) {
  __shared__ TailSmem sm;
  const int rep = rs.rep0 + blockIdx.x;
  block_inverse(Gx + rep * sGx, Gy + rep * sGy, rs.R, Vinv + rep * rs.sG, sm, pinv_count);
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
  inverse_kernel<<<rs.nrep, 256, 0, s>>>(rs, Gx, sGx, Gy, sGy, Vinv, pinv_count);
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

hipError_t launch_tail(const RepSet& rs, const AlsTail& t, hipStream_t s) {
  TailArgs ta{t.U, t.sU, t.rows, t.Gout, t.invlam_out, t.lam_out, t.Gx, t.Gy, t.Vinv_out,
              t.sG, t.pinv_count};
  tail_kernel<<<rs.nrep, 256, 0, s>>>(rs, ta);
  return hipGetLastError();
}

hipError_t launch_pw(int prec, const RepSet& rs, const void* Z, const double* Cf,
                     const double* invlamC, void* W, hipStream_t s) {
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  const int ns = rs.nsplit < 1 ? 1 : rs.nsplit;
  const int csz = (rs.n3 + ns - 1) / ns;
#define SBT_PW(TZ, RPV)                                                                       \
  do {                                                                                        \
    dim3 grid((unsigned)((n12 + 255) / 256), (unsigned)ns, (unsigned)rs.nrep);                \
    pw_kernel<TZ, RPV, 1><<<grid, 256, 0, s>>>(rs, csz, (const TZ*)Z, Cf, invlamC,            \
                                               (typename AccT<TZ>::type*)W);                  \
  } while (0)
  SBT_RP_SWITCH(rs.R, {
    if (prec == kF64)
      SBT_PW(double, RP);
    else if (prec == kF32)
      SBT_PW(float, RP);
    else
      SBT_PW(uint16_t, RP);
  });
#undef SBT_PW
  return hipGetLastError();
}

hipError_t launch_cw(int prec, const RepSet& rs, int mode, const void* W, const double* F,
                     const double* invlamF, const double* Vinv, double* U, int64_t sU,
                     hipStream_t s) {
  const int nrows = mode == 0 ? rs.n1 : rs.n2;
  dim3 grid((unsigned)((nrows + kRowsPerBlock - 1) / kRowsPerBlock), (unsigned)rs.nrep);
  SBT_RP_SWITCH(rs.R, {
    if (prec == kF64)
      cw_kernel<double, RP><<<grid, 256, 0, s>>>(rs, mode, (const double*)W, F, invlamF, Vinv,
                                                 U, sU);
    else
      cw_kernel<float, RP><<<grid, 256, 0, s>>>(rs, mode, (const float*)W, F, invlamF, Vinv, U,
                                                sU);
  });
  return hipGetLastError();
}

hipError_t launch_p3(int prec, const RepSet& rs, bool row_solve, const void* Z, const double* Af,
                     const double* invlamA, const double* Bf, const double* invlamB,
                     const double* Vinv, const double* lam_div, double* U, int64_t sU,
                     hipStream_t s) {
  dim3 grid((unsigned)((rs.n3 + kSpb - 1) / kSpb), (unsigned)rs.nrep);
  const int vw = prec == kF64 ? (rs.n1 % 2 == 0 ? 2 : 1)
                              : (rs.n1 % 4 == 0 ? 4 : (rs.n1 % 2 == 0 ? 2 : 1));
#define SBT_P3(TZ, RPV, VV)                                                                    \
  do {                                                                                         \
    if (row_solve)                                                                             \
      p3_kernel<TZ, RPV, VV, true><<<grid, 256, 0, s>>>(rs, (const TZ*)Z, Af, invlamA, Bf,     \
                                                        invlamB, Vinv, lam_div, U, sU);        \
    else                                                                                       \
      p3_kernel<TZ, RPV, VV, false><<<grid, 256, 0, s>>>(rs, (const TZ*)Z, Af, invlamA, Bf,    \
                                                         invlamB, Vinv, lam_div, U, sU);       \
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
  return hipGetLastError();
}

}  // namespace sbt
