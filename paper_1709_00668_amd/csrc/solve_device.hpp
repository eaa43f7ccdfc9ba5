// Block-level FP64 normal-equation solve of one ALS mode update (Sec. 3.1
// "Decompose": CP-ALS), used inside the fused MTTKRP kernels and on its own.
//
//   V = G1 .* G2            (Hadamard product of the other two Gram matrices)
//   V^-1 by Gauss-Jordan    (in one wavefront's registers; symmetric positive
//                            definite: no pivoting; a pivot that is not
//                            positive means V is singular and the
//                            pseudo-inverse, cut-off R eps max|eig|, is used)
//   U = M V^-1              (rows staged through LDS in chunks)
//   normalize: lambda_f = ||U(:,f)||, U(:,f) /= lambda_f (lambda_f > 0),
//              Gout = U^T U;  otherwise U(:,f) /= lam_div[f] (0 if lam_div[f]=0)
// All reductions have a fixed assignment of rows to threads and a fixed
// combination order, so results do not depend on timing.
#pragma once

#include "device_common.hpp"
#include "kernels.hpp"

namespace sbt {

constexpr int kSolveBuf = 2304;  // doubles of row staging (>= 2 x 32 x 33 for Jacobi)

struct SolveSmem {
  double V[kMaxRank][kMaxRank + 1];  // V, then V^-1 (or the pseudo-inverse)
  double buf[kSolveBuf];             // row chunk (row-major), or Jacobi scratch
  double red[256];
  double wred[4][kMaxRank];
  double lam[kMaxRank];
  int fail;
};

struct SolveArgs {
  const double* M;
  int64_t sM;
  const double* G1;
  int64_t sG1;
  const double* G2;
  int64_t sG2;
  double* U;
  int64_t sU;
  double* Gout;        // R*R per repetition (normalize only)
  int64_t sGout;
  double* lam_out;     // R per repetition (normalize only)
  const double* lam_div;  // R, shared (row solve only)
  int normalize;
  uint32_t* pinv_count;
  // with gmask != 0, V is instead the Hadamard product, in mode order, of the
  // Gram matrices Gm + m * sGmode (per repetition stride sG1) of the modes m
  // whose bit is set (order-N tensors)
  uint32_t gmask;
  const double* Gm;
  int64_t sGmode;
};

__device__ inline double solve_v(const SolveArgs& a, int rep, int q) {
  if (!a.gmask) return a.G1[rep * a.sG1 + q] * a.G2[rep * a.sG2 + q];
  // branch-free: every mode's load in flight at once (a mode outside the
  // mask reads mode 0's matrix and contributes a factor of one)
  double g[kMaxOrder];
#pragma unroll
  for (int m = 0; m < kMaxOrder; ++m) {
    const bool on = (a.gmask >> m) & 1u;
    g[m] = a.Gm[(on ? m : 0) * a.sGmode + rep * a.sG1 + q];
  }
  double v = 1.0;
#pragma unroll
  for (int m = 0; m < kMaxOrder; ++m)
    if ((a.gmask >> m) & 1u) v *= g[m];
  return v;
}

__device__ inline void solve_pair_fg(int p, int R, int& f, int& g) {
  f = 0;
  while (p >= R - f) {
    p -= R - f;
    ++f;
  }
  g = f + p;
}

// Cyclic Jacobi eigen-decomposition of the symmetric A (R x R, row stride ld,
// destroyed) with eigenvectors in Q; P = pseudo-inverse.  One thread.
__device__ inline void jacobi_pinv_1t(double* A, double* Q, double* P, int ld, int R) {
  for (int i = 0; i < R; ++i)
    for (int j = 0; j < R; ++j) Q[i * ld + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < R; ++i) {
      dia += A[i * ld + i] * A[i * ld + i];
      for (int j = i + 1; j < R; ++j) off += A[i * ld + j] * A[i * ld + j];
    }
    if (off <= 1e-32 * dia || off == 0.0) break;
    for (int p = 0; p < R; ++p)
      for (int q = p + 1; q < R; ++q) {
        const double apq = A[p * ld + q];
        if (apq == 0.0) continue;
        const double theta = (A[q * ld + q] - A[p * ld + p]) / (2.0 * apq);
        const double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
        for (int k = 0; k < R; ++k) {
          const double akp = A[k * ld + p], akq = A[k * ld + q];
          A[k * ld + p] = c * akp - s * akq;
          A[k * ld + q] = s * akp + c * akq;
        }
        for (int k = 0; k < R; ++k) {
          const double apk = A[p * ld + k], aqk = A[q * ld + k];
          A[p * ld + k] = c * apk - s * aqk;
          A[q * ld + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < R; ++k) {
          const double qkp = Q[k * ld + p], qkq = Q[k * ld + q];
          Q[k * ld + p] = c * qkp - s * qkq;
          Q[k * ld + q] = s * qkp + c * qkq;
        }
      }
  }
  double emax = 0.0;
  for (int i = 0; i < R; ++i) emax = fmax(emax, fabs(A[i * ld + i]));
  const double cut = (double)R * 2.220446049250313e-16 * emax;
  for (int i = 0; i < R; ++i)
    for (int j = 0; j < R; ++j) {
      double s = 0.0;
      for (int k = 0; k < R; ++k)
        if (fabs(A[k * ld + k]) > cut) s += Q[i * ld + k] * Q[j * ld + k] / A[k * ld + k];
      P[i * ld + j] = s;
    }
}

__device__ inline double readlane_f64(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xFFFFFFFFull), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Gauss-Jordan inverse of the symmetric positive definite V (R x R, in LDS)
// by the first wavefront, without pivoting: lane i holds row i of [V | I]
// and the pivot row is broadcast with readlane, so no barriers are needed.
// Returns false (uniform over the wave) when a pivot is not positive; the
// result is in V only when it returns true.
template <int RP>
__device__ bool wave_gj_inverse_v(double (*V)[kMaxRank + 1], int R) {
  const int i = lane_id();
  double a[RP], b[RP];
#pragma unroll
  for (int j = 0; j < RP; ++j) {
    a[j] = (i < R && j < R) ? V[i][j] : 0.0;
    b[j] = (i == j) ? 1.0 : 0.0;
  }
  bool ok = true;
#pragma unroll
  for (int k = 0; k < RP; ++k) {
    if (k < R) {
      const double piv = readlane_f64(a[k], k);
      if (!(piv > 0.0)) {
        ok = false;
        break;
      }
      const double rp = 1.0 / piv;
      const double m = a[k] * rp;
      // pivot row: columns j < k of a and j > k of b are zero at this point
      double pa[RP], pb[RP];
#pragma unroll
      for (int j = 0; j < RP; ++j) {
        pa[j] = j >= k ? readlane_f64(a[j], k) : 0.0;
        pb[j] = j <= k ? readlane_f64(b[j], k) : 0.0;
      }
      if (i == k) {
#pragma unroll
        for (int j = 0; j < RP; ++j) {
          a[j] = pa[j] * rp;
          b[j] = pb[j] * rp;
        }
      } else {
#pragma unroll
        for (int j = 0; j < RP; ++j) {
          if (j >= k) a[j] = a[j] - m * pa[j];
          if (j <= k) b[j] = b[j] - m * pb[j];
        }
      }
    }
  }
  if (ok && i < R) {
#pragma unroll
    for (int j = 0; j < RP; ++j)
      if (j < R) V[i][j] = b[j];
  }
  return ok;
}

template <int RP>
__device__ void block_solve(const SolveArgs& a, int rep, int rows, int R, SolveSmem& s) {
  const int tid = threadIdx.x;
  const double* M = a.M + rep * a.sM;
  double* U = a.U + rep * a.sU;
  __syncthreads();
  for (int q = tid; q < R * R; q += 256) s.V[q / R][q % R] = solve_v(a, rep, q);
  if (tid == 0) s.fail = 0;
  __syncthreads();
  // Gauss-Jordan inversion in the registers of the first wavefront
  if (tid < kWave) {
    const bool ok = wave_gj_inverse_v<RP>(s.V, R);
    if (tid == 0 && !ok) s.fail = 1;
  }
  __syncthreads();
  if (s.fail) {
    // singular V: pseudo-inverse from the original V (rebuilt in buf)
    double* A0 = s.buf;
    double* Q = s.buf + kMaxRank * (kMaxRank + 1);
    for (int q = tid; q < R * R; q += 256) A0[(q / R) * (kMaxRank + 1) + q % R] = solve_v(a, rep, q);
    __syncthreads();
    if (tid == 0) {
      jacobi_pinv_1t(A0, Q, &s.V[0][0], kMaxRank + 1, R);
      if (a.pinv_count) atomicAdd(a.pinv_count, 1u);
    }
    __syncthreads();
  }

  // pass A: U = M V^-1 chunk by chunk (thread per output element); for the
  // ALS update also the Gram matrix of the unnormalised U, whose diagonal
  // gives the column norms.
  const int crows = kSolveBuf / R;
  const int nchunks = (rows + crows - 1) / crows;
  constexpr int kPer = (kSolveBuf + 255) / 256;
  const int P = R * (R + 1) / 2;
  const int S = P >= 256 ? 1 : 256 / P;
  double gacc[3] = {0.0, 0.0, 0.0};
  for (int r0 = 0; r0 < rows; r0 += crows) {
    const int cn = rows - r0 < crows ? rows - r0 : crows;
    const int ne = cn * R;
    __syncthreads();
    for (int q = tid; q < ne; q += 256) s.buf[q] = M[(int64_t)r0 * R + q];
    __syncthreads();
    double uo[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int q = tid + 256 * j;
      double acc = 0.0;
      if (q < ne) {
        const int i = q / R, f = q % R;
        const double* mrow = s.buf + i * R;
#pragma unroll 4
        for (int k = 0; k < R; ++k) acc += mrow[k] * s.V[k][f];
        if (!a.normalize) {
          const double l = a.lam_div[f];
          acc = l > 0.0 ? acc / l : 0.0;
        }
      }
      uo[j] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int q = tid + 256 * j;
      if (q < ne) s.buf[q] = uo[j];
    }
    __syncthreads();
    if (!a.normalize || nchunks > 1)
      for (int q = tid; q < ne; q += 256) U[(int64_t)r0 * R + q] = s.buf[q];
    if (!a.normalize) continue;
    if (P <= 256) {
      const int p = tid % P, sl = tid / P;
      if (sl < S) {
        int f, g;
        solve_pair_fg(p, R, f, g);
        for (int i = sl; i < cn; i += S) gacc[0] += s.buf[i * R + f] * s.buf[i * R + g];
      }
    } else {
      for (int j = 0; j < 3; ++j) {
        const int p = tid + 256 * j;
        if (p < P) {
          int f, g;
          solve_pair_fg(p, R, f, g);
          for (int i = 0; i < cn; ++i) gacc[j] += s.buf[i * R + f] * s.buf[i * R + g];
        }
      }
    }
  }
  if (!a.normalize) return;

  // Gram of the unnormalised U -> lambda and the Gram of the normalised U
  __syncthreads();
  double* Gu = &s.V[0][0];  // V^-1 is no longer needed; R x R, row stride kMaxRank + 1
  if (P <= 256) {
    s.red[tid] = gacc[0];
    __syncthreads();
    if (tid < P) {
      double acc = 0.0;
      for (int sl = 0; sl < S; ++sl) acc += s.red[sl * P + tid];
      int f, g;
      solve_pair_fg(tid, R, f, g);
      Gu[f * (kMaxRank + 1) + g] = acc;
      Gu[g * (kMaxRank + 1) + f] = acc;
    }
  } else {
    for (int j = 0; j < 3; ++j) {
      const int p = tid + 256 * j;
      if (p < P) {
        int f, g;
        solve_pair_fg(p, R, f, g);
        Gu[f * (kMaxRank + 1) + g] = gacc[j];
        Gu[g * (kMaxRank + 1) + f] = gacc[j];
      }
    }
  }
  __syncthreads();
  if (tid < R) {
    const double l = sqrt(Gu[tid * (kMaxRank + 1) + tid]);
    s.lam[tid] = l;
    a.lam_out[rep * R + tid] = l;
  }
  __syncthreads();
  double* G = a.Gout + rep * a.sGout;
  for (int q = tid; q < R * R; q += 256) {
    const int f = q / R, g = q % R;
    const double lf = s.lam[f], lg = s.lam[g];
    double v = Gu[f * (kMaxRank + 1) + g];
    if (lf > 0.0) v = v / lf;
    if (lg > 0.0) v = v / lg;
    G[q] = v;
  }
  // pass B: normalise and write U
  for (int r0 = 0; r0 < rows; r0 += crows) {
    const int cn = rows - r0 < crows ? rows - r0 : crows;
    if (nchunks > 1) {
      __syncthreads();
      for (int q = tid; q < cn * R; q += 256) s.buf[q] = U[(int64_t)r0 * R + q];
      __syncthreads();
    }
    for (int q = tid; q < cn * R; q += 256) {
      const double l = s.lam[q % R];
      U[(int64_t)r0 * R + q] = l > 0.0 ? s.buf[q] / l : s.buf[q];
    }
  }
}

}  // namespace sbt
