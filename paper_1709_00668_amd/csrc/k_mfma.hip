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
// mode 3) is formed in FP32 and split into two BF16 parts, hi = bf16(x) and
// lo = bf16(x - hi), each contracted with the summary (two MFMAs into one
// accumulator): the factor side then carries about 16 bits, and only the data
// are BF16.  Rounding the factor operand itself to BF16 makes the MTTKRP
// inconsistent with the FP64 Gram matrices of the normal equations, and with
// the nearly collinear factors of non-negative data that inconsistency is
// amplified by the conditioning of the solve (the fit of an update drops by
// several 1e-3); the split removes it at the price of MFMA issue slots the
// memory-bound passes have to spare.  Modes 1 and 2 then contract W (FP32) as
// in the other precisions; Gram matrices, solves and normalisation stay in
// FP64.
//
// Lane layout of the 16 x 16 x 32 operation (wave of 64): operand A row
// i = lane % 16 holds 8 consecutive K entries of group lane / 16; operand B
// column j = lane % 16 likewise; result lane holds rows 4 (lane / 16) + v,
// v = 0..3, of column lane % 16.  A and B use the same K grouping, so the
// hardware's internal order of K does not matter.
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
// thread = (e, group of 8 third-mode positions); c >= K' are written as zeros
// in Zc (the K range of pass W is K' rounded up to 32).
template <typename TIn>
__global__ __launch_bounds__(256) void gather_mfma_kernel(const TIn* X, int64_t I, int64_t J,
                                                         const int32_t* idx, int64_t idx_stride,
                                                         int64_t offJ, int64_t offK, int n3old,
                                                         int64_t Kold, RepSet rs, MfmaLayout L,
                                                         uint16_t* Zk, uint16_t* Zc) {
  const int rep = rs.rep0 + blockIdx.z;
  const int cg = blockIdx.y;
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n12) return;
  const int a = (int)(e % rs.n1), b = (int)(e / rs.n1);
  const int32_t* Is = idx + rep * idx_stride;
  const int64_t base = (int64_t)Is[a] + I * (int64_t)Is[offJ + b];
  uint16_t* zk = Zk + rep * L.sZk + a + (int64_t)L.ld1 * b;
  uint16_t v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int c = cg * 8 + j;
    v[j] = 0;
    if (c < rs.n3) {
      const int64_t kk = c < n3old ? (int64_t)Is[offK + c] : Kold + (c - n3old);
      v[j] = f32_to_bf16_rne((float)X[base + I * J * kk]);
      zk[L.sk * c] = v[j];
    }
  }
  uint4 pk;
  pk.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
  pk.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
  pk.z = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
  pk.w = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
  *reinterpret_cast<uint4*>(Zc + rep * L.sZc + e * L.ldc + cg * 8) = pk;
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
// pass W on the matrix cores
// ---------------------------------------------------------------------------
// Block = 4 wavefronts x 16 rows e of one repetition; every wave runs the
// whole K range (K' rounded up to 32) against C~^T staged in LDS as BF16.
constexpr int kWPre = 8;  // K steps whose operand loads are in flight at once

template <int NT>
__global__ __launch_bounds__(256) void pw_mfma_kernel(RepSet rs, MfmaLayout L, int kp32,
                                                     const uint16_t* Zc, const double* Cf,
                                                     const double* invlamC, float* W) {
  extern __shared__ __align__(16) unsigned char pwm_smem[];
  const int ldt = kp32 + 8;
  uint16_t* Ct = reinterpret_cast<uint16_t*>(pwm_smem);  // hi part [16 NT][ldt]
  uint16_t* Cl = Ct + 16 * NT * ldt;                      // lo part
  const int rep = rs.rep0 + blockIdx.y;
  const int R = rs.R;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  const int64_t e0 = (int64_t)blockIdx.x * 64 + wave * 16;
  const int64_t erow = e0 + (lane & 15) < n12 ? e0 + (lane & 15) : n12 - 1;
  const int kq = lane >> 4;
  const uint16_t* zrow = Zc + rep * L.sZc + erow * L.ldc + 8 * kq;
  const int ksteps = kp32 / 32;
  // first operand loads before the staging
  bf16x8_t af[kWPre];
#pragma unroll
  for (int u = 0; u < kWPre; ++u)
    if (u < ksteps) af[u] = ld_bf16x8(zrow + 32 * u);
  {
    const double* C = Cf + rep * rs.sC;
    const double* il = invlamC ? invlamC + rep * 3 * R : nullptr;
    const int n = 16 * NT * kp32;
    for (int q = tid; q < n; q += 256) {
      const int f = q / kp32, c = q % kp32;
      float x = 0.0f;
      if (f < R && c < rs.n3) x = (float)(C[(int64_t)c * R + f] * (il ? il[f] : 1.0));
      const uint16_t h = f32_to_bf16_rne(x);
      Ct[f * ldt + c] = h;
      Cl[f * ldt + c] = f32_to_bf16_rne(x - bf16_to_f32(h));
    }
  }
  __syncthreads();
  f32x4_t acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < ksteps; k0 += kWPre) {
    if (k0 > 0) {
#pragma unroll
      for (int u = 0; u < kWPre; ++u)
        if (k0 + u < ksteps) af[u] = ld_bf16x8(zrow + 32 * (k0 + u));
    }
#pragma unroll
    for (int u = 0; u < kWPre; ++u) {
      if (k0 + u < ksteps) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int o = (16 * t + (lane & 15)) * ldt + 32 * (k0 + u) + 8 * kq;
          acc[t] = mfma16x16x32(af[u], ld_bf16x8(Ct + o), acc[t]);
          acc[t] = mfma16x16x32(af[u], ld_bf16x8(Cl + o), acc[t]);
        }
      }
    }
  }
  float* Wr = W + rep * rs.sW;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int f = 16 * t + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t e = e0 + 4 * kq + v;
      if (e < n12 && f < R) Wr[e * R + f] = acc[t][v];
    }
  }
}

// ---------------------------------------------------------------------------
// mode 3 on the matrix cores
// ---------------------------------------------------------------------------
// Block = 4 wavefronts x 16 rows c (64 consecutive c) of one repetition over
// one of nsplit ranges of the K steps; the wave forms its Khatri-Rao operand
// from A~^T (all of it) and the B~^T rows its K range touches, both in LDS
// as FP32.  Partial rows go to P[rep][split][c][16 NT]; mode3_finish adds the
// ranges in order and applies V^-1.
template <int NT>
__global__ __launch_bounds__(256) void p3_mfma_kernel(RepSet rs, MfmaLayout L, int nsplit,
                                                     const uint16_t* Zk, const double* Af,
                                                     const double* invlamA, const double* Bf,
                                                     const double* invlamB, float* P,
                                                     int64_t sP) {
  extern __shared__ __align__(16) unsigned char p3m_smem[];
  float* At = reinterpret_cast<float*>(p3m_smem);  // [16 NT][ld1]
  const int rep = rs.rep0 + blockIdx.z;
  const int split = blockIdx.y;
  const int R = rs.R, n1 = rs.n1, n2 = rs.n2, n3 = rs.n3, ld1 = L.ld1;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int ksteps = (int)(L.sk / 32);
  const int ks_lo = (int)((int64_t)split * ksteps / nsplit);
  const int ks_hi = (int)((int64_t)(split + 1) * ksteps / nsplit);
  const int b_lo = (ks_lo * 32) / ld1;
  int b_hi = ks_hi > ks_lo ? (ks_hi * 32 - 1) / ld1 : b_lo;
  if (b_hi > n2 - 1) b_hi = n2 - 1;
  const int nb = b_hi >= b_lo ? b_hi - b_lo + 1 : 0;
  float* Bt = At + 16 * NT * ld1;  // [16 NT][nb]
  const int c0 = blockIdx.x * 64 + wave * 16;
  const int crow = c0 + (lane & 15) < n3 ? c0 + (lane & 15) : n3 - 1;
  const int kq = lane >> 4;
  const uint16_t* zrow = Zk + rep * L.sZk + (int64_t)crow * L.sk + 8 * kq;
  bf16x8_t af[kWPre];
#pragma unroll
  for (int u = 0; u < kWPre; ++u)
    if (ks_lo + u < ks_hi) af[u] = ld_bf16x8(zrow + 32 * (ks_lo + u));
  {
    const double* A = Af + rep * rs.sA;
    const double* B = Bf + rep * rs.sB;
    const double* ilA = invlamA ? invlamA + rep * 3 * R : nullptr;
    const double* ilB = invlamB ? invlamB + rep * 3 * R : nullptr;
    const int na = 16 * NT * ld1;
    for (int q = tid; q < na; q += 256) {
      const int f = q / ld1, a = q % ld1;
      float x = 0.0f;
      if (f < R && a < n1) x = (float)(A[(int64_t)a * R + f] * (ilA ? ilA[f] : 1.0));
      At[q] = x;
    }
    const int nbb = 16 * NT * nb;
    for (int q = tid; q < nbb; q += 256) {
      const int f = q / nb, bb = q % nb;
      float x = 0.0f;
      if (f < R) x = (float)(B[(int64_t)(b_lo + bb) * R + f] * (ilB ? ilB[f] : 1.0));
      Bt[q] = x;
    }
  }
  __syncthreads();
  f32x4_t acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  for (int k0 = ks_lo; k0 < ks_hi; k0 += kWPre) {
    if (k0 > ks_lo) {
#pragma unroll
      for (int u = 0; u < kWPre; ++u)
        if (k0 + u < ks_hi) af[u] = ld_bf16x8(zrow + 32 * (k0 + u));
    }
#pragma unroll
    for (int u = 0; u < kWPre; ++u) {
      if (k0 + u < ks_hi) {
        // this lane's 8 consecutive e' share one b (ld1 is a multiple of 8)
        const int ep = 32 * (k0 + u) + 8 * kq;
        const int a0 = ep % ld1, b = ep / ld1;
        const bool bin = b <= b_hi;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int f = 16 * t + (lane & 15);
          const float4 x0 = *reinterpret_cast<const float4*>(At + f * ld1 + a0);
          const float4 x1 = *reinterpret_cast<const float4*>(At + f * ld1 + a0 + 4);
          const float bv = bin ? Bt[f * nb + (b - b_lo)] : 0.0f;
          const float x[8] = {x0.x * bv, x0.y * bv, x0.z * bv, x0.w * bv,
                              x1.x * bv, x1.y * bv, x1.z * bv, x1.w * bv};
          bf16x8_t kh, kl;
          split_bf16x8(x, kh, kl);
          acc[t] = mfma16x16x32(af[u], kh, acc[t]);
          acc[t] = mfma16x16x32(af[u], kl, acc[t]);
        }
      }
    }
  }
  float* Pr = P + (rep * (int64_t)nsplit + split) * sP;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int f = 16 * t + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = c0 + 4 * kq + v;
      if (c < n3) Pr[(int64_t)c * (16 * NT) + f] = acc[t][v];
    }
  }
}

// rows of C: sum of the split partials (in split order), times V^-1, divided
// by lam_div for the row solve.  Block = 8 rows of one repetition.
__global__ __launch_bounds__(256) void mode3_finish_kernel(RepSet rs, int nsplit, int ldp,
                                                          const float* P, int64_t sP,
                                                          const double* Vinv,
                                                          const double* lam_div, double* Uout,
                                                          int64_t sU) {
  __shared__ double M[8][kMaxRank];
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
  if (c < rs.n3 && f < R) {
    double u = 0.0;
    for (int k = 0; k < R; ++k) u += M[r][k] * Vi[k][f];
    if (lam_div) {
      const double l = lam_div[f];
      u = l > 0.0 ? u / l : 0.0;
    }
    Uout[rep * sU + (int64_t)c * R + f] = u;
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

bool mfma_supported(int n1, int n2, int R) {
  if (R > 32 || n1 < 1 || n2 < 1) return false;
  // LDS of the mode-3 kernel: A~^T plus at most all of B~^T
  const size_t lds = (size_t)16 * ntiles(R) * 4 * ((size_t)(n1 + 7) / 8 * 8 + n2);
  return lds <= 65536;
}

int mfma_mode3_splits(const RepSet& rs, const MfmaLayout& L) {
  const int cblocks = (rs.n3 + 63) / 64;
  const int ksteps = (int)(L.sk / 32);
  int ns = (2048 + cblocks * rs.nrep - 1) / (cblocks * rs.nrep);
  const int cap = ksteps / 8 > 0 ? ksteps / 8 : 1;
  if (ns > cap) ns = cap;
  if (ns < 1) ns = 1;
  return ns;
}

hipError_t launch_gather_mfma(int store_prec, const void* X, int64_t I, int64_t J,
                              const int32_t* idx, int64_t idx_stride, int64_t offJ, int64_t offK,
                              int n3old, int64_t Kold, const RepSet& rs, const MfmaLayout& L,
                              uint16_t* Zk, uint16_t* Zc, hipStream_t s) {
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  const int kp32 = (rs.n3 + 31) / 32 * 32;
  dim3 grid((unsigned)((n12 + 255) / 256), (unsigned)(kp32 / 8), (unsigned)rs.nrep);
  if (store_prec == kF64)
    gather_mfma_kernel<double><<<grid, 256, 0, s>>>((const double*)X, I, J, idx, idx_stride, offJ,
                                                    offK, n3old, Kold, rs, L, Zk, Zc);
  else
    gather_mfma_kernel<float><<<grid, 256, 0, s>>>((const float*)X, I, J, idx, idx_stride, offJ,
                                                   offK, n3old, Kold, rs, L, Zk, Zc);
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

hipError_t launch_pw_mfma(const RepSet& rs, const MfmaLayout& L, const uint16_t* Zc,
                          const double* Cf, const double* invlamC, float* W, hipStream_t s) {
  const int64_t n12 = (int64_t)rs.n1 * rs.n2;
  const int kp32 = (rs.n3 + 31) / 32 * 32;
  if (kp32 > L.ldc) return hipErrorInvalidValue;
  dim3 grid((unsigned)((n12 + 63) / 64), (unsigned)rs.nrep);
  const size_t sh = (size_t)2 * 16 * ntiles(rs.R) * (kp32 + 8) * 2;
  if (sh > 65536) return hipErrorInvalidValue;
  if (ntiles(rs.R) == 1)
    pw_mfma_kernel<1><<<grid, 256, sh, s>>>(rs, L, kp32, Zc, Cf, invlamC, W);
  else
    pw_mfma_kernel<2><<<grid, 256, sh, s>>>(rs, L, kp32, Zc, Cf, invlamC, W);
  return hipGetLastError();
}

hipError_t launch_p3_mfma(const RepSet& rs, const MfmaLayout& L, int nsplit, const uint16_t* Zk,
                          const double* Af, const double* invlamA, const double* Bf,
                          const double* invlamB, float* P, int64_t sP, hipStream_t s) {
  dim3 grid((unsigned)((rs.n3 + 63) / 64), (unsigned)nsplit, (unsigned)rs.nrep);
  const int nt = ntiles(rs.R);
  // B~ rows touched by one split: at most all n2
  const size_t sh = (size_t)16 * nt * 4 * ((size_t)L.ld1 + rs.n2);
  if (sh > 65536 || sP < (int64_t)rs.n3 * 16 * nt) return hipErrorInvalidValue;
  if (nt == 1)
    p3_mfma_kernel<1><<<grid, 256, sh, s>>>(rs, L, nsplit, Zk, Af, invlamA, Bf, invlamB, P, sP);
  else
    p3_mfma_kernel<2><<<grid, 256, sh, s>>>(rs, L, nsplit, Zk, Af, invlamA, Bf, invlamB, P, sP);
  return hipGetLastError();
}

hipError_t launch_mode3_finish(const RepSet& rs, int nsplit, const float* P, int64_t sP,
                               const double* Vinv, const double* lam_div, double* U, int64_t sU,
                               hipStream_t s) {
  dim3 grid((unsigned)((rs.n3 + 7) / 8), (unsigned)rs.nrep);
  mode3_finish_kernel<<<grid, 256, 0, s>>>(rs, nsplit, 16 * ntiles(rs.R), P, sP, Vinv, lam_div,
                                           U, sU);
  return hipGetLastError();
}

}  // namespace sbt
