// GetRank (Sec. 3.2, Alg. 2): the core consistency of a rank-i CP model of
// every dense summary, and the choice of the summary's rank.
//
// Core consistency: with the weights moved into the third factor, the
// least-squares Tucker core for the model's factors is
//   G = Z x1 pinv(A) x2 pinv(B) x3 pinv(C diag(lambda)),
// and CC = 100 (1 - ||G - T||^2 / i) with T superdiagonal ones.  For factors of
// full column rank pinv(U) = (U^T U)^-1 U^T, so G is the projected core
//   P = Z x1 A^T x2 B^T x3 C^T   (i x i x i)
// followed by the three small inverses: G = P x1 GA^-1 x2 GB^-1 x3 diag(1/lambda) GC^-1.
// P is built from W = Z x3 C^T (the mode-3 contraction kernel of the plain
// schedule, W stored [f][e]); then one block per (c, repetition) forms
// P(:, :, c) = A^T W_c B with W_c the n1 x n2 slab of component c.
#include "device_common.hpp"
#include "kernels.hpp"

namespace sbt {

namespace {

constexpr int kCoreJ = 64;  // columns j per staged chunk

// P(a, b, c) for one c and one repetition; P stored [rep][a][b][c] (stride sP)
template <typename TA>
__global__ __launch_bounds__(256) void core_kernel(RepSet rs, const TA* W, const double* Ap,
                                                  const double* Bp, double* P, int64_t sP) {
  const int c = blockIdx.x, rep = rs.rep0 + blockIdx.y;
  const int ir = rs.R, n1 = rs.n1, n2 = rs.n2;
  const int64_t n12 = (int64_t)n1 * n2;
  const TA* Wc = W + rep * rs.sW + (int64_t)c * n12;
  const double* A = Ap + rep * rs.sA;
  const double* B = Bp + rep * rs.sB;
  __shared__ double T[kMaxRank][kCoreJ + 1];  // T(a, jj) = sum_i A(i, a) W_c(i, j0 + jj)
  __shared__ double Bs[kCoreJ][kMaxRank + 1];
  const int tid = threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // pairs (a, b) = tid + 256 k
  for (int j0 = 0; j0 < n2; j0 += kCoreJ) {
    const int jn = n2 - j0 < kCoreJ ? n2 - j0 : kCoreJ;
    for (int q = tid; q < ir * jn; q += 256) {
      const int jj = q / ir, a = q % ir;
      const TA* col = Wc + (int64_t)(j0 + jj) * n1;
      double s = 0.0;
      for (int i = 0; i < n1; ++i) s += A[(int64_t)i * ir + a] * (double)col[i];
      T[a][jj] = s;
    }
    for (int q = tid; q < ir * jn; q += 256) {
      const int jj = q / ir, b = q % ir;
      Bs[jj][b] = B[(int64_t)(j0 + jj) * ir + b];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int p = tid + 256 * k;
      if (p < ir * ir) {
        const int a = p / ir, b = p % ir;
        double s = acc[k];
        for (int jj = 0; jj < jn; ++jj) s += T[a][jj] * Bs[jj][b];
        acc[k] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int p = tid + 256 * k;
    if (p < ir * ir) P[rep * sP + (int64_t)p * ir + c] = acc[k];
  }
}

// The projected core of sparse summaries, P(a, b, c) = sum over the entries
// (x, y, z, v) of v A(x, a) B(y, b) C(z, c), in two steps through the slices
// of the third mode (the entries are stored slice by slice):
//   Wz(a, b) = sum over the entries of slice z of v A(x, a) B(y, b),
//   P(a, b, c) = sum_z C(z, c) Wz(a, b).
// Every product and sum in FP64.  One block per (slice, repetition); the
// slice's entries pass through LDS in chunks with their two factor rows.
constexpr int kCoreE = 64;  // entries per staged chunk

__global__ __launch_bounds__(256) void core_slices_coo_kernel(
    RepSet rs, const int32_t* za, const int32_t* zb, const float* zv, const int64_t* offC,
    int64_t sOffC, const double* Ap, const double* Bp, double* Wz, int64_t sWz) {
  const int z = blockIdx.x, rep = rs.rep0 + blockIdx.y;
  const int ir = rs.R;
  const int64_t o0 = offC[rep * sOffC + z], o1 = offC[rep * sOffC + z + 1];
  const double* A = Ap + rep * rs.sA;
  const double* B = Bp + rep * rs.sB;
  __shared__ double As[kCoreE][kMaxRank + 1];
  __shared__ double Bs[kCoreE][kMaxRank + 1];
  const int tid = threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // pairs (a, b) = tid + 256 k
  for (int64_t e0 = o0; e0 < o1; e0 += kCoreE) {
    const int en = o1 - e0 < kCoreE ? (int)(o1 - e0) : kCoreE;
    for (int q = tid; q < en * ir; q += 256) {
      const int e = q / ir, f = q % ir;
      const double v = (double)zv[e0 + e];
      As[e][f] = v * A[(int64_t)za[e0 + e] * ir + f];
      Bs[e][f] = B[(int64_t)zb[e0 + e] * ir + f];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int p = tid + 256 * k;
      if (p < ir * ir) {
        const int a = p / ir, b = p % ir;
        double s = acc[k];
        for (int e = 0; e < en; ++e) s += As[e][a] * Bs[e][b];
        acc[k] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int p = tid + 256 * k;
    if (p < ir * ir) Wz[rep * sWz + (int64_t)z * ir * ir + p] = acc[k];
  }
}

// P(a, b, c) = sum_z C(z, c) Wz(a, b): one block per (c, repetition), P
// stored [rep][a][b][c] (stride sP) as the dense core kernel writes it
__global__ __launch_bounds__(256) void core_from_slices_kernel(RepSet rs, const double* Wz,
                                                               int64_t sWz, const double* Cp,
                                                               double* P, int64_t sP) {
  const int c = blockIdx.x, rep = rs.rep0 + blockIdx.y;
  const int ir = rs.R, n3 = rs.n3;
  const double* W = Wz + rep * sWz;
  const double* C = Cp + rep * rs.sC;
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int p = tid + 256 * k;
    if (p < ir * ir) {
      double s = 0.0;
      for (int z = 0; z < n3; ++z) s += C[(int64_t)z * ir + c] * W[(int64_t)z * ir * ir + p];
      P[rep * sP + (int64_t)p * ir + c] = s;
    }
  }
}

// G from P by the three small inverses (Gi: GA^-1, GB^-1, GC^-1 at offsets 0,
// sGi, 2 sGi, each [rep][i x i] with stride sG), lambda of the run (stride i),
// then cc[rep].  X1, X2: scratch of the same shape as P.  One block per
// repetition; every stage writes a buffer the block has not read before.
__global__ __launch_bounds__(256) void cc_kernel(RepSet rs, const double* P, double* X1,
                                                double* X2, int64_t sP, const double* Gi,
                                                int64_t sGi, const double* lam, double* cc) {
  const int rep = rs.rep0 + blockIdx.x;
  const int ir = rs.R, n = ir * ir * ir;
  const int tid = threadIdx.x;
  const double* Pr = P + rep * sP;
  double* Y1 = X1 + rep * sP;
  double* Y2 = X2 + rep * sP;
  const double* GA = Gi + rep * rs.sG;
  const double* GB = Gi + sGi + rep * rs.sG;
  const double* GC = Gi + 2 * sGi + rep * rs.sG;
  const double* l = lam + (int64_t)rep * ir;
  // index q = (a * ir + b) * ir + c
  for (int q = tid; q < n; q += 256) {  // Y1(a, e, g) = sum_d GA(a, d) P(d, e, g)
    const int a = q / (ir * ir), eg = q % (ir * ir);
    double s = 0.0;
    for (int d = 0; d < ir; ++d) s += GA[a * ir + d] * Pr[d * ir * ir + eg];
    Y1[q] = s;
  }
  __syncthreads();
  for (int q = tid; q < n; q += 256) {  // Y2(a, b, g) = sum_e GB(b, e) Y1(a, e, g)
    const int a = q / (ir * ir), b = (q / ir) % ir, g = q % ir;
    double s = 0.0;
    for (int e = 0; e < ir; ++e) s += GB[b * ir + e] * Y1[(a * ir + e) * ir + g];
    Y2[q] = s;
  }
  __syncthreads();
  __shared__ double red[256];
  double part = 0.0;
  for (int q = tid; q < n; q += 256) {  // G(a, b, c) = (1 / lam_c) sum_g GC(c, g) Y2(a, b, g)
    const int ab = q / ir, c = q % ir;
    double s = 0.0;
    for (int g = 0; g < ir; ++g) s += GC[c * ir + g] * Y2[ab * ir + g];
    const double G = l[c] != 0.0 ? s / l[c] : 0.0;
    const int a = ab / ir, b = ab % ir;
    const double dlt = (a == b && b == c) ? G - 1.0 : G;
    part += dlt * dlt;
  }
  red[tid] = part;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) cc[rep] = 100.0 * (1.0 - red[0] / ir);
}

// Keep the run when it is the best so far at this rank and the rank counts
// (rank 1 always, else core consistency >= tau): factors copied into the
// kept buffers with rows padded to Rf columns (zeros past i), rnew = i.
__global__ __launch_bounds__(256) void select_kernel(RepSet rs, int Rf, int runs, int j,
                                                    int force, double tau, const double* cc,
                                                    double* bestcc, double* cctab,
                                                    int32_t* rnew, const double* Ap,
                                                    const double* Bp, const double* Cp,
                                                    const double* lamp, double* Ak, double* Bk,
                                                    double* Ck, double* lamk) {
  const int rep = rs.rep0 + blockIdx.x;
  const int ir = rs.R;
  __shared__ int take;
  if (threadIdx.x == 0) {
    const double c = cc[rep];
    cctab[((int64_t)rep * Rf + (ir - 1)) * runs + j] = c;
    const bool better = force || c > bestcc[rep];
    if (better) bestcc[rep] = c;
    take = better && (ir == 1 || c >= tau);
    if (take) rnew[rep] = ir;
  }
  __syncthreads();
  if (!take) return;
  const int64_t na = (int64_t)rs.n1 * Rf, nb = (int64_t)rs.n2 * Rf, nc = (int64_t)rs.n3 * Rf;
  for (int64_t q = threadIdx.x; q < na + nb + nc + Rf; q += 256) {
    if (q < na) {
      const int64_t a = q / Rf;
      const int f = (int)(q % Rf);
      Ak[rep * rs.sA + q] = f < ir ? Ap[rep * rs.sA + a * ir + f] : 0.0;
    } else if (q < na + nb) {
      const int64_t qq = q - na, b = qq / Rf;
      const int f = (int)(qq % Rf);
      Bk[rep * rs.sB + qq] = f < ir ? Bp[rep * rs.sB + b * ir + f] : 0.0;
    } else if (q < na + nb + nc) {
      const int64_t qq = q - na - nb, k = qq / Rf;
      const int f = (int)(qq % Rf);
      Ck[rep * rs.sC + qq] = f < ir ? Cp[rep * rs.sC + k * ir + f] : 0.0;
    } else {
      const int f = (int)(q - na - nb - nc);
      lamk[(int64_t)rep * Rf + f] = f < ir ? lamp[(int64_t)rep * ir + f] : 0.0;
    }
  }
}

}  // namespace

hipError_t launch_core(int prec, const RepSet& rs, const void* W, const double* Ap,
                       const double* Bp, double* P, int64_t sP, hipStream_t s) {
  dim3 grid((unsigned)rs.R, (unsigned)rs.nrep);
  if (prec == kF64)
    core_kernel<double><<<grid, 256, 0, s>>>(rs, (const double*)W, Ap, Bp, P, sP);
  else
    core_kernel<float><<<grid, 256, 0, s>>>(rs, (const float*)W, Ap, Bp, P, sP);
  return hipGetLastError();
}

hipError_t launch_core_coo(const RepSet& rs, const int32_t* za, const int32_t* zb,
                           const float* zv, const int64_t* offC, int64_t sOffC, const double* Ap,
                           const double* Bp, const double* Cp, double* Wz, int64_t sWz,
                           double* P, int64_t sP, hipStream_t s) {
  if (rs.R * rs.R > 1024 || (int64_t)rs.n3 * rs.R * rs.R > sWz) return hipErrorInvalidValue;
  if (rs.n3 > 0) {
    core_slices_coo_kernel<<<dim3((unsigned)rs.n3, (unsigned)rs.nrep), 256, 0, s>>>(
        rs, za, zb, zv, offC, sOffC, Ap, Bp, Wz, sWz);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  core_from_slices_kernel<<<dim3((unsigned)rs.R, (unsigned)rs.nrep), 256, 0, s>>>(rs, Wz, sWz, Cp,
                                                                                 P, sP);
  return hipGetLastError();
}

hipError_t launch_corcondia(const RepSet& rs, const double* P, double* X1, double* X2, int64_t sP,
                            const double* Gi, int64_t sGi, const double* lam, double* cc,
                            hipStream_t s) {
  cc_kernel<<<rs.nrep, 256, 0, s>>>(rs, P, X1, X2, sP, Gi, sGi, lam, cc);
  return hipGetLastError();
}

hipError_t launch_rank_select(const RepSet& rs, int Rf, int runs, int j, bool force, double tau,
                              const double* cc, double* bestcc, double* cctab, int32_t* rnew,
                              const double* Ap, const double* Bp, const double* Cp,
                              const double* lamp, double* Ak, double* Bk, double* Ck,
                              double* lamk, hipStream_t s) {
  select_kernel<<<rs.nrep, 256, 0, s>>>(rs, Rf, runs, j, force ? 1 : 0, tau, cc, bestcc, cctab,
                                        rnew, Ap, Bp, Cp, lamp, Ak, Bk, Ck, lamk);
  return hipGetLastError();
}

}  // namespace sbt
