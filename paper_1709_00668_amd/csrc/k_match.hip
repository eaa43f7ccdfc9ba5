// Normalise + match (Sec. 3.1 "Project back", Lemma 1), the zero-entry fill,
// the average of the new rows over the repetitions, the append of C and the
// importance commit (Algorithm 1), and the fit of Sec. 4.2.
#include "device_common.hpp"
#include "kernels.hpp"
#include "assign_device.hpp"

namespace sbt {

namespace {

__device__ inline void pair_fg2(int p, int R, int& f, int& g) {
  f = 0;
  while (p >= R - f) {
    p -= R - f;
    ++f;
  }
  g = f + p;
}

// One block per repetition, on the R x R cross products only (computed over
// the rows beforehand): norms, similarity, assignment, signs, the column
// scales of the matched factors and Gt = (At^T At) .* (Bt^T Bt).
__global__ __launch_bounds__(256) void match_kernel(RepSet rs, MatchArgs m) {
  const int rep = rs.rep0 + blockIdx.x;
  const int R = rs.R, RR = R * R;
  const int tid = threadIdx.x;
  const double* xo = m.xo + (int64_t)rep * 9 * RR;
  const int Rn = m.rnew ? m.rnew[rep] : R;
  __shared__ double S[kMaxRank][kMaxRank + 1];
  __shared__ double nrm[6][kMaxRank];  // A anchor, B anchor, C anchor, A', B', C'(anchor rows)
  __shared__ int pi_s[kMaxRank];
  __shared__ double sA[kMaxRank], sB[kMaxRank];
  if (tid < 6 * R) {
    const int which = tid / R, f = tid % R;
    const double d = xo[(3 + which) * RR + f * R + f];
    nrm[which][f] = sqrt(d > 0.0 ? d : 0.0);
  }
  __syncthreads();
  // similarity: product over the modes of |cosine|
  for (int q = tid; q < RR; q += 256) {
    const int f = q / R, g = q % R;
    const double dA = nrm[0][f] * nrm[3][g], dB = nrm[1][f] * nrm[4][g],
                 dC = nrm[2][f] * nrm[5][g];
    const double cA = dA > 0.0 ? xo[0 * RR + q] / dA : 0.0;
    const double cB = dB > 0.0 ? xo[1 * RR + q] / dB : 0.0;
    const double cC = dC > 0.0 ? xo[2 * RR + q] / dC : 0.0;
    const double sv = fabs(cA) * fabs(cB) * fabs(cC);
    // a non-finite similarity counts as none; so do the sample columns past
    // the summary's rank (GetRank), which leaves R - R_new components unmatched
    S[f][g] = (sv >= 0.0 && g < Rn) ? sv : 0.0;
  }
  __syncthreads();
  if (tid < R) pi_s[tid] = tid;
  __syncthreads();
  if (tid < kWave) hungarian_wave(S, R, pi_s);
  __syncthreads();
  if (tid < R) {
    const int f = tid, g = pi_s[f];
    const double sa = xo[0 * RR + f * R + g] < 0.0 ? -1.0 : 1.0;
    const double sb = xo[1 * RR + f * R + g] < 0.0 ? -1.0 : 1.0;
    // At(:, f) = sigA nA(f) A'(:, g) / ||A'(:, g)||, likewise Bt
    sA[f] = (g < Rn && nrm[3][g] > 0.0) ? sa * nrm[0][f] / nrm[3][g] : 0.0;
    sB[f] = (g < Rn && nrm[4][g] > 0.0) ? sb * nrm[1][f] / nrm[4][g] : 0.0;
    m.scl[(int64_t)rep * 2 * R + f] = sA[f];
    m.scl[(int64_t)rep * 2 * R + R + f] = sB[f];
    m.pi[rep * R + f] = g;
    m.valid[rep * R + f] = (nrm[0][f] > 0.0 && nrm[1][f] > 0.0 && g < Rn) ? 1 : 0;
  }
  __syncthreads();
  for (int q = tid; q < RR; q += 256) {
    const int f = q / R, g = q % R, pf = pi_s[f], pg = pi_s[g];
    const double ga = sA[f] * sA[g] * xo[6 * RR + pf * R + pg];
    const double gb = sB[f] * sB[g] * xo[7 * RR + pf * R + pg];
    // an unmatched component gets a unit diagonal: its rows come out zero
    const bool un = pf >= Rn || pg >= Rn;
    m.Gt[rep * rs.sG + q] = un ? (f == g ? 1.0 : 0.0) : ga * gb;
  }
}

// matched, rescaled sample factors: At(a, f) = scale_A(f) A'(a, pi(f)), Bt likewise
__global__ __launch_bounds__(256) void match_rows_kernel(RepSet rs, MatchArgs m) {
  const int rep = rs.rep0 + blockIdx.y;
  const int R = rs.R;
  const int64_t na = (int64_t)rs.n1 * R, nb = (int64_t)rs.n2 * R;
  const double* scl = m.scl + (int64_t)rep * 2 * R;
  const int32_t* pi = m.pi + rep * R;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < na + nb;
       q += (int64_t)gridDim.x * blockDim.x) {
    if (q < na) {
      const int64_t a = q / R;
      const int f = (int)(q % R);
      m.At[rep * rs.sA + q] = scl[f] * m.Ap[rep * rs.sA + a * R + pi[f]];
    } else {
      const int64_t qq = q - na, b = qq / R;
      const int f = (int)(qq % R);
      m.Bt[rep * rs.sB + qq] = scl[R + f] * m.Bp[rep * rs.sB + b * R + pi[f]];
    }
  }
}

// position of v in the ascending list s[0..n), or -1
__device__ inline int find_sorted(const int32_t* s, int n, int64_t v) {
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

__global__ __launch_bounds__(256) void commit_kernel(CommitArgs c) {
  if (*c.err) return;
  const int R = c.R;
  const int64_t nA = c.I * R, nB = c.J * R, nCo = c.Kold * R, nCn = c.Knew * R;
  const int64_t total = nA + nB + nCo + nCn + c.I + c.J + c.Knew;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = q;
    if (r < nA + nB + nCo) {
      // zero-entry fill: mean over the valid repetitions whose sample covers the row
      double* target;
      const double* src;
      int64_t srow, sstride, off;
      int nsamp;
      int f;
      if (r < nA) {
        target = c.A; src = c.At; sstride = c.sA; off = 0; nsamp = c.n1;
        srow = r / R; f = (int)(r % R);
      } else if (r < nA + nB) {
        r -= nA;
        target = c.B; src = c.Bt; sstride = c.sB; off = c.offJ; nsamp = c.n2;
        srow = r / R; f = (int)(r % R);
      } else {
        r -= nA + nB;
        target = c.C; src = c.Ct; sstride = c.sC; off = c.offK; nsamp = c.n3old;
        srow = r / R; f = (int)(r % R);
      }
      if (target[srow * R + f] != 0.0) continue;
      double acc = 0.0;
      int cnt = 0;
      for (int rep = 0; rep < c.nrep; ++rep) {
        if (!c.valid[rep * R + f]) continue;
        const int p = find_sorted(c.idx + rep * c.idx_stride + off, nsamp, srow);
        if (p < 0) continue;
        acc = acc + src[rep * sstride + (int64_t)p * R + f];
        ++cnt;
      }
      if (cnt) target[srow * R + f] = acc / (double)cnt;
      continue;
    }
    r -= nA + nB + nCo;
    if (r < nCn) {
      const int64_t k = r / R;
      const int f = (int)(r % R);
      double acc = 0.0;
      int cnt = 0;
      for (int rep = 0; rep < c.nrep; ++rep) {
        if (!c.valid[rep * R + f]) continue;
        acc = acc + c.Ct[rep * c.sC + (int64_t)(c.n3old + k) * R + f];
        ++cnt;
      }
      c.C[(c.Kold + k) * R + f] = cnt ? acc / (double)cnt : 0.0;
      continue;
    }
    r -= nCn;
    if (r < c.I) {
      c.w1[r] += c.dw1[r];
      continue;
    }
    r -= c.I;
    if (r < c.J) {
      c.w2[r] += c.dw2[r];
      continue;
    }
    r -= c.J;
    c.w3[c.Kold + r] = c.dw3[r];
  }
}

__global__ __launch_bounds__(256) void fit_final_kernel(const double* G3, const double* C,
                                                       const double* lam, const double* M3,
                                                       const double* nrm, int64_t K, int R,
                                                       double* fit) {
  __shared__ double red[256];
  const double* GA = G3;
  const double* GB = G3 + R * R;
  const double* GC = G3 + 2 * R * R;
  // <X, Xhat> and ||X||^2
  double inner = 0.0, nx = 0.0;
  for (int64_t q = threadIdx.x; q < K * R; q += 256) inner += lam[q % R] * C[q] * M3[q];
  for (int64_t k = threadIdx.x; k < K; k += 256) nx += nrm[k];
  red[threadIdx.x] = inner;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double inner_t = red[0];
  __syncthreads();
  red[threadIdx.x] = nx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double nx_t = red[0];
  if (threadIdx.x == 0) {
    double xh = 0.0;
    for (int f = 0; f < R; ++f)
      for (int g = 0; g < R; ++g)
        xh += lam[f] * lam[g] * GA[f * R + g] * GB[f * R + g] * GC[f * R + g];
    double res2 = nx_t - 2.0 * inner_t + xh;
    if (res2 < 0.0) res2 = 0.0;
    *fit = 1.0 - sqrt(res2) / sqrt(nx_t);
  }
}

__global__ __launch_bounds__(256) void sort_components_kernel(double* A, double* B, double* C,
                                                             double* lam, int64_t I, int64_t J,
                                                             int64_t K, int R) {
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
  double row[kMaxRank];
  for (int64_t r = threadIdx.x; r < I + J + K; r += 256) {
    double* M = r < I ? A + r * R : (r < I + J ? B + (r - I) * R : C + (r - I - J) * R);
    for (int f = 0; f < R; ++f) row[f] = M[f];
    for (int f = 0; f < R; ++f) M[f] = row[perm[f]];
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int f = 0; f < R; ++f) lam[f] = lam_s[perm[f]];
}

// Factor match score of two R-component models (Sec. 4.4) from nine R x R
// cross products: xo[0..2] = A1^T A2, B1^T B2, C1^T C2, xo[3..5] = the Gram
// matrices of model 1, xo[6..8] those of model 2.  Columns are compared after
// scaling to unit norm (the norms go into the weights); the similarity of
// component f of model 1 and g of model 2 is the product over the modes of
// |cosine|; the components are paired by the maximum-weight assignment on it;
// each pair scores its similarity times 1 - |l1 - l2| / max(l1, l2), and the
// score is the mean over the pairs.  One block.
__global__ __launch_bounds__(256) void fms_kernel(const double* xo, const double* lam1,
                                                 const double* lam2, int R, double* out) {
  const int RR = R * R;
  const int tid = threadIdx.x;
  __shared__ double S[kMaxRank][kMaxRank + 1];
  __shared__ double nrm[6][kMaxRank];  // model 1: A, B, C; model 2: A, B, C
  __shared__ int pi_s[kMaxRank];
  __shared__ double part[kMaxRank];
  if (tid < 6 * R) {
    const int which = tid / R, f = tid % R;
    const double d = xo[(3 + which) * RR + f * R + f];
    nrm[which][f] = sqrt(d > 0.0 ? d : 0.0);
  }
  __syncthreads();
  for (int q = tid; q < RR; q += 256) {
    const int f = q / R, g = q % R;
    double sv = 1.0;
    for (int n = 0; n < 3; ++n) {
      const double d = nrm[n][f] * nrm[3 + n][g];
      sv *= d > 0.0 ? fabs(xo[n * RR + q]) / d : 0.0;
    }
    S[f][g] = sv >= 0.0 ? sv : 0.0;
  }
  __syncthreads();
  if (tid < R) pi_s[tid] = tid;
  __syncthreads();
  if (tid < kWave) hungarian_wave(S, R, pi_s);
  __syncthreads();
  if (tid < R) {
    const int f = tid, g = pi_s[f];
    const double l1 = fabs(lam1[f]) * nrm[0][f] * nrm[1][f] * nrm[2][f];
    const double l2 = fabs(lam2[g]) * nrm[3][g] * nrm[4][g] * nrm[5][g];
    const double mx = l1 > l2 ? l1 : l2;
    const double pen = mx > 0.0 ? 1.0 - fabs(l1 - l2) / mx : 1.0;
    part[f] = pen * S[f][g];
  }
  __syncthreads();
  if (tid == 0) {
    double sc = 0.0;
    for (int f = 0; f < R; ++f) sc += part[f];
    *out = sc / R;
  }
}

// Weight of each matched summary component in the current model's units:
// lambda'_g ||C'(anchor rows, g)|| / (||A(I_s, f)|| ||B(J_s, f)|| ||C(K_s, f)||)
// for g = pi(f), from the cross products of the matching (the diagonals of
// A(Is)^T A(Is), B(Js)^T B(Js), C(Ks)^T C(Ks) and of C'^T C' over the anchor
// rows); -1 where the repetition is not valid for f or C(K_s, f) is zero.
__global__ void lambda_hat_kernel(RepSet rs, const double* xo, const double* lamp,
                                  const int32_t* pi, const int32_t* valid, double* lhat) {
  const int R = rs.R;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= rs.nrep * R) return;
  const int rep = rs.rep0 + q / R, f = q % R;
  const int64_t RR = (int64_t)R * R;
  const double* x = xo + (int64_t)rep * 9 * RR;
  const int g = pi[rep * R + f];
  double out = -1.0;
  if (valid[rep * R + f] && g >= 0 && g < R) {
    const double nA2 = x[3 * RR + f * R + f], nB2 = x[4 * RR + f * R + f];
    const double nC2 = x[5 * RR + f * R + f], cp2 = x[8 * RR + g * R + g];
    if (nA2 > 0.0 && nB2 > 0.0 && nC2 > 0.0)
      out = lamp[rep * R + g] * sqrt(cp2) / (sqrt(nA2) * sqrt(nB2) * sqrt(nC2));
  }
  lhat[rep * R + f] = out;
}

// lambda <- (lambda + mean over the repetitions of lhat) / 2 where some
// repetition gives a weight (ascending repetition order); nothing after a
// device error (the commit is predicated the same way)
__global__ void lambda_avg_kernel(const uint32_t* err, double* lam, const double* lhat, int nrep,
                                  int R) {
  const int f = threadIdx.x;
  if (f >= R || *err) return;
  double acc = 0.0;
  int cnt = 0;
  for (int rep = 0; rep < nrep; ++rep) {
    const double v = lhat[rep * R + f];
    if (v >= 0.0) {
      acc = acc + v;
      ++cnt;
    }
  }
  if (cnt) lam[f] = 0.5 * (lam[f] + acc / cnt);
}

}  // namespace

hipError_t launch_lambda_hat(const RepSet& rs, const double* xo, const double* lamp,
                             const int32_t* pi, const int32_t* valid, double* lhat,
                             hipStream_t s) {
  const int n = rs.nrep * rs.R;
  lambda_hat_kernel<<<(n + 255) / 256, 256, 0, s>>>(rs, xo, lamp, pi, valid, lhat);
  return hipGetLastError();
}

hipError_t launch_lambda_avg(const uint32_t* err, double* lam, const double* lhat, int nrep,
                             int R, hipStream_t s) {
  lambda_avg_kernel<<<1, 64, 0, s>>>(err, lam, lhat, nrep, R);
  return hipGetLastError();
}

hipError_t launch_match(const RepSet& rs, const MatchArgs& m, hipStream_t s) {
  match_kernel<<<rs.nrep, 256, 0, s>>>(rs, m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)(rs.n1 + rs.n2) * rs.R;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 512) blocks = 512;
  match_rows_kernel<<<dim3((unsigned)blocks, (unsigned)rs.nrep), 256, 0, s>>>(rs, m);
  return hipGetLastError();
}

hipError_t launch_commit(const CommitArgs& c, hipStream_t s) {
  const int64_t total = (c.I + c.J + c.Kold + c.Knew) * c.R + c.I + c.J + c.Knew;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  commit_kernel<<<(unsigned)blocks, 256, 0, s>>>(c);
  return hipGetLastError();
}

hipError_t launch_fit_final(const double* G3, const double* C, const double* lam,
                            const double* M3, const double* nrm, int64_t K, int R, double* fit,
                            hipStream_t s) {
  fit_final_kernel<<<1, 256, 0, s>>>(G3, C, lam, M3, nrm, K, R, fit);
  return hipGetLastError();
}

hipError_t launch_fms(const double* xo, const double* lam1, const double* lam2, int R,
                      double* out, hipStream_t s) {
  fms_kernel<<<1, 256, 0, s>>>(xo, lam1, lam2, R, out);
  return hipGetLastError();
}

hipError_t launch_sort_components(double* A, double* B, double* C, double* lam, int64_t I,
                                  int64_t J, int64_t K, int R, hipStream_t s) {
  sort_components_kernel<<<1, 256, 0, s>>>(A, B, C, lam, I, J, K, R);
  return hipGetLastError();
}

}  // namespace sbt
