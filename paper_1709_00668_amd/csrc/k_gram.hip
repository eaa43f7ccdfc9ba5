// Small cross-product matrices X^T Y (R x R) over many rows, for every
// repetition at once: the Gram matrices of the ALS steps, the anchor and
// sample products of the matching (Sec. 3.1, Lemma 1) and the Gram matrices
// of the fit.  Rows are cut into chunks of kXChunk; one block per (chunk,
// job, repetition) stages its rows in LDS and writes a partial matrix; a
// second kernel adds the partials of each matrix in chunk order.  The work
// is spread over the whole GPU however long the factors are, and the result
// does not depend on the launch shape beyond the fixed chunking.
#include "device_common.hpp"
#include "kernels.hpp"

namespace sbt {

namespace {

constexpr int kXChunk = 64;

__global__ __launch_bounds__(256) void xprod_partial_kernel(XProd xp) {
  __shared__ double Xs[kXChunk][kMaxRank + 1];
  __shared__ double Ys[kXChunk][kMaxRank + 1];
  __shared__ double red[256];
  const int blk = blockIdx.x, j = blockIdx.y, rep = xp.rep0 + blockIdx.z;
  const XJob& jb = xp.job[j];
  const int R = xp.R, RR = R * R;
  const int tid = threadIdx.x;
  const int r0 = blk * kXChunk;
  const int n = jb.rows - r0 < kXChunk ? (jb.rows - r0 > 0 ? jb.rows - r0 : 0) : kXChunk;
  {
    const int32_t* ix = jb.ix ? jb.ix + rep * jb.six : nullptr;
    const int32_t* iy = jb.iy ? jb.iy + rep * jb.siy : nullptr;
    const double* X = jb.X + rep * jb.sX;
    const double* Y = jb.Y + rep * jb.sY;
    for (int q = tid; q < n * R; q += 256) {
      const int i = q / R, f = q % R;
      const int64_t rx = ix ? (int64_t)ix[r0 + i] : (int64_t)(r0 + i);
      const int64_t ry = iy ? (int64_t)iy[r0 + i] : (int64_t)(r0 + i);
      Xs[i][f] = X[rx * R + f];
      Ys[i][f] = Y[ry * R + f];
    }
  }
  __syncthreads();
  double* part = xp.part + (((int64_t)rep * xp.njobs + j) * xp.nblk + blk) * RR;
  if (RR >= 256) {
    for (int p = tid; p < RR; p += 256) {
      const int f = p / R, g = p % R;
      double acc = 0.0;
      for (int i = 0; i < n; ++i) acc += Xs[i][f] * Ys[i][g];
      part[p] = acc;
    }
    return;
  }
  const int nsl = 256 / RR;
  const int p = tid % RR, sl = tid / RR;
  double acc = 0.0;
  if (sl < nsl) {
    const int f = p / R, g = p % R;
    for (int i = sl; i < n; i += nsl) acc += Xs[i][f] * Ys[i][g];
  }
  red[tid] = acc;
  __syncthreads();
  if (tid < RR) {
    double s = 0.0;
    for (int q = 0; q < nsl; ++q) s += red[q * RR + tid];
    part[tid] = s;
  }
}

// one block per 64 entries of a matrix: the four wavefronts take every fourth
// partial, each lane with four independent sums, combined in a fixed order
__global__ __launch_bounds__(256) void xprod_reduce_kernel(XProd xp) {
  __shared__ double red[4][64];
  const int j = blockIdx.y, rep = xp.rep0 + blockIdx.z;
  const int RR = xp.R * xp.R;
  const int nb = (xp.job[j].rows + kXChunk - 1) / kXChunk;
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int p = blockIdx.x * 64 + lane;
  const double* part = xp.part + ((int64_t)rep * xp.njobs + j) * xp.nblk * RR;
  double s = 0.0;
  if (p < RR) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int b = w;
    for (; b + 12 < nb; b += 16) {
      a0 += part[(int64_t)b * RR + p];
      a1 += part[(int64_t)(b + 4) * RR + p];
      a2 += part[(int64_t)(b + 8) * RR + p];
      a3 += part[(int64_t)(b + 12) * RR + p];
    }
    for (; b < nb; b += 4) a0 += part[(int64_t)b * RR + p];
    s = (a0 + a1) + (a2 + a3);
  }
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && p < RR) {
    double* out = xp.out + ((int64_t)rep * xp.njobs + j) * (xp.sOut > 0 ? xp.sOut : RR);
    out[p] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
  }
}

}  // namespace

int xprod_blocks(int max_rows) { return (max_rows + kXChunk - 1) / kXChunk; }

hipError_t launch_xprod(XProd xp, hipStream_t s) {
  int mx = 1;
  for (int j = 0; j < xp.njobs; ++j) mx = xp.job[j].rows > mx ? xp.job[j].rows : mx;
  const int nb = xprod_blocks(mx);
  if (nb > xp.nblk || xp.njobs < 1 || xp.njobs > kXJobs || xp.R < 1 || xp.R > kMaxRank)
    return hipErrorInvalidValue;
  dim3 grid((unsigned)nb, (unsigned)xp.njobs, (unsigned)xp.nrep);
  xprod_partial_kernel<<<grid, 256, 0, s>>>(xp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned tiles = (unsigned)((xp.R * xp.R + 63) / 64);
  xprod_reduce_kernel<<<dim3(tiles, (unsigned)xp.njobs, (unsigned)xp.nrep), 256, 0, s>>>(xp);
  return hipGetLastError();
}

}  // namespace sbt
