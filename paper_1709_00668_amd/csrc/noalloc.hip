// The dense MTTKRP entry point without allocation: the same kernels as
// sbt_mttkrp_dense, with every temporary buffer carved from one fixed device
// array instead of hipMallocAsync, and every constant operand (the identity
// V^-1, unit column scales) written by a kernel instead of a host copy, so
// the call only enqueues kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/sambaten.h"
#include "kernels.hpp"

using namespace sbt;

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

// One copy per GPU, alive until the process ends.  Host code never uses this
// name as an address: the per-device pointer from hipGetSymbolAddress is.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of `scratch`, resolved once per device.
sbt_status scratch_of_current_device(unsigned char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SBT_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return SBT_E_DEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = (unsigned char*)g_scratch_ptr[dev];
  return SBT_OK;
}

// Consecutive 256-byte aligned pieces of the scratch array.
struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t at = off;
    off = (off + (bytes ? bytes : 1) + 255) & ~size_t(255);
    return at;
  }
};

// eye = R x R identity, one = n ones
__global__ void eye_ones_kernel(double* eye, int R, double* one, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < R * R) eye[i] = (i / R == i % R) ? 1.0 : 0.0;
  if (i < n) one[i] = 1.0;
}

#define NA_CK(expr)                                                    \
  do {                                                                 \
    hipError_t e_ = (expr);                                            \
    if (e_ != hipSuccess)                                              \
      return e_ == hipErrorOutOfMemory ? SBT_E_NOMEM : SBT_E_DEVICE;   \
  } while (0)

}  // namespace

extern "C" sbt_status sbt_mttkrp_dense_noalloc(int32_t precision, int32_t schedule,
                                               const void* Z_dev, int64_t n1, int64_t n2,
                                               int64_t n3, int32_t R, const double* U0_dev,
                                               const double* U1_dev, const double* U2_dev,
                                               int32_t mode, double* out_dev, void* stream) {
  if (!Z_dev || !out_dev || R < 1 || R > kMaxRank || n1 < 1 || n2 < 1 || n3 < 1 || mode < 0 ||
      mode > 2 || precision < SBT_P_F64 || precision > SBT_P_BF16 ||
      (schedule != SBT_SCHED_BATCHED && schedule != SBT_SCHED_PLAIN))
    return SBT_E_INVALID;
  if ((mode != 0 && !U0_dev) || (mode != 1 && !U1_dev) || (mode != 2 && !U2_dev))
    return SBT_E_INVALID;
  if (n1 > INT32_MAX || n2 > INT32_MAX || n3 > INT32_MAX) return SBT_E_SHAPE;
  const int prec = precision == SBT_P_F64 ? kF64 : (precision == SBT_P_F32 ? kF32 : kBF16);
  hipStream_t st = (hipStream_t)stream;
  RepSet rs;
  rs.n1 = (int)n1;
  rs.n2 = (int)n2;
  rs.n3 = (int)n3;
  rs.R = R;
  rs.rep0 = 0;
  rs.nrep = 1;
  rs.sZ = n1 * n2 * n3;
  rs.sA = n1 * R;
  rs.sB = n2 * R;
  rs.sC = n3 * R;
  rs.sW = n1 * n2 * R;
  rs.sM = 0;
  rs.sG = (int64_t)R * R;
  rs.nsplit = 1;
  const bool mfma = prec == kBF16 && mfma_supported(rs.n1, rs.n2, R);
  const bool batched = !mfma && prec != kBF16 && schedule == SBT_SCHED_BATCHED;
  if (batched && mode == 2 && !p3_fits(prec, rs.n1, rs.n2, R)) return SBT_E_SHAPE;

  // the pieces this call needs, in the order of sbt_mttkrp_dense's buffers
  Carve cv;
  size_t o_eye = 0, o_one = 0, o_W = 0, o_Zk = 0, o_Zc = 0, o_P = 0, o_ops = 0;
  MfmaLayout L{};
  int ns = 0;
  int64_t sP = 0;
  if (mfma) {
    L = mfma_layout(rs.n1, rs.n2, rs.n3);
    rs.sZ = 0;
    ns = mfma_mode3_splits(rs, L);
    sP = (int64_t)rs.n3 * (R <= 16 ? 16 : 32);
    o_Zk = cv.take(sizeof(uint16_t) * ((L.sZk + 1) & ~int64_t(1)));
    o_Zc = cv.take(sizeof(uint16_t) * L.sZc);
    o_eye = cv.take(sizeof(double) * R * R);
    o_one = cv.take(sizeof(double) * 3 * R);
    o_W = cv.take(sizeof(float) * rs.sW);
    o_P = cv.take(sizeof(float) * ns * sP);
    o_ops = cv.take(sizeof(float) * mfma_operand_floats(L, rs.n2, R));
  } else if (batched) {
    o_eye = cv.take(sizeof(double) * R * R);
    o_one = cv.take(sizeof(double) * 3 * R);
    if (mode != 2) o_W = cv.take((size_t)rs.sW * acc_bytes(prec));
  } else if (mode != 2) {
    o_W = cv.take((size_t)rs.sW * acc_bytes(prec));
  }
  if (cv.off > kScratchBytes) return SBT_E_SHAPE;  // beyond the fixed scratch array

  unsigned char* base = nullptr;
  const sbt_status sb = scratch_of_current_device(&base);
  if (sb != SBT_OK) return sb;
  double* eye = (double*)(base + o_eye);
  double* one = (double*)(base + o_one);
  void* W = base + o_W;
  if (mfma || batched) {
    const int n = R * R > 3 * R ? R * R : 3 * R;
    hipLaunchKernelGGL(eye_ones_kernel, dim3((n + 255) / 256), dim3(256), 0, st, eye, R, one,
                       3 * R);
    NA_CK(hipGetLastError());
  }
  if (mfma) {
    uint16_t* Zk = (uint16_t*)(base + o_Zk);
    uint16_t* Zc = (uint16_t*)(base + o_Zc);
    float* P = (float*)(base + o_P);
    float* ops = (float*)(base + o_ops);
    // the padding of Zk must read zero; the array keeps the previous call's data
    NA_CK(launch_fill_u32((uint32_t*)Zk, (L.sZk + 1) / 2, 0u, st));
    NA_CK(launch_relayout_bf16((const uint16_t*)Z_dev, rs, L, Zk, Zc, st));
    if (mode == 2) {
      NA_CK(launch_p3_mfma(rs, L, ns, Zk, U0_dev, nullptr, U1_dev, nullptr, P, sP, ops, st));
      NA_CK(launch_mode3_finish(rs, ns, P, sP, eye, nullptr, out_dev, 0, st));
    } else {
      NA_CK(launch_pw_mfma(rs, L, Zc, U2_dev, nullptr, (float*)W, ops, st));
      NA_CK(launch_cw(kF32, rs, mode, W, mode == 0 ? U1_dev : U0_dev, one, eye, out_dev, 0,
                      st));
    }
    return SBT_OK;
  }
  if (batched) {
    if (mode == 2) {
      NA_CK(launch_p3(prec, rs, false, Z_dev, U0_dev, one, U1_dev, one, eye, nullptr, out_dev,
                      0, st));
    } else {
      NA_CK(launch_pw(prec, rs, Z_dev, U2_dev, one, W, st));
      NA_CK(launch_cw(prec, rs, mode, W, mode == 0 ? U1_dev : U0_dev, one, eye, out_dev, 0,
                      st));
    }
    return SBT_OK;
  }
  if (mode == 2) {
    NA_CK(launch_p2(prec, rs, Z_dev, U0_dev, U1_dev, out_dev, st));
    return SBT_OK;
  }
  NA_CK(launch_p1(prec, rs, Z_dev, U2_dev, W, st));
  if (mode == 0)
    NA_CK(launch_cw1(prec, rs, W, U1_dev, out_dev, st));
  else
    NA_CK(launch_cw2(prec, rs, W, U0_dev, out_dev, st));
  return SBT_OK;
}
