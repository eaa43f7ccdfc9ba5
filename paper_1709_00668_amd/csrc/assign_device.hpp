// Maximum-weight assignment on the GPU (the matching of Sec. 3.1, "Project
// back"), shared by the third-order and the N-mode update.
#pragma once

#include "device_common.hpp"
#include "kernels.hpp"

namespace sbt {

constexpr double kAssignInf = 1e300;

// Maximum-weight perfect assignment on S (R x R, R <= 32) by the Hungarian
// method with potentials, run by one wavefront: lane j owns column j
// (column 0 is the virtual start column), lane r owns the potential of row r.
// Ties in the minimum slack go to the smallest column.  Output: pi[f] =
// column assigned to row f (0-based).
__device__ inline void hungarian_wave(const double (*S)[kMaxRank + 1], int R, int* pi) {
  const int lane = lane_id();
  double u = 0.0;            // potential of row `lane` (rows 1..R)
  double v = 0.0;            // potential of column `lane` (0..R)
  int p = 0;                 // row assigned to column `lane` (0 = none)
  int way = 0;
  for (int i = 1; i <= R; ++i) {
    if (lane == 0) p = i;
    int j0 = 0;
    double minv = kAssignInf;
    bool used = false;
    bool in_tree = false;  // row `lane` reached in this phase
    // every step marks one more column used, so a phase takes at most R steps
    for (int step = 0; step <= R; ++step) {
      if (lane == j0) used = true;
      const int i0 = __shfl(p, j0, kWave);
      if (lane == i0) in_tree = true;
      const double ui0 = __shfl(u, i0, kWave);
      const bool elig = lane >= 1 && lane <= R && !used;
      double cand = kAssignInf;
      int cj = kWave + lane;  // ineligible lanes never win a tie
      if (elig) {
        const double cur = -S[i0 - 1][lane - 1] - ui0 - v;
        if (cur < minv) {
          minv = cur;
          way = j0;
        }
        cand = minv;
        cj = lane;
      }
      // wave argmin of (cand, cj), ties to the smaller column
      double bv = cand;
      int bj = cj;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, kWave);
        const int oj = __shfl_xor(bj, off, kWave);
        if (ov < bv || (ov == bv && oj < bj)) {
          bv = ov;
          bj = oj;
        }
      }
      if (bj >= kWave) break;  // no eligible column: cannot happen for finite S
      const double delta = bv;
      if (lane <= R) {
        if (used)
          v -= delta;
        else if (lane >= 1)
          minv -= delta;
      }
      if (in_tree && lane >= 1 && lane <= R) u += delta;
      j0 = bj;
      if (__shfl(p, j0, kWave) == 0) break;
    }
    // augment along the alternating path back to the virtual column
    for (int step = 0; step <= R && j0 != 0; ++step) {
      const int j1 = __shfl(way, j0, kWave);
      const int pj1 = __shfl(p, j1, kWave);
      if (lane == j0) p = pj1;
      j0 = j1;
    }
  }
  if (lane >= 1 && lane <= R && p >= 1 && p <= R) pi[p - 1] = lane - 1;
}


}  // namespace sbt
