// Launch-shape tuner.
//
// Some kernels can be launched in several shapes that compute identical
// results (rows per block, loads in flight, positions per thread: the sums
// of every output run over the same terms in the same order whatever the
// shape).  For such a kernel the tuner picks the shape by measuring the
// launches the hot path makes anyway: the first launches of a new shape key
// take the candidates in turn, each with an event pair recorded around it;
// once every candidate has kTuneTrials finished trials the cheapest one
// (least milliseconds per unit of work, the minimum over its trials) is used
// for that key from then on.  Trials are read back without waiting
// (hipEventQuery), so a launch whose key is still being decided runs in the
// default shape (choice 0).  The table is process-wide, shared by every
// tensor and host thread, and can be written to and read from a text file.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sbt {

enum TuneKernel : int { kTuneGather = 0, kTunePw = 1, kTuneP3 = 2, kTuneKernels = 3 };

constexpr int kTuneTrials = 2;

struct TuneSlot {
  int choice = 0;
  bool timed = false;
  hipEvent_t start = nullptr, stop = nullptr;
  int kernel = 0;
  int64_t shape[4] = {0, 0, 0, 0};
  double work = 1.0;
  int device = 0;
};

// The shape to launch `kernel` in for this key (`nchoices` candidates,
// `work` > 0 the launch's units of work); when the launch is a trial, the
// start event is recorded on `s` here.  may_time = false (e.g. while a
// stream is being captured into a graph) never starts a trial.
TuneSlot tune_begin(int kernel, int nchoices, const int64_t (&shape)[4], double work,
                    bool may_time, hipStream_t s);
// Records the trial's stop event after the launch (no-op for other launches).
void tune_end(const TuneSlot& slot, hipStream_t s);
// In place of tune_end when the launch failed: the trial does not count and
// its events go back to the pool.
void tune_cancel(const TuneSlot& slot);

}  // namespace sbt
