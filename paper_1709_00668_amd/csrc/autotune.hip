// Launch-shape tuner: process-wide table of shape keys and their chosen
// launch shapes, online trials on the hot path's own launches, and the text
// cache file (see autotune.h and the sbt_autotune_* entry points).
#include "autotune.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/sambaten.h"

namespace sbt {
namespace {

constexpr int kMaxChoices = 8;
constexpr int kMaxDev = 64;
constexpr const char* kCacheHeader = "# sambaten launch-shape cache v1";

struct Key {
  std::string arch;
  int kernel;
  int64_t shape[4];
  bool operator<(const Key& o) const {
    return std::tie(arch, kernel, shape[0], shape[1], shape[2], shape[3]) <
           std::tie(o.arch, o.kernel, o.shape[0], o.shape[1], o.shape[2], o.shape[3]);
  }
};

struct Entry {
  int nchoices = 0;
  int best = -1;  // decided shape, -1 while the trials run
  int issued[kMaxChoices] = {};
  int done[kMaxChoices] = {};
  double cost[kMaxChoices];  // least ms per unit of work over the finished trials
  Entry() {
    for (double& c : cost) c = HUGE_VAL;
  }
};

struct Pending {
  Key key;
  int choice;
  int device;
  double work;
  hipEvent_t a, b;
};

std::mutex g_mu;
std::map<Key, Entry> g_table;
std::vector<Pending> g_pending;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_free[kMaxDev];
std::string g_arch[kMaxDev];
int g_mode = SBT_TUNE_ON;
int g_fixed = 0;

// gcnArchName of the device (e.g. "gfx950:sramecc+:xnack-"), read once; the
// feature suffix is dropped
const std::string& arch_of(int dev) {
  if (g_arch[dev].empty()) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) {
      std::string a = p.gcnArchName;
      g_arch[dev] = a.substr(0, a.find(':'));
    } else {
      g_arch[dev] = "unknown";
    }
  }
  return g_arch[dev];
}

void decide(Entry& e) {
  for (int c = 0; c < e.nchoices; ++c)
    if (e.done[c] < kTuneTrials) return;
  int b = 0;
  for (int c = 1; c < e.nchoices; ++c)
    if (e.cost[c] < e.cost[b]) b = c;
  e.best = b;
}

// Finished trials into the table (caller holds g_mu).
void harvest() {
  size_t w = 0;
  for (size_t i = 0; i < g_pending.size(); ++i) {
    Pending& p = g_pending[i];
    const hipError_t q = hipEventQuery(p.b);
    if (q == hipErrorNotReady) {
      // not a failure, but HIP may keep it as the thread's last error, which
      // the next launch's error check would read
      (void)hipGetLastError();
      g_pending[w++] = p;
      continue;
    }
    auto it = g_table.find(p.key);
    float ms = 0.f;
    const bool ok = q == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess;
    if (ok) {
      g_free[p.device].push_back({p.a, p.b});
    } else {
      (void)hipGetLastError();
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    if (it == g_table.end() || it->second.best >= 0) continue;
    Entry& e = it->second;
    if (!ok) {
      e.best = 0;  // a trial that cannot be read ends the tuning of this key
      continue;
    }
    const double c = (double)ms / p.work;
    if (c < e.cost[p.choice]) e.cost[p.choice] = c;
    ++e.done[p.choice];
    decide(e);
  }
  g_pending.resize(w);
}

}  // namespace

TuneSlot tune_begin(int kernel, int nchoices, const int64_t (&shape)[4], double work,
                    bool may_time, hipStream_t s) {
  TuneSlot slot;
  slot.kernel = kernel;
  for (int i = 0; i < 4; ++i) slot.shape[i] = shape[i];
  slot.work = work > 0 ? work : 1.0;
  if (nchoices < 1 || nchoices > kMaxChoices) return slot;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_mode == SBT_TUNE_OFF) return slot;
  if (g_mode == SBT_TUNE_FIXED) {
    slot.choice = g_fixed < nchoices ? g_fixed : 0;
    return slot;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return slot;
  slot.device = dev;
  if (may_time) harvest();
  Key k{arch_of(dev), kernel, {shape[0], shape[1], shape[2], shape[3]}};
  auto it = g_table.find(k);
  if (it != g_table.end() && it->second.best >= 0) {
    slot.choice = it->second.best < nchoices ? it->second.best : 0;
    return slot;
  }
  if (g_mode != SBT_TUNE_ON || !may_time) return slot;
  Entry& e = g_table[k];
  if (e.nchoices == 0) e.nchoices = nchoices;
  if (e.nchoices != nchoices) return slot;
  // the candidate with the fewest trials so far (the lowest first)
  int c = -1;
  for (int i = 0; i < nchoices; ++i)
    if (e.issued[i] < kTuneTrials && (c < 0 || e.issued[i] < e.issued[c])) c = i;
  if (c < 0) return slot;  // every trial issued, some still running
  hipEvent_t a = nullptr, b = nullptr;
  if (!g_free[dev].empty()) {
    a = g_free[dev].back().first;
    b = g_free[dev].back().second;
    g_free[dev].pop_back();
  } else if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    (void)hipGetLastError();
    return slot;
  }
  if (hipEventRecord(a, s) != hipSuccess) {
    (void)hipGetLastError();
    g_free[dev].push_back({a, b});
    return slot;
  }
  ++e.issued[c];
  slot.choice = c;
  slot.timed = true;
  slot.start = a;
  slot.stop = b;
  return slot;
}

void tune_end(const TuneSlot& slot, hipStream_t s) {
  if (!slot.timed) return;
  std::lock_guard<std::mutex> lock(g_mu);
  Key k{arch_of(slot.device), slot.kernel,
        {slot.shape[0], slot.shape[1], slot.shape[2], slot.shape[3]}};
  if (hipEventRecord(slot.stop, s) != hipSuccess) {
    (void)hipGetLastError();
    auto it = g_table.find(k);
    if (it != g_table.end() && it->second.best < 0) it->second.best = 0;
    return;
  }
  g_pending.push_back(Pending{k, slot.choice, slot.device, slot.work, slot.start, slot.stop});
}

void tune_cancel(const TuneSlot& slot) {
  if (!slot.timed) return;
  std::lock_guard<std::mutex> lock(g_mu);
  Key k{arch_of(slot.device), slot.kernel,
        {slot.shape[0], slot.shape[1], slot.shape[2], slot.shape[3]}};
  auto it = g_table.find(k);
  if (it != g_table.end() && it->second.issued[slot.choice] > 0) --it->second.issued[slot.choice];
  g_free[slot.device].push_back({slot.start, slot.stop});
}

}  // namespace sbt

using namespace sbt;

extern "C" {

sbt_status sbt_autotune_set(int32_t mode, int32_t shape) {
  if (mode < SBT_TUNE_OFF || mode > SBT_TUNE_FIXED) return SBT_E_INVALID;
  if (mode == SBT_TUNE_FIXED && (shape < 0 || shape >= kMaxChoices)) return SBT_E_INVALID;
  std::lock_guard<std::mutex> lock(g_mu);
  g_mode = mode;
  g_fixed = mode == SBT_TUNE_FIXED ? shape : 0;
  return SBT_OK;
}

sbt_status sbt_autotune_clear(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_table.clear();
  // trials still in flight are forgotten; their events are released once
  // they have finished
  size_t w = 0;
  for (size_t i = 0; i < g_pending.size(); ++i) {
    if (hipEventQuery(g_pending[i].b) == hipErrorNotReady) {
      (void)hipGetLastError();
      g_pending[w++] = g_pending[i];
    } else {
      (void)hipGetLastError();
      g_free[g_pending[i].device].push_back({g_pending[i].a, g_pending[i].b});
    }
  }
  g_pending.resize(w);
  return SBT_OK;
}

sbt_status sbt_autotune_count(int64_t* decided, int64_t* tuning) {
  if (!decided || !tuning) return SBT_E_INVALID;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_pending.empty()) harvest();
  int64_t d = 0, u = 0;
  for (const auto& kv : g_table) (kv.second.best >= 0 ? d : u) += 1;
  *decided = d;
  *tuning = u;
  return SBT_OK;
}

sbt_status sbt_autotune_save(const char* path) {
  if (!path) return SBT_E_INVALID;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_pending.empty()) harvest();
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return SBT_E_INVALID;
  bool ok = std::fprintf(f, "%s\n# arch kernel s0 s1 s2 s3 shape choices\n", kCacheHeader) > 0;
  for (const auto& kv : g_table) {
    if (kv.second.best < 0) continue;
    const Key& k = kv.first;
    ok = ok && std::fprintf(f, "%s %d %lld %lld %lld %lld %d %d\n", k.arch.c_str(), k.kernel,
                            (long long)k.shape[0], (long long)k.shape[1], (long long)k.shape[2],
                            (long long)k.shape[3], kv.second.best, kv.second.nchoices) > 0;
  }
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return SBT_E_INVALID;
  }
  return SBT_OK;
}

sbt_status sbt_autotune_load(const char* path) {
  if (!path) return SBT_E_INVALID;
  FILE* f = std::fopen(path, "r");
  if (!f) return SBT_E_INVALID;
  std::vector<std::pair<Key, Entry>> rows;
  char line[512];
  bool ok = std::fgets(line, sizeof line, f) != nullptr &&
            std::strncmp(line, kCacheHeader, std::strlen(kCacheHeader)) == 0;
  while (ok && std::fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    char arch[128];
    int kernel, best, nch;
    long long s0, s1, s2, s3;
    if (std::sscanf(line, "%127s %d %lld %lld %lld %lld %d %d", arch, &kernel, &s0, &s1, &s2,
                    &s3, &best, &nch) != 8 ||
        kernel < 0 || kernel >= kTuneKernels || nch < 1 || nch > kMaxChoices || best < 0 ||
        best >= nch) {
      ok = false;
      break;
    }
    Entry e;
    e.nchoices = nch;
    e.best = best;
    rows.push_back({Key{arch, kernel, {s0, s1, s2, s3}}, e});
  }
  std::fclose(f);
  if (!ok) return SBT_E_INVALID;  // nothing is taken from a malformed file
  std::lock_guard<std::mutex> lock(g_mu);
  for (auto& r : rows) g_table[r.first] = r.second;
  return SBT_OK;
}

}  // extern "C"
