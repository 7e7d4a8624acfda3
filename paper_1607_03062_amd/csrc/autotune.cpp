// Launch-shape autotuner (declared and documented in include/pd.h).
//
// A candidate shape is timed with HIP events on the caller's stream over the
// first `trial_steps` steps of the grid's own solve (chunked propagation, so the
// state goes through device memory exactly as in a long solve); the fastest is
// kept.  Results can be cached in a text file named by PD_AUTOTUNE_CACHE, one
// line per key "arch precision scheme[-xy] form size_class" with the chosen
// points_per_lane, block_threads, table_stage and chunk_steps.
#include <hip/hip_runtime_api.h>

#include <fcntl.h>
#include <unistd.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "pd.h"
#include "pd_internal.h"

using namespace pdx;

namespace {

struct Shape {
  int ppl, block, stage, chunk;
};

std::string arch_name(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

std::string cache_key(pd_grid g) {
  int size_class = (int)std::floor(std::log2((double)g->grid.points()));
  std::ostringstream k;
  static const char* const kSchemes[] = {"strang", "midpoint", "strang4", "midpoint4"};
  static const char* const kPrecisions[] = {"fp64", "fp32", "fp32fast"};
  k << arch_name(g->device) << " " << kPrecisions[g->precision] << " " << kSchemes[g->scheme]
    << (g->field.elliptic ? "-xy" : "") << " " << g->form << " " << size_class;
  return k.str();
}

bool cache_lookup(const std::string& key, Shape* out) {
  const char* path = std::getenv("PD_AUTOTUNE_CACHE");
  if (!path || !*path) return false;
  std::ifstream in(path);
  std::string line;
  bool found = false;
  while (std::getline(in, line)) {
    if (line.compare(0, key.size(), key) != 0 || line.size() <= key.size() || line[key.size()] != '\t') continue;
    std::istringstream v(line.substr(key.size() + 1));
    Shape s{};
    if (v >> s.ppl >> s.block >> s.stage >> s.chunk) {
      *out = s;  // the last entry for a key wins
      found = true;
    }
  }
  return found;
}

// One line per store, written by a single append-mode write so that lines stored at the
// same time by several threads or processes do not interleave.
void cache_store(const std::string& key, const Shape& s, float ms) {
  const char* path = std::getenv("PD_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  std::ostringstream line;
  line << key << '\t' << s.ppl << ' ' << s.block << ' ' << s.stage << ' ' << s.chunk << ' ' << ms << '\n';
  const std::string text = line.str();
  const int fd = ::open(path, O_WRONLY | O_APPEND | O_CREAT, 0644);
  if (fd < 0) return;
  (void)!::write(fd, text.data(), text.size());
  ::close(fd);
}

// Time `run` (which enqueues work on `st`) as the fastest of `reps` repetitions.
template <typename F>
pd_status time_best(F run, hipStream_t st, int reps, float* best_ms) {
  hipEvent_t e0, e1;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_error(e, "hipEventCreate");
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_error(e, "hipEventCreate");
  }
  pd_status s = PD_OK;
  *best_ms = 1e30f;
  for (int r = 0; r < reps && s == PD_OK; ++r) {
    (void)hipEventRecord(e0, st);
    s = run();
    (void)hipEventRecord(e1, st);
    if (s != PD_OK) break;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) {
      s = hip_error(e, "hipEventSynchronize");
      break;
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < *best_ms) *best_ms = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return s;
}

}  // namespace

extern "C" {

pd_status pd_autotune(pd_grid g, long long trial_steps, int use_cache, void* stream) {
  TraceCall trace("pd_autotune");
  if (!g) return set_error(PD_ERR_INVALID, "null handle");
  if (!g->field_set) return set_error(PD_ERR_STATE, "pd_autotune before pd_set_field");
  if (trial_steps < 1) return set_error(PD_ERR_INVALID, "trial_steps must be >= 1");
  DeviceScope scope(g->device);
  if (!scope.ok) return set_error(PD_ERR_DEVICE, "cannot select device %d", g->device);
  const std::string key = cache_key(g);
  Shape best{};
  if (use_cache && cache_lookup(key, &best)) {
    pd_status s = pd_set_launch(g, best.ppl, best.block, best.stage, best.chunk);
    if (s == PD_OK) g->steps_done = 0;
    return s;
  }
  std::vector<Shape> cands;
  for (int ppl : {1, 2, 4})
    for (int block : {64, 256}) {
      cands.push_back({ppl, block, 2, g->chunk_steps});
      if (base_scheme(g->scheme) == PD_SCHEME_STRANG)
        for (int chunk : {256, 1024}) cands.push_back({ppl, block, 1, chunk});
    }
  const long long steps = trial_steps < g->field.n_steps ? trial_steps : g->field.n_steps;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float best_ms = 1e30f;
  for (const Shape& c : cands) {
    pd_status s = pd_set_launch(g, c.ppl, c.block, c.stage, c.chunk);
    if (s != PD_OK) return s;
    float ms = 0;
    s = time_best(
        [&]() {
          g->steps_done = 0;
          return pd_propagate(g, steps, st);
        },
        st, 2, &ms);
    if (s != PD_OK) return s;
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  g->steps_done = 0;
  pd_status s = pd_set_launch(g, best.ppl, best.block, best.stage, best.chunk);
  if (s == PD_OK && use_cache) cache_store(key, best, best_ms);
  return s;
}

pd_status pd_batch_autotune(pd_batch b, long long trial_steps, void* stream) {
  TraceCall trace("pd_batch_autotune");
  if (!b) return set_error(PD_ERR_INVALID, "null handle");
  if (trial_steps < 1) return set_error(PD_ERR_INVALID, "trial_steps must be >= 1");
  const int n = pd_batch_size(b);
  if (n == 0) return set_error(PD_ERR_STATE, "empty batch");
  std::vector<pd_grid> grids(n);
  pd_status s = pd_batch_members(b, grids.data(), n);
  if (s != PD_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int best_ppl = 1, best_block = 256;
  float best_ms = 1e30f;
  for (int ppl : {1, 2, 4})
    for (int block : {64, 128, 256}) {
      if ((s = pd_batch_set_launch(b, ppl, block)) != PD_OK) return s;
      float ms = 0;
      s = time_best(
          [&]() {
            for (pd_grid g : grids) g->steps_done = 0;
            return pd_batch_step(b, trial_steps, nullptr, nullptr, st);
          },
          st, 2, &ms);
      if (s != PD_OK) return s;
      if (ms < best_ms) {
        best_ms = ms;
        best_ppl = ppl;
        best_block = block;
      }
    }
  for (pd_grid g : grids) g->steps_done = 0;
  return pd_batch_set_launch(b, best_ppl, best_block);
}

}  // extern "C"
