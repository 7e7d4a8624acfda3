// Batched solves (declared and documented in include/pd.h): many grids, of any
// size, field, step count and precision.  Second-order Strang solves of fields
// without a y component share one persistent launch; every other member runs its
// own single-solve launch in the same enqueued (and captured) sequence.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "pd.h"
#include "pd_internal.h"

using namespace pdx;

// Device descriptors of one launch sequence in one allocation that one copy fills:
// the work counter, the solves, the work items and the density jobs, each at a
// 256-byte boundary; and one rho per member.
struct BatchDescriptors {
  unsigned char* d_block = nullptr;
  size_t cap_block = 0;
  unsigned int* d_counter = nullptr;  // the pointers below point into d_block
  BatchSolve* d_solves = nullptr;
  BatchItem* d_items = nullptr;
  DensityJob* d_jobs = nullptr;
  double* d_rho = nullptr;  // one rho per member, in member order
  size_t cap_rho = 0;
};

struct pd_batch_s {
  std::vector<pd_grid> grids;
  int device = -1;
  int points_per_lane = 4;  // fastest measured for FP32, FP64 and mixed batches on MI355X
  int block_threads = 256;

  // Two descriptor sets: the captured whole-solve graph reads its own, which only a
  // new capture writes, so that epochs (pd_batch_step, the autotuner) between two
  // replays cannot change what a replay does.
  BatchDescriptors epoch;
  BatchDescriptors whole;

  // pinned host staging of the descriptors and of rho
  unsigned char* h_stage = nullptr;
  size_t cap_stage = 0;
  double* h_rho = nullptr;
  size_t cap_rho = 0;
  hipEvent_t staged = nullptr;      // recorded after the last upload from h_stage
  hipEvent_t epoch_done = nullptr;  // after the last epoch's launches (its descriptors are free again)
  hipEvent_t whole_done = nullptr;  // after the last replay of the graph
  // the members outside the persistent kernel run on the side stream, forked from
  // and joined back into the caller's stream
  hipStream_t side_stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;

  // captured whole-solve launch
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<pd_grid> graph_grids;
  std::vector<long long> graph_versions;
  int graph_ppl = 0, graph_block = 0;
  int n_items_last = 0;
  int n_separate_last = 0;

  // blocks of the persistent kernel resident at once (its launch size) for the launch
  // shape slots_ppl x slots_block
  long long slots = 0;
  int slots_ppl = 0, slots_block = 0;
};

namespace {

void free_dev(void* p) {
  if (p) (void)hipFree(p);
}

// Grow a buffer to at least n elements (at least doubling, so that a slowly
// rising high-water mark reallocates rarely); the old content is not kept.
template <typename T>
pd_status ensure_device(T** p, size_t* cap, size_t n) {
  if (n <= *cap) return PD_OK;
  const size_t want = std::max(n, *cap * 2);
  free_dev(*p);
  *p = nullptr;
  *cap = 0;
  hipError_t e = device_malloc(reinterpret_cast<void**>(p), want * sizeof(T));
  if (e != hipSuccess) return hip_error(e, "hipMalloc(batch descriptors)");
  *cap = want;
  return PD_OK;
}

pd_status ensure_pinned(unsigned char** p, size_t* cap, size_t n) {
  if (n <= *cap) return PD_OK;
  const size_t want = std::max(n, *cap * 2);
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *cap = 0;
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(p), want, hipHostMallocDefault);
  if (e != hipSuccess) return hip_error(e, "hipHostMalloc(batch staging)");
  *cap = want;
  return PD_OK;
}

void drop_graph(pd_batch b) {
  if (b->exec) {
    (void)hipEventSynchronize(b->whole_done);  // no replay still in flight
    (void)hipGraphExecDestroy(b->exec);
  }
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_grids.clear();
  b->graph_versions.clear();
}

bool graph_current(pd_batch b) {
  if (!b->exec || b->graph_grids != b->grids || b->graph_ppl != b->points_per_lane ||
      b->graph_block != b->block_threads)
    return false;
  for (size_t i = 0; i < b->grids.size(); ++i)
    if (b->graph_versions[i] != b->grids[i]->version) return false;
  return true;
}

struct Plan {
  std::vector<BatchSolve> solves;
  std::vector<BatchItem> items;
  std::vector<DensityJob> jobs;
  std::vector<std::pair<size_t, SolveParams>> separate;  // members run by their own launch
  long long density_tiles = 0;
};

// Blocks of the persistent kernel resident on the device at once for the batch's
// launch shape: the number it is launched with (at most one per work item).
long long persistent_slots(pd_batch b) {
  if (b->slots <= 0 || b->slots_ppl != b->points_per_lane || b->slots_block != b->block_threads) {
    const int per_cu = batch_blocks_per_cu(b->points_per_lane, b->block_threads);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess || cus <= 0)
      cus = 1;
    b->slots = (long long)cus * per_cu;
    b->slots_ppl = b->points_per_lane;
    b->slots_block = b->block_threads;
  }
  return b->slots;
}

// Members the persistent kernel runs: second-order Strang, no y component, with
// fewer tiles than it has resident blocks.  A member with at least that many tiles
// fills the device by itself; its own launch (its grid's shape, blocks scheduled by
// the hardware) then runs at the rate of the solve alone, where the persistent
// kernel's equal items would leave a partly filled last round of blocks (a lone
// 2048^2 member in a 3000-step epoch ran at 0.90 of that rate, against 0.96 in its
// own launch).
bool persistent_member(pd_batch b, pd_grid g) {
  if (g->scheme != PD_SCHEME_STRANG || g->field.elliptic) return false;
  const long long tile = (long long)b->block_threads * b->points_per_lane;
  return (g->grid.points() + tile - 1) / tile < persistent_slots(b);
}

// Descriptors for advancing member i over steps [begin[i], end[i]) (no work
// where begin == end); jobs for the members whose end reaches their last step,
// each also writing its rho to rho_copies[i].
pd_status make_plan(pd_batch b, double* rho_copies, const std::vector<long long>& begin, const std::vector<long long>& end,
                    Plan* plan) {
  const size_t n = b->grids.size();
  plan->solves.resize(n);
  std::vector<size_t> order;
  for (size_t i = 0; i < n; ++i) {
    pd_grid g = b->grids[i];
    void* st = nullptr;
    if (begin[i] < end[i] && (begin[i] > 0 || end[i] < g->field.n_steps)) {
      pd_status s = grid_state_buffer(g, &st);
      if (s != PD_OK) return s;
    }
    plan->solves[i].p = g->solve_params(begin[i], end[i], st);
    plan->solves[i].p.stage = 0;  // the persistent kernel reads field rows with the scalar unit
    plan->solves[i].precision = g->precision;
    plan->solves[i].form = g->form;
    if (begin[i] < end[i]) {
      if (persistent_member(b, g))
        order.push_back(i);
      else
        plan->separate.emplace_back(i, g->solve_params(begin[i], end[i], st));  // its own launch shape
    }
  }
  // Longest first: every tile of a solve costs (end - begin) steps per point.
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t a, size_t c) { return end[a] - begin[a] > end[c] - begin[c]; });
  const long long tile = (long long)b->block_threads * b->points_per_lane;
  plan->items.clear();
  for (size_t i : order) {
    long long npts = b->grids[i]->grid.points();
    for (long long base = 0; base < npts; base += tile) plan->items.push_back(BatchItem{(int)i, 0, base});
  }
  if (plan->items.size() > (size_t)0x7fffffff) return set_error(PD_ERR_INVALID, "too many work items");
  plan->jobs.clear();
  plan->density_tiles = 0;
  for (size_t i = 0; i < n; ++i) {
    pd_grid g = b->grids[i];
    if (!(begin[i] < end[i] && end[i] == g->field.n_steps)) continue;
    DensityJob j{};
    j.n = g->d_n;
    j.npts = g->grid.points();
    j.tile_begin = plan->density_tiles;
    j.partial = g->d_partial;
    j.rho = g->d_rho;
    j.rho_copy = rho_copies + i;
    j.scale = g->density_scale();
    plan->jobs.push_back(j);
    plan->density_tiles += density_partials(j.npts);
  }
  return PD_OK;
}

// Copy the plan's descriptors to the set D through the pinned staging buffer: one
// copy (the counter's slot goes along; a kernel clears it before each launch).
pd_status upload(pd_batch b, BatchDescriptors& D, const Plan& plan, hipStream_t stream) {
  const auto round_up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t a = plan.solves.size() * sizeof(BatchSolve), c = plan.items.size() * sizeof(BatchItem),
               d = plan.jobs.size() * sizeof(DensityJob);
  const size_t o_solves = 256, o_items = o_solves + round_up(a), o_jobs = o_items + round_up(c),
               total = o_jobs + round_up(std::max<size_t>(d, 1));
  pd_status s;
  if ((s = ensure_device(&D.d_block, &D.cap_block, total)) != PD_OK) return s;
  D.d_counter = reinterpret_cast<unsigned int*>(D.d_block);
  D.d_solves = reinterpret_cast<BatchSolve*>(D.d_block + o_solves);
  D.d_items = reinterpret_cast<BatchItem*>(D.d_block + o_items);
  D.d_jobs = reinterpret_cast<DensityJob*>(D.d_block + o_jobs);
  // the previous upload from the staging buffer must have been consumed
  hipError_t e = hipEventSynchronize(b->staged);
  if (e != hipSuccess) return hip_error(e, "hipEventSynchronize");
  if ((s = ensure_pinned(&b->h_stage, &b->cap_stage, total)) != PD_OK) return s;
  std::memset(b->h_stage, 0, total);
  std::memcpy(b->h_stage + o_solves, plan.solves.data(), a);
  std::memcpy(b->h_stage + o_items, plan.items.data(), c);
  std::memcpy(b->h_stage + o_jobs, plan.jobs.data(), d);
  if ((e = hipMemcpyAsync(D.d_block, b->h_stage, o_jobs + d, hipMemcpyHostToDevice, stream)) != hipSuccess)
    return hip_error(e, "hipMemcpyAsync(descriptors)");
  if ((e = hipEventRecord(b->staged, stream)) != hipSuccess) return hip_error(e, "hipEventRecord");
  return PD_OK;
}

// Enqueue one launch sequence on `stream`: the persistent kernel over the plan's
// items and, concurrently on the side stream (forked from and joined back into
// `stream` with events, so the sequence stays one stream-ordered unit and one
// captured graph), the other members' own launches; then the batched density.
// The side launches take the compute units that the persistent kernel's blocks
// leave as its queue drains.
pd_status enqueue(pd_batch b, BatchDescriptors& D, const Plan& plan, hipStream_t stream) {
  hipError_t e;
  const bool fork = !plan.separate.empty();
  if (fork) {
    if ((e = hipEventRecord(b->fork, stream)) != hipSuccess) return hip_error(e, "hipEventRecord(fork)");
    if ((e = hipStreamWaitEvent(b->side_stream, b->fork, 0)) != hipSuccess) return hip_error(e, "hipStreamWaitEvent");
  }
  if (!plan.items.empty()) {
    long long blocks = std::min<long long>(persistent_slots(b), (long long)plan.items.size());
    e = launch_batch(b->points_per_lane, b->block_threads, (int)blocks, D.d_solves, D.d_items,
                     (int)plan.items.size(), D.d_counter, stream);
    if (e != hipSuccess) return hip_error(e, "batch launch");
  }
  // the other members: the single-solve kernels, exactly as a solve alone
  for (const auto& m : plan.separate) {
    pd_grid g = b->grids[m.first];
    e = launch_propagate(g->scheme, g->precision, g->points_per_lane, g->block_threads, g->taylor,
                         g->field.elliptic ? 1 : 0, m.second, b->side_stream);
    if (e != hipSuccess) return hip_error(e, "member launch");
  }
  if (fork) {
    if ((e = hipEventRecord(b->join, b->side_stream)) != hipSuccess) return hip_error(e, "hipEventRecord(join)");
    if ((e = hipStreamWaitEvent(stream, b->join, 0)) != hipSuccess) return hip_error(e, "hipStreamWaitEvent");
  }
  e = launch_batch_density(D.d_jobs, (int)plan.jobs.size(), plan.density_tiles, stream);
  if (e != hipSuccess) return hip_error(e, "batch density launch");
  return PD_OK;
}

pd_status check_members(pd_batch b) {
  if (b->grids.empty()) return set_error(PD_ERR_STATE, "empty batch");
  for (pd_grid g : b->grids) {
    if (!g->field_set) return set_error(PD_ERR_STATE, "a member grid has no field");
    if (g->device != b->device) return set_error(PD_ERR_INVALID, "member grids are on different devices");
  }
  return PD_OK;
}

// Copy the members' rho from the set D to rho_out; only members with completed[i]
// set (all if completed is null) are written.
pd_status copy_rho(pd_batch b, const BatchDescriptors& D, double* rho_out, const std::vector<char>* completed,
                   hipStream_t stream) {
  if (!rho_out) return PD_OK;
  const size_t n = b->grids.size();
  pd_status s = ensure_pinned(reinterpret_cast<unsigned char**>(&b->h_rho), &b->cap_rho, n * sizeof(double));
  if (s != PD_OK) return s;
  hipError_t e = hipMemcpyAsync(b->h_rho, D.d_rho, n * sizeof(double), hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return hip_error(e, "copy of rho");
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_error(e, "hipStreamSynchronize");
  for (size_t i = 0; i < n; ++i)
    if (!completed || (*completed)[i]) rho_out[i] = b->h_rho[i];
  return PD_OK;
}

pd_status prepare_device(pd_batch b) {
  if (b->device >= 0) return PD_OK;
  b->device = b->grids.empty() ? -1 : b->grids[0]->device;
  if (b->device < 0) return set_error(PD_ERR_STATE, "a member grid has no field");
  DeviceScope scope(b->device);
  hipError_t e;
  for (hipEvent_t* ev : {&b->staged, &b->fork, &b->join, &b->epoch_done, &b->whole_done})
    if ((e = hipEventCreateWithFlags(ev, hipEventDisableTiming)) != hipSuccess) return hip_error(e, "hipEventCreate");
  // both streams at the default priority
  if ((e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking)) != hipSuccess)
    return hip_error(e, "hipStreamCreate");
  if ((e = hipStreamCreateWithFlags(&b->side_stream, hipStreamNonBlocking)) != hipSuccess)
    return hip_error(e, "hipStreamCreate");
  return PD_OK;
}

bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Advance member i by up to max_steps[i] steps (one epoch of pd_batch_step / _each).
pd_status step_members(pd_batch b, const long long* max_steps, double* rho_out, int* finished_out, void* stream) {
  pd_status s = PD_OK;
  if (!b->grids.empty() && b->device < 0 && b->grids[0]->field_set && (s = prepare_device(b)) != PD_OK) return s;
  if ((s = check_members(b)) != PD_OK) return s;
  DeviceScope scope(b->device);
  if (!scope.ok) return set_error(PD_ERR_DEVICE, "cannot select device %d", b->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t n = b->grids.size();
  hipError_t e;
  // the epoch descriptors are rewritten below: the previous epoch, on whatever stream
  // it ran, must have finished reading them (the completion events are recorded and
  // waited for outside stream capture only)
  if (fault_now(kFaultLaunch)) return set_error(PD_ERR_DEVICE, "injected launch fault (PD_FAULT)");
  const bool cap = capturing(st);
  if (!cap && (e = hipStreamWaitEvent(st, b->epoch_done, 0)) != hipSuccess) return hip_error(e, "hipStreamWaitEvent");
  if ((s = ensure_device(&b->epoch.d_rho, &b->epoch.cap_rho, n)) != PD_OK) return s;
  std::vector<long long> begin(n), end(n);
  for (size_t i = 0; i < n; ++i) {
    pd_grid g = b->grids[i];
    begin[i] = g->steps_done;
    end[i] = g->steps_done + std::min(g->field.n_steps - g->steps_done, max_steps[i]);
  }
  Plan plan;
  if ((s = make_plan(b, b->epoch.d_rho, begin, end, &plan)) != PD_OK) return s;
  if ((s = upload(b, b->epoch, plan, st)) != PD_OK) return s;
  if ((s = enqueue(b, b->epoch, plan, st)) != PD_OK) return s;
  if (!cap && (e = hipEventRecord(b->epoch_done, st)) != hipSuccess) return hip_error(e, "hipEventRecord");
  for (pd_grid g : b->grids)
    if ((s = mark_use(g, st)) != PD_OK) return s;
  b->n_items_last = (int)plan.items.size();
  b->n_separate_last = (int)plan.separate.size();
  std::vector<char> completed(n, 0);
  for (size_t i = 0; i < n; ++i) {
    completed[i] = begin[i] < end[i] && end[i] == b->grids[i]->field.n_steps;
    b->grids[i]->steps_done = end[i];
  }
  if (finished_out)
    for (size_t i = 0; i < n; ++i) finished_out[i] = b->grids[i]->steps_done == b->grids[i]->field.n_steps;
  return copy_rho(b, b->epoch, rho_out, &completed, st);
}

}  // namespace

extern "C" {

pd_status pd_batch_create(pd_batch* out) {
  if (!out) return set_error(PD_ERR_INVALID, "null output handle pointer");
  *out = new (std::nothrow) pd_batch_s();
  if (!*out) return set_error(PD_ERR_NOMEM, "host allocation failed");
  return PD_OK;
}

pd_status pd_batch_add(pd_batch b, pd_grid g) {
  if (!b || !g) return set_error(PD_ERR_INVALID, "null handle");
  if (std::find(b->grids.begin(), b->grids.end(), g) != b->grids.end())
    return set_error(PD_ERR_INVALID, "grid already in the batch");
  b->grids.push_back(g);
  return PD_OK;
}

pd_status pd_batch_remove(pd_batch b, pd_grid g) {
  if (!b || !g) return set_error(PD_ERR_INVALID, "null handle");
  auto it = std::find(b->grids.begin(), b->grids.end(), g);
  if (it == b->grids.end()) return set_error(PD_ERR_INVALID, "grid is not in the batch");
  b->grids.erase(it);
  // a captured graph may still name the grid: drop it so no replay can reach it
  if (std::find(b->graph_grids.begin(), b->graph_grids.end(), g) != b->graph_grids.end()) {
    DeviceScope scope(b->device);
    drop_graph(b);
  }
  return PD_OK;
}

pd_status pd_batch_clear(pd_batch b) {
  if (!b) return set_error(PD_ERR_INVALID, "null handle");
  b->grids.clear();
  if (b->exec) {
    DeviceScope scope(b->device);
    drop_graph(b);
  }
  return PD_OK;
}

int pd_batch_size(pd_batch b) { return b ? (int)b->grids.size() : 0; }

pd_status pd_batch_members(pd_batch b, pd_grid* out, int capacity) {
  if (!b || (!out && capacity > 0)) return set_error(PD_ERR_INVALID, "null argument");
  if (capacity < (int)b->grids.size()) return set_error(PD_ERR_INVALID, "capacity smaller than the batch");
  for (size_t i = 0; i < b->grids.size(); ++i) out[i] = b->grids[i];
  return PD_OK;
}

pd_status pd_batch_set_launch(pd_batch b, int points_per_lane, int block_threads) {
  if (!b) return set_error(PD_ERR_INVALID, "null handle");
  if (points_per_lane != 0 && points_per_lane != 1 && points_per_lane != 2 && points_per_lane != 4)
    return set_error(PD_ERR_INVALID, "points_per_lane must be 1, 2 or 4");
  if (block_threads != 0 && block_threads != 64 && block_threads != 128 && block_threads != 256)
    return set_error(PD_ERR_INVALID, "block_threads must be 64, 128 or 256");
  if (points_per_lane) b->points_per_lane = points_per_lane;
  if (block_threads) b->block_threads = block_threads;
  return PD_OK;
}

pd_status pd_batch_run(pd_batch b, double* rho_out, void* stream) {
  TraceCall trace("pd_batch_run");
  if (!b) return set_error(PD_ERR_INVALID, "null handle");
  pd_status s = PD_OK;
  if (!b->grids.empty() && b->device < 0 && b->grids[0]->field_set && (s = prepare_device(b)) != PD_OK) return s;
  if ((s = check_members(b)) != PD_OK) return s;
  DeviceScope scope(b->device);
  if (!scope.ok) return set_error(PD_ERR_DEVICE, "cannot select device %d", b->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (fault_now(kFaultLaunch)) return set_error(PD_ERR_DEVICE, "injected launch fault (PD_FAULT)");
  if (!graph_current(b)) {
    drop_graph(b);
    // the graph's descriptors are rewritten below: the last replay must be done with them
    hipError_t e = hipEventSynchronize(b->whole_done);
    if (e != hipSuccess) return hip_error(e, "hipEventSynchronize");
    const size_t n = b->grids.size();
    if ((s = ensure_device(&b->whole.d_rho, &b->whole.cap_rho, n)) != PD_OK) return s;
    std::vector<long long> begin(n, 0), end(n);
    for (size_t i = 0; i < n; ++i) end[i] = b->grids[i]->field.n_steps;
    Plan plan;
    if ((s = make_plan(b, b->whole.d_rho, begin, end, &plan)) != PD_OK) return s;
    if ((s = upload(b, b->whole, plan, b->capture_stream)) != PD_OK) return s;
    if ((e = hipStreamSynchronize(b->capture_stream)) != hipSuccess) return hip_error(e, "hipStreamSynchronize");
    // Capture: counter reset, persistent kernel and the other members' launches on
    // two branches, batched density (kernel nodes only).
    if ((e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_error(e, "hipStreamBeginCapture");
    pd_status se = enqueue(b, b->whole, plan, b->capture_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(b->capture_stream, &graph);
    if (se != PD_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return se;
    }
    if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
    b->graph = graph;
    if ((e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
      drop_graph(b);
      return hip_error(e, "hipGraphInstantiate");
    }
    b->graph_grids = b->grids;
    b->graph_versions.clear();
    for (pd_grid g : b->grids) b->graph_versions.push_back(g->version);
    b->graph_ppl = b->points_per_lane;
    b->graph_block = b->block_threads;
    b->n_items_last = (int)plan.items.size();
    b->n_separate_last = (int)plan.separate.size();
  }
  hipError_t e = hipGraphLaunch(b->exec, st);
  if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
  if (!capturing(st) && (e = hipEventRecord(b->whole_done, st)) != hipSuccess) return hip_error(e, "hipEventRecord");
  for (pd_grid g : b->grids) {
    g->steps_done = g->field.n_steps;
    if ((s = mark_use(g, st)) != PD_OK) return s;
  }
  return copy_rho(b, b->whole, rho_out, nullptr, st);
}

pd_status pd_batch_step(pd_batch b, long long max_steps, double* rho_out, int* finished_out, void* stream) {
  TraceCall trace("pd_batch_step");
  if (!b) return set_error(PD_ERR_INVALID, "null handle");
  if (max_steps < 1) return set_error(PD_ERR_INVALID, "max_steps must be >= 1");
  std::vector<long long> limits(b->grids.size(), max_steps);
  return step_members(b, limits.data(), rho_out, finished_out, stream);
}

pd_status pd_batch_step_each(pd_batch b, const long long* max_steps, double* rho_out, int* finished_out,
                             void* stream) {
  TraceCall trace("pd_batch_step_each");
  if (!b) return set_error(PD_ERR_INVALID, "null handle");
  if (!max_steps && !b->grids.empty()) return set_error(PD_ERR_INVALID, "null max_steps");
  for (size_t i = 0; i < b->grids.size(); ++i)
    if (max_steps[i] < 0) return set_error(PD_ERR_INVALID, "max_steps[%zu] = %lld is negative", i, max_steps[i]);
  return step_members(b, max_steps, rho_out, finished_out, stream);
}

pd_status pd_batch_get_info(pd_batch b, pd_batch_info* out) {
  if (!b || !out) return set_error(PD_ERR_INVALID, "null argument");
  std::memset(out, 0, sizeof *out);
  out->n_grids = (int)b->grids.size();
  out->points_per_lane = b->points_per_lane;
  out->block_threads = b->block_threads;
  out->graph_captured = graph_current(b) ? 1 : 0;
  out->work_items = b->n_items_last;
  out->separate_launches = b->n_separate_last;
  for (pd_grid g : b->grids) {
    out->n_points += g->grid.points();
    out->point_steps += (double)g->grid.points() * (double)g->field.n_steps;
  }
  return PD_OK;
}

void pd_batch_destroy(pd_batch b) {
  if (!b) return;
  if (b->device >= 0) {
    DeviceScope scope(b->device);
    drop_graph(b);
    if (b->staged) (void)hipEventSynchronize(b->staged);
    if (b->epoch_done) (void)hipEventSynchronize(b->epoch_done);
    if (b->whole_done) (void)hipEventSynchronize(b->whole_done);
    for (hipEvent_t ev : {b->staged, b->fork, b->join, b->epoch_done, b->whole_done})
      if (ev) (void)hipEventDestroy(ev);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    if (b->side_stream) (void)hipStreamDestroy(b->side_stream);
    for (BatchDescriptors* D : {&b->epoch, &b->whole}) {
      free_dev(D->d_block);
      free_dev(D->d_rho);
    }
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    if (b->h_rho) (void)hipHostFree(b->h_rho);
  }
  delete b;
}

}  // extern "C"
