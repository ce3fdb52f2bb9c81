// Heterogeneous batch: several imaging configurations (grid size, antennas,
// channels) advanced together.  Each block owns a context whose kernels run on
// a stream of their own; a call forks from the caller's stream to the block
// streams and joins back, so independent blocks share the GPU.  The same
// fork-join can be captured once into a HIP graph and replayed with one launch
// per batch.  The autotuner measures, per block, the persistent-grid size
// (fused path) or the sample batch (staged path), then picks, by timing the
// whole batch, between running every block at its best standalone setting
// concurrently, a work-proportional split of the GPU between concurrent
// blocks, and the blocks one after another (each persistent launch then has
// the whole GPU); the choice is cached in a text file keyed by the device and
// the block shapes.
#pragma once

#include <fstream>
#include <sstream>

struct epic_batch {
  int device = 0;
  hipStream_t main = nullptr;         // the caller's stream (may be the null stream)
  hipStream_t cap = nullptr;          // fork stream used while capturing a graph
  std::vector<epic_ctx*> ctx;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done;
  hipEvent_t fork = nullptr, t0 = nullptr, t1 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool serial = false;                // blocks one after another instead of concurrently
  std::string err;

  epic_status fail(epic_status s, const std::string& m) {
    err = m;
    return s;
  }
};

namespace {

thread_local std::string g_batch_init_error;

epic_status batch_enqueue(epic_batch* b, hipStream_t root, const uint8_t* const* efields,
                          int64_t n_time, const float* const* gains, double* const* images,
                          int32_t reset) {
  if (hipEventRecord(b->fork, root) != hipSuccess)
    return b->fail(EPIC_E_LAUNCH, "event record failed");
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    // concurrent: every block waits for the fork; serial: for the block before
    const hipEvent_t after = (b->serial && i > 0) ? b->done[i - 1] : b->fork;
    if (hipStreamWaitEvent(b->streams[i], after, 0) != hipSuccess)
      return b->fail(EPIC_E_LAUNCH, "stream wait failed");
    const epic_status s = epic_image_accumulate(b->ctx[i], efields[i], n_time, gains[i], images[i], reset);
    if (s != EPIC_OK)
      return b->fail(s, "block " + std::to_string(i) + ": " + b->ctx[i]->err);
    if (hipEventRecord(b->done[i], b->streams[i]) != hipSuccess)
      return b->fail(EPIC_E_LAUNCH, "event record failed");
  }
  for (size_t i = b->serial ? b->ctx.size() - 1 : 0; i < b->ctx.size(); ++i)
    if (hipStreamWaitEvent(root, b->done[i], 0) != hipSuccess)
      return b->fail(EPIC_E_LAUNCH, "stream wait failed");
  return EPIC_OK;
}

epic_status batch_check(epic_batch* b, const uint8_t* const* efields, const float* const* gains,
                        double* const* images, int64_t n_time) {
  if (!efields || !gains || !images) return b->fail(EPIC_E_INVALID, "NULL pointer array");
  if (n_time <= 0) return b->fail(EPIC_E_INVALID, "n_time must be positive");
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    if (!b->ctx[i]->have_geom)
      return b->fail(EPIC_E_STATE, "block " + std::to_string(i) + " has no antennas");
    if (!efields[i] || !gains[i] || !images[i])
      return b->fail(EPIC_E_INVALID, "NULL device pointer for block " + std::to_string(i));
  }
  return EPIC_OK;
}

// Median of reps timings (ms) of fn() enqueued on stream s.
template <typename F>
float time_on(hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps, F fn) {
  std::vector<float> v;
  for (int r = 0; r < reps; ++r) {
    (void)hipEventRecord(e0, s);
    fn();
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    v.push_back(ms);
  }
  std::sort(v.begin(), v.end());
  return v[v.size() / 2];
}

std::string batch_key(const epic_batch* b, int64_t n_time) {
  std::ostringstream k;
  k << "gfx950 v3 T=" << n_time;
  for (const epic_ctx* x : b->ctx)
    k << " [N=" << x->cfg.grid_n << ",P=" << x->cfg.n_pol << ",A=" << x->cfg.n_ant << ",C="
      << x->cfg.n_chan << ",prec=" << x->cfg.precision << ",path=" << (x->fused ? "fused" : "staged")
      << "]";
  return k.str();
}

}  // namespace

extern "C" {

epic_status epic_batch_create(const epic_config* cfgs, int32_t n_blocks, int device,
                              void* hip_stream, epic_batch** out) {
  g_batch_init_error.clear();
  if (!out) { g_batch_init_error = "out is NULL"; return EPIC_E_INVALID; }
  *out = nullptr;
  if (!cfgs || n_blocks < 1 || n_blocks > 64) {
    g_batch_init_error = "n_blocks must be in 1..64";
    return EPIC_E_INVALID;
  }
  epic_batch* b = new (std::nothrow) epic_batch();
  if (!b) { g_batch_init_error = "host allocation failed"; return EPIC_E_NOMEM; }
  b->device = device;
  b->main = static_cast<hipStream_t>(hip_stream);
  auto bail = [&](epic_status s, const std::string& m) {
    g_batch_init_error = m;
    epic_batch_destroy(b);
    return s;
  };
  {
    DeviceGuard guard(device);
    for (int i = 0; i < n_blocks; ++i) {
      hipStream_t st = nullptr;
      hipEvent_t ev = nullptr;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
        return bail(EPIC_E_DEVICE, "stream creation failed");
      b->streams.push_back(st);
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
        return bail(EPIC_E_DEVICE, "event creation failed");
      b->done.push_back(ev);
    }
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
      return bail(EPIC_E_DEVICE, "stream creation failed");
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&b->t0) != hipSuccess || hipEventCreate(&b->t1) != hipSuccess)
      return bail(EPIC_E_DEVICE, "event creation failed");
  }
  for (int i = 0; i < n_blocks; ++i) {
    epic_config c = cfgs[i];
    c.flags &= ~EPIC_FLAG_TIMING;
    epic_ctx* x = nullptr;
    const epic_status s = epic_init(&c, device, b->streams[i], &x);
    if (s != EPIC_OK)
      return bail(s, "block " + std::to_string(i) + ": " + epic_last_error(nullptr));
    b->ctx.push_back(x);
  }
  *out = b;
  return EPIC_OK;
}

epic_status epic_batch_set_antennas(epic_batch* b, int32_t block, const double* xy_m,
                                    const double* freq_hz) {
  if (!b) return EPIC_E_INVALID;
  if (block < 0 || block >= (int32_t)b->ctx.size()) return b->fail(EPIC_E_INVALID, "no such block");
  const epic_status s = epic_set_antennas(b->ctx[block], xy_m, freq_hz);
  if (s != EPIC_OK) return b->fail(s, b->ctx[block]->err);
  return EPIC_OK;
}

epic_status epic_batch_accumulate(epic_batch* b, const uint8_t* const* efields, int64_t n_time,
                                  const float* const* gains, double* const* images, int32_t reset) {
  if (!b) return EPIC_E_INVALID;
  epic_status s = batch_check(b, efields, gains, images, n_time);
  if (s != EPIC_OK) return s;
  DeviceGuard guard(b->device);
  return batch_enqueue(b, b->main, efields, n_time, gains, images, reset);
}

epic_status epic_batch_capture(epic_batch* b, const uint8_t* const* efields, int64_t n_time,
                               const float* const* gains, double* const* images, int32_t reset) {
  if (!b) return EPIC_E_INVALID;
  epic_status s = batch_check(b, efields, gains, images, n_time);
  if (s != EPIC_OK) return s;
  DeviceGuard guard(b->device);
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  // Capture on the batch's own stream (capture is not possible on the null
  // stream); the graph is launched on the caller's stream by epic_batch_replay.
  if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(b->cap, &st) == hipSuccess && st != hipStreamCaptureStatusNone) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(b->cap, &junk);
      if (junk) (void)hipGraphDestroy(junk);
    }
    return b->fail(EPIC_E_LAUNCH, "graph capture could not start");
  }
  s = batch_enqueue(b, b->cap, efields, n_time, gains, images, reset);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (s != EPIC_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess || !g) return b->fail(EPIC_E_LAUNCH, "graph capture failed");
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    b->exec = nullptr;
    return b->fail(EPIC_E_LAUNCH, "graph instantiation failed");
  }
  return EPIC_OK;
}

epic_status epic_batch_replay(epic_batch* b) {
  if (!b) return EPIC_E_INVALID;
  if (!b->exec) return b->fail(EPIC_E_STATE, "no captured graph");
  DeviceGuard guard(b->device);
  if (hipGraphLaunch(b->exec, b->main) != hipSuccess) return b->fail(EPIC_E_LAUNCH, "graph launch failed");
  return EPIC_OK;
}

epic_status epic_batch_tune(epic_batch* b, const uint8_t* const* efields, int64_t n_time,
                            const float* const* gains, double* const* images,
                            const char* cache_path, int32_t* measured) {
  if (!b) return EPIC_E_INVALID;
  epic_status s = batch_check(b, efields, gains, images, n_time);
  if (s != EPIC_OK) return s;
  DeviceGuard guard(b->device);
  const size_t nb = b->ctx.size();
  const std::string key = batch_key(b, n_time);
  if (measured) *measured = 0;
  auto apply = [&](const std::vector<std::pair<int, int>>& plan) {
    for (size_t i = 0; i < nb; ++i) {
      b->ctx[i]->w_override = plan[i].first;
      b->ctx[i]->tb_override = plan[i].second;
    }
  };
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      const size_t sep = line.find(" => ");
      if (sep == std::string::npos || line.compare(0, sep, key) != 0 || sep != key.size()) continue;
      std::vector<std::pair<int, int>> plan;
      std::istringstream vals(line.substr(sep + 4));
      int w = 0, tb = 0, serial = 0;
      char comma = 0;
      if (!(vals >> serial)) continue;
      while (vals >> w >> comma >> tb) plan.push_back({w, tb});
      if (plan.size() == nb) {
        apply(plan);
        b->serial = serial != 0;
        return EPIC_OK;
      }
    }
  }
  if (hipStreamSynchronize(b->main) != hipSuccess) return b->fail(EPIC_E_DEVICE, "stream sync failed");
  // 1. standalone cost of every block for a few settings
  std::vector<std::pair<int, int>> best(nb);
  std::vector<float> best_ms(nb);
  for (size_t i = 0; i < nb; ++i) {
    epic_ctx* x = b->ctx[i];
    std::vector<std::pair<int, int>> cands;
    if (x->fused) {
      for (int den : {1, 2, 4}) cands.push_back({std::max(1, x->fused_w / den), 0});
      cands.push_back({std::max(1, x->fused_w * 3 / 4), 0});
    } else {
      for (int den : {1, 2, 4}) cands.push_back({0, std::max(1, x->tb / den)});
    }
    best_ms[i] = 1e30f;
    for (const auto& c : cands) {
      x->w_override = c.first;
      x->tb_override = c.second;
      s = epic_image_accumulate(x, efields[i], n_time, gains[i], images[i], 1);      // warm
      if (s != EPIC_OK) return b->fail(s, x->err);
      const float ms = time_on(b->streams[i], b->t0, b->t1, 3, [&] {
        (void)epic_image_accumulate(x, efields[i], n_time, gains[i], images[i], 1);
      });
      if (ms < best_ms[i]) { best_ms[i] = ms; best[i] = c; }
    }
  }
  // 2. the whole batch: every block at its standalone best, or the GPU split
  //    between the fused blocks in proportion to their standalone time
  std::vector<std::pair<int, int>> split = best;
  double tot = 0.0;
  for (size_t i = 0; i < nb; ++i) if (b->ctx[i]->fused) tot += best_ms[i];
  for (size_t i = 0; i < nb; ++i)
    if (b->ctx[i]->fused && tot > 0)
      split[i].first = std::max(1, (int)std::lround(b->ctx[i]->fused_w * best_ms[i] / tot));
  std::vector<std::pair<int, int>> chosen = best;
  bool chosen_serial = false;
  float chosen_ms = 1e30f;
  const std::pair<const std::vector<std::pair<int, int>>*, bool> trials[] = {
      {&best, false}, {&split, false}, {&best, true}};
  // each trial is timed as it will run: captured into a graph and replayed
  // (concurrent persistent launches behave differently when launched eagerly)
  for (const auto& tr : trials) {
    apply(*tr.first);
    b->serial = tr.second;
    s = batch_enqueue(b, b->main, efields, n_time, gains, images, 1);
    if (s != EPIC_OK) return s;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    bool graphed = false;
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      const epic_status cs = batch_enqueue(b, b->cap, efields, n_time, gains, images, 1);
      const hipError_t e = hipStreamEndCapture(b->cap, &g);
      graphed = cs == EPIC_OK && e == hipSuccess && g &&
                hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess;
    }
    float ms;
    if (graphed) {
      (void)hipGraphLaunch(ge, b->main);
      ms = time_on(b->main, b->t0, b->t1, 3, [&] { (void)hipGraphLaunch(ge, b->main); });
    } else {
      ms = time_on(b->main, b->t0, b->t1, 3, [&] {
        (void)batch_enqueue(b, b->main, efields, n_time, gains, images, 1);
      });
    }
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    if (ms < chosen_ms) { chosen_ms = ms; chosen = *tr.first; chosen_serial = tr.second; }
  }
  apply(chosen);
  b->serial = chosen_serial;
  if (measured) *measured = 1;
  if (cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    out << key << " => " << (chosen_serial ? 1 : 0);
    for (const auto& p : chosen) out << " " << p.first << "," << p.second;
    out << "\n";
  }
  return EPIC_OK;
}

epic_status epic_batch_plan(const epic_batch* b, int32_t block, int32_t* grid, int32_t* staged_batch) {
  if (!b || block < 0 || block >= (int32_t)b->ctx.size()) return EPIC_E_INVALID;
  const epic_ctx* x = b->ctx[block];
  if (grid) *grid = x->fused ? (x->w_override > 0 ? std::min(x->w_override, x->fused_w) : x->fused_w) : 0;
  if (staged_batch) *staged_batch = x->fused ? 0 : (x->tb_override > 0 ? std::min(x->tb_override, x->tb) : x->tb);
  return EPIC_OK;
}

int32_t epic_batch_serial(const epic_batch* b) { return b && b->serial ? 1 : 0; }

epic_status epic_batch_set_serial(epic_batch* b, int32_t serial) {
  if (!b) return EPIC_E_INVALID;
  b->serial = serial != 0;
  return EPIC_OK;
}

void epic_batch_destroy(epic_batch* b) {
  if (!b) return;
  DeviceGuard guard(b->device);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (epic_ctx* x : b->ctx) epic_destroy(x);
  for (hipStream_t s : b->streams) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  for (hipEvent_t e : b->done) (void)hipEventDestroy(e);
  if (b->cap) {
    (void)hipStreamSynchronize(b->cap);
    (void)hipStreamDestroy(b->cap);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->t0) (void)hipEventDestroy(b->t0);
  if (b->t1) (void)hipEventDestroy(b->t1);
  delete b;
}

const char* epic_batch_last_error(const epic_batch* b) {
  return b ? b->err.c_str() : g_batch_init_error.c_str();
}

}  // extern "C"
