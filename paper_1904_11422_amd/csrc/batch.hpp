// Heterogeneous batch: several imaging configurations (grid size, antennas,
// channels) advanced together, the paper sizing its gulp, channel count and
// grid by measurement (Sec. 5.1) made a per-batch tuning step.
//
// The blocks' work is cut into launches.  Blocks that run the fused float32
// kernels and share a grid side, polarisation count, sample bytes per thread
// and aperture class form one launch: a single persistent kernel
// (fused_multi_image_kernel / fused_multi_image128_kernel) walks their
// channels as one flattened (channel, time) list, every workgroup taking an
// equal contiguous range of it across block boundaries, followed by one
// reduction that writes every block's image.  A block on another path
// (staged, split precision, autocorrelation removal) is a launch of its own
// through its context.  Each launch runs on a stream of its own; a call forks
// from the caller's stream to the launch streams and joins back, with the
// launches concurrent or one after another.  The same fork-join can be
// captured once into a HIP graph and replayed with one graph launch per
// step.  The autotuner measures, per launch, its shape -- persistent grid
// size (samples per workgroup), float32 block length before a float64 flush,
// and the order in which workgroups are dealt to the XCDs -- or, for a
// single block, its context's grid or staged batch; then it times the whole
// batch with every launch at its best shape concurrently, with the GPU split
// between concurrent launches in proportion to their standalone time, and
// one after another, and caches the winner in a text file keyed by the
// device and the block shapes.
#pragma once

#include <fstream>
#include <memory>
#include <sstream>

// One launch of the batch (see above).
struct BatchLaunch {
  std::vector<int> blocks;            // in channel order
  bool grouped = false;               // a fused_multi launch over `blocks`
  int N = 0, P = 0, gpt = 0;
  bool wide = false;
  int C = 0;                          // channels of all its blocks
  int w_cap = 0;                      // persistent workgroups (occupancy x CUs)
  DevMem partial;                     // grouped: the partial-image slots of w_cap, teams up to kMaxTeam
  int W = 0;                          // tuned grid (0: w_cap)
  int team = 0;                       // tuned team size (0: by n_time)
  int kblock = epic::FusedShape<64>::KBLOCK;
  int xcd = 1;
};

struct epic_batch {
  int device = 0;
  hipStream_t main = nullptr;         // the caller's stream (may be the null stream)
  hipStream_t cap = nullptr;          // fork stream used while capturing a graph
  std::vector<epic_ctx*> ctx;
  std::vector<hipStream_t> streams;   // one per block; a launch uses its first block's
  std::vector<hipEvent_t> done;       // one per launch (at most one per block)
  std::vector<std::unique_ptr<BatchLaunch>> launches;
  hipEvent_t fork = nullptr, t0 = nullptr, t1 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool serial = false;                // launches one after another instead of concurrently
  std::string err;

  epic_status fail(epic_status s, const std::string& m) {
    err = m;
    return s;
  }
};

namespace {

thread_local std::string g_batch_init_error;

template <int N, int P, int GPT, bool WIDE>
int multi_blocks_per_cu() {
  return occupancy_blocks(epic::fused_multi_image_kernel<N, P, GPT, WIDE>, epic::FusedShape<N>::NT);
}

template <int P, int GPT>
int multi128_blocks_per_cu() {
  return occupancy_blocks(epic::fused_multi_image128_kernel<P, GPT>, epic::FusedShape<128>::NT);
}

int multi_blocks_per_cu(int N, int P, int gpt, bool wide) {
#define EPIC_MO(NN, PP, GG, WW) \
  if (N == NN && P == PP && gpt == GG && wide == WW) return multi_blocks_per_cu<NN, PP, GG, WW>();
  EPIC_MO(32, 1, 1, false) EPIC_MO(32, 1, 2, false) EPIC_MO(32, 1, 4, false)
  EPIC_MO(32, 2, 1, false) EPIC_MO(32, 2, 2, false) EPIC_MO(32, 2, 4, false)
  EPIC_MO(64, 1, 1, false) EPIC_MO(64, 1, 2, false) EPIC_MO(64, 1, 4, false)
  EPIC_MO(64, 2, 1, false) EPIC_MO(64, 2, 2, false) EPIC_MO(64, 2, 4, false)
  EPIC_MO(64, 1, 1, true) EPIC_MO(64, 1, 2, true) EPIC_MO(64, 1, 4, true)
  EPIC_MO(64, 2, 1, true) EPIC_MO(64, 2, 2, true) EPIC_MO(64, 2, 4, true)
#undef EPIC_MO
  if (N == 128 && P == 1) return gpt == 1 ? multi128_blocks_per_cu<1, 1>()
                               : gpt == 2 ? multi128_blocks_per_cu<1, 2>() : multi128_blocks_per_cu<1, 4>();
  if (N == 128 && P == 2) return gpt == 1 ? multi128_blocks_per_cu<2, 1>()
                               : gpt == 2 ? multi128_blocks_per_cu<2, 2>() : multi128_blocks_per_cu<2, 4>();
  return 0;
}

bool launch_multi(const BatchLaunch& L, dim3 grid, hipStream_t s, const epic::FusedArgs& a) {
  const dim3 block(fused_threads(L.N));
#define EPIC_ML(NN, PP, GG, WW)                                                                     \
  if (L.N == NN && L.P == PP && L.gpt == GG && L.wide == WW) {                                      \
    hipLaunchKernelGGL((epic::fused_multi_image_kernel<NN, PP, GG, WW>), grid, block, 0, s, a);     \
    return true;                                                                                    \
  }
  EPIC_ML(32, 1, 1, false) EPIC_ML(32, 1, 2, false) EPIC_ML(32, 1, 4, false)
  EPIC_ML(32, 2, 1, false) EPIC_ML(32, 2, 2, false) EPIC_ML(32, 2, 4, false)
  EPIC_ML(64, 1, 1, false) EPIC_ML(64, 1, 2, false) EPIC_ML(64, 1, 4, false)
  EPIC_ML(64, 2, 1, false) EPIC_ML(64, 2, 2, false) EPIC_ML(64, 2, 4, false)
  EPIC_ML(64, 1, 1, true) EPIC_ML(64, 1, 2, true) EPIC_ML(64, 1, 4, true)
  EPIC_ML(64, 2, 1, true) EPIC_ML(64, 2, 2, true) EPIC_ML(64, 2, 4, true)
#undef EPIC_ML
#define EPIC_ML128(PP, GG)                                                                          \
  if (L.N == 128 && L.P == PP && L.gpt == GG) {                                                     \
    hipLaunchKernelGGL((epic::fused_multi_image128_kernel<PP, GG>), grid, block, 0, s, a);          \
    return true;                                                                                    \
  }
  EPIC_ML128(1, 1) EPIC_ML128(1, 2) EPIC_ML128(1, 4) EPIC_ML128(2, 1) EPIC_ML128(2, 2) EPIC_ML128(2, 4)
#undef EPIC_ML128
  return false;
}

// Blocks whose fused kernels one multi-block launch can walk together.
bool groupable(const epic_ctx* x) {
  return x->have_geom && x->fused && x->cfg.precision == EPIC_FP32 && !x->autos && !x->cpx;
}

// Cut the blocks into launches (see the file comment) and size the grouped
// launches' slots.  Called once every block has its geometry.
epic_status batch_plan_launches(epic_batch* b) {
  b->launches.clear();
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    const epic_ctx* x = b->ctx[i];
    const bool gr = groupable(x);
    BatchLaunch* into = nullptr;
    if (gr)
      for (auto& L : b->launches)
        if (L->grouped && L->N == x->cfg.grid_n && L->P == x->cfg.n_pol && L->gpt == x->fused_gpt &&
            L->wide == x->wide && (int)L->blocks.size() < epic::kMaxLaunchBlocks)
          into = L.get();
    if (!into) {
      b->launches.push_back(std::make_unique<BatchLaunch>());
      into = b->launches.back().get();
      into->grouped = gr;
      into->N = x->cfg.grid_n;
      into->P = x->cfg.n_pol;
      into->gpt = x->fused_gpt;
      into->wide = x->wide;
    }
    into->blocks.push_back((int)i);
    into->C += x->cfg.n_chan;
  }
  for (auto& L : b->launches) {
    if (!L->grouped) continue;
    const int bpc = multi_blocks_per_cu(L->N, L->P, L->gpt, L->wide);
    if (bpc <= 0) return b->fail(EPIC_E_UNSUPPORTED, "no multi-block kernel for a group of the batch");
    L->w_cap = bpc * b->ctx[L->blocks[0]]->n_cu;
    const int nacc = L->P == 2 ? 4 : 1;
    const int64_t segs = L->N == 128 ? 2 * (int64_t)L->C : (int64_t)L->C;
    const size_t slots = (size_t)max_slot_count(segs, L->w_cap);
    if (!L->partial.alloc(slots * fused_slot_values(L->N, nacc) * sizeof(double)))
      return b->fail(EPIC_E_NOMEM, "batch partial-image workspace allocation failed");
  }
  return EPIC_OK;
}

// Enqueue a grouped launch on stream s: the multi-block imaging kernel, then
// one reduction writing every block's image.
epic_status enqueue_group(epic_batch* b, const BatchLaunch& L, hipStream_t s, const uint8_t* const* efields,
                          int64_t n_time, const float* const* gains, double* const* images, int32_t reset) {
  const epic_ctx* x0 = b->ctx[L.blocks[0]];
  epic::FusedArgs a{};
  int c0 = 0;
  for (size_t k = 0; k < L.blocks.size(); ++k) {
    const int i = L.blocks[k];
    const epic_ctx* x = b->ctx[i];
    epic::FusedBlock& fb = a.blk[k];
    fb.efield = efields[i];
    fb.gains = reinterpret_cast<const float2*>(gains[i]);
    fb.prog = x->prog.as<uint2>();
    fb.wim = nullptr;
    fb.c0 = c0;
    fb.n_chan = x->cfg.n_chan;
    fb.n_ant = x->cfg.n_ant;
    fb.L = x->L;
    fb.wrows = x->wide ? x->wide_rows : epic::FusedShape<64>::HW;
    c0 += x->cfg.n_chan;
  }
  a.n_blk = (int)L.blocks.size();
  a.twiddle = x0->twiddle.as<float2>();
  a.partial = L.partial.as<double>();
  a.n_time = n_time;
  const int64_t total = (int64_t)L.C * n_time;
  a.total = L.N == 128 ? 2 * total : total;
  const int w_max = L.W > 0 ? std::min(L.W, L.w_cap) : L.w_cap;
  const int w0 = (int)std::min<int64_t>(w_max, a.total);
  a.team = team_for(n_time, L.team);
  while (a.team > 1 && a.team > w0) a.team /= 2;
  a.W = (w0 / a.team) * a.team;
  a.kblock = L.kblock;
  a.xcd = L.xcd;
  if (!launch_multi(L, dim3(a.W), s, a)) return b->fail(EPIC_E_UNSUPPORTED, "no multi-block kernel");
  const int sub = fused_reduce_sub(n_time, a.total, a.W, a.team);
  const int64_t n = (int64_t)L.C * L.N * L.N, ppb = 256 / sub;
  const dim3 rgrid((unsigned)((n + ppb - 1) / ppb)), rblock(256);
  if (L.N == 128) {
    epic::Reduce128Args r{};
    r.partial = a.partial;
    for (int k = 0; k < a.n_blk; ++k) {
      r.image[k] = images[L.blocks[k]];
      r.img_c0[k] = a.blk[k].c0;
    }
    r.n_img = a.n_blk;
    r.n_time = n_time;
    r.total = a.total;
    r.n_chan = L.C;
    r.W = a.W;
    r.team = a.team;
    r.kblock = a.kblock;
    r.reset = reset ? 1 : 0;
    r.sub = sub;
    if (L.P == 2) hipLaunchKernelGGL(epic::reduce_image128_kernel<2>, rgrid, rblock, 0, s, r);
    else hipLaunchKernelGGL(epic::reduce_image128_kernel<1>, rgrid, rblock, 0, s, r);
  } else {
    epic::ReduceArgs r{};
    r.partial = a.partial;
    for (int k = 0; k < a.n_blk; ++k) {
      r.image[k] = images[L.blocks[k]];
      r.img_c0[k] = a.blk[k].c0;
      if (b->ctx[L.blocks[k]]->transposed) r.transposed |= 1 << k;
    }
    r.n_img = a.n_blk;
    r.n_time = n_time;
    r.total = a.total;
    r.n_chan = L.C;
    r.W = a.W;
    r.team = a.team;
    r.kblock = a.kblock;
    r.f32 = 1;
    r.reset = reset ? 1 : 0;
    r.sub = sub;
    r.autos = nullptr;
    r.K = x0->cfg.kernel_support;
    r.autos_cpx = 0;
#define EPIC_MR(NN, PP)                                                                       \
    if (L.N == NN && L.P == PP)                                                               \
      hipLaunchKernelGGL((epic::reduce_image_kernel<NN, PP, true>), rgrid, rblock, 0, s, r);
    EPIC_MR(32, 1) EPIC_MR(32, 2) EPIC_MR(64, 1) EPIC_MR(64, 2)
#undef EPIC_MR
  }
  return EPIC_OK;
}

// Enqueue launch li (grouped, or its single block through its context) on
// its stream.
epic_status enqueue_launch(epic_batch* b, size_t li, const uint8_t* const* efields, int64_t n_time,
                           const float* const* gains, double* const* images, int32_t reset) {
  const BatchLaunch& L = *b->launches[li];
  if (L.grouped)
    return enqueue_group(b, L, b->streams[L.blocks[0]], efields, n_time, gains, images, reset);
  const int i = L.blocks[0];
  const epic_status s = epic_image_accumulate(b->ctx[i], efields[i], n_time, gains[i], images[i], reset);
  if (s != EPIC_OK) return b->fail(s, "block " + std::to_string(i) + ": " + b->ctx[i]->err);
  return EPIC_OK;
}

epic_status batch_enqueue(epic_batch* b, hipStream_t root, const uint8_t* const* efields,
                          int64_t n_time, const float* const* gains, double* const* images,
                          int32_t reset) {
  if (hipEventRecord(b->fork, root) != hipSuccess)
    return b->fail(EPIC_E_LAUNCH, "event record failed");
  const size_t nl = b->launches.size();
  for (size_t li = 0; li < nl; ++li) {
    const hipStream_t st = b->streams[b->launches[li]->blocks[0]];
    // concurrent: every launch waits for the fork; serial: for the launch before
    const hipEvent_t after = (b->serial && li > 0) ? b->done[li - 1] : b->fork;
    if (hipStreamWaitEvent(st, after, 0) != hipSuccess)
      return b->fail(EPIC_E_LAUNCH, "stream wait failed");
    const epic_status s = enqueue_launch(b, li, efields, n_time, gains, images, reset);
    if (s != EPIC_OK) return s;
    if (hipEventRecord(b->done[li], st) != hipSuccess)
      return b->fail(EPIC_E_LAUNCH, "event record failed");
  }
  for (size_t li = b->serial ? nl - 1 : 0; li < nl; ++li)
    if (hipStreamWaitEvent(root, b->done[li], 0) != hipSuccess)
      return b->fail(EPIC_E_LAUNCH, "stream wait failed");
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return b->fail(EPIC_E_LAUNCH, std::string("launch failed: ") + hipGetErrorString(e));
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
  if (b->launches.empty()) return b->fail(EPIC_E_STATE, "the batch has no launch plan");
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
  k << "gfx950 v5 T=" << n_time;
  for (const epic_ctx* x : b->ctx)
    k << " [N=" << x->cfg.grid_n << ",P=" << x->cfg.n_pol << ",A=" << x->cfg.n_ant << ",C="
      << x->cfg.n_chan << ",prec=" << x->cfg.precision << ",flags=" << x->cfg.flags
      << ",path=" << (x->fused ? (x->wide ? "wide" : "fused") : "staged") << "]";
  return k.str();
}

// Launch shape of one launch: grouped {W, team, kblock, xcd}, single block {W, tb}.
struct LaunchShape {
  int W = 0, kblock = epic::FusedShape<64>::KBLOCK, xcd = 1, tb = 0, team = 0;
};

void apply_shape(epic_batch* b, size_t li, const LaunchShape& sh) {
  BatchLaunch& L = *b->launches[li];
  if (L.grouped) {
    L.W = sh.W;
    L.team = sh.team;
    L.kblock = sh.kblock;
    L.xcd = sh.xcd;
  } else {
    epic_ctx* x = b->ctx[L.blocks[0]];
    x->w_override = sh.W;
    x->tb_override = sh.tb;
  }
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
  // once every block has its geometry: cut the launches (a new geometry can
  // change a block's path, so the plan is rebuilt and the graph dropped)
  b->launches.clear();
  DeviceGuard guard(b->device);
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  for (const epic_ctx* x : b->ctx)
    if (!x->have_geom) return EPIC_OK;
  return batch_plan_launches(b);
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
  const size_t nl = b->launches.size();
  const std::string key = batch_key(b, n_time);
  if (measured) *measured = 0;
  auto apply = [&](const std::vector<LaunchShape>& plan) {
    for (size_t li = 0; li < nl; ++li) apply_shape(b, li, plan[li]);
  };
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      const size_t sep = line.find(" => ");
      if (sep == std::string::npos || line.compare(0, sep, key) != 0 || sep != key.size()) continue;
      std::vector<LaunchShape> plan;
      std::istringstream vals(line.substr(sep + 4));
      int serial = 0;
      if (!(vals >> serial)) continue;
      LaunchShape sh;
      char c1 = 0, c2 = 0, c3 = 0, c4 = 0;
      while (vals >> sh.W >> c1 >> sh.kblock >> c2 >> sh.xcd >> c3 >> sh.tb >> c4 >> sh.team) plan.push_back(sh);
      if (plan.size() == nl) {
        apply(plan);
        b->serial = serial != 0;
        return EPIC_OK;
      }
    }
  }
  if (hipStreamSynchronize(b->main) != hipSuccess) return b->fail(EPIC_E_DEVICE, "stream sync failed");
  // 1. standalone cost of every launch for its candidate shapes
  std::vector<LaunchShape> best(nl);
  std::vector<float> best_ms(nl);
  for (size_t li = 0; li < nl; ++li) {
    const BatchLaunch& L = *b->launches[li];
    const hipStream_t st = b->streams[L.blocks[0]];
    std::vector<LaunchShape> cands;
    if (L.grouped) {
      // samples per workgroup (grid w_cap den / 4) x time chunk (team: parts
      // of T / team samples; 0 = the smallest team with parts <= 128), then
      // the float32 block length and the XCD order at the default shape
      for (int den : {4, 3, 2, 1})
        for (int team : {0, 1, 2, 4, 8}) {
          LaunchShape sh;
          sh.W = std::max(1, L.w_cap * den / 4);
          sh.team = team;
          cands.push_back(sh);
        }
      LaunchShape sh;
      sh.W = L.w_cap;
      sh.kblock = epic::FusedShape<64>::KBLOCK / 2;
      cands.push_back(sh);
      sh.kblock = epic::FusedShape<64>::KBLOCK;
      sh.xcd = 0;
      cands.push_back(sh);
    } else {
      const epic_ctx* x = b->ctx[L.blocks[0]];
      if (x->fused) {
        for (int den : {1, 2, 4}) { LaunchShape sh; sh.W = std::max(1, x->fused_w / den); cands.push_back(sh); }
        LaunchShape sh;
        sh.W = std::max(1, x->fused_w * 3 / 4);
        cands.push_back(sh);
      } else {
        for (int den : {1, 2, 4}) { LaunchShape sh; sh.tb = std::max(1, x->tb / den); cands.push_back(sh); }
      }
    }
    best_ms[li] = 1e30f;
    for (const auto& c : cands) {
      apply_shape(b, li, c);
      s = enqueue_launch(b, li, efields, n_time, gains, images, 1);      // warm
      if (s != EPIC_OK) return s;
      const float ms = time_on(st, b->t0, b->t1, 3, [&] {
        (void)enqueue_launch(b, li, efields, n_time, gains, images, 1);
      });
      if (ms < best_ms[li]) { best_ms[li] = ms; best[li] = c; }
    }
    apply_shape(b, li, best[li]);
  }
  // 2. the whole batch: every launch at its standalone best, or the GPU split
  //    between the fused launches in proportion to their standalone time
  std::vector<LaunchShape> split = best;
  double tot = 0.0;
  auto cap_of = [&](size_t li) {
    const BatchLaunch& L = *b->launches[li];
    if (L.grouped) return L.w_cap;
    const epic_ctx* x = b->ctx[L.blocks[0]];
    return x->fused ? x->fused_w : 0;
  };
  for (size_t li = 0; li < nl; ++li) if (cap_of(li) > 0) tot += best_ms[li];
  for (size_t li = 0; li < nl; ++li)
    if (cap_of(li) > 0 && tot > 0)
      split[li].W = std::max(1, (int)std::lround(cap_of(li) * best_ms[li] / tot));
  std::vector<LaunchShape> chosen = best;
  bool chosen_serial = false;
  float chosen_ms = 1e30f;
  const std::pair<const std::vector<LaunchShape>*, bool> trials[] = {
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
    for (const auto& p : chosen) out << " " << p.W << "," << p.kblock << "," << p.xcd << "," << p.tb << "," << p.team;
    out << "\n";
  }
  return EPIC_OK;
}

epic_status epic_batch_plan(const epic_batch* b, int32_t block, int32_t* grid, int32_t* staged_batch) {
  if (!b || block < 0 || block >= (int32_t)b->ctx.size()) return EPIC_E_INVALID;
  const epic_ctx* x = b->ctx[block];
  for (const auto& L : b->launches)
    if (L->grouped && std::find(L->blocks.begin(), L->blocks.end(), block) != L->blocks.end()) {
      if (grid) *grid = L->W > 0 ? std::min(L->W, L->w_cap) : L->w_cap;
      if (staged_batch) *staged_batch = 0;
      return EPIC_OK;
    }
  if (grid) *grid = x->fused ? (x->w_override > 0 ? std::min(x->w_override, x->fused_w) : x->fused_w) : 0;
  if (staged_batch) *staged_batch = x->fused ? 0 : (x->tb_override > 0 ? std::min(x->tb_override, x->tb) : x->tb);
  return EPIC_OK;
}

epic_status epic_batch_launch_plan(const epic_batch* b, int32_t block, int32_t* launch, int32_t* n_blocks,
                                   int32_t* team, int32_t* kblock, int32_t* xcd) {
  if (!b || block < 0 || block >= (int32_t)b->ctx.size()) return EPIC_E_INVALID;
  for (size_t li = 0; li < b->launches.size(); ++li) {
    const BatchLaunch& L = *b->launches[li];
    if (std::find(L.blocks.begin(), L.blocks.end(), block) == L.blocks.end()) continue;
    if (launch) *launch = (int32_t)li;
    if (n_blocks) *n_blocks = L.grouped ? (int32_t)L.blocks.size() : 0;
    if (team) *team = L.grouped ? L.team : 0;
    if (kblock) *kblock = L.grouped ? L.kblock : epic::FusedShape<64>::KBLOCK;
    if (xcd) *xcd = L.grouped ? L.xcd : 0;
    return EPIC_OK;
  }
  return EPIC_E_STATE;
}

epic_status epic_batch_set_launch(epic_batch* b, int32_t launch, int32_t grid, int32_t team, int32_t kblock,
                                  int32_t xcd) {
  if (!b) return EPIC_E_INVALID;
  if (launch < 0 || launch >= (int32_t)b->launches.size()) return b->fail(EPIC_E_INVALID, "no such launch");
  BatchLaunch& L = *b->launches[launch];
  if (!L.grouped) return b->fail(EPIC_E_UNSUPPORTED, "a block running alone has no grouped launch shape");
  if (grid < 0 || kblock < 1 || kblock > epic::FusedShape<64>::KBLOCK ||
      !(team == 0 || team == 1 || team == 2 || team == 4 || team == 8))
    return b->fail(EPIC_E_INVALID, "grid must be >= 0, team 0, 1, 2, 4 or 8 and kblock in 1..128");
  L.W = grid;
  L.team = team;
  L.kblock = kblock;
  L.xcd = xcd ? 1 : 0;
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
  for (hipStream_t s : b->streams) (void)hipStreamSynchronize(s);
  b->launches.clear();
  for (epic_ctx* x : b->ctx) epic_destroy(x);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
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
