// Streaming ingest (paper Sec. 3.2 pipeline, Sec. 5.1 real-time margin): gulps
// of channelised bytes in arrival order [Time, Channel, Antenna, Polarisation]
// are copied from host memory to one of two device buffers on a copy stream
// while the previous gulp is decimated, transposed and imaged on the context's
// stream.  Buffer i is overwritten only after the front end of the gulp that
// last used it has finished (an event per buffer), so two gulps are in flight.
// A contiguous channel selection (c_step = 1) copies only the selected
// sub-band over the host link (a 2-D copy); a strided one copies the gulp whole
// and selects on the device.
//
// Timing: four events per gulp (copy start / end on the copy stream, compute
// start / end on the context's stream), kept in a ring of kRing gulps and
// folded into running statistics before a slot is reused.  A gulp's
// processing time is the time from the later of (its copy start, the previous
// gulp's end) to its end: the pipeline's own time for that gulp, without the
// time it waited for the producer.  A gulp is over budget when that exceeds
// 90 % of its duration (n_time * sample_s): the margin the paper found
// necessary to keep up without losing packets.
#pragma once

struct epic_pipeline {
  static constexpr int kRing = 64;
  epic_ctx* ctx = nullptr;
  int64_t n_time = 0;
  int c_in = 0, c0 = 0, c_step = 1;
  int dev_c_in = 0, dev_c0 = 0;       // channel geometry of the device copy
  double gulp_ms = 0;
  size_t row_bytes = 0;               // bytes of one sample of the device copy
  DevMem raw[2], ef;
  hipStream_t copy = nullptr;
  hipEvent_t freed[2] = {nullptr, nullptr};
  hipEvent_t ev[kRing][4] = {};
  int64_t pushed = 0, folded = 0;
  // statistics over folded gulps
  int64_t over = 0;
  double sum_t = 0, max_t = 0, sum_copy = 0, sum_comp = 0;
  std::string err;

  epic_status fail(epic_status s, const std::string& m) {
    err = m;
    return s;
  }
};

namespace {

thread_local std::string g_pipeline_init_error;

bool frontend_ok(const epic_ctx* x, int c_in, int c0, int c_step, std::string& m) {
  const int C = x->cfg.n_chan;
  if (c_in < 1 || c0 < 0 || c_step < 1 ||
      (int64_t)c0 + (int64_t)(C - 1) * c_step >= (int64_t)c_in) {
    m = "channel selection c0 + i * c_step (i < n_chan) must lie in [0, c_in)";
    return false;
  }
  return true;
}

void launch_frontend(epic_ctx* x, const uint8_t* raw, int64_t n_time, int c_in, int c0, int c_step,
                     uint8_t* efield) {
  const int A = x->cfg.n_ant, P = x->cfg.n_pol;
  epic::FrontendArgs a;
  a.raw = raw;
  a.efield = efield;
  a.n_rows = n_time * x->cfg.n_chan;
  a.c_in = c_in;
  a.n_chan = x->cfg.n_chan;
  a.c0 = c0;
  a.c_step = c_step;
  a.n_ant = A;
  const bool vec = A % 8 == 0 && (reinterpret_cast<uintptr_t>(raw) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(efield) & 7) == 0;
  const int64_t n = a.n_rows * (vec ? A / 8 : A);
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (P == 2) {
    if (vec) hipLaunchKernelGGL((epic::frontend_kernel<2, 8>), grid, block, 0, x->stream, a);
    else hipLaunchKernelGGL((epic::frontend_kernel<2, 1>), grid, block, 0, x->stream, a);
  } else {
    if (vec) hipLaunchKernelGGL((epic::frontend_kernel<1, 8>), grid, block, 0, x->stream, a);
    else hipLaunchKernelGGL((epic::frontend_kernel<1, 1>), grid, block, 0, x->stream, a);
  }
}

float elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  return ms;
}

// Fold gulp g (complete) into the statistics; slots of g and g - 1 intact.
void pipeline_fold(epic_pipeline* p, int64_t g) {
  hipEvent_t* e = p->ev[g % epic_pipeline::kRing];
  (void)hipEventSynchronize(e[3]);
  float t = elapsed_ms(e[0], e[3]);
  if (g > 0) t = std::min(t, elapsed_ms(p->ev[(g - 1) % epic_pipeline::kRing][3], e[3]));
  p->sum_t += t;
  p->max_t = std::max(p->max_t, (double)t);
  p->sum_copy += elapsed_ms(e[0], e[1]);
  p->sum_comp += elapsed_ms(e[2], e[3]);
  if (t > 0.9 * p->gulp_ms) ++p->over;
  p->folded = g + 1;
}

}  // namespace

extern "C" {

epic_status epic_frontend(epic_ctx* x, const uint8_t* raw, int64_t n_time, int32_t c_in,
                          int32_t c0, int32_t c_step, uint8_t* efield) {
  if (!x) return EPIC_E_INVALID;
  if (!raw || !efield) return x->fail(EPIC_E_INVALID, "NULL device pointer");
  if (n_time <= 0) return x->fail(EPIC_E_INVALID, "n_time must be positive");
  std::string m;
  if (!frontend_ok(x, c_in, c0, c_step, m)) return x->fail(EPIC_E_INVALID, m);
  DeviceGuard guard(x->device);
  (void)hipGetLastError();
  launch_frontend(x, raw, n_time, c_in, c0, c_step, efield);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return x->fail(EPIC_E_LAUNCH, std::string("launch failed: ") + hipGetErrorString(e));
  return EPIC_OK;
}

epic_status epic_pipeline_create(epic_ctx* x, int64_t n_time, int32_t c_in, int32_t c0,
                                 int32_t c_step, double sample_s, epic_pipeline** out) {
  g_pipeline_init_error.clear();
  if (!out) { g_pipeline_init_error = "out is NULL"; return EPIC_E_INVALID; }
  *out = nullptr;
  if (!x) { g_pipeline_init_error = "ctx is NULL"; return EPIC_E_INVALID; }
  std::string m;
  if (n_time <= 0 || !(sample_s > 0) || !std::isfinite(sample_s)) {
    g_pipeline_init_error = "n_time and sample_s must be positive";
    return EPIC_E_INVALID;
  }
  if (!frontend_ok(x, c_in, c0, c_step, m)) { g_pipeline_init_error = m; return EPIC_E_INVALID; }
  epic_pipeline* p = new (std::nothrow) epic_pipeline();
  if (!p) { g_pipeline_init_error = "host allocation failed"; return EPIC_E_NOMEM; }
  p->ctx = x;
  p->n_time = n_time;
  p->c_in = c_in;
  p->c0 = c0;
  p->c_step = c_step;
  p->gulp_ms = (double)n_time * sample_s * 1e3;
  const int C = x->cfg.n_chan;
  const size_t ap = (size_t)x->cfg.n_ant * x->cfg.n_pol;
  // contiguous selection: only the sub-band travels; else the whole gulp
  p->dev_c_in = c_step == 1 ? C : c_in;
  p->dev_c0 = c_step == 1 ? 0 : c0;
  p->row_bytes = (size_t)p->dev_c_in * ap;
  auto bail = [&](epic_status s, const std::string& msg) {
    g_pipeline_init_error = msg;
    epic_pipeline_destroy(p);
    return s;
  };
  DeviceGuard guard(x->device);
  if (!p->raw[0].alloc(p->row_bytes * n_time) || !p->raw[1].alloc(p->row_bytes * n_time) ||
      !p->ef.alloc((size_t)C * ap * n_time))
    return bail(EPIC_E_NOMEM, "pipeline buffer allocation failed");
  if (hipStreamCreateWithFlags(&p->copy, hipStreamNonBlocking) != hipSuccess)
    return bail(EPIC_E_DEVICE, "stream creation failed");
  for (auto& e : p->freed)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
      return bail(EPIC_E_DEVICE, "event creation failed");
  for (auto& r : p->ev)
    for (auto& e : r)
      if (hipEventCreate(&e) != hipSuccess) return bail(EPIC_E_DEVICE, "event creation failed");
  *out = p;
  return EPIC_OK;
}

epic_status epic_pipeline_push(epic_pipeline* p, const uint8_t* host_raw, const float* gains,
                               double* image, int32_t reset) {
  if (!p) return EPIC_E_INVALID;
  epic_ctx* x = p->ctx;
  if (!host_raw || !gains || !image) return p->fail(EPIC_E_INVALID, "NULL pointer");
  if (!x->have_geom) return p->fail(EPIC_E_STATE, "epic_set_antennas has not succeeded");
  if (x->autos && p->n_time > epic::AUTO_SEG_MAX_SAMPLES)
    return p->fail(EPIC_E_UNSUPPORTED, "with EPIC_FLAG_REMOVE_AUTOS a gulp takes at most 2^24 - 1 samples");
  DeviceGuard guard(x->device);
  const int64_t i = p->pushed;
  const int b = (int)(i & 1);
  // the ring slot of gulp i last held gulp i - kRing: fold it (and any
  // earlier gulp still unfolded) while the slot before it is intact
  while (p->folded <= i - epic_pipeline::kRing + 1 && p->folded < i) pipeline_fold(p, p->folded);
  hipEvent_t* e = p->ev[i % epic_pipeline::kRing];
  (void)hipGetLastError();
  bool ok = true;
  if (i >= 2) ok &= hipStreamWaitEvent(p->copy, p->freed[b], 0) == hipSuccess;
  ok &= hipEventRecord(e[0], p->copy) == hipSuccess;
  const size_t ap = (size_t)x->cfg.n_ant * x->cfg.n_pol;
  if (p->c_step == 1)
    ok &= hipMemcpy2DAsync(p->raw[b].p, p->row_bytes, host_raw + (size_t)p->c0 * ap,
                           (size_t)p->c_in * ap, p->row_bytes, (size_t)p->n_time,
                           hipMemcpyHostToDevice, p->copy) == hipSuccess;
  else
    ok &= hipMemcpyAsync(p->raw[b].p, host_raw, p->row_bytes * p->n_time, hipMemcpyHostToDevice,
                         p->copy) == hipSuccess;
  ok &= hipEventRecord(e[1], p->copy) == hipSuccess;
  ok &= hipStreamWaitEvent(x->stream, e[1], 0) == hipSuccess;
  ok &= hipEventRecord(e[2], x->stream) == hipSuccess;
  if (!ok) return p->fail(EPIC_E_DEVICE, "copy or event enqueue failed");
  launch_frontend(x, p->raw[b].as<uint8_t>(), p->n_time, p->dev_c_in, p->dev_c0, p->c_step,
                  p->ef.as<uint8_t>());
  if (hipEventRecord(p->freed[b], x->stream) != hipSuccess)
    return p->fail(EPIC_E_DEVICE, "event record failed");
  const epic_status s = epic_image_accumulate(x, p->ef.as<uint8_t>(), p->n_time, gains, image, reset);
  // the events stay balanced even if imaging was refused
  (void)hipEventRecord(e[3], x->stream);
  ++p->pushed;
  if (s != EPIC_OK) return p->fail(s, x->err);
  return EPIC_OK;
}

epic_status epic_pipeline_report(epic_pipeline* p, epic_pipeline_stats* out) {
  if (!p || !out) return EPIC_E_INVALID;
  DeviceGuard guard(p->ctx->device);
  while (p->folded < p->pushed) pipeline_fold(p, p->folded);
  const int64_t n = p->folded;
  out->gulps = n;
  out->over_budget = p->over;
  out->gulp_ms = p->gulp_ms;
  out->mean_ms = n ? p->sum_t / n : 0.0;
  out->max_ms = p->max_t;
  out->mean_copy_ms = n ? p->sum_copy / n : 0.0;
  out->mean_compute_ms = n ? p->sum_comp / n : 0.0;
  return EPIC_OK;
}

void epic_pipeline_destroy(epic_pipeline* p) {
  if (!p) return;
  {
    DeviceGuard guard(p->ctx ? p->ctx->device : 0);
    if (p->copy) (void)hipStreamSynchronize(p->copy);
    if (p->ctx) (void)hipStreamSynchronize(p->ctx->stream);
    for (auto& e : p->freed)
      if (e) (void)hipEventDestroy(e);
    for (auto& r : p->ev)
      for (auto& e : r)
        if (e) (void)hipEventDestroy(e);
    if (p->copy) (void)hipStreamDestroy(p->copy);
    p->raw[0].reset(); p->raw[1].reset(); p->ef.reset();
  }
  delete p;
}

const char* epic_pipeline_last_error(const epic_pipeline* p) {
  return p ? p->err.c_str() : g_pipeline_init_error.c_str();
}

}  // extern "C"
