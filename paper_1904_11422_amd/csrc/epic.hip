// Host side of the C ABI declared in include/epic.h: context, argument
// validation, float64 geometry precompute, table upload and kernel launches.
#include "epic.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <queue>
#include <string>
#include <utility>
#include <vector>

#include "dft.hpp"
#include "fused.hpp"
#include "staged.hpp"
#include "adjoint.hpp"
#include "split.hpp"
#include "fused128.hpp"
#include "adjoint128.hpp"
#include "autos.hpp"
#include "frontend.hpp"
#include "post.hpp"

namespace {

constexpr double kC0 = 299792458.0;
thread_local std::string g_init_error;

struct DevMem {
  void* p = nullptr;
  size_t bytes = 0;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  ~DevMem() { reset(); }
  void reset() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  bool alloc(size_t n) {
    reset();
    if (n == 0) n = 16;
    if (hipMalloc(&p, n) != hipSuccess) { p = nullptr; return false; }
    bytes = n;
    return true;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// Host-side per-channel geometry (float64 maths, float32 weights).
struct Geometry {
  int C = 0, A = 0, KK = 0;
  std::vector<int> cell;              // [C][A][KK] j*N + i on the centred grid
  std::vector<int> tcell;             // [C][A][KK] the same taps translated to start at (0, 0)
  std::vector<float> w;               // [C][A][KK] (real parts for complex kernels)
  std::vector<float> wi;              // [C][A][KK] imaginary parts, empty for real kernels
  bool fits_half = true;              // every channel's taps fit an N/2 x N/2 block
  bool fits_wide = true;              // ... a 3N/4 x 3N/4 block (the wide fused variant,
                                      // whose rows orient_wide then trims)
  int ext_j = 0, ext_i = 0;           // largest extent of a channel's taps in rows, columns
  // the wide block (orient_wide): rows transformed in the row pass (a multiple
  // of 8, at least N/2), and whether tcell holds the taps transposed (row and
  // column swapped, so that the narrower extent lies along the rows)
  int wide_rows = 0;
  bool transposed = false;
};

// Orientation and row count of the wide block (N = 64, an aperture wider
// than N/2): the row pass transforms one line per aperture row and
// polarisation, the column pass all N columns, so the narrower extent goes
// along the rows.  The rows become the smallest multiple of 8 (at least N/2)
// that holds it; the block keeps 3N/4 columns.  Rotating the grid by a
// transposition transposes each image, which the reduction and the gradient
// table undo.
void orient_wide(Geometry& g, int N) {
  g.transposed = g.ext_j > g.ext_i;
  const int narrow = std::min(g.ext_j, g.ext_i);
  g.wide_rows = std::max(N / 2, (narrow + 7) / 8 * 8);
  if (g.transposed)
    for (int& t : g.tcell) t = (t % N) * N + t / N;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace

// Partial-image slots of epic_image_accumulate_noalloc: a static device array,
// so that call allocates nothing.  Every device the library runs on holds its
// own copy for the life of the process.  Host code never passes `scratch`
// itself to a kernel (on the host the name is a stand-in, not a device
// address): epic_init looks up each device's address once and keeps it.
constexpr size_t kScratchBytes = (size_t)96 << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_tried[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device;
// looked up on the first call per device, nullptr if that failed.
void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_tried[device]) {
    g_scratch_tried[device] = true;
    void* ptr = nullptr;
    g_scratch_err[device] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_ptr[device] = g_scratch_err[device] == hipSuccess ? ptr : nullptr;
  }
  return g_scratch_ptr[device];
}

}  // namespace

struct epic_ctx {
  epic_config cfg{};
  void* scratch = nullptr;            // this device's address of `scratch` (no-allocation call)
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int nprod = 1, nacc = 1, PA = 0;
  int n_cu = 0;

  // path selection: fused_ok = the configuration has fused kernels (decided at
  // init); fused = the current geometry uses them (decided at set_antennas)
  bool fused_ok = true, fused = false;
  bool wide = false;                  // fused, with the wide variant (N = 64, apertures up to 3N/4)
  int fused_w_wide = 0, fused_w_wide_cpx = 0, adj_w_wide = 0, adj_w_wide_cpx = 0;
  int wide_rows = 0;                  // rows of the wide block (32, 40 or 48)
  bool transposed = false;            // the fused programs image the transposed aperture
  int fused_gpt = 1;
  int fused_w = 0;                    // persistent workgroups (upper bound)
  int w_override = 0;                 // tuned grid size (0: fused_w)
  int team_override = 0;              // team size of the fused imaging launch (0: by n_time)
  int tb_override = 0;                // tuned staged batch (0: tb)
  int adj_w = 0;
  const char* last_kernel = "none";

  // tables
  bool have_geom = false;
  int L = 0;
  DevMem prog, twiddle, taps;
  DevMem prog_im, taps_im;            // imaginary weights of programs and taps (complex kernels)
  bool cpx = false;                   // the geometry carries complex kernels
  int fused_w_cpx = 0, adj_w_cpx = 0; // persistent grids of the complex-kernel variants
  DevMem csr_off, csr_ent, csr_im;
  DevMem taper, tmax;                 // kernel taper [C][N][N] (fftshifted) and its maxima [C]
  int nnz = 0;

  // workspace
  DevMem partial;                     // fused: [(W + C - 1)][nacc][N*N] thread-major
  DevMem gpartial;                    // adjoint: [(W + C - 1)][P*A] complex f64
  DevMem gtab;                        // adjoint: [C][S][NT] float4 upstream gradient at owned pixels
  DevMem st_e, st_grid, st_acc;       // staged
  int tb = 0;
  // split-precision matrix form
  DevMem sp_beta, sp_betamax, sp_bmat, sp_scale, sp_partial;
  int sp_apad = 0, sp_qb = 0, sp_max_chunks = 0;
  int sp_wgs_per_cu[2] = {1, 1};     // resident split-image workgroups per CU (byte, 8-byte loads)

  // timing
  bool timing = false, timed = false;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  // the main kernels of the last kTimingRing timed calls: event pairs
  // [slot][begin, end], slot = call index mod kTimingRing
  static constexpr int kTimingRing = 256;
  std::vector<hipEvent_t> ring;
  int64_t ring_calls = 0;
  bool autos_timed = false;

  // autocorrelation removal (EPIC_FLAG_REMOVE_AUTOS)
  bool autos = false;
  int au_nseg_cap = 0;
  int au_bpc[2] = {1, 1};             // resident auto_sum_kernel workgroups per CU (VEC 1, 4)
  DevMem au_part;                     // [nseg][C][A][NQ] int32 sums per time segment
  DevMem au_tab;                      // [C][(2K-1)^2][NQ] float64
  DevMem au_sums;                     // [C][A][NQ] float64 (exact integer sums)
  DevMem au_w;                        // [C][A][K*K] float32 tap weights
  DevMem au_wi;                       // [C][A][K*K] imaginary parts (complex kernels)
  DevMem au_hat;                      // [C][(2K-1)^2][NQ] float64 upstream-gradient sums
  DevMem au_gauto;                    // [C][P][A] complex float64 gradient of the removed term

  epic_status fail(epic_status s, const std::string& m) {
    err = m;
    return s;
  }
};

namespace {

// Timing events around a call's main kernel (EPIC_FLAG_TIMING): the pair
// that epic_last_timing reads, and the call's slot of the ring that
// epic_timing_history reads.
void mark_main_begin(epic_ctx* x) {
  if (!x->timing) return;
  (void)hipEventRecord(x->ev[0], x->stream);
  (void)hipEventRecord(x->ring[2 * (x->ring_calls % epic_ctx::kTimingRing)], x->stream);
}
void mark_main_end(epic_ctx* x) {
  if (!x->timing) return;
  (void)hipEventRecord(x->ev[1], x->stream);
  (void)hipEventRecord(x->ring[2 * (x->ring_calls % epic_ctx::kTimingRing) + 1], x->stream);
  ++x->ring_calls;
}

epic_status check_config(const epic_config* c, std::string& m) {
  if (!c) { m = "config is NULL"; return EPIC_E_INVALID; }
  if (c->grid_n != 32 && c->grid_n != 64 && c->grid_n != 128) {
    m = "grid_n must be 32, 64 or 128"; return EPIC_E_INVALID;
  }
  if (c->n_pol != 1 && c->n_pol != 2) { m = "n_pol must be 1 or 2"; return EPIC_E_INVALID; }
  if (c->n_chan < 1 || c->n_chan > 65536) { m = "n_chan out of range"; return EPIC_E_INVALID; }
  if (c->n_ant < 1 || c->n_ant > 4096) { m = "n_ant must be in 1..4096"; return EPIC_E_INVALID; }
  if (c->kernel_support < 1 || c->kernel_support > 15 || c->kernel_support % 2 == 0) {
    m = "kernel_support must be odd and in 1..15"; return EPIC_E_INVALID;
  }
  if (!(c->kernel_sigma_cells > 0) || !std::isfinite(c->kernel_sigma_cells)) {
    m = "kernel_sigma_cells must be finite and positive"; return EPIC_E_INVALID;
  }
  if (!(c->cell_wavelengths > 0) || !std::isfinite(c->cell_wavelengths)) {
    m = "cell_wavelengths must be finite and positive"; return EPIC_E_INVALID;
  }
  if (c->precision != EPIC_FP32 && c->precision != EPIC_SPLIT_FP16 &&
      c->precision != EPIC_SPLIT_BF16) {
    m = "unknown precision"; return EPIC_E_INVALID;
  }
  if (c->flags & ~(EPIC_FLAG_STAGED | EPIC_FLAG_TIMING | EPIC_FLAG_REMOVE_AUTOS)) {
    m = "unknown flag"; return EPIC_E_INVALID;
  }
  return EPIC_OK;
}

// The split-precision matrix form keeps a 32-pixel tile of the matrix in
// registers: A <= 32 antennas for one polarisation, A <= 16 for two, and the
// float64 matrix of every channel (C * N^2 * A entries) within 2^24 entries.
epic_status check_split(const epic_config* c, std::string& m) {
  const int amax = c->n_pol == 1 ? 16 * epic::kSplitMaxBlocks : 16;
  if (c->n_ant > amax) {
    m = "split-precision forms take at most " + std::to_string(amax) + " antennas at n_pol = " +
        std::to_string(c->n_pol);
    return EPIC_E_UNSUPPORTED;
  }
  if ((double)c->n_chan * c->grid_n * c->grid_n * c->n_ant > (double)(1 << 24)) {
    m = "split-precision forms: n_chan * N^2 * n_ant above 2^24";
    return EPIC_E_UNSUPPORTED;
  }
  return EPIC_OK;
}

// Kernel taps of every antenna for every channel, with the grid bounds check.
// Tap order: dj outer, di inner.  kernels == NULL: the Gaussian evaluated in
// float64 at each tap's offset, rounded once; else the caller's complex
// kernels [C][A][K][K] (interleaved float32 re, im) on the same cells.
epic_status build_geometry(const epic_config& cfg, const double* xy, const double* freq,
                           const float* kernels, Geometry& g, std::string& m) {
  const int N = cfg.grid_n, C = cfg.n_chan, A = cfg.n_ant, K = cfg.kernel_support;
  const int h = K / 2;
  g.C = C; g.A = A; g.KK = K * K;
  g.cell.assign((size_t)C * A * K * K, 0);
  g.w.assign((size_t)C * A * K * K, 0.f);
  for (int a = 0; a < A; ++a)
    if (!std::isfinite(xy[2 * a]) || !std::isfinite(xy[2 * a + 1])) {
      m = "antenna position is not finite"; return EPIC_E_INVALID;
    }
  for (int c = 0; c < C; ++c)
    if (!std::isfinite(freq[c]) || !(freq[c] > 0)) {
      m = "channel frequency must be finite and positive"; return EPIC_E_INVALID;
    }
  const double inv2s2 = 1.0 / (2.0 * cfg.kernel_sigma_cells * cfg.kernel_sigma_cells);
  g.tcell.assign((size_t)C * A * K * K, 0);
  if (kernels) {
    g.wi.assign((size_t)C * A * K * K, 0.f);
    for (size_t o = 0; o < 2 * (size_t)C * A * K * K; ++o)
      if (!std::isfinite(kernels[o])) { m = "kernel value is not finite"; return EPIC_E_INVALID; }
  }
  g.fits_half = true;
  g.fits_wide = true;
  g.ext_j = g.ext_i = 0;
  g.wide_rows = 0;
  g.transposed = false;
  for (int c = 0; c < C; ++c) {
    const double cell_m = kC0 / freq[c] * cfg.cell_wavelengths;
    int jmin = N, jmax = -1, imin = N, imax = -1;
    for (int a = 0; a < A; ++a) {
      const double X = xy[2 * a] / cell_m + N / 2.0;
      const double Y = xy[2 * a + 1] / cell_m + N / 2.0;
      const double i0 = std::floor(X + 0.5), j0 = std::floor(Y + 0.5);
      if (i0 - h < 0 || j0 - h < 0 || i0 + h > N - 1 || j0 + h > N - 1) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "antenna %d leaves the %dx%d grid at channel %d "
                      "(cell %.1f, %.1f)", a, N, N, c, X, Y);
        m = buf;
        return EPIC_E_OFFGRID;
      }
      int k = 0;
      for (int dj = -h; dj <= h; ++dj)
        for (int di = -h; di <= h; ++di, ++k) {
          const double i = i0 + di, j = j0 + dj;
          const size_t o = ((size_t)c * A + a) * g.KK + k;
          g.cell[o] = (int)j * N + (int)i;
          if (kernels) {
            g.w[o] = kernels[2 * o];
            g.wi[o] = kernels[2 * o + 1];
          } else {
            g.w[o] = (float)std::exp(-((i - X) * (i - X) + (j - Y) * (j - Y)) * inv2s2);
          }
          jmin = std::min(jmin, (int)j);
          jmax = std::max(jmax, (int)j);
          imin = std::min(imin, (int)i);
          imax = std::max(imax, (int)i);
        }
    }
    g.ext_j = std::max(g.ext_j, jmax - jmin + 1);
    g.ext_i = std::max(g.ext_i, imax - imin + 1);
    if (jmax - jmin + 1 > N / 2 || imax - imin + 1 > N / 2) g.fits_half = false;
    if (jmax - jmin + 1 > 3 * N / 4 || imax - imin + 1 > 3 * N / 4) g.fits_wide = false;
    for (size_t o = (size_t)c * A * g.KK; o < (size_t)(c + 1) * A * g.KK; ++o)
      g.tcell[o] = (g.cell[o] / N - jmin) * N + (g.cell[o] % N - imin);
  }
  return EPIC_OK;
}

// Gridding programs of the fused kernels, per channel: a header row with the
// row-pass line of every thread (p << 16 | j, or -1), then L steps per thread.
//  * Rows: each wave transforms CPW/P aperture rows of every polarisation and
//    grids exactly those rows, so gridding and the row pass are separated by
//    a wave-level fence only.  The row slots of a wave follow a residue rule
//    (below) that keeps the row transform free of LDS bank conflicts; within
//    it rows are dealt heaviest first to the least loaded wave.  Rows are
//    stored at their physical rows (FusedShape::phys_row).  A wave's cells
//    are dealt longest first to the least loaded of its 64 threads.
//  * Banks: LDS serves 64-bit reads 32 lanes at a time from 64 four-byte
//    banks and 64-bit writes 16 lanes at a time from 32 banks.  A cell is
//    written once, at its last entry, so few lanes of a quarter-wave write at
//    the same step.  The entries of a cell may be taken in any order: step by
//    step, lanes with one entry left take it, then the others take the
//    remaining entry whose bank (float2 address modulo 16) the quarter-wave
//    uses least.  Empty cells read one of 16 zero slots of E' (slots
//    A .. A+15) on the least used bank and write zero; padding steps add zero
//    and write nothing.
template <int N>
void build_programs(const Geometry& g, int P, int gpt, std::vector<uint32_t>& out, int& L,
                    std::vector<float>* out_im = nullptr, bool wide = false) {
  constexpr int NT = epic::FusedShape<N>::NT, RS = epic::FusedShape<N>::RS, H = N / 2;
  constexpr int CPW = epic::FusedShape<N>::CPW, NWAVE = NT / 64;
  const int C = g.C, A = g.A, KK = g.KK;
  const int ES = NT * gpt / P + 64;                    // EStride<NT, gpt, P>
  const int XB = P * ES;                               // grid base, float2 units
  using SH = epic::FusedShape<N>;
  // row slots per wave: CPW / P lines of one polarisation each, or at N = 128
  // CPW rows whose lane group takes both polarisations
  const int SPW = N == 128 ? CPW : CPW / P;
  // wide (N = 64): a block of HR = g.wide_rows (32, 40 or 48) rows by HW
  // columns.  Its HR rows per polarisation fill HR P / 64 row passes of the 8
  // waves (1, 1.25 or 1.5 at P = 2); rather than every wave running a second
  // pass with part of its lanes, whole waves take two full passes or one: at
  // P = 2, (HR - N/2) / 4 waves own 2 SPW rows (the header's second word holds
  // the second pass's line) and the others SPW rows; at P = 1, HR / SPW waves
  // own SPW rows and the others none.  The two-pass waves are 0-3 (HR = 48)
  // or 0 and 1 (HR = 40): a CU puts waves w and w + 4 of a workgroup on one
  // SIMD (measured), so these sit on different SIMDs; of the pairs that do,
  // 0 and 1 (like 0 and 3, or 1 and 2) measured 2 % faster than 0 and 2, and
  // a pair on one SIMD (0 and 4) 4 % slower.  Results do not depend on the
  // choice.
  const int HR = wide ? g.wide_rows : H;               // aperture rows of the block
  const int HC = wide ? SH::HW : H;                    // aperture columns of the block
  const int NWR = wide ? (P == 2 ? NWAVE : HR / SPW) : H / SPW;   // waves that own rows
  const int NTWO = wide && P == 2 ? (HR - H) / 4 : 0;  // two-pass waves
  auto two_pass = [&](int w) { return NTWO == 4 ? w < 4 : NTWO == 2 && w < 2; };
  std::vector<int> rpw(NWAVE, 0);                      // rows per wave
  for (int w = 0; w < NWR; ++w) rpw[w] = two_pass(w) ? 2 * SPW : SPW;
  const int RPW = *std::max_element(rpw.begin(), rpw.end());
  // residue rule (row j of slot s in a wave of group t has j mod M = residue):
  // at N = 64 it puts the 4 (P = 2) or 8 (P = 1) rows a half-wave transforms
  // on distinct bank ranges given the interleaved physical rows and the
  // polarisation stride; at N = 32 rows of a wave are distinct modulo 8 / 16,
  // at N = 128 (a lane group per row, both polarisations) modulo 8
  const int M = N == 128 ? 8 : N == 64 ? 8 : (P == 2 ? 8 : 16);
  const int NGRP = (N == 64 && P == 2) ? 2 : 1;
  auto residue = [&](int sl, int t) {
    if (N != 64) return sl;
    if (P == 1) return (sl >> 1) + 4 * (sl & 1);
    static const int rho[4] = {0, 4, 1, 5};
    return rho[sl] + 2 * t;
  };
  auto code = [](int cell_f2, int e, bool last) {
    return ((uint32_t)(cell_f2 * 8) << epic::STEP_CELL_SHIFT) | (uint32_t)(e * 8) |
           (last ? epic::STEP_LAST_BIT : 0u);
  };
  // the fields of a step word: cell byte offsets (the aperture rows of one
  // polarisation) below 2^17, E' byte offsets (both polarisations) below 2^15
  static_assert(H * SH::RS * 8 <= (1 << (32 - epic::STEP_CELL_SHIFT)), "cell offsets exceed the step field");
  if ((int64_t)P * ES * 8 > (int64_t)epic::STEP_E_MASK + 8) {   // not reached by the shapes the kernels take
    out.clear();
    L = 0;
    return;
  }
  auto wbits = [](float w) {
    uint32_t b;
    std::memcpy(&b, &w, 4);
    return b;
  };
  const bool cpx = !g.wi.empty() && out_im;
  constexpr size_t kNoTap = ~(size_t)0;
  struct Run {
    int cell;
    std::vector<std::pair<int, size_t>> ent;           // (antenna, tap index)
  };
  std::vector<std::vector<uint32_t>> words((size_t)C * NT);   // [c][thread] -> step words
  std::vector<std::vector<float>> wims(cpx ? (size_t)C * NT : 0);
  std::vector<int32_t> header((size_t)C * NT, -1), header2((size_t)C * NT, -1);
  std::vector<int> wave_steps((size_t)C * NWAVE, 0);
  L = 1;
  for (int c = 0; c < C; ++c) {
    std::vector<Run> cells(HR * HC);
    for (int j = 0; j < HR; ++j)
      for (int i = 0; i < HC; ++i) cells[j * HC + i].cell = SH::phys_row(j) * RS + i;
    for (int a = 0; a < A; ++a)
      for (int k = 0; k < KK; ++k) {
        const size_t o = ((size_t)c * A + a) * KK + k;
        const int j = g.tcell[o] / N, i = g.tcell[o] % N;
        cells[j * HC + i].ent.push_back({a, o});
      }
    // rows to (wave, slot): slot s of a wave in group t takes a row j with
    // j mod M = residue(s, t); each residue class has exactly as many rows as
    // the group has waves, dealt heaviest first to the least loaded wave
    std::vector<int> row_load(HR, 0);
    for (int j = 0; j < HR; ++j)
      for (int i = 0; i < HC; ++i) row_load[j] += (int)std::max<size_t>(1, cells[j * HC + i].ent.size());
    std::vector<int> wave_load(NWAVE, 0);
    std::vector<std::vector<int>> row_of(NWAVE, std::vector<int>(RPW, -1));
    const int WPG = NWR / NGRP;                        // waves per group
    for (int t = 0; t < (wide ? 0 : NGRP); ++t)
      for (int sl = 0; sl < SPW; ++sl) {
        const int rho = residue(sl, t);
        std::vector<int> rows;
        for (int j = rho; j < H; j += M) rows.push_back(j);
        std::stable_sort(rows.begin(), rows.end(), [&](int x, int y) { return row_load[x] > row_load[y]; });
        for (int j : rows) {
          int bw = -1;
          for (int w = t * WPG; w < (t + 1) * WPG; ++w)
            if (row_of[w][sl] < 0 && (bw < 0 || wave_load[w] < wave_load[bw])) bw = w;
          row_of[bw][sl] = j;
          wave_load[bw] += row_load[j];
        }
      }
    if (wide) {
      // Rows a row pass loads together must fall on distinct bank ranges: with
      // the interleaved rows this holds when, per pass, a wave's rows differ in
      // cls(j) = 2 (j & 1) + ((j >> 2) & 1) (P = 2: phys_row mod 4, both
      // polarisations at once) or in j mod 8 (P = 1, phys_row mod 8).  So
      // slot s of either pass takes class s mod SPW.  Within a class, heaviest
      // row first to the wave with a free slot of that class and the least
      // cost: its gridding steps so far, plus, for a two-pass wave, the
      // second pass counted as kPassSteps steps of each of its 64 lanes, so
      // that the two-pass waves take the lighter rows.
      constexpr int kPassSteps = 12;
      const int NCLS = P == 2 ? 4 : 8;
      auto cls = [&](int j) { return P == 2 ? 2 * (j & 1) + ((j >> 2) & 1) : (j & 7); };
      auto cost = [&](int w) { return wave_load[w] + (rpw[w] > SPW ? 64 * kPassSteps : 0); };
      for (int k = 0; k < NCLS; ++k) {
        std::vector<int> rows;
        for (int j = 0; j < HR; ++j)
          if (cls(j) == k) rows.push_back(j);
        std::stable_sort(rows.begin(), rows.end(), [&](int x, int y) { return row_load[x] > row_load[y]; });
        for (int j : rows) {
          int bw = -1, bs = -1;
          for (int w = 0; w < NWR; ++w)
            for (int sl = k % SPW; sl < rpw[w]; sl += SPW)
              if (row_of[w][sl] < 0 && (bw < 0 || cost(w) < cost(bw))) {
                bw = w;
                bs = sl;
                break;
              }
          if (bw < 0) {                                // not reached: the classes fill every slot
            out.clear();
            L = 0;
            return;
          }
          row_of[bw][bs] = j;
          wave_load[bw] += row_load[j];
        }
      }
    }
    for (int t = 0; t < NT; ++t) {
      const epic::Roles<N> ro(t);
      if (ro.wave >= NWR) continue;
      const int p = ro.sub / SPW, sl = ro.sub % SPW;     // N = 128: p = 0, both polarisations
      if (p >= P) continue;
      if (sl < rpw[ro.wave]) header[(size_t)c * NT + t] = (p << 16) | SH::phys_row(row_of[ro.wave][sl]);
      if (wide && SPW + sl < rpw[ro.wave])
        header2[(size_t)c * NT + t] = (p << 16) | SH::phys_row(row_of[ro.wave][SPW + sl]);
    }
    // cells of each wave's rows, longest first, to the least loaded lane of the wave
    std::vector<std::vector<const Run*>> lane_runs(NT);
    std::vector<int> load(NT, 0);
    std::vector<std::vector<std::vector<const Run*>>> spat_w(NWR);
    std::vector<std::vector<int>> spat_ld(NWR);
    int plain_max = 1;
    for (int w = 0; w < NWR; ++w) {
      std::vector<const Run*> wc;
      for (int sl = 0; sl < rpw[w]; ++sl)
        for (int i = 0; i < HC; ++i) wc.push_back(&cells[row_of[w][sl] * HC + i]);
      using Load = std::pair<int, int>;                // (steps, thread)
      auto steps_of = [](const Run* r) { return (int)std::max<size_t>(1, r->ent.size()); };
      // longest cell first to the least loaded of the given lanes
      auto lpt = [&](const std::vector<const Run*>& cells_in, int t0, int nl,
                     std::vector<std::vector<const Run*>>& out, std::vector<int>& ld_out) {
        std::vector<const Run*> cs(cells_in);
        std::stable_sort(cs.begin(), cs.end(), [&](const Run* x, const Run* y) { return steps_of(x) > steps_of(y); });
        std::priority_queue<Load, std::vector<Load>, std::greater<Load>> pq;
        for (int t = t0; t < t0 + nl; ++t) pq.push({0, t});
        for (const Run* r : cs) {
          Load ld = pq.top();
          pq.pop();
          out[ld.second - 64 * w].push_back(r);
          ld.first += steps_of(r);
          ld_out[ld.second - 64 * w] = ld.first;
          pq.push(ld);
        }
      };
      // the whole wave by longest cell first
      std::vector<std::vector<const Run*>> plain(64), spat(64);
      std::vector<int> lp(64, 0), ls(64, 0);
      lpt(wc, 64 * w, 64, plain, lp);
      // each half-wave a run of neighbouring cells (the wave's cells in
      // column-major order cut into two runs of equal step counts), so that
      // lanes reading E' together grid cells that share antennas and their
      // reads can be broadcasts
      std::vector<const Run*> sp(wc);
      std::stable_sort(sp.begin(), sp.end(), [&](const Run* x, const Run* y) {
        const int cx = x->cell % RS, cy = y->cell % RS;
        return cx != cy ? cx < cy : x->cell < y->cell;
      });
      int tot = 0;
      for (const Run* r : sp) tot += steps_of(r);
      std::vector<const Run*> half[2];
      {
        int acc = 0;
        for (const Run* r : sp) {
          half[std::min(1, (int)((acc + steps_of(r) / 2) * 2LL / std::max(1, tot)))].push_back(r);
          acc += steps_of(r);
        }
      }
      lpt(half[0], 64 * w, 32, spat, ls);
      lpt(half[1], 64 * w + 32, 32, spat, ls);
      for (int l = 0; l < 64; ++l) {
        lane_runs[64 * w + l] = plain[l];
        load[64 * w + l] = lp[l];
      }
      plain_max = std::max(plain_max, *std::max_element(lp.begin(), lp.end()));
      spat_w[w] = std::move(spat);
      spat_ld[w] = std::move(ls);
    }
    // the spatial assignment of a wave wherever it does not lengthen the program
    for (int w = 0; w < NWR; ++w)
      if (*std::max_element(spat_ld[w].begin(), spat_ld[w].end()) <= plain_max)
        for (int l = 0; l < 64; ++l) {
          lane_runs[64 * w + l] = spat_w[w][l];
          load[64 * w + l] = spat_ld[w][l];
        }
    const int Lc = std::max(1, *std::max_element(load.begin(), load.end()));
    L = std::max(L, Lc);
    // each wave stops after its own longest lane (the later steps of its
    // lanes are padding), rounded like L to whole chunks past the fixed forms
    for (int w = 0; w < NWAVE; ++w) {
      int lw = std::max(1, *std::max_element(load.begin() + 64 * w, load.begin() + 64 * w + 64));
      if (lw > epic::kMaxFixedSteps + epic::kStepChunk)
        lw = (lw + epic::kStepChunk - 1) / epic::kStepChunk * epic::kStepChunk;
      wave_steps[(size_t)c * NWAVE + w] = lw <= 255 ? lw : 0;
    }
    // step-by-step choice of the E' entries, per quarter-wave (measured faster
    // than choosing per half-wave for these paired reads)
    for (int q = 0; q < NT / 16; ++q) {
      struct Lane {
        size_t run = 0;
        std::vector<std::pair<int, size_t>> left;      // entries of the current run not yet taken
        bool started = false;
      };
      Lane st[16];
      for (int step = 0; step < Lc; ++step) {
        int used[16] = {0};
        int pick_e[16], pick_cell[16];
        size_t pick_w[16];                             // tap index, or kNoTap
        bool pick_last[16];
        bool decided[16] = {false};
        for (int l = 0; l < 16; ++l) {                 // open the current run
          Lane& s = st[l];
          const auto& runs = lane_runs[16 * q + l];
          if (!s.started && s.run < runs.size()) {
            s.left = runs[s.run]->ent;
            s.started = true;
          }
        }
        // lanes reading the same antenna share one LDS access (a broadcast),
        // so only the distinct antennas of the step load the banks
        int picked[16], npicked = 0;
        auto is_picked = [&](int ant) {
          for (int i = 0; i < npicked; ++i)
            if (picked[i] == ant) return true;
          return false;
        };
        auto take = [&](int ant) {
          if (is_picked(ant)) return;
          picked[npicked++] = ant;
          used[ant % 16]++;
        };
        for (int l = 0; l < 16; ++l) {                 // lanes with one entry left
          Lane& s = st[l];
          const auto& runs = lane_runs[16 * q + l];
          if (s.run < runs.size() && s.left.size() == 1) {
            pick_e[l] = s.left[0].first;
            pick_w[l] = s.left[0].second;
            pick_cell[l] = runs[s.run]->cell;
            pick_last[l] = true;
            take(pick_e[l]);
            decided[l] = true;
          }
        }
        for (int l = 0; l < 16; ++l) {                 // lanes with several entries left
          if (decided[l]) continue;
          Lane& s = st[l];
          const auto& runs = lane_runs[16 * q + l];
          if (s.run >= runs.size() || s.left.empty()) continue;
          // an antenna another lane already reads costs nothing, else its bank's load
          auto cost = [&](int ant) { return is_picked(ant) ? -1 : used[ant % 16]; };
          size_t best = 0;
          for (size_t k = 1; k < s.left.size(); ++k)
            if (cost(s.left[k].first) < cost(s.left[best].first)) best = k;
          pick_e[l] = s.left[best].first;
          pick_w[l] = s.left[best].second;
          pick_cell[l] = runs[s.run]->cell;
          pick_last[l] = false;
          take(pick_e[l]);
          decided[l] = true;
        }
        for (int l = 0; l < 16; ++l) {                 // empty cells and padding
          if (decided[l]) continue;
          // a zero slot another lane already reads (a broadcast), else the
          // zero slot on the least loaded bank
          int z = -1;
          for (int k = 0; k < 16 && z < 0; ++k)
            if (is_picked(A + k)) z = k;
          if (z < 0) {
            z = 0;
            for (int k = 1; k < 16; ++k)
              if (used[(A + k) % 16] < used[(A + z) % 16]) z = k;
          }
          take(A + z);
          pick_e[l] = A + z;
          pick_w[l] = kNoTap;
          const Lane& s = st[l];
          const auto& runs = lane_runs[16 * q + l];
          pick_last[l] = s.run < runs.size();          // empty cell: write zero; padding: no write
          pick_cell[l] = s.run < runs.size() ? runs[s.run]->cell : 0;
          decided[l] = true;
        }
        for (int l = 0; l < 16; ++l) {
          auto& wv = words[(size_t)c * NT + 16 * q + l];
          wv.push_back(code(pick_cell[l], pick_e[l], pick_last[l]));
          wv.push_back(wbits(pick_w[l] == kNoTap ? 0.f : g.w[pick_w[l]]));
          if (cpx) wims[(size_t)c * NT + 16 * q + l].push_back(pick_w[l] == kNoTap ? 0.f : g.wi[pick_w[l]]);
          Lane& s = st[l];
          const auto& runs = lane_runs[16 * q + l];
          if (s.run < runs.size()) {
            for (size_t k = 0; k < s.left.size(); ++k)   // an antenna enters a cell once
              if (s.left[k].first == pick_e[l]) {
                s.left.erase(s.left.begin() + (long)k);
                break;
              }
            if (s.left.empty()) {                      // run finished
              ++s.run;
              s.started = false;
            }
          }
        }
      }
    }
  }
  if (L > epic::kMaxFixedSteps) L = (L + epic::kStepChunk - 1) / epic::kStepChunk * epic::kStepChunk;
  out.assign((size_t)C * (L + 1) * NT * 2, 0u);
  if (cpx) out_im->assign((size_t)C * (L + 1) * NT, 0.f);
  for (int c = 0; c < C; ++c)
    for (int t = 0; t < NT; ++t) {
      const size_t h = ((size_t)c * (L + 1) * NT + t) * 2;
      out[h] = (uint32_t)header[(size_t)c * NT + t];
      const int32_t l2 = header2[(size_t)c * NT + t];
      out[h + 1] = (l2 < 0 ? epic::HDR_LINE2_NONE : (uint32_t)l2) |
                   (uint32_t)wave_steps[(size_t)c * NWAVE + t / 64] << 24;
      const auto& wv = words[(size_t)c * NT + t];
      const uint32_t pad = code(0, A + t % 16, false);
      for (int s2 = 0; s2 < L; ++s2) {
        const size_t o = (((size_t)c * (L + 1) + 1 + s2) * NT + t) * 2;
        if ((size_t)s2 < wv.size() / 2) {
          out[o] = wv[2 * s2];
          out[o + 1] = wv[2 * s2 + 1];
          if (cpx) (*out_im)[o / 2] = wims[(size_t)c * NT + t][s2];
        } else {
          out[o] = pad;
          out[o + 1] = wbits(0.f);
        }
      }
    }
}

template <typename F>
int occupancy_blocks(F kernel, int threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess) nb = 1;
  return std::max(1, nb);
}

template <int N, int P, int GPT>
int fused_blocks_per_cu(bool cpx) {
  return cpx ? occupancy_blocks(epic::fused_image_kernel<N, P, GPT, true>, epic::FusedShape<N>::NT)
             : occupancy_blocks(epic::fused_image_kernel<N, P, GPT, false>, epic::FusedShape<N>::NT);
}

template <int P, int GPT>
int fused_wide_blocks_per_cu(bool cpx) {
  return cpx ? occupancy_blocks(epic::fused_wide_image_kernel<64, P, GPT, true>, epic::FusedShape<64>::NT)
             : occupancy_blocks(epic::fused_wide_image_kernel<64, P, GPT, false>, epic::FusedShape<64>::NT);
}

int fused_wide_blocks_per_cu(int P, int gpt, bool cpx) {
  if (P == 1) return gpt == 1 ? fused_wide_blocks_per_cu<1, 1>(cpx)
                   : gpt == 2 ? fused_wide_blocks_per_cu<1, 2>(cpx) : fused_wide_blocks_per_cu<1, 4>(cpx);
  return gpt == 1 ? fused_wide_blocks_per_cu<2, 1>(cpx)
       : gpt == 2 ? fused_wide_blocks_per_cu<2, 2>(cpx) : fused_wide_blocks_per_cu<2, 4>(cpx);
}

template <int P>
int fused128_blocks_per_cu(int gpt, bool cpx) {
  const int NT = epic::FusedShape<128>::NT;
  if (gpt == 1) return cpx ? occupancy_blocks(epic::fused_image128_kernel<P, 1, true>, NT)
                           : occupancy_blocks(epic::fused_image128_kernel<P, 1, false>, NT);
  if (gpt == 2) return cpx ? occupancy_blocks(epic::fused_image128_kernel<P, 2, true>, NT)
                           : occupancy_blocks(epic::fused_image128_kernel<P, 2, false>, NT);
  return cpx ? occupancy_blocks(epic::fused_image128_kernel<P, 4, true>, NT)
             : occupancy_blocks(epic::fused_image128_kernel<P, 4, false>, NT);
}

int fused_blocks_per_cu(int N, int P, int gpt, bool cpx) {
  if (N == 128) return P == 2 ? fused128_blocks_per_cu<2>(gpt, cpx) : fused128_blocks_per_cu<1>(gpt, cpx);
#define EPIC_OCC(NN, PP, GG) if (N == NN && P == PP && gpt == GG) return fused_blocks_per_cu<NN, PP, GG>(cpx);
  EPIC_OCC(32, 1, 1) EPIC_OCC(32, 1, 2) EPIC_OCC(32, 1, 4)
  EPIC_OCC(32, 2, 1) EPIC_OCC(32, 2, 2) EPIC_OCC(32, 2, 4)
  EPIC_OCC(64, 1, 1) EPIC_OCC(64, 1, 2) EPIC_OCC(64, 1, 4)
  EPIC_OCC(64, 2, 1) EPIC_OCC(64, 2, 2) EPIC_OCC(64, 2, 4)
#undef EPIC_OCC
  return 1;
}

template <int P, bool CPX>
int adjoint_wide_blocks_per_cu(int gpt) {
  if (gpt == 1) return occupancy_blocks(epic::adjoint_wide_kernel<64, P, 1, CPX>, epic::FusedShape<64>::NT);
  if (gpt == 2) return occupancy_blocks(epic::adjoint_wide_kernel<64, P, 2, CPX>, epic::FusedShape<64>::NT);
  return occupancy_blocks(epic::adjoint_wide_kernel<64, P, 4, CPX>, epic::FusedShape<64>::NT);
}

int adjoint_wide_blocks_per_cu(int P, int gpt, bool cpx) {
  if (cpx) return P == 1 ? adjoint_wide_blocks_per_cu<1, true>(gpt) : adjoint_wide_blocks_per_cu<2, true>(gpt);
  return P == 1 ? adjoint_wide_blocks_per_cu<1, false>(gpt) : adjoint_wide_blocks_per_cu<2, false>(gpt);
}

template <int N, int P, bool CPX>
int adjoint_blocks_per_cu(int gpt) {
  if (gpt == 1) return occupancy_blocks(epic::adjoint_kernel<N, P, 1, CPX>, epic::FusedShape<N>::NT);
  if (gpt == 2) return occupancy_blocks(epic::adjoint_kernel<N, P, 2, CPX>, epic::FusedShape<N>::NT);
  return occupancy_blocks(epic::adjoint_kernel<N, P, 4, CPX>, epic::FusedShape<N>::NT);
}

template <int P, bool CPX>
int adjoint128_blocks_per_cu(int gpt) {
  const int NT = epic::FusedShape<128>::NT;
  if (gpt == 1) return occupancy_blocks(epic::adjoint128_kernel<P, 1, CPX>, NT);
  if (gpt == 2) return occupancy_blocks(epic::adjoint128_kernel<P, 2, CPX>, NT);
  return occupancy_blocks(epic::adjoint128_kernel<P, 4, CPX>, NT);
}

int adjoint_blocks_per_cu(int N, int P, int gpt, bool cpx) {
  if (N == 128) {
    if (cpx) return P == 1 ? adjoint128_blocks_per_cu<1, true>(gpt) : adjoint128_blocks_per_cu<2, true>(gpt);
    return P == 1 ? adjoint128_blocks_per_cu<1, false>(gpt) : adjoint128_blocks_per_cu<2, false>(gpt);
  }
  if (cpx) {
    if (N == 32) return P == 1 ? adjoint_blocks_per_cu<32, 1, true>(gpt) : adjoint_blocks_per_cu<32, 2, true>(gpt);
    return P == 1 ? adjoint_blocks_per_cu<64, 1, true>(gpt) : adjoint_blocks_per_cu<64, 2, true>(gpt);
  }
  if (N == 32) return P == 1 ? adjoint_blocks_per_cu<32, 1, false>(gpt) : adjoint_blocks_per_cu<32, 2, false>(gpt);
  return P == 1 ? adjoint_blocks_per_cu<64, 1, false>(gpt) : adjoint_blocks_per_cu<64, 2, false>(gpt);
}

int fused_threads(int N) {
  return N == 32 ? epic::FusedShape<32>::NT : N == 64 ? epic::FusedShape<64>::NT : epic::FusedShape<128>::NT;
}

bool launch_fused(epic_ctx* x, const epic::FusedArgs& a) {
  const int N = x->cfg.grid_n, P = x->cfg.n_pol, G = x->fused_gpt;
  const dim3 grid(a.W), block(fused_threads(N));
  if (x->wide) {
    if (N != 64) return false;
    if (P == 2 && G == 1 && !x->cpx && x->wide_rows == 40) {   // the deployed array's block
      hipLaunchKernelGGL((epic::fused_wide_image_kernel<64, 2, 1, false, 40>), grid, block, 0, x->stream, a);
      return true;
    }
#define EPIC_LW(PP, GG)                                                                      \
    if (P == PP && G == GG) {                                                                \
      if (x->cpx) hipLaunchKernelGGL((epic::fused_wide_image_kernel<64, PP, GG, true>), grid, block, 0, \
                                     x->stream, a);                                          \
      else hipLaunchKernelGGL((epic::fused_wide_image_kernel<64, PP, GG, false>), grid, block, 0, \
                              x->stream, a);                                                 \
      return true;                                                                           \
    }
    EPIC_LW(1, 1) EPIC_LW(1, 2) EPIC_LW(1, 4) EPIC_LW(2, 1) EPIC_LW(2, 2) EPIC_LW(2, 4)
#undef EPIC_LW
    return false;
  }
#define EPIC_LF(NN, PP, GG)                                                                 \
  if (N == NN && P == PP && G == GG) {                                                      \
    if (x->cpx) hipLaunchKernelGGL((epic::fused_image_kernel<NN, PP, GG, true>), grid, block, 0, \
                                   x->stream, a);                                           \
    else hipLaunchKernelGGL((epic::fused_image_kernel<NN, PP, GG, false>), grid, block, 0,   \
                            x->stream, a);                                                  \
    return true;                                                                            \
  }
  EPIC_LF(32, 1, 1) EPIC_LF(32, 1, 2) EPIC_LF(32, 1, 4)
  EPIC_LF(32, 2, 1) EPIC_LF(32, 2, 2) EPIC_LF(32, 2, 4)
  EPIC_LF(64, 1, 1) EPIC_LF(64, 1, 2) EPIC_LF(64, 1, 4)
  EPIC_LF(64, 2, 1) EPIC_LF(64, 2, 2) EPIC_LF(64, 2, 4)
#undef EPIC_LF
  return false;
}

template <int P>
bool launch_fused128(epic_ctx* x, const epic::FusedArgs& a) {
  const dim3 grid(a.W), block(epic::FusedShape<128>::NT);
  if (x->cpx) {
    switch (x->fused_gpt) {
      case 1: hipLaunchKernelGGL((epic::fused_image128_kernel<P, 1, true>), grid, block, 0, x->stream, a); return true;
      case 2: hipLaunchKernelGGL((epic::fused_image128_kernel<P, 2, true>), grid, block, 0, x->stream, a); return true;
      case 4: hipLaunchKernelGGL((epic::fused_image128_kernel<P, 4, true>), grid, block, 0, x->stream, a); return true;
      default: return false;
    }
  }
  switch (x->fused_gpt) {
    case 1: hipLaunchKernelGGL((epic::fused_image128_kernel<P, 1, false>), grid, block, 0, x->stream, a); return true;
    case 2: hipLaunchKernelGGL((epic::fused_image128_kernel<P, 2, false>), grid, block, 0, x->stream, a); return true;
    case 4: hipLaunchKernelGGL((epic::fused_image128_kernel<P, 4, false>), grid, block, 0, x->stream, a); return true;
    default: return false;
  }
}

bool launch_fused128(epic_ctx* x, const epic::FusedArgs& a) {
  return x->cfg.n_pol == 2 ? launch_fused128<2>(x, a) : launch_fused128<1>(x, a);
}

// Sub-lanes per output value in the reduction kernels: enough that a channel
// covered by many workgroup slots (or time chunks) is summed by several
// threads with independent loads in flight.
int reduce_sub(int64_t slots_per_value) {
  return slots_per_value > 32 ? 16 : (slots_per_value > 4 ? 4 : 1);
}

// Upper bound on the workgroup slots covering one channel of a persistent launch.
int64_t slots_per_channel(int64_t n_time, int64_t total, int64_t W) {
  return (n_time * W + total - 1) / total + 1;
}

// Teams of the fused imaging launches (FusedArgs): the smallest power of two
// that cuts a segment of n_time units into member parts of at most KBLOCK
// units, at most kMaxTeam; `over` > 0 replaces it (a power of two <= kMaxTeam).
constexpr int kMaxTeam = 8;
int team_for(int64_t n_time, int over) {
  if (over > 0) return over;
  int m = 1;
  while (m < kMaxTeam && (n_time + m - 1) / m > epic::FusedShape<64>::KBLOCK) m *= 2;
  return m;
}

// Partial-image slots of a fused launch of W workgroups in teams of m over
// segs segments: (segs + W / m - 1) m.
int64_t slot_count(int64_t segs, int64_t W, int64_t m) { return (segs + W / m - 1) * m; }

// The most slots any team size gives a launch of at most w_cap workgroups.
int64_t max_slot_count(int64_t segs, int64_t w_cap) {
  int64_t n = 0;
  for (int m = 1; m <= kMaxTeam; m *= 2)
    if (w_cap >= m) n = std::max(n, slot_count(segs, (w_cap / m) * m, m));
  return n;
}

// float64 values per slot: NACC N^2 (N <= 64) or NACC N^2 / 2 (one parity at N = 128).
size_t fused_slot_values(int N, int nacc) { return (size_t)nacc * N * N / (N == 128 ? 2 : 1); }

// Sub-lanes of the fused reductions: parts per segment are about m times the
// teams covering it (one long channel: up to one part per workgroup).
int fused_reduce_sub(int64_t n_time, int64_t units, int W, int m) {
  const int64_t parts = slots_per_channel(n_time, units, W / m) * m;
  return parts > 256 ? 64 : reduce_sub(parts);
}

bool launch_reduce(epic_ctx* x, const epic::ReduceArgs& a, bool thread_major) {
  const int N = x->cfg.grid_n, P = x->cfg.n_pol;
  const int64_t n = (int64_t)x->cfg.n_chan * N * N;
  const int64_t ppb = 256 / a.sub;
  const dim3 grid((unsigned)((n + ppb - 1) / ppb)), block(256);
#define EPIC_LR(NN, PP, TM)                                                                    \
  if (N == NN && P == PP && thread_major == TM) {                                              \
    hipLaunchKernelGGL((epic::reduce_image_kernel<NN, PP, TM>), grid, block, 0, x->stream, a); \
    return true;                                                                               \
  }
  EPIC_LR(32, 1, true) EPIC_LR(32, 2, true) EPIC_LR(64, 1, true) EPIC_LR(64, 2, true)
  EPIC_LR(32, 1, false) EPIC_LR(32, 2, false) EPIC_LR(64, 1, false) EPIC_LR(64, 2, false)
  EPIC_LR(128, 1, false) EPIC_LR(128, 2, false)
#undef EPIC_LR
  return false;
}

bool launch_adjoint(epic_ctx* x, const epic::AdjointArgs& a) {
  const int N = x->cfg.grid_n, P = x->cfg.n_pol, G = x->fused_gpt;
  const dim3 grid(a.W), block(fused_threads(N));
  if (x->wide) {
    if (N != 64) return false;
#define EPIC_LAW(PP, GG)                                                                     \
    if (P == PP && G == GG) {                                                                \
      if (x->cpx) hipLaunchKernelGGL((epic::adjoint_wide_kernel<64, PP, GG, true>), grid, block, 0, \
                                     x->stream, a);                                          \
      else hipLaunchKernelGGL((epic::adjoint_wide_kernel<64, PP, GG, false>), grid, block, 0, \
                              x->stream, a);                                                 \
      return true;                                                                           \
    }
    EPIC_LAW(1, 1) EPIC_LAW(1, 2) EPIC_LAW(1, 4) EPIC_LAW(2, 1) EPIC_LAW(2, 2) EPIC_LAW(2, 4)
#undef EPIC_LAW
    return false;
  }
#define EPIC_LA(NN, PP, GG)                                                                  \
  if (N == NN && P == PP && G == GG) {                                                       \
    if (x->cpx) hipLaunchKernelGGL((epic::adjoint_kernel<NN, PP, GG, true>), grid, block, 0,  \
                                   x->stream, a);                                            \
    else hipLaunchKernelGGL((epic::adjoint_kernel<NN, PP, GG, false>), grid, block, 0,        \
                            x->stream, a);                                                   \
    return true;                                                                             \
  }
  EPIC_LA(32, 1, 1) EPIC_LA(32, 1, 2) EPIC_LA(32, 1, 4)
  EPIC_LA(32, 2, 1) EPIC_LA(32, 2, 2) EPIC_LA(32, 2, 4)
  EPIC_LA(64, 1, 1) EPIC_LA(64, 1, 2) EPIC_LA(64, 1, 4)
  EPIC_LA(64, 2, 1) EPIC_LA(64, 2, 2) EPIC_LA(64, 2, 4)
#undef EPIC_LA
#define EPIC_LA128(PP, GG)                                                                   \
  if (N == 128 && P == PP && G == GG) {                                                      \
    if (x->cpx) hipLaunchKernelGGL((epic::adjoint128_kernel<PP, GG, true>), grid, block, 0,   \
                                   x->stream, a);                                            \
    else hipLaunchKernelGGL((epic::adjoint128_kernel<PP, GG, false>), grid, block, 0,         \
                            x->stream, a);                                                   \
    return true;                                                                             \
  }
  EPIC_LA128(1, 1) EPIC_LA128(1, 2) EPIC_LA128(1, 4)
  EPIC_LA128(2, 1) EPIC_LA128(2, 2) EPIC_LA128(2, 4)
#undef EPIC_LA128
  return false;
}

bool launch_staged_fft(epic_ctx* x, float2* grid, int64_t nimg) {
  const int N = x->cfg.grid_n;
  const float2* tw = x->twiddle.as<float2>();
  if (N == 32) {
    hipLaunchKernelGGL(epic::staged_fft_kernel<32>, dim3((unsigned)nimg),
                       dim3(epic::StagedFftShape<32>::NT), 0, x->stream, grid, tw);
  } else if (N == 64) {
    hipLaunchKernelGGL(epic::staged_fft_kernel<64>, dim3((unsigned)nimg),
                       dim3(epic::StagedFftShape<64>::NT), 0, x->stream, grid, tw);
  } else {
    hipLaunchKernelGGL(epic::staged_fft_kernel<128>, dim3((unsigned)nimg),
                       dim3(epic::StagedFftShape<128>::NT), 0, x->stream, grid, tw);
  }
  return true;
}

// Staged-path workspace: batches of tb samples, intermediates bounded to ~512 MiB.
bool alloc_staged(epic_ctx* x) {
  if (x->tb > 0) return true;
  const epic_config& c = x->cfg;
  const size_t N = (size_t)c.grid_n;
  const size_t per_t = (size_t)c.n_chan * c.n_pol * (N * N + c.n_ant) * sizeof(float2);
  const int tb = (int)std::max<size_t>(1, std::min<size_t>(64, (512ull << 20) / per_t));
  if (!x->st_e.alloc((size_t)tb * c.n_chan * x->PA * sizeof(float2)) ||
      !x->st_grid.alloc((size_t)tb * c.n_chan * c.n_pol * N * N * sizeof(float2)) ||
      !x->st_acc.alloc((size_t)c.n_chan * x->nacc * N * N * sizeof(double)))
    return false;
  // the staged gradient: upstream gradient table [C][N*N] and per-antenna
  // float64 sums [C][P*A] (a context with fused kernels already holds both,
  // sized at least that large)
  if (c.precision == EPIC_FP32 &&
      ((!x->gtab.p && !x->gtab.alloc((size_t)c.n_chan * N * N * sizeof(float4))) ||
       (!x->gpartial.p && !x->gpartial.alloc((size_t)c.n_chan * x->PA * 2 * sizeof(double)))))
    return false;
  x->tb = tb;
  return true;
}

// Split-precision tables: beta[c][pix][a] = sum_taps w exp(+2 pi i (i kl + j km)/N)
// in float64 (pix = km*N + kl), its per-channel maximum modulus, and the
// workspace of the matrix kernels.
// pixel tiles per wave of the split-image kernel: two for one polarisation and
// one antenna block (the sample conversion is shared by both tiles), else one
int split_tpw(int P, int qb) { return (P == 1 && qb == 1) ? 2 : 1; }

template <int P, bool BF, int QB, int TPW>
void launch_split_image(epic_ctx* x, const epic::SplitArgs& a, dim3 grid, bool vec) {
  if (vec) hipLaunchKernelGGL((epic::split_image_kernel<P, BF, QB, TPW, true>), grid, dim3(256), 0, x->stream, a);
  else hipLaunchKernelGGL((epic::split_image_kernel<P, BF, QB, TPW, false>), grid, dim3(256), 0, x->stream, a);
}

template <int P, bool BF, int QB, int TPW>
void split_occupancy(epic_ctx* x) {
  x->sp_wgs_per_cu[0] = occupancy_blocks(epic::split_image_kernel<P, BF, QB, TPW, false>, 256);
  x->sp_wgs_per_cu[1] = occupancy_blocks(epic::split_image_kernel<P, BF, QB, TPW, true>, 256);
}

struct SplitOccupancy {
  epic_ctx* x;
  template <int P, bool BF, int QB, int TPW> void operator()() const { split_occupancy<P, BF, QB, TPW>(x); }
};
struct SplitLaunch {
  epic_ctx* x;
  const epic::SplitArgs* a;
  dim3 grid;
  bool vec;
  template <int P, bool BF, int QB, int TPW> void operator()() const {
    launch_split_image<P, BF, QB, TPW>(x, *a, grid, vec);
  }
};

// dispatch on (P, precision, antenna blocks) to the instantiated split-image
// kernels: f.operator()<P, BF, QB, TPW>()
template <typename F>
void split_dispatch(int P, bool bf, int qb, F&& f) {
  if (P == 1) {
    if (bf) { if (qb == 1) f.template operator()<1, true, 1, 2>(); else f.template operator()<1, true, 2, 1>(); }
    else    { if (qb == 1) f.template operator()<1, false, 1, 2>(); else f.template operator()<1, false, 2, 1>(); }
  } else {
    if (bf) f.template operator()<2, true, 1, 1>();
    else f.template operator()<2, false, 1, 1>();
  }
}

epic_status build_split_tables(epic_ctx* x, const Geometry& g) {
  const int N = x->cfg.grid_n, C = x->cfg.n_chan, A = x->cfg.n_ant, P = x->cfg.n_pol;
  const int NG = N * N;
  std::vector<double> cs(N * N), sn(N * N);            // exp(2 pi i u k / N) for u, k < N
  for (int u = 0; u < N; ++u)
    for (int k = 0; k < N; ++k) {
      const double ang = 2.0 * M_PI * (double)((u * k) % N) / (double)N;
      cs[u * N + k] = std::cos(ang);
      sn[u * N + k] = std::sin(ang);
    }
  std::vector<double2> beta((size_t)C * NG * A);
  std::vector<double> bmax(C, 0.0);
  for (int c = 0; c < C; ++c)
    for (int a = 0; a < A; ++a)
      for (int km = 0; km < N; ++km)
        for (int kl = 0; kl < N; ++kl) {
          double re = 0.0, im = 0.0;
          for (int k = 0; k < g.KK; ++k) {
            const size_t o = ((size_t)c * A + a) * g.KK + k;
            const int j = g.cell[o] / N, i = g.cell[o] % N;
            const double w = g.w[o], wi = g.wi.empty() ? 0.0 : g.wi[o];
            // (w + i wi) exp(i (x + y)) with x = 2 pi i kl / N, y = 2 pi j km / N
            const double cx = cs[i * N + kl], sx = sn[i * N + kl];
            const double cy = cs[j * N + km], sy = sn[j * N + km];
            const double er = cx * cy - sx * sy, ei = sx * cy + cx * sy;
            re += w * er - wi * ei;
            im += w * ei + wi * er;
          }
          beta[((size_t)c * NG + km * N + kl) * A + a] = make_double2(re, im);
          bmax[c] = std::max(bmax[c], std::hypot(re, im));
        }
  const int qb = (A + 15) / 16;
  const int apad = 16 * qb;
  const int nacc = P == 2 ? 4 : 1;
  const size_t per_chunk = (size_t)C * nacc * 2 * NG * sizeof(double);
  const int max_chunks = (int)std::max<size_t>(1, std::min<size_t>(1024, (256ull << 20) / per_chunk));
  if (!x->sp_beta.alloc(beta.size() * sizeof(double2)) || !x->sp_betamax.alloc(C * sizeof(double)) ||
      !x->sp_bmat.alloc((size_t)C * P * epic::kSplitParts * 2 * NG * apad * sizeof(uint16_t)) ||
      !x->sp_scale.alloc((size_t)C * P * sizeof(float)) ||
      !x->sp_partial.alloc(per_chunk * max_chunks) ||
      hipMemcpy(x->sp_beta.p, beta.data(), beta.size() * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(x->sp_betamax.p, bmax.data(), C * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return x->fail(EPIC_E_NOMEM, "split-precision table allocation failed");
  x->sp_apad = apad;
  x->sp_qb = qb;
  x->sp_max_chunks = max_chunks;
  split_dispatch(P, x->cfg.precision == EPIC_SPLIT_BF16, qb, SplitOccupancy{x});
  return EPIC_OK;
}


epic_status run_split(epic_ctx* x, const uint8_t* efield, int64_t n_time, const float* gains,
                      double* image, int32_t reset) {
  const int N = x->cfg.grid_n, C = x->cfg.n_chan, P = x->cfg.n_pol, A = x->cfg.n_ant;
  const int NG = N * N;
  const bool bf = x->cfg.precision == EPIC_SPLIT_BF16;
  epic::SplitPrepArgs pa;
  pa.gains = reinterpret_cast<const float2*>(gains);
  pa.beta = x->sp_beta.as<double2>();
  pa.beta_max = x->sp_betamax.as<double>();
  pa.bmat = x->sp_bmat.as<uint16_t>();
  pa.scale = x->sp_scale.as<float>();
  pa.n_chan = C;
  pa.n_pol = P;
  pa.n_ant = A;
  pa.a_pad = x->sp_apad;
  pa.ng = NG;
  // chunks of about 256 matrix entries per workgroup (one per thread: the
  // work is latency-bound, not bandwidth-bound)
  const unsigned pchunks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, ((int64_t)NG * x->sp_apad + 255) / 256));
  const dim3 pgrid((unsigned)(C * P), pchunks);
  if (bf) hipLaunchKernelGGL(epic::split_prep_kernel<true>, pgrid, dim3(256), 0, x->stream, pa);
  else hipLaunchKernelGGL(epic::split_prep_kernel<false>, pgrid, dim3(256), 0, x->stream, pa);
  // tile groups of split_tpw(P, qb) 32-pixel tiles per wave; time chunks so
  // that the resident waves (the kernel's occupancy, queried once per
  // geometry) fill every SIMD, each at least 256 samples long
  const int qb = x->sp_qb;
  const int tpw = split_tpw(P, qb);
  // 8-byte sample loads need A % 8 == 0 and an 8-byte aligned E-field
  const bool vec = A % 8 == 0 && (reinterpret_cast<uintptr_t>(efield) & 7) == 0;
  const int64_t groups = (int64_t)(NG / 32 / tpw) * C;
  const int64_t want_waves = (int64_t)x->sp_wgs_per_cu[vec ? 1 : 0] * 4 * x->n_cu;
  int64_t n_ch = std::max<int64_t>(1, (want_waves + groups - 1) / groups);
  int64_t chunk = (n_time + n_ch - 1) / n_ch;
  chunk = std::max<int64_t>(256, (chunk + 31) / 32 * 32);
  chunk = std::max<int64_t>(chunk, (n_time + x->sp_max_chunks - 1) / x->sp_max_chunks);
  chunk = (chunk + 31) / 32 * 32;
  const int n_chunks = (int)((n_time + chunk - 1) / chunk);
  epic::SplitArgs sa;
  sa.efield = efield;
  sa.bmat = x->sp_bmat.as<uint16_t>();
  sa.partial = x->sp_partial.as<double>();
  sa.n_time = n_time;
  sa.n_chan = C;
  sa.n_ant = A;
  sa.a_pad = x->sp_apad;
  sa.ng = NG;
  sa.chunk = (int)chunk;
  sa.n_chunks = n_chunks;
  sa.tile_wgs = (NG / 32 / tpw + 3) / 4;
  const dim3 grid((unsigned)((int64_t)sa.tile_wgs * n_chunks * C));
  mark_main_begin(x);
  split_dispatch(P, bf, qb, SplitLaunch{x, &sa, grid, vec});
  x->last_kernel = "split_image_kernel";
  mark_main_end(x);
  epic::SplitReduceArgs ra;
  ra.partial = x->sp_partial.as<double>();
  ra.scale = x->sp_scale.as<float>();
  ra.image = image;
  ra.n_chan = C;
  ra.n_chunks = n_chunks;
  ra.ng = NG;
  ra.n = N;
  ra.reset = reset ? 1 : 0;
  ra.sub = reduce_sub(n_chunks);
  const int64_t rppb = 256 / ra.sub;
  const unsigned rg = (unsigned)(((int64_t)C * NG + rppb - 1) / rppb);
  if (P == 2) hipLaunchKernelGGL(epic::split_reduce_kernel<2>, dim3(rg), dim3(256), 0, x->stream, ra);
  else hipLaunchKernelGGL(epic::split_reduce_kernel<1>, dim3(rg), dim3(256), 0, x->stream, ra);
  return EPIC_OK;
}

unsigned grid_for(int64_t n, int64_t cap = 1 << 16) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cap, (n + 255) / 256));
}

// Exact per-antenna sums of e_P conj(e_Q) over the samples (auto_sum_kernel);
// returns the number of time segments (partial sums) written.
int launch_auto_sum(epic_ctx* x, const uint8_t* efield, int64_t n_time) {
  const int C = x->cfg.n_chan, A = x->cfg.n_ant, P = x->cfg.n_pol;
  const bool vec4 = A % 4 == 0 && (reinterpret_cast<uintptr_t>(efield) & 3) == 0;
  const int VEC = vec4 ? 4 : 1;
  const int64_t gx = ((int64_t)C * (A / VEC) + epic::AUTO_LANES - 1) / epic::AUTO_LANES;
  // as many time segments as keep every workgroup resident at once (one if
  // the antennas alone fill the GPU), at least 64 samples per segment
  int64_t nseg = std::max<int64_t>(1, (int64_t)x->n_cu * x->au_bpc[vec4 ? 1 : 0] / gx);
  nseg = std::min<int64_t>(nseg, std::max<int64_t>(1, n_time / 64));
  nseg = std::min<int64_t>(nseg, x->au_nseg_cap);
  epic::AutoSumArgs sa;
  sa.efield = efield;
  sa.part = x->au_part.as<int32_t>();
  sa.n_time = n_time;
  sa.n_chan = C;
  sa.n_ant = A;
  sa.nseg = (int)nseg;
  const dim3 sg((unsigned)gx, (unsigned)nseg), sb(epic::AUTO_LANES * epic::AUTO_TL);
  if (P == 2) {
    if (vec4) hipLaunchKernelGGL((epic::auto_sum_kernel<2, 4>), sg, sb, 0, x->stream, sa);
    else hipLaunchKernelGGL((epic::auto_sum_kernel<2, 1>), sg, sb, 0, x->stream, sa);
  } else {
    if (vec4) hipLaunchKernelGGL((epic::auto_sum_kernel<1, 4>), sg, sb, 0, x->stream, sa);
    else hipLaunchKernelGGL((epic::auto_sum_kernel<1, 1>), sg, sb, 0, x->stream, sa);
  }
  return (int)nseg;
}

// The segments' partial sums added into x->au_sums.
void launch_auto_fold(epic_ctx* x, int nseg) {
  epic::AutoFoldArgs fa;
  fa.part = x->au_part.as<int32_t>();
  fa.sums = x->au_sums.as<double>();
  fa.n = (int64_t)x->cfg.n_chan * x->cfg.n_ant;
  fa.nseg = nseg;
  const dim3 fg((unsigned)((fa.n + 255) / 256));
  if (x->cfg.n_pol == 2) hipLaunchKernelGGL(epic::auto_fold_kernel<2>, fg, dim3(256), 0, x->stream, fa);
  else hipLaunchKernelGGL(epic::auto_fold_kernel<1>, fg, dim3(256), 0, x->stream, fa);
}

// Autocorrelation sums and the per-channel table of the removed term.
void launch_auto_table(epic_ctx* x, const uint8_t* efield, int64_t n_time, const float* gains) {
  const int C = x->cfg.n_chan, A = x->cfg.n_ant, P = x->cfg.n_pol;
  const int K = x->cfg.kernel_support, D2 = (2 * K - 1) * (2 * K - 1);
  if (x->timing) (void)hipEventRecord(x->ev[3], x->stream);
  const int nseg = launch_auto_sum(x, efield, n_time);
  if (x->timing) (void)hipEventRecord(x->ev[4], x->stream);
  launch_auto_fold(x, nseg);
  epic::AutoTableArgs ta;
  ta.sums = x->au_sums.as<double>();
  ta.gains = reinterpret_cast<const float2*>(gains);
  ta.w = x->au_w.as<float>();
  ta.wi = x->cpx ? x->au_wi.as<float>() : nullptr;
  ta.table = x->au_tab.as<double>();
  ta.n_chan = C;
  ta.n_ant = A;
  const dim3 tg((unsigned)((int64_t)8 * ((C + 7) / 8) * ((D2 + 3) / 4)));
#define EPIC_AT(PP, KK_)                                                                           \
  if (P == PP && K == KK_) {                                                                       \
    if (x->cpx) hipLaunchKernelGGL((epic::auto_table_kernel<PP, KK_, true>), tg, dim3(256), 0,      \
                                   x->stream, ta);                                                 \
    else hipLaunchKernelGGL((epic::auto_table_kernel<PP, KK_, false>), tg, dim3(256), 0, x->stream, \
                            ta);                                                                   \
  }
  EPIC_AT(1, 1) EPIC_AT(1, 3) EPIC_AT(1, 5) EPIC_AT(1, 7)
  EPIC_AT(2, 1) EPIC_AT(2, 3) EPIC_AT(2, 5) EPIC_AT(2, 7)
#undef EPIC_AT
}

// Subtract the removed term (table from launch_auto_table) from the image.
void launch_auto_remove(epic_ctx* x, double* image) {
  const int C = x->cfg.n_chan, P = x->cfg.n_pol, N = x->cfg.grid_n, K = x->cfg.kernel_support;
  epic::AutoRemoveArgs ra;
  ra.table = x->au_tab.as<double>();
  ra.image = reinterpret_cast<double2*>(image);
  ra.n_chan = C;
  ra.N = N;
  ra.K = K;
  ra.cpx = x->cpx ? 1 : 0;
  const dim3 rg((unsigned)((int64_t)C * ((N * N + 255) / 256)));
  if (P == 2) hipLaunchKernelGGL(epic::auto_remove_kernel<2>, rg, dim3(256), 0, x->stream, ra);
  else hipLaunchKernelGGL(epic::auto_remove_kernel<1>, rg, dim3(256), 0, x->stream, ra);
}

// Gradient of the removed autocorrelation term into x->au_gauto.
void launch_autos_grad(epic_ctx* x, const uint8_t* efield, int64_t n_time, const float* gains,
                       const double* grad_image) {
  const int C = x->cfg.n_chan, A = x->cfg.n_ant, P = x->cfg.n_pol, N = x->cfg.grid_n;
  const int K = x->cfg.kernel_support, D2 = (2 * K - 1) * (2 * K - 1);
  launch_auto_fold(x, launch_auto_sum(x, efield, n_time));
  epic::AutoHatArgs ha;
  ha.grad_image = reinterpret_cast<const double2*>(grad_image);
  ha.hat = x->au_hat.as<double>();
  ha.n_chan = C;
  ha.N = N;
  ha.K = K;
  const dim3 hg((unsigned)((int64_t)8 * ((C + 7) / 8) * D2));
  if (P == 2) {
    if (x->cpx) hipLaunchKernelGGL((epic::auto_hat_kernel<2, true>), hg, dim3(256), 0, x->stream, ha);
    else hipLaunchKernelGGL((epic::auto_hat_kernel<2, false>), hg, dim3(256), 0, x->stream, ha);
  } else {
    if (x->cpx) hipLaunchKernelGGL((epic::auto_hat_kernel<1, true>), hg, dim3(256), 0, x->stream, ha);
    else hipLaunchKernelGGL((epic::auto_hat_kernel<1, false>), hg, dim3(256), 0, x->stream, ha);
  }
  epic::AutoGradArgs ga;
  ga.sums = x->au_sums.as<double>();
  ga.gains = reinterpret_cast<const float2*>(gains);
  ga.w = x->au_w.as<float>();
  ga.wi = x->cpx ? x->au_wi.as<float>() : nullptr;
  ga.hat = x->au_hat.as<double>();
  ga.gauto = x->au_gauto.as<double2>();
  ga.n_chan = C;
  ga.n_ant = A;
  const dim3 gg((unsigned)(((int64_t)C * A + 255) / 256));
#define EPIC_AG(PP, KK_)                                                                          \
  if (P == PP && K == KK_) {                                                                      \
    if (x->cpx) hipLaunchKernelGGL((epic::auto_grad_kernel<PP, KK_, true>), gg, dim3(256), 0,      \
                                   x->stream, ga);                                                \
    else hipLaunchKernelGGL((epic::auto_grad_kernel<PP, KK_, false>), gg, dim3(256), 0, x->stream, \
                            ga);                                                                  \
  }
  EPIC_AG(1, 1) EPIC_AG(1, 3) EPIC_AG(1, 5) EPIC_AG(1, 7)
  EPIC_AG(2, 1) EPIC_AG(2, 3) EPIC_AG(2, 5) EPIC_AG(2, 7)
#undef EPIC_AG
}

// Kernel taper of the current geometry (post.hpp), built on the context's
// stream at epic_set_antennas; the per-channel maxima are taken on the host.
epic_status build_taper(epic_ctx* x, const Geometry& g) {
  const int C = x->cfg.n_chan, A = x->cfg.n_ant, N = x->cfg.grid_n, K = x->cfg.kernel_support;
  const int D2 = (2 * K - 1) * (2 * K - 1);
  DevMem w, wi, coeff;
  const size_t nw = g.w.size();
  if (!w.alloc(nw * 4) || (!g.wi.empty() && !wi.alloc(nw * 4)) ||
      !coeff.alloc((size_t)C * D2 * sizeof(double2)) ||
      !x->taper.alloc((size_t)C * N * N * sizeof(double)) || !x->tmax.alloc((size_t)C * sizeof(double)) ||
      hipMemcpy(w.p, g.w.data(), nw * 4, hipMemcpyHostToDevice) != hipSuccess ||
      (!g.wi.empty() && hipMemcpy(wi.p, g.wi.data(), nw * 4, hipMemcpyHostToDevice) != hipSuccess))
    return x->fail(EPIC_E_NOMEM, "kernel taper allocation failed");
  (void)hipGetLastError();
  epic::TaperCoeffArgs ca;
  ca.w = w.as<float>();
  ca.wi = g.wi.empty() ? nullptr : wi.as<float>();
  ca.coeff = coeff.as<double2>();
  ca.n_chan = C;
  ca.n_ant = A;
  ca.K = K;
  hipLaunchKernelGGL(epic::taper_coeff_kernel, dim3((unsigned)((int64_t)C * ((D2 + 255) / 256))), dim3(256), 0,
                     x->stream, ca);
  epic::TaperImageArgs ia;
  ia.coeff = coeff.as<double2>();
  ia.taper = x->taper.as<double>();
  ia.n_chan = C;
  ia.n_ant = A;
  ia.N = N;
  ia.K = K;
  hipLaunchKernelGGL(epic::taper_image_kernel, dim3((unsigned)((int64_t)C * ((N * N + 255) / 256))),
                     dim3(256), 0, x->stream, ia);
  std::vector<double> t((size_t)C * N * N), mx(C, 0.0);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(x->stream) != hipSuccess ||
      hipMemcpy(t.data(), x->taper.p, t.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return x->fail(EPIC_E_DEVICE, "kernel taper computation failed");
  for (int c = 0; c < C; ++c)
    for (int i = 0; i < N * N; ++i) mx[c] = std::max(mx[c], t[(size_t)c * N * N + i]);
  if (hipMemcpy(x->tmax.p, mx.data(), C * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return x->fail(EPIC_E_DEVICE, "kernel taper upload failed");
  return EPIC_OK;
}

// The float32 paths: fused kernels, or the staged comparator.
// Arguments of a fused imaging launch over this context alone (one block,
// all channels); total and W are set by the caller.
epic::FusedArgs single_block_args(const epic_ctx* x, const uint8_t* efield, const float* gains,
                                  double* partial, int64_t n_time) {
  epic::FusedArgs a{};
  epic::FusedBlock& b = a.blk[0];
  b.efield = efield;
  b.gains = reinterpret_cast<const float2*>(gains);
  b.prog = x->prog.as<uint2>();
  b.wim = x->cpx ? x->prog_im.as<float>() : nullptr;
  b.c0 = 0;
  b.n_chan = x->cfg.n_chan;
  b.n_ant = x->cfg.n_ant;
  b.L = x->L;
  b.wrows = x->wide ? x->wide_rows : epic::FusedShape<64>::HW;
  a.n_blk = 1;
  a.twiddle = x->twiddle.as<float2>();
  a.partial = partial;
  a.n_time = n_time;
  a.total = (int64_t)x->cfg.n_chan * n_time;
  a.kblock = epic::FusedShape<64>::KBLOCK;
  a.xcd = 1;
  return a;
}

// Persistent grid of the fused imaging kernels for n_time samples: W
// workgroups in teams of `team` (FusedArgs), and the bytes of partial-image
// slots that grid writes.  max_team caps the team (the no-allocation call
// lowers it until the slots fit its array).
struct FusedGrid {
  int W, team;
  size_t slot_bytes;
};

FusedGrid fused_grid(const epic_ctx* x, int64_t n_time, int max_team = kMaxTeam) {
  const int N = x->cfg.grid_n, C = x->cfg.n_chan;
  const int64_t segs = N == 128 ? 2 * (int64_t)C : (int64_t)C;
  const int64_t units = segs * n_time;
  int w_cap;
  if (N == 128) w_cap = x->cpx ? x->fused_w_cpx : x->fused_w;
  else w_cap = x->wide ? (x->cpx ? x->fused_w_wide_cpx : x->fused_w_wide) : (x->cpx ? x->fused_w_cpx : x->fused_w);
  const int w_max = x->w_override > 0 ? std::min(x->w_override, w_cap) : w_cap;
  const int w0 = (int)std::min<int64_t>(w_max, units);
  FusedGrid g;
  g.team = std::min(team_for(n_time, x->team_override), max_team);
  while (g.team > 1 && g.team > w0) g.team /= 2;
  g.W = (w0 / g.team) * g.team;
  g.slot_bytes = (size_t)slot_count(segs, g.W, g.team) * fused_slot_values(N, x->nacc) * sizeof(double);
  return g;
}

// partial: the fused kernels' partial-image slots (the context's workspace,
// or the static scratch of the no-allocation call); unused on the staged path.
epic_status run_fp32(epic_ctx* x, const uint8_t* efield, int64_t n_time, const float* gains,
                     double* image, int32_t reset, double* partial, int max_team = kMaxTeam) {
  const int N = x->cfg.grid_n, C = x->cfg.n_chan, P = x->cfg.n_pol;
  const int64_t total = (int64_t)C * n_time;
  mark_main_begin(x);
  if (x->fused && N == 128) {
    epic::FusedArgs a = single_block_args(x, efield, gains, partial, n_time);
    a.total = 2 * total;
    const FusedGrid fg = fused_grid(x, n_time, max_team);
    a.W = fg.W;
    a.team = fg.team;
    if (!launch_fused128(x, a)) return x->fail(EPIC_E_UNSUPPORTED, "no fused kernel for this shape");
    x->last_kernel = "fused_image128_kernel";
    mark_main_end(x);
    epic::Reduce128Args r;
    r.partial = partial;
    r.image[0] = image;
    r.img_c0[0] = 0;
    r.n_img = 1;
    r.n_time = n_time;
    r.total = a.total;
    r.n_chan = C;
    r.W = a.W;
    r.team = a.team;
    r.kblock = a.kblock;
    r.reset = reset ? 1 : 0;
    r.sub = fused_reduce_sub(n_time, a.total, a.W, a.team);
    const int64_t n = (int64_t)C * N * N, ppb = 256 / r.sub;
    if (P == 2)
      hipLaunchKernelGGL(epic::reduce_image128_kernel<2>, dim3((unsigned)((n + ppb - 1) / ppb)), dim3(256), 0,
                         x->stream, r);
    else
      hipLaunchKernelGGL(epic::reduce_image128_kernel<1>, dim3((unsigned)((n + ppb - 1) / ppb)), dim3(256), 0,
                         x->stream, r);
  } else if (x->fused) {
    epic::FusedArgs a = single_block_args(x, efield, gains, partial, n_time);
    const FusedGrid fg = fused_grid(x, n_time, max_team);
    a.W = fg.W;
    a.team = fg.team;
    if (!launch_fused(x, a)) return x->fail(EPIC_E_UNSUPPORTED, "no fused kernel for this shape");
    x->last_kernel = x->wide ? "fused_wide_image_kernel" : "fused_image_kernel";
    mark_main_end(x);
    epic::ReduceArgs r;
    r.partial = partial;
    r.image[0] = image;
    r.img_c0[0] = 0;
    r.n_img = 1;
    r.n_time = n_time;
    r.total = total;
    r.n_chan = C;
    r.W = a.W;
    r.team = a.team;
    r.kblock = a.kblock;
    r.f32 = 1;
    r.reset = reset ? 1 : 0;
    r.sub = fused_reduce_sub(n_time, total, a.W, a.team);
    r.autos = nullptr;
    r.K = x->cfg.kernel_support;
    r.autos_cpx = x->cpx ? 1 : 0;
    r.transposed = x->transposed ? 1 : 0;
    if (x->autos) {
      launch_auto_table(x, efield, n_time, gains);
      r.autos = x->au_tab.as<double>();
    }
    launch_reduce(x, r, true);
  } else {
    const int npix = N * N;
    const int tbu = x->tb_override > 0 ? std::min(x->tb_override, x->tb) : x->tb;
    for (int64_t t0 = 0; t0 < n_time; t0 += tbu) {
      const int tb = (int)std::min<int64_t>(tbu, n_time - t0);
      epic::StagedUnpackArgs u;
      u.efield = efield;
      u.gains = reinterpret_cast<const float2*>(gains);
      u.e = x->st_e.as<float2>();
      u.t0 = t0;
      u.per_t = (int64_t)C * x->PA;
      u.count = tb * u.per_t;
      u.PA = x->PA;
      hipLaunchKernelGGL(epic::staged_unpack_kernel, dim3(grid_for(u.count)), dim3(256), 0,
                         x->stream, u);
      epic::StagedGridArgs gr;
      gr.e = x->st_e.as<float2>();
      gr.off = x->csr_off.as<int>();
      gr.ent = x->csr_ent.as<uint2>();
      gr.ent_im = x->cpx ? x->csr_im.as<float>() : nullptr;
      gr.grid = x->st_grid.as<float2>();
      gr.count = (int64_t)tb * C * P * npix;
      gr.n_chan = C;
      gr.n_pol = P;
      gr.n_ant = x->cfg.n_ant;
      gr.nnz = x->nnz;
      gr.npix = npix;
      hipLaunchKernelGGL(epic::staged_grid_kernel, dim3(grid_for(gr.count)), dim3(256), 0,
                         x->stream, gr);
      launch_staged_fft(x, x->st_grid.as<float2>(), (int64_t)tb * C * P);
      epic::StagedAccumArgs ac;
      ac.img = x->st_grid.as<float2>();
      ac.acc = x->st_acc.as<double>();
      ac.count = (int64_t)C * npix;
      ac.n_chan = C;
      ac.npix = npix;
      ac.tb = tb;
      ac.first = t0 == 0;
      if (P == 2)
        hipLaunchKernelGGL(epic::staged_accum_kernel<2>, dim3(grid_for(ac.count, 1 << 30)),
                           dim3(256), 0, x->stream, ac);
      else
        hipLaunchKernelGGL(epic::staged_accum_kernel<1>, dim3(grid_for(ac.count, 1 << 30)),
                           dim3(256), 0, x->stream, ac);
    }
    x->last_kernel = "staged_fft_kernel";
    mark_main_end(x);
    epic::ReduceArgs r;
    r.partial = x->st_acc.as<double>();
    r.image[0] = image;
    r.img_c0[0] = 0;
    r.n_img = 1;
    r.n_time = n_time;
    r.total = total;
    r.n_chan = C;
    r.W = 1;
    r.team = 1;
    r.kblock = epic::FusedShape<64>::KBLOCK;
    r.f32 = 0;
    r.reset = reset ? 1 : 0;
    r.sub = 1;
    r.autos = nullptr;
    r.K = x->cfg.kernel_support;
    r.autos_cpx = x->cpx ? 1 : 0;
    r.transposed = 0;
    if (x->autos) {
      launch_auto_table(x, efield, n_time, gains);
      r.autos = x->au_tab.as<double>();
    }
    launch_reduce(x, r, false);
  }
  return EPIC_OK;
}

// Gain gradient on the staged kernels (EPIC_FLAG_STAGED, or apertures wider
// than N/2): per batch, the forward stages, then the adjoint stages of
// staged.hpp, float64 sums per (channel, polarisation, antenna) in time order.
epic_status staged_backward(epic_ctx* x, const uint8_t* efield, int64_t n_time, const float* gains,
                            const double* grad_image, float* grad_gains) {
  const int N = x->cfg.grid_n, C = x->cfg.n_chan, P = x->cfg.n_pol, npix = N * N;
  (void)hipGetLastError();
  {
    epic::StagedGradTableArgs ta;
    ta.grad_image = reinterpret_cast<const double2*>(grad_image);
    ta.gtab = x->gtab.as<float4>();
    ta.n_chan = C;
    ta.N = N;
    const dim3 tg((unsigned)(((int64_t)C * npix + 255) / 256));
    if (P == 2) hipLaunchKernelGGL(epic::staged_grad_table_kernel<2>, tg, dim3(256), 0, x->stream, ta);
    else hipLaunchKernelGGL(epic::staged_grad_table_kernel<1>, tg, dim3(256), 0, x->stream, ta);
  }
  mark_main_begin(x);
  const int tbu = x->tb_override > 0 ? std::min(x->tb_override, x->tb) : x->tb;
  for (int64_t t0 = 0; t0 < n_time; t0 += tbu) {
    const int tb = (int)std::min<int64_t>(tbu, n_time - t0);
    epic::StagedUnpackArgs u;
    u.efield = efield;
    u.gains = reinterpret_cast<const float2*>(gains);
    u.e = x->st_e.as<float2>();
    u.t0 = t0;
    u.per_t = (int64_t)C * x->PA;
    u.count = tb * u.per_t;
    u.PA = x->PA;
    hipLaunchKernelGGL(epic::staged_unpack_kernel, dim3(grid_for(u.count)), dim3(256), 0, x->stream, u);
    epic::StagedGridArgs gr;
    gr.e = x->st_e.as<float2>();
    gr.off = x->csr_off.as<int>();
    gr.ent = x->csr_ent.as<uint2>();
    gr.ent_im = x->cpx ? x->csr_im.as<float>() : nullptr;
    gr.grid = x->st_grid.as<float2>();
    gr.count = (int64_t)tb * C * P * npix;
    gr.n_chan = C;
    gr.n_pol = P;
    gr.n_ant = x->cfg.n_ant;
    gr.nnz = x->nnz;
    gr.npix = npix;
    hipLaunchKernelGGL(epic::staged_grid_kernel, dim3(grid_for(gr.count)), dim3(256), 0, x->stream, gr);
    launch_staged_fft(x, x->st_grid.as<float2>(), (int64_t)tb * C * P);
    epic::StagedGformArgs gf;
    gf.img = x->st_grid.as<float2>();
    gf.gtab = x->gtab.as<float4>();
    gf.count = (int64_t)tb * C * npix;
    gf.n_chan = C;
    gf.npix = npix;
    if (P == 2) hipLaunchKernelGGL(epic::staged_gform_kernel<2>, dim3(grid_for(gf.count)), dim3(256), 0, x->stream, gf);
    else hipLaunchKernelGGL(epic::staged_gform_kernel<1>, dim3(grid_for(gf.count)), dim3(256), 0, x->stream, gf);
    launch_staged_fft(x, x->st_grid.as<float2>(), (int64_t)tb * C * P);
    epic::StagedDegridArgs dg;
    dg.img = x->st_grid.as<float2>();
    dg.efield = efield;
    dg.taps = x->taps.as<uint2>();
    dg.tapim = x->cpx ? x->taps_im.as<float>() : nullptr;
    dg.gsum = x->gpartial.as<double2>();
    dg.t0 = t0;
    dg.tb = tb;
    dg.n_chan = C;
    dg.n_ant = x->cfg.n_ant;
    dg.kk = x->cfg.kernel_support * x->cfg.kernel_support;
    dg.npix = npix;
    dg.PA = x->PA;
    dg.first = t0 == 0;
    hipLaunchKernelGGL(epic::staged_degrid_kernel, dim3((unsigned)(((int64_t)C * x->PA + 255) / 256)),
                       dim3(256), 0, x->stream, dg);
  }
  x->last_kernel = "staged_degrid_kernel";
  mark_main_end(x);
  if (x->autos) launch_autos_grad(x, efield, n_time, gains, grad_image);
  // 2 dL/dg* (minus the autocorrelation term) from the single slot per channel
  epic::GradReduceArgs r;
  r.gpartial = x->gpartial.as<double2>();
  r.grad = reinterpret_cast<float2*>(grad_gains);
  r.n_time = n_time;
  r.total = (int64_t)C * n_time;
  r.n_chan = C;
  r.PA = x->PA;
  r.W = 1;
  r.sub = 1;
  r.minus = x->autos ? x->au_gauto.as<double2>() : nullptr;
  const int64_t n = (int64_t)C * x->PA;
  hipLaunchKernelGGL(epic::reduce_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, x->stream, r);
  if (x->timing) {
    (void)hipEventRecord(x->ev[2], x->stream);
    x->timed = true;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return x->fail(EPIC_E_LAUNCH, std::string("launch failed: ") + hipGetErrorString(e));
  return EPIC_OK;
}

// After the imaging kernels of an accumulate call: the autocorrelation pass
// where the reduction does not subtract it (N = 128, split), the closing
// timing event, the launch status.
epic_status finish_accumulate(epic_ctx* x, const uint8_t* efield, int64_t n_time, const float* gains,
                              double* image) {
  // the N <= 64 reductions subtract the table themselves; the others need a pass
  if (x->autos && (x->cfg.precision != EPIC_FP32 || (x->fused && x->cfg.grid_n == 128))) {
    launch_auto_table(x, efield, n_time, gains);
    launch_auto_remove(x, image);
  }
  x->autos_timed = x->autos && x->timing;
  if (x->timing) {
    (void)hipEventRecord(x->ev[2], x->stream);
    x->timed = true;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return x->fail(EPIC_E_LAUNCH, std::string("launch failed: ") + hipGetErrorString(e));
  return EPIC_OK;
}

}  // namespace

extern "C" {

epic_status epic_init(const epic_config* cfg, int device, void* hip_stream, epic_ctx** out) {
  g_init_error.clear();
  if (!out) { g_init_error = "out is NULL"; return EPIC_E_INVALID; }
  *out = nullptr;
  std::string m;
  epic_status s = check_config(cfg, m);
  if (s == EPIC_OK && cfg->precision != EPIC_FP32) s = check_split(cfg, m);
  if (s != EPIC_OK) { g_init_error = m; return s; }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    g_init_error = "no such HIP device";
    return EPIC_E_DEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    g_init_error = "hipGetDeviceProperties failed";
    return EPIC_E_DEVICE;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    g_init_error = std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950";
    return EPIC_E_DEVICE;
  }
  DeviceGuard guard(device);
  epic_ctx* x = new (std::nothrow) epic_ctx();
  if (!x) { g_init_error = "host allocation failed"; return EPIC_E_NOMEM; }
  x->cfg = *cfg;
  x->device = device;
  x->scratch = scratch_address(device);
  x->stream = static_cast<hipStream_t>(hip_stream);
  x->nprod = cfg->n_pol == 2 ? 4 : 1;
  x->nacc = cfg->n_pol == 2 ? 4 : 1;
  x->PA = cfg->n_pol * cfg->n_ant;
  x->n_cu = prop.multiProcessorCount;
  const int N = cfg->grid_n;

  // twiddles exp(+2 pi i k / N), float64 then rounded once
  std::vector<float2> tw(N);
  for (int k = 0; k < N; ++k) {
    const double ang = 2.0 * M_PI * (double)k / (double)N;
    tw[k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  if (!x->twiddle.alloc(N * sizeof(float2)) ||
      hipMemcpy(x->twiddle.p, tw.data(), N * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) {
    g_init_error = "twiddle table allocation failed";
    delete x;
    return EPIC_E_NOMEM;
  }

  const bool want_staged = (cfg->flags & EPIC_FLAG_STAGED) != 0;
  // fused kernels: N = 32, 64 and 128, one or two polarisations
  x->fused_ok = !want_staged && cfg->precision == EPIC_FP32;
  if (x->fused_ok) {
    const int NT = fused_threads(N);
    int gpt = (x->PA + NT - 1) / NT;
    gpt = gpt <= 1 ? 1 : gpt <= 2 ? 2 : gpt <= 4 ? 4 : 0;
    if (gpt == 0) x->fused_ok = false;
    else x->fused_gpt = gpt;
  }
  if (x->fused_ok) {
    const int bpc = fused_blocks_per_cu(N, cfg->n_pol, x->fused_gpt, false);
    x->fused_w = bpc * x->n_cu;
    // complex-kernel variants: never more workgroups than the slots allow
    x->fused_w_cpx = std::min(x->fused_w, fused_blocks_per_cu(N, cfg->n_pol, x->fused_gpt, true) * x->n_cu);
    if (N == 64) {
      x->fused_w_wide = std::min(x->fused_w, fused_wide_blocks_per_cu(cfg->n_pol, x->fused_gpt, false) * x->n_cu);
      x->fused_w_wide_cpx = std::min(x->fused_w, fused_wide_blocks_per_cu(cfg->n_pol, x->fused_gpt, true) * x->n_cu);
    }
    // N = 128: two accumulation segments (column parities) per channel; slots
    // for the largest team (FusedArgs)
    const int64_t segs = N == 128 ? 2 * (int64_t)cfg->n_chan : (int64_t)cfg->n_chan;
    const size_t slots = (size_t)max_slot_count(segs, x->fused_w);
    const size_t per_slot = fused_slot_values(N, x->nacc);
    if (!x->partial.alloc(slots * per_slot * sizeof(double))) {
      g_init_error = "partial-image workspace allocation failed";
      delete x;
      return EPIC_E_NOMEM;
    }
    x->adj_w = adjoint_blocks_per_cu(N, cfg->n_pol, x->fused_gpt, false) * x->n_cu;
    x->adj_w_cpx = std::min(x->adj_w, adjoint_blocks_per_cu(N, cfg->n_pol, x->fused_gpt, true) * x->n_cu);
    if (N == 64) {
      x->adj_w_wide = std::min(x->adj_w, adjoint_wide_blocks_per_cu(cfg->n_pol, x->fused_gpt, false) * x->n_cu);
      x->adj_w_wide_cpx = std::min(x->adj_w, adjoint_wide_blocks_per_cu(cfg->n_pol, x->fused_gpt, true) * x->n_cu);
    }
    const size_t gslots = (size_t)x->adj_w + cfg->n_chan - 1;
    if (!x->gpartial.alloc(gslots * x->PA * 2 * sizeof(double)) ||
        !x->gtab.alloc((size_t)cfg->n_chan * N * N * sizeof(float4))) {
      g_init_error = "gradient workspace allocation failed";
      delete x;
      return EPIC_E_NOMEM;
    }
  }
  if ((cfg->flags & EPIC_FLAG_REMOVE_AUTOS) && cfg->kernel_support > epic::AUTO_MAX_K) {
    g_init_error = "EPIC_FLAG_REMOVE_AUTOS takes kernel_support <= 7";
    delete x;
    return EPIC_E_UNSUPPORTED;
  }
  if (cfg->flags & EPIC_FLAG_REMOVE_AUTOS) {
    const int NQ = cfg->n_pol == 2 ? 4 : 1, D = 2 * cfg->kernel_support - 1;
    const size_t per_seg = (size_t)cfg->n_chan * cfg->n_ant * NQ * sizeof(int32_t);
    x->autos = true;
    const int st = epic::AUTO_LANES * epic::AUTO_TL;
    x->au_bpc[0] = cfg->n_pol == 2 ? occupancy_blocks(epic::auto_sum_kernel<2, 1>, st)
                                   : occupancy_blocks(epic::auto_sum_kernel<1, 1>, st);
    x->au_bpc[1] = cfg->n_pol == 2 ? occupancy_blocks(epic::auto_sum_kernel<2, 4>, st)
                                   : occupancy_blocks(epic::auto_sum_kernel<1, 4>, st);
    x->au_nseg_cap = (int)std::max<size_t>(1, std::min<size_t>(epic::AUTO_MAX_SEG, (256u << 20) / per_seg));
    if (!x->au_part.alloc(x->au_nseg_cap * per_seg) ||
        !x->au_tab.alloc((size_t)cfg->n_chan * D * D * 2 * NQ * sizeof(double)) ||
        !x->au_sums.alloc((size_t)cfg->n_chan * cfg->n_ant * NQ * sizeof(double)) ||
        !x->au_hat.alloc((size_t)cfg->n_chan * D * D * 2 * NQ * sizeof(double)) ||
        !x->au_gauto.alloc((size_t)cfg->n_chan * x->PA * 2 * sizeof(double))) {
      g_init_error = "autocorrelation workspace allocation failed";
      delete x;
      return EPIC_E_NOMEM;
    }
  }
  if (cfg->flags & EPIC_FLAG_TIMING) {
    x->timing = true;
    x->ring.assign(2 * epic_ctx::kTimingRing, nullptr);
    bool ok = true;
    for (auto& e : x->ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    for (auto& e : x->ring) ok = ok && hipEventCreate(&e) == hipSuccess;
    if (!ok) {
      g_init_error = "hipEventCreate failed";
      epic_destroy(x);
      return EPIC_E_DEVICE;
    }
  }
  *out = x;
  return EPIC_OK;
}

epic_status epic_set_stream(epic_ctx* x, void* hip_stream) {
  if (!x) return EPIC_E_INVALID;
  x->stream = static_cast<hipStream_t>(hip_stream);
  return EPIC_OK;
}

epic_status epic_gridding_program(const epic_config* cfg, const double* xy_m, const double* freq_hz,
                                  uint32_t* out, int64_t* words, int32_t* layout) {
  g_init_error.clear();
  std::string m;
  epic_status s = check_config(cfg, m);
  if (s != EPIC_OK) { g_init_error = m; return s; }
  if (!xy_m || !freq_hz || !words || !layout) { g_init_error = "null pointer"; return EPIC_E_INVALID; }
  const int N = cfg->grid_n, P = cfg->n_pol;
  if (cfg->precision != EPIC_FP32 || (cfg->flags & EPIC_FLAG_STAGED)) {
    g_init_error = "the configuration has no fused kernel";
    return EPIC_E_UNSUPPORTED;
  }
  const int NT = fused_threads(N);
  int gpt = (P * cfg->n_ant + NT - 1) / NT;
  gpt = gpt <= 1 ? 1 : gpt <= 2 ? 2 : gpt <= 4 ? 4 : 0;
  if (gpt == 0) {
    g_init_error = "too many antennas for the fused kernel";
    return EPIC_E_UNSUPPORTED;
  }
  Geometry g;
  s = build_geometry(*cfg, xy_m, freq_hz, nullptr, g, m);
  if (s != EPIC_OK) { g_init_error = m; return s; }
  const bool wide = N == 64 && !g.fits_half && g.fits_wide;
  if (!g.fits_half && !wide) { g_init_error = "taps do not fit the fused kernels' aperture block"; return EPIC_E_UNSUPPORTED; }
  if (wide) orient_wide(g, N);
  std::vector<uint32_t> prog;
  int L = 0;
  if (N == 32) build_programs<32>(g, P, gpt, prog, L);
  else if (N == 64) build_programs<64>(g, P, gpt, prog, L, nullptr, wide);
  else build_programs<128>(g, P, gpt, prog, L);
  if (L == 0) { g_init_error = "gridding program fields overflow"; return EPIC_E_UNSUPPORTED; }
  const int64_t need = (int64_t)prog.size(), cap = *words;
  *words = need;
  const int ES = NT * gpt / P + 64;
  layout[0] = NT;
  layout[1] = L;
  layout[2] = N == 32 ? epic::FusedShape<32>::RS : N == 64 ? epic::FusedShape<64>::RS : epic::FusedShape<128>::RS;
  layout[3] = N == 32 ? epic::FusedShape<32>::PSTRIDE
            : N == 64 ? epic::FusedShape<64>::PSTRIDE : epic::FusedShape<128>::PSTRIDE;
  layout[4] = P * ES;
  layout[5] = ES;
  layout[6] = N == 64 ? 1 : 0;
  layout[7] = wide && g.transposed ? 1 : 0;
  layout[8] = wide ? g.wide_rows : N == 128 ? 64 : N / 2;
  layout[9] = wide ? epic::FusedShape<64>::HW : N == 128 ? 64 : N / 2;
  if (cap == 0) return EPIC_OK;
  if (!out || cap < need) { g_init_error = "output capacity too small"; return EPIC_E_NOMEM; }
  std::memcpy(out, prog.data(), prog.size() * sizeof(uint32_t));
  return EPIC_OK;
}

epic_status epic_set_antennas(epic_ctx* x, const double* xy_m, const double* freq_hz) {
  return epic_set_antennas_kernels(x, xy_m, freq_hz, nullptr);
}

epic_status epic_set_antennas_kernels(epic_ctx* x, const double* xy_m, const double* freq_hz,
                                      const float* kernels) {
  if (!x) return EPIC_E_INVALID;
  if (!xy_m || !freq_hz) return x->fail(EPIC_E_INVALID, "xy_m or freq_hz is NULL");
  Geometry g;
  std::string m;
  epic_status s = build_geometry(x->cfg, xy_m, freq_hz, kernels, g, m);
  if (s != EPIC_OK) return x->fail(s, m);
  DeviceGuard guard(x->device);
  const int N = x->cfg.grid_n, C = x->cfg.n_chan, A = x->cfg.n_ant, P = x->cfg.n_pol;
  if (hipStreamSynchronize(x->stream) != hipSuccess)
    return x->fail(EPIC_E_DEVICE, "stream synchronisation failed");
  x->have_geom = false;
  x->cpx = kernels != nullptr;
  if (x->autos &&
      (!x->au_w.alloc(g.w.size() * sizeof(float)) ||
       hipMemcpy(x->au_w.p, g.w.data(), g.w.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
       (x->cpx && (!x->au_wi.alloc(g.wi.size() * sizeof(float)) ||
                   hipMemcpy(x->au_wi.p, g.wi.data(), g.wi.size() * sizeof(float),
                             hipMemcpyHostToDevice) != hipSuccess))))
    return x->fail(EPIC_E_NOMEM, "kernel weight upload failed");
  s = build_taper(x, g);
  if (s != EPIC_OK) return s;
  if (x->cfg.precision != EPIC_FP32) {
    s = build_split_tables(x, g);
    if (s != EPIC_OK) return s;
    x->have_geom = true;
    return EPIC_OK;
  }
  // The fused kernels need every channel's taps inside an N/2 x N/2 block, or
  // at N = 64 inside a 3N/4 x 3N/4 block (wide variant); larger apertures
  // (aliased images) run the staged kernels.
  x->wide = x->fused_ok && N == 64 && !g.fits_half && g.fits_wide;
  x->fused = x->fused_ok && (g.fits_half || x->wide);
  if (x->wide) orient_wide(g, N);
  x->wide_rows = x->wide ? g.wide_rows : 0;
  x->transposed = x->wide && g.transposed;

  if (x->fused) {
    // adjoint taps [C][A][KK] {translated cell as a float2 offset in the
    // kernels' LDS grid (physical row times the row stride, plus column), w}
    const int RSN = N == 32 ? epic::FusedShape<32>::RS : N == 64 ? epic::FusedShape<64>::RS
                                                                 : epic::FusedShape<128>::RS;
    std::vector<uint32_t> taps((size_t)C * A * g.KK * 2);
    for (size_t o = 0; o < (size_t)C * A * g.KK; ++o) {
      const int j = g.tcell[o] / N, i = g.tcell[o] % N;
      taps[2 * o] = (uint32_t)((N == 64 ? epic::FusedShape<64>::phys_row(j) : j) * RSN + i);
      std::memcpy(&taps[2 * o + 1], &g.w[o], 4);
    }
    std::vector<uint32_t> prog;
    std::vector<float> prog_im;
    int L = 0;
    if (N == 32) build_programs<32>(g, P, x->fused_gpt, prog, L, &prog_im);
    else if (N == 64) build_programs<64>(g, P, x->fused_gpt, prog, L, &prog_im, x->wide);
    else build_programs<128>(g, P, x->fused_gpt, prog, L, &prog_im);
    if (L == 0) return x->fail(EPIC_E_UNSUPPORTED, "gridding program fields overflow");
    if (!x->taps.alloc(taps.size() * 4) || !x->prog.alloc(prog.size() * 4) ||
        hipMemcpy(x->taps.p, taps.data(), taps.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(x->prog.p, prog.data(), prog.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
      return x->fail(EPIC_E_NOMEM, "gridding program upload failed");
    if (x->cpx &&
        (!x->prog_im.alloc(prog_im.size() * 4) || !x->taps_im.alloc(g.wi.size() * 4) ||
         hipMemcpy(x->prog_im.p, prog_im.data(), prog_im.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
         hipMemcpy(x->taps_im.p, g.wi.data(), g.wi.size() * 4, hipMemcpyHostToDevice) != hipSuccess))
      return x->fail(EPIC_E_NOMEM, "gridding program upload failed");
    x->L = L;
  } else {
    if (!alloc_staged(x)) return x->fail(EPIC_E_NOMEM, "staged workspace allocation failed");
    // per-cell CSR over the whole grid, entries in (antenna, tap) order
    const int npix = N * N, nnz = A * g.KK;
    std::vector<int> off((size_t)C * (npix + 1));
    std::vector<uint32_t> ent((size_t)C * nnz * 2);
    std::vector<float> ent_im(x->cpx ? (size_t)C * nnz : 0);
    for (int c = 0; c < C; ++c) {
      std::vector<int> cnt(npix, 0);
      for (int a = 0; a < A; ++a)
        for (int k = 0; k < g.KK; ++k) cnt[g.cell[((size_t)c * A + a) * g.KK + k]]++;
      int* o = &off[(size_t)c * (npix + 1)];
      o[0] = 0;
      for (int i = 0; i < npix; ++i) o[i + 1] = o[i] + cnt[i];
      std::vector<int> fill(o, o + npix);
      for (int a = 0; a < A; ++a)
        for (int k = 0; k < g.KK; ++k) {
          const size_t src = ((size_t)c * A + a) * g.KK + k;
          const size_t dst = (size_t)c * nnz + fill[g.cell[src]]++;
          ent[2 * dst] = (uint32_t)a;
          std::memcpy(&ent[2 * dst + 1], &g.w[src], 4);
          if (x->cpx) ent_im[dst] = g.wi[src];
        }
    }
    if (!x->csr_off.alloc(off.size() * 4) || !x->csr_ent.alloc(ent.size() * 4) ||
        hipMemcpy(x->csr_off.p, off.data(), off.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(x->csr_ent.p, ent.data(), ent.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
      return x->fail(EPIC_E_NOMEM, "gridding table upload failed");
    if (x->cpx && (!x->csr_im.alloc(ent_im.size() * 4) ||
                   hipMemcpy(x->csr_im.p, ent_im.data(), ent_im.size() * 4, hipMemcpyHostToDevice) != hipSuccess))
      return x->fail(EPIC_E_NOMEM, "gridding table upload failed");
    x->nnz = nnz;
    // degridding taps of the staged gradient [C][A][KK] {cell j*N + i, w}
    std::vector<uint32_t> taps((size_t)C * A * g.KK * 2);
    for (size_t o = 0; o < (size_t)C * A * g.KK; ++o) {
      taps[2 * o] = (uint32_t)g.cell[o];
      std::memcpy(&taps[2 * o + 1], &g.w[o], 4);
    }
    if (!x->taps.alloc(taps.size() * 4) ||
        hipMemcpy(x->taps.p, taps.data(), taps.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        (x->cpx && (!x->taps_im.alloc(g.wi.size() * 4) ||
                    hipMemcpy(x->taps_im.p, g.wi.data(), g.wi.size() * 4, hipMemcpyHostToDevice) != hipSuccess)))
      return x->fail(EPIC_E_NOMEM, "degridding table upload failed");
  }
  x->have_geom = true;
  return EPIC_OK;
}

epic_status epic_image_accumulate(epic_ctx* x, const uint8_t* efield, int64_t n_time,
                                  const float* gains, double* image, int32_t reset) {
  if (!x) return EPIC_E_INVALID;
  if (!x->have_geom) return x->fail(EPIC_E_STATE, "epic_set_antennas has not succeeded");
  if (!efield || !gains || !image) return x->fail(EPIC_E_INVALID, "NULL device pointer");
  if (n_time <= 0) return x->fail(EPIC_E_INVALID, "n_time must be positive");
  if (x->autos && n_time > epic::AUTO_SEG_MAX_SAMPLES)
    return x->fail(EPIC_E_UNSUPPORTED, "with EPIC_FLAG_REMOVE_AUTOS a call takes at most 2^24 - 1 samples");
  DeviceGuard guard(x->device);
  (void)hipGetLastError();
  const epic_status s = x->cfg.precision != EPIC_FP32
                            ? run_split(x, efield, n_time, gains, image, reset)
                            : run_fp32(x, efield, n_time, gains, image, reset, x->partial.as<double>());
  if (s != EPIC_OK) return s;
  return finish_accumulate(x, efield, n_time, gains, image);
}

epic_status epic_image_accumulate_noalloc(epic_ctx* x, const uint8_t* efield, int64_t n_time,
                                          const float* gains, double* image, int32_t reset) {
  if (!x) return EPIC_E_INVALID;
  if (!x->have_geom) return x->fail(EPIC_E_STATE, "epic_set_antennas has not succeeded");
  if (!efield || !gains || !image) return x->fail(EPIC_E_INVALID, "NULL device pointer");
  if (n_time <= 0) return x->fail(EPIC_E_INVALID, "n_time must be positive");
  if (x->autos && n_time > epic::AUTO_SEG_MAX_SAMPLES)
    return x->fail(EPIC_E_UNSUPPORTED, "with EPIC_FLAG_REMOVE_AUTOS a call takes at most 2^24 - 1 samples");
  if (x->cfg.precision != EPIC_FP32 || !x->fused)
    return x->fail(EPIC_E_UNSUPPORTED,
                   "the no-allocation call runs the fused float32 kernels only (not the staged or split paths)");
  if (!x->scratch)
    return x->fail(EPIC_E_DEVICE, "the static scratch array has no device address on this device");
  // the largest team whose slots fit the array
  int max_team = kMaxTeam;
  FusedGrid fg = fused_grid(x, n_time, max_team);
  while (fg.slot_bytes > kScratchBytes && max_team > 1) {
    max_team /= 2;
    fg = fused_grid(x, n_time, max_team);
  }
  if (fg.slot_bytes > kScratchBytes)
    return x->fail(EPIC_E_UNSUPPORTED,
                   "this call needs " + std::to_string(fg.slot_bytes) + " bytes of partial-image slots; the "
                   "static scratch holds " + std::to_string(kScratchBytes) + " (fewer channels per call fit)");
  DeviceGuard guard(x->device);
  (void)hipGetLastError();
  const epic_status s =
      run_fp32(x, efield, n_time, gains, image, reset, static_cast<double*>(x->scratch), max_team);
  if (s != EPIC_OK) return s;
  return finish_accumulate(x, efield, n_time, gains, image);
}
epic_status epic_image_backward(epic_ctx* x, const uint8_t* efield, int64_t n_time,
                                const float* gains, const double* grad_image, float* grad_gains) {
  if (!x) return EPIC_E_INVALID;
  if (!x->have_geom) return x->fail(EPIC_E_STATE, "epic_set_antennas has not succeeded");
  if (!efield || !gains || !grad_image || !grad_gains)
    return x->fail(EPIC_E_INVALID, "NULL device pointer");
  if (n_time <= 0) return x->fail(EPIC_E_INVALID, "n_time must be positive");
  if (x->autos && n_time > epic::AUTO_SEG_MAX_SAMPLES)
    return x->fail(EPIC_E_UNSUPPORTED, "with EPIC_FLAG_REMOVE_AUTOS a call takes at most 2^24 - 1 samples");
  if (x->cfg.precision != EPIC_FP32)
    return x->fail(EPIC_E_UNSUPPORTED, "the gain gradient runs on the float32 paths");
  DeviceGuard guard(x->device);
  if (!x->fused) return staged_backward(x, efield, n_time, gains, grad_image, grad_gains);
  const int C = x->cfg.n_chan;
  // work units per channel: samples, or (parity, sample) pairs at N = 128
  const int64_t upc = x->cfg.grid_n == 128 ? 2 * n_time : n_time;
  const int64_t total = (int64_t)C * upc;
  (void)hipGetLastError();
  {
    epic::GradTableArgs ta;
    ta.grad_image = reinterpret_cast<const double2*>(grad_image);
    ta.gtab = x->gtab.as<float4>();
    ta.n_chan = C;
    ta.transposed = x->transposed ? 1 : 0;
    const int N = x->cfg.grid_n, P = x->cfg.n_pol;
    const dim3 tg((unsigned)(((int64_t)C * N * N + 255) / 256));
    if (N == 32 && P == 1) hipLaunchKernelGGL((epic::grad_table_kernel<32, 1>), tg, dim3(256), 0, x->stream, ta);
    else if (N == 32) hipLaunchKernelGGL((epic::grad_table_kernel<32, 2>), tg, dim3(256), 0, x->stream, ta);
    else if (N == 64 && P == 1) hipLaunchKernelGGL((epic::grad_table_kernel<64, 1>), tg, dim3(256), 0, x->stream, ta);
    else if (N == 64) hipLaunchKernelGGL((epic::grad_table_kernel<64, 2>), tg, dim3(256), 0, x->stream, ta);
    else if (P == 1) hipLaunchKernelGGL((epic::grad_table128_kernel<1>), tg, dim3(256), 0, x->stream, ta);
    else hipLaunchKernelGGL((epic::grad_table128_kernel<2>), tg, dim3(256), 0, x->stream, ta);
  }
  mark_main_begin(x);
  epic::AdjointArgs a;
  a.efield = efield;
  a.gains = reinterpret_cast<const float2*>(gains);
  a.gtab = x->gtab.as<float4>();
  a.prog = x->prog.as<uint2>();
  a.wim = x->cpx ? x->prog_im.as<float>() : nullptr;
  a.taps = x->taps.as<uint2>();
  a.tapim = x->cpx ? x->taps_im.as<float>() : nullptr;
  a.twiddle = x->twiddle.as<float2>();
  a.gpartial = x->gpartial.as<double2>();
  a.n_time = n_time;
  a.total = total;
  a.n_chan = C;
  a.n_ant = x->cfg.n_ant;
  a.kk = x->cfg.kernel_support * x->cfg.kernel_support;
  a.L = x->L;
  a.wrows = x->wide ? x->wide_rows : epic::FusedShape<64>::HW;
  const int aw = x->wide ? (x->cpx ? x->adj_w_wide_cpx : x->adj_w_wide) : (x->cpx ? x->adj_w_cpx : x->adj_w);
  a.W = (int)std::min<int64_t>(aw, total);
  if (!launch_adjoint(x, a)) return x->fail(EPIC_E_UNSUPPORTED, "no adjoint kernel for this shape");
  x->last_kernel = x->cfg.grid_n == 128 ? "adjoint128_kernel" : x->wide ? "adjoint_wide_kernel" : "adjoint_kernel";
  mark_main_end(x);
  if (x->autos) launch_autos_grad(x, efield, n_time, gains, grad_image);
  epic::GradReduceArgs r;
  r.gpartial = x->gpartial.as<double2>();
  r.grad = reinterpret_cast<float2*>(grad_gains);
  r.n_time = upc;                              // the kernel's units per channel
  r.total = total;
  r.n_chan = C;
  r.PA = x->PA;
  r.W = a.W;
  r.sub = reduce_sub(slots_per_channel(upc, total, a.W));
  r.minus = x->autos ? x->au_gauto.as<double2>() : nullptr;
  const int64_t n = (int64_t)C * x->PA, gppb = 256 / r.sub;
  hipLaunchKernelGGL(epic::reduce_grad_kernel, dim3((unsigned)((n + gppb - 1) / gppb)), dim3(256), 0,
                     x->stream, r);
  if (x->timing) {
    (void)hipEventRecord(x->ev[2], x->stream);
    x->timed = true;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return x->fail(EPIC_E_LAUNCH, std::string("launch failed: ") + hipGetErrorString(e));
  return EPIC_OK;
}

epic_status epic_last_timing(epic_ctx* x, float* main_ms, float* call_ms) {
  if (!x) return EPIC_E_INVALID;
  if (!x->timing || !x->timed) return x->fail(EPIC_E_STATE, "no timed call (EPIC_FLAG_TIMING)");
  DeviceGuard guard(x->device);
  if (hipEventSynchronize(x->ev[2]) != hipSuccess) return x->fail(EPIC_E_DEVICE, "event wait failed");
  float m = 0.f, c = 0.f;
  (void)hipEventElapsedTime(&m, x->ev[0], x->ev[1]);
  (void)hipEventElapsedTime(&c, x->ev[0], x->ev[2]);
  if (main_ms) *main_ms = m;
  if (call_ms) *call_ms = c;
  return EPIC_OK;
}

epic_status epic_timing_history(epic_ctx* x, int32_t n, float* main_ms) {
  if (!x) return EPIC_E_INVALID;
  if (!x->timing) return x->fail(EPIC_E_STATE, "timing history needs EPIC_FLAG_TIMING");
  if (!main_ms || n < 1 || n > epic_ctx::kTimingRing)
    return x->fail(EPIC_E_INVALID, "n must be 1 .. 256 with an output array");
  if (x->ring_calls < n) return x->fail(EPIC_E_STATE, "fewer timed calls than requested");
  DeviceGuard guard(x->device);
  const int64_t last = x->ring_calls - 1;
  if (hipEventSynchronize(x->ring[2 * (last % epic_ctx::kTimingRing) + 1]) != hipSuccess)
    return x->fail(EPIC_E_DEVICE, "event wait failed");
  for (int32_t i = 0; i < n; ++i) {
    const int64_t slot = (x->ring_calls - n + i) % epic_ctx::kTimingRing;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, x->ring[2 * slot], x->ring[2 * slot + 1]) != hipSuccess)
      return x->fail(EPIC_E_DEVICE, "event timing failed");
    main_ms[i] = ms;
  }
  return EPIC_OK;
}

epic_status epic_last_autos_timing(epic_ctx* x, float* sum_kernel_ms, float* removal_ms) {
  if (!x) return EPIC_E_INVALID;
  if (!x->timing || !x->timed || !x->autos_timed)
    return x->fail(EPIC_E_STATE, "no timed call with EPIC_FLAG_REMOVE_AUTOS and EPIC_FLAG_TIMING");
  DeviceGuard guard(x->device);
  if (hipEventSynchronize(x->ev[2]) != hipSuccess) return x->fail(EPIC_E_DEVICE, "event wait failed");
  float m = 0.f, r = 0.f;
  (void)hipEventElapsedTime(&m, x->ev[3], x->ev[4]);
  (void)hipEventElapsedTime(&r, x->ev[3], x->ev[2]);
  if (sum_kernel_ms) *sum_kernel_ms = m;
  if (removal_ms) *removal_ms = r;
  return EPIC_OK;
}

epic_status epic_postprocess(epic_ctx* x, const double* image, double taper_floor, double* out) {
  if (!x) return EPIC_E_INVALID;
  if (!x->have_geom) return x->fail(EPIC_E_STATE, "epic_set_antennas has not succeeded");
  if (!image || !out) return x->fail(EPIC_E_INVALID, "NULL device pointer");
  if (std::isnan(taper_floor) || taper_floor > 1.0)
    return x->fail(EPIC_E_INVALID, "taper_floor must be <= 1 (negative: no correction)");
  DeviceGuard guard(x->device);
  const int N = x->cfg.grid_n;
  epic::PostArgs a;
  a.image = reinterpret_cast<const double2*>(image);
  a.taper = taper_floor >= 0.0 ? x->taper.as<double>() : nullptr;
  a.tmax = x->tmax.as<double>();
  a.out = out;
  a.floor = taper_floor;
  a.npix = N * N;
  a.n = (int64_t)x->cfg.n_chan * N * N;
  (void)hipGetLastError();
  const dim3 grid((unsigned)((a.n + 255) / 256));
  if (x->cfg.n_pol == 2) hipLaunchKernelGGL(epic::postprocess_kernel<2>, grid, dim3(256), 0, x->stream, a);
  else hipLaunchKernelGGL(epic::postprocess_kernel<1>, grid, dim3(256), 0, x->stream, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return x->fail(EPIC_E_LAUNCH, std::string("launch failed: ") + hipGetErrorString(e));
  return EPIC_OK;
}

epic_status epic_kernel_taper(epic_ctx* x, double* taper) {
  if (!x) return EPIC_E_INVALID;
  if (!x->have_geom) return x->fail(EPIC_E_STATE, "epic_set_antennas has not succeeded");
  if (!taper) return x->fail(EPIC_E_INVALID, "NULL device pointer");
  DeviceGuard guard(x->device);
  const size_t bytes = (size_t)x->cfg.n_chan * x->cfg.grid_n * x->cfg.grid_n * sizeof(double);
  if (hipMemcpyAsync(taper, x->taper.p, bytes, hipMemcpyDeviceToDevice, x->stream) != hipSuccess)
    return x->fail(EPIC_E_LAUNCH, "copy failed");
  return EPIC_OK;
}

const char* epic_last_kernel_name(const epic_ctx* x) { return x ? x->last_kernel : "none"; }

void epic_destroy(epic_ctx* x) {
  if (!x) return;
  {
    DeviceGuard guard(x->device);
    (void)hipStreamSynchronize(x->stream);
    for (auto& e : x->ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : x->ring)
      if (e) (void)hipEventDestroy(e);
    x->prog.reset(); x->twiddle.reset(); x->taps.reset(); x->prog_im.reset(); x->taps_im.reset();
    x->csr_im.reset(); x->taper.reset(); x->tmax.reset();
    x->csr_off.reset(); x->csr_ent.reset(); x->partial.reset(); x->gpartial.reset(); x->gtab.reset();
    x->st_e.reset(); x->st_grid.reset(); x->st_acc.reset();
    x->sp_beta.reset(); x->sp_betamax.reset(); x->sp_bmat.reset(); x->sp_scale.reset();
    x->sp_partial.reset();
    x->au_part.reset(); x->au_tab.reset(); x->au_sums.reset(); x->au_wi.reset(); x->au_w.reset(); x->au_hat.reset();
    x->au_gauto.reset();
  }
  delete x;
}

const char* epic_last_error(const epic_ctx* x) {
  return x ? x->err.c_str() : g_init_error.c_str();
}

}  // extern "C"

#include "batch.hpp"
#include "pipeline.hpp"
