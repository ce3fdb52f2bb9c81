// Fused imaging kernel: one workgroup walks a contiguous range of the
// flattened (channel, time) index space and, for every sample, runs the whole
// hot path with the data resident in LDS and registers:
//
//   1. unpack the P*A 4+4-bit samples of (t, c) and multiply by the gains
//      (paper Sec. 3.2), into LDS;
//   2. grid them with the illumination kernel (Sec. 2.1, Eq. (4)-(5)) by a
//      gather: every thread runs a precomputed list of (cell, sample, weight)
//      steps and owns whole cells, so no atomics are needed;
//   3. transform rows then columns with the +i sign (Sec. 2.1, Eq. (5));
//      the row transform works in place in each row's LDS storage, the column
//      transform keeps its results in registers;
//   4. form XX, YY and XY (YX = conj XY) for the pixels each thread owns and
//      add them to float32 block sums, flushed to float64 every KBLOCK samples
//      (Sec. 2.1, Sec. 3.2: products accumulated over time).
//
// Every channel's aperture is translated by whole cells so that its kernel
// taps start at row 0 and column 0 (a common whole-cell shift multiplies both
// polarisations' transforms by the same phase ramp, so every product is
// unchanged).  The kernel requires the taps to fit the N/2 x N/2 corner of the
// grid -- the condition for an unaliased image -- so only N/2 rows are
// transformed along rows and the first radix stage of every line transform
// has half of its inputs equal to zero.
//
// At a channel boundary (and at the end of its range) a workgroup adds its
// sums into its own float64 partial-image slot; a second kernel adds the slots
// of each channel in workgroup order.
#pragma once
#include "autos.hpp"
#include "dft.hpp"
#include "reduce.hpp"

namespace epic {

// Gridding step: {code, weight bits}.  code = LDS byte offset of the cell
// (pol 0, relative to the grid base) << 15 | byte offset of E'[e] (pol 0, a
// multiple of 8), with bit 0 set on the last entry of a cell.  Every step
// reads E' of both polarisations and adds w * E' to the running sums; the
// last entry of a cell stores the sums to the cell and restarts them.  Cells
// with no antenna read a zero slot of E'; padding steps add zero and store
// nothing.  With complex kernels (CPX) a parallel array holds each step's
// imaginary weight.  The host orders the steps so that the lanes of a
// quarter-wave mostly touch distinct LDS banks.
constexpr int STEP_CELL_SHIFT = 15;            // cell byte offset < 128 KB
constexpr uint32_t STEP_E_MASK = 0x7FF8u;      // E' byte offset < 32 KB, 8-byte aligned
constexpr uint32_t STEP_LAST_BIT = 1u;         // in the code word
constexpr int kMaxFixedSteps = 8;              // held in registers across the barrier;
constexpr int kStepChunk = 4;                  // up to 4 more loaded after it; longer
                                               // lists run in chunks of 4

// The second word of a thread's program header: bits 0-23 the line of the
// wide block's second row pass (HDR_LINE2_NONE: none), bits 24-31 the steps
// of the thread's wave (0: the block's step count L).  Every lane of a wave
// holds the same step count, so it is read once per wave.
constexpr uint32_t HDR_LINE2_NONE = 0xFFFFFFu;
__device__ __forceinline__ int header_line2(uint32_t h) {
  return (h & HDR_LINE2_NONE) == HDR_LINE2_NONE ? -1 : (int)(h & HDR_LINE2_NONE);
}
__device__ __forceinline__ int header_steps(uint32_t h, int L) {
  const int s = __builtin_amdgcn_readfirstlane((int)(h >> 24));
  return s ? s : L;
}

template <int N> struct FusedShape {
  static constexpr int S = Line<N>::S, R = Line<N>::R, D = Line<N>::D;
  // threads per workgroup: one lane group per line; at N = 128 a lane group
  // takes both polarisations of a row (and of a column), 512 threads
  static constexpr int NT = N == 128 ? 512 : N * R;
  static constexpr int CPW = 64 / R;           // columns (or rows) per wave
  // LDS geometry in float2 units.  LDS serves 64-bit reads 32 lanes at a time
  // from 64 four-byte banks (conflict-free when a half-wave's addresses differ
  // modulo 32) and 64-bit writes 16 lanes at a time from 32 banks (a
  // quarter-wave's addresses differing modulo 16).  With the lane roles below,
  // the row stride RS, the polarisation stride PSTRIDE, the physical order of
  // the aperture rows (phys_row), the exchange skews and the rule the host
  // follows when it deals rows to waves, every access of the N = 64 row and
  // column transforms is conflict-free under that model.
  static constexpr int RS = N == 32 ? N + 1 : N + 4;
  // rows of the LDS grid per polarisation: N (the column transforms exchange
  // through all N rows of their column) or, at N = 128, N/2 (the aperture
  // rows; columns exchange through their upper half instead)
  static constexpr int XROWS = N == 128 ? N / 2 : N;
  static constexpr int PSTRIDE = XROWS * RS + (N == 32 ? 8 : 16);
  static constexpr int COL_SKEW = N == 64 ? 2 : 1;   // exchange skew of the forward column pass
  // physical row of aperture row j < N/2: at N = 64 rows are interleaved so
  // that the 8 rows a column lane loads fall on distinct banks
  static __host__ __device__ constexpr int phys_row(int j) {
    return N == 64 ? 8 * (j >> 3) + 2 * (j & 3) + ((j >> 2) & 1) : j;
  }
  static constexpr int H = N / 2;              // aperture block side
  // aperture block side of the wide variant (N = 64): rows and columns
  // R n1 + n0 < HW are the inputs n1 < HW / R of a line
  static constexpr int HW = 3 * N / 4;
  static constexpr int KBLOCK = 128;           // samples summed in float32 before a float64 flush
  // waves per SIMD the register budget is sized for: two resident workgroups
  // per CU (4 waves/SIMD, <= 128 VGPRs) at N = 64
  static constexpr int MIN_WAVES_PER_EU = 4;
};

// E' stride between polarisations: the largest A a variant takes (NT*GPT/P)
// plus 64 float2 (the 16 zero slots, and a multiple of 64 so that both
// polarisations load with one paired LDS read whose second offset is an
// immediate).
template <int NT, int GPT, int P> struct EStride {
  static constexpr int value = (NT * GPT) / P + 64;
};

// One imaging configuration of a launch: its inputs, its gridding programs
// and the place of its channels in the launch's channel order.  A launch of
// the batch walks the channels of up to kMaxLaunchBlocks blocks (the same
// grid, polarisations and sample bytes per thread; different antenna counts
// and channel counts) as one flattened (channel, time) space; a launch of a
// single context has one block.
constexpr int kMaxLaunchBlocks = 8;
struct FusedBlock {
  const uint8_t* efield;    // [T][C_b][P][A_b]
  const float2* gains;      // [C_b][P][A_b]
  const uint2* prog;        // [C_b][1 + L_b][NT]: row-pass line of each thread, then L_b steps
  const float* wim;         // [C_b][1 + L_b][NT] imaginary step weights (complex kernels), or null
  int c0;                   // first channel of the block in the launch's channel order
  int n_chan, n_ant, L;
  int wrows;                // wide block: its row count (the column pass reads rows below it)
};

// Work partition of a persistent launch.  The launch's units form one flat
// list of S segments of T units each, segment-major (N <= 64: a segment is a
// channel and a unit a sample; N = 128: a segment is a (channel, parity)
// pair).  The W workgroups form W / team teams of `team` workgroups; team tm
// takes the contiguous range [tm U / n_team, (tm + 1) U / n_team) of the list
// (U = S T), and member k of the team takes the k-th of `team` equal parts of
// each segment piece in that range.  The members of a team thus work on the
// same segment at the same time, and with xcd = 1 (a team's workgroups on one
// XCD, see wg_range_index) one XCD holds the gridding programs of few
// channels in its L2 at any time; the total work per workgroup stays balanced
// to a unit per piece.  A member's part of a piece is one accumulation
// segment with its own partial slot, (s + tm) team + k (at most
// (S + n_team - 1) team slots); a part of at most kblock units is written
// once as float32, a longer one is summed in float64 (first flush writes,
// later ones add).
struct FusedArgs {
  FusedBlock blk[kMaxLaunchBlocks];   // in channel order: blk[i + 1].c0 = blk[i].c0 + blk[i].n_chan
  int n_blk;
  const float2* twiddle;    // [N] exp(+2 pi i k / N)
  double* partial;          // [(S + W / team - 1) team][NACC][NV][NT] (thread-major), NV sums per thread
  int64_t n_time;           // T
  int64_t total;            // U = S * T
  int W;                    // workgroups, a multiple of team
  int team;                 // workgroups per team, 1 .. 8
  int kblock;               // samples summed in float32 before a float64 flush, 1 .. KBLOCK
  int xcd;                  // 1: consecutive workgroup indices dealt XCD by XCD (see wg_range_index)
};

// Workgroup ids are dealt to the 8 XCDs round-robin.  With xcd = 1 the
// logical index of workgroup id is chosen so that consecutive indices (the
// members of a team, which share a channel and its gridding program) run on
// one XCD and its L2.
__device__ __forceinline__ int wg_range_index(int id, int n, int xcd) {
  if (!xcd) return id;
  const int q = n >> 3, r = n & 7, j = id & 7;
  return j * q + (j < r ? j : r) + (id >> 3);
}

// Part of member k (of m, a power of two) of the piece of segment sg inside
// team range [ra, rb): first unit a (flat index) and length len (0: none).
__host__ __device__ __forceinline__ void member_part(int64_t sg, int64_t T, int64_t ra, int64_t rb, int m,
                                                     int k, int64_t& a, int64_t& len) {
  const int64_t pa = sg * T > ra ? sg * T : ra;
  const int64_t pb = (sg + 1) * T < rb ? (sg + 1) * T : rb;
  const int64_t L = pb > pa ? pb - pa : 0;
  const int lg = __builtin_ctz((unsigned)m);
  a = pa + ((k * L) >> lg);
  len = pa + (((k + 1) * L) >> lg) - a;
}

// Walks the units of one member: segment s, time t, units left in the
// current part (including the current one).
struct UnitWalk {
  int64_t T, ra, rb;
  int m, k;
  int64_t s, t, left;
  // move to the first unit of the first non-empty part at or after segment sg
  __device__ __forceinline__ bool seek(int64_t sg) {
    for (; sg * T < rb; ++sg) {
      int64_t a, len;
      member_part(sg, T, ra, rb, m, k, a, len);
      if (len > 0) {
        s = sg;
        t = a - sg * T;
        left = len;
        return true;
      }
    }
    return false;
  }
  __device__ __forceinline__ void next() {
    if (--left > 0) ++t;
    else seek(s + 1);
  }
};

// Units of member k of team range [ra, rb).
__device__ __forceinline__ int64_t member_units(int64_t T, int64_t ra, int64_t rb, int m, int k) {
  int64_t n = 0;
  for (int64_t sg = ra / T; sg * T < rb; ++sg) {
    int64_t a, len;
    member_part(sg, T, ra, rb, m, k, a, len);
    n += len;
  }
  return n;
}

// Block of channel c: the last block whose first channel is <= c.
__device__ __forceinline__ int block_of(const FusedArgs& a, int c) {
  int b = 0;
  for (int i = 1; i < a.n_blk; ++i)
    if (a.blk[i].c0 <= c) b = i;
  return b;
}

// Flat range of workgroup w: [w*total/W, (w+1)*total/W).
__device__ __forceinline__ int64_t range_begin(int64_t w, int64_t total, int64_t W) {
  return (w * total) / W;
}

// Lane roles shared by the row and column passes (so both use the same
// twiddles): n0 is the lane's index inside its line, sub the line of the
// wave.  R = 8: each group of 16 lanes holds 4 n0 x 4 lines (lane = 16 G +
// 4 a + b, n0 = 4 (G >> 1) + a, sub = 4 (G & 1) + b), which makes the row and
// the column accesses the same 4 x 4 shape.  R = 4: lane = n0 * CPW + sub.
template <int N> struct Roles {
  int tid, wave, n0, sub, kl;
  __host__ __device__ __forceinline__ explicit Roles(int t) {
    constexpr int R = FusedShape<N>::R, CPW = FusedShape<N>::CPW;
    tid = t;
    wave = t >> 6;
    const int lane = t & 63;
    if (R == 8) {
      const int G = lane >> 4, a = (lane >> 2) & 3, b = lane & 3;
      n0 = 4 * (G >> 1) + a;
      sub = 4 * (G & 1) + b;
    } else {
      n0 = lane / CPW;
      sub = lane % CPW;
    }
    kl = wave * CPW + sub;
  }
};

__device__ __forceinline__ float2 unpack_ci4(uint32_t b) {
  const int v = (int)b;
  return make_float2((float)((v >> 4) - ((v & 0x80) ? 16 : 0)),
                     (float)((v & 0xF) - ((v & 0x8) ? 16 : 0)));
}

// Slots of E' for this thread's items k = tid + i*NT (k = p*A + a), and the
// 16 zero slots (a = A .. A+15, one per LDS bank pair of a quarter-wave) of
// each polarisation.
template <int NT, int GPT, int ES>
__device__ __forceinline__ void init_stage(float2* E, int (&eidx)[GPT], int tid, int n_ant, int P) {
#pragma unroll
  for (int i = 0; i < GPT; ++i) {
    const int k = tid + i * NT;
    const int p = k >= n_ant ? 1 : 0;
    eidx[i] = k + p * (ES - n_ant);
  }
  if (tid < 16 * P) E[(tid >> 4) * ES + n_ant + (tid & 15)] = make_float2(0.f, 0.f);
}

// 1. E'[p][a] = g * e.  RECOMPUTE (where registers are short): the slots are
// recomputed with every sample from an opaque copy of tid, so that they are
// not held (or spilled) across the sample loop.
template <int NT, int GPT, int ES, int P, bool RECOMPUTE>
__device__ __forceinline__ void stage_samples(float2* E, const uint32_t (&cur)[GPT],
                                              const float2 (&g)[GPT], const int (&eidx)[GPT],
                                              int tid, int PA) {
  int t = tid;
  if constexpr (RECOMPUTE) asm volatile("" : "+v"(t));
#pragma unroll
  for (int i = 0; i < GPT; ++i) {
    const int k = t + i * NT;
    const int slot = RECOMPUTE ? k + (k >= PA / P ? ES - PA / P : 0) : eidx[i];
    if (k < PA) E[slot] = cmul(g[i], unpack_ci4(cur[i]));
  }
}

// One gridding step on the running sums (s0, s1) of the current cell.
// xlds is the start of the grid in the shared buffer (the step's cell offset
// is relative to it).  CPX: the weight is w + i wi.
template <int N, int P, int RS, int ES, bool CPX>
__device__ __forceinline__ void grid_step(char* xlds, uint2 step, float wi, float2 e0,
                                          float2 e1, float2& s0, float2& s1) {
  const float w = __uint_as_float(step.y);
  s0.x = fmaf(w, e0.x, s0.x);
  s0.y = fmaf(w, e0.y, s0.y);
  if (CPX) {
    s0.x = fmaf(-wi, e0.y, s0.x);
    s0.y = fmaf(wi, e0.x, s0.y);
  }
  if (P == 2) {
    s1.x = fmaf(w, e1.x, s1.x);
    s1.y = fmaf(w, e1.y, s1.y);
    if (CPX) {
      s1.x = fmaf(-wi, e1.y, s1.x);
      s1.y = fmaf(wi, e1.x, s1.y);
    }
  }
  if (step.x & STEP_LAST_BIT) {                 // last entry of the cell
    float2* cell = reinterpret_cast<float2*>(xlds + (step.x >> STEP_CELL_SHIFT));
    cell[0] = s0;
    if (P == 2) cell[FusedShape<N>::PSTRIDE] = s1;
    s0 = make_float2(0.f, 0.f);
    s1 = make_float2(0.f, 0.f);
  }
}

// elds: the start of E' in the shared buffer (the step's E' offset is
// relative to it).
template <int P, int ES>
__device__ __forceinline__ void read_e(const char* elds, uint2 step, float2& e0, float2& e1) {
  const float2* e = reinterpret_cast<const float2*>(elds + (step.x & STEP_E_MASK));
  e0 = e[0];
  if (P == 2) e1 = e[ES];
}

// 2. Gather gridding with exactly LS steps, steps[OFF .. OFF + LS), already
// loaded into registers (wis: the imaginary weights, read only when CPX);
// s0, s1 carry the sums of a cell whose entries continue in the next call.
template <int N, int P, int RS, int ES, int LS, bool CPX, int OFF = 0, int SZ>
__device__ __forceinline__ void grid_fixed(const char* elds, char* xlds, const uint2 (&steps)[SZ],
                                           const float (&wis)[SZ], float2& s0, float2& s1) {
  static_assert(OFF + LS <= SZ, "more steps than loaded");
#pragma unroll
  for (int st0 = OFF; st0 < OFF + LS; st0 += kStepChunk) {   // E' reads in groups of 4
    constexpr int G = kStepChunk;
    float2 e0[G], e1[G];
#pragma unroll
    for (int st = 0; st < G; ++st)
      if (st0 + st < OFF + LS) read_e<P, ES>(elds, steps[st0 + st], e0[st], e1[st]);
#pragma unroll
    for (int st = 0; st < G; ++st)
      if (st0 + st < OFF + LS)
        grid_step<N, P, RS, ES, CPX>(xlds, steps[st0 + st], wis[st0 + st], e0[st], e1[st], s0, s1);
  }
}

// 2'. Gather gridding of a long list (L a multiple of kStepChunk).  The
// steps come from global memory (L2) a chunk at a time; the next chunk is
// loaded while the current one is gridded, so its latency is hidden.
template <int N, int P, int RS, int ES, bool CPX>
__device__ __forceinline__ void grid_chunked(const char* elds, char* xlds, const uint2* prog, const float* wim,
                                             int stride, int L) {
  float2 s0 = make_float2(0.f, 0.f), s1 = make_float2(0.f, 0.f);
  uint2 nsteps[kStepChunk];
  float nwis[kStepChunk];
#pragma unroll
  for (int st = 0; st < kStepChunk; ++st) {
    nsteps[st] = prog[st * stride];
    nwis[st] = CPX ? wim[st * stride] : 0.f;
  }
  for (int st0 = 0; st0 < L; st0 += kStepChunk) {
    uint2 steps[kStepChunk];
    float wis[kStepChunk];
    float2 e0[kStepChunk], e1[kStepChunk];
#pragma unroll
    for (int st = 0; st < kStepChunk; ++st) {
      steps[st] = nsteps[st];
      wis[st] = nwis[st];
    }
    if (st0 + kStepChunk < L) {
#pragma unroll
      for (int st = 0; st < kStepChunk; ++st) {
        nsteps[st] = prog[(st0 + kStepChunk + st) * stride];
        nwis[st] = CPX ? wim[(st0 + kStepChunk + st) * stride] : 0.f;
      }
    }
#pragma unroll
    for (int st = 0; st < kStepChunk; ++st) read_e<P, ES>(elds, steps[st], e0[st], e1[st]);
#pragma unroll
    for (int st = 0; st < kStepChunk; ++st)
      grid_step<N, P, RS, ES, CPX>(xlds, steps[st], wis[st], e0[st], e1[st], s0, s1);
  }
}

// 2. (fixed path) Gridding of L <= kMaxFixedSteps + kStepChunk steps whose
// first kMaxFixedSteps are loaded (steps, wis); steps past them are loaded
// from prog (wim) once the first G are gridded.
template <int N, int P, int NT, int RS, int ES, bool CPX>
__device__ __forceinline__ void grid_loaded(const char* elds, char* xlds,
                                            const uint2 (&steps)[kMaxFixedSteps],
                                            const float (&wis)[kMaxFixedSteps], const uint2* prog,
                                            const float* wim, int L, int tid) {
  constexpr int F = kMaxFixedSteps, G = kStepChunk;
  float2 s0 = make_float2(0.f, 0.f), s1 = make_float2(0.f, 0.f);
  if (L > F) {
    static_assert(F == 2 * G, "the first G steps are gridded before the rest load");
    grid_fixed<N, P, RS, ES, G, CPX>(elds, xlds, steps, wis, s0, s1);
    uint2 more[G];
    float wmore[G];
#pragma unroll
    for (int st = 0; st < G; ++st) {
      if (F + st < L) more[st] = prog[(F + st) * NT + tid];
      wmore[st] = (CPX && F + st < L) ? wim[(F + st) * NT + tid] : 0.f;
    }
    grid_fixed<N, P, RS, ES, G, CPX, G>(elds, xlds, steps, wis, s0, s1);
    switch (L - F) {
      case 1: grid_fixed<N, P, RS, ES, 1, CPX>(elds, xlds, more, wmore, s0, s1); break;
      case 2: grid_fixed<N, P, RS, ES, 2, CPX>(elds, xlds, more, wmore, s0, s1); break;
      case 3: grid_fixed<N, P, RS, ES, 3, CPX>(elds, xlds, more, wmore, s0, s1); break;
      default: grid_fixed<N, P, RS, ES, 4, CPX>(elds, xlds, more, wmore, s0, s1); break;
    }
  } else {
    switch (L) {
      case 1: grid_fixed<N, P, RS, ES, 1, CPX>(elds, xlds, steps, wis, s0, s1); break;
      case 2: grid_fixed<N, P, RS, ES, 2, CPX>(elds, xlds, steps, wis, s0, s1); break;
      case 3: grid_fixed<N, P, RS, ES, 3, CPX>(elds, xlds, steps, wis, s0, s1); break;
      case 4: grid_fixed<N, P, RS, ES, 4, CPX>(elds, xlds, steps, wis, s0, s1); break;
      case 5: grid_fixed<N, P, RS, ES, 5, CPX>(elds, xlds, steps, wis, s0, s1); break;
      case 6: grid_fixed<N, P, RS, ES, 6, CPX>(elds, xlds, steps, wis, s0, s1); break;
      case 7: grid_fixed<N, P, RS, ES, 7, CPX>(elds, xlds, steps, wis, s0, s1); break;
      default: grid_fixed<N, P, RS, ES, 8, CPX>(elds, xlds, steps, wis, s0, s1); break;
    }
  }
}

// Steps 1-2 of one sample: load the gridding program (exactly L steps for
// L <= kMaxFixedSteps + kStepChunk), stage E', barrier, grid.  A thread grids
// only cells of rows its own wave transforms next, so gridding ends with a
// wave-level fence.  E (= elds) is E' and xlds the grid in the shared buffer;
// prog is the channel's step list (wim: its imaginary weights when CPX), of
// at least L steps; L is the wave's own step count, uniform over the wave.
// Steps past kMaxFixedSteps are loaded after the barrier, once the first G
// are gridded (their registers free), while the next G are.
template <int N, int P, int NT, int RS, int ES, int GPT, bool CPX, bool RECOMPUTE = false,
          bool AHEAD = false>
__device__ __forceinline__ void stage_and_grid(const char* elds, char* xlds, float2* E,
                                               const uint2* prog, const float* wim, int L,
                                               const uint32_t (&cur)[GPT], const float2 (&g)[GPT],
                                               const int (&eidx)[GPT], int tid, int PA,
                                               bool stage = true) {
  constexpr int F = kMaxFixedSteps, G = kStepChunk;
  // AHEAD: the sample gridded here is already staged and visible (elds); E
  // is the other buffer, into which the next sample is staged (if stage)
  // while the steps load, with no barrier.
  auto stage_e = [&]() {
    if (AHEAD) {
      if (stage) stage_samples<NT, GPT, ES, P, RECOMPUTE>(E, cur, g, eidx, tid, PA);
    } else {
      stage_samples<NT, GPT, ES, P, RECOMPUTE>(E, cur, g, eidx, tid, PA);
      __syncthreads();
    }
  };
  if (L <= F + G) {
    uint2 steps[F];
    float wis[F];
#pragma unroll
    for (int st = 0; st < F; ++st) {
      if (st < L) steps[st] = prog[st * NT + tid];
      wis[st] = (CPX && st < L) ? wim[st * NT + tid] : 0.f;
    }
    stage_e();
    grid_loaded<N, P, NT, RS, ES, CPX>(elds, xlds, steps, wis, prog, wim, L, tid);
  } else {
    stage_e();
    grid_chunked<N, P, RS, ES, CPX>(elds, xlds, prog + tid, CPX ? wim + tid : nullptr, NT, L);
  }
  wave_lds_sync();
}

// 3a. Row transforms of the H = N/2 aperture rows of each polarisation, in
// place.  line = p << 16 | j is the row this thread's R lanes transform (from
// the channel's program; < 0: none); each wave transforms the rows it has
// just gridded, so only a wave-level fence separates the two.  SG > 0:
// forward, the row holds cells at columns < H.  SG < 0: adjoint, the row
// holds the forward output layout and the columns < H of the result are
// written back.
// WIDE: forward, the row holds cells at columns < HW (the inputs n1 >= HW / R
// are zero); adjoint, the columns < HW of the result are written back.
template <int N, int P, int SG, bool WIDE = false>
__device__ __forceinline__ void row_pass(float2* X, const Roles<N>& r, const float2* tw, int line) {
  constexpr int S = Line<N>::S, R = Line<N>::R, D = Line<N>::D;
  constexpr int RS = FusedShape<N>::RS, PS = FusedShape<N>::PSTRIDE;
  static_assert(!WIDE || FusedShape<N>::HW % R == 0, "wide rows: whole inputs");
  if (line >= 0) {
    float2* row = X + (line >> 16) * PS + (line & 0xFFFF) * RS;
    float2 v[1][S];
    if constexpr (SG > 0 && WIDE) {
      constexpr int NIN = FusedShape<N>::HW / R;
#pragma unroll
      for (int n1 = 0; n1 < S; ++n1) v[0][n1] = n1 < NIN ? row[R * n1 + r.n0] : make_float2(0.f, 0.f);
      line_transform<N, +1, 1, NIN>(v, tw, r.n0, row, [](int, int s) { return s; });
#pragma unroll
      for (int q = 0; q < D; ++q)
#pragma unroll
        for (int k1 = 0; k1 < R; ++k1) row[r.n0 * D + q + S * k1] = v[0][q * R + k1];
    } else if (SG > 0) {
#pragma unroll
      for (int n1 = 0; n1 < S / 2; ++n1) v[0][n1] = row[R * n1 + r.n0];
      line_transform<N, +1, 1, S / 2>(v, tw, r.n0, row, [](int, int s) { return s; });
#pragma unroll
      for (int q = 0; q < D; ++q)
#pragma unroll
        for (int k1 = 0; k1 < R; ++k1) row[r.n0 * D + q + S * k1] = v[0][q * R + k1];
    } else {
#pragma unroll
      for (int q = 0; q < D; ++q)
#pragma unroll
        for (int k1 = 0; k1 < R; ++k1) v[0][q * R + k1] = row[r.n0 * D + q + S * k1];
      line_transform_rev<N, -1, 1>(v, tw, r.n0, row, [](int, int s) { return s; });
      constexpr int NOUT = WIDE ? FusedShape<N>::HW / R : S / 2;
#pragma unroll
      for (int n1 = 0; n1 < NOUT; ++n1) row[R * n1 + r.n0] = v[0][n1];
    }
  }
}

// 3b. Forward column transforms of column r.kl for all polarisations; only
// rows < H (WIDE: < rows, the wide block's row count, a multiple of R from
// H to HW, uniform) are nonzero (stored at their physical rows, which for
// whole groups of R rows are the same rows); the other rows of the grid are
// not read.  Out: v[p][q R + k1] = F_p[n0 D + q + S k1][kl].
// XSHARE: every polarisation exchanges through the first one's column (a
// column belongs to the lanes of one wave, which finish each polarisation's
// transform before the next one writes), leaving the rows >= H of the
// others untouched.
// WR > 0 (WIDE): the block's row count is WR, fixed at compile time: only
// the WR / R inputs that can be nonzero are read and transformed.
template <int N, int P, bool WIDE = false, bool XSHARE = false, int WR = 0>
__device__ __forceinline__ void column_pass_fwd(float2 (&v)[P][Line<N>::S], float2* X,
                                                const Roles<N>& r, const float2* tw, int rows = 0) {
  using SH = FusedShape<N>;
  constexpr int S = Line<N>::S, R = Line<N>::R, RS = SH::RS, PS = SH::PSTRIDE;
  static_assert(WR == 0 || (WIDE && WR % R == 0 && WR >= SH::H && WR <= SH::HW), "wide block rows");
  constexpr int NIN = WR > 0 ? WR / R : WIDE ? SH::HW / R : S / 2;
  if constexpr (WR > 0) rows = WR;
  const int kl = r.kl;
#pragma unroll
  for (int p = 0; p < P; ++p) {                 // one polarisation at a time
    float2 (&vp)[1][S] = *reinterpret_cast<float2 (*)[1][S]>(&v[p]);
#pragma unroll
    for (int n1 = 0; n1 < S; ++n1)
      if (n1 < S / 2 || (n1 < NIN && R * n1 < rows))
        vp[0][n1] = X[p * PS + SH::phys_row(R * n1 + r.n0) * RS + kl];
      else if (WIDE) vp[0][n1] = make_float2(0.f, 0.f);
    line_transform<N, +1, 1, NIN, SH::COL_SKEW>(vp, tw, r.n0, XSHARE ? X : X + p * PS,
                                    [kl](int, int s) { return s * RS + kl; });
  }
}

// The whole per-workgroup loop, two workgroup barriers per sample (the
// N = 64 dual-polarisation form with at most 256 antennas and Gaussian taps
// runs fused_image_body_pipe instead).  WIDE (N = 64): the wide block of up to HW
// columns and wrows (32, 40 or 48) rows; the programs' header gives each
// thread a second row-pass line (header_line2, -1: none; whole waves have
// none, so they skip the pass); the row passes take their lines' inputs
// n1 < HW / R, the column pass those of rows below wrows.
// MULTI: the launch walks several blocks (FusedArgs::blk); a workgroup whose
// range crosses into the next block switches inputs, gains, programs and the
// E' layout of its antenna count at that channel boundary.  Without MULTI
// the launch has one block.
template <int N, int P, int GPT, bool CPX, bool WIDE, bool MULTI, int WR = 0>
__device__ __forceinline__ void fused_image_body(const FusedArgs& a) {
  using SH = FusedShape<N>;
  constexpr int S = SH::S, NT = SH::NT, RS = SH::RS;
  constexpr int NACC = (P == 2) ? 4 : 1;
  constexpr int ES = EStride<NT, GPT, P>::value;
  // E'[p][a] (zero slots at a = A .. A+15), then the grid.  EINGRID: E' of
  // more than 512 antennas does not fit beside the grid if two workgroups
  // are to share a CU.  It takes the second polarisation's grid rows
  // N/2 .. N-1 instead (from a multiple of 64 float2, so that the paired
  // E' read keeps its offsets; 48 float2 past the grid's end): the column
  // transforms of that polarisation exchange through the first one's
  // column (which the same wave has just finished with), so nothing else
  // touches those rows and staging needs no extra barrier.
  constexpr bool EINGRID = N == 64 && P == 2 && GPT == 4 && !WIDE;
  constexpr int GRID = (P - 1) * SH::PSTRIDE + N * RS;           // float2
  constexpr int EOFF = (SH::PSTRIDE + (N / 2) * RS + 63) / 64 * 64;
  constexpr int LDS = EINGRID ? (EOFF + P * ES > GRID ? EOFF + P * ES : GRID) : P * ES + GRID;
  __shared__ __attribute__((aligned(16))) float2 lds2[LDS];
  float2* X = lds2 + (EINGRID ? 0 : P * ES);
  float2* E = EINGRID ? lds2 + EOFF : lds2;

  const Roles<N> r(threadIdx.x);
  const int tid = r.tid;
  const int wl = wg_range_index((int)blockIdx.x, (int)gridDim.x, a.xcd);
  const int m = a.team, tm = wl / m, mk = wl - tm * m, n_team = a.W / m;
  UnitWalk it;
  it.T = a.n_time;
  it.ra = range_begin(tm, a.total, n_team);
  it.rb = range_begin(tm + 1, a.total, n_team);
  it.m = m;
  it.k = mk;
  if (tm >= n_team || !it.seek(it.ra / a.n_time)) return;
  const int64_t n_units = member_units(a.n_time, it.ra, it.rb, m, mk);

  float2 tw[S];
#pragma unroll
  for (int k0 = 0; k0 < S; ++k0) tw[k0] = a.twiddle[(r.n0 * k0) % N];

  // block of the sample being prefetched (nb) and of the one being imaged (b)
  int nb = MULTI ? block_of(a, (int)it.s) : 0;
  int b = nb;
  int PA = P * a.blk[b].n_ant;                 // of block b
  int L = a.blk[b].L, Lw = L;                  // L: of block b; Lw: of this wave
  const int KB = a.kblock;
  // the prefetched sample's block: bytes per time sample, first channel
  int64_t n_row = (int64_t)a.blk[nb].n_chan * P * a.blk[nb].n_ant;
  int n_pa = P * a.blk[nb].n_ant, n_c0 = a.blk[nb].c0;
  const uint8_t* n_src = a.blk[nb].efield;
  int eidx[GPT];
  init_stage<NT, GPT, ES>(E, eidx, tid, a.blk[b].n_ant, P);
  int wrows = a.blk[b].wrows;                  // wide block rows of block b

  float acc[S][NACC];                          // float32 sums over <= KB samples
  float2 g[GPT];
  uint32_t nxt[GPT];
  int c = -1, nblk = 0, nflush = 0, line = -1, line2 = -1;
  int64_t part_len = 0, slot = 0;
  const uint2* prog = nullptr;
  const float* wim = nullptr;

  auto load_bytes = [&](int ch, int64_t t, uint32_t (&dst)[GPT]) {
    const uint8_t* src = n_src + t * n_row + (int64_t)(ch - n_c0) * n_pa;
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int k = tid + i * NT;
      dst[i] = (k < n_pa) ? (uint32_t)src[k] : 0u;
    }
  };
  // the float32 sums of the current part into its slot: written once as
  // float32 if the part fits one block, else added in float64
  auto flush = [&]() {
    double* out = a.partial + slot * (NACC * S * NT) + tid;
    if (part_len <= KB) {
      float* o32 = reinterpret_cast<float*>(a.partial + slot * (NACC * S * NT)) + tid;
#pragma unroll
      for (int u = 0; u < NACC; ++u)
#pragma unroll
        for (int i = 0; i < S; ++i) {
          o32[(u * S + i) * NT] = acc[i][u];
          acc[i][u] = 0.f;
        }
    } else {
#pragma unroll
      for (int u = 0; u < NACC; ++u)
#pragma unroll
        for (int i = 0; i < S; ++i) {
          double* o = out + (u * S + i) * NT;
          *o = (nflush ? *o : 0.0) + (double)acc[i][u];
          acc[i][u] = 0.f;
        }
    }
    ++nflush;
    nblk = 0;
  };

  load_bytes((int)it.s, it.t, nxt);
  for (int64_t left = n_units; left > 0; --left) {
    const int cc = (int)it.s;                  // channel of the current sample
    if (cc != c) {                             // a part (accumulation segment) starts
      if (c >= 0) flush();
      c = cc;
      nflush = 0;
      part_len = it.left;
      slot = ((int64_t)c + tm) * m + mk;
      if (MULTI && nb != b) {                  // and a block: its antennas' E' layout
        b = nb;
        PA = P * a.blk[b].n_ant;
        L = a.blk[b].L;
        init_stage<NT, GPT, ES>(E, eidx, tid, a.blk[b].n_ant, P);
        wrows = a.blk[b].wrows;
      }
      const int64_t cl = c - a.blk[b].c0;      // channel within the block
      prog = a.blk[b].prog + cl * (L + 1) * NT;
      if (CPX) wim = a.blk[b].wim + cl * (L + 1) * NT + NT;
      line = (int)prog[tid].x;
      if (WIDE) line2 = header_line2(prog[tid].y);
      Lw = header_steps(prog[tid].y, L);
      prog += NT;
#pragma unroll
      for (int i = 0; i < S; ++i)
#pragma unroll
        for (int u = 0; u < NACC; ++u) acc[i][u] = 0.f;
#pragma unroll
      for (int i = 0; i < GPT; ++i) {
        const int k = tid + i * NT;
        g[i] = (k < PA) ? a.blk[b].gains[cl * PA + k] : make_float2(0.f, 0.f);
      }
    } else if (nblk == KB) {
      flush();
    }
    uint32_t cur[GPT];
#pragma unroll
    for (int i = 0; i < GPT; ++i) cur[i] = nxt[i];
    it.next();                                 // advance, prefetch the next sample
    if (left > 1) {
      if (MULTI && it.s != cc) {               // the next part may be in another block
        const int nnb = block_of(a, (int)it.s);
        if (nnb != nb) {
          nb = nnb;
          n_row = (int64_t)a.blk[nb].n_chan * P * a.blk[nb].n_ant;
          n_pa = P * a.blk[nb].n_ant;
          n_c0 = a.blk[nb].c0;
          n_src = a.blk[nb].efield;
        }
      }
      load_bytes((int)it.s, it.t, nxt);
    }

    stage_and_grid<N, P, NT, RS, ES, GPT, CPX, EINGRID>(reinterpret_cast<const char*>(E),
                                                        reinterpret_cast<char*>(X), E, prog, wim, Lw,
                                                        cur, g, eidx, tid, PA);
    row_pass<N, P, +1, WIDE>(X, r, tw, line);
    if (WIDE) row_pass<N, P, +1, WIDE>(X, r, tw, line2);
    __syncthreads();
    float2 v[P][S];
    column_pass_fwd<N, P, WIDE, EINGRID, WR>(v, X, r, tw, wrows);

    // 4. polarisation products: XX, YY, Re XY, Im XY (XY = F_X conj(F_Y))
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const float2 fx = v[0][i];
      acc[i][0] = fmaf(fx.y, fx.y, fmaf(fx.x, fx.x, acc[i][0]));
      if (P == 2) {
        const float2 fy = v[P - 1][i];
        acc[i][1 % NACC] = fmaf(fy.y, fy.y, fmaf(fy.x, fy.x, acc[i][1 % NACC]));
        acc[i][2 % NACC] = fmaf(fx.y, fy.y, fmaf(fx.x, fy.x, acc[i][2 % NACC]));
        acc[i][3 % NACC] = fmaf(-fx.x, fy.y, fmaf(fx.y, fy.x, acc[i][3 % NACC]));
      }
    }
    ++nblk;
  }
  flush();
}

template <int V> struct IntC { static constexpr int value = V; };

// 3b'. Forward column transforms of column r.kl of both polarisations from
// the aperture buffer Xb (rows < H of each polarisation at stride PSTRIDE),
// exchanging through the 2H slots that this column's rows < H of the two
// polarisations form (slot j < H: first polarisation, row j; j >= H:
// second, row j - H).  Both polarisations' inputs are read before the first
// exchange; nothing outside the buffer is touched.  A column belongs to the
// lanes of one wave, so the second polarisation's exchange follows the
// first's behind the transform's own wave-level fences.
template <int N>
__device__ __forceinline__ void column_pass_buf(float2 (&v)[2][Line<N>::S], float2* Xb,
                                                const Roles<N>& r, const float2* tw) {
  using SH = FusedShape<N>;
  constexpr int S = Line<N>::S, R = Line<N>::R, RS = SH::RS, PS = SH::PSTRIDE, H = N / 2;
  const int kl = r.kl;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int n1 = 0; n1 < S / 2; ++n1) v[p][n1] = Xb[p * PS + SH::phys_row(R * n1 + r.n0) * RS + kl];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    float2 (&vp)[1][S] = *reinterpret_cast<float2 (*)[1][S]>(&v[p]);
    line_transform<N, +1, 1, S / 2, SH::COL_SKEW>(vp, tw, r.n0, Xb, [kl](int, int j) {
      return j * RS + kl + (j / H) * (PS - H * RS);
    });
  }
}

// The per-workgroup loop with one workgroup barrier per sample (N = 64, two
// polarisations, at most 256 antennas, Gaussian taps, one block).  E' and
// the aperture rows are double-buffered: sample s grids from E' buffer s & 1
// into aperture buffer s & 1 (grid rows 32 (s & 1) .. 32 (s & 1) + 31 of each
// polarisation) and transforms its rows; sample s + 1 is staged into the
// other E' buffer while sample s's gridding program loads.  After the
// barrier the column transforms of sample s run inside buffer s & 1 while
// faster waves grid sample s + 1 into the other.  A buffer is written again
// two samples after it was last read, behind the next barrier, by which
// every wave has finished with it.  The loop is unrolled by two so that the
// buffers' offsets are immediates.
template <int N, int P, int GPT>
__device__ __forceinline__ void fused_image_body_pipe(const FusedArgs& a) {
  static_assert(N == 64 && P == 2 && GPT == 1, "the double-buffered form: N = 64, P = 2, GPT = 1");
  constexpr bool CPX = false;
  using SH = FusedShape<N>;
  constexpr int S = SH::S, NT = SH::NT, RS = SH::RS, NACC = 4;
  constexpr int ES = EStride<NT, GPT, P>::value;
  constexpr int EB = P * ES;                   // one E' buffer (float2)
  constexpr int HB = (N / 2) * RS;             // the second aperture buffer, 32 rows down
  __shared__ __attribute__((aligned(16))) float2 lds2[2 * EB + (P - 1) * SH::PSTRIDE + N * RS];
  float2* X = lds2 + 2 * EB;

  const Roles<N> r(threadIdx.x);
  const int tid = r.tid;
  const int wl = wg_range_index((int)blockIdx.x, (int)gridDim.x, a.xcd);
  const int m = a.team, tm = wl / m, mk = wl - tm * m, n_team = a.W / m;
  UnitWalk w;                                  // the unit being imaged
  w.T = a.n_time;
  w.ra = range_begin(tm, a.total, n_team);
  w.rb = range_begin(tm + 1, a.total, n_team);
  w.m = m;
  w.k = mk;
  if (tm >= n_team || !w.seek(w.ra / a.n_time)) return;
  int64_t left = member_units(a.n_time, w.ra, w.rb, m, mk);

  float2 tw[S];
#pragma unroll
  for (int k0 = 0; k0 < S; ++k0) tw[k0] = a.twiddle[(r.n0 * k0) % N];

  const int PA = P * a.blk[0].n_ant, L = a.blk[0].L, KB = a.kblock, c0 = a.blk[0].c0;
  const int64_t n_row = (int64_t)a.blk[0].n_chan * PA;
  int eidx[GPT];
  init_stage<NT, GPT, ES>(lds2 + EB, eidx, tid, a.blk[0].n_ant, P);
  init_stage<NT, GPT, ES>(lds2, eidx, tid, a.blk[0].n_ant, P);

  auto load_bytes = [&](int ch, int64_t t, uint32_t (&dst)[GPT]) {
    const uint8_t* src = a.blk[0].efield + t * n_row + (int64_t)(ch - c0) * PA;
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int k = tid + i * NT;
      dst[i] = (k < PA) ? (uint32_t)src[k] : 0u;
    }
  };
  auto load_gains = [&](int ch, float2 (&dst)[GPT]) {
    int t = tid;                               // opaque: the address is not held across the loop
    asm volatile("" : "+v"(t));
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int k = t + i * NT;
      dst[i] = (k < PA) ? a.blk[0].gains[(int64_t)(ch - c0) * PA + k] : make_float2(0.f, 0.f);
    }
  };

  float acc[S][NACC];
  int c = -1, nblk = 0, nflush = 0, line = -1, Lw = L;
  int64_t part_len = 0, slot = 0;
  const uint2* prog = nullptr;
  const float* wim = nullptr;
  auto flush = [&]() {
    double* out = a.partial + slot * (NACC * S * NT) + tid;
    if (part_len <= KB) {
      float* o32 = reinterpret_cast<float*>(a.partial + slot * (NACC * S * NT)) + tid;
#pragma unroll
      for (int u = 0; u < NACC; ++u)
#pragma unroll
        for (int i = 0; i < S; ++i) {
          o32[(u * S + i) * NT] = acc[i][u];
          acc[i][u] = 0.f;
        }
    } else {
#pragma unroll
      for (int u = 0; u < NACC; ++u)
#pragma unroll
        for (int i = 0; i < S; ++i) {
          double* o = out + (u * S + i) * NT;
          *o = (nflush ? *o : 0.0) + (double)acc[i][u];
          acc[i][u] = 0.f;
        }
    }
    ++nflush;
    nblk = 0;
  };

  // the first unit: staged into E' buffer 0 before the loop
  float2 g[GPT];
  uint32_t nxt[GPT];
  int gch = (int)w.s;                          // channel of the gains in g
  load_gains(gch, g);
  load_bytes(gch, w.t, nxt);
  stage_samples<NT, GPT, ES, P, true>(lds2, nxt, g, eidx, tid, PA);
  if (left > 1) {
    UnitWalk wn = w;
    wn.next();
    load_bytes((int)wn.s, wn.t, nxt);
  }
  __syncthreads();

  auto step = [&](auto bc) -> bool {
    constexpr int BUF = decltype(bc)::value;
    float2* Eb = lds2 + BUF * EB;              // E' of this unit
    float2* Xb = X + BUF * HB;                 // its aperture rows
    const int cc = (int)w.s;
    if (cc != c) {                             // a part (accumulation segment) starts
      if (c >= 0) flush();
      c = cc;
      nflush = 0;
      part_len = w.left;
      slot = ((int64_t)c + tm) * m + mk;
      const int64_t cl = c - c0;
      prog = a.blk[0].prog + cl * (L + 1) * NT;
      if (CPX) wim = a.blk[0].wim + cl * (L + 1) * NT + NT;
      line = (int)prog[tid].x;
      Lw = header_steps(prog[tid].y, L);
      prog += NT;
#pragma unroll
      for (int i = 0; i < S; ++i)
#pragma unroll
        for (int u = 0; u < NACC; ++u) acc[i][u] = 0.f;
    } else if (nblk == KB) {
      flush();
    }
    const bool more = left > 1;                // the next unit: staged into the other buffer
    UnitWalk wn = w;
    if (more) {
      wn.next();
      if ((int)wn.s != gch) {
        gch = (int)wn.s;
        load_gains(gch, g);
      }
    }
    stage_and_grid<N, P, NT, RS, ES, GPT, CPX, true, true>(reinterpret_cast<const char*>(Eb),
                                                           reinterpret_cast<char*>(Xb),
                                                           lds2 + (1 - BUF) * EB, prog, wim, Lw,
                                                           nxt, g, eidx, tid, PA, more);
    row_pass<N, P, +1, false>(Xb, r, tw, line);
    if (more) {
      if (left > 2) {                          // prefetch the unit after it
        UnitWalk wnn = wn;
        wnn.next();
        load_bytes((int)wnn.s, wnn.t, nxt);
      }
      w = wn;
    }
    __syncthreads();
    float2 v[P][S];
    column_pass_buf<N>(v, Xb, r, tw);

    // 4. polarisation products: XX, YY, Re XY, Im XY (XY = F_X conj(F_Y))
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const float2 fx = v[0][i], fy = v[1][i];
      acc[i][0] = fmaf(fx.y, fx.y, fmaf(fx.x, fx.x, acc[i][0]));
      acc[i][1] = fmaf(fy.y, fy.y, fmaf(fy.x, fy.x, acc[i][1]));
      acc[i][2] = fmaf(fx.y, fy.y, fmaf(fx.x, fy.x, acc[i][2]));
      acc[i][3] = fmaf(-fx.x, fy.y, fmaf(fx.y, fy.x, acc[i][3]));
    }
    ++nblk;
    return --left > 0;
  };
  while (step(IntC<0>{}) && step(IntC<1>{})) {
  }
  flush();
}

template <int N, int P, int GPT, bool CPX>
__global__ void __launch_bounds__(FusedShape<N>::NT)
__attribute__((amdgpu_waves_per_eu(FusedShape<N>::MIN_WAVES_PER_EU)))
fused_image_kernel(FusedArgs a) {
  if constexpr (N == 64 && P == 2 && GPT == 1 && !CPX) fused_image_body_pipe<N, P, GPT>(a);
  else fused_image_body<N, P, GPT, CPX, false, false>(a);
}

// Apertures wider than N/2 cells (up to 3N/4) at N = 64.  WR > 0: a wide
// block of exactly WR rows (the host launches WR = 40, the deployed array's
// block, with its row count fixed at compile time).
template <int N, int P, int GPT, bool CPX, int WR = 0>
__global__ void __launch_bounds__(FusedShape<N>::NT)
__attribute__((amdgpu_waves_per_eu(FusedShape<N>::MIN_WAVES_PER_EU)))
fused_wide_image_kernel(FusedArgs a) {
  static_assert(N == 64, "the wide variant is built for N = 64");
  fused_image_body<N, P, GPT, CPX, true, false, WR>(a);
}

// The heterogeneous batch: one launch over the channels of several blocks
// of the same grid (WIDE at N = 64: apertures up to 3N/4 cells).
template <int N, int P, int GPT, bool WIDE>
__global__ void __launch_bounds__(FusedShape<N>::NT)
__attribute__((amdgpu_waves_per_eu(FusedShape<N>::MIN_WAVES_PER_EU)))
fused_multi_image_kernel(FusedArgs a) {
  static_assert(!WIDE || N == 64, "the wide variant is built for N = 64");
  fused_image_body<N, P, GPT, false, WIDE, true>(a);
}

// image[c][prod][qm][ql] (+)= sum over the parts of channel c (the members'
// parts of the teams covering it, FusedArgs) of their partial slot.
// THREAD_MAJOR: slots are [NACC][S][NT] as written by the fused kernel (value
// i of thread tid); otherwise [NACC][N*N] in natural pixel order (staged path,
// W = team = 1, float64).  A block of 256 threads handles 256/sub pixels (sub =
// 1, 4, 16 or 64);
// sub-lane j of a pixel sums the parts j, j + sub, ... (in team, then member
// order) and the sub-lane sums are added in the order j = 0, 1, ...: a fixed
// order for a given (W, team, C, T, sub), so the result is reproducible run to
// run.
struct ReduceArgs {
  const double* partial;
  // complex128 [C_b][NPROD][N][N] per block of the launch; channel c of the
  // launch is channel c - img_c0[b] of image[b], b the last block with
  // img_c0[b] <= c
  double* image[kMaxLaunchBlocks];
  int img_c0[kMaxLaunchBlocks];
  int n_img;
  int64_t n_time, total;
  int n_chan, W, reset;     // n_chan: all channels of the launch
  int team, kblock;         // the imaging launch's partition (FusedArgs)
  int f32;                  // parts of <= kblock units hold float32 sums (fused slots)
  int sub;                  // 1, 4, 16 or 64 sub-lanes per pixel
  const double* autos;      // table of the antenna autocorrelations to subtract
                            // ([C][(2K-1)^2][NACC (x2 with autos_cpx)], autos.hpp), or null
  int K;
  int autos_cpx;            // the table has the sin part (complex kernels)
  int transposed;           // bit b set: the slots of image b hold the transposed image
};

// Team whose range contains flat index f: the largest w with
// floor(w * total / W) <= f, i.e. ceil((f + 1) W / total) - 1 (W: the number
// of teams).  Launches take W <= total, so every range is non-empty.
__device__ __forceinline__ int64_t owner_of(int64_t f, int64_t total, int64_t W) {
  return ((f + 1) * W + total - 1) / total - 1;
}

// Sum of the NV values at offset pix of every part of segment sg, sub-lane j
// of sub: the parts of the teams covering the segment, in team then member
// order.  Slots hold NV * stride values (float64, or float32 for parts of at
// most kblock units when f32).
template <int NV>
__device__ __forceinline__ void sum_parts(const double* partial, int64_t sg, int64_t T, int64_t U, int W,
                                          int m, int kblock, int f32, int64_t slot_vals, int64_t stride,
                                          int64_t pix, int j, int sub, double (&s)[NV]) {
  const int64_t n_team = W / m;
  const int lg = __builtin_ctz((unsigned)m);
  const int64_t t_lo = owner_of(sg * T, U, n_team);
  const int64_t t_hi = owner_of((sg + 1) * T - 1, U, n_team);
  const int64_t nq = (t_hi - t_lo + 1) << lg;
  // team ranges [tm U / n_team, (tm + 1) U / n_team) in 32-bit arithmetic where it is exact
  const bool small = (uint64_t)U * (uint64_t)n_team < (1ull << 32);
  auto team_begin = [&](int64_t tm) -> int64_t {
    return small ? (int64_t)((uint32_t)(tm * U) / (uint32_t)n_team) : range_begin(tm, U, n_team);
  };
  int64_t tm_c = -1, L = 0;
#pragma unroll 4
  for (int64_t q = j; q < nq; q += sub) {        // this sub-lane's (team, member) pairs
    const int64_t tm = t_lo + (q >> lg);
    const int k = (int)(q & (m - 1));
    if (tm != tm_c) {                            // the team's piece of segment sg
      tm_c = tm;
      const int64_t ra = team_begin(tm), rb = team_begin(tm + 1);
      const int64_t pa = sg * T > ra ? sg * T : ra;
      const int64_t pb = (sg + 1) * T < rb ? (sg + 1) * T : rb;
      L = pb - pa;
    }
    const int64_t len = (((k + 1) * L) >> lg) - ((k * L) >> lg);
    if (len == 0) continue;
    const int64_t slot = ((sg + tm) << lg) + k;
    if (f32 && len <= kblock) {
      const float* src = reinterpret_cast<const float*>(partial + slot * slot_vals) + pix;
#pragma unroll
      for (int u = 0; u < NV; ++u) s[u] += (double)src[u * stride];
    } else {
      const double* src = partial + slot * slot_vals + pix;
#pragma unroll
      for (int u = 0; u < NV; ++u) s[u] += src[u * stride];
    }
  }
}

// Pixel (km, kl) owned by value i of thread tid in the fused kernel.
template <int N> __device__ __forceinline__ void owned_pixel(int tid, int i, int& km, int& kl) {
  constexpr int S = Line<N>::S, R = Line<N>::R, D = Line<N>::D;
  const Roles<N> r(tid);
  const int q = i / R, k1 = i % R;
  kl = r.kl;
  km = r.n0 * D + q + S * k1;
}

template <int N, int P, bool THREAD_MAJOR>
__global__ void __launch_bounds__(256) reduce_image_kernel(ReduceArgs a) {
  constexpr int NACC = (P == 2) ? 4 : 1;
  constexpr int NPIX = N * N;
  __shared__ double red[NACC * 256];
  __shared__ double ast[AUTO_MAX_D2 * 2 * NACC];
  __shared__ double acs[128], asn[128];
  const int ppb = 256 / a.sub;
  const int j = threadIdx.x / ppb, lp = threadIdx.x % ppb;
  const int64_t idx = (int64_t)blockIdx.x * ppb + lp;
  const bool valid = idx < (int64_t)a.n_chan * NPIX;
  const int c = valid ? (int)(idx / NPIX) : 0;
  const int pix = (int)(idx % NPIX);         // THREAD_MAJOR: i * NT + tid
  double s[NACC];
#pragma unroll
  for (int u = 0; u < NACC; ++u) s[u] = 0.0;
  if (valid)
    sum_parts<NACC>(a.partial, c, a.n_time, a.total, a.W, a.team, a.kblock, a.f32, (int64_t)NACC * NPIX,
                    NPIX, pix, j, a.sub, s);
  // a workgroup's pixels lie in one channel (N^2 is a multiple of 256 / sub)
  if (a.autos)
    stage_autos(a.autos, (int)((int64_t)blockIdx.x * ppb / NPIX), N, a.K,
                a.autos_cpx ? 2 * NACC : NACC, ast, acs, asn);
  combine_sublanes<NACC>(s, a.sub, ppb, j, lp, red);
  if (!valid || j != 0) return;
  int b = 0;                                 // the image of channel c
  for (int i = 1; i < a.n_img; ++i)
    if (a.img_c0[i] <= c) b = i;
  int km, kl;
  if (THREAD_MAJOR) {
    constexpr int NT = FusedShape<N>::NT;
    owned_pixel<N>(pix % NT, pix / NT, km, kl);
    if ((a.transposed >> b) & 1) {           // the kernel imaged the transposed aperture
      const int t = km;
      km = kl;
      kl = t;
    }
  } else {
    km = pix / N;
    kl = pix % N;
  }
  const int qm = (km + N / 2) % N, ql = (kl + N / 2) % N;
  double2* img = reinterpret_cast<double2*>(a.image[b]);
  constexpr int NPROD = (P == 2) ? 4 : 1;
  const int64_t base = (int64_t)(c - a.img_c0[b]) * NPROD * NPIX + qm * N + ql;
  double2 val[NPROD];
  if (P == 2) {
    val[0] = make_double2(s[0], 0.0);                          // XX
    val[1 % NPROD] = make_double2(s[2 % NACC], s[3 % NACC]);   // XY
    val[2 % NPROD] = make_double2(s[2 % NACC], -s[3 % NACC]);  // YX
    val[3 % NPROD] = make_double2(s[1 % NACC], 0.0);           // YY
  } else {
    val[0] = make_double2(s[0], 0.0);
  }
  if (a.autos) {
    double v[NACC];
    if (a.autos_cpx) autos_at<NACC, true>(ast, acs, asn, N, a.K, km, kl, v);
    else autos_at<NACC, false>(ast, acs, asn, N, a.K, km, kl, v);
    val[0].x -= v[0];
    if (P == 2) {
      val[3 % NPROD].x -= v[1 % NACC];
      val[1 % NPROD].x -= v[2 % NACC];
      val[1 % NPROD].y -= v[3 % NACC];
      val[2 % NPROD].x -= v[2 % NACC];
      val[2 % NPROD].y += v[3 % NACC];
    }
  }
#pragma unroll
  for (int pr = 0; pr < NPROD; ++pr) {
    double2* o = img + base + (int64_t)pr * NPIX;
    if (a.reset) {
      *o = val[pr];
    } else {
      const double2 old = *o;
      *o = make_double2(old.x + val[pr].x, old.y + val[pr].y);
    }
  }
}

}  // namespace epic
