// Fused imaging kernel: one workgroup walks a contiguous range of the
// flattened (channel, time) index space and, for every sample, runs the whole
// hot path with the data resident in LDS and registers:
//
//   1. unpack the P*A 4+4-bit samples of (t, c) and multiply by the gains
//      (paper Sec. 3.2), into LDS;
//   2. grid them with the illumination kernel (Sec. 2.1, Eq. (4)-(5)) by a
//      gather: every thread runs a precomputed list of (cell, antenna, weight)
//      steps and writes whole cells, so no two threads touch the same cell and
//      no atomics are needed; only the rows the aperture touches (the "band")
//      are gridded and transformed along rows;
//   3. transform rows then columns with the +i sign (Sec. 2.1, Eq. (5));
//      the row transform works in place in each row's LDS storage, the column
//      transform reads the band rows and keeps its results in registers;
//   4. form XX, YY and XY (YX = conj XY) for the pixels each thread owns and
//      add them to float64 accumulators held in registers (Sec. 2.1, Sec. 3.2).
//
// At a channel boundary (and at the end of its range) a workgroup writes its
// float64 sums to its own partial-image slot; a second kernel adds the slots
// of each channel in workgroup order.
#pragma once
#include "dft.hpp"

namespace epic {

// Gridding step encoding (one uint2 per step: {code, weight bits}).
constexpr uint32_t STEP_CELL_MASK = 0x3FFFu;   // cell index j*N + i (N <= 128)
constexpr uint32_t STEP_HAS = 1u << 14;        // accumulate w * E'[ant]
constexpr uint32_t STEP_LAST = 1u << 15;       // write the cell, restart the sum
constexpr int STEP_ANT_SHIFT = 16;             // antenna index in bits 16..31

template <int N> struct FusedShape {
  static constexpr int S = Line<N>::S, R = Line<N>::R, D = Line<N>::D;
  static constexpr int NT = N * R;             // threads per workgroup
  static constexpr int CPW = 64 / R;           // columns (or rows) per wave
  static constexpr int RS = N + 4;             // LDS row stride in float2
};

struct FusedArgs {
  const uint8_t* efield;    // [T][C][P][A]
  const float2* gains;      // [C][P][A]
  const uint2* prog;        // [C][L][NT]
  const int4* chan;         // [C] {j_lo, nb, L, 0}
  const float2* twiddle;    // [N] exp(+2 pi i k / N)
  double* partial;          // [W + C - 1][NACC][N*N], pixel = km*N + kl
  int64_t n_time;
  int64_t total;            // C * T
  int n_chan, n_ant, L, W;
};

// Flat range of workgroup w: [w*total/W, (w+1)*total/W).
__device__ __forceinline__ int64_t range_begin(int64_t w, int64_t total, int64_t W) {
  return (w * total) / W;
}

// Lane roles shared by the row and column passes: the R lanes of a line are
// n0-major inside a wave (lane = n0 * CPW + sub), so both passes use the same
// twiddles.
template <int N> struct Roles {
  int tid, wave, n0, sub, kl;
  __device__ __forceinline__ explicit Roles(int t) {
    constexpr int CPW = FusedShape<N>::CPW;
    tid = t;
    wave = t >> 6;
    const int lane = t & 63;
    n0 = lane / CPW;
    sub = lane % CPW;
    kl = wave * CPW + sub;
  }
};

__device__ __forceinline__ float2 unpack_ci4(uint32_t b) {
  const int v = (int)b;
  return make_float2((float)((v >> 4) - ((v & 0x80) ? 16 : 0)),
                     (float)((v & 0xF) - ((v & 0x8) ? 16 : 0)));
}

// 1. E'[k] = g[k] * e[k] for the items k = tid + i*NT of this thread.
template <int NT, int GPT>
__device__ __forceinline__ void stage_samples(float2* E, const uint32_t (&cur)[GPT],
                                              const float2 (&g)[GPT], int tid, int PA) {
#pragma unroll
  for (int i = 0; i < GPT; ++i) {
    const int k = tid + i * NT;
    if (k < PA) {
      const float2 e = unpack_ci4(cur[i]);
      E[k] = cmul(g[i], e);
    }
  }
}

constexpr int kStepChunk = 16;

template <int NT>
__device__ __forceinline__ void load_steps(uint2 (&steps)[kStepChunk], const uint2* prog, int st0,
                                           int L) {
#pragma unroll
  for (int st = 0; st < kStepChunk; ++st)
    steps[st] = (st0 + st < L) ? prog[(int64_t)(st0 + st) * NT] : make_uint2(0u, 0u);
}

// 2. Gather gridding of the band cells, both polarisations per step.  The
// first chunk of steps has been loaded by the caller.
template <int N, int P, int NT, int RS>
__device__ __forceinline__ void grid_band(float2* X, const float2* E, uint2 (&steps)[kStepChunk],
                                          const uint2* prog, int L, int n_ant) {
  float2 s0 = make_float2(0.f, 0.f), s1 = make_float2(0.f, 0.f);
  for (int st0 = 0; st0 < L; st0 += kStepChunk) {
    if (st0 > 0) load_steps<NT>(steps, prog, st0, L);
#pragma unroll
    for (int st = 0; st < kStepChunk; ++st) {
      const uint32_t code = steps[st].x;
      const float w = __uint_as_float(steps[st].y);
      if (code & STEP_HAS) {
        const int ant = (int)(code >> STEP_ANT_SHIFT);
        const float2 e0 = E[ant];
        s0.x = fmaf(w, e0.x, s0.x);
        s0.y = fmaf(w, e0.y, s0.y);
        if (P == 2) {
          const float2 e1 = E[n_ant + ant];
          s1.x = fmaf(w, e1.x, s1.x);
          s1.y = fmaf(w, e1.y, s1.y);
        }
      }
      if (code & STEP_LAST) {
        const int cell = (int)(code & STEP_CELL_MASK);
        const int j = cell / N, i = cell % N;
        X[j * RS + i] = s0;
        if (P == 2) X[(N + j) * RS + i] = s1;
        s0 = make_float2(0.f, 0.f);
        s1 = make_float2(0.f, 0.f);
      }
    }
  }
}

// 3a. Row transforms of the P*nb band rows, in place (each row private to the
// R lanes of one wave).
template <int N, int P, int SG>
__device__ __forceinline__ void row_pass(float2* X, const Roles<N>& r, const float2* tw, int j_lo,
                                         int nb) {
  constexpr int S = Line<N>::S, R = Line<N>::R, D = Line<N>::D;
  constexpr int NT = FusedShape<N>::NT, CPW = FusedShape<N>::CPW, RS = FusedShape<N>::RS;
  for (int line0 = r.wave * CPW; line0 < P * nb; line0 += NT / R) {
    const int line = line0 + r.sub;
    if (line < P * nb) {
      const int p = line / nb;
      const int j = j_lo + (line - p * nb);
      float2* row = X + (p * N + j) * RS;
      float2 v[1][S];
      if (SG > 0) {
#pragma unroll
        for (int n1 = 0; n1 < S; ++n1) v[0][n1] = row[R * n1 + r.n0];
        line_transform<N, +1, 1>(v, tw, r.n0, row, [](int, int s) { return s; });
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
#pragma unroll
        for (int n1 = 0; n1 < S; ++n1) row[R * n1 + r.n0] = v[0][n1];
      }
    }
  }
}

// 3b. Forward column transforms of column r.kl for all polarisations; rows
// outside the band are zero.  Out: v[p][q R + k1] = F_p[n0 D + q + S k1][kl].
template <int N, int P>
__device__ __forceinline__ void column_pass_fwd(float2 (&v)[P][Line<N>::S], float2* X,
                                                const Roles<N>& r, const float2* tw, int j_lo,
                                                int nb) {
  constexpr int S = Line<N>::S, R = Line<N>::R, RS = FusedShape<N>::RS;
  const int kl = r.kl;
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int n1 = 0; n1 < S; ++n1) {
      const int j = R * n1 + r.n0;
      v[p][n1] = ((unsigned)(j - j_lo) < (unsigned)nb) ? X[(p * N + j) * RS + kl]
                                                       : make_float2(0.f, 0.f);
    }
  line_transform<N, +1, P>(v, tw, r.n0, X, [kl](int p, int s) { return (p * N + s) * RS + kl; });
}

template <int N, int P, int GPT>
__global__ void __launch_bounds__(FusedShape<N>::NT)
fused_image_kernel(FusedArgs a) {
  using SH = FusedShape<N>;
  constexpr int S = SH::S, R = SH::R, D = SH::D, NT = SH::NT, RS = SH::RS;
  constexpr int NACC = (P == 2) ? 4 : 1;
  __shared__ float2 X[P * N * RS];             // gridded aperture / row transforms
  __shared__ float2 E[NT * GPT];               // calibrated samples E'[p][a]

  const Roles<N> r(threadIdx.x);
  const int tid = r.tid;
  const int64_t fb = range_begin(blockIdx.x, a.total, a.W);
  const int64_t fe = range_begin(blockIdx.x + 1, a.total, a.W);
  if (fb >= fe) return;

  float2 tw[S];
#pragma unroll
  for (int k0 = 0; k0 < S; ++k0) tw[k0] = a.twiddle[(r.n0 * k0) % N];

  const int PA = P * a.n_ant;
  const int64_t row_bytes = (int64_t)a.n_chan * PA;   // bytes per time sample

  double acc[S][NACC];
  float2 g[GPT];
  uint32_t nxt[GPT];
  int c = -1, j_lo = 0, nb = 0;
  const uint2* prog = nullptr;

  auto load_bytes = [&](int cc, int64_t tt, uint32_t (&dst)[GPT]) {
    const uint8_t* src = a.efield + tt * row_bytes + (int64_t)cc * PA;
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int k = tid + i * NT;
      dst[i] = (k < PA) ? (uint32_t)src[k] : 0u;
    }
  };

  auto flush = [&]() {
    double* out = a.partial + (int64_t)(blockIdx.x + c) * NACC * N * N;
#pragma unroll
    for (int q = 0; q < D; ++q)
#pragma unroll
      for (int k1 = 0; k1 < R; ++k1) {
        const int km = r.n0 * D + q + S * k1;
#pragma unroll
        for (int u = 0; u < NACC; ++u)
          out[(int64_t)u * N * N + km * N + r.kl] = acc[q * R + k1][u];
      }
  };

  // current sample (cc, tt); one division per workgroup
  int cc = (int)(fb / a.n_time);
  int64_t tt = fb - (int64_t)cc * a.n_time;
  load_bytes(cc, tt, nxt);
  for (int64_t left = fe - fb; left > 0; --left) {
    if (cc != c) {                             // channel segment starts
      if (c >= 0) flush();
      c = cc;
      const int4 ci = a.chan[c];
      j_lo = ci.x;
      nb = ci.y;
      prog = a.prog + (int64_t)c * a.L * NT + tid;
#pragma unroll
      for (int i = 0; i < S; ++i)
#pragma unroll
        for (int u = 0; u < NACC; ++u) acc[i][u] = 0.0;
#pragma unroll
      for (int i = 0; i < GPT; ++i) {
        const int k = tid + i * NT;
        g[i] = (k < PA) ? a.gains[(int64_t)c * PA + k] : make_float2(0.f, 0.f);
      }
    }
    uint32_t cur[GPT];
#pragma unroll
    for (int i = 0; i < GPT; ++i) cur[i] = nxt[i];
    ++tt;                                      // advance, prefetch the next sample
    if (tt == a.n_time) { tt = 0; ++cc; }
    if (left > 1) load_bytes(cc, tt, nxt);

    uint2 steps[kStepChunk];
    load_steps<NT>(steps, prog, 0, a.L);       // latency overlaps the barrier below
    stage_samples<NT, GPT>(E, cur, g, tid, PA);
    __syncthreads();
    grid_band<N, P, NT, RS>(X, E, steps, prog, a.L, a.n_ant);
    __syncthreads();
    row_pass<N, P, +1>(X, r, tw, j_lo, nb);
    __syncthreads();
    float2 v[P][S];
    column_pass_fwd<N, P>(v, X, r, tw, j_lo, nb);

    // 4. polarisation products into float64 sums
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const float2 fx = v[0][i];
      acc[i][0] += (double)fmaf(fx.x, fx.x, fx.y * fx.y);
      if (P == 2) {
        const float2 fy = v[P - 1][i];
        acc[i][1 % NACC] += (double)fmaf(fy.x, fy.x, fy.y * fy.y);
        acc[i][2 % NACC] += (double)fmaf(fx.x, fy.x, fx.y * fy.y);
        acc[i][3 % NACC] += (double)fmaf(fx.y, fy.x, -fx.x * fy.y);
      }
    }
  }
  flush();
}

// image[c][prod][qm][ql] (+)= sum over the workgroups covering channel c of
// their partial slot, in workgroup order.  One thread per (c, pixel).
struct ReduceArgs {
  const double* partial;    // [W + C - 1][NACC][N*N]
  double* image;            // complex128 [C][NPROD][N][N]
  int64_t n_time, total;
  int n_chan, W, reset;
};

// Workgroup whose range contains flat index f: the largest w with
// floor(w * total / W) <= f, i.e. ceil((f + 1) W / total) - 1.
__device__ __forceinline__ int64_t owner_of(int64_t f, int64_t total, int64_t W) {
  return ((f + 1) * W + total - 1) / total - 1;
}

template <int N, int P>
__global__ void __launch_bounds__(256) reduce_image_kernel(ReduceArgs a) {
  constexpr int NACC = (P == 2) ? 4 : 1;
  constexpr int NPIX = N * N;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)a.n_chan * NPIX) return;
  const int c = (int)(idx / NPIX);
  const int pix = (int)(idx % NPIX);
  const int km = pix / N, kl = pix % N;
  const int64_t w_lo = owner_of((int64_t)c * a.n_time, a.total, a.W);
  const int64_t w_hi = owner_of((int64_t)(c + 1) * a.n_time - 1, a.total, a.W);
  double s[NACC];
#pragma unroll
  for (int u = 0; u < NACC; ++u) s[u] = 0.0;
  for (int64_t w = w_lo; w <= w_hi; ++w) {
    if (range_begin(w, a.total, a.W) == range_begin(w + 1, a.total, a.W)) continue;
    const double* src = a.partial + (w + c) * NACC * NPIX + pix;
#pragma unroll
    for (int u = 0; u < NACC; ++u) s[u] += src[(int64_t)u * NPIX];
  }
  const int qm = (km + N / 2) % N, ql = (kl + N / 2) % N;
  double2* img = reinterpret_cast<double2*>(a.image);
  constexpr int NPROD = (P == 2) ? 4 : 1;
  const int64_t base = (int64_t)c * NPROD * NPIX + qm * N + ql;
  double2 val[NPROD];
  if (P == 2) {
    val[0] = make_double2(s[0], 0.0);          // XX
    val[1 % NPROD] = make_double2(s[2], s[3]); // XY
    val[2 % NPROD] = make_double2(s[2], -s[3]);// YX
    val[3 % NPROD] = make_double2(s[1], 0.0);  // YY
  } else {
    val[0] = make_double2(s[0], 0.0);
  }
#pragma unroll
  for (int pr = 0; pr < NPROD; ++pr) {
    double2* o = img + base + (int64_t)pr * NPIX;
    if (a.reset) {
      *o = val[pr];
    } else {
      double2 old = *o;
      *o = make_double2(old.x + val[pr].x, old.y + val[pr].y);
    }
  }
}

}  // namespace epic
