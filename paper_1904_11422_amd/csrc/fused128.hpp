// Fused imaging kernel for 128 x 128 grids (paper Sec. 2.1 Eq. (4)-(5),
// Sec. 3.2), the same per-sample path as fused_image_kernel with a different
// split of the work.
//
// With two polarisations the 64 x 64 aperture block fills most of the LDS,
// and the float32 sums of all 128 x 128 pixels would not fit the registers of
// one workgroup.  So a workgroup of 512 threads images one half of the output
// columns of a sample, kl in [64 h, 64 h + 64):
//   1. unpack + gain, barrier, gridding of the whole aperture (wave-local rows,
//      as fused_image_kernel);
//   2. row transforms: a group of 8 lanes takes one aperture row of every
//      polarisation (16-point first pass with half of its inputs zero, one
//      exchange through the row's 128 slots, two 8-point passes) and writes
//      the 64 outputs of half h back to the row's first 64 columns;  barrier;
//   3. column transforms: a group of 8 lanes takes one local column of every
//      polarisation, exchanging through the column's 64 aperture rows and the
//      same rows' upper 64 columns; every lane then holds F_X (and F_Y) of 16
//      pixels;
//   4. XX (and YY, Re XY, Im XY) into float32 sums, added every 128 samples
//      and at a segment boundary into the workgroup's float64 slot.
// One polarisation uses the same split: half the LDS (two workgroups per CU)
// and a quarter of the sums.
// Work units are (channel, half, sample), flattened as ((2 c + h) T + t); a
// (channel, half) pair is one accumulation segment.
#pragma once
#include "fused.hpp"

namespace epic {

struct Fused128Args {
  const uint8_t* efield;    // [T][C][P][A]
  const float2* gains;      // [C][P][A]
  const uint2* prog;        // [C][1 + L][NT], as fused_image_kernel
  const float* wim;         // [C][1 + L][NT] imaginary step weights (complex kernels), or null
  const float2* twiddle;    // [128] exp(+2 pi i k / 128)
  double* partial;          // [W + 2 C - 1][NACC][16][NT] (thread-major)
  int64_t n_time;
  int64_t total;            // 2 C T units
  int n_chan, n_ant, L, W;
};

// Local pixel of float32 sum i of a thread: km = 2 n0 + q + 16 k1 with
// q = i >> 3 and k1 = i & 7; kl = the thread's local column (Roles::kl).
__host__ __device__ __forceinline__ int km128(int n0, int i) {
  return 2 * n0 + (i >> 3) + 16 * (i & 7);
}

// Two polarisations: one workgroup per CU (LDS), registers up to 256; one
// polarisation: two workgroups per CU, so at most 128 VGPRs.
template <int P> struct Fused128Waves { static constexpr int value = P == 2 ? 2 : 4; };

template <int P, int GPT, bool CPX>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(Fused128Waves<P>::value)))
fused_image128_kernel(Fused128Args a) {
  using SH = FusedShape<128>;
  constexpr int N = 128, S = SH::S, R = SH::R, NT = SH::NT, RS = SH::RS, PS = SH::PSTRIDE;
  constexpr int NACC = P == 2 ? 4 : 1, KB = SH::KBLOCK, H = N / 2, NPX = 16;
  constexpr int ES = EStride<NT, GPT, P>::value;
  constexpr int XBASE = P * ES * (int)sizeof(float2);
  // E'[p][a] (zero slots at a = A .. A+15), the grid (64 rows per
  // polarisation), then the twiddles w^(n0 k0) of the 8 lane roles n0, rows of
  // 17 so that the roles of a half-wave read distinct banks
  constexpr int TWS = 17;
  __shared__ float2 lds2[P * ES + (P - 1) * PS + H * RS + R * TWS];
  char* lds = reinterpret_cast<char*>(lds2);
  float2* E = lds2;
  float2* X = lds2 + P * ES;
  float2* TW = X + (P - 1) * PS + H * RS;

  const Roles<N> r(threadIdx.x);
  const int tid = r.tid;
  const int64_t fb = range_begin(blockIdx.x, a.total, a.W);
  const int64_t fe = range_begin(blockIdx.x + 1, a.total, a.W);
  if (fb >= fe) return;

  if (tid < R * S) TW[(tid / S) * TWS + tid % S] = a.twiddle[((tid / S) * (tid % S)) % N];
  const float2* tw = TW + r.n0 * TWS;          // read after the first barrier

  const int PA = P * a.n_ant;
  const int64_t row_bytes = (int64_t)a.n_chan * PA;
  int eidx[GPT];
  init_stage<NT, GPT, ES>(E, eidx, tid, a.n_ant, P);

  float acc[NPX][NACC];
  float2 g[GPT];
  uint32_t nxt[GPT];
  int seg = -1, nblk = 0, nflush = 0, line = -1, h = 0;
  const uint2* prog = nullptr;
  const float* wim = nullptr;

  auto load_bytes = [&](int64_t sg, int64_t tt, uint32_t (&dst)[GPT]) {
    const uint8_t* src = a.efield + tt * row_bytes + (sg >> 1) * PA;
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int k = tid + i * NT;
      dst[i] = (k < PA) ? (uint32_t)src[k] : 0u;
    }
  };
  auto flush = [&]() {
    double* out = a.partial + (int64_t)(blockIdx.x + seg) * NACC * NPX * NT + tid;
#pragma unroll
    for (int u = 0; u < NACC; ++u)
#pragma unroll
      for (int i = 0; i < NPX; ++i) {
        double* o = out + (u * NPX + i) * NT;
        *o = (nflush ? *o : 0.0) + (double)acc[i][u];
        acc[i][u] = 0.f;
      }
    ++nflush;
    nblk = 0;
  };

  int64_t sg = fb / a.n_time;                  // segment 2 c + h of the current unit
  int64_t tt = fb - sg * a.n_time;
  load_bytes(sg, tt, nxt);
  for (int64_t left = fe - fb; left > 0; --left) {
    if ((int)sg != seg) {
      if (seg >= 0) flush();
      const int c_old = seg >> 1;
      seg = (int)sg;
      const int c = seg >> 1;
      h = seg & 1;
      nflush = 0;
#pragma unroll
      for (int i = 0; i < NPX; ++i)
#pragma unroll
        for (int u = 0; u < NACC; ++u) acc[i][u] = 0.f;
      if (c != c_old) {
        prog = a.prog + (int64_t)c * (a.L + 1) * NT;
        if (CPX) wim = a.wim + (int64_t)c * (a.L + 1) * NT + NT;
        line = (int)prog[tid].x;
        prog += NT;
#pragma unroll
        for (int i = 0; i < GPT; ++i) {
          const int k = tid + i * NT;
          g[i] = (k < PA) ? a.gains[(int64_t)c * PA + k] : make_float2(0.f, 0.f);
        }
      }
    } else if (nblk == KB) {
      flush();
    }
    uint32_t cur[GPT];
#pragma unroll
    for (int i = 0; i < GPT; ++i) cur[i] = nxt[i];
    ++tt;                                      // advance, prefetch the next unit
    if (tt == a.n_time) { tt = 0; ++sg; }
    if (left > 1) load_bytes(sg, tt, nxt);

    // 1. stage and grid the aperture (both halves grid the whole aperture)
    stage_and_grid<N, P, NT, RS, ES, GPT, CPX>(lds, XBASE, E, prog, wim, a.L, cur, g, eidx, tid, PA);

    // 2. row transforms of row `line` of both polarisations; keep half h
    if (line >= 0) {
      const int rb = (line & 0xFFFF) * RS;
      float2 v[P][S];
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int n1 = 0; n1 < S / 2; ++n1) v[p][n1] = X[p * PS + rb + R * n1 + r.n0];
      line_transform<N, +1, P, true>(v, tw, r.n0, X, [rb](int p, int s) { return p * PS + rb + s; });
      // v[p][q R + k1] = X_p[2 n0 + q + 16 k1]; half h holds k1 in [4 h, 4 h + 4)
      // (h is uniform over the workgroup: a branch, not a per-value select)
      if (h) {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
          for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int k = 0; k < 4; ++k) X[p * PS + rb + 2 * r.n0 + q + 16 * k] = v[p][q * R + 4 + k];
      } else {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
          for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int k = 0; k < 4; ++k) X[p * PS + rb + 2 * r.n0 + q + 16 * k] = v[p][q * R + k];
      }
    }
    __syncthreads();

    // 3. column transforms of local column r.kl of both polarisations
    const int kl = r.kl;
    float2 v[P][S];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int n1 = 0; n1 < S / 2; ++n1) v[p][n1] = X[p * PS + (R * n1 + r.n0) * RS + kl];
    line_transform<N, +1, P, true>(v, tw, r.n0, X,
                                   [kl](int p, int s) { return p * PS + (s & 63) * RS + kl + (s & 64); });
    // v[p][q R + k1] = F_p[2 n0 + q + 16 k1][64 h + kl]

    // 4. products of the 16 pixels: XX (, YY, Re XY, Im XY; XY = F_X conj(F_Y))
#pragma unroll
    for (int i = 0; i < NPX; ++i) {
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

// image[c][prod][qm][ql] (+)= sum of the slots of segment 2 c + h, for the
// pixels of half h; sub-lanes as reduce_image_kernel.
struct Reduce128Args {
  const double* partial;
  double* image;            // complex128 [C][NPROD][128][128]
  int64_t n_time, total;
  int n_chan, W, reset, sub;
};

template <int P>
__global__ void __launch_bounds__(256) reduce_image128_kernel(Reduce128Args a) {
  constexpr int N = 128, NT = FusedShape<128>::NT, NLOC = 16 * NT;   // local pixels per half
  constexpr int NACC = P == 2 ? 4 : 1, NPROD = P == 2 ? 4 : 1;
  __shared__ double red[NACC * 256];
  const int ppb = 256 / a.sub;
  const int j = threadIdx.x / ppb, lp = threadIdx.x % ppb;
  const int64_t idx = (int64_t)blockIdx.x * ppb + lp;
  const bool valid = idx < (int64_t)a.n_chan * 2 * NLOC;
  const int sgm = valid ? (int)(idx / NLOC) : 0;            // 2 c + h
  const int pix = (int)(idx % NLOC);                        // i * NT + tid
  double s[NACC];
#pragma unroll
  for (int u = 0; u < NACC; ++u) s[u] = 0.0;
  if (valid) {
    const int64_t w_lo = owner_of((int64_t)sgm * a.n_time, a.total, a.W);
    const int64_t w_hi = owner_of((int64_t)(sgm + 1) * a.n_time - 1, a.total, a.W);
#pragma unroll 4
    for (int64_t w = w_lo + j; w <= w_hi; w += a.sub) {
      const double* src = a.partial + (w + sgm) * NACC * NLOC + pix;
#pragma unroll
      for (int u = 0; u < NACC; ++u) s[u] += src[(int64_t)u * NLOC];
    }
  }
  combine_sublanes<NACC>(s, a.sub, ppb, j, lp, red);
  if (!valid || j != 0) return;
  const int tid = pix % NT, i = pix / NT;
  const Roles<N> r(tid);
  const int c = sgm >> 1, h = sgm & 1;
  const int km = km128(r.n0, i), kl = 64 * h + r.kl;
  const int qm = (km + N / 2) % N, ql = (kl + N / 2) % N;
  double2* img = reinterpret_cast<double2*>(a.image);
  const int64_t base = (int64_t)c * NPROD * N * N + qm * N + ql;
  double2 val[NPROD];
  val[0] = make_double2(s[0], 0.0);
  if (P == 2) {
    val[1 % NPROD] = make_double2(s[2 % NACC], s[3 % NACC]);
    val[2 % NPROD] = make_double2(s[2 % NACC], -s[3 % NACC]);
    val[3 % NPROD] = make_double2(s[1 % NACC], 0.0);
  }
#pragma unroll
  for (int pr = 0; pr < NPROD; ++pr) {
    double2* o = img + base + (int64_t)pr * N * N;
    if (a.reset) {
      *o = val[pr];
    } else {
      const double2 old = *o;
      *o = make_double2(old.x + val[pr].x, old.y + val[pr].y);
    }
  }
}

}  // namespace epic
