// Adjoint of the fused imaging kernel: gradient of a real loss with respect
// to the per-antenna complex gains, given dL/dI for the accumulated image.
//
// Per sample (nothing is stored across samples, the forward is recomputed):
//   F_p      = forward transform of the gridded aperture (as in the imager)
//   G_X      = Re(Gxx) F_X + h F_Y,   G_Y = Re(Gyy) F_Y + conj(h) F_X,
//              h = (Gxy + conj(Gyx)) / 2          (dL/dF_p*, Wirtinger calculus)
//   H_p      = adjoint transform of G_p (negative exponent), columns then rows
//   dL/dg*   += sum_taps conj(w) * conj(e[t,c,p,a]) * H_p[tap]
// The per-antenna sums are float64, one slot per (workgroup, channel); a
// second kernel adds the slots in workgroup order and returns 2 dL/dg*, i.e.
// dL/dRe(g) + i dL/dIm(g).
#pragma once
#include "fused.hpp"

namespace epic {

struct AdjointArgs {
  const uint8_t* efield;    // [T][C][P][A]
  const float2* gains;      // [C][P][A]
  const float4* gtab;       // [C][S][NT]: {Re Gxx, Re Gyy, Re h, Im h} at owned pixels
  const uint2* prog;        // gridding programs and row-pass lines, as the imager
  const float* wim;         // imaginary step weights (complex kernels), or null
  const float* tapim;       // [C][A][KK] imaginary tap weights (complex kernels), or null
  const uint2* taps;        // [C][A][KK] {translated cell's grid offset phys_row(j)*RS + i, w bits}
  const float2* twiddle;
  double2* gpartial;        // [W + C - 1][P*A]
  int64_t n_time, total;
  int n_chan, n_ant, kk, L, W;
  int wrows;                // wide block: its row count (the column pass reads rows below it)
};

// The upstream gradient at the pixels each thread of the fused kernels owns,
// as float32 {Re Gxx, Re Gyy, Re h, Im h} with h = (Gxy + conj(Gyx)) / 2:
// gtab[c][i][tid] for value i of thread tid.  Read once per sample by the
// adjoint kernel (L2-resident), so it need not occupy registers.
struct GradTableArgs {
  const double2* grad_image;// [C][NPROD][N][N] (fftshifted)
  float4* gtab;
  int n_chan;
  int transposed;           // the imaging programs grid the transposed aperture
};

template <int N, int P>
__global__ void __launch_bounds__(256) grad_table_kernel(GradTableArgs a) {
  using SH = FusedShape<N>;
  constexpr int S = SH::S, R = SH::R, D = SH::D, NT = SH::NT, NPROD = (P == 2) ? 4 : 1;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)a.n_chan * S * NT) return;
  const int c = (int)(idx / (S * NT));
  const int i = (int)((idx / NT) % S), tid = (int)(idx % NT);
  const Roles<N> r(tid);
  const int q = i / R, k1 = i % R;
  const int km = r.n0 * D + q + S * k1;
  const int pm = a.transposed ? r.kl : km, pl = a.transposed ? km : r.kl;   // image row, column
  const int pix = ((pm + N / 2) % N) * N + (pl + N / 2) % N;
  const double2* gi = a.grad_image + (int64_t)c * NPROD * N * N;
  float4 t;
  t.x = (float)gi[pix].x;
  if (P == 2) {
    const double2 xy = gi[N * N + pix], yx = gi[2 * N * N + pix];
    t.y = (float)gi[3 * N * N + pix].x;
    t.z = (float)(0.5 * (xy.x + yx.x));
    t.w = (float)(0.5 * (xy.y - yx.y));
  } else {
    t.y = t.z = t.w = 0.f;
  }
  a.gtab[idx] = t;
}

// WIDE (N = 64): the wide block of the forward (columns < HW, rows < wrows, a
// second row-pass line per thread in the program header's second word); the
// adjoint column transforms write back rows < HW, of which the adjoint row
// passes and the degridding read those of the block.
template <int N, int P, int GPT, bool CPX, bool WIDE>
__device__ __forceinline__ void adjoint_body(const AdjointArgs& a) {
  using SH = FusedShape<N>;
  constexpr int S = SH::S, R = SH::R, D = SH::D, NT = SH::NT, RS = SH::RS;
  constexpr int ES = EStride<NT, GPT, P>::value;
  constexpr int XBASE = P * ES * (int)sizeof(float2);
  constexpr int PS = SH::PSTRIDE;
  // E'[p][a] (zero slots at a = A .. A+15), then the grid
  __shared__ __attribute__((aligned(16))) float2 lds2[P * ES + (P - 1) * PS + N * RS];
  char* lds = reinterpret_cast<char*>(lds2);
  float2* E = lds2;
  float2* X = lds2 + P * ES;

  const Roles<N> r(threadIdx.x);
  const int tid = r.tid;
  const int64_t fb = range_begin(blockIdx.x, a.total, a.W);
  const int64_t fe = range_begin(blockIdx.x + 1, a.total, a.W);
  if (fb >= fe) return;

  float2 tw[S];
#pragma unroll
  for (int k0 = 0; k0 < S; ++k0) tw[k0] = a.twiddle[(r.n0 * k0) % N];

  const int PA = P * a.n_ant;
  const int64_t row_bytes = (int64_t)a.n_chan * PA;
  int eidx[GPT];
  init_stage<NT, GPT, ES>(E, eidx, tid, a.n_ant, P);

  double2 gacc[GPT];
  float2 g[GPT];
  uint32_t nxt[GPT];
  int c = -1, line = -1, line2 = -1, Lw = a.L;
  const uint2* prog = nullptr;
  const float* wim = nullptr;

  auto load_bytes = [&](int cc, int64_t tt, uint32_t (&dst)[GPT]) {
    const uint8_t* src = a.efield + tt * row_bytes + (int64_t)cc * PA;
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int k = tid + i * NT;
      dst[i] = (k < PA) ? (uint32_t)src[k] : 0u;
    }
  };
  auto flush = [&]() {
    double2* out = a.gpartial + (int64_t)(blockIdx.x + c) * PA;
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int k = tid + i * NT;
      if (k < PA) out[k] = gacc[i];
    }
  };

  int cc = (int)(fb / a.n_time);
  int64_t tt = fb - (int64_t)cc * a.n_time;
  load_bytes(cc, tt, nxt);
  for (int64_t left = fe - fb; left > 0; --left) {
    if (cc != c) {
      if (c >= 0) flush();
      c = cc;
      prog = a.prog + (int64_t)c * (a.L + 1) * NT;
      if (CPX) wim = a.wim + (int64_t)c * (a.L + 1) * NT + NT;
      line = (int)prog[tid].x;
      if (WIDE) line2 = header_line2(prog[tid].y);
      Lw = header_steps(prog[tid].y, a.L);
      prog += NT;
#pragma unroll
      for (int i = 0; i < GPT; ++i) {
        const int k = tid + i * NT;
        g[i] = (k < PA) ? a.gains[(int64_t)c * PA + k] : make_float2(0.f, 0.f);
        gacc[i] = make_double2(0.0, 0.0);
      }
    }
    uint32_t cur[GPT];
#pragma unroll
    for (int i = 0; i < GPT; ++i) cur[i] = nxt[i];
    ++tt;
    if (tt == a.n_time) { tt = 0; ++cc; }
    if (left > 1) load_bytes(cc, tt, nxt);

    stage_and_grid<N, P, NT, RS, ES, GPT, CPX>(lds, lds + XBASE, E, prog, wim, Lw, cur, g, eidx, tid, PA);
    row_pass<N, P, +1, WIDE>(X, r, tw, line);
    if (WIDE) row_pass<N, P, +1, WIDE>(X, r, tw, line2);
    __syncthreads();
    float2 v[P][S];
    column_pass_fwd<N, P, WIDE>(v, X, r, tw, a.wrows);

    // dL/dF* at the owned pixels
    const float4* gt = a.gtab + (int64_t)c * S * NT + tid;
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const float4 t = gt[i * NT];
      const float2 fx = v[0][i];
      if (P == 2) {
        const float2 fy = v[P - 1][i];
        const float2 gh = make_float2(t.z, t.w);
        const float2 hx = cmul(gh, fy);         // h F_Y
        const float2 hy = cmulc(fx, gh);        // conj(h) F_X
        v[0][i] = make_float2(fmaf(t.x, fx.x, hx.x), fmaf(t.x, fx.y, hx.y));
        v[P - 1][i] = make_float2(fmaf(t.y, fy.x, hy.x), fmaf(t.y, fy.y, hy.y));
      } else {
        v[0][i] = cscale(fx, t.x);
      }
    }
    // adjoint column transforms, results to the aperture rows of each column
    const int kl = r.kl;
    line_transform_rev<N, -1, P>(v, tw, r.n0, X,
                                 [kl](int p, int s) { return p * PS + s * RS + kl; });
    constexpr int NOUT = WIDE ? SH::HW / R : S / 2;   // aperture rows written back
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int n1 = 0; n1 < NOUT; ++n1) X[p * PS + SH::phys_row(R * n1 + r.n0) * RS + kl] = v[p][n1];
    __syncthreads();
    row_pass<N, P, -1, WIDE>(X, r, tw, line);
    if (WIDE) row_pass<N, P, -1, WIDE>(X, r, tw, line2);
    __syncthreads();

    // degrid: dL/de'* at each antenna, times conj(e)
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int k = tid + i * NT;
      if (k < PA) {
        const int p = k / a.n_ant, ant = k - p * a.n_ant;
        const int64_t tbase = ((int64_t)c * a.n_ant + ant) * a.kk;
        const uint2* tp = a.taps + tbase;
        float2 s = make_float2(0.f, 0.f);
        for (int q = 0; q < a.kk; ++q) {       // sum_taps conj(w) h
          const uint2 t = tp[q];
          const int cell = (int)t.x;
          const float w = __uint_as_float(t.y);
          const float2 h = X[p * PS + cell];
          s.x = fmaf(w, h.x, s.x);
          s.y = fmaf(w, h.y, s.y);
          if (CPX) {
            const float wi = a.tapim[tbase + q];
            s.x = fmaf(wi, h.y, s.x);
            s.y = fmaf(-wi, h.x, s.y);
          }
        }
        const float2 e = unpack_ci4(cur[i]);
        const float2 d = cmulc(s, e);           // s * conj(e)
        gacc[i].x += (double)d.x;
        gacc[i].y += (double)d.y;
      }
    }
  }
  flush();
}

template <int N, int P, int GPT, bool CPX>
__global__ void __launch_bounds__(FusedShape<N>::NT)
__attribute__((amdgpu_waves_per_eu(FusedShape<N>::MIN_WAVES_PER_EU)))
adjoint_kernel(AdjointArgs a) {
  adjoint_body<N, P, GPT, CPX, false>(a);
}

// The adjoint of fused_wide_image_kernel (N = 64, apertures up to 48 cells).
template <int N, int P, int GPT, bool CPX>
__global__ void __launch_bounds__(FusedShape<N>::NT)
__attribute__((amdgpu_waves_per_eu(FusedShape<N>::MIN_WAVES_PER_EU)))
adjoint_wide_kernel(AdjointArgs a) {
  static_assert(N == 64, "the wide variant is built for N = 64");
  adjoint_body<N, P, GPT, CPX, true>(a);
}

struct GradReduceArgs {
  const double2* gpartial;
  float2* grad;             // [C][P*A]
  int64_t n_time, total;
  int n_chan, PA, W;
  int sub;                  // sub-lanes per (c, p, a), as in reduce_image_kernel
  const double2* minus;     // [C][P*A] float64 term subtracted before rounding, or null
};

__global__ void __launch_bounds__(256) reduce_grad_kernel(GradReduceArgs a) {
  __shared__ double red[2 * 256];
  const int ppb = 256 / a.sub;
  const int j = threadIdx.x / ppb, lp = threadIdx.x % ppb;
  const int64_t idx = (int64_t)blockIdx.x * ppb + lp;
  const bool valid = idx < (int64_t)a.n_chan * a.PA;
  double s[2] = {0.0, 0.0};
  if (valid) {
    const int c = (int)(idx / a.PA);
    const int k = (int)(idx % a.PA);
    const int64_t w_lo = owner_of((int64_t)c * a.n_time, a.total, a.W);
    const int64_t w_hi = owner_of((int64_t)(c + 1) * a.n_time - 1, a.total, a.W);
#pragma unroll 4
    for (int64_t w = w_lo + j; w <= w_hi; w += a.sub) {
      const double2 v = a.gpartial[(w + c) * a.PA + k];
      s[0] += v.x;
      s[1] += v.y;
    }
  }
  combine_sublanes<2>(s, a.sub, ppb, j, lp, red);
  if (valid && j == 0) {
    double gr = 2.0 * s[0], gim = 2.0 * s[1];
    if (a.minus) {
      gr -= a.minus[idx].x;
      gim -= a.minus[idx].y;
    }
    a.grad[idx] = make_float2((float)gr, (float)gim);
  }
}

}  // namespace epic
