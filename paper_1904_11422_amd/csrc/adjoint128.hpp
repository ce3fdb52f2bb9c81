// Adjoint of fused_image128_kernel: gradient of a real loss with respect to
// the per-antenna complex gains at 128 x 128, given dL/dI.
//
// Work units are (channel, parity, sample), as in the imager.  A unit
// recomputes the image of its sample at the columns of parity h (gridding,
// row transforms onto those 64 frequency columns, column transforms), forms
// G = dL/dF* at its pixels (Wirtinger calculus, as adjoint_kernel), and
// applies the adjoint of that restricted transform:
//   1. column transforms with the negative exponent, from the 128 image rows
//      of each local column back to the 64 aperture rows;  barrier;
//   2. row transforms with the negative exponent, from the 64 frequency
//      columns of parity h back to the 64 aperture columns (the 64-point
//      adjoint, then the factor conj(w128^(n h)));  barrier;
//   3. degridding: dL/dg* += sum_taps conj(w) conj(e) H_h[tap].
// The full adjoint is the sum of the two parities' contributions (it is
// linear in G), so a channel's per-antenna float64 sums run over both
// parities and all samples; one slot per (workgroup, channel), reduced by
// reduce_grad_kernel.
#pragma once
#include "adjoint.hpp"
#include "fused128.hpp"

namespace epic {

// The upstream gradient at the pixels of the imager's threads, per parity:
// gtab[c][h][i][tid] = {Re Gxx, Re Gyy, Re h, Im h} at km = km128(n0, i),
// kl = kl128(h, kl_local) (fftshifted image coordinates undone).
template <int P>
__global__ void __launch_bounds__(256) grad_table128_kernel(GradTableArgs a) {
  constexpr int N = 128, NT = FusedShape<128>::NT, NPROD = (P == 2) ? 4 : 1;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)a.n_chan * 2 * 16 * NT) return;
  const int c = (int)(idx / (2 * 16 * NT));
  const int h = (int)((idx / (16 * NT)) % 2);
  const int i = (int)((idx / NT) % 16), tid = (int)(idx % NT);
  const Roles<N> r(tid);
  const int km = km128(r.n0, i), kl = kl128(h, r.kl);
  const int pix = ((km + N / 2) % N) * N + (kl + N / 2) % N;
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

template <int P, int GPT, bool CPX>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(Fused128Waves<P>::value)))
adjoint128_kernel(AdjointArgs a) {
  using SH = FusedShape<128>;
  constexpr int N = 128, S = SH::S, R = SH::R, NT = SH::NT, RS = SH::RS, PS = SH::PSTRIDE;
  constexpr int H = N / 2, NPX = 16;
  constexpr int ES = EStride<NT, GPT, P>::value;
  constexpr int XBASE = P * ES * (int)sizeof(float2);
  constexpr int TWS = 17, TW64S = 9;
  // the LDS layout of fused_image128_kernel
  __shared__ float2 lds2[P * ES + (P - 1) * PS + H * RS + R * TWS + R * TW64S + H];
  char* lds = reinterpret_cast<char*>(lds2);
  float2* E = lds2;
  float2* X = lds2 + P * ES;
  float2* TW = X + (P - 1) * PS + H * RS;
  float2* TW64 = TW + R * TWS;
  float2* ODD = TW64 + R * TW64S;

  const Roles<N> r(threadIdx.x);
  const int tid = r.tid;
  const int64_t fb = range_begin(blockIdx.x, a.total, a.W);
  const int64_t fe = range_begin(blockIdx.x + 1, a.total, a.W);
  if (fb >= fe) return;

  if (tid < R * S) TW[(tid / S) * TWS + tid % S] = a.twiddle[((tid / S) * (tid % S)) % N];
  if (tid < R * 8) TW64[(tid / 8) * TW64S + tid % 8] = a.twiddle[(2 * (tid / 8) * (tid % 8)) % N];
  if (tid < H) ODD[tid] = a.twiddle[tid];
  const float2* tw = TW + r.n0 * TWS;          // read after the first barrier
  const float2* tw64 = TW64 + r.n0 * TW64S;

  const int PA = P * a.n_ant;
  const int64_t row_bytes = (int64_t)a.n_chan * PA;
  int eidx[GPT];
  init_stage<NT, GPT, ES>(E, eidx, tid, a.n_ant, P);

  double2 gacc[GPT];
  float2 g[GPT];
  uint32_t nxt[GPT];
  int c = -1, line = -1, Lw = a.L;
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
    double2* out = a.gpartial + (int64_t)(blockIdx.x + c) * PA;
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int k = tid + i * NT;
      if (k < PA) out[k] = gacc[i];
    }
  };

  int64_t sg = fb / a.n_time;                  // segment 2 c + h of the current unit
  int64_t tt = fb - sg * a.n_time;
  load_bytes(sg, tt, nxt);
  for (int64_t left = fe - fb; left > 0; --left) {
    const int cc = (int)(sg >> 1), h = (int)(sg & 1);
    if (cc != c) {
      if (c >= 0) flush();
      c = cc;
      prog = a.prog + (int64_t)c * (a.L + 1) * NT;
      if (CPX) wim = a.wim + (int64_t)c * (a.L + 1) * NT + NT;
      line = (int)prog[tid].x;
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
    ++tt;                                      // advance, prefetch the next unit
    if (tt == a.n_time) { tt = 0; ++sg; }
    if (left > 1) load_bytes(sg, tt, nxt);

    // forward: stage and grid the aperture, row transforms onto the columns
    // of parity h (as fused_image128_kernel)
    stage_and_grid<N, P, NT, RS, ES, GPT, CPX>(lds, lds + XBASE, E, prog, wim, Lw, cur, g, eidx, tid, PA);
    const int rb = (line & 0xFFFF) * RS;
    if (line >= 0) {
      float2 v[P][8];
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int n1 = 0; n1 < 8; ++n1) v[p][n1] = X[p * PS + rb + R * n1 + r.n0];
      if (h) {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
          for (int n1 = 0; n1 < 8; ++n1) v[p][n1] = cmul(v[p][n1], ODD[R * n1 + r.n0]);
      }
      line_transform<64, +1, P>(v, tw64, r.n0, X, [rb](int p, int s) { return p * PS + rb + s; });
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) X[p * PS + rb + r.n0 + 8 * k1] = v[p][k1];
    }
    __syncthreads();

    // forward column transforms of local column kl: v[p][q R + k1] = F_p[2 n0 + q + 16 k1][2 kl + h]
    const int kl = r.kl;
    auto colslot = [kl](int p, int s) { return p * PS + (s & 63) * RS + kl + (s & 64); };
    float2 v[P][S];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int n1 = 0; n1 < S / 2; ++n1) v[p][n1] = X[p * PS + (R * n1 + r.n0) * RS + kl];
    line_transform<N, +1, P, Line<N>::S / 2>(v, tw, r.n0, X, colslot);

    // dL/dF* at the owned pixels
    const float4* gt = a.gtab + ((int64_t)c * 2 + h) * NPX * NT + tid;
#pragma unroll
    for (int i = 0; i < NPX; ++i) {
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
    // 1. adjoint column transforms: v[p][n1] = row 8 n1 + n0 of the column;
    //    the aperture rows are n1 < 8
    line_transform_rev<N, -1, P>(v, tw, r.n0, X, colslot);
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int n1 = 0; n1 < S / 2; ++n1) X[p * PS + (R * n1 + r.n0) * RS + kl] = v[p][n1];
    __syncthreads();

    // 2. adjoint row transforms of row `line`: its 64 local values are the
    //    frequencies 2 m + h, m = n0 + 8 k1 in the forward's output layout;
    //    the 64-point adjoint gives the aperture columns n = 8 n1 + n0, then
    //    the odd parity's factor conj(w128^n)
    if (line >= 0) {
      float2 u[P][8];
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) u[p][k1] = X[p * PS + rb + r.n0 + 8 * k1];
      line_transform_rev<64, -1, P>(u, tw64, r.n0, X, [rb](int p, int s) { return p * PS + rb + s; });
      if (h) {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
          for (int n1 = 0; n1 < 8; ++n1) u[p][n1] = cmulc(u[p][n1], ODD[R * n1 + r.n0]);
      }
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int n1 = 0; n1 < 8; ++n1) X[p * PS + rb + R * n1 + r.n0] = u[p][n1];
    }
    __syncthreads();

    // 3. degrid: dL/de'* at each antenna, times conj(e)
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
          const float2 hv = X[p * PS + cell];
          s.x = fmaf(w, hv.x, s.x);
          s.y = fmaf(w, hv.y, s.y);
          if (CPX) {
            const float wi = a.tapim[tbase + q];
            s.x = fmaf(wi, hv.y, s.x);
            s.y = fmaf(-wi, hv.x, s.y);
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

}  // namespace epic
