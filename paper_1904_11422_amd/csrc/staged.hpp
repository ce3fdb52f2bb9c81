// Plain staged path: the same hot path as one kernel per stage with float32
// intermediates in HBM, the shape of a pipeline built from generic blocks.
// It is the comparator for the fused kernel, and it also runs the 128 x 128
// grids whose two polarisations do not fit one workgroup's LDS.
//
//   unpack_gain:  efield [Tb][C][P][A] bytes -> E' float2 [Tb][C][P][A]
//   grid_gather:  E' -> aperture float2 [Tb][C][P][N][N]   (per-cell CSR gather)
//   fft2d:        aperture -> image, in place, one workgroup per (t, c, p)
//   xpol_accum:   image -> float64 sums [C][NACC][N*N] (time order, per pixel)
#pragma once
#include "dft.hpp"

namespace epic {

struct StagedUnpackArgs {
  const uint8_t* efield;    // full [T][C][P][A]
  const float2* gains;      // [C][P][A]
  float2* e;                // [Tb][C][P][A]
  int64_t t0;               // first sample of the batch
  int64_t count;            // Tb * C * P * A
  int64_t per_t;            // C * P * A
  int PA;
};

__global__ void __launch_bounds__(256) staged_unpack_kernel(StagedUnpackArgs a) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.count;
       i += (int64_t)gridDim.x * 256) {
    const int64_t tl = i / a.per_t;
    const int64_t r = i - tl * a.per_t;              // c*PA + k
    const int b = a.efield[(a.t0 + tl) * a.per_t + r];
    const float re = (float)((b >> 4) - ((b & 0x80) ? 16 : 0));
    const float im = (float)((b & 0xF) - ((b & 0x8) ? 16 : 0));
    const float2 g = a.gains[r];
    a.e[i] = make_float2(fmaf(g.x, re, -g.y * im), fmaf(g.x, im, g.y * re));
  }
}

struct StagedGridArgs {
  const float2* e;          // [Tb][C][P][A]
  const int* off;           // [C][N*N + 1]
  const uint2* ent;         // [C][nnz] {ant, w bits}
  float2* grid;             // [Tb][C][P][N*N]
  int64_t count;            // Tb * C * P * N*N
  int n_chan, n_pol, n_ant, nnz, npix;
  const float* ent_im;      // [C][nnz] imaginary weights (complex kernels), or null
};

__global__ void __launch_bounds__(256) staged_grid_kernel(StagedGridArgs a) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.count;
       i += (int64_t)gridDim.x * 256) {
    const int cell = (int)(i % a.npix);
    const int64_t img = i / a.npix;                  // (t*C + c)*P + p
    const int p = (int)(img % a.n_pol);
    const int64_t tc = img / a.n_pol;
    const int c = (int)(tc % a.n_chan);
    const int* off = a.off + (int64_t)c * (a.npix + 1);
    const uint2* ent = a.ent + (int64_t)c * a.nnz;
    const float* eim = a.ent_im ? a.ent_im + (int64_t)c * a.nnz : nullptr;
    const float2* e = a.e + (tc * a.n_pol + p) * a.n_ant;
    float2 s = make_float2(0.f, 0.f);
    for (int k = off[cell]; k < off[cell + 1]; ++k) {
      const uint2 en = ent[k];
      const float w = __uint_as_float(en.y);
      const float2 v = e[en.x];
      s.x = fmaf(w, v.x, s.x);
      s.y = fmaf(w, v.y, s.y);
      if (eim) {                                  // complex kernel: + i wi v
        const float wi = eim[k];
        s.x = fmaf(-wi, v.y, s.x);
        s.y = fmaf(wi, v.x, s.y);
      }
    }
    a.grid[i] = s;
  }
}

template <int N> struct StagedFftShape {
  static constexpr int S = Line<N>::S, R = Line<N>::R, D = Line<N>::D;
  static constexpr int NT = N * R;
  static constexpr int CPW = 64 / R;
  static constexpr int RS = N + 4;
};

// One workgroup transforms one N x N image (natural order in and out).
template <int N>
__global__ void __launch_bounds__(StagedFftShape<N>::NT)
staged_fft_kernel(float2* grid, const float2* twiddle) {
  using SH = StagedFftShape<N>;
  constexpr int S = SH::S, R = SH::R, D = SH::D, NT = SH::NT, CPW = SH::CPW, RS = SH::RS;
  __shared__ float2 X[N * RS];
  float2* img = grid + (int64_t)blockIdx.x * N * N;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int n0 = lane / CPW, sub = lane % CPW;
  const int line = wave * CPW + sub;               // row in pass 1, column in pass 2
  float2 tw[S];
#pragma unroll
  for (int k0 = 0; k0 < S; ++k0) tw[k0] = twiddle[(n0 * k0) % N];

  for (int i = tid; i < N * N; i += NT) X[(i / N) * RS + (i % N)] = img[i];
  __syncthreads();
  {
    float2* row = X + line * RS;
    float2 v[1][S];
#pragma unroll
    for (int n1 = 0; n1 < S; ++n1) v[0][n1] = row[R * n1 + n0];
    line_transform<N, +1, 1>(v, tw, n0, row, [](int, int s) { return s; });
#pragma unroll
    for (int q = 0; q < D; ++q)
#pragma unroll
      for (int k1 = 0; k1 < R; ++k1) row[n0 * D + q + S * k1] = v[0][q * R + k1];
  }
  __syncthreads();
  {
    const int kl = line;
    float2 v[1][S];
#pragma unroll
    for (int n1 = 0; n1 < S; ++n1) v[0][n1] = X[(R * n1 + n0) * RS + kl];
    line_transform<N, +1, 1>(v, tw, n0, X, [kl](int, int s) { return s * RS + kl; });
#pragma unroll
    for (int q = 0; q < D; ++q)
#pragma unroll
      for (int k1 = 0; k1 < R; ++k1) img[(n0 * D + q + S * k1) * N + kl] = v[0][q * R + k1];
  }
}

struct StagedAccumArgs {
  const float2* img;        // [Tb][C][P][N*N]
  double* acc;              // [C][NACC][N*N]
  int64_t count;            // C * N*N
  int n_chan, npix, tb, first;
};

template <int P>
__global__ void __launch_bounds__(256) staged_accum_kernel(StagedAccumArgs a) {
  constexpr int NACC = (P == 2) ? 4 : 1;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.count) return;
  const int c = (int)(i / a.npix);
  const int pix = (int)(i % a.npix);
  double s[NACC];
  double* out = a.acc + (int64_t)c * NACC * a.npix + pix;
#pragma unroll
  for (int u = 0; u < NACC; ++u) s[u] = a.first ? 0.0 : out[(int64_t)u * a.npix];
  for (int t = 0; t < a.tb; ++t) {
    const float2* base = a.img + ((int64_t)t * a.n_chan + c) * P * a.npix + pix;
    const float2 fx = base[0];
    s[0] += (double)fmaf(fx.x, fx.x, fx.y * fx.y);
    if (P == 2) {
      const float2 fy = base[a.npix];
      s[1 % NACC] += (double)fmaf(fy.x, fy.x, fy.y * fy.y);
      s[2 % NACC] += (double)fmaf(fx.x, fy.x, fx.y * fy.y);
      s[3 % NACC] += (double)fmaf(fx.y, fy.x, -fx.x * fy.y);
    }
  }
#pragma unroll
  for (int u = 0; u < NACC; ++u) out[(int64_t)u * a.npix] = s[u];
}

}  // namespace epic
