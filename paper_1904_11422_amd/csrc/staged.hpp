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

// ---- gain gradient on the staged path (the adjoint of the stages above) ----
//
// Per batch of samples: the forward stages recompute F; staged_gform_kernel
// replaces F by conj(dL/dF*) (Wirtinger calculus, as adjoint_kernel); the same
// forward transform then gives conj(H) with H = sum_k G exp(-2 pi i ...), the
// adjoint transform of G; staged_degrid_kernel gathers H at every antenna's
// taps and adds conj(w) H conj(e) to float64 sums per (channel, polarisation,
// antenna), in time order.

// The upstream gradient in natural pixel order: gtab[c][pix] =
// {Re Gxx, Re Gyy, Re h, Im h}, h = (Gxy + conj(Gyx)) / 2, from the
// fftshifted complex128 image gradient.
struct StagedGradTableArgs {
  const double2* grad_image;  // [C][NPROD][N][N] (fftshifted)
  float4* gtab;               // [C][N*N]
  int n_chan, N;
};

template <int P>
__global__ void __launch_bounds__(256) staged_grad_table_kernel(StagedGradTableArgs a) {
  constexpr int NPROD = (P == 2) ? 4 : 1;
  const int N = a.N, npix = N * N;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)a.n_chan * npix) return;
  const int c = (int)(idx / npix), pix = (int)(idx % npix);
  const int km = pix / N, kl = pix % N;
  const int sp = ((km + N / 2) % N) * N + (kl + N / 2) % N;
  const double2* gi = a.grad_image + (int64_t)c * NPROD * npix;
  float4 t;
  t.x = (float)gi[sp].x;
  if (P == 2) {
    const double2 xy = gi[npix + sp], yx = gi[2 * npix + sp];
    t.y = (float)gi[3 * npix + sp].x;
    t.z = (float)(0.5 * (xy.x + yx.x));
    t.w = (float)(0.5 * (xy.y - yx.y));
  } else {
    t.y = t.z = t.w = 0.f;
  }
  a.gtab[idx] = t;
}

struct StagedGformArgs {
  float2* img;              // [Tb][C][P][N*N]: F in, conj(dL/dF*) out
  const float4* gtab;       // [C][N*N]
  int64_t count;            // Tb * C * N*N
  int n_chan, npix;
};

template <int P>
__global__ void __launch_bounds__(256) staged_gform_kernel(StagedGformArgs a) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.count;
       i += (int64_t)gridDim.x * 256) {
    const int pix = (int)(i % a.npix);
    const int64_t tc = i / a.npix;                   // t*C + c
    const int c = (int)(tc % a.n_chan);
    const float4 t = a.gtab[(int64_t)c * a.npix + pix];
    float2* f = a.img + tc * P * a.npix + pix;
    const float2 fx = f[0];
    if (P == 2) {
      const float2 fy = f[a.npix];
      // G_X = Re Gxx F_X + h F_Y,  G_Y = Re Gyy F_Y + conj(h) F_X
      const float2 gx = make_float2(fmaf(t.x, fx.x, t.z * fy.x - t.w * fy.y),
                                    fmaf(t.x, fx.y, t.z * fy.y + t.w * fy.x));
      const float2 gy = make_float2(fmaf(t.y, fy.x, t.z * fx.x + t.w * fx.y),
                                    fmaf(t.y, fy.y, t.z * fx.y - t.w * fx.x));
      f[0] = make_float2(gx.x, -gx.y);
      f[a.npix] = make_float2(gy.x, -gy.y);
    } else {
      f[0] = make_float2(t.x * fx.x, -t.x * fx.y);
    }
  }
}

struct StagedDegridArgs {
  const float2* img;        // [Tb][C][P][N*N]: conj(H)
  const uint8_t* efield;    // full [T][C][P][A]
  const uint2* taps;        // [C][A][KK] {natural cell j*N + i, w bits}
  const float* tapim;       // [C][A][KK] imaginary tap weights (complex kernels), or null
  double2* gsum;            // [C][P*A]: float64 sums of dL/dg* over the samples so far
  int64_t t0;               // first sample of the batch
  int tb, n_chan, n_ant, kk, npix, PA, first;
};

// One thread per (channel, polarisation, antenna); the batch's samples in order.
__global__ void __launch_bounds__(256) staged_degrid_kernel(StagedDegridArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)a.n_chan * a.PA) return;
  const int c = (int)(idx / a.PA), k = (int)(idx % a.PA);
  const int p = k / a.n_ant, ant = k - p * a.n_ant;
  const int64_t tbase = ((int64_t)c * a.n_ant + ant) * a.kk;
  const int P = a.PA / a.n_ant;
  double2 acc = a.first ? make_double2(0.0, 0.0) : a.gsum[idx];
  for (int t = 0; t < a.tb; ++t) {
    const float2* h = a.img + (((int64_t)t * a.n_chan + c) * P + p) * a.npix;
    float2 s = make_float2(0.f, 0.f);
    for (int q = 0; q < a.kk; ++q) {                // sum_taps conj(w) H, H = conj(stored)
      const uint2 tq = a.taps[tbase + q];
      const float w = __uint_as_float(tq.y);
      const float2 y = h[tq.x];
      s.x = fmaf(w, y.x, s.x);
      s.y = fmaf(-w, y.y, s.y);
      if (a.tapim) {
        const float wi = a.tapim[tbase + q];
        s.x = fmaf(-wi, y.y, s.x);                  // conj(w) H with w = wr + i wi, H = y*
        s.y = fmaf(-wi, y.x, s.y);
      }
    }
    const int b = a.efield[((a.t0 + t) * a.n_chan + c) * a.PA + k];
    const float er = (float)((b >> 4) - ((b & 0x80) ? 16 : 0));
    const float ei = (float)((b & 0xF) - ((b & 0x8) ? 16 : 0));
    // s conj(e)
    acc.x += (double)fmaf(s.x, er, s.y * ei);
    acc.y += (double)fmaf(s.y, er, -s.x * ei);
  }
  a.gsum[idx] = acc;
}

}  // namespace epic
