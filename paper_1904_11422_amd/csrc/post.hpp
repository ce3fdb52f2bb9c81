// Post-processing of accumulated images (paper Sec. 3.2: the imprint of the
// gridding kernels is known in advance and can be removed after the fact;
// Sec. 4.3: pseudo-Stokes images are linear combinations of the
// linear-polarisation products).
//
// Kernel taper: every product is built from b_a(k) conj(b_b(k)), b_a the
// transform of antenna a's kernel taps; when all antennas share one kernel up
// to a whole-cell shift, each product is a point-kernel image times
// |b(k)|^2.  The taper is the antennas' mean kernel power pattern
//   T_c(k) = (1/A) sum_a |b_a(k)|^2 = (1/A) Re sum_d S_c(d) exp(+2 pi i d.k / N),
//   S_c(d) = sum_a sum_u w_a(u) conj(w_a(u - d))          ((2K-1)^2 offsets),
// built once per geometry (taper_coeff_kernel, taper_image_kernel).
// postprocess_kernel forms I = XX + YY, Q = XX - YY, U = XY + YX,
// V = -i (XY - YX) (one polarisation: XX) and, on request, divides by T
// where T is at least a floor times the channel's maximum (zero elsewhere).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace epic {

constexpr int TAPER_MAX_D2 = 29 * 29;          // (2K-1)^2 for K <= 15

struct TaperCoeffArgs {
  const float* w;           // [C][A][K*K] real parts
  const float* wi;          // [C][A][K*K] imaginary parts, or null (real kernels)
  double2* coeff;           // [C][(2K-1)^2]
  int n_chan, n_ant, K;
};

constexpr int TAPER_MAX_KK = 15 * 15;
constexpr int TAPER_ANT_BATCH = 8;             // antennas staged through LDS at a time

// One workgroup per (channel, block of 256 offsets d), one thread per offset;
// the antennas' taps are staged through LDS a batch at a time and every
// thread adds its offset's overlap sum antenna by antenna, in antenna order.
__global__ void __launch_bounds__(256) taper_coeff_kernel(TaperCoeffArgs a) {
  __shared__ double2 wt[TAPER_ANT_BATCH][TAPER_MAX_KK];
  const int K = a.K, D = 2 * K - 1, D2 = D * D, KK = K * K;
  const int blocks = (D2 + 255) / 256;
  const int c = blockIdx.x / blocks, d = (blockIdx.x % blocks) * 256 + threadIdx.x;
  const bool valid = d < D2;
  const int dj = valid ? d / D - (K - 1) : 0, di = valid ? d % D - (K - 1) : 0;
  const int uj0 = dj > 0 ? dj : 0, uj1 = dj < 0 ? K + dj : K;
  const int ui0 = di > 0 ? di : 0, ui1 = di < 0 ? K + di : K;
  double sr = 0.0, si = 0.0;
  for (int a0 = 0; a0 < a.n_ant; a0 += TAPER_ANT_BATCH) {
    const int nb = a.n_ant - a0 < TAPER_ANT_BATCH ? a.n_ant - a0 : TAPER_ANT_BATCH;
    __syncthreads();
    for (int i = threadIdx.x; i < nb * KK; i += 256) {
      const int64_t o = ((int64_t)c * a.n_ant + a0) * KK + i;
      wt[i / KK][i % KK] = make_double2(a.w[o], a.wi ? a.wi[o] : 0.0);
    }
    __syncthreads();
    if (!valid) continue;
    for (int b = 0; b < nb; ++b)
      for (int uj = uj0; uj < uj1; ++uj)
        for (int ui = ui0; ui < ui1; ++ui) {
          // w(u) conj(w(u - d))
          const double2 x = wt[b][uj * K + ui], y = wt[b][(uj - dj) * K + (ui - di)];
          sr = fma(x.x, y.x, fma(x.y, y.y, sr));
          si = fma(x.y, y.x, fma(-x.x, y.y, si));
        }
  }
  if (valid) a.coeff[(int64_t)c * D2 + d] = make_double2(sr, si);
}

struct TaperImageArgs {
  const double2* coeff;     // [C][(2K-1)^2]
  double* taper;            // [C][N][N], fftshifted
  int n_chan, n_ant, N, K;
};

// Grid: C * ceil(N^2 / 256) workgroups, channel-major; one thread per pixel.
__global__ void __launch_bounds__(256) taper_image_kernel(TaperImageArgs a) {
  __shared__ double2 st[TAPER_MAX_D2];
  __shared__ double2 ex[128];                   // exp(+2 pi i m / N)
  const int N = a.N, K = a.K, D = 2 * K - 1, D2 = D * D, tiles = (N * N + 255) / 256;
  const int c = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  for (int i = threadIdx.x; i < D2; i += 256) st[i] = a.coeff[(int64_t)c * D2 + i];
  for (int m = threadIdx.x; m < N; m += 256) {
    double s, co;
    sincospi(2.0 * m / N, &s, &co);
    ex[m] = make_double2(co, s);
  }
  __syncthreads();
  const int pix = tile * 256 + threadIdx.x;
  if (pix >= N * N) return;
  const int km = (pix / N + N / 2) & (N - 1), kl = (pix % N + N / 2) & (N - 1);
  double t = 0.0;
  for (int dj = -(K - 1), d = 0; dj <= K - 1; ++dj)
    for (int di = -(K - 1); di <= K - 1; ++di, ++d) {
      const double2 e = ex[(di * kl + dj * km) & (N - 1)];
      t = fma(st[d].x, e.x, fma(-st[d].y, e.y, t));      // Re(S e)
    }
  a.taper[(int64_t)c * N * N + pix] = t / a.n_ant;
}

struct PostArgs {
  const double2* image;     // [C][NPROD][N][N]
  const double* taper;      // [C][N][N] or null (no correction)
  const double* tmax;       // [C] maxima of the taper
  double* out;              // [C][NOUT][N][N]: I, Q, U, V (P = 2) or XX (P = 1)
  double floor;             // keep pixels with T >= floor * tmax[c]
  int64_t n;                // C * N * N
  int npix;
};

template <int P>
__global__ void __launch_bounds__(256) postprocess_kernel(PostArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= a.n) return;
  const int64_t c = idx / a.npix;
  const int pix = (int)(idx - c * a.npix);
  constexpr int NPROD = P == 2 ? 4 : 1;
  const double2* im = a.image + c * NPROD * a.npix + pix;
  double v[NPROD];
  if (P == 2) {
    const double xx = im[0].x, yy = im[3 * a.npix].x;
    const double2 xy = im[a.npix], yx = im[2 * a.npix];
    v[0] = xx + yy;
    v[1 % NPROD] = xx - yy;
    v[2 % NPROD] = xy.x + yx.x;
    v[3 % NPROD] = xy.y - yx.y;                          // -i (XY - YX), real part
  } else {
    v[0] = im[0].x;
  }
  double scale = 1.0;
  if (a.taper) {
    const double t = a.taper[idx];
    scale = t >= a.floor * a.tmax[c] ? 1.0 / t : 0.0;
  }
  double* o = a.out + c * NPROD * a.npix + pix;
#pragma unroll
  for (int q = 0; q < NPROD; ++q) o[(int64_t)q * a.npix] = v[q] * scale;
}

}  // namespace epic
