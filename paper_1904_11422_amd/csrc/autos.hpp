// Antenna autocorrelations and their removal from accumulated images
// (paper Sec. 3.2 and Fig. 2: the zero-spacing power of every antenna is
// summed beside the imaging and taken out after squaring and accumulation).
//
// The image of one sample is |sum_a e'_a b_a(k)|^2 (and the cross products of
// the polarisations), b_a(k) the transform of antenna a's kernel footprint.
// Its a = b terms, summed over the samples, are
//   autos_PQ(k) = sum_a V_PQ[a] |b_a(k)|^2,  V_PQ[a] = g_P conj(g_Q) sum_t e_P conj(e_Q),
// and |b_a(k)|^2 = sum_d R_a(d) exp(+2 pi i d.k / N), where
// R_a(d) = sum_u w_a(u) w_a(u - d) is the autocorrelation of the antenna's
// K x K tap weights over tap offsets d in [-(K-1), K-1]^2 (where the antenna
// sits only moves the footprint, which the magnitude does not see).  Hence,
// per channel and product,
//   S_PQ(d)     = sum_a V_PQ[a] R_a(d)                 ((2K-1)^2 values)
//   autos_PQ(k) = sum_d S_PQ(d) cos(2 pi d.k / N)      (S_PQ(d) = S_PQ(-d))
// and YX = conj(XY).  Three kernels:
//   auto_sum_kernel    streams the 4+4-bit samples once (HBM bound) and forms
//                      the integer sums sum_t e_P conj(e_Q) of every antenna
//                      exactly, four samples per signed 4-bit dot product;
//   auto_table_kernel  one workgroup per channel: S_PQ(d) in float64;
//   auto_remove_kernel subtracts autos_PQ(k) from the image in float64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace epic {

constexpr int AUTO_LANES = 64;      // antenna groups per workgroup (one per lane of a wave)
constexpr int AUTO_TL = 8;          // time lanes (waves) per workgroup
constexpr int AUTO_ROWS = 8;        // samples each lane loads per iteration
constexpr int AUTO_MAX_SEG = 16;    // time segments (partial sums) at most
constexpr int AUTO_MAX_K = 7;
constexpr int AUTO_MAX_D2 = (2 * AUTO_MAX_K - 1) * (2 * AUTO_MAX_K - 1);
constexpr int64_t AUTO_SEG_MAX_SAMPLES = (1 << 24) - 1;  // int32 sums stay exact

template <int P> struct AutoShape {
  // integer sums per antenna: {sum |e_X|^2, sum |e_Y|^2, Re sum e_X conj(e_Y),
  // Im sum e_X conj(e_Y)} for two polarisations, {sum |e|^2} for one
  static constexpr int NQ = P == 2 ? 4 : 1;
};

struct AutoSumArgs {
  const uint8_t* efield;    // [T][C][P][A]
  int32_t* part;            // [nseg][C][A][NQ]
  int64_t n_time;
  int n_chan, n_ant, nseg;
};

// Byte k of the words w[0..3] gathered into word k: the four samples of one
// antenna side by side (a 4 x 4 byte transpose).
__device__ __forceinline__ void transpose4(const uint32_t* w, uint32_t* u) {
  const uint32_t lo01 = __builtin_amdgcn_perm(w[1], w[0], 0x05010400u);
  const uint32_t hi01 = __builtin_amdgcn_perm(w[1], w[0], 0x07030602u);
  const uint32_t lo23 = __builtin_amdgcn_perm(w[3], w[2], 0x05010400u);
  const uint32_t hi23 = __builtin_amdgcn_perm(w[3], w[2], 0x07030602u);
  u[0] = __builtin_amdgcn_perm(lo23, lo01, 0x05040100u);
  u[1] = __builtin_amdgcn_perm(lo23, lo01, 0x07060302u);
  u[2] = __builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
  u[3] = __builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
}

// A word of four samples of one antenna holds eight signed nibbles
// (imaginary low, real high), so one signed 4-bit dot product of two such
// words is sum_t (xi yi + xr yr) = Re sum_t x conj(y).  The imaginary part
// sum_t (xi yr - xr yi) takes the low nibbles of one word against the high
// nibbles of the other.
template <int P>
__device__ __forceinline__ void auto_accumulate(uint32_t ux, uint32_t uy, int* acc) {
  constexpr uint32_t LO = 0x0F0F0F0Fu;
  acc[0] = __builtin_amdgcn_sdot8((int)ux, (int)ux, acc[0], false);
  if constexpr (P == 2) {
    acc[1] = __builtin_amdgcn_sdot8((int)uy, (int)uy, acc[1], false);
    acc[2] = __builtin_amdgcn_sdot8((int)ux, (int)uy, acc[2], false);
    acc[3] = __builtin_amdgcn_sdot8((int)(ux & LO), (int)((uy >> 4) & LO), acc[3], false);
    acc[4] = __builtin_amdgcn_sdot8((int)((ux >> 4) & LO), (int)(uy & LO), acc[4], false);
  }
}

// Grid: (ceil(C * A / VEC / AUTO_LANES), nseg).  Lane l of every wave takes
// VEC consecutive antennas of one channel (group blockIdx.x * 64 + l of the
// flattened (channel, antenna) order); the AUTO_TL waves of a workgroup take
// interleaved blocks of AUTO_ROWS samples of the workgroup's time segment.
// VEC = 4 loads one 32-bit word per sample and polarisation (A % 4 == 0 and a
// 4-byte aligned E-field), VEC = 1 one byte.  Every sum is exact: a segment
// holds at most 2^24 - 1 samples and |e|^2 <= 128.
template <int P, int VEC>
__global__ void __launch_bounds__(AUTO_LANES * AUTO_TL) auto_sum_kernel(AutoSumArgs a) {
  constexpr int NQ = AutoShape<P>::NQ;
  constexpr int NACC = P == 2 ? 5 : 1;
  constexpr int NT = AUTO_LANES * AUTO_TL;
  __shared__ int red[NQ * VEC][AUTO_LANES + 1];
  const int lane = threadIdx.x % AUTO_LANES, tl = threadIdx.x / AUTO_LANES;
  const int gpc = a.n_ant / VEC;
  const int64_t ngroups = (int64_t)a.n_chan * gpc;
  const int64_t gbase = (int64_t)blockIdx.x * AUTO_LANES;
  const int64_t g = gbase + lane;
  const bool valid = g < ngroups;
  for (int i = threadIdx.x; i < NQ * VEC * (AUTO_LANES + 1); i += NT) (&red[0][0])[i] = 0;

  int acc[VEC][NACC];
#pragma unroll
  for (int k = 0; k < VEC; ++k)
#pragma unroll
    for (int q = 0; q < NACC; ++q) acc[k][q] = 0;

  if (valid) {
    const int c = (int)(g / gpc), a0 = (int)(g % gpc) * VEC;
    const int64_t row = (int64_t)a.n_chan * P * a.n_ant;
    const uint8_t* px = a.efield + (int64_t)c * P * a.n_ant + a0;
    const int64_t t_lo = (int64_t)blockIdx.y * a.n_time / a.nseg;
    const int64_t t_hi = (int64_t)(blockIdx.y + 1) * a.n_time / a.nseg;
    for (int64_t t0 = t_lo + (int64_t)AUTO_ROWS * tl; t0 < t_hi; t0 += (int64_t)AUTO_ROWS * AUTO_TL) {
      uint32_t wx[AUTO_ROWS], wy[AUTO_ROWS];
#pragma unroll
      for (int r = 0; r < AUTO_ROWS; ++r) {
        const int64_t t = t0 + r;
        const uint8_t* p = px + t * row;
        if (VEC == 4) {
          wx[r] = t < t_hi ? *reinterpret_cast<const uint32_t*>(p) : 0u;
          wy[r] = (P == 2 && t < t_hi) ? *reinterpret_cast<const uint32_t*>(p + a.n_ant) : 0u;
        } else {
          wx[r] = t < t_hi ? (uint32_t)p[0] : 0u;
          wy[r] = (P == 2 && t < t_hi) ? (uint32_t)p[a.n_ant] : 0u;
        }
      }
#pragma unroll
      for (int h = 0; h < AUTO_ROWS / 4; ++h) {
        uint32_t ux[4], uy[4];
        if (VEC == 4) {
          transpose4(wx + 4 * h, ux);
          if (P == 2) transpose4(wy + 4 * h, uy);
          else uy[0] = uy[1] = uy[2] = uy[3] = 0u;
        } else {
          ux[0] = wx[4 * h] | wx[4 * h + 1] << 8 | wx[4 * h + 2] << 16 | wx[4 * h + 3] << 24;
          uy[0] = wy[4 * h] | wy[4 * h + 1] << 8 | wy[4 * h + 2] << 16 | wy[4 * h + 3] << 24;
        }
#pragma unroll
        for (int k = 0; k < VEC; ++k) auto_accumulate<P>(ux[k], uy[k], acc[k]);
      }
    }
  }
  __syncthreads();
  if (valid) {
    // integer adds in LDS: exact in any order
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      atomicAdd(&red[0 * VEC + k][lane], acc[k][0]);
      if constexpr (P == 2) {
        atomicAdd(&red[1 * VEC + k][lane], acc[k][1]);
        atomicAdd(&red[2 * VEC + k][lane], acc[k][2]);
        atomicAdd(&red[3 * VEC + k][lane], acc[k][3] - acc[k][4]);
      }
    }
  }
  __syncthreads();
  const int64_t left = ngroups - gbase;
  const int n_out = (int)(left < AUTO_LANES ? left : AUTO_LANES) * VEC * NQ;
  int32_t* out = a.part + ((int64_t)blockIdx.y * ngroups + gbase) * VEC * NQ;
  for (int i = threadIdx.x; i < n_out; i += NT) {
    const int gl = i / (VEC * NQ), r = i % (VEC * NQ);
    out[i] = red[(r % NQ) * VEC + r / NQ][gl];
  }
}

struct AutoTableArgs {
  const int32_t* part;      // [nseg][C][A][NQ]
  const float2* gains;      // [C][P][A]
  const float* w;           // [C][A][K*K] tap weights, tap order dj outer, di inner
  double* table;            // [C][(2K-1)^2][NQ]: {XX, YY, Re XY, Im XY} or {XX}
  int n_chan, n_ant, nseg, K;
};

// Sum of NV values over a 256-thread workgroup in a fixed order (halving
// within each wave, then the four waves in order); the result is valid in
// thread 0.  red: NV * 4 doubles of LDS.
template <int NV>
__device__ __forceinline__ void block_sum256(double (&v)[NV], double (*red)[4]) {
#pragma unroll
  for (int q = 0; q < NV; ++q)
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_down(v[q], off, 64);
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) red[q][w] = v[q];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = ((red[q][0] + red[q][1]) + red[q][2]) + red[q][3];
}

// Workgroups (c, d) for channel c and tap offset d, laid out so that the
// (2K-1)^2 workgroups of a channel share blockIdx.x % 8 (one XCD, one L2):
// grid 8 * ceil(C / 8) * (2K-1)^2.
__device__ __forceinline__ void xcd_channel_offset(int D2, int& c, int& d) {
  const int r = blockIdx.x / 8;
  c = (r / D2) * 8 + blockIdx.x % 8;
  d = r % D2;
}

// R_a(d) = sum_u w(u) w(u - d) over the taps u with u and u - d in the K x K
// footprint, in float64 from the float32 weights w[K*K].
__device__ __forceinline__ double tap_autocorrelation(const float* w, int K, int dj, int di) {
  const int uj0 = dj > 0 ? dj : 0, uj1 = dj < 0 ? K + dj : K;
  const int ui0 = di > 0 ? di : 0, ui1 = di < 0 ? K + di : K;
  double r = 0.0;
  for (int uj = uj0; uj < uj1; ++uj)
    for (int ui = ui0; ui < ui1; ++ui)
      r = fma((double)w[uj * K + ui], (double)w[(uj - dj) * K + (ui - di)], r);
  return r;
}

// S_PQ(d) for one (channel, tap offset) per workgroup; one antenna per thread
// at a time.  d = (dj, di): dj = d / (2K-1) - (K-1), di = d % (2K-1) - (K-1).
template <int P>
__global__ void __launch_bounds__(256) auto_table_kernel(AutoTableArgs a) {
  constexpr int NQ = AutoShape<P>::NQ;
  __shared__ double red[NQ][4];
  const int K = a.K, D = 2 * K - 1, D2 = D * D, KK = K * K;
  int c, d;
  xcd_channel_offset(D2, c, d);
  if (c >= a.n_chan) return;
  const int dj = d / D - (K - 1), di = d % D - (K - 1);
  const int64_t CA = (int64_t)a.n_chan * a.n_ant;
  double s[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) s[q] = 0.0;
  for (int ant = threadIdx.x; ant < a.n_ant; ant += 256) {
    const int64_t ca = (int64_t)c * a.n_ant + ant;
    int64_t m[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) m[q] = 0;
    for (int seg = 0; seg < a.nseg; ++seg) {
      const int32_t* p = a.part + ((int64_t)seg * CA + ca) * NQ;
#pragma unroll
      for (int q = 0; q < NQ; ++q) m[q] += p[q];
    }
    const double r = tap_autocorrelation(a.w + ca * KK, K, dj, di);
    const float2 gx = a.gains[(int64_t)c * P * a.n_ant + ant];
    const double gxr = gx.x, gxi = gx.y;
    s[0] = fma((gxr * gxr + gxi * gxi) * (double)m[0], r, s[0]);
    if constexpr (P == 2) {
      const float2 gy = a.gains[((int64_t)c * P + 1) * a.n_ant + ant];
      const double gyr = gy.x, gyi = gy.y;
      s[1] = fma((gyr * gyr + gyi * gyi) * (double)m[1], r, s[1]);
      // g_X conj(g_Y) (m2 + i m3)
      const double hr = gxr * gyr + gxi * gyi, hi = gxi * gyr - gxr * gyi;
      s[2] = fma(hr * (double)m[2] - hi * (double)m[3], r, s[2]);
      s[3] = fma(hr * (double)m[3] + hi * (double)m[2], r, s[3]);
    }
  }
  block_sum256<NQ>(s, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) a.table[((int64_t)c * D2 + d) * NQ + q] = s[q];
}

struct AutoRemoveArgs {
  const double* table;      // [C][(2K-1)^2][NQ]
  double2* image;           // [C][NPROD][N][N], fftshifted
  int n_chan, N, K;
};

// Grid: C * ceil(N^2 / 256) workgroups, channel-major; one thread per pixel.
template <int P>
__global__ void __launch_bounds__(256) auto_remove_kernel(AutoRemoveArgs a) {
  constexpr int NQ = AutoShape<P>::NQ;
  __shared__ double st[AUTO_MAX_D2][NQ];
  __shared__ double cs[128];
  const int N = a.N, K = a.K, D = 2 * K - 1, tiles = (N * N + 255) / 256;
  const int c = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  for (int i = threadIdx.x; i < D * D * NQ; i += 256)
    (&st[0][0])[i] = a.table[(int64_t)c * D * D * NQ + i];
  for (int m = threadIdx.x; m < N; m += 256) cs[m] = cospi(2.0 * m / N);
  __syncthreads();
  const int pix = tile * 256 + threadIdx.x;
  if (pix >= N * N) return;
  // pixel (q_m, q_l) of the shifted image holds k = (q - N/2) mod N
  const int km = (pix / N + N / 2) & (N - 1), kl = (pix % N + N / 2) & (N - 1);
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  for (int dj = -(K - 1), d = 0; dj <= K - 1; ++dj)
    for (int di = -(K - 1); di <= K - 1; ++di, ++d) {
      const double e = cs[(di * kl + dj * km) & (N - 1)];
#pragma unroll
      for (int q = 0; q < NQ; ++q) v[q] = fma(st[d][q], e, v[q]);
    }
  constexpr int NPROD = P == 2 ? 4 : 1;
  double2* img = a.image + (int64_t)c * NPROD * N * N + pix;
  img[0].x -= v[0];
  if (P == 2) {
    img[3 * N * N].x -= v[1];
    double2 xy = img[N * N], yx = img[2 * N * N];
    xy.x -= v[2]; xy.y -= v[3];
    yx.x -= v[2]; yx.y += v[3];
    img[N * N] = xy;
    img[2 * N * N] = yx;
  }
}

// ---------------------------------------------------------------------------
// Gain gradient of the removed term.  For a real loss with upstream gradient
// Gamma (dL/dRe + i dL/dIm of the image), the removed term contributes, with
// U_PQ[a] = sum_k Gamma_PQ(k) |b_a(k)|^2 = sum_d R_a(d) Ghat_PQ(d) and
// Ghat_PQ(d) = sum_k Gamma_PQ(k) cos(2 pi d.k / N):
//   to g_X:  2 Re(U_XX) s_XX g_X + H conj(s_XY) g_Y,
//   to g_Y:  2 Re(U_YY) s_YY g_Y + conj(H) s_XY g_X,   H = U_XY + conj(U_YX),
// s_PQ the integer sums of auto_sum_kernel (returned as dL/dRe g + i dL/dIm g).
struct AutoHatArgs {
  const double2* grad_image;  // [C][NPROD][N][N], fftshifted
  double* hat;                // [C][(2K-1)^2][NQ]: {Re Gxx, Re Gyy, Re H, Im H} or {Re Gxx}
  int n_chan, N, K;
};

// Workgroup (c, d) as in auto_table_kernel (grid 8 * ceil(C / 8) * (2K-1)^2),
// so a channel's upstream gradient is read through one XCD's L2.
template <int P>
__global__ void __launch_bounds__(256) auto_hat_kernel(AutoHatArgs a) {
  constexpr int NQ = AutoShape<P>::NQ, NPROD = P == 2 ? 4 : 1;
  __shared__ double cs[128];
  __shared__ double red[NQ][4];
  const int N = a.N, K = a.K, D = 2 * K - 1, D2 = D * D;
  int c, d;
  xcd_channel_offset(D2, c, d);
  if (c >= a.n_chan) return;
  const int dj = d / D - (K - 1), di = d % D - (K - 1);
  for (int m = threadIdx.x; m < N; m += 256) cs[m] = cospi(2.0 * m / N);
  __syncthreads();
  const double2* gi = a.grad_image + (int64_t)c * NPROD * N * N;
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  for (int pix = threadIdx.x; pix < N * N; pix += 256) {
    const int km = (pix / N + N / 2) & (N - 1), kl = (pix % N + N / 2) & (N - 1);
    const double e = cs[(di * kl + dj * km) & (N - 1)];
    v[0] = fma(gi[pix].x, e, v[0]);
    if constexpr (P == 2) {
      v[1] = fma(gi[3 * N * N + pix].x, e, v[1]);
      const double2 xy = gi[N * N + pix], yx = gi[2 * N * N + pix];
      v[2] = fma(xy.x + yx.x, e, v[2]);
      v[3] = fma(xy.y - yx.y, e, v[3]);
    }
  }
  block_sum256<NQ>(v, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) a.hat[((int64_t)c * D2 + d) * NQ + q] = v[q];
}

struct AutoGradArgs {
  const int32_t* part;      // [nseg][C][A][NQ] integer sums
  const float2* gains;      // [C][P][A]
  const float* w;           // [C][A][K*K]
  const double* hat;        // [C][(2K-1)^2][NQ]
  double2* gauto;           // [C][P][A]: the removed term's gradient
  int n_chan, n_ant, nseg, K;
};

// One thread per (channel, antenna).
template <int P>
__global__ void __launch_bounds__(256) auto_grad_kernel(AutoGradArgs a) {
  constexpr int NQ = AutoShape<P>::NQ;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t CA = (int64_t)a.n_chan * a.n_ant;
  if (idx >= CA) return;
  const int c = (int)(idx / a.n_ant), ant = (int)(idx % a.n_ant);
  const int K = a.K, D = 2 * K - 1, KK = K * K;
  const float* w = a.w + idx * KK;
  double u[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) u[q] = 0.0;
  const double* hc = a.hat + (int64_t)c * D * D * NQ;
  for (int dj = -(K - 1), d = 0; dj <= K - 1; ++dj)
    for (int di = -(K - 1); di <= K - 1; ++di, ++d) {
      const double r = tap_autocorrelation(w, K, dj, di);
#pragma unroll
      for (int q = 0; q < NQ; ++q) u[q] = fma(r, hc[d * NQ + q], u[q]);
    }
  int64_t m[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) m[q] = 0;
  for (int seg = 0; seg < a.nseg; ++seg)
#pragma unroll
    for (int q = 0; q < NQ; ++q) m[q] += a.part[((int64_t)seg * CA + idx) * NQ + q];
  const float2 gxf = a.gains[(int64_t)c * P * a.n_ant + ant];
  const double gxr = gxf.x, gxi = gxf.y;
  const double fx = 2.0 * u[0] * (double)m[0];
  double2 ox = make_double2(fx * gxr, fx * gxi);
  if constexpr (P == 2) {
    const float2 gyf = a.gains[((int64_t)c * P + 1) * a.n_ant + ant];
    const double gyr = gyf.x, gyi = gyf.y;
    const double fy = 2.0 * u[1] * (double)m[1];
    double2 oy = make_double2(fy * gyr, fy * gyi);
    const double hr = u[2], hi = u[3], sr = (double)m[2], si = (double)m[3];
    // H conj(s) g_Y
    const double tr = hr * sr + hi * si, ti = hi * sr - hr * si;
    ox.x += tr * gyr - ti * gyi;
    ox.y += tr * gyi + ti * gyr;
    // conj(H) s g_X = conj(H conj(s)) g_X
    oy.x += tr * gxr + ti * gxi;
    oy.y += tr * gxi - ti * gxr;
    a.gauto[((int64_t)c * P + 1) * a.n_ant + ant] = oy;
  }
  a.gauto[(int64_t)c * P * a.n_ant + ant] = ox;
}

}  // namespace epic
