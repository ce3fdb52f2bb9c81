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
// and YX = conj(XY).  With complex kernels R_a(d) = sum_u w_a(u) conj(w_a(u - d))
// is Hermitian, and autos_PQ(k) = sum_d [S^c_PQ(d) cos - S^s_PQ(d) sin](2 pi d.k / N)
// with S^c, S^s the sums of V_PQ[a] Re R_a(d) and V_PQ[a] Im R_a(d): the
// tables then hold both (NQT = 2 NQ values per offset).  Kernels:
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

struct AutoFoldArgs {
  const int32_t* part;      // [nseg][C][A][NQ]
  double* sums;             // [C][A][NQ], exact (integers below 2^31)
  int64_t n;                // C * A
  int nseg;
};

// The time segments' partial sums added up: one thread per (channel, antenna),
// all segment loads issued together.
template <int P>
__global__ void __launch_bounds__(256) auto_fold_kernel(AutoFoldArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= a.n) return;
  if constexpr (P == 2) {
    const int4* p = reinterpret_cast<const int4*>(a.part) + idx;
    int4 v[AUTO_MAX_SEG];
#pragma unroll
    for (int seg = 0; seg < AUTO_MAX_SEG; ++seg)
      v[seg] = seg < a.nseg ? p[seg * a.n] : make_int4(0, 0, 0, 0);
    int64_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
#pragma unroll
    for (int seg = 0; seg < AUTO_MAX_SEG; ++seg) {
      m0 += v[seg].x; m1 += v[seg].y; m2 += v[seg].z; m3 += v[seg].w;
    }
    double2* o = reinterpret_cast<double2*>(a.sums) + 2 * idx;
    o[0] = make_double2((double)m0, (double)m1);
    o[1] = make_double2((double)m2, (double)m3);
  } else {
    int v[AUTO_MAX_SEG];
#pragma unroll
    for (int seg = 0; seg < AUTO_MAX_SEG; ++seg) v[seg] = seg < a.nseg ? a.part[seg * a.n + idx] : 0;
    int64_t m0 = 0;
#pragma unroll
    for (int seg = 0; seg < AUTO_MAX_SEG; ++seg) m0 += v[seg];
    a.sums[idx] = (double)m0;
  }
}

struct AutoTableArgs {
  const double* sums;       // [C][A][NQ] from auto_fold_kernel
  const float2* gains;      // [C][P][A]
  const float* w;           // [C][A][K*K] tap weights, tap order dj outer, di inner
  const float* wi;          // [C][A][K*K] imaginary parts (complex kernels)
  double* table;            // [C][(2K-1)^2][NQT]: {XX, YY, Re XY, Im XY} (cos part, then
                            // for complex kernels the sin part), or {XX}[, {XX}]
  int n_chan, n_ant;
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
// footprint, in float64 from the float32 weights w[K*K] (in registers: K is a
// template argument, every loop unrolls).
template <int K>
__device__ __forceinline__ double tap_autocorrelation(const float (&w)[K * K], int dj, int di) {
  double r = 0.0;
#pragma unroll
  for (int uj = 0; uj < K; ++uj)
#pragma unroll
    for (int ui = 0; ui < K; ++ui) {
      const int vj = uj - dj, vi = ui - di;
      if (vj >= 0 && vj < K && vi >= 0 && vi < K)
        r = fma((double)w[uj * K + ui], (double)w[vj * K + vi], r);
    }
  return r;
}

template <int K>
__device__ __forceinline__ void load_taps(const float* src, float (&w)[K * K]) {
#pragma unroll
  for (int i = 0; i < K * K; ++i) w[i] = src[i];
}

// Complex kernel: R(d) = sum_u w(u) conj(w(u - d)) = rr + i ri.
template <int K>
__device__ __forceinline__ void tap_autocorrelation_c(const float (&w)[K * K], const float (&wi)[K * K],
                                                      int dj, int di, double& rr, double& ri) {
  rr = 0.0;
  ri = 0.0;
#pragma unroll
  for (int uj = 0; uj < K; ++uj)
#pragma unroll
    for (int ui = 0; ui < K; ++ui) {
      const int vj = uj - dj, vi = ui - di;
      if (vj >= 0 && vj < K && vi >= 0 && vi < K) {
        const double ar = w[uj * K + ui], ai = wi[uj * K + ui];
        const double br = w[vj * K + vi], bi = wi[vj * K + vi];
        rr = fma(ar, br, fma(ai, bi, rr));
        ri = fma(ai, br, fma(-ar, bi, ri));
      }
    }
}

// S_PQ(d) for one (channel, tap offset) per wave, the wave's lanes taking
// antennas lane, lane + 64, ...  Grid: 8 * ceil(C / 8) * ceil((2K-1)^2 / 4)
// workgroups of four waves; workgroup b takes channel
// (r / G) * 8 + b % 8 and offsets 4 (r % G) + wave, r = b / 8, G =
// ceil((2K-1)^2 / 4), so the workgroups of a channel share one XCD.
template <int P, int K, bool CPX>
__global__ void __launch_bounds__(256) auto_table_kernel(AutoTableArgs a) {
  constexpr int NQ = AutoShape<P>::NQ, NQT = CPX ? 2 * NQ : NQ;
  constexpr int D = 2 * K - 1, D2 = D * D, KK = K * K, G = (D2 + 3) / 4;
  const int r = blockIdx.x / 8, wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int c = (r / G) * 8 + blockIdx.x % 8, d = (r % G) * 4 + wave;
  if (c >= a.n_chan || d >= D2) return;
  const int dj = d / D - (K - 1), di = d % D - (K - 1);
  double s[NQT];
#pragma unroll
  for (int q = 0; q < NQT; ++q) s[q] = 0.0;
#pragma unroll 4
  for (int ant = lane; ant < a.n_ant; ant += 64) {
    const int64_t ca = (int64_t)c * a.n_ant + ant;
    double m[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) m[q] = a.sums[ca * NQ + q];
    float w[KK];
    load_taps<K>(a.w + ca * KK, w);
    double rr, ri = 0.0;
    if constexpr (CPX) {
      float wi[KK];
      load_taps<K>(a.wi + ca * KK, wi);
      tap_autocorrelation_c<K>(w, wi, dj, di, rr, ri);
    } else {
      rr = tap_autocorrelation<K>(w, dj, di);
    }
    // V_PQ[a] as NQ reals: |g_X|^2 m0, |g_Y|^2 m1, g_X conj(g_Y) (m2 + i m3)
    double v[NQ];
    const float2 gx = a.gains[(int64_t)c * P * a.n_ant + ant];
    const double gxr = gx.x, gxi = gx.y;
    v[0] = (gxr * gxr + gxi * gxi) * m[0];
    if constexpr (P == 2) {
      const float2 gy = a.gains[((int64_t)c * P + 1) * a.n_ant + ant];
      const double gyr = gy.x, gyi = gy.y;
      v[1 % NQ] = (gyr * gyr + gyi * gyi) * m[1 % NQ];
      const double hr = gxr * gyr + gxi * gyi, hi = gxi * gyr - gxr * gyi;
      v[2 % NQ] = hr * m[2 % NQ] - hi * m[3 % NQ];
      v[3 % NQ] = hr * m[3 % NQ] + hi * m[2 % NQ];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      s[q] = fma(v[q], rr, s[q]);
      if constexpr (CPX) s[NQ + q] = fma(v[q], ri, s[NQ + q]);
    }
  }
  // fixed-order sum over the wave
#pragma unroll
  for (int q = 0; q < NQT; ++q)
    for (int off = 32; off > 0; off >>= 1) s[q] += __shfl_down(s[q], off, 64);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NQT; ++q) a.table[((int64_t)c * D2 + d) * NQT + q] = s[q];
}

// The removed term at unshifted pixel (km, kl) from a channel's table st (in
// LDS, [(2K-1)^2][NQT]) and cs[m], sn[m] = cos, sin(2 pi m / N): v[q] =
// sum_d st[d][q] cos(2 pi (di kl + dj km) / N) (- st[d][NQ + q] sin(...) when CPX).
template <int NQ, bool CPX>
__device__ __forceinline__ void autos_at(const double* st, const double* cs, const double* sn, int N,
                                         int K, int km, int kl, double (&v)[NQ]) {
  constexpr int NQT = CPX ? 2 * NQ : NQ;
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  for (int dj = -(K - 1), d = 0; dj <= K - 1; ++dj)
    for (int di = -(K - 1); di <= K - 1; ++di, ++d) {
      const int m = (di * kl + dj * km) & (N - 1);
      const double e = cs[m];
#pragma unroll
      for (int q = 0; q < NQ; ++q) v[q] = fma(st[d * NQT + q], e, v[q]);
      if constexpr (CPX) {
        const double f = sn[m];
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = fma(-st[d * NQT + NQ + q], f, v[q]);
      }
    }
}

// Stage channel c's table (nqt values per offset) and the cosine and sine
// tables into LDS (all threads of the workgroup take part; a barrier follows).
__device__ __forceinline__ void stage_autos(const double* table, int c, int N, int K, int nqt,
                                            double* st, double* cs, double* sn) {
  const int D = 2 * K - 1;
  for (int i = threadIdx.x; i < D * D * nqt; i += blockDim.x)
    st[i] = table[(int64_t)c * D * D * nqt + i];
  for (int m = threadIdx.x; m < N; m += blockDim.x) sincospi(2.0 * m / N, &sn[m], &cs[m]);
  __syncthreads();
}

struct AutoRemoveArgs {
  const double* table;      // [C][(2K-1)^2][NQT]
  double2* image;           // [C][NPROD][N][N], fftshifted
  int n_chan, N, K;
  int cpx;                  // the table holds the sin part too (complex kernels)
};

// Grid: C * ceil(N^2 / 256) workgroups, channel-major; one thread per pixel.
template <int P>
__global__ void __launch_bounds__(256) auto_remove_kernel(AutoRemoveArgs a) {
  constexpr int NQ = AutoShape<P>::NQ;
  __shared__ double st[AUTO_MAX_D2 * 2 * NQ];
  __shared__ double cs[128], sn[128];
  const int N = a.N, K = a.K, tiles = (N * N + 255) / 256;
  const int c = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  stage_autos(a.table, c, N, K, a.cpx ? 2 * NQ : NQ, st, cs, sn);
  const int pix = tile * 256 + threadIdx.x;
  if (pix >= N * N) return;
  // pixel (q_m, q_l) of the shifted image holds k = (q - N/2) mod N
  const int km = (pix / N + N / 2) & (N - 1), kl = (pix % N + N / 2) & (N - 1);
  double v[NQ];
  if (a.cpx) autos_at<NQ, true>(st, cs, sn, N, K, km, kl, v);
  else autos_at<NQ, false>(st, cs, sn, N, K, km, kl, v);
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
  double* hat;                // [C][(2K-1)^2][NQT]: {Re Gxx, Re Gyy, Re H, Im H} or {Re Gxx}
                              // summed against cos, then (complex kernels) against sin
  int n_chan, N, K;
};

// Workgroup (c, d) as in auto_table_kernel (grid 8 * ceil(C / 8) * (2K-1)^2),
// so a channel's upstream gradient is read through one XCD's L2.
template <int P, bool CPX>
__global__ void __launch_bounds__(256) auto_hat_kernel(AutoHatArgs a) {
  constexpr int NQ = AutoShape<P>::NQ, NPROD = P == 2 ? 4 : 1, NQT = CPX ? 2 * NQ : NQ;
  __shared__ double cs[128], sn[128];
  __shared__ double red[NQT][4];
  const int N = a.N, K = a.K, D = 2 * K - 1, D2 = D * D;
  int c, d;
  xcd_channel_offset(D2, c, d);
  if (c >= a.n_chan) return;
  const int dj = d / D - (K - 1), di = d % D - (K - 1);
  for (int m = threadIdx.x; m < N; m += 256) sincospi(2.0 * m / N, &sn[m], &cs[m]);
  __syncthreads();
  const double2* gi = a.grad_image + (int64_t)c * NPROD * N * N;
  double v[NQT];
#pragma unroll
  for (int q = 0; q < NQT; ++q) v[q] = 0.0;
  for (int pix = threadIdx.x; pix < N * N; pix += 256) {
    const int km = (pix / N + N / 2) & (N - 1), kl = (pix % N + N / 2) & (N - 1);
    const int m = (di * kl + dj * km) & (N - 1);
    double gq[NQ];
    gq[0] = gi[pix].x;
    if constexpr (P == 2) {
      gq[1 % NQ] = gi[3 * N * N + pix].x;
      const double2 xy = gi[N * N + pix], yx = gi[2 * N * N + pix];
      gq[2 % NQ] = xy.x + yx.x;
      gq[3 % NQ] = xy.y - yx.y;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      v[q] = fma(gq[q], cs[m], v[q]);
      if constexpr (CPX) v[NQ + q] = fma(gq[q], sn[m], v[NQ + q]);
    }
  }
  block_sum256<NQT>(v, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NQT; ++q) a.hat[((int64_t)c * D2 + d) * NQT + q] = v[q];
}

struct AutoGradArgs {
  const double* sums;       // [C][A][NQ] from auto_fold_kernel
  const float2* gains;      // [C][P][A]
  const float* w;           // [C][A][K*K]
  const float* wi;          // [C][A][K*K] imaginary parts (complex kernels)
  const double* hat;        // [C][(2K-1)^2][NQT]
  double2* gauto;           // [C][P][A]: the removed term's gradient
  int n_chan, n_ant;
};

// One thread per (channel, antenna); U = sum_d Re R(d) Ghat_cos(d) - Im R(d) Ghat_sin(d).
template <int P, int K, bool CPX>
__global__ void __launch_bounds__(256) auto_grad_kernel(AutoGradArgs a) {
  constexpr int NQ = AutoShape<P>::NQ, D = 2 * K - 1, KK = K * K, NQT = CPX ? 2 * NQ : NQ;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t CA = (int64_t)a.n_chan * a.n_ant;
  if (idx >= CA) return;
  const int c = (int)(idx / a.n_ant), ant = (int)(idx % a.n_ant);
  float w[KK], wi[CPX ? KK : 1];
  load_taps<K>(a.w + idx * KK, w);
  if constexpr (CPX) load_taps<K>(a.wi + idx * KK, wi);
  double u[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) u[q] = 0.0;
  const double* hc = a.hat + (int64_t)c * D * D * NQT;
  for (int dj = -(K - 1), d = 0; dj <= K - 1; ++dj)
    for (int di = -(K - 1); di <= K - 1; ++di, ++d) {
      if constexpr (CPX) {
        double rr, ri;
        tap_autocorrelation_c<K>(w, wi, dj, di, rr, ri);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          u[q] = fma(rr, hc[d * NQT + q], fma(-ri, hc[d * NQT + NQ + q], u[q]));
      } else {
        const double r = tap_autocorrelation<K>(w, dj, di);
#pragma unroll
        for (int q = 0; q < NQ; ++q) u[q] = fma(r, hc[d * NQ + q], u[q]);
      }
    }
  double m[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) m[q] = a.sums[idx * NQ + q];
  const float2 gxf = a.gains[(int64_t)c * P * a.n_ant + ant];
  const double gxr = gxf.x, gxi = gxf.y;
  const double fx = 2.0 * u[0] * m[0];
  double2 ox = make_double2(fx * gxr, fx * gxi);
  if constexpr (P == 2) {
    const float2 gyf = a.gains[((int64_t)c * P + 1) * a.n_ant + ant];
    const double gyr = gyf.x, gyi = gyf.y;
    const double fy = 2.0 * u[1] * m[1];
    double2 oy = make_double2(fy * gyr, fy * gyi);
    const double hr = u[2], hi = u[3], sr = m[2], si = m[3];
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
