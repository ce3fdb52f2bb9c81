// Split-precision matrix form of gridding + transform (the operator view of
// the imaging step, paper Sec. 3.3: gridding as a matrix product), on the
// MFMA units.
//
// For one channel and polarisation the gridded-and-transformed field is
// linear in the samples:  F[pix] = sum_a B[pix][a] e[a],  with
//   B[pix][a] = g[a] * beta_a(pix),  beta_a(k) = sum_taps w exp(+2 pi i (i kl + j km)/N),
// i.e. the transform of antenna a's kernel footprint times its gain.  beta is
// computed once in float64 on the host; B is formed per call, scaled by a
// power of two s (per channel and polarisation) and split as
// B s = B_hi + B_lo with B_hi = rnd(B s), B_lo = rnd(B s - B_hi) in float16 or
// bfloat16.  The samples are small integers, exact in both formats, so
//   F s = B_hi e + B_lo e
// with float32 accumulation.  In real form, over K' = 2A (re then im parts):
//   Re(F s) = Br er - Bi ei,  Im(F s) = Bi er + Br ei.
//
// MFMA tiling (v_mfma_f32_32x32x16_{f16,bf16}): D[time][pixel] = E[time][k] B[k][pixel]
// for 32 samples x 32 pixels, k over 16 antennas.  Lane l supplies
// E[t = l%32][k = 8(l/32) .. +7] and B[k = 8(l/32) .. +7][pix = l%32]; it receives
// D[8(r/4) + 4(l/32) + r%4][l%32] in register r, so every lane owns one pixel
// and 16 of the 32 samples: |F|^2 (or F_X conj F_Y) is summed over time inside
// the lane, in float64 per tile.  The matrix operands of one 32-pixel tile stay
// in registers for the whole time range of the wave.
#pragma once
#include <hip/hip_runtime.h>

#include "reduce.hpp"
#include <stdint.h>

namespace epic {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float16v_t __attribute__((ext_vector_type(16)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t f32_to_f16_bits(float x) {
  const _Float16 h = (_Float16)x;
  return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_bits_to_f32(uint16_t b) {
  return (float)__builtin_bit_cast(_Float16, b);
}

constexpr int kSplitParts = 3;     // Br, Bi, -Bi
constexpr int kSplitMaxBlocks = 2; // antenna blocks of 16 held in registers (A <= 32)

struct SplitPrepArgs {
  const float2* gains;      // [C][P][A]
  const double2* beta;      // [C][NG][A]
  const double* beta_max;   // [C] max |beta|
  uint16_t* bmat;           // [C][P][part][hi/lo][NG][AP]
  float* scale;             // [C][P]: s
  int n_chan, n_pol, n_ant, a_pad, ng;
};

// Workgroups (channel and polarisation, chunk of about 256 matrix entries,
// one per thread); every wave computes the scale of its (channel,
// polarisation) from the gains itself (A <= 32 values, a wave-wide maximum).
template <bool BF>
__global__ void __launch_bounds__(256) split_prep_kernel(SplitPrepArgs a) {
  const int cp = blockIdx.x;
  const int c = cp / a.n_pol;
  const float2* g = a.gains + (int64_t)cp * a.n_ant;
  double m = 0.0;
  for (int i = threadIdx.x & 63; i < a.n_ant; i += 64) m = fmax(m, hypot((double)g[i].x, (double)g[i].y));
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  const double bmax = m * a.beta_max[c];
  // scale so that |B s| < 2^14: the hi parts stay finite, the lo parts normal
  const double sc = bmax > 0.0 ? ldexp(1.0, 13 - ilogb(bmax)) : 1.0;
  if (threadIdx.x == 0 && blockIdx.y == 0) a.scale[cp] = (float)sc;
  const int64_t plane = (int64_t)a.ng * a.a_pad;
  uint16_t* out = a.bmat + (int64_t)cp * kSplitParts * 2 * plane;
  const double2* beta = a.beta + (int64_t)c * a.ng * a.n_ant;
  const int64_t per = (plane + gridDim.y - 1) / gridDim.y;
  const int64_t end = plane < (int64_t)(blockIdx.y + 1) * per ? plane : (int64_t)(blockIdx.y + 1) * per;
  for (int64_t idx = (int64_t)blockIdx.y * per + threadIdx.x; idx < end; idx += 256) {
    const int pix = (int)(idx / a.a_pad), ant = (int)(idx % a.a_pad);
    double br = 0.0, bi = 0.0;
    if (ant < a.n_ant) {
      const double2 b = beta[(int64_t)pix * a.n_ant + ant];
      const double gr = g[ant].x, gi = g[ant].y;
      br = (gr * b.x - gi * b.y) * sc;
      bi = (gr * b.y + gi * b.x) * sc;
    }
    const double v[kSplitParts] = {br, bi, -bi};
#pragma unroll
    for (int part = 0; part < kSplitParts; ++part) {
      const float x = (float)v[part];
      uint16_t hi, lo;
      if (BF) {
        hi = f32_to_bf16_bits(x);
        lo = f32_to_bf16_bits((float)(v[part] - (double)bf16_bits_to_f32(hi)));
      } else {
        hi = f32_to_f16_bits(x);
        lo = f32_to_f16_bits((float)(v[part] - (double)f16_bits_to_f32(hi)));
      }
      out[(part * 2 + 0) * plane + idx] = hi;
      out[(part * 2 + 1) * plane + idx] = lo;
    }
  }
}

struct SplitArgs {
  const uint8_t* efield;    // [T][C][P][A]
  const uint16_t* bmat;     // as written by split_prep_kernel
  double* partial;          // [C][n_chunks][NACC][2][NG]
  int64_t n_time;
  int n_chan, n_ant, a_pad, ng, chunk, n_chunks;
  int tile_wgs;             // workgroups per (chunk, channel)
};

template <bool BF> struct SplitOps;
template <> struct SplitOps<false> {
  using v8 = half8_t;
  static __device__ __forceinline__ float16v_t mfma(v8 x, v8 y, float16v_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(x, y, c, 0, 0, 0);
  }
  // The 8 complex samples of one row (a byte each: real part in the high
  // nibble, imaginary in the low, two's complement) as float16 real and
  // imaginary parts.  w ^ 0x88888888 biases every nibble by 8 (m = v + 8 in
  // 0..15); m placed under the high byte 0x64 is the float16 pattern of
  // 1024 + m, exactly, and one packed subtraction of 1032 leaves v.
  static __device__ __forceinline__ void unpack(uint2 w, v8& er, v8& ei) {
    const uint32_t tx = w.x ^ 0x88888888u, ty = w.y ^ 0x88888888u;
    const uint32_t ix = tx & 0x0F0F0F0Fu, iy = ty & 0x0F0F0F0Fu;
    const uint32_t rx = (tx >> 4) & 0x0F0F0F0Fu, ry = (ty >> 4) & 0x0F0F0F0Fu;
    constexpr uint32_t kExp = 0x64646464u;
    // bytes m0 m1 (selectors 0x04010400) or m2 m3 (0x04030402), each under 0x64
    const uint4 rb = make_uint4(__builtin_amdgcn_perm(kExp, rx, 0x04010400u),
                                __builtin_amdgcn_perm(kExp, rx, 0x04030402u),
                                __builtin_amdgcn_perm(kExp, ry, 0x04010400u),
                                __builtin_amdgcn_perm(kExp, ry, 0x04030402u));
    const uint4 ib = make_uint4(__builtin_amdgcn_perm(kExp, ix, 0x04010400u),
                                __builtin_amdgcn_perm(kExp, ix, 0x04030402u),
                                __builtin_amdgcn_perm(kExp, iy, 0x04010400u),
                                __builtin_amdgcn_perm(kExp, iy, 0x04030402u));
    const _Float16 b = (_Float16)1032.0f;
    const v8 bias = {b, b, b, b, b, b, b, b};
    er = __builtin_bit_cast(v8, rb) - bias;
    ei = __builtin_bit_cast(v8, ib) - bias;
  }
};
template <> struct SplitOps<true> {
  using v8 = bf16x8_t;
  static __device__ __forceinline__ float16v_t mfma(v8 x, v8 y, float16v_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, c, 0, 0, 0);
  }
  // as for float16, through the sign-extended nibbles (no packed bfloat16
  // add on this chip); small integers are exact in bfloat16.  The sign
  // extension is written as shifts: the compiler used here converts the
  // result of __builtin_amdgcn_sbfe to float as if it were unsigned.
  static __device__ __forceinline__ void unpack(uint2 w, v8& er, v8& ei) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t x = (i < 4) ? w.x : w.y;
      const int sh = 8 * (i & 3);
      er[i] = (__bf16)(float)((int)(x << (24 - sh)) >> 28);   // high nibble
      ei[i] = (__bf16)(float)((int)(x << (28 - sh)) >> 28);   // low nibble
    }
  }
};

template <bool BF> __device__ __forceinline__ typename SplitOps<BF>::v8 load8(const uint16_t* p) {
  const uint4 u = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(typename SplitOps<BF>::v8, u);
}

// The 8 bytes of antennas 16 q + 8 h .. + 7 of sample row t (zero past the
// end of the chunk or of the antennas).  VEC: A is a multiple of 8, so the
// 8 bytes are one aligned 8-byte load or all out of range.
template <bool VEC>
__device__ __forceinline__ uint2 load_e8(const uint8_t* row, int first_ant, int n_ant, bool in_time) {
  if (VEC) {
    if (!in_time || first_ant >= n_ant) return make_uint2(0u, 0u);
    return *reinterpret_cast<const uint2*>(row + first_ant);
  }
  uint32_t w[2] = {0u, 0u};
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int ant = first_ant + i;
    const uint32_t b = (in_time && ant < n_ant) ? (uint32_t)row[ant] : 0u;
    w[i >> 2] |= b << (8 * (i & 3));
  }
  return make_uint2(w[0], w[1]);
}

// Sample-row blocks loaded ahead of the one on the matrix units: the rows
// come from HBM and a block's matrix work is shorter than that latency
// (two polarisations: half the depth, which keeps three waves per SIMD).
template <int P> constexpr int split_prefetch() { return P == 2 ? 2 : 4; }
static_assert(split_prefetch<1>() % 2 == 0 && split_prefetch<2>() % 2 == 0,
              "the accumulator double buffer takes block parity from the ring slot");

// Workgroup id -> logical index such that consecutive logical indices share
// an XCD (workgroups are dealt to the 8 XCDs round-robin by id): XCD j holds
// logical indices [j q + min(j, r), ...) of the n = 8 q + r workgroups.
__device__ __forceinline__ int xcd_contiguous_index(int id, int n) {
  const int q = n >> 3, r = n & 7, j = id & 7;
  return j * q + (j < r ? j : r) + (id >> 3);
}

// One wave per (TPW 32-pixel tiles, time chunk, channel); 4 waves per
// workgroup on consecutive tile groups; the workgroups of one (chunk,
// channel), which read the same sample rows, share an XCD and its L2.  QB
// antenna blocks of 16 (A <= 16 QB).
template <int P, bool BF, int QB, int TPW, bool VEC>
__global__ void __launch_bounds__(256) split_image_kernel(SplitArgs a) {
  using Ops = SplitOps<BF>;
  using v8 = typename Ops::v8;
  constexpr int NACC = (P == 2) ? 4 : 1;
  constexpr int PD = split_prefetch<P>();
  const int lane = threadIdx.x & 63;
  const int logical = xcd_contiguous_index((int)blockIdx.x, (int)gridDim.x);
  const int rest = logical / a.tile_wgs;
  const int tile0 = ((logical - rest * a.tile_wgs) * 4 + (threadIdx.x >> 6)) * TPW;
  const int chunk = rest % a.n_chunks;
  const int c = rest / a.n_chunks;
  if (tile0 * 32 >= a.ng) return;
  const int n = lane & 31, h = lane >> 5;

  // matrix operands of the tiles: [tile][pol][block][part][hi/lo]
  v8 bm[TPW][P][QB][kSplitParts][2];
  const int64_t plane = (int64_t)a.ng * a.a_pad;
#pragma unroll
  for (int u = 0; u < TPW; ++u)
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const uint16_t* base = a.bmat + ((int64_t)c * P + p) * kSplitParts * 2 * plane +
                             (int64_t)((tile0 + u) * 32 + n) * a.a_pad + 8 * h;
#pragma unroll
      for (int q = 0; q < QB; ++q)
#pragma unroll
        for (int part = 0; part < kSplitParts; ++part)
#pragma unroll
          for (int hl = 0; hl < 2; ++hl)
            bm[u][p][q][part][hl] = load8<BF>(base + (part * 2 + hl) * plane + 16 * q);
    }

  double acc[TPW][NACC];
#pragma unroll
  for (int u = 0; u < TPW; ++u)
#pragma unroll
    for (int k = 0; k < NACC; ++k) acc[u][k] = 0.0;
  const int64_t t_begin = (int64_t)chunk * a.chunk;
  const int64_t t_end = t_begin + a.chunk < a.n_time ? t_begin + a.chunk : a.n_time;
  const int64_t row_bytes = (int64_t)a.n_chan * P * a.n_ant;
  const uint8_t* chan = a.efield + (int64_t)c * P * a.n_ant;

  // ring of PD sample-row blocks; block k sits in slot k % PD
  uint2 ring[PD][P][QB];
  auto load_block = [&](uint2 (&dst)[P][QB], int64_t t0) {
    const int64_t t = t0 + n;                  // this lane's sample row of E
    const uint8_t* row = chan + t * row_bytes;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int q = 0; q < QB; ++q)
        dst[p][q] = load_e8<VEC>(row + p * a.n_ant, 16 * q + 8 * h, a.n_ant, t < t_end);
  };
  // Software pipeline over blocks: the matrix products of block k go into
  // accumulator set k % 2 while the epilogue of block k - 1 reads the other
  // set, so the epilogue's VALU work is independent of the MFMAs in flight.
  float16v_t dre[2][TPW][P], dim[2][TPW][P];
  auto products = [&](const uint2 (&cur)[P][QB], float16v_t (&xr)[TPW][P], float16v_t (&xi)[TPW][P]) {
#pragma unroll
    for (int u = 0; u < TPW; ++u)
#pragma unroll
      for (int p = 0; p < P; ++p) {
        xr[u][p] = float16v_t{};
        xi[u][p] = float16v_t{};
      }
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        v8 er, ei;
        Ops::unpack(cur[p][q], er, ei);
        // Re(F s) = Br er - Bi ei ; Im(F s) = Bi er + Br ei   (hi and lo terms)
#pragma unroll
        for (int u = 0; u < TPW; ++u)
#pragma unroll
          for (int hl = 0; hl < 2; ++hl) {
            xr[u][p] = Ops::mfma(er, bm[u][p][q][0][hl], xr[u][p]);
            xr[u][p] = Ops::mfma(ei, bm[u][p][q][2][hl], xr[u][p]);
            xi[u][p] = Ops::mfma(er, bm[u][p][q][1][hl], xi[u][p]);
            xi[u][p] = Ops::mfma(ei, bm[u][p][q][0][hl], xi[u][p]);
          }
      }
  };
  // products summed over the 16 samples of this lane, then into float64
  auto epilogue = [&](const float16v_t (&xr)[TPW][P], const float16v_t (&xi)[TPW][P]) {
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
      float sm[NACC];
#pragma unroll
      for (int k = 0; k < NACC; ++k) sm[k] = 0.f;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float fxr = xr[u][0][r], fxi = xi[u][0][r];
        sm[0] = fmaf(fxi, fxi, fmaf(fxr, fxr, sm[0]));
        if (P == 2) {
          const float fyr = xr[u][P - 1][r], fyi = xi[u][P - 1][r];
          sm[1 % NACC] = fmaf(fyi, fyi, fmaf(fyr, fyr, sm[1 % NACC]));
          sm[2 % NACC] = fmaf(fxi, fyi, fmaf(fxr, fyr, sm[2 % NACC]));
          sm[3 % NACC] = fmaf(-fxr, fyi, fmaf(fxi, fyr, sm[3 % NACC]));
        }
      }
#pragma unroll
      for (int k = 0; k < NACC; ++k) acc[u][k] += (double)sm[k];
    }
  };
#pragma unroll
  for (int d = 0; d < PD; ++d) load_block(ring[d], t_begin + 32 * d);
  // Block k of the chunk uses accumulator set k % 2 = d % 2 (PD is even and
  // tb advances by 32 PD).  The first block's predecessor is an all-zero set,
  // whose epilogue adds exact zeros.
#pragma unroll
  for (int u = 0; u < TPW; ++u)
#pragma unroll
    for (int p = 0; p < P; ++p) {
      dre[1][u][p] = float16v_t{};
      dim[1][u][p] = float16v_t{};
    }
  // instruction counts of one block, for the issue pattern below: the sample
  // conversion, then one MFMA followed by an equal share of the epilogue
  constexpr int kMfma = 8 * TPW * P * QB;
  constexpr int kConv = (BF ? 40 : 24) * P * QB;
  constexpr int kEpi = TPW * (32 * NACC + 2 * NACC);
  constexpr int kPer = (kEpi + kMfma - 1) / kMfma;
  for (int64_t tb = t_begin; tb < t_end; tb += 32 * PD)
#pragma unroll
  for (int d = 0; d < PD; ++d) {
    const int64_t t0 = tb + 32 * d;
    if (t0 >= t_end) break;
    uint2 cur[P][QB];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int q = 0; q < QB; ++q) cur[p][q] = ring[d][p][q];
    if (t0 + 32 * PD < t_end) load_block(ring[d], t0 + 32 * PD);
    products(cur, dre[d & 1], dim[d & 1]);
    epilogue(dre[(d & 1) ^ 1], dim[(d & 1) ^ 1]);
    __builtin_amdgcn_sched_group_barrier(0x002, kConv, 0);      // VALU: conversion
#pragma unroll
    for (int i = 0; i < kMfma; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);        // one MFMA
      __builtin_amdgcn_sched_group_barrier(0x002, kPer, 0);     // VALU: epilogue share
    }
  }
  // the last block's epilogue
  const int last = (int)(((t_end - t_begin + 31) / 32 - 1) & 1);
  if (last == 0) epilogue(dre[0], dim[0]);
  else epilogue(dre[1], dim[1]);
  double* out = a.partial + (((int64_t)c * a.n_chunks + chunk) * NACC * 2) * a.ng;
#pragma unroll
  for (int u = 0; u < TPW; ++u)
#pragma unroll
    for (int k = 0; k < NACC; ++k) out[((int64_t)k * 2 + h) * a.ng + (tile0 + u) * 32 + n] = acc[u][k];
}

struct SplitReduceArgs {
  const double* partial;    // [C][n_chunks][NACC][2][NG]
  const float* scale;       // [C][P]
  double* image;            // complex128 [C][NPROD][N][N]
  int n_chan, n_chunks, ng, n, reset;
  int sub;                  // sub-lanes per pixel, as in reduce_image_kernel
};

// image (+)= (sum over chunks and the two lane halves, sub-lane j taking
// chunks j, j + sub, ... and the sub-lanes added in order) / scales,
// fftshifted and expanded to XX, XY, YX, YY.
template <int P>
__global__ void __launch_bounds__(256) split_reduce_kernel(SplitReduceArgs a) {
  constexpr int NACC = (P == 2) ? 4 : 1;
  constexpr int NPROD = (P == 2) ? 4 : 1;
  __shared__ double red[NACC * 256];
  const int ppb = 256 / a.sub;
  const int j = threadIdx.x / ppb, lp = threadIdx.x % ppb;
  const int64_t idx = (int64_t)blockIdx.x * ppb + lp;
  const bool valid = idx < (int64_t)a.n_chan * a.ng;
  const int c = valid ? (int)(idx / a.ng) : 0, pix = (int)(idx % a.ng);
  double s[NACC];
#pragma unroll
  for (int u = 0; u < NACC; ++u) s[u] = 0.0;
  if (valid) {
#pragma unroll 4
    for (int k = j; k < a.n_chunks; k += a.sub) {
      const double* src = a.partial + (((int64_t)c * a.n_chunks + k) * NACC * 2) * a.ng + pix;
#pragma unroll
      for (int u = 0; u < NACC; ++u)
        s[u] += src[(int64_t)(2 * u) * a.ng] + src[(int64_t)(2 * u + 1) * a.ng];
    }
  }
  combine_sublanes<NACC>(s, a.sub, ppb, j, lp, red);
  if (!valid || j != 0) return;
  const double sx = a.scale[c * P], sy = a.scale[c * P + P - 1];
  const int N = a.n;
  const int km = pix / N, kl = pix % N;
  const int qm = (km + N / 2) % N, ql = (kl + N / 2) % N;
  double2* img = reinterpret_cast<double2*>(a.image) + (int64_t)c * NPROD * a.ng + qm * N + ql;
  double2 val[NPROD];
  val[0] = make_double2(s[0] / (sx * sx), 0.0);
  if (P == 2) {
    const double xy = 1.0 / (sx * sy);
    val[1 % NPROD] = make_double2(s[2 % NACC] * xy, s[3 % NACC] * xy);
    val[2 % NPROD] = make_double2(s[2 % NACC] * xy, -s[3 % NACC] * xy);
    val[3 % NPROD] = make_double2(s[1 % NACC] / (sy * sy), 0.0);
  }
#pragma unroll
  for (int pr = 0; pr < NPROD; ++pr) {
    double2* o = img + (int64_t)pr * a.ng;
    if (a.reset) {
      *o = val[pr];
    } else {
      const double2 old = *o;
      *o = make_double2(old.x + val[pr].x, old.y + val[pr].y);
    }
  }
}

}  // namespace epic
