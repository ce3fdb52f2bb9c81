// Complex arithmetic and small DFTs in registers, plus the two-pass line
// transform used by every 2-D transform of the library.
//
// Sign convention: SG = +1 computes X[k] = sum_n x[n] exp(+2 pi i n k / M)
// (the imaging direction of the paper's Eq. (5)); SG = -1 the conjugate
// (adjoint) direction.  Internal constants are exact values of cos/sin at
// multiples of pi/8; all other twiddles come from a host table computed in
// float64 and rounded once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace epic {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * b
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
template <int SG> __device__ __forceinline__ float2 twiddle_mul(float2 a, float2 w) {
  return SG > 0 ? cmul(a, w) : cmulc(a, w);
}
// multiply by SG * i
template <int SG> __device__ __forceinline__ float2 mul_i(float2 a) {
  return SG > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int SG> __device__ __forceinline__ void dft2(float2& a, float2& b) {
  const float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int SG> __device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  const float2 t0 = cadd(x0, x2), t1 = csub(x0, x2);
  const float2 t2 = cadd(x1, x3), t3 = mul_i<SG>(csub(x1, x3));
  x0 = cadd(t0, t2);
  x2 = csub(t0, t2);
  x1 = cadd(t1, t3);
  x3 = csub(t1, t3);
}

// 8-point DFT: even/odd split into two 4-point DFTs, then w8^k o[k].
template <int SG> __device__ __forceinline__ void dft8(float2* x) {
  float2 e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  float2 o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
  dft4<SG>(e0, e1, e2, e3);
  dft4<SG>(o0, o1, o2, o3);
  const float r = 0.70710678118654752440f;  // cos(pi/4)
  float2 t1, t3;
  if (SG > 0) {  // w = (1 + i)/sqrt2, w^3 = (-1 + i)/sqrt2
    t1 = make_float2((o1.x - o1.y) * r, (o1.x + o1.y) * r);
    t3 = make_float2((-o3.x - o3.y) * r, (o3.x - o3.y) * r);
  } else {       // w = (1 - i)/sqrt2, w^3 = (-1 - i)/sqrt2
    t1 = make_float2((o1.x + o1.y) * r, (o1.y - o1.x) * r);
    t3 = make_float2((o3.y - o3.x) * r, (-o3.x - o3.y) * r);
  }
  const float2 t2 = mul_i<SG>(o2);
  x[0] = cadd(e0, o0); x[4] = csub(e0, o0);
  x[1] = cadd(e1, t1); x[5] = csub(e1, t1);
  x[2] = cadd(e2, t2); x[6] = csub(e2, t2);
  x[3] = cadd(e3, t3); x[7] = csub(e3, t3);
}

// 16-point DFT as 4 x 4: x[4 n1 + n0] -> X[k0 + 4 k1].
template <int SG> __device__ __forceinline__ void dft16(float2* x) {
  const float c1 = 0.92387953251128675613f;  // cos(pi/8)
  const float s1 = 0.38268343236508977173f;  // sin(pi/8)
  const float r = 0.70710678118654752440f;   // cos(pi/4)
  float2 y[16];
#pragma unroll
  for (int n0 = 0; n0 < 4; ++n0) {
    float2 a = x[n0], b = x[4 + n0], c = x[8 + n0], d = x[12 + n0];
    dft4<SG>(a, b, c, d);           // over n1 -> k0 = 0..3
    y[4 * 0 + n0] = a; y[4 * 1 + n0] = b; y[4 * 2 + n0] = c; y[4 * 3 + n0] = d;
  }
  // twiddle w16^(n0 k0), stored at y[4 k0 + n0]
  const float2 w1 = make_float2(c1, SG * s1), w2 = make_float2(r, SG * r), w3 = make_float2(s1, SG * c1);
  const float2 w6 = make_float2(-r, SG * r), w9 = make_float2(-c1, -SG * s1);
  y[4 * 1 + 1] = cmul(y[5], w1);
  y[4 * 1 + 2] = cmul(y[6], w2);
  y[4 * 1 + 3] = cmul(y[7], w3);
  y[4 * 2 + 1] = cmul(y[9], w2);
  y[4 * 2 + 2] = mul_i<SG>(y[10]);
  y[4 * 2 + 3] = cmul(y[11], w6);
  y[4 * 3 + 1] = cmul(y[13], w3);
  y[4 * 3 + 2] = cmul(y[14], w6);
  y[4 * 3 + 3] = cmul(y[15], w9);
#pragma unroll
  for (int k0 = 0; k0 < 4; ++k0) {
    float2 a = y[4 * k0], b = y[4 * k0 + 1], c = y[4 * k0 + 2], d = y[4 * k0 + 3];
    dft4<SG>(a, b, c, d);           // over n0 -> k1
    x[k0] = a; x[k0 + 4] = b; x[k0 + 8] = c; x[k0 + 12] = d;
  }
}

// 8-point DFT whose inputs x[4..7] are zero (they are not read).
template <int SG> __device__ __forceinline__ void dft8_half(float2* x) {
  // 4-point DFTs of (a, b, 0, 0): a + b, a + SG i b, a - b, a - SG i b
  const float2 ib0 = mul_i<SG>(x[2]), ib1 = mul_i<SG>(x[3]);
  const float2 e0 = cadd(x[0], x[2]), e1 = cadd(x[0], ib0), e2 = csub(x[0], x[2]), e3 = csub(x[0], ib0);
  const float2 o0 = cadd(x[1], x[3]), o1 = cadd(x[1], ib1), o2 = csub(x[1], x[3]), o3 = csub(x[1], ib1);
  const float r = 0.70710678118654752440f;
  float2 t1, t3;
  if (SG > 0) {
    t1 = make_float2((o1.x - o1.y) * r, (o1.x + o1.y) * r);
    t3 = make_float2((-o3.x - o3.y) * r, (o3.x - o3.y) * r);
  } else {
    t1 = make_float2((o1.x + o1.y) * r, (o1.y - o1.x) * r);
    t3 = make_float2((o3.y - o3.x) * r, (-o3.x - o3.y) * r);
  }
  const float2 t2 = mul_i<SG>(o2);
  x[0] = cadd(e0, o0); x[4] = csub(e0, o0);
  x[1] = cadd(e1, t1); x[5] = csub(e1, t1);
  x[2] = cadd(e2, t2); x[6] = csub(e2, t2);
  x[3] = cadd(e3, t3); x[7] = csub(e3, t3);
}

// 8-point DFT whose inputs x[6], x[7] are zero (they are not read): the
// 4-point DFTs of (a, b, c, 0) are a + c +- b and a - c +- SG i b.
template <int SG> __device__ __forceinline__ void dft8_six(float2* x) {
  const float2 te = cadd(x[0], x[4]), ue = csub(x[0], x[4]), ie = mul_i<SG>(x[2]);
  const float2 to = cadd(x[1], x[5]), uo = csub(x[1], x[5]), io = mul_i<SG>(x[3]);
  const float2 e0 = cadd(te, x[2]), e1 = cadd(ue, ie), e2 = csub(te, x[2]), e3 = csub(ue, ie);
  const float2 o0 = cadd(to, x[3]), o1 = cadd(uo, io), o2 = csub(to, x[3]), o3 = csub(uo, io);
  const float r = 0.70710678118654752440f;
  float2 t1, t3;
  if (SG > 0) {
    t1 = make_float2((o1.x - o1.y) * r, (o1.x + o1.y) * r);
    t3 = make_float2((-o3.x - o3.y) * r, (o3.x - o3.y) * r);
  } else {
    t1 = make_float2((o1.x + o1.y) * r, (o1.y - o1.x) * r);
    t3 = make_float2((o3.y - o3.x) * r, (-o3.x - o3.y) * r);
  }
  const float2 t2 = mul_i<SG>(o2);
  x[0] = cadd(e0, o0); x[4] = csub(e0, o0);
  x[1] = cadd(e1, t1); x[5] = csub(e1, t1);
  x[2] = cadd(e2, t2); x[6] = csub(e2, t2);
  x[3] = cadd(e3, t3); x[7] = csub(e3, t3);
}

// 8-point DFT whose inputs x[5], x[6], x[7] are zero (they are not read):
// dft8_six with the odd half's first butterfly (x[1], x[5]) reduced to x[1].
template <int SG> __device__ __forceinline__ void dft8_five(float2* x) {
  const float2 te = cadd(x[0], x[4]), ue = csub(x[0], x[4]), ie = mul_i<SG>(x[2]);
  const float2 io = mul_i<SG>(x[3]);
  const float2 e0 = cadd(te, x[2]), e1 = cadd(ue, ie), e2 = csub(te, x[2]), e3 = csub(ue, ie);
  const float2 o0 = cadd(x[1], x[3]), o1 = cadd(x[1], io), o2 = csub(x[1], x[3]), o3 = csub(x[1], io);
  const float r = 0.70710678118654752440f;
  float2 t1, t3;
  if (SG > 0) {
    t1 = make_float2((o1.x - o1.y) * r, (o1.x + o1.y) * r);
    t3 = make_float2((-o3.x - o3.y) * r, (o3.x - o3.y) * r);
  } else {
    t1 = make_float2((o1.x + o1.y) * r, (o1.y - o1.x) * r);
    t3 = make_float2((o3.y - o3.x) * r, (-o3.x - o3.y) * r);
  }
  const float2 t2 = mul_i<SG>(o2);
  x[0] = cadd(e0, o0); x[4] = csub(e0, o0);
  x[1] = cadd(e1, t1); x[5] = csub(e1, t1);
  x[2] = cadd(e2, t2); x[6] = csub(e2, t2);
  x[3] = cadd(e3, t3); x[7] = csub(e3, t3);
}

// 16-point DFT whose inputs x[8..15] are zero (they are not read): the 4 x 4
// form of dft16 with a first stage of two-input 4-point DFTs.
template <int SG> __device__ __forceinline__ void dft16_half(float2* x) {
  const float c1 = 0.92387953251128675613f;  // cos(pi/8)
  const float s1 = 0.38268343236508977173f;  // sin(pi/8)
  const float r = 0.70710678118654752440f;   // cos(pi/4)
  float2 y[16];
#pragma unroll
  for (int n0 = 0; n0 < 4; ++n0) {
    const float2 a = x[n0], b = x[4 + n0], ib = mul_i<SG>(b);   // inputs 8 + n0, 12 + n0 are zero
    y[n0] = cadd(a, b);
    y[4 + n0] = cadd(a, ib);
    y[8 + n0] = csub(a, b);
    y[12 + n0] = csub(a, ib);
  }
  const float2 w1 = make_float2(c1, SG * s1), w2 = make_float2(r, SG * r), w3 = make_float2(s1, SG * c1);
  const float2 w6 = make_float2(-r, SG * r), w9 = make_float2(-c1, -SG * s1);
  y[4 * 1 + 1] = cmul(y[5], w1);
  y[4 * 1 + 2] = cmul(y[6], w2);
  y[4 * 1 + 3] = cmul(y[7], w3);
  y[4 * 2 + 1] = cmul(y[9], w2);
  y[4 * 2 + 2] = mul_i<SG>(y[10]);
  y[4 * 2 + 3] = cmul(y[11], w6);
  y[4 * 3 + 1] = cmul(y[13], w3);
  y[4 * 3 + 2] = cmul(y[14], w6);
  y[4 * 3 + 3] = cmul(y[15], w9);
#pragma unroll
  for (int k0 = 0; k0 < 4; ++k0) {
    float2 a = y[4 * k0], b = y[4 * k0 + 1], c = y[4 * k0 + 2], d = y[4 * k0 + 3];
    dft4<SG>(a, b, c, d);
    x[k0] = a; x[k0 + 4] = b; x[k0 + 8] = c; x[k0 + 12] = d;
  }
}

template <int M, int SG> __device__ __forceinline__ void dft(float2* x) {
  if constexpr (M == 2) dft2<SG>(x[0], x[1]);
  else if constexpr (M == 4) dft4<SG>(x[0], x[1], x[2], x[3]);
  else if constexpr (M == 8) dft8<SG>(x);
  else if constexpr (M == 16) dft16<SG>(x);
  else static_assert(M == 2, "unsupported radix");
}

// Orders the LDS traffic of the lanes of one wave around a cross-lane exchange.
// A wave's LDS instructions execute in issue order, so a compiler barrier is
// enough: no workgroup barrier is needed for data private to one wave.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Shape of a length-N line transform done by R lanes holding S values each
// (N = R * S): pass 1 is an S-point DFT over the high digit n1 of
// n = R n1 + n0, then the twiddle w_N^(n0 k0), then D = S / R R-point DFTs
// over n0 per lane.
template <int N> struct Line;
template <> struct Line<32>  { static constexpr int S = 8,  R = 4, D = 2; };
template <> struct Line<64>  { static constexpr int S = 8,  R = 8, D = 1; };
template <> struct Line<128> { static constexpr int S = 16, R = 8, D = 2; };

// Forward or adjoint line transform of NP independent lines that share the
// lane role n0.  Slot s of line p is at lds + slot(p, s).
//   in:  v[p][n1] = x_p[R n1 + n0]                      (n1 < S)
//   out: v[p][q R + k1] = X_p[(n0 D + q) + S k1]        (q < D, k1 < R)
// tw[k0] = exp(+2 pi i n0 k0 / N) (conjugated here when SG < 0).
// The exchange between the passes goes through the line's own slots: value k0
// of lane n0 goes to slot k0 R + (n0 + SKEW k0) mod R, a skew chosen per
// access pattern so that the lanes of the exchange hit different LDS banks.
// NZ > 0: only the inputs n1 < NZ are nonzero (the others are not read);
// taken for NZ = S/2 (radix 8 and 16) and NZ = 5, 6 (radix 8).  NZ = 0: all.
template <int N, int SG, int NP, int NZ = 0, int SKEW = 1, typename SlotF>
__device__ __forceinline__ void line_transform(float2 (&v)[NP][Line<N>::S], const float2* tw,
                                               int n0, float2* lds, SlotF slot) {
  constexpr int S = Line<N>::S, R = Line<N>::R, D = Line<N>::D;
  static_assert(NZ == 0 || NZ == S || (NZ == S / 2 && (S == 8 || S == 16)) ||
                    ((NZ == 5 || NZ == 6) && S == 8),
                "zero-input forms implemented: half of radix 8 and 16, five and six of radix 8");
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    if constexpr (NZ == S / 2 && S == 8) dft8_half<SG>(v[p]);
    else if constexpr (NZ == S / 2) dft16_half<SG>(v[p]);
    else if constexpr (NZ == 6) dft8_six<SG>(v[p]);
    else if constexpr (NZ == 5) dft8_five<SG>(v[p]);
    else dft<S, SG>(v[p]);
#pragma unroll
    for (int k0 = 1; k0 < S; ++k0) v[p][k0] = twiddle_mul<SG>(v[p][k0], tw[k0]);
  }
  wave_lds_sync();
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int k0 = 0; k0 < S; ++k0) lds[slot(p, k0 * R + ((n0 + SKEW * k0) % R))] = v[p][k0];
  wave_lds_sync();
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const int k0 = n0 * D + q;
#pragma unroll
      for (int m = 0; m < R; ++m) v[p][q * R + m] = lds[slot(p, k0 * R + ((m + SKEW * k0) % R))];
    }
  wave_lds_sync();
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int q = 0; q < D; ++q) dft<R, SG>(&v[p][q * R]);
}

// Exact inverse route of line_transform with the conjugate sign: takes values
// in the output layout of line_transform and returns v[p][n1] = y_p[R n1 + n0]
// where y = sum_k X[k] exp(-2 pi i n k / N) (SG = -1) -- the adjoint of the
// forward line transform when applied to the forward's output positions.
template <int N, int SG, int NP, int SKEW = 1, typename SlotF>
__device__ __forceinline__ void line_transform_rev(float2 (&v)[NP][Line<N>::S], const float2* tw,
                                                   int n0, float2* lds, SlotF slot) {
  constexpr int S = Line<N>::S, R = Line<N>::R, D = Line<N>::D;
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int q = 0; q < D; ++q) dft<R, SG>(&v[p][q * R]);   // over k1 -> n0'
  wave_lds_sync();
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const int k0 = n0 * D + q;
#pragma unroll
      for (int m = 0; m < R; ++m) lds[slot(p, k0 * R + ((m + SKEW * k0) % R))] = v[p][q * R + m];
    }
  wave_lds_sync();
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int k0 = 0; k0 < S; ++k0) v[p][k0] = lds[slot(p, k0 * R + ((n0 + SKEW * k0) % R))];
  wave_lds_sync();
#pragma unroll
  for (int p = 0; p < NP; ++p) {
#pragma unroll
    for (int k0 = 1; k0 < S; ++k0) v[p][k0] = twiddle_mul<SG>(v[p][k0], tw[k0]);
    dft<S, SG>(v[p]);                                       // over k0 -> n1
  }
}

// The output order of dft<M> for M = 16 is natural (it reorders itself), and
// for M <= 8 the butterflies above already produce natural order.

}  // namespace epic
