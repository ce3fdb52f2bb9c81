// Front end of the imager (paper Sec. 3.2 and Fig. 2): the channelised bytes
// arrive as [Time, Channel, Antenna, Polarisation]; they are decimated in
// frequency (output channel i = input channel c0 + i * c_step) and transposed
// to [Time, Channel, Polarisation, Antenna], the order in which the imaging
// kernels read whole rows of antennas.  Bytes are moved, never changed.
//
// One pass over HBM: every selected byte is read once and written once.  A
// thread takes eight antennas of one (t, c): one 16-byte load of the
// interleaved pairs (X0 Y0 X1 Y1 ... X7 Y7), two byte permutes, and one
// 8-byte store into each polarisation's row.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace epic {

struct FrontendArgs {
  const uint8_t* raw;       // [T][c_in][A][P]
  uint8_t* efield;          // [T][C][P][A]
  int64_t n_rows;           // T * C
  int c_in, n_chan, c0, c_step, n_ant;
};

// VEC = 8: A % 8 == 0, raw 16-byte and efield 8-byte aligned; VEC = 1: any.
template <int P, int VEC>
__global__ void __launch_bounds__(256) frontend_kernel(FrontendArgs a) {
  const int gpr = a.n_ant / VEC;              // groups of VEC antennas per row
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= a.n_rows * gpr) return;
  const int64_t row = idx / gpr;
  const int g = (int)(idx - row * gpr);
  const int64_t t = row / a.n_chan;
  const int c = (int)(row - t * a.n_chan);
  const int64_t ch = t * a.c_in + a.c0 + (int64_t)c * a.c_step;
  const uint8_t* src = a.raw + (ch * a.n_ant + (int64_t)g * VEC) * P;
  uint8_t* dst = a.efield + row * P * a.n_ant + (int64_t)g * VEC;
  if constexpr (VEC == 8 && P == 2) {
    const uint4 w = *reinterpret_cast<const uint4*>(src);
    uint2 x, y;
    x.x = __builtin_amdgcn_perm(w.y, w.x, 0x06040200u);   // bytes 0 2 4 6: X of antennas 0..3
    x.y = __builtin_amdgcn_perm(w.w, w.z, 0x06040200u);
    y.x = __builtin_amdgcn_perm(w.y, w.x, 0x07050301u);   // bytes 1 3 5 7: Y
    y.y = __builtin_amdgcn_perm(w.w, w.z, 0x07050301u);
    *reinterpret_cast<uint2*>(dst) = x;
    *reinterpret_cast<uint2*>(dst + a.n_ant) = y;
  } else if constexpr (VEC == 8) {
    *reinterpret_cast<uint2*>(dst) = *reinterpret_cast<const uint2*>(src);
  } else {
#pragma unroll
    for (int p = 0; p < P; ++p) dst[(int64_t)p * a.n_ant] = src[p];
  }
}

}  // namespace epic
