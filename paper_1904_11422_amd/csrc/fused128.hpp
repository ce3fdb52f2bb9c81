// Fused imaging kernel for 128 x 128 grids (paper Sec. 2.1 Eq. (4)-(5),
// Sec. 3.2), the same per-sample path as fused_image_kernel with a different
// split of the work.
//
// With two polarisations the 64 x 64 aperture block fills most of the LDS,
// and the float32 sums of all 128 x 128 pixels would not fit the registers of
// one workgroup.  So a workgroup of 512 threads images the output columns of
// one parity h of a sample, kl = 2 m + h (m < 64):
//   1. unpack + gain, barrier, gridding of the whole aperture (wave-local rows,
//      as fused_image_kernel);
//   2. row transforms: a group of 8 lanes takes one aperture row of every
//      polarisation.  The row has 64 nonzero cells x[n], so its 128-point
//      transform at the columns of parity h is the 64-point transform of
//      x[n] w128^(n h):  X[2 m + h] = sum_n x[n] w128^(n h) w64^(n m).  A
//      radix-8 x 8 line transform writes the 64 values back to the row's
//      first 64 slots;  barrier;
//   3. column transforms: a group of 8 lanes takes one local column m of every
//      polarisation (128 points, the 64 aperture rows nonzero), exchanging
//      through the column's 64 aperture rows and the same rows' upper 64
//      columns; every lane then holds F_X (and F_Y) of 16 pixels;
//   4. XX (and YY, Re XY, Im XY) into float32 sums, added every KBLOCK samples
//      and at a segment boundary into the workgroup's float64 slot.
// Splitting the columns by parity instead of into two contiguous halves makes
// the two units' row transforms together cost one 128-point transform of the
// row: every row value is computed once per sample.  The gridding is still
// done by both units.
// One polarisation uses the same split: half the LDS (two workgroups per CU)
// and a quarter of the sums.
// Work units are (channel, parity, sample), flattened as ((2 c + h) T + t); a
// (channel, parity) pair is one accumulation segment.
#pragma once
#include "fused.hpp"

namespace epic {

// Launch arguments: FusedArgs (fused.hpp) with total = 2 C T units, C the
// launch's channels, and partial = [W + 2 C - 1][NACC][16][NT] (thread-major).

// Local pixel of float32 sum i of a thread: km = 2 n0 + q + 16 k1 with
// q = i >> 3 and k1 = i & 7; kl = the thread's local column (Roles::kl).
__host__ __device__ __forceinline__ int km128(int n0, int i) {
  return 2 * n0 + (i >> 3) + 16 * (i & 7);
}

// Image column of local column m of the unit of parity h.
__host__ __device__ __forceinline__ int kl128(int h, int m) { return 2 * m + h; }

// Two polarisations: one workgroup per CU (LDS), registers up to 256; one
// polarisation: two workgroups per CU, so at most 128 VGPRs.
template <int P> struct Fused128Waves { static constexpr int value = P == 2 ? 2 : 4; };

// MULTI: the launch walks several blocks (as fused_image_body).
template <int P, int GPT, bool CPX, bool MULTI>
__device__ __forceinline__ void fused_image128_body(const FusedArgs& a) {
  using SH = FusedShape<128>;
  constexpr int N = 128, S = SH::S, R = SH::R, NT = SH::NT, RS = SH::RS, PS = SH::PSTRIDE;
  constexpr int NACC = P == 2 ? 4 : 1, H = N / 2, NPX = 16;
  constexpr int ES = EStride<NT, GPT, P>::value;
  constexpr int XBASE = P * ES * (int)sizeof(float2);
  // E'[p][a] (zero slots at a = A .. A+15), the grid (64 rows per
  // polarisation), then the twiddles w128^(n0 k0) of the 8 lane roles n0 in
  // rows of 17 (the roles of a half-wave read distinct banks), the twiddles
  // w64^(n0 k0) = w128^(2 n0 k0) in rows of 9, and w128^n (n < 64), the
  // factor of the odd columns' row transform
  constexpr int TWS = 17, TW64S = 9;
  __shared__ float2 lds2[P * ES + (P - 1) * PS + H * RS + R * TWS + R * TW64S + H];
  char* lds = reinterpret_cast<char*>(lds2);
  float2* E = lds2;
  float2* X = lds2 + P * ES;
  float2* TW = X + (P - 1) * PS + H * RS;
  float2* TW64 = TW + R * TWS;
  float2* ODD = TW64 + R * TW64S;

  const Roles<N> r(threadIdx.x);
  const int tid = r.tid;
  const int wl = wg_range_index((int)blockIdx.x, (int)gridDim.x, a.xcd);
  const int m = a.team, tm = wl / m, mk = wl - tm * m, n_team = a.W / m;
  UnitWalk it;
  it.T = a.n_time;
  it.ra = range_begin(tm, a.total, n_team);
  it.rb = range_begin(tm + 1, a.total, n_team);
  it.m = m;
  it.k = mk;
  if (tm >= n_team || !it.seek(it.ra / a.n_time)) return;
  const int64_t n_units = member_units(a.n_time, it.ra, it.rb, m, mk);

  if (tid < R * S) TW[(tid / S) * TWS + tid % S] = a.twiddle[((tid / S) * (tid % S)) % N];
  if (tid < R * 8) TW64[(tid / 8) * TW64S + tid % 8] = a.twiddle[(2 * (tid / 8) * (tid % 8)) % N];
  if (tid < H) ODD[tid] = a.twiddle[tid];
  const float2* tw = TW + r.n0 * TWS;          // read after the first barrier
  const float2* tw64 = TW64 + r.n0 * TW64S;

  // block of the unit being prefetched (nb) and of the one being imaged (b)
  int nb = MULTI ? block_of(a, (int)(it.s >> 1)) : 0;
  int b = nb;
  int PA = P * a.blk[b].n_ant;
  int L = a.blk[b].L, Lw = L;                  // L: of block b; Lw: of this wave
  const int KB = a.kblock;
  int64_t n_row = (int64_t)a.blk[nb].n_chan * P * a.blk[nb].n_ant;
  int n_pa = P * a.blk[nb].n_ant, n_c0 = a.blk[nb].c0;
  const uint8_t* n_src = a.blk[nb].efield;
  int eidx[GPT];
  init_stage<NT, GPT, ES>(E, eidx, tid, a.blk[b].n_ant, P);

  float acc[NPX][NACC];
  float2 g[GPT];
  uint32_t nxt[GPT];
  int seg = -1, nblk = 0, nflush = 0, line = -1, h = 0;
  int64_t part_len = 0, slot = 0;
  const uint2* prog = nullptr;
  const float* wim = nullptr;

  auto load_bytes = [&](int64_t sgm, int64_t t, uint32_t (&dst)[GPT]) {
    const uint8_t* src = n_src + t * n_row + ((sgm >> 1) - n_c0) * n_pa;
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int k = tid + i * NT;
      dst[i] = (k < n_pa) ? (uint32_t)src[k] : 0u;
    }
  };
  // the float32 sums of the current part into its slot: written once as
  // float32 if the part fits one block, else added in float64
  auto flush = [&]() {
    if (part_len <= KB) {
      float* o32 = reinterpret_cast<float*>(a.partial + slot * (NACC * NPX * NT)) + tid;
#pragma unroll
      for (int u = 0; u < NACC; ++u)
#pragma unroll
        for (int i = 0; i < NPX; ++i) {
          o32[(u * NPX + i) * NT] = acc[i][u];
          acc[i][u] = 0.f;
        }
    } else {
      double* out = a.partial + slot * (NACC * NPX * NT) + tid;
#pragma unroll
      for (int u = 0; u < NACC; ++u)
#pragma unroll
        for (int i = 0; i < NPX; ++i) {
          double* o = out + (u * NPX + i) * NT;
          *o = (nflush ? *o : 0.0) + (double)acc[i][u];
          acc[i][u] = 0.f;
        }
    }
    ++nflush;
    nblk = 0;
  };

  load_bytes(it.s, it.t, nxt);
  for (int64_t left = n_units; left > 0; --left) {
    const int64_t sg = it.s;                   // segment 2 c + h of the current unit
    if ((int)sg != seg) {                      // a part (accumulation segment) starts
      if (seg >= 0) flush();
      const int c_old = seg >> 1;
      seg = (int)sg;
      const int c = seg >> 1;
      h = seg & 1;
      nflush = 0;
      part_len = it.left;
      slot = (sg + tm) * m + mk;
#pragma unroll
      for (int i = 0; i < NPX; ++i)
#pragma unroll
        for (int u = 0; u < NACC; ++u) acc[i][u] = 0.f;
      if (c != c_old) {
        if (MULTI && nb != b) {                // a new block: its antennas' E' layout
          b = nb;
          PA = P * a.blk[b].n_ant;
          L = a.blk[b].L;
          init_stage<NT, GPT, ES>(E, eidx, tid, a.blk[b].n_ant, P);
        }
        const int64_t cl = c - a.blk[b].c0;
        prog = a.blk[b].prog + cl * (L + 1) * NT;
        if (CPX) wim = a.blk[b].wim + cl * (L + 1) * NT + NT;
        line = (int)prog[tid].x;
        Lw = header_steps(prog[tid].y, L);
        prog += NT;
#pragma unroll
        for (int i = 0; i < GPT; ++i) {
          const int k = tid + i * NT;
          g[i] = (k < PA) ? a.blk[b].gains[cl * PA + k] : make_float2(0.f, 0.f);
        }
      }
    } else if (nblk == KB) {
      flush();
    }
    uint32_t cur[GPT];
#pragma unroll
    for (int i = 0; i < GPT; ++i) cur[i] = nxt[i];
    it.next();                                 // advance, prefetch the next unit
    if (left > 1) {
      if (MULTI && (it.s >> 1) != (sg >> 1)) {  // the next part may be in another block
        const int nnb = block_of(a, (int)(it.s >> 1));
        if (nnb != nb) {
          nb = nnb;
          n_row = (int64_t)a.blk[nb].n_chan * P * a.blk[nb].n_ant;
          n_pa = P * a.blk[nb].n_ant;
          n_c0 = a.blk[nb].c0;
          n_src = a.blk[nb].efield;
        }
      }
      load_bytes(it.s, it.t, nxt);
    }

    // 1. stage and grid the aperture (both parities grid the whole aperture)
    stage_and_grid<N, P, NT, RS, ES, GPT, CPX>(lds, lds + XBASE, E, prog, wim, Lw, cur, g, eidx, tid, PA);
    // 2. row transforms of row `line` of both polarisations onto the
    //    columns of parity h (h is uniform over the workgroup)
    if (line >= 0) {
      const int rb = (line & 0xFFFF) * RS;
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
      // v[p][k1] = X_p[2 (n0 + 8 k1) + h]
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) X[p * PS + rb + r.n0 + 8 * k1] = v[p][k1];
    }
    __syncthreads();

    // 3. column transforms of local column r.kl of both polarisations
    const int kl = r.kl;
    float2 v[P][S];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int n1 = 0; n1 < S / 2; ++n1) v[p][n1] = X[p * PS + (R * n1 + r.n0) * RS + kl];
    line_transform<N, +1, P, Line<N>::S / 2>(v, tw, r.n0, X,
                                   [kl](int p, int s) { return p * PS + (s & 63) * RS + kl + (s & 64); });
    // v[p][q R + k1] = F_p[2 n0 + q + 16 k1][2 kl + h]

    // 4. products of the 16 pixels: XX (, YY, Re XY, Im XY; XY = F_X conj(F_Y))
#pragma unroll
    for (int i = 0; i < NPX; ++i) {
      const float2 fx = v[0][i];
      acc[i][0] = fmaf(fx.y, fx.y, fmaf(fx.x, fx.x, acc[i][0]));
      if (P == 2) {
        const float2 fy = v[P - 1][i];
        acc[i][1 % NACC] = fmaf(fy.y, fy.y, fmaf(fy.x, fy.x, acc[i][1 % NACC]));
        acc[i][2 % NACC] = fmaf(fx.y, fy.y, fmaf(fx.x, fy.x, acc[i][2 % NACC]));
        acc[i][3 % NACC] = fmaf(-fx.x, fy.y, fmaf(fx.y, fy.x, acc[i][3 % NACC]));
      }
    }
    ++nblk;
  }
  flush();
}


template <int P, int GPT, bool CPX>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(Fused128Waves<P>::value)))
fused_image128_kernel(FusedArgs a) {
  fused_image128_body<P, GPT, CPX, false>(a);
}

// The heterogeneous batch: one launch over the channels of several 128 x 128 blocks.
template <int P, int GPT>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(Fused128Waves<P>::value)))
fused_multi_image128_kernel(FusedArgs a) {
  fused_image128_body<P, GPT, false, true>(a);
}

// image[c][prod][qm][ql] (+)= sum of the slots of segment 2 c + h, for the
// pixels of columns of parity h; sub-lanes as reduce_image_kernel.
struct Reduce128Args {
  const double* partial;
  // complex128 [C_b][NPROD][128][128] per block of the launch (as ReduceArgs)
  double* image[kMaxLaunchBlocks];
  int img_c0[kMaxLaunchBlocks];
  int n_img;
  int64_t n_time, total;
  int n_chan, W, reset, sub;   // n_chan: all channels of the launch
  int team, kblock;            // the imaging launch's partition (FusedArgs)
};

template <int P>
__global__ void __launch_bounds__(256) reduce_image128_kernel(Reduce128Args a) {
  constexpr int N = 128, NT = FusedShape<128>::NT, NLOC = 16 * NT;   // local pixels per parity
  constexpr int NACC = P == 2 ? 4 : 1, NPROD = P == 2 ? 4 : 1;
  __shared__ double red[NACC * 256];
  const int ppb = 256 / a.sub;
  const int j = threadIdx.x / ppb, lp = threadIdx.x % ppb;
  const int64_t idx = (int64_t)blockIdx.x * ppb + lp;
  const bool valid = idx < (int64_t)a.n_chan * 2 * NLOC;
  const int sgm = valid ? (int)(idx / NLOC) : 0;            // 2 c + h
  const int pix = (int)(idx % NLOC);                        // i * NT + tid
  double s[NACC];
#pragma unroll
  for (int u = 0; u < NACC; ++u) s[u] = 0.0;
  if (valid)
    sum_parts<NACC>(a.partial, sgm, a.n_time, a.total, a.W, a.team, a.kblock, 1, (int64_t)NACC * NLOC, NLOC,
                    pix, j, a.sub, s);
  combine_sublanes<NACC>(s, a.sub, ppb, j, lp, red);
  if (!valid || j != 0) return;
  const int tid = pix % NT, i = pix / NT;
  const Roles<N> r(tid);
  const int c = sgm >> 1, h = sgm & 1;
  const int km = km128(r.n0, i), kl = kl128(h, r.kl);
  const int qm = (km + N / 2) % N, ql = (kl + N / 2) % N;
  int b = 0;                                 // the image of channel c
  for (int bi = 1; bi < a.n_img; ++bi)
    if (a.img_c0[bi] <= c) b = bi;
  double2* img = reinterpret_cast<double2*>(a.image[b]);
  const int64_t base = (int64_t)(c - a.img_c0[b]) * NPROD * N * N + qm * N + ql;
  double2 val[NPROD];
  val[0] = make_double2(s[0], 0.0);
  if (P == 2) {
    val[1 % NPROD] = make_double2(s[2 % NACC], s[3 % NACC]);
    val[2 % NPROD] = make_double2(s[2 % NACC], -s[3 % NACC]);
    val[3 % NPROD] = make_double2(s[1 % NACC], 0.0);
  }
#pragma unroll
  for (int pr = 0; pr < NPROD; ++pr) {
    double2* o = img + base + (int64_t)pr * N * N;
    if (a.reset) {
      *o = val[pr];
    } else {
      const double2 old = *o;
      *o = make_double2(old.x + val[pr].x, old.y + val[pr].y);
    }
  }
}

}  // namespace epic
