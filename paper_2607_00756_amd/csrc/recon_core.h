// Natural-neighbour combination of de-tilted parent windows (step b), shared
// by the reconstruction kernels and the probe fold.
//
// The weights of a target beam are read from a padded ("ELL") copy of the
// CSR rows: slots 0..5 hold parent index and weight (index 0, weight 0 when
// the row is shorter), slot 6 the row length and slot 7 the row start in the
// CSR.  All six parent reads are issued unconditionally, so they are in flight
// together; rows longer than six (not produced by square-lattice Sibson
// weights) continue from the CSR.
#pragma once

#include "bip_internal.h"

namespace bip {

constexpr int ELL_W = 8;  // int32 / float entries per padded row
constexpr int ELL_K = 6;  // weights held in the padded row
constexpr int TILE_B = 64;   // target beams per reconstruction tile
constexpr int TILE_NP = 64;  // parents of a tile that fit the LDS slab

// The six padded parent values of one target beam at pixel rr.
__device__ inline void recon_load(const float2* __restrict__ win, int W2, int rr, const int32_t* ec,
                                  float2 (&D)[ELL_K]) {
#pragma unroll
  for (int j = 0; j < ELL_K; ++j) D[j] = win[(int64_t)ec[j] * W2 + rr];
}

// |v| with the hardware square root (within 1 ulp, no denormal rescaling).
__device__ inline float habs(float2 v) { return __builtin_amdgcn_sqrtf(v.x * v.x + v.y * v.y); }

// m z/|z| (eq. magpreserve), 0 where z = 0.  The hardware reciprocal square
// root (within 1 ulp) serves every |z|^2 above 1e-30; smaller ones take the
// correctly rounded square root and division.
__device__ inline float2 mag_rescale(float2 z, float m) {
  const float q = z.x * z.x + z.y * z.y;
  if (q >= 1e-30f) return cscale(z, m * __builtin_amdgcn_rsqf(q));
  const float az = sqrtf(q);
  return az > 0.f ? cscale(z, m / az) : make_float2(0.f, 0.f);
}

// Parents beyond the six padded slots of a row (rows longer than six), read
// from the CSR and added to z and m.
__device__ inline void recon_tail(float2& z, float& m, const float2* __restrict__ win, int W2, int rr,
                                  const int32_t* ec, const int32_t* __restrict__ col,
                                  const float* __restrict__ w) {
  const int cnt = ec[6], lo = ec[7];
  for (int j = lo + ELL_K; j < lo + cnt; ++j) {
    const float2 Dj = win[(int64_t)col[j] * W2 + rr];
    const float wj = w[j];
    z.x += wj * Dj.x;
    z.y += wj * Dj.y;
    m += wj * habs(Dj);
  }
}

// z and m of one target beam from loaded parent values (the intermediates of
// the reconstruction that its adjoint needs).
__device__ inline void recon_zm(const float2 (&D)[ELL_K], const float2* __restrict__ win, int W2,
                                int rr, const int32_t* ec, const float* ew,
                                const int32_t* __restrict__ col, const float* __restrict__ w,
                                float2& z, float& m) {
  z = make_float2(0.f, 0.f);
  m = 0.f;
#pragma unroll
  for (int j = 0; j < ELL_K; ++j) {
    const float wj = ew[j];
    z.x += wj * D[j].x;
    z.y += wj * D[j].y;
    m += wj * habs(D[j]);
  }
  recon_tail(z, m, win, W2, rr, ec, col, w);
}

// Combination of loaded parent values (see recon_combine).
__device__ inline float2 recon_finish(const float2 (&D)[ELL_K], const float2* __restrict__ win,
                                      int W2, int rr, const int32_t* ec, const float* ew,
                                      const int32_t* __restrict__ col,
                                      const float* __restrict__ w, int mode) {
  float2 z;
  float m;
  recon_zm(D, win, W2, rr, ec, ew, col, w, z, m);
  return mode == BIP_RECON_MAGNITUDE ? mag_rescale(z, m) : z;
}

// z = sum_p w_p D_p(r), m = sum_p w_p |D_p(r)| (eq. window-recon); returns
// m z/|z| in magnitude mode (eq. magpreserve, 0 where z = 0) or z.
__device__ inline float2 recon_combine(const float2* __restrict__ win, int W2, int rr,
                                       const int32_t* ec, const float* ew,
                                       const int32_t* __restrict__ col,
                                       const float* __restrict__ w, int mode) {
  float2 D[ELL_K];
  recon_load(win, W2, rr, ec, D);
  return recon_finish(D, win, W2, rr, ec, ew, col, w, mode);
}

}  // namespace bip
