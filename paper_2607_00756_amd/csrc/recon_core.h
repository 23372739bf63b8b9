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

// The six padded parent values of one target beam at pixel rr.
__device__ inline void recon_load(const float2* __restrict__ win, int W2, int rr, const int32_t* ec,
                                  float2 (&D)[ELL_K]) {
#pragma unroll
  for (int j = 0; j < ELL_K; ++j) D[j] = win[(int64_t)ec[j] * W2 + rr];
}

// Combination of loaded parent values (see recon_combine).
__device__ inline float2 recon_finish(const float2 (&D)[ELL_K], const float2* __restrict__ win,
                                      int W2, int rr, const int32_t* ec, const float* ew,
                                      const int32_t* __restrict__ col,
                                      const float* __restrict__ w, int mode) {
  float2 z = make_float2(0.f, 0.f);
  float m = 0.f;
#pragma unroll
  for (int j = 0; j < ELL_K; ++j) {
    const float wj = ew[j];
    z.x += wj * D[j].x;
    z.y += wj * D[j].y;
    m += wj * sqrtf(D[j].x * D[j].x + D[j].y * D[j].y);
  }
  const int cnt = ec[6], lo = ec[7];
  for (int j = lo + ELL_K; j < lo + cnt; ++j) {
    const float2 Dj = win[(int64_t)col[j] * W2 + rr];
    const float wj = w[j];
    z.x += wj * Dj.x;
    z.y += wj * Dj.y;
    m += wj * sqrtf(Dj.x * Dj.x + Dj.y * Dj.y);
  }
  if (mode == BIP_RECON_MAGNITUDE) {
    const float az = sqrtf(z.x * z.x + z.y * z.y);
    return az > 0.f ? cscale(z, m / az) : make_float2(0.f, 0.f);
  }
  return z;
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
    m += wj * sqrtf(D[j].x * D[j].x + D[j].y * D[j].y);
  }
  const int cnt = ec[6], lo = ec[7];
  for (int j = lo + ELL_K; j < lo + cnt; ++j) {
    const float2 Dj = win[(int64_t)col[j] * W2 + rr];
    const float wj = w[j];
    z.x += wj * Dj.x;
    z.y += wj * Dj.y;
    m += wj * sqrtf(Dj.x * Dj.x + Dj.y * Dj.y);
  }
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
