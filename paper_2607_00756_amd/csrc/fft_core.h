// Register/LDS Stockham FFT used by the multislice passes.
//
// A transform of length N (power of two, 64..1024) is carried by N/16
// threads holding 16 elements each.  Between stages a thread holds the
// "strided" layout: thread t owns elements t + (N/16) e, e = 0..15.  A stage
// of radix R performs 16/R butterflies per thread on elements spaced N/R
// apart (these are exactly its registers), applies the Stockham twiddles
// exp(-/+ 2 pi i j k/(p R)) (p = product of the earlier radices), and writes
// the result to y[(i/p) p R + (i mod p) + j p]; after the last stage the data
// is in natural order and already in the strided layout, so the final stage
// needs no LDS exchange.  Radix plans: 64 = 16*4, 128 = 16*8, 256 = 16*16,
// 512 = 16*16*2, 1024 = 16*16*4.
#pragma once

#include "bip_internal.h"

namespace bip {
namespace fft {

constexpr float kSqrtHalf = 0.70710678118654752f;
constexpr float kC16_1 = 0.92387953251128674f;  // cos(pi/8)
constexpr float kS16_1 = 0.38268343236508978f;  // sin(pi/8)

// multiply by exp(-i theta) (forward) or exp(+i theta) (inverse), given
// (cos theta, sin theta)
template <bool INV>
__device__ inline float2 rot(float2 a, float c, float s) {
  return INV ? make_float2(a.x * c - a.y * s, a.x * s + a.y * c)
             : make_float2(a.x * c + a.y * s, a.y * c - a.x * s);
}

// multiply by -i (forward) / +i (inverse)
template <bool INV>
__device__ inline float2 mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ inline void dft2(float2& a, float2& b) {
  float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <bool INV>
__device__ inline void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  float2 a = cadd(x0, x2), b = csub(x0, x2), c = cadd(x1, x3), d = mi<INV>(csub(x1, x3));
  x0 = cadd(a, c);
  x2 = csub(a, c);
  x1 = cadd(b, d);
  x3 = csub(b, d);
}

// natural order in, natural order out
template <int R, bool INV>
__device__ inline void dft(float2* u);

template <>
__device__ inline void dft<2, false>(float2* u) { dft2<false>(u[0], u[1]); }
template <>
__device__ inline void dft<2, true>(float2* u) { dft2<true>(u[0], u[1]); }

template <bool INV>
__device__ inline void dft4n(float2* u) {
  dft4<INV>(u[0], u[1], u[2], u[3]);
}
template <>
__device__ inline void dft<4, false>(float2* u) { dft4n<false>(u); }
template <>
__device__ inline void dft<4, true>(float2* u) { dft4n<true>(u); }

// 8 = 4 x 2: n = 2 n1 + n2, k = k1 + 4 k2
template <bool INV>
__device__ inline void dft8n(float2* u) {
  float2 a0 = u[0], a1 = u[2], a2 = u[4], a3 = u[6];
  float2 b0 = u[1], b1 = u[3], b2 = u[5], b3 = u[7];
  dft4<INV>(a0, a1, a2, a3);
  dft4<INV>(b0, b1, b2, b3);
  b1 = rot<INV>(b1, kSqrtHalf, kSqrtHalf);
  b2 = mi<INV>(b2);
  b3 = rot<INV>(b3, -kSqrtHalf, kSqrtHalf);
  u[0] = cadd(a0, b0); u[4] = csub(a0, b0);
  u[1] = cadd(a1, b1); u[5] = csub(a1, b1);
  u[2] = cadd(a2, b2); u[6] = csub(a2, b2);
  u[3] = cadd(a3, b3); u[7] = csub(a3, b3);
}
template <>
__device__ inline void dft<8, false>(float2* u) { dft8n<false>(u); }
template <>
__device__ inline void dft<8, true>(float2* u) { dft8n<true>(u); }

// 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2; twiddle w16^(n2 k1)
template <bool INV>
__device__ inline void dft16n(float2* u) {
  float2 y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    y[n2][0] = u[n2];
    y[n2][1] = u[4 + n2];
    y[n2][2] = u[8 + n2];
    y[n2][3] = u[12 + n2];
    dft4<INV>(y[n2][0], y[n2][1], y[n2][2], y[n2][3]);
  }
  // n2 = 1: k1 = 1,2,3 -> angles pi/8, pi/4, 3pi/8
  y[1][1] = rot<INV>(y[1][1], kC16_1, kS16_1);
  y[1][2] = rot<INV>(y[1][2], kSqrtHalf, kSqrtHalf);
  y[1][3] = rot<INV>(y[1][3], kS16_1, kC16_1);
  // n2 = 2: angles pi/4, pi/2, 3pi/4
  y[2][1] = rot<INV>(y[2][1], kSqrtHalf, kSqrtHalf);
  y[2][2] = mi<INV>(y[2][2]);
  y[2][3] = rot<INV>(y[2][3], -kSqrtHalf, kSqrtHalf);
  // n2 = 3: angles 3pi/8, 3pi/4, 9pi/8
  y[3][1] = rot<INV>(y[3][1], kS16_1, kC16_1);
  y[3][2] = rot<INV>(y[3][2], -kSqrtHalf, kSqrtHalf);
  y[3][3] = rot<INV>(y[3][3], -kC16_1, -kS16_1);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 a = y[0][k1], b = y[1][k1], c = y[2][k1], d = y[3][k1];
    dft4<INV>(a, b, c, d);
    u[k1] = a;
    u[k1 + 4] = b;
    u[k1 + 8] = c;
    u[k1 + 12] = d;
  }
}
template <>
__device__ inline void dft<16, false>(float2* u) { dft16n<false>(u); }
template <>
__device__ inline void dft<16, true>(float2* u) { dft16n<true>(u); }

// LDS addressing of element idx of one transform: base[idx*STRIDE (+ idx/16)]
template <int STRIDE, bool PAD>
__device__ inline int lds_index(int idx) {
  return idx * STRIDE + (PAD ? (idx >> 4) : 0);
}

// Orders the LDS exchange of a stage.  WAVE: every transform lives inside one
// wavefront (its N/16 lanes are consecutive lanes of one wave), whose LDS
// instructions execute in issue order, so keeping the compiler from moving
// LDS accesses across this point is enough; otherwise a workgroup barrier.
template <bool WAVE>
__device__ inline void exchange_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// One Stockham stage.  v: strided-layout registers.  tw: exp(-2 pi i m/L)
// table; twstep = L / N.
template <int N, int R, int P, bool LAST, bool INV, int STRIDE, bool PAD, bool WAVE = false>
__device__ inline void stage(float2 (&v)[16], float2* lds, int t, const float2* __restrict__ tw,
                             int twstep) {
  constexpr int T = N / 16;
  constexpr int NB = 16 / R;
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    const int i = t + T * m;
    const int k = i & (P - 1);
    float2 u[R];
#pragma unroll
    for (int j = 0; j < R; ++j) u[j] = v[m + j * NB];
    if (P > 1) {
#pragma unroll
      for (int j = 1; j < R; ++j) {
        const float2 w = tw[(j * k * (N / (P * R))) * twstep];
        u[j] = INV ? cmulc(u[j], w) : cmul(u[j], w);
      }
    }
    dft<R, INV>(u);
    if (LAST) {
#pragma unroll
      for (int j = 0; j < R; ++j) v[m + j * NB] = u[j];
    } else {
      const int j0 = (i / P) * P * R + k;
#pragma unroll
      for (int j = 0; j < R; ++j) lds[lds_index<STRIDE, PAD>(j0 + j * P)] = u[j];
    }
  }
  if (!LAST) {
    exchange_sync<WAVE>();
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = lds[lds_index<STRIDE, PAD>(t + T * e)];
    exchange_sync<WAVE>();
  }
}

// Full transform (unnormalized; inverse uses exp(+2 pi i ...)).  WAVE: see
// exchange_sync (STRIDE 1 with N/16 consecutive lanes per transform).
template <int N, bool INV, int STRIDE, bool PAD, bool WAVE = false>
__device__ inline void transform(float2 (&v)[16], float2* lds, int t, const float2* tw, int L) {
  static_assert(!WAVE || (STRIDE == 1 && N / 16 <= 64), "a wave-synchronized transform must fit one wave");
  const int twstep = L / N;
  if constexpr (N == 64) {
    stage<64, 16, 1, false, INV, STRIDE, PAD, WAVE>(v, lds, t, tw, twstep);
    stage<64, 4, 16, true, INV, STRIDE, PAD, WAVE>(v, lds, t, tw, twstep);
  } else if constexpr (N == 128) {
    stage<128, 16, 1, false, INV, STRIDE, PAD, WAVE>(v, lds, t, tw, twstep);
    stage<128, 8, 16, true, INV, STRIDE, PAD, WAVE>(v, lds, t, tw, twstep);
  } else if constexpr (N == 256) {
    stage<256, 16, 1, false, INV, STRIDE, PAD, WAVE>(v, lds, t, tw, twstep);
    stage<256, 16, 16, true, INV, STRIDE, PAD, WAVE>(v, lds, t, tw, twstep);
  } else if constexpr (N == 512) {
    stage<512, 16, 1, false, INV, STRIDE, PAD, WAVE>(v, lds, t, tw, twstep);
    stage<512, 16, 16, false, INV, STRIDE, PAD, WAVE>(v, lds, t, tw, twstep);
    stage<512, 2, 256, true, INV, STRIDE, PAD, WAVE>(v, lds, t, tw, twstep);
  } else {
    static_assert(N == 1024, "unsupported FFT length");
    stage<1024, 16, 1, false, INV, STRIDE, PAD, WAVE>(v, lds, t, tw, twstep);
    stage<1024, 16, 16, false, INV, STRIDE, PAD, WAVE>(v, lds, t, tw, twstep);
    stage<1024, 4, 256, true, INV, STRIDE, PAD, WAVE>(v, lds, t, tw, twstep);
  }
}

}  // namespace fft
}  // namespace bip
