// Complex contraction on the matrix cores (step c).
//
// Both contractions are "NT" complex products C[m][n] = sum_k A[m][k] B[n][k]
// with K contiguous in both operands, stored as separate real planes:
//   FP32        : re, im                         (v_mfma_f32_16x16x4_f32)
//   SPLIT_BF16  : re_hi, re_lo, im_hi, im_lo      (v_mfma_f32_16x16x32_bf16,
//                 hi*hi + hi*lo + lo*hi per real product, FP32 accumulate)
//   BF16        : re, im                         (v_mfma_f32_16x16x32_bf16)
// A complex product is four real products (re*re - im*im, re*im + im*re);
// the minus sign is applied by flipping the sign of the A imaginary
// fragment.  A workgroup of 4 wave64s owns a 128 x 128 output tile, each
// wave a 64 x 64 sub-tile of 4 x 4 MFMA blocks; K advances in chunks staged
// through LDS with the next chunk prefetched into registers.
//
// Probe synthesis (eq. coupling, probe order): psi^T[rho][r] =
//   sum_b c_b(rho) S1~^b(r); the epilogue multiplies by H_n(r) for every
//   channel and writes U_n[rho][r] directly in the operand format of the
//   detector contraction.
// Detector contraction: A[d][rho] = sum_r S2~^d(r) U_n(r, rho); the epilogue
//   accumulates |A|^2 over the (atom, channel) jobs of the launch in
//   registers and then reduces over d (map) or adds into [rho][d] (beams).
#include "bip_internal.h"

namespace bip {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

template <int PREC>
struct PT;
template <>
struct PT<BIP_PREC_FP32> {
  static constexpr int PLANES = 2, ESZ = 4, BK = 16, PITCH = 20;  // elements
};
template <>
struct PT<BIP_PREC_SPLIT_BF16> {
  static constexpr int PLANES = 4, ESZ = 2, BK = 32, PITCH = 40;
};
template <>
struct PT<BIP_PREC_BF16> {
  static constexpr int PLANES = 2, ESZ = 2, BK = 32, PITCH = 40;
};

constexpr int BM = 128, BN = 128, NTHREADS = 256;

__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline v8bf neg8(v8bf a) {
  v4u u = __builtin_bit_cast(v4u, a);
  u ^= 0x80008000u;
  return __builtin_bit_cast(v8bf, u);
}

// Stage one K chunk of a 128-row operand tile (all planes) into registers.
// Each plane-row is 64 bytes = 4 x 16-byte segments; 512 segments per plane.
template <int PREC>
struct Stage {
  static constexpr int P = PT<PREC>::PLANES;
  uint4 r[P][2];

  __device__ inline void load(const char* base, int64_t plane_bytes, int64_t ld_bytes, int k0_bytes,
                              int tid) {
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int c = tid + NTHREADS * i;
        const int row = c >> 2, seg = c & 3;
        r[p][i] = *(const uint4*)(base + p * plane_bytes + row * ld_bytes + k0_bytes + seg * 16);
      }
  }
  __device__ inline void store(char* lds, int tid) const {
    constexpr int ROWB = PT<PREC>::PITCH * PT<PREC>::ESZ;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int c = tid + NTHREADS * i;
        const int row = c >> 2, seg = c & 3;
        *(uint4*)(lds + (p * 128 + row) * ROWB + seg * 16) = r[p][i];
      }
  }
};

struct Acc {
  v4f re[4][4], im[4][4];
  __device__ inline void zero() {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        re[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
        im[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
      }
  }
};

// Multiply the LDS-resident chunk into the accumulators.
template <int PREC>
__device__ inline void mma_chunk(const char* sA, const char* sB, int wm, int wn, int lane, Acc& acc) {
  constexpr int ROWB = PT<PREC>::PITCH * PT<PREC>::ESZ;
  const int lr = lane & 15, kg = lane >> 4;
  if constexpr (PREC == BIP_PREC_FP32) {
    float4 bR[4], bI[4];
#pragma unroll
    for (int bn = 0; bn < 4; ++bn) {
      const int row = wn * 64 + bn * 16 + lr;
      bR[bn] = *(const float4*)(sB + (0 * 128 + row) * ROWB + kg * 16);
      bI[bn] = *(const float4*)(sB + (1 * 128 + row) * ROWB + kg * 16);
    }
#pragma unroll
    for (int bm = 0; bm < 4; ++bm) {
      const int row = wm * 64 + bm * 16 + lr;
      const float4 aR = *(const float4*)(sA + (0 * 128 + row) * ROWB + kg * 16);
      const float4 aI = *(const float4*)(sA + (1 * 128 + row) * ROWB + kg * 16);
      const float ar[4] = {aR.x, aR.y, aR.z, aR.w};
      const float ai[4] = {aI.x, aI.y, aI.z, aI.w};
#pragma unroll
      for (int bn = 0; bn < 4; ++bn) {
        const float br[4] = {bR[bn].x, bR[bn].y, bR[bn].z, bR[bn].w};
        const float bi[4] = {bI[bn].x, bI[bn].y, bI[bn].z, bI[bn].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc.re[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[q], br[q], acc.re[bm][bn], 0, 0, 0);
          acc.re[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[q], bi[q], acc.re[bm][bn], 0, 0, 0);
          acc.im[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[q], bi[q], acc.im[bm][bn], 0, 0, 0);
          acc.im[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[q], br[q], acc.im[bm][bn], 0, 0, 0);
        }
      }
    }
  } else if constexpr (PREC == BIP_PREC_SPLIT_BF16) {
    v8bf bRh[4], bRl[4], bIh[4], bIl[4];
#pragma unroll
    for (int bn = 0; bn < 4; ++bn) {
      const int row = wn * 64 + bn * 16 + lr;
      bRh[bn] = *(const v8bf*)(sB + (0 * 128 + row) * ROWB + kg * 16);
      bRl[bn] = *(const v8bf*)(sB + (1 * 128 + row) * ROWB + kg * 16);
      bIh[bn] = *(const v8bf*)(sB + (2 * 128 + row) * ROWB + kg * 16);
      bIl[bn] = *(const v8bf*)(sB + (3 * 128 + row) * ROWB + kg * 16);
    }
#pragma unroll
    for (int bm = 0; bm < 4; ++bm) {
      const int row = wm * 64 + bm * 16 + lr;
      const v8bf aRh = *(const v8bf*)(sA + (0 * 128 + row) * ROWB + kg * 16);
      const v8bf aRl = *(const v8bf*)(sA + (1 * 128 + row) * ROWB + kg * 16);
      const v8bf aIh = *(const v8bf*)(sA + (2 * 128 + row) * ROWB + kg * 16);
      const v8bf aIl = *(const v8bf*)(sA + (3 * 128 + row) * ROWB + kg * 16);
      const v8bf nIh = neg8(aIh), nIl = neg8(aIl);
#pragma unroll
      for (int bn = 0; bn < 4; ++bn) {
        v4f r = acc.re[bm][bn], i = acc.im[bm][bn];
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aRl, bRh[bn], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aRh, bRl[bn], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nIl, bIh[bn], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nIh, bIl[bn], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aRh, bRh[bn], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nIh, bIh[bn], r, 0, 0, 0);
        i = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aRl, bIh[bn], i, 0, 0, 0);
        i = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aRh, bIl[bn], i, 0, 0, 0);
        i = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aIl, bRh[bn], i, 0, 0, 0);
        i = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aIh, bRl[bn], i, 0, 0, 0);
        i = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aRh, bIh[bn], i, 0, 0, 0);
        i = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aIh, bRh[bn], i, 0, 0, 0);
        acc.re[bm][bn] = r;
        acc.im[bm][bn] = i;
      }
    }
  } else {
    v8bf bR[4], bI[4];
#pragma unroll
    for (int bn = 0; bn < 4; ++bn) {
      const int row = wn * 64 + bn * 16 + lr;
      bR[bn] = *(const v8bf*)(sB + (0 * 128 + row) * ROWB + kg * 16);
      bI[bn] = *(const v8bf*)(sB + (1 * 128 + row) * ROWB + kg * 16);
    }
#pragma unroll
    for (int bm = 0; bm < 4; ++bm) {
      const int row = wm * 64 + bm * 16 + lr;
      const v8bf aR = *(const v8bf*)(sA + (0 * 128 + row) * ROWB + kg * 16);
      const v8bf aI = *(const v8bf*)(sA + (1 * 128 + row) * ROWB + kg * 16);
      const v8bf nI = neg8(aI);
#pragma unroll
      for (int bn = 0; bn < 4; ++bn) {
        acc.re[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aR, bR[bn], acc.re[bm][bn], 0, 0, 0);
        acc.re[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nI, bI[bn], acc.re[bm][bn], 0, 0, 0);
        acc.im[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aR, bI[bn], acc.im[bm][bn], 0, 0, 0);
        acc.im[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aI, bR[bn], acc.im[bm][bn], 0, 0, 0);
      }
    }
  }
}

// Full K loop for one output tile: acc = sum_k A[m0 + .][k] B[n0 + .][k].
template <int PREC>
__device__ inline void tile_product(const char* A, int64_t a_plane_b, int64_t lda_b, const char* B,
                                    int64_t b_plane_b, int64_t ldb_b, int K, char* sA, char* sB,
                                    int tid, int wm, int wn, int lane, Acc& acc) {
  constexpr int BKB = PT<PREC>::BK * PT<PREC>::ESZ;  // 64 bytes
  const int nk = K / PT<PREC>::BK;
  Stage<PREC> sa, sb;
  sa.load(A, a_plane_b, lda_b, 0, tid);
  sb.load(B, b_plane_b, ldb_b, 0, tid);
  sa.store(sA, tid);
  sb.store(sB, tid);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const bool more = kc + 1 < nk;
    if (more) {
      sa.load(A, a_plane_b, lda_b, (kc + 1) * BKB, tid);
      sb.load(B, b_plane_b, ldb_b, (kc + 1) * BKB, tid);
    }
    mma_chunk<PREC>(sA, sB, wm, wn, lane, acc);
    __syncthreads();
    if (more) {
      sa.store(sA, tid);
      sb.store(sB, tid);
      __syncthreads();
    }
  }
}

template <int PREC>
constexpr int lds_bytes() {
  return 2 * PT<PREC>::PLANES * 128 * PT<PREC>::PITCH * PT<PREC>::ESZ;
}

template <int PREC>
__device__ inline void store_u(void* U, int64_t idx, int64_t plane, float re, float im) {
  if (PREC == BIP_PREC_FP32) {
    float* o = (float*)U;
    o[idx] = re;
    o[idx + plane] = im;
  } else if (PREC == BIP_PREC_SPLIT_BF16) {
    uint16_t* o = (uint16_t*)U;
    const uint16_t rh = f2bf(re), ih = f2bf(im);
    o[idx] = rh;
    o[idx + plane] = f2bf(re - bf2f(rh));
    o[idx + 2 * plane] = ih;
    o[idx + 3 * plane] = f2bf(im - bf2f(ih));
  } else {
    uint16_t* o = (uint16_t*)U;
    o[idx] = f2bf(re);
    o[idx + plane] = f2bf(im);
  }
}

// --------------------------------------------------------- probe synthesis
template <int PREC>
__global__ __launch_bounds__(NTHREADS) void k_probe_gemm(const void* __restrict__ Cm,
                                                         int64_t c_plane, int Kb,
                                                         const void* __restrict__ S1op,
                                                         int64_t s1_plane, void* __restrict__ U,
                                                         int64_t u_plane, int64_t Ppad,
                                                         const float2* __restrict__ H,
                                                         const ProbeJob* __restrict__ jobs,
                                                         int n_ch) {
  extern __shared__ char smem[];
  constexpr int ESZ = PT<PREC>::ESZ;
  char* sA = smem;
  char* sB = smem + lds_bytes<PREC>() / 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const ProbeJob job = jobs[blockIdx.z];
  const int n0 = blockIdx.x * BN, m0 = blockIdx.y * BM;
  if (n0 >= job.W2) return;  // this atom's window has fewer column tiles
  const char* A = (const char*)Cm + (int64_t)m0 * Kb * ESZ;
  const char* B = (const char*)S1op + (job.b_off + (int64_t)n0 * Kb) * ESZ;
  Acc acc;
  acc.zero();
  tile_product<PREC>(A, c_plane * ESZ, (int64_t)Kb * ESZ, B, s1_plane * ESZ, (int64_t)Kb * ESZ, Kb,
                     sA, sB, tid, wm, wn, lane, acc);
  // epilogue: U_n[rho][r] = H_n(r) psi^T[rho][r]
  const int lr = lane & 15, kg = lane >> 4;
#pragma unroll
  for (int bn = 0; bn < 4; ++bn) {
    const int r = n0 + wn * 64 + bn * 16 + lr;
    if (r >= job.Kd) continue;
#pragma unroll
    for (int bm = 0; bm < 4; ++bm)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rho = m0 + wm * 64 + bm * 16 + kg * 4 + v;
        const float pr = acc.re[bm][bn][v], pi = acc.im[bm][bn][v];
        for (int n = 0; n < n_ch; ++n) {
          float ur = 0.f, ui = 0.f;
          if (r < job.W2) {
            const float2 h = H[job.h_off + (int64_t)n * job.W2 + r];
            ur = h.x * pr - h.y * pi;
            ui = h.x * pi + h.y * pr;
          }
          store_u<PREC>(U, job.u_off + ((int64_t)n * Ppad + rho) * job.Kd + r, u_plane, ur,
                        ui);
        }
      }
  }
}

// ------------------------------------------------------ detector contraction
template <int PREC, int MODE>
__global__ __launch_bounds__(NTHREADS) void k_det_gemm(const void* __restrict__ A, int64_t a_plane,
                                                       const void* __restrict__ Bm,
                                                       int64_t b_plane,
                                                       const GemmJob* __restrict__ jobs, int njobs,
                                                       float* __restrict__ partial,
                                                       float* __restrict__ out_beams, int ndet,
                                                       int P, int Npad) {
  extern __shared__ char smem[];
  constexpr int ESZ = PT<PREC>::ESZ;
  char* sA = smem;
  char* sB = smem + lds_bytes<PREC>() / 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int n0 = blockIdx.x * BN, m0 = blockIdx.y * BM;
  v4f sq[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) sq[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int jb = 0; jb < njobs; ++jb) {
    const GemmJob job = jobs[jb];
    const char* Ap = (const char*)A + (job.a_off + (int64_t)m0 * job.K) * ESZ;
    const char* Bp = (const char*)Bm + (job.b_off + (int64_t)n0 * job.K) * ESZ;
    Acc acc;
    acc.zero();
    tile_product<PREC>(Ap, a_plane * ESZ, (int64_t)job.K * ESZ, Bp, b_plane * ESZ,
                       (int64_t)job.K * ESZ, job.K, sA, sB, tid, wm, wn, lane, acc);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        sq[i][j] += acc.re[i][j] * acc.re[i][j] + acc.im[i][j] * acc.im[i][j];
  }
  const int lr = lane & 15, kg = lane >> 4;
  if (MODE == BIP_OUT_MAP) {
    // column sums over the 128 rows (d) of the tile, in a fixed order
    __shared__ float red[2][BN];
    float cs[4];
#pragma unroll
    for (int bn = 0; bn < 4; ++bn) {
      float s = 0.f;
#pragma unroll
      for (int bm = 0; bm < 4; ++bm) s += (sq[bm][bn][0] + sq[bm][bn][1]) + (sq[bm][bn][2] + sq[bm][bn][3]);
      s += __shfl_xor(s, 16);
      s += __shfl_xor(s, 32);
      cs[bn] = s;
    }
    __syncthreads();
    if (kg == 0) {
#pragma unroll
      for (int bn = 0; bn < 4; ++bn) red[wm][wn * 64 + bn * 16 + lr] = cs[bn];
    }
    __syncthreads();
    if (tid < BN) partial[(int64_t)blockIdx.y * Npad + n0 + tid] = red[0][tid] + red[1][tid];
  } else {
#pragma unroll
    for (int bn = 0; bn < 4; ++bn) {
      const int rho = n0 + wn * 64 + bn * 16 + lr;
      if (rho >= P) continue;
#pragma unroll
      for (int bm = 0; bm < 4; ++bm)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int d = m0 + wm * 64 + bm * 16 + kg * 4 + v;
          if (d < ndet) out_beams[(int64_t)rho * ndet + d] += sq[bm][bn][v];
        }
    }
  }
}

// -------------------------------------------------------------- helpers
template <int PREC>
__global__ void k_illumination(void* Cm, int64_t plane, int Bpad, int Ppad,
                               const int2* __restrict__ beams, int B, int sy, int sx, float cb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)Ppad * Bpad) return;
  const int rho = (int)(i / Bpad);
  const int b = (int)(i - (int64_t)rho * Bpad);
  float re = 0.f, im = 0.f;
  if (b < B && rho < sy * sx) {
    const int u = rho / sx, v = rho - u * sx;
    const int2 h = beams[b];
    // exp(-2 pi i (h_y u / S_y + h_x v / S_x)) with an exact integer phase
    const int64_t M = (int64_t)sy * sx;
    int64_t m = ((int64_t)h.x * u * sx + (int64_t)h.y * v * sy) % M;
    if (m < 0) m += M;
    double s, c;
    sincospi(-2.0 * (double)m / (double)M, &s, &c);
    re = (float)(cb * c);
    im = (float)(cb * s);
  }
  store_u<PREC>(Cm, i, plane, re, im);
}

__global__ void k_reduce_map(const float* __restrict__ partial, int ntiles, int Ppad, int P,
                             float* out, int accumulate) {
  const int rho = blockIdx.x * blockDim.x + threadIdx.x;
  if (rho >= P) return;
  float s = 0.f;
  for (int t = 0; t < ntiles; ++t) s += partial[(int64_t)t * Ppad + rho];
  out[rho] = accumulate ? out[rho] + s : s;
}

// qEELS: sum the per-beam intensities over h_y at fixed h_x, in detector order
__global__ void k_qeels(const float* __restrict__ beams_out, const int32_t* __restrict__ bin_start,
                        const int32_t* __restrict__ bin_list, int ndet, int P, int nq,
                        float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)P * nq) return;
  const int rho = (int)(i / nq);
  const int q = (int)(i - (int64_t)rho * nq);
  float s = 0.f;
  for (int k = bin_start[q]; k < bin_start[q + 1]; ++k)
    s += beams_out[(int64_t)rho * ndet + bin_list[k]];
  out[i] = s;
}

}  // namespace

hipError_t launch_probe_gemm(int prec, const void* Cm, int64_t c_plane, int Mpad, int Kb,
                             const void* S1op, int64_t s1_plane, int Npad, void* U,
                             int64_t u_plane, const float2* H,
                             const ProbeJob* jobs, int njobs, int n_ch, hipStream_t s) {
  if (njobs == 0) return hipSuccess;
  dim3 grid(Npad / BN, Mpad / BM, njobs);
#define PG(P)                                                                               \
  if (prec == P) {                                                                          \
    hipError_t ea = hipFuncSetAttribute((const void*)k_probe_gemm<P>,                       \
                        hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes<P>());        \
    if (ea != hipSuccess) return ea;                                                        \
    hipLaunchKernelGGL(k_probe_gemm<P>, grid, dim3(NTHREADS), lds_bytes<P>(), s, Cm, c_plane, \
                       Kb, S1op, s1_plane, U, u_plane, (int64_t)Mpad, H, jobs, n_ch);       \
    return hipGetLastError();                                                               \
  }
  PG(BIP_PREC_FP32)
  PG(BIP_PREC_SPLIT_BF16)
  PG(BIP_PREC_BF16)
#undef PG
  return hipErrorInvalidValue;
}

hipError_t launch_det_gemm(int prec, int mode, const void* A, int64_t a_plane, int Mpad,
                           const void* Bm, int64_t b_plane, int Npad, const GemmJob* jobs,
                           int njobs, float* partial, float* out_beams, int ndet, int P,
                           hipStream_t s) {
  if (njobs == 0) return hipSuccess;
  dim3 grid(Npad / BN, Mpad / BM);
#define DG(PR, MO)                                                                           \
  if (prec == PR && mode == MO) {                                                            \
    hipError_t ea = hipFuncSetAttribute((const void*)k_det_gemm<PR, MO>,                     \
                        hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes<PR>());        \
    if (ea != hipSuccess) return ea;                                                         \
    hipLaunchKernelGGL((k_det_gemm<PR, MO>), grid, dim3(NTHREADS), lds_bytes<PR>(), s, A,     \
                       a_plane, Bm, b_plane, jobs, njobs, partial, out_beams, ndet, P, Npad); \
    return hipGetLastError();                                                                \
  }
  DG(BIP_PREC_FP32, BIP_OUT_MAP)
  DG(BIP_PREC_FP32, BIP_OUT_BEAMS)
  DG(BIP_PREC_SPLIT_BF16, BIP_OUT_MAP)
  DG(BIP_PREC_SPLIT_BF16, BIP_OUT_BEAMS)
  DG(BIP_PREC_BF16, BIP_OUT_MAP)
  DG(BIP_PREC_BF16, BIP_OUT_BEAMS)
#undef DG
  return hipErrorInvalidValue;
}

hipError_t launch_illumination(void* Cm, int prec, int64_t plane, int Bpad, int Ppad,
                               const int2* beams, int B, int sy, int sx, float cb, hipStream_t s) {
  const int64_t n = (int64_t)Ppad * Bpad;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
#define IL(P)                                                                                    \
  if (prec == P) {                                                                               \
    hipLaunchKernelGGL(k_illumination<P>, grid, block, 0, s, Cm, plane, Bpad, Ppad, beams, B, sy, \
                       sx, cb);                                                                  \
    return hipGetLastError();                                                                    \
  }
  IL(BIP_PREC_FP32)
  IL(BIP_PREC_SPLIT_BF16)
  IL(BIP_PREC_BF16)
#undef IL
  return hipErrorInvalidValue;
}

hipError_t launch_reduce_map(const float* partial, int ntiles, int Ppad, int P, float* out,
                             int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_map, dim3((P + 255) / 256), dim3(256), 0, s, partial, ntiles, Ppad,
                     P, out, accumulate);
  return hipGetLastError();
}

hipError_t launch_qeels_from_beams(const float* beams_out, const int32_t* bin_start,
                                   const int32_t* bin_list, int ndet, int P, int nq, float* out,
                                   hipStream_t s) {
  const int64_t n = (int64_t)P * nq;
  hipLaunchKernelGGL(k_qeels, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, beams_out,
                     bin_start, bin_list, ndet, P, nq, out);
  return hipGetLastError();
}

}  // namespace bip
