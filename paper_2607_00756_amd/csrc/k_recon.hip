// Windowed natural-neighbour reconstruction (step b).
//
// For every target beam b and window pixel r (eq. window-recon):
//   z = sum_p w_{b,p} D_p(r),   m = sum_p w_{b,p} |D_p(r)|
// with D_p the de-tilted parent windows (already de-tilted by the gather).
// Magnitude-preserving mode (eq. magpreserve) returns m * z/|z| (0 where
// z = 0), complex mode returns z; either is re-tilted by the beam's own
// carrier exp(+/- 2 pi i h_b.r/N), whose phase index is exact integer
// arithmetic on the absolute pixel.
#include "bip_internal.h"
#include "planes.h"
#include "recon_core.h"

namespace bip {

namespace {

__device__ inline float2 recon_value(const ReconArgs& a, int b, int r) {
  const int W2 = a.W * a.W;
  float2 z = make_float2(0.f, 0.f);
  float m = 0.f;
  const int k1 = a.rowptr[b + 1];
  for (int k = a.rowptr[b]; k < k1; ++k) {
    const float2 D = a.win[(int64_t)a.col[k] * W2 + r];
    const float w = a.w[k];
    z.x += w * D.x;
    z.y += w * D.y;
    m += w * sqrtf(D.x * D.x + D.y * D.y);
  }
  float2 s = z;
  if (a.mode == BIP_RECON_MAGNITUDE) {
    const float az = sqrtf(z.x * z.x + z.y * z.y);
    s = az > 0.f ? cscale(z, m / az) : make_float2(0.f, 0.f);
  }
  const int ry = r / a.W, rx = r - ry * a.W;
  const int y = (a.oy + ry) & (a.ny - 1);
  const int x = (a.ox + rx) & (a.nx - 1);
  const int2 h = a.beams[b];
  const int ph = (h.x * y * (a.L / a.ny) + h.y * x * (a.L / a.nx)) & (a.L - 1);
  const float2 w = a.tw[ph];  // exp(-2 pi i h.r/N)
  return a.retilt_sign > 0 ? cmulc(s, w) : cmul(s, w);
}

__global__ void k_recon_plain(ReconArgs a, float2* out) {
  const int W2 = a.W * a.W;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)a.nb * W2) return;
  const int b = (int)(i / W2);
  const int r = (int)(i - (int64_t)b * W2);
  out[i] = recon_value(a, b, r);
}

// GEMM operand output, one 64-beam x 32-pixel tile per workgroup.
// kind 0: S2~^T for the Gram matrix, K-blocked: element (r, b) at
//         ((b / KB) nrows + r) KB + b mod KB, KB = beams per 64-byte row of a
//         plane, so each 64-byte column block is contiguous (ld unused)
// kind 1: element (b, r) at b*ld + r  (r fastest; S2~ for the detector contraction)
// Each half-wave computes one beam on 32 consecutive pixels, so every parent
// read is a coalesced 256-byte row segment; the padded weight rows of the
// tile's beams are staged in LDS first and the parent reads of a value are
// issued together.  Kind 0 transposes through LDS so that each stored row holds
// 64 consecutive beams.  The small LDS footprint (~21 KB) keeps 7 workgroups
// per CU resident to hide the read latency.  Rows and columns beyond the beams
// or the window are written as zeros.
constexpr int TB = 64, TR = 32;

template <int PREC, int KIND>
__global__ __launch_bounds__(256) void k_recon_operand(ReconArgs a, void* out, int64_t ld,
                                                       int nrows, int ncols, int64_t plane) {
  __shared__ float2 tile[TB][TR + 1];
  __shared__ int s_ec[TB][ELL_W];
  __shared__ float s_ew[TB][ELL_W];
  __shared__ int2 s_h[TB];
  const int n_b = KIND == 0 ? ncols : nrows;  // beams to write (padded)
  const int n_r = KIND == 0 ? nrows : ncols;  // pixels to write (padded)
  const int nbt = (n_b + TB - 1) / TB, nrt = (n_r + TR - 1) / TR;
  const int nt = nbt * nrt;
  // workgroup i runs on XCD i mod 8: give each XCD a contiguous range of beam
  // tiles so that the parents it reads stay in its L2
  const int per = (int)(gridDim.x / 8);
  const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (t >= nt) return;
  const int b0 = (t / nrt) * TB, r0 = (t % nrt) * TR;
  for (int i = threadIdx.x; i < TB * ELL_W; i += 256) {
    const int bl = i / ELL_W, j = i % ELL_W;
    const bool in = b0 + bl < a.nb;
    s_ec[bl][j] = in ? a.ellc[(int64_t)(b0 + bl) * ELL_W + j] : 0;
    s_ew[bl][j] = in ? a.ellw[(int64_t)(b0 + bl) * ELL_W + j] : 0.f;
  }
  if (threadIdx.x < TB) s_h[threadIdx.x] = b0 + (int)threadIdx.x < a.nb ? a.beams[b0 + threadIdx.x] : make_int2(0, 0);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int half = lane >> 5, px32 = lane & 31;
  const int W2 = a.W * a.W;
  const int r = r0 + px32;
  const bool live = r < W2;
  const int rr = live ? r : 0;
  const int ry = rr / a.W, rx = rr - ry * a.W;
  const int py = ((a.oy + ry) & (a.ny - 1)) * (a.L / a.ny);
  const int px = ((a.ox + rx) & (a.nx - 1)) * (a.L / a.nx);
  __syncthreads();
  // four beams per batch: all their parent and carrier reads are issued
  // before any of them is combined
  constexpr int NBATCH = 4;
  for (int k0 = 0; k0 < TB / 8; k0 += NBATCH) {
    float2 D[NBATCH][ELL_K], tw[NBATCH];
#pragma unroll
    for (int i = 0; i < NBATCH; ++i) {
      const int bl = 2 * wave + half + 8 * (k0 + i);
      const int2 h = s_h[bl];
      tw[i] = a.tw[(h.x * py + h.y * px) & (a.L - 1)];  // exp(-2 pi i h.r/N)
      recon_load(a.win, W2, rr, s_ec[bl], D[i]);
    }
#pragma unroll
    for (int i = 0; i < NBATCH; ++i) {
      const int bl = 2 * wave + half + 8 * (k0 + i);
      const float2 s = recon_finish(D[i], a.win, W2, rr, s_ec[bl], s_ew[bl], a.col, a.w, a.mode);
      float2 v = make_float2(0.f, 0.f);
      if (b0 + bl < a.nb && live) v = a.retilt_sign > 0 ? cmulc(s, tw[i]) : cmul(s, tw[i]);
      tile[bl][px32] = v;
    }
  }
  __syncthreads();
  if (KIND == 0) {  // rows r0 + j (8 per wave), 64 consecutive beams per row, K-blocked
    constexpr int KB = PREC == BIP_PREC_FP32 ? 16 : 32;  // beams per 64-byte block row
#pragma unroll 2
    for (int k = 0; k < TR / 4; ++k) {
      const int j = wave + 4 * k;
      const int ro = r0 + j, bo = b0 + lane;
      if (ro < n_r && bo < n_b) {
        const float2 v = tile[lane][j];
        store_planes<PREC>(out, ((int64_t)(bo / KB) * n_r + ro) * KB + bo % KB, plane, v.x, v.y);
      }
    }
  } else {  // rows b0 + j, 32 consecutive pixels per half-wave
#pragma unroll 2
    for (int k = 0; k < TB / 8; ++k) {
      const int j = 2 * wave + half + 8 * k;
      const int bo = b0 + j, ro = r0 + px32;
      if (bo < n_b && ro < n_r) {
        const float2 v = tile[j][px32];
        store_planes<PREC>(out, (int64_t)bo * ld + ro, plane, v.x, v.y);
      }
    }
  }
}

}  // namespace

hipError_t launch_recon_plain(const ReconArgs& a, float2* out, hipStream_t s) {
  const int64_t n = (int64_t)a.nb * a.W * a.W;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_recon_plain, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, out);
  return hipGetLastError();
}

hipError_t launch_recon_operand(const ReconArgs& a, void* out, int kind, int prec, int64_t ld,
                                int64_t nrows_pad, int64_t ncols_pad, int64_t plane_stride,
                                hipStream_t s) {
  if (nrows_pad <= 0 || ncols_pad <= 0) return hipSuccess;
  if (nrows_pad > INT32_MAX || ncols_pad > INT32_MAX) return hipErrorInvalidValue;
  const int64_t n_b = kind == 0 ? ncols_pad : nrows_pad, n_r = kind == 0 ? nrows_pad : ncols_pad;
  const int64_t nt = ((n_b + TB - 1) / TB) * ((n_r + TR - 1) / TR);
  const int64_t nblk = (nt + 7) / 8 * 8;
  if (nblk > INT32_MAX) return hipErrorInvalidValue;
  dim3 grid((unsigned)nblk), block(256);
#define RC(P, K)                                                                            \
  if (prec == P && kind == K) {                                                             \
    hipLaunchKernelGGL((k_recon_operand<P, K>), grid, block, 0, s, a, out, ld, (int)nrows_pad, \
                       (int)ncols_pad, plane_stride);                                       \
    return hipGetLastError();                                                               \
  }
  RC(BIP_PREC_FP32, 0)
  RC(BIP_PREC_FP32, 1)
  RC(BIP_PREC_SPLIT_BF16, 0)
  RC(BIP_PREC_SPLIT_BF16, 1)
  RC(BIP_PREC_BF16, 0)
  RC(BIP_PREC_BF16, 1)
#undef RC
  return hipErrorInvalidValue;
}

}  // namespace bip
