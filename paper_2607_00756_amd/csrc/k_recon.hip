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

// kind 0: element (r, b) at r*ld + b  (b fastest; S1~ as probe-GEMM operand)
// kind 1: element (b, r) at b*ld + r  (r fastest; S2~ as detector-GEMM operand)
template <int PREC, int KIND>
__global__ void k_recon_operand(ReconArgs a, void* out, int64_t ld, int64_t nrows, int64_t ncols,
                                int64_t plane) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows * ncols) return;
  const int64_t row = i / ncols;
  const int64_t c = i - row * ncols;
  const int W2 = a.W * a.W;
  int b, r;
  if (KIND == 0) {
    r = (int)row;
    b = (int)c;
  } else {
    b = (int)row;
    r = (int)c;
  }
  float2 v = make_float2(0.f, 0.f);
  if (b < a.nb && r < W2) v = recon_value(a, b, r);
  store_planes<PREC>(out, row * ld + c, plane, v.x, v.y);
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
  const int64_t n = nrows_pad * ncols_pad;
  if (n == 0) return hipSuccess;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
#define RC(P, K)                                                                          \
  if (prec == P && kind == K) {                                                           \
    hipLaunchKernelGGL((k_recon_operand<P, K>), grid, block, 0, s, a, out, ld, nrows_pad, \
                       ncols_pad, plane_stride);                                          \
    return hipGetLastError();                                                             \
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
