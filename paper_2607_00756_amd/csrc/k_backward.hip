// Gradient of the map loss: contraction and reconstruction adjoints.
//
// Cotangents are Wirtinger derivatives g_z = dL/d conj(z) (dL = 2 Re sum
// conj(g_z) dz).  With Ibar(rho) = dL/dI(rho) and the map of one atom written
// as I = sum_n u_n^H G u_n, u_n = H_n psi, G = S2~^* S2~^T (eq. coupling, eq.
// map-sum):
//   R[r][r'] = sum_rho Ibar(rho) conj(psi(r, rho)) psi(r', rho)
//   g_psi(r, rho) = Ibar(rho) (Q psi)(r, rho),      Q = G o Hc
//   g_S2~^d(r) = sum_r' S2~^d(r') K[r][r'],           K = Hc o R
//   g_H_n(r) = sum_r' (G o R)[r][r'] H_n(r'),        Hc[r][r'] = sum_n conj(H_n(r)) H_n(r')
// (R, the products with Q and with K run on the matrix cores, k_gemm.hip).
// The reconstruction s = m z/|z| (eq. magpreserve), re-tilted by t, gives
//   g_s = conj(t) g_out,  g_z = m/(2|z|) (g_s - conj(g_s) phi^2),  gamma = Re(conj(g_s) phi)
// with phi = z/|z|, and for the parent windows D_p (z = sum w D, m = sum w |D|)
//   g_D_p = sum_b w_bp (g_z,b + gamma_b D_p/|D_p|);
// the cotangent of the parent column is conj(de-tilt carrier) g_D_p.
#include "bip_internal.h"
#include "planes.h"
#include "recon_core.h"

namespace bip {

namespace {

// A1[r][rho] = psi(r, rho), B1[r][rho] = Ibar(rho) psi(r, rho) (operand planes
// of precision PREC, rows up to n1, columns up to Ppad) from psi^T [rho][r]
// (planes of the same precision).
template <int PREC>
__global__ void k_psi_transpose(const void* __restrict__ psiT, int64_t psp, int kd, int W2, int P,
                                int Ppad, const float* __restrict__ ibar, void* A1, void* B1,
                                int64_t apl) {
  __shared__ float2 tile[32][33];
  const int rho0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int k = 0; k < 32; k += 8) {
    const int rho = rho0 + ty + k, r = r0 + tx;
    float2 v = make_float2(0.f, 0.f);
    if (rho < P && r < W2) v = load_planes<PREC>(psiT, (int64_t)rho * kd + r, psp);
    tile[ty + k][tx] = v;
  }
  __syncthreads();
  for (int k = 0; k < 32; k += 8) {
    const int r = r0 + ty + k, rho = rho0 + tx;
    const float2 v = tile[tx][ty + k];
    const float s = rho < P ? ibar[rho] : 0.f;
    const int64_t i = (int64_t)r * Ppad + rho;
    store_planes<PREC>(A1, i, apl, v.x, v.y);
    store_planes<PREC>(B1, i, apl, s * v.x, s * v.y);
  }
}

// K[r][r'] = R[r][r'] sum_n conj(H_n(r)) H_n(r') as operand planes of
// precision PREC (zero outside the window), rows up to n1, columns up to kd.
template <int PREC>
__global__ void k_kmat(const float2* __restrict__ R, const float2* __restrict__ H, int n_ch, int W2,
                       int kd, int n1, void* Kp, int64_t kpl) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n1 * kd) return;
  const int r = (int)(i / kd), c = (int)(i - (int64_t)r * kd);
  float kr = 0.f, ki = 0.f;
  if (r < W2 && c < W2) {
    float hr = 0.f, hi = 0.f;
    for (int n = 0; n < n_ch; ++n) {
      const float2 a = H[(int64_t)n * W2 + r], b = H[(int64_t)n * W2 + c];
      hr += a.x * b.x + a.y * b.y;
      hi += a.x * b.y - a.y * b.x;
    }
    const float2 q = R[i];
    kr = q.x * hr - q.y * hi;
    ki = q.x * hi + q.y * hr;
  }
  store_planes<PREC>(Kp, i, kpl, kr, ki);
}

// Fixed-order reduction of a float2 over a 256-thread block.
__device__ inline float2 block_sum(float2 v, float2* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return cadd(cadd(red[0], red[1]), cadd(red[2], red[3]));
}

// g_H_n(r) = sum_r' G[r][r'] R[r][r'] H_n(r'), one workgroup per pixel r.
__global__ __launch_bounds__(256) void k_grad_h(const float2* __restrict__ G,
                                                const float2* __restrict__ R,
                                                const float2* __restrict__ H, int n_ch, int W2,
                                                int kd, float2* gH) {
  __shared__ float2 red[4];
  const int r = blockIdx.x;
  for (int n = 0; n < n_ch; ++n) {
    float2 acc = make_float2(0.f, 0.f);
    for (int c = threadIdx.x; c < W2; c += 256) {
      const int64_t i = (int64_t)r * kd + c;
      acc = cadd(acc, cmul(cmul(G[i], R[i]), H[(int64_t)n * W2 + c]));
    }
    const float2 s = block_sum(acc, red);
    if (threadIdx.x == 0) gH[(int64_t)n * W2 + r] = s;
  }
}

// dL/dtau = 2 Re sum conj(g_H) dH/dtau over one atom's channels and pixels.
__global__ __launch_bounds__(256) void k_grad_tau(const float2* __restrict__ gH,
                                                  const float2* __restrict__ dHx,
                                                  const float2* __restrict__ dHy, int n,
                                                  double* out) {
  __shared__ double red[2][4];
  double sx = 0.0, sy = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const float2 g = gH[i], ax = dHx[i], ay = dHy[i];
    sx += (double)g.x * ax.x + (double)g.y * ax.y;
    sy += (double)g.x * ay.x + (double)g.y * ay.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sx += __shfl_xor(sx, o);
    sy += __shfl_xor(sy, o);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = sx;
    red[1][wave] = sy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = 2.0 * ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3]));
    out[1] = 2.0 * ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3]));
  }
}

// Phase A of the reconstruction adjoint, per target beam b (one wave) and
// window pixel r (one lane): g_z and gamma from the beam's cotangent.
// SIDE 1: the cotangent of S1~^b is c Z[cell(b)][r] (the adjoint of the
// probe sum, see k_probe.hip); SIDE 2: g_S2~ [d][r] from the contraction.
template <int SIDE>
__global__ __launch_bounds__(256) void k_recon_adj_a(ReconArgs a, const float2* __restrict__ gsrc,
                                                     int64_t ld_src, int Sy, int Sx, float cb,
                                                     float2* gz, float* gam) {
  const int b = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (b >= a.nb) return;
  const int W2 = a.W * a.W;
  const int r = blockIdx.x * 64 + (threadIdx.x & 63);
  if (r >= W2) return;
  const int ry = r / a.W, rx = r - ry * a.W;
  const int py = ((a.oy + ry) & (a.ny - 1)) * (a.L / a.ny);
  const int px = ((a.ox + rx) & (a.nx - 1)) * (a.L / a.nx);
  const int2 h = a.beams[b];
  const float2 tw = a.tw[(h.x * py + h.y * px) & (a.L - 1)];  // exp(-2 pi i h.r/N)
  float2 gout;
  if (SIDE == 1) {
    const int ca = ((h.x % Sy) + Sy) % Sy, cc = ((h.y % Sx) + Sx) % Sx;
    gout = cscale(gsrc[(int64_t)(ca * Sx + cc) * ld_src + r], cb);
  } else {
    gout = gsrc[(int64_t)b * ld_src + r];
  }
  // re-tilt t = conj(tw) for S1, tw for S2; g_s = conj(t) g_out
  const float2 gs = SIDE == 1 ? cmul(gout, tw) : cmulc(gout, tw);
  float2 g_z = gs;
  float gamma = 0.f;
  if (a.mode == BIP_RECON_MAGNITUDE) {
    float2 D[ELL_K];
    const int32_t* ec = a.ellc + (int64_t)b * ELL_W;
    recon_load(a.win, W2, r, ec, D);
    float2 z;
    float m;
    recon_zm(D, a.win, W2, r, ec, a.ellw + (int64_t)b * ELL_W, a.col, a.w, z, m);
    const float az = sqrtf(z.x * z.x + z.y * z.y);
    if (az > 0.f) {
      const float2 phi = cscale(z, 1.f / az);
      const float2 phi2 = cmul(phi, phi);
      const float2 cgs = make_float2(gs.x, -gs.y);
      g_z = cscale(csub(gs, cmul(cgs, phi2)), m / (2.f * az));
      gamma = gs.x * phi.x + gs.y * phi.y;  // Re(conj(g_s) phi)
    } else {
      g_z = make_float2(0.f, 0.f);
    }
  }
  gz[(int64_t)b * W2 + r] = g_z;
  gam[(int64_t)b * W2 + r] = gamma;
}

// Phase B: per parent p (one wave) and pixel r (one lane), the cotangent of
// the cropped parent column, conj(e_p) sum_b w_bp (g_z,b + gamma_b D_p/|D_p|)
// over the beams that use p (transposed weights, fixed order).
__global__ __launch_bounds__(256) void k_recon_adj_b(ReconArgs a, const int2* __restrict__ parents,
                                                     int Bp, const int32_t* __restrict__ tp_rp,
                                                     const int32_t* __restrict__ tp_b,
                                                     const float* __restrict__ tp_w,
                                                     const float2* __restrict__ gz,
                                                     const float* __restrict__ gam, int detilt_sign,
                                                     float2* gwin) {
  const int p = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (p >= Bp) return;
  const int W2 = a.W * a.W;
  const int r = blockIdx.x * 64 + (threadIdx.x & 63);
  if (r >= W2) return;
  const float2 D = a.win[(int64_t)p * W2 + r];
  const float aD = sqrtf(D.x * D.x + D.y * D.y);
  const float2 u = aD > 0.f ? cscale(D, 1.f / aD) : make_float2(0.f, 0.f);
  float2 acc = make_float2(0.f, 0.f);
  const int k1 = tp_rp[p + 1];
  for (int k = tp_rp[p]; k < k1; ++k) {
    const int b = tp_b[k];
    const float w = tp_w[k];
    const float2 g = gz[(int64_t)b * W2 + r];
    const float ga = gam[(int64_t)b * W2 + r];
    acc.x += w * (g.x + ga * u.x);
    acc.y += w * (g.y + ga * u.y);
  }
  const int ry = r / a.W, rx = r - ry * a.W;
  const int py = ((a.oy + ry) & (a.ny - 1)) * (a.L / a.ny);
  const int px = ((a.ox + rx) & (a.nx - 1)) * (a.L / a.nx);
  const int2 h = parents[p];
  const float2 tw = a.tw[(h.x * py + h.y * px) & (a.L - 1)];  // exp(-2 pi i h_p.r/N)
  // de-tilt e_p = tw (S1, sign +1) or conj(tw) (S2); multiply by conj(e_p)
  gwin[(int64_t)p * W2 + r] = detilt_sign > 0 ? cmulc(acc, tw) : cmul(acc, tw);
}

}  // namespace

hipError_t launch_psi_transpose(int prec, const void* psiT, int64_t psp, int kd, int W2, int P,
                                int Ppad, int n1, const float* ibar, void* A1, void* B1, int64_t apl,
                                hipStream_t s) {
  const dim3 grid(Ppad / 32, n1 / 32);
  if (prec == BIP_PREC_FP32)
    hipLaunchKernelGGL(k_psi_transpose<BIP_PREC_FP32>, grid, dim3(256), 0, s, psiT, psp, kd, W2, P,
                       Ppad, ibar, A1, B1, apl);
  else if (prec == BIP_PREC_SPLIT_BF16)
    hipLaunchKernelGGL(k_psi_transpose<BIP_PREC_SPLIT_BF16>, grid, dim3(256), 0, s, psiT, psp, kd, W2,
                       P, Ppad, ibar, A1, B1, apl);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_kmat(int prec, const float2* R, const float2* H, int n_ch, int W2, int kd, int n1,
                       void* Kp, int64_t kpl, hipStream_t s) {
  const int64_t n = (int64_t)n1 * kd;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (prec == BIP_PREC_FP32)
    hipLaunchKernelGGL(k_kmat<BIP_PREC_FP32>, grid, dim3(256), 0, s, R, H, n_ch, W2, kd, n1, Kp, kpl);
  else if (prec == BIP_PREC_SPLIT_BF16)
    hipLaunchKernelGGL(k_kmat<BIP_PREC_SPLIT_BF16>, grid, dim3(256), 0, s, R, H, n_ch, W2, kd, n1, Kp, kpl);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_grad_h(const float2* G, const float2* R, const float2* H, int n_ch, int W2, int kd,
                         float2* gH, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_h, dim3(W2), dim3(256), 0, s, G, R, H, n_ch, W2, kd, gH);
  return hipGetLastError();
}

hipError_t launch_grad_tau(const float2* gH, const float2* dHx, const float2* dHy, int n,
                           double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_tau, dim3(1), dim3(256), 0, s, gH, dHx, dHy, n, out);
  return hipGetLastError();
}

hipError_t launch_recon_adjoint(const ReconArgs& a, int side, const float2* gsrc, int64_t ld_src,
                                int Sy, int Sx, float cb, float2* gz, float* gam,
                                const int2* parents, int Bp, const int32_t* tp_rp,
                                const int32_t* tp_b, const float* tp_w, float2* gwin,
                                hipStream_t s) {
  const int W2 = a.W * a.W;
  const dim3 ga((W2 + 63) / 64, (a.nb + 3) / 4), gb((W2 + 63) / 64, (Bp + 3) / 4);
  if (side == 1)
    hipLaunchKernelGGL(k_recon_adj_a<1>, ga, dim3(256), 0, s, a, gsrc, ld_src, Sy, Sx, cb, gz, gam);
  else
    hipLaunchKernelGGL(k_recon_adj_a<2>, ga, dim3(256), 0, s, a, gsrc, ld_src, Sy, Sx, cb, gz, gam);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_recon_adj_b, gb, dim3(256), 0, s, a, parents, Bp, tp_rp, tp_b, tp_w, gz, gam,
                     side == 1 ? +1 : -1, gwin);
  return hipGetLastError();
}

}  // namespace bip
