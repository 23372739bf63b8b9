// Slice potentials from atom positions, and their position gradient.
//
// Reading of the forward model's projected potential: an atom contributes
// v(r) = sum_k A_k exp(-|r - r_a|^2 / (2 w_k^2)) to the slice floor(z/dz), the
// Gaussians summed over periodic images out to 10 w_k along each axis.  Each
// term (atom a, Gaussian k) is separable, A_k g_y(y) g_x(x), so a slice is a
// sum of outer products of 1-D profiles.  The profiles, the sums and the
// gradient reductions run in FP64; V is rounded to float32 once.
//   dL/dx_a = sum_k A_k sum_y g_y(y) sum_x dL/dV(y, x) dg_x/dx_a(x)   (likewise y)
// with dg/dc = sum_m exp(-d^2/2w^2) d / w^2, d = t - c - m L.
#include "bip_internal.h"

namespace bip {

namespace {

// Profiles of one slice's terms: prof[t][0 .. ny) = g_y, [ny .. ny+nx) = g_x,
// and when deriv != 0 dprof likewise with the coordinate derivatives.
__global__ void k_profiles(const double* __restrict__ terms, int n_terms, int ny, int nx, double ly,
                           double lx, int deriv, double* prof, double* dprof) {
  const int t = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_terms || i >= ny + nx) return;
  const double* tm = terms + 4 * (int64_t)t;  // x, y, A, w
  const bool is_y = i < ny;
  const int n = is_y ? ny : nx;
  const double L = is_y ? ly : lx;
  const double c = is_y ? tm[1] : tm[0];
  const double w = tm[3];
  const double pos = (is_y ? i : i - ny) * (L / n);
  const double cut = 10.0 * w;
  const int m_lo = (int)floor((0.0 - c - cut) / L), m_hi = (int)ceil((L - c + cut) / L);
  double g = 0.0, dg = 0.0;
  for (int m = m_lo; m <= m_hi; ++m) {
    const double d = pos - c - m * L;
    if (fabs(d) <= cut) {
      const double e = exp(-d * d / (2.0 * w * w));
      g += e;
      dg += e * d / (w * w);
    }
  }
  prof[(int64_t)t * (ny + nx) + i] = g;
  if (deriv) dprof[(int64_t)t * (ny + nx) + i] = dg;
}

// V_j(y, x) = sum_t A_t g_y,t(y) g_x,t(x) over the terms of slice j.
__global__ void k_build_slice(const double* __restrict__ terms, const double* __restrict__ prof,
                              int n_terms, int ny, int nx, float* V) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= nx) return;
  double s = 0.0;
  for (int t = 0; t < n_terms; ++t) {
    const double* p = prof + (int64_t)t * (ny + nx);
    s += terms[4 * (int64_t)t + 2] * p[y] * p[ny + x];
  }
  V[(int64_t)y * nx + x] = (float)s;
}

// One workgroup per term: out[t] = (A sum g_y dV dg_x, A sum dg_y dV g_x).
__global__ __launch_bounds__(256) void k_grad_terms(const double* __restrict__ terms,
                                                    const double* __restrict__ prof,
                                                    const double* __restrict__ dprof, int ny, int nx,
                                                    const float* __restrict__ dV, double* out) {
  __shared__ double red[2][4];
  const int t = blockIdx.x;
  const double* p = prof + (int64_t)t * (ny + nx);
  const double* dp = dprof + (int64_t)t * (ny + nx);
  double sx = 0.0, sy = 0.0;
  for (int y = 0; y < ny; ++y) {
    const float* row = dV + (int64_t)y * nx;
    double ax = 0.0, ay = 0.0;
    for (int x = threadIdx.x; x < nx; x += 256) {
      ax += (double)row[x] * dp[ny + x];
      ay += (double)row[x] * p[ny + x];
    }
    sx += p[y] * ax;
    sy += dp[y] * ay;
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
    const double A = terms[4 * (int64_t)t + 2];
    out[2 * (int64_t)t] = A * ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3]));
    out[2 * (int64_t)t + 1] = A * ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3]));
  }
}

}  // namespace

hipError_t launch_profiles(const double* terms, int n_terms, int ny, int nx, double ly, double lx,
                           int deriv, double* prof, double* dprof, hipStream_t s) {
  if (n_terms == 0) return hipSuccess;
  hipLaunchKernelGGL(k_profiles, dim3((ny + nx + 255) / 256, n_terms), dim3(256), 0, s, terms,
                     n_terms, ny, nx, ly, lx, deriv, prof, dprof);
  return hipGetLastError();
}

hipError_t launch_build_slice(const double* terms, const double* prof, int n_terms, int ny, int nx,
                              float* V, hipStream_t s) {
  hipLaunchKernelGGL(k_build_slice, dim3((nx + 255) / 256, ny), dim3(256), 0, s, terms, prof,
                     n_terms, ny, nx, V);
  return hipGetLastError();
}

hipError_t launch_grad_terms(const double* terms, const double* prof, const double* dprof,
                             int n_terms, int ny, int nx, const float* dV, double* out,
                             hipStream_t s) {
  if (n_terms == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_terms, dim3(n_terms), dim3(256), 0, s, terms, prof, dprof, ny, nx, dV,
                     out);
  return hipGetLastError();
}

}  // namespace bip
