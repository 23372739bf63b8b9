// Focal back-propagation of S1 (section "Magnitude-preserving reconstruction
// and focal back-propagation"): the S1 parent columns, cropped to an enlarged
// M x M window around the atom's W x W window, are Fresnel-stepped back from
// the ionization plane to the scattering centroid of the entrance-to-ionization
// path, interpolated there, and the synthesized probe is stepped forward again
// and cropped to the atom's window.
//
// The Fresnel step of a window takes it as periodic: the window's 2-D DFT is
// multiplied by exp(s i pi lambda dist |q|^2) with q the frequencies of the
// window grid (k / (M delta) per axis, signed k), s = +1 back, -1 forward.
// It runs in LDS: the window is placed at bit-reversed positions, transformed
// by a radix-2 decimation-in-time pass (natural-order spectrum), multiplied,
// and inverted by a decimation-in-frequency pass, whose bit-reversed output
// is read back at bit-reversed positions.  M is a power of two from 8 to 128.
#include "bip_internal.h"
#include "planes.h"

namespace bip {

namespace {

constexpr int NT = 256;

__device__ inline int bitrev(int v, int logm) { return (int)(__brev((unsigned)v) >> (32 - logm)); }

// One radix-2 pass over the rows (dim 0) or the columns (dim 1) of the M x M
// LDS array a: decimation in time (dit, len = 2 .. M) or in frequency (len =
// M .. 2); tw[k] = exp(-2 pi i k / M), conjugated for the inverse.
__device__ inline void fft_dim(float2* a, int M, int logm, const float2* tw, bool inverse, bool dit,
                               int dim) {
  const int nb = M * M / 2;
  for (int s = 0; s < logm; ++s) {
    const int len = dit ? (2 << s) : (M >> s), half = len >> 1;
    for (int t = threadIdx.x; t < nb; t += NT) {
      const int line = t / (M / 2), k = t - line * (M / 2);
      const int g = k / half, j = k - g * half;
      const int i0 = g * len + j, i1 = i0 + half;
      const int e0 = dim == 0 ? line * M + i0 : i0 * M + line;
      const int e1 = dim == 0 ? line * M + i1 : i1 * M + line;
      float2 w = tw[j * (M / len)];
      if (inverse) w.y = -w.y;
      const float2 u = a[e0], v = a[e1];
      if (dit) {
        const float2 vw = cmul(v, w);
        a[e0] = cadd(u, vw);
        a[e1] = csub(u, vw);
      } else {
        a[e0] = cadd(u, v);
        a[e1] = cmul(csub(u, v), w);
      }
    }
    __syncthreads();
  }
}

// exp(sign i pi lambda dist (qy^2 + qx^2)) at natural-order bin (ky, kx) of
// the M x M window grid, the phase in FP64 and reduced mod 2 pi.
__device__ inline float2 fresnel_factor(int ky, int kx, int M, double dy, double dx, double lambda,
                                        double dist, int sign) {
  const int sy = ky < M / 2 ? ky : ky - M, sx = kx < M / 2 ? kx : kx - M;
  const double qy = sy / (M * dy), qx = sx / (M * dx);
  double ph = 3.14159265358979323846 * lambda * dist * (qy * qy + qx * qx);
  ph -= 6.28318530717958647692 * floor(ph / 6.28318530717958647692);
  double s, c;
  sincos(ph, &s, &c);
  return make_float2((float)c, (float)(sign * s));
}

// The Fresnel step of the window in LDS a (natural order in, bit-reversed out).
__device__ inline void window_fresnel(float2* a, int M, int logm, const float2* tw, double dy, double dx,
                                      double lambda, double dist, int sign) {
  fft_dim(a, M, logm, tw, false, true, 0);
  fft_dim(a, M, logm, tw, false, true, 1);
  const float inv = 1.f / (float)(M * M);
  for (int e = threadIdx.x; e < M * M; e += NT) {
    const int ky = e / M, kx = e - ky * M;
    a[e] = cscale(cmul(a[e], fresnel_factor(ky, kx, M, dy, dx, lambda, dist, sign)), inv);
  }
  __syncthreads();
  fft_dim(a, M, logm, tw, true, false, 0);
  fft_dim(a, M, logm, tw, true, false, 1);
}

__device__ inline int ilog2(int m) { return 31 - __clz(m); }

// Back-step of every S1 parent window of every atom (grid: parents x atoms),
// in place in the window stack; the stored windows are de-tilted, so each is
// re-tilted by its parent's carrier first and de-tilted again after the step.
__global__ __launch_bounds__(NT) void k_focal_parents(float2* win, const FocalAtom* __restrict__ atoms,
                                                      const double* __restrict__ dist,
                                                      const int2* __restrict__ parents, int ny, int nx,
                                                      double dy, double dx, double lambda,
                                                      const float2* __restrict__ gtw, int L) {
  extern __shared__ float2 sm[];
  const FocalAtom fa = atoms[blockIdx.y];
  const int M = fa.M, logm = ilog2(M);
  float2* a = sm;
  float2* tw = sm + M * M;
  for (int k = threadIdx.x; k < M; k += NT) tw[k] = gtw[(int64_t)k * (L / M)];
  const int2 h = parents[blockIdx.x];
  float2* wp = win + fa.win_off + (int64_t)blockIdx.x * M * M;
  for (int e = threadIdx.x; e < M * M; e += NT) {
    const int ry = e / M, rx = e - ry * M;
    const int y = (fa.oy + ry) & (ny - 1), x = (fa.ox + rx) & (nx - 1);
    const float2 c = gtw[(h.x * y * (L / ny) + h.y * x * (L / nx)) & (L - 1)];  // exp(-2 pi i h.r/N)
    a[bitrev(ry, logm) * M + bitrev(rx, logm)] = cmulc(wp[e], c);               // re-tilt
  }
  __syncthreads();
  window_fresnel(a, M, logm, tw, dy, dx, lambda, dist[fa.atom], +1);
  for (int e = threadIdx.x; e < M * M; e += NT) {
    const int ry = e / M, rx = e - ry * M;
    const int y = (fa.oy + ry) & (ny - 1), x = (fa.ox + rx) & (nx - 1);
    const float2 c = gtw[(h.x * y * (L / ny) + h.y * x * (L / nx)) & (L - 1)];
    wp[e] = cmul(a[bitrev(ry, logm) * M + bitrev(rx, logm)], c);                 // de-tilt
  }
}

// Forward step of the probe of every scan position (grid: P x atoms of the
// chunk): psi_c [rho][r] (FP32 planes, pitch kd_c) on the enlarged window,
// stepped forward, cropped to the atom's W x W window and stored as the
// contraction operand (psi^T, or U_n = H_n psi), rows P .. Ppad-1 zero.
template <int PREC, bool U>
__global__ __launch_bounds__(NT) void k_focal_probe(FocalProbeArgs fp) {
  extern __shared__ float2 sm[];
  const FocalProbeJob job = fp.jobs[blockIdx.y];
  const int M = job.M, logm = ilog2(M), W = job.W, W2 = W * W, pad = (M - W) / 2;
  const int rho = blockIdx.x;
  float2* a = sm;
  float2* tw = sm + M * M;
  auto put = [&](int row, int r, float re, float im) {
    if constexpr (U) {
      for (int n = 0; n < fp.n_ch; ++n) {
        const float2 hn = r < W2 ? fp.H[job.h_off + (int64_t)n * W2 + r] : make_float2(0.f, 0.f);
        store_planes<PREC>(fp.out, job.out_off + ((int64_t)n * fp.Ppad + row) * job.kd + r, fp.out_plane,
                           hn.x * re - hn.y * im, hn.x * im + hn.y * re);
      }
    } else {
      store_planes<PREC>(fp.out, job.out_off + (int64_t)row * job.kd + r, fp.out_plane, re, im);
    }
  };
  if (rho >= fp.P) {  // padding rows
    for (int r = threadIdx.x; r < job.kd; r += NT) put(rho, r, 0.f, 0.f);
    return;
  }
  for (int k = threadIdx.x; k < M; k += NT) tw[k] = fp.tw[(int64_t)k * (fp.L / M)];
  const float* re = fp.psi_c + job.psi_off + (int64_t)rho * job.kd_c;
  const float* im = re + fp.psi_plane;
  for (int e = threadIdx.x; e < M * M; e += NT) {
    const int ry = e / M, rx = e - ry * M;
    a[bitrev(ry, logm) * M + bitrev(rx, logm)] = make_float2(re[e], im[e]);
  }
  __syncthreads();
  window_fresnel(a, M, logm, tw, fp.dy, fp.dx, fp.lambda, fp.dist[job.atom], -1);
  for (int r = threadIdx.x; r < job.kd; r += NT) {
    float2 v = make_float2(0.f, 0.f);
    if (r < W2) {
      const int ry = r / W + pad, rx = r % W + pad;
      v = a[bitrev(ry, logm) * M + bitrev(rx, logm)];
    }
    put(rho, r, v.x, v.y);
  }
}

// Depth of the scattering centroid of each atom's entrance-to-ionization path
// and the back-step distance (one workgroup per atom): the mean of the slice
// mid-depths (j + 1/2) dz over the slices above the ionization plane, each
// weighted by its projected potential summed over the atom's W x W window;
// distance 0 at plane 0 or with no potential on the path.  FP64 sums.
__global__ __launch_bounds__(NT) void k_focal_dist(const float* __restrict__ V, const FocalAtom* __restrict__ atoms,
                                                   int n_atoms, int ny, int nx, double dz,
                                                   double* __restrict__ dist) {
  __shared__ double red[NT];
  const FocalAtom fa = atoms[blockIdx.x];
  const int W = fa.W, pad = (fa.M - W) / 2;
  double num = 0.0, den = 0.0;
  for (int j = 0; j < fa.plane; ++j) {
    double s = 0.0;
    for (int e = threadIdx.x; e < W * W; e += NT) {
      const int ry = e / W, rx = e - ry * W;
      const int y = (fa.oy + pad + ry) & (ny - 1), x = (fa.ox + pad + rx) & (nx - 1);
      s += (double)V[((int64_t)j * ny + y) * nx + x];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = NT / 2; k > 0; k >>= 1) {
      if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
      __syncthreads();
    }
    const double m = red[0];
    __syncthreads();
    num += (j + 0.5) * dz * m;
    den += m;
  }
  if (threadIdx.x == 0)
    dist[fa.atom] = (fa.plane > 0 && den > 0.0) ? fa.plane * dz - num / den : 0.0;
}

}  // namespace

hipError_t launch_focal_dist(const float* V, const FocalAtom* atoms, int n_atoms, int ny, int nx,
                             double dz, double* dist, hipStream_t s) {
  if (n_atoms <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_focal_dist, dim3(n_atoms), dim3(NT), 0, s, V, atoms, n_atoms, ny, nx, dz, dist);
  return hipGetLastError();
}

hipError_t launch_focal_parents(float2* win, const FocalAtom* atoms, int n_atoms, const double* dist,
                                const int2* parents, int n_par, int max_m, int ny, int nx, double dy,
                                double dx, double lambda, const float2* tw, int L, hipStream_t s) {
  if (n_atoms <= 0 || n_par <= 0) return hipSuccess;
  const size_t lds = (size_t)(max_m * max_m + max_m) * sizeof(float2);
  hipError_t e = hipFuncSetAttribute((const void*)k_focal_parents,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_focal_parents, dim3(n_par, n_atoms), dim3(NT), lds, s, win, atoms, dist, parents,
                     ny, nx, dy, dx, lambda, tw, L);
  return hipGetLastError();
}

hipError_t launch_focal_probe(const FocalProbeArgs& fp, int prec, bool u, int n_jobs, int max_m,
                              hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  const size_t lds = (size_t)(max_m * max_m + max_m) * sizeof(float2);
  const dim3 grid((unsigned)fp.Ppad, (unsigned)n_jobs);
#define FP(P)                                                                                      \
  if (prec == P) {                                                                                 \
    const void* f = u ? (const void*)k_focal_probe<P, true> : (const void*)k_focal_probe<P, false>; \
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
    if (e != hipSuccess) return e;                                                                 \
    if (u)                                                                                         \
      hipLaunchKernelGGL((k_focal_probe<P, true>), grid, dim3(NT), lds, s, fp);                    \
    else                                                                                           \
      hipLaunchKernelGGL((k_focal_probe<P, false>), grid, dim3(NT), lds, s, fp);                   \
    return hipGetLastError();                                                                      \
  }
  FP(BIP_PREC_FP32)
  FP(BIP_PREC_SPLIT_BF16)
  FP(BIP_PREC_BF16)
  FP(BIP_PREC_FP16)
#undef FP
  return hipErrorInvalidValue;
}

}  // namespace bip
