// Setup kernels: twiddle table, FP64 Fresnel phase table, transmission
// functions, plane-wave parent columns and the FP64 Sibson geometry.
#include "bip_internal.h"

namespace bip {

// exp(-2 pi i m / L), evaluated in FP64 and rounded once to complex64.
__global__ void k_twiddles(float2* tw, int L) {
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= L) return;
  double s, c;
  sincospi(-2.0 * (double)m / (double)L, &s, &c);
  tw[m] = make_float2((float)c, (float)s);
}

hipError_t launch_twiddles(float2* tw, int L, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles, dim3((L + 255) / 256), dim3(256), 0, s, tw, L);
  return hipGetLastError();
}

// Fresnel transfer function P(q) = exp(-i pi lambda dz |q|^2) (eq. propagator),
// divided by G so that the unnormalized inverse FFTs of a step come out
// normalized.  The phase reaches tens of radians on large grids, so it is
// formed and reduced in FP64.
__global__ void k_prop_table(float2* prop, int ny, int nx, double ly, double lx, double lambda,
                             double dz, int conj) {
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  int y = blockIdx.y;
  if (x >= nx) return;
  int hy = y < ny / 2 ? y : y - ny;
  int hx = x < nx / 2 ? x : x - nx;
  double qy = hy / ly, qx = hx / lx;
  // phase / pi = -lambda dz |q|^2 ; reduce modulo 2 before sincospi
  double t = -lambda * dz * (qy * qy + qx * qx);
  t = t - 2.0 * floor(t * 0.5);
  double s, c;
  sincospi(t, &s, &c);
  double g = 1.0 / ((double)ny * (double)nx);
  prop[(size_t)y * nx + x] = make_float2((float)(c * g), (float)((conj ? -s : s) * g));
}

hipError_t launch_prop_table(float2* prop, int ny, int nx, double ly, double lx, double lambda,
                             double dz, int conj, hipStream_t s) {
  hipLaunchKernelGGL(k_prop_table, dim3((nx + 255) / 256, ny), dim3(256), 0, s, prop, ny, nx, ly,
                     lx, lambda, dz, conj);
  return hipGetLastError();
}

// T_j(r) = exp(i sigma V_j(r)) for all slices.
__global__ void k_transmit(float2* T, const float* __restrict__ V, int64_t n, float sigma) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s, c;
  sincosf(sigma * V[i], &s, &c);
  T[i] = make_float2(c, s);
}

hipError_t launch_transmit(float2* T, const float* V, int64_t n, float sigma, hipStream_t s) {
  hipLaunchKernelGGL(k_transmit, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, T, V, n,
                     sigma);
  return hipGetLastError();
}

// Plane-wave columns scale * exp(sign 2 pi i h.r/N); the phase index
// (h_y y L/N_y + h_x x L/N_x) mod L is exact integer arithmetic.  Grid: y =
// parent column, x = kInitBlocks workgroups striding over the column's
// element pairs (two adjacent pixels of a row, one 16-byte store).
constexpr int kInitBlocks = 32;

__global__ void k_init_planewaves(float2* state, const int2* __restrict__ h, int ny, int nx,
                                  const float2* __restrict__ tw, int L, int sign, float scale) {
  const int p = blockIdx.y;
  const int2 hp = h[p];
  const int64_t npair = (int64_t)ny * nx / 2;
  float4* out = (float4*)(state + (int64_t)p * ny * nx);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npair;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(2 * i), y = e / nx, x = e - y * nx;
    const int my = hp.x * y * (L / ny);
    float2 w0 = tw[(my + hp.y * x * (L / nx)) & (L - 1)];  // exp(-2 pi i m / L)
    float2 w1 = tw[(my + hp.y * (x + 1) * (L / nx)) & (L - 1)];
    if (sign > 0) {
      w0.y = -w0.y;
      w1.y = -w1.y;
    }
    w0 = cscale(w0, scale);
    w1 = cscale(w1, scale);
    out[i] = make_float4(w0.x, w0.y, w1.x, w1.y);
  }
}

hipError_t launch_init_planewaves(float2* state, const int2* h, int nb, int ny, int nx,
                                  const float2* tw, int L, int sign, float scale, hipStream_t s) {
  if (nb == 0) return hipSuccess;
  if ((nx & 1) || nb > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_init_planewaves, dim3(kInitBlocks, nb), dim3(256), 0, s, state, h, ny, nx, tw, L,
                     sign, scale);
  return hipGetLastError();
}

// The same plane waves with sign -1, already row-transformed: the forward
// row DFT of scale exp(-2 pi i (h_y y/ny + h_x x/nx)) is scale nx
// exp(-2 pi i h_y y/ny) at k_x = -h_x (mod nx) and zero at every other k_x.
__global__ void k_init_planewaves_rowft(float2* state, const int2* __restrict__ h, int ny, int nx,
                                        const float2* __restrict__ tw, int L, float scale) {
  const int p = blockIdx.y;
  const int2 hp = h[p];
  const int kx = ((-hp.y) % nx + nx) % nx;
  const int64_t npair = (int64_t)ny * nx / 2;
  float4* out = (float4*)(state + (int64_t)p * ny * nx);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npair;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(2 * i), y = e / nx, x = e - y * nx;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (x == kx || x + 1 == kx) {
      const float2 t = cscale(tw[(hp.x * y * (L / ny)) & (L - 1)], scale * (float)nx);
      if (x == kx) {
        v.x = t.x;
        v.y = t.y;
      } else {
        v.z = t.x;
        v.w = t.y;
      }
    }
    out[i] = v;
  }
}

hipError_t launch_init_planewaves_rowft(float2* state, const int2* h, int nb, int ny, int nx,
                                        const float2* tw, int L, float scale, hipStream_t s) {
  if (nb == 0) return hipSuccess;
  if ((nx & 1) || nb > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_init_planewaves_rowft, dim3(kInitBlocks, nb), dim3(256), 0, s, state, h, ny, nx,
                     tw, L, scale);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Sibson
// Natural-neighbour (Sibson) coordinates of a query beam x against the
// infinite parent lattice s Z^2 (eq. nnw): w_p = |V+(x) ∩ V(p)| / |V+(x)|,
// where V+(x) is the Voronoi cell of x after inserting it and V(p) the s x s
// square cell of lattice point p.  Every lattice point whose square can meet
// V+(x) lies in the 4 x 4 block around the cell containing x, because V+(x)
// is within s/sqrt(2) of x.  All geometry is FP64.
namespace {
constexpr int kMaxVerts = 24;

struct Poly {
  double x[kMaxVerts], y[kMaxVerts];
  int n;
};

// keep the part of `in` where a*x + b*y <= c
__device__ inline void clip(const Poly& in, double a, double b, double c, Poly& out) {
  out.n = 0;
  for (int i = 0; i < in.n; ++i) {
    int k = (i + 1 == in.n) ? 0 : i + 1;
    double px = in.x[i], py = in.y[i], qx = in.x[k], qy = in.y[k];
    double fp = a * px + b * py - c;
    double fq = a * qx + b * qy - c;
    if (fp <= 0.0 && out.n < kMaxVerts) {
      out.x[out.n] = px;
      out.y[out.n] = py;
      ++out.n;
    }
    if (((fp < 0.0 && fq > 0.0) || (fp > 0.0 && fq < 0.0)) && out.n < kMaxVerts) {
      double t = fp / (fp - fq);
      out.x[out.n] = px + t * (qx - px);
      out.y[out.n] = py + t * (qy - py);
      ++out.n;
    }
  }
}

__device__ inline double poly_area(const Poly& p) {
  if (p.n < 3) return 0.0;
  double s = 0.0;
  for (int i = 0; i < p.n; ++i) {
    int k = (i + 1 == p.n) ? 0 : i + 1;
    s += p.x[i] * p.y[k] - p.x[k] * p.y[i];
  }
  return fabs(s) * 0.5;
}
}  // namespace

__global__ void k_sibson(const int2* __restrict__ query, int nq, int s, int2* slot_p,
                         double* slot_w) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  int2 h = query[q];
  int2* sp = slot_p + (size_t)q * 16;
  double* sw = slot_w + (size_t)q * 16;
  // lattice cell of x (floor division valid for negative indices)
  int cy = (h.x >= 0) ? h.x / s : -((-h.x + s - 1) / s);
  int cx = (h.y >= 0) ? h.y / s : -((-h.y + s - 1) / s);
  for (int k = 0; k < 16; ++k) {
    sp[k] = make_int2((cy + k / 4 - 1) * s, (cx + k % 4 - 1) * s);
    sw[k] = 0.0;
  }
  if (h.x == cy * s && h.y == cx * s) {  // query coincides with a parent
    sw[5] = 1.0;                           // block offset (1, 1) is (cy, cx)
    return;
  }
  const double x0 = h.x, x1 = h.y, ds = s;
  Poly a, b;
  a.n = 4;
  a.x[0] = x0 - ds; a.y[0] = x1 - ds;
  a.x[1] = x0 + ds; a.y[1] = x1 - ds;
  a.x[2] = x0 + ds; a.y[2] = x1 + ds;
  a.x[3] = x0 - ds; a.y[3] = x1 + ds;
  for (int k = 0; k < 16; ++k) {
    double p0 = sp[k].x, p1 = sp[k].y;
    // |z - x|^2 <= |z - p|^2  <=>  2 (p - x) . z <= |p|^2 - |x|^2
    clip(a, 2.0 * (p0 - x0), 2.0 * (p1 - x1), p0 * p0 + p1 * p1 - x0 * x0 - x1 * x1, b);
    a = b;
  }
  double total = poly_area(a);
  for (int k = 0; k < 16; ++k) {
    double p0 = sp[k].x, p1 = sp[k].y, hs = 0.5 * ds;
    Poly c, d;
    clip(a, 1.0, 0.0, p0 + hs, c);
    clip(c, -1.0, 0.0, -(p0 - hs), d);
    clip(d, 0.0, 1.0, p1 + hs, c);
    clip(c, 0.0, -1.0, -(p1 - hs), d);
    sw[k] = poly_area(d) / total;
  }
}

hipError_t launch_sibson(const int2* query, int nq, int s_lattice, int2* slot_p, double* slot_w,
                         hipStream_t st) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sibson, dim3((nq + 127) / 128), dim3(128), 0, st, query, nq, s_lattice,
                     slot_p, slot_w);
  return hipGetLastError();
}

// Sibson coordinates against a finite parent set (hex-ring parents).  The
// cell of x and the pieces of its natural neighbours are clipped against
// every parent.
// Queries not strictly inside the parents' convex hull (hull: CCW vertices)
// take the weights of their nearest hull-boundary point: linear interpolation
// between the two ends of the nearest hull edge.  FP64.
namespace {
constexpr int kGenVerts = 48;
constexpr double kHullEps = 1e-9;

struct GPoly {
  double x[kGenVerts], y[kGenVerts];
  int n;
};

__device__ inline void gclip(const GPoly& in, double a, double b, double c, GPoly& out) {
  out.n = 0;
  for (int i = 0; i < in.n; ++i) {
    const int k = (i + 1 == in.n) ? 0 : i + 1;
    const double px = in.x[i], py = in.y[i], qx = in.x[k], qy = in.y[k];
    const double fp = a * px + b * py - c, fq = a * qx + b * qy - c;
    if (fp <= 0.0 && out.n < kGenVerts) {
      out.x[out.n] = px;
      out.y[out.n] = py;
      ++out.n;
    }
    if (((fp < 0.0 && fq > 0.0) || (fp > 0.0 && fq < 0.0)) && out.n < kGenVerts) {
      const double t = fp / (fp - fq);
      out.x[out.n] = px + t * (qx - px);
      out.y[out.n] = py + t * (qy - py);
      ++out.n;
    }
  }
}

__device__ inline double garea(const GPoly& p) {
  if (p.n < 3) return 0.0;
  double s = 0.0;
  for (int i = 0; i < p.n; ++i) {
    const int k = (i + 1 == p.n) ? 0 : i + 1;
    s += p.x[i] * p.y[k] - p.x[k] * p.y[i];
  }
  return fabs(s) * 0.5;
}
}  // namespace

__global__ void k_sibson_general(const int2* __restrict__ query, int nq, const int2* __restrict__ par,
                                 int np, const double2* __restrict__ hull, int nh, int2* slot_p,
                                 double* slot_w, int* overflow) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const int2 h = query[q];
  int2* sp = slot_p + (size_t)q * 16;
  double* sw = slot_w + (size_t)q * 16;
  for (int k = 0; k < 16; ++k) {
    sp[k] = make_int2(0, 0);
    sw[k] = 0.0;
  }
  const double x0 = h.x, x1 = h.y;
  for (int i = 0; i < np; ++i)
    if (par[i].x == h.x && par[i].y == h.y) {  // query coincides with a parent
      sp[0] = par[i];
      sw[0] = 1.0;
      return;
    }
  // hull rule
  bool inside = nh >= 3;
  double best = 1e300;
  int be = 0;
  double bt = 0.0;
  for (int i = 0; i < nh; ++i) {
    const double2 a = hull[i], b = hull[(i + 1) % nh];
    const double ex = b.x - a.x, ey = b.y - a.y;
    const double s = (ex * (x1 - a.y) - ey * (x0 - a.x)) / sqrt(ex * ex + ey * ey);
    if (s <= kHullEps) inside = false;
    double t = ((x0 - a.x) * ex + (x1 - a.y) * ey) / (ex * ex + ey * ey);
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    const double dx = a.x + t * ex - x0, dy = a.y + t * ey - x1;
    const double d = sqrt(dx * dx + dy * dy);
    if (d < best) {
      best = d;
      be = i;
      bt = t;
    }
  }
  if (!inside) {
    const double2 a = hull[be], b = hull[(be + 1) % nh];
    sp[0] = make_int2((int)llrint(a.x), (int)llrint(a.y));
    sw[0] = 1.0 - bt;
    sp[1] = make_int2((int)llrint(b.x), (int)llrint(b.y));
    sw[1] = bt;
    return;
  }
  // Voronoi cell of x among the parents and x: bounded (x is strictly inside
  // the hull) but possibly reaching far out near the hull, so the starting
  // box grows until no vertex of the cell lies on it
  double span = 0.0;
  for (int k = 0; k < np; ++k) span = fmax(span, fmax(fabs(par[k].x - x0), fabs(par[k].y - x1)));
  GPoly a, b;
  for (int round = 0; round < 12; ++round) {
    a.n = 4;
    a.x[0] = x0 - span; a.y[0] = x1 - span;
    a.x[1] = x0 + span; a.y[1] = x1 - span;
    a.x[2] = x0 + span; a.y[2] = x1 + span;
    a.x[3] = x0 - span; a.y[3] = x1 + span;
    for (int k = 0; k < np; ++k) {
      const double p0 = par[k].x, p1 = par[k].y;
      gclip(a, 2.0 * (p0 - x0), 2.0 * (p1 - x1), p0 * p0 + p1 * p1 - x0 * x0 - x1 * x1, b);
      a = b;
    }
    double reach = 0.0;
    for (int v = 0; v < a.n; ++v) reach = fmax(reach, fmax(fabs(a.x[v] - x0), fabs(a.y[v] - x1)));
    if (reach < span * (1.0 - 1e-9)) break;
    span *= 8.0;
  }
  const double total = garea(a);
  int ns = 0;
  for (int k = 0; k < np; ++k) {
    const double p0 = par[k].x, p1 = par[k].y;
    const double la = 2.0 * (p0 - x0), lb = 2.0 * (p1 - x1), lc = p0 * p0 + p1 * p1 - x0 * x0 - x1 * x1;
    double reach = -1e300;  // natural neighbour: the cell touches p's bisector with x
    for (int v = 0; v < a.n; ++v) reach = fmax(reach, la * a.x[v] + lb * a.y[v] - lc);
    if (reach < -1e-9 * (1.0 + span * span)) continue;
    GPoly c = a, d;
    for (int m = 0; m < np && c.n >= 3; ++m) {
      if (m == k) continue;
      const double r0 = par[m].x, r1 = par[m].y;
      gclip(c, 2.0 * (r0 - p0), 2.0 * (r1 - p1), r0 * r0 + r1 * r1 - p0 * p0 - p1 * p1, d);
      c = d;
    }
    const double w = garea(c) / total;
    if (w > 1e-12) {
      if (ns == 16) {
        *overflow = 1;
        return;
      }
      sp[ns] = par[k];
      sw[ns] = w;
      ++ns;
    }
  }
}

hipError_t launch_sibson_general(const int2* query, int nq, const int2* parents, int np,
                                 const double2* hull, int nh, int2* slot_p, double* slot_w,
                                 int* overflow, hipStream_t st) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sibson_general, dim3((nq + 63) / 64), dim3(64), 0, st, query, nq, parents, np,
                     hull, nh, slot_p, slot_w, overflow);
  return hipGetLastError();
}

__global__ void k_zero(float* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

hipError_t launch_zero(float* p, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

__global__ void k_axpy(float* out, const float* __restrict__ src, int64_t n, float w, int accumulate) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = accumulate ? out[i] + w * src[i] : w * src[i];
}

hipError_t launch_axpy(float* out, const float* src, int64_t n, float w, int accumulate, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, src, n, w, accumulate);
  return hipGetLastError();
}

}  // namespace bip
