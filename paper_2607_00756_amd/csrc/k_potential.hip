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

// Profiles of the terms: prof[t][0 .. ny) = g_y, [ny .. ny+nx) = g_x, and
// when deriv != 0 dprof likewise with the coordinate derivatives.
__global__ void k_profiles(const double* __restrict__ terms, int n_terms, int ny, int nx, double ly,
                           double lx, int deriv, double* prof, double* dprof) {
  const int t = blockIdx.x;
  const int i = blockIdx.y * blockDim.x + threadIdx.x;
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

// V_j(y, x) = sum_t A_t g_y,t(y) g_x,t(x) over the terms of slice j: a
// product of the [T][ny] and [T][nx] profile tables along the terms.  A
// workgroup owns 64 x 64 pixels (4 x 4 per thread) and walks the terms in
// chunks of 16 staged in LDS; the sum runs in term order.
constexpr int PT = 64, PK = 16;
__global__ __launch_bounds__(256) void k_build_slice(const double* __restrict__ terms_all,
                                                     const double* __restrict__ prof_all,
                                                     const int64_t* __restrict__ start, int ny,
                                                     int nx, float* V_all) {
  __shared__ double sy[PK][PT], sx[PK][PT];
  const int z = blockIdx.z;  // slice: its terms are start[z] .. start[z + 1]
  const int n_terms = (int)(start[z + 1] - start[z]);
  const double* terms = terms_all + 4 * start[z];
  const double* prof = prof_all + start[z] * (int64_t)(ny + nx);
  float* V = V_all + (int64_t)z * ny * nx;
  const int y0 = blockIdx.y * PT, x0 = blockIdx.x * PT;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t ld = ny + nx;
  double acc[4][4] = {};
  for (int t0 = 0; t0 < n_terms; t0 += PK) {
    for (int i = threadIdx.x; i < PK * PT; i += 256) {
      const int k = i / PT, c = i % PT, t = t0 + k;
      const bool in = t < n_terms;
      sy[k][c] = (in && y0 + c < ny) ? terms[4 * (int64_t)t + 2] * prof[t * ld + y0 + c] : 0.0;
      sx[k][c] = (in && x0 + c < nx) ? prof[t * ld + ny + x0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < PK; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = sy[k][ty + 16 * i];
        b[i] = sx[k][tx + 16 * i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int y = y0 + ty + 16 * i, x = x0 + tx + 16 * j;
      if (y < ny && x < nx) V[(int64_t)y * nx + x] = (float)acc[i][j];
    }
}

// Position gradient of the terms of one slice, in two steps.  Step 1: a
// workgroup owns 64 terms x 64 rows and forms, by a product along x in chunks
// of 16 staged in LDS,
//   M[y][t] = sum_x dV(y, x) dg_x,t(x),   N[y][t] = sum_x dV(y, x) g_x,t(x),
// then reduces its rows to part[yb][t] = (sum_y g_y,t(y) M, sum_y dg_y,t(y) N)
// in a fixed order.  Step 2 (k_grad_sum) adds the row blocks in order and
// scales by A_t.
__global__ __launch_bounds__(256) void k_grad_tiles(const double* __restrict__ prof_all,
                                                    const double* __restrict__ dprof_all,
                                                    const int64_t* __restrict__ start, int64_t nt_all,
                                                    int ny, int nx, const float* __restrict__ dV_all,
                                                    double* part_all) {
  __shared__ double sv[PT][PK + 1];       // dV rows
  __shared__ double sg[PK][PT], sd[PK][PT];  // g_x and dg_x of the term block
  __shared__ double red[2][16][PT];
  const int z = blockIdx.z;  // slice: its terms are start[z] .. start[z + 1]
  const int n_terms = (int)(start[z + 1] - start[z]);
  const int t0 = blockIdx.x * PT, yb = blockIdx.y, y0 = yb * PT;
  if (t0 >= n_terms) return;  // uniform per workgroup
  const double* prof = prof_all + start[z] * (int64_t)(ny + nx);
  const double* dprof = dprof_all + start[z] * (int64_t)(ny + nx);
  const float* dV = dV_all + (int64_t)z * ny * nx;
  double* part = part_all + 2 * start[z];  // [yb][all terms][2]
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;  // tx: terms, ty: rows
  const int64_t ld = ny + nx;
  double m[4][4] = {}, n[4][4] = {};
  for (int x0 = 0; x0 < nx; x0 += PK) {
    for (int i = threadIdx.x; i < PT * PK; i += 256) {
      const int r = i / PK, c = i % PK;  // dV row, x
      sv[r][c] = (y0 + r < ny && x0 + c < nx) ? (double)dV[(int64_t)(y0 + r) * nx + x0 + c] : 0.0;
      const int k = i / PT, tt = i % PT, t = t0 + tt;  // x, term
      const bool in = t < n_terms && x0 + k < nx;
      sg[k][tt] = in ? prof[t * ld + ny + x0 + k] : 0.0;
      sd[k][tt] = in ? dprof[t * ld + ny + x0 + k] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < PK; ++k) {
      double v[4], g[4], d[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[i] = sv[ty + 16 * i][k];
        g[i] = sg[k][tx + 16 * i];
        d[i] = sd[k][tx + 16 * i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          m[i][j] = fma(v[i], d[j], m[i][j]);
          n[i][j] = fma(v[i], g[j], n[i][j]);
        }
    }
    __syncthreads();
  }
  // weight the rows by the y profiles and sum this thread's four rows
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int tt = tx + 16 * j, t = t0 + tt;
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int y = y0 + ty + 16 * i;
      if (t < n_terms && y < ny) {
        sx += prof[t * ld + y] * m[i][j];
        sy += dprof[t * ld + y] * n[i][j];
      }
    }
    red[0][ty][tt] = sx;
    red[1][ty][tt] = sy;
  }
  __syncthreads();
  if (threadIdx.x < PT) {
    const int tt = threadIdx.x, t = t0 + tt;
    double sx = 0.0, sy = 0.0;
    for (int r = 0; r < 16; ++r) {
      sx += red[0][r][tt];
      sy += red[1][r][tt];
    }
    if (t < n_terms) {
      part[((int64_t)yb * nt_all + t) * 2] = sx;
      part[((int64_t)yb * nt_all + t) * 2 + 1] = sy;
    }
  }
}

__global__ void k_grad_sum(const double* __restrict__ terms, const double* __restrict__ part,
                           int64_t n_terms, int nyb, double* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_terms) return;
  double sx = 0.0, sy = 0.0;
  for (int b = 0; b < nyb; ++b) {
    sx += part[((int64_t)b * n_terms + t) * 2];
    sy += part[((int64_t)b * n_terms + t) * 2 + 1];
  }
  const double A = terms[4 * (int64_t)t + 2];
  out[2 * (int64_t)t] = A * sx;
  out[2 * (int64_t)t + 1] = A * sy;
}

// dL/d(x, y) of each atom: the sum of its terms (consecutive, starting at
// first[a]) in term order; dL/dz = 0.
__global__ void k_atom_sum(const double* __restrict__ out, const int64_t* __restrict__ first,
                           int n_atoms, int n_terms, double* __restrict__ dxyz) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_atoms) return;
  double sx = 0.0, sy = 0.0;
  const int64_t t0 = first[a];
  for (int k = 0; k < n_terms; ++k) {
    sx += out[2 * (t0 + k)];
    sy += out[2 * (t0 + k) + 1];
  }
  dxyz[3 * (int64_t)a] = sx;
  dxyz[3 * (int64_t)a + 1] = sy;
  dxyz[3 * (int64_t)a + 2] = 0.0;
}

}  // namespace

hipError_t launch_atom_grad_sum(const double* out, const int64_t* first, int n_atoms, int n_terms,
                                double* dxyz, hipStream_t s) {
  if (n_atoms == 0) return hipSuccess;
  hipLaunchKernelGGL(k_atom_sum, dim3((n_atoms + 255) / 256), dim3(256), 0, s, out, first, n_atoms,
                     n_terms, dxyz);
  return hipGetLastError();
}

hipError_t launch_profiles(const double* terms, int64_t n_terms, int ny, int nx, double ly,
                           double lx, int deriv, double* prof, double* dprof, hipStream_t s) {
  if (n_terms == 0) return hipSuccess;
  if (n_terms > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_profiles, dim3((unsigned)n_terms, (ny + nx + 255) / 256), dim3(256), 0, s,
                     terms, (int)n_terms, ny, nx, ly, lx, deriv, prof, dprof);
  return hipGetLastError();
}

hipError_t launch_build_slices(const double* terms, const double* prof, const int64_t* start, int nz,
                               int ny, int nx, float* V, hipStream_t s) {
  hipLaunchKernelGGL(k_build_slice, dim3((nx + PT - 1) / PT, (ny + PT - 1) / PT, nz), dim3(256), 0, s,
                     terms, prof, start, ny, nx, V);
  return hipGetLastError();
}

int64_t grad_part_doubles(int64_t n_terms, int ny) { return 2 * n_terms * ((ny + PT - 1) / PT); }

hipError_t launch_grad_terms(const double* terms, const double* prof, const double* dprof,
                             const int64_t* start, int64_t nt_all, int most, int nz, int ny, int nx,
                             const float* dV, double* part, double* out, hipStream_t s) {
  if (nt_all == 0) return hipSuccess;
  const int nyb = (ny + PT - 1) / PT;
  hipLaunchKernelGGL(k_grad_tiles, dim3((most + PT - 1) / PT, nyb, nz), dim3(256), 0, s, prof, dprof,
                     start, nt_all, ny, nx, dV, part);
  hipLaunchKernelGGL(k_grad_sum, dim3((unsigned)((nt_all + 255) / 256)), dim3(256), 0, s, terms, part,
                     nt_all, nyb, out);
  return hipGetLastError();
}

}  // namespace bip
