// Probe synthesis on the atom's window (step c, the sum over aperture beams).
//
// psi(r, rho) = sum_b c_b(rho) S1~^b(r) with the raster coefficients
// c_b(rho) = c exp(-2 pi i (h_y u / S_y + h_x v / S_x)), rho = (u, v) (eq.
// probe, illumination coefficients of eq. coupling).  The phase depends on the
// beam only through the residues (h_y mod S_y, h_x mod S_x), so the beams are
// first summed into an S_y x S_x grid of residues (the fold) and psi is the
// unnormalised forward 2-D DFT of that grid, evaluated as two 1-D DFTs.  This
// is the same sum, reordered: 8 W^2 P (S_y + S_x) flops per atom instead of
// 8 W^2 P B for the dense product with the coefficient matrix.
//
// The windowed reconstruction of S1~ (eq. window-recon, eq. magpreserve) is
// fused into the fold, so S1~ never reaches memory.
//
// Pass 1, k_probe_fold_x: a workgroup owns 64 window pixels (one per lane) and
//   one residue row a.  F[c][r] = sum over beams in cell (a, c) of S1~^b(r) is
//   built in LDS, then X[a][v][r] = sum_c exp(-2 pi i c v / S_x) F[c][r] goes
//   to the workspace (complex64, r fastest).
// Pass 2, k_probe_y: a workgroup owns 64 window pixels and one scan column v;
//   psi[u][v][r] = c sum_a exp(-2 pi i a u / S_y) X[a][v][r] is stored as the
//   contraction operand psi^T[rho][r] (map) or as U_n = H_n psi (detector
//   contraction), in the planes of the requested precision.
// Both DFTs run in FP32 on the vector ALUs with twiddles rounded from FP64.
#include "bip_internal.h"
#include "planes.h"
#include "recon_core.h"

namespace bip {

namespace {

constexpr int RT = 64;     // window pixels per workgroup
constexpr int NT = 256;    // threads per workgroup (4 wave64)
constexpr int VG = 16;     // DFT outputs per thread per pass over the LDS tile

// acc[k] += sum_j F[j] * T[(j * o_k) mod S] for the outputs o_k = o0 + wave + 4 k,
// F read from the LDS column of this lane.  The twiddle index advances by o_k
// per step (wave-uniform scalar arithmetic, no division).
__device__ inline void dft_group(const float2* sF, const float2* sT, int S, int o0, int wave,
                                 int lane, float2 (&acc)[VG]) {
  int idx[VG];
#pragma unroll
  for (int k = 0; k < VG; ++k) {
    acc[k] = make_float2(0.f, 0.f);
    idx[k] = 0;
  }
  for (int j = 0; j < S; ++j) {
    const float2 F = sF[j * RT + lane];
#pragma unroll
    for (int k = 0; k < VG; ++k) {
      const int o = o0 + wave + 4 * k;
      if (o < S) {
        const float2 t = sT[idx[k]];
        acc[k].x += F.x * t.x - F.y * t.y;
        acc[k].y += F.x * t.y + F.y * t.x;
        idx[k] += o;
        if (idx[k] >= S) idx[k] -= S;
      }
    }
  }
}

__global__ __launch_bounds__(NT) void k_probe_fold_x(const ProbeArgs pa) {
  extern __shared__ float2 sm[];
  const int Sx = pa.Sx;
  float2* sF = sm;            // [Sx][RT]
  float2* sT = sm + Sx * RT;  // [Sx]
  const ProbeJob job = pa.jobs[blockIdx.z];
  const int W = job.W, W2 = W * W;
  const int r0 = blockIdx.x * RT;
  if (r0 >= W2) return;  // uniform: this atom's window is smaller than the grid
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int a = blockIdx.y;
  for (int i = threadIdx.x; i < Sx; i += NT) sT[i] = pa.twx[i];
  const int r = r0 + lane;
  const bool live = r < W2;
  const int rr = live ? r : 0;
  const int ry = rr / W, rx = rr - ry * W;
  const int py = ((job.oy + ry) & (pa.ny - 1)) * (pa.L / pa.ny);
  const int px = ((job.ox + rx) & (pa.nx - 1)) * (pa.L / pa.nx);
  const float2* win = pa.win + job.win_off;
  for (int c = wave; c < Sx; c += 4) {
    const int cell = a * Sx + c;
    const int k1 = pa.cell_start[cell + 1];
    float2 F = make_float2(0.f, 0.f);
    for (int k = pa.cell_start[cell]; k < k1; ++k) {
      const int b = pa.cell_beams[k];
      const int2 h = pa.beams[b];
      const float2 t = pa.tw[(h.x * py + h.y * px) & (pa.L - 1)];  // exp(-2 pi i h.r/N)
      const float2 s = recon_combine(win, W2, rr, pa.ellc + (int64_t)b * ELL_W,
                                     pa.ellw + (int64_t)b * ELL_W, pa.col, pa.w, pa.mode);
      F = cadd(F, cmulc(s, t));  // re-tilt by exp(+2 pi i h.r/N)
    }
    sF[c * RT + lane] = live ? F : make_float2(0.f, 0.f);
  }
  __syncthreads();
  float2* X = pa.fx + job.fx_off + (int64_t)a * Sx * job.ldf + r;
  for (int v0 = 0; v0 < Sx; v0 += 4 * VG) {
    float2 acc[VG];
    dft_group(sF, sT, Sx, v0, wave, lane, acc);
#pragma unroll
    for (int k = 0; k < VG; ++k) {
      const int v = v0 + wave + 4 * k;
      if (v < Sx) X[(int64_t)v * job.ldf] = acc[k];
    }
  }
}

template <int PREC, bool U>
__global__ __launch_bounds__(NT) void k_probe_y(const ProbeArgs pa) {
  extern __shared__ float2 sm[];
  const int Sy = pa.Sy, Sx = pa.Sx;
  float2* sG = sm;            // [Sy][RT]
  float2* sT = sm + Sy * RT;  // [Sy]
  const ProbeJob job = pa.jobs[blockIdx.z];
  const int W2 = job.W * job.W;
  const int kd = job.kd;
  const int r0 = blockIdx.x * RT;
  if (r0 >= kd) return;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int v = blockIdx.y;
  for (int i = threadIdx.x; i < Sy; i += NT) sT[i] = pa.twy[i];
  const int r = r0 + lane;
  const bool live = r < W2;
  const float2* X = pa.fx + job.fx_off + (int64_t)v * job.ldf + r;
  for (int a = wave; a < Sy; a += 4)
    sG[a * RT + lane] = live ? X[(int64_t)a * Sx * job.ldf] : make_float2(0.f, 0.f);
  __syncthreads();
  const bool in = r < kd;
  auto put = [&](int rho, float re, float im) {
    if constexpr (U) {
      for (int n = 0; n < pa.n_ch; ++n) {
        const float2 hn = live ? pa.H[job.h_off + (int64_t)n * W2 + r] : make_float2(0.f, 0.f);
        store_planes<PREC>(pa.out, job.out_off + ((int64_t)n * pa.Ppad + rho) * kd + r,
                           pa.out_plane, hn.x * re - hn.y * im, hn.x * im + hn.y * re);
      }
    } else {
      store_planes<PREC>(pa.out, job.out_off + (int64_t)rho * kd + r, pa.out_plane, re, im);
    }
  };
  for (int u0 = 0; u0 < Sy; u0 += 4 * VG) {
    float2 acc[VG];
    dft_group(sG, sT, Sy, u0, wave, lane, acc);
    if (in) {
#pragma unroll
      for (int k = 0; k < VG; ++k) {
        const int u = u0 + wave + 4 * k;
        if (u < Sy) put(u * Sx + v, pa.cb * acc[k].x, pa.cb * acc[k].y);
      }
    }
  }
  // rows P .. Ppad-1 of the operand are zero
  if (blockIdx.y == 0 && in)
    for (int rho = pa.P + wave; rho < pa.Ppad; rho += 4) put(rho, 0.f, 0.f);
}

template <typename K>
hipError_t launch_lds(K kernel, dim3 grid, size_t lds, const ProbeArgs& pa, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kernel, grid, dim3(NT), lds, s, pa);
  return hipGetLastError();
}

}  // namespace

size_t probe_lds_bytes(int S) { return (size_t)(S * RT + S) * sizeof(float2); }

hipError_t launch_probe_fold_x(const ProbeArgs& pa, int max_w2, int n_jobs, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  const dim3 grid((unsigned)((max_w2 + RT - 1) / RT), (unsigned)pa.Sy, (unsigned)n_jobs);
  return launch_lds(k_probe_fold_x, grid, probe_lds_bytes(pa.Sx), pa, s);
}

hipError_t launch_probe_y(const ProbeArgs& pa, int prec, bool u, int max_kd, int n_jobs,
                          hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  const dim3 grid((unsigned)((max_kd + RT - 1) / RT), (unsigned)pa.Sx, (unsigned)n_jobs);
  const size_t lds = probe_lds_bytes(pa.Sy);
#define PY(P)                                                              \
  if (prec == P)                                                           \
    return u ? launch_lds(k_probe_y<P, true>, grid, lds, pa, s)            \
             : launch_lds(k_probe_y<P, false>, grid, lds, pa, s);
  PY(BIP_PREC_FP32)
  PY(BIP_PREC_SPLIT_BF16)
  PY(BIP_PREC_BF16)
#undef PY
  return hipErrorInvalidValue;
}

}  // namespace bip
