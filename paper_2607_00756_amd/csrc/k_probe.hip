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
//   to the workspace (complex64, r fastest).  The S_y workgroups of one pixel
//   tile run on one XCD, so the tile's parent windows are read from its L2.
// Pass 2, k_probe_y: a workgroup owns 64 window pixels and one scan column v;
//   psi[u][v][r] = c sum_a exp(-2 pi i a u / S_y) X[a][v][r] is stored as the
//   contraction operand psi^T[rho][r] (map) or as U_n = H_n psi (detector
//   contraction), in the planes of the requested precision.
// Both DFTs run on the FP32 matrix cores with twiddles rounded from FP64.
#include "bip_internal.h"
#include "planes.h"
#include "recon_core.h"

namespace bip {

namespace {

constexpr int RT = 64;     // window pixels per workgroup (16 per wave)
constexpr int kBufferWord3 = 0x00020000;  // raw (untyped) buffer descriptor, 32-bit data
constexpr int NT = 256;    // threads per workgroup (4 wave64)

typedef float v4f __attribute__((ext_vector_type(4)));

// Four 16 x 16 output blocks of a DFT along the LDS rows, on the FP32 matrix
// cores: X[o][r] = sum_{j < S} T[(o j) mod S] F[j][r] for o in
// [obase, obase + 64) and this wave's pixels r in [16 wave, 16 wave + 16).
// F rows S .. Sc-1 (Sc = S rounded up to 4) must be zero.  A complex block is
// four real v_mfma_f32_16x16x4f32 products (the A operand is the twiddle,
// lane l holding row l mod 16 and K index l / 16; the B operand is F, lane l
// holding K index l / 16 and column l mod 16).  Output: lane l holds rows
// obase + 16 ob + 4 (l / 16) + q, column 16 wave + l mod 16, in xr / xi[ob][q].
// The same product restricted to K rows [jb, je) (je - jb a multiple of 4),
// sF holding row j at j - jb, added to xr / xi.
__device__ inline void dft_mfma_part(const float2* sF, const float2* sT, int S, int obase, int jb, int je,
                                     int wave, int lane, v4f (&xr)[4], v4f (&xi)[4]) {
  const int li = lane & 15, lk = lane >> 4;
  int idx[4], step[4];
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    const int o = obase + 16 * ob + li;
    const int oo = o < S ? o : 0;
    idx[ob] = (oo * (jb + lk)) % S;
    step[ob] = (4 * oo) % S;
  }
  for (int j0 = jb; j0 < je; j0 += 4) {
    const float2 f = sF[(j0 - jb + lk) * RT + 16 * wave + li];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      if (obase + 16 * ob < S) {  // wave-uniform
        const float2 e = sT[idx[ob]];
        xr[ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(e.x, f.x, xr[ob], 0, 0, 0);
        xr[ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(-e.y, f.y, xr[ob], 0, 0, 0);
        xi[ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(e.x, f.y, xi[ob], 0, 0, 0);
        xi[ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(e.y, f.x, xi[ob], 0, 0, 0);
      }
      idx[ob] += step[ob];
      if (idx[ob] >= S) idx[ob] -= S;
    }
  }
}

__device__ inline void dft_mfma(const float2* sF, const float2* sT, int S, int obase, int wave,
                                int lane, v4f (&xr)[4], v4f (&xi)[4]) {
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    xr[ob] = v4f{0.f, 0.f, 0.f, 0.f};
    xi[ob] = v4f{0.f, 0.f, 0.f, 0.f};
  }
  dft_mfma_part(sF, sT, S, obase, 0, (S + 3) & ~3, wave, lane, xr, xi);
}

constexpr int FOLD_CH = 64;  // residue cells of the fold held in LDS at a time

// 1-D grid.  Workgroups are dispatched to the 8 XCDs in turn, so blocks x,
// x + 8, x + 16, ... share XCD x: its slot s takes residue row s mod S_y of
// pixel tile unit0 + 8 (s / S_y) + x, and the S_y rows of a tile run together
// in one L2.  A tile is 64 pixels of one job (the job with the last t0 <= the
// tile).  The dispatch order only affects speed.
// The residue cells are folded FOLD_CH at a time into LDS, and each chunk's
// share of the DFT over x is added to the NV = ceil(S_x / 64) output blocks
// held in registers (the products run in the same K order as one pass).
template <int NV>
__global__ __launch_bounds__(NT) void k_probe_fold_x(const ProbeArgs pa) {
  extern __shared__ float2 sm[];
  const int Sx = pa.Sx;
  const int CH = min((Sx + 3) & ~3, FOLD_CH);
  float2* sF = sm;           // [CH][RT]
  float2* sT = sm + CH * RT; // [Sx]
  float2* sW = sT + Sx;      // [L] exp(-2 pi i m / L), gathered per lane
  const int slot = blockIdx.x >> 3;
  const int k8 = slot / pa.Sy;
  const int a = slot - k8 * pa.Sy;
  const int u = pa.unit0 + 8 * k8 + (blockIdx.x & 7);
  if (u >= pa.unit0 + pa.n_units) return;  // the grid's last row of 8 tiles
  int lo = 0, hi = pa.n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pa.jobs[mid].t0 <= u) lo = mid;
    else hi = mid - 1;
  }
  const ProbeJob job = pa.jobs[lo];
  const int W = job.W, W2 = W * W;
  const int r0 = (u - job.t0) * RT;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int i = threadIdx.x; i < Sx; i += NT) sT[i] = pa.twx[i];
  for (int i = threadIdx.x; i < pa.L; i += NT) sW[i] = pa.tw[i];
  __syncthreads();
  const int r = r0 + lane;
  const bool live = r < W2;
  const int rr = live ? r : 0;
  const int ry = rr / W, rx = rr - ry * W;
  const int py = ((job.oy + ry) & (pa.ny - 1)) * (pa.L / pa.ny);
  const int px = ((job.ox + rx) & (pa.nx - 1)) * (pa.L / pa.nx);
  const float2* win = pa.win + job.win_off;
  // The parent values are read through a buffer descriptor of the atom's
  // window stack: the parent's offset in a scalar register, the pixel's in a
  // vector one, so a load needs no per-lane address arithmetic.  A stack
  // block beyond the descriptor's 32-bit offsets (2 GiB) is read through
  // 64-bit pointers instead (a choice uniform over the workgroup).
  const bool rsrc_ok = (int64_t)pa.n_par * W2 * (int64_t)sizeof(float2) <= 0x7fffffff;
  const __amdgpu_buffer_rsrc_t rwin = __builtin_amdgcn_make_buffer_rsrc(
      (void*)win, (short)0, rsrc_ok ? pa.n_par * W2 * (int)sizeof(float2) : 0, kBufferWord3);
  const int voff = rr * (int)sizeof(float2);
  v4f xr[NV][4], xi[NV][4];
#pragma unroll
  for (int vi = 0; vi < NV; ++vi)
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      xr[vi][ob] = v4f{0.f, 0.f, 0.f, 0.f};
      xi[vi][ob] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  for (int cc = 0; cc < Sx; cc += CH) {
    const int ce = min(Sx, cc + CH);
    const int cp = cc + ((ce - cc + 3) & ~3);  // the chunk's K rows, zero beyond ce
    for (int c = cc + wave; c < ce; c += 4) {
      const int cell = a * Sx + c;
      const int k1 = pa.cell_start[cell + 1];
      float2 F = make_float2(0.f, 0.f);
      for (int k = pa.cell_start[cell]; k < k1; ++k) {
        const int b = pa.cell_beams[k];
        const int2 h = pa.beams[b];
        const float2 t = sW[(h.x * py + h.y * px) & (pa.L - 1)];  // exp(-2 pi i h.r/N)
        const int32_t* ec = pa.ellc + (int64_t)b * ELL_W;
        const float* ew = pa.ellw + (int64_t)b * ELL_W;
        float2 D[ELL_K];
        if (rsrc_ok) {
#pragma unroll
          for (int j = 0; j < ELL_K; ++j)
            D[j] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(
                                                  rwin, voff, ec[j] * W2 * (int)sizeof(float2), 0));
        } else {
          recon_load(win, W2, rr, ec, D);
        }
        const float2 sv = recon_finish(D, win, W2, rr, ec, ew, pa.col, pa.w, pa.mode);
        F = cadd(F, cmulc(sv, t));  // re-tilt by exp(+2 pi i h.r/N)
      }
      sF[(c - cc) * RT + lane] = live ? F : make_float2(0.f, 0.f);
    }
    for (int c = ce + wave; c < cp; c += 4) sF[(c - cc) * RT + lane] = make_float2(0.f, 0.f);
    __syncthreads();
#pragma unroll
    for (int vi = 0; vi < NV; ++vi) dft_mfma_part(sF, sT, Sx, 64 * vi, cc, cp, wave, lane, xr[vi], xi[vi]);
    __syncthreads();  // the chunk is consumed before the next one is folded
  }
  const int li = lane & 15, lk = lane >> 4;
  float2* X = pa.fx + job.fx_off + (int64_t)a * Sx * job.ldf + r0 + 16 * wave + li;
#pragma unroll
  for (int vi = 0; vi < NV; ++vi)
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int v = 64 * vi + 16 * ob + 4 * lk + q;
        if (v < Sx) X[(int64_t)v * job.ldf] = make_float2(xr[vi][ob][q], xi[vi][ob][q]);
      }
}

// The residue rows a are staged FOLD_CH at a time, each chunk's share of the
// DFT over y added to the NV = ceil(S_y / 64) output blocks in registers.
template <int PREC, bool U, int NV>
__global__ __launch_bounds__(NT) void k_probe_y(const ProbeArgs pa) {
  extern __shared__ float2 sm[];
  const int Sy = pa.Sy, Sx = pa.Sx;
  const int CH = min((Sy + 3) & ~3, FOLD_CH);
  float2* sG = sm;            // [CH][RT]
  float2* sT = sm + CH * RT;  // [Sy]
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
  v4f xr[NV][4], xi[NV][4];
#pragma unroll
  for (int vi = 0; vi < NV; ++vi)
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      xr[vi][ob] = v4f{0.f, 0.f, 0.f, 0.f};
      xi[vi][ob] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  for (int ac = 0; ac < Sy; ac += CH) {
    const int ap = ac + ((min(Sy, ac + CH) - ac + 3) & ~3);  // the chunk's K rows, zero from S_y
    // this wave's rows of the chunk: all loads in flight before the LDS stores
    float2 xg[FOLD_CH / 4];
#pragma unroll
    for (int q = 0; q < FOLD_CH / 4; ++q) {
      const int a = ac + wave + 4 * q;
      xg[q] = (a < ap && live && a < Sy) ? X[(int64_t)a * Sx * job.ldf] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int q = 0; q < FOLD_CH / 4; ++q) {
      const int a = ac + wave + 4 * q;
      if (a < ap) sG[(a - ac) * RT + lane] = xg[q];
    }
    __syncthreads();
#pragma unroll
    for (int vi = 0; vi < NV; ++vi) dft_mfma_part(sG, sT, Sy, 64 * vi, ac, ap, wave, lane, xr[vi], xi[vi]);
    __syncthreads();  // the chunk is consumed before the next one is staged
  }
  // this lane's output pixel
  const int li = lane & 15, lk = lane >> 4;
  const int ro = r0 + 16 * wave + li;
  const bool in = ro < kd, live_o = ro < W2;
  auto put = [&](int rho, float re, float im) {
    if constexpr (U) {
      for (int n = 0; n < pa.n_ch; ++n) {
        const float2 hn = live_o ? pa.H[job.h_off + (int64_t)n * W2 + ro] : make_float2(0.f, 0.f);
        store_planes<PREC>(pa.out, job.out_off + ((int64_t)n * pa.Ppad + rho) * kd + ro,
                           pa.out_plane, hn.x * re - hn.y * im, hn.x * im + hn.y * re);
      }
    } else {
      store_planes<PREC>(pa.out, job.out_off + (int64_t)rho * kd + ro, pa.out_plane, re, im);
    }
  };
  if (in) {
#pragma unroll
    for (int vi = 0; vi < NV; ++vi)
#pragma unroll
      for (int ob = 0; ob < 4; ++ob)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int u = 64 * vi + 16 * ob + 4 * lk + q;
          if (u < Sy) put(u * Sx + v, pa.cb * xr[vi][ob][q], pa.cb * xi[vi][ob][q]);
        }
  }
  // rows P .. Ppad-1 of the operand are zero
  if (blockIdx.y == 0 && in)
    for (int rho = pa.P + lk; rho < pa.Ppad; rho += 4) put(rho, 0.f, 0.f);
}

// One strided DFT pass of the probe-sum adjoint: for every outer index o and
// window pixel r < W2,
//   out[k ks + o os2 + r] = sum_j T[(j k) mod S] in[j js + o os + r],
// with T = exp(+2 pi i k/S) (the conjugate of the synthesis twiddles).
__global__ __launch_bounds__(NT) void k_dft_pass(const float2* __restrict__ in, float2* out, int S,
                                                 int64_t js, int64_t os, int64_t ks, int64_t os2,
                                                 int W2, const float2* __restrict__ tws) {
  extern __shared__ float2 sm[];
  float2* sF = sm;
  float2* sT = sm + ((S + 3) & ~3) * RT;
  const int o = blockIdx.y;
  const int r0 = blockIdx.x * RT;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int i = threadIdx.x; i < S; i += NT) sT[i] = tws[i];
  const int r = r0 + lane;
  // this wave's rows, 16 loads in flight before their LDS stores
  const int Sc = (S + 3) & ~3;
  for (int j0 = wave; j0 < Sc; j0 += 64) {
    float2 v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = j0 + 4 * q;
      v[q] = (r < W2 && j < S) ? in[(int64_t)j * js + (int64_t)o * os + r] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = j0 + 4 * q;
      if (j < Sc) sF[j * RT + lane] = v[q];
    }
  }
  __syncthreads();
  const int li = lane & 15, lk = lane >> 4;
  const int ro = r0 + 16 * wave + li;
  for (int k0 = 0; k0 < S; k0 += 64) {
    v4f xr[4], xi[4];
    dft_mfma(sF, sT, S, k0, wave, lane, xr, xi);
    if (ro < W2) {
#pragma unroll
      for (int ob = 0; ob < 4; ++ob)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int k = k0 + 16 * ob + 4 * lk + q;
          if (k < S) out[(int64_t)k * ks + (int64_t)o * os2 + ro] = make_float2(xr[ob][q], xi[ob][q]);
        }
    }
  }
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

size_t probe_lds_bytes(int S) { return (size_t)(((S + 3) & ~3) * RT + S) * sizeof(float2); }

hipError_t launch_dft_pass(const float2* in, float2* out, int S, int64_t js, int64_t os, int64_t ks,
                          int64_t os2, int n_outer, int W2, const float2* tws, hipStream_t s) {
  if (n_outer <= 0 || W2 <= 0) return hipSuccess;
  const size_t lds = probe_lds_bytes(S);
  hipError_t e = hipFuncSetAttribute((const void*)k_dft_pass,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dft_pass, dim3((W2 + RT - 1) / RT, n_outer), dim3(NT), lds, s, in, out, S,
                     js, os, ks, os2, W2, tws);
  return hipGetLastError();
}

hipError_t launch_probe_fold_x(const ProbeArgs& pa, int unit0, int n_units, int n_jobs, hipStream_t s) {
  if (n_jobs <= 0 || n_units <= 0) return hipSuccess;
  if (unit0 < 0 || pa.Sy < 1) return hipErrorInvalidValue;
  const int64_t blocks = (int64_t)((n_units + 7) / 8) * 8 * pa.Sy;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  ProbeArgs q = pa;
  q.unit0 = unit0;
  q.n_units = n_units;
  q.n_jobs = n_jobs;
  const size_t lds = ((size_t)std::min((pa.Sx + 3) & ~3, FOLD_CH) * RT + pa.Sx + pa.L) * sizeof(float2);
  switch ((pa.Sx + 63) / 64) {
    case 1: return launch_lds(k_probe_fold_x<1>, dim3((unsigned)blocks), lds, q, s);
    case 2: return launch_lds(k_probe_fold_x<2>, dim3((unsigned)blocks), lds, q, s);
    case 3: return launch_lds(k_probe_fold_x<3>, dim3((unsigned)blocks), lds, q, s);
    case 4: return launch_lds(k_probe_fold_x<4>, dim3((unsigned)blocks), lds, q, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_probe_y(const ProbeArgs& pa, int prec, bool u, int max_kd, int n_jobs,
                          hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  const dim3 grid((unsigned)((max_kd + RT - 1) / RT), (unsigned)pa.Sx, (unsigned)n_jobs);
  const size_t lds = ((size_t)std::min((pa.Sy + 3) & ~3, FOLD_CH) * RT + pa.Sy) * sizeof(float2);
  const int nv = (pa.Sy + 63) / 64;
#define PYV(P, UU, NV) \
  if (nv == NV) return launch_lds(k_probe_y<P, UU, NV>, grid, lds, pa, s);
#define PY(P)                                                                                  \
  if (prec == P) {                                                                             \
    if (u) {                                                                                   \
      PYV(P, true, 1) PYV(P, true, 2) PYV(P, true, 3) PYV(P, true, 4)                          \
    } else {                                                                                   \
      PYV(P, false, 1) PYV(P, false, 2) PYV(P, false, 3) PYV(P, false, 4)                      \
    }                                                                                          \
    return hipErrorInvalidValue;                                                               \
  }
  PY(BIP_PREC_FP32)
  PY(BIP_PREC_SPLIT_BF16)
  PY(BIP_PREC_BF16)
  PY(BIP_PREC_FP16)
#undef PY
#undef PYV
  return hipErrorInvalidValue;
}

}  // namespace bip
