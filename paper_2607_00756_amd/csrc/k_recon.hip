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
    m += w * habs(D);
  }
  const float2 s = a.mode == BIP_RECON_MAGNITUDE ? mag_rescale(z, m) : z;
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

// GEMM operand output, one tile of 64 beams per workgroup, 32 pixels at a time.
// kind 0: S2~^T for the Gram matrix, K-blocked: element (r, b) at
//         ((b / KB) nrows + r) KB + b mod KB, KB = beams per 64-byte row of a
//         plane, so each 64-byte column block is contiguous (ld unused)
// kind 1: element (b, r) at b*ld + r  (r fastest; S2~ for the detector contraction)
// The distinct parents of the tile's 64 beams (at most 64 for square-lattice
// parents) are staged in LDS, 32 pixels at a time, with coalesced 256-byte
// reads; the slab of the next 32 pixels is loaded into registers while the
// current one is combined, so every parent value is read from memory once and
// the weights are staged once per tile.  Each half-wave combines one beam on
// 32 consecutive pixels from LDS.  Kind 0 transposes through LDS so that each stored row holds
// 64 consecutive beams.  The small LDS footprint (~21 KB) keeps 7 workgroups
// per CU resident to hide the read latency.  Rows and columns beyond the beams
// or the window are written as zeros.
constexpr int TB = TILE_B, TR = 32;

template <int PREC, int KIND>
__global__ __launch_bounds__(256) void k_recon_operand(ReconArgs a, void* out, int64_t ld,
                                                       int nrows, int ncols, int64_t plane, int rpw) {
  __shared__ float2 tile[TB][TR + 1];
  __shared__ float2 sP[TILE_NP][TR];  // the tile's parent windows on the current 32 pixels
  __shared__ float sM[TILE_NP][TR];   // and their magnitudes
  extern __shared__ float2 s_tw[];    // exp(-2 pi i k/L), L entries
  __shared__ int s_ec[TB][ELL_W];
  __shared__ float s_ew[TB][ELL_W];
  __shared__ int2 s_h[TB];
  constexpr int NPF = TILE_NP * TR / 256;  // slab elements per thread
  const int n_b = KIND == 0 ? ncols : nrows;  // beams to write (padded)
  const int n_r = KIND == 0 ? nrows : ncols;  // pixels to write (padded)
  const int nbt = (n_b + TB - 1) / TB, nrt = (n_r + TR - 1) / TR;
  // one workgroup per beam tile and run of rpw pixel tiles.  Workgroup i runs
  // on XCD i mod 8: each XCD takes a contiguous range of (run, beam tile)
  // pairs, neighbouring beam tiles on the same pixels, so that the parents
  // they share stay in its L2
  const int nch = (nrt + rpw - 1) / rpw;
  const int per = (int)(gridDim.x / 8);
  const int lin = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (lin >= nbt * nch) return;
  const int bt = lin % nbt, ch = lin / nbt;
  const int rt_lo = ch * rpw, rt_hi = min(nrt, rt_lo + rpw);
  const int b0 = bt * TB;
  const int W2 = a.W * a.W;
  // the tile's distinct parents are staged in LDS when they fit (always, for
  // square-lattice parents); otherwise the parent reads go to memory
  int ts = 0, n_t = 0;
  if (b0 < a.nb) {
    ts = a.tstart[bt];
    n_t = a.tstart[bt + 1] - ts;
  }
  const bool fast = n_t <= TILE_NP;
  for (int i = threadIdx.x; i < TB * ELL_W; i += 256) {
    const int bl = i / ELL_W, j = i % ELL_W;
    const int64_t e = (int64_t)(b0 + bl) * ELL_W + j;
    const bool in = b0 + bl < a.nb;
    s_ec[bl][j] = in ? ((fast && j < ELL_K) ? a.ell_loc[e] : a.ellc[e]) : 0;
    s_ew[bl][j] = in ? a.ellw[e] : 0.f;
  }
  if (threadIdx.x < TB) s_h[threadIdx.x] = b0 + (int)threadIdx.x < a.nb ? a.beams[b0 + threadIdx.x] : make_int2(0, 0);
  for (int i = threadIdx.x; i < a.L; i += 256) s_tw[i] = a.tw[i];
  // parent slab of pixel tile rt: element i = (parent pi = i / TR, pixel i % TR)
  int prow[NPF];
#pragma unroll
  for (int q = 0; q < NPF; ++q) {
    const int i = threadIdx.x + 256 * q;
    prow[q] = (fast && i < n_t * TR) ? a.tpar[ts + i / TR] : -1;
  }
  float2 pre[NPF];
  auto load_slab = [&](int rt) {
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int r = rt * TR + ((threadIdx.x + 256 * q) % TR);
      pre[q] = (prow[q] >= 0 && r < W2) ? a.win[(int64_t)prow[q] * W2 + r] : make_float2(0.f, 0.f);
    }
  };
  auto store_slab = [&]() {
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int i = threadIdx.x + 256 * q;
      if (i < n_t * TR) {
        sP[i / TR][i % TR] = pre[q];
        sM[i / TR][i % TR] = habs(pre[q]);
      }
    }
  };
  load_slab(rt_lo);
  store_slab();
  if (rt_lo + 1 < rt_hi) load_slab(rt_lo + 1);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int half = lane >> 5, px32 = lane & 31;
  for (int rt = rt_lo; rt < rt_hi; ++rt) {
    const int r0 = rt * TR;
    const int r = r0 + px32;
    const bool live = r < W2;
    const int rr = live ? r : 0;
    const int ry = rr / a.W, rx = rr - ry * a.W;
    const int py = ((a.oy + ry) & (a.ny - 1)) * (a.L / a.ny);
    const int px = ((a.ox + rx) & (a.nx - 1)) * (a.L / a.nx);
    if (fast) {
      // parent values and magnitudes from the slab
#pragma unroll 2
      for (int k = 0; k < TB / 8; ++k) {
        const int bl = 2 * wave + half + 8 * k;
        const int2 h = s_h[bl];
        const float2 tw = s_tw[(h.x * py + h.y * px) & (a.L - 1)];  // exp(-2 pi i h.r/N)
        float2 z = make_float2(0.f, 0.f);
        float m = 0.f;
#pragma unroll
        for (int j = 0; j < ELL_K; ++j) {
          const int c = s_ec[bl][j];
          const float wj = s_ew[bl][j];
          const float2 d = sP[c][px32];
          z.x += wj * d.x;
          z.y += wj * d.y;
          m += wj * sM[c][px32];
        }
        recon_tail(z, m, a.win, W2, rr, s_ec[bl], a.col, a.w);
        const float2 sv = a.mode == BIP_RECON_MAGNITUDE ? mag_rescale(z, m) : z;
        float2 v = make_float2(0.f, 0.f);
        if (b0 + bl < a.nb && live) v = cscale(a.retilt_sign > 0 ? cmulc(sv, tw) : cmul(sv, tw), a.scale);
        tile[bl][px32] = v;
      }
    } else {
      // four beams per batch: all their parent reads are issued before any of
      // them is combined
      constexpr int NBATCH = 4;
      for (int k0 = 0; k0 < TB / 8; k0 += NBATCH) {
        float2 D[NBATCH][ELL_K];
#pragma unroll
        for (int i = 0; i < NBATCH; ++i) recon_load(a.win, W2, rr, s_ec[2 * wave + half + 8 * (k0 + i)], D[i]);
#pragma unroll
        for (int i = 0; i < NBATCH; ++i) {
          const int bl = 2 * wave + half + 8 * (k0 + i);
          const int2 h = s_h[bl];
          const float2 tw = s_tw[(h.x * py + h.y * px) & (a.L - 1)];
          const float2 sv = recon_finish(D[i], a.win, W2, rr, s_ec[bl], s_ew[bl], a.col, a.w, a.mode);
          float2 v = make_float2(0.f, 0.f);
          if (b0 + bl < a.nb && live) v = cscale(a.retilt_sign > 0 ? cmulc(sv, tw) : cmul(sv, tw), a.scale);
          tile[bl][px32] = v;
        }
      }
    }
    __syncthreads();  // tile complete, slab of rt consumed
    if (rt + 1 < rt_hi) {
      store_slab();                        // slab rt + 1, loaded during the compute of rt
      if (rt + 2 < rt_hi) load_slab(rt + 2);
    }
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
    __syncthreads();  // tile read out, next slab visible
  }
}

// K-blocked GEMM operand (kind 0) when every 64-beam tile has at most
// TILE_NP distinct parents: one lane per target beam.  A workgroup owns 64
// beams and a run of 32-pixel slabs; the slab of the tile's parent windows
// (values and magnitudes, rows padded to 33 so that lanes on different parents
// fall in different banks) is staged in LDS, the next one prefetched into
// registers meanwhile.  Every lane keeps its beam's six slot offsets and
// weights in registers for the whole run; wave w combines slab pixels
// 8w .. 8w+7, all lanes on the same pixel, so the slab reads take immediate
// offsets and the stores of a wave cover 64 consecutive beams of one row.
constexpr int KR = 33;  // padded LDS row of the slab

// One beam tile bt of one atom over pixel tiles rt_lo .. rt_hi - 1 (a holds
// the atom's window; out its operand block).
template <int PREC>
__device__ inline void recon_kblk_tile(const ReconArgs& a, void* out, int n_r, int n_b, int64_t plane,
                                       int bt, int rt_lo, int rt_hi) {
  __shared__ float2 sP[TILE_NP][KR];
  __shared__ float sM[TILE_NP][KR];
  extern __shared__ float2 s_tw[];  // exp(-2 pi i k/L), L entries
  constexpr int NPF = TILE_NP * TR / 256;
  constexpr int KB = PREC == BIP_PREC_FP32 ? 16 : 32;  // beams per 64-byte block row
  const int b0 = bt * TB;
  const int W2 = a.W * a.W;
  // the wave index in a scalar register: the pixel of each step of the pixel
  // loop below (and its row, column and carrier offsets) is then wave-uniform
  // scalar work rather than per-lane vector work
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int ts = 0, n_t = 0;
  if (b0 < a.nb) {
    ts = a.tstart[bt];
    n_t = a.tstart[bt + 1] - ts;
  }
  for (int i = threadIdx.x; i < a.L; i += 256) s_tw[i] = a.tw[i];
  // this lane's beam: slot offsets (LDS bytes, including the wave's first
  // pixel), weights, CSR tail, carrier frequencies
  const int b = b0 + lane;
  const bool bvalid = b < a.nb;
  int oP[ELL_K], oM[ELL_K];
  float wt[ELL_K];
  int ec[ELL_W];
#pragma unroll
  for (int j = 0; j < ELL_K; ++j) {
    const int c = bvalid ? a.ell_loc[(int64_t)b * ELL_W + j] : 0;
    wt[j] = bvalid ? a.ellw[(int64_t)b * ELL_W + j] : 0.f;
    oP[j] = (c * KR + 8 * wave) * (int)sizeof(float2);
    oM[j] = (c * KR + 8 * wave) * (int)sizeof(float);
  }
  ec[6] = bvalid ? a.ellc[(int64_t)b * ELL_W + 6] : 0;
  ec[7] = bvalid ? a.ellc[(int64_t)b * ELL_W + 7] : 0;
  const int2 h = bvalid ? a.beams[b] : make_int2(0, 0);
  const int ky = h.x * (a.L / a.ny), kx = h.y * (a.L / a.nx);
  // slab rows: element i = (parent i / TR, pixel i % TR); each thread reads
  // pixel threadIdx.x % TR of parents threadIdx.x / TR + 8q (row pointers kept)
  const float2* prow[NPF];
#pragma unroll
  for (int q = 0; q < NPF; ++q) {
    const int i = threadIdx.x + 256 * q;
    prow[q] = i < n_t * TR ? a.win + (int64_t)a.tpar[ts + i / TR] * W2 + (threadIdx.x % TR) : nullptr;
  }
  float2 pre[NPF];
  auto load_slab = [&](int rt) {
    const int r = rt * TR + (int)(threadIdx.x % TR);
#pragma unroll
    for (int q = 0; q < NPF; ++q)
      pre[q] = (prow[q] && r < W2) ? prow[q][rt * TR] : make_float2(0.f, 0.f);
  };
  auto store_slab = [&]() {
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int i = threadIdx.x + 256 * q;
      if (i < n_t * TR) {
        sP[i / TR][i % TR] = pre[q];
        sM[i / TR][i % TR] = habs(pre[q]);
      }
    }
  };
  load_slab(rt_lo);
  store_slab();
  if (rt_lo + 1 < rt_hi) load_slab(rt_lo + 1);
  __syncthreads();
  const char* sPb = (const char*)&sP[0][0];
  const char* sMb = (const char*)&sM[0][0];
  const int64_t ob = (int64_t)(b / KB) * n_r * KB + b % KB;  // this lane's column of the blocks
  const bool bstore = b < n_b;
  // Lanes of padded beams have zero weights, so their outputs come out zero
  // without a select; pixels beyond the window and tiles of padded beams only
  // (no slab) store zeros.  The CSR tail is taken only by waves that hold a
  // row longer than six.
  const bool live = b0 < a.nb;
  const bool wave_tail = __ballot(ec[6] > ELL_K) != 0;
  const bool mag = a.mode == BIP_RECON_MAGNITUDE;
  const float sc = a.retilt_sign > 0 ? -a.scale : a.scale;  // conj(t) = (t.x, -t.y) via the sign
  constexpr int ES = PREC == BIP_PREC_FP32 ? 4 : 2;  // bytes per plane element
  for (int rt = rt_lo; rt < rt_hi; ++rt) {
    // this lane's output column at the wave's first pixel: the pixel loop
    // below stores at immediate offsets from it
    char* obase = (char*)out + (ob + (int64_t)(rt * TR + 8 * wave) * KB) * ES;
#pragma unroll
    for (int i = 0; i < TR / 4; ++i) {
      const int r = rt * TR + 8 * wave + i;  // window pixel (wave-uniform)
      if (r >= n_r) break;
      float2 v = make_float2(0.f, 0.f);
      if (live && r < W2) {
        const int ry = r / a.W, rx = r - ry * a.W;
        const int py = (a.oy + ry) & (a.ny - 1), px = (a.ox + rx) & (a.nx - 1);
        float2 z = make_float2(0.f, 0.f);
        float m = 0.f;
#pragma unroll
        for (int j = 0; j < ELL_K; ++j) {
          const float2 d = *(const float2*)(sPb + oP[j] + i * (int)sizeof(float2));
          const float dm = *(const float*)(sMb + oM[j] + i * (int)sizeof(float));
          z.x += wt[j] * d.x;
          z.y += wt[j] * d.y;
          m += wt[j] * dm;
        }
        if (wave_tail) recon_tail(z, m, a.win, W2, r, ec, a.col, a.w);
        if (mag) {
          // m z/|z| with the hardware reciprocal square root (0 where z = 0,
          // e.g. padded beams); 0 < |z|^2 < 1e-30 (no such lane in practice)
          // takes mag_rescale's exact path
          const float q = z.x * z.x + z.y * z.y;
          if (__ballot(q > 0.f && q < 1e-30f) != 0) {
            z = mag_rescale(z, m);
          } else {
            const float f = q > 0.f ? m * __builtin_amdgcn_rsqf(q) : 0.f;
            z.x *= f;
            z.y *= f;
          }
        }
        // re-tilt: z conj(t) (S1) or z t (S2), t = exp(-2 pi i h.r/N), times the operand scale
        const float2 tw = s_tw[(ky * py + kx * px) & (a.L - 1)];
        const float ti = sc * tw.y, tr = fabsf(sc) * tw.x;
        v.x = z.x * tr - z.y * ti;
        v.y = z.x * ti + z.y * tr;
      }
      if (bstore) store_planes<PREC>(obase, (int64_t)i * KB, plane, v.x, v.y);
    }
    __syncthreads();  // slab of rt consumed
    if (rt + 1 < rt_hi) {
      store_slab();
      if (rt + 2 < rt_hi) load_slab(rt + 2);
    }
    __syncthreads();  // next slab visible
  }
}

// One atom: a workgroup per beam tile and run of rpw pixel tiles.  Workgroup i
// runs on XCD i mod 8; each XCD takes a contiguous range of (run, beam tile)
// pairs, neighbouring beam tiles on the same pixels, so that the parents they
// share stay in its L2.
template <int PREC>
__global__ __launch_bounds__(256) void k_recon_kblk(ReconArgs a, void* out, int nrows, int ncols,
                                                    int64_t plane, int rpw) {
  const int nbt = (ncols + TB - 1) / TB, nrt = (nrows + TR - 1) / TR;
  const int nch = (nrt + rpw - 1) / rpw;
  const int per = (int)(gridDim.x / 8);
  const int lin = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (lin >= nbt * nch) return;
  const int bt = lin % nbt, ch = lin / nbt;
  recon_kblk_tile<PREC>(a, out, nrows, ncols, plane, bt, ch * rpw, min(nrt, ch * rpw + rpw));
}

// Every atom of a chunk in one launch: a workgroup per (atom, beam tile) over
// all the atom's pixel tiles; an XCD takes a contiguous range of them, so the
// beam tiles of one atom, which share parents, meet in its L2.
template <int PREC>
__global__ __launch_bounds__(256) void k_recon_kblk_atoms(ReconArgs a, const ReconAtom* __restrict__ atoms,
                                                          int n_atoms, char* out, int ncols,
                                                          int64_t plane) {
  const int nbt = (ncols + TB - 1) / TB;
  const int per = (int)(gridDim.x / 8);
  const int lin = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (lin >= nbt * n_atoms) return;
  const int bt = lin % nbt;
  const ReconAtom at = atoms[lin / nbt];
  a.win += at.win_off;
  a.W = at.W;
  a.oy = at.oy;
  a.ox = at.ox;
  constexpr int ES = PREC == BIP_PREC_FP32 ? 4 : 2;
  recon_kblk_tile<PREC>(a, out + at.out_off * ES, at.n_r, ncols, plane, bt, 0, (at.n_r + TR - 1) / TR);
}

}  // namespace

hipError_t launch_recon_kblk_atoms(const ReconArgs& a, const ReconAtom* atoms, int n_atoms, void* out,
                                   int prec, int64_t ncols_pad, int64_t plane_stride, hipStream_t s) {
  if (n_atoms <= 0 || ncols_pad <= 0) return hipSuccess;
  if (a.tile_np > TILE_NP || ncols_pad > INT32_MAX) return hipErrorInvalidValue;
  const int64_t nt = ((ncols_pad + TB - 1) / TB) * n_atoms;
  const int64_t nblk = (nt + 7) / 8 * 8;
  if (nblk > INT32_MAX) return hipErrorInvalidValue;
#define RA(P)                                                                                    \
  if (prec == P) {                                                                               \
    hipLaunchKernelGGL((k_recon_kblk_atoms<P>), dim3((unsigned)nblk), dim3(256),                 \
                       a.L * sizeof(float2), s, a, atoms, n_atoms, (char*)out, (int)ncols_pad,   \
                       plane_stride);                                                            \
    return hipGetLastError();                                                                    \
  }
  RA(BIP_PREC_FP32)
  RA(BIP_PREC_SPLIT_BF16)
  RA(BIP_PREC_BF16)
  RA(BIP_PREC_FP16)
#undef RA
  return hipErrorInvalidValue;
}

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
  const int64_t nbt = (n_b + TB - 1) / TB, nrt = (n_r + TR - 1) / TR;
  // runs of pixel tiles long enough to reuse the staged weights, short
  // enough that the launch still has about 2048 workgroups
  const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(nrt, (2048 + nbt - 1) / nbt));
  const int64_t rpw = (nrt + nch - 1) / nch;
  const int64_t nt = nbt * ((nrt + rpw - 1) / rpw);
  const int64_t nblk = (nt + 7) / 8 * 8;
  if (nblk > INT32_MAX) return hipErrorInvalidValue;
  dim3 grid((unsigned)nblk), block(256);
  if (kind == 0 && a.tile_np <= TILE_NP) {
#define RK(P)                                                                                    \
  if (prec == P) {                                                                               \
    hipLaunchKernelGGL((k_recon_kblk<P>), grid, block, a.L * sizeof(float2), s, a, out,          \
                       (int)nrows_pad, (int)ncols_pad, plane_stride, (int)rpw);                  \
    return hipGetLastError();                                                                    \
  }
    RK(BIP_PREC_FP32)
    RK(BIP_PREC_SPLIT_BF16)
    RK(BIP_PREC_BF16)
    RK(BIP_PREC_FP16)
#undef RK
    return hipErrorInvalidValue;
  }
#define RC(P, K)                                                                            \
  if (prec == P && kind == K) {                                                             \
    hipLaunchKernelGGL((k_recon_operand<P, K>), grid, block, a.L * sizeof(float2), s, a, out, ld, (int)nrows_pad, \
                       (int)ncols_pad, plane_stride, (int)rpw);                             \
    return hipGetLastError();                                                               \
  }
  RC(BIP_PREC_FP32, 0)
  RC(BIP_PREC_FP32, 1)
  RC(BIP_PREC_SPLIT_BF16, 0)
  RC(BIP_PREC_SPLIT_BF16, 1)
  RC(BIP_PREC_BF16, 0)
  RC(BIP_PREC_BF16, 1)
  RC(BIP_PREC_FP16, 0)
  RC(BIP_PREC_FP16, 1)
#undef RC
  return hipErrorInvalidValue;
}

}  // namespace bip
