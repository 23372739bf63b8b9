// Multislice passes over batches of parent columns (step a).
//
// A slice step psi <- F^-1[P F[T_j psi]] (eq. propagator, eq.
// smatrix-advance) is split into two HBM passes over the column stack:
//   row pass:    [row inverse FFT] -> [window gather] -> x T_j -> [gather]
//                -> [row FFT]
//   column pass: column FFT -> x P(q)/G -> column inverse FFT
// Between passes the state is kept row-transformed (F_row psi), so a row pass
// fuses the inverse row transform of one step with the forward row transform
// of the next, and the real-space wave is only ever materialized in
// registers -- which is where the ionized atoms' windows are cropped.  The S2
// sweep (transpose multislice, eq. s2) runs the same passes in the other
// order (column pass, then row pass with T after the propagation).
#include "fft_core.h"

namespace bip {

namespace {

template <int NX>
struct RowShape {
  static constexpr int T = NX / 16;            // threads per row transform
  static constexpr int ROWS = 256 / T;         // rows per block
  static constexpr int LDS_ROW = NX + NX / 16; // padded complex elements per row
};

constexpr int GREC_LDS = 64;  // gather records of a plane staged in LDS

// Crop the real-space row segment that falls into the windows of the atoms
// of this plane; de-tilt by exp(-sign 2 pi i h_p.r/N) on the way.  Records
// q < GREC_LDS come from LDS, the rest from memory.
template <int NX>
__device__ inline void gather_row(const float2 (&v)[16], int t, int y, int col, int ny,
                                  const GatherArgs& ga, const GatherRec* srec, int gb, int ge,
                                  int2 hp, const float2* __restrict__ tw, int L, int sign) {
  constexpr int T = RowShape<NX>::T;
  const int my = hp.x * y * (L / ny);
  for (int q = 0; q < ge - gb; ++q) {
    const GatherRec g = q < GREC_LDS ? srec[q] : ga.rec[gb + q];
    int ry = y - g.oy;
    if (ry < 0) ry += ny;
    if (ry >= g.W) continue;
    float2* dst = ga.win + g.off + ((int64_t)col * g.W + ry) * g.W;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int x = t + T * e;
      int rx = x - g.ox;
      if (rx < 0) rx += NX;
      if (rx < g.W) {
        const int m = (my + hp.y * x * (L / NX)) & (L - 1);
        const float2 w = tw[m];  // exp(-2 pi i h_p.r/N)
        dst[rx] = sign > 0 ? cmul(v[e], w) : cmulc(v[e], w);
      }
    }
  }
}

template <int NX, int FLAGS>
__global__ __launch_bounds__(256) void k_row_pass(float2* __restrict__ state, int ny,
                                                  const float2* __restrict__ T,
                                                  const float2* __restrict__ twg, int L,
                                                  const int2* __restrict__ parents, int sign,
                                                  GatherArgs ga, int gb, int ge, int col0,
                                                  float2* __restrict__ save) {
  using S = RowShape<NX>;
  __shared__ float2 lds[S::ROWS * S::LDS_ROW];
  extern __shared__ float2 tw[];  // [L] twiddle table
  __shared__ GatherRec srec[(FLAGS & (ROW_GATHER_BEFORE_T | ROW_GATHER_AFTER_T)) ? GREC_LDS : 1];
  for (int i = threadIdx.x; i < L; i += 256) tw[i] = twg[i];
  if constexpr ((FLAGS & (ROW_GATHER_BEFORE_T | ROW_GATHER_AFTER_T)) != 0) {
    if ((int)threadIdx.x < ge - gb && threadIdx.x < GREC_LDS) srec[threadIdx.x] = ga.rec[gb + threadIdx.x];
  }
  // the only workgroup barrier: a row and its LDS row belong to one wave, so
  // the transforms order their exchanges per wave
  __syncthreads();
  const int t = threadIdx.x % S::T;
  const int f = threadIdx.x / S::T;
  const int y = blockIdx.x * S::ROWS + f;
  const int col = blockIdx.y;   // column of this launch's batch
  const int pcol = col0 + col;  // parent index
  float2* row = state + ((int64_t)col * ny + y) * NX;
  float2* my_lds = lds + f * S::LDS_ROW;
  float2 v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) v[e] = row[t + S::T * e];
  if (FLAGS & ROW_INV) fft::transform<NX, true, 1, true, true>(v, my_lds, t, tw, L);
  if constexpr ((FLAGS & ROW_GATHER_BEFORE_T) != 0) {
    if (ge > gb) gather_row<NX>(v, t, y, pcol, ny, ga, srec, gb, ge, parents[pcol], tw, L, sign);
  }
  if (FLAGS & ROW_T) {
    const float2* Trow = T + (int64_t)y * NX;
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = cmul(v[e], Trow[t + S::T * e]);
  }
  if constexpr ((FLAGS & ROW_SAVE) != 0) {  // slice checkpoint: the state after T_j
    float2* srow = save + ((int64_t)col * ny + y) * NX;
#pragma unroll
    for (int e = 0; e < 16; ++e) srow[t + S::T * e] = v[e];
  }
  if constexpr ((FLAGS & ROW_GATHER_AFTER_T) != 0) {
    if (ge > gb) gather_row<NX>(v, t, y, pcol, ny, ga, srec, gb, ge, parents[pcol], tw, L, sign);
  }
  if (FLAGS & ROW_FWD) {
    fft::transform<NX, false, 1, true, true>(v, my_lds, t, tw, L);
#pragma unroll
    for (int e = 0; e < 16; ++e) row[t + S::T * e] = v[e];
  }
}

// Scatter-add of window cotangents into a real-space row (adjoint of the
// gather; the cotangents are already multiplied by the conjugate de-tilt).
template <int NX>
__device__ inline void inject_row(float2 (&v)[16], int t, int y, int col, int ny,
                                  const GatherArgs& ga, const GatherRec* srec, int gb, int ge) {
  constexpr int T = RowShape<NX>::T;
  for (int q = 0; q < ge - gb; ++q) {
    const GatherRec g = q < GREC_LDS ? srec[q] : ga.rec[gb + q];
    int ry = y - g.oy;
    if (ry < 0) ry += ny;
    if (ry >= g.W) continue;
    const float2* src = ga.win + g.off + ((int64_t)col * g.W + ry) * g.W;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int x = t + T * e;
      int rx = x - g.ox;
      if (rx < 0) rx += NX;
      if (rx < g.W) v[e] = cadd(v[e], src[rx]);
    }
  }
}

// Adjoint row pass over the columns of one batch (reverse sweeps).  The state
// holds the cotangent of the parent columns, row-transformed between passes
// like the forward state.  Per column, in order: [load or start from zero]
// -> [row inverse FFT] -> [inject window cotangents] -> [slice-potential
// gradient against the checkpointed forward state after T_j] -> [x conj(T_j)]
// -> [inject] -> [row FFT, store].  A workgroup owns ROWS rows and the
// columns cg, cg + CG, ...: it sums the gradient over its columns in
// registers and writes one partial row block, reduced later in a fixed order.
// dL/dV_j(r) = 2 Re[conj(c(r)) i sigma f(r)] = 2 sigma (c_im f_re - c_re f_im)
// with c the cotangent and f the forward state after T_j.
template <int NX, int FLAGS>
__global__ __launch_bounds__(256) void k_row_adjoint(float2* __restrict__ state, int ny, int ncols,
                                                     const float2* __restrict__ T,
                                                     const float2* __restrict__ twg, int L,
                                                     GatherArgs inj, int gb, int ge, int col0,
                                                     const float2* __restrict__ ckpt,
                                                     float two_sigma, float* __restrict__ dv_partial) {
  using S = RowShape<NX>;
  __shared__ float2 lds[S::ROWS * S::LDS_ROW];
  __shared__ GatherRec srec[GREC_LDS];
  extern __shared__ float2 tw[];  // [L]
  if ((int)threadIdx.x < ge - gb && threadIdx.x < GREC_LDS) srec[threadIdx.x] = inj.rec[gb + threadIdx.x];
  for (int i = threadIdx.x; i < L; i += 256) tw[i] = twg[i];
  __syncthreads();
  const int t = threadIdx.x % S::T;
  const int f = threadIdx.x / S::T;
  const int y = blockIdx.x * S::ROWS + f;
  float2* my_lds = lds + f * S::LDS_ROW;
  float dv[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) dv[e] = 0.f;
  for (int col = blockIdx.y; col < ncols; col += gridDim.y) {
    const int pcol = col0 + col;
    float2* row = state + ((int64_t)col * ny + y) * NX;
    float2 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = (FLAGS & ADJ_ZERO) ? make_float2(0.f, 0.f) : row[t + S::T * e];
    if constexpr ((FLAGS & ADJ_INV) != 0) fft::transform<NX, true, 1, true, true>(v, my_lds, t, tw, L);
    if constexpr ((FLAGS & ADJ_INJ_BEFORE) != 0)
      if (ge > gb) inject_row<NX>(v, t, y, pcol, ny, inj, srec, gb, ge);
    if constexpr ((FLAGS & ADJ_DV) != 0) {
      const float2* fr = ckpt + ((int64_t)col * ny + y) * NX;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const float2 fw = fr[t + S::T * e];
        dv[e] += two_sigma * (v[e].y * fw.x - v[e].x * fw.y);
      }
    }
    if constexpr ((FLAGS & ADJ_CONJT) != 0) {
      const float2* Trow = T + (int64_t)y * NX;
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = cmulc(v[e], Trow[t + S::T * e]);
    }
    if constexpr ((FLAGS & ADJ_INJ_AFTER) != 0)
      if (ge > gb) inject_row<NX>(v, t, y, pcol, ny, inj, srec, gb, ge);
    if constexpr ((FLAGS & ADJ_FWD) != 0) {
      fft::transform<NX, false, 1, true, true>(v, my_lds, t, tw, L);
#pragma unroll
      for (int e = 0; e < 16; ++e) row[t + S::T * e] = v[e];
    }
  }
  if constexpr ((FLAGS & ADJ_DV) != 0) {
    float* pr = dv_partial + ((int64_t)blockIdx.y * ny + y) * NX;
#pragma unroll
    for (int e = 0; e < 16; ++e) pr[t + S::T * e] = dv[e];
  }
}

// dV[i] += sum_{g < n_groups} partial[g][i], groups in order.
__global__ void k_dv_reduce(const float* __restrict__ partial, int n_groups, int64_t n, float* dv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int g = 0; g < n_groups; ++g) s += partial[(int64_t)g * n + i];
  dv[i] += s;
}

template <int NY>
struct ColShape {
  static constexpr int T = NY / 16;                       // threads per column transform
  // adjacent columns per block (measured: 16 at 256 and 1024, 8 at 512)
  static constexpr int CB = NY == 512 ? 8 : (NY >= 256) ? 16 : 4096 / NY;
  static constexpr int THREADS = CB * T;
};

template <int NY>
__global__ __launch_bounds__(ColShape<NY>::THREADS) void k_col_pass(
    float2* __restrict__ state, int nx, const float2* __restrict__ prop,
    const float2* __restrict__ twg, int L) {
  using S = ColShape<NY>;
  __shared__ float2 lds[S::CB * NY];
  extern __shared__ float2 tw[];  // [L] twiddle table: the transforms' barriers order the fill
  for (int i = threadIdx.x; i < L; i += S::THREADS) tw[i] = twg[i];
  const int c = threadIdx.x % S::CB;
  const int t = threadIdx.x / S::CB;
  const int x = blockIdx.x * S::CB + c;
  const int col = blockIdx.y;
  float2* base = state + (int64_t)col * NY * nx + x;
  float2 v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) v[e] = base[(int64_t)(t + S::T * e) * nx];
  fft::transform<NY, false, S::CB, false>(v, lds + c, t, tw, L);
#pragma unroll
  for (int e = 0; e < 16; ++e) v[e] = cmul(v[e], prop[(int64_t)(t + S::T * e) * nx + x]);
  fft::transform<NY, true, S::CB, false>(v, lds + c, t, tw, L);
#pragma unroll
  for (int e = 0; e < 16; ++e) base[(int64_t)(t + S::T * e) * nx] = v[e];
}

template <int NX, int FLAGS>
hipError_t row_launch(float2* state, int ncols, int ny, const float2* T, const float2* tw, int L,
                      const int2* parents, int sign, const GatherArgs& ga, int gb, int ge,
                      int col0, float2* save, hipStream_t s) {
  using S = RowShape<NX>;
  dim3 grid(ny / S::ROWS, ncols);
  hipLaunchKernelGGL((k_row_pass<NX, FLAGS>), grid, dim3(256), L * sizeof(float2), s, state, ny, T, tw, L, parents,
                     sign, ga, gb, ge, col0, save);
  return hipGetLastError();
}

template <int NX>
hipError_t row_dispatch(int flags, float2* state, int ncols, int ny, const float2* T,
                        const float2* tw, int L, const int2* parents, int sign,
                        const GatherArgs& ga, int gb, int ge, int col0, float2* save,
                        hipStream_t s) {
#define ROW_CASE(F) \
  case F:           \
    return row_launch<NX, F>(state, ncols, ny, T, tw, L, parents, sign, ga, gb, ge, col0, save, s);
  switch (flags) {
    ROW_CASE(ROW_GATHER_BEFORE_T | ROW_T | ROW_FWD | ROW_SAVE)
    ROW_CASE(ROW_INV | ROW_GATHER_BEFORE_T | ROW_T | ROW_FWD | ROW_SAVE)
    ROW_CASE(ROW_INV | ROW_T | ROW_GATHER_AFTER_T | ROW_FWD | ROW_SAVE)
    ROW_CASE(ROW_INV | ROW_T | ROW_GATHER_AFTER_T | ROW_SAVE)
    ROW_CASE(ROW_T | ROW_GATHER_AFTER_T | ROW_SAVE)
    ROW_CASE(ROW_GATHER_BEFORE_T | ROW_T | ROW_FWD)
    ROW_CASE(ROW_INV | ROW_GATHER_BEFORE_T | ROW_T | ROW_FWD)
    ROW_CASE(ROW_INV | ROW_GATHER_BEFORE_T)
    ROW_CASE(ROW_GATHER_BEFORE_T)
    ROW_CASE(ROW_FWD)
    ROW_CASE(ROW_INV | ROW_T | ROW_FWD | ROW_SAVE)  // recomputing a checkpoint segment
    ROW_CASE(ROW_INV | ROW_T | ROW_GATHER_AFTER_T | ROW_FWD)
    ROW_CASE(ROW_INV | ROW_T | ROW_GATHER_AFTER_T)
    ROW_CASE(ROW_T | ROW_GATHER_AFTER_T)
    default:
      return hipErrorInvalidValue;
  }
#undef ROW_CASE
}

template <int NX, int FLAGS>
hipError_t adj_launch(float2* state, int ncols, int ny, const float2* T, const float2* tw, int L,
                      const GatherArgs& inj, int gb, int ge, int col0, const float2* ckpt,
                      float two_sigma, float* dv_partial, int groups, hipStream_t s) {
  using S = RowShape<NX>;
  hipLaunchKernelGGL((k_row_adjoint<NX, FLAGS>), dim3(ny / S::ROWS, groups), dim3(256), L * sizeof(float2), s,
                     state, ny, ncols, T, tw, L, inj, gb, ge, col0, ckpt, two_sigma, dv_partial);
  return hipGetLastError();
}

template <int NX>
hipError_t adj_dispatch(int flags, float2* state, int ncols, int ny, const float2* T,
                        const float2* tw, int L, const GatherArgs& inj, int gb, int ge, int col0,
                        const float2* ckpt, float two_sigma, float* dv_partial, int groups,
                        hipStream_t s) {
#define ADJ_CASE(F) \
  case F:           \
    return adj_launch<NX, F>(state, ncols, ny, T, tw, L, inj, gb, ge, col0, ckpt, two_sigma, dv_partial, groups, s);
  switch (flags) {
    ADJ_CASE(ADJ_ZERO | ADJ_INJ_AFTER | ADJ_FWD)                              // S1, deepest plane
    ADJ_CASE(ADJ_INV | ADJ_DV | ADJ_CONJT | ADJ_INJ_AFTER | ADJ_FWD)          // S1, slice j > 0
    ADJ_CASE(ADJ_INV | ADJ_DV)                                                // S1 slice 0, S2 last
    ADJ_CASE(ADJ_ZERO | ADJ_INJ_BEFORE | ADJ_DV | ADJ_CONJT | ADJ_FWD)         // S2, shallowest plane
    ADJ_CASE(ADJ_ZERO | ADJ_INJ_BEFORE | ADJ_DV)                              // S2, single slice
    ADJ_CASE(ADJ_INV | ADJ_INJ_BEFORE | ADJ_DV | ADJ_CONJT | ADJ_FWD)          // S2, slice j
    ADJ_CASE(ADJ_INV | ADJ_INJ_BEFORE | ADJ_DV)                               // S2, exit slice
    default:
      return hipErrorInvalidValue;
  }
#undef ADJ_CASE
}

}  // namespace

hipError_t launch_row_adjoint(int flags, float2* state, int ncols, int ny, int nx, const float2* T,
                              const float2* tw, int L, const GatherArgs& inj, int gb, int ge,
                              int col0, const float2* ckpt, float two_sigma, float* dv_partial,
                              int groups, hipStream_t s) {
  if (ncols == 0) return hipSuccess;
  if (groups < 1 || ((flags & ADJ_DV) && (!ckpt || !dv_partial))) return hipErrorInvalidValue;
  switch (nx) {
    case 64: return adj_dispatch<64>(flags, state, ncols, ny, T, tw, L, inj, gb, ge, col0, ckpt, two_sigma, dv_partial, groups, s);
    case 128: return adj_dispatch<128>(flags, state, ncols, ny, T, tw, L, inj, gb, ge, col0, ckpt, two_sigma, dv_partial, groups, s);
    case 256: return adj_dispatch<256>(flags, state, ncols, ny, T, tw, L, inj, gb, ge, col0, ckpt, two_sigma, dv_partial, groups, s);
    case 512: return adj_dispatch<512>(flags, state, ncols, ny, T, tw, L, inj, gb, ge, col0, ckpt, two_sigma, dv_partial, groups, s);
    case 1024: return adj_dispatch<1024>(flags, state, ncols, ny, T, tw, L, inj, gb, ge, col0, ckpt, two_sigma, dv_partial, groups, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_dv_reduce(const float* partial, int n_groups, int64_t n, float* dv, hipStream_t s) {
  hipLaunchKernelGGL(k_dv_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, partial,
                     n_groups, n, dv);
  return hipGetLastError();
}

hipError_t launch_row_pass(int flags, float2* state, int ncols, int ny, int nx, const float2* T,
                           const float2* tw, int L, const int2* parents, int detilt_sign,
                           const GatherArgs& ga, int gather_begin, int gather_end, int col0,
                           float2* save, hipStream_t s) {
  if (ncols == 0) return hipSuccess;
  if ((flags & ROW_SAVE) && !save) return hipErrorInvalidValue;
  switch (nx) {
    case 64: return row_dispatch<64>(flags, state, ncols, ny, T, tw, L, parents, detilt_sign, ga, gather_begin, gather_end, col0, save, s);
    case 128: return row_dispatch<128>(flags, state, ncols, ny, T, tw, L, parents, detilt_sign, ga, gather_begin, gather_end, col0, save, s);
    case 256: return row_dispatch<256>(flags, state, ncols, ny, T, tw, L, parents, detilt_sign, ga, gather_begin, gather_end, col0, save, s);
    case 512: return row_dispatch<512>(flags, state, ncols, ny, T, tw, L, parents, detilt_sign, ga, gather_begin, gather_end, col0, save, s);
    case 1024: return row_dispatch<1024>(flags, state, ncols, ny, T, tw, L, parents, detilt_sign, ga, gather_begin, gather_end, col0, save, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_col_pass(float2* state, int ncols, int ny, int nx, const float2* prop,
                           const float2* tw, int L, hipStream_t s) {
  if (ncols == 0) return hipSuccess;
#define COL_CASE(N)                                                                  \
  case N: {                                                                          \
    using S = ColShape<N>;                                                           \
    if (nx % S::CB) return hipErrorInvalidValue;                                     \
    hipLaunchKernelGGL(k_col_pass<N>, dim3(nx / S::CB, ncols), dim3(S::THREADS), L * sizeof(float2), s, \
                       state, nx, prop, tw, L);                                      \
    return hipGetLastError();                                                        \
  }
  switch (ny) {
    COL_CASE(64)
    COL_CASE(128)
    COL_CASE(256)
    COL_CASE(512)
    COL_CASE(1024)
    default:
      return hipErrorInvalidValue;
  }
#undef COL_CASE
}

}  // namespace bip
