// Complex contractions on the matrix cores (step c).
//
// Every contraction is an "NT" complex product C[m][n] = sum_k A[m][k] B[n][k]
// (optionally with conj(A)), K running along the rows of both operands, each
// operand stored as separate real planes:
//   FP32        : re, im                          (v_mfma_f32_16x16x4_f32)
//   SPLIT_BF16  : re_hi, re_lo, im_hi, im_lo       (v_mfma_f32_16x16x32_bf16;
//                 hi*hi + hi*lo + lo*hi per real product, FP32 accumulate)
//   BF16        : re, im                          (v_mfma_f32_16x16x32_bf16)
//   FP16        : re, im                          (v_mfma_f32_16x16x32_f16)
// A complex product is four real products; the minus sign of re*re - im*im is
// applied by flipping the sign bit of the A imaginary fragment.
//
// Tiling: a workgroup of 4 wave64s owns a 128 x 128 output tile (each wave a
// 64 x 64 sub-tile of 4 x 4 MFMA blocks).  K advances in 64-byte chunks per
// plane row (16 FP32 or 32 BF16 values); consecutive chunks of a row are
// either adjacent (K contiguous) or a fixed stride apart (K-blocked operands,
// where every 64-byte column block of the matrix is stored contiguously).  Operand chunks move from global
// memory straight into LDS with global_load_lds_dwordx4 (no VGPR staging),
// double buffered, one barrier per chunk; the 16-byte slots of each LDS row
// are XOR-permuted (swz) so that the 16 rows read by one MFMA fragment load
// hit distinct banks.
//
// Roles (epilogues):
//   EPI_ABS2_MAP / EPI_ABS2_BEAMS
//              a_d(rho) = sum_r S2~^d(r) U_n(r, rho), U_n = H_n psi from the
//              probe synthesis; |a|^2 accumulated over
//              the (atom, channel) jobs in registers, then summed over d (map)
//              or added into [rho][d] (beams)
//   EPI_GRAMQ  G[r][r'] = sum_d conj(S2~^d(r)) S2~^d(r') and its product with
//              sum_n conj(H_n(r)) H_n(r') -> Q (operand of EPI_QUAD)
//   EPI_QUAD   (Q psi)(r, rho); I(rho) += Re sum_r conj(psi(r, rho)) (Q psi)(r, rho)
//              accumulated over atoms, then summed over the tile's r
//   EPI_STORE  the product itself as complex64 (optionally scaled per row):
//              the contractions of the map-loss gradient
// For the map, sum_n sum_d |a_d|^2 = psi^H Q psi exactly, which replaces the
// n_det x N_ch P detector contraction by a W^2 x W^2 Gram matrix per atom.
#include "bip_internal.h"
#include "planes.h"

namespace bip {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

template <int PREC>
struct PT;
template <>
struct PT<BIP_PREC_FP32> {
  static constexpr int PLANES = 2, ESZ = 4, BK = 16;
};
template <>
struct PT<BIP_PREC_SPLIT_BF16> {
  static constexpr int PLANES = 4, ESZ = 2, BK = 32;
};
template <>
struct PT<BIP_PREC_BF16> {
  static constexpr int PLANES = 2, ESZ = 2, BK = 32;
};
template <>
struct PT<BIP_PREC_FP16> {
  static constexpr int PLANES = 2, ESZ = 2, BK = 32;
};

constexpr int BM = 128, BN = 128, NTHREADS = 256;
constexpr int PLANE_TILE = 128 * 64;  // bytes of one plane of one operand tile chunk

template <int PREC>
constexpr int stage_bytes() {
  return 2 * PT<PREC>::PLANES * PLANE_TILE;
}
// Workgroups per CU the kernel is built for.  The Gram and plain-store
// products of two-plane operands run two workgroups (two waves per SIMD, at
// most 256 registers per lane each), so that one workgroup's barrier and
// fragment-load waits are covered by the other's matrix work; the other
// roles keep one, with their larger register sets (running sums, split
// planes).
template <int PREC, int EPI>
constexpr int occupancy() {
  return (EPI == EPI_GRAMQ || EPI == EPI_STORE) && PT<PREC>::PLANES == 2 && PREC != BIP_PREC_FP32 ? 2 : 1;
}
// The FP32 Gram matrix sums its K products (all detector beams) in segments
// of KSEG: each segment in its own accumulators, added to a running total.
// v_mfma_f32_16x16x4f32 rounds the accumulator every 4 products, so an
// unsegmented sum over 10^5 beams rounds ~5*10^4 times per element; the
// segments bound that to KSEG/4 + K/KSEG.  (The 16-bit products accumulate
// 32 products per rounding and are not segmented.)
template <int PREC, int EPI>
constexpr bool k_segmented() {
  return EPI == EPI_GRAMQ && PREC == BIP_PREC_FP32;
}
constexpr int KSEG = 2048;
// K chunks in flight.  One workgroup per CU: the chunk buffers fill 128 KB of
// LDS (two 64 KB stages for the four split planes, four 32 KB stages
// otherwise), so that a chunk's loads have NSTAGE - 1 chunks of matrix work
// to land.  Two per CU: two 32 KB stages each (64 KB), the loads of the next
// chunk landing under the current chunk's work of both workgroups.
template <int PREC, int EPI>
constexpr int nstage() {
  return occupancy<PREC, EPI>() == 2 ? 2 : (PT<PREC>::PLANES == 4 ? 2 : 4);
}
template <int PREC, int EPI>
constexpr int lds_bytes() {
  return nstage<PREC, EPI>() * stage_bytes<PREC>();
}

// The quadratic form's epilogue stages the job's psi^T tile [128 rho][128 r]
// in LDS once the K loop is done, rows padded by 16 bytes against bank
// conflicts of the per-lane reads.
template <int PREC>
constexpr int quad_row() {
  return BN + 16 / PT<PREC>::ESZ;
}
template <int PREC>
constexpr int quad_lds_bytes() {
  return PT<PREC>::PLANES * BM * quad_row<PREC>() * PT<PREC>::ESZ;
}
template <int PREC, int EPI>
constexpr int kernel_lds_bytes() {
  return (EPI == EPI_QUAD && quad_lds_bytes<PREC>() > lds_bytes<PREC, EPI>()) ? quad_lds_bytes<PREC>()
                                                                              : lds_bytes<PREC, EPI>();
}

// s_waitcnt vmcnt(N) lgkmcnt(0): this wave's loads older than its last N
// have landed and its LDS reads are complete
template <int N>
__device__ inline void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt is six bits");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (0 << 8) | ((N >> 4) << 14));
}

// Workgroup barrier without the memory fence of __syncthreads, which would
// wait for every load in flight; the waits before it are explicit (wait_vm).
// The clobber keeps the compiler from moving memory accesses across it.
__device__ inline void chunk_barrier() { asm volatile("s_barrier" ::: "memory"); }

// 16-byte slot permutation of LDS row `row`.  A 16-byte-per-lane LDS read is
// served in groups of 8 lanes, 128 bytes per cycle: lanes 0-3 with 20-23,
// 4-7 with 16-19, 8-11 with 28-31, 12-15 with 24-27 (and the same 32 lanes
// higher).  With fragment lane l reading row l%16, slot (l/16) ^ swz(row),
// every group then hits eight distinct 16-byte bank quads; the permutation
// also keeps 8 or 16 consecutive lanes conflict-free.
__device__ inline int swz(int row) { return ((row >> 1) & 3) ^ ((row >> 3) & 1); }

template <typename T>
__device__ inline T neg8(T a) {  // sign flip of eight 16-bit floats (bf16 or fp16)
  v4u u = __builtin_bit_cast(v4u, a);
  u ^= 0x80008000u;
  return __builtin_bit_cast(T, u);
}

typedef const __attribute__((address_space(1))) void* gptr_t;
typedef __attribute__((address_space(3))) void* lptr_t;

// Issue the direct-to-LDS loads of one K chunk of one operand (all planes).
// Wave w, instruction i covers tile rows 16 (2 w + i) .. +15; lane l writes
// LDS bytes [16 l, 16 l + 16) of that 1 KB block = row 16 (2w+i) + l/4, slot
// l%4, which receives global segment (l%4) ^ swz(row).
template <int PREC>
__device__ inline void issue_chunk(const char* gbase, int64_t plane_bytes, int64_t ld_bytes,
                                   int64_t k0_bytes, char* lds_op, int wave, int lane) {
#pragma unroll
  for (int p = 0; p < PT<PREC>::PLANES; ++p)
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int blk = 2 * wave + i;
      const int row = 16 * blk + (lane >> 2);
      const int seg = (lane & 3) ^ swz(row);
      const char* src = gbase + p * plane_bytes + row * ld_bytes + k0_bytes + seg * 16;
      char* dst = lds_op + p * PLANE_TILE + blk * 1024;
      __builtin_amdgcn_global_load_lds((gptr_t)src, (lptr_t)dst, 16, 0, 0);
    }
}

template <typename T>
__device__ inline T lds_frag(const char* lds_op, int plane, int row, int kg) {
  return *(const T*)(lds_op + plane * PLANE_TILE + row * 64 + ((kg ^ swz(row)) << 4));
}

struct Acc {
  v4f re[4][4], im[4][4];
  __device__ inline void zero() {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        re[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
        im[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
      }
  }
};

// Multiply one LDS-resident chunk into the accumulators.
template <int PREC, bool CONJA>
__device__ inline void mma_chunk(const char* sA, const char* sB, int wm, int wn, int lane, Acc& acc) {
  const int lr = lane & 15, kg = lane >> 4;
  // scheduling hint: interleave the fragment reads with the products of a
  // chunk as for a single wave per SIMD (3-5% on the Gram matrix and the
  // quadratic form, no change on the per-beam products)
  __builtin_amdgcn_iglp_opt(1);
  if constexpr (PREC == BIP_PREC_FP32) {
    float4 bR[4], bI[4];
#pragma unroll
    for (int bn = 0; bn < 4; ++bn) {
      const int row = wn * 64 + bn * 16 + lr;
      bR[bn] = lds_frag<float4>(sB, 0, row, kg);
      bI[bn] = lds_frag<float4>(sB, 1, row, kg);
    }
#pragma unroll
    for (int bm = 0; bm < 4; ++bm) {
      const int row = wm * 64 + bm * 16 + lr;
      const float4 aR = lds_frag<float4>(sA, 0, row, kg);
      const float4 aI = lds_frag<float4>(sA, 1, row, kg);
      const float ar[4] = {aR.x, aR.y, aR.z, aR.w};
      const float ai[4] = {aI.x, aI.y, aI.z, aI.w};
#pragma unroll
      for (int bn = 0; bn < 4; ++bn) {
        const float br[4] = {bR[bn].x, bR[bn].y, bR[bn].z, bR[bn].w};
        const float bi[4] = {bI[bn].x, bI[bn].y, bI[bn].z, bI[bn].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          // (ar + i s ai)(br + i bi), s = -1 for conj(A)
          const float ain = CONJA ? ai[q] : -ai[q];
          const float aip = CONJA ? -ai[q] : ai[q];
          acc.re[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[q], br[q], acc.re[bm][bn], 0, 0, 0);
          acc.re[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x4f32(ain, bi[q], acc.re[bm][bn], 0, 0, 0);
          acc.im[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[q], bi[q], acc.im[bm][bn], 0, 0, 0);
          acc.im[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x4f32(aip, br[q], acc.im[bm][bn], 0, 0, 0);
        }
      }
    }
  } else if constexpr (PREC == BIP_PREC_SPLIT_BF16) {
    v8bf bRh[4], bRl[4], bIh[4], bIl[4];
#pragma unroll
    for (int bn = 0; bn < 4; ++bn) {
      const int row = wn * 64 + bn * 16 + lr;
      bRh[bn] = lds_frag<v8bf>(sB, 0, row, kg);
      bRl[bn] = lds_frag<v8bf>(sB, 1, row, kg);
      bIh[bn] = lds_frag<v8bf>(sB, 2, row, kg);
      bIl[bn] = lds_frag<v8bf>(sB, 3, row, kg);
    }
#pragma unroll
    for (int bm = 0; bm < 4; ++bm) {
      const int row = wm * 64 + bm * 16 + lr;
      const v8bf aRh = lds_frag<v8bf>(sA, 0, row, kg);
      const v8bf aRl = lds_frag<v8bf>(sA, 1, row, kg);
      const v8bf aIh = lds_frag<v8bf>(sA, 2, row, kg);
      const v8bf aIl = lds_frag<v8bf>(sA, 3, row, kg);
      const v8bf nIh = neg8(aIh), nIl = neg8(aIl);
      // the re accumulation takes -aI (+aI for conj(A)); the im one +aI (-aI)
      const v8bf rIh = CONJA ? aIh : nIh, rIl = CONJA ? aIl : nIl;
      const v8bf iIh = CONJA ? nIh : aIh, iIl = CONJA ? nIl : aIl;
#pragma unroll
      for (int bn = 0; bn < 4; ++bn) {
        v4f r = acc.re[bm][bn], m = acc.im[bm][bn];
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aRl, bRh[bn], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aRh, bRl[bn], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(rIl, bIh[bn], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(rIh, bIl[bn], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aRh, bRh[bn], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(rIh, bIh[bn], r, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aRl, bIh[bn], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aRh, bIl[bn], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(iIl, bRh[bn], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(iIh, bRl[bn], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aRh, bIh[bn], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(iIh, bRh[bn], m, 0, 0, 0);
        acc.re[bm][bn] = r;
        acc.im[bm][bn] = m;
      }
    }
  } else if constexpr (PREC == BIP_PREC_FP16) {
    v8h bR[4], bI[4];
#pragma unroll
    for (int bn = 0; bn < 4; ++bn) {
      const int row = wn * 64 + bn * 16 + lr;
      bR[bn] = lds_frag<v8h>(sB, 0, row, kg);
      bI[bn] = lds_frag<v8h>(sB, 1, row, kg);
    }
#pragma unroll
    for (int bm = 0; bm < 4; ++bm) {
      const int row = wm * 64 + bm * 16 + lr;
      const v8h aR = lds_frag<v8h>(sA, 0, row, kg);
      const v8h aI = lds_frag<v8h>(sA, 1, row, kg);
      const v8h nI = neg8(aI);
      const v8h rI = CONJA ? aI : nI, iI = CONJA ? nI : aI;
#pragma unroll
      for (int bn = 0; bn < 4; ++bn) {
        acc.re[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_f16(aR, bR[bn], acc.re[bm][bn], 0, 0, 0);
        acc.re[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_f16(rI, bI[bn], acc.re[bm][bn], 0, 0, 0);
        acc.im[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_f16(aR, bI[bn], acc.im[bm][bn], 0, 0, 0);
        acc.im[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_f16(iI, bR[bn], acc.im[bm][bn], 0, 0, 0);
      }
    }
  } else {
    v8bf bR[4], bI[4];
#pragma unroll
    for (int bn = 0; bn < 4; ++bn) {
      const int row = wn * 64 + bn * 16 + lr;
      bR[bn] = lds_frag<v8bf>(sB, 0, row, kg);
      bI[bn] = lds_frag<v8bf>(sB, 1, row, kg);
    }
#pragma unroll
    for (int bm = 0; bm < 4; ++bm) {
      const int row = wm * 64 + bm * 16 + lr;
      const v8bf aR = lds_frag<v8bf>(sA, 0, row, kg);
      const v8bf aI = lds_frag<v8bf>(sA, 1, row, kg);
      const v8bf nI = neg8(aI);
      const v8bf rI = CONJA ? aI : nI, iI = CONJA ? nI : aI;
#pragma unroll
      for (int bn = 0; bn < 4; ++bn) {
        acc.re[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aR, bR[bn], acc.re[bm][bn], 0, 0, 0);
        acc.re[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(rI, bI[bn], acc.re[bm][bn], 0, 0, 0);
        acc.im[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aR, bI[bn], acc.im[bm][bn], 0, 0, 0);
        acc.im[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(iI, bR[bn], acc.im[bm][bn], 0, 0, 0);
      }
    }
  }
}

// acc = sum over K of A[m0 + .][k] B[n0 + .][k] (A and B point at the tile origins).
// Chunk kc lives in LDS buffer kc mod NS; the loads of chunks kc+1 .. kc+NS-2
// may still be in flight while chunk kc is multiplied.
template <int PREC, bool CONJA, int NS>
__device__ inline void tile_product(const char* A, int64_t a_plane_b, int64_t lda_b, const char* B,
                                    int64_t b_plane_b, int64_t ldb_b, int K, int64_t CH, char* lds,
                                    int wave, int lane, int wm, int wn, Acc& acc) {
  // CH: bytes between consecutive K chunks of a row (64 when K is contiguous)
  constexpr int SB = stage_bytes<PREC>();
  constexpr int OPB = PT<PREC>::PLANES * PLANE_TILE;
  constexpr int LPC = 4 * PT<PREC>::PLANES;  // global_load_lds per wave per chunk
  const int nk = K / PT<PREC>::BK;
  auto issue = [&](int kc) {
    char* buf = lds + (kc % NS) * SB;
    issue_chunk<PREC>(A, a_plane_b, lda_b, kc * CH, buf, wave, lane);
    issue_chunk<PREC>(B, b_plane_b, ldb_b, kc * CH, buf + OPB, wave, lane);
  };
  for (int kc = 0; kc < NS - 1 && kc < nk; ++kc) issue(kc);
  for (int kc = 0; kc < nk; ++kc) {
    // chunk kc has landed for every wave (the later chunks issued so far may
    // still be in flight), and every wave is done with chunk kc - 1
    const int later = min(NS - 2, nk - 1 - kc);
    if constexpr (NS == 4) {
      if (later >= 2) wait_vm<2 * LPC>();
      else if (later == 1) wait_vm<LPC>();
      else wait_vm<0>();
    } else {
      wait_vm<0>();
    }
    chunk_barrier();
    if (kc + NS - 1 < nk) issue(kc + NS - 1);  // into the buffer of chunk kc - 1
    const char* cur = lds + (kc % NS) * SB;
    mma_chunk<PREC, CONJA>(cur, cur + OPB, wm, wn, lane, acc);
  }
  // all reads of the last buffer finish before the caller reuses LDS
  __syncthreads();
}

// ------------------------------------------------------------- the kernel
// Crop mask of a job (PRISM interpolation factor > 1): scan rho = u S_x + v
// is kept when (u - cu0) mod S_y < cnu and (v - cv0) mod S_x < cnv.
__device__ inline bool crop_in(const GemmJob& j, int rho, int Sy, int Sx) {
  const int u = rho / Sx, v = rho - u * Sx;
  return (u - j.cu0 + Sy) % Sy < j.cnu && (v - j.cv0 + Sx) % Sx < j.cnv;
}
// Whether any raster row of the scans rho0 .. rho1 is inside the job's crop
// rows (uniform per workgroup: a tile with none skips the job).
__device__ inline bool crop_rows_any(const GemmJob& j, int rho0, int rho1, int Sy, int Sx) {
  if (j.cnu <= 0 || j.cnv <= 0) return false;
  for (int u = rho0 / Sx; u <= rho1 / Sx && u < Sy; ++u)
    if ((u - j.cu0 + Sy) % Sy < j.cnu) return true;
  return false;
}

// Upper-triangle tile e of an nt x nt tile grid in blocked order: super-blocks
// of GS x GS tiles, row-major over the super-blocks with I <= J, row-major
// inside each (the diagonal ones triangular).  A run of consecutive e then
// touches few distinct row blocks of the operand.
constexpr int GS = 8;
__host__ __device__ inline void blocked_tile(int e, int nt, int& ti, int& tj) {
  const int ns = (nt + GS - 1) / GS;
  for (int I = 0; I < ns; ++I) {
    const int ri = GS < nt - I * GS ? GS : nt - I * GS;
    for (int J = I; J < ns; ++J) {
      const int cj = GS < nt - J * GS ? GS : nt - J * GS;
      const int sz = I == J ? ri * (ri + 1) / 2 : ri * cj;
      if (e >= sz) {
        e -= sz;
        continue;
      }
      int i = 0, j;
      if (I == J) {
        while (e >= ri - i) {
          e -= ri - i;
          ++i;
        }
        j = i + e;
      } else {
        i = e / cj;
        j = e - i * cj;
      }
      ti = I * GS + i;
      tj = J * GS + j;
      return;
    }
  }
  ti = tj = nt;  // not reached for e < nt (nt + 1) / 2
}

template <int PREC, int EPI, bool CONJA, int OPREC = PREC>
__global__ __launch_bounds__(NTHREADS, (occupancy<PREC, EPI>())) void k_zgemm(const GemmArgs g) {
  extern __shared__ char smem[];
  constexpr int ESZ = PT<PREC>::ESZ;
  constexpr bool ACCUM = (EPI == EPI_ABS2_MAP || EPI == EPI_ABS2_BEAMS || EPI == EPI_QUAD);
  // wave index in a scalar register: the LDS destinations of the direct loads
  // and the wave's tile offsets are then scalar values
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, kg = lane >> 4;
  int m0, n0, jb0, jb1;
  if constexpr (EPI == EPI_GRAMQ) {
    // 1-D grid.  Workgroup i runs on XCD i mod 8.  When every job of the
    // launch has fewer than 64 tiles, all the upper-triangle tiles of a job
    // go to one XCD, so the job's operand rows are shared through its L2.
    // Otherwise each job's own tiles (ceil(W^2 / 128) per side) are cut into
    // eight equal contiguous runs of the blocked order, one per XCD: the
    // tiles an XCD runs at once then share a few operand row blocks in its
    // L2, and every XCD holds an equal share of every job, whatever the
    // window sizes mixed in the launch.  A job's runs occupy slot rows
    // s0 .. s0 + ceil(T_j / 8) - 1 (eight workgroups a row), so a launch of
    // mixed window sizes has no empty workgroups beyond each job's last row.
    const int nt = g.tiles, T = nt * (nt + 1) / 2;
    int ti, tj;
    if (T < 64) {
      const int slot = (int)(blockIdx.x >> 3);
      jb0 = (slot / T) * 8 + (int)(blockIdx.x & 7);
      if (jb0 >= g.njobs) return;  // uniform per workgroup
      int tl = slot % T;
      ti = 0;
      while (tl >= nt - ti) {
        tl -= nt - ti;
        ++ti;
      }
      tj = ti + tl;
    } else {
      const int row = (int)(blockIdx.x >> 3);
      int lo = 0, hi = g.njobs - 1;  // the job: the last with s0 <= row
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g.jobs[mid].s0 <= row) lo = mid;
        else hi = mid - 1;
      }
      jb0 = lo;
      const int ntj = (g.jobs[jb0].n_lim + BN - 1) / BN, Tj = ntj * (ntj + 1) / 2;
      const int perj = (Tj + 7) / 8;
      const int lr = row - g.jobs[jb0].s0;
      const int e = (int)(blockIdx.x & 7) * perj + lr;
      if (lr >= perj || e >= Tj) return;  // uniform per workgroup
      blocked_tile(e, ntj, ti, tj);
    }
    jb1 = jb0 + 1;
    m0 = ti * BM;
    n0 = tj * BN;
  } else if constexpr (EPI == EPI_ABS2_MAP || EPI == EPI_ABS2_BEAMS) {
    // 1-D grid of 16 x 16-tile super-blocks, 256 workgroups each; workgroup i
    // runs on XCD i mod 8, and each XCD takes a 4 x 8 block of the super-block,
    // so the tiles an XCD runs together share 4 row blocks of A and 8 of B
    // in its L2 (consecutive super-blocks run down M)
    const int b = (int)blockIdx.x, sblk = b >> 8, l = b & 255, x = l & 7, i = l >> 3;
    const int SM = (g.mtiles + 15) >> 4;
    const int mt = (sblk % SM) * 16 + (x >> 1) * 4 + (i >> 3);
    const int nt = (sblk / SM) * 16 + (x & 1) * 8 + (i & 7);
    if (mt >= g.mtiles || nt >= g.ntiles) return;  // uniform per workgroup
    m0 = mt * BM;
    n0 = nt * BN;
    jb0 = 0;
    jb1 = g.njobs;
  } else {
    // consecutive workgroups take consecutive M tiles of one N tile
    m0 = blockIdx.x * BM;
    n0 = blockIdx.y * BN;
    if constexpr (EPI == EPI_QUAD) {  // job group z of g.zsplit
      jb0 = (int)((int64_t)g.njobs * blockIdx.z / g.zsplit);
      jb1 = (int)((int64_t)g.njobs * (blockIdx.z + 1) / g.zsplit);
    } else if constexpr (EPI == EPI_STORE) {  // one job per grid z
      jb0 = (int)blockIdx.z;
      jb1 = jb0 + 1;
    } else {
      jb0 = 0;
      jb1 = g.njobs;
    }
  }
  v4f sq[4][4];
  if constexpr (ACCUM) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) sq[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  }
  for (int jb = jb0; jb < jb1; ++jb) {
    const GemmJob job = g.jobs[jb];
    if (n0 >= job.n_lim || m0 >= job.m_lim) continue;  // uniform per workgroup
    if constexpr (EPI == EPI_QUAD || EPI == EPI_ABS2_MAP || EPI == EPI_ABS2_BEAMS) {
      // scans along M (quadratic form) or N (detector products); a tile
      // holding no row of the job's crop mask skips the job
      const int s0 = EPI == EPI_QUAD ? m0 : n0;
      if (g.crop && !crop_rows_any(job, s0, min(s0 + 127, g.P - 1), g.Sy, g.Sx)) continue;
    }
    // the block-triangular quadratic form runs K over r' >= the tile's first r
    const int k0 = (EPI == EPI_QUAD && g.qtri) ? n0 : 0;
    const char* Ap = (const char*)g.A + (job.a_off + (int64_t)m0 * job.lda + k0) * ESZ;
    const char* Bp = (const char*)g.B + (job.b_off + (int64_t)n0 * job.ldb + k0) * ESZ;
    Acc acc;
    acc.zero();
    const int64_t ch = (job.kstride ? (int64_t)job.kstride : (int64_t)PT<PREC>::BK) * ESZ;
    if constexpr (k_segmented<PREC, EPI>()) {
      Acc seg;
      for (int ks = 0; ks < job.K - k0; ks += KSEG) {
        seg.zero();
        const int64_t koff = (int64_t)(ks / PT<PREC>::BK) * ch;  // K chunks of the segment's start
        tile_product<PREC, CONJA, nstage<PREC, EPI>()>(Ap + koff, g.a_plane * ESZ, (int64_t)job.lda * ESZ,
                                                       Bp + koff, g.b_plane * ESZ, (int64_t)job.ldb * ESZ,
                                                       min(KSEG, job.K - k0 - ks), ch, smem, wave, lane, wm,
                                                       wn, seg);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            acc.re[i][j] += seg.re[i][j];
            acc.im[i][j] += seg.im[i][j];
          }
      }
    } else {
      tile_product<PREC, CONJA, nstage<PREC, EPI>()>(Ap, g.a_plane * ESZ, (int64_t)job.lda * ESZ, Bp,
                                                     g.b_plane * ESZ, (int64_t)job.ldb * ESZ, job.K - k0, ch,
                                                     smem, wave, lane, wm, wn, acc);
    }
    if constexpr (EPI == EPI_ABS2_MAP || EPI == EPI_ABS2_BEAMS) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        // column n = scan rho of this lane's block j
        const bool keep = !g.crop || crop_in(job, n0 + wn * 64 + j * 16 + lr, g.Sy, g.Sx);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (keep) sq[i][j] += acc.re[i][j] * acc.re[i][j] + acc.im[i][j] * acc.im[i][j];
      }
    } else if constexpr (EPI == EPI_QUAD) {
      // Re conj(psi^T[rho][r]) (Q psi)^T[rho][r]; psi is read back from the A
      // operand: the tile's rows m0.. and columns n0.. (columns below the
      // row length lda, which K-chunks never straddle) go to LDS in 16-byte
      // coalesced pieces, then every lane reads its elements from there
      constexpr int QR = quad_row<PREC>(), QPL = BM * QR, CH = 16 / ESZ;
      constexpr int NCH = BN / CH;  // 16-byte pieces per row
      constexpr int NPC = PT<PREC>::PLANES * BM * NCH;  // pieces of the tile
      constexpr int QB = 16;  // loads in flight per thread before their LDS stores
      static_assert(NPC % (NTHREADS * QB) == 0, "whole rounds of pieces");
      for (int i0 = tid; i0 < NPC; i0 += NTHREADS * QB) {
        uint4 val[QB];
#pragma unroll
        for (int u = 0; u < QB; ++u) {
          const int i = i0 + u * NTHREADS;
          const int pl = i / (BM * NCH), rem = i - pl * (BM * NCH);
          const int row = rem / NCH, ch = rem - row * NCH;
          const int r = n0 + ch * CH;
          val[u] = make_uint4(0u, 0u, 0u, 0u);
          if (r < job.lda)
            val[u] = *(const uint4*)((const char*)g.A +
                                     (job.a_off + (int64_t)(m0 + row) * job.lda + r + pl * g.a_plane) * ESZ);
        }
#pragma unroll
        for (int u = 0; u < QB; ++u) {
          const int i = i0 + u * NTHREADS;
          const int pl = i / (BM * NCH), rem = i - pl * (BM * NCH);
          const int row = rem / NCH, ch = rem - row * NCH;
          *(uint4*)(smem + ((int64_t)pl * QPL + row * QR + ch * CH) * ESZ) = val[u];
        }
      }
      __syncthreads();
#pragma unroll
      for (int bn = 0; bn < 4; ++bn) {
        const int rl = wn * 64 + bn * 16 + lr;  // r - n0
        if (n0 + rl >= job.W2) continue;
#pragma unroll
        for (int bm = 0; bm < 4; ++bm)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int rhol = wm * 64 + bm * 16 + kg * 4 + v;  // rho - m0
            if (g.crop && !crop_in(job, m0 + rhol, g.Sy, g.Sx)) continue;
            const float2 ps = load_planes<PREC>(smem, (int64_t)rhol * QR + rl, QPL);
            sq[bm][bn][v] += ps.x * acc.re[bm][bn][v] + ps.y * acc.im[bm][bn][v];
          }
      }
      __syncthreads();  // the next job's K loop refills LDS
    } else if constexpr (EPI == EPI_STORE) {
      float2* o = (float2*)g.out;
#pragma unroll
      for (int bn = 0; bn < 4; ++bn) {
        const int n = n0 + wn * 64 + bn * 16 + lr;
        if (n >= job.ldo) continue;
#pragma unroll
        for (int bm = 0; bm < 4; ++bm)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int m = m0 + wm * 64 + bm * 16 + kg * 4 + v;
            if (m >= g.m_store) continue;
            const float s = g.rowscale ? g.rowscale[m] : 1.f;
            o[job.out_off + (int64_t)m * job.ldo + n] =
                make_float2(s * acc.re[bm][bn][v], s * acc.im[bm][bn][v]);
          }
      }
    } else {
      // EPI_GRAMQ: element (m, n) = (r, r') of Q = G * sum_c conj(H_c(r)) H_c(r')
      // H of the tile's 128 rows and 128 columns, every channel, staged in the
      // (now free) LDS when it fits, so that the per-element channel sums read
      // LDS instead of waiting on memory once per channel
      const bool hlds = g.n_ch * 2 * BM * (int)sizeof(float2) <= lds_bytes<PREC, EPI>();
      float2* sHm = (float2*)smem;
      float2* sHn = sHm + (hlds ? g.n_ch * BM : 0);
      if (hlds) {
        for (int i = tid; i < g.n_ch * BM; i += NTHREADS) {
          const int c = i / BM, j = i - c * BM;
          const int64_t hc = job.h_off + (int64_t)c * job.W2;
          sHm[i] = m0 + j < job.W2 ? g.H[hc + m0 + j] : make_float2(0.f, 0.f);
          sHn[i] = n0 + j < job.W2 ? g.H[hc + n0 + j] : make_float2(0.f, 0.f);
        }
        __syncthreads();
      }
#pragma unroll
      for (int bn = 0; bn < 4; ++bn) {
        const int n = n0 + wn * 64 + bn * 16 + lr;
        if (n >= job.ldo) continue;
#pragma unroll
        for (int bm = 0; bm < 4; ++bm)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int m = m0 + wm * 64 + bm * 16 + kg * 4 + v;
            const float cr = g.gscale * acc.re[bm][bn][v], ci = g.gscale * acc.im[bm][bn][v];
            float qr = 0.f, qi = 0.f;
            if (m < job.W2 && n < job.W2) {
              float hr = 0.f, hi = 0.f;
              if (hlds) {
                for (int c = 0; c < g.n_ch; ++c) {
                  const float2 a = sHm[c * BM + (m - m0)];
                  const float2 b = sHn[c * BM + (n - n0)];
                  hr += a.x * b.x + a.y * b.y;
                  hi += a.x * b.y - a.y * b.x;
                }
              } else {
                for (int c = 0; c < g.n_ch; ++c) {
                  const float2 a = g.H[job.h_off + (int64_t)c * job.W2 + m];
                  const float2 b = g.H[job.h_off + (int64_t)c * job.W2 + n];
                  hr += a.x * b.x + a.y * b.y;
                  hi += a.x * b.y - a.y * b.x;
                }
              }
              qr = cr * hr - ci * hi;
              qi = cr * hi + ci * hr;
            }
            if (g.qtri && m0 != n0) {
              // block-triangular Q for the quadratic form: psi^H Q psi sums each
              // block pair r < r' twice (Q Hermitian), so the tile above the
              // diagonal is stored doubled and the one below is never read
              store_planes<OPREC>(g.out, job.out_off + (int64_t)m * job.ldo + n, g.out_plane, 2.f * qr,
                                  2.f * qi);
            } else {
              store_planes<OPREC>(g.out, job.out_off + (int64_t)m * job.ldo + n, g.out_plane, qr, qi);
              // Q is Hermitian: the tile below the diagonal is the conjugate transpose
              if (m0 != n0 && m < job.ldo)
                store_planes<OPREC>(g.out, job.out_off + (int64_t)n * job.ldo + m, g.out_plane, qr,
                                    -qi);
            }
            if (g.out2) {  // G itself, for the gradient
              const bool in = m < job.W2 && n < job.W2;
              g.out2[job.out_off + (int64_t)m * job.ldo + n] = in ? make_float2(cr, ci) : make_float2(0.f, 0.f);
              if (m0 != n0 && m < job.ldo)
                g.out2[job.out_off + (int64_t)n * job.ldo + m] = in ? make_float2(cr, -ci) : make_float2(0.f, 0.f);
            }
          }
      }
    }
  }
  if constexpr (EPI == EPI_ABS2_MAP || EPI == EPI_QUAD) {
    // map partial sums over the tile's d (rows, ABS2) or r (columns, QUAD), fixed order
    __shared__ float red[2][128];
    if constexpr (EPI == EPI_ABS2_MAP) {
      float cs[4];
#pragma unroll
      for (int bn = 0; bn < 4; ++bn) {
        float s = 0.f;
#pragma unroll
        for (int bm = 0; bm < 4; ++bm)
          s += (sq[bm][bn][0] + sq[bm][bn][1]) + (sq[bm][bn][2] + sq[bm][bn][3]);
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        cs[bn] = s;
      }
      if (kg == 0) {
#pragma unroll
        for (int bn = 0; bn < 4; ++bn) red[wm][wn * 64 + bn * 16 + lr] = cs[bn];
      }
      __syncthreads();
      if (tid < BN) g.partial[(int64_t)(m0 / BM) * g.Npad + n0 + tid] = g.oscale * (red[0][tid] + red[1][tid]);
    } else {
      // rows rho = m0 + 64 wm + 16 bm + 4 kg + v; sum over r (lanes lr, blocks bn, waves wn)
#pragma unroll
      for (int bm = 0; bm < 4; ++bm)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float s = (sq[bm][0][v] + sq[bm][1][v]) + (sq[bm][2][v] + sq[bm][3][v]);
          s += __shfl_xor(s, 1);
          s += __shfl_xor(s, 2);
          s += __shfl_xor(s, 4);
          s += __shfl_xor(s, 8);
          if (lr == 0) red[wn][wm * 64 + bm * 16 + kg * 4 + v] = s;
        }
      __syncthreads();
      if (tid < BM)
        g.partial[((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * g.Mpad + m0 + tid] =
            red[0][tid] + red[1][tid];
    }
  } else if constexpr (EPI == EPI_ABS2_BEAMS) {
#pragma unroll
    for (int bn = 0; bn < 4; ++bn) {
      const int rho = n0 + wn * 64 + bn * 16 + lr;
      if (rho >= g.P) continue;
#pragma unroll
      for (int bm = 0; bm < 4; ++bm)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int d = m0 + wm * 64 + bm * 16 + kg * 4 + v;
          if (d < g.ndet) g.out_beams[(int64_t)rho * g.ndet + d] += g.oscale * sq[bm][bn][v];
        }
    }
  }
}

// -------------------------------------------------------------- helpers
__global__ void k_reduce_map(const float* __restrict__ partial, int ntiles, int Ppad, int P,
                             float* out, int accumulate) {
  const int rho = blockIdx.x * blockDim.x + threadIdx.x;
  if (rho >= P) return;
  float s = 0.f;
  for (int t = 0; t < ntiles; ++t) s += partial[(int64_t)t * Ppad + rho];
  out[rho] = accumulate ? out[rho] + s : s;
}

// qEELS: sum the per-beam intensities over h_y at fixed h_x, in detector order
__global__ void k_qeels(const float* __restrict__ beams_out, const int32_t* __restrict__ bin_start,
                        const int32_t* __restrict__ bin_list, int ndet, int P, int nq,
                        float* out, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)P * nq) return;
  const int rho = (int)(i / nq);
  const int q = (int)(i - (int64_t)rho * nq);
  float s = 0.f;
  for (int k = bin_start[q]; k < bin_start[q + 1]; ++k)
    s += beams_out[(int64_t)rho * ndet + bin_list[k]];
  out[i] = accumulate ? out[i] + s : s;
}

template <int PREC, int EPI, bool CONJA, int OPREC = PREC>
hipError_t zgemm_launch(const GemmArgs& g, dim3 grid, hipStream_t s) {
  const void* f = (const void*)k_zgemm<PREC, EPI, CONJA, OPREC>;
  constexpr int lds = kernel_lds_bytes<PREC, EPI>();
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_zgemm<PREC, EPI, CONJA, OPREC>), grid, dim3(NTHREADS), lds, s, g);
  return hipGetLastError();
}

template <int PREC>
hipError_t zgemm_prec(int epi, const GemmArgs& g, dim3 grid, hipStream_t s) {
  switch (epi) {
    case EPI_ABS2_MAP: return zgemm_launch<PREC, EPI_ABS2_MAP, false>(g, grid, s);
    case EPI_ABS2_BEAMS: return zgemm_launch<PREC, EPI_ABS2_BEAMS, false>(g, grid, s);
    case EPI_QUAD: return zgemm_launch<PREC, EPI_QUAD, false>(g, grid, s);
    case EPI_STORE: return zgemm_launch<PREC, EPI_STORE, false>(g, grid, s);
    case EPI_STORE + EPI_CONJ_A: return zgemm_launch<PREC, EPI_STORE, true>(g, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_zgemm_gram(int in_prec, int out_prec, const GemmArgs& g, int gx, hipStream_t s) {
  if (gx <= 0 || g.njobs <= 0) return hipSuccess;
  if (g.tiles <= 0 || !(g.gscale > 0.f)) return hipErrorInvalidValue;
  const int64_t T = (int64_t)g.tiles * (g.tiles + 1) / 2;
  if (T < 64 && gx != 8 * (int64_t)((g.njobs + 7) / 8) * T) return hipErrorInvalidValue;
  const dim3 grid(gx, 1, 1);
  if (in_prec == BIP_PREC_FP16 && out_prec == BIP_PREC_SPLIT_BF16)
    return zgemm_launch<BIP_PREC_FP16, EPI_GRAMQ, true, BIP_PREC_SPLIT_BF16>(g, grid, s);
  if (in_prec != out_prec) return hipErrorInvalidValue;
  switch (in_prec) {
    case BIP_PREC_FP32: return zgemm_launch<BIP_PREC_FP32, EPI_GRAMQ, true>(g, grid, s);
    case BIP_PREC_SPLIT_BF16: return zgemm_launch<BIP_PREC_SPLIT_BF16, EPI_GRAMQ, true>(g, grid, s);
    case BIP_PREC_BF16: return zgemm_launch<BIP_PREC_BF16, EPI_GRAMQ, true>(g, grid, s);
    case BIP_PREC_FP16: return zgemm_launch<BIP_PREC_FP16, EPI_GRAMQ, true>(g, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_zgemm(int prec, int epi, const GemmArgs& g, int gx, int gy, int gz,
                        hipStream_t s) {
  if (gx <= 0 || gy <= 0 || gz <= 0 || g.njobs <= 0) return hipSuccess;
  if (epi == EPI_QUAD && (g.zsplit != gz || gz > g.njobs)) return hipErrorInvalidValue;
  if (epi == EPI_GRAMQ) return hipErrorInvalidValue;  // launch_zgemm_gram
  dim3 grid(gx, gy, gz);
  GemmArgs ga = g;
  if (epi == EPI_ABS2_MAP || epi == EPI_ABS2_BEAMS) {
    if (gz != 1) return hipErrorInvalidValue;
    ga.mtiles = gx;
    ga.ntiles = gy;
    const int64_t nsb = (int64_t)((gx + 15) / 16) * ((gy + 15) / 16);
    if (nsb * 256 > INT32_MAX) return hipErrorInvalidValue;
    grid = dim3((unsigned)(nsb * 256), 1, 1);
  }
  switch (prec) {
    case BIP_PREC_FP32: return zgemm_prec<BIP_PREC_FP32>(epi, ga, grid, s);
    case BIP_PREC_SPLIT_BF16: return zgemm_prec<BIP_PREC_SPLIT_BF16>(epi, ga, grid, s);
    case BIP_PREC_BF16: return zgemm_prec<BIP_PREC_BF16>(epi, ga, grid, s);
    case BIP_PREC_FP16: return zgemm_prec<BIP_PREC_FP16>(epi, ga, grid, s);
    default: return hipErrorInvalidValue;
  }
}

int64_t gemm_gram_plan(GemmJob* jobs, int njobs, int tiles) {
  const int64_t T = (int64_t)tiles * (tiles + 1) / 2;
  if (T < 64) return 8 * (int64_t)((njobs + 7) / 8) * T;
  int64_t rows = 0;
  for (int j = 0; j < njobs; ++j) {
    const int64_t ntj = (jobs[j].n_lim + BN - 1) / BN, Tj = ntj * (ntj + 1) / 2;
    jobs[j].s0 = (int32_t)rows;
    rows += (Tj + 7) / 8;
  }
  return 8 * rows;
}

int gemm_bk(int prec) { return prec == BIP_PREC_FP32 ? PT<BIP_PREC_FP32>::BK : 32; }

hipError_t launch_reduce_map(const float* partial, int ntiles, int Ppad, int P, float* out,
                             int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_map, dim3((P + 255) / 256), dim3(256), 0, s, partial, ntiles, Ppad,
                     P, out, accumulate);
  return hipGetLastError();
}

hipError_t launch_qeels_from_beams(const float* beams_out, const int32_t* bin_start,
                                   const int32_t* bin_list, int ndet, int P, int nq, float* out,
                                   int accumulate, hipStream_t s) {
  const int64_t n = (int64_t)P * nq;
  hipLaunchKernelGGL(k_qeels, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, beams_out,
                     bin_start, bin_list, ndet, P, nq, out, accumulate);
  return hipGetLastError();
}

}  // namespace bip
