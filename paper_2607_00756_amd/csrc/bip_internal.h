// Internal declarations of the BiP-PRISM HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bip.h"

namespace bip {

// ------------------------------------------------------------ complex helpers
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__host__ __device__ inline float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__host__ __device__ inline float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// ------------------------------------------------------------- plan layout
// One atom's window as seen by the sweep gathers, in plane order.
struct GatherRec {
  int32_t W, oy, ox, pad;
  int64_t off;  // element offset of the atom's [Bp][W][W] block in this side's window stack
};

struct GatherArgs {
  const GatherRec* rec;  // [n_atoms] records grouped by plane; plane j owns [begin_j, end_j)
  float2* win;           // window stack of this side
};

// One product of the complex contraction kernel (offsets in plane elements).
struct GemmJob {
  int64_t a_off, b_off;  // origins of the A and B operands
  int64_t out_off;       // origin of the output (store epilogues)
  int64_t h_off;         // first H element of the atom (complex elements)
  int32_t K;             // contraction length (multiple of the K chunk)
  int32_t lda, ldb;      // row pitches of A and B
  int32_t ldo;           // row pitch of the output; columns >= ldo are not written
  int32_t m_lim, n_lim;  // tiles starting at or beyond these skip the job
  int32_t W2;            // window pixels of the atom
  int32_t kstride;       // elements between consecutive 64-byte K chunks of a row of A and
                         // B (0: contiguous; K-blocked operands: row count x chunk width)
  int32_t cu0, cnu;      // crop mask of the atom (GemmArgs::crop): raster rows u with
  int32_t cv0, cnv;      // (u - cu0) mod S_y < cnu and columns v with (v - cv0) mod S_x < cnv
  int32_t s0;            // EPI_GRAMQ: first slot row of the job's tiles (set by gemm_gram_plan)
  int32_t pad;
};

// One atom of a batched K-blocked operand reconstruction.
struct ReconAtom {
  int64_t win_off;  // the atom's parent windows in the window stack (complex elements)
  int64_t out_off;  // the atom's operand block (plane elements)
  int32_t W, oy, ox;
  int32_t n_r;      // operand rows (window pixels rounded up to whole tiles)
};

enum Epilogue { EPI_ABS2_MAP = 0, EPI_ABS2_BEAMS, EPI_GRAMQ, EPI_QUAD, EPI_STORE };

struct GemmArgs {
  const void* A;
  const void* B;
  int64_t a_plane, b_plane;  // plane strides (elements)
  const GemmJob* jobs;
  int njobs;
  void* out;                 // store epilogues
  int64_t out_plane;
  const float2* H;           // transition potentials (EPI_GRAMQ)
  int n_ch;
  int Mpad, Npad;            // padded extents of the output (map partial pitches)
  float* partial;            // map partial sums
  float* out_beams;          // [P][ndet] (EPI_ABS2_BEAMS)
  int ndet, P;
  int tiles;                 // EPI_GRAMQ: 128-row tiles per side (upper triangle launched)
  int zsplit;                // EPI_QUAD: job groups along grid z, one partial row each
  float2* out2;              // EPI_GRAMQ: also store G itself (complex64 [r][r'], pitch ldo)
  const float* rowscale;     // EPI_STORE: optional real factor per output row
  int m_store;               // EPI_STORE: rows >= m_store are not written
  float gscale;              // EPI_GRAMQ: factor on G (undoes a scaling of the operand), > 0
  int qtri;                  // EPI_GRAMQ: Q block-triangular (upper tiles doubled, lower not
                             // stored); EPI_QUAD: K from the tile's first column (reads that form)
  int crop;                  // EPI_ABS2_*, EPI_QUAD: keep scan rho = u S_x + v only inside the
  int Sy, Sx;                // job's crop mask (PRISM interpolation factor > 1)
  float oscale;              // EPI_ABS2_*: factor on the intensities (f^2 of the detector sum)
  int mtiles, ntiles;        // EPI_ABS2_*: output tiles along M and N (set by launch_zgemm)
};
// One atom of the probe synthesis (offsets in elements of their buffers).
struct ProbeJob {
  int64_t win_off;   // the atom's S1 parent windows [Bp1][W*W] in the window stack
  int64_t fx_off;    // the atom's [S_y][S_x][ldf] block of the DFT workspace
  int64_t out_off;   // the atom's operand block (plane elements)
  int64_t h_off;     // first H element of the atom
  int32_t W, oy, ox; // window
  int32_t kd;        // row pitch of the operand (padded window pixels)
  int32_t ldf;       // row pitch of the DFT workspace
  int32_t t0;        // first 64-pixel tile of this job: prefix of ceil(W^2 / 64) over the jobs
};

struct ProbeArgs {
  const ProbeJob* jobs;
  const float2* win;        // S1 window stack
  int n_par;                // parents per atom block of the stack
  const int32_t* rowptr;    // CSR of w(1)
  const int32_t* col;
  const float* w;
  const int32_t* ellc;      // padded rows of w(1) [B][8]
  const float* ellw;
  const int2* beams;        // aperture beams [B]
  const int32_t* cell_start;  // [S_y S_x + 1] beams of residue cell (a, c)
  const int32_t* cell_beams;  // beam ids grouped by cell, ascending within a cell
  const float2* twx;        // [S_x] exp(-2 pi i k / S_x)
  const float2* twy;        // [S_y] exp(-2 pi i k / S_y)
  const float2* tw;         // [L] exp(-2 pi i m / L)
  int L, ny, nx, mode;
  int Sy, Sx, P, Ppad;
  float cb;                 // probe coefficient c_b
  int unit0, n_units;       // the launch's pixel tiles (job t0 numbering) and their count
  int n_jobs;               // jobs of the launch
  float2* fx;               // DFT workspace
  void* out;                // operand planes
  int64_t out_plane;
  const float2* H;          // U_n = H_n psi when the detector contraction follows
  int n_ch;
};

// Focal back-propagation of S1: one atom's enlarged window and its plane.
struct FocalAtom {
  int64_t win_off;  // the atom's S1 parent windows [Bp1][M][M] in the window stack
  int32_t M, W;     // enlarged window side (power of two) and the atom's window side
  int32_t oy, ox;   // enlarged window origin (pixels, mod N)
  int32_t plane, atom;
};

struct FocalProbeJob {
  int64_t psi_off;  // the atom's psi at the centroid [Ppad][kd_c] (FP32 planes)
  int64_t out_off;  // the atom's operand block (plane elements)
  int64_t h_off;    // first H element of the atom
  int32_t M, W, kd, kd_c, atom, pad;
};

struct FocalProbeArgs {
  const FocalProbeJob* jobs;
  const float* psi_c;
  int64_t psi_plane;
  void* out;
  int64_t out_plane;
  const float2* H;
  int n_ch, P, Ppad, L;
  const float2* tw;       // exp(-2 pi i m / L)
  double dy, dx, lambda;  // pixel sizes (A) and wavelength (A)
  const double* dist;     // back-step distance of each atom (A)
};

}  // namespace bip

struct bip_plan {
  bip_grid g;
  bip_optics o;
  double lambda = 0, sigma = 0;
  int L = 0;  // max(ny, nx): size of the twiddle table
  // geometry (host copies, sorted by (h_y, h_x))
  std::vector<int32_t> beams, det, par1, par2;  // pairs
  std::vector<int32_t> rp1, col1, rp2, col2;    // CSR of w(1), w(2)
  std::vector<double> w1, w2;
  int B = 0, ndet = 0, Bp1 = 0, Bp2 = 0, nq = 0, nq_half = 0;
  int f = 1;           // PRISM interpolation factor (beams kept at h = 0 mod f)
  int B_full = 0;      // aperture beams before the subsampling (probe normalization)
  std::vector<double> tau_y, tau_x;  // atom positions (pixels), for the crop mask
  // atoms
  int n_atoms = 0;
  std::vector<int32_t> W, oy, ox, plane;
  std::vector<int64_t> off1, off2;
  std::vector<int32_t> plane_start, plane_atoms;
  int i_min = 0, i_max = 0;
  bool built = false;
  // S2 streamed in plane segments (window stacks of all atoms above the budget):
  // segment k covers planes seg_hi[k] .. seg_lo[k] (descending); off2 of an atom is
  // relative to its segment's block, d_win2 holds one segment
  bool s2_stream = false;
  std::vector<int32_t> seg_hi, seg_lo, seg_of;
  int column_batch = 0;  // parent columns per sweep batch of the last build
  int n_cu = 256;        // compute units of the plan's device
  // device buffers
  float2* d_tw = nullptr;       // [L] exp(-2 pi i m / L)
  float2* d_prop = nullptr;     // [ny][nx] P(q) / G
  float2* d_T = nullptr;        // [nz][ny][nx]
  int2* d_beams = nullptr;      // [B]
  int2* d_det = nullptr;        // [ndet]
  int2* d_par1 = nullptr;       // [Bp1]
  int2* d_par2 = nullptr;       // [Bp2]
  int32_t *d_rp1 = nullptr, *d_col1 = nullptr, *d_rp2 = nullptr, *d_col2 = nullptr;
  float *d_w1 = nullptr, *d_w2 = nullptr;
  int32_t *d_ellc1 = nullptr, *d_ellc2 = nullptr;  // padded CSR rows
  float *d_ellw1 = nullptr, *d_ellw2 = nullptr;
  int32_t *d_tstart1 = nullptr, *d_tpar1 = nullptr, *d_eloc1 = nullptr;  // 64-beam tiles
  int32_t *d_tstart2 = nullptr, *d_tpar2 = nullptr, *d_eloc2 = nullptr;
  int tile_np1 = 0, tile_np2 = 0;  // most distinct parents of any 64-beam tile
  int32_t *d_W = nullptr, *d_oy = nullptr, *d_ox = nullptr;
  // S1 windows: the atom's own (W, oy, ox), or the enlarged focal ones
  bool focal = false;
  std::vector<int32_t> W1, oy1, ox1;
  int focal_max_m = 0;
  bip::FocalAtom* d_fatoms = nullptr;
  double* d_fdist = nullptr;       // back-step distance per atom (A), set by each build
  std::vector<bip::FocalProbeJob> h_fjobs;
  int64_t *d_off1 = nullptr, *d_off2 = nullptr;
  bip::GatherRec *d_grec1 = nullptr, *d_grec2 = nullptr;  // gather records in plane order
  float2* d_state1 = nullptr;   // [Bp1][G]
  float2* d_state2 = nullptr;   // [Bp2][G]
  float2* d_win1 = nullptr;     // window stacks
  float2* d_win2 = nullptr;
  // gradient state (ckpt_stride = 1)
  float2* d_prop_conj = nullptr;  // conj(P(q)) / G
  float2* d_ckpt1 = nullptr;      // [i_max][Bp1][G]: S1 after T_j, slices 0 .. i_max-1
  float2* d_ckpt2 = nullptr;      // [nz - i_min][Bp2][G]: S2 after T_j, slices i_min .. nz-1
  float2* d_gwin1 = nullptr;      // window cotangents, laid out like the window stacks
  float2* d_gwin2 = nullptr;
  int32_t *d_tp1_rp = nullptr, *d_tp1_b = nullptr, *d_tp2_rp = nullptr, *d_tp2_b = nullptr;
  float *d_tp1_w = nullptr, *d_tp2_w = nullptr;  // parent -> beam weights (backward)
  int64_t win1_elems = 0, win2_elems = 0;
  // signal workspace (grown on demand)
  void* d_work = nullptr;
  size_t work_bytes = 0;
  float* d_tmp = nullptr;  // output of weighted / accumulated signals before the sum
  size_t tmp_bytes = 0;
  // host tables read by asynchronous copies; kept alive until the next call
  std::vector<bip::GemmJob> h_jobs2, h_jobs3;
  std::vector<bip::ReconAtom> h_ratoms;
  std::vector<int32_t> h_qstart, h_qlist;
  std::vector<bip::ProbeJob> h_probe;
  std::vector<int32_t> h_cells;   // cell_start then cell_beams
  std::vector<float2> h_tws;      // twx then twy
  // device blocks of the plan, all from `alloc` (or hipMallocAsync when it is absent)
  struct Block { void* ptr; size_t bytes; };
  std::vector<Block> allocations;
  bip_alloc alloc{};
  bool has_alloc = false;
  hipStream_t stream = nullptr;  // stream of the latest call (destroy synchronizes it)
  int64_t bytes_now = 0, bytes_peak = 0;
  // opt-in stage timing with HIP events on the caller's stream
  bool profiling = false;
  struct Timed { int stage; hipEvent_t a, b; };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> event_pool;
  double stage_ms[16] = {0};
  int64_t stage_launches[16] = {0};
};

namespace bip {

enum Stage {
  ST_TRANSMIT = 0, ST_S1_ROW, ST_S1_COL, ST_S2_ROW, ST_S2_COL, ST_INIT, ST_RECON, ST_FOLD,
  ST_PROBE, ST_DET, ST_REDUCE, ST_GRAM, ST_COUNT
};

void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

// bip_eels_signal with an optional caller-given workspace (ext_work, ext_bytes):
// with one, nothing is allocated and requests that do not fit are refused.
int eels_signal_impl(bip_plan* p, int32_t n_ch, const float* H, const int64_t* H_off,
                     const int32_t* atom_subset, int32_t n_subset, int32_t scan_sy, int32_t scan_sx,
                     int32_t out_mode, int32_t precision, float* out, void* ext_work, size_t ext_bytes,
                     void* stream);
// Several edges (each its own H, channels, atoms and output) in one call;
// accumulate / weight: out += weight x signal (out = weight x signal when not
// accumulating).  With a caller-given workspace only weight 1 without
// accumulation is served.
int signal_edges_impl(bip_plan* p, int32_t n_edges, const bip_edge* edges, int32_t scan_sy,
                      int32_t scan_sx, int32_t out_mode, int32_t precision, int32_t accumulate,
                      float weight, void* ext_work, size_t ext_bytes, void* stream);
// The S2 transpose sweep over slices j_hi .. j_lo (descending) for every
// column batch, gathering the windows of the atoms at those planes.  With
// init, the parents start over from the exit.
int sweep_s2(bip_plan* p, int j_hi, int j_lo, bool init, hipStream_t st);

// ----------------------------------------------------------- launchers
// setup (k_setup.hip)
hipError_t launch_twiddles(float2* tw, int L, hipStream_t s);
// P(q)/G, or its conjugate (the inverse propagation of the adjoint sweeps)
hipError_t launch_prop_table(float2* prop, int ny, int nx, double ly, double lx, double lambda,
                             double dz, int conj, hipStream_t s);
hipError_t launch_transmit(float2* T, const float* V, int64_t n, float sigma, hipStream_t s);
hipError_t launch_init_planewaves(float2* state, const int2* h, int nb, int ny, int nx,
                                  const float2* tw, int L, int sign, float scale, hipStream_t s);
// sign -1 plane waves written row-transformed (the state between passes)
hipError_t launch_init_planewaves_rowft(float2* state, const int2* h, int nb, int ny, int nx,
                                        const float2* tw, int L, float scale, hipStream_t s);
hipError_t launch_sibson(const int2* query, int nq, int s_lattice, int2* slot_p, double* slot_w,
                         hipStream_t st);
// against a finite parent set with its convex hull (CCW); *overflow set when a
// query has more than 16 natural neighbours
hipError_t launch_sibson_general(const int2* query, int nq, const int2* parents, int np,
                                 const double2* hull, int nh, int2* slot_p, double* slot_w,
                                 int* overflow, hipStream_t st);

// multislice (k_multislice.hip)
enum RowFlags {
  ROW_INV = 1, ROW_T = 2, ROW_FWD = 4, ROW_GATHER_BEFORE_T = 8, ROW_GATHER_AFTER_T = 16,
  ROW_SAVE = 32  // write the state after T_j to `save` (slice checkpoint, [ncols][ny][nx])
};
// state (and save) point at the first column of the batch; col0 is that column's parent index
hipError_t launch_row_pass(int flags, float2* state, int ncols, int ny, int nx, const float2* T,
                           const float2* tw, int L, const int2* parents, int detilt_sign,
                           const GatherArgs& ga, int gather_begin, int gather_end, int col0,
                           float2* save, hipStream_t s);
// adjoint sweeps (the cotangent state replaces the forward state)
enum AdjFlags {
  ADJ_ZERO = 1, ADJ_INV = 2, ADJ_INJ_BEFORE = 4, ADJ_DV = 8, ADJ_CONJT = 16, ADJ_INJ_AFTER = 32,
  ADJ_FWD = 64
};
// grid: (ny / rows-per-block, groups); dv_partial [groups][ny][nx]; ckpt at the batch's first column
hipError_t launch_row_adjoint(int flags, float2* state, int ncols, int ny, int nx, const float2* T,
                              const float2* tw, int L, const GatherArgs& inj, int gb, int ge,
                              int col0, const float2* ckpt, float two_sigma, float* dv_partial,
                              int groups, hipStream_t s);
hipError_t launch_dv_reduce(const float* partial, int n_groups, int64_t n, float* dv, hipStream_t s);
hipError_t launch_col_pass(float2* state, int ncols, int ny, int nx, const float2* prop,
                           const float2* tw, int L, hipStream_t s);

// reconstruction (k_recon.hip)
struct ReconArgs {
  const float2* win;     // de-tilted parent windows of this atom [Bp][W*W]
  const int32_t* rowptr; // CSR of the weights
  const int32_t* col;
  const float* w;
  const int32_t* ellc;   // padded rows of the CSR [nb][8] (parents, length, start)
  const float* ellw;     // padded weights [nb][8]
  const int32_t* tstart; // [nb/64 + 1] parents of each 64-beam tile: tpar[tstart[t] ..)
  const int32_t* tpar;   // distinct parents of the tiles, ascending
  const int32_t* ell_loc;// [nb][8] slots 0..5 as indices into the tile's parent list
  int tile_np;           // most distinct parents of any 64-beam tile
  float scale;           // factor on the stored operand (exact power of two)
  const int2* beams;     // target beams [nb]
  int nb;                // number of target beams
  int W, oy, ox;         // window
  int ny, nx;
  const float2* tw;
  int L;
  int retilt_sign;       // +1: exp(+2 pi i h.r/N) (S1), -1 (S2)
  int mode;              // BIP_RECON_*
};
// plain complex64 output [nb][W*W]
hipError_t launch_recon_plain(const ReconArgs& a, float2* out, hipStream_t s);
// K-blocked operands (kind 0) of n_atoms atoms in one launch; a.win is the
// window stack, the per-atom fields of a are taken from atoms (device).
// Needs a.tile_np <= 64 (square-lattice parents).
hipError_t launch_recon_kblk_atoms(const ReconArgs& a, const ReconAtom* atoms, int n_atoms, void* out,
                                   int prec, int64_t ncols_pad, int64_t plane_stride, hipStream_t s);
// GEMM operand outputs; layout kind 0: [r][b] (b fastest, ld = ldk, rows up to nrows)
// kind 1: [b][r] (r fastest).  prec: BIP_PREC_*; planes at stride plane_stride elements.
hipError_t launch_recon_operand(const ReconArgs& a, void* out, int kind, int prec, int64_t ld,
                                int64_t nrows_pad, int64_t ncols_pad, int64_t plane_stride,
                                hipStream_t s);

// probe synthesis (k_probe.hip); scan dimensions up to BIP_MAX_SCAN
constexpr int BIP_MAX_SCAN = 256;
size_t probe_lds_bytes(int S);
hipError_t launch_probe_fold_x(const ProbeArgs& pa, int unit0, int n_units, int n_jobs, hipStream_t s);
hipError_t launch_probe_y(const ProbeArgs& pa, int prec, bool u, int max_kd, int n_jobs,
                          hipStream_t s);

// strided DFT pass of the probe-sum adjoint (k_probe.hip)
hipError_t launch_dft_pass(const float2* in, float2* out, int S, int64_t js, int64_t os, int64_t ks,
                           int64_t os2, int n_outer, int W2, const float2* tws, hipStream_t s);

// gradient kernels (k_backward.hip)
// prec: BIP_PREC_FP32 or BIP_PREC_SPLIT_BF16 (operand planes)
hipError_t launch_psi_transpose(int prec, const void* psiT, int64_t psp, int kd, int W2, int P,
                                int Ppad, int n1, const float* ibar, void* A1, void* B1, int64_t apl,
                                hipStream_t s);
hipError_t launch_kmat(int prec, const float2* R, const float2* H, int n_ch, int W2, int kd, int n1,
                       void* Kp, int64_t kpl, hipStream_t s);
hipError_t launch_grad_h(const float2* G, const float2* R, const float2* H, int n_ch, int W2, int kd,
                         float2* gH, hipStream_t s);
hipError_t launch_grad_tau(const float2* gH, const float2* dHx, const float2* dHy, int n,
                           double* out, hipStream_t s);
hipError_t launch_recon_adjoint(const ReconArgs& a, int side, const float2* gsrc, int64_t ld_src,
                                int Sy, int Sx, float cb, float2* gz, float* gam,
                                const int2* parents, int Bp, const int32_t* tp_rp,
                                const int32_t* tp_b, const float* tp_w, float2* gwin,
                                hipStream_t s);

// focal back-propagation (k_focal.hip)
hipError_t launch_focal_dist(const float* V, const FocalAtom* atoms, int n_atoms, int ny, int nx,
                             double dz, double* dist, hipStream_t s);
hipError_t launch_focal_parents(float2* win, const FocalAtom* atoms, int n_atoms, const double* dist,
                                const int2* parents, int n_par, int max_m, int ny, int nx, double dy,
                                double dx, double lambda, const float2* tw, int L, hipStream_t s);
hipError_t launch_focal_probe(const FocalProbeArgs& fp, int prec, bool u, int n_jobs, int max_m,
                              hipStream_t s);

// slice potentials (k_potential.hip).  Terms are (x, y, A, w) quadruples
// grouped by slice: slice z holds terms start[z] .. start[z + 1] (device i64).
hipError_t launch_profiles(const double* terms, int64_t n_terms, int ny, int nx, double ly,
                           double lx, int deriv, double* prof, double* dprof, hipStream_t s);
hipError_t launch_build_slices(const double* terms, const double* prof, const int64_t* start, int nz,
                               int ny, int nx, float* V, hipStream_t s);
// partials of launch_grad_terms: grad_part_doubles(nt_all, ny) doubles
int64_t grad_part_doubles(int64_t n_terms, int ny);
// most: the largest term count of a slice
hipError_t launch_grad_terms(const double* terms, const double* prof, const double* dprof,
                             const int64_t* start, int64_t nt_all, int most, int nz, int ny, int nx,
                             const float* dV, double* part, double* out, hipStream_t s);
// dxyz [n_atoms][3] from the per-term outputs; atom a owns terms first[a] .. + n_terms
hipError_t launch_atom_grad_sum(const double* out, const int64_t* first, int n_atoms, int n_terms,
                                double* dxyz, hipStream_t s);

// contraction (k_gemm.hip)
// grid: (m_tiles, n_tiles, z) for EPI_ABS2_* and EPI_QUAD (z = g.zsplit), (m_tiles,
// n_tiles, njobs) for EPI_STORE; for EPI_GRAMQ a 1-D grid of the gemm_gram_plan count
// for the launch's jobs.  epi EPI_STORE + EPI_CONJ_A conjugates the A operand.
constexpr int EPI_CONJ_A = 16;
// EPI_GRAMQ: operands in in_prec, Q stored in out_prec (equal, or FP16 -> SPLIT_BF16)
hipError_t launch_zgemm_gram(int in_prec, int out_prec, const GemmArgs& g, int gx, hipStream_t s);
hipError_t launch_zgemm(int prec, int epi, const GemmArgs& g, int gx, int gy, int gz,
                        hipStream_t s);
// Workgroups of an EPI_GRAMQ launch over the host copies jobs[0 .. njobs) (tiles:
// the largest job's tiles per side, g.tiles); sets each job's s0.  Call before the
// jobs are uploaded.
int64_t gemm_gram_plan(GemmJob* jobs, int njobs, int tiles);
constexpr int GEMM_MAX_ZSPLIT = 16;
int gemm_bk(int prec);
hipError_t launch_reduce_map(const float* partial, int ntiles, int Ppad, int P, float* out,
                             int accumulate, hipStream_t s);
hipError_t launch_qeels_from_beams(const float* beams_out, const int32_t* bin_start,
                                   const int32_t* bin_list, int ndet, int P, int nq, float* out,
                                   int accumulate, hipStream_t s);
hipError_t launch_zero(float* p, int64_t n, hipStream_t s);
// out = (accumulate ? out : 0) + w x src
hipError_t launch_axpy(float* out, const float* src, int64_t n, float w, int accumulate, hipStream_t s);

}  // namespace bip
