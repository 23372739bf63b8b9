/*
 * bip.h -- C ABI of the BiP-PRISM core-loss STEM-EELS hot path on MI355X.
 *
 * The library computes the bi-partitioned PRISM-EELS map of Pelz,
 * "The BiP-PRISM algorithm for fast and scalable core-loss STEM-EELS
 * simulations" (Alg. 5, section "Bi-partitioned PRISM-EELS"):
 *   (a) multislice of the parent beams of the probe-forming matrix S1
 *       (eq. smatrix-advance) and of the detector matrix S2 by transpose
 *       multislice (eq. s2), with the parent columns cropped to each ionized
 *       atom's window as the sweep passes its plane;
 *   (b) Sibson natural-neighbour reconstruction of S1 and S2 on the window
 *       (eq. nnw, eq. window-recon, magnitude preserving eq. magpreserve);
 *   (c) the contraction of illumination coefficients x S1 x H_n x S2 into
 *       intensities (eq. coupling, eq. map-sum, section "Output modes").
 *
 * Conventions shared by every entry point
 *   - Units: Angstrom, eV, rad.  V is the projected potential in V*A.
 *   - Grid: corner-origin DFT grid, pixel (y, x), x fastest; beam index
 *     h = (h_y, h_x) signed in [-N/2, N/2); q = h / L.
 *   - Complex arrays are interleaved float pairs (re, im) ("complex64").
 *   - Every pointer is owned by the caller and must stay valid until the
 *     work queued on `stream` has finished.  `stream` is a hipStream_t
 *     (NULL = the default stream).  Device pointers are marked "device",
 *     host pointers "host".
 *   - All calls return 0 (BIP_OK) or a negative BIP_E* code, never abort;
 *     bip_last_error() gives a message.  Argument validation happens on the
 *     host before anything is launched.  After an error the plan stays
 *     valid and the outputs are undefined.
 *   - A plan is not thread safe; different plans are independent.
 *   - Results are bitwise reproducible for identical inputs (no atomics in
 *     any reduction).
 */
#ifndef BIP_H
#define BIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  BIP_OK = 0,
  BIP_EINVAL = -1,       /* bad shape, range, or non power-of-two grid        */
  BIP_EUNSUPPORTED = -2, /* valid request outside what the library implements */
  BIP_ENOMEM = -3,       /* device allocation failed                          */
  BIP_EHIP = -4,         /* a HIP runtime call failed                         */
  BIP_ESTATE = -5        /* call out of order (e.g. signal before build)      */
};

enum { BIP_RECON_MAGNITUDE = 0, BIP_RECON_COMPLEX = 1 };
enum { BIP_PARENTS_LATTICE = 0, BIP_PARENTS_HEX = 1 };
enum { BIP_OUT_MAP = 0, BIP_OUT_QEELS = 1, BIP_OUT_BEAMS = 2, BIP_OUT_MAP_DIRECT = 3, BIP_OUT_CUBE = 4 };
enum { BIP_PREC_FP32 = 0, BIP_PREC_SPLIT_BF16 = 1, BIP_PREC_BF16 = 2, BIP_PREC_FP16 = 3 };

typedef struct bip_grid {
  int32_t ny, nx, nz;   /* pixels (powers of two, 64..1024) and slice count */
  double ly, lx, dz;    /* field of view and slice thickness (A)            */
} bip_grid;

typedef struct bip_optics {
  double energy_ev;     /* beam energy                                       */
  double alpha_rad;     /* probe convergence semi-angle: aperture |q| <= alpha/lambda */
  double theta_rad;     /* collection semi-angle: detector |q| <= theta/lambda        */
  int32_t partition;    /* parent lattice factor s >= 1 (s = 1: exact PRISM)         */
  int32_t recon_mode;   /* BIP_RECON_MAGNITUDE (eq. magpreserve) or BIP_RECON_COMPLEX */
  int32_t ckpt_stride;  /* 0: forward only; k >= 1: bip_build_smatrix also keeps the
                           transmitted state of every parent column at every k-th
                           slice (slice checkpoints) so that bip_eels_backward can
                           run; it recomputes the other slices of a segment from
                           its checkpoint (k = 1: nothing recomputed) */
  double s2_window_gb;  /* budget of the S2 window stacks (GiB; 0 = 48).  When the
                           windows of all atoms exceed it, the S2 sweep runs inside
                           bip_eels_signal in plane segments whose windows fit the
                           budget, each segment's atoms contracted before the next
                           segment is swept (one sweep per signal call) */
  int32_t parent_set;   /* BIP_PARENTS_LATTICE: parents on s Z^2 (`partition`);
                           BIP_PARENTS_HEX: the paper's hex rings (Alg. 3 build step):
                           DC plus n_radial rings, ring i (0-based) of n_angular (1 + i)
                           samples at radius (i + 1) / n_radial of the aperture (S1)
                           or detector (S2) disc, snapped to the nearest beam of the
                           set; Sibson weights against the finite parent set, beams
                           not strictly inside the parents' convex hull taking the
                           weights of their nearest hull-boundary point */
  int32_t n_radial, n_angular;  /* hex rings (>= 1 each); ignored for the lattice */
  int32_t focal;        /* 1: focal back-propagation of S1 (section "Magnitude-preserving
                           reconstruction and focal back-propagation"): the S1 parent
                           columns are gathered on an enlarged M x M window (M the
                           smallest power of two >= 2W, W <= 64), stepped back to the
                           scattering centroid of the atom's entrance-to-ionization
                           path (slice mid-depths above the plane weighted by their
                           projected potential on the window), interpolated there,
                           and the probe is stepped forward again and cropped to the
                           window; the steps treat the window as periodic.  Forward
                           only (bip_eels_backward returns BIP_EUNSUPPORTED). */
  int32_t s2_exact;     /* 1: S2 over every detector beam (each its own parent, no
                           interpolation): the exit side is exact, as Alg. 3 needs for
                           the energy-filtered 4D cube (BIP_OUT_CUBE) */
  int32_t interp_f;     /* PRISM interpolation factor f (section "Exact PRISM-EELS",
                           Alg. 2; Alg. 4 for the detector and the crop mask); 0 or 1:
                           every beam.  f > 1 (dividing ny and nx): only the aperture
                           and detector beams with h_y = h_x = 0 (mod f) are kept (the
                           lattice parents sit on the (s f)-lattice), the retained probe
                           coefficients and the detector sums are scaled by f^2, and an
                           atom contributes only at the scans of its crop mask: those
                           whose minimum-image displacement atom - rho (pixels, per
                           axis) lies in [-N/(2f), N/(2f)), the atom inside the
                           alias-free window of the N/f-periodic probe.  Forward only
                           (bip_eels_backward returns BIP_EUNSUPPORTED); not with
                           s2_exact (BIP_EUNSUPPORTED). */
} bip_optics;

typedef struct bip_plan bip_plan;

/*
 * bip_alloc -- device memory callbacks (optional).  Passage: the problem
 * statement of Algs. 4/5 ("Require") names the inputs; where their working
 * memory comes from is the caller's choice, so that e.g. a framework's
 * caching allocator serves it.
 *   alloc    returns `bytes` of device memory usable in stream order on
 *            `stream` (the hipStream_t of the call that allocates), or NULL
 *            on failure (the call then returns BIP_ENOMEM).
 *   release  gives back a block from alloc (same size and stream); the
 *            library calls it in stream order: work queued on `stream`
 *            before the call may still use the block, none after it.
 *   ctx      passed through unchanged.
 * With a NULL bip_alloc the library uses hipMallocAsync / hipFreeAsync on
 * the call's stream.  A plan's blocks are made on the stream of the call
 * that needs them; using one plan from several streams at once is not
 * supported.
 */
typedef struct bip_alloc {
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  void (*release)(void* ptr, size_t bytes, void* stream, void* ctx);
  void* ctx;
} bip_alloc;

/*
 * bip_plan_create -- geometry and workspace for one specimen.
 * Passage: Alg. 5 "Require" (aperture, detector semi-angle, crop windows,
 * parent counts) and the build step of Alg. 3 (parent set, cached
 * natural-neighbour weights, eq. nnw).
 *   grid, optics   host structs (copied).
 *   n_atoms        number of ionized atoms (>= 1).
 *   tau_xyz        host f64 [n_atoms][3] positions (x, y, z) in A; the atom
 *                  ionizes at the entrance of slice floor(z / dz) (clamped).
 *   win_size       host i32 [n_atoms] window side W (4 <= W <= min(ny, nx),
 *                  W % 4 == 0).
 *   win_origin     host i32 [n_atoms][2] window origin (oy, ox) in pixels,
 *                  taken mod N; the window wraps periodically.
 *   alloc          host struct (copied) or NULL: where every device block of
 *                  the plan comes from (plan tables, parent columns, window
 *                  stacks, checkpoints, workspaces of later calls).
 * Aperture and detector beams are enumerated on the host (q^2 <= (angle /
 * lambda)^2 in FP64, sorted by (h_y, h_x)); the Sibson weights of every beam
 * on the parent lattice s Z^2 and the propagator phase table are computed on
 * the GPU in FP64.  Parents are the lattice points with a weight > 1e-12 for
 * some beam.  Synchronizes `stream` (to size the parent sets).
 * Errors: BIP_EINVAL (shapes/ranges), BIP_EUNSUPPORTED (a parent outside the
 * signed index range [-N/2, N/2) of the grid, which would alias),
 * BIP_ENOMEM, BIP_EHIP.
 */
int bip_plan_create(const bip_grid* grid, const bip_optics* optics, int32_t n_atoms,
                    const double* tau_xyz, const int32_t* win_size, const int32_t* win_origin,
                    const bip_alloc* alloc, void* stream, bip_plan** out);

/*
 * bip_build_smatrix -- step (a): parent sweeps and window gathers.
 * Passage: eq. smatrix-advance (S1 advance), eq. s2 (S2 by transpose
 * multislice), eq. window-recon (cropped parent columns), Alg. 5 steps 1-4.
 *   V  device f32 [nz][ny][nx] projected potential (V*A); read only.
 * S1 parents start as unit plane waves exp(+2 pi i h_p.r/N) and advance
 * psi <- F^-1[P F[T_j psi]], T_j = exp(i sigma V_j); at each atom's plane
 * (before T_i) the W x W window is cropped and de-tilted by
 * exp(-2 pi i h_p.r/N).  S2 parents start as G^-1/2 exp(-2 pi i h_p.r/N) and
 * step v <- T_j F^-1[P F[v]] from slice nz-1 down; at each atom's plane
 * (after T_i) the window is cropped and de-tilted by exp(+2 pi i h_p.r/N).
 * Asynchronous on `stream`.  Errors: BIP_EINVAL, BIP_EHIP.
 */
int bip_build_smatrix(bip_plan* plan, const float* V, void* stream);

/*
 * bip_reconstruct_local -- step (b), materialized for one atom.
 * Passage: eq. window-recon with eq. magpreserve (or the complex sum).
 *   atom     index in [0, n_atoms).
 *   s1_out   device complex64 [B][W][W]: S1~^b on the window (aperture beam
 *            order of bip_query BIP_Q_BEAMS), or NULL.
 *   s2_out   device complex64 [n_det][W][W]: S2~^d (BIP_Q_DETECTOR order),
 *            or NULL.
 * Requires a prior bip_build_smatrix (else BIP_ESTATE).
 */
int bip_reconstruct_local(bip_plan* plan, int32_t atom, float* s1_out, float* s2_out,
                          void* stream);

/*
 * bip_eels_signal -- steps (b) + (c): core-loss intensities.
 * Passage: eq. coupling evaluated in probe order (psi = sum_b c_b(rho) S1~^b
 * on the window, U_n = H_n psi, a_d = sum_r S2~^d U_n), eq. map-sum and the
 * output reductions of section "Output modes".
 *   n_ch         channels per atom (>= 1).
 *   H            device complex64, ragged [atom][n_ch][W_a][W_a]: H_n0 on
 *                each atom's window (zero outside it).
 *   H_off        host i64 [n_atoms + 1] element offsets of each atom in H.
 *   atom_subset  host i32 [n_subset] atoms to include (NULL = all atoms);
 *                contributions are summed in the listed order.
 *   scan_sy/sx   raster S_y x S_x over the whole cell: rho_(u,v) =
 *                (u N_y/S_y, v N_x/S_x) pixels; output row p = u S_x + v.
 *   out_mode     BIP_OUT_MAP: out f32 [P]; BIP_OUT_QEELS: f32 [P][n_q]
 *                (h_x resolved, bin h_x + floor(theta L_x / lambda));
 *                BIP_OUT_BEAMS: f32 [P][n_det] (detector order of bip_query);
 *                BIP_OUT_CUBE: f32 [P][n_det], the energy-filtered 4D cube of
 *                Alg. 3 (eq. cube: partitioned S1, exact exit propagation);
 *                needs a plan with s2_exact = 1 (else BIP_EINVAL), on which
 *                the exact detector matrix carries the exit multislice of
 *                every scan position (eq. s2).
 *   precision    BIP_PREC_FP32 (FP32 MFMA), BIP_PREC_SPLIT_BF16 (hi+lo
 *                bf16 products, FP32 accumulate), BIP_PREC_BF16 or
 *                BIP_PREC_FP16 (one bf16 / fp16 product, FP32 accumulate).
 *                fp16 operands hold |values| up to 65504: the probe (unit
 *                norm) and S2 (|G_rr'| <= 1) fit for any input; the Gram
 *                operand Q needs n_ch * max|H|^2 below 65504 (overflow gives
 *                inf in the output).
 *   out          device f32, overwritten.
 * Probe coefficients are c_b = 1/sqrt(G B) (unit-norm probe, no aberrations).
 * The probe sum over beams is evaluated exactly as a fold of the beams by
 * (h_y mod S_y, h_x mod S_x) followed by an S_y x S_x DFT over the raster.
 * Errors: BIP_EINVAL, BIP_ESTATE (no build), BIP_ENOMEM, BIP_EHIP,
 * BIP_EUNSUPPORTED (S_y or S_x above 256).
 */
int bip_eels_signal(bip_plan* plan, int32_t n_ch, const float* H, const int64_t* H_off,
                    const int32_t* atom_subset, int32_t n_subset, int32_t scan_sy,
                    int32_t scan_sx, int32_t out_mode, int32_t precision, float* out,
                    void* stream);

/*
 * bip_eels_signal_edges -- several ionization edges and the configuration
 * average in one call, reusing the elastic matrices of the last
 * bip_build_smatrix.  Passage: the discussion's multi-edge batching and
 * frozen-phonon averaging (the final intensity is averaged over frozen-phonon
 * configurations, forward model), both on the same S1/S2 of Alg. 5.
 *   edges[e]   n_ch, H, H_off, atom_subset, n_subset and out as for
 *              bip_eels_signal, per edge (e.g. the sites and transition
 *              potentials of one element's edge); H_off is read only for the
 *              edge's atoms.
 *   accumulate 0: out = weight x signal; 1: out += weight x signal, so that
 *              calls after bip_build_smatrix of each frozen-phonon
 *              configuration k (with that configuration's H) and weight 1/K
 *              average the K intensities.
 * A plan whose S2 is streamed sweeps S2 once per call for all edges.
 * Errors as bip_eels_signal; BIP_EINVAL for a non-finite weight.
 */
typedef struct bip_edge {
  int32_t n_ch;
  const float* H;         /* device complex64 ragged [atom][n_ch][W][W] */
  const int64_t* H_off;   /* host i64 [n_atoms + 1] */
  const int32_t* atom_subset;  /* host i32 [n_subset], or NULL = all atoms */
  int32_t n_subset;
  float* out;             /* device f32, shape of out_mode */
} bip_edge;
int bip_eels_signal_edges(bip_plan* plan, int32_t n_edges, const bip_edge* edges, int32_t scan_sy,
                          int32_t scan_sx, int32_t out_mode, int32_t precision, int32_t accumulate,
                          float weight, void* stream);

/*
 * bip_eels_signal_noalloc -- bip_eels_signal for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, outputs and errors as
 * bip_eels_signal (same kernels); its workspace is a fixed device array of
 * bip_noalloc_scratch_bytes() bytes (64 MiB) inside the library, which every
 * device the library runs on holds until the process ends.  The call makes
 * no allocation of any kind; a request whose workspace exceeds the array is
 * refused with BIP_EUNSUPPORTED before anything is launched.  Every call on
 * one device shares that device's array (it keeps the last call's contents;
 * nothing read is assumed zero): calls that overlap in time on one device
 * race, so serialize them (one stream, or events).  The plan itself must
 * have been created beforehand (bip_plan_create allocates).
 */
int bip_eels_signal_noalloc(bip_plan* plan, int32_t n_ch, const float* H, const int64_t* H_off,
                            const int32_t* atom_subset, int32_t n_subset, int32_t scan_sy,
                            int32_t scan_sx, int32_t out_mode, int32_t precision, float* out,
                            void* stream);
size_t bip_noalloc_scratch_bytes(void);

/*
 * bip_eels_backward -- gradient of a map loss (step a16: adjoint of steps
 * a5..a14).  Passage: the forward model's multislice (eq. smatrix-advance,
 * eq. s2), eq. window-recon / eq. magpreserve and eq. coupling / eq. map-sum,
 * differentiated by hand in reverse order.
 * Requires a plan created with ckpt_stride >= 1 and a bip_build_smatrix of the
 * same V: the reverse sweeps read the slice checkpoints it kept.  All atoms
 * of the plan contribute; the map is the one bip_eels_signal returns for
 * out_mode BIP_OUT_MAP with the same H and raster.  The contraction and its
 * adjoint products are recomputed atom by atom (batched over chunks of atoms)
 * in `precision`.
 *   H, H_off, n_ch, scan_sy/sx   as for bip_eels_signal.
 *   precision  BIP_PREC_FP32 or BIP_PREC_SPLIT_BF16 (the products of the
 *              forward's split precision: FP16 Gram matrix, hi+lo BF16 for
 *              the rest); other values give BIP_EINVAL.
 *   dL_dI      device f32 [P]: dL/dI(rho) of the loss L(I) (e.g. 2 (I - I_t)).
 *   dL_dV      device f32 [nz][ny][nx], overwritten: dL/dV_j(r).
 *   dL_dHconj  device complex64, ragged like H, or NULL: the Wirtinger
 *              derivative dL/d conj(H_n(r)) (dL = 2 Re sum conj(g) dH).
 *   dHdx, dHdy device complex64, ragged like H, or NULL: dH/dtau_x, dH/dtau_y
 *              of each atom's transition potentials on its window.
 *   dL_dtau_xy device f64 [n_atoms][2] or NULL (needs dHdx, dHdy): the
 *              position gradient through the transition potentials,
 *              2 Re sum conj(g) dH/dtau.
 * The position gradient through the slice potentials is bip_potential_grad
 * of dL_dV.  Deterministic: no atomics, fixed reduction orders.
 * Errors: BIP_EINVAL, BIP_ESTATE (no build, or no checkpoints),
 * BIP_EUNSUPPORTED (raster sides above 256), BIP_ENOMEM, BIP_EHIP.
 */
int bip_eels_backward(bip_plan* plan, int32_t n_ch, const float* H, const int64_t* H_off,
                      int32_t scan_sy, int32_t scan_sx, int32_t precision, const float* dL_dI,
                      float* dL_dV,
                      float* dL_dHconj, const float* dHdx, const float* dHdy, double* dL_dtau_xy,
                      void* stream);

/*
 * bip_potential_build -- slice potentials from atom positions (the forward
 * model's projected potential, read as a Gaussian sum): atom a adds
 * sum_k amp[a][k] exp(-|r - r_a|^2 / (2 width[k]^2)) to slice floor(z_a/dz)
 * (clamped), periodic images out to 10 width[k]; evaluated in FP64.
 *   xyz    host f64 [n_atoms][3] (x, y, z) in A.
 *   amp    host f64 [n_atoms][n_terms] in V*A; width host f64 [n_terms] in A.
 *   alloc  as for bip_plan_create (its temporaries), or NULL.
 *   V      device f32 [nz][ny][nx], overwritten.
 * Asynchronous on `stream`: the host arrays are copied before the call
 * returns; the temporaries are released in stream order.
 */
int bip_potential_build(const bip_grid* grid, int32_t n_atoms, const double* xyz, int32_t n_terms,
                        const double* amp, const double* width, float* V, const bip_alloc* alloc,
                        void* stream);

/*
 * bip_potential_grad -- dL/dxyz of every atom from dL/dV (the adjoint of
 * bip_potential_build): dL/dx_a = sum_r dL/dV_j(r) dv_a(r)/dx_a, likewise y;
 * dL/dz = 0 (slice membership is piecewise constant).  FP64 reductions in a
 * fixed order (bitwise reproducible).
 *   dL_dV    device f32 [nz][ny][nx];
 *   dL_dxyz  device f64 [n_atoms][3], overwritten.
 * Asynchronous on `stream`, like bip_potential_build.
 */
int bip_potential_grad(const bip_grid* grid, int32_t n_atoms, const double* xyz, int32_t n_terms,
                       const double* amp, const double* width, const float* dL_dV,
                       double* dL_dxyz, const bip_alloc* alloc, void* stream);

/*
 * bip_parent_windows -- the cropped, de-tilted parent windows gathered by
 * bip_build_smatrix for one atom (step a8), for inspection and parity tests.
 *   which   1 (S1 parents) or 2 (S2 parents).
 *   out     device complex64 [Bp][W][W]; D_p(r) = S_p(r) exp(-/+ 2 pi i h_p.r/N).
 */
int bip_parent_windows(bip_plan* plan, int32_t atom, int32_t which, float* out, void* stream);

enum {
  BIP_Q_COUNTS = 0,   /* i64[8]: B, n_det, Bp1, Bp2, n_q, n_atoms, nnz1, nnz2 */
  BIP_Q_BEAMS = 1,    /* i32 [B][2]     aperture beams (h_y, h_x), sorted     */
  BIP_Q_DETECTOR = 2, /* i32 [n_det][2] detector beams, sorted                */
  BIP_Q_PARENTS1 = 3, /* i32 [Bp1][2]   S1 parents, sorted                    */
  BIP_Q_PARENTS2 = 4, /* i32 [Bp2][2]   S2 parents, sorted                    */
  BIP_Q_PLANES = 5,   /* i32 [n_atoms]  ionization plane of each atom         */
  BIP_Q_WEIGHTS1 = 6, /* CSR of w(1): i32 rowptr[B+1], i32 col[nnz1], f64 w[nnz1] packed
                         back to back in that order (host buffer)             */
  BIP_Q_WEIGHTS2 = 7, /* same for the detector weights w(2)                   */
  BIP_Q_SCALARS = 8,  /* f64[4]: lambda (A), sigma (rad/(V A)), parent columns per
                         sweep batch of the last sweep (0 before), number of S2
                         plane segments (0: S2 windows resident) */
  BIP_Q_MEMORY = 9    /* i64[3]: device bytes the plan holds now, the most it has
                         held, and the number of blocks it holds */
};

/* bip_query -- copy plan metadata into the host buffer `out`. */
int bip_query(const bip_plan* plan, int32_t what, void* out);

/*
 * bip_set_profiling -- when enable != 0, every kernel launch of the plan is
 * bracketed by HIP events recorded on the caller's stream (adds two event
 * records per launch; off by default).
 */
int bip_set_profiling(bip_plan* plan, int32_t enable);

/*
 * bip_stage_timings -- device time per stage accumulated while profiling was
 * on.  Synchronizes the recorded events.  ms, launches: host arrays of
 * BIP_N_STAGES entries, indexed by BIP_ST_*.  reset != 0 clears the totals.
 * Stages: TRANSMIT exp(i sigma V); S1_ROW / S1_COL and S2_ROW / S2_COL the
 * row and column FFT passes of the two parent sweeps (window gathers fused
 * into the row passes); INIT plane-wave parents; RECON S2~ reconstruction;
 * FOLD S1~ reconstruction fused with the residue fold and the first DFT of
 * the probe synthesis; PROBE its second DFT and operand store; DET the
 * detector contraction (beams, qEELS, direct map) or the quadratic form of
 * the map; REDUCE map partial sums; GRAM the Gram matrix of S2~.
 */
enum {
  BIP_ST_TRANSMIT = 0, BIP_ST_S1_ROW, BIP_ST_S1_COL, BIP_ST_S2_ROW, BIP_ST_S2_COL, BIP_ST_INIT,
  BIP_ST_RECON, BIP_ST_FOLD, BIP_ST_PROBE, BIP_ST_DET, BIP_ST_REDUCE, BIP_ST_GRAM, BIP_N_STAGES
};
int bip_stage_timings(bip_plan* plan, double* ms, int64_t* launches, int32_t reset);

/* bip_plan_destroy -- synchronizes the stream of the plan's last call and
 * releases every device block of the plan (through its bip_alloc). */
void bip_plan_destroy(bip_plan* plan);

/* bip_last_error -- message of the last failure on this thread ("" if none). */
const char* bip_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BIP_H */
