// C ABI of the map-loss gradient: bip_eels_backward, and the slice-potential
// helpers bip_potential_build / bip_potential_grad.
//
// The backward recomputes, atom by atom, what the forward contraction used
// (psi, S2~, the Gram matrix) in FP32, forms the cotangents of the parent
// windows, then runs the two parent sweeps in reverse with the slice
// checkpoints kept by bip_build_smatrix (every ckpt_stride-th slice; the slices
// between two checkpoints are recomputed per column batch), injecting the
// window cotangents at their planes and reducing dL/dV in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "bip_internal.h"
#include "host_common.h"

namespace bip {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kAdjGroups = 32;  // column groups of the adjoint row pass

// parent -> (beam, weight) lists of a CSR beam -> parent weight matrix
void transpose_csr(const std::vector<int32_t>& rp, const std::vector<int32_t>& col,
                   const std::vector<double>& w, int n_par, std::vector<int32_t>& trp,
                   std::vector<int32_t>& tb, std::vector<float>& tw) {
  const int nb = (int)rp.size() - 1;
  trp.assign(n_par + 1, 0);
  for (int32_t c : col) trp[c + 1]++;
  for (int p = 0; p < n_par; ++p) trp[p + 1] += trp[p];
  std::vector<int32_t> fill(trp.begin(), trp.end() - 1);
  tb.assign(col.size(), 0);
  tw.assign(col.size(), 0.f);
  for (int b = 0; b < nb; ++b)
    for (int k = rp[b]; k < rp[b + 1]; ++k) {
      const int q = fill[col[k]]++;
      tb[q] = b;
      tw[q] = (float)w[k];
    }
}

}  // namespace
}  // namespace bip

using namespace bip;

extern "C" {

int bip_eels_backward(bip_plan* p, int32_t n_ch, const float* H, const int64_t* H_off,
                      int32_t scan_sy, int32_t scan_sx, int32_t precision, const float* dL_dI,
                      float* dL_dV,
                      float* dL_dHconj, const float* dHdx, const float* dHdy, double* dL_dtau_xy,
                      void* stream) {
  if (!p || !H || !H_off || !dL_dI || !dL_dV) return err(BIP_EINVAL, "NULL argument");
  if (p->f > 1) return err(BIP_EUNSUPPORTED, "interp_f > 1 is forward only");
  if (!p->built) return err(BIP_ESTATE, "bip_build_smatrix has not run");
  if (!p->d_ckpt2) return err(BIP_ESTATE, "plan created without slice checkpoints (ckpt_stride 0)");
  if (p->focal) return err(BIP_EUNSUPPORTED, "focal back-propagation is forward only");
  if (n_ch < 1) return err(BIP_EINVAL, "n_ch must be >= 1");
  if (scan_sy < 1 || scan_sx < 1) return err(BIP_EINVAL, "scan raster must be >= 1 x 1");
  if (scan_sy > BIP_MAX_SCAN || scan_sx > BIP_MAX_SCAN)
    return err(BIP_EUNSUPPORTED, "scan raster sides above " + std::to_string(BIP_MAX_SCAN));
  if (precision != BIP_PREC_FP32 && precision != BIP_PREC_SPLIT_BF16)
    return err(BIP_EINVAL, "backward precision must be BIP_PREC_FP32 or BIP_PREC_SPLIT_BF16");
  if ((dHdx == nullptr) != (dHdy == nullptr)) return err(BIP_EINVAL, "dHdx and dHdy go together");
  if (dL_dtau_xy && !dHdx) return err(BIP_EINVAL, "dL_dtau_xy needs dHdx and dHdy");
  for (int a = 0; a < p->n_atoms; ++a)
    if (H_off[a + 1] - H_off[a] != (int64_t)n_ch * p->W[a] * p->W[a] || H_off[a] < 0)
      return err(BIP_EINVAL, "H_off inconsistent with n_ch and the window of atom " + std::to_string(a));
  hipStream_t st = (hipStream_t)stream;
  p->stream = st;
  const bip_grid& g = p->g;
  const int64_t G = (int64_t)g.ny * g.nx;
  const int P = scan_sy * scan_sx;
  const int64_t Ppad = roundup(P, 128);
  const int64_t Dpad = roundup(p->ndet, 128), Dk = roundup(p->ndet, 32);
  // operand precisions: as the forward's map (the Gram matrix on FP16 products
  // of a 2^8-scaled operand in split precision)
  const int prec = precision;
  const int gprec = gram_precision(prec, p->ndet);
  const float gsc = gprec == BIP_PREC_FP16 ? 256.f : 1.f;
  const int64_t esz = prec == BIP_PREC_FP32 ? 4 : 2, gesz = gprec == BIP_PREC_FP32 ? 4 : 2;
  const int BKF = gemm_bk(gprec);
  int Wmax = 0;
  for (int a = 0; a < p->n_atoms; ++a) Wmax = std::max(Wmax, p->W[a]);
  const int64_t W2m = (int64_t)Wmax * Wmax, kdm = roundup(W2m, 32), n1m = roundup(W2m, 128),
                ldfm = roundup(W2m, 64);
  // host tables: residue cells, synthesis and adjoint twiddles, probe jobs
  std::vector<int32_t>& cells = p->h_cells;
  cells.assign((size_t)P + 1 + p->B, 0);
  {
    std::vector<int32_t> cell_of(p->B);
    for (int b = 0; b < p->B; ++b) {
      const int hy = p->beams[2 * b], hx = p->beams[2 * b + 1];
      cell_of[b] = (((hy % scan_sy) + scan_sy) % scan_sy) * scan_sx + ((hx % scan_sx) + scan_sx) % scan_sx;
      cells[cell_of[b] + 1]++;
    }
    for (int i = 0; i < P; ++i) cells[i + 1] += cells[i];
    std::vector<int32_t> fill(cells.begin(), cells.begin() + P);
    for (int b = 0; b < p->B; ++b) cells[P + 1 + fill[cell_of[b]]++] = b;
  }
  std::vector<float2>& tws = p->h_tws;  // twx, twy, conj(twx), conj(twy)
  tws.resize(2 * ((size_t)scan_sx + scan_sy));
  for (int k = 0; k < scan_sx; ++k) {
    const double t = 2.0 * kPi * k / scan_sx;
    tws[k] = make_float2((float)std::cos(t), (float)-std::sin(t));
    tws[scan_sx + scan_sy + k] = make_float2((float)std::cos(t), (float)std::sin(t));
  }
  for (int k = 0; k < scan_sy; ++k) {
    const double t = 2.0 * kPi * k / scan_sy;
    tws[scan_sx + k] = make_float2((float)std::cos(t), (float)-std::sin(t));
    tws[2 * scan_sx + scan_sy + k] = make_float2((float)std::cos(t), (float)std::sin(t));
  }
  std::vector<ProbeJob>& jprobe = p->h_probe;
  jprobe.assign(p->n_atoms, ProbeJob{});
  for (int a = 0; a < p->n_atoms; ++a) {
    ProbeJob& j = jprobe[a];
    j.win_off = p->off1[a];
    j.h_off = H_off[a];
    j.W = p->W[a];
    j.oy = p->oy[a];
    j.ox = p->ox[a];
    j.kd = (int32_t)roundup((int64_t)p->W[a] * p->W[a], 32);
    j.ldf = (int32_t)roundup((int64_t)p->W[a] * p->W[a], 64);
    j.t0 = a == 0 ? 0 : jprobe[a - 1].t0 + (jprobe[a - 1].W * jprobe[a - 1].W + 63) / 64;
  }
  // transposed weights (parent -> beams), built once per plan
  if (!p->d_tp1_rp) {
    std::vector<int32_t> rp1, tb1, rp2, tb2;
    std::vector<float> tw1, tw2;
    int rc;
    transpose_csr(p->rp1, p->col1, p->w1, p->Bp1, rp1, tb1, tw1);
    transpose_csr(p->rp2, p->col2, p->w2, p->Bp2, rp2, tb2, tw2);
    if ((rc = upload(p, &p->d_tp1_rp, rp1, st)) || (rc = upload(p, &p->d_tp1_b, tb1, st)) ||
        (rc = upload(p, &p->d_tp1_w, tw1, st)) || (rc = upload(p, &p->d_tp2_rp, rp2, st)) ||
        (rc = upload(p, &p->d_tp2_b, tb2, st)) || (rc = upload(p, &p->d_tp2_w, tw2, st)))
      return rc;
    HIPCHK(hipStreamSynchronize(st), "weight tables");  // once per plan: the host vectors go out of scope
  }
  // Workspace.  The products of the contraction backward run batched over
  // chunks of atoms (one launch per product and chunk, grid z or the Gram job
  // list over the atoms), so that small windows still fill the chip; every
  // atom of a chunk gets a block sized for the largest window.
  const int nbmax = std::max(p->B, p->ndet);
  const int batch = p->column_batch > 0 ? p->column_batch : std::max(p->Bp1, p->Bp2);
  const int groups = std::min(kAdjGroups, std::max(1, batch));
  const int64_t bX = (int64_t)P * ldfm;  // raster DFT workspace (complex)
  const int64_t bPsi = Ppad * kdm;       // psi^T [Ppad][kd] (FP32 planes)
  const int64_t bS2b = n1m * Dk;         // S2~ K-blocked
  const int64_t bS2d = Dpad * kdm;       // S2~ [d][r]
  const int64_t bQ = n1m * kdm;          // Q, K (planes); G, R (complex) [n1][kd]
  const int64_t bA = n1m * Ppad;         // A1, B1 [n1][Ppad] (planes)
  const int64_t bGp = Ppad * kdm;        // g_psi (complex)
  const int64_t bGs = Dpad * kdm;        // g_S2~ (complex)
  const int64_t per_atom = 8 * (bX + bPsi + bS2b + bS2d + 4 * bQ + 2 * bA + bGp + bGs) + 16 * 256;
  size_t fixed = 0;
  auto sz = [&](size_t bytes) { fixed += (size_t)roundup((int64_t)bytes, 256); };
  sz((size_t)bX * 8);              // Z
  sz((size_t)nbmax * W2m * 8);     // g_z
  sz((size_t)nbmax * W2m * 4);     // gamma
  sz((size_t)n_ch * W2m * 8);      // g_H scratch
  sz((size_t)Ppad * 4);            // Ibar
  sz((size_t)p->n_atoms * 16);     // dtau
  sz((size_t)groups * G * 4);      // dV partials
  sz(cells.size() * 4);
  sz(tws.size() * 8);
  sz(jprobe.size() * sizeof(ProbeJob));
  sz(4 * (size_t)p->n_atoms * sizeof(GemmJob));
  // checkpoint segments longer than one slice are recomputed per column batch:
  // a forward state [batch][G] and the K - 1 recomputed slices [K - 1][batch][G]
  const int K = p->o.ckpt_stride;
  const int bmax = std::max(balanced_batch(p->Bp1, batch), balanced_batch(p->Bp2, batch));
  if (K > 1) sz((size_t)K * bmax * G * 8);
  const char* env = std::getenv("BIP_WORKSPACE_GB");
  const double budget_gb = env ? std::atof(env) : 24.0;
  const int64_t budget = (int64_t)(budget_gb * (1 << 30));
  const int nat_max =
      (int)std::max<int64_t>(1, std::min<int64_t>(p->n_atoms, (budget - (int64_t)fixed) / per_atom));
  int rc = ensure_work(p, fixed + (size_t)nat_max * per_atom + 4096, st);
  if (rc) return rc;
  Workspace ws{(char*)p->d_work, 0};
  float2* Z = (float2*)ws.take((size_t)bX * 8);
  float2* gz = (float2*)ws.take((size_t)nbmax * W2m * 8);
  float* gam = (float*)ws.take((size_t)nbmax * W2m * 4);
  float2* gHs = (float2*)ws.take((size_t)n_ch * W2m * 8);
  float* ibar = (float*)ws.take((size_t)Ppad * 4);
  double* dtau = (double*)ws.take((size_t)p->n_atoms * 16);
  float* dvp = (float*)ws.take((size_t)groups * G * 4);
  int32_t* d_cells = (int32_t*)ws.take(cells.size() * 4);
  float2* d_tws = (float2*)ws.take(tws.size() * 8);
  ProbeJob* d_probe = (ProbeJob*)ws.take(jprobe.size() * sizeof(ProbeJob));
  GemmJob* d_jobs = (GemmJob*)ws.take(4 * (size_t)p->n_atoms * sizeof(GemmJob));
  const int64_t NA = nat_max;
  float2* X = (float2*)ws.take((size_t)(NA * bX) * 8);
  // operand planes: 8 bytes per element in FP32 (two planes) and in split
  // precision (four 2-byte planes); plane strides below are in elements
  char* psiT = (char*)ws.take((size_t)(2 * NA * bPsi) * 4);
  char* S2b = (char*)ws.take((size_t)(2 * NA * bS2b) * 4);
  char* S2d = (char*)ws.take((size_t)(2 * NA * bS2d) * 4);
  char* Qp = (char*)ws.take((size_t)(2 * NA * bQ) * 4);
  float2* Gm = (float2*)ws.take((size_t)(NA * bQ) * 8);
  char* A1 = (char*)ws.take((size_t)(2 * NA * bA) * 4);
  char* B1 = (char*)ws.take((size_t)(2 * NA * bA) * 4);
  float2* R = (float2*)ws.take((size_t)(NA * bQ) * 8);
  char* Kp = (char*)ws.take((size_t)(2 * NA * bQ) * 4);
  float2* gpsi = (float2*)ws.take((size_t)(NA * bGp) * 8);
  float2* gS2 = (float2*)ws.take((size_t)(NA * bGs) * 8);
  float2* rec = K > 1 ? (float2*)ws.take((size_t)K * bmax * G * 8) : nullptr;
  if (ws.used > p->work_bytes) return err(BIP_ENOMEM, "internal: backward workspace");
  // the atom's slot in its chunk (chunks are consecutive runs of nat_max atoms)
  for (int a = 0; a < p->n_atoms; ++a) {
    jprobe[a].fx_off = (a % nat_max) * bX;
    jprobe[a].out_off = (a % nat_max) * bPsi;
  }
  HIPCHK(hipMemcpyAsync(d_cells, cells.data(), cells.size() * 4, hipMemcpyHostToDevice, st), "cells");
  HIPCHK(hipMemcpyAsync(d_tws, tws.data(), tws.size() * 8, hipMemcpyHostToDevice, st), "twiddles");
  HIPCHK(hipMemcpyAsync(d_probe, jprobe.data(), jprobe.size() * sizeof(ProbeJob), hipMemcpyHostToDevice, st), "jobs");
  HIPCHK(launch_zero(ibar, Ppad, st), "zero");
  HIPCHK(hipMemcpyAsync(ibar, dL_dI, (size_t)P * 4, hipMemcpyDeviceToDevice, st), "dL/dI");
  HIPCHK(launch_zero((float*)p->d_gwin1, 2 * p->win1_elems, st), "zero");
  HIPCHK(launch_zero((float*)p->d_gwin2, 2 * p->win2_elems, st), "zero");
  const float cb = (float)(1.0 / std::sqrt((double)g.ny * g.nx * p->B));
  ProbeArgs pa{};
  pa.win = p->d_win1;
  pa.n_par = p->Bp1;
  pa.rowptr = p->d_rp1;
  pa.col = p->d_col1;
  pa.w = p->d_w1;
  pa.ellc = p->d_ellc1;
  pa.ellw = p->d_ellw1;
  pa.beams = p->d_beams;
  pa.cell_start = d_cells;
  pa.cell_beams = d_cells + P + 1;
  pa.twx = d_tws;
  pa.twy = d_tws + scan_sx;
  pa.tw = p->d_tw;
  pa.L = p->L;
  pa.ny = g.ny;
  pa.nx = g.nx;
  pa.mode = p->o.recon_mode;
  pa.Sy = scan_sy;
  pa.Sx = scan_sx;
  pa.P = P;
  pa.Ppad = (int)Ppad;
  pa.cb = cb;
  pa.fx = X;
  pa.out = psiT;
  pa.out_plane = NA * bPsi;
  pa.H = (const float2*)H;
  pa.n_ch = n_ch;
  const float2* twxc = d_tws + scan_sx + scan_sy;
  const float2* twyc = twxc + scan_sx;
  // four products per atom: Gram (G, Q), R, g_psi and g_S2~, each with the
  // atom's blocks as operand and output offsets
  std::vector<GemmJob>& hj = p->h_jobs2;
  hj.assign(4 * (size_t)p->n_atoms, GemmJob{});
  const int na = p->n_atoms;
  for (int a = 0; a < na; ++a) {
    const int64_t i = a % nat_max;
    const int W2 = p->W[a] * p->W[a];
    const int64_t kd = roundup(W2, 32), n1 = roundup(W2, 128);
    GemmJob& q = hj[a];
    q.a_off = q.b_off = i * bS2b;
    q.out_off = i * bQ;
    q.K = (int32_t)Dk;
    q.lda = q.ldb = BKF;
    q.kstride = (int32_t)(n1 * BKF);
    q.m_lim = q.n_lim = W2;
    q.W2 = W2;
    q.ldo = (int32_t)kd;
    q.h_off = H_off[a];
    GemmJob& rj = hj[na + a];
    rj.a_off = rj.b_off = i * bA;
    rj.out_off = i * bQ;
    rj.K = rj.lda = rj.ldb = (int32_t)Ppad;
    rj.m_lim = rj.n_lim = W2;
    rj.W2 = W2;
    rj.ldo = (int32_t)kd;
    GemmJob& pj = hj[2 * na + a];
    pj.a_off = i * bPsi;
    pj.b_off = i * bQ;
    pj.out_off = i * bGp;
    pj.K = pj.lda = pj.ldb = (int32_t)kd;
    pj.m_lim = (int32_t)Ppad;
    pj.n_lim = W2;
    pj.W2 = W2;
    pj.ldo = (int32_t)kd;
    GemmJob& sj = hj[3 * na + a];
    sj.a_off = i * bS2d;
    sj.b_off = i * bQ;
    sj.out_off = i * bGs;
    sj.K = sj.lda = sj.ldb = (int32_t)kd;
    sj.m_lim = (int32_t)Dpad;
    sj.n_lim = W2;
    sj.W2 = W2;
    sj.ldo = (int32_t)kd;
  }
  // Gram launches: one per chunk of nat_max atoms (their slot rows set here)
  std::vector<int64_t> gram_gx;
  for (int c0 = 0; c0 < na; c0 += nat_max) {
    const int nat = std::min(nat_max, na - c0);
    int tiles = 0;
    for (int a = c0; a < c0 + nat; ++a) tiles = std::max(tiles, (int)(roundup((int64_t)p->W[a] * p->W[a], 128) / 128));
    gram_gx.push_back(gemm_gram_plan(&hj[c0], nat, tiles));
    if (gram_gx.back() > 0x7fffffff) return err(BIP_EUNSUPPORTED, "Gram launch beyond the grid limit");
  }
  HIPCHK(hipMemcpyAsync(d_jobs, hj.data(), hj.size() * sizeof(GemmJob), hipMemcpyHostToDevice, st), "jobs");
  for (int c0 = 0; c0 < na; c0 += nat_max) {
    const int nat = std::min(nat_max, na - c0);
    int max_n1 = 0, max_kd = 0;
    for (int a = c0; a < c0 + nat; ++a) {
      const int W2 = p->W[a] * p->W[a];
      max_n1 = std::max(max_n1, (int)roundup(W2, 128));
      max_kd = std::max(max_kd, (int)roundup(W2, 32));
    }
    // psi^T [rho][r] (FP32) of every atom of the chunk, exactly as the forward synthesis
    pa.jobs = d_probe + c0;
    const ProbeJob& jl = jprobe[c0 + nat - 1];
    HIPCHK(launch_probe_fold_x(pa, jprobe[c0].t0, jl.t0 + (jl.W * jl.W + 63) / 64 - jprobe[c0].t0, nat, st),
           "probe fold");
    HIPCHK(launch_probe_y(pa, prec, false, max_kd, nat, st), "probe synthesis");
    for (int a = c0; a < c0 + nat; ++a) {
      const int64_t i = a - c0;
      const int W2 = p->W[a] * p->W[a];
      const int64_t kd = roundup(W2, 32), n1 = roundup(W2, 128);
      // S2~ K-blocked (Gram) and [d][r] (gradient product)
      ReconArgs ra = recon_args(p, a, 2);
      ra.scale = gsc;
      HIPCHK(launch_recon_operand(ra, S2b + i * bS2b * gesz, 0, gprec, Dk, n1, Dk, NA * bS2b, st),
             "recon S2");
      HIPCHK(launch_recon_operand(recon_args(p, a, 2), S2d + i * bS2d * esz, 1, prec, kd, Dpad, kd,
                                  NA * bS2d, st), "recon S2");
      // conj(psi) and Ibar psi as [r][rho] operands of R
      HIPCHK(launch_psi_transpose(prec, psiT + i * bPsi * esz, NA * bPsi, (int)kd, W2, P, (int)Ppad,
                                  (int)n1, ibar, A1 + i * bA * esz, B1 + i * bA * esz, NA * bA, st),
             "psi transpose");
    }
    // Gram matrix G and Q = G o Hc
    GemmArgs ga{};
    ga.H = (const float2*)H;
    ga.n_ch = n_ch;
    ga.A = ga.B = S2b;
    ga.a_plane = ga.b_plane = NA * bS2b;
    ga.jobs = d_jobs + c0;
    ga.njobs = nat;
    ga.out = Qp;
    ga.out_plane = NA * bQ;
    ga.out2 = Gm;
    ga.tiles = max_n1 / 128;
    ga.gscale = 1.f / (gsc * gsc);
    HIPCHK(launch_zgemm_gram(gprec, prec, ga, (int)gram_gx[c0 / nat_max], st), "Gram");
    // R = conj(psi) diag(Ibar) psi^T over the raster
    GemmArgs gr{};
    gr.A = A1;
    gr.B = B1;
    gr.a_plane = gr.b_plane = NA * bA;
    gr.jobs = d_jobs + na + c0;
    gr.njobs = nat;
    gr.out = R;
    gr.m_store = max_n1;
    HIPCHK(launch_zgemm(prec, EPI_STORE + EPI_CONJ_A, gr, max_n1 / 128, max_n1 / 128, nat, st), "R");
    for (int a = c0; a < c0 + nat; ++a) {
      const int64_t i = a - c0;
      const int W2 = p->W[a] * p->W[a];
      const int64_t kd = roundup(W2, 32), n1 = roundup(W2, 128);
      HIPCHK(launch_kmat(prec, R + i * bQ, (const float2*)H + H_off[a], n_ch, W2, (int)kd, (int)n1,
                         Kp + i * bQ * esz, NA * bQ, st), "K");
    }
    // g_psi = Ibar (Q psi) and g_S2~ = S2~ K^T
    GemmArgs gp{};
    gp.A = psiT;
    gp.a_plane = NA * bPsi;
    gp.B = Qp;
    gp.b_plane = NA * bQ;
    gp.jobs = d_jobs + 2 * na + c0;
    gp.njobs = nat;
    gp.out = gpsi;
    gp.rowscale = ibar;
    gp.m_store = (int)Ppad;
    HIPCHK(launch_zgemm(prec, EPI_STORE, gp, (int)(Ppad / 128), max_n1 / 128, nat, st), "g_psi");
    GemmArgs gs{};
    gs.A = S2d;
    gs.a_plane = NA * bS2d;
    gs.B = Kp;
    gs.b_plane = NA * bQ;
    gs.jobs = d_jobs + 3 * na + c0;
    gs.njobs = nat;
    gs.out = gS2;
    gs.m_store = (int)Dpad;
    HIPCHK(launch_zgemm(prec, EPI_STORE, gs, (int)(Dpad / 128), max_n1 / 128, nat, st), "g_S2");
    for (int a = c0; a < c0 + nat; ++a) {
      const int64_t i = a - c0;
      const int W2 = p->W[a] * p->W[a];
      const int64_t kd = roundup(W2, 32), ldf = roundup(W2, 64);
      const float2* Ha = (const float2*)H + H_off[a];
      // transition-potential cotangent and the position gradient through H
      float2* gH = dL_dHconj ? (float2*)dL_dHconj + H_off[a] : gHs;
      HIPCHK(launch_grad_h(Gm + i * bQ, R + i * bQ, Ha, n_ch, W2, (int)kd, gH, st), "g_H");
      if (dHdx)
        HIPCHK(launch_grad_tau(gH, (const float2*)dHdx + H_off[a], (const float2*)dHdy + H_off[a],
                               n_ch * W2, dtau + 2 * a, st), "dtau");
      // adjoint of the probe sum: Z[a][c][r] = sum_{u,v} exp(+2 pi i (a u/S_y + c v/S_x)) g_psi
      HIPCHK(launch_dft_pass(gpsi + i * bGp, X, scan_sx, kd, scan_sx * kd, ldf, scan_sx * ldf, scan_sy, W2,
                             twxc, st), "adjoint DFT x");
      HIPCHK(launch_dft_pass(X, Z, scan_sy, scan_sx * ldf, ldf, scan_sx * ldf, ldf, scan_sx, W2, twyc, st),
             "adjoint DFT y");
      // reconstruction adjoints -> window cotangents
      HIPCHK(launch_recon_adjoint(recon_args(p, a, 1), 1, Z, ldf, scan_sy, scan_sx, cb, gz, gam,
                                  p->d_par1, p->Bp1, p->d_tp1_rp, p->d_tp1_b, p->d_tp1_w,
                                  p->d_gwin1 + p->off1[a], st), "recon adjoint S1");
      HIPCHK(launch_recon_adjoint(recon_args(p, a, 2), 2, gS2 + i * bGs, kd, scan_sy, scan_sx, cb, gz, gam,
                                  p->d_par2, p->Bp2, p->d_tp2_rp, p->d_tp2_b, p->d_tp2_w,
                                  p->d_gwin2 + p->off2[a], st), "recon adjoint S2");
    }
  }
  // ----------------------------------------------------- reverse sweeps
  HIPCHK(launch_zero(dL_dV, G * g.nz, st), "zero dV");
  const float two_sigma = (float)(2.0 * p->sigma);
  GatherArgs inj1{p->d_grec1, p->d_gwin1}, inj2{p->d_grec2, p->d_gwin2};
  auto ps = [&](int j) { return p->plane_start[j]; };
  // The state after T_j of slice j: the checkpoint itself at a segment start,
  // else recomputed for the batch.  recompute() advances a copy of a segment's
  // checkpoint through the later slices of the segment, keeping each one.
  auto seg_slot = [&](int r) { return rec + (int64_t)(1 + r) * bmax * G; };
  auto recompute = [&](const float2* ck, int nc, int n_more, auto slice_of, const int2* par) -> int {
    if (n_more <= 0) return BIP_OK;
    HIPCHK(hipMemcpyAsync(rec, ck, (size_t)nc * G * 8, hipMemcpyDeviceToDevice, st), "segment copy");
    GatherArgs none{nullptr, nullptr};
    HIPCHK(launch_row_pass(ROW_FWD, rec, nc, g.ny, g.nx, nullptr, p->d_tw, p->L, par, 0, none, 0, 0, 0,
                           nullptr, st),
           "segment row transform");
    for (int r = 0; r < n_more; ++r) {
      const int j = slice_of(r);
      HIPCHK(launch_col_pass(rec, nc, g.ny, g.nx, p->d_prop, p->d_tw, p->L, st), "segment column pass");
      HIPCHK(launch_row_pass(ROW_INV | ROW_T | ROW_FWD | ROW_SAVE, rec, nc, g.ny, g.nx, p->d_T + j * G,
                             p->d_tw, p->L, par, 0, none, 0, 0, 0, seg_slot(r), st),
             "segment row pass");
    }
    return BIP_OK;
  };
  // S1: psi_{j+1} = P(T_j psi_j); windows of plane j come from psi_j
  if (p->i_max > 0) {
    const int batch1 = balanced_batch(p->Bp1, batch);
    for (int c0 = 0; c0 < p->Bp1; c0 += batch1) {
      const int nc = std::min(batch1, p->Bp1 - c0);
      float2* s1 = p->d_state1 + (int64_t)c0 * G;
      const int grp = std::min(groups, nc);
      const int i = p->i_max;
      HIPCHK(launch_row_adjoint(ADJ_ZERO | ADJ_INJ_AFTER | ADJ_FWD, s1, nc, g.ny, g.nx, nullptr,
                                p->d_tw, p->L, inj1, ps(i), ps(i + 1), c0, nullptr, 0.f, nullptr, grp, st),
             "S1 adjoint start");
      for (int m = (p->i_max - 1) / K; m >= 0; --m) {
        const int js = m * K, je = std::min(js + K, p->i_max) - 1;  // slices js .. je
        const float2* ck = p->d_ckpt1 + ((int64_t)m * p->Bp1 + c0) * G;
        int rc = recompute(ck, nc, je - js, [&](int r) { return js + 1 + r; }, p->d_par1 + c0);
        if (rc) return rc;
        for (int j = je; j >= js; --j) {
          const float2* u = j == js ? ck : seg_slot(j - js - 1);
          HIPCHK(launch_col_pass(s1, nc, g.ny, g.nx, p->d_prop_conj, p->d_tw, p->L, st), "S1 adjoint column pass");
          int flags = ADJ_INV | ADJ_DV;
          if (j > 0) flags |= ADJ_CONJT | ADJ_INJ_AFTER | ADJ_FWD;
          HIPCHK(launch_row_adjoint(flags, s1, nc, g.ny, g.nx, p->d_T + j * G, p->d_tw, p->L, inj1,
                                    ps(j), ps(j + 1), c0, u, two_sigma, dvp, grp, st),
                 "S1 adjoint row pass");
          HIPCHK(launch_dv_reduce(dvp, grp, G, dL_dV + j * G, st), "dV reduce");
        }
      }
    }
  }
  // S2: v_j = T_j P v_{j+1}; windows of plane j come from v_j.  Segments from
  // the exit: m covers slices nz-1-mK down to nz-K-mK (and not below i_min).
  const int batch2 = balanced_batch(p->Bp2, batch);
  const int nseg2 = (g.nz - p->i_min + K - 1) / K;
  for (int c0 = 0; c0 < p->Bp2; c0 += batch2) {
    const int nc = std::min(batch2, p->Bp2 - c0);
    float2* s2 = p->d_state2 + (int64_t)c0 * G;
    const int grp = std::min(groups, nc);
    for (int m = nseg2 - 1; m >= 0; --m) {
      const int jh = g.nz - 1 - m * K, jl = std::max(p->i_min, jh - K + 1);  // slices jh .. jl
      const float2* ck = p->d_ckpt2 + ((int64_t)m * p->Bp2 + c0) * G;
      int rc = recompute(ck, nc, jh - jl, [&](int r) { return jh - 1 - r; }, p->d_par2 + c0);
      if (rc) return rc;
      for (int j = jl; j <= jh; ++j) {
        const float2* v = j == jh ? ck : seg_slot(jh - 1 - j);
        int flags = ADJ_INJ_BEFORE | ADJ_DV;
        flags |= j == p->i_min ? ADJ_ZERO : ADJ_INV;
        if (j < g.nz - 1) flags |= ADJ_CONJT | ADJ_FWD;
        if (j > p->i_min)
          HIPCHK(launch_col_pass(s2, nc, g.ny, g.nx, p->d_prop_conj, p->d_tw, p->L, st), "S2 adjoint column pass");
        HIPCHK(launch_row_adjoint(flags, s2, nc, g.ny, g.nx, p->d_T + j * G, p->d_tw, p->L, inj2, ps(j),
                                  ps(j + 1), c0, v, two_sigma, dvp, grp, st),
               "S2 adjoint row pass");
        HIPCHK(launch_dv_reduce(dvp, grp, G, dL_dV + j * G, st), "dV reduce");
      }
    }
  }
  if (dL_dtau_xy)
    HIPCHK(hipMemcpyAsync(dL_dtau_xy, dtau, (size_t)p->n_atoms * 16, hipMemcpyDeviceToDevice, st), "dtau");
  return BIP_OK;
}

}  // extern "C"

namespace {

// Device temporaries of the potential helpers, released in stream order.
struct Temps {
  const bip_alloc* al;
  hipStream_t st;
  std::vector<std::pair<void*, size_t>> blocks;
  template <typename T>
  T* take(size_t count) {
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    void* p = raw_alloc(al, bytes, st);
    if (p) blocks.push_back({p, bytes});
    return (T*)p;
  }
  ~Temps() {
    for (auto& b : blocks) raw_release(al, b.first, b.second, st);
  }
};

// Terms (x, y, A, w) of every (atom, Gaussian) grouped by slice.
int slice_terms(const bip_grid& g, int n_atoms, const double* xyz, int n_terms, const double* amp,
                const double* width, std::vector<double>& terms, std::vector<int64_t>& start,
                std::vector<int32_t>& owner) {
  if (g.nz < 1 || g.ny < 1 || g.nx < 1 || !(g.ly > 0) || !(g.lx > 0) || !(g.dz > 0))
    return err(BIP_EINVAL, "bad grid");
  if (n_atoms < 0 || n_terms < 1) return err(BIP_EINVAL, "n_atoms >= 0 and n_terms >= 1");
  for (int k = 0; k < n_terms; ++k)
    if (!(width[k] > 0)) return err(BIP_EINVAL, "widths must be > 0");
  std::vector<std::vector<int32_t>> by(g.nz);
  for (int a = 0; a < n_atoms; ++a) {
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(xyz[3 * a + c])) return err(BIP_EINVAL, "non-finite atom position");
    const int j = std::min(std::max((int)std::floor(xyz[3 * a + 2] / g.dz), 0), g.nz - 1);
    by[j].push_back(a);
  }
  terms.clear();
  owner.clear();
  start.assign(g.nz + 1, 0);
  for (int j = 0; j < g.nz; ++j) {
    for (int a : by[j])
      for (int k = 0; k < n_terms; ++k) {
        terms.insert(terms.end(), {xyz[3 * a], xyz[3 * a + 1], amp[(int64_t)a * n_terms + k], width[k]});
        owner.push_back(a);
      }
    start[j + 1] = (int64_t)owner.size();
  }
  return BIP_OK;
}

}  // namespace

extern "C" {

int bip_potential_build(const bip_grid* grid, int32_t n_atoms, const double* xyz, int32_t n_terms,
                        const double* amp, const double* width, float* V, const bip_alloc* alloc,
                        void* stream) {
  if (!grid || !V || (n_atoms > 0 && (!xyz || !amp)) || !width) return err(BIP_EINVAL, "NULL argument");
  if (alloc && (!alloc->alloc || !alloc->release)) return err(BIP_EINVAL, "bip_alloc needs both callbacks");
  const bip_grid g = *grid;
  std::vector<double> terms;
  std::vector<int64_t> start;
  std::vector<int32_t> owner;
  int rc = slice_terms(g, n_atoms, xyz, n_terms, amp, width, terms, start, owner);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const int64_t nt_all = (int64_t)owner.size();
  Temps tmp{alloc, st, {}};
  double* d_terms = tmp.take<double>(terms.size());
  double* d_prof = tmp.take<double>((size_t)nt_all * (g.ny + g.nx));
  int64_t* d_start = tmp.take<int64_t>(start.size());
  if (!d_terms || !d_prof || !d_start) return err(BIP_ENOMEM, "potential build temporaries");
  // pageable host sources: HIP copies them synchronously, so the vectors may
  // go out of scope when the calls return
  if (!terms.empty())
    HIPCHK(hipMemcpyAsync(d_terms, terms.data(), terms.size() * 8, hipMemcpyHostToDevice, st), "terms");
  HIPCHK(hipMemcpyAsync(d_start, start.data(), start.size() * 8, hipMemcpyHostToDevice, st), "terms");
  HIPCHK(launch_profiles(d_terms, nt_all, g.ny, g.nx, g.ly, g.lx, 0, d_prof, nullptr, st), "profiles");
  HIPCHK(launch_build_slices(d_terms, d_prof, d_start, g.nz, g.ny, g.nx, V, st), "potential build");
  return BIP_OK;
}

int bip_potential_grad(const bip_grid* grid, int32_t n_atoms, const double* xyz, int32_t n_terms,
                       const double* amp, const double* width, const float* dL_dV,
                       double* dL_dxyz, const bip_alloc* alloc, void* stream) {
  if (!grid || !dL_dV || !dL_dxyz || (n_atoms > 0 && (!xyz || !amp)) || !width)
    return err(BIP_EINVAL, "NULL argument");
  if (alloc && (!alloc->alloc || !alloc->release)) return err(BIP_EINVAL, "bip_alloc needs both callbacks");
  const bip_grid g = *grid;
  std::vector<double> terms;
  std::vector<int64_t> start;
  std::vector<int32_t> owner;
  int rc = slice_terms(g, n_atoms, xyz, n_terms, amp, width, terms, start, owner);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  int64_t most = 1;
  for (int j = 0; j < g.nz; ++j) most = std::max(most, start[j + 1] - start[j]);
  const int64_t nt_all = (int64_t)owner.size();
  // terms of one atom are consecutive: its first term
  std::vector<int64_t> first(std::max(n_atoms, 1), 0);
  for (int64_t t = nt_all - 1; t >= 0; --t) first[owner[t]] = t;
  Temps tmp{alloc, st, {}};
  double* d_terms = tmp.take<double>(terms.size());
  double* d_prof = tmp.take<double>((size_t)nt_all * (g.ny + g.nx));
  double* d_dprof = tmp.take<double>((size_t)nt_all * (g.ny + g.nx));
  double* d_out = tmp.take<double>(2 * (size_t)nt_all);
  double* d_part = tmp.take<double>((size_t)grad_part_doubles(nt_all, g.ny));
  int64_t* d_start = tmp.take<int64_t>(start.size());
  int64_t* d_first = tmp.take<int64_t>(first.size());
  if (!d_terms || !d_prof || !d_dprof || !d_out || !d_part || !d_start || !d_first)
    return err(BIP_ENOMEM, "potential gradient temporaries");
  if (!terms.empty())
    HIPCHK(hipMemcpyAsync(d_terms, terms.data(), terms.size() * 8, hipMemcpyHostToDevice, st), "terms");
  HIPCHK(hipMemcpyAsync(d_start, start.data(), start.size() * 8, hipMemcpyHostToDevice, st), "terms");
  HIPCHK(hipMemcpyAsync(d_first, first.data(), first.size() * 8, hipMemcpyHostToDevice, st), "terms");
  HIPCHK(launch_profiles(d_terms, nt_all, g.ny, g.nx, g.ly, g.lx, 1, d_prof, d_dprof, st), "profiles");
  HIPCHK(launch_grad_terms(d_terms, d_prof, d_dprof, d_start, nt_all, (int)most, g.nz, g.ny, g.nx, dL_dV,
                           d_part, d_out, st),
         "potential gradient");
  HIPCHK(launch_atom_grad_sum(d_out, d_first, n_atoms, n_terms, dL_dxyz, st), "potential gradient");
  return BIP_OK;
}

}  // extern "C"
