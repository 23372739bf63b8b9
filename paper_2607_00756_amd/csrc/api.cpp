// C ABI of the BiP-PRISM hot path: validation, plan geometry, and the
// stream-ordered orchestration of the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "bip_internal.h"
#include "host_common.h"
#include "recon_core.h"

namespace bip {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return BIP_EHIP;
}

namespace {

constexpr double kH = 6.62607015e-34, kE = 1.602176634e-19, kC = 299792458.0,
                 kM = 9.1093837015e-31, kPi = 3.14159265358979323846;

// relativistic wavelength (A) and interaction constant (rad / (V A))
double wavelength(double ev) {
  const double e = kE * ev, mc2 = kM * kC * kC;
  return kH / std::sqrt(2.0 * kM * e * (1.0 + e / (2.0 * mc2))) * 1e10;
}
double interaction(double ev) {
  const double mc2 = kM * kC * kC / kE;
  return 2.0 * kPi / (wavelength(ev) * ev) * (mc2 + ev) / (2.0 * mc2 + ev);
}

bool pow2_in_range(int n) { return n >= 64 && n <= 1024 && (n & (n - 1)) == 0; }
// Fold recorded event pairs into the per-stage totals (synchronizes them).
int collect_timings(bip_plan* p) {
  for (auto& t : p->timed) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(t.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.a, t.b);
    if (e != hipSuccess) return hip_fail(e, "stage timing");
    p->stage_ms[t.stage] += ms;
    p->stage_launches[t.stage] += 1;
    p->event_pool.push_back(t.a);
    p->event_pool.push_back(t.b);
  }
  p->timed.clear();
  return BIP_OK;
}

// beams h (sorted by (h_y, h_x)) with (h_y/L_y)^2 + (h_x/L_x)^2 <= qmax^2
std::vector<int32_t> beams_within(int ny, int nx, double ly, double lx, double qmax) {
  std::vector<int32_t> out;
  for (int hy = -ny / 2; hy < ny / 2; ++hy)
    for (int hx = -nx / 2; hx < nx / 2; ++hx) {
      const double qy = hy / ly, qx = hx / lx;
      if (qy * qy + qx * qx <= qmax * qmax) {
        out.push_back(hy);
        out.push_back(hx);
      }
    }
  return out;
}

// Run the FP64 Sibson kernel on `query` and build the parent set + CSR.
// Crop mask of one axis (PRISM interpolation factor f): the raster indices u
// in [0, S) whose minimum-image displacement t - u N / S (pixels) lies in
// [-N/(2f), N/(2f)), as the cyclic run [start, start + count) mod S (an
// interval of the circle); f = 1 keeps the whole raster.
void crop_run(double t, int N, int S, int f, int32_t& start, int32_t& count) {
  start = 0;
  count = S;
  if (f <= 1) return;
  std::vector<char> in(S);
  int n = 0;
  for (int u = 0; u < S; ++u) {
    double d = t - (double)u * N / S + N / 2.0;
    d = d - N * std::floor(d / N) - N / 2.0;
    in[u] = d >= -N / (2.0 * f) && d < N / (2.0 * f);
    n += in[u];
  }
  count = n;
  if (n == 0 || n == S) return;
  for (int u = 0; u < S; ++u)
    if (in[u] && !in[(u + S - 1) % S]) {
      start = u;
      break;
    }
}

// Lattice partition of `query` (pairs): parents on the (s f)-lattice, weights
// of the Sibson kernel evaluated on query / f (all query beams are multiples
// of f; the weights do not change under the scaling).
int partition(bip_plan* p, const std::vector<int32_t>& query_h, int s, int f, std::vector<int32_t>& parents,
              std::vector<int32_t>& rowptr, std::vector<int32_t>& col, std::vector<double>& w,
              hipStream_t st) {
  std::vector<int32_t> query(query_h.size());
  for (size_t i = 0; i < query.size(); ++i) query[i] = query_h[i] / f;
  const int nq = (int)query.size() / 2;
  int2* dq = nullptr;
  int2* dslot = nullptr;
  double* dw = nullptr;
  void* tmp[3] = {nullptr, nullptr, nullptr};
  const size_t tb[3] = {std::max<size_t>(4, query.size() * sizeof(int32_t)),
                        std::max<size_t>(4, (size_t)nq * 16 * sizeof(int2)),
                        std::max<size_t>(4, (size_t)nq * 16 * sizeof(double))};
  for (int i = 0; i < 3; ++i) {
    tmp[i] = raw_alloc(plan_alloc(p), tb[i], st);
    if (!tmp[i]) {
      for (int k = 0; k < i; ++k) raw_release(plan_alloc(p), tmp[k], tb[k], st);
      return err(BIP_ENOMEM, "Sibson temporaries");
    }
  }
  dq = (int2*)tmp[0];
  dslot = (int2*)tmp[1];
  dw = (double*)tmp[2];
  std::vector<int2> slot((size_t)nq * 16);
  std::vector<double> sw((size_t)nq * 16);
  hipError_t e = hipMemcpyAsync(dq, query.data(), query.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_sibson(dq, nq, s, dslot, dw, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(slot.data(), dslot, slot.size() * sizeof(int2), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sw.data(), dw, sw.size() * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  for (int i = 0; i < 3; ++i) raw_release(plan_alloc(p), tmp[i], tb[i], st);
  if (e != hipSuccess) return hip_fail(e, "sibson weights");
  const double eps = 1e-12;
  std::map<std::pair<int, int>, int> index;
  for (size_t i = 0; i < slot.size(); ++i)
    if (sw[i] > eps) index[{slot[i].x, slot[i].y}] = 0;
  parents.clear();
  int k = 0;
  for (auto& kv : index) {
    kv.second = k++;
    parents.push_back(kv.first.first * f);
    parents.push_back(kv.first.second * f);
  }
  rowptr.assign(nq + 1, 0);
  col.clear();
  w.clear();
  for (int q = 0; q < nq; ++q) {
    // order the nonzeros of a row by parent index
    std::vector<std::pair<int, double>> row;
    for (int j = 0; j < 16; ++j) {
      const size_t i = (size_t)q * 16 + j;
      if (sw[i] > eps) row.push_back({index[{slot[i].x, slot[i].y}], sw[i]});
    }
    std::sort(row.begin(), row.end());
    for (auto& rw : row) {
      col.push_back(rw.first);
      w.push_back(rw.second);
    }
    rowptr[q + 1] = (int32_t)col.size();
  }
  return BIP_OK;
}

// Hex-ring parents of a beam set (pairs, sorted by (h_y, h_x)): the DC beam
// and n_radial rings, ring i (0-based) with n_angular (1 + i) samples at
// radius (i + 1) / n_radial of the disc (radius_y, radius_x in beam-index
// units), each snapped to the nearest beam of the set (ties: the smaller
// (h_y, h_x)), duplicates dropped.
std::vector<int32_t> hex_ring_parents(const std::vector<int32_t>& beams, int n_radial, int n_angular,
                                      double radius_y, double radius_x) {
  const int nb = (int)beams.size() / 2;
  std::vector<std::pair<int, int>> chosen;
  auto snap = [&](double py, double px) {
    double best = 1e300;
    int bk = 0;
    for (int b = 0; b < nb; ++b) {
      const double dy = beams[2 * b] - py, dx = beams[2 * b + 1] - px, d = dy * dy + dx * dx;
      if (d < best) {  // beams are sorted, so the first of equal distances is the smaller
        best = d;
        bk = b;
      }
    }
    chosen.push_back({beams[2 * bk], beams[2 * bk + 1]});
  };
  snap(0.0, 0.0);
  for (int i = 0; i < n_radial; ++i) {
    const double frac = (double)(i + 1) / n_radial;
    const int m = n_angular * (1 + i);
    for (int k = 0; k < m; ++k) {
      const double t = 2.0 * kPi * k / m;
      snap(frac * radius_y * std::sin(t), frac * radius_x * std::cos(t));
    }
  }
  std::sort(chosen.begin(), chosen.end());
  chosen.erase(std::unique(chosen.begin(), chosen.end()), chosen.end());
  std::vector<int32_t> out;
  for (auto& c : chosen) {
    out.push_back(c.first);
    out.push_back(c.second);
  }
  return out;
}

// Convex hull (counter-clockwise, no collinear vertices) of integer points.
std::vector<double2> convex_hull(const std::vector<int32_t>& pts) {
  std::vector<std::pair<long long, long long>> v;
  for (size_t i = 0; i < pts.size(); i += 2) v.push_back({pts[i], pts[i + 1]});
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
  if (v.size() < 3) {
    std::vector<double2> h;
    for (auto& q : v) h.push_back(make_double2((double)q.first, (double)q.second));
    return h;
  }
  auto cross = [](std::pair<long long, long long> o, std::pair<long long, long long> a,
                  std::pair<long long, long long> b) {
    return (a.first - o.first) * (b.second - o.second) - (a.second - o.second) * (b.first - o.first);
  };
  std::vector<std::pair<long long, long long>> lo, up;
  for (auto& q : v) {
    while (lo.size() >= 2 && cross(lo[lo.size() - 2], lo.back(), q) <= 0) lo.pop_back();
    lo.push_back(q);
  }
  for (auto it = v.rbegin(); it != v.rend(); ++it) {
    while (up.size() >= 2 && cross(up[up.size() - 2], up.back(), *it) <= 0) up.pop_back();
    up.push_back(*it);
  }
  lo.pop_back();
  up.pop_back();
  std::vector<double2> h;
  for (auto& q : lo) h.push_back(make_double2((double)q.first, (double)q.second));
  for (auto& q : up) h.push_back(make_double2((double)q.first, (double)q.second));
  return h;
}

// Weights of `query` against the given finite parent set (FP64 kernel) and
// their CSR, parent indices in the order of `parents`.
int partition_general(bip_plan* p, const std::vector<int32_t>& query, const std::vector<int32_t>& parents,
                      std::vector<int32_t>& rowptr, std::vector<int32_t>& col, std::vector<double>& w,
                      hipStream_t st) {
  const int nq = (int)query.size() / 2, np = (int)parents.size() / 2;
  const std::vector<double2> hull = convex_hull(parents);
  void* tmp[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  const size_t tb[5] = {std::max<size_t>(8, query.size() * 4), std::max<size_t>(8, parents.size() * 4),
                        std::max<size_t>(16, hull.size() * sizeof(double2)),
                        std::max<size_t>(8, (size_t)nq * 16 * sizeof(int2)),
                        std::max<size_t>(8, (size_t)nq * 16 * sizeof(double) + 16)};
  for (int i = 0; i < 5; ++i) {
    tmp[i] = raw_alloc(plan_alloc(p), tb[i], st);
    if (!tmp[i]) {
      for (int k = 0; k < i; ++k) raw_release(plan_alloc(p), tmp[k], tb[k], st);
      return err(BIP_ENOMEM, "Sibson temporaries");
    }
  }
  int* d_over = (int*)((char*)tmp[4] + (size_t)nq * 16 * sizeof(double));
  std::vector<int2> slot((size_t)nq * 16);
  std::vector<double> sw((size_t)nq * 16);
  int over = 0;
  hipError_t e = hipMemcpyAsync(tmp[0], query.data(), query.size() * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(tmp[1], parents.data(), parents.size() * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !hull.empty())
    e = hipMemcpyAsync(tmp[2], hull.data(), hull.size() * sizeof(double2), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(d_over, 0, sizeof(int), st);
  if (e == hipSuccess)
    e = launch_sibson_general((const int2*)tmp[0], nq, (const int2*)tmp[1], np, (const double2*)tmp[2],
                              (int)hull.size(), (int2*)tmp[3], (double*)tmp[4], d_over, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(slot.data(), tmp[3], slot.size() * sizeof(int2), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(sw.data(), tmp[4], sw.size() * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&over, d_over, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  for (int i = 0; i < 5; ++i) raw_release(plan_alloc(p), tmp[i], tb[i], st);
  if (e != hipSuccess) return hip_fail(e, "sibson weights");
  if (over) return err(BIP_EUNSUPPORTED, "a beam has more than 16 natural-neighbour parents");
  std::map<std::pair<int, int>, int> index;
  for (int i = 0; i < np; ++i) index[{parents[2 * i], parents[2 * i + 1]}] = i;
  rowptr.assign(nq + 1, 0);
  col.clear();
  w.clear();
  for (int q = 0; q < nq; ++q) {
    std::vector<std::pair<int, double>> row;
    for (int j = 0; j < 16; ++j) {
      const size_t i = (size_t)q * 16 + j;
      if (sw[i] > 1e-12) {
        auto it = index.find({slot[i].x, slot[i].y});
        if (it == index.end()) return err(BIP_EHIP, "internal: Sibson slot outside the parent set");
        row.push_back({it->second, sw[i]});
      }
    }
    std::sort(row.begin(), row.end());
    for (auto& rw : row) {
      col.push_back(rw.first);
      w.push_back(rw.second);
    }
    rowptr[q + 1] = (int32_t)col.size();
  }
  return BIP_OK;
}

}  // namespace
}  // namespace bip

using namespace bip;

extern "C" {

const char* bip_last_error(void) { return g_err.c_str(); }

void bip_plan_destroy(bip_plan* p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  for (auto& b : p->allocations) raw_release(plan_alloc(p), b.ptr, b.bytes, p->stream);
  p->allocations.clear();
  for (auto& t : p->timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
  (void)hipStreamSynchronize(p->stream);  // stream-ordered releases complete before return
  delete p;
}

int bip_plan_create(const bip_grid* grid, const bip_optics* optics, int32_t n_atoms,
                    const double* tau_xyz, const int32_t* win_size, const int32_t* win_origin,
                    const bip_alloc* alloc, void* stream, bip_plan** out) {
  if (!out) return err(BIP_EINVAL, "out is NULL");
  *out = nullptr;
  if (!grid || !optics || !tau_xyz || !win_size || !win_origin)
    return err(BIP_EINVAL, "NULL argument");
  const bip_grid g = *grid;
  const bip_optics o = *optics;
  if (!pow2_in_range(g.ny) || !pow2_in_range(g.nx))
    return err(BIP_EINVAL, "ny and nx must be powers of two in [64, 1024]");
  if (g.nz < 1) return err(BIP_EINVAL, "nz must be >= 1");
  if (!(g.ly > 0) || !(g.lx > 0) || !(g.dz > 0)) return err(BIP_EINVAL, "ly, lx, dz must be > 0");
  if (!(o.energy_ev > 0) || !(o.alpha_rad > 0) || !(o.theta_rad > 0))
    return err(BIP_EINVAL, "energy, alpha and theta must be > 0");
  if (o.partition < 1) return err(BIP_EINVAL, "partition must be >= 1");
  if (o.parent_set != BIP_PARENTS_LATTICE && o.parent_set != BIP_PARENTS_HEX)
    return err(BIP_EINVAL, "unknown parent_set");
  if (o.parent_set == BIP_PARENTS_HEX && (o.n_radial < 1 || o.n_angular < 1))
    return err(BIP_EINVAL, "hex rings need n_radial >= 1 and n_angular >= 1");
  if (o.focal != 0 && o.focal != 1) return err(BIP_EINVAL, "focal must be 0 or 1");
  if (o.s2_exact != 0 && o.s2_exact != 1) return err(BIP_EINVAL, "s2_exact must be 0 or 1");
  const int fi = o.interp_f == 0 ? 1 : o.interp_f;
  if (fi < 1 || g.ny % fi != 0 || g.nx % fi != 0)
    return err(BIP_EINVAL, "interp_f must be >= 1 and divide ny and nx");
  if (fi > 1 && o.s2_exact)
    return err(BIP_EUNSUPPORTED, "the exact detector matrix (4D cube) keeps every exit beam: interp_f 1 only");
  if (fi > 1 && o.ckpt_stride != 0)
    return err(BIP_EUNSUPPORTED, "interp_f > 1 is forward only (ckpt_stride must be 0)");
  if (o.focal && o.ckpt_stride != 0)
    return err(BIP_EUNSUPPORTED, "focal back-propagation is forward only (ckpt_stride must be 0)");
  if (o.recon_mode != BIP_RECON_MAGNITUDE && o.recon_mode != BIP_RECON_COMPLEX)
    return err(BIP_EINVAL, "unknown recon_mode");
  if (o.ckpt_stride < 0) return err(BIP_EINVAL, "ckpt_stride must be >= 0");
  if (alloc && (!alloc->alloc || !alloc->release))
    return err(BIP_EINVAL, "bip_alloc needs both alloc and release");
  if (n_atoms < 1) return err(BIP_EINVAL, "n_atoms must be >= 1");
  for (int a = 0; a < n_atoms; ++a) {
    const int W = win_size[a];
    if (W < 4 || W > std::min(g.ny, g.nx) || W % 4 != 0)
      return err(BIP_EINVAL, "window size of atom " + std::to_string(a) +
                                 " must be a multiple of 4 in [4, min(ny, nx)]");
    if (o.focal && (W > 64 || 2 * W > std::min(g.ny, g.nx)))
      return err(BIP_EUNSUPPORTED, "focal back-propagation needs W <= 64 and 2W <= min(ny, nx)");
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(tau_xyz[3 * a + k]))
        return err(BIP_EINVAL, "non-finite atom position");
  }
  hipStream_t st = (hipStream_t)stream;
  bip_plan* p = new bip_plan();
  p->g = g;
  p->o = o;
  p->stream = st;
  if (alloc) {
    p->alloc = *alloc;
    p->has_alloc = true;
  }
  p->lambda = wavelength(o.energy_ev);
  p->sigma = interaction(o.energy_ev);
  p->L = std::max(g.ny, g.nx);
  p->beams = beams_within(g.ny, g.nx, g.ly, g.lx, o.alpha_rad / p->lambda);
  p->det = beams_within(g.ny, g.nx, g.ly, g.lx, o.theta_rad / p->lambda);
  p->f = fi;
  p->B_full = (int)p->beams.size() / 2;
  if (fi > 1) {  // Alg. 2 subsampling of the aperture, and of the detector (Alg. 4)
    for (auto* set : {&p->beams, &p->det}) {
      std::vector<int32_t> kept;
      for (size_t i = 0; i < set->size(); i += 2)
        if ((*set)[i] % fi == 0 && (*set)[i + 1] % fi == 0) {
          kept.push_back((*set)[i]);
          kept.push_back((*set)[i + 1]);
        }
      set->swap(kept);
    }
  }
  p->B = (int)p->beams.size() / 2;
  p->ndet = (int)p->det.size() / 2;
  const double rq = o.theta_rad / p->lambda * g.lx;
  p->nq_half = (int)std::floor(rq + 1e-12);
  p->nq = 2 * p->nq_half + 1;
  int rc = BIP_OK;
  auto fail = [&](int code) {
    bip_plan_destroy(p);
    return code;
  };
  {
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n_cu > 0)
      p->n_cu = n_cu;
  }
  if (p->B < 1 || p->ndet < 1) return fail(err(BIP_EINVAL, "empty aperture or detector"));
  if (o.parent_set == BIP_PARENTS_HEX) {
    p->par1 = hex_ring_parents(p->beams, o.n_radial, o.n_angular, o.alpha_rad / p->lambda * g.ly,
                               o.alpha_rad / p->lambda * g.lx);
    p->par2 = hex_ring_parents(p->det, o.n_radial, o.n_angular, o.theta_rad / p->lambda * g.ly,
                               o.theta_rad / p->lambda * g.lx);
    if ((rc = partition_general(p, p->beams, p->par1, p->rp1, p->col1, p->w1, st))) return fail(rc);
    if ((rc = partition_general(p, p->det, p->par2, p->rp2, p->col2, p->w2, st))) return fail(rc);
  } else {
    if ((rc = partition(p, p->beams, o.partition, fi, p->par1, p->rp1, p->col1, p->w1, st))) return fail(rc);
    if ((rc = partition(p, p->det, o.partition, fi, p->par2, p->rp2, p->col2, p->w2, st))) return fail(rc);
  }
  if (o.s2_exact) {  // every detector beam its own parent: identity weights
    if ((rc = partition(p, p->det, 1, 1, p->par2, p->rp2, p->col2, p->w2, st))) return fail(rc);
  }
  p->Bp1 = (int)p->par1.size() / 2;
  p->Bp2 = (int)p->par2.size() / 2;
  // a parent past the signed index range would alias to another frequency of
  // the grid (its plane wave and propagator phase would be the alias's)
  for (const auto* par : {&p->par1, &p->par2})
    for (size_t i = 0; i < par->size(); i += 2)
      if ((*par)[i] < -g.ny / 2 || (*par)[i] >= g.ny / 2 || (*par)[i + 1] < -g.nx / 2 ||
          (*par)[i + 1] >= g.nx / 2)
        return fail(err(BIP_EUNSUPPORTED, "parent beam (" + std::to_string((*par)[i]) + ", " +
                                              std::to_string((*par)[i + 1]) +
                                              ") outside the grid's frequency range; use a "
                                              "smaller aperture/detector or partition factor"));
  // atoms
  p->n_atoms = n_atoms;
  p->W.resize(n_atoms);
  p->oy.resize(n_atoms);
  p->ox.resize(n_atoms);
  p->plane.resize(n_atoms);
  p->off1.resize(n_atoms);
  p->off2.resize(n_atoms);
  int64_t o1 = 0, o2 = 0;
  p->focal = o.focal != 0;
  p->W1.resize(n_atoms);
  p->oy1.resize(n_atoms);
  p->ox1.resize(n_atoms);
  p->tau_y.resize(n_atoms);
  p->tau_x.resize(n_atoms);
  for (int a = 0; a < n_atoms; ++a) {
    const int W = win_size[a];
    p->W[a] = W;
    p->tau_y[a] = tau_xyz[3 * a + 1] * g.ny / g.ly;
    p->tau_x[a] = tau_xyz[3 * a] * g.nx / g.lx;
    p->oy[a] = ((win_origin[2 * a] % g.ny) + g.ny) % g.ny;
    p->ox[a] = ((win_origin[2 * a + 1] % g.nx) + g.nx) % g.nx;
    // S1 window: the enlarged M x M one (M the smallest power of two >= 2W),
    // centred on the atom's window, when S1 is focally back-propagated
    int M = W;
    if (p->focal) {
      M = 8;
      while (M < 2 * W) M *= 2;
    }
    const int pad = (M - W) / 2;
    p->W1[a] = M;
    p->oy1[a] = ((p->oy[a] - pad) % g.ny + g.ny) % g.ny;
    p->ox1[a] = ((p->ox[a] - pad) % g.nx + g.nx) % g.nx;
    p->focal_max_m = std::max(p->focal_max_m, M);
    const int pl = (int)std::floor(tau_xyz[3 * a + 2] / g.dz);
    p->plane[a] = std::min(std::max(pl, 0), g.nz - 1);
    p->off1[a] = o1;
    p->off2[a] = o2;
    o1 += (int64_t)p->Bp1 * M * M;
    o2 += (int64_t)p->Bp2 * W * W;
  }
  p->win1_elems = o1;
  p->win2_elems = o2;
  p->seg_of.assign(n_atoms, 0);
  p->plane_start.assign(g.nz + 1, 0);
  for (int a = 0; a < n_atoms; ++a) p->plane_start[p->plane[a] + 1]++;
  for (int j = 0; j < g.nz; ++j) p->plane_start[j + 1] += p->plane_start[j];
  p->plane_atoms.assign(n_atoms, 0);
  {
    std::vector<int32_t> fill(p->plane_start.begin(), p->plane_start.end() - 1);
    for (int a = 0; a < n_atoms; ++a) p->plane_atoms[fill[p->plane[a]]++] = a;
  }
  p->i_min = *std::min_element(p->plane.begin(), p->plane.end());
  p->i_max = *std::max_element(p->plane.begin(), p->plane.end());
  {
    // S2 windows of all atoms above the budget: plane segments (from the exit
    // down) whose windows fit it, one segment's block reused for the next
    const double gb = o.s2_window_gb > 0 ? o.s2_window_gb : 48.0;
    const int64_t budget = (int64_t)(gb * (double)(1ll << 30)) / 8;  // complex64 elements
    if (p->win2_elems > budget) {
      if (o.ckpt_stride != 0)
        return fail(err(BIP_EUNSUPPORTED, "the S2 windows exceed s2_window_gb: streamed S2 has no "
                                          "checkpoints for bip_eels_backward"));
      p->s2_stream = true;
      int64_t cur = 0, most = 0;
      int hi = -1, lo = -1;
      auto close = [&] {
        p->seg_hi.push_back(hi);
        p->seg_lo.push_back(lo);
        most = std::max(most, cur);
        cur = 0;
        hi = -1;
      };
      for (int j = g.nz - 1; j >= 0; --j) {
        int64_t pj = 0;
        for (int q = p->plane_start[j]; q < p->plane_start[j + 1]; ++q)
          pj += (int64_t)p->Bp2 * p->W[p->plane_atoms[q]] * p->W[p->plane_atoms[q]];
        if (pj == 0) continue;
        if (hi >= 0 && cur + pj > budget) close();
        if (hi < 0) hi = j;
        lo = j;
        for (int q = p->plane_start[j]; q < p->plane_start[j + 1]; ++q) {
          const int a = p->plane_atoms[q];
          p->seg_of[a] = (int)p->seg_hi.size();
          p->off2[a] = cur;
          cur += (int64_t)p->Bp2 * p->W[a] * p->W[a];
        }
      }
      close();
      p->win2_elems = most;
    }
  }
  // device buffers
  const int64_t G = (int64_t)g.ny * g.nx;
  auto as_int2 = [](const std::vector<int32_t>& v) {
    std::vector<int2> r(v.size() / 2);
    for (size_t i = 0; i < r.size(); ++i) r[i] = make_int2(v[2 * i], v[2 * i + 1]);
    return r;
  };
  std::vector<float> w1f(p->w1.begin(), p->w1.end()), w2f(p->w2.begin(), p->w2.end());
  std::vector<GatherRec> grec1(n_atoms), grec2(n_atoms);
  for (int q = 0; q < n_atoms; ++q) {
    const int a = p->plane_atoms[q];
    grec1[q] = GatherRec{p->W1[a], p->oy1[a], p->ox1[a], 0, p->off1[a]};
    grec2[q] = GatherRec{p->W[a], p->oy[a], p->ox[a], 0, p->off2[a]};
  }
  // padded copies of the CSR rows: six (parent, weight) slots, row length, row start
  auto ell = [](const std::vector<int32_t>& rp, const std::vector<int32_t>& cl,
                const std::vector<double>& w, std::vector<int32_t>& ec, std::vector<float>& ew) {
    const int nb = (int)rp.size() - 1;
    ec.assign((size_t)nb * ELL_W, 0);
    ew.assign((size_t)nb * ELL_W, 0.f);
    for (int b = 0; b < nb; ++b) {
      const int lo = rp[b], n = rp[b + 1] - lo;
      for (int j = 0; j < std::min(n, ELL_K); ++j) {
        ec[(size_t)b * ELL_W + j] = cl[lo + j];
        ew[(size_t)b * ELL_W + j] = (float)w[lo + j];
      }
      ec[(size_t)b * ELL_W + 6] = n;
      ec[(size_t)b * ELL_W + 7] = lo;
    }
  };
  std::vector<int32_t> ec1, ec2;
  std::vector<float> ew1, ew2;
  ell(p->rp1, p->col1, p->w1, ec1, ew1);
  ell(p->rp2, p->col2, p->w2, ec2, ew2);
  // per tile of TILE_B consecutive beams: its distinct parents, and each
  // beam's padded slots as indices into that list
  auto tiles = [](const std::vector<int32_t>& rp, const std::vector<int32_t>& ec,
                  std::vector<int32_t>& ts, std::vector<int32_t>& tp, std::vector<int32_t>& el) {
    const int nb = (int)rp.size() - 1;
    const int nt = (nb + TILE_B - 1) / TILE_B;
    ts.assign(nt + 1, 0);
    tp.clear();
    el.assign((size_t)nb * ELL_W, 0);
    for (int t = 0; t < nt; ++t) {
      std::vector<int32_t> ps;
      for (int b = t * TILE_B; b < std::min(nb, (t + 1) * TILE_B); ++b)
        for (int j = 0; j < std::min(ELL_K, rp[b + 1] - rp[b]); ++j) ps.push_back(ec[(size_t)b * ELL_W + j]);
      std::sort(ps.begin(), ps.end());
      ps.erase(std::unique(ps.begin(), ps.end()), ps.end());
      for (int b = t * TILE_B; b < std::min(nb, (t + 1) * TILE_B); ++b)
        for (int j = 0; j < ELL_K; ++j) {
          const int32_t q = ec[(size_t)b * ELL_W + j];
          const auto it = std::lower_bound(ps.begin(), ps.end(), q);
          el[(size_t)b * ELL_W + j] = (it != ps.end() && *it == q) ? (int32_t)(it - ps.begin()) : 0;
        }
      tp.insert(tp.end(), ps.begin(), ps.end());
      ts[t + 1] = (int32_t)tp.size();
    }
  };
  std::vector<int32_t> ts1, tp1, el1, ts2, tp2, el2;
  tiles(p->rp1, ec1, ts1, tp1, el1);
  tiles(p->rp2, ec2, ts2, tp2, el2);
  for (size_t t = 0; t + 1 < ts1.size(); ++t) p->tile_np1 = std::max(p->tile_np1, ts1[t + 1] - ts1[t]);
  for (size_t t = 0; t + 1 < ts2.size(); ++t) p->tile_np2 = std::max(p->tile_np2, ts2[t + 1] - ts2[t]);
  // host sources of the uploads live until the stream synchronization below
  const std::vector<int2> beams2 = as_int2(p->beams), det2 = as_int2(p->det),
                          par12 = as_int2(p->par1), par22 = as_int2(p->par2);
  if ((rc = dalloc(p, &p->d_tw, p->L, st)) || (rc = dalloc(p, &p->d_prop, G, st)) ||
      (rc = dalloc(p, &p->d_T, G * g.nz, st)) || (rc = upload(p, &p->d_beams, beams2, st)) ||
      (rc = upload(p, &p->d_det, det2, st)) ||
      (rc = upload(p, &p->d_par1, par12, st)) ||
      (rc = upload(p, &p->d_par2, par22, st)) ||
      (rc = upload(p, &p->d_rp1, p->rp1, st)) || (rc = upload(p, &p->d_col1, p->col1, st)) ||
      (rc = upload(p, &p->d_w1, w1f, st)) || (rc = upload(p, &p->d_rp2, p->rp2, st)) ||
      (rc = upload(p, &p->d_col2, p->col2, st)) || (rc = upload(p, &p->d_w2, w2f, st)) ||
      (rc = upload(p, &p->d_ellc1, ec1, st)) || (rc = upload(p, &p->d_ellw1, ew1, st)) ||
      (rc = upload(p, &p->d_ellc2, ec2, st)) || (rc = upload(p, &p->d_ellw2, ew2, st)) ||
      (rc = upload(p, &p->d_tstart1, ts1, st)) || (rc = upload(p, &p->d_tpar1, tp1, st)) ||
      (rc = upload(p, &p->d_eloc1, el1, st)) || (rc = upload(p, &p->d_tstart2, ts2, st)) ||
      (rc = upload(p, &p->d_tpar2, tp2, st)) || (rc = upload(p, &p->d_eloc2, el2, st)) ||
      (rc = upload(p, &p->d_W, p->W, st)) || (rc = upload(p, &p->d_oy, p->oy, st)) ||
      (rc = upload(p, &p->d_ox, p->ox, st)) || (rc = upload(p, &p->d_off1, p->off1, st)) ||
      (rc = upload(p, &p->d_off2, p->off2, st)) ||
      (rc = upload(p, &p->d_grec1, grec1, st)) || (rc = upload(p, &p->d_grec2, grec2, st)) ||
      (rc = dalloc(p, &p->d_state1, (size_t)p->Bp1 * G, st)) ||
      (rc = dalloc(p, &p->d_state2, (size_t)p->Bp2 * G, st)) ||
      (rc = dalloc(p, &p->d_win1, (size_t)p->win1_elems, st)) ||
      (rc = dalloc(p, &p->d_win2, (size_t)p->win2_elems, st)))
    return fail(rc);
  std::vector<FocalAtom> fatoms;
  if (p->focal) {
    for (int a = 0; a < n_atoms; ++a)
      fatoms.push_back(FocalAtom{p->off1[a], p->W1[a], p->W[a], p->oy1[a], p->ox1[a], p->plane[a], a});
    if ((rc = upload(p, &p->d_fatoms, fatoms, st)) || (rc = dalloc(p, &p->d_fdist, (size_t)n_atoms, st)))
      return fail(rc);
  }
  if (o.ckpt_stride >= 1) {
    // one checkpoint per segment of ckpt_stride slices: S1 slices 0 .. i_max-1
    // in segments [mK, mK + K), S2 slices nz-1 .. i_min in segments from the exit
    const int K = o.ckpt_stride;
    const size_t n1 = (size_t)((p->i_max + K - 1) / K) * p->Bp1 * G,
                 n2 = (size_t)((g.nz - p->i_min + K - 1) / K) * p->Bp2 * G;
    if ((rc = dalloc(p, &p->d_prop_conj, G, st)) || (n1 && (rc = dalloc(p, &p->d_ckpt1, n1, st))) ||
        (rc = dalloc(p, &p->d_ckpt2, n2, st)) || (rc = dalloc(p, &p->d_gwin1, (size_t)p->win1_elems, st)) ||
        (rc = dalloc(p, &p->d_gwin2, (size_t)p->win2_elems, st)))
      return fail(rc);
  }
  hipError_t e = launch_twiddles(p->d_tw, p->L, st);
  if (e == hipSuccess)
    e = launch_prop_table(p->d_prop, g.ny, g.nx, g.ly, g.lx, p->lambda, g.dz, 0, st);
  if (e == hipSuccess && p->d_prop_conj)
    e = launch_prop_table(p->d_prop_conj, g.ny, g.nx, g.ly, g.lx, p->lambda, g.dz, 1, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(hip_fail(e, "plan tables"));
  *out = p;
  return BIP_OK;
}

int bip_build_smatrix(bip_plan* p, const float* V, void* stream) {
  if (!p || !V) return err(BIP_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  p->stream = st;
  const bip_grid& g = p->g;
  const int64_t G = (int64_t)g.ny * g.nx;
  HIPCHK(timed(p, ST_TRANSMIT, st, [&] { return launch_transmit(p->d_T, V, G * g.nz, (float)p->sigma, st); }), "transmit");
  // Columns are advanced in batches, every slice of a batch before the next
  // batch, so that a batch (both passes of every slice) can stay resident in
  // the last-level cache; a batch of all columns is the plain slice-major sweep.
  const int batch = column_batch(G);
  p->column_batch = batch;
  // ---- S1: entrance -> deepest ionization plane
  HIPCHK(timed(p, ST_INIT, st, [&] { return launch_init_planewaves(p->d_state1, p->d_par1, p->Bp1, g.ny, g.nx, p->d_tw, p->L, +1, 1.0f, st); }),
         "init S1");
  GatherArgs g1 = gather_args(p, 1);
  const int batch1 = balanced_batch(p->Bp1, batch);
  for (int c0 = 0; c0 < p->Bp1; c0 += batch1) {
    const int nc = std::min(batch1, p->Bp1 - c0);
    float2* s1 = p->d_state1 + (int64_t)c0 * G;
    for (int j = 0; j <= p->i_max; ++j) {
      int flags = ROW_GATHER_BEFORE_T;
      if (j > 0) flags |= ROW_INV;
      if (j < p->i_max) flags |= ROW_T | ROW_FWD;
      float2* save = nullptr;
      if (p->d_ckpt1 && j < p->i_max && j % p->o.ckpt_stride == 0) {
        flags |= ROW_SAVE;
        save = p->d_ckpt1 + ((int64_t)(j / p->o.ckpt_stride) * p->Bp1 + c0) * G;
      }
      HIPCHK(timed(p, ST_S1_ROW, st, [&] { return launch_row_pass(flags, s1, nc, g.ny, g.nx, p->d_T + j * G, p->d_tw, p->L,
                             p->d_par1, +1, g1, p->plane_start[j], p->plane_start[j + 1], c0, save, st); }),
             "S1 row pass");
      if (j < p->i_max)
        HIPCHK(timed(p, ST_S1_COL, st, [&] { return launch_col_pass(s1, nc, g.ny, g.nx, p->d_prop, p->d_tw, p->L, st); }),
               "S1 column pass");
    }
  }
  // ---- focal back-propagation of the S1 windows to each atom's centroid plane
  if (p->focal) {
    HIPCHK(launch_focal_dist(V, p->d_fatoms, p->n_atoms, g.ny, g.nx, g.dz, p->d_fdist, st), "focal distance");
    HIPCHK(launch_focal_parents(p->d_win1, p->d_fatoms, p->n_atoms, p->d_fdist, p->d_par1, p->Bp1,
                                p->focal_max_m, g.ny, g.nx, g.ly / g.ny, g.lx / g.nx, p->lambda, p->d_tw, p->L,
                                st),
           "focal back-step");
  }
  // ---- S2: exit -> shallowest ionization plane (transpose multislice);
  // streamed plans sweep S2 inside bip_eels_signal, segment by segment
  if (!p->s2_stream) {
    int rc = sweep_s2(p, g.nz - 1, p->i_min, true, st);
    if (rc) return rc;
  }
  p->built = true;
  return BIP_OK;
}

}  // extern "C"

int bip::sweep_s2(bip_plan* p, int j_hi, int j_lo, bool init, hipStream_t st) {
  const bip_grid& g = p->g;
  const int64_t G = (int64_t)g.ny * g.nx;
  const int batch = column_batch(G);
  p->column_batch = batch;
  const int batch2 = balanced_batch(p->Bp2, batch);
  // The parents start row-transformed, the form the state keeps between passes.
  if (init)
    HIPCHK(timed(p, ST_INIT, st, [&] { return launch_init_planewaves_rowft(p->d_state2, p->d_par2, p->Bp2, g.ny, g.nx, p->d_tw,
                                  p->L, (float)(1.0 / std::sqrt((double)G)), st); }),
           "init S2");
  GatherArgs g2 = gather_args(p, 2);
  for (int c0 = 0; c0 < p->Bp2; c0 += batch2) {
    const int nc = std::min(batch2, p->Bp2 - c0);
    float2* s2 = p->d_state2 + (int64_t)c0 * G;
    for (int j = j_hi; j >= j_lo; --j) {
      HIPCHK(timed(p, ST_S2_COL, st, [&] { return launch_col_pass(s2, nc, g.ny, g.nx, p->d_prop, p->d_tw, p->L, st); }),
             "S2 column pass");
      int flags = ROW_INV | ROW_T | ROW_GATHER_AFTER_T;
      if (j > p->i_min) flags |= ROW_FWD;  // keep the state row-transformed until the last plane
      float2* save = nullptr;
      if (p->d_ckpt2 && (g.nz - 1 - j) % p->o.ckpt_stride == 0) {
        flags |= ROW_SAVE;
        save = p->d_ckpt2 + ((int64_t)((g.nz - 1 - j) / p->o.ckpt_stride) * p->Bp2 + c0) * G;
      }
      HIPCHK(timed(p, ST_S2_ROW, st, [&] { return launch_row_pass(flags, s2, nc, g.ny, g.nx, p->d_T + j * G, p->d_tw, p->L,
                             p->d_par2, -1, g2, p->plane_start[j], p->plane_start[j + 1], c0, save, st); }),
             "S2 row pass");
    }
  }
  return BIP_OK;
}

extern "C" {

int bip_parent_windows(bip_plan* p, int32_t atom, int32_t which, float* out, void* stream) {
  if (!p || !out) return err(BIP_EINVAL, "NULL argument");
  if (atom < 0 || atom >= p->n_atoms) return err(BIP_EINVAL, "atom out of range");
  if (which != 1 && which != 2) return err(BIP_EINVAL, "which must be 1 or 2");
  if (!p->built) return err(BIP_ESTATE, "bip_build_smatrix has not run");
  if (which == 2 && p->s2_stream)
    return err(BIP_EUNSUPPORTED, "S2 windows of this plan are streamed inside bip_eels_signal");
  const int W = which == 1 ? p->W1[atom] : p->W[atom];
  const size_t n = (size_t)(which == 1 ? p->Bp1 : p->Bp2) * W * W;
  const float2* src = which == 1 ? p->d_win1 + p->off1[atom] : p->d_win2 + p->off2[atom];
  HIPCHK(hipMemcpyAsync(out, src, n * sizeof(float2), hipMemcpyDeviceToDevice, (hipStream_t)stream),
         "copy windows");
  return BIP_OK;
}

int bip_reconstruct_local(bip_plan* p, int32_t atom, float* s1_out, float* s2_out, void* stream) {
  if (!p) return err(BIP_EINVAL, "NULL plan");
  if (atom < 0 || atom >= p->n_atoms) return err(BIP_EINVAL, "atom out of range");
  if (!p->built) return err(BIP_ESTATE, "bip_build_smatrix has not run");
  hipStream_t st = (hipStream_t)stream;
  if (s2_out && p->s2_stream)
    return err(BIP_EUNSUPPORTED, "S2 windows of this plan are streamed inside bip_eels_signal");
  if (s1_out && p->focal)
    return err(BIP_EUNSUPPORTED, "focal mode: S1 is reconstructed at the centroid plane only");
  if (s1_out) HIPCHK(launch_recon_plain(recon_args(p, atom, 1), (float2*)s1_out, st), "recon S1");
  if (s2_out) HIPCHK(launch_recon_plain(recon_args(p, atom, 2), (float2*)s2_out, st), "recon S2");
  return BIP_OK;
}

int bip_eels_signal_edges(bip_plan* p, int32_t n_edges, const bip_edge* edges, int32_t scan_sy,
                          int32_t scan_sx, int32_t out_mode, int32_t precision, int32_t accumulate,
                          float weight, void* stream) {
  return bip::signal_edges_impl(p, n_edges, edges, scan_sy, scan_sx, out_mode, precision, accumulate,
                                weight, nullptr, 0, stream);
}

int bip_eels_signal(bip_plan* p, int32_t n_ch, const float* H, const int64_t* H_off,
                    const int32_t* atom_subset, int32_t n_subset, int32_t scan_sy,
                    int32_t scan_sx, int32_t out_mode, int32_t precision, float* out,
                    void* stream) {
  return bip::eels_signal_impl(p, n_ch, H, H_off, atom_subset, n_subset, scan_sy, scan_sx, out_mode,
                               precision, out, nullptr, 0, stream);
}

}  // extern "C"

static int signal_atoms(bip_plan* p, const std::vector<int32_t>& atoms, int32_t n_ch, const float* H,
                        const int64_t* H_off, int32_t scan_sy, int32_t scan_sx, int32_t out_mode,
                        int32_t precision, float* out, void* ext_work, size_t ext_bytes,
                        bool accumulate, hipStream_t st);

// Steps (b) + (c).  With `ext_work` the workspace is that caller-given device
// block of `ext_bytes` (nothing is allocated); else the plan's own workspace,
// grown on demand.
int bip::eels_signal_impl(bip_plan* p, int32_t n_ch, const float* H, const int64_t* H_off,
                          const int32_t* atom_subset, int32_t n_subset, int32_t scan_sy,
                          int32_t scan_sx, int32_t out_mode, int32_t precision, float* out,
                          void* ext_work, size_t ext_bytes, void* stream) {
  bip_edge e{n_ch, H, H_off, atom_subset, n_subset, out};
  return signal_edges_impl(p, 1, &e, scan_sy, scan_sx, out_mode, precision, 0, 1.f, ext_work,
                           ext_bytes, stream);
}

int bip::signal_edges_impl(bip_plan* p, int32_t n_edges, const bip_edge* edges, int32_t scan_sy,
                           int32_t scan_sx, int32_t out_mode, int32_t precision, int32_t accumulate,
                           float weight, void* ext_work, size_t ext_bytes, void* stream) {
  if (!p || !edges || n_edges < 1) return err(BIP_EINVAL, "NULL argument or no edge");
  if (!p->built) return err(BIP_ESTATE, "bip_build_smatrix has not run");
  if (scan_sy < 1 || scan_sx < 1) return err(BIP_EINVAL, "scan raster must be >= 1 x 1");
  if (scan_sy > BIP_MAX_SCAN || scan_sx > BIP_MAX_SCAN)
    return err(BIP_EUNSUPPORTED, "scan raster sides above " + std::to_string(BIP_MAX_SCAN));
  if (out_mode != BIP_OUT_MAP && out_mode != BIP_OUT_QEELS && out_mode != BIP_OUT_BEAMS &&
      out_mode != BIP_OUT_MAP_DIRECT && out_mode != BIP_OUT_CUBE)
    return err(BIP_EINVAL, "unknown out_mode");
  if (out_mode == BIP_OUT_CUBE) {
    if (!p->o.s2_exact)
      return err(BIP_EINVAL, "the 4D cube needs the exact detector matrix (plan with s2_exact = 1)");
    out_mode = BIP_OUT_BEAMS;  // every detector beam of the exact S2: the cube
  }
  if (precision != BIP_PREC_FP32 && precision != BIP_PREC_SPLIT_BF16 && precision != BIP_PREC_BF16 &&
      precision != BIP_PREC_FP16)
    return err(BIP_EINVAL, "unknown precision");
  if (!std::isfinite(weight)) return err(BIP_EINVAL, "weight must be finite");
  const bool weighted = accumulate || weight != 1.f;
  if (weighted && ext_work) return err(BIP_EUNSUPPORTED, "accumulate/weight need a workspace");
  std::vector<std::vector<int32_t>> atoms(n_edges);
  for (int e = 0; e < n_edges; ++e) {
    const bip_edge& E = edges[e];
    if (!E.H || !E.H_off || !E.out) return err(BIP_EINVAL, "NULL argument in edge " + std::to_string(e));
    if (E.n_ch < 1) return err(BIP_EINVAL, "n_ch must be >= 1");
    if (E.atom_subset) {
      if (E.n_subset < 0) return err(BIP_EINVAL, "n_subset < 0");
      for (int i = 0; i < E.n_subset; ++i) {
        if (E.atom_subset[i] < 0 || E.atom_subset[i] >= p->n_atoms)
          return err(BIP_EINVAL, "atom_subset entry out of range");
        atoms[e].push_back(E.atom_subset[i]);
      }
    } else {
      for (int a = 0; a < p->n_atoms; ++a) atoms[e].push_back(a);
    }
    for (int a : atoms[e])  // only the atoms an edge contracts read its H
      if (E.H_off[a + 1] - E.H_off[a] != (int64_t)E.n_ch * p->W[a] * p->W[a] || E.H_off[a] < 0)
        return err(BIP_EINVAL, "H_off inconsistent with n_ch and the window of atom " + std::to_string(a));
  }
  hipStream_t st = (hipStream_t)stream;
  p->stream = st;
  const int P = scan_sy * scan_sx;
  const int64_t n_out = out_mode == BIP_OUT_QEELS ? (int64_t)P * p->nq
                        : out_mode == BIP_OUT_BEAMS ? (int64_t)P * p->ndet : (int64_t)P;
  // weighted / accumulating calls contract into a plan-owned block, then add
  // weight times it into the edge's output
  float* tmp = nullptr;
  if (weighted) {
    if (p->tmp_bytes < (size_t)n_out * 4) {
      if (p->d_tmp) plan_release(p, p->d_tmp, st);
      p->d_tmp = nullptr;
      p->tmp_bytes = 0;
      void* ptr = nullptr;
      int rc = plan_block(p, &ptr, (size_t)n_out * 4, st);
      if (rc) return rc;
      p->d_tmp = (float*)ptr;
      p->tmp_bytes = (size_t)n_out * 4;
    }
    tmp = p->d_tmp;
  }
  std::vector<int> contributions(n_edges, 0);
  // one edge's atoms of a segment (seg < 0: every atom of the edge)
  auto run = [&](int e, const std::vector<int32_t>& list) -> int {
    const bip_edge& E = edges[e];
    if (!weighted) {
      int rc = signal_atoms(p, list, E.n_ch, E.H, E.H_off, scan_sy, scan_sx, out_mode, precision, E.out,
                            ext_work, ext_bytes, contributions[e] > 0, st);
      ++contributions[e];
      return rc;
    }
    int rc = signal_atoms(p, list, E.n_ch, E.H, E.H_off, scan_sy, scan_sx, out_mode, precision, tmp,
                          nullptr, 0, false, st);
    if (rc) return rc;
    HIPCHK(launch_axpy(E.out, tmp, n_out, weight, accumulate || contributions[e] > 0, st), "weighted sum");
    ++contributions[e];
    return BIP_OK;
  };
  if (!p->s2_stream) {
    for (int e = 0; e < n_edges; ++e) {
      int rc = run(e, atoms[e]);
      if (rc) return rc;
    }
    return BIP_OK;
  }
  // S2 streamed: sweep a plane segment, contract its atoms of every edge (in
  // each edge's listed order), then the next segment; the outputs accumulate
  // over the segments
  int last = -1;
  for (auto& l : atoms)
    for (int a : l) last = std::max(last, p->seg_of[a]);
  for (int k = 0; k <= last; ++k) {
    const int j_from = k == 0 ? p->g.nz - 1 : p->seg_lo[k - 1] - 1;
    int rc = sweep_s2(p, j_from, p->seg_lo[k], k == 0, st);
    if (rc) return rc;
    for (int e = 0; e < n_edges; ++e) {
      std::vector<int32_t> seg;
      for (int a : atoms[e])
        if (p->seg_of[a] == k) seg.push_back(a);
      if (seg.empty()) continue;
      rc = run(e, seg);
      if (rc) return rc;
    }
  }
  for (int e = 0; e < n_edges; ++e)  // an edge without atoms: its outputs are zero (or unchanged)
    if (contributions[e] == 0 && !accumulate) {
      HIPCHK(launch_zero(edges[e].out, n_out, st), "zero");
    }
  return BIP_OK;
}

// Reconstruction and contraction of `atoms` (whose S2 windows are in the
// plan's window stack); accumulate: add to the outputs instead of
// overwriting them.
static int signal_atoms(bip_plan* p, const std::vector<int32_t>& atoms, int32_t n_ch, const float* H,
                        const int64_t* H_off, int32_t scan_sy, int32_t scan_sx, int32_t out_mode,
                        int32_t precision, float* out, void* ext_work, size_t ext_bytes,
                        bool accumulate, hipStream_t st) {
  const bool gram = out_mode == BIP_OUT_MAP;          // map via psi^H Q psi
  const bool map_direct = out_mode == BIP_OUT_MAP_DIRECT;
  const int P = scan_sy * scan_sx;
  const int64_t Ppad = roundup(P, 128);
  const int64_t Dpad = roundup(p->ndet, 128);  // detector rows (direct path)
  const int64_t Dk = roundup(p->ndet, 32);     // detector as contraction index (Gram path)
  const int64_t csz = (precision == BIP_PREC_BF16 || precision == BIP_PREC_FP16) ? 4 : 8;  // bytes per complex element
  const int planes = precision == BIP_PREC_SPLIT_BF16 ? 4 : 2;
  const int64_t esz = csz / planes;                         // bytes per plane element
  // The Gram matrix sums products over all n_det detector beams, which
  // averages the operand rounding: in split mode with a large detector it runs
  // as single FP16 products (FP32 accumulate), the operand scaled by 2^8 so
  // that its typical magnitude G^-1/2 ~ 2^-8..2^-10 sits well inside the FP16
  // normal range; Q is stored split for the quadratic form, whose rounding does
  // not average.
  const int gram_prec = gram_precision(precision, p->ndet);
  const float gram_scale = gram_prec == BIP_PREC_FP16 ? 256.f : 1.f;
  auto kd_of = [](int W) { return roundup((int64_t)W * W, 32); };   // padded window pixels
  auto n1_of = [](int W) { return roundup((int64_t)W * W, 128); };  // ... to whole tiles
  auto ldf_of = [](int W) { return roundup((int64_t)W * W, 64); };  // DFT workspace pitch
  // per-atom blocks, in buffer order: [0] DFT workspace (complex64 elements),
  // [1..3] contraction operands (plane elements), [4] in focal mode the probe
  // at the centroid on the enlarged window (FP32 planes)
  auto sizes = [&](int a, int64_t* s) {
    const int W = p->W[a], W1 = p->W1[a];
    s[0] = (int64_t)P * ldf_of(W1);                                // X [S_y][S_x][r] (S1 window)
    s[1] = gram ? n1_of(W) * Dk : Dpad * kd_of(W);                 // S2~^T [r][d] | S2~ [d][r]
    s[2] = gram ? n1_of(W) * kd_of(W) : (int64_t)n_ch * Ppad * kd_of(W);  // Q [r][r'] | U_n [rho][r]
    s[3] = gram ? Ppad * kd_of(W) : 0;                             // psi^T [rho][r]
    s[4] = p->focal ? Ppad * kd_of(W1) : 0;                        // psi at the centroid
  };
  auto atom_bytes = [&](int a) {
    int64_t s[5];
    sizes(a, s);
    return s[0] * 8 + (s[1] + s[2] + s[3]) * csz + s[4] * 8;
  };
  int max_n1_all = 0;
  for (int a : atoms) max_n1_all = std::max<int>(max_n1_all, (int)n1_of(p->W[a]));
  const int64_t n_partial_tiles = gram ? GEMM_MAX_ZSPLIT * (max_n1_all / 128) : Dpad / 128;
  // residue cells of the aperture beams (h_y mod S_y, h_x mod S_x), beams ascending in each
  std::vector<int32_t>& cells = p->h_cells;
  cells.assign((size_t)P + 1 + p->B, 0);
  {
    std::vector<int32_t> cell_of(p->B);
    for (int b = 0; b < p->B; ++b) {
      const int hy = p->beams[2 * b], hx = p->beams[2 * b + 1];
      const int a = ((hy % scan_sy) + scan_sy) % scan_sy, c = ((hx % scan_sx) + scan_sx) % scan_sx;
      cell_of[b] = a * scan_sx + c;
      cells[cell_of[b] + 1]++;
    }
    for (int i = 0; i < P; ++i) cells[i + 1] += cells[i];
    std::vector<int32_t> fill(cells.begin(), cells.begin() + P);
    for (int b = 0; b < p->B; ++b) cells[P + 1 + fill[cell_of[b]]++] = b;
  }
  // twiddles exp(-2 pi i k / S) of the raster DFTs, rounded from double
  std::vector<float2>& tws = p->h_tws;
  tws.resize((size_t)scan_sx + scan_sy);
  for (int k = 0; k < scan_sx; ++k) {
    const double t = 2.0 * kPi * k / scan_sx;
    tws[k] = make_float2((float)std::cos(t), (float)-std::sin(t));
  }
  for (int k = 0; k < scan_sy; ++k) {
    const double t = 2.0 * kPi * k / scan_sy;
    tws[scan_sx + k] = make_float2((float)std::cos(t), (float)-std::sin(t));
  }
  const char* env = std::getenv("BIP_WORKSPACE_GB");
  const double budget_gb = env ? std::atof(env) : 24.0;
  const int64_t budget = ext_work ? (int64_t)ext_bytes - 16 * 256 : (int64_t)(budget_gb * (1 << 30));
  const int64_t n_jobs_total = (int64_t)atoms.size() * (n_ch + 2);
  const int64_t fixed = n_partial_tiles * Ppad * 4 +
                        (out_mode == BIP_OUT_QEELS ? (int64_t)P * p->ndet * 4 : 0) +
                        n_jobs_total * (int64_t)sizeof(GemmJob) +
                        (int64_t)atoms.size() * (int64_t)(sizeof(ProbeJob) + sizeof(FocalProbeJob)) + 64 +
                        (int64_t)cells.size() * 4 + (int64_t)tws.size() * 8 + (1 << 20);
  // chunking: consecutive atoms while the per-chunk operands fit the budget
  std::vector<std::pair<int, int>> chunks;
  int64_t max_chunk = 0;
  {
    int b = 0;
    while (b < (int)atoms.size()) {
      int e = b;
      int64_t bytes = 0;
      while (e < (int)atoms.size() && (e == b || bytes + atom_bytes(atoms[e]) + fixed <= budget)) {
        bytes += atom_bytes(atoms[e]);
        ++e;
      }
      chunks.push_back({b, e});
      max_chunk = std::max(max_chunk, bytes);
      b = e;
    }
  }
  const size_t need = (size_t)(fixed + max_chunk + 16 * 256);
  char* work_base = nullptr;
  size_t work_cap = 0;
  if (ext_work) {
    if (need > ext_bytes)
      return err(BIP_EUNSUPPORTED, "this signal needs " + std::to_string(need) +
                                       " bytes of workspace; the allocation-free entry point has " +
                                       std::to_string(ext_bytes));
    work_base = (char*)ext_work;
    work_cap = ext_bytes;
  } else {
    int rc = ensure_work(p, need, st);
    if (rc) return rc;
    work_base = (char*)p->d_work;
    work_cap = p->work_bytes;
  }
  Workspace ws{work_base, 0};
  float* partial = (float*)ws.take(n_partial_tiles * Ppad * 4);
  float* beams_out = out_mode == BIP_OUT_BEAMS ? out : nullptr;
  float* beams_tmp = nullptr;
  if (out_mode == BIP_OUT_QEELS) {
    beams_tmp = (float*)ws.take((int64_t)P * p->ndet * 4);
    beams_out = beams_tmp;
  }
  GemmJob* d_jobs = (GemmJob*)ws.take(n_jobs_total * sizeof(GemmJob) + 64);
  ProbeJob* d_probe = (ProbeJob*)ws.take(atoms.size() * sizeof(ProbeJob));
  int32_t* d_cells = (int32_t*)ws.take(cells.size() * 4);
  float2* d_tws = (float2*)ws.take(tws.size() * 8);
  ReconAtom* d_ratoms = (ReconAtom*)ws.take(atoms.size() * sizeof(ReconAtom));
  FocalProbeJob* d_fjobs = p->focal ? (FocalProbeJob*)ws.take(atoms.size() * sizeof(FocalProbeJob) + 64) : nullptr;
  const size_t chunk_base = ws.used;
  if (ws.used > work_cap) return err(BIP_ENOMEM, "internal: tables exceed the workspace");
  HIPCHK(hipMemcpyAsync(d_cells, cells.data(), cells.size() * 4, hipMemcpyHostToDevice, st), "cells");
  HIPCHK(hipMemcpyAsync(d_tws, tws.data(), tws.size() * 8, hipMemcpyHostToDevice, st), "twiddles");
  if ((out_mode == BIP_OUT_MAP || map_direct) && !accumulate) HIPCHK(launch_zero(out, P, st), "zero");
  if (beams_out && (beams_tmp || !accumulate)) HIPCHK(launch_zero(beams_out, (int64_t)P * p->ndet, st), "zero");
  // job tables, chunk-relative offsets
  std::vector<ProbeJob>& jprobe = p->h_probe;
  std::vector<GemmJob>& jdet = p->h_jobs2;
  std::vector<GemmJob>& jquad = p->h_jobs3;
  jprobe.clear();
  jdet.clear();
  jquad.clear();
  std::vector<int64_t> off[5];
  std::vector<int64_t> chunk_plane[5];
  for (auto& v : chunk_plane) v.assign(chunks.size(), 0);
  for (size_t c = 0; c < chunks.size(); ++c) {
    int64_t acc[5] = {0, 0, 0, 0, 0};
    for (int i = chunks[c].first; i < chunks[c].second; ++i) {
      int64_t s[5];
      sizes(atoms[i], s);
      for (int k = 0; k < 5; ++k) {
        off[k].push_back(acc[k]);
        acc[k] += s[k];
      }
    }
    for (int k = 0; k < 5; ++k) chunk_plane[k][c] = acc[k];
  }
  std::vector<FocalProbeJob>& jfocal = p->h_fjobs;
  jfocal.clear();
  std::vector<int64_t> det_first(atoms.size());
  for (size_t i = 0; i < atoms.size(); ++i) {
    const int a = atoms[i];
    const int W = p->W[a];
    const int32_t W2 = W * W, kd = (int32_t)kd_of(W);
    int32_t cu0, cnu, cv0, cnv;
    crop_run(p->tau_y[a], p->g.ny, scan_sy, p->f, cu0, cnu);
    crop_run(p->tau_x[a], p->g.nx, scan_sx, p->f, cv0, cnv);
    ProbeJob pj{};
    pj.win_off = p->off1[a];
    pj.fx_off = off[0][i];
    pj.out_off = gram ? off[3][i] : off[2][i];
    pj.h_off = H_off[a];
    pj.W = W;
    pj.oy = p->oy[a];
    pj.ox = p->ox[a];
    pj.kd = kd;
    pj.ldf = (int32_t)ldf_of(W);
    if (p->focal) {  // the probe at the centroid on the enlarged window, then the forward step
      const int W1 = p->W1[a];
      pj.out_off = off[4][i];
      pj.W = W1;
      pj.oy = p->oy1[a];
      pj.ox = p->ox1[a];
      pj.kd = (int32_t)kd_of(W1);
      pj.ldf = (int32_t)ldf_of(W1);
      jfocal.push_back(FocalProbeJob{off[4][i], gram ? off[3][i] : off[2][i], H_off[a], W1, W, kd,
                                     (int32_t)kd_of(W1), a, 0});
    }
    pj.t0 = jprobe.empty() ? 0 : jprobe.back().t0 + (jprobe.back().W * jprobe.back().W + 63) / 64;
    jprobe.push_back(pj);
    det_first[i] = (int64_t)jdet.size();
    if (gram) {
      // Gram: A = B = S2~^T [r][d] (A conjugated, K-blocked), output Q [r][r']
      GemmJob q{};
      q.a_off = q.b_off = off[1][i];
      q.K = (int32_t)Dk;
      q.lda = q.ldb = gemm_bk(precision);
      q.kstride = (int32_t)(n1_of(W) * gemm_bk(precision));
      q.m_lim = q.n_lim = W2;
      q.W2 = W2;
      q.ldo = kd;
      q.h_off = H_off[a];
      q.out_off = off[2][i];
      jdet.push_back(q);
      // quadratic form: A = psi^T [rho][r'], B = Q [r][r']
      GemmJob u{};
      u.a_off = off[3][i];
      u.b_off = off[2][i];
      u.K = u.lda = u.ldb = kd;
      u.m_lim = (int32_t)Ppad;
      u.n_lim = W2;
      u.W2 = W2;
      u.cu0 = cu0;
      u.cnu = cnu;
      u.cv0 = cv0;
      u.cnv = cnv;
      jquad.push_back(u);
    } else {
      for (int n = 0; n < n_ch; ++n) {
        // detector contraction: A = S2~ [d][r], B = U_n [rho][r]
        GemmJob d{};
        d.a_off = off[1][i];
        d.b_off = off[2][i] + (int64_t)n * Ppad * kd;
        d.K = d.lda = d.ldb = kd;
        d.m_lim = (int32_t)Dpad;
        d.n_lim = (int32_t)Ppad;
        d.W2 = W2;
        d.cu0 = cu0;
        d.cnu = cnu;
        d.cv0 = cv0;
        d.cnv = cnv;
        jdet.push_back(d);
      }
    }
  }
  // batched S2~ operand reconstruction of the Gram path (square-lattice parents)
  const bool recon_batched = gram && p->tile_np2 <= TILE_NP;
  std::vector<ReconAtom>& ratoms = p->h_ratoms;
  ratoms.clear();
  if (recon_batched) {
    for (size_t i = 0; i < atoms.size(); ++i) {
      const int a = atoms[i];
      ratoms.push_back(ReconAtom{p->off2[a], off[1][i], p->W[a], p->oy[a], p->ox[a], (int32_t)n1_of(p->W[a])});
    }
    HIPCHK(hipMemcpyAsync(d_ratoms, ratoms.data(), ratoms.size() * sizeof(ReconAtom), hipMemcpyHostToDevice, st),
           "recon atoms");
  }
  GemmJob* d_jdet = d_jobs;
  GemmJob* d_jquad = d_jdet + jdet.size();
  // Gram launches: one per chunk over its atoms' jobs (their slot rows set here)
  std::vector<int64_t> gram_gx(chunks.size(), 0);
  if (gram)
    for (size_t c = 0; c < chunks.size(); ++c) {
      int tiles = 0;
      for (int i = chunks[c].first; i < chunks[c].second; ++i)
        tiles = std::max(tiles, (int)(n1_of(p->W[atoms[i]]) / 128));
      gram_gx[c] = gemm_gram_plan(&jdet[det_first[chunks[c].first]], chunks[c].second - chunks[c].first, tiles);
      if (gram_gx[c] > 0x7fffffff) return err(BIP_EUNSUPPORTED, "Gram launch beyond the grid limit");
    }
  HIPCHK(hipMemcpyAsync(d_probe, jprobe.data(), jprobe.size() * sizeof(ProbeJob), hipMemcpyHostToDevice, st), "jobs");
  if (p->focal && !jfocal.empty())
    HIPCHK(hipMemcpyAsync(d_fjobs, jfocal.data(), jfocal.size() * sizeof(FocalProbeJob), hipMemcpyHostToDevice, st),
           "jobs");
  HIPCHK(hipMemcpyAsync(d_jdet, jdet.data(), jdet.size() * sizeof(GemmJob), hipMemcpyHostToDevice, st), "jobs");
  if (!jquad.empty())
    HIPCHK(hipMemcpyAsync(d_jquad, jquad.data(), jquad.size() * sizeof(GemmJob), hipMemcpyHostToDevice, st), "jobs");
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
  pa.ny = p->g.ny;
  pa.nx = p->g.nx;
  pa.mode = p->o.recon_mode;
  pa.Sy = scan_sy;
  pa.Sx = scan_sx;
  pa.P = P;
  pa.Ppad = (int)Ppad;
  // probe coefficients of the whole aperture; retained beams scaled by f^2
  pa.cb = (float)((double)p->f * p->f / std::sqrt((double)p->g.ny * p->g.nx * p->B_full));
  pa.H = (const float2*)H;
  pa.n_ch = n_ch;
  for (size_t c = 0; c < chunks.size(); ++c) {
    ws.used = chunk_base;
    const int64_t pl0 = chunk_plane[0][c], pl1 = chunk_plane[1][c], pl2 = chunk_plane[2][c],
                  pl3 = chunk_plane[3][c], pl4 = chunk_plane[4][c];
    float2* X = (float2*)ws.take(pl0 * 8);
    char* S2op = (char*)ws.take(pl1 * csz);
    char* X2 = (char*)ws.take(pl2 * csz);   // Q (Gram) or U (direct)
    char* PsiT = (char*)ws.take(std::max<int64_t>(pl3, 1) * csz);
    float* PsiC = p->focal ? (float*)ws.take(std::max<int64_t>(pl4, 1) * 8) : nullptr;
    if (ws.used > work_cap) return err(BIP_ENOMEM, "internal: chunk exceeds the workspace");
    int max_n1 = 0, max_kd = 0, max_m = 0;
    const int c0 = chunks[c].first, c1 = chunks[c].second, nat = c1 - c0;
    for (int i = c0; i < c1; ++i) {
      const int a = atoms[i];
      const int W = p->W[a], W1 = p->W1[a];
      int64_t s[5];
      sizes(a, s);
      max_n1 = std::max<int>(max_n1, (int)n1_of(W));
      max_kd = std::max<int>(max_kd, (int)kd_of(W1));
      max_m = std::max(max_m, W1);
      if (off[0][i] + s[0] > pl0 || off[1][i] + s[1] > pl1 || off[2][i] + s[2] > pl2 ||
          off[3][i] + s[3] > pl3 || off[4][i] + s[4] > pl4)
        return err(BIP_EINVAL, "internal: operand block outside its buffer");
      if (gram && !recon_batched) {
        ReconArgs ra = recon_args(p, a, 2);
        ra.scale = gram_scale;
        HIPCHK(timed(p, ST_RECON, st, [&] {
                 return launch_recon_operand(ra, S2op + off[1][i] * esz, 0, gram_prec, Dk, n1_of(W), Dk,
                                             pl1, st);
               }),
               "recon S2 operand");
      } else if (!gram)
        HIPCHK(timed(p, ST_RECON, st, [&] {
                 return launch_recon_operand(recon_args(p, a, 2), S2op + off[1][i] * esz, 1, precision,
                                             kd_of(W), Dpad, kd_of(W), pl1, st);
               }),
               "recon S2 operand");
    }
    if (recon_batched) {
      ReconArgs ra = recon_args(p, atoms[c0], 2);
      ra.win = p->d_win2;
      ra.scale = gram_scale;
      HIPCHK(timed(p, ST_RECON, st, [&] {
               return launch_recon_kblk_atoms(ra, d_ratoms + c0, nat, S2op, gram_prec, Dk, pl1, st);
             }),
             "recon S2 operand");
    }
    // probe synthesis for every atom of the chunk (grid z = atom)
    pa.jobs = d_probe + c0;
    pa.fx = X;
    pa.out = gram ? (void*)PsiT : (void*)X2;
    pa.out_plane = gram ? pl3 : pl2;
    const int unit0 = jprobe[c0].t0;
    const int n_units = jprobe[c1 - 1].t0 + (jprobe[c1 - 1].W * jprobe[c1 - 1].W + 63) / 64 - unit0;
    HIPCHK(timed(p, ST_FOLD, st, [&] { return launch_probe_fold_x(pa, unit0, n_units, nat, st); }),
           "probe fold");
    if (!p->focal) {
      HIPCHK(timed(p, ST_PROBE, st, [&] { return launch_probe_y(pa, precision, !gram, max_kd, nat, st); }),
             "probe synthesis");
    } else {
      // the probe at the centroid (FP32) on the enlarged window, then its forward
      // step to the ionization plane, cropped to the window, into the operand
      pa.out = PsiC;
      pa.out_plane = pl4;
      HIPCHK(timed(p, ST_PROBE, st, [&] { return launch_probe_y(pa, BIP_PREC_FP32, false, max_kd, nat, st); }),
             "probe synthesis");
      FocalProbeArgs fp{};
      fp.jobs = d_fjobs + c0;
      fp.psi_c = PsiC;
      fp.psi_plane = pl4;
      fp.out = gram ? (void*)PsiT : (void*)X2;
      fp.out_plane = gram ? pl3 : pl2;
      fp.H = (const float2*)H;
      fp.n_ch = n_ch;
      fp.P = P;
      fp.Ppad = (int)Ppad;
      fp.L = p->L;
      fp.tw = p->d_tw;
      fp.dy = p->g.ly / p->g.ny;
      fp.dx = p->g.lx / p->g.nx;
      fp.lambda = p->lambda;
      fp.dist = p->d_fdist;
      HIPCHK(timed(p, ST_PROBE, st, [&] { return launch_focal_probe(fp, precision, !gram, nat, max_m, st); }),
             "focal probe step");
    }
    GemmArgs g{};
    g.H = (const float2*)H;
    g.n_ch = n_ch;
    g.ndet = p->ndet;
    g.P = P;
    g.Mpad = (int)Ppad;
    // PRISM interpolation factor: crop masks and the f^2 of the detector sum
    g.crop = p->f > 1 ? 1 : 0;
    g.Sy = scan_sy;
    g.Sx = scan_sx;
    g.oscale = (float)(p->f * p->f);
    if (gram) {
      GemmArgs q = g;
      q.A = S2op;
      q.a_plane = pl1;
      q.B = S2op;
      q.b_plane = pl1;
      q.jobs = d_jdet + det_first[c0];
      q.njobs = nat;
      q.out = X2;
      q.out_plane = pl2;
      q.tiles = max_n1 / 128;
      q.gscale = (float)(p->f * p->f) / (gram_scale * gram_scale);
      q.qtri = 1;
      HIPCHK(timed(p, ST_GRAM, st, [&] {
               return launch_zgemm_gram(gram_prec, precision, q, (int)gram_gx[c], st);
             }),
             "Gram contraction");
      GemmArgs u = g;
      u.A = PsiT;
      u.a_plane = pl3;
      u.B = X2;
      u.b_plane = pl2;
      u.jobs = d_jquad + c0;
      u.njobs = nat;
      u.partial = partial;
      u.qtri = 1;
      // job groups that fill the chip evenly; partial rows reduced in a fixed order
      const int qt = (int)(Ppad / 128) * (max_n1 / 128);
      u.zsplit = quad_groups(qt, nat, p->n_cu);
      HIPCHK(timed(p, ST_DET, st, [&] {
               return launch_zgemm(precision, EPI_QUAD, u, (int)(Ppad / 128), max_n1 / 128, u.zsplit, st);
             }),
             "quadratic form");
      HIPCHK(timed(p, ST_REDUCE, st, [&] {
               return launch_reduce_map(partial, u.zsplit * (max_n1 / 128), (int)Ppad, P, out, 1, st);
             }),
             "reduce");
    } else {
      GemmArgs d = g;
      d.A = S2op;
      d.a_plane = pl1;
      d.B = X2;
      d.b_plane = pl2;
      d.jobs = d_jdet + det_first[c0];
      d.njobs = nat * n_ch;
      d.partial = partial;
      d.out_beams = beams_out;
      d.Npad = (int)Ppad;
      HIPCHK(timed(p, ST_DET, st, [&] {
               return launch_zgemm(precision, map_direct ? EPI_ABS2_MAP : EPI_ABS2_BEAMS, d,
                                   (int)(Dpad / 128), (int)(Ppad / 128), 1, st);
             }),
             "detector contraction");
      if (map_direct)
        HIPCHK(timed(p, ST_REDUCE, st, [&] {
                 return launch_reduce_map(partial, (int)(Dpad / 128), (int)Ppad, P, out, 1, st);
               }),
               "reduce");
    }
  }
  if (out_mode == BIP_OUT_QEELS) {
    // bins of h_x, each listing its detector beams in detector order
    std::vector<int32_t>& start = p->h_qstart;
    std::vector<int32_t>& list = p->h_qlist;
    start.assign(p->nq + 1, 0);
    list.clear();
    std::vector<std::vector<int32_t>> bins(p->nq);
    for (int d = 0; d < p->ndet; ++d) {
      const int q = p->det[2 * d + 1] + p->nq_half;
      if (q >= 0 && q < p->nq) bins[q].push_back(d);
    }
    for (int q = 0; q < p->nq; ++q) {
      start[q + 1] = start[q] + (int)bins[q].size();
      list.insert(list.end(), bins[q].begin(), bins[q].end());
    }
    int32_t* d_start = (int32_t*)ws.take(start.size() * 4);
    int32_t* d_list = (int32_t*)ws.take(list.size() * 4 + 4);
    if (ws.used > work_cap) return err(BIP_ENOMEM, "qEELS bin tables exceed the workspace");
    HIPCHK(hipMemcpyAsync(d_start, start.data(), start.size() * 4, hipMemcpyHostToDevice, st), "bins");
    HIPCHK(hipMemcpyAsync(d_list, list.data(), list.size() * 4, hipMemcpyHostToDevice, st), "bins");
    HIPCHK(launch_qeels_from_beams(beams_tmp, d_start, d_list, p->ndet, P, p->nq, out, accumulate ? 1 : 0, st),
           "qeels");
  }
  return BIP_OK;
}

extern "C" {

int bip_set_profiling(bip_plan* p, int32_t enable) {
  if (!p) return err(BIP_EINVAL, "NULL plan");
  p->profiling = enable != 0;
  return BIP_OK;
}

int bip_stage_timings(bip_plan* p, double* ms, int64_t* launches, int32_t reset) {
  if (!p || !ms || !launches) return err(BIP_EINVAL, "NULL argument");
  int rc = collect_timings(p);
  if (rc) return rc;
  for (int i = 0; i < ST_COUNT; ++i) {
    ms[i] = p->stage_ms[i];
    launches[i] = p->stage_launches[i];
    if (reset) {
      p->stage_ms[i] = 0;
      p->stage_launches[i] = 0;
    }
  }
  return BIP_OK;
}

int bip_query(const bip_plan* p, int32_t what, void* out) {
  if (!p || !out) return err(BIP_EINVAL, "NULL argument");
  switch (what) {
    case BIP_Q_COUNTS: {
      int64_t* o = (int64_t*)out;
      o[0] = p->B;
      o[1] = p->ndet;
      o[2] = p->Bp1;
      o[3] = p->Bp2;
      o[4] = p->nq;
      o[5] = p->n_atoms;
      o[6] = (int64_t)p->col1.size();
      o[7] = (int64_t)p->col2.size();
      return BIP_OK;
    }
    case BIP_Q_BEAMS: std::memcpy(out, p->beams.data(), p->beams.size() * 4); return BIP_OK;
    case BIP_Q_DETECTOR: std::memcpy(out, p->det.data(), p->det.size() * 4); return BIP_OK;
    case BIP_Q_PARENTS1: std::memcpy(out, p->par1.data(), p->par1.size() * 4); return BIP_OK;
    case BIP_Q_PARENTS2: std::memcpy(out, p->par2.data(), p->par2.size() * 4); return BIP_OK;
    case BIP_Q_PLANES: std::memcpy(out, p->plane.data(), p->plane.size() * 4); return BIP_OK;
    case BIP_Q_WEIGHTS1:
    case BIP_Q_WEIGHTS2: {
      const bool one = what == BIP_Q_WEIGHTS1;
      const auto& rp = one ? p->rp1 : p->rp2;
      const auto& cl = one ? p->col1 : p->col2;
      const auto& w = one ? p->w1 : p->w2;
      char* o = (char*)out;
      std::memcpy(o, rp.data(), rp.size() * 4);
      o += rp.size() * 4;
      std::memcpy(o, cl.data(), cl.size() * 4);
      o += cl.size() * 4;
      std::memcpy(o, w.data(), w.size() * 8);
      return BIP_OK;
    }
    case BIP_Q_MEMORY: {
      int64_t* o = (int64_t*)out;
      o[0] = p->bytes_now;
      o[1] = p->bytes_peak;
      o[2] = (int64_t)p->allocations.size();
      return BIP_OK;
    }
    case BIP_Q_SCALARS: {
      double* o = (double*)out;
      o[0] = p->lambda;
      o[1] = p->sigma;
      o[2] = p->column_batch;
      o[3] = p->s2_stream ? (double)p->seg_hi.size() : 0.0;
      return BIP_OK;
    }
    default:
      return err(BIP_EINVAL, "unknown query");
  }
}

}  // extern "C"
