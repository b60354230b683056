// Host side of liblgbr: contexts, workspaces, the stage pipeline of the three RHS forms,
// SSP-RK3 and graph-captured multi-problem batches (C ABI declared in include/lgbr.h).
//
// Stage pipeline (Alg. 1-3 of the paper, in data-parallel form):
//   ghost images -> primitives (+ troubled flags) ->
//   [C-GBR] gradients per direction (E6 explicit or C4 line solves) -> Omega sensor
//           (-> C-GBR viscous node fluxes when viscous)
//   [LAD]   |S|, div u, e -> raw mu*, beta*, kappa* -> truncated Gaussian per direction
//           -> node fluxes F^c + F^v per direction
//   [hyb]   flag dilation (per-cell) or any-flag reduction (global)
//   -> one interface sweep per direction (flux + FP64 difference into dQ/dt)
//   [LAD-C6] compact gradients -> LAD coefficients and node fluxes from them -> compact
//           interface-flux solves per direction
// RK3: dt reduction from U^n, then three (stage RHS -> stage combination) passes; LAD-C6
// steps end with the implicit filter along each direction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "lgbr.h"
#include "lgbr_kernels.h"

using lg::Launch;
using lg::Prob;
using lg::RKRef;
using lg::StateRef;

namespace {

void* (*g_alloc)(size_t, void*) = nullptr;
void (*g_free)(void*, void*) = nullptr;
void* g_user = nullptr;

void* dev_alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (g_alloc) return g_alloc(bytes, g_user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  if (g_free) g_free(p, g_user);
  else (void)hipFree(p);
}

struct Cfg {
  int ndim, precision, grad, hybrid_mode, viscous, dilate;
  int lad_c6;           // the LAD scheme is LAD-C6
  int filter;           // steps whose last stage ran LAD end with the implicit filter
  double falpha;
  int filter_all;       // ... or every stage that ran LAD is followed by it
  int rk4;              // LAD steps march with the classic RK4
};

}  // namespace

struct lg_ctx {
  Prob hp;
  Prob* dp = nullptr;
  Launch L{};
  lg::Prof prof{};
  Cfg cfg;
  hipStream_t stream = nullptr;
  std::vector<void*> allocs;
  size_t ws_bytes = 0;
  void* alloc(size_t bytes) {
    void* p = dev_alloc(bytes);
    if (p) {
      allocs.push_back(p);
      ws_bytes += bytes;
    }
    return p;
  }
};

struct lg_batch {
  std::vector<Prob> hps;
  Prob* dps = nullptr;
  Launch L{};
  Cfg cfg;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int nsteps = 0, scheme = 0;
};

namespace {

const double RK_A[3] = {0.0, 0.75, 1.0 / 3.0};
const double RK_B[3] = {1.0, 0.25, 2.0 / 3.0};

// One right-hand side evaluation of the state `ref`.  With rk set, the RK stage
// combination follows: inside the all-LAD interface pass where that pass runs, as its own
// kernel after the per-direction sweeps otherwise.
// LAD-C6 stage (Alg. 1): compact gradients of the primitives, the LAD coefficients and
// node fluxes from them, then the compact interface fluxes differenced per direction (the
// last direction forms the RK stage).
template <typename R>
void enqueue_rhs_c6(const Launch& L, const Cfg& c, StateRef ref, const RKRef* rk, int stage) {
  for (int d = 0; d < c.ndim; ++d) lg::launch_bc_cons(L, ref, d);
  lg::launch_prim<R>(L, ref, 0, nullptr);
  for (int d = 0; d < c.ndim; ++d) lg::launch_grad_c6<R>(L, ref, d);
  lg::launch_lad<R>(L, -1, 1);
  lg::launch_lad_nodeflux<R>(L, -1, 1);
  const double a = rk ? RK_A[stage] : 0.0, b = rk ? RK_B[stage] : 0.0;
  for (int d = 0; d < c.ndim; ++d)
    lg::launch_c6_faces<R>(L, ref, d, d > 0 ? 1 : 0, d == c.ndim - 1 ? rk : nullptr, stage, a, b);
  if (rk) lg::launch_stage_ghosts(L, *rk, stage, -1);
}

template <typename R>
// prim_ghosts: the k_prim mode (0 every node; 1 / 2 the ghosts only, see k_basic.hip)
void enqueue_rhs(const Launch& L, const Cfg& c, int scheme, StateRef ref, const uint8_t* force,
                 const RKRef* rk = nullptr, int stage = 0, int prim_ghosts = 0) {
  if (scheme == LG_SCHEME_LAD && c.lad_c6) {
    enqueue_rhs_c6<R>(L, c, ref, rk, stage);
    return;
  }
  for (int d = 0; d < c.ndim; ++d) lg::launch_bc_cons(L, ref, d);
  const bool hyb = scheme == LG_SCHEME_HYBRID;
  lg::launch_prim<R>(L, ref, hyb ? 1 : 0, force, force ? 0 : prim_ghosts);
  int sel, skip_gbr = -1, skip_lad = -1;
  if (scheme == LG_SCHEME_CGBR) {
    sel = lg::SEL_GBR;
  } else if (scheme == LG_SCHEME_LAD) {
    sel = lg::SEL_LAD;
  } else if (c.hybrid_mode == LG_HYB_GLOBAL) {
    sel = lg::SEL_GLOBAL;
    lg::launch_any_flag(L, 1);
    lg::launch_switch_count(L);
    skip_gbr = 0;  // C-GBR inputs are skipped when no interior node is troubled
    skip_lad = 1;  // LAD inputs are skipped when one is
  } else {
    sel = lg::SEL_PERCELL;
  }
  int region = 0;
  if (sel == lg::SEL_PERCELL) {
    // interface selection: flags dilated by the hybrid radius (-> ft); C-GBR inputs are
    // only needed within three more nodes of those (-> fg), and only the compact lines
    // that cross fg are solved.  With no troubled node at all (any_flag == 0) every
    // interface is LAD and all of this, and the C-GBR inputs, are skipped on the device.
    // With some: the C-GBR interfaces are compacted into a work queue (one persistent pass
    // computes their fluxes, an assembly pass forms the node derivatives with the LAD
    // fluxes of the others); with every interior node troubled, the plain C-GBR sweeps run
    // and the LAD inputs are skipped.
    lg::launch_any_flag(L, 0);
    lg::launch_switch_count(L);
    lg::launch_dilate(L, c.ndim, c.dilate, 0, 2);
    lg::launch_dilate(L, c.ndim, 3, 2, 3);
    lg::launch_hyb_queue(L, c.ndim);
    if (c.grad == LG_GRAD_C4) lg::launch_line_lists(L, c.ndim);
    region = 1;
    skip_gbr = lg::GATE_ANY;
    skip_lad = lg::GATE_NOTALL;
  }
  if (sel != lg::SEL_LAD) {
    for (int d = 0; d < c.ndim; ++d) {
      if (c.grad == LG_GRAD_C4) lg::launch_grad_c4<R>(L, ref, d, skip_gbr, region);
      else lg::launch_grad_explicit<R>(L, d, 6, skip_gbr, region);
    }
    if (c.viscous) {  // the Omega sensor drives the selection in viscous flow only (Sec. 2.3)
      lg::launch_sensor<R>(L, skip_gbr, region);
      lg::launch_gbr_viscflux<R>(L, skip_gbr, region);
    }
  }
  if (sel != lg::SEL_GBR) {
    lg::launch_lad<R>(L, skip_lad);
    lg::launch_lad_nodeflux<R>(L, skip_lad);
  }
  // interfaces: the all-LAD pass (LAD scheme; hybrid with no troubled node), else the
  // per-direction C-GBR sweeps (C-GBR scheme; global hybrid with a troubled node; per-cell
  // hybrid with every node troubled), else the compacted per-cell pass; the hybrid decides
  // on the device, so every applicable form is launched and returns at once unless chosen
  const double a = rk ? RK_A[stage] : 0.0, b = rk ? RK_B[stage] : 0.0;
  const int skip_fused = sel == lg::SEL_LAD ? lg::GATE_NEVER : lg::GATE_NONE;
  const int skip_dir = sel == lg::SEL_GBR ? lg::GATE_NEVER : (sel == lg::SEL_PERCELL ? lg::GATE_ALL : lg::GATE_ANY);
  const int sweep_sel = sel == lg::SEL_PERCELL ? lg::SEL_GBR : sel;
  if (sel != lg::SEL_GBR) lg::launch_lad_sweep<R>(L, ref, rk, stage, a, b, skip_fused);
  if (sel != lg::SEL_LAD) {
    // the last direction's sweep forms the RK stage itself
    for (int d = 0; d < c.ndim; ++d)
      lg::launch_sweep<R>(L, ref, d, sweep_sel, d > 0 ? 1 : 0, skip_dir, d == c.ndim - 1 ? rk : nullptr, stage, a, b);
    if (rk) lg::launch_stage_ghosts(L, *rk, stage, skip_dir);
  }
  if (sel == lg::SEL_PERCELL) {
    lg::launch_gbr_items<R>(L);
    lg::launch_hyb_assemble<R>(L, ref, rk, stage, a, b);
  }
}

// FILTER_CALLS of Alg. 1 after a stage that ran the LAD-based solver: the LAD scheme
// filters every stage result it is asked to; a hybrid stage filters where it ran LAD,
// which the device decides from the stage's troubled-cell reduction (the whole field under
// the global switch when nothing was troubled; the nodes outside the dilated troubled set
// under the per-cell switch).  C-GBR stages are never filtered (Alg. 2).
int filter_mode(const Cfg& c, int scheme) {
  if (!c.filter || scheme == LG_SCHEME_CGBR) return -1;
  if (scheme == LG_SCHEME_LAD) return lg::FILT_ALL;
  return c.hybrid_mode == LG_HYB_GLOBAL ? lg::FILT_GLOBAL : lg::FILT_PERCELL;
}

// Classic RK4 (LAD scheme; Sec. 2.1): each stage's right-hand side into the derivative
// workspace, then the combination (running sum of b_s dt k_s; next stage input U^n + c_s dt
// k_s), the filter after the fourth stage (Alg. 1).
const double RK4_B[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
const double RK4_C[3] = {0.5, 0.5, 1.0};

template <typename R>
void enqueue_rk4(const Launch& L, const Cfg& c, int scheme, double* Qx, double* tx, double t_end) {
  lg::launch_dt(L, Qx, tx, t_end, 1);
  const int fmode = filter_mode(c, scheme);
  for (int s = 0; s < 4; ++s) {
    const StateRef ref{s == 0 ? Qx : nullptr, nullptr, s == 0 ? 0 : 1};
    enqueue_rhs<R>(L, c, scheme, ref, nullptr);
    lg::launch_rk4_combine(L, Qx, s, RK4_B[s], s < 3 ? RK4_C[s] : 0.0);
    if (s < 3) lg::launch_stage_ghosts(L, RKRef{Qx, nullptr, nullptr}, 0, -1);   // FIXED ghosts of U^n
    if (fmode >= 0 && (s == 3 || c.filter_all)) {
      const StateRef out{s == 3 ? Qx : nullptr, nullptr, s == 3 ? 0 : 1};   // the stage result
      for (int d = 0; d < c.ndim; ++d) lg::launch_filter(L, out, d, fmode);
    }
  }
}

template <typename R>
void enqueue_rk3(const Launch& L, const Cfg& c, int scheme, double* Qx, double* tx, double t_end) {
  lg::launch_dt(L, Qx, tx, t_end, 1);
  const int fmode = filter_mode(c, scheme);
  for (int s = 0; s < 3; ++s) {
    StateRef ref{s == 0 ? Qx : nullptr, nullptr, s == 0 ? 0 : 1};
    // a hybrid stage keeps the unfiltered state where the filter would leave a
    // non-physical node (a troubled node, which its C-GBR phases never filter); under the
    // global switch the last stage is filtered only where it ran all-LAD, and that pass
    // leaves the copy the guard restores from
    const bool guard = scheme == LG_SCHEME_HYBRID && fmode >= 0 && (s == 2 || c.filter_all);
    const bool fused_save = guard && fmode == lg::FILT_GLOBAL && s == 2;
    // the all-LAD pass of stages 1 and 2 also converts its result for the next stage (not
    // when a filter follows the stage, nor where LAD-C6 forms the stage in its face solves)
    const bool lad_e4 = scheme == LG_SCHEME_LAD && !c.lad_c6;
    const bool global = scheme == LG_SCHEME_HYBRID && c.hybrid_mode == LG_HYB_GLOBAL;
    const bool fuse_prim = !c.filter_all && (lad_e4 || global);
    const int prim_out = fuse_prim && s < 2 ? (global ? 2 : 1) : 0;
    const int prim_ghosts = fuse_prim && s > 0 ? (global ? 2 : 1) : 0;
    RKRef rr{Qx, nullptr, nullptr, fused_save ? 1 : 0, prim_out};
    enqueue_rhs<R>(L, c, scheme, ref, nullptr, &rr, s, prim_ghosts);
    if (fmode >= 0 && (s == 2 || c.filter_all)) {   // after the last stage (Alg. 1)
      const StateRef out{s == 2 ? Qx : nullptr, nullptr, s == 2 ? 0 : 1};   // the stage result
      if (guard && !fused_save) lg::launch_filter_save(L, out, fmode);
      for (int d = 0; d < c.ndim; ++d) lg::launch_filter(L, out, d, fmode);
      if (guard) lg::launch_filter_guard(L, out, fmode);
    }
  }
}

lg_status last_hip() { return hipGetLastError() == hipSuccess ? LG_OK : LG_EHIP; }

bool valid_bc(int b) { return b >= LG_BC_PERIODIC && b <= LG_BC_NOSLIP_ISOTHERMAL; }

// LU tables of the compact-gradient systems (see k_grad.hip for the layout)
std::vector<double> tri_bounded(int N) {
  std::vector<double> t(2 * N, 0.0);
  double* cp = t.data();
  double* inv = t.data() + N;
  cp[0] = 0.0;
  inv[0] = 1.0;
  for (int i = 1; i < N - 1; ++i) {
    double den = 1.0 - 0.25 * cp[i - 1];
    inv[i] = 1.0 / den;
    cp[i] = 0.25 / den;
  }
  cp[N - 1] = 0.0;
  inv[N - 1] = 1.0;
  return t;
}

void append_band_header(std::vector<double>& t, int L, int steps);

// PCR elimination factors of the C4 matrix (see k_grad_c4_pcr): k1[steps][L], k2[steps][L],
// binv[L], then the band header; periodic lines wrap their indices.
std::vector<double> pcr_table(int L, bool periodic, int steps) {
  std::vector<double> a(L), b(L), c(L), na(L), nb(L), nc(L);
  for (int i = 0; i < L; ++i) {
    bool end = !periodic && (i == 0 || i == L - 1);
    a[i] = end ? 0.0 : 0.25;
    c[i] = end ? 0.0 : 0.25;
    b[i] = 1.0;
  }
  std::vector<double> t((size_t)(2 * steps + 1) * L, 0.0);
  for (int st = 0; st < steps; ++st) {
    const int s = 1 << st;
    for (int i = 0; i < L; ++i) {
      int im = i - s, ip = i + s;
      bool hm = true, hp = true;
      if (periodic) {
        im = ((im % L) + L) % L;
        ip = ip % L;
      } else {
        hm = im >= 0;
        hp = ip < L;
      }
      double k1 = hm ? a[i] / b[im] : 0.0;
      double k2 = hp ? c[i] / b[ip] : 0.0;
      na[i] = hm ? -k1 * a[im] : 0.0;
      nc[i] = hp ? -k2 * c[ip] : 0.0;
      nb[i] = b[i] - (hm ? k1 * c[im] : 0.0) - (hp ? k2 * a[ip] : 0.0);
      t[(size_t)st * L + i] = k1;
      t[(size_t)(steps + st) * L + i] = k2;
    }
    a.swap(na);
    b.swap(nb);
    c.swap(nc);
  }
  for (int i = 0; i < L; ++i) t[(size_t)2 * steps * L + i] = 1.0 / b[i];
  append_band_header(t, L, steps);
  return t;
}

// Thomas tables (cp[m], inv[m], a[m]; see k_compact.hip) of the unit-diagonal tridiagonal
// system with sub-diagonal a[i] and super-diagonal c[i] (a[0] = c[m-1] = 0)
std::vector<double> thomas_table(const std::vector<double>& a, const std::vector<double>& c) {
  const int m = (int)a.size();
  std::vector<double> t(3 * (size_t)m, 0.0);
  double* cp = t.data();
  double* inv = t.data() + m;
  for (int i = 0; i < m; ++i) {
    const double den = 1.0 - (i > 0 ? a[i] * cp[i - 1] : 0.0);
    inv[i] = 1.0 / den;
    cp[i] = c[i] / den;
    t[2 * (size_t)m + i] = a[i];
  }
  return t;
}

// cyclic [alpha, 1, alpha] of n unknowns: cp[n], inv[n], z[n], fac, alpha (see k_compact.hip)
// Cyclic factors of the system with unit diagonal and off-diagonals al (n unknowns):
// cp[n], inv[n], z[n], fac, al, then c[n] with y_0 = sum_k c_k d_k for the forward
// values d_k (c_0 = 1, c_k = -c_{k-1} cp_{k-1}), so that the one back substitution can
// emit x = y - (y_0 - al y_{n-1}) fac z directly.
std::vector<double> cyclic_table(int n, double al) {
  std::vector<double> t(4 * (size_t)n + 2, 0.0);
  double* cp = t.data();
  double* inv = t.data() + n;
  double* z = t.data() + 2 * n;
  std::vector<double> b(n, 1.0);
  b[0] = 2.0;
  b[n - 1] = 1.0 + al * al;
  for (int i = 0; i < n; ++i) {
    const double den = b[i] - (i > 0 ? al * cp[i - 1] : 0.0);
    inv[i] = 1.0 / den;
    cp[i] = (i < n - 1 ? al : 0.0) / den;
  }
  std::vector<double> u(n, 0.0), dp(n);
  u[0] = -1.0;
  u[n - 1] = al;
  for (int i = 0; i < n; ++i) dp[i] = (u[i] - (i > 0 ? al * dp[i - 1] : 0.0)) * inv[i];
  z[n - 1] = dp[n - 1];
  for (int i = n - 2; i >= 0; --i) z[i] = dp[i] - cp[i] * z[i + 1];
  t[3 * (size_t)n] = 1.0 / (1.0 + z[0] - al * z[n - 1]);
  t[3 * (size_t)n + 1] = al;
  double* c = t.data() + 3 * (size_t)n + 2;
  c[0] = 1.0;
  for (int k = 1; k < n; ++k) c[k] = -c[k - 1] * cp[k - 1];
  return t;
}

// PCR elimination factors k1[steps][L], k2[steps][L], binv[L] of the unit-diagonal system
// with sub / super-diagonals a, c (periodic: cyclic, indices wrapped)
std::vector<double> pcr_table_ac(std::vector<double> a, std::vector<double> c, bool periodic, int steps) {
  const int L = (int)a.size();
  std::vector<double> b(L, 1.0), na(L), nb(L), nc(L);
  std::vector<double> t((size_t)(2 * steps + 1) * L, 0.0);
  for (int st = 0; st < steps; ++st) {
    const int s = 1 << st;
    for (int i = 0; i < L; ++i) {
      int im = i - s, ip = i + s;
      bool hm = true, hp = true;
      if (periodic) {
        im = ((im % L) + L) % L;
        ip = ip % L;
      } else {
        hm = im >= 0;
        hp = ip < L;
      }
      const double k1 = hm ? a[i] / b[im] : 0.0;
      const double k2 = hp ? c[i] / b[ip] : 0.0;
      na[i] = hm ? -k1 * a[im] : 0.0;
      nc[i] = hp ? -k2 * c[ip] : 0.0;
      nb[i] = b[i] - (hm ? k1 * c[im] : 0.0) - (hp ? k2 * a[ip] : 0.0);
      t[(size_t)st * L + i] = k1;
      t[(size_t)(steps + st) * L + i] = k2;
    }
    a.swap(na);
    b.swap(nb);
    c.swap(nc);
  }
  for (int i = 0; i < L; ++i) t[(size_t)2 * steps * L + i] = 1.0 / b[i];
  append_band_header(t, L, steps);
  return t;
}

// Band header of a PCR table (read by the LDS line tiles): for every step the factors of
// rows away from the line ends are bit-identical, so kernels use two constants there; per
// step st: {k1, k2, first row, last row} of the band around the middle row, then
// {binv, 0, lo, hi}
void append_band_header(std::vector<double>& t, int L, int steps) {
  const size_t h0 = t.size();
  t.resize(h0 + 4 * (size_t)(steps + 1), 0.0);
  const int mid = L / 2;
  for (int st = 0; st <= steps; ++st) {
    const double* r1 = t.data() + (st < steps ? (size_t)st * L : (size_t)2 * steps * L);
    const double* r2 = st < steps ? t.data() + (size_t)(steps + st) * L : nullptr;
    auto same = [&](int i) { return r1[i] == r1[mid] && (!r2 || r2[i] == r2[mid]); };
    int lo = mid, hi = mid;
    while (lo > 0 && same(lo - 1)) --lo;
    while (hi < L - 1 && same(hi + 1)) ++hi;
    double* hd = t.data() + h0 + 4 * (size_t)st;
    hd[0] = r1[mid];
    hd[1] = r2 ? r2[mid] : 0.0;
    hd[2] = lo;
    hd[3] = hi;
  }
}

// Right-hand-side weights of the tenth-order implicit filter: the maximal-order member has
// T(w) = 1 - (1 - 2 alpha) sin^10(w/2) / (1 + 2 alpha cos w); with
// sin^10(w/2) = (252 - 420 cos w + 240 cos 2w - 90 cos 3w + 20 cos 4w - 2 cos 5w) / 1024
// the numerator sum_k a_k cos(k w) gives a_k directly.
// Tables of k_filter_seg for lines of n unknowns (see k_compact.hip): the forward factors
// cp_i, 1 / pivot_i of the segment system [a, 1, a] (rows in order, the same for every
// segment length), the responses u = T^{-1} e_1 and v = T^{-1} e_L for the two segment
// lengths base and base + 1, and the LU factors (no pivoting) of the joint matrix of the
// segments' first and last unknowns; layout fseg_offsets() of lgbr_kernels.h.
std::vector<double> fseg_table(int n, double al, bool periodic) {
  const int LM = lg::FSEG_LM, M2 = 2 * lg::FSEG_SMAX, S = lg::fseg_count(n);
  const int base = n / S, extra = n % S;
  std::vector<double> t(lg::FSEG_TABLE, 0.0);
  double* tcp = t.data() + lg::FSEG_CP;
  double* tinv = t.data() + lg::FSEG_INV;
  double c = 0.0;
  for (int i = 0; i < base + 1 && i <= LM; ++i) {
    const double den = 1.0 - (i > 0 ? al * c : 0.0);
    tinv[i] = 1.0 / den;
    c = al / den;
    tcp[i] = c;
  }
  for (int which = 0; which < 2; ++which)
    for (int uv = 0; uv < 2; ++uv) {
      const int L = base + which;
      if (L > LM) continue;
      double* out = t.data() + (uv == 0 ? lg::FSEG_U : lg::FSEG_V) + which * (LM + 1);
      double prev = 0.0;
      for (int i = 0; i < L; ++i) {
        const double rhs = uv == 0 ? (i == 0 ? 1.0 : 0.0) : (i == L - 1 ? 1.0 : 0.0);
        prev = (rhs - (i > 0 ? al * prev : 0.0)) * tinv[i];
        out[i] = prev;
      }
      double y = out[L - 1];
      for (int i = L - 2; i >= 0; --i) {
        y = out[i] - tcp[i] * y;
        out[i] = y;
      }
    }
  double* lu = t.data() + lg::FSEG_LU;
  const int m = 2 * S;
  if (S > lg::FSEG_SMAX) return t;
  for (int r = 0; r < m; ++r) lu[r * M2 + r] = 1.0;
  for (int sg = 0; sg < S; ++sg) {
    const int wl = sg < extra ? 1 : 0, Ls = base + wl;
    const double* u = t.data() + lg::FSEG_U + wl * (LM + 1);
    const double* v = t.data() + lg::FSEG_V + wl * (LM + 1);
    const int sp = sg - 1, sn = sg + 1;
    const int cpv = 2 * ((sp + S) % S) + 1, cnv = 2 * (sn % S);   // columns of B_{s-1}, A_{s+1}
    if (periodic || sp >= 0) {
      lu[(2 * sg) * M2 + cpv] += al * u[0];
      lu[(2 * sg + 1) * M2 + cpv] += al * u[Ls - 1];
    }
    if (periodic || sn < S) {
      lu[(2 * sg) * M2 + cnv] += al * v[0];
      lu[(2 * sg + 1) * M2 + cnv] += al * v[Ls - 1];
    }
  }
  for (int k = 0; k < m; ++k)
    for (int r = k + 1; r < m; ++r) {
      const double f = lu[r * M2 + k] / lu[k * M2 + k];
      lu[r * M2 + k] = f;
      for (int cc = k + 1; cc < m; ++cc) lu[r * M2 + cc] -= f * lu[k * M2 + cc];
    }
  return t;
}

// The partition solve of the LAD-C6 gradients along xi (k_grad_part) solves the constant
// [1/3, 1, 1/3] system T of the M unknowns between the end rows and corrects for the 1/4
// neighbours of the first and last rows: z_0 = T^{-1} e_0 (entries 0..63; the rest fall
// below 1e-26 of the first) and (I - W)^{-1}, W = [[z_0[1], z_M[1]], [z_0[M-2], z_M[M-2]]] / 12
// with z_M the mirror image of z_0.
std::vector<double> c6_grad_woodbury_table(int M) {
  const double a = 1.0 / 3.0;
  std::vector<double> cp(M), z(M);
  double den = 1.0;
  z[0] = 1.0;   // forward elimination of e_0
  cp[0] = a;
  for (int i = 1; i < M; ++i) {
    den = 1.0 - a * cp[i - 1];
    cp[i] = a / den;
    z[i] = (0.0 - a * z[i - 1]) / den;
  }
  for (int i = M - 2; i >= 0; --i) z[i] = z[i] - cp[i] * z[i + 1];
  std::vector<double> t(68, 0.0);
  for (int i = 0; i < 64; ++i) t[i] = z[i];
  const double w00 = z[1] / 12.0, w01 = z[M - 2] / 12.0;   // z_M[1] = z_0[M-2], z_M[M-2] = z_0[1]
  const double m00 = 1.0 - w00, m01 = -w01, m10 = -w01, m11 = 1.0 - w00;
  const double det = m00 * m11 - m01 * m10;
  t[64] = m11 / det;
  t[65] = -m01 / det;
  t[66] = -m10 / det;
  t[67] = m00 / det;
  return t;
}

void filter_weights(double al, double a[6]) {
  const double e = (1.0 - 2.0 * al) / 1024.0;
  a[0] = 1.0 - 252.0 * e;
  a[1] = 2.0 * al + 420.0 * e;
  a[2] = -240.0 * e;
  a[3] = 90.0 * e;
  a[4] = -20.0 * e;
  a[5] = 2.0 * e;
}

// PCR steps that leave couplings below 1e-22 of the diagonal: the eliminated couplings of
// [alpha, 1, alpha] shrink as r^(2^k), r = (1 - sqrt(1 - 4 alpha^2)) / (2 alpha)
int filter_pcr_steps(double al) {
  if (!(al > 0.0)) return 1;
  const double r = (1.0 - std::sqrt(1.0 - 4.0 * al * al)) / (2.0 * al);
  int k = 1;
  while (k < 12 && std::pow(r, std::ldexp(1.0, k)) > 1e-22) ++k;
  return k;
}

void fill_launch(Launch& L, const Prob& P) {
  for (int d = 0; d < P.ndim; ++d) {
    // mirror of use_pcr() in k_grad.hip
    int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
    long long nlines = (long long)P.N[o1] * P.N[o2];
    bool periodic = P.bc[d][0] == LG_BC_PERIODIC;
    int Lline = periodic ? P.n[d] : P.N[d];
    bool pcr = !(P.N[d] > 4096 || (periodic && Lline < (2 << lg::LG_PCR_STEPS))) &&
               (d == 0 || 5 * nlines < 131072);
    if (pcr) L.pcr_dir[d] = 1;
    else L.thomas_dir[d] = 1;
    if (P.grad_c4) {
      if (lg::c4_part_use(P, d, L.tile_mask)) L.c4part = 1;
      else if (lg::tile_use(P, d, lg::TK_GRAD4, L.tile_mask)) L.ctile[lg::TK_GRAD4][d] = 1;
      else if (lg::c4_seg_use(P, d, L.tile_mask))
        L.c4seg[d] = std::max(L.c4seg[d], lg::fseg_count(lg::c4_seg_unknowns(P, d)));
      else if (pcr) L.c4_rest_pcr[d] = 1;
      else L.c4_rest_thomas[d] = 1;
    }
    if (periodic && P.n[d] < 128) L.has_short_periodic = 1;
    if (P.bc[d][0] == LG_BC_FIXED || P.bc[d][1] == LG_BC_FIXED) L.has_fixed = 1;
    if (P.lad_c6 || P.falpha < 0.5) {
      for (int k = 0; k < 3; ++k) {
        if (k == lg::TK_FILTER ? !(P.falpha < 0.5) : !P.lad_c6) continue;
        if (k == lg::TK_FILTER && lg::filt_part_use(P, d, L.tile_mask)) {
          L.fpart = 1;
          continue;
        }
        if (k == lg::TK_GRAD6 && lg::c6g_part_use(P, d, L.tile_mask)) {
          L.c6gpart = 1;
          continue;
        }
        if (k == lg::TK_FACES && lg::c6f_part_use(P, d, L.tile_mask)) {
          L.c6fpart = 1;
          continue;
        }
        if (k == lg::TK_GRAD6 && lg::c6g_seg_use(P, d, L.tile_mask)) {
          L.c6gseg[d] = std::max(L.c6gseg[d], lg::fseg_count(P.n[d]));
          continue;
        }
        if (k == lg::TK_FACES && lg::c6f_seg_use(P, d, L.tile_mask)) {
          L.c6fseg[d] = std::max(L.c6fseg[d], lg::fseg_count(lg::c6f_seg_unknowns(P, d)));
          continue;
        }
        if (k == lg::TK_FILTER && lg::filt_seg_use(P, d, L.tile_mask)) {
          L.fseg[d] = std::max(L.fseg[d], lg::fseg_count(P.n[d]));
          continue;
        }
        const bool pcr = k == lg::TK_GRAD6 ? lg::c6_grad_pcr(P, d)
                                           : (k == lg::TK_FACES ? lg::c6_face_pcr(P, d) : lg::filt_pcr(P, d));
        if (lg::tile_use(P, d, k, L.tile_mask)) L.ctile[k][d] = 1;
        else (pcr ? L.cpcr : L.cthomas)[k][d] = 1;
      }
    }
  }
  // 32-bit element offsets address every field of the problem (five FP64 planes)
  if (40LL * P.total >= (1LL << 32)) L.o64 = 1;
  if (!(P.ndim == 3 && P.curvilinear && P.met_planar)) L.geo_generic = 1;
  if (!P.viscous) L.inviscid = 1;
  if (P.total % 2 || ((unsigned long long)P.Q | (unsigned long long)P.Us) % 16) L.prim_scalar = 1;
  L.max_fsteps = std::max(L.max_fsteps, P.fsteps);
  L.max_total = std::max<long long>(L.max_total, P.total);
  L.max_cells = std::max<long long>(L.max_cells, (long long)P.n[0] * P.n[1] * P.n[2]);
  for (int d = 0; d < 3; ++d) {
    int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
    L.ghost_work[d] = std::max<long long>(L.ghost_work[d], 2LL * P.g[d] * P.N[o1] * P.N[o2]);
    L.lines[d] = std::max<long long>(L.lines[d], (long long)P.N[o1] * P.N[o2]);
    L.max_N[d] = std::max<long long>(L.max_N[d], P.N[d]);
    L.max_n[d] = std::max<long long>(L.max_n[d], P.n[d]);
    L.sweep_rows[d] = std::max<long long>(L.sweep_rows[d], (long long)P.n[o1] * P.n[o2]);
  }
}

template <typename F>
lg_status dispatch(int precision, F&& f) {
  if (precision == LG_MIXED) f(float(0));
  else f(double(0));
  return last_hip();
}

}  // namespace

// digital-filter inflow helpers
namespace {
// b_i = exp(-pi |i| / n) / sqrt(sum b^2), |i| <= ceil(2 n)
std::vector<double> df_coef(double n) {
  n = std::max(n, 1e-12);
  const int N = (int)std::ceil(2.0 * n);
  std::vector<double> b(2 * N + 1);
  double ss = 0.0;
  for (int i = -N; i <= N; ++i) {
    b[i + N] = std::exp(-M_PI * std::abs(i) / n);
    ss += b[i + N] * b[i + N];
  }
  const double inv = 1.0 / std::sqrt(ss);
  for (double& v : b) v *= inv;
  return b;
}
bool pos_finite(double v) { return v > 0.0 && std::isfinite(v); }
}  // namespace

extern "C" {

lg_status lg_set_allocator(void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* user) {
  if ((alloc == nullptr) != (free_ == nullptr)) return LG_EINVAL;
  g_alloc = alloc;
  g_free = free_;
  g_user = user;
  return LG_OK;
}

const char* lg_strerror(lg_status s) {
  switch (s) {
    case LG_OK: return "ok";
    case LG_EINVAL: return "invalid argument";
    case LG_ENOMEM: return "out of device memory";
    case LG_EHIP: return "HIP runtime error";
    case LG_ENONPHYS: return "non-physical state (rho <= 0, p <= 0 or not finite)";
    case LG_EUNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

lg_status lg_create(lg_ctx** out, const lg_grid* grid, const double* node_metrics, const double* coords,
                    const lg_gas* gas, const lg_opts* opts, void* stream) {
  if (!out || !grid || !gas || !opts) return LG_EINVAL;
  *out = nullptr;
  const lg_grid& G = *grid;
  if (G.ndim < 1 || G.ndim > 3 || G.ng != lg::NG) return LG_EINVAL;
  long long total = 1;
  for (int d = 0; d < 3; ++d) {
    if (d < G.ndim) {
      if (G.n[d] < 5) return LG_EINVAL;
      if (!valid_bc(G.bc[d][0]) || !valid_bc(G.bc[d][1])) return LG_EINVAL;
      if ((G.bc[d][0] == LG_BC_PERIODIC) != (G.bc[d][1] == LG_BC_PERIODIC)) return LG_EINVAL;
      for (int sd = 0; sd < 2; ++sd)
        if (G.bc[d][sd] == LG_BC_NOSLIP_ISOTHERMAL && !(G.wall_T[d][sd] > 0.0 && std::isfinite(G.wall_T[d][sd])))
          return LG_EINVAL;
      if (!G.curvilinear && !(G.h[d] > 0.0)) return LG_EINVAL;
    } else if (G.n[d] != 1) {
      return LG_EINVAL;
    }
    total *= G.n[d] + (d < G.ndim ? 2 * lg::NG : 0);
  }
  if (total * 5 >= (1LL << 31)) return LG_EUNSUPPORTED;
  if (G.curvilinear && (!node_metrics || !coords)) return LG_EINVAL;
  if (!(gas->gamma > 1.0)) return LG_EINVAL;
  if (gas->viscous && !(gas->Re > 0.0 && gas->Pr > 0.0 && gas->Mref > 0.0)) return LG_EINVAL;
  if (opts->grad != LG_GRAD_E6 && opts->grad != LG_GRAD_C4) return LG_EINVAL;
  if (opts->precision != LG_FP64 && opts->precision != LG_MIXED) return LG_EINVAL;
  if (opts->hybrid_mode != LG_HYB_PERCELL && opts->hybrid_mode != LG_HYB_GLOBAL) return LG_EINVAL;
  if (opts->dilate < 0 || opts->dilate > 4 || opts->seg < 0) return LG_EINVAL;
  if (!(opts->cfl > 0.0)) return LG_EINVAL;
  if (opts->lad_scheme != LG_LAD_E4 && opts->lad_scheme != LG_LAD_C6) return LG_EINVAL;
  if (opts->time_scheme != LG_RK3 && opts->time_scheme != LG_RK4) return LG_EINVAL;
  if (!(opts->filter_alpha >= 0.0 && opts->filter_alpha <= 0.5)) return LG_EINVAL;

  lg_ctx* c = new (std::nothrow) lg_ctx();
  if (!c) return LG_ENOMEM;
  c->stream = static_cast<hipStream_t>(stream);
  Prob& P = c->hp;
  std::memset(&P, 0, sizeof(P));
  P.ndim = G.ndim;
  for (int d = 0; d < 3; ++d) {
    P.n[d] = G.n[d];
    P.g[d] = d < G.ndim ? lg::NG : 0;
    P.N[d] = P.n[d] + 2 * P.g[d];
    P.bc[d][0] = d < G.ndim ? G.bc[d][0] : LG_BC_TRANSMISSIVE;
    P.bc[d][1] = d < G.ndim ? G.bc[d][1] : LG_BC_TRANSMISSIVE;
    P.wall_T[d][0] = G.wall_T[d][0];
    P.wall_T[d][1] = G.wall_T[d][1];
    P.h[d] = G.h[d];
  }
  P.s[0] = 1;
  P.s[1] = P.N[0];
  P.s[2] = P.N[0] * P.N[1];
  P.total = (int)total;
  P.curvilinear = G.curvilinear;
  P.cm[0] = G.h[1] * G.h[2];
  P.cm[4] = G.h[0] * G.h[2];
  P.cm[8] = G.h[0] * G.h[1];
  P.cm[9] = 1.0 / (G.h[0] * G.h[1] * G.h[2]);
  P.gamma = gas->gamma;
  P.Re = gas->Re;
  P.Pr = gas->Pr;
  P.Mref = gas->Mref;
  P.suth = gas->suth;
  P.viscous = gas->viscous;
  P.omega_thr = opts->omega_thr;
  P.mp_eps = opts->mp_eps;
  P.mp_alpha = opts->mp_alpha;
  P.C_mu = opts->C_mu;
  P.C_beta = opts->C_beta;
  P.C_kappa = opts->C_kappa;
  P.rho_thr = opts->rho_thr;
  P.p_thr = opts->p_thr;
  P.cfl = opts->cfl;
  P.dilate = opts->dilate;
  P.grad_c4 = opts->grad == LG_GRAD_C4;
  const int c6 = opts->lad_scheme == LG_LAD_C6;
  P.lad_c6 = c6;
  P.falpha = opts->filter_alpha;
  const int filt = P.falpha < 0.5;
  filter_weights(P.falpha, P.fcoef);
  P.fsteps = filt ? filter_pcr_steps(P.falpha) : 0;
  c->cfg = Cfg{G.ndim, opts->precision, opts->grad, opts->hybrid_mode, gas->viscous, opts->dilate, c6, filt,
               P.falpha, opts->filter_every_stage ? 1 : 0, opts->time_scheme == LG_RK4 ? 1 : 0};

  const size_t T = (size_t)total;
  const size_t rs = opts->precision == LG_MIXED ? sizeof(float) : sizeof(double);
  bool ok = true;
  auto A = [&](size_t bytes) {
    void* p = c->alloc(bytes);
    if (!p) ok = false;
    return p;
  };
  P.W = A(5 * T * rs);
  for (int d = 0; d < G.ndim; ++d) P.G[d] = A(5 * T * rs);
  if (opts->grad == LG_GRAD_C4 || c6 || filt) P.T64 = static_cast<double*>(A(5 * T * sizeof(double)));
  P.Om = A(T * rs);
  P.f = static_cast<uint8_t*>(A(T));
  P.ft = static_cast<uint8_t*>(A(T));
  P.ftmp = static_cast<uint8_t*>(A(T));
  P.fg = static_cast<uint8_t*>(A(T));
  for (int d = 0; d < G.ndim; ++d) {
    int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
    P.llist[d] = static_cast<int*>(A(sizeof(int) * (size_t)P.N[o1] * P.N[o2]));
  }
  P.S3 = A(2 * T * rs);
  P.CA = A(3 * T * rs);
  P.CB = A(3 * T * rs);
  for (int d = 0; d < G.ndim; ++d) P.FL[d] = A(5 * T * rs);
  if (gas->viscous)
    for (int d = 0; d < G.ndim; ++d) P.FV[d] = A(5 * T * rs);
  P.Us = static_cast<double*>(A(5 * T * sizeof(double)));
  P.dQ = static_cast<double*>(A(5 * T * sizeof(double)));
  if (opts->time_scheme == LG_RK4) P.acc = static_cast<double*>(A(5 * T * sizeof(double)));
  if (opts->hybrid_mode == LG_HYB_PERCELL) {   // the compacted C-GBR interface queue and fluxes
    P.gq = static_cast<int*>(A(3 * T * sizeof(int)));
    for (int d = 0; d < G.ndim; ++d) P.FG[d] = A(5 * T * rs);
  }
  double* scal = static_cast<double*>(A(16 * sizeof(double)));
  if (!ok) {
    lg_destroy(c);
    return LG_ENOMEM;
  }
  P.dt = scal;
  P.t = scal + 1;
  P.smax = reinterpret_cast<unsigned long long*>(scal + 2);
  P.status = static_cast<int*>(A(lg::STATUS_SLOTS * lg::STATUS_STRIDE * sizeof(int)));
  if (!ok) {
    lg_destroy(c);
    return LG_ENOMEM;
  }
  P.any_flag = reinterpret_cast<int*>(scal + 4);
  P.lcount = reinterpret_cast<int*>(scal + 5);   // three ints
  P.sw = reinterpret_cast<unsigned*>(scal + 7);   // two counters
  P.all_flag = reinterpret_cast<int*>(scal + 8);
  P.gcount = reinterpret_cast<int*>(scal + 9);    // three ints
  P.t_end = 0.0;
  P.met_T = P.total;
  if (G.curvilinear) {
    P.coords = coords;
    // A grid whose metrics and grid factors do not vary along zeta (a 2D section extruded
    // spanwise) keeps one plane of them: the stencil kernels then read no metric bytes per
    // node.  Deviations up to 1e-12 of the plane's values (rounding of the extrusion) are
    // accepted.
    if (G.ndim == 3) {
      unsigned long long* dbits = reinterpret_cast<unsigned long long*>(scal + 7);
      unsigned long long bits = 0;
      if (hipMemcpy(dbits, &bits, sizeof(bits), hipMemcpyHostToDevice) != hipSuccess) {
        lg_destroy(c);
        return LG_EHIP;
      }
      lg::launch_planar_dev(P.N[0], P.N[1], P.N[2], lg::NG, node_metrics, coords, dbits, c->stream);
      if (hipMemcpyAsync(&bits, dbits, sizeof(bits), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
          hipStreamSynchronize(c->stream) != hipSuccess) {
        lg_destroy(c);
        return LG_EHIP;
      }
      double dev;
      std::memcpy(&dev, &bits, sizeof(dev));
      P.met_planar = dev <= 1e-12 ? 1 : 0;
    }
    const size_t MT = P.met_planar ? (size_t)P.s[2] : T;
    P.met_T = (int)MT;
    if (P.met_planar) {
      double* m64 = static_cast<double*>(A(10 * MT * sizeof(double)));
      if (!ok) {
        lg_destroy(c);
        return LG_ENOMEM;
      }
      for (int cc = 0; cc < 10; ++cc)
        if (hipMemcpyAsync(m64 + cc * MT, node_metrics + cc * T + (size_t)lg::NG * MT, MT * sizeof(double),
                           hipMemcpyDeviceToDevice, c->stream) != hipSuccess) {
          lg_destroy(c);
          return LG_EHIP;
        }
      P.M64 = m64;
    } else {
      P.M64 = node_metrics;
    }
    if (opts->precision == LG_MIXED) {
      float* mr = static_cast<float*>(A(10 * MT * sizeof(float)));
      if (!ok) {
        lg_destroy(c);
        return LG_ENOMEM;
      }
      lg::launch_convert<float>(P.M64, mr, 10 * MT, c->stream);
      P.MR = mr;
    } else {
      P.MR = P.M64;
    }
    P.GX = A(9 * MT * rs);
    if (!ok) {
      lg_destroy(c);
      return LG_ENOMEM;
    }
  }
  if (opts->grad == LG_GRAD_C4) {
    for (int d = 0; d < G.ndim; ++d) {
      std::vector<double> tab = P.bc[d][0] == LG_BC_PERIODIC ? cyclic_table(P.n[d], 0.25) : tri_bounded(P.N[d]);
      double* dt = static_cast<double*>(A(tab.size() * sizeof(double)));
      if (!ok) {
        lg_destroy(c);
        return LG_ENOMEM;
      }
      if (hipMemcpy(dt, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        lg_destroy(c);
        return LG_EHIP;
      }
      P.tri[d] = dt;
      std::vector<double> pt = pcr_table(P.bc[d][0] == LG_BC_PERIODIC ? P.n[d] : P.N[d],
                                         P.bc[d][0] == LG_BC_PERIODIC, lg::LG_PCR_STEPS);
      double* pd = static_cast<double*>(A(pt.size() * sizeof(double)));
      if (!ok || hipMemcpy(pd, pt.data(), pt.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        lg_destroy(c);
        return ok ? LG_EHIP : LG_ENOMEM;
      }
      P.pcr[d] = pd;
      const bool periodic = P.bc[d][0] == LG_BC_PERIODIC;
      const int m = periodic ? P.n[d] : P.N[d] - 2;   // unknowns (c4_seg_unknowns)
      if (d > 0 && lg::fseg_count(m) <= lg::FSEG_SMAX && m >= 16) {
        const std::vector<double> cs = fseg_table(m, 0.25, periodic);
        double* t3 = static_cast<double*>(A(cs.size() * sizeof(double)));
        if (!ok || hipMemcpy(t3, cs.data(), cs.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
          lg_destroy(c);
          return ok ? LG_EHIP : LG_ENOMEM;
        }
        P.c4segt[d] = t3;
      }
    }
  }
  if (c6) {
    // factor tables of the LAD-C6 systems (layouts in k_compact.hip)
    auto upload = [&](const std::vector<double>& v) -> const double* {
      double* p = static_cast<double*>(A(v.size() * sizeof(double)));
      if (!ok) return nullptr;
      if (hipMemcpy(p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        ok = false;
        return nullptr;
      }
      return p;
    };
    const double a3 = 1.0 / 3.0;
    for (int d = 0; d < G.ndim && ok; ++d) {
      const bool periodic = P.bc[d][0] == LG_BC_PERIODIC;
      const int n = P.n[d], N = P.N[d];
      // gradients: all N nodes, one-sided end rows, C4 rows next to them
      std::vector<double> ga(N, a3), gc(N, a3);
      ga[0] = gc[0] = ga[N - 1] = gc[N - 1] = 0.0;
      ga[1] = gc[1] = ga[N - 2] = gc[N - 2] = 0.25;
      std::vector<double> pa(n, a3), pc(n, a3);   // cyclic rows
      P.tri6[d] = upload(periodic ? cyclic_table(n, a3) : thomas_table(ga, gc));
      P.pcr6[d] = upload(periodic ? pcr_table_ac(pa, pc, true, lg::LG_PCR_STEPS)
                                  : pcr_table_ac(ga, gc, false, lg::LG_PCR_STEPS));
      // interface fluxes: n - 1 interior faces between I4 boundary faces, or n cyclic faces
      std::vector<double> fa(n - 1, a3), fc(n - 1, a3);
      fa[0] = 0.0;
      fc[n - 2] = 0.0;
      P.trc[d] = upload(periodic ? cyclic_table(n, a3) : thomas_table(fa, fc));
      P.pcrc[d] = upload(periodic ? pcr_table_ac(pa, pc, true, lg::LG_PCR_STEPS)
                                  : pcr_table_ac(fa, fc, false, lg::LG_PCR_STEPS));
      if (d == 0 && !periodic && N - 2 >= 128 && N - 2 <= 2048) P.c6gz = upload(c6_grad_woodbury_table(N - 2));
      if (d > 0 && periodic && lg::fseg_count(n) <= lg::C6FSEG_SMAX && n >= 16)
        P.c6gsegt[d] = upload(fseg_table(n, a3, true));
      const int mf = periodic ? n : n - 1;   // faces solved (c6f_seg_unknowns)
      if (d > 0 && lg::fseg_count(mf) <= lg::C6FSEG_SMAX && mf >= 16) P.c6fsegt[d] = upload(fseg_table(mf, a3, periodic));
    }
    if (!ok) {
      lg_destroy(c);
      return LG_ENOMEM;
    }
  }
  if (filt) {
    // tables of the implicit filter (every LAD phase ends with it, Alg. 1)
    for (int d = 0; d < G.ndim && ok; ++d) {
      const bool periodic = P.bc[d][0] == LG_BC_PERIODIC;
      const int n = P.n[d];
      const double al = P.falpha;
      std::vector<double> ka(n, al), kc(n, al);
      std::vector<double> qa(n, al), qc(n, al);
      ka[0] = 0.0;
      kc[n - 1] = 0.0;
      const std::vector<double> tri = periodic ? cyclic_table(n, al) : thomas_table(ka, kc);
      const std::vector<double> pcr = pcr_table_ac(periodic ? qa : ka, periodic ? qc : kc, periodic, P.fsteps);
      double* t1 = static_cast<double*>(A(tri.size() * sizeof(double)));
      double* t2 = static_cast<double*>(A(pcr.size() * sizeof(double)));
      if (!ok || hipMemcpy(t1, tri.data(), tri.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(t2, pcr.data(), pcr.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        lg_destroy(c);
        return ok ? LG_EHIP : LG_ENOMEM;
      }
      P.trf[d] = t1;
      P.pcrf[d] = t2;
      if (d > 0 && lg::fseg_count(n) <= lg::FSEG_SMAX && n >= 16) {
        const std::vector<double> fs = fseg_table(n, al, periodic);
        double* t3 = static_cast<double*>(A(fs.size() * sizeof(double)));
        if (!ok || hipMemcpy(t3, fs.data(), fs.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
          lg_destroy(c);
          return ok ? LG_EHIP : LG_ENOMEM;
        }
        P.fsegt[d] = t3;
      }
    }
    if (!ok) {
      lg_destroy(c);
      return LG_ENOMEM;
    }
  }
  c->dp = static_cast<Prob*>(A(sizeof(Prob)));
  if (!ok) {
    lg_destroy(c);
    return LG_ENOMEM;
  }
  if (hipMemcpy(c->dp, &P, sizeof(Prob), hipMemcpyHostToDevice) != hipSuccess) {
    lg_destroy(c);
    return LG_EHIP;
  }
  // zero the device scalars and status slots with kernel-free synchronous copies (setup only)
  double zeros[16] = {0};
  std::vector<int> zslots(lg::STATUS_SLOTS * lg::STATUS_STRIDE, 0);
  if (hipMemcpy(scal, zeros, sizeof(zeros), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P.status, zslots.data(), zslots.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    lg_destroy(c);
    return LG_EHIP;
  }
  std::memset(&c->L, 0, sizeof(Launch));
  c->L.probs = c->dp;
  c->L.nprob = 1;
  c->L.stream = c->stream;
  c->L.ndim = G.ndim;
  c->L.seg = opts->seg;
  c->L.tile_mask = lg::TILE_MASK_DEFAULT;
  fill_launch(c->L, P);
  if (G.curvilinear) {
    if (dispatch(opts->precision, [&](auto r) { lg::launch_lad_geometry<decltype(r)>(c->L); }) != LG_OK) {
      lg_destroy(c);
      return LG_EHIP;
    }
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) {
    lg_destroy(c);
    return LG_EHIP;
  }
  *out = c;
  return LG_OK;
}

static void prof_release(lg_ctx* c) {
  if (c->prof.ev) {
    for (int i = 0; i < 2 * c->prof.cap; ++i) (void)hipEventDestroy(c->prof.ev[i]);
    delete[] c->prof.ev;
    delete[] c->prof.cls;
  }
  c->prof = lg::Prof{};
  c->L.prof = nullptr;
}

lg_status lg_prof_start(lg_ctx* c, int kernel_class, int max_launches) {
  if (!c || max_launches < 1 || kernel_class < -1 || kernel_class >= lg::KC_COUNT) return LG_EINVAL;
  prof_release(c);
  c->prof.ev = new (std::nothrow) hipEvent_t[2 * max_launches];
  c->prof.cls = new (std::nothrow) int[max_launches];
  if (!c->prof.ev || !c->prof.cls) return LG_ENOMEM;
  for (int i = 0; i < 2 * max_launches; ++i)
    if (hipEventCreate(&c->prof.ev[i]) != hipSuccess) {
      c->prof.cap = i / 2;
      prof_release(c);
      return LG_EHIP;
    }
  c->prof.cap = max_launches;
  c->prof.n = 0;
  c->prof.target = kernel_class;
  c->prof.enabled = 1;
  c->L.prof = &c->prof;
  return LG_OK;
}

lg_status lg_prof_stop(lg_ctx* c, double* ms, int* launches) {
  return lg_prof_stop_launches(c, ms, launches, nullptr, nullptr, 0, nullptr);
}

lg_status lg_prof_stop_launches(lg_ctx* c, double* ms, int* launches, float* each_ms, int* each_class, int cap,
                                int* n_out) {
  if (!c || !ms || !launches || cap < 0 || (cap > 0 && (!each_ms || !each_class))) return LG_EINVAL;
  if (n_out) *n_out = 0;
  for (int k = 0; k < lg::KC_COUNT; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  if (!c->prof.ev) return LG_EINVAL;
  lg_status st = hipStreamSynchronize(c->stream) == hipSuccess ? LG_OK : LG_EHIP;
  for (int i = 0; i < c->prof.n && st == LG_OK; ++i) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, c->prof.ev[2 * i], c->prof.ev[2 * i + 1]) != hipSuccess) {
      st = LG_EHIP;
      break;
    }
    ms[c->prof.cls[i]] += t;
    launches[c->prof.cls[i]] += 1;
    if (i < cap) {
      each_ms[i] = t;
      each_class[i] = c->prof.cls[i];
      if (n_out) *n_out = i + 1;
    }
  }
  prof_release(c);
  return st;
}

void lg_destroy(lg_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  prof_release(c);
  for (void* p : c->allocs) dev_free(p);
  delete c;
}

size_t lg_workspace_bytes(const lg_ctx* c) { return c ? c->ws_bytes : 0; }

int lg_metrics_planar(const lg_ctx* c) { return c ? c->hp.met_planar : -1; }

lg_status lg_metrics_from_coords(const lg_grid* grid, const double* coords, double* node_metrics, void* stream) {
  if (!grid || !coords || !node_metrics) return LG_EINVAL;
  if (grid->ndim < 1 || grid->ndim > 3 || grid->ng != lg::NG) return LG_EINVAL;
  int N[3];
  for (int d = 0; d < 3; ++d) {
    if (d >= grid->ndim && grid->n[d] != 1) return LG_EINVAL;
    if (d < grid->ndim && grid->n[d] < 5) return LG_EINVAL;
    N[d] = grid->n[d] + (d < grid->ndim ? 2 * lg::NG : 0);
  }
  size_t total = (size_t)N[0] * N[1] * N[2];
  double* scratch = nullptr;
  if (hipMalloc(&scratch, 9 * total * sizeof(double)) != hipSuccess) return LG_ENOMEM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  lg::launch_metrics(grid->ndim, N, coords, scratch, node_metrics, s);
  lg_status st = last_hip();
  if (hipStreamSynchronize(s) != hipSuccess) st = LG_EHIP;
  (void)hipFree(scratch);
  return st;
}

static lg_status rhs_common(lg_ctx* c, int scheme, double* Q, double* dQ, const uint8_t* fin, uint8_t* fout) {
  if (!c || !Q || !dQ) return LG_EINVAL;
  StateRef ref{Q, dQ, 0};
  lg_status st = dispatch(c->cfg.precision, [&](auto r) {
    using R = decltype(r);
    enqueue_rhs<R>(c->L, c->cfg, scheme, ref, fin);
  });
  if (st == LG_OK && fout) {
    if (hipMemcpyAsync(fout, c->hp.f, (size_t)c->hp.total, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
      return LG_EHIP;
  }
  return st;
}

lg_status cgbr_rhs(lg_ctx* c, double* Q, double* dQdt) { return rhs_common(c, LG_SCHEME_CGBR, Q, dQdt, nullptr, nullptr); }
lg_status lad_rhs(lg_ctx* c, double* Q, double* dQdt) { return rhs_common(c, LG_SCHEME_LAD, Q, dQdt, nullptr, nullptr); }
lg_status hybrid_rhs(lg_ctx* c, double* Q, double* dQdt, const uint8_t* flags_in, uint8_t* flags_out) {
  if (c && c->cfg.lad_c6) return LG_EUNSUPPORTED;
  return rhs_common(c, LG_SCHEME_HYBRID, Q, dQdt, flags_in, flags_out);
}

lg_status lad_filter(lg_ctx* c, double* Q) {
  if (!c || !Q) return LG_EINVAL;
  if (!c->cfg.filter) return LG_EUNSUPPORTED;
  for (int d = 0; d < c->cfg.ndim; ++d) lg::launch_filter(c->L, StateRef{Q, nullptr, 0}, d, lg::FILT_ALL);
  return last_hip();
}

lg_status rk3_step(lg_ctx* c, int scheme, double* Q, double t_end, double* t_inout) {
  if (!c || !Q || !t_inout) return LG_EINVAL;
  if (scheme < LG_SCHEME_CGBR || scheme > LG_SCHEME_HYBRID) return LG_EINVAL;
  if (scheme == LG_SCHEME_HYBRID && c->cfg.lad_c6) return LG_EUNSUPPORTED;
  if (c->cfg.rk4 && scheme != LG_SCHEME_LAD) return LG_EUNSUPPORTED;
  return dispatch(c->cfg.precision, [&](auto r) {
    using R = decltype(r);
    if (c->cfg.rk4) enqueue_rk4<R>(c->L, c->cfg, scheme, Q, t_inout, t_end);
    else enqueue_rk3<R>(c->L, c->cfg, scheme, Q, t_inout, t_end);
  });
}

lg_status lg_rk3_stage(lg_ctx* c, int scheme, int stage, const double* Un, double* Us, double dt) {
  if (!c || !Un || !Us || stage < 0 || stage > 2) return LG_EINVAL;
  if (scheme < LG_SCHEME_CGBR || scheme > LG_SCHEME_HYBRID) return LG_EINVAL;
  if (scheme == LG_SCHEME_HYBRID && c->cfg.lad_c6) return LG_EUNSUPPORTED;
  return dispatch(c->cfg.precision, [&](auto r) {
    using R = decltype(r);
    lg::launch_set_dt(c->L, dt);
    RKRef rr{Un, Us, Us};
    enqueue_rhs<R>(c->L, c->cfg, scheme, StateRef{Us, nullptr, 0}, nullptr, &rr, stage);
  });
}

lg_status lg_compute_dt(lg_ctx* c, const double* Q, double* dt_out) {
  if (!c || !Q || !dt_out) return LG_EINVAL;
  lg::launch_dt(c->L, Q, nullptr, 0.0, 0);
  if (last_hip() != LG_OK) return LG_EHIP;
  if (hipMemcpyAsync(dt_out, c->hp.dt, sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return LG_EHIP;
  return LG_OK;
}

lg_status lg_set_tuning(lg_ctx* c, int seg, int pcr_blocks, int zc) {
  if (!c || seg < 0 || (seg > 0 && (seg < 2 || seg > 64)) || pcr_blocks < 0 ||
      (pcr_blocks > 0 && (pcr_blocks < 256 || pcr_blocks > 65536)) || zc < 0 || zc > 1024)
    return LG_EINVAL;
  c->L.seg = seg;
  c->L.pcr_blocks = pcr_blocks;
  c->L.zc = zc;
  return LG_OK;
}

lg_status lg_set_line_tiles(lg_ctx* c, int mask) {
  if (!c || mask < -1 ||
      mask > (lg::TILE_MASK_ALL | lg::TILE_MASK_FORCE_STRIDED | lg::TILE_MASK_NO_PART | lg::TILE_MASK_NO_SEG))
    return LG_EINVAL;
  c->L.tile_mask = mask < 0 ? lg::TILE_MASK_DEFAULT : mask;
  for (int d = 0; d < 3; ++d) {
    for (int k = 0; k < 3; ++k) c->L.cpcr[k][d] = c->L.cthomas[k][d] = 0;
    for (int k = 0; k < 4; ++k) c->L.ctile[k][d] = 0;
    c->L.c4_rest_pcr[d] = c->L.c4_rest_thomas[d] = 0;
  }
  c->L.fpart = c->L.c4part = c->L.c6fpart = c->L.c6gpart = 0;
  for (int d = 0; d < 3; ++d) c->L.fseg[d] = c->L.c4seg[d] = c->L.c6fseg[d] = c->L.c6gseg[d] = 0;
  fill_launch(c->L, c->hp);
  return LG_OK;
}

int lg_get_line_tiles(const lg_ctx* c) { return c ? c->L.tile_mask : -1; }

lg_status lg_set_generic_access(lg_ctx* c, int generic) {
  if (!c || generic < 0 || generic > 3) return LG_EINVAL;
  c->L.o64 = c->L.prim_scalar = c->L.geo_generic = 0;
  fill_launch(c->L, c->hp);
  if (generic & 1) c->L.o64 = c->L.prim_scalar = 1;
  if (generic & 2) c->L.geo_generic = 1;
  return LG_OK;
}

lg_status lg_set_tile_shape(lg_ctx* c, int zm_width, int line_batch) {
  if (!c || !(zm_width == 0 || zm_width == 32 || zm_width == 64 || zm_width == 128) || line_batch < 0 ||
      line_batch > lg::TILE_MAX_TX)
    return LG_EINVAL;
  c->L.ztx = zm_width;
  c->L.tile_lines = line_batch;
  return LG_OK;
}

lg_status lg_get_tile_shape(const lg_ctx* c, int* zm_width, int* line_batch) {
  if (!c || !zm_width || !line_batch) return LG_EINVAL;
  *zm_width = lg::zm_width(c->L);
  *line_batch = c->L.tile_lines;
  return LG_OK;
}

lg_status lg_get_tuning(const lg_ctx* c, int* seg, int* pcr_blocks, int* zc) {
  if (!c || !seg || !pcr_blocks || !zc) return LG_EINVAL;
  *seg = lg::sweep_seg(c->L, c->cfg.ndim > 1 ? 1 : 0);
  *pcr_blocks = c->L.pcr_blocks > 0 ? c->L.pcr_blocks : 16384;
  *zc = lg::zm_chunk(c->L, 0, 0);
  return LG_OK;
}

lg_status lg_poll_status(lg_ctx* c, int* count) {
  if (!c || !count) return LG_EINVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LG_EHIP;
  std::vector<int> slots(lg::STATUS_SLOTS * lg::STATUS_STRIDE);
  if (hipMemcpy(slots.data(), c->hp.status, slots.size() * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return LG_EHIP;
  long long sum = 0;
  for (int i = 0; i < lg::STATUS_SLOTS; ++i) sum += slots[(size_t)i * lg::STATUS_STRIDE];
  const int v = (int)std::min<long long>(sum, 2147483647LL);
  lg::launch_zero_status(c->L);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LG_EHIP;
  *count = v;
  return v ? LG_ENONPHYS : LG_OK;
}

// ------------------------------------------------------------------ digital-filter inflow
struct lg_df {
  lg_ctx* ctx = nullptr;
  lg::DFDev D{};
  std::vector<void*> allocs;
  long long nrand = 0;
};

void lg_df_destroy(lg_df* f) {
  if (!f) return;
  if (f->ctx) (void)hipStreamSynchronize(f->ctx->stream);
  for (void* p : f->allocs) dev_free(p);
  delete f;
}


lg_status lg_df_create(lg_ctx* c, const lg_df_spec* s, lg_df** out) {
  if (!c || !s || !out) return LG_EINVAL;
  *out = nullptr;
  const Prob& P = c->hp;
  if (P.ndim < 2 || P.bc[0][0] != LG_BC_FIXED) return LG_EINVAL;
  if (s->ny != P.n[1] || s->nz != (P.ndim == 3 ? P.n[2] : 1)) return LG_EINVAL;
  if (!s->dy || !s->y || !s->mean || !s->rey) return LG_EINVAL;
  if (!pos_finite(s->U_ref) || !pos_finite(s->p) || !std::isfinite(s->M_sra) || !std::isfinite(s->y_lim)) return LG_EINVAL;
  if (P.ndim == 3 && !pos_finite(s->dz)) return LG_EINVAL;
  const int ny = s->ny, nz = s->nz;
  for (int q = 0; q < 3; ++q) {
    if (!pos_finite(s->Iy[q][0]) || !pos_finite(s->Iy[q][1]) || !pos_finite(s->Iz[q]) || !pos_finite(s->Ix[q]))
      return LG_EINVAL;
  }
  for (int j = 0; j < ny; ++j) {
    if (!pos_finite(s->dy[j]) || !std::isfinite(s->y[j]) || !pos_finite(s->mean[j])) return LG_EINVAL;
    for (int q = 1; q < 4; ++q)
      if (!std::isfinite(s->mean[q * ny + j])) return LG_EINVAL;
    const double R11 = s->rey[j], R21 = s->rey[ny + j], R22 = s->rey[2 * ny + j], R33 = s->rey[3 * ny + j];
    if (!(R11 >= 0.0) || !(R22 >= 0.0) || !(R33 >= 0.0) || !std::isfinite(R21) || !std::isfinite(R11 + R22 + R33))
      return LG_EINVAL;
  }
  lg_df* f = new (std::nothrow) lg_df();
  if (!f) return LG_ENOMEM;
  f->ctx = c;
  lg::DFDev& D = f->D;
  D.ny = ny;
  D.nz = nz;
  // eta coefficients per component and row (zone by wall distance, local spacing)
  std::vector<std::vector<double>> rowc(3 * (size_t)ny);
  int pad = 0;
  for (int q = 0; q < 3; ++q)
    for (int j = 0; j < ny; ++j) {
      const double I = s->Iy[q][s->y[j] <= s->y_lim ? 0 : 1];
      rowc[(size_t)q * ny + j] = df_coef(I / s->dy[j]);
      pad = std::max(pad, (int)(rowc[(size_t)q * ny + j].size() - 1) / 2);
    }
  D.pad = pad;
  std::vector<double> by(3 * (size_t)ny * (2 * pad + 1), 0.0);
  std::vector<int> nyh(3 * (size_t)ny);
  for (size_t r = 0; r < rowc.size(); ++r) {
    const int h = (int)(rowc[r].size() - 1) / 2;
    nyh[r] = h;
    for (int i = -h; i <= h; ++i) by[r * (2 * pad + 1) + pad + i] = rowc[r][i + h];
  }
  std::vector<std::vector<double>> zc(3);
  int nzmax = 0;
  for (int q = 0; q < 3; ++q) {
    zc[q] = df_coef(s->Iz[q] / (P.ndim == 3 ? s->dz : 1.0));
    D.nzh[q] = (int)(zc[q].size() - 1) / 2;
    nzmax = std::max(nzmax, D.nzh[q]);
  }
  D.nzmax = nzmax;
  std::vector<double> bz(3 * (size_t)(2 * nzmax + 1), 0.0);
  for (int q = 0; q < 3; ++q)
    for (int l = -D.nzh[q]; l <= D.nzh[q]; ++l) bz[(size_t)q * (2 * nzmax + 1) + nzmax + l] = zc[q][l + D.nzh[q]];
  // Cholesky factor of the Reynolds stresses
  std::vector<double> a(4 * (size_t)ny);
  for (int j = 0; j < ny; ++j) {
    const double a11 = std::sqrt(s->rey[j]);
    const double a21 = a11 > 0.0 ? s->rey[ny + j] / a11 : 0.0;
    a[j] = a11;
    a[ny + j] = a21;
    a[2 * ny + j] = std::sqrt(std::max(s->rey[2 * ny + j] - a21 * a21, 0.0));
    a[3 * ny + j] = std::sqrt(s->rey[3 * ny + j]);
  }
  for (int q = 0; q < 3; ++q) D.Tc[q] = s->Ix[q] / s->U_ref;
  D.gm1 = P.gamma - 1.0;
  D.M2 = s->M_sra * s->M_sra;
  D.U_ref = s->U_ref;
  D.p = s->p;
  bool ok = true;
  auto up = [&](const void* src, size_t bytes) -> void* {
    void* d = dev_alloc(bytes);
    if (!d) {
      ok = false;
      return nullptr;
    }
    f->allocs.push_back(d);
    if (src && hipMemcpy(d, src, bytes, hipMemcpyHostToDevice) != hipSuccess) ok = false;
    return d;
  };
  D.by = static_cast<const double*>(up(by.data(), by.size() * sizeof(double)));
  D.nyh = static_cast<const int*>(up(nyh.data(), nyh.size() * sizeof(int)));
  D.bz = static_cast<const double*>(up(bz.data(), bz.size() * sizeof(double)));
  D.a = static_cast<const double*>(up(a.data(), a.size() * sizeof(double)));
  D.mean = static_cast<const double*>(up(s->mean, 4 * (size_t)ny * sizeof(double)));
  const long long rows = ny + 2LL * pad;
  D.rz = static_cast<double*>(up(nullptr, 3 * rows * nz * sizeof(double)));
  D.psi = static_cast<double*>(up(nullptr, 3 * (size_t)ny * nz * sizeof(double)));
  f->nrand = 3 * rows * nz;
  if (!ok) {
    lg_df_destroy(f);
    return LG_ENOMEM;
  }
  *out = f;
  return LG_OK;
}

lg_status lg_df_random_count(const lg_df* f, long long* count) {
  if (!f || !count) return LG_EINVAL;
  *count = f->nrand;
  return LG_OK;
}

lg_status lg_df_update(lg_df* f, const double* rnd, double* Q, double dt, int first) {
  if (!f || !rnd || !Q || !std::isfinite(dt)) return LG_EINVAL;
  lg::launch_df_update(f->D, f->ctx->dp, rnd, Q, dt, first, f->ctx->stream);
  return last_hip();
}

lg_status lg_switch_stats(lg_ctx* c, int* hybrid_stages, int* troubled_stages, int reset) {
  if (!c || !hybrid_stages || !troubled_stages) return LG_EINVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LG_EHIP;
  unsigned v[2] = {0u, 0u};
  if (hipMemcpy(v, c->hp.sw, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return LG_EHIP;
  if (reset) {
    const unsigned z[2] = {0u, 0u};
    if (hipMemcpy(c->hp.sw, z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess) return LG_EHIP;
  }
  *hybrid_stages = (int)v[0];
  *troubled_stages = (int)v[1];
  return LG_OK;
}

lg_status lg_batch_create(lg_batch** out, lg_ctx* const* ctxs, double* const* Q, double* const* t,
                          const double* t_end, int n, int nsteps, int scheme) {
  if (!out || !ctxs || !Q || !t || !t_end || n < 1 || nsteps < 1) return LG_EINVAL;
  if (scheme < LG_SCHEME_CGBR || scheme > LG_SCHEME_HYBRID) return LG_EINVAL;
  *out = nullptr;
  for (int i = 0; i < n; ++i)
    if (!ctxs[i]) return LG_EINVAL;
  const Cfg& c0 = ctxs[0]->cfg;
  if (scheme == LG_SCHEME_HYBRID && c0.lad_c6) return LG_EUNSUPPORTED;
  if (c0.rk4 && scheme != LG_SCHEME_LAD) return LG_EUNSUPPORTED;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i] || !Q[i] || !t[i]) return LG_EINVAL;
    const Cfg& ci = ctxs[i]->cfg;
    if (ci.ndim != c0.ndim || ci.precision != c0.precision || ci.grad != c0.grad ||
        ci.hybrid_mode != c0.hybrid_mode || ci.viscous != c0.viscous || ci.dilate != c0.dilate ||
        ci.lad_c6 != c0.lad_c6 || ci.filter != c0.filter || ci.filter_all != c0.filter_all || ci.rk4 != c0.rk4)
      return LG_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return LG_EINVAL;  // workspaces must not be shared
  }
  lg_batch* b = new (std::nothrow) lg_batch();
  if (!b) return LG_ENOMEM;
  b->cfg = c0;
  b->stream = ctxs[0]->stream;
  b->nsteps = nsteps;
  b->scheme = scheme;
  std::memset(&b->L, 0, sizeof(Launch));
  b->L.nprob = n;
  b->L.ndim = c0.ndim;
  b->L.seg = ctxs[0]->L.seg;
  b->L.pcr_blocks = ctxs[0]->L.pcr_blocks;
  b->L.zc = ctxs[0]->L.zc;
  b->L.ztx = ctxs[0]->L.ztx;
  b->L.tile_lines = ctxs[0]->L.tile_lines;
  b->L.tile_mask = ctxs[0]->L.tile_mask;
  for (int i = 0; i < n; ++i) {
    Prob P = ctxs[i]->hp;
    P.Q = Q[i];
    P.t = t[i];
    P.t_end = t_end[i];
    b->hps.push_back(P);
    fill_launch(b->L, P);
  }
  if (hipMalloc(&b->dps, n * sizeof(Prob)) != hipSuccess) {
    delete b;
    return LG_ENOMEM;
  }
  if (hipMemcpy(b->dps, b->hps.data(), n * sizeof(Prob), hipMemcpyHostToDevice) != hipSuccess) {
    lg_batch_destroy(b);
    return LG_EHIP;
  }
  b->L.probs = b->dps;
  hipStream_t cap;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
    lg_batch_destroy(b);
    return LG_EHIP;
  }
  Launch Lc = b->L;
  Lc.stream = cap;
  lg_status st = LG_OK;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) st = LG_EHIP;
  if (st == LG_OK) {
    for (int s = 0; s < nsteps; ++s) {
      if (c0.rk4) {
        if (c0.precision == LG_MIXED) enqueue_rk4<float>(Lc, c0, scheme, nullptr, nullptr, 0.0);
        else enqueue_rk4<double>(Lc, c0, scheme, nullptr, nullptr, 0.0);
      } else if (c0.precision == LG_MIXED) {
        enqueue_rk3<float>(Lc, c0, scheme, nullptr, nullptr, 0.0);
      } else {
        enqueue_rk3<double>(Lc, c0, scheme, nullptr, nullptr, 0.0);
      }
    }
    if (hipStreamEndCapture(cap, &b->graph) != hipSuccess) st = LG_EHIP;
  }
  if (st == LG_OK && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) st = LG_EHIP;
  (void)hipStreamDestroy(cap);
  if (st != LG_OK) {
    lg_batch_destroy(b);
    return st;
  }
  *out = b;
  return LG_OK;
}

lg_status lg_batch_run(lg_batch* b) {
  if (!b || !b->exec) return LG_EINVAL;
  return hipGraphLaunch(b->exec, b->stream) == hipSuccess ? LG_OK : LG_EHIP;
}

void lg_batch_destroy(lg_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->dps) (void)hipFree(b->dps);
  delete b;
}

}  // extern "C"
