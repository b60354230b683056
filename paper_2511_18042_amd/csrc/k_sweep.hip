// Omega sensor and the interface sweeps of the three right-hand-side forms.
//
// Paper: Sec. 2.3 -- conservative finite difference (fluxes at half nodes, node
// derivative = flux difference); characteristic transformation of the primitives
// with waves acoustic (1,5), entropy (2), shear (3,4); centralised interpolation
// C^C = (C^{L,Lin} + C^{R,Lin}) / 2; selection rule: acoustic -> MP5 where the
// over-barred sensor exceeds 0.01, else the linear (upwind GBR) state; entropy -> MP
// criterion with threshold 1e-20 (central value when it holds, MP5 otherwise); shear
// -> MP5 where the sensor exceeds 0.01, else the central value; curvilinear HLLC with
// Roe-averaged wave speeds and interface metrics interpolated from the nodes.
// Sec. 5 / Alg. 3 -- hybrid: the LAD-E4 interface flux unless the interface touches a
// (dilated) troubled cell.
//
// GBR linear states (gradient-based reconstruction, unit spacing):
//   C^{L,Lin} = C_i + C'_i/2 + C''_i/12,  C^{R,Lin} = C_{i+1} - C'_{i+1}/2 + C''_{i+1}/12,
//   C''_j = 2 (C_{j+1} - 2 C_j + C_{j-1}) - (C'_{j+1} - C'_{j-1}) / 2.
// MP5 = Suresh & Huynh (1997), alpha = 4, beta = 4/3.
// Frozen characteristic state: Roe average of nodes i, i+1; basis n = xi~/|xi~|,
// t1 = normalise(n x e_m) with m = argmin |n_m| (lowest index on ties), t2 = n x t1.
// Omega = pressure switch x Ducros ratio (theta^2 + eps) / (theta^2 + |omega|^2 + eps),
// eps = 1e-32, so that a pressure jump in a flow at rest is still detected; over-bar =
// max over the node and its two neighbours along the sweep; the left state uses node i,
// the right node i+1.
// Interface metrics: I4 of the node metrics.  The flux difference is formed in FP64.
// Positivity of the reconstruction: a side whose state has no positive density and pressure
// falls back to its upwind node's state (the paper prints no safeguard but reports C-GBR
// stable where the limited characteristic reconstruction returns such states).
#include "lgbr_dev.h"
#include "lgbr_kernels.h"

namespace lg {

__device__ __forceinline__ bool sw_skip(const Prob& P, int skip_if_any) {
  return gate_skip(P, skip_if_any);
}

__device__ __forceinline__ bool band(const Prob& P, int idx, int lo, int hi) {
  int p[3] = {idx % P.N[0], (idx / P.N[0]) % P.N[1], idx / (P.N[0] * P.N[1])};
  for (int l = 0; l < P.ndim; ++l)
    if (p[l] < P.g[l] + lo || p[l] >= P.g[l] + P.n[l] + hi) return false;
  return true;
}

// ------------------------------------------------------------------ sensor
template <typename R>
__global__ void __launch_bounds__(256) k_sensor(const Prob* __restrict__ probs, int skip_if_any, int region) {
  const Prob& P = probs[blockIdx.y];
  if (sw_skip(P, skip_if_any)) return;
  const R* W = static_cast<const R*>(P.W);
  R* Om = static_cast<R*>(P.Om);
  const size_t T = P.total;
  const R* p = W + 4 * T;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < P.total; idx += gridDim.x * blockDim.x) {
    if (!band(P, idx, -2, 2)) continue;
    if (region && !P.fg[idx]) continue;
    R phi = R(0);
    for (int l = 0; l < P.ndim; ++l) {
      int s = P.s[l];
      R pp = p[idx + s], p0 = p[idx], pm = p[idx - s];
      R r = fabs(pp - R(2) * p0 + pm) / (pp + R(2) * p0 + pm);
      phi = fmax(phi, r);
    }
    R du[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) du[i][j] = R(0);
    R J = met<R>(P, 9, idx);
    for (int l = 0; l < P.ndim; ++l) {
      const R* G = static_cast<const R*>(P.G[l]);
      for (int j = 0; j < 3; ++j) {
        R m = J * met<R>(P, 3 * l + j, idx);
        for (int i = 0; i < 3; ++i) du[i][j] += m * G[(1 + i) * T + idx];
      }
    }
    R th = du[0][0] + du[1][1] + du[2][2];
    R w1 = du[2][1] - du[1][2], w2 = du[0][2] - du[2][0], w3 = du[1][0] - du[0][1];
    R om2 = w1 * w1 + w2 * w2 + w3 * w3;
    Om[idx] = phi * ((th * th + R(1e-32)) / (th * th + om2 + R(1e-32)));
  }
}

// ------------------------------------------------------------------ pieces of the GBR flux
template <typename R>
__device__ __forceinline__ R mp5(R vm2, R vm1, R v0, R vp1, R vp2, R alpha, R eps) {
  R vor = bdiv(R(2) * vm2 - R(13) * vm1 + R(47) * v0 + R(27) * vp1 - R(3) * vp2, R(60));
  R vmp = v0 + minmod2(vp1 - v0, alpha * (v0 - vm1));
  if ((vor - v0) * (vor - vmp) <= eps) return vor;
  R djm1 = vm2 - R(2) * vm1 + v0;
  R dj = vm1 - R(2) * v0 + vp1;
  R djp1 = v0 - R(2) * vp1 + vp2;
  R dm4p = minmod4(R(4) * dj - djp1, R(4) * djp1 - dj, dj, djp1);
  R dm4m = minmod4(R(4) * dj - djm1, R(4) * djm1 - dj, dj, djm1);
  R vul = v0 + alpha * (v0 - vm1);
  R vav = R(0.5) * (v0 + vp1);
  R vmd = vav - R(0.5) * dm4p;
  R vlc = v0 + R(0.5) * (v0 - vm1) + R(4.0 / 3.0) * dm4m;
  R vmin = fmax(fmin(fmin(v0, vp1), vmd), fmin(fmin(v0, vul), vlc));
  R vmax = fmin(fmax(fmax(v0, vp1), vmd), fmax(fmax(v0, vul), vlc));
  return vor + minmod2(vmin - vor, vmax - vor);
}

template <typename R>
struct Frame {
  R n[3], t1[3], t2[3];
  R k, cb2inv, cb, rb;  // k = rb / (2 cb)
};

template <typename R>
__device__ __forceinline__ void to_char(const Frame<R>& f, R r, R u, R v, R w, R p, R C[5]) {
  R un = f.n[0] * u + f.n[1] * v + f.n[2] * w;
  R pc = bdiv(p, R(2) * f.cb * f.cb);
  C[0] = -f.k * un + pc;
  C[1] = r - bdiv(p, f.cb * f.cb);
  C[2] = f.t1[0] * u + f.t1[1] * v + f.t1[2] * w;
  C[3] = f.t2[0] * u + f.t2[1] * v + f.t2[2] * w;
  C[4] = f.k * un + pc;
}

template <typename R>
__device__ __forceinline__ void from_char(const Frame<R>& f, const R C[5], R Wo[5]) {
  R un = bdiv(f.cb, f.rb) * (C[4] - C[0]);
  Wo[0] = C[0] + C[1] + C[4];
  Wo[1] = f.n[0] * un + f.t1[0] * C[2] + f.t2[0] * C[3];
  Wo[2] = f.n[1] * un + f.t1[1] * C[2] + f.t2[1] * C[3];
  Wo[3] = f.n[2] * un + f.t1[2] * C[2] + f.t2[2] * C[3];
  Wo[4] = f.cb * f.cb * (C[0] + C[4]);
}

template <typename R>
__device__ __forceinline__ void hllc(const R WL[5], const R WR[5], const R xt[3], R gamma, R F[5]) {
  R xn2 = xt[0] * xt[0] + xt[1] * xt[1] + xt[2] * xt[2];
  R xn = sqrt(xn2);
  R rL = WL[0], pL = WL[4], rR = WR[0], pR = WR[4];
  R EL = bdiv(pL, gamma - R(1)) + R(0.5) * rL * (WL[1] * WL[1] + WL[2] * WL[2] + WL[3] * WL[3]);
  R ER = bdiv(pR, gamma - R(1)) + R(0.5) * rR * (WR[1] * WR[1] + WR[2] * WR[2] + WR[3] * WR[3]);
  R HL = bdiv(EL + pL, rL), HR = bdiv(ER + pR, rR);
  R cL = sqrt(bdiv(gamma * pL, rL)), cR = sqrt(bdiv(gamma * pR, rR));
  R UL = xt[0] * WL[1] + xt[1] * WL[2] + xt[2] * WL[3];
  R UR = xt[0] * WR[1] + xt[1] * WR[2] + xt[2] * WR[3];
  R Rr = sqrt(bdiv(rR, rL));
  R ub[3];
  for (int m = 0; m < 3; ++m) ub[m] = bdiv(WL[1 + m] + Rr * WR[1 + m], R(1) + Rr);
  R Hb = bdiv(HL + Rr * HR, R(1) + Rr);
  R cb = sqrt((gamma - R(1)) * (Hb - R(0.5) * (ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2])));
  R Ub = xt[0] * ub[0] + xt[1] * ub[1] + xt[2] * ub[2];
  R SL = fmin(UL - cL * xn, Ub - cb * xn);
  R SR = fmax(UR + cR * xn, Ub + cb * xn);
  R Ss = bdiv(rR * UR * (SR - UR) - rL * UL * (SL - UL) + (pL - pR) * xn2, rR * (SR - UR) - rL * (SL - UL));
  // pick the side whose flux (or star flux) is needed:
  // S_L >= 0 -> F_L; S* >= 0 -> F*_L; S_R > 0 -> F*_R; else F_R
  bool left = (SL >= R(0)) || (Ss >= R(0));
  const R* Wk = left ? WL : WR;
  R rho = left ? rL : rR, p = left ? pL : pR, E = left ? EL : ER, U = left ? UL : UR, S = left ? SL : SR;
  F[0] = rho * U;
  F[1] = rho * Wk[1] * U + xt[0] * p;
  F[2] = rho * Wk[2] * U + xt[1] * p;
  F[3] = rho * Wk[3] * U + xt[2] * p;
  F[4] = (E + p) * U;
  bool star = left ? !(SL >= R(0)) : (SR > R(0));
  if (star) {
    R fac = bdiv(rho * (S - U), S - Ss);
    R Qs[5], Qk[5];
    Qs[0] = fac;
    for (int m = 0; m < 3; ++m) Qs[1 + m] = fac * (Wk[1 + m] + bdiv(xt[m] * (Ss - U), xn2));
    Qs[4] = fac * (bdiv(E, rho) + (Ss - U) * (bdiv(Ss, xn2) + bdiv(p, rho * (S - U))));
    Qk[0] = rho;
    for (int m = 0; m < 3; ++m) Qk[1 + m] = rho * Wk[1 + m];
    Qk[4] = E;
    for (int q = 0; q < 5; ++q) F[q] = F[q] + S * (Qs[q] - Qk[q]);
  }
}

// The inputs of one C-GBR interface flux between nodes i and i + 1 along d: primitives at
// offsets -2 .. 3, their d-gradients, Omega and the node metrics of direction d at -1 .. 2,
// loaded together before the arithmetic.  (A strided sweep that slid this window along its
// line, loading one node per interface, ran no faster on the 1024 x 384 x 128 ramp: its
// extra registers halved the waves per SIMD.)
template <typename R>
struct GbrWin {
  R w[6][5], g[4][5], om[4], m[4][3];
};

template <typename R>
__host__ __device__ __forceinline__ void gbr_load_w(const Prob& P, int id, R out[5]) {
  const R* W = static_cast<const R*>(P.W);
  for (int q = 0; q < 5; ++q) out[q] = W[q * P.total + id];
}

// C3V: the problem is known to be 3D, curvilinear with metrics planar along zeta, and
// viscous (branches on these folded at compile time); false: read from the descriptor.
// id: the node; mid: its index in the metric arrays (met_idx)
template <typename R, bool C3V = false>
__host__ __device__ __forceinline__ void gbr_load_gom(const Prob& P, int d, int id, int mid, R g[5], R& om, R m[3]) {
  const R* G = static_cast<const R*>(P.G[d]);
  for (int q = 0; q < 5; ++q) g[q] = G[q * P.total + id];
  om = (C3V || P.viscous) ? static_cast<const R*>(P.Om)[id] : R(0);
  const R* M = static_cast<const R*>(P.MR);
  for (int c = 0; c < 3; ++c)
    m[c] = (C3V || P.curvilinear) ? M[(size_t)(3 * d + c) * P.met_T + mid] : (R)P.cm[3 * d + c];
}

// Step of the metric index along direction d: the node step, or 0 along zeta where the
// metrics are stored for one plane.  Every node of a window lies in its interface's row
// (all interior and ghost positions of the other two directions), so its metric index is
// the interface node's plus a multiple of this step, without a division.
template <bool C3V = false>
__host__ __device__ __forceinline__ int met_step(const Prob& P, int d) {
  return ((C3V || P.met_planar) && d == 2) ? 0 : P.s[d];
}

// the whole window of the interface between idx and idx + s (mi = met_idx(P, idx))
template <typename R, bool C3V = false>
__host__ __device__ __forceinline__ void gbr_fill(const Prob& P, int d, int idx, int mi, GbrWin<R>& wn) {
  const int s = P.s[d], ms = met_step<C3V>(P, d);
  for (int o = -2; o <= 3; ++o) gbr_load_w(P, idx + o * s, wn.w[o + 2]);
  for (int o = -1; o <= 2; ++o)
    gbr_load_gom<R, C3V>(P, d, idx + o * s, mi + o * ms, wn.g[o + 1], wn.om[o + 1], wn.m[o + 1]);
}

// C-GBR convective flux at the interface between the window's nodes 0 and 1
template <typename R, bool C3V = false>
__device__ __forceinline__ void gbr_flux_win(const Prob& P, const GbrWin<R>& wn, R F[5]) {
  // interface metrics (I4 of node metrics)
  R xt[3];
  for (int c = 0; c < 3; ++c) {
    R a0 = wn.m[0][c], a1 = wn.m[1][c], a2 = wn.m[2][c], a3 = wn.m[3][c];
    xt[c] = bdiv(R(7) * (a1 + a2) - (a0 + a3), R(12));
  }
  Frame<R> fr;
  R xn = sqrt(xt[0] * xt[0] + xt[1] * xt[1] + xt[2] * xt[2]);
  for (int c = 0; c < 3; ++c) fr.n[c] = bdiv(xt[c], xn);
  {
    R a0 = fabs(fr.n[0]), a1 = fabs(fr.n[1]), a2 = fabs(fr.n[2]);
    int m = (a0 <= a1 && a0 <= a2) ? 0 : (a1 <= a2 ? 1 : 2);
    R t[3];
    if (m == 0) { t[0] = R(0); t[1] = fr.n[2]; t[2] = -fr.n[1]; }
    else if (m == 1) { t[0] = -fr.n[2]; t[1] = R(0); t[2] = fr.n[0]; }
    else { t[0] = fr.n[1]; t[1] = -fr.n[0]; t[2] = R(0); }
    R tn = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    for (int c = 0; c < 3; ++c) fr.t1[c] = bdiv(t[c], tn);
    fr.t2[0] = fr.n[1] * fr.t1[2] - fr.n[2] * fr.t1[1];
    fr.t2[1] = fr.n[2] * fr.t1[0] - fr.n[0] * fr.t1[2];
    fr.t2[2] = fr.n[0] * fr.t1[1] - fr.n[1] * fr.t1[0];
  }
  const R gamma = (R)P.gamma;
  {
    // frozen state: Roe average of the two nodes (density sqrt(r0 r1); velocity and total
    // enthalpy weighted by sqrt(rho); sound speed from them)
    const R r0 = wn.w[2][0], r1 = wn.w[3][0];
    const R sl = sqrt(r0), sr = sqrt(r1);
    const R wl = bdiv(sl, sl + sr), wr = bdiv(sr, sl + sr);
    R q0 = R(0), q1 = R(0), ub2 = R(0);
    for (int m = 1; m <= 3; ++m) {
      const R a = wn.w[2][m], b = wn.w[3][m];
      q0 += a * a;
      q1 += b * b;
      const R ub = wl * a + wr * b;
      ub2 += ub * ub;
    }
    const R gg = bdiv(gamma, gamma - R(1));
    const R H0 = bdiv(gg * wn.w[2][4], r0) + R(0.5) * q0;
    const R H1 = bdiv(gg * wn.w[3][4], r1) + R(0.5) * q1;
    const R Hb = wl * H0 + wr * H1;
    fr.rb = sl * sr;
    fr.cb = sqrt((gamma - R(1)) * (Hb - R(0.5) * ub2));
  }
  fr.k = bdiv(fr.rb, R(2) * fr.cb);

  R C[6][5], D[4][5];
  for (int o = 0; o < 6; ++o) to_char(fr, wn.w[o][0], wn.w[o][1], wn.w[o][2], wn.w[o][3], wn.w[o][4], C[o]);
  for (int o = 0; o < 4; ++o) to_char(fr, wn.g[o][0], wn.g[o][1], wn.g[o][2], wn.g[o][3], wn.g[o][4], D[o]);
  const R thr = (R)P.omega_thr, eps = (R)P.mp_eps, alpha = (R)P.mp_alpha;
  // inviscid flow: the MP criterion alone governs every field and the Omega sensor is not
  // evaluated (Sec. 2.3); viscous flow: the wave-appropriate rule
  const bool mp_only = !(C3V || P.viscous);
  bool shockL = false, shockR = false;
  if (!mp_only) {
    R om_m1 = wn.om[0], om_0 = wn.om[1], om_1 = wn.om[2], om_2 = wn.om[3];
    shockL = fmax(fmax(om_m1, om_0), om_1) > thr;
    shockR = fmax(fmax(om_0, om_1), om_2) > thr;
  }

  R CL[5], CR[5];
  for (int b = 0; b < 5; ++b) {
    // C[k] <-> offset k-2 ; D[k] <-> offset k-1
    R cm2 = C[0][b], cm1 = C[1][b], c0 = C[2][b], c1 = C[3][b], c2 = C[4][b], c3 = C[5][b];
    R dm1 = D[0][b], d0 = D[1][b], d1 = D[2][b], d2 = D[3][b];
    R c2i = R(2) * (c1 - R(2) * c0 + cm1) - R(0.5) * (d1 - dm1);
    R c2p = R(2) * (c2 - R(2) * c1 + c0) - R(0.5) * (d2 - d0);
    R Llin = c0 + R(0.5) * d0 + bdiv(c2i, R(12));
    R Rlin = c1 - R(0.5) * d1 + bdiv(c2p, R(12));
    R cc = R(0.5) * (Llin + Rlin);
    bool useL, useR;  // use MP5?
    R Lalt, Ralt;     // value otherwise
    if (mp_only || b == 1) {
      R cmpL = c0 + minmod2(c1 - c0, alpha * (c0 - cm1));
      R cmpR = c1 + minmod2(c0 - c1, alpha * (c1 - c2));
      useL = !((Llin - c0) * (Llin - cmpL) <= eps);
      useR = !((Rlin - c1) * (Rlin - cmpR) <= eps);
      const bool acoustic = b == 0 || b == 4;
      Lalt = acoustic ? Llin : cc;
      Ralt = acoustic ? Rlin : cc;
    } else if (b == 0 || b == 4) {
      useL = shockL; useR = shockR; Lalt = Llin; Ralt = Rlin;
    } else {
      useL = shockL; useR = shockR; Lalt = cc; Ralt = cc;
    }
    CL[b] = useL ? mp5(cm2, cm1, c0, c1, c2, alpha, eps) : Lalt;
    CR[b] = useR ? mp5(c3, c2, c1, c0, cm1, alpha, eps) : Ralt;
  }
  R WL[5], WR[5];
  from_char(fr, CL, WL);
  from_char(fr, CR, WR);
  // a side whose reconstructed density or pressure is not positive takes its upwind node's
  // own primitive state (first order on that side)
  if (!(WL[0] > R(0) && WL[4] > R(0)))
    for (int q = 0; q < 5; ++q) WL[q] = wn.w[2][q];
  if (!(WR[0] > R(0) && WR[4] > R(0)))
    for (int q = 0; q < 5; ++q) WR[q] = wn.w[3][q];
  hllc(WL, WR, xt, gamma, F);
}

// C-GBR convective flux at the interface between node idx and idx + s (direction d;
// mi = met_idx(P, idx))
template <typename R, bool C3V = false>
__device__ __forceinline__ void gbr_flux(const Prob& P, int d, int idx, int mi, R F[5]) {
  GbrWin<R> wn;
  gbr_fill<R, C3V>(P, d, idx, mi, wn);
  gbr_flux_win<R, C3V>(P, wn, F);
}

template <typename R>
__host__ __device__ __forceinline__ void i4_flux(const R* Fn, size_t T, int idx, int s, R F[5]) {
  for (int q = 0; q < 5; ++q) {
    const R* f = Fn + q * T + idx;
    F[q] = (R(7) * (f[0] + f[s]) - (f[-s] + f[2 * s])) * R(1.0 / 12.0);
  }
}

template <typename R, bool C3V = false>
__device__ __forceinline__ void interface_flux(const Prob& P, int d, int idx, int mi, int sel, R F[5]) {
  const int s = P.s[d];
  const size_t T = P.total;
  bool gbr;
  if (sel == SEL_GBR) gbr = true;
  else if (sel == SEL_LAD) gbr = false;
  else if (sel == SEL_PERCELL) gbr = *P.any_flag != 0 && (P.ft[idx] | P.ft[idx + s]) != 0;
  else gbr = *P.any_flag != 0;
  if (gbr) {
    gbr_flux<R, C3V>(P, d, idx, mi, F);
    if (C3V || P.viscous) {
      R Fv[5];
      i4_flux(static_cast<const R*>(P.FV[d]), T, idx, s, Fv);
      for (int q = 0; q < 5; ++q) F[q] = F[q] + Fv[q];
    }
  } else {
    i4_flux(static_cast<const R*>(P.FL[d]), T, idx, s, F);
  }
}

// J at the node whose metric index is mi
template <bool C3V = false>
__device__ __forceinline__ double node_J(const Prob& P, int mi) {
  return (C3V || P.curvilinear) ? P.M64[(size_t)9 * P.met_T + mi] : P.cm[9];
}

// ------------------------------------------------------------------ x sweep: one wave per
// row segment of 63 nodes; lane t computes the interface left of node (seg*63 + t - 1) + 1
// and the flux difference uses the neighbour lane's flux.
// With rk = 1 the sweep is the last direction's: it adds its differences to the partial
// derivative and forms the RK stage result at once (the combination kernel's work).
// FP32: capped at 128 registers (four waves per SIMD; a few spill slots): 2.70 -> 2.50 ms on
// the 1024 x 384 x 128 ramp (the strided sweeps get slower under the same cap).
template <typename R, bool C3V>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1))) k_sweep_x(const Prob* __restrict__ probs, StateRef ref, int sel, int accumulate,
                                                 int skip_if_any, int rk, RKRef rr, int stage, double ca, double cb) {
  const Prob& P = probs[blockIdx.y];
  if (gate_skip(P, skip_if_any)) return;
  const int lane = threadIdx.x & 63;
  const int n0 = P.n[0];
  const int nseg = (n0 + 62) / 63;
  const int rows = P.n[1] * P.n[2];
  double* dQ = ref.deriv(P);
  const size_t T = P.total;
  int bad = 0;
  // waves stride over the (segment, row) items: a capped grid, so that a launch the hybrid
  // switch skips costs few workgroups (the loop bound is uniform in the wave)
  for (int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; wave < nseg * rows;
       wave += (gridDim.x * blockDim.x) >> 6) {
    const int seg = wave % nseg, row = wave / nseg;
    const int j = row % P.n[1], k = row / P.n[1];
    const int il = seg * 63 - 1 + lane;  // interface il + 1/2
    const bool valid = il <= n0 - 1;
    const int idx = pos_to_idx(P, il + P.g[0], j + P.g[1], k + P.g[2]);
    const int mi = (C3V || P.met_planar) ? pos_to_idx(P, il + P.g[0], j + P.g[1], 0) : idx;
    R F[5] = {R(0), R(0), R(0), R(0), R(0)};
    if (valid) interface_flux<R, C3V>(P, 0, idx, mi, sel, F);
    double Fp[5];
    for (int q = 0; q < 5; ++q) Fp[q] = (double)__shfl_up(F[q], 1);
    if (lane >= 1 && valid) {
      double J = node_J<C3V>(P, mi);
      double Lq[5];
      for (int q = 0; q < 5; ++q) {
        double v = -J * ((double)F[q] - Fp[q]);
        size_t o = q * T + idx;
        Lq[q] = accumulate ? dQ[o] + v : v;
        if (!rk) dQ[o] = Lq[q];
      }
      if (rk && rk_combine_node(P, rr, stage, ca, cb, *P.dt, idx, Lq)) ++bad;
    }
  }
  add_bad(P, bad);
}

// ------------------------------------------------------------------ strided sweeps: one
// lane per line segment of `seg` nodes, sliding along the line.
template <typename R, bool C3V>
__global__ void __launch_bounds__(256) k_sweep_s(const Prob* __restrict__ probs, StateRef ref, int d, int sel,
                                                 int accumulate, int seg, int skip_if_any, int rk, RKRef rr, int stage,
                                                 double ca, double cb) {
  const Prob& P = probs[blockIdx.y];
  if (d >= (C3V ? 3 : P.ndim) || gate_skip(P, skip_if_any)) return;
  const int o2 = d == 1 ? 2 : 1;
  const int na = P.n[0], nb = P.n[o2], nd = P.n[d];
  const int nch = (nd + seg - 1) / seg;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= na * nb * nch) return;
  const int a = t % na, r = t / na;
  const int b = r % nb, ch = r / nb;
  const int start = ch * seg, end = min(start + seg, nd);
  int pos[3];
  pos[0] = a + P.g[0];
  pos[o2] = b + P.g[o2];
  pos[d] = start - 1 + P.g[d];
  int idx = pos_to_idx(P, pos[0], pos[1], pos[2]);
  int mi = (C3V || P.met_planar) ? pos_to_idx(P, pos[0], pos[1], 0) : idx;
  const int s = P.s[d], ms = met_step<C3V>(P, d);
  const size_t T = P.total;
  double* dQ = ref.deriv(P);
  const double dt = rk ? *P.dt : 0.0;
  int bad = 0;
  // one flux evaluation site: interface p + 1/2 at node p, for p = start - 1 .. end - 1
  double Fp[5];
  for (int p = start - 1; p < end; ++p, idx += s, mi += ms) {
    R F[5];
    interface_flux<R, C3V>(P, d, idx, mi, sel, F);
    if (p >= start) {
      const double J = node_J<C3V>(P, mi);
      double Lq[5];
      for (int q = 0; q < 5; ++q) {
        const double v = -J * ((double)F[q] - Fp[q]);
        const size_t o = q * T + idx;
        Lq[q] = accumulate ? dQ[o] + v : v;
        if (!rk) dQ[o] = Lq[q];
      }
      if (rk && rk_combine_node(P, rr, stage, ca, cb, dt, idx, Lq)) ++bad;
    }
    for (int q = 0; q < 5; ++q) Fp[q] = (double)F[q];
  }
  add_bad(P, bad);
}

// ------------------------------------------------------------------ compacted C-GBR interfaces
// One persistent launch over the work queue of the per-cell hybrid's C-GBR interfaces (all
// directions, one after the other, each strided over the whole grid): the C-GBR flux of
// every queued interface (plus the interpolated viscous flux) into FG[d] at its left node.
// The LAD interfaces are not visited here; the assembly pass forms them from the node fluxes.
template <typename R>
__global__ void __launch_bounds__(256) k_gbr_items(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.y];
  if (gate_skip(P, GATE_MIXED)) return;
  const size_t T = P.total;
  const int stride = (int)(gridDim.x * blockDim.x);
  for (int d = 0; d < P.ndim; ++d) {
    const int cnt = P.gcount[d];
    const int* q = P.gq + (size_t)d * T;
    R* FG = static_cast<R*>(P.FG[d]);
    const int s = P.s[d];
    for (int it = (int)(blockIdx.x * blockDim.x + threadIdx.x); it < cnt; it += stride) {
      const int idx = q[it];
      R F[5];
      gbr_flux(P, d, idx, met_idx(P, idx), F);
      if (P.viscous) {
        R Fv[5];
        i4_flux(static_cast<const R*>(P.FV[d]), T, idx, s, Fv);
        for (int c = 0; c < 5; ++c) F[c] = F[c] + Fv[c];
      }
      for (int c = 0; c < 5; ++c) FG[c * T + idx] = F[c];
    }
  }
}

template <typename R>
void launch_gbr_items(const Launch& L) {
  // persistent: a fixed grid that fills the chip (8 workgroups of 4 waves per CU), the
  // queue lengths are known on the device only
  const unsigned blocks = L.item_blocks > 0 ? (unsigned)L.item_blocks : 2048u;
  LG_TIMED(L, KC_GBR_ITEMS, hipLaunchKernelGGL(k_gbr_items<R>, dim3(blocks, L.nprob), dim3(256), 0, L.stream,
                                               L.probs));
}

template <typename R>
void launch_sensor(const Launch& L, int skip_if_any, int region) {
  long long b = (L.max_total + 255) / 256;
  if (b > 8192) b = 8192;
  LG_TIMED(L, KC_SENSOR, hipLaunchKernelGGL(k_sensor<R>, dim3((unsigned)b, L.nprob), dim3(256), 0, L.stream,
                                            L.probs, skip_if_any, region));
}

int sweep_seg(const Launch& L, int d) {
  // nodes per lane: the longest segment that still gives >= 8 waves per CU (256 CUs)
  int seg = L.seg;
  if (seg <= 0) {
    seg = 4;
    for (int c = 32; c >= 4; c >>= 1)
      if (((L.max_n[d] + c - 1) / c) * L.sweep_rows[d] * L.nprob >= 256LL * 8 * 64) {
        seg = c;
        break;
      }
  }
  return seg;
}

template <typename R>
void launch_sweep(const Launch& L, StateRef ref, int d, int sel, int accumulate, int skip_if_any, const RKRef* rr,
                  int stage, double a, double b) {
  const RKRef r = rr ? *rr : RKRef{nullptr, nullptr, nullptr};
  const int rk = rr ? 1 : 0;
  // every problem 3D, curvilinear with metrics planar along zeta, and viscous
  const bool c3v = !L.geo_generic && !L.inviscid;
  if (d == 0) {
    long long nseg = (L.max_n[0] + 62) / 63;
    long long waves = nseg * L.sweep_rows[0];
    long long blocks = (waves + 3) / 4;
    if (blocks < 1) blocks = 1;
    if (blocks > 16384) blocks = 16384;   // the kernel strides over the rest
    if (c3v)
      LG_TIMED(L, KC_SWEEP_X, hipLaunchKernelGGL((k_sweep_x<R, true>), dim3((unsigned)blocks, L.nprob), dim3(256), 0,
                                                 L.stream, L.probs, ref, sel, accumulate, skip_if_any, rk, r, stage, a,
                                                 b));
    else
      LG_TIMED(L, KC_SWEEP_X, hipLaunchKernelGGL((k_sweep_x<R, false>), dim3((unsigned)blocks, L.nprob), dim3(256),
                                                 0, L.stream, L.probs, ref, sel, accumulate, skip_if_any, rk, r, stage,
                                                 a, b));
  } else {
    const int seg = sweep_seg(L, d);
    long long nch = (L.max_n[d] + seg - 1) / seg;
    long long work = nch * L.sweep_rows[d];
    long long blocks = (work + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (c3v)
      LG_TIMED(L, d == 1 ? KC_SWEEP_Y : KC_SWEEP_Z,
               hipLaunchKernelGGL((k_sweep_s<R, true>), dim3((unsigned)blocks, L.nprob), dim3(256), 0, L.stream,
                                  L.probs, ref, d, sel, accumulate, seg, skip_if_any, rk, r, stage, a, b));
    else
      LG_TIMED(L, d == 1 ? KC_SWEEP_Y : KC_SWEEP_Z,
               hipLaunchKernelGGL((k_sweep_s<R, false>), dim3((unsigned)blocks, L.nprob), dim3(256), 0, L.stream,
                                  L.probs, ref, d, sel, accumulate, seg, skip_if_any, rk, r, stage, a, b));
  }
}

template void launch_gbr_items<float>(const Launch&);
template void launch_gbr_items<double>(const Launch&);
template void launch_sensor<float>(const Launch&, int, int);
template void launch_sensor<double>(const Launch&, int, int);
template void launch_sweep<float>(const Launch&, StateRef, int, int, int, int, const RKRef*, int, double, double);
template void launch_sweep<double>(const Launch&, StateRef, int, int, int, int, const RKRef*, int, double, double);

}  // namespace lg
