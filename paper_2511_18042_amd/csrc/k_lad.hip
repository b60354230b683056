// Localized artificial diffusivity (LAD) and the node fluxes of the central (flux-form
// E4) scheme, plus the viscous node fluxes of the C-GBR scheme.
//
// Paper: Sec. 2.2 -- mu = mu_f + mu*, beta = beta_f + beta*, kappa = kappa_f + kappa*;
//   mu*    = C_mu    over-bar( rho |sum_l d4(|S|) Delta_{l,mu}^2| )
//   beta*  = C_beta  over-bar( rho f_sw |sum_l d4(div u) Delta_{l,beta}^2| )
//   kappa* = C_kappa over-bar( rho c / T |sum_l d4(e) Delta_{l,kappa}| )
//   f_sw = H(-div u) (div u)^2 / ((div u)^2 + |curl u|^2 + 1e-32)
//   Delta_{l,mu} = |Delta x_l|, Delta_{l,beta} = |Delta x_l . grad rho / |grad rho||,
//   Delta_{l,kappa} = |Delta x_l . grad e / |grad e||, Delta x_l = (x_{+1} - x_{-1}) / 2;
// over-bar = truncated Gaussian (Kawai & Lele, 9 points) along xi, eta, zeta in turn.
// Eq. tauij: tau_ij = mu (u_i,j + u_j,i) + (beta - 2 mu / 3) div u delta_ij,
//            phi_i  = u_j tau_ij + kappa T_,i;
// viscous node flux of direction l: -l_hat . [0, tau, phi] (Sec. 2.1), Sutherland law,
// kappa_hat = mu_hat / ((gamma - 1) Pr M^2), T = gamma M^2 p / rho.
//
// The central convective flux of LAD-E4 is written in flux form: the E4 derivative of a
// node flux equals the difference of its fourth-order interface interpolation, so the
// node fluxes F^c + F^v are stored here and interpolated in the interface sweep.  LAD-C6
// (Sec. 3, Alg. 1) runs the same kernels on compact sixth-order gradients solved
// beforehand (k_compact.hip), and its interface fluxes are tridiagonal solves there.
// Fourth differences use five points; all derivatives use unit computational spacing.
#include "lgbr_dev.h"
#include "lgbr_kernels.h"

namespace lg {

__device__ __forceinline__ bool lad_skip(const Prob& P, int skip_if_any) {
  return gate_skip(P, skip_if_any);
}

template <typename R>
__device__ __forceinline__ R e4_at(const R* f, int idx, int s) {
  return (R(8) * (f[idx + s] - f[idx - s]) - (f[idx + 2 * s] - f[idx - 2 * s])) * R(1.0 / 12.0);
}

// physical gradients D[q][j] of the 5 primitives at node idx from computational
// derivatives gl[l][q] (l < ndim)
// Direction loops run over the three directions with a uniform exit, so that every
// register array index is a constant (a runtime bound indexes registers indirectly).  The
// shear kernel keeps the runtime bound (UNROLL false): it is faster that way.
template <typename R, bool UNROLL = true>
__device__ __forceinline__ void to_physical(int ndim, const R mt[10], const R gl[3][5], R D[5][3]) {
  R J = mt[9];
  for (int q = 0; q < 5; ++q)
    for (int j = 0; j < 3; ++j) D[q][j] = R(0);
  if constexpr (UNROLL) {
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      if (l >= ndim) break;
      for (int j = 0; j < 3; ++j) {
        R m = J * mt[3 * l + j];
        for (int q = 0; q < 5; ++q) D[q][j] += m * gl[l][q];
      }
    }
  } else {
    for (int l = 0; l < ndim; ++l)
      for (int j = 0; j < 3; ++j) {
        R m = J * mt[3 * l + j];
        for (int q = 0; q < 5; ++q) D[q][j] += m * gl[l][q];
      }
  }
}

// Sutherland viscosity and conductivity from rho, p (ri = 1 / rho)
template <typename R>
__device__ __forceinline__ void transport(const Prob& P, R ri, R p, R& mu, R& kappa) {
  if (!P.viscous) {
    mu = R(0);
    kappa = R(0);
    return;
  }
  R T = R(P.gamma * P.Mref * P.Mref) * p * ri;
  R S = (R)P.suth;
  mu = T * sqrt(T) * (R(1) + S) * rcp(T + S) * R(1.0 / P.Re);
  kappa = mu * R(1.0 / ((P.gamma - 1.0) * P.Pr * P.Mref * P.Mref));
}

// -l_hat . [0, tau, phi] with l_hat = (m0, m1, m2) (Eq. tauij); ri = 1 / rho
template <typename R>
__device__ __forceinline__ void viscous_flux(const Prob& P, R m0, R m1, R m2, const R w[5], R ri, const R D[5][3],
                                             R mu, R beta, R kappa, R F[5]) {
  R du[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) du[i][j] = D[1 + i][j];
  R theta = du[0][0] + du[1][1] + du[2][2];
  R g2 = R(P.gamma * P.Mref * P.Mref);
  R p = w[4];
  R tau[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      tau[i][j] = mu * (du[i][j] + du[j][i]);
      if (i == j) tau[i][j] += (beta - R(2.0 / 3.0) * mu) * theta;
    }
  R phi[3];
  for (int i = 0; i < 3; ++i) {
    R dT = g2 * (D[4][i] * ri - p * D[0][i] * (ri * ri));
    phi[i] = w[1] * tau[i][0] + w[2] * tau[i][1] + w[3] * tau[i][2] + kappa * dT;
  }
  F[0] = R(0);
  for (int i = 0; i < 3; ++i) F[1 + i] = -(m0 * tau[i][0] + m1 * tau[i][1] + m2 * tau[i][2]);
  F[4] = -(m0 * phi[0] + m1 * phi[1] + m2 * phi[2]);
}

__device__ __forceinline__ bool in_band(const Prob& P, int idx, int lo, int hi) {
  int p[3] = {idx % P.N[0], (idx / P.N[0]) % P.N[1], idx / (P.N[0] * P.N[1])};
#pragma unroll
  for (int l = 0; l < 3; ++l)
    if (l < P.ndim && (p[l] < P.g[l] + lo || p[l] >= P.g[l] + P.n[l] + hi)) return false;
  return true;
}

__device__ __forceinline__ bool is_interior(const Prob& P, int idx) { return in_band(P, idx, 0, 0); }

// ------------------------------------------------------------------ z-marching helpers
// E4 derivative from the values at offsets -2, -1, +1, +2 (same rounding as e4_at).
template <typename R>
__device__ __forceinline__ R e4v(R m2, R m1, R p1, R p2) {
  return (R(8) * (p1 - m1) - (p2 - m2)) * R(1.0 / 12.0);
}

// fourth difference from the values at offsets -2 .. 2 (same rounding as delta4)
template <typename R>
__device__ __forceinline__ R d4v(R m2, R m1, R c0, R p1, R p2) {
  return m2 - R(4) * m1 + R(6) * c0 - R(4) * p1 + p2;
}

template <typename R>
__device__ __forceinline__ R delta4(const R* f, int idx, int s) {
  return f[idx - 2 * s] - R(4) * f[idx - s] + R(6) * f[idx] - R(4) * f[idx + s] + f[idx + 2 * s];
}

// Register queue of NV fields at planes k-2 .. k+2 of one column (3D z-marching).
template <typename R, int NV>
struct ZQ5 {
  R v[5][NV];
  // before the first plane k0: planes k0-2 .. k0+1 into slots 1..4
  __device__ __forceinline__ void prime(const R* f, size_t T, int idx, int sz) {
    for (int p = 1; p < 5; ++p)
      for (int q = 0; q < NV; ++q) v[p][q] = f[q * T + idx + (p - 3) * sz];
  }
  // advance to plane k (idx): slots 0..4 = planes k-2 .. k+2
  __device__ __forceinline__ void step(const R* f, size_t T, int idx, int sz) {
    for (int p = 0; p < 4; ++p)
      for (int q = 0; q < NV; ++q) v[p][q] = v[p + 1][q];
    for (int q = 0; q < NV; ++q) v[4][q] = f[q * T + idx + 2 * sz];
  }
};

// computational E4 derivatives of the 5 primitives at idx; z from the queue (3D)
template <typename R>
__device__ __forceinline__ void e4_grads_zm(const Prob& P, int nd, const R* W, int idx, const ZQ5<R, 5>& qz,
                                            R gl[3][5]) {
  const size_t T = P.total;
  for (int l = 0; l < 3; ++l)
    for (int q = 0; q < 5; ++q) gl[l][q] = R(0);
  for (int q = 0; q < 5; ++q) {
    gl[0][q] = e4_at(W + q * T, idx, P.s[0]);
    if (nd > 1) gl[1][q] = e4_at(W + q * T, idx, P.s[1]);
    if (nd > 2) gl[2][q] = e4v(qz.v[0][q], qz.v[1][q], qz.v[3][q], qz.v[4][q]);
  }
}

// computational derivatives of the 5 primitives at idx read from the gradient arrays
// (LAD-C6: compact sixth-order gradients solved beforehand)
template <typename R>
__device__ __forceinline__ void stored_grads(const Prob& P, int idx, R gl[3][5]) {
  const size_t T = P.total;
  for (int l = 0; l < 3; ++l)
    for (int q = 0; q < 5; ++q) gl[l][q] = l < P.ndim ? static_cast<const R*>(P.G[l])[q * T + idx] : R(0);
}

// ------------------------------------------------------------------ grid factors
// Delta x_l at interior nodes (curvilinear grids; once per context); when the grid is
// planar along zeta, only the first interior plane is stored
template <typename R>
__global__ void __launch_bounds__(256) k_lad_dx(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.y];
  if (!P.curvilinear) return;
  R* GX = static_cast<R*>(P.GX);
  const size_t T = P.total;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < P.total; idx += gridDim.x * blockDim.x) {
    if (!is_interior(P, idx)) continue;
    if (P.met_planar && idx / P.s[2] != P.g[2]) continue;
    for (int l = 0; l < 3; ++l)
      for (int cc = 0; cc < 3; ++cc) {
        R v = R(0);
        if (l < P.ndim) {
          const double* X = P.coords + (size_t)cc * T;
          v = (R)(0.5 * (X[idx + P.s[l]] - X[idx - P.s[l]]));
        }
        GX[(size_t)(3 * l + cc) * P.met_T + met_idx(P, idx)] = v;
      }
  }
}

// ------------------------------------------------------------------ |S| and theta
// at positions -2 .. n+1 (the fourth differences of the raw coefficients reach two nodes
// past the interior); E4 physical gradients recomputed from W (CG: stored gradients)
template <typename R, bool CG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 6 : 4)))
k_lad_shear(const Prob* __restrict__ probs, int skip_if_any, int zc) {
  const Prob& P = probs[blockIdx.y];
  if (lad_skip(P, skip_if_any)) return;
  ZCol c;
  if (!zm_column(P, -2, 2, zc, c)) return;
  const R* W = static_cast<const R*>(P.W);
  R* S = static_cast<R*>(P.S3);
  const size_t T = P.total;
  const int sz = P.s[2];
  const int nd = P.ndim;
  const bool z3 = nd == 3 && !CG;
  int idx = pos_to_idx(P, c.i, c.j, c.k0);
  ZQ5<R, 5> qz;
  if (z3) qz.prime(W, T, idx, sz);
  R mt[10];
  const bool mplane = P.met_planar;
  if (mplane) load_met(P, idx, mt);   // one plane of metrics serves the whole column
  for (int k = c.k0; k < c.k1; ++k, idx += sz) {
    if (z3) qz.step(W, T, idx, sz);
    if (!mplane) load_met(P, idx, mt);
    R gl[3][5], D[5][3];
    if (CG) stored_grads(P, idx, gl);
    else e4_grads_zm(P, nd, W, idx, qz, gl);
    to_physical<R, false>(nd, mt, gl, D);
    R S2 = R(0);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        R sij = R(0.5) * (D[1 + i][j] + D[1 + j][i]);
        S2 += sij * sij;
      }
    S[idx] = sqrt(S2);
    S[T + idx] = D[1][0] + D[2][1] + D[3][2];
  }
}

// ------------------------------------------------------------------ raw coefficients
// 1 / (|g| + 1e-32), the factor of the regularised unit vector g / (|g| + 1e-32).  In FP32
// the squares of components below 2^-63 underflow (1e-32 lies below the square root of the
// normal range) and would leave an unbounded projection: FP32 vectors whose largest
// component is non-zero and below 2^-60 are normalised in FP64, all others in FP32.
template <typename R>
__device__ __forceinline__ R inv_norm_reg(const R g[3]) {
  if constexpr (sizeof(R) == 4) {
    const float m = fmaxf(fabsf(g[0]), fmaxf(fabsf(g[1]), fabsf(g[2])));
    if (m == 0.0f || m >= 0x1p-60f) return 1.0f / (sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + 1e-32f);
  }
  return (R)(1.0 / (sqrt((double)g[0] * g[0] + (double)g[1] * g[1] + (double)g[2] * g[2]) + 1e-32));
}

// at interior nodes; e = p / ((gamma - 1) rho) from W wherever needed
// C3P: every problem of the launch is 3D and curvilinear with metrics planar along zeta
// (branches on the geometry folded at compile time)
template <typename R, bool CG, bool C3P>
__global__ void __launch_bounds__(256) k_lad_raw(const Prob* __restrict__ probs, int skip_if_any, int zc) {
  const Prob& P = probs[blockIdx.y];
  if (lad_skip(P, skip_if_any)) return;
  ZCol c;
  if (!zm_column(P, 0, 0, zc, c)) return;
  const R* W = static_cast<const R*>(P.W);
  const R* S = static_cast<const R*>(P.S3);
  const R* GX = static_cast<const R*>(P.GX);
  R* C = static_cast<R*>(P.CA);
  const size_t T = P.total;
  const int sz = P.s[2];
  const int nd = C3P ? 3 : P.ndim;
  const bool curv = C3P || P.curvilinear;
  const bool z3 = nd == 3;
  const R gm1 = R(P.gamma - 1.0), igm1 = R(1.0 / (P.gamma - 1.0));
  int idx = pos_to_idx(P, c.i, c.j, c.k0);
  ZQ5<R, 5> qz;
  ZQ5<R, 2> qs;
  if (z3) {
    qz.prime(W, T, idx, sz);
    qs.prime(S, T, idx, sz);
  }
  R mt[10], gx[9];
  const bool mplane = C3P || P.met_planar;
  auto load_gx = [&](int id) {
    for (int m = 0; m < 9; ++m) gx[m] = curv ? GX[(size_t)m * P.met_T + met_idx(P, id)] : R(0);
  };
  if (mplane) {   // one plane of metrics and grid factors serves the whole column
    load_met(P, idx, mt);
    load_gx(idx);
  }
  for (int k = c.k0; k < c.k1; ++k, idx += sz) {
    if (z3) {
      qz.step(W, T, idx, sz);
      qs.step(S, T, idx, sz);
    }
    if (!mplane) {
      load_met(P, idx, mt);
      load_gx(idx);
    }
    R gl[3][5], D[5][3];
    if (CG) stored_grads(P, idx, gl);
    else e4_grads_zm(P, nd, W, idx, qz, gl);
    to_physical(nd, mt, gl, D);
    R rho = W[idx], p = W[4 * T + idx];
    R ri = rcp(rho);
    R theta = D[1][0] + D[2][1] + D[3][2];
    R w1 = D[3][1] - D[2][2], w2 = D[1][2] - D[3][0], w3 = D[2][0] - D[1][1];
    R om2 = w1 * w1 + w2 * w2 + w3 * w3;
    R de[3], gr[3];
    for (int j = 0; j < 3; ++j) {
      de[j] = (D[4][j] * ri - p * D[0][j] * (ri * ri)) * igm1;
      gr[j] = D[0][j];
    }
    const R inr = inv_norm_reg(gr), ine = inv_norm_reg(de);
    R Tt = R(P.gamma * P.Mref * P.Mref) * p * ri;
    R cs = sqrt(R(P.gamma) * p * ri);
    R fsw = theta < R(0) ? theta * theta * rcp(theta * theta + om2 + R(1e-32)) : R(0);
    R smu = R(0), sbeta = R(0), skap = R(0);
    #pragma unroll
    for (int l = 0; l < 3; ++l) {
      if (l >= nd) break;
      R dx[3];
      if (curv) {
        for (int cc = 0; cc < 3; ++cc) dx[cc] = gx[3 * l + cc];
      } else {
        dx[0] = dx[1] = dx[2] = R(0);
        dx[l] = (R)P.h[l];
      }
      R dmu2 = dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2];
      R dbeta = (dx[0] * gr[0] + dx[1] * gr[1] + dx[2] * gr[2]) * inr;
      R dkap = fabs(dx[0] * de[0] + dx[1] * de[1] + dx[2] * de[2]) * ine;
      R f4S, f4t, f4e;
      if (l < 2) {
        const int s = P.s[l];
        f4S = delta4(S, idx, s);
        f4t = delta4(S + T, idx, s);
        R e[5];
        for (int o = -2; o <= 2; ++o) {
          const int id = idx + o * s;
          e[o + 2] = W[4 * T + id] * rcp(gm1 * W[id]);
        }
        f4e = d4v(e[0], e[1], e[2], e[3], e[4]);
      } else {
        f4S = d4v(qs.v[0][0], qs.v[1][0], qs.v[2][0], qs.v[3][0], qs.v[4][0]);
        f4t = d4v(qs.v[0][1], qs.v[1][1], qs.v[2][1], qs.v[3][1], qs.v[4][1]);
        R e[5];
        for (int o = 0; o < 5; ++o) e[o] = qz.v[o][4] * rcp(gm1 * qz.v[o][0]);
        f4e = d4v(e[0], e[1], e[2], e[3], e[4]);
      }
      smu += f4S * dmu2;
      sbeta += f4t * dbeta * dbeta;
      skap += f4e * dkap;
    }
    C[idx] = R(P.C_mu) * rho * fabs(smu);
    C[T + idx] = R(P.C_beta) * rho * fsw * fabs(sbeta);
    C[2 * T + idx] = R(P.C_kappa) * rho * cs * rcp(Tt) * fabs(skap);
  }
}

// ------------------------------------------------------------------ truncated Gaussian
// The three one-directional passes of the filter, each followed by ghost images, read
// the previous pass at image positions: the xi and eta passes run together on LDS tiles
// of one plane (rows mapped to their images, columns through the images of the raw
// coefficients), the zeta pass z-marches with a nine-plane register queue.  No ghost
// refill launches are needed; consumers read the result through scalar_image().
template <typename R>
struct GaussW {
  static constexpr R w0 = R(3565.0 / 10368.0), w1 = R(3091.0 / 12960.0), w2 = R(1997.0 / 25920.0),
                     w3 = R(149.0 / 12960.0), w4 = R(107.0 / 103680.0);
};

// f[-4*s] .. f[4*s] around f (same rounding as one pass of the filter)
template <typename R>
__device__ __forceinline__ R gauss9(const R* f, int s) {
  R v = GaussW<R>::w0 * f[0];
  v = v + GaussW<R>::w1 * (f[s] + f[-s]);
  v = v + GaussW<R>::w2 * (f[2 * s] + f[-2 * s]);
  v = v + GaussW<R>::w3 * (f[3 * s] + f[-3 * s]);
  v = v + GaussW<R>::w4 * (f[4 * s] + f[-4 * s]);
  return v;
}

template <typename R, int TY>
__global__ void __launch_bounds__(256) k_gauss_xy(const Prob* __restrict__ probs, int skip_if_any, int zc) {
  constexpr int TX = 64, RX = TX + 8, RY = TY + 8;
  constexpr int LR = (RY + 2) / 3;  // region rows per loading thread (216 threads: 72 columns x 3)
  constexpr int XR = RY / 4;        // xi-pass rows per thread (64 columns x 4)
  constexpr int YR = TY / 4;        // output rows per thread
  __shared__ R sC[3][RY][RX];
  __shared__ R sX[3][RY][TX];
  const Prob& P = probs[blockIdx.y];
  if (lad_skip(P, skip_if_any)) return;
  int org[3], ext[3];
  zm_band(P, 0, 0, org, ext);
  int ti0, tj0, k0, k1;
  if (!zm_tile<TX, TY>(ext, zc, ti0, tj0, k0, k1)) return;
  const R* C = static_cast<const R*>(P.CA);
  R* out = static_cast<R*>(P.CB);
  const size_t T = P.total;
  const int tid = threadIdx.x;
  const bool two = P.ndim > 1;
  // region loads: column tid % 72 and rows tid / 72 + 3 m, through their ghost images;
  // -1 marks columns / rows past what this tile's nodes reach (left unused)
  const int lc = tid % RX, lr = tid / RX;
  int lbase[LR];
  {
    const int pi = org[0] + ti0 - 4 + lc;
    const bool okc = tid < 3 * RX && pi < org[0] + ext[0] + 4;
    const int gi = okc ? scalar_image(P, 0, pi) : 0;
    for (int m = 0; m < LR; ++m) {
      const int r = lr + 3 * m;
      const int pj = org[1] + tj0 - 4 + r;
      const bool ok = okc && r < RY && (!two || pj < org[1] + ext[1] + 4);
      lbase[m] = ok ? gi + P.s[1] * (two ? scalar_image(P, 1, pj) : 0) : -1;
    }
  }
  const int cx = tid % TX, rg = tid / TX;
  int obase[YR];
  for (int m = 0; m < YR; ++m) {
    const int ti = ti0 + cx, tj = tj0 + rg + 4 * m;
    obase[m] = (ti < ext[0] && tj < ext[1]) ? pos_to_idx(P, org[0] + ti, org[1] + tj, 0) : -1;
  }
  // the region of the next plane is fetched into registers while this plane is filtered
  R pre[LR][3];
  auto fetch = [&](int kk) {
    const int koff = P.s[2] * (org[2] + kk);
    for (int m = 0; m < LR; ++m) {
      const int r = lr + 3 * m;
      if (r < RY && tid < 3 * RX)
        for (int q = 0; q < 3; ++q) pre[m][q] = lbase[m] >= 0 ? C[q * T + lbase[m] + koff] : R(0);
    }
  };
  if (k0 < k1) fetch(k0);
  for (int kk = k0; kk < k1; ++kk) {
    const int koff = P.s[2] * (org[2] + kk);
    // sC is free: every read of the previous plane's xi pass precedes the last barrier
    for (int m = 0; m < LR; ++m) {
      const int r = lr + 3 * m;
      if (r < RY && tid < 3 * RX)
        for (int q = 0; q < 3; ++q) sC[q][r][lc] = pre[m][q];
    }
    __syncthreads();
    if (kk + 1 < k1) fetch(kk + 1);
    for (int m = 0; m < XR; ++m)
      for (int q = 0; q < 3; ++q) sX[q][rg + 4 * m][cx] = gauss9(&sC[q][rg + 4 * m][cx + 4], 1);
    __syncthreads();
    // the next plane's loads touch sC only, and its xi pass (which rewrites sX) starts
    // after a barrier that every read below precedes
    for (int m = 0; m < YR; ++m) {
      if (obase[m] < 0) continue;
      const int r = rg + 4 * m;
      for (int q = 0; q < 3; ++q) {
        const R v = two ? gauss9(&sX[q][r + 4][cx], TX) : sX[q][r + 4][cx];
        out[q * T + obase[m] + koff] = v;
      }
    }
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_gauss_z(const Prob* __restrict__ probs, int skip_if_any, int zc) {
  const Prob& P = probs[blockIdx.y];
  if (P.ndim < 3 || lad_skip(P, skip_if_any)) return;
  ZCol c;
  if (!zm_column(P, 0, 0, zc, c)) return;
  const R* in = static_cast<const R*>(P.CB);
  R* out = static_cast<R*>(P.CA);
  const size_t T = P.total;
  const int col = pos_to_idx(P, c.i, c.j, 0);
  R qz[9][3];  // planes k-4 .. k+4 (ghost planes through their images)
  for (int p = 1; p < 9; ++p) {
    const int id = col + P.s[2] * scalar_image(P, 2, c.k0 - 5 + p);
    for (int q = 0; q < 3; ++q) qz[p][q] = in[q * T + id];
  }
  for (int k = c.k0; k < c.k1; ++k) {
    for (int p = 0; p < 8; ++p)
      for (int q = 0; q < 3; ++q) qz[p][q] = qz[p + 1][q];
    const int id = col + P.s[2] * scalar_image(P, 2, k + 4);
    for (int q = 0; q < 3; ++q) qz[8][q] = in[q * T + id];
    for (int q = 0; q < 3; ++q) {
      R v = GaussW<R>::w0 * qz[4][q];
      v = v + GaussW<R>::w1 * (qz[5][q] + qz[3][q]);
      v = v + GaussW<R>::w2 * (qz[6][q] + qz[2][q]);
      v = v + GaussW<R>::w3 * (qz[7][q] + qz[1][q]);
      v = v + GaussW<R>::w4 * (qz[8][q] + qz[0][q]);
      out[q * T + col + P.s[2] * k] = v;
    }
  }
}

// ------------------------------------------------------------------ LAD node fluxes
// What the node flux of any direction needs at one node.
template <typename R>
struct LadNode {
  R w[5], D[5][3];
  R ri, mu, beta, kappa, E;
};

// w: primitives at the node; cf: the (ghost-imaged) coefficients mu*, beta*, kappa* there;
// gl: computational E4 derivatives; mt: metrics
template <typename R>
__device__ __forceinline__ void lad_node_state(const Prob& P, int nd, const R w[5], const R cf[3], const R mt[10],
                                               const R gl[3][5], LadNode<R>& s) {
  for (int q = 0; q < 5; ++q) s.w[q] = w[q];
  to_physical(nd, mt, gl, s.D);
  s.ri = rcp(s.w[0]);
  R muf, kapf;
  transport(P, s.ri, s.w[4], muf, kapf);
  s.mu = muf + cf[0];
  s.beta = cf[1];
  s.kappa = kapf + cf[2];
  s.E = s.w[4] * R(1.0 / (P.gamma - 1.0)) + R(0.5) * s.w[0] * (s.w[1] * s.w[1] + s.w[2] * s.w[2] + s.w[3] * s.w[3]);
}

// F^c_l + F^v_l at the node
template <typename R>
__device__ __forceinline__ void lad_node_flux(const Prob& P, const LadNode<R>& s, const R mt[10], int l, R out[5]) {
  const R m0 = mt[3 * l], m1 = mt[3 * l + 1], m2 = mt[3 * l + 2];
  R F[5];
  viscous_flux(P, m0, m1, m2, s.w, s.ri, s.D, s.mu, s.beta, s.kappa, F);
  const R U = m0 * s.w[1] + m1 * s.w[2] + m2 * s.w[3];
  out[0] = s.w[0] * U + F[0];
  out[1] = s.w[0] * s.w[1] * U + m0 * s.w[4] + F[1];
  out[2] = s.w[0] * s.w[2] * U + m1 * s.w[4] + F[2];
  out[3] = s.w[0] * s.w[3] * U + m2 * s.w[4] + F[3];
  out[4] = (s.E + s.w[4]) * U + F[4];
}

// F^c + F^v for every active direction at positions -2 .. n+1; gradients recomputed from
// W (CG: stored gradients), coefficients read at the image of the node
// C3P: every problem 3D and curvilinear with metrics planar along zeta (as in k_lad_raw)
template <typename R, bool CG, bool O32, bool C3P>
__global__ void __launch_bounds__(256) k_lad_nodeflux(const Prob* __restrict__ probs, int coef_buf, int skip_if_any,
                                                      int zc) {
  using IX = sidx_t<O32>;
  const Prob& P = probs[blockIdx.y];
  if (lad_skip(P, skip_if_any)) return;
  ZCol c;
  if (!zm_column(P, -2, 2, zc, c)) return;
  const R* W = static_cast<const R*>(P.W);
  const R* C = static_cast<const R*>(coef_buf == 0 ? P.CA : P.CB);
  const R* MR = static_cast<const R*>(P.MR);
  const IX T = (IX)P.total;
  const int sz = P.s[2];
  const int nd = C3P ? 3 : P.ndim;
  const bool curv = C3P || P.curvilinear;
  const bool z3 = nd == 3;
  const bool zq = z3 && !CG;
  const int ci = scalar_image(P, 0, c.i);
  const int cj = nd > 1 ? scalar_image(P, 1, c.j) : c.j;
  int idx = pos_to_idx(P, c.i, c.j, c.k0);
  R qz[5][5];   // planes k-2 .. k+2 of the primitives
  if (zq)
    for (int p = 1; p < 5; ++p)
      for (int q = 0; q < 5; ++q) qz[p][q] = gld<R, O32>(W, (IX)q * T + (IX)(idx + (p - 3) * sz));
  R mt[10];
  const bool mplane = C3P || P.met_planar;
  auto load_mt = [&](int id) {
    const IX mi = (IX)met_idx(P, id), mT = (IX)P.met_T;
    for (int m = 0; m < 10; ++m) mt[m] = curv ? gld<R, O32>(MR, (IX)m * mT + mi) : (R)P.cm[m];
  };
  if (mplane) load_mt(idx);   // one plane of metrics serves the whole column
  for (int k = c.k0; k < c.k1; ++k, idx += sz) {
    if (zq) {
      for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 5; ++q) qz[p][q] = qz[p + 1][q];
      for (int q = 0; q < 5; ++q) qz[4][q] = gld<R, O32>(W, (IX)q * T + (IX)(idx + 2 * sz));
    }
    if (!mplane) load_mt(idx);
    R gl[3][5], w[5];
    for (int l = 0; l < 3; ++l)
      for (int q = 0; q < 5; ++q) gl[l][q] = R(0);
    for (int q = 0; q < 5; ++q) {
      const IX o = (IX)q * T + (IX)idx;
      w[q] = zq ? qz[2][q] : gld<R, O32>(W, o);
      if (CG) {
#pragma unroll
        for (int l = 0; l < 3; ++l)
          if (l < nd) gl[l][q] = gld<R, O32>(static_cast<const R*>(P.G[l]), o);
      } else {
        gl[0][q] = e4v(gld<R, O32>(W, o - 2), gld<R, O32>(W, o - 1), gld<R, O32>(W, o + 1), gld<R, O32>(W, o + 2));
        if (nd > 1) {
          const IX s1 = (IX)P.s[1];
          gl[1][q] = e4v(gld<R, O32>(W, o - 2 * s1), gld<R, O32>(W, o - s1), gld<R, O32>(W, o + s1),
                         gld<R, O32>(W, o + 2 * s1));
        }
        if (z3) gl[2][q] = e4v(qz[0][q], qz[1][q], qz[3][q], qz[4][q]);
      }
    }
    const IX cidx = (IX)pos_to_idx(P, ci, cj, z3 ? scalar_image(P, 2, k) : k);
    const R cf[3] = {gld<R, O32>(C, cidx), gld<R, O32>(C, T + cidx), gld<R, O32>(C, 2 * T + cidx)};
    LadNode<R> s;
    lad_node_state(P, nd, w, cf, mt, gl, s);
    #pragma unroll
    for (int l = 0; l < 3; ++l) {
      if (l >= nd) break;
      R F[5];
      lad_node_flux(P, s, mt, l, F);
      R* out = static_cast<R*>(P.FL[l]);
      for (int q = 0; q < 5; ++q) gst<R, O32>(out, (IX)q * T + (IX)idx, F[q]);
    }
  }
}

// ------------------------------------------------------------------ all-LAD interfaces
// dQ/dt = -J sum_l (F_{l,+1/2} - F_{l,-1/2}) with F = I4 of the node fluxes (fourth-order
// midpoint interpolation), the differences in FP64 in the order xi, eta, zeta; mode 0
// stores it, mode 1 forms the RK stage a U^n + b (U^s + dt L) in place of the combination
// kernel (interior nodes; non-physical results are counted), and with rr.save_dq also
// writes it to dQ/dt, the copy the filter guard restores from; with rr.prim_out also its
// primitives (and troubled flags), which the next stage would otherwise convert.
template <typename R>
__device__ __forceinline__ R i4v(R m1, R c0, R p1, R p2) {
  return (R(7) * (c0 + p1) - (m1 + p2)) * R(1.0 / 12.0);
}

template <typename R, bool O32>
__global__ void __launch_bounds__(256) k_lad_sweep(const Prob* __restrict__ probs, StateRef ref, RKRef rr, int mode,
                                                   int stage, double a, double b, int skip_if_any, int zc) {
  using IX = sidx_t<O32>;
  const Prob& P = probs[blockIdx.y];
  if (lad_skip(P, skip_if_any)) return;
  ZCol c;
  if (!zm_column(P, 0, 0, zc, c)) return;
  const IX T = (IX)P.total;
  const int sz = P.s[2];
  const bool z3 = P.ndim == 3;
  const R* Fx = static_cast<const R*>(P.FL[0]);
  const R* Fy = static_cast<const R*>(P.FL[1]);
  const R* Fz = static_cast<const R*>(P.FL[2]);
  double* dQ = ref.deriv(P);
  const double* Un = rr.Un ? rr.Un : P.Q;
  const double* Us = rr.Us ? rr.Us : (stage == 0 ? Un : P.Us);
  double* out = rr.out ? rr.out : (stage == 2 ? const_cast<double*>(Un) : P.Us);
  const double dt = mode ? *P.dt : 0.0;
  int bad = 0;
  int idx = pos_to_idx(P, c.i, c.j, c.k0);
  R qz[5][5];   // planes k-2 .. k+2 of the zeta fluxes
  if (z3)
    for (int p = 1; p < 5; ++p)
      for (int q = 0; q < 5; ++q) qz[p][q] = gld<R, O32>(Fz, (IX)q * T + (IX)(idx + (p - 3) * sz));
  const bool mplane = P.met_planar;
  const double Jcol = met64(P, 9, idx);
  for (int k = c.k0; k < c.k1; ++k, idx += sz) {
    if (z3) {
      for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 5; ++q) qz[p][q] = qz[p + 1][q];
      for (int q = 0; q < 5; ++q) qz[4][q] = gld<R, O32>(Fz, (IX)q * T + (IX)(idx + 2 * sz));
    }
    const double J = mplane ? Jcol : met64(P, 9, idx);
    double Lq[5];
    for (int q = 0; q < 5; ++q) {
      const IX o = (IX)q * T + (IX)idx;
      R fp = i4v(gld<R, O32>(Fx, o - 1), gld<R, O32>(Fx, o), gld<R, O32>(Fx, o + 1), gld<R, O32>(Fx, o + 2));
      R fm = i4v(gld<R, O32>(Fx, o - 2), gld<R, O32>(Fx, o - 1), gld<R, O32>(Fx, o), gld<R, O32>(Fx, o + 1));
      Lq[q] = -J * ((double)fp - (double)fm);
    }
    if (P.ndim > 1) {
      const IX s = (IX)P.s[1];
      for (int q = 0; q < 5; ++q) {
        const IX o = (IX)q * T + (IX)idx;
        const R m2 = gld<R, O32>(Fy, o - 2 * s), m1 = gld<R, O32>(Fy, o - s), c0 = gld<R, O32>(Fy, o),
                p1 = gld<R, O32>(Fy, o + s), p2 = gld<R, O32>(Fy, o + 2 * s);
        R fp = i4v(m1, c0, p1, p2), fm = i4v(m2, m1, c0, p1);
        Lq[q] = Lq[q] + -J * ((double)fp - (double)fm);
      }
    }
    if (z3) {
      for (int q = 0; q < 5; ++q) {
        R fp = i4v(qz[1][q], qz[2][q], qz[3][q], qz[4][q]);
        R fm = i4v(qz[0][q], qz[1][q], qz[2][q], qz[3][q]);
        Lq[q] = Lq[q] + -J * ((double)fp - (double)fm);
      }
    }
    if (mode == 0) {
      for (int q = 0; q < 5; ++q) gst<double, O32>(dQ, (IX)q * T + (IX)idx, Lq[q]);
    } else {
      // rk_combine_node with the same accesses
      double v[5];
      for (int q = 0; q < 5; ++q) {
        const IX o = (IX)q * T + (IX)idx;
        v[q] = a * gld<double, O32>(Un, o) + b * (gld<double, O32>(Us, o) + dt * Lq[q]);
        gst<double, O32>(out, o, v[q]);
        if (rr.save_dq) gst<double, O32>(P.dQ, o, v[q]);
      }
      if (rr.prim_out) {   // the next stage's primitives (and troubled flags) at this node
        double pp;
        R w[5];
        prim_node<R>(P, v[0], v[1], v[2], v[3], v[4], w[0], w[1], w[2], w[3], w[4], pp);
        R* W = static_cast<R*>(P.W);
        for (int q = 0; q < 5; ++q) gst<R, O32>(W, (IX)q * T + (IX)idx, w[q]);
        if (rr.prim_out == 2) P.f[idx] = (uint8_t)troubled(v[0], pp, P);
      }
      const double rho = v[0];
      const double ke = 0.5 * (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / rho;
      const double p = (P.gamma - 1.0) * (v[4] - ke);
      const bool ok = rho > 0.0 && p > 0.0 && isfinite(rho) && isfinite(p) && isfinite(v[1]) && isfinite(v[2]) &&
                      isfinite(v[3]);
      bad += !ok;
    }
  }
  add_bad(P, bad);
}

// Assembly pass of the compacted per-cell hybrid: the node derivative from the interface
// fluxes of every direction, where an interface touching the dilated troubled set
// (ft_i | ft_{i+1}) takes the C-GBR flux the queue pass stored at its left node and every
// other interface the I4 interpolation of the LAD node fluxes; then dQ/dt or the RK stage.
// The same z-marching layout as the all-LAD pass (zeta node fluxes in a register queue).
template <typename R, bool O32>
__global__ void __launch_bounds__(256) k_hyb_assemble(const Prob* __restrict__ probs, StateRef ref, RKRef rr,
                                                      int mode, int stage, double a, double b, int zc) {
  using IX = sidx_t<O32>;
  const Prob& P = probs[blockIdx.y];
  if (lad_skip(P, GATE_MIXED)) return;
  ZCol c;
  if (!zm_column(P, 0, 0, zc, c)) return;
  const IX T = (IX)P.total;
  const int sz = P.s[2];
  const bool z3 = P.ndim == 3;
  const R* Fz = static_cast<const R*>(P.FL[2]);
  const uint8_t* ft = P.ft;
  double* dQ = ref.deriv(P);
  const double* Un = rr.Un ? rr.Un : P.Q;
  const double* Us = rr.Us ? rr.Us : (stage == 0 ? Un : P.Us);
  double* out = rr.out ? rr.out : (stage == 2 ? const_cast<double*>(Un) : P.Us);
  const double dt = mode ? *P.dt : 0.0;
  int bad = 0;
  int idx = pos_to_idx(P, c.i, c.j, c.k0);
  R qz[5][5];   // planes k-2 .. k+2 of the zeta node fluxes
  if (z3)
    for (int p = 1; p < 5; ++p)
      for (int q = 0; q < 5; ++q) qz[p][q] = gld<R, O32>(Fz, (IX)q * T + (IX)(idx + (p - 3) * sz));
  int fz_m = z3 ? ft[idx - sz] : 0;   // flag of plane k-1
  const bool mplane = P.met_planar;
  const double Jcol = met64(P, 9, idx);
  for (int k = c.k0; k < c.k1; ++k, idx += sz) {
    if (z3) {
      for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 5; ++q) qz[p][q] = qz[p + 1][q];
      for (int q = 0; q < 5; ++q) qz[4][q] = gld<R, O32>(Fz, (IX)q * T + (IX)(idx + 2 * sz));
    }
    const double J = mplane ? Jcol : met64(P, 9, idx);
    const int f0 = ft[idx];
    double Lq[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    // xi and eta: the five-point stencil of the node fluxes gives both I4 interfaces
    for (int d = 0; d < 2; ++d) {
      if (d >= P.ndim) break;
      const int s = P.s[d];
      const bool gp = (f0 | ft[idx + s]) != 0, gm = (ft[idx - s] | f0) != 0;
      const R* F = static_cast<const R*>(P.FL[d]);
      const R* G = static_cast<const R*>(P.FG[d]);
      const IX si = (IX)s;
      for (int q = 0; q < 5; ++q) {
        const IX o = (IX)q * T + (IX)idx;
        R fp, fm;
        if (gp && gm) {
          fp = gld<R, O32>(G, o);
          fm = gld<R, O32>(G, o - si);
        } else {
          const R m2 = gld<R, O32>(F, o - 2 * si), m1 = gld<R, O32>(F, o - si), c0 = gld<R, O32>(F, o),
                  p1 = gld<R, O32>(F, o + si), p2 = gld<R, O32>(F, o + 2 * si);
          fp = gp ? gld<R, O32>(G, o) : i4v(m1, c0, p1, p2);
          fm = gm ? gld<R, O32>(G, o - si) : i4v(m2, m1, c0, p1);
        }
        Lq[q] = Lq[q] + -J * ((double)fp - (double)fm);
      }
    }
    if (z3) {
      const int fz_p = ft[idx + sz];
      const bool gp = (f0 | fz_p) != 0, gm = (fz_m | f0) != 0;
      const R* G = static_cast<const R*>(P.FG[2]);
      for (int q = 0; q < 5; ++q) {
        const IX o = (IX)q * T + (IX)idx;
        const R fp = gp ? gld<R, O32>(G, o) : i4v(qz[1][q], qz[2][q], qz[3][q], qz[4][q]);
        const R fm = gm ? gld<R, O32>(G, o - (IX)sz) : i4v(qz[0][q], qz[1][q], qz[2][q], qz[3][q]);
        Lq[q] = Lq[q] + -J * ((double)fp - (double)fm);
      }
      fz_m = f0;
    }
    if (mode == 0) {
      for (int q = 0; q < 5; ++q) gst<double, O32>(dQ, (IX)q * T + (IX)idx, Lq[q]);
    } else {
      double v[5];
      for (int q = 0; q < 5; ++q) {
        const IX o = (IX)q * T + (IX)idx;
        v[q] = a * gld<double, O32>(Un, o) + b * (gld<double, O32>(Us, o) + dt * Lq[q]);
        gst<double, O32>(out, o, v[q]);
      }
      const double rho = v[0];
      const double ke = 0.5 * (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / rho;
      const double p = (P.gamma - 1.0) * (v[4] - ke);
      const bool ok = rho > 0.0 && p > 0.0 && isfinite(rho) && isfinite(p) && isfinite(v[1]) && isfinite(v[2]) &&
                      isfinite(v[3]);
      bad += !ok;
    }
  }
  add_bad(P, bad);
}

// Ghost nodes of the stage result = U^n, as the combination kernel does off the interior.
// Inside rk3_step (no explicit output) only the ghosts of FIXED faces are copied: every
// other ghost is rewritten from the interior before the next stage reads it.
__global__ void __launch_bounds__(256) k_stage_ghosts(const Prob* __restrict__ probs, RKRef rr, int stage,
                                                      int skip_if_any) {
  const Prob& P = probs[blockIdx.y];
  if (lad_skip(P, skip_if_any)) return;
  const double* Un = rr.Un ? rr.Un : P.Q;
  double* out = rr.out ? rr.out : (stage == 2 ? const_cast<double*>(Un) : P.Us);
  if (out == Un) return;
  const bool all = rr.out != nullptr;
  const size_t T = P.total;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < P.total; idx += gridDim.x * blockDim.x) {
    const int p[3] = {idx % P.N[0], (idx / P.N[0]) % P.N[1], idx / (P.N[0] * P.N[1])};
    bool ghost = false, fixed = false;
    for (int d = 0; d < P.ndim; ++d) {
      const bool lo = p[d] < P.g[d], hi = p[d] >= P.g[d] + P.n[d];
      ghost |= lo || hi;
      fixed |= (lo && P.bc[d][0] == BC_FIXED) || (hi && P.bc[d][1] == BC_FIXED);
    }
    if (!ghost || !(all || fixed)) continue;
    for (int q = 0; q < 5; ++q) out[q * T + idx] = Un[q * T + idx];
  }
}

// Classic RK4 (the LAD scheme's alternative integrator, Sec. 2.1): with k_s the right-hand
// side of stage s (in the derivative workspace), acc = acc + b_s dt k_s (acc = b_0 dt k_0 at
// s = 0); s < 3: the next stage input U^n + c_s dt k_s into the stage buffer; s = 3: U^{n+1} =
// U^n + acc in place of U^n.  Interior nodes; non-physical results are counted.
__global__ void __launch_bounds__(256) k_rk4_combine(const Prob* __restrict__ probs, const double* Unx, int stage,
                                                     double b, double c) {
  const Prob& P = probs[blockIdx.y];
  const double* Un = Unx ? Unx : P.Q;
  double* out = stage < 3 ? P.Us : const_cast<double*>(Un);
  const double* k = P.dQ;
  double* acc = P.acc;
  const size_t T = P.total;
  const double dt = *P.dt;
  const double bdt = b * dt, cdt = c * dt;
  int bad = 0;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < P.total; idx += gridDim.x * blockDim.x) {
    if (!is_interior(P, idx)) continue;
    double v[5];
    for (int q = 0; q < 5; ++q) {
      const size_t o = q * T + idx;
      const double kq = k[o];
      const double a = (stage == 0 ? 0.0 : acc[o]) + bdt * kq;
      if (stage < 3) {
        acc[o] = a;
        v[q] = Un[o] + cdt * kq;
      } else {
        v[q] = Un[o] + a;
      }
      out[o] = v[q];
    }
    const double rho = v[0];
    const double p = (P.gamma - 1.0) * (v[4] - 0.5 * (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / rho);
    bad += !(rho > 0.0 && p > 0.0 && isfinite(rho) && isfinite(p));
  }
  add_bad(P, bad);
}

// The ghost layers of the FIXED faces along d (all positions of the other directions):
// the only ghosts a stage inside rk3_step must carry over from U^n.
// (rr.out null: the stage's own result buffer.)
__global__ void __launch_bounds__(256) k_fixed_ghosts(const Prob* __restrict__ probs, RKRef rr, int stage,
                                                      int skip_if_any, int d) {
  const Prob& P = probs[blockIdx.y];
  if (lad_skip(P, skip_if_any) || d >= P.ndim) return;
  const double* Un = rr.Un ? rr.Un : P.Q;
  double* out = stage == 2 ? const_cast<double*>(Un) : P.Us;
  if (out == Un) return;
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const int g = P.g[d], n1 = P.N[o1], n2 = P.N[o2];
  const long long slab = (long long)g * n1 * n2;
  const size_t T = P.total;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < 2 * slab;
       t += (long long)gridDim.x * blockDim.x) {
    const int side = t >= slab;
    if (P.bc[d][side] != BC_FIXED) continue;
    const long long r = t - side * slab;
    const int a = (int)(r % g), b = (int)((r / g) % n1), c = (int)(r / ((long long)g * n1));
    const int pd = side ? g + P.n[d] + a : a;
    int pos[3];
    pos[d] = pd;
    pos[o1] = b;
    pos[o2] = c;
    const size_t idx = (size_t)pos[0] * P.s[0] + (size_t)pos[1] * P.s[1] + (size_t)pos[2] * P.s[2];
    for (int q = 0; q < 5; ++q) out[q * T + idx] = Un[q * T + idx];
  }
}

// C-GBR viscous node fluxes (physical coefficients, the scheme's gradients)
template <typename R>
__global__ void __launch_bounds__(256) k_gbr_viscflux(const Prob* __restrict__ probs, int skip_if_any, int region) {
  const Prob& P = probs[blockIdx.y];
  if (lad_skip(P, skip_if_any)) return;
  const R* W = static_cast<const R*>(P.W);
  const size_t T = P.total;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < P.total; idx += gridDim.x * blockDim.x) {
    if (!in_band(P, idx, -2, 2)) continue;
    if (region && !P.fg[idx]) continue;
    R w[5];
    for (int q = 0; q < 5; ++q) w[q] = W[q * T + idx];
    R gl[3][5], D[5][3], mt[10];
    for (int l = 0; l < 3; ++l)
      for (int q = 0; q < 5; ++q) gl[l][q] = l < P.ndim ? static_cast<const R*>(P.G[l])[q * T + idx] : R(0);
    load_met(P, idx, mt);
    to_physical(P.ndim, mt, gl, D);
    const R ri = rcp(w[0]);
    R mu, kappa;
    transport(P, ri, w[4], mu, kappa);
    #pragma unroll
    for (int l = 0; l < 3; ++l) {
      if (l >= P.ndim) break;
      R F[5];
      viscous_flux(P, mt[3 * l], mt[3 * l + 1], mt[3 * l + 2], w, ri, D, mu, R(0), kappa, F);
      R* out = static_cast<R*>(P.FV[l]);
      for (int q = 0; q < 5; ++q) out[q * T + idx] = F[q];
    }
  }
}

static inline dim3 g1(long long work, int nprob, long long cap = 1LL << 30) {
  long long b = (work + 255) / 256;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return dim3((unsigned)b, nprob);
}

void launch_rk4_combine(const Launch& L, double* Un, int stage, double b, double c) {
  LG_TIMED(L, KC_COMBINE, hipLaunchKernelGGL(k_rk4_combine, g1(L.max_total, L.nprob, 1 << 16), dim3(256), 0, L.stream,
                                             L.probs, Un, stage, b, c));
}


template <typename R>
void launch_lad(const Launch& L, int skip_if_any, int cg) {
  const int zb = zm_arg(L, -2, 2), zi = zm_arg(L, 0, 0);
  if (cg) {
    LG_TIMED(L, KC_LAD_NODE, hipLaunchKernelGGL((k_lad_shear<R, true>), zm_grid_col(L, -2, 2), dim3(256),
                                                0, L.stream, L.probs, skip_if_any, zb));
    LG_TIMED(L, KC_LAD_RAW, hipLaunchKernelGGL((k_lad_raw<R, true, false>), zm_grid_col(L, 0, 0), dim3(256), 0,
                                               L.stream, L.probs, skip_if_any, zi));
  } else {
    LG_TIMED(L, KC_LAD_NODE, hipLaunchKernelGGL((k_lad_shear<R, false>), zm_grid_col(L, -2, 2), dim3(256),
                                                0, L.stream, L.probs, skip_if_any, zb));
    // the specialised geometry: FP32 1.50x faster on the ramp; FP64 needs 256 registers
    // that way and runs slower
    if (sizeof(R) == 4 && !L.geo_generic)
      LG_TIMED(L, KC_LAD_RAW, hipLaunchKernelGGL((k_lad_raw<R, false, true>), zm_grid_col(L, 0, 0), dim3(256), 0,
                                                 L.stream, L.probs, skip_if_any, zi));
    else
      LG_TIMED(L, KC_LAD_RAW, hipLaunchKernelGGL((k_lad_raw<R, false, false>), zm_grid_col(L, 0, 0), dim3(256), 0,
                                                 L.stream, L.probs, skip_if_any, zi));
  }
  constexpr int GTY = sizeof(R) == 4 ? 16 : 8;
  LG_TIMED(L, KC_GAUSS, hipLaunchKernelGGL((k_gauss_xy<R, GTY>), zm_grid(L, 0, 0, 64, GTY), dim3(256), 0, L.stream,
                                           L.probs, skip_if_any, zm_chunk(L, 0, 0)));
  if (L.ndim > 2)
    LG_TIMED(L, KC_GAUSS, hipLaunchKernelGGL(k_gauss_z<R>, zm_grid_col(L, 0, 0), dim3(256), 0, L.stream,
                                             L.probs, skip_if_any, zi));
}

// the filtered coefficients end in CA after the zeta pass (3D), in CB otherwise
static inline int lad_coef_buf(const Launch& L) { return L.ndim > 2 ? 0 : 1; }

template <typename R>
void launch_lad_nodeflux(const Launch& L, int skip_if_any, int cg) {
  const dim3 grid = zm_grid_col(L, -2, 2);
  const int zb = zm_arg(L, -2, 2);
  // FP32: 32-bit element offsets, general geometry (3 % faster on the ramp than generic
  // addressing, the specialised geometry slower); FP64: generic addressing, the specialised
  // geometry where it applies (6 % faster)
  const bool o32 = sizeof(R) == 4 && !L.o64;
  if (cg)
    LG_TIMED(L, KC_LAD_FLUX, hipLaunchKernelGGL((k_lad_nodeflux<R, true, false, false>), grid, dim3(256), 0,
                                                L.stream, L.probs, lad_coef_buf(L), skip_if_any, zb));
  else if (o32)
    LG_TIMED(L, KC_LAD_FLUX, hipLaunchKernelGGL((k_lad_nodeflux<R, false, true, false>), grid, dim3(256), 0,
                                                L.stream, L.probs, lad_coef_buf(L), skip_if_any, zb));
  else if (sizeof(R) == 8 && !L.geo_generic)
    LG_TIMED(L, KC_LAD_FLUX, hipLaunchKernelGGL((k_lad_nodeflux<R, false, false, true>), grid, dim3(256), 0,
                                                L.stream, L.probs, lad_coef_buf(L), skip_if_any, zb));
  else
    LG_TIMED(L, KC_LAD_FLUX, hipLaunchKernelGGL((k_lad_nodeflux<R, false, false, false>), grid, dim3(256), 0,
                                                L.stream, L.probs, lad_coef_buf(L), skip_if_any, zb));
}

template <typename R>
void launch_lad_geometry(const Launch& L) {
  hipLaunchKernelGGL(k_lad_dx<R>, g1(L.max_total, L.nprob), dim3(256), 0, L.stream, L.probs);
}

template <typename R>
void launch_lad_sweep(const Launch& L, StateRef ref, const RKRef* rr, int stage, double a, double b, int skip_if_any) {
  RKRef r = rr ? *rr : RKRef{nullptr, nullptr, nullptr};
  const dim3 grid = zm_grid_col(L, 0, 0);
  // FP32 fluxes: 115 registers with 32-bit offsets (4 waves per SIMD), 7 % faster on the
  // ramp; FP64 needs 164 that way (3 waves) and runs faster with generic addressing
  if (sizeof(R) == 4 && !L.o64)
    LG_TIMED(L, KC_LAD_SWEEP, hipLaunchKernelGGL((k_lad_sweep<R, true>), grid, dim3(256), 0, L.stream, L.probs, ref,
                                                 r, rr ? 1 : 0, stage, a, b, skip_if_any, zm_arg(L, 0, 0)));
  else
    LG_TIMED(L, KC_LAD_SWEEP, hipLaunchKernelGGL((k_lad_sweep<R, false>), grid, dim3(256), 0, L.stream, L.probs, ref,
                                                 r, rr ? 1 : 0, stage, a, b, skip_if_any, zm_arg(L, 0, 0)));
  if (rr) launch_stage_ghosts(L, *rr, stage, skip_if_any);
}

template <typename R>
void launch_hyb_assemble(const Launch& L, StateRef ref, const RKRef* rr, int stage, double a, double b) {
  RKRef r = rr ? *rr : RKRef{nullptr, nullptr, nullptr};
  const dim3 grid = zm_grid_col(L, 0, 0);
  if (sizeof(R) == 4 && !L.o64)
    LG_TIMED(L, KC_HYB_ASSEMBLE, hipLaunchKernelGGL((k_hyb_assemble<R, true>), grid, dim3(256), 0, L.stream, L.probs,
                                                    ref, r, rr ? 1 : 0, stage, a, b, zm_arg(L, 0, 0)));
  else
    LG_TIMED(L, KC_HYB_ASSEMBLE, hipLaunchKernelGGL((k_hyb_assemble<R, false>), grid, dim3(256), 0, L.stream, L.probs,
                                                    ref, r, rr ? 1 : 0, stage, a, b, zm_arg(L, 0, 0)));
  if (rr) launch_stage_ghosts(L, *rr, stage, GATE_MIXED);
}

void launch_stage_ghosts(const Launch& L, const RKRef& rr, int stage, int skip_if_any) {
  if (rr.out) {   // an explicit output: every ghost of the result
    LG_TIMED(L, KC_COMBINE, hipLaunchKernelGGL(k_stage_ghosts, g1(L.max_total, L.nprob), dim3(256), 0, L.stream,
                                               L.probs, rr, stage, skip_if_any));
    return;
  }
  if (!L.has_fixed) return;
  for (int d = 0; d < L.ndim; ++d)   // the FIXED faces' layers only
    LG_TIMED(L, KC_COMBINE, hipLaunchKernelGGL(k_fixed_ghosts, g1(L.ghost_work[d], L.nprob), dim3(256), 0, L.stream,
                                               L.probs, rr, stage, skip_if_any, d));
}

template <typename R>
void launch_gbr_viscflux(const Launch& L, int skip_if_any, int region) {
  LG_TIMED(L, KC_VISC, hipLaunchKernelGGL(k_gbr_viscflux<R>, g1(L.max_total, L.nprob, 16384), dim3(256), 0, L.stream,
                                          L.probs, skip_if_any, region));
}

template void launch_lad<float>(const Launch&, int, int);
template void launch_lad<double>(const Launch&, int, int);
template void launch_lad_geometry<float>(const Launch&);
template void launch_lad_geometry<double>(const Launch&);
template void launch_hyb_assemble<float>(const Launch&, StateRef, const RKRef*, int, double, double);
template void launch_hyb_assemble<double>(const Launch&, StateRef, const RKRef*, int, double, double);
template void launch_lad_sweep<float>(const Launch&, StateRef, const RKRef*, int, double, double, int);
template void launch_lad_sweep<double>(const Launch&, StateRef, const RKRef*, int, double, double, int);
template void launch_lad_nodeflux<float>(const Launch&, int, int);
template void launch_lad_nodeflux<double>(const Launch&, int, int);
template void launch_gbr_viscflux<float>(const Launch&, int, int);
template void launch_gbr_viscflux<double>(const Launch&, int, int);

}  // namespace lg
