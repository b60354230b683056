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
// node fluxes F^c + F^v are stored here and interpolated in the interface sweep.
// Fourth differences use five points; all derivatives use unit computational spacing.
#include "lgbr_dev.h"
#include "lgbr_kernels.h"

namespace lg {

__device__ __forceinline__ bool lad_skip(const Prob& P, int skip_if_any) {
  return skip_if_any >= 0 && P.any_flag && (*P.any_flag != 0) == (skip_if_any != 0);
}

template <typename R>
__device__ __forceinline__ R e4_at(const R* f, int idx, int s) {
  return (R(8) * (f[idx + s] - f[idx - s]) - (f[idx + 2 * s] - f[idx - 2 * s])) / R(12);
}

// physical gradients D[q][j] of the 5 primitives at node idx from computational
// derivatives gl[l][q] (l < ndim)
template <typename R>
__device__ __forceinline__ void to_physical(const Prob& P, int idx, const R gl[3][5], R D[5][3]) {
  R J = met<R>(P, 9, idx);
  for (int q = 0; q < 5; ++q)
    for (int j = 0; j < 3; ++j) D[q][j] = R(0);
  for (int l = 0; l < P.ndim; ++l)
    for (int j = 0; j < 3; ++j) {
      R m = J * met<R>(P, 3 * l + j, idx);
      for (int q = 0; q < 5; ++q) D[q][j] += m * gl[l][q];
    }
}

template <typename R>
__device__ __forceinline__ void e4_grads(const Prob& P, const R* W, int idx, R gl[3][5]) {
  const size_t T = P.total;
  for (int l = 0; l < 3; ++l)
    for (int q = 0; q < 5; ++q) gl[l][q] = R(0);
  for (int l = 0; l < P.ndim; ++l)
    for (int q = 0; q < 5; ++q) gl[l][q] = e4_at(W + q * T, idx, P.s[l]);
}

template <typename R>
__device__ __forceinline__ void transport(const Prob& P, R rho, R p, R& mu, R& kappa) {
  if (!P.viscous) {
    mu = R(0);
    kappa = R(0);
    return;
  }
  R T = R(P.gamma * P.Mref * P.Mref) * p / rho;
  R S = (R)P.suth;
  mu = T * sqrt(T) * (R(1) + S) / (T + S) / R(P.Re);
  kappa = mu / R((P.gamma - 1.0) * P.Pr * P.Mref * P.Mref);
}

// -l_hat . [0, tau, phi] at node idx (Eq. tauij)
template <typename R>
__device__ __forceinline__ void viscous_flux(const Prob& P, int idx, int l, const R w[5], const R D[5][3],
                                             R mu, R beta, R kappa, R F[5]) {
  R du[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) du[i][j] = D[1 + i][j];
  R theta = du[0][0] + du[1][1] + du[2][2];
  R g2 = R(P.gamma * P.Mref * P.Mref);
  R rho = w[0], p = w[4];
  R tau[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      tau[i][j] = mu * (du[i][j] + du[j][i]);
      if (i == j) tau[i][j] += (beta - R(2.0 / 3.0) * mu) * theta;
    }
  R phi[3];
  for (int i = 0; i < 3; ++i) {
    R dT = g2 * (D[4][i] / rho - p * D[0][i] / (rho * rho));
    phi[i] = w[1] * tau[i][0] + w[2] * tau[i][1] + w[3] * tau[i][2] + kappa * dT;
  }
  R m0 = met<R>(P, 3 * l, idx), m1 = met<R>(P, 3 * l + 1, idx), m2 = met<R>(P, 3 * l + 2, idx);
  F[0] = R(0);
  for (int i = 0; i < 3; ++i) F[1 + i] = -(m0 * tau[i][0] + m1 * tau[i][1] + m2 * tau[i][2]);
  F[4] = -(m0 * phi[0] + m1 * phi[1] + m2 * phi[2]);
}

__device__ __forceinline__ bool in_band(const Prob& P, int idx, int lo, int hi) {
  int p[3] = {idx % P.N[0], (idx / P.N[0]) % P.N[1], idx / (P.N[0] * P.N[1])};
  for (int l = 0; l < P.ndim; ++l)
    if (p[l] < P.g[l] + lo || p[l] >= P.g[l] + P.n[l] + hi) return false;
  return true;
}

__device__ __forceinline__ bool is_interior(const Prob& P, int idx) { return in_band(P, idx, 0, 0); }

// E4 physical gradients D (stored for the raw coefficients and the node fluxes) and
// |S|, div u, e at every node where E4 fits (positions -3 .. n+2)
template <typename R>
__global__ void __launch_bounds__(256) k_lad_grad(const Prob* __restrict__ probs, int skip_if_any) {
  const Prob& P = probs[blockIdx.y];
  if (lad_skip(P, skip_if_any)) return;
  const R* W = static_cast<const R*>(P.W);
  R* S3 = static_cast<R*>(P.S3);
  R* DD = static_cast<R*>(P.D4);
  const size_t T = P.total;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < P.total; idx += gridDim.x * blockDim.x) {
    if (!in_band(P, idx, -3, 3)) continue;
    R gl[3][5], D[5][3];
    e4_grads(P, W, idx, gl);
    to_physical(P, idx, gl, D);
    for (int q = 0; q < 5; ++q)
      for (int j = 0; j < 3; ++j) DD[(size_t)(3 * q + j) * T + idx] = D[q][j];
    R S2 = R(0);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        R sij = R(0.5) * (D[1 + i][j] + D[1 + j][i]);
        S2 += sij * sij;
      }
    R rho = W[idx], p = W[4 * T + idx];
    S3[idx] = sqrt(S2);
    S3[T + idx] = D[1][0] + D[2][1] + D[3][2];
    S3[2 * T + idx] = p / (R(P.gamma - 1.0) * rho);
  }
}

template <typename R>
__device__ __forceinline__ void load_D(const Prob& P, int idx, R D[5][3]) {
  const R* DD = static_cast<const R*>(P.D4);
  const size_t T = P.total;
  for (int q = 0; q < 5; ++q)
    for (int j = 0; j < 3; ++j) D[q][j] = DD[(size_t)(3 * q + j) * T + idx];
}

template <typename R>
__device__ __forceinline__ R delta4(const R* f, int idx, int s) {
  return f[idx - 2 * s] - R(4) * f[idx - s] + R(6) * f[idx] - R(4) * f[idx + s] + f[idx + 2 * s];
}

// raw (unfiltered) coefficients at interior nodes
template <typename R>
__global__ void __launch_bounds__(256) k_lad_raw(const Prob* __restrict__ probs, int skip_if_any) {
  const Prob& P = probs[blockIdx.y];
  if (lad_skip(P, skip_if_any)) return;
  const R* W = static_cast<const R*>(P.W);
  const R* S3 = static_cast<const R*>(P.S3);
  R* C = static_cast<R*>(P.CA);
  const size_t T = P.total;
  const R gm1 = R(P.gamma - 1.0);
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < P.total; idx += gridDim.x * blockDim.x) {
    if (!is_interior(P, idx)) continue;
    R D[5][3];
    load_D(P, idx, D);
    R rho = W[idx], p = W[4 * T + idx];
    R theta = D[1][0] + D[2][1] + D[3][2];
    R w1 = D[3][1] - D[2][2], w2 = D[1][2] - D[3][0], w3 = D[2][0] - D[1][1];
    R om2 = w1 * w1 + w2 * w2 + w3 * w3;
    R de[3], gr[3];
    for (int j = 0; j < 3; ++j) {
      de[j] = (D[4][j] / rho - p * D[0][j] / (rho * rho)) / gm1;
      gr[j] = D[0][j];
    }
    R nr = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]) + R(1e-32);
    R ne = sqrt(de[0] * de[0] + de[1] * de[1] + de[2] * de[2]) + R(1e-32);
    R Tt = R(P.gamma * P.Mref * P.Mref) * p / rho;
    R c = sqrt(R(P.gamma) * p / rho);
    R fsw = theta < R(0) ? theta * theta / (theta * theta + om2 + R(1e-32)) : R(0);
    R smu = R(0), sbeta = R(0), skap = R(0);
    for (int l = 0; l < P.ndim; ++l) {
      R dx[3];
      if (P.curvilinear) {
        for (int cc = 0; cc < 3; ++cc) {
          const double* X = P.coords + (size_t)cc * T;
          dx[cc] = (R)(0.5 * (X[idx + P.s[l]] - X[idx - P.s[l]]));
        }
      } else {
        dx[0] = dx[1] = dx[2] = R(0);
        dx[l] = (R)P.h[l];
      }
      R dmu2 = dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2];
      R dbeta = (dx[0] * gr[0] + dx[1] * gr[1] + dx[2] * gr[2]) / nr;
      R dkap = fabs(dx[0] * de[0] + dx[1] * de[1] + dx[2] * de[2]) / ne;
      smu += delta4(S3, idx, P.s[l]) * dmu2;
      sbeta += delta4(S3 + T, idx, P.s[l]) * dbeta * dbeta;
      skap += delta4(S3 + 2 * T, idx, P.s[l]) * dkap;
    }
    C[idx] = R(P.C_mu) * rho * fabs(smu);
    C[T + idx] = R(P.C_beta) * rho * fsw * fabs(sbeta);
    C[2 * T + idx] = R(P.C_kappa) * rho * c / Tt * fabs(skap);
  }
}

// one truncated-Gaussian pass along d at interior nodes (3 fields)
template <typename R>
__global__ void __launch_bounds__(256) k_gauss(const Prob* __restrict__ probs, int d, int src, int skip_if_any) {
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || lad_skip(P, skip_if_any)) return;
  const R* in = static_cast<const R*>(src == 0 ? P.CA : P.CB);
  R* out = static_cast<R*>(src == 0 ? P.CB : P.CA);
  const size_t T = P.total;
  const R w0 = R(3565.0 / 10368.0), w1 = R(3091.0 / 12960.0), w2 = R(1997.0 / 25920.0),
          w3 = R(149.0 / 12960.0), w4 = R(107.0 / 103680.0);
  const int s = P.s[d];
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < P.total; idx += gridDim.x * blockDim.x) {
    if (!is_interior(P, idx)) continue;
    for (int q = 0; q < 3; ++q) {
      const R* f = in + q * T + idx;
      R v = w0 * f[0];
      v = v + w1 * (f[s] + f[-s]);
      v = v + w2 * (f[2 * s] + f[-2 * s]);
      v = v + w3 * (f[3 * s] + f[-3 * s]);
      v = v + w4 * (f[4 * s] + f[-4 * s]);
      out[q * T + idx] = v;
    }
  }
}

// LAD node fluxes F^c + F^v for every active direction at positions -2 .. n+1
template <typename R>
__global__ void __launch_bounds__(256) k_lad_nodeflux(const Prob* __restrict__ probs, int coef_buf, int skip_if_any) {
  const Prob& P = probs[blockIdx.y];
  if (lad_skip(P, skip_if_any)) return;
  const R* W = static_cast<const R*>(P.W);
  const R* C = static_cast<const R*>(coef_buf == 0 ? P.CA : P.CB);
  const size_t T = P.total;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < P.total; idx += gridDim.x * blockDim.x) {
    if (!in_band(P, idx, -2, 2)) continue;
    R w[5];
    for (int q = 0; q < 5; ++q) w[q] = W[q * T + idx];
    R D[5][3];
    load_D(P, idx, D);
    R muf, kapf;
    transport(P, w[0], w[4], muf, kapf);
    R mu = muf + C[idx], beta = C[T + idx], kappa = kapf + C[2 * T + idx];
    R E = w[4] / R(P.gamma - 1.0) + R(0.5) * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
    for (int l = 0; l < P.ndim; ++l) {
      R F[5];
      viscous_flux(P, idx, l, w, D, mu, beta, kappa, F);
      R m0 = met<R>(P, 3 * l, idx), m1 = met<R>(P, 3 * l + 1, idx), m2 = met<R>(P, 3 * l + 2, idx);
      R U = m0 * w[1] + m1 * w[2] + m2 * w[3];
      R* out = static_cast<R*>(P.FL[l]);
      out[idx] = w[0] * U + F[0];
      out[T + idx] = w[0] * w[1] * U + m0 * w[4] + F[1];
      out[2 * T + idx] = w[0] * w[2] * U + m1 * w[4] + F[2];
      out[3 * T + idx] = w[0] * w[3] * U + m2 * w[4] + F[3];
      out[4 * T + idx] = (E + w[4]) * U + F[4];
    }
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
    R gl[3][5], D[5][3];
    for (int l = 0; l < 3; ++l)
      for (int q = 0; q < 5; ++q) gl[l][q] = l < P.ndim ? static_cast<const R*>(P.G[l])[q * T + idx] : R(0);
    to_physical(P, idx, gl, D);
    R mu, kappa;
    transport(P, w[0], w[4], mu, kappa);
    for (int l = 0; l < P.ndim; ++l) {
      R F[5];
      viscous_flux(P, idx, l, w, D, mu, R(0), kappa, F);
      R* out = static_cast<R*>(P.FV[l]);
      for (int q = 0; q < 5; ++q) out[q * T + idx] = F[q];
    }
  }
}

static inline dim3 g1(long long work, int nprob) {
  long long b = (work + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return dim3((unsigned)b, nprob);
}

template <typename R>
void launch_lad(const Launch& L, int skip_if_any) {
  LG_TIMED(L, KC_LAD_NODE, hipLaunchKernelGGL(k_lad_grad<R>, g1(L.max_total, L.nprob), dim3(256), 0, L.stream,
                                              L.probs, skip_if_any));
  LG_TIMED(L, KC_LAD_RAW, hipLaunchKernelGGL(k_lad_raw<R>, g1(L.max_total, L.nprob), dim3(256), 0, L.stream,
                                             L.probs, skip_if_any));
  for (int d = 0; d < L.ndim; ++d) launch_bc_scalar<R>(L, 0, 3, d);
  int src = 0;
  for (int d = 0; d < L.ndim; ++d) {
    LG_TIMED(L, KC_GAUSS, hipLaunchKernelGGL(k_gauss<R>, g1(L.max_total, L.nprob), dim3(256), 0, L.stream,
                                             L.probs, d, src, skip_if_any));
    src ^= 1;
    for (int e = 0; e < L.ndim; ++e) launch_bc_scalar<R>(L, src, 3, e);
  }
  LG_TIMED(L, KC_LAD_FLUX, hipLaunchKernelGGL(k_lad_nodeflux<R>, g1(L.max_total, L.nprob), dim3(256), 0,
                                              L.stream, L.probs, src, skip_if_any));
}

template <typename R>
void launch_gbr_viscflux(const Launch& L, int skip_if_any, int region) {
  LG_TIMED(L, KC_VISC, hipLaunchKernelGGL(k_gbr_viscflux<R>, g1(L.max_total, L.nprob), dim3(256), 0, L.stream,
                                          L.probs, skip_if_any, region));
}

template void launch_lad<float>(const Launch&, int);
template void launch_lad<double>(const Launch&, int);
template void launch_gbr_viscflux<float>(const Launch&, int, int);
template void launch_gbr_viscflux<double>(const Launch&, int, int);

}  // namespace lg
