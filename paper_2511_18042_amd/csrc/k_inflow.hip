// Digital-filter inflow turbulence (Sec. 4: the 3D cases' inflow; digital filters with
// per-component length scales in two wall-normal zones, strong Reynolds analogy).
//
// One update: zeta filter of the caller's normal numbers (periodic), eta filter with the
// row's coefficients and time correlation, then the inflow state written into every
// ghost layer of the low-xi face.  Coefficients, zones and the Cholesky factors of the
// Reynolds stresses are host tables.  FP64 throughout; one lane per output value.
#include "lgbr_dev.h"
#include "lgbr_kernels.h"

#include <algorithm>

namespace lg {

// rz[c][jp][k] = sum_l bz_c(l) rnd[c][jp][(k + l) mod nz]
__global__ void __launch_bounds__(256) k_df_zeta(DFDev D, const double* __restrict__ rnd) {
  const int rows = D.ny + 2 * D.pad;
  const long long cnt = 3LL * rows * D.nz;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < cnt; t += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(t % D.nz);
    const long long r = t / D.nz;
    const int c = (int)(r / rows);
    const double* row = rnd + r * D.nz;
    const double* b = D.bz + (size_t)c * (2 * D.nzmax + 1) + D.nzmax;
    const int h = D.nzh[c];
    double acc = 0.0;
    for (int l = -h; l <= h; ++l) {
      int kk = (k + l) % D.nz;
      kk = kk < 0 ? kk + D.nz : kk;
      acc = acc + b[l] * row[kk];
    }
    D.rz[t] = acc;
  }
}

// psi[c][j][k]: eta filter of rz at the row's coefficients, correlated in time
__global__ void __launch_bounds__(256) k_df_eta(DFDev D, const Prob* __restrict__ probs, double dt, int first) {
  const Prob& P = probs[0];
  const int rows = D.ny + 2 * D.pad;
  const long long cnt = 3LL * D.ny * D.nz;
  const double dtv = dt < 0.0 ? *P.dt : dt;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < cnt; t += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(t % D.nz);
    const long long r = t / D.nz;
    const int j = (int)(r % D.ny), c = (int)(r / D.ny);
    const double* b = D.by + ((size_t)c * D.ny + j) * (2 * D.pad + 1) + D.pad;
    const double* z = D.rz + (size_t)c * rows * D.nz;
    const int h = D.nyh[c * D.ny + j];
    double acc = 0.0;
    for (int i = -h; i <= h; ++i) acc = acc + b[i] * z[(size_t)(D.pad + j + i) * D.nz + k];
    if (first) {
      D.psi[t] = acc;
    } else {
      const double T = D.Tc[c];
      D.psi[t] = D.psi[t] * exp(-M_PI * dtv / (2.0 * T)) + acc * sqrt(1.0 - exp(-M_PI * dtv / T));
    }
  }
}

// the inflow state into every ghost layer of the low-xi face (interior eta, zeta)
__global__ void __launch_bounds__(256) k_df_ghosts(DFDev D, const Prob* __restrict__ probs, double* Q) {
  const Prob& P = probs[0];
  const size_t T = P.total;
  const long long cnt = (long long)D.ny * D.nz;
  const size_t pl = (size_t)D.ny * D.nz;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < cnt; t += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(t % D.nz), j = (int)(t / D.nz);
    const double a11 = D.a[j], a21 = D.a[D.ny + j], a22 = D.a[2 * D.ny + j], a33 = D.a[3 * D.ny + j];
    const double pu = D.psi[t], pv = D.psi[pl + t], pw = D.psi[2 * pl + t];
    const double up = a11 * pu, vp = a21 * pu + a22 * pv, wp = a33 * pw;
    // T'/T by the strong Reynolds analogy at the local mean Mach number
    const double Um = D.mean[D.ny + j], Tm = D.mean[3 * D.ny + j];
    const double tr = -D.gm1 * D.M2 * Um * up / (D.U_ref * D.U_ref * Tm);
    const double rho = D.mean[j] * (1.0 - tr);
    const double u = Um + up, v = D.mean[2 * D.ny + j] + vp, w = wp;
    const double cons[5] = {rho, rho * u, rho * v, rho * w, D.p / D.gm1 + 0.5 * rho * (u * u + v * v + w * w)};
    const size_t col = (size_t)(P.g[1] + j) * P.s[1] + (size_t)(P.g[2] + k) * P.s[2];
    for (int m = 0; m < NG; ++m)
      for (int q = 0; q < 5; ++q) Q[q * T + col + (size_t)m * P.s[0]] = cons[q];
  }
}

static inline unsigned df_blocks(long long work) {
  return (unsigned)std::max<long long>(1, std::min<long long>((work + 255) / 256, 65536));
}

void launch_df_update(const DFDev& D, const Prob* prob, const double* rnd, double* Q, double dt, int first,
                      hipStream_t s) {
  const long long rows = D.ny + 2LL * D.pad;
  hipLaunchKernelGGL(k_df_zeta, dim3(df_blocks(3 * rows * D.nz)), dim3(256), 0, s, D, rnd);
  hipLaunchKernelGGL(k_df_eta, dim3(df_blocks(3LL * D.ny * D.nz)), dim3(256), 0, s, D, prob, dt, first);
  hipLaunchKernelGGL(k_df_ghosts, dim3(df_blocks((long long)D.ny * D.nz)), dim3(256), 0, s, D, prob, Q);
}

}  // namespace lg
