// Device-side definitions shared by the HIP kernels of the hybrid LAD-GBR right-hand side.
//
// Layout: every field lives on the ghost-padded node grid of one problem, i fastest:
//   idx = i + N0 * (j + N1 * k),  0 <= i < N0 = n0 + 2 g0, ...
// with g = 5 ghost layers in active directions and none in inactive ones.  A stack of
// nv fields is stored field-major: field q at [q * total + idx].  The conserved state,
// its time derivative, the RK stage buffer and the compact-gradient solves are FP64;
// every other intermediate uses the template type R (double for the plain FP64 path,
// float for the mixed path).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lg {

enum { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_REFLECTIVE = 2, BC_NOSLIP = 3, BC_FIXED = 4 };
// Interface flux selection of one sweep.
enum { SEL_GBR = 0, SEL_LAD = 1, SEL_PERCELL = 2, SEL_GLOBAL = 3 };

constexpr int NG = 5;

// Everything a kernel needs to know about one problem.  Kept in device memory (one per
// problem) so that a batch of independent problems can be processed by one launch.
struct Prob {
  int ndim;
  int n[3], g[3], N[3];
  int s[3];          // strides of i, j, k
  int total;         // N0 * N1 * N2
  int bc[3][2];
  int curvilinear;
  double h[3];
  double cm[10];     // Cartesian metrics (xi_x .. zeta_z)/J and J
  // gas (Sec. 2.1)
  double gamma, Re, Pr, Mref, suth;
  int viscous;
  // scheme options
  double omega_thr, mp_eps, mp_alpha, C_mu, C_beta, C_kappa, rho_thr, p_thr, cfl;
  int dilate;
  int grad_c4;       // 0: explicit E6 gradients, 1: compact C4 gradients
  // buffers (device)
  double* Q;         // conserved state (caller)
  double* dQ;        // time derivative (caller for *_rhs, workspace for rk3)
  double* Us;        // RK stage state (workspace)
  void* W;           // primitives rho,u,v,w,p          [5][total]  R
  void* G[3];        // d(primitives)/d xi_l             [5][total]  R
  double* T64;       // FP64 scratch of the line solves  [5][total]
  void* Om;          // Omega sensor                     [total]     R
  uint8_t* f;        // troubled flags                   [total]
  uint8_t* ft;       // dilated flags                    [total]
  uint8_t* ftmp;     // dilation scratch                 [total]
  uint8_t* fg;       // nodes whose C-GBR inputs are needed (per-cell hybrid) [total]
  int* llist[3];     // compacted lines of each direction that touch fg
  int* lcount;       // [3] number of listed lines
  void* S3;          // |S|, theta, e                    [3][total]  R
  void* D4;          // E4 physical gradients d(rho,u,v,w,p)/dx_j [15][total] R (q*3 + j)
  void* CA;          // LAD coefficients mu*,beta*,kappa* [3][total] R (result)
  void* CB;          // LAD filter scratch               [3][total]  R
  void* FL[3];       // LAD node fluxes per direction    [5][total]  R
  void* FV[3];       // C-GBR viscous node fluxes        [5][total]  R
  const void* MR;    // node metrics in R                [10][total] (curvilinear only)
  const double* M64; // node metrics in FP64             [10][total] (curvilinear only)
  const double* coords;  // node coordinates             [3][total]  (curvilinear only)
  const double* tri[3];  // compact-solve LU tables per direction (see k_grad.hip)
  const double* pcr[3];  // compact-solve PCR factors per direction (see k_grad.hip)
  // device scalars
  double* dt;
  double* t;
  double t_end;
  unsigned long long* smax;  // max spectral radius (bit pattern of a positive double)
  int* status;               // non-physical node count
  int* any_flag;             // global hybrid switch: any troubled interior node
};

__host__ __device__ __forceinline__ int pos_to_idx(const Prob& P, int i, int j, int k) {
  return i + P.s[1] * j + P.s[2] * k;
}

// Node metric component c (0..8: l_hat_j for l = c/3, j = c%3; 9: J) at node idx.
template <typename R>
__host__ __device__ __forceinline__ R met(const Prob& P, int c, int idx) {
  if (P.curvilinear) return static_cast<const R*>(P.MR)[(size_t)c * P.total + idx];
  return (R)P.cm[c];
}

__host__ __device__ __forceinline__ double met64(const Prob& P, int c, int idx) {
  if (P.curvilinear) return P.M64[(size_t)c * P.total + idx];
  return P.cm[c];
}

template <typename R>
__host__ __device__ __forceinline__ R sgn(R a) {
  return a > R(0) ? R(1) : (a < R(0) ? R(-1) : R(0));
}

template <typename R>
__host__ __device__ __forceinline__ R minmod2(R a, R b) {
  return R(0.5) * (sgn(a) + sgn(b)) * fmin(fabs(a), fabs(b));
}

template <typename R>
__host__ __device__ __forceinline__ R minmod4(R w, R x, R y, R z) {
  R sw = sgn(w);
  return R(0.125) * (sw + sgn(x)) * fabs((sw + sgn(y)) * (sw + sgn(z))) *
         fmin(fmin(fabs(w), fabs(x)), fmin(fabs(y), fabs(z)));
}

}  // namespace lg
