// Gradients of the primitives along one computational direction.
//
// Paper: Sec. 2.3 -- MEG6 reconstructs from explicit sixth-order gradients, MIG4 from
// implicit fourth-order (compact) gradients, which requires "solving several 1D
// tridiagonal matrices" (Sec. 4.2).  Unit computational spacing (Sec. 2.2).
//
//   E6: f'_i = [45 (f_{i+1}-f_{i-1}) - 9 (f_{i+2}-f_{i-2}) + (f_{i+3}-f_{i-3})] / 60
//   C4: f'_{i-1}/4 + f'_i + f'_{i+1}/4 = 3 (f_{i+1} - f_{i-1}) / 4
//
// C4 closure: a bounded line is solved over all of its nodes (ghosts included) with
// second-order one-sided end rows; a periodic line is solved cyclically over its
// interior nodes (Sherman-Morrison on top of a bounded solve) and its ghost values are
// the periodic images.  The solves run in FP64 from primitives formed in FP64 from the
// conserved state, whatever the bulk precision.  Each thread owns one line; the LU
// factors of the constant-coefficient matrices are precomputed on the host (tables
// below), so a solve is one forward and one backward sweep.
//
// Table layout for direction d (double):
//   bounded  line of N nodes: cp[0..N), inv[0..N)
//   periodic line of n nodes: cp[0..n), inv[0..n), z[0..n), fac   (B z = u, fac = 1/(1 + v.z))
#include "lgbr_dev.h"
#include "lgbr_kernels.h"

namespace lg {

__device__ __forceinline__ bool skip_launch(const Prob& P, int skip_if_any) {
  return skip_if_any >= 0 && P.any_flag && (*P.any_flag != 0) == (skip_if_any != 0);
}

template <typename R, int ORDER>
__global__ void __launch_bounds__(256) k_grad_explicit(const Prob* probs, int d, int skip_if_any) {
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || skip_launch(P, skip_if_any)) return;
  const R* W = static_cast<const R*>(P.W);
  R* G = static_cast<R*>(P.G[d]);
  const int r = ORDER / 2, Nd = P.N[d], sd = P.s[d];
  const size_t T = P.total;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < P.total; idx += gridDim.x * blockDim.x) {
    int c = (idx / sd) % Nd;
    if (c < r || c >= Nd - r) continue;
    for (int q = 0; q < 5; ++q) {
      const R* f = W + q * T + idx;
      R v;
      if (ORDER == 6)
        v = (R(45) * (f[sd] - f[-sd]) - R(9) * (f[2 * sd] - f[-2 * sd]) + (f[3 * sd] - f[-3 * sd])) / R(60);
      else
        v = (R(8) * (f[sd] - f[-sd]) - (f[2 * sd] - f[-2 * sd])) / R(12);
      G[q * T + idx] = v;
    }
  }
}

__device__ __forceinline__ void prim64(const double* Q, size_t T, size_t o, double gamma, double w[5]) {
  double rho = Q[o];
  double u = Q[T + o] / rho, v = Q[2 * T + o] / rho, ww = Q[3 * T + o] / rho;
  w[0] = rho;
  w[1] = u;
  w[2] = v;
  w[3] = ww;
  w[4] = (gamma - 1.0) * (Q[4 * T + o] - 0.5 * rho * (u * u + v * v + ww * ww));
}

template <typename R>
__global__ void __launch_bounds__(256) k_grad_c4(const Prob* probs, StateRef ref, int d, int skip_if_any) {
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || skip_launch(P, skip_if_any)) return;
  const double* Q = ref.state(P);
  R* G = static_cast<R*>(P.G[d]);
  double* S = P.T64;
  const double* tab = P.tri[d];
  const size_t T = P.total;
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const int nlines = P.N[o1] * P.N[o2];
  const int line = blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= nlines) return;
  const int a = line % P.N[o1], b = line / P.N[o1];
  const size_t base = (size_t)a * P.s[o1] + (size_t)b * P.s[o2];
  const int sd = P.s[d], g = P.g[d], n = P.n[d], N = P.N[d];
  const double gam = P.gamma;

  if (P.bc[d][0] != BC_PERIODIC) {
    const double* cp = tab;
    const double* inv = tab + N;
    // forward sweep: d'_i stored in S
    double wm[5], w0[5], wp[5], dprev[5];
    prim64(Q, T, base, gam, w0);
    prim64(Q, T, base + sd, gam, wp);
    {
      double w2[5];
      prim64(Q, T, base + 2 * sd, gam, w2);
      for (int q = 0; q < 5; ++q) {
        double rhs = (-3.0 * w0[q] + 4.0 * wp[q] - w2[q]) / 2.0;
        dprev[q] = rhs;
        S[q * T + base] = rhs;
      }
    }
    for (int i = 1; i < N - 1; ++i) {
      for (int q = 0; q < 5; ++q) { wm[q] = w0[q]; w0[q] = wp[q]; }
      prim64(Q, T, base + (size_t)(i + 1) * sd, gam, wp);
      for (int q = 0; q < 5; ++q) {
        double rhs = 0.75 * (wp[q] - wm[q]);
        double dd = (rhs - 0.25 * dprev[q]) * inv[i];
        dprev[q] = dd;
        S[q * T + base + (size_t)i * sd] = dd;
      }
    }
    // last row: one-sided, decoupled
    double y[5];
    {
      double w3[5];
      prim64(Q, T, base + (size_t)(N - 3) * sd, gam, w3);
      for (int q = 0; q < 5; ++q) y[q] = (3.0 * wp[q] - 4.0 * w0[q] + w3[q]) / 2.0;
    }
    for (int q = 0; q < 5; ++q) G[q * T + base + (size_t)(N - 1) * sd] = (R)y[q];
    for (int i = N - 2; i >= 0; --i) {
      for (int q = 0; q < 5; ++q) {
        y[q] = S[q * T + base + (size_t)i * sd] - cp[i] * y[q];
        G[q * T + base + (size_t)i * sd] = (R)y[q];
      }
    }
  } else {
    const double* cp = tab;
    const double* inv = tab + n;
    const double* z = tab + 2 * n;
    const double fac = tab[3 * n];
    // B y = r over the interior; r_i = 3/4 (f_{i+1} - f_{i-1}) with periodic neighbours
    // (the ghosts already hold the periodic images)
    const size_t b0 = base + (size_t)g * sd;
    double wm[5], w0[5], wp[5], dprev[5];
    prim64(Q, T, b0 - sd, gam, wm);
    prim64(Q, T, b0, gam, w0);
    for (int i = 0; i < n; ++i) {
      prim64(Q, T, b0 + (size_t)(i + 1) * sd, gam, wp);
      for (int q = 0; q < 5; ++q) {
        double rhs = 0.75 * (wp[q] - wm[q]);
        double dd = (i == 0 ? rhs : rhs - 0.25 * dprev[q]) * inv[i];
        dprev[q] = dd;
        S[q * T + b0 + (size_t)i * sd] = dd;
        wm[q] = w0[q];
        w0[q] = wp[q];
      }
    }
    double y[5], ylast[5];
    for (int q = 0; q < 5; ++q) { y[q] = dprev[q]; ylast[q] = y[q]; }
    for (int i = n - 2; i >= 0; --i)
      for (int q = 0; q < 5; ++q) {
        y[q] = S[q * T + b0 + (size_t)i * sd] - cp[i] * y[q];
        S[q * T + b0 + (size_t)i * sd] = y[q];
      }
    // y now holds y_0; Sherman-Morrison correction x = y - (v.y) fac z, v.y = y_0 - y_{n-1}/4
    double vy[5];
    for (int q = 0; q < 5; ++q) vy[q] = (y[q] - 0.25 * ylast[q]) * fac;
    S[0 * T + b0 + (size_t)(n - 1) * sd] = ylast[0];
    for (int q = 1; q < 5; ++q) S[q * T + b0 + (size_t)(n - 1) * sd] = ylast[q];
    for (int i = 0; i < n; ++i) {
      for (int q = 0; q < 5; ++q) {
        double x = S[q * T + b0 + (size_t)i * sd] - vy[q] * z[i];
        R xv = (R)x;
        G[q * T + b0 + (size_t)i * sd] = xv;
        if (i >= n - g) G[q * T + b0 + (size_t)(i - n) * sd] = xv;   // low ghosts
        if (i < g) G[q * T + b0 + (size_t)(i + n) * sd] = xv;        // high ghosts
      }
    }
  }
}

template <typename R>
void launch_grad_explicit(const Launch& L, int d, int order, int skip_if_any) {
  long long b = (L.max_total + 255) / 256;
  if (b > 8192) b = 8192;
  dim3 grid((unsigned)b, L.nprob);
  if (order == 6)
    LG_TIMED(L, KC_GRAD_E6,
             hipLaunchKernelGGL((k_grad_explicit<R, 6>), grid, dim3(256), 0, L.stream, L.probs, d, skip_if_any));
  else
    LG_TIMED(L, KC_GRAD_E6,
             hipLaunchKernelGGL((k_grad_explicit<R, 4>), grid, dim3(256), 0, L.stream, L.probs, d, skip_if_any));
}

template <typename R>
void launch_grad_c4(const Launch& L, StateRef ref, int d, int skip_if_any) {
  long long b = (L.lines[d] + 63) / 64;
  if (b < 1) b = 1;
  LG_TIMED(L, KC_GRAD_C4, hipLaunchKernelGGL(k_grad_c4<R>, dim3((unsigned)b, L.nprob), dim3(64), 0, L.stream,
                                             L.probs, ref, d, skip_if_any));
}

template void launch_grad_explicit<float>(const Launch&, int, int, int);
template void launch_grad_explicit<double>(const Launch&, int, int, int);
template void launch_grad_c4<float>(const Launch&, StateRef, int, int);
template void launch_grad_c4<double>(const Launch&, StateRef, int, int);

}  // namespace lg
