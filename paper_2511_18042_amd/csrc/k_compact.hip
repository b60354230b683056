// LAD-C6: compact sixth-order differences and the low-pass implicit filter.
//
// Paper: Sec. 3 and Alg. 1 -- the stand-alone LAD scheme differences its fluxes with a
// sixth-order compact central scheme, and after the solution update of the last
// Runge-Kutta stage it filters the solution along i, j and k with the implicit filter
// of Gaitonde & Visbal (Sec. 2.1).  Unit computational spacing.
//
//   C6 gradient  (1/3) f'_{i-1} + f'_i + (1/3) f'_{i+1} = (7/9)(f_{i+1} - f_{i-1}) + (1/36)(f_{i+2} - f_{i-2})
//   C6 faces     (1/3) F_{i-1/2} + F_{i+1/2} + (1/3) F_{i+3/2}
//                    = (29/36)(F_i + F_{i+1}) + (1/36)(F_{i-1} + F_{i+2})
//                (subtracting the rows of i+1/2 and i-1/2 gives the C6 relation for the node
//                derivative F_{i+1/2} - F_{i-1/2}: the flux form of the scheme)
//   filter       a_f phi^_{i-1} + phi^_i + a_f phi^_{i+1} = sum_{k=0}^{5} (a_k / 2)(phi_{i+k} + phi_{i-k})
//                (tenth order; a_k from the maximal-order conditions, computed on the host)
//
// Closures of bounded lines: the gradient line spans all nodes with second-order
// one-sided end rows and C4 rows next to them; the face system's unknowns are the
// interior faces, the boundary faces -1/2 and n-1/2 being the fourth-order I4 values of
// the node fluxes; the filter's unknowns are the interior nodes, their neighbours across
// the boundary entering with the ghost values.  Periodic lines are cyclic over the
// interior.  All solves run in FP64.
//
// Each system has constant coefficients, so its factors are tables built on the host:
//   bounded, m unknowns (Thomas):  cp[m], inv[m], a[m]      (a = sub-diagonal of each row)
//   cyclic, n unknowns:            cp[n], inv[n], z[n], fac, alpha, c[n]
//       (A = B + u v^T with u = (-1, 0.., alpha), v = (1, 0.., -alpha); B z = u,
//        x = y - (y_0 - alpha y_{n-1}) fac z with B y = r, fac = 1 / (1 + v.z);
//        y_0 = sum_k c_k d_k over the forward-eliminated d, so one back substitution
//        emits x)
//   PCR factors:                   k1[steps][L], k2[steps][L], binv[L]
// Lines along the contiguous direction are solved by parallel cyclic reduction in LDS, one
// workgroup per (line, variable); strided lines one lane per line, coalesced across lanes.
#include "lgbr_dev.h"
#include "lgbr_kernels.h"

#include <algorithm>

namespace lg {

constexpr double C6_A = 7.0 / 9.0, C6_B = 1.0 / 36.0;
constexpr double C6F_A = 29.0 / 36.0, C6F_B = 1.0 / 36.0, C6_ALPHA = 1.0 / 3.0;
constexpr int CPCR_THREADS = 512;   // lanes per workgroup of the one-line PCR kernels
constexpr int CPCR_MAXPT = 4096 / CPCR_THREADS;

// Parallel cyclic reduction of r[0..L) in LDS by the whole (CPCR_THREADS-lane) workgroup; the
// solution x_i = r_i / b_i is left in r.  Periodic lines wrap their indices (L must be at
// least 2^(steps+1)); the couplings left after `steps` steps are below rounding.
__device__ void pcr_lds(double* r, int L, bool periodic, const double* tab, int steps) {
  double nv[CPCR_MAXPT];
  const double* hdr = tab + (size_t)(2 * steps + 1) * L;   // band header (see the line tiles)
  for (int st = 0; st < steps; ++st) {
    const int s = 1 << st;
    const double* k1 = tab + (size_t)st * L;
    const double* k2 = tab + (size_t)(steps + st) * L;
    const double c1 = hdr[4 * st], c2 = hdr[4 * st + 1];
    const int blo = (int)hdr[4 * st + 2], bhi = (int)hdr[4 * st + 3];
#pragma unroll
    for (int m = 0; m < CPCR_MAXPT; ++m) {
      const int i = threadIdx.x + m * CPCR_THREADS;
      if (i < L) {
        int im = i - s, ip = i + s;
        double rm, rp;
        if (periodic) {
          im = im < 0 ? im + L : im;
          ip = ip >= L ? ip - L : ip;
          rm = r[im];
          rp = r[ip];
        } else {
          rm = im >= 0 ? r[im] : 0.0;
          rp = ip < L ? r[ip] : 0.0;
        }
        double f1 = c1, f2 = c2;
        if (i < blo || i > bhi) {
          f1 = k1[i];
          f2 = k2[i];
        }
        nv[m] = r[i] - f1 * rm - f2 * rp;
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < CPCR_MAXPT; ++m) {
      const int i = threadIdx.x + m * CPCR_THREADS;
      if (i < L) r[i] = nv[m];
    }
    __syncthreads();
  }
  const double* binv = tab + (size_t)2 * steps * L;
  const double cb = hdr[4 * steps];
  const int blo = (int)hdr[4 * steps + 2], bhi = (int)hdr[4 * steps + 3];
  for (int i = threadIdx.x; i < L; i += blockDim.x) r[i] *= (i < blo || i > bhi) ? binv[i] : cb;
  __syncthreads();
}

// interior line t of direction d (positions of the other two directions inside the grid)
__device__ __forceinline__ size_t interior_line_base(const Prob& P, int d, int t) {
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const int a = t % P.n[o1], b = t / P.n[o1];
  return (size_t)(P.g[o1] + a) * P.s[o1] + (size_t)(P.g[o2] + b) * P.s[o2];
}

__device__ __forceinline__ int interior_lines(const Prob& P, int d) {
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  return P.n[o1] * P.n[o2];
}

__device__ __forceinline__ int wrap(int p, int n) { return p < 0 ? p + n : (p >= n ? p - n : p); }

__device__ __forceinline__ void prims5c(const double* Q, size_t T, size_t o, double gm1, double w[5]) {
  const double rho = Q[o], ri = 1.0 / rho;
  const double u = Q[T + o] * ri, v = Q[2 * T + o] * ri, x = Q[3 * T + o] * ri;
  w[0] = rho;
  w[1] = u;
  w[2] = v;
  w[3] = x;
  w[4] = gm1 * (Q[4 * T + o] - 0.5 * rho * (u * u + v * v + x * x));
}

// primitives q0 .. q0 + NQ - 1 of node o (NQ = 5: all, as prims5c; NQ = 1: the one, with
// the same arithmetic)
template <int NQ>
__device__ __forceinline__ void prims_q(const double* Q, size_t T, size_t o, double gm1, int q0, double w[NQ]) {
  if constexpr (NQ == 5) {
    prims5c(Q, T, o, gm1, w);
  } else if (q0 == 0) {
    w[0] = Q[o];
  } else if (q0 < 4) {
    w[0] = Q[(size_t)q0 * T + o] * (1.0 / Q[o]);
  } else {
    double a[5];
    prims5c(Q, T, o, gm1, a);
    w[0] = a[4];
  }
}

// ------------------------------------------------------------------ C6 gradients
// right-hand side of row i of a bounded gradient line of N nodes from the values at
// i-2 .. i+2 (entries outside the line unused)
__device__ __forceinline__ double c6_grad_rhs(int i, int N, double m2, double m1, double c0, double p1, double p2) {
  if (i == 0) return (-3.0 * c0 + 4.0 * p1 - p2) / 2.0;
  if (i == N - 1) return (3.0 * c0 - 4.0 * m1 + m2) / 2.0;
  if (i == 1 || i == N - 2) return 0.75 * (p1 - m1);
  return C6_A * (p1 - m1) + C6_B * (p2 - m2);
}

// One lane per line (all nodes of the other two directions), all five primitives formed
// in FP64 from the conserved state; forward elimination into the FP64 scratch, back
// substitution into the gradient array.
template <typename R, int NQ>
__global__ void __launch_bounds__(320) k_grad_c6(const Prob* __restrict__ probs, StateRef ref, int d, int mask) {
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || tile_use(P, d, TK_GRAD6, mask) || c6_grad_pcr(P, d) || c6g_part_use(P, d, mask) ||
      c6g_seg_use(P, d, mask))
    return;
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  // NQ = 5: one lane per line; NQ = 1: a workgroup of five waves solves the five primitives
  // of 64 lines, wave w primitive w (the waves share the state's cache lines)
  const int t = NQ == 5 ? (int)(blockIdx.x * blockDim.x + threadIdx.x) : (int)(blockIdx.x * 64 + (threadIdx.x & 63));
  const int q0 = NQ == 5 ? 0 : (int)(threadIdx.x >> 6);
  if (t >= P.N[o1] * P.N[o2]) return;
  const double* Q = ref.state(P);
  R* G = static_cast<R*>(P.G[d]);
  const size_t T = P.total;
  double* S = P.T64;
  const double* tab = P.tri6[d];
  const int a = t % P.N[o1], b = t / P.N[o1];
  const size_t base = (size_t)a * P.s[o1] + (size_t)b * P.s[o2];
  const int sd = P.s[d], g = P.g[d], n = P.n[d], N = P.N[d];
  const double gm1 = P.gamma - 1.0;
  double w[5][NQ];   // window: positions i-2 .. i+2
  if (P.bc[d][0] != BC_PERIODIC) {
    const double* cp = tab;
    const double* inv = tab + N;
    const double* sub = tab + 2 * N;
    for (int q = 0; q < NQ; ++q) w[0][q] = w[1][q] = 0.0;
    prims_q<NQ>(Q, T, base, gm1, q0, w[2]);
    prims_q<NQ>(Q, T, base + (size_t)sd, gm1, q0, w[3]);
    prims_q<NQ>(Q, T, base + (size_t)2 * sd, gm1, q0, w[4]);
    double dprev[NQ] = {};
    for (int i = 0; i < N; ++i) {
      for (int q = 0; q < NQ; ++q) {
        const double r = c6_grad_rhs(i, N, w[0][q], w[1][q], w[2][q], w[3][q], w[4][q]);
        const double dd = (r - sub[i] * dprev[q]) * inv[i];
        S[(q0 + q) * T + base + (size_t)i * sd] = dd;
        dprev[q] = dd;
      }
      for (int p = 0; p < 4; ++p)
        for (int q = 0; q < NQ; ++q) w[p][q] = w[p + 1][q];
      if (i + 3 < N) prims_q<NQ>(Q, T, base + (size_t)(i + 3) * sd, gm1, q0, w[4]);
      else
        for (int q = 0; q < NQ; ++q) w[4][q] = 0.0;
    }
    double y[NQ];
    for (int q = 0; q < NQ; ++q) {
      y[q] = dprev[q];
      G[(q0 + q) * T + base + (size_t)(N - 1) * sd] = (R)y[q];
    }
    for (int i = N - 2; i >= 0; --i)
      for (int q = 0; q < NQ; ++q) {
        y[q] = S[(q0 + q) * T + base + (size_t)i * sd] - cp[i] * y[q];
        G[(q0 + q) * T + base + (size_t)i * sd] = (R)y[q];
      }
  } else {
    const double* cp = tab;
    const double* inv = tab + n;
    const double* z = tab + 2 * n;
    const double fac = tab[3 * n], al = tab[3 * n + 1];
    const double* y0c = tab + 3 * n + 2;
    const size_t b0 = base + (size_t)g * sd;
    for (int p = 0; p < 4; ++p) prims_q<NQ>(Q, T, base + (size_t)(g + wrap(p - 2, n)) * sd, gm1, q0, w[p]);
    double dprev[NQ] = {}, y0[NQ] = {};
    for (int i = 0; i < n; ++i) {
      prims_q<NQ>(Q, T, base + (size_t)(g + wrap(i + 2, n)) * sd, gm1, q0, w[4]);
      for (int q = 0; q < NQ; ++q) {
        const double r = C6_A * (w[3][q] - w[1][q]) + C6_B * (w[4][q] - w[0][q]);
        const double dd = (i == 0 ? r : r - al * dprev[q]) * inv[i];
        S[(q0 + q) * T + b0 + (size_t)i * sd] = dd;
        dprev[q] = dd;
        y0[q] = y0[q] + y0c[i] * dd;
      }
      for (int p = 0; p < 4; ++p)
        for (int q = 0; q < NQ; ++q) w[p][q] = w[p + 1][q];
    }
    // one back substitution emitting x = y - (y_0 - al y_{n-1}) fac z
    double y[NQ], vy[NQ];
    for (int q = 0; q < NQ; ++q) {
      y[q] = dprev[q];
      vy[q] = (y0[q] - al * dprev[q]) * fac;
    }
    for (int i = n - 1; i >= 0; --i)
      for (int q = 0; q < NQ; ++q) {
        if (i < n - 1) y[q] = S[(q0 + q) * T + b0 + (size_t)i * sd] - cp[i] * y[q];
        const R xv = (R)(y[q] - vy[q] * z[i]);
        G[(q0 + q) * T + b0 + (size_t)i * sd] = xv;
        if (i >= n - g) G[(q0 + q) * T + b0 + (size_t)(i - n) * sd] = xv;   // low ghosts
        if (i < g) G[(q0 + q) * T + b0 + (size_t)(i + n) * sd] = xv;        // high ghosts
      }
  }
}

// One workgroup per (line, primitive), persistent over the items; the primitive along the
// line in LDS, the right-hand side reduced by PCR.
template <typename R>
__global__ void __launch_bounds__(CPCR_THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_grad_c6_pcr(const Prob* __restrict__ probs, StateRef ref, int d,
                                                     int mask) {
  extern __shared__ double lds[];
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || tile_use(P, d, TK_GRAD6, mask) || !c6_grad_pcr(P, d) || c6g_part_use(P, d, mask) ||
      c6g_seg_use(P, d, mask))
    return;
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const int nlines = P.N[o1] * P.N[o2];
  const bool periodic = P.bc[d][0] == BC_PERIODIC;
  const int g = P.g[d], N = P.N[d], n = P.n[d];
  const int L = periodic ? n : N;
  const int off0 = periodic ? g : 0;
  const int sd = P.s[d];
  const double* Q = ref.state(P);
  const size_t T = P.total;
  const double gm1 = P.gamma - 1.0;
  double* f = lds;
  double* r = lds + N;
  for (int blk = blockIdx.x; blk < 5 * nlines; blk += gridDim.x) {
    const int line = blk % nlines, q = blk / nlines;
    const int a = line % P.N[o1], b = line / P.N[o1];
    const size_t base = (size_t)a * P.s[o1] + (size_t)b * P.s[o2];
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      const size_t o = base + (size_t)i * sd;
      const double rho = Q[o];
      double v;
      if (q == 0) {
        v = rho;
      } else {
        const double ri = 1.0 / rho;
        if (q <= 3) {
          v = Q[q * T + o] * ri;
        } else {
          const double u = Q[T + o] * ri, vv = Q[2 * T + o] * ri, w = Q[3 * T + o] * ri;
          v = gm1 * (Q[4 * T + o] - 0.5 * rho * (u * u + vv * vv + w * w));
        }
      }
      f[i] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
      double v;
      if (periodic) {
        v = C6_A * (f[off0 + wrap(i + 1, n)] - f[off0 + wrap(i - 1, n)]) +
            C6_B * (f[off0 + wrap(i + 2, n)] - f[off0 + wrap(i - 2, n)]);
      } else {
        v = c6_grad_rhs(i, N, i >= 2 ? f[i - 2] : 0.0, i >= 1 ? f[i - 1] : 0.0, f[i], i + 1 < N ? f[i + 1] : 0.0,
                        i + 2 < N ? f[i + 2] : 0.0);
      }
      r[i] = v;
    }
    __syncthreads();
    pcr_lds(r, L, periodic, P.pcr6[d], LG_PCR_STEPS);
    R* G = static_cast<R*>(P.G[d]) + (size_t)q * T;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
      const R y = (R)r[i];
      G[base + (size_t)(i + off0) * sd] = y;
      if (periodic) {
        if (i >= n - g) G[base + (size_t)(i + off0 - n) * sd] = y;   // low ghosts
        if (i < g) G[base + (size_t)(i + off0 + n) * sd] = y;        // high ghosts
      }
    }
    __syncthreads();   // the next item reuses the LDS line
  }
}

// ------------------------------------------------------------------ C6 interface fluxes
// What one node's derivative does: -J D (first direction), added to dQ/dt (later ones),
// or, in the last direction of an RK stage, the stage combination.
struct FaceOut {
  StateRef ref;
  RKRef rr;
  int accumulate, rk, stage;
  double a, b;
};

__device__ __forceinline__ bool face_emit(const Prob& P, const FaceOut& o, double* dQ, double dt, size_t idx,
                                          const double D[5]) {
  const size_t T = P.total;
  const double J = met64(P, 9, (int)idx);
  double Lq[5];
  for (int q = 0; q < 5; ++q) {
    Lq[q] = -J * D[q];
    if (o.accumulate) Lq[q] = dQ[q * T + idx] + Lq[q];
  }
  if (o.rk) return rk_combine_node(P, o.rr, o.stage, o.a, o.b, dt, (int)idx, Lq);
  for (int q = 0; q < 5; ++q) dQ[q * T + idx] = Lq[q];
  return false;
}

// face_emit for NQ components starting at q0 (one component: never the RK stage)
template <int NQ>
__device__ __forceinline__ bool face_emit_q(const Prob& P, const FaceOut& o, double* dQ, double dt, int q0,
                                            size_t idx, const double D[NQ]) {
  if constexpr (NQ == 5) {
    return face_emit(P, o, dQ, dt, idx, D);
  } else {
    const size_t at = (size_t)q0 * P.total + idx;
    const double L = -met64(P, 9, (int)idx) * D[0];
    dQ[at] = o.accumulate ? dQ[at] + L : L;
    return false;
  }
}

// One lane per interior line and NQ flux components (all five where the RK stage needs
// them together, else one: five times the lanes); forward elimination into the FP64
// scratch, back substitution emitting the node derivatives.
template <typename R, int NQ>
__global__ void __launch_bounds__(256) k_c6_faces(const Prob* __restrict__ probs, FaceOut o, int d, int mask) {
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || tile_use(P, d, TK_FACES, mask) || c6_face_pcr(P, d) || c6f_part_use(P, d, mask) ||
      c6f_seg_use(P, d, mask))
    return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nl = interior_lines(P, d);
  if (t >= (5 / NQ) * nl) return;
  const int line = NQ == 5 ? t : t % nl, q0 = NQ == 5 ? 0 : t / nl;
  const R* F = static_cast<const R*>(P.FL[d]);
  const size_t T = P.total;
  double* S = P.T64;
  double* dQ = o.ref.deriv(P);
  const double dt = o.rk ? *P.dt : 0.0;
  const double* tab = P.trc[d];
  const size_t base = interior_line_base(P, d, line);
  const int sd = P.s[d], g = P.g[d], n = P.n[d];
  int bad = 0;
  auto at = [&](int q, int p) { return (double)F[(q0 + q) * T + base + (size_t)(g + p) * sd]; };
  if (P.bc[d][0] != BC_PERIODIC) {
    const int m = n - 1;
    const double* cp = tab;
    const double* inv = tab + m;
    const double* sub = tab + 2 * m;
    double lo[NQ], hi[NQ], w[4][NQ], dprev[NQ];
    for (int q = 0; q < NQ; ++q) {
      lo[q] = (7.0 * (at(q, -1) + at(q, 0)) - (at(q, -2) + at(q, 1))) / 12.0;
      hi[q] = (7.0 * (at(q, n - 1) + at(q, n)) - (at(q, n - 2) + at(q, n + 1))) / 12.0;
      for (int p = 0; p < 3; ++p) w[p][q] = at(q, p - 1);
      dprev[q] = 0.0;
    }
    for (int k = 0; k < m; ++k) {
      for (int q = 0; q < NQ; ++q) {
        w[3][q] = at(q, k + 2);
        double r = C6F_A * (w[1][q] + w[2][q]) + C6F_B * (w[0][q] + w[3][q]);
        if (k == 0) r = r - C6_ALPHA * lo[q];
        if (k == m - 1) r = r - C6_ALPHA * hi[q];
        const double dd = (r - sub[k] * dprev[q]) * inv[k];
        S[(q0 + q) * T + base + (size_t)(g + k) * sd] = dd;
        dprev[q] = dd;
        w[0][q] = w[1][q];
        w[1][q] = w[2][q];
        w[2][q] = w[3][q];
      }
    }
    double prev[NQ], D[NQ];
    for (int q = 0; q < NQ; ++q) prev[q] = hi[q];
    for (int k = m - 1; k >= 0; --k) {
      for (int q = 0; q < NQ; ++q) {
        const double x = S[(q0 + q) * T + base + (size_t)(g + k) * sd] - cp[k] * (k == m - 1 ? 0.0 : prev[q]);
        D[q] = prev[q] - x;
        prev[q] = x;
      }
      if (face_emit_q<NQ>(P, o, dQ, dt, q0, base + (size_t)(g + k + 1) * sd, D)) ++bad;
    }
    for (int q = 0; q < NQ; ++q) D[q] = prev[q] - lo[q];
    if (face_emit_q<NQ>(P, o, dQ, dt, q0, base + (size_t)g * sd, D)) ++bad;
  } else {
    const double* cp = tab;
    const double* inv = tab + n;
    const double* z = tab + 2 * n;
    const double fac = tab[3 * n], al = tab[3 * n + 1];
    const double* y0c = tab + 3 * n + 2;
    auto atw = [&](int q, int p) { return at(q, wrap(p, n)); };
    double w[4][NQ], dprev[NQ], y0[NQ];
    for (int q = 0; q < NQ; ++q) {
      for (int p = 0; p < 3; ++p) w[p][q] = atw(q, p - 1);
      dprev[q] = y0[q] = 0.0;
    }
    for (int k = 0; k < n; ++k) {
      for (int q = 0; q < NQ; ++q) {
        w[3][q] = atw(q, k + 2);
        const double r = C6F_A * (w[1][q] + w[2][q]) + C6F_B * (w[0][q] + w[3][q]);
        const double dd = (k == 0 ? r : r - al * dprev[q]) * inv[k];
        S[(q0 + q) * T + base + (size_t)(g + k) * sd] = dd;
        dprev[q] = dd;
        y0[q] = y0[q] + y0c[k] * dd;
        w[0][q] = w[1][q];
        w[1][q] = w[2][q];
        w[2][q] = w[3][q];
      }
    }
    // one back substitution emitting the faces x = y - (y_0 - al y_{n-1}) fac z and, from
    // each pair of neighbouring faces, the node difference D_{k+1} = x_{k+1} - x_k
    double y[NQ], vy[NQ], xlast[NQ], xnext[NQ], D[NQ];
    for (int q = 0; q < NQ; ++q) {
      y[q] = dprev[q];
      vy[q] = (y0[q] - al * dprev[q]) * fac;
      xlast[q] = xnext[q] = y[q] - vy[q] * z[n - 1];
    }
    for (int k = n - 2; k >= 0; --k) {
      for (int q = 0; q < NQ; ++q) {
        y[q] = S[(q0 + q) * T + base + (size_t)(g + k) * sd] - cp[k] * y[q];
        const double x = y[q] - vy[q] * z[k];
        D[q] = xnext[q] - x;
        xnext[q] = x;
      }
      if (face_emit_q<NQ>(P, o, dQ, dt, q0, base + (size_t)(g + k + 1) * sd, D)) ++bad;
    }
    for (int q = 0; q < NQ; ++q) D[q] = xnext[q] - xlast[q];   // node 0: x_0 - x_{n-1}
    if (face_emit_q<NQ>(P, o, dQ, dt, q0, base + (size_t)g * sd, D)) ++bad;
  }
  add_bad(P, bad);
}

// Contiguous lines (the first direction of a 2D / 3D grid): one workgroup per (interior
// line, component); node fluxes at positions -2 .. n+1 and the face right-hand sides in
// LDS; writes -J D into dQ/dt.
template <typename R>
__global__ void __launch_bounds__(CPCR_THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_c6_faces_pcr(const Prob* __restrict__ probs, StateRef ref, int d,
                                                      int mask) {
  extern __shared__ double lds[];
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || tile_use(P, d, TK_FACES, mask) || !c6_face_pcr(P, d) || c6f_part_use(P, d, mask)) return;
  const int nlines = interior_lines(P, d);
  const bool periodic = P.bc[d][0] == BC_PERIODIC;
  const int g = P.g[d], n = P.n[d], sd = P.s[d];
  const int m = periodic ? n : n - 1;
  const R* F = static_cast<const R*>(P.FL[d]);
  double* dQ = ref.deriv(P);
  const size_t T = P.total;
  double* f = lds;          // positions -2 .. n+1
  double* r = lds + n + 4;  // faces
  for (int blk = blockIdx.x; blk < 5 * nlines; blk += gridDim.x) {
    const int line = blk % nlines, q = blk / nlines;
    const size_t base = interior_line_base(P, d, line);
    for (int p = threadIdx.x; p < n + 4; p += blockDim.x) f[p] = (double)F[q * T + base + (size_t)(g - 2 + p) * sd];
    __syncthreads();
    // boundary faces (bounded lines): I4 of the node fluxes
    const double lo = (7.0 * (f[1] + f[2]) - (f[0] + f[3])) / 12.0;
    const double hi = (7.0 * (f[n + 1] + f[n + 2]) - (f[n] + f[n + 3])) / 12.0;
    for (int k = threadIdx.x; k < m; k += blockDim.x) {
      double v;
      if (periodic) {
        v = C6F_A * (f[2 + k] + f[2 + wrap(k + 1, n)]) + C6F_B * (f[2 + wrap(k - 1, n)] + f[2 + wrap(k + 2, n)]);
      } else {
        v = C6F_A * (f[2 + k] + f[3 + k]) + C6F_B * (f[1 + k] + f[4 + k]);
        if (k == 0) v = v - C6_ALPHA * lo;
        if (k == m - 1) v = v - C6_ALPHA * hi;
      }
      r[k] = v;
    }
    __syncthreads();
    pcr_lds(r, m, periodic, P.pcrc[d], LG_PCR_STEPS);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      double fp, fm;
      if (periodic) {
        fp = r[i];
        fm = r[wrap(i - 1, n)];
      } else {
        fp = i < m ? r[i] : hi;
        fm = i > 0 ? r[i - 1] : lo;
      }
      const size_t idx = base + (size_t)(g + i) * sd;
      dQ[q * T + idx] = -met64(P, 9, (int)idx) * (fp - fm);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ implicit filter
// right-hand side of row i from the window w[0..10] = phi_{i-5} .. phi_{i+5}
__device__ __forceinline__ double filt_rhs(const Prob& P, const double w[11]) {
  double v = P.fcoef[0] * w[5];
  for (int k = 1; k <= 5; ++k) v = v + (0.5 * P.fcoef[k]) * (w[5 + k] + w[5 - k]);
  return v;
}

// Which filter runs after a stage (host-chosen mode, decided on the device from the stage's
// troubled-cell reduction): FILT_ALL filters every interior node (LAD scheme); FILT_GLOBAL
// filters every interior node unless the stage ran C-GBR (global hybrid: any troubled
// node); FILT_PERCELL keeps the values of the nodes in the dilated troubled set ft when
// the stage had any troubled node (per-cell hybrid).
__device__ __forceinline__ bool filt_skip(const Prob& P, int mode) {
  return mode == FILT_GLOBAL && *P.any_flag != 0;
}
__device__ __forceinline__ bool filt_keep(const Prob& P, int mode, size_t node) {
  return mode == FILT_PERCELL && *P.any_flag != 0 && P.ft[node] != 0;
}

// One lane per (interior line, conserved variable); in place on the state.
__global__ void __launch_bounds__(256) k_filter(const Prob* __restrict__ probs, StateRef ref, int d, int mask,
                                                int mode) {
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || !(P.falpha < 0.5) || filt_part_use(P, d, mask) || tile_use(P, d, TK_FILTER, mask) ||
      filt_pcr(P, d) || filt_seg_use(P, d, mask))
    return;
  if (filt_skip(P, mode)) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nl = interior_lines(P, d);
  if (t >= 5 * nl) return;
  const int line = t % nl, q = t / nl;
  double* Q = ref.state(P);
  const size_t T = P.total;
  double* S = P.T64;
  const double* tab = P.trf[d];
  const size_t base = interior_line_base(P, d, line);
  const int sd = P.s[d], g = P.g[d], n = P.n[d];
  const double al = P.falpha;
  const bool periodic = P.bc[d][0] == BC_PERIODIC;
  {
    double* phi = Q + (size_t)q * T + base;
    double* Sq = S + (size_t)q * T + base;
    auto at = [&](int p) { return phi[(size_t)(g + (periodic ? wrap(p, n) : p)) * sd]; };
    const double* cp = tab;
    const double* inv = tab + n;
    double w[11];
    for (int p = 0; p < 10; ++p) w[p] = at(p - 5);
    double dprev = 0.0;
    if (!periodic) {
      const double* sub = tab + 2 * n;
      const double gl = at(-1), gh = at(n);
      for (int i = 0; i < n; ++i) {
        w[10] = at(i + 5);
        double r = filt_rhs(P, w);
        if (i == 0) r = r - al * gl;
        if (i == n - 1) r = r - al * gh;
        const double dd = (r - sub[i] * dprev) * inv[i];
        Sq[(size_t)(g + i) * sd] = dd;
        dprev = dd;
        for (int p = 0; p < 10; ++p) w[p] = w[p + 1];
      }
      double y = dprev;
      if (!filt_keep(P, mode, base + (size_t)(g + n - 1) * sd)) phi[(size_t)(g + n - 1) * sd] = y;
      for (int i = n - 2; i >= 0; --i) {
        y = Sq[(size_t)(g + i) * sd] - cp[i] * y;
        if (!filt_keep(P, mode, base + (size_t)(g + i) * sd)) phi[(size_t)(g + i) * sd] = y;
      }
    } else {
      const double* z = tab + 2 * n;
      const double fac = tab[3 * n];
      const double* y0c = tab + 3 * n + 2;
      double y0 = 0.0;
      for (int i = 0; i < n; ++i) {
        w[10] = at(i + 5);
        const double r = filt_rhs(P, w);
        const double dd = (i == 0 ? r : r - al * dprev) * inv[i];
        Sq[(size_t)(g + i) * sd] = dd;
        dprev = dd;
        y0 = y0 + y0c[i] * dd;
        for (int p = 0; p < 10; ++p) w[p] = w[p + 1];
      }
      // one back substitution writing x = y - (y_0 - al y_{n-1}) fac z (the forward pass
      // has read every input it needs)
      const double vy = (y0 - al * dprev) * fac;
      double y = dprev;
      if (!filt_keep(P, mode, base + (size_t)(g + n - 1) * sd)) phi[(size_t)(g + n - 1) * sd] = y - vy * z[n - 1];
      for (int i = n - 2; i >= 0; --i) {
        y = Sq[(size_t)(g + i) * sd] - cp[i] * y;
        if (!filt_keep(P, mode, base + (size_t)(g + i) * sd)) phi[(size_t)(g + i) * sd] = y - vy * z[i];
      }
    }
  }
}

// Contiguous lines: one workgroup per (interior line, variable); the line in LDS, the
// interior unknowns reduced by PCR, written back in place.
__global__ void __launch_bounds__(CPCR_THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_filter_pcr(const Prob* __restrict__ probs, StateRef ref, int d,
                                                    int mask, int mode) {
  extern __shared__ double lds[];
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || !(P.falpha < 0.5) || filt_part_use(P, d, mask) || tile_use(P, d, TK_FILTER, mask) ||
      !filt_pcr(P, d))
    return;
  if (filt_skip(P, mode)) return;
  const int nlines = interior_lines(P, d);
  const bool periodic = P.bc[d][0] == BC_PERIODIC;
  const int g = P.g[d], n = P.n[d], N = P.N[d], sd = P.s[d];
  const double al = P.falpha;
  double* Q = ref.state(P);
  const size_t T = P.total;
  double* f = lds;       // the whole line
  double* r = lds + N;   // interior unknowns
  for (int blk = blockIdx.x; blk < 5 * nlines; blk += gridDim.x) {
    const int line = blk % nlines, q = blk / nlines;
    const size_t lb0 = interior_line_base(P, d, line);
    double* phi = Q + (size_t)q * T + lb0;
    for (int p = threadIdx.x; p < N; p += blockDim.x) f[p] = phi[(size_t)p * sd];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      double w[11];
      for (int k = -5; k <= 5; ++k) w[k + 5] = f[g + (periodic ? wrap(i + k, n) : i + k)];
      double v = filt_rhs(P, w);
      if (!periodic) {
        if (i == 0) v = v - al * f[g - 1];
        if (i == n - 1) v = v - al * f[g + n];
      }
      r[i] = v;
    }
    __syncthreads();
    pcr_lds(r, n, periodic, P.pcrf[d], P.fsteps);
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      if (!filt_keep(P, mode, lb0 + (size_t)(g + i) * sd)) phi[(size_t)(g + i) * sd] = r[i];
    __syncthreads();
  }
}

// ------------------------------------------------------------------ filter, strided segments
// Lines along eta / zeta of n <= FSEG_SMAX * FSEG_LM unknowns, bounded or periodic.  A
// workgroup takes 64 neighbouring lines (consecutive along xi, so every load and store of a
// wave is one contiguous run) and one variable; wave s holds segment s of all 64 lines,
// S = ceil(n / FSEG_LM) segments of L = n / S or one more unknowns.  Each lane reads its
// segment and the five values on either side once, forms the right-hand sides and solves
// the segment's own [a, 1, a] system T y = r in registers (the forward values overwrite the
// window slots they no longer need), so the line never goes through FP64 scratch.  With
// u = T^{-1} e_1 and v = T^{-1} e_L the solution is x = y - a u B_{s-1} - a v A_{s+1}
// (A_s, B_s: first and last unknown of segment s; bounded lines drop the terms past their
// ends, periodic lines wrap), so the 2S joint unknowns solve M z = (y_s[0], y_s[L-1])_s.
// M depends on n, S and a only: its LU factors (no pivoting: M inherits the diagonal
// dominance of the filter matrix), the segment factors and u, v are host-built tables, and
// lane t of wave 0 solves the joint system of line t.
template <int LM>
__global__ void __launch_bounds__(64 * FSEG_SMAX) k_filter_seg(const Prob* __restrict__ probs, StateRef ref, int d,
                                                                int mask, int mode) {
  constexpr int SM = FSEG_SMAX, M2 = 2 * SM;
  __shared__ double tab[FSEG_TABLE];      // cp, 1 / pivot, u, v, joint LU (host-built, see lgbr.cpp)
  __shared__ double ends[SM][2][64];      // y_s[0], y_s[L-1] of each line; then A_s, B_s
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || !(P.falpha < 0.5) || !filt_seg_use(P, d, mask) || filt_skip(P, mode)) return;
  const int n = P.n[d], g = P.g[d], sd = P.s[d];
  const int S = fseg_count(n);
  const int base = n / S, extra = n % S;   // the first `extra` segments have base + 1
  const int nlines = interior_lines(P, d);
  const int q = blockIdx.x % 5, grp = blockIdx.x / 5;
  if (grp * 64 >= nlines) return;
  const bool periodic = P.bc[d][0] == BC_PERIODIC;
  const double al = P.falpha;
  const int lane = threadIdx.x & 63, s = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < FSEG_TABLE; e += blockDim.x) tab[e] = P.fsegt[d][e];
  const double* tcp = tab + FSEG_CP;
  const double* tinv = tab + FSEG_INV;
  const int line = grp * 64 + lane;
  const bool act = s < S && line < nlines;
  const int L = base + (s < extra ? 1 : 0);
  const int j0 = s * base + min(s, extra);   // first unknown of this lane's segment
  const double* tu = tab + FSEG_U + (s < extra ? LM + 1 : 0);
  const double* tv = tab + FSEG_V + (s < extra ? LM + 1 : 0);
  double* Q = ref.state(P);
  const size_t T = P.total;
  const size_t lb = act ? interior_line_base(P, d, line) : 0;
  double* phi = Q + (size_t)q * T + lb;
  auto at = [&](int p) { return phi[(ptrdiff_t)(g + (periodic ? wrap(p, n) : p)) * sd]; };
  // w[i] = phi_{j0 + i - 5}; after row i, w[i] (no longer read) holds the forward value d_i,
  // then y_i after the back substitution
  double w[LM + 10];
  if (act) {
#pragma unroll
    for (int i = 0; i < LM + 10; ++i)
      if (i < L + 10) w[i] = at(j0 + i - 5);
  }
  __syncthreads();   // every lane has read its window before any lane writes a result; tables in LDS
  double ya = 0.0, yb = 0.0;
  if (act) {
    double prev = 0.0;
#pragma unroll
    for (int i = 0; i < LM; ++i) {
      if (i < L) {
        double r = filt_rhs(P, &w[i]);
        const int j = j0 + i;
        if (!periodic && j == 0) r = r - al * w[i + 4];
        if (!periodic && j == n - 1) r = r - al * w[i + 6];
        prev = (r - (i > 0 ? al * prev : 0.0)) * tinv[i];
        w[i] = prev;
      }
    }
    yb = prev;
    double v = prev;
#pragma unroll
    for (int i = LM - 2; i >= 0; --i) {
      if (i < L - 1) {
        v = w[i] - tcp[i] * v;
        w[i] = v;
      }
    }
    ya = w[0];
    ends[s][0][lane] = ya;
    ends[s][1][lane] = yb;
  }
  __syncthreads();
  if (s == 0 && line < nlines) {   // L U z = (y_s[0], y_s[L-1])_s, in place in ends
    const double* lu = tab + FSEG_LU;
    const int m = 2 * S;
    double z[M2];
#pragma unroll
    for (int r = 0; r < M2; ++r) {
      if (r < m) {
        double v = ends[r >> 1][r & 1][lane];
#pragma unroll
        for (int c = 0; c < r; ++c) v -= lu[r * M2 + c] * z[c];
        z[r] = v;
      }
    }
#pragma unroll
    for (int r = M2 - 1; r >= 0; --r) {
      if (r < m) {
        double v = z[r];
#pragma unroll
        for (int c = r + 1; c < M2; ++c)
          if (c < m) v -= lu[r * M2 + c] * z[c];
        z[r] = v / lu[r * M2 + r];
        ends[r >> 1][r & 1][lane] = z[r];
      }
    }
  }
  __syncthreads();
  if (act) {
    const int sp = s - 1, sn = s + 1;
    const double Bm = (periodic || sp >= 0) ? ends[(sp + S) % S][1][lane] : 0.0;
    const double Ap = (periodic || sn < S) ? ends[sn % S][0][lane] : 0.0;
#pragma unroll
    for (int i = 0; i < LM; ++i) {
      if (i < L) {
        const size_t node = lb + (size_t)(g + j0 + i) * sd;
        if (!filt_keep(P, mode, node)) phi[(size_t)(g + j0 + i) * sd] = w[i] - al * tu[i] * Bm - al * tv[i] * Ap;
      }
    }
  }
}

// ------------------------------------------------------------------ C4 gradients, strided segments
// MIG4 gradients along eta / zeta (Sec. 2.3; the C4 rows of k_grad.hip) in register
// segments, as k_filter_seg filters: 64 neighbouring lines (consecutive along xi) and one
// primitive per workgroup, wave s segment s of every line, the segments joined through the
// LU of their first and last unknowns (host tables for a = 1/4).  A bounded line of N nodes
// has one-sided end rows that decouple: its unknowns are rows 1 .. N-2, the two end values
// moved to the right-hand side.  A periodic line's unknowns are its n interior nodes
// (cyclic), and its ghosts take the periodic images.  Right-hand sides 3 (f_{i+1} -
// f_{i-1}) / 4 from FP64 primitives formed from the state; the gradients go to G in the bulk
// type.  Region-free launches only (every line; in a per-cell stage, when most lines are
// listed).  C6: the LAD-C6 gradients of periodic lines, the cyclic [1/3, 1, 1/3] system with
// the sixth-order right-hand side (tables for a = 1/3).
template <typename R, int LM, bool C6>
__global__ void __launch_bounds__(64 * FSEG_SMAX) k_grad_c4_seg(const Prob* __restrict__ probs, StateRef ref, int d,
                                                                 int skip_if_any, int dense_only, int mask) {
  constexpr int SM = FSEG_SMAX, M2 = 2 * SM;
  __shared__ double tab[FSEG_TABLE];      // cp, 1 / pivot, u, v, joint LU (host-built)
  __shared__ double ends[SM][2][64];      // y_s[0], y_s[L-1] of each line; then A_s, B_s
  const Prob& P = probs[blockIdx.y];
  if (!(C6 ? c6g_seg_use(P, d, mask) : c4_seg_use(P, d, mask)) || gate_skip(P, skip_if_any)) return;
  if (dense_only && !dense_lines(P, d)) return;
  const bool periodic = C6 || P.bc[d][0] == BC_PERIODIC;   // C6: periodic lines only
  const int N = P.N[d], n = P.n[d], g = P.g[d], sd = P.s[d];
  const int m = C6 ? n : c4_seg_unknowns(P, d);
  const int S = fseg_count(m);
  const int base = m / S, extra = m % S;   // the first `extra` segments have base + 1
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const int nlines = P.N[o1] * P.N[o2];
  const int q = blockIdx.x % 5, grp = blockIdx.x / 5;
  if (grp * 64 >= nlines) return;
  const double al = C6 ? C6_ALPHA : 0.25;
  const int lane = threadIdx.x & 63, s = threadIdx.x >> 6;
  const double* tsrc = C6 ? P.c6gsegt[d] : P.c4segt[d];
  for (int e = threadIdx.x; e < FSEG_TABLE; e += blockDim.x) tab[e] = tsrc[e];
  const double* tcp = tab + FSEG_CP;
  const double* tinv = tab + FSEG_INV;
  const int line = grp * 64 + lane;
  const bool act = s < S && line < nlines;
  const int L = base + (s < extra ? 1 : 0);
  const int j0 = s * base + min(s, extra);   // first unknown of this lane's segment
  const double* tu = tab + FSEG_U + (s < extra ? LM + 1 : 0);
  const double* tv = tab + FSEG_V + (s < extra ? LM + 1 : 0);
  const double* Q = ref.state(P);
  R* G = static_cast<R*>(P.G[d]);
  const size_t T = P.total;
  const double gm1 = P.gamma - 1.0;
  const size_t lb = act ? (size_t)(line % P.N[o1]) * P.s[o1] + (size_t)(line / P.N[o1]) * P.s[o2] : 0;
  // line position of window slot i: the rows j0 .. j0 + L + 1 around this segment's rows
  // j0 + 1 .. j0 + L (bounded), the interior nodes j0 - 1 .. j0 + L wrapped (periodic)
  constexpr int WX = C6 ? 4 : 2;   // window slots beyond the segment's rows
  auto pos = [&](int i) { return periodic ? g + wrap(j0 + i - WX / 2, n) : j0 + i; };
  // w[i] = f at pos(i); after row i, w[i] (no longer read) holds the forward value, then y_i
  double w[LM + WX];
  double d0 = 0.0, dN = 0.0;   // the decoupled end rows of a bounded line
  if (act) {
#pragma unroll
    for (int i = 0; i < LM + WX; ++i)
      if (i < L + WX) prims_q<1>(Q, T, lb + (size_t)pos(i) * sd, gm1, q, &w[i]);
    if (!periodic && s == 0) d0 = (-3.0 * w[0] + 4.0 * w[1] - w[2]) / 2.0;
  }
  __syncthreads();   // tables in LDS
  double ya = 0.0, yb = 0.0;
  if (act) {
    double prev = 0.0;
#pragma unroll
    for (int i = 0; i < LM; ++i) {
      if (i < L) {
        double r = C6 ? C6_A * (w[i + 3] - w[i + 1]) + C6_B * (w[i + 4] - w[i]) : 0.75 * (w[i + 2] - w[i]);
        const int j = j0 + i;
        if (!periodic && j == 0) r = r - al * d0;
        if (!periodic && j == m - 1) {   // rows N-3 .. N-1 are slots i .. i + 2 here
          dN = (3.0 * w[i + 2] - 4.0 * w[i + 1] + w[i]) / 2.0;
          r = r - al * dN;
        }
        prev = (r - (i > 0 ? al * prev : 0.0)) * tinv[i];
        w[i] = prev;
      }
    }
    yb = prev;
    double v = prev;
#pragma unroll
    for (int i = LM - 2; i >= 0; --i) {
      if (i < L - 1) {
        v = w[i] - tcp[i] * v;
        w[i] = v;
      }
    }
    ya = w[0];
    ends[s][0][lane] = ya;
    ends[s][1][lane] = yb;
  }
  __syncthreads();
  if (s == 0 && line < nlines) {   // L U z = (y_s[0], y_s[L-1])_s, in place in ends
    const double* lu = tab + FSEG_LU;
    const int m2 = 2 * S;
    double z[M2];
#pragma unroll
    for (int r = 0; r < M2; ++r) {
      if (r < m2) {
        double v = ends[r >> 1][r & 1][lane];
#pragma unroll
        for (int c = 0; c < r; ++c) v -= lu[r * M2 + c] * z[c];
        z[r] = v;
      }
    }
#pragma unroll
    for (int r = M2 - 1; r >= 0; --r) {
      if (r < m2) {
        double v = z[r];
#pragma unroll
        for (int c = r + 1; c < M2; ++c)
          if (c < m2) v -= lu[r * M2 + c] * z[c];
        z[r] = v / lu[r * M2 + r];
        ends[r >> 1][r & 1][lane] = z[r];
      }
    }
  }
  __syncthreads();
  if (act) {
    const int sp = s - 1, sn = s + 1;
    const double Bm = (periodic || sp >= 0) ? ends[(sp + S) % S][1][lane] : 0.0;
    const double Ap = (periodic || sn < S) ? ends[sn % S][0][lane] : 0.0;
    R* Gl = G + (size_t)q * T + lb;
#pragma unroll
    for (int i = 0; i < LM; ++i) {
      if (i < L) {
        const int j = j0 + i;
        const R x = (R)(w[i] - al * tu[i] * Bm - al * tv[i] * Ap);
        if (periodic) {
          Gl[(size_t)(g + j) * sd] = x;
          if (j < g) Gl[(size_t)(g + n + j) * sd] = x;            // ghost images past the end
          if (j >= n - g) Gl[(size_t)(j - (n - g)) * sd] = x;     // ... and before the start
        } else {
          Gl[(size_t)(j + 1) * sd] = x;
        }
      }
    }
    if (!periodic && s == 0) Gl[0] = (R)d0;
    if (!periodic && s == S - 1) Gl[(size_t)(N - 1) * sd] = (R)dN;
  }
}

// ------------------------------------------------------------------ C6 interface fluxes, strided segments
// LAD-C6 interface fluxes along eta / zeta (the [1/3, 1, 1/3] face system of k_c6_faces) in
// register segments, as k_filter_seg filters: 64 neighbouring lines (consecutive along xi)
// and one flux component per workgroup, wave s segment s of every line, the segments
// joined through the LU of their first and last faces (host tables for a = 1/3).  A
// bounded line's unknowns are its n - 1 interior faces (face j between nodes j and j + 1),
// the fourth-order boundary faces moved to the right-hand side; a periodic line's are its
// n faces.  Each segment then emits -J D for its own nodes j0 .. j0 + L - 1 (D = right
// face - left face; the left face of node j0 is the previous segment's last face, the low
// boundary face, or the periodic image), the last segment of a bounded line also node
// n - 1, into dQ/dt (accumulated after the first direction), or, in the last direction of
// an RK stage, the stage combination of its component (a U^n + b (U^s + dt L)); the
// non-physical count of the stage result then takes its own pass (k_c6_seg_check), since it
// needs the five components of a node together.  Region-free stages only.
template <typename R, int LM, bool RK>
__global__ void __launch_bounds__(64 * C6FSEG_SMAX) k_c6_faces_seg(const Prob* __restrict__ probs, StateRef ref, int d,
                                                                  int accumulate, int mask, RKRef rr, int stage,
                                                                  double a, double b) {
  constexpr int SM = C6FSEG_SMAX, M2 = 2 * SM, M2T = 2 * FSEG_SMAX;   // joint unknowns; table row stride
  __shared__ double tab[FSEG_TABLE];      // cp, 1 / pivot, u, v, joint LU (host-built)
  __shared__ double ends[SM][2][64];      // y_s[0], y_s[L-1] of each line; then A_s, B_s
  const Prob& P = probs[blockIdx.y];
  if (!c6f_seg_use(P, d, mask)) return;
  const bool periodic = P.bc[d][0] == BC_PERIODIC;
  const int n = P.n[d], g = P.g[d], sd = P.s[d];
  const int m = c6f_seg_unknowns(P, d);
  const int S = fseg_count(m);
  const int base = m / S, extra = m % S;   // the first `extra` segments have base + 1
  const int nlines = interior_lines(P, d);
  const int q = blockIdx.x % 5, grp = blockIdx.x / 5;
  if (grp * 64 >= nlines) return;
  const double al = C6_ALPHA;
  const int lane = threadIdx.x & 63, s = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < FSEG_TABLE; e += blockDim.x) tab[e] = P.c6fsegt[d][e];
  const double* tcp = tab + FSEG_CP;
  const double* tinv = tab + FSEG_INV;
  const int line = grp * 64 + lane;
  const bool act = s < S && line < nlines;
  const int L = base + (s < extra ? 1 : 0);
  const int j0 = s * base + min(s, extra);   // first face of this lane's segment
  const double* tu = tab + FSEG_U + (s < extra ? LM + 1 : 0);
  const double* tv = tab + FSEG_V + (s < extra ? LM + 1 : 0);
  const size_t T = P.total;
  const size_t lb = act ? interior_line_base(P, d, line) : 0;
  const R* F = static_cast<const R*>(P.FL[d]) + (size_t)q * T + lb;
  auto at = [&](int p) { return (double)F[(ptrdiff_t)(g + (periodic ? wrap(p, n) : p)) * sd]; };
  // w[i] = F at node j0 + i - 1 (faces j0 + i use nodes j0 + i - 1 .. j0 + i + 2); after row
  // i, w[i] (no longer read) holds the forward value, then y_i, then the face
  double w[LM + 3];
  double lo = 0.0, hi = 0.0;   // boundary faces of a bounded line
  if (act) {
#pragma unroll
    for (int i = 0; i < LM + 3; ++i)
      if (i < L + 3) w[i] = at(j0 + i - 1);
    if (!periodic && s == 0) lo = (7.0 * (w[0] + w[1]) - (at(-2) + w[2])) / 12.0;
    if (!periodic && s == S - 1) {   // nodes n - 2 .. n are slots L .. L + 2
#pragma unroll
      for (int i = 0; i < LM; ++i)
        if (i == L - 1) hi = (7.0 * (w[i + 2] + w[i + 3]) - (w[i + 1] + at(n + 1))) / 12.0;
    }
  }
  __syncthreads();   // tables in LDS
  if (act) {
    double prev = 0.0;
#pragma unroll
    for (int i = 0; i < LM; ++i) {
      if (i < L) {
        double r = C6F_A * (w[i + 1] + w[i + 2]) + C6F_B * (w[i] + w[i + 3]);
        const int j = j0 + i;
        if (!periodic && j == 0) r = r - al * lo;
        if (!periodic && j == m - 1) r = r - al * hi;
        prev = (r - (i > 0 ? al * prev : 0.0)) * tinv[i];
        w[i] = prev;
      }
    }
    double v = prev;
#pragma unroll
    for (int i = LM - 2; i >= 0; --i) {
      if (i < L - 1) {
        v = w[i] - tcp[i] * v;
        w[i] = v;
      }
    }
    ends[s][0][lane] = w[0];
    ends[s][1][lane] = prev;
  }
  __syncthreads();
  if (s == 0 && line < nlines) {   // L U z = (y_s[0], y_s[L-1])_s, in place in ends
    const double* lu = tab + FSEG_LU;
    const int m2 = 2 * S;
    double z[M2];
#pragma unroll
    for (int r = 0; r < M2; ++r) {
      if (r < m2) {
        double v = ends[r >> 1][r & 1][lane];
#pragma unroll
        for (int c = 0; c < r; ++c) v -= lu[r * M2T + c] * z[c];
        z[r] = v;
      }
    }
#pragma unroll
    for (int r = M2 - 1; r >= 0; --r) {
      if (r < m2) {
        double v = z[r];
#pragma unroll
        for (int c = r + 1; c < M2; ++c)
          if (c < m2) v -= lu[r * M2T + c] * z[c];
        z[r] = v / lu[r * M2T + r];
        ends[r >> 1][r & 1][lane] = z[r];
      }
    }
  }
  __syncthreads();
  if (act) {
    const int sp = s - 1, sn = s + 1;
    const double Bm = (periodic || sp >= 0) ? ends[(sp + S) % S][1][lane] : 0.0;
    const double Ap = (periodic || sn < S) ? ends[sn % S][0][lane] : 0.0;
    double* dQ = ref.deriv(P) + (size_t)q * T + lb;
    // the RK stage's arrays (as rk_combine_node): U^n, U^s and the result, this component
    const double* Un = (rr.Un ? rr.Un : P.Q) + (size_t)q * T + lb;
    const double* Us = RK ? (rr.Us ? rr.Us + (size_t)q * T + lb : (stage == 0 ? Un : P.Us + (size_t)q * T + lb)) : Un;
    double* out = rr.out ? rr.out + (size_t)q * T + lb
                         : (stage == 2 ? const_cast<double*>(Un) : P.Us + (size_t)q * T + lb);
    const double dt = RK ? *P.dt : 0.0;
    double left = sp >= 0 ? Bm : (periodic ? ends[S - 1][1][lane] : lo);
    // eight nodes at a time: their loads are all in flight before the stores
    constexpr int CH = 8;
#pragma unroll
    for (int c = 0; c < LM; c += CH) {
      if (c < L) {
        double Jv[CH], dv[CH], un[CH], us[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          if (c + u < L) {
            const size_t o = (size_t)(g + j0 + c + u) * sd;
            Jv[u] = met64(P, 9, (int)(lb + o));
            dv[u] = accumulate ? dQ[o] : 0.0;
            if (RK) {
              un[u] = Un[o];
              us[u] = Us[o];
            }
          }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          if (c + u < L) {
            const double x = w[c + u] - al * tu[c + u] * Bm - al * tv[c + u] * Ap;
            const double Lv = dv[u] - Jv[u] * (x - left);
            const size_t o = (size_t)(g + j0 + c + u) * sd;
            if (RK) out[o] = a * un[u] + b * (us[u] + dt * Lv);
            else dQ[o] = Lv;
            left = x;
          }
        }
      }
    }
    if (!periodic && s == S - 1) {   // node n - 1: the high boundary face on its right
      const size_t o = (size_t)(g + n - 1) * sd;
      const double Lv = (accumulate ? dQ[o] : 0.0) - met64(P, 9, (int)(lb + o)) * (hi - left);
      if (RK) out[o] = a * Un[o] + b * (Us[o] + dt * Lv);
      else dQ[o] = Lv;
    }
  }
}

// Non-physical count of an RK stage whose last direction k_c6_faces_seg combined: interior
// nodes of the result, tested as rk_combine_node tests them.
__global__ void __launch_bounds__(256) k_c6_seg_check(const Prob* __restrict__ probs, RKRef rr, int stage, int mask) {
  const Prob& P = probs[blockIdx.y];
  if (!c6f_seg_use(P, P.ndim - 1, mask)) return;
  const size_t T = P.total;
  const double* Un = rr.Un ? rr.Un : P.Q;
  const double* out = rr.out ? rr.out : (stage == 2 ? Un : P.Us);
  const int n0 = P.n[0], n1 = P.n[1], rows = n1 * P.n[2];
  int bad = 0;
  for (int r = blockIdx.x; r < rows; r += gridDim.x) {   // one xi row of interior nodes per step
    const int row0 = (P.g[1] + r % n1) * P.s[1] + (P.g[2] + r / n1) * P.s[2] + P.g[0];
    for (int i = threadIdx.x; i < n0; i += blockDim.x) {
      const int idx = row0 + i;
      double v[5];
      for (int q = 0; q < 5; ++q) v[q] = out[(size_t)q * T + idx];
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

// ------------------------------------------------------------------ filter positivity guard
// A hybrid stage's filter (the LAD phase's FILTER_CALLS) must not hand the next stage a
// non-physical node: the filter's ringing at a sharp jump that the LAD stage has not yet
// smoothed can drive a small density or pressure below zero.  Such a node is troubled in
// the sense of the hybrid's criterion (Sec. 5) and keeps its unfiltered state: the stage
// result is saved before the passes (into the time-derivative workspace, free once the
// stage is combined) and restored after them wherever the filtered density or pressure is
// not positive or not finite.  The test forms p as the primitives kernel does (FP64).
__global__ void __launch_bounds__(256) k_filter_save(const Prob* __restrict__ probs, StateRef ref, int mode) {
  const Prob& P = probs[blockIdx.y];
  if (!(P.falpha < 0.5) || filt_skip(P, mode)) return;
  const double* Q = ref.state(P);
  double* S = P.dQ;
  const size_t n5 = 5 * (size_t)P.total;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n5; e += (size_t)gridDim.x * blockDim.x)
    S[e] = Q[e];
}

__global__ void __launch_bounds__(256) k_filter_guard(const Prob* __restrict__ probs, StateRef ref, int mode) {
  const Prob& P = probs[blockIdx.y];
  if (!(P.falpha < 0.5) || filt_skip(P, mode)) return;
  double* Q = ref.state(P);
  const double* S = P.dQ;
  const size_t T = P.total;
  const double gm1 = P.gamma - 1.0;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < P.total; idx += gridDim.x * blockDim.x) {
    const int p[3] = {idx % P.N[0], (idx / P.N[0]) % P.N[1], idx / (P.N[0] * P.N[1])};
    bool inner = true;
    for (int l = 0; l < 3; ++l)
      if (l < P.ndim && (p[l] < P.g[l] || p[l] >= P.g[l] + P.n[l])) inner = false;
    if (!inner) continue;
    double v[5];
    bool fin = true;
    for (int q = 0; q < 5; ++q) {
      v[q] = Q[q * T + idx];
      fin = fin && isfinite(v[q]);
    }
    const double rho = v[0], u = v[1] / rho, w1 = v[2] / rho, w2 = v[3] / rho;
    const double pr = gm1 * (v[4] - 0.5 * rho * (u * u + w1 * w1 + w2 * w2));
    if (fin && rho > 0.0 && pr > 0.0) continue;
    for (int q = 0; q < 5; ++q) Q[q * T + idx] = S[q * T + idx];
  }
}

// ------------------------------------------------------------------ filter, partition method
// Contiguous bounded lines of n interior unknowns (the tridiagonal [a, 1, a] system of the
// filter with the boundary neighbours moved to the right-hand side), one wave per (line,
// variable).  The line is staged in LDS with coalesced loads; lane s owns segment s of
// nseg = min(64, n / 2) segments of length n / nseg or one more and solves its segment
// system T y = r in registers.  With u = T^{-1} e_1 and v = T^{-1} e_L (a segment's response
// to its left and right neighbours, the same for every segment of one length) the solution
// is x = y - a u B_{s-1} - a v A_{s+1}, where A_s and B_s are the first and last unknowns of
// segment s.  Eliminating forward, B_{s-1} = gb_{s-1} - Gb_{s-1} A_s, and back,
// A_s = ga_s - Ga_s A_{s+1}: the factors da_s = 1 - a u1 Gb_{s-1}, Ga_s = a v1 / da_s and
// Gb_s = a vL + a uL Gb_{s-1} Ga_s do not depend on the data (tables per workgroup), and the
// data-dependent parts are first-order linear recurrences across the lanes,
//   gb_s = -(a uL / da_s) gb_{s-1} + yb_s + a uL Gb_{s-1} ya_s / da_s,
//   A_s = -Ga_s A_{s+1} + ga_s,   ga_s = (ya_s - a u1 gb_{s-1}) / da_s,
// solved by two wave-wide scans (six shuffle steps each).  Waves of a workgroup work on
// separate items and synchronise only among their own lanes.
constexpr int FPART_LMAX = 33;   // longest segment (n <= 2048 with 64 segments)
constexpr int FPART_LSHORT = 17;  // segments of lines of at most 1088 unknowns (register arrays sized to it)
constexpr int FPART_WAVES = 4;   // most (line, variable) items in flight per workgroup (one per wave)
// LDS doubles of one wave's staged line (interior + ghosts, one pad slot per 16)
__host__ __device__ inline int fpart_lds_slots(int nmax) { return (nmax + 10) + (nmax + 10) / 16 + 1; }

// orders the LDS accesses of the lanes of one wave (no other wave takes part)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// inclusive scan of x_s = m_s x_{s-1} + c_s over lanes 0..63 (x_{-1} = 0); returns x_lane
__device__ __forceinline__ double scan_up(double m, double c, int lane) {
#pragma unroll
  for (int k = 1; k < 64; k <<= 1) {
    const double mp = __shfl_up(m, k), cp = __shfl_up(c, k);
    if (lane >= k) {
      c = m * cp + c;
      m = m * mp;
    }
  }
  return c;
}

// the same recurrence run from lane 63 down to lane 0: x_s = m_s x_{s+1} + c_s (x_64 = 0)
__device__ __forceinline__ double scan_down(double m, double c, int lane) {
#pragma unroll
  for (int k = 1; k < 64; k <<= 1) {
    const double mp = __shfl_down(m, k), cp = __shfl_down(c, k);
    if (lane + k < 64) {
      c = m * cp + c;
      m = m * mp;
    }
  }
  return c;
}

template <int LM>
__global__ void __launch_bounds__(64 * FPART_WAVES) k_filter_part(const Prob* __restrict__ probs, StateRef ref,
                                                                  int mode, int nmax, int mask) {
  extern __shared__ double dyn[];   // per wave: the staged line [nmax + 10]
  __shared__ double tcp[FPART_LMAX], tinv[FPART_LMAX];
  __shared__ double tu[2][FPART_LMAX], tv[2][FPART_LMAX];   // segment lengths base and base + 1
  __shared__ double tda[64], tGa[64], tGb[64];
  const Prob& P = probs[blockIdx.y];
  if (!(P.falpha < 0.5) || !filt_part_use(P, 0, mask) || P.n[0] > nmax || filt_skip(P, mode)) return;
  if (P.n[0] / min(64, P.n[0] / 2) + 1 > LM) return;   // segments longer than the register arrays
  const int n = P.n[0], g = P.g[0], N = P.N[0];
  const int nseg = min(64, n / 2);
  const int base = n / nseg, extra = n % nseg;   // the first `extra` segments have base + 1
  const double al = P.falpha;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // segment factors (they depend on the row index only), the responses u, v, and the
  // data-independent elimination factors of the joint unknowns
  if (threadIdx.x == 0) {
    double c = 0.0;
    for (int i = 0; i < base + 1; ++i) {
      const double den = 1.0 - (i > 0 ? al * c : 0.0);
      tinv[i] = 1.0 / den;
      c = al / den;
      tcp[i] = c;
    }
  }
  __syncthreads();
  if (threadIdx.x < 4) {   // threads 0 / 1: u for base / base + 1; 2 / 3: v
    const int which = threadIdx.x & 1, L = base + which;
    const bool is_u = threadIdx.x < 2;
    double* out = is_u ? tu[which] : tv[which];
    double prev = 0.0;
    for (int i = 0; i < L; ++i) {
      const double rhs = is_u ? (i == 0 ? 1.0 : 0.0) : (i == L - 1 ? 1.0 : 0.0);
      prev = (rhs - (i > 0 ? al * prev : 0.0)) * tinv[i];
      out[i] = prev;
    }
    double y = out[L - 1];
    for (int i = L - 2; i >= 0; --i) {
      y = out[i] - tcp[i] * y;
      out[i] = y;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double Gbp = 0.0;
    for (int sg = 0; sg < nseg; ++sg) {
      const int lw = sg < extra ? 1 : 0, Ls = base + lw;
      const double da = 1.0 - al * tu[lw][0] * Gbp;
      const double Ga = al * tv[lw][0] / da;
      tda[sg] = da;
      tGa[sg] = Ga;
      tGb[sg] = al * tv[lw][Ls - 1] + al * tu[lw][Ls - 1] * Gbp * Ga;
      Gbp = tGb[sg];
    }
  }
  __syncthreads();
  // the staged line, padded by one slot every 16 so that the lanes' segments (16 and more
  // apart) fall into different LDS banks
  double* f = dyn + (size_t)w * fpart_lds_slots(nmax);
  auto F = [f](int p) -> double& { return f[p + (p >> 4)]; };
  const int nlines = interior_lines(P, 0);
  const size_t T = P.total;
  double* Q = ref.state(P);
  const bool act = lane < nseg;
  const int L = base + (lane < extra ? 1 : 0);
  const int j0 = lane * base + min(lane, extra);   // first unknown of this lane's segment
  const int wl = lane < extra ? 1 : 0;             // which u / v table
  const double u1 = act ? tu[wl][0] : 0.0, uL = act ? tu[wl][L - 1] : 0.0;
  const double da = act ? tda[lane] : 1.0, Ga = act ? tGa[lane] : 0.0, Gb = act ? tGb[lane] : 0.0;
  const double Gbm = act && lane > 0 ? tGb[lane - 1] : 0.0;
  for (int item = blockIdx.x * nw + w; item < 5 * nlines; item += gridDim.x * nw) {
    const int line = item % nlines, q = item / nlines;
    const size_t lb = interior_line_base(P, 0, line);
    double* phi = Q + (size_t)q * T + lb;
    for (int p = lane; p < N; p += 64) F(p) = phi[p];
    wave_lds_sync();
    double y[LM];
    double ya = 0.0, yb = 0.0;
    if (act) {
      double win[11];   // the staged values g + j - 5 .. g + j + 5 of the current unknown j
      for (int k = 0; k < 10; ++k) win[k + 1] = F(g + j0 - 5 + k);
      double prev = 0.0;
#pragma unroll
      for (int i = 0; i < LM; ++i) {
        if (i < L) {
          const int j = j0 + i;
#pragma unroll
          for (int k = 0; k < 10; ++k) win[k] = win[k + 1];
          win[10] = F(g + j + 5);
          double r = filt_rhs(P, win);
          if (j == 0) r = r - al * F(g - 1);
          if (j == n - 1) r = r - al * F(g + n);
          prev = (r - (i > 0 ? al * prev : 0.0)) * tinv[i];
          y[i] = prev;
        }
      }
      yb = prev;   // y_{L-1} = d_{L-1}
      double v = prev;
#pragma unroll
      for (int i = LM - 2; i >= 0; --i) {
        if (i < L - 1) {
          v = y[i] - tcp[i] * v;
          y[i] = v;
        }
      }
      ya = y[0];
    }
    // joint unknowns: gb by a forward scan, then ga, then A by a backward scan, then B
    const double gbv = scan_up(act ? -al * uL / da : 0.0, act ? yb + al * uL * Gbm * ya / da : 0.0, lane);
    double gbm = __shfl_up(gbv, 1);
    if (lane == 0) gbm = 0.0;
    const double gav = act ? (ya - al * u1 * gbm) / da : 0.0;
    const double A = scan_down(act ? -Ga : 0.0, gav, lane);
    double Ap = __shfl_down(A, 1);
    if (lane + 1 >= nseg) Ap = 0.0;
    const double B = gbv - Gb * Ap;
    double Bm = __shfl_up(B, 1);
    if (lane == 0) Bm = 0.0;
    if (act) {
#pragma unroll
      for (int i = 0; i < LM; ++i)
        if (i < L) F(g + j0 + i) = y[i] - al * tu[wl][i] * Bm - al * tv[wl][i] * Ap;
    }
    wave_lds_sync();
    for (int p = lane; p < n; p += 64)
      if (!filt_keep(P, mode, lb + (size_t)(g + p))) phi[g + p] = F(g + p);
    wave_lds_sync();   // the next item's staging overwrites f
  }
}

// ------------------------------------------------------------------ C4 / C6 gradients, partition method
// MIG4 gradients along xi on bounded lines (Sec. 2.3; the C4 rows of k_grad.hip), and the
// LAD-C6 gradients (Sec. 3; the rows of k_grad_c6).  The one-sided end rows of the padded
// line of N nodes decouple, so rows 1 .. N-2 form a system of M = N - 2 unknowns with the
// two end values moved to the right-hand side.  C4: the [1/4, 1, 1/4] system, which
// k_filter_part solves with a = alpha_f, solved the same way here (segments per lane, joint
// unknowns by two wave-wide scans).  C6: the [1/3, 1, 1/3] system T except that the first
// row's upper and the last row's lower neighbour carry 1/4 (the C4 rows next to the ends),
// T' = T - (e_0 e_1^T + e_{M-1} e_{M-2}^T) / 12; the scans solve T y = r, and the
// Sherman-Morrison-Woodbury identity gives x = y + (c_0 z_0 + c_M z_M) / 12, with z_0 =
// T^{-1} e_0, z_M = T^{-1} e_{M-1} (its mirror image) and (c_0, c_M) = (I - W)^{-1}
// (y_1, y_{M-2}) for W = [z_0 z_M] rows 1 and M-2 / 12.  z_0 decays by 0.38 per row, so
// its first 64 entries and the 2x2 inverse (host tables) carry the correction to FP64
// precision.  One wave per (line, primitive) over every line of the direction; the five
// primitives of a line are consecutive items, so their staging reads of the state share
// the cache.  Region-free launches only (every line; in a per-cell stage, when most lines
// are listed).
template <typename R, int LM, bool C6>
__global__ void __launch_bounds__(64 * FPART_WAVES) k_grad_part(const Prob* __restrict__ probs, StateRef ref,
                                                                int nmax, int skip_if_any, int dense_only,
                                                                int mask) {
  extern __shared__ double dyn[];   // per wave: the staged line [nmax + 10]
  __shared__ double tcp[FPART_LMAX], tinv[FPART_LMAX];
  __shared__ double tu[2][FPART_LMAX], tv[2][FPART_LMAX];   // segment lengths base and base + 1
  __shared__ double tda[64], tGa[64], tGb[64];
  const Prob& P = probs[blockIdx.y];
  if (!(C6 ? c6g_part_use(P, 0, mask) : c4_part_use(P, 0, mask)) || P.n[0] > nmax || gate_skip(P, skip_if_any))
    return;
  if (dense_only && !dense_lines(P, 0)) return;
  const int N = P.N[0], M = N - 2;
  const int nseg = min(64, M / 2);
  const int base = M / nseg, extra = M % nseg;   // the first `extra` segments have base + 1
  if (base + 1 > LM) return;   // segments longer than the register arrays
  const double al = C6 ? C6_ALPHA : 0.25;   // the system solved by the scans
  constexpr double ae = 0.25;                // coupling of rows 1 and N-2 to the end values
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // segment factors, the responses u = T^{-1} e_1 and v = T^{-1} e_L, and the
  // data-independent elimination factors of the joint unknowns (as in k_filter_part)
  if (threadIdx.x == 0) {
    double c = 0.0;
    for (int i = 0; i < base + 1; ++i) {
      const double den = 1.0 - (i > 0 ? al * c : 0.0);
      tinv[i] = 1.0 / den;
      c = al / den;
      tcp[i] = c;
    }
  }
  __syncthreads();
  if (threadIdx.x < 4) {   // threads 0 / 1: u for base / base + 1; 2 / 3: v
    const int which = threadIdx.x & 1, L = base + which;
    const bool is_u = threadIdx.x < 2;
    double* out = is_u ? tu[which] : tv[which];
    double prev = 0.0;
    for (int i = 0; i < L; ++i) {
      const double rhs = is_u ? (i == 0 ? 1.0 : 0.0) : (i == L - 1 ? 1.0 : 0.0);
      prev = (rhs - (i > 0 ? al * prev : 0.0)) * tinv[i];
      out[i] = prev;
    }
    double y = out[L - 1];
    for (int i = L - 2; i >= 0; --i) {
      y = out[i] - tcp[i] * y;
      out[i] = y;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double Gbp = 0.0;
    for (int sg = 0; sg < nseg; ++sg) {
      const int lw = sg < extra ? 1 : 0, Ls = base + lw;
      const double da = 1.0 - al * tu[lw][0] * Gbp;
      const double Ga = al * tv[lw][0] / da;
      tda[sg] = da;
      tGa[sg] = Ga;
      tGb[sg] = al * tv[lw][Ls - 1] + al * tu[lw][Ls - 1] * Gbp * Ga;
      Gbp = tGb[sg];
    }
  }
  __syncthreads();
  double* f = dyn + (size_t)w * fpart_lds_slots(nmax);
  auto F = [f](int p) -> double& { return f[p + (p >> 4)]; };
  const int nlines = P.N[1] * P.N[2];
  const size_t T = P.total;
  const double* Q = ref.state(P);
  R* G = static_cast<R*>(P.G[0]);
  const double gm1 = P.gamma - 1.0;
  const bool act = lane < nseg;
  const int L = base + (lane < extra ? 1 : 0);
  const int j0 = lane * base + min(lane, extra);   // first unknown of this lane's segment
  const int wl = lane < extra ? 1 : 0;             // which u / v table
  const double u1 = act ? tu[wl][0] : 0.0, uL = act ? tu[wl][L - 1] : 0.0;
  const double da = act ? tda[lane] : 1.0, Ga = act ? tGa[lane] : 0.0, Gb = act ? tGb[lane] : 0.0;
  const double Gbm = act && lane > 0 ? tGb[lane - 1] : 0.0;
  for (int item = blockIdx.x * nw + w; item < 5 * nlines; item += gridDim.x * nw) {
    const int line = item / 5, q = item % 5;
    const size_t lb = (size_t)(line % P.N[1]) * P.s[1] + (size_t)(line / P.N[1]) * P.s[2];
    for (int p = lane; p < N; p += 64) {
      double v;
      prims_q<1>(Q, T, lb + (size_t)p, gm1, q, &v);
      F(p) = v;
    }
    wave_lds_sync();
    // the decoupled end rows (second-order one-sided)
    const double d0 = (-3.0 * F(0) + 4.0 * F(1) - F(2)) / 2.0;
    const double dN = (3.0 * F(N - 1) - 4.0 * F(N - 2) + F(N - 3)) / 2.0;
    double y[LM];
    double ya = 0.0, yb = 0.0;
    if (act) {
      // unknown j is row j + 1: 3 (f_{j+2} - f_j) / 4 (C4, and the C6 rows next to the
      // ends, less 1/4 times the end value), else C6_A (f_{j+2} - f_j) + C6_B (f_{j+3} - f_{j-1})
      double fa = C6 && j0 > 0 ? F(j0 - 1) : 0.0, fm = F(j0), f0 = F(j0 + 1);
      double prev = 0.0;
#pragma unroll
      for (int i = 0; i < LM; ++i) {
        if (i < L) {
          const int j = j0 + i;
          const double fp = F(j + 2);
          const double fe = C6 && j + 3 < N ? F(j + 3) : 0.0;
          double r = C6 && j > 0 && j < M - 1 ? C6_A * (fp - fm) + C6_B * (fe - fa) : 0.75 * (fp - fm);
          if (j == 0) r = r - ae * d0;
          if (j == M - 1) r = r - ae * dN;
          prev = (r - (i > 0 ? al * prev : 0.0)) * tinv[i];
          y[i] = prev;
          fa = fm;
          fm = f0;
          f0 = fp;
        }
      }
      yb = prev;
      double v = prev;
#pragma unroll
      for (int i = LM - 2; i >= 0; --i) {
        if (i < L - 1) {
          v = y[i] - tcp[i] * v;
          y[i] = v;
        }
      }
      ya = y[0];
    }
    const double gbv = scan_up(act ? -al * uL / da : 0.0, act ? yb + al * uL * Gbm * ya / da : 0.0, lane);
    double gbm = __shfl_up(gbv, 1);
    if (lane == 0) gbm = 0.0;
    const double gav = act ? (ya - al * u1 * gbm) / da : 0.0;
    const double A = scan_down(act ? -Ga : 0.0, gav, lane);
    double Ap = __shfl_down(A, 1);
    if (lane + 1 >= nseg) Ap = 0.0;
    const double B = gbv - Gb * Ap;
    double Bm = __shfl_up(B, 1);
    if (lane == 0) Bm = 0.0;
    wave_lds_sync();   // every lane has read its window before the solution overwrites it
    if (act) {
#pragma unroll
      for (int i = 0; i < LM; ++i)
        if (i < L) F(1 + j0 + i) = y[i] - al * tu[wl][i] * Bm - al * tv[wl][i] * Ap;
    }
    if (lane == 0) {
      F(0) = d0;
      F(N - 1) = dN;
    }
    wave_lds_sync();
    if (C6) {   // x = y + (c_0 z_0 + c_M z_M) / 12 on the first and last 64 unknowns
      const double* zt = P.c6gz;
      const double y1 = F(2), yM = F(M - 1);   // unknowns 1 and M-2
      const double c0 = (zt[64] * y1 + zt[65] * yM) / 12.0, cM = (zt[66] * y1 + zt[67] * yM) / 12.0;
      const double z = zt[lane];
      wave_lds_sync();   // every lane has read y_1 and y_{M-2}
      F(1 + lane) = F(1 + lane) + c0 * z;     // unknown lane
      F(M - lane) = F(M - lane) + cM * z;     // unknown M - 1 - lane
      wave_lds_sync();
    }
    for (int p = lane; p < N; p += 64) G[(size_t)q * T + lb + (size_t)p] = (R)F(p);
    wave_lds_sync();   // the next item's staging overwrites f
  }
}

// ------------------------------------------------------------------ C6 faces, partition method
// LAD-C6 interface fluxes along xi (Sec. 3) on bounded lines of 129 to 2049 nodes: the
// n - 1 interior faces form the [1/3, 1, 1/3] system with the two I4 boundary faces on the
// right-hand side (the system k_c6_faces_pcr reduces), solved as k_filter_part solves the
// filter's with a = 1/3: one wave per (line, flux component), the line's node fluxes staged
// in LDS, segments per lane joined by two wave-wide scans.  The faces go back to LDS and
// each node's derivative -J (F_{i+1/2} - F_{i-1/2}) to dQ/dt.  Xi is the first of two or
// three directions here, so the derivative is written, not accumulated, and never forms
// the RK stage (as in k_c6_faces_pcr).
template <typename R, int LM>
__global__ void __launch_bounds__(64 * FPART_WAVES) k_c6_faces_part(const Prob* __restrict__ probs, StateRef ref,
                                                                    int nmax, int mask) {
  extern __shared__ double dyn[];   // per wave: the staged node fluxes [nmax + 4]
  __shared__ double tcp[FPART_LMAX], tinv[FPART_LMAX];
  __shared__ double tu[2][FPART_LMAX], tv[2][FPART_LMAX];   // segment lengths base and base + 1
  __shared__ double tda[64], tGa[64], tGb[64];
  const Prob& P = probs[blockIdx.y];
  if (!c6f_part_use(P, 0, mask) || P.n[0] > nmax) return;
  const int n = P.n[0], g = P.g[0], M = n - 1;
  const int nseg = min(64, M / 2);
  const int base = M / nseg, extra = M % nseg;   // the first `extra` segments have base + 1
  if (base + 1 > LM) return;   // segments longer than the register arrays
  const double al = C6_ALPHA;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // segment factors, the responses u = T^{-1} e_1 and v = T^{-1} e_L, and the
  // data-independent elimination factors of the joint unknowns (as in k_filter_part)
  if (threadIdx.x == 0) {
    double c = 0.0;
    for (int i = 0; i < base + 1; ++i) {
      const double den = 1.0 - (i > 0 ? al * c : 0.0);
      tinv[i] = 1.0 / den;
      c = al / den;
      tcp[i] = c;
    }
  }
  __syncthreads();
  if (threadIdx.x < 4) {   // threads 0 / 1: u for base / base + 1; 2 / 3: v
    const int which = threadIdx.x & 1, L = base + which;
    const bool is_u = threadIdx.x < 2;
    double* out = is_u ? tu[which] : tv[which];
    double prev = 0.0;
    for (int i = 0; i < L; ++i) {
      const double rhs = is_u ? (i == 0 ? 1.0 : 0.0) : (i == L - 1 ? 1.0 : 0.0);
      prev = (rhs - (i > 0 ? al * prev : 0.0)) * tinv[i];
      out[i] = prev;
    }
    double y = out[L - 1];
    for (int i = L - 2; i >= 0; --i) {
      y = out[i] - tcp[i] * y;
      out[i] = y;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double Gbp = 0.0;
    for (int sg = 0; sg < nseg; ++sg) {
      const int lw = sg < extra ? 1 : 0, Ls = base + lw;
      const double da = 1.0 - al * tu[lw][0] * Gbp;
      const double Ga = al * tv[lw][0] / da;
      tda[sg] = da;
      tGa[sg] = Ga;
      tGb[sg] = al * tv[lw][Ls - 1] + al * tu[lw][Ls - 1] * Gbp * Ga;
      Gbp = tGb[sg];
    }
  }
  __syncthreads();
  double* f = dyn + (size_t)w * fpart_lds_slots(nmax);
  auto F = [f](int p) -> double& { return f[p + (p >> 4)]; };   // p = node position + 2
  const int nlines = interior_lines(P, 0);
  const size_t T = P.total;
  const R* FL = static_cast<const R*>(P.FL[0]);
  double* dQ = ref.deriv(P);
  const bool act = lane < nseg;
  const int L = base + (lane < extra ? 1 : 0);
  const int j0 = lane * base + min(lane, extra);   // first face of this lane's segment
  const int wl = lane < extra ? 1 : 0;             // which u / v table
  const double u1 = act ? tu[wl][0] : 0.0, uL = act ? tu[wl][L - 1] : 0.0;
  const double da = act ? tda[lane] : 1.0, Ga = act ? tGa[lane] : 0.0, Gb = act ? tGb[lane] : 0.0;
  const double Gbm = act && lane > 0 ? tGb[lane - 1] : 0.0;
  for (int item = blockIdx.x * nw + w; item < 5 * nlines; item += gridDim.x * nw) {
    const int line = item / 5, q = item % 5;
    const size_t lb = interior_line_base(P, 0, line);
    const R* Fq = FL + (size_t)q * T + lb;
    for (int p = lane; p < n + 4; p += 64) F(p) = (double)Fq[g - 2 + p];
    wave_lds_sync();
    // boundary faces (I4 of the node fluxes)
    const double lo = (7.0 * (F(1) + F(2)) - (F(0) + F(3))) / 12.0;
    const double hi = (7.0 * (F(n + 1) + F(n + 2)) - (F(n) + F(n + 3))) / 12.0;
    double y[LM];
    double ya = 0.0, yb = 0.0;
    if (act) {
      // face k between nodes k and k + 1: C6 interpolation of the nodes k - 1 .. k + 2
      double fm1 = F(j0 + 1), f0 = F(j0 + 2), f1 = F(j0 + 3);
      double prev = 0.0;
#pragma unroll
      for (int i = 0; i < LM; ++i) {
        if (i < L) {
          const int k = j0 + i;
          const double f2 = F(k + 4);
          double r = C6F_A * (f0 + f1) + C6F_B * (fm1 + f2);
          if (k == 0) r = r - al * lo;
          if (k == M - 1) r = r - al * hi;
          prev = (r - (i > 0 ? al * prev : 0.0)) * tinv[i];
          y[i] = prev;
          fm1 = f0;
          f0 = f1;
          f1 = f2;
        }
      }
      yb = prev;
      double v = prev;
#pragma unroll
      for (int i = LM - 2; i >= 0; --i) {
        if (i < L - 1) {
          v = y[i] - tcp[i] * v;
          y[i] = v;
        }
      }
      ya = y[0];
    }
    const double gbv = scan_up(act ? -al * uL / da : 0.0, act ? yb + al * uL * Gbm * ya / da : 0.0, lane);
    double gbm = __shfl_up(gbv, 1);
    if (lane == 0) gbm = 0.0;
    const double gav = act ? (ya - al * u1 * gbm) / da : 0.0;
    const double A = scan_down(act ? -Ga : 0.0, gav, lane);
    double Ap = __shfl_down(A, 1);
    if (lane + 1 >= nseg) Ap = 0.0;
    const double B = gbv - Gb * Ap;
    double Bm = __shfl_up(B, 1);
    if (lane == 0) Bm = 0.0;
    wave_lds_sync();   // every lane has read its window before the faces overwrite it
    if (act) {
#pragma unroll
      for (int i = 0; i < LM; ++i)
        if (i < L) F(j0 + i) = y[i] - al * tu[wl][i] * Bm - al * tv[wl][i] * Ap;   // face j0 + i
    }
    wave_lds_sync();
    for (int i = lane; i < n; i += 64) {
      const double fp = i < M ? F(i) : hi;
      const double fm = i > 0 ? F(i - 1) : lo;
      const size_t idx = lb + (size_t)(g + i);
      dQ[(size_t)q * T + idx] = -met64(P, 9, (int)idx) * (fp - fm);
    }
    wave_lds_sync();   // the next item's staging overwrites f
  }
}

// ------------------------------------------------------------------ line tiles
// One workgroup holds all five variables of TX neighbouring lines of one direction in LDS
// (TX * 5 * positions <= TILE_ELEMS doubles), forms the right-hand sides there, reduces
// them by PCR and writes the outputs: no FP64 scratch round trip, and many workgroups in
// flight whatever the direction.  Neighbouring lines are adjacent along the contiguous
// other direction (x for eta / zeta lines), so a tile reads and writes TX consecutive
// values per line position; tiles of neighbouring columns run on the same XCD (L2).
//   TK_GRAD6   C6 gradients: FP64 primitives of all nodes in, G out
//   TK_FACES   C6 interface fluxes: node fluxes at -2 .. n+1 in, -J D into dQ/dt (or the
//              RK stage in the last direction)
//   TK_FILTER  implicit filter: the state in, its interior filtered in place
//   TK_GRAD4   C4 gradients (MIG4 of C-GBR): as TK_GRAD6 with the C4 rows and tables
// Division by a per-workgroup constant d >= 1 for dividends e with e * d < 2^32 (tile
// indices: both below 6144): q = hi32(e * ceil(2^32 / d)) is exact there (d = 1 apart,
// whose multiplier does not fit 32 bits).
struct SmallDiv {
  unsigned m;
  int d;
  __device__ explicit SmallDiv(int dv) : m(dv > 1 ? 0xFFFFFFFFu / (unsigned)dv + 1u : 0u), d(dv) {}
  __device__ __forceinline__ int div(int e) const { return d > 1 ? (int)__umulhi((unsigned)e, m) : e; }
};

struct TileArgs {
  StateRef ref;
  RKRef rr;
  int d, TX, accumulate, rk, stage, mask, skip_if_any;
  double a, b;
  int keep_ft;   // filter of a per-cell hybrid stage: nodes in the dilated troubled set keep their values
  int dense_only;   // MIG4 gradients of a per-cell stage: only when most lines are listed (dense_lines)
};

// the LDS index of (variable q, column c, position p) is (q * TX + c) * Lin + p
__device__ __forceinline__ void tile_geom(const Prob& P, int d, int kind, int& Lin, int& off, int& U, int& la,
                                          int& lb, int& ba, int& bb) {
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const bool periodic = P.bc[d][0] == BC_PERIODIC;
  const int n = P.n[d], g = P.g[d];
  if (kind == TK_GRAD6 || kind == TK_GRAD4) {
    Lin = P.N[d];
    off = -g;
    U = periodic ? n : P.N[d];
    la = P.N[o1];
    lb = P.N[o2];
    ba = bb = 0;
  } else {
    Lin = kind == TK_FACES ? n + 4 : P.N[d];
    off = kind == TK_FACES ? -2 : -g;
    U = kind == TK_FACES ? (periodic ? n : n - 1) : n;
    la = P.n[o1];
    lb = P.n[o2];
    ba = P.g[o1];
    bb = P.g[o2];
  }
}

template <typename R, int KIND, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT >= 512 ? 4 : 1)))
k_line_tiles(const Prob* __restrict__ probs, TileArgs A) {
  constexpr int PT = TILE_ELEMS / NT;   // slots per lane
  __shared__ double buf[TILE_ELEMS];
  __shared__ double lohi[2 * 5 * TILE_MAX_TX];
  const Prob& P = probs[blockIdx.y];
  const int d = A.d, TX = A.TX;
  if (d >= P.ndim || !tile_use(P, d, KIND, A.mask)) return;
  if (KIND == TK_FILTER && filt_part_use(P, d, A.mask)) return;   // partition-method kernel
  if (gate_skip(P, A.skip_if_any)) return;
  if (A.dense_only && !dense_lines(P, d)) return;
  int Lin, off, U, la, lb, ba, bb;
  tile_geom(P, d, KIND, Lin, off, U, la, lb, ba, bb);
  if (5 * TX * Lin > TILE_ELEMS || TX > TILE_MAX_TX) return;   // the host sizes TX so that this never holds
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const int ta = (la + TX - 1) / TX;
  const SmallDiv dLin(Lin), dTX(TX), dU(U), dn(P.n[d]);
  const int ntiles = ta * lb;
  const int per = (ntiles + 7) >> 3;
  if ((int)(blockIdx.x >> 3) >= per) return;
  const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (tile >= ntiles) return;
  const int a0 = (tile % ta) * TX, bpos = tile / ta;
  const int ncol = min(TX, la - a0);
  const int g = P.g[d], n = P.n[d], sd = P.s[d];
  const bool periodic = P.bc[d][0] == BC_PERIODIC;
  const size_t T = P.total;
  const size_t lbase = (size_t)(ba + a0) * P.s[o1] + (size_t)(bb + bpos) * P.s[o2];
  const int tid = threadIdx.x;
  const int ncp = TX * Lin;   // (column, position) pairs
  // element e of a (column, position) sweep: positions fastest on contiguous lines,
  // columns fastest on strided ones (coalesced either way)
  auto cp_of = [d, dLin, dTX](int e, int& c, int& p) {
    // both quotients, then a choice of values (a choice of destinations keeps c and p in
    // memory)
    const int qa = dLin.div(e), qb = dTX.div(e);
    c = d == 0 ? qa : e - qb * dTX.d;
    p = d == 0 ? e - qa * dLin.d : qb;
  };
  // ---- load
  for (int e = tid; e < ncp; e += NT) {
    int c, p;
    cp_of(e, c, p);
    double v[5] = {0, 0, 0, 0, 0};
    if (c < ncol) {
      const size_t node = lbase + (size_t)c * P.s[o1] + (size_t)(g + off + p) * sd;
      if (KIND == TK_GRAD6 || KIND == TK_GRAD4) {
        prims5c(A.ref.state(P), T, node, P.gamma - 1.0, v);
      } else if (KIND == TK_FACES) {
        const R* F = static_cast<const R*>(P.FL[d]);
        for (int q = 0; q < 5; ++q) v[q] = (double)F[q * T + node];
      } else {
        const double* Q = A.ref.state(P);
        for (int q = 0; q < 5; ++q) v[q] = Q[q * T + node];
      }
    }
    for (int q = 0; q < 5; ++q) buf[(q * TX + c) * Lin + p] = v[q];
  }
  __syncthreads();
  // ---- right-hand sides (registers, then over the inputs)
  const int nel = 5 * TX * Lin;
  double nv[PT];
#pragma unroll
  for (int m = 0; m < PT; ++m) {
    const int e = tid + m * NT;
    nv[m] = 0.0;
    if (e < nel) {
      int line, k;
      line = dLin.div(e);
      k = e - line * dLin.d;
      const double* f = buf + line * Lin;
      if (k < U) {
        double r;
        if (KIND == TK_GRAD4) {
          if (periodic)
            r = 0.75 * (f[g + wrap(k + 1, n)] - f[g + wrap(k - 1, n)]);
          else if (k == 0)
            r = (-3.0 * f[0] + 4.0 * f[1] - f[2]) / 2.0;
          else if (k == U - 1)
            r = (3.0 * f[U - 1] - 4.0 * f[U - 2] + f[U - 3]) / 2.0;
          else
            r = 0.75 * (f[k + 1] - f[k - 1]);
        } else if (KIND == TK_GRAD6) {
          if (periodic)
            r = C6_A * (f[g + wrap(k + 1, n)] - f[g + wrap(k - 1, n)]) +
                C6_B * (f[g + wrap(k + 2, n)] - f[g + wrap(k - 2, n)]);
          else
            r = c6_grad_rhs(k, U, k >= 2 ? f[k - 2] : 0.0, k >= 1 ? f[k - 1] : 0.0, f[k], k + 1 < U ? f[k + 1] : 0.0,
                            k + 2 < U ? f[k + 2] : 0.0);
        } else if (KIND == TK_FACES) {
          // node position p sits at f[p + 2]
          if (periodic) {
            r = C6F_A * (f[2 + k] + f[2 + wrap(k + 1, n)]) + C6F_B * (f[2 + wrap(k - 1, n)] + f[2 + wrap(k + 2, n)]);
          } else {
            r = C6F_A * (f[2 + k] + f[3 + k]) + C6F_B * (f[1 + k] + f[4 + k]);
            if (k == 0 || k == U - 1) {
              const double lo = (7.0 * (f[1] + f[2]) - (f[0] + f[3])) / 12.0;
              const double hi = (7.0 * (f[n + 1] + f[n + 2]) - (f[n] + f[n + 3])) / 12.0;
              if (k == 0) {
                r = r - C6_ALPHA * lo;
                lohi[2 * line] = lo;
              }
              if (k == U - 1) {
                r = r - C6_ALPHA * hi;
                lohi[2 * line + 1] = hi;
              }
            }
          }
        } else {
          double w[11];
          for (int j = -5; j <= 5; ++j) w[j + 5] = f[g + (periodic ? wrap(k + j, n) : k + j)];
          r = filt_rhs(P, w);
          if (!periodic) {
            if (k == 0) r = r - P.falpha * f[g - 1];
            if (k == n - 1) r = r - P.falpha * f[g + n];
          }
        }
        nv[m] = r;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < PT; ++m) {
    const int e = tid + m * NT;
    if (e < nel) buf[e] = nv[m];
  }
  __syncthreads();
  // ---- PCR over all 5 TX lines at once.  Each slot keeps its row (its line starts at
  // its LDS index minus the row); the factors of rows inside a step's band are two constants (see the table header), so only
  // rows near the line ends read the table.
  const double* tab =
      KIND == TK_GRAD4 ? P.pcr[d] : (KIND == TK_GRAD6 ? P.pcr6[d] : (KIND == TK_FACES ? P.pcrc[d] : P.pcrf[d]));
  const int steps = KIND == TK_FILTER ? P.fsteps : LG_PCR_STEPS;
  const double* hdr = tab + (size_t)(2 * steps + 1) * U;
  int erow[PT];
#pragma unroll
  for (int m = 0; m < PT; ++m) {
    const int e = tid + m * NT;
    const int k = e - dLin.div(e) * Lin;
    erow[m] = (e < nel && k < U) ? k : -1;
  }
  for (int st = 0; st < steps; ++st) {
    const int s = 1 << st;
    const double* k1 = tab + (size_t)st * U;
    const double* k2 = tab + (size_t)(steps + st) * U;
    const double c1 = hdr[4 * st], c2 = hdr[4 * st + 1];
    const int blo = (int)hdr[4 * st + 2], bhi = (int)hdr[4 * st + 3];
#pragma unroll
    for (int m = 0; m < PT; ++m) {
      const int k = erow[m];
      if (k >= 0) {
        const double* r = buf + (tid + m * NT - k);
        int km = k - s, kp = k + s;
        double rm, rp;
        if (periodic) {
          km = km < 0 ? km + U : km;
          kp = kp >= U ? kp - U : kp;
          rm = r[km];
          rp = r[kp];
        } else {
          rm = km >= 0 ? r[km] : 0.0;
          rp = kp < U ? r[kp] : 0.0;
        }
        double f1 = c1, f2 = c2;
        if (k < blo || k > bhi) {
          f1 = k1[k];
          f2 = k2[k];
        }
        nv[m] = r[k] - f1 * rm - f2 * rp;
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < PT; ++m)
      if (erow[m] >= 0) buf[tid + m * NT] = nv[m];
    __syncthreads();
  }
  {
    const double* binv = tab + (size_t)2 * steps * U;
    const double cb = hdr[4 * steps];
    const int blo = (int)hdr[4 * steps + 2], bhi = (int)hdr[4 * steps + 3];
#pragma unroll
    for (int m = 0; m < PT; ++m) {
      const int k = erow[m];
      if (k >= 0) buf[tid + m * NT] *= (k < blo || k > bhi) ? binv[k] : cb;
    }
  }
  __syncthreads();
  // ---- outputs
  if (KIND == TK_GRAD6 || KIND == TK_GRAD4) {
    R* G = static_cast<R*>(P.G[d]);
    const int pos0 = periodic ? g : 0;   // position of unknown 0
    for (int e = tid; e < TX * U; e += NT) {
      int c, k;
      const int qa = dU.div(e), qb = dTX.div(e);
      c = d == 0 ? qa : e - qb * dTX.d;
      k = d == 0 ? e - qa * dU.d : qb;
      if (c >= ncol) continue;
      const size_t col = lbase + (size_t)c * P.s[o1];
      for (int q = 0; q < 5; ++q) {
        const R y = (R)buf[(q * TX + c) * Lin + k];
        G[q * T + col + (size_t)(pos0 + k) * sd] = y;
        if (periodic) {
          if (k >= n - g) G[q * T + col + (size_t)(g + k - n) * sd] = y;   // low ghosts
          if (k < g) G[q * T + col + (size_t)(g + k + n) * sd] = y;        // high ghosts
        }
      }
    }
  } else if (KIND == TK_FACES) {
    double* dQ = A.ref.deriv(P);
    FaceOut o{A.ref, A.rr, A.accumulate, A.rk, A.stage, A.a, A.b};
    const double dt = A.rk ? *P.dt : 0.0;
    int bad = 0;
    for (int e = tid; e < TX * n; e += NT) {
      int c, i;
      const int qa = dn.div(e), qb = dTX.div(e);
      c = d == 0 ? qa : e - qb * dTX.d;
      i = d == 0 ? e - qa * dn.d : qb;
      if (c >= ncol) continue;
      double D[5];
      for (int q = 0; q < 5; ++q) {
        const int line = q * TX + c;
        const double* r = buf + line * Lin;
        double fp, fm;
        if (periodic) {
          fp = r[i];
          fm = r[wrap(i - 1, n)];
        } else {
          fp = i < U ? r[i] : lohi[2 * line + 1];
          fm = i > 0 ? r[i - 1] : lohi[2 * line];
        }
        D[q] = fp - fm;
      }
      if (face_emit(P, o, dQ, dt, lbase + (size_t)c * P.s[o1] + (size_t)(g + i) * sd, D)) ++bad;
    }
    add_bad(P, bad);
  } else {
    double* Q = A.ref.state(P);
    for (int e = tid; e < TX * n; e += NT) {
      int c, k;
      const int qa = dn.div(e), qb = dTX.div(e);
      c = d == 0 ? qa : e - qb * dTX.d;
      k = d == 0 ? e - qa * dn.d : qb;
      if (c >= ncol) continue;
      const size_t node = lbase + (size_t)c * P.s[o1] + (size_t)(g + k) * sd;
      if (filt_keep(P, A.keep_ft, node)) continue;
      for (int q = 0; q < 5; ++q) Q[q * T + node] = buf[(q * TX + c) * Lin + k];
    }
  }
}

// columns per tile so that 5 TX positions fit the LDS tile
static inline int tile_tx(long long Lmax) {
  long long tx = TILE_ELEMS / (5 * std::max<long long>(Lmax, 1));
  return (int)std::max<long long>(1, std::min<long long>(tx, TILE_MAX_TX));
}

template <typename R, int KIND>
static void launch_tiles(const Launch& L, int kc, long long Lmax, long long lines_a, long long lines_b, TileArgs A) {
  A.TX = tile_tx(Lmax);
  if (L.tile_lines > 0) A.TX = std::min(A.TX, L.tile_lines);
  const long long nt = ((lines_a + A.TX - 1) / A.TX) * lines_b;
  const unsigned grid = (unsigned)(8 * ((nt + 7) / 8));
  if (A.d == 0 || A.TX >= 8)
    LG_TIMED(L, kc, hipLaunchKernelGGL((k_line_tiles<R, KIND, TILE_THREADS_CONTIG>), dim3(grid, L.nprob),
                                       dim3(TILE_THREADS_CONTIG), 0, L.stream, L.probs, A));
  else
    LG_TIMED(L, kc, hipLaunchKernelGGL((k_line_tiles<R, KIND, TILE_THREADS_STRIDED>), dim3(grid, L.nprob),
                                       dim3(TILE_THREADS_STRIDED), 0, L.stream, L.probs, A));
}

// ------------------------------------------------------------------ launches
static inline unsigned blocks_for(long long work) { return (unsigned)std::max<long long>(1, (work + 255) / 256); }

static inline unsigned pcr_grid(const Launch& L, long long items) {
  return (unsigned)std::max<long long>(1, std::min<long long>(items, L.pcr_blocks > 0 ? L.pcr_blocks : 16384));
}

// which kernels a system's direction takes: LDS tiles when enabled (for the problems that
// fit them), the fallback kernels for the others (or for all when tiles are off)
struct SysLaunch {
  int tiles, pcr, thomas;
};
static inline SysLaunch sys_launch(const Launch& L, int kind, int d) {
  return SysLaunch{L.ctile[kind][d], L.cpcr[kind][d], L.cthomas[kind][d]};
}

template <typename R, bool C6>
static void launch_grad_part(const Launch& L, StateRef ref, int skip_if_any, int dense_only);

template <typename R>
void launch_grad_c6(const Launch& L, StateRef ref, int d) {
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const SysLaunch sl = sys_launch(L, TK_GRAD6, d);
  if (d == 0 && L.c6gpart) launch_grad_part<R, true>(L, ref, -1, 0);
  if (d > 0 && L.c6gseg[d] > 0) {   // periodic lines in register segments: 64 lines x one primitive per workgroup
    const long long groups = (L.lines[d] + 63) / 64;
    LG_TIMED(L, KC_GRAD_C4, hipLaunchKernelGGL((k_grad_c4_seg<R, FSEG_LM, true>), dim3((unsigned)(5 * groups), L.nprob),
                                               dim3(64 * L.c6gseg[d]), 0, L.stream, L.probs, ref, d, -1, 0,
                                               L.tile_mask));
  }
  if (sl.tiles)
    launch_tiles<R, TK_GRAD6>(L, KC_GRAD_C4, L.max_N[d], L.max_N[o1], L.max_N[o2],
                              TileArgs{ref, RKRef{nullptr, nullptr, nullptr}, d, 1, 0, 0, 0, L.tile_mask, -1, 0.0, 0.0, 0});
  if (sl.pcr) {
    const unsigned lds = (unsigned)(2 * std::min<long long>(L.max_N[d], 4096) * sizeof(double));
    LG_TIMED(L, KC_GRAD_C4, hipLaunchKernelGGL(k_grad_c6_pcr<R>, dim3(pcr_grid(L, 5 * L.lines[d]), L.nprob),
                                               dim3(CPCR_THREADS), lds, L.stream, L.probs, ref, d, L.tile_mask));
  }
  if (sl.thomas)   // five waves per 64 lines, one primitive each
    LG_TIMED(L, KC_GRAD_C4, hipLaunchKernelGGL((k_grad_c6<R, 1>), dim3((unsigned)((L.lines[d] + 63) / 64), L.nprob),
                                               dim3(320), 0, L.stream, L.probs, ref, d, L.tile_mask));
}

template <typename R>
void launch_c6_faces(const Launch& L, StateRef ref, int d, int accumulate, const RKRef* rr, int stage, double a,
                     double b) {
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const SysLaunch sl = sys_launch(L, TK_FACES, d);
  if (d == 0 && L.c6fpart && !accumulate && !rr) {
    // one wave per (line, component), as the C4 partition kernel
    const long long nmax = L.max_n[0];
    const size_t per_wave = (size_t)fpart_lds_slots((int)nmax) * sizeof(double);
    const int nw = 4 * per_wave <= 60 * 1024 ? 4 : 2;
    const long long items = 5 * L.sweep_rows[0];
    const unsigned blocks = (unsigned)std::max<long long>(1, std::min<long long>((items + nw - 1) / nw, 4096));
    if ((nmax - 1) / 64 + 1 <= FPART_LSHORT)
      LG_TIMED(L, KC_C6_FACES, hipLaunchKernelGGL((k_c6_faces_part<R, FPART_LSHORT>), dim3(blocks, L.nprob),
                                                  dim3(64 * nw), nw * per_wave, L.stream, L.probs, ref, (int)nmax,
                                                  L.tile_mask));
    else
      LG_TIMED(L, KC_C6_FACES, hipLaunchKernelGGL((k_c6_faces_part<R, FPART_LMAX>), dim3(blocks, L.nprob),
                                                  dim3(64 * nw), nw * per_wave, L.stream, L.probs, ref, (int)nmax,
                                                  L.tile_mask));
  }
  if (d > 0 && L.c6fseg[d] > 0) {
    // 64 lines x one component per workgroup, one wave per segment; where this is the last
    // direction of an RK stage, the combination in the same pass and the non-physical count
    // in its own
    const long long groups = (L.sweep_rows[d] + 63) / 64;
    const dim3 grid((unsigned)(5 * groups), L.nprob), block(64 * L.c6fseg[d]);
    if (rr)
      LG_TIMED(L, KC_C6_FACES, hipLaunchKernelGGL((k_c6_faces_seg<R, FSEG_LM, true>), grid, block, 0, L.stream,
                                                  L.probs, ref, d, accumulate, L.tile_mask, *rr, stage, a, b));
    else
      LG_TIMED(L, KC_C6_FACES, hipLaunchKernelGGL((k_c6_faces_seg<R, FSEG_LM, false>), grid, block, 0, L.stream,
                                                  L.probs, ref, d, accumulate, L.tile_mask,
                                                  RKRef{nullptr, nullptr, nullptr}, stage, a, b));
    if (rr)
      LG_TIMED(L, KC_COMBINE, hipLaunchKernelGGL(k_c6_seg_check,
                                                 dim3((unsigned)std::min<long long>(L.sweep_rows[0], 1 << 16), L.nprob),
                                                 dim3(256), 0, L.stream, L.probs, *rr, stage, L.tile_mask));
  }
  if (sl.tiles)
    launch_tiles<R, TK_FACES>(L, KC_C6_FACES, L.max_n[d] + 4, L.max_n[o1], L.max_n[o2],
                              TileArgs{ref, rr ? *rr : RKRef{nullptr, nullptr, nullptr}, d, 1, accumulate, rr ? 1 : 0,
                                       stage, L.tile_mask, -1, a, b, 0});
  if (sl.pcr) {
    const unsigned lds = (unsigned)((2 * std::min<long long>(L.max_n[d], 3990) + 4) * sizeof(double));
    LG_TIMED(L, KC_C6_FACES, hipLaunchKernelGGL(k_c6_faces_pcr<R>, dim3(pcr_grid(L, 5 * L.sweep_rows[d]), L.nprob),
                                                dim3(CPCR_THREADS), lds, L.stream, L.probs, ref, d, L.tile_mask));
  }
  if (sl.thomas) {
    FaceOut o{ref, rr ? *rr : RKRef{nullptr, nullptr, nullptr}, accumulate, rr ? 1 : 0, stage, a, b};
    if (rr)   // the RK stage needs the five components of a node together
      LG_TIMED(L, KC_C6_FACES, hipLaunchKernelGGL((k_c6_faces<R, 5>), dim3(blocks_for(L.sweep_rows[d]), L.nprob),
                                                  dim3(256), 0, L.stream, L.probs, o, d, L.tile_mask));
    else
      LG_TIMED(L, KC_C6_FACES, hipLaunchKernelGGL((k_c6_faces<R, 1>), dim3(blocks_for(5 * L.sweep_rows[d]), L.nprob),
                                                  dim3(256), 0, L.stream, L.probs, o, d, L.tile_mask));
  }
}

void launch_filter_save(const Launch& L, StateRef ref, int mode) {
  const long long work = 5LL * L.max_total;
  LG_TIMED(L, KC_FILTER_GUARD, hipLaunchKernelGGL(k_filter_save, dim3(blocks_for(std::min(work, 1LL << 24)), L.nprob),
                                                  dim3(256), 0, L.stream, L.probs, ref, mode));
}

void launch_filter_guard(const Launch& L, StateRef ref, int mode) {
  LG_TIMED(L, KC_FILTER_GUARD, hipLaunchKernelGGL(k_filter_guard, dim3(blocks_for(std::min(L.max_total, 1LL << 22)),
                                                  L.nprob), dim3(256), 0, L.stream, L.probs, ref, mode));
}

void launch_filter(const Launch& L, StateRef ref, int d, int mode) {
  launch_bc_cons(L, ref, d);
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  if (d == 0 && L.fpart) {
    // one wave per (line, variable); four waves per workgroup while their staged lines fit
    // 60 KB of LDS, two otherwise (lines of up to 2048 unknowns)
    const long long nmax = L.max_n[0];
    const size_t per_wave = (size_t)fpart_lds_slots((int)nmax) * sizeof(double);
    const int nw = 4 * per_wave <= 60 * 1024 ? 4 : 2;
    const long long items = 5 * L.sweep_rows[0];
    const unsigned blocks = (unsigned)std::max<long long>(1, std::min<long long>((items + nw - 1) / nw, 4096));
    // register arrays sized to the longest segment: short ones when every line has at most
    // 1088 unknowns (segments of at most 17)
    if (nmax <= 64 * (FPART_LSHORT - 1))
      LG_TIMED(L, KC_FILTER, hipLaunchKernelGGL(k_filter_part<FPART_LSHORT>, dim3(blocks, L.nprob), dim3(64 * nw),
                                                nw * per_wave, L.stream, L.probs, ref, mode, (int)nmax, L.tile_mask));
    else
      LG_TIMED(L, KC_FILTER, hipLaunchKernelGGL(k_filter_part<FPART_LMAX>, dim3(blocks, L.nprob), dim3(64 * nw),
                                                nw * per_wave, L.stream, L.probs, ref, mode, (int)nmax, L.tile_mask));
  }
  if (L.fseg[d] > 0) {
    // 64 lines x one variable per workgroup, one wave per segment
    const long long groups = (L.sweep_rows[d] + 63) / 64;
    LG_TIMED(L, KC_FILTER, hipLaunchKernelGGL(k_filter_seg<FSEG_LM>, dim3((unsigned)(5 * groups), L.nprob),
                                              dim3(64 * L.fseg[d]), 0, L.stream, L.probs, ref, d, L.tile_mask, mode));
  }
  const SysLaunch sl = sys_launch(L, TK_FILTER, d);
  if (sl.tiles)
    launch_tiles<double, TK_FILTER>(L, KC_FILTER, L.max_N[d], L.max_n[o1], L.max_n[o2],
                                    TileArgs{ref, RKRef{nullptr, nullptr, nullptr}, d, 1, 0, 0, 0, L.tile_mask,
                                             mode == FILT_GLOBAL ? 1 : -1, 0.0, 0.0, mode});
  if (sl.pcr) {
    const unsigned lds = (unsigned)(std::min<long long>(L.max_N[d] + L.max_n[d], 7990) * sizeof(double));
    LG_TIMED(L, KC_FILTER, hipLaunchKernelGGL(k_filter_pcr, dim3(pcr_grid(L, 5 * L.sweep_rows[d]), L.nprob),
                                              dim3(CPCR_THREADS), lds, L.stream, L.probs, ref, d, L.tile_mask, mode));
  }
  if (sl.thomas)
    LG_TIMED(L, KC_FILTER, hipLaunchKernelGGL(k_filter, dim3(blocks_for(5 * L.sweep_rows[d]), L.nprob), dim3(256), 0,
                                              L.stream, L.probs, ref, d, L.tile_mask, mode));
}

template <typename R>
void launch_grad_c4_tiles(const Launch& L, StateRef ref, int d, int skip_if_any, int dense_only) {
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  if (L.ctile[TK_GRAD4][d])
    launch_tiles<R, TK_GRAD4>(L, KC_GRAD_C4, L.max_N[d], L.max_N[o1], L.max_N[o2],
                              TileArgs{ref, RKRef{nullptr, nullptr, nullptr}, d, 1, 0, 0, 0, L.tile_mask, skip_if_any,
                                       0.0, 0.0, 0, dense_only});
}

template <typename R, bool C6>
static void launch_grad_part(const Launch& L, StateRef ref, int skip_if_any, int dense_only) {
  // one wave per (line, primitive); four waves per workgroup while their staged lines fit
  // 60 KB of LDS, two otherwise
  const long long nmax = L.max_n[0];
  const size_t per_wave = (size_t)fpart_lds_slots((int)nmax) * sizeof(double);
  const int nw = 4 * per_wave <= 60 * 1024 ? 4 : 2;
  const long long items = 5 * L.lines[0];
  const unsigned blocks = (unsigned)std::max<long long>(1, std::min<long long>((items + nw - 1) / nw, 4096));
  // register arrays sized to the longest segment: short ones when every line has fewer
  // than 64 * 17 unknowns (the n + 8 between its end rows; segments of at most 17)
  if ((nmax + 8) / 64 + 1 <= FPART_LSHORT)
    LG_TIMED(L, KC_GRAD_C4, hipLaunchKernelGGL((k_grad_part<R, FPART_LSHORT, C6>), dim3(blocks, L.nprob),
                                               dim3(64 * nw), nw * per_wave, L.stream, L.probs, ref, (int)nmax,
                                               skip_if_any, dense_only, L.tile_mask));
  else
    LG_TIMED(L, KC_GRAD_C4, hipLaunchKernelGGL((k_grad_part<R, FPART_LMAX, C6>), dim3(blocks, L.nprob),
                                               dim3(64 * nw), nw * per_wave, L.stream, L.probs, ref, (int)nmax,
                                               skip_if_any, dense_only, L.tile_mask));
}

template <typename R>
void launch_grad_c4_part(const Launch& L, StateRef ref, int skip_if_any, int dense_only) {
  if (L.c4part) launch_grad_part<R, false>(L, ref, skip_if_any, dense_only);
}

template void launch_grad_c4_tiles<float>(const Launch&, StateRef, int, int, int);
template void launch_grad_c4_tiles<double>(const Launch&, StateRef, int, int, int);
template <typename R>
void launch_grad_c4_seg(const Launch& L, StateRef ref, int d, int skip_if_any, int dense_only) {
  if (L.c4seg[d] <= 0) return;
  // 64 lines x one primitive per workgroup, one wave per segment
  const long long groups = (L.lines[d] + 63) / 64;
  LG_TIMED(L, KC_GRAD_C4, hipLaunchKernelGGL((k_grad_c4_seg<R, FSEG_LM, false>), dim3((unsigned)(5 * groups), L.nprob),
                                             dim3(64 * L.c4seg[d]), 0, L.stream, L.probs, ref, d, skip_if_any,
                                             dense_only, L.tile_mask));
}

template void launch_grad_c4_part<float>(const Launch&, StateRef, int, int);
template void launch_grad_c4_part<double>(const Launch&, StateRef, int, int);
template void launch_grad_c4_seg<float>(const Launch&, StateRef, int, int, int);
template void launch_grad_c4_seg<double>(const Launch&, StateRef, int, int, int);
template void launch_grad_c6<float>(const Launch&, StateRef, int);
template void launch_grad_c6<double>(const Launch&, StateRef, int);
template void launch_c6_faces<float>(const Launch&, StateRef, int, int, const RKRef*, int, double, double);
template void launch_c6_faces<double>(const Launch&, StateRef, int, int, const RKRef*, int, double, double);

}  // namespace lg
