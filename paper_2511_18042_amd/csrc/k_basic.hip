// Ghost images, primitives, troubled flags, RK3 stage combination, CFL time step,
// flag dilation and grid metrics.
//
// Paper: Sec. 2.1 (primitives, metrics xi_hat = xi_x / J), Alg. 1-2 (SET_BCS,
// SET_PRIMITIVES, NETFLUX_LOOP), Alg. 3 / Sec. 5 (troubled cells: density or pressure
// below a threshold), third-order TVD Runge-Kutta (Sec. 2.1, 2.3), CFL 0.2 (Sec. 3).
#include "lgbr_dev.h"
#include "lgbr_kernels.h"

namespace lg {

// ------------------------------------------------------------------ ghost images
// Ghost layers of direction d: periodic images, zeroth-order copies, or mirrors
// (normal momentum negated at reflective walls, all momentum at no-slip adiabatic
// walls; at no-slip isothermal walls velocity odd, pressure even and temperature odd
// about the wall temperature, density from the equation of state); FIXED ghosts belong
// to the caller.  Ghost layers are filled over the full
// extent of the other two directions, direction by direction, so corners are set.
__device__ __forceinline__ bool ghost_src(int bct, int side, int m, int g, int n, int& dst, int& src) {
  if (bct == BC_FIXED) return false;
  dst = side == 0 ? g - 1 - m : g + n + m;
  if (bct == BC_PERIODIC) src = side == 0 ? dst + n : dst - n;
  else if (bct == BC_TRANSMISSIVE) src = side == 0 ? g : g + n - 1;
  else src = side == 0 ? g + m : g + n - 1 - m;
  return true;
}

__global__ void __launch_bounds__(256) k_bc_cons(const Prob* __restrict__ probs, StateRef ref, int d) {
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim) return;
  double* Q = ref.state(P);
  const int g = P.g[d], n = P.n[d];
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const int N1 = P.N[o1], N2 = P.N[o2];
  const int cnt = 2 * g * N1 * N2;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cnt; t += gridDim.x * blockDim.x) {
    int a = t % N1, r = t / N1;
    int b = r % N2;
    r /= N2;
    int m = r % g, side = r / g;
    int bct = P.bc[d][side];
    int dst, src;
    if (!ghost_src(bct, side, m, g, n, dst, src)) continue;
    int base = a * P.s[o1] + b * P.s[o2];
    size_t id = base + dst * P.s[d], is = base + src * P.s[d];
    const size_t T = P.total;
    if (bct == BC_NOSLIP_T) {
      const double rs = Q[is], u = Q[T + is] / rs, v = Q[2 * T + is] / rs, w = Q[3 * T + is] / rs;
      const double u2 = u * u + v * v + w * w;
      const double ps = (P.gamma - 1.0) * (Q[4 * T + is] - 0.5 * rs * u2);
      const double gM2 = P.gamma * P.Mref * P.Mref;
      const double Tg = 2.0 * P.wall_T[d][side] - gM2 * ps / rs;
      const double rg = gM2 * ps / Tg;
      Q[id] = rg;
      Q[T + id] = -rg * u;
      Q[2 * T + id] = -rg * v;
      Q[3 * T + id] = -rg * w;
      Q[4 * T + id] = ps / (P.gamma - 1.0) + 0.5 * rg * u2;
      continue;
    }
    for (int q = 0; q < 5; ++q) {
      double v = Q[q * T + is];
      if (bct == BC_REFLECTIVE && q == 1 + d) v = -v;
      if (bct == BC_NOSLIP && q >= 1 && q <= 3) v = -v;
      Q[q * T + id] = v;
    }
  }
}

// Scalar intermediate fields: same images with even parity; FIXED -> nearest copy.
template <typename R>
__global__ void __launch_bounds__(256) k_bc_scalar(const Prob* __restrict__ probs, int which, int nf, int d) {
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim) return;
  R* F = static_cast<R*>(which == 0 ? P.CA : P.CB);
  const int g = P.g[d], n = P.n[d];
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const int N1 = P.N[o1], N2 = P.N[o2];
  const int cnt = 2 * g * N1 * N2;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cnt; t += gridDim.x * blockDim.x) {
    int a = t % N1, r = t / N1;
    int b = r % N2;
    r /= N2;
    int m = r % g, side = r / g;
    int bct = P.bc[d][side];
    if (bct == BC_FIXED) bct = BC_TRANSMISSIVE;
    int dst, src;
    ghost_src(bct, side, m, g, n, dst, src);
    int base = a * P.s[o1] + b * P.s[o2];
    size_t id = base + dst * P.s[d], is = base + src * P.s[d];
    for (int q = 0; q < nf; ++q) F[q * (size_t)P.total + id] = F[q * (size_t)P.total + is];
  }
}

// ------------------------------------------------------------------ primitives + flags
// PAIR: each lane converts two neighbouring nodes (2t, 2t + 1) with 16-byte state loads and
// 8-byte (FP32) primitive stores; needs an even node count and 16-byte aligned state
// (checked on the host).  Otherwise one node per lane.
// ghosts: 0 converts every node; 1 the ghost nodes only (the previous stage's all-LAD pass
// wrote the interior primitives and flags with the stage result); 2 the ghost nodes only if
// that pass ran, i.e. the previous stage of the global hybrid found no troubled node (its
// any_flag, not yet reset for this stage), every node otherwise.
__device__ __forceinline__ bool interior_node(const Prob& P, int idx) {
  const int p[3] = {idx % P.N[0], (idx / P.N[0]) % P.N[1], idx / (P.N[0] * P.N[1])};
#pragma unroll
  for (int l = 0; l < 3; ++l)
    if (l < P.ndim && (p[l] < P.g[l] || p[l] >= P.g[l] + P.n[l])) return false;
  return true;
}

template <typename R, bool PAIR>
__global__ void __launch_bounds__(256) k_prim(const Prob* __restrict__ probs, StateRef ref, int want_flags,
                                              const uint8_t* force, int ghosts) {
  const Prob& P = probs[blockIdx.y];
  const double* Q = ref.state(P);
  R* W = static_cast<R*>(P.W);
  const size_t T = P.total;
  const bool skip_in = ghosts == 1 || (ghosts == 2 && *P.any_flag == 0);
  if constexpr (PAIR) {
    using D2 = double __attribute__((ext_vector_type(2)));
    using R2 = R __attribute__((ext_vector_type(2)));
    const int npair = (int)(T / 2);
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < npair; t += gridDim.x * blockDim.x) {
      const size_t idx = 2 * (size_t)t;
      if (skip_in && interior_node(P, (int)idx) && interior_node(P, (int)idx + 1)) continue;
      D2 q[5];
      for (int c = 0; c < 5; ++c) q[c] = *reinterpret_cast<const D2*>(Q + c * T + idx);
      R ra[5], rb[5];
      double pa, pb;
      prim_node<R>(P, q[0].x, q[1].x, q[2].x, q[3].x, q[4].x, ra[0], ra[1], ra[2], ra[3], ra[4], pa);
      prim_node<R>(P, q[0].y, q[1].y, q[2].y, q[3].y, q[4].y, rb[0], rb[1], rb[2], rb[3], rb[4], pb);
      for (int c = 0; c < 5; ++c) {
        R2 o;
        o.x = ra[c];
        o.y = rb[c];
        *reinterpret_cast<R2*>(W + c * T + idx) = o;
      }
      if (want_flags) {
        uint8_t fa, fb;
        if (force) {
          fa = (uint8_t)(force[idx] != 0);
          fb = (uint8_t)(force[idx + 1] != 0);
        } else {
          fa = (uint8_t)troubled(q[0].x, pa, P);
          fb = (uint8_t)troubled(q[0].y, pb, P);
        }
        P.f[idx] = fa;
        P.f[idx + 1] = fb;
      }
    }
  } else {
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < P.total; idx += gridDim.x * blockDim.x) {
      if (skip_in && interior_node(P, idx)) continue;
      double p;
      R r[5];
      prim_node<R>(P, Q[idx], Q[T + idx], Q[2 * T + idx], Q[3 * T + idx], Q[4 * T + idx], r[0], r[1], r[2], r[3],
                   r[4], p);
      for (int c = 0; c < 5; ++c) W[c * T + idx] = r[c];
      if (want_flags) {
        uint8_t f = force ? (uint8_t)(force[idx] != 0) : (uint8_t)troubled(Q[idx], p, P);
        P.f[idx] = f;
      }
    }
  }
}

// ------------------------------------------------------------------ global hybrid switch
__global__ void __launch_bounds__(256) k_any_flag(const Prob* __restrict__ probs, int interior_only, int zc) {
  const Prob& P = probs[blockIdx.y];
  int found = 0;
  if (interior_only) {   // z-marching columns of the interior (launched with zm_grid)
    ZCol c;
    if (zm_column(P, 0, 0, zc, c)) {
      int idx = pos_to_idx(P, c.i, c.j, c.k0);
      for (int k = c.k0; k < c.k1; ++k, idx += P.s[2]) found |= P.f[idx];
    }
  } else {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < P.total; t += gridDim.x * blockDim.x)
      if (P.f[t]) found = 1;
  }
  // one atomic per wave that found a flag, and none once the word is set (many waves find
  // flags in a troubled field; atomics on one address serialise)
  if (__any(found) && (threadIdx.x & 63) == 0 && __atomic_load_n(P.any_flag, __ATOMIC_RELAXED) == 0)
    atomicOr(P.any_flag, 1);
}

// ------------------------------------------------------------------ compacted per-cell hybrid
// After the flag dilation: all_flag starts as any_flag and is cleared by any interior node
// outside the dilated troubled set; the queue counts restart at zero.
__global__ void k_hyb_init(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.y];
  if (threadIdx.x == 0) {
    *P.all_flag = *P.any_flag != 0 ? 1 : 0;
    for (int d = 0; d < 3; ++d) P.gcount[d] = 0;
  }
}

__global__ void __launch_bounds__(256) k_all_flag(const Prob* __restrict__ probs, int zc) {
  const Prob& P = probs[blockIdx.y];
  if (*P.any_flag == 0) return;
  int clear = 0;
  ZCol c;
  if (zm_column(P, 0, 0, zc, c)) {
    int idx = pos_to_idx(P, c.i, c.j, c.k0);
    for (int k = c.k0; k < c.k1; ++k, idx += P.s[2]) clear |= P.ft[idx] == 0;
  }
  if (__any(clear) && (threadIdx.x & 63) == 0 && __atomic_load_n(P.all_flag, __ATOMIC_RELAXED) != 0)
    atomicAnd(P.all_flag, 0);
}

// Work queue of the C-GBR interfaces along d: the interfaces i+1/2 of the interior lines
// (i from -1 to n-1, stored by their left node) with ft_i | ft_{i+1}.  Each workgroup scans
// one chunk of QCHUNK interfaces in node order, collects its entries in LDS (a ballot and a
// prefix count per wave, one LDS atomic per wave) and appends them with a single global
// atomic, so that neighbouring queue entries are mostly neighbouring nodes.  Only when some,
// but not all, interfaces are C-GBR.
constexpr int QCHUNK = 4096;

__global__ void __launch_bounds__(256) k_gbr_queue(const Prob* __restrict__ probs, int d) {
  __shared__ int list[QCHUNK];
  __shared__ int n_loc, base;
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || gate_skip(P, GATE_MIXED)) return;
  int E[3], o[3];
  for (int l = 0; l < 3; ++l) {
    E[l] = P.n[l] + (l == d ? 1 : 0);
    o[l] = P.g[l] - (l == d ? 1 : 0);
  }
  // interface counts stay below the node count, which int node indices already bound
  const int tot = E[0] * E[1] * E[2];
  const int c0 = (int)blockIdx.x * QCHUNK;
  if (c0 >= tot) return;
  const int s = P.s[d];
  const int lane = threadIdx.x & 63;
  if (threadIdx.x == 0) n_loc = 0;
  __syncthreads();
  for (int r = 0; r < QCHUNK; r += 256) {
    const int t = c0 + r + (int)threadIdx.x;
    int idx = 0, flag = 0;
    if (t < tot) {
      const int i = t % E[0] + o[0];
      const int j = (t / E[0]) % E[1] + o[1];
      const int k = t / (E[0] * E[1]) + o[2];
      idx = pos_to_idx(P, i, j, k);
      flag = (P.ft[idx] | P.ft[idx + s]) != 0;
    }
    const unsigned long long m = __ballot(flag);
    const int cnt = __popcll(m);
    int off = 0;
    if (lane == 0 && cnt) off = atomicAdd(&n_loc, cnt);
    off = __shfl(off, 0);
    if (flag) list[off + __popcll(m & ((1ull << lane) - 1ull))] = idx;
  }
  __syncthreads();
  if (threadIdx.x == 0) base = n_loc ? atomicAdd(&P.gcount[d], n_loc) : 0;
  __syncthreads();
  int* q = P.gq + (size_t)d * P.total + base;
  for (int i = threadIdx.x; i < n_loc; i += blockDim.x) q[i] = list[i];
}

// Separable box dilation by r nodes along direction d.
// src/dst: 0 = f, 1 = ftmp, 2 = ft, 3 = fg.
__device__ __forceinline__ uint8_t* flag_buf(const Prob& P, int b) {
  return b == 0 ? P.f : (b == 1 ? P.ftmp : (b == 2 ? P.ft : P.fg));
}

// RR > 0: the radius is RR, and only its window is read; RR = 0: any radius up to 7.
template <int RR>
__global__ void __launch_bounds__(256) k_dilate(const Prob* __restrict__ probs, int d, int src, int dst, int radius) {
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || *P.any_flag == 0) return;   // nothing flagged: consumers check any_flag
  const uint8_t* in = flag_buf(P, src);
  uint8_t* out = flag_buf(P, dst);
  const int r = RR > 0 ? RR : radius, Nd = P.N[d], sd = P.s[d];
  constexpr int RMAX = RR > 0 ? RR : 7;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < P.total; idx += gridDim.x * blockDim.x) {
    const int c = (idx / sd) % Nd;
    uint8_t v[2 * RMAX + 1];
#pragma unroll
    for (int s = -RMAX; s <= RMAX; ++s) {   // independent loads, clamped into the line
      int cc = min(max(c + s, 0), Nd - 1);
      v[s + RMAX] = in[idx + (cc - c) * sd];
    }
    uint8_t acc = 0;
#pragma unroll
    for (int s = -RMAX; s <= RMAX; ++s) {
      int cc = c + s;
      if (s >= -r && s <= r && cc >= 0 && cc < Nd) acc |= v[s + RMAX];
    }
    out[idx] = acc;
  }
}

// Compacted list of the lines along d that cross the C-GBR input region fg (one lane
// per line; wave-aggregated append).
__global__ void __launch_bounds__(256) k_line_list(const Prob* __restrict__ probs, int d) {
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || *P.any_flag == 0) return;
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const int nlines = P.N[o1] * P.N[o2];
  const int line = blockIdx.x * blockDim.x + threadIdx.x;
  bool act = false;
  if (line < nlines) {
    const int a = line % P.N[o1], b = line / P.N[o1];
    const uint8_t* f = P.fg + a * P.s[o1] + b * P.s[o2];
    const int Nd = P.N[d], sd = P.s[d];
    for (int i = 0; i < Nd && !act; ++i) act = f[i * sd] != 0;
  }
  const unsigned long long m = __ballot(act);
  if (m == 0ull) return;
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (lane == __ffsll((long long)m) - 1) base = atomicAdd(&P.lcount[d], __popcll(m));
  base = __shfl(base, __ffsll((long long)m) - 1);
  if (act) P.llist[d][base + __popcll(m & ((1ull << lane) - 1ull))] = line;
}

__global__ void k_zero_lcount(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.y];
  if (threadIdx.x < 3) P.lcount[threadIdx.x] = 0;
}

// ------------------------------------------------------------------ CFL time step
// Spectral radius sum_l (|xi_l . u| + c |xi_l|) with xi_l = J l_hat, max over the
// interior; kept as the bit pattern of a positive double so that an integer max works.
__global__ void __launch_bounds__(256) k_dt_reduce(const Prob* __restrict__ probs, const double* Qx, int zc) {
  const Prob& P = probs[blockIdx.y];
  const double* Q = Qx ? Qx : P.Q;
  const size_t T = P.total;
  double smax = 0.0;
  // z-marching columns: the metrics of a grid planar along zeta are read once per column
  ZCol c;
  if (zm_column(P, 0, 0, zc, c)) {
    const int sz = P.s[2];
    int idx = pos_to_idx(P, c.i, c.j, c.k0);
    const bool mplane = P.met_planar || !P.curvilinear;
    double m[10];
    if (mplane)
      for (int q = 0; q < 10; ++q) m[q] = met64(P, q, idx);
    for (int k = c.k0; k < c.k1; ++k, idx += sz) {
      if (!mplane)
        for (int q = 0; q < 10; ++q) m[q] = met64(P, q, idx);
      double rho = Q[idx], ri = 1.0 / rho;
      double u = Q[T + idx] * ri, v = Q[2 * T + idx] * ri, w = Q[3 * T + idx] * ri;
      double p = (P.gamma - 1.0) * (Q[4 * T + idx] - 0.5 * rho * (u * u + v * v + w * w));
      double cs = sqrt(P.gamma * p * ri);
      double J = m[9];
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < 3; ++l) {   // constant register indices (uniform exit)
        if (l >= P.ndim) break;
        double x0 = J * m[3 * l], x1 = J * m[3 * l + 1], x2 = J * m[3 * l + 2];
        s += fabs(x0 * u + x1 * v + x2 * w) + cs * sqrt(x0 * x0 + x1 * x1 + x2 * x2);
      }
      if (!(s <= smax)) smax = s;  // NaN propagates as "larger"
    }
  }
  // wave, then block reduction; one atomic per block
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_down(smax, off);
    if (!(o <= smax)) smax = o;
  }
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = smax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = part[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      if (!(part[w] <= m)) m = part[w];
    atomicMax(P.smax, (unsigned long long)__double_as_longlong(m));
  }
}

__global__ void k_dt_reset(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.y];
  if (threadIdx.x == 0) *P.smax = 0ull;
}

__global__ void k_dt_finalize(const Prob* __restrict__ probs, double* tx, double t_end, int advance_t) {
  const Prob& P = probs[blockIdx.y];
  if (threadIdx.x != 0) return;
  double smax = __longlong_as_double((long long)*P.smax);
  double dt = P.cfl / smax;
  if (advance_t) {
    double* t = tx ? tx : P.t;
    double te = tx ? t_end : P.t_end;
    double rem = te - *t;
    if (dt > rem) dt = rem;
    if (!(dt > 0.0)) dt = 0.0;
    *t = *t + dt;
  }
  *P.dt = dt;
}

__global__ void k_set_dt(const Prob* __restrict__ probs, double dt) {
  const Prob& P = probs[blockIdx.y];
  if (threadIdx.x == 0) *P.dt = dt;
}

__global__ void k_zero_status(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.y];
  if (threadIdx.x < STATUS_SLOTS) P.status[STATUS_STRIDE * threadIdx.x] = 0;
}

// one hybrid stage done: count it, and whether it had a troubled node (the global switch
// then runs it on C-GBR)
__global__ void k_switch_count(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.y];
  if (threadIdx.x == 0) {
    P.sw[0] += 1u;
    if (*P.any_flag != 0) P.sw[1] += 1u;
  }
}

__global__ void k_zero_any(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.y];
  if (threadIdx.x == 0) *P.any_flag = 0;
}

// ------------------------------------------------------------------ metrics from coordinates
// Conservative node metrics with the fourth-order central difference D4 as the outer
// operator (2D: xi_hat = (y_eta, -x_eta), eta_hat = (-y_xi, x_xi); 3D: xi_hat_x =
// (y_eta z)_zeta - (y_zeta z)_eta and cyclic), J = 1 / det of the D4 coordinate Jacobian.
__device__ __forceinline__ double d4at(const double* f, int idx, int s) {
  return (8.0 * (f[idx + s] - f[idx - s]) - (f[idx + 2 * s] - f[idx - 2 * s])) / 12.0;
}

__global__ void __launch_bounds__(256) k_metric_inner(int ndim, int N0, int N1, int N2, const double* X,
                                                      double* D) {
  // D[3*c + l] = D4_l(coord c) where the stencil fits, 0 elsewhere
  const int total = N0 * N1 * N2;
  const int Ns[3] = {N0, N1, N2}, ss[3] = {1, N0, N0 * N1};
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    int p[3] = {idx % N0, (idx / N0) % N1, idx / (N0 * N1)};
    for (int c = 0; c < 3; ++c)
      for (int l = 0; l < 3; ++l) {
        double v = 0.0;
        if (l < ndim && p[l] >= 2 && p[l] < Ns[l] - 2) v = d4at(X + (size_t)c * total, idx, ss[l]);
        D[(size_t)(3 * c + l) * total + idx] = v;
      }
  }
}

__global__ void __launch_bounds__(256) k_metric_outer(int ndim, int N0, int N1, int N2, const double* X,
                                                      const double* D, double* M) {
  const int total = N0 * N1 * N2;
  const int Ns[3] = {N0, N1, N2}, ss[3] = {1, N0, N0 * N1};
  const double* x = X;
  const double* y = X + total;
  const double* z = X + 2 * (size_t)total;
#define DD(c, l) (D + (size_t)(3 * (c) + (l)) * total)
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    int p[3] = {idx % N0, (idx / N0) % N1, idx / (N0 * N1)};
    bool ok = true;
    for (int l = 0; l < ndim; ++l) ok = ok && p[l] >= 2 && p[l] < Ns[l] - 2;
    double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (ok) {
      if (ndim == 1) {
        double xx = DD(0, 0)[idx];
        m[0] = 1.0; m[4] = xx; m[8] = xx; m[9] = 1.0 / xx;
      } else if (ndim == 2) {
        double xxi = DD(0, 0)[idx], xet = DD(0, 1)[idx], yxi = DD(1, 0)[idx], yet = DD(1, 1)[idx];
        m[0] = yet; m[1] = -xet; m[3] = -yxi; m[4] = xxi;
        double det = xxi * yet - xet * yxi;
        m[8] = det; m[9] = 1.0 / det;
      } else {
        // outer D4 of products of an inner derivative and a coordinate
        auto od = [&](int c, int li, const double* w, int lo) {
          const double* a = DD(c, li);
          int s = ss[lo];
          return (8.0 * (a[idx + s] * w[idx + s] - a[idx - s] * w[idx - s]) -
                  (a[idx + 2 * s] * w[idx + 2 * s] - a[idx - 2 * s] * w[idx - 2 * s])) / 12.0;
        };
        m[0] = od(1, 1, z, 2) - od(1, 2, z, 1);
        m[1] = od(2, 1, x, 2) - od(2, 2, x, 1);
        m[2] = od(0, 1, y, 2) - od(0, 2, y, 1);
        m[3] = od(1, 2, z, 0) - od(1, 0, z, 2);
        m[4] = od(2, 2, x, 0) - od(2, 0, x, 2);
        m[5] = od(0, 2, y, 0) - od(0, 0, y, 2);
        m[6] = od(1, 0, z, 1) - od(1, 1, z, 0);
        m[7] = od(2, 0, x, 1) - od(2, 1, x, 0);
        m[8] = od(0, 0, y, 1) - od(0, 1, y, 0);
        double xx = DD(0, 0)[idx], xe = DD(0, 1)[idx], xz = DD(0, 2)[idx];
        double yx = DD(1, 0)[idx], ye = DD(1, 1)[idx], yz = DD(1, 2)[idx];
        double zx = DD(2, 0)[idx], ze = DD(2, 1)[idx], zz = DD(2, 2)[idx];
        double det = xx * (ye * zz - yz * ze) - xe * (yx * zz - yz * zx) + xz * (yx * ze - ye * zx);
        m[9] = 1.0 / det;
      }
    }
    for (int c = 0; c < 10; ++c) M[(size_t)c * total + idx] = m[c];
  }
#undef DD
}

template <typename R>
__global__ void __launch_bounds__(256) k_convert(const double* src, R* dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (R)src[i];
}

// ------------------------------------------------------------------ planar grids
// Largest deviation, over planes 2 <= k < N2 - 2 (where node metrics are defined), of the
// node metrics and, at interior nodes, of Delta x_l from their values on the first interior
// plane, relative to the largest metric component (resp. component of Delta x_l) there.
// Stored as the bit pattern of a non-negative double (integer max orders them).
__global__ void __launch_bounds__(256) k_planar_dev(int N0, int N1, int N2, int g, const double* __restrict__ M,
                                                    const double* __restrict__ X, unsigned long long* out) {
  const size_t s2 = (size_t)N0 * N1, T = s2 * N2;
  double dev = 0.0;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < T; idx += (size_t)gridDim.x * blockDim.x) {
    const size_t k = idx / s2, col = idx % s2;
    const int i = (int)(col % N0), j = (int)(col / N0);
    if (k < 2 || k >= (size_t)N2 - 2 || i < 2 || i >= N0 - 2 || j < 2 || j >= N1 - 2) continue;
    const size_t ref = (size_t)g * s2 + col;
    double sc = 0.0;
    for (int c = 0; c < 9; ++c) sc = fmax(sc, fabs(M[c * T + ref]));
    if (sc > 0.0)
      for (int c = 0; c < 9; ++c) dev = fmax(dev, fabs(M[c * T + idx] - M[c * T + ref]) / sc);
    const double J0 = fabs(M[9 * T + ref]);
    if (J0 > 0.0) dev = fmax(dev, fabs(M[9 * T + idx] - M[9 * T + ref]) / J0);
    if (i >= g && i < N0 - g && j >= g && j < N1 - g && k >= (size_t)g && k < (size_t)(N2 - g)) {
      const size_t st[3] = {1, (size_t)N0, s2};
      for (int l = 0; l < 3; ++l) {
        double a[3], b[3], nb = 0.0;
        for (int c = 0; c < 3; ++c) {
          a[c] = 0.5 * (X[c * T + idx + st[l]] - X[c * T + idx - st[l]]);
          b[c] = 0.5 * (X[c * T + ref + st[l]] - X[c * T + ref - st[l]]);
          nb = fmax(nb, fabs(b[c]));
        }
        if (nb > 0.0)
          for (int c = 0; c < 3; ++c) dev = fmax(dev, fabs(a[c] - b[c]) / nb);
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_down(dev, off));
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(dev));
}

// ------------------------------------------------------------------ launchers
static inline dim3 grid_for(long long work, int nprob, int block = 256, int cap = 8192) {
  long long b = (work + block - 1) / block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return dim3((unsigned)b, (unsigned)nprob);
}

void launch_bc_cons(const Launch& L, StateRef ref, int d) {
  LG_TIMED(L, KC_BC, hipLaunchKernelGGL(k_bc_cons, grid_for(L.ghost_work[d], L.nprob), dim3(256), 0, L.stream,
                                        L.probs, ref, d));
}

template <typename R>
void launch_bc_scalar(const Launch& L, int which, int nf, int d) {
  LG_TIMED(L, KC_BC_SCALAR, hipLaunchKernelGGL(k_bc_scalar<R>, grid_for(L.ghost_work[d], L.nprob), dim3(256), 0,
                                               L.stream, L.probs, which, nf, d));
}

template <typename R>
void launch_prim(const Launch& L, StateRef ref, int want_flags, const uint8_t* force, int ghosts) {
  // pairs pay off with FP32 primitives (0.80 -> 0.78 ms on the ramp); FP64 runs faster one node per lane
  if (sizeof(R) == 4 && !L.prim_scalar && (unsigned long long)ref.Qx % 16 == 0)
    LG_TIMED(L, KC_PRIM, hipLaunchKernelGGL((k_prim<R, true>), grid_for(L.max_total / 2, L.nprob), dim3(256), 0,
                                            L.stream, L.probs, ref, want_flags, force, ghosts));
  else
    LG_TIMED(L, KC_PRIM, hipLaunchKernelGGL((k_prim<R, false>), grid_for(L.max_total, L.nprob), dim3(256), 0,
                                            L.stream, L.probs, ref, want_flags, force, ghosts));
}

void launch_any_flag(const Launch& L, int interior_only) {
  hipLaunchKernelGGL(k_zero_any, dim3(1, L.nprob), dim3(64), 0, L.stream, L.probs);
  const dim3 grid = interior_only ? zm_grid_col(L, 0, 0) : grid_for(L.max_total, L.nprob);
  LG_TIMED(L, KC_FLAGS, hipLaunchKernelGGL(k_any_flag, grid, dim3(256), 0, L.stream, L.probs, interior_only,
                                           zm_arg(L, 0, 0)));
}

void launch_dilate(const Launch& L, int ndim, int radius, int first_src, int final_buf) {
  // first_src -> ... -> final_buf, alternating with ftmp so that the last pass lands in final_buf
  int src = first_src;
  for (int d = 0; d < ndim; ++d) {
    int dst = ((ndim - 1 - d) % 2 == 0) ? final_buf : 1;
    if (radius == 3)   // the hybrid's radius: a window of seven loads instead of fifteen
      LG_TIMED(L, KC_FLAGS, hipLaunchKernelGGL(k_dilate<3>, grid_for(L.max_total, L.nprob), dim3(256), 0, L.stream,
                                               L.probs, d, src, dst, radius));
    else
      LG_TIMED(L, KC_FLAGS, hipLaunchKernelGGL(k_dilate<0>, grid_for(L.max_total, L.nprob), dim3(256), 0, L.stream,
                                               L.probs, d, src, dst, radius));
    src = dst;
  }
}

void launch_hyb_queue(const Launch& L, int ndim) {
  hipLaunchKernelGGL(k_hyb_init, dim3(1, L.nprob), dim3(64), 0, L.stream, L.probs);
  LG_TIMED(L, KC_FLAGS, hipLaunchKernelGGL(k_all_flag, zm_grid_col(L, 0, 0), dim3(256), 0, L.stream,
                                           L.probs, zm_arg(L, 0, 0)));
  for (int d = 0; d < ndim; ++d) {
    long long tot = 1;
    for (int l = 0; l < 3; ++l) tot *= L.max_n[l] + (l == d ? 1 : 0);
    const unsigned chunks = (unsigned)std::max<long long>(1, (tot + QCHUNK - 1) / QCHUNK);
    LG_TIMED(L, KC_FLAGS, hipLaunchKernelGGL(k_gbr_queue, dim3(chunks, L.nprob), dim3(256), 0, L.stream, L.probs,
                                             d));
  }
}

void launch_line_lists(const Launch& L, int ndim) {
  hipLaunchKernelGGL(k_zero_lcount, dim3(1, L.nprob), dim3(64), 0, L.stream, L.probs);
  for (int d = 0; d < ndim; ++d) {
    long long b = (L.lines[d] + 255) / 256;
    LG_TIMED(L, KC_FLAGS, hipLaunchKernelGGL(k_line_list, dim3((unsigned)(b < 1 ? 1 : b), L.nprob), dim3(256), 0,
                                             L.stream, L.probs, d));
  }
}

void launch_dt(const Launch& L, const double* Qx, double* tx, double t_end, int advance_t) {
  hipLaunchKernelGGL(k_dt_reset, dim3(1, L.nprob), dim3(64), 0, L.stream, L.probs);
  LG_TIMED(L, KC_DT, hipLaunchKernelGGL(k_dt_reduce, zm_grid_col(L, 0, 0), dim3(256), 0, L.stream,
                                        L.probs, Qx, zm_arg(L, 0, 0)));
  hipLaunchKernelGGL(k_dt_finalize, dim3(1, L.nprob), dim3(64), 0, L.stream, L.probs, tx, t_end, advance_t);
}

void launch_set_dt(const Launch& L, double dt) {
  hipLaunchKernelGGL(k_set_dt, dim3(1, L.nprob), dim3(64), 0, L.stream, L.probs, dt);
}

void launch_switch_count(const Launch& L) {
  hipLaunchKernelGGL(k_switch_count, dim3(1, L.nprob), dim3(64), 0, L.stream, L.probs);
}

void launch_zero_status(const Launch& L) {
  hipLaunchKernelGGL(k_zero_status, dim3(1, L.nprob), dim3(64), 0, L.stream, L.probs);
}

void launch_metrics(int ndim, const int N[3], const double* coords, double* scratch9, double* metrics,
                    hipStream_t s) {
  long long total = (long long)N[0] * N[1] * N[2];
  hipLaunchKernelGGL(k_metric_inner, grid_for(total, 1), dim3(256), 0, s, ndim, N[0], N[1], N[2], coords,
                     scratch9);
  hipLaunchKernelGGL(k_metric_outer, grid_for(total, 1), dim3(256), 0, s, ndim, N[0], N[1], N[2], coords,
                     scratch9, metrics);
}

void launch_planar_dev(int N0, int N1, int N2, int g, const double* M, const double* X, unsigned long long* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_planar_dev, grid_for((long long)N0 * N1 * N2, 1), dim3(256), 0, s, N0, N1, N2, g, M, X, out);
}

template <typename R>
void launch_convert(const double* src, R* dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_convert<R>, grid_for((long long)n, 1), dim3(256), 0, s, src, dst, n);
}

template void launch_bc_scalar<float>(const Launch&, int, int, int);
template void launch_bc_scalar<double>(const Launch&, int, int, int);
template void launch_prim<float>(const Launch&, StateRef, int, const uint8_t*, int);
template void launch_prim<double>(const Launch&, StateRef, int, const uint8_t*, int);
template void launch_convert<float>(const double*, float*, size_t, hipStream_t);
template void launch_convert<double>(const double*, double*, size_t, hipStream_t);

}  // namespace lg
