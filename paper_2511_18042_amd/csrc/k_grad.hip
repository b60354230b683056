// Gradients of the primitives along one computational direction.
//
// Paper: Sec. 2.3 -- MEG6 reconstructs from explicit sixth-order gradients, MIG4 from
// implicit fourth-order (compact) gradients, which cost one tridiagonal solve per line
// and primitive (Sec. 4.2).  Unit computational spacing (Sec. 2.2).
//
//   E6: f'_i = [45 (f_{i+1}-f_{i-1}) - 9 (f_{i+2}-f_{i-2}) + (f_{i+3}-f_{i-3})] / 60
//   C4: f'_{i-1}/4 + f'_i + f'_{i+1}/4 = 3 (f_{i+1} - f_{i-1}) / 4
//
// C4 closure: a bounded line is solved over all of its nodes (ghosts included) with
// second-order one-sided end rows; a periodic line is solved cyclically over its
// interior nodes (Sherman-Morrison on top of a bounded solve) and its ghost values are
// the periodic images.  The solves run in FP64 from primitives formed in FP64 from the
// conserved state, whatever the bulk precision.  Each lane owns one (line, primitive)
// pair; the LU factors of the constant-coefficient matrices are precomputed on the host
// (tables below), so a solve is one forward and one backward sweep.
//
// Table layout for direction d (double), after the PCR factors (see k_grad_c4_pcr):
//   bounded  line of N nodes: cp[0..N), inv[0..N)
//   periodic line of n nodes: cp[0..n), inv[0..n), z[0..n), fac   (B z = u, fac = 1/(1 + v.z))
#include "lgbr_dev.h"
#include "lgbr_kernels.h"

#include <algorithm>

namespace lg {

__device__ __forceinline__ bool skip_launch(const Prob& P, int skip_if_any) {
  return gate_skip(P, skip_if_any);
}

template <typename R, int ORDER>
__global__ void __launch_bounds__(256) k_grad_explicit(const Prob* __restrict__ probs, int d, int skip_if_any,
                                                       int region) {
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || skip_launch(P, skip_if_any)) return;
  const R* W = static_cast<const R*>(P.W);
  R* G = static_cast<R*>(P.G[d]);
  const int r = ORDER / 2, Nd = P.N[d], sd = P.s[d];
  const size_t T = P.total;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < P.total; idx += gridDim.x * blockDim.x) {
    int c = (idx / sd) % Nd;
    if (c < r || c >= Nd - r) continue;
    if (region && !P.fg[idx]) continue;
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

constexpr int PCR_STEPS = LG_PCR_STEPS;
constexpr int PCR_MAX_LINE = 4096;          // longest line held in LDS (2 x 32 KB)
constexpr long long PCR_FEW_LINES = 131072; // below this many (line, variable) lanes, PCR for strided lines

// Which kernel solves the lines of direction d of problem P: the PCR kernel takes the
// contiguous direction, and strided directions with few lines; periodic lines need at
// least 2^(PCR_STEPS+1) nodes so that no reduction step wraps onto itself.
__device__ __forceinline__ bool use_pcr(const Prob& P, int d) {
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const long long nlines = (long long)P.N[o1] * P.N[o2];
  const bool periodic = P.bc[d][0] == BC_PERIODIC;
  const int L = periodic ? P.n[d] : P.N[d];
  if (P.N[d] > PCR_MAX_LINE || (periodic && L < (2 << PCR_STEPS))) return false;
  return d == 0 || 5 * nlines < PCR_FEW_LINES;
}

__device__ __forceinline__ double prim_q(int q, const double* Q, size_t T, size_t o, double gm1) {
  double rho = Q[o];
  if (q == 0) return rho;
  if (q <= 3) return Q[q * T + o] / rho;
  double u = Q[T + o] / rho, v = Q[2 * T + o] / rho, w = Q[3 * T + o] / rho;
  return gm1 * (Q[4 * T + o] - 0.5 * rho * (u * u + v * v + w * w));
}

// all five FP64 primitives at offset o (one reciprocal of rho)
__device__ __forceinline__ void prims5(const double* Q, size_t T, size_t o, double gm1, double w[5]) {
  const double rho = Q[o], ri = 1.0 / rho;
  const double u = Q[T + o] * ri, v = Q[2 * T + o] * ri, x = Q[3 * T + o] * ri;
  w[0] = rho;
  w[1] = u;
  w[2] = v;
  w[3] = x;
  w[4] = gm1 * (Q[4 * T + o] - 0.5 * rho * (u * u + v * v + x * x));
}

// One lane per line, all five primitives at once (the state is read once per node):
// forward elimination stores d' in the FP64 scratch, back substitution writes the
// gradients.
template <typename R>
__global__ void __launch_bounds__(256) k_grad_c4(const Prob* __restrict__ probs, StateRef ref, int d, int skip_if_any,
                                                 int region, int mask) {
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || skip_launch(P, skip_if_any)) return;
  if (use_pcr(P, d)) return;   // done by the PCR kernel
  // region 1: the listed lines (unless most lines are listed); 2: every line, when most are
  if (region == 1 && dense_lines(P, d)) return;
  if (region == 2 && !dense_lines(P, d)) return;
  const bool listed = region == 1;
  if (!listed && tile_use(P, d, TK_GRAD4, mask)) return;   // done in LDS tiles
  if (!listed && c4_part_use(P, d, mask)) return;          // done by the partition method
  if (!listed && c4_seg_use(P, d, mask)) return;           // done in register segments
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const int nlines = P.N[o1] * P.N[o2];
  const int cnt = listed ? P.lcount[d] : nlines;   // compacted list of lines that need solving
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const int line = listed ? P.llist[d][t] : t;
  const double* Q = ref.state(P);
  R* G = static_cast<R*>(P.G[d]);
  const size_t T = P.total;
  double* S = P.T64;
  const double* tab = P.tri[d];
  const int a = line % P.N[o1], b = line / P.N[o1];
  const size_t base = (size_t)a * P.s[o1] + (size_t)b * P.s[o2];
  const int sd = P.s[d], g = P.g[d], n = P.n[d], N = P.N[d];
  const double gm1 = P.gamma - 1.0;
  auto f = [&](int pos, double w[5]) { prims5(Q, T, base + (size_t)pos * sd, gm1, w); };

  if (P.bc[d][0] != BC_PERIODIC) {
    const double* cp = tab;
    const double* inv = tab + N;
    double fm[5], f0[5], fp[5], dprev[5];
    f(0, fm);
    f(1, f0);
    f(2, fp);
    for (int q = 0; q < 5; ++q) {
      dprev[q] = (-3.0 * fm[q] + 4.0 * f0[q] - fp[q]) / 2.0;   // row 0 (one-sided, decoupled)
      S[q * T + base] = dprev[q];
    }
    double fmm[5];   // f(N-3) once the sweep ends
    for (int i = 1; i < N - 1; ++i) {
      if (i > 1) f(i + 1, fp);
      for (int q = 0; q < 5; ++q) {
        const double dd = (0.75 * (fp[q] - fm[q]) - 0.25 * dprev[q]) * inv[i];
        S[q * T + base + (size_t)i * sd] = dd;
        dprev[q] = dd;
        fmm[q] = fm[q];
        fm[q] = f0[q];
        f0[q] = fp[q];
      }
    }
    // last row (one-sided, decoupled): f0 = f(N-1), fm = f(N-2), fmm = f(N-3)
    double y[5];
    for (int q = 0; q < 5; ++q) {
      y[q] = (3.0 * f0[q] - 4.0 * fm[q] + fmm[q]) / 2.0;
      G[q * T + base + (size_t)(N - 1) * sd] = (R)y[q];
    }
    for (int i = N - 2; i >= 0; --i)
      for (int q = 0; q < 5; ++q) {
        y[q] = S[q * T + base + (size_t)i * sd] - cp[i] * y[q];
        G[q * T + base + (size_t)i * sd] = (R)y[q];
      }
  } else {
    // cyclic system over the interior (the ghosts hold the periodic images):
    // B y = r, x = y - (v.y) fac z with v.y = y_0 - y_{n-1}/4 (Sherman-Morrison)
    const double* cp = tab;
    const double* inv = tab + n;
    const double* z = tab + 2 * n;
    const double fac = tab[3 * n];
    const double* y0c = tab + 3 * n + 2;   // y_0 = sum_k c_k d_k (see the host table)
    const size_t b0 = base + (size_t)g * sd;
    double fm[5], f0[5], fp[5], dprev[5], y0[5] = {0, 0, 0, 0, 0};
    f(g - 1, fm);
    f(g, f0);
    for (int i = 0; i < n; ++i) {
      f(g + i + 1, fp);
      for (int q = 0; q < 5; ++q) {
        const double rhs = 0.75 * (fp[q] - fm[q]);
        const double dd = (i == 0 ? rhs : rhs - 0.25 * dprev[q]) * inv[i];
        S[q * T + b0 + (size_t)i * sd] = dd;
        dprev[q] = dd;
        y0[q] = y0[q] + y0c[i] * dd;
        fm[q] = f0[q];
        f0[q] = fp[q];
      }
    }
    // one back substitution emitting x = y - (y_0 - y_{n-1}/4) fac z
    double y[5], vy[5];
    for (int q = 0; q < 5; ++q) {
      y[q] = dprev[q];
      vy[q] = (y0[q] - 0.25 * dprev[q]) * fac;
    }
    for (int i = n - 1; i >= 0; --i)
      for (int q = 0; q < 5; ++q) {
        if (i < n - 1) y[q] = S[q * T + b0 + (size_t)i * sd] - cp[i] * y[q];
        const R xv = (R)(y[q] - vy[q] * z[i]);
        G[q * T + b0 + (size_t)i * sd] = xv;
        if (i >= n - g) G[q * T + b0 + (size_t)(i - n) * sd] = xv;   // low ghosts
        if (i < g) G[q * T + b0 + (size_t)(i + n) * sd] = xv;        // high ghosts
      }
  }
}

// ------------------------------------------------------------------ line solves by PCR
// One workgroup per (line, primitive): the line's right-hand side is formed in LDS from
// FP64 primitives and reduced by parallel cyclic reduction.  The matrix is the same for
// every line of a direction, so the elimination factors k1 = a_i / b_{i-s} and
// k2 = c_i / b_{i+s} of every step and the final 1/b_i are precomputed on the host
// (table layout: k1[PCR_STEPS][L], k2[PCR_STEPS][L], binv[L], then per step the band of
// rows sharing one pair of factors).  For the C4 matrix the couplings shrink as
// (2 - sqrt 3)^(2^k), so after PCR_STEPS = 6 steps they are below 1e-36 of the diagonal
// and x_i = d_i / b_i is the direct solution up to rounding.
// Periodic lines reduce the cyclic system over the interior with wrapped indices.
template <typename R>
__global__ void __launch_bounds__(256) k_grad_c4_pcr(const Prob* __restrict__ probs, StateRef ref, int d,
                                                     int skip_if_any, int region, int mask) {
  extern __shared__ double lds[];
  const Prob& P = probs[blockIdx.y];
  if (d >= P.ndim || skip_launch(P, skip_if_any)) return;
  if (!use_pcr(P, d)) return;   // the lane-per-line kernel does these
  // region 1: the listed lines (unless most lines are listed); 2: every line, when most are
  if (region == 1 && dense_lines(P, d)) return;
  if (region == 2 && !dense_lines(P, d)) return;
  const bool listed = region == 1;
  if (!listed && tile_use(P, d, TK_GRAD4, mask)) return;   // done in LDS tiles
  if (!listed && c4_part_use(P, d, mask)) return;          // done by the partition method
  if (!listed && c4_seg_use(P, d, mask)) return;           // done in register segments
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const int nlines = P.N[o1] * P.N[o2];
  const int cnt = listed ? P.lcount[d] : nlines;   // compacted list of lines that need solving
  // persistent workgroups walk the (line, primitive) items
  for (int blk = blockIdx.x; blk < 5 * cnt; blk += gridDim.x) {
  const int line = listed ? P.llist[d][blk % cnt] : blk % nlines, q = blk / cnt;
  const bool periodic = P.bc[d][0] == BC_PERIODIC;
  const int g = P.g[d], N = P.N[d], n = P.n[d];
  const int L = periodic ? n : N;
  const int off0 = periodic ? g : 0;
  const int a = line % P.N[o1], b = line / P.N[o1];
  const size_t base = (size_t)a * P.s[o1] + (size_t)b * P.s[o2];
  const int sd = P.s[d];
  const double* Q = ref.state(P);
  const size_t T = P.total;
  const double gm1 = P.gamma - 1.0;
  const double* tab = P.pcr[d];
  double* f = lds;        // primitive along the line (all N nodes)
  double* r = lds + N;    // right-hand side, reduced in place
  for (int i = threadIdx.x; i < N; i += blockDim.x) f[i] = prim_q(q, Q, T, base + (size_t)i * sd, gm1);
  __syncthreads();
  for (int i = threadIdx.x; i < L; i += blockDim.x) {
    double v;
    if (periodic) {
      v = 0.75 * (f[off0 + i + 1] - f[off0 + i - 1]);
    } else if (i == 0) {
      v = (-3.0 * f[0] + 4.0 * f[1] - f[2]) / 2.0;
    } else if (i == L - 1) {
      v = (3.0 * f[L - 1] - 4.0 * f[L - 2] + f[L - 3]) / 2.0;
    } else {
      v = 0.75 * (f[i + 1] - f[i - 1]);
    }
    r[i] = v;
  }
  __syncthreads();
  constexpr int MAXPT = PCR_MAX_LINE / 256;
  double nv[MAXPT];
  // rows inside a step's band share two factors (band header after the table), so only
  // rows near the line ends read the table
  const double* hdr = tab + (size_t)(2 * PCR_STEPS + 1) * L;
  for (int st = 0; st < PCR_STEPS; ++st) {
    const int s = 1 << st;
    const double* k1 = tab + (size_t)st * L;
    const double* k2 = tab + (size_t)(PCR_STEPS + st) * L;
    const double c1 = hdr[4 * st], c2 = hdr[4 * st + 1];
    const int blo = (int)hdr[4 * st + 2], bhi = (int)hdr[4 * st + 3];
#pragma unroll
    for (int m = 0; m < MAXPT; ++m) {
      int i = threadIdx.x + m * 256;
      if (i < L) {
        int im = i - s, ip = i + s;
        double rm, rp;
        if (periodic) {
          im = ((im % L) + L) % L;
          ip = ip % L;
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
    for (int m = 0; m < MAXPT; ++m) {
      int i = threadIdx.x + m * 256;
      if (i < L) r[i] = nv[m];
    }
    __syncthreads();
  }
  const double* binv = tab + (size_t)2 * PCR_STEPS * L;
  const double cb = hdr[4 * PCR_STEPS];
  const int blo = (int)hdr[4 * PCR_STEPS + 2], bhi = (int)hdr[4 * PCR_STEPS + 3];
  R* G = static_cast<R*>(P.G[d]) + (size_t)q * T;
  for (int i = threadIdx.x; i < L; i += blockDim.x) {
    R y = (R)(r[i] * ((i < blo || i > bhi) ? binv[i] : cb));
    G[base + (size_t)(i + off0) * sd] = y;
    if (periodic) {
      if (i >= n - g) G[base + (size_t)(i + off0 - n) * sd] = y;   // low ghosts
      if (i < g) G[base + (size_t)(i + off0 + n) * sd] = y;        // high ghosts
    }
  }
  __syncthreads();   // the next item reuses the LDS line
  }
}

template <typename R>
void launch_grad_explicit(const Launch& L, int d, int order, int skip_if_any, int region) {
  long long b = (L.max_total + 255) / 256;
  if (b > 8192) b = 8192;
  dim3 grid((unsigned)b, L.nprob);
  if (order == 6)
    LG_TIMED(L, KC_GRAD_E6, hipLaunchKernelGGL((k_grad_explicit<R, 6>), grid, dim3(256), 0, L.stream, L.probs, d,
                                               skip_if_any, region));
  else
    LG_TIMED(L, KC_GRAD_E6, hipLaunchKernelGGL((k_grad_explicit<R, 4>), grid, dim3(256), 0, L.stream, L.probs, d,
                                               skip_if_any, region));
}

template <typename R>
void launch_grad_c4(const Launch& L, StateRef ref, int d, int skip_if_any, int region) {
  // each problem's direction is taken by exactly one kernel: LDS line tiles (region-free
  // launches, tile_use), PCR in LDS with persistent workgroups over the (line, primitive)
  // items, or one lane per line.  With a region (per-cell hybrid) the listed lines are
  // solved, or, when most lines are listed, every line by the region-free kernels (the
  // device picks one of the two sets).
  auto full = [&](int reg) {
    launch_grad_c4_tiles<R>(L, ref, d, skip_if_any, reg == 2);
    if (d == 0) launch_grad_c4_part<R>(L, ref, skip_if_any, reg == 2);
    else launch_grad_c4_seg<R>(L, ref, d, skip_if_any, reg == 2);
    if (L.c4_rest_pcr[d]) {
      const long long N = std::min<long long>(L.max_N[d], PCR_MAX_LINE);
      const unsigned lds = (unsigned)(2 * N * sizeof(double));
      long long blocks = std::min<long long>(5 * L.lines[d], L.pcr_blocks > 0 ? L.pcr_blocks : 16384);
      LG_TIMED(L, KC_GRAD_C4, hipLaunchKernelGGL(k_grad_c4_pcr<R>, dim3((unsigned)blocks, L.nprob), dim3(256), lds,
                                                 L.stream, L.probs, ref, d, skip_if_any, reg, L.tile_mask));
    }
    if (L.c4_rest_thomas[d]) {
      long long b = (L.lines[d] + 255) / 256;
      LG_TIMED(L, KC_GRAD_C4, hipLaunchKernelGGL(k_grad_c4<R>, dim3((unsigned)b, L.nprob), dim3(256), 0, L.stream,
                                                 L.probs, ref, d, skip_if_any, reg, L.tile_mask));
    }
  };
  if (!region) {
    full(0);
    return;
  }
  if (L.pcr_dir[d]) {
    const long long N = std::min<long long>(L.max_N[d], PCR_MAX_LINE);
    const unsigned lds = (unsigned)(2 * N * sizeof(double));
    long long blocks = std::min<long long>(5 * L.lines[d], L.pcr_blocks > 0 ? L.pcr_blocks : 16384);
    LG_TIMED(L, KC_GRAD_C4, hipLaunchKernelGGL(k_grad_c4_pcr<R>, dim3((unsigned)blocks, L.nprob), dim3(256), lds,
                                               L.stream, L.probs, ref, d, skip_if_any, 1, 0));
  }
  if (L.thomas_dir[d]) {
    long long b = (L.lines[d] + 255) / 256;
    LG_TIMED(L, KC_GRAD_C4, hipLaunchKernelGGL(k_grad_c4<R>, dim3((unsigned)b, L.nprob), dim3(256), 0, L.stream,
                                               L.probs, ref, d, skip_if_any, 1, 0));
  }
  full(2);
}

template void launch_grad_explicit<float>(const Launch&, int, int, int, int);
template void launch_grad_explicit<double>(const Launch&, int, int, int, int);
template void launch_grad_c4<float>(const Launch&, StateRef, int, int, int);
template void launch_grad_c4<double>(const Launch&, StateRef, int, int, int);

}  // namespace lg
