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

#include <type_traits>
#include <stdint.h>

namespace lg {

enum { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_REFLECTIVE = 2, BC_NOSLIP = 3, BC_FIXED = 4, BC_NOSLIP_T = 5 };
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
  double wall_T[3][2];   // wall temperature of isothermal no-slip faces (BC_NOSLIP_T)
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
  double* acc;       // classic RK4: sum of b_s dt k_s over the stages so far (workspace; RK4 contexts)
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
  void* S3;          // |S|, theta (LAD)                 [2][total]  R
  void* GX;          // Delta x_l = (x_{+1} - x_{-1}) / 2 [3 l + c][met_T] R (curvilinear only)
  void* CA;          // LAD coefficients mu*,beta*,kappa* [3][total] R (result)
  void* CB;          // LAD filter scratch               [3][total]  R
  void* FL[3];       // LAD node fluxes per direction    [5][total]  R
  void* FV[3];       // C-GBR viscous node fluxes        [5][total]  R
  const void* MR;    // node metrics in R                [10][met_T] (curvilinear only)
  const double* M64; // node metrics in FP64             [10][met_T] (curvilinear only)
  int met_planar;    // 1: metrics and Delta x_l do not vary along zeta; MR, M64, GX hold one plane
  int met_T;         // field stride of MR, M64 and GX: total, or N0 N1 when planar
  const double* coords;  // node coordinates             [3][total]  (curvilinear only)
  const double* tri[3];  // compact-solve LU tables per direction (see k_grad.hip)
  const double* pcr[3];  // compact-solve PCR factors per direction (see k_grad.hip)
  // LAD-C6 (see k_compact.hip for the table layouts)
  int lad_c6;            // the LAD scheme uses compact sixth-order differences
  double falpha;         // alpha_f of the implicit filter (0.5: no filter)
  double fcoef[6];       // filter right-hand-side weights a_0 .. a_5
  int fsteps;            // PCR reduction steps of the filter systems
  const double* tri6[3]; // C6 gradient systems: Thomas / cyclic tables
  const double* pcr6[3]; //   and PCR factors
  const double* trc[3];  // C6 interface-flux systems
  const double* pcrc[3];
  const double* trf[3];  // filter systems
  const double* pcrf[3];
  const double* fsegt[3]; // filter along eta / zeta by register segments (k_filter_seg tables)
  const double* c4segt[3];  // MIG4 gradients along eta / zeta by register segments (k_grad_c4_seg tables)
  const double* c6fsegt[3]; // LAD-C6 interface fluxes along eta / zeta by register segments (k_c6_faces_seg tables)
  const double* c6gz;       // LAD-C6 gradients along xi by the partition method: z_0 [64], (I - W)^{-1} [4]
  const double* c6gsegt[3]; // LAD-C6 gradients of periodic eta / zeta lines by register segments (k_grad_c4_seg tables)
  // device scalars
  double* dt;
  double* t;
  double t_end;
  unsigned long long* smax;  // max spectral radius (bit pattern of a positive double)
  int* status;               // non-physical node counts (STATUS_SLOTS slots, see add_bad)
  int* any_flag;             // global hybrid switch: any troubled interior node
  unsigned* sw;              // switching record: [0] hybrid stages, [1] those with a troubled node
  // compacted per-cell hybrid: work queue of the C-GBR interfaces and their fluxes
  int* all_flag;             // every interior node lies in the dilated troubled set
  int* gcount;               // [3] queued C-GBR interfaces per direction
  int* gq;                   // [3][total] queue: left-node index of each C-GBR interface
  void* FG[3];               // C-GBR interface fluxes per direction [5][total] R (at the left node)
};

__host__ __device__ __forceinline__ int pos_to_idx(const Prob& P, int i, int j, int k) {
  return i + P.s[1] * j + P.s[2] * k;
}

// Position of node idx in the metric arrays (its (i, j) column when they hold one plane).
__host__ __device__ __forceinline__ int met_idx(const Prob& P, int idx) {
  return P.met_planar ? idx % P.s[2] : idx;
}

// Node metric component c (0..8: l_hat_j for l = c/3, j = c%3; 9: J) at node idx.
template <typename R>
__host__ __device__ __forceinline__ R met(const Prob& P, int c, int idx) {
  if (P.curvilinear) return static_cast<const R*>(P.MR)[(size_t)c * P.met_T + met_idx(P, idx)];
  return (R)P.cm[c];
}

// all node metrics at idx: m[3 l + j] = l_hat_j of direction l, m[9] = J
template <typename R>
__device__ __forceinline__ void load_met(const Prob& P, int idx, R m[10]) {
  if (P.curvilinear) {
    const R* M = static_cast<const R*>(P.MR);
    const int mi = met_idx(P, idx);
    for (int c = 0; c < 10; ++c) m[c] = M[(size_t)c * P.met_T + mi];
  } else {
    for (int c = 0; c < 10; ++c) m[c] = (R)P.cm[c];
  }
}

__host__ __device__ __forceinline__ double met64(const Prob& P, int c, int idx) {
  if (P.curvilinear) return P.M64[(size_t)c * P.met_T + met_idx(P, idx)];
  return P.cm[c];
}

// Device-side switch of the hybrid.  any_flag: some troubled node; all_flag (per-cell form,
// valid after the flag dilation): every interior node is in the dilated troubled set, so
// every interface is C-GBR.  Gate codes of a launch:
//   GATE_NEVER (-1) always runs;
//   GATE_ANY   (0)  runs when a troubled node exists (C-GBR inputs, global C-GBR sweeps);
//   GATE_NONE  (1)  runs when none does (the all-LAD pass);
//   GATE_NOTALL(2)  runs unless every interface is C-GBR (LAD inputs of the per-cell form);
//   GATE_ALL   (3)  runs when every interface is C-GBR (plain direction sweeps);
//   GATE_MIXED (4)  runs when some but not all interfaces are C-GBR (compacted path).
enum { GATE_NEVER = -1, GATE_ANY = 0, GATE_NONE = 1, GATE_NOTALL = 2, GATE_ALL = 3, GATE_MIXED = 4 };
__device__ __forceinline__ bool gate_skip(const Prob& P, int gate) {
  if (gate < 0) return false;
  const bool any = *P.any_flag != 0;
  if (gate <= GATE_NONE) return any == (gate == GATE_NONE);
  const bool all = any && *P.all_flag != 0;
  if (gate == GATE_NOTALL) return all;
  if (gate == GATE_ALL) return !all;
  return !(any && !all);
}

// Per-cell stages solve the MIG4 lines that cross the C-GBR input region fg (compacted
// list, lcount[d] lines); when more than half of all lines of d are listed, the region-free
// kernels solving every line are cheaper, and the device takes them instead.
__device__ __forceinline__ bool dense_lines(const Prob& P, int d) {
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  return 2LL * P.lcount[d] > (long long)P.N[o1] * P.N[o2];
}

// Ghost image of position p along d for scalar intermediate fields (even parity; FIXED
// faces behave as transmissive): the interior position whose value the ghost holds.
__device__ __forceinline__ int scalar_image(const Prob& P, int d, int p) {
  const int g = P.g[d], n = P.n[d];
  if (p >= g && p < g + n) return p;
  const int side = p < g ? 0 : 1;
  int bct = P.bc[d][side];
  if (bct == BC_PERIODIC) {
    int r = (p - g) % n;
    return g + (r < 0 ? r + n : r);
  }
  if (bct == BC_TRANSMISSIVE || bct == BC_FIXED) return side == 0 ? g : g + n - 1;
  // mirror; within the ghost depth (n >= 5) the image is interior, the clamp only keeps
  // positions farther out in bounds
  const int m = side == 0 ? 2 * g - 1 - p : 2 * (g + n) - 1 - p;
  return m < g ? g : (m > g + n - 1 ? g + n - 1 : m);
}

// ------------------------------------------------------------------ z-marching tiles
// A z-marching launch covers the band [g + lo, g + n + hi) of every active direction
// (node 0 of inactive ones) with tiles of TX x TY columns (i, j); a workgroup walks its
// columns through one chunk of zc planes, so values along z are reused from registers.
// Hardware workgroups are dealt round-robin to the eight XCDs (workgroup b runs on XCD
// b mod 8, gridDim.x is a multiple of 8): the logical order hands each XCD one
// contiguous range of tiles -- whole z-chunks -- so that neighbouring rows meet in the
// same L2.  The decode is uniform over the workgroup.
__device__ __forceinline__ void zm_band(const Prob& P, int lo, int hi, int org[3], int ext[3]) {
  for (int d = 0; d < 3; ++d) {
    const bool a = d < P.ndim;
    org[d] = a ? P.g[d] + lo : 0;
    ext[d] = a ? P.n[d] + hi - lo : 1;
  }
}

__device__ __forceinline__ bool zm_tile_rt(const int ext[3], int zc, int TX, int TY, int& ti0, int& tj0, int& k0,
                                           int& k1) {
  const int ntx = (ext[0] + TX - 1) / TX, nty = (ext[1] + TY - 1) / TY, nch = (ext[2] + zc - 1) / zc;
  const int nblk = ntx * nty * nch;
  const int per = (nblk + 7) >> 3;
  if ((int)(blockIdx.x >> 3) >= per) return false;
  const int L = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (L >= nblk) return false;
  const int t = L % (ntx * nty), ch = L / (ntx * nty);
  ti0 = (t % ntx) * TX;
  tj0 = (t / ntx) * TY;
  k0 = ch * zc;
  k1 = min(ext[2], k0 + zc);
  return true;
}

template <int TX, int TY>
__device__ __forceinline__ bool zm_tile(const int ext[3], int zc, int& ti0, int& tj0, int& k0, int& k1) {
  return zm_tile_rt(ext, zc, TX, TY, ti0, tj0, k0, k1);
}

constexpr int ZM_TX = 64, ZM_TY = 4;

struct ZCol {
  int i, j, k0, k1;  // padded positions of the column; planes [k0, k1)
};

// This thread's column of a z-marching launch of 256 lanes; false if it has none.  zcw: the
// planes per chunk in its low 16 bits, above them log2 of the tile width along xi (the tile
// has 256 / width rows; 0: the default 64 x 4).
__device__ __forceinline__ bool zm_column(const Prob& P, int lo, int hi, int zcw, ZCol& c) {
  int org[3], ext[3];
  zm_band(P, lo, hi, org, ext);
  const int lt = zcw >> 16;
  const int TX = lt ? 1 << lt : ZM_TX, TY = 256 / TX;
  int ti0, tj0, k0, k1;
  if (!zm_tile_rt(ext, zcw & 0xFFFF, TX, TY, ti0, tj0, k0, k1)) return false;
  const int ti = ti0 + (int)(threadIdx.x & (TX - 1)), tj = tj0 + (int)(threadIdx.x >> (lt ? lt : 6));
  if (ti >= ext[0] || tj >= ext[1]) return false;
  c.i = org[0] + ti;
  c.j = org[1] + tj;
  c.k0 = org[2] + k0;
  c.k1 = org[2] + k1;
  return true;
}

// Fields addressed as global memory (the descriptor's pointers are otherwise generic) by
// 32-bit element offsets from a scalar base when O32 (every field below 2^32 bytes; chosen
// on the host): per-lane addresses then take one register instead of two, and the loads
// wait on the vector-memory counter only.
#define LG_GLOBAL __attribute__((address_space(1)))
template <bool O32>
using sidx_t = typename std::conditional<O32, unsigned, size_t>::type;

template <typename T, bool O32>
__device__ __forceinline__ T gld(const T* base, sidx_t<O32> e) {
  if constexpr (O32)
    return *(const LG_GLOBAL T*)((const LG_GLOBAL char*)base + e * (unsigned)sizeof(T));
  else
    return base[e];
}
template <typename T, bool O32>
__device__ __forceinline__ void gst(T* base, sidx_t<O32> e, T v) {
  if constexpr (O32)
    *(LG_GLOBAL T*)((LG_GLOBAL char*)base + e * (unsigned)sizeof(T)) = v;
  else
    base[e] = v;
}

// Non-physical node counts: STATUS_SLOTS counters STATUS_STRIDE ints (one 128-byte line)
// apart, workgroup b adding to slot b mod STATUS_SLOTS (an address uniform in the wave).
// One shared counter serialises when a whole field goes bad (every wave adding to one
// address); the host sums the slots.
constexpr int STATUS_SLOTS = 64, STATUS_STRIDE = 32;
__device__ __forceinline__ void add_bad(const Prob& P, int bad) {
  if (bad) atomicAdd(P.status + STATUS_STRIDE * (blockIdx.x & (STATUS_SLOTS - 1)), bad);
}

// Reciprocal in the bulk arithmetic: the hardware estimate (within 1 ulp) in FP32, the
// correctly rounded quotient in FP64.
template <typename R>
__device__ __forceinline__ R rcp(R x);
template <>
__device__ __forceinline__ float rcp<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}
template <>
__device__ __forceinline__ double rcp<double>(double x) {
  return 1.0 / x;
}

// a / b in the bulk type of the C-GBR flux: FP64 divides (correctly rounded); FP32
// multiplies by the hardware reciprocal (within 1 ulp, one instruction against the ten of
// a correctly rounded division), which the FP32 bulk's own accuracy allows
template <typename R>
__device__ __forceinline__ R bdiv(R a, R b) {
  return a / b;
}
template <>
__device__ __forceinline__ float bdiv<float>(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);
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
