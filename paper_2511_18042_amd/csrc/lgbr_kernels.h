// Launch interface between the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include "lgbr_dev.h"

namespace lg {

// Which conserved state / derivative a launch works on.  Single-problem calls pass
// caller pointers (Qx, dQx); batched launches pass null and each problem uses its own
// buffers (src = 0: P.Q, src = 1: P.Us).
struct StateRef {
  double* Qx;
  double* dQx;
  int src;
  __device__ __forceinline__ double* state(const Prob& P) const { return Qx ? Qx : (src ? P.Us : P.Q); }
  __device__ __forceinline__ double* deriv(const Prob& P) const { return dQx ? dQx : P.dQ; }
};

// RK stage combination operands (null -> the problem's own buffers by stage).
struct RKRef {
  const double* Un;
  const double* Us;
  double* out;
  int save_dq;    // the all-LAD pass also copies the stage result into dQ/dt (the filter guard's copy)
  int prim_out;   // the all-LAD pass also writes the primitives of the stage result (1), and its
                  // troubled flags (2), at interior nodes: the next stage converts the ghosts only
};

// Primitives of one node in the bulk type, p in FP64 (the conversion of k_prim)
template <typename R>
__device__ __forceinline__ void prim_node(const Prob& P, double rho, double m1, double m2, double m3, double E,
                                          R& r0, R& r1, R& r2, R& r3, R& r4, double& p) {
  double u = m1 / rho, v = m2 / rho, w = m3 / rho;
  p = (P.gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v + w * w));
  r0 = (R)rho;
  r1 = (R)u;
  r2 = (R)v;
  r3 = (R)w;
  r4 = (R)p;
}

// Troubled-cell test (Sec. 5): density or pressure below its threshold (strict); a value
// that is not a number also counts, so that a broken state is never taken for a smooth one.
__device__ __forceinline__ bool troubled(double rho, double p, const Prob& P) {
  return !(rho >= P.rho_thr) || !(p >= P.p_thr);
}

// Stage result at interior node idx: out = a U^n + b (U^s + dt L); true if non-physical
// (rho <= 0, p <= 0 or not finite).  U^s may alias out (each node reads before it writes).
__device__ __forceinline__ bool rk_combine_node(const Prob& P, const RKRef& rr, int stage, double a, double b,
                                                double dt, int idx, const double L[5]) {
  const double* Un = rr.Un ? rr.Un : P.Q;
  const double* Us = rr.Us ? rr.Us : (stage == 0 ? Un : P.Us);
  double* out = rr.out ? rr.out : (stage == 2 ? const_cast<double*>(Un) : P.Us);
  const size_t T = P.total;
  double v[5];
  for (int q = 0; q < 5; ++q) {
    const size_t o = q * T + idx;
    v[q] = a * Un[o] + b * (Us[o] + dt * L[q]);
    out[o] = v[q];
  }
  const double rho = v[0];
  const double ke = 0.5 * (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / rho;
  const double p = (P.gamma - 1.0) * (v[4] - ke);
  const bool ok = rho > 0.0 && p > 0.0 && isfinite(rho) && isfinite(p) && isfinite(v[1]) && isfinite(v[2]) &&
                  isfinite(v[3]);
  return !ok;
}

// Kernel classes for the optional per-launch event timing (lg_prof_start / lg_prof_stop).
enum KClass {
  KC_BC = 0, KC_PRIM, KC_FLAGS, KC_GRAD_E6, KC_GRAD_C4, KC_SENSOR, KC_VISC, KC_LAD_NODE, KC_LAD_RAW,
  KC_GAUSS, KC_LAD_FLUX, KC_SWEEP_X, KC_SWEEP_Y, KC_SWEEP_Z, KC_COMBINE, KC_DT, KC_BC_SCALAR, KC_LAD_SWEEP,
  KC_C6_FACES, KC_FILTER, KC_GBR_ITEMS, KC_HYB_ASSEMBLE, KC_FILTER_GUARD, KC_COUNT
};

// Event pairs recorded around launches while enabled (never during graph capture).
struct Prof {
  int enabled;
  int target;       // KClass to time, or -1 for all
  int n, cap;
  hipEvent_t* ev;   // 2 * cap events
  int* cls;         // class of each recorded launch
};

// Reduction steps of the PCR line solves (host tables and device kernel must agree).
constexpr int LG_PCR_STEPS = 6;

// Launch geometry shared by all problems of one launch (maxima over the problems).
struct Launch {
  const Prob* probs;   // device array
  int nprob;
  hipStream_t stream;
  long long max_total;     // ghost-padded nodes
  long long max_cells;     // interior nodes
  long long ghost_work[3]; // ghost nodes of one direction (2 g N_other1 N_other2)
  long long lines[3];      // lines along each direction (all nodes of the other two dims)
  long long max_N[3];      // ghost-padded extent per direction
  long long max_n[3];      // interior extent per direction
  long long sweep_rows[3]; // interior lines (interior of the other two dims) per direction
  int has_short_periodic;  // some periodic direction has fewer than 128 interior nodes
  int has_fixed;           // some problem has a FIXED face (caller-owned ghosts)
  int o64;                 // some problem's fields need 64-bit offsets (5 FP64 planes >= 2^32 B)
  int geo_generic;         // some problem is not 3D curvilinear with metrics planar along zeta
  int inviscid;            // some problem is inviscid
  int prim_scalar;         // some problem rules out two nodes per lane in k_prim (odd count, alignment)
  int pcr_dir[3];          // some problem solves its lines along d by PCR
  int thomas_dir[3];       // some problem solves its lines along d one lane per line
  // LAD-C6 line systems [TK_*][d]: which kernels some problem needs (tile_use with this
  // launch's tile_mask): LDS line tiles, PCR per (line, variable), one lane per line
  int ctile[4][3], cpcr[3][3], cthomas[3][3];
  int c4_rest_pcr[3], c4_rest_thomas[3];   // C4 gradients of region-free launches not in tiles
  int tile_mask;           // bit 3 TK_* + d: LDS tiles allowed for that system and direction
  int max_fsteps;          // most PCR steps of any problem's filter systems
  int ndim;
  int seg;                 // nodes per thread in the strided sweeps (0: heuristic)
  int pcr_blocks;          // persistent workgroups of the PCR line solves (0: heuristic)
  int zc;                  // planes per chunk of the z-marching kernels (0: heuristic)
  int ztx;                 // width along xi of the z-marching tiles (32, 64, 128; 0: 64)
  int tile_lines;          // most lines per LDS line tile (0: as many as fit)
  int item_blocks;         // persistent workgroups of the compacted C-GBR interface pass (0: 2048)
  int fpart;               // some problem filters along xi with the partition-method kernel
  int c4part;              // some problem solves its MIG4 gradients along xi by the partition method
  int c6fpart;             // some problem solves its LAD-C6 faces along xi by the partition method
  int c6gpart;             // some problem solves its LAD-C6 gradients along xi by the partition method
  int c4seg[3];            // most segments per line of the problems solving MIG4 gradients along d in k_grad_c4_seg (0: none)
  int c6fseg[3];           // most segments per line of the problems solving LAD-C6 faces along d in k_c6_faces_seg (0: none)
  int c6gseg[3];           // most segments per line of the problems solving LAD-C6 gradients along d in k_grad_c4_seg (0: none)
  int fseg[3];             // most segments per line of the problems filtering along d by k_filter_seg (0: none)
  Prof* prof;              // optional launch timing (null: off)
};

inline bool prof_on(const Launch& L, int k) {
  return L.prof && L.prof->enabled && (L.prof->target < 0 || L.prof->target == k) && L.prof->n < L.prof->cap;
}
inline void prof_begin(const Launch& L, int k) {
  if (prof_on(L, k)) {
    (void)hipEventRecord(L.prof->ev[2 * L.prof->n], L.stream);
    L.prof->cls[L.prof->n] = k;
  }
}
inline void prof_end(const Launch& L, int k) {
  if (L.prof && L.prof->enabled && L.prof->n < L.prof->cap && L.prof->cls[L.prof->n] == k &&
      (L.prof->target < 0 || L.prof->target == k)) {
    (void)hipEventRecord(L.prof->ev[2 * L.prof->n + 1], L.stream);
    L.prof->n++;
  }
}

// RAII-free helper: time one launch statement
#define LG_TIMED(L, k, stmt) \
  do {                       \
    prof_begin((L), (k));    \
    stmt;                    \
    prof_end((L), (k));      \
  } while (0)

void launch_bc_cons(const Launch& L, StateRef ref, int d);
template <typename R> void launch_bc_scalar(const Launch& L, int which, int nf, int d);
template <typename R>
void launch_prim(const Launch& L, StateRef ref, int want_flags, const uint8_t* force, int ghosts = 0);
void launch_any_flag(const Launch& L, int interior_only);
void launch_dilate(const Launch& L, int ndim, int radius, int first_src, int final_buf);
void launch_line_lists(const Launch& L, int ndim);
// compacted per-cell hybrid: all_flag, then the C-GBR interface queue of each direction;
// the persistent C-GBR interface pass over the queue; the assembly of the node derivatives
// (C-GBR interface fluxes from the queue pass, LAD ones from the node fluxes), with the RK
// stage when rr is given
void launch_hyb_queue(const Launch& L, int ndim);
template <typename R> void launch_gbr_items(const Launch& L);
template <typename R>
void launch_hyb_assemble(const Launch& L, StateRef ref, const RKRef* rr, int stage, double a, double b);
void launch_dt(const Launch& L, const double* Qx, double* tx, double t_end, int advance_t);
void launch_set_dt(const Launch& L, double dt);
void launch_zero_status(const Launch& L);
void launch_switch_count(const Launch& L);
// digital-filter inflow: device tables and state of one generator (host code builds the
// tables; see k_inflow.hip)
struct DFDev {
  int ny, nz, pad, nzmax;
  int nzh[3];           // half-width of the zeta filter per component
  const int* nyh;       // [3][ny] half-width of the eta filter per component and row
  const double* by;     // [3][ny][2 pad + 1] eta coefficients, centred at pad
  const double* bz;     // [3][2 nzmax + 1] zeta coefficients, centred at nzmax
  const double* a;      // [4][ny] a11, a21, a22, a33
  const double* mean;   // [4][ny] rho, U, V, T
  double Tc[3];         // Ix / U_ref
  double gm1, M2, U_ref, p;
  double* rz;           // [3][ny + 2 pad][nz] zeta-filtered numbers
  double* psi;          // [3][ny][nz] time-correlated field
};
void launch_df_update(const DFDev& D, const Prob* prob, const double* rnd, double* Q, double dt, int first,
                      hipStream_t s);
void launch_metrics(int ndim, const int N[3], const double* coords, double* scratch9, double* metrics,
                    hipStream_t s);
template <typename R> void launch_convert(const double* src, R* dst, size_t n, hipStream_t s);
// deviation of a 3D grid from planarity along zeta (see k_planar_dev); *out must be 0 first
void launch_planar_dev(int N0, int N1, int N2, int g, const double* M, const double* X, unsigned long long* out,
                       hipStream_t s);

int sweep_seg(const Launch& L, int d);   // segment length in effect for direction d

// z-marching launches (see zm_tile): planes per chunk and grid over the band [lo, hi)
inline int zm_chunk(const Launch& L, int lo, int hi) {
  if (L.zc > 0) return L.zc;
  long long e2 = L.ndim > 2 ? L.max_n[2] + hi - lo : 1;
  long long c = (e2 + 7) / 8;
  return (int)(c < 8 ? 8 : c);
}
inline dim3 zm_grid(const Launch& L, int lo, int hi, int TX, int TY) {
  long long e[3];
  for (int d = 0; d < 3; ++d) e[d] = d < L.ndim ? L.max_n[d] + hi - lo : 1;
  const int zc = zm_chunk(L, lo, hi);
  long long nblk = ((e[0] + TX - 1) / TX) * ((e[1] + TY - 1) / TY) * ((e[2] + zc - 1) / zc);
  return dim3((unsigned)(8 * ((nblk + 7) / 8)), L.nprob);
}
// tile width of the z-marching column kernels, their grid, and their zc argument (the
// chunk length with log2 of a non-default width above bit 16; see zm_column)
inline int zm_width(const Launch& L) { return L.ztx > 0 ? L.ztx : ZM_TX; }
inline dim3 zm_grid_col(const Launch& L, int lo, int hi) { return zm_grid(L, lo, hi, zm_width(L), 256 / zm_width(L)); }
inline int zm_arg(const Launch& L, int lo, int hi) {
  int lt = 0;
  if (L.ztx > 0 && L.ztx != ZM_TX)
    while ((1 << lt) < L.ztx) ++lt;
  return zm_chunk(L, lo, hi) | (lt << 16);
}

// gradients (region = 1: only where the per-cell hybrid needs C-GBR inputs)
template <typename R> void launch_grad_explicit(const Launch& L, int d, int order, int skip_if_any, int region);
template <typename R> void launch_grad_c4(const Launch& L, StateRef ref, int d, int skip_if_any, int region);
// C4 gradients of whole lines in LDS tiles (region-free launches; see tile_use), and along xi
// by the partition method (see c4_part_use)
template <typename R> void launch_grad_c4_tiles(const Launch& L, StateRef ref, int d, int skip_if_any, int dense_only);
template <typename R> void launch_grad_c4_part(const Launch& L, StateRef ref, int skip_if_any, int dense_only);
template <typename R> void launch_grad_c4_seg(const Launch& L, StateRef ref, int d, int skip_if_any, int dense_only);
// sensor and C-GBR viscous node fluxes
template <typename R> void launch_sensor(const Launch& L, int skip_if_any, int region);
template <typename R> void launch_gbr_viscflux(const Launch& L, int skip_if_any, int region);
// LAD: filtered coefficients; node fluxes; the grid factors Delta x_l once per context
// (cg = 1: gradients read from the gradient arrays instead of E4 from the primitives)
template <typename R> void launch_lad(const Launch& L, int skip_if_any, int cg = 0);
template <typename R> void launch_lad_nodeflux(const Launch& L, int skip_if_any, int cg = 0);
template <typename R> void launch_lad_geometry(const Launch& L);
// all-LAD interfaces of every direction in one pass; rr == nullptr writes the time
// derivative, else the RK stage combination (and the ghost copy of the stage result)
template <typename R>
void launch_lad_sweep(const Launch& L, StateRef ref, const RKRef* rr, int stage, double a, double b, int skip_if_any);
// interface sweeps
// rr != nullptr: this is the last direction and the sweep also forms the RK stage (and the
// ghost copy of the stage result)
template <typename R>
void launch_sweep(const Launch& L, StateRef ref, int d, int sel, int accumulate, int skip_if_any,
                  const RKRef* rr = nullptr, int stage = 0, double a = 0.0, double b = 0.0);
void launch_stage_ghosts(const Launch& L, const RKRef& rr, int stage, int skip_if_any);
// classic RK4 after stage s's right-hand side (in the derivative workspace): the sum
// acc += b dt k_s, and U^n + c dt k_s into the stage buffer (s < 3) or U^n + acc into U^n (s = 3)
void launch_rk4_combine(const Launch& L, double* Un, int stage, double b, double c);
// LAD-C6: compact sixth-order gradients of the primitives along d; compact interface
// fluxes along d differenced into dQ/dt (accumulate: add to what earlier directions
// wrote; rr != nullptr: this is the last direction and it forms the RK stage); one pass
// of the implicit filter along d on the state of ref (ghosts of d refilled first)
template <typename R> void launch_grad_c6(const Launch& L, StateRef ref, int d);
template <typename R>
void launch_c6_faces(const Launch& L, StateRef ref, int d, int accumulate, const RKRef* rr, int stage, double a,
                     double b);
enum { FILT_ALL = 0, FILT_GLOBAL = 1, FILT_PERCELL = 2 };
void launch_filter(const Launch& L, StateRef ref, int d, int mode);
// positivity guard of a hybrid stage's filter: the stage result saved before the passes,
// nodes the filter made non-physical restored after them
void launch_filter_save(const Launch& L, StateRef ref, int mode);
void launch_filter_guard(const Launch& L, StateRef ref, int mode);
// which kernel solves the lines of each system (shared by the host and the kernels):
// LDS line tiles when all five variables of one line fit the tile and a periodic line is
// long enough for the PCR steps; otherwise the policies below
enum { TK_GRAD6 = 0, TK_FACES = 1, TK_FILTER = 2, TK_GRAD4 = 3 };
constexpr int TILE_MASK_ALL = 0xFFF;
constexpr int TILE_MASK_FORCE_STRIDED = 0x1000;   // tiles on strided directions whatever their line count
constexpr int TILE_MASK_NO_PART = 0x2000;          // no partition-method kernels along xi (filter, MIG4 gradients)
constexpr int TILE_MASK_NO_SEG = 0x4000;           // no register-segment kernels along eta / zeta (filter, MIG4 gradients, LAD-C6 faces)
constexpr int TILE_MASK_DEFAULT = TILE_MASK_ALL;
constexpr int TILE_ELEMS = 6144;   // doubles per tile (48 KB of LDS)
// lanes per tile workgroup: contiguous lines take 512 (128 VGPRs, four waves per SIMD);
// strided tiles of long lines hold one or few columns, whose strided reads stay in L2 only
// while few workgroups are in flight: 256 lanes and no register cap
constexpr int TILE_THREADS_CONTIG = 512, TILE_THREADS_STRIDED = 256;
constexpr int TILE_MAX_TX = 16;
__host__ __device__ inline bool tile_ok(const Prob& P, int d, int kind) {
  const bool periodic = P.bc[d][0] == BC_PERIODIC;
  const int n = P.n[d];
  const int Lin = kind == TK_FACES ? n + 4 : P.N[d];
  if (5 * Lin > TILE_ELEMS) return false;
  const int steps = kind == TK_FILTER ? P.fsteps : LG_PCR_STEPS;   // TK_GRAD4: the C4 tables
  return !(periodic && n < (2 << steps));
}
// Where tiles are allowed (tile_mask), they are used for the contiguous direction, and for
// strided directions with few lines: strided lines solved one lane per line are coalesced
// across neighbouring lines and faster once there are enough of them to fill the chip
// (1024 x 384 x 128 ramp: 4.3 ms vs 11 ms for the C6 gradients along xi; along eta,
// 142 k lines, 2.5 ms one lane per line vs 4.4 ms in tiles; a 1792 x 768 plane has only
// 1802 eta lines, far too few lanes)
constexpr long long TILE_FEW_LINES = 32768;
// MIG4 gradients along xi on bounded lines of 128..2048 unknowns (the padded line less its
// two decoupled end rows): partition method (k_grad_c4_part) unless mask bit 13 turns it off
__host__ __device__ inline bool c4_part_use(const Prob& P, int d, int mask) {
  return !(mask & TILE_MASK_NO_PART) && d == 0 && P.bc[0][0] != BC_PERIODIC && P.N[0] - 2 >= 128 &&
         P.N[0] - 2 <= 2048;
}
// LAD-C6 interface fluxes along xi on bounded lines of 129..2049 nodes of 2D and 3D
// problems (the n - 1 interior faces): partition method (k_c6_faces_part) unless mask bit
// 13 turns it off
__host__ __device__ inline bool c6f_part_use(const Prob& P, int d, int mask) {
  return !(mask & TILE_MASK_NO_PART) && d == 0 && P.ndim > 1 && P.bc[0][0] != BC_PERIODIC && P.n[0] - 1 >= 128 &&
         P.n[0] - 1 <= 2048;
}
// LAD-C6 gradients along xi on bounded lines of 130..2050 nodes (the N - 2 unknowns between
// the decoupled end rows): partition method (k_grad_part) unless mask bit 13 turns it off
__host__ __device__ inline bool c6g_part_use(const Prob& P, int d, int mask) {
  return !(mask & TILE_MASK_NO_PART) && d == 0 && P.c6gz && P.bc[0][0] != BC_PERIODIC && P.N[0] - 2 >= 128 &&
         P.N[0] - 2 <= 2048;
}
__host__ __device__ inline bool tile_use(const Prob& P, int d, int kind, int mask) {
  if (!((mask >> (3 * kind + d)) & 1) || !tile_ok(P, d, kind)) return false;
  if (kind == TK_GRAD4 && c4_part_use(P, d, mask)) return false;
  if (kind == TK_FACES && c6f_part_use(P, d, mask)) return false;
  if (kind == TK_GRAD6 && c6g_part_use(P, d, mask)) return false;
  if (d == 0 || (mask & TILE_MASK_FORCE_STRIDED)) return true;
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const bool all_nodes = kind == TK_GRAD6 || kind == TK_GRAD4;
  const long long lines = all_nodes ? (long long)P.N[o1] * P.N[o2] : (long long)P.n[o1] * P.n[o2];
  return lines < TILE_FEW_LINES;
}
__host__ __device__ inline bool c6_grad_pcr(const Prob& P, int d) {
  const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
  const long long nlines = (long long)P.N[o1] * P.N[o2];
  const bool periodic = P.bc[d][0] == BC_PERIODIC;
  if (P.N[d] > 4096 || (periodic && P.n[d] < (2 << LG_PCR_STEPS))) return false;   // as the C4 solves
  return d == 0 || 5 * nlines < 131072;
}
__host__ __device__ inline bool c6_face_pcr(const Prob& P, int d) {
  const bool periodic = P.bc[d][0] == BC_PERIODIC;
  return d == 0 && P.ndim > 1 && P.n[d] <= 3990 && !(periodic && P.n[d] < (2 << LG_PCR_STEPS));
}
// the implicit filter along xi on bounded lines of 128..2048 unknowns: partition method
// (k_filter_part) unless mask bit 13 turns it off
__host__ __device__ inline bool filt_part_use(const Prob& P, int d, int mask) {
  return !(mask & TILE_MASK_NO_PART) && d == 0 && P.bc[0][0] != BC_PERIODIC && P.n[0] >= 128 && P.n[0] <= 2048;
}
__host__ __device__ inline bool filt_pcr(const Prob& P, int d) {
  const bool periodic = P.bc[d][0] == BC_PERIODIC;
  return d == 0 && P.N[d] <= 4000 && !(periodic && P.n[d] < (2 << P.fsteps));
}
// the implicit filter along eta / zeta where the lines would otherwise be solved one lane per
// line through FP64 scratch: k_filter_seg, segments of at most FSEG_LM unknowns held in
// registers, at most FSEG_SMAX per line (lines of 16 to 512 unknowns)
constexpr int FSEG_LM = 64, FSEG_SMAX = 8;
// host-built tables per direction: cp, 1 / pivot [LM + 1] each, u and v [2][LM + 1] each,
// the joint LU [2 SMAX][2 SMAX]
constexpr int FSEG_CP = 0, FSEG_INV = FSEG_LM + 1, FSEG_U = 2 * (FSEG_LM + 1), FSEG_V = 4 * (FSEG_LM + 1),
              FSEG_LU = 6 * (FSEG_LM + 1), FSEG_TABLE = FSEG_LU + 4 * FSEG_SMAX * FSEG_SMAX;
__host__ __device__ inline int fseg_count(int n) { return (n + FSEG_LM - 1) / FSEG_LM; }
__host__ __device__ inline bool filt_seg_use(const Prob& P, int d, int mask) {
  if ((mask & TILE_MASK_NO_SEG) || d == 0 || d >= P.ndim || !P.fsegt[d] || tile_use(P, d, TK_FILTER, mask))
    return false;
  const int S = fseg_count(P.n[d]);
  return S <= FSEG_SMAX && P.n[d] >= 16;
}
// MIG4 gradients along eta / zeta in register segments (k_grad_c4_seg, tables of the same
// layout for a = 1/4): bounded lines (their N - 2 unknowns between the decoupled end rows)
// and periodic lines (n interior unknowns) of 16 to 512 unknowns that the LDS tiles do not
// take, outside the listed lines of per-cell stages, unless mask bit 14 is set
__host__ __device__ inline int c4_seg_unknowns(const Prob& P, int d) {
  return P.bc[d][0] == BC_PERIODIC ? P.n[d] : P.N[d] - 2;
}
__host__ __device__ inline bool c4_seg_use(const Prob& P, int d, int mask) {
  if ((mask & TILE_MASK_NO_SEG) || d == 0 || d >= P.ndim || !P.c4segt[d] || tile_use(P, d, TK_GRAD4, mask))
    return false;
  const int m = c4_seg_unknowns(P, d);
  return fseg_count(m) <= FSEG_SMAX && m >= 16;
}
// LAD-C6 interface fluxes along eta / zeta in register segments (k_c6_faces_seg, tables of
// the same layout for a = 1/3): the n - 1 interior faces of a bounded line between its
// fourth-order boundary faces, or the n faces of a periodic line, 16 to 256 of them (at most
// four segments: with two waves per SIMD at the kernel's register count, two workgroups
// share a CU; six-segment workgroups, alone on their CU, were slower than one lane per line),
// where the LDS tiles do not take the direction, unless mask bit 14 is set
constexpr int C6FSEG_SMAX = 4;
__host__ __device__ inline int c6f_seg_unknowns(const Prob& P, int d) {
  return P.bc[d][0] == BC_PERIODIC ? P.n[d] : P.n[d] - 1;
}
// LAD-C6 gradients of periodic eta / zeta lines of 16 to 256 interior nodes in register
// segments (k_grad_c4_seg with the cyclic [1/3, 1, 1/3] tables), where the LDS tiles do not
// take the direction, unless mask bit 14 is set
__host__ __device__ inline bool c6g_seg_use(const Prob& P, int d, int mask) {
  if ((mask & TILE_MASK_NO_SEG) || d == 0 || d >= P.ndim || !P.c6gsegt[d] || P.bc[d][0] != BC_PERIODIC ||
      tile_use(P, d, TK_GRAD6, mask))
    return false;
  return fseg_count(P.n[d]) <= C6FSEG_SMAX && P.n[d] >= 16;
}
__host__ __device__ inline bool c6f_seg_use(const Prob& P, int d, int mask) {
  if ((mask & TILE_MASK_NO_SEG) || d == 0 || d >= P.ndim || !P.c6fsegt[d] || tile_use(P, d, TK_FACES, mask))
    return false;
  const int m = c6f_seg_unknowns(P, d);
  return fseg_count(m) <= C6FSEG_SMAX && m >= 16;
}

}  // namespace lg
