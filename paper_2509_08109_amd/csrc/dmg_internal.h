// Internal declarations shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dmg.h"

namespace dmg {

// ---- error reporting -------------------------------------------------------------------
dmg_status fail(dmg_status code, const char* fmt, ...);
void clear_error();

#define DMG_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::dmg::fail(DMG_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
  } while (0)

#define DMG_CHECK(expr)                      \
  do {                                       \
    dmg_status s_ = (expr);                  \
    if (s_ != DMG_OK) return s_;             \
  } while (0)

inline dmg_status launch_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(DMG_ERR_HIP, "launch of %s failed: %s", what, hipGetErrorString(e));
  return DMG_OK;
}

// ---- a bump allocator over the caller's workspace -------------------------------------
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  template <class T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    size_t bytes = count * sizeof(T);
    used = off + ((bytes + 255) & ~size_t(255));
    if (base == nullptr) return nullptr;  // sizing pass
    return reinterpret_cast<T*>(base + off);
  }
};

// Launch shape of the fused strip kernels on one level (bitwise neutral within one kernel
// family; the LDS and one-wavefront families round differently).
struct StripConfig {
  int bw = 128;     // columns (threads) per workgroup: 64, 128 or 256
  int seg_h = 32;   // rows per segment (even)
  int wave = 0;     // 1: one-wavefront strips with DPP lane exchange (bw = 64)
};

// ---- hierarchy ---------------------------------------------------------------------------
struct Level {
  StripConfig cfg;        // fused-kernel launch shape (levels above the tail), float64 pre sweeps
  StripConfig cfg32;      // the same for the float32 kernels
  StripConfig cfgp;       // ... and for the post sweeps (tuned separately)
  StripConfig cfgp32;
  int nx = 0, ny = 0;
  double* S = nullptr;    // [5][ny][nx]
  double* Sp = nullptr;   // [ny][nx][5] point-major copy of S read by the strip sweeps (levels
                          // above the tail, and level 0 always: the refinement residual)
  float* Sp32 = nullptr;  // its fp32 rounding for DMG_FP32_IR (levels above the tail)
  double* P = nullptr;    // [8][nyc][nxc] weights to the next coarser level (null at coarsest)
  double* u = nullptr;    // correction on coarse levels (level 0 uses the caller's array)
  double* t = nullptr;    // second iterate buffer for the out-of-place strip sweeps
  double* b = nullptr;    // right-hand side on coarse levels
  double* r = nullptr;    // residual scratch
  double* lf = nullptr;   // line relaxation (levels above the tail): [4][ny][nx] Thomas factors
                          // of the x-lines (super-diagonal, reciprocal pivot), then the y-lines
  float* lf32 = nullptr;  // its float32 counterpart (line relaxation with DMG_FP32_IR)
  float* S32 = nullptr;   // fp32 copies for DMG_FP32_IR (S32: tail levels, and every level
                          // with line relaxation)
  float* P32 = nullptr;
  float* u32 = nullptr;
  float* t32 = nullptr;
  float* b32 = nullptr;
  float* r32 = nullptr;
  size_t n() const { return size_t(nx) * size_t(ny); }
};

constexpr int kReduceBlocks = 1024;  // fixed partial count: reductions are order-deterministic
constexpr int kMaxPartials = 16384;  // capacity of the partials buffer
constexpr int kTailMaxN = 65;    // levels with max(nx, ny) <= this may run in the coarse tail
constexpr int kMaxTail = 12;     // at most this many levels in the coarse tail
constexpr int kSmallSetupN = 33;  // levels with max(nx, ny) <= this are set up in one workgroup
constexpr int kMaxLevels = 32;
constexpr int kDenseMax = 64;    // interior unknowns of a level whose sub-cycle is a dense matrix
constexpr int kGemvMax = 1024;   // ... applied inside the tail kernel; up to this many, by the
                                 // whole GPU in place of the tail kernel
constexpr int kMaxHistory = 4096;
constexpr int kChunk = 4;            // solve steps per host synchronisation

struct Graph {
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  const void* key_u = nullptr;
  const void* key_b = nullptr;
  hipStream_t stream = nullptr;
  int kind = -1;
  double rtol = -1.0;  // the solve start's arguments, for a graph that holds the start
  int max_iters = -1;
};

}  // namespace dmg

struct dmg_hier {
  dmg_options opts;
  std::vector<dmg::Level> L;
  int tail = 0;               // first level handled by the coarse-tail kernel
  int tail_threads = 1024;    // workgroup size of the coarse-tail kernel (tuned; no effect on
                              // the result)
  int m_coarse = 0;           // unknowns of the coarsest interior system
  int* coarse_idx = nullptr;  // [m] vertex index of each coarsest unknown
  double* chol = nullptr;     // [m][m] Cholesky factor (lower), float64
  double* partials = nullptr; // [kReduceBlocks] reduction partials
  double* scalars = nullptr;  // [16] device scalars (norms, IR scale)
  int* flag = nullptr;        // device ints: [0] pivot flag, [4..6] solve state (stop, steps, max),
                              // [8] initial iterate is zero
  double* hist = nullptr;     // device history of relative residuals [kMaxHistory]
  double* host = nullptr;     // pinned host scalars [16]
  // With a coarse tail below level 0: its levels' S, P and right-hand sides stored in one block
  // laid out as the tail kernel's LDS (iterate slots zero), which the kernel stages in one copy
  double* tail_img = nullptr;
  float* tail_img32 = nullptr;  // the same for the float32 tail (DMG_FP32_IR)
  int tail_img_n = 0;           // elements of each
  // The tail kernel holds levels [tail, tail + tail_nlev).  With tail_dense its last level (the
  // first with at most kDenseMax interior unknowns, tail_m of them) is solved by the dense
  // matrix `basis` (float32 copy basis32), the cycle from that level down applied exactly as
  // the linear map it is; the levels below it are then used only to compute that matrix.
  int tail_nlev = 0;
  int tail_m = 0;
  int tail_dense = 0;
  double* basis = nullptr;
  float* basis32 = nullptr;
  // gemv: the tail's top level (a coarse level with at most kGemvMax interior unknowns) is
  // solved by gbasis (row-major, float32 copy gbasis32), the exact linear map of the whole
  // cycle from that level down, in one matrix-vector product over the whole GPU instead of the
  // one-workgroup tail kernel; gscratch holds its columns while it is built
  int gemv = 0;
  double* gbasis = nullptr;
  float* gbasis32 = nullptr;
  double* gscratch = nullptr;
  dmg::Graph graph[dmg::kChunk];  // captured solve chunks of 1..kChunk steps
  dmg::Graph first_graph;         // the solve's start followed by its first kChunk steps
  // refresh: replayed as a captured graph from the second consecutive call with the same
  // stencil array and stream (the first of such a run goes eagerly: capture costs more than a
  // one-off setup)
  dmg::Graph setup_graph;
  const void* last_refresh_S = nullptr;
  const void* last_refresh_K = nullptr;  // refreshes from coefficients: (jac, K)
  hipStream_t last_refresh_stream = nullptr;
  ~dmg_hier();
};

namespace dmg {

// ---- kernels (launchers return DMG_OK or DMG_ERR_HIP) --------------------------------------
// S planar [5][ny][nx]; Sp (nullable) the same point-major [ny][nx][5]
dmg_status launch_assemble(const double* jac, const double* K, int nx, int ny, double* S,
                           hipStream_t s, double* Sp = nullptr);
dmg_status launch_interp_weights(const double* S, int nx, int ny, double* P, hipStream_t s);
// SHp (nullable): also write the coarse stencil point-major [nyc][nxc][5]
dmg_status launch_rap(const double* S, const double* P, int nx, int ny, double* SH,
                      double* SHp, hipStream_t s);
// Setup of levels small enough for one workgroup: level k = 0..nlev-1 of this list is
// (S[k] planar, Sp[k] point-major or null, P[k], nx[k], ny[k]); computes P[k] and S[k+1]
// (and Sp[k+1]) for k < nlev-1, then the Cholesky factor of the last level.
struct SmallSetup {
  double* S[kMaxTail + 1];
  double* Sp[kMaxTail + 1];
  double* P[kMaxTail + 1];
  int nx[kMaxTail + 1], ny[kMaxTail + 1];
  int nlev = 0;
  int m = 0;
  int* idx = nullptr;
  double* chol = nullptr;
  int* flag = nullptr;
};
dmg_status launch_setup_small(const SmallSetup& a, hipStream_t s);
// level 0: S (caller, planar) -> Sd (planar) and Sp (point-major, nullable)
dmg_status launch_copy_pack(const double* S, double* Sd, double* Sp, size_t n, hipStream_t s);
// point-major copy of a planar stencil: out[5 v + k] = T(S[k n + v])
template <class T>
dmg_status launch_pack(const double* S, T* out, size_t n, hipStream_t s);
dmg_status launch_cast(const double* in, float* out, size_t n, hipStream_t s);
// Float32 roundings of several arrays in one launch: plain copies (pack 0: dst[v] = src[v],
// v < n) and point-major packs of planar stencils (pack 1: dst[5 v + k] = src[k n + v]).
struct F32Seg {
  const double* src;
  float* dst;
  size_t n;
  int pack;
  int blocks;
};
constexpr int kMaxF32Segs = 48;
struct F32Batch {
  F32Seg seg[kMaxF32Segs];
  int count = 0;
  dmg_status add(const double* src, float* dst, size_t n, int pack);
};
dmg_status launch_f32_batch(const F32Batch& a, hipStream_t s);
dmg_status launch_grad_K(const double* jac, const double* lam, const double* u, int nx, int ny,
                         double* dK, hipStream_t s);

// u = B b on the interior of one coarse level (nx x ny, m = (nx-2)(ny-2) interior unknowns in
// row-major order, B row-major [m][m]), u = 0 on its boundary ring; a no-op once *stop is set.
template <class T>
struct DenseArgs {
  const T* B;
  const T* b;
  T* u;
  int nx, ny;
  const int* stop;
};
template <class T>
dmg_status launch_dense(const DenseArgs<T>& a, hipStream_t s);
// list: device array of count instances, each with at most max_m interior unknowns
template <class T>
dmg_status launch_dense_multi(const DenseArgs<T>* list, int count, int max_m, hipStream_t s);
dmg_status launch_transpose(const double* in, double* out, int n, hipStream_t s);

template <class T>
dmg_status launch_fill(T* x, T v, size_t n, hipStream_t s);
template <class T>
dmg_status launch_copy(const T* x, T* y, size_t n, const int* stop, hipStream_t s);

// ||b - A u||^2 partials (fixed block count) and sum(x^2) partials; finalize sums the
// partials in a fixed order into out[0] (and sqrt into out[1]).
// zero (nullable, with pb): device flag; when set, u is taken as zero and the partials are
// copied from the b-norm partials pb of launch_sq_partials / launch_start_norms (bitwise the
// partials the residual pass would form from u = 0).
dmg_status launch_resid_sq_partials(const double* S, const double* u, const double* b, int nx,
                                    int ny, double* partials, hipStream_t s,
                                    const int* stop = nullptr, const int* zero = nullptr,
                                    const double* pb = nullptr);
dmg_status launch_sq_partials(const double* x, size_t n, int nx, int ny, double* partials,
                              hipStream_t s);
// The b-norm partials of launch_sq_partials (pb, bitwise the same) and, from one read of u,
// *zero = 1 when every entry of u (boundary included) is zero, else 0; nonzero receives
// kReduceBlocks per-block counts.
dmg_status launch_start_norms(const double* b, const double* u, int nx, int ny, double* pb,
                              double* nonzero, int* zero, hipStream_t s);
dmg_status launch_finalize(const double* partials, double* out, hipStream_t s,
                           int count = kReduceBlocks);

// Kernel arguments of one strip sweep (one instance, one level).
template <class T>
struct StripArgs {
  const T* S;         // [ny][nx][5] point-major stencil (C, W, S, SW, SE of each point)
  const T* uin;       // [ny][nx] iterate before the sweep (pre: nullptr = zero)
  T* u;               // [ny][nx] iterate after the sweep (written)
  const T* b;         // [ny][nx]
  const T* P;         // [8][ncy][ncx] interpolation weights to the next coarser level
  T* bH;              // pre: [ncy][ncx] restricted residual (coarse right-hand side)
  const T* e;         // post: [ncy][ncx] coarse correction
  double* partials;   // post: squared-residual partial per workgroup (nullptr: none)
  int nx, ny;
  int seg_h;          // rows per segment (even)
  int nstrips, nsegs;
  int pf;             // row parity smoothed first
  int cA, cB;         // column parity smoothed first on A-rows / on B-rows
  const int* stop;    // nullable: when *stop != 0 the kernel does nothing (converged solve)
  double* x64;        // float post sweeps only (nullable): float64 iterate that receives the
                      // sweep's output, x += s u, at the points this workgroup writes
  const double* xscale;  // with x64: device address of the scale s (nullable: s = 1)
};

// Kernel arguments of the coarse tail (one instance).
template <class T>
struct TailLevel {
  const T* S;  // [5][ny][nx] planar (unused at the coarsest level)
  T* u;        // top level: iterate in/out; others unused
  const T* b;  // top level: right-hand side; others unused
  const T* P;  // [8][nyc][nxc] (unused at the coarsest level)
  int nx, ny;
};

template <class T>
struct TailArgs {
  TailLevel<T> L[kMaxTail];
  int oS[kMaxTail], ou[kMaxTail], ob[kMaxTail], oP[kMaxTail];  // LDS offsets, elements of T
  int o_r;            // LDS offset of the residual scratch, elements of T
  int o_y;            // LDS byte offset of the float64 coarsest-solve scratch
  int nlev;           // levels in the tail (the last one is the coarsest)
  int zero_top;       // the top level starts from u = 0 (it is a coarse level)
  int m;              // coarsest unknowns
  const int* idx;
  const double* chol;
  int pre[4], post[4];
  int nu_pre, nu_post;
  int smoother;       // 0: 4-colour point Gauss-Seidel; 1-3: zebra lines (x, y, alternating)
  const int* stop;
  const T* image;     // nullable: prepacked LDS image of the first image_n elements
  int image_n;
  int dense;          // the last level's solve is the dense matrix at LDS offset oB
  int oB;
  const T* Bg;        // that matrix in global memory (staged from here without an image)
  T* basis_out;       // basis run: [m0][m0] top-level interior results, one column per workgroup
  int unstaged;       // S, P and B read in global memory (no LDS copies: more workgroups per CU)
};

// fused strip kernels (fused_kernels.hip)
int strip_blocks(int nx, int ny, int bw, int seg_h, int* nstrips, int* nsegs);
// Out-of-place: u_in (pre: nullptr = zero) -> u_out, u_in != u_out.  S is the point-major
// [ny][nx][5] stencil copy.
// stop (nullable): device flag; the kernels do nothing once it is set (converged solves).
template <class T>
dmg_status launch_pre(const StripConfig& cfg, const T* S, const T* uin, T* u, const T* b,
                      const T* P, T* bH, int nx, int ny, int pf, int cA, int cB, const int* stop,
                      hipStream_t s);
template <class T>
dmg_status launch_post(const StripConfig& cfg, const T* S, const T* uin, T* u, const T* b,
                       const T* P, const T* e, double* partials, int nx, int ny, int pf, int cA,
                       int cB, const int* stop, hipStream_t s, double* x64 = nullptr,
                       const double* xscale = nullptr);
template <class T>
struct TailSpec {
  const T* S[kMaxTail];
  T* u[kMaxTail];
  T* b[kMaxTail];
  const T* P[kMaxTail];
  int nx[kMaxTail], ny[kMaxTail];
  int nlev = 0;
  int zero_top = 1;
  int m = 0;
  const int* idx = nullptr;
  const double* chol = nullptr;
  int pre[4], post[4];
  int nu_pre = 1, nu_post = 1;
  int smoother = 0;    // as dmg_options::smoother
  const int* stop = nullptr;
  int threads = 1024;  // workgroup size: a multiple of 64 in [64, 1024]
  // nullable: the first image_n elements of the kernel's LDS layout, prepacked in global memory
  // (S and P of the levels, zero iterates, the top right-hand side in its b slot); only with
  // zero_top, and b[0] must then be the image's top b slot
  const T* image = nullptr;
  int image_n = 0;
  // dense: the last level is solved by B (m = its interior count, transposed: B[j m + i] is
  // interior point i of the cycle's result for the j-th interior unit vector), the exact linear
  // map of the cycle from that level down, instead of by the Cholesky factor
  int dense = 0;
  const T* B = nullptr;
  // S, P and B are read where they are in global memory instead of being staged in LDS (the
  // kernel then needs only the iterates, right-hand sides and scratch in LDS)
  int unstaged = 0;
};
// LDS layout of the coarse-tail kernel for levels nx[0..nlev) (the last one the coarsest, with
// m unknowns): per level S [5 n] and P [8 n_next] (not at the coarsest), u [n], b [n]; then the
// residual scratch and the float64 coarsest-solve scratch.  Offsets in elements of `elem`
// bytes, except y (bytes).
struct TailLayout {
  int S[kMaxTail], u[kMaxTail], b[kMaxTail], P[kMaxTail];
  int B = 0;  // dense coarse operator [m][m] (empty unless dense)
  int r = 0;
  int y = 0;
  size_t bytes = 0;
};
TailLayout tail_layout(const int* nx, const int* ny, int nlev, int m, int elem, int dense,
                       int staged);
// The dense operator of a tail's top level: one workgroup per top-level interior unknown j runs
// the cycle (spec: no image, zero_top) on the j-th unit vector and writes the top level's
// interior result to out[j m0 ...] (column j of the operator).
dmg_status launch_tail_basis(const TailSpec<double>& spec, double* out, hipStream_t s);
// Kernel arguments of hierarchy h's coarse tail (api.hip), the top level's iterate and
// right-hand side at (u_top, b_top); the prepacked image is used when b_top is its top slot.
template <class T>
void tail_spec(const dmg_hier* h, T* u_top, const T* b_top, bool zero_top, const int* stop,
               TailSpec<T>* out);
int device_lds_limit();  // LDS bytes one workgroup may use on the current device
template <class T>
dmg_status launch_tail(const TailSpec<T>& spec, hipStream_t s);
// Fills the kernel arguments of one tail (and its LDS bytes) without launching.
template <class T>
dmg_status make_tail_args(const TailSpec<T>& spec, TailArgs<T>* out, size_t* lds_bytes);
// Multi-instance launches over device arrays of arguments (see k_tail_multi, k_wave_multi):
// the tails run one workgroup per instance with lds_bytes of LDS (the largest instance's);
// the wave sweeps (mode 1 pre, 2 post with prolongation, 3 post) cover count x tiles_per
// tiles, all instances of one level size and launch shape.
template <class T>
dmg_status launch_tail_multi(const TailArgs<T>* list, int count, size_t lds_bytes, int threads,
                             hipStream_t s);
template <class T>
dmg_status launch_wave_multi(const StripArgs<T>* list, int count, int tiles_per, int mode, int pf,
                             hipStream_t s);

// Sets a hierarchy's pre/post colour orders (4 colours each) and rebuilds what depends on them
// (the dense coarse operators); captured solve graphs are dropped.  Asynchronous on s.
dmg_status set_colour_orders(dmg_hier* h, const int32_t* pre, const int32_t* post, hipStream_t s);

// iterative refinement helpers (stop: nullable device flag, see launch_check_step)
// x += s e over n points, s = *scale (used when no float strip sweep carries the update)
dmg_status launch_ir_update(double* x, const float* e, size_t n, const double* scale,
                            hipStream_t s, const int* stop = nullptr);
// r = b - A x in float64 with A (point-major [ny][nx][5]) (zero on the boundary ring), plus one
// squared-norm partial per workgroup; ir_residual_blocks gives the number of partials written
int ir_residual_blocks(int nx, int ny);
// zero (nullable): device flag; when set, x is taken as zero and r = b is written without
// reading S or x (bitwise what the full pass gives for x = 0).
dmg_status launch_ir_residual(const double* S, const double* x, const double* b, double* r,
                              int nx, int ny, double* partials, hipStream_t s,
                              const int* stop = nullptr, const int* zero = nullptr);
// r32 = fl32(r / s) over n points, s = *norm (r32 = 0 where s = 0)
dmg_status launch_ir_scale(const double* r, float* r32, size_t n, const double* norm,
                           hipStream_t s, const int* stop = nullptr);
// Per-instance arguments of the batched convergence check (k_check on each instance) and of the
// batched start of a solve (norms of b and b - A u, solve state).
struct CheckArgs {
  const double* partials;  // squared-residual partials of the level-0 post sweep
  int count;               // number of partials
  double* out;             // [2] ||r||^2, ||r||
  const double* sc;        // sc[1] = ||b||, sc[6] = target^2
  int* st;                 // [3] stop, steps, max steps
  double* hist;            // relative residual history
  int hist_cap;
};
struct NormArgs {
  const double* S;  // planar [5][ny][nx] level-0 stencil
  const double* u;  // initial iterate (nullptr: zero)
  const double* b;
  int nx, ny;
  double* sc;       // instance scalars (see k_init_multi)
  int* st;          // [3] solve state
  double rtol;
  int max_iters;
  double* partials; // k_resid_multi output (instances whose cycle is all coarse tail)
};
dmg_status launch_check_multi(const CheckArgs* list, int count, hipStream_t s);
// Start of a solve on the device: sums the b-norm and residual-norm partials (fixed order) into
// sc_b[0..1] = ||b||^2, ||b|| and sc_r[0..1] = ||r||^2, ||r||, sets sc_b[6] = (rtol ||b||)^2,
// sc_b[7] = ||r|| (kept: later steps overwrite sc_r) and
// the state st = {stop, steps = 0, max}: stop when ||r|| <= rtol ||b||, max_iters <= 0, b = 0 or
// a norm is not finite.  When b = 0 it also zeroes u (n values).
dmg_status launch_solve_start(const double* pb, int nb, const double* pr, int nr, double* sc_b,
                              double* sc_r, int* st, double rtol, int max_iters, double* u,
                              size_t n, hipStream_t s);
dmg_status launch_norms_multi(const NormArgs* list, int count, int blocks_per, double* partials,
                              double* summary, hipStream_t s);
dmg_status launch_gather_multi(const CheckArgs* list, int count, double* rel, int* steps,
                               hipStream_t s);
dmg_status launch_resid_multi(const NormArgs* list, int count, int blocks_per, hipStream_t s);
// device-side convergence check of one solve step (see k_check)
dmg_status launch_check_step(const double* partials, int count, double* out, const double* sc,
                             int* st, double* hist, int hist_cap, hipStream_t s);

// y = A x for the planar stencil S [5][ny][nx] on interior rows (boundary ring of y set to 0;
// x is read at the boundary ring as the stencil's couplings there are zero)
dmg_status launch_stencil_apply(const double* S, const double* x, double* y, int nx, int ny,
                                hipStream_t s);

// Zebra line relaxation on the levels above the coarse tail (line_smoother.hip), in T = double
// (S, P, lf, r, b of the level) or T = float (their float32 copies S32, P32, lf32, r32, b32).
// Every kernel is a no-op once *stop (nullable) is set.
// The line sweeps of smoother 1-3 on level L (pre order, or reversed for the post sweep).
template <class T>
dmg_status line_sweep(const Level& L, T* u, const T* b, int smoother, bool pre, const int* stop,
                      hipStream_t s);
// The Thomas factors of every x-line and y-line of level L into L.lf / L.lf32 (at setup).
template <class T>
dmg_status line_factors(const Level& L, hipStream_t s);
// r = b - A u into the level's residual scratch, then the coarse right-hand side P^T r.
template <class T>
dmg_status line_resid_restrict(const Level& L, const Level& Lc, const T* u, const T* b,
                               const int* stop, hipStream_t s);
// u += P e.
template <class T>
dmg_status line_prolong(const Level& L, const T* e, T* u, const int* stop, hipStream_t s);

// One instance's arrays at one level for the batched line cycle (line_smoother.hip): planar
// stencil, line factors, weights to the next coarser level, iterate (in place), right-hand side,
// residual / sweep scratch, the coarse right-hand side written by the restriction, the coarse
// correction read by the interpolation, dims, and the instance's stop flag.
template <class T>
struct LineArgs {
  const T* S;
  const T* lf;
  const T* P;
  T* u;
  const T* b;
  T* r;
  T* bH;
  const T* e;
  int nx, ny;
  const int* stop;
};
enum class LineStep { kZero, kSweep, kResidual, kRestrict, kProlong };
// One step over `count` instances of one level size nx x ny (list in device memory); kSweep
// sweeps the lines of direction dir (0: x-lines, 1: y-lines) and the given parity.
dmg_status launch_line_multi(LineStep step, const LineArgs<double>* list, int count, int nx,
                             int ny, int dir, int parity, hipStream_t s);

// One float64 V-cycle of hierarchy h on level-0 arrays (u, b); u_zero: start from u = 0
// without reading u.  Every kernel is a no-op once *stop (nullable) is set.
dmg_status grid_vcycle(dmg_hier* h, double* u, const double* b, bool u_zero, const int* stop,
                       hipStream_t s);

}  // namespace dmg
