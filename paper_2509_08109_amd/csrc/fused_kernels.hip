// Fused, row-pipelined V-cycle kernels for large levels, and a one-workgroup kernel for the
// small coarse levels.
//
// Strip kernels.  A workgroup of BW threads owns BW consecutive columns (one per thread) of a
// vertical strip and walks down a segment of rows, holding a ring of rows of u, b, the five
// stencil planes and the residual in LDS.  Four-colour Gauss-Seidel (colour = (i&1) + 2(j&1))
// is pipelined by row parity: with "A" the row parity smoothed first, step t smooths A-row a
// (its two colours one after the other, from old values on the neighbouring B-rows), then
// B-row a-1 (from the new A-rows a-2 and a).  Every row is therefore read from HBM once and
// updated in the same colour order as a sweep over the whole grid, so the result is
// identical to four separate colour passes.  Behind the smoothing front the kernel forms
// residuals and (pre-smoothing) the restriction P^T r, or (post-smoothing) the squared
// residual partials.  Columns near the strip edges are recomputed by both neighbouring
// strips: only the middle BW - 2*HALO columns are written.
//
// Halo rows and columns of one workgroup are written by its neighbours, so the kernels work out
// of place: they read u_in and write u_out (the driver alternates two buffers per level).
//
//   pre  : u_out <- 4-colour sweep(u_in, b) [u_in = 0: not read]; b_H <- P^T (b - A u_out)
//   post : u_out <- 4-colour sweep(u_in + P e_H, b); optional partials of ||b - A u_out||^2
#include <type_traits>

#include "dmg_internal.h"

namespace dmg {
namespace {

constexpr int HALO = 6;   // columns recomputed on each side of a strip
constexpr int RU = 8;     // ring rows of u
constexpr int RS = 4;     // ring rows of S, b, r


// Ring slots are taken relative to base = (first A-row) - 1: row j lives in u slot
// (j - base) mod RU and in stencil/b/residual slot (j - base) mod RS.
constexpr int umod(int x) { return ((x % RU) + RU) % RU; }
constexpr int smod(int x) { return ((x % RS) + RS) % RS; }

// x + s e with the product rounded before the sum (no contraction): the float64 update of
// iterative refinement, x += s e.
__device__ __forceinline__ double add_scaled(double x, double s, double e) {
#pragma clang fp contract(off)
  const double p = s * e;
  return x + p;
}

// This thread's column of the ring rows, in registers (slots are compile-time constants).
template <class T>
struct ColRing {
  T u[RU];
  T s[5][RS];  // C, W, S, SW, SE
  T b[RS];
};

// LDS rings: u of every column and the couplings that neighbouring columns read
// (W of the right neighbour, SW of the upper-right and SE of the upper-left neighbour).
template <class T>
struct LdsRing {
  T* u;   // [RU][BW]
  T* W;   // [RS][BW]
  T* SW;  // [RS][BW]
  T* SE;  // [RS][BW]
  T* r;   // [RS][BW] residuals (pre)
};

// Off-diagonal part of row j of the operator applied to u, j given by its slots.
template <class T, int BW, int UM, int U0, int UP, int S0, int SP>
__device__ __forceinline__ T offdiag_r(const ColRing<T>& c, const LdsRing<T>& L, int tm, int tp) {
  const T sw = c.s[3][S0] * L.u[UM * BW + tm];
  const T s = c.s[2][S0] * c.u[UM];
  const T se = c.s[4][S0] * L.u[UM * BW + tp];
  const T w = c.s[1][S0] * L.u[U0 * BW + tm];
  const T e = L.W[S0 * BW + tp] * L.u[U0 * BW + tp];
  const T nw = L.SE[SP * BW + tm] * L.u[UP * BW + tm];
  const T n = c.s[2][SP] * c.u[UP];
  const T ne = L.SW[SP * BW + tp] * L.u[UP * BW + tp];
  return ((((((sw + s) + se) + w) + e) + nw) + n) + ne;
}

// Gauss-Seidel update of this thread's point on the row at relative index JR (interior only).
template <class T, int BW, int JR>
__device__ __forceinline__ void gs_col(ColRing<T>& c, const LdsRing<T>& L, int t, int tm, int tp,
                                       bool interior) {
  constexpr int U0 = umod(JR), UM = umod(JR - 1), UP = umod(JR + 1);
  constexpr int S0 = smod(JR), SP = smod(JR + 1);
  if (!interior) return;
  const T off = offdiag_r<T, BW, UM, U0, UP, S0, SP>(c, L, tm, tp);
  const T v = (c.b[S0] - off) / c.s[0][S0];
  c.u[U0] = v;
  L.u[U0 * BW + t] = v;
}

template <class T, int BW, int JR>
__device__ __forceinline__ T resid_col(const ColRing<T>& c, const LdsRing<T>& L, int tm, int tp,
                                       bool interior) {
  constexpr int U0 = umod(JR), UM = umod(JR - 1), UP = umod(JR + 1);
  constexpr int S0 = smod(JR), SP = smod(JR + 1);
  if (!interior) return T(0);
  const T off = offdiag_r<T, BW, UM, U0, UP, S0, SP>(c, L, tm, tp);
  return c.b[S0] - (off + c.s[0][S0] * c.u[U0]);
}

// Registers holding one prefetched row for this thread's column.
template <class T>
struct RowRegs {
  T u, b, s[5];
};

// Branch-free loads: every lane issues the same loads (out-of-range lanes read a clamped,
// valid address and discard the value), so the number of memory operations in flight is the
// same on every path and the compiler can wait for exactly the rows it consumes.
// UREAD: 0 the sweep starts from u = 0 (u is not read), 1 u is read from a.uin, 2 a.uin may be
// null (then u = 0; the load goes to b, which is read anyway).
template <class T, int UREAD>
__device__ __forceinline__ void load_row(const StripArgs<T>& a, int i, int j, RowRegs<T>& g) {
  const bool ok = i >= 0 && i < a.nx && j >= 0 && j < a.ny;
  const size_t v = ok ? size_t(j) * a.nx + i : 0;
  T s[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) s[k] = a.S[5 * v + k];
  const T bb = a.b[v];
  T uu = T(0);
  if constexpr (UREAD == 1) {
    uu = a.uin[v];
  } else if constexpr (UREAD == 2) {
    const T* src = a.uin ? a.uin : a.b;
    const T tu = src[v];
    uu = a.uin ? tu : T(0);
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) g.s[k] = ok ? s[k] : T(0);
  g.b = ok ? bb : T(0);
  g.u = ok ? uu : T(0);
}

template <class T, int BW, int JR>
__device__ __forceinline__ void store_row(ColRing<T>& c, const LdsRing<T>& L, int t,
                                          const RowRegs<T>& g) {
  constexpr int U0 = umod(JR), S0 = smod(JR);
  c.u[U0] = g.u;
  c.b[S0] = g.b;
#pragma unroll
  for (int k = 0; k < 5; ++k) c.s[k][S0] = g.s[k];
  L.u[U0 * BW + t] = g.u;
  L.W[S0 * BW + t] = g.s[1];
  L.SW[S0 * BW + t] = g.s[3];
  L.SE[S0 * BW + t] = g.s[4];
}

// (P e)(i, j) for interior fine point (i, j), read straight from global memory.
// The prolongation helpers below keep multiply and add separate (no FMA contraction): the
// first row of a segment is corrected by prolong_global and the others by the staged
// variants, and all must round identically for launch shapes to be bitwise neutral.
template <class T>
__device__ __forceinline__ T prolong_global(const StripArgs<T>& a, int i, int j) {
#pragma clang fp contract(off)
  const int ncx = (a.nx + 1) / 2, ncy = (a.ny + 1) / 2;
  const size_t NC = size_t(ncx) * ncy;
  const size_t c = size_t(j >> 1) * ncx + (i >> 1);
  const T* P = a.P;
  const T* e = a.e;
  if (!(i & 1) && !(j & 1)) return e[c];
  if ((i & 1) && !(j & 1)) return P[c] * e[c] + P[NC + c] * e[c + 1];
  if (!(i & 1) && (j & 1)) return P[2 * NC + c] * e[c] + P[3 * NC + c] * e[c + ncx];
  return ((P[4 * NC + c] * e[c] + P[5 * NC + c] * e[c + 1]) + P[6 * NC + c] * e[c + ncx]) +
         P[7 * NC + c] * e[c + ncx + 1];
}

// Coarse data of one row step of the post kernel (two fine rows, one of each parity), one
// coarse column per thread (threads t < CW): slot 0 e(J_even), 1-2 P0/P1(J_even),
// 3-4 e(J_odd), e(J_odd+1), 5-10 P2..P7(J_odd).
constexpr int kCoarseSlots = 11;

template <class T>
struct CoarseRegs {
  T v[kCoarseSlots];
};

template <class T>
__device__ __forceinline__ void load_coarse(const StripArgs<T>& a, int I, int r0,
                                            CoarseRegs<T>& c) {
  const int ncx = (a.nx + 1) / 2, ncy = (a.ny + 1) / 2;
  const int je = (r0 & 1) ? (r0 + 1) >> 1 : r0 >> 1;  // coarse row of the even fine row
  const int jo = r0 >> 1;                              // coarse row J of the odd fine row 2J+1
  const bool okI = I >= 0 && I < ncx;
  const bool oke = okI && je >= 0 && je < ncy;
  const bool oko = okI && jo >= 0 && jo < ncy;
  const bool oko1 = oko && jo + 1 < ncy;
  const size_t NC = size_t(ncx) * ncy;
  const size_t ce = oke ? size_t(je) * ncx + I : 0;
  const size_t co = oko ? size_t(jo) * ncx + I : 0;
  const size_t co1 = oko1 ? co + ncx : 0;
  const T* P = a.P;
  const T* e = a.e;
  T v[kCoarseSlots];
  v[0] = e[ce];
  v[1] = P[ce];
  v[2] = P[NC + ce];
  v[3] = e[co];
  v[4] = e[co1];
#pragma unroll
  for (int k = 0; k < 6; ++k) v[5 + k] = P[(2 + k) * NC + co];
  c.v[0] = oke ? v[0] : T(0);
  c.v[1] = oke ? v[1] : T(0);
  c.v[2] = oke ? v[2] : T(0);
  c.v[3] = oko ? v[3] : T(0);
  c.v[4] = oko1 ? v[4] : T(0);
#pragma unroll
  for (int k = 5; k < kCoarseSlots; ++k) c.v[k] = oko ? v[k] : T(0);
}

// (P e)(i, j) from the staged coarse rows; k = local coarse column of i.
template <class T>
__device__ __forceinline__ T prolong_lds(const T* cb, int cw, int k, int i, int j) {
#pragma clang fp contract(off)
  if (!(j & 1)) {
    const T* e = cb;
    if (!(i & 1)) return e[k];
    return cb[cw + k] * e[k] + cb[2 * cw + k] * e[k + 1];
  }
  const T* e0 = cb + 3 * cw;
  const T* e1 = cb + 4 * cw;
  const T* Pq = cb + 5 * cw;  // P2..P7
  if (!(i & 1)) return Pq[k] * e0[k] + Pq[cw + k] * e1[k];
  return ((Pq[2 * cw + k] * e0[k] + Pq[3 * cw + k] * e0[k + 1]) + Pq[4 * cw + k] * e1[k]) +
         Pq[5 * cw + k] * e1[k + 1];
}

__device__ __forceinline__ double block_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double ws[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();  // earlier readers of ws (a previous call) are done
  if (lane == 0) ws[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < int(blockDim.x >> 6); ++k) t += ws[k];
  return t;
}

template <int BW>
constexpr int coarse_width() { return BW / 2 + 2; }

template <int BW>
constexpr int strip_lds_elems(bool post) {
  return (RU + 4 * RS) * BW + (post ? 2 * kCoarseSlots * coarse_width<BW>() : 0);
}

// MODE: 0 pre from u = 0, 1 pre from u_in, 2 post with prolongation, 3 post without.
template <class T, int BW, int MODE>
__global__ __launch_bounds__(BW) void k_strip(StripArgs<T> a) {
  constexpr bool POST = MODE >= 2;
  constexpr int UREAD = MODE != 0 ? 1 : 0;
  constexpr bool prol = MODE == 2;
  // the stop flag is tested only after the first rows' loads are issued, so that its memory
  // latency overlaps theirs (a converged solve's kernels still exit before any write)
  const int stopped = a.stop ? *a.stop : 0;
  extern __shared__ __align__(16) unsigned char smem[];
  T* base_l = reinterpret_cast<T*>(smem);
  LdsRing<T> L{base_l, base_l + RU * BW, base_l + (RU + RS) * BW, base_l + (RU + 2 * RS) * BW,
               base_l + (RU + 3 * RS) * BW};
  constexpr int CW = coarse_width<BW>();
  T* cbuf = base_l + (RU + 4 * RS) * BW;  // post: 2 x kCoarseSlots x CW staged coarse rows

  // XCD-aware tile order: the hardware hands workgroup ids to the 8 XCDs round-robin, so
  // give each XCD a contiguous run of tiles (adjacent strips and segments share halos in
  // that XCD's L2).
  const int ntiles = a.nstrips * a.nsegs;
  const int per = (int(gridDim.x) + 7) >> 3;
  const int tile = (int(blockIdx.x) & 7) * per + (int(blockIdx.x) >> 3);
  const bool active = tile < ntiles;
  const int seg = active ? tile / a.nstrips : 0;
  const int strip = active ? tile % a.nstrips : 0;

  const int t = threadIdx.x;
  const int tm = t > 0 ? t - 1 : 0, tp = t < BW - 1 ? t + 1 : BW - 1;
  const int out_w = BW - 2 * HALO;
  const int x0 = strip * out_w;
  const int i = x0 - HALO + t;
  const int cI = ((x0 - HALO) >> 1) + t;  // coarse column staged by thread t (t < CW)
  const int j0 = seg * a.seg_h;
  const int j1 = min(j0 + a.seg_h, a.ny);
  // first A-row: the largest row of parity pf not after j0-2 (pre) / j0-1 (post)
  const int lim = POST ? j0 - 1 : j0 - 2;
  const int a0 = lim - (((lim - a.pf) % 2) + 2) % 2;
  // last A-row: residual rows up to j1-1 must be complete -> front a >= j1
  const int alast = j1 + (((j1 - a.pf) % 2) + 2) % 2;
  // rows past alast + 1 are never consumed: their prefetch slots read row -1, which the
  // loader maps to a fixed, cached address instead of streaming unused rows from memory
  auto live = [&](int r) { return r <= alast + 1 ? r : -1; };
  const double xs = (POST && a.x64 && a.xscale) ? *a.xscale : 1.0;
  auto emit = [&](size_t v, T val) {
    a.u[v] = val;
    if constexpr (POST && std::is_same<T, float>::value)
      if (a.x64) a.x64[v] = add_scaled(a.x64[v], xs, double(val));
  };
  const int base = a0 - 1;
  const bool interior_i = i >= 1 && i <= a.nx - 2;
  const bool out_col = active && t >= HALO && t < BW - HALO && i < a.nx;
  const int ncx = (a.nx + 1) / 2, ncy = (a.ny + 1) / 2;
  auto row_ok = [&](int j) { return interior_i && j >= 1 && j <= a.ny - 2; };

  ColRing<T> c;
#pragma unroll
  for (int k = 0; k < RU; ++k) c.u[k] = T(0);
#pragma unroll
  for (int k = 0; k < RS; ++k) {
    c.b[k] = T(0);
#pragma unroll
    for (int q = 0; q < 5; ++q) c.s[q][k] = T(0);
  }
  for (int k = t; k < (RU + 4 * RS) * BW; k += BW) base_l[k] = T(0);
  RowRegs<T> gM, gA0, gA1, gB0, gB1;
  CoarseRegs<T> cr;
  T pm = T(0);
  if (active) {  // every load of the prologue, then their uses
    load_row<T, UREAD>(a, i, a0 - 1, gM);
    if (prol && row_ok(a0 - 1)) pm = prolong_global<T>(a, i, a0 - 1);
    if (prol) load_coarse<T>(a, cI, a0, cr);
    load_row<T, UREAD>(a, i, a0, gA0);
    load_row<T, UREAD>(a, i, a0 + 1, gA1);
    load_row<T, UREAD>(a, i, live(a0 + 2), gB0);
    load_row<T, UREAD>(a, i, live(a0 + 3), gB1);
  }
  __syncthreads();  // the LDS rings are zero before any row is stored
  if (stopped) return;  // the same for every thread of the workgroup
  if (active) {
    if (prol && row_ok(a0 - 1)) gM.u = gM.u + pm;
    store_row<T, BW, 0>(c, L, t, gM);
    if (prol && t < CW) {
#pragma unroll
      for (int k = 0; k < kCoarseSlots; ++k) cbuf[k * CW + t] = cr.v[k];
    }
  }
  __syncthreads();
  double acc = 0.0;

  // One row step with ar = base + 1 + 2K (mod the ring period): smooth A-row ar and B-row
  // ar-1 from the rows in (g0, g1), then prefetch the rows two steps ahead into (g0, g1).
  auto step = [&](auto KC, int ar, RowRegs<T>& g0, RowRegs<T>& g1) {
    constexpr int K = decltype(KC)::value;
    constexpr int JA = 1 + 2 * K;  // relative index of A-row ar
    if (prol) {
      const T* cb = cbuf + (K & 1) * kCoarseSlots * CW;
      const int kk = t >> 1;
      if (row_ok(ar)) g0.u = g0.u + prolong_lds<T>(cb, CW, kk, i, ar);
      if (row_ok(ar + 1)) g1.u = g1.u + prolong_lds<T>(cb, CW, kk, i, ar + 1);
    }
    store_row<T, BW, JA>(c, L, t, g0);
    store_row<T, BW, JA + 1>(c, L, t, g1);
    __syncthreads();
    // loads consumed at the end of this step first (vector memory returns in issue order),
    // then the rows of the step after next
    if (prol) load_coarse<T>(a, cI, ar + 2, cr);
    const int fj = (ar - 2) & ~1;  // fine row 2J of the coarse row restricted in this step
    const int J = fj >> 1;
    const int I = i >> 1;
    const bool do_restrict = !POST && out_col && !(i & 1) && fj >= j0 && fj < j1;
    const bool inner_c = I >= 1 && I <= ncx - 2 && J >= 1 && J <= ncy - 2;
    T pw[8];
    if (!POST) {
      const size_t NC = size_t(ncx) * ncy;
      const size_t cc = (do_restrict && inner_c) ? size_t(J) * ncx + I : size_t(ncx) + 1;
      const T* P = a.P;
      pw[0] = P[7 * NC + cc - ncx - 1];
      pw[1] = P[3 * NC + cc - ncx];
      pw[2] = P[6 * NC + cc - ncx];
      pw[3] = P[1 * NC + cc - 1];
      pw[4] = P[0 * NC + cc];
      pw[5] = P[5 * NC + cc - 1];
      pw[6] = P[2 * NC + cc];
      pw[7] = P[4 * NC + cc];
    }
    load_row<T, UREAD>(a, i, live(ar + 4), g0);
    load_row<T, UREAD>(a, i, live(ar + 5), g1);
    // A-row ar: column parity cA first, then the other; then B-row ar-1
    const bool okA = row_ok(ar), okB = row_ok(ar - 1);
    const bool firstA = (i & 1) == a.cA, firstB = (i & 1) == a.cB;
    gs_col<T, BW, JA>(c, L, t, tm, tp, okA && firstA);
    __syncthreads();
    gs_col<T, BW, JA>(c, L, t, tm, tp, okA && !firstA);
    __syncthreads();
    gs_col<T, BW, JA - 1>(c, L, t, tm, tp, okB && firstB);
    __syncthreads();
    gs_col<T, BW, JA - 1>(c, L, t, tm, tp, okB && !firstB);
    __syncthreads();
    // rows ar-1 and ar are final: write them out
    if (out_col) {
      if (ar - 1 >= j0 && ar - 1 < j1) emit(size_t(ar - 1) * a.nx + i, c.u[umod(JA - 1)]);
      if (ar >= j0 && ar < j1) emit(size_t(ar) * a.nx + i, c.u[umod(JA)]);
    }
    // residual rows ar-2 and ar-1
    const T r2 = resid_col<T, BW, JA - 2>(c, L, tm, tp, row_ok(ar - 2));
    const T r1 = resid_col<T, BW, JA - 1>(c, L, tm, tp, okB);
    if (POST) {
      if (out_col && a.partials) {
        if (ar - 2 >= j0 && ar - 2 < j1) acc += double(r2) * double(r2);
        if (ar - 1 >= j0 && ar - 1 < j1) acc += double(r1) * double(r1);
      }
      if (prol && t < CW) {  // stage the next step's coarse rows
        T* cbn = cbuf + ((K + 1) & 1) * kCoarseSlots * CW;
#pragma unroll
        for (int k = 0; k < kCoarseSlots; ++k) cbn[k * CW + t] = cr.v[k];
      }
    } else {
      L.r[smod(JA - 2) * BW + t] = r2;
      L.r[smod(JA - 1) * BW + t] = r1;
      __syncthreads();
      // restriction for the coarse row whose fine rows 2J-1..2J+1 are now complete
      if (do_restrict) {
        T acc2 = T(0);
        if (inner_c) {
          const int rel = fj - base;  // relative index of fine row 2J
          const T* rm = L.r + smod(rel - 1) * BW;
          const T* r0 = L.r + smod(rel) * BW;
          const T* rp = L.r + smod(rel + 1) * BW;
          acc2 = pw[0] * rm[t - 1];
          acc2 += pw[1] * rm[t];
          acc2 += pw[2] * rm[t + 1];
          acc2 += pw[3] * r0[t - 1];
          acc2 += r0[t];
          acc2 += pw[4] * r0[t + 1];
          acc2 += pw[5] * rp[t - 1];
          acc2 += pw[6] * rp[t];
          acc2 += pw[7] * rp[t + 1];
        }
        if (J < ncy) a.bH[size_t(J) * ncx + I] = acc2;
      }
    }
    __syncthreads();
  };

  // steps k = 0, 1, 2, ...: ring slots repeat every 4 steps and the prefetch registers
  // alternate, so the period is unrolled straight-line (uniform early exits)
  for (int ar = a0; active && ar <= alast; ar += 8) {
    step(std::integral_constant<int, 0>{}, ar, gA0, gA1);
    if (ar + 2 > alast) break;
    step(std::integral_constant<int, 1>{}, ar + 2, gB0, gB1);
    if (ar + 4 > alast) break;
    step(std::integral_constant<int, 2>{}, ar + 4, gA0, gA1);
    if (ar + 6 > alast) break;
    step(std::integral_constant<int, 3>{}, ar + 6, gB0, gB1);
  }
  if (POST && a.partials) {
    const double sacc = block_sum(acc);
    if (t == 0) a.partials[blockIdx.x] = sacc;
  }
}

// -----------------------------------------------------------------------------------------
// Coarse tail: one workgroup runs the V-cycle from level `top` down to the coarsest level and
// back, entirely in LDS.  It stages the stencils and weights of its levels and the top level's
// right-hand side (and iterate) once per cycle, separates the colour passes with workgroup
// barriers, and writes back only the top level's iterate, which is all the levels above read.
// -----------------------------------------------------------------------------------------

template <class T>
__device__ __forceinline__ T offdiag_s(const T* S, const T* u, int N, int nx, int v) {
  const T sw = S[3 * N + v] * u[v - nx - 1];
  const T s = S[2 * N + v] * u[v - nx];
  const T se = S[4 * N + v] * u[v - nx + 1];
  const T w = S[N + v] * u[v - 1];
  const T e = S[N + v + 1] * u[v + 1];
  const T nw = S[4 * N + v + nx - 1] * u[v + nx - 1];
  const T n = S[2 * N + v + nx] * u[v + nx];
  const T ne = S[3 * N + v + nx + 1] * u[v + nx + 1];
  return ((((((sw + s) + se) + w) + e) + nw) + n) + ne;
}

template <class T>
__device__ void tail_colour(const T* S, T* u, const T* b, int nx, int ny, int c) {
  const int ci = c & 1, cj = c >> 1;
  const int px = (nx - ci + 1) / 2, py = (ny - cj + 1) / 2;
  const int N = nx * ny;
  for (int k = threadIdx.x; k < px * py; k += blockDim.x) {
    const int i = ci + 2 * (k % px), j = cj + 2 * (k / px);
    if (i <= 0 || i >= nx - 1 || j <= 0 || j >= ny - 1) continue;
    const int v = j * nx + i;
    u[v] = (b[v] - offdiag_s(S, u, N, nx, v)) / S[v];
  }
  __syncthreads();
}

// One zebra line sweep in LDS: dir 0 x-lines (rows), 1 y-lines (columns), interior lines of
// one parity, one thread per line by the Thomas algorithm (modified super-diagonal in cp).
template <class T>
__device__ void tail_line(const T* S, T* u, const T* b, T* cp, int nx, int ny, int dir,
                          int parity) {
  const int N = nx * ny;
  const T *C = S, *W = S + N, *So = S + 2 * N, *SW = S + 3 * N, *SE = S + 4 * N;
  const int first = parity == 0 ? 2 : 1;
  const int len = dir == 0 ? nx : ny;       // points along a line, boundary included
  const int step = dir == 0 ? 1 : nx;       // index step along a line
  const int count = dir == 0 ? ny : nx;
  for (int t = threadIdx.x; first + 2 * t <= count - 2; t += blockDim.x) {
    const int line = first + 2 * t;
    const int v0 = dir == 0 ? line * nx : line;
    T pc = T(0), pd = T(0);
    for (int k = 1; k <= len - 2; ++k) {
      const int v = v0 + k * step;
      T off, a, c;
      if (dir == 0) {
        off = ((((So[v] * u[v - nx] + So[v + nx] * u[v + nx]) + SW[v] * u[v - nx - 1]) +
                SE[v] * u[v - nx + 1]) +
               SE[v + nx - 1] * u[v + nx - 1]) +
              SW[v + nx + 1] * u[v + nx + 1];
        a = W[v];
        c = W[v + 1];
      } else {
        off = ((((W[v] * u[v - 1] + W[v + 1] * u[v + 1]) + SW[v] * u[v - nx - 1]) +
                SE[v] * u[v - nx + 1]) +
               SE[v + nx - 1] * u[v + nx - 1]) +
              SW[v + nx + 1] * u[v + nx + 1];
        a = So[v];
        c = So[v + nx];
      }
      const T im = T(1) / (C[v] - a * pc);  // one division per step
      pc = c * im;
      pd = ((b[v] - off) - a * pd) * im;
      cp[v] = pc;
      u[v] = pd;
    }
    for (int k = len - 3; k >= 1; --k) {
      const int v = v0 + k * step;
      u[v] = u[v] - cp[v] * u[v + step];
    }
  }
  __syncthreads();
}

// One smoothing sweep of the tail (pre: the pre order, else the post order / reversed lines).
template <class T>
__device__ void tail_smooth(const TailArgs<T>& a, const T* S, T* u, const T* b, T* cp, int nx,
                            int ny, bool pre) {
  if (a.smoother == 0) {
    for (int c = 0; c < 4; ++c) tail_colour(S, u, b, nx, ny, pre ? a.pre[c] : a.post[c]);
    return;
  }
  int dir[4], par[4], n = 0;
  if (a.smoother == 1 || a.smoother == 3) {
    dir[n] = 0, par[n++] = 0;
    dir[n] = 0, par[n++] = 1;
  }
  if (a.smoother == 2 || a.smoother == 3) {
    dir[n] = 1, par[n++] = 0;
    dir[n] = 1, par[n++] = 1;
  }
  for (int k = 0; k < n; ++k) {
    const int q = pre ? k : n - 1 - k;
    tail_line(S, u, b, cp, nx, ny, dir[q], par[q]);
  }
}

// Copies n elements from global src to LDS dst (both 16-byte aligned) in 16-byte words; each
// thread issues all loads of a round before its stores, so a round costs one memory latency.
template <class T>
__device__ __forceinline__ void stage_lds(T* dst, const T* src, int n, int tid, int nt) {
  constexpr int K = 8;
  const int nv = int((size_t(n) * sizeof(T)) / 16);
  // a native vector type: the HIP vector struct kept the array on the stack in some callers
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const u32x4* s4 = reinterpret_cast<const u32x4*>(src);
  u32x4* d4 = reinterpret_cast<u32x4*>(dst);
  for (int base = tid; base < nv; base += K * nt) {
    u32x4 v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int q = base + k * nt;
      v[k] = s4[q < nv ? q : 0];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int q = base + k * nt;
      if (q < nv) d4[q] = v[k];
    }
  }
  for (int k = int(size_t(nv) * 16 / sizeof(T)) + tid; k < n; k += nt) dst[k] = src[k];
}

// U: S, P and the dense operator are read in global memory (a.unstaged), not staged in LDS.
template <class T, bool U>
__device__ __forceinline__ void tail_body(const TailArgs<T>& a) {
  // the stop flag is tested after the staging loads are issued (their latencies overlap)
  const int stopped = a.stop ? *a.stop : 0;
  extern __shared__ __align__(16) unsigned char smem[];
  T* sm = reinterpret_cast<T*>(smem);
  const int nl = a.nlev, tid = threadIdx.x, nt = blockDim.x;
  // stage the level data: the prepacked image in one copy, else array by array
  if (a.image) stage_lds(sm, a.image, a.image_n, tid, nt);
  // basis run (workgroup j): the top right-hand side is the j-th interior unit vector
  const int vj = a.basis_out ? (int(blockIdx.x) / (a.L[0].nx - 2) + 1) * a.L[0].nx +
                                   int(blockIdx.x) % (a.L[0].nx - 2) + 1
                             : -1;
  if (a.dense && !a.image && !U)
    for (int k = tid; k < a.m * a.m; k += nt) sm[a.oB + k] = a.Bg[k];
  // S, P and B in LDS, or (U) read where they are in global memory
  auto Sl = [&](int l) -> const T* {
    if constexpr (U) return a.L[l].S;
    else return sm + a.oS[l];
  };
  auto Pl = [&](int l) -> const T* {
    if constexpr (U) return a.L[l].P;
    else return sm + a.oP[l];
  };
  for (int l = 0; l < nl && !a.image; ++l) {
    const TailLevel<T>& G = a.L[l];
    const int n = G.nx * G.ny;
    T* u = sm + a.ou[l];
    if (l + 1 < nl && !U) {
      const int nc = a.L[l + 1].nx * a.L[l + 1].ny;
      T* S = sm + a.oS[l];
      T* P = sm + a.oP[l];
      for (int k = tid; k < 5 * n; k += nt) S[k] = G.S[k];
      for (int k = tid; k < 8 * nc; k += nt) P[k] = G.P[k];
    }
    if (l == 0) {
      T* b = sm + a.ob[l];
      for (int k = tid; k < n; k += nt) {
        b[k] = a.basis_out ? T(k == vj ? 1 : 0) : G.b[k];
        u[k] = a.zero_top ? T(0) : G.u[k];
      }
    } else {
      for (int k = tid; k < n; k += nt) u[k] = T(0);  // b_l is written by the restriction
    }
  }
  __syncthreads();
  if (stopped) return;  // the same for the whole workgroup
  T* r = sm + a.o_r;
  for (int l = 0; l + 1 < nl; ++l) {
    const int nx = a.L[l].nx, ny = a.L[l].ny, N = nx * ny;
    const T* S = Sl(l);
    T* u = sm + a.ou[l];
    const T* b = sm + a.ob[l];
    for (int s = 0; s < a.nu_pre; ++s) tail_smooth(a, S, u, b, r, nx, ny, true);
    for (int v = tid; v < N; v += nt) {
      const int i = v % nx, j = v / nx;
      T rv = T(0);
      if (i > 0 && i < nx - 1 && j > 0 && j < ny - 1)
        rv = b[v] - (offdiag_s(S, u, N, nx, v) + S[v] * u[v]);
      r[v] = rv;
    }
    __syncthreads();
    const int ncx = a.L[l + 1].nx, ncy = a.L[l + 1].ny, NC = ncx * ncy;
    const T* P = Pl(l);
    T* bH = sm + a.ob[l + 1];
    for (int c = tid; c < NC; c += nt) {
      const int I = c % ncx, J = c / ncx;
      T acc = T(0);
      if (I > 0 && I < ncx - 1 && J > 0 && J < ncy - 1) {
        const int f = 2 * J * nx + 2 * I;
        acc = P[7 * NC + c - ncx - 1] * r[f - nx - 1];
        acc += P[3 * NC + c - ncx] * r[f - nx];
        acc += P[6 * NC + c - ncx] * r[f - nx + 1];
        acc += P[1 * NC + c - 1] * r[f - 1];
        acc += r[f];
        acc += P[0 * NC + c] * r[f + 1];
        acc += P[5 * NC + c - 1] * r[f + nx - 1];
        acc += P[2 * NC + c] * r[f + nx];
        acc += P[4 * NC + c] * r[f + nx + 1];
      }
      bH[c] = acc;
    }
    __syncthreads();
  }
  if (a.dense) {
    // last level: its precomputed dense operator B (transposed, [j][i]) on the interior, the
    // exact linear map of the cycle from this level down; on a top level that carries an
    // iterate (u != 0) the cycle is u + B (b - A u)
    const int cx = a.L[nl - 1].nx, cy = a.L[nl - 1].ny, mx = cx - 2, m = a.m, N = cx * cy;
    T* uc = sm + a.ou[nl - 1];
    const T* bc = sm + a.ob[nl - 1];
    const T* B = U ? a.Bg : sm + a.oB;
    const bool corr = nl == 1 && !a.zero_top;
    T* rr = sm + a.o_r;
    if (corr) {  // this level's stencil is not staged: read it from global memory
      const T* Sg = a.L[nl - 1].S;
      for (int v = tid; v < N; v += nt) {
        const int i = v % cx, j = v / cx;
        T rv = T(0);
        if (i > 0 && i < cx - 1 && j > 0 && j < cy - 1)
          rv = bc[v] - (offdiag_s(Sg, uc, N, cx, v) + Sg[v] * uc[v]);
        rr[v] = rv;
      }
      __syncthreads();
    }
    const T* rhs = corr ? rr : bc;
    for (int i = tid; i < m; i += nt) {
      T acc = T(0);
      int j = 0;
      for (int jy = 1; jy < cy - 1; ++jy)
        for (int jx = 1; jx < cx - 1; ++jx, ++j) acc += B[j * m + i] * rhs[jy * cx + jx];
      const int v = (i / mx + 1) * cx + i % mx + 1;
      uc[v] = corr ? uc[v] + acc : acc;
    }
    __syncthreads();
  } else {
    // coarsest: dense Cholesky solve in float64
    T* uc = sm + a.ou[nl - 1];
    const T* bc = sm + a.ob[nl - 1];
    double* y = reinterpret_cast<double*>(smem + a.o_y);
    const int m = a.m;
    const double* L = a.chol;
    const int ncn = a.L[nl - 1].nx * a.L[nl - 1].ny;
    for (int k = tid; k < m; k += nt) y[k] = double(bc[a.idx[k]]);
    for (int k = tid; k < ncn; k += nt) uc[k] = T(0);  // the direct solve ignores the guess
    __syncthreads();
    for (int k = 0; k < m; ++k) {
      if (tid == 0) y[k] /= L[k * m + k];
      __syncthreads();
      for (int q = k + 1 + tid; q < m; q += nt) y[q] -= L[q * m + k] * y[k];
      __syncthreads();
    }
    for (int k = m - 1; k >= 0; --k) {
      if (tid == 0) y[k] /= L[k * m + k];
      __syncthreads();
      for (int q = tid; q < k; q += nt) y[q] -= L[k * m + q] * y[k];
      __syncthreads();
    }
    for (int k = tid; k < m; k += nt) uc[a.idx[k]] = T(y[k]);
    __syncthreads();
  }
  for (int l = nl - 2; l >= 0; --l) {
    const int nx = a.L[l].nx, ny = a.L[l].ny, N = nx * ny;
    const int ncx = a.L[l + 1].nx, ncy = a.L[l + 1].ny, NC = ncx * ncy;
    const T* S = Sl(l);
    const T* P = Pl(l);
    const T* e = sm + a.ou[l + 1];
    T* u = sm + a.ou[l];
    const T* b = sm + a.ob[l];
    for (int v = tid; v < N; v += nt) {
      const int i = v % nx, j = v / nx;
      if (i <= 0 || i >= nx - 1 || j <= 0 || j >= ny - 1) continue;
      const int c = (j >> 1) * ncx + (i >> 1);
      T corr;
      if (!(i & 1) && !(j & 1)) {
        corr = e[c];
      } else if ((i & 1) && !(j & 1)) {
        corr = P[c] * e[c] + P[NC + c] * e[c + 1];
      } else if (!(i & 1) && (j & 1)) {
        corr = P[2 * NC + c] * e[c] + P[3 * NC + c] * e[c + ncx];
      } else {
        corr = ((P[4 * NC + c] * e[c] + P[5 * NC + c] * e[c + 1]) + P[6 * NC + c] * e[c + ncx]) +
               P[7 * NC + c] * e[c + ncx + 1];
      }
      u[v] = u[v] + corr;
    }
    __syncthreads();
    for (int s = 0; s < a.nu_post; ++s) tail_smooth(a, S, u, b, sm + a.o_r, nx, ny, false);
  }
  // write back the top level's iterate (basis run: its interior as column blockIdx.x)
  {
    const TailLevel<T>& G = a.L[0];
    const T* u = sm + a.ou[0];
    if (a.basis_out) {
      const int mx = G.nx - 2, m0 = mx * (G.ny - 2);
      for (int i = tid; i < m0; i += nt)
        a.basis_out[size_t(blockIdx.x) * m0 + i] = u[(i / mx + 1) * G.nx + i % mx + 1];
    } else {
      for (int k = tid; k < G.nx * G.ny; k += nt) G.u[k] = u[k];
    }
  }
}

template <class T>
__global__ __launch_bounds__(1024) void k_tail(TailArgs<T> a) {
  tail_body<T, false>(a);
}

// Basis runs of a dense operator: the tail with its stencils read in global memory.
__global__ __launch_bounds__(256) void k_tail_unstaged(TailArgs<double> a) {
  tail_body<double, true>(a);
}

// One workgroup per instance: list[blockIdx.x] holds that instance's tail.
template <class T>
__global__ __launch_bounds__(1024) void k_tail_multi(const TailArgs<T>* __restrict__ list) {
  tail_body<T, false>(list[blockIdx.x]);
}

}  // namespace

// -----------------------------------------------------------------------------------------
// Wave-strip kernels: the same row pipeline with one wavefront per strip of 64 columns.  Each
// lane owns one column and keeps its ring rows in registers; values of the neighbouring
// columns come from the neighbouring lanes through DPP whole-wave shifts, so the kernel uses
// no LDS and no barriers.  Lanes 0 and 63 receive their own value from a shift (they are halo
// columns, whose results are never written).
// -----------------------------------------------------------------------------------------
__device__ __forceinline__ int lane_from_left(int v) {   // value held by lane - 1
  return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false);  // wave_shr:1
}
__device__ __forceinline__ int lane_from_right(int v) {  // value held by lane + 1
  return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false);  // wave_shl:1
}
__device__ __forceinline__ double from_left(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = lane_from_left(int(x & 0xffffffffll)), hi = lane_from_left(int(x >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double from_right(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = lane_from_right(int(x & 0xffffffffll)), hi = lane_from_right(int(x >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ float from_left(float v) {
  return __int_as_float(lane_from_left(__float_as_int(v)));
}
__device__ __forceinline__ float from_right(float v) {
  return __int_as_float(lane_from_right(__float_as_int(v)));
}

template <class T>
struct WaveCol {
  T u[RU];
  T C[RS], W[RS], Sv[RS], SW[RS], SE[RS], b[RS];
  T rC[RS];                    // 1 / C, formed when the row is stored
  T Er[RS], NEr[RS], NWl[RS];  // W and SW of lane+1, SE of lane-1, same row
  T r[RS];                     // residuals (pre)
};

// Fused multiply-adds are written out: the step copies of the unrolled ring period share
// products between the smoothing update and the residual, and implicit contraction would then
// fuse them in some copies and not in others, making the rounding depend on the segment height.
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Off-diagonal part of row JR's stencil applied to u, summed per stencil row (south, own, north)
// and then (south + north) + own: each group waits only for its own row of u, so the group fed
// by the update just made is short.
template <class T, int UM, int U0, int UP, int S0, int SP>
__device__ __forceinline__ T offdiag_w(const WaveCol<T>& c) {
#pragma clang fp contract(off)
  const T um = c.u[UM], u0 = c.u[U0], up = c.u[UP];
  T s1 = c.SW[S0] * from_left(um);
  s1 = fmad(c.Sv[S0], um, s1);
  s1 = fmad(c.SE[S0], from_right(um), s1);
  T s3 = c.NWl[SP] * from_left(up);
  s3 = fmad(c.Sv[SP], up, s3);
  s3 = fmad(c.NEr[SP], from_right(up), s3);
  T s2 = c.W[S0] * from_left(u0);
  s2 = fmad(c.Er[S0], from_right(u0), s2);
  return (s1 + s3) + s2;
}

// Gauss-Seidel update of this lane's point on the row at relative index JR where `ok` holds.
// Every lane evaluates (the shifts need all lanes); the others keep their value.
template <class T, int JR>
__device__ __forceinline__ void gs_wave(WaveCol<T>& c, bool ok) {
  constexpr int U0 = umod(JR), UM = umod(JR - 1), UP = umod(JR + 1);
  constexpr int S0 = smod(JR), SP = smod(JR + 1);
  const T num = c.b[S0] - offdiag_w<T, UM, U0, UP, S0, SP>(c);
  // num / C from the stored reciprocal and one residual correction
  const T q0 = num * c.rC[S0];
  const T v = fmad(fmad(-q0, c.C[S0], num), c.rC[S0], q0);
  c.u[U0] = ok ? v : c.u[U0];
}

template <class T, int JR>
__device__ __forceinline__ T resid_wave(const WaveCol<T>& c, bool ok) {
  constexpr int U0 = umod(JR), UM = umod(JR - 1), UP = umod(JR + 1);
  constexpr int S0 = smod(JR), SP = smod(JR + 1);
  const T off = offdiag_w<T, UM, U0, UP, S0, SP>(c);
  const T r = c.b[S0] - fmad(c.C[S0], c.u[U0], off);
  return ok ? r : T(0);
}

template <class T, int JR>
__device__ __forceinline__ void store_row_w(WaveCol<T>& c, const RowRegs<T>& g) {
  constexpr int U0 = umod(JR), S0 = smod(JR);
  c.u[U0] = g.u;
  c.b[S0] = g.b;
  c.C[S0] = g.s[0];
  c.rC[S0] = T(1) / (g.s[0] != T(0) ? g.s[0] : T(1));
  c.W[S0] = g.s[1];
  c.Sv[S0] = g.s[2];
  c.SW[S0] = g.s[3];
  c.SE[S0] = g.s[4];
  c.Er[S0] = from_right(g.s[1]);
  c.NEr[S0] = from_right(g.s[3]);
  c.NWl[S0] = from_left(g.s[4]);
}

// Coarse values of coarse column I for one row step of the post kernel (see load_coarse):
// v[0] e(J_even), v[1..2] P0/P1(J_even), v[3..4] e(J_odd), e(J_odd+1), v[5..10] P2..P7(J_odd).
template <class T>
__device__ __forceinline__ T prolong_wave(const CoarseRegs<T>& cv, int i, int j) {
#pragma clang fp contract(off)
  if (!(j & 1)) {
    const T e = cv.v[0];
    const T e1 = from_right(from_right(e));  // coarse column I+1 lives two lanes to the right
    return (i & 1) ? cv.v[1] * e + cv.v[2] * e1 : e;
  }
  const T e0 = cv.v[3], e1 = cv.v[4];
  const T e0r = from_right(from_right(e0)), e1r = from_right(from_right(e1));
  if (!(i & 1)) return cv.v[5] * e0 + cv.v[6] * e1;
  return ((cv.v[7] * e0 + cv.v[8] * e0r) + cv.v[9] * e1) + cv.v[10] * e1r;
}

// MODE as k_strip; PF = row parity smoothed first.
// One tile of a wave-strip sweep; the squared-residual partial (post, when a.partials is set)
// goes to a.partials[pidx].
template <class T, int MODE, int PF, int UREAD>
__device__ __forceinline__ void wave_tile(const StripArgs<T>& a, int tile, int pidx) {
  constexpr bool POST = MODE >= 2;
  constexpr bool prol = MODE == 2;
  constexpr int BW = 64;
  const int seg = tile / a.nstrips;
  const int strip = tile % a.nstrips;
  const int t = threadIdx.x;
  const int out_w = BW - 2 * HALO;
  const int x0 = strip * out_w;
  const int i = x0 - HALO + t;
  // coarse column whose values this lane loads: lanes 2m and 2m+1 share column I = i >> 1
  const int cI = i >> 1;
  const int j0 = seg * a.seg_h;
  const int j1 = min(j0 + a.seg_h, a.ny);
  const int lim = POST ? j0 - 1 : j0 - 2;
  const int a0 = lim - (((lim - PF) % 2) + 2) % 2;
  const int alast = j1 + (((j1 - PF) % 2) + 2) % 2;
  // rows past alast + 1 are never consumed: their prefetch slots read row -1, which the
  // loader maps to a fixed, cached address instead of streaming unused rows from memory
  auto live = [&](int r) { return r <= alast + 1 ? r : -1; };
  const double xs = (POST && a.x64 && a.xscale) ? *a.xscale : 1.0;
  auto emit = [&](size_t v, T val) {
    a.u[v] = val;
    if constexpr (POST && std::is_same<T, float>::value)
      if (a.x64) a.x64[v] = add_scaled(a.x64[v], xs, double(val));
  };
  const int base = a0 - 1;
  (void)base;
  const bool interior_i = i >= 1 && i <= a.nx - 2;
  const bool out_col = t >= HALO && t < BW - HALO && i < a.nx;
  const int ncx = (a.nx + 1) / 2, ncy = (a.ny + 1) / 2;
  auto row_ok = [&](int j) { return interior_i && j >= 1 && j <= a.ny - 2; };

  WaveCol<T> c;
#pragma unroll
  for (int k = 0; k < RU; ++k) c.u[k] = T(0);
#pragma unroll
  for (int k = 0; k < RS; ++k)
    c.C[k] = c.rC[k] = c.W[k] = c.Sv[k] = c.SW[k] = c.SE[k] = c.b[k] = c.Er[k] = c.NEr[k] =
        c.NWl[k] = c.r[k] = T(0);
  // every load of the prologue is issued before the stop flag is tested and before any of
  // them is used, so that their memory latencies overlap
  const int stopped = a.stop ? *a.stop : 0;
  RowRegs<T> gM, gA0, gA1, gB0, gB1;
  CoarseRegs<T> cr;
  load_row<T, UREAD>(a, i, a0 - 1, gM);
  const T pm = (prol && row_ok(a0 - 1)) ? prolong_global<T>(a, i, a0 - 1) : T(0);
  if (prol) load_coarse<T>(a, cI, a0, cr);
  load_row<T, UREAD>(a, i, a0, gA0);
  load_row<T, UREAD>(a, i, a0 + 1, gA1);
  load_row<T, UREAD>(a, i, live(a0 + 2), gB0);
  load_row<T, UREAD>(a, i, live(a0 + 3), gB1);
  if (stopped) return;
  if (prol && row_ok(a0 - 1)) gM.u = gM.u + pm;
  store_row_w<T, 0>(c, gM);
  double acc = 0.0;

  auto step = [&](auto KC, int ar, RowRegs<T>& g0, RowRegs<T>& g1) {
    constexpr int K = decltype(KC)::value;
    constexpr int JA = 1 + 2 * K;
    if (prol) {
      const T c0 = prolong_wave<T>(cr, i, ar), c1 = prolong_wave<T>(cr, i, ar + 1);
      if (row_ok(ar)) g0.u = g0.u + c0;
      if (row_ok(ar + 1)) g1.u = g1.u + c1;
    }
    store_row_w<T, JA>(c, g0);
    store_row_w<T, JA + 1>(c, g1);
    // loads in the order they are consumed: restriction weights (end of this step), coarse
    // values (top of the next step), rows of the step after next
    const int fj = (ar - 2) & ~1;
    const int J = fj >> 1;
    const int I = i >> 1;
    const bool do_restrict = !POST && out_col && !(i & 1) && fj >= j0 && fj < j1;
    const bool inner_c = I >= 1 && I <= ncx - 2 && J >= 1 && J <= ncy - 2;
    T pw[8];
    if (!POST) {
      const size_t NC = size_t(ncx) * ncy;
      const size_t cc = (do_restrict && inner_c) ? size_t(J) * ncx + I : size_t(ncx) + 1;
      const T* P = a.P;
      pw[0] = P[7 * NC + cc - ncx - 1];
      pw[1] = P[3 * NC + cc - ncx];
      pw[2] = P[6 * NC + cc - ncx];
      pw[3] = P[1 * NC + cc - 1];
      pw[4] = P[0 * NC + cc];
      pw[5] = P[5 * NC + cc - 1];
      pw[6] = P[2 * NC + cc];
      pw[7] = P[4 * NC + cc];
    }
    if (prol) load_coarse<T>(a, cI, ar + 2, cr);
    load_row<T, UREAD>(a, i, live(ar + 4), g0);
    load_row<T, UREAD>(a, i, live(ar + 5), g1);
    const bool okA = row_ok(ar), okB = row_ok(ar - 1);
    const bool firstA = (i & 1) == a.cA, firstB = (i & 1) == a.cB;
    gs_wave<T, JA>(c, okA && firstA);
    gs_wave<T, JA>(c, okA && !firstA);
    gs_wave<T, JA - 1>(c, okB && firstB);
    gs_wave<T, JA - 1>(c, okB && !firstB);
    if (out_col) {
      if (ar - 1 >= j0 && ar - 1 < j1) emit(size_t(ar - 1) * a.nx + i, c.u[umod(JA - 1)]);
      if (ar >= j0 && ar < j1) emit(size_t(ar) * a.nx + i, c.u[umod(JA)]);
    }
    const T r2 = resid_wave<T, JA - 2>(c, row_ok(ar - 2));
    const T r1 = resid_wave<T, JA - 1>(c, okB);
    if (POST) {
      if (out_col && a.partials) {
        if (ar - 2 >= j0 && ar - 2 < j1) acc += double(r2) * double(r2);
        if (ar - 1 >= j0 && ar - 1 < j1) acc += double(r1) * double(r1);
      }
    } else {
      c.r[smod(JA - 2)] = r2;
      c.r[smod(JA - 1)] = r1;
      constexpr int RF = JA - 2 - PF;  // relative index of fine row 2J
      const T rm = c.r[smod(RF - 1)], r0 = c.r[smod(RF)], rp = c.r[smod(RF + 1)];
      const T rml = from_left(rm), rmr = from_right(rm);
      const T r0l = from_left(r0), r0r = from_right(r0);
      const T rpl = from_left(rp), rpr = from_right(rp);
      if (do_restrict) {
        T acc2 = T(0);
        if (inner_c) {
#pragma clang fp contract(off)
          T g1 = pw[0] * rml;
          g1 = fmad(pw[1], rm, g1);
          g1 = fmad(pw[2], rmr, g1);
          T g2 = fmad(pw[3], r0l, r0);
          g2 = fmad(pw[4], r0r, g2);
          T g3 = pw[5] * rpl;
          g3 = fmad(pw[6], rp, g3);
          g3 = fmad(pw[7], rpr, g3);
          acc2 = (g1 + g2) + g3;
        }
        if (J < ncy) a.bH[size_t(J) * ncx + I] = acc2;
      }
    }
  };

  for (int ar = a0; ar <= alast; ar += 8) {
    step(std::integral_constant<int, 0>{}, ar, gA0, gA1);
    if (ar + 2 > alast) break;
    step(std::integral_constant<int, 1>{}, ar + 2, gB0, gB1);
    if (ar + 4 > alast) break;
    step(std::integral_constant<int, 2>{}, ar + 4, gA0, gA1);
    if (ar + 6 > alast) break;
    step(std::integral_constant<int, 3>{}, ar + 6, gB0, gB1);
  }
  if (POST && a.partials) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (t == 0) a.partials[pidx] = acc;
  }
}

// MODE as k_strip; PF = row parity smoothed first.
template <class T, int MODE, int PF>
__global__ __launch_bounds__(64) void k_wave(StripArgs<T> a) {
  const int ntiles = a.nstrips * a.nsegs;
  const int per = (int(gridDim.x) + 7) >> 3;
  const int tile = (int(blockIdx.x) & 7) * per + (int(blockIdx.x) >> 3);
  if (tile >= ntiles) {
    if (MODE >= 2 && a.partials && threadIdx.x == 0 && !(a.stop && *a.stop))
      a.partials[blockIdx.x] = 0.0;
    return;
  }
  wave_tile<T, MODE, PF, MODE != 0 ? 1 : 0>(a, tile, int(blockIdx.x));  // tests a.stop itself
}

// The same sweep over the tiles of several instances of one level size at once: list[k] is
// instance k's arguments (all with the same nx, ny, seg_h), tiles_per its tile count.  Pre
// sweeps (MODE 1) read u where list[k].uin is set and start from zero elsewhere; partials go to
// list[k].partials[tile].
template <class T, int MODE, int PF>
__global__ __launch_bounds__(64) void k_wave_multi(const StripArgs<T>* __restrict__ list,
                                                   int tiles_per, int total) {
  const int per = (int(gridDim.x) + 7) >> 3;
  const int g = (int(blockIdx.x) & 7) * per + (int(blockIdx.x) >> 3);
  if (g >= total) return;
  const int inst = g / tiles_per, tile = g - inst * tiles_per;
  const StripArgs<T> a = list[inst];
  wave_tile<T, MODE, PF, MODE == 1 ? 2 : (MODE == 0 ? 0 : 1)>(a, tile, tile);  // tests a.stop
}

// ---- float64 residual of the refinement loop ----------------------------------------------
// One wavefront per strip of 62 output columns and `rows` rows: lane t holds column
// i = 62 strip - 1 + t (lanes 0 and 63 are halo), rows slide through registers one ahead of use,
// and the neighbouring columns come from DPP lane shifts.  The off-diagonal sum runs in the same
// order, with the same explicit fused multiply-adds, as in the wave sweeps.
constexpr int kResidOut = 62;

struct ResRow {
  double x, b, C, W, S, SW, SE;
};

__device__ __forceinline__ void res_load(const double* S, const double* x, const double* b,
                                         int nx, int ny, int i, int j, ResRow& r) {
  const bool ok = i >= 0 && i < nx && j >= 0 && j < ny;
  const size_t v = ok ? size_t(j) * nx + i : 0;
  const double* sv = S + 5 * v;
  const double t0 = x[v], t1 = b[v], t2 = sv[0], t3 = sv[1], t4 = sv[2], t5 = sv[3], t6 = sv[4];
  r.x = ok ? t0 : 0.0;
  r.b = ok ? t1 : 0.0;
  r.C = ok ? t2 : 0.0;
  r.W = ok ? t3 : 0.0;
  r.S = ok ? t4 : 0.0;
  r.SW = ok ? t5 : 0.0;
  r.SE = ok ? t6 : 0.0;
}

__global__ __launch_bounds__(64) void k_ir_resid(const double* __restrict__ S,
                                                 const double* __restrict__ x,
                                                 const double* __restrict__ b,
                                                 double* __restrict__ r64, int nx, int ny, int rows,
                                                 int nstrips, double* __restrict__ partials,
                                                 const int* __restrict__ stop,
                                                 const int* __restrict__ zero) {
  if (stop && *stop) return;
  const int strip = int(blockIdx.x) % nstrips, seg = int(blockIdx.x) / nstrips;
  const int t = threadIdx.x;
  const int i = strip * kResidOut - 1 + t;
  const int j0 = seg * rows, j1 = min(j0 + rows, ny);
  const bool out_col = t >= 1 && t <= kResidOut && i < nx;
  const bool int_col = i >= 1 && i <= nx - 2;
  if (zero && *zero) {
    // x = 0: A x vanishes and r = b; the same points are summed in the same order
    double acc = 0.0;
    for (int j = j0; j < j1; ++j) {
      const bool interior = int_col && j >= 1 && j <= ny - 2;
      if (out_col) {
        const size_t v = size_t(j) * nx + i;
        const double rv = interior ? b[v] : 0.0;
        r64[v] = rv;
        acc += rv * rv;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (t == 0) partials[blockIdx.x] = acc;
    return;
  }
  ResRow m, c, n, nn;  // rows j - 1, j, j + 1 and the prefetched j + 2
  res_load(S, x, b, nx, ny, i, j0 - 1, m);
  res_load(S, x, b, nx, ny, i, j0, c);
  res_load(S, x, b, nx, ny, i, j0 + 1, n);
  double acc = 0.0;
  for (int j = j0; j < j1; ++j) {
    // row j + 2 is needed for the next row only (rows past the segment read a cached address)
    res_load(S, x, b, nx, ny, i, j + 2 <= j1 ? j + 2 : -1, nn);
    double o;
    {
#pragma clang fp contract(off)
      o = c.SW * from_left(m.x);
      o = fmad(c.S, m.x, o);
      o = fmad(c.SE, from_right(m.x), o);
      o = fmad(c.W, from_left(c.x), o);
      o = fmad(from_right(c.W), from_right(c.x), o);
      o = fmad(from_left(n.SE), from_left(n.x), o);
      o = fmad(n.S, n.x, o);
      o = fmad(from_right(n.SW), from_right(n.x), o);
    }
    const double r = c.b - fmad(c.C, c.x, o);
    const bool interior = int_col && j >= 1 && j <= ny - 2;
    const double rv = interior ? r : 0.0;
    if (out_col) {
      r64[size_t(j) * nx + i] = rv;
      acc += rv * rv;
    }
    m = c;
    c = n;
    n = nn;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (t == 0) partials[blockIdx.x] = acc;
}

// x += s e (float64 += float64 * float32), s = *scale, where no float strip sweep carries the
// update.
__global__ __launch_bounds__(256) void k_ir_add(double* __restrict__ x, const float* __restrict__ e,
                                                size_t n, const double* __restrict__ scale,
                                                const int* __restrict__ stop) {
  if (stop && *stop) return;
  const double s = *scale;
  for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < n;
       k += size_t(gridDim.x) * blockDim.x)
    x[k] = add_scaled(x[k], s, double(e[k]));
}

// r32 = fl32(r / s), s = *norm: the float64 quotient rounded once more to float32 (zero where
// s = 0, a solve that is already done).
__global__ __launch_bounds__(256) void k_ir_scale(const double* __restrict__ r,
                                                  float* __restrict__ r32, size_t n,
                                                  const double* __restrict__ norm,
                                                  const int* __restrict__ stop) {
  if (stop && *stop) return;
  const double s = *norm;
  for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < n;
       k += size_t(gridDim.x) * blockDim.x)
    r32[k] = s > 0.0 ? float(r[k] / s) : 0.f;
}

namespace {
void resid_shape(int nx, int ny, int* rows, int* nstrips, int* nblocks) {
  *nstrips = (nx + kResidOut - 1) / kResidOut;
  int r = 64;
  auto blocks = [&](int rr) { return *nstrips * ((ny + rr - 1) / rr); };
  while (r > 2 && blocks(r) < 2048) r /= 2;
  while (blocks(r) > kMaxPartials) r *= 2;
  *rows = r;
  *nblocks = blocks(r);
}
}  // namespace

int ir_residual_blocks(int nx, int ny) {
  int rows = 0, ns = 0, nb = 0;
  resid_shape(nx, ny, &rows, &ns, &nb);
  return nb;
}

dmg_status launch_ir_residual(const double* S, const double* x, const double* b, double* r,
                              int nx, int ny, double* partials, hipStream_t s, const int* stop,
                              const int* zero) {
  int rows = 0, ns = 0, nb = 0;
  resid_shape(nx, ny, &rows, &ns, &nb);
  k_ir_resid<<<nb, 64, 0, s>>>(S, x, b, r, nx, ny, rows, ns, partials, stop, zero);
  return launch_check("ir_residual");
}

dmg_status launch_ir_update(double* x, const float* e, size_t n, const double* scale,
                            hipStream_t s, const int* stop) {
  const size_t nb = (n + 255) / 256;
  k_ir_add<<<unsigned(nb < 4096 ? (nb ? nb : 1) : 4096), 256, 0, s>>>(x, e, n, scale, stop);
  return launch_check("ir_update");
}

dmg_status launch_ir_scale(const double* r, float* r32, size_t n, const double* norm,
                           hipStream_t s, const int* stop) {
  const size_t nb = (n + 255) / 256;
  k_ir_scale<<<unsigned(nb < 4096 ? (nb ? nb : 1) : 4096), 256, 0, s>>>(r, r32, n, norm, stop);
  return launch_check("ir_scale");
}

// ---- launchers -----------------------------------------------------------------------------
int strip_blocks(int nx, int ny, int bw, int seg_h, int* nstrips, int* nsegs) {
  const int out_w = bw - 2 * HALO;
  *nstrips = (nx + out_w - 1) / out_w;
  *nsegs = (ny + seg_h - 1) / seg_h;
  const int nt = *nstrips * *nsegs;
  return (nt + 7) & ~7;
}

template <class T, bool POST>
dmg_status launch_strip(const StripConfig& cfg, const T* S, const T* uin, T* u, const T* b,
                        const T* P, T* bH, const T* e, double* partials, int nx, int ny, int pf,
                        int cA, int cB, const int* stop, hipStream_t s, double* x64 = nullptr,
                        const double* xscale = nullptr) {
  if (POST && !uin) return fail(DMG_ERR_INVALID_ARG, "post sweep needs an input iterate");
  if (uin == u) return fail(DMG_ERR_INVALID_ARG, "strip sweeps work out of place");
  StripArgs<T> a;
  a.S = S;
  a.uin = uin;
  a.u = u;
  a.b = b;
  a.P = P;
  a.bH = bH;
  a.e = e;
  a.partials = partials;
  a.nx = nx;
  a.ny = ny;
  a.seg_h = cfg.seg_h;
  a.pf = pf;
  a.cA = cA;
  a.cB = cB;
  a.stop = stop;
  a.x64 = x64;
  a.xscale = xscale;
  const int nb = strip_blocks(nx, ny, cfg.bw, cfg.seg_h, &a.nstrips, &a.nsegs);
  const size_t lds =
      (size_t(RU + 4 * RS) * cfg.bw + (POST ? size_t(2 * kCoarseSlots) * (cfg.bw / 2 + 2) : 0)) *
      sizeof(T);
  const int mode = POST ? (e ? 2 : 3) : (uin ? 1 : 0);
  if (cfg.wave) {
    if (cfg.bw != 64) return fail(DMG_ERR_INVALID_ARG, "wave strips are 64 columns wide");
#define DMG_WAVE(M)                                                                  \
  (pf ? (void)(k_wave<T, M, 1><<<nb, 64, 0, s>>>(a)) : (void)(k_wave<T, M, 0><<<nb, 64, 0, s>>>(a)))
    switch (mode) {
      case 0: DMG_WAVE(0); break;
      case 1: DMG_WAVE(1); break;
      case 2: DMG_WAVE(2); break;
      default: DMG_WAVE(3); break;
    }
#undef DMG_WAVE
    return launch_check(POST ? "wave_post" : "wave_pre");
  }
#define DMG_STRIP_BW(BWV)                                                   \
  switch (mode) {                                                           \
    case 0: k_strip<T, BWV, 0><<<nb, BWV, lds, s>>>(a); break;              \
    case 1: k_strip<T, BWV, 1><<<nb, BWV, lds, s>>>(a); break;              \
    case 2: k_strip<T, BWV, 2><<<nb, BWV, lds, s>>>(a); break;              \
    default: k_strip<T, BWV, 3><<<nb, BWV, lds, s>>>(a); break;             \
  }
  switch (cfg.bw) {
    case 64: DMG_STRIP_BW(64) break;
    case 128: DMG_STRIP_BW(128) break;
    case 256: DMG_STRIP_BW(256) break;
    default:
      return fail(DMG_ERR_INVALID_ARG, "unsupported strip width %d", cfg.bw);
  }
#undef DMG_STRIP_BW
  return launch_check(POST ? "strip_post" : "strip_pre");
}

template <class T>
dmg_status launch_pre(const StripConfig& cfg, const T* S, const T* uin, T* u, const T* b,
                      const T* P, T* bH, int nx, int ny, int pf, int cA, int cB, const int* stop,
                      hipStream_t s) {
  return launch_strip<T, false>(cfg, S, uin, u, b, P, bH, nullptr, nullptr, nx, ny, pf, cA, cB,
                                stop, s);
}

template <class T>
dmg_status launch_post(const StripConfig& cfg, const T* S, const T* uin, T* u, const T* b,
                       const T* P, const T* e, double* partials, int nx, int ny, int pf, int cA,
                       int cB, const int* stop, hipStream_t s, double* x64,
                       const double* xscale) {
  if (x64 && !std::is_same<T, float>::value)
    return fail(DMG_ERR_INVALID_ARG, "the float64 iterate update belongs to float sweeps");
  return launch_strip<T, true>(cfg, S, uin, u, b, P, nullptr, e, partials, nx, ny, pf, cA, cB,
                               stop, s, x64, xscale);
}

TailLayout tail_layout(const int* nx, const int* ny, int nlev, int m, int elem, int dense,
                       int staged) {
  TailLayout t;
  int off = 0;
  int rmax = 0;
  for (int l = 0; l < nlev; ++l) {
    const int n = nx[l] * ny[l];
    if (dense && l + 1 == nlev) rmax = n > rmax ? n : rmax;  // the residual of a dense top level
    if (l + 1 < nlev) {
      t.S[l] = staged ? off : -1;
      off += staged ? 5 * n : 0;
      t.P[l] = staged ? off : -1;
      off += staged ? 8 * nx[l + 1] * ny[l + 1] : 0;
      rmax = n > rmax ? n : rmax;
    } else {
      t.S[l] = t.P[l] = -1;
    }
    t.u[l] = off;
    off += n;
    t.b[l] = off;
    off += n;
  }
  t.B = off;
  off += (dense && staged) ? m * m : 0;
  t.r = off;
  off += rmax;
  size_t bytes = size_t(off) * elem;
  bytes = (bytes + 15) & ~size_t(15);
  t.y = int(bytes);
  t.bytes = bytes + size_t(m > 0 ? m : 1) * sizeof(double);
  return t;
}

int device_lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 65536;
  return v > 0 ? v : 65536;
}

template <class T>
dmg_status make_tail_args(const TailSpec<T>& spec, TailArgs<T>* out, size_t* lds_bytes) {
  TailArgs<T>& a = *out;
  if (spec.nlev > kMaxTail) return fail(DMG_ERR_INVALID_ARG, "tail too deep (%d)", spec.nlev);
  if (spec.dense && spec.m != (spec.nx[spec.nlev - 1] - 2) * (spec.ny[spec.nlev - 1] - 2))
    return fail(DMG_ERR_INVALID_ARG, "dense coarse operator size does not match its level");
  if (spec.unstaged && spec.image)
    return fail(DMG_ERR_INVALID_ARG, "an unstaged coarse tail has no LDS image");
  const TailLayout lay = tail_layout(spec.nx, spec.ny, spec.nlev, spec.m, int(sizeof(T)),
                                     spec.dense, !spec.unstaged);
  if (lay.bytes > size_t(device_lds_limit()))
    return fail(DMG_ERR_INVALID_ARG, "coarse tail needs %zu bytes of LDS", lay.bytes);
  for (int l = 0; l < spec.nlev; ++l) {
    a.L[l].S = spec.S[l];
    a.L[l].u = spec.u[l];
    a.L[l].b = spec.b[l];
    a.L[l].P = spec.P[l];
    a.L[l].nx = spec.nx[l];
    a.L[l].ny = spec.ny[l];
    a.oS[l] = lay.S[l];
    a.ou[l] = lay.u[l];
    a.ob[l] = lay.b[l];
    a.oP[l] = lay.P[l];
  }
  a.o_r = lay.r;
  a.o_y = lay.y;
  a.nlev = spec.nlev;
  a.zero_top = spec.zero_top;
  a.m = spec.m;
  a.idx = spec.idx;
  a.chol = spec.chol;
  for (int k = 0; k < 4; ++k) {
    a.pre[k] = spec.pre[k];
    a.post[k] = spec.post[k];
  }
  a.nu_pre = spec.nu_pre;
  a.nu_post = spec.nu_post;
  a.smoother = spec.smoother;
  a.stop = spec.stop;
  a.image = nullptr;
  a.image_n = 0;
  a.dense = spec.dense;
  a.oB = lay.B;
  a.Bg = spec.B;
  a.basis_out = nullptr;
  a.unstaged = spec.unstaged;
  if (spec.dense && !spec.B) return fail(DMG_ERR_INVALID_ARG, "dense coarse tail without its matrix");
  if (spec.image) {
    if (!spec.zero_top || spec.image_n != lay.r || spec.b[0] != spec.image + lay.b[0] ||
        (spec.dense && spec.B != spec.image + lay.B))
      return fail(DMG_ERR_INVALID_ARG, "coarse tail image does not match its layout");
    a.image = spec.image;
    a.image_n = spec.image_n;
  }
  *lds_bytes = lay.bytes;
  return DMG_OK;
}

template <class T>
dmg_status launch_tail(const TailSpec<T>& spec, hipStream_t s) {
  if (spec.threads < 64 || spec.threads > 1024 || spec.threads % 64)
    return fail(DMG_ERR_INVALID_ARG, "coarse tail workgroup size %d", spec.threads);
  TailArgs<T> a;
  size_t bytes = 0;
  DMG_CHECK(make_tail_args<T>(spec, &a, &bytes));
  k_tail<T><<<1, spec.threads, bytes, s>>>(a);
  return launch_check("tail");
}

dmg_status launch_tail_basis(const TailSpec<double>& spec, double* out, hipStream_t s) {
  if (spec.threads < 64 || spec.threads > 1024 || spec.threads % 64)
    return fail(DMG_ERR_INVALID_ARG, "coarse tail workgroup size %d", spec.threads);
  if (spec.image || !spec.zero_top || !out)
    return fail(DMG_ERR_INVALID_ARG, "basis run of a coarse tail: full cycle from zero only");
  TailArgs<double> a;
  size_t bytes = 0;
  DMG_CHECK(make_tail_args<double>(spec, &a, &bytes));
  a.basis_out = out;
  const int m0 = (spec.nx[0] - 2) * (spec.ny[0] - 2);
  if (spec.unstaged) {
    if (spec.threads > 256) return fail(DMG_ERR_INVALID_ARG, "unstaged basis runs use <= 256 threads");
    k_tail_unstaged<<<m0, spec.threads, bytes, s>>>(a);
  } else {
    k_tail<double><<<m0, spec.threads, bytes, s>>>(a);
  }
  return launch_check("tail basis");
}

template <class T>
dmg_status launch_tail_multi(const TailArgs<T>* list, int count, size_t lds_bytes, int threads,
                             hipStream_t s) {
  if (threads < 64 || threads > 1024 || threads % 64)
    return fail(DMG_ERR_INVALID_ARG, "coarse tail workgroup size %d", threads);
  if (count < 1) return DMG_OK;
  k_tail_multi<T><<<count, threads, lds_bytes, s>>>(list);
  return launch_check("tail_multi");
}

template <class T>
dmg_status launch_wave_multi(const StripArgs<T>* list, int count, int tiles_per, int mode, int pf,
                             hipStream_t s) {
  if (count < 1 || tiles_per < 1) return DMG_OK;
  const long total = long(count) * tiles_per;
  if (total > (1l << 30)) return fail(DMG_ERR_INVALID_ARG, "too many tiles in one launch");
  const int nb = int((total + 7) & ~7l);
#define DMG_WAVE_M(M)                                                                          \
  (pf ? (void)(k_wave_multi<T, M, 1><<<nb, 64, 0, s>>>(list, tiles_per, int(total)))           \
      : (void)(k_wave_multi<T, M, 0><<<nb, 64, 0, s>>>(list, tiles_per, int(total))))
  switch (mode) {
    case 1: DMG_WAVE_M(1); break;
    case 2: DMG_WAVE_M(2); break;
    case 3: DMG_WAVE_M(3); break;
    default: return fail(DMG_ERR_INVALID_ARG, "multi-instance sweep mode %d", mode);
  }
#undef DMG_WAVE_M
  return launch_check("wave_multi");
}

#define DMG_INST(T)                                                                            \
  template dmg_status launch_pre<T>(const StripConfig&, const T*, const T*, T*, const T*,      \
                                    const T*, T*, int, int, int, int, int, const int*,         \
                                    hipStream_t);                                              \
  template dmg_status launch_post<T>(const StripConfig&, const T*, const T*, T*, const T*,     \
                                     const T*, const T*, double*, int, int, int, int, int,     \
                                     const int*, hipStream_t, double*, const double*);         \
  template dmg_status launch_tail<T>(const TailSpec<T>&, hipStream_t);                        \
  template dmg_status make_tail_args<T>(const TailSpec<T>&, TailArgs<T>*, size_t*);           \
  template dmg_status launch_tail_multi<T>(const TailArgs<T>*, int, size_t, int, hipStream_t); \
  template dmg_status launch_wave_multi<T>(const StripArgs<T>*, int, int, int, int, hipStream_t);
DMG_INST(double)
DMG_INST(float)
#undef DMG_INST

}  // namespace dmg
