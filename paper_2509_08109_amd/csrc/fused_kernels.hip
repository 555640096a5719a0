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
#include "dmg_internal.h"

namespace dmg {
namespace {

constexpr int HALO = 6;   // columns recomputed on each side of a strip
constexpr int RU = 8;     // ring rows of u
constexpr int RS = 4;     // ring rows of S, b, r

template <class T>
struct StripArgs {
  const T* S;         // [5][ny][nx]
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
};

template <class T>
struct Ring {
  T* u;   // [RU][BW]
  T* S;   // [5][RS][BW]
  T* b;   // [RS][BW]
  T* r;   // [RS][BW]
};

// Update (residual) of interior point (i, j) held in ring slot sj of thread t.
template <class T, int BW>
__device__ __forceinline__ T offdiag_l(const Ring<T>& R, int t, int j) {
  const int tm = t > 0 ? t - 1 : 0, tp = t < BW - 1 ? t + 1 : BW - 1;
  const int sj = j & (RS - 1), sjp = (j + 1) & (RS - 1);
  const T* uj = R.u + (j & (RU - 1)) * BW;
  const T* ujm = R.u + ((j - 1) & (RU - 1)) * BW;
  const T* ujp = R.u + ((j + 1) & (RU - 1)) * BW;
  const T* W = R.S + (1 * RS) * BW;
  const T* Sv = R.S + (2 * RS) * BW;
  const T* SW = R.S + (3 * RS) * BW;
  const T* SE = R.S + (4 * RS) * BW;
  const T sw = SW[sj * BW + t] * ujm[tm];
  const T s = Sv[sj * BW + t] * ujm[t];
  const T se = SE[sj * BW + t] * ujm[tp];
  const T w = W[sj * BW + t] * uj[tm];
  const T e = W[sj * BW + tp] * uj[tp];
  const T nw = SE[sjp * BW + tm] * ujp[tm];
  const T n = Sv[sjp * BW + t] * ujp[t];
  const T ne = SW[sjp * BW + tp] * ujp[tp];
  return ((((((sw + s) + se) + w) + e) + nw) + n) + ne;
}

template <class T, int BW>
__device__ __forceinline__ void gs_point(const Ring<T>& R, int t, int i, int j, int nx, int ny) {
  if (i < 1 || i > nx - 2 || j < 1 || j > ny - 2) return;
  const T off = offdiag_l<T, BW>(R, t, j);
  const int sj = j & (RS - 1);
  R.u[(j & (RU - 1)) * BW + t] = (R.b[sj * BW + t] - off) / R.S[sj * BW + t];
}

template <class T, int BW>
__device__ __forceinline__ T resid_point(const Ring<T>& R, int t, int i, int j, int nx, int ny) {
  if (i < 1 || i > nx - 2 || j < 1 || j > ny - 2) return T(0);
  const T off = offdiag_l<T, BW>(R, t, j);
  const int sj = j & (RS - 1);
  return R.b[sj * BW + t] - (off + R.S[sj * BW + t] * R.u[(j & (RU - 1)) * BW + t]);
}

// Registers holding one prefetched row for this thread's column.
template <class T>
struct RowRegs {
  T u, b, s[5];
};

template <class T, bool POST>
__device__ __forceinline__ void load_row(const StripArgs<T>& a, int i, int j, RowRegs<T>& g) {
  g.u = T(0);
  g.b = T(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) g.s[k] = T(0);
  if (i < 0 || i >= a.nx || j < 0 || j >= a.ny) return;
  const size_t N = size_t(a.nx) * a.ny;
  const size_t v = size_t(j) * a.nx + i;
#pragma unroll
  for (int k = 0; k < 5; ++k) g.s[k] = a.S[k * N + v];
  g.b = a.b[v];
  if (POST) {
    T uo = a.uin[v];
    if (a.e && i >= 1 && i <= a.nx - 2 && j >= 1 && j <= a.ny - 2) {
      const int ncx = (a.nx + 1) / 2, ncy = (a.ny + 1) / 2;
      const size_t NC = size_t(ncx) * ncy;
      const size_t c = size_t(j >> 1) * ncx + (i >> 1);
      const T* P = a.P;
      const T* e = a.e;
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
      uo = uo + corr;
    }
    g.u = uo;
  } else if (a.uin) {
    g.u = a.uin[v];
  }
}

template <class T, int BW>
__device__ __forceinline__ void store_row(const Ring<T>& R, int t, int j, const RowRegs<T>& g) {
  R.u[(j & (RU - 1)) * BW + t] = g.u;
  R.b[(j & (RS - 1)) * BW + t] = g.b;
#pragma unroll
  for (int k = 0; k < 5; ++k) R.S[(k * RS + (j & (RS - 1))) * BW + t] = g.s[k];
}

__device__ __forceinline__ double block_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double ws[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) ws[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < int(blockDim.x >> 6); ++k) t += ws[k];
  return t;
}

template <class T, int BW, bool POST>
__global__ __launch_bounds__(BW) void k_strip(StripArgs<T> a) {
  if (a.stop && *a.stop) return;
  extern __shared__ __align__(16) unsigned char smem[];
  T* base = reinterpret_cast<T*>(smem);
  Ring<T> R{base, base + RU * BW, base + (RU + 5 * RS) * BW, base + (RU + 6 * RS) * BW};

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
  const int out_w = BW - 2 * HALO;
  const int x0 = strip * out_w;
  const int i = x0 - HALO + t;
  const int j0 = seg * a.seg_h;
  const int j1 = min(j0 + a.seg_h, a.ny);
  // first A-row: the largest row of parity pf not after j0-2 (pre) / j0-1 (post)
  const int lim = POST ? j0 - 1 : j0 - 2;
  const int a0 = lim - (((lim - a.pf) % 2) + 2) % 2;
  // last A-row: residual rows up to j1-1 must be complete -> front a >= j1
  const int alast = j1 + (((j1 - a.pf) % 2) + 2) % 2;

  // zero the ring, then prime it with row a0-1
  for (int k = t; k < (RU + 7 * RS) * BW; k += BW) base[k] = T(0);
  __syncthreads();
  RowRegs<T> g0, g1;
  if (active) {
    load_row<T, POST>(a, i, a0 - 1, g0);
    store_row<T, BW>(R, t, a0 - 1, g0);
    load_row<T, POST>(a, i, a0, g0);
    load_row<T, POST>(a, i, a0 + 1, g1);
  }
  __syncthreads();
  double acc = 0.0;
  const bool out_col = active && t >= HALO && t < BW - HALO && i < a.nx;
  const int ncx = (a.nx + 1) / 2, ncy = (a.ny + 1) / 2;

  for (int ar = a0; active && ar <= alast; ar += 2) {
    store_row<T, BW>(R, t, ar, g0);
    store_row<T, BW>(R, t, ar + 1, g1);
    __syncthreads();
    if (ar + 2 <= alast) {  // prefetch the next two rows while this step computes
      load_row<T, POST>(a, i, ar + 2, g0);
      load_row<T, POST>(a, i, ar + 3, g1);
    }
    // restriction weights of this step's coarse row, loaded now and used after the sweep
    const int fj = (ar - 2) & ~1;  // fine row 2J of the coarse row restricted in this step
    const int J = fj >> 1;
    const int I = i >> 1;
    const bool do_restrict = !POST && out_col && !(i & 1) && fj >= j0 && fj < j1;
    const bool inner_c = I >= 1 && I <= ncx - 2 && J >= 1 && J <= ncy - 2;
    T pw[8];
    if (do_restrict && inner_c) {
      const size_t NC = size_t(ncx) * ncy;
      const size_t c = size_t(J) * ncx + I;
      const T* P = a.P;
      pw[0] = P[7 * NC + c - ncx - 1];
      pw[1] = P[3 * NC + c - ncx];
      pw[2] = P[6 * NC + c - ncx];
      pw[3] = P[1 * NC + c - 1];
      pw[4] = P[0 * NC + c];
      pw[5] = P[5 * NC + c - 1];
      pw[6] = P[2 * NC + c];
      pw[7] = P[4 * NC + c];
    }
    // A-row ar: column parity cA first, then the other
    if ((i & 1) == a.cA) gs_point<T, BW>(R, t, i, ar, a.nx, a.ny);
    __syncthreads();
    if ((i & 1) != a.cA) gs_point<T, BW>(R, t, i, ar, a.nx, a.ny);
    __syncthreads();
    // B-row ar-1
    if ((i & 1) == a.cB) gs_point<T, BW>(R, t, i, ar - 1, a.nx, a.ny);
    __syncthreads();
    if ((i & 1) != a.cB) gs_point<T, BW>(R, t, i, ar - 1, a.nx, a.ny);
    __syncthreads();
    // rows ar-1 and ar are final: write them out
    if (out_col) {
      const int rows[2] = {ar - 1, ar};
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int j = rows[q];
        if (j >= j0 && j < j1) a.u[size_t(j) * a.nx + i] = R.u[(j & (RU - 1)) * BW + t];
      }
    }
    // residual rows ar-2 and ar-1
    const T r2 = resid_point<T, BW>(R, t, i, ar - 2, a.nx, a.ny);
    const T r1 = resid_point<T, BW>(R, t, i, ar - 1, a.nx, a.ny);
    if (POST) {
      if (out_col && a.partials) {
        if (ar - 2 >= j0 && ar - 2 < j1) acc += double(r2) * double(r2);
        if (ar - 1 >= j0 && ar - 1 < j1) acc += double(r1) * double(r1);
      }
    } else {
      R.r[((ar - 2) & (RS - 1)) * BW + t] = r2;
      R.r[((ar - 1) & (RS - 1)) * BW + t] = r1;
      __syncthreads();
      // restriction for the coarse row whose fine rows 2J-1..2J+1 are now complete
      if (do_restrict) {
        T acc2 = T(0);
        if (inner_c) {
          const T* rm = R.r + ((fj - 1) & (RS - 1)) * BW;
          const T* r0 = R.r + (fj & (RS - 1)) * BW;
          const T* rp = R.r + ((fj + 1) & (RS - 1)) * BW;
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
  }
  if (POST && a.partials) {
    const double s = block_sum(acc);
    if (t == 0) a.partials[blockIdx.x] = s;
  }
}

// -----------------------------------------------------------------------------------------
// Coarse tail: one workgroup runs the V-cycle from level `top` down to the coarsest level
// and back, with workgroup barriers between the colour passes.  Level data lives in the
// hierarchy arrays (small enough to stay in L2).
// -----------------------------------------------------------------------------------------
template <class T>
struct TailLevel {
  const T* S;
  T* u;
  T* b;
  T* r;
  const T* P;
  int nx, ny;
};

constexpr int kMaxTail = 12;

template <class T>
struct TailArgs {
  TailLevel<T> L[kMaxTail];
  int nlev;           // levels in the tail (the last one is the coarsest)
  int zero_top;       // the top level starts from u = 0 (it is a coarse level)
  int m;              // coarsest unknowns
  const int* idx;
  const double* chol;
  int pre[4], post[4];
  int nu_pre, nu_post;
  const int* stop;
};

template <class T>
__device__ __forceinline__ T offdiag_g(const T* __restrict__ S, const T* __restrict__ u, size_t N,
                                       int nx, size_t v) {
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
__device__ void tail_colour(const TailLevel<T>& L, int c) {
  const int ci = c & 1, cj = c >> 1;
  const int px = (L.nx - ci + 1) / 2, py = (L.ny - cj + 1) / 2;
  const size_t N = size_t(L.nx) * L.ny;
  for (int k = threadIdx.x; k < px * py; k += blockDim.x) {
    const int i = ci + 2 * (k % px), j = cj + 2 * (k / px);
    if (i <= 0 || i >= L.nx - 1 || j <= 0 || j >= L.ny - 1) continue;
    const size_t v = size_t(j) * L.nx + i;
    L.u[v] = (L.b[v] - offdiag_g(L.S, L.u, N, L.nx, v)) / L.S[v];
  }
  __syncthreads();
}

template <class T>
__global__ __launch_bounds__(1024) void k_tail(TailArgs<T> a) {
  if (a.stop && *a.stop) return;
  extern __shared__ double y[];
  const int nl = a.nlev;
  for (int l = 0; l < nl - 1; ++l) {
    const TailLevel<T>& L = a.L[l];
    const size_t N = size_t(L.nx) * L.ny;
    if (l > 0 || a.zero_top)
      for (size_t v = threadIdx.x; v < N; v += blockDim.x) L.u[v] = T(0);
    __syncthreads();
    for (int s = 0; s < a.nu_pre; ++s)
      for (int c = 0; c < 4; ++c) tail_colour(L, a.pre[c]);
    for (size_t v = threadIdx.x; v < N; v += blockDim.x) {
      const int i = int(v % L.nx), j = int(v / L.nx);
      T r = T(0);
      if (i > 0 && i < L.nx - 1 && j > 0 && j < L.ny - 1)
        r = L.b[v] - (offdiag_g(L.S, L.u, N, L.nx, v) + L.S[v] * L.u[v]);
      L.r[v] = r;
    }
    __syncthreads();
    const TailLevel<T>& Cn = a.L[l + 1];
    const int ncx = Cn.nx, ncy = Cn.ny;
    const size_t NC = size_t(ncx) * ncy;
    for (size_t c = threadIdx.x; c < NC; c += blockDim.x) {
      const int I = int(c % ncx), J = int(c / ncx);
      T acc = T(0);
      if (I > 0 && I < ncx - 1 && J > 0 && J < ncy - 1) {
        const T* P = L.P;
        const T* r = L.r;
        const size_t f = size_t(2 * J) * L.nx + 2 * I;
        const int nx = L.nx;
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
      Cn.b[c] = acc;
    }
    __syncthreads();
  }
  // coarsest: dense Cholesky solve in float64
  {
    const TailLevel<T>& C = a.L[nl - 1];
    const size_t N = size_t(C.nx) * C.ny;
    const int m = a.m;
    const double* L = a.chol;
    for (size_t v = threadIdx.x; v < N; v += blockDim.x) C.u[v] = T(0);
    for (int k = threadIdx.x; k < m; k += blockDim.x) y[k] = double(C.b[a.idx[k]]);
    __syncthreads();
    for (int k = 0; k < m; ++k) {
      if (threadIdx.x == 0) y[k] /= L[k * m + k];
      __syncthreads();
      for (int r = k + 1 + threadIdx.x; r < m; r += blockDim.x) y[r] -= L[r * m + k] * y[k];
      __syncthreads();
    }
    for (int k = m - 1; k >= 0; --k) {
      if (threadIdx.x == 0) y[k] /= L[k * m + k];
      __syncthreads();
      for (int r = threadIdx.x; r < k; r += blockDim.x) y[r] -= L[k * m + r] * y[k];
      __syncthreads();
    }
    for (int k = threadIdx.x; k < m; k += blockDim.x) C.u[a.idx[k]] = T(y[k]);
    __syncthreads();
  }
  for (int l = nl - 2; l >= 0; --l) {
    const TailLevel<T>& L = a.L[l];
    const TailLevel<T>& Cn = a.L[l + 1];
    const int ncx = Cn.nx, ncy = Cn.ny;
    const size_t NC = size_t(ncx) * ncy;
    const size_t N = size_t(L.nx) * L.ny;
    for (size_t v = threadIdx.x; v < N; v += blockDim.x) {
      const int i = int(v % L.nx), j = int(v / L.nx);
      if (i <= 0 || i >= L.nx - 1 || j <= 0 || j >= L.ny - 1) continue;
      const size_t c = size_t(j >> 1) * ncx + (i >> 1);
      const T* P = L.P;
      const T* e = Cn.u;
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
      L.u[v] = L.u[v] + corr;
    }
    __syncthreads();
    for (int s = 0; s < a.nu_post; ++s)
      for (int c = 0; c < 4; ++c) tail_colour(L, a.post[c]);
  }
}

}  // namespace

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
                        int cA, int cB, const int* stop, hipStream_t s) {
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
  const int nb = strip_blocks(nx, ny, cfg.bw, cfg.seg_h, &a.nstrips, &a.nsegs);
  const size_t lds = size_t(RU + 7 * RS) * cfg.bw * sizeof(T);
  switch (cfg.bw) {
    case 64:
      k_strip<T, 64, POST><<<nb, 64, lds, s>>>(a);
      break;
    case 128:
      k_strip<T, 128, POST><<<nb, 128, lds, s>>>(a);
      break;
    case 256:
      k_strip<T, 256, POST><<<nb, 256, lds, s>>>(a);
      break;
    default:
      return fail(DMG_ERR_INVALID_ARG, "unsupported strip width %d", cfg.bw);
  }
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
                       int cB, const int* stop, hipStream_t s) {
  return launch_strip<T, true>(cfg, S, uin, u, b, P, nullptr, e, partials, nx, ny, pf, cA, cB,
                               stop, s);
}

template <class T>
dmg_status launch_tail(const TailSpec<T>& spec, hipStream_t s) {
  TailArgs<T> a;
  if (spec.nlev > kMaxTail) return fail(DMG_ERR_INVALID_ARG, "tail too deep (%d)", spec.nlev);
  for (int l = 0; l < spec.nlev; ++l) {
    a.L[l].S = spec.S[l];
    a.L[l].u = spec.u[l];
    a.L[l].b = spec.b[l];
    a.L[l].r = spec.r[l];
    a.L[l].P = spec.P[l];
    a.L[l].nx = spec.nx[l];
    a.L[l].ny = spec.ny[l];
  }
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
  a.stop = spec.stop;
  k_tail<T><<<1, 1024, sizeof(double) * size_t(spec.m > 0 ? spec.m : 1), s>>>(a);
  return launch_check("tail");
}

#define DMG_INST(T)                                                                            \
  template dmg_status launch_pre<T>(const StripConfig&, const T*, const T*, T*, const T*,      \
                                    const T*, T*, int, int, int, int, int, const int*,         \
                                    hipStream_t);                                              \
  template dmg_status launch_post<T>(const StripConfig&, const T*, const T*, T*, const T*,     \
                                     const T*, const T*, double*, int, int, int, int, int,     \
                                     const int*, hipStream_t);                                 \
  template dmg_status launch_tail<T>(const TailSpec<T>&, hipStream_t);
DMG_INST(double)
DMG_INST(float)
#undef DMG_INST

}  // namespace dmg
