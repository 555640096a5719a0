// V-cycles with zebra line relaxation, the smoother for anisotropic operators, in float64 or (the
// inner cycles of float32 refinement) float32: every kernel is a template on the arithmetic type,
// reading that precision's copies of the stencil, weights and line factors.
//
// A line sweep solves, for every interior line of one parity, the line's own equations exactly
// with the unknowns of the other lines held: the tridiagonal system of the couplings along the
// line, right-hand side b minus the couplings to the two neighbouring lines.  Lines of one parity
// are not coupled by a 9-point stencil, so they are solved at once, one wavefront per line, by
// the Thomas algorithm.  Its factors (modified super-diagonal, reciprocal pivots) depend on the
// stencil only and are computed at setup, so a sweep is a forward pass d = (rhs - a d') / m into
// scratch, which only reads u, and a back substitution into the line of u; both recurrences are
// split over the 64 lanes of the line's wavefront through a scan of their affine maps.
//
// Levels above the coarse tail run these unfused kernels: sweeps, residual, restriction P^T r,
// interpolation u += P e, sweeps in reverse order; the tail levels run in the one-workgroup
// coarse kernel with its own line sweeps.  Every kernel is a no-op once *stop (nullable) is set.
#include <algorithm>

#include "dmg_internal.h"

namespace dmg {
namespace {

__device__ __forceinline__ bool halted(const int* stop) { return stop && *stop; }

// 2x2 matrix t <- t / 2^e with 2^e the power of two at or above its largest entry: an exact
// rescaling, which leaves the ratio p / q it produces unchanged and keeps long products finite.
template <class T>
__device__ __forceinline__ void rescale(T t[4]) {
  const T mx = fmax(fmax(fabs(t[0]), fabs(t[1])), fmax(fabs(t[2]), fabs(t[3])));
  if (!(mx > 0.0) || !isfinite(mx)) return;
  int ex = 0;
  (void)frexp(mx, &ex);
#pragma unroll
  for (int k = 0; k < 4; ++k) t[k] = ldexp(t[k], -ex);
}

// Thomas factors of every interior line (DIR 0: rows, DIR 1: columns), one wavefront per line.
// Walking the line, the pivot is m_k = C_k - a_k cp_{k-1} (a the sub-diagonal: W along x, S
// along y) and cp_k = e_k / m_k with e_k the super-diagonal (W or S of the next point), stored
// as cp and 1 / m; they depend on the stencil only, so the sweeps need no divisions.  The map
// cp_{k-1} -> cp_k is projective: with cp = p / q it is (p, q) -> (e q, C q - a p), a 2x2 matrix.
// Lane p multiplies the matrices of its chunk of consecutive points (as in the sweeps), a scan
// over the lanes gives each chunk its incoming cp, and the lane then runs the recurrence itself
// over its points (lane 0 exactly as the sequential recurrence).
template <int DIR, class T>
__global__ __launch_bounds__(256) void k_line_factor_scan(const T* __restrict__ S,
                                                          T* __restrict__ lf, int nx, int ny) {
  const size_t N = size_t(nx) * ny;
  const int lane = int(threadIdx.x) & 63;
  const int line = 1 + int(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const int len = DIR == 0 ? nx : ny, count = DIR == 0 ? ny : nx;
  if (line > count - 2) return;  // the whole wavefront
  const int n = len - 2;
  const int L = (n + 63) / 64;
  const int k0 = 1 + lane * L, k1 = min(1 + (lane + 1) * L, n + 1);
  const size_t step = DIR == 0 ? 1 : size_t(nx);
  const size_t v0 = DIR == 0 ? size_t(line) * nx : size_t(line);
  const T* C = S;
  const T* a = S + (DIR == 0 ? N : 2 * N);
  T* cpo = lf + (DIR == 0 ? 0 : 2 * N);
  T* imo = lf + (DIR == 0 ? N : 3 * N);
  T t[4] = {T(1), T(0), T(0), T(1)};  // [[t0, t1], [t2, t3]] on (p, q)
  for (int k = k0; k < k1; ++k) {
    const size_t v = v0 + size_t(k) * step;
    const T e = a[v + step], c = C[v], w = a[v];
    const T n0 = e * t[2], n1 = e * t[3];
    const T n2 = c * t[2] - w * t[0], n3 = c * t[3] - w * t[1];
    t[0] = n0, t[1] = n1, t[2] = n2, t[3] = n3;
    rescale(t);
  }
  // inclusive scan: lane p holds the product of chunks 0..p (later chunks on the left)
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = __shfl_up(t[k], d, 64);
    if (lane >= d) {
      const T n0 = t[0] * q[0] + t[1] * q[2], n1 = t[0] * q[1] + t[1] * q[3];
      const T n2 = t[2] * q[0] + t[3] * q[2], n3 = t[2] * q[1] + t[3] * q[3];
      t[0] = n0, t[1] = n1, t[2] = n2, t[3] = n3;
      rescale(t);
    }
  }
  // incoming (p, q): the product of the earlier chunks applied to (0, 1)
  const T p_in = __shfl_up(t[1], 1, 64), q_in = __shfl_up(t[3], 1, 64);
  T pc = lane == 0 ? T(0) : p_in / q_in;
  for (int k = k0; k < k1; ++k) {
    const size_t v = v0 + size_t(k) * step;
    const T im = T(1) / (C[v] - a[v] * pc);
    pc = a[v + step] * im;
    cpo[v] = pc;
    imo[v] = im;
  }
}

// One line sweep: interior lines of one parity (DIR 0: x-lines = rows j, DIR 1: y-lines =
// columns i), one wavefront per line.  Stencil planes (planar, N = nx ny): C, W, S, SW, SE;
// E(i,j) = W(i+1,j), N(i,j) = S(i,j+1), NE(i,j) = SW(i+1,j+1), NW(i,j) = SE(i-1,j+1).  Along a
// line of n interior points k = 1..n, with x = b minus the couplings to the two neighbouring
// lines, a the sub-diagonal and the stored factors cp and 1 / m, the forward recurrence is
// pd_k = (x_k - a_k pd_{k-1}) / m_k (pd_0 = 0) and the back substitution u_k = pd_k - cp_k
// u_{k+1} (u_n = pd_n).  Both are affine in the carried value, so lane p takes the consecutive
// points k in [1 + p L, 1 + (p + 1) L) (L = ceil(n / 64)), composes its points' maps, a scan over
// the 64 lanes gives every lane its incoming value, and the lane then runs the recurrence itself
// over its points.  Lane 0's points round exactly as the sequential recurrence; a later lane's
// starting value comes from the composed maps, whose rounding differs at the level of a few ulps.
// dp (scratch) holds x, then pd.  u is read (neighbouring lines) and written (this line).
// (blk: the workgroup's index among the sweep's workgroups)
template <int DIR, class T>
__device__ __forceinline__ void line_scan_body(const T* __restrict__ S, const T* uin,
                                               const T* __restrict__ b, const T* __restrict__ lf,
                                               T* __restrict__ dp, int nx, int ny, int parity,
                                               T* u, unsigned blk) {
  const size_t N = size_t(nx) * ny;
  const int lane = int(threadIdx.x) & 63;
  const int first = parity == 0 ? 2 : 1;
  const int line = first + 2 * int(blk * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const int len = DIR == 0 ? nx : ny;     // points along a line, boundary included
  const int count = DIR == 0 ? ny : nx;   // lines
  if (line > count - 2) return;           // the whole wavefront
  const int n = len - 2;
  const int L = (n + 63) / 64;
  const int k0 = 1 + lane * L, k1 = min(1 + (lane + 1) * L, n + 1);  // may be empty
  const size_t step = DIR == 0 ? 1 : size_t(nx);
  const size_t v0 = DIR == 0 ? size_t(line) * nx : size_t(line);  // point k = 0 of the line
  const T *W = S + N, *So = S + 2 * N, *SW = S + 3 * N, *SE = S + 4 * N;
  const T* a = DIR == 0 ? W : So;  // coupling to the previous point of the line
  const T* cp = lf + (DIR == 0 ? 0 : 2 * N);
  const T* im = lf + (DIR == 0 ? N : 3 * N);
  // forward: x into dp; this lane's map pd_out = fa + fb pd_in
  T fa = T(0), fb = T(1);
  // (the unrolled loops keep the loads of several points in flight ahead of the recurrence)
#pragma unroll 4
  for (int k = k0; k < k1; ++k) {
    const size_t v = v0 + size_t(k) * step;
    T off;
    if (DIR == 0)
      off = ((((So[v] * uin[v - nx] + So[v + nx] * uin[v + nx]) + SW[v] * uin[v - nx - 1]) +
              SE[v] * uin[v - nx + 1]) +
             SE[v + nx - 1] * uin[v + nx - 1]) +
            SW[v + nx + 1] * uin[v + nx + 1];
    else
      off = ((((W[v] * uin[v - 1] + W[v + 1] * uin[v + 1]) + SW[v] * uin[v - nx - 1]) +
              SE[v] * uin[v - nx + 1]) +
             SE[v + nx - 1] * uin[v + nx - 1]) +
            SW[v + nx + 1] * uin[v + nx + 1];
    const T x = b[v] - off;
    dp[v] = x;
    const T av = a[v], m = im[v];
    fa = (x - av * fa) * m;
    fb = -(av * fb) * m;
  }
  // inclusive scan of the maps over the lanes (lane p after lane p - 1), then the incoming value
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T pa = __shfl_up(fa, d, 64), pb = __shfl_up(fb, d, 64);
    if (lane >= d) {
      fa = fa + fb * pa;
      fb = fb * pb;
    }
  }
  T pd = __shfl_up(fa, 1, 64);
  if (lane == 0) pd = T(0);
#pragma unroll 4
  for (int k = k0; k < k1; ++k) {
    const size_t v = v0 + size_t(k) * step;
    pd = (dp[v] - a[v] * pd) * im[v];
    dp[v] = pd;
  }
  // backward: this lane's map u_{k0} = ba + bb u_{k1} (cp of the last point taken as 0)
  T ba = T(0), bb = T(1);
#pragma unroll 4
  for (int k = k1 - 1; k >= k0; --k) {
    const size_t v = v0 + size_t(k) * step;
    const T c = k == n ? T(0) : cp[v];
    ba = dp[v] - c * ba;
    bb = -(c * bb);
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T na = __shfl_down(ba, d, 64), nb = __shfl_down(bb, d, 64);
    if (lane + d < 64) {
      ba = ba + bb * na;
      bb = bb * nb;
    }
  }
  T x = __shfl_down(ba, 1, 64);
  if (lane == 63) x = T(0);
#pragma unroll 4
  for (int k = k1 - 1; k >= k0; --k) {
    const size_t v = v0 + size_t(k) * step;
    const T c = k == n ? T(0) : cp[v];
    x = dp[v] - c * x;
    u[v] = x;
  }
}

template <int DIR, class T>
__global__ __launch_bounds__(256) void k_line_scan(const T* __restrict__ S, const T* uin,
                                                   const T* __restrict__ b,
                                                   const T* __restrict__ lf, T* __restrict__ dp,
                                                   int nx, int ny, int parity,
                                                   const int* __restrict__ stop, T* u) {
  if (halted(stop)) return;
  line_scan_body<DIR, T>(S, uin, b, lf, dp, nx, ny, parity, u, blockIdx.x);
}

// The same sweep over the instances of a batch that share one level size: instance blockIdx.y.
template <int DIR, class T>
__global__ __launch_bounds__(256) void k_line_scan_multi(const LineArgs<T>* __restrict__ list,
                                                         int parity) {
  const LineArgs<T> a = list[blockIdx.y];
  if (halted(a.stop)) return;
  line_scan_body<DIR, T>(a.S, a.u, a.b, a.lf, a.r, a.nx, a.ny, parity, a.u, blockIdx.x);
}

// r = b - A u on interior points, 0 on the boundary ring (blk of nblk workgroups, grid-stride).
template <class T>
__device__ __forceinline__ void line_resid_body(const T* __restrict__ S, const T* __restrict__ u,
                                                const T* __restrict__ b, T* __restrict__ r,
                                                int nx, int ny, unsigned blk, unsigned nblk) {
  const size_t N = size_t(nx) * ny;
  for (size_t v = blk * 256u + threadIdx.x; v < N; v += size_t(nblk) * 256u) {
    const int j = int(v / nx), i = int(v % nx);
    if (i > 0 && i < nx - 1 && j > 0 && j < ny - 1) {
      const T off = ((((((S[3 * N + v] * u[v - nx - 1] + S[2 * N + v] * u[v - nx]) +
                              S[4 * N + v] * u[v - nx + 1]) +
                             S[N + v] * u[v - 1]) +
                            S[N + v + 1] * u[v + 1]) +
                           S[4 * N + v + nx - 1] * u[v + nx - 1]) +
                          S[2 * N + v + nx] * u[v + nx]) +
                         S[3 * N + v + nx + 1] * u[v + nx + 1];
      r[v] = b[v] - (off + S[v] * u[v]);
    } else {
      r[v] = T(0);
    }
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_line_resid(const T* __restrict__ S,
                                                    const T* __restrict__ u,
                                                    const T* __restrict__ b, T* __restrict__ r,
                                                    int nx, int ny,
                                                    const int* __restrict__ stop) {
  if (halted(stop)) return;
  line_resid_body<T>(S, u, b, r, nx, ny, blockIdx.x, gridDim.x);
}

// b_H = P^T r on interior coarse points (boundary 0).  P per coarse cell c = J ncx + I: planes
// 0-1 the x-line weights of fine (2I+1, 2J) on coarse (I, J), (I+1, J); 2-3 the y-line weights
// of (2I, 2J+1) on (I, J), (I, J+1); 4-7 the centre weights of (2I+1, 2J+1) on (I, J), (I+1, J),
// (I, J+1), (I+1, J+1).
template <class T>
__device__ __forceinline__ void line_restrict_body(const T* __restrict__ P,
                                                   const T* __restrict__ r, T* __restrict__ bH,
                                                   int nx, int ny, unsigned blk, unsigned nblk) {
  const int ncx = (nx + 1) / 2, ncy = (ny + 1) / 2;
  const size_t NC = size_t(ncx) * ncy;
  for (size_t k = blk * 256u + threadIdx.x; k < NC; k += size_t(nblk) * 256u) {
    const int J = int(k / ncx), I = int(k % ncx);
    if (I == 0 || I == ncx - 1 || J == 0 || J == ncy - 1) {
      bH[k] = T(0);
      continue;
    }
    const size_t f = size_t(2 * J) * nx + 2 * I;  // fine (2I, 2J)
    const size_t c = k, cw = k - 1, cs = k - ncx, csw = k - ncx - 1;
    T acc = r[f];
    acc += P[c] * r[f + 1] + P[NC + cw] * r[f - 1];
    acc += P[2 * NC + c] * r[f + nx] + P[3 * NC + cs] * r[f - nx];
    acc += P[4 * NC + c] * r[f + nx + 1] + P[5 * NC + cw] * r[f + nx - 1];
    acc += P[6 * NC + cs] * r[f - nx + 1] + P[7 * NC + csw] * r[f - nx - 1];
    bH[k] = acc;
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_line_restrict(const T* __restrict__ P,
                                                       const T* __restrict__ r,
                                                       T* __restrict__ bH, int nx, int ny,
                                                       const int* __restrict__ stop) {
  if (halted(stop)) return;
  line_restrict_body<T>(P, r, bH, nx, ny, blockIdx.x, gridDim.x);
}

// u += P e on interior fine points.
template <class T>
__device__ __forceinline__ void line_prolong_body(const T* __restrict__ P,
                                                  const T* __restrict__ e, T* __restrict__ u,
                                                  int nx, int ny, unsigned blk, unsigned nblk) {
  const int ncx = (nx + 1) / 2, ncy = (ny + 1) / 2;
  const size_t NC = size_t(ncx) * ncy, N = size_t(nx) * ny;
  for (size_t v = blk * 256u + threadIdx.x; v < N; v += size_t(nblk) * 256u) {
    const int j = int(v / nx), i = int(v % nx);
    if (i == 0 || i == nx - 1 || j == 0 || j == ny - 1) continue;
    const size_t c = size_t(j >> 1) * ncx + (i >> 1);
    T x;
    if (!(i & 1) && !(j & 1))
      x = e[c];
    else if ((i & 1) && !(j & 1))
      x = P[c] * e[c] + P[NC + c] * e[c + 1];
    else if (!(i & 1) && (j & 1))
      x = P[2 * NC + c] * e[c] + P[3 * NC + c] * e[c + ncx];
    else
      x = ((P[4 * NC + c] * e[c] + P[5 * NC + c] * e[c + 1]) + P[6 * NC + c] * e[c + ncx]) +
          P[7 * NC + c] * e[c + ncx + 1];
    u[v] += x;
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_line_prolong(const T* __restrict__ P,
                                                      const T* __restrict__ e, T* __restrict__ u,
                                                      int nx, int ny,
                                                      const int* __restrict__ stop) {
  if (halted(stop)) return;
  line_prolong_body<T>(P, e, u, nx, ny, blockIdx.x, gridDim.x);
}

// The unfused steps of a batched line V-cycle over the instances of one level size (instance
// blockIdx.y): u = 0 (a coarse level's start), r = b - A u then b_H = P^T r, u += P e.
template <class T>
__global__ __launch_bounds__(256) void k_line_zero_multi(const LineArgs<T>* __restrict__ list) {
  const LineArgs<T> a = list[blockIdx.y];
  if (halted(a.stop)) return;
  const size_t N = size_t(a.nx) * a.ny;
  for (size_t v = blockIdx.x * 256u + threadIdx.x; v < N; v += size_t(gridDim.x) * 256u)
    a.u[v] = T(0);
}
template <class T>
__global__ __launch_bounds__(256) void k_line_resid_multi(const LineArgs<T>* __restrict__ list) {
  const LineArgs<T> a = list[blockIdx.y];
  if (halted(a.stop)) return;
  line_resid_body<T>(a.S, a.u, a.b, a.r, a.nx, a.ny, blockIdx.x, gridDim.x);
}
template <class T>
__global__ __launch_bounds__(256) void k_line_restrict_multi(const LineArgs<T>* __restrict__ list) {
  const LineArgs<T> a = list[blockIdx.y];
  if (halted(a.stop)) return;
  line_restrict_body<T>(a.P, a.r, a.bH, a.nx, a.ny, blockIdx.x, gridDim.x);
}
template <class T>
__global__ __launch_bounds__(256) void k_line_prolong_multi(const LineArgs<T>* __restrict__ list) {
  const LineArgs<T> a = list[blockIdx.y];
  if (halted(a.stop)) return;
  line_prolong_body<T>(a.P, a.e, a.u, a.nx, a.ny, blockIdx.x, gridDim.x);
}

unsigned grid_blocks(size_t n) {
  return unsigned(std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 16384)));
}

// the pre-smoothing sweeps of smoother s as (direction, parity): 0 = x-lines, 1 = y-lines
int line_sweeps(int smoother, int dir[4], int par[4]) {
  int n = 0;
  if (smoother == 1 || smoother == 3) {
    dir[n] = 0, par[n++] = 0;
    dir[n] = 0, par[n++] = 1;
  }
  if (smoother == 2 || smoother == 3) {
    dir[n] = 1, par[n++] = 0;
    dir[n] = 1, par[n++] = 1;
  }
  return n;
}

// The arrays of level L in precision T: stencil (planar), weights, line factors, residual
// scratch, right-hand side.
template <class T>
struct LineArrays;
template <>
struct LineArrays<double> {
  const double *S, *P, *lf;
  double *r, *b;
  explicit LineArrays(const Level& L) : S(L.S), P(L.P), lf(L.lf), r(L.r), b(L.b) {}
};
template <>
struct LineArrays<float> {
  const float *S, *P, *lf;
  float *r, *b;
  explicit LineArrays(const Level& L) : S(L.S32), P(L.P32), lf(L.lf32), r(L.r32), b(L.b32) {}
};

}  // namespace

template <class T>
dmg_status line_sweep(const Level& L, T* u, const T* b, int smoother, bool pre, const int* stop,
                      hipStream_t s) {
  const LineArrays<T> A(L);
  int dir[4], par[4];
  const int n = line_sweeps(smoother, dir, par);
  for (int k = 0; k < n; ++k) {
    const int q = pre ? k : n - 1 - k;
    // dp scratch: r (free during the sweeps); one wavefront per line, four per workgroup
    if (dir[q] == 0) {
      const int lines = (L.ny - 2 + 1) / 2;
      k_line_scan<0, T><<<(lines + 3) / 4, 256, 0, s>>>(A.S, u, b, A.lf, A.r, L.nx, L.ny, par[q],
                                                        stop, u);
    } else {
      const int lines = (L.nx - 2 + 1) / 2;
      k_line_scan<1, T><<<(lines + 3) / 4, 256, 0, s>>>(A.S, u, b, A.lf, A.r, L.nx, L.ny, par[q],
                                                        stop, u);
    }
    DMG_CHECK(launch_check("line sweep"));
  }
  return DMG_OK;
}

template <class T>
dmg_status line_factors(const Level& L, hipStream_t s) {
  const LineArrays<T> A(L);
  T* lf = const_cast<T*>(A.lf);
  k_line_factor_scan<0, T><<<(L.ny - 2 + 3) / 4, 256, 0, s>>>(A.S, lf, L.nx, L.ny);
  DMG_CHECK(launch_check("line factors x"));
  k_line_factor_scan<1, T><<<(L.nx - 2 + 3) / 4, 256, 0, s>>>(A.S, lf, L.nx, L.ny);
  return launch_check("line factors y");
}

template <class T>
dmg_status line_resid_restrict(const Level& L, const Level& Lc, const T* u, const T* b,
                               const int* stop, hipStream_t s) {
  const LineArrays<T> A(L);
  T* bc = LineArrays<T>(Lc).b;
  k_line_resid<T><<<grid_blocks(L.n()), 256, 0, s>>>(A.S, u, b, A.r, L.nx, L.ny, stop);
  DMG_CHECK(launch_check("line residual"));
  k_line_restrict<T><<<grid_blocks(Lc.n()), 256, 0, s>>>(A.P, A.r, bc, L.nx, L.ny, stop);
  return launch_check("line restriction");
}

template <class T>
dmg_status line_prolong(const Level& L, const T* e, T* u, const int* stop, hipStream_t s) {
  const LineArrays<T> A(L);
  k_line_prolong<T><<<grid_blocks(L.n()), 256, 0, s>>>(A.P, e, u, L.nx, L.ny, stop);
  return launch_check("line interpolation");
}

dmg_status launch_line_multi(LineStep step, const LineArgs<double>* list, int count, int nx,
                             int ny, int dir, int parity, hipStream_t s) {
  if (count <= 0) return DMG_OK;
  const size_t n = size_t(nx) * ny;
  // grid-stride steps: enough workgroups per instance that the launch fills the GPU
  const unsigned per = std::max(1u, std::min(grid_blocks(n), unsigned(4096 / count + 1)));
  switch (step) {
    case LineStep::kSweep: {
      const int lines = dir == 0 ? (ny - 2 + 1) / 2 : (nx - 2 + 1) / 2;
      const dim3 grid(unsigned((lines + 3) / 4), unsigned(count));
      if (dir == 0) k_line_scan_multi<0, double><<<grid, 256, 0, s>>>(list, parity);
      else k_line_scan_multi<1, double><<<grid, 256, 0, s>>>(list, parity);
      return launch_check("batched line sweep");
    }
    case LineStep::kZero:
      k_line_zero_multi<double><<<dim3(per, unsigned(count)), 256, 0, s>>>(list);
      return launch_check("batched coarse start");
    case LineStep::kResidual:
      k_line_resid_multi<double><<<dim3(per, unsigned(count)), 256, 0, s>>>(list);
      return launch_check("batched line residual");
    case LineStep::kRestrict: {
      const size_t nc = size_t((nx + 1) / 2) * ((ny + 1) / 2);
      const unsigned pc = std::max(1u, std::min(grid_blocks(nc), unsigned(4096 / count + 1)));
      k_line_restrict_multi<double><<<dim3(pc, unsigned(count)), 256, 0, s>>>(list);
      return launch_check("batched line restriction");
    }
    case LineStep::kProlong:
      k_line_prolong_multi<double><<<dim3(per, unsigned(count)), 256, 0, s>>>(list);
      return launch_check("batched line interpolation");
  }
  return fail(DMG_ERR_INVALID_ARG, "unknown batched line step");
}

#define DMG_LINE_INST(T)                                                                       \
  template dmg_status line_sweep<T>(const Level&, T*, const T*, int, bool, const int*,         \
                                    hipStream_t);                                              \
  template dmg_status line_factors<T>(const Level&, hipStream_t);                              \
  template dmg_status line_resid_restrict<T>(const Level&, const Level&, const T*, const T*,   \
                                             const int*, hipStream_t);                         \
  template dmg_status line_prolong<T>(const Level&, const T*, T*, const int*, hipStream_t);
DMG_LINE_INST(double)
DMG_LINE_INST(float)
#undef DMG_LINE_INST

}  // namespace dmg
