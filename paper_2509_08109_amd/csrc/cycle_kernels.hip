// Small cycle-side kernels: deterministic norms and the device convergence check (single and
// multi-instance), fills and copies.  The sweeps themselves live in fused_kernels.hip.
#include "dmg_internal.h"

namespace dmg {
namespace {

// Off-diagonal part of row (i,j) applied to u, summed in ascending neighbour index order.
template <class T>
__device__ __forceinline__ T offdiag(const T* __restrict__ S, const T* __restrict__ u, size_t N,
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


// y = A x on interior rows; the boundary ring of y is set to 0.
__global__ __launch_bounds__(256) void k_stencil_apply(const double* __restrict__ S,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ y, int nx, int ny) {
  const size_t N = size_t(nx) * ny;
  for (size_t v = blockIdx.x * size_t(blockDim.x) + threadIdx.x; v < N;
       v += size_t(gridDim.x) * blockDim.x) {
    const int j = int(v / nx), i = int(v % nx);
    if (i > 0 && i < nx - 1 && j > 0 && j < ny - 1)
      y[v] = offdiag(S, x, N, nx, v) + S[v] * x[v];
    else
      y[v] = 0.0;
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_copy(const T* __restrict__ x, T* __restrict__ y, size_t n,
                                              const int* __restrict__ stop) {
  if (stop && *stop) return;
  for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < n;
       k += size_t(gridDim.x) * blockDim.x)
    y[k] = x[k];
}

template <class T>
__global__ __launch_bounds__(256) void k_fill(T* __restrict__ x, T val, size_t n) {
  for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < n;
       k += size_t(gridDim.x) * blockDim.x)
    x[k] = val;
}

// ---- deterministic reductions ---------------------------------------------------------
__device__ __forceinline__ double block_sum(double v) {
  // 64-lane wavefront tree, then the 4 wavefront sums in order.
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double ws[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();  // earlier readers of ws (a previous call) are done
  if (lane == 0) ws[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = ((ws[0] + ws[1]) + ws[2]) + ws[3];
  return t;
}

// partials[blk] = sum over interior rows assigned to blk of (b - A u)^2.  When *zero is set
// (u is zero everywhere) the residual is b: the block copies its b-norm partial pb[blk] (k_sq's,
// which sums the same terms in the same order) instead of reading S and u.
__global__ __launch_bounds__(256) void k_resid_sq(const double* __restrict__ S,
                                                  const double* __restrict__ u,
                                                  const double* __restrict__ b, int nx, int ny,
                                                  double* __restrict__ partials,
                                                  const int* __restrict__ stop,
                                                  const int* __restrict__ zero,
                                                  const double* __restrict__ pb) {
  if (stop && *stop) return;
  if (zero && *zero) {
    if (threadIdx.x == 0) partials[blockIdx.x] = pb[blockIdx.x];
    return;
  }
  const size_t N = size_t(nx) * ny;
  const size_t m = size_t(nx - 2) * (ny - 2);
  double acc = 0.0;
  for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < m;
       k += size_t(gridDim.x) * blockDim.x) {
    const size_t jj = k / (nx - 2), ii = k % (nx - 2);
    const size_t v = (jj + 1) * nx + ii + 1;
    const double r = b[v] - (offdiag(S, u, N, nx, v) + S[v] * u[v]);
    acc += r * r;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// partials[blk] = sum of x^2 over the interior points assigned to blk; with u, also
// nonzero[blk] = number of the entries of u (every point, boundary included) assigned to blk
// that are not zero (NaN counts as not zero).
__global__ __launch_bounds__(256) void k_sq(const double* __restrict__ x, int nx, int ny,
                                            double* __restrict__ partials,
                                            const double* __restrict__ u,
                                            double* __restrict__ nonzero) {
  const size_t m = size_t(nx - 2) * (ny - 2);
  double acc = 0.0;
  for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < m;
       k += size_t(gridDim.x) * blockDim.x) {
    const size_t jj = k / (nx - 2), ii = k % (nx - 2);
    const double v = x[(jj + 1) * nx + ii + 1];
    acc += v * v;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
  if (!u) return;
  const size_t n = size_t(nx) * ny;
  double cnt = 0.0;
  for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < n;
       k += size_t(gridDim.x) * blockDim.x)
    cnt += u[k] == 0.0 ? 0.0 : 1.0;
  const double c = block_sum(cnt);
  if (threadIdx.x == 0) nonzero[blockIdx.x] = c;
}

// *zero = 1 when the nonzero counts of k_sq sum to zero, else 0
__global__ __launch_bounds__(256) void k_zero_flag(const double* __restrict__ nonzero, int count,
                                                   int* __restrict__ zero) {
  double acc = 0.0;
  for (int k = threadIdx.x; k < count; k += 256) acc += nonzero[k];
  const double t = block_sum(acc);
  if (threadIdx.x == 0) *zero = t == 0.0 ? 1 : 0;
}

// out[0] = sum of the partials (fixed order), out[1] = sqrt(out[0])
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ partials,
                                                  double* __restrict__ out, int count) {
  double acc = 0.0;
  for (int k = threadIdx.x; k < count; k += 256) acc += partials[k];
  const double t = block_sum(acc);
  if (threadIdx.x == 0) {
    out[0] = t;
    out[1] = sqrt(t);
  }
}

constexpr int kCheckThreads = 1024;

// Sum over a kCheckThreads workgroup in a fixed order (wavefront trees, then the wavefront sums
// in index order); the total is returned to thread 0.
__device__ __forceinline__ double block_sum_check(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double ws[kCheckThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) ws[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kCheckThreads / 64; ++w) t += ws[w];
  return t;
}

// Convergence bookkeeping of a solve step, on the device: sums the partials into out[0..1]
// (||r||^2, ||r||), appends ||r||/||b|| to the history and raises *stop when
// ||r||^2 <= target^2, the step budget is spent, or the norm is not finite.
// st[0] = stop flag, st[1] = steps done, st[2] = max steps; sc[1] = ||b||, sc[6] = target^2.
__device__ __forceinline__ void check_body(const double* __restrict__ partials, int count,
                                           double* __restrict__ out, const double* __restrict__ sc,
                                           int* __restrict__ st, double* __restrict__ hist,
                                           int hist_cap) {
  // every load first (the state, the scalars, the partials), so that their latencies overlap;
  // nothing is written once the solve has stopped
  const int stopped = st[0], steps = st[1], max_steps = st[2];
  const double bnorm = sc[1], target = sc[6];
  // thread k sums partials k, k + 1024, ... in four interleaved running sums, so that four loads
  // are in flight at a time; then the fixed-order tree over the workgroup
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int k = threadIdx.x;
  for (; k + 3 * kCheckThreads < count; k += 4 * kCheckThreads) {
    a0 += partials[k];
    a1 += partials[k + kCheckThreads];
    a2 += partials[k + 2 * kCheckThreads];
    a3 += partials[k + 3 * kCheckThreads];
  }
  for (; k < count; k += kCheckThreads) a0 += partials[k];
  const double t = block_sum_check((a0 + a1) + (a2 + a3));
  if (stopped) return;
  if (threadIdx.x == 0) {
    out[0] = t;
    out[1] = sqrt(t);
    const int k = steps + 1;
    st[1] = k;
    if (k <= hist_cap) hist[k - 1] = bnorm > 0.0 ? sqrt(t) / bnorm : sqrt(t);
    if (!(t > target) || k >= max_steps || !isfinite(t)) st[0] = 1;
  }
}

__global__ __launch_bounds__(kCheckThreads) void k_check(const double* __restrict__ partials, int count,
                                               double* __restrict__ out,
                                               const double* __restrict__ sc,
                                               int* __restrict__ st, double* __restrict__ hist,
                                               int hist_cap) {
  check_body(partials, count, out, sc, st, hist, hist_cap);
}

// One workgroup per instance.
__global__ __launch_bounds__(kCheckThreads) void k_check_multi(const CheckArgs* __restrict__ list) {
  const CheckArgs& c = list[blockIdx.x];
  check_body(c.partials, c.count, c.out, c.sc, c.st, c.hist, c.hist_cap);
}

// Squared norms of b and of b - A u over the interior of each instance: blocks_per workgroups
// per instance, partials [instance][workgroup][2] (u null: r = b).
__global__ __launch_bounds__(256) void k_norms_multi(const NormArgs* __restrict__ list,
                                                     int blocks_per, double* __restrict__ partials) {
  const int inst = int(blockIdx.x) / blocks_per, sub = int(blockIdx.x) % blocks_per;
  const NormArgs& a = list[inst];
  const int nx = a.nx, ny = a.ny;
  const size_t N = size_t(nx) * ny;
  double sb = 0.0, sr = 0.0;
  for (size_t v = size_t(sub) * 256 + threadIdx.x; v < N; v += size_t(blocks_per) * 256) {
    const int j = int(v / nx), i = int(v % nx);
    if (i <= 0 || i >= nx - 1 || j <= 0 || j >= ny - 1) continue;
    const double bv = a.b[v];
    const double r = a.u ? bv - (offdiag(a.S, a.u, N, nx, v) + a.S[v] * a.u[v]) : bv;
    sb += bv * bv;
    sr += r * r;
  }
  const double tb = block_sum(sb);
  const double tr = block_sum(sr);
  if (threadIdx.x == 0) {
    partials[2 * size_t(blockIdx.x)] = tb;
    partials[2 * size_t(blockIdx.x) + 1] = tr;
  }
}

__global__ __launch_bounds__(256) void k_solve_start(const double* __restrict__ pb, int nb,
                                                     const double* __restrict__ pr, int nr,
                                                     double* __restrict__ sc_b,
                                                     double* __restrict__ sc_r,
                                                     int* __restrict__ st, double rtol,
                                                     int max_iters) {
  double ab = 0.0, ar = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) ab += pb[k];
  for (int k = threadIdx.x; k < nr; k += 256) ar += pr[k];
  const double tb = block_sum(ab);
  const double tr = block_sum(ar);
  if (threadIdx.x == 0) {
    const double bn = sqrt(tb), rn = sqrt(tr);
    const double target = rtol * bn;
    sc_b[0] = tb;
    sc_b[1] = bn;
    sc_r[0] = tr;
    sc_r[1] = rn;
    sc_b[6] = target * target;
    sc_b[7] = rn;  // the initial residual norm, kept for the host's step-count prediction
    st[0] = (bn == 0.0 || !(rn > target) || max_iters <= 0 || !isfinite(tb) || !isfinite(tr)) ? 1 : 0;
    st[1] = 0;
    st[2] = max_iters;
  }
}

// u = 0 when ||b|| (sc_b[1]) is zero: the solution of A u = 0
__global__ __launch_bounds__(256) void k_zero_if_b0(double* __restrict__ u, size_t n,
                                                    const double* __restrict__ sc_b) {
  if (sc_b[1] != 0.0) return;
  for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < n;
       k += size_t(gridDim.x) * blockDim.x)
    u[k] = 0.0;
}

// Squared-residual partials of instances whose whole cycle runs in the coarse tail (no strip
// sweep produces them): blocks_per workgroups per instance into list[k].partials[0..blocks_per).
__global__ __launch_bounds__(256) void k_resid_multi(const NormArgs* __restrict__ list,
                                                     int blocks_per) {
  const int inst = int(blockIdx.x) / blocks_per, sub = int(blockIdx.x) % blocks_per;
  const NormArgs& a = list[inst];
  if (a.st[0]) return;
  const int nx = a.nx, ny = a.ny;
  const size_t N = size_t(nx) * ny;
  double sr = 0.0;
  for (size_t v = size_t(sub) * 256 + threadIdx.x; v < N; v += size_t(blocks_per) * 256) {
    const int j = int(v / nx), i = int(v % nx);
    if (i <= 0 || i >= nx - 1 || j <= 0 || j >= ny - 1) continue;
    const double r = a.b[v] - (offdiag(a.S, a.u, N, nx, v) + a.S[v] * a.u[v]);
    sr += r * r;
  }
  const double tr = block_sum(sr);
  if (threadIdx.x == 0) a.partials[sub] = tr;
}

// Starts each instance's solve state from its norms: sc[0..3] = ||b||^2, ||b||, ||r||^2, ||r||,
// sc[6] = (rtol ||b||)^2; st = {stop, steps = 0, max}; summary[2k..2k+1] = ||b||, ||r||.
__global__ __launch_bounds__(256) void k_init_multi(const NormArgs* __restrict__ list,
                                                    int blocks_per,
                                                    const double* __restrict__ partials,
                                                    double* __restrict__ summary) {
  const NormArgs& a = list[blockIdx.x];
  double sb = 0.0, sr = 0.0;
  for (int k = threadIdx.x; k < blocks_per; k += 256) {
    sb += partials[2 * (size_t(blockIdx.x) * blocks_per + k)];
    sr += partials[2 * (size_t(blockIdx.x) * blocks_per + k) + 1];
  }
  const double tb = block_sum(sb);
  const double tr = block_sum(sr);
  if (threadIdx.x == 0) {
    const double bn = sqrt(tb), rn = sqrt(tr);
    const double target = a.rtol * bn;
    a.sc[0] = tb;
    a.sc[1] = bn;
    a.sc[2] = tr;
    a.sc[3] = rn;
    a.sc[6] = target * target;
    a.st[0] = (bn == 0.0 || !(rn > target) || a.max_iters <= 0 || !isfinite(tr) || !isfinite(tb))
                  ? 1 : 0;
    a.st[1] = 0;
    a.st[2] = a.max_iters;
    summary[2 * blockIdx.x] = bn;
    summary[2 * blockIdx.x + 1] = rn;
  }
}

// Final relative residuals and step counts of every instance, gathered for one host copy.
__global__ __launch_bounds__(256) void k_gather_multi(const CheckArgs* __restrict__ list, int count,
                                                      double* __restrict__ rel,
                                                      int* __restrict__ steps) {
  for (int k = int(blockIdx.x) * 256 + threadIdx.x; k < count; k += int(gridDim.x) * 256) {
    const CheckArgs& c = list[k];
    const double rn = c.out[1], bn = c.sc[1];
    rel[k] = bn > 0.0 ? rn / bn : rn;
    steps[k] = c.st[1];
  }
}

unsigned stride_blocks(size_t n) {
  const size_t b = (n + 255) / 256;
  return unsigned(b < 4096 ? (b ? b : 1) : 4096);
}

// ---- dense coarse operator ------------------------------------------------------------
// u = B b on the interior of one coarse level (B row-major [m][m], interior unknowns in row-major
// order of the level's interior points), boundary ring of u = 0.  One wavefront per row: lane
// l sums the terms j = l, l + 64, ... in order, then the 64 lane sums are added by a fixed tree.
template <class T>
__device__ __forceinline__ void dense_rows(const DenseArgs<T>& a, int row_block) {
  // the stop flag is tested after the row's loads are issued (their latencies overlap)
  const int stopped = a.stop ? *a.stop : 0;
  const int mx = a.nx - 2, m = mx * (a.ny - 2);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = row_block * (blockDim.x >> 6) + wave;
  T acc = T(0);
  if (i < m) {
    // all of this lane's terms (m <= kGemvMax = 16 x 64) are loaded before the first product,
    // then summed in order j = lane, lane + 64, ...
    const T* row = a.B + size_t(i) * m;
    constexpr int kTerms = kGemvMax / 64;
    T bv[kTerms], xv[kTerms];
#pragma unroll
    for (int q = 0; q < kTerms; ++q) {
      const int j = lane + 64 * q;
      const bool ok = j < m;
      const int jj = ok ? j : 0;
      bv[q] = row[jj];
      xv[q] = a.b[(jj / mx + 1) * a.nx + jj % mx + 1];
      if (!ok) bv[q] = xv[q] = T(0);
    }
#pragma unroll
    for (int q = 0; q < kTerms; ++q)
      if (lane + 64 * q < m) acc += bv[q] * xv[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  }
  if (stopped) return;
  if (i < m && lane == 0) a.u[(i / mx + 1) * a.nx + i % mx + 1] = acc;
  // the boundary ring, by the first workgroup
  if (row_block == 0) {
    const int nb = 2 * a.nx + 2 * (a.ny - 2);
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
      int v;
      if (k < a.nx) v = k;
      else if (k < 2 * a.nx) v = (a.ny - 1) * a.nx + (k - a.nx);
      else {
        const int r = k - 2 * a.nx;  // rows 1..ny-2, left then right
        v = (r / 2 + 1) * a.nx + ((r & 1) ? a.nx - 1 : 0);
      }
      a.u[v] = T(0);
    }
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_dense(DenseArgs<T> a) {
  dense_rows<T>(a, int(blockIdx.x));
}

// The same over many instances: workgroup g serves instance g / blocks_per.
template <class T>
__global__ __launch_bounds__(256) void k_dense_multi(const DenseArgs<T>* __restrict__ list,
                                                     int blocks_per) {
  const int inst = int(blockIdx.x) / blocks_per;
  dense_rows<T>(list[inst], int(blockIdx.x) - inst * blocks_per);
}

// out[c][r] = in[r][c] for an n x n float64 matrix, through 64 x 64 LDS tiles.
__global__ __launch_bounds__(256) void k_transpose(const double* __restrict__ in,
                                                   double* __restrict__ out, int n) {
  __shared__ double tile[64][65];
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4)
    if (r0 + r < n && c0 + tx < n) tile[r][tx] = in[size_t(r0 + r) * n + c0 + tx];
  __syncthreads();
  for (int c = ty; c < 64; c += 4)
    if (c0 + c < n && r0 + tx < n) out[size_t(c0 + c) * n + r0 + tx] = tile[tx][c];
}

}  // namespace

template <class T>
dmg_status launch_dense(const DenseArgs<T>& a, hipStream_t s) {
  const int m = (a.nx - 2) * (a.ny - 2);
  if (m < 1 || m > kGemvMax || !a.B || !a.b || !a.u)
    return fail(DMG_ERR_INVALID_ARG, "dense coarse operator arguments (m = %d)", m);
  k_dense<T><<<(m + 3) / 4, 256, 0, s>>>(a);
  return launch_check("dense");
}

template <class T>
dmg_status launch_dense_multi(const DenseArgs<T>* list, int count, int max_m, hipStream_t s) {
  if (count < 1) return DMG_OK;
  if (max_m < 1 || max_m > kGemvMax)
    return fail(DMG_ERR_INVALID_ARG, "dense coarse operator size %d", max_m);
  const int per = (max_m + 3) / 4;
  k_dense_multi<T><<<count * per, 256, 0, s>>>(list, per);
  return launch_check("dense multi");
}
template dmg_status launch_dense<double>(const DenseArgs<double>&, hipStream_t);
template dmg_status launch_dense<float>(const DenseArgs<float>&, hipStream_t);
template dmg_status launch_dense_multi<double>(const DenseArgs<double>*, int, int, hipStream_t);

dmg_status launch_transpose(const double* in, double* out, int n, hipStream_t s) {
  if (n < 1) return DMG_OK;
  const unsigned g = unsigned((n + 63) / 64);
  k_transpose<<<dim3(g, g), 256, 0, s>>>(in, out, n);
  return launch_check("transpose");
}

template <class T>
dmg_status launch_copy(const T* x, T* y, size_t n, const int* stop, hipStream_t s) {
  k_copy<T><<<stride_blocks(n), 256, 0, s>>>(x, y, n, stop);
  return launch_check("copy");
}

template <class T>
dmg_status launch_fill(T* x, T v, size_t n, hipStream_t s) {
  k_fill<T><<<stride_blocks(n), 256, 0, s>>>(x, v, n);
  return launch_check("fill");
}

#define DMG_INST(T)                                                                          \
  template dmg_status launch_fill<T>(T*, T, size_t, hipStream_t);                            \
  template dmg_status launch_copy<T>(const T*, T*, size_t, const int*, hipStream_t);
DMG_INST(double)
DMG_INST(float)
#undef DMG_INST

dmg_status launch_resid_sq_partials(const double* S, const double* u, const double* b, int nx,
                                    int ny, double* partials, hipStream_t s, const int* stop,
                                    const int* zero, const double* pb) {
  if (zero && !pb) return fail(DMG_ERR_INVALID_ARG, "a zero-iterate residual needs the b partials");
  k_resid_sq<<<kReduceBlocks, 256, 0, s>>>(S, u, b, nx, ny, partials, stop, zero, pb);
  return launch_check("resid_sq");
}

dmg_status launch_sq_partials(const double* x, size_t, int nx, int ny, double* partials,
                              hipStream_t s) {
  k_sq<<<kReduceBlocks, 256, 0, s>>>(x, nx, ny, partials, nullptr, nullptr);
  return launch_check("sq");
}

dmg_status launch_start_norms(const double* b, const double* u, int nx, int ny, double* pb,
                              double* nonzero, int* zero, hipStream_t s) {
  k_sq<<<kReduceBlocks, 256, 0, s>>>(b, nx, ny, pb, u, nonzero);
  DMG_CHECK(launch_check("sq"));
  k_zero_flag<<<1, 256, 0, s>>>(nonzero, kReduceBlocks, zero);
  return launch_check("zero_flag");
}

dmg_status launch_stencil_apply(const double* S, const double* x, double* y, int nx, int ny,
                                hipStream_t s) {
  k_stencil_apply<<<stride_blocks(size_t(nx) * ny), 256, 0, s>>>(S, x, y, nx, ny);
  return launch_check("stencil_apply");
}

dmg_status launch_finalize(const double* partials, double* out, hipStream_t s, int count) {
  k_finalize<<<1, 256, 0, s>>>(partials, out, count);
  return launch_check("finalize");
}

dmg_status launch_solve_start(const double* pb, int nb, const double* pr, int nr, double* sc_b,
                              double* sc_r, int* st, double rtol, int max_iters, double* u,
                              size_t n, hipStream_t s) {
  k_solve_start<<<1, 256, 0, s>>>(pb, nb, pr, nr, sc_b, sc_r, st, rtol, max_iters);
  DMG_CHECK(launch_check("solve_start"));
  k_zero_if_b0<<<stride_blocks(n), 256, 0, s>>>(u, n, sc_b);
  return launch_check("zero_if_b0");
}

dmg_status launch_check_multi(const CheckArgs* list, int count, hipStream_t s) {
  if (count < 1) return DMG_OK;
  k_check_multi<<<count, kCheckThreads, 0, s>>>(list);
  return launch_check("check_multi");
}

dmg_status launch_norms_multi(const NormArgs* list, int count, int blocks_per, double* partials,
                              double* summary, hipStream_t s) {
  if (count < 1) return DMG_OK;
  k_norms_multi<<<count * blocks_per, 256, 0, s>>>(list, blocks_per, partials);
  DMG_CHECK(launch_check("norms_multi"));
  k_init_multi<<<count, 256, 0, s>>>(list, blocks_per, partials, summary);
  return launch_check("init_multi");
}

dmg_status launch_resid_multi(const NormArgs* list, int count, int blocks_per, hipStream_t s) {
  if (count < 1) return DMG_OK;
  k_resid_multi<<<count * blocks_per, 256, 0, s>>>(list, blocks_per);
  return launch_check("resid_multi");
}

dmg_status launch_gather_multi(const CheckArgs* list, int count, double* rel, int* steps,
                               hipStream_t s) {
  if (count < 1) return DMG_OK;
  k_gather_multi<<<(count + 255) / 256, 256, 0, s>>>(list, count, rel, steps);
  return launch_check("gather_multi");
}

dmg_status launch_check_step(const double* partials, int count, double* out, const double* sc,
                             int* st, double* hist, int hist_cap, hipStream_t s) {
  k_check<<<1, kCheckThreads, 0, s>>>(partials, count, out, sc, st, hist, hist_cap);
  return launch_check("check");
}

}  // namespace dmg
