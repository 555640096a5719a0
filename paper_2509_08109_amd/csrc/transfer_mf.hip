// Matrix-free coupled mass (Sec. 2.3.1, its closing remark): instead of storing C, the setup
// keeps the overlap sets -- for every mapped triangle the box of grid cells it may overlap, and
// for every grid cell the triangles whose box holds it -- and each application recomputes the
// triangle-cell integrals on the fly with the same routine as the assembly (cell_integrals).
//
//   C x   (from_grid's start): one thread per triangle sums w[a][g] x[g] over the cells of its
//         box and the interior grid corners g, times its Jacobian factor, into y[3 t + a]; one
//         group of lanes per mesh row then adds the y entries of its incident triangles (ascending
//         triangle order, lane l taking entries l, l + 4, ...) and forms the squared-norm partials CG2
//         starts from.
//   C^T y (to_grid's end): a group of lanes per grid cell sums, over the triangles of its list,
//         the four corner values J sum_a w[a][g] y[v_a] (Dirichlet vertices count as zero); one
//         thread per interior grid vertex adds the matching corners of its four cells.
//
// Every sum runs in a fixed order and nothing is scattered, so results do not depend on the
// launch; they equal the assembled operator's to rounding (the same integrals, summed in another
// order).  Device state: the vertices' images, three vertex indices and one Jacobian factor per
// triangle, the two incidence lists, and one buffer of max(3 nt, 4 cells) float64 between the two
// kernels of an application -- no C and no C^T.  Degenerate mapped triangles (zero area) add
// nothing, as in the assembly.
#include <algorithm>
#include <cmath>

#include "mesh_internal.h"

namespace dmg {
namespace {

__device__ __forceinline__ bool mf_stopped(const int* stop) { return stop && *stop; }

unsigned mf_grid(size_t n) {
  return unsigned(std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 65535)));
}

__device__ __forceinline__ void mf_load(const double* __restrict__ xy, const int* __restrict__ tv,
                                        int t, double tri[3][2], int v[3]) {
  for (int a = 0; a < 3; ++a) {
    v[a] = tv[3 * size_t(t) + a];
    tri[a][0] = xy[2 * size_t(v[a])];
    tri[a][1] = xy[2 * size_t(v[a]) + 1];
  }
}

__device__ __forceinline__ double mf_det(const double tri[3][2]) {
#pragma clang fp contract(off)
  return (tri[1][0] - tri[0][0]) * (tri[2][1] - tri[0][1]) -
         (tri[2][0] - tri[0][0]) * (tri[1][1] - tri[0][1]);
}

// The nq x nq rule of cell_integrals without its divisions.  A point counts when no barycentric
// coordinate is negative; lambda_a = num_a / det is negative exactly when num_a is nonzero and
// its sign differs from det's, so testing the numerators (computed by the same expression, with
// contraction off) classifies every point as the assembly does.  lambda_a is then num_a times
// 1/det, and the cell coordinates of a point are the rule's nodes themselves instead of
// (X - X0) / h: values that differ from the assembly's by rounding only.
__device__ __forceinline__ void mf_raster(const double tri[3][2], double det, int ci, int cj,
                                          double hx, double hy, int nq,
                                          const double* __restrict__ qx,
                                          const double* __restrict__ qw, double w[3][4]) {
#pragma clang fp contract(off)
  for (int a = 0; a < 3; ++a)
    for (int g = 0; g < 4; ++g) w[a][g] = 0.0;
  const double X0 = -1.0 + ci * hx, Y0 = -1.0 + cj * hy;
  double e[3][3];
  for (int a = 0; a < 3; ++a) {
    const double* p = tri[(a + 1) % 3];
    const double* q = tri[(a + 2) % 3];
    e[a][0] = p[0] * q[1] - q[0] * p[1];
    e[a][1] = p[1] - q[1];
    e[a][2] = q[0] - p[0];
  }
  const double rdet = 1.0 / det;
  const bool neg = det < 0.0;
  for (int sy = 0; sy < nq; ++sy) {
    const double Y = Y0 + qx[sy] * hy, t = qx[sy];
    for (int sx = 0; sx < nq; ++sx) {
      const double X = X0 + qx[sx] * hx, s = qx[sx];
      double num[3];
      bool out = false;
      for (int a = 0; a < 3; ++a) {
        num[a] = e[a][0] + e[a][1] * X + e[a][2] * Y;
        out |= num[a] != 0.0 && ((num[a] < 0.0) != neg);
      }
      if (out) continue;
      const double wt = qw[sx] * qw[sy] * hx * hy;
      const double ph[4] = {(1 - s) * (1 - t), s * (1 - t), (1 - s) * t, s * t};
      for (int a = 0; a < 3; ++a) {
        const double wa = wt * (num[a] * rdet);
        for (int g = 0; g < 4; ++g) w[a][g] += wa * ph[g];
      }
    }
  }
}

// The integrals of one triangle over one cell: EXACT (nq == 0, the overlap polygon, as the
// assembly computes them) or the nq x nq rule; one kernel instance per case keeps the other
// path out of its registers.
template <bool EXACT>
__device__ __forceinline__ void mf_integrals(const double tri[3][2], double det, int ci, int cj,
                                             double hx, double hy, int nq, const double* q,
                                             double w[3][4]) {
  if constexpr (EXACT) {
    cell_integrals(tri, det, ci, cj, hx, hy, 0, q, q, w);
  } else {
    mf_raster(tri, det, ci, cj, hx, hy, nq, q, q + nq, w);
  }
}

// y[3 t + a] = J_t * sum over the cells of t's box and their interior corners g of w[a][g] x[g]
template <bool EXACT>
__global__ __launch_bounds__(256) void k_mf_tri(const double* __restrict__ xy,
                                                const int* __restrict__ tv,
                                                const double* __restrict__ jac, int nt, int nx,
                                                int ny, double hx, double hy, int nq,
                                                const double* __restrict__ q,
                                                const double* __restrict__ x,
                                                double* __restrict__ y,
                                                const int* __restrict__ stop) {
  if (mf_stopped(stop)) return;
  for (int64_t tt = int64_t(blockIdx.x) * 256 + threadIdx.x; tt < nt; tt += int64_t(gridDim.x) * 256) {
    const int t = int(tt);
    const double J = jac[t];
    double acc[3] = {0.0, 0.0, 0.0};
    if (J != 0.0) {
      double tri[3][2];
      int v[3];
      mf_load(xy, tv, t, tri, v);
      const double det = mf_det(tri);
      const int i0 = grid_cell(fmin(fmin(tri[0][0], tri[1][0]), tri[2][0]), hx, nx);
      const int i1 = grid_cell(fmax(fmax(tri[0][0], tri[1][0]), tri[2][0]), hx, nx);
      const int j0 = grid_cell(fmin(fmin(tri[0][1], tri[1][1]), tri[2][1]), hy, ny);
      const int j1 = grid_cell(fmax(fmax(tri[0][1], tri[1][1]), tri[2][1]), hy, ny);
      for (int cj = j0; cj <= j1; ++cj)
        for (int ci = i0; ci <= i1; ++ci) {
          double w[3][4];
          mf_integrals<EXACT>(tri, det, ci, cj, hx, hy, nq, q, w);
          for (int g = 0; g < 4; ++g) {
            const int gx = ci + (g & 1), gy = cj + (g >> 1);
            if (gx == 0 || gx == nx - 1 || gy == 0 || gy == ny - 1) continue;
            const double xg = x[size_t(gy) * nx + gx];
            for (int a = 0; a < 3; ++a) acc[a] = __builtin_fma(w[a][g], xg, acc[a]);
          }
        }
    }
    for (int a = 0; a < 3; ++a) y[3 * size_t(t) + a] = J * acc[a];
  }
}

// r0[r] = dof[r] * (sum of y over r's incidence list); partials of r0.r0 (one per workgroup,
// tblocks(n, kMG) workgroups as the CG2 tail expects)
__global__ __launch_bounds__(256) void k_mf_rows(const int* __restrict__ vt_ptr,
                                                 const int* __restrict__ vt,
                                                 const double* __restrict__ y,
                                                 const unsigned char* __restrict__ dof,
                                                 double* __restrict__ r0, int n,
                                                 double* __restrict__ partials,
                                                 const int* __restrict__ stop) {
  if (mf_stopped(stop)) return;
  // kMG lanes per row: lane l adds entries l, l + kMG, ...; the group sums by xor shuffles
  const int lane = int(threadIdx.x) & (kMG - 1);
  const int64_t g0 = (blockIdx.x * 256u + threadIdx.x) / kMG, gstep = gridDim.x * 256u / kMG;
  double acc = 0.0;
  for (int64_t rr = g0; rr < n; rr += gstep) {  // uniform over a row's lanes
    const int r = int(rr);
    double s = 0.0;
    for (int k = vt_ptr[r] + lane; k < vt_ptr[r + 1]; k += kMG) s += y[vt[k]];
#pragma unroll
    for (int off = kMG / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kMG);
    if (lane == 0) {
      const double val = dof[r] ? s : 0.0;
      r0[r] = val;
      acc += val * val;
    }
  }
  const double t = mesh_block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// z[4 c + g] = sum over the triangles t of cell c's list of J_t sum_a w[a][g] y[v_a].  A cell's
// list (~20 triangles on a mesh finer than the grid) is split over kCellLanes consecutive lanes
// (lane l takes entries l, l + kCellLanes, ...), whose sums are combined by xor shuffles in a
// fixed order.
constexpr int kCellLanes = 4;
template <bool EXACT>
__global__ __launch_bounds__(256) void k_mf_cells(const double* __restrict__ xy,
                                                  const int* __restrict__ tv,
                                                  const double* __restrict__ jac,
                                                  const int* __restrict__ ct_ptr,
                                                  const int* __restrict__ ct, int nx, int ny,
                                                  double hx, double hy, int nq,
                                                  const double* __restrict__ q,
                                                  const double* __restrict__ yv,
                                                  const unsigned char* __restrict__ dof,
                                                  double* __restrict__ z,
                                                  const int* __restrict__ stop) {
  if (mf_stopped(stop)) return;
  const int ncx = nx - 1;
  const int64_t ncell = int64_t(ncx) * (ny - 1);
  const int lane = int(threadIdx.x) & (kCellLanes - 1);
  const int64_t c0 = (blockIdx.x * 256u + threadIdx.x) / kCellLanes;
  const int64_t cstep = gridDim.x * 256u / kCellLanes;
  for (int64_t c = c0; c < ncell; c += cstep) {  // uniform over the lanes of a cell's group
    const int ci = int(c % ncx), cj = int(c / ncx);
    double zc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = ct_ptr[c] + lane; k < ct_ptr[c + 1]; k += kCellLanes) {
      const int t = ct[k];
      double tri[3][2];
      int v[3];
      mf_load(xy, tv, t, tri, v);
      const double J = jac[t];
      double ya[3];
      for (int a = 0; a < 3; ++a) ya[a] = dof[v[a]] ? yv[v[a]] : 0.0;
      double w[3][4];
      mf_integrals<EXACT>(tri, mf_det(tri), ci, cj, hx, hy, nq, q, w);
      for (int g = 0; g < 4; ++g) {
        const double s = __builtin_fma(w[2][g], ya[2], __builtin_fma(w[1][g], ya[1], w[0][g] * ya[0]));
        zc[g] = __builtin_fma(J, s, zc[g]);
      }
    }
    for (int g = 0; g < 4; ++g) {
#pragma unroll
      for (int off = kCellLanes / 2; off > 0; off >>= 1)
        zc[g] += __shfl_xor(zc[g], off, kCellLanes);
    }
    if (lane == 0)
      for (int g = 0; g < 4; ++g) z[4 * size_t(c) + g] = zc[g];
  }
}

// r_c at interior grid vertex (i, j): corners 3, 2, 1, 0 of cells (i-1, j-1), (i, j-1), (i-1, j),
// (i, j); zero on the grid boundary
__global__ __launch_bounds__(256) void k_mf_verts(const double* __restrict__ z, int nx, int ny,
                                                  double* __restrict__ out,
                                                  const int* __restrict__ stop) {
  if (mf_stopped(stop)) return;
  const int64_t ng = int64_t(nx) * ny;
  const int ncx = nx - 1;
  for (int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x; p < ng; p += int64_t(gridDim.x) * 256) {
    const int i = int(p % nx), j = int(p / nx);
    double s = 0.0;
    if (i > 0 && i < nx - 1 && j > 0 && j < ny - 1) {
      const size_t c00 = size_t(j - 1) * ncx + (i - 1), c01 = c00 + ncx;
      s = ((z[4 * c00 + 3] + z[4 * (c00 + 1) + 2]) + z[4 * c01 + 1]) + z[4 * (c01 + 1) + 0];
    }
    out[p] = s;
  }
}

// Host bounding box of a triangle in cells, with the device kernels' clamping.
void host_box(const double tri[3][2], double hx, double hy, int nx, int ny, int b[4]) {
  b[0] = grid_cell(std::min({tri[0][0], tri[1][0], tri[2][0]}), hx, nx);
  b[1] = grid_cell(std::max({tri[0][0], tri[1][0], tri[2][0]}), hx, nx);
  b[2] = grid_cell(std::min({tri[0][1], tri[1][1], tri[2][1]}), hy, ny);
  b[3] = grid_cell(std::max({tri[0][1], tri[1][1], tri[2][1]}), hy, ny);
}

}  // namespace

dmg_status mf_build(const Mesh& m, int nx, int ny, int nq, const std::vector<int>& perm,
                    hipStream_t s, dmg_transfer* t) {
  const int nv = m.nv, nt = m.nt;
  const size_t ncell = size_t(nx - 1) * (ny - 1);
  if (ncell >= (size_t(1) << 31)) return fail(DMG_ERR_DIMS, "grid too large for the cell lists");
  if (nt > (INT32_MAX - 3) / 3)  // the incidence entries 3 t + slot are int32
    return fail(DMG_ERR_INVALID_ARG, "too many triangles for the matrix-free form (%d)", nt);
  const double hx = 2.0 / (nx - 1), hy = 2.0 / (ny - 1);
  std::vector<int> newidx(nv);
  for (int i = 0; i < nv; ++i) newidx[perm[i]] = i;
  // triangles ordered by their lowest internal vertex index (counting sort, stable), so that
  // triangles used together sit together, as the vertices do
  std::vector<int> key(nt), start(size_t(nv) + 1, 0), order(nt);
  for (int k = 0; k < nt; ++k) {
    const int* tv = m.tris + 3 * size_t(k);
    key[k] = std::min({newidx[tv[0]], newidx[tv[1]], newidx[tv[2]]});
    start[size_t(key[k]) + 1]++;
  }
  for (int v = 0; v < nv; ++v) start[v + 1] += start[v];
  for (int k = 0; k < nt; ++k) order[start[key[k]]++] = k;
  // per triangle (new order): internal vertex indices (caller's slot order), Jacobian factor
  std::vector<int> tv(3 * size_t(nt));
  std::vector<double> jac(nt), xy(2 * size_t(nv));
  for (int i = 0; i < nv; ++i) {
    xy[2 * size_t(i)] = m.xy_c[2 * size_t(perm[i])];
    xy[2 * size_t(i) + 1] = m.xy_c[2 * size_t(perm[i]) + 1];
  }
  for (int k = 0; k < nt; ++k) {
    const int* src = m.tris + 3 * size_t(order[k]);
    for (int a = 0; a < 3; ++a) tv[3 * size_t(k) + a] = newidx[src[a]];
    const double det = tri_area2(m.xy_c, src);
    jac[k] = det == 0.0 ? 0.0 : std::fabs(tri_area2(m.xy_p, src)) / std::fabs(det);
  }
  // mesh row -> 3 t + a, ascending t
  std::vector<int> vt_ptr(size_t(nv) + 1, 0), vt(3 * size_t(nt));
  for (int v : tv) vt_ptr[size_t(v) + 1]++;
  for (int v = 0; v < nv; ++v) vt_ptr[v + 1] += vt_ptr[v];
  {
    std::vector<int> fill(vt_ptr.begin(), vt_ptr.end() - 1);
    for (int k = 0; k < nt; ++k)
      for (int a = 0; a < 3; ++a) vt[fill[tv[3 * size_t(k) + a]]++] = 3 * k + a;
  }
  // cell -> triangles whose box holds it, ascending t (degenerate triangles left out)
  std::vector<int> box(4 * size_t(nt));
  std::vector<int64_t> ct_cnt(ncell + 1, 0);
  for (int k = 0; k < nt; ++k) {
    if (jac[k] == 0.0) continue;
    double tri[3][2];
    for (int a = 0; a < 3; ++a) {
      tri[a][0] = xy[2 * size_t(tv[3 * size_t(k) + a])];
      tri[a][1] = xy[2 * size_t(tv[3 * size_t(k) + a]) + 1];
    }
    int* b = &box[4 * size_t(k)];
    host_box(tri, hx, hy, nx, ny, b);
    for (int cj = b[2]; cj <= b[3]; ++cj)
      for (int ci = b[0]; ci <= b[1]; ++ci) ct_cnt[size_t(cj) * (nx - 1) + ci + 1]++;
  }
  for (size_t c = 0; c < ncell; ++c) ct_cnt[c + 1] += ct_cnt[c];
  const int64_t pairs = ct_cnt[ncell];
  if (pairs >= (int64_t(1) << 31))
    return fail(DMG_ERR_INVALID_ARG, "overlap sets exceed 2^31 triangle-cell pairs");
  std::vector<int> ct_ptr(ncell + 1), ct(size_t(pairs) + 1);
  for (size_t c = 0; c <= ncell; ++c) ct_ptr[c] = int(ct_cnt[c]);
  {
    std::vector<int64_t> fill(ct_cnt.begin(), ct_cnt.end() - 1);
    for (int k = 0; k < nt; ++k) {
      if (jac[k] == 0.0) continue;
      const int* b = &box[4 * size_t(k)];
      for (int cj = b[2]; cj <= b[3]; ++cj)
        for (int ci = b[0]; ci <= b[1]; ++ci) ct[fill[size_t(cj) * (nx - 1) + ci]++] = k;
    }
  }
  std::vector<double> q(2 * size_t(std::max(nq, 1)), 0.0);
  if (nq > 0) {
    std::vector<double> qx, qw;
    gauss_rule01(nq, qx, qw);
    std::copy(qx.begin(), qx.end(), q.begin());
    std::copy(qw.begin(), qw.end(), q.begin() + nq);
  }
  const size_t nbuf = std::max(3 * size_t(nt), 4 * ncell);
  double *d_xy, *d_jac, *d_q;
  int *d_tv, *d_vtp, *d_vt, *d_ctp, *d_ct;
  auto layout = [&](Arena& a) {
    d_xy = a.take<double>(2 * size_t(nv));
    d_jac = a.take<double>(nt);
    d_q = a.take<double>(q.size());
    t->mf_buf = a.take<double>(nbuf);
    d_tv = a.take<int>(3 * size_t(nt));
    d_vtp = a.take<int>(size_t(nv) + 1);
    d_vt = a.take<int>(3 * size_t(nt));
    d_ctp = a.take<int>(ncell + 1);
    d_ct = a.take<int>(size_t(pairs) + 1);
  };
  Arena sz;
  layout(sz);
  DMG_HIP(hipMalloc(&t->mfblock, sz.used));
  Arena a;
  a.base = static_cast<char*>(t->mfblock);
  a.cap = sz.used;
  layout(a);
  auto up = [&](void* dst, const void* src, size_t bytes) -> dmg_status {
    if (bytes) DMG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    return DMG_OK;
  };
  DMG_CHECK(up(d_xy, xy.data(), xy.size() * sizeof(double)));
  DMG_CHECK(up(d_jac, jac.data(), jac.size() * sizeof(double)));
  DMG_CHECK(up(d_q, q.data(), q.size() * sizeof(double)));
  DMG_CHECK(up(d_tv, tv.data(), tv.size() * sizeof(int)));
  DMG_CHECK(up(d_vtp, vt_ptr.data(), vt_ptr.size() * sizeof(int)));
  DMG_CHECK(up(d_vt, vt.data(), vt.size() * sizeof(int)));
  DMG_CHECK(up(d_ctp, ct_ptr.data(), ct_ptr.size() * sizeof(int)));
  DMG_CHECK(up(d_ct, ct.data(), size_t(pairs) * sizeof(int)));
  DMG_HIP(hipStreamSynchronize(s));  // host vectors go out of scope
  t->mf = true;
  t->nt = nt;
  t->nq = nq;
  t->mf_xy = d_xy;
  t->mf_jac = d_jac;
  t->mf_q = d_q;
  t->mf_tv = d_tv;
  t->mf_vt_ptr = d_vtp;
  t->mf_vt = d_vt;
  t->mf_ct_ptr = d_ctp;
  t->mf_ct = d_ct;
  t->mf_pairs = pairs;
  t->mf_bytes = sz.used;
  return DMG_OK;
}

dmg_status mf_launch_from(dmg_transfer* t, const double* u_c, const int* stop, hipStream_t s) {
  const double hx = 2.0 / (t->nx - 1), hy = 2.0 / (t->ny - 1);
  auto k = t->nq == 0 ? k_mf_tri<true> : k_mf_tri<false>;
  k<<<mf_grid(size_t(t->nt)), 256, 0, s>>>(t->mf_xy, t->mf_tv, t->mf_jac, t->nt, t->nx, t->ny, hx,
                                           hy, t->nq, t->mf_q, u_c, t->mf_buf, stop);
  DMG_CHECK(launch_check("matrix-free C u (triangles)"));
  k_mf_rows<<<tblocks(t->nv, kMG), 256, 0, s>>>(t->mf_vt_ptr, t->mf_vt, t->mf_buf, t->dof, t->r,
                                                t->nv, t->partials, stop);
  return launch_check("matrix-free C u (rows)");
}

dmg_status mf_launch_ct(dmg_transfer* t, const double* x, double* r_c, const int* stop,
                        hipStream_t s) {
  const double hx = 2.0 / (t->nx - 1), hy = 2.0 / (t->ny - 1);
  const size_t ncell = size_t(t->nx - 1) * (t->ny - 1);
  auto k = t->nq == 0 ? k_mf_cells<true> : k_mf_cells<false>;
  k<<<mf_grid(ncell * kCellLanes), 256, 0, s>>>(t->mf_xy, t->mf_tv, t->mf_jac, t->mf_ct_ptr, t->mf_ct, t->nx,
                                   t->ny, hx, hy, t->nq, t->mf_q, x, t->dof, t->mf_buf, stop);
  DMG_CHECK(launch_check("matrix-free C^T x (cells)"));
  k_mf_verts<<<mf_grid(size_t(t->nx) * t->ny), 256, 0, s>>>(t->mf_buf, t->nx, t->ny, r_c, stop);
  return launch_check("matrix-free C^T x (vertices)");
}

}  // namespace dmg
