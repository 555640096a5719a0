// Grid <-> mesh transfers by L2 projection: P = M_p^{-1} C and R = P^T = C^T M_p^{-1}
// (paper Sec. 2.3), with M_p^{-1} applied by two iterations of unpreconditioned CG.
//
// Setup (host, C++, once per mesh): the coupled mass C of Sec. 2.3.1 is evaluated in the
// computational domain.  Every physical triangle is mapped to a straight triangle through the
// images of its vertices; the grid cells overlapping its bounding box are visited with an
// nq x nq Gauss rule per cell; quadrature points outside the mapped triangle contribute nothing;
// inside, the P1 basis is evaluated through the mapped triangle's barycentric coordinates and
// the Jacobian factor is the constant area(tau_p)/area(mapped tau).  nq = 0 integrates exactly
// instead: the mapped triangle is clipped against each cell and the cubic integrand is
// integrated over the overlap polygon (the limit of the rasterised rule).  Rows are assembled
// independently (vertex -> incident triangles) on host threads, giving CSR directly.
// M_p is the P1 mass matrix (element matrix area/12 [[2,1,1],[1,2,1],[1,1,2]]).
// Dirichlet vertices: empty rows of C, identity rows of M_p.  Grid boundary columns dropped.
//
// Apply (device): CSR products, CG2 with fixed-order reductions; nothing is allocated.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <unordered_map>

#include "mesh_internal.h"

namespace dmg {
namespace {

void gauss01(int nq, std::vector<double>& x, std::vector<double>& w) {
  // Gauss-Legendre nodes on [-1,1] by Newton iteration on P_nq, mapped to [0,1].
  x.assign(nq, 0.0);
  w.assign(nq, 0.0);
  for (int k = 0; k < nq; ++k) {
    double z = std::cos(M_PI * (k + 0.75) / (nq + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int n = 2; n <= nq; ++n) {
        const double p2 = ((2.0 * n - 1.0) * z * p1 - (n - 1.0) * p0) / n;
        p0 = p1;
        p1 = p2;
      }
      if (nq == 1) { p1 = z; p0 = 1.0; }
      dp = nq * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[k] = 0.5 * (1.0 - z);
    w[k] = 1.0 / ((1.0 - z * z) * dp * dp);  // = 0.5 * 2/((1-z^2) P'^2)
  }
}

// Merge per-thread row blocks (rows [r0,r1) of thread t) into one CSR.
Csr merge(int n, const std::vector<Csr>& parts, const std::vector<int>& first_row) {
  Csr out;
  out.rp.assign(n + 1, 0);
  size_t nnz = 0;
  for (const auto& p : parts) nnz += p.ci.size();
  out.ci.reserve(nnz);
  out.v.reserve(nnz);
  for (size_t t = 0; t < parts.size(); ++t) {
    const Csr& p = parts[t];
    const int r0 = first_row[t];
    const int rows = int(p.rp.size()) - 1;
    const int base = int(out.ci.size());
    for (int k = 0; k < rows; ++k) out.rp[r0 + k + 1] = base + p.rp[k + 1];
    out.ci.insert(out.ci.end(), p.ci.begin(), p.ci.end());
    out.v.insert(out.v.end(), p.v.begin(), p.v.end());
  }
  return out;
}

}  // namespace

void build_adjacency(Mesh& m) {
  m.vt_ptr.assign(m.nv + 1, 0);
  for (int t = 0; t < m.nt; ++t)
    for (int a = 0; a < 3; ++a) m.vt_ptr[m.tris[3 * t + a] + 1]++;
  for (int v = 0; v < m.nv; ++v) m.vt_ptr[v + 1] += m.vt_ptr[v];
  m.vt.assign(m.vt_ptr[m.nv], 0);
  std::vector<int> fill(m.vt_ptr.begin(), m.vt_ptr.end() - 1);
  for (int t = 0; t < m.nt; ++t)
    for (int a = 0; a < 3; ++a) m.vt[fill[m.tris[3 * t + a]]++] = t;
}

double tri_area2(const double* xy, const int* tv) {
  const double* a = xy + 2 * tv[0];
  const double* b = xy + 2 * tv[1];
  const double* c = xy + 2 * tv[2];
  return (b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1]);
}

namespace {

// Part of triangle tri inside the box [x0, x1] x [y0, y1] (Sutherland-Hodgman, one pass per box
// side); returns its vertex count (a triangle cut by four half-planes keeps at most 7).
int clip_triangle(const double tri[3][2], double x0, double x1, double y0, double y1,
                  double out[8][2]) {
  double a[8][2], b[8][2];
  int n = 3;
  for (int k = 0; k < 3; ++k) {
    a[k][0] = tri[k][0];
    a[k][1] = tri[k][1];
  }
  // keep the side where sign * (p[axis] - lim) >= 0
  auto pass = [](const double (*src)[2], int ns, double (*dst)[2], int axis, double lim,
                 double sign) {
    int nd = 0;
    for (int k = 0; k < ns; ++k) {
      const double* p = src[(k + ns - 1) % ns];
      const double* q = src[k];
      const bool ip = sign * (p[axis] - lim) >= 0.0, iq = sign * (q[axis] - lim) >= 0.0;
      if (ip != iq) {
        const double t = (lim - p[axis]) / (q[axis] - p[axis]);
        dst[nd][axis] = lim;
        dst[nd][1 - axis] = p[1 - axis] + t * (q[1 - axis] - p[1 - axis]);
        ++nd;
      }
      if (iq) {
        dst[nd][0] = q[0];
        dst[nd][1] = q[1];
        ++nd;
      }
    }
    return nd;
  };
  n = pass(a, n, b, 0, x0, 1.0);
  n = n ? pass(b, n, a, 0, x1, -1.0) : 0;
  n = n ? pass(a, n, b, 1, y0, 1.0) : 0;
  n = n ? pass(b, n, a, 1, y1, -1.0) : 0;
  for (int k = 0; k < n; ++k) {
    out[k][0] = a[k][0];
    out[k][1] = a[k][1];
  }
  return n;
}

// Dunavant's symmetric 6-point rule on a triangle, exact for degree 4: barycentric orbits
// (a, a, 1 - 2a) with weights relative to the area.
constexpr double kTriA1 = 0.445948490915965, kTriW1 = 0.223381589678011;
constexpr double kTriA2 = 0.091576213509771, kTriW2 = 1.0 / 3.0 - kTriW1;

// Row v of C from triangle tv (a = v's slot in tv) integrated exactly over the overlap of the
// mapped triangle with each grid cell: the integrand lambda_a * phi_g is a cubic there.
template <class Acc>
void exact_row_triangle(const Mesh& m, const int* tv, int a, double hx, double hy, int nx, int ny,
                        double jac, Acc&& acc) {
  double tri[3][2];
  for (int k = 0; k < 3; ++k) {
    tri[k][0] = m.xy_c[2 * tv[k]];
    tri[k][1] = m.xy_c[2 * tv[k] + 1];
  }
  const double det = (tri[1][0] - tri[0][0]) * (tri[2][1] - tri[0][1]) -
                     (tri[2][0] - tri[0][0]) * (tri[1][1] - tri[0][1]);
  // lambda_a(X, Y) = (e0 + e1 X + e2 Y) / det from the edge opposite vertex a
  const double* p = tri[(a + 1) % 3];
  const double* q = tri[(a + 2) % 3];
  const double e1 = p[1] - q[1], e2 = q[0] - p[0], e0 = p[0] * q[1] - q[0] * p[1];
  const double xmin = std::min({tri[0][0], tri[1][0], tri[2][0]});
  const double xmax = std::max({tri[0][0], tri[1][0], tri[2][0]});
  const double ymin = std::min({tri[0][1], tri[1][1], tri[2][1]});
  const double ymax = std::max({tri[0][1], tri[1][1], tri[2][1]});
  auto cell = [](double x, double h, int n) {
    const int c = int(std::floor((x + 1.0) / h));
    return std::min(std::max(c, 0), n - 2);
  };
  const int i0 = cell(xmin, hx, nx), i1 = cell(xmax, hx, nx);
  const int j0 = cell(ymin, hy, ny), j1 = cell(ymax, hy, ny);
  static const double orbit[2][2] = {{kTriA1, kTriW1}, {kTriA2, kTriW2}};
  double poly[8][2];
  for (int cj = j0; cj <= j1; ++cj)
    for (int ci = i0; ci <= i1; ++ci) {
      const double X0 = -1.0 + ci * hx, Y0 = -1.0 + cj * hy;
      const int np = clip_triangle(tri, X0, X0 + hx, Y0, Y0 + hy, poly);
      if (np < 3) continue;
      double w4[4] = {0.0, 0.0, 0.0, 0.0};
      for (int k = 1; k + 1 < np; ++k) {
        const double* A = poly[0];
        const double* B = poly[k];
        const double* D = poly[k + 1];
        const double area =
            0.5 * std::fabs((B[0] - A[0]) * (D[1] - A[1]) - (D[0] - A[0]) * (B[1] - A[1]));
        if (area == 0.0) continue;
        for (const auto& o : orbit) {
          const double la = o[0], lb = 1.0 - 2.0 * o[0];
          const double bary[3][3] = {{la, la, lb}, {la, lb, la}, {lb, la, la}};
          for (const auto& l : bary) {
            const double X = l[0] * A[0] + l[1] * B[0] + l[2] * D[0];
            const double Y = l[0] * A[1] + l[1] * B[1] + l[2] * D[1];
            const double w = o[1] * area * (e0 + e1 * X + e2 * Y) / det;
            const double s = (X - X0) / hx, t = (Y - Y0) / hy;
            w4[0] += w * (1 - s) * (1 - t);
            w4[1] += w * s * (1 - t);
            w4[2] += w * (1 - s) * t;
            w4[3] += w * s * t;
          }
        }
      }
      const int g00 = cj * nx + ci;
      const int gi[4] = {g00, g00 + 1, g00 + nx, g00 + nx + 1};
      for (int g = 0; g < 4; ++g) acc(gi[g], jac * w4[g]);
    }
}

// nq >= 1: the rasterised rule (nq x nq Gauss points per overlapped cell, zero outside the
// mapped triangle); nq == 0: exact integration over the triangle-cell overlaps.
Csr assemble_C(const Mesh& m, int nx, int ny, int nq) {
  std::vector<double> qx, qw;
  if (nq > 0) gauss01(nq, qx, qw);
  const double hx = 2.0 / (nx - 1), hy = 2.0 / (ny - 1);
  unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (m.nv < 4096) nthreads = 1;
  std::vector<Csr> parts(nthreads);
  std::vector<int> first(nthreads);
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nthreads; ++t) {
    const int r0 = int(int64_t(m.nv) * t / nthreads), r1 = int(int64_t(m.nv) * (t + 1) / nthreads);
    first[t] = r0;
    th.emplace_back([&, t, r0, r1]() {
      Csr& out = parts[t];
      out.rp.assign(1, 0);
      std::unordered_map<int, double> row;
      std::vector<std::pair<int, double>> sorted;
      for (int v = r0; v < r1; ++v) {
        row.clear();
        if (m.dof[v]) {
          for (int k = m.vt_ptr[v]; k < m.vt_ptr[v + 1]; ++k) {
            const int* tv = m.tris + 3 * m.vt[k];
            const int a = tv[0] == v ? 0 : (tv[1] == v ? 1 : 2);
            const double ac2 = tri_area2(m.xy_c, tv);
            if (ac2 == 0.0) continue;
            const double jac = std::fabs(tri_area2(m.xy_p, tv)) / std::fabs(ac2);
            if (nq == 0) {
              exact_row_triangle(m, tv, a, hx, hy, nx, ny, jac, [&](int g, double val) {
                const int gx = g % nx, gy = g / nx;
                if (gx == 0 || gx == nx - 1 || gy == 0 || gy == ny - 1) return;
                row[g] += val;
              });
              continue;
            }
            const double* c0 = m.xy_c + 2 * tv[0];
            const double* c1 = m.xy_c + 2 * tv[1];
            const double* c2 = m.xy_c + 2 * tv[2];
            const double xmin = std::min({c0[0], c1[0], c2[0]}), xmax = std::max({c0[0], c1[0], c2[0]});
            const double ymin = std::min({c0[1], c1[1], c2[1]}), ymax = std::max({c0[1], c1[1], c2[1]});
            auto cell = [](double x, double h, int n) {
              int c = int(std::floor((x + 1.0) / h));
              return std::min(std::max(c, 0), n - 2);
            };
            const int i0 = cell(xmin, hx, nx), i1 = cell(xmax, hx, nx);
            const int j0 = cell(ymin, hy, ny), j1 = cell(ymax, hy, ny);
            for (int cj = j0; cj <= j1; ++cj)
              for (int ci = i0; ci <= i1; ++ci)
                for (int sy = 0; sy < nq; ++sy)
                  for (int sx = 0; sx < nq; ++sx) {
                    const double s = qx[sx], tt = qx[sy];
                    const double X = -1.0 + (ci + s) * hx, Y = -1.0 + (cj + tt) * hy;
                    const double l1 = ((c2[1] - c0[1]) * (X - c0[0]) - (c2[0] - c0[0]) * (Y - c0[1])) / ac2;
                    const double l2 = ((c1[0] - c0[0]) * (Y - c0[1]) - (c1[1] - c0[1]) * (X - c0[0])) / ac2;
                    const double l0 = 1.0 - l1 - l2;
                    if (l0 < 0.0 || l1 < 0.0 || l2 < 0.0) continue;
                    const double la = a == 0 ? l0 : (a == 1 ? l1 : l2);
                    const double w = qw[sx] * qw[sy] * hx * hy * jac * la;
                    const int g00 = cj * nx + ci;
                    const double ph[4] = {(1 - s) * (1 - tt), s * (1 - tt), (1 - s) * tt, s * tt};
                    const int gi[4] = {g00, g00 + 1, g00 + nx, g00 + nx + 1};
                    for (int g = 0; g < 4; ++g) {
                      const int gx = gi[g] % nx, gy = gi[g] / nx;
                      if (gx == 0 || gx == nx - 1 || gy == 0 || gy == ny - 1) continue;
                      row[gi[g]] += w * ph[g];
                    }
                  }
          }
        }
        sorted.assign(row.begin(), row.end());
        std::sort(sorted.begin(), sorted.end());
        for (auto& e : sorted) {
          if (e.second == 0.0) continue;
          out.ci.push_back(e.first);
          out.v.push_back(e.second);
        }
        out.rp.push_back(int(out.ci.size()));
      }
    });
  }
  for (auto& x : th) x.join();
  return merge(m.nv, parts, first);
}

Csr assemble_M(const Mesh& m) {
  Csr out;
  out.rp.assign(1, 0);
  std::vector<std::pair<int, double>> row;
  for (int v = 0; v < m.nv; ++v) {
    row.clear();
    if (!m.dof[v]) {
      row.emplace_back(v, 1.0);
    } else {
      for (int k = m.vt_ptr[v]; k < m.vt_ptr[v + 1]; ++k) {
        const int* tv = m.tris + 3 * m.vt[k];
        const double area = 0.5 * std::fabs(tri_area2(m.xy_p, tv));
        for (int b = 0; b < 3; ++b) {
          if (!m.dof[tv[b]]) continue;
          row.emplace_back(tv[b], (tv[b] == v ? 2.0 : 1.0) * area / 12.0);
        }
      }
      std::sort(row.begin(), row.end());
      size_t w = 0;
      for (size_t k = 0; k < row.size(); ++k) {
        if (w > 0 && row[w - 1].first == row[k].first) row[w - 1].second += row[k].second;
        else row[w++] = row[k];
      }
      row.resize(w);
    }
    for (auto& e : row) {
      out.ci.push_back(e.first);
      out.v.push_back(e.second);
    }
    out.rp.push_back(int(out.ci.size()));
  }
  return out;
}

Csr transpose(const Csr& a, int ncols) {
  Csr t;
  const int nrows = int(a.rp.size()) - 1;
  t.rp.assign(ncols + 1, 0);
  for (int c : a.ci) t.rp[c + 1]++;
  for (int c = 0; c < ncols; ++c) t.rp[c + 1] += t.rp[c];
  t.ci.assign(a.ci.size(), 0);
  t.v.assign(a.v.size(), 0.0);
  std::vector<int> fill(t.rp.begin(), t.rp.end() - 1);
  for (int r = 0; r < nrows; ++r)
    for (int k = a.rp[r]; k < a.rp[r + 1]; ++k) {
      const int dst = fill[a.ci[k]]++;
      t.ci[dst] = r;
      t.v[dst] = a.v[k];
    }
  return t;
}

// ---- device kernels ----------------------------------------------------------------------
// stop (nullable): the kernel does nothing once the device flag is set.
__device__ __forceinline__ bool stopped(const int* stop) { return stop && *stop; }

// from_grid start: r0 = dof * (C u_c) (mesh rows in the internal order); partials of r0.r0
__global__ __launch_bounds__(256) void k_t_init_from(const int* __restrict__ rp,
                                                     const int* __restrict__ ci,
                                                     const double* __restrict__ v,
                                                     const double* __restrict__ u_c,
                                                     const unsigned char* __restrict__ dof,
                                                     double* __restrict__ r0, int n,
                                                     double* __restrict__ partials,
                                                     const int* __restrict__ stop) {
  if (stopped(stop)) return;
  const int lane = threadIdx.x & (kMG - 1);
  const int g0 = int((blockIdx.x * 256u + threadIdx.x) / kMG), ng = int(gridDim.x * 256u / kMG);
  double acc = 0.0;
  for (int r = g0; r < n; r += ng) {
    const double y = row_dot<kMG>(rp, ci, v, r, lane, [&](int c) { return u_c[c]; });
    const double val = dof[r] ? y : 0.0;
    if (lane == 0) {
      r0[r] = val;
      acc += val * val;
    }
  }
  const double t = mesh_block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// to_grid start: r0 = dof * r_p taken into the internal order; partials of r0.r0
__global__ __launch_bounds__(256) void k_t_init_to(const double* __restrict__ r_p,
                                                   const int* __restrict__ perm,
                                                   const unsigned char* __restrict__ dof,
                                                   double* __restrict__ r0, int n,
                                                   double* __restrict__ partials) {
  double acc = 0.0;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
    const double val = dof[r] ? r_p[perm[r]] : 0.0;
    r0[r] = val;
    acc += val * val;
  }
  const double t = mesh_block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// q0 = M r0; partials of r0.q0
__global__ __launch_bounds__(256) void k_t_mq(const int* __restrict__ rp, const int* __restrict__ ci,
                                              const double* __restrict__ v,
                                              const double* __restrict__ p, double* __restrict__ q,
                                              int n, double* __restrict__ partials,
                                              const int* __restrict__ stop) {
  if (stopped(stop)) return;
  const int lane = threadIdx.x & (kMG - 1);
  const int g0 = int((blockIdx.x * 256u + threadIdx.x) / kMG), ng = int(gridDim.x * 256u / kMG);
  double acc = 0.0;
  for (int r = g0; r < n; r += ng) {
    const double s = row_dot<kMG>(rp, ci, v, r, lane, [&](int c) { return p[c]; });
    if (lane == 0) {
      q[r] = s;
      acc += p[r] * s;
    }
  }
  const double t = mesh_block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// scalars: sc[0] rr0, sc[2] pq0, sc[4] rr1, sc[6] pq1 (textbook CG: a zero rr gives a zero step)
__device__ __forceinline__ double cg_alpha0(const double* sc) { return sc[0] == 0.0 ? 0.0 : sc[0] / sc[2]; }
__device__ __forceinline__ double cg_beta(const double* sc) { return sc[0] == 0.0 ? 0.0 : sc[4] / sc[0]; }
__device__ __forceinline__ double cg_alpha1(const double* sc) { return sc[4] == 0.0 ? 0.0 : sc[4] / sc[6]; }

// r1 = r0 - alpha0 q0; partials of r1.r1
__global__ __launch_bounds__(256) void k_t_r1(const double* __restrict__ r0,
                                              const double* __restrict__ q0,
                                              double* __restrict__ r1,
                                              const double* __restrict__ sc, int n,
                                              double* __restrict__ partials,
                                              const int* __restrict__ stop) {
  if (stopped(stop)) return;
  const double alpha = cg_alpha0(sc);
  double acc = 0.0;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
    const double rv = __builtin_fma(-alpha, q0[r], r0[r]);
    r1[r] = rv;
    acc += rv * rv;
  }
  const double t = mesh_block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// p1 = r1 + beta r0 (formed where read); partials of p1.(M p1) -- M p1 itself is not needed
__global__ __launch_bounds__(256) void k_t_mp1(const int* __restrict__ rp, const int* __restrict__ ci,
                                               const double* __restrict__ v,
                                               const double* __restrict__ r0,
                                               const double* __restrict__ r1,
                                               const double* __restrict__ sc, int n,
                                               double* __restrict__ partials,
                                               const int* __restrict__ stop) {
  if (stopped(stop)) return;
  const double beta = cg_beta(sc);
  const int lane = threadIdx.x & (kMG - 1);
  const int g0 = int((blockIdx.x * 256u + threadIdx.x) / kMG), ng = int(gridDim.x * 256u / kMG);
  double acc = 0.0;
  for (int r = g0; r < n; r += ng) {
    const double s = row_dot<kMG>(rp, ci, v, r, lane,
                                  [&](int c) { return __builtin_fma(beta, r0[c], r1[c]); });
    if (lane == 0) acc += __builtin_fma(beta, r0[r], r1[r]) * s;
  }
  const double t = mesh_block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// x2 = alpha0 r0 + alpha1 p1, stored in the internal order, scattered to the caller's order
// (out[perm[r]]), or added (times scale) into an internal-order vector
template <X2Mode MODE>
__global__ __launch_bounds__(256) void k_t_x(const double* __restrict__ r0,
                                             const double* __restrict__ r1,
                                             const double* __restrict__ sc,
                                             const int* __restrict__ perm,
                                             double* __restrict__ out, int n,
                                             const int* __restrict__ stop, double scale) {
  if (stopped(stop)) return;
  const double alpha0 = cg_alpha0(sc), beta = cg_beta(sc), alpha1 = cg_alpha1(sc);
  for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
    const double x1 = alpha0 * r0[r];
    const double p1 = __builtin_fma(beta, r0[r], r1[r]);
    const double x2 = __builtin_fma(alpha1, p1, x1);
    if constexpr (MODE == X2Mode::kScatter) out[perm[r]] = x2;
    else if constexpr (MODE == X2Mode::kAdd) out[r] += scale * x2;
    else out[r] = x2;
  }
}

// r_c = C^T x over the grid rows
__global__ __launch_bounds__(256) void k_t_ct(const int* __restrict__ rp, const int* __restrict__ ci,
                                              const double* __restrict__ v,
                                              const double* __restrict__ x,
                                              double* __restrict__ out, int n,
                                              const int* __restrict__ stop) {
  if (stopped(stop)) return;
  const int lane = threadIdx.x & (kCG - 1);
  const int g0 = int((blockIdx.x * 256u + threadIdx.x) / kCG), ng = int(gridDim.x * 256u / kCG);
  for (int r = g0; r < n; r += ng) {
    const double s = row_dot<kCG>(rp, ci, v, r, lane, [&](int c) { return x[c]; });
    if (lane == 0) out[r] = s;
  }
}

}  // namespace

dmg_status launch_from_start(dmg_transfer* t, const double* u_c, const int* stop, hipStream_t s) {
  k_t_init_from<<<tblocks(t->nv, kMG), 256, 0, s>>>(t->Crp, t->Cci, t->Cv, u_c, t->dof, t->r,
                                                     t->nv, t->partials, stop);
  return launch_check("transfer C u");
}

dmg_status cg2_tail(dmg_transfer* t, double* out, X2Mode mode, const int* stop, hipStream_t s,
                    double scale) {
  const int n = t->nv, nb = tblocks(n, kMG);
  double* sc = t->scal;
  DMG_CHECK(launch_finalize(t->partials, sc + 0, s, nb));
  k_t_mq<<<nb, 256, 0, s>>>(t->Mrp, t->Mci, t->Mv, t->r, t->q, n, t->partials, stop);
  DMG_CHECK(launch_check("transfer M r0"));
  DMG_CHECK(launch_finalize(t->partials, sc + 2, s, nb));
  k_t_r1<<<nb, 256, 0, s>>>(t->r, t->q, t->p, sc, n, t->partials, stop);
  DMG_CHECK(launch_check("transfer r1"));
  DMG_CHECK(launch_finalize(t->partials, sc + 4, s, nb));
  k_t_mp1<<<nb, 256, 0, s>>>(t->Mrp, t->Mci, t->Mv, t->r, t->p, sc, n, t->partials, stop);
  DMG_CHECK(launch_check("transfer M p1"));
  DMG_CHECK(launch_finalize(t->partials, sc + 6, s, nb));
  switch (mode) {
    case X2Mode::kStore:
      k_t_x<X2Mode::kStore><<<nb, 256, 0, s>>>(t->r, t->p, sc, t->perm, out, n, stop, 1.0);
      break;
    case X2Mode::kScatter:
      k_t_x<X2Mode::kScatter><<<nb, 256, 0, s>>>(t->r, t->p, sc, t->perm, out, n, stop, 1.0);
      break;
    case X2Mode::kAdd:
      k_t_x<X2Mode::kAdd><<<nb, 256, 0, s>>>(t->r, t->p, sc, t->perm, out, n, stop, scale);
      break;
  }
  return launch_check("transfer x2");
}

dmg_status launch_ct(dmg_transfer* t, const double* x, double* r_c, const int* stop, hipStream_t s) {
  const int ng = t->nx * t->ny;
  k_t_ct<<<tblocks(ng, kCG), 256, 0, s>>>(t->CTrp, t->CTci, t->CTv, x, r_c, ng, stop);
  return launch_check("transfer C^T x");
}

// Internal vertex order: by the grid cell holding each vertex's image (row-major), so that the
// rows of C and M_p that are used together sit together and their gathers stay in cache.
std::vector<int> locality_order(const Mesh& m, int nx, int ny) {
  const double hx = 2.0 / (nx - 1), hy = 2.0 / (ny - 1);
  std::vector<long> key(m.nv);
  for (int v = 0; v < m.nv; ++v) {
    const int ix = std::min(std::max(int(std::floor((m.xy_c[2 * v] + 1.0) / hx)), 0), nx - 2);
    const int iy = std::min(std::max(int(std::floor((m.xy_c[2 * v + 1] + 1.0) / hy)), 0), ny - 2);
    key[v] = long(iy) * (nx - 1) + ix;
  }
  std::vector<int> perm(m.nv);
  for (int v = 0; v < m.nv; ++v) perm[v] = v;
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return key[a] < key[b]; });
  return perm;
}

Csr permute_rows(const Csr& a, const std::vector<int>& perm, const std::vector<int>* colmap) {
  Csr out;
  const int n = int(perm.size());
  out.rp.assign(n + 1, 0);
  out.ci.reserve(a.ci.size());
  out.v.reserve(a.v.size());
  std::vector<std::pair<int, double>> row;
  for (int i = 0; i < n; ++i) {
    const int o = perm[i];
    row.clear();
    for (int k = a.rp[o]; k < a.rp[o + 1]; ++k)
      row.emplace_back(colmap ? (*colmap)[a.ci[k]] : a.ci[k], a.v[k]);
    if (colmap) std::sort(row.begin(), row.end());
    for (auto& e : row) {
      out.ci.push_back(e.first);
      out.v.push_back(e.second);
    }
    out.rp[i + 1] = int(out.ci.size());
  }
  return out;
}

dmg_status transfer_build(const Mesh& m, int nx, int ny, int nq, const std::vector<int>& perm,
                          hipStream_t stream, std::unique_ptr<dmg_transfer>& out) {
  const int nv = m.nv;
  std::vector<int> newidx(nv);
  for (int i = 0; i < nv; ++i) newidx[perm[i]] = i;
  const Csr C = permute_rows(assemble_C(m, nx, ny, nq), perm, nullptr);
  const Csr M = permute_rows(assemble_M(m), perm, &newidx);
  const Csr CT = transpose(C, nx * ny);
  std::vector<uint8_t> dof_p(nv);
  for (int i = 0; i < nv; ++i) dof_p[i] = m.dof[perm[i]];
  if (C.ci.size() >= (size_t(1) << 31) || M.ci.size() >= (size_t(1) << 31))
    return fail(DMG_ERR_INVALID_ARG, "transfer matrices exceed 2^31 nonzeros");
  std::unique_ptr<dmg_transfer> t(new dmg_transfer);
  t->nv = nv;
  t->nx = nx;
  t->ny = ny;
  t->nnzC = int64_t(C.ci.size());
  t->nnzM = int64_t(M.ci.size());
  const size_t ng = size_t(nx) * ny;
  Arena sz;
  auto layout = [&](Arena& a) {
    t->Crp = a.take<int>(nv + 1);
    t->Cci = a.take<int>(C.ci.size() + 1);
    t->Cv = a.take<double>(C.v.size() + 1);
    t->CTrp = a.take<int>(ng + 1);
    t->CTci = a.take<int>(CT.ci.size() + 1);
    t->CTv = a.take<double>(CT.v.size() + 1);
    t->Mrp = a.take<int>(nv + 1);
    t->Mci = a.take<int>(M.ci.size() + 1);
    t->Mv = a.take<double>(M.v.size() + 1);
    t->dof = a.take<unsigned char>(nv);
    t->perm = a.take<int>(nv);
    t->x = a.take<double>(nv);
    t->r = a.take<double>(nv);
    t->p = a.take<double>(nv);
    t->q = a.take<double>(nv);
    t->partials = a.take<double>(kTBlocks);
    t->scal = a.take<double>(16);
  };
  layout(sz);
  DMG_HIP(hipMalloc(&t->block, sz.used));
  Arena a;
  a.base = static_cast<char*>(t->block);
  a.cap = sz.used;
  layout(a);
  auto up = [&](void* dst, const void* src, size_t bytes) -> dmg_status {
    if (bytes) DMG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream));
    return DMG_OK;
  };
  DMG_CHECK(up(t->Crp, C.rp.data(), C.rp.size() * sizeof(int)));
  DMG_CHECK(up(t->Cci, C.ci.data(), C.ci.size() * sizeof(int)));
  DMG_CHECK(up(t->Cv, C.v.data(), C.v.size() * sizeof(double)));
  DMG_CHECK(up(t->CTrp, CT.rp.data(), CT.rp.size() * sizeof(int)));
  DMG_CHECK(up(t->CTci, CT.ci.data(), CT.ci.size() * sizeof(int)));
  DMG_CHECK(up(t->CTv, CT.v.data(), CT.v.size() * sizeof(double)));
  DMG_CHECK(up(t->Mrp, M.rp.data(), M.rp.size() * sizeof(int)));
  DMG_CHECK(up(t->Mci, M.ci.data(), M.ci.size() * sizeof(int)));
  DMG_CHECK(up(t->Mv, M.v.data(), M.v.size() * sizeof(double)));
  DMG_CHECK(up(t->dof, dof_p.data(), size_t(nv)));
  DMG_CHECK(up(t->perm, perm.data(), size_t(nv) * sizeof(int)));
  DMG_HIP(hipStreamSynchronize(stream));  // host vectors go out of scope
  out = std::move(t);
  return DMG_OK;
}

}  // namespace dmg

using namespace dmg;

extern "C" {

dmg_status dmg_transfer_create(int32_t nv, int32_t nt, const double* xy_c, const double* xy_p,
                               const int32_t* tris, const uint8_t* dof, int32_t nx, int32_t ny,
                               int32_t nq, hipStream_t stream, dmg_transfer** out) {
  clear_error();
  if (!out) return fail(DMG_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (!xy_c || !xy_p || !tris || !dof) return fail(DMG_ERR_INVALID_ARG, "null mesh array");
  if (nv <= 0 || nt <= 0) return fail(DMG_ERR_INVALID_ARG, "empty mesh (nv=%d, nt=%d)", nv, nt);
  if (nx < 3 || ny < 3) return fail(DMG_ERR_DIMS, "grid dims must be >= 3");
  if (nq < 0 || nq > 32) return fail(DMG_ERR_INVALID_ARG, "nq must be in [0,32]");
  for (int64_t k = 0; k < int64_t(nt) * 3; ++k)
    if (tris[k] < 0 || tris[k] >= nv)
      return fail(DMG_ERR_INVALID_ARG, "triangle vertex index %d out of range", tris[k]);
  Mesh m{nv, nt, xy_c, xy_p, tris, dof, {}, {}};
  build_adjacency(m);
  std::unique_ptr<dmg_transfer> t;
  DMG_CHECK(transfer_build(m, nx, ny, nq, locality_order(m, nx, ny), stream, t));
  *out = t.release();
  return DMG_OK;
}

dmg_status dmg_transfer_info(const dmg_transfer* t, int64_t* nnz_C, int64_t* nnz_M) {
  clear_error();
  if (!t) return fail(DMG_ERR_INVALID_ARG, "null transfer");
  if (nnz_C) *nnz_C = t->nnzC;
  if (nnz_M) *nnz_M = t->nnzM;
  return DMG_OK;
}

dmg_status dmg_transfer_from_grid(dmg_transfer* t, const double* u_c, double* u_p,
                                  hipStream_t stream) {
  clear_error();
  if (!t || !u_c || !u_p) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  DMG_CHECK(launch_from_start(t, u_c, nullptr, stream));
  return cg2_tail(t, u_p, X2Mode::kScatter, nullptr, stream);
}

dmg_status dmg_transfer_to_grid(dmg_transfer* t, const double* r_p, double* r_c,
                                hipStream_t stream) {
  clear_error();
  if (!t || !r_p || !r_c) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  k_t_init_to<<<tblocks(t->nv, kMG), 256, 0, stream>>>(r_p, t->perm, t->dof, t->r, t->nv,
                                                       t->partials);
  DMG_CHECK(launch_check("transfer r_p"));
  DMG_CHECK(cg2_tail(t, t->x, X2Mode::kStore, nullptr, stream));
  return launch_ct(t, t->x, r_c, nullptr, stream);
}

void dmg_transfer_destroy(dmg_transfer* t) { delete t; }

}  // extern "C"
