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

void gauss_rule01(int nq, std::vector<double>& x, std::vector<double>& w) { gauss01(nq, x, w); }

namespace {

// nq >= 1: the rasterised rule (nq x nq Gauss points per overlapped cell, zero outside the
// mapped triangle); nq == 0: exact integration over the triangle-cell overlaps.
Csr assemble_C(const Mesh& m, int nx, int ny, int nq) {
  std::vector<double> qx, qw;
  if (nq > 0) gauss01(nq, qx, qw);
  const double hx = 2.0 / (nx - 1), hy = 2.0 / (ny - 1);
  return rows_parallel(m.nv, [&](int r0, int r1, Csr& out) {
    std::unordered_map<int, double> row;
    std::vector<std::pair<int, double>> sorted;
    for (int v = r0; v < r1; ++v) {
      row.clear();
      if (m.dof[v]) {
        for (int k = m.vt_ptr[v]; k < m.vt_ptr[v + 1]; ++k) {
          const int* tv = m.tris + 3 * m.vt[k];
          const int a = tv[0] == v ? 0 : (tv[1] == v ? 1 : 2);
          const double det = tri_area2(m.xy_c, tv);
          if (det == 0.0) continue;
          const double jac = std::fabs(tri_area2(m.xy_p, tv)) / std::fabs(det);
          double tri[3][2];
          for (int q = 0; q < 3; ++q) {
            tri[q][0] = m.xy_c[2 * tv[q]];
            tri[q][1] = m.xy_c[2 * tv[q] + 1];
          }
          const int i0 = grid_cell(std::min({tri[0][0], tri[1][0], tri[2][0]}), hx, nx);
          const int i1 = grid_cell(std::max({tri[0][0], tri[1][0], tri[2][0]}), hx, nx);
          const int j0 = grid_cell(std::min({tri[0][1], tri[1][1], tri[2][1]}), hy, ny);
          const int j1 = grid_cell(std::max({tri[0][1], tri[1][1], tri[2][1]}), hy, ny);
          for (int cj = j0; cj <= j1; ++cj)
            for (int ci = i0; ci <= i1; ++ci) {
              double w[3][4];
              cell_integrals(tri, det, ci, cj, hx, hy, nq, qx.data(), qw.data(), w);
              const int g00 = cj * nx + ci;
              const int gi[4] = {g00, g00 + 1, g00 + nx, g00 + nx + 1};
              for (int g = 0; g < 4; ++g) {
                const int gx = gi[g] % nx, gy = gi[g] / nx;
                if (gx == 0 || gx == nx - 1 || gy == 0 || gy == ny - 1) continue;
                row[gi[g]] += jac * w[a][g];
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

Csr assemble_M(const Mesh& m) {
  return rows_parallel(m.nv, [&](int r0, int r1, Csr& out) {
  std::vector<std::pair<int, double>> row;
  for (int v = r0; v < r1; ++v) {
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
  });
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

// from_grid start: r0 = dof * (C u_c) (mesh rows in the internal order; dof nullable: all ones);
// partials of r0.r0
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
    const double val = (!dof || dof[r]) ? y : 0.0;
    if (lane == 0) {
      r0[r] = val;
      acc += val * val;
    }
  }
  const double t = mesh_block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// to_grid start: r0 = dof * r_p taken into the internal order (dof, perm nullable: all ones, the
// identity); partials of r0.r0
__global__ __launch_bounds__(256) void k_t_init_to(const double* __restrict__ r_p,
                                                   const int* __restrict__ perm,
                                                   const unsigned char* __restrict__ dof,
                                                   double* __restrict__ r0, int n,
                                                   double* __restrict__ partials) {
  double acc = 0.0;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
    const double val = (!dof || dof[r]) ? r_p[perm ? perm[r] : r] : 0.0;
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
  if (t->mf) return mf_launch_from(t, u_c, stop, s);
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
  if (t->mf) return mf_launch_ct(t, x, r_c, stop, s);
  const int ng = t->nx * t->ny;
  k_t_ct<<<tblocks(ng, kCG), 256, 0, s>>>(t->CTrp, t->CTci, t->CTv, x, r_c, ng, stop);
  return launch_check("transfer C^T x");
}

// Internal vertex order: by the grid cell holding each vertex's image (row-major), so that the
// rows of C and M_p that are used together sit together and their gathers stay in cache.
std::vector<int> locality_order(const Mesh& m, int nx, int ny) {
  // counting sort by cell (stable: vertices of one cell keep their index order)
  const double hx = 2.0 / (nx - 1), hy = 2.0 / (ny - 1);
  const size_t ncell = size_t(nx - 1) * (ny - 1);
  std::vector<int> key(m.nv);
  std::vector<int> start(ncell + 1, 0);
  for (int v = 0; v < m.nv; ++v) {
    const int ix = std::min(std::max(int(std::floor((m.xy_c[2 * v] + 1.0) / hx)), 0), nx - 2);
    const int iy = std::min(std::max(int(std::floor((m.xy_c[2 * v + 1] + 1.0) / hy)), 0), ny - 2);
    key[v] = iy * (nx - 1) + ix;
    start[size_t(key[v]) + 1]++;
  }
  for (size_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
  std::vector<int> perm(m.nv);
  for (int v = 0; v < m.nv; ++v) perm[start[key[v]]++] = v;
  return perm;
}

Csr permute_rows(const Csr& a, const std::vector<int>& perm, const std::vector<int>* colmap) {
  return rows_parallel(int(perm.size()), [&](int r0, int r1, Csr& out) {
    std::vector<std::pair<int, double>> row;
    for (int i = r0; i < r1; ++i) {
      const int o = perm[i];
      row.clear();
      for (int k = a.rp[o]; k < a.rp[o + 1]; ++k)
        row.emplace_back(colmap ? (*colmap)[a.ci[k]] : a.ci[k], a.v[k]);
      if (colmap) std::sort(row.begin(), row.end());
      for (auto& e : row) {
        out.ci.push_back(e.first);
        out.v.push_back(e.second);
      }
      out.rp.push_back(int(out.ci.size()));
    }
  });
}

dmg_status transfer_build(const Mesh& m, int nx, int ny, int nq, const std::vector<int>& perm,
                          CForm form, hipStream_t stream, std::unique_ptr<dmg_transfer>& out) {
  const int nv = m.nv;
  const size_t ng = size_t(nx) * ny;
  std::unique_ptr<dmg_transfer> t(new dmg_transfer);
  t->nv = nv;
  t->nx = nx;
  t->ny = ny;
  auto up = [&](void* dst, const void* src, size_t bytes) -> dmg_status {
    if (bytes) DMG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream));
    return DMG_OK;
  };
  // C and C^T: on the device, else (or when a row is too long for the device merge) on the host;
  // or neither, the overlap sets instead
  bool have_C = false;
  if (form == CForm::kMatrixFree) {
    DMG_CHECK(mf_build(m, nx, ny, nq, perm, stream, t.get()));
    have_C = true;
  } else if (form == CForm::kDevice) {
    DeviceCsrPair d;
    const dmg_status st = device_assemble_C(m, nx, ny, nq, perm, stream, d);
    if (st == DMG_OK) {
      t->cblock = d.block;
      t->Crp = d.rp;
      t->Cci = d.ci;
      t->Cv = d.v;
      t->CTrp = d.trp;
      t->CTci = d.tci;
      t->CTv = d.tv;
      t->nnzC = d.nnz;
      t->device_C = have_C = true;
    } else if (st != DMG_ERR_UNSUPPORTED) {
      return st;
    }
    clear_error();
  }
  if (!have_C) {
    const Csr C = permute_rows(assemble_C(m, nx, ny, nq), perm, nullptr);
    if (C.ci.size() >= (size_t(1) << 31))
      return fail(DMG_ERR_INVALID_ARG, "transfer matrices exceed 2^31 nonzeros");
    const Csr CT = transpose(C, int(ng));
    t->nnzC = int64_t(C.ci.size());
    Arena sz;
    auto layout = [&](Arena& a) {
      t->Crp = a.take<int>(nv + 1);
      t->Cci = a.take<int>(C.ci.size() + 1);
      t->Cv = a.take<double>(C.v.size() + 1);
      t->CTrp = a.take<int>(ng + 1);
      t->CTci = a.take<int>(CT.ci.size() + 1);
      t->CTv = a.take<double>(CT.v.size() + 1);
    };
    layout(sz);
    DMG_HIP(hipMalloc(&t->cblock, sz.used));
    Arena a;
    a.base = static_cast<char*>(t->cblock);
    a.cap = sz.used;
    layout(a);
    DMG_CHECK(up(t->Crp, C.rp.data(), C.rp.size() * sizeof(int)));
    DMG_CHECK(up(t->Cci, C.ci.data(), C.ci.size() * sizeof(int)));
    DMG_CHECK(up(t->Cv, C.v.data(), C.v.size() * sizeof(double)));
    DMG_CHECK(up(t->CTrp, CT.rp.data(), CT.rp.size() * sizeof(int)));
    DMG_CHECK(up(t->CTci, CT.ci.data(), CT.ci.size() * sizeof(int)));
    DMG_CHECK(up(t->CTv, CT.v.data(), CT.v.size() * sizeof(double)));
    DMG_HIP(hipStreamSynchronize(stream));  // host vectors go out of scope
  }
  std::vector<int> newidx(nv);
  for (int i = 0; i < nv; ++i) newidx[perm[i]] = i;
  const Csr M = permute_rows(assemble_M(m), perm, &newidx);
  if (M.ci.size() >= (size_t(1) << 31))
    return fail(DMG_ERR_INVALID_ARG, "transfer matrices exceed 2^31 nonzeros");
  std::vector<uint8_t> dof_p(nv);
  for (int i = 0; i < nv; ++i) dof_p[i] = m.dof[perm[i]];
  t->nnzM = int64_t(M.ci.size());
  Arena sz;
  auto layout = [&](Arena& a) {
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
  DMG_CHECK(up(t->Mrp, M.rp.data(), M.rp.size() * sizeof(int)));
  DMG_CHECK(up(t->Mci, M.ci.data(), M.ci.size() * sizeof(int)));
  DMG_CHECK(up(t->Mv, M.v.data(), M.v.size() * sizeof(double)));
  DMG_CHECK(up(t->dof, dof_p.data(), size_t(nv)));
  DMG_CHECK(up(t->perm, perm.data(), size_t(nv) * sizeof(int)));
  DMG_HIP(hipStreamSynchronize(stream));  // host vectors go out of scope
  out = std::move(t);
  return DMG_OK;
}

// Workspace of a transfer created from caller CSR matrices: C^T, the CG vectors, partials and
// scalars, and the transpose's integer scratch.
void csr_transfer_layout(Arena& a, dmg_transfer* t, int np, int nc, int64_t nnz, int** cnt,
                         int** pos, int** sums, int** flag) {
  t->CTrp = a.take<int>(size_t(nc) + 1);
  t->CTci = a.take<int>(size_t(nnz) + 1);
  t->CTv = a.take<double>(size_t(nnz) + 1);
  t->x = a.take<double>(np);
  t->r = a.take<double>(np);
  t->p = a.take<double>(np);
  t->q = a.take<double>(np);
  t->partials = a.take<double>(kTBlocks);
  t->scal = a.take<double>(16);
  *cnt = a.take<int>(size_t(nc) + 1);
  *pos = a.take<int>(size_t(nc));
  *sums = a.take<int>(size_t(transpose_sums(nc)));
  *flag = a.take<int>(1);
}

}  // namespace dmg

using namespace dmg;

extern "C" {

dmg_status dmg_transfer_workspace_bytes(int32_t np, int32_t nc, int64_t nnz_C, size_t* bytes) {
  clear_error();
  if (!bytes) return fail(DMG_ERR_INVALID_ARG, "null output");
  if (np <= 0 || nc <= 0 || nnz_C < 0 || nnz_C >= (int64_t(1) << 31))
    return fail(DMG_ERR_INVALID_ARG, "bad sizes (Np=%d, Nc=%d, nnz_C=%lld)", np, nc,
                (long long)nnz_C);
  dmg_transfer t;
  Arena sz;
  int *cnt, *pos, *sums, *flag;
  csr_transfer_layout(sz, &t, np, nc, nnz_C, &cnt, &pos, &sums, &flag);
  *bytes = sz.used;
  return DMG_OK;
}

dmg_status dmg_transfer_create(int32_t np, int32_t nc, const int32_t* C_rowptr,
                               const int32_t* C_col, const double* C_val, const int32_t* M_rowptr,
                               const int32_t* M_col, const double* M_val, void* workspace,
                               size_t ws_bytes, hipStream_t stream, dmg_transfer** out) {
  clear_error();
  if (!out) return fail(DMG_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (np <= 0 || nc <= 0) return fail(DMG_ERR_INVALID_ARG, "bad sizes (Np=%d, Nc=%d)", np, nc);
  if (!C_rowptr || !C_col || !C_val || !M_rowptr || !M_col || !M_val)
    return fail(DMG_ERR_INVALID_ARG, "null CSR array");
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return fail(DMG_ERR_WORKSPACE, "workspace missing or not 256-byte aligned");
  // the entry counts sit on the device: read them (this call synchronises `stream`)
  int ends[4] = {0, 0, 0, 0};
  DMG_HIP(hipMemcpyAsync(&ends[0], C_rowptr, sizeof(int), hipMemcpyDeviceToHost, stream));
  DMG_HIP(hipMemcpyAsync(&ends[1], C_rowptr + np, sizeof(int), hipMemcpyDeviceToHost, stream));
  DMG_HIP(hipMemcpyAsync(&ends[2], M_rowptr, sizeof(int), hipMemcpyDeviceToHost, stream));
  DMG_HIP(hipMemcpyAsync(&ends[3], M_rowptr + np, sizeof(int), hipMemcpyDeviceToHost, stream));
  DMG_HIP(hipStreamSynchronize(stream));
  if (ends[0] != 0 || ends[2] != 0 || ends[1] < 0 || ends[3] < 0)
    return fail(DMG_ERR_INVALID_ARG, "row pointers must start at 0 and end at the entry count");
  std::unique_ptr<dmg_transfer> t(new dmg_transfer);
  Arena sz;
  int *cnt, *pos, *sums, *flag;
  csr_transfer_layout(sz, t.get(), np, nc, ends[1], &cnt, &pos, &sums, &flag);
  if (ws_bytes < sz.used)
    return fail(DMG_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, sz.used);
  Arena a;
  a.base = static_cast<char*>(workspace);
  a.cap = ws_bytes;
  csr_transfer_layout(a, t.get(), np, nc, ends[1], &cnt, &pos, &sums, &flag);
  // structure of both matrices (M_p square), checked on the device before C^T is formed
  bool okC = false, okM = false;
  DMG_CHECK(device_check_csr(C_rowptr, C_col, np, nc, ends[1], flag, &okC, stream));
  DMG_CHECK(device_check_csr(M_rowptr, M_col, np, np, ends[3], flag, &okM, stream));
  if (!okC || !okM)
    return fail(DMG_ERR_INVALID_ARG, "CSR structure of %s: row pointers not non-decreasing from 0 "
                "to the entry count, or a column index out of range", okC ? "M_p" : "C");
  t->nv = np;
  t->nx = nc;
  t->ny = 1;
  t->nnzC = ends[1];
  t->nnzM = ends[3];
  t->Crp = const_cast<int*>(C_rowptr);
  t->Cci = const_cast<int*>(C_col);
  t->Cv = const_cast<double*>(C_val);
  t->Mrp = const_cast<int*>(M_rowptr);
  t->Mci = const_cast<int*>(M_col);
  t->Mv = const_cast<double*>(M_val);
  t->dof = nullptr;
  t->perm = nullptr;
  t->borrowed = true;
  DMG_CHECK(device_transpose(C_rowptr, C_col, C_val, np, nc, t->CTrp, t->CTci, t->CTv, cnt, pos,
                             sums, stream));
  *out = t.release();
  return DMG_OK;
}

dmg_status dmg_transfer_create_mesh(int32_t nv, int32_t nt, const double* xy_c,
                                    const double* xy_p, const int32_t* tris, const uint8_t* dof,
                                    int32_t nx, int32_t ny, int32_t nq, int32_t flags,
                                    hipStream_t stream, dmg_transfer** out) {
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
  DMG_CHECK(transfer_build(m, nx, ny, nq, locality_order(m, nx, ny), c_form(flags), stream, t));
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

dmg_status dmg_transfer_memory(const dmg_transfer* t, size_t* bytes_C, int64_t* overlap_pairs) {
  clear_error();
  if (!t) return fail(DMG_ERR_INVALID_ARG, "null transfer");
  if (bytes_C) {
    const size_t nc = size_t(t->nx) * t->ny;
    *bytes_C = t->mf ? t->mf_bytes
                     : (size_t(t->nv) + 1 + nc + 1) * sizeof(int) +
                           2 * size_t(t->nnzC) * (sizeof(int) + sizeof(double));
  }
  if (overlap_pairs) *overlap_pairs = t->mf ? t->mf_pairs : 0;
  return DMG_OK;
}

dmg_status dmg_transfer_copy_C(const dmg_transfer* t, int32_t* rp, int32_t* ci, double* v) {
  clear_error();
  if (!t || !rp || (t->nnzC > 0 && (!ci || !v)))
    return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  if (t->mf) return fail(DMG_ERR_UNSUPPORTED, "a matrix-free transfer stores no C");
  const int n = t->nv;
  std::vector<int> irp(n + 1), perm(n), ici(size_t(t->nnzC));
  std::vector<double> iv(size_t(t->nnzC));
  DMG_HIP(hipMemcpy(irp.data(), t->Crp, (n + 1) * sizeof(int), hipMemcpyDeviceToHost));
  if (t->perm) {
    DMG_HIP(hipMemcpy(perm.data(), t->perm, n * sizeof(int), hipMemcpyDeviceToHost));
  } else {
    for (int i = 0; i < n; ++i) perm[i] = i;
  }
  if (t->nnzC > 0) {
    DMG_HIP(hipMemcpy(ici.data(), t->Cci, ici.size() * sizeof(int), hipMemcpyDeviceToHost));
    DMG_HIP(hipMemcpy(iv.data(), t->Cv, iv.size() * sizeof(double), hipMemcpyDeviceToHost));
  }
  // internal row i is the caller's row perm[i]
  std::vector<int> len(n);
  for (int i = 0; i < n; ++i) len[perm[i]] = irp[i + 1] - irp[i];
  rp[0] = 0;
  for (int r = 0; r < n; ++r) rp[r + 1] = rp[r] + len[r];
  for (int i = 0; i < n; ++i) {
    const int dst = rp[perm[i]];
    for (int k = irp[i]; k < irp[i + 1]; ++k) {
      ci[dst + k - irp[i]] = ici[k];
      v[dst + k - irp[i]] = iv[k];
    }
  }
  return DMG_OK;
}

dmg_status dmg_transfer_from_grid(dmg_transfer* t, const double* u_c, double* u_p,
                                  hipStream_t stream) {
  clear_error();
  if (!t || !u_c || !u_p) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  DMG_CHECK(launch_from_start(t, u_c, nullptr, stream));
  return cg2_tail(t, u_p, t->perm ? X2Mode::kScatter : X2Mode::kStore, nullptr, stream);
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
