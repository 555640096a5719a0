// Grid <-> mesh transfers by L2 projection: P = M_p^{-1} C and R = P^T = C^T M_p^{-1}
// (paper Sec. 2.3), with M_p^{-1} applied by two iterations of unpreconditioned CG.
//
// Setup (host, C++, once per mesh): the coupled mass C of Sec. 2.3.1 is evaluated in the
// computational domain.  Every physical triangle is mapped to a straight triangle through the
// images of its vertices; the grid cells overlapping its bounding box are visited with an
// nq x nq Gauss rule per cell; quadrature points outside the mapped triangle contribute nothing;
// inside, the P1 basis is evaluated through the mapped triangle's barycentric coordinates and
// the Jacobian factor is the constant area(tau_p)/area(mapped tau).  Rows are assembled
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

#include "dmg_internal.h"

struct dmg_transfer {
  int nv = 0, nx = 0, ny = 0;
  int64_t nnzC = 0, nnzM = 0;
  int *Crp = nullptr, *Cci = nullptr, *CTrp = nullptr, *CTci = nullptr, *Mrp = nullptr,
      *Mci = nullptr;
  double *Cv = nullptr, *CTv = nullptr, *Mv = nullptr;
  unsigned char* dof = nullptr;
  double *y = nullptr, *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr;
  double *partials = nullptr, *scal = nullptr;
  void* block = nullptr;
  ~dmg_transfer() {
    if (block) (void)hipFree(block);
  }
};

namespace dmg {
namespace {

struct Csr {
  std::vector<int> rp, ci;
  std::vector<double> v;
};

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

struct Mesh {
  int nv, nt;
  const double *xy_c, *xy_p;
  const int* tris;
  const uint8_t* dof;
  std::vector<int> vt_ptr, vt;  // vertex -> incident triangles
};

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

Csr assemble_C(const Mesh& m, int nx, int ny, int nq) {
  std::vector<double> qx, qw;
  gauss01(nq, qx, qw);
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
__device__ __forceinline__ double block_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double ws[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) ws[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = ((ws[0] + ws[1]) + ws[2]) + ws[3];
  return t;
}

// y = A x, one row per thread
__global__ __launch_bounds__(256) void k_spmv(const int* __restrict__ rp, const int* __restrict__ ci,
                                              const double* __restrict__ v,
                                              const double* __restrict__ x, double* __restrict__ y,
                                              int n) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int k = rp[r]; k < rp[r + 1]; ++k) acc += v[k] * x[ci[k]];
    y[r] = acc;
  }
}

// q = M p; partials of p.q
__global__ __launch_bounds__(256) void k_spmv_dot(const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const double* __restrict__ v,
                                                  const double* __restrict__ p,
                                                  double* __restrict__ q, int n,
                                                  double* __restrict__ partials) {
  double acc = 0.0;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int k = rp[r]; k < rp[r + 1]; ++k) s += v[k] * p[ci[k]];
    q[r] = s;
    acc += p[r] * s;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// r = p = mask * y; x = 0; partials of r.r
__global__ __launch_bounds__(256) void k_cg_init(const double* __restrict__ y,
                                                 const unsigned char* __restrict__ dof,
                                                 double* __restrict__ x, double* __restrict__ r,
                                                 double* __restrict__ p, int n,
                                                 double* __restrict__ partials) {
  double acc = 0.0;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const double val = dof[k] ? y[k] : 0.0;
    r[k] = val;
    p[k] = val;
    x[k] = 0.0;
    acc += val * val;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// alpha = rr/pq (0 when rr == 0); x += alpha p; optionally r -= alpha q with partials of r.r
__global__ __launch_bounds__(256) void k_cg_xr(double* __restrict__ x, double* __restrict__ r,
                                               const double* __restrict__ p,
                                               const double* __restrict__ q,
                                               const double* __restrict__ rr,
                                               const double* __restrict__ pq, int n,
                                               int update_r, double* __restrict__ partials) {
  const double alpha = rr[0] == 0.0 ? 0.0 : rr[0] / pq[0];
  double acc = 0.0;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    x[k] = x[k] + alpha * p[k];
    if (update_r) {
      const double rv = r[k] - alpha * q[k];
      r[k] = rv;
      acc += rv * rv;
    }
  }
  if (update_r) {
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
  }
}

// p = r + (rr_new / rr_old) p
__global__ __launch_bounds__(256) void k_cg_p(double* __restrict__ p, const double* __restrict__ r,
                                              const double* __restrict__ rr_old,
                                              const double* __restrict__ rr_new, int n) {
  const double beta = rr_old[0] == 0.0 ? 0.0 : rr_new[0] / rr_old[0];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    p[k] = r[k] + beta * p[k];
}

__global__ __launch_bounds__(256) void k_zero_ring(double* __restrict__ v, int nx, int ny) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nx) {
    v[k] = 0.0;
    v[size_t(ny - 1) * nx + k] = 0.0;
  }
  if (k < ny) {
    v[size_t(k) * nx] = 0.0;
    v[size_t(k) * nx + nx - 1] = 0.0;
  }
}

unsigned nblocks(int n) {
  const int b = (n + 255) / 256;
  return unsigned(std::max(1, std::min(b, kReduceBlocks)));
}

// x = CG2(M, y) on the transfer's vectors (x is t->x).
dmg_status cg2(dmg_transfer* t, const double* y, hipStream_t s) {
  const int n = t->nv;
  double* sc = t->scal;  // pairs: [0] rr0, [2] pq0, [4] rr1, [6] pq1
  k_cg_init<<<kReduceBlocks, 256, 0, s>>>(y, t->dof, t->x, t->r, t->p, n, t->partials);
  DMG_CHECK(launch_check("cg_init"));
  DMG_CHECK(launch_finalize(t->partials, sc + 0, s));
  // iteration 1
  k_spmv_dot<<<kReduceBlocks, 256, 0, s>>>(t->Mrp, t->Mci, t->Mv, t->p, t->q, n, t->partials);
  DMG_CHECK(launch_check("spmv_dot"));
  DMG_CHECK(launch_finalize(t->partials, sc + 2, s));
  k_cg_xr<<<kReduceBlocks, 256, 0, s>>>(t->x, t->r, t->p, t->q, sc + 0, sc + 2, n, 1, t->partials);
  DMG_CHECK(launch_check("cg_xr"));
  DMG_CHECK(launch_finalize(t->partials, sc + 4, s));
  k_cg_p<<<nblocks(n), 256, 0, s>>>(t->p, t->r, sc + 0, sc + 4, n);
  DMG_CHECK(launch_check("cg_p"));
  // iteration 2 (r and p are not needed afterwards)
  k_spmv_dot<<<kReduceBlocks, 256, 0, s>>>(t->Mrp, t->Mci, t->Mv, t->p, t->q, n, t->partials);
  DMG_CHECK(launch_check("spmv_dot"));
  DMG_CHECK(launch_finalize(t->partials, sc + 6, s));
  k_cg_xr<<<kReduceBlocks, 256, 0, s>>>(t->x, t->r, t->p, t->q, sc + 4, sc + 6, n, 0, t->partials);
  return launch_check("cg_xr");
}

}  // namespace
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
  if (nq < 1 || nq > 32) return fail(DMG_ERR_INVALID_ARG, "nq must be in [1,32]");
  for (int64_t k = 0; k < int64_t(nt) * 3; ++k)
    if (tris[k] < 0 || tris[k] >= nv)
      return fail(DMG_ERR_INVALID_ARG, "triangle vertex index %d out of range", tris[k]);
  Mesh m{nv, nt, xy_c, xy_p, tris, dof, {}, {}};
  build_adjacency(m);
  Csr C = assemble_C(m, nx, ny, nq);
  Csr M = assemble_M(m);
  Csr CT = transpose(C, nx * ny);
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
    t->y = a.take<double>(nv);
    t->x = a.take<double>(nv);
    t->r = a.take<double>(nv);
    t->p = a.take<double>(nv);
    t->q = a.take<double>(nv);
    t->partials = a.take<double>(kReduceBlocks);
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
  DMG_CHECK(up(t->dof, dof, size_t(nv)));
  DMG_HIP(hipStreamSynchronize(stream));  // host vectors go out of scope
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
  k_spmv<<<nblocks(t->nv), 256, 0, stream>>>(t->Crp, t->Cci, t->Cv, u_c, t->y, t->nv);
  DMG_CHECK(launch_check("spmv C"));
  DMG_CHECK(cg2(t, t->y, stream));
  DMG_HIP(hipMemcpyAsync(u_p, t->x, size_t(t->nv) * sizeof(double), hipMemcpyDeviceToDevice,
                         stream));
  return DMG_OK;
}

dmg_status dmg_transfer_to_grid(dmg_transfer* t, const double* r_p, double* r_c,
                                hipStream_t stream) {
  clear_error();
  if (!t || !r_p || !r_c) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  DMG_CHECK(cg2(t, r_p, stream));
  const int ng = t->nx * t->ny;
  k_spmv<<<nblocks(ng), 256, 0, stream>>>(t->CTrp, t->CTci, t->CTv, t->x, r_c, ng);
  DMG_CHECK(launch_check("spmv C^T"));
  return DMG_OK;
}

void dmg_transfer_destroy(dmg_transfer* t) { delete t; }

}  // extern "C"
