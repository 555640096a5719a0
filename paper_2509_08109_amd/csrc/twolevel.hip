// The two-level cycle of diffeomorphic multigrid (paper Sec. 2.2, solution phase) on the
// physical P1 system A_p u_p = f_p: symmetric multicolour Gauss-Seidel on the mesh, the residual
// restricted to the grid by R = C^T M_p^{-1}, one BoxMG V-cycle on the grid from zero, the
// correction interpolated by P = M_p^{-1} C, and a second symmetric sweep.  M_p^{-1} is the
// lumped mass (row sums of M_p) or two CG iterations on M_p (Sec. 2.3).
//
// Setup (host, once per mesh): A_p = sum_t K_t G_t with G_t the P1 element stiffness on the
// physical triangle (Dirichlet rows and columns replaced by the identity); colours by a greedy
// pass over the mesh graph (unknowns sharing a triangle are neighbours; Dirichlet vertices have
// none) in smallest-last order, which needs fewer colours, and so fewer sequential passes per
// sweep, than the caller's index order; internal vertex order colour-major,
// each colour in the grid-cell order of the transfers, so one colour is one contiguous row range.
// The transfers (C, C^T, M_p) are built in the same internal order.
//
// Solve (device): the state and the vectors live in the handle in the internal order; the caller's
// u_p and f_p are gathered at the start and u_p scattered back at the end.  Chunks of cycles run
// in one captured graph; the convergence test is taken on the device after every cycle, and
// every kernel of the chunk is a no-op once it has stopped the solve.
#include <algorithm>
#include <cmath>
#include <set>

#include "mesh_internal.h"

struct dmg_twolevel {
  std::unique_ptr<dmg_transfer> t;
  dmg_hier* grid = nullptr;  // borrowed
  int nv = 0, nx = 0, ny = 0, mass = 0;
  double gamma = 1.0;  // coarse-grid scaling: u_p += gamma P e_c
  int64_t nnzA = 0;  // stored off-diagonal entries of A_p
  std::vector<int> cs;      // colour c holds internal rows [cs[c], cs[c + 1])
  std::vector<int> colour;  // colour of each vertex, caller order
  int *Arp = nullptr, *Aci = nullptr;  // off-diagonal part of A_p, internal order
  double *Av = nullptr, *Ad = nullptr;  // its values; the diagonal
  double* ML = nullptr;                 // lumped mass (1 on Dirichlet rows)
  double *u = nullptr, *f = nullptr;    // iterate and right-hand side, internal order
  double *w = nullptr;                  // scaled residual, internal order
  double *ec = nullptr, *rc = nullptr;  // grid correction and restricted residual [ny][nx]
  double *partials = nullptr, *scal = nullptr, *hist = nullptr;
  int* flag = nullptr;  // [0] stop, [1] cycles done, [2] max cycles
  void* block = nullptr;
  double* host = nullptr;  // pinned: scalars [0..7], flags at [8..]
  double* lz = nullptr;    // lumped mass only: the scaling estimate's six grid vectors, dot
                           // partials and scalars (part of block)
  // captured chunks of 1..kChunk cycles
  hipGraphExec_t exec[dmg::kChunk] = {};
  hipGraph_t graph[dmg::kChunk] = {};
  hipStream_t graph_stream[dmg::kChunk] = {};
  void reset_graph() {
    for (int k = 0; k < dmg::kChunk; ++k) {
      if (exec[k]) (void)hipGraphExecDestroy(exec[k]);
      if (graph[k]) (void)hipGraphDestroy(graph[k]);
      exec[k] = nullptr;
      graph[k] = nullptr;
      graph_stream[k] = nullptr;
    }
  }
  ~dmg_twolevel() {
    reset_graph();
    if (block) (void)hipFree(block);
    if (host) (void)hipHostFree(host);
  }
};

namespace dmg {
namespace {

__device__ __forceinline__ bool halted(const int* stop) { return stop && *stop; }

// One colour of the sweep: u_r = (f_r - sum_{k != r} a_rk u_k) / a_rr for the rows of one colour
// [r0, r1).  Rows of one colour are not coupled, so every u_k read belongs to another colour and
// the update can be made in place.
__global__ __launch_bounds__(256) void k_tl_colour(const int* __restrict__ rp,
                                                   const int* __restrict__ ci,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ d,
                                                   const double* __restrict__ f, double* u, int r0,
                                                   int r1, const int* __restrict__ stop) {
  if (halted(stop)) return;
  const int lane = threadIdx.x & (kMG - 1);
  const int g0 = int((blockIdx.x * 256u + threadIdx.x) / kMG), ng = int(gridDim.x * 256u / kMG);
  for (int r = r0 + g0; r < r1; r += ng) {
    const double s = row_dot<kMG>(rp, ci, v, r, lane, [&](int c) { return u[c]; });
    if (lane == 0) u[r] = (f[r] - s) / d[r];
  }
}

// Residual r = f - A_p u.  kLumped: w = dof ? r / ML : 0.  kMasked: w = dof ? r : 0 with partials
// of w.w (the start of CG on M_p).  kNorm: partials of r.r only.
enum class RMode { kLumped, kMasked, kNorm };

template <RMode MODE>
__global__ __launch_bounds__(256) void k_tl_resid(const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const double* __restrict__ v,
                                                  const double* __restrict__ d,
                                                  const double* __restrict__ f,
                                                  const double* __restrict__ u,
                                                  const double* __restrict__ ML,
                                                  const unsigned char* __restrict__ dof,
                                                  double* __restrict__ w, int n,
                                                  double* __restrict__ partials,
                                                  const int* __restrict__ stop) {
  if (halted(stop)) return;
  const int lane = threadIdx.x & (kMG - 1);
  const int g0 = int((blockIdx.x * 256u + threadIdx.x) / kMG), ng = int(gridDim.x * 256u / kMG);
  double acc = 0.0;
  for (int r = g0; r < n; r += ng) {
    const double s = row_dot<kMG>(rp, ci, v, r, lane, [&](int c) { return u[c]; });
    if (lane == 0) {
      const double res = f[r] - __builtin_fma(d[r], u[r], s);
      if constexpr (MODE == RMode::kLumped) {
        w[r] = dof[r] ? res / ML[r] : 0.0;
      } else if constexpr (MODE == RMode::kMasked) {
        const double m = dof[r] ? res : 0.0;
        w[r] = m;
        acc += m * m;
      } else {
        acc += res * res;
      }
    }
  }
  if constexpr (MODE != RMode::kLumped) {
    const double t = mesh_block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
  }
}

// u += gamma * dof * (C e_c) / ML: the lumped interpolation of the grid correction, scaled and
// added in place.
__global__ __launch_bounds__(256) void k_tl_prolong(const int* __restrict__ rp,
                                                    const int* __restrict__ ci,
                                                    const double* __restrict__ v,
                                                    const double* __restrict__ ec,
                                                    const double* __restrict__ ML,
                                                    const unsigned char* __restrict__ dof,
                                                    double* __restrict__ u, int n, double gamma,
                                                    const int* __restrict__ stop) {
  if (halted(stop)) return;
  const int lane = threadIdx.x & (kMG - 1);
  const int g0 = int((blockIdx.x * 256u + threadIdx.x) / kMG), ng = int(gridDim.x * 256u / kMG);
  for (int r = g0; r < n; r += ng) {
    const double s = row_dot<kMG>(rp, ci, v, r, lane, [&](int c) { return ec[c]; });
    if (lane == 0 && dof[r]) u[r] += gamma * (s / ML[r]);
  }
}

// The same two operations from C v formed beforehand (cx = dof * (C v), a matrix-free transfer):
// u += gamma cx / ML on the free rows, or x = cx / ML stored (zero on Dirichlet rows).
template <bool ADD>
__global__ __launch_bounds__(256) void k_tl_lumped(const double* __restrict__ cx,
                                                   const double* __restrict__ ML,
                                                   const unsigned char* __restrict__ dof,
                                                   double* __restrict__ out, int n, double gamma,
                                                   const int* __restrict__ stop) {
  if (halted(stop)) return;
  for (int r = int(blockIdx.x) * 256 + int(threadIdx.x); r < n; r += int(gridDim.x) * 256) {
    if constexpr (ADD) {
      if (dof[r]) out[r] += gamma * (cx[r] / ML[r]);
    } else {
      out[r] = dof[r] ? cx[r] / ML[r] : 0.0;
    }
  }
}

// ---- the scaling estimate (generalized Lanczos on grid vectors) ----------------------------
// x = P v = dof * (C v) / ML on the mesh (lumped interpolation, stored).
__global__ __launch_bounds__(256) void k_tl_interp(const int* __restrict__ rp,
                                                   const int* __restrict__ ci,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ vc,
                                                   const double* __restrict__ ML,
                                                   const unsigned char* __restrict__ dof,
                                                   double* __restrict__ x, int n) {
  const int lane = threadIdx.x & (kMG - 1);
  const int g0 = int((blockIdx.x * 256u + threadIdx.x) / kMG), ng = int(gridDim.x * 256u / kMG);
  for (int r = g0; r < n; r += ng) {
    const double s = row_dot<kMG>(rp, ci, v, r, lane, [&](int c) { return vc[c]; });
    if (lane == 0) x[r] = dof[r] ? s / ML[r] : 0.0;
  }
}

// y = dof * (A_p x) / ML on the mesh (the stiffness product followed by the lumped mass of R).
__global__ __launch_bounds__(256) void k_tl_apply_scaled(const int* __restrict__ rp,
                                                         const int* __restrict__ ci,
                                                         const double* __restrict__ v,
                                                         const double* __restrict__ d,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ ML,
                                                         const unsigned char* __restrict__ dof,
                                                         double* __restrict__ y, int n) {
  const int lane = threadIdx.x & (kMG - 1);
  const int g0 = int((blockIdx.x * 256u + threadIdx.x) / kMG), ng = int(gridDim.x * 256u / kMG);
  for (int r = g0; r < n; r += ng) {
    const double s = row_dot<kMG>(rp, ci, v, r, lane, [&](int c) { return x[c]; });
    if (lane == 0) y[r] = dof[r] ? __builtin_fma(d[r], x[r], s) / ML[r] : 0.0;
  }
}

constexpr int kLzBlocks = 1024;  // fixed partial count of the Lanczos dot products

// Interior part of v0 (boundary ring 0).
__global__ __launch_bounds__(256) void k_lz_mask(const double* __restrict__ v0,
                                                 double* __restrict__ x, int nx, int ny) {
  const size_t N = size_t(nx) * ny;
  for (size_t v = blockIdx.x * 256u + threadIdx.x; v < N; v += size_t(gridDim.x) * 256u) {
    const int j = int(v / nx), i = int(v % nx);
    x[v] = (i > 0 && i < nx - 1 && j > 0 && j < ny - 1) ? v0[v] : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_lz_dot(const double* __restrict__ x,
                                                const double* __restrict__ y, size_t n,
                                                double* __restrict__ partials) {
  double acc = 0.0;
  for (size_t k = blockIdx.x * 256u + threadIdx.x; k < n; k += size_t(gridDim.x) * 256u)
    acc = __builtin_fma(x[k], y[k], acc);
  const double t = mesh_block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// x *= a, y *= a
__global__ __launch_bounds__(256) void k_lz_scale2(double* __restrict__ x, double* __restrict__ y,
                                                   double a, size_t n) {
  for (size_t k = blockIdx.x * 256u + threadIdx.x; k < n; k += size_t(gridDim.x) * 256u) {
    x[k] *= a;
    y[k] *= a;
  }
}

// w = (w - alpha v) - beta vp and g = (g - alpha Av) - beta Avp (then g = A w)
__global__ __launch_bounds__(256) void k_lz_update(double* __restrict__ w,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ vp,
                                                   double* __restrict__ g,
                                                   const double* __restrict__ Av,
                                                   const double* __restrict__ Avp, double alpha,
                                                   double beta, size_t n) {
  for (size_t k = blockIdx.x * 256u + threadIdx.x; k < n; k += size_t(gridDim.x) * 256u) {
    w[k] = (w[k] - alpha * v[k]) - beta * vp[k];
    g[k] = (g[k] - alpha * Av[k]) - beta * Avp[k];
  }
}

// Internal-order copies of the caller's vectors (u_p may be null) and the way back.
__global__ __launch_bounds__(256) void k_tl_gather(const double* __restrict__ u_p,
                                                   const double* __restrict__ f_p,
                                                   const int* __restrict__ perm,
                                                   double* __restrict__ u, double* __restrict__ f,
                                                   int n) {
  for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
    const int o = perm[r];
    u[r] = u_p ? u_p[o] : 0.0;
    f[r] = f_p[o];
  }
}

__global__ __launch_bounds__(256) void k_tl_scatter(const double* __restrict__ u,
                                                    const int* __restrict__ perm,
                                                    double* __restrict__ u_p, int n) {
  for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) u_p[perm[r]] = u[r];
}

// Solve start from the partials of ||f - A u_0||^2: sc[0..1] = sc[2..3] = (r0^2, r0) (the
// history's denominator and the current residual), sc[6] = (rtol r0)^2; the solve stops at once
// only when r0 is zero or not finite, or when no cycle is allowed.
__global__ __launch_bounds__(256) void k_tl_start(const double* __restrict__ partials, int count,
                                                  double* __restrict__ sc, int* __restrict__ st,
                                                  double rtol, int max_iters) {
  double acc = 0.0;
  for (int k = threadIdx.x; k < count; k += 256) acc += partials[k];
  const double t = mesh_block_sum(acc);
  if (threadIdx.x == 0) {
    const double r0 = sqrt(t), target = rtol * r0;
    sc[0] = t;
    sc[1] = r0;
    sc[2] = t;
    sc[3] = r0;
    sc[6] = target * target;
    st[0] = (t == 0.0 || max_iters <= 0 || !isfinite(t)) ? 1 : 0;
    st[1] = 0;
    st[2] = max_iters;
  }
}

inline int row_blocks(int rows) { return tblocks(rows, kMG); }

dmg_status sweep_colour(dmg_twolevel* tl, int c, const int* stop, hipStream_t s) {
  const int r0 = tl->cs[c], r1 = tl->cs[c + 1];
  if (r1 == r0) return DMG_OK;
  k_tl_colour<<<row_blocks(r1 - r0), 256, 0, s>>>(tl->Arp, tl->Aci, tl->Av, tl->Ad, tl->f, tl->u,
                                                  r0, r1, stop);
  return launch_check("two-level colour sweep");
}

// Forward over colours first..C-1, then backward.  The backward sweep starts with the colour
// just swept; sweeping it again would recompute the same values from the same inputs, so it
// starts one colour lower.
dmg_status symmetric_sweep(dmg_twolevel* tl, const int* stop, hipStream_t s, int first = 0) {
  const int nc = int(tl->cs.size()) - 1;
  for (int c = first; c < nc; ++c) DMG_CHECK(sweep_colour(tl, c, stop, s));
  for (int c = nc - 2; c >= 0; --c) DMG_CHECK(sweep_colour(tl, c, stop, s));
  return DMG_OK;
}

// One two-level cycle on tl->u.  lead = false leaves out the pre-relaxation's first colour
// pass: right after a post-relaxation (which ends with colour 0) and a residual norm, that pass
// would reproduce the same values bit for bit.
dmg_status cycle(dmg_twolevel* tl, const int* stop, hipStream_t s, bool lead = true) {
  dmg_transfer* t = tl->t.get();
  const int n = tl->nv, nb = row_blocks(n);
  DMG_CHECK(symmetric_sweep(tl, stop, s, lead ? 0 : 1));
  if (tl->mass == 0) {
    k_tl_resid<RMode::kLumped><<<nb, 256, 0, s>>>(tl->Arp, tl->Aci, tl->Av, tl->Ad, tl->f, tl->u,
                                                  tl->ML, t->dof, tl->w, n, nullptr, stop);
    DMG_CHECK(launch_check("two-level residual"));
    DMG_CHECK(launch_ct(t, tl->w, tl->rc, stop, s));
  } else {
    // r0 of CG on M_p (and its partials) straight into the transfer's CG state
    k_tl_resid<RMode::kMasked><<<nb, 256, 0, s>>>(tl->Arp, tl->Aci, tl->Av, tl->Ad, tl->f, tl->u,
                                                  tl->ML, t->dof, t->r, n, t->partials, stop);
    DMG_CHECK(launch_check("two-level residual"));
    DMG_CHECK(cg2_tail(t, tl->w, X2Mode::kStore, stop, s));
    DMG_CHECK(launch_ct(t, tl->w, tl->rc, stop, s));
  }
  DMG_CHECK(grid_vcycle(tl->grid, tl->ec, tl->rc, true, stop, s));
  if (tl->mass == 0 && t->mf) {
    DMG_CHECK(launch_from_start(t, tl->ec, stop, s));
    k_tl_lumped<true><<<nb, 256, 0, s>>>(t->r, tl->ML, t->dof, tl->u, n, tl->gamma, stop);
    DMG_CHECK(launch_check("two-level interpolation"));
  } else if (tl->mass == 0) {
    k_tl_prolong<<<nb, 256, 0, s>>>(t->Crp, t->Cci, t->Cv, tl->ec, tl->ML, t->dof, tl->u, n,
                                    tl->gamma, stop);
    DMG_CHECK(launch_check("two-level interpolation"));
  } else {
    DMG_CHECK(launch_from_start(t, tl->ec, stop, s));
    DMG_CHECK(cg2_tail(t, tl->u, X2Mode::kAdd, stop, s, tl->gamma));
  }
  return symmetric_sweep(tl, stop, s);
}

// The repeated step of a solve: one cycle, the residual norm, the convergence test.  The solve
// sweeps colour 0 once before its first step, so every step starts its pre-relaxation at
// colour 1 (the previous step ended with colour 0 and left u unchanged since).
dmg_status step(dmg_twolevel* tl, hipStream_t s) {
  const int* stop = tl->flag;
  DMG_CHECK(cycle(tl, stop, s, false));
  const int nb = row_blocks(tl->nv);
  k_tl_resid<RMode::kNorm><<<nb, 256, 0, s>>>(tl->Arp, tl->Aci, tl->Av, tl->Ad, tl->f, tl->u,
                                              tl->ML, tl->t->dof, nullptr, tl->nv, tl->partials,
                                              stop);
  DMG_CHECK(launch_check("two-level residual norm"));
  return launch_check_step(tl->partials, nb, tl->scal + 2, tl->scal, tl->flag, tl->hist,
                           kMaxHistory, s);
}

// len (1..kChunk) cycles, through the captured graph of that chunk length.
dmg_status run_chunk(dmg_twolevel* tl, int len, hipStream_t s) {
  auto chunk = [&]() -> dmg_status {
    for (int k = 0; k < len; ++k) DMG_CHECK(step(tl, s));
    return DMG_OK;
  };
  if (s == nullptr) return chunk();  // the legacy default stream cannot be captured
  const int q = len - 1;
  if (!(tl->exec[q] && tl->graph_stream[q] == s)) {
    if (tl->exec[q]) (void)hipGraphExecDestroy(tl->exec[q]);
    if (tl->graph[q]) (void)hipGraphDestroy(tl->graph[q]);
    tl->exec[q] = nullptr;
    tl->graph[q] = nullptr;
    DMG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const dmg_status st = chunk();
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st != DMG_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(DMG_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    tl->graph[q] = g;
    e = hipGraphInstantiate(&tl->exec[q], g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      tl->reset_graph();
      return fail(DMG_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    tl->graph_stream[q] = s;
  }
  DMG_HIP(hipGraphLaunch(tl->exec[q], s));
  return DMG_OK;
}

// P1 element stiffness of triangle tv (physical coordinates xy): area * grad l_a . grad l_b with
// grad l_a = (y_b - y_c, x_c - x_b) / det over the cyclic triple (a, b, c).
void element_stiffness(const double* xy, const int* tv, double G[3][3]) {
  const double* P[3] = {xy + 2 * tv[0], xy + 2 * tv[1], xy + 2 * tv[2]};
  const double det = tri_area2(xy, tv);
  double g[3][2];
  for (int a = 0; a < 3; ++a) {
    const double* pb = P[(a + 1) % 3];
    const double* pc = P[(a + 2) % 3];
    g[a][0] = (pb[1] - pc[1]) / det;
    g[a][1] = (pc[0] - pb[0]) / det;
  }
  const double area = 0.5 * std::fabs(det);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) G[a][b] = area * (g[a][0] * g[b][0] + g[a][1] * g[b][1]);
}

// A_p in the caller's order, split into its diagonal and its off-diagonal CSR.
void assemble_A(const Mesh& m, const double* K_t, Csr& off, std::vector<double>& diag) {
  diag.assign(m.nv, 1.0);
  off = rows_parallel(m.nv, [&](int r0, int r1, Csr& out) {
  std::vector<std::pair<int, double>> row;
  for (int v = r0; v < r1; ++v) {
    row.clear();
    if (m.dof[v]) {
      double dv = 0.0;
      for (int k = m.vt_ptr[v]; k < m.vt_ptr[v + 1]; ++k) {
        const int* tv = m.tris + 3 * m.vt[k];
        const int a = tv[0] == v ? 0 : (tv[1] == v ? 1 : 2);
        double G[3][3];
        element_stiffness(m.xy_p, tv, G);
        const double kt = K_t ? K_t[m.vt[k]] : 1.0;
        for (int b = 0; b < 3; ++b) {
          if (b == a) dv += kt * G[a][a];
          else if (m.dof[tv[b]]) row.emplace_back(tv[b], kt * G[a][b]);
        }
      }
      diag[v] = dv;
      std::stable_sort(row.begin(), row.end(),
                       [](const std::pair<int, double>& x, const std::pair<int, double>& y) {
                         return x.first < y.first;
                       });
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

// The smallest member of a set of indices in [0, n): a three-level bit tree (insert, erase
// and first in a few word operations).
struct MinSet {
  std::vector<uint64_t> w0, w1, w2;
  int count = 0;
  void init(int n) {
    w0.assign((size_t(n) + 63) / 64, 0);
    w1.assign((w0.size() + 63) / 64, 0);
    w2.assign((w1.size() + 63) / 64, 0);
  }
  void insert(int v) {
    const size_t i0 = size_t(v) >> 6, i1 = i0 >> 6;
    if (!w0[i0]) {
      if (!w1[i1]) w2[i1 >> 6] |= uint64_t(1) << (i1 & 63);
      w1[i1] |= uint64_t(1) << (i0 & 63);
    }
    w0[i0] |= uint64_t(1) << (v & 63);
    ++count;
  }
  void erase(int v) {
    const size_t i0 = size_t(v) >> 6, i1 = i0 >> 6;
    w0[i0] &= ~(uint64_t(1) << (v & 63));
    if (!w0[i0]) {
      w1[i1] &= ~(uint64_t(1) << (i0 & 63));
      if (!w1[i1]) w2[i1 >> 6] &= ~(uint64_t(1) << (i1 & 63));
    }
    --count;
  }
  int first() const {
    for (size_t k = 0; k < w2.size(); ++k)
      if (w2[k]) {
        const size_t i1 = k * 64 + size_t(__builtin_ctzll(w2[k]));
        const size_t i0 = i1 * 64 + size_t(__builtin_ctzll(w1[i1]));
        return int(i0 * 64 + size_t(__builtin_ctzll(w0[i0])));
      }
    return -1;
  }
};

// Greedy colours on the mesh graph in smallest-last order (Matula and Beck): the vertices are
// taken out one at a time, each of least degree among those left (counting only neighbours
// still left; the smallest index among equals), and coloured in the reverse order, each with
// the smallest colour no coloured neighbour has.  A graph in which every subgraph has a vertex
// of degree <= d gets at most d + 1 colours this way (6 for a planar mesh graph).  The graph is
// the pattern of A_p's off-diagonal part (every coupling of unknowns sharing a triangle is
// stored, even one that sums to zero); Dirichlet vertices are isolated and take colour 0.
// Vertices wait in one index set per degree below kLowDeg, and in an ordered set of
// (degree, index) above it.
std::vector<int> greedy_colours(int nv, const Csr& g) {
  constexpr int kLowDeg = 32;
  std::vector<int> deg(nv);
  std::vector<MinSet> bucket(kLowDeg);
  std::set<int64_t> high;
  auto put = [&](int v) {
    if (deg[v] < kLowDeg) {
      if (bucket[deg[v]].w0.empty()) bucket[deg[v]].init(nv);
      bucket[deg[v]].insert(v);
    } else {
      high.insert((int64_t(deg[v]) << 32) | int64_t(v));
    }
  };
  auto take = [&](int v) {
    if (deg[v] < kLowDeg) bucket[deg[v]].erase(v);
    else high.erase((int64_t(deg[v]) << 32) | int64_t(v));
  };
  for (int v = 0; v < nv; ++v) {
    deg[v] = g.rp[v + 1] - g.rp[v];
    put(v);
  }
  std::vector<char> gone(nv, 0);
  std::vector<int> removed;
  removed.reserve(nv);
  int dmin = 0;  // no vertex left has a smaller degree
  for (int step = 0; step < nv; ++step) {
    while (dmin < kLowDeg && bucket[dmin].count == 0) ++dmin;
    const int v = dmin < kLowDeg ? bucket[dmin].first() : int(*high.begin() & 0xffffffff);
    take(v);
    gone[v] = 1;
    removed.push_back(v);
    for (int k = g.rp[v]; k < g.rp[v + 1]; ++k) {
      const int w = g.ci[k];
      if (gone[w]) continue;
      take(w);
      --deg[w];
      put(w);
    }
    // each neighbour left lost one; the least degree fell by at most one
    dmin = std::max(0, std::min(dmin, kLowDeg) - 1);
  }
  std::vector<int> col(nv, -1);
  std::vector<int> mark;  // mark[c] == v: colour c is taken by a neighbour of v
  for (auto it = removed.rbegin(); it != removed.rend(); ++it) {
    const int v = *it;
    for (int k = g.rp[v]; k < g.rp[v + 1]; ++k) {
      const int c = col[g.ci[k]];
      if (c < 0) continue;
      if (c >= int(mark.size())) mark.resize(c + 1, -1);
      mark[c] = v;
    }
    int c = 0;
    while (c < int(mark.size()) && mark[c] == v) ++c;
    col[v] = c;
  }
  return col;
}

}  // namespace
}  // namespace dmg

using namespace dmg;

extern "C" {

dmg_status dmg_twolevel_create(int32_t nv, int32_t nt, const double* xy_c, const double* xy_p,
                               const int32_t* tris, const uint8_t* dof, const double* K_t,
                               dmg_hier* grid, int32_t nq, int32_t mass, int32_t flags,
                               hipStream_t stream, dmg_twolevel** out) {
  clear_error();
  if (!out) return fail(DMG_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (!xy_c || !xy_p || !tris || !dof || !grid) return fail(DMG_ERR_INVALID_ARG, "null argument");
  if (nv <= 0 || nt <= 0) return fail(DMG_ERR_INVALID_ARG, "empty mesh (nv=%d, nt=%d)", nv, nt);
  if (nq < 0 || nq > 32) return fail(DMG_ERR_INVALID_ARG, "nq must be in [0,32]");
  if (mass != 0 && mass != 2) return fail(DMG_ERR_INVALID_ARG, "mass must be 0 (lumped) or 2 (CG2)");
  for (int64_t k = 0; k < int64_t(nt) * 3; ++k)
    if (tris[k] < 0 || tris[k] >= nv)
      return fail(DMG_ERR_INVALID_ARG, "triangle vertex index %d out of range", tris[k]);
  for (int t = 0; t < nt; ++t)
    if (tri_area2(xy_p, tris + 3 * t) == 0.0)
      return fail(DMG_ERR_INVALID_ARG, "physical triangle %d is degenerate", t);
  const int nx = grid->L[0].nx, ny = grid->L[0].ny;
  Mesh m{nv, nt, xy_c, xy_p, tris, dof, {}, {}};
  build_adjacency(m);
  std::unique_ptr<dmg_twolevel> tl(new dmg_twolevel);
  tl->grid = grid;
  tl->nv = nv;
  tl->nx = nx;
  tl->ny = ny;
  tl->mass = mass;
  Csr off;
  std::vector<double> diag;
  assemble_A(m, K_t, off, diag);
  for (int v = 0; v < nv; ++v)
    if (!(diag[v] > 0.0) || !std::isfinite(diag[v]))
      return fail(DMG_ERR_INVALID_ARG, "A_p has a non-positive diagonal at vertex %d", v);
  tl->colour = greedy_colours(nv, off);
  const int ncol = 1 + *std::max_element(tl->colour.begin(), tl->colour.end());
  // internal order: colour-major, the transfers' grid-cell order within a colour (a stable
  // counting sort of the cell order by colour)
  tl->cs.assign(ncol + 1, 0);
  for (int v = 0; v < nv; ++v) tl->cs[tl->colour[v] + 1]++;
  for (int c = 0; c < ncol; ++c) tl->cs[c + 1] += tl->cs[c];
  std::vector<int> perm(nv);
  {
    const std::vector<int> cell = locality_order(m, nx, ny);
    std::vector<int> pos(tl->cs.begin(), tl->cs.end() - 1);
    for (int v : cell) perm[pos[tl->colour[v]]++] = v;
  }
  DMG_CHECK(transfer_build(m, nx, ny, nq, perm, c_form(flags), stream, tl->t));
  std::vector<int> newidx(nv);
  for (int i = 0; i < nv; ++i) newidx[perm[i]] = i;
  const Csr A = permute_rows(off, perm, &newidx);
  std::vector<double> d(nv), ml(nv, 0.0);
  for (int i = 0; i < nv; ++i) d[i] = diag[perm[i]];
  // lumped mass: the row sums of M_p, whose element entries are area/12 times 2 (diagonal) or 1
  // (a free neighbour in the triangle); 1 on the identity rows of Dirichlet vertices
  for (int v = 0; v < nv; ++v) {
    double s = 0.0;
    if (!dof[v]) {
      s = 1.0;
    } else {
      for (int k = m.vt_ptr[v]; k < m.vt_ptr[v + 1]; ++k) {
        const int* tv = tris + 3 * m.vt[k];
        const double area = 0.5 * std::fabs(tri_area2(xy_p, tv));
        for (int b = 0; b < 3; ++b)
          if (dof[tv[b]]) s += (tv[b] == v ? 2.0 : 1.0) * area / 12.0;
      }
    }
    ml[newidx[v]] = s;
  }
  tl->nnzA = int64_t(A.ci.size());
  const size_t ng = size_t(nx) * ny;
  Arena sz;
  auto layout = [&](Arena& a) {
    tl->Arp = a.take<int>(nv + 1);
    tl->Aci = a.take<int>(A.ci.size() + 1);
    tl->Av = a.take<double>(A.v.size() + 1);
    tl->Ad = a.take<double>(nv);
    tl->ML = a.take<double>(nv);
    tl->u = a.take<double>(nv);
    tl->f = a.take<double>(nv);
    tl->w = a.take<double>(nv);
    tl->ec = a.take<double>(ng);
    tl->rc = a.take<double>(ng);
    tl->partials = a.take<double>(kTBlocks);
    tl->scal = a.take<double>(16);
    tl->hist = a.take<double>(kMaxHistory);
    tl->flag = a.take<int>(4);
    tl->lz = mass == 0 ? a.take<double>(6 * ng + kLzBlocks + 4) : nullptr;
  };
  layout(sz);
  DMG_HIP(hipMalloc(&tl->block, sz.used));
  Arena a;
  a.base = static_cast<char*>(tl->block);
  a.cap = sz.used;
  layout(a);
  DMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&tl->host), 16 * sizeof(double),
                        hipHostMallocDefault));
  auto up = [&](void* dst, const void* src, size_t bytes) -> dmg_status {
    if (bytes) DMG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream));
    return DMG_OK;
  };
  DMG_CHECK(up(tl->Arp, A.rp.data(), A.rp.size() * sizeof(int)));
  DMG_CHECK(up(tl->Aci, A.ci.data(), A.ci.size() * sizeof(int)));
  DMG_CHECK(up(tl->Av, A.v.data(), A.v.size() * sizeof(double)));
  DMG_CHECK(up(tl->Ad, d.data(), size_t(nv) * sizeof(double)));
  DMG_CHECK(up(tl->ML, ml.data(), size_t(nv) * sizeof(double)));
  // the grid correction's boundary stays zero (the V-cycle writes interior points only)
  DMG_HIP(hipMemsetAsync(tl->ec, 0, ng * sizeof(double), stream));
  DMG_HIP(hipMemsetAsync(tl->rc, 0, ng * sizeof(double), stream));
  DMG_HIP(hipMemsetAsync(tl->flag, 0, 4 * sizeof(int), stream));
  DMG_HIP(hipStreamSynchronize(stream));  // host vectors go out of scope
  *out = tl.release();
  return DMG_OK;
}

dmg_status dmg_twolevel_info(const dmg_twolevel* tl, int32_t* colours, int64_t* nnz_A,
                             int32_t* colour) {
  clear_error();
  if (!tl) return fail(DMG_ERR_INVALID_ARG, "null two-level handle");
  if (colours) *colours = int32_t(tl->cs.size()) - 1;
  if (nnz_A) *nnz_A = tl->nnzA + tl->nv;
  if (colour) std::copy(tl->colour.begin(), tl->colour.end(), colour);
  return DMG_OK;
}

dmg_status dmg_twolevel_cycle(dmg_twolevel* tl, double* u_p, const double* f_p,
                              hipStream_t stream) {
  clear_error();
  if (!tl || !u_p || !f_p) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  const int n = tl->nv, nb = row_blocks(n);
  k_tl_gather<<<nb, 256, 0, stream>>>(u_p, f_p, tl->t->perm, tl->u, tl->f, n);
  DMG_CHECK(launch_check("two-level gather"));
  DMG_CHECK(cycle(tl, nullptr, stream));
  k_tl_scatter<<<nb, 256, 0, stream>>>(tl->u, tl->t->perm, u_p, n);
  return launch_check("two-level scatter");
}

dmg_status dmg_twolevel_solve(dmg_twolevel* tl, double* u_p, const double* f_p, double rtol,
                              int32_t max_iters, int32_t* iters, double* relres, double* history,
                              hipStream_t stream) {
  clear_error();
  if (!tl || !u_p || !f_p) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  if (!(rtol >= 0.0) || max_iters < 0) return fail(DMG_ERR_INVALID_ARG, "bad rtol/max_iters");
  if (iters) *iters = 0;
  const int n = tl->nv, nb = row_blocks(n);
  k_tl_gather<<<nb, 256, 0, stream>>>(u_p, f_p, tl->t->perm, tl->u, tl->f, n);
  DMG_CHECK(launch_check("two-level gather"));
  k_tl_resid<RMode::kNorm><<<nb, 256, 0, stream>>>(tl->Arp, tl->Aci, tl->Av, tl->Ad, tl->f, tl->u,
                                                   tl->ML, tl->t->dof, nullptr, n, tl->partials,
                                                   nullptr);
  DMG_CHECK(launch_check("two-level initial residual"));
  k_tl_start<<<1, 256, 0, stream>>>(tl->partials, nb, tl->scal, tl->flag, rtol, max_iters);
  DMG_CHECK(launch_check("two-level start"));
  DMG_CHECK(sweep_colour(tl, 0, tl->flag, stream));  // the first step's leading colour pass
  int* hs = reinterpret_cast<int*>(tl->host + 8);
  double* hsc = tl->host;
  // The first kChunk cycles, then a synchronisation.  From then on the rate per cycle (from r0
  // over the first chunk, then between synchronisations) predicts the cycles left: that many
  // are enqueued as back-to-back chunk graphs (up to kAhead cycles) before the next
  // synchronisation.  The device test stops at the exact cycle anyway.
  constexpr int kAhead = 4 * kChunk;
  int todo = kChunk, prev_k = -1;
  double prev_rn = 0.0;
  for (;;) {
    for (int done = 0; done < todo;) {
      const int len = std::min(kChunk, todo - done);
      DMG_CHECK(run_chunk(tl, len, stream));
      done += len;
    }
    DMG_HIP(hipMemcpyAsync(hs, tl->flag, 2 * sizeof(int), hipMemcpyDeviceToHost, stream));
    DMG_HIP(hipMemcpyAsync(hsc, tl->scal, 8 * sizeof(double), hipMemcpyDeviceToHost, stream));
    DMG_HIP(hipStreamSynchronize(stream));
    if (hs[0]) break;
    const int k_now = hs[1];
    const double rn = hsc[3], target = std::sqrt(std::max(hsc[6], 0.0));
    if (prev_k < 0) {  // first synchronisation: measure from the initial residual r0
      prev_k = 0;
      prev_rn = hsc[1];
    }
    todo = kChunk;
    if (k_now > prev_k && prev_rn > 0.0 && rn > 0.0 && target > 0.0) {
      const double rate = std::pow(rn / prev_rn, 1.0 / double(k_now - prev_k));
      if (rate > 0.0 && rate < 0.95) {
        const double left = std::ceil(std::log(target / rn) / std::log(rate) - 1e-9);
        if (left >= 1.0) todo = int(std::min(left, double(kAhead)));
      }
    }
    prev_k = k_now;
    prev_rn = rn;
  }
  k_tl_scatter<<<nb, 256, 0, stream>>>(tl->u, tl->t->perm, u_p, n);
  DMG_CHECK(launch_check("two-level scatter"));
  const int k = hs[1];
  const double r0 = hsc[1], rn = hsc[3];
  if (!std::isfinite(r0)) return fail(DMG_ERR_NONFINITE, "initial residual norm is not finite");
  if (r0 == 0.0) {  // u_0 already solves the system
    if (relres) *relres = 0.0;
    return DMG_OK;
  }
  if (history && k > 0)
    DMG_HIP(hipMemcpy(history, tl->hist, size_t(std::min(k, kMaxHistory)) * sizeof(double),
                      hipMemcpyDeviceToHost));
  if (iters) *iters = k;
  if (relres) *relres = rn / r0;
  if (!std::isfinite(rn))
    return fail(DMG_ERR_NONFINITE, "residual norm became non-finite at cycle %d", k);
  if (rn > rtol * r0)
    return fail(DMG_ERR_NO_CONVERGENCE, "no convergence in %d cycles (rel. residual %.3e)", k,
                rn / r0);
  return DMG_OK;
}

dmg_status dmg_twolevel_set_scaling(dmg_twolevel* tl, double gamma) {
  clear_error();
  if (!tl) return fail(DMG_ERR_INVALID_ARG, "null two-level handle");
  if (!std::isfinite(gamma)) return fail(DMG_ERR_INVALID_ARG, "gamma must be finite");
  tl->gamma = gamma;
  tl->reset_graph();  // captured cycles hold the previous value
  return DMG_OK;
}

dmg_status dmg_twolevel_scaling(dmg_twolevel* tl, const double* v0, int32_t k, double* gamma,
                                double* T, int32_t* steps, hipStream_t stream) {
  clear_error();
  if (!tl || !v0 || !gamma) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  if (k < 1 || k > 64) return fail(DMG_ERR_INVALID_ARG, "k must be in [1, 64]");
  if (tl->mass != 0)
    return fail(DMG_ERR_UNSUPPORTED, "the scaling estimate needs the linear (lumped) transfer");
  dmg_transfer* t = tl->t.get();
  dmg_hier* h = tl->grid;
  const int nx = tl->nx, ny = tl->ny, n = tl->nv, nb = row_blocks(n);
  const size_t ng = size_t(nx) * ny;
  // scratch kept in the handle since creation: six grid vectors, dot partials, device scalars
  double* vec[6];
  for (int q = 0; q < 6; ++q) vec[q] = tl->lz + size_t(q) * ng;
  double* partials = tl->lz + 6 * ng;
  double* dscal = partials + kLzBlocks;
  double *v = vec[0], *Av = vec[1], *vp = vec[2], *Avp = vec[3], *w = vec[4], *g = vec[5];
  const unsigned gb = unsigned(std::min<size_t>((ng + 255) / 256, 4096));
  auto dot = [&](const double* x, const double* y, double* out) -> dmg_status {
    k_lz_dot<<<kLzBlocks, 256, 0, stream>>>(x, y, ng, partials);
    DMG_CHECK(launch_check("lanczos dot"));
    DMG_CHECK(launch_finalize(partials, dscal, stream, kLzBlocks));
    DMG_HIP(hipMemcpyAsync(out, dscal, sizeof(double), hipMemcpyDeviceToHost, stream));
    DMG_HIP(hipStreamSynchronize(stream));
    return DMG_OK;
  };
  auto scale2 = [&](double* x, double* y, double f) -> dmg_status {
    k_lz_scale2<<<gb, 256, 0, stream>>>(x, y, f, ng);
    return launch_check("lanczos scale");
  };
  // G x = R A_p P x on grid vectors, R = C^T ML^{-1}
  auto applyG = [&](const double* x, double* out) -> dmg_status {
    if (t->mf) {
      DMG_CHECK(launch_from_start(t, x, nullptr, stream));
      k_tl_lumped<false><<<nb, 256, 0, stream>>>(t->r, tl->ML, t->dof, tl->w, n, 0.0, nullptr);
    } else {
      k_tl_interp<<<nb, 256, 0, stream>>>(t->Crp, t->Cci, t->Cv, x, tl->ML, t->dof, tl->w, n);
    }
    DMG_CHECK(launch_check("lanczos P"));
    k_tl_apply_scaled<<<nb, 256, 0, stream>>>(tl->Arp, tl->Aci, tl->Av, tl->Ad, tl->w, tl->ML,
                                              t->dof, t->x, n);
    DMG_CHECK(launch_check("lanczos A_p"));
    return launch_ct(t, t->x, out, nullptr, stream);
  };
  k_lz_mask<<<gb, 256, 0, stream>>>(v0, v, nx, ny);
  DMG_CHECK(launch_check("lanczos start"));
  DMG_CHECK(launch_stencil_apply(h->L[0].S, v, Av, nx, ny, stream));
  double vAv = 0.0;
  DMG_CHECK(dot(v, Av, &vAv));
  if (!(vAv > 0.0) || !std::isfinite(vAv))
    return fail(DMG_ERR_INVALID_ARG, "start vector has no interior part");
  DMG_CHECK(scale2(v, Av, 1.0 / std::sqrt(vAv)));
  DMG_CHECK(launch_fill<double>(vp, 0.0, ng, stream));
  DMG_CHECK(launch_fill<double>(Avp, 0.0, ng, stream));
  std::vector<double> alphas, betas;
  double beta = 0.0;
  for (int j = 0; j < k; ++j) {
    DMG_CHECK(applyG(v, g));
    double alpha = 0.0;
    DMG_CHECK(dot(g, v, &alpha));
    alphas.push_back(alpha);
    if (j + 1 == k) break;
    // w = A_c^{-1} g by the grid solve, to a relative residual of 1e-13 or its stagnation
    DMG_CHECK(launch_fill<double>(w, 0.0, ng, stream));
    int32_t it = 0;
    double rr = 0.0;
    const dmg_status st = dmg_solve(h, w, g, 1e-13, 100, &it, &rr, nullptr, stream);
    if (st != DMG_OK && !(st == DMG_ERR_NO_CONVERGENCE && rr <= 1e-11)) return st;
    clear_error();
    k_lz_update<<<gb, 256, 0, stream>>>(w, v, vp, g, Av, Avp, alpha, beta, ng);
    DMG_CHECK(launch_check("lanczos update"));
    double wAw = 0.0;
    DMG_CHECK(dot(w, g, &wAw));
    const double bnew = std::sqrt(std::max(wAw, 0.0));
    if (!(bnew > 1e-13 * std::fabs(alpha))) break;  // invariant Krylov space
    betas.push_back(bnew);
    // (vp, v, w) <- (v, w / beta, vp) and the same for the A_c images
    std::swap(vp, v);
    std::swap(v, w);
    std::swap(Avp, Av);
    std::swap(Av, g);
    DMG_CHECK(scale2(v, Av, 1.0 / bnew));
    beta = bnew;
  }
  const int m = int(alphas.size());
  double sum = 0.0;
  for (double x : alphas) sum += x;
  *gamma = sum / m;
  if (steps) *steps = m;
  if (T) {
    std::fill(T, T + size_t(k) * k, 0.0);
    for (int i = 0; i < m; ++i) {
      T[size_t(i) * k + i] = alphas[i];
      if (i + 1 < m) T[size_t(i) * k + i + 1] = T[size_t(i + 1) * k + i] = betas[i];
    }
  }
  return DMG_OK;
}

void dmg_twolevel_destroy(dmg_twolevel* tl) { delete tl; }

}  // extern "C"
