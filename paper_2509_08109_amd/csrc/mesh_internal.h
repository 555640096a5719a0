// Internal interface of the mesh side: the device state of the grid <-> mesh transfers and the
// host and device pieces that the transfers and the two-level cycle share.
#pragma once

#include <algorithm>
#include <memory>
#include <thread>
#include <vector>

#include "dmg_internal.h"

struct dmg_transfer {
  int nv = 0, nx = 0, ny = 0;
  int64_t nnzC = 0, nnzM = 0;
  int *Crp = nullptr, *Cci = nullptr, *CTrp = nullptr, *CTci = nullptr, *Mrp = nullptr,
      *Mci = nullptr;
  double *Cv = nullptr, *CTv = nullptr, *Mv = nullptr;
  unsigned char* dof = nullptr;  // internal order
  int* perm = nullptr;           // internal row i holds the caller's vertex perm[i]
  double *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr;
  double *partials = nullptr, *scal = nullptr;
  void* block = nullptr;   // M_p, vectors, scalars
  void* cblock = nullptr;  // C and C^T
  bool device_C = false;   // C was assembled on the device
  bool borrowed = false;   // C and M_p are the caller's device CSR arrays (created from CSR)
  // matrix-free C (DMG_MESH_MATRIX_FREE): the overlap sets in mfblock, no stored C or C^T
  bool mf = false;
  int nt = 0, nq = 0;
  double* mf_xy = nullptr;      // [nv][2] vertex images T(x_v), internal order
  double* mf_jac = nullptr;     // [nt] Jacobian factor area(tau_p) / area(mapped tau), 0: skipped
  double* mf_q = nullptr;       // Gauss nodes [nq] then weights [nq] on [0, 1]
  double* mf_buf = nullptr;     // [max(3 nt, 4 cells)]: per-triangle or per-cell partial sums
  int* mf_tv = nullptr;         // [nt][3] internal vertex indices
  int* mf_vt_ptr = nullptr;     // [nv + 1]: mesh row -> entries 3 t + slot, ascending t
  int* mf_vt = nullptr;
  int* mf_ct_ptr = nullptr;     // [(nx - 1)(ny - 1) + 1]: cell -> triangles whose box holds it
  int* mf_ct = nullptr;         // ascending t
  int64_t mf_pairs = 0;         // triangle-cell pairs of the boxes
  size_t mf_bytes = 0;          // device bytes of mfblock
  void* mfblock = nullptr;
  ~dmg_transfer() {
    if (block) (void)hipFree(block);
    if (cblock) (void)hipFree(cblock);
    if (mfblock) (void)hipFree(mfblock);
  }
};

namespace dmg {

struct Csr {
  std::vector<int> rp, ci;
  std::vector<double> v;
};

// Concatenation of per-thread row blocks (rows [first_row[t], ...) of parts[t]) into one CSR.
inline Csr merge_rows(int n, const std::vector<Csr>& parts, const std::vector<int>& first_row) {
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

// Rows [0, n) of a CSR built in contiguous blocks on up to 16 host threads (one thread below
// 4096 rows): build(r0, r1, out) appends rows r0..r1-1 to out, whose rp starts as {0}.  Each row
// is built by one thread in a fixed order, so the result does not depend on the thread count.
template <class Build>
Csr rows_parallel(int n, Build&& build) {
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 4096) nth = 1;
  std::vector<Csr> parts(nth);
  std::vector<int> first(nth);
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nth; ++t) {
    const int r0 = int(int64_t(n) * t / nth), r1 = int(int64_t(n) * (t + 1) / nth);
    first[t] = r0;
    th.emplace_back([&, t, r0, r1]() {
      parts[t].rp.assign(1, 0);
      build(r0, r1, parts[t]);
    });
  }
  for (auto& x : th) x.join();
  return merge_rows(n, parts, first);
}

// Host view of a caller's mesh (vertex arrays in the caller's order).
struct Mesh {
  int nv, nt;
  const double *xy_c, *xy_p;
  const int* tris;
  const uint8_t* dof;
  std::vector<int> vt_ptr, vt;  // vertex -> incident triangles, in triangle order
};

void build_adjacency(Mesh& m);
// Twice the signed area of triangle tv with vertex coordinates xy.
__host__ __device__ inline double tri_area2(const double* xy, const int* tv) {
#pragma clang fp contract(off)
  const double* a = xy + 2 * tv[0];
  const double* b = xy + 2 * tv[1];
  const double* c = xy + 2 * tv[2];
  return (b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1]);
}
// Gauss-Legendre nodes and weights on [0, 1].
void gauss_rule01(int nq, std::vector<double>& x, std::vector<double>& w);
// Vertices ordered by the grid cell that holds their computational image (row-major).
std::vector<int> locality_order(const Mesh& m, int nx, int ny);
// Rows of a in the order perm (new row i = old row perm[i]); columns through colmap when given.
Csr permute_rows(const Csr& a, const std::vector<int>& perm, const std::vector<int>* colmap);

// How a transfer holds C: assembled on the device (the host assembly takes over when a row is
// too long for the device merge), assembled on the host, or matrix-free over the overlap sets.
enum class CForm { kDevice, kHost, kMatrixFree };
inline CForm c_form(int flags) {
  return (flags & DMG_MESH_MATRIX_FREE) ? CForm::kMatrixFree
         : (flags & DMG_MESH_HOST_SETUP) ? CForm::kHost : CForm::kDevice;
}

// Transfer operators of mesh m on the nx x ny grid with internal row i = caller vertex perm[i].
dmg_status transfer_build(const Mesh& m, int nx, int ny, int nq, const std::vector<int>& perm,
                          CForm form, hipStream_t s, std::unique_ptr<dmg_transfer>& out);

// ---- the coupled-mass integrals of one mapped triangle over one grid cell -------------------
// Shared by the host and the device assembly, with contraction off, so both give the same bits.
// Dunavant's symmetric 6-point rule on a triangle, exact for degree 4: barycentric orbits
// (a, a, 1 - 2a) with weights relative to the area.
constexpr double kTriA1 = 0.445948490915965, kTriW1 = 0.223381589678011;
constexpr double kTriA2 = 0.091576213509771, kTriW2 = 1.0 / 3.0 - kTriW1;

// Part of triangle tri inside the box [x0, x1] x [y0, y1] (Sutherland-Hodgman, one pass per box
// side); returns its vertex count (a triangle cut by four half-planes keeps at most 7).
__host__ __device__ inline int clip_triangle(const double tri[3][2], double x0, double x1,
                                             double y0, double y1, double out[8][2]) {
#pragma clang fp contract(off)
  double a[8][2], b[8][2];
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
  int n = pass(a, 3, b, 0, x0, 1.0);
  n = n ? pass(b, n, a, 0, x1, -1.0) : 0;
  n = n ? pass(a, n, b, 1, y0, 1.0) : 0;
  n = n ? pass(b, n, a, 1, y1, -1.0) : 0;
  for (int k = 0; k < n; ++k) {
    out[k][0] = a[k][0];
    out[k][1] = a[k][1];
  }
  return n;
}

// w[a][g] = integral over grid cell (ci, cj) of lambda_a * phi_g for the mapped triangle tri
// (computational coordinates, det = twice its signed area), without the Jacobian factor; g runs
// over the corners (ci, cj), (ci + 1, cj), (ci, cj + 1), (ci + 1, cj + 1).  nq == 0: exact, over
// the triangle-cell overlap polygon (fan triangles, Dunavant's rule; the integrand is a cubic);
// nq > 0: the nq x nq Gauss rule (nodes qx, weights qw on [0, 1]) on the cell, points outside
// the triangle counting as zero.
__host__ __device__ inline void cell_integrals(const double tri[3][2], double det, int ci, int cj,
                                               double hx, double hy, int nq, const double* qx,
                                               const double* qw, double w[3][4]) {
#pragma clang fp contract(off)
  for (int a = 0; a < 3; ++a)
    for (int g = 0; g < 4; ++g) w[a][g] = 0.0;
  const double X0 = -1.0 + ci * hx, Y0 = -1.0 + cj * hy;
  // lambda_a(X, Y) = (e0 + e1 X + e2 Y) / det from the edge opposite vertex a
  double e[3][3];
  for (int a = 0; a < 3; ++a) {
    const double* p = tri[(a + 1) % 3];
    const double* q = tri[(a + 2) % 3];
    e[a][0] = p[0] * q[1] - q[0] * p[1];
    e[a][1] = p[1] - q[1];
    e[a][2] = q[0] - p[0];
  }
  auto accumulate = [&](double wt, double X, double Y, bool inside_only) {
    double lam[3];
    for (int a = 0; a < 3; ++a) lam[a] = (e[a][0] + e[a][1] * X + e[a][2] * Y) / det;
    if (inside_only && (lam[0] < 0.0 || lam[1] < 0.0 || lam[2] < 0.0)) return;
    const double s = (X - X0) / hx, t = (Y - Y0) / hy;
    const double ph[4] = {(1 - s) * (1 - t), s * (1 - t), (1 - s) * t, s * t};
    for (int a = 0; a < 3; ++a) {
      const double wa = wt * lam[a];
      for (int g = 0; g < 4; ++g) w[a][g] += wa * ph[g];
    }
  };
  if (nq > 0) {
    for (int sy = 0; sy < nq; ++sy)
      for (int sx = 0; sx < nq; ++sx)
        accumulate(qw[sx] * qw[sy] * hx * hy, X0 + qx[sx] * hx, Y0 + qx[sy] * hy, true);
    return;
  }
  double poly[8][2];
  const int np = clip_triangle(tri, X0, X0 + hx, Y0, Y0 + hy, poly);
  const double orbit[2][2] = {{kTriA1, kTriW1}, {kTriA2, kTriW2}};
  for (int k = 1; k + 1 < np; ++k) {
    const double* A = poly[0];
    const double* B = poly[k];
    const double* D = poly[k + 1];
    const double area2 = (B[0] - A[0]) * (D[1] - A[1]) - (D[0] - A[0]) * (B[1] - A[1]);
    const double area = 0.5 * (area2 < 0.0 ? -area2 : area2);
    if (area == 0.0) continue;
    for (int o = 0; o < 2; ++o) {
      const double la = orbit[o][0], lb = 1.0 - 2.0 * orbit[o][0];
      const double bary[3][3] = {{la, la, lb}, {la, lb, la}, {lb, la, la}};
      for (int q = 0; q < 3; ++q) {
        const double X = bary[q][0] * A[0] + bary[q][1] * B[0] + bary[q][2] * D[0];
        const double Y = bary[q][0] * A[1] + bary[q][1] * B[1] + bary[q][2] * D[1];
        accumulate(orbit[o][1] * area, X, Y, false);
      }
    }
  }
}

// Grid cell of coordinate x (cell width h, n grid points), clamped to [0, n - 2].
__host__ __device__ inline int grid_cell(double x, double h, int n) {
  const int c = int(floor((x + 1.0) / h));
  return c < 0 ? 0 : (c > n - 2 ? n - 2 : c);
}

// Device assembly of C (rows in the internal order perm) and C^T into one owned device block.
struct DeviceCsrPair {
  void* block = nullptr;
  int *rp = nullptr, *ci = nullptr, *trp = nullptr, *tci = nullptr;
  double *v = nullptr, *tv = nullptr;
  int64_t nnz = 0;
};
// Returns DMG_ERR_UNSUPPORTED (nothing kept) when a row has more distinct grid columns than the
// device merge holds; the caller then assembles on the host.
dmg_status device_assemble_C(const Mesh& m, int nx, int ny, int nq,
                             const std::vector<int>& perm, hipStream_t s, DeviceCsrPair& out);

// C^T of a device CSR (nr rows, nc columns, nnz entries) into caller buffers trp [nc + 1], tci and
// tv [nnz], each transposed row in ascending source-row order (deterministic).  Scratch: cnt
// [nc + 1], pos [nc], sums [transpose_sums(nc)] ints.  Asynchronous on s.
int transpose_sums(int nc);
dmg_status device_transpose(const int* rp, const int* ci, const double* v, int nr, int nc,
                            int* trp, int* tci, double* tv, int* cnt, int* pos, int* sums,
                            hipStream_t s);
// Structure check of a device CSR with nr rows, nc columns and nnz entries: rp[0] = 0, rp
// non-decreasing and at most nnz (checked first, reading rp only), then every column in [0, nc).
// *ok receives the result of the check; flag is one device int of scratch.  Synchronises s.
dmg_status device_check_csr(const int* rp, const int* ci, int nr, int nc, int nnz, int* flag,
                            bool* ok, hipStream_t s);

// Matrix-free C over the overlap sets W_i (transfer_mf.hip): builds t's lists from the mesh
// (internal vertex order perm); the apply kernels replace the CSR products of C and C^T.
dmg_status mf_build(const Mesh& m, int nx, int ny, int nq, const std::vector<int>& perm,
                    hipStream_t s, dmg_transfer* t);
// t->r = dof * (C u_c) and its squared-norm partials (tblocks(nv, kMG) of them)
dmg_status mf_launch_from(dmg_transfer* t, const double* u_c, const int* stop, hipStream_t s);
// r_c = C^T x (x in the internal order)
dmg_status mf_launch_ct(dmg_transfer* t, const double* x, double* r_c, const int* stop,
                        hipStream_t s);

// Row products run on groups of G consecutive lanes (G divides 64): lane l of a group reads
// entries rp[r] + l, rp[r] + l + G, ... (coalesced), and the group sums its lanes with xor
// shuffles in a fixed order.  Kernels walk row groups grid-stride; kernels that reduce write one
// partial per workgroup.
constexpr int kTBlocks = 4096;  // workgroup cap of the mesh kernels (= partials capacity)
constexpr int kMG = 4;  // lanes per mesh row (rows of C, M_p and A_p hold ~7-9 entries)
constexpr int kCG = 8;  // lanes per grid row of C^T (~30 entries)

inline int tblocks(int n, int lanes) {
  const long b = (long(n) * lanes + 255) / 256;
  return b < 1 ? 1 : (b > kTBlocks ? kTBlocks : int(b));
}

template <int G, class X>
__device__ __forceinline__ double row_dot(const int* __restrict__ rp, const int* __restrict__ ci,
                                          const double* __restrict__ v, int r, int lane, X&& x) {
  const int e = rp[r + 1];
  double acc = 0.0;
  for (int k = rp[r] + lane; k < e; k += G) acc = __builtin_fma(v[k], x(ci[k]), acc);
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
  return acc;
}

// Sum over a 256-thread workgroup; the total is returned to thread 0.
__device__ __forceinline__ double mesh_block_sum(double v) {
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

// Where CG2's result x2 goes: the internal order (store), the caller's order (scatter), or added
// into an internal-order vector (add).
enum class X2Mode { kStore, kScatter, kAdd };

// stop (nullable device flag): every kernel below is a no-op once it is set.
// t->r = dof * (C u_c) and its squared-norm partials: the start of from_grid.
dmg_status launch_from_start(dmg_transfer* t, const double* u_c, const int* stop, hipStream_t s);
// Two CG iterations on M_p from x = 0, continuing from r0 in t->r with its partials; the add
// mode adds scale * x2.
dmg_status cg2_tail(dmg_transfer* t, double* out, X2Mode mode, const int* stop, hipStream_t s,
                    double scale = 1.0);
// r_c = C^T x over the grid rows (x in the internal order).
dmg_status launch_ct(dmg_transfer* t, const double* x, double* r_c, const int* stop, hipStream_t s);

}  // namespace dmg
