// Internal interface of the mesh side: the device state of the grid <-> mesh transfers and the
// host and device pieces that the transfers and the two-level cycle share.
#pragma once

#include <memory>
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
  void* block = nullptr;
  ~dmg_transfer() {
    if (block) (void)hipFree(block);
  }
};

namespace dmg {

struct Csr {
  std::vector<int> rp, ci;
  std::vector<double> v;
};

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
double tri_area2(const double* xy, const int* tv);
// Vertices ordered by the grid cell that holds their computational image (row-major).
std::vector<int> locality_order(const Mesh& m, int nx, int ny);
// Rows of a in the order perm (new row i = old row perm[i]); columns through colmap when given.
Csr permute_rows(const Csr& a, const std::vector<int>& perm, const std::vector<int>* colmap);

// Transfer operators of mesh m on the nx x ny grid with internal row i = caller vertex perm[i].
dmg_status transfer_build(const Mesh& m, int nx, int ny, int nq, const std::vector<int>& perm,
                          hipStream_t s, std::unique_ptr<dmg_transfer>& out);

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
