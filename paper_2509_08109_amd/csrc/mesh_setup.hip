// Device assembly of the coupled mass C (Sec. 2.3.1) and its transpose, the setup work the paper
// names as its bottleneck.  The result equals the host assembly bit for bit: both evaluate the
// same per-cell integrals (cell_integrals, contraction off) and sum each entry in the same order
// (incident triangles in index order, their cells row by row).
//
//   1. per triangle: the cells of its bounding box; per vertex: its incident triangles (counts,
//      prefix sums, filled lists sorted into triangle order);
//   2. per triangle: the integrals of its three basis functions over each of its cells, once
//      (the host assembly visits each triangle from each of its three vertices);
//   3. per mesh row (internal order): the contributions of its incident triangles merged into a
//      short sorted list of grid columns -- counted, prefix-summed, then written;
//   4. C^T: entries counted per grid column, scattered, and each row sorted by mesh row.
// Scratch is allocated for the call and freed before it returns.
#include "mesh_internal.h"

namespace dmg {
namespace {

constexpr int kRowCap = 64;  // distinct grid columns one row merge holds (rows hold ~10-20)

unsigned grid_for(size_t n) { return unsigned(std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 16384))); }

// ---- exclusive prefix sums of int arrays (three passes, 1024 items per workgroup) ------------
__global__ __launch_bounds__(256) void k_scan_local(const int* __restrict__ in,
                                                    int* __restrict__ out, int n,
                                                    int* __restrict__ sums) {
  __shared__ int ws[256];
  const int base = int(blockIdx.x) * 1024 + int(threadIdx.x) * 4;
  int v[4], tsum = 0;
  for (int q = 0; q < 4; ++q) {
    v[q] = base + q < n ? in[base + q] : 0;
    tsum += v[q];
  }
  ws[threadIdx.x] = tsum;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int x = int(threadIdx.x) >= off ? ws[threadIdx.x - off] : 0;
    __syncthreads();
    ws[threadIdx.x] += x;
    __syncthreads();
  }
  int run = ws[threadIdx.x] - tsum;
  for (int q = 0; q < 4; ++q) {
    if (base + q < n) out[base + q] = run;
    run += v[q];
  }
  if (threadIdx.x == 255) sums[blockIdx.x] = ws[255];
}

// In-place exclusive scan of the nb workgroup sums by one workgroup.
__global__ __launch_bounds__(256) void k_scan_sums(int* __restrict__ sums, int nb) {
  __shared__ int ws[256];
  int carry = 0;
  for (int c0 = 0; c0 < nb; c0 += 256) {
    const int i = c0 + int(threadIdx.x);
    const int x = i < nb ? sums[i] : 0;
    ws[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int y = int(threadIdx.x) >= off ? ws[threadIdx.x - off] : 0;
      __syncthreads();
      ws[threadIdx.x] += y;
      __syncthreads();
    }
    if (i < nb) sums[i] = carry + ws[threadIdx.x] - x;
    carry += ws[255];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_scan_add(int* __restrict__ out, int n,
                                                  const int* __restrict__ sums) {
  for (int i = int(blockIdx.x) * 256 + int(threadIdx.x); i < n; i += int(gridDim.x) * 256)
    out[i] += sums[i / 1024];
}

__global__ __launch_bounds__(256) void k_fill_int(int* __restrict__ x, int v, size_t n) {
  for (size_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += size_t(gridDim.x) * 256u) x[i] = v;
}

// ---- step 1: cells per triangle, incident triangles per vertex ----------------------------
struct CellBox {
  int i0, i1, j0, j1;
};

__device__ __forceinline__ CellBox cell_box(const double tri[3][2], double hx, double hy, int nx,
                                            int ny) {
  CellBox b;
  b.i0 = grid_cell(fmin(fmin(tri[0][0], tri[1][0]), tri[2][0]), hx, nx);
  b.i1 = grid_cell(fmax(fmax(tri[0][0], tri[1][0]), tri[2][0]), hx, nx);
  b.j0 = grid_cell(fmin(fmin(tri[0][1], tri[1][1]), tri[2][1]), hy, ny);
  b.j1 = grid_cell(fmax(fmax(tri[0][1], tri[1][1]), tri[2][1]), hy, ny);
  return b;
}

__device__ __forceinline__ void load_tri(const double* __restrict__ xy, const int* tv,
                                         double tri[3][2]) {
  for (int q = 0; q < 3; ++q) {
    tri[q][0] = xy[2 * tv[q]];
    tri[q][1] = xy[2 * tv[q] + 1];
  }
}

__global__ __launch_bounds__(256) void k_cs_cells(const int* __restrict__ tris,
                                                  const double* __restrict__ xyc, int nt, int nx,
                                                  int ny, double hx, double hy,
                                                  int* __restrict__ ncell,
                                                  int* __restrict__ deg) {
  for (int t = int(blockIdx.x) * 256 + int(threadIdx.x); t < nt; t += int(gridDim.x) * 256) {
    const int* tv = tris + 3 * size_t(t);
    double tri[3][2];
    load_tri(xyc, tv, tri);
    const CellBox b = cell_box(tri, hx, hy, nx, ny);
    ncell[t] = (b.i1 - b.i0 + 1) * (b.j1 - b.j0 + 1);
    for (int a = 0; a < 3; ++a) atomicAdd(&deg[tv[a]], 1);
  }
}

__global__ __launch_bounds__(256) void k_cs_fill_vt(const int* __restrict__ tris, int nt,
                                                    const int* __restrict__ vt_ptr,
                                                    int* __restrict__ pos, int* __restrict__ vt) {
  for (int t = int(blockIdx.x) * 256 + int(threadIdx.x); t < nt; t += int(gridDim.x) * 256)
    for (int a = 0; a < 3; ++a) {
      const int v = tris[3 * size_t(t) + a];
      vt[vt_ptr[v] + atomicAdd(&pos[v], 1)] = t;
    }
}

// incident-triangle lists into triangle order (insertion sort; a vertex has a handful)
__global__ __launch_bounds__(256) void k_cs_sort_vt(const int* __restrict__ vt_ptr,
                                                    int* __restrict__ vt, int nv) {
  for (int v = int(blockIdx.x) * 256 + int(threadIdx.x); v < nv; v += int(gridDim.x) * 256) {
    const int b = vt_ptr[v], e = vt_ptr[v + 1];
    for (int i = b + 1; i < e; ++i) {
      const int x = vt[i];
      int j = i - 1;
      while (j >= b && vt[j] > x) {
        vt[j + 1] = vt[j];
        --j;
      }
      vt[j + 1] = x;
    }
  }
}

// ---- step 2: per-triangle cell integrals, times the Jacobian factor -----------------------
// rec[(coff[t] + c) * 12 + a * 4 + g] for cell c of t's box (row by row), vertex slot a, corner g
__global__ __launch_bounds__(256) void k_cs_integrate(const int* __restrict__ tris,
                                                      const double* __restrict__ xyc,
                                                      const double* __restrict__ xyp, int nt,
                                                      int nx, int ny, double hx, double hy,
                                                      int nq, const double* __restrict__ qx,
                                                      const double* __restrict__ qw,
                                                      const int* __restrict__ coff,
                                                      double* __restrict__ rec) {
  for (int t = int(blockIdx.x) * 256 + int(threadIdx.x); t < nt; t += int(gridDim.x) * 256) {
    const int* tv = tris + 3 * size_t(t);
    double tri[3][2];
    load_tri(xyc, tv, tri);
    const CellBox b = cell_box(tri, hx, hy, nx, ny);
    const double det = tri_area2(xyc, tv);
    const double jac = det == 0.0 ? 0.0 : fabs(tri_area2(xyp, tv)) / fabs(det);
    size_t c = size_t(coff[t]);
    for (int cj = b.j0; cj <= b.j1; ++cj)
      for (int ci = b.i0; ci <= b.i1; ++ci, ++c) {
        double* r = rec + 12 * c;
        if (det == 0.0) {
          for (int k = 0; k < 12; ++k) r[k] = 0.0;
          continue;
        }
        double w[3][4];
        cell_integrals(tri, det, ci, cj, hx, hy, nq, qx, qw, w);
        for (int a = 0; a < 3; ++a)
          for (int g = 0; g < 4; ++g) r[4 * a + g] = jac * w[a][g];
      }
  }
}

// ---- step 3: rows of C in the internal order ----------------------------------------------
// COUNT: cnt[i] = nonzero entries of row i; otherwise rows are written at rp[i].
template <bool COUNT>
__global__ __launch_bounds__(256) void k_cs_rows(const int* __restrict__ perm,
                                                 const unsigned char* __restrict__ dof,
                                                 const int* __restrict__ vt_ptr,
                                                 const int* __restrict__ vt,
                                                 const int* __restrict__ tris,
                                                 const double* __restrict__ xyc, int nv, int nx,
                                                 int ny, double hx, double hy,
                                                 const int* __restrict__ coff,
                                                 const double* __restrict__ rec,
                                                 int* __restrict__ cnt,
                                                 const int* __restrict__ rp,
                                                 int* __restrict__ ci_out,
                                                 double* __restrict__ v_out,
                                                 int* __restrict__ overflow) {
  for (int i = int(blockIdx.x) * 256 + int(threadIdx.x); i < nv; i += int(gridDim.x) * 256) {
    const int v = perm[i];
    int cols[kRowCap];
    double vals[kRowCap];
    int n = 0;
    bool ovf = false;
    if (dof[v]) {
      for (int k = vt_ptr[v]; k < vt_ptr[v + 1] && !ovf; ++k) {
        const int t = vt[k];
        const int* tv = tris + 3 * size_t(t);
        if (tri_area2(xyc, tv) == 0.0) continue;
        const int a = tv[0] == v ? 0 : (tv[1] == v ? 1 : 2);
        double tri[3][2];
        load_tri(xyc, tv, tri);
        const CellBox b = cell_box(tri, hx, hy, nx, ny);
        size_t c = size_t(coff[t]);
        for (int cj = b.j0; cj <= b.j1 && !ovf; ++cj)
          for (int cc = b.i0; cc <= b.i1 && !ovf; ++cc, ++c) {
            const int g00 = cj * nx + cc;
            const int gi[4] = {g00, g00 + 1, g00 + nx, g00 + nx + 1};
            for (int g = 0; g < 4; ++g) {
              const int gx = gi[g] % nx, gy = gi[g] / nx;
              if (gx == 0 || gx == nx - 1 || gy == 0 || gy == ny - 1) continue;
              const double val = rec[12 * c + 4 * a + g];
              int p = 0;
              while (p < n && cols[p] < gi[g]) ++p;
              if (p < n && cols[p] == gi[g]) {
                vals[p] += val;
              } else if (n == kRowCap) {
                ovf = true;
                break;
              } else {
                for (int q = n; q > p; --q) {
                  cols[q] = cols[q - 1];
                  vals[q] = vals[q - 1];
                }
                cols[p] = gi[g];
                vals[p] = 0.0 + val;
                ++n;
              }
            }
          }
      }
    }
    if (ovf) {
      *overflow = 1;
      if (COUNT) cnt[i] = 0;
      continue;
    }
    if (COUNT) {
      int nz = 0;
      for (int p = 0; p < n; ++p) nz += vals[p] != 0.0;
      cnt[i] = nz;
    } else {
      int o = rp[i];
      for (int p = 0; p < n; ++p)
        if (vals[p] != 0.0) {
          ci_out[o] = cols[p];
          v_out[o] = vals[p];
          ++o;
        }
    }
  }
}

// ---- step 4: C^T ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cs_colcount(const int* __restrict__ rp,
                                                     const int* __restrict__ ci, int nv,
                                                     int* __restrict__ ccount) {
  for (int i = int(blockIdx.x) * 256 + int(threadIdx.x); i < nv; i += int(gridDim.x) * 256)
    for (int k = rp[i]; k < rp[i + 1]; ++k) atomicAdd(&ccount[ci[k]], 1);
}

__global__ __launch_bounds__(256) void k_cs_tfill(const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const double* __restrict__ v, int nv,
                                                  const int* __restrict__ trp,
                                                  int* __restrict__ tpos, int* __restrict__ tci,
                                                  double* __restrict__ tv) {
  for (int i = int(blockIdx.x) * 256 + int(threadIdx.x); i < nv; i += int(gridDim.x) * 256)
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const int c = ci[k];
      const int p = trp[c] + atomicAdd(&tpos[c], 1);
      tci[p] = i;
      tv[p] = v[k];
    }
}

__global__ __launch_bounds__(256) void k_cs_tsort(const int* __restrict__ trp,
                                                  int* __restrict__ tci, double* __restrict__ tv,
                                                  int ng) {
  for (int r = int(blockIdx.x) * 256 + int(threadIdx.x); r < ng; r += int(gridDim.x) * 256) {
    const int b = trp[r], e = trp[r + 1];
    for (int i = b + 1; i < e; ++i) {
      const int x = tci[i];
      const double y = tv[i];
      int j = i - 1;
      while (j >= b && tci[j] > x) {
        tci[j + 1] = tci[j];
        tv[j + 1] = tv[j];
        --j;
      }
      tci[j + 1] = x;
      tv[j + 1] = y;
    }
  }
}

// RAII for the call's scratch allocations
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

// out[0..n) = exclusive prefix sums of in[0..n) (in and out distinct); sums: >= ceil(n/1024)
dmg_status scan(const int* in, int* out, int n, int* sums, hipStream_t s) {
  const int nb = (n + 1023) / 1024;
  k_scan_local<<<nb, 256, 0, s>>>(in, out, n, sums);
  DMG_CHECK(launch_check("scan local"));
  k_scan_sums<<<1, 256, 0, s>>>(sums, nb);
  DMG_CHECK(launch_check("scan sums"));
  k_scan_add<<<grid_for(size_t(n)), 256, 0, s>>>(out, n, sums);
  return launch_check("scan add");
}

// Row pointers only: rp[0] = 0 and 0 <= rp[i] <= rp[i + 1] <= nnz.
__global__ __launch_bounds__(256) void k_check_rowptr(const int* __restrict__ rp, int nr, int nnz,
                                                      int* __restrict__ flag) {
  for (int i = int(blockIdx.x) * 256 + int(threadIdx.x); i < nr; i += int(gridDim.x) * 256) {
    const int b = rp[i], e = rp[i + 1];
    if ((i == 0 && b != 0) || b < 0 || e < b || e > nnz) atomicOr(flag, 1);
  }
}

// Column indices of rows whose pointers were checked: every column in [0, nc).
__global__ __launch_bounds__(256) void k_check_cols(const int* __restrict__ rp,
                                                    const int* __restrict__ ci, int nr, int nc,
                                                    int* __restrict__ flag) {
  for (int i = int(blockIdx.x) * 256 + int(threadIdx.x); i < nr; i += int(gridDim.x) * 256) {
    bool bad = false;
    for (int k = rp[i]; k < rp[i + 1] && !bad; ++k) bad = ci[k] < 0 || ci[k] >= nc;
    if (bad) atomicOr(flag, 1);
  }
}

}  // namespace

int transpose_sums(int nc) { return (nc + 1 + 1023) / 1024 + 2; }

dmg_status device_transpose(const int* rp, const int* ci, const double* v, int nr, int nc,
                            int* trp, int* tci, double* tv, int* cnt, int* pos, int* sums,
                            hipStream_t s) {
  k_fill_int<<<grid_for(size_t(nc) + 1), 256, 0, s>>>(cnt, 0, size_t(nc) + 1);
  DMG_CHECK(launch_check("fill"));
  k_cs_colcount<<<grid_for(size_t(nr)), 256, 0, s>>>(rp, ci, nr, cnt);
  DMG_CHECK(launch_check("column counts"));
  DMG_CHECK(scan(cnt, trp, nc + 1, sums, s));
  k_fill_int<<<grid_for(size_t(nc)), 256, 0, s>>>(pos, 0, size_t(nc));
  DMG_CHECK(launch_check("fill"));
  k_cs_tfill<<<grid_for(size_t(nr)), 256, 0, s>>>(rp, ci, v, nr, trp, pos, tci, tv);
  DMG_CHECK(launch_check("transpose"));
  k_cs_tsort<<<grid_for(size_t(nc)), 256, 0, s>>>(trp, tci, tv, nc);
  return launch_check("transpose order");
}

dmg_status device_check_csr(const int* rp, const int* ci, int nr, int nc, int nnz, int* flag,
                            bool* ok, hipStream_t s) {
  int bad = 0;
  k_fill_int<<<1, 256, 0, s>>>(flag, 0, 1);
  DMG_CHECK(launch_check("fill"));
  k_check_rowptr<<<grid_for(size_t(nr)), 256, 0, s>>>(rp, nr, nnz, flag);
  DMG_CHECK(launch_check("row pointer check"));
  DMG_HIP(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  DMG_HIP(hipStreamSynchronize(s));
  if (!bad) {  // the pointers bound every column read below
    k_check_cols<<<grid_for(size_t(nr)), 256, 0, s>>>(rp, ci, nr, nc, flag);
    DMG_CHECK(launch_check("column check"));
    DMG_HIP(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    DMG_HIP(hipStreamSynchronize(s));
  }
  *ok = !bad;
  return DMG_OK;
}

dmg_status device_assemble_C(const Mesh& m, int nx, int ny, int nq,
                             const std::vector<int>& perm, hipStream_t s, DeviceCsrPair& out) {
  const int nv = m.nv, nt = m.nt;
  const size_t ng = size_t(nx) * ny;
  if (size_t(nt) * 3 >= (size_t(1) << 31) || ng + 1 >= (size_t(1) << 31))
    return fail(DMG_ERR_UNSUPPORTED, "mesh too large for the device assembly");
  const double hx = 2.0 / (nx - 1), hy = 2.0 / (ny - 1);
  std::vector<double> qx(1, 0.0), qw(1, 0.0);
  if (nq > 0) gauss_rule01(nq, qx, qw);
  const int nscan = int(std::max<size_t>({size_t(nt), size_t(nv), ng}) + 1);
  // inputs and integer scratch in one block
  Arena sz;
  double *xyc, *xyp, *dqx, *dqw;
  int *tris, *dperm, *ncell, *coff, *deg, *vt_ptr, *pos, *vt, *cnt, *rp_tmp, *sums, *flag;
  unsigned char* dof;
  auto layout = [&](Arena& a) {
    xyc = a.take<double>(2 * size_t(nv));
    xyp = a.take<double>(2 * size_t(nv));
    dqx = a.take<double>(qx.size());
    dqw = a.take<double>(qw.size());
    tris = a.take<int>(3 * size_t(nt));
    dperm = a.take<int>(nv);
    dof = a.take<unsigned char>(nv);
    ncell = a.take<int>(size_t(nt) + 1);
    coff = a.take<int>(size_t(nt) + 1);
    deg = a.take<int>(size_t(nv) + 1);
    vt_ptr = a.take<int>(size_t(nv) + 1);
    pos = a.take<int>(nv);
    vt = a.take<int>(3 * size_t(nt));
    cnt = a.take<int>(size_t(nv) + 1);
    rp_tmp = a.take<int>(size_t(nv) + 1);
    sums = a.take<int>(size_t(nscan) / 1024 + 2);
    flag = a.take<int>(4);
  };
  layout(sz);
  DevBuf scratch;
  DMG_HIP(hipMalloc(&scratch.p, sz.used));
  Arena a;
  a.base = static_cast<char*>(scratch.p);
  a.cap = sz.used;
  layout(a);
  auto up = [&](void* dst, const void* src, size_t bytes) -> dmg_status {
    DMG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    return DMG_OK;
  };
  auto fill = [&](int* x, int v, size_t n) -> dmg_status {
    k_fill_int<<<grid_for(n), 256, 0, s>>>(x, v, n);
    return launch_check("fill");
  };
  auto read_int = [&](const int* src, int* dst) -> dmg_status {
    DMG_HIP(hipMemcpyAsync(dst, src, sizeof(int), hipMemcpyDeviceToHost, s));
    DMG_HIP(hipStreamSynchronize(s));
    return DMG_OK;
  };
  DMG_CHECK(up(xyc, m.xy_c, 2 * size_t(nv) * sizeof(double)));
  DMG_CHECK(up(xyp, m.xy_p, 2 * size_t(nv) * sizeof(double)));
  DMG_CHECK(up(dqx, qx.data(), qx.size() * sizeof(double)));
  DMG_CHECK(up(dqw, qw.data(), qw.size() * sizeof(double)));
  DMG_CHECK(up(tris, m.tris, 3 * size_t(nt) * sizeof(int)));
  DMG_CHECK(up(dperm, perm.data(), size_t(nv) * sizeof(int)));
  DMG_CHECK(up(dof, m.dof, size_t(nv)));
  // 1. boxes and incidence
  DMG_CHECK(fill(deg, 0, size_t(nv) + 1));
  DMG_CHECK(fill(ncell + nt, 0, 1));
  k_cs_cells<<<grid_for(nt), 256, 0, s>>>(tris, xyc, nt, nx, ny, hx, hy, ncell, deg);
  DMG_CHECK(launch_check("cells"));
  DMG_CHECK(scan(ncell, coff, nt + 1, sums, s));
  DMG_CHECK(scan(deg, vt_ptr, nv + 1, sums, s));
  DMG_CHECK(fill(pos, 0, size_t(nv)));
  k_cs_fill_vt<<<grid_for(nt), 256, 0, s>>>(tris, nt, vt_ptr, pos, vt);
  DMG_CHECK(launch_check("incidence"));
  k_cs_sort_vt<<<grid_for(nv), 256, 0, s>>>(vt_ptr, vt, nv);
  DMG_CHECK(launch_check("incidence order"));
  int total = 0;
  DMG_CHECK(read_int(coff + nt, &total));
  if (total < 0 || size_t(total) * 12 >= (size_t(1) << 40))
    return fail(DMG_ERR_UNSUPPORTED, "triangle-cell pairs exceed the device assembly's range");
  // 2. integrals
  DevBuf recbuf;
  DMG_HIP(hipMalloc(&recbuf.p, std::max<size_t>(1, size_t(total) * 12 * sizeof(double))));
  double* rec = static_cast<double*>(recbuf.p);
  k_cs_integrate<<<grid_for(nt), 256, 0, s>>>(tris, xyc, xyp, nt, nx, ny, hx, hy, nq, dqx, dqw,
                                              coff, rec);
  DMG_CHECK(launch_check("cell integrals"));
  // 3. rows: count, prefix sums, fill
  DMG_CHECK(fill(flag, 0, 1));
  DMG_CHECK(fill(cnt + nv, 0, 1));
  k_cs_rows<true><<<grid_for(nv), 256, 0, s>>>(dperm, dof, vt_ptr, vt, tris, xyc, nv, nx, ny, hx,
                                               hy, coff, rec, cnt, nullptr, nullptr, nullptr,
                                               flag);
  DMG_CHECK(launch_check("row counts"));
  DMG_CHECK(scan(cnt, rp_tmp, nv + 1, sums, s));
  int ovf = 0, nnz = 0;
  DMG_CHECK(read_int(flag, &ovf));
  if (ovf) return fail(DMG_ERR_UNSUPPORTED, "a row of C exceeds the device merge");
  DMG_CHECK(read_int(rp_tmp + nv, &nnz));
  Arena osz;
  DeviceCsrPair r;
  auto olayout = [&](Arena& o) {
    r.rp = o.take<int>(size_t(nv) + 1);
    r.ci = o.take<int>(size_t(nnz) + 1);
    r.v = o.take<double>(size_t(nnz) + 1);
    r.trp = o.take<int>(ng + 1);
    r.tci = o.take<int>(size_t(nnz) + 1);
    r.tv = o.take<double>(size_t(nnz) + 1);
  };
  olayout(osz);
  DevBuf result;
  DMG_HIP(hipMalloc(&result.p, osz.used));
  Arena o;
  o.base = static_cast<char*>(result.p);
  o.cap = osz.used;
  olayout(o);
  DMG_HIP(hipMemcpyAsync(r.rp, rp_tmp, (size_t(nv) + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
  k_cs_rows<false><<<grid_for(nv), 256, 0, s>>>(dperm, dof, vt_ptr, vt, tris, xyc, nv, nx, ny, hx,
                                                hy, coff, rec, nullptr, r.rp, r.ci, r.v, flag);
  DMG_CHECK(launch_check("rows"));
  // 4. transpose: counts per grid column, prefix sums, scatter, rows into mesh order
  int* ccount = cnt;  // reuse: nscan >= ng + 1
  DevBuf cbuf;
  if (ng + 1 > size_t(nv) + 1) {
    DMG_HIP(hipMalloc(&cbuf.p, 2 * (ng + 1) * sizeof(int)));
    ccount = static_cast<int*>(cbuf.p);
  }
  int* tpos = ccount == cnt ? pos : ccount + ng + 1;
  DMG_CHECK(fill(ccount, 0, ng + 1));
  k_cs_colcount<<<grid_for(nv), 256, 0, s>>>(r.rp, r.ci, nv, ccount);
  DMG_CHECK(launch_check("column counts"));
  DMG_CHECK(scan(ccount, r.trp, int(ng) + 1, sums, s));
  DMG_CHECK(fill(tpos, 0, ng));
  k_cs_tfill<<<grid_for(nv), 256, 0, s>>>(r.rp, r.ci, r.v, nv, r.trp, tpos, r.tci, r.tv);
  DMG_CHECK(launch_check("transpose"));
  k_cs_tsort<<<grid_for(ng), 256, 0, s>>>(r.trp, r.tci, r.tv, int(ng));
  DMG_CHECK(launch_check("transpose order"));
  DMG_HIP(hipStreamSynchronize(s));
  r.nnz = nnz;
  r.block = result.p;
  result.p = nullptr;
  out = r;
  return DMG_OK;
}

}  // namespace dmg
