// Setup-phase kernels: Q1 stencil assembly from map Jacobians, operator-induced interpolation
// weights, Galerkin coarse stencils, dense Cholesky of the coarsest interior system, fp32
// casts, and the per-cell adjoint gradient (which reuses the element-matrix code).
//
// Stencil storage: planes C, W, S, SW, SE of [ny][nx]; see include/dmg.h.
#include "dmg_internal.h"

namespace dmg {
namespace {

constexpr int kBX = 64, kBY = 4;
// workgroup of the small-level setup: one wave per SIMD, so that the Galerkin product of a
// coarse point keeps all its operands in registers
constexpr int kSmallThreads = 256;

// ---------------------------------------------------------------------------------------
// Element matrices.  On cell e with widths hx, hy and reference coordinates (s,t) in [0,1]^2
// the bilinear basis has reference gradients (d_s, d_t); in (xi, eta) they are
// (d_s/hx, d_t/hy) and dxi = hx hy ds dt.  With the metric M = det J J^{-1} J^{-T} at the
// 2x2 Gauss points (weights 1/4):
//   G[a][b] = sum_q 1/4 [ M11 ds_a ds_b hy/hx + M12 (ds_a dt_b + dt_a ds_b) + M22 dt_a dt_b hx/hy ].
// Local nodes: 0 = SW (0,0), 1 = SE (1,0), 2 = NW (0,1), 3 = NE (1,1).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void ref_grad(int a, double s, double t, double& ds, double& dt) {
  switch (a) {
    case 0: ds = -(1.0 - t); dt = -(1.0 - s); break;
    case 1: ds = (1.0 - t);  dt = -s;         break;
    case 2: ds = -t;         dt = (1.0 - s);  break;
    default: ds = t;         dt = s;          break;
  }
}

// The four rows of the element matrix of cell c (row a = node a), each accumulated over the
// Gauss points in order; the metric of each Gauss point is formed once for all four rows.
__device__ __forceinline__ void element_rows(const double* __restrict__ jac, size_t ncell,
                                             size_t c, double rx, double ry, double rows[4][4]) {
  const double g0 = 0.5 - 0.28867513459481287;  // 1/2 - 1/(2 sqrt 3)
  const double g1 = 0.5 + 0.28867513459481287;
#pragma unroll
  for (int a = 0; a < 4; ++a) rows[a][0] = rows[a][1] = rows[a][2] = rows[a][3] = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double s = (q & 1) ? g1 : g0;
    const double t = (q & 2) ? g1 : g0;
    const double J11 = jac[(4 * q + 0) * ncell + c];
    const double J12 = jac[(4 * q + 1) * ncell + c];
    const double J21 = jac[(4 * q + 2) * ncell + c];
    const double J22 = jac[(4 * q + 3) * ncell + c];
    const double inv = 1.0 / (J11 * J22 - J12 * J21);
    const double M11 = (J22 * J22 + J12 * J12) * inv;
    const double M12 = -(J22 * J21 + J12 * J11) * inv;
    const double M22 = (J21 * J21 + J11 * J11) * inv;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      double das, dat;
      ref_grad(a, s, t, das, dat);
      // M applied to the scaled gradient of phi_a: (M11 das*ry + M12 dat, M12 das + M22 dat*rx)
      const double va = 0.25 * (M11 * das * ry + M12 * dat);
      const double vb = 0.25 * (M12 * das + M22 * dat * rx);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        double dbs, dbt;
        ref_grad(b, s, t, dbs, dbt);
        rows[a][b] += va * dbs + vb * dbt;
      }
    }
  }
}

// The stencil of a 64 x 4 tile of vertices.  Each of the 65 x 5 cells under the tile gets its
// element rows once, scaled by its K, in LDS (the ten entries the vertices read: row 3 of the
// cell for its NE vertex, row 2 for the NW, row 1 for the SE, row 0 for the SW); each vertex
// then sums the rows of its four cells in the order SW cell, SE cell, NW cell, NE cell.
constexpr int kTileCX = kBX + 1, kTileCY = kBY + 1, kTileCells = kTileCX * kTileCY;
// Sp (nullable): the same stencil point-major as well, each tile row staged in LDS and stored as
// one contiguous run (the hierarchy's level 0, assembled in place).
__global__ __launch_bounds__(256) void k_assemble(const double* __restrict__ jac,
                                                  const double* __restrict__ K, int nx, int ny,
                                                  double* __restrict__ S, double* __restrict__ Sp) {
  // g[e][c]: e = 0..3 row 3 (C, W, S, SW), 4..6 row 2 (C, S, SE), 7..8 row 1 (C, W), 9 row 0 (C)
  __shared__ double g[10][kTileCells];
  const int i0 = blockIdx.x * kBX, j0 = blockIdx.y * kBY;
  const int tid = threadIdx.y * kBX + threadIdx.x;
  const size_t ncell = size_t(nx - 1) * (ny - 1);
  const double rx = double(ny - 1) / double(nx - 1);  // hx/hy with hx = 2/(nx-1), hy = 2/(ny-1)
  const double ry = double(nx - 1) / double(ny - 1);  // hy/hx
  for (int q = tid; q < kTileCells; q += kBX * kBY) {
    const int cx = i0 - 1 + q % kTileCX, cy = j0 - 1 + q / kTileCX;
    if (cx < 0 || cx > nx - 2 || cy < 0 || cy > ny - 2) continue;
    const size_t c = size_t(cy) * (nx - 1) + cx;
    double rows[4][4];
    element_rows(jac, ncell, c, rx, ry, rows);
    const double k = K[c];
    g[0][q] = k * rows[3][3];
    g[1][q] = k * rows[3][2];
    g[2][q] = k * rows[3][1];
    g[3][q] = k * rows[3][0];
    g[4][q] = k * rows[2][2];
    g[5][q] = k * rows[2][0];
    g[6][q] = k * rows[2][1];
    g[7][q] = k * rows[1][1];
    g[8][q] = k * rows[1][0];
    g[9][q] = k * rows[0][0];
  }
  __syncthreads();
  const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
  const bool in = i < nx && j < ny;
  const size_t N = size_t(nx) * ny;
  const size_t v = size_t(j) * nx + i;
  double C = 0, W = 0, So = 0, SW = 0, SE = 0;
  if (in && i > 0 && i < nx - 1 && j > 0 && j < ny - 1) {
    const int qsw = threadIdx.y * kTileCX + threadIdx.x;  // cell (i-1, j-1): v is its NE node
    const int qse = qsw + 1;                              // cell (i, j-1): v is its NW node
    const int qnw = qsw + kTileCX;                        // cell (i-1, j): v is its SE node
    const int qne = qnw + 1;                              // cell (i, j): v is its SW node
    C += g[0][qsw];
    if (i - 1 > 0) W += g[1][qsw];
    if (j - 1 > 0) So += g[2][qsw];
    if (i - 1 > 0 && j - 1 > 0) SW += g[3][qsw];
    C += g[4][qse];
    if (j - 1 > 0) So += g[5][qse];
    if (j - 1 > 0 && i + 1 < nx - 1) SE += g[6][qse];
    C += g[7][qnw];
    if (i - 1 > 0) W += g[8][qnw];
    C += g[9][qne];
  }
  if (in) {
    S[0 * N + v] = C;
    S[1 * N + v] = W;
    S[2 * N + v] = So;
    S[3 * N + v] = SW;
    S[4 * N + v] = SE;
  }
  if (!Sp) return;  // uniform over the workgroup
  __shared__ double sp[kBY][5 * kBX];
  const double vals[5] = {C, W, So, SW, SE};
#pragma unroll
  for (int k = 0; k < 5; ++k) sp[threadIdx.y][5 * threadIdx.x + k] = vals[k];
  __syncthreads();
  const int cnt = 5 * (nx - i0 < kBX ? nx - i0 : kBX);  // values of one tile row
  for (int q = tid; q < kBY * 5 * kBX; q += kBX * kBY) {
    const int r = q / (5 * kBX), k = q % (5 * kBX);
    if (k < cnt && j0 + r < ny) Sp[5 * (size_t(j0 + r) * nx + i0) + k] = sp[r][k];
  }
}

__global__ __launch_bounds__(256) void k_grad_K(const double* __restrict__ jac,
                                                const double* __restrict__ lam,
                                                const double* __restrict__ u, int nx, int ny,
                                                double* __restrict__ dK) {
  const int i = blockIdx.x * kBX + threadIdx.x;
  const int j = blockIdx.y * kBY + threadIdx.y;
  if (i >= nx - 1 || j >= ny - 1) return;
  const size_t ncell = size_t(nx - 1) * (ny - 1);
  const size_t c = size_t(j) * (nx - 1) + i;
  const double rx = double(ny - 1) / double(nx - 1);
  const double ry = double(nx - 1) / double(ny - 1);
  const size_t v0 = size_t(j) * nx + i;
  const double uv[4] = {u[v0], u[v0 + 1], u[v0 + nx], u[v0 + nx + 1]};
  const double lv[4] = {lam[v0], lam[v0 + 1], lam[v0 + nx], lam[v0 + nx + 1]};
  double acc = 0.0;
  double rows[4][4];
  element_rows(jac, ncell, c, rx, ry, rows);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const double* row = rows[a];
    acc += lv[a] * (row[0] * uv[0] + row[1] * uv[1] + row[2] * uv[2] + row[3] * uv[3]);
  }
  dK[c] = -acc;
}

// ---------------------------------------------------------------------------------------
// Operator-induced interpolation.  Full 9-point couplings of fine point (i,j) read from the
// symmetric storage: E = W(i+1,j), N = S(i,j+1), NE = SW(i+1,j+1), NW = SE(i-1,j+1).
// ---------------------------------------------------------------------------------------
struct Nine {
  double C, W, E, S, N, SW, SE, NW, NE;
};

__device__ __forceinline__ Nine load9(const double* __restrict__ S, size_t N, int nx, int i,
                                      int j) {
  // only called for interior (i,j): all neighbours exist
  const size_t v = size_t(j) * nx + i;
  Nine a;
  a.C = S[v];
  a.W = S[N + v];
  a.E = S[N + v + 1];
  a.S = S[2 * N + v];
  a.N = S[2 * N + v + nx];
  a.SW = S[3 * N + v];
  a.NE = S[3 * N + v + nx + 1];
  a.SE = S[4 * N + v];
  a.NW = S[4 * N + v + nx - 1];
  return a;
}

// x-line fine point (i,j) (odd i, even j): weights to (i-1,j) and (i+1,j); 0 on the boundary.
__device__ __forceinline__ void xline_w(const double* S, size_t N, int nx, int ny, int i, int j,
                                        double& wW, double& wE) {
  if (j <= 0 || j >= ny - 1) { wW = wE = 0.0; return; }
  const Nine a = load9(S, N, nx, i, j);
  const double d = a.C + a.N + a.S;
  wW = -(a.W + a.NW + a.SW) / d;
  wE = -(a.E + a.NE + a.SE) / d;
}

// y-line fine point (i,j) (even i, odd j): weights to (i,j-1) and (i,j+1).
__device__ __forceinline__ void yline_w(const double* S, size_t N, int nx, int ny, int i, int j,
                                        double& wS, double& wN) {
  if (i <= 0 || i >= nx - 1) { wS = wN = 0.0; return; }
  const Nine a = load9(S, N, nx, i, j);
  const double d = a.C + a.W + a.E;
  wS = -(a.S + a.SW + a.SE) / d;
  wN = -(a.N + a.NW + a.NE) / d;
}

// Line weights from a loaded stencil, as xline_w / yline_w.
__device__ __forceinline__ void xline_of(const Nine& a, double& wW, double& wE) {
  const double d = a.C + a.N + a.S;
  wW = -(a.W + a.NW + a.SW) / d;
  wE = -(a.E + a.NE + a.SE) / d;
}
__device__ __forceinline__ void yline_of(const Nine& a, double& wS, double& wN) {
  const double d = a.C + a.W + a.E;
  wS = -(a.S + a.SW + a.SE) / d;
  wN = -(a.N + a.NW + a.NE) / d;
}

// Weights of coarse point (I, J) (see the layout of P in the library header).  The five fine
// stencils involved are loaded first (one memory round trip); the x-line point (2I+1, 2J) and
// the y-line point (2I, 2J+1) also serve as the S and W neighbours of the centre point.
__device__ __forceinline__ void interp_point(const double* __restrict__ S, int nx, int ny,
                                             double* __restrict__ P, int I, int J) {
  const int ncx = (nx + 1) / 2, ncy = (ny + 1) / 2;
  const size_t N = size_t(nx) * ny;
  const size_t NC = size_t(ncx) * ncy;
  const size_t c = size_t(J) * ncx + I;
  const bool hasX = I < ncx - 1, hasY = J < ncy - 1, hasC = hasX && hasY;
  // a line weight is 0 on a boundary row (x-lines) or column (y-lines)
  const bool xa = hasX && 2 * J > 0 && 2 * J < ny - 1;   // x-line point (2I+1, 2J)
  const bool ya = hasY && 2 * I > 0 && 2 * I < nx - 1;   // y-line point (2I, 2J+1)
  const bool xb = hasC && 2 * J + 2 < ny - 1;            // x-line point (2I+1, 2J+2)
  const bool yb = hasC && 2 * I + 2 < nx - 1;            // y-line point (2I+2, 2J+1)
  // stencils not needed are read at (1, 1), an interior point, and not used
  const Nine sxa = load9(S, N, nx, xa ? 2 * I + 1 : 1, xa ? 2 * J : 1);
  const Nine sya = load9(S, N, nx, ya ? 2 * I : 1, ya ? 2 * J + 1 : 1);
  const Nine sc = load9(S, N, nx, hasC ? 2 * I + 1 : 1, hasC ? 2 * J + 1 : 1);
  const Nine sxb = load9(S, N, nx, xb ? 2 * I + 1 : 1, xb ? 2 * J + 2 : 1);
  const Nine syb = load9(S, N, nx, yb ? 2 * I + 2 : 1, yb ? 2 * J + 1 : 1);
  __builtin_amdgcn_sched_barrier(0);
  double w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (xa) xline_of(sxa, w[0], w[1]);
  if (ya) yline_of(sya, w[2], w[3]);
  if (hasC) {
    double wSe = 0, wNe = 0, wWn = 0, wEn = 0;
    if (yb) yline_of(syb, wSe, wNe);  // E neighbour
    if (xb) xline_of(sxb, wWn, wEn);  // N neighbour
    // W neighbour = the y-line point, S neighbour = the x-line point
    const double wSw = w[2], wNw = w[3], wWs = w[0], wEs = w[1];
    const Nine& a = sc;
    w[4] = -(a.SW + a.W * wSw + a.S * wWs) / a.C;
    w[5] = -(a.SE + a.E * wSe + a.S * wEs) / a.C;
    w[6] = -(a.NW + a.W * wNw + a.N * wWn) / a.C;
    w[7] = -(a.NE + a.E * wNe + a.N * wEn) / a.C;
  }
#pragma unroll
  for (int p = 0; p < 8; ++p) P[p * NC + c] = w[p];
}

__global__ __launch_bounds__(256) void k_interp(const double* __restrict__ S, int nx, int ny,
                                                double* __restrict__ P) {
  const int I = blockIdx.x * kBX + threadIdx.x;
  const int J = blockIdx.y * kBY + threadIdx.y;
  if (I >= (nx + 1) / 2 || J >= (ny + 1) / 2) return;
  interp_point(S, nx, ny, P, I, J);
}

// ---------------------------------------------------------------------------------------
// Galerkin coarse stencil A_H = P^T A P.  Coarse column (I,J) of P is supported on the fine
// 3x3 block around (2I,2J); pw9() returns its weights at the fine offsets (a,b) in {-1,0,1}^2.
// ---------------------------------------------------------------------------------------
// fine matrix entry A[(i,j), (i+da, j+db)]
__device__ __forceinline__ double aentry(const double* __restrict__ S, size_t N, int nx, int i,
                                         int j, int da, int db) {
  const size_t v = size_t(j) * nx + i;
  if (db == 0) {
    if (da == 0) return S[v];
    return da < 0 ? S[N + v] : S[N + v + 1];
  }
  if (da == 0) return db < 0 ? S[2 * N + v] : S[2 * N + v + nx];
  if (da < 0 && db < 0) return S[3 * N + v];
  if (da > 0 && db > 0) return S[3 * N + v + nx + 1];
  if (da > 0 && db < 0) return S[4 * N + v];
  return S[4 * N + v + nx - 1];  // da < 0, db > 0
}

// The weights of coarse column (I, J) of P at the fine offsets (a, b) in {-1,0,1}^2, as
// w[3 (b + 1) + (a + 1)] (the centre weight is 1).
__device__ __forceinline__ void pw9(const double* __restrict__ P, size_t NC, int ncx, int I, int J,
                                    double w[9]) {
  const size_t c = size_t(J) * ncx + I;
  w[0] = P[7 * NC + c - ncx - 1];
  w[1] = P[3 * NC + c - ncx];
  w[2] = P[6 * NC + c - ncx];
  w[3] = P[1 * NC + c - 1];
  w[4] = 1.0;
  w[5] = P[0 * NC + c];
  w[6] = P[5 * NC + c - 1];
  w[7] = P[2 * NC + c];
  w[8] = P[4 * NC + c];
}

// Coarse stencil at (I, J): planar into SH and, when SHp is given, point-major into SHp.
// Every operand is loaded up front (the 3x3 fine stencils under the coarse point and the
// weights of the five target columns), then the triple product is summed with compile-time
// offsets in the order (fine point, its neighbour, target).  Zero weights and couplings add
// exact zeros, so the sums equal those that skip them.
__device__ __forceinline__ void rap_point(const double* __restrict__ S,
                                          const double* __restrict__ P, int nx, int ny,
                                          double* __restrict__ SH, double* __restrict__ SHp,
                                          int I, int J) {
  const int ncx = (nx + 1) / 2, ncy = (ny + 1) / 2;
  const size_t N = size_t(nx) * ny;
  const size_t NC = size_t(ncx) * ncy;
  const size_t c = size_t(J) * ncx + I;
  // targets: C (0,0), W (-1,0), S (0,-1), SW (-1,-1), SE (1,-1)
  constexpr int tI[5] = {0, -1, 0, -1, 1};
  constexpr int tJ[5] = {0, 0, -1, -1, -1};
  double acc[5] = {0, 0, 0, 0, 0};
  const bool interior = I > 0 && I < ncx - 1 && J > 0 && J < ncy - 1;
  if (interior) {
    bool live[5];
    double wt[5][9];
#pragma unroll
    for (int t = 0; t < 5; ++t) {
      const int I2 = I + tI[t], J2 = J + tJ[t];
      live[t] = I2 > 0 && I2 < ncx - 1 && J2 > 0 && J2 < ncy - 1;
      // a boundary target contributes nothing: read the centre's weights in its place
      pw9(P, NC, ncx, live[t] ? I2 : I, live[t] ? J2 : J, wt[t]);
    }
    Nine a9[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) a9[q] = load9(S, N, nx, 2 * I + q % 3 - 1, 2 * J + q / 3 - 1);
    // every load above is issued before any product below: one memory round trip per point
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b1 = -1; b1 <= 1; ++b1) {
#pragma unroll
      for (int a1 = -1; a1 <= 1; ++a1) {
        const double w1 = wt[0][3 * (b1 + 1) + (a1 + 1)];
        const Nine& A = a9[3 * (b1 + 1) + (a1 + 1)];
        const double av9[9] = {A.SW, A.S, A.SE, A.W, A.C, A.E, A.NW, A.N, A.NE};
#pragma unroll
        for (int db = -1; db <= 1; ++db) {
#pragma unroll
          for (int da = -1; da <= 1; ++da) {
            const double wa = w1 * av9[3 * (db + 1) + (da + 1)];
#pragma unroll
            for (int t = 0; t < 5; ++t) {
              // offset of the fine neighbour from the target coarse point's fine position
              const int oa = a1 + da - 2 * tI[t];
              const int ob = b1 + db - 2 * tJ[t];
              if (oa < -1 || oa > 1 || ob < -1 || ob > 1) continue;
              const double v = acc[t] + wa * wt[t][3 * (ob + 1) + (oa + 1)];
              acc[t] = live[t] ? v : acc[t];
            }
          }
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 5; ++t) SH[t * NC + c] = acc[t];
  if (SHp) {
#pragma unroll
    for (int t = 0; t < 5; ++t) SHp[5 * c + t] = acc[t];
  }
}

// One wave per SIMD: the ~120 operands of a coarse point stay in registers.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_rap(
    const double* __restrict__ S,
                                             const double* __restrict__ P, int nx, int ny,
                                             double* __restrict__ SH, double* __restrict__ SHp) {
  const int I = blockIdx.x * kBX + threadIdx.x;
  const int J = blockIdx.y * kBY + threadIdx.y;
  if (I >= (nx + 1) / 2 || J >= (ny + 1) / 2) return;
  rap_point(S, P, nx, ny, SH, SHp, I, J);
}

// ---------------------------------------------------------------------------------------
// Coarsest level: gather the m interior unknowns into a dense matrix and factor it in place
// (lower Cholesky) with one workgroup.  flag[0] = 1 on a non-positive pivot.
// ---------------------------------------------------------------------------------------
__device__ void coarse_factor_body(const double* __restrict__ S, int nx, int ny, int m,
                                   int* __restrict__ idx, double* __restrict__ L,
                                   int* __restrict__ flag) {
  const size_t N = size_t(nx) * ny;
  const int mx = nx - 2;
  for (int k = threadIdx.x; k < m; k += blockDim.x) idx[k] = (k / mx + 1) * nx + (k % mx + 1);
  // dense symmetric matrix over interior unknowns r = (j-1)*mx + (i-1)
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int r = e / m, c = e % m;
    const int ir = r % mx + 1, jr = r / mx + 1;
    const int ic = c % mx + 1, jc = c / mx + 1;
    const int da = ic - ir, db = jc - jr;
    double v = 0.0;
    if (da >= -1 && da <= 1 && db >= -1 && db <= 1) v = aentry(S, N, nx, ir, jr, da, db);
    L[e] = v;
  }
  if (threadIdx.x == 0) flag[0] = 0;
  __syncthreads();
  __shared__ double piv;
  for (int k = 0; k < m; ++k) {
    if (threadIdx.x == 0) {
      const double d = L[k * m + k];
      if (!(d > 0.0)) flag[0] = 1;
      piv = d > 0.0 ? sqrt(d) : 1.0;
      L[k * m + k] = piv;
    }
    __syncthreads();
    for (int r = k + 1 + threadIdx.x; r < m; r += blockDim.x) L[r * m + k] /= piv;
    __syncthreads();
    const int rem = m - k - 1;
    for (int e = threadIdx.x; e < rem * rem; e += blockDim.x) {
      const int r = k + 1 + e / rem, c = k + 1 + e % rem;
      if (c <= r) L[r * m + c] -= L[r * m + k] * L[c * m + k];
    }
    __syncthreads();
  }
}



// Setup of the small levels in one workgroup: for k = 0..nlev-2, the weights P[k] of level k and
// the Galerkin stencil of level k+1 (planar, and point-major where Sp[k+1] is set), then the
// Cholesky factor of the last level.
__global__ __launch_bounds__(kSmallThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void
k_setup_small(SmallSetup a) {
  for (int k = 0; k + 1 < a.nlev; ++k) {
    const int nx = a.nx[k], ny = a.ny[k];
    const int ncx = (nx + 1) / 2, ncy = (ny + 1) / 2;
    for (int c = threadIdx.x; c < ncx * ncy; c += blockDim.x) interp_point(a.S[k], nx, ny, a.P[k], c % ncx, c / ncx);
    __syncthreads();
    for (int c = threadIdx.x; c < ncx * ncy; c += blockDim.x)
      rap_point(a.S[k], a.P[k], nx, ny, a.S[k + 1], a.Sp[k + 1], c % ncx, c / ncx);
    __syncthreads();
  }
  const int l = a.nlev - 1;
  coarse_factor_body(a.S[l], a.nx[l], a.ny[l], a.m, a.idx, a.chol, a.flag);
}

// Level 0: the caller's planar stencil copied into the hierarchy, planar and point-major.  Each
// workgroup takes 256 consecutive points: the five planes are read and copied coalesced, the
// point-major block goes through LDS so that it is written as one contiguous run.
__global__ __launch_bounds__(256) void k_copy_pack(const double* __restrict__ S,
                                                   double* __restrict__ Sd,
                                                   double* __restrict__ Sp, size_t n) {
  __shared__ double tile[5 * 256];
  const int t = int(threadIdx.x);
  for (size_t base = size_t(blockIdx.x) * 256; base < n; base += size_t(gridDim.x) * 256) {
    const size_t v = base + t;
    const int cnt = int(n - base < 256 ? n - base : 256);
    double x[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) x[k] = v < n ? S[k * n + v] : 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      if (v < n) Sd[k * n + v] = x[k];
      tile[5 * t + k] = x[k];
    }
    __syncthreads();
    if (Sp)
      for (int q = t; q < 5 * cnt; q += 256) Sp[5 * base + q] = tile[q];
    __syncthreads();  // the tile is rewritten by the next chunk
  }
}

__global__ __launch_bounds__(256) void k_cast(const double* __restrict__ in, float* __restrict__ out,
                                              size_t n) {
  for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < n;
       k += size_t(gridDim.x) * blockDim.x)
    out[k] = float(in[k]);
}

template <class T>
__global__ __launch_bounds__(256) void k_pack(const double* __restrict__ S, T* __restrict__ out,
                                              size_t n) {
  for (size_t v = blockIdx.x * size_t(blockDim.x) + threadIdx.x; v < n;
       v += size_t(gridDim.x) * blockDim.x) {
#pragma unroll
    for (int k = 0; k < 5; ++k) out[5 * v + k] = T(S[k * n + v]);
  }
}

// Several float32 roundings in one launch: workgroup b serves the segment whose block range
// holds b (a scan over the segment table, uniform per workgroup).
__global__ __launch_bounds__(256) void k_f32_batch(F32Batch a) {
  int b = blockIdx.x, k = 0;
  while (k < a.count && b >= a.seg[k].blocks) b -= a.seg[k++].blocks;
  if (k >= a.count) return;
  const F32Seg g = a.seg[k];
  const size_t step = size_t(g.blocks) * blockDim.x;
  if (g.pack) {  // point-major: 256 points per chunk, staged in LDS, written as one run
    __shared__ float tile[5 * 256];
    const int t = int(threadIdx.x);
    for (size_t base = size_t(b) * 256; base < g.n; base += step) {
      const size_t v = base + t;
      const int cnt = int(g.n - base < 256 ? g.n - base : 256);
#pragma unroll
      for (int c = 0; c < 5; ++c) tile[5 * t + c] = v < g.n ? float(g.src[c * g.n + v]) : 0.f;
      __syncthreads();
      for (int q = t; q < 5 * cnt; q += 256) g.dst[5 * base + q] = tile[q];
      __syncthreads();
    }
    return;
  }
  for (size_t v = size_t(b) * blockDim.x + threadIdx.x; v < g.n; v += step)
    g.dst[v] = float(g.src[v]);
}

dim3 grid2(int nx, int ny) { return dim3((nx + kBX - 1) / kBX, (ny + kBY - 1) / kBY); }

}  // namespace

dmg_status F32Batch::add(const double* src, float* dst, size_t n, int pack) {
  if (n == 0) return DMG_OK;
  if (count >= kMaxF32Segs) return fail(DMG_ERR_INVALID_ARG, "too many float32 segments");
  F32Seg& g = seg[count++];
  g.src = src;
  g.dst = dst;
  g.n = n;
  g.pack = pack;
  const size_t blocks = (n + 255) / 256;
  g.blocks = int(blocks < 2048 ? blocks : 2048);
  return DMG_OK;
}

dmg_status launch_f32_batch(const F32Batch& a, hipStream_t s) {
  if (a.count == 0) return DMG_OK;
  long blocks = 0;
  for (int k = 0; k < a.count; ++k) blocks += a.seg[k].blocks;
  k_f32_batch<<<dim3(unsigned(blocks)), 256, 0, s>>>(a);
  return launch_check("f32 batch");
}

dmg_status launch_assemble(const double* jac, const double* K, int nx, int ny, double* S,
                           hipStream_t s, double* Sp) {
  k_assemble<<<grid2(nx, ny), dim3(kBX, kBY), 0, s>>>(jac, K, nx, ny, S, Sp);
  return launch_check("assemble");
}

dmg_status launch_grad_K(const double* jac, const double* lam, const double* u, int nx, int ny,
                         double* dK, hipStream_t s) {
  k_grad_K<<<grid2(nx - 1, ny - 1), dim3(kBX, kBY), 0, s>>>(jac, lam, u, nx, ny, dK);
  return launch_check("grad_K");
}

dmg_status launch_interp_weights(const double* S, int nx, int ny, double* P, hipStream_t s) {
  k_interp<<<grid2((nx + 1) / 2, (ny + 1) / 2), dim3(kBX, kBY), 0, s>>>(S, nx, ny, P);
  return launch_check("interp_weights");
}

dmg_status launch_rap(const double* S, const double* P, int nx, int ny, double* SH,
                      double* SHp, hipStream_t s) {
  k_rap<<<grid2((nx + 1) / 2, (ny + 1) / 2), dim3(kBX, kBY), 0, s>>>(S, P, nx, ny, SH, SHp);
  return launch_check("rap");
}



dmg_status launch_setup_small(const SmallSetup& a, hipStream_t s) {
  if (a.nlev < 1 || a.nlev > kMaxTail + 1) return fail(DMG_ERR_INVALID_ARG, "small setup depth %d", a.nlev);
  k_setup_small<<<1, kSmallThreads, 0, s>>>(a);
  return launch_check("setup_small");
}

dmg_status launch_copy_pack(const double* S, double* Sd, double* Sp, size_t n, hipStream_t s) {
  const size_t blocks = (n + 255) / 256;
  k_copy_pack<<<dim3(unsigned(blocks < 65535 ? (blocks ? blocks : 1) : 65535)), 256, 0, s>>>(S, Sd, Sp, n);
  return launch_check("copy_pack");
}

template <class T>
dmg_status launch_pack(const double* S, T* out, size_t n, hipStream_t s) {
  const size_t blocks = (n + 255) / 256;
  k_pack<T><<<dim3(unsigned(blocks < 65535 ? (blocks ? blocks : 1) : 65535)), 256, 0, s>>>(S, out, n);
  return launch_check("pack");
}
template dmg_status launch_pack<double>(const double*, double*, size_t, hipStream_t);
template dmg_status launch_pack<float>(const double*, float*, size_t, hipStream_t);

dmg_status launch_cast(const double* in, float* out, size_t n, hipStream_t s) {
  const size_t blocks = (n + 255) / 256;
  k_cast<<<dim3(unsigned(blocks < 65535 ? blocks : 65535)), 256, 0, s>>>(in, out, n);
  return launch_check("cast");
}

}  // namespace dmg
