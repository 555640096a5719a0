// Internal declarations shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dmg.h"

namespace dmg {

// ---- error reporting -------------------------------------------------------------------
dmg_status fail(dmg_status code, const char* fmt, ...);
void clear_error();

#define DMG_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::dmg::fail(DMG_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
  } while (0)

#define DMG_CHECK(expr)                      \
  do {                                       \
    dmg_status s_ = (expr);                  \
    if (s_ != DMG_OK) return s_;             \
  } while (0)

inline dmg_status launch_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(DMG_ERR_HIP, "launch of %s failed: %s", what, hipGetErrorString(e));
  return DMG_OK;
}

// ---- a bump allocator over the caller's workspace -------------------------------------
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  template <class T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    size_t bytes = count * sizeof(T);
    used = off + ((bytes + 255) & ~size_t(255));
    if (base == nullptr) return nullptr;  // sizing pass
    return reinterpret_cast<T*>(base + off);
  }
};

// ---- hierarchy ---------------------------------------------------------------------------
struct Level {
  int nx = 0, ny = 0;
  double* S = nullptr;    // [5][ny][nx]
  double* P = nullptr;    // [8][nyc][nxc] weights to the next coarser level (null at coarsest)
  double* u = nullptr;    // correction on coarse levels (level 0 uses the caller's array)
  double* b = nullptr;    // right-hand side on coarse levels
  double* r = nullptr;    // residual scratch
  float* S32 = nullptr;   // fp32 copies for DMG_FP32_IR
  float* P32 = nullptr;
  float* u32 = nullptr;
  float* b32 = nullptr;
  float* r32 = nullptr;
  size_t n() const { return size_t(nx) * size_t(ny); }
};

constexpr int kReduceBlocks = 1024;  // fixed partial count: reductions are order-deterministic

struct Graph {
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  const void* key_u = nullptr;
  const void* key_b = nullptr;
  hipStream_t stream = nullptr;
  int kind = -1;
};

}  // namespace dmg

struct dmg_hier {
  dmg_options opts;
  std::vector<dmg::Level> L;
  int m_coarse = 0;           // unknowns of the coarsest interior system
  int* coarse_idx = nullptr;  // [m] vertex index of each coarsest unknown
  double* chol = nullptr;     // [m][m] Cholesky factor (lower), float64
  double* partials = nullptr; // [kReduceBlocks] reduction partials
  double* scalars = nullptr;  // [16] device scalars (norms, IR scale)
  double* r64 = nullptr;      // fp64 fine residual for iterative refinement
  int* flag = nullptr;        // device status flag
  double* host = nullptr;     // pinned host scalars [16]
  dmg::Graph graph;
  ~dmg_hier();
};

namespace dmg {

// ---- kernels (launchers return DMG_OK or DMG_ERR_HIP) --------------------------------------
dmg_status launch_assemble(const double* jac, const double* K, int nx, int ny, double* S,
                           hipStream_t s);
dmg_status launch_interp_weights(const double* S, int nx, int ny, double* P, hipStream_t s);
dmg_status launch_rap(const double* S, const double* P, int nx, int ny, double* SH,
                      hipStream_t s);
dmg_status launch_coarse_factor(const double* S, int nx, int ny, int m, int* idx, double* chol,
                                int* flag, hipStream_t s);
dmg_status launch_cast(const double* in, float* out, size_t n, hipStream_t s);
dmg_status launch_grad_K(const double* jac, const double* lam, const double* u, int nx, int ny,
                         double* dK, hipStream_t s);

template <class T>
dmg_status launch_coarse_solve(const T* b, T* u, int m, const int* idx, const double* chol,
                               size_t n, hipStream_t s);
template <class T>
dmg_status launch_smooth(const T* S, T* u, const T* b, int nx, int ny, int colour,
                         hipStream_t s);
template <class T>
dmg_status launch_residual(const T* S, const T* u, const T* b, T* r, int nx, int ny,
                           hipStream_t s);
template <class T>
dmg_status launch_restrict(const T* P, const T* r, T* bH, int nx, int ny, hipStream_t s);
template <class T>
dmg_status launch_prolong_add(const T* P, const T* eH, T* u, int nx, int ny, hipStream_t s);
template <class T>
dmg_status launch_fill(T* x, T v, size_t n, hipStream_t s);

// ||b - A u||^2 partials (fixed block count) and sum(x^2) partials; finalize sums the
// partials in a fixed order into out[0] (and sqrt into out[1]).
dmg_status launch_resid_sq_partials(const double* S, const double* u, const double* b, int nx,
                                    int ny, double* partials, hipStream_t s);
dmg_status launch_sq_partials(const double* x, size_t n, int nx, int ny, double* partials,
                              hipStream_t s);
dmg_status launch_finalize(const double* partials, double* out, hipStream_t s);

// iterative refinement helpers
dmg_status launch_ir_update(double* x, const float* e, const double* s_dev, size_t n,
                            hipStream_t s);
dmg_status launch_ir_residual(const double* S, const double* x, const double* b, double* r,
                              int nx, int ny, double* partials, hipStream_t s);
dmg_status launch_ir_scale(const double* r, const double* s_dev, float* r32, size_t n,
                           hipStream_t s);

}  // namespace dmg
