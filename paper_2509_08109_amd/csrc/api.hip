// C-ABI entry points: validation, workspace carving, hierarchy setup, V-cycles and solve
// drivers (float64 and float32-in-float64 refinement), adjoint gradient, batched solves.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>

#include "dmg_internal.h"

namespace dmg {

namespace {
thread_local char g_err[1024] = "";
}

dmg_status fail(dmg_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_err[0] = 0; }

namespace {

bool pow2p1(int n) {
  if (n < 3) return false;
  const int m = n - 1;
  return (m & (m - 1)) == 0;
}

dmg_status check_options(const dmg_options* o) {
  if (!o) return fail(DMG_ERR_INVALID_ARG, "options pointer is null");
  if (o->nu_pre < 0 || o->nu_post < 0 || o->nu_pre + o->nu_post == 0 || o->nu_pre > 8 ||
      o->nu_post > 8)
    return fail(DMG_ERR_INVALID_ARG, "nu_pre/nu_post must be in [0,8] and not both 0");
  for (const int32_t* ord : {o->pre_order, o->post_order}) {
    int seen = 0;
    for (int k = 0; k < 4; ++k) {
      if (ord[k] < 0 || ord[k] > 3 || (seen >> ord[k]) & 1)
        return fail(DMG_ERR_INVALID_ARG, "colour orders must be permutations of 0..3");
      seen |= 1 << ord[k];
    }
  }
  for (const int32_t* ord : {o->pre_order, o->post_order})
    if ((ord[0] >> 1) != (ord[1] >> 1))
      return fail(DMG_ERR_UNSUPPORTED,
                  "colour orders must visit both colours of one row parity first "
                  "(e.g. 0,1,2,3 or 3,2,1,0)");
  if (o->coarsest_n < 3) return fail(DMG_ERR_INVALID_ARG, "coarsest_n must be >= 3");
  if (o->precision != DMG_FP64 && o->precision != DMG_FP32_IR)
    return fail(DMG_ERR_INVALID_ARG, "unknown precision %d", o->precision);
  if (o->inner_cycles < 1 || o->inner_cycles > 16)
    return fail(DMG_ERR_INVALID_ARG, "inner_cycles must be in [1,16]");
  return DMG_OK;
}

dmg_status level_dims(int nx, int ny, int coarsest_n, std::vector<std::pair<int, int>>& dims) {
  if (!pow2p1(nx) || !pow2p1(ny))
    return fail(DMG_ERR_DIMS, "grid dims %d x %d: each must be 2^k+1 with k >= 1", nx, ny);
  dims.clear();
  dims.emplace_back(nx, ny);
  while (std::min(dims.back().first, dims.back().second) > coarsest_n)
    dims.emplace_back((dims.back().first + 1) / 2, (dims.back().second + 1) / 2);
  const auto& c = dims.back();
  const long m = long(c.first - 2) * long(c.second - 2);
  if (m > 4096)
    return fail(DMG_ERR_DIMS, "coarsest system has %ld unknowns (max 4096); lower coarsest_n", m);
  return DMG_OK;
}

// Launch shape of the strip kernels on an nx x ny level: enough workgroups to fill the chip
// with as few recomputed halo rows/columns as possible.  tile_rows overrides the segment height.
StripConfig default_strip_config(int nx, int ny, const dmg_options& o) {
  StripConfig c;
  c.bw = nx >= 257 ? 128 : 64;
  int ns = 0, nseg = 0;
  c.seg_h = 16;
  for (int h = 128; h >= 16; h >>= 1) {
    strip_blocks(nx, ny, c.bw, h, &ns, &nseg);
    if (ns * nseg >= 1024) {
      c.seg_h = h;
      break;
    }
  }
  if (o.tile_rows >= 2) c.seg_h = o.tile_rows & ~1;
  while (strip_blocks(nx, ny, c.bw, c.seg_h, &ns, &nseg) > kMaxPartials) c.seg_h *= 2;
  return c;
}

// Lays out a hierarchy in the arena (sizing pass when a.base is null).
void carve(dmg_hier& h, Arena& a, const std::vector<std::pair<int, int>>& dims,
           const dmg_options& o) {
  const bool fp32 = o.precision == DMG_FP32_IR;
  h.L.assign(dims.size(), Level{});
  h.tail = int(dims.size()) - 1;
  while (h.tail > 0 && std::max(dims[h.tail - 1].first, dims[h.tail - 1].second) <= kTailMaxN)
    --h.tail;
  for (size_t l = 0; l < dims.size(); ++l) {
    Level& L = h.L[l];
    L.nx = dims[l].first;
    L.ny = dims[l].second;
    const size_t n = L.n();
    L.S = a.take<double>(5 * n);
    if (int(l) < h.tail) {
      L.t = a.take<double>(n);
      if (fp32) L.t32 = a.take<float>(n);
    }
    if (l + 1 < dims.size()) {
      const size_t nc = size_t(dims[l + 1].first) * dims[l + 1].second;
      L.P = a.take<double>(8 * nc);
      L.r = a.take<double>(n);
      if (fp32) {
        L.P32 = a.take<float>(8 * nc);
        L.r32 = a.take<float>(n);
      }
    }
    if (l > 0) {
      L.u = a.take<double>(n);
      L.b = a.take<double>(n);
    }
    if (fp32) {
      L.S32 = a.take<float>(5 * n);
      L.u32 = a.take<float>(n);
      L.b32 = a.take<float>(n);
    }
  }
  const auto& c = dims.back();
  h.m_coarse = (c.first - 2) * (c.second - 2);
  h.coarse_idx = a.take<int>(size_t(h.m_coarse));
  h.chol = a.take<double>(size_t(h.m_coarse) * h.m_coarse);
  h.partials = a.take<double>(kMaxPartials);
  for (size_t l = 0; l < dims.size(); ++l) h.L[l].cfg = default_strip_config(dims[l].first, dims[l].second, o);
  h.scalars = a.take<double>(16);
  h.flag = a.take<int>(16);
  if (fp32) h.r64 = a.take<double>(size_t(dims[0].first) * dims[0].second);
}

template <class T>
struct Prec;
template <>
struct Prec<double> {
  static double* t(const Level& L) { return L.t; }
  static const double* S(const Level& L) { return L.S; }
  static const double* P(const Level& L) { return L.P; }
  static double* u(const Level& L) { return L.u; }
  static double* b(const Level& L) { return L.b; }
  static double* r(const Level& L) { return L.r; }
};
template <>
struct Prec<float> {
  static float* t(const Level& L) { return L.t32; }
  static const float* S(const Level& L) { return L.S32; }
  static const float* P(const Level& L) { return L.P32; }
  static float* u(const Level& L) { return L.u32; }
  static float* b(const Level& L) { return L.b32; }
  static float* r(const Level& L) { return L.r32; }
};

// Strip-kernel colour-order parameters: row parity smoothed first and the column parity
// smoothed first on each row parity.
struct OrderParams {
  int pf, cA, cB;
};
OrderParams order_params(const int32_t* ord) {
  return OrderParams{ord[0] >> 1, ord[0] & 1, ord[2] & 1};
}

template <class T>
dmg_status tail_launch(dmg_hier* h, T* u_top, const T* b_top, hipStream_t s, bool u0_zero) {
  using Pr = Prec<T>;
  TailSpec<T> sp;
  const int nl = int(h->L.size());
  sp.nlev = nl - h->tail;
  for (int l = h->tail; l < nl; ++l) {
    const Level& L = h->L[l];
    const int k = l - h->tail;
    sp.S[k] = Pr::S(L);
    sp.u[k] = l == 0 ? u_top : Pr::u(L);
    sp.b[k] = l == 0 ? const_cast<T*>(b_top) : Pr::b(L);
    sp.r[k] = Pr::r(L);
    sp.P[k] = Pr::P(L);
    sp.nx[k] = L.nx;
    sp.ny[k] = L.ny;
  }
  sp.zero_top = h->tail > 0 || u0_zero;
  sp.m = h->m_coarse;
  sp.idx = h->coarse_idx;
  sp.chol = h->chol;
  for (int k = 0; k < 4; ++k) {
    sp.pre[k] = h->opts.pre_order[k];
    sp.post[k] = h->opts.post_order[k];
  }
  sp.nu_pre = h->opts.nu_pre;
  sp.nu_post = h->opts.nu_post;
  return launch_tail<T>(sp, s);
}

// One V-cycle in precision T on level-0 arrays (u0, b0); coarse levels use hierarchy arrays.
// Levels above the tail: fused pre kernels on the way down (the first sweep of a coarse level
// starts from u = 0; u0_zero says the same of level 0), fused post kernels on the way up.  The
// strip kernels are out of place: each level alternates between its two iterate buffers and
// the cycle ends with the level-0 iterate back in u0.  partials (optional) receives the
// squared-residual partials of the final level-0 iterate.
template <class T>
dmg_status vcycle_impl(dmg_hier* h, T* u0, const T* b0, hipStream_t s, double* partials = nullptr,
                       bool u0_zero = false) {
  using Pr = Prec<T>;
  const dmg_options& o = h->opts;
  const OrderParams pre = order_params(o.pre_order), post = order_params(o.post_order);
  T* cur[kMaxLevels];
  auto other = [&](int l, const T* x) -> T* {
    T* a = l == 0 ? u0 : Pr::u(h->L[l]);
    return x == a ? Pr::t(h->L[l]) : a;
  };
  for (int l = 0; l < h->tail; ++l) {
    const Level& L = h->L[l];
    const T* b = l == 0 ? b0 : Pr::b(L);
    const T* src = (l == 0 && !u0_zero) ? u0 : nullptr;
    // every sweep writes the restriction of its residual; the last sweep's is the one used
    for (int k = 0; k < o.nu_pre; ++k) {
      T* dst = src ? other(l, src) : Pr::t(L);
      DMG_CHECK(launch_pre<T>(L.cfg, Pr::S(L), src, dst, b, Pr::P(L), Pr::b(h->L[l + 1]), L.nx,
                              L.ny, pre.pf, pre.cA, pre.cB, s));
      src = dst;
    }
    cur[l] = const_cast<T*>(src);
  }
  T* ut = h->tail == 0 ? u0 : Pr::u(h->L[h->tail]);
  const T* bt = h->tail == 0 ? b0 : Pr::b(h->L[h->tail]);
  DMG_CHECK(tail_launch<T>(h, ut, bt, s, u0_zero));
  const T* e = ut;
  for (int l = h->tail - 1; l >= 0; --l) {
    const Level& L = h->L[l];
    const T* b = l == 0 ? b0 : Pr::b(L);
    for (int k = 0; k < o.nu_post; ++k) {
      const bool first = k == 0, last = k + 1 == o.nu_post;  // prolongate once, norm once
      T* dst = other(l, cur[l]);
      DMG_CHECK(launch_post<T>(L.cfg, Pr::S(L), cur[l], dst, b, Pr::P(L), first ? e : nullptr,
                               (l == 0 && last) ? partials : nullptr, L.nx, L.ny, post.pf, post.cA,
                               post.cB, s));
      cur[l] = dst;
    }
    e = cur[l];
  }
  if (h->tail > 0 && cur[0] != u0)
    DMG_HIP(hipMemcpyAsync(u0, cur[0], h->L[0].n() * sizeof(T), hipMemcpyDeviceToDevice, s));
  return DMG_OK;
}

int post_partials_count(const dmg_hier* h) {
  const Level& L = h->L[0];
  int ns = 0, nseg = 0;
  return strip_blocks(L.nx, L.ny, L.cfg.bw, L.cfg.seg_h, &ns, &nseg);
}

dmg_status read_scalar(dmg_hier* h, int slot, double* out, hipStream_t s) {
  DMG_HIP(hipMemcpyAsync(h->host + slot, h->scalars + slot, sizeof(double),
                         hipMemcpyDeviceToHost, s));
  DMG_HIP(hipStreamSynchronize(s));
  *out = h->host[slot];
  return DMG_OK;
}

// ||b||_2 over interior vertices into scalars[0..1]
dmg_status norm_b(dmg_hier* h, const double* b, hipStream_t s) {
  const Level& L = h->L[0];
  DMG_CHECK(launch_sq_partials(b, L.n(), L.nx, L.ny, h->partials, s));
  return launch_finalize(h->partials, h->scalars + 0, s);
}

// ||b - A u||_2 into scalars[slot..slot+1]
dmg_status norm_r(dmg_hier* h, const double* u, const double* b, int slot, hipStream_t s) {
  const Level& L = h->L[0];
  DMG_CHECK(launch_resid_sq_partials(L.S, u, b, L.nx, L.ny, h->partials, s));
  return launch_finalize(h->partials, h->scalars + slot, s);
}

// The repeated step of a float64 solve: one V-cycle and the new residual norm (slot 2).  When
// the finest level runs in the strip kernels, the norm comes from the last post kernel.
dmg_status step_fp64(dmg_hier* h, double* u, const double* b, hipStream_t s) {
  if (h->tail == 0) {
    DMG_CHECK(vcycle_impl<double>(h, u, b, s));
    return norm_r(h, u, b, 2, s);
  }
  DMG_CHECK(vcycle_impl<double>(h, u, b, s, h->partials));
  return launch_finalize(h->partials, h->scalars + 2, s, post_partials_count(h));
}

// The repeated step of float32 refinement: r32 = r/s, e = 0, inner fp32 cycles, x += s e,
// r = b - A x and its norm (slot 4).
dmg_status step_ir(dmg_hier* h, double* x, const double* b, hipStream_t s) {
  const Level& L = h->L[0];
  DMG_CHECK(launch_ir_scale(h->r64, h->scalars + 4, L.b32, L.n(), s));
  for (int k = 0; k < h->opts.inner_cycles; ++k)
    DMG_CHECK(vcycle_impl<float>(h, L.u32, L.b32, s, nullptr, k == 0));
  DMG_CHECK(launch_ir_update(x, L.u32, h->scalars + 4, L.n(), s));
  DMG_CHECK(launch_ir_residual(L.S, x, b, h->r64, L.nx, L.ny, h->partials, s));
  return launch_finalize(h->partials, h->scalars + 4, s);
}

void graph_reset(Graph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g = Graph{};
}

// Runs the solve step for (u, b) on stream s, through a captured graph when enabled.  The
// graph is re-captured when the arrays or the stream change.
dmg_status run_step(dmg_hier* h, int kind, double* u, const double* b, hipStream_t s) {
  auto step = [&]() { return kind == 0 ? step_fp64(h, u, b, s) : step_ir(h, u, b, s); };
  // the legacy default stream cannot be captured: run eagerly there
  if (!h->opts.use_graph || s == nullptr) return step();
  Graph& g = h->graph;
  if (!(g.exec && g.key_u == u && g.key_b == b && g.stream == s && g.kind == kind)) {
    graph_reset(g);
    DMG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    dmg_status st = step();
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (st != DMG_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return fail(DMG_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    g.graph = graph;
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      graph_reset(g);
      return fail(DMG_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    g.key_u = u;
    g.key_b = b;
    g.stream = s;
    g.kind = kind;
  }
  DMG_HIP(hipGraphLaunch(g.exec, s));
  return DMG_OK;
}

dmg_status setup_impl(dmg_hier* h, const double* S, hipStream_t s) {
  const size_t n0 = h->L[0].n();
  DMG_HIP(hipMemcpyAsync(h->L[0].S, S, 5 * n0 * sizeof(double), hipMemcpyDeviceToDevice, s));
  for (size_t l = 0; l + 1 < h->L.size(); ++l) {
    const Level& L = h->L[l];
    DMG_CHECK(launch_interp_weights(L.S, L.nx, L.ny, L.P, s));
    DMG_CHECK(launch_rap(L.S, L.P, L.nx, L.ny, h->L[l + 1].S, s));
  }
  const Level& C = h->L.back();
  DMG_CHECK(launch_coarse_factor(C.S, C.nx, C.ny, h->m_coarse, h->coarse_idx, h->chol, h->flag, s));
  if (h->opts.precision == DMG_FP32_IR) {
    for (size_t l = 0; l < h->L.size(); ++l) {
      const Level& L = h->L[l];
      DMG_CHECK(launch_cast(L.S, L.S32, 5 * L.n(), s));
      if (L.P) {
        const Level& Cn = h->L[l + 1];
        DMG_CHECK(launch_cast(L.P, L.P32, 8 * Cn.n(), s));
      }
    }
  }
  int flag = 0;
  DMG_HIP(hipMemcpyAsync(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, s));
  DMG_HIP(hipStreamSynchronize(s));
  if (flag) return fail(DMG_ERR_NOT_SPD, "coarsest-level Cholesky met a non-positive pivot");
  return DMG_OK;
}

}  // namespace
}  // namespace dmg

dmg_hier::~dmg_hier() {
  dmg::graph_reset(graph);
  if (host) (void)hipHostFree(host);
}

using namespace dmg;

extern "C" {

void dmg_default_options(dmg_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->nu_pre = 1;
  o->nu_post = 1;
  for (int k = 0; k < 4; ++k) {
    o->pre_order[k] = k;
    o->post_order[k] = 3 - k;
  }
  o->coarsest_n = 3;
  o->precision = DMG_FP64;
  o->inner_cycles = 1;
  o->use_graph = 1;
  o->tile_rows = 0;
}

const char* dmg_last_error(void) { return g_err; }

const char* dmg_version(void) { return "dmg 0.1 (gfx950)"; }

dmg_status dmg_assemble_stencil(const double* jac, const double* K, int32_t nx, int32_t ny,
                                double* S, hipStream_t stream) {
  clear_error();
  if (!jac || !K || !S) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  if (nx < 3 || ny < 3) return fail(DMG_ERR_DIMS, "grid dims must be >= 3 (got %d x %d)", nx, ny);
  if (long(nx) * long(ny) > (1L << 31))
    return fail(DMG_ERR_DIMS, "grid too large (%d x %d)", nx, ny);
  return launch_assemble(jac, K, nx, ny, S, stream);
}

dmg_status dmg_grad_K(const double* jac, const double* lambda, const double* u, int32_t nx,
                      int32_t ny, double* dK, hipStream_t stream) {
  clear_error();
  if (!jac || !lambda || !u || !dK) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  if (nx < 3 || ny < 3) return fail(DMG_ERR_DIMS, "grid dims must be >= 3 (got %d x %d)", nx, ny);
  return launch_grad_K(jac, lambda, u, nx, ny, dK, stream);
}

dmg_status dmg_workspace_bytes(int32_t nx, int32_t ny, const dmg_options* opts, size_t* bytes) {
  clear_error();
  if (!bytes) return fail(DMG_ERR_INVALID_ARG, "bytes pointer is null");
  dmg_options def;
  dmg_default_options(&def);
  const dmg_options& o = opts ? *opts : def;
  DMG_CHECK(check_options(&o));
  std::vector<std::pair<int, int>> dims;
  DMG_CHECK(level_dims(nx, ny, o.coarsest_n, dims));
  dmg_hier tmp;
  Arena a;
  carve(tmp, a, dims, o);
  *bytes = a.used;
  return DMG_OK;
}

dmg_status dmg_setup(const double* S, int32_t nx, int32_t ny, const dmg_options* opts,
                     void* workspace, size_t ws_bytes, hipStream_t stream, dmg_hier** out) {
  clear_error();
  if (!S || !out) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  *out = nullptr;
  dmg_options def;
  dmg_default_options(&def);
  const dmg_options& o = opts ? *opts : def;
  DMG_CHECK(check_options(&o));
  std::vector<std::pair<int, int>> dims;
  DMG_CHECK(level_dims(nx, ny, o.coarsest_n, dims));
  if (!workspace) return fail(DMG_ERR_WORKSPACE, "workspace pointer is null");
  if (reinterpret_cast<uintptr_t>(workspace) & 255)
    return fail(DMG_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  std::unique_ptr<dmg_hier> h(new (std::nothrow) dmg_hier);
  if (!h) return fail(DMG_ERR_INVALID_ARG, "out of host memory");
  h->opts = o;
  Arena sizing;
  carve(*h, sizing, dims, o);
  if (ws_bytes < sizing.used)
    return fail(DMG_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, sizing.used);
  Arena a;
  a.base = static_cast<char*>(workspace);
  a.cap = ws_bytes;
  carve(*h, a, dims, o);
  DMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->host), 16 * sizeof(double),
                        hipHostMallocDefault));
  DMG_CHECK(setup_impl(h.get(), S, stream));
  *out = h.release();
  return DMG_OK;
}

void dmg_destroy(dmg_hier* h) { delete h; }

dmg_status dmg_refresh(dmg_hier* h, const double* S, hipStream_t stream) {
  clear_error();
  if (!h || !S) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  return setup_impl(h, S, stream);
}

dmg_status dmg_sweep(dmg_hier* h, int32_t level, int32_t kind, double* u, const double* b,
                     hipStream_t stream) {
  clear_error();
  if (!h || !u || !b) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  if (level < 0 || level >= h->tail)
    return fail(DMG_ERR_INVALID_ARG, "level %d is not a strip-kernel level (0..%d)", level,
                h->tail - 1);
  if (kind != 0 && kind != 1) return fail(DMG_ERR_INVALID_ARG, "kind must be 0 or 1");
  const Level& L = h->L[level];
  const OrderParams pre = order_params(h->opts.pre_order), post = order_params(h->opts.post_order);
  if (kind == 0)
    return launch_pre<double>(L.cfg, L.S, u, L.t, b, L.P, h->L[level + 1].b, L.nx, L.ny, pre.pf,
                              pre.cA, pre.cB, stream);
  return launch_post<double>(L.cfg, L.S, u, L.t, b, L.P, h->L[level + 1].u, nullptr, L.nx, L.ny,
                             post.pf, post.cA, post.cB, stream);
}

dmg_status dmg_hier_level(const dmg_hier* h, int32_t level, int32_t* nx, int32_t* ny,
                          const double** S, const double** P) {
  clear_error();
  if (!h) return fail(DMG_ERR_INVALID_ARG, "null hierarchy");
  if (level < 0 || level >= int(h->L.size()))
    return fail(DMG_ERR_INVALID_ARG, "level %d out of range [0,%zu)", level, h->L.size());
  const Level& L = h->L[level];
  if (nx) *nx = L.nx;
  if (ny) *ny = L.ny;
  if (S) *S = L.S;
  if (P) *P = L.P;
  return DMG_OK;
}

dmg_status dmg_stats(const dmg_hier* h, int32_t* levels, double* gc, double* oc) {
  clear_error();
  if (!h) return fail(DMG_ERR_INVALID_ARG, "null hierarchy");
  double N = 0, N0 = 0, Z = 0, Z0 = 0;
  for (size_t l = 0; l < h->L.size(); ++l) {
    const double m = double(h->L[l].nx - 2) * double(h->L[l].ny - 2);
    const double mx = h->L[l].nx - 2, my = h->L[l].ny - 2;
    // nonzeros of a 9-point operator on an mx x my interior grid
    const double z = 9 * m - 6 * (mx + my) + 4;
    N += m;
    Z += z > 0 ? z : m;
    if (l == 0) {
      N0 = m;
      Z0 = z > 0 ? z : m;
    }
  }
  if (levels) *levels = int32_t(h->L.size());
  if (gc) *gc = N / N0;
  if (oc) *oc = Z / Z0;
  return DMG_OK;
}

dmg_status dmg_vcycle(dmg_hier* h, double* u, const double* b, hipStream_t stream) {
  clear_error();
  if (!h || !u || !b) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  return vcycle_impl<double>(h, u, b, stream);
}

dmg_status dmg_residual_norm(dmg_hier* h, const double* u, const double* b, double* norm,
                             hipStream_t stream) {
  clear_error();
  if (!h || !u || !b || !norm) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  DMG_CHECK(norm_r(h, u, b, 2, stream));
  return read_scalar(h, 3, norm, stream);
}

dmg_status dmg_solve(dmg_hier* h, double* u, const double* b, double rtol, int32_t max_iters,
                     int32_t* iters, double* relres, double* history, hipStream_t stream) {
  clear_error();
  if (!h || !u || !b) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  if (!(rtol >= 0.0) || max_iters < 0) return fail(DMG_ERR_INVALID_ARG, "bad rtol/max_iters");
  if (iters) *iters = 0;
  double bn = 0.0, rn = 0.0;
  DMG_CHECK(norm_b(h, b, stream));
  DMG_CHECK(read_scalar(h, 1, &bn, stream));
  if (!std::isfinite(bn)) return fail(DMG_ERR_NONFINITE, "right-hand side norm is not finite");
  if (bn == 0.0) {  // the solution of A u = 0 is u = 0
    DMG_CHECK(launch_fill<double>(u, 0.0, h->L[0].n(), stream));
    if (relres) *relres = 0.0;
    return DMG_OK;
  }
  const bool ir = h->opts.precision == DMG_FP32_IR;
  const int slot = ir ? 4 : 2;
  if (ir) {
    const Level& L = h->L[0];
    DMG_CHECK(launch_ir_residual(L.S, u, b, h->r64, L.nx, L.ny, h->partials, stream));
    DMG_CHECK(launch_finalize(h->partials, h->scalars + 4, stream));
  } else {
    DMG_CHECK(norm_r(h, u, b, 2, stream));
  }
  DMG_CHECK(read_scalar(h, slot + 1, &rn, stream));
  if (!std::isfinite(rn)) return fail(DMG_ERR_NONFINITE, "initial residual norm is not finite");
  const double target = rtol * bn;
  int k = 0;
  while (rn > target && k < max_iters) {
    DMG_CHECK(run_step(h, ir ? 1 : 0, u, b, stream));
    DMG_CHECK(read_scalar(h, slot + 1, &rn, stream));
    ++k;
    if (history) history[k - 1] = bn > 0 ? rn / bn : rn;
    if (!std::isfinite(rn)) {
      if (iters) *iters = k;
      return fail(DMG_ERR_NONFINITE, "residual norm became non-finite at step %d", k);
    }
  }
  if (iters) *iters = k;
  if (relres) *relres = bn > 0 ? rn / bn : rn;
  if (rn > target)
    return fail(DMG_ERR_NO_CONVERGENCE, "no convergence in %d steps (rel. residual %.3e)", k,
                bn > 0 ? rn / bn : rn);
  return DMG_OK;
}

}  // extern "C"
