// C-ABI entry points: validation, workspace carving, hierarchy setup, V-cycles and solve
// drivers (float64 and float32-in-float64 refinement), adjoint gradient, batched solves.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
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
  if (o->strip_kernel != 0 && o->strip_kernel != 1)
    return fail(DMG_ERR_INVALID_ARG, "strip_kernel must be 0 or 1");
  if (o->smoother < 0 || o->smoother > 3)
    return fail(DMG_ERR_INVALID_ARG, "smoother must be 0 (point), 1 (x-lines), 2 (y-lines) or 3");
  if (o->coarse_gemv != 0 && o->coarse_gemv != 1)
    return fail(DMG_ERR_INVALID_ARG, "coarse_gemv must be 0 or 1");
  return DMG_OK;
}

// Levels: an odd n coarsens to (n + 1) / 2, which keeps the boundaries aligned; coarsening stops
// at the first level with min(nx, ny) <= coarsest_n or with an even dimension, which is the
// coarsest (solved directly).  2^k + 1 dims coarsen down to 3; n = c 2^k + 1 (c odd) down to
// c + 1.
dmg_status level_dims(int nx, int ny, int coarsest_n, std::vector<std::pair<int, int>>& dims) {
  if (nx < 3 || ny < 3 || nx % 2 == 0 || ny % 2 == 0)
    return fail(DMG_ERR_DIMS, "grid dims %d x %d: each must be odd and >= 3", nx, ny);
  dims.clear();
  dims.emplace_back(nx, ny);
  for (;;) {
    const auto c = dims.back();
    if (std::min(c.first, c.second) <= coarsest_n || c.first % 2 == 0 || c.second % 2 == 0) break;
    dims.emplace_back((c.first + 1) / 2, (c.second + 1) / 2);
  }
  const auto& c = dims.back();
  if (std::max(c.first, c.second) > kTailMaxN)
    return fail(DMG_ERR_DIMS,
                "coarsest grid %d x %d is wider than %d points; use dims of the form c 2^k + 1 "
                "with a small odd c", c.first, c.second, kTailMaxN);
  const long m = long(c.first - 2) * long(c.second - 2);
  if (m > 4096)
    return fail(DMG_ERR_DIMS, "coarsest system has %ld unknowns (max 4096); lower coarsest_n", m);
  return DMG_OK;
}

// Launch shape of the strip kernels on an nx x ny level: enough workgroups to fill the chip
// with as few recomputed halo rows/columns as possible.  tile_rows overrides the segment height.
StripConfig default_strip_config(int nx, int ny, const dmg_options& o) {
  StripConfig c;
  c.wave = o.strip_kernel == 1;
  c.bw = (c.wave || nx < 257) ? 64 : 128;
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
  // the coarse tail takes the coarsest levels up to kTailMaxN whose float64 data fits in the
  // LDS of one workgroup (it always holds the coarsest level, or the dense level above it)
  const int lds = device_lds_limit();
  const int nl = int(dims.size());
  auto interior = [&](int l) { return (dims[l].first - 2) * (dims[l].second - 2); };
  // levels the tail kernel holds when it starts at `top`: down to the first level with at most
  // kDenseMax interior unknowns (solved by its dense matrix), else down to the coarsest
  auto shape = [&](int top, int* nlev, int* mm, int* dense) {
    *nlev = nl - top;
    *mm = interior(nl - 1);
    *dense = 0;
    for (int l = top; l < nl; ++l)
      if (interior(l) <= kDenseMax) {
        *nlev = l - top + 1;
        *mm = interior(l);
        *dense = 1;
        break;
      }
  };
  auto layout = [&](int top) {
    int nlev = 0, mm = 0, dense = 0;
    shape(top, &nlev, &mm, &dense);
    int nx[kMaxTail], ny[kMaxTail];
    for (int k = 0; k < nlev && k < kMaxTail; ++k) {
      nx[k] = dims[top + k].first;
      ny[k] = dims[top + k].second;
    }
    return std::make_pair(nlev, nlev > kMaxTail ? TailLayout{}
                                                : tail_layout(nx, ny, nlev, mm, int(sizeof(double)), dense, 1));
  };
  auto fits = [&](int top) {
    const auto t = layout(top);
    return t.first <= kMaxTail && t.second.bytes <= size_t(lds);
  };
  h.tail = nl - 1;
  while (h.tail > 0 && std::max(dims[h.tail - 1].first, dims[h.tail - 1].second) <= kTailMaxN &&
         fits(h.tail - 1))
    --h.tail;
  shape(h.tail, &h.tail_nlev, &h.tail_m, &h.tail_dense);
  // Below level 0 the tail levels' S, P and right-hand sides (and the dense matrix) are slots of
  // one block laid out as the tail kernel's LDS (see TailSpec::image); its iterate slots are
  // zeroed at setup.
  const TailLayout img = layout(h.tail).second;
  h.tail_img = nullptr;
  h.tail_img32 = nullptr;
  h.tail_img_n = 0;
  h.basis = nullptr;
  h.basis32 = nullptr;
  if (h.tail > 0) {
    h.tail_img_n = img.r;
    h.tail_img = a.take<double>(size_t(img.r));
    if (fp32) h.tail_img32 = a.take<float>(size_t(img.r));
  }
  auto slot = [](auto* base, int off) { return base ? base + off : nullptr; };
  h.gemv = 0;
  h.gbasis = h.gscratch = nullptr;
  h.gbasis32 = nullptr;
  if (o.coarse_gemv && h.tail > 0 && interior(h.tail) > kDenseMax &&
      interior(h.tail) <= kGemvMax) {
    const size_t mm = size_t(interior(h.tail)) * interior(h.tail);
    h.gemv = 1;
    h.gbasis = a.take<double>(mm);
    h.gscratch = a.take<double>(mm);
    if (fp32) h.gbasis32 = a.take<float>(mm);
  }
  if (h.tail_dense) {
    const size_t mm = size_t(h.tail_m) * h.tail_m;
    h.basis = h.tail > 0 ? slot(h.tail_img, img.B) : a.take<double>(mm);
    if (fp32) h.basis32 = h.tail > 0 ? slot(h.tail_img32, img.B) : a.take<float>(mm);
  }
  for (size_t l = 0; l < dims.size(); ++l) {
    Level& L = h.L[l];
    L.nx = dims[l].first;
    L.ny = dims[l].second;
    const size_t n = L.n();
    const int k = int(l) - h.tail;  // index within the tail kernel's levels
    const bool in_img = h.tail > 0 && k >= 0 && k < h.tail_nlev;
    const bool staged = in_img && k + 1 < h.tail_nlev;  // S and P of the tail's last level are not
    L.S = staged ? slot(h.tail_img, img.S[k]) : a.take<double>(5 * n);
    if (int(l) < h.tail || l == 0) L.Sp = a.take<double>(5 * n);
    if (int(l) < h.tail) {
      L.t = a.take<double>(n);
      if (fp32) {
        L.t32 = a.take<float>(n);
        L.Sp32 = a.take<float>(5 * n);
      }
    }
    if (l + 1 < dims.size() || (l == 0 && fp32)) L.r = a.take<double>(n);  // level 0: r = b - A x
    if (l + 1 < dims.size()) {
      const size_t nc = size_t(dims[l + 1].first) * dims[l + 1].second;
      L.P = staged ? slot(h.tail_img, img.P[k]) : a.take<double>(8 * nc);
      if (fp32) {
        L.P32 = staged ? slot(h.tail_img32, img.P[k]) : a.take<float>(8 * nc);
        L.r32 = a.take<float>(n);
      }
    }
    if (l > 0) {
      L.u = a.take<double>(n);
      L.b = in_img ? slot(h.tail_img, img.b[k]) : a.take<double>(n);
    }
    if (o.smoother != 0 && int(l) < h.tail) {
      L.lf = a.take<double>(4 * n);
      if (fp32) L.lf32 = a.take<float>(4 * n);
    }
    if (fp32) {
      if (int(l) >= h.tail || o.smoother != 0)
        L.S32 = staged ? slot(h.tail_img32, img.S[k]) : a.take<float>(5 * n);
      L.u32 = a.take<float>(n);
      L.b32 = in_img ? slot(h.tail_img32, img.b[k]) : a.take<float>(n);
    }
  }
  const auto& c = dims.back();
  h.m_coarse = (c.first - 2) * (c.second - 2);
  h.coarse_idx = a.take<int>(size_t(h.m_coarse));
  h.chol = a.take<double>(size_t(h.m_coarse) * h.m_coarse);
  // + the b-norm partials of a solve start and its counts of nonzero initial-iterate entries
  h.partials = a.take<double>(kMaxPartials + 2 * kReduceBlocks);
  for (size_t l = 0; l < dims.size(); ++l) {
    h.L[l].cfg = default_strip_config(dims[l].first, dims[l].second, o);
    h.L[l].cfg32 = h.L[l].cfgp = h.L[l].cfgp32 = h.L[l].cfg;
  }
  h.scalars = a.take<double>(16);
  h.flag = a.take<int>(16);
  h.hist = a.take<double>(kMaxHistory);
}

template <class T>
struct Prec;
template <>
struct Prec<double> {
  static const StripConfig& cfg(const Level& L) { return L.cfg; }
  static const StripConfig& cfgp(const Level& L) { return L.cfgp; }
  static double* t(const Level& L) { return L.t; }
  static const double* S(const Level& L) { return L.S; }
  static const double* Sp(const Level& L) { return L.Sp; }
  static const double* P(const Level& L) { return L.P; }
  static double* u(const Level& L) { return L.u; }
  static double* b(const Level& L) { return L.b; }
  static double* r(const Level& L) { return L.r; }
  static const double* img(const dmg_hier& h) { return h.tail_img; }
  static const double* basis(const dmg_hier& h) { return h.basis; }
  static const double* gbasis(const dmg_hier& h) { return h.gbasis; }
};
template <>
struct Prec<float> {
  static const StripConfig& cfg(const Level& L) { return L.cfg32; }
  static const StripConfig& cfgp(const Level& L) { return L.cfgp32; }
  static float* t(const Level& L) { return L.t32; }
  static const float* S(const Level& L) { return L.S32; }
  static const float* Sp(const Level& L) { return L.Sp32; }
  static const float* P(const Level& L) { return L.P32; }
  static float* u(const Level& L) { return L.u32; }
  static float* b(const Level& L) { return L.b32; }
  static float* r(const Level& L) { return L.r32; }
  static const float* img(const dmg_hier& h) { return h.tail_img32; }
  static const float* basis(const dmg_hier& h) { return h.basis32; }
  static const float* gbasis(const dmg_hier& h) { return h.gbasis32; }
};

}  // namespace

// Kernel arguments of a hierarchy's coarse tail: levels [tail, tail + tail_nlev), the top one's
// iterate and right-hand side at (u_top, b_top).
template <class T>
void tail_spec(const dmg_hier* h, T* u_top, const T* b_top, bool zero_top, const int* stop,
               TailSpec<T>* out) {
  using Pr = Prec<T>;
  TailSpec<T>& sp = *out;
  sp.nlev = h->tail_nlev;
  for (int k = 0; k < sp.nlev; ++k) {
    const Level& L = h->L[h->tail + k];
    sp.S[k] = Pr::S(L);
    sp.u[k] = k == 0 ? u_top : Pr::u(L);
    sp.b[k] = k == 0 ? const_cast<T*>(b_top) : Pr::b(L);
    sp.P[k] = Pr::P(L);
    sp.nx[k] = L.nx;
    sp.ny[k] = L.ny;
  }
  sp.zero_top = zero_top;
  sp.m = h->tail_dense ? h->tail_m : h->m_coarse;
  sp.idx = h->coarse_idx;
  sp.chol = h->chol;
  sp.dense = h->tail_dense;
  sp.B = Pr::basis(*h);
  for (int k = 0; k < 4; ++k) {
    sp.pre[k] = h->opts.pre_order[k];
    sp.post[k] = h->opts.post_order[k];
  }
  sp.nu_pre = h->opts.nu_pre;
  sp.nu_post = h->opts.nu_post;
  sp.smoother = h->opts.smoother;
  sp.stop = stop;
  sp.threads = h->tail_threads;
  const T* img = Pr::img(*h);
  if (img && h->tail > 0 && zero_top && b_top == Pr::b(h->L[h->tail])) {
    sp.image = img;
    sp.image_n = h->tail_img_n;
  }
}
template void tail_spec<double>(const dmg_hier*, double*, const double*, bool, const int*,
                                TailSpec<double>*);
template void tail_spec<float>(const dmg_hier*, float*, const float*, bool, const int*,
                               TailSpec<float>*);

namespace {

// The dense operator of the tail's last level (when it has one): the cycle from that level
// down, run on each of its interior unit vectors with the current options, in float64 (and
// rounded to float32 for the float tail).  Depends on the smoother, the colour orders and the
// sweep counts, so it is recomputed whenever one of them changes.
dmg_status compute_basis(dmg_hier* h, hipStream_t s) {
  if (!h->tail_dense) return DMG_OK;
  const int nl = int(h->L.size());
  const int c = h->tail + h->tail_nlev - 1;
  TailSpec<double> sp;
  sp.nlev = nl - c;
  for (int k = 0; k < sp.nlev; ++k) {
    const Level& L = h->L[c + k];
    sp.S[k] = L.S;
    sp.u[k] = L.u;
    sp.b[k] = L.b;
    sp.P[k] = L.P;
    sp.nx[k] = L.nx;
    sp.ny[k] = L.ny;
  }
  sp.zero_top = 1;
  sp.m = h->m_coarse;
  sp.idx = h->coarse_idx;
  sp.chol = h->chol;
  for (int k = 0; k < 4; ++k) {
    sp.pre[k] = h->opts.pre_order[k];
    sp.post[k] = h->opts.post_order[k];
  }
  sp.nu_pre = h->opts.nu_pre;
  sp.nu_post = h->opts.nu_post;
  sp.smoother = h->opts.smoother;
  sp.threads = 256;
  DMG_CHECK(launch_tail_basis(sp, h->basis, s));
  if (h->basis32)
    DMG_CHECK(launch_cast(h->basis, h->basis32, size_t(h->tail_m) * h->tail_m, s));
  return DMG_OK;
}

// The whole-GPU dense operator of the tail's top level (when gemv): the tail's cycle from that
// level down (with its own dense level) run on each interior unit vector, the stencils read in
// global memory so that several runs share a CU, then transposed to row-major.
dmg_status compute_gemv_basis(dmg_hier* h, hipStream_t s) {
  if (!h->gemv) return DMG_OK;
  const Level& Lt = h->L[h->tail];
  const int m = (Lt.nx - 2) * (Lt.ny - 2);
  TailSpec<double> sp;
  tail_spec<double>(h, Lt.u, Lt.b, true, nullptr, &sp);
  sp.image = nullptr;
  sp.image_n = 0;
  sp.unstaged = 1;
  sp.threads = 256;  // measured fastest for the 961 runs of 33 x 33 (128: +10%, 512: +30%)
  DMG_CHECK(launch_tail_basis(sp, h->gscratch, s));
  DMG_CHECK(launch_transpose(h->gscratch, h->gbasis, m, s));
  if (h->gbasis32) DMG_CHECK(launch_cast(h->gbasis, h->gbasis32, size_t(m) * m, s));
  return DMG_OK;
}


// Strip-kernel colour-order parameters: row parity smoothed first and the column parity
// smoothed first on each row parity.
struct OrderParams {
  int pf, cA, cB;
};
OrderParams order_params(const int32_t* ord) {
  return OrderParams{ord[0] >> 1, ord[0] & 1, ord[2] & 1};
}

template <class T>
dmg_status tail_launch(dmg_hier* h, T* u_top, const T* b_top, hipStream_t s, bool u0_zero,
                       const int* stop) {
  TailSpec<T> sp;
  tail_spec<T>(h, u_top, b_top, h->tail > 0 || u0_zero, stop, &sp);
  return launch_tail<T>(sp, s);
}

// The cycle from the tail's top level down: its dense operator over the whole GPU (gemv), else
// the one-workgroup tail kernel.
template <class T>
dmg_status coarse_launch(dmg_hier* h, T* u_top, const T* b_top, hipStream_t s, bool u0_zero,
                         const int* stop) {
  using Pr = Prec<T>;
  if (h->gemv && h->tail > 0) {
    const Level& Lt = h->L[h->tail];
    return launch_dense<T>(DenseArgs<T>{Pr::gbasis(*h), b_top, u_top, Lt.nx, Lt.ny, stop}, s);
  }
  return tail_launch<T>(h, u_top, b_top, s, u0_zero, stop);
}

// One V-cycle in precision T with zebra line relaxation: unfused kernels on the levels above the
// coarse tail (coarse levels start from u = 0; u0_zero says the same of level 0), the tail levels
// with their line sweeps and the coarsest solve in the one-workgroup coarse kernel (or the dense
// coarse operator).  x64 (float cycles, nullable): x += *xscale u0 once the cycle is done.
template <class Tp>
dmg_status vcycle_line(dmg_hier* h, Tp* u0, const Tp* b0, bool u0_zero, const int* stop,
                       hipStream_t s, double* x64 = nullptr, const double* xscale = nullptr) {
  using Pr = Prec<Tp>;
  const dmg_options& o = h->opts;
  const int T = h->tail;
  auto U = [&](int l) { return l == 0 ? u0 : Pr::u(h->L[l]); };
  auto B = [&](int l) { return l == 0 ? b0 : static_cast<const Tp*>(Pr::b(h->L[l])); };
  for (int l = 0; l < T; ++l) {
    const Level& L = h->L[l];
    if (l > 0 || u0_zero) DMG_CHECK(launch_fill<Tp>(U(l), Tp(0), L.n(), s));
    for (int k = 0; k < o.nu_pre; ++k)
      DMG_CHECK(line_sweep<Tp>(L, U(l), B(l), o.smoother, true, stop, s));
    DMG_CHECK(line_resid_restrict<Tp>(L, h->L[l + 1], U(l), B(l), stop, s));
  }
  DMG_CHECK(coarse_launch<Tp>(h, U(T), B(T), s, T == 0 && u0_zero, stop));
  for (int l = T - 1; l >= 0; --l) {
    const Level& L = h->L[l];
    DMG_CHECK(line_prolong<Tp>(L, U(l + 1), U(l), stop, s));
    for (int k = 0; k < o.nu_post; ++k)
      DMG_CHECK(line_sweep<Tp>(L, U(l), B(l), o.smoother, false, stop, s));
  }
  if constexpr (std::is_same<Tp, float>::value) {
    if (x64) DMG_CHECK(launch_ir_update(x64, u0, h->L[0].n(), xscale, s, stop));
  }
  return DMG_OK;
}

// One V-cycle in precision T on level-0 arrays (u0, b0); coarse levels use hierarchy arrays.
// Levels above the tail: fused pre kernels on the way down (the first sweep of a coarse level
// starts from u = 0; u0_zero says the same of level 0), fused post kernels on the way up.  The
// strip kernels are out of place: each level alternates between its two iterate buffers and
// the cycle ends with the level-0 iterate back in u0.  partials (optional) receives the
// squared-residual partials of the final level-0 iterate.
// x64 (float cycles only, nullable): float64 iterate that receives the cycle's result scaled by
// the device scalar *xscale, x += s u0, fused into the last level-0 sweep.
template <class T>
dmg_status vcycle_impl(dmg_hier* h, T* u0, const T* b0, hipStream_t s, double* partials = nullptr,
                       bool u0_zero = false, const int* stop = nullptr, double* x64 = nullptr,
                       const double* xscale = nullptr) {
  using Pr = Prec<T>;
  const dmg_options& o = h->opts;
  if (o.smoother != 0) return vcycle_line<T>(h, u0, b0, u0_zero, stop, s, x64, xscale);
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
      DMG_CHECK(launch_pre<T>(Pr::cfg(L), Pr::Sp(L), src, dst, b, Pr::P(L), Pr::b(h->L[l + 1]), L.nx,
                              L.ny, pre.pf, pre.cA, pre.cB, stop, s));
      src = dst;
    }
    cur[l] = const_cast<T*>(src);
  }
  T* ut = h->tail == 0 ? u0 : Pr::u(h->L[h->tail]);
  const T* bt = h->tail == 0 ? b0 : Pr::b(h->L[h->tail]);
  DMG_CHECK(coarse_launch<T>(h, ut, bt, s, u0_zero, stop));
  const T* e = ut;
  for (int l = h->tail - 1; l >= 0; --l) {
    const Level& L = h->L[l];
    const T* b = l == 0 ? b0 : Pr::b(L);
    for (int k = 0; k < o.nu_post; ++k) {
      const bool first = k == 0, last = k + 1 == o.nu_post;  // prolongate once, norm once
      T* dst = other(l, cur[l]);
      DMG_CHECK(launch_post<T>(Pr::cfgp(L), Pr::Sp(L), cur[l], dst, b, Pr::P(L), first ? e : nullptr,
                               (l == 0 && last) ? partials : nullptr, L.nx, L.ny, post.pf, post.cA,
                               post.cB, stop, s, (l == 0 && last) ? x64 : nullptr, xscale));
      cur[l] = dst;
    }
    e = cur[l];
  }
  if (h->tail > 0 && cur[0] != u0)  // odd total sweep count: the iterate ends in the buffer
    DMG_CHECK(launch_copy<T>(cur[0], u0, h->L[0].n(), stop, s));
  if constexpr (std::is_same<T, float>::value) {
    if (x64 && h->tail == 0) DMG_CHECK(launch_ir_update(x64, u0, h->L[0].n(), xscale, s, stop));
  }
  return DMG_OK;
}

int post_partials_count(const dmg_hier* h) {
  const Level& L = h->L[0];
  int ns = 0, nseg = 0;
  return strip_blocks(L.nx, L.ny, L.cfgp.bw, L.cfgp.seg_h, &ns, &nseg);
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

// Device solve state: flag[4] = stop, flag[5] = steps done, flag[6] = max steps;
// scalars[6] = (rtol ||b||)^2.
int* stop_flag(dmg_hier* h) { return h->flag + 4; }
// flag[8]: set by a solve's start when the initial iterate is zero
int* zero_flag(dmg_hier* h) { return h->flag + 8; }

// The repeated step of a float64 solve: one V-cycle, then the residual norm of the new iterate
// (slot 2) and the convergence check.  When the finest level runs in the strip kernels, the
// norm partials come from the last post kernel.  Every kernel is a no-op once stop is set.
dmg_status step_fp64(dmg_hier* h, double* u, const double* b, hipStream_t s) {
  const int* stop = stop_flag(h);
  int count = kReduceBlocks;
  if (h->tail == 0 || h->opts.smoother != 0) {  // no fused post sweep carries the norm
    DMG_CHECK(vcycle_impl<double>(h, u, b, s, nullptr, false, stop));
    const Level& L = h->L[0];
    DMG_CHECK(launch_resid_sq_partials(L.S, u, b, L.nx, L.ny, h->partials, s, stop));
  } else {
    DMG_CHECK(vcycle_impl<double>(h, u, b, s, h->partials, false, stop));
    count = post_partials_count(h);
  }
  return launch_check_step(h->partials, count, h->scalars + 2, h->scalars, h->flag + 4, h->hist,
                           kMaxHistory, s);
}

// The repeated step of float32 refinement: r32 = fl32(r / s) with s = ||r||, e = 0, inner fp32
// cycles, x += s e, r = b - A x, its norm (slot 4) and the convergence check.
dmg_status step_ir(dmg_hier* h, double* x, const double* b, hipStream_t s) {
  // L.r holds r = b - A x of the current x and scalars[5] its norm s (from the previous step or
  // the solve's start).  The float cycles solve A e = r / s from e = 0; the last one adds s e
  // into x.  Dividing by ||r|| keeps r32 in float32's normal range whatever the scale of b.
  const int* stop = stop_flag(h);
  const Level& L = h->L[0];
  const int m = h->opts.inner_cycles;
  const double* norm = h->scalars + 5;
  DMG_CHECK(launch_ir_scale(L.r, L.b32, L.n(), norm, s, stop));
  for (int k = 0; k < m; ++k)
    DMG_CHECK(vcycle_impl<float>(h, L.u32, L.b32, s, nullptr, k == 0, stop, k + 1 == m ? x : nullptr,
                                 norm));
  DMG_CHECK(launch_ir_residual(L.Sp, x, b, L.r, L.nx, L.ny, h->partials, s, stop));
  return launch_check_step(h->partials, ir_residual_blocks(L.nx, L.ny), h->scalars + 4, h->scalars,
                           h->flag + 4, h->hist, kMaxHistory, s);
}

void graph_reset(Graph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g = Graph{};
}

void reset_solve_graphs(dmg_hier* h) {
  for (auto& g : h->graph) graph_reset(g);
  graph_reset(h->first_graph);
}

// The solve's start on the device: ||b|| and the initial residual's norm, the target and the
// solve state (no host synchronisation; a solve that is done at the start runs its first
// chunk of steps as skipped kernels).  The pass over b also tests whether u is zero; then the
// initial residual is b, and its pass reads neither the stencil nor u (same partials, same bits).
dmg_status solve_start(dmg_hier* h, int kind, double* u, const double* b, double rtol,
                       int max_iters, hipStream_t s) {
  const Level& L0 = h->L[0];
  const int slot = kind ? 4 : 2;
  double* pb = h->partials + kMaxPartials;
  double* nonzero = pb + kReduceBlocks;
  int* zero = zero_flag(h);
  DMG_CHECK(launch_start_norms(b, u, L0.nx, L0.ny, pb, nonzero, zero, s));
  int nr = kReduceBlocks;
  if (kind) {
    DMG_CHECK(launch_ir_residual(L0.Sp, u, b, L0.r, L0.nx, L0.ny, h->partials, s, nullptr, zero));
    nr = ir_residual_blocks(L0.nx, L0.ny);
  } else {
    DMG_CHECK(launch_resid_sq_partials(L0.S, u, b, L0.nx, L0.ny, h->partials, s, nullptr, zero, pb));
  }
  return launch_solve_start(pb, kReduceBlocks, h->partials, nr, h->scalars, h->scalars + slot,
                            h->flag + 4, rtol, max_iters, u, L0.n(), s);
}

// Runs len (1..kChunk) solve steps for (u, b) on stream s, preceded by the solve's start when
// `start` is set (then len = kChunk), through a captured graph when enabled (one per chunk
// length, and one for the start with the first chunk), re-captured when the arrays, the stream
// or the start's arguments change.
dmg_status run_step(dmg_hier* h, int kind, int len, double* u, const double* b, hipStream_t s,
                    bool start = false, double rtol = 0.0, int max_iters = 0) {
  auto step = [&]() -> dmg_status {
    if (start) DMG_CHECK(solve_start(h, kind, u, b, rtol, max_iters, s));
    for (int k = 0; k < len; ++k)
      DMG_CHECK(kind == 0 ? step_fp64(h, u, b, s) : step_ir(h, u, b, s));
    return DMG_OK;
  };
  // the legacy default stream cannot be captured: run eagerly there
  if (!h->opts.use_graph || s == nullptr) return step();
  Graph& g = start ? h->first_graph : h->graph[len - 1];
  if (!(g.exec && g.key_u == u && g.key_b == b && g.stream == s && g.kind == kind &&
        (!start || (g.rtol == rtol && g.max_iters == max_iters)))) {
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
    g.rtol = rtol;
    g.max_iters = max_iters;
  }
  DMG_HIP(hipGraphLaunch(g.exec, s));
  return DMG_OK;
}

// Mean duration (ms) of run() over `reps` back-to-back runs, timed on the device.  The runs are
// captured into one graph and replayed, so that host launch overhead (larger than a small
// level's kernels) neither enters the timing nor hides the difference between launch shapes;
// the legacy default stream cannot be captured and is timed with eager launches.
template <class F>
dmg_status time_runs(F&& run, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float* ms) {
  DMG_CHECK(run());  // warm-up, and the argument checks outside any capture
  hipGraphExec_t exec = nullptr;
  if (s != nullptr) {
    DMG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    dmg_status st = DMG_OK;
    for (int k = 0; k < reps && st == DMG_OK; ++k) st = run();
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st == DMG_OK && e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (st != DMG_OK) return st;
    if (e != hipSuccess) return fail(DMG_ERR_HIP, "timing graph failed: %s", hipGetErrorString(e));
  }
  auto once = [&]() -> hipError_t {
    if (exec) return hipGraphLaunch(exec, s);
    for (int k = 0; k < reps; ++k)
      if (run() != DMG_OK) return hipErrorLaunchFailure;
    return hipSuccess;
  };
  hipError_t e = once();  // uploads the graph
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess) e = once();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t_ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t_ms, e0, e1);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (e != hipSuccess) return fail(DMG_ERR_HIP, "kernel timing failed: %s", hipGetErrorString(e));
  *ms = t_ms / float(reps);
  return DMG_OK;
}

// Mean durations (ms) of `reps` pre launches and of `reps` post launches of level l in
// precision T with shape c.
template <class T>
dmg_status time_level(dmg_hier* h, int l, const StripConfig& c, int reps, hipStream_t s,
                      hipEvent_t e0, hipEvent_t e1, float* ms_pre, float* ms_post) {
  using Pr = Prec<T>;
  const Level& L = h->L[l];
  const OrderParams pre = order_params(h->opts.pre_order), post = order_params(h->opts.post_order);
  // level-shaped arrays whose contents do not matter; u, t (written) and b (read) distinct.
  // Level 0 has no u/b of its own: use the residual scratch and the stencil's first plane.
  T* u = l == 0 ? Pr::r(L) : Pr::u(L);
  T* t = Pr::t(L);
  const T* b = l == 0 ? Pr::Sp(L) : Pr::b(L);
  // the pre sweep in the form the cycle runs it: from the iterate on level 0, from zero on the
  // coarser levels (that kernel reads no iterate, and its best shape can differ)
  const T* uin = l == 0 ? u : nullptr;
  DMG_CHECK(time_runs([&]() {
    return launch_pre<T>(c, Pr::Sp(L), uin, t, b, Pr::P(L), Pr::b(h->L[l + 1]), L.nx, L.ny, pre.pf,
                         pre.cA, pre.cB, nullptr, s);
  }, reps, s, e0, e1, ms_pre));
  return time_runs([&]() {
    return launch_post<T>(c, Pr::Sp(L), t, u, b, Pr::P(L), Pr::u(h->L[l + 1]), nullptr, L.nx, L.ny,
                          post.pf, post.cA, post.cB, nullptr, s);
  }, reps, s, e0, e1, ms_post);
}

template <class T>
dmg_status tune_levels(dmg_hier* h, int reps, hipStream_t s) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  DMG_HIP(hipEventCreate(&e0));
  DMG_HIP(hipEventCreate(&e1));
  dmg_status st = DMG_OK;
  for (int l = 0; l < h->tail && st == DMG_OK; ++l) {
    Level& L = h->L[l];
    StripConfig best_pre = Prec<T>::cfg(L), best_post = Prec<T>::cfgp(L);
    float best_pre_ms = 1e30f, best_post_ms = 1e30f;
    for (int bw : {1, 64, 128, 256}) {  // 1: one-wavefront DPP strips (64 columns)
      if (bw == 256 && sizeof(T) == 8) continue;  // a 256-wide float64 ring exceeds 64 KiB of LDS
      for (int sh = 2; sh <= 128 && st == DMG_OK; sh *= 2) {
        int ns = 0, nseg = 0;
        StripConfig c;
        c.wave = bw == 1;
        c.bw = bw == 1 ? 64 : bw;
        c.seg_h = sh;
        if (strip_blocks(L.nx, L.ny, c.bw, sh, &ns, &nseg) > kMaxPartials) continue;
        float ms_pre = 0.f, ms_post = 0.f;
        st = time_level<T>(h, l, c, reps, s, e0, e1, &ms_pre, &ms_post);
        if (st == DMG_OK && ms_pre < best_pre_ms) {
          best_pre_ms = ms_pre;
          best_pre = c;
        }
        if (st == DMG_OK && ms_post < best_post_ms) {
          best_post_ms = ms_post;
          best_post = c;
        }
        if (sh * 2 > L.ny + 1) break;
      }
    }
    if (sizeof(T) == 8) {
      L.cfg = best_pre;
      L.cfgp = best_post;
    } else {
      L.cfg32 = best_pre;
      L.cfgp32 = best_post;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// Second tuning pass, in the cycle itself: for each strip level and each sweep kind in turn,
// every launch shape is timed as a graph of `reps` whole V-cycles (u, b of level 0) with the
// other levels' shapes held, and the fastest is kept.  A kernel timed alone replays on data
// that stays in the caches; inside the cycle it competes with the other levels for them, which
// can favour another shape.
template <class T>
dmg_status refine_levels(dmg_hier* h, T* u, const T* b, int reps, hipStream_t s) {
  if (h->opts.smoother != 0 || h->tail == 0) return DMG_OK;  // no fused strip sweeps to shape
  hipEvent_t e0 = nullptr, e1 = nullptr;
  DMG_HIP(hipEventCreate(&e0));
  DMG_HIP(hipEventCreate(&e1));
  dmg_status st = DMG_OK;
  // the faster of two timings of `reps` cycles: a shape is kept only for a difference the
  // timing noise of one cycle graph does not produce
  auto cycles = [&](float* ms) {
    float t0 = 0.f, t1 = 0.f;
    DMG_CHECK(time_runs([&]() { return vcycle_impl<T>(h, u, b, s); }, reps, s, e0, e1, &t0));
    DMG_CHECK(time_runs([&]() { return vcycle_impl<T>(h, u, b, s); }, reps, s, e0, e1, &t1));
    *ms = std::min(t0, t1);
    return DMG_OK;
  };
  for (int l = 0; l < h->tail && st == DMG_OK; ++l) {
    Level& L = h->L[l];
    for (int kind = 0; kind < 2 && st == DMG_OK; ++kind) {
      StripConfig& cur = sizeof(T) == 8 ? (kind == 0 ? L.cfg : L.cfgp)
                                        : (kind == 0 ? L.cfg32 : L.cfgp32);
      StripConfig best = cur;
      float best_ms = 1e30f;
      st = cycles(&best_ms);
      for (int bw : {1, 64, 128, 256}) {
        if (bw == 256 && sizeof(T) == 8) continue;
        for (int sh = 2; sh <= 128 && st == DMG_OK; sh *= 2) {
          int ns = 0, nseg = 0;
          StripConfig c;
          c.wave = bw == 1;
          c.bw = bw == 1 ? 64 : bw;
          c.seg_h = sh;
          if (strip_blocks(L.nx, L.ny, c.bw, sh, &ns, &nseg) > kMaxPartials) continue;
          if (c.wave == best.wave && c.bw == best.bw && c.seg_h == best.seg_h) continue;
          cur = c;
          float ms = 0.f;
          st = cycles(&ms);
          if (st == DMG_OK && ms < best_ms) {
            best_ms = ms;
            best = c;
          }
          if (sh * 2 > L.ny + 1) break;
        }
      }
      cur = best;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// Picks the coarse-tail workgroup size by timing the tail alone on (u_top, b_top).
template <class T>
dmg_status tune_tail(dmg_hier* h, T* u_top, const T* b_top, int reps, hipStream_t s) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  DMG_HIP(hipEventCreate(&e0));
  DMG_HIP(hipEventCreate(&e1));
  dmg_status st = DMG_OK;
  int best = h->tail_threads;
  float best_ms = 1e30f;
  for (int nt : {256, 512, 1024}) {
    h->tail_threads = nt;
    float ms = 0.f;
    st = time_runs([&]() { return tail_launch<T>(h, u_top, b_top, s, true, nullptr); }, reps, s, e0,
                   e1, &ms);
    if (st != DMG_OK) break;
    if (ms < best_ms) {
      best_ms = ms;
      best = nt;
    }
  }
  h->tail_threads = best;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// first: the hierarchy's initial setup, which zeroes the tail image, waits for the setup and
// reports a non-positive coarsest pivot; otherwise a refresh, only enqueued (the next solve
// reports the pivot).  jac and K (with S null): the fine stencil is assembled from them straight
// into level 0, planar and point-major, in place of the copy of a caller's S.
dmg_status setup_impl(dmg_hier* h, const double* S, hipStream_t s, bool first,
                      const double* jac = nullptr, const double* K = nullptr) {
  const int nl = int(h->L.size());
  // levels from first_small down run their whole setup in one single-workgroup kernel
  int first_small = nl - 1;
  while (first_small > 0 && std::max(h->L[first_small - 1].nx, h->L[first_small - 1].ny) <= kSmallSetupN &&
         nl - (first_small - 1) <= kMaxTail + 1)
    --first_small;
  // the tail image's iterate (and unused right-hand side) slots are zero from the first setup
  // on (nothing writes them; a refresh rewrites only the S, P and dense-operator slots)
  if (first && h->tail_img) DMG_CHECK(launch_fill<double>(h->tail_img, 0.0, size_t(h->tail_img_n), s));
  if (first && h->tail_img32) DMG_CHECK(launch_fill<float>(h->tail_img32, 0.f, size_t(h->tail_img_n), s));
  if (jac)
    DMG_CHECK(launch_assemble(jac, K, h->L[0].nx, h->L[0].ny, h->L[0].S, s, h->L[0].Sp));
  else
    DMG_CHECK(launch_copy_pack(S, h->L[0].S, h->L[0].Sp, h->L[0].n(), s));
  for (int l = 0; l < first_small; ++l) {
    const Level& L = h->L[l];
    DMG_CHECK(launch_interp_weights(L.S, L.nx, L.ny, L.P, s));
    DMG_CHECK(launch_rap(L.S, L.P, L.nx, L.ny, h->L[l + 1].S, h->L[l + 1].Sp, s));
  }
  SmallSetup ss;
  ss.nlev = nl - first_small;
  for (int k = 0; k < ss.nlev; ++k) {
    const Level& L = h->L[first_small + k];
    ss.S[k] = L.S;
    ss.Sp[k] = L.Sp;
    ss.P[k] = L.P;
    ss.nx[k] = L.nx;
    ss.ny[k] = L.ny;
  }
  ss.m = h->m_coarse;
  ss.idx = h->coarse_idx;
  ss.chol = h->chol;
  ss.flag = h->flag;
  DMG_CHECK(launch_setup_small(ss, s));
  if (h->opts.precision == DMG_FP32_IR) {  // the float32 copies, in one launch
    F32Batch fb;
    for (int l = 0; l < nl; ++l) {
      const Level& L = h->L[l];
      if (fb.count + 3 > kMaxF32Segs) {
        DMG_CHECK(launch_f32_batch(fb, s));
        fb.count = 0;
      }
      if (L.Sp32) DMG_CHECK(fb.add(L.S, L.Sp32, L.n(), 1));
      if (L.S32) DMG_CHECK(fb.add(L.S, L.S32, 5 * L.n(), 0));
      if (L.P && L.P32) DMG_CHECK(fb.add(L.P, L.P32, 8 * h->L[l + 1].n(), 0));
    }
    DMG_CHECK(launch_f32_batch(fb, s));
  }
  if (h->opts.smoother != 0)
    for (int l = 0; l < h->tail; ++l) {
      DMG_CHECK(line_factors<double>(h->L[l], s));
      if (h->opts.precision == DMG_FP32_IR) DMG_CHECK(line_factors<float>(h->L[l], s));
    }
  DMG_CHECK(compute_basis(h, s));
  DMG_CHECK(compute_gemv_basis(h, s));
  if (!first) return DMG_OK;
  int flag = 0;
  DMG_HIP(hipMemcpyAsync(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, s));
  DMG_HIP(hipStreamSynchronize(s));
  if (flag) return fail(DMG_ERR_NOT_SPD, "coarsest-level Cholesky met a non-positive pivot");
  return DMG_OK;
}

}  // namespace

// New colour orders for a hierarchy: the dense coarse operators carry the orders, so they are
// rebuilt, and graphs captured with the old ones are dropped.
dmg_status set_colour_orders(dmg_hier* h, const int32_t* pre, const int32_t* post, hipStream_t s) {
  for (int k = 0; k < 4; ++k) {
    h->opts.pre_order[k] = pre[k];
    h->opts.post_order[k] = post[k];
  }
  reset_solve_graphs(h);
  graph_reset(h->setup_graph);
  h->last_refresh_S = nullptr;
  h->last_refresh_K = nullptr;
  DMG_CHECK(compute_basis(h, s));
  return compute_gemv_basis(h, s);
}

dmg_status grid_vcycle(dmg_hier* h, double* u, const double* b, bool u_zero, const int* stop,
                       hipStream_t s) {
  return vcycle_impl<double>(h, u, b, s, nullptr, u_zero, stop);
}

}  // namespace dmg

dmg_hier::~dmg_hier() {
  for (auto& g : graph) dmg::graph_reset(g);
  dmg::graph_reset(first_graph);
  dmg::graph_reset(setup_graph);
  if (host) (void)hipHostFree(host);
}

using namespace dmg;

// ---- scratch of the allocation-free residual norm ------------------------------------------
// dmg_residual_norm_noalloc keeps its kReduceBlocks reduction partials (8 KiB) in this file-scope
// device array; every device that runs it holds its own copy until the process ends.  In host
// code the name is only a host-side stand-in: the array's device address is taken once per device
// with hipGetSymbolAddress (that device current) and only that address reaches kernels.
static __device__ __align__(256) double scratch[kReduceBlocks];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_addr[kMaxScratchDevices] = {};

// The current device's address of `scratch`, looked up on this device's first call.
dmg_status scratch_address(double** out) {
  int dev = -1;
  DMG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(DMG_ERR_INVALID_ARG, "device index %d beyond the %d the scratch table covers", dev,
                kMaxScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DMG_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_addr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_addr[dev];
  return DMG_OK;
}
}  // namespace

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
  o->strip_kernel = 1;
  o->coarse_gemv = 1;
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
  DMG_CHECK(setup_impl(h.get(), S, stream, true));
  *out = h.release();
  return DMG_OK;
}

void dmg_destroy(dmg_hier* h) { delete h; }

}  // extern "C"

namespace {

// A refresh from the stencil S, or (S null) from the coefficients (jac, K).  From the second
// consecutive refresh from the same arrays on the same stream, the setup is captured once and
// replayed (its ~25 small launches are otherwise paced by the host).
dmg_status refresh_impl(dmg_hier* h, const double* S, const double* jac, const double* K,
                        hipStream_t stream) {
  const void* key = S ? static_cast<const void*>(S) : static_cast<const void*>(jac);
  const void* key2 = S ? nullptr : static_cast<const void*>(K);
  // the legacy default stream cannot be captured
  if (!h->opts.use_graph || stream == nullptr) return setup_impl(h, S, stream, false, jac, K);
  Graph& g = h->setup_graph;
  if (g.exec && g.key_u == key && g.key_b == key2 && g.stream == stream) {
    DMG_HIP(hipGraphLaunch(g.exec, stream));
    return DMG_OK;
  }
  const bool again = h->last_refresh_S == key && h->last_refresh_K == key2 &&
                     h->last_refresh_stream == stream;
  h->last_refresh_S = key;
  h->last_refresh_K = key2;
  h->last_refresh_stream = stream;
  graph_reset(g);
  if (!again) return setup_impl(h, S, stream, false, jac, K);
  DMG_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  const dmg_status st = setup_impl(h, S, stream, false, jac, K);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(stream, &graph);
  if (st != DMG_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail(DMG_ERR_HIP, "setup capture failed: %s", hipGetErrorString(e));
  g.graph = graph;
  e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    graph_reset(g);
    return fail(DMG_ERR_HIP, "setup graph instantiate failed: %s", hipGetErrorString(e));
  }
  g.key_u = key;
  g.key_b = key2;
  g.stream = stream;
  DMG_HIP(hipGraphLaunch(g.exec, stream));
  return DMG_OK;
}

}  // namespace

extern "C" {

dmg_status dmg_refresh(dmg_hier* h, const double* S, hipStream_t stream) {
  clear_error();
  if (!h || !S) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  return refresh_impl(h, S, nullptr, nullptr, stream);
}

dmg_status dmg_refresh_assembled(dmg_hier* h, const double* jac, const double* K,
                                 hipStream_t stream) {
  clear_error();
  if (!h || !jac || !K) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  return refresh_impl(h, nullptr, jac, K, stream);
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
    return launch_pre<double>(L.cfg, L.Sp, u, L.t, b, L.P, h->L[level + 1].b, L.nx, L.ny, pre.pf,
                              pre.cA, pre.cB, nullptr, stream);
  return launch_post<double>(L.cfgp, L.Sp, u, L.t, b, L.P, h->L[level + 1].u, nullptr, L.nx, L.ny,
                             post.pf, post.cA, post.cB, nullptr, stream);
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

dmg_status dmg_hier_config(const dmg_hier* h, int32_t level, int32_t* bw, int32_t* seg_h,
                           int32_t* pre_order, int32_t* post_order) {
  clear_error();
  if (!h) return fail(DMG_ERR_INVALID_ARG, "null hierarchy");
  if (level < 0 || level >= int(h->L.size()))
    return fail(DMG_ERR_INVALID_ARG, "level %d out of range", level);
  const bool strip = level < h->tail;
  if (bw) *bw = strip ? (h->L[level].cfg.wave ? 1 : h->L[level].cfg.bw) : 0;
  if (seg_h) *seg_h = strip ? h->L[level].cfg.seg_h : 0;
  for (int k = 0; k < 4; ++k) {
    if (pre_order) pre_order[k] = h->opts.pre_order[k];
    if (post_order) post_order[k] = h->opts.post_order[k];
  }
  return DMG_OK;
}

dmg_status dmg_hier_inner_cycles(const dmg_hier* h, int32_t* inner_cycles) {
  clear_error();
  if (!h || !inner_cycles) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  *inner_cycles = h->opts.inner_cycles;
  return DMG_OK;
}

dmg_status dmg_hier_sweep_config(const dmg_hier* h, int32_t level, int32_t kind, int32_t* bw,
                                 int32_t* seg_h) {
  clear_error();
  if (!h) return fail(DMG_ERR_INVALID_ARG, "null hierarchy");
  if (level < 0 || level >= int(h->L.size()))
    return fail(DMG_ERR_INVALID_ARG, "level %d out of range", level);
  if (kind != 0 && kind != 1) return fail(DMG_ERR_INVALID_ARG, "kind must be 0 or 1");
  const bool strip = level < h->tail;
  const StripConfig& c = kind == 0 ? h->L[level].cfg : h->L[level].cfgp;
  if (bw) *bw = strip ? (c.wave ? 1 : c.bw) : 0;
  if (seg_h) *seg_h = strip ? c.seg_h : 0;
  return DMG_OK;
}

dmg_status dmg_autotune(dmg_hier* h, double* u, const double* b, int32_t flags, int32_t reps,
                        hipStream_t stream) {
  clear_error();
  if (!h || !u || !b) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  if (reps < 1 || reps > 1000) return fail(DMG_ERR_INVALID_ARG, "reps must be in [1,1000]");
  reset_solve_graphs(h);
  graph_reset(h->setup_graph);  // its dense-operator runs carry the colour orders
  h->last_refresh_S = nullptr;
  h->last_refresh_K = nullptr;
  if (flags & 1) {
    DMG_CHECK(tune_levels<double>(h, reps, stream));
    Level& T0 = h->L[h->tail];
    if (h->opts.precision == DMG_FP32_IR) {
      DMG_CHECK(tune_levels<float>(h, reps, stream));
      DMG_CHECK(tune_tail<float>(h, T0.u32, T0.b32, reps, stream));
    } else if (!h->gemv) {  // with the dense coarse operator the tail kernel does not run
      DMG_CHECK(tune_tail<double>(h, h->tail == 0 ? u : T0.u, h->tail == 0 ? b : T0.b, reps, stream));
    }
    DMG_CHECK(launch_fill<double>(u, 0.0, h->L[0].n(), stream));
    DMG_CHECK(refine_levels<double>(h, u, b, std::max(4, reps), stream));
    if (h->opts.precision == DMG_FP32_IR) {
      const Level& L0 = h->L[0];
      DMG_CHECK(launch_fill<float>(L0.u32, 0.f, L0.n(), stream));
      DMG_CHECK(launch_cast(b, L0.b32, L0.n(), stream));
      DMG_CHECK(refine_levels<float>(h, L0.u32, L0.b32, std::max(4, reps), stream));
    }
  }
  if (flags & 2) {
    static const int32_t cand[4][4] = {{0, 1, 2, 3}, {1, 0, 3, 2}, {2, 3, 0, 1}, {3, 2, 1, 0}};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    DMG_HIP(hipEventCreate(&e0));
    DMG_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    int best = -1;
    const dmg_options saved = h->opts;
    for (int c = 0; c < 4; ++c) {
      for (int k = 0; k < 4; ++k) {
        h->opts.pre_order[k] = cand[c][k];
        h->opts.post_order[k] = cand[c][3 - k];
      }
      reset_solve_graphs(h);
      DMG_CHECK(compute_basis(h, stream));
      DMG_CHECK(compute_gemv_basis(h, stream));
      float total = 0.f;
      dmg_status st = DMG_OK;
      for (int r = 0; r < std::max(1, reps / 4) && st == DMG_OK; ++r) {
        DMG_CHECK(launch_fill<double>(u, 0.0, h->L[0].n(), stream));
        DMG_HIP(hipEventRecord(e0, stream));
        int32_t it = 0;
        st = dmg_solve(h, u, b, 1e-10, 500, &it, nullptr, nullptr, stream);
        DMG_HIP(hipEventRecord(e1, stream));
        DMG_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        DMG_HIP(hipEventElapsedTime(&ms, e0, e1));
        total += ms;
      }
      if (st == DMG_OK && total < best_ms) {
        best_ms = total;
        best = c;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->opts = saved;
    if (best >= 0)
      for (int k = 0; k < 4; ++k) {
        h->opts.pre_order[k] = cand[best][k];
        h->opts.post_order[k] = cand[best][3 - k];
      }
    reset_solve_graphs(h);
    clear_error();
    DMG_CHECK(compute_basis(h, stream));  // for the order kept
    DMG_CHECK(compute_gemv_basis(h, stream));
  }
  if ((flags & 4) && h->opts.precision == DMG_FP32_IR) {
    // float32 cycles per refinement step: more cycles per float64 residual trade cheap float
    // work against the float64 residual pass; keep the count with the fastest solve (float32
    // rounding caps what one step can reach at ~1e-7, so 1e-10 needs at least two steps and
    // counts beyond 8 only add cycles)
    hipEvent_t e0 = nullptr, e1 = nullptr;
    DMG_HIP(hipEventCreate(&e0));
    DMG_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    int best = h->opts.inner_cycles;
    dmg_status st = DMG_OK;
    for (int m = 1; m <= 8 && st == DMG_OK; ++m) {
      h->opts.inner_cycles = m;
      reset_solve_graphs(h);
      float total = 0.f;
      for (int r = 0; r < 3 && st == DMG_OK; ++r) {  // the first captures the graph: untimed
        st = launch_fill<double>(u, 0.0, h->L[0].n(), stream);
        if (st == DMG_OK && hipEventRecord(e0, stream) != hipSuccess) st = fail(DMG_ERR_HIP, "event");
        int32_t it = 0;
        if (st == DMG_OK) st = dmg_solve(h, u, b, 1e-10, 500, &it, nullptr, nullptr, stream);
        float ms = 0.f;
        if (st == DMG_OK && (hipEventRecord(e1, stream) != hipSuccess ||
                             hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          st = fail(DMG_ERR_HIP, "event timing failed");
        if (r > 0) total += ms;
      }
      if (st == DMG_OK && total < best_ms) {
        best_ms = total;
        best = m;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->opts.inner_cycles = best;
    reset_solve_graphs(h);
    if (st != DMG_OK) return st;
  }
  return DMG_OK;
}

dmg_status dmg_residual_norm(dmg_hier* h, const double* u, const double* b, double* norm,
                             hipStream_t stream) {
  clear_error();
  if (!h || !u || !b || !norm) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  DMG_CHECK(norm_r(h, u, b, 2, stream));
  return read_scalar(h, 3, norm, stream);
}

dmg_status dmg_residual_norm_noalloc(const double* S, const double* u, const double* b, int32_t nx,
                                     int32_t ny, double* norm, hipStream_t stream) {
  clear_error();
  if (!S || !u || !b || !norm) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  if (nx < 3 || ny < 3) return fail(DMG_ERR_DIMS, "grid dims must be >= 3 (got %d x %d)", nx, ny);
  double* partials = nullptr;
  DMG_CHECK(scratch_address(&partials));
  // the partials kernel writes every one of the kReduceBlocks entries: nothing to clear first
  DMG_CHECK(launch_resid_sq_partials(S, u, b, nx, ny, partials, stream));
  return launch_finalize(partials, norm, stream, kReduceBlocks);
}

dmg_status dmg_solve(dmg_hier* h, double* u, const double* b, double rtol, int32_t max_iters,
                     int32_t* iters, double* relres, double* history, hipStream_t stream) {
  clear_error();
  if (!h || !u || !b) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  if (!(rtol >= 0.0) || max_iters < 0) return fail(DMG_ERR_INVALID_ARG, "bad rtol/max_iters");
  if (iters) *iters = 0;
  const bool ir = h->opts.precision == DMG_FP32_IR;
  const int slot = ir ? 4 : 2;
  int* hs = reinterpret_cast<int*>(h->host + 8);  // device flags [0..8): pivot, -, -, -, stop, steps
  double* hsc = h->host;  // scalars [0..7]
  // The start and the first kChunk steps run as one graph, then the host synchronises.  From
  // then on the rate per step (from the initial residual norm, then from the previous
  // synchronisation) predicts the steps left: that many are enqueued as back-to-back chunk
  // graphs (up to kAhead steps) before the next synchronisation.  A step beyond convergence
  // still costs its launches, and the device stopping test makes any count exact.
  constexpr int kAhead = 4 * kChunk;
  int todo = kChunk, prev_k = -1;
  double prev_rn = 0.0;
  for (bool first = true;; first = false) {
    for (int done = 0; done < todo;) {
      const int len = first ? kChunk : std::min(kChunk, todo - done);
      DMG_CHECK(run_step(h, ir ? 1 : 0, len, u, b, stream, first && done == 0, rtol, max_iters));
      done += len;
    }
    DMG_HIP(hipMemcpyAsync(hs, h->flag, 8 * sizeof(int), hipMemcpyDeviceToHost, stream));
    DMG_HIP(hipMemcpyAsync(hsc, h->scalars, 8 * sizeof(double), hipMemcpyDeviceToHost, stream));
    DMG_HIP(hipStreamSynchronize(stream));
    if (hs[4] || hs[0]) break;
    const int k_now = hs[5];
    const double rn = hsc[slot + 1], target = std::sqrt(std::max(hsc[6], 0.0));
    if (prev_k < 0) {  // first synchronisation: measure from the start's residual
      prev_k = 0;
      prev_rn = hsc[7];
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
  // a refresh does not wait for its setup: its coarsest factorisation is checked here
  if (hs[0]) return fail(DMG_ERR_NOT_SPD, "coarsest-level Cholesky met a non-positive pivot");
  const int k = hs[5];
  const double bn = hsc[1], rn = hsc[slot + 1];
  if (!std::isfinite(bn)) return fail(DMG_ERR_NONFINITE, "right-hand side norm is not finite");
  if (bn == 0.0) {  // u was set to 0, the solution of A u = 0
    if (relres) *relres = 0.0;
    return DMG_OK;
  }
  if (history && k > 0)
    DMG_HIP(hipMemcpy(history, h->hist, size_t(std::min(k, kMaxHistory)) * sizeof(double),
                      hipMemcpyDeviceToHost));
  if (iters) *iters = k;
  if (relres) *relres = rn / bn;
  if (!std::isfinite(rn))
    return fail(DMG_ERR_NONFINITE, k > 0 ? "residual norm became non-finite at step %d"
                                         : "initial residual norm is not finite", k);
  if (rn > rtol * bn)
    return fail(DMG_ERR_NO_CONVERGENCE, "no convergence in %d steps (rel. residual %.3e)", k,
                rn / bn);
  return DMG_OK;
}

}  // extern "C"
