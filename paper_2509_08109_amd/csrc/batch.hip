// Batched solves of independent instances (uneven sizes).  Every instance's hierarchy is carved
// out of one caller workspace.  One batched V-cycle launches each fused sweep once per level
// size, over the tiles of every instance that has a level of that size: largest size first on
// the way down and smallest first on the way up, which keeps each instance's own level order.
// Then come the coarse tails (one workgroup per instance) and the convergence checks (one
// workgroup per instance).  Four such steps are captured in one hipGraph and replayed until
// every instance has stopped; each instance has its own stop flag, so the tiles of converged
// instances exit at once.  Results equal bitwise those of dmg_solve on each instance alone with
// one-wavefront sweeps and coarse_gemv = 0 (the wave sweeps, the tail and the check do the same
// arithmetic, and segment heights change no bit).  With line relaxation the levels above the
// tails run the unfused line steps instead, each launched once per level size over its
// instances (one argument list per level size serves every step: the sweeps are in place),
// and the residual norms come from a per-instance norm kernel.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

#include "dmg_internal.h"

namespace {

constexpr int kNormBlocks = 64;     // workgroups per instance for the starting norms
constexpr size_t kArgAlign = 256;   // alignment of each argument list in the argument buffer

struct Launch {
  enum Kind { WAVE, TAIL, DENSE, RESID, CHECK, LINE } kind;
  int mode = 0;        // WAVE: 1 pre, 2 post with prolongation, 3 post
  int count = 0;       // instances (list length)
  int tiles_per = 0;   // WAVE: tiles per instance; DENSE: largest interior unknown count
  size_t off = 0;      // byte offset of the list in the device argument buffer
  size_t lds = 0;      // TAIL: LDS bytes
  dmg::LineStep step = dmg::LineStep::kSweep;  // LINE: which step, on which lines, at which size
  int dir = 0, parity = 0, nx = 0, ny = 0;
  int pf = 0;  // WAVE: the row parity smoothed first (one per launch)
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct dmg_batch {
  dmg_options opts;
  std::vector<dmg_hier*> inst;
  int* state = nullptr;           // [count][4] device: stop, steps, max steps, unused
  double* summary = nullptr;      // [count][2] device: ||b||, starting ||r||
  double* rel = nullptr;          // [count] device: final relative residual
  int* steps = nullptr;           // [count] device: steps taken
  double* npart = nullptr;        // [count][kNormBlocks][2] device
  unsigned char* args = nullptr;  // device argument lists
  size_t args_cap = 0;
  int tail_threads = 256;
  std::map<std::pair<int, int>, int> seg_h;  // wave-strip rows per segment, per level size
  // schedule for the current arrays
  std::vector<Launch> step;
  size_t norm_off = 0, check_off = 0;
  std::vector<const void*> key;
  double key_rtol = -1.0;
  int key_max = -1;
  bool built = false;
  // graph of kChunk steps
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t gstream = nullptr;
  // pinned host mirrors
  int* h_state = nullptr;
  double* h_summary = nullptr;
  double* h_rel = nullptr;
  int* h_steps = nullptr;

  void reset_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    gstream = nullptr;
  }
  ~dmg_batch() {
    reset_graph();
    if (h_state) (void)hipHostFree(h_state);
    if (h_summary) (void)hipHostFree(h_summary);
    if (h_rel) (void)hipHostFree(h_rel);
    if (h_steps) (void)hipHostFree(h_steps);
    for (auto* h : inst) dmg_destroy(h);
  }
};

using namespace dmg;

namespace {

size_t args_capacity(int count, const dmg_options& o) {
  const size_t sweeps = size_t(o.nu_pre + o.nu_post);
  size_t per_inst = size_t(kMaxLevels) * sweeps * sizeof(StripArgs<double>) +
                    sizeof(TailArgs<double>) + sizeof(CheckArgs) + 2 * sizeof(NormArgs);
  size_t lists = size_t(count) * kMaxLevels * sweeps + 8;
  if (o.smoother != 0) {  // line cycles: per level size one list for every step, one for u = 0
    per_inst += 2 * size_t(kMaxLevels) * sizeof(LineArgs<double>);
    lists += 2 * size_t(count) * kMaxLevels;
  }
  return size_t(count) * per_inst + lists * kArgAlign;
}

// The line sweeps of one pre-smoothing pass as (direction, parity), even lines first; the post
// pass runs them in reverse.
int line_seq(int smoother, int dir[4], int par[4]) {
  int n = 0;
  if (smoother == 1 || smoother == 3) {
    dir[n] = 0, par[n++] = 0;
    dir[n] = 0, par[n++] = 1;
  }
  if (smoother == 2 || smoother == 3) {
    dir[n] = 1, par[n++] = 0;
    dir[n] = 1, par[n++] = 1;
  }
  return n;
}

size_t batch_extra_bytes(int count, const dmg_options& o) {
  size_t b = 0;
  b += align_up(size_t(count) * 4 * sizeof(int), 256);
  b += align_up(size_t(count) * 2 * sizeof(double), 256);
  b += align_up(size_t(count) * sizeof(double), 256);
  b += align_up(size_t(count) * sizeof(int), 256);
  b += align_up(size_t(count) * kNormBlocks * 2 * sizeof(double), 256);
  b += align_up(args_capacity(count, o), 256);
  return b;
}

int tiles_of(int nx, int ny, int seg_h) {
  int ns = 0, nseg = 0;
  strip_blocks(nx, ny, 64, seg_h, &ns, &nseg);
  return ns * nseg;
}

// Default launch shape of one level size shared by `members` instances: the tallest segment that
// still gives >= 2048 tiles in the launch, within the per-instance partials capacity.
int default_seg_h(int nx, int ny, int members) {
  int h = 8;
  for (int c = 128; c >= 8; c >>= 1)
    if (long(members) * tiles_of(nx, ny, c) >= 2048) {
      h = c;
      break;
    }
  while (tiles_of(nx, ny, h) > kMaxPartials) h *= 2;
  return h;
}

struct OrderP {
  int pf, cA, cB;
};
OrderP order_of(const int32_t* ord) { return OrderP{ord[0] >> 1, ord[0] & 1, ord[2] & 1}; }

// Builds the argument lists and launch sequence of one batched step for arrays (u, b).
dmg_status build_schedule(dmg_batch* bt, double* const* u, const double* const* b, double rtol,
                          int32_t max_iters) {
  const int count = int(bt->inst.size());
  const dmg_options& o = bt->opts;
  std::vector<unsigned char> host(bt->args_cap);
  size_t used = 0;
  auto put = [&](const void* p, size_t n, size_t* off) -> dmg_status {
    const size_t at = align_up(used, kArgAlign);
    if (at + n > host.size()) return fail(DMG_ERR_WORKSPACE, "batch argument buffer too small");
    std::memcpy(host.data() + at, p, n);
    used = at + n;
    *off = at;
    return DMG_OK;
  };
  struct Sweep {
    const double* uin;
    double* u;
    const double* e;
    double* partials;
  };
  const bool line = o.smoother != 0;
  // per instance and strip level: the buffers of each pre and post sweep (as in one V-cycle)
  std::vector<std::vector<std::vector<Sweep>>> pre_sw(count), post_sw(count);
  for (int k = 0; k < count && !line; ++k) {
    dmg_hier* h = bt->inst[k];
    const int T = h->tail;
    double* u0 = u[k];
    auto other = [&](int l, const double* x) -> double* {
      double* a = l == 0 ? u0 : h->L[l].u;
      return x == a ? h->L[l].t : a;
    };
    std::vector<const double*> cur(size_t(T) + 1, nullptr);
    pre_sw[k].assign(size_t(T), {});
    post_sw[k].assign(size_t(T), {});
    for (int l = 0; l < T; ++l) {
      const double* src = l == 0 ? u0 : nullptr;
      for (int s = 0; s < o.nu_pre; ++s) {
        double* dst = src ? other(l, src) : h->L[l].t;
        pre_sw[k][l].push_back(Sweep{src, dst, nullptr, nullptr});
        src = dst;
      }
      cur[l] = src;
    }
    const double* e = T == 0 ? u0 : h->L[T].u;
    for (int l = T - 1; l >= 0; --l) {
      for (int s = 0; s < o.nu_post; ++s) {
        double* dst = other(l, cur[l]);
        const bool last = s + 1 == o.nu_post;
        post_sw[k][l].push_back(
            Sweep{cur[l], dst, s == 0 ? e : nullptr, (l == 0 && last) ? h->partials : nullptr});
        cur[l] = dst;
      }
      e = cur[l];
    }
    if (T > 0 && cur[0] != u0)
      return fail(DMG_ERR_UNSUPPORTED, "batched cycles need an even number of level-0 sweeps");
  }
  // level sizes, largest first
  std::map<std::tuple<long, int, int>, std::vector<std::pair<int, int>>, std::greater<>> groups;
  for (int k = 0; k < count; ++k)
    for (int l = 0; l < bt->inst[k]->tail; ++l) {
      const Level& L = bt->inst[k]->L[l];
      groups[{long(L.nx) * L.ny, L.nx, L.ny}].push_back({k, l});
    }
  std::vector<int> level0_tiles(count, 0);
  auto wave_list = [&](const std::vector<std::pair<int, int>>& mem, bool is_pre, int s,
                       Launch* out) -> dmg_status {
    std::vector<StripArgs<double>> list;
    int tiles_per = 0;
    for (auto [k, l] : mem) {
      dmg_hier* h = bt->inst[k];
      const Level& L = h->L[l];
      const Sweep& sw = is_pre ? pre_sw[k][l][s] : post_sw[k][l][s];
      StripArgs<double> a{};
      a.S = L.Sp;
      a.uin = sw.uin;
      a.u = sw.u;
      a.b = l == 0 ? b[k] : L.b;
      a.P = L.P;
      a.bH = is_pre ? h->L[l + 1].b : nullptr;
      a.e = sw.e;
      a.partials = sw.partials;
      a.nx = L.nx;
      a.ny = L.ny;
      a.seg_h = bt->seg_h[{L.nx, L.ny}];
      strip_blocks(L.nx, L.ny, 64, a.seg_h, &a.nstrips, &a.nsegs);
      // each instance's own colour orders (the batch tuner may give each size class its own)
      const OrderP op = order_of(is_pre ? h->opts.pre_order : h->opts.post_order);
      a.pf = op.pf;
      a.cA = op.cA;
      a.cB = op.cB;
      a.stop = bt->state + 4 * k;
      a.x64 = nullptr;
      tiles_per = a.nstrips * a.nsegs;
      if (l == 0) level0_tiles[k] = tiles_per;
      list.push_back(a);
    }
    out->kind = Launch::WAVE;
    out->count = int(list.size());
    out->tiles_per = tiles_per;
    out->pf = list.empty() ? 0 : list[0].pf;
    return put(list.data(), list.size() * sizeof(list[0]), &out->off);
  };
  // the members of a level size whose pre (post) order smooths row parity pf first: one wave
  // launch per parity, since the kernel takes it as a compile-time parameter
  auto by_pf = [&](const std::vector<std::pair<int, int>>& mem, bool is_pre, int pf) {
    std::vector<std::pair<int, int>> out;
    for (auto kl : mem) {
      const dmg_hier* h = bt->inst[kl.first];
      if (order_of(is_pre ? h->opts.pre_order : h->opts.post_order).pf == pf) out.push_back(kl);
    }
    return out;
  };
  // line cycles: every step of a level size reads one argument list (the sweeps are in place)
  std::map<std::tuple<long, int, int>, std::pair<size_t, size_t>> line_lists;  // (all, l > 0)
  std::map<std::tuple<long, int, int>, int> zero_count;
  if (line) {
    for (auto& [key, mem] : groups) {
      std::vector<LineArgs<double>> all, coarse;
      for (auto [k, l] : mem) {
        dmg_hier* h = bt->inst[k];
        const Level& L = h->L[l];
        LineArgs<double> a{};
        a.S = L.S;
        a.lf = L.lf;
        a.P = L.P;
        a.u = l == 0 ? u[k] : L.u;
        a.b = l == 0 ? b[k] : L.b;
        a.r = L.r;
        a.bH = h->L[l + 1].b;
        a.e = h->L[l + 1].u;
        a.nx = L.nx;
        a.ny = L.ny;
        a.stop = bt->state + 4 * k;
        all.push_back(a);
        if (l > 0) coarse.push_back(a);
      }
      size_t off_all = 0, off_coarse = 0;
      DMG_CHECK(put(all.data(), all.size() * sizeof(all[0]), &off_all));
      if (!coarse.empty()) DMG_CHECK(put(coarse.data(), coarse.size() * sizeof(coarse[0]), &off_coarse));
      line_lists[key] = {off_all, off_coarse};
      zero_count[key] = int(coarse.size());
    }
  }
  int ldir[4], lpar[4];
  const int nls = line ? line_seq(o.smoother, ldir, lpar) : 0;
  auto line_launch = [&](const std::tuple<long, int, int>& key, LineStep step, int dir, int par,
                         bool coarse_only) {
    Launch L;
    L.kind = Launch::LINE;
    L.step = step;
    L.dir = dir;
    L.parity = par;
    L.nx = std::get<1>(key);
    L.ny = std::get<2>(key);
    L.count = coarse_only ? zero_count[key] : int(groups[key].size());
    L.off = coarse_only ? line_lists[key].second : line_lists[key].first;
    return L;
  };
  std::vector<Launch> seq;
  for (auto& [key, mem] : groups) {
    if (line) {  // coarse levels start from 0; pre sweeps; residual; restriction
      if (zero_count[key] > 0) seq.push_back(line_launch(key, LineStep::kZero, 0, 0, true));
      for (int s = 0; s < o.nu_pre; ++s)
        for (int q = 0; q < nls; ++q)
          seq.push_back(line_launch(key, LineStep::kSweep, ldir[q], lpar[q], false));
      seq.push_back(line_launch(key, LineStep::kResidual, 0, 0, false));
      seq.push_back(line_launch(key, LineStep::kRestrict, 0, 0, false));
      continue;
    }
    for (int s = 0; s < o.nu_pre; ++s)
      for (int pf = 0; pf < 2; ++pf) {
        const auto part = by_pf(mem, true, pf);
        if (part.empty()) continue;
        Launch L;
        DMG_CHECK(wave_list(part, true, s, &L));
        L.mode = 1;
        seq.push_back(L);
      }
  }
  {  // coarse tails: the one-workgroup tail kernel, or the dense operator of the tail's top
    std::vector<TailArgs<double>> list;
    std::vector<DenseArgs<double>> dense;
    size_t lds = 0;
    int max_m = 0;
    for (int k = 0; k < count; ++k) {
      dmg_hier* h = bt->inst[k];
      const int T = h->tail;
      if (h->gemv) {
        const Level& Lt = h->L[T];
        dense.push_back(DenseArgs<double>{h->gbasis, Lt.b, Lt.u, Lt.nx, Lt.ny, bt->state + 4 * k});
        max_m = std::max(max_m, (Lt.nx - 2) * (Lt.ny - 2));
        continue;
      }
      TailSpec<double> sp;
      tail_spec<double>(h, T == 0 ? u[k] : h->L[T].u, T == 0 ? b[k] : h->L[T].b, T > 0,
                        bt->state + 4 * k, &sp);
      sp.threads = bt->tail_threads;
      size_t bytes = 0;
      list.emplace_back();
      DMG_CHECK(make_tail_args<double>(sp, &list.back(), &bytes));
      lds = std::max(lds, bytes);
    }
    if (!list.empty()) {
      Launch L;
      L.kind = Launch::TAIL;
      L.count = int(list.size());
      L.lds = lds;
      DMG_CHECK(put(list.data(), list.size() * sizeof(list[0]), &L.off));
      seq.push_back(L);
    }
    if (!dense.empty()) {
      Launch L;
      L.kind = Launch::DENSE;
      L.count = int(dense.size());
      L.tiles_per = max_m;
      DMG_CHECK(put(dense.data(), dense.size() * sizeof(dense[0]), &L.off));
      seq.push_back(L);
    }
  }
  for (auto it = groups.rbegin(); it != groups.rend(); ++it) {
    if (line) {  // interpolation, then the post sweeps in reverse
      seq.push_back(line_launch(it->first, LineStep::kProlong, 0, 0, false));
      for (int s = 0; s < o.nu_post; ++s)
        for (int q = nls - 1; q >= 0; --q)
          seq.push_back(line_launch(it->first, LineStep::kSweep, ldir[q], lpar[q], false));
      continue;
    }
    for (int s = 0; s < o.nu_post; ++s)
      for (int pf = 0; pf < 2; ++pf) {
        const auto part = by_pf(it->second, false, pf);
        if (part.empty()) continue;
        Launch L;
        DMG_CHECK(wave_list(part, false, s, &L));
        L.mode = s == 0 ? 2 : 3;
        seq.push_back(L);
      }
  }
  // per-instance norm arguments (starting norms; residual partials of all-tail instances)
  std::vector<NormArgs> norms(count), tail_only;
  for (int k = 0; k < count; ++k) {
    dmg_hier* h = bt->inst[k];
    const Level& L0 = h->L[0];
    norms[k] = NormArgs{L0.S, u[k], b[k], L0.nx, L0.ny, h->scalars, bt->state + 4 * k, rtol,
                        max_iters, h->partials};
    if (h->tail == 0 || line) tail_only.push_back(norms[k]);  // no fused sweep gives partials
  }
  if (!tail_only.empty()) {
    Launch L;
    L.kind = Launch::RESID;
    L.count = int(tail_only.size());
    DMG_CHECK(put(tail_only.data(), tail_only.size() * sizeof(NormArgs), &L.off));
    seq.push_back(L);
  }
  {
    std::vector<CheckArgs> list(count);
    for (int k = 0; k < count; ++k) {
      dmg_hier* h = bt->inst[k];
      list[k] = CheckArgs{h->partials, (h->tail > 0 && !line) ? level0_tiles[k] : kNormBlocks,
                          h->scalars + 2, h->scalars, bt->state + 4 * k, h->hist, kMaxHistory};
    }
    Launch L;
    L.kind = Launch::CHECK;
    L.count = count;
    DMG_CHECK(put(list.data(), list.size() * sizeof(CheckArgs), &L.off));
    bt->check_off = L.off;
    seq.push_back(L);
  }
  DMG_CHECK(put(norms.data(), norms.size() * sizeof(NormArgs), &bt->norm_off));
  DMG_HIP(hipMemcpy(bt->args, host.data(), used, hipMemcpyHostToDevice));
  bt->step = std::move(seq);
  bt->built = true;
  return DMG_OK;
}

dmg_status run_step(dmg_batch* bt, hipStream_t s) {
  for (const Launch& L : bt->step) {
    const unsigned char* p = bt->args + L.off;
    switch (L.kind) {
      case Launch::WAVE:
        DMG_CHECK(launch_wave_multi<double>(reinterpret_cast<const StripArgs<double>*>(p), L.count,
                                            L.tiles_per, L.mode, L.pf, s));
        break;
      case Launch::TAIL:
        DMG_CHECK(launch_tail_multi<double>(reinterpret_cast<const TailArgs<double>*>(p), L.count,
                                            L.lds, bt->tail_threads, s));
        break;
      case Launch::DENSE:
        DMG_CHECK(launch_dense_multi<double>(reinterpret_cast<const DenseArgs<double>*>(p), L.count,
                                             L.tiles_per, s));
        break;
      case Launch::RESID:
        DMG_CHECK(launch_resid_multi(reinterpret_cast<const NormArgs*>(p), L.count, kNormBlocks, s));
        break;
      case Launch::CHECK:
        DMG_CHECK(launch_check_multi(reinterpret_cast<const CheckArgs*>(p), L.count, s));
        break;
      case Launch::LINE:
        DMG_CHECK(launch_line_multi(L.step, reinterpret_cast<const LineArgs<double>*>(p), L.count,
                                    L.nx, L.ny, L.dir, L.parity, s));
        break;
    }
  }
  return DMG_OK;
}

// kChunk batched steps, through one captured graph when the stream allows capture.
dmg_status run_chunk(dmg_batch* bt, hipStream_t s) {
  auto steps = [&]() -> dmg_status {
    for (int k = 0; k < kChunk; ++k) DMG_CHECK(run_step(bt, s));
    return DMG_OK;
  };
  if (!bt->opts.use_graph || s == nullptr) return steps();
  if (!(bt->exec && bt->gstream == s)) {
    bt->reset_graph();
    DMG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const dmg_status st = steps();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (st != DMG_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(DMG_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    bt->graph = g;
    const hipError_t ei = hipGraphInstantiate(&bt->exec, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      bt->reset_graph();
      return fail(DMG_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(ei));
    }
    bt->gstream = s;
  }
  DMG_HIP(hipGraphLaunch(bt->exec, s));
  return DMG_OK;
}

dmg_status ensure_schedule(dmg_batch* bt, double* const* u, const double* const* b, double rtol,
                           int32_t max_iters) {
  const int count = int(bt->inst.size());
  std::vector<const void*> key;
  key.reserve(2 * size_t(count));
  for (int k = 0; k < count; ++k) {
    key.push_back(u[k]);
    key.push_back(b[k]);
  }
  if (bt->built && key == bt->key && rtol == bt->key_rtol && max_iters == bt->key_max)
    return DMG_OK;
  bt->reset_graph();
  bt->built = false;
  DMG_CHECK(build_schedule(bt, u, b, rtol, max_iters));
  bt->key = std::move(key);
  bt->key_rtol = rtol;
  bt->key_max = max_iters;
  return DMG_OK;
}

// Solve state of every instance from its starting norms; returns the count still to iterate.
dmg_status start_solve(dmg_batch* bt, double* const* u, double rtol, hipStream_t s, int* active) {
  const int count = int(bt->inst.size());
  DMG_CHECK(launch_norms_multi(reinterpret_cast<const NormArgs*>(bt->args + bt->norm_off), count,
                               kNormBlocks, bt->npart, bt->summary, s));
  DMG_HIP(hipMemcpyAsync(bt->h_summary, bt->summary, size_t(count) * 2 * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  DMG_HIP(hipMemcpyAsync(bt->h_state, bt->state, size_t(count) * 4 * sizeof(int),
                         hipMemcpyDeviceToHost, s));
  DMG_HIP(hipStreamSynchronize(s));
  int n = 0;
  for (int k = 0; k < count; ++k) {
    const double bn = bt->h_summary[2 * k], rn = bt->h_summary[2 * k + 1];
    if (!std::isfinite(bn))
      return fail(DMG_ERR_NONFINITE, "instance %d: right-hand side norm is not finite", k);
    if (!std::isfinite(rn))
      return fail(DMG_ERR_NONFINITE, "instance %d: initial residual norm is not finite", k);
    if (bn == 0.0) DMG_CHECK(launch_fill<double>(u[k], 0.0, bt->inst[k]->L[0].n(), s));
    if (!bt->h_state[4 * k]) ++n;
  }
  (void)rtol;
  *active = n;
  return DMG_OK;
}

}  // namespace

extern "C" {

dmg_status dmg_batch_workspace_bytes(int32_t count, const int32_t* nx, const int32_t* ny,
                                     const dmg_options* opts, size_t* bytes) {
  clear_error();
  if (count <= 0 || !nx || !ny || !bytes) return fail(DMG_ERR_INVALID_ARG, "bad batch arguments");
  dmg_options o;
  dmg_default_options(&o);
  if (opts) o = *opts;
  o.coarse_gemv = 0;  // the batch runs its coarse levels in the one-workgroup coarse kernel
  size_t total = 0;
  for (int k = 0; k < count; ++k) {
    size_t b = 0;
    DMG_CHECK(dmg_workspace_bytes(nx[k], ny[k], &o, &b));
    total += align_up(b, 256);
  }
  *bytes = total + batch_extra_bytes(count, o);
  return DMG_OK;
}

dmg_status dmg_batch_setup(int32_t count, const int32_t* nx, const int32_t* ny,
                           const double* const* S, const dmg_options* opts, void* workspace,
                           size_t ws_bytes, hipStream_t stream, dmg_batch** out) {
  clear_error();
  if (!out) return fail(DMG_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (count <= 0 || !nx || !ny || !S) return fail(DMG_ERR_INVALID_ARG, "bad batch arguments");
  dmg_options o;
  dmg_default_options(&o);
  if (opts) o = *opts;
  o.coarse_gemv = 0;  // the batch runs its coarse levels in the one-workgroup coarse kernel
  if (o.precision != DMG_FP64)
    return fail(DMG_ERR_UNSUPPORTED, "batched solves run in float64 (precision DMG_FP64)");
  if (o.smoother != 0 && count > 65535)  // the line steps index instances by blockIdx.y
    return fail(DMG_ERR_UNSUPPORTED, "batched line relaxation takes at most 65535 instances");
  size_t need = 0;
  DMG_CHECK(dmg_batch_workspace_bytes(count, nx, ny, &o, &need));
  if (!workspace || ws_bytes < need)
    return fail(DMG_ERR_WORKSPACE, "batch workspace too small: %zu < %zu bytes", ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(DMG_ERR_WORKSPACE, "batch workspace must be 256-byte aligned");
  std::unique_ptr<dmg_batch> bt(new dmg_batch);
  bt->opts = o;
  char* base = static_cast<char*>(workspace);
  size_t off = 0;
  for (int k = 0; k < count; ++k) {
    size_t b = 0;
    DMG_CHECK(dmg_workspace_bytes(nx[k], ny[k], &o, &b));
    b = align_up(b, 256);
    dmg_hier* h = nullptr;
    const dmg_status st = dmg_setup(S[k], nx[k], ny[k], &o, base + off, b, stream, &h);
    if (st != DMG_OK) return st;
    bt->inst.push_back(h);
    off += b;
  }
  auto take = [&](size_t n) {
    void* p = base + off;
    off += align_up(n, 256);
    return p;
  };
  bt->state = static_cast<int*>(take(size_t(count) * 4 * sizeof(int)));
  bt->summary = static_cast<double*>(take(size_t(count) * 2 * sizeof(double)));
  bt->rel = static_cast<double*>(take(size_t(count) * sizeof(double)));
  bt->steps = static_cast<int*>(take(size_t(count) * sizeof(int)));
  bt->npart = static_cast<double*>(take(size_t(count) * kNormBlocks * 2 * sizeof(double)));
  bt->args_cap = args_capacity(count, o);
  bt->args = static_cast<unsigned char*>(take(bt->args_cap));
  DMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&bt->h_state), size_t(count) * 4 * sizeof(int)));
  DMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&bt->h_summary),
                        size_t(count) * 2 * sizeof(double)));
  DMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&bt->h_rel), size_t(count) * sizeof(double)));
  DMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&bt->h_steps), size_t(count) * sizeof(int)));
  // launch shapes: one per level size, shared by every instance that has that size
  std::map<std::pair<int, int>, int> members;  // (line cycles launch no strip kernels)
  for (auto* h : bt->inst)
    for (int l = 0; l < h->tail && o.smoother == 0; ++l) ++members[{h->L[l].nx, h->L[l].ny}];
  for (auto& [d, m] : members) bt->seg_h[d] = default_seg_h(d.first, d.second, m);
  *out = bt.release();
  return DMG_OK;
}

dmg_status dmg_batch_solve(dmg_batch* bt, double* const* u, const double* const* b, double rtol,
                           int32_t max_iters, int32_t* iters, double* relres, hipStream_t stream) {
  clear_error();
  if (!bt || !u || !b) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  if (!(rtol >= 0.0) || max_iters < 0) return fail(DMG_ERR_INVALID_ARG, "bad rtol/max_iters");
  const int count = int(bt->inst.size());
  for (int k = 0; k < count; ++k)
    if (!u[k] || !b[k]) return fail(DMG_ERR_INVALID_ARG, "instance %d: null array", k);
  DMG_CHECK(ensure_schedule(bt, u, b, rtol, max_iters));
  int active = 0;
  DMG_CHECK(start_solve(bt, u, rtol, stream, &active));
  while (active > 0) {
    DMG_CHECK(run_chunk(bt, stream));
    DMG_HIP(hipMemcpyAsync(bt->h_state, bt->state, size_t(count) * 4 * sizeof(int),
                           hipMemcpyDeviceToHost, stream));
    DMG_HIP(hipStreamSynchronize(stream));
    active = 0;
    for (int k = 0; k < count; ++k) active += bt->h_state[4 * k] ? 0 : 1;
  }
  DMG_CHECK(launch_gather_multi(reinterpret_cast<const CheckArgs*>(bt->args + bt->check_off), count,
                                bt->rel, bt->steps, stream));
  DMG_HIP(hipMemcpyAsync(bt->h_rel, bt->rel, size_t(count) * sizeof(double), hipMemcpyDeviceToHost,
                         stream));
  DMG_HIP(hipMemcpyAsync(bt->h_steps, bt->steps, size_t(count) * sizeof(int),
                         hipMemcpyDeviceToHost, stream));
  DMG_HIP(hipStreamSynchronize(stream));
  int failed = -1, nonfinite = -1;
  for (int k = 0; k < count; ++k) {
    const bool zero_b = bt->h_summary[2 * k] == 0.0;
    const double r = zero_b ? 0.0 : bt->h_rel[k];
    if (iters) iters[k] = zero_b ? 0 : bt->h_steps[k];
    if (relres) relres[k] = r;
    if (!std::isfinite(r)) nonfinite = k;
    else if (r > rtol && failed < 0) failed = k;
  }
  if (nonfinite >= 0)
    return fail(DMG_ERR_NONFINITE, "instance %d: residual norm became non-finite", nonfinite);
  if (failed >= 0)
    return fail(DMG_ERR_NO_CONVERGENCE, "instance %d (and maybe others) did not converge", failed);
  return DMG_OK;
}

dmg_status dmg_batch_autotune(dmg_batch* bt, double* const* u, const double* const* b,
                              int32_t flags, int32_t reps, hipStream_t stream) {
  clear_error();
  if (!bt || !u || !b) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  if (reps < 1 || reps > 1000) return fail(DMG_ERR_INVALID_ARG, "reps must be in [1,1000]");
  if (flags & ~3) return fail(DMG_ERR_INVALID_ARG, "unknown autotune flags 0x%x", flags);
  const int count = int(bt->inst.size());
  for (int k = 0; k < count; ++k)
    if (!u[k] || !b[k]) return fail(DMG_ERR_INVALID_ARG, "instance %d: null array", k);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  DMG_HIP(hipEventCreate(&e0));
  DMG_HIP(hipEventCreate(&e1));
  // time `reps` batched steps with every instance active (rtol 0, no step limit reached)
  auto time_steps = [&](float* ms) -> dmg_status {
    bt->built = false;
    bt->reset_graph();
    DMG_CHECK(ensure_schedule(bt, u, b, 0.0, 1 << 30));
    int active = 0;
    DMG_CHECK(start_solve(bt, u, 0.0, stream, &active));
    DMG_CHECK(run_step(bt, stream));
    DMG_HIP(hipEventRecord(e0, stream));
    for (int r = 0; r < reps; ++r) DMG_CHECK(run_step(bt, stream));
    DMG_HIP(hipEventRecord(e1, stream));
    DMG_HIP(hipEventSynchronize(e1));
    DMG_HIP(hipEventElapsedTime(ms, e0, e1));
    return DMG_OK;
  };
  dmg_status st = DMG_OK;
  if ((flags & 2) && bt->opts.smoother == 0) {  // (line relaxation visits no colours)
    // colour orders: the row-separable pairs whose post order reverses the pre order (the
    // V-cycle stays symmetric), chosen per size class (instances of one finest grid size), one
    // class after another (coordinate descent), each candidate timed as whole batched solves to
    // 1e-10 from zero, which counts the cycles it saves or costs
    static const int32_t cand[4][4] = {{0, 1, 2, 3}, {1, 0, 3, 2}, {2, 3, 0, 1}, {3, 2, 1, 0}};
    std::map<std::pair<int, int>, std::vector<int>> classes;
    for (int k = 0; k < count; ++k) classes[{bt->inst[k]->L[0].nx, bt->inst[k]->L[0].ny}].push_back(k);
    auto set_class = [&](const std::vector<int>& mem, int c) -> dmg_status {
      int32_t post[4];
      for (int k = 0; k < 4; ++k) post[k] = cand[c][3 - k];
      for (int k : mem) DMG_CHECK(set_colour_orders(bt->inst[k], cand[c], post, stream));
      bt->built = false;
      bt->reset_graph();
      return DMG_OK;
    };
    for (auto& [dims, mem] : classes) {
      if (st != DMG_OK) break;
      float best_ms = 1e30f;
      int best = -1;
      for (int c = 0; c < 4 && st == DMG_OK; ++c) {
        st = set_class(mem, c);
        float total = 0.f;
        for (int r = 0; r <= std::max(1, reps / 4) && st == DMG_OK; ++r) {
          for (int k = 0; k < count && st == DMG_OK; ++k)
            st = launch_fill<double>(u[k], 0.0, bt->inst[k]->L[0].n(), stream);
          if (st != DMG_OK) break;
          DMG_HIP(hipEventRecord(e0, stream));
          st = dmg_batch_solve(bt, u, b, 1e-10, 500, nullptr, nullptr, stream);
          DMG_HIP(hipEventRecord(e1, stream));
          DMG_HIP(hipEventSynchronize(e1));
          float ms = 0.f;
          DMG_HIP(hipEventElapsedTime(&ms, e0, e1));
          if (r > 0) total += ms;  // the first solve builds the schedule and captures the graph
        }
        if (st == DMG_ERR_NO_CONVERGENCE) {  // this order does not reach the tolerance in 500 steps
          st = DMG_OK;
          clear_error();
          continue;
        }
        if (st == DMG_OK && total < best_ms) {
          best_ms = total;
          best = c;
        }
      }
      if (st == DMG_OK) st = set_class(mem, best >= 0 ? best : 0);
    }
    if (st == DMG_OK)  // the batch-wide record: instance 0's pair
      for (int k = 0; k < 4; ++k) {
        bt->opts.pre_order[k] = bt->inst[0]->opts.pre_order[k];
        bt->opts.post_order[k] = bt->inst[0]->opts.post_order[k];
      }
  }
  for (auto& [d, h] : bt->seg_h) {
    if (!(flags & 1) || st != DMG_OK) break;
    int best = h;
    float best_ms = 1e30f;
    for (int c = 2; c <= 128 && st == DMG_OK; c *= 2) {
      if (tiles_of(d.first, d.second, c) > kMaxPartials) continue;
      h = c;
      float ms = 0.f;
      st = time_steps(&ms);
      if (st == DMG_OK && ms < best_ms) {
        best_ms = ms;
        best = c;
      }
      if (c * 2 > d.second + 1) break;
    }
    h = best;
  }
  if (st == DMG_OK && (flags & 1)) {
    int best = bt->tail_threads;
    float best_ms = 1e30f;
    for (int t : {256, 512, 1024}) {
      bt->tail_threads = t;
      float ms = 0.f;
      st = time_steps(&ms);
      if (st != DMG_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best = t;
      }
    }
    bt->tail_threads = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  bt->built = false;
  bt->reset_graph();
  return st;
}

dmg_status dmg_batch_config(const dmg_batch* bt, int32_t* pre_order, int32_t* post_order,
                            int32_t* tail_threads) {
  clear_error();
  if (!bt) return fail(DMG_ERR_INVALID_ARG, "null batch");
  for (int k = 0; k < 4; ++k) {
    if (pre_order) pre_order[k] = bt->opts.pre_order[k];
    if (post_order) post_order[k] = bt->opts.post_order[k];
  }
  if (tail_threads) *tail_threads = bt->tail_threads;
  return DMG_OK;
}

dmg_status dmg_batch_instance_orders(const dmg_batch* bt, int32_t k, int32_t* pre_order,
                                     int32_t* post_order) {
  clear_error();
  if (!bt) return fail(DMG_ERR_INVALID_ARG, "null batch");
  if (k < 0 || k >= int(bt->inst.size()))
    return fail(DMG_ERR_INVALID_ARG, "instance %d out of range [0,%zu)", k, bt->inst.size());
  for (int q = 0; q < 4; ++q) {
    if (pre_order) pre_order[q] = bt->inst[k]->opts.pre_order[q];
    if (post_order) post_order[q] = bt->inst[k]->opts.post_order[q];
  }
  return DMG_OK;
}

void dmg_batch_destroy(dmg_batch* bt) { delete bt; }

}  // extern "C"
