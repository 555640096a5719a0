// Batched solves of independent instances.  Every instance's hierarchy is carved out of one
// caller workspace; dmg_batch_solve advances all unconverged instances cycle by cycle.
#include <memory>

#include "dmg_internal.h"

struct dmg_batch {
  std::vector<dmg_hier*> inst;
  ~dmg_batch() {
    for (auto* h : inst) dmg_destroy(h);
  }
};

using namespace dmg;

extern "C" {

dmg_status dmg_batch_workspace_bytes(int32_t count, const int32_t* nx, const int32_t* ny,
                                     const dmg_options* opts, size_t* bytes) {
  clear_error();
  if (count <= 0 || !nx || !ny || !bytes) return fail(DMG_ERR_INVALID_ARG, "bad batch arguments");
  size_t total = 0;
  for (int k = 0; k < count; ++k) {
    size_t b = 0;
    DMG_CHECK(dmg_workspace_bytes(nx[k], ny[k], opts, &b));
    total += (b + 255) & ~size_t(255);
  }
  *bytes = total;
  return DMG_OK;
}

dmg_status dmg_batch_setup(int32_t count, const int32_t* nx, const int32_t* ny,
                           const double* const* S, const dmg_options* opts, void* workspace,
                           size_t ws_bytes, hipStream_t stream, dmg_batch** out) {
  clear_error();
  if (!out) return fail(DMG_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (count <= 0 || !nx || !ny || !S) return fail(DMG_ERR_INVALID_ARG, "bad batch arguments");
  size_t need = 0;
  DMG_CHECK(dmg_batch_workspace_bytes(count, nx, ny, opts, &need));
  if (!workspace || ws_bytes < need)
    return fail(DMG_ERR_WORKSPACE, "batch workspace too small: %zu < %zu bytes", ws_bytes, need);
  std::unique_ptr<dmg_batch> bt(new dmg_batch);
  char* base = static_cast<char*>(workspace);
  size_t off = 0;
  for (int k = 0; k < count; ++k) {
    size_t b = 0;
    DMG_CHECK(dmg_workspace_bytes(nx[k], ny[k], opts, &b));
    b = (b + 255) & ~size_t(255);
    dmg_hier* h = nullptr;
    dmg_status st = dmg_setup(S[k], nx[k], ny[k], opts, base + off, b, stream, &h);
    if (st != DMG_OK) return st;
    bt->inst.push_back(h);
    off += b;
  }
  *out = bt.release();
  return DMG_OK;
}

dmg_status dmg_batch_solve(dmg_batch* bt, double* const* u, const double* const* b, double rtol,
                           int32_t max_iters, int32_t* iters, double* relres, hipStream_t stream) {
  clear_error();
  if (!bt || !u || !b) return fail(DMG_ERR_INVALID_ARG, "null pointer argument");
  dmg_status worst = DMG_OK;
  for (size_t k = 0; k < bt->inst.size(); ++k) {
    int32_t it = 0;
    double rr = 0.0;
    dmg_status st = dmg_solve(bt->inst[k], u[k], b[k], rtol, max_iters, &it, &rr, nullptr, stream);
    if (iters) iters[k] = it;
    if (relres) relres[k] = rr;
    if (st != DMG_OK && st != DMG_ERR_NO_CONVERGENCE) return st;
    if (st != DMG_OK) worst = st;
  }
  if (worst != DMG_OK) return fail(worst, "at least one instance did not converge");
  return DMG_OK;
}

void dmg_batch_destroy(dmg_batch* bt) { delete bt; }

}  // extern "C"
