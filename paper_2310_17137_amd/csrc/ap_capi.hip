// C ABI of the alternating-projection solver (declared in include/ap.h):
// argument validation, workspace layout, launch sequencing and status codes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/ap.h"
#include "ap_internal.h"

struct ap_problem {
  ap::Layout L;
  ap::Dev D;
  ap::Params P;
  ap_config cfg;  // copy; cfg.lengthscale is not kept
  const float* X;
  void* ws;
  int device;
  hipEvent_t ev[4];
  // per-phase event pairs (ap_profile): solve, update, select, check, refine
  bool prof = false;
  std::vector<hipEvent_t> pool[5];
  size_t used[5] = {0, 0, 0, 0, 0};
  // one epoch's launches captured as a HIP graph, replayed on the caller's
  // stream; re-captured when the state buffers or the tile mode change
  hipStream_t cap = nullptr;
  hipGraphExec_t epoch_exec = nullptr;
  const void* key[4] = {nullptr, nullptr, nullptr, nullptr};
  // batch steps: the descriptor grouped launches read (host copy and its place
  // in the workspace), and a stream plus pinned buffer for progress snapshots
  ap::Desc desc;
  ap::Desc* desc_dev = nullptr;
  hipStream_t peek_stream = nullptr;
  ap::Ctl* peek_buf = nullptr;
};

namespace {

// Description of the last HIP failure on this thread (ap_last_error).
thread_local char g_last_error[256] = "";

ap_status note_hip(hipError_t e, const char* where) {
  if (e == hipSuccess) return AP_OK;
  std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", where, hipGetErrorName(e),
                (int)e);
  return AP_ERR_HIP;
}

// Second stream of batch steps, one per device, created on first use and kept
// for the life of the process, with the events of its fork from and join to
// the caller's stream.
struct Aux {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
constexpr int kMaxDevices = 64;
Aux g_aux[kMaxDevices];
std::mutex g_aux_mu;

// The launchers check their launches with hipGetLastError, which also returns
// an error that an earlier HIP call elsewhere in the process left unread. Such
// an error is not this library's: it is taken off (and kept for ap_last_error)
// before the library launches anything.
void clear_foreign_error() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    std::snprintf(g_last_error, sizeof(g_last_error),
                  "discarded an unread error left by an earlier HIP call outside this library: "
                  "%s (%d)", hipGetErrorName(e), (int)e);
}

#define hip_fail(call) note_hip((call), #call)

#define AP_HIP(call)                                      \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return note_hip(e_, #call);     \
  } while (0)

ap_status aux_stream(int device, Aux** out) {
  if (device < 0 || device >= kMaxDevices) return AP_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_aux_mu);
  Aux& a = g_aux[device];
  if (!a.s) {
    AP_HIP(hipStreamCreateWithFlags(&a.s, hipStreamNonBlocking));
    AP_HIP(hipEventCreateWithFlags(&a.fork, hipEventDisableTiming));
    AP_HIP(hipEventCreateWithFlags(&a.join, hipEventDisableTiming));
  }
  *out = &a;
  return AP_OK;
}

// Checks every scalar field of the configuration. Returns AP_OK,
// AP_ERR_INVALID_ARG (out of the method's domain) or AP_ERR_UNSUPPORTED
// (inside the domain, outside this build's limits).
ap_status check_config(const ap_config* c) {
  if (!c || !c->lengthscale) return AP_ERR_INVALID_ARG;
  if (c->n < 1 || c->d < 1 || c->l < 1 || c->b < 1 || c->b > c->n) return AP_ERR_INVALID_ARG;
  if (c->kernel < AP_RBF || c->kernel > AP_MATERN52) return AP_ERR_INVALID_ARG;
  if (c->order != AP_CYCLIC && c->order != AP_GREEDY && c->order != AP_RANDOM)
    return AP_ERR_INVALID_ARG;
  if (c->tile < AP_TILE_FP32 || c->tile > AP_TILE_FP64) return AP_ERR_INVALID_ARG;
  if (!(c->outputscale > 0.0) || !std::isfinite(c->outputscale)) return AP_ERR_INVALID_ARG;
  if (!(c->noise >= 0.0) || !std::isfinite(c->noise)) return AP_ERR_INVALID_ARG;
  if (!(c->tol >= 0.0) || std::isnan(c->tol)) return AP_ERR_INVALID_ARG;
  if (c->min_epochs < 0 || c->max_epochs < 1 || c->refine_every < 0) return AP_ERR_INVALID_ARG;
  for (int k = 0; k < c->d && k < ap::kMaxD; ++k)
    if (!(c->lengthscale[k] > 0.0) || !std::isfinite(c->lengthscale[k])) return AP_ERR_INVALID_ARG;
  if (c->d > ap::kMaxD || c->l > ap::kMaxL || c->b > 4096 || c->n >= (int64_t(1) << 31))
    return AP_ERR_UNSUPPORTED;
  return AP_OK;
}

bool valid_handle(const ap_problem* h) { return h != nullptr && h->ws != nullptr; }

bool valid_state(const ap_state* st) { return st && st->B && st->W && st->R; }

ap_status read_ctl(ap_problem* h, hipStream_t s, ap::Ctl* out) {
  AP_HIP(hipMemcpyAsync(out, h->D.ctl, sizeof(ap::Ctl), hipMemcpyDeviceToHost, s));
  AP_HIP(hipStreamSynchronize(s));
  return AP_OK;
}

enum Phase { kSolve = 0, kUpdate = 1, kSelect = 2, kCheck = 3, kRefine = 4 };

// Records one event of a begin/end pair for `phase` when profiling is on.
hipError_t mark(ap_problem* h, int phase, hipStream_t s) {
  if (!h->prof) return hipSuccess;
  std::vector<hipEvent_t>& pool = h->pool[phase];
  if (h->used[phase] == pool.size()) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    pool.push_back(e);
  }
  return hipEventRecord(pool[h->used[phase]++], s);
}

#define AP_PHASE(phase, call)                  \
  do {                                         \
    AP_HIP(mark(h, phase, s));                 \
    AP_HIP(call);                              \
    AP_HIP(mark(h, phase, s));                 \
  } while (0)

// One block update (inner loop of Algorithm 1). block < 0: the greedy or
// random selection, whose index is already in the control block; a random
// update then draws the next one.
ap_status one_update(ap_problem* h, const ap_state* st, int32_t block, bool last,
                     hipStream_t s) {
  const bool greedy = h->L.order == AP_GREEDY;
  AP_PHASE(kSolve, ap::launch_block_solve(h->L, h->D, h->P, block, st->R, st->W, s));
  if (h->L.tile == AP_TILE_FP64)
    AP_PHASE(kUpdate, ap::launch_fused_update64(h->L, h->D, h->P, h->X, block, st->R, greedy,
                                                last, s));
  else
    AP_PHASE(kUpdate, ap::launch_fused_update(h->L, h->D, block, st->R, greedy, last, s));
  if (greedy) AP_PHASE(kSelect, ap::launch_select(h->L, h->D, s));
  if (h->L.order == AP_RANDOM && block < 0)
    AP_PHASE(kSelect, ap::launch_random_select(h->L, h->D, s));
  return AP_OK;
}

ap_status refine(ap_problem* h, const ap_state* st, hipStream_t s) {
  AP_PHASE(kRefine, ap::launch_residual(h->L, h->D, h->P, h->X, st->B, st->W, st->R, true, s));
  if (h->L.order == AP_GREEDY) AP_PHASE(kSelect, ap::launch_select(h->L, h->D, s));
  return AP_OK;
}

ap_status enqueue_epoch(ap_problem* h, const ap_state* st, hipStream_t s) {
  const bool cyclic = h->L.order == AP_CYCLIC;
  for (int32_t u = 0; u < h->L.m; ++u) {
    ap_status r = one_update(h, st, cyclic ? u : -1, u == h->L.m - 1, s);
    if (r != AP_OK) return r;
  }
  AP_PHASE(kCheck, ap::launch_epoch_check(h->L, h->D, s));
  return AP_OK;
}

void drop_graph(ap_problem* h) {
  if (h->epoch_exec) (void)hipGraphExecDestroy(h->epoch_exec);
  h->epoch_exec = nullptr;
}

// An epoch is the same launch sequence every time (cyclic blocks by index,
// greedy blocks read from the control block), so it is captured once as a
// graph and replayed; with profiling on, the launches go out one by one.
ap_status run_epoch(ap_problem* h, const ap_state* st, hipStream_t s) {
  if (h->prof) return enqueue_epoch(h, st, s);
  const void* key[4] = {st->B, st->W, st->R, (const void*)(intptr_t)(h->L.tile + 1)};
  if (!h->epoch_exec || std::memcmp(key, h->key, sizeof(key)) != 0) {
    drop_graph(h);
    if (!h->cap) AP_HIP(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    AP_HIP(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    ap_status r = enqueue_epoch(h, st, h->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->cap, &g);
    if (r != AP_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return r != AP_OK ? r : note_hip(e, "hipStreamEndCapture");
    }
    e = hipGraphInstantiate(&h->epoch_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      h->epoch_exec = nullptr;
      return note_hip(e, "hipGraphInstantiate");
    }
    std::memcpy(h->key, key, sizeof(key));
  }
  AP_HIP(hipGraphLaunch(h->epoch_exec, s));
  return AP_OK;
}

}  // namespace

namespace ap {
int note_error(const char* where, hipError_t e) { return (int)note_hip(e, where); }
void note_text(const char* msg) { std::snprintf(g_last_error, sizeof(g_last_error), "%s", msg); }
void take_foreign_error() { clear_foreign_error(); }
}  // namespace ap

extern "C" {

size_t ap_workspace_bytes(const ap_config* cfg) {
  if (check_config(cfg) != AP_OK) return 0;
  ap::Layout L;
  if (!ap::make_layout(cfg->n, cfg->d, cfg->l, cfg->b, cfg->kernel, cfg->order, cfg->tile, &L))
    return 0;
  return L.total;
}

ap_status ap_factor_blocks(const ap_config* cfg, const float* X, void* ws, size_t ws_bytes,
                           hipStream_t stream, ap_handle* out, int64_t* bad_block) {
  ap_status cs = check_config(cfg);
  if (cs != AP_OK) return cs;
  if (!X || !ws || !out) return AP_ERR_INVALID_ARG;
  if (((uintptr_t)ws & 255) != 0) return AP_ERR_INVALID_ARG;
  ap::Layout L;
  if (!ap::make_layout(cfg->n, cfg->d, cfg->l, cfg->b, cfg->kernel, cfg->order, cfg->tile, &L))
    return AP_ERR_UNSUPPORTED;
  L.seed = cfg->seed;
  if (ws_bytes < L.total) return AP_ERR_WORKSPACE;
  ap_problem* h = new (std::nothrow) ap_problem();
  if (!h) {
    std::snprintf(g_last_error, sizeof(g_last_error), "host allocation of the handle failed");
    return AP_ERR_HIP;
  }
  h->L = L;
  h->D = ap::bind(L, ws);
  h->cfg = *cfg;
  h->cfg.lengthscale = nullptr;
  h->X = X;
  h->ws = ws;
  for (int k = 0; k < ap::kMaxD; ++k) h->P.ell[k] = k < cfg->d ? cfg->lengthscale[k] : 1.0;
  h->P.s = cfg->outputscale;
  h->P.noise = cfg->noise;
  clear_foreign_error();
  hipError_t he = hipGetDevice(&h->device);
  if (he != hipSuccess) {
    delete h;
    return note_hip(he, "hipGetDevice");
  }
  he = hipStreamCreateWithFlags(&h->peek_stream, hipStreamNonBlocking);
  if (he == hipSuccess) he = hipHostMalloc((void**)&h->peek_buf, sizeof(ap::Ctl), hipHostMallocDefault);
  if (he != hipSuccess) {
    ap_destroy(h);
    return note_hip(he, "peek stream or buffer");
  }
  for (int i = 0; i < 4; ++i) {
    he = hipEventCreate(&h->ev[i]);
    if (he != hipSuccess) {
      for (int k = 0; k < i; ++k) (void)hipEventDestroy(h->ev[k]);
      delete h;
      return note_hip(he, "hipEventCreate");
    }
  }
  h->desc = ap::Desc{};
  h->desc.L = L;
  h->desc.D = h->D;
  h->desc.P = h->P;
  h->desc.X = X;
  h->desc.tol = cfg->tol;
  h->desc.min_epochs = cfg->min_epochs;
  h->desc.max_epochs = cfg->max_epochs;
  h->desc.refine_every = cfg->refine_every;
  h->desc_dev = (ap::Desc*)((char*)ws + L.off_desc);
  ap_status r = hip_fail(ap::launch_prep(L, h->D, h->P, X, stream));
  if (r == AP_OK) r = hip_fail(ap::launch_factor(L, h->D, h->P, X, stream));
  if (r == AP_OK)
    r = hip_fail(hipMemcpyAsync(h->desc_dev, &h->desc, sizeof(ap::Desc), hipMemcpyHostToDevice,
                                stream));
  ap::Ctl ctl;
  if (r == AP_OK) r = read_ctl(h, stream, &ctl);
  if (r == AP_OK && ctl.fail != ~0ull) {
    if (bad_block) *bad_block = (int64_t)(ctl.fail >> 32);
    r = AP_ERR_NOT_PD;
  }
  if (r != AP_OK) {
    ap_destroy(h);
    return r;
  }
  *out = h;
  return AP_OK;
}

ap_status ap_reset(ap_handle h, const ap_state* st, hipStream_t stream) {
  if (!valid_handle(h) || !valid_state(st)) return AP_ERR_INVALID_ARG;
  clear_foreign_error();
  return hip_fail(ap::launch_reset(h->L, h->D, st->B, st->W, st->R, false, stream));
}

ap_status ap_warm_start(ap_handle h, const ap_state* st, hipStream_t stream) {
  if (!valid_handle(h) || !valid_state(st)) return AP_ERR_INVALID_ARG;
  clear_foreign_error();
  ap_status r = hip_fail(ap::launch_reset(h->L, h->D, st->B, st->W, st->R, true, stream));
  if (r != AP_OK) return r;
  return refine(h, st, stream);
}

ap_status ap_epoch(const ap_handle* h, const ap_state* st, int32_t count, int32_t epochs,
                   hipStream_t stream) {
  if (!h || !st || count < 1 || epochs < 0) return AP_ERR_INVALID_ARG;
  for (int32_t p = 0; p < count; ++p)
    if (!valid_handle(h[p]) || !valid_state(&st[p])) return AP_ERR_INVALID_ARG;
  clear_foreign_error();
  for (int32_t e = 0; e < epochs; ++e)
    for (int32_t p = 0; p < count; ++p) {
      ap_status r = run_epoch(h[p], &st[p], stream);
      if (r != AP_OK) return r;
    }
  return AP_OK;
}

ap_status ap_update(ap_handle h, const ap_state* st, int32_t block, hipStream_t stream) {
  if (!valid_handle(h) || !valid_state(st)) return AP_ERR_INVALID_ARG;
  if (block < 0 || block >= h->L.m) return AP_ERR_INVALID_ARG;
  clear_foreign_error();
  return one_update(h, st, block, true, stream);
}

ap_status ap_rel_residual(ap_handle h, hipStream_t stream, double* rho, double* col_ratio) {
  if (!valid_handle(h) || !rho) return AP_ERR_INVALID_ARG;
  ap::Ctl c;
  ap_status r = read_ctl(h, stream, &c);
  if (r != AP_OK) return r;
  if (c.status != 0 || !std::isfinite(c.rho)) return AP_ERR_NONFINITE;
  *rho = c.rho;
  if (col_ratio)
    for (int i = 0; i < h->L.l; ++i) col_ratio[i] = c.colrel[i];
  return AP_OK;
}

ap_status ap_residual(ap_handle h, const ap_state* st, float* R_out, double* col_rel,
                      hipStream_t stream) {
  if (!valid_handle(h) || !valid_state(st)) return AP_ERR_INVALID_ARG;
  clear_foreign_error();
  const bool in_place = R_out == nullptr || R_out == st->R;
  if (in_place) {
    ap_status r = refine(h, st, stream);
    if (r != AP_OK) return r;
  } else {
    hipStream_t s = stream;
    AP_PHASE(kRefine, ap::launch_residual(h->L, h->D, h->P, h->X, st->B, st->W, R_out, false, s));
  }
  if (col_rel) {
    ap::Ctl c;
    ap_status r = read_ctl(h, stream, &c);
    if (r != AP_OK) return r;
    if (c.status != 0) return AP_ERR_NONFINITE;
    for (int i = 0; i < h->L.l; ++i) col_rel[i] = c.colrel_true[i];
  }
  return AP_OK;
}

// ap_solve from W = 0 (warm = false) or from the caller's W (ap_solve_from)
static ap_status solve_impl(ap_handle h, const ap_state* st, hipStream_t stream, ap_stats* out,
                            bool warm) {
  if (!valid_handle(h) || !valid_state(st)) return AP_ERR_INVALID_ARG;
  const ap_config& c = h->cfg;
  // The solve may move to FP64 tiles; the mode the handle held on entry (its
  // configured one, or FP64 after ap_set_tile) is put back on every return.
  struct TileGuard {
    ap_problem* h;
    int32_t tile;
    ~TileGuard() { h->L.tile = tile; }
  } guard{h, h->L.tile};
  ap_stats s{};
  s.rho_true = NAN;
  s.escalated_at = -1;
  s.restarted_at = -1;
  ap_status r = warm ? ap_warm_start(h, st, stream) : ap_reset(h, st, stream);
  if (r != AP_OK) return r;
  ap_status result = AP_NOT_CONVERGED;
  ap::Ctl ctl;
  double t_ep = 0.0, t_ref = 0.0;
  // epochs between true residuals: doubles (up to 16 refine_every) while the
  // true and maintained ratios agree to 1e-5, back to refine_every otherwise
  int32_t interval = c.refine_every, next_ref = c.refine_every;
  for (int32_t t = 1; t <= c.max_epochs; ++t) {
    AP_HIP(hipEventRecord(h->ev[0], stream));
    r = run_epoch(h, st, stream);
    if (r != AP_OK) return r;
    AP_HIP(hipEventRecord(h->ev[1], stream));
    r = read_ctl(h, stream, &ctl);
    if (r != AP_OK) return r;
    if (ctl.status != 0 || !std::isfinite(ctl.rho)) {
      // a reduced-precision tile mode overflowed, so W may hold non-finite
      // steps: restart Algorithm 1 (W = 0, R = B) on FP64 tiles, or give up if
      // already there
      if (h->L.tile == AP_TILE_FP64) return AP_ERR_NONFINITE;
      h->L.tile = AP_TILE_FP64;
      s.escalated_at = t;
      s.restarted_at = t;
      r = ap_reset(h, st, stream);
      if (r != AP_OK) return r;
      s.epochs = t;
      s.rho_maintained = 1.0;
      continue;
    }
    float ms = 0.f;
    AP_HIP(hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
    t_ep += ms * 1e-3;
    s.epochs = t;
    s.rho_maintained = ctl.rho;
    const bool scheduled = c.refine_every > 0 && t >= next_ref;
    const bool hit = ctl.rho < c.tol && t >= c.min_epochs;
    const bool check = scheduled || (hit && (c.refine_every > 0 || h->L.tile != AP_TILE_FP32));
    double rho = ctl.rho;
    if (check) {
      // FP64 true residual replaces R (Lemma residual_equality); when it and
      // the maintained residual disagree by more than 5%, the remaining
      // epochs run on FP64 tiles
      const double maintained = ctl.rho;
      AP_HIP(hipEventRecord(h->ev[1], stream));
      r = refine(h, st, stream);
      if (r != AP_OK) return r;
      AP_HIP(hipEventRecord(h->ev[2], stream));
      r = read_ctl(h, stream, &ctl);
      if (r != AP_OK) return r;
      AP_HIP(hipEventElapsedTime(&ms, h->ev[1], h->ev[2]));
      t_ref += ms * 1e-3;
      s.refines++;
      if (ctl.status != 0 || !std::isfinite(ctl.rho_true)) return AP_ERR_NONFINITE;
      s.rho_true = ctl.rho_true;
      rho = ctl.rho_true;
      const double drift = std::fabs(ctl.rho_true - maintained) / ctl.rho_true;
      if (h->L.tile != AP_TILE_FP64 && drift > 0.05) {
        h->L.tile = AP_TILE_FP64;
        s.escalated_at = t;
        if (ctl.rho_true >= 1.0) {
          // the drifted W is no better than W = 0 (ratio 1): restart
          // Algorithm 1 from W = 0 on FP64 tiles instead of continuing from it
          s.restarted_at = t;
          r = ap_reset(h, st, stream);
          if (r != AP_OK) return r;
          if (scheduled) next_ref = t + c.refine_every;
          continue;
        }
      }
      if (scheduled) {
        interval = drift < 1e-5 ? std::min(2 * interval, 16 * c.refine_every) : c.refine_every;
        next_ref = t + interval;
      }
    }
    if (rho < c.tol && t >= c.min_epochs) {
      result = AP_OK;
      break;
    }
  }
  s.t_epochs = t_ep;
  s.t_refine = t_ref;
  s.tile = h->L.tile;
  if (out) *out = s;
  return result;
}

ap_status ap_solve(ap_handle h, const ap_state* st, hipStream_t stream, ap_stats* out) {
  return solve_impl(h, st, stream, out, false);
}

ap_status ap_solve_from(ap_handle h, const ap_state* st, hipStream_t stream, ap_stats* out) {
  return solve_impl(h, st, stream, out, true);
}

ap_status ap_set_tile(ap_handle h, int32_t tile) {
  if (!valid_handle(h)) return AP_ERR_INVALID_ARG;
  if (tile != h->cfg.tile && tile != AP_TILE_FP64) return AP_ERR_INVALID_ARG;
  h->L.tile = tile;
  return AP_OK;
}

ap_status ap_mll_grad(ap_handle h, const ap_state* st, double* grad, double* partials,
                      hipStream_t stream) {
  if (!valid_handle(h) || !valid_state(st) || !grad) return AP_ERR_INVALID_ARG;
  clear_foreign_error();
  AP_HIP(ap::launch_mll_grad(h->L, h->D, h->P, h->X, st->B, st->W, stream));
  if (partials)
    AP_HIP(hipMemcpyAsync(partials, h->D.gpart,
                          (size_t)h->L.nwg_mll * (ap::kMaxD + 2) * sizeof(double),
                          hipMemcpyDeviceToDevice, stream));
  ap::Ctl c;
  ap_status r = read_ctl(h, stream, &c);
  if (r != AP_OK) return r;
  for (int m = 0; m < h->L.d + 2; ++m) {
    if (!std::isfinite(c.mll_grad[m])) return AP_ERR_NONFINITE;
    grad[m] = c.mll_grad[m];
  }
  return AP_OK;
}

ap_status ap_predict(ap_handle h, const double* W, const float* Xs, int64_t ns, double* mean,
                     hipStream_t stream) {
  if (!valid_handle(h) || ns < 0 || (ns > 0 && (!W || !Xs || !mean))) return AP_ERR_INVALID_ARG;
  if (ns >= (int64_t(1) << 31)) return AP_ERR_UNSUPPORTED;
  clear_foreign_error();
  return hip_fail(ap::launch_predict(h->L, h->P, h->X, W, Xs, ns, mean, stream));
}

ap_status ap_block_inverse(ap_handle h, int32_t j, double* dst, hipStream_t stream) {
  if (!valid_handle(h) || !dst || j < 0 || j >= h->L.m) return AP_ERR_INVALID_ARG;
  clear_foreign_error();
  return hip_fail(ap::launch_copy_inverse(h->L, h->D, j, dst, stream));
}

ap_status ap_profile(ap_handle h, int32_t enable) {
  if (!valid_handle(h)) return AP_ERR_INVALID_ARG;
  h->prof = enable != 0;
  for (int p = 0; p < 5; ++p) h->used[p] = 0;
  return AP_OK;
}

ap_status ap_profile_read(ap_handle h, hipStream_t stream, double* seconds, int64_t* launches) {
  if (!valid_handle(h) || !seconds || !launches) return AP_ERR_INVALID_ARG;
  AP_HIP(hipStreamSynchronize(stream));
  for (int p = 0; p < 5; ++p) {
    double tot = 0.0;
    for (size_t i = 0; i + 1 < h->used[p]; i += 2) {
      float ms = 0.f;
      AP_HIP(hipEventElapsedTime(&ms, h->pool[p][i], h->pool[p][i + 1]));
      tot += ms * 1e-3;
    }
    seconds[p] = tot;
    launches[p] = (int64_t)(h->used[p] / 2);
  }
  return AP_OK;
}

ap_status ap_batch_step(const ap_handle* h, const ap_state* st, int32_t count, int32_t steps,
                        hipStream_t stream) {
  if (!h || !st || count < 1 || count > ap::kMaxBatch || steps < 0) return AP_ERR_INVALID_ARG;
  for (int32_t p = 0; p < count; ++p) {
    if (!valid_handle(h[p]) || !valid_state(&st[p])) return AP_ERR_INVALID_ARG;
    for (int32_t q = 0; q < p; ++q)
      if (h[q] == h[p]) return AP_ERR_INVALID_ARG;
  }
  clear_foreign_error();
  // gp: solve partials, gf: solve finish, ga: advance (all problems); gs[0]
  // and gs[1]: the fused updates of the problems on split tiles with narrow
  // (d <= 8) and wide features; problems on other tiles get launches of their own
  ap::Group gp{}, gf{}, ga{}, gs[2]{};
  int32_t n_other = 0;
  for (int32_t p = 0; p < count; ++p) {
    const ap::Layout& L = h[p]->L;
    for (ap::Group* g : {&gp, &gf, &ga}) {
      g->desc[p] = h[p]->desc_dev;
      g->R[p] = st[p].R;
      g->W[p] = st[p].W;
      g->tile[p] = L.tile;
    }
    gp.wg0[p + 1] = gp.wg0[p] + (L.b_pad / 64) * ap::kBsSplit;
    gf.wg0[p + 1] = gf.wg0[p] + (L.b_pad * ap::kMaxL + 255) / 256;
    ga.wg0[p + 1] = ga.wg0[p] + 1;
    if (L.tile == AP_TILE_SPLIT) {
      ap::Group& g = gs[L.dp > 8 ? 1 : 0];
      const int32_t k = g.count++;
      g.desc[k] = h[p]->desc_dev;
      g.R[k] = st[p].R;
      g.W[k] = st[p].W;
      g.tile[k] = L.tile;
      g.wg0[k + 1] = g.wg0[k] + L.nwg;
    } else {
      ++n_other;
    }
  }
  gp.count = gf.count = ga.count = count;
  // greedy selection after the updates: block norms (one workgroup per block)
  // and argmax (one per problem) of the greedy problems
  ap::Group gsel_n{}, gsel_a{};
  for (int32_t p = 0; p < count; ++p) {
    if (h[p]->L.order != AP_GREEDY) continue;
    const int32_t k = gsel_n.count++;
    gsel_n.desc[k] = gsel_a.desc[k] = h[p]->desc_dev;
    gsel_n.wg0[k + 1] = gsel_n.wg0[k] + h[p]->L.m;
    gsel_a.wg0[k + 1] = gsel_a.wg0[k] + 1;
  }
  gsel_a.count = gsel_n.count;
  // random order: the next draw of every random problem whose update ran
  ap::Group grnd{};
  for (int32_t p = 0; p < count; ++p) {
    if (h[p]->L.order != AP_RANDOM) continue;
    const int32_t k = grnd.count++;
    grnd.desc[k] = h[p]->desc_dev;
    grnd.wg0[k + 1] = grnd.wg0[k] + 1;
  }
  // The wide split group and the other tiles run on a second stream beside
  // the narrow group, between a fork after the solves and a join before the
  // epoch advance.
  const bool fork = gs[1].count > 0 || n_other > 0;
  Aux* aux = nullptr;
  if (fork) {
    ap_status r = aux_stream(h[0]->device, &aux);
    if (r != AP_OK) return r;
  }
  for (int32_t s = 0; s < steps; ++s) {
    AP_HIP(ap::launch_group_solve(gp, gf, stream));
    if (fork) {
      AP_HIP(hipEventRecord(aux->fork, stream));
      AP_HIP(hipStreamWaitEvent(aux->s, aux->fork, 0));
    }
    if (gs[0].count > 0) AP_HIP(ap::launch_group_split(gs[0], false, stream));
    if (gs[1].count > 0) AP_HIP(ap::launch_group_split(gs[1], true, aux->s));
    for (int32_t p = 0; p < count && n_other > 0; ++p) {
      ap_problem* q = h[p];
      if (q->L.tile == AP_TILE_SPLIT) continue;
      const bool greedy = q->L.order == AP_GREEDY;
      const int code = q->L.order != AP_CYCLIC ? ap::kBlockBatchSel : ap::kBlockBatchCyclic;
      if (q->L.tile == AP_TILE_FP64)
        AP_HIP(ap::launch_fused_update64(q->L, q->D, q->P, q->X, code, st[p].R, greedy, true,
                                         aux->s));
      else
        AP_HIP(ap::launch_fused_update(q->L, q->D, code, st[p].R, greedy, true, aux->s));
    }
    if (fork) {
      AP_HIP(hipEventRecord(aux->join, aux->s));
      AP_HIP(hipStreamWaitEvent(stream, aux->join, 0));
    }
    if (gsel_n.count > 0) AP_HIP(ap::launch_group_select(gsel_n, gsel_a, stream));
    if (grnd.count > 0) AP_HIP(ap::launch_group_random(grnd, stream));
    AP_HIP(ap::launch_group_advance(ga, stream));
  }
  return AP_OK;
}

ap_status ap_batch_peek(ap_handle h, ap_progress* out) {
  if (!valid_handle(h) || !out) return AP_ERR_INVALID_ARG;
  AP_HIP(hipMemcpyAsync(h->peek_buf, h->D.ctl, sizeof(ap::Ctl), hipMemcpyDeviceToHost,
                        h->peek_stream));
  AP_HIP(hipStreamSynchronize(h->peek_stream));
  const ap::Ctl& c = *h->peek_buf;
  out->state = c.state;
  out->epoch = c.epoch;
  out->cursor = c.cursor;
  out->status = c.status;
  out->rho = c.rho;
  out->rho_true = c.rho_true;
  return AP_OK;
}

ap_status ap_batch_release(ap_handle h, int32_t next_refine, hipStream_t stream) {
  if (!valid_handle(h) || next_refine < 0) return AP_ERR_INVALID_ARG;
  clear_foreign_error();
  return hip_fail(ap::launch_release(h->D, next_refine, stream));
}

void ap_destroy(ap_handle h) {
  if (!h) return;
  drop_graph(h);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  if (h->peek_stream) (void)hipStreamDestroy(h->peek_stream);
  if (h->peek_buf) (void)hipHostFree(h->peek_buf);
  for (int i = 0; i < 4; ++i)
    if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
  for (int p = 0; p < 5; ++p)
    for (hipEvent_t e : h->pool[p]) (void)hipEventDestroy(e);
  delete h;
}

const char* ap_last_error(void) { return g_last_error; }

const char* ap_status_str(ap_status s) {
  switch (s) {
    case AP_OK: return "ok";
    case AP_NOT_CONVERGED: return "not converged within max_epochs";
    case AP_ERR_INVALID_ARG: return "invalid argument";
    case AP_ERR_NOT_PD: return "a diagonal block is not positive definite";
    case AP_ERR_NONFINITE: return "non-finite residual";
    case AP_ERR_WORKSPACE: return "workspace too small";
    case AP_ERR_HIP: return "HIP runtime error";
    case AP_ERR_UNSUPPORTED: return "size not supported by this build";
  }
  return "unknown status";
}

}  // extern "C"
