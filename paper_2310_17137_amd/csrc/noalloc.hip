// ap_residual_noalloc: the FP64 true residual R = B - K^ W of ap_residual for
// callers that cannot allocate device memory and hold no solver workspace. The
// kernels are ap_residual's; their scratch (a control block for the column norms
// and ratios, and the per-workgroup column partials) lives in one file-scope
// device array per GPU instead of a caller's workspace.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "../../include/ap.h"
#include "ap_internal.h"

namespace {

// [0, kCtlBytes): control block; then the column partials, one row of kMaxL
// doubles per workgroup (max(kResetGroups, residual workgroups at the largest n)).
constexpr size_t kCtlBytes = 4096;
constexpr size_t kPartRows = (size_t)(AP_NOALLOC_MAX_N / 256);
constexpr size_t kScratchBytes = kCtlBytes + kPartRows * ap::kMaxL * sizeof(double);
static_assert(sizeof(ap::Ctl) <= kCtlBytes, "control block does not fit");
static_assert(kPartRows >= (size_t)ap::kResetGroups, "too few partial rows for the norms of B");
static_assert(kScratchBytes == AP_NOALLOC_SCRATCH_BYTES, "ap.h states another scratch size");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` on each GPU

// The array's device address on the current device, looked up on the first
// call there (hipGetSymbolAddress with that device current).
ap_status scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (ap_status)ap::note_error("hipGetDevice", e);
  if (dev < 0 || dev >= kMaxDevices) return AP_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (ap_status)ap::note_error("hipGetSymbolAddress(scratch)", e);
    if (p == nullptr) return (ap_status)ap::note_error("hipGetSymbolAddress(scratch)", hipErrorNotFound);
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return AP_OK;
}

}  // namespace

extern "C" ap_status ap_residual_noalloc(const ap_config* cfg, const float* X, const float* B,
                                         const double* W, float* R_out, double* col_rel,
                                         hipStream_t stream) {
  if (!cfg || !cfg->lengthscale || !X || !B || !W || !R_out) return AP_ERR_INVALID_ARG;
  if (cfg->n < 1 || cfg->d < 1 || cfg->l < 1) return AP_ERR_INVALID_ARG;
  if (cfg->kernel < AP_RBF || cfg->kernel > AP_MATERN52) return AP_ERR_INVALID_ARG;
  if (!(cfg->outputscale > 0.0) || !std::isfinite(cfg->outputscale)) return AP_ERR_INVALID_ARG;
  if (!(cfg->noise >= 0.0) || !std::isfinite(cfg->noise)) return AP_ERR_INVALID_ARG;
  for (int k = 0; k < cfg->d && k < ap::kMaxD; ++k)
    if (!(cfg->lengthscale[k] > 0.0) || !std::isfinite(cfg->lengthscale[k]))
      return AP_ERR_INVALID_ARG;
  if (cfg->n > AP_NOALLOC_MAX_N) {
    ap::note_text("ap_residual_noalloc: n exceeds AP_NOALLOC_MAX_N, the size its static scratch holds");
    return AP_ERR_UNSUPPORTED;
  }
  if (cfg->d > ap::kMaxD || cfg->l > ap::kMaxL) return AP_ERR_UNSUPPORTED;
  // the residual does not use the block partition: one block of all n rows
  ap::Layout L;
  if (!ap::make_layout(cfg->n, cfg->d, cfg->l, (int32_t)std::min<int64_t>(cfg->n, 4096),
                       cfg->kernel, AP_CYCLIC, AP_TILE_FP64, &L))
    return AP_ERR_UNSUPPORTED;
  ap::take_foreign_error();
  void* base = nullptr;
  ap_status r = scratch_ptr(&base);
  if (r != AP_OK) return r;
  ap::Dev D{};
  D.ctl = (ap::Ctl*)base;
  D.respart = (double*)((char*)base + kCtlBytes);
  ap::Params P{};
  for (int k = 0; k < ap::kMaxD; ++k) P.ell[k] = k < cfg->d ? cfg->lengthscale[k] : 1.0;
  P.s = cfg->outputscale;
  P.noise = cfg->noise;
  hipError_t e = ap::launch_bnorm(L, D, B, stream);  // also clears the status word
  if (e == hipSuccess) e = ap::launch_residual(L, D, P, X, B, W, R_out, false, stream);
  if (e != hipSuccess) return (ap_status)ap::note_error("true-residual launch", e);
  if (col_rel) {
    ap::Ctl c;
    e = hipMemcpyAsync(&c, D.ctl, sizeof(ap::Ctl), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return (ap_status)ap::note_error("reading the column ratios", e);
    if (c.status != 0) return AP_ERR_NONFINITE;
    for (int i = 0; i < L.l; ++i) col_rel[i] = c.colrel_true[i];
  }
  return AP_OK;
}
