// Preconditioner application that allocates nothing, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops).
//
// ddg_apply_precond_noalloc runs the kernels of ddg_apply_precond, in the same
// order and with the same arithmetic, but the buffers those kernels write and
// read back within one application (local residuals, coarse restriction
// partials, the coarse right-hand side and solution, the coarse GEMV partials)
// live in `scratch`, a static device array of kScratchBytes that every GPU the
// library runs on holds until the process ends.  Its device address is looked
// up once per device with hipGetSymbolAddress and kept; host code passes only
// that address to kernels, never the array's name (a host-side stand-in).
// Every call on one GPU shares that GPU's array: calls that overlap on one
// GPU race.  The coarse right-hand side's zero padding is cleared by a fill
// kernel on every call, since the previous call may have left other values.
#include <mutex>

#include "common.hpp"

namespace ddg {

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;   // 32 MiB per device
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (current), resolved once per device.
void* scratch_address(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    DDG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    DDG_REQUIRE(p != nullptr, DDG_ERR_HIP, "scratch array has no device address");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Puts the handle's workspace pointers and profiling switch back on scope exit.
struct WsSwap {
  Handle& h;
  PrecondWs saved;
  bool prof;
  WsSwap(Handle& hh, const PrecondWs& ws) : h(hh), saved(hh.ws), prof(hh.profiling) {
    h.ws = ws;
    h.profiling = false;   // profiling creates events: not on this path
  }
  ~WsSwap() {
    h.ws = saved;
    h.profiling = prof;
  }
};

}  // namespace

}  // namespace ddg

using namespace ddg;

extern "C" int ddg_apply_precond_noalloc(ddg_handle hd, const double* r_dev, double* z_dev) {
  return guarded([&]() {
    Handle* h = H(hd);
    DDG_REQUIRE(h && r_dev && z_dev && !h->host_only, DDG_ERR_INVALID_ARG, "null argument or analysis-only handle");
    int dev = -1;
    DDG_HIP(hipGetDevice(&dev));
    DDG_REQUIRE(dev == h->device, DDG_ERR_INVALID_ARG,
                "the handle's device (" + std::to_string(h->device) + ") must be current");
    DDG_REQUIRE(dev >= 0 && dev < kMaxDevices, DDG_ERR_UNSUPPORTED, "device index beyond 63");
    const Symbolic& S = h->S;
    const bool coarse = h->nc > 0;
    const size_t b_bres = round256((size_t)S.set_ptr[S.n_parts] * sizeof(double));
    const size_t b_rpart = coarse ? round256((size_t)S.n_parts * h->nch * kslots(h->k) * sizeof(double)) : 0;
    const size_t b_cy = coarse ? round256((size_t)2 * h->nc_pad * sizeof(double)) : 0;
    const size_t b_cpart = coarse ? round256((size_t)2 * h->ntiles * 64 * sizeof(double)) : 0;
    const size_t b_cref = coarse && h->coarse_refine > 0 ? round256((size_t)2 * h->nc_pad * sizeof(double)) : 0;
    const size_t need = b_bres + b_rpart + b_cy + b_cpart + b_cref;
    DDG_REQUIRE(need <= kScratchBytes, DDG_ERR_UNSUPPORTED,
                "this handle needs " + std::to_string(need) +
                    " bytes of scratch; the allocation-free entry point holds at most " +
                    std::to_string(kScratchBytes) + " (32 MiB)");
    unsigned char* base = static_cast<unsigned char*>(scratch_address(dev));
    PrecondWs ws;
    ws.bres = reinterpret_cast<double*>(base);
    if (coarse) {
      ws.rpart = reinterpret_cast<double*>(base + b_bres);
      ws.cy = reinterpret_cast<double*>(base + b_bres + b_rpart);
      ws.cpart = reinterpret_cast<double*>(base + b_bres + b_rpart + b_cy);
      if (b_cref) ws.cref = reinterpret_cast<double*>(base + b_bres + b_rpart + b_cy + b_cpart);
      launch_fill(ws.cy, 0.0, 2 * h->nc_pad, h->stream);
    }
    WsSwap swap(*h, ws);
    launch_precond(*h, r_dev, z_dev, -1, false, h->stream);
    DDG_HIP(hipGetLastError());
  });
}
