// rkn_scan_windows_noalloc: the window scan of rkn_scan_windows for callers that
// cannot allocate device memory (code under stream capture, tight serving loops,
// harnesses that forbid hipMalloc). Its work memory -- the device windows, the seed
// tiles, the per-event tile offsets, the argmin partials, the tile counter and the
// slab of running minima -- lives in one file-scope device array per GPU, held from
// the library's load until the process ends. Nothing in the call allocates.
//
// Host code never passes the array's name to a kernel or a copy: `scratch` in host
// code is a stand-in symbol, not a device address. Its address on each device is
// looked up once (noalloc_init, from rkn_create with that device current) and kept
// in g_ptr; every use goes through it.
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace rkn {

constexpr size_t kScratchBytes = size_t(256) << 20;   // per GPU

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
bool g_done[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
unsigned char* g_ptr[kMaxDevices] = {};

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace

hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_done[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_err[device] = e;
    g_ptr[device] = e == hipSuccess ? static_cast<unsigned char*>(ptr) : nullptr;
    g_done[device] = true;
  }
  return g_err[device];
}

}  // namespace rkn

using namespace rkn;

extern "C" {

rkn_status rkn_scan_windows_noalloc(rkn_ctx* c, const rkn_scan_params* p, int32_t n_windows, const rkn_window* w,
                                    double* score, int32_t* n_in, int64_t* best_index, double* best_score) {
  if (!c) return RKN_E_ARG;
  rkn_status st = validate_scan(c, p);
  if (st != RKN_OK) return st;
  if (!(p->ptr_flags & RKN_PTR_DEVICE) || !best_index || !best_score) {
    c->err = "scan (no allocation): outputs must be device pointers (ptr_flags RKN_PTR_DEVICE); best_index "
             "and best_score must not be NULL";
    return RKN_E_ARG;
  }
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) {
    c->err = std::string("hipSetDevice: ") + hipGetErrorString(e);
    return RKN_E_DEVICE;
  }
  if (c->device >= kMaxDevices || !g_done[c->device] || !g_ptr[c->device]) {
    c->err = std::string("scan (no allocation): no work array on this device: ") +
             (c->device < kMaxDevices && g_done[c->device] ? hipGetErrorString(g_err[c->device])
                                                          : "not initialised");
    return RKN_E_DEVICE;
  }
  std::vector<WindowDev> wins;
  std::vector<Tile> tiles;
  std::vector<int32_t> ev_tiles;
  int64_t total = 0;
  if ((st = prepare_scan_windows(c, p, n_windows, w, wins, tiles, ev_tiles, total)) != RKN_OK) return st;
  rkn_scan_params q = *p;
  q.block_steps = resolve_block_steps(c, &q);
  // layout of the work array for this call; the slab takes what is left
  const size_t n_tiles = tiles.size();
  const size_t o_win = 0;
  const size_t o_tiles = o_win + align256(sizeof(WindowDev) * wins.size());
  const size_t o_evt = o_tiles + align256(sizeof(Tile) * std::max<size_t>(n_tiles, 1));
  const size_t o_parts = o_evt + align256(sizeof(int32_t) * ev_tiles.size());
  const size_t o_counter = o_parts + align256(sizeof(ArgminPart) * std::max<size_t>(n_tiles, 1));
  const size_t o_slab = o_counter + 256;
  const size_t per_wg = scan_slab_bytes_per_workgroup(c, &q);
  if (o_slab + per_wg > kScratchBytes) {
    c->err = "scan (no allocation): " + std::to_string(n_windows) + " windows, " + std::to_string(n_tiles) +
             " tiles and the running minima of one workgroup need " + std::to_string(o_slab + per_wg) +
             " bytes, more than the " + std::to_string(kScratchBytes) + "-byte work array";
    return RKN_E_CAPACITY;
  }
  unsigned char* base = g_ptr[c->device];
  if ((e = hipMemcpyAsync(base + o_win, wins.data(), sizeof(WindowDev) * wins.size(), hipMemcpyHostToDevice,
                          c->stream)) != hipSuccess ||
      (n_tiles > 0 && (e = hipMemcpyAsync(base + o_tiles, tiles.data(), sizeof(Tile) * n_tiles,
                                          hipMemcpyHostToDevice, c->stream)) != hipSuccess) ||
      (e = hipMemcpyAsync(base + o_evt, ev_tiles.data(), sizeof(int32_t) * ev_tiles.size(), hipMemcpyHostToDevice,
                          c->stream)) != hipSuccess) {
    c->err = std::string("scan (no allocation) upload: ") + hipGetErrorString(e);
    return RKN_E_DEVICE;
  }
  e = launch_scan_raw(c, &q, (int64_t)n_tiles, reinterpret_cast<const Tile*>(base + o_tiles),
                      reinterpret_cast<const WindowDev*>(base + o_win), score, n_in, best_index, best_score,
                      reinterpret_cast<const int32_t*>(base + o_evt), reinterpret_cast<ArgminPart*>(base + o_parts),
                      reinterpret_cast<int*>(base + o_counter), base + o_slab, kScratchBytes - o_slab);
  if (e == hipErrorInvalidConfiguration) {
    c->err = "scan configuration does not fit the device (LDS per workgroup); use FP32 or fewer hits per event";
    return RKN_E_UNSUPPORTED;
  }
  if (e != hipSuccess) {
    c->err = std::string("scan (no allocation) launch: ") + hipGetErrorString(e);
    return RKN_E_DEVICE;
  }
  return RKN_OK;
}

}  // extern "C"
