// Allocation-free GMRES entry point: sa_gmres_solve with every workspace
// buffer carved from one statically sized device array instead of memory the
// context allocates, for callers that cannot allocate device memory.
//
// The array is a file-scope __device__ variable.  Its name in host code is a
// host-side stand-in, not a device address, so its device address is
// resolved once per device with hipGetSymbolAddress (sa_create calls
// scratch_init with the device current) and only that address is handed to
// kernels.  Each device holds one copy for the life of the process; every
// call on a device shares it and keeps the last call's contents, so buffers
// that must start at zero are cleared by a kernel in each call, and calls
// that overlap on one device (contexts on different streams) race.
#include <cstring>
#include <mutex>

#include "sa_runtime.h"

namespace sa {
namespace {

constexpr size_t SCRATCH_BYTES = SA_NOALLOC_SCRATCH_BYTES;
static_assert(SCRATCH_BYTES % 256 == 0, "scratch size");

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};            // device address of `scratch` per device
hipError_t g_err[MAX_DEVICES] = {};       // result of its resolution
bool g_done[MAX_DEVICES] = {};

__global__ void zero_fill_kernel(uint4* __restrict__ p, size_t n16) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = t; i < n16; i += stride) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

void zero_fill(void* p, size_t bytes, hipStream_t s) {
  const size_t n16 = (bytes + 15) / 16;
  if (n16 == 0) return;
  const size_t blocks = std::min<size_t>((n16 + 255) / 256, 2048);
  zero_fill_kernel<<<(unsigned)blocks, 256, 0, s>>>(reinterpret_cast<uint4*>(p), n16);
}

void scratch_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_done[device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_err[device] = e;
  g_ptr[device] = e == hipSuccess ? ptr : nullptr;
  g_done[device] = true;
}

}  // namespace sa

using namespace sa;

extern "C" int sa_gmres_solve_noalloc(sa_ctx* c, const sa_gmres_opts* o, int nshift, const double* sigma_host,
                                      const void* b_dev, void* x_dev, sa_gmres_info* info) {
  if (!c) return SA_EINVAL;
  const char* who = "sa_gmres_solve_noalloc";
  int rc = gmres_check(c, o, nshift, sigma_host, b_dev, x_dev, info, who);
  if (rc != SA_OK) return rc;
  if (c->device < 0 || c->device >= MAX_DEVICES) return c->fail(SA_EDEVICE, "%s: device %d out of range", who, c->device);
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_done[c->device]) return c->fail(SA_EDEVICE, "%s: scratch of device %d not resolved", who, c->device);
    if (g_err[c->device] != hipSuccess)
      return c->fail(SA_EDEVICE, "%s: hipGetSymbolAddress: %s", who, hipGetErrorString(g_err[c->device]));
    base = g_ptr[c->device];
  }
  sa_gmres_opts oo = *o;
  oo.use_graph = 0;   // captured cycles need a capture stream and graph memory
  const size_t need = gmres_workspace_bytes(c, oo, nshift);
  if (need > SCRATCH_BYTES)
    return c->fail(SA_EINVAL,
                   "%s: the solve needs %zu bytes of workspace (n = %lld, %d systems, restart %d, augment %d), "
                   "more than the %zu-byte scratch; use sa_gmres_solve",
                   who, need, c->n, nshift, oo.restart, oo.augment, SCRATCH_BYTES);
  Ctx::Arena arena;
  arena.base = static_cast<unsigned char*>(base);
  arena.cap = SCRATCH_BYTES;
  c->arena = &arena;
  rc = gmres_dispatch(c, oo, nshift, sigma_host, b_dev, x_dev, info);
  c->arena = nullptr;
  return rc;
}
