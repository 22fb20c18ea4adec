// gf_noalloc.hip -- the reduction region of gf_reduce on a static device
// array instead of the context's allocated scratch, for callers that cannot
// allocate device memory at call time (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// The array holds one 256-byte counter line and kNaPartials per-workgroup
// partials. Each device has its own copy at its own address; host code
// never names the array after set-up, only the address hipGetSymbolAddress
// returned for that device. Every call on a device shares that device's
// copy: calls that overlap on one GPU (two streams, two host threads)
// race and give wrong results.
#include <mutex>

#include "gf_internal.h"

namespace gf {
namespace {
constexpr int64_t kNaPartials = 1024;  // 8-byte partials: the grid never exceeds this many workgroups
constexpr size_t kNaLine = 256;        // counter line (its first word counts finished workgroups)
constexpr size_t kNaBytes = kNaLine + (size_t)kNaPartials * 8;
constexpr int kNaMaxDevices = 64;
}  // namespace
}  // namespace gf

static __device__ __align__(256) unsigned char scratch[gf::kNaBytes];

namespace gf {
namespace {
std::mutex g_na_mu;
void *g_na_ptr[kNaMaxDevices];  // per device: the array's device address
}  // namespace

size_t noalloc_scratch_bytes() { return kNaBytes; }

// Resolve `device`'s copy of the array (device current) and clear its
// counter line; once per device, later calls return at once.
hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= kNaMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_na_mu);
    if (g_na_ptr[device])
        return hipSuccess;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess)
        return e;
    if (!p)
        return hipErrorInvalidSymbol;
    // a kernel, not a memset, clears the counter (memset nodes are kept out
    // of anything a caller may capture)
    if ((e = launch_clear_u32((uint32_t *)p, (int32_t)(kNaLine / 4), nullptr)) != hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(nullptr)) != hipSuccess)
        return e;
    g_na_ptr[device] = p;
    return hipSuccess;
}

// The address set-up resolved for `device`, or nullptr before set-up.
void *noalloc_ptr(int device)
{
    if (device < 0 || device >= kNaMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> g(g_na_mu);
    return g_na_ptr[device];
}

// Enqueue the reduction on `device`'s array (device current, set up): clear
// the counter word with a small kernel, then the two-level reduction with
// at most kNaPartials workgroups. Allocates nothing.
hipError_t noalloc_reduce(int device, int num_cu, int op, int dt, const void *in, int64_t n, void *out,
                          hipStream_t s, int64_t *grid_out)
{
    char *p = (char *)noalloc_ptr(device);
    if (!p)
        return hipErrorNotInitialized;
    const int64_t g = reduce_grid(n, num_cu, kNaPartials);
    if (g < 1 || g > kNaPartials)
        return hipErrorInvalidValue;
    if (grid_out)
        *grid_out = g;
    uint32_t *cnt = (uint32_t *)p;
    hipError_t e = launch_clear_u32(cnt, 1, s);
    if (e != hipSuccess)
        return e;
    return launch_reduce_into(op, dt, in, n, out, p + kNaLine, cnt, g, s);
}

}  // namespace gf
