// noalloc.hip -- the demag evaluation of mm_demag_apply for callers that
// cannot allocate device memory at all (code under HIP graph capture, tight
// serving loops, harnesses that forbid allocation): the half-spectrum
// buffers X1 and X2 live in a file-scope device array of fixed size instead
// of the plan's workspace.  The plan still supplies K~ and the twiddles.
#include <mutex>

#include "mm_internal.hpp"

namespace mmk {

// The array's size bounds the grids this entry point takes.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)64 << 20;

// Every GPU the library runs on holds its own copy until the process ends.
// Host code never uses this name as an address: the device address comes
// from hipGetSymbolAddress, once per device.
static __device__ __align__(256) char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[MAX_DEVICES];  // device ordinal -> address of `scratch` there

// Address of `scratch` on device `dev`, looked up with that device current.
static int scratch_on(int dev, char **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return fail(MM_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) {
        *out = g_scratch_ptr[dev];
        return MM_OK;
    }
    int cur = 0;
    MMK_HIP(hipGetDevice(&cur));
    if (cur != dev) MMK_HIP(hipSetDevice(dev));
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr)
        return fail(MM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (char *)ptr;
    *out = (char *)ptr;
    return MM_OK;
}

// Bytes of X1 and X2 for a plan, each rounded to 256.
static size_t static_need(const Plan &p)
{
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t x1 = sizeof(float2) * 3 * (size_t)p.nz * p.ny * p.xp;
    const size_t x2 = p.nz > 1 ? sizeof(float2) * 3 * (size_t)p.nz * x2_plane_stride(p.Ly, p.xp) : 0;
    return al(x1) + al(x2);
}

}  // namespace mmk

using namespace mmk;

extern "C" {

size_t mm_demag_static_scratch_bytes(void) { return STATIC_SCRATCH_BYTES; }

int mm_demag_apply_static(mm_plan plan, const float *M, float *H, void *stream)
{
    Plan *p = plan_of(plan);
    int rc = plan_ready(p);
    if (rc != MM_OK) return rc;
    if (!M || !H) return fail(MM_EINVAL, "NULL pointer");
    if ((const void *)M == (const void *)H) return fail(MM_EINVAL, "M and H alias");
    const size_t need = static_need(*p);
    if (need > STATIC_SCRATCH_BYTES)
        return fail(MM_EINVAL, "grid needs " + std::to_string(need) + " bytes of half spectra; the static scratch holds " +
                                   std::to_string(STATIC_SCRATCH_BYTES));
    char *base = nullptr;
    if ((rc = scratch_on(p->device, &base)) != MM_OK) return rc;
    const size_t x1 = (sizeof(float2) * 3 * (size_t)p->nz * p->ny * p->xp + 255) & ~(size_t)255;
    float2 *keep1 = p->X1, *keep2 = p->X2;
    // the launches take the buffer addresses as arguments when enqueued, so
    // the plan's own buffers are back in place as soon as this returns
    p->X1 = reinterpret_cast<float2 *>(base);
    p->X2 = p->nz > 1 ? reinterpret_cast<float2 *>(base + x1) : nullptr;
    rc = demag_enqueue(*p, M, H, (hipStream_t)stream);
    p->X1 = keep1;
    p->X2 = keep2;
    return rc;
}

}  // extern "C"
