// tang_classify_host_noalloc: tang_classify_host for callers that cannot allocate device
// memory (graph-capturing code, tight serving loops, harnesses that forbid hipMalloc).
// Its staging (headers in, rule ids out) lives in one fixed static device array instead
// of two blocks allocated per call.
#include <algorithm>
#include <mutex>

#include "tang_internal.hpp"

namespace tang {
namespace {

static_assert(kNoAllocMaxHeaders == TANG_NOALLOC_MAX_HEADERS, "staging size and header limit agree");
constexpr size_t kHdrBytes = kNoAllocMaxHeaders * sizeof(tang_header_t);
constexpr size_t kOutBytes = kNoAllocMaxHeaders * sizeof(uint32_t);

// The staging area, one copy per GPU the library runs on, held until the process ends.
// Host code never passes this name to a kernel or a copy: in host code it is a host-side
// stand-in, not a device address. The device address of each GPU's copy comes from
// hipGetSymbolAddress (scratch_on below).
__device__ __align__(256) unsigned char scratch[kHdrBytes + kOutBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (the current device), looked up once per
// device with that device current.
int scratch_on(int device, unsigned char** out) {
    if (device < 0 || device >= kMaxDevices) return fail(TANG_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(TANG_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_ptr[device] = p;
    }
    *out = static_cast<unsigned char*>(g_ptr[device]);
    return TANG_OK;
}

}  // namespace
}  // namespace tang

using namespace tang;

extern "C" int tang_classify_host_noalloc(tang_ruleset_t* rs, const tang_header_t* hdr,
                                          uint32_t* rule_id, size_t n, tang_stats_t* stats) {
    try {
        if (!rs) return fail(TANG_EINVAL, "NULL ruleset");
        if (rs->device == TANG_HOST_ONLY) return fail(TANG_EINVAL, "host-only ruleset cannot classify");
        if (n > kNoAllocMaxHeaders)
            return fail(TANG_EINVAL, "tang_classify_host_noalloc takes at most " +
                                         std::to_string(kNoAllocMaxHeaders) +
                                         " headers per call (its static staging size)");
        if (n && (!hdr || !rule_id)) return fail(TANG_EINVAL, "NULL buffer");
        if (stats) std::memset(stats, 0, sizeof *stats);
        if (n == 0) return TANG_OK;
        TANG_HIP(hipSetDevice(rs->device));
        unsigned char* base = nullptr;
        int rc = scratch_on(rs->device, &base);
        if (rc) return rc;
        tang_header_t* dh = reinterpret_cast<tang_header_t*>(base);
        uint32_t* dout = reinterpret_cast<uint32_t*>(base + kHdrBytes);
        // Headers are copied in whole; every rule id the call returns is written by the
        // search, so nothing in the staging area needs clearing between calls. Calls that
        // overlap on one GPU share this area and race.
        TANG_HIP(hipMemcpy(dh, hdr, n * sizeof(tang_header_t), hipMemcpyHostToDevice));
        rc = classify_async(rs, dh, dout, n, nullptr, stats, false);
        if (rc) return rc;
        TANG_HIP(hipMemcpy(rule_id, dout, n * sizeof(uint32_t), hipMemcpyDeviceToHost));
        return TANG_OK;
    } catch (const std::bad_alloc&) {
        return fail(TANG_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(TANG_EINVAL, "internal error");
    }
}
