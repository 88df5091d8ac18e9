// h2dlp_apply_noalloc: the apply with its workspace in a fixed device array of
// the library, for callers that cannot allocate device memory.
//
// The array `scratch` exists once per GPU the library runs on, from the load
// of the library until the process ends.  Its address on a device comes from
// hipGetSymbolAddress, taken once per device with that device current; host
// code passes that address to the kernels (never the array's name, which in
// host code is not a device address).  The apply needs nothing in it to start
// at zero: every workspace value is written before it is read.  All calls on
// one GPU share the array, so calls that overlap on one GPU (other streams,
// other threads, other handles) race; the caller runs them one at a time.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/h2dlp.h"
#include "entry.h"

namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;   // H2DLP_NOALLOC_SCRATCH_BYTES
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

}  // namespace

static_assert(kScratchBytes == H2DLP_NOALLOC_SCRATCH_BYTES, "header and library disagree on the scratch size");

extern "C" int h2dlp_apply_noalloc(h2dlp_handle h, const void* u1, void* u2, int nrhs, int io_dtype, void* stream) {
    using h2dlp::set_error;
    if (h == nullptr) return set_error(H2DLP_EINVAL, "handle is NULL");
    const int dev = h2dlp::handle_device(h);
    if (dev < 0) return set_error(H2DLP_EINVAL, "handle comes from h2dlp_plan: nothing on the device");
    if (dev >= kMaxDevices) return set_error(H2DLP_ENOTSUP, "device ordinal beyond the scratch table");
    h2dlp_stats st;
    const int rc = h2dlp_info(h, &st);
    if (rc != H2DLP_OK) return rc;
    if (size_t(st.workspace_bytes) > kScratchBytes)
        return set_error(H2DLP_ENOMEM, "the operator needs " + std::to_string(st.workspace_bytes) +
                                           " bytes of workspace, the library's scratch holds " +
                                           std::to_string(kScratchBytes) +
                                           ": use h2dlp_apply_ex with a caller workspace");
    void* ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (g_scratch[dev] == nullptr) {
            int cur = 0;
            if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(dev) != hipSuccess)
                return set_error(H2DLP_EDEVICE, "hipSetDevice failed");
            void* p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            (void)hipSetDevice(cur);
            if (e != hipSuccess || p == nullptr)
                return set_error(H2DLP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            g_scratch[dev] = p;
        }
        ws = g_scratch[dev];
    }
    return h2dlp::apply_entry(h, u1, u2, nrhs, io_dtype, stream, ws, kScratchBytes, true);
}
