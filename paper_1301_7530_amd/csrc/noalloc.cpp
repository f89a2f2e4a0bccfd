// Allocation-free variant of the basis export: krs_seq_basis_noalloc.
//
// krs_seq_basis converts each column of the device basis to double in a
// staging buffer the library allocates (n doubles) and copies it to the
// caller.  The variant here stages through `scratch`, a file-scope device
// array of kScratchBytes, so that it calls no allocating routine.  Host code
// never uses the array's name as an address: the device address is looked
// up once per device (noalloc_init, called by krs_ctx_create with the device
// current) and kept in g_scratch_ptr.
#include <mutex>

#include "seq.h"

namespace krs {

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB: n <= 4,194,304
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

krs_status noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("device index beyond the scratch table");
        return KRS_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return KRS_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        set_error(std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        return KRS_E_DEVICE;
    }
    g_scratch_ptr[device] = ptr;
    return KRS_OK;
}

size_t noalloc_scratch_bytes() { return kScratchBytes; }

void* noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace krs
