// Scratch memory of the allocation-free repair (mf_apply_batch_device_noalloc).
//
// One static device array per GPU holds the batch scratch that
// mf_apply_batch_device otherwise allocates per handle: the slot located for
// each update, the updates that changed a capacity, and the hash table of
// absent pairs.  Host code never passes the array's name to a kernel: its
// device address is looked up once per device with hipGetSymbolAddress (with
// that device current) and kept here.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "mf.h"
#include "mf_internal.h"

namespace mf {

namespace {

constexpr size_t KEY_BYTES = sizeof(unsigned long long) * (size_t)NOALLOC_TABLE;
constexpr size_t WIN_BYTES = sizeof(int32_t) * 2 * (size_t)NOALLOC_TABLE;
constexpr size_t SLOT_BYTES = sizeof(int32_t) * 2 * (size_t)NOALLOC_TABLE;
constexpr size_t LIST_BYTES = sizeof(int32_t) * (size_t)NOALLOC_MAX_UPDATES;
constexpr size_t SCRATCH_BYTES = KEY_BYTES + WIN_BYTES + SLOT_BYTES + 2 * LIST_BYTES;

// every part starts on a 256-byte boundary
static_assert(KEY_BYTES % 256 == 0 && WIN_BYTES % 256 == 0 && LIST_BYTES % 256 == 0, "layout");

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex addr_mu;
unsigned char* addr[MAX_DEVICES] = {};

}  // namespace

mf_status noalloc_scratch(int device, NoallocScratch* out) {
    if (device < 0 || device >= MAX_DEVICES) return MF_ERR_INVALID;
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(addr_mu);
        if (!addr[device]) {
            // the caller made `device` current; each GPU has its own copy of the array
            void* p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
                (void)hipGetLastError();
                return MF_ERR_DEVICE;
            }
            addr[device] = static_cast<unsigned char*>(p);
        }
        base = addr[device];
    }
    out->table_key = reinterpret_cast<unsigned long long*>(base);
    out->table_win = reinterpret_cast<int32_t*>(base + KEY_BYTES);
    out->table_slot = reinterpret_cast<int32_t*>(base + KEY_BYTES + WIN_BYTES);
    out->slot_of = reinterpret_cast<int32_t*>(base + KEY_BYTES + WIN_BYTES + SLOT_BYTES);
    out->touched = reinterpret_cast<int32_t*>(base + KEY_BYTES + WIN_BYTES + SLOT_BYTES + LIST_BYTES);
    out->bytes = SCRATCH_BYTES;
    return MF_OK;
}

}  // namespace mf
