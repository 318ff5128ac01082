// Device relayout of Bi-CSR slot arrays: gives rows that ran out of free
// slots room for the inserts of the batch being applied.  Residuals,
// capacities and the pair links move with their slots; excesses and heights
// are per vertex and stay where they are.  Runs entirely on the device: the
// host only reads the new slot count and allocates.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "mf.h"
#include "mf_internal.h"

namespace mf {

namespace {

struct Scratch {
    const DeviceAllocator& mem;
    int64_t *size = nullptr, *start = nullptr, *tile = nullptr;
    int32_t *sort_rows = nullptr, *sort_count = nullptr, *src_of = nullptr, *where = nullptr;
    SlotArrays to{nullptr, nullptr, nullptr, nullptr};
    explicit Scratch(const DeviceAllocator& m) : mem(m) {}
    template <class T>
    hipError_t alloc(T** p, int64_t count) {
        return mem.allocate((void**)p, sizeof(T) * (size_t)(count > 0 ? count : 1));
    }
    template <class T>
    void release(T*& p) {
        mem.release((void*)p);
        p = nullptr;
    }
    ~Scratch() {
        release(size); release(start); release(tile); release(sort_rows); release(sort_count);
        release(src_of); release(where);
        release(to.cr); release(to.rev); release(to.cap); release(to.capsum);
    }
};

}  // namespace

mf_status relayout_device(RelayoutPlan p, SlotArrays* arrays, int64_t S_old, int64_t* S_new, int32_t* row_ptr,
                          int32_t* row_sorted, hipStream_t st, const DeviceAllocator& mem) {
    Scratch x(mem);
    if (x.alloc(&x.size, p.V) || x.alloc(&x.start, (int64_t)p.V + 1) || x.alloc(&x.tile, relayout_tiles(p.V)) ||
        x.alloc(&x.sort_rows, p.V) || x.alloc(&x.sort_count, 1))
        return MF_ERR_OUT_OF_MEMORY;
    p.size = x.size;
    p.start = x.start;
    p.tile = x.tile;
    p.sort_rows = x.sort_rows;
    p.sort_count = x.sort_count;
    launch_relayout_plan(p, st);
    if (hipGetLastError() != hipSuccess) return MF_ERR_DEVICE;
    int64_t total = 0;
    int32_t sorts = 0;
    if (hipMemcpyAsync(&total, x.start + p.V, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&sorts, x.sort_count, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return MF_ERR_DEVICE;
    if (total < S_old || total > (int64_t)INT_MAX - 1) return MF_ERR_OVERFLOW;
    if (x.alloc(&x.src_of, total) || x.alloc(&x.where, S_old) || x.alloc(&x.to.cr, total) ||
        x.alloc(&x.to.rev, total) || x.alloc(&x.to.cap, total) || x.alloc(&x.to.capsum, total))
        return MF_ERR_OUT_OF_MEMORY;
    launch_relayout_move(p, sorts, total, *arrays, x.to, x.src_of, x.where, row_ptr, row_sorted, st);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return MF_ERR_DEVICE;
    // swap: the old arrays are released with the scratch
    SlotArrays old = *arrays;
    *arrays = x.to;
    x.to = old;
    *S_new = total;
    return MF_OK;
}

}  // namespace mf
