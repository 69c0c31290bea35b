// Batched CAT step: many independent automata of different sizes, radii and rules advance in
// one launch per T steps.
//
// The host lays out the work list: an entry per (instance, tile), sorted by decreasing
// estimated cost (longest first). The launch has one workgroup per entry; the hardware
// dispatcher starts workgroups in index order as compute units free up, so the most expensive
// tiles start first and the cheap ones fill the tail. Each entry's instance descriptor
// carries its launch parameters (grid, radius, band operands, rule constants, tile shape,
// LDS layout), and the entry runs the same per-tile code as the single-grid kernel with the
// epilogue of its instance's rule.
//
// A persistent form (cat_batch_persist, below) is offered as a tuning option; it spills at the
// register budget of two 8-wave workgroups per compute unit and measures slower than this one.
#include "cat_device.h"

namespace ltl {

// Work-list entry k: its instance descriptor is read once, then the single-grid tile code runs
// with the epilogue of the instance's rule.
template <int ELEM, class Side = NoSideLoad>
__device__ __forceinline__ void batch_entry(const BatchParams &bp, int k, uint8_t *lds, int tid, int lane, int wave,
                                            int nwaves, const Codec &cd, Side &&side = Side()) {
    const BatchItem item = bp.items[k];
    const CatParams p = bp.inst[item.inst].p;
    if (item.epi == EPI_BYTE)
        cat_tile<ELEM, EPI_BYTE>(p, item.tile, lds, tid, lane, wave, nwaves, cd, side);
    else if (item.epi == EPI_WIN) {
        if constexpr (ELEM == ELEM_I8) cat_tile<ELEM, EPI_WIN>(p, item.tile, lds, tid, lane, wave, nwaves, cd, side);
    } else if (item.epi == EPI_HALF)
        cat_tile<ELEM, EPI_HALF>(p, item.tile, lds, tid, lane, wave, nwaves, cd, side);
    else if (item.epi == EPI_DECAY8) {
        if constexpr (ELEM == ELEM_I8) cat_tile<ELEM, EPI_DECAY8>(p, item.tile, lds, tid, lane, wave, nwaves, cd, side);
    } else if (item.epi == EPI_WIN8) {
        if constexpr (ELEM == ELEM_I8) cat_tile<ELEM, EPI_WIN8>(p, item.tile, lds, tid, lane, wave, nwaves, cd, side);
    } else if (item.epi == EPI_DECAY8W) {
        if constexpr (ELEM == ELEM_I8) cat_tile<ELEM, EPI_DECAY8W>(p, item.tile, lds, tid, lane, wave, nwaves, cd, side);
    } else
        cat_tile<ELEM, EPI_DECAY>(p, item.tile, lds, tid, lane, wave, nwaves, cd, side);
}

template <int ELEM>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) cat_batch(BatchParams bp) {
    extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    batch_entry<ELEM>(bp, blockIdx.x, lds, tid, tid & 63, wave, blockDim.x >> 6, make_codec());
}

// The persistent form's draw of its next entry, overlapped with the current tile's window load:
// thread 0 adds one to its XCD's entry counter when the loads are issued and stores the entry
// that draw names into an LDS slot once they landed, so no register stays live across the
// tile's steps.
struct DrawNext {
    uint32_t *counter;   // this XCD's next-entry counter
    int32_t *slot;
    int32_t first;       // entry of draw 0: gridDim.x + the XCD index
    uint32_t drawn;
    __device__ __forceinline__ void issue(int tid) {
        if (tid == 0) drawn = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ void land(int tid) {
        if (tid == 0) *slot = first + 8 * (int32_t)drawn;
    }
};

// Persistent form (tuning.persistent = 1): a grid of resident workgroups (a multiple of 8: the
// co-resident slots, capped by the entry count) walks the work list. The list is laid out for
// workgroup k running on XCD k mod 8, and each XCD keeps to its own entries: workgroup b starts
// with entry b, then draws entries gridDim.x + 8 j + (b mod 8), j = 0, 1, ... from a counter of
// its XCD, while the current entry's window loads. A workgroup that draws an index past the
// list leaves the loop and counts itself in a last counter; the last one to do so resets every
// counter to zero, so each launch (and each replay of a graph holding it) starts from zero. No
// workgroup waits on another, so the form needs no co-residency guarantee.
template <int ELEM>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) cat_batch_persist(BatchParams bp) {
    extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
    __shared__ int32_t next_entry[2];   // alternate slots: a slot is rewritten two entries later,
                                        // after every wave passed the barrier that follows its read
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = blockDim.x >> 6;
    const Codec cd = make_codec();
    const int xcd = blockIdx.x & 7;
    int k = blockIdx.x;
    int slot = 0;
    while (k < bp.nitems) {
        batch_entry<ELEM>(bp, k, lds, tid, lane, wave, nwaves, cd,
                          DrawNext{bp.counters + xcd, next_entry + slot, (int32_t)gridDim.x + xcd, 0u});
        __syncthreads();   // every wave is done with the tile's LDS
        k = __builtin_amdgcn_readfirstlane(next_entry[slot]);
        slot ^= 1;
    }
    if (tid == 0) {
        const uint32_t done = __hip_atomic_fetch_add(bp.counters + 8, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {   // every workgroup has drawn its last index
            for (int c = 0; c < 9; ++c) __hip_atomic_store(bp.counters + c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

const void *cat_batch_func(int elem, int persistent) {
    if (persistent) {
        if (elem == ELEM_F16) return (const void *)&cat_batch_persist<ELEM_F16>;
        if (elem == ELEM_F8) return (const void *)&cat_batch_persist<ELEM_F8>;
        return (const void *)&cat_batch_persist<ELEM_I8>;
    }
    if (elem == ELEM_F16) return (const void *)&cat_batch<ELEM_F16>;
    if (elem == ELEM_F8) return (const void *)&cat_batch<ELEM_F8>;
    return (const void *)&cat_batch<ELEM_I8>;
}

int cat_batch_occupancy(int elem, int waves, size_t lds, int persistent) {
    const void *f = cat_batch_func(elem, persistent);
    // a shape the device cannot run reads as zero workgroups; its HIP error is not left pending
    if (lds > 65536 && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, 64 * waves, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

}  // namespace ltl
