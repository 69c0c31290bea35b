// Batched CAT step: many independent automata of different sizes, radii and rules advance in
// one persistent launch per T steps.
//
// The host lays out the work list: an entry per (instance, tile), grouped by the epilogue
// class of the instance's rule and sorted by decreasing estimated cost within a class. A grid
// of (resident workgroups per CU) x (CUs) workgroups drains the classes in turn, taking entries
// from a device-wide counter per class, so the most expensive tiles start first and the tail
// is balanced dynamically. Each entry's instance descriptor carries its launch parameters
// (grid, radius, band operands, rule constants, tile shape, LDS layout), and the entry runs
// the same per-tile code as the single-grid kernel. (One loop per class keeps each loop's
// register allocation that of a single-rule kernel.)
//
// Counter protocol: queue[c] numbers the takes of class c in a launch, queue[3] counts the
// workgroups that have finished. A workgroup takes from class c until it gets an index
// >= count[c], exactly once per workgroup and class; the last workgroup to finish (all others
// have made all of their takes by then) rewinds every counter to 0 for the next launch.
#include "cat_device.h"

namespace ltl {

// Take entries of one epilogue class until its list is exhausted. The slot a wave reads after
// an entry's closing barrier is written again two entries later, after a barrier that every
// wave reaches only once it has read it.
template <int ELEM, int EPI>
__device__ __forceinline__ void drain_class(const BatchParams &bp, uint8_t *lds, uint32_t *slot, int tid, int lane,
                                            int wave, int nwaves, const Codec &cd) {
    const uint32_t n = (uint32_t)bp.count[EPI];
    if (n == 0) return;
    const BatchItem *items = bp.items + bp.start[EPI];
    uint32_t *queue = bp.queue + EPI;
    __syncthreads();   // the previous class's last slot read is done
    if (tid == 0) slot[0] = atomicAdd(queue, 1u);
    __syncthreads();
    uint32_t k = __builtin_amdgcn_readfirstlane(slot[0]);
    int it = 1;
    while (k < n) {
        const BatchItem item = items[k];
        // read through the constant address space: the descriptor is invariant for the launch,
        // so its fields load like kernel arguments (scalar loads the compiler may repeat
        // instead of keeping them live), which keeps the tile code within its register budget
        typedef __attribute__((address_space(4))) const BatchInst cinst;
        const CatParams &p = *(const CatParams *)&((const cinst *)bp.inst)[item.inst].p;
        // take the next entry now; the tile code stores it to the slot once its own loads
        // have been waited for
        uint32_t next = 0;
        if (tid == 0) next = atomicAdd(queue, 1u);
        cat_tile<ELEM, EPI>(p, item.tile, lds, tid, lane, wave, nwaves, cd, slot + it, next);
        __syncthreads();   // every wave is done with this tile's LDS before the next load
        k = __builtin_amdgcn_readfirstlane(slot[it]);
        it ^= 1;
    }
}

// Classes run in a fixed order, the 16-bit-count class (large radii, dearest entries) first
// and the 8-bit-count class (r <= 5) last, so the launch ends on its cheapest entries.
template <int ELEM>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) cat_batch(BatchParams bp) {
    extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = blockDim.x >> 6;
    uint32_t *slot = reinterpret_cast<uint32_t *>(lds + bp.slot);   // two dwords, used alternately
    const Codec cd = make_codec();

    drain_class<ELEM, EPI_HALF>(bp, lds, slot, tid, lane, wave, nwaves, cd);
    drain_class<ELEM, EPI_DECAY>(bp, lds, slot, tid, lane, wave, nwaves, cd);
    drain_class<ELEM, EPI_BYTE>(bp, lds, slot, tid, lane, wave, nwaves, cd);
    if (tid == 0) {
        const uint32_t d = atomicAdd(&bp.queue[3], 1u);
        if (d == gridDim.x - 1) {   // every other workgroup has made all of its takes
            atomicExch(&bp.queue[0], 0u);
            atomicExch(&bp.queue[1], 0u);
            atomicExch(&bp.queue[2], 0u);
            atomicExch(&bp.queue[3], 0u);
        }
    }
}

const void *cat_batch_func(int elem) {
    if (elem == ELEM_F16) return (const void *)&cat_batch<ELEM_F16>;
    if (elem == ELEM_F8) return (const void *)&cat_batch<ELEM_F8>;
    return (const void *)&cat_batch<ELEM_I8>;
}

int cat_batch_occupancy(int elem, int waves, size_t lds) {
    const void *f = cat_batch_func(elem);
    if (lds > 65536 && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, 64 * waves, lds) != hipSuccess) return 0;
    return nb;
}

}  // namespace ltl
