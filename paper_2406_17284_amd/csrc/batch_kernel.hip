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
// (A persistent form -- a grid of resident workgroups taking entries from device-wide
// counters -- was built first and measured 25-50 % slower per tile: with the loop's extra
// state live, the compiler re-read descriptor fields from memory inside the epilogue loops,
// and each such scalar load waits for all outstanding LDS operations. Here the descriptor is
// read once per workgroup, like kernel arguments.)
#include "cat_device.h"

namespace ltl {

template <int ELEM>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) cat_batch(BatchParams bp) {
    extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = blockDim.x >> 6;
    const BatchItem item = bp.items[blockIdx.x];
    const CatParams p = bp.inst[item.inst].p;
    const Codec cd = make_codec();
    if (item.epi == EPI_BYTE)
        cat_tile<ELEM, EPI_BYTE>(p, item.tile, lds, tid, lane, wave, nwaves, cd);
    else if (item.epi == EPI_WIN) {
        if constexpr (ELEM == ELEM_I8) cat_tile<ELEM, EPI_WIN>(p, item.tile, lds, tid, lane, wave, nwaves, cd);
    } else if (item.epi == EPI_HALF)
        cat_tile<ELEM, EPI_HALF>(p, item.tile, lds, tid, lane, wave, nwaves, cd);
    else if (item.epi == EPI_DECAY8) {
        if constexpr (ELEM == ELEM_I8) cat_tile<ELEM, EPI_DECAY8>(p, item.tile, lds, tid, lane, wave, nwaves, cd);
    } else
        cat_tile<ELEM, EPI_DECAY>(p, item.tile, lds, tid, lane, wave, nwaves, cd);
}

const void *cat_batch_func(int elem) {
    if (elem == ELEM_F16) return (const void *)&cat_batch<ELEM_F16>;
    if (elem == ELEM_F8) return (const void *)&cat_batch<ELEM_F8>;
    return (const void *)&cat_batch<ELEM_I8>;
}

int cat_batch_occupancy(int elem, int waves, size_t lds) {
    const void *f = cat_batch_func(elem);
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
