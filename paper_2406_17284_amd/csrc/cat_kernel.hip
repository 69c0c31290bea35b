// Single-grid CAT step kernel and its launchers; the per-tile device code (method, operand
// layouts, precision variants, temporal blocking) is in cat_device.h.
#include "cat_device.h"

namespace ltl {

// One workgroup per tile; workgroups of one XCD take consecutive tiles, so the halos of
// neighbouring tiles meet in that XCD's L2.
template <int ELEM, int EPI>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) cat_step(CatParams p) {
    extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: keeps item code scalar
    const int nwaves = blockDim.x >> 6;

    // The grid is the tile count rounded up to a multiple of 8: workgroup b runs on XCD b mod 8,
    // which takes the contiguous block of tiles (b mod 8) * nb/8 ...; surplus workgroups exit.
    const int ntiles = p.ntx * p.nty;
    const int nb = gridDim.x;
    const int bid = blockIdx.x;
    const int tile = (bid & 7) * (nb >> 3) + (bid >> 3);
    if (tile >= ntiles) return;
    const Codec cd = make_codec();
    cat_tile<ELEM, EPI>(p, tile, lds, tid, lane, wave, nwaves, cd);
}
size_t cat_lds_bytes(const CatParams &p, int elem, int epi) {
    (void)elem;
    (void)epi;
    return (size_t)p.lds_total;
}

static const void *cat_func(int elem, int epi) {
#define CAT_F(E) \
    (epi == EPI_BYTE ? (const void *)&cat_step<E, EPI_BYTE> : epi == EPI_HALF ? (const void *)&cat_step<E, EPI_HALF> \
                                                                             : (const void *)&cat_step<E, EPI_DECAY>)
    if (elem == ELEM_F16) return CAT_F(ELEM_F16);
    if (elem == ELEM_F8) return CAT_F(ELEM_F8);
    if (elem == ELEM_I8X)   // cross counts are at most 4r + 1 <= 65: no 16-bit epilogue
        return epi == EPI_DECAY ? (const void *)&cat_step<ELEM_I8X, EPI_DECAY> : (const void *)&cat_step<ELEM_I8X, EPI_BYTE>;
    if (elem == ELEM_I8W)   // radii 17..32 always have counts > 126: no 8-bit epilogue
        return epi == EPI_DECAY ? (const void *)&cat_step<ELEM_I8W, EPI_DECAY> : (const void *)&cat_step<ELEM_I8W, EPI_HALF>;
    return CAT_F(ELEM_I8);
#undef CAT_F
}

int cat_occupancy(const CatParams &p, int elem, int epi, int waves) {
    const void *f = cat_func(elem, epi);
    size_t lds = cat_lds_bytes(p, elem, epi);
    if (lds > 65536 && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, 64 * waves, lds) != hipSuccess) return 0;
    return nb;
}

KernelLaunch cat_launch_shape(const CatParams &p, int elem, int epi, int waves) {
    KernelLaunch k;
    k.func = cat_func(elem, epi);
    k.lds = cat_lds_bytes(p, elem, epi);
    k.grid = dim3((unsigned)roundup(p.ntx * p.nty, 8), 1, 1);
    k.block = dim3(64 * waves, 1, 1);
    return k;
}

hipError_t launch_cat(const CatParams &p, int elem, int epi, int waves, hipStream_t s) {
    KernelLaunch k = cat_launch_shape(p, elem, epi, waves);
    if (k.lds > 65536) {
        hipError_t e = hipFuncSetAttribute(k.func, hipFuncAttributeMaxDynamicSharedMemorySize, (int)k.lds);
        if (e != hipSuccess) return e;
    }
    void *args[] = {(void *)&p};
    return hipLaunchKernel(k.func, k.grid, k.block, args, k.lds, s);
}

}  // namespace ltl

