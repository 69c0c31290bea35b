// Single-grid CAT step kernel and its launchers; the per-tile device code (method, operand
// layouts, precision variants, temporal blocking) is in cat_device.h.
#include <algorithm>

#include "cat_device.h"

namespace ltl {

// One workgroup per tile; workgroups of one XCD take consecutive tiles, so the halos of
// neighbouring tiles meet in that XCD's L2.
//
// FIXED != 0: a copy of the kernel for one launch-shape class, picked by the launcher where the
// launch belongs to it: 224-column tiles with a 32-cell margin and no LDS padding (row pitch
// FIXED = 304 for states and alive bits alike), and with THC != 0 also tiles of THC rows. With
// these compile-time constants the block-row offsets of the LDS accesses become instruction
// offsets instead of per-block address arithmetic (with phase B's SPLIT form of the state
// accesses), each step's extent is known (a 32-cell margin leaves 16 for every step but the
// last), and with the height fixed the guards of the unrolled block loops fold away (and the
// last step runs as a copy of its own, so every step's geometry is a constant).
template <int ELEM, int EPI, int FIXED = 0, int THC = 0>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) cat_step(CatParams p) {
    if constexpr (FIXED != 0) {
        p.PS = FIXED;
        p.PA = FIXED;
        p.TW = 224;
        p.L = 32;
    }
    if constexpr (THC != 0) p.TH = THC;
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
    cat_tile<ELEM, EPI, NoSideLoad, FIXED == 0 ? 0 : THC == 0 ? 1 : 2>(p, tile, lds, tid, lane, wave, nwaves, cd);
}

// Persistent form (tuning.persistent = 1), for grids whose tiles stream from HBM: one
// workgroup per CU slot walks
// a static sequence of tiles with two LDS buffers, so the next tile's direct loads are in
// flight while the current tile computes. Workgroup b runs on XCD b mod 8 and takes every gx-th
// tile (gx = workgroups per XCD) of that XCD's contiguous block of tiles, so the tiles one XCD
// processes at a time are neighbours and share its L2.
template <int ELEM, int EPI>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) cat_persist(CatParams p) {
    extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = blockDim.x >> 6;
    const int ntiles = p.ntx * p.nty;
    const int gx = gridDim.x >> 3;                 // the grid is a multiple of 8 workgroups
    const int chunk = (ntiles + 7) >> 3;
    const int t_hi = min(ntiles, ((int)blockIdx.x & 7) * chunk + chunk);
    int tile = ((int)blockIdx.x & 7) * chunk + ((int)blockIdx.x >> 3);
    const float inv_ps = __builtin_amdgcn_rcpf((float)p.PS);   // estimate: row_col corrects it
    const Codec cd = make_codec();
    const Bands bd = load_bands<ELEM>(p, lane, cd);
    const uint32_t bufsz = (uint32_t)p.lds_total;  // one buffer: state tile (+ alive tile)
    if (tile < t_hi)
        issue_tile_load(p, (tile / p.ntx) * p.TH, (tile % p.ntx) * p.TW, lds, wave, nwaves, lane, inv_ps);
    uint32_t buf = 0;
    while (tile < t_hi) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();   // this tile's window landed; every wave is done with the other buffer
        const int next = tile + gx;
        if (next < t_hi)
            issue_tile_load(p, (next / p.ntx) * p.TH, (next % p.ntx) * p.TW, lds + (buf ^ bufsz), wave, nwaves,
                            lane, inv_ps);
        uint8_t *Qt = lds + buf;
        tile_steps<ELEM, EPI>(p, (tile / p.ntx) * p.TH, (tile % p.ntx) * p.TW, Qt, Qt + p.a_tile, tid, lane, wave,
                              nwaves, bd, cd);
        tile = next;
        buf ^= bufsz;
    }
}

size_t cat_lds_bytes(const CatParams &p, int elem, int epi, int persistent) {
    (void)elem;
    (void)epi;
    return (size_t)p.lds_total * (persistent ? 2 : 1);
}

// Kernel symbol of an (element, epilogue) pair; KERNEL is cat_step or cat_persist.
#define CAT_PICK(KERNEL)                                                                                           \
    static const void *KERNEL##_func(int elem, int epi) {                                                          \
        const bool dec = (epi == EPI_DECAY);                                                                       \
        if (elem == ELEM_F16)                                                                                      \
            return dec ? (const void *)&KERNEL<ELEM_F16, EPI_DECAY>                                                \
                       : epi == EPI_HALF ? (const void *)&KERNEL<ELEM_F16, EPI_HALF> : (const void *)&KERNEL<ELEM_F16, EPI_BYTE>; \
        if (elem == ELEM_F8)                                                                                       \
            return dec ? (const void *)&KERNEL<ELEM_F8, EPI_DECAY>                                                 \
                       : epi == EPI_HALF ? (const void *)&KERNEL<ELEM_F8, EPI_HALF> : (const void *)&KERNEL<ELEM_F8, EPI_BYTE>; \
        if (elem == ELEM_I8X)   /* cross counts are at most 4r + 1 <= 65: no 16-bit epilogue */                   \
            return dec ? (const void *)&KERNEL<ELEM_I8X, EPI_DECAY> : (const void *)&KERNEL<ELEM_I8X, EPI_BYTE>;   \
        if (elem == ELEM_I8W)   /* radii 17..32 always have counts > 126: no 8-bit epilogue */                     \
            return dec ? (const void *)&KERNEL<ELEM_I8W, EPI_DECAY> : (const void *)&KERNEL<ELEM_I8W, EPI_HALF>;   \
        if (epi == EPI_WIN) return (const void *)&KERNEL<ELEM_I8, EPI_WIN>;                                        \
        if (epi == EPI_WIN8) return (const void *)&KERNEL<ELEM_I8, EPI_WIN8>;                                      \
        if (epi == EPI_DECAY8) return (const void *)&KERNEL<ELEM_I8, EPI_DECAY8>;                                  \
        if (epi == EPI_DECAY8W) return (const void *)&KERNEL<ELEM_I8, EPI_DECAY8W>;                                \
        return dec ? (const void *)&KERNEL<ELEM_I8, EPI_DECAY>                                                     \
                   : epi == EPI_HALF ? (const void *)&KERNEL<ELEM_I8, EPI_HALF> : (const void *)&KERNEL<ELEM_I8, EPI_BYTE>; \
    }
CAT_PICK(cat_step)
CAT_PICK(cat_persist)
#undef CAT_PICK

// The fixed shape class: 224-column tiles, a 32-cell margin (steps per launch T with
// r (T - 1) <= 16), no LDS padding: row pitch TW + 2L + 16 = 304. The tuning table holds it for
// most int8 Moore rules on large grids (192 rows) and for the Bosco rule on 4096^2 (160 rows).
constexpr int kFixedPitch = 304;

static bool fixed_class(const CatParams &p) {
    return p.PS == kFixedPitch && p.PA == kFixedPitch && p.TW == 224 && p.L == 32;
}

static const void *cat_step_fixed_func(int epi) {
    switch (epi) {
        case EPI_BYTE: return (const void *)&cat_step<ELEM_I8, EPI_BYTE, kFixedPitch>;
        case EPI_HALF: return (const void *)&cat_step<ELEM_I8, EPI_HALF, kFixedPitch>;
        case EPI_DECAY: return (const void *)&cat_step<ELEM_I8, EPI_DECAY, kFixedPitch>;
        case EPI_WIN: return (const void *)&cat_step<ELEM_I8, EPI_WIN, kFixedPitch>;
        case EPI_DECAY8: return (const void *)&cat_step<ELEM_I8, EPI_DECAY8, kFixedPitch>;
        case EPI_WIN8: return (const void *)&cat_step<ELEM_I8, EPI_WIN8, kFixedPitch>;
        case EPI_DECAY8W: return (const void *)&cat_step<ELEM_I8, EPI_DECAY8W, kFixedPitch>;
        default: return nullptr;
    }
}

// 160-row tiles of the fixed class, every epilogue. With the height fixed the 192-row tiles
// exceed the 128-register budget of two 8-wave workgroups per CU and spill (measured slower),
// so they keep the height a launch parameter.
static const void *cat_step_fixed160_func(int epi) {
    switch (epi) {
        case EPI_BYTE: return (const void *)&cat_step<ELEM_I8, EPI_BYTE, kFixedPitch, 160>;
        case EPI_HALF: return (const void *)&cat_step<ELEM_I8, EPI_HALF, kFixedPitch, 160>;
        case EPI_DECAY: return (const void *)&cat_step<ELEM_I8, EPI_DECAY, kFixedPitch, 160>;
        case EPI_WIN: return (const void *)&cat_step<ELEM_I8, EPI_WIN, kFixedPitch, 160>;
        case EPI_DECAY8: return (const void *)&cat_step<ELEM_I8, EPI_DECAY8, kFixedPitch, 160>;
        case EPI_WIN8: return (const void *)&cat_step<ELEM_I8, EPI_WIN8, kFixedPitch, 160>;
        case EPI_DECAY8W: return (const void *)&cat_step<ELEM_I8, EPI_DECAY8W, kFixedPitch, 160>;
        default: return nullptr;
    }
}

static const void *cat_func(const CatParams &p, int elem, int epi, int persistent) {
    if (persistent) return cat_persist_func(elem, epi);
    if (elem == ELEM_I8 && fixed_class(p)) {
        if (p.TH == 160) {
            if (const void *f = cat_step_fixed160_func(epi)) return f;
        }
        if (const void *f = cat_step_fixed_func(epi)) return f;
    }
    return cat_step_func(elem, epi);
}

int cat_occupancy(const CatParams &p, int elem, int epi, int waves, int persistent) {
    const void *f = cat_func(p, elem, epi, persistent);
    size_t lds = cat_lds_bytes(p, elem, epi, persistent);
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

static int device_cus() {
    int dev = 0, x = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&x, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        x > 0)
        return x;
    return 8;
}

KernelLaunch cat_launch_shape(const CatParams &p, int elem, int epi, int waves, int persistent) {
    KernelLaunch k;
    k.func = cat_func(p, elem, epi, persistent);
    k.lds = cat_lds_bytes(p, elem, epi, persistent);
    const int ntiles = p.ntx * p.nty;
    if (persistent) {
        // resident workgroups, 8 x (per XCD), no more per XCD than that XCD has tiles
        const int per_xcd = std::max(1, std::min((ntiles + 7) / 8, std::max(1, cat_occupancy(p, elem, epi, waves, 1)) * device_cus() / 8));
        k.grid = dim3((unsigned)(8 * per_xcd), 1, 1);
    } else {
        k.grid = dim3((unsigned)roundup(ntiles, 8), 1, 1);
    }
    k.block = dim3(64 * waves, 1, 1);
    return k;
}

}  // namespace ltl

