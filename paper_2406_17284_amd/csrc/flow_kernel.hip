// Dataflow form of the single-grid CAT step (tuning.persistent = 2): one launch runs every
// T-step round of an ltl_step call. Workgroup b owns one tile for the whole launch and, per
// round, loads the tile's window from the buffer of the previous round, runs the T steps of
// Algorithm 1 on it (the same per-tile code as cat_step) and stores the tile into the other
// buffer of the ping-pong pair. Instead of a kernel boundary between rounds, a tile starts
// round k as soon as the (up to) eight tiles its window overlaps have finished round k - 1,
// which they publish in a per-tile counter. So neighbouring tiles, not the whole grid,
// synchronise, and a compute unit's two workgroups drift out of phase (one loads while the
// other computes) instead of starting and ending every round together.
//
// Ordering. A tile's stores of round k go to buf[(first + k + 1) & 1]; its neighbours read that
// buffer in round k + 1 (their windows overlap the tile) and last read it in round k - 1. Waiting
// for every neighbour to finish round k - 1 before starting round k therefore covers both the
// read-after-write and the write-after-read order. The counter store is a release at agent scope
// (write-back of this XCD's L2) after every wave's stores completed; the waiting side polls with
// agent-scope atomic loads and then acquires at agent scope (invalidation of its L1/L2), before
// the window load of the round.
//
// Every wait is bounded (spin_limit polls): a wait that runs out counts one timeout in *err and
// goes on, so each workgroup always finishes; the host reports the timeout. Co-residency of all
// workgroups (which the waits rely on) is what a cooperative launch guarantees.
#include "cat_device.h"

namespace ltl {

template <int ELEM, int EPI>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) cat_flow(CatParams p, FlowParams f) {
    extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = blockDim.x >> 6;
    // workgroup b runs on XCD b mod 8 and takes the contiguous block of tiles (b mod 8) * nb/8 ...,
    // as cat_step does; surplus workgroups exit
    const int ntiles = p.ntx * p.nty;
    const int nb = gridDim.x;
    const int bid = blockIdx.x;
    const int tile = (bid & 7) * (nb >> 3) + (bid >> 3);
    if (tile >= ntiles) return;
    const Codec cd = make_codec();
    const int ty = tile / p.ntx;
    const int tx = tile - ty * p.ntx;
    // threads 0..8 of wave 0 (except the centre, 4) each watch one neighbouring tile
    int watch = -1;
    if (tid < 9 && tid != 4) {
        int ny = ty + tid / 3 - 1, nx = tx + tid % 3 - 1;
        if (p.periodic) {
            ny = (ny + p.nty) % p.nty;
            nx = (nx + p.ntx) % p.ntx;
            watch = ny * p.ntx + nx;
            if (watch == tile) watch = -1;
        } else if (ny >= 0 && ny < p.nty && nx >= 0 && nx < p.ntx) {
            watch = ny * p.ntx + nx;
        }
    }
    for (int k = 0; k < f.rounds; ++k) {
        if (k > 0) {
            if (wave == 0) {
                if (watch >= 0) {
                    const uint32_t target = f.epoch + (uint32_t)k;
                    int spins = 0;
                    while ((int32_t)(__hip_atomic_load(f.flags + watch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                                     target) < 0) {
                        if (++spins > f.spin_limit) {
                            __hip_atomic_fetch_add(f.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            __syncthreads();
        }
        CatParams q = p;
        q.src = f.buf[(f.first + k) & 1];
        q.dst = f.buf[(f.first + k + 1) & 1];
        if (k == f.rounds - 1) q.T = f.last_T;
        cat_tile<ELEM, EPI>(q, tile, lds, tid, lane, wave, nwaves, cd);
        // publish: every wave's stores have reached the L2, then one release + counter store
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(f.flags + tile, f.epoch + (uint32_t)k + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

static const void *cat_flow_func(int elem, int epi) {
    const bool dec = (epi == EPI_DECAY);
    if (elem == ELEM_F16)
        return dec ? (const void *)&cat_flow<ELEM_F16, EPI_DECAY>
                   : epi == EPI_HALF ? (const void *)&cat_flow<ELEM_F16, EPI_HALF> : (const void *)&cat_flow<ELEM_F16, EPI_BYTE>;
    if (elem == ELEM_F8)
        return dec ? (const void *)&cat_flow<ELEM_F8, EPI_DECAY>
                   : epi == EPI_HALF ? (const void *)&cat_flow<ELEM_F8, EPI_HALF> : (const void *)&cat_flow<ELEM_F8, EPI_BYTE>;
    if (elem == ELEM_I8X)
        return dec ? (const void *)&cat_flow<ELEM_I8X, EPI_DECAY> : (const void *)&cat_flow<ELEM_I8X, EPI_BYTE>;
    if (elem == ELEM_I8W)
        return dec ? (const void *)&cat_flow<ELEM_I8W, EPI_DECAY> : (const void *)&cat_flow<ELEM_I8W, EPI_HALF>;
    if (epi == EPI_WIN) return (const void *)&cat_flow<ELEM_I8, EPI_WIN>;
    if (epi == EPI_WIN8) return (const void *)&cat_flow<ELEM_I8, EPI_WIN8>;
    if (epi == EPI_DECAY8) return (const void *)&cat_flow<ELEM_I8, EPI_DECAY8>;
    if (epi == EPI_DECAY8W) return (const void *)&cat_flow<ELEM_I8, EPI_DECAY8W>;
    return dec ? (const void *)&cat_flow<ELEM_I8, EPI_DECAY>
               : epi == EPI_HALF ? (const void *)&cat_flow<ELEM_I8, EPI_HALF> : (const void *)&cat_flow<ELEM_I8, EPI_BYTE>;
}

int cat_flow_occupancy(const CatParams &p, int elem, int epi, int waves) {
    const void *f = cat_flow_func(elem, epi);
    const size_t lds = (size_t)p.lds_total;
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

hipError_t launch_cat_flow(const CatParams &p, const FlowParams &f, int elem, int epi, int waves, hipStream_t s) {
    const void *func = cat_flow_func(elem, epi);
    const size_t lds = (size_t)p.lds_total;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(func, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int ntiles = p.ntx * p.nty;
    void *args[2] = {(void *)&p, (void *)&f};
    return hipLaunchCooperativeKernel(func, dim3((unsigned)roundup(ntiles, 8)), dim3(64 * waves), args, (unsigned)lds, s);
}

}  // namespace ltl
