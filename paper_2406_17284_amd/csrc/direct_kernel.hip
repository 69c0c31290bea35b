// Comparison method: LDS direct-stencil step (the classic shared-memory out-halo tile of
// the paper's SHARED approach, "Approaches Selected for Evaluation"). The alive map of a
// (TH + 2r) x (TW + 2r) tile is staged in LDS and every cell sums its (2r+1)^2 box
// directly, so the work per cell grows as (2r+1)^2 (the Omega(r^2) cost the paper's
// introduction attributes to this scheme). A thread computes 4 horizontally adjacent
// cells and reads each LDS byte of their joint window once per row.
// Also here: the state-range validation used at creation.
#include "ltl_internal.h"

namespace ltl {

static constexpr int DIRECT_TH = 32;
static constexpr int DIRECT_TW = 64;
static constexpr int DIRECT_THREADS = 256;

__device__ __forceinline__ int direct_next(int s, int n, const RuleConsts &rc) {
    // n: box count including the centre
    if (s == 0) return (rc.b1 <= n && n <= rc.b2) ? 1 : 0;
    if (s == 1) {
        int k = n - (rc.M == 0 ? 1 : 0);
        if (rc.s1 <= k && k <= rc.s2) return 1;
        return rc.C > 2 ? 2 : 0;
    }
    return (s + 1 < rc.C) ? s + 1 : 0;
}

// One DIRECT_TH x DIRECT_TW output tile whose top-left cell is (gi0, gj0).
__device__ __forceinline__ void direct_tile(const DirectParams &p, int gi0, int gj0, uint8_t *lds) {
    const int r = p.r;
    const int rows = DIRECT_TH + 2 * r;
    const int cols = DIRECT_TW + 2 * r;
    for (int idx = threadIdx.x; idx < rows * cols; idx += blockDim.x) {
        int lr = idx / cols;
        int lc = idx - lr * cols;
        int gr = gi0 - r + lr;
        int gc = gj0 - r + lc;
        uint8_t v = 0;
        if (p.periodic) {   // torus: wrap both coordinates
            int wr = gr % p.H, wc = gc % p.W;
            wr += (wr < 0) ? p.H : 0;
            wc += (wc < 0) ? p.W : 0;
            v = p.src[(size_t)wr * p.pitch + wc];
        } else if ((unsigned)gr < (unsigned)p.H && (unsigned)gc < (unsigned)p.W) {
            v = p.src[(size_t)gr * p.pitch + gc];
        }
        lds[lr * p.LP + lc] = (v == 1) ? 1 : 0;
    }
    __syncthreads();

    const int tx = threadIdx.x & 15;       // 16 groups of 4 columns
    const int ty = threadIdx.x >> 4;       // 16 rows per pass
    const int w = 2 * r;
    for (int ly = ty; ly < DIRECT_TH; ly += 16) {
        const int lx = 4 * tx;
        int acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
        // Moore: every row of the box; cross: the centre row only, plus the centre column
        for (int di = p.cross ? r : 0; di <= (p.cross ? r : w); ++di) {
            const uint8_t *row = lds + (ly + di) * p.LP + lx;
            for (int dj = 0; dj <= w + 3; ++dj) {
                int b = row[dj];
                acc0 += (dj <= w) ? b : 0;
                acc1 += (dj >= 1 && dj <= w + 1) ? b : 0;
                acc2 += (dj >= 2 && dj <= w + 2) ? b : 0;
                acc3 += (dj >= 3) ? b : 0;
            }
        }
        if (p.cross) {
            for (int di = 0; di <= w; ++di) {
                if (di == r) continue;
                const uint8_t *col = lds + (ly + di) * p.LP + lx + r;
                acc0 += col[0];
                acc1 += col[1];
                acc2 += col[2];
                acc3 += col[3];
            }
        }
        const int gr = gi0 + ly;
        const int gc = gj0 + lx;
        if (gr >= p.H || gc >= p.pitch) continue;
        const uint8_t *srow = p.src + (size_t)gr * p.pitch + gc;
        uint32_t s4 = *reinterpret_cast<const uint32_t *>(srow);
        int acc[4] = {acc0, acc1, acc2, acc3};
        uint32_t out = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int s = (int)((s4 >> (8 * k)) & 0xFFu);
            int nx = direct_next(s, acc[k], p.rc);
            if (gc + k >= p.W) nx = 0;
            out |= (uint32_t)nx << (8 * k);
        }
        *reinterpret_cast<uint32_t *>(p.dst + (size_t)gr * p.pitch + gc) = out;
    }
}

__global__ void __launch_bounds__(DIRECT_THREADS) direct_step(DirectParams p) {
    extern __shared__ uint8_t lds[];
    direct_tile(p, blockIdx.y * DIRECT_TH, blockIdx.x * DIRECT_TW, lds);
}

// Batched form: one workgroup per work-list entry (instance, tile).
__global__ void __launch_bounds__(DIRECT_THREADS) direct_batch(DirectBatchParams bp) {
    extern __shared__ uint8_t lds[];
    const BatchItem item = bp.items[blockIdx.x];
    const DirectBatchInst *bi = bp.inst + item.inst;
    const DirectParams p = bi->p;
    const int ty = item.tile / bi->ntx;
    const int tx = item.tile - ty * bi->ntx;
    direct_tile(p, ty * DIRECT_TH, tx * DIRECT_TW, lds);
}

const void *direct_batch_func() { return (const void *)&direct_batch; }
int direct_tile_rows() { return DIRECT_TH; }
int direct_tile_cols() { return DIRECT_TW; }
int direct_threads() { return DIRECT_THREADS; }

KernelLaunch direct_launch_shape(const DirectParams &p) {
    KernelLaunch k;
    k.func = (const void *)&direct_step;
    k.grid = dim3((p.W + DIRECT_TW - 1) / DIRECT_TW, (p.H + DIRECT_TH - 1) / DIRECT_TH, 1);
    k.block = dim3(DIRECT_THREADS, 1, 1);
    k.lds = (size_t)(DIRECT_TH + 2 * p.r) * p.LP;
    return k;
}

hipError_t launch_direct(const DirectParams &p, hipStream_t s) {
    KernelLaunch k = direct_launch_shape(p);
    void *args[] = {(void *)&p};
    return hipLaunchKernel(k.func, k.grid, k.block, args, k.lds, s);
}

// flag |= 1 if any of the H x W cells holds a state >= states
__global__ void validate_states(const uint8_t *src, int H, int W, size_t pitch, int states, uint32_t *flag) {
    const size_t n = (size_t)H * W;
    uint32_t bad = 0;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
        size_t i = k / W, j = k - i * W;
        bad |= (src[i * pitch + j] >= states) ? 1u : 0u;
    }
    if (bad) atomicOr(flag, 1u);
}

hipError_t launch_validate(const uint8_t *src, int H, int W, size_t pitch, int states, uint32_t *flag,
                           hipStream_t s) {
    size_t n = (size_t)H * W;
    unsigned blocks = (unsigned)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    void *args[] = {(void *)&src, (void *)&H, (void *)&W, (void *)&pitch, (void *)&states, (void *)&flag};
    return hipLaunchKernel((const void *)&validate_states, dim3(blocks), dim3(256), args, 0, s);
}

}  // namespace ltl
