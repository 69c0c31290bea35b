// Comparison method: LDS direct-stencil step (the shared-memory out-halo tile of the paper's
// SHARED approach, "Approaches Selected for Evaluation"). The alive map of a tile plus its
// halo is staged in LDS and every cell sums its whole (2r+1)^2 box (or its 4r+1 cross), so the
// work per cell grows as (2r+1)^2 -- the Omega(r^2) cost the paper's introduction attributes to
// this scheme. No sum is shared between cells.
//
// MI355X form: 128 x 256 output tiles staged with 16-byte loads (the halo re-reads are
// (128 + 2r)(256 + 2 roundup16(r)) / (128 x 256) of the tile, 1.21x at r = 5; with neighbouring
// tiles on one XCD they hit its L2, and HBM reads stay within a few per cent of the grid). A thread computes
// four horizontally adjacent cells at once with byte-lane SWAR: for each row of the box it reads
// the aligned LDS dwords around the four cells and adds, for every column offset, the dword of
// the four cells' neighbours at that offset (one funnel shift to realign it, one packed add), so
// each add performs the four cells' additions of that term. Counts up to 255 stay in the byte
// lanes (r <= 7 and every cross); larger boxes fold each row's byte sums into 16-bit lanes. The
// radius is a template parameter so the offsets unroll at compile time. Lanes of a wave take
// consecutive dwords of one row: conflict-free LDS reads, coalesced stores.
//
// Also here: the state-range validation used at creation.
#include <algorithm>

#include "ltl_internal.h"

namespace ltl {

// Next state of one cell from its state s and its box count n (centre included), as selects.
__device__ __forceinline__ int direct_next(int s, int n, const RuleConsts &rc) {
    const int k = n - ((s == 1 && rc.M == 0) ? 1 : 0);
    const int born = (rc.b1 <= k && k <= rc.b2) ? 1 : 0;
    const int stay = (rc.s1 <= k && k <= rc.s2) ? 1 : (rc.C > 2 ? 2 : 0);
    const int decay = (s + 1 < rc.C) ? s + 1 : 0;
    return s == 0 ? born : s == 1 ? stay : decay;
}

// alive indicator (byte == 1) of a dword of states, any byte values
__device__ __forceinline__ uint32_t direct_alive(uint32_t s) {
    uint32_t x = s ^ 0x01010101u;                              // zero byte iff state == 1
    uint32_t y = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;         // bit 7 iff byte != 0
    return (~y & 0x80808080u) >> 7;
}

// Byte-lane sum over one LDS row of the 2R+1 column offsets of four cells. `row` points at the
// first of the ND aligned dwords that cover columns j - R .. j + 3 + R of the cells j..j+3.
template <int R>
__device__ __forceinline__ uint32_t row_sum(const uint32_t *row) {
    constexpr int R4 = (R + 3) & ~3;
    constexpr int ND = (2 * R + R4 - R + 3) / 4 + 1;
    uint32_t dw[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) dw[k] = row[k];
    uint32_t acc = 0;
#pragma unroll
    for (int dj = 0; dj <= 2 * R; ++dj) {
        constexpr int base = R4 - R;
        const int o = dj + base;   // byte offset of the four cells' neighbours at column offset dj - R
        acc += (o & 3) ? __builtin_amdgcn_alignbyte(dw[(o >> 2) + 1], dw[o >> 2], o & 3) : dw[o >> 2];
    }
    return acc;
}

// One kDirectTH x kDirectTW output tile whose top-left cell is (gi0, gj0).
template <int R>
__device__ __forceinline__ void direct_tile(const DirectParams &p, int gi0, int gj0, uint8_t *lds) {
    constexpr int R16 = (R + 15) & ~15;
    constexpr int R4 = (R + 3) & ~3;
    constexpr int LP = kDirectTW + 2 * R16;          // LDS pitch, multiple of 16
    constexpr int ROWS = kDirectTH + 2 * R;
    constexpr int VPR = LP / 16;                      // 16-byte vectors per LDS row
    // stage the alive map of rows gi0 - R .. gi0 + TH + R - 1, columns gj0 - R16 .. gj0 + TW + R16 - 1
    for (int v = threadIdx.x; v < ROWS * VPR; v += kDirectThreads) {
        const int lr = v / VPR;
        const int lc = (v - lr * VPR) * 16;
        const int gr = gi0 - R + lr;
        const int gc = gj0 - R16 + lc;
        uint4 q = make_uint4(0u, 0u, 0u, 0u);
        if (p.periodic) {   // torus: W % 16 == 0, so a 16-byte vector at a 16-aligned column wraps whole
            int wr = gr % p.H, wc = gc % p.W;
            wr += (wr < 0) ? p.H : 0;
            wc += (wc < 0) ? p.W : 0;
            q = *reinterpret_cast<const uint4 *>(p.src + (size_t)wr * p.pitch + wc);
        } else if ((unsigned)gr < (unsigned)p.H && (unsigned)gc < (unsigned)p.pitch) {
            q = *reinterpret_cast<const uint4 *>(p.src + (size_t)gr * p.pitch + gc);   // padding columns are 0
        }
        q = make_uint4(direct_alive(q.x), direct_alive(q.y), direct_alive(q.z), direct_alive(q.w));
        *reinterpret_cast<uint4 *>(lds + lr * LP + lc) = q;
    }
    __syncthreads();

    const int cg = threadIdx.x & 63;                  // four-cell column group
    const int rg = threadIdx.x >> 6;                  // first row of this wave
    const int gc = gj0 + 4 * cg;
    if (gc >= p.pitch) return;
    // aligned dword where the neighbourhood rows of this thread's cells begin
    const int dbase = (4 * cg + R16 - R4) >> 2;
    for (int ly = rg; ly < kDirectTH; ly += 4) {
        const int gr = gi0 + ly;
        if (gr >= p.H) break;
        const uint32_t *w0 = reinterpret_cast<const uint32_t *>(lds + ly * LP) + dbase;
        // centre states: two-state rules read them from the staged alive map (state == alive bit);
        // decay rules load them from the grid, issued before the sums so the load overlaps them
        uint32_t s4;
        if (p.rc.C > 2) s4 = *reinterpret_cast<const uint32_t *>(p.src + (size_t)gr * p.pitch + gc);
        else s4 = w0[R * (LP / 4) + (R4 >> 2)];
        uint32_t n[4];
        if (p.cross) {
            // centre row (2R+1 cells) plus the centre column above and below (2R cells): <= 129
            uint32_t acc = row_sum<R>(w0 + R * (LP / 4));
            constexpr int own = R4 >> 2;               // dword of the four cells' own column
#pragma unroll 4
            for (int dy = 0; dy <= 2 * R; ++dy)
                if (dy != R) acc += w0[dy * (LP / 4) + own];
#pragma unroll
            for (int k = 0; k < 4; ++k) n[k] = (acc >> (8 * k)) & 0xFFu;
        } else if constexpr ((2 * R + 1) * (2 * R + 1) <= 255) {
            uint32_t acc = 0;
#pragma unroll 1
            for (int dy = 0; dy <= 2 * R; ++dy) acc += row_sum<R>(w0 + dy * (LP / 4));
#pragma unroll
            for (int k = 0; k < 4; ++k) n[k] = (acc >> (8 * k)) & 0xFFu;
        } else {
            // row sums (<= 2R+1 per byte) folded into 16-bit lanes: cells 0, 2 and cells 1, 3
            uint32_t lo = 0, hi = 0;
#pragma unroll 1
            for (int dy = 0; dy <= 2 * R; ++dy) {
                const uint32_t rs = row_sum<R>(w0 + dy * (LP / 4));
                lo += rs & 0x00FF00FFu;
                hi += (rs >> 8) & 0x00FF00FFu;
            }
            n[0] = lo & 0xFFFFu;
            n[1] = hi & 0xFFFFu;
            n[2] = lo >> 16;
            n[3] = hi >> 16;
        }
        uint32_t out = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int nx = direct_next((int)((s4 >> (8 * k)) & 0xFFu), (int)n[k], p.rc);
            if (gc + k >= p.W) nx = 0;
            out |= (uint32_t)nx << (8 * k);
        }
        *reinterpret_cast<uint32_t *>(p.dst + (size_t)gr * p.pitch + gc) = out;
    }
}

// Workgroup b runs on XCD b mod 8; the grid is the tile count rounded up to a multiple of 8 and
// XCD x takes the contiguous run of tiles x * nb/8 ... (row-major), so the tiles whose halos
// overlap (left/right neighbours, and the tile row below) are staged through the same L2.
// Surplus workgroups exit before the first barrier.
template <int R>
__global__ void __launch_bounds__(kDirectThreads) direct_step(DirectParams p) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const int ntx = (p.W + kDirectTW - 1) / kDirectTW;
    const int ntiles = ntx * ((p.H + kDirectTH - 1) / kDirectTH);
    const int b = blockIdx.x;
    const int tile = (b & 7) * (int)(gridDim.x >> 3) + (b >> 3);
    if (tile >= ntiles) return;
    const int ty = tile / ntx;
    direct_tile<R>(p, ty * kDirectTH, (tile - ty * ntx) * kDirectTW, lds);
}

// Radius dispatch over 1..32 (RADII(X) expands X(1) ... X(32)).
#define DIRECT_RADII(X)                                                                                   \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18)   \
    X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)

// Batched form: one workgroup per work-list entry (instance, tile), the radius of its instance.
__global__ void __launch_bounds__(kDirectThreads) direct_batch(DirectBatchParams bp) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const BatchItem item = bp.items[blockIdx.x];
    const DirectBatchInst *bi = bp.inst + item.inst;
    const DirectParams p = bi->p;
    const int ty = item.tile / bi->ntx;
    const int tx = item.tile - ty * bi->ntx;
    switch (p.r) {
#define DIRECT_CASE(RR) case RR: direct_tile<RR>(p, ty * kDirectTH, tx * kDirectTW, lds); break;
        DIRECT_RADII(DIRECT_CASE)
#undef DIRECT_CASE
        default: break;
    }
}

static const void *direct_func(int r) {
    switch (r) {
#define DIRECT_CASE(RR) case RR: return (const void *)&direct_step<RR>;
        DIRECT_RADII(DIRECT_CASE)
#undef DIRECT_CASE
        default: return nullptr;
    }
}

const void *direct_batch_func() { return (const void *)&direct_batch; }
int direct_tile_rows() { return kDirectTH; }
int direct_tile_cols() { return kDirectTW; }
int direct_threads() { return kDirectThreads; }

KernelLaunch direct_launch_shape(const DirectParams &p) {
    KernelLaunch k;
    k.func = direct_func(p.r);
    const int ntiles = ((p.W + kDirectTW - 1) / kDirectTW) * ((p.H + kDirectTH - 1) / kDirectTH);
    k.grid = dim3((unsigned)((ntiles + 7) & ~7), 1, 1);   // a multiple of 8 (see direct_step)
    k.block = dim3(kDirectThreads, 1, 1);
    k.lds = direct_lds_bytes(p.r);
    return k;
}

hipError_t launch_direct(const DirectParams &p, hipStream_t s) {
    KernelLaunch k = direct_launch_shape(p);
    if (!k.func) return hipErrorInvalidValue;
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

// Device constants of a CAT launch written on the device: the band table of (elem, r) in the
// band_table layout (LTL_BAND_OPS x 64 lanes x 4 dwords), then `zero_bytes` zero bytes (the
// page out-of-grid tile loads read). Every byte of the range is written.
__global__ void fill_constants(uint32_t *dst, int elem, int r, int zero_dwords) {
    const int n = LTL_BAND_TABLE_INTS + zero_dwords;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        dst[i] = i < LTL_BAND_TABLE_INTS ? band_dword(elem, r, i >> 8, (i >> 2) & 63, i & 3) : 0u;
}

hipError_t launch_fill_constants(uint8_t *dst, int elem, int r, size_t zero_bytes, hipStream_t s) {
    uint32_t *d = reinterpret_cast<uint32_t *>(dst);
    int zd = (int)(zero_bytes / 4);
    void *args[] = {(void *)&d, (void *)&elem, (void *)&r, (void *)&zd};
    return hipLaunchKernel((const void *)&fill_constants, dim3(16), dim3(256), args, 0, s);
}

// Ping-pong buffers of an H x pitch grid from a caller's initial grid: a = init with the
// columns W..pitch-1 zero, b = all zero. One thread per dword of each row (pitch % 64 == 0).
__global__ void prepare_grids(uint8_t *a, uint8_t *b, const uint8_t *init, size_t init_pitch, int H, int W,
                              int pitch) {
    const int dpr = pitch >> 2;
    const size_t n = (size_t)H * dpr;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
        const size_t i = k / dpr;
        const int j0 = (int)(k - i * dpr) << 2;
        const uint8_t *src = init + i * init_pitch;
        uint32_t v = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            v |= (j0 + e < W ? (uint32_t)src[j0 + e] : 0u) << (8 * e);
        reinterpret_cast<uint32_t *>(a)[k] = v;
        reinterpret_cast<uint32_t *>(b)[k] = 0u;
    }
}

hipError_t launch_prepare_grids(uint8_t *a, uint8_t *b, const uint8_t *init, size_t init_pitch, int H, int W,
                                int pitch, hipStream_t s) {
    const size_t n = (size_t)H * (size_t)(pitch >> 2);
    unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
    if (blocks == 0) blocks = 1;
    void *args[] = {(void *)&a, (void *)&b, (void *)&init, (void *)&init_pitch, (void *)&H, (void *)&W, (void *)&pitch};
    return hipLaunchKernel((const void *)&prepare_grids, dim3(blocks), dim3(256), args, 0, s);
}

}  // namespace ltl
