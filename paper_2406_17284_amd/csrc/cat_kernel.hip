// CAT step on gfx950: Moore neighbourhood counts as two band-matrix products per tile on
// MFMA, followed by the LTL transition, with T steps fused per launch.
//
// Method (paper, "Formulation of CAT", Eq. 2-3 and Eq. F^H / F^R; Algorithm 1):
//   H = Lambda x Pi   (horizontal window sums of the alive map)
//   R = Pi x H        (vertical window sums of H) = box count of radius r, centre included
// with Pi[a][b] = 1 iff |a - b| <= r. The paper splits Pi into three 16x16 band fragments
// and runs 3 + 3 FP16 16x16x16 MMAs per 16x16 fragment. Here one int8 16x16x64 MFMA covers
// the 48 columns a 16-column output needs (16 + 2r <= 48 for r <= 16), so each direction
// costs one MFMA per 16x16 block:
//
//  * MFMA #1 (horizontal): A = 16 grid rows x 64 columns of the LDS tile, read as one 16-byte
//    chunk per lane; B = band operand built in registers. One A load feeds two MFMAs (the two
//    16-column halves of a 32-column strip) with two different bands, because the 64-column
//    window holds both halves' neighbourhoods. Output: lane (col j, group g) holds H rows
//    4g..4g+3 of column j, which are exact small integers (<= 33) and pack into one dword.
//  * MFMA #2 (vertical) computes R^T = H^T x Pi (Pi is symmetric). Its A operand needs, per
//    lane (col c, group g), four consecutive H rows of column c -- exactly the dword MFMA #1
//    left in that lane. So the int32 -> int8 repack between the products (named as the
//    obstacle to INT8 MMAs in the paper's conclusions) is three register ops, with no LDS
//    round trip: the K index of MFMA #2 is laid out as a ring of four 16-row H blocks, one
//    dword each, and the band operand comes in four phases that follow the ring.
//  * The R^T accumulator gives each lane 4 horizontally adjacent counts of one row, so the
//    epilogue reads one dword of centre states and writes one dword of next states.
//
// The K order inside an operand is immaterial as long as A and B agree on it (a dot product
// is invariant under a common permutation), which is how the bands are built below.
//
// Temporal blocking (multi-step idea cited in the paper's related work): the tile plus a
// margin L = roundup16(r (T-1)) + 16 is loaded once into LDS; step t recomputes the tile
// grown by roundup16(r (T - t)) cells, so after T steps the tile itself is exact. Cells
// outside the grid are forced to 0 after every step (dead ghost halo).
#include "ltl_internal.h"

namespace ltl {

typedef int32_t v4i __attribute__((ext_vector_type(4)));
// global-memory dword (explicit address space: global_store_*, not flat_* which would also
// count against the LDS wait counter)
typedef __attribute__((address_space(1))) uint32_t gdword;

// Low bytes of the four int32 lanes of d packed into one dword (three byte permutes).
__device__ __forceinline__ uint32_t pack_bytes(v4i d) {
    uint32_t lo = __builtin_amdgcn_perm((uint32_t)d[1], (uint32_t)d[0], 0x0c0c0400u);  // d0.b0, d1.b0
    uint32_t hi = __builtin_amdgcn_perm((uint32_t)d[3], (uint32_t)d[2], 0x0c0c0400u);  // d2.b0, d3.b0
    return __builtin_amdgcn_perm(hi, lo, 0x05040100u);
}

__device__ __forceinline__ uint32_t bfi(uint32_t mask, uint32_t a, uint32_t b) {
    return (mask & a) | (~mask & b);
}

// Byte mask (0xFF per byte) of the four cells gc..gc+3 that lie inside [0, W).
__device__ __forceinline__ uint32_t col_mask(int gc, int W) {
    uint32_t m = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v)
        m |= ((unsigned)(gc + v) < (unsigned)W ? 0xFFu : 0u) << (8 * v);
    return m;
}

// Next states of 4 adjacent cells from their box counts n (centre included) and states s.
// `m` is the validity mask of the 4 cells (0xFF per byte inside the grid); cells outside get 0.
// Returns the state dword; *alive receives the alive-indicator dword (state == 1).
//
// Two-state rules test lo(s) <= n <= hi(s) on 8-bit (BYTE) or 16-bit (HALF) SWAR lanes:
// a = 0x80 + n - lo has its top bit set iff n >= lo, b = 0x80 + hi - n iff n <= hi, and the
// per-lane offsets come from the centre state in one 3-input bitwise op each.
template <int EPI>
__device__ __forceinline__ uint32_t transition4(v4i n, uint32_t s, uint32_t m, const RuleConsts &rc,
                                                uint32_t *alive) {
    if constexpr (EPI == EPI_BYTE) {
        uint32_t N = pack_bytes(n);
        uint32_t sm = 0x80808080u - s;                 // 0x80 per dead lane, 0x7F per alive lane
        uint32_t a = N + (rc.Klo ^ (sm & rc.Dlo));
        uint32_t b = (rc.Khi ^ (sm & rc.Dhi)) - N;
        uint32_t x = (a & b & (m & 0x80808080u)) >> 7;
        *alive = x;
        return x;
    } else if constexpr (EPI == EPI_HALF) {
        uint32_t p01 = (uint32_t)n[0] | ((uint32_t)n[1] << 16);
        uint32_t p23 = (uint32_t)n[2] | ((uint32_t)n[3] << 16);
        uint32_t s01 = __builtin_amdgcn_perm(0u, s, 0x0c010c00u);  // bytes 0, 1 -> 16-bit lanes
        uint32_t s23 = __builtin_amdgcn_perm(0u, s, 0x0c030c02u);
        uint32_t m01 = __builtin_amdgcn_perm(0u, m, 0x010c000cu);  // mask bytes 0, 1 -> lane top bytes
        uint32_t m23 = __builtin_amdgcn_perm(0u, m, 0x030c020cu);
        uint32_t sm01 = 0x80008000u - s01;
        uint32_t sm23 = 0x80008000u - s23;
        uint32_t x01 = (p01 + (rc.Klo ^ (sm01 & rc.Dlo))) & ((rc.Khi ^ (sm01 & rc.Dhi)) - p01) & (m01 & 0x80008000u);
        uint32_t x23 = (p23 + (rc.Klo ^ (sm23 & rc.Dlo))) & ((rc.Khi ^ (sm23 & rc.Dhi)) - p23) & (m23 & 0x80008000u);
        // bits 15 and 31 of x01, x23 -> bit 7 of bytes 0..3, then down to bit 0
        uint32_t x = __builtin_amdgcn_perm(x23, x01, 0x07050301u) >> 7;
        *alive = x;
        return x;
    } else {
        uint32_t out = 0, al = 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int sv = (int)((s >> (8 * v)) & 0xFFu);
            int c = n[v];
            int nx;
            if (sv == 0) {
                nx = (rc.b1 <= c && c <= rc.b2) ? 1 : 0;
            } else if (sv == 1) {
                int k = c - (rc.M == 0 ? 1 : 0);
                nx = (rc.s1 <= k && k <= rc.s2) ? 1 : 2;
            } else {
                nx = (sv + 1 < rc.C) ? sv + 1 : 0;
            }
            out |= (uint32_t)nx << (8 * v);
            al |= (uint32_t)(nx == 1) << (8 * v);
        }
        *alive = al & m;
        return out & m;
    }
}

// alive indicator (byte == 1) of a dword of states, any byte values
__device__ __forceinline__ uint32_t alive_of(uint32_t s) {
    uint32_t x = s ^ 0x01010101u;                              // zero byte iff state == 1
    uint32_t y = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;         // bit 7 iff byte != 0
    return (~y & 0x80808080u) >> 7;
}

// Geometry of one step: strips of 32 columns, each cut into `nseg` row segments of at most
// CAT_MAXC 16-row blocks. Every segment is one wave's work item; a step needs
// items <= waves (the host planner checks this for every step of a launch).
struct StepGeom {
    int E, nstrips, nrb, nseg, seglen;
};

__device__ __forceinline__ StepGeom step_geom(const CatParams &p, int t) {
    StepGeom g;
    g.E = (p.r * (p.T - t) + 15) & ~15;
    g.nstrips = (p.TW + 2 * g.E) >> 5;
    g.nrb = (p.TH + 2 * g.E) >> 4;
    g.nseg = (g.nrb + CAT_MAXC - 1) / CAT_MAXC;
    g.seglen = (g.nrb + g.nseg - 1) / g.nseg;
    return g;
}

// H of one item and one 16-column half: the packed dword of H block rb0 - 1 + k in element
// k (k = 0 .. count + 1 <= 15) of a 16-register tuple. Output block M needs k = M, M+1, M+2;
// MFMA #2 reads the even-aligned 4-register window starting at M (M even: the blocks sit in
// slots 0, 1, 2) or at M - 1 (M odd: slots 1, 2, 3), so the band operand has two phases and
// every output block costs one MFMA, with no register copies.
typedef int32_t v16i __attribute__((ext_vector_type(16)));

template <int K>
__device__ __forceinline__ v4i window4(const v16i &h) {
    return __builtin_shufflevector(h, h, K, K + 1, K + 2, K + 3);
}

// Phase A of one item: H (horizontal band sums) of blocks rb0 - 1 .. rb0 + count for both
// 16-column halves of the strip, packed to bytes, in registers. Software-pipelined in pairs of
// blocks: the A chunks of the next pair are read from LDS before the MFMAs of this pair run.
__device__ __forceinline__ void phase_a(const uint8_t *At, uint32_t a_off, uint32_t PS, int rb0, int count,
                                        const v4i &bh0, const v4i &bh1, v16i &Ha, v16i &Hb) {
    const v4i zero = {0, 0, 0, 0};
    const int nh = count + 2;
    v4i a[4];
#define CAT_LDA(K) a[(K) & 3] = *reinterpret_cast<const v4i *>(At + (a_off + (uint32_t)(16 * (rb0 - 1 + (K))) * PS));
#define CAT_HB(K)                                                                                  \
    {                                                                                              \
        v4i da = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[(K) & 3], bh0, zero, 0, 0, 0);            \
        v4i db = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[(K) & 3], bh1, zero, 0, 0, 0);            \
        Ha[(K)] = (int32_t)pack_bytes(da);                                                         \
        Hb[(K)] = (int32_t)pack_bytes(db);                                                         \
    }
#define CAT_APAIR(P)                                                                               \
    if (2 * (P) < nh) {                                                                            \
        if (2 * (P) + 2 < nh) {                                                                    \
            CAT_LDA(2 * (P) + 2)                                                                   \
            if (2 * (P) + 3 < nh) CAT_LDA(2 * (P) + 3)                                             \
        }                                                                                          \
        CAT_HB(2 * (P))                                                                            \
        if (2 * (P) + 1 < nh) CAT_HB(2 * (P) + 1)                                                  \
    }
    CAT_LDA(0) CAT_LDA(1)
    CAT_APAIR(0) CAT_APAIR(1) CAT_APAIR(2) CAT_APAIR(3) CAT_APAIR(4) CAT_APAIR(5) CAT_APAIR(6) CAT_APAIR(7)
#undef CAT_APAIR
#undef CAT_HB
#undef CAT_LDA
}

// Phase B of one item: vertical band products, transition, store (in place in LDS for an
// intermediate step, to the output grid on the last step of the launch). Software-pipelined in
// pairs of output blocks: the MFMAs and centre-state reads of the next pair are issued before
// the VALU transition of this pair, so their latencies overlap it.
template <int EPI, bool MASKED, bool LAST>
__device__ __forceinline__ void phase_b(const CatParams &p, uint8_t *At, uint8_t *Qt, uint32_t c_off, int rb0,
                                        int count, int gr0, uint32_t goff0, int gca, uint32_t cma, uint32_t cmb,
                                        const v4i &bve, const v4i &bvo, const v16i &Ha, const v16i &Hb) {
    const v4i zero = {0, 0, 0, 0};
    const uint32_t PS = (uint32_t)p.PS;
    const uint8_t *Sc = (EPI == EPI_DECAY) ? Qt : At;
    v4i ca[4], cb[4];
    uint32_t sa[4], sb[4];
    // counts and centre states of block M (slot M & 3)
#define CAT_ISSUE(M)                                                                               \
    {                                                                                              \
        constexpr int W0 = ((M) & 1) ? (M) - 1 : (M);                                              \
        const v4i &bv = ((M) & 1) ? bvo : bve;                                                     \
        ca[(M) & 3] = __builtin_amdgcn_mfma_i32_16x16x64_i8(window4<W0>(Ha), bv, zero, 0, 0, 0);   \
        cb[(M) & 3] = __builtin_amdgcn_mfma_i32_16x16x64_i8(window4<W0>(Hb), bv, zero, 0, 0, 0);   \
        const uint32_t co = c_off + (uint32_t)(16 * (rb0 + (M))) * PS;                             \
        sa[(M) & 3] = *reinterpret_cast<const uint32_t *>(Sc + co);                                \
        sb[(M) & 3] = *reinterpret_cast<const uint32_t *>(Sc + co + 16);                           \
    }
    // transition and store of block M
#define CAT_FINISH(M)                                                                              \
    {                                                                                              \
        const uint32_t co = c_off + (uint32_t)(16 * (rb0 + (M))) * PS;                             \
        const int grow = gr0 + 16 * (M);                                                           \
        uint32_t rowm = 0xFFFFFFFFu;                                                               \
        if (MASKED) rowm = ((unsigned)grow < (unsigned)p.H) ? 0xFFFFFFFFu : 0u;                    \
        uint32_t ala, alb;                                                                         \
        const uint32_t na = transition4<EPI>(ca[(M) & 3], sa[(M) & 3], rowm & cma, p.rc, &ala);    \
        const uint32_t nb = transition4<EPI>(cb[(M) & 3], sb[(M) & 3], rowm & cmb, p.rc, &alb);    \
        if constexpr (LAST) {                                                                      \
            const uint32_t go = goff0 + (uint32_t)(16 * (M)) * (uint32_t)p.pitch;                  \
            if (!MASKED || rowm) {                                                                 \
                if (!MASKED || (unsigned)gca < (unsigned)p.pitch) *(gdword *)(p.dst + go) = na;    \
                if (!MASKED || (unsigned)(gca + 16) < (unsigned)p.pitch) *(gdword *)(p.dst + go + 16) = nb; \
            }                                                                                      \
        } else if constexpr (EPI == EPI_DECAY) {                                                   \
            *reinterpret_cast<uint32_t *>(Qt + co) = na;                                           \
            *reinterpret_cast<uint32_t *>(Qt + co + 16) = nb;                                      \
            *reinterpret_cast<uint32_t *>(At + co) = ala;                                          \
            *reinterpret_cast<uint32_t *>(At + co + 16) = alb;                                     \
        } else {                                                                                   \
            *reinterpret_cast<uint32_t *>(At + co) = na;                                           \
            *reinterpret_cast<uint32_t *>(At + co + 16) = nb;                                      \
        }                                                                                          \
    }
    // pair P = blocks 2P, 2P + 1; block `count` (one past the item) may be issued: its window
    // and centre row are inside the tile and nothing is stored for it
#define CAT_BPAIR(P, NEXT)                                                                         \
    if (2 * (P) < count) {                                                                         \
        if (NEXT && 2 * (P) + 2 < count) { CAT_ISSUE(2 * (P) + 2) CAT_ISSUE(2 * (P) + 3) }         \
        CAT_FINISH(2 * (P))                                                                        \
        if (2 * (P) + 1 < count) CAT_FINISH(2 * (P) + 1)                                           \
    }
    CAT_ISSUE(0) CAT_ISSUE(1)
    CAT_BPAIR(0, 1) CAT_BPAIR(1, 1) CAT_BPAIR(2, 1) CAT_BPAIR(3, 1) CAT_BPAIR(4, 1) CAT_BPAIR(5, 1)
    CAT_BPAIR(6, 0)
#undef CAT_BPAIR
#undef CAT_FINISH
#undef CAT_ISSUE
}

// T steps of one tile, in place in LDS (the last step writes the output grid).
// bve: window slots 0, 1, 2 = blocks m-1, m, m+1; bvo: slots 1, 2, 3.
template <int EPI, bool MASKED>
__device__ __forceinline__ void cat_steps(const CatParams &p, uint8_t *At, uint8_t *Qt, int gi0, int gj0, int wave,
                                          int lane, const v4i &bh0, const v4i &bh1, const v4i &bve, const v4i &bvo) {
    const int li = lane & 15, lg = lane >> 4;
    const uint32_t PS = (uint32_t)p.PS;
    const int L = p.L;
    for (int t = 1; t <= p.T; ++t) {
        const bool last = (t == p.T);
        const StepGeom g = step_geom(p, t);
        const int items = g.nstrips * g.nseg;
        int j0 = 0, rb0 = 0, count = 0;
        if (wave < items) {
            const int strip = wave % g.nstrips;
            const int seg = wave / g.nstrips;
            const int mb_lo = seg * g.seglen;
            const int mb_hi = min(g.nrb, mb_lo + g.seglen);
            j0 = -g.E + 32 * strip;
            rb0 = -(g.E >> 4) + mb_lo;
            count = max(0, mb_hi - mb_lo);
        }
        v16i Ha, Hb;
        // LDS offsets of this lane's A chunk (row li of a block, 16 bytes at column
        // j0 - 16 + 16 lg) and centre dword (row li, column j0 + 4 lg), block row 0
        const uint32_t a_off = (uint32_t)((L + li) * (int)PS + (L + j0 - 16 + 16 * lg));
        const uint32_t c_off = (uint32_t)((L + li) * (int)PS + (L + j0 + 4 * lg));
        if (count > 0) phase_a(At, a_off, PS, rb0, count, bh0, bh1, Ha, Hb);
        if (!last) __syncthreads();   // every read of the old states precedes any in-place write
        if (count > 0) {
            const int gca = gj0 + j0 + 4 * lg;
            uint32_t cma = 0xFFFFFFFFu, cmb = 0xFFFFFFFFu;
            if constexpr (MASKED) {
                cma = col_mask(gca, p.W);
                cmb = col_mask(gca + 16, p.W);
            }
            const int gr0 = gi0 + 16 * rb0 + li;
            const uint32_t goff0 = (uint32_t)(gr0 * p.pitch + gca);
            if (last)
                phase_b<EPI, MASKED, true>(p, At, Qt, c_off, rb0, count, gr0, goff0, gca, cma, cmb, bve, bvo, Ha, Hb);
            else
                phase_b<EPI, MASKED, false>(p, At, Qt, c_off, rb0, count, gr0, goff0, gca, cma, cmb, bve, bvo, Ha, Hb);
        }
        if (!last) __syncthreads();   // new states complete before the next step reads them
    }
}

// Stream the (TH + 2L) x PS window of tile `tile` into the LDS buffer `buf` with direct
// global->LDS loads: wave w moves KiB chunks w, w + nwaves, ...; lane l of a chunk carries
// the 16 bytes at buffer offset 1024 c + 16 l. Cells outside the grid come from the zero page.
__device__ __forceinline__ void issue_tile_load(const CatParams &p, int gi0, int gj0, uint8_t *buf, int wave,
                                                int nwaves, int lane, float inv_ps) {
    const int rows = p.TH + 2 * p.L;
    const int nchunks = p.lds_tile >> 10;
    for (int c = wave; c < nchunks; c += nwaves) {
        const int o = (c << 10) + (lane << 4);
        int lr = (int)((float)o * inv_ps);
        int lc = o - lr * p.PS;
        if (lc < 0) { lr -= 1; lc += p.PS; }
        if (lc >= p.PS) { lr += 1; lc -= p.PS; }
        const int gr = gi0 - p.L + lr;
        const int gc = gj0 - p.L + lc;
        const uint8_t *g = p.zero;
        if (lr < rows && (unsigned)gr < (unsigned)p.H && (unsigned)gc < (unsigned)p.pitch)
            g = p.src + (size_t)gr * p.pitch + gc;
        // The load is issued from inline assembly: the compiler cannot see which LDS bytes an
        // LDS-DMA writes, so for its own builtin it would make every later LDS access wait for
        // all outstanding vector-memory operations. The caller waits (vmcnt(0) + barrier) before
        // the buffer is read.
        const uint32_t lds_addr = (uint32_t)(uintptr_t)(buf + (c << 10));
        asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                     :
                     : "s"(__builtin_amdgcn_readfirstlane(lds_addr)), "v"(g)
                     : "memory", "m0");
    }
}

// One workgroup per tile (workgroups of one XCD take consecutive tiles, so the halos of
// neighbouring tiles meet in that XCD's L2): load the window with direct LDS loads, then T
// steps in place.
template <int EPI>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) cat_step_i8(CatParams p) {
    extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: keeps item code scalar
    const int nwaves = blockDim.x >> 6;
    const uint32_t tile_bytes = (uint32_t)p.lds_tile;

    const int ntiles = p.ntx * p.nty;
    const int nb = gridDim.x;
    const int bid = blockIdx.x;
    const int tile = (nb & 7) ? bid : (bid & 7) * (nb >> 3) + (bid >> 3);
    if (tile >= ntiles) return;
    const int gi0 = (tile / p.ntx) * p.TH;
    const int gj0 = (tile % p.ntx) * p.TW;

    issue_tile_load(p, gi0, gj0, lds, wave, nwaves, lane, 1.0f / (float)p.PS);
    const v4i *bt = reinterpret_cast<const v4i *>(p.bands);
    const v4i bh0 = bt[0 * 64 + lane], bh1 = bt[1 * 64 + lane];
    const v4i bve = bt[2 * 64 + lane], bvo = bt[3 * 64 + lane];
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();

    uint8_t *At = lds;
    uint8_t *Qt = lds;
    if constexpr (EPI == EPI_DECAY) {
        // the window holds states; derive the alive map the band products read
        uint8_t *Alive = lds + tile_bytes;
        const int nvec = (p.TH + 2 * p.L) * p.PS >> 4;
        for (int v = tid; v < nvec; v += blockDim.x) {
            uint4 q = *reinterpret_cast<const uint4 *>(Qt + (v << 4));
            *reinterpret_cast<uint4 *>(Alive + (v << 4)) =
                make_uint4(alive_of(q.x), alive_of(q.y), alive_of(q.z), alive_of(q.w));
        }
        __syncthreads();
        At = Alive;
    }
    // no masking needed when every cell this tile computes lies inside the grid
    const int E1 = p.L - 16;
    const bool interior = gi0 - E1 >= 0 && gi0 + p.TH + E1 <= p.H && gj0 - E1 >= 0 && gj0 + p.TW + E1 <= p.W;
    if (interior)
        cat_steps<EPI, false>(p, At, Qt, gi0, gj0, wave, lane, bh0, bh1, bve, bvo);
    else
        cat_steps<EPI, true>(p, At, Qt, gi0, gj0, wave, lane, bh0, bh1, bve, bvo);
}

size_t cat_lds_bytes(const CatParams &p, int elem, int epi) {
    (void)elem;
    return (size_t)cat_tiles_in_lds(p.T, epi) * (size_t)p.lds_tile;
}

static const void *cat_func(int epi) {
    if (epi == EPI_BYTE) return (const void *)&cat_step_i8<EPI_BYTE>;
    if (epi == EPI_HALF) return (const void *)&cat_step_i8<EPI_HALF>;
    return (const void *)&cat_step_i8<EPI_DECAY>;
}

int cat_occupancy(const CatParams &p, int elem, int epi, int waves) {
    const void *f = cat_func(epi);
    size_t lds = cat_lds_bytes(p, elem, epi);
    if (lds > 65536 && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, 64 * waves, lds) != hipSuccess) return 0;
    return nb;
}

KernelLaunch cat_launch_shape(const CatParams &p, int elem, int epi, int waves) {
    KernelLaunch k;
    k.func = cat_func(epi);
    k.lds = cat_lds_bytes(p, elem, epi);
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int x = 0;
        if (hipDeviceGetAttribute(&x, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && x > 0) ncu = x;
    }
    (void)ncu;
    k.grid = dim3((unsigned)((long)p.ntx * p.nty), 1, 1);
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
