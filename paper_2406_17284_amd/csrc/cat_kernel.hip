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

__device__ __forceinline__ uint32_t pack_bytes(v4i d) {
    return (uint32_t)d[0] | ((uint32_t)d[1] << 8) | ((uint32_t)d[2] << 16) | ((uint32_t)d[3] << 24);
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

// Next states of 4 adjacent cells from their box counts (centre included) and states.
// Returns the state dword; *alive receives the alive-indicator dword (state == 1).
template <int EPI>
__device__ __forceinline__ uint32_t transition4(v4i n, uint32_t s, const RuleConsts &rc, uint32_t *alive) {
    if constexpr (EPI == EPI_BYTE) {
        // counts <= 126: per byte a = 0x80 + n - lo has bit 7 iff n >= lo,
        // b = 0x80 + hi - n has bit 7 iff n <= hi; lo/hi picked per byte by the centre state
        uint32_t N = pack_bytes(n);
        uint32_t sm = (0x80808080u - s) ^ 0x80808080u;  // 0xFF where s == 1
        uint32_t a = N + bfi(sm, rc.klo_s, rc.klo_b);
        uint32_t b = bfi(sm, rc.khi_s, rc.khi_b) - N;
        uint32_t x = ((a & b) >> 7) & 0x01010101u;
        *alive = x;
        return x;
    } else if constexpr (EPI == EPI_HALF) {
        // the same test on 16-bit lanes, two cells per dword
        uint32_t p01 = (uint32_t)n[0] | ((uint32_t)n[1] << 16);
        uint32_t p23 = (uint32_t)n[2] | ((uint32_t)n[3] << 16);
        uint32_t s01 = (s & 0xFFu) | ((s & 0xFF00u) << 8);
        uint32_t s23 = ((s >> 16) & 0xFFu) | ((s >> 8) & 0xFF0000u);
        uint32_t m01 = (0x80008000u - s01) ^ 0x80008000u;
        uint32_t m23 = (0x80008000u - s23) ^ 0x80008000u;
        uint32_t x01 = (p01 + bfi(m01, rc.klo_s, rc.klo_b)) & (bfi(m01, rc.khi_s, rc.khi_b) - p01);
        uint32_t x23 = (p23 + bfi(m23, rc.klo_s, rc.klo_b)) & (bfi(m23, rc.khi_s, rc.khi_b) - p23);
        // bits 15 and 31 of x01, x23 -> bit 7 of bytes 0..3, then down to bit 0
        uint32_t y = __builtin_amdgcn_perm(x23, x01, 0x07050301u);
        uint32_t x = (y >> 7) & 0x01010101u;
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
        *alive = al;
        return out;
    }
}

// alive indicator (byte == 1) of a dword of states, any byte values
__device__ __forceinline__ uint32_t alive_of(uint32_t s) {
    uint32_t x = s ^ 0x01010101u;                              // zero byte iff state == 1
    uint32_t y = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;         // bit 7 iff byte != 0
    return (~y & 0x80808080u) >> 7;
}

// Band operands. Lane (n = lane % 16, g = lane / 16); byte e of dword d is K slot 16 g + 4 d + e.
//  MFMA #1, half h (output columns 16 h .. 16 h + 15 of a 32-column strip whose 64-column
//  window starts 16 columns left of the strip): weight 1 iff |k - 16 - 16 h - n| <= r.
__device__ __forceinline__ v4i band_h(int r, int half, int lane) {
    int n = lane & 15, g = lane >> 4;
    v4i b;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        uint32_t w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int k = 16 * g + 4 * d + e;
            int dist = k - 16 - 16 * half - n;
            w |= (uint32_t)((dist >= -r && dist <= r) ? 1 : 0) << (8 * e);
        }
        b[d] = (int32_t)w;
    }
    return b;
}

//  MFMA #2, ring phase p: dword d of every lane holds the H block whose distance to the
//  output block is delta = ((d - p) & 3) - 1 (in units of 16 rows); byte e of that dword is
//  H row 16 delta + 4 g + e relative to the output block. Weight 1 iff |row - n| <= r.
__device__ __forceinline__ v4i band_v(int r, int phase, int lane) {
    int n = lane & 15, g = lane >> 4;
    v4i b;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        int delta = ((d - phase) & 3) - 1;
        uint32_t w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int row = 16 * delta + 4 * g + e;
            int dist = row - n;
            w |= (uint32_t)((dist >= -r && dist <= r) ? 1 : 0) << (8 * e);
        }
        b[d] = (int32_t)w;
    }
    return b;
}

template <int EPI>
__global__ void __launch_bounds__(1024) cat_step_i8(CatParams p) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int nwaves = blockDim.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int PS = p.PS;
    const int L = p.L;
    const size_t tile_bytes = (size_t)p.lds_rows * PS;
    const bool multi = p.T > 1;
    // LDS tiles: alive maps A[0..1] and, for decay, state maps Q[0..1]
    uint8_t *A0 = lds;
    uint8_t *A1 = multi ? lds + tile_bytes : lds;
    uint8_t *Q0 = lds + (multi ? 2 : 1) * tile_bytes;
    uint8_t *Q1 = multi ? Q0 + tile_bytes : Q0;

    const int gi0 = blockIdx.y * p.TH;
    const int gj0 = blockIdx.x * p.TW;

    // ---- load the tile + margin (16-byte vectors, zero outside the grid)
    {
        const int vpr = (p.TW + 2 * L) >> 4;
        const int nvec = p.lds_rows * vpr;
        for (int v = tid; v < nvec; v += blockDim.x) {
            int lr = v / vpr;
            int lc = (v - lr * vpr) << 4;
            int gr = gi0 - L + lr;
            int gc = gj0 - L + lc;
            uint4 x = make_uint4(0, 0, 0, 0);
            if ((unsigned)gr < (unsigned)p.H && (unsigned)gc < (unsigned)p.pitch)
                x = *reinterpret_cast<const uint4 *>(p.src + (size_t)gr * p.pitch + gc);
            size_t off = (size_t)lr * PS + lc;
            if constexpr (EPI == EPI_DECAY) {
                uint4 a = make_uint4(alive_of(x.x), alive_of(x.y), alive_of(x.z), alive_of(x.w));
                *reinterpret_cast<uint4 *>(A0 + off) = a;
                *reinterpret_cast<uint4 *>(Q0 + off) = x;
                if (multi) {
                    *reinterpret_cast<uint4 *>(A1 + off) = a;
                    *reinterpret_cast<uint4 *>(Q1 + off) = x;
                }
            } else {
                *reinterpret_cast<uint4 *>(A0 + off) = x;
                if (multi) *reinterpret_cast<uint4 *>(A1 + off) = x;
            }
        }
    }

    const v4i bh0 = band_h(p.r, 0, lane);
    const v4i bh1 = band_h(p.r, 1, lane);
    const v4i bv0 = band_v(p.r, 0, lane);
    const v4i bv1 = band_v(p.r, 1, lane);
    const v4i bv2 = band_v(p.r, 2, lane);
    const v4i bv3 = band_v(p.r, 3, lane);
    const v4i zero = {0, 0, 0, 0};
    __syncthreads();

    int cur = 0;
    for (int t = 1; t <= p.T; ++t) {
        const bool last = (t == p.T);
        const int E = (p.r * (p.T - t) + 15) & ~15;
        const int nstrips = (p.TW + 2 * E) >> 5;
        const int nrb = (p.TH + 2 * E) >> 4;
        const int nseg = (nwaves + nstrips - 1) / nstrips;
        const int seglen = (nrb + nseg - 1) / nseg;
        const int items = nstrips * nseg;
        const uint8_t *Ac = cur ? A1 : A0;
        uint8_t *An = cur ? A0 : A1;
        const uint8_t *Qc = cur ? Q1 : Q0;
        uint8_t *Qn = cur ? Q0 : Q1;

        for (int it = wave; it < items; it += nwaves) {
            const int strip = it % nstrips;
            const int seg = it / nstrips;
            const int mb_lo = seg * seglen;
            const int mb_hi = min(nrb, mb_lo + seglen);
            if (mb_lo >= mb_hi) continue;
            const int j0 = -E + 32 * strip;           // strip's first column, tile-relative
            const int rb0 = -(E >> 4) + mb_lo;        // first output row block, tile-relative
            const int count = mb_hi - mb_lo;

            // column masks of this lane's 4 output cells in the two halves
            const int gca = gj0 + j0 + 4 * lg;
            const int gcb = gca + 16;
            const uint32_t cma = col_mask(gca, p.W);
            const uint32_t cmb = col_mask(gcb, p.W);

            // LDS address of this lane's 16-byte A chunk for H block b:
            // row 16 b + li, columns j0 - 16 + 16 lg .. + 16
            const uint8_t *abase = Ac + (size_t)(L + li) * PS + (L + j0 - 16 + 16 * lg);
            auto h_block = [&](int b, uint32_t &ha, uint32_t &hb) {
                v4i a = *reinterpret_cast<const v4i *>(abase + (ptrdiff_t)(16 * b) * PS);
                v4i da = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, bh0, zero, 0, 0, 0);
                v4i db = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, bh1, zero, 0, 0, 0);
                ha = pack_bytes(da);
                hb = pack_bytes(db);
            };

            // ring: slot d holds H block rb0 - 1 + d (mod 4)
            v4i ra = zero, rbv = zero;
            {
                uint32_t x, y;
                h_block(rb0 - 1, x, y);
                ra[0] = (int32_t)x; rbv[0] = (int32_t)y;
                h_block(rb0, x, y);
                ra[1] = (int32_t)x; rbv[1] = (int32_t)y;
            }

            auto out_block = [&](int m, v4i ca, v4i cb) {
                // tile-relative row of this lane's cells; columns j0 + 4 lg (+16)
                const int rr = 16 * m + li;
                const int gr = gi0 + rr;
                const uint32_t rowm = ((unsigned)gr < (unsigned)p.H) ? 0xFFFFFFFFu : 0u;
                const size_t loff = (size_t)(L + rr) * PS + (L + j0 + 4 * lg);
                uint32_t sa, sb;
                if constexpr (EPI == EPI_DECAY) {
                    sa = *reinterpret_cast<const uint32_t *>(Qc + loff);
                    sb = *reinterpret_cast<const uint32_t *>(Qc + loff + 16);
                } else {
                    sa = *reinterpret_cast<const uint32_t *>(Ac + loff);
                    sb = *reinterpret_cast<const uint32_t *>(Ac + loff + 16);
                }
                uint32_t ala, alb;
                uint32_t na = transition4<EPI>(ca, sa, p.rc, &ala) & (rowm & cma);
                uint32_t nb = transition4<EPI>(cb, sb, p.rc, &alb) & (rowm & cmb);
                if (last) {
                    if (rowm) {
                        uint8_t *drow = p.dst + (size_t)gr * p.pitch;
                        if ((unsigned)gca < (unsigned)p.pitch) *reinterpret_cast<uint32_t *>(drow + gca) = na;
                        if ((unsigned)gcb < (unsigned)p.pitch) *reinterpret_cast<uint32_t *>(drow + gcb) = nb;
                    }
                } else {
                    if constexpr (EPI == EPI_DECAY) {
                        *reinterpret_cast<uint32_t *>(Qn + loff) = na;
                        *reinterpret_cast<uint32_t *>(Qn + loff + 16) = nb;
                        *reinterpret_cast<uint32_t *>(An + loff) = ala & (rowm & cma);
                        *reinterpret_cast<uint32_t *>(An + loff + 16) = alb & (rowm & cmb);
                    } else {
                        *reinterpret_cast<uint32_t *>(An + loff) = na;
                        *reinterpret_cast<uint32_t *>(An + loff + 16) = nb;
                    }
                }
            };

            // one output row block: H block m + 1 into ring slot (q + 2) & 3, then MFMA #2
            // with the band phase q & 3, then the transition
#define CAT_STEP(Q)                                                                   \
    if (q + (Q) < count) {                                                            \
        const int m = rb0 + q + (Q);                                                  \
        uint32_t x, y;                                                                \
        h_block(m + 1, x, y);                                                         \
        ra[((Q) + 2) & 3] = (int32_t)x;                                               \
        rbv[((Q) + 2) & 3] = (int32_t)y;                                              \
        const v4i bv = ((Q) & 3) == 0 ? bv0 : ((Q) & 3) == 1 ? bv1 : ((Q) & 3) == 2 ? bv2 : bv3; \
        v4i ca = __builtin_amdgcn_mfma_i32_16x16x64_i8(ra, bv, zero, 0, 0, 0);       \
        v4i cb = __builtin_amdgcn_mfma_i32_16x16x64_i8(rbv, bv, zero, 0, 0, 0);      \
        out_block(m, ca, cb);                                                         \
    }
            for (int q = 0; q < count; q += 4) {
                CAT_STEP(0)
                CAT_STEP(1)
                CAT_STEP(2)
                CAT_STEP(3)
            }
#undef CAT_STEP
        }
        if (!last) __syncthreads();
        cur ^= 1;
    }
}

size_t cat_lds_bytes(const CatParams &p, int elem, int epi) {
    (void)elem;
    return (size_t)cat_tiles_in_lds(p.T, epi) * p.lds_rows * p.PS;
}

KernelLaunch cat_launch_shape(const CatParams &p, int elem, int epi, int waves) {
    KernelLaunch k;
    (void)elem;
    if (epi == EPI_BYTE) k.func = (const void *)&cat_step_i8<EPI_BYTE>;
    else if (epi == EPI_HALF) k.func = (const void *)&cat_step_i8<EPI_HALF>;
    else k.func = (const void *)&cat_step_i8<EPI_DECAY>;
    k.grid = dim3((p.W + p.TW - 1) / p.TW, (p.H + p.TH - 1) / p.TH, 1);
    k.block = dim3(64 * waves, 1, 1);
    k.lds = cat_lds_bytes(p, elem, epi);
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
