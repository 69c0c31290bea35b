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
// Precision variants (all exact by construction, so every variant gives the same grid):
//  * ELEM_I8  int8 operands, int32 accumulation (v_mfma_i32_16x16x64_i8): exact for r <= 16.
//  * ELEM_F8  fp8-e4m3 operands (v_mfma_f32_16x16x32_fp8_fp8), fp32 accumulation: H <= 2r+1 is
//             exact in e4m3 only while 2r+1 <= 16 (r <= 7; the host refuses larger r).
//  * ELEM_F16 fp16 operands (v_mfma_f32_16x16x32_f16), fp32 accumulation: exact for r <= 16
//             (the paper's own precision argument: counts <= 33^2 - 1 < 2^11).
// The fp32 accumulators of MFMA #2 start at 2^23, so the count lands in the low mantissa bits
// and the same integer epilogue applies. The fp8 encoding of 1.0 is taken from the hardware
// conversion instruction, so tile, band and H encodings always match the MFMA's format.
//
// Temporal blocking (multi-step idea cited in the paper's related work): the tile plus a
// margin L = roundup16(r (T-1)) + 16 is loaded once into LDS; step t recomputes the tile
// grown by roundup16(r (T - t)) cells, so after T steps the tile itself is exact. Cells
// outside the grid are forced to 0 after every step (dead ghost halo).
#pragma once
#include "ltl_internal.h"

namespace ltl {

typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef int32_t v2i __attribute__((ext_vector_type(2)));
typedef int32_t v16i __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef uint16_t us2 __attribute__((ext_vector_type(2)));

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

// alive indicator (byte == 1) of a dword of states, any byte values
__device__ __forceinline__ uint32_t alive_of(uint32_t s) {
    uint32_t x = s ^ 0x01010101u;                              // zero byte iff state == 1
    uint32_t y = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;         // bit 7 iff byte != 0
    return (~y & 0x80808080u) >> 7;
}

// Range test of 4 cells on 16-bit SWAR lanes (counts up to 32767): byte v of the result is 1
// iff lo(a) <= n[v] <= hi(a), a = byte v of `a` (0: birth range, 1: survival range), with
// a = 0x8000 + n - lo and b = 0x8000 + hi - n as for the byte lanes. Only the low 16 bits of
// each count are used, which also strips the 2^23 bias of the fp32 accumulators.
__device__ __forceinline__ uint32_t inrange16(v4i n, uint32_t a, const RuleConsts &rc) {
    const uint32_t p01 = __builtin_amdgcn_perm((uint32_t)n[1], (uint32_t)n[0], 0x05040100u);
    const uint32_t p23 = __builtin_amdgcn_perm((uint32_t)n[3], (uint32_t)n[2], 0x05040100u);
    const uint32_t s01 = __builtin_amdgcn_perm(0u, a, 0x0c010c00u);  // bytes 0, 1 -> 16-bit lanes
    const uint32_t s23 = __builtin_amdgcn_perm(0u, a, 0x0c030c02u);
    const uint32_t sm01 = 0x80008000u - s01;
    const uint32_t sm23 = 0x80008000u - s23;
    const uint32_t x01 = (p01 + (rc.Klo ^ (sm01 & rc.Dlo))) & ((rc.Khi ^ (sm01 & rc.Dhi)) - p01) & 0x80008000u;
    const uint32_t x23 = (p23 + (rc.Klo ^ (sm23 & rc.Dlo))) & ((rc.Khi ^ (sm23 & rc.Dhi)) - p23) & 0x80008000u;
    // bits 15 and 31 of x01, x23 -> bit 7 of bytes 0..3, then down to bit 0
    return __builtin_amdgcn_perm(x23, x01, 0x07050301u) >> 7;
}

// Counts n - c of 4 cells (int32, c the window offset) as bytes, clamped to 255: the low 16 bits
// of each go through an unsigned 16-bit min, so values above the window and negative ones (whose
// low halves are at least 0x8000) both become 255, which lies outside every range of the window.
__device__ __forceinline__ uint32_t window_bytes255(v4i n) {
    const us2 cap = {255, 255};
    const us2 p01 = __builtin_elementwise_min(
        __builtin_bit_cast(us2, __builtin_amdgcn_perm((uint32_t)n[1], (uint32_t)n[0], 0x05040100u)), cap);
    const us2 p23 = __builtin_elementwise_min(
        __builtin_bit_cast(us2, __builtin_amdgcn_perm((uint32_t)n[3], (uint32_t)n[2], 0x05040100u)), cap);
    return __builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, p23), __builtin_bit_cast(uint32_t, p01), 0x06040200u);
}

// Range test of 4 byte counts x (0..255): bit 7 of byte v of the result is set iff
// lo(s) <= x[v] <= hi(s), with s the byte v of `s` selecting byte s of the tables Tlo = 256 - lo,
// Thi = hi + 1 (1 <= lo, hi <= 254). v_lerp_u8 gives (a + b) >> 1 per byte from a 9-bit sum, so
// its bit 7 is the carry out of a + b: x + 256 - lo >= 256 iff x >= lo, and
// (255 - x) + hi + 1 >= 256 iff x <= hi.
__device__ __forceinline__ uint32_t inrange8(uint32_t x, uint32_t s, const RuleConsts &rc) {
    const uint32_t ge = __builtin_amdgcn_lerp(x, __builtin_amdgcn_perm(rc.Tlo, rc.Tlo, s), 0u);
    const uint32_t le = __builtin_amdgcn_lerp(~x, __builtin_amdgcn_perm(rc.Thi, rc.Thi, s), 0u);
    return ge & le;
}

// Next states of 4 adjacent cells from their box counts n (centre included) and states s.
// `m` is the validity mask of the 4 cells (0xFF per byte inside the grid); cells outside get 0.
// Returns the state dword; *alive receives the alive-indicator dword (state == 1).
//
// Two-state rules test lo(s) <= n <= hi(s) on 8-bit (BYTE) or 16-bit (HALF) SWAR lanes:
// a = 0x80 + n - lo has its top bit set iff n >= lo, b = 0x80 + hi - n iff n <= hi (no lane
// carries or borrows: n, lo, hi <= 127, resp. 2047). BYTE takes the per-lane offsets from the
// centre states (0 or 1 per byte) with one byte permute each, the states acting as byte
// selectors into a two-entry table; HALF derives them with 3-input bitwise ops.
template <int EPI>
__device__ __forceinline__ uint32_t transition4(v4i n, uint32_t s, uint32_t m, const RuleConsts &rc,
                                                uint32_t *alive) {
    if constexpr (EPI == EPI_BYTE || EPI == EPI_WIN) {
        uint32_t N;
        if constexpr (EPI == EPI_BYTE) {
            N = pack_bytes(n);
        } else {
            // counts arrive as n - c: low 16 bits clamped to 127 (values above the window and
            // negative ones both become 127, outside every shifted range), then one byte each
            const us2 cap = {127, 127};
            const us2 p01 = __builtin_elementwise_min(
                __builtin_bit_cast(us2, __builtin_amdgcn_perm((uint32_t)n[1], (uint32_t)n[0], 0x05040100u)), cap);
            const us2 p23 = __builtin_elementwise_min(
                __builtin_bit_cast(us2, __builtin_amdgcn_perm((uint32_t)n[3], (uint32_t)n[2], 0x05040100u)), cap);
            N = __builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, p23), __builtin_bit_cast(uint32_t, p01),
                                      0x06040200u);
        }
        uint32_t a = N + __builtin_amdgcn_perm(rc.Tlo, rc.Tlo, s);
        uint32_t b = __builtin_amdgcn_perm(rc.Thi, rc.Thi, s) - N;
        uint32_t x = (a & b & (m & 0x80808080u)) >> 7;
        *alive = x;
        return x;
    } else if constexpr (EPI == EPI_WIN8) {
        // counts arrive as n - c (window up to 254 wide)
        const uint32_t x = (inrange8(window_bytes255(n), s, rc) & (m & 0x80808080u)) >> 7;
        *alive = x;
        return x;
    } else if constexpr (EPI == EPI_HALF) {
        const uint32_t x = inrange16(n, s, rc) & m;
        *alive = x;
        return x;
    } else if constexpr (EPI == EPI_DECAY8W) {
        // as EPI_DECAY8, with the range test on the windowed bytes; the tables are read with any
        // state byte 0..7 (states >= 2 decay whatever the test gives)
        const uint32_t x = (inrange8(window_bytes255(n), s, rc) & 0x80808080u) >> 7;
        const uint32_t n0 = __builtin_amdgcn_perm(rc.N0hi, rc.N0lo, s);
        const uint32_t n1 = __builtin_amdgcn_perm(rc.N1hi, rc.N1lo, s);
        const uint32_t nx = __builtin_amdgcn_perm(n1, n0, (x << 2) | 0x03020100u) & m;
        *alive = __builtin_amdgcn_perm(0u, 0x00000100u, nx);         // next state == 1
        return nx;
    } else if constexpr (EPI == EPI_DECAY8) {
        // C <= 8: the state bytes (0..7) select from 8-byte tables with one byte permute each:
        // the alive bit (state == 1), and the next state when the range test fails (N0) or holds
        // (N1); the test result (0/1 per byte) then picks N1's byte over N0's as a selector offset.
        const uint32_t a1 = __builtin_amdgcn_perm(0u, 0x00000100u, s);
        const uint32_t x = inrange16(n, a1, rc);                     // range of the s in {0, 1} case
        const uint32_t n0 = __builtin_amdgcn_perm(rc.N0hi, rc.N0lo, s);
        const uint32_t n1 = __builtin_amdgcn_perm(rc.N1hi, rc.N1lo, s);
        const uint32_t nx = __builtin_amdgcn_perm(n1, n0, (x << 2) | 0x03020100u) & m;
        *alive = __builtin_amdgcn_perm(0u, 0x00000100u, nx);         // next state == 1
        return nx;
    } else {
        // C >= 3. Per byte, g = 1 where the cell leaves its state: birth (s = 0, n in the birth
        // range), death (s = 1, n outside the survival range) or decay (s >= 2); the next state
        // is s + g, and a byte that reaches C wraps to 0 (only decaying cells get there).
        const uint32_t a1 = alive_of(s);
        const uint32_t x = inrange16(n, a1, rc);                     // range of the s in {0, 1} case
        const uint32_t d = ((((s & 0x7E7E7E7Eu) + 0x7E7E7E7Eu) | s) >> 7) & 0x01010101u;   // s >= 2
        const uint32_t nx = s + ((x ^ a1) | d);
        const uint32_t e = nx ^ rc.Crep;                             // zero byte where nx == C
        const uint32_t keep = (((e & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | e) & 0x80808080u;
        const uint32_t km = keep | (keep - (keep >> 7));             // 0xFF per byte to keep
        *alive = x & ~d & m;                                         // next state == 1
        return nx & km & m;
    }
}



// ---------------------------------------------------------------- element encodings
// Per element type: bytes per cell of the alive map in LDS, the longest run of output blocks a
// wave handles per step (bounded by the register tuple that holds H), the number of band
// operands, and the encode / decode between alive bytes (0/1) and the LDS encoding.
template <int ELEM> struct ElemT;
template <> struct ElemT<ELEM_I8> { static constexpr int CELL = 1, MAXC = CAT_MAXC_I8, NOPS = 4; };
template <> struct ElemT<ELEM_I8W> { static constexpr int CELL = 1, MAXC = CAT_MAXC_I8W, NOPS = 8; };
template <> struct ElemT<ELEM_I8X> { static constexpr int CELL = 1, MAXC = CAT_MAXC_I8X, NOPS = 8; };
// int8 element types (0/1 bytes, the state tile is the alive map for two-state rules)
template <int ELEM> constexpr bool kIsI8 = (ELEM == ELEM_I8 || ELEM == ELEM_I8W || ELEM == ELEM_I8X);
template <> struct ElemT<ELEM_F8> { static constexpr int CELL = 1, MAXC = CAT_MAXC_F8, NOPS = 8; };
template <> struct ElemT<ELEM_F16> { static constexpr int CELL = 1, MAXC = CAT_MAXC_F16, NOPS = 6; };

struct Codec {
    uint32_t one8;   // fp8 encoding of 1.0 (byte), as the hardware converts it
    uint32_t sh8;    // its lowest set bit
};

__device__ __forceinline__ Codec make_codec() {
    Codec c;
    c.one8 = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(1.0f, 0.0f, 0, false) & 0xFFu;
    c.sh8 = (uint32_t)__builtin_ctz(c.one8);
    return c;
}

// alive bytes (0/1) -> fp8 bytes (0 / 1.0): a byte permute with the alive bytes as selectors
__device__ __forceinline__ uint32_t enc8(uint32_t alive, const Codec &c) {
    return __builtin_amdgcn_perm(0u, c.one8 << 8, alive);
}
__device__ __forceinline__ uint32_t dec8(uint32_t x, const Codec &c) { return (x >> c.sh8) & 0x01010101u; }
// alive bytes -> four fp16 (0 / 1.0 = 0x3C00), two per dword
__device__ __forceinline__ uint2 enc16(uint32_t alive) {
    uint32_t lo = __builtin_amdgcn_perm(0u, alive, 0x0c010c00u);   // bytes 0, 1 -> 16-bit lanes
    uint32_t hi = __builtin_amdgcn_perm(0u, alive, 0x0c030c02u);
    return make_uint2(__umul24(lo, 0x3C00u), __umul24(hi, 0x3C00u));
}

// Geometry of one step: strips of 32 columns, each cut into `nseg` row segments of at most
// MAXC 16-row blocks. Every segment is one wave's work item; a step needs items <= waves (the
// host planner checks this for every step of a launch).
struct StepGeom {
    int E, nstrips, nrb, nseg, seglen;
};

// `last`: t == p.T (passed in, so that a caller that peels the last step folds it).
template <int MAXC>
__device__ __forceinline__ StepGeom step_geom(const CatParams &p, int t, bool last) {
    StepGeom g;
    // the margin is roundup16(r (T - 1)) + 16 (+ 48 for the wide element, never 32), so a
    // 32-cell margin means 1 <= r (T - 1) <= 16 and every step but the last extends exactly 16:
    // the general rule's value, in a form a kernel with the margin fixed folds
    g.E = (p.L == 32) ? (last ? 0 : 16) : ((p.r * (p.T - t) + 15) & ~15);
    g.nstrips = (p.TW + 2 * g.E) >> 5;
    g.nrb = (p.TH + 2 * g.E) >> 4;
    if (g.nrb <= MAXC) {   // one segment per strip (the usual case): no integer division
        g.nseg = 1;
        g.seglen = g.nrb;
    } else {
        g.nseg = (g.nrb + MAXC - 1) / MAXC;
        g.seglen = (g.nrb + g.nseg - 1) / g.nseg;
    }
    return g;
}

// Band operands of one launch (up to 8 per lane, 16 bytes each; fp8 operands use 8 bytes).
struct Bands {
    v4i op[8];
};

template <int K>
__device__ __forceinline__ v4i window4(const v16i &h) {
    return __builtin_shufflevector(h, h, K, K + 1, K + 2, K + 3);
}
template <int K>
__device__ __forceinline__ long window2(const v16i &h) {
    v2i w = __builtin_shufflevector(h, h, K, K + 1);
    return __builtin_bit_cast(long, w);
}
__device__ __forceinline__ long lo8(const v4i &x) {
    v2i w = __builtin_shufflevector(x, x, 0, 1);
    return __builtin_bit_cast(long, w);
}
__device__ __forceinline__ v8h as_h8(const v4i &x) { return __builtin_bit_cast(v8h, x); }
__device__ __forceinline__ uint32_t pack_f8(v4f d) {
    int x = __builtin_amdgcn_cvt_pk_fp8_f32(d[0], d[1], 0, false);
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(d[2], d[3], x, true);
}
__device__ __forceinline__ uint32_t pack_f16(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(a, b));
}

// H of one item and one 16-column half lives in a 16-register tuple: element k holds the
// packed H of block rb0 - 1 + k (fp16: elements 2k, 2k + 1). Output block M needs
// k = M, M+1, M+2. int8: MFMA #2 reads the even-aligned 4-register window starting at M (M
// even) or M - 1 (M odd), one MFMA per block and two band phases. fp8 (K = 32): two MFMAs on
// 2-register windows. fp16 (K = 32): two MFMAs on the 4-register windows of blocks (M, M+1)
// and (M+2, M+3). No register copies in any case.

// Phase A of one item: H (horizontal band sums) of blocks rb0 - 1 .. rb0 + count for both
// 16-column halves of the strip, packed, in registers. Software-pipelined in pairs of blocks:
// the A chunks of the next pair are read from LDS before the MFMAs of this pair run.
// FROM_STATES: At holds states (int8 Moore with decay): each chunk's alive bits (state == 1)
// are derived in registers as it is read, with SWAR arithmetic (1, any state byte) or one byte
// permute per dword (2, states 0..7).
template <int ELEM, int FROM_STATES = 0>
__device__ __forceinline__ void phase_a(const uint8_t *At, uint32_t a_off, uint32_t a_off2, uint32_t PA, int rb0,
                                        int count, const Bands &bd, v16i &Ha, v16i &Hb, v16i &La, v16i &Lb) {
    if constexpr (ELEM == ELEM_I8X) {
        // cross: per 16-row block and half, H (horizontal arm) and the alive map itself in the
        // same register layout (identity band), both from the one A chunk
        const int nh = count + 2;
        const v4i zero = {0, 0, 0, 0};
        v4i a[4];
#define CAT_LDA(K) a[(K) & 3] = *reinterpret_cast<const v4i *>(At + (a_off + (uint32_t)(16 * (rb0 - 1 + (K))) * PA));
#define CAT_HB(K)                                                                                  \
        {                                                                                          \
            Ha[(K)] = (int32_t)pack_bytes(__builtin_amdgcn_mfma_i32_16x16x64_i8(a[(K) & 3], bd.op[0], zero, 0, 0, 0)); \
            Hb[(K)] = (int32_t)pack_bytes(__builtin_amdgcn_mfma_i32_16x16x64_i8(a[(K) & 3], bd.op[1], zero, 0, 0, 0)); \
            La[(K)] = (int32_t)pack_bytes(__builtin_amdgcn_mfma_i32_16x16x64_i8(a[(K) & 3], bd.op[2], zero, 0, 0, 0)); \
            Lb[(K)] = (int32_t)pack_bytes(__builtin_amdgcn_mfma_i32_16x16x64_i8(a[(K) & 3], bd.op[3], zero, 0, 0, 0)); \
        }
#define CAT_APAIR(P)                                                                               \
        if (2 * (P) < nh) {                                                                        \
            if (2 * (P) + 2 < nh) {                                                                \
                CAT_LDA(2 * (P) + 2)                                                               \
                if (2 * (P) + 3 < nh) CAT_LDA(2 * (P) + 3)                                         \
            }                                                                                      \
            CAT_HB(2 * (P))                                                                        \
            if (2 * (P) + 1 < nh) CAT_HB(2 * (P) + 1)                                              \
        }
        CAT_LDA(0) CAT_LDA(1)
        CAT_APAIR(0) CAT_APAIR(1) CAT_APAIR(2) CAT_APAIR(3)   // at most CAT_MAXC_I8X + 2 = 8 blocks
#undef CAT_APAIR
#undef CAT_HB
#undef CAT_LDA
        return;
    }
    (void)La;
    (void)Lb;
    if constexpr (ELEM == ELEM_I8W) {
        // radius 17..32: H blocks rb0 - 2 .. rb0 + count + 2; per half a K = 64 product on the
        // chunk at a_off plus a product on the 8 bytes at a_off2 (32 columns). The second product
        // also runs as 16x16x64: its band has zero weight in the upper 8 bytes of every lane, so
        // the A operand's upper half is left undefined, and the two products chain through the
        // accumulator of one instruction shape (a 16x16x64 result fed as the accumulator of a
        // 16x16x32 instruction gave wrong sums on gfx950 with this toolchain).
        const int nh = count + 5;
        const v4i zero = {0, 0, 0, 0};
        v4i a[4];
        long b[4];
#define CAT_LDA(K)                                                                                 \
        {                                                                                          \
            const uint32_t ro = (uint32_t)(16 * (rb0 - 2 + (K))) * PA;                             \
            a[(K) & 3] = *reinterpret_cast<const v4i *>(At + (a_off + ro));                        \
            b[(K) & 3] = *reinterpret_cast<const long *>(At + (a_off2 + ro));                      \
        }
#define CAT_HB(K)                                                                                  \
        {                                                                                          \
            const v2i b2 = __builtin_bit_cast(v2i, b[(K) & 3]);                                    \
            const v4i b4 = __builtin_shufflevector(b2, b2, 0, 1, -1, -1);                          \
            v4i da = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[(K) & 3], bd.op[0], zero, 0, 0, 0);   \
            da = __builtin_amdgcn_mfma_i32_16x16x64_i8(b4, bd.op[1], da, 0, 0, 0);                 \
            v4i db = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[(K) & 3], bd.op[2], zero, 0, 0, 0);   \
            db = __builtin_amdgcn_mfma_i32_16x16x64_i8(b4, bd.op[3], db, 0, 0, 0);                 \
            Ha[(K)] = (int32_t)pack_bytes(da);                                                     \
            Hb[(K)] = (int32_t)pack_bytes(db);                                                     \
        }
#define CAT_APAIR(P)                                                                               \
        if (2 * (P) < nh) {                                                                        \
            if (2 * (P) + 2 < nh) {                                                                \
                CAT_LDA(2 * (P) + 2)                                                               \
                if (2 * (P) + 3 < nh) CAT_LDA(2 * (P) + 3)                                         \
            }                                                                                      \
            CAT_HB(2 * (P))                                                                        \
            if (2 * (P) + 1 < nh) CAT_HB(2 * (P) + 1)                                              \
        }
        CAT_LDA(0) CAT_LDA(1)
        CAT_APAIR(0) CAT_APAIR(1) CAT_APAIR(2) CAT_APAIR(3) CAT_APAIR(4) CAT_APAIR(5) CAT_APAIR(6) CAT_APAIR(7)
#undef CAT_APAIR
#undef CAT_HB
#undef CAT_LDA
        return;
    }
    (void)a_off2;
    const int nh = count + 2;
    if constexpr (ELEM == ELEM_I8) {
        const v4i zero = {0, 0, 0, 0};
        v4i a[4];
#define CAT_LDA(K)                                                                                 \
        {                                                                                          \
            v4i q = *reinterpret_cast<const v4i *>(At + (a_off + (uint32_t)(16 * (rb0 - 1 + (K))) * PA)); \
            if constexpr (FROM_STATES == 1) {                                                      \
                q[0] = (int32_t)alive_of((uint32_t)q[0]);                                          \
                q[1] = (int32_t)alive_of((uint32_t)q[1]);                                          \
                q[2] = (int32_t)alive_of((uint32_t)q[2]);                                          \
                q[3] = (int32_t)alive_of((uint32_t)q[3]);                                          \
            } else if constexpr (FROM_STATES == 2) {                                               \
                q[0] = (int32_t)__builtin_amdgcn_perm(0u, 0x00000100u, (uint32_t)q[0]);            \
                q[1] = (int32_t)__builtin_amdgcn_perm(0u, 0x00000100u, (uint32_t)q[1]);            \
                q[2] = (int32_t)__builtin_amdgcn_perm(0u, 0x00000100u, (uint32_t)q[2]);            \
                q[3] = (int32_t)__builtin_amdgcn_perm(0u, 0x00000100u, (uint32_t)q[3]);            \
            }                                                                                      \
            a[(K) & 3] = q;                                                                        \
        }
#define CAT_HB(K)                                                                                  \
        {                                                                                          \
            v4i da = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[(K) & 3], bd.op[0], zero, 0, 0, 0);   \
            v4i db = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[(K) & 3], bd.op[1], zero, 0, 0, 0);   \
            Ha[(K)] = (int32_t)pack_bytes(da);                                                     \
            Hb[(K)] = (int32_t)pack_bytes(db);                                                     \
        }
#define CAT_APAIR(P)                                                                               \
        if (2 * (P) < nh) {                                                                        \
            if (2 * (P) + 2 < nh) {                                                                \
                CAT_LDA(2 * (P) + 2)                                                               \
                if (2 * (P) + 3 < nh) CAT_LDA(2 * (P) + 3)                                         \
            }                                                                                      \
            CAT_HB(2 * (P))                                                                        \
            CAT_HB(2 * (P) + 1)    /* one past the item when nh is odd: zero weight */               \
        }
        CAT_LDA(0) CAT_LDA(1)
        CAT_APAIR(0) CAT_APAIR(1) CAT_APAIR(2) CAT_APAIR(3) CAT_APAIR(4) CAT_APAIR(5) CAT_APAIR(6) CAT_APAIR(7)
#undef CAT_APAIR
#undef CAT_HB
#undef CAT_LDA
    } else if constexpr (ELEM == ELEM_F8) {
        // two K = 32 chunks (8 bytes per lane each, 32 columns apart) per 64-column window
        const v4f zf = {0.f, 0.f, 0.f, 0.f};
        long a0[4], a1[4];
#define CAT_LDA(K)                                                                                 \
        {                                                                                          \
            const uint8_t *q = At + (a_off + (uint32_t)(16 * (rb0 - 1 + (K))) * PA);               \
            a0[(K) & 3] = *reinterpret_cast<const long *>(q);                                      \
            a1[(K) & 3] = *reinterpret_cast<const long *>(q + 32);                                 \
        }
#define CAT_HB(K)                                                                                  \
        {                                                                                          \
            v4f da = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a0[(K) & 3], lo8(bd.op[0]), zf, 0, 0, 0); \
            da = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a1[(K) & 3], lo8(bd.op[1]), da, 0, 0, 0); \
            v4f db = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a0[(K) & 3], lo8(bd.op[2]), zf, 0, 0, 0); \
            db = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a1[(K) & 3], lo8(bd.op[3]), db, 0, 0, 0); \
            Ha[(K)] = (int32_t)pack_f8(da);                                                        \
            Hb[(K)] = (int32_t)pack_f8(db);                                                        \
        }
#define CAT_APAIR(P)                                                                               \
        if (2 * (P) < nh) {                                                                        \
            if (2 * (P) + 2 < nh) {                                                                \
                CAT_LDA(2 * (P) + 2)                                                               \
                if (2 * (P) + 3 < nh) CAT_LDA(2 * (P) + 3)                                         \
            }                                                                                      \
            CAT_HB(2 * (P))                                                                        \
            if (2 * (P) + 1 < nh) CAT_HB(2 * (P) + 1)                                              \
        }
        CAT_LDA(0) CAT_LDA(1)
        CAT_APAIR(0) CAT_APAIR(1) CAT_APAIR(2) CAT_APAIR(3) CAT_APAIR(4) CAT_APAIR(5) CAT_APAIR(6) CAT_APAIR(7)
#undef CAT_APAIR
#undef CAT_HB
#undef CAT_LDA
    } else {
        // fp16: two K = 32 chunks of 8 cells (32 columns apart), read as state bytes from the
        // one tile and expanded in registers to fp16 0 / 1.0 (alive: state == 1)
        const v4f zf = {0.f, 0.f, 0.f, 0.f};
        v4i a0[4], a1[4];
#define CAT_LDA(K)                                                                                 \
        {                                                                                          \
            const uint8_t *q = At + (a_off + (uint32_t)(16 * (rb0 - 1 + (K))) * PA);               \
            uint2 s0 = *reinterpret_cast<const uint2 *>(q);                                        \
            uint2 s1 = *reinterpret_cast<const uint2 *>(q + 32);                                   \
            if constexpr (FROM_STATES != 0) {                                                      \
                s0 = make_uint2(alive_of(s0.x), alive_of(s0.y));                                   \
                s1 = make_uint2(alive_of(s1.x), alive_of(s1.y));                                   \
            }                                                                                      \
            const uint2 e00 = enc16(s0.x), e01 = enc16(s0.y), e10 = enc16(s1.x), e11 = enc16(s1.y); \
            a0[(K) & 3] = v4i{(int32_t)e00.x, (int32_t)e00.y, (int32_t)e01.x, (int32_t)e01.y};     \
            a1[(K) & 3] = v4i{(int32_t)e10.x, (int32_t)e10.y, (int32_t)e11.x, (int32_t)e11.y};     \
        }
#define CAT_HB(K)                                                                                  \
        {                                                                                          \
            v4f da = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_h8(a0[(K) & 3]), as_h8(bd.op[0]), zf, 0, 0, 0); \
            da = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_h8(a1[(K) & 3]), as_h8(bd.op[1]), da, 0, 0, 0); \
            v4f db = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_h8(a0[(K) & 3]), as_h8(bd.op[2]), zf, 0, 0, 0); \
            db = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_h8(a1[(K) & 3]), as_h8(bd.op[3]), db, 0, 0, 0); \
            Ha[2 * (K)] = (int32_t)pack_f16(da[0], da[1]);                                         \
            Ha[2 * (K) + 1] = (int32_t)pack_f16(da[2], da[3]);                                     \
            Hb[2 * (K)] = (int32_t)pack_f16(db[0], db[1]);                                         \
            Hb[2 * (K) + 1] = (int32_t)pack_f16(db[2], db[3]);                                     \
        }
#define CAT_APAIR(P)                                                                               \
        if (2 * (P) < nh) {                                                                        \
            if (2 * (P) + 2 < nh) {                                                                \
                CAT_LDA(2 * (P) + 2)                                                               \
                if (2 * (P) + 3 < nh) CAT_LDA(2 * (P) + 3)                                         \
            }                                                                                      \
            CAT_HB(2 * (P))                                                                        \
            if (2 * (P) + 1 < nh) CAT_HB(2 * (P) + 1)                                              \
        }
        CAT_LDA(0) CAT_LDA(1)
        CAT_APAIR(0) CAT_APAIR(1) CAT_APAIR(2) CAT_APAIR(3)
#undef CAT_APAIR
#undef CAT_HB
#undef CAT_LDA
    }
}

// Vertical band product of output block M for one half (counts as int32 or biased fp32 bits).
// `acc` is the int8 product's starting accumulator (0, or -c for the windowed epilogue).
template <int ELEM, int M>
__device__ __forceinline__ v4i vproduct(const v16i &H, const v16i &L, const Bands &bd, const v4i &acc) {
    if constexpr (ELEM == ELEM_I8X) {
        // cross: H at the centre row (identity window) plus the vertical arm of the alive map
        // (centre excluded), same window of blocks, same instruction, one accumulator
        const v4i zero = {0, 0, 0, 0};
        constexpr int W0 = (M & 1) ? M - 1 : M;
        v4i c = __builtin_amdgcn_mfma_i32_16x16x64_i8(window4<W0>(H), (M & 1) ? bd.op[7] : bd.op[6], zero, 0, 0, 0);
        return __builtin_amdgcn_mfma_i32_16x16x64_i8(window4<W0>(L), (M & 1) ? bd.op[5] : bd.op[4], c, 0, 0, 0);
    } else if constexpr (ELEM == ELEM_I8W) {
        // tuple element k holds block rb0 - 2 + k; output block rb0 + M needs elements M .. M+4.
        // The pair window is the 4-element window from M + 4 (M + 3) whose upper two elements
        // have zero weight (the band's upper 8 bytes per lane are 0).
        const v4i zero = {0, 0, 0, 0};
        if constexpr ((M & 1) == 0) {
            v4i c = __builtin_amdgcn_mfma_i32_16x16x64_i8(window4<M>(H), bd.op[4], zero, 0, 0, 0);
            return __builtin_amdgcn_mfma_i32_16x16x64_i8(window4<M + 4>(H), bd.op[5], c, 0, 0, 0);
        } else {
            v4i c = __builtin_amdgcn_mfma_i32_16x16x64_i8(window4<M - 1>(H), bd.op[6], zero, 0, 0, 0);
            return __builtin_amdgcn_mfma_i32_16x16x64_i8(window4<M + 3>(H), bd.op[7], c, 0, 0, 0);
        }
    } else if constexpr (ELEM == ELEM_I8) {
        constexpr int W0 = (M & 1) ? M - 1 : M;
        return __builtin_amdgcn_mfma_i32_16x16x64_i8(window4<W0>(H), (M & 1) ? bd.op[3] : bd.op[2], acc, 0, 0, 0);
    } else if constexpr (ELEM == ELEM_F8) {
        const v4f bias = {8388608.f, 8388608.f, 8388608.f, 8388608.f};
        constexpr int W0 = (M & 1) ? M - 1 : M;
        v4f c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(window2<W0>(H), lo8((M & 1) ? bd.op[6] : bd.op[4]), bias,
                                                           0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(window2<W0 + 2>(H), lo8((M & 1) ? bd.op[7] : bd.op[5]), c, 0,
                                                       0, 0);
        return __builtin_bit_cast(v4i, c);
    } else {
        const v4f bias = {8388608.f, 8388608.f, 8388608.f, 8388608.f};
        v4f c = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_h8(window4<2 * M>(H)), as_h8(bd.op[4]), bias, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_h8(window4<2 * M + 4>(H)), as_h8(bd.op[5]), c, 0, 0, 0);
        return __builtin_bit_cast(v4i, c);
    }
}

// Offsets of this lane's cells in the LDS tiles: Q holds states (pitch PS, one byte per cell),
// A the alive map in the element encoding (pitch PA). The two are the same bytes except for
// decay rules on fp8 and on the wide and cross int8 elements, which keep a second tile; fp16
// and int8 Moore build their operands (alive bits for decay) in registers from Q.
struct LaneOff {
    uint32_t q, a;   // block-row-0 offset of the lane's first cell of half a (half b: +16 cells)
};

// Phase B of one item: vertical band products, transition, in-place store of the new states in
// LDS (the tile goes to the output grid after the last step, with 16-byte stores). Software-
// pipelined in pairs of output blocks: the MFMAs and centre-state reads of the next pair are
// issued before the VALU transition of this pair, so their latencies overlap it.
// SPLIT (int8, the fixed-shape kernel copies, whose row pitch is a compile-time constant): the
// two halves' state dwords are addressed from two base registers, so each block's accesses
// take its row offset as an instruction offset instead of one merged access per block after a
// per-block base add. With a run-time pitch the merged form is the cheaper one.
template <int ELEM, int EPI, bool MASKED, bool SPLIT = false>
__device__ __forceinline__ void phase_b(const CatParams &p, uint8_t *Qt, uint8_t *At, LaneOff lo, int rb0, int count,
                                        int gr0, uint32_t cma, uint32_t cmb, const Bands &bd,
                                        const Codec &cd, const v16i &Ha, const v16i &Hb, const v16i &La,
                                        const v16i &Lb) {
    constexpr int CELL = ElemT<ELEM>::CELL;
    // Q and A are distinct tiles (int8 Moore decay reads its alive bits from Q)
    constexpr bool SEPARATE = epi_decays(EPI) && ELEM != ELEM_I8 && ELEM != ELEM_F16;
    const uint32_t PS = (uint32_t)p.PS, PA = (uint32_t)p.PA;
    v4i ca[4], cb[4];
    uint32_t sa[4], sb[4];
    const int cw = epi_windowed(EPI) ? -p.rc.cwin : 0;
    const v4i acc0 = {cw, cw, cw, cw};
    constexpr bool SPLIT8 = SPLIT && ELEM == ELEM_I8;   // int8: At == Qt and PA == PS
    const uint32_t qa0 = lo.q + (uint32_t)(16 * rb0) * PS;
    uint32_t qb0 = qa0 + 16;
    // an opaque second base: kept from being folded back into qa0 + 16 (and the pair merged)
    if constexpr (SPLIT8) asm volatile("" : "+v"(qb0));
    // counts and centre states of block M (slot M & 3)
#define CAT_ISSUE(M)                                                                               \
    {                                                                                              \
        ca[(M) & 3] = vproduct<ELEM, (M)>(Ha, La, bd, acc0);                                       \
        cb[(M) & 3] = vproduct<ELEM, (M)>(Hb, Lb, bd, acc0);                                       \
        if constexpr (SPLIT8) {                                                                    \
            sa[(M) & 3] = *reinterpret_cast<const uint32_t *>(Qt + qa0 + (uint32_t)(16 * (M)) * PS); \
            sb[(M) & 3] = *reinterpret_cast<const uint32_t *>(Qt + qb0 + (uint32_t)(16 * (M)) * PS); \
        } else if constexpr (epi_decays(EPI) || kIsI8<ELEM> || ELEM == ELEM_F16) {                 \
            const uint32_t qo = lo.q + (uint32_t)(16 * (rb0 + (M))) * PS;                          \
            sa[(M) & 3] = *reinterpret_cast<const uint32_t *>(Qt + qo);                            \
            sb[(M) & 3] = *reinterpret_cast<const uint32_t *>(Qt + qo + 16);                       \
        } else {   /* fp8 without decay: states decoded from its encoding */                      \
            const uint32_t ao = lo.a + (uint32_t)(16 * (rb0 + (M))) * PA;                          \
            sa[(M) & 3] = dec8(*reinterpret_cast<const uint32_t *>(At + ao), cd);                  \
            sb[(M) & 3] = dec8(*reinterpret_cast<const uint32_t *>(At + ao + 16), cd);             \
        }                                                                                          \
    }
    // transition and store of block M
#define CAT_FINISH(M)                                                                              \
    {                                                                                              \
        const int grow = gr0 + 16 * (M);                                                           \
        /* rows outside the grid: dead (forced to 0) under the dead halo, torus copies otherwise */ \
        const bool rowin = !MASKED || (unsigned)grow < (unsigned)p.H;                              \
        const uint32_t rowm = (rowin || p.periodic) ? 0xFFFFFFFFu : 0u;                            \
        uint32_t ala, alb;                                                                         \
        const uint32_t na = transition4<EPI>(ca[(M) & 3], sa[(M) & 3], rowm & cma, p.rc, &ala);    \
        const uint32_t nb = transition4<EPI>(cb[(M) & 3], sb[(M) & 3], rowm & cmb, p.rc, &alb);    \
        {                                                                                          \
            const uint32_t qo = lo.q + (uint32_t)(16 * (rb0 + (M))) * PS;                          \
            const uint32_t ao = lo.a + (uint32_t)(16 * (rb0 + (M))) * PA;                          \
            if constexpr (SPLIT8 && epi_decays(EPI)) {                                             \
                *reinterpret_cast<uint32_t *>(Qt + qa0 + (uint32_t)(16 * (M)) * PS) = na;           \
                *reinterpret_cast<uint32_t *>(Qt + qb0 + (uint32_t)(16 * (M)) * PS) = nb;           \
            } else if constexpr (epi_decays(EPI)) {                                                \
                *reinterpret_cast<uint32_t *>(Qt + qo) = na;                                       \
                *reinterpret_cast<uint32_t *>(Qt + qo + 16) = nb;                                  \
            }                                                                                      \
            if constexpr ((ELEM == ELEM_I8 || ELEM == ELEM_F16) && epi_decays(EPI)) {              \
                (void)ala;   /* int8 Moore and fp16 decay derive the alive bits from Q when read */ \
                (void)alb;                                                                         \
            } else if constexpr (SPLIT8) {   /* two-state: the state, At == Qt */                  \
                *reinterpret_cast<uint32_t *>(At + qa0 + (uint32_t)(16 * (M)) * PS) = ala;          \
                *reinterpret_cast<uint32_t *>(At + qb0 + (uint32_t)(16 * (M)) * PS) = alb;          \
            } else if constexpr (kIsI8<ELEM> || ELEM == ELEM_F16) {   /* two-state: the state */   \
                *reinterpret_cast<uint32_t *>(At + ao) = ala;                                      \
                *reinterpret_cast<uint32_t *>(At + ao + 16) = alb;                                 \
            } else {   /* fp8: its encoding of 1.0 */                                              \
                *reinterpret_cast<uint32_t *>(At + ao) = enc8(ala, cd);                            \
                *reinterpret_cast<uint32_t *>(At + ao + 16) = enc8(alb, cd);                       \
            }                                                                                      \
        }                                                                                          \
    }
    // pair P = blocks 2P, 2P + 1; block `count` (one past the item) may be issued: its windows
    // and centre row are inside the tile and nothing is stored for it
#define CAT_BPAIR(P, NEXT)                                                                         \
    if (2 * (P) < count) {                                                                         \
        if (NEXT && 2 * (P) + 2 < count) { CAT_ISSUE(2 * (P) + 2) CAT_ISSUE(2 * (P) + 3) }         \
        CAT_FINISH(2 * (P))                                                                        \
        if (2 * (P) + 1 < count) CAT_FINISH(2 * (P) + 1)                                           \
    }
    (void)CELL;
    (void)SEPARATE;
    if constexpr (ELEM == ELEM_F16) {
        CAT_ISSUE(0) CAT_ISSUE(1)
        CAT_BPAIR(0, 1) CAT_BPAIR(1, 1)
        CAT_BPAIR(2, 0)
    } else if constexpr (ELEM == ELEM_I8X) {   // at most CAT_MAXC_I8X = 6 blocks
        CAT_ISSUE(0) CAT_ISSUE(1)
        CAT_BPAIR(0, 1) CAT_BPAIR(1, 1)
        CAT_BPAIR(2, 0)
    } else if constexpr (ELEM == ELEM_I8W) {   // at most CAT_MAXC_I8W = 9 blocks
        CAT_ISSUE(0) CAT_ISSUE(1)
        CAT_BPAIR(0, 1) CAT_BPAIR(1, 1) CAT_BPAIR(2, 1) CAT_BPAIR(3, 1)
        CAT_BPAIR(4, 0)
    } else {
        CAT_ISSUE(0) CAT_ISSUE(1)
        CAT_BPAIR(0, 1) CAT_BPAIR(1, 1) CAT_BPAIR(2, 1) CAT_BPAIR(3, 1) CAT_BPAIR(4, 1) CAT_BPAIR(5, 1)
        CAT_BPAIR(6, 0)
    }
#undef CAT_BPAIR
#undef CAT_FINISH
#undef CAT_ISSUE
}

// T steps of one tile, in place in LDS; ends with a barrier after the last step's writes.
// FIX (the fixed-shape kernel copies): 1 = pitch, width and 32-cell margin compiled in (phase
// B's SPLIT accesses); 2 = the height too, and the last step (extent 0) runs as a copy of its
// own after the loop over the others (extent 16), so each copy's geometry is constant.
template <int ELEM, int EPI, bool MASKED, int FIX = 0>
__device__ __forceinline__ void cat_steps(const CatParams &p, uint8_t *Qt, uint8_t *At, int gi0, int gj0, int wave,
                                          int lane, const Bands &bd, const Codec &cd) {
    constexpr int CELL = ElemT<ELEM>::CELL;
    constexpr int MAXC = ElemT<ELEM>::MAXC;
    const int li = lane & 15, lg = lane >> 4;
    const uint32_t PS = (uint32_t)p.PS, PA = (uint32_t)p.PA;
    const int L = p.L;
    auto step = [&](const int t, const bool last) {
        const StepGeom g = step_geom<MAXC>(p, t, last);
        const int items = g.nstrips * g.nseg;
        int j0 = 0, rb0 = 0, count = 0;
        if (wave < items) {
            const int strip = g.nseg == 1 ? wave : wave % g.nstrips;
            const int seg = g.nseg == 1 ? 0 : wave / g.nstrips;
            const int mb_lo = seg * g.seglen;
            const int mb_hi = min(g.nrb, mb_lo + g.seglen);
            j0 = -g.E + 32 * strip;
            rb0 = -(g.E >> 4) + mb_lo;
            count = max(0, mb_hi - mb_lo);
        }
        v16i Ha, Hb;
        v16i La, Lb;   // cross only: the packed alive map
        if constexpr (!kIsI8<ELEM>) {
            // slots no block fills may enter a window with zero weight; keep them finite
            Ha = (v16i)0;
            Hb = (v16i)0;
        }
        // this lane's A chunk (row li of a block, from column j0 - 16 + 16 lg, or + 8 lg for the
        // K = 32 element types) and its first centre cell (row li, column j0 + 4 lg)
        const int chunk_col = (ELEM == ELEM_I8W) ? (L + j0 - 32 + 16 * lg)
                              : kIsI8<ELEM> ? (L + j0 - 16 + 16 * lg) : (L + j0 - 16 + 8 * lg);
        const uint32_t a_off = (uint32_t)((L + li) * (int)PA + chunk_col * CELL);
        // int8 wide: the K = 32 chunk, columns j0 + 32 + 8 lg .. + 7
        const uint32_t a_off2 = (uint32_t)((L + li) * (int)PA + (L + j0 + 32 + 8 * lg) * CELL);
        LaneOff lo;
        lo.q = (uint32_t)((L + li) * (int)PS + (L + j0 + 4 * lg));
        lo.a = (uint32_t)((L + li) * (int)PA + (L + j0 + 4 * lg) * CELL);
        if (count > 0)
            phase_a<ELEM, !((ELEM == ELEM_I8 || ELEM == ELEM_F16) && epi_decays(EPI)) ? 0
                                                                                  : (EPI == EPI_DECAY8 || EPI == EPI_DECAY8W) ? 2
                                                                                                                               : 1>(
                At, a_off, a_off2, PA, rb0, count,
                                                                                   bd, Ha, Hb, La, Lb);
        __syncthreads();   // every read of the old states precedes any in-place write
        if (count > 0) {
            const int gca = gj0 + j0 + 4 * lg;
            uint32_t cma = 0xFFFFFFFFu, cmb = 0xFFFFFFFFu;
            if constexpr (MASKED) {   // dead halo: cells right of the grid stay 0
                if (!p.periodic) {
                    cma = col_mask(gca, p.W);
                    cmb = col_mask(gca + 16, p.W);
                }
            }
            const int gr0 = gi0 + 16 * rb0 + li;
            phase_b<ELEM, EPI, MASKED, (FIX >= 1)>(p, Qt, At, lo, rb0, count, gr0, cma, cmb, bd, cd, Ha, Hb, La, Lb);
        }
        __syncthreads();   // new states complete before the next step (or the copy-out) reads them
    };
    if constexpr (FIX >= 2) {
        for (int t = 1; t < p.T; ++t) step(t, false);
        step(p.T, true);
    } else {
        for (int t = 1; t <= p.T; ++t) step(t, t == p.T);
    }
}

// One 16-byte global->LDS DMA per lane into the KiB of LDS at `chunk`: from the 64-bit address
// g, or (second form) from the grid base `base` (scalar) plus a 32-bit byte offset.
//
// The loads are issued from inline assembly: the compiler cannot see which LDS bytes an LDS-DMA
// writes, so for its own builtin it would make every later LDS access wait for all outstanding
// vector-memory operations. The caller waits (vmcnt(0) + barrier) before the buffer is read. m0
// (the DMA's LDS address) is a register the compiler reserves; no other code of these kernels
// uses it (checked in the generated ISA), so clobbering it here is safe and the corresponding
// warning is silenced for these statements only.
__device__ __forceinline__ void lds_dma16(uint8_t *chunk, const uint8_t *g) {
    const uint32_t lds_addr = (uint32_t)(uintptr_t)chunk;
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                 :
                 : "s"(__builtin_amdgcn_readfirstlane(lds_addr)), "v"(g)
                 : "memory", "m0");
#pragma clang diagnostic pop
}
__device__ __forceinline__ void lds_dma16(uint8_t *chunk, const uint8_t *base, uint32_t off) {
    const uint32_t lds_addr = (uint32_t)(uintptr_t)chunk;
    // the base is the same in every lane (a tile's grid); read through the first lane it sits in
    // scalar registers also where the compiler cannot prove that (a descriptor read per entry)
    // (the builtin returns int: each half goes back through uint32_t, so the low half is not
    // sign-extended into the high one)
    const uint64_t b = (uint64_t)(uintptr_t)base;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    const uint64_t sb = ((uint64_t)hi << 32) | (uint64_t)lo;
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, %2"
                 :
                 : "s"(__builtin_amdgcn_readfirstlane(lds_addr)), "v"(off), "s"(sb)
                 : "memory", "m0");
#pragma clang diagnostic pop
}

// Row and column of byte offset o of a buffer with rows of PS bytes: a reciprocal estimate,
// corrected by one either way (exact for the offsets of a tile buffer).
__device__ __forceinline__ void row_col(int o, int PS, float inv_ps, int *row, int *col) {
    int r = (int)((float)o * inv_ps);
    int c = o - r * PS;
    if (c < 0) { r -= 1; c += PS; }
    if (c >= PS) { r += 1; c -= PS; }
    *row = r;
    *col = c;
}

// Stream the (TH + 2L) x PS window of the tile at (gi0, gj0) into LDS at `buf` with direct
// global->LDS loads: wave w moves KiB chunks w, w + nwaves, ...; lane l of a chunk carries
// the 16 bytes at buffer offset 1024 c + 16 l. Cells outside the grid come from the zero page
// (dead halo) or from the opposite edge (torus); so do the bytes past the window's last row
// that the KiB rounding of the buffer adds. A lane's (row, column) is computed once; each
// later chunk of its wave lies nwaves KiB further on (dr rows and dc columns, one more row when
// the column passes PS). When the whole window lies inside the grid (most tiles), the lane
// advances a 32-bit offset from the grid base instead and tests no bounds.
__device__ __forceinline__ void issue_tile_load(const CatParams &p, int gi0, int gj0, uint8_t *buf, int wave,
                                                int nwaves, int lane, float inv_ps) {
    const int rows = p.TH + 2 * p.L;
    const int PS = p.PS;
    const int nchunks = p.lds_tile >> 10;
    const int gr0 = gi0 - p.L, gc0 = gj0 - p.L;
    int lr, lc, dr, dc;
    row_col((wave << 10) + (lane << 4), PS, inv_ps, &lr, &lc);
    row_col(nwaves << 10, PS, inv_ps, &dr, &dc);
    const bool inside = !p.periodic && gr0 >= 0 && gc0 >= 0 && gr0 + rows <= p.H && gc0 + PS <= p.pitch;
    if (inside) {
        uint32_t off = (uint32_t)((gr0 + lr) * p.pitch + gc0 + lc);
        const uint32_t adv = (uint32_t)(dr * p.pitch + dc);
        const uint32_t wrap = (uint32_t)(p.pitch - PS);
        const int window = rows * PS;   // bytes of the window; the last chunk may run past it
        for (int c = wave; c < nchunks; c += nwaves) {
            uint8_t *chunk = buf + (c << 10);
            if (c == nchunks - 1)
                lds_dma16(chunk, ((c << 10) + (lane << 4) < window) ? p.src + off : p.zero);
            else
                lds_dma16(chunk, p.src, off);
            off += adv;
            lc += dc;
            if (lc >= PS) {
                lc -= PS;
                off += wrap;
            }
        }
        return;
    }
    for (int c = wave; c < nchunks; c += nwaves) {
        const int gr = gr0 + lr;
        const int gc = gc0 + lc;
        const uint8_t *g = p.zero;
        if (p.periodic) {
            // torus: wrap both coordinates (W is a multiple of 16, so a 16-byte vector at a
            // 16-aligned column wraps as a whole)
            if (lr < rows) {
                int wr = gr % p.H, wc = gc % p.W;
                wr += (wr < 0) ? p.H : 0;
                wc += (wc < 0) ? p.W : 0;
                g = p.src + (size_t)wr * p.pitch + wc;
            }
        } else if (lr < rows && (unsigned)gr < (unsigned)p.H && (unsigned)gc < (unsigned)p.pitch) {
            g = p.src + (size_t)gr * p.pitch + gc;
        }
        lds_dma16(buf + (c << 10), g);
        lr += dr;
        lc += dc;
        if (lc >= PS) {
            lc -= PS;
            lr += 1;
        }
    }
}

// Band operands of a launch, per lane (the fp8 table holds 0/1 bytes and is encoded here).
template <int ELEM>
__device__ __forceinline__ Bands load_bands(const CatParams &p, int lane, const Codec &cd) {
    Bands bd;
    const v4i *bt = reinterpret_cast<const v4i *>(p.bands);
#pragma unroll
    for (int k = 0; k < ElemT<ELEM>::NOPS; ++k) {
        bd.op[k] = bt[k * 64 + lane];
        if constexpr (ELEM == ELEM_F8) {
            bd.op[k][0] = (int32_t)enc8((uint32_t)bd.op[k][0], cd);
            bd.op[k][1] = (int32_t)enc8((uint32_t)bd.op[k][1], cd);
        }
    }
    return bd;
}

// Copy the tile's final states from LDS to the output grid with 16-byte stores: the rows inside
// the grid and the columns below store_w (a dead halo's padding columns, which the steps kept
// at 0, included). Consecutive threads take consecutive vectors of a row, so a wave writes whole
// row segments instead of the 16-byte pieces of 16 rows a phase-B lane holds. fp8 two-state
// tiles hold the fp8 encoding of the alive bit in place of the state and are decoded here.
template <int ELEM, int EPI, bool NONTEMPORAL>
__device__ __forceinline__ void store_tile(const CatParams &p, const uint8_t *Qt, int gi0, int gj0, int tid,
                                           int nthreads, const Codec &cd) {
    const int vpr = p.TW >> 4;                                   // 16-byte vectors per tile row
    const int rows = min(p.TH, p.H - gi0);
    const int vcols = min(p.TW, p.store_w - gj0) >> 4;           // store_w is a multiple of 16
    const int n = rows * vpr;
    // this thread's first vector and the per-iteration advance, as (row, vector) pairs
    const int di = nthreads / vpr, dc = nthreads - di * vpr;
    int i = tid / vpr;
    int c = tid - i * vpr;
    const uint8_t *src = Qt + p.L * p.PS + p.L;
    for (int v = tid; v < n; v += nthreads) {
        if (c < vcols) {
            v4i x = *reinterpret_cast<const v4i *>(src + i * p.PS + 16 * c);
            if constexpr (ELEM == ELEM_F8 && !epi_decays(EPI)) {
#pragma unroll
                for (int k = 0; k < 4; ++k) x[k] = (int32_t)dec8((uint32_t)x[k], cd);
            }
            // explicit global address space: a global store, not a flat one, which would also count
            // against the LDS wait counter
            __attribute__((address_space(1))) v4i *g =
                (__attribute__((address_space(1))) v4i *)(p.dst + (size_t)(gi0 + i) * p.pitch + gj0 + 16 * c);
            if constexpr (NONTEMPORAL)
                __builtin_nontemporal_store(x, g);
            else
                *g = x;
        }
        i += di;
        c += dc;
        if (c >= vpr) {
            c -= vpr;
            i += 1;
        }
    }
}

// The window of the tile at (gi0, gj0) is in LDS at Qt (visible to every wave): derive the
// alive map in the element encoding at At, run T steps in place, then copy the tile to the
// output grid. Ends without a barrier.
template <int ELEM, int EPI, int FIX = 0>
__device__ __forceinline__ void tile_steps(const CatParams &p, int gi0, int gj0, uint8_t *Qt, uint8_t *At, int tid,
                                           int lane, int wave, int nwaves, const Bands &bd, const Codec &cd) {
    // alive map from the loaded states, where a kernel keeps one: fp8 (its encoding of 1.0, in
    // place) and the int8 wide and cross elements with decay (a second tile). int8 Moore and
    // fp16 read the states and derive the alive bits in registers.
    if constexpr (ELEM == ELEM_F8 || ((ELEM == ELEM_I8W || ELEM == ELEM_I8X) && epi_decays(EPI))) {
        const int W2 = p.TW + 2 * p.L;          // window columns (the PS - W2 pad is never read)
        const int vpr = W2 >> 4;
        const int nvec = (p.TH + 2 * p.L) * vpr;
        for (int v = tid; v < nvec; v += 64 * nwaves) {
            const int row = v / vpr;
            const int col = (v - row * vpr) << 4;
            const uint4 q = *reinterpret_cast<const uint4 *>(Qt + row * p.PS + col);
            uint4 al = q;
            if constexpr (epi_decays(EPI))
                al = make_uint4(alive_of(q.x), alive_of(q.y), alive_of(q.z), alive_of(q.w));
            if constexpr (kIsI8<ELEM>) {
                *reinterpret_cast<uint4 *>(At + row * p.PA + col) = al;
            } else {
                *reinterpret_cast<uint4 *>(At + row * p.PA + col) =
                    make_uint4(enc8(al.x, cd), enc8(al.y, cd), enc8(al.z, cd), enc8(al.w, cd));
            }
        }
        __syncthreads();
    }
    // no masking needed when every cell this tile computes lies inside the grid
    const int E1 = (p.r * (p.T - 1) + 15) & ~15;
    const bool interior = gi0 - E1 >= 0 && gi0 + p.TH + E1 <= p.H && gj0 - E1 >= 0 && gj0 + p.TW + E1 <= p.W;
    if (interior)
        cat_steps<ELEM, EPI, false, FIX>(p, Qt, At, gi0, gj0, wave, lane, bd, cd);
    else
        cat_steps<ELEM, EPI, true, FIX>(p, Qt, At, gi0, gj0, wave, lane, bd, cd);
    // With several steps per launch the copy-out carries the non-temporal hint (+2 % at Bosco
    // 4096², T = 4); at one step per launch, where the kernel streams the grid and the next launch
    // re-reads it at once, plain stores are 13 % faster (16384², 2.04 vs 1.78 T cell-updates/s).
    if (p.T > 1)
        store_tile<ELEM, EPI, true>(p, Qt, gi0, gj0, tid, 64 * nwaves, cd);
    else
        store_tile<ELEM, EPI, false>(p, Qt, gi0, gj0, tid, 64 * nwaves, cd);
}

// Work a caller overlaps with a tile's window load: issue() runs after the loads are issued,
// land() after they (and whatever issue() started) completed, before the barrier that opens
// the tile. The default does nothing.
struct NoSideLoad {
    __device__ __forceinline__ void issue(int) {}
    __device__ __forceinline__ void land(int) {}
};

// One tile: load the window with direct LDS loads, then the alive map and T steps in place.
// Ends without a barrier: a caller that reuses the LDS for another tile synchronizes first.
template <int ELEM, int EPI, class Side = NoSideLoad, int FIX = 0>
__device__ __forceinline__ void cat_tile(const CatParams &p, int tile, uint8_t *lds, int tid, int lane, int wave,
                                         int nwaves, const Codec &cd, Side &&side = Side()) {
    const int gi0 = (tile / p.ntx) * p.TH;
    const int gj0 = (tile % p.ntx) * p.TW;
    uint8_t *Qt = lds;                 // loaded window: states, one byte per cell
    uint8_t *At = lds + p.a_tile;      // alive map in the element encoding (== Qt when shared)
    issue_tile_load(p, gi0, gj0, Qt, wave, nwaves, lane, __builtin_amdgcn_rcpf((float)p.PS));
    const Bands bd = load_bands<ELEM>(p, lane, cd);
    side.issue(tid);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    side.land(tid);
    __syncthreads();
    tile_steps<ELEM, EPI, FIX>(p, gi0, gj0, Qt, At, tid, lane, wave, nwaves, bd, cd);
}

}  // namespace ltl
