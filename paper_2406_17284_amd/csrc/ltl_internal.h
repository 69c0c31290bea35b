// Internal interface between the host library (ltl_api.cpp) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ltl {

// Epilogue flavour, chosen on the host from the rule:
//  EPI_BYTE  two states, every count fits in 7 bits ((2r+1)^2 <= 126): 4 cells per dword SWAR
//  EPI_HALF  two states, counts up to 1089: 2 cells per dword SWAR on 16-bit lanes
//  EPI_DECAY C >= 3 states: per-cell transition with decay
//  EPI_WIN   two states, counts above 126, int8 element, every finite range bound within a
//            window c+1..c+126: the vertical product starts from -c, the counts n - c are
//            clamped to 127 (all values outside the window land there, outside every range)
//            and the EPI_BYTE transition runs on them
//  EPI_DECAY8 C in 3..8 states, int8 element: every state fits in 3 bits, so the alive bit and
//            the next state come from per-byte tables indexed by the state (one byte permute
//            each) instead of the SWAR arithmetic of EPI_DECAY
//  EPI_WIN8  as EPI_WIN with a window c+1..c+254: the counts n - c are clamped to 255 and the
//            range tests run on full bytes with v_lerp_u8 (a per-byte (a + b) >> 1 whose top
//            bit is the carry of a + b), so the 8-bit lanes need no spare top bit
//  EPI_DECAY8W EPI_DECAY8 with the range test of EPI_WIN8 (both ranges inside a 254 window)
enum Epi { EPI_BYTE = 0, EPI_HALF = 1, EPI_DECAY = 2, EPI_WIN = 3, EPI_DECAY8 = 4, EPI_WIN8 = 5, EPI_DECAY8W = 6 };
__host__ __device__ constexpr bool epi_decays(int epi) {
    return epi == EPI_DECAY || epi == EPI_DECAY8 || epi == EPI_DECAY8W;
}
// epilogues whose vertical product starts from -c (the window offset)
__host__ __device__ constexpr bool epi_windowed(int epi) {
    return epi == EPI_WIN || epi == EPI_WIN8 || epi == EPI_DECAY8W;
}

// Element type of the band-product operands. ELEM_I8W is int8 for radii 17..32: every
// 16-column half needs 16 + 2r <= 80 columns (a K = 64 and a K = 32 product) and every
// output block the H blocks two above to two below it (a 4-block and a 2-block window).
// ELEM_I8X is int8 for the cross neighbourhood (rule code N_N, r <= 16): besides H it packs
// the alive map itself into the H register layout, for the vertical arm of the cross.
enum Elem { ELEM_I8 = 0, ELEM_F16 = 1, ELEM_F8 = 2, ELEM_I8W = 3, ELEM_I8X = 4 };
inline bool elem_is_i8(int elem) { return elem == ELEM_I8 || elem == ELEM_I8W || elem == ELEM_I8X; }

// Rule constants prepared on the host (thresholds on the box count n that includes
// the centre: for an alive centre with M = 0 the survival range is shifted by one).
struct RuleConsts {
    int32_t C;             // number of states (2 for C in {0, 2})
    int32_t M;             // 1: centre counted
    int32_t s1, s2, b1, b2;  // raw rule thresholds (per-cell decay epilogue and direct kernel)
    // SWAR constants of the two-state epilogues, per lane of 8 bits (BYTE) or 16 bits (HALF):
    // with sm = 0x80 - s per lane (0x80 dead, 0x7F alive), the per-lane offsets
    //   klo = Klo ^ (sm & Dlo)   equal 0x80 - lo(s)
    //   khi = Khi ^ (sm & Dhi)   equal 0x80 + hi(s)
    // (0x8000-based for HALF), lo/hi being the birth range for s = 0 and the survival range
    // for s = 1.
    uint32_t Klo, Dlo, Khi, Dhi;
    // BYTE lookup tables of the same offsets, indexed by the centre state (0 or 1) with one
    // byte permute per dword of four cells: byte 0 holds the dead-centre offset, byte 1 the
    // alive-centre offset (Tlo: 0x80 - lo(s), Thi: 0x80 + hi(s); EPI_WIN8 and EPI_DECAY8W:
    // Tlo: 256 - lo(s), Thi: hi(s) + 1, bounds relative to the window).
    uint32_t Tlo, Thi;
    int32_t cwin;          // EPI_WIN, EPI_WIN8, EPI_DECAY8W: window offset c (the vertical product
                           // starts from -c)
    uint32_t Crep;         // EPI_DECAY: C in every byte (a state reaching C wraps to 0)
    // EPI_DECAY8: next state by state byte k = 0..7 when the range test fails (N0) or holds (N1),
    // as the 8-byte tables {N0hi:N0lo}, {N1hi:N1lo} of a byte permute
    uint32_t N0lo, N0hi, N1lo, N1hi;
};

struct CatParams {
    const uint8_t *src;
    uint8_t *dst;
    const int32_t *bands;    // band operands of this radius and element type (band_table layout)
    const uint8_t *zero;     // >= 16 zero bytes in device memory (source of out-of-grid loads)
    int32_t H, W, pitch;     // grid rows, columns, row pitch (bytes)
    int32_t r;               // radius 1..16
    int32_t T;               // steps in this launch
    int32_t TH, TW;          // output tile (multiples of 16 / 32)
    int32_t L;               // LDS margin around the output tile: roundup16(r (T-1)) + 16
    int32_t PS;              // state tile pitch (bytes) = TW + 2L + 16, rows stored densely
    int32_t PA;              // alive tile pitch (bytes) in the element encoding
    int32_t lds_rows;        // TH + 2L
    int32_t lds_tile;        // bytes of the state tile: lds_rows * PS rounded up to 1 KiB
    int32_t a_tile;          // LDS offset of the alive tile (0: the state tile itself)
    int32_t lds_total;       // dynamic LDS bytes of the launch
    int32_t ntx, nty;        // tiles across / down the grid
    int32_t periodic;        // 1: the grid is a torus (W % 16 == 0); 0: dead ghost halo
    int32_t store_w;         // columns the copy-out stores: W (torus) or pitch (dead halo, zero padding)
    RuleConsts rc;
};

// Band operands, host-built per (element type, radius): LTL_BAND_OPS operands x 64 lanes x 4
// dwords. Lane l = 16 g + n (n = output index, g = lane group); the K slots a lane carries are
// numbered as the MFMA A operand numbers them (int8 16x16x64: 16 bytes, K = 16 g + 4 d + e;
// fp8 16x16x32: 8 bytes, K = 8 g + 4 d + e; fp16 16x16x32: 8 halves, K = 8 g + j).
//  int8 : 0, 1  MFMA #1, halves 0/1 of a 32-column strip whose 64-column window starts 16
//               columns left of it: weight 1 iff |k - 16 - 16 h - n| <= r
//         2, 3  MFMA #2, 4-block window (slot d = dword d) starting at block m-1 (2) or m-2 (3)
//  fp8  : 0..3  MFMA #1 (half h, chunk c) = op 2h + c, chunk c covers window columns 32c..32c+31
//         4..7  MFMA #2 on 2-block windows: (m-1, m), (m+1, m+2), (m-2, m-1), (m, m+1)
//  fp16 : 0..3  MFMA #1 as fp8; 4, 5 MFMA #2 on the 2-block windows (m-1, m), (m+1, m+2)
//  int8 wide (r 17..32): 0, 2  MFMA #1 halves 0/1, K = 64 chunk starting 32 columns left of
//               the strip (K = 16 g + 4 d + e); 1, 3  the K = 32 chunk 32 columns right of the
//               strip start (8 bytes, K = 8 g + j)
//         4, 5  MFMA #2 for an even block offset: 4-block window m-2..m+1, pair m+2, m+3
//         6, 7  odd offset: 4-block window m-3..m, pair m+1, m+2
//  int8 cross (N_N): 0, 1  MFMA #1 halves as int8 (H = horizontal arm, centre included)
//         2, 3  MFMA #1 identity for halves 0/1: weight 1 iff k - 16 - 16 h == n (packs the
//               alive map itself into the H layout)
//         4, 5  MFMA #2 on the alive map, windows from block m-1 / m-2: vertical arm without
//               the centre (1 iff 0 < |row - n| <= r)
//         6, 7  MFMA #2 on H, windows from block m-1 / m-2: identity (1 iff row == n)
// MFMA #2 rows: block at distance delta from the output block, row 4 g + e of it, weight 1 iff
// |16 delta + 4 g + e - n| <= r. int8 and fp8 tables hold 0/1 bytes (fp8 is encoded on the
// device with the hardware's 1.0); fp16 holds 0x3C00 halves.
#define LTL_BAND_OPS 8
#define LTL_BAND_TABLE_INTS (LTL_BAND_OPS * 64 * 4)   // per (element type, radius)

__host__ __device__ inline bool band_hit(int dist, int r) { return dist >= -r && dist <= r; }

// Dword d (0..3) of lane `lane` of band operand `op` for an element type and radius, in the
// layout described above (host tables and the device-side fill of the allocation-free entry
// point both evaluate it). Bytes hold 0/1 (int8, fp8), halves 0 / 0x3C00 (fp16).
__host__ __device__ inline uint32_t band_dword(int elem, int r, int op, int lane, int d) {
    const int n = lane & 15, g = lane >> 4;
    uint32_t v = 0;
    if (elem == ELEM_F16) {
        for (int q = 0; q < 2; ++q) {   // halves j = 2d, 2d + 1 of the lane's 8 K slots
            const int j = 2 * d + q;
            bool on = false;
            if (op < 4) on = band_hit(32 * (op & 1) + 8 * g + j - 16 - 16 * (op >> 1) - n, r);
            else if (op < 6) on = band_hit(16 * ((op == 4 ? -1 : 1) + j / 4) + 4 * g + (j % 4) - n, r);
            v |= on ? (0x3C00u << (16 * q)) : 0u;
        }
        return v;
    }
    for (int e = 0; e < 4; ++e) {
        const int k = 16 * g + 4 * d + e;   // K slot of a 16-byte int8 operand
        const int j = 4 * d + e;            // K slot of an 8-byte operand (d < 2)
        bool on = false;
        if (elem == ELEM_I8X) {
            const int row1 = 16 * (d - 1) + 4 * g + e - n, row2 = 16 * (d - 2) + 4 * g + e - n;
            switch (op) {
                case 0: on = band_hit(k - 16 - n, r); break;
                case 1: on = band_hit(k - 32 - n, r); break;
                case 2: on = (k - 16 == n); break;
                case 3: on = (k - 32 == n); break;
                case 4: on = row1 != 0 && band_hit(row1, r); break;
                case 5: on = row2 != 0 && band_hit(row2, r); break;
                case 6: on = (row1 == 0); break;
                default: on = (row2 == 0); break;
            }
        } else if (elem == ELEM_I8W) {
            switch (op) {
                case 0: case 2: on = band_hit(k - 32 - 16 * (op >> 1) - n, r); break;
                case 1: case 3: on = d < 2 && band_hit(32 + 8 * g + j - 16 * (op >> 1) - n, r); break;
                case 4: on = band_hit(16 * (d - 2) + 4 * g + e - n, r); break;
                case 6: on = band_hit(16 * (d - 3) + 4 * g + e - n, r); break;
                case 5: on = d < 2 && band_hit(16 * (2 + d) + 4 * g + e - n, r); break;
                default: on = d < 2 && band_hit(16 * (1 + d) + 4 * g + e - n, r); break;
            }
        } else if (elem == ELEM_I8) {
            switch (op) {
                case 0: on = band_hit(k - 16 - n, r); break;
                case 1: on = band_hit(k - 32 - n, r); break;
                // window slot d of a window starting at block m-1 (op 2) or m-2 (op 3)
                case 2: on = band_hit(16 * (d - 1) + 4 * g + e - n, r); break;
                case 3: on = band_hit(16 * (d - 2) + 4 * g + e - n, r); break;
                default: break;
            }
        } else {   // ELEM_F8: 8-byte operands (dwords 0, 1)
            if (d < 2) {
                if (op < 4) {
                    on = band_hit(32 * (op & 1) + 8 * g + j - 16 - 16 * (op >> 1) - n, r);
                } else {
                    const int start = op == 4 ? -1 : op == 5 ? 1 : op == 6 ? -2 : 0;   // first block of the window
                    on = band_hit(16 * (start + d) + 4 * g + e - n, r);
                }
            }
        }
        v |= on ? (1u << (8 * e)) : 0u;
    }
    return v;
}

inline void band_table(int elem, int r, int32_t *out) {
    for (int op = 0; op < LTL_BAND_OPS; ++op)
        for (int lane = 0; lane < 64; ++lane)
            for (int d = 0; d < 4; ++d) out[(op * 64 + lane) * 4 + d] = (int32_t)band_dword(elem, r, op, lane, d);
}

// Direct-stencil comparison kernel: 128 x 256 output tiles, 256 threads (64 four-cell column
// groups x 4 rows at a time); the LDS window holds the alive bytes of the tile plus r rows above
// and below and roundup16(r) columns left and right (16-byte aligned vector loads).
constexpr int kDirectTH = 128;
constexpr int kDirectTW = 256;
constexpr int kDirectThreads = 256;
inline int direct_lds_pitch(int r) { return kDirectTW + 2 * ((r + 15) & ~15); }
inline size_t direct_lds_bytes(int r) { return (size_t)(kDirectTH + 2 * r) * direct_lds_pitch(r); }

struct DirectParams {
    const uint8_t *src;
    uint8_t *dst;
    int32_t H, W, pitch;
    int32_t r;
    int32_t TH, TW;       // output tile of the direct kernel (kDirectTH x kDirectTW)
    int32_t LP;           // LDS row pitch (direct_lds_pitch(r))
    int32_t periodic;     // 1: the grid is a torus; 0: dead ghost halo
    int32_t cross;        // 1: cross neighbourhood (N_N); 0: Moore box
    RuleConsts rc;
};

// Per-kernel geometry helpers shared by the host planner.
inline int roundup(int x, int m) { return (x + m - 1) / m * m; }

// LDS margin around the output tile: the growth of the T-step dependency cone plus the H rows
// and columns one step reads beyond its output (one 16-row block / 16 columns; int8 wide:
// 32 columns and three 16-row blocks below, two above).
inline int cat_margin(int elem, int r, int T) { return roundup(r * (T - 1), 16) + (elem == ELEM_I8W ? 48 : 16); }

// Longest run of 16-row output blocks one wave handles per step, per element type (bounded by
// the 16-register tuple that holds an item's H blocks).
#define CAT_MAXC_I8 14
#define CAT_MAXC_F8 14
#define CAT_MAXC_F16 5
#define CAT_MAXC_I8W 9    // the pair window of the last block (one past included) ends at element 15
#define CAT_MAXC_I8X 6
inline int cat_maxc(int elem) {
    return elem == ELEM_F16 ? CAT_MAXC_F16 : elem == ELEM_F8 ? CAT_MAXC_F8 : elem == ELEM_I8W ? CAT_MAXC_I8W
         : elem == ELEM_I8X ? CAT_MAXC_I8X : CAT_MAXC_I8;
}
inline int cat_cell_bytes(int elem) { (void)elem; return 1; }   // every element reads state bytes

// Whether a launch shape can run: in every step of a T-step launch the strips x segments
// must not outnumber the waves (each wave keeps one item's H blocks in registers across the
// barrier that separates the reads of the old states from the in-place writes).
inline bool cat_shape_fits(int elem, int r, int T, int TH, int TW, int waves) {
    const int maxc = cat_maxc(elem);
    for (int t = 1; t <= T; ++t) {
        int E = roundup(r * (T - t), 16);
        int nstrips = (TW + 2 * E) / 32;
        int nrb = (TH + 2 * E) / 16;
        int nseg = (nrb + maxc - 1) / maxc;
        if (nstrips * nseg > waves) return false;
    }
    return true;
}

// LDS geometry of a launch: the state tile holds the loaded window, TW + 2L columns (a
// multiple of 32) plus 16 more bytes per row, so its pitch is = 16 (mod 32) and the 16 rows of
// a 16-byte-per-lane operand read fall into distinct bank groups; rows are dense so 1 KiB of
// consecutive LDS maps to consecutive window bytes (one direct global->LDS load per wave).
// `pad` (a tuning knob, multiple of 16 bytes) widens every row further, which moves the bank
// each row starts in. The alive tile is the state tile itself, except for decay rules on fp8
// and on the wide and cross int8 elements, which keep a second tile in the element encoding.
inline void cat_lds_layout(int elem, int epi, int TH, int TW, int L, int pad, int *PS, int *PA, int *lds_tile,
                           int *a_tile, int *lds_total) {
    const int rows = TH + 2 * L;
    *PS = TW + 2 * L + 16 + pad;
    *lds_tile = roundup(rows * *PS, 1024);
    // int8 Moore and fp16 derive the alive bits from the states as they read them (no second tile)
    const bool separate = epi_decays(epi) && elem != ELEM_I8 && elem != ELEM_F16;
    *PA = cat_cell_bytes(elem) * (TW + 2 * L) + 16 + pad;
    *a_tile = separate ? *lds_tile : 0;
    *lds_total = *lds_tile + (separate ? roundup(rows * *PA, 1024) : 0);
}

// Batched simulation: one launch advances every instance by T steps. The instances' grids sit
// at their own offsets of two arenas; the work list holds one entry per (instance, tile),
// sorted by decreasing estimated cost, and the launch has one workgroup per entry.
struct BatchInst {
    CatParams p;           // launch parameters of the instance (src/dst of the launch's parity)
};

struct BatchItem {
    int32_t inst, tile;
    int32_t epi;           // Epi of the instance's rule
    int32_t pad;
};

struct BatchParams {
    const BatchInst *inst;     // per instance, for the arena this launch reads
    const BatchItem *items;    // workgroup k takes items[k] (and, persistent, the entries it draws)
    uint32_t *counters;        // persistent form: 8 next-entry counters (one per XCD), then the
                               // finished-workgroup counter; all zero between launches
    int32_t nitems;
    int32_t pad;
};

// Direct-stencil comparison method over the same work-list idea (one workgroup per entry).
struct DirectBatchInst {
    DirectParams p;        // src/dst of the launch's parity
    int32_t ntx;           // direct tiles across the grid
    int32_t pad[3];
};

struct DirectBatchParams {
    const DirectBatchInst *inst;   // per instance, for the arena this launch reads
    const BatchItem *items;
    int32_t nitems;
    int32_t pad;
};

// Launchers (return the HIP status of the launch).
hipError_t launch_direct(const DirectParams &p, hipStream_t s);
hipError_t launch_validate(const uint8_t *src, int H, int W, size_t pitch, int states,
                           uint32_t *flag, hipStream_t s);
// Band table of (elem, r) followed by zero_bytes zero bytes, written by a kernel at dst.
hipError_t launch_fill_constants(uint8_t *dst, int elem, int r, size_t zero_bytes, hipStream_t s);
// a = init (H x W, init_pitch) with zero columns up to pitch; b = 0 (both H x pitch).
hipError_t launch_prepare_grids(uint8_t *a, uint8_t *b, const uint8_t *init, size_t init_pitch, int H, int W,
                                int pitch, hipStream_t s);

// Dataflow form of the single-grid CAT step (tuning.persistent = 2): the arguments of one
// launch besides CatParams (whose src/dst the kernel sets per round).
struct FlowParams {
    uint8_t *buf[2];       // the ping-pong buffers: round k reads buf[(first + k) & 1], writes the other
    uint32_t *flags;       // per tile: counter of its last finished round (epoch-based, never reset)
    uint32_t *err;         // number of bounded waits that ran out (never reset; the host compares)
    uint32_t epoch;        // counter value before the launch's first round
    int32_t first;         // index of the buffer holding the input
    int32_t rounds;        // rounds of T = CatParams.T steps, the last one of last_T steps
    int32_t last_T;
    int32_t spin_limit;    // polls per wait before it counts as timed out
    int32_t pad;
};
// Tiles the dataflow form can track (flag words of a handle: this many plus the timeout counter).
constexpr int kFlowMaxTiles = 4096;
hipError_t launch_cat_flow(const CatParams &p, const FlowParams &f, int elem, int epi, int waves, hipStream_t s);
// Resident workgroups of the dataflow kernel per compute unit for this shape (0 if it cannot run).
int cat_flow_occupancy(const CatParams &p, int elem, int epi, int waves);

// Kernel symbol and launch shape, for building graph nodes.
struct KernelLaunch {
    const void *func;
    dim3 grid, block;
    size_t lds;
};
// persistent = 1: the persistent double-buffered form (one workgroup per CU slot walking tiles).
KernelLaunch cat_launch_shape(const CatParams &p, int elem, int epi, int waves, int persistent);
// Resident workgroups of the CAT kernel per compute unit for this shape (0 if it cannot run).
int cat_occupancy(const CatParams &p, int elem, int epi, int waves, int persistent);
KernelLaunch direct_launch_shape(const DirectParams &p);
size_t cat_lds_bytes(const CatParams &p, int elem, int epi, int persistent);
// Batched launches. cat_batch_func: the batch kernel of an element type, launched with
// workgroups of 64 * waves threads and the batch's largest dynamic LDS: one workgroup per
// work-list entry, or (persistent = 1) resident workgroups that draw entries from a counter.
const void *cat_batch_func(int elem, int persistent);
int cat_batch_occupancy(int elem, int waves, size_t lds, int persistent);
const void *direct_batch_func();
int direct_tile_rows();
int direct_tile_cols();
int direct_threads();

}  // namespace ltl
