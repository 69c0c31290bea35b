// Internal interface between the host library (ltl_api.cpp) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ltl {

// Epilogue flavour, chosen on the host from the rule:
//  EPI_BYTE  two states, every count fits in 7 bits ((2r+1)^2 <= 126): 4 cells per dword SWAR
//  EPI_HALF  two states, counts up to 1089: 2 cells per dword SWAR on 16-bit lanes
//  EPI_DECAY C >= 3 states: per-cell transition with decay
enum Epi { EPI_BYTE = 0, EPI_HALF = 1, EPI_DECAY = 2 };

// Element type of the band-product operands.
enum Elem { ELEM_I8 = 0, ELEM_F16 = 1, ELEM_F8 = 2 };

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
};

struct CatParams {
    const uint8_t *src;
    uint8_t *dst;
    const int32_t *bands;    // band operands for radius r: [4][64 lanes][4 dwords] (band_table layout)
    const uint8_t *zero;     // >= 16 zero bytes in device memory (source of out-of-grid loads)
    int32_t H, W, pitch;     // grid rows, columns, row pitch (bytes)
    int32_t r;               // radius 1..16
    int32_t T;               // steps in this launch
    int32_t TH, TW;          // output tile (multiples of 16 / 32)
    int32_t L;               // LDS margin around the output tile: roundup16(r (T-1)) + 16
    int32_t PS;              // LDS row pitch = TW + 2L + 16 (rows stored densely)
    int32_t lds_rows;        // TH + 2L
    int32_t lds_tile;        // bytes of one LDS tile buffer: lds_rows * PS rounded up to 1 KiB
    int32_t ntx, nty;        // tiles across / down the grid
    RuleConsts rc;
};

// Band operands (one v4i per lane, 16 bytes, K slot 16 g + 4 d + e = byte e of dword d of lane
// group g = lane / 16; n = lane % 16 is the output index):
//  0, 1: MFMA #1 for the two 16-column halves of a 32-column strip whose 64-column window
//        starts 16 columns left of the strip: weight 1 iff |k - 16 - 16 h - n| <= r;
//  2, 3: MFMA #2, dword d holding the H block at distance ((d - p) & 3) - 1 (in 16-row
//        blocks) from the output block, p = 0, 1: weight 1 iff |16 delta + 4 g + e - n| <= r.
#define LTL_BAND_OPERANDS 4
#define LTL_BAND_TABLE_INTS (LTL_BAND_OPERANDS * 64 * 4)   // per radius
__host__ __device__ inline int32_t band_dword(int r, int which, int lane, int d) {
    int n = lane & 15, g = lane >> 4;
    uint32_t w = 0;
    for (int e = 0; e < 4; ++e) {
        int dist;
        if (which < 2) {
            dist = 16 * g + 4 * d + e - 16 - 16 * which - n;
        } else {
            int delta = ((d - (which - 2)) & 3) - 1;
            dist = 16 * delta + 4 * g + e - n;
        }
        w |= (uint32_t)((dist >= -r && dist <= r) ? 1 : 0) << (8 * e);
    }
    return (int32_t)w;
}

struct DirectParams {
    const uint8_t *src;
    uint8_t *dst;
    int32_t H, W, pitch;
    int32_t r;
    int32_t TH, TW;       // output tile of the direct kernel
    int32_t LP;           // LDS row pitch
    RuleConsts rc;
};

// Per-kernel geometry helpers shared by the host planner.
inline int roundup(int x, int m) { return (x + m - 1) / m * m; }

inline int cat_margin(int r, int T) { return roundup(r * (T - 1), 16) + 16; }

inline int cat_lds_pitch(int TW, int L, int elem_bytes) {
    // bytes per LDS row: the loaded window is TW + 2L columns (a multiple of 32) plus 16 more,
    // so the pitch is = 16 (mod 32) and the 16 rows of a 16-byte-per-lane operand read fall
    // into distinct bank groups; rows are stored densely so 1 KiB of consecutive LDS maps to
    // consecutive window bytes (one direct global->LDS load per wave)
    return (TW + 2 * L) * elem_bytes + 16;
}

// LDS tile buffers of a workgroup: the tile stepped in place, plus the alive map for decay
// rules (the loaded tile then holds states).
inline int cat_tiles_in_lds(int T, int epi) {
    (void)T;
    return (epi == EPI_DECAY) ? 2 : 1;
}

// Longest 16-row run of output blocks one wave handles in one step.
#define CAT_MAXC 14

// Whether a launch shape can run: in every step of a T-step launch the strips x segments
// must not outnumber the waves (each wave keeps one item's H blocks in registers across the
// barrier that separates the reads of the old states from the in-place writes).
inline bool cat_shape_fits(int r, int T, int TH, int TW, int waves) {
    for (int t = 1; t <= T; ++t) {
        int E = roundup(r * (T - t), 16);
        int nstrips = (TW + 2 * E) / 32;
        int nrb = (TH + 2 * E) / 16;
        int nseg = (nrb + CAT_MAXC - 1) / CAT_MAXC;
        if (nstrips * nseg > waves) return false;
    }
    return true;
}

// Launchers (return the HIP status of the launch).
hipError_t launch_cat(const CatParams &p, int elem, int epi, int waves, hipStream_t s);
hipError_t launch_direct(const DirectParams &p, hipStream_t s);
hipError_t launch_validate(const uint8_t *src, int H, int W, size_t pitch, int states,
                           uint32_t *flag, hipStream_t s);

// Kernel symbol and launch shape, for building graph nodes.
struct KernelLaunch {
    const void *func;
    dim3 grid, block;
    size_t lds;
};
KernelLaunch cat_launch_shape(const CatParams &p, int elem, int epi, int waves);
// Resident workgroups of the CAT kernel per compute unit for this shape (0 if it cannot run).
int cat_occupancy(const CatParams &p, int elem, int epi, int waves);
KernelLaunch direct_launch_shape(const DirectParams &p);
size_t cat_lds_bytes(const CatParams &p, int elem, int epi);

}  // namespace ltl
