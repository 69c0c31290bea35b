// Host side of libltl, single grids: argument and rule validation, launch planning (tile
// shape, steps per launch), the ping-pong driver with hipGraph replay of multi-launch loops,
// and the autotuner. Every step of the automaton itself runs in the kernels of this library.
// The batched API is in batch_api.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "ltl.h"
#include "host_common.h"
#include "ltl_internal.h"
#include "tuning_cache.h"

using namespace ltl;

namespace ltl {
namespace host {

thread_local std::string g_err;
thread_local int32_t g_code = LTL_OK;

int32_t fail(int32_t code, const std::string &msg) {
    g_err = msg;
    g_code = code;
    return code;
}

int32_t hip_fail(hipError_t e, const char *what) {
    (void)hipGetLastError();
    return fail(LTL_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int32_t validate_rule(const ltl_rule_t *r, int method) {
    if (!r) return fail(LTL_ERR_ARG, "rule is NULL");
    if (r->N != 'M' && r->N != 'N')
        return fail(LTL_ERR_UNSUPPORTED, "neighbourhood N must be 'M' (Moore) or 'N' (cross, simplified Von Neumann)");
    if (r->R < 1 || r->R > 32) return fail(LTL_ERR_RULE, "radius R must be in 1..32");
    if (r->C < 0 || r->C == 1 || r->C > 255) return fail(LTL_ERR_RULE, "C must be 0 or in 2..255");
    if (r->M != 0 && r->M != 1) return fail(LTL_ERR_RULE, "M must be 0 or 1");
    const int nmax = (2 * r->R + 1) * (2 * r->R + 1);
    const int th[4] = {r->S1, r->S2, r->B1, r->B2};
    for (int v : th)
        if (v < 0 || v > nmax) return fail(LTL_ERR_RULE, "S and B thresholds must be in 0..(2R+1)^2");
    if (method < LTL_CAT_I8 || method > LTL_DIRECT) return fail(LTL_ERR_ARG, "unknown method");
    if (method == LTL_CAT_F8 && 2 * r->R + 1 > 16)
        return fail(LTL_ERR_INEXACT, "FP8 (e4m3) counts are exact only for 2R+1 <= 16");
    if (method == LTL_CAT_F16 && r->R > 16)
        return fail(LTL_ERR_UNSUPPORTED, "the FP16 method covers radii 1..16 (int8 covers 1..32)");
    if (r->N == 'N' && (method == LTL_CAT_F16 || method == LTL_CAT_F8))
        return fail(LTL_ERR_UNSUPPORTED, "the cross neighbourhood runs on the int8 CAT and direct methods");
    if (r->N == 'N' && method == LTL_CAT_I8 && r->R > 16)
        return fail(LTL_ERR_UNSUPPORTED, "the int8 CAT cross neighbourhood covers radii 1..16");
    return LTL_OK;
}

int max_count(const ltl_rule_t &r) { return r.N == 'N' ? 4 * r.R + 1 : (2 * r.R + 1) * (2 * r.R + 1); }

// Survival (alive centre) and birth ranges on the box count n (centre included), clipped to
// 0..nmax; an alive centre with M = 0 sees n - 1, so its survival range moves up by one. An
// empty range is returned as lo = `cap`, hi = 0 (no count satisfies both tests).
struct Ranges {
    int ls, hs, lb, hb;
    bool s_empty, b_empty;
};
static Ranges rule_ranges(const ltl_rule_t &r, int cap) {
    const int nmax = max_count(r);
    const int shift = (r.M == 0) ? 1 : 0;
    Ranges g;
    auto norm = [&](int lo, int hi, int &olo, int &ohi, bool &empty) {
        empty = (lo > hi || lo > nmax || hi < 0);
        if (empty) { olo = cap; ohi = 0; return; }
        olo = std::max(lo, 0);
        ohi = std::min(hi, nmax);
    };
    norm(r.S1 + shift, r.S2 + shift, g.ls, g.hs, g.s_empty);
    norm(r.B1, r.B2, g.lb, g.hb, g.b_empty);
    return g;
}

// Window offset of the windowed epilogues: c = (smallest lower bound) - 1, valid when every
// upper bound is at most c + width (126 for EPI_WIN's 7-bit lanes, 254 for the full bytes of
// EPI_WIN8 and EPI_DECAY8W). Returns false when the ranges span more than that.
static bool window_of(const ltl_rule_t &r, int width, int *c) {
    const Ranges g = rule_ranges(r, 127);
    int lo = 1 << 30, hi = -(1 << 30);
    if (!g.s_empty) { lo = std::min(lo, g.ls); hi = std::max(hi, g.hs); }
    if (!g.b_empty) { lo = std::min(lo, g.lb); hi = std::max(hi, g.hb); }
    if (g.s_empty && g.b_empty) { *c = 0; return true; }
    *c = lo - 1;
    return hi - *c <= width;
}

int epi_of(const ltl_rule_t &r, int elem) {
    int c = 0;
    if (r.C >= 3) {
        if (r.C <= 8 && elem == ELEM_I8) return window_of(r, 254, &c) ? EPI_DECAY8W : EPI_DECAY8;
        return EPI_DECAY;
    }
    if (max_count(r) <= 126) return EPI_BYTE;
    if (elem == ELEM_I8 && window_of(r, 126, &c)) return EPI_WIN;
    if (elem == ELEM_I8 && window_of(r, 254, &c)) return EPI_WIN8;
    return EPI_HALF;
}

// Next-state tables of the C <= 8 decay epilogues: state k -> next state when the range test
// fails (N0) or holds (N1): 0 -> born (1) or stays 0, 1 -> survives (1) or starts to decay (2),
// k >= 2 -> k + 1, wrapping to 0 at C; bytes k >= C are never selected.
static void decay_tables(RuleConsts &c) {
    uint64_t t0 = 0, t1 = 0;
    for (int k = 0; k < 8; ++k) {
        const int dec = (k >= 2 && k < c.C) ? (k + 1 < c.C ? k + 1 : 0) : 0;
        const int f = k == 0 ? 0 : k == 1 ? 2 : dec;
        const int h = k == 0 ? 1 : k == 1 ? 1 : dec;
        t0 |= (uint64_t)f << (8 * k);
        t1 |= (uint64_t)h << (8 * k);
    }
    c.N0lo = (uint32_t)t0; c.N0hi = (uint32_t)(t0 >> 32);
    c.N1lo = (uint32_t)t1; c.N1hi = (uint32_t)(t1 >> 32);
}

// Thresholds on the box count n (centre included) and the SWAR constants of the two-state
// epilogues. An alive centre with M = 0 sees n - 1, so its survival range moves up by one.
RuleConsts make_consts(const ltl_rule_t &r, int epi) {
    RuleConsts c;
    std::memset(&c, 0, sizeof(c));
    c.C = r.C >= 3 ? r.C : 2;
    c.M = r.M;
    c.s1 = r.S1; c.s2 = r.S2; c.b1 = r.B1; c.b2 = r.B2;
    int ls, hs, lb, hb;
    uint32_t rep, top, klo_s, klo_b, khi_s, khi_b;
    if (epi == EPI_WIN8 || epi == EPI_DECAY8W) {
        // full-byte range tests on n - c: Tlo = 256 - lo, Thi = hi + 1 per centre state (byte 0
        // dead, byte 1 alive), bounds relative to the window (1 <= lo, hi <= 254); an empty range
        // becomes lo = 255, hi = 0, which no byte satisfies
        const Ranges g = rule_ranges(r, 127);
        (void)window_of(r, 254, &c.cwin);
        const int lb = g.b_empty ? 255 : g.lb - c.cwin, hb = g.b_empty ? 0 : g.hb - c.cwin;
        const int ls = g.s_empty ? 255 : g.ls - c.cwin, hs = g.s_empty ? 0 : g.hs - c.cwin;
        c.Tlo = (uint32_t)(256 - lb) | ((uint32_t)(256 - ls) << 8);
        c.Thi = (uint32_t)(hb + 1) | ((uint32_t)(hs + 1) << 8);
        if (epi == EPI_DECAY8W) {
            c.Crep = (uint32_t)c.C * 0x01010101u;
            decay_tables(c);
        }
        return c;
    }
    if (epi == EPI_BYTE || epi == EPI_WIN) {
        Ranges g = rule_ranges(r, 127);
        if (epi == EPI_WIN) {   // thresholds relative to the window offset (non-empty ranges)
            (void)window_of(r, 126, &c.cwin);
            if (!g.s_empty) { g.ls -= c.cwin; g.hs -= c.cwin; }
            if (!g.b_empty) { g.lb -= c.cwin; g.hb -= c.cwin; }
        }
        ls = g.ls; hs = g.hs; lb = g.lb; hb = g.hb;
        rep = 0x01010101u;
        top = 0x80u;
    } else if (epi == EPI_HALF || epi_decays(epi)) {   // decay: the range test of the s in {0, 1} case
        const Ranges g = rule_ranges(r, 2047);
        c.Crep = (uint32_t)c.C * 0x01010101u;
        if (epi == EPI_DECAY8) decay_tables(c);
        ls = g.ls; hs = g.hs; lb = g.lb; hb = g.hb;
        rep = 0x00010001u;
        top = 0x8000u;
    } else {
        return c;
    }
    klo_s = (top - (uint32_t)ls) * rep;
    klo_b = (top - (uint32_t)lb) * rep;
    khi_s = (top + (uint32_t)hs) * rep;
    khi_b = (top + (uint32_t)hb) * rep;
    // select x_s where the lane mask m = sm ^ (top * rep) is all ones (alive centre), x_b where it
    // is zero:  x_b ^ (m & (x_s ^ x_b))  =  [x_b ^ (top*rep & D)] ^ (sm & D),  D = x_s ^ x_b
    c.Dlo = klo_s ^ klo_b;
    c.Klo = klo_b ^ ((top * rep) & c.Dlo);
    c.Dhi = khi_s ^ khi_b;
    c.Khi = khi_b ^ ((top * rep) & c.Dhi);
    if (epi == EPI_BYTE || epi == EPI_WIN) {
        c.Tlo = (klo_b & 0xFFu) | ((klo_s & 0xFFu) << 8);
        c.Thi = (khi_b & 0xFFu) | ((khi_s & 0xFFu) << 8);
    }
    return c;
}

int pitch_of(int W) { return roundup(W, 64); }

// Largest grid the kernels address: row offsets are 32-bit (H x pitch < 2^31 bytes).
constexpr size_t kMaxGridBytes = 0x7FFFFFFF;
bool grid_too_large(int H, int W) { return (size_t)H * (size_t)pitch_of(W) > kMaxGridBytes; }

size_t max_lds_bytes() {
    static size_t v = 0;
    if (v == 0) {
        int dev = 0, x = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&x, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && x > 0)
            v = (size_t)x;
        else
            v = 65536;
    }
    return v;
}

int elem_of(int method, int R, int N) {
    if (method == LTL_CAT_I8 && N == 'N') return ELEM_I8X;
    if (method == LTL_CAT_I8 && R > 16) return ELEM_I8W;
    return method == LTL_CAT_F16 ? ELEM_F16 : method == LTL_CAT_F8 ? ELEM_F8 : ELEM_I8;
}

}  // namespace host
}  // namespace ltl

using namespace ltl::host;

struct ltl_sim {
    int32_t H = 0, W = 0, pitch = 0;
    ltl_rule_t rule{};
    int method = 0;
    int epi = 0;
    RuleConsts rc{};
    uint8_t *buf[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t steps_done = 0;
    hipStream_t stream = nullptr;
    ltl_tuning_t tuning{};
    uint32_t *dflag = nullptr;
    uint8_t *dconst = nullptr;   // band tables for r = 1..16, then a zero page
    int periodic = 0;            // LTL_BOUNDARY_PERIODIC: the grid is a torus
    bool user_tuned = false;     // the launch shape came from set_tuning / autotune (not the table)
    std::map<std::pair<int32_t, int>, hipGraphExec_t> graphs;
    // dataflow form (persistent = 2): kFlowMaxTiles per-tile round counters, then the timeout
    // counter; the counters only grow (flow_epoch), so they are zeroed once, at creation
    uint32_t *dflow = nullptr;
    uint32_t flow_epoch = 0;
    uint32_t *herr = nullptr;    // pinned host copy of the timeout counter, refreshed after each launch
    uint32_t err_seen = 0;
};

namespace {

// Device constants shared by the CAT launches of a handle: the band operands of its radius and
// element type (band_table layout, 8 KiB) followed by a 4 KiB zero page.
constexpr size_t kConstBytes = kBandBytes + 4096;

std::vector<uint8_t> host_constants(int elem, int r) {
    std::vector<uint8_t> h(kConstBytes, 0);
    band_table(elem, r, reinterpret_cast<int32_t *>(h.data()));
    return h;
}

ltl_tuning_t default_tuning(const ltl_sim &s) {
    ltl_tuning_t t;
    t.steps_per_launch = 1;
    t.tile_rows = 64;
    t.tile_cols = 64;
    t.waves = 4;
    // grow the wave count until the widest step fits (one strip segment per wave)
    while (t.waves < 8 && !cat_shape_fits(elem_of(s.method, s.rule.R, s.rule.N), s.rule.R, t.steps_per_launch, t.tile_rows, t.tile_cols,
                                          t.waves))
        t.waves *= 2;
    t.use_graph = 1;
    t.persistent = 0;
    t.lds_pad = 0;
    return t;
}

CatParams cat_params(const ltl_sim &s, const ltl_tuning_t &t, int T, const uint8_t *src, uint8_t *dst) {
    CatParams p;
    p.src = src;
    p.dst = dst;
    p.H = s.H;
    p.W = s.W;
    p.pitch = s.pitch;
    p.r = s.rule.R;
    p.T = T;
    p.TH = t.tile_rows;
    p.TW = t.tile_cols;
    p.L = cat_margin(elem_of(s.method, s.rule.R, s.rule.N), p.r, T);
    p.lds_rows = p.TH + 2 * p.L;
    cat_lds_layout(elem_of(s.method, s.rule.R, s.rule.N), s.epi, p.TH, p.TW, p.L, t.lds_pad, &p.PS, &p.PA, &p.lds_tile,
                   &p.a_tile, &p.lds_total);
    p.ntx = (s.W + p.TW - 1) / p.TW;
    p.nty = (s.H + p.TH - 1) / p.TH;
    p.bands = reinterpret_cast<const int32_t *>(s.dconst);
    p.zero = s.dconst + kBandBytes;
    p.periodic = s.periodic;
    p.store_w = s.periodic ? s.W : s.pitch;
    p.rc = s.rc;
    return p;
}

DirectParams direct_params(const ltl_sim &s, const uint8_t *src, uint8_t *dst) {
    DirectParams p;
    p.src = src;
    p.dst = dst;
    p.H = s.H;
    p.W = s.W;
    p.pitch = s.pitch;
    p.r = s.rule.R;
    p.TH = kDirectTH;
    p.TW = kDirectTW;
    p.LP = direct_lds_pitch(p.r);
    p.periodic = s.periodic;
    p.cross = (s.rule.N == 'N') ? 1 : 0;
    p.rc = s.rc;
    return p;
}

bool cooperative_launch_supported() {
    int dev = 0, v = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&v, hipDeviceAttributeCooperativeLaunch, dev);
    quiet(e);
    return e == hipSuccess && v != 0;
}

int cu_count() {
    int dev = 0, v = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
    quiet(e);
    return e == hipSuccess ? v : 0;
}

// The dataflow form needs every tile's workgroup resident at once, at most kFlowMaxTiles tiles,
// and windows that reach no further than the eight neighbouring tiles (margin <= the tile's
// rows and columns; on a torus also <= the partial last tile row / column that wraps around).
int32_t check_flow(const ltl_sim &s, const ltl_tuning_t &t) {
    const int elem = elem_of(s.method, s.rule.R, s.rule.N);
    const int L = cat_margin(elem, s.rule.R, t.steps_per_launch);
    const int ntx = (s.W + t.tile_cols - 1) / t.tile_cols, nty = (s.H + t.tile_rows - 1) / t.tile_rows;
    if (ntx * nty > kFlowMaxTiles) return fail(LTL_ERR_ARG, "the dataflow form (persistent = 2) tracks at most 4096 tiles");
    if (L > t.tile_rows || L > t.tile_cols)
        return fail(LTL_ERR_ARG, "the dataflow form needs a margin (" + std::to_string(L) + ") no wider than the tile");
    if (s.periodic) {
        const int rw = s.W % t.tile_cols, rh = s.H % t.tile_rows;
        if ((rw && rw < L) || (rh && rh < L))
            return fail(LTL_ERR_ARG, "the dataflow form on a torus needs partial edge tiles at least as wide as the margin");
    }
    if (s.dconst) {   // device checks, once the handle exists
        if (!cooperative_launch_supported()) return fail(LTL_ERR_UNSUPPORTED, "the device has no cooperative launch");
        CatParams p = cat_params(s, t, t.steps_per_launch, nullptr, nullptr);
        const int occ = cat_flow_occupancy(p, elem, s.epi, t.waves);
        if (roundup(ntx * nty, 8) > occ * cu_count())
            return fail(LTL_ERR_ARG, "the dataflow form needs all " + std::to_string(ntx * nty) +
                                         " tiles resident at once (" + std::to_string(occ) + " workgroups per CU)");
    }
    return LTL_OK;
}

int32_t check_tuning(const ltl_sim &s, const ltl_tuning_t &t) {
    if (t.steps_per_launch < 1 || t.steps_per_launch > 64) return fail(LTL_ERR_ARG, "steps_per_launch must be in 1..64");
    if (t.tile_rows < 16 || t.tile_rows > 512 || t.tile_rows % 16) return fail(LTL_ERR_ARG, "tile_rows must be a multiple of 16 in 16..512");
    if (t.tile_cols < 32 || t.tile_cols > 512 || t.tile_cols % 32) return fail(LTL_ERR_ARG, "tile_cols must be a multiple of 32 in 32..512");
    if (t.waves < 1 || t.waves > (s.method == LTL_DIRECT ? 16 : 8)) return fail(LTL_ERR_ARG, "waves must be in 1..8 (1..16 for the direct method)");
    if (t.lds_pad < 0 || t.lds_pad > 128 || t.lds_pad % 16) return fail(LTL_ERR_ARG, "lds_pad must be a multiple of 16 in 0..128");
    if (t.persistent < 0 || t.persistent > 2) return fail(LTL_ERR_ARG, "persistent must be 0, 1 or 2");
    if (s.method != LTL_DIRECT) {
        // host-side checks first: the device queries below must only see shapes that can exist
        CatParams p = cat_params(s, t, t.steps_per_launch, nullptr, nullptr);
        size_t lds = cat_lds_bytes(p, elem_of(s.method, s.rule.R, s.rule.N), s.epi, t.persistent == 1);
        if (lds > max_lds_bytes()) return fail(LTL_ERR_ARG, "launch shape needs " + std::to_string(lds) + " bytes of LDS");
        if (!cat_shape_fits(elem_of(s.method, s.rule.R, s.rule.N), s.rule.R, t.steps_per_launch, t.tile_rows, t.tile_cols, t.waves))
            return fail(LTL_ERR_ARG, "launch shape has more strip segments than waves in some step");
        if (t.persistent == 2) {
            int32_t rc = check_flow(s, t);
            if (rc != LTL_OK) return rc;
        } else if (s.dconst && cat_occupancy(p, elem_of(s.method, s.rule.R, s.rule.N), s.epi, t.waves, t.persistent) < 1) {
            return fail(LTL_ERR_ARG, "launch shape does not fit on a compute unit (registers or LDS)");
        }
    } else if (t.steps_per_launch != 1) {
        return fail(LTL_ERR_ARG, "the direct method takes one step per launch");
    } else if (t.persistent) {
        return fail(LTL_ERR_ARG, "the direct method has no persistent form");
    }
    return LTL_OK;
}

// Launch shape and argument block of launch number k (steps_in_launch steps) starting
// from buffer `from`.
struct PlannedLaunch {
    KernelLaunch k;
    CatParams cp;
    DirectParams dp;
    bool direct;
};

PlannedLaunch plan(const ltl_sim &s, int steps_in_launch, int from) {
    PlannedLaunch pl;
    const uint8_t *src = s.buf[from];
    uint8_t *dst = s.buf[from ^ 1];
    pl.direct = (s.method == LTL_DIRECT);
    if (pl.direct) {
        pl.dp = direct_params(s, src, dst);
        pl.k = direct_launch_shape(pl.dp);
    } else {
        pl.cp = cat_params(s, s.tuning, steps_in_launch, src, dst);
        pl.k = cat_launch_shape(pl.cp, elem_of(s.method, s.rule.R, s.rule.N), s.epi, s.tuning.waves, s.tuning.persistent);
    }
    return pl;
}

std::vector<int> launch_sizes(const ltl_sim &s, int n) {
    std::vector<int> v;
    int T = (s.method == LTL_DIRECT) ? 1 : s.tuning.steps_per_launch;
    while (n > 0) {
        int t = std::min(T, n);
        v.push_back(t);
        n -= t;
    }
    return v;
}

hipError_t enqueue_one(ltl_sim &s, const PlannedLaunch &pl) {
    if (pl.k.lds > 65536) {
        hipError_t e = hipFuncSetAttribute(pl.k.func, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.k.lds);
        if (e != hipSuccess) return e;
    }
    void *args[1];
    args[0] = pl.direct ? (void *)&pl.dp : (void *)&pl.cp;
    return hipLaunchKernel(pl.k.func, pl.k.grid, pl.k.block, args, pl.k.lds, s.stream);
}

// Executable graphs are destroyed only once the stream has drained: a replay enqueued by an
// earlier step call may still be running.
void clear_graphs(ltl_sim &s) {
    if (s.graphs.empty()) return;
    quiet(hipStreamSynchronize(s.stream));
    for (auto &kv : s.graphs) quiet(hipGraphExecDestroy(kv.second));
    s.graphs.clear();
}

int32_t build_graph(ltl_sim &s, int n, int from, hipGraphExec_t *out) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipGraphCreate(&g, 0), "hipGraphCreate");
    hipGraphNode_t prev = nullptr;
    int b = from;
    std::vector<int> sizes = launch_sizes(s, n);
    for (int t : sizes) {
        PlannedLaunch pl = plan(s, t, b);
        if (pl.k.lds > 65536) {
            hipError_t e = hipFuncSetAttribute(pl.k.func, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.k.lds);
            if (e != hipSuccess) { quiet(hipGraphDestroy(g)); return hip_fail(e, "hipFuncSetAttribute"); }
        }
        hipKernelNodeParams kp;
        std::memset(&kp, 0, sizeof(kp));
        void *args[1];
        args[0] = pl.direct ? (void *)&pl.dp : (void *)&pl.cp;
        kp.func = const_cast<void *>(pl.k.func);
        kp.gridDim = pl.k.grid;
        kp.blockDim = pl.k.block;
        kp.sharedMemBytes = (unsigned)pl.k.lds;
        kp.kernelParams = args;
        kp.extra = nullptr;
        hipGraphNode_t node;
        hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
        if (e != hipSuccess) { quiet(hipGraphDestroy(g)); return hip_fail(e, "hipGraphAddKernelNode"); }
        prev = node;
        b ^= 1;
    }
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    quiet(hipGraphDestroy(g));
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    *out = ex;
    return LTL_OK;
}

// Polls per dataflow wait before it counts as timed out (LTL_FLOW_SPIN_LIMIT overrides it; the
// tests force the timeout path with a tiny limit). One poll sleeps about 64 clock cycles, so the
// default is a fraction of a second, far beyond any round.
int flow_spin_limit() {
    const char *e = std::getenv("LTL_FLOW_SPIN_LIMIT");
    if (e && *e) {
        char *end = nullptr;
        const long v = std::strtol(e, &end, 10);
        if (end != e && !*end && v >= 0 && v <= (1L << 30)) return (int)v;
    }
    return 1 << 24;
}

// One cooperative launch of the dataflow kernel covering all n steps of the chunk, followed by
// an asynchronous copy of the timeout counter into the handle's pinned host word.
int32_t do_flow_chunk(ltl_sim &s, int32_t n) {
    const int T = s.tuning.steps_per_launch;
    FlowParams f;
    f.buf[0] = s.buf[0];
    f.buf[1] = s.buf[1];
    f.flags = s.dflow;
    f.err = s.dflow + kFlowMaxTiles;
    f.epoch = s.flow_epoch;
    f.first = s.cur;
    f.rounds = (n + T - 1) / T;
    f.last_T = n - (f.rounds - 1) * T;
    f.spin_limit = flow_spin_limit();
    f.pad = 0;
    CatParams p = cat_params(s, s.tuning, T, nullptr, nullptr);
    HIP_TRY(launch_cat_flow(p, f, elem_of(s.method, s.rule.R, s.rule.N), s.epi, s.tuning.waves, s.stream),
            "cooperative launch of the dataflow kernel");
    HIP_TRY(hipMemcpyAsync(s.herr, f.err, sizeof(uint32_t), hipMemcpyDeviceToHost, s.stream), "hipMemcpyAsync");
    s.flow_epoch += (uint32_t)f.rounds;
    s.cur ^= (f.rounds & 1);
    s.steps_done += n;
    return LTL_OK;
}

// A dataflow wait that ran out in an earlier call (seen once its counter copy has landed).
int32_t check_flow_timeouts(ltl_sim &s) {
    if (!s.herr) return LTL_OK;
    const uint32_t v = __atomic_load_n(s.herr, __ATOMIC_ACQUIRE);
    if (v != s.err_seen) {
        s.err_seen = v;
        return fail(LTL_ERR_HIP, "a dataflow wait of an earlier step call timed out (its grid is not valid)");
    }
    return LTL_OK;
}

int32_t do_chunk(ltl_sim &s, int32_t n) {
    if (s.method != LTL_DIRECT && s.tuning.persistent == 2) return do_flow_chunk(s, n);
    std::vector<int> sizes = launch_sizes(s, n);
    if (s.tuning.use_graph && sizes.size() > 1) {
        auto key = std::make_pair(n, s.cur);
        auto it = s.graphs.find(key);
        hipGraphExec_t ex = nullptr;
        if (it == s.graphs.end()) {
            if (s.graphs.size() >= 32) clear_graphs(s);
            int32_t rc = build_graph(s, n, s.cur, &ex);
            if (rc != LTL_OK) return rc;
            s.graphs[key] = ex;
        } else {
            ex = it->second;
        }
        HIP_TRY(hipGraphLaunch(ex, s.stream), "hipGraphLaunch");
        s.cur ^= (int)(sizes.size() & 1);
    } else {
        for (int t : sizes) {
            PlannedLaunch pl = plan(s, t, s.cur);
            HIP_TRY(enqueue_one(s, pl), "kernel launch");
            s.cur ^= 1;
        }
    }
    s.steps_done += n;
    return LTL_OK;
}

int32_t do_steps(ltl_sim &s, int32_t n) {
    const int T = (s.method == LTL_DIRECT) ? 1 : s.tuning.steps_per_launch;
    const int32_t chunk = T * kMaxChunkLaunches;
    while (n > 0) {
        const int32_t m = std::min(n, chunk);
        int32_t rc = do_chunk(s, m);
        if (rc != LTL_OK) return rc;
        n -= m;
    }
    return LTL_OK;
}

// Launch shape of a new handle: LTL_TILE if set (refused if malformed or infeasible), else the
// first tuning-table candidate (nearest radius, then size bucket) that is feasible for this
// grid, else the built-in default.
int32_t initial_tuning(ltl_sim &s) {
    ltl_tuning_t t;
    std::string err;
    const int env = env_tile(&t, &err);
    if (env < 0) return fail(LTL_ERR_ARG, err);
    if (env > 0) {
        if (s.method == LTL_DIRECT) { t.steps_per_launch = 1; t.persistent = 0; }
        if (check_tuning(s, t) != LTL_OK) return fail(LTL_ERR_ARG, "LTL_TILE: " + g_err);
        s.tuning = t;
        return LTL_OK;
    }
    const SavedError saved = save_error();
    for (const ltl_tuning_t &c : tuning_candidates(make_key(s.H, s.W, s.rule, s.method, s.periodic, 0), nullptr)) {
        if (check_tuning(s, c) == LTL_OK) {
            s.tuning = c;
            restore_error(saved);
            return LTL_OK;
        }
    }
    restore_error(saved);
    s.tuning = default_tuning(s);
    return LTL_OK;
}

// ---- allocation-free runs (ltl_run_noalloc)
// The device constants of those runs (one band table and the zero page, 12 KiB) live in this
// file-scope array. In host code its name is only a stand-in; the device address comes from
// hipGetSymbolAddress, once per device, on the first allocation-free call with that device
// current. Every allocation-free call on a device rewrites that device's copy, so such calls
// must not overlap on one device (they would race on the band table).
constexpr size_t kScratchBytes = kConstBytes;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];
static_assert(kBandBytes + 16 <= kScratchBytes, "a band table and a zero vector fit in the static area");
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};

int32_t scratch_of_current_device(uint8_t **out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(LTL_ERR_ARG, "device index outside 0..63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
        if (!ptr) return fail(LTL_ERR_HIP, "hipGetSymbolAddress returned NULL");
        g_scratch_ptr[dev] = static_cast<uint8_t *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return LTL_OK;
}

}  // namespace

extern "C" {

const char *ltl_last_error(void) { return g_err.c_str(); }

int32_t ltl_last_error_code(void) { return g_code; }

int32_t ltl_pitch(int32_t W, int32_t *pitch) {
    if (!pitch || W < 1) return fail(LTL_ERR_ARG, "W must be >= 1 and pitch non-NULL");
    *pitch = pitch_of(W);
    return LTL_OK;
}

size_t ltl_buffer_bytes(int32_t H, int32_t W, int32_t R, int32_t method) {
    if (H < 1 || W < 1) { fail(LTL_ERR_ARG, "H and W must be >= 1"); return 0; }
    if (R < 1 || R > 32) { fail(LTL_ERR_RULE, "radius R must be in 1..32"); return 0; }
    if (method < LTL_CAT_I8 || method > LTL_DIRECT) { fail(LTL_ERR_ARG, "unknown method"); return 0; }
    return (size_t)H * (size_t)pitch_of(W);
}

int32_t ltl_create(ltl_sim_t **out, int32_t H, int32_t W, const ltl_rule_t *rule, int32_t method,
                   void *buf_a, void *buf_b, size_t buf_bytes, const void *init, size_t init_pitch,
                   hipStream_t stream) {
    if (!out) return fail(LTL_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (H < 1 || W < 1) return fail(LTL_ERR_ARG, "H and W must be >= 1");
    if (!buf_a || !buf_b || !init) return fail(LTL_ERR_ARG, "NULL buffer");
    if (buf_a == buf_b) return fail(LTL_ERR_ARG, "the two buffers must differ");
    if (init_pitch < (size_t)W) return fail(LTL_ERR_ARG, "init_pitch < W");
    if (grid_too_large(H, W)) return fail(LTL_ERR_SIZE, "grid larger than 2^31 - 1 bytes (H x ltl_pitch(W))");
    if (((uintptr_t)buf_a & 255) || ((uintptr_t)buf_b & 255)) return fail(LTL_ERR_ARG, "buffers must be 256-byte aligned");
    int32_t rc = validate_rule(rule, method);
    if (rc != LTL_OK) return rc;
    size_t need = (size_t)H * (size_t)pitch_of(W);
    if (buf_bytes < need) return fail(LTL_ERR_SIZE, "buffers need " + std::to_string(need) + " bytes each");
    {
        ltl_tuning_t t;
        std::string err;
        if (env_tile(&t, &err) < 0) return fail(LTL_ERR_ARG, err);   // malformed LTL_TILE, before any device work
    }

    ltl_sim *s = new (std::nothrow) ltl_sim();
    if (!s) return fail(LTL_ERR_ARG, "out of host memory");
    s->H = H;
    s->W = W;
    s->pitch = pitch_of(W);
    s->rule = *rule;
    s->method = method;
    s->epi = epi_of(*rule, elem_of(method, rule->R, rule->N));
    s->rc = make_consts(*rule, s->epi);
    s->buf[0] = (uint8_t *)buf_a;
    s->buf[1] = (uint8_t *)buf_b;
    s->stream = stream;
    s->tuning = default_tuning(*s);   // replaced below, once the device constants exist

    auto bail = [&](int32_t code) {
        if (s->dflag) quiet(hipFree(s->dflag));
        if (s->dconst) quiet(hipFree(s->dconst));
        if (s->dflow) quiet(hipFree(s->dflow));
        if (s->herr) quiet(hipHostFree(s->herr));
        delete s;
        return code;
    };
    hipError_t e;
    if ((e = hipMalloc(&s->dflag, sizeof(uint32_t))) != hipSuccess) { s->dflag = nullptr; return bail(hip_fail(e, "hipMalloc")); }
    if ((e = hipMalloc(&s->dflow, (kFlowMaxTiles + 1) * sizeof(uint32_t))) != hipSuccess) {
        s->dflow = nullptr;
        return bail(hip_fail(e, "hipMalloc"));
    }
    if ((e = hipHostMalloc(&s->herr, sizeof(uint32_t), hipHostMallocDefault)) != hipSuccess) {
        s->herr = nullptr;
        return bail(hip_fail(e, "hipHostMalloc"));
    }
    *s->herr = 0;
    if ((e = hipMemsetAsync(s->dflow, 0, (kFlowMaxTiles + 1) * sizeof(uint32_t), stream)) != hipSuccess)
        return bail(hip_fail(e, "hipMemsetAsync"));
    if ((e = hipMalloc(&s->dconst, kConstBytes)) != hipSuccess) { s->dconst = nullptr; return bail(hip_fail(e, "hipMalloc")); }
    {
        std::vector<uint8_t> hc = host_constants(elem_of(method, rule->R, rule->N), rule->R);
        if ((e = hipMemcpyAsync(s->dconst, hc.data(), kConstBytes, hipMemcpyHostToDevice, stream)) != hipSuccess)
            return bail(hip_fail(e, "hipMemcpyAsync"));
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return bail(hip_fail(e, "hipStreamSynchronize"));
    }
    if ((e = hipMemsetAsync(s->dflag, 0, sizeof(uint32_t), stream)) != hipSuccess) return bail(hip_fail(e, "hipMemsetAsync"));
    if ((e = launch_validate((const uint8_t *)init, H, W, init_pitch, s->rc.C, s->dflag, stream)) != hipSuccess)
        return bail(hip_fail(e, "validate launch"));
    uint32_t bad = 0;
    if ((e = hipMemcpyAsync(&bad, s->dflag, sizeof(bad), hipMemcpyDeviceToHost, stream)) != hipSuccess) return bail(hip_fail(e, "hipMemcpyAsync"));
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return bail(hip_fail(e, "hipStreamSynchronize"));
    if (bad) return bail(fail(LTL_ERR_STATE, "initial grid holds a state >= max(C, 2)"));
    for (int b = 0; b < 2; ++b)
        if ((e = hipMemsetAsync(s->buf[b], 0, need, stream)) != hipSuccess) return bail(hip_fail(e, "hipMemsetAsync"));
    if ((e = hipMemcpy2DAsync(s->buf[0], s->pitch, init, init_pitch, W, H, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
        return bail(hip_fail(e, "hipMemcpy2DAsync"));
    if ((rc = initial_tuning(*s)) != LTL_OK) return bail(rc);
    *out = s;
    return LTL_OK;
}

int32_t ltl_step(ltl_sim_t *sim, int32_t n_steps) {
    if (!sim) return fail(LTL_ERR_ARG, "sim is NULL");
    if (n_steps < 0) return fail(LTL_ERR_ARG, "n_steps must be >= 0");
    int32_t rc = check_flow_timeouts(*sim);
    if (rc != LTL_OK) return rc;
    return do_steps(*sim, n_steps);
}

int32_t ltl_read(ltl_sim_t *sim, void *dst, size_t dst_pitch) {
    if (!sim || !dst) return fail(LTL_ERR_ARG, "NULL argument");
    if (dst_pitch < (size_t)sim->W) return fail(LTL_ERR_ARG, "dst_pitch < W");
    int32_t rc = check_flow_timeouts(*sim);
    if (rc != LTL_OK) return rc;
    HIP_TRY(hipMemcpy2DAsync(dst, dst_pitch, sim->buf[sim->cur], sim->pitch, sim->W, sim->H,
                             hipMemcpyDeviceToDevice, sim->stream), "hipMemcpy2DAsync");
    return LTL_OK;
}

int32_t ltl_current(ltl_sim_t *sim, void **buf, size_t *pitch, int64_t *steps_done) {
    if (!sim) return fail(LTL_ERR_ARG, "sim is NULL");
    if (buf) *buf = sim->buf[sim->cur];
    if (pitch) *pitch = (size_t)sim->pitch;
    if (steps_done) *steps_done = sim->steps_done;
    return LTL_OK;
}

int32_t ltl_get_tuning(ltl_sim_t *sim, ltl_tuning_t *tuning) {
    if (!sim || !tuning) return fail(LTL_ERR_ARG, "NULL argument");
    *tuning = sim->tuning;
    return LTL_OK;
}

static bool s_fits(const ltl_sim &s, const ltl_tuning_t &t) {
    return s.method != LTL_DIRECT &&
           !cat_shape_fits(elem_of(s.method, s.rule.R, s.rule.N), s.rule.R, t.steps_per_launch, t.tile_rows, t.tile_cols, t.waves);
}

int32_t ltl_set_tuning(ltl_sim_t *sim, const ltl_tuning_t *tuning) {
    if (!sim || !tuning) return fail(LTL_ERR_ARG, "NULL argument");
    ltl_tuning_t t = *tuning;
    ltl_tuning_t d = default_tuning(*sim);
    if (t.steps_per_launch == 0) t.steps_per_launch = d.steps_per_launch;
    if (t.tile_rows == 0) t.tile_rows = d.tile_rows;
    if (t.tile_cols == 0) t.tile_cols = d.tile_cols;
    if (t.waves == 0) {  // smallest wave count (power of two) whose every step fits
        t.waves = 1;
        while (t.waves < 8 && s_fits(*sim, t)) t.waves *= 2;
    }
    t.use_graph = t.use_graph ? 1 : 0;
    if (sim->method == LTL_DIRECT) t.lds_pad = 0;
    int32_t rc = check_tuning(*sim, t);
    if (rc != LTL_OK) return rc;
    clear_graphs(*sim);
    sim->tuning = t;
    sim->user_tuned = true;
    return LTL_OK;
}

int32_t ltl_autotune(ltl_sim_t *sim, int32_t probe_steps, void *scratch, size_t scratch_bytes, ltl_tuning_t *best) {
    if (!sim) return fail(LTL_ERR_ARG, "sim is NULL");
    if (probe_steps < 1 || probe_steps > 4096) return fail(LTL_ERR_ARG, "probe_steps must be in 1..4096");
    ltl_sim &s = *sim;
    if (s.method == LTL_DIRECT) {
        if (best) *best = s.tuning;
        return LTL_OK;
    }
    const size_t bytes = (size_t)s.H * s.pitch;
    if (!scratch) return fail(LTL_ERR_ARG, "scratch is NULL");
    if (scratch_bytes < bytes) return fail(LTL_ERR_SIZE, "scratch needs " + std::to_string(bytes) + " bytes");
    if (scratch == s.buf[0] || scratch == s.buf[1]) return fail(LTL_ERR_ARG, "scratch must not be one of the grid buffers");
    // The probes run on the handle's own buffers (a probe handle sharing them, with its own graph
    // cache); the current state is saved in the caller's scratch, every candidate starts from it
    // and it is restored at the end.
    HIP_TRY(hipMemcpyAsync(scratch, s.buf[s.cur], bytes, hipMemcpyDeviceToDevice, s.stream), "hipMemcpyAsync");
    ltl_sim probe;
    probe.H = s.H; probe.W = s.W; probe.pitch = s.pitch; probe.rule = s.rule; probe.method = s.method;
    probe.epi = s.epi; probe.rc = s.rc; probe.buf[0] = s.buf[0]; probe.buf[1] = s.buf[1];
    probe.periodic = s.periodic;
    probe.dconst = s.dconst;
    probe.dflow = s.dflow;
    probe.herr = s.herr;
    probe.flow_epoch = s.flow_epoch;
    probe.err_seen = s.err_seen;
    probe.stream = s.stream;
    hipEvent_t ev0, ev1;
    HIP_TRY(hipEventCreate(&ev0), "hipEventCreate");
    if (hipEventCreate(&ev1) != hipSuccess) { quiet(hipEventDestroy(ev0)); return fail(LTL_ERR_HIP, "hipEventCreate"); }
    float best_ms = 1e30f;
    ltl_tuning_t best_t = s.tuning;
    int32_t rc = LTL_OK;
    // time one candidate: ms per step, or a negative value if it is infeasible
    auto time_one = [&](const ltl_tuning_t &t, float *ms_out) -> int32_t {
        *ms_out = -1.f;
        const SavedError saved = save_error();
        if (check_tuning(s, t) != LTL_OK) { restore_error(saved); return LTL_OK; }
        // each candidate runs a whole number of its own launches (no shorter remainder launch
        // to bias it) covering at least probe_steps steps; candidates compare per step
        const int T = t.steps_per_launch;
        const int n = T * ((probe_steps + T - 1) / T);
        clear_graphs(probe);
        probe.tuning = t;
        HIP_TRY(hipMemcpyAsync(s.buf[s.cur], scratch, bytes, hipMemcpyDeviceToDevice, s.stream), "hipMemcpyAsync");
        probe.cur = s.cur;
        int32_t r2 = do_steps(probe, n);   // warm-up + graph build
        if (r2 != LTL_OK) return r2;
        float ms = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {   // the faster of two timed runs
            HIP_TRY(hipEventRecord(ev0, s.stream), "hipEventRecord");
            if ((r2 = do_steps(probe, n)) != LTL_OK) return r2;
            HIP_TRY(hipEventRecord(ev1, s.stream), "hipEventRecord");
            HIP_TRY(hipEventSynchronize(ev1), "autotune sync");
            float m = 0;
            HIP_TRY(hipEventElapsedTime(&m, ev0, ev1), "hipEventElapsedTime");
            ms = std::min(ms, m);
        }
        *ms_out = ms / (float)n;
        return LTL_OK;
    };
    const int Ts[] = {1, 2, 3, 4, 5, 6, 8, 12, 16};
    const int tiles[][2] = {{64, 64}, {96, 96}, {128, 128}, {128, 192}, {160, 160}, {192, 128}, {192, 192},
                            {192, 224}, {128, 224}, {160, 224}, {176, 224}, {224, 224}, {64, 128}, {128, 96},
                            {32, 64}};
    const int wavess[] = {0, 8};  // 0: fewest waves that fit every step
    for (int T : Ts)
        for (auto &tl : tiles)
            for (int wv : wavess)
                for (int pers = 0; pers < 3; ++pers) {
                    ltl_tuning_t t;
                    t.steps_per_launch = T; t.tile_rows = tl[0]; t.tile_cols = tl[1]; t.waves = wv; t.use_graph = 1;
                    t.persistent = pers;
                    t.lds_pad = 0;
                    if (wv == 0) {
                        t.waves = 1;
                        while (t.waves < 8 && s_fits(s, t)) t.waves *= 2;
                    }
                    float ms;
                    if ((rc = time_one(t, &ms)) != LTL_OK) goto done;
                    if (ms >= 0 && ms < best_ms) { best_ms = ms; best_t = t; }
                }
    // second stage: LDS row padding of the best shape
    for (int pad : {16, 32, 48, 64, 96}) {
        ltl_tuning_t t = best_t;
        t.lds_pad = pad;
        float ms;
        if ((rc = time_one(t, &ms)) != LTL_OK) goto done;
        if (ms >= 0 && ms < best_ms) { best_ms = ms; best_t = t; }
    }
done:
    clear_graphs(probe);
    s.flow_epoch = probe.flow_epoch;   // the probes advanced the shared round counters
    s.err_seen = probe.err_seen;
    // restore the state the probes started from (also after a failed probe)
    hipError_t re = hipMemcpyAsync(s.buf[s.cur], scratch, bytes, hipMemcpyDeviceToDevice, s.stream);
    if (re == hipSuccess) re = hipStreamSynchronize(s.stream);
    quiet(hipEventDestroy(ev0));
    quiet(hipEventDestroy(ev1));
    if (rc != LTL_OK) return rc;
    if (re != hipSuccess) return hip_fail(re, "autotune restore");
    clear_graphs(s);
    s.tuning = best_t;
    s.user_tuned = true;
    if (best) *best = best_t;
    std::string err;
    if (best_ms < 1e29f && !user_cache_path().empty())
        (void)store_tuning(make_key(s.H, s.W, s.rule, s.method, s.periodic, 0), best_t, best_ms, &err);
    return LTL_OK;
}

int32_t ltl_set_boundary(ltl_sim_t *sim, int32_t boundary) {
    if (!sim) return fail(LTL_ERR_ARG, "sim is NULL");
    if (boundary != LTL_BOUNDARY_DEAD && boundary != LTL_BOUNDARY_PERIODIC) return fail(LTL_ERR_ARG, "unknown boundary");
    if (boundary == LTL_BOUNDARY_PERIODIC && sim->W % 16 != 0)
        return fail(LTL_ERR_UNSUPPORTED, "a periodic grid needs W divisible by 16");
    clear_graphs(*sim);
    const int old_periodic = sim->periodic;
    sim->periodic = (boundary == LTL_BOUNDARY_PERIODIC) ? 1 : 0;
    if (sim->user_tuned) {   // a shape the caller chose must still fit this boundary
        int32_t rc = check_tuning(*sim, sim->tuning);
        if (rc != LTL_OK) {
            sim->periodic = old_periodic;
            return rc;
        }
    }
    // a shape taken from the tuning table follows the boundary's own entry
    if (!sim->user_tuned) return initial_tuning(*sim);
    return LTL_OK;
}

int32_t ltl_run_noalloc(int32_t H, int32_t W, const ltl_rule_t *rule, int32_t method, int32_t boundary,
                        void *buf_a, void *buf_b, size_t buf_bytes, const void *init, size_t init_pitch,
                        int32_t n_steps, void *dst, size_t dst_pitch, hipStream_t stream) {
    if (H < 1 || W < 1) return fail(LTL_ERR_ARG, "H and W must be >= 1");
    if (!buf_a || !buf_b || !init || !dst) return fail(LTL_ERR_ARG, "NULL buffer");
    if (buf_a == buf_b) return fail(LTL_ERR_ARG, "the two buffers must differ");
    if (init_pitch < (size_t)W) return fail(LTL_ERR_ARG, "init_pitch < W");
    if (dst_pitch < (size_t)W) return fail(LTL_ERR_ARG, "dst_pitch < W");
    if (n_steps < 0) return fail(LTL_ERR_ARG, "n_steps must be >= 0");
    if (grid_too_large(H, W)) return fail(LTL_ERR_SIZE, "grid larger than 2^31 - 1 bytes (H x ltl_pitch(W))");
    if (((uintptr_t)buf_a & 255) || ((uintptr_t)buf_b & 255)) return fail(LTL_ERR_ARG, "buffers must be 256-byte aligned");
    if (boundary != LTL_BOUNDARY_DEAD && boundary != LTL_BOUNDARY_PERIODIC) return fail(LTL_ERR_ARG, "unknown boundary");
    if (boundary == LTL_BOUNDARY_PERIODIC && W % 16 != 0)
        return fail(LTL_ERR_UNSUPPORTED, "a periodic grid needs W divisible by 16");
    int32_t rc = validate_rule(rule, method);
    if (rc != LTL_OK) return rc;
    const size_t need = (size_t)H * (size_t)pitch_of(W);
    if (buf_bytes < need) return fail(LTL_ERR_SIZE, "buffers need " + std::to_string(need) + " bytes each");
    {
        ltl_tuning_t t;
        std::string err;
        if (env_tile(&t, &err) < 0) return fail(LTL_ERR_ARG, err);
    }
    uint8_t *sp = nullptr;
    if ((rc = scratch_of_current_device(&sp)) != LTL_OK) return rc;

    // a handle on the stack: host metadata only, constants in the static area, no graphs
    ltl_sim s;
    s.H = H;
    s.W = W;
    s.pitch = pitch_of(W);
    s.rule = *rule;
    s.method = method;
    s.epi = epi_of(*rule, elem_of(method, rule->R, rule->N));
    s.rc = make_consts(*rule, s.epi);
    s.buf[0] = (uint8_t *)buf_a;
    s.buf[1] = (uint8_t *)buf_b;
    s.stream = stream;
    s.dconst = sp;
    s.periodic = (boundary == LTL_BOUNDARY_PERIODIC) ? 1 : 0;
    if ((rc = initial_tuning(s)) != LTL_OK) return rc;
    s.tuning.use_graph = 0;   // plain launches: a graph instantiation allocates
    if (s.tuning.persistent == 2) s.tuning.persistent = 0;   // the dataflow form keeps counters in handle memory

    HIP_TRY(launch_fill_constants(sp, elem_of(method, rule->R, rule->N), rule->R, kConstBytes - kBandBytes, stream),
            "constants kernel launch");
    HIP_TRY(launch_prepare_grids(s.buf[0], s.buf[1], (const uint8_t *)init, init_pitch, H, W, s.pitch, stream),
            "prepare kernel launch");
    if ((rc = do_steps(s, n_steps)) != LTL_OK) return rc;
    HIP_TRY(hipMemcpy2DAsync(dst, dst_pitch, s.buf[s.cur], s.pitch, W, H, hipMemcpyDeviceToDevice, stream),
            "hipMemcpy2DAsync");
    return LTL_OK;
}

int32_t ltl_destroy(ltl_sim_t *sim) {
    if (!sim) return LTL_OK;
    clear_graphs(*sim);
    if (sim->dflag) quiet(hipFree(sim->dflag));
    if (sim->dconst) quiet(hipFree(sim->dconst));
    if (sim->dflow) quiet(hipFree(sim->dflow));
    if (sim->herr) quiet(hipHostFree(sim->herr));
    delete sim;
    return LTL_OK;
}

}  // extern "C"
