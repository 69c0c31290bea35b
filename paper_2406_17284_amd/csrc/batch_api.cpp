// Host side of libltl, batched simulations: per-instance launch descriptors, the cost-sorted
// work list, hipGraph replay and the autotuner of the ltl_batch_* entry points. Every step of
// the automata runs in the kernels of this library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "host_common.h"
#include "ltl.h"
#include "ltl_internal.h"
#include "tuning_cache.h"

using namespace ltl;
using namespace ltl::host;

namespace {

// ---------------------------------------------------------------------- batched simulation

// Device descriptors of the launches that advance every instance by T' steps (T' = 1..T of
// the tuning; the remainder of an n-step call uses a shorter launch).
struct BatchLaunchPlan {
    void *dinst = nullptr;       // BatchInst[2][count] (CAT) or DirectBatchInst[2][count], by source arena
    size_t lds = 0;              // dynamic LDS bytes
    int32_t grid = 0;            // workgroups (one per work-list entry, or the persistent grid)
};

}  // namespace

struct ltl_batch {
    int32_t count = 0;
    int method = 0;
    std::vector<int32_t> H, W, pitch;
    std::vector<ltl_rule_t> rule;
    std::vector<int> epi;
    std::vector<RuleConsts> rc;
    std::vector<size_t> off;         // byte offset of instance i in either arena
    size_t arena_bytes = 0;
    uint8_t *arena[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t steps_done = 0;
    hipStream_t stream = nullptr;
    ltl_tuning_t tuning{};
    bool owns_shared = true;         // false for the autotuner's probe, which borrows the below
    uint8_t *dconst = nullptr;       // band tables for r = 1..16 of the method's element type, zero page
    uint32_t *dflag = nullptr;       // kFlagWords words: [0] initial-state check, [kCounters..] the
                                     // persistent form's counters (zero between launches)
    BatchItem *ditems = nullptr;     // work list of the tuning
    int32_t nitems = 0;
    std::vector<BatchLaunchPlan> plans;
    std::map<std::pair<int32_t, int>, hipGraphExec_t> graphs;
};

namespace {

constexpr int kMaxR = 16;
constexpr int kFlagWords = 32;
constexpr int kCounters = 16;   // 8 per-XCD next-entry counters and the finished-workgroup counter

size_t batch_const_bytes() { return kMaxR * kBandBytes + 4096; }

// Bytes of an instance in an arena: its rows at the library pitch, 256-byte aligned.
size_t arena_slot_bytes(int H, int W) { return ((size_t)H * pitch_of(W) + 255) / 256 * 256; }

// Tile of instance i: the nominal tile grid over the instance, with the tiles shrunk evenly
// (to multiples of 16 rows / 32 columns) so it is covered with the least padding.
void instance_tile(int H, int W, int TH, int TW, int *th, int *tw) {
    const int ny = (H + TH - 1) / TH;
    const int nx = (W + TW - 1) / TW;
    *th = roundup((H + ny - 1) / ny, 16);
    *tw = roundup((W + nx - 1) / nx, 32);
}

CatParams batch_cat_params(const ltl_batch &b, int i, const ltl_tuning_t &t, int T, int from = 0) {
    CatParams p;
    std::memset(&p, 0, sizeof(p));
    p.src = b.arena[from] + b.off[i];
    p.dst = b.arena[from ^ 1] + b.off[i];
    p.H = b.H[i];
    p.W = b.W[i];
    p.pitch = b.pitch[i];
    p.r = b.rule[i].R;
    p.T = T;
    instance_tile(p.H, p.W, t.tile_rows, t.tile_cols, &p.TH, &p.TW);
    p.L = cat_margin(elem_of(b.method, 16, 'M'), p.r, T);
    p.lds_rows = p.TH + 2 * p.L;
    cat_lds_layout(elem_of(b.method, 16, 'M'), b.epi[i], p.TH, p.TW, p.L, t.lds_pad, &p.PS, &p.PA, &p.lds_tile,
                   &p.a_tile, &p.lds_total);
    p.ntx = (p.W + p.TW - 1) / p.TW;
    p.nty = (p.H + p.TH - 1) / p.TH;
    p.bands = reinterpret_cast<const int32_t *>(b.dconst + (p.r - 1) * kBandBytes);
    p.zero = b.dconst + kMaxR * kBandBytes;
    p.periodic = 0;              // batched instances have a dead ghost halo
    p.store_w = p.pitch;
    p.rc = b.rc[i];
    return p;
}

DirectParams batch_direct_params(const ltl_batch &b, int i, int from) {
    DirectParams p;
    std::memset(&p, 0, sizeof(p));
    p.src = b.arena[from] + b.off[i];
    p.dst = b.arena[from ^ 1] + b.off[i];
    p.H = b.H[i];
    p.W = b.W[i];
    p.pitch = b.pitch[i];
    p.r = b.rule[i].R;
    p.TH = direct_tile_rows();
    p.TW = direct_tile_cols();
    p.LP = direct_lds_pitch(p.r);
    p.cross = (b.rule[i].N == 'N') ? 1 : 0;
    p.rc = b.rc[i];
    return p;
}

bool batch_fits(const ltl_batch &b, const ltl_tuning_t &t) {
    for (int i = 0; i < b.count; ++i) {
        int th, tw;
        instance_tile(b.H[i], b.W[i], t.tile_rows, t.tile_cols, &th, &tw);
        if (!cat_shape_fits(elem_of(b.method, 16, 'M'), b.rule[i].R, t.steps_per_launch, th, tw, t.waves)) return false;
    }
    return true;
}

ltl_tuning_t batch_fill_tuning(const ltl_batch &b, const ltl_tuning_t &in) {
    ltl_tuning_t t = in;
    if (t.steps_per_launch == 0) t.steps_per_launch = 1;
    if (t.tile_rows == 0) t.tile_rows = 128;
    if (t.tile_cols == 0) t.tile_cols = 192;
    if (b.method == LTL_DIRECT) {
        t.waves = direct_threads() / 64;
        t.lds_pad = 0;
    } else if (t.waves == 0) {   // fewest waves (power of two) that fit every instance
        t.waves = 1;
        while (t.waves < 8 && !batch_fits(b, t)) t.waves *= 2;
    }
    t.use_graph = t.use_graph ? 1 : 0;
    return t;
}

// Default: one step per launch, 128 x 192 tiles (rows shrunk by 16 at a time until every
// instance's strips x segments fit 8 waves; fp16 holds fewer row blocks per wave).
ltl_tuning_t batch_default_tuning(const ltl_batch &b) {
    ltl_tuning_t t;
    std::memset(&t, 0, sizeof(t));
    t.use_graph = 1;
    t = batch_fill_tuning(b, t);
    if (b.method != LTL_DIRECT) {
        while (t.tile_rows > 16 && !batch_fits(b, t)) {
            t.tile_rows -= 16;
            t.waves = 0;
            t = batch_fill_tuning(b, t);
        }
    }
    return t;
}

size_t batch_cat_lds(const ltl_batch &b, const ltl_tuning_t &t, int T) {
    int32_t m = 0;
    for (int i = 0; i < b.count; ++i) m = std::max(m, batch_cat_params(b, i, t, T).lds_total);
    return (size_t)m;
}

int32_t batch_check_tuning(const ltl_batch &b, const ltl_tuning_t &t) {
    if (t.steps_per_launch < 1 || t.steps_per_launch > 64) return fail(LTL_ERR_ARG, "steps_per_launch must be in 1..64");
    if (t.tile_rows < 16 || t.tile_rows > 512 || t.tile_rows % 16) return fail(LTL_ERR_ARG, "tile_rows must be a multiple of 16 in 16..512");
    if (t.tile_cols < 32 || t.tile_cols > 512 || t.tile_cols % 32) return fail(LTL_ERR_ARG, "tile_cols must be a multiple of 32 in 32..512");
    if (t.persistent < 0 || t.persistent > 1)
        return fail(LTL_ERR_ARG, "batches take persistent 0 (one workgroup per entry) or 1 (resident workgroups)");
    if (t.lds_pad < 0 || t.lds_pad > 128 || t.lds_pad % 16) return fail(LTL_ERR_ARG, "lds_pad must be a multiple of 16 in 0..128");
    if (b.method == LTL_DIRECT) {
        if (t.steps_per_launch != 1) return fail(LTL_ERR_ARG, "the direct method takes one step per launch");
        if (t.persistent) return fail(LTL_ERR_ARG, "the batched direct method has no persistent form");
        return LTL_OK;
    }
    if (t.waves < 1 || t.waves > 8) return fail(LTL_ERR_ARG, "waves must be in 1..8");
    if (!batch_fits(b, t)) return fail(LTL_ERR_ARG, "launch shape has more strip segments than waves for some instance");
    size_t lds = batch_cat_lds(b, t, t.steps_per_launch);
    if (lds > max_lds_bytes()) return fail(LTL_ERR_ARG, "launch shape needs " + std::to_string(lds) + " bytes of LDS");
    if (b.dconst && cat_batch_occupancy(elem_of(b.method, 16, 'M'), t.waves, lds, t.persistent) < 1)
        return fail(LTL_ERR_ARG, "launch shape does not fit on a compute unit (registers or LDS)");
    return LTL_OK;
}

// Executable graphs are destroyed only once the stream has drained: a replay enqueued by an
// earlier step call may still be running.
void batch_clear_graphs(ltl_batch &b) {
    if (b.graphs.empty()) return;
    quiet(hipStreamSynchronize(b.stream));
    for (auto &kv : b.graphs) quiet(hipGraphExecDestroy(kv.second));
    b.graphs.clear();
}

void batch_free_plans(ltl_batch &b) {
    batch_clear_graphs(b);
    if (!b.plans.empty() || b.ditems) quiet(hipStreamSynchronize(b.stream));   // descriptors in use by queued launches
    for (auto &pl : b.plans)
        if (pl.dinst) quiet(hipFree(pl.dinst));
    b.plans.clear();
    if (b.ditems) quiet(hipFree(b.ditems));
    b.ditems = nullptr;
    b.nitems = 0;
}

void batch_release(ltl_batch &b) {
    batch_free_plans(b);
    if (b.owns_shared) {
        if (b.dconst) quiet(hipFree(b.dconst));
        if (b.dflag) quiet(hipFree(b.dflag));
    }
    b.dconst = nullptr;
    b.dflag = nullptr;
}

// Copy a host array to a new device allocation (the copy is complete on return).
template <typename X>
int32_t upload(const std::vector<X> &h, hipStream_t s, void **out) {
    *out = nullptr;
    void *d = nullptr;
    HIP_TRY(hipMalloc(&d, std::max<size_t>(h.size() * sizeof(X), 16)), "hipMalloc");
    hipError_t e = hipMemcpyAsync(d, h.data(), h.size() * sizeof(X), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        quiet(hipFree(d));
        return hip_fail(e, "descriptor upload");
    }
    *out = d;
    return LTL_OK;
}

// Work list of the current tuning: every (instance, tile), most expensive first (workgroups are
// dispatched in entry order). The cost model counts the cells each step of a launch recomputes
// (tile plus its shrinking margin; 16-bit and decay epilogues a little dearer) and a quarter of
// the loaded window.
int32_t batch_prepare(ltl_batch &b) {
    batch_free_plans(b);
    const ltl_tuning_t &t = b.tuning;
    struct Entry {
        double cost;
        BatchItem it;
    };
    std::vector<Entry> list;
    for (int i = 0; i < b.count; ++i) {
        int ntiles;
        double cost;
        const int r = b.rule[i].R;
        if (b.method == LTL_DIRECT) {
            ntiles = ((b.W[i] + direct_tile_cols() - 1) / direct_tile_cols()) * ((b.H[i] + direct_tile_rows() - 1) / direct_tile_rows());
            cost = (double)(2 * r + 1) * (2 * r + 4);
        } else {
            CatParams p = batch_cat_params(b, i, t, t.steps_per_launch);
            ntiles = p.ntx * p.nty;
            cost = 0.25 * (double)(p.TH + 2 * p.L) * (p.TW + 2 * p.L);
            for (int st = 1; st <= p.T; ++st) {
                const int E = roundup(r * (p.T - st), 16);
                cost += (double)(p.TH + 2 * E) * (p.TW + 2 * E) * ((b.epi[i] == EPI_BYTE || b.epi[i] == EPI_WIN || b.epi[i] == EPI_WIN8) ? 1.0 : 1.15);
            }
        }
        for (int k = 0; k < ntiles; ++k) list.push_back({cost, {i, k, b.epi[i], 0}});
    }
    std::stable_sort(list.begin(), list.end(), [](const Entry &x, const Entry &y) { return x.cost > y.cost; });
    std::vector<BatchItem> items;
    items.reserve(list.size());
    for (auto &e : list) items.push_back(e.it);
    // Workgroup k runs on XCD k mod 8. The tiles of one instance are a run of equal cost; within
    // each run, give every XCD a contiguous block of tiles (row-major), so neighbouring tiles
    // share that XCD's L2 and their halo re-reads hit it. The cost order is unchanged.
    for (size_t a = 0; a < items.size();) {
        size_t e = a;
        while (e < items.size() && items[e].inst == items[a].inst) ++e;
        std::vector<size_t> pos;
        for (size_t x = 0; x < 8; ++x)
            for (size_t q = a; q < e; ++q)
                if (q % 8 == (a + x) % 8) pos.push_back(q);
        std::vector<BatchItem> run(items.begin() + a, items.begin() + e);
        std::sort(run.begin(), run.end(), [](const BatchItem &x, const BatchItem &y) { return x.tile < y.tile; });
        for (size_t t = 0; t < run.size(); ++t) items[pos[t]] = run[t];
        a = e;
    }
    void *d = nullptr;
    int32_t rc = upload(items, b.stream, &d);
    if (rc != LTL_OK) return rc;
    b.ditems = (BatchItem *)d;
    b.nitems = (int32_t)items.size();
    b.plans.assign(b.method == LTL_DIRECT ? 1 : t.steps_per_launch, BatchLaunchPlan());
    return LTL_OK;
}

int32_t batch_plan(ltl_batch &b, int T, BatchLaunchPlan **out) {
    BatchLaunchPlan &pl = b.plans[T - 1];
    if (!pl.dinst) {
        if (b.method == LTL_DIRECT) {
            std::vector<DirectBatchInst> h(2 * b.count);
            size_t lds = 0;
            for (int par = 0; par < 2; ++par)
                for (int i = 0; i < b.count; ++i) {
                    DirectBatchInst &x = h[par * b.count + i];
                    std::memset(&x, 0, sizeof(x));
                    x.p = batch_direct_params(b, i, par);
                    x.ntx = (b.W[i] + direct_tile_cols() - 1) / direct_tile_cols();
                    lds = std::max(lds, direct_lds_bytes(x.p.r));
                }
            int32_t rc = upload(h, b.stream, &pl.dinst);
            if (rc != LTL_OK) return rc;
            pl.lds = lds;
            pl.grid = b.nitems;
        } else {
            std::vector<BatchInst> h(2 * b.count);
            for (int par = 0; par < 2; ++par)
                for (int i = 0; i < b.count; ++i) {
                    BatchInst &x = h[par * b.count + i];
                    std::memset(&x, 0, sizeof(x));
                    x.p = batch_cat_params(b, i, b.tuning, T, par);
                }
            pl.lds = batch_cat_lds(b, b.tuning, T);
            const int occ = cat_batch_occupancy(elem_of(b.method, 16, 'M'), b.tuning.waves, pl.lds, b.tuning.persistent);
            if (occ < 1) return fail(LTL_ERR_ARG, "batched launch does not fit on a compute unit");
            pl.grid = b.nitems;
            if (b.tuning.persistent) {   // resident workgroups, a multiple of 8 (one run per XCD)
                int dev = 0, cus = 0;
                if (hipGetDevice(&dev) != hipSuccess ||
                    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
                    (void)hipGetLastError();
                    cus = 8;
                }
                pl.grid = std::min(roundup(b.nitems, 8), roundup(occ * cus, 8));
            }
            int32_t rc = upload(h, b.stream, &pl.dinst);
            if (rc != LTL_OK) return rc;
        }
    }
    *out = &pl;
    return LTL_OK;
}

// Kernel node of one launch advancing every instance by T steps from arena `from`.
struct BatchLaunch {
    const void *func;
    dim3 grid, block;
    size_t lds;
    BatchParams bp;
    DirectBatchParams dp;
    bool direct;
    void *arg() { return direct ? (void *)&dp : (void *)&bp; }
};

int32_t batch_launch(ltl_batch &b, int T, int from, BatchLaunch *l) {
    BatchLaunchPlan *pl = nullptr;
    int32_t rc = batch_plan(b, T, &pl);
    if (rc != LTL_OK) return rc;
    std::memset(l, 0, sizeof(*l));
    l->direct = (b.method == LTL_DIRECT);
    l->lds = pl->lds;
    l->grid = dim3((unsigned)pl->grid, 1, 1);
    if (l->direct) {
        l->func = direct_batch_func();
        l->block = dim3((unsigned)direct_threads(), 1, 1);
        l->dp.inst = (const DirectBatchInst *)pl->dinst + from * b.count;
        l->dp.items = b.ditems;
        l->dp.nitems = b.nitems;
    } else {
        l->func = cat_batch_func(elem_of(b.method, 16, 'M'), b.tuning.persistent);
        l->block = dim3((unsigned)(64 * b.tuning.waves), 1, 1);
        l->bp.inst = (const BatchInst *)pl->dinst + from * b.count;
        l->bp.items = b.ditems;
        l->bp.counters = b.dflag + kCounters;
        l->bp.nitems = b.nitems;
    }
    if (l->lds > 65536)
        HIP_TRY(hipFuncSetAttribute(l->func, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l->lds), "hipFuncSetAttribute");
    return LTL_OK;
}

std::vector<int> batch_sizes(const ltl_batch &b, int n) {
    std::vector<int> v;
    const int T = (b.method == LTL_DIRECT) ? 1 : b.tuning.steps_per_launch;
    while (n > 0) {
        const int t = std::min(T, n);
        v.push_back(t);
        n -= t;
    }
    return v;
}

int32_t batch_build_graph(ltl_batch &b, int n, hipGraphExec_t *out) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipGraphCreate(&g, 0), "hipGraphCreate");
    hipGraphNode_t prev = nullptr;
    int from = b.cur;
    for (int T : batch_sizes(b, n)) {
        BatchLaunch l;
        int32_t rc = batch_launch(b, T, from, &l);
        if (rc != LTL_OK) { quiet(hipGraphDestroy(g)); return rc; }
        hipKernelNodeParams kp;
        std::memset(&kp, 0, sizeof(kp));
        void *args[1] = {l.arg()};
        kp.func = const_cast<void *>(l.func);
        kp.gridDim = l.grid;
        kp.blockDim = l.block;
        kp.sharedMemBytes = (unsigned)l.lds;
        kp.kernelParams = args;
        hipGraphNode_t node;
        hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
        if (e != hipSuccess) { quiet(hipGraphDestroy(g)); return hip_fail(e, "hipGraphAddKernelNode"); }
        prev = node;
        from ^= 1;
    }
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    quiet(hipGraphDestroy(g));
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    *out = ex;
    return LTL_OK;
}

int32_t batch_chunk(ltl_batch &b, int32_t n) {
    std::vector<int> sizes = batch_sizes(b, n);
    if (b.tuning.use_graph && sizes.size() > 1) {
        auto key = std::make_pair(n, b.cur);
        auto it = b.graphs.find(key);
        hipGraphExec_t ex = nullptr;
        if (it == b.graphs.end()) {
            if (b.graphs.size() >= 32) batch_clear_graphs(b);
            int32_t rc = batch_build_graph(b, n, &ex);
            if (rc != LTL_OK) return rc;
            b.graphs[key] = ex;
        } else {
            ex = it->second;
        }
        HIP_TRY(hipGraphLaunch(ex, b.stream), "hipGraphLaunch");
        b.cur ^= (int)(sizes.size() & 1);
    } else {
        for (int T : sizes) {
            BatchLaunch l;
            int32_t rc = batch_launch(b, T, b.cur, &l);
            if (rc != LTL_OK) return rc;
            void *args[1] = {l.arg()};
            HIP_TRY(hipLaunchKernel(l.func, l.grid, l.block, args, l.lds, b.stream), "kernel launch");
            b.cur ^= 1;
        }
    }
    b.steps_done += n;
    return LTL_OK;
}

int32_t batch_steps(ltl_batch &b, int32_t n) {
    const int T = (b.method == LTL_DIRECT) ? 1 : b.tuning.steps_per_launch;
    const int32_t chunk = T * kMaxChunkLaunches;
    while (n > 0) {
        const int32_t m = std::min(n, chunk);
        int32_t rc = batch_chunk(b, m);
        if (rc != LTL_OK) return rc;
        n -= m;
    }
    return LTL_OK;
}

// Key of the batch in the tuning table: its total cells and largest radius.
TuneKey batch_key(const ltl_batch &b) {
    double cells = 0;
    int rmax = 1;
    for (int i = 0; i < b.count; ++i) {
        cells += (double)b.H[i] * b.W[i];
        rmax = std::max(rmax, (int)b.rule[i].R);
    }
    ltl_rule_t r = b.rule[0];
    r.R = rmax;
    TuneKey k = make_key(1, 1, r, b.method, LTL_BOUNDARY_DEAD, 1);
    k.bucket = size_bucket(cells);
    return k;
}

// Launch shape of a new batch: LTL_TILE if set (refused if malformed or infeasible), else the
// first feasible tuning-table candidate, else the built-in default.
int32_t batch_initial_tuning(ltl_batch &b, ltl_tuning_t *out) {
    ltl_tuning_t t;
    std::string err;
    const int env = env_tile(&t, &err);
    if (env < 0) return fail(LTL_ERR_ARG, err);
    if (env > 0) {
        if (b.method == LTL_DIRECT) t.steps_per_launch = 1;
        t.persistent = 0;
        t = batch_fill_tuning(b, t);
        if (batch_check_tuning(b, t) != LTL_OK) return fail(LTL_ERR_ARG, "LTL_TILE: " + g_err);
        *out = t;
        return LTL_OK;
    }
    const SavedError saved = save_error();
    for (ltl_tuning_t c : tuning_candidates(batch_key(b), nullptr)) {
        c = batch_fill_tuning(b, c);
        if (batch_check_tuning(b, c) == LTL_OK) {
            *out = c;
            restore_error(saved);
            return LTL_OK;
        }
    }
    restore_error(saved);
    *out = batch_default_tuning(b);
    return batch_check_tuning(b, *out);
}

// Time candidate launch shapes on the batch's own arenas (the current state saved in the
// caller's scratch and restored before each candidate and at the end); keep the fastest.
int32_t batch_autotune(ltl_batch &b, int probe_steps, void *scratch, size_t scratch_bytes, ltl_tuning_t *best) {
    if (b.method == LTL_DIRECT) {
        if (best) *best = b.tuning;
        return LTL_OK;
    }
    if (!scratch) return fail(LTL_ERR_ARG, "scratch is NULL");
    if (scratch_bytes < b.arena_bytes) return fail(LTL_ERR_SIZE, "scratch needs " + std::to_string(b.arena_bytes) + " bytes");
    if (scratch == b.arena[0] || scratch == b.arena[1]) return fail(LTL_ERR_ARG, "scratch must not be one of the arenas");
    HIP_TRY(hipMemcpyAsync(scratch, b.arena[b.cur], b.arena_bytes, hipMemcpyDeviceToDevice, b.stream), "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(b.stream), "hipStreamSynchronize");
    ltl_batch probe;
    probe.count = b.count; probe.method = b.method; probe.H = b.H; probe.W = b.W; probe.pitch = b.pitch;
    probe.rule = b.rule; probe.epi = b.epi; probe.rc = b.rc; probe.off = b.off; probe.arena_bytes = b.arena_bytes;
    probe.stream = b.stream; probe.owns_shared = false;
    probe.dconst = b.dconst; probe.dflag = b.dflag;
    probe.arena[0] = b.arena[0];
    probe.arena[1] = b.arena[1];
    hipEvent_t ev0, ev1;
    HIP_TRY(hipEventCreate(&ev0), "hipEventCreate");
    if (hipEventCreate(&ev1) != hipSuccess) { quiet(hipEventDestroy(ev0)); return fail(LTL_ERR_HIP, "hipEventCreate"); }
    float best_ms = 1e30f;
    ltl_tuning_t best_t = b.tuning;
    int32_t rc = LTL_OK;
    auto time_one = [&](ltl_tuning_t t, float *ms_out) -> int32_t {
        *ms_out = -1.f;
        t = batch_fill_tuning(probe, t);
        const SavedError saved = save_error();
        if (batch_check_tuning(probe, t) != LTL_OK) { restore_error(saved); return LTL_OK; }
        // each candidate runs a whole number of its own launches (no shorter remainder launch
        // to bias it) covering at least probe_steps steps; candidates compare per step
        const int T = t.steps_per_launch;
        const int n = T * ((probe_steps + T - 1) / T);
        probe.tuning = t;
        int32_t r2 = batch_prepare(probe);
        if (r2 != LTL_OK) return r2;
        HIP_TRY(hipMemcpyAsync(b.arena[b.cur], scratch, b.arena_bytes, hipMemcpyDeviceToDevice, b.stream), "hipMemcpyAsync");
        probe.cur = b.cur;
        if ((r2 = batch_steps(probe, n)) != LTL_OK) return r2;   // warm-up + graph build
        float ms = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {   // the faster of two timed runs
            HIP_TRY(hipEventRecord(ev0, b.stream), "hipEventRecord");
            if ((r2 = batch_steps(probe, n)) != LTL_OK) return r2;
            HIP_TRY(hipEventRecord(ev1, b.stream), "hipEventRecord");
            HIP_TRY(hipEventSynchronize(ev1), "autotune sync");
            float m = 0;
            HIP_TRY(hipEventElapsedTime(&m, ev0, ev1), "hipEventElapsedTime");
            ms = std::min(ms, m);
        }
        *ms_out = ms / (float)n;
        return LTL_OK;
    };
    const int Ts[] = {1, 2, 3, 4};
    const int tiles[][2] = {{64, 64}, {64, 128}, {128, 128}, {128, 192}, {192, 128}, {128, 224}, {160, 160},
                            {192, 192}, {160, 224}, {176, 224}};
    const int wavess[] = {0, 8};
    for (int T : Ts)
        for (auto &tl : tiles)
            for (int wv : wavess)
                for (int pers = 0; pers < 2; ++pers) {
                    ltl_tuning_t t;
                    std::memset(&t, 0, sizeof(t));
                    t.steps_per_launch = T; t.tile_rows = tl[0]; t.tile_cols = tl[1]; t.waves = wv; t.use_graph = 1;
                    t.persistent = pers;
                    float ms;
                    if ((rc = time_one(t, &ms)) != LTL_OK) goto done;
                    if (ms >= 0 && ms < best_ms) { best_ms = ms; best_t = batch_fill_tuning(probe, t); }
                }
    for (int pad : {16, 32, 64}) {
        ltl_tuning_t t = best_t;
        t.lds_pad = pad;
        float ms;
        if ((rc = time_one(t, &ms)) != LTL_OK) goto done;
        if (ms >= 0 && ms < best_ms) { best_ms = ms; best_t = t; }
    }
done:
    {
        hipError_t re = hipMemcpyAsync(b.arena[b.cur], scratch, b.arena_bytes, hipMemcpyDeviceToDevice, b.stream);
        if (re == hipSuccess) re = hipStreamSynchronize(b.stream);
        batch_release(probe);
        quiet(hipEventDestroy(ev0));
        quiet(hipEventDestroy(ev1));
        if (rc != LTL_OK) return rc;
        if (re != hipSuccess) return hip_fail(re, "autotune restore");
    }
    b.tuning = best_t;
    if ((rc = batch_prepare(b)) != LTL_OK) return rc;
    if (best) *best = best_t;
    std::string err;
    if (best_ms < 1e29f && !user_cache_path().empty()) (void)store_tuning(batch_key(b), best_t, best_ms, &err);
    return LTL_OK;
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------------- batched API
size_t ltl_batch_buffer_bytes(int32_t count, const int32_t *H, const int32_t *W) {
    if (!H || !W || count < 1) { fail(LTL_ERR_ARG, "count must be >= 1 and arrays non-NULL"); return 0; }
    size_t total = 0;
    for (int i = 0; i < count; ++i) {
        if (H[i] < 1 || W[i] < 1) { fail(LTL_ERR_ARG, "every H and W must be >= 1"); return 0; }
        total += arena_slot_bytes(H[i], W[i]);
    }
    return total;
}

int32_t ltl_batch_create(ltl_batch_t **out, int32_t count, const int32_t *H, const int32_t *W,
                         const ltl_rule_t *rules, int32_t method, void *arena_a, void *arena_b,
                         size_t bytes, const void *const *init, const size_t *init_pitch,
                         hipStream_t stream) {
    if (!out) return fail(LTL_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1 || !H || !W || !rules || !init || !init_pitch) return fail(LTL_ERR_ARG, "count must be >= 1 and arrays non-NULL");
    if (!arena_a || !arena_b) return fail(LTL_ERR_ARG, "NULL arena");
    if (arena_a == arena_b) return fail(LTL_ERR_ARG, "the two arenas must differ");
    if (((uintptr_t)arena_a & 255) || ((uintptr_t)arena_b & 255)) return fail(LTL_ERR_ARG, "arenas must be 256-byte aligned");
    const size_t need = ltl_batch_buffer_bytes(count, H, W);
    if (need == 0) return LTL_ERR_ARG;
    int32_t rc = LTL_OK;
    for (int i = 0; i < count; ++i) {
        if ((rc = validate_rule(rules + i, method)) != LTL_OK) return fail(rc, "instance " + std::to_string(i) + ": " + g_err);
        if (method != LTL_DIRECT && rules[i].R > 16)
            return fail(LTL_ERR_UNSUPPORTED, "instance " + std::to_string(i) + ": batched CAT covers radii 1..16");
        if (method != LTL_DIRECT && rules[i].N != 'M')
            return fail(LTL_ERR_UNSUPPORTED, "instance " + std::to_string(i) + ": batched CAT covers the Moore neighbourhood");
        if (!init[i]) return fail(LTL_ERR_ARG, "instance " + std::to_string(i) + ": NULL initial grid");
        if (init_pitch[i] < (size_t)W[i]) return fail(LTL_ERR_ARG, "instance " + std::to_string(i) + ": init_pitch < W");
        if (grid_too_large(H[i], W[i]))
            return fail(LTL_ERR_SIZE, "instance " + std::to_string(i) + ": grid larger than 2^31 - 1 bytes");
    }
    if (bytes < need) return fail(LTL_ERR_SIZE, "arenas need " + std::to_string(need) + " bytes each");
    {
        ltl_tuning_t t;
        std::string err;
        if (env_tile(&t, &err) < 0) return fail(LTL_ERR_ARG, err);   // malformed LTL_TILE, before any device work
    }

    ltl_batch *b = new (std::nothrow) ltl_batch();
    if (!b) return fail(LTL_ERR_ARG, "out of host memory");
    b->count = count;
    b->method = method;
    b->stream = stream;
    b->arena[0] = (uint8_t *)arena_a;
    b->arena[1] = (uint8_t *)arena_b;
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        b->H.push_back(H[i]);
        b->W.push_back(W[i]);
        b->pitch.push_back(pitch_of(W[i]));
        b->rule.push_back(rules[i]);
        b->epi.push_back(epi_of(rules[i], elem_of(b->method, rules[i].R, rules[i].N)));
        b->rc.push_back(make_consts(rules[i], b->epi.back()));
        b->off.push_back(off);
        off += arena_slot_bytes(H[i], W[i]);
    }
    b->arena_bytes = off;

    auto bail = [&](int32_t code) {
        batch_release(*b);
        delete b;
        return code;
    };
    hipError_t e;
    const size_t cbytes = batch_const_bytes();
    if ((e = hipMalloc(&b->dconst, cbytes)) != hipSuccess) { b->dconst = nullptr; return bail(hip_fail(e, "hipMalloc")); }
    if ((e = hipMalloc(&b->dflag, kFlagWords * sizeof(uint32_t))) != hipSuccess) { b->dflag = nullptr; return bail(hip_fail(e, "hipMalloc")); }
    {
        std::vector<uint8_t> hc(cbytes, 0);
        if (method != LTL_DIRECT)
            for (int r = 1; r <= kMaxR; ++r)
                band_table(elem_of(method, 16, 'M'), r, reinterpret_cast<int32_t *>(hc.data() + (r - 1) * kBandBytes));
        if ((e = hipMemcpyAsync(b->dconst, hc.data(), cbytes, hipMemcpyHostToDevice, stream)) != hipSuccess)
            return bail(hip_fail(e, "hipMemcpyAsync"));
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return bail(hip_fail(e, "hipStreamSynchronize"));
    }
    if ((e = hipMemsetAsync(b->dflag, 0, kFlagWords * sizeof(uint32_t), stream)) != hipSuccess) return bail(hip_fail(e, "hipMemsetAsync"));
    for (int i = 0; i < count; ++i)
        if ((e = launch_validate((const uint8_t *)init[i], H[i], W[i], init_pitch[i], b->rc[i].C, b->dflag, stream)) != hipSuccess)
            return bail(hip_fail(e, "validate launch"));
    uint32_t bad = 0;
    if ((e = hipMemcpyAsync(&bad, b->dflag, sizeof(bad), hipMemcpyDeviceToHost, stream)) != hipSuccess) return bail(hip_fail(e, "hipMemcpyAsync"));
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return bail(hip_fail(e, "hipStreamSynchronize"));
    if (bad) return bail(fail(LTL_ERR_STATE, "an initial grid holds a state >= max(C, 2) of its rule"));
    for (int a = 0; a < 2; ++a)
        if ((e = hipMemsetAsync(b->arena[a], 0, b->arena_bytes, stream)) != hipSuccess) return bail(hip_fail(e, "hipMemsetAsync"));
    for (int i = 0; i < count; ++i)
        if ((e = hipMemcpy2DAsync(b->arena[0] + b->off[i], b->pitch[i], init[i], init_pitch[i], W[i], H[i],
                                  hipMemcpyDeviceToDevice, stream)) != hipSuccess)
            return bail(hip_fail(e, "hipMemcpy2DAsync"));
    ltl_tuning_t t;
    if ((rc = batch_initial_tuning(*b, &t)) != LTL_OK) return bail(rc);
    b->tuning = t;
    if ((rc = batch_prepare(*b)) != LTL_OK) return bail(rc);
    *out = b;
    return LTL_OK;
}

int32_t ltl_batch_step(ltl_batch_t *batch, int32_t n_steps) {
    if (!batch) return fail(LTL_ERR_ARG, "batch is NULL");
    if (n_steps < 0) return fail(LTL_ERR_ARG, "n_steps must be >= 0");
    return batch_steps(*batch, n_steps);
}

int32_t ltl_batch_read(ltl_batch_t *batch, int32_t index, void *dst, size_t dst_pitch) {
    if (!batch || !dst) return fail(LTL_ERR_ARG, "NULL argument");
    if (index < 0 || index >= batch->count) return fail(LTL_ERR_ARG, "index out of range");
    if (dst_pitch < (size_t)batch->W[index]) return fail(LTL_ERR_ARG, "dst_pitch < W");
    HIP_TRY(hipMemcpy2DAsync(dst, dst_pitch, batch->arena[batch->cur] + batch->off[index], batch->pitch[index],
                             batch->W[index], batch->H[index], hipMemcpyDeviceToDevice, batch->stream),
            "hipMemcpy2DAsync");
    return LTL_OK;
}

int32_t ltl_batch_current(ltl_batch_t *batch, int32_t index, void **buf, size_t *pitch, int64_t *steps_done) {
    if (!batch) return fail(LTL_ERR_ARG, "batch is NULL");
    if (index < 0 || index >= batch->count) return fail(LTL_ERR_ARG, "index out of range");
    if (buf) *buf = batch->arena[batch->cur] + batch->off[index];
    if (pitch) *pitch = (size_t)batch->pitch[index];
    if (steps_done) *steps_done = batch->steps_done;
    return LTL_OK;
}

int32_t ltl_batch_get_tuning(ltl_batch_t *batch, ltl_tuning_t *tuning) {
    if (!batch || !tuning) return fail(LTL_ERR_ARG, "NULL argument");
    *tuning = batch->tuning;
    return LTL_OK;
}

int32_t ltl_batch_set_tuning(ltl_batch_t *batch, const ltl_tuning_t *tuning) {
    if (!batch || !tuning) return fail(LTL_ERR_ARG, "NULL argument");
    ltl_tuning_t t = batch_fill_tuning(*batch, *tuning);
    int32_t rc = batch_check_tuning(*batch, t);
    if (rc != LTL_OK) return rc;
    HIP_TRY(hipStreamSynchronize(batch->stream), "hipStreamSynchronize");   // plans in use by queued launches
    batch->tuning = t;
    return batch_prepare(*batch);
}

int32_t ltl_batch_autotune(ltl_batch_t *batch, int32_t probe_steps, void *scratch, size_t scratch_bytes,
                           ltl_tuning_t *best) {
    if (!batch) return fail(LTL_ERR_ARG, "batch is NULL");
    if (probe_steps < 1 || probe_steps > 4096) return fail(LTL_ERR_ARG, "probe_steps must be in 1..4096");
    return batch_autotune(*batch, probe_steps, scratch, scratch_bytes, best);
}

int32_t ltl_batch_destroy(ltl_batch_t *batch) {
    if (!batch) return LTL_OK;
    batch_release(*batch);
    delete batch;
    return LTL_OK;
}

}  // extern "C"
