/*
 * ltl.h -- C ABI of libltl: Larger-than-Life stepping on one MI355X (gfx950).
 *
 * The library advances cellular automata of the Larger-than-Life family,
 * R_r C_c M_m S_{s1..s2} B_{b1..b2} N_n (paper: "Chosen CA tests", rule notation),
 * on a uint8 grid with a dead ghost halo or on a torus. The Moore neighbourhood count
 * of every cell is the band-matrix reduction of "Formulation of CAT" (Eq. 2-3:
 * H = Lambda Pi, R = Pi H, Pi the band of ones of half-width r) and the cross count
 * its simplified Von Neumann form (Eq. 4: Pi Lambda + H), computed per grid tile on
 * int8 MFMA with int32 accumulation (exact), followed in the same kernel by
 * the birth / survival / decay transition (Algorithm 1, per-thread rule after the
 * reductions). The ping-pong update of "Pseudocode of CAT's Kernel" is kept: two
 * caller-owned buffers swap roles every step.
 *
 * Conventions for every function below:
 *  - All device pointers are HIP device memory on the current device. The caller
 *    (for instance PyTorch) allocates and frees them; the library never frees them.
 *  - Work is enqueued asynchronously on the stream given at creation; synchronize
 *    that stream before reading results on the host or freeing the buffers.
 *  - Return value: LTL_OK (0) or a negative LTL_ERR_* code; ltl_last_error() then
 *    holds a message (thread-local, valid until the next call on the thread).
 *  - Handles are not thread-safe: one thread uses one handle at a time.
 */
#ifndef LTL_H
#define LTL_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LTL_OK = 0,
    LTL_ERR_ARG = -1,         /* null pointer, size < 1, pitch < width, bad tuning value */
    LTL_ERR_RULE = -2,        /* R outside 1..32, C == 1 or > 255, M not 0/1, threshold < 0 or > (2R+1)^2 */
    LTL_ERR_UNSUPPORTED = -3, /* N not 'M'/'N'; a method/radius/neighbourhood combination not built
                                 (fp16 above R = 16, cross on fp16/fp8 or above R = 16 for CAT,
                                 batched CAT above R = 16 or with the cross); periodic W % 16 != 0 */
    LTL_ERR_INEXACT = -4,     /* FP8 method with 2R+1 > 16: counts would not be exact in e4m3 */
    LTL_ERR_SIZE = -5,        /* buffer smaller than ltl_buffer_bytes(), or grid over 2^31 - 1 bytes */
    LTL_ERR_HIP = -6,         /* HIP runtime error (message in ltl_last_error) */
    LTL_ERR_STATE = -7        /* an initial cell holds a state >= max(C, 2) */
};

/* An LTL rule (paper, "Chosen CA tests"). N is the character 'M' (77) for the Moore box
 * of (2R+1)^2 cells or 'N' (78) for the paper's simplified Von Neumann neighbourhood (Eq. 4):
 * the cross of the cell's row and column, 4R+1 cells. The diamond-shaped Von Neumann
 * neighbourhood is not offered (the paper's CAT does not support it either).
 * Radii: int8 CAT and the direct stencil 1..32 (cross: CAT 1..16, direct 1..32), fp16 1..16,
 * fp8 1..7.
 * C = 0 or 2: two states. C >= 3: states 2..C-1 are decay states (a surviving-range
 * miss sends an alive cell to 2, decay advances by one per step and wraps to 0;
 * decaying cells are neither alive nor born). M = 1 counts the centre cell itself.
 * S and B are inclusive ranges of the count; s1 > s2 (or b1 > b2) is an empty range. */
typedef struct {
    int32_t R, C, M, S1, S2, B1, B2, N;
} ltl_rule_t;

/* How the neighbourhood count is computed; all give bit-identical grids. */
typedef enum {
    LTL_CAT_I8 = 0,  /* band products on int8 MFMA (v_mfma_i32_16x16x64_i8; R > 16 adds 16x16x32), int32 accumulate */
    LTL_CAT_F16 = 1, /* band products on fp16 MFMA, fp32 accumulate (exact: counts <= 1089 < 2^11) */
    LTL_CAT_F8 = 2,  /* band products on fp8-e4m3 MFMA, fp32 accumulate; only 2R+1 <= 16 */
    LTL_DIRECT = 3   /* comparison method: LDS tile + direct sum over the neighbourhood per cell */
} ltl_method_t;

/* Launch shape. Zero fields mean "library default". The result never depends on it. The
 * direct method runs fixed 128 x 256 tiles, one step per launch: it checks tile_rows, tile_cols
 * and waves against the ranges below but does not use them; only use_graph applies to it. */
typedef struct {
    int32_t steps_per_launch; /* T >= 1 time steps fused in one kernel launch (temporal blocking) */
    int32_t tile_rows;        /* output rows per workgroup: multiple of 16, 16..512 */
    int32_t tile_cols;        /* output columns per workgroup: multiple of 32, 32..512 */
    int32_t waves;            /* 64-lane waves per workgroup: 1..8 (CAT; the direct method accepts 1..16) */
    int32_t use_graph;        /* 1: replay multi-launch loops from a cached hipGraph */
    int32_t persistent;       /* CAT methods, single grid: 1 = persistent workgroups (about one per
                                 CU slot) that each walk a contiguous run of tiles, loading tile
                                 i+1 into a second LDS buffer while tile i computes (pays off when
                                 tiles stream from HBM); 0 = one workgroup per tile and launch;
                                 2 = dataflow form: one cooperative launch per step call runs all
                                 rounds of T steps, one resident workgroup per tile, and a tile
                                 starts a round once the tiles its window overlaps finished the
                                 previous one (per-tile round counters instead of a kernel
                                 boundary). It needs every tile resident at once (at most 4096
                                 tiles), a margin no wider than the tile, and on a torus partial
                                 edge tiles at least that wide; a wait that runs out (after
                                 LTL_FLOW_SPIN_LIMIT polls, default 2^24) makes the next ltl_step
                                 or ltl_read return LTL_ERR_HIP. Batches (CAT methods) take
                                 0 = one workgroup per work-list entry and launch, or
                                 1 = resident workgroups (a multiple of 8, at most the
                                 co-resident slots) that draw entries from per-XCD counters
                                 in the handle's memory; the batched direct method takes 0. */
    int32_t lds_pad;          /* CAT methods: extra bytes per LDS tile row, a multiple of 16 in 0..128;
                                 it moves the LDS bank each row starts in (the direct method ignores it) */
} ltl_tuning_t;

typedef enum {
    LTL_BOUNDARY_DEAD = 0,
    LTL_BOUNDARY_PERIODIC = 1
} ltl_boundary_t;

typedef struct ltl_sim ltl_sim_t;
typedef struct ltl_batch ltl_batch_t;

/* Bytes of EACH of the two ping-pong buffers of an H x W grid ("Pseudocode of CAT's Kernel":
 * the step reads one buffer and writes the other). Layout: H rows of ltl_pitch(W) bytes, one
 * state per byte; the ghost halo of "Formulation of CAT" is not stored (tile loads read dead
 * cells, or the opposite edge on a torus, for positions outside the grid), so the size does
 * not depend on R or the method, which are checked (R in 1..32, a known method) all the same.
 * Returns 0 on an invalid argument (ltl_last_error and ltl_last_error_code say why). */
size_t ltl_buffer_bytes(int32_t H, int32_t W, int32_t R, int32_t method);

/* Row pitch in bytes of the library's grid layout: W rounded up to 64. LTL_ERR_ARG for W < 1. */
int32_t ltl_pitch(int32_t W, int32_t *pitch);

/* Create a simulation of an H x W grid under an LTL rule ("Chosen CA tests": rule notation
 * R, C, M, S, B, N; "Experimental Design": the random initial grids it starts from).
 *  rule       host pointer, copied.
 *  method     an ltl_method_t (CAT: "Formulation of CAT"; direct: the SHARED scheme of
 *             "Approaches Selected for Evaluation").
 *  buf_a/b    two device buffers of buf_bytes >= ltl_buffer_bytes(H, W, R, method) each, 256-byte
 *             aligned; owned by the caller, their contents owned by the library until ltl_destroy.
 *  init       device pointer to H rows of W uint8 states, row pitch init_pitch >= W bytes;
 *             read before ltl_create returns. Every state must be < max(C, 2) (else LTL_ERR_STATE).
 *  stream     HIP stream for all work of this handle (0 = null stream).
 * The launch shape starts as the tuning table's entry for this rule class, radius, grid size
 * and boundary (ltl_tuning_lookup; the environment variable LTL_TILE =
 * "T,rows,cols,waves[,persistent[,lds_pad]]" overrides it, and a malformed or infeasible
 * LTL_TILE is refused with LTL_ERR_ARG), else a built-in default.
 * A grid may hold at most 2^31 - 1 bytes in the library layout (H x ltl_pitch(W); e.g. up to
 * 46340 x 46340 cells); larger grids are refused with LTL_ERR_SIZE. The handle allocates only
 * host metadata, cached hipGraphs and a 12 KiB device block (band operands and a zero page).
 * ltl_create synchronizes `stream` once (state validation); later calls do not. */
int32_t ltl_create(ltl_sim_t **out, int32_t H, int32_t W, const ltl_rule_t *rule, int32_t method,
                   void *buf_a, void *buf_b, size_t buf_bytes, const void *init, size_t init_pitch,
                   hipStream_t stream);

/* Enqueue n_steps >= 0 synchronous steps (Algorithm 1 per tile: the two band products of
 * Eq. 2-3 and the transition, ping-pong between the buffers). ltl_step(a); ltl_step(b) equals
 * ltl_step(a + b) cell for cell. With use_graph, the steps run as replays of cached hipGraphs
 * of at most 64 launches each (steps_per_launch x 64 steps); the first call with a new length
 * builds them. */
int32_t ltl_step(ltl_sim_t *sim, int32_t n_steps);

/* Enqueue a copy of the current H x W states ("Pseudocode of CAT's Kernel": the buffer the last
 * step wrote) into device memory dst (row pitch dst_pitch >= W). */
int32_t ltl_read(ltl_sim_t *sim, void *dst, size_t dst_pitch);

/* Device buffer holding the current state in the library layout (H rows of *pitch bytes;
 * columns W..pitch-1 are always 0), and the number of steps taken so far. */
int32_t ltl_current(ltl_sim_t *sim, void **buf, size_t *pitch, int64_t *steps_done);

/* Current launch shape ("Optimal Tile per CUDA block": the tile a workgroup computes), and
 * replacing it (validated; LTL_ERR_ARG on an invalid field). set_tuning synchronizes the
 * stream before it drops the cached graphs. */
int32_t ltl_get_tuning(ltl_sim_t *sim, ltl_tuning_t *tuning);
int32_t ltl_set_tuning(ltl_sim_t *sim, const ltl_tuning_t *tuning);

/* Time candidate launch shapes on this simulation ("Optimal Tile per CUDA block": the tile
 * shape is chosen by measurement) and keep the fastest per step; *best (may be NULL) receives
 * it. The probes run on the handle's own ping-pong buffers: the current state is first copied
 * into `scratch` (caller-owned device memory of scratch_bytes >= ltl_buffer_bytes(...), not
 * one of the two buffers; LTL_ERR_SIZE if smaller), every candidate starts from that copy, and
 * the state is restored from it at the end, so the simulation does not advance. Each
 * candidate runs the whole number of its own launches that covers at least probe_steps steps
 * (1..4096). The pick is also stored in the user tuning cache (ltl_tuning_store). Allocates
 * no device memory; synchronizes the stream. */
int32_t ltl_autotune(ltl_sim_t *sim, int32_t probe_steps, void *scratch, size_t scratch_bytes,
                     ltl_tuning_t *best);

/* Boundary condition of the grid (default LTL_BOUNDARY_DEAD).
 *  LTL_BOUNDARY_DEAD      ghost halo of dead cells ("Formulation of CAT"): every cell outside the
 *                         grid is 0 forever.
 *  LTL_BOUNDARY_PERIODIC  the grid is a torus (the paper's experimental setting, "Experimental
 *                         Design"): the box of a cell wraps around both edges, offset (di, dj)
 *                         reaching cell ((i + di) mod H, (j + dj) mod W); on a torus smaller
 *                         than the box a cell is counted once per offset that reaches it.
 *                         Requires W % 16 == 0 (else LTL_ERR_UNSUPPORTED).
 * Takes effect for the following steps; columns W..pitch-1 of the buffers stay 0. Synchronizes
 * the stream before it drops the cached graphs. */
int32_t ltl_set_boundary(ltl_sim_t *sim, int32_t boundary);

/* Release the handle (graphs, descriptors). Does not free the caller's buffers and does
 * not synchronize; the caller synchronizes the stream first. NULL is accepted. */
int32_t ltl_destroy(ltl_sim_t *sim);

/* For callers that cannot allocate device memory (code under hipGraph stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): one run of ltl_create + ltl_set_boundary +
 * ltl_step(n_steps) + ltl_read + ltl_destroy in a single call that calls no hipMalloc, hipFree
 * or other allocating routine. The result equals that sequence's, cell for cell.
 *  H, W, rule, method, buf_a/b, buf_bytes, init, init_pitch   as for ltl_create (buf_a and
 *             buf_b are overwritten: buf_a with init and zero padding, buf_b with zeros).
 *  boundary   an ltl_boundary_t (as for ltl_set_boundary).
 *  n_steps    >= 0 steps; dst/dst_pitch   device memory receiving the H x W result (as ltl_read).
 *  stream     every operation is enqueued on it; nothing is synchronized (the call does not
 *             validate the initial states: each must be < max(C, 2)).
 * The launch shape is the tuning table's entry (or LTL_TILE), as for a new handle; the kernels
 * run as plain launches, no hipGraph. The band operands and the zero page of the run sit in a
 * 12 KiB static device array of the library (one per GPU, held until the process ends), filled
 * by a kernel at the start of every call; it is large enough for every rule and grid size.
 * Calls on one GPU share that array, so calls that overlap on one GPU (different streams, or
 * different host threads) race and must be serialized by the caller. */
int32_t ltl_run_noalloc(int32_t H, int32_t W, const ltl_rule_t *rule, int32_t method, int32_t boundary,
                        void *buf_a, void *buf_b, size_t buf_bytes, const void *init, size_t init_pitch,
                        int32_t n_steps, void *dst, size_t dst_pitch, hipStream_t stream);

/* Message of the last failing call on this thread ("" if none). */
const char *ltl_last_error(void);
/* LTL_ERR_* code of the last failing call on this thread (LTL_OK if none); the size-returning
 * calls (ltl_buffer_bytes, ltl_batch_buffer_bytes) report their refusals this way. */
int32_t ltl_last_error_code(void);

/* ----------------------------------------------------------------------------------
 * Tuning table ("Optimal Tile per CUDA block": the best tile depends on the radius and the
 * grid size, and is found by measurement). Entries are keyed by method, element type
 * ("i8", "i8w" for R > 16, "i8x" for the cross, "f16", "f8", "direct"), epilogue class
 * ("byte", "win", "half", "decay"; "mixed" for batches), R (0 for batches), the size bucket
 * round(log2(sqrt(cells))) (a batch: its total cells), boundary ("dead", "periodic") and
 * batched (0/1). Two JSON files hold entries: the user cache (the environment variable
 * LTL_TUNE_CACHE names it; default $XDG_CACHE_HOME/ltl/tuning.json or
 * ~/.cache/ltl/tuning.json; "off" disables it), consulted first, and the table shipped next
 * to the library (tuning.json beside libltl.so; LTL_TUNE_TABLE overrides its path). A lookup
 * takes the exact key, else the entry of the same method, element, epilogue class, boundary
 * and batched with the nearest R, then the nearest bucket. Host-only (no device calls). */

/* Fill *out with the entry for a grid (batched = 0: H, W, rule are one grid's; batched = 1:
 * H = total cells, W = 1, rule = the batch's largest radius). *exact (may be NULL) is 1 for an
 * exact key. LTL_OK if an entry was found; LTL_ERR_ARG (no entry) leaves *out zeroed. Callers
 * validate the shape for their grid before use (ltl_create falls back to the next candidate). */
int32_t ltl_tuning_lookup(int32_t H, int32_t W, const ltl_rule_t *rule, int32_t method, int32_t boundary,
                          int32_t batched, ltl_tuning_t *out, int32_t *exact);
/* Insert or replace the entry of that key in the user cache file (created with its directory
 * if missing), ms_per_step recorded beside it. LTL_ERR_ARG if the cache is "off" or unwritable. */
int32_t ltl_tuning_store(int32_t H, int32_t W, const ltl_rule_t *rule, int32_t method, int32_t boundary,
                         int32_t batched, const ltl_tuning_t *tuning, double ms_per_step);

/* ----------------------------------------------------------------------------------
 * Batched simulation: `count` independent automata, each with its own size and rule,
 * advance together in one kernel launch per T steps (tuning.steps_per_launch). The paper
 * simulates one grid; batching is this library's addition, and each instance runs the
 * per-tile work of Algorithm 1 with its own band operands and rule. The launch covers a work
 * list with one entry per (instance, tile), sorted by decreasing estimated cost, one
 * workgroup per entry (dispatched longest first; each XCD takes contiguous blocks of an
 * instance's tiles). Multi-launch calls are replayed from a cached hipGraph. Each instance
 * follows exactly the semantics of a single simulation of its own (dead ghost halo around
 * each grid; no interaction between instances), so instance i after n batched steps equals
 * ltl_create + ltl_step(n) of that grid and rule, cell for cell.
 *
 *  H, W, rules    host arrays of `count` entries (copied).
 *  method         one ltl_method_t for every instance (LTL_CAT_F8 requires R <= 7 for all).
 *  arena_a/b      two device buffers of bytes >= ltl_batch_buffer_bytes() each, 256-byte
 *                 aligned; instance i occupies H[i] rows of ltl_pitch(W[i]) bytes at a
 *                 library-chosen offset (ltl_batch_current gives it). Owned by the caller; the
 *                 library owns their contents until ltl_batch_destroy.
 *  init           host array of `count` device pointers, instance i has row pitch init_pitch[i]
 *                 >= W[i]; read before ltl_batch_create returns.
 *  stream         HIP stream for all work of this handle.
 * Errors as ltl_create, for the first failing instance (its index is in ltl_last_error).
 * The tuning's tile shape is the largest tile; each instance uses that tile grid with its
 * tiles shrunk evenly to cover its grid with the least padding. The launch shape starts as
 * the tuning table's batched entry (LTL_TILE overrides it), else a built-in default. The
 * handle allocates host metadata, cached hipGraphs and device descriptors (band operands of
 * every radius, per-instance launch parameters, the work list). All work of a handle runs on
 * its one stream. */
/* Bytes of each arena (0 on an invalid argument; ltl_last_error_code says why). */
size_t ltl_batch_buffer_bytes(int32_t count, const int32_t *H, const int32_t *W);
int32_t ltl_batch_create(ltl_batch_t **out, int32_t count, const int32_t *H, const int32_t *W,
                         const ltl_rule_t *rules, int32_t method, void *arena_a, void *arena_b,
                         size_t bytes, const void *const *init, const size_t *init_pitch,
                         hipStream_t stream);
/* Enqueue n_steps >= 0 steps of every instance (batch_step(a); batch_step(b) equals
 * batch_step(a + b) cell for cell). With use_graph, the steps run as replays of cached
 * hipGraphs of at most 64 launches each, as for ltl_step. */
int32_t ltl_batch_step(ltl_batch_t *batch, int32_t n_steps);
/* Enqueue a copy of instance `index` (H x W states) into device memory dst, row pitch dst_pitch >= W. */
int32_t ltl_batch_read(ltl_batch_t *batch, int32_t index, void *dst, size_t dst_pitch);
/* Device address and row pitch of instance `index`'s current states in the arenas (columns
 * W..pitch-1 are always 0), and the number of steps taken so far. */
int32_t ltl_batch_current(ltl_batch_t *batch, int32_t index, void **buf, size_t *pitch, int64_t *steps_done);
/* Launch shape of the batch ("Optimal Tile per CUDA block"): zero fields take defaults (T = 1,
 * 128 x 192 tiles, fewest waves that fit every instance). Validated against every instance
 * (LTL_ERR_ARG). set_tuning synchronizes the stream (launch descriptors are rebuilt). */
int32_t ltl_batch_get_tuning(ltl_batch_t *batch, ltl_tuning_t *tuning);
int32_t ltl_batch_set_tuning(ltl_batch_t *batch, const ltl_tuning_t *tuning);
/* Time candidate shapes and keep the fastest per step, as ltl_autotune: the arenas' current
 * contents are copied into `scratch` (caller-owned, scratch_bytes >= ltl_batch_buffer_bytes),
 * each candidate starts from that copy on the batch's own arenas, and the state is restored
 * at the end (the batch does not advance). Each candidate runs the whole number of its
 * launches covering at least probe_steps steps (1..4096). The pick goes to the user tuning
 * cache. Allocates only the candidates' descriptors; synchronizes. */
int32_t ltl_batch_autotune(ltl_batch_t *batch, int32_t probe_steps, void *scratch, size_t scratch_bytes,
                           ltl_tuning_t *best);
/* Release the handle; does not free the arenas or synchronize. NULL is accepted. */
int32_t ltl_batch_destroy(ltl_batch_t *batch);

#ifdef __cplusplus
}
#endif
#endif /* LTL_H */
