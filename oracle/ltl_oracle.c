/*
 * Larger-than-Life oracle: plain CPU reference for the step the GPU library computes.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's CPU
 * baseline call this code; the product path never links or loads it, and it shares
 * no code with the HIP kernels.
 *
 * What it computes (paper, "Formulation of CAT", Eq. 2-3 and the rule notation of
 * "Chosen CA tests"): for a grid S of H x W cells with a dead ghost halo, the Moore
 * neighbourhood count of radius r is the number of alive cells in the
 * (2r+1) x (2r+1) box around each cell, cells outside the grid counting as dead.
 * Eq. 2-3 compute exactly this box sum as Lambda x Pi followed by Pi x H with Pi the
 * band matrix of ones of half-width r; the oracle writes the sum out directly.
 *
 * Periodic boundary (the paper's experimental setting, "Experimental design"; the overview
 * figure fills the ghost halo from the opposite edges): the grid is a torus and the count
 * sums the (2r+1)^2 offsets (di, dj) of the cell at ((i + di) mod H, (j + dj) mod W). On a
 * torus smaller than the box, one cell can be reached by several offsets and is then
 * counted once per offset (the sum is the cyclic convolution with the box).
 *
 * Cross neighbourhood (rule code N_N, the paper's "simplified Von Neumann" of Eq. 4): the
 * count sums the 2r + 1 cells of the cell's row and the 2r cells above and below it in its
 * column (a plus sign of arm r, 4r + 1 cells, the centre once). Eq. 4 writes the same sum
 * as Pi x Lambda + H, which holds the centre twice; the rule's M then decides whether the
 * centre is counted, exactly as for Moore.
 *
 * Readings taken where the paper is silent (each is listed in the design notes):
 *  - only state 1 is alive; with M = 0 the centre's own alive bit is removed once
 *    (the band of Eq. 2-3 holds the diagonal once, so the box counts the centre once);
 *  - C in {0, 2} means two states; C >= 3 adds decay states 2..C-1: an alive cell
 *    whose count leaves S becomes 2, a decaying cell advances by one per step and
 *    wraps to 0 after C-1; decaying cells are neither alive nor born;
 *  - S and B ranges are inclusive and empty when lo > hi;
 *  - any byte value is accepted: a state >= max(C, 2) behaves like the last decay
 *    state (next state 0) and is not alive.
 *
 * Pins (tests): Life still lifes / oscillators / spaceships, brute force over every
 * 3x3 and 5x5 neighbourhood, closed forms of the count, SciPy convolution, the band
 * product of Eq. 2-3, D4 symmetry, M0/M1 equivalence, the decay countdown.
 *
 * Parity unpinned: the decay semantics themselves (C >= 3). The paper defines C but prints
 * no multi-state example, so the reading above is the standard Larger-than-Life one; the
 * countdown closed form and the decay brute force pin this code to that reading, not the
 * reading to the paper.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int imax(int a, int b) { return a > b ? a : b; }
static int imin(int a, int b) { return a < b ? a : b; }

/* Box count of alive cells (state == 1) of radius r around every cell, centre
 * included, cells outside the H x W grid dead. cnt is H*W int32, row-major. */
void oracle_count(const uint8_t *s, int64_t H, int64_t W, int r, int32_t *cnt)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < H; ++i) {
        int lo_i = (int)imax(-r, (int)-i);
        int hi_i = (int)imin(r, (int)(H - 1 - i));
        for (int64_t j = 0; j < W; ++j) {
            int lo_j = imax(-r, (int)-j);
            int hi_j = imin(r, (int)(W - 1 - j));
            int32_t c = 0;
            for (int di = lo_i; di <= hi_i; ++di) {
                const uint8_t *row = s + (i + di) * W + j;
                for (int dj = lo_j; dj <= hi_j; ++dj)
                    c += (row[dj] == 1);
            }
            cnt[i * W + j] = c;
        }
    }
}

/* Periodic box count: offsets wrap around both dimensions (cyclic convolution of the
 * alive map with the (2r+1) x (2r+1) box). */
void oracle_count_periodic(const uint8_t *s, int64_t H, int64_t W, int r, int32_t *cnt)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < H; ++i) {
        for (int64_t j = 0; j < W; ++j) {
            int32_t c = 0;
            for (int di = -r; di <= r; ++di) {
                int64_t ii = ((i + di) % H + H) % H;
                const uint8_t *row = s + ii * W;
                for (int dj = -r; dj <= r; ++dj) {
                    int64_t jj = ((j + dj) % W + W) % W;
                    c += (row[jj] == 1);
                }
            }
            cnt[i * W + j] = c;
        }
    }
}

/* Cross count of radius r (centre once), dead outside the grid or on a torus. */
void oracle_count_cross(const uint8_t *s, int64_t H, int64_t W, int r, int periodic, int32_t *cnt)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < H; ++i) {
        for (int64_t j = 0; j < W; ++j) {
            int32_t c = 0;
            for (int d = -r; d <= r; ++d) {
                int64_t jj = j + d, ii = i + d;
                if (periodic) {
                    jj = (jj % W + W) % W;
                    ii = (ii % H + H) % H;
                    c += (s[i * W + jj] == 1);
                    if (d != 0)
                        c += (s[ii * W + j] == 1);
                } else {
                    if (jj >= 0 && jj < W)
                        c += (s[i * W + jj] == 1);
                    if (d != 0 && ii >= 0 && ii < H)
                        c += (s[ii * W + j] == 1);
                }
            }
            cnt[i * W + j] = c;
        }
    }
}

/* The transition of one cell given its state and its box count n (centre included). */
static uint8_t transition(uint8_t s, int32_t n, int C, int M, int S1, int S2, int B1, int B2)
{
    int states = C >= 3 ? C : 2;
    int32_t c = n;
    if (M == 0 && s == 1)
        c -= 1;
    if (s == 0)
        return (uint8_t)((B1 <= c && c <= B2) ? 1 : 0);
    if (s == 1) {
        if (S1 <= c && c <= S2)
            return 1;
        return (uint8_t)(states > 2 ? 2 : 0);
    }
    return (uint8_t)((s + 1 < states) ? s + 1 : 0);
}

/* One synchronous step: out = f(s). out must not alias s. periodic: 0 dead ghost halo,
 * 1 torus. Returns 0 or -1 on bad args. */
int oracle_step_nb(const uint8_t *s, uint8_t *out, int64_t H, int64_t W,
                   int R, int C, int M, int S1, int S2, int B1, int B2, int periodic, int cross)
{
    if (!s || !out || H < 0 || W < 0 || R < 0)
        return -1;
    if (H == 0 || W == 0)
        return 0;
    int32_t *cnt = (int32_t *)malloc((size_t)H * (size_t)W * sizeof(int32_t));
    if (!cnt)
        return -1;
    if (cross)
        oracle_count_cross(s, H, W, R, periodic, cnt);
    else if (periodic)
        oracle_count_periodic(s, H, W, R, cnt);
    else
        oracle_count(s, H, W, R, cnt);
    int64_t k, n = H * W;
#pragma omp parallel for schedule(static)
    for (k = 0; k < n; ++k)
        out[k] = transition(s[k], cnt[k], C, M, S1, S2, B1, B2);
    free(cnt);
    return 0;
}

int oracle_step_b(const uint8_t *s, uint8_t *out, int64_t H, int64_t W,
                  int R, int C, int M, int S1, int S2, int B1, int B2, int periodic)
{
    return oracle_step_nb(s, out, H, W, R, C, M, S1, S2, B1, B2, periodic, 0);
}

int oracle_step(const uint8_t *s, uint8_t *out, int64_t H, int64_t W,
                int R, int C, int M, int S1, int S2, int B1, int B2)
{
    return oracle_step_b(s, out, H, W, R, C, M, S1, S2, B1, B2, 0);
}

/* steps synchronous steps applied to grid in place (ping-pong with a scratch copy). */
int oracle_run_nb(uint8_t *grid, int64_t H, int64_t W, int R, int C, int M,
                  int S1, int S2, int B1, int B2, int steps, int periodic, int cross)
{
    if (!grid || steps < 0)
        return -1;
    if (steps == 0 || H == 0 || W == 0)
        return 0;
    uint8_t *tmp = (uint8_t *)malloc((size_t)H * (size_t)W);
    if (!tmp)
        return -1;
    uint8_t *a = grid, *b = tmp;
    for (int t = 0; t < steps; ++t) {
        if (oracle_step_nb(a, b, H, W, R, C, M, S1, S2, B1, B2, periodic, cross) != 0) {
            free(tmp);
            return -1;
        }
        uint8_t *x = a; a = b; b = x;
    }
    if (a != grid)
        memcpy(grid, a, (size_t)H * (size_t)W);
    free(tmp);
    return 0;
}

int oracle_run_b(uint8_t *grid, int64_t H, int64_t W, int R, int C, int M,
                 int S1, int S2, int B1, int B2, int steps, int periodic)
{
    return oracle_run_nb(grid, H, W, R, C, M, S1, S2, B1, B2, steps, periodic, 0);
}

int oracle_run(uint8_t *grid, int64_t H, int64_t W, int R, int C, int M,
               int S1, int S2, int B1, int B2, int steps)
{
    return oracle_run_b(grid, H, W, R, C, M, S1, S2, B1, B2, steps, 0);
}

int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
