// Host-side helpers shared by the single-grid (ltl_api.cpp) and batched (batch_api.cpp) parts
// of the C ABI: error reporting, rule validation and constants, grid limits, element choice.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "ltl.h"
#include "ltl_internal.h"

namespace ltl {
namespace host {

// Message and code of the last failing call on this thread (ltl_last_error, ltl_last_error_code).
extern thread_local std::string g_err;
extern thread_local int32_t g_code;

// The error state around a probe whose failure is expected (an infeasible candidate shape).
struct SavedError {
    std::string msg;
    int32_t code;
};
inline SavedError save_error() { return SavedError{g_err, g_code}; }
inline void restore_error(const SavedError &e) {
    g_err = e.msg;
    g_code = e.code;
}

int32_t fail(int32_t code, const std::string &msg);
// A HIP failure reported as LTL_ERR_HIP. The runtime's last-error slot is cleared as well: the
// error is reported through this library's code, and a stale entry would otherwise surface at
// the caller's next unrelated HIP call (torch checks it after every kernel launch).
int32_t hip_fail(hipError_t e, const char *what);
// The result of a HIP call whose failure needs no report (releases, synchronizations before
// them, capability probes): a failure is dropped from the last-error slot for the same reason.
inline void quiet(hipError_t e) {
    if (e != hipSuccess) (void)hipGetLastError();
}

#define HIP_TRY(expr, what)                               \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return ltl::host::hip_fail(e_, what); \
    } while (0)

// Rule checks of ltl_create / ltl_batch_create (LTL_OK or an LTL_ERR_* code with a message).
int32_t validate_rule(const ltl_rule_t *r, int method);
// Largest count of the rule's neighbourhood (centre included).
int max_count(const ltl_rule_t &r);
// Epilogue flavour (Epi) of a rule.
int epi_of(const ltl_rule_t &r, int elem);
// Thresholds and SWAR constants of a rule for an epilogue flavour.
RuleConsts make_consts(const ltl_rule_t &r, int epi);
// Row pitch of the library layout: W rounded up to 64 bytes.
int pitch_of(int W);
// Whether an H x W grid exceeds the 2^31 - 1 bytes the kernels' 32-bit row offsets address.
bool grid_too_large(int H, int W);
// Largest dynamic LDS allocation of a workgroup on the current device.
size_t max_lds_bytes();
// Element type of the band products for a method, radius and neighbourhood code.
int elem_of(int method, int R, int N);

// Launches per step chunk: a call of n steps runs as chunks of at most this many launches,
// each one cached hipGraph (or that many plain launches), so the graph size and the host
// vectors stay bounded whatever n is.
constexpr int kMaxChunkLaunches = 64;

// Bytes of one band table (LTL_BAND_OPS operands x 64 lanes x 16 bytes).
constexpr size_t kBandBytes = LTL_BAND_TABLE_INTS * sizeof(int32_t);

}  // namespace host
}  // namespace ltl
