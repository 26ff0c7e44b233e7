// lra_internal.h -- structures shared by the host runtime and the gfx950
// engine kernels.  Not part of the public ABI (see include/lra.h).
#pragma once
#include <stdint.h>

namespace lra {

// Entry source as the device sees it (device pointers).
struct DevSource {
    int32_t kind;       // 0 dense, 1 Cauchy 1/(x_i - y_j), 2 inverse distance 1/|x_i - y_j|,
                        // 3 dense pre-processed by abridged Hadamard multipliers, F A H
    int32_t dtype;      // 0 float32, 1 float64
    const void* a;
    int64_t lda;
    int32_t col_major;
    int32_t depth;      // kind 3: recursion depth d (2^d divides pm and pn)
    const void* x;
    const void* y;
    uint64_t seed;      // kind 3: sign streams seed (rows) and seed + 1 (columns)
    int64_t pm, pn;     // kind 3: dimensions of a
};

// PH_REDUCE: the Cynical step (an r x r generator inside the k x k one).
enum Phase : int32_t { PH_COL = 0, PH_ROW = 1, PH_FINAL = 2, PH_DONE = 3, PH_REDUCE = 4 };

enum Warn : int32_t { W_TOL = 1, W_CAP = 2, W_NUMRANK = 4 };

// Resumable per-problem state; the team leader writes it at the end of every
// phase, every workgroup of the team reads it when a task starts.
struct TaskState {
    int32_t phase;
    int32_t k;
    int32_t sweep_in_level;
    int32_t status;          // 0, or a negative lra_status
    int32_t warn;            // Warn bits
    int32_t have_I;
    int32_t had_I_sweep;     // have_I when the current sweep started
    int32_t k_sweep_start;   // k when the current sweep started
    int32_t swaps_total;
    int32_t sweeps_done;
    int64_t cand_next;
    int64_t entries_read;
    double est_rel, est_abs, mean, var, cond1;
    int32_t phases_run;
    int32_t w_valid;         // the work buffer holds C[X,:]^{-1} of the last step (binary64)
};

// One C-A / CUR problem.
struct TaskDesc {
    DevSource src;
    int64_t m, n;
    int32_t k0, kmax, kstep, sweeps;
    double tol, tau;
    int32_t max_swaps, warm_start;
    int32_t q, s;
    const int64_t* cand;
    int64_t n_cand;
    const int64_t* Q;
    const int64_t* S;
    int64_t* I;        // kcap
    int64_t* J;        // kcap
    int64_t* prevI;    // kcap
    int64_t* prevJ;    // kcap
    double* G;         // kcap^2, row-major k x k
    double* U;         // kcap^2, row-major k x k
    double* work;      // q*kcap + kcap*s + q*s doubles
    void* strip;       // max(m,n) * kcap strip elements, or null when the rows fit in LDS
    void* C_out;       // optional: A[:,J], m x k column-major, strip precision
    void* R_out;       // optional: A[I,:], k x n row-major, strip precision
    TaskState* st;
    int32_t variant;   // kernel variant: 4 * (binary64 strips) + log2(KMAX / 8)
    int32_t cur_rank;      // Cynical reduction to this rank after the sweeps (0: none)
    int32_t inner_sweeps;  // C-A sweeps of the reduction inside the k x k block
    int32_t nucleus_rank;  // truncated pseudo-inverse nucleus of this rank (0: inverse)
    int32_t bf16_select;   // binary32 path: BF16 shortlist + binary32 recheck in the swaps
    int32_t pad_t;
};

constexpr int NVARIANT = 8;
inline int variant_index(int prec64, int kmax)
{
    return 4 * (prec64 ? 1 : 0) + (kmax <= 8 ? 0 : kmax <= 16 ? 1 : kmax <= 32 ? 2 : 3);
}

struct TeamInfo {
    int32_t first_wg;
    int32_t size;      // workgroups in the team
    int32_t queue;     // which work queue the team pulls from
    int32_t pad;
};

struct EngineArgs {
    TaskDesc* tasks;
    const int32_t* queue_items;   // concatenated task lists of all queues
    const int32_t* queue_off;
    const int32_t* queue_len;
    uint32_t* queue_head;         // one pull counter per queue, zero at launch
    const TeamInfo* teams;
    const int32_t* wg_team;       // team of each workgroup
    uint8_t* team_ctl;            // per-team control block, zero at launch
    int64_t team_ctl_stride;
    int32_t phase_budget;         // phases per task per launch (large: run to completion)
    int32_t lds_b[8];             // LDS bytes for a workgroup's strip rows, per variant
    uint32_t* error_flag;         // bit 0: a team barrier timed out
    int64_t timeout_ticks;        // in wall_clock64() ticks
    uint64_t* trace;              // optional event trace: [0] = count, then (event, clock) pairs
    int32_t trace_cap;            // pairs
};

// Trace events (recorded by thread 0 of a team's first workgroup).
enum TraceEv : int32_t {
    EV_STEP_BEGIN = 1, EV_WARM_LU = 2, EV_GATHERED = 3, EV_BASIS = 4, EV_SWAP = 5, EV_STEP_END = 6,
    EV_FINAL_BEGIN = 7, EV_FINAL_END = 8, EV_TASK_BEGIN = 9, EV_TASK_END = 10, EV_PIVOT = 11,
    EV_SWAP_RED = 12, EV_SWAP_XCH = 13, EV_PHASE_END = 14, EV_DISPATCH = 15
};

// Team control block layout: [0, 64): barrier counter; [64, 72): fetched task
// (two int32 by barrier parity); slots start at CTL_HDR, two banks (barrier
// parity) of `team size` slots of SLOT_STRIDE bytes.
constexpr int CTL_HDR = 256;
constexpr int SLOT_STRIDE = 544;  // 32-byte header (two key words) + 64 binary64 payload
constexpr int KMAX_ALL = 64;
constexpr int NT = 256;           // threads per workgroup

inline int64_t team_ctl_bytes(int team_size)
{
    return CTL_HDR + 2ll * team_size * SLOT_STRIDE;
}

// Device workspace of the allocation-free entry point: a fixed array per
// device (the upload image, team control blocks, per-problem scratch and any
// global strip of one problem must fit in it).
constexpr int64_t NOALLOC_SCRATCH_BYTES = 64ll << 20;
// Host staging of that entry point (upload and read-back image).
constexpr int64_t NOALLOC_HOST_BYTES = 1ll << 20;

}  // namespace lra
