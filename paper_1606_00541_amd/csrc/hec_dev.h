// Device-side structures and launch interfaces of the HEC triangular solves.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "hec_host.h"

namespace hec {

// Owning device buffer.
struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    ~DevMem() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t b);
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

void hip_check(hipError_t e, const char *what);

// Thread-local last-error text of the C ABI (hec_last_error).
void set_last_error(const std::string &m);

// Run `f` (which returns a status) and convert exceptions to status codes.
template <typename F> hec_status_t guard_status(F &&f)
{
    try {
        hec_status_t s = f();
        if (s == HEC_OK) set_last_error("");
        return s;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return HEC_ERR_ALLOC;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return HEC_ERR_INVALID_ARG;
    } catch (...) {
        set_last_error("unknown error");
        return HEC_ERR_INVALID_ARG;
    }
}
template <typename F> hec_status_t guard(F &&f)
{
    return guard_status([&]() -> hec_status_t {
        f();
        return HEC_OK;
    });
}
template <typename T> void upload(DevMem &m, const std::vector<T> &v)
{
    m.release();
    if (v.empty()) return;
    m.alloc(v.size() * sizeof(T));
    hip_check(hipMemcpy(m.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy H2D");
}
// Upload doubles converted to the plan's value type.
void upload_values(DevMem &m, const std::vector<double> &v, hec_dtype_t dt);

// Mailbox sentinels: NaN bit patterns arithmetic never produces (computed
// NaNs are the canonical quiet NaN).  A slot holding the sentinel has not
// received its value yet.
constexpr unsigned long long kSentinel64 = 0x7FF4DEADBEEF0001ull;
constexpr unsigned int kSentinel32 = 0x7FA0BEEFu;

// Kernel arguments of one triangular solve launch (passed by value).
struct TriArgs {
    int32_t n, w, ld, R;
    const int32_t *ell_col;
    const void *ell_val;
    const int32_t *tail_ptr, *tail_col;
    const void *tail_val;
    const void *dinv;
    const int32_t *step_ptr, *step_row, *step_lanes, *window;
    const int32_t *exp_slot, *exp_ptr;
    const int32_t *chunk_ptr, *chunk_step;  // owner schedule: LDS-staged chunks
    const int32_t *rem_ptr, *rem_ent;       // owner schedule: cross-group entries per step
    const int32_t *imp_ptr, *imp_slot, *exp_row;  // dataflow owner kernel: imports and exports
    const int32_t *wave_ptr;                      // dataflow owner kernel: steps per wavefront
    const int8_t *act;                            // barrier-free kernel: problems still to solve, or null
    const int32_t *seg;                           // barrier-free kernel: device row -> system, or null
    int32_t chunk_rows;
    int32_t in_f64, out_f64;                // vector types of bin / xout
    void *mbox;          // [2][nexp][mbox_stride] values crossing workgroups
    int32_t nexp, mbox_stride;
    unsigned int *epoch;
    int *err_dev;        // device-side abort flag
    int *err_host;       // host-mapped copy, read by the host without a sync
    const void *bin;     // right-hand side, indexed bin[gather[x]*R + k]
    const int32_t *gather;
    void *xw;            // device-order solution [n][R] (plan value type)
    void *xout;          // optional scatter target xout[scatter[x]*R + k]
    const int32_t *scatter;
    int32_t row_begin, row_end;  // level-launch row range
    int32_t write_xw;            // persistent: also store every row to xw
    unsigned long long *trace;   // optional per-step clocks [groups][trace_stride][2]
    int32_t trace_stride;
    unsigned spin;               // polls before a bounded wait gives up
    int32_t nparts;              // dataflow kernel: parts of the plan; system queue: systems
    int32_t queue;               // dataflow kernel: workgroups take parts from a counter (epoch[2])
    const int32_t *sq_lvp, *sq_lvrow, *sq_ring;  // system queue: levels per system, level rows, rings
    const int8_t *sq_keep;                        // system queue: rows also stored to xw (read beyond a ring)
};

// Polls of a bounded device-side wait before it is declared hung (a plan may
// set its own, tri_plan_set_wait_limit); at most kMaxSpin so that the
// sixteen-fold limit of LDS polls stays within 32 bits.
constexpr unsigned kDefaultSpin = 1u << 22;
constexpr unsigned kMaxSpin = 1u << 27;

// Device copy of one triangular plan.
struct DevTri {
    int device = -1;
    int32_t n = 0, w = 0, ld = 0, nlev = 0;
    hec_dtype_t dt = HEC_F64;
    int32_t kind = HEC_SCHED_LEVEL_PERSISTENT;
    int32_t groups = 0, block = 256, max_window = 0, nexp = 0;
    bool unit = false, has_tail = false;
    DevMem ell_col, ell_val, tail_ptr, tail_col, tail_val, dinv, orig;
    DevMem step_ptr, step_row, step_lanes, window, exp_slot, exp_ptr, chunk_ptr, chunk_step, rem_ptr, rem_ent;
    int32_t variant = 0;           // persistent kernel choice (hec_tune_t.kernel_variant)
    bool dataflow = false;         // columns encode group-local imports (dataflow kernel only)
    DevMem imp_ptr, imp_slot, exp_row, wave_ptr;
    DevMem seg;                    // device row -> independent system (batches; empty: one system)
    const int8_t *act = nullptr;   // per-launch: active (system, rhs) problems; others may be skipped
    int32_t df_waves = 0;          // compute wavefronts per group (block = 64 * df_waves + 128)
    int32_t df_rows = 0, df_ints = 0;
    int32_t df_step_rows = 0;      // longest step (one wavefront covers step rows x nrhs)
    bool queue = false;            // dataflow parts taken from a counter (more parts than workgroups)
    bool sysq = false, sq_global = false;  // system queue kernel; some dependencies read from xw
    int32_t sq_lds_rows = 0;
    std::vector<int32_t> sq_widths;  // rows of every level of every system
    int32_t sq_median_rows = 0;      // their median
    DevMem sq_lvp, sq_lvrow, sq_ring, sq_keep;
    int32_t chunk_rows = 0;
    bool max_lanes_one = true;     // every step runs one thread per (row, rhs)
    DevMem epoch, err, mbox;
    int *err_host = nullptr;      // pinned, device-visible
    std::vector<int32_t> levelptr;  // level-launch bounds (host)
    DevMem xw;                      // workspace [n][ws_R]
    int32_t ws_R = 0;
    unsigned long long *trace = nullptr;  // caller-owned profiling buffer
    int32_t trace_stride = 0;
    unsigned spin = kDefaultSpin;         // bounded-wait limit of this plan's launches
    ~DevTri();
};

// Device numeric refactorization of an ILU(0)/ILU(k) factor over its fixed
// pattern: F = L\U in CSR (sorted rows, diagonal present), A's entries mapped
// into it, rows in level order of L, and the positions of every factor
// entry in the two plans' execution layouts (ELL index e*ld + row, or
// -1 - tail index).
constexpr int kRefactorMaxRow = 1024;   // longest factor row (LDS staging)
struct DevRefactor {
    int32_t n = 0, max_row = 1;           // longest factor row
    int64_t nnz_a = 0, nnz_f = 0, nl = 0, nu = 0;
    std::vector<int32_t> a_rp, a_ci;      // pattern of A the map was built for
    std::vector<int32_t> levelptr;        // levels of L (host bounds into rows)
    DevMem a2f, frp, fci, fdpos, fval, rows, err;
    DevMem fwork;                         // elimination target; swapped with fval on success
    DevMem l_src, l_dst, u_src, u_dst, u_diag, d_src;
    // row-per-lane elimination in one launch (0: rows too long, one launch
    // per level instead): the rows' longest length it is built for, and per
    // row (original index) the factor positions it reads from its pivot
    // rows in pivot order, each pivot's diagonal followed by the entries
    // that update the row (sdst: -1 for a pivot, else the updated entry's
    // index in the row)
    int32_t flow_row = 0;
    DevMem sptr, spos, sdst, fflow;
};
// Scatter A's device values into F and eliminate level by level; synchronizes
// `st` and throws ZERO_PIVOT on a zero or non-finite pivot.  The elimination
// runs in fwork, which replaces fval only on success: after a failure fval
// still holds the last good factors.
void refactor_numeric(DevRefactor &r, const double *aval, hipStream_t st);
// Write F's values into the plans (L as is, U scaled by its reciprocal
// diagonal, U's reciprocal diagonal array).
void refactor_refill(const DevRefactor &r, DevTri &L, DevTri &U, hipStream_t st);

// Fill `count` values of type dt with the mailbox sentinel (synchronous).
void fill_sentinel(void *p, size_t count, hec_dtype_t dt);
void upload_tri(DevTri &d, const TriHost &t, int32_t max_nrhs);
void ensure_workspace(DevTri &d, int32_t R);
// Largest number of co-resident workgroups of the persistent kernel for the
// given value type, block size and dynamic LDS bytes on the current device.
int32_t persistent_capacity(hec_dtype_t dt, int32_t block, size_t lds_bytes);
int32_t device_max_lds();
int32_t device_cus();
// Launch one triangular solve: rows gathered from `bin` (type in_dt) through
// `gather`, device-order solution written to `xw`, optionally scattered to
// `xout` (type out_dt) through `scatter`.
void launch_tri(DevTri &d, const void *bin, hec_dtype_t in_dt, const int32_t *gather, void *xw,
                void *xout, hec_dtype_t out_dt, const int32_t *scatter, int32_t R, hipStream_t st);
// Throws HEC_ERR_TIMEOUT if a persistent launch of this plan aborted a wait.
void check_device_error(const DevTri &d);
// Both plans of a preconditioner: clears both flags, throws once.
void check_device_error(const DevTri &a, const DevTri &b);

// ---- Krylov / SpMV / vector support (krylov.hip) ----
struct DevHec {   // general HEC matrix for y = A x
    int device = -1;
    int32_t n = 0, w = 0, ld = 0;
    hec_dtype_t dt = HEC_F64;
    DevMem ell_col, ell_val, tail_ptr, tail_col, tail_val;
    HecHost host;   // host copy (export)
    int64_t tail_nnz = 0;
};
// Upload a general matrix as HEC (ELL width -1 = median row length).
void build_devhec(DevHec &d, const Csr &a, hec_dtype_t dt, int32_t ell_width);
void spmv(const DevHec &A, const double *x, double *y, int32_t R, hipStream_t st);
// r = b - A x
void residual(const DevHec &A, const double *b, const double *x, double *r, int32_t R, hipStream_t st);
void convert_vec(const void *src, hec_dtype_t sdt, void *dst, hec_dtype_t ddt, size_t count, hipStream_t st);
// gather dst[t*R+k] = src[idx[t]*R+k] (f64 -> f64/f32) ; scatter for owned rows
void gather_rows(const double *src, const int32_t *idx, void *dst, hec_dtype_t ddt, int32_t m, int32_t R,
                 hipStream_t st);
void scatter_owned(const void *src, hec_dtype_t sdt, const int32_t *idx, const int32_t *owned, double *dst,
                   int32_t m, int32_t R, hipStream_t st);

}  // namespace hec
