// Host-side structures of the HEC triangular-solve library: analysis plans,
// execution layouts and schedules.  Pure C++ (no HIP), shared by the analysis,
// factorization and C-ABI translation units.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/hec.h"

namespace hec {

// Error carrier used inside the library; converted to hec_status_t at the ABI.
struct Error {
    hec_status_t code;
    std::string msg;
};

[[noreturn]] void fail(hec_status_t code, const std::string &msg);

// A CSR view of a square host matrix with double values.
struct Csr {
    int32_t n = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> v;
    int64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

Csr csr_copy(int32_t n, const int32_t *rowptr, const int32_t *col, const void *val, hec_dtype_t dt);
void check_csr_structure(const Csr &a);  // rowptr, bounds, strict ascending order

// Level-set analysis of one triangle (Algorithm 1, steps 1-2).
struct Levels {
    int32_t nlev = 0;
    std::vector<int32_t> level;     // per original row, 1-based
    std::vector<int32_t> levelptr;  // [nlev+1]
    std::vector<int32_t> perm;      // new (level-order) position -> original row
    std::vector<int32_t> iperm;     // original row -> new position (the map m)
};

// Paper-layout HEC of L' (Algorithm 1, steps 3-4): ELL column-major, padding
// value 0 / column n; CSR remainder holds the rest and the diagonal last.
struct HecHost {
    int32_t n = 0, w = 0, ld = 0;
    std::vector<int32_t> ell_col;
    std::vector<double> ell_val;
    std::vector<int32_t> csr_ptr, csr_col;
    std::vector<double> csr_val;
};

// A schedule for the persistent executor: every workgroup runs its steps in
// order; a step is a contiguous range of device rows (rows of one level, or a
// chunk of one).  Rows read by a workgroup other than their owner are
// "exported": their values also travel through a double-buffered mailbox
// whose slots consumers poll until the value has arrived.
struct Schedule {
    int32_t kind = HEC_SCHED_LEVEL_PERSISTENT;
    int32_t groups = 0;
    std::vector<int32_t> step_ptr;   // [groups+1]
    std::vector<int32_t> step_row;   // [2*nsteps]: begin, end (device rows)
    std::vector<int32_t> step_lanes; // [nsteps]: lanes cooperating per row (1 = thread per row)
    std::vector<int32_t> window;     // [2*groups]: LDS window (device rows lo, hi)
    int32_t max_window = 0;          // largest window (rows)
    int32_t nexp = 0;                // exported rows
    std::vector<int32_t> exp_slot;   // [n]: device row -> mailbox slot, or -1
    std::vector<int32_t> exp_ptr;    // [groups+1]: mailbox slots of each group (contiguous)
    int64_t remote_reads = 0;        // dependency entries that cross workgroups
    int32_t crit_hops = 0;           // most workgroup handoffs along one dependency chain
    // owner schedule: each group's steps are cut into chunks of at most
    // chunk_rows rows whose matrix data is staged in LDS one chunk ahead
    int32_t chunk_rows = 256;
    std::vector<int32_t> chunk_ptr;  // [groups+1] into chunk_step
    std::vector<int32_t> chunk_step; // [2*nchunks]: first step, end step
    // owner schedule: per step, the cross-group ELL entries as (position in
    // the chunk's entry grid (row - chunk start) * w + slot index, mailbox slot)
    std::vector<int32_t> rem_ptr;    // [nsteps+1]
    std::vector<int32_t> rem_ent;    // [2*nrem]
    int32_t max_rem_window = 0;      // most entries in any 8 consecutive steps of a group
    // dataflow owner kernel: every step is one wavefront's unit of rows of one
    // level; a column is a row of the group's LDS value area (own rows, then
    // imports after the right-hand-side copy, then a zero row for padding).
    // Import j of group g reads mailbox slot imp_slot[imp_ptr[g] + j]
    // (imports ordered by first use, so in level order).
    bool dataflow = false;
    std::vector<int32_t> imp_ptr;    // [groups+1]
    std::vector<int32_t> imp_slot;   // [nimp]
    std::vector<int32_t> exp_row;    // [nexp]: device row of each mailbox slot
    int32_t max_imp = 0;             // most imports of one group
    int32_t df_rows = 0;             // max over groups of 2 * window rows + imports + 1
    int32_t df_ints = 0;             // max over groups of imports + exports + 2 * steps
    int32_t df_waves = 0;            // compute wavefronts per group
    std::vector<int32_t> wave_ptr;   // [groups*df_waves+1]: steps of wavefront w of group g
    // queue mode: `groups` parts, more than the workgroups that run them; the
    // parts are numbered so that every part reads only lower-numbered ones
    bool queue = false;
    // system queue (kernel variant 7): `groups` independent systems, taken
    // whole by the workgroups; system k (queue order) has levels
    // sq_lvp[k]..sq_lvp[k+1]-1, level l its device rows sq_lvrow[l]..sq_lvrow[l+1]-1;
    // its LDS ring has sq_ring[2k] slots of sq_ring[2k+1] rows
    bool sysq = false;
    bool sq_global = false;          // some dependency is read from the global workspace
    int32_t sq_lds_rows = 0;         // largest ring plus the zero row, in rows
    std::vector<int32_t> sq_lvp, sq_lvrow, sq_ring;
    std::vector<int8_t> sq_keep;     // rows read back from the global workspace
    int32_t nsteps() const { return (int32_t)step_lanes.size(); }
};

// Device-order (execution) layout of one triangle: rows permuted into the
// schedule's order, ELL/CSR columns renumbered to device rows, the diagonal
// split into its own dense array (stored as its reciprocal).  Under a
// persistent schedule a column c > n names mailbox slot c - n - 1 (a value
// produced by another workgroup); c == n is ELL padding.
struct ExecHost {
    int32_t n = 0, w = 0, ld = 0;
    std::vector<int32_t> xord;   // device row -> level-order row
    std::vector<int32_t> xinv;   // level-order row -> device row
    std::vector<int32_t> orig;   // device row -> original row
    std::vector<int32_t> owner;  // device row -> workgroup
    std::vector<int32_t> ell_col;
    std::vector<double> ell_val;
    std::vector<int32_t> tail_ptr, tail_col;  // empty when no row overflows the ELL part
    std::vector<double> tail_val;
    std::vector<double> dinv;                 // empty for a unit diagonal
    std::vector<int32_t> levelptr;            // level-launch schedule: device-row bounds per level
    Schedule sched;
};

struct TriHost {
    int32_t n = 0;
    bool upper = false, unit = false;
    int32_t variant = 0;  // kernel the plan runs (hec_tune_t.kernel_variant, automatic choices resolved)
    hec_dtype_t dt = HEC_F64;
    Levels lev;
    HecHost hec;
    ExecHost ex;
    int64_t nnz_off = 0, nnz_tail = 0;
};

struct Tune {
    int32_t ell_width = -1;
    int32_t schedule = HEC_SCHED_AUTO;
    int32_t num_groups = 0;
    int32_t merge_rows = 0;
    int32_t group_lanes = 0;
    int32_t long_row = 0;
    int32_t part_rows = 0;
    int32_t host_only = 0;
    int32_t max_nrhs = 1;
    int32_t block_threads = 256;
    int32_t chunk_rows = 256;
    int32_t partition = 0;   // owner parts: 0 auto (grid blocks, else contiguous), 1 contiguous, 2 bisection, 3 grid
    int32_t variant = 0;     // persistent kernel: 0 auto, 1 generic, 2 owner chunked, 3 owner split waves,
                             // 4 owner dataflow
};
// LDS bytes of the dataflow owner kernel: `rows` value rows (x window, b
// window and imports) of R right-hand sides, then `ints` int32 entries
// (import slots, export rows, step bounds).
size_t dataflow_lds_bytes(int32_t rows, int32_t ints, int32_t R, size_t tsize);
// Smallest ELL width >= w the dataflow kernel is built for (1..8, 10, 12,
// 16), or -1 above 16; and its largest workgroup (threads) at that width.
int32_t dataflow_width(int32_t w);
int32_t dataflow_max_block(int32_t w);
// Tuning with every field at its documented default.
Tune default_tune();
Tune tune_from(const hec_tune_t *t);

// Algorithm 1 on one triangle.  `groups_cap` is the largest persistent grid
// the device can hold (0 = unknown; a default is used).  `sys_ptr` (optional)
// marks independent diagonal blocks for the owner schedule.
void validate_triangle(const Csr &a, bool upper, bool unit);
Levels compute_levels(const Csr &a, bool upper);
int32_t auto_ell_width(const Csr &a, bool upper);
HecHost build_hec(const Csr &a, bool upper, bool unit, const Levels &lv, int32_t w);
std::vector<int32_t> bisect_parts(const Csr &a, int32_t parts);
bool detect_grid(const Csr &a, int32_t &nx, int32_t &ny, int32_t &nz);
std::vector<int32_t> grid_parts(int32_t n, int32_t nx, int32_t ny, int32_t nz, int32_t parts);
int32_t critical_hops(const Csr &a, bool upper, const std::vector<int32_t> &own);
// Device facts the schedules are sized by (zeros when unknown / host-only).
struct DeviceShape {
    int32_t groups_cap = 0;  // co-resident persistent workgroups
    int32_t cus = 0;         // compute units
    int32_t xcds = 8;        // L2 domains; workgroup i runs on domain i % xcds
    int32_t lds = 0;         // LDS bytes one workgroup may use (0: 160 KiB)
};
void build_exec(TriHost &t, const Csr &a, const Tune &tune, const DeviceShape &dev,
                const std::vector<int32_t> *sys_ptr);
TriHost analyze(const Csr &a, bool upper, bool unit, hec_dtype_t dt, const Tune &tune,
                const DeviceShape &dev, const std::vector<int32_t> *sys_ptr = nullptr);

// Incomplete factorizations (Section 3), each returning L (strict part plus a
// stored unit diagonal last in each row) and U (diagonal first).
void ilu0(const Csr &a, Csr &L, Csr &U);
void iluk(const Csr &a, int32_t k, Csr &L, Csr &U);
void ilut(const Csr &a, int32_t p, double tau, Csr &L, Csr &U);
void factor_blocks(const Csr &a, const std::vector<int32_t> &block_ptr,
                   const std::function<void(const Csr &, Csr &, Csr &)> &fac, Csr &L, Csr &U);

// Restricted Additive Schwarz setup: extended subdomains (ascending global
// rows) and the block-diagonal matrix of the A_s = A[ext_s, ext_s].
struct RasLayout {
    int32_t nsub = 0;
    std::vector<int32_t> ext_ptr;   // [nsub+1] into ext
    std::vector<int32_t> ext;       // global row of each extended position
    std::vector<int32_t> owned;     // [ext.size()] 1 if the position is owned by its subdomain
    Csr blockdiag;                  // n = ext.size(), block s = rows ext_ptr[s]..ext_ptr[s+1]-1
};
RasLayout ras_layout(const Csr &a, int32_t nsub, const int32_t *owner, int32_t overlap);

}  // namespace hec
