// Algorithm 1 (Section 2.2) of the paper on the host: level of every unknown
// (eq. (2)), the level map m (eq. (3)), the reordered L' and its HEC form
// (Section 2.1), plus the device execution layout and the persistent
// schedule built on top of the level sets.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>

#include "hec_host.h"

namespace hec {

void fail(hec_status_t code, const std::string &msg) { throw Error{code, msg}; }

Tune default_tune()
{
    hec_tune_t t;
    std::memset(&t, 0, sizeof(t));
    t.ell_width = -1;
    t.max_nrhs = 1;
    t.block_threads = 256;
    return tune_from(&t);
}

Tune tune_from(const hec_tune_t *t)
{
    if (!t) return default_tune();
    Tune u;
    u.ell_width = t->ell_width;
    u.schedule = t->schedule;
    u.num_groups = t->num_groups;
    u.merge_rows = t->merge_rows;
    u.group_lanes = t->group_lanes;
    u.long_row = t->long_row;
    u.part_rows = t->part_rows;
    u.host_only = t->host_only;
    u.max_nrhs = t->max_nrhs > 0 ? t->max_nrhs : 1;
    u.block_threads = t->block_threads > 0 ? t->block_threads : 256;
    // Default chunk: the smallest of 1, 2 or 4 blocks that holds at least 256 rows.
    u.chunk_rows = t->chunk_rows > 0 ? t->chunk_rows
                 : u.block_threads * (u.block_threads >= 256 ? 1 : (u.block_threads >= 128 ? 2 : 4));
    u.partition = t->partition;
    u.variant = t->kernel_variant;
    if (u.variant < 0 || u.variant > 7) fail(HEC_ERR_INVALID_ARG, "tune.kernel_variant out of range");
    if (u.variant == 5 && u.schedule != HEC_SCHED_AUTO && u.schedule != HEC_SCHED_LEVEL_LAUNCH)
        fail(HEC_ERR_INVALID_ARG, "kernel_variant 5 runs the level-ordered layout (schedule AUTO or LEVEL_LAUNCH)");
    if (u.partition < 0 || u.partition > 3) fail(HEC_ERR_INVALID_ARG, "tune.partition out of range");
    if (u.schedule < HEC_SCHED_AUTO || u.schedule > HEC_SCHED_OWNER_PERSISTENT)
        fail(HEC_ERR_INVALID_ARG, "tune.schedule out of range");
    if (u.block_threads % 64 != 0 || u.block_threads > 1024)
        fail(HEC_ERR_INVALID_ARG, "tune.block_threads must be a multiple of 64 up to 1024");
    if (u.group_lanes != 0 && (u.group_lanes < 1 || u.group_lanes > 64 ||
                               (u.group_lanes & (u.group_lanes - 1)) != 0))
        fail(HEC_ERR_INVALID_ARG, "tune.group_lanes must be a power of two in 1..64");
    if (u.ell_width < -1 || u.ell_width > 64) fail(HEC_ERR_INVALID_ARG, "tune.ell_width out of range");
    if (u.num_groups < 0 || u.merge_rows < 0 || u.long_row < 0 || u.part_rows < 0)
        fail(HEC_ERR_INVALID_ARG, "negative tuning value");
    if (u.chunk_rows != u.block_threads && u.chunk_rows != 2 * u.block_threads && u.chunk_rows != 4 * u.block_threads)
        fail(HEC_ERR_INVALID_ARG, "tune.chunk_rows must be 1, 2 or 4 times block_threads");
    return u;
}

Csr csr_copy(int32_t n, const int32_t *rowptr, const int32_t *col, const void *val, hec_dtype_t dt)
{
    if (n < 0) fail(HEC_ERR_INVALID_ARG, "n < 0");
    if (dt != HEC_F64 && dt != HEC_F32) fail(HEC_ERR_INVALID_ARG, "unknown dtype");
    Csr a;
    a.n = n;
    if (!rowptr) fail(HEC_ERR_INVALID_ARG, "rowptr is NULL");
    a.rp.assign(rowptr, rowptr + (size_t)n + 1);
    if (a.rp[0] != 0) fail(HEC_ERR_INVALID_ARG, "rowptr[0] != 0");
    for (int32_t i = 0; i < n; ++i)
        if (a.rp[i + 1] < a.rp[i]) fail(HEC_ERR_INVALID_ARG, "rowptr not monotone");
    int64_t nnz = a.rp[n];
    if (nnz > 0 && (!col || !val)) fail(HEC_ERR_INVALID_ARG, "col or val is NULL");
    a.ci.assign(col, col + nnz);
    a.v.resize(nnz);
    if (dt == HEC_F64) {
        const double *d = static_cast<const double *>(val);
        std::copy(d, d + nnz, a.v.begin());
    } else {
        const float *f = static_cast<const float *>(val);
        for (int64_t p = 0; p < nnz; ++p) a.v[p] = f[p];
    }
    check_csr_structure(a);
    return a;
}

void check_csr_structure(const Csr &a)
{
    for (int32_t i = 0; i < a.n; ++i) {
        for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
            int32_t j = a.ci[p];
            if (j < 0 || j >= a.n) fail(HEC_ERR_INVALID_ARG, "column index out of range in row " + std::to_string(i));
            if (p > a.rp[i] && a.ci[p - 1] >= j)
                fail(HEC_ERR_UNSORTED, "row " + std::to_string(i) + " is not sorted by strictly ascending column");
        }
    }
}

void validate_triangle(const Csr &a, bool upper, bool unit)
{
    for (int32_t i = 0; i < a.n; ++i) {
        bool diag = false;
        for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
            int32_t j = a.ci[p];
            if ((!upper && j > i) || (upper && j < i))
                fail(HEC_ERR_NOT_TRIANGULAR, "entry (" + std::to_string(i) + ", " + std::to_string(j) +
                                                 ") is on the wrong side of the diagonal");
            if (j == i) {
                diag = true;
                if (!unit && (a.v[p] == 0.0 || !std::isfinite(a.v[p])))
                    fail(HEC_ERR_ZERO_PIVOT, "zero or non-finite diagonal in row " + std::to_string(i));
            }
        }
        if (!unit && !diag) fail(HEC_ERR_MISSING_DIAG, "row " + std::to_string(i) + " has no diagonal");
    }
}

// eq. (2): l(i) = 1 + max l(j) over the stored off-diagonal entries of row i,
// evaluated in the order of the problem being solved (ascending i for a lower
// triangle, descending i for an upper triangle, i.e. ascending t(i) = n-1-i).
// Then eq. (3): a stable counting sort of the problem's rows by level.
Levels compute_levels(const Csr &a, bool upper)
{
    const int32_t n = a.n;
    Levels lv;
    lv.level.assign(n, 0);
    int32_t nlev = 0;
    for (int32_t q = 0; q < n; ++q) {
        int32_t i = upper ? n - 1 - q : q;
        int32_t m = 0;
        for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
            int32_t j = a.ci[p];
            if (j != i) m = std::max(m, lv.level[j]);
        }
        lv.level[i] = m + 1;
        nlev = std::max(nlev, m + 1);
    }
    lv.nlev = nlev;
    lv.levelptr.assign((size_t)nlev + 1, 0);
    for (int32_t i = 0; i < n; ++i) lv.levelptr[lv.level[i]] += 1;
    for (int32_t k = 0; k < nlev; ++k) lv.levelptr[k + 1] += lv.levelptr[k];
    std::vector<int32_t> cursor(lv.levelptr.begin(), lv.levelptr.end() - 1);
    lv.perm.assign(n, 0);
    lv.iperm.assign(n, 0);
    for (int32_t q = 0; q < n; ++q) {
        int32_t i = upper ? n - 1 - q : q;
        int32_t r = cursor[lv.level[i] - 1]++;
        lv.perm[r] = i;
        lv.iperm[i] = r;
    }
    return lv;
}

static int32_t offdiag_count(const Csr &a, int32_t i)
{
    int32_t c = a.rp[i + 1] - a.rp[i];
    // a stored diagonal is not an off-diagonal entry
    for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p)
        if (a.ci[p] == i) { --c; break; }
    return c;
}

// Smallest w with at most half the rows holding more than w off-diagonals.
int32_t auto_ell_width(const Csr &a, bool /*upper*/)
{
    if (a.n == 0) return 0;
    std::vector<int64_t> hist(65, 0);
    for (int32_t i = 0; i < a.n; ++i) hist[std::min(offdiag_count(a, i), 64)] += 1;
    int64_t above = a.n;
    for (int32_t w = 0; w <= 64; ++w) {
        above -= hist[w];  // rows with more than w off-diagonals
        if (2 * above <= a.n) return w;
    }
    return 64;
}

HecHost build_hec(const Csr &a, bool upper, bool unit, const Levels &lv, int32_t w)
{
    (void)upper;
    const int32_t n = a.n;
    HecHost h;
    h.n = n;
    h.w = w;
    h.ld = (n + 63) / 64 * 64;
    h.ell_col.assign((size_t)w * h.ld, n);
    h.ell_val.assign((size_t)w * h.ld, 0.0);
    h.csr_ptr.assign((size_t)n + 1, 0);
    h.csr_col.reserve((size_t)n);
    h.csr_val.reserve((size_t)n);
    for (int32_t r = 0; r < n; ++r) {
        int32_t i = lv.perm[r];
        int32_t e = 0;
        double d = 1.0;
        for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
            int32_t j = a.ci[p];
            if (j == i) {
                if (!unit) d = a.v[p];
                continue;
            }
            int32_t c = lv.iperm[j];
            if (e < w) {
                h.ell_col[(size_t)e * h.ld + r] = c;
                h.ell_val[(size_t)e * h.ld + r] = a.v[p];
                ++e;
            } else {
                h.csr_col.push_back(c);
                h.csr_val.push_back(a.v[p]);
            }
        }
        h.csr_col.push_back(r);  // the diagonal closes every CSR row
        h.csr_val.push_back(d);
        h.csr_ptr[r + 1] = (int32_t)h.csr_col.size();
    }
    return h;
}

namespace {

// Fill step structures from a device-row order in which every group's rows
// are contiguous per step.  `runs` lists, per group, the (begin, end) device
// row ranges of its steps in execution order.
void finish_schedule(Schedule &s, ExecHost &ex, const std::vector<std::vector<std::pair<int32_t, int32_t>>> &runs,
                     const Tune &tune)
{
    const int32_t G = (int32_t)runs.size();
    s.groups = G;
    s.step_ptr.assign((size_t)G + 1, 0);
    for (int32_t g = 0; g < G; ++g) s.step_ptr[g + 1] = s.step_ptr[g] + (int32_t)runs[g].size();
    const int32_t S = s.step_ptr[G];
    s.step_row.resize(2 * (size_t)S);
    s.step_lanes.assign(S, 1);
    std::vector<int32_t> step_of(ex.n, -1);
    for (int32_t g = 0; g < G; ++g)
        for (size_t t = 0; t < runs[g].size(); ++t) {
            int32_t sid = s.step_ptr[g] + (int32_t)t;
            s.step_row[2 * sid] = runs[g][t].first;
            s.step_row[2 * sid + 1] = runs[g][t].second;
            for (int32_t x = runs[g][t].first; x < runs[g][t].second; ++x) step_of[x] = sid;
        }
    for (int32_t x = 0; x < ex.n; ++x)
        if (step_of[x] < 0) fail(HEC_ERR_INVALID_ARG, "internal: row without a step");
    // lanes per row: steps holding long CSR tails get cooperating lanes
    const int32_t long_row = tune.long_row > 0 ? tune.long_row : 24;
    const int32_t lanes = tune.group_lanes > 0 ? tune.group_lanes : 8;
    if (!ex.tail_ptr.empty()) {
        for (int32_t sid = 0; sid < S; ++sid) {
            int32_t mx = 0;
            for (int32_t x = s.step_row[2 * sid]; x < s.step_row[2 * sid + 1]; ++x)
                mx = std::max(mx, ex.tail_ptr[x + 1] - ex.tail_ptr[x]);
            if (mx + ex.w >= long_row) s.step_lanes[sid] = lanes;
        }
    }
    // exported rows: produced by one group, read by another.  Check that
    // every same-group dependency comes from an earlier step, count the
    // cross-group reads, then give exported rows mailbox slots group by group
    // and re-encode cross-group columns as n + 1 + slot.
    std::vector<char> exported(ex.n, 0);
    s.remote_reads = 0;
    auto scan = [&](int32_t g, int32_t sid, int32_t c) {
        if (c >= ex.n) return;  // ELL padding
        if (ex.owner[c] == g) {
            if (step_of[c] >= sid) fail(HEC_ERR_INVALID_ARG, "internal: dependency not ordered by the schedule");
            return;
        }
        exported[c] = 1;
        s.remote_reads += 1;
    };
    for (int32_t g = 0; g < G; ++g)
        for (int32_t sid = s.step_ptr[g]; sid < s.step_ptr[g + 1]; ++sid)
            for (int32_t x = s.step_row[2 * sid]; x < s.step_row[2 * sid + 1]; ++x) {
                for (int32_t e = 0; e < ex.w; ++e) scan(g, sid, ex.ell_col[(size_t)e * ex.ld + x]);
                if (!ex.tail_ptr.empty())
                    for (int32_t p = ex.tail_ptr[x]; p < ex.tail_ptr[x + 1]; ++p) scan(g, sid, ex.tail_col[p]);
            }
    s.exp_slot.assign(ex.n, -1);
    s.exp_ptr.assign((size_t)G + 1, 0);
    int32_t slot = 0;
    for (int32_t g = 0; g < G; ++g) {
        for (int32_t sid = s.step_ptr[g]; sid < s.step_ptr[g + 1]; ++sid)
            for (int32_t x = s.step_row[2 * sid]; x < s.step_row[2 * sid + 1]; ++x)
                if (exported[x]) s.exp_slot[x] = slot++;
        s.exp_ptr[g + 1] = slot;
    }
    s.nexp = slot;
    auto encode = [&](int32_t x, int32_t &c) {
        if (c < ex.n && ex.owner[c] != ex.owner[x]) c = ex.n + 1 + s.exp_slot[c];
    };
    for (int32_t x = 0; x < ex.n; ++x) {
        for (int32_t e = 0; e < ex.w; ++e) encode(x, ex.ell_col[(size_t)e * ex.ld + x]);
        if (!ex.tail_ptr.empty())
            for (int32_t p = ex.tail_ptr[x]; p < ex.tail_ptr[x + 1]; ++p) encode(x, ex.tail_col[p]);
    }
    // chunks (owner schedule): consecutive steps of a group holding at most
    // chunk_rows rows together (steps were cut to fit beforehand)
    s.chunk_ptr.assign((size_t)G + 1, 0);
    s.chunk_step.clear();
    if (s.kind == HEC_SCHED_OWNER_PERSISTENT) {
        s.chunk_rows = tune.chunk_rows;
        for (int32_t g = 0; g < G; ++g) {
            int32_t sid = s.step_ptr[g];
            while (sid < s.step_ptr[g + 1]) {
                const int32_t first = sid, r0 = s.step_row[2 * sid];
                while (sid < s.step_ptr[g + 1] && s.step_row[2 * sid + 1] - r0 <= s.chunk_rows) ++sid;
                if (sid == first) fail(HEC_ERR_INVALID_ARG, "internal: step larger than a chunk");
                s.chunk_step.push_back(first);
                s.chunk_step.push_back(sid);
            }
            s.chunk_ptr[g + 1] = (int32_t)(s.chunk_step.size() / 2);
        }
    }
    // cross-group entry lists per step (owner schedule, ELL part; plans with
    // a CSR tail do not use them)
    s.rem_ptr.assign((size_t)S + 1, 0);
    s.rem_ent.clear();
    s.max_rem_window = 0;
    if (s.kind == HEC_SCHED_OWNER_PERSISTENT) {
        for (int32_t g = 0; g < G; ++g)
            for (int32_t q = s.chunk_ptr[g]; q < s.chunk_ptr[g + 1]; ++q) {
                const int32_t f = s.chunk_step[2 * q], e = s.chunk_step[2 * q + 1];
                const int32_t r0 = s.step_row[2 * f];
                for (int32_t sid = f; sid < e; ++sid) {
                    for (int32_t x = s.step_row[2 * sid]; x < s.step_row[2 * sid + 1]; ++x)
                        for (int32_t k = 0; k < ex.w; ++k) {
                            const int32_t c = ex.ell_col[(size_t)k * ex.ld + x];
                            if (c > ex.n) {
                                s.rem_ent.push_back((x - r0) * ex.w + k);
                                s.rem_ent.push_back(c - ex.n - 1);
                            }
                        }
                    s.rem_ptr[sid + 1] = (int32_t)(s.rem_ent.size() / 2);
                }
            }
        for (int32_t g = 0; g < G; ++g)
            for (int32_t sid = s.step_ptr[g]; sid < s.step_ptr[g + 1]; ++sid) {
                const int32_t e = std::min(s.step_ptr[g + 1], sid + 8);
                s.max_rem_window = std::max(s.max_rem_window, s.rem_ptr[e] - s.rem_ptr[sid]);
            }
    }
    // LDS windows: a group's contiguous device-row span (owner schedule only)
    s.window.assign(2 * (size_t)G, 0);
    s.max_window = 0;
    if (s.kind == HEC_SCHED_OWNER_PERSISTENT) {
        for (int32_t g = 0; g < G; ++g) {
            if (runs[g].empty()) continue;
            int32_t lo = runs[g].front().first, hi = runs[g].back().second;
            s.window[2 * g] = lo;
            s.window[2 * g + 1] = hi;
            s.max_window = std::max(s.max_window, hi - lo);
        }
    }
}

}  // namespace

// Recursive bisection of the undirected graph of a triangle (its pattern
// plus the transpose, diagonal dropped) into `parts` parts of near-equal
// size.  A set is split by one breadth-first sweep from a pseudo-peripheral
// vertex (found by repeated sweeps): the first vertices reached form the
// first half.  Disconnected pieces are swept in ascending index order.
// Sibling parts get consecutive ids, so nearby ids are nearby rows.
std::vector<int32_t> bisect_parts(const Csr &a, int32_t P)
{
    const int32_t n = a.n;
    std::vector<int32_t> part(n, 0);
    if (P <= 1 || n == 0) return part;
    std::vector<int32_t> aptr((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p)
            if (a.ci[p] != i) {
                aptr[i + 1] += 1;
                aptr[a.ci[p] + 1] += 1;
            }
    for (int32_t i = 0; i < n; ++i) aptr[i + 1] += aptr[i];
    std::vector<int32_t> adj(aptr[n]), cur(aptr.begin(), aptr.end() - 1);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p)
            if (a.ci[p] != i) {
                adj[cur[i]++] = a.ci[p];
                adj[cur[a.ci[p]]++] = i;
            }
    for (int32_t i = 0; i < n; ++i) std::sort(adj.begin() + aptr[i], adj.begin() + aptr[i + 1]);
    std::vector<int32_t> in_set(n, -1), seen(n, -1), order;
    order.reserve(n);
    int32_t set_tag = 0, seen_tag = 0;
    struct Job {
        std::vector<int32_t> mem;
        int32_t k, first;
    };
    std::vector<Job> stack;
    {
        Job j;
        j.mem.resize(n);
        std::iota(j.mem.begin(), j.mem.end(), 0);
        j.k = P;
        j.first = 0;
        stack.push_back(std::move(j));
    }
    // breadth-first sweep inside the current set from r; returns the last vertex
    auto sweep = [&](int32_t r, bool append) {
        const size_t head0 = order.size();
        if (!append) order.resize(head0);
        seen[r] = seen_tag;
        order.push_back(r);
        for (size_t h = head0; h < order.size(); ++h) {
            const int32_t v = order[h];
            for (int32_t q = aptr[v]; q < aptr[v + 1]; ++q) {
                const int32_t w = adj[q];
                if (in_set[w] == set_tag && seen[w] != seen_tag) {
                    seen[w] = seen_tag;
                    order.push_back(w);
                }
            }
        }
        return order.back();
    };
    while (!stack.empty()) {
        Job job = std::move(stack.back());
        stack.pop_back();
        if (job.k <= 1 || job.mem.size() <= 1) {
            for (int32_t v : job.mem) part[v] = job.first;
            continue;
        }
        ++set_tag;
        for (int32_t v : job.mem) in_set[v] = set_tag;
        int32_t root = job.mem.front();
        for (int it = 0; it < 2; ++it) {  // pseudo-peripheral vertex
            ++seen_tag;
            order.clear();
            root = sweep(root, false);
        }
        ++seen_tag;
        order.clear();
        sweep(root, true);
        for (int32_t v : job.mem)  // disconnected remainder, ascending index
            if (seen[v] != seen_tag) sweep(v, true);
        const int32_t k1 = job.k / 2, k2 = job.k - k1;
        const size_t m1 = (size_t)((double)job.mem.size() * k1 / job.k + 0.5);
        Job a1, a2;
        a1.mem.assign(order.begin(), order.begin() + m1);
        a2.mem.assign(order.begin() + m1, order.end());
        a1.k = k1;
        a1.first = job.first;
        a2.k = k2;
        a2.first = job.first + k1;
        std::sort(a1.mem.begin(), a1.mem.end());
        std::sort(a2.mem.begin(), a2.mem.end());
        stack.push_back(std::move(a2));
        stack.push_back(std::move(a1));
    }
    return part;
}

// Structured-grid detection: the natural order of a 2D/3D stencil matrix
// shows up as dominant column offsets 1, nx and nx*ny.  Returns false when
// the pattern does not look like a grid.
bool detect_grid(const Csr &a, int32_t &nx, int32_t &ny, int32_t &nz)
{
    const int32_t n = a.n;
    if (n < 64) return false;
    std::vector<std::pair<int64_t, int32_t>> cnt;  // offset -> count (sparse)
    {
        std::vector<int32_t> offs;
        offs.reserve(a.nnz());
        for (int32_t i = 0; i < n; ++i)
            for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p)
                if (a.ci[p] != i) offs.push_back(std::abs(a.ci[p] - i));
        if (offs.empty()) return false;
        std::sort(offs.begin(), offs.end());
        for (size_t k = 0; k < offs.size();) {
            size_t e = k;
            while (e < offs.size() && offs[e] == offs[k]) ++e;
            cnt.push_back({offs[k], (int32_t)(e - k)});
            k = e;
        }
    }
    auto freq = [&](int64_t o) {
        for (auto &c : cnt)
            if (c.first == o) return c.second;
        return 0;
    };
    const int32_t dominant = n / 4;
    // nx: the most frequent offset >= 2 that divides n
    int64_t bx = 0;
    int32_t fx = 0;
    for (auto &c : cnt)
        if (c.first >= 2 && c.second >= dominant && n % c.first == 0 && c.second > fx) {
            bx = c.first;
            fx = c.second;
        }
    if (bx == 0 || freq(1) < dominant) return false;
    // nx*ny: the most frequent larger multiple of nx that divides n
    int64_t bxy = 0;
    int32_t fxy = 0;
    for (auto &c : cnt)
        if (c.first > bx && c.first % bx == 0 && n % c.first == 0 && c.second >= dominant && c.second > fxy) {
            bxy = c.first;
            fxy = c.second;
        }
    nx = (int32_t)bx;
    if (bxy == 0) {
        ny = n / nx;
        nz = 1;
    } else {
        ny = (int32_t)(bxy / bx);
        nz = (int32_t)(n / bxy);
    }
    return nx > 1 && ny > 1;
}

// Blocks of a detected grid: P = px*py*pz with the smallest px+py+pz (the
// handoffs a monotone dependency chain can make), x split least so that rows
// of a block stay long in memory.  Part ids run x fastest, then y, then z, so
// consecutive ids are neighbouring blocks.
std::vector<int32_t> grid_parts(int32_t n, int32_t nx, int32_t ny, int32_t nz, int32_t P)
{
    int32_t best[3] = {1, 1, P};
    int64_t best_cost = INT64_MAX;
    for (int32_t px = 1; px <= P; ++px) {
        if (P % px || px > nx) continue;
        for (int32_t py = 1; py <= P / px; ++py) {
            if ((P / px) % py || py > ny) continue;
            const int32_t pz = P / px / py;
            if (pz > nz) continue;
            const int64_t cost = (int64_t)(px + py + pz) * 4 + px;  // ties: fewer x cuts
            if (cost < best_cost) {
                best_cost = cost;
                best[0] = px;
                best[1] = py;
                best[2] = pz;
            }
        }
    }
    std::vector<int32_t> part(n, 0);
    if (best_cost == INT64_MAX) {
        for (int32_t i = 0; i < n; ++i) part[i] = (int32_t)((int64_t)i * P / n);
        return part;
    }
    const int32_t px = best[0], py = best[1], pz = best[2];
    for (int32_t i = 0; i < n; ++i) {
        const int32_t x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
        const int32_t bx = (int32_t)((int64_t)x * px / nx), by = (int32_t)((int64_t)y * py / ny),
                      bz = (int32_t)((int64_t)z * pz / nz);
        part[i] = bx + px * (by + py * bz);
    }
    return part;
}

// Largest number of workgroup-to-workgroup handoffs along any dependency
// chain of the triangle, given the owner of every row.
int32_t critical_hops(const Csr &a, bool upper, const std::vector<int32_t> &own)
{
    const int32_t n = a.n;
    std::vector<int32_t> hop(n, 0);
    int32_t best = 0;
    for (int32_t q = 0; q < n; ++q) {
        const int32_t i = upper ? n - 1 - q : q;
        int32_t h = 0;
        for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
            const int32_t j = a.ci[p];
            if (j != i) h = std::max(h, hop[j] + (own[j] != own[i] ? 1 : 0));
        }
        hop[i] = h;
        best = std::max(best, h);
    }
    return best;
}

int32_t dataflow_width(int32_t w)
{
    if (w <= 8) return w;
    if (w <= 10) return 10;
    if (w <= 12) return 12;
    if (w <= 16) return 16;
    return -1;
}

int32_t dataflow_max_block(int32_t /*w*/) { return 512; }

size_t dataflow_lds_bytes(int32_t rows, int32_t ints, int32_t R, size_t tsize)
{
    const size_t vals = (size_t)rows * R * tsize;
    return ((vals + 15) & ~(size_t)15) + (((size_t)ints * 4 + 15) & ~(size_t)15);
}

namespace {

// Prepare an owner schedule for the dataflow kernel.  Each group's exported
// rows get their mailbox slots in level order and each group numbers the
// slots it reads in level order of their first consumer: the kernel's export
// and import wavefronts walk these lists in order, and a list ordered by
// level never waits on an entry whose producer depends on a later entry.
// Then every column becomes a row of the group's LDS value area.
void make_dataflow(Schedule &s, ExecHost &ex, const std::vector<int32_t> &xlev,
                   const std::vector<std::vector<int32_t>> &run_wave, int32_t waves)
{
    const int32_t G = s.groups, n = ex.n;
    auto each_col = [&](int32_t x, const std::function<void(int32_t &)> &f) {
        for (int32_t e = 0; e < ex.w; ++e) f(ex.ell_col[(size_t)e * ex.ld + x]);
        if (!ex.tail_ptr.empty())
            for (int32_t p = ex.tail_ptr[x]; p < ex.tail_ptr[x + 1]; ++p) f(ex.tail_col[p]);
    };
    // 1. export slots in level order within each group
    std::vector<int32_t> remap((size_t)s.nexp, -1);
    for (int32_t g = 0; g < G; ++g) {
        std::vector<int32_t> rows;
        for (int32_t x = s.window[2 * g]; x < s.window[2 * g + 1]; ++x)
            if (s.exp_slot[x] >= 0) rows.push_back(x);
        std::stable_sort(rows.begin(), rows.end(), [&](int32_t p, int32_t q) { return xlev[p] < xlev[q]; });
        for (size_t k = 0; k < rows.size(); ++k) remap[s.exp_slot[rows[k]]] = s.exp_ptr[g] + (int32_t)k;
    }
    for (int32_t x = 0; x < n; ++x) {
        if (s.exp_slot[x] >= 0) s.exp_slot[x] = remap[s.exp_slot[x]];
        each_col(x, [&](int32_t &c) {
            if (c > n) c = n + 1 + remap[c - n - 1];
        });
    }
    s.exp_row.assign((size_t)s.nexp, 0);
    for (int32_t x = 0; x < n; ++x)
        if (s.exp_slot[x] >= 0) s.exp_row[s.exp_slot[x]] = x;
    // 2. imports per group, ordered by the level of their first consumer
    s.imp_ptr.assign((size_t)G + 1, 0);
    s.imp_slot.clear();
    s.max_imp = 0;
    std::vector<int32_t> first_lev((size_t)s.nexp, INT32_MAX), stamp((size_t)s.nexp, -1), local((size_t)s.nexp, -1);
    for (int32_t g = 0; g < G; ++g) {
        std::vector<int32_t> slots;
        for (int32_t x = s.window[2 * g]; x < s.window[2 * g + 1]; ++x)
            each_col(x, [&](int32_t &c) {
                if (c <= n) return;
                const int32_t slot = c - n - 1;
                if (stamp[slot] != g) {
                    stamp[slot] = g;
                    first_lev[slot] = xlev[x];
                    slots.push_back(slot);
                } else {
                    first_lev[slot] = std::min(first_lev[slot], xlev[x]);
                }
            });
        std::stable_sort(slots.begin(), slots.end(),
                         [&](int32_t p, int32_t q) { return first_lev[p] < first_lev[q]; });
        s.imp_ptr[g] = (int32_t)s.imp_slot.size();
        for (size_t k = 0; k < slots.size(); ++k) {
            local[slots[k]] = (int32_t)k;
            s.imp_slot.push_back(slots[k]);
        }
        s.imp_ptr[g + 1] = (int32_t)s.imp_slot.size();
        const int32_t ni = s.imp_ptr[g + 1] - s.imp_ptr[g];
        s.max_imp = std::max(s.max_imp, ni);
        s.df_rows = std::max(s.df_rows, 2 * (s.window[2 * g + 1] - s.window[2 * g]) + ni + 1);
        s.df_ints = std::max(s.df_ints, ni + (s.exp_ptr[g + 1] - s.exp_ptr[g]) +
                                            2 * (s.step_ptr[g + 1] - s.step_ptr[g]));
        // 3. columns become rows of the group's LDS value area: its own rows
        // 0..win-1, imports from 2*win (after the right-hand-side copy), and a
        // zero row 2*win + nimp for ELL padding (padding then subtracts 0 * 0,
        // which leaves every value unchanged, so no test is needed)
        const int32_t lo = s.window[2 * g], hi = s.window[2 * g + 1], win = hi - lo;
        for (int32_t x = lo; x < hi; ++x)
            each_col(x, [&](int32_t &c) {
                if (c < n) c -= lo;
                else if (c == n) c = 2 * win + ni;
                else c = 2 * win + local[c - n - 1];
            });
    }
    // 4. the steps of each group's wavefronts (contiguous, in wavefront order)
    s.df_waves = waves;
    s.wave_ptr.assign((size_t)G * waves + 1, 0);
    for (int32_t g = 0; g < G; ++g) {
        const int32_t s0 = s.step_ptr[g], ns = s.step_ptr[g + 1] - s0;
        if ((int32_t)run_wave[g].size() != ns) fail(HEC_ERR_INVALID_ARG, "internal: wavefront list mismatch");
        int32_t k = 0;
        for (int32_t w2 = 0; w2 < waves; ++w2) {
            s.wave_ptr[(size_t)g * waves + w2] = s0 + k;
            while (k < ns && run_wave[g][k] == w2) ++k;
        }
        if (k != ns) fail(HEC_ERR_INVALID_ARG, "internal: wavefront pieces out of order");
    }
    s.wave_ptr[(size_t)G * waves] = s.step_ptr[G];
    s.dataflow = true;
}

// Parts of the queue-mode dataflow kernel.  Every independent system (the
// diagonal blocks sys_ptr, or the whole matrix) is cut into contiguous
// ranges of the problem order (ascending rows for a lower triangle,
// descending for an upper one), so a part reads only from earlier parts of
// its own system: numbered system by system, the parts form a queue in
// which each part depends on lower numbers only.  Systems come deepest
// first (most levels, then most rows), so the longest dependency chains
// start first.  A part whose LDS need (solution, right-hand side and imported
// values, plus the index lists, bounded from above) exceeds the workgroup's
// LDS is halved until every part fits.  Returns the part of every row and
// sets `parts`.
std::vector<int32_t> queue_parts(const Csr &a, bool upper, const Levels &lv, const std::vector<int32_t> *sys_ptr,
                                 const Tune &tune, const DeviceShape &dev, hec_dtype_t dt, int32_t &parts)
{
    const int32_t n = a.n;
    std::vector<int32_t> sp = sys_ptr && sys_ptr->size() >= 2 ? *sys_ptr : std::vector<int32_t>{0, n};
    const int32_t nsys = (int32_t)sp.size() - 1;
    const int32_t R = std::max(1, tune.max_nrhs);
    const size_t ts = dt == HEC_F64 ? 8 : 4;
    const size_t cap = dev.lds > 0 ? (size_t)dev.lds : 163840;
    // a first cut: parts of about as many rows as the LDS holds with no imports
    const int32_t prow = tune.part_rows > 0 ? tune.part_rows
                                            : std::max<int32_t>(64, (int32_t)(cap / (2 * R * ts + 16)));
    std::vector<int32_t> depth(nsys, 0);
    for (int32_t q = 0; q < nsys; ++q)
        for (int32_t i = sp[q]; i < sp[q + 1]; ++i) depth[q] = std::max(depth[q], lv.level[i]);
    std::vector<int32_t> order(nsys);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        if (depth[x] != depth[y]) return depth[x] > depth[y];
        return sp[x + 1] - sp[x] > sp[y + 1] - sp[y];
    });
    // ranges of the problem order: [first, last) positions q, row = upper ? n-1-q : q
    std::vector<std::pair<int32_t, int32_t>> ranges;
    for (int32_t sy : order) {
        const int32_t m = sp[sy + 1] - sp[sy];
        if (m <= 0) continue;
        const int32_t q0 = upper ? n - sp[sy + 1] : sp[sy];
        const int32_t k = (m + prow - 1) / prow;
        for (int32_t c = 0; c < k; ++c)
            ranges.push_back({q0 + (int32_t)((int64_t)m * c / k), q0 + (int32_t)((int64_t)m * (c + 1) / k)});
    }
    auto row_at = [&](int32_t q) { return upper ? n - 1 - q : q; };
    std::vector<int32_t> stamp(n, -1), seen(n, -1);
    auto need = [&](int32_t q0, int32_t q1, int32_t tag) {
        for (int32_t q = q0; q < q1; ++q) stamp[row_at(q)] = tag;
        int64_t nimp = 0;
        for (int32_t q = q0; q < q1; ++q) {
            const int32_t i = row_at(q);
            for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
                const int32_t j = a.ci[p];
                if (j == i || stamp[j] == tag || seen[j] == tag) continue;
                seen[j] = tag;
                ++nimp;
            }
        }
        const int64_t win = q1 - q0;
        return (size_t)(2 * win + nimp + 1) * R * ts + 4 * (size_t)(nimp + 3 * win) + 64;
    };
    std::vector<std::pair<int32_t, int32_t>> out;
    int32_t tag = 0;
    for (size_t r = 0; r < ranges.size(); ++r) {
        std::vector<std::pair<int32_t, int32_t>> work{ranges[r]};
        while (!work.empty()) {
            auto cur = work.back();
            work.pop_back();
            if (cur.second - cur.first > 1 && need(cur.first, cur.second, tag++) > cap) {
                const int32_t mid = cur.first + (cur.second - cur.first) / 2;
                work.push_back({mid, cur.second});  // processed after the first half
                work.push_back({cur.first, mid});
                continue;
            }
            out.push_back(cur);
        }
    }
    std::vector<int32_t> po(n, 0);
    for (size_t g = 0; g < out.size(); ++g)
        for (int32_t q = out[g].first; q < out[g].second; ++q) po[row_at(q)] = (int32_t)g;
    parts = std::max<int32_t>(1, (int32_t)out.size());
    return po;
}

// System queue: every column becomes a row of its system's LDS ring, which
// holds the last D+1 levels of the system (D = the largest level distance of
// a dependency in it) in D+1 slots of W rows (W = its widest level): a value
// of local level l sits in slot l mod (D+1).  If the ring of a system does
// not fit the LDS, D shrinks and the dependencies further back are read from
// the global workspace instead (column -2 - device row).  ELL padding becomes
// kSqPad, which the kernel maps to a zero row after the ring.
constexpr int32_t kSqPad = INT32_MAX;

void build_sysq(ExecHost &ex, const Levels &lv, const std::vector<int32_t> &sys, const std::vector<int32_t> &lvrow,
                const std::vector<int32_t> &lvp, int32_t R, size_t ts, const DeviceShape &dev)
{
    (void)lv;
    const int32_t n = ex.n, S = (int32_t)sys.size();
    Schedule &s = ex.sched;
    s.sysq = true;
    s.groups = S;
    s.sq_lvrow = lvrow;
    s.sq_lvp = lvp;
    s.sq_ring.assign(2 * (size_t)S, 0);
    std::vector<int32_t> lev_of(n, 0), sys_of(n, 0);  // local level, queue position of each device row
    for (int32_t k = 0; k < S; ++k)
        for (int32_t l = lvp[k]; l < lvp[k + 1]; ++l)
            for (int32_t x = lvrow[l]; x < lvrow[l + 1]; ++x) {
                lev_of[x] = l - lvp[k];
                sys_of[x] = k;
            }
    auto each_col = [&](int32_t x, const std::function<void(int32_t &)> &f) {
        for (int32_t e = 0; e < ex.w; ++e) f(ex.ell_col[(size_t)e * ex.ld + x]);
        if (!ex.tail_ptr.empty())
            for (int32_t p = ex.tail_ptr[x]; p < ex.tail_ptr[x + 1]; ++p) f(ex.tail_col[p]);
    };
    const size_t cap = dev.lds > 0 ? (size_t)dev.lds : 163840;
    std::vector<int32_t> D(S, 0), W(S, 1);
    for (int32_t k = 0; k < S; ++k) {
        for (int32_t l = lvp[k]; l < lvp[k + 1]; ++l) W[k] = std::max(W[k], lvrow[l + 1] - lvrow[l]);
        for (int32_t l = lvp[k]; l < lvp[k + 1]; ++l)
            for (int32_t x = lvrow[l]; x < lvrow[l + 1]; ++x)
                each_col(x, [&](int32_t &c) {
                    if (c < n) D[k] = std::max(D[k], lev_of[x] - lev_of[c]);
                });
        // shrink the ring until it fits (global reads beyond it)
        while (D[k] > 0 && ((size_t)(D[k] + 1) * W[k] + 1) * R * ts > cap) --D[k];
        if (((size_t)(D[k] + 1) * W[k] + 1) * R * ts > cap) D[k] = -1;  // not even one level: all global
    }
    s.sq_global = false;
    int64_t lds_rows = 1;
    for (int32_t k = 0; k < S; ++k) {
        const int32_t slots = D[k] + 1;  // 0: no ring
        s.sq_ring[2 * k] = slots;
        s.sq_ring[2 * k + 1] = W[k];
        lds_rows = std::max<int64_t>(lds_rows, (int64_t)slots * W[k] + 1);
    }
    s.sq_keep.assign(n, 0);
    for (int32_t x = 0; x < n; ++x) {
        const int32_t k = sys_of[x];
        each_col(x, [&](int32_t &c) {
            if (c >= n) {
                c = kSqPad;
                return;
            }
            if (sys_of[c] != k) fail(HEC_ERR_INVALID_ARG, "internal: a dependency crosses two systems");
            const int32_t dist = lev_of[x] - lev_of[c];
            if (dist <= D[k]) {
                const int32_t l = lvp[k] + lev_of[c];
                c = (lev_of[c] % (D[k] + 1)) * W[k] + (c - lvrow[l]);
            } else {
                s.sq_keep[c] = 1;
                c = -2 - c;
                s.sq_global = true;
            }
        });
    }
    s.sq_lds_rows = (int32_t)lds_rows;
    s.window.assign(2 * (size_t)S, 0);
    s.step_ptr.assign((size_t)S + 1, 0);
    s.exp_ptr.assign((size_t)S + 1, 0);
    s.exp_slot.assign(n, -1);
    s.nexp = 0;
}

}  // namespace

void build_exec(TriHost &t, const Csr &a, const Tune &tune, const DeviceShape &dev,
                const std::vector<int32_t> *sys_ptr)
{
    (void)sys_ptr;
    const int32_t n = t.n;
    const Levels &lv = t.lev;
    const HecHost &h = t.hec;
    ExecHost &ex = t.ex;
    ex = ExecHost();
    ex.n = n;
    ex.w = h.w;
    ex.ld = h.ld;
    int32_t kind = tune.schedule;
    if (kind == HEC_SCHED_AUTO) kind = HEC_SCHED_LEVEL_PERSISTENT;
    const int32_t groups_cap = dev.groups_cap;
    const int32_t cap = groups_cap > 0 ? groups_cap : 256;
    const int32_t cus = dev.cus > 0 ? dev.cus : 256;
    // one workgroup per CU by default: every workgroup of a persistent grid
    // must be resident at once, and one per CU does not lean on the last
    // wavefront slot the occupancy query promises
    int32_t G = tune.num_groups > 0 ? tune.num_groups : std::min(cap, cus);
    if (tune.num_groups > 0 && groups_cap > 0 && tune.num_groups > groups_cap)
        fail(HEC_ERR_CAPACITY, "num_groups " + std::to_string(tune.num_groups) +
                                   " exceeds the co-resident capacity " + std::to_string(groups_cap));
    G = std::max(1, G);
    const int32_t R = std::max(1, tune.max_nrhs);
    const int32_t merge = tune.merge_rows > 0 ? tune.merge_rows : std::max(1, tune.block_threads / R);
    // the dataflow owner kernel: one wavefront per piece of a part
    const bool want_df = kind == HEC_SCHED_OWNER_PERSISTENT && (tune.variant == 4 || tune.variant == 6);
    const bool queue = want_df && tune.variant == 6;
    const int32_t df_waves = std::max(1, tune.block_threads / 64);
    std::vector<std::vector<int32_t>> run_wave;  // dataflow: wavefront of each run

    // 1. device-row order and owner of each row
    ex.xord.resize(n);
    ex.owner.assign(n, 0);
    std::vector<std::vector<std::pair<int32_t, int32_t>>> runs;
    const bool sysq = tune.variant == 7;
    std::vector<int32_t> sq_sys, sq_lvrow, sq_lvp;  // system queue: systems in queue order, level bounds
    if (sysq) {
        // one workgroup per independent system: device rows system by system
        // in queue order (longest first), each system in level order
        std::vector<int32_t> sp = sys_ptr && sys_ptr->size() >= 2 ? *sys_ptr : std::vector<int32_t>{0, n};
        const int32_t S = (int32_t)sp.size() - 1;
        const int32_t nt = std::max(64, tune.block_threads);
        std::vector<std::vector<int32_t>> width(S);
        for (int32_t q = 0; q < S; ++q)
            for (int32_t i = sp[q]; i < sp[q + 1]; ++i) {
                const int32_t l = lv.level[i] - 1;
                if ((int32_t)width[q].size() <= l) width[q].resize(l + 1, 0);
                width[q][l] += 1;
            }
        std::vector<int64_t> est(S, 0);
        for (int32_t q = 0; q < S; ++q)
            for (int32_t w2 : width[q]) est[q] += 1 + ((int64_t)w2 * R) / nt;
        sq_sys.resize(S);
        std::iota(sq_sys.begin(), sq_sys.end(), 0);
        std::stable_sort(sq_sys.begin(), sq_sys.end(), [&](int32_t x, int32_t y) { return est[x] > est[y]; });
        // rows of each system by (level, problem order): a stable sort of the
        // level order (lv.perm lists rows by level, problem order inside)
        std::vector<int32_t> sys_of(n);
        for (int32_t q = 0; q < S; ++q)
            for (int32_t i = sp[q]; i < sp[q + 1]; ++i) sys_of[i] = q;
        std::vector<int32_t> rank(S);
        for (int32_t k = 0; k < S; ++k) rank[sq_sys[k]] = k;
        std::vector<int32_t> cnt(S + 1, 0);
        for (int32_t i = 0; i < n; ++i) cnt[rank[sys_of[i]] + 1] += 1;
        for (int32_t k = 0; k < S; ++k) cnt[k + 1] += cnt[k];
        std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
        for (int32_t r = 0; r < n; ++r) {  // r: level-order row
            const int32_t i = lv.perm[r];
            ex.xord[pos[rank[sys_of[i]]]++] = r;
        }
        sq_lvp.assign(1, 0);
        sq_lvrow.clear();
        for (int32_t k = 0; k < S; ++k) {
            const int32_t q = sq_sys[k];
            int32_t row = cnt[k];
            for (int32_t w2 : width[q]) {
                sq_lvrow.push_back(row);
                row += w2;
            }
            sq_lvp.push_back((int32_t)sq_lvrow.size());
        }
        sq_lvrow.push_back(n);
        for (int32_t x = 0; x < n; ++x) ex.owner[x] = 0;
    } else if (kind == HEC_SCHED_LEVEL_LAUNCH || kind == HEC_SCHED_LEVEL_PERSISTENT) {
        std::iota(ex.xord.begin(), ex.xord.end(), 0);
        ex.levelptr = lv.levelptr;
        if (kind == HEC_SCHED_LEVEL_PERSISTENT) {
            runs.assign(G, {});
            for (int32_t k = 0; k < lv.nlev; ++k) {
                int32_t b = lv.levelptr[k], e = lv.levelptr[k + 1], nk = e - b;
                int32_t nch = std::max(1, std::min(G, nk / merge));
                for (int32_t c = 0; c < nch; ++c) {
                    int32_t cb = b + (int32_t)((int64_t)nk * c / nch);
                    int32_t ce = b + (int32_t)((int64_t)nk * (c + 1) / nch);
                    if (ce > cb) {
                        runs[c].push_back({cb, ce});
                        for (int32_t x = cb; x < ce; ++x) ex.owner[x] = c;
                    }
                }
            }
        }
    } else {
        // owner schedule: each group owns one part of the rows and solves it
        // level by level.  Parts come from recursive graph bisection (compact
        // parts: few dependency edges and few group-to-group handoffs along
        // any chain) or, on request, from contiguous ranges of the problem
        // order (natural order for L, reversed for U).
        int32_t parts = G;
        if (tune.part_rows > 0) parts = std::min(G, std::max(1, (n + tune.part_rows - 1) / tune.part_rows));
        parts = std::max(1, std::min(parts, std::max(1, n)));
        std::vector<int32_t> part_of;
        int32_t gx = 0, gy = 0, gz = 0;
        const bool grid = !queue && (tune.partition == 0 || tune.partition == 3) && detect_grid(a, gx, gy, gz);
        auto contiguous = [&]() {
            std::vector<int32_t> po(n);
            for (int32_t g = 0; g < parts; ++g) {
                int32_t qb = (int32_t)((int64_t)n * g / parts), qe = (int32_t)((int64_t)n * (g + 1) / parts);
                for (int32_t q = qb; q < qe; ++q) po[t.upper ? n - 1 - q : q] = g;
            }
            return po;
        };
        if (queue) {
            part_of = queue_parts(a, t.upper, lv, sys_ptr, tune, dev, t.dt, parts);
        } else if (grid) {
            part_of = grid_parts(n, gx, gy, gz, parts);
            if (tune.partition == 0) {
                // automatic: grid blocks unless contiguous ranges put fewer
                // workgroup handoffs on the longest dependency chain (fill-in
                // can make chains wander across block faces)
                std::vector<int32_t> po = contiguous();
                if (critical_hops(a, t.upper, po) < critical_hops(a, t.upper, part_of)) part_of.swap(po);
            }
        } else if (tune.partition != 2) {
            part_of = contiguous();
        } else {
            part_of = bisect_parts(a, parts);
        }
        std::vector<std::vector<int32_t>> members(parts);
        for (int32_t q = 0; q < n; ++q) {
            const int32_t i = t.upper ? n - 1 - q : q;  // problem order
            members[part_of[i]].push_back(i);
        }
        runs.assign(parts, {});
        run_wave.assign(parts, {});
        int32_t x = 0;
        for (int32_t g = 0; g < parts; ++g) {
            // rows of the part in level order, ties by problem index.  For the
            // dataflow kernel the part is first cut into one contiguous piece
            // (in problem order) per compute wavefront, each in level order:
            // a wavefront then walks its own piece, and only dependencies
            // between pieces need a wait.
            std::vector<int32_t> &rows = members[g];
            const int32_t pieces = want_df ? df_waves : 1;
            const size_t m = rows.size();
            for (int32_t w2 = 0; w2 < pieces; ++w2) {
                const size_t pb = m * w2 / pieces, pe = m * (w2 + 1) / pieces;
                std::stable_sort(rows.begin() + pb, rows.begin() + pe,
                                 [&](int32_t i, int32_t j) { return lv.level[i] < lv.level[j]; });
                int32_t start = x;
                for (size_t u = pb; u < pe; ++u) {
                    ex.xord[x] = lv.iperm[rows[u]];
                    ex.owner[x] = g;
                    if (u > pb && lv.level[rows[u]] != lv.level[rows[u - 1]]) {
                        runs[g].push_back({start, x});
                        run_wave[g].push_back(w2);
                        start = x;
                    }
                    ++x;
                }
                if (x > start) {
                    runs[g].push_back({start, x});
                    run_wave[g].push_back(w2);
                }
            }
        }
        // Consecutive parts depend on each other; give them workgroups that
        // share an L2 domain (workgroup i runs on domain i % xcds), so that
        // most part-to-part handoffs stay inside one XCD.
        const int32_t X = std::max(1, dev.xcds);
        if (!queue && parts % X == 0 && parts >= X) {
            const int32_t per = parts / X;
            std::vector<int32_t> gid(parts);
            for (int32_t p = 0; p < parts; ++p) gid[p] = (p % per) * X + p / per;
            std::vector<std::vector<std::pair<int32_t, int32_t>>> relabeled(parts);
            std::vector<std::vector<int32_t>> rw(parts);
            for (int32_t p = 0; p < parts; ++p) {
                relabeled[gid[p]] = std::move(runs[p]);
                rw[gid[p]] = std::move(run_wave[p]);
            }
            runs.swap(relabeled);
            run_wave.swap(rw);
            for (int32_t x2 = 0; x2 < n; ++x2) ex.owner[x2] = gid[ex.owner[x2]];
        }
    }
    ex.xinv.assign(n, 0);
    for (int32_t x = 0; x < n; ++x) ex.xinv[ex.xord[x]] = x;
    ex.orig.resize(n);
    for (int32_t x = 0; x < n; ++x) ex.orig[x] = lv.perm[ex.xord[x]];

    // 2. HEC in device order; the diagonal goes to its own array
    const int32_t w = h.w, ld = h.ld;
    ex.ell_col.assign((size_t)w * ld, n);
    ex.ell_val.assign((size_t)w * ld, 0.0);
    bool has_tail = false;
    for (int32_t r = 0; r < n; ++r)
        if (h.csr_ptr[r + 1] - h.csr_ptr[r] > 1) { has_tail = true; break; }
    if (has_tail) ex.tail_ptr.assign((size_t)n + 1, 0);
    if (!t.unit) ex.dinv.resize(n);
    for (int32_t x = 0; x < n; ++x) {
        int32_t r = ex.xord[x];
        for (int32_t e = 0; e < w; ++e) {
            int32_t c = h.ell_col[(size_t)e * ld + r];
            ex.ell_col[(size_t)e * ld + x] = (c == n) ? n : ex.xinv[c];
            ex.ell_val[(size_t)e * ld + x] = h.ell_val[(size_t)e * ld + r];
        }
        int32_t pb = h.csr_ptr[r], pe = h.csr_ptr[r + 1] - 1;  // last entry: diagonal
        if (has_tail) {
            for (int32_t p = pb; p < pe; ++p) {
                ex.tail_col.push_back(ex.xinv[h.csr_col[p]]);
                ex.tail_val.push_back(h.csr_val[p]);
            }
            ex.tail_ptr[x + 1] = (int32_t)ex.tail_col.size();
        }
        if (!t.unit) ex.dinv[x] = 1.0 / h.csr_val[pe];
    }
    t.nnz_tail = (int64_t)ex.tail_col.size();
    // Fold the reciprocal diagonal into the row: x = d b - sum (d a_j) x_j, so
    // the kernels scale b once when they read it and the dependency chain of
    // a row ends with its last multiply-add (no trailing multiply).
    if (!t.unit) {
        for (int32_t x = 0; x < n; ++x) {
            for (int32_t e = 0; e < w; ++e) ex.ell_val[(size_t)e * ld + x] *= ex.dinv[x];
            if (has_tail)
                for (int32_t p = ex.tail_ptr[x]; p < ex.tail_ptr[x + 1]; ++p) ex.tail_val[p] *= ex.dinv[x];
        }
    }

    // 3. schedule
    ex.sched = Schedule();
    ex.sched.kind = kind;
    if (sysq) {
        build_sysq(ex, lv, sq_sys, sq_lvrow, sq_lvp, R, t.dt == HEC_F64 ? 8 : 4, dev);
        return;
    }
    // the dataflow owner kernel runs each step as one wavefront's unit (at
    // most 64 (row, rhs) items); the other owner kernels cut steps to chunks
    if (want_df && dataflow_width(w) != w)
        fail(HEC_ERR_INVALID_ARG, "dataflow kernel: ELL width must be 1..8, 10, 12 or 16");
    if (want_df && R > 64) fail(HEC_ERR_INVALID_ARG, "dataflow kernel: max_nrhs above 64");
    if (want_df && (size_t)w * ld * 8 > (size_t)INT32_MAX)
        fail(HEC_ERR_CAPACITY, "dataflow kernel: ELL part beyond 2 GiB (32-bit buffer offsets)");
    if (want_df && tune.block_threads > dataflow_max_block(w) - 128)
        fail(HEC_ERR_CAPACITY, "dataflow kernel: block_threads above " + std::to_string(dataflow_max_block(w) - 128) +
                                   " for ELL width " + std::to_string(w) + " (two more wavefronts are added)");
    if (kind == HEC_SCHED_OWNER_PERSISTENT) {
        const int32_t piece = want_df ? std::max(1, 64 / R) : tune.chunk_rows;
        if (piece <= 0) fail(HEC_ERR_INVALID_ARG, "internal: chunk_rows must be positive");
        // cut longer levels into pieces (rows of one level are independent)
        for (size_t g = 0; g < runs.size(); ++g) {
            std::vector<std::pair<int32_t, int32_t>> cut;
            std::vector<int32_t> cw;
            for (size_t k = 0; k < runs[g].size(); ++k) {
                const auto &r = runs[g][k];
                for (int32_t b = r.first; b < r.second; b += piece) {
                    cut.push_back({b, std::min(r.second, b + piece)});
                    if (want_df) cw.push_back(run_wave[g][k]);
                }
            }
            runs[g].swap(cut);
            if (want_df) run_wave[g].swap(cw);
        }
    }
    if (kind != HEC_SCHED_LEVEL_LAUNCH) {
        Tune tu = tune;
        if (want_df) tu.group_lanes = 1;  // one lane per (row, rhs): tails are summed serially
        finish_schedule(ex.sched, ex, runs, tu);
        if (want_df) {
            std::vector<int32_t> xlev(n);
            for (int32_t x2 = 0; x2 < n; ++x2) xlev[x2] = lv.level[ex.orig[x2]];
            make_dataflow(ex.sched, ex, xlev, run_wave, df_waves);
            ex.sched.queue = queue;
            const size_t lds_cap = dev.lds > 0 ? (size_t)dev.lds : 163840;
            const size_t need = dataflow_lds_bytes(ex.sched.df_rows, ex.sched.df_ints, R, t.dt == HEC_F64 ? 8 : 4);
            if (need > lds_cap)
                fail(HEC_ERR_CAPACITY, "dataflow kernel: a group needs " + std::to_string(need) +
                                           " bytes of LDS (use more groups or fewer right-hand sides)");
        }
        std::vector<int32_t> own(n);
        for (int32_t x2 = 0; x2 < n; ++x2) own[ex.orig[x2]] = ex.owner[x2];
        ex.sched.crit_hops = critical_hops(a, t.upper, own);
    }
}

TriHost analyze(const Csr &a, bool upper, bool unit, hec_dtype_t dt, const Tune &tune, const DeviceShape &dev,
                const std::vector<int32_t> *sys_ptr)
{
    validate_triangle(a, upper, unit);
    TriHost t;
    t.n = a.n;
    t.upper = upper;
    t.unit = unit;
    t.dt = dt;
    t.lev = compute_levels(a, upper);
    int64_t off = 0;
    for (int32_t i = 0; i < a.n; ++i) off += offdiag_count(a, i);
    t.nnz_off = off;
    auto attempt = [&](const Tune &u) {
        int32_t w = u.ell_width >= 0 ? u.ell_width : auto_ell_width(a, upper);
        // The dataflow kernel holds the ELL slots of a row in registers (widths
        // 1..8, 10, 12, 16).  Its CSR tail is read with an exposed load
        // latency on the dependency chain, so the automatic width covers the
        // longest row when that fits; padding costs bytes, not latency.
        if ((u.variant == 4 || u.variant == 6) && u.schedule == HEC_SCHED_OWNER_PERSISTENT) {
            if (u.ell_width < 0) {
                int32_t wmax = 0;
                for (int32_t i = 0; i < a.n; ++i) wmax = std::max(wmax, offdiag_count(a, i));
                w = std::min(std::max(w, wmax), 16);
            }
            w = dataflow_width(std::min(std::max(w, 1), 16));
        }
        // The pipelined system queue holds a row's ELL slots in registers and
        // reads no CSR tail: the automatic width covers the longest row when
        // it has at most 8 off-diagonals.
        if (u.variant == 7 && u.ell_width < 0) {
            int32_t wmax = 0;
            for (int32_t i = 0; i < a.n; ++i) wmax = std::max(wmax, offdiag_count(a, i));
            if (wmax <= 8) w = std::max(w, std::max(wmax, 1));
        }
        t.hec = build_hec(a, upper, unit, t.lev, w);
        build_exec(t, a, u, dev, sys_ptr);
    };
    // Automatic schedule: the owner schedule on the dataflow kernel when its
    // LDS holds every part (rows x right-hand sides); otherwise the system is
    // large, its levels are wide, and one launch per level keeps the whole
    // GPU busy without any cross-workgroup waits.  An explicit owner
    // schedule without a kernel choice falls back to the LDS-chunked kernel.
    Tune tu = tune;
    t.variant = tu.variant;
    if (tu.variant == 5) {  // the barrier-free kernel over the level-ordered layout
        tu.schedule = HEC_SCHED_LEVEL_LAUNCH;
        attempt(tu);
        return t;
    }
    const bool auto_sched = tu.schedule == HEC_SCHED_AUTO;
    if (auto_sched) tu.schedule = HEC_SCHED_OWNER_PERSISTENT;
    if (tu.variant == 7) {  // the system queue: one workgroup per independent system
        if (tu.schedule != HEC_SCHED_LEVEL_PERSISTENT)
            fail(HEC_ERR_INVALID_ARG, "kernel_variant 7 runs the level schedule (schedule AUTO or LEVEL_PERSISTENT)");
        attempt(tu);
        return t;
    }
    if (tu.variant == 6) {
        if (tu.schedule != HEC_SCHED_OWNER_PERSISTENT)
            fail(HEC_ERR_INVALID_ARG, "kernel_variant 6 runs the owner schedule (schedule AUTO or OWNER_PERSISTENT)");
        attempt(tu);
        return t;
    }
    if (tu.schedule == HEC_SCHED_OWNER_PERSISTENT && tu.variant == 0) {
        Tune d = tu;
        d.variant = 4;
        const bool df_ok = d.block_threads <= 384 && d.max_nrhs <= 64 && d.ell_width <= 16;
        if (df_ok) {
            try {
                attempt(d);
                return t;
            } catch (const Error &e) {
                if (e.code != HEC_ERR_CAPACITY) throw;
            }
        }
        // too large for LDS with enough independent systems to give every
        // other compute unit one (a batch, RAS subdomains): the system
        // queue, whose levels are separated by workgroup barriers with the
        // last levels' values in LDS (256 systems of ILU(1), 8 RHS: 4.2 ms
        // FP32 against 7.4 ms for the barrier-free kernel; 64 subdomains
        // leave most of the GPU idle and stay on the barrier-free kernel)
        const int32_t nsys = sys_ptr && sys_ptr->size() >= 2 ? (int32_t)sys_ptr->size() - 1 : 1;
        if (auto_sched && nsys >= std::max(2, (dev.cus > 0 ? dev.cus : 256) / 2) && tu.max_nrhs <= 64) {
            Tune q = tu;
            q.schedule = HEC_SCHED_LEVEL_PERSISTENT;
            q.variant = 7;
            t.variant = 7;
            attempt(q);
            return t;
        }
        if (auto_sched) {
            // too large for LDS: the barrier-free kernel (its per-level cost
            // is one memory round trip; measured faster than one launch per
            // level up to 256k (row, rhs) items per level), one launch per
            // level only when levels average above 2^20 items
            tu.schedule = HEC_SCHED_LEVEL_LAUNCH;
            const double items = (double)a.n * std::max(1, tu.max_nrhs);
            if (items < (double)(1 << 20) * std::max(1, t.lev.nlev)) t.variant = tu.variant = 5;
        } else {
            tu.variant = 2;
        }
    }
    attempt(tu);
    return t;
}

}  // namespace hec
