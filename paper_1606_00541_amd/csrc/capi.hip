// C ABI of the HEC triangular-solve library (declared in include/hec.h):
// plan construction (Algorithm 1), device upload, the solves of Algorithm 2,
// the ILU / RAS / batched preconditioners of Section 3 and graph capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <cstdlib>
#include <cstdio>
#include <chrono>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <new>

#include "hec_dev.h"

namespace hec {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string &m) { g_last_error = m; }

void hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess) return;
    (void)hipGetLastError();
    if (e == hipErrorNoDevice || e == hipErrorInvalidDevice)
        fail(HEC_ERR_NO_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        fail(HEC_ERR_ALLOC, std::string(what) + ": " + hipGetErrorString(e));
    fail(HEC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

void DevMem::alloc(size_t b)
{
    release();
    if (b == 0) return;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, b);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(HEC_ERR_ALLOC, "hipMalloc of " + std::to_string(b) + " bytes failed");
    }
    p = q;
    bytes = b;
}

void upload_values(DevMem &m, const std::vector<double> &v, hec_dtype_t dt)
{
    if (dt == HEC_F64) {
        upload(m, v);
    } else {
        std::vector<float> f(v.begin(), v.end());
        upload(m, f);
    }
}

DevTri::~DevTri()
{
    if (err_host) (void)hipHostFree(err_host);
}

static size_t vsize(hec_dtype_t dt) { return dt == HEC_F64 ? 8 : 4; }

void ensure_workspace(DevTri &d, int32_t R)
{
    if (R <= d.ws_R) return;
    d.xw.alloc(((size_t)d.n + 1) * R * vsize(d.dt));
    if (d.nexp > 0) {
        // both halves start empty; the stride stays the allocated width so
        // that every launch resets exactly what any later launch may read
        const size_t cnt = 2 * (size_t)d.nexp * R;
        d.mbox.alloc(cnt * vsize(d.dt));
        fill_sentinel(d.mbox.p, cnt, d.dt);
    }
    d.ws_R = R;
}

void upload_tri(DevTri &d, const TriHost &t, int32_t max_nrhs)
{
    hip_check(hipGetDevice(&d.device), "hipGetDevice");
    const ExecHost &ex = t.ex;
    d.n = t.n;
    d.w = ex.w;
    d.ld = ex.ld;
    d.nlev = t.lev.nlev;
    d.dt = t.dt;
    d.kind = ex.sched.kind;
    d.unit = t.unit;
    d.has_tail = !ex.tail_ptr.empty();
    upload(d.ell_col, ex.ell_col);
    upload_values(d.ell_val, ex.ell_val, t.dt);
    if (d.has_tail) {
        upload(d.tail_ptr, ex.tail_ptr);
        upload(d.tail_col, ex.tail_col);
        upload_values(d.tail_val, ex.tail_val, t.dt);
    }
    if (!t.unit) upload_values(d.dinv, ex.dinv, t.dt);
    upload(d.orig, ex.orig);
    d.levelptr = ex.levelptr;
    if (d.kind != HEC_SCHED_LEVEL_LAUNCH) {
        const Schedule &s = ex.sched;
        d.groups = s.groups;
        d.max_window = s.max_window;
        upload(d.step_ptr, s.step_ptr);
        upload(d.step_row, s.step_row);
        upload(d.step_lanes, s.step_lanes);
        upload(d.window, s.window);
        d.nexp = s.nexp;
        upload(d.exp_slot, s.exp_slot);
        upload(d.exp_ptr, s.exp_ptr);
        upload(d.chunk_ptr, s.chunk_ptr);
        upload(d.chunk_step, s.chunk_step);
        upload(d.rem_ptr, s.rem_ptr);
        std::vector<int32_t> re = s.rem_ent;
        if (re.empty()) re.assign(2, 0);
        upload(d.rem_ent, re);
        d.chunk_rows = s.chunk_rows;
        d.dataflow = s.dataflow;
        if (s.dataflow) {
            upload(d.imp_ptr, s.imp_ptr);
            std::vector<int32_t> v = s.imp_slot;
            if (v.empty()) v.assign(1, 0);
            upload(d.imp_slot, v);
            v = s.exp_row;
            if (v.empty()) v.assign(1, 0);
            upload(d.exp_row, v);
            d.df_rows = s.df_rows;
            d.df_ints = s.df_ints;
            d.df_waves = s.df_waves;
            d.queue = s.queue;
            upload(d.wave_ptr, s.wave_ptr);
            d.df_step_rows = 0;
            for (int32_t q = 0; q < s.nsteps(); ++q)
                d.df_step_rows = std::max(d.df_step_rows, s.step_row[2 * q + 1] - s.step_row[2 * q]);
        }
        d.max_lanes_one = std::all_of(s.step_lanes.begin(), s.step_lanes.end(), [](int32_t v) { return v == 1; });
        if (s.sysq) {
            d.sysq = true;
            d.sq_global = s.sq_global;
            d.sq_lds_rows = s.sq_lds_rows;
            d.sq_widths.clear();
            for (size_t l = 0; l + 1 < s.sq_lvrow.size(); ++l) d.sq_widths.push_back(s.sq_lvrow[l + 1] - s.sq_lvrow[l]);
            d.sq_median_rows = 0;
            if (!d.sq_widths.empty()) {
                std::vector<int32_t> w = d.sq_widths;
                std::nth_element(w.begin(), w.begin() + w.size() / 2, w.end());
                d.sq_median_rows = w[w.size() / 2];
            }
            upload(d.sq_lvp, s.sq_lvp);
            upload(d.sq_lvrow, s.sq_lvrow);
            upload(d.sq_ring, s.sq_ring);
            upload(d.sq_keep, s.sq_keep);
        }
    }
    // epoch, workgroups done, work counter (part queue / chunk batches)
    d.epoch.alloc(4 * sizeof(unsigned int));
    hip_check(hipMemset(d.epoch.p, 0, d.epoch.bytes), "hipMemset");
    d.err.alloc(sizeof(int));
    hip_check(hipMemset(d.err.p, 0, sizeof(int)), "hipMemset");
    void *hp = nullptr;
    hip_check(hipHostMalloc(&hp, sizeof(int), hipHostMallocMapped), "hipHostMalloc");
    *static_cast<volatile int *>(hp) = 0;
    void *dp = nullptr;
    hip_check(hipHostGetDevicePointer(&dp, hp, 0), "hipHostGetDevicePointer");
    d.err_host = static_cast<int *>(dp);
    ensure_workspace(d, std::max(1, max_nrhs));
    hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
}

namespace {
// Read and clear a plan's abort flags; true if a launch had aborted.
bool take_abort(const DevTri &d)
{
    if (!d.err_host) return false;
    volatile int *f = d.err_host;
    if (*f == 0) return false;
    *f = 0;
    (void)hipMemset(d.err.p, 0, sizeof(int));
    return true;
}
}  // namespace

// Launches of the plan may still be in flight when an abort is seen (the
// host issues work ahead): let them finish, so that none raises the flag
// again after it is cleared, then clear and report once.
static bool abort_seen(const DevTri &d) { return d.err_host && *static_cast<volatile int *>(d.err_host) != 0; }

void check_device_error(const DevTri &d)
{
    if (!abort_seen(d)) return;
    (void)hipDeviceSynchronize();
    take_abort(d);
    fail(HEC_ERR_TIMEOUT, "a persistent solve aborted a device-side wait (spin limit reached)");
}

void check_device_error(const DevTri &a, const DevTri &b)
{
    if (!abort_seen(a) && !abort_seen(b)) return;
    (void)hipDeviceSynchronize();
    take_abort(a);  // both cleared: one report per abort
    take_abort(b);
    fail(HEC_ERR_TIMEOUT, "a persistent solve aborted a device-side wait (spin limit reached)");
}

}  // namespace hec

using namespace hec;

namespace hec {
// dst[t] = src[idx[t]] on the device (refactor.hip)
void gather_f64(const double *src, const int32_t *idx, int64_t cnt, double *dst, hipStream_t st);
}  // namespace hec

struct tri_plan_s {
    TriHost h;
    DevTri d;
    bool on_device = false;
    bool upper = false;
};

struct ilu_s {
    int32_t n = 0;
    hec_dtype_t fdt = HEC_F64;
    Csr Lf, Uf;                  // host FP64 factors
    tri_plan_s L, U;
    DevMem qmap;                 // U device row -> L device row of the same original row
    std::vector<int32_t> sys_ptr;
    hec_ilu_kind_t kind = HEC_ILU0;
    std::unique_ptr<DevRefactor> rf;  // device refactorization data (built on first use)
    bool dev_newer = false;      // the device factors are newer than Lf, Uf
};

struct sor_s {
    int32_t n = 0;
    double omega = 1.0;
    tri_plan_s fwd, bwd;         // D/omega + L (lower), D/omega + U (upper)
    DevHec nf, nb;               // U + (1 - 1/omega) D, L + (1 - 1/omega) D
    DevMem t;                    // right-hand side of the current sweep, [n][R]
    int32_t t_R = 0;
};

struct ras_s {
    int32_t n = 0, nsub = 0;
    RasLayout lay;
    ilu_s f;                     // factors of the block-diagonal matrix
    // device refactorization: A's pattern, each block-diagonal entry's index in A's
    // values, and the gathered block-diagonal values
    std::vector<int32_t> a_rp, a_ci;
    DevMem a2bd, bdval;
    DevMem gather_L;             // L device row -> global row of r
    DevMem scatter_U;            // U device row -> global row of z, or -1 when not owned
};

struct hec_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~hec_graph_s()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace {

DeviceShape device_shape(const Tune &tu, hec_dtype_t dt)
{
    DeviceShape s;
    if (tu.host_only) return s;
    s.groups_cap = persistent_capacity(dt, tu.block_threads, 0);
    s.cus = device_cus();
    s.xcds = 8;
    s.lds = device_max_lds();
    return s;
}

// blocks: independent diagonal blocks (batched systems, RAS subdomains) that
// the owner schedule's queue mode cuts into parts separately
void build_plan(tri_plan_s &p, const Csr &a, bool upper, bool unit, hec_dtype_t dt, const Tune &tu,
                const std::vector<int32_t> *blocks = nullptr)
{
    p.upper = upper;
    p.h = analyze(a, upper, unit, dt, tu, device_shape(tu, dt), blocks);
    p.d.block = tu.block_threads;
    p.d.variant = p.h.variant;
    if (!tu.host_only) {
        upload_tri(p.d, p.h, tu.max_nrhs);
        p.on_device = true;
    }
}

void require_device(const tri_plan_s &p)
{
    if (!p.on_device) fail(HEC_ERR_NO_DEVICE, "plan was built host-only");
    int dev = -1;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev != p.d.device) fail(HEC_ERR_INVALID_ARG, "current device differs from the plan's device");
}

void check_vec(hec_dtype_t dt)
{
    if (dt != HEC_F64 && dt != HEC_F32) fail(HEC_ERR_INVALID_ARG, "vector dtype must be HEC_F64 or HEC_F32");
}

void solve_one(tri_plan_s *p, const void *b, void *x, int32_t nrhs, hec_dtype_t vdt, hipStream_t st, bool upper)
{
    if (!p) fail(HEC_ERR_INVALID_ARG, "plan is NULL");
    if (p->upper != upper) fail(HEC_ERR_INVALID_ARG, upper ? "plan is lower triangular" : "plan is upper triangular");
    if (nrhs < 1) fail(HEC_ERR_INVALID_ARG, "nrhs must be >= 1");
    check_vec(vdt);
    require_device(*p);
    if (p->h.n > 0 && (!b || !x)) fail(HEC_ERR_INVALID_ARG, "vector pointer is NULL");
    check_device_error(p->d);
    ensure_workspace(p->d, nrhs);
    const int32_t *orig = p->d.orig.as<int32_t>();
    launch_tri(p->d, b, vdt, orig, p->d.xw.p, x, vdt, orig, nrhs, st);
}

void export_hec(const HecHost &h, int32_t *width, int32_t *ld, int64_t *tail_nnz, int32_t *ell_col,
                double *ell_val, int32_t *csr_ptr, int32_t *csr_col, double *csr_val)
{
    if (width) *width = h.w;
    if (ld) *ld = h.ld;
    if (tail_nnz) *tail_nnz = (int64_t)h.csr_col.size();
    if (ell_col) std::copy(h.ell_col.begin(), h.ell_col.end(), ell_col);
    if (ell_val) std::copy(h.ell_val.begin(), h.ell_val.end(), ell_val);
    if (csr_ptr) std::copy(h.csr_ptr.begin(), h.csr_ptr.end(), csr_ptr);
    if (csr_col) std::copy(h.csr_col.begin(), h.csr_col.end(), csr_col);
    if (csr_val) std::copy(h.csr_val.begin(), h.csr_val.end(), csr_val);
}

void factor(const Csr &a, hec_ilu_kind_t kind, int32_t k, double tol, int32_t p, Csr &L, Csr &U,
            const std::vector<int32_t> *blocks = nullptr)
{
    std::function<void(const Csr &, Csr &, Csr &)> fac;
    switch (kind) {
    case HEC_ILU0: fac = [](const Csr &m, Csr &l, Csr &u) { ilu0(m, l, u); }; break;
    case HEC_ILUK: fac = [k](const Csr &m, Csr &l, Csr &u) { iluk(m, k, l, u); }; break;
    case HEC_ILUT: fac = [p, tol](const Csr &m, Csr &l, Csr &u) { ilut(m, p, tol, l, u); }; break;
    default: fail(HEC_ERR_INVALID_ARG, "unknown ILU kind");
    }
    if (blocks && blocks->size() > 2)
        factor_blocks(a, *blocks, fac, L, U);
    else
        fac(a, L, U);
}

// Plans of L (unit lower) and U, and the map joining them: U's solve reads L's
// device-order output through qmap (eq. (1): y never returns to natural order).
void build_ilu(ilu_s &f, const Csr &L, const Csr &U, hec_dtype_t fdt, const Tune &tu,
               const std::vector<int32_t> *blocks = nullptr)
{
    f.n = L.n;
    f.fdt = fdt;
    build_plan(f.L, L, false, true, fdt, tu, blocks);
    build_plan(f.U, U, true, false, fdt, tu, blocks);
    if (!tu.host_only) {
        const int32_t n = L.n;
        std::vector<int32_t> q(n);
        for (int32_t x = 0; x < n; ++x) {
            const int32_t i = f.U.h.ex.orig[x];
            q[x] = f.L.h.ex.xinv[f.L.h.lev.iperm[i]];
        }
        upload(f.qmap, q);
    }
}

void ilu_apply_impl(ilu_s *f, const void *r, void *z, int32_t nrhs, hec_dtype_t vdt, hipStream_t st,
                    const int8_t *act = nullptr)
{
    if (!f) fail(HEC_ERR_INVALID_ARG, "ilu is NULL");
    if (nrhs < 1) fail(HEC_ERR_INVALID_ARG, "nrhs must be >= 1");
    check_vec(vdt);
    require_device(f->L);
    if (f->n > 0 && (!r || !z)) fail(HEC_ERR_INVALID_ARG, "vector pointer is NULL");
    check_device_error(f->L.d, f->U.d);
    ensure_workspace(f->L.d, nrhs);
    ensure_workspace(f->U.d, nrhs);
    f->L.d.act = f->U.d.act = act;
    launch_tri(f->L.d, r, vdt, f->L.d.orig.as<int32_t>(), f->L.d.xw.p, nullptr, vdt, nullptr, nrhs, st);
    launch_tri(f->U.d, f->L.d.xw.p, f->fdt, f->qmap.as<int32_t>(), f->U.d.xw.p, z, vdt,
               f->U.d.orig.as<int32_t>(), nrhs, st);
    f->L.d.act = f->U.d.act = nullptr;
}

// Device refactorization data of an ILU(0)/ILU(k) handle for A's pattern
// (rowptr, col): the combined factor pattern F, A's entries in F, rows in
// L's level order, and where each factor entry lives in the two plans.
void build_refactor(ilu_s &f, const int32_t *rowptr, const int32_t *col)
{
    const int32_t n = f.n;
    auto r = std::make_unique<DevRefactor>();
    r->n = n;
    std::vector<int32_t> frp((size_t)n + 1, 0), fci, fdpos(n);
    fci.reserve((size_t)(f.Lf.nnz() + f.Uf.nnz()));
    int32_t maxrow = 0;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t p = f.Lf.rp[i]; p < f.Lf.rp[i + 1]; ++p)
            if (f.Lf.ci[p] < i) fci.push_back(f.Lf.ci[p]);
        fdpos[i] = (int32_t)fci.size();
        for (int32_t p = f.Uf.rp[i]; p < f.Uf.rp[i + 1]; ++p) fci.push_back(f.Uf.ci[p]);
        frp[i + 1] = (int32_t)fci.size();
        maxrow = std::max(maxrow, frp[i + 1] - frp[i]);
    }
    if (maxrow > kRefactorMaxRow)
        fail(HEC_ERR_CAPACITY, "a factor row has " + std::to_string(maxrow) + " entries; the device refactorization "
             "stages at most " + std::to_string(kRefactorMaxRow));
    // A's entries inside F's pattern
    if (rowptr[0] != 0) fail(HEC_ERR_INVALID_ARG, "rowptr[0] must be 0");
    const int64_t nnz_a = rowptr[n];
    std::vector<int32_t> a2f((size_t)nnz_a);
    for (int32_t i = 0; i < n; ++i) {
        if (rowptr[i + 1] < rowptr[i]) fail(HEC_ERR_INVALID_ARG, "rowptr is not monotone");
        auto b = fci.begin() + frp[i], e = fci.begin() + frp[i + 1];
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            auto it = std::lower_bound(b, e, col[p]);
            if (it == e || *it != col[p])
                fail(HEC_ERR_INVALID_ARG, "entry (" + std::to_string(i) + ", " + std::to_string(col[p]) +
                     ") of A is not in the factor pattern built at setup");
            a2f[p] = (int32_t)(it - fci.begin());
        }
    }
    // plan positions: the off-diagonals of a row keep their order in both layouts
    auto place = [](const ExecHost &ex, int32_t x, int32_t e) {
        return e < ex.w ? e * ex.ld + x : -1 - (ex.tail_ptr[x] + (e - ex.w));
    };
    std::vector<int32_t> l_src, l_dst, u_src, u_dst, u_diag, d_src(n);
    const ExecHost &el = f.L.h.ex, &eu = f.U.h.ex;
    for (int32_t x = 0; x < n; ++x) {
        const int32_t i = el.orig[x];
        int32_t e = 0;
        for (int32_t p = frp[i]; p < fdpos[i]; ++p, ++e) {
            l_src.push_back(p);
            l_dst.push_back(place(el, x, e));
        }
    }
    for (int32_t x = 0; x < n; ++x) {
        const int32_t i = eu.orig[x];
        int32_t e = 0;
        d_src[x] = fdpos[i];
        for (int32_t p = fdpos[i] + 1; p < frp[i + 1]; ++p, ++e) {
            u_src.push_back(p);
            u_dst.push_back(place(eu, x, e));
            u_diag.push_back(fdpos[i]);
        }
    }
    // sources of the row-per-lane elimination, in the order the host
    // factorization uses them: pivots ascending, each pivot's diagonal, then
    // the pivot row's later entries that the row holds
    std::vector<int32_t> sptr((size_t)n + 1, 0), spos, sdst;
    int32_t maxsrc = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t b = frp[i], e = frp[i + 1];
        for (int32_t p = b; p < fdpos[i]; ++p) {
            const int32_t k = fci[p], pk = fdpos[k];
            spos.push_back(pk);
            sdst.push_back(-1);
            for (int32_t pp = pk + 1; pp < frp[k + 1]; ++pp) {
                auto it = std::lower_bound(fci.begin() + p + 1, fci.begin() + e, fci[pp]);
                if (it != fci.begin() + e && *it == fci[pp]) {
                    spos.push_back(pp);
                    sdst.push_back((int32_t)(it - fci.begin()) - b);
                }
            }
        }
        sptr[i + 1] = (int32_t)spos.size();
        maxsrc = std::max(maxsrc, sptr[i + 1] - sptr[i]);
    }
    r->flow_row = maxrow <= 8 && maxsrc <= 16 ? 8 : (maxrow <= 16 && maxsrc <= 32 ? 16 : 0);
    if (r->flow_row > 0) {
        // one padding entry: a row without sources starts at the lists' end,
        // and the kernel's clamped (unconditional) loads read that position
        spos.push_back(0);
        sdst.push_back(0);
        upload(r->sptr, sptr);
        upload(r->spos, spos);
        upload(r->sdst, sdst);
    }
    const Levels &lv = f.L.h.lev;
    r->max_row = std::max(1, maxrow);
    r->levelptr = lv.levelptr;
    r->nnz_a = nnz_a;
    r->nnz_f = (int64_t)fci.size();
    r->nl = (int64_t)l_src.size();
    r->nu = (int64_t)u_src.size();
    r->a_rp.assign(rowptr, rowptr + n + 1);
    r->a_ci.assign(col, col + nnz_a);
    upload(r->a2f, a2f);
    upload(r->frp, frp);
    upload(r->fci, fci);
    upload(r->fdpos, fdpos);
    upload(r->rows, lv.perm);
    upload(r->l_src, l_src);
    upload(r->l_dst, l_dst);
    upload(r->u_src, u_src);
    upload(r->u_dst, u_dst);
    upload(r->u_diag, u_diag);
    upload(r->d_src, d_src);
    r->fval.alloc(std::max<size_t>(1, fci.size()) * sizeof(double));
    r->err.alloc(sizeof(int));
    f.rf = std::move(r);
}

// Copy the device factors back into Lf and Uf after a device refactorization.
void sync_host_factors(ilu_s &f)
{
    if (!f.dev_newer || !f.rf) return;
    const DevRefactor &r = *f.rf;
    std::vector<double> fv((size_t)r.nnz_f);
    if (r.nnz_f > 0)
        hip_check(hipMemcpy(fv.data(), r.fval.p, fv.size() * sizeof(double), hipMemcpyDeviceToHost), "factor download");
    int64_t q = 0;
    for (int32_t i = 0; i < f.n; ++i) {
        for (int32_t p = f.Lf.rp[i]; p < f.Lf.rp[i + 1]; ++p)
            if (f.Lf.ci[p] < i) f.Lf.v[p] = fv[q++];
        for (int32_t p = f.Uf.rp[i]; p < f.Uf.rp[i + 1]; ++p) f.Uf.v[p] = fv[q++];
    }
    f.dev_newer = false;
}

void ras_apply_impl(ras_s *s, const double *r, double *z, int32_t nrhs, hipStream_t st,
                    const int8_t *act = nullptr)
{
    if (!s) fail(HEC_ERR_INVALID_ARG, "ras is NULL");
    if (nrhs < 1) fail(HEC_ERR_INVALID_ARG, "nrhs must be >= 1");
    require_device(s->f.L);
    if (s->n > 0 && (!r || !z)) fail(HEC_ERR_INVALID_ARG, "vector pointer is NULL");
    if (r == z) fail(HEC_ERR_INVALID_ARG, "ras_apply needs distinct r and z");
    ilu_s &f = s->f;
    check_device_error(f.L.d, f.U.d);
    ensure_workspace(f.L.d, nrhs);
    ensure_workspace(f.U.d, nrhs);
    // restriction fused into L's gather, restricted prolongation into U's scatter
    f.L.d.act = f.U.d.act = act;
    launch_tri(f.L.d, r, HEC_F64, s->gather_L.as<int32_t>(), f.L.d.xw.p, nullptr, HEC_F64, nullptr, nrhs, st);
    launch_tri(f.U.d, f.L.d.xw.p, f.fdt, f.qmap.as<int32_t>(), f.U.d.xw.p, z, HEC_F64,
               s->scatter_U.as<int32_t>(), nrhs, st);
    f.L.d.act = f.U.d.act = nullptr;
}

}  // namespace

namespace hec {

void precond_check(const hec_precond_t &M, int32_t n)
{
    if (M.kind == HEC_PRECOND_NONE) return;
    if (!M.handle) fail(HEC_ERR_INVALID_ARG, "preconditioner handle is NULL");
    if (M.kind == HEC_PRECOND_ILU) {
        ilu_s *f = static_cast<ilu_s *>(M.handle);
        if (f->n != n) fail(HEC_ERR_INVALID_ARG, "preconditioner size differs from the matrix");
        require_device(f->L);
    } else if (M.kind == HEC_PRECOND_RAS) {
        ras_s *s = static_cast<ras_s *>(M.handle);
        if (s->n != n) fail(HEC_ERR_INVALID_ARG, "preconditioner size differs from the matrix");
        require_device(s->f.L);
    } else {
        fail(HEC_ERR_INVALID_ARG, "unknown preconditioner kind");
    }
}

void precond_check_error(const hec_precond_t &M)
{
    if (M.kind == HEC_PRECOND_ILU) {
        ilu_s *f = static_cast<ilu_s *>(M.handle);
        check_device_error(f->L.d, f->U.d);
    } else if (M.kind == HEC_PRECOND_RAS) {
        ras_s *s = static_cast<ras_s *>(M.handle);
        check_device_error(s->f.L.d, s->f.U.d);
    }
}

void precond_apply(const hec_precond_t &M, const double *r, double *z, int32_t R, hipStream_t st,
                   const int8_t *act)
{
    if (M.kind == HEC_PRECOND_ILU)
        ilu_apply_impl(static_cast<ilu_s *>(M.handle), r, z, R, HEC_F64, st, act);
    else
        ras_apply_impl(static_cast<ras_s *>(M.handle), r, z, R, st, act);
}

}  // namespace hec

extern "C" {

const char *hec_last_error(void) { return hec::g_last_error.c_str(); }

hec_status_t hec_tune_default(hec_tune_t *t)
{
    return guard([&] {
        if (!t) fail(HEC_ERR_INVALID_ARG, "tune is NULL");
        std::memset(t, 0, sizeof(*t));
        t->ell_width = -1;
        t->schedule = HEC_SCHED_AUTO;
        t->max_nrhs = 1;
        t->block_threads = 256;
    });
}

hec_status_t tri_analyze(int32_t n, const int32_t *rowptr, const int32_t *col, const void *val, hec_dtype_t dt,
                         hec_uplo_t uplo, int32_t unit_diag, const hec_tune_t *tune, tri_plan_t *out)
{
    return guard([&] {
        if (!out) fail(HEC_ERR_INVALID_ARG, "out is NULL");
        if (uplo != HEC_LOWER && uplo != HEC_UPPER) fail(HEC_ERR_INVALID_ARG, "bad uplo");
        Tune tu = tune_from(tune);
        Csr a = csr_copy(n, rowptr, col, val, dt);
        auto p = std::make_unique<tri_plan_s>();
        build_plan(*p, a, uplo == HEC_UPPER, unit_diag != 0, dt, tu);
        *out = p.release();
    });
}

hec_status_t tri_plan_info(tri_plan_t p, int32_t *n, int32_t *nlev, int32_t *levelptr, int32_t *perm)
{
    return guard([&] {
        if (!p) fail(HEC_ERR_INVALID_ARG, "plan is NULL");
        const Levels &lv = p->h.lev;
        if (n) *n = p->h.n;
        if (nlev) *nlev = lv.nlev;
        if (levelptr) std::copy(lv.levelptr.begin(), lv.levelptr.end(), levelptr);
        if (perm) std::copy(lv.perm.begin(), lv.perm.end(), perm);
    });
}

hec_status_t tri_plan_hec(tri_plan_t p, int32_t *width, int32_t *ld, int64_t *tail_nnz, int32_t *ell_col,
                          double *ell_val, int32_t *csr_ptr, int32_t *csr_col, double *csr_val)
{
    return guard([&] {
        if (!p) fail(HEC_ERR_INVALID_ARG, "plan is NULL");
        export_hec(p->h.hec, width, ld, tail_nnz, ell_col, ell_val, csr_ptr, csr_col, csr_val);
    });
}

hec_status_t tri_plan_stats(tri_plan_t p, tri_stats_t *s)
{
    return guard([&] {
        if (!p || !s) fail(HEC_ERR_INVALID_ARG, "NULL argument");
        const TriHost &h = p->h;
        std::memset(s, 0, sizeof(*s));
        s->n = h.n;
        s->nlev = h.lev.nlev;
        s->ell_width = h.ex.w;
        s->ld = h.ex.ld;
        s->schedule = h.ex.sched.kind;
        s->num_groups = h.ex.sched.groups;
        s->nsteps = h.ex.sched.nsteps();
        s->nexport = h.ex.sched.nexp;
        s->nremote = h.ex.sched.remote_reads;
        s->nnz_offdiag = h.nnz_off;
        s->nnz_tail = h.nnz_tail;
        s->lds_rows = h.ex.sched.max_window;
        s->crit_hops = h.ex.sched.crit_hops;
        s->dataflow = h.ex.sched.dataflow ? 1 : 0;
        s->syncfree = (h.ex.sched.kind == HEC_SCHED_LEVEL_LAUNCH && h.variant == 5) ? 1 : 0;
        s->queue = h.ex.sched.dataflow && h.ex.sched.queue ? 1 : 0;
        s->sysq = h.ex.sched.sysq ? 1 : 0;
        s->unit_diag = h.unit ? 1 : 0;
        s->dtype = h.dt;
    });
}

hec_status_t tri_plan_layout(tri_plan_t p, int32_t *xperm, int32_t *owner)
{
    return guard([&] {
        if (!p) fail(HEC_ERR_INVALID_ARG, "plan is NULL");
        if (xperm) std::copy(p->h.ex.orig.begin(), p->h.ex.orig.end(), xperm);
        if (owner) std::copy(p->h.ex.owner.begin(), p->h.ex.owner.end(), owner);
    });
}

hec_status_t tri_plan_trace(tri_plan_t p, void *trace, int32_t stride)
{
    return guard([&] {
        if (!p || stride < 0) fail(HEC_ERR_INVALID_ARG, "bad arguments");
        p->d.trace = static_cast<unsigned long long *>(trace);
        p->d.trace_stride = trace ? stride : 0;
    });
}

hec_status_t tri_plan_set_wait_limit(tri_plan_t p, uint32_t polls)
{
    return guard([&] {
        if (!p) fail(HEC_ERR_INVALID_ARG, "plan is NULL");
        if (polls > kMaxSpin) fail(HEC_ERR_INVALID_ARG, "wait limit above 2^27 polls");
        p->d.spin = polls == 0 ? kDefaultSpin : polls;
    });
}

hec_status_t tri_plan_check(tri_plan_t p)
{
    return guard([&] {
        if (!p) fail(HEC_ERR_INVALID_ARG, "plan is NULL");
        check_device_error(p->d);
    });
}

hec_status_t tri_solve_lower(tri_plan_t L, const void *b, void *x, int32_t nrhs, hec_dtype_t vdt, hipStream_t st)
{
    return guard([&] { solve_one(L, b, x, nrhs, vdt, st, false); });
}

hec_status_t tri_solve_upper(tri_plan_t U, const void *b, void *x, int32_t nrhs, hec_dtype_t vdt, hipStream_t st)
{
    return guard([&] { solve_one(U, b, x, nrhs, vdt, st, true); });
}

void tri_plan_destroy(tri_plan_t p) { delete p; }

hec_status_t ilu_setup(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                       hec_ilu_kind_t kind, int32_t k, double tol, int32_t p, hec_dtype_t fdt,
                       const hec_tune_t *tune, ilu_t *out)
{
    return guard([&] {
        if (!out) fail(HEC_ERR_INVALID_ARG, "out is NULL");
        if (fdt != HEC_F64 && fdt != HEC_F32) fail(HEC_ERR_INVALID_ARG, "bad factor dtype");
        Tune tu = tune_from(tune);
        Csr a = csr_copy(n, rowptr, col, val, HEC_F64);
        auto f = std::make_unique<ilu_s>();
        factor(a, kind, k, tol, p, f->Lf, f->Uf);
        f->kind = kind;
        build_ilu(*f, f->Lf, f->Uf, fdt, tu);
        *out = f.release();
    });
}

hec_status_t batch_setup(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val, int32_t nsys,
                         const int32_t *sys_ptr, hec_ilu_kind_t kind, int32_t k, double tol, int32_t p,
                         hec_dtype_t fdt, const hec_tune_t *tune, ilu_t *out)
{
    return guard([&] {
        if (!out || !sys_ptr || nsys < 1) fail(HEC_ERR_INVALID_ARG, "bad batch arguments");
        if (fdt != HEC_F64 && fdt != HEC_F32) fail(HEC_ERR_INVALID_ARG, "bad factor dtype");
        if (sys_ptr[0] != 0 || sys_ptr[nsys] != n) fail(HEC_ERR_INVALID_ARG, "sys_ptr must run from 0 to n");
        for (int32_t s = 0; s < nsys; ++s)
            if (sys_ptr[s + 1] < sys_ptr[s]) fail(HEC_ERR_INVALID_ARG, "sys_ptr not monotone");
        Tune tu = tune_from(tune);
        Csr a = csr_copy(n, rowptr, col, val, HEC_F64);
        // eq. (4): the systems must not couple
        for (int32_t s = 0; s < nsys; ++s)
            for (int32_t i = sys_ptr[s]; i < sys_ptr[s + 1]; ++i)
                for (int32_t q = a.rp[i]; q < a.rp[i + 1]; ++q)
                    if (a.ci[q] < sys_ptr[s] || a.ci[q] >= sys_ptr[s + 1])
                        fail(HEC_ERR_INVALID_ARG, "an entry couples two systems (row " + std::to_string(i) + ")");
        auto f = std::make_unique<ilu_s>();
        f->sys_ptr.assign(sys_ptr, sys_ptr + nsys + 1);
        factor(a, kind, k, tol, p, f->Lf, f->Uf, &f->sys_ptr);
        f->kind = kind;
        build_ilu(*f, f->Lf, f->Uf, fdt, tu, &f->sys_ptr);
        if (!tu.host_only) {
            // device row -> system, so that a solve can skip finished problems
            for (tri_plan_s *pl : {&f->L, &f->U}) {
                std::vector<int32_t> sg(n);
                for (int32_t x = 0; x < n; ++x) {
                    const int32_t i = pl->h.ex.orig[x];
                    sg[x] = (int32_t)(std::upper_bound(f->sys_ptr.begin(), f->sys_ptr.end(), i) -
                                      f->sys_ptr.begin()) - 1;
                }
                upload(pl->d.seg, sg);
            }
        }
        *out = f.release();
    });
}

hec_status_t ilu_factor(ilu_t f, int32_t which, int64_t *nnz, int32_t *rowptr, int32_t *col, double *val)
{
    return guard([&] {
        if (!f || (which != 0 && which != 1)) fail(HEC_ERR_INVALID_ARG, "bad arguments");
        sync_host_factors(*f);
        const Csr &c = which == 0 ? f->Lf : f->Uf;
        if (nnz) *nnz = c.nnz();
        if (rowptr) std::copy(c.rp.begin(), c.rp.end(), rowptr);
        if (col) std::copy(c.ci.begin(), c.ci.end(), col);
        if (val) std::copy(c.v.begin(), c.v.end(), val);
    });
}

hec_status_t ilu_plans(ilu_t f, tri_plan_t *L, tri_plan_t *U)
{
    return guard([&] {
        if (!f) fail(HEC_ERR_INVALID_ARG, "ilu is NULL");
        if (L) *L = &f->L;
        if (U) *U = &f->U;
    });
}

// Workspace of ilu_apply_noalloc: the intermediate y = L^{-1} r and the U
// solve's own device-order workspace live in one file-scope device array,
// so that the entry point never allocates.  Each GPU holds its own copy for
// the life of the process; its address is taken once per device.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device -> address of that device's scratch

void *scratch_on_current_device()
{
    int dev = -1;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) return it->second;
    void *ptr = nullptr;
    hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) fail(HEC_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = ptr;
    return ptr;
}
}  // namespace

hec_status_t ilu_apply_noalloc(ilu_t f, const void *r, void *z, int32_t nrhs, hec_dtype_t vdt, hipStream_t st)
{
    return guard([&] {
        if (!f) fail(HEC_ERR_INVALID_ARG, "ilu is NULL");
        if (nrhs < 1) fail(HEC_ERR_INVALID_ARG, "nrhs must be >= 1");
        check_vec(vdt);
        require_device(f->L);
        if (f->n > 0 && (!r || !z)) fail(HEC_ERR_INVALID_ARG, "vector pointer is NULL");
        // the plans' mailboxes and counters were sized at setup; this entry
        // point never grows them
        if (nrhs > f->L.d.ws_R || nrhs > f->U.d.ws_R)
            fail(HEC_ERR_INVALID_ARG, "nrhs " + std::to_string(nrhs) + " exceeds the handle's max_nrhs " +
                                          std::to_string(std::min(f->L.d.ws_R, f->U.d.ws_R)) +
                                          " (ilu_apply_noalloc never enlarges workspaces)");
        const size_t ts = f->fdt == HEC_F64 ? 8 : 4;
        const size_t part = (((size_t)f->n + 1) * (size_t)nrhs * ts + 255) & ~(size_t)255;
        if (2 * part > kScratchBytes)
            fail(HEC_ERR_CAPACITY, "ilu_apply_noalloc needs " + std::to_string(2 * part) + " bytes of scratch for n = " +
                                       std::to_string(f->n) + " and nrhs = " + std::to_string(nrhs) +
                                       "; its fixed scratch holds " + std::to_string(kScratchBytes) +
                                       " (use ilu_apply)");
        unsigned char *base = static_cast<unsigned char *>(scratch_on_current_device());
        void *y = base;          // L's device-order output, U's input
        void *uw = base + part;  // U's own workspace (kernels that keep the solution in global memory)
        check_device_error(f->L.d, f->U.d);
        launch_tri(f->L.d, r, vdt, f->L.d.orig.as<int32_t>(), y, nullptr, vdt, nullptr, nrhs, st);
        launch_tri(f->U.d, y, f->fdt, f->qmap.as<int32_t>(), uw, z, vdt, f->U.d.orig.as<int32_t>(), nrhs, st);
    });
}

hec_status_t ilu_apply(ilu_t f, const void *r, void *z, int32_t nrhs, hec_dtype_t vdt, hipStream_t st)
{
    return guard([&] { ilu_apply_impl(f, r, z, nrhs, vdt, st); });
}

void ilu_destroy(ilu_t f) { delete f; }

hec_status_t ilu_refactor(ilu_t f, const int32_t *rowptr, const int32_t *col, const double *val, hipStream_t st)
{
    return guard([&] {
        if (!f) fail(HEC_ERR_INVALID_ARG, "ilu is NULL");
        if (f->kind == HEC_ILUT) fail(HEC_ERR_INVALID_ARG, "ILUT's pattern depends on the values; refactor needs ILU(0) or ILU(k)");
        require_device(f->L);
        const int32_t n = f->n;
        if (!rowptr && !col) {
            if (!f->rf) fail(HEC_ERR_INVALID_ARG, "no pattern given and none from an earlier call");
        } else {
            if (!rowptr || (!col && rowptr[n] > 0)) fail(HEC_ERR_INVALID_ARG, "rowptr or col is NULL");
            const bool same = f->rf && f->rf->a_rp.size() == (size_t)n + 1 &&
                              std::equal(f->rf->a_rp.begin(), f->rf->a_rp.end(), rowptr) &&
                              (int64_t)f->rf->a_ci.size() == (int64_t)rowptr[n] &&
                              std::equal(f->rf->a_ci.begin(), f->rf->a_ci.end(), col);
            if (!same) {
                // the new maps start without factors: bring the current ones
                // (held only by the device) to the host first
                sync_host_factors(*f);
                build_refactor(*f, rowptr, col);
            }
        }
        if (f->rf->nnz_a > 0 && !val) fail(HEC_ERR_INVALID_ARG, "val is NULL");
        check_device_error(f->L.d, f->U.d);
        refactor_numeric(*f->rf, val, st);
        refactor_refill(*f->rf, f->L.d, f->U.d, st);
        f->dev_newer = true;
    });
}

hec_status_t ras_refactor(ras_t s, const int32_t *rowptr, const int32_t *col, const double *val, hipStream_t st)
{
    return guard([&] {
        if (!s) fail(HEC_ERR_INVALID_ARG, "ras is NULL");
        ilu_s &f = s->f;
        if (f.kind == HEC_ILUT) fail(HEC_ERR_INVALID_ARG, "ILUT's pattern depends on the values; refactor needs ILU(0) or ILU(k)");
        require_device(f.L);
        const int32_t n = s->n;
        if (!rowptr && !col) {
            if (s->a_rp.empty()) fail(HEC_ERR_INVALID_ARG, "no pattern given and none from an earlier call");
        } else {
            if (!rowptr || (!col && rowptr[n] > 0)) fail(HEC_ERR_INVALID_ARG, "rowptr or col is NULL");
            const bool same = s->a_rp.size() == (size_t)n + 1 && std::equal(s->a_rp.begin(), s->a_rp.end(), rowptr) &&
                              (int64_t)s->a_ci.size() == (int64_t)rowptr[n] &&
                              std::equal(s->a_ci.begin(), s->a_ci.end(), col);
            if (!same) {
                // each entry of A_s = A[ext_s, ext_s] is an entry of A
                if (rowptr[0] != 0) fail(HEC_ERR_INVALID_ARG, "rowptr[0] must be 0");
                const Csr &bd = s->lay.blockdiag;
                std::vector<int32_t> idx((size_t)bd.nnz());
                for (int32_t r = 0; r < bd.n; ++r) {
                    const int32_t g = s->lay.ext[r];
                    const int32_t *b = col + rowptr[g], *e = col + rowptr[g + 1];
                    for (int32_t q = bd.rp[r]; q < bd.rp[r + 1]; ++q) {
                        const int32_t gc = s->lay.ext[bd.ci[q]];
                        const int32_t *it = std::lower_bound(b, e, gc);
                        if (it == e || *it != gc)
                            fail(HEC_ERR_INVALID_ARG, "entry (" + std::to_string(g) + ", " + std::to_string(gc) +
                                 ") of a subdomain matrix is not in A's pattern");
                        idx[q] = (int32_t)(it - col);
                    }
                }
                upload(s->a2bd, idx);
                s->bdval.alloc(std::max<size_t>(1, idx.size()) * sizeof(double));
                if (!f.rf) build_refactor(f, bd.rp.data(), bd.ci.data());
                s->a_rp.assign(rowptr, rowptr + n + 1);
                s->a_ci.assign(col, col + rowptr[n]);
            }
        }
        if (s->lay.blockdiag.nnz() > 0 && !val) fail(HEC_ERR_INVALID_ARG, "val is NULL");
        check_device_error(f.L.d, f.U.d);
        gather_f64(val, s->a2bd.as<int32_t>(), s->lay.blockdiag.nnz(), s->bdval.as<double>(), st);
        refactor_numeric(*f.rf, s->bdval.as<double>(), st);
        refactor_refill(*f.rf, f.L.d, f.U.d, st);
        f.dev_newer = true;
    });
}

hec_status_t ras_setup(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val, int32_t nsub,
                       const int32_t *owner, int32_t overlap, hec_dtype_t fdt, const hec_tune_t *tune, ras_t *out)
{
    return ras_setup_ilu(n, rowptr, col, val, nsub, owner, overlap, HEC_ILU0, 0, 0.0, 0, fdt, tune, out);
}

hec_status_t ras_setup_ilu(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val, int32_t nsub,
                           const int32_t *owner, int32_t overlap, hec_ilu_kind_t kind, int32_t k, double tol,
                           int32_t p, hec_dtype_t fdt, const hec_tune_t *tune, ras_t *out)
{
    return guard([&] {
        if (!out) fail(HEC_ERR_INVALID_ARG, "out is NULL");
        if (fdt != HEC_F64 && fdt != HEC_F32) fail(HEC_ERR_INVALID_ARG, "bad factor dtype");
        if (kind != HEC_ILU0 && kind != HEC_ILUK && kind != HEC_ILUT) fail(HEC_ERR_INVALID_ARG, "unknown ILU kind");
        Tune tu = tune_from(tune);
        Csr a = csr_copy(n, rowptr, col, val, HEC_F64);
        auto s = std::make_unique<ras_s>();
        s->n = n;
        s->nsub = nsub;
        s->lay = ras_layout(a, nsub, owner, overlap);
        ilu_s &f = s->f;
        factor(s->lay.blockdiag, kind, k, tol, p, f.Lf, f.Uf, &s->lay.ext_ptr);
        f.kind = kind;
        build_ilu(f, f.Lf, f.Uf, fdt, tu, &s->lay.ext_ptr);
        if (!tu.host_only) {
            const int32_t m = s->lay.blockdiag.n;
            std::vector<int32_t> g(m), sc(m);
            for (int32_t x = 0; x < m; ++x) g[x] = s->lay.ext[f.L.h.ex.orig[x]];
            for (int32_t x = 0; x < m; ++x) {
                const int32_t e = f.U.h.ex.orig[x];
                sc[x] = s->lay.owned[e] ? s->lay.ext[e] : -1;
            }
            upload(s->gather_L, g);
            upload(s->scatter_U, sc);
        }
        *out = s.release();
    });
}

hec_status_t ras_apply(ras_t s, const double *r, double *z, int32_t nrhs, hipStream_t st)
{
    return guard([&] { ras_apply_impl(s, r, z, nrhs, st); });
}

hec_status_t ras_info(ras_t s, int32_t *nsub, int64_t *total_ext, int32_t *ext_sizes)
{
    return guard([&] {
        if (!s) fail(HEC_ERR_INVALID_ARG, "ras is NULL");
        if (nsub) *nsub = s->nsub;
        if (total_ext) *total_ext = (int64_t)s->lay.ext.size();
        if (ext_sizes)
            for (int32_t i = 0; i < s->nsub; ++i) ext_sizes[i] = s->lay.ext_ptr[i + 1] - s->lay.ext_ptr[i];
    });
}

hec_status_t ras_plans(ras_t s, tri_plan_t *L, tri_plan_t *U)
{
    return guard([&] {
        if (!s) fail(HEC_ERR_INVALID_ARG, "ras is NULL");
        if (L) *L = &s->f.L;
        if (U) *U = &s->f.U;
    });
}

void ras_destroy(ras_t s) { delete s; }

hec_status_t sor_setup(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val, double omega,
                       const hec_tune_t *tune, sor_t *out)
{
    return guard([&] {
        if (!out) fail(HEC_ERR_INVALID_ARG, "out is NULL");
        if (!(omega > 0.0 && omega < 2.0)) fail(HEC_ERR_INVALID_ARG, "omega must lie in (0, 2)");
        Tune tu = tune_from(tune);
        Csr a = csr_copy(n, rowptr, col, val, HEC_F64);
        check_csr_structure(a);
        // split A = D + L + U row by row; entry order inside a row is kept
        Csr ml, mu, nl, nu;
        for (Csr *c : {&ml, &mu, &nl, &nu}) {
            c->n = n;
            c->rp.assign((size_t)n + 1, 0);
        }
        const double shift = 1.0 - 1.0 / omega;
        for (int32_t i = 0; i < n; ++i) {
            double d = 0.0;
            bool have = false;
            for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p)
                if (a.ci[p] == i) { d = a.v[p]; have = true; }
            if (!have) fail(HEC_ERR_MISSING_DIAG, "row " + std::to_string(i) + " has no diagonal entry");
            if (d == 0.0 || !std::isfinite(d)) fail(HEC_ERR_ZERO_PIVOT, "zero or non-finite diagonal in row " + std::to_string(i));
            for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
                const int32_t j = a.ci[p];
                const double v = a.v[p];
                if (j < i) {
                    ml.ci.push_back(j), ml.v.push_back(v);
                    nl.ci.push_back(j), nl.v.push_back(v);
                } else if (j > i) {
                    mu.ci.push_back(j), mu.v.push_back(v);
                    nu.ci.push_back(j), nu.v.push_back(v);
                } else {
                    ml.ci.push_back(i), ml.v.push_back(d / omega);
                    mu.ci.push_back(i), mu.v.push_back(d / omega);
                    if (shift != 0.0) {
                        nl.ci.push_back(i), nl.v.push_back(shift * d);
                        nu.ci.push_back(i), nu.v.push_back(shift * d);
                    }
                }
            }
            for (Csr *c : {&ml, &mu, &nl, &nu}) c->rp[i + 1] = (int32_t)c->ci.size();
        }
        auto s = std::make_unique<sor_s>();
        s->n = n;
        s->omega = omega;
        build_plan(s->fwd, ml, false, false, HEC_F64, tu);
        build_plan(s->bwd, mu, true, false, HEC_F64, tu);
        if (!tu.host_only) {
            build_devhec(s->nf, nu, HEC_F64, -1);
            build_devhec(s->nb, nl, HEC_F64, -1);
        }
        *out = s.release();
    });
}

hec_status_t sor_apply(sor_t s, const double *b, double *x, int32_t nrhs, int32_t sweeps, int32_t symmetric,
                       hipStream_t st)
{
    return guard([&] {
        if (!s) fail(HEC_ERR_INVALID_ARG, "sor is NULL");
        if (nrhs < 1 || sweeps < 0) fail(HEC_ERR_INVALID_ARG, "nrhs must be >= 1 and sweeps >= 0");
        require_device(s->fwd);
        if (s->n > 0 && (!b || !x)) fail(HEC_ERR_INVALID_ARG, "vector pointer is NULL");
        if (b == x && s->n > 0) fail(HEC_ERR_INVALID_ARG, "sor_apply needs distinct b and x");
        check_device_error(s->fwd.d);
        check_device_error(s->bwd.d);
        ensure_workspace(s->fwd.d, nrhs);
        ensure_workspace(s->bwd.d, nrhs);
        if (nrhs > s->t_R) {
            s->t.alloc(((size_t)s->n + 1) * nrhs * sizeof(double));
            s->t_R = nrhs;
        }
        double *t = s->t.as<double>();
        const int32_t *of = s->fwd.d.orig.as<int32_t>(), *ob = s->bwd.d.orig.as<int32_t>();
        for (int32_t k = 0; k < sweeps; ++k) {
            residual(s->nf, b, x, t, nrhs, st);  // t = b - (U + (1 - 1/omega) D) x
            launch_tri(s->fwd.d, t, HEC_F64, of, s->fwd.d.xw.p, x, HEC_F64, of, nrhs, st);
            if (symmetric) {
                residual(s->nb, b, x, t, nrhs, st);  // t = b - (L + (1 - 1/omega) D) x
                launch_tri(s->bwd.d, t, HEC_F64, ob, s->bwd.d.xw.p, x, HEC_F64, ob, nrhs, st);
            }
        }
    });
}

void sor_destroy(sor_t s) { delete s; }

hec_status_t hec_graph_capture(hec_precond_t M, const void *r, void *z, int32_t nrhs, hec_dtype_t vdt,
                               hipStream_t st, hec_graph_t *out)
{
    return guard([&] {
        if (!out) fail(HEC_ERR_INVALID_ARG, "out is NULL");
        if (M.kind != HEC_PRECOND_ILU && M.kind != HEC_PRECOND_RAS) fail(HEC_ERR_INVALID_ARG, "bad preconditioner kind");
        if (!M.handle) fail(HEC_ERR_INVALID_ARG, "preconditioner handle is NULL");
        if (nrhs < 1) fail(HEC_ERR_INVALID_ARG, "nrhs must be >= 1");
        // workspaces must exist before capture (no allocation inside it)
        if (M.kind == HEC_PRECOND_ILU) {
            ilu_s *f = static_cast<ilu_s *>(M.handle);
            require_device(f->L);
            ensure_workspace(f->L.d, nrhs);
            ensure_workspace(f->U.d, nrhs);
        } else {
            if (vdt != HEC_F64) fail(HEC_ERR_INVALID_ARG, "RAS vectors are FP64");
            ras_s *s = static_cast<ras_s *>(M.handle);
            require_device(s->f.L);
            ensure_workspace(s->f.L.d, nrhs);
            ensure_workspace(s->f.U.d, nrhs);
        }
        hipStream_t cap = st;
        bool own = false;
        if (!cap) {
            hip_check(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "hipStreamCreate");
            own = true;
        }
        auto g = std::make_unique<hec_graph_s>();
        hip_check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        try {
            if (M.kind == HEC_PRECOND_ILU)
                ilu_apply_impl(static_cast<ilu_s *>(M.handle), r, z, nrhs, vdt, cap);
            else
                ras_apply_impl(static_cast<ras_s *>(M.handle), static_cast<const double *>(r),
                               static_cast<double *>(z), nrhs, cap);
        } catch (...) {
            hipGraph_t tmp = nullptr;
            (void)hipStreamEndCapture(cap, &tmp);
            if (tmp) (void)hipGraphDestroy(tmp);
            if (own) (void)hipStreamDestroy(cap);
            throw;
        }
        hipError_t e = hipStreamEndCapture(cap, &g->graph);
        if (own) (void)hipStreamDestroy(cap);
        hip_check(e, "hipStreamEndCapture");
        hip_check(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        *out = g.release();
    });
}

hec_status_t hec_graph_launch(hec_graph_t g, hipStream_t st)
{
    return guard([&] {
        if (!g) fail(HEC_ERR_INVALID_ARG, "graph is NULL");
        hip_check(hipGraphLaunch(g->exec, st), "hipGraphLaunch");
    });
}

void hec_graph_destroy(hec_graph_t g) { delete g; }

hec_status_t tri_autotune(int32_t n, const int32_t *rowptr, const int32_t *col, const void *val, hec_dtype_t dt,
                          hec_uplo_t uplo, int32_t unit_diag, int32_t nrhs, int32_t nsys, const int32_t *sys_ptr,
                          const char *cache_path, double max_seconds, hipStream_t st, hec_tune_t *best,
                          double *best_us)
{
    return guard([&] {
        if (!best || nrhs < 1) fail(HEC_ERR_INVALID_ARG, "bad arguments");
        if (uplo != HEC_LOWER && uplo != HEC_UPPER) fail(HEC_ERR_INVALID_ARG, "bad uplo");
        if (nsys < 0 || (nsys > 0 && !sys_ptr)) fail(HEC_ERR_INVALID_ARG, "bad system blocks");
        Csr a = csr_copy(n, rowptr, col, val, dt);
        const bool upper = uplo == HEC_UPPER, unit = unit_diag != 0;
        validate_triangle(a, upper, unit);
        std::vector<int32_t> blocks;
        if (nsys > 0) {
            blocks.assign(sys_ptr, sys_ptr + nsys + 1);
            if (blocks.front() != 0 || blocks.back() != n) fail(HEC_ERR_INVALID_ARG, "sys_ptr must run from 0 to n");
            for (int32_t q = 0; q < nsys; ++q)
                if (blocks[q + 1] < blocks[q]) fail(HEC_ERR_INVALID_ARG, "sys_ptr not monotone");
        }
        const std::vector<int32_t> *bp = blocks.empty() ? nullptr : &blocks;
        // signature of the problem: sizes, type, right-hand sides, blocks and
        // the level histogram (eq. (2)-(3)), FNV-1a hashed
        const Levels lv = compute_levels(a, upper);
        uint64_t h = 1469598103934665603ull;
        auto mix = [&](int64_t v) {
            for (int b = 0; b < 8; ++b) {
                h ^= (uint64_t)((v >> (8 * b)) & 0xff);
                h *= 1099511628211ull;
            }
        };
        for (int64_t v : {(int64_t)n, (int64_t)a.nnz(), (int64_t)upper, (int64_t)unit, (int64_t)nrhs, (int64_t)dt,
                          (int64_t)nsys})
            mix(v);
        for (int32_t k = 0; k < lv.nlev; ++k) mix(lv.levelptr[k + 1] - lv.levelptr[k]);
        for (int32_t v : blocks) mix(v);
        char sig[64];
        std::snprintf(sig, sizeof sig, "%016llx", (unsigned long long)h);
        static const char *kFields[] = {"ell_width", "schedule", "num_groups", "merge_rows", "group_lanes",
                                        "long_row", "part_rows", "max_nrhs", "block_threads", "chunk_rows",
                                        "partition", "kernel_variant"};
        auto field = [](hec_tune_t &t, int i) -> int32_t & {
            int32_t *f[] = {&t.ell_width, &t.schedule,  &t.num_groups,    &t.merge_rows,
                            &t.group_lanes, &t.long_row, &t.part_rows,    &t.max_nrhs,
                            &t.block_threads, &t.chunk_rows, &t.partition, &t.kernel_variant};
            return *f[i];
        };
        // cache: one JSON object per line, {"sig": "...", "us": t, "tune": {...}}; the last line
        // with a matching signature wins
        if (cache_path && *cache_path) {
            std::FILE *fp = std::fopen(cache_path, "r");
            if (fp) {
                char line[4096];
                bool found = false;
                hec_tune_t got;
                double got_us = 0;
                const std::string key = std::string("\"sig\": \"") + sig + "\"";
                while (std::fgets(line, sizeof line, fp)) {
                    const std::string ln(line);
                    if (ln.find(key) == std::string::npos) continue;
                    hec_tune_default(&got);
                    bool ok = true;
                    for (int i = 0; i < 12 && ok; ++i) {
                        const std::string fk = std::string("\"") + kFields[i] + "\": ";
                        const size_t pos = ln.find(fk);
                        if (pos == std::string::npos) ok = false;
                        else field(got, i) = (int32_t)std::strtol(ln.c_str() + pos + fk.size(), nullptr, 10);
                    }
                    const size_t pu = ln.find("\"us\": ");
                    if (ok && pu != std::string::npos) {
                        got_us = std::strtod(ln.c_str() + pu + 6, nullptr);
                        found = true;
                    }
                }
                std::fclose(fp);
                if (found) {
                    *best = got;
                    if (best_us) *best_us = got_us;
                    return;
                }
            }
        }
        const int32_t w0 = auto_ell_width(a, upper);
        int32_t wmax = 0;
        for (int32_t i = 0; i < a.n; ++i) wmax = std::max(wmax, a.rp[i + 1] - a.rp[i] - (unit ? 0 : 1));
        // candidates, cheapest first: the automatic choice; the dataflow kernel
        // with one part per workgroup (compute wavefronts x partition shape);
        // the part queue (compute wavefronts x rows per part); the barrier-free
        // kernel; one launch per level; the level-persistent schedule with
        // level-merge thresholds; wider ELL parts when rows overflow
        std::vector<Tune> cands;
        Tune base = default_tune();
        base.max_nrhs = nrhs;
        cands.push_back(base);
        // one part per workgroup holds about n / CUs rows of solution and
        // right-hand side in LDS: skip those candidates when that cannot fit
        const size_t part_lds = 2 * (size_t)((n + device_cus() - 1) / std::max(1, device_cus())) * (size_t)nrhs *
                                (dt == HEC_F64 ? 8 : 4);
        const bool parts_fit = part_lds <= (size_t)device_max_lds();
        if (nrhs <= 64 && parts_fit) {
            for (int32_t blk : {256, 128, 384})
                for (int32_t part : {0, 1, 2}) {
                    Tune t = base;
                    t.schedule = HEC_SCHED_OWNER_PERSISTENT;
                    t.variant = 4;
                    t.block_threads = blk;
                    t.chunk_rows = std::max(256, blk);  // a valid multiple of the block
                    t.partition = part;
                    cands.push_back(t);
                }
        }
        if (nrhs <= 64) {
            for (int32_t blk : {256, 384})
                for (int32_t rows : {0, 1024, 4096}) {
                    Tune t = base;
                    t.schedule = HEC_SCHED_OWNER_PERSISTENT;
                    t.variant = 6;
                    t.block_threads = blk;
                    t.chunk_rows = std::max(256, blk);
                    t.part_rows = rows;
                    cands.push_back(t);
                }
            if (wmax > w0 && wmax <= 16 && parts_fit) {
                Tune t = base;
                t.schedule = HEC_SCHED_OWNER_PERSISTENT;
                t.variant = 4;
                t.ell_width = dataflow_width(std::max(1, (w0 + wmax) / 2));
                cands.push_back(t);
            }
        }
        for (int32_t blk : {512, 1024}) {  // the system queue (one workgroup per system)
            Tune t = base;
            t.schedule = HEC_SCHED_LEVEL_PERSISTENT;
            t.variant = 7;
            t.block_threads = blk;
            t.chunk_rows = blk;
            cands.push_back(t);
        }
        {
            Tune t = base;
            t.schedule = HEC_SCHED_LEVEL_LAUNCH;
            t.variant = 5;
            cands.push_back(t);
            Tune u = base;
            u.schedule = HEC_SCHED_LEVEL_LAUNCH;
            cands.push_back(u);
        }
        for (int32_t mul : {1, 4}) {
            Tune u = base;
            u.schedule = HEC_SCHED_LEVEL_PERSISTENT;
            u.merge_rows = std::max(1, mul * u.block_threads / nrhs);
            cands.push_back(u);
        }
        if (wmax > w0) {
            Tune u = base;
            u.schedule = HEC_SCHED_LEVEL_PERSISTENT;
            u.group_lanes = 4;
            u.long_row = 8;
            cands.push_back(u);
        }
        const hec_dtype_t vdt = dt;
        const size_t bytes = ((size_t)std::max(1, n)) * nrhs * (vdt == HEC_F64 ? 8 : 4);
        DevMem b, x;
        b.alloc(bytes);
        x.alloc(bytes);
        hip_check(hipMemset(b.p, 0, bytes), "hipMemset");
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "hipEventCreate");
        hip_check(hipEventCreate(&e1), "hipEventCreate");
        struct EvFree {
            hipEvent_t a, b;
            ~EvFree()
            {
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
            }
        } ev_free{e0, e1};
        double best_t = 1e300;
        Tune best_tune = cands.front();
        const auto t_start = std::chrono::steady_clock::now();
        for (size_t ci = 0; ci < cands.size(); ++ci) {
            const Tune &t = cands[ci];
            if (ci > 0 && max_seconds > 0 &&
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count() > max_seconds)
                break;
            tri_plan_s p;
            try {
                build_plan(p, a, upper, unit, dt, t, bp);
                for (int rep = 0; rep < 2; ++rep) solve_one(&p, b.p, x.p, nrhs, vdt, st, upper);
                hip_check(hipEventRecord(e0, st), "hipEventRecord");
                const int reps = 5;
                for (int rep = 0; rep < reps; ++rep) solve_one(&p, b.p, x.p, nrhs, vdt, st, upper);
                hip_check(hipEventRecord(e1, st), "hipEventRecord");
                hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
                // a candidate whose waits gave up exits early: never time it
                check_device_error(p.d);
                float ms = 0.f;
                hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
                const double us = 1000.0 * ms / reps;
                if (us < best_t) {
                    best_t = us;
                    best_tune = t;
                }
            } catch (const Error &e) {
                if (e.code != HEC_ERR_CAPACITY && e.code != HEC_ERR_ALLOC && e.code != HEC_ERR_TIMEOUT &&
                    e.code != HEC_ERR_INVALID_ARG)
                    throw;
            }
        }
        if (best_t >= 1e300) fail(HEC_ERR_CAPACITY, "no candidate schedule could run this triangle");
        hec_tune_default(best);
        best->ell_width = best_tune.ell_width;
        best->schedule = best_tune.schedule;
        best->num_groups = best_tune.num_groups;
        best->merge_rows = best_tune.merge_rows;
        best->group_lanes = best_tune.group_lanes;
        best->long_row = best_tune.long_row;
        best->part_rows = best_tune.part_rows;
        best->max_nrhs = best_tune.max_nrhs;
        best->block_threads = best_tune.block_threads;
        best->chunk_rows = best_tune.chunk_rows;
        best->partition = best_tune.partition;
        best->kernel_variant = best_tune.variant;
        if (best_us) *best_us = best_t;
        if (cache_path && *cache_path) {
            std::FILE *fp = std::fopen(cache_path, "a");
            if (!fp) fail(HEC_ERR_INVALID_ARG, std::string("cannot append to the tuning cache ") + cache_path);
            std::fprintf(fp, "{\"sig\": \"%s\", \"n\": %d, \"nnz\": %lld, \"nlev\": %d, \"nrhs\": %d, \"dtype\": %d, "
                             "\"us\": %.3f, \"tune\": {",
                         sig, n, (long long)a.nnz(), lv.nlev, nrhs, (int)dt, best_t);
            for (int i = 0; i < 12; ++i) std::fprintf(fp, "%s\"%s\": %d", i ? ", " : "", kFields[i], field(*best, i));
            std::fprintf(fp, "}}\n");
            std::fclose(fp);
        }
    });
}

}  // extern "C"
