// Level-scheduled sparse triangular solve kernels for gfx950 (CDNA4).
//
// Algorithm 2 of the paper: the right-hand side is permuted into level order,
// the levels are solved one after the other with every row of a level solved
// simultaneously, and the solution is permuted back.  Both permutations are
// fused into the row routine (the gather of b on the first read, the scatter
// of x on the final write).  Upper solves use the same code on the plan built
// from U reversed by t(i) = n-1-i (end of Section 2.2).
//
// Two executions of the same row routine:
//   k_level       one launch per level (the paper's shape);
//   k_persistent  one launch for the whole solve: every workgroup runs its
//                 list of steps (a contiguous range of device rows of one
//                 level).  A dependency produced by the same workgroup is
//                 read from LDS (owner schedule) or from the workspace after
//                 the step barrier; a dependency produced by another
//                 workgroup is read from a mailbox slot, polled until the
//                 producer's value replaces the sentinel.
// The row routine subtracts the ELL terms in slot order, then the CSR-tail
// terms, then multiplies by the stored reciprocal diagonal, so both
// executions produce bit-identical results for rows run one thread per
// (row, rhs); steps tuned to split long rows over several lanes sum in a
// different order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "hec_dev.h"

namespace hec {

namespace {


int32_t capacity_of(const void *kern, int32_t block, size_t lds);

template <typename T> __device__ __forceinline__ T sentinel();
template <> __device__ __forceinline__ double sentinel<double>() { return __longlong_as_double((long long)kSentinel64); }
template <> __device__ __forceinline__ float sentinel<float>() { return __uint_as_float(kSentinel32); }
__device__ __forceinline__ bool is_sentinel(double v) { return __double_as_longlong(v) == (long long)kSentinel64; }
__device__ __forceinline__ bool is_sentinel(float v) { return __float_as_uint(v) == kSentinel32; }

// A right-hand-side value as a kernel publishes it: an input whose bits
// happen to equal the sentinel becomes the canonical quiet NaN, so that no
// input value can stand for "not solved yet" (a row without dependencies
// publishes its right-hand side unchanged).
template <typename T> __device__ __forceinline__ T canon(T v)
{
    return is_sentinel(v) ? __builtin_nan("") : v;
}
template <> __device__ __forceinline__ float canon<float>(float v)
{
    return is_sentinel(v) ? __builtin_nanf("") : v;
}

// Right-hand side times the reciprocal diagonal, rounded on its own (never
// contracted into the first multiply-add), identically in every kernel.
__device__ __forceinline__ double scale_rhs(double b, double d)
{
#pragma clang fp contract(off)
    return b * d;
}
__device__ __forceinline__ float scale_rhs(float b, float d)
{
#pragma clang fp contract(off)
    return b * d;
}

// Per-launch state of the persistent kernel shared by the row routine.
template <typename T> struct Ctx {
    T *xl;          // LDS window (device rows lo..hi-1), holds b then x
    int lo, hi;
    T *mbox_rd;     // this launch's mailbox half
    int *abort;     // LDS flag: a poll gave up
};

// Mailbox slots are written with agent-scope relaxed atomic stores, which go
// through to the point of coherence shared by all XCDs, and polled with
// agent-scope relaxed atomic loads, which do not hit stale cache lines.  The
// value itself is the signal, so no flag, fence or cache-wide writeback is
// needed.  The poll is bounded; on expiry it raises the abort flags.
template <typename T>
__device__ __forceinline__ T poll_slot(const T *p, int *err_dev, int *err_host, int *abort, unsigned limit)
{
    T v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!is_sentinel(v)) return v;
    unsigned spins = 0;
    for (;;) {
        __builtin_amdgcn_s_sleep(1);
        v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!is_sentinel(v)) return v;
        ++spins;
        if (spins > limit ||
            ((spins & 255u) == 0 && __hip_atomic_load(err_dev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
            __hip_atomic_store(err_dev, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(err_host, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            *abort = 1;
            return T(0);
        }
    }
}

// Value of dependency column c for right-hand side k.
template <typename T, bool PERS, bool LDS>
__device__ __forceinline__ T dep_value(const TriArgs &a, const Ctx<T> &cx, int c, int k)
{
    if (PERS && c > a.n)
        return poll_slot<T>(cx.mbox_rd + (size_t)(c - a.n - 1) * a.mbox_stride + k, a.err_dev, a.err_host,
                            cx.abort, a.spin);
    if (LDS && c >= cx.lo && c < cx.hi) return cx.xl[(c - cx.lo) * a.R + k];
    const T *p = static_cast<const T *>(a.xw) + (size_t)c * a.R + k;
    // a value of this workgroup from an earlier step (persistent) or of an
    // earlier launch (per-level): workgroup-scope coherence suffices
    if (PERS) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return *p;
}

template <typename T, typename TIn, bool LDS>
__device__ __forceinline__ T rhs_value(const TriArgs &a, const Ctx<T> &cx, int x, int k)
{
    if (LDS) return cx.xl[(x - cx.lo) * a.R + k];  // gathered (and scaled) at kernel start
    const T b = canon(static_cast<T>(static_cast<const TIn *>(a.bin)[(size_t)a.gather[x] * a.R + k]));
    return a.dinv ? scale_rhs(b, static_cast<const T *>(a.dinv)[x]) : b;
}

// Partial sum of one row's off-diagonal terms (lane `lane` of `lanes`).
template <typename T, bool PERS, bool LDS>
__device__ __forceinline__ T row_terms(const TriArgs &a, const Ctx<T> &cx, int x, int k, int lane, int lanes)
{
    const T *ev = static_cast<const T *>(a.ell_val);
    T part = T(0);
    for (int e = lane; e < a.w; e += lanes) {
        const int c = a.ell_col[(size_t)e * a.ld + x];
        const T v = ev[(size_t)e * a.ld + x];
        if (c != a.n) part += v * dep_value<T, PERS, LDS>(a, cx, c, k);
    }
    if (a.tail_ptr) {
        const T *tv = static_cast<const T *>(a.tail_val);
        for (int p = a.tail_ptr[x] + lane; p < a.tail_ptr[x + 1]; p += lanes)
            part += tv[p] * dep_value<T, PERS, LDS>(a, cx, a.tail_col[p], k);
    }
    return part;
}

template <typename T, typename TOut, bool PERS, bool LDS>
__device__ __forceinline__ void finish_row(const TriArgs &a, const Ctx<T> &cx, int x, int k, T s)
{
    if (LDS) cx.xl[(x - cx.lo) * a.R + k] = s;
    if (!PERS) {
        static_cast<T *>(a.xw)[(size_t)x * a.R + k] = s;
    } else if (!LDS || a.write_xw) {
        __hip_atomic_store(static_cast<T *>(a.xw) + (size_t)x * a.R + k, s, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if (PERS) {
        const int slot = a.exp_slot[x];
        if (slot >= 0)
            __hip_atomic_store(cx.mbox_rd + (size_t)slot * a.mbox_stride + k, s, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    if (a.xout) {
        const int dst = a.scatter[x];
        if (dst >= 0) static_cast<TOut *>(a.xout)[(size_t)dst * a.R + k] = static_cast<TOut>(s);
    }
}

// Thread-per-(row, rhs) solve of one row: s = b - sum, in slot order.
template <typename T, typename TIn, typename TOut, bool PERS, bool LDS>
__device__ __forceinline__ void solve_item(const TriArgs &a, const Ctx<T> &cx, int x, int k)
{
    const T *ev = static_cast<const T *>(a.ell_val);
    T s = rhs_value<T, TIn, LDS>(a, cx, x, k);
    for (int e = 0; e < a.w; ++e) {
        const int c = a.ell_col[(size_t)e * a.ld + x];
        const T v = ev[(size_t)e * a.ld + x];
        if (c != a.n) s -= v * dep_value<T, PERS, LDS>(a, cx, c, k);
    }
    if (a.tail_ptr) {
        const T *tv = static_cast<const T *>(a.tail_val);
        for (int p = a.tail_ptr[x]; p < a.tail_ptr[x + 1]; ++p)
            s -= tv[p] * dep_value<T, PERS, LDS>(a, cx, a.tail_col[p], k);
    }
    finish_row<T, TOut, PERS, LDS>(a, cx, x, k, s);
}

// Rows [rb, re) x R right-hand sides, `lanes` lanes per (row, rhs).  With
// lanes > 1 the lanes of a group split the row's terms and combine them with
// a butterfly of cross-lane shuffles inside the wavefront.
template <typename T, typename TIn, typename TOut, bool LDS>
__device__ __forceinline__ void solve_range(const TriArgs &a, const Ctx<T> &cx, int rb, int re, int lanes)
{
    const int R = a.R;
    if (lanes == 1) {
        const int items = (re - rb) * R;
        for (int t = threadIdx.x; t < items; t += blockDim.x) {
            const int q = t / R;
            solve_item<T, TIn, TOut, true, LDS>(a, cx, rb + q, t - q * R);
        }
        return;
    }
    const int items = (re - rb) * R * lanes;
    for (int t0 = 0; t0 < items; t0 += blockDim.x) {
        const int t = t0 + threadIdx.x;
        const bool act = t < items;
        const int lane = t & (lanes - 1);
        const int q = t / lanes;
        const int x = rb + q / R, k = q - (q / R) * R;
        T part = act ? row_terms<T, true, LDS>(a, cx, x, k, lane, lanes) : T(0);
        for (int off = lanes >> 1; off > 0; off >>= 1) part += __shfl_xor(part, off, lanes);
        if (act && lane == 0) finish_row<T, TOut, true, LDS>(a, cx, x, k, rhs_value<T, TIn, LDS>(a, cx, x, k) - part);
    }
}

// One launch per level: rows [row_begin, row_end) of the device order.
template <typename T, typename TIn, typename TOut>
__global__ void __launch_bounds__(256) k_level(TriArgs a)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int items = (a.row_end - a.row_begin) * a.R;
    if (t >= items) return;
    const int q = t / a.R;
    Ctx<T> cx{nullptr, 0, 0, nullptr, nullptr};
    solve_item<T, TIn, TOut, false, false>(a, cx, a.row_begin + q, t - q * a.R);
}

// One launch for the whole solve.  The mailbox half used by a launch is the
// parity of the plan's epoch word; the epoch is read at kernel start and
// advanced by the last workgroup to finish, so consecutive launches (also
// graph replays) alternate halves.  Each workgroup first resets its own slots
// of the other half to the sentinel, ready for the next launch.
template <typename T, typename TIn, typename TOut, bool LDS>
__global__ void __launch_bounds__(1024) k_persistent(TriArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned s_epoch;
    __shared__ int s_abort;
    const int g = blockIdx.x;
    if (threadIdx.x == 0) {
        s_epoch = __hip_atomic_load(a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_abort = 0;
    }
    __syncthreads();
    const unsigned par = s_epoch & 1u;
    T *mbox = static_cast<T *>(a.mbox);
    const size_t half = (size_t)a.nexp * a.mbox_stride;
    Ctx<T> cx;
    cx.xl = reinterpret_cast<T *>(smem);
    cx.lo = LDS ? a.window[2 * g] : 0;
    cx.hi = LDS ? a.window[2 * g + 1] : 0;
    cx.mbox_rd = mbox + (par ? half : 0);
    cx.abort = &s_abort;
    if (a.nexp > 0) {
        T *other = mbox + (par ? 0 : half);
        const size_t e0 = (size_t)a.exp_ptr[g] * a.mbox_stride, e1 = (size_t)a.exp_ptr[g + 1] * a.mbox_stride;
        for (size_t i = e0 + threadIdx.x; i < e1; i += blockDim.x) other[i] = sentinel<T>();
    }
    if (LDS) {
        const TIn *bin = static_cast<const TIn *>(a.bin);
        const int items = (cx.hi - cx.lo) * a.R;
        for (int t = threadIdx.x; t < items; t += blockDim.x) {
            const int q = t / a.R, k = t - q * a.R;
            const T b = canon(static_cast<T>(bin[(size_t)a.gather[cx.lo + q] * a.R + k]));
            cx.xl[t] = a.dinv ? scale_rhs(b, static_cast<const T *>(a.dinv)[cx.lo + q]) : b;
        }
        __syncthreads();
    }
    const int s0 = a.step_ptr[g], s1 = a.step_ptr[g + 1];
    int rb = 0, re = 0, ln = 1;
    if (s0 < s1) {
        rb = a.step_row[2 * s0];
        re = a.step_row[2 * s0 + 1];
        ln = a.step_lanes[s0];
    }
    for (int s = s0; s < s1; ++s) {
        // next step's bounds are loaded while this step runs
        int nrb = 0, nre = 0, nln = 1;
        if (s + 1 < s1) {
            nrb = a.step_row[2 * s + 2];
            nre = a.step_row[2 * s + 3];
            nln = a.step_lanes[s + 1];
        }
        solve_range<T, TIn, TOut, LDS>(a, cx, rb, re, ln);
        __syncthreads();
        if (s_abort) break;
        rb = nrb;
        re = nre;
        ln = nln;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned done = __hip_atomic_fetch_add(&a.epoch[1], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {
            __hip_atomic_store(&a.epoch[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.epoch[0], s_epoch + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Owner-schedule kernel with LDS-staged matrix data.  Workgroup g owns the
// device rows [lo, hi): their right-hand side is gathered into an LDS window
// at kernel start and every solved value replaces its row's b there.  The
// group's steps are cut into chunks of at most RPT * blockDim rows; the ELL
// columns and values, reciprocal diagonal, mailbox slot and scatter target
// of chunk q+1 are loaded into registers while chunk q is solved, then stored
// to the other half of a double buffer in LDS, so a step reads everything but
// cross-group values from LDS.  W is the ELL width; plans with a CSR tail,
// W > 8 or cooperative lanes use k_persistent.
template <typename T, int W, int RPT, bool UNIT>
__global__ void __launch_bounds__(1024) k_owner(TriArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned s_epoch;
    __shared__ int s_abort;
    const int g = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int R = a.R, n = a.n;
    if (tid == 0) {
        s_epoch = __hip_atomic_load(a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_abort = 0;
    }
    __syncthreads();
    const unsigned par = s_epoch & 1u;
    T *mbox = static_cast<T *>(a.mbox);
    const size_t half = (size_t)a.nexp * a.mbox_stride;
    T *mrd = mbox + (par ? half : 0);
    const int lo = a.window[2 * g], hi = a.window[2 * g + 1];
    const int CH = RPT * nt;
    // LDS: window [win*R] T, then two buffers of { vals[W][CH] T, cols[W][CH], slot[CH], dst[CH] }
    T *xl = reinterpret_cast<T *>(smem);
    const size_t win_bytes = (((size_t)(hi - lo) * R * sizeof(T)) + 15) & ~(size_t)15;
    const size_t buf_bytes = (size_t)CH * (W * sizeof(T) + (W + 2) * sizeof(int));
    auto bvals = [&](int b) { return reinterpret_cast<T *>(smem + win_bytes + b * buf_bytes); };
    auto bcols = [&](int b) { return reinterpret_cast<int *>(smem + win_bytes + b * buf_bytes + (size_t)CH * W * sizeof(T)); };
    auto bslot = [&](int b) { return bcols(b) + (size_t)W * CH; };
    auto bdst = [&](int b) { return bslot(b) + CH; };

    if (a.nexp > 0) {
        T *other = mbox + (par ? 0 : half);
        const size_t e0 = (size_t)a.exp_ptr[g] * a.mbox_stride, e1 = (size_t)a.exp_ptr[g + 1] * a.mbox_stride;
        for (size_t i = e0 + tid; i < e1; i += nt) other[i] = sentinel<T>();
    }
    {
        const int items = (hi - lo) * R;
        for (int t = tid; t < items; t += nt) {
            const int q = t / R, k = t - q * R;
            const size_t src = (size_t)a.gather[lo + q] * R + k;
            const T b = canon(a.in_f64 ? static_cast<T>(static_cast<const double *>(a.bin)[src])
                                       : static_cast<T>(static_cast<const float *>(a.bin)[src]));
            xl[t] = UNIT ? b : scale_rhs(b, static_cast<const T *>(a.dinv)[lo + q]);
        }
    }
    const T *ev = static_cast<const T *>(a.ell_val);
    // registers of one chunk prefetch
    int rc[RPT][W];
    T rv[RPT][W];
    int rs[RPT], rt[RPT];
    auto chunk_rows = [&](int q, int &r0, int &r1) {
        const int f = a.chunk_step[2 * q], e = a.chunk_step[2 * q + 1];
        r0 = a.step_row[2 * f];
        r1 = a.step_row[2 * (e - 1) + 1];
    };
    auto load_chunk = [&](int q) {
        int r0, r1;
        chunk_rows(q, r0, r1);
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int row = r0 + tid + i * nt;
            if (row < r1) {
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    rc[i][e] = a.ell_col[(size_t)e * a.ld + row];
                    rv[i][e] = ev[(size_t)e * a.ld + row];
                }
                rs[i] = a.exp_slot[row];
                rt[i] = a.xout ? a.scatter[row] : -1;
            }
        }
    };
    auto store_chunk = [&](int q, int b) {
        int r0, r1;
        chunk_rows(q, r0, r1);
        T *vb = bvals(b);
        int *cb = bcols(b);
        int *sb = bslot(b);
        int *tb = bdst(b);
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int rr = tid + i * nt;
            if (r0 + rr < r1) {
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    cb[e * CH + rr] = rc[i][e];
                    vb[e * CH + rr] = rv[i][e];
                }
                sb[rr] = rs[i];
                tb[rr] = rt[i];
            }
        }
    };
    const int c0 = a.chunk_ptr[g], c1 = a.chunk_ptr[g + 1];
    if (c0 < c1) {
        load_chunk(c0);
        store_chunk(c0, 0);
    }
    __syncthreads();
    bool aborted = false;
    for (int q = c0; q < c1 && !aborted; ++q) {
        const int b = (q - c0) & 1;
        if (q + 1 < c1) load_chunk(q + 1);
        int cr0, cr1;
        chunk_rows(q, cr0, cr1);
        const T *vb = bvals(b);
        const int *cb = bcols(b);
        const int *sb = bslot(b);
        const int *tb = bdst(b);
        const int f = a.chunk_step[2 * q], e_ = a.chunk_step[2 * q + 1];
        for (int s = f; s < e_; ++s) {
            const int rb = a.step_row[2 * s], re = a.step_row[2 * s + 1];
            const int items = (re - rb) * R;
            const int js = s - a.step_ptr[g];
            const bool tr = a.trace && tid == 0 && js < a.trace_stride;
            if (tr) a.trace[2 * ((size_t)g * a.trace_stride + js)] = __builtin_amdgcn_s_memrealtime();
            for (int t = tid; t < items; t += nt) {
                const int qq = t / R, k = t - qq * R;
                const int x = rb + qq, i = x - cr0;
                T sv = xl[(x - lo) * R + k];
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    const int c = cb[e * CH + i];
                    if (c != n) {
                        T dep;
                        if (c > n)
                            dep = poll_slot<T>(mrd + (size_t)(c - n - 1) * a.mbox_stride + k, a.err_dev, a.err_host,
                                               &s_abort, a.spin);
                        else
                            dep = xl[(c - lo) * R + k];
                        sv -= vb[e * CH + i] * dep;
                    }
                }
                xl[(x - lo) * R + k] = sv;
                if (a.write_xw) static_cast<T *>(a.xw)[(size_t)x * R + k] = sv;
                const int slot = sb[i];
                if (slot >= 0)
                    __hip_atomic_store(mrd + (size_t)slot * a.mbox_stride + k, sv, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                const int dst = tb[i];
                if (dst >= 0) {
                    if (a.out_f64) static_cast<double *>(a.xout)[(size_t)dst * R + k] = static_cast<double>(sv);
                    else static_cast<float *>(a.xout)[(size_t)dst * R + k] = static_cast<float>(sv);
                }
            }
            __syncthreads();
            if (tr) a.trace[2 * ((size_t)g * a.trace_stride + js) + 1] = __builtin_amdgcn_s_memrealtime();
            if (s_abort) {
                aborted = true;
                break;
            }
        }
        if (!aborted && q + 1 < c1) {
            store_chunk(q + 1, b ^ 1);
            __syncthreads();
        }
    }
    __syncthreads();
    if (tid == 0) {
        const unsigned done = __hip_atomic_fetch_add(&a.epoch[1], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {
            __hip_atomic_store(&a.epoch[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.epoch[0], s_epoch + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// LDS bytes of k_owner for a window of `win` rows.
size_t owner_lds_bytes(int win, int R, int W, int rows_per_chunk, bool unit, size_t tsize)
{
    const size_t win_bytes = (((size_t)win * R * tsize) + 15) & ~(size_t)15;
    (void)unit;
    const size_t buf = (size_t)rows_per_chunk * (W * tsize + (W + 2) * sizeof(int));
    return win_bytes + 2 * buf;
}

using OwnerKernel = void (*)(TriArgs);

template <typename T, int W, int RPT>
OwnerKernel owner_kernel_w(bool unit)
{
    return unit ? k_owner<T, W, RPT, true> : k_owner<T, W, RPT, false>;
}

template <typename T, int RPT>
OwnerKernel owner_kernel_r(int w, bool unit)
{
    switch (w) {
    case 1: return owner_kernel_w<T, 1, RPT>(unit);
    case 2: return owner_kernel_w<T, 2, RPT>(unit);
    case 3: return owner_kernel_w<T, 3, RPT>(unit);
    case 4: return owner_kernel_w<T, 4, RPT>(unit);
    case 5: return owner_kernel_w<T, 5, RPT>(unit);
    case 6: return owner_kernel_w<T, 6, RPT>(unit);
    case 7: return owner_kernel_w<T, 7, RPT>(unit);
    case 8: return owner_kernel_w<T, 8, RPT>(unit);
    default: return nullptr;
    }
}

template <typename T>
OwnerKernel owner_kernel(int w, int rpt, bool unit)
{
    if (rpt == 1) return owner_kernel_r<T, 1>(w, unit);
    if (rpt == 2) return owner_kernel_r<T, 2>(w, unit);
    if (rpt == 4) return owner_kernel_r<T, 4>(w, unit);
    return nullptr;
}

// Owner-schedule kernel with one compute wave and one fetch wave (one RHS).
// The compute wave only reads LDS, does the arithmetic and issues stores, so
// it never waits on global memory.  The fetch wave (a) streams each chunk
// (ELL columns and values, reciprocal diagonal, mailbox slot and scatter
// target per row, the chunk's step bounds and its cross-group entry list)
// into a ring of three LDS buffers, and (b) polls the mailbox slots of the
// cross-group entries of the next steps, up to 64 * kWsPerLane entries at
// once, writing arrived values into the buffer's staging grid and publishing
// in LDS the last step whose entries have all arrived.  The compute wave
// solves step s once that counter reaches s and reports each finished step,
// which frees buffers for the fetch wave.  All waits in both roles are
// bounded.
constexpr int kWsBuffers = 3;
constexpr int kWsPerLane = 16;
constexpr int kWsHead = 8;  // ints: first step, end step, first row, first entry, end entry

template <typename T, int W>
struct WsLayout {
    size_t win, buf;
    size_t o_vals, o_stage, o_cols, o_slot, o_dst, o_ent, o_head, o_step;
    __host__ __device__ WsLayout(int rows, int CH, bool unit)
    {
        win = (((size_t)rows * sizeof(T)) + 15) & ~(size_t)15;
        o_vals = 0;
        (void)unit;
        o_stage = o_vals + (size_t)W * CH * sizeof(T);
        o_cols = o_stage + (size_t)W * CH * sizeof(T);
        o_slot = o_cols + (size_t)W * CH * sizeof(int);
        o_dst = o_slot + (size_t)CH * sizeof(int);
        o_ent = o_dst + (size_t)CH * sizeof(int);
        o_head = o_ent + 2 * (size_t)W * CH * sizeof(int);
        o_step = o_head + kWsHead * sizeof(int);
        buf = (o_step + 3 * (size_t)CH * sizeof(int) + 15) & ~(size_t)15;
    }
    __host__ __device__ size_t total() const { return win + kWsBuffers * buf; }
};

template <typename T, int W, bool UNIT>
__global__ void __launch_bounds__(128) k_owner_split(TriArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned s_epoch;
    __shared__ int s_abort;
    __shared__ int s_fetched;  // last step whose cross-group values are staged
    __shared__ int s_done;     // last step the compute wave finished
    const int g = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = a.n, CH = a.chunk_rows;
    const int s0 = a.step_ptr[g], s1 = a.step_ptr[g + 1];
    const int c0 = a.chunk_ptr[g], c1 = a.chunk_ptr[g + 1];
    if (tid == 0) {
        s_epoch = __hip_atomic_load(a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_abort = 0;
        s_fetched = s0 - 1;
        s_done = s0 - 1;
    }
    __syncthreads();
    const unsigned par = s_epoch & 1u;
    T *mbox = static_cast<T *>(a.mbox);
    const size_t half = (size_t)a.nexp * a.mbox_stride;
    T *mrd = mbox + (par ? half : 0);
    const int lo = a.window[2 * g], hi = a.window[2 * g + 1];
    const WsLayout<T, W> L(hi - lo, CH, UNIT);
    T *xl = reinterpret_cast<T *>(smem);
    auto buf = [&](int q) { return smem + L.win + (size_t)((q - c0) % kWsBuffers) * L.buf; };
    if (a.nexp > 0) {
        T *other = mbox + (par ? 0 : half);
        const size_t e0 = (size_t)a.exp_ptr[g] * a.mbox_stride, e1 = (size_t)a.exp_ptr[g + 1] * a.mbox_stride;
        for (size_t i = e0 + tid; i < e1; i += blockDim.x) other[i] = sentinel<T>();
    }
    for (int t = tid; t < hi - lo; t += blockDim.x) {
        const size_t src = (size_t)a.gather[lo + t];
        const T b = canon(a.in_f64 ? static_cast<T>(static_cast<const double *>(a.bin)[src])
                                   : static_cast<T>(static_cast<const float *>(a.bin)[src]));
        xl[t] = UNIT ? b : scale_rhs(b, static_cast<const T *>(a.dinv)[lo + t]);
    }
    __syncthreads();
    volatile int *v_fetched = &s_fetched;
    volatile int *v_done = &s_done;
    volatile int *v_abort = &s_abort;
    auto raise = [&]() {
        *v_abort = 1;
        __hip_atomic_store(a.err_dev, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.err_host, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    };
    if (wave == 1) {
        // ---------------- fetch wave ----------------
        const T *ev = static_cast<const T *>(a.ell_val);
        int q_next = c0;          // next chunk to load
        int loaded_end = s0;      // steps below this lie in loaded chunks
        int pub = s0 - 1;         // last published step
        int qa = c0;              // chunk holding step pub + 1
        int e_cur = a.rem_ptr[s0];
        unsigned idle = 0;
        while (pub < s1 - 1 && !*v_abort) {
            // keep chunk qa and the next one resident
            while (q_next < c1 && q_next <= qa + 1) {
                if (q_next - c0 >= kWsBuffers) {
                    const int need = a.chunk_step[2 * (q_next - kWsBuffers) + 1] - 1;
                    unsigned spins = 0;
                    while (*v_done < need && !*v_abort) {
                        if (++spins > a.spin) raise();
                        __builtin_amdgcn_s_sleep(1);
                    }
                    if (*v_abort) break;
                }
                unsigned char *B = buf(q_next);
                T *vb = reinterpret_cast<T *>(B + L.o_vals);
                int *cb = reinterpret_cast<int *>(B + L.o_cols);
                int *sb = reinterpret_cast<int *>(B + L.o_slot);
                int *tb = reinterpret_cast<int *>(B + L.o_dst);
                int *eb = reinterpret_cast<int *>(B + L.o_ent);
                int *hb = reinterpret_cast<int *>(B + L.o_head);
                int *pb = reinterpret_cast<int *>(B + L.o_step);
                const int f = a.chunk_step[2 * q_next], e = a.chunk_step[2 * q_next + 1];
                const int r0 = a.step_row[2 * f], r1 = a.step_row[2 * (e - 1) + 1];
                const int x0 = a.rem_ptr[f], x1 = a.rem_ptr[e];
                for (int i = lane; i < r1 - r0; i += 64) {
                    const int row = r0 + i;
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        cb[k * CH + i] = a.ell_col[(size_t)k * a.ld + row];
                        vb[k * CH + i] = ev[(size_t)k * a.ld + row];
                    }
                    sb[i] = a.exp_slot[row];
                    tb[i] = a.xout ? a.scatter[row] : -1;
                }
                for (int i = lane; i < 2 * (x1 - x0); i += 64) eb[i] = a.rem_ent[2 * x0 + i];
                for (int i = lane; i < e - f; i += 64) {
                    pb[3 * i] = a.step_row[2 * (f + i)];
                    pb[3 * i + 1] = a.step_row[2 * (f + i) + 1];
                    pb[3 * i + 2] = a.rem_ptr[f + i + 1];
                }
                if (lane == 0) {
                    hb[0] = f;
                    hb[1] = e;
                    hb[2] = r0;
                    hb[3] = x0;
                    hb[4] = x1;
                }
                loaded_end = e;
                ++q_next;
            }
            if (*v_abort) break;
            // resident chunks qa and (if loaded) qa + 1
            const int *ha = reinterpret_cast<const int *>(buf(qa) + L.o_head);
            const bool has_b = qa + 1 < q_next;
            const int *hbn = reinterpret_cast<const int *>(buf(qa + 1) + L.o_head);
            const int ent_split = has_b ? hbn[3] : ha[4];
            const int e_lim = has_b ? hbn[4] : ha[4];
            const int e_end = min(e_cur + 64 * kWsPerLane, e_lim);
            int first_pending = e_end;
#pragma unroll
            for (int j = 0; j < kWsPerLane; ++j) {
                const int idx = e_cur + lane + 64 * j;
                if (idx < e_end) {
                    const bool in_b = idx >= ent_split;
                    unsigned char *B = in_b ? buf(qa + 1) : buf(qa);
                    const int li = idx - (in_b ? hbn[3] : ha[3]);
                    const int *eb = reinterpret_cast<const int *>(B + L.o_ent);
                    const int pos = eb[2 * li], slot = eb[2 * li + 1];
                    const T v = __hip_atomic_load(mrd + (size_t)slot * a.mbox_stride, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
                    if (is_sentinel(v)) first_pending = min(first_pending, idx);
                    else reinterpret_cast<T *>(B + L.o_stage)[pos] = v;
                }
            }
            for (int off = 32; off > 0; off >>= 1) first_pending = min(first_pending, __shfl_xor(first_pending, off));
            // publish every step whose entries all lie before first_pending
            int np = pub;
            for (;;) {
                const int s = np + 1;
                if (s >= loaded_end) break;
                const int *hs = (s < ha[1]) ? ha : hbn;
                const int *ps = reinterpret_cast<const int *>(reinterpret_cast<const unsigned char *>(hs) - L.o_head +
                                                              L.o_step);
                if (ps[3 * (s - hs[0]) + 2] > first_pending) break;
                np = s;
            }
            e_cur = first_pending;
            if (np > pub) {
                pub = np;
                if (lane == 0) *v_fetched = pub;
                idle = 0;
                while (qa + 1 < q_next && a.chunk_step[2 * qa + 1] <= pub + 1) ++qa;
            } else {
                if (++idle > a.spin) {
                    raise();
                    break;
                }
                if ((idle & 255u) == 0 && __hip_atomic_load(a.err_dev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    *v_abort = 1;
                __builtin_amdgcn_s_sleep(1);
            }
        }
    } else {
        // ---------------- compute wave ----------------
        int q = c0;
        const unsigned char *B = buf(q);
        const int *hb = reinterpret_cast<const int *>(B + L.o_head);
        for (int s = s0; s < s1; ++s) {
            const bool tr = a.trace && lane == 0 && (s - s0) < a.trace_stride;
            if (tr) a.trace[2 * ((size_t)g * a.trace_stride + (s - s0))] = __builtin_amdgcn_s_memrealtime();
            unsigned spins = 0;
            while (*v_fetched < s) {
                if (*v_abort) break;
                if (++spins > (a.spin << 4)) {
                    raise();
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (*v_abort) break;
            if (s >= hb[1]) {  // next chunk (its header is valid once step s is published)
                ++q;
                B = buf(q);
                hb = reinterpret_cast<const int *>(B + L.o_head);
            }
            const T *vb = reinterpret_cast<const T *>(B + L.o_vals);
            const T *st = reinterpret_cast<const T *>(B + L.o_stage);
            const int *cb = reinterpret_cast<const int *>(B + L.o_cols);
            const int *sb = reinterpret_cast<const int *>(B + L.o_slot);
            const int *tb = reinterpret_cast<const int *>(B + L.o_dst);
            const int *pb = reinterpret_cast<const int *>(B + L.o_step);
            const int cr0 = hb[2];
            const int js = s - hb[0];
            const int rb = pb[3 * js], re = pb[3 * js + 1];
            for (int x = rb + lane; x < re; x += 64) {
                const int i = x - cr0;
                T sv = xl[x - lo];
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    const int c = cb[k * CH + i];
                    if (c != n) sv -= vb[k * CH + i] * (c > n ? st[i * W + k] : xl[c - lo]);
                }
                xl[x - lo] = sv;
                if (a.write_xw) static_cast<T *>(a.xw)[x] = sv;
                const int slot = sb[i];
                if (slot >= 0)
                    __hip_atomic_store(mrd + (size_t)slot * a.mbox_stride, sv, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                const int dst = tb[i];
                if (dst >= 0) {
                    if (a.out_f64) static_cast<double *>(a.xout)[dst] = static_cast<double>(sv);
                    else static_cast<float *>(a.xout)[dst] = static_cast<float>(sv);
                }
            }
            if (tr) a.trace[2 * ((size_t)g * a.trace_stride + (s - s0)) + 1] = __builtin_amdgcn_s_memrealtime();
            if (lane == 0) *v_done = s;
        }
    }
    __syncthreads();
    if (tid == 0) {
        const unsigned done = __hip_atomic_fetch_add(&a.epoch[1], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {
            __hip_atomic_store(&a.epoch[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.epoch[0], s_epoch + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Dataflow owner kernel.  A workgroup owns a part of the rows (a contiguous
// device-row window in level order) and runs three kinds of wavefronts:
//   compute waves  take the group's steps round-robin; a step is one level
//                  piece of at most 64 (row, rhs) items, solved one item per
//                  lane.  Each dependency is read from LDS and re-read until
//                  it no longer holds the sentinel, so a row starts as soon
//                  as its own inputs exist: there is no per-level barrier.
//                  The matrix data of a wave's next step is loaded into
//                  registers while the current one is solved; compute waves
//                  issue no global stores, so their waits cover loads only.
//   import wave    polls the mailbox slots this group reads (lane l takes
//                  imports l, l+64, ... in order of first use) and copies
//                  each value into LDS when it arrives;
//   export wave    watches the group's exported rows in LDS and writes each
//                  one to its mailbox slot as soon as it is solved.
// Any row waits only on rows of lower levels, and every wave handles its
// items in level order, so the row of lowest level not yet solved can always
// proceed: the grid drains as long as all workgroups are co-resident.
// The summation order (ELL slots, then the CSR tail, then the reciprocal
// diagonal) is the one of k_level, so results are bit-identical to it.
template <typename T> __device__ __forceinline__ T lds_get(const T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T> __device__ __forceinline__ void lds_put(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <typename T, int W> struct DfRegs {
    int c[W];  // columns as loaded, then LDS byte offsets
    T v[W];
    T b;       // right-hand side of the lane's item
    int r, k;  // the lane's item: window row, right-hand side
    int xo;    // LDS byte offset of the item's value
};

// TRACE: per-step clocks (tri_plan_trace).  Untraced instances read no clock
// in the step loop: the clock is a scalar-memory read, and with one possibly
// outstanding the compiler must drain every LDS access before the next step.
template <typename T, int W, bool UNIT, bool TAIL, bool R1, bool TRACE>
__global__ void __launch_bounds__(512) k_dataflow(TriArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned s_epoch;
    __shared__ int s_abort;
    __shared__ int s_part;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwc = (nt >> 6) - 2;
    const int R = R1 ? 1 : a.R;
    if (tid == 0) {
        s_epoch = __hip_atomic_load(a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_abort = 0;
    }
    __syncthreads();
    const unsigned par = s_epoch & 1u;
    T *mbox = static_cast<T *>(a.mbox);
    const size_t half = (size_t)a.nexp * a.mbox_stride;
    T *mrd = mbox + (par ? half : 0);
    // Parts: workgroup g runs part g, or (queue mode) the workgroups take
    // parts from a counter in index order until none is left.  Queue-mode
    // parts are numbered so that a part reads only from lower-numbered ones,
    // and a part is taken only by a running workgroup, so the solve needs no
    // more workgroups resident than one.
    for (int round = 0;; ++round) {
    if (a.queue) {
        if (tid == 0) s_part = (int)__hip_atomic_fetch_add(&a.epoch[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
    } else if (round > 0) {
        break;
    }
    const int g = a.queue ? s_part : (int)blockIdx.x;
    if (g >= a.nparts) break;
    const int lo = a.window[2 * g], hi = a.window[2 * g + 1], win = hi - lo;
    const int i0 = a.imp_ptr[g], nimp = a.imp_ptr[g + 1] - i0;
    const int e0 = a.exp_ptr[g], nex = a.exp_ptr[g + 1] - e0;
    const int s0 = a.step_ptr[g], ns = a.step_ptr[g + 1] - s0;
    // LDS value rows: x [win][R], b [win][R], imports [nimp][R], one zero
    // row (the target of ELL padding); then import slots, export rows
    // (window offsets) and step bounds (window offsets)
    T *xl = reinterpret_cast<T *>(smem);
    T *bl = xl + (size_t)win * R;
    T *im = bl + (size_t)win * R;
    const size_t ib = (((size_t)2 * win + nimp + 1) * R * sizeof(T) + 15) & ~(size_t)15;
    int *isl = reinterpret_cast<int *>(smem + ib);
    int *erl = isl + nimp;
    int *stl = erl + nex;
    // when tracing: 2*ns clocks after the ints, at an 8-byte boundary
    unsigned long long *ltr =
        reinterpret_cast<unsigned long long *>(smem + ((ib + (size_t)(nimp + nex + 2 * ns) * 4 + 7) & ~(size_t)7));

    if (a.nexp > 0) {
        T *other = mbox + (par ? 0 : half);
        const size_t m0 = (size_t)e0 * a.mbox_stride, m1 = (size_t)(e0 + nex) * a.mbox_stride;
        for (size_t i = m0 + tid; i < m1; i += nt) other[i] = sentinel<T>();
    }
    // Fill LDS.  Every thread keeps kFill independent loads in flight (the
    // start-up of all groups delays the first rows of the solve).
    constexpr int kFill = 8;
    for (int t = tid; t < win * R; t += nt) xl[t] = sentinel<T>();
    for (int t = tid; t < (nimp + 1) * R; t += nt) im[t] = t < nimp * R ? sentinel<T>() : T(0);
    auto fill_b = [&](const auto *bin) {
        for (int t0 = tid; t0 < win * R; t0 += kFill * nt) {
            int gi[kFill];
#pragma unroll
            for (int u = 0; u < kFill; ++u) {
                const int t = min(t0 + u * nt, win * R - 1);
                gi[u] = a.gather[lo + (R1 ? t : t / R)];
            }
            T bv[kFill], dd[kFill];
#pragma unroll
            for (int u = 0; u < kFill; ++u) {
                const int t = min(t0 + u * nt, win * R - 1);
                bv[u] = canon(static_cast<T>(bin[(size_t)gi[u] * R + (R1 ? 0 : t % R)]));
                if (!UNIT) dd[u] = static_cast<const T *>(a.dinv)[lo + (R1 ? t : t / R)];
            }
            if (!UNIT) {
#pragma unroll
                for (int u = 0; u < kFill; ++u) bv[u] = scale_rhs(bv[u], dd[u]);
            }
#pragma unroll
            for (int u = 0; u < kFill; ++u)
                if (t0 + u * nt < win * R) bl[t0 + u * nt] = bv[u];
        }
    };
    if (a.in_f64) fill_b(static_cast<const double *>(a.bin));
    else fill_b(static_cast<const float *>(a.bin));
    auto copy_ints = [&](int *dst, const int32_t *src, int count, int add) {
        for (int t0 = tid; t0 < count; t0 += kFill * nt) {
            int v[kFill];
#pragma unroll
            for (int u = 0; u < kFill; ++u) v[u] = src[min(t0 + u * nt, count - 1)];
#pragma unroll
            for (int u = 0; u < kFill; ++u)
                if (t0 + u * nt < count) dst[t0 + u * nt] = v[u] + add;
        }
    };
    copy_ints(isl, a.imp_slot + i0, nimp, 0);
    copy_ints(erl, a.exp_row + e0, nex, -lo);
    copy_ints(stl, a.step_row + 2 * s0, 2 * ns, -lo);
    __syncthreads();
    const unsigned long long t_fill = TRACE ? __builtin_amdgcn_s_memrealtime() : 0ull;

    if (wv < nwc) {
        const T *ev = static_cast<const T *>(a.ell_val);
        const T *tv = static_cast<const T *>(a.tail_val);
        // Lanes past the step's items repeat its last item, so loads and
        // their uses are unconditional and the compiler's load waits stay
        // exact.  The ELL slots of a step's rows are contiguous per slot:
        // buffer loads with one per-lane byte offset and a per-slot scalar
        // offset (no 64-bit address arithmetic per load).
        const int nb_col = (int)min((size_t)0x7fffffff, (size_t)a.w * a.ld * sizeof(int32_t));
        const int nb_val = (int)min((size_t)0x7fffffff, (size_t)a.w * a.ld * sizeof(T));
        const __amdgpu_buffer_rsrc_t rcol =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t *>(a.ell_col), 0, nb_col, 0x00020000);
        const __amdgpu_buffer_rsrc_t rval =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(ev), 0, nb_val, 0x00020000);
        unsigned char *xb = reinterpret_cast<unsigned char *>(xl);
        // Everything a step needs besides its inputs is prepared when its
        // register set is filled, steps ahead: the matrix loads, the lane's
        // item (row r, right-hand side k), its right-hand-side value from LDS
        // and the LDS byte offset its result goes to.
        auto load = [&](DfRegs<T, W> &u, int rb, int re) {
            const int it = min(lane, (re - rb) * R - 1);
            const int q = R1 ? it : it / R;
            u.k = R1 ? 0 : it - q * R;
            u.r = rb + q;
            const int x = lo + u.r;
#pragma unroll
            for (int e = 0; e < W; ++e) {
                u.c[e] = (int)__builtin_amdgcn_raw_buffer_load_b32(rcol, x * (int)sizeof(int32_t),
                                                                   e * a.ld * (int)sizeof(int32_t), 0);
                if constexpr (sizeof(T) == 8)
                    u.v[e] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rval, x * 8, e * a.ld * 8, 0));
                else
                    u.v[e] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rval, x * 4, e * a.ld * 4, 0));
            }
            u.xo = (u.r * R + u.k) * (int)sizeof(T);
            u.b = bl[u.r * R + u.k];
        };
        // columns (LDS value rows; ELL padding names the zero row) become
        // LDS byte offsets one step before their use
        auto to_offsets = [&](DfRegs<T, W> &u) {
#pragma unroll
            for (int e = 0; e < W; ++e) u.c[e] = (R1 ? u.c[e] : u.c[e] * R + u.k) * (int)sizeof(T);
        };
        const int ntr = TRACE ? min(ns, a.trace_stride - 1) : 0;
        bool aborted = false;
        // Solve step j from registers u.  Its inputs are read first; while
        // they are in flight the loads of step j+K-1 (bounds fb, fe, read one
        // step earlier) go into `fill` and the bounds of step j+K are read;
        // after the result is stored the next step's columns become offsets.  Padding subtracts 0 * 0,
        // which leaves the value unchanged bit for bit.  An input not solved
        // yet holds the sentinel (a NaN), so a lane that read one ends with a
        // NaN: one test of the result covers every input.  Only then are the
        // inputs checked one by one (the result may be a NaN of the data,
        // which passes) and re-read until none holds the sentinel, and the
        // value is recomputed in the same order.
        auto process = [&](const DfRegs<T, W> &u, DfRegs<T, W> &fill, DfRegs<T, W> &next, int j, int &fb, int &fe,
                           int nq) {
            if (TRACE && j < ntr && lane == 0) ltr[2 * j] = __builtin_amdgcn_s_memrealtime();
            T dep[W];
#pragma unroll
            for (int e = 0; e < W; ++e) dep[e] = lds_get(reinterpret_cast<const T *>(xb + u.c[e]));
            __builtin_amdgcn_sched_barrier(0);  // the reads go first
            load(fill, fb, fe);
            fb = stl[2 * nq];
            fe = stl[2 * nq + 1];
            T acc = u.b;
#pragma unroll
            for (int e = 0; e < W; ++e) acc -= u.v[e] * dep[e];
            if (__ballot(acc != acc) != 0) {
                bool pend = false;
#pragma unroll
                for (int e = 0; e < W; ++e) pend |= is_sentinel(dep[e]);
                unsigned spins = 0;
                while (pend) {
                    // re-read every input (one LDS round trip per poll; inputs
                    // already present do not change)
#pragma unroll
                    for (int e = 0; e < W; ++e) dep[e] = lds_get(reinterpret_cast<const T *>(xb + u.c[e]));
                    pend = false;
#pragma unroll
                    for (int e = 0; e < W; ++e) pend |= is_sentinel(dep[e]);
                    if (pend && (++spins & 63u) == 0) {
                        if (lds_get(&s_abort)) {
                            aborted = true;
                            break;
                        }
                        if (spins > (a.spin << 4)) {
                            lds_put(&s_abort, 2);
                            aborted = true;
                            break;
                        }
                    }
                }
                acc = u.b;
#pragma unroll
                for (int e = 0; e < W; ++e) acc -= u.v[e] * dep[e];
            }
            if (TAIL) {
                const int x = lo + u.r;
                for (int p = a.tail_ptr[x]; p < a.tail_ptr[x + 1]; ++p) {
                    const int o = a.tail_col[p] * R + u.k;
                    T dd = lds_get(xl + o);
                    unsigned sp = 0;
                    while (is_sentinel(dd)) {
                        dd = lds_get(xl + o);
                        if ((++sp & 63u) == 0) {
                            if (lds_get(&s_abort)) {
                                aborted = true;
                                break;
                            }
                            if (sp > (a.spin << 4)) {
                                lds_put(&s_abort, 2);
                                aborted = true;
                                break;
                            }
                        }
                    }
                    acc -= tv[p] * dd;
                }
            }
            // lanes past the items store the same value as the last item's lane;
            // the store is the end of the dependency chain, so nothing of the
            // next step (which waits for this step's bounds read) is
            // scheduled above it
            lds_put(reinterpret_cast<T *>(xb + u.xo), acc);
            __builtin_amdgcn_sched_barrier(0);
            to_offsets(next);
            if (TRACE && j < ntr && lane == 0) ltr[2 * j + 1] = __builtin_amdgcn_s_memrealtime();
        };
        // The wave walks its own steps [j, jend) in order.  K register sets
        // rotate: while step j is solved from one, the next K-2 steps have
        // their matrix loads in flight and step j+K-1's loads are issued into
        // the set just freed.  K is as large as the vector-memory counter
        // allows (it holds 63 outstanding loads; a step issues 2W), so a step
        // finds its data loaded although the memory latency spans several
        // steps.  Loads past the last step repeat it, so every path issues
        // the same loads; the loop runs whole rotations with a single exit at
        // the bottom and no register moves, so the compiler's load waits are
        // exact.
        int j = a.wave_ptr[g * nwc + wv] - s0;
        const int jend = a.wave_ptr[g * nwc + wv + 1] - s0;
        const int last = jend - 1;
        constexpr int K = W == 1 ? 12 : (W == 2 ? 10 : (W == 3 ? (R1 ? 9 : 8) : (W <= 5 ? 6 : (W <= 8 ? 4 : 3))));
        constexpr int kAhead = K - 1;
        DfRegs<T, W> S[K];
        auto first = [&](DfRegs<T, W> &u, int q) {
            q = min(q, last);
            load(u, stl[2 * q], stl[2 * q + 1]);
        };
        int fb = 0, fe = 0;
        auto run = [&](const DfRegs<T, W> &u, DfRegs<T, W> &fill, DfRegs<T, W> &next) {
            process(u, fill, next, j, fb, fe, min(j + kAhead + 1, last));
            j += 1;
        };
        if (j < jend) {
#pragma unroll
            for (int p = 0; p < K - 1; ++p) first(S[p], j + p);
            to_offsets(S[0]);
            fb = stl[2 * min(j + kAhead, last)];
            fe = stl[2 * min(j + kAhead, last) + 1];
            const int rounds = (jend - j) / K, rest = (jend - j) - K * rounds;
            for (int q = 0; q < rounds; ++q) {
#pragma unroll
                for (int p = 0; p < K; ++p) run(S[p], S[(p + K - 1) % K], S[(p + 1) % K]);
                if (__ballot(aborted) != 0) break;
            }
#pragma unroll
            for (int p = 0; p < K - 1; ++p)
                if (rest > p && __ballot(aborted) == 0) run(S[p], S[(p + K - 1) % K], S[(p + 1) % K]);
        }
    } else if (wv == nwc) {
        // import wave: lane l owns items l, l+64, l+128, ... (level order).
        // Each poll round reads those of the lane's next kLook items that have
        // not arrived yet, copies every new arrival into LDS, and moves the
        // lane past the delivered prefix.  One round trip thus delivers
        // several levels' worth of a lane's items without re-reading any.
        constexpr int kLook = 2;
        const int items = nimp * R;
        const int xoff = 2 * win * R;
        int it = lane;
        unsigned got = 0;  // bit u: item it + 64 u already delivered
        unsigned idle = 0;
        while (__ballot(it < items) != 0) {
            if (it < items) {
                T v[kLook];
#pragma unroll
                for (int u = 0; u < kLook; ++u) {
                    const int i2 = it + 64 * u;
                    v[u] = sentinel<T>();
                    if (i2 < items && !((got >> u) & 1u)) {
                        const int q = i2 / R, k = i2 - q * R;
                        v[u] = __hip_atomic_load(mrd + (size_t)isl[q] * a.mbox_stride + k, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                bool fresh = false;
#pragma unroll
                for (int u = 0; u < kLook; ++u) {
                    if (!is_sentinel(v[u])) {
                        lds_put(xl + xoff + it + 64 * u, v[u]);
                        got |= 1u << u;
                        fresh = true;
                    }
                }
                while (got & 1u) {
                    got >>= 1;
                    it += 64;
                }
                if (fresh) {
                    idle = 0;
                } else if (++idle > a.spin) {
                    lds_put(&s_abort, 2);
                    it = items;
                } else if ((idle & 255u) == 0 &&
                           __hip_atomic_load(a.err_dev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    lds_put(&s_abort, 1);  // another workgroup gave up
                    it = items;
                }
            }
            if (lds_get(&s_abort)) break;
        }
    } else {
        // export wave: each lane watches its next exported item; a round in
        // which no lane found a new value sleeps briefly, so the wave does
        // not take issue slots and LDS bandwidth from the compute waves
        const int items = nex * R;
        int it = lane;
        unsigned idle = 0, rounds = 0;
        int q = it / R, k = it - q * R;
        int row = it < items ? erl[q] : 0;
        while (__ballot(it < items) != 0) {
            bool moved = false;
            if (it < items) {
                const T v = lds_get(xl + row * R + k);
                if (!is_sentinel(v)) {
                    __hip_atomic_store(mrd + (size_t)(e0 + q) * a.mbox_stride + k, v, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    it += 64;
                    idle = 0;
                    moved = true;
                    if (it < items) {
                        q = it / R;
                        k = it - q * R;
                        row = erl[q];
                    }
                } else if (++idle > (a.spin << 4)) {
                    lds_put(&s_abort, 2);
                    it = items;
                }
            }
            if (__ballot(moved) == 0) {
                __builtin_amdgcn_s_sleep(1);
                if ((++rounds & 15u) == 0 && lds_get(&s_abort)) break;
            }
        }
    }
    __syncthreads();
    const unsigned long long t_done = TRACE ? __builtin_amdgcn_s_memrealtime() : 0ull;
    if (tid == 0 && s_abort == 2) {
        __hip_atomic_store(a.err_dev, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.err_host, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        s_abort = 1;
    }
    if (TRACE) {
        const int ntr = min(ns, a.trace_stride - 1);
        for (int t = tid; t < 2 * ntr; t += nt) a.trace[2 * (size_t)g * a.trace_stride + t] = ltr[t];
        if (tid == 0) {
            a.trace[2 * ((size_t)g * a.trace_stride + a.trace_stride - 1)] = t_fill;
            a.trace[2 * ((size_t)g * a.trace_stride + a.trace_stride - 1) + 1] = t_done;
        }
    }
    if (!s_abort) {
        for (int t = tid; t < win * R; t += nt) {
            const int q = t / R, k = t - q * R;
            const int x = lo + q;
            const T v = xl[t];
            if (a.write_xw) static_cast<T *>(a.xw)[(size_t)x * R + k] = v;
            if (a.xout) {
                const int d = a.scatter[x];  // negative: the row is not written (RAS overlap rows)
                if (d >= 0) {
                    const size_t dst = (size_t)d * R + k;
                    if (a.out_f64) static_cast<double *>(a.xout)[dst] = static_cast<double>(v);
                    else static_cast<float *>(a.xout)[dst] = static_cast<float>(v);
                }
            }
        }
    }
    __syncthreads();  // LDS is refilled by the next part
    if (s_abort) break;
    }  // parts
    if (tid == 0) {
        const unsigned done = __hip_atomic_fetch_add(&a.epoch[1], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {
            // last workgroup out: every claim is over; reset the queue
            __hip_atomic_store(&a.epoch[2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.epoch[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.epoch[0], s_epoch + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <typename T, bool UNIT, bool TAIL, bool R1, bool TRACE>
OwnerKernel dataflow_kernel_w(int w)
{
    switch (w) {
    case 1: return k_dataflow<T, 1, UNIT, TAIL, R1, TRACE>;
    case 2: return k_dataflow<T, 2, UNIT, TAIL, R1, TRACE>;
    case 3: return k_dataflow<T, 3, UNIT, TAIL, R1, TRACE>;
    case 4: return k_dataflow<T, 4, UNIT, TAIL, R1, TRACE>;
    case 5: return k_dataflow<T, 5, UNIT, TAIL, R1, TRACE>;
    case 6: return k_dataflow<T, 6, UNIT, TAIL, R1, TRACE>;
    case 7: return k_dataflow<T, 7, UNIT, TAIL, R1, TRACE>;
    case 8: return k_dataflow<T, 8, UNIT, TAIL, R1, TRACE>;
    case 10: return k_dataflow<T, 10, UNIT, TAIL, R1, TRACE>;
    case 12: return k_dataflow<T, 12, UNIT, TAIL, R1, TRACE>;
    case 16: return k_dataflow<T, 16, UNIT, TAIL, R1, TRACE>;
    default: return nullptr;
    }
}

template <typename T, bool R1, bool TRACE>
OwnerKernel dataflow_kernel_r(int w, bool unit, bool tail)
{
    if (unit)
        return tail ? dataflow_kernel_w<T, true, true, R1, TRACE>(w) : dataflow_kernel_w<T, true, false, R1, TRACE>(w);
    return tail ? dataflow_kernel_w<T, false, true, R1, TRACE>(w) : dataflow_kernel_w<T, false, false, R1, TRACE>(w);
}

template <typename T>
OwnerKernel dataflow_kernel(int w, bool unit, bool tail, int R, bool trace)
{
    if (trace)
        return R == 1 ? dataflow_kernel_r<T, true, true>(w, unit, tail) : dataflow_kernel_r<T, false, true>(w, unit, tail);
    return R == 1 ? dataflow_kernel_r<T, true, false>(w, unit, tail) : dataflow_kernel_r<T, false, false>(w, unit, tail);
}

template <typename T>
OwnerKernel split_kernel(int w, bool unit, size_t &lds, int rows, int CH)
{
    switch (w) {
#define HEC_SPLIT_CASE(WW)                                                                              \
    case WW:                                                                                            \
        lds = WsLayout<T, WW>(rows, CH, unit).total();                                                  \
        return unit ? k_owner_split<T, WW, true> : k_owner_split<T, WW, false>;
        HEC_SPLIT_CASE(1)
        HEC_SPLIT_CASE(2)
        HEC_SPLIT_CASE(3)
        HEC_SPLIT_CASE(4)
        HEC_SPLIT_CASE(5)
        HEC_SPLIT_CASE(6)
#undef HEC_SPLIT_CASE
    default: return nullptr;
    }
}

// Barrier-free solve of a level-ordered plan through global memory, for
// solutions too large for LDS (the alternative to one launch per level).  The
// (row, rhs) items in level order are cut into chunks of 64, dealt
// round-robin to the wavefronts of the grid.  A chunk depends only on earlier
// chunks, and the earliest unfinished chunk belongs to a wavefront that has
// finished all its earlier ones, so the solve progresses when every
// wavefront is resident: the kernel is launched cooperatively, so that the
// runtime either makes the whole grid co-resident or refuses the launch.
// (Taking chunks from one shared counter instead needs no co-residency, but
// the counter serializes: with batches of 8 chunks per claim, 288K claims on
// one address made an application of the batched 256-system workload 3.7x
// slower.)  xw starts as the sentinel; an item reads its inputs with
// agent-scope loads and, once none holds the sentinel, computes exactly as
// solve_item does and publishes its value with an agent-scope store.  Lanes
// whose inputs are ready finish inside the wait loop, so a wavefront never
// waits on one of its own lanes.
// MAXW > 0: rows of at most MAXW ELL slots keep their columns and values in
// registers, loaded once, and every poll issues all input loads together (one
// memory round trip per poll); MAXW = 0: any width, columns re-read per poll.
template <typename T, typename TIn, typename TOut, int MAXW>
__global__ void __launch_bounds__(256) k_syncfree(TriArgs a, int waves)
{
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const long items = (long)a.n * a.R;
    const long nch = (items + 63) >> 6;
    const T *ev = static_cast<const T *>(a.ell_val);
    T *xw = static_cast<T *>(a.xw);
    constexpr int NW = MAXW > 0 ? MAXW : 1;
    for (long ch = wave; ch < nch; ch += waves) {
        const long t = (ch << 6) + lane;
        bool todo = t < items;
        const int x = todo ? (int)(t / a.R) : 0;
        const int k = todo ? (int)(t - (long)x * a.R) : 0;
        // a finished problem's rows are skipped: they feed only that problem
        if (todo && a.act && !a.act[(a.seg ? a.seg[x] : 0) * a.R + k]) todo = false;
        T b = T(0);
        if (todo) {
            b = canon(static_cast<T>(static_cast<const TIn *>(a.bin)[(size_t)a.gather[x] * a.R + k]));
            if (a.dinv) b = scale_rhs(b, static_cast<const T *>(a.dinv)[x]);
        }
        int cr[NW];
        T vr[NW];
        if (MAXW > 0) {
#pragma unroll
            for (int e = 0; e < NW; ++e) {
                cr[e] = e < a.w ? a.ell_col[(size_t)e * a.ld + x] : a.n;
                vr[e] = e < a.w ? ev[(size_t)e * a.ld + x] : T(0);
            }
        }
        unsigned spins = 0;
        while (__ballot(todo)) {
            if (todo) {
                T s = b;
                bool ready = true;
                if (MAXW > 0) {
                    T dv[NW];
#pragma unroll
                    for (int e = 0; e < NW; ++e)
                        dv[e] = cr[e] != a.n ? __hip_atomic_load(xw + (size_t)cr[e] * a.R + k, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT)
                                             : T(0);
                    __builtin_amdgcn_sched_barrier(0);  // all loads out before the first test
#pragma unroll
                    for (int e = 0; e < NW; ++e)
                        if (cr[e] != a.n && is_sentinel(dv[e])) ready = false;
                    if (ready) {
#pragma unroll
                        for (int e = 0; e < NW; ++e)
                            if (cr[e] != a.n) s -= vr[e] * dv[e];
                    }
                } else {
                    for (int e = 0; e < a.w && ready; ++e) {
                        const int c = a.ell_col[(size_t)e * a.ld + x];
                        if (c != a.n) {
                            const T v = __hip_atomic_load(xw + (size_t)c * a.R + k, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                            if (is_sentinel(v)) ready = false;
                            else s -= ev[(size_t)e * a.ld + x] * v;
                        }
                    }
                }
                if (ready && a.tail_ptr) {
                    const T *tv = static_cast<const T *>(a.tail_val);
                    for (int p = a.tail_ptr[x]; p < a.tail_ptr[x + 1] && ready; ++p) {
                        const T v = __hip_atomic_load(xw + (size_t)a.tail_col[p] * a.R + k, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                        if (is_sentinel(v)) ready = false;
                        else s -= tv[p] * v;
                    }
                }
                if (ready) {
                    __hip_atomic_store(xw + (size_t)x * a.R + k, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (a.xout) {
                        const int d = a.scatter[x];
                        if (d >= 0) static_cast<TOut *>(a.xout)[(size_t)d * a.R + k] = static_cast<TOut>(s);
                    }
                    todo = false;
                }
            }
            if (__ballot(todo)) {
                __builtin_amdgcn_s_sleep(1);
                if ((++spins & 255u) == 0 &&
                    (spins > a.spin ||
                     __hip_atomic_load(a.err_dev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
                    __hip_atomic_store(a.err_dev, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(a.err_host, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    return;
                }
            }
        }
    }
}

// System queue: every workgroup takes whole independent systems from a
// counter (largest first) and solves one system's levels in order, all of a
// level's (row, rhs) items spread over the workgroup, with a workgroup
// barrier between levels.  The values of the system's last levels stay in an
// LDS ring (slot = local level mod slots); a dependency further back is read
// from the workspace, which this workgroup wrote before an earlier barrier.
// A system is never shared between workgroups, so the solve needs no
// co-residency.  Rows are computed exactly as in k_level (ELL slots in order,
// then the CSR tail; ELL padding reads a zero row of the ring and subtracts
// 0 * 0), so results are bit-identical to it.
template <typename T, typename TIn, typename TOut>
__global__ void __launch_bounds__(1024) k_sysq(TriArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_q;
    __shared__ unsigned s_epoch;
    T *ring = reinterpret_cast<T *>(smem);
    const int tid = threadIdx.x, nt = blockDim.x;
    const int R = a.R;
    const T *ev = static_cast<const T *>(a.ell_val);
    const T *tv = static_cast<const T *>(a.tail_val);
    T *xw = static_cast<T *>(a.xw);
    if (tid == 0) s_epoch = __hip_atomic_load(a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (tid == 0)
            s_q = (int)__hip_atomic_fetch_add(&a.epoch[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int q = s_q;
        if (q >= a.nparts) break;
        const int slots = a.sq_ring[2 * q], W = a.sq_ring[2 * q + 1];
        const int zrow = slots * W;
        for (int t = tid; t < R; t += nt) ring[(size_t)zrow * R + t] = T(0);
        __syncthreads();
        const int l0 = a.sq_lvp[q], l1 = a.sq_lvp[q + 1];
        for (int l = l0; l < l1; ++l) {
            const int rb = a.sq_lvrow[l], re = a.sq_lvrow[l + 1];
            const int base = slots ? ((l - l0) % slots) * W : 0;
            const int items = (re - rb) * R;
            for (int t = tid; t < items; t += nt) {
                const int i = t / R, k = t - i * R;
                const int x = rb + i;
                T sv = canon(static_cast<T>(static_cast<const TIn *>(a.bin)[(size_t)a.gather[x] * R + k]));
                if (a.dinv) sv = scale_rhs(sv, static_cast<const T *>(a.dinv)[x]);
                for (int e = 0; e < a.w; ++e) {
                    const int c = a.ell_col[(size_t)e * a.ld + x];
                    const T v = ev[(size_t)e * a.ld + x];
                    const T dep = c >= 0 ? ring[(size_t)min(c, zrow) * R + k]
                                         : __hip_atomic_load(xw + (size_t)(-2 - c) * R + k, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_WORKGROUP);
                    sv -= v * dep;
                }
                if (a.tail_ptr) {
                    for (int p = a.tail_ptr[x]; p < a.tail_ptr[x + 1]; ++p) {
                        const int c = a.tail_col[p];
                        const T dep = c >= 0 ? ring[(size_t)min(c, zrow) * R + k]
                                             : __hip_atomic_load(xw + (size_t)(-2 - c) * R + k, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
                        sv -= tv[p] * dep;
                    }
                }
                if (slots) ring[(size_t)(base + i) * R + k] = sv;
                if (a.write_xw)
                    __hip_atomic_store(xw + (size_t)x * R + k, sv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (a.xout) {
                    const int d = a.scatter[x];
                    if (d >= 0) static_cast<TOut *>(a.xout)[(size_t)d * R + k] = static_cast<TOut>(sv);
                }
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        const unsigned done = __hip_atomic_fetch_add(&a.epoch[1], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {
            // last workgroup out: every claim is over; reset the queue
            __hip_atomic_store(&a.epoch[2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.epoch[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.epoch[0], s_epoch + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// One item of the pipelined system queue: a row's G right-hand sides, with
// the row's data loaded P levels before its level is solved and its
// right-hand sides H levels before.
template <typename T, typename TIn, int G, int MW> struct SqItem {
    // integers, not bools: a bool becomes a lane mask as soon as it is
    // formed, which would wait for the load it comes from
    int ok;        // a real row of the level (else loads of a clamped row, unused)
    int keep;      // also stored to xw (read beyond a ring)
    int x, gi, dst;
    int c[MW];
    T v[MW];
    T d;
    TIn b[G];
};

// Row data of local row i of level lf (clamped into the system's levels and
// into the level, so that every load stays inside the plan's arrays).
template <typename T, typename TIn, int G, int MW>
__device__ __forceinline__ void sq_rows(const TriArgs &a, const int32_t *__restrict__ lvrow,
                                       SqItem<T, TIn, G, MW> &u, int lf, int l1, int i)
{
    const int lc = min(lf, l1 - 1);
    const int rb = lvrow[lc], re = lvrow[lc + 1];
    u.ok = lf < l1 && rb + i < re;
    const int x = max(0, min(rb + i, re - 1));
    u.x = x;
    u.gi = a.gather[x];
    const T *ev = static_cast<const T *>(a.ell_val);
#pragma unroll
    for (int e = 0; e < MW; ++e) {
        const size_t o = (size_t)min(e, a.w - 1) * a.ld + x;
        u.c[e] = a.ell_col[o];
        u.v[e] = ev[o];
    }
    // unconditional loads (from a stand-in array when there is no diagonal
    // or scatter), so that every set issues the same number of loads and
    // the compiler's memory counters wait only for the set being solved
    u.d = (a.dinv ? static_cast<const T *>(a.dinv) : ev)[x];
    u.dst = (a.xout ? a.scatter : a.gather)[x];
    u.keep = a.sq_keep[x];
}

template <typename T, typename TIn, int G, int MW>
__device__ __forceinline__ void sq_rhs(const TriArgs &a, SqItem<T, TIn, G, MW> &u, int g0)
{
    const TIn *src = static_cast<const TIn *>(a.bin) + (size_t)u.gi * a.R + g0;
#pragma unroll
    for (int g = 0; g < G; ++g) u.b[g] = src[g];
}

// The row's value for its G right-hand sides, computed as k_level does
// (right-hand side, scaled by the reciprocal diagonal if any, then the ELL
// slots in order; padding reads the ring's zero row, a dependency beyond the
// ring the workspace, which this workgroup wrote before an earlier barrier).
template <typename T, typename TIn, int G, int MW>
__device__ __forceinline__ void sq_solve(const TriArgs &a, const SqItem<T, TIn, G, MW> &u, T *ring, int zrow,
                                         int slots, int slotrow, int g0)
{
    if (!u.ok) return;
    const int R = a.R;
    T s[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        T sv = canon(static_cast<T>(u.b[g]));
        if (a.dinv) sv = scale_rhs(sv, u.d);
        s[g] = sv;
    }
    const int dst = a.xout ? u.dst : -1;
#pragma unroll
    for (int e = 0; e < MW; ++e) {
        if (e < a.w) {
            const int c = u.c[e];
            const T v = u.v[e];
            if (c >= 0) {
                const T *dp = ring + (size_t)min(c, zrow) * R + g0;
#pragma unroll
                for (int g = 0; g < G; ++g) s[g] -= v * dp[g];
            } else {
                const T *dp = static_cast<const T *>(a.xw) + (size_t)(-2 - c) * R + g0;
#pragma unroll
                for (int g = 0; g < G; ++g) s[g] -= v * dp[g];
            }
        }
    }
    if (slots) {
        T *o = ring + (size_t)slotrow * R + g0;
#pragma unroll
        for (int g = 0; g < G; ++g) o[g] = s[g];
    }
    if (a.write_xw || u.keep) {
        T *w = static_cast<T *>(a.xw) + (size_t)u.x * R + g0;
#pragma unroll
        for (int g = 0; g < G; ++g) w[g] = s[g];
    }
    if (dst >= 0) {  // the output type is a launch argument (one instance serves both)
        if (a.out_f64) {
            double *w = static_cast<double *>(a.xout) + (size_t)dst * R + g0;
#pragma unroll
            for (int g = 0; g < G; ++g) w[g] = static_cast<double>(s[g]);
        } else {
            float *w = static_cast<float *>(a.xout) + (size_t)dst * R + g0;
#pragma unroll
            for (int g = 0; g < G; ++g) w[g] = static_cast<float>(s[g]);
        }
    }
}

// System queue with software pipelining: the same work and results as
// k_sysq (workgroups take whole systems from a counter, a workgroup barrier
// between levels, the last levels' values in an LDS ring), but the
// wavefronts form k groups that take a system's levels in turn, and each
// thread owns M items of its group's levels (item t = thread in group +
// m * group size, G right-hand sides of one row), held in P register sets:
// a set's row data is loaded P turns (P * k levels) before its level is
// solved and its right-hand sides (whose address needs the row's gather
// index) H = P / 2 turns before, so that the barrier-separated levels do
// not wait on memory.  k is as large as the system's widest level allows.
// Items beyond M * group size of a wide level are solved directly.  Needs no
// CSR tail, ELL width 1..MW and R a multiple of G (checked by the host); rows
// read beyond a ring are also stored to xw.  The level tables come as
// separate restrict arguments, so that their uniform reads are scalar loads
// (a vector load waited for inside a level would also wait for every
// prefetch issued before it).
template <typename T, typename TIn, int G, int MW, int M, int P>
__global__ void __launch_bounds__(512) k_sysq_pipe(TriArgs a, const int32_t *__restrict__ lvp,
                                                   const int32_t *__restrict__ lvrow,
                                                   const int32_t *__restrict__ rings)
{
    constexpr int H = P / 2;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_q;
    __shared__ unsigned s_epoch;
    T *ring = reinterpret_cast<T *>(smem);
    const int tid = threadIdx.x, nt = blockDim.x;
    // the wavefront index as a uniform value: level numbers derived from it
    // stay scalar, so the level table reads remain scalar loads
    const int nw = nt >> 6, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int R = a.R, NG = R / G;
    SqItem<T, TIn, G, MW> S[P][M];
    if (tid == 0) s_epoch = __hip_atomic_load(a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (tid == 0)
            s_q = (int)__hip_atomic_fetch_add(&a.epoch[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int q = s_q;
        if (q >= a.nparts) break;
        const int slots = rings[2 * q], W = rings[2 * q + 1];
        const int zrow = slots * W;
        // optional clocks per system: start, end
        if (a.trace && tid == 0 && a.trace_stride > 0)
            a.trace[2 * (size_t)q * a.trace_stride] = __builtin_amdgcn_s_memrealtime();
        for (int t = tid; t < R; t += nt) ring[(size_t)zrow * R + t] = T(0);
        const int l0 = lvp[q], l1 = lvp[q + 1];
        // a Krylov solve's mask of unfinished (system, rhs) problems: a
        // system whose right-hand sides have all finished is skipped (its
        // rows feed only its own problems)
        if (a.act && l1 > l0) {
            const int sys = a.seg ? a.seg[lvrow[l0]] : 0;
            int live = 0;
            for (int k2 = 0; k2 < R; ++k2) live |= a.act[(size_t)sys * R + k2];
            if (!live) {
                __syncthreads();  // every thread has read s_q before it is reused
                continue;
            }
        }
        // wavefront groups: the system's widest level needs `need`
        // wavefronts (M items per thread); k = nw / wpg groups take the
        // levels in turn (group g solves levels l0 + g, l0 + g + k, ...), so
        // a wavefront's P register sets reach P * k levels ahead
        const int need = (W * NG + 64 * M - 1) / (64 * M);
        int wpg = 1;
        while (wpg < need && wpg < nw) wpg *= 2;
        const int k = nw / wpg, grp = wave / wpg, ng = wpg * 64, tl = tid - grp * ng;
        int im[M], gm[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int t = tl + m * ng;
            im[m] = t / NG;
            gm[m] = (t - im[m] * NG) * G;
        }
        if (l1 > l0) {
            // each set's right-hand sides right after its row data, so that
            // (as in the steady state) many loads follow them: the counter
            // wait before the first level then covers that set alone
#pragma unroll
            for (int p = 0; p < P; ++p) {
#pragma unroll
                for (int m = 0; m < M; ++m) sq_rows(a, lvrow, S[p][m], l0 + grp + p * k, l1, im[m]);
                if (p < H) {
#pragma unroll
                    for (int m = 0; m < M; ++m) sq_rhs(a, S[p][m], gm[m]);
                }
            }
        }
        __syncthreads();
        // one barrier per level, for every wavefront: the levels of the
        // other groups before and after this group's level of the round
        const int nr = (l1 - l0 + k - 1) / k;
        for (int r0 = 0; r0 < nr; r0 += P) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int r = r0 + p;
                if (r >= nr) break;
                const int nlr = min(k, l1 - l0 - r * k);  // levels in this round
                for (int g = 0; g < min(grp, nlr); ++g) __syncthreads();
                // this group's level (past the system's end in a short last
                // round: nothing is solved there, the loads are clamped)
                const int l = l0 + r * k + grp;
#pragma unroll
                for (int m = 0; m < M; ++m) sq_rhs(a, S[(p + H) % P][m], gm[m]);
                const int base = slots ? ((l - l0) % slots) * W : 0;
#pragma unroll
                for (int m = 0; m < M; ++m)
                    sq_solve<T, TIn, G, MW>(a, S[p][m], ring, zrow, slots, base + im[m], gm[m]);
                // items beyond the pipeline (two at a time per thread
                // measured slower: more registers)
                const int items = l < l1 ? (lvrow[l + 1] - lvrow[l]) * NG : 0;
                for (int t = tl + M * ng; t < items; t += ng) {
                    SqItem<T, TIn, G, MW> u;
                    const int i = t / NG;
                    sq_rows(a, lvrow, u, l, l1, i);
                    sq_rhs(a, u, (t - i * NG) * G);
                    sq_solve<T, TIn, G, MW>(a, u, ring, zrow, slots, base + i, (t - i * NG) * G);
                }
#pragma unroll
                for (int m = 0; m < M; ++m) sq_rows(a, lvrow, S[p][m], l + P * k, l1, im[m]);
                if (grp < nlr) __syncthreads();
                for (int g = grp + 1; g < nlr; ++g) __syncthreads();
            }
        }
        if (a.trace && tid == 0 && a.trace_stride > 0)
            a.trace[2 * (size_t)q * a.trace_stride + 1] = __builtin_amdgcn_s_memrealtime();
    }
    if (tid == 0) {
        const unsigned done = __hip_atomic_fetch_add(&a.epoch[1], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {
            // last workgroup out: every claim is over; reset the queue
            __hip_atomic_store(&a.epoch[2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.epoch[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.epoch[0], s_epoch + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_fill_sentinel(T *p, size_t count, unsigned *counter)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = sentinel<T>();
    if (counter && i == 0) *counter = 0u;  // the next launch's chunk counter
}

using SqKernel = void (*)(TriArgs, const int32_t *, const int32_t *, const int32_t *);

// Pipelined system-queue instance for ELL width w: one item per thread
// (wider levels solve their items beyond 512 directly), or, when at least a
// quarter of the levels hold more than 512 items, two items per thread; two
// register sets either way (four sets measured 7% slower on 256 batched
// systems: more loads in flight per wavefront; more items per thread spill
// registers).
template <typename T, typename TIn, int G, int MW>
SqKernel sysq_pipe_width(bool wide)
{
    if (!wide) return k_sysq_pipe<T, TIn, G, MW, 1, 2>;
    return k_sysq_pipe<T, TIn, G, MW, 2, 2>;
}

// Right-hand sides per thread: 4 (pairs of lanes share a row, so a
// wavefront's right-hand-side loads and result stores touch half as many
// scattered cache lines as with 8) when the median level then still fits one
// item per thread, else 8.
inline int sysq_group(int R, int median_rows)
{
    if (R % 4 == 0 && (R % 8 != 0 || (int64_t)median_rows * (R / 4) <= 512)) return 4;
    return 8;
}

template <typename T, typename TIn>
SqKernel sysq_pipe_kernel(int w, const std::vector<int32_t> &widths, int G, int R)
{
    const int groups = R / G;
    size_t wide = 0;
    for (const int32_t r : widths) wide += (size_t)r * groups > 512;
    const bool many = 4 * wide >= widths.size();
    if (G == 4) return w <= 4 ? sysq_pipe_width<T, TIn, 4, 4>(many) : sysq_pipe_width<T, TIn, 4, 8>(many);
    return w <= 4 ? sysq_pipe_width<T, TIn, 8, 4>(many) : sysq_pipe_width<T, TIn, 8, 8>(many);
}

template <typename T, typename TIn, typename TOut>
void launch_typed(DevTri &d, TriArgs a, hipStream_t st)
{
    if (d.n == 0) return;
    if (d.kind == HEC_SCHED_LEVEL_LAUNCH && d.variant == 5) {
        const size_t cnt = ((size_t)d.n + 1) * a.R;
        hipLaunchKernelGGL(k_fill_sentinel<T>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st,
                           static_cast<T *>(a.xw), cnt, (unsigned *)nullptr);
        // about one wavefront per chunk of an average level (at least two
        // workgroups per compute unit), within half the occupancy; the
        // cooperative launch guarantees co-residency (it costs tens of
        // microseconds, small beside this kernel's milliseconds)
        const long chunks = ((long)d.n * a.R + 63) / 64;
        // rows of at most 8 (or 16) ELL slots keep them in registers
        const void *kern = d.w <= 8 ? (const void *)k_syncfree<T, TIn, TOut, 8>
                         : (d.w <= 16 ? (const void *)k_syncfree<T, TIn, TOut, 16> : (const void *)k_syncfree<T, TIn, TOut, 0>);
        const int cap = capacity_of(kern, 256, 0);
        const long per_level = chunks / std::max(1, d.nlev);
        const long lim = std::min<long>(std::max(1, cap / 2), std::max<long>(2L * device_cus(), per_level / 4));
        const int grid = (int)std::max<long>(1, std::min<long>(lim, (chunks + 3) / 4));
        int waves = grid * 4;
        void *args[] = {(void *)&a, (void *)&waves};
        hip_check(hipLaunchCooperativeKernel(kern, dim3(grid), dim3(256), args, 0, st), "k_syncfree cooperative launch");
        return;
    }
    if (d.sysq) {
        const size_t lds = (size_t)std::max(1, d.sq_lds_rows) * a.R * sizeof(T);
        if (lds > (size_t)device_max_lds())
            fail(HEC_ERR_CAPACITY, "system queue: the LDS ring exceeds the device limit at this nrhs");
        a.nparts = d.groups;
        // no CSR tail, ELL width 1..8 and right-hand sides in groups of
        // 4 or 8: the pipelined kernel
        if (!d.has_tail && d.w >= 1 && d.w <= 8 && a.R % 4 == 0) {
            const SqKernel k =
                sysq_pipe_kernel<T, TIn>(d.w, d.sq_widths, sysq_group(a.R, d.sq_median_rows), a.R);
            const int32_t cap = capacity_of((const void *)k, 512, lds);
            const int grid = std::max(1, std::min(d.groups, cap));
            hipLaunchKernelGGL(k, dim3(grid), dim3(512), lds, st, a, a.sq_lvp, a.sq_lvrow, a.sq_ring);
            hip_check(hipGetLastError(), "k_sysq_pipe launch");
            return;
        }
        const int block = std::max(64, std::min(1024, d.block));
        const int32_t cap = capacity_of((const void *)k_sysq<T, TIn, TOut>, block, lds);
        a.nparts = d.groups;
        if (d.sq_global) a.write_xw = 1;  // dependencies beyond the ring are read back from xw
        const int grid = std::max(1, std::min(d.groups, cap));
        hipLaunchKernelGGL((k_sysq<T, TIn, TOut>), dim3(grid), dim3(block), lds, st, a);
        hip_check(hipGetLastError(), "k_sysq launch");
        return;
    }
    if (d.kind == HEC_SCHED_LEVEL_LAUNCH) {
        for (int32_t k = 0; k < d.nlev; ++k) {
            a.row_begin = d.levelptr[k];
            a.row_end = d.levelptr[k + 1];
            const int items = (a.row_end - a.row_begin) * a.R;
            const int grid = (items + 255) / 256;
            hipLaunchKernelGGL((k_level<T, TIn, TOut>), dim3(grid), dim3(256), 0, st, a);
        }
        hip_check(hipGetLastError(), "k_level launch");
        return;
    }
    if (d.dataflow) {
        // the plan's columns name group-local imports: only this kernel reads them
        OwnerKernel k = dataflow_kernel<T>(d.w, d.unit, d.has_tail, a.R, a.trace != nullptr);
        if (!k) fail(HEC_ERR_INVALID_ARG, "internal: dataflow plan with an unsupported ELL width");
        if ((int64_t)d.df_step_rows * a.R > 64)
            fail(HEC_ERR_INVALID_ARG, "dataflow plan: nrhs exceeds the plan's max_nrhs (steps are sized for it)");
        size_t lds = dataflow_lds_bytes(d.df_rows, d.df_ints, a.R, sizeof(T));
        if (a.trace) lds += 8 + 16 * (size_t)std::min(d.df_ints / 2, a.trace_stride);  // per-step clocks
        const int block = 64 * d.df_waves + 128;
        if (block > dataflow_max_block(d.w)) fail(HEC_ERR_INVALID_ARG, "dataflow kernel: block too large");
        if (lds > (size_t)device_max_lds())
            fail(HEC_ERR_CAPACITY, "dataflow kernel: LDS need exceeds the device limit at this nrhs");
        const int32_t cap = capacity_of((const void *)k, block, lds);
        a.nparts = d.groups;
        a.queue = d.queue ? 1 : 0;
        int32_t grid = d.groups;
        if (d.queue) {
            // parts wait only on lower-numbered parts, which running
            // workgroups hold: any grid size makes progress
            grid = std::max(1, std::min(d.groups, cap));
        } else if (cap < d.groups) {
            fail(HEC_ERR_CAPACITY, "dataflow grid exceeds the co-resident capacity");
        }
        hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds, st, a);
        hip_check(hipGetLastError(), "k_dataflow launch");
        return;
    }
    if (d.kind == HEC_SCHED_OWNER_PERSISTENT && d.variant == 3 && a.R == 1 && !d.has_tail && d.max_lanes_one &&
        d.w >= 1 && d.w <= 6 && d.chunk_rows > 0) {
        size_t lds = 0;
        OwnerKernel k = split_kernel<T>(d.w, d.unit, lds, d.max_window, d.chunk_rows);
        if (k && lds <= (size_t)device_max_lds() && capacity_of((const void *)k, 128, lds) >= d.groups) {
            hipLaunchKernelGGL(k, dim3(d.groups), dim3(128), lds, st, a);
            hip_check(hipGetLastError(), "k_owner_split launch");
            return;
        }
    }
    if (d.kind == HEC_SCHED_OWNER_PERSISTENT && (d.variant == 0 || d.variant >= 2) && !d.has_tail &&
        d.max_lanes_one && d.w >= 1 && d.w <= 8 && d.chunk_rows > 0 && d.chunk_rows % d.block == 0) {
        const int rpt = d.chunk_rows / d.block;
        OwnerKernel k = owner_kernel<T>(d.w, rpt, d.unit);
        const size_t lds = owner_lds_bytes(d.max_window, a.R, d.w, d.chunk_rows, d.unit, sizeof(T));
        if (k && lds <= (size_t)device_max_lds() && capacity_of((const void *)k, d.block, lds) >= d.groups) {
            hipLaunchKernelGGL(k, dim3(d.groups), dim3(d.block), lds, st, a);
            hip_check(hipGetLastError(), "k_owner launch");
            return;
        }
    }
    size_t lds = 0;
    bool use_lds = false;
    auto k_lds = k_persistent<T, TIn, TOut, true>;
    auto k_glb = k_persistent<T, TIn, TOut, false>;
    if (d.kind == HEC_SCHED_OWNER_PERSISTENT && d.max_window > 0) {
        lds = (size_t)d.max_window * a.R * sizeof(T);
        use_lds = lds <= (size_t)device_max_lds() && capacity_of((const void *)k_lds, d.block, lds) >= d.groups;
        if (!use_lds) lds = 0;
    }
    if (!use_lds && capacity_of((const void *)k_glb, d.block, 0) < d.groups)
        fail(HEC_ERR_CAPACITY, "persistent grid exceeds the co-resident capacity");
    if (use_lds)
        hipLaunchKernelGGL(k_lds, dim3(d.groups), dim3(d.block), lds, st, a);
    else
        hipLaunchKernelGGL(k_glb, dim3(d.groups), dim3(d.block), 0, st, a);
    hip_check(hipGetLastError(), "k_persistent launch");
}

template <typename T>
void launch_in(DevTri &d, const TriArgs &a, hec_dtype_t in_dt, hec_dtype_t out_dt, hipStream_t st)
{
    if (in_dt == HEC_F64) {
        if (out_dt == HEC_F64) launch_typed<T, double, double>(d, a, st);
        else launch_typed<T, double, float>(d, a, st);
    } else {
        if (out_dt == HEC_F64) launch_typed<T, float, double>(d, a, st);
        else launch_typed<T, float, float>(d, a, st);
    }
}

// Co-resident workgroups of one kernel instance on the current device
// (cached: the occupancy query and the LDS attribute are set once per
// kernel, block size, LDS size and device).
int32_t capacity_of(const void *kern, int32_t block, size_t lds)
{
    struct Key {
        const void *k;
        int32_t block;
        size_t lds;
        int dev;
        bool operator<(const Key &o) const
        {
            return std::tie(k, block, lds, dev) < std::tie(o.k, o.block, o.lds, o.dev);
        }
    };
    static std::mutex mu;
    static std::map<Key, int32_t> cache;
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    const Key key{kern, block, lds, dev};
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    int cus = 0, per = 0;
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "attr CUs");
    if (lds > 0)
        hip_check(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                  "hipFuncSetAttribute");
    hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, block, lds), "occupancy");
    std::lock_guard<std::mutex> g(mu);
    cache[key] = per * cus;
    return per * cus;
}

template <typename T, bool LDS>
int32_t capacity_all(int32_t block, size_t lds)
{
    int32_t c = capacity_of((const void *)k_persistent<T, double, double, LDS>, block, lds);
    c = std::min(c, capacity_of((const void *)k_persistent<T, double, float, LDS>, block, lds));
    c = std::min(c, capacity_of((const void *)k_persistent<T, float, double, LDS>, block, lds));
    c = std::min(c, capacity_of((const void *)k_persistent<T, float, float, LDS>, block, lds));
    return c;
}

}  // namespace

int32_t persistent_capacity(hec_dtype_t dt, int32_t block, size_t lds)
{
    if (dt == HEC_F64) return lds ? capacity_all<double, true>(block, lds) : capacity_all<double, false>(block, 0);
    return lds ? capacity_all<float, true>(block, lds) : capacity_all<float, false>(block, 0);
}

namespace {
int32_t device_attr(hipDeviceAttribute_t attr)
{
    static std::mutex mu;
    static std::map<std::pair<int, int>, int32_t> cache;
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> g(mu);
    auto key = std::make_pair(dev, (int)attr);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int v = 0;
    hip_check(hipDeviceGetAttribute(&v, attr, dev), "hipDeviceGetAttribute");
    cache[key] = v;
    return v;
}
}  // namespace

int32_t device_cus() { return device_attr(hipDeviceAttributeMultiprocessorCount); }

int32_t device_max_lds() { return device_attr(hipDeviceAttributeMaxSharedMemoryPerBlock); }

void fill_sentinel(void *p, size_t count, hec_dtype_t dt)
{
    if (count == 0) return;
    const unsigned grid = (unsigned)((count + 255) / 256);
    if (dt == HEC_F64)
        hipLaunchKernelGGL(k_fill_sentinel<double>, dim3(grid), dim3(256), 0, 0, static_cast<double *>(p), count,
                           nullptr);
    else
        hipLaunchKernelGGL(k_fill_sentinel<float>, dim3(grid), dim3(256), 0, 0, static_cast<float *>(p), count,
                           nullptr);
    hip_check(hipGetLastError(), "k_fill_sentinel launch");
    hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
}

void launch_tri(DevTri &d, const void *bin, hec_dtype_t in_dt, const int32_t *gather, void *xw, void *xout,
                hec_dtype_t out_dt, const int32_t *scatter, int32_t R, hipStream_t st)
{
    if (R > d.ws_R) fail(HEC_ERR_INVALID_ARG, "internal: workspace narrower than nrhs");
    TriArgs a{};
    a.n = d.n;
    a.w = d.w;
    a.ld = d.ld;
    a.R = R;
    a.ell_col = d.ell_col.as<int32_t>();
    a.ell_val = d.ell_val.p;
    a.tail_ptr = d.has_tail ? d.tail_ptr.as<int32_t>() : nullptr;
    a.tail_col = d.tail_col.as<int32_t>();
    a.tail_val = d.tail_val.p;
    a.dinv = d.unit ? nullptr : d.dinv.p;
    a.step_ptr = d.step_ptr.as<int32_t>();
    a.step_row = d.step_row.as<int32_t>();
    a.step_lanes = d.step_lanes.as<int32_t>();
    a.window = d.window.as<int32_t>();
    a.exp_slot = d.exp_slot.as<int32_t>();
    a.exp_ptr = d.exp_ptr.as<int32_t>();
    a.mbox = d.mbox.p;
    a.nexp = d.nexp;
    a.mbox_stride = d.ws_R;
    a.epoch = d.epoch.as<unsigned int>();
    a.err_dev = d.err.as<int>();
    a.err_host = d.err_host;
    a.bin = bin;
    a.gather = gather;
    a.xw = xw;
    a.xout = xout;
    a.scatter = scatter;
    a.write_xw = xout ? 0 : 1;
    a.chunk_ptr = d.chunk_ptr.as<int32_t>();
    a.rem_ptr = d.rem_ptr.as<int32_t>();
    a.rem_ent = d.rem_ent.as<int32_t>();
    a.chunk_step = d.chunk_step.as<int32_t>();
    a.chunk_rows = d.chunk_rows;
    a.imp_ptr = d.imp_ptr.as<int32_t>();
    a.imp_slot = d.imp_slot.as<int32_t>();
    a.exp_row = d.exp_row.as<int32_t>();
    a.wave_ptr = d.wave_ptr.as<int32_t>();
    a.act = d.act;
    a.seg = d.seg.p ? d.seg.as<int32_t>() : nullptr;
    a.trace = d.trace;
    a.trace_stride = d.trace_stride;
    a.spin = d.spin;
    a.sq_lvp = d.sq_lvp.as<int32_t>();
    a.sq_lvrow = d.sq_lvrow.as<int32_t>();
    a.sq_ring = d.sq_ring.as<int32_t>();
    a.sq_keep = d.sq_keep.as<int8_t>();
    a.in_f64 = in_dt == HEC_F64 ? 1 : 0;
    a.out_f64 = out_dt == HEC_F64 ? 1 : 0;
    if (d.dt == HEC_F64) launch_in<double>(d, a, in_dt, out_dt, st);
    else launch_in<float>(d, a, in_dt, out_dt, st);
}

}  // namespace hec
