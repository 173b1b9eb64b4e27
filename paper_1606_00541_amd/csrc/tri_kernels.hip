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
//                 list of steps (a contiguous range of device rows), waiting
//                 before a step on the progress counters of the workgroups
//                 that produce its inputs.  Under the owner schedule the
//                 workgroup's own solution values also live in LDS.
// The row routine subtracts the ELL terms in slot order, then the CSR-tail
// terms, then multiplies by the stored reciprocal diagonal, so both
// executions produce bit-identical results for rows run one thread per
// (row, rhs); steps tuned to split long rows over several lanes sum in a
// different order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "hec_dev.h"

namespace hec {

namespace {

constexpr unsigned kSpinLimit = 1u << 22;  // polls before a wait is declared hung

int32_t capacity_of(const void *kern, int32_t block, size_t lds);

// Solution values that other workgroups of a persistent launch may read are
// written and read as agent-scope relaxed atomics: the stores go through to
// the point of coherence shared by all XCDs and the loads do not hit stale
// cache lines, so no cache-wide writeback or invalidate is needed.  A
// producer waits for its stores to complete before it bumps its progress
// counter; a consumer reads the values only after it saw the counter.  The
// per-level launch (COH = false) relies on kernel boundaries instead.
template <typename T, bool COH>
__device__ __forceinline__ T gload(const T *p)
{
    if (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *p;
}

template <typename T, bool COH>
__device__ __forceinline__ void gstore(T *p, T v)
{
    if (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

template <typename T, bool LDS, bool COH>
__device__ __forceinline__ T load_x(const TriArgs &a, const T *xw, const T *xl, int lo, int hi, int c, int k)
{
    if (LDS && c >= lo && c < hi) return xl[(c - lo) * a.R + k];
    return gload<T, COH>(xw + (size_t)c * a.R + k);
}

// Partial sum of one row's off-diagonal terms (lane `lane` of `lanes`).
template <typename T, bool LDS, bool COH>
__device__ __forceinline__ T row_terms(const TriArgs &a, int x, int k, int lane, int lanes, const T *xl, int lo,
                                       int hi)
{
    const T *ev = static_cast<const T *>(a.ell_val);
    const T *xw = static_cast<const T *>(a.xw);
    T part = T(0);
    for (int e = lane; e < a.w; e += lanes) {
        const int c = a.ell_col[(size_t)e * a.ld + x];
        const T v = ev[(size_t)e * a.ld + x];
        if (c < a.n) part += v * load_x<T, LDS, COH>(a, xw, xl, lo, hi, c, k);
    }
    if (a.tail_ptr) {
        const T *tv = static_cast<const T *>(a.tail_val);
        for (int p = a.tail_ptr[x] + lane; p < a.tail_ptr[x + 1]; p += lanes)
            part += tv[p] * load_x<T, LDS, COH>(a, xw, xl, lo, hi, a.tail_col[p], k);
    }
    return part;
}

template <typename T, typename TOut, bool LDS, bool COH>
__device__ __forceinline__ void finish_row(const TriArgs &a, int x, int k, T s, T *xl, int lo, int hi)
{
    if (a.dinv) s *= static_cast<const T *>(a.dinv)[x];
    gstore<T, COH>(static_cast<T *>(a.xw) + (size_t)x * a.R + k, s);
    if (LDS && x >= lo && x < hi) xl[(x - lo) * a.R + k] = s;
    if (a.xout) {
        const int dst = a.scatter[x];
        if (dst >= 0) static_cast<TOut *>(a.xout)[(size_t)dst * a.R + k] = static_cast<TOut>(s);
    }
}

// Thread-per-(row, rhs) solve of one row: s = b - sum, in slot order.
template <typename T, typename TIn, typename TOut, bool LDS, bool COH>
__device__ __forceinline__ void solve_item(const TriArgs &a, int x, int k, T *xl, int lo, int hi)
{
    const T *ev = static_cast<const T *>(a.ell_val);
    const T *xw = static_cast<const T *>(a.xw);
    T s = static_cast<T>(static_cast<const TIn *>(a.bin)[(size_t)a.gather[x] * a.R + k]);
    for (int e = 0; e < a.w; ++e) {
        const int c = a.ell_col[(size_t)e * a.ld + x];
        const T v = ev[(size_t)e * a.ld + x];
        if (c < a.n) s -= v * load_x<T, LDS, COH>(a, xw, xl, lo, hi, c, k);
    }
    if (a.tail_ptr) {
        const T *tv = static_cast<const T *>(a.tail_val);
        for (int p = a.tail_ptr[x]; p < a.tail_ptr[x + 1]; ++p)
            s -= tv[p] * load_x<T, LDS, COH>(a, xw, xl, lo, hi, a.tail_col[p], k);
    }
    finish_row<T, TOut, LDS, COH>(a, x, k, s, xl, lo, hi);
}

// Rows [rb, re) x R right-hand sides, `lanes` lanes per (row, rhs).  With
// lanes > 1 the lanes of a group split the row's terms and combine them with
// a butterfly of cross-lane shuffles inside the wavefront.
template <typename T, typename TIn, typename TOut, bool LDS, bool COH>
__device__ __forceinline__ void solve_range(const TriArgs &a, int rb, int re, int lanes, T *xl, int lo, int hi)
{
    const int R = a.R;
    if (lanes == 1) {
        const int items = (re - rb) * R;
        for (int t = threadIdx.x; t < items; t += blockDim.x) {
            const int q = t / R;
            solve_item<T, TIn, TOut, LDS, COH>(a, rb + q, t - q * R, xl, lo, hi);
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
        T part = act ? row_terms<T, LDS, COH>(a, x, k, lane, lanes, xl, lo, hi) : T(0);
        for (int off = lanes >> 1; off > 0; off >>= 1) part += __shfl_xor(part, off, lanes);
        if (act && lane == 0) {
            T s = static_cast<T>(static_cast<const TIn *>(a.bin)[(size_t)a.gather[x] * R + k]) - part;
            finish_row<T, TOut, LDS, COH>(a, x, k, s, xl, lo, hi);
        }
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
    solve_item<T, TIn, TOut, false, false>(a, a.row_begin + q, t - q * a.R, nullptr, 0, 0);
}

// One launch for the whole solve (see the file comment).  The progress
// counter of workgroup g holds (epoch << 32) | completed steps; the epoch is
// read at kernel start and advanced by the last workgroup to finish, so the
// counters never need clearing between launches (also under graph replay).
template <typename T, typename TIn, typename TOut, bool LDS>
__global__ void __launch_bounds__(1024) k_persistent(TriArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    T *xl = reinterpret_cast<T *>(smem);
    __shared__ unsigned s_epoch;
    __shared__ int s_abort;
    const int g = blockIdx.x;
    if (threadIdx.x == 0) {
        s_epoch = __hip_atomic_load(a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_abort = 0;
    }
    __syncthreads();
    const unsigned long long base = (unsigned long long)s_epoch << 32;
    int lo = 0, hi = 0;
    if (LDS) {
        lo = a.window[2 * g];
        hi = a.window[2 * g + 1];
    }
    const int s0 = a.step_ptr[g], s1 = a.step_ptr[g + 1];
    for (int s = s0; s < s1; ++s) {
        const int wb = a.wait_ptr[s], we = a.wait_ptr[s + 1];
        if (we > wb) {
            for (int q = wb + (int)threadIdx.x; q < we; q += blockDim.x) {
                const int h = a.waits[2 * q];
                const unsigned long long need = base | (unsigned)a.waits[2 * q + 1];
                unsigned spins = 0;
                while (__hip_atomic_load(&a.progress[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    ++spins;
                    if ((spins & 255u) == 0 &&
                        (spins > kSpinLimit ||
                         __hip_atomic_load(a.err_dev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
                        __hip_atomic_store(a.err_dev, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(a.err_host, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                        s_abort = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __syncthreads();
            if (s_abort) break;
        }
        solve_range<T, TIn, TOut, LDS, true>(a, a.step_row[2 * s], a.step_row[2 * s + 1], a.step_lanes[s], xl, lo,
                                             hi);
        // every store of this step has completed before the counter moves
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(&a.progress[g], base | (unsigned)(s - s0 + 1), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
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

template <typename T, typename TIn, typename TOut>
void launch_typed(DevTri &d, TriArgs a, hipStream_t st)
{
    if (d.n == 0) return;
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
    a.use_lds = use_lds ? 1 : 0;
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

// Co-resident workgroups of one kernel instance on the current device.
int32_t capacity_of(const void *kern, int32_t block, size_t lds)
{
    int dev = 0, cus = 0, per = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "attr CUs");
    if (lds > 0)
        hip_check(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                  "hipFuncSetAttribute");
    hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, block, lds), "occupancy");
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

int32_t device_cus()
{
    int dev = 0, cus = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "attr CUs");
    return cus;
}

int32_t device_max_lds()
{
    int dev = 0, v = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    hip_check(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "attr LDS");
    return v;
}

void launch_tri(DevTri &d, const void *bin, hec_dtype_t in_dt, const int32_t *gather, void *xw, void *xout,
                hec_dtype_t out_dt, const int32_t *scatter, int32_t R, hipStream_t st)
{
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
    a.wait_ptr = d.wait_ptr.as<int32_t>();
    a.waits = d.waits.as<int32_t>();
    a.window = d.window.as<int32_t>();
    a.progress = d.progress.as<unsigned long long>();
    a.epoch = d.epoch.as<unsigned int>();
    a.err_dev = d.err.as<int>();
    a.err_host = d.err_host;
    a.bin = bin;
    a.gather = gather;
    a.xw = xw;
    a.xout = xout;
    a.scatter = scatter;
    if (d.dt == HEC_F64) launch_in<double>(d, a, in_dt, out_dt, st);
    else launch_in<float>(d, a, in_dt, out_dt, st);
}

}  // namespace hec
