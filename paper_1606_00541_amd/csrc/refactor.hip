// Numeric ILU(0) / ILU(k) refactorization on the device (Section 3's
// incomplete factorizations, computed over the level sets of eq. (2)).
//
// The pattern of the combined factor F = L\U (sorted rows, diagonal present)
// is fixed at setup; new values of A are scattered into it (zero at fill
// positions) and eliminated row by row.  Row i needs the finished rows k < i
// with f_ik stored, which are exactly its dependencies in L, so the rows of
// one level of L are independent.  Short rows are eliminated in one launch,
// a lane per row waiting on the rows it needs (k_ilu_flow); longer ones take
// one launch per level (k_ilu_row).  Inside a row
// the pivots are taken in ascending order, l_ik = f_ik / u_kk and then
// f_ij -= l_ik u_kj for every j > k of row k that row i holds, with separate
// roundings (no fused multiply-add), so the factors equal the host
// factorization bit for bit.  The finished factors are then written into the
// two triangular plans in their execution layout: L's entries as they are,
// U's scaled by the reciprocal diagonal, which itself fills U's diagonal array.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

#include "hec_dev.h"

namespace hec {

namespace {

constexpr int kRowThreads = 64;

__global__ void __launch_bounds__(256) k_zero_f64(double *p, long n)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0;
}

__global__ void __launch_bounds__(64) k_zero_flag(int *p)
{
    if (threadIdx.x == 0) p[0] = 0;
}

__global__ void __launch_bounds__(256) k_scatter_a(const double *aval, const int32_t *a2f, long nnz, double *f)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nnz) f[a2f[t]] = aval[t];
}

// LDS bytes of k_ilu_row for factor rows of at most `maxrow` entries.
size_t ilu_row_lds(int maxrow)
{
    const int np = maxrow < kRowThreads ? maxrow : kRowThreads;
    return (size_t)maxrow * sizeof(double) + (size_t)np * sizeof(double) + (size_t)maxrow * sizeof(int32_t) +
           2 * (size_t)np * sizeof(int32_t);
}

// One workgroup (one wavefront) per row of the level.  The row is staged in
// LDS (sized for the pattern's longest row, so that many rows are resident);
// lane-parallel over the entries of each pivot row.
__global__ void __launch_bounds__(kRowThreads) k_ilu_row(const int32_t *rows, int nrows, const int32_t *rp,
                                                         const int32_t *ci, const int32_t *dpos, double *f,
                                                         int *err, int maxrow)
{
    // the host factorization rounds the product and the difference separately
#pragma clang fp contract(off)
    extern __shared__ __align__(16) unsigned char smem[];
    const int np = maxrow < kRowThreads ? maxrow : kRowThreads;
    double *sval = reinterpret_cast<double *>(smem);
    // the first np pivot rows' pivot value, diagonal position and end,
    // fetched by one lane each before the elimination starts
    double *spiv = sval + maxrow;
    int32_t *scol = reinterpret_cast<int32_t *>(spiv + np);
    int32_t *spk = scol + maxrow;
    int32_t *spe = spk + np;
    const int q = blockIdx.x;
    if (q >= nrows) return;
    const int i = rows[q];
    const int b = rp[i], len = rp[i + 1] - b, di = dpos[i] - b;
    for (int t = threadIdx.x; t < len; t += kRowThreads) {
        scol[t] = ci[b + t];
        sval[t] = f[b + t];
    }
    if (threadIdx.x < di && threadIdx.x < np) {
        const int k = ci[b + threadIdx.x];
        const int pk = dpos[k];
        spk[threadIdx.x] = pk;
        spe[threadIdx.x] = rp[k + 1];
        spiv[threadIdx.x] = f[pk];
    }
    __syncthreads();
    for (int kk = 0; kk < di; ++kk) {
        const bool tab = kk < np;
        const int k = scol[kk];
        const int pk = tab ? spk[kk] : dpos[k];
        const double lik = sval[kk] / (tab ? spiv[kk] : f[pk]);
        __syncthreads();
        if (threadIdx.x == 0) sval[kk] = lik;
        const int pe = tab ? spe[kk] : rp[k + 1];
        for (int p = pk + 1 + threadIdx.x; p < pe; p += kRowThreads) {
            const int j = ci[p];
            // row i's entries after kk are sorted: binary search for column j
            int lo = kk + 1, hi = len;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (scol[mid] < j) lo = mid + 1;
                else hi = mid;
            }
            if (lo < len && scol[lo] == j) sval[lo] = sval[lo] - lik * f[p];
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < len; t += kRowThreads) f[b + t] = sval[t];
    if (threadIdx.x == 0) {
        const double d = sval[di];
        if (d == 0.0 || !isfinite(d)) err[0] = 1;
    }
}

// The elimination in one launch, one lane per row.  Rows in level order are
// cut into chunks of 64, dealt round-robin to the wavefronts of a
// cooperative launch (every wavefront is resident).  A lane copies its row
// of A (zero at fill positions) into LDS, reads the entries of its pivot
// rows it needs from the output, which starts as the sentinel and receives
// every row's final values, re-reading until none holds the sentinel (they
// come from earlier chunks, held by running wavefronts, so the solve always
// progresses), then eliminates in the host factorization's order with
// separate roundings and writes its row.  A copied entry whose bits equal the
// sentinel is written as the canonical quiet NaN, so no value can look
// unwritten.  err: 1 for a zero or non-finite pivot, 2 when a wait gave up
// after `spin` polls (every wavefront then stops).
__device__ __forceinline__ bool rf_unset(double v) { return __double_as_longlong(v) == (long long)kSentinel64; }

__global__ void __launch_bounds__(256) k_fill_unset(double *p, long n)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = __longlong_as_double((long long)kSentinel64);
}

template <int MAXR, int MAXS>
__global__ void __launch_bounds__(64) k_ilu_flow(const int32_t *rows, int n, const int32_t *rp, const int32_t *dpos,
                                                 const int32_t *sptr, const int32_t *spos, const int32_t *sdst,
                                                 const double *init, double *f, int *err, unsigned spin)
{
#pragma clang fp contract(off)
    __shared__ double buf[MAXR][64];
    const int lane = threadIdx.x;
    const long nch = ((long)n + 63) / 64;
    for (long ch = blockIdx.x; ch < nch; ch += gridDim.x) {
        const long t = ch * 64 + lane;
        const bool live = t < n;
        const int i = live ? rows[t] : 0;
        const int b = live ? rp[i] : 0, len = live ? rp[i + 1] - b : 0, d = live ? dpos[i] - b : 0;
        const int s0 = live ? sptr[i] : 0, ns = live ? sptr[i + 1] - s0 : 0;
        // loads are unconditional (indices clamped to valid entries, the
        // surplus masked afterwards) so that they issue back to back
        const int slast = s0 + (ns > 0 ? ns - 1 : 0), blast = b + (len > 0 ? len - 1 : 0);
        int pos[MAXS], dq[MAXS];
#pragma unroll
        for (int s = 0; s < MAXS; ++s) {
            pos[s] = spos[min(s0 + s, slast)];
            dq[s] = sdst[min(s0 + s, slast)];
        }
        double iv[MAXR];
#pragma unroll
        for (int q = 0; q < MAXR; ++q) iv[q] = init[min(b + q, blast)];
#pragma unroll
        for (int q = 0; q < MAXR; ++q)
            if (q < len) buf[q][lane] = rf_unset(iv[q]) ? __builtin_nan("") : iv[q];
        double v[MAXS];
        unsigned long long need = ns >= 64 ? ~0ull : ((1ull << ns) - 1ull);
        bool todo = live;
        unsigned spins = 0;
        // a lane finishes its row inside the loop as soon as its own inputs
        // are there, so a wavefront never waits on one of its own lanes (a
        // chunk can hold the end of one level and the start of the next)
        while (__ballot(todo) != 0) {
            if (todo) {
                // every pending load is issued before any is tested, so a poll
                // costs one memory round trip however many entries it reads
                double x[MAXS];
#pragma unroll
                for (int s = 0; s < MAXS; ++s)
                    x[s] = ((need >> s) & 1ull)
                               ? __hip_atomic_load(f + pos[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                               : 0.0;
                __builtin_amdgcn_sched_barrier(0);  // all loads out before the first test
#pragma unroll
                for (int s = 0; s < MAXS; ++s)
                    if (((need >> s) & 1ull) && !rf_unset(x[s])) {
                        v[s] = x[s];
                        need &= ~(1ull << s);
                    }
                if (need == 0ull) {
                    int piv = -1;
                    double lik = 0.0;
#pragma unroll
                    for (int s = 0; s < MAXS; ++s)
                        if (s < ns) {
                            if (dq[s] < 0) {
                                ++piv;
                                lik = buf[piv][lane] / v[s];
                                buf[piv][lane] = lik;
                            } else {
                                buf[dq[s]][lane] = buf[dq[s]][lane] - lik * v[s];
                            }
                        }
#pragma unroll
                    for (int q = 0; q < MAXR; ++q)
                        if (q < len)
                            __hip_atomic_store(f + b + q, buf[q][lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const double dd = buf[d][lane];
                    if (dd == 0.0 || !isfinite(dd)) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    todo = false;
                }
            }
            if (__ballot(todo) != 0) {
                // uncached polls from every waiting lane load the memory
                // system that the rows being waited for store through
                __builtin_amdgcn_s_sleep(1);
                if ((++spins & 255u) == 0) {
                    if (spins > spin) __hip_atomic_store(err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 2) return;
                }
            }
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_refill_l(const double *f, const int32_t *src, const int32_t *dst, long cnt,
                                                  T *ell, T *tail)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const T v = (T)f[src[t]];
    const int32_t d = dst[t];
    if (d >= 0) ell[d] = v;
    else tail[-1 - d] = v;
}

template <typename T>
__global__ void __launch_bounds__(256) k_refill_u(const double *f, const int32_t *src, const int32_t *dst,
                                                  const int32_t *diag, long cnt, T *ell, T *tail)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const double dinv = 1.0 / f[diag[t]];
    const T v = (T)(f[src[t]] * dinv);
    const int32_t d = dst[t];
    if (d >= 0) ell[d] = v;
    else tail[-1 - d] = v;
}

template <typename T>
__global__ void __launch_bounds__(256) k_refill_dinv(const double *f, const int32_t *src, int n, T *dinv)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) dinv[t] = (T)(1.0 / f[src[t]]);
}

__global__ void __launch_bounds__(256) k_gather_f64(const double *src, const int32_t *idx, long cnt, double *dst)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < cnt) dst[t] = src[idx[t]];
}

int grid_for(long cnt) { return (int)((cnt + 255) / 256); }

template <typename T>
void refill_typed(const DevRefactor &r, DevTri &L, DevTri &U, hipStream_t st)
{
    const double *f = r.fval.as<double>();
    if (r.nl > 0)
        hipLaunchKernelGGL(k_refill_l<T>, dim3(grid_for(r.nl)), dim3(256), 0, st, f, r.l_src.as<int32_t>(),
                           r.l_dst.as<int32_t>(), (long)r.nl, L.ell_val.as<T>(), L.tail_val.as<T>());
    if (r.nu > 0)
        hipLaunchKernelGGL(k_refill_u<T>, dim3(grid_for(r.nu)), dim3(256), 0, st, f, r.u_src.as<int32_t>(),
                           r.u_dst.as<int32_t>(), r.u_diag.as<int32_t>(), (long)r.nu, U.ell_val.as<T>(),
                           U.tail_val.as<T>());
    if (r.n > 0)
        hipLaunchKernelGGL(k_refill_dinv<T>, dim3(grid_for(r.n)), dim3(256), 0, st, f, r.d_src.as<int32_t>(), r.n,
                           U.dinv.as<T>());
}

}  // namespace

template <int MAXR, int MAXS>
void launch_flow(DevRefactor &r, const double *init, double *f, int *err, hipStream_t st)
{
    const void *kern = (const void *)k_ilu_flow<MAXR, MAXS>;
    int per_cu = 0;
    hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, 0), "occupancy query");
    // about two levels' worth of chunks in flight (waves further ahead only
    // poll, and their uncached polls slow the stores being waited for), at
    // least one wavefront per compute unit, at most half the co-resident
    // wavefronts (the cooperative launch refuses more than can be resident),
    // and no more than there are chunks.  128^3 ILU(0): 256 wavefronts
    // 1.92 ms, 512 2.24 ms, 1024 2.71 ms, 128 2.38 ms.
    const long chunks = ((long)r.n + 63) / 64;
    const long nlev = std::max<long>(1, (long)r.levelptr.size() - 1);
    const long want = std::max<long>((long)device_cus(), 2 * ((chunks + nlev - 1) / nlev));
    const int grid = (int)std::max<long>(1, std::min<long>({chunks, want, (long)std::max(1, per_cu * device_cus() / 2)}));
    const int32_t *rows = r.rows.as<int32_t>(), *rp = r.frp.as<int32_t>(), *dpos = r.fdpos.as<int32_t>();
    const int32_t *sp = r.sptr.as<int32_t>(), *so = r.spos.as<int32_t>(), *sd = r.sdst.as<int32_t>();
    int n = r.n;
    unsigned spin = kDefaultSpin;
    void *args[] = {(void *)&rows, (void *)&n, (void *)&rp, (void *)&dpos, (void *)&sp, (void *)&so, (void *)&sd,
                    (void *)&init, (void *)&f, (void *)&err, (void *)&spin};
    hip_check(hipLaunchCooperativeKernel(kern, dim3(grid), dim3(64), args, 0, st), "refactor cooperative launch");
}

void refactor_numeric(DevRefactor &r, const double *aval, hipStream_t st)
{
    if (r.fwork.bytes < r.fval.bytes) r.fwork.alloc(r.fval.bytes);
    const bool flow = r.flow_row > 0 && r.n > 0;
    if (flow && r.fflow.bytes < r.fval.bytes) r.fflow.alloc(r.fval.bytes);
    double *f = r.fwork.as<double>();
    int *err = r.err.as<int>();
    if (r.nnz_f > 0)
        hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(r.nnz_f)), dim3(256), 0, st, f, (long)r.nnz_f);
    hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(64), 0, st, err);
    if (r.nnz_a > 0)
        hipLaunchKernelGGL(k_scatter_a, dim3(grid_for(r.nnz_a)), dim3(256), 0, st, aval, r.a2f.as<int32_t>(),
                           (long)r.nnz_a, f);
    DevMem *out = &r.fwork;
    if (flow) {
        // one launch: rows read the finished rows they need from fflow
        double *g = r.fflow.as<double>();
        if (r.nnz_f > 0)
            hipLaunchKernelGGL(k_fill_unset, dim3(grid_for(r.nnz_f)), dim3(256), 0, st, g, (long)r.nnz_f);
        if (r.flow_row == 8) launch_flow<8, 16>(r, f, g, err, st);
        else launch_flow<16, 32>(r, f, g, err, st);
        out = &r.fflow;
    } else {
        const int32_t *rows = r.rows.as<int32_t>();
        for (size_t k = 0; k + 1 < r.levelptr.size(); ++k) {
            const int nr = r.levelptr[k + 1] - r.levelptr[k];
            if (nr == 0) continue;
            hipLaunchKernelGGL(k_ilu_row, dim3(nr), dim3(kRowThreads), ilu_row_lds(r.max_row), st,
                               rows + r.levelptr[k], nr, r.frp.as<int32_t>(), r.fci.as<int32_t>(),
                               r.fdpos.as<int32_t>(), f, err, r.max_row);
        }
    }
    hip_check(hipGetLastError(), "refactor launch");
    int flag = 0;
    hip_check(hipMemcpyAsync(&flag, err, sizeof(int), hipMemcpyDeviceToHost, st), "refactor flag copy");
    hip_check(hipStreamSynchronize(st), "refactor synchronize");
    if (flag == 2) fail(HEC_ERR_TIMEOUT, "the device refactorization gave up waiting for a pivot row");
    if (flag) fail(HEC_ERR_ZERO_PIVOT, "zero or non-finite pivot in the device refactorization");
    std::swap(r.fval.p, out->p);
    std::swap(r.fval.bytes, out->bytes);
}

void gather_f64(const double *src, const int32_t *idx, int64_t cnt, double *dst, hipStream_t st)
{
    if (cnt <= 0) return;
    hipLaunchKernelGGL(k_gather_f64, dim3(grid_for(cnt)), dim3(256), 0, st, src, idx, (long)cnt, dst);
    hip_check(hipGetLastError(), "gather launch");
}

void refactor_refill(const DevRefactor &r, DevTri &L, DevTri &U, hipStream_t st)
{
    if (L.dt == HEC_F64) refill_typed<double>(r, L, U, st);
    else refill_typed<float>(r, L, U, st);
    hip_check(hipGetLastError(), "refill launch");
}

}  // namespace hec
