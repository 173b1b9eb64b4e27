// Numeric ILU(0) / ILU(k) refactorization on the device (Section 3's
// incomplete factorizations, computed over the level sets of eq. (2)).
//
// The pattern of the combined factor F = L\U (sorted rows, diagonal present)
// is fixed at setup; new values of A are scattered into it (zero at fill
// positions) and eliminated row by row.  Row i needs the finished rows k < i
// with f_ik stored, which are exactly its dependencies in L, so the rows of
// one level of L are independent and each level is one launch.  Inside a row
// the pivots are taken in ascending order, l_ik = f_ik / u_kk and then
// f_ij -= l_ik u_kj for every j > k of row k that row i holds, with separate
// roundings (no fused multiply-add), so the factors equal the host
// factorization bit for bit.  The finished factors are then written into the
// two triangular plans in their execution layout: L's entries as they are,
// U's scaled by the reciprocal diagonal, which itself fills U's diagonal array.
#include <hip/hip_runtime.h>

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

void refactor_numeric(DevRefactor &r, const double *aval, hipStream_t st)
{
    if (r.fwork.bytes < r.fval.bytes) r.fwork.alloc(r.fval.bytes);
    double *f = r.fwork.as<double>();
    int *err = r.err.as<int>();
    if (r.nnz_f > 0)
        hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(r.nnz_f)), dim3(256), 0, st, f, (long)r.nnz_f);
    hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(64), 0, st, err);
    if (r.nnz_a > 0)
        hipLaunchKernelGGL(k_scatter_a, dim3(grid_for(r.nnz_a)), dim3(256), 0, st, aval, r.a2f.as<int32_t>(),
                           (long)r.nnz_a, f);
    const int32_t *rows = r.rows.as<int32_t>();
    for (size_t k = 0; k + 1 < r.levelptr.size(); ++k) {
        const int nr = r.levelptr[k + 1] - r.levelptr[k];
        if (nr == 0) continue;
        hipLaunchKernelGGL(k_ilu_row, dim3(nr), dim3(kRowThreads), ilu_row_lds(r.max_row), st, rows + r.levelptr[k],
                           nr, r.frp.as<int32_t>(), r.fci.as<int32_t>(), r.fdpos.as<int32_t>(), f, err, r.max_row);
    }
    hip_check(hipGetLastError(), "refactor launch");
    int flag = 0;
    hip_check(hipMemcpyAsync(&flag, err, sizeof(int), hipMemcpyDeviceToHost, st), "refactor flag copy");
    hip_check(hipStreamSynchronize(st), "refactor synchronize");
    if (flag) fail(HEC_ERR_ZERO_PIVOT, "zero or non-finite pivot in the device refactorization");
    std::swap(r.fval.p, r.fwork.p);
    std::swap(r.fval.bytes, r.fwork.bytes);
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
