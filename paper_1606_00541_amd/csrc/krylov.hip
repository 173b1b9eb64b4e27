// Outer Krylov loop of the preconditioned solve (Section 4 uses restarted
// GMRES): general HEC matrices for the residual b - A x, deterministic
// multi-RHS inner products, vector updates, restarted (F)GMRES(m) with
// classical Gram-Schmidt with one re-orthogonalization (delayed by one step,
// two passes over the basis per step), and BiCGSTAB.  All
// vectors are FP64 [n][R] on the device; only the small per-RHS scalars
// (Hessenberg columns, inner products) travel to the host.  The autotuner for
// the triangular plans lives here as well.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "hec_dev.h"

struct hec_matrix_s {
    hec::DevHec d;
};
struct tri_plan_s;
struct ilu_s;
struct ras_s;

namespace hec {

namespace {

constexpr int kMaxPairs = 32;
constexpr int kMaxTerms = 4;

// ---- kernels -------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(256) k_spmv(int n, int w, int ld, const int32_t *ell_col, const T *ell_val,
                                                const int32_t *tail_ptr, const int32_t *tail_col,
                                                const T *tail_val, const double *x, const double *b,
                                                double *y, int R)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)n * R) return;
    const int i = (int)(t / R), k = (int)(t - (long)i * R);
    double s = 0.0;
    // the matrix streams through non-temporally: inside a Krylov solve the
    // preconditioner's factors are the data worth keeping in the caches
    for (int e = 0; e < w; ++e) {
        const int c = __builtin_nontemporal_load(ell_col + (size_t)e * ld + i);
        if (c < n) s += (double)__builtin_nontemporal_load(ell_val + (size_t)e * ld + i) * x[(size_t)c * R + k];
    }
    if (tail_ptr)
        for (int p = tail_ptr[i]; p < tail_ptr[i + 1]; ++p) s += (double)tail_val[p] * x[(size_t)tail_col[p] * R + k];
    y[t] = b ? b[t] - s : s;
}

struct DotArgs {
    const double *a[kMaxPairs];
    const double *b[kMaxPairs];
    int np;
};

// Column of vector element t of an [n][R] vector: the right-hand side k, or
// for a batch of independent systems (seg = system of each row) the problem
// (system, k) numbered system-major.
__device__ __forceinline__ int col_of(long t, int R, const int32_t *seg)
{
    const long row = t / R;
    const int k = (int)(t - row * R);
    return seg ? seg[row] * R + k : k;
}

// partial[blk][pair][k] = sum over the block's rows [brow[2 blk], brow[2 blk + 1])
// of a_pair * b_pair (a block never spans two systems).  Threads of a block
// are arranged as (rows x R): thread t owns rhs t % R.  When every pair shares
// its second vector (Gram-Schmidt: V_i . w) that vector is read once per row.
__global__ void __launch_bounds__(256) k_dot_partial(DotArgs d, int R, int rows_per_iter, const int32_t *brow,
                                                     const int32_t *bsys, const int8_t *act, double *partial)
{
    __shared__ double red[256];
    __shared__ int s_live;
    const int tid = threadIdx.x;
    const int used = rows_per_iter * R;
    const int k = tid % R, r0 = tid / R;
    long row0 = brow[2 * blockIdx.x], row1 = brow[2 * blockIdx.x + 1];
    if (act) {
        // a block whose system has no active problem contributes zeros
        if (tid == 0) {
            int live = 0;
            for (int q = 0; q < R; ++q) live |= act[bsys[blockIdx.x] * R + q];
            s_live = live;
        }
        __syncthreads();
        if (!s_live) row1 = row0;
    }
    bool same_b = true;
    for (int p = 1; p < d.np; ++p) same_b = same_b && d.b[p] == d.b[0];
    double acc[kMaxPairs];
#pragma unroll
    for (int p = 0; p < kMaxPairs; ++p) acc[p] = 0.0;
    if (tid < used) {
        if (same_b) {
            for (long row = row0 + r0; row < row1; row += rows_per_iter) {
                const double bv = d.b[0][row * R + k];
#pragma unroll
                for (int p = 0; p < kMaxPairs; ++p)
                    if (p < d.np) acc[p] += d.a[p][row * R + k] * bv;
            }
        } else {
#pragma unroll
            for (int p = 0; p < kMaxPairs; ++p)
                if (p < d.np)
                    for (long row = row0 + r0; row < row1; row += rows_per_iter)
                        acc[p] += d.a[p][row * R + k] * d.b[p][row * R + k];
        }
    }
#pragma unroll
    for (int p = 0; p < kMaxPairs; ++p) {
        if (p < d.np) {  // uniform across the block
            red[tid] = acc[p];
            __syncthreads();
            // fold the rows dimension: threads with the same k
            for (int span = rows_per_iter; span > 1;) {
                const int half = (span + 1) / 2;
                if (tid < used && r0 < span - half) red[tid] += red[tid + half * R];
                __syncthreads();
                span = half;
            }
            if (tid < R) partial[((size_t)blockIdx.x * d.np + p) * R + tid] = red[tid];
            __syncthreads();
        }
    }
}

// out[p][col] = sum of the partials of the blocks of col's system: one
// workgroup per (pair, column); thread i adds blocks i, i+256, ... in order,
// then a fixed tree folds the 256 sums (deterministic).
__global__ void __launch_bounds__(256) k_dot_final(const double *partial, const int32_t *bptr, int np, int R, int P,
                                                   double *out)
{
    __shared__ double red[256];
    const int t = blockIdx.x;  // p * P + col
    const int p = t / P, col = t - p * P, sys = col / R, k = col - sys * R;
    double s = 0.0;
    for (int b = bptr[sys] + (int)threadIdx.x; b < bptr[sys + 1]; b += 256)
        s += partial[((size_t)b * np + p) * R + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int half = 128; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) red[threadIdx.x] += red[threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[t] = red[0];
}

struct LinArgs {
    const double *in[kMaxTerms];
    int nt;
    const double *coef;  // [nt][P]
    double *out;
    double *out2;        // optional second output receiving the same value
};

// out[:,c] = sum_t coef[t][c] * in_t[:,c]; terms with a zero coefficient are
// left out, so a stopped problem's stale vectors (possibly NaN) never reach
// its output
__global__ void __launch_bounds__(256) k_lincomb(LinArgs a, long total, int R, int P, const int32_t *seg)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int c = col_of(t, R, seg);
    double s = 0.0;
    for (int q = 0; q < a.nt; ++q) {
        const double cf = a.coef[q * P + c];
        if (cf != 0.0) s += cf * a.in[q][t];
    }
    a.out[t] = s;
    if (a.out2) a.out2[t] = s;
}

// w[:,c] -= sum_{i<nv} h[i][c] * V_i[:,c]   (V_i = V + i*stride); problems
// that are no longer active (act[c] == 0) are left untouched
__global__ void __launch_bounds__(256) k_gs_update(double *w, const double *V, long stride, const double *h, int nv,
                                                  long total, int R, int P, const int32_t *seg, const int8_t *act)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int c = col_of(t, R, seg);
    if (act && !act[c]) return;
    double s = w[t];
    for (int i = 0; i < nv; ++i) s -= h[i * P + c] * V[i * stride + t];
    w[t] = s;
}

// x[:,c] += sum_{i<kd[c]} y[i][c] * Z_i[:,c]: each problem sums only the
// basis vectors it built in this cycle (the others hold whatever an earlier
// use of the memory left there, possibly a NaN pattern)
__global__ void __launch_bounds__(256) k_basis_update(double *x, const double *Z, long stride, const double *y,
                                                     const int32_t *kd, long total, int R, int P, const int32_t *seg)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int c = col_of(t, R, seg);
    const int nv = kd[c];
    if (nv == 0) return;
    double s = 0.0;
    for (int i = 0; i < nv; ++i) s += y[i * P + c] * Z[i * stride + t];
    x[t] += s;
}

// Largest RHS count of the delayed-re-orthogonalization kernels (R a power
// of two up to it); other counts take the two-pass classical path.
constexpr int kGsMaxR = 16;

// ---- Gram-Schmidt with delayed re-orthogonalization -----------------------
// Arnoldi step j holds the final orthonormal q_0..q_{j-1} in V slots 0..j-1
// and in slot j a candidate c_j: the previous Krylov vector projected once
// against the basis and scaled to about unit length, not yet final.  The
// step applies the preconditioner to the candidate itself (z_j = M^{-1} c_j,
// w = A z_j), then one pass of inner products gives s = Q^T c_j, t = Q^T w,
// c_j.c_j, c_j.w and w.w.  From them alpha = ||c_j - Q s|| makes
// q_j = (c_j - Q s)/alpha (the second projection of c_j), and w is
// projected once against [Q, q_j]: c_{j+1} = (w - Q t - tau q_j)/beta with
// tau = q_j.w = (c_j.w - s.t)/alpha and beta its length, both written in a
// second pass.  Since w = Q t + tau q_j + beta c_{j+1} and c_{j+1} =
// alpha' q_{j+1} + [Q, q_j] s' one step later, the Hessenberg column j is
// [t; tau] + beta [s'; alpha'], finished at step j+1 (z_j, as stored, is
// exactly the vector with A z_j = w, so x += Z y needs no correction).  Two
// passes over the basis per step instead of three; the last column of a
// cycle takes one more inner-product pass without a new vector.

// s_i = Q_i . c and t_i = Q_i . w (i < nq), then c.c, c.w and w.w (w set), or
// s_i and c.c (w null), per block into partial[blk][np][R]: slot i for s_i,
// nq + i for t_i, then 2nq, 2nq+1, 2nq+2 (np = 2nq + 3); without w slot nq
// holds c.c (np = nq + 1).  Blocks as in k_dot_partial; R a power of two up
// to kGsMaxR.  Wavefront q of the block's WV takes the basis vectors q,
// q+WV, ... over all of the block's rows (each basis element is read once) and
// every wavefront reads c and w; each product is summed by one wavefront only,
// so no cross-wavefront step is needed (deterministic).  A thread loads U rows
// before it computes on them.
template <int U, bool R1, int WV>
__global__ void __launch_bounds__(WV * 64) k_dcgs_dots(const double *Q, long stride, int nq, const double *cv,
                                                      const double *w, int R_, int P, const int32_t *brow,
                                                      const int32_t *bsys, const int8_t *act, double *partial)
{
    constexpr int NQ = 16 / U;  // basis vectors per wavefront
    const int R = R1 ? 1 : R_;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int k = lane & (R - 1), r0 = lane / R, rpw = 64 / R;
    const int c = bsys[blockIdx.x] * R + k;
    const long row0 = brow[2 * blockIdx.x], row1 = brow[2 * blockIdx.x + 1];
    const bool live = act == nullptr || act[c];
    const bool hw = w != nullptr;
    const int mine = nq > wave ? (nq - wave + WV - 1) / WV : 0;
    double as[NQ], at[NQ], s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) as[q] = at[q] = 0.0;
    if (live) {
        for (long row = row0 + r0; row < row1; row += (long)rpw * U) {
            double vq[U][NQ], cu[U], wu[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                long ru = row + (long)u * rpw;
                ru = ru < row1 ? ru : row;  // past the block's rows: load a valid row, skip it below
                const long t = ru * R + k;
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    if (q < mine) vq[u][q] = __builtin_nontemporal_load(Q + (wave + WV * q) * stride + t);
                cu[u] = cv[t];
                wu[u] = hw ? w[t] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (row + (long)u * rpw >= row1) break;
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    if (q < mine) {
                        as[q] += vq[u][q] * cu[u];
                        at[q] += vq[u][q] * wu[u];
                    }
                if (wave == 0) s0 += cu[u] * cu[u];
                if (wave == 1 % WV) s1 += cu[u] * wu[u];
                if (wave == 2 % WV) s2 += wu[u] * wu[u];
            }
        }
    }
    const int np = hw ? 2 * nq + 3 : nq + 1;
    double *out = partial + (size_t)blockIdx.x * np * R;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (q < mine) {  // uniform across the wavefront
            double a = as[q], b = at[q];
            for (int off = R; off < 64; off <<= 1) {
                a += __shfl_xor(a, off);
                b += __shfl_xor(b, off);
            }
            if (lane < R) {
                out[(wave + WV * q) * R + lane] = a;
                if (hw) out[(nq + wave + WV * q) * R + lane] = b;
            }
        }
    }
    // c.c, c.w and w.w, each summed by one wavefront (wave j takes product
    // j mod WV)
    const int base = hw ? 2 * nq : nq;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (j > 0 && !hw) break;
        if (wave != j % WV) continue;
        double v = j == 0 ? s0 : (j == 1 ? s1 : s2);
        for (int off = R; off < 64; off <<= 1) v += __shfl_xor(v, off);
        if (lane < R) out[(base + j) * R + lane] = v;
    }
}

// The second pass of a step, one element per thread: q = (c - sum_{i<nq}
// s_i Q_i) / alpha written over c, and the next candidate c' = (w -
// sum_{i<nq} t_i Q_i - tau q) / beta.  s and t come from the step's inner
// products (red[i][P], red[nq+i][P]), alpha, tau and beta from k_dcgs_step
// (sc[0..2][P]).  Problems that are no longer active are left as they are.
// With one problem (UNI) every coefficient is uniform and read once per
// wavefront.
template <bool UNI>
__global__ void __launch_bounds__(256) k_dcgs_update(const double *__restrict__ Q, long stride, int nq,
                                                    double *__restrict__ cv, const double *__restrict__ w,
                                                    double *__restrict__ cnext, const double *__restrict__ red,
                                                    const double *__restrict__ sc, long total, int R, int P,
                                                    const int32_t *seg, const int8_t *act)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int c = UNI ? 0 : col_of(t, R, seg);
    if (act && !act[c]) return;
    double ss = 0.0, tt = 0.0;
#pragma unroll 8
    for (int i = 0; i < nq; ++i) {
        const double qv = __builtin_nontemporal_load(Q + i * stride + t);
        ss += red[i * P + c] * qv;
        tt += red[(nq + i) * P + c] * qv;
    }
    const double q = (cv[t] - ss) / sc[c];
    cv[t] = q;
    __builtin_nontemporal_store((w[t] - tt - sc[P + c] * q) / sc[2 * P + c], cnext + t);
}

// The small work of step j for each problem still active, one wavefront per
// problem.  For j >= 1 it first finishes Hessenberg column j-1 from the
// previous step's [t; tau] and beta (tprev, sc[2][P]) and this step's s and
// alpha = sqrt(c.c - s.s): the earlier Givens rotations, a new one, the
// rotated right-hand side g and the stopping test |g_j| / ||b|| <= rtol (a
// zero or non-finite column stops the problem with BREAKDOWN).  Unless the
// problem stops or this is the cycle's closing pass (fin), it then sets
// alpha, tau and beta for k_dcgs_update and keeps [t; tau] for the next
// step.  H holds the rotated upper triangle, column l at H[(l*m + i)*P + c].
__global__ void __launch_bounds__(64) k_dcgs_step(int j, int m, int P, int fin, const double *red, double *tprev,
                                                  double *sc, double *H, double *cs, double *sn, double *g,
                                                  const double *bnorm, double rtol, int maxit, int8_t *act,
                                                  int32_t *kdim, int32_t *iters, int32_t *applies, int32_t *status,
                                                  int32_t *flag)
{
    __shared__ double sh[kMaxPairs + 1];
    __shared__ int s_stop;
    const int c = blockIdx.x, lane = threadIdx.x;
    if (!act[c]) return;  // uniform across the wavefront
    const int nq = j;
    const double s = lane < nq ? red[lane * P + c] : 0.0;
    const double t = (!fin && lane < nq) ? red[(nq + lane) * P + c] : 0.0;
    const double tp = lane < nq ? tprev[lane * P + c] : 0.0;
    double ss = s * s, tt = t * t, st = s * t;
    for (int off = 32; off > 0; off >>= 1) {
        ss += __shfl_xor(ss, off);
        tt += __shfl_xor(tt, off);
        st += __shfl_xor(st, off);
    }
    const double cc = red[(fin ? nq : 2 * nq) * P + c];
    const double bprev = sc[2 * P + c];
    double alpha = 1.0;
    if (lane == 0) {
        s_stop = 0;
        if (!fin) applies[c] += 1;  // M was applied to this step's candidate
    }
    if (j >= 1) {
        alpha = sqrt(fmax(0.0, cc - ss));
        if (lane < nq) sh[lane] = tp + bprev * s;
        __syncthreads();
        if (lane == 0) {
            const int col = j - 1;
            const double hn = bprev * alpha;
            double h = sh[0];  // h_i after the rotations before i
            for (int i = 0; i < col; ++i) {
                const double nx = sh[i + 1], ci = cs[i * P + c], si = sn[i * P + c];
                H[((size_t)col * m + i) * P + c] = ci * h + si * nx;
                h = -si * h + ci * nx;
            }
            const int it = iters[c] + 1;
            iters[c] = it;
            const double den = hypot(h, hn);
            if (!(den > 0.0) || !isfinite(den)) {
                status[c] = HEC_ERR_BREAKDOWN;
                act[c] = 0;
                s_stop = 1;
            } else {
                const double cj = h / den, sj = hn / den;
                cs[col * P + c] = cj;
                sn[col * P + c] = sj;
                H[((size_t)col * m + col) * P + c] = den;
                const double gj = g[col * P + c];
                g[(col + 1) * P + c] = -sj * gj;
                g[col * P + c] = cj * gj;
                kdim[c] = col + 1;
                if (fin || fabs(g[(col + 1) * P + c]) / bnorm[c] <= rtol || hn == 0.0 || it >= maxit) {
                    act[c] = 0;
                    s_stop = 1;
                }
            }
        }
        __syncthreads();
        if (s_stop) return;
    }
    if (fin) return;
    const double cw = red[(2 * nq + 1) * P + c], ww = red[(2 * nq + 2) * P + c];
    const double tau = (cw - st) / alpha;
    const double est = ww - tt - tau * tau;
    const double beta = est > 0.0 ? sqrt(est) : (ww > 0.0 ? sqrt(ww) : 1.0);
    if (lane < nq) tprev[lane * P + c] = t;
    if (lane == 0) {
        tprev[nq * P + c] = tau;
        if (!isfinite(tau) || !isfinite(beta)) {
            status[c] = HEC_ERR_BREAKDOWN;
            act[c] = 0;
            return;
        }
        sc[c] = alpha;
        sc[P + c] = tau;
        sc[2 * P + c] = beta;
        atomicOr(flag + j, 1);
    }
}

// v[:,c] = w[:,c] / ||w[:,c]|| for active problems (norm^2 in d[c]), else 0
__global__ void __launch_bounds__(256) k_normalize(double *v, const double *w, const double *d, const int8_t *act,
                                                  long total, int R, const int32_t *seg)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int c = col_of(t, R, seg);
    const double hn = sqrt(fmax(0.0, d[c]));
    // a stopped problem gets exact zeros, whatever its w holds
    v[t] = (act[c] && hn > 0.0) ? (1.0 / hn) * w[t] : 0.0;
}

template <typename TS, typename TD>
__global__ void __launch_bounds__(256) k_convert(const TS *s, TD *d, long count)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) d[t] = (TD)s[t];
}

__global__ void __launch_bounds__(256) k_fill_i32(int32_t *p, long count, int32_t v)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) p[t] = v;
}

// One Arnoldi step's small work, one wavefront per problem c still active:
// the new Hessenberg column h_{0..j+1, j} (the two Gram-Schmidt passes'
// coefficients summed, and ||w||), the earlier Givens rotations applied to
// it, a new rotation annihilating h_{j+1,j}, the rotated right-hand side g,
// and the stopping test |g_{j+1}| / ||b|| <= rtol.  The lanes fetch the
// column and the rotations together; lane 0 applies the rotations in order.
// A zero or non-finite column stops the problem with BREAKDOWN and leaves
// its basis at j vectors.  H holds the rotated upper triangle, column j at
// H[(j*m + i)*P + c].
__global__ void __launch_bounds__(64) k_arnoldi(int j, int m, int P, const double *d1, const double *d2,
                                                const double *dn, double *H, double *cs, double *sn, double *g,
                                                const double *bnorm, double rtol, int maxit, int8_t *act,
                                                int32_t *kdim, int32_t *iters, int32_t *status, int32_t *flag)
{
    __shared__ double sh[kMaxPairs + 1], scs[kMaxPairs], ssn[kMaxPairs];
    const int c = blockIdx.x, lane = threadIdx.x;
    if (!act[c]) return;  // uniform across the wavefront
    if (lane <= j) sh[lane] = d1[lane * P + c] + d2[lane * P + c];
    if (lane < j) {
        scs[lane] = cs[lane * P + c];
        ssn[lane] = sn[lane * P + c];
    }
    __syncthreads();
    if (lane != 0) return;
    const double hn = sqrt(fmax(0.0, dn[c]));
    double t = sh[0];  // h_i after the rotations before i
    for (int i = 0; i < j; ++i) {
        const double nx = sh[i + 1], ci = scs[i], si = ssn[i];
        H[((size_t)j * m + i) * P + c] = ci * t + si * nx;
        t = -si * t + ci * nx;
    }
    const int it = iters[c] + 1;
    iters[c] = it;
    const double den = hypot(t, hn);
    if (!(den > 0.0) || !isfinite(den)) {
        status[c] = HEC_ERR_BREAKDOWN;
        act[c] = 0;
        return;
    }
    const double cj = t / den, sj = hn / den;
    cs[j * P + c] = cj;
    sn[j * P + c] = sj;
    H[((size_t)j * m + j) * P + c] = den;
    const double gj = g[j * P + c];
    g[(j + 1) * P + c] = -sj * gj;
    g[j * P + c] = cj * gj;
    kdim[c] = j + 1;
    if (fabs(g[(j + 1) * P + c]) / bnorm[c] <= rtol || hn == 0.0 || it >= maxit) act[c] = 0;
    else atomicOr(flag + j, 1);
}

// y = R^{-1} g per problem over its kdim[c] columns (back substitution on the
// rotated Hessenberg triangle), one wavefront per problem: the triangle is
// staged in LDS, lane i holds g_i and finally y_i, and each solved y_i is
// subtracted from the lanes above it (column order).  Counts a completed
// cycle for every problem that extended its basis.
__global__ void __launch_bounds__(64) k_hess_solve(int m, int P, const double *H, const double *g,
                                                   const int32_t *kdim, double *y, int32_t *restarts)
{
    __shared__ double T[kMaxPairs][kMaxPairs];  // T[l][i] = H_{i,l}
    const int c = blockIdx.x, lane = threadIdx.x;
    const int kk = kdim[c];
    if (kk == 0) return;  // uniform across the wavefront
#pragma unroll 4
    for (int e = lane; e < kk * kk; e += 64) {
        const int l = e / kk, i = e - l * kk;
        if (i <= l) T[l][i] = H[((size_t)l * m + i) * P + c];
    }
    double s = lane < kk ? g[lane * P + c] : 0.0;
    __syncthreads();
    for (int i = kk - 1; i >= 0; --i) {
        const double yi = __shfl(s, i) / T[i][i];
        if (lane == i) s = yi;
        else if (lane < i) s -= T[i][lane] * yi;
    }
    if (lane < kk) y[lane * P + c] = s;
    if (lane == 0) restarts[c] += 1;
}

inline int blocks_for(long total) { return (int)std::max<long>(1, (total + 255) / 256); }

}  // namespace

// ---- public support functions -------------------------------------------

void spmv(const DevHec &A, const double *x, double *y, int32_t R, hipStream_t st)
{
    residual(A, nullptr, x, y, R, st);
}

void residual(const DevHec &A, const double *b, const double *x, double *r, int32_t R, hipStream_t st)
{
    const long total = (long)A.n * R;
    if (total == 0) return;
    const int32_t *tp = A.tail_nnz > 0 ? A.tail_ptr.as<int32_t>() : nullptr;
    if (A.dt == HEC_F64)
        hipLaunchKernelGGL(k_spmv<double>, dim3(blocks_for(total)), dim3(256), 0, st, A.n, A.w, A.ld,
                           A.ell_col.as<int32_t>(), A.ell_val.as<double>(), tp, A.tail_col.as<int32_t>(),
                           A.tail_val.as<double>(), x, b, r, R);
    else
        hipLaunchKernelGGL(k_spmv<float>, dim3(blocks_for(total)), dim3(256), 0, st, A.n, A.w, A.ld,
                           A.ell_col.as<int32_t>(), A.ell_val.as<float>(), tp, A.tail_col.as<int32_t>(),
                           A.tail_val.as<float>(), x, b, r, R);
    hip_check(hipGetLastError(), "k_spmv launch");
}

void convert_vec(const void *src, hec_dtype_t sdt, void *dst, hec_dtype_t ddt, size_t count, hipStream_t st)
{
    if (count == 0) return;
    const int g = blocks_for((long)count);
    if (sdt == HEC_F64 && ddt == HEC_F32)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(g), dim3(256), 0, st, (const double *)src, (float *)dst,
                           (long)count);
    else if (sdt == HEC_F32 && ddt == HEC_F64)
        hipLaunchKernelGGL((k_convert<float, double>), dim3(g), dim3(256), 0, st, (const float *)src, (double *)dst,
                           (long)count);
    else
        hip_check(hipMemcpyAsync(dst, src, count * (sdt == HEC_F64 ? 8 : 4), hipMemcpyDeviceToDevice, st),
                  "hipMemcpyAsync");
    hip_check(hipGetLastError(), "k_convert launch");
}

namespace {

// Scratch and helpers of one Krylov solve.  The vectors are [n][R]; the
// solve runs P independent problems: the R right-hand sides, or for a batch
// of nsys independent diagonal blocks (rows sys_ptr[s]..sys_ptr[s+1]-1) the
// nsys x R pairs (system, rhs), numbered system-major.  Inner products are
// taken per problem, in a fixed block order (deterministic).
struct Ctx {
    hipStream_t st;
    long n;
    int R, P;
    DevMem partial, dots, coef, segm, browm, bptrm, bsysm;
    DevMem d1m, d2m, dnm, actm;     // device-resident Gram-Schmidt coefficients and active mask
    DevMem kdm;                     // basis length of each problem in the current cycle
    int8_t *hact = nullptr;         // pinned staging of the active mask
    const int32_t *seg = nullptr;  // row -> system (batches only)
    double *hbuf = nullptr;        // pinned host scalars
    int nblk, rows_per_iter;
    bool dcgs_ok;  // R is a power of two up to kGsMaxR: the delayed re-orthogonalization applies
    Ctx(long n_, int R_, hipStream_t s, int nsys = 1, const int32_t *sys_ptr = nullptr) : st(s), n(n_), R(R_)
    {
        P = nsys * R;
        dcgs_ok = R >= 1 && R <= kGsMaxR && (R & (R - 1)) == 0;
        rows_per_iter = std::max(1, 256 / R);
        // reduction blocks: each covers rows of one system only
        const long chunk = std::max<long>((long)rows_per_iter * 4, (n + 1023) / 1024);
        std::vector<int32_t> brow, bptr(1, 0), bsys;
        for (int sy = 0; sy < nsys; ++sy) {
            const long r0 = sys_ptr ? sys_ptr[sy] : 0, r1 = sys_ptr ? sys_ptr[sy + 1] : n;
            for (long r = r0; r < r1; r += chunk) {
                brow.push_back((int32_t)r);
                brow.push_back((int32_t)std::min(r1, r + chunk));
                bsys.push_back(sy);
            }
            bptr.push_back((int32_t)(brow.size() / 2));
        }
        if (brow.empty()) {
            brow = {0, 0};
            bsys = {0};
        }
        nblk = (int)(brow.size() / 2);
        upload(browm, brow);
        upload(bptrm, bptr);
        upload(bsysm, bsys);
        if (nsys > 1) {
            std::vector<int32_t> sg((size_t)n);
            for (int sy = 0; sy < nsys; ++sy)
                for (int32_t i = sys_ptr[sy]; i < sys_ptr[sy + 1]; ++i) sg[i] = sy;
            upload(segm, sg);
            seg = segm.as<int32_t>();
        }
        partial.alloc(sizeof(double) * (size_t)nblk * (2 * kMaxPairs + 4) * R);
        dots.alloc(sizeof(double) * kMaxPairs * P);
        coef.alloc(sizeof(double) * (size_t)std::max(kMaxPairs, kMaxTerms) * P);
        hip_check(hipHostMalloc((void **)&hbuf, sizeof(double) * (size_t)std::max(kMaxPairs, kMaxTerms) * P, 0),
                  "hipHostMalloc");
        d1m.alloc(sizeof(double) * kMaxPairs * P);
        d2m.alloc(sizeof(double) * kMaxPairs * P);
        dnm.alloc(sizeof(double) * P);
        actm.alloc((size_t)P);
        kdm.alloc(sizeof(int32_t) * (size_t)P);
        hip_check(hipHostMalloc((void **)&hact, (size_t)P, 0), "hipHostMalloc");
    }
    ~Ctx()
    {
        if (hbuf) (void)hipHostFree(hbuf);
        if (hact) (void)hipHostFree(hact);
    }
    // inner products of np pairs, per problem, into out[p*P + c] on the device
    void dots_dev(const double *const *a, const double *const *b, int np, double *out, const int8_t *act = nullptr)
    {
        DotArgs d{};
        for (int p = 0; p < np; ++p) {
            d.a[p] = a[p];
            d.b[p] = b[p];
        }
        d.np = np;
        hipLaunchKernelGGL(k_dot_partial, dim3(nblk), dim3(256), 0, st, d, R, rows_per_iter, browm.as<int32_t>(),
                           bsysm.as<int32_t>(), act, partial.as<double>());
        hipLaunchKernelGGL(k_dot_final, dim3(np * P), dim3(256), 0, st, partial.as<double>(), bptrm.as<int32_t>(),
                           np, R, P, out);
        hip_check(hipGetLastError(), "dot launch");
    }
    // the inner products of one delayed-re-orthogonalization step
    // (k_dcgs_dots), finished per problem into out[p*P + c]
    void dcgs_dots(const double *Q, long stride, int nq, const double *cv, const double *w, double *out,
                   const int8_t *act)
    {
        const int np = w ? 2 * nq + 3 : nq + 1;
        const dim3 g(nblk), b(256);
        const int32_t *br = browm.as<int32_t>(), *bs = bsysm.as<int32_t>();
        double *pt = partial.as<double>();
        // two wavefronts per workgroup, each over half the basis (both read
        // the candidate and the new vector; four wavefronts measured 1.6%
        // slower for the whole solve)
#define HEC_DCGS_DOTS(U, R1)                                                                                   \
    hipLaunchKernelGGL((k_dcgs_dots<U, R1, 2>), g, dim3(128), 0, st, Q, stride, nq, cv, w, R, P, br, bs, act, pt)
        if (R == 1) {
            if (nq <= 8) HEC_DCGS_DOTS(4, true);
            else if (nq <= 16) HEC_DCGS_DOTS(2, true);
            else HEC_DCGS_DOTS(1, true);
        } else {
            if (nq <= 8) HEC_DCGS_DOTS(4, false);
            else if (nq <= 16) HEC_DCGS_DOTS(2, false);
            else HEC_DCGS_DOTS(1, false);
        }
#undef HEC_DCGS_DOTS
        hipLaunchKernelGGL(k_dot_final, dim3(np * P), dim3(256), 0, st, pt, bptrm.as<int32_t>(), np, R, P, out);
        hip_check(hipGetLastError(), "k_dcgs_dots launch");
    }
    // stream-ordered upload of the active mask; the host rewrites the staging
    // area only after the next synchronization, when the copy has landed
    void upload_active(const std::vector<char> &active)
    {
        for (int q = 0; q < P; ++q) hact[q] = active[q] ? 1 : 0;
        hip_check(hipMemcpyAsync(actm.p, hact, (size_t)P, hipMemcpyHostToDevice, st), "H2D");
    }
    // inner products of np pairs, per problem, returned in hbuf[p*P + c]
    void dots_to_host(const double *const *a, const double *const *b, int np)
    {
        DotArgs d{};
        for (int p = 0; p < np; ++p) {
            d.a[p] = a[p];
            d.b[p] = b[p];
        }
        d.np = np;
        hipLaunchKernelGGL(k_dot_partial, dim3(nblk), dim3(256), 0, st, d, R, rows_per_iter, browm.as<int32_t>(),
                           bsysm.as<int32_t>(), (const int8_t *)nullptr, partial.as<double>());
        hipLaunchKernelGGL(k_dot_final, dim3(np * P), dim3(256), 0, st, partial.as<double>(), bptrm.as<int32_t>(),
                           np, R, P, dots.as<double>());
        hip_check(hipGetLastError(), "dot launch");
        hip_check(hipMemcpyAsync(hbuf, dots.p, sizeof(double) * np * P, hipMemcpyDeviceToHost, st), "D2H");
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    }
    // out = sum_t c[t][col] in_t   (coefficients given on the host, [nt][P])
    void lincomb(double *out, const std::vector<const double *> &in, const std::vector<double> &c,
                 double *out2 = nullptr)
    {
        LinArgs a{};
        a.nt = (int)in.size();
        for (int t = 0; t < a.nt; ++t) a.in[t] = in[t];
        a.out = out;
        a.out2 = out2;
        upload_coef(c);
        a.coef = coef.as<double>();
        const long total = n * R;
        if (total == 0) return;
        hipLaunchKernelGGL(k_lincomb, dim3(blocks_for(total)), dim3(256), 0, st, a, total, R, P, seg);
        hip_check(hipGetLastError(), "k_lincomb launch");
    }
    void upload_coef(const std::vector<double> &c)
    {
        // stream-ordered copy through a pinned staging area; wait for it to
        // land so that the staging area can be reused
        std::memcpy(hbuf, c.data(), sizeof(double) * c.size());
        hip_check(hipMemcpyAsync(coef.p, hbuf, sizeof(double) * c.size(), hipMemcpyHostToDevice, st), "H2D");
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    }
};

}  // namespace

}  // namespace hec

// Preconditioner application hooks defined in capi.hip.
namespace hec {
// act: device mask of the (system, rhs) problems still being solved (or
// null); a kernel may skip the others, whose output is then left stale.
void precond_apply(const hec_precond_t &M, const double *r, double *z, int32_t R, hipStream_t st,
                   const int8_t *act = nullptr);
void precond_check(const hec_precond_t &M, int32_t n);
// Throws HEC_ERR_TIMEOUT if an application of M aborted a device-side wait
// (the stream must have been synchronized).
void precond_check_error(const hec_precond_t &M);
}  // namespace hec

using namespace hec;

namespace {

void apply_M(const hec_precond_t &M, const double *r, double *z, int R, long n, hipStream_t st,
             const int8_t *act = nullptr)
{
    if (M.kind == HEC_PRECOND_NONE) {
        if (z != r) hip_check(hipMemcpyAsync(z, r, sizeof(double) * n * R, hipMemcpyDeviceToDevice, st), "copy");
        return;
    }
    precond_apply(M, r, z, R, st, act);
}

// Final outcome of every problem from its true residual norm^2 rr2[k]: a
// finite relative residual at most rtol is a success (also after a lucky
// breakdown); otherwise a problem keeps the BREAKDOWN it stopped with (a
// non-finite b, a zero or non-finite scalar) or is NOT_CONVERGED.  A NaN
// never compares as converged.  The call returns the first BREAKDOWN, else
// the first NOT_CONVERGED, else OK.
hec_status_t final_status(hec_krylov_info_t *info, const std::vector<double> &bnorm, const double *rr2, int P,
                          double rtol, hec_status_t hint)
{
    hec_status_t out = HEC_OK;
    for (int k = 0; k < P; ++k) {
        const double rn = std::sqrt(rr2[k]);
        info[k].relres = !std::isfinite(bnorm[k]) ? std::nan("") : (bnorm[k] > 0 ? rn / bnorm[k] : rn);
        if (info[k].relres <= rtol) {
            info[k].status = HEC_OK;
            continue;
        }
        if (info[k].status == HEC_OK)
            info[k].status = hint == HEC_ERR_BREAKDOWN ? HEC_ERR_BREAKDOWN : HEC_ERR_NOT_CONVERGED;
        if (out == HEC_OK || (out == HEC_ERR_NOT_CONVERGED && info[k].status != HEC_ERR_NOT_CONVERGED))
            out = (hec_status_t)info[k].status;
    }
    return out;
}

// Restarted (F)GMRES(m): right preconditioning with the preconditioned basis
// Z stored (flexible form), CGS with one re-orthogonalization: delayed by
// one step (k_dcgs_*: two passes over the basis per step) when R is a power
// of two up to kGsMaxR, else two classical passes per step.  Every
// problem runs its own Arnoldi process in lockstep with the others; the
// Hessenberg columns, Givens rotations, rotated residual and each problem's
// stopping test live on the device (k_dcgs_step, k_arnoldi), so the host does not wait
// for a step to finish before issuing the next: it keeps two steps in
// flight and reads back one "any problem still active" flag per step, then
// synchronizes once per restart cycle for the true residual.  A problem whose
// rotated residual reaches rtol stops extending its basis.
hec_status_t gmres(const DevHec &A, const hec_precond_t &M, int m, const double *b, double *x, int R, double rtol,
                   int maxit, hec_krylov_info_t *info, hipStream_t st, int nsys, const int32_t *sys_ptr)
{
    const long n = A.n;
    const long nR = n * R;
    Ctx c(n, R, st, nsys, sys_ptr);
    const int P = c.P;
    DevMem Vm, Zm, wm, rm, Hm, csm, snm, gm, bnm, cnt, flg, redm, tpm, scm;
    Vm.alloc(sizeof(double) * (size_t)(m + 1) * nR);
    const bool dcgs = c.dcgs_ok;
    if (dcgs) {
        redm.alloc(sizeof(double) * (size_t)(2 * m + 3) * P);  // one step's inner products
        tpm.alloc(sizeof(double) * (size_t)(m + 1) * P);       // [t; tau] of the previous step
        scm.alloc(sizeof(double) * 3 * (size_t)P);             // alpha, tau, beta
    }
    Zm.alloc(sizeof(double) * (size_t)m * nR);
    wm.alloc(sizeof(double) * (size_t)nR);
    rm.alloc(sizeof(double) * (size_t)nR);
    Hm.alloc(sizeof(double) * (size_t)m * m * P);     // upper triangle of the rotated H, [j][i][P]
    csm.alloc(sizeof(double) * (size_t)m * P);
    snm.alloc(sizeof(double) * (size_t)m * P);
    gm.alloc(sizeof(double) * (size_t)(m + 1) * P);
    bnm.alloc(sizeof(double) * (size_t)P);
    cnt.alloc(sizeof(int32_t) * 4 * (size_t)P);        // iters, restarts, status, spare
    flg.alloc(sizeof(int32_t) * (size_t)m);            // per step: some problem still active
    double *V = Vm.as<double>(), *Z = Zm.as<double>(), *w = wm.as<double>(), *r = rm.as<double>();
    int32_t *d_iters = cnt.as<int32_t>(), *d_rest = d_iters + P, *d_stat = d_iters + 2 * P;
    auto Vi = [&](int i) { return V + (size_t)i * nR; };
    auto Zi = [&](int i) { return Z + (size_t)i * nR; };
    int32_t *hflag = nullptr;
    hip_check(hipHostMalloc((void **)&hflag, sizeof(int32_t) * (size_t)m, 0), "hipHostMalloc");
    std::unique_ptr<int32_t, void (*)(int32_t *)> hflag_own(hflag, [](int32_t *q) { (void)hipHostFree(q); });
    std::vector<hipEvent_t> ev(m, nullptr);
    for (auto &e : ev) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    struct EvFree {
        std::vector<hipEvent_t> *v;
        ~EvFree()
        {
            for (auto e : *v)
                if (e) (void)hipEventDestroy(e);
        }
    } ev_free{&ev};

    std::vector<double> bnorm(P);
    {
        const double *a[1] = {b};
        c.dots_to_host(a, a, 1);
        for (int k = 0; k < P; ++k) bnorm[k] = std::sqrt(c.hbuf[k]);
    }
    std::vector<char> done(P, 0);
    bool zero_rhs = false;
    hec_status_t status = HEC_OK;
    for (int k = 0; k < P; ++k) {
        info[k] = hec_krylov_info_t{HEC_OK, 0, 0, 0, 0.0};
        if (!std::isfinite(bnorm[k])) {
            // a NaN or infinity in b: this problem is not iterated
            done[k] = 1;
            info[k].status = HEC_ERR_BREAKDOWN;
        } else if (bnorm[k] == 0.0) {
            done[k] = 1, zero_rhs = true;
        }
    }
    if (zero_rhs) {
        // a zero right-hand side has the solution x = 0
        std::vector<double> keep(P);
        for (int k = 0; k < P; ++k) keep[k] = bnorm[k] == 0.0 ? 0.0 : 1.0;
        c.lincomb(x, {x}, keep);
    }
    {
        std::vector<double> bn(bnorm);
        for (double &v : bn) v = std::isfinite(v) && v > 0 ? v : 1.0;
        c.upload_coef(bn);
        hip_check(hipMemcpyAsync(bnm.p, c.coef.p, sizeof(double) * P, hipMemcpyDeviceToDevice, st), "copy");
    }
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(4L * P)), dim3(256), 0, st, d_iters, 4L * P, 0);
    hip_check(hipGetLastError(), "k_fill_i32");
    std::vector<int32_t> hcnt(4 * (size_t)P, 0);
    std::vector<const double *> pa(kMaxPairs), pb(kMaxPairs);
    auto launch_dcgs_step = [&](int j, int fin) {
        hipLaunchKernelGGL(k_dcgs_step, dim3(P), dim3(64), 0, st, j, m, P, fin, redm.as<double>(), tpm.as<double>(),
                           scm.as<double>(), Hm.as<double>(), csm.as<double>(), snm.as<double>(), gm.as<double>(),
                           bnm.as<double>(), rtol, maxit, c.actm.as<int8_t>(), c.kdm.as<int32_t>(), d_iters,
                           d_iters + 3 * P, d_stat, flg.as<int32_t>());
        hip_check(hipGetLastError(), "k_dcgs_step");
    };
    for (;;) {
        // true residual and convergence test (the one full synchronization
        // of a restart cycle)
        residual(A, b, x, r, R, st);
        hip_check(hipMemcpyAsync(hcnt.data(), d_iters, sizeof(int32_t) * 4 * P, hipMemcpyDeviceToHost, st), "D2H");
        {
            const double *a[1] = {r};
            c.dots_to_host(a, a, 1);
        }
        bool any = false;
        std::vector<double> beta(P);
        for (int k = 0; k < P; ++k) {
            beta[k] = std::sqrt(c.hbuf[k]);
            const double rr = bnorm[k] > 0 ? beta[k] / bnorm[k] : 0.0;
            if (!done[k]) {
                if (hcnt[2 * P + k] == HEC_ERR_BREAKDOWN || !std::isfinite(rr)) {
                    // a zero or non-finite Hessenberg column, or a non-finite
                    // iterate: stop this problem
                    done[k] = 1;
                    info[k].status = HEC_ERR_BREAKDOWN;
                } else if (rr <= rtol) {
                    done[k] = 1;
                }
            }
            any = any || !done[k];
        }
        int max_iters = 0;
        for (int k = 0; k < P; ++k) max_iters = std::max(max_iters, done[k] ? 0 : (int)hcnt[k]);
        if (!any) break;
        if (max_iters >= maxit) {
            status = HEC_ERR_NOT_CONVERGED;
            break;
        }
        // v_0 = r / beta, g = beta e_1, active mask
        std::vector<double> cf(P);
        for (int k = 0; k < P; ++k) cf[k] = done[k] ? 0.0 : 1.0 / beta[k];
        c.lincomb(Vi(0), {r}, cf);
        std::vector<double> g0((size_t)(m + 1) * P, 0.0);
        for (int k = 0; k < P; ++k) g0[k] = done[k] ? 0.0 : beta[k];
        c.upload_coef(g0);
        hip_check(hipMemcpyAsync(gm.p, c.coef.p, sizeof(double) * (m + 1) * P, hipMemcpyDeviceToDevice, st), "copy");
        std::vector<char> active(P);
        for (int k = 0; k < P; ++k) active[k] = !done[k];
        c.upload_active(active);
        hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(P)), dim3(256), 0, st, c.kdm.as<int32_t>(), (long)P, 0);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, flg.as<int32_t>(), (long)m, 0);
        hip_check(hipGetLastError(), "k_fill_i32");
        int steps = 0;
        for (int j = 0; j < m; ++j) {
            // two steps stay in flight: before issuing step j, wait for step
            // j-2 and stop if it left no problem active
            if (j >= 2) {
                hip_check(hipEventSynchronize(ev[j - 2]), "hipEventSynchronize");
                if (!hflag[j - 2]) break;
            }
            // problems already finished are skipped (their basis stops growing)
            apply_M(M, Vi(j), Zi(j), R, n, st, c.actm.as<int8_t>());
            spmv(A, Zi(j), w, R, st);
            const int8_t *act = c.actm.as<int8_t>();
            if (dcgs) {
                // slot j holds the candidate: inner products, column j-1 and
                // the coefficients, then q_j over the candidate and the next
                // candidate into slot j+1
                c.dcgs_dots(V, nR, j, Vi(j), w, redm.as<double>(), act);
                launch_dcgs_step(j, 0);
                if (P == 1)
                    hipLaunchKernelGGL(k_dcgs_update<true>, dim3(blocks_for(nR)), dim3(256), 0, st, V, nR, j, Vi(j), w,
                                       Vi(j + 1), redm.as<double>(), scm.as<double>(), nR, R, P, c.seg, act);
                else
                    hipLaunchKernelGGL(k_dcgs_update<false>, dim3(blocks_for(nR)), dim3(256), 0, st, V, nR, j, Vi(j),
                                       w, Vi(j + 1), redm.as<double>(), scm.as<double>(), nR, R, P, c.seg, act);
                hip_check(hipGetLastError(), "k_dcgs_update");
                hip_check(hipMemcpyAsync(hflag + j, flg.as<int32_t>() + j, sizeof(int32_t), hipMemcpyDeviceToHost,
                                         st), "D2H");
                hip_check(hipEventRecord(ev[j], st), "hipEventRecord");
                ++steps;
                continue;
            }
            // classical Gram-Schmidt, two passes
            for (int i = 0; i <= j; ++i) {
                pa[i] = Vi(i);
                pb[i] = w;
            }
            for (int pass = 0; pass < 2; ++pass) {
                double *dp = pass == 0 ? c.d1m.as<double>() : c.d2m.as<double>();
                c.dots_dev(pa.data(), pb.data(), j + 1, dp, act);
                hipLaunchKernelGGL(k_gs_update, dim3(blocks_for(nR)), dim3(256), 0, st, w, V, nR, dp, j + 1, nR, R,
                                   P, c.seg, act);
                hip_check(hipGetLastError(), "k_gs_update");
            }
            {
                const double *a[1] = {w};
                c.dots_dev(a, a, 1, c.dnm.as<double>(), act);
            }
            // v_{j+1} = w / h_{j+1,j} for the problems still active at step j
            hipLaunchKernelGGL(k_normalize, dim3(blocks_for(nR)), dim3(256), 0, st, Vi(j + 1), w, c.dnm.as<double>(),
                               act, nR, R, c.seg);
            hipLaunchKernelGGL(k_arnoldi, dim3(P), dim3(64), 0, st, j, m, P, c.d1m.as<double>(),
                               c.d2m.as<double>(), c.dnm.as<double>(), Hm.as<double>(), csm.as<double>(),
                               snm.as<double>(), gm.as<double>(), bnm.as<double>(), rtol, maxit, c.actm.as<int8_t>(),
                               c.kdm.as<int32_t>(), d_iters, d_stat, flg.as<int32_t>());
            hip_check(hipGetLastError(), "k_arnoldi");
            hip_check(hipMemcpyAsync(hflag + j, flg.as<int32_t>() + j, sizeof(int32_t), hipMemcpyDeviceToHost, st),
                      "D2H");
            hip_check(hipEventRecord(ev[j], st), "hipEventRecord");
            ++steps;
        }
        if (dcgs && steps == m) {
            // close the cycle: the last candidate's inner products finish
            // column m-1 of the problems still active
            c.dcgs_dots(V, nR, m, Vi(m), nullptr, redm.as<double>(), c.actm.as<int8_t>());
            launch_dcgs_step(m, 1);
        }
        // y = H^{-1} g per problem, x += Z y (each problem over its own basis)
        if (steps > 0) {
            hipLaunchKernelGGL(k_hess_solve, dim3(P), dim3(64), 0, st, m, P, Hm.as<double>(),
                               gm.as<double>(), c.kdm.as<int32_t>(), c.coef.as<double>(), d_rest);
            hipLaunchKernelGGL(k_basis_update, dim3(blocks_for(nR)), dim3(256), 0, st, x, Z, nR, c.coef.as<double>(),
                               c.kdm.as<int32_t>(), nR, R, P, c.seg);
            hip_check(hipGetLastError(), "k_basis_update");
        }
    }
    hip_check(hipMemcpyAsync(hcnt.data(), d_iters, sizeof(int32_t) * 4 * P, hipMemcpyDeviceToHost, st), "D2H");
    residual(A, b, x, r, R, st);
    {
        const double *a[1] = {r};
        c.dots_to_host(a, a, 1);
    }
    for (int k = 0; k < P; ++k) {
        info[k].iters = hcnt[k];
        info[k].precond_applies = dcgs ? hcnt[3 * P + k] : hcnt[k];
        info[k].restarts = hcnt[P + k];
        if (info[k].status == HEC_OK && hcnt[2 * P + k] == HEC_ERR_BREAKDOWN) info[k].status = HEC_ERR_BREAKDOWN;
    }
    precond_check_error(M);  // an aborted application voids the iterates
    return final_status(info, bnorm, c.hbuf, P, rtol, status);
}

// Right-preconditioned BiCGSTAB (van der Vorst) per RHS, shadow residual
// r0; when rho or (r0, v) vanishes the recurrence restarts from the current
// true residual.  Convergence is tested on the true residual.
hec_status_t bicgstab(const DevHec &A, const hec_precond_t &M, const double *b, double *x, int R, double rtol,
                      int maxit, hec_krylov_info_t *info, hipStream_t st, int nsys, const int32_t *sys_ptr)
{
    const long n = A.n, nR = n * R;
    Ctx c(n, R, st, nsys, sys_ptr);
    const int P = c.P;
    DevMem rm, rhm, pm, vm, phm, sm, shm, tm;
    for (DevMem *d : {&rm, &rhm, &pm, &vm, &phm, &sm, &shm, &tm}) d->alloc(sizeof(double) * (size_t)std::max<long>(1, nR));
    double *r = rm.as<double>(), *rh = rhm.as<double>(), *p = pm.as<double>(), *v = vm.as<double>(),
           *ph = phm.as<double>(), *s = sm.as<double>(), *sh = shm.as<double>(), *t = tm.as<double>();
    std::vector<double> bnorm(P);
    {
        const double *a[1] = {b};
        c.dots_to_host(a, a, 1);
        for (int k = 0; k < P; ++k) bnorm[k] = std::sqrt(c.hbuf[k]);
    }
    std::vector<char> done(P, 0);
    for (int k = 0; k < P; ++k) {
        info[k] = hec_krylov_info_t{HEC_OK, 0, 0, 0, 0.0};
        if (!std::isfinite(bnorm[k])) {
            // a NaN or infinity in b: this problem is not iterated
            done[k] = 1;
            info[k].status = HEC_ERR_BREAKDOWN;
        }
    }
    {
        std::vector<double> keep(P);
        bool zero_rhs = false;
        for (int k = 0; k < P; ++k) {
            keep[k] = bnorm[k] == 0.0 ? 0.0 : 1.0;
            zero_rhs = zero_rhs || bnorm[k] == 0.0;
        }
        if (zero_rhs) c.lincomb(x, {x}, keep);
    }
    int iters = 0, breakdowns = 0;
    hec_status_t status = HEC_OK;
    std::vector<double> rho(P), rho_old(P), alpha(P), omega(P), cf;
    for (;;) {
        residual(A, b, x, r, R, st);
        {
            const double *a[1] = {r};
            c.dots_to_host(a, a, 1);
        }
        bool any = false;
        for (int k = 0; k < P; ++k) {
            if (done[k]) continue;
            const double rr = bnorm[k] > 0 ? std::sqrt(c.hbuf[k]) / bnorm[k] : 0.0;
            if (!std::isfinite(rr)) {
                done[k] = 1;
                info[k].status = HEC_ERR_BREAKDOWN;
            } else if (bnorm[k] == 0.0 || rr <= rtol) {
                done[k] = 1;
            }
            any = any || !done[k];
        }
        if (!any) break;
        if (iters >= maxit) {
            status = HEC_ERR_NOT_CONVERGED;
            break;
        }
        if (breakdowns > 50) {
            status = HEC_ERR_BREAKDOWN;
            break;
        }
        hip_check(hipMemcpyAsync(rh, r, sizeof(double) * nR, hipMemcpyDeviceToDevice, st), "copy");
        hip_check(hipMemsetAsync(p, 0, sizeof(double) * nR, st), "memset");
        hip_check(hipMemsetAsync(v, 0, sizeof(double) * nR, st), "memset");
        std::fill(rho_old.begin(), rho_old.end(), 1.0);
        std::fill(alpha.begin(), alpha.end(), 1.0);
        std::fill(omega.begin(), omega.end(), 1.0);
        std::vector<char> act(P);
        for (int k = 0; k < P; ++k) act[k] = !done[k];
        // a non-finite scalar stops its problem before it reaches x
        auto stop_bad = [&](int k) {
            act[k] = 0;
            done[k] = 1;
            info[k].status = HEC_ERR_BREAKDOWN;
        };
        bool restart = false;
        while (iters < maxit && !restart) {
            {
                const double *a[1] = {rh}, *bb[1] = {r};
                c.dots_to_host(a, bb, 1);
            }
            for (int k = 0; k < P; ++k) {
                rho[k] = c.hbuf[k];
                if (act[k] && !std::isfinite(rho[k])) stop_bad(k);
                if (act[k] && rho[k] == 0.0) restart = true;
            }
            if (restart) {
                ++breakdowns;
                break;
            }
            // p = r + beta (p - omega v)
            cf.assign(3 * (size_t)P, 0.0);
            for (int k = 0; k < P; ++k) {
                if (!act[k]) continue;
                const double beta = (rho[k] / rho_old[k]) * (alpha[k] / omega[k]);
                cf[k] = 1.0;
                cf[P + k] = beta;
                cf[2 * P + k] = -beta * omega[k];
            }
            c.lincomb(p, {r, p, v}, cf);
            apply_M(M, p, ph, R, n, st);
            spmv(A, ph, v, R, st);
            {
                const double *a[1] = {rh}, *bb[1] = {v};
                c.dots_to_host(a, bb, 1);
            }
            for (int k = 0; k < P; ++k) {
                if (act[k] && !std::isfinite(c.hbuf[k])) stop_bad(k);
                if (!act[k]) {
                    alpha[k] = 0.0;
                    continue;
                }
                if (c.hbuf[k] == 0.0) restart = true;
                alpha[k] = c.hbuf[k] != 0.0 ? rho[k] / c.hbuf[k] : 0.0;
            }
            if (restart) {
                ++breakdowns;
                break;
            }
            // s = r - alpha v
            cf.assign(2 * (size_t)P, 0.0);
            for (int k = 0; k < P; ++k) {
                cf[k] = 1.0;
                cf[P + k] = -alpha[k];
            }
            c.lincomb(s, {r, v}, cf);
            ++iters;
            for (int k = 0; k < P; ++k)
                if (act[k]) {
                    info[k].iters += 1;
                    info[k].precond_applies += 1;
                }
            {
                const double *a[1] = {s};
                c.dots_to_host(a, a, 1);
            }
            bool early = false;
            std::vector<char> sdone(P, 0);
            for (int k = 0; k < P; ++k)
                if (act[k] && std::sqrt(c.hbuf[k]) / bnorm[k] <= rtol) sdone[k] = 1, early = true;
            apply_M(M, s, sh, R, n, st);
            spmv(A, sh, t, R, st);
            {
                const double *a[2] = {t, t}, *bb[2] = {s, t};
                c.dots_to_host(a, bb, 2);
            }
            for (int k = 0; k < P; ++k) {
                if (act[k] && !sdone[k] && !(std::isfinite(c.hbuf[k]) && std::isfinite(c.hbuf[P + k]))) stop_bad(k);
                if (!act[k] || sdone[k]) {
                    omega[k] = 0.0;
                    continue;
                }
                const double ts = c.hbuf[k], tt = c.hbuf[P + k];
                omega[k] = tt != 0.0 ? ts / tt : 0.0;
                info[k].precond_applies += 1;
            }
            // x += alpha ph + omega sh ; r = s - omega t
            cf.assign(3 * (size_t)P, 0.0);
            for (int k = 0; k < P; ++k) {
                cf[k] = 1.0;
                cf[P + k] = act[k] ? alpha[k] : 0.0;
                cf[2 * P + k] = act[k] ? omega[k] : 0.0;
            }
            c.lincomb(x, {x, ph, sh}, cf);
            cf.assign(2 * (size_t)P, 0.0);
            for (int k = 0; k < P; ++k) {
                cf[k] = 1.0;
                cf[P + k] = -omega[k];
            }
            c.lincomb(r, {s, t}, cf);
            {
                const double *a[1] = {r};
                c.dots_to_host(a, a, 1);
            }
            bool any_act = false;
            for (int k = 0; k < P; ++k) {
                if (!act[k]) continue;
                const double rr = std::sqrt(c.hbuf[k]) / bnorm[k];
                if (sdone[k] || rr <= rtol || omega[k] == 0.0) {
                    act[k] = 0;
                    restart = true;  // confirm on the true residual
                }
                any_act = any_act || act[k];
                rho_old[k] = rho[k];
            }
            if (early || !any_act) restart = true;
        }
    }
    residual(A, b, x, r, R, st);
    {
        const double *a[1] = {r};
        c.dots_to_host(a, a, 1);
    }
    precond_check_error(M);  // an aborted application voids the iterates
    return final_status(info, bnorm, c.hbuf, P, rtol, status);
}

}  // namespace

namespace hec {

void build_devhec(DevHec &d, const Csr &a, hec_dtype_t dt, int32_t ell_width)
{
    const int32_t n = a.n;
    d.n = n;
    d.dt = dt;
    int32_t w = ell_width;
    if (w < 0) {
        std::vector<int32_t> len(n);
        for (int32_t i = 0; i < n; ++i) len[i] = a.rp[i + 1] - a.rp[i];
        std::vector<int32_t> srt = len;
        std::sort(srt.begin(), srt.end());
        w = n ? srt[(n - 1) / 2] : 0;
        w = std::min(w, 64);
    }
    HecHost &h = d.host;
    h.n = n;
    h.w = w;
    h.ld = (n + 63) / 64 * 64;
    h.ell_col.assign((size_t)w * h.ld, n);
    h.ell_val.assign((size_t)w * h.ld, 0.0);
    h.csr_ptr.assign((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i) {
        int32_t e = 0;
        for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
            if (e < w) {
                h.ell_col[(size_t)e * h.ld + i] = a.ci[p];
                h.ell_val[(size_t)e * h.ld + i] = a.v[p];
                ++e;
            } else {
                h.csr_col.push_back(a.ci[p]);
                h.csr_val.push_back(a.v[p]);
            }
        }
        h.csr_ptr[i + 1] = (int32_t)h.csr_col.size();
    }
    d.w = w;
    d.ld = h.ld;
    d.tail_nnz = (int64_t)h.csr_col.size();
    hip_check(hipGetDevice(&d.device), "hipGetDevice");
    upload(d.ell_col, h.ell_col);
    upload_values(d.ell_val, h.ell_val, dt);
    if (d.tail_nnz > 0) {
        upload(d.tail_ptr, h.csr_ptr);
        upload(d.tail_col, h.csr_col);
        upload_values(d.tail_val, h.csr_val, dt);
    }
}

}  // namespace hec

extern "C" {

hec_status_t hec_from_csr(int32_t n, const int32_t *rowptr, const int32_t *col, const void *val, hec_dtype_t dt,
                          int32_t ell_width, hec_matrix_t *out)
{
    return guard_status([&]() -> hec_status_t {
            if (!out) fail(HEC_ERR_INVALID_ARG, "out is NULL");
            if (ell_width < -1 || ell_width > 64) fail(HEC_ERR_INVALID_ARG, "ell_width out of range");
            Csr a = csr_copy(n, rowptr, col, val, dt);
            auto m = std::make_unique<hec_matrix_s>();
            build_devhec(m->d, a, dt, ell_width);
            *out = m.release();
            return HEC_OK;
    });
}

hec_status_t hec_spmv(hec_matrix_t A, const double *x, double *y, int32_t nrhs, hipStream_t st)
{
    return guard_status([&]() -> hec_status_t {
            if (!A || nrhs < 1) fail(HEC_ERR_INVALID_ARG, "bad arguments");
            if (A->d.n > 0 && (!x || !y)) fail(HEC_ERR_INVALID_ARG, "vector pointer is NULL");
            spmv(A->d, x, y, nrhs, st);
            return HEC_OK;
    });
}

hec_status_t hec_matrix_export(hec_matrix_t A, int32_t *width, int32_t *ld, int64_t *tail_nnz, int32_t *ell_col,
                               double *ell_val, int32_t *csr_ptr, int32_t *csr_col, double *csr_val)
{
    return guard([&] {
    if (!A) fail(HEC_ERR_INVALID_ARG, "matrix is NULL");
    const HecHost &h = A->d.host;
    if (width) *width = h.w;
    if (ld) *ld = h.ld;
    if (tail_nnz) *tail_nnz = (int64_t)h.csr_col.size();
    if (ell_col) std::copy(h.ell_col.begin(), h.ell_col.end(), ell_col);
    if (ell_val) std::copy(h.ell_val.begin(), h.ell_val.end(), ell_val);
    if (csr_ptr) std::copy(h.csr_ptr.begin(), h.csr_ptr.end(), csr_ptr);
    if (csr_col) std::copy(h.csr_col.begin(), h.csr_col.end(), csr_col);
    if (csr_val) std::copy(h.csr_val.begin(), h.csr_val.end(), csr_val);
    });
}

void hec_matrix_destroy(hec_matrix_t A) { delete A; }

hec_status_t krylov_solve(hec_matrix_t A, hec_precond_t M, hec_krylov_t method, int32_t m, const double *b,
                          double *x, int32_t nrhs, double rtol, int32_t maxit, hec_krylov_info_t *info,
                          hipStream_t st)
{
    return guard_status([&]() -> hec_status_t {
            if (!A || !info || nrhs < 1 || maxit < 0 || !(rtol > 0.0)) fail(HEC_ERR_INVALID_ARG, "bad arguments");
            if (nrhs > 256) fail(HEC_ERR_INVALID_ARG, "at most 256 right-hand sides per solve");
            if (A->d.n > 0 && (!b || !x)) fail(HEC_ERR_INVALID_ARG, "vector pointer is NULL");
            precond_check(M, A->d.n);
            if (method == HEC_GMRES || method == HEC_FGMRES) {
                if (m < 1 || m > kMaxPairs - 1) fail(HEC_ERR_INVALID_ARG, "GMRES restart length must be 1..31");
                return gmres(A->d, M, m, b, x, nrhs, rtol, maxit, info, st, 1, nullptr);
            }
            if (method == HEC_BICGSTAB) return bicgstab(A->d, M, b, x, nrhs, rtol, maxit, info, st, 1, nullptr);
            fail(HEC_ERR_INVALID_ARG, "unknown Krylov method");
    });
}

hec_status_t krylov_solve_batch(hec_matrix_t A, hec_precond_t M, hec_krylov_t method, int32_t m, int32_t nsys,
                                const int32_t *sys_ptr, const double *b, double *x, int32_t nrhs, double rtol,
                                int32_t maxit, hec_krylov_info_t *info, hipStream_t st)
{
    return guard_status([&]() -> hec_status_t {
            if (!A || !info || !sys_ptr || nsys < 1 || nrhs < 1 || maxit < 0 || !(rtol > 0.0))
                fail(HEC_ERR_INVALID_ARG, "bad arguments");
            if (nrhs > 256) fail(HEC_ERR_INVALID_ARG, "at most 256 right-hand sides per solve");
            if ((int64_t)nsys * nrhs > 16384) fail(HEC_ERR_INVALID_ARG, "at most 16384 (system, rhs) problems");
            const int32_t n = A->d.n;
            if (sys_ptr[0] != 0 || sys_ptr[nsys] != n) fail(HEC_ERR_INVALID_ARG, "sys_ptr must run from 0 to n");
            for (int32_t s = 0; s < nsys; ++s)
                if (sys_ptr[s + 1] < sys_ptr[s]) fail(HEC_ERR_INVALID_ARG, "sys_ptr not monotone");
            if (n > 0 && (!b || !x)) fail(HEC_ERR_INVALID_ARG, "vector pointer is NULL");
            // the systems must not couple through A (the preconditioner's own
            // setup checks its blocks)
            for (int32_t s = 0; s < nsys; ++s)
                for (int32_t i = sys_ptr[s]; i < sys_ptr[s + 1]; ++i) {
                    const HecHost &h = A->d.host;
                    for (int32_t e = 0; e < h.w; ++e) {
                        const int32_t c = h.ell_col[(size_t)e * h.ld + i];
                        if (c < n && (c < sys_ptr[s] || c >= sys_ptr[s + 1]))
                            fail(HEC_ERR_INVALID_ARG, "A couples two systems (row " + std::to_string(i) + ")");
                    }
                    for (int32_t q = h.csr_ptr[i]; q < h.csr_ptr[i + 1]; ++q)
                        if (h.csr_col[q] < sys_ptr[s] || h.csr_col[q] >= sys_ptr[s + 1])
                            fail(HEC_ERR_INVALID_ARG, "A couples two systems (row " + std::to_string(i) + ")");
                }
            precond_check(M, n);
            if (method == HEC_GMRES || method == HEC_FGMRES) {
                if (m < 1 || m > kMaxPairs - 1) fail(HEC_ERR_INVALID_ARG, "GMRES restart length must be 1..31");
                return gmres(A->d, M, m, b, x, nrhs, rtol, maxit, info, st, nsys, sys_ptr);
            }
            if (method == HEC_BICGSTAB) return bicgstab(A->d, M, b, x, nrhs, rtol, maxit, info, st, nsys, sys_ptr);
            fail(HEC_ERR_INVALID_ARG, "unknown Krylov method");
    });
}

}  // extern "C"
