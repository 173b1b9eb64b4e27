/*
 * Multithreaded level-scheduled CPU triangular solve: the host-side
 * comparison baseline that runs Algorithm 2 of Section 2.2 on all host cores
 * (rows of one level in parallel, a barrier between levels).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the benchmark's CPU baseline leg and the tests load
 * it.  It shares no code with the GPU path and is kept out of the plain
 * oracle library so that the oracle itself stays serial.
 *
 * The level sets come from the caller (the oracle's own level analysis,
 * eq. (2) and eq. (3)).  Each row does exactly the serial oracle's arithmetic
 * (start from b_i, subtract the stored off-diagonal terms in entry order,
 * divide by the diagonal unless it is a unit), so the result is bit-identical
 * to the serial substitution whatever the thread count.  Build with
 * -O2 -ffp-contract=off -fopenmp.
 *
 * Return codes: 0 ok, -2 missing diagonal, -5 bad argument.
 */
#include <omp.h>
#include <stdint.h>

int orc_omp_threads(void) { return omp_get_max_threads(); }

/* x = T^{-1} b for a lower (upper = 0) or upper (upper = 1) triangle T in
 * CSR; levelptr[nlev+1] / perm[n] list the rows of each level (level k's rows
 * are perm[levelptr[k] .. levelptr[k+1]-1]).  b, x: [n][nrhs], RHS fastest;
 * must not alias.  nthreads <= 0 uses the OpenMP default. */
int orc_level_solve_omp(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int unit,
                        int upper, int32_t nlev, const int32_t *levelptr, const int32_t *perm,
                        int32_t nrhs, const double *b, double *x, int32_t nthreads)
{
    if (n < 0 || nrhs < 1 || nlev < 0 || (n > 0 && levelptr[nlev] != n)) return -5;
    int bad = 0;
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel num_threads(nt) reduction(| : bad)
    for (int32_t k = 0; k < nlev; ++k) {
#pragma omp for schedule(static)
        for (int32_t q = levelptr[k]; q < levelptr[k + 1]; ++q) {
            const int32_t i = perm[q];
            double d = 0.0;
            int have_d = 0;
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
                if (ci[p] == i) { d = v[p]; have_d = 1; }
            if (!unit && !have_d) { bad = 1; continue; }
            for (int32_t r = 0; r < nrhs; ++r) {
                double s = b[(int64_t)i * nrhs + r];
                for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
                    const int32_t j = ci[p];
                    if (upper ? j > i : j < i) s = s - v[p] * x[(int64_t)j * nrhs + r];
                }
                x[(int64_t)i * nrhs + r] = unit ? s : s / d;
            }
        }
        /* the implicit barrier of the worksharing loop separates the levels */
    }
    return bad ? -2 : 0;
}
