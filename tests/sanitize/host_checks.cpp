// Host-side code paths under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Built with g++ -fsanitize=address,undefined from the library's host
// translation units (level analysis, HEC construction, execution schedules,
// factorizations, RAS layout) and the oracle's C file, then run on seeded
// synthetic matrices: 2D/3D Laplacians with lognormal coefficients and random
// lower triangles.  Every analysis path (level launches, level-persistent and
// owner schedules, the dataflow kernel with one part per workgroup and with a
// part queue, several group counts and right-hand-side widths) and every
// factorization runs; the results are checked against the oracle where the
// two define the same thing bit for bit (levels of eq. (2), ILU(0) values),
// so a silently wrong access that does not trap is still likely to show.
// Exit status 0 = every check passed; the sanitizers abort on their own.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "hec_host.h"

extern "C" {
int orc_levels_kahn(int32_t n, const int32_t *rp, const int32_t *ci, int upper, int32_t *level, int32_t *nlev_out);
int orc_ilu0(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, double *lu);
int orc_iluk(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t K, int32_t **out_rp,
             int32_t **out_ci, double **out_v);
int orc_ilut(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t p, double tau,
             int32_t **lrp, int32_t **lci, double **lv, int32_t **urp, int32_t **uci, double **uv);
int orc_lower_solve(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int unit, int32_t nrhs,
                    const double *b, double *x);
int orc_upper_solve(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int unit, int32_t nrhs,
                    const double *b, double *x);
int orc_sor(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, double omega, int32_t nrhs,
            const double *b, double *x, int32_t sweeps, int symmetric);
void orc_spmv(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t nrhs, const double *x,
              double *y);
void orc_free(void *p);
}

using hec::Csr;

static int failures = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                           \
        }                                                                         \
    } while (0)

// 7-point (3D) or 5-point (2D) finite-volume diffusion with lognormal cell
// coefficients (harmonic means on faces), natural order, rows sorted.
static Csr grid(int nx, int ny, int nz, double sigma, unsigned seed)
{
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    const int n = nx * ny * nz;
    std::vector<double> k(n);
    for (double &v : k) v = std::exp(sigma * nd(rng));
    Csr a;
    a.n = n;
    a.rp.assign(1, 0);
    auto id = [&](int x, int y, int z) { return x + nx * (y + ny * z); };
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int i = id(x, y, z);
                double diag = 0.0;
                std::vector<std::pair<int, double>> row;
                const int nb[6][3] = {{0, 0, -1}, {0, -1, 0}, {-1, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
                for (auto &d : nb) {
                    const int X = x + d[0], Y = y + d[1], Z = z + d[2];
                    if (nz == 1 && d[2] != 0) continue;
                    if (X < 0 || Y < 0 || Z < 0 || X >= nx || Y >= ny || Z >= nz) {
                        diag += k[i];
                        continue;
                    }
                    const int j = id(X, Y, Z);
                    const double f = 2.0 * k[i] * k[j] / (k[i] + k[j]);
                    diag += f;
                    row.push_back({j, -f});
                }
                row.push_back({i, diag});
                std::sort(row.begin(), row.end());
                for (auto &e : row) {
                    a.ci.push_back(e.first);
                    a.v.push_back(e.second);
                }
                a.rp.push_back((int32_t)a.ci.size());
            }
    return a;
}

// Random lower triangle with a dominant diagonal.
static Csr random_lower(int n, double density, unsigned seed)
{
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    Csr a;
    a.n = n;
    a.rp.assign(1, 0);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < i; ++j)
            if (u(rng) < density) {
                a.ci.push_back(j);
                a.v.push_back(u(rng) - 0.5);
            }
        a.ci.push_back(i);
        a.v.push_back(4.0 + u(rng));
        a.rp.push_back((int32_t)a.ci.size());
    }
    return a;
}

static void check_levels(const Csr &t, bool upper)
{
    hec::Levels lv = hec::compute_levels(t, upper);
    std::vector<int32_t> lev(t.n);
    int32_t nlev = 0;
    CHECK(orc_levels_kahn(t.n, t.rp.data(), t.ci.data(), upper ? 1 : 0, lev.data(), &nlev) == 0);
    CHECK(nlev == lv.nlev);
    for (int i = 0; i < t.n; ++i) CHECK(lev[i] == lv.level[i]);
}

static void analyses(const Csr &t, bool upper, bool unit, const std::vector<int32_t> *blocks)
{
    check_levels(t, upper);
    const hec_dtype_t dts[2] = {HEC_F64, HEC_F32};
    struct Shape {
        int sched, variant, groups, nrhs, partition;
    };
    const Shape shapes[] = {
        {HEC_SCHED_LEVEL_LAUNCH, 0, 0, 1, 0},      {HEC_SCHED_LEVEL_LAUNCH, 5, 0, 3, 0},
        {HEC_SCHED_LEVEL_PERSISTENT, 0, 7, 2, 0},  {HEC_SCHED_OWNER_PERSISTENT, 2, 5, 1, 1},
        {HEC_SCHED_OWNER_PERSISTENT, 2, 6, 2, 2},  {HEC_SCHED_OWNER_PERSISTENT, 4, 9, 1, 0},
        {HEC_SCHED_OWNER_PERSISTENT, 4, 4, 8, 1},  {HEC_SCHED_OWNER_PERSISTENT, 6, 3, 4, 0},
        {HEC_SCHED_AUTO, 0, 0, 16, 0},             {HEC_SCHED_AUTO, 0, 2, 1, 0},
    };
    for (const Shape &sh : shapes)
        for (hec_dtype_t dt : dts) {
            hec::Tune tu = hec::default_tune();
            tu.schedule = sh.sched;
            tu.variant = sh.variant;
            tu.num_groups = sh.groups;
            tu.max_nrhs = sh.nrhs;
            tu.partition = sh.partition;
            tu.host_only = 1;
            if (sh.variant == 6) tu.part_rows = 37;  // many small parts
            hec::DeviceShape dev;
            dev.lds = 32768;  // a small LDS forces the larger plans through the part queue
            try {
                hec::TriHost h = hec::analyze(t, upper, unit, dt, tu, dev, blocks);
                CHECK(h.n == t.n && (int)h.ex.orig.size() == t.n);
            } catch (const hec::Error &e) {
                // a dataflow plan that cannot fit is refused, not mis-built
                CHECK(e.code == HEC_ERR_CAPACITY || e.code == HEC_ERR_INVALID_ARG);
            }
        }
}

static void factorizations(const Csr &a)
{
    const int n = a.n;
    // ILU(0): the product's L and U against the oracle's combined factor
    Csr L, U;
    hec::ilu0(a, L, U);
    std::vector<double> lu(a.v.size());
    CHECK(orc_ilu0(n, a.rp.data(), a.ci.data(), a.v.data(), lu.data()) == 0);
    for (int i = 0; i < n; ++i) {
        int pl = L.rp[i], pu = U.rp[i];
        for (int p = a.rp[i]; p < a.rp[i + 1]; ++p) {
            const int j = a.ci[p];
            if (j < i) CHECK(L.ci[pl] == j && L.v[pl++] == lu[p]);
            else CHECK(U.ci[pu] == j && U.v[pu++] == lu[p]);
        }
    }
    // ILU(k) and ILUT: both implementations run; entry counts agree
    for (int K : {1, 2}) {
        Csr Lk, Uk;
        hec::iluk(a, K, Lk, Uk);
        int32_t *rp = nullptr, *ci = nullptr;
        double *v = nullptr;
        CHECK(orc_iluk(n, a.rp.data(), a.ci.data(), a.v.data(), K, &rp, &ci, &v) == 0);
        CHECK((int64_t)rp[n] + n == Lk.nnz() + Uk.nnz());  // the product stores L's unit diagonal
        orc_free(rp);
        orc_free(ci);
        orc_free(v);
    }
    {
        Csr Lt, Ut;
        hec::ilut(a, 5, 1e-2, Lt, Ut);
        int32_t *lrp, *lci, *urp, *uci;
        double *lv, *uv;
        CHECK(orc_ilut(n, a.rp.data(), a.ci.data(), a.v.data(), 5, 1e-2, &lrp, &lci, &lv, &urp, &uci, &uv) == 0);
        CHECK(urp[n] == Ut.nnz());
        for (void *q : {(void *)lrp, (void *)lci, (void *)lv, (void *)urp, (void *)uci, (void *)uv}) orc_free(q);
    }
    // the oracle's solves, SOR sweeps and product on the same matrix
    std::vector<double> b((size_t)n * 2, 1.0), x((size_t)n * 2), y((size_t)n * 2);
    CHECK(orc_lower_solve(n, L.rp.data(), L.ci.data(), L.v.data(), 1, 2, b.data(), y.data()) == 0);
    CHECK(orc_upper_solve(n, U.rp.data(), U.ci.data(), U.v.data(), 0, 2, y.data(), x.data()) == 0);
    orc_spmv(n, a.rp.data(), a.ci.data(), a.v.data(), 2, x.data(), y.data());
    std::fill(x.begin(), x.end(), 0.0);
    CHECK(orc_sor(n, a.rp.data(), a.ci.data(), a.v.data(), 1.3, 2, b.data(), x.data(), 2, 1) == 0);
    // the triangles through every analysis path
    analyses(L, false, true, nullptr);
    analyses(U, true, false, nullptr);
}

int main()
{
    // grids: natural-order 3D and 2D, one of them large enough for many parts
    factorizations(grid(9, 8, 7, 1.0, 1));
    factorizations(grid(31, 17, 1, 2.0, 2));
    factorizations(grid(6, 5, 4, 0.0, 3));
    // random lower triangles, unit and non-unit
    for (unsigned s = 0; s < 3; ++s) {
        Csr t = random_lower(300 + 50 * s, 0.02, 10 + s);
        analyses(t, false, false, nullptr);
    }
    // block-diagonal batch: three grids as independent systems, and RAS
    // layouts with overlap 0 and 1 on a grid
    {
        Csr g1 = grid(12, 11, 1, 1.0, 20), g2 = grid(5, 5, 5, 1.0, 21), g3 = grid(40, 9, 1, 1.0, 22);
        Csr bd;
        bd.n = g1.n + g2.n + g3.n;
        bd.rp.assign(1, 0);
        std::vector<int32_t> sp{0};
        int off = 0;
        for (const Csr *g : {&g1, &g2, &g3}) {
            for (int i = 0; i < g->n; ++i) {
                for (int p = g->rp[i]; p < g->rp[i + 1]; ++p) {
                    bd.ci.push_back(g->ci[p] + off);
                    bd.v.push_back(g->v[p]);
                }
                bd.rp.push_back((int32_t)bd.ci.size());
            }
            off += g->n;
            sp.push_back(off);
        }
        Csr L, U;
        hec::factor_blocks(bd, sp, [](const Csr &m, Csr &l, Csr &u) { hec::iluk(m, 1, l, u); }, L, U);
        analyses(L, false, true, &sp);
        analyses(U, true, false, &sp);
        Csr a = grid(14, 12, 10, 1.0, 23);
        std::vector<int32_t> owner(a.n);
        for (int i = 0; i < a.n; ++i) owner[i] = (int32_t)((int64_t)i * 6 / a.n);
        for (int ov : {0, 1, 2}) {
            hec::RasLayout lay = hec::ras_layout(a, 6, owner.data(), ov);
            Csr Lb, Ub;
            hec::factor_blocks(lay.blockdiag, lay.ext_ptr, [](const Csr &m, Csr &l, Csr &u) { hec::ilu0(m, l, u); },
                               Lb, Ub);
            analyses(Lb, false, true, &lay.ext_ptr);
            analyses(Ub, true, false, &lay.ext_ptr);
        }
    }
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
