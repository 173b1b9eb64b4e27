// Incomplete LU factorizations of Section 3 (host setup; the factors feed the
// level-scheduled solves): ILU(0) (no fill), ILU(k) (fill limited by level k,
// the level-of-fill rule) and ILUT(p, tol) (dual dropping), plus the
// Restricted Additive Schwarz subdomain construction of eq. (4).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <functional>
#include <numeric>
#include <thread>

#include "hec_host.h"

namespace hec {

namespace {

// Row-wise numeric elimination on a fixed pattern.  `f` holds the pattern
// (sorted rows, diagonal present) with A's values scattered in (zero at fill
// positions).  For each row i, pivots k < i are taken in ascending order:
// l_ik = a_ik / u_kk, then a_ij -= l_ik * u_kj for every j > k of row k that
// row i also holds.  The matching is a merge of the two sorted rows.
void eliminate(Csr &f)
{
    const int32_t n = f.n;
    std::vector<int32_t> dpos(n, -1);
    for (int32_t i = 0; i < n; ++i) {
        auto b = f.ci.begin() + f.rp[i], e = f.ci.begin() + f.rp[i + 1];
        auto it = std::lower_bound(b, e, i);
        if (it == e || *it != i) fail(HEC_ERR_MISSING_DIAG, "row " + std::to_string(i) + " has no diagonal");
        dpos[i] = (int32_t)(it - f.ci.begin());
    }
    for (int32_t i = 0; i < n; ++i) {
        const int32_t ib = f.rp[i], ie = f.rp[i + 1];
        for (int32_t p = ib; p < dpos[i]; ++p) {
            const int32_t k = f.ci[p];
            const double piv = f.v[dpos[k]];
            if (piv == 0.0 || !std::isfinite(piv))
                fail(HEC_ERR_ZERO_PIVOT, "zero pivot at row " + std::to_string(k));
            const double lik = f.v[p] / piv;
            f.v[p] = lik;
            // merge row k's strict upper part with row i's entries after p
            int32_t q = dpos[k] + 1, qe = f.rp[k + 1], t = p + 1;
            while (q < qe && t < ie) {
                const int32_t cq = f.ci[q], ct = f.ci[t];
                if (cq == ct) {
                    f.v[t] = f.v[t] - lik * f.v[q];
                    ++q;
                    ++t;
                } else if (cq < ct) {
                    ++q;
                } else {
                    ++t;
                }
            }
        }
        const double d = f.v[dpos[i]];
        if (d == 0.0 || !std::isfinite(d)) fail(HEC_ERR_ZERO_PIVOT, "zero pivot at row " + std::to_string(i));
    }
}

// Split a combined factor into L (strict lower part plus a stored 1.0
// diagonal at the end of each row) and U (diagonal first).
void split(const Csr &f, Csr &L, Csr &U)
{
    const int32_t n = f.n;
    L = Csr();
    U = Csr();
    L.n = U.n = n;
    L.rp.assign((size_t)n + 1, 0);
    U.rp.assign((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t p = f.rp[i]; p < f.rp[i + 1]; ++p) {
            if (f.ci[p] < i) {
                L.ci.push_back(f.ci[p]);
                L.v.push_back(f.v[p]);
            } else {
                U.ci.push_back(f.ci[p]);
                U.v.push_back(f.v[p]);
            }
        }
        L.ci.push_back(i);
        L.v.push_back(1.0);
        L.rp[i + 1] = (int32_t)L.ci.size();
        U.rp[i + 1] = (int32_t)U.ci.size();
    }
}

void require_diagonals(const Csr &a)
{
    for (int32_t i = 0; i < a.n; ++i) {
        auto b = a.ci.begin() + a.rp[i], e = a.ci.begin() + a.rp[i + 1];
        if (!std::binary_search(b, e, i)) fail(HEC_ERR_MISSING_DIAG, "row " + std::to_string(i) + " of A has no diagonal");
    }
}

}  // namespace

void ilu0(const Csr &a, Csr &L, Csr &U)
{
    require_diagonals(a);
    Csr f = a;
    eliminate(f);
    split(f, L, U);
}

// Level of fill: entries of A have level 0; eliminating with pivot k gives
// entry (i, j) the level lev(i,k) + lev(k,j) + 1, the minimum over all k being
// kept; entries of level above k are not created.  Row i's pattern is kept in
// a sorted singly linked list so that fill created between two pivots is
// visited in ascending order.
void iluk(const Csr &a, int32_t K, Csr &L, Csr &U)
{
    require_diagonals(a);
    if (K < 0) fail(HEC_ERR_INVALID_ARG, "ILU(k) needs k >= 0");
    const int32_t n = a.n;
    Csr f;
    f.n = n;
    f.rp.assign((size_t)n + 1, 0);
    std::vector<int32_t> flev;           // level of each factor entry
    std::vector<int32_t> udiag(n, 0);    // position of each row's diagonal in f
    std::vector<int32_t> next(n + 1, -1), lev(n, 0);
    const int32_t HEAD = n;
    for (int32_t i = 0; i < n; ++i) {
        // linked list of row i's columns, seeded with A's pattern
        int32_t prev = HEAD;
        for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
            next[prev] = a.ci[p];
            lev[a.ci[p]] = 0;
            prev = a.ci[p];
        }
        next[prev] = -1;
        for (int32_t k = next[HEAD]; k != -1 && k < i; k = next[k]) {
            const int32_t lik = lev[k];
            int32_t at = k;  // insertion cursor: columns after k
            for (int32_t q = udiag[k] + 1; q < f.rp[k + 1]; ++q) {
                const int32_t j = f.ci[q];
                const int32_t nl = lik + flev[q] + 1;
                if (nl > K) continue;
                while (next[at] != -1 && next[at] < j) at = next[at];
                if (next[at] == j) {
                    lev[j] = std::min(lev[j], nl);
                } else {
                    next[j] = next[at];
                    next[at] = j;
                    lev[j] = nl;
                }
                at = j;
            }
        }
        for (int32_t j = next[HEAD]; j != -1; j = next[j]) {
            if (j == i) udiag[i] = (int32_t)f.ci.size();
            f.ci.push_back(j);
            flev.push_back(lev[j]);
        }
        f.rp[i + 1] = (int32_t)f.ci.size();
    }
    f.v.assign(f.ci.size(), 0.0);
    for (int32_t i = 0; i < n; ++i) {
        int32_t q = f.rp[i];
        for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
            while (f.ci[q] < a.ci[p]) ++q;
            f.v[q] = a.v[p];
        }
    }
    eliminate(f);
    split(f, L, U);
}

// ILUT(p, tau): row i starts as a dense work row w = a_i; tau_i = tau *
// ||a_i||_2.  Pivots k < i are taken in ascending order (a min-heap over the
// row's lower columns, which grows with fill): w_k /= u_kk; w_k is dropped if
// |w_k| < tau_i, otherwise w -= w_k * (strict upper part of U row k).  After
// the sweep, off-diagonals with |w_j| < tau_i are dropped and only the p
// largest magnitudes of the L part and of the strict U part are kept (ties to
// the smaller column); the diagonal is always kept.
void ilut(const Csr &a, int32_t p, double tau, Csr &L, Csr &U)
{
    require_diagonals(a);
    if (p < 0 || !(tau >= 0.0)) fail(HEC_ERR_INVALID_ARG, "ILUT needs p >= 0 and tol >= 0");
    const int32_t n = a.n;
    L = Csr();
    U = Csr();
    L.n = U.n = n;
    L.rp.assign((size_t)n + 1, 0);
    U.rp.assign((size_t)n + 1, 0);
    std::vector<double> w(n, 0.0);
    std::vector<char> in(n, 0);
    std::vector<int32_t> cols;
    std::vector<int32_t> heap;
    std::vector<std::pair<double, int32_t>> cand;
    auto by_mag = [](const std::pair<double, int32_t> &x, const std::pair<double, int32_t> &y) {
        return x.first > y.first || (x.first == y.first && x.second < y.second);
    };
    for (int32_t i = 0; i < n; ++i) {
        cols.clear();
        heap.clear();
        double nrm2 = 0.0;
        for (int32_t q = a.rp[i]; q < a.rp[i + 1]; ++q) {
            const int32_t j = a.ci[q];
            nrm2 = nrm2 + a.v[q] * a.v[q];
            w[j] = a.v[q];
            in[j] = 1;
            cols.push_back(j);
            if (j < i) heap.push_back(j);
        }
        const double tau_i = tau * std::sqrt(nrm2);
        std::make_heap(heap.begin(), heap.end(), std::greater<int32_t>());
        while (!heap.empty()) {
            std::pop_heap(heap.begin(), heap.end(), std::greater<int32_t>());
            const int32_t k = heap.back();
            heap.pop_back();
            const int32_t ub = U.rp[k], ue = U.rp[k + 1];  // U row k: diagonal first
            const double wk = w[k] / U.v[ub];
            if (std::fabs(wk) < tau_i) {
                w[k] = 0.0;
                continue;
            }
            w[k] = wk;
            for (int32_t q = ub + 1; q < ue; ++q) {
                const int32_t j = U.ci[q];
                if (!in[j]) {
                    in[j] = 1;
                    w[j] = 0.0;
                    cols.push_back(j);
                    if (j < i) {
                        heap.push_back(j);
                        std::push_heap(heap.begin(), heap.end(), std::greater<int32_t>());
                    }
                }
                w[j] = w[j] - wk * U.v[q];
            }
        }
        // L part
        cand.clear();
        for (int32_t j : cols)
            if (j < i && w[j] != 0.0 && std::fabs(w[j]) >= tau_i) cand.push_back({std::fabs(w[j]), j});
        std::sort(cand.begin(), cand.end(), by_mag);
        if ((int32_t)cand.size() > p) cand.resize(p);
        std::sort(cand.begin(), cand.end(), [](auto &x, auto &y) { return x.second < y.second; });
        for (auto &c : cand) {
            L.ci.push_back(c.second);
            L.v.push_back(w[c.second]);
        }
        L.ci.push_back(i);
        L.v.push_back(1.0);
        L.rp[i + 1] = (int32_t)L.ci.size();
        // U part: diagonal, then the p largest strict-upper entries
        const double d = in[i] ? w[i] : 0.0;
        if (d == 0.0 || !std::isfinite(d)) fail(HEC_ERR_ZERO_PIVOT, "ILUT zero pivot at row " + std::to_string(i));
        U.ci.push_back(i);
        U.v.push_back(d);
        cand.clear();
        for (int32_t j : cols)
            if (j > i && w[j] != 0.0 && std::fabs(w[j]) >= tau_i) cand.push_back({std::fabs(w[j]), j});
        std::sort(cand.begin(), cand.end(), by_mag);
        if ((int32_t)cand.size() > p) cand.resize(p);
        std::sort(cand.begin(), cand.end(), [](auto &x, auto &y) { return x.second < y.second; });
        for (auto &c : cand) {
            U.ci.push_back(c.second);
            U.v.push_back(w[c.second]);
        }
        U.rp[i + 1] = (int32_t)U.ci.size();
        for (int32_t j : cols) {
            w[j] = 0.0;
            in[j] = 0;
        }
    }
}

// Factor a block-diagonal matrix block by block on host threads.  Block b
// is rows block_ptr[b]..block_ptr[b+1]-1 and has no entry outside its own
// columns, so every row's elimination stays inside its block and the result
// equals factoring the whole matrix at once, bit for bit.
void factor_blocks(const Csr &a, const std::vector<int32_t> &block_ptr,
                   const std::function<void(const Csr &, Csr &, Csr &)> &fac, Csr &L, Csr &U)
{
    const int32_t nb = (int32_t)block_ptr.size() - 1;
    std::vector<Csr> Ls(nb), Us(nb);
    std::atomic<int32_t> next{0};
    std::atomic<bool> failed{false};
    Error first_err{HEC_OK, ""};
    auto work = [&]() {
        for (;;) {
            const int32_t b = next.fetch_add(1);
            if (b >= nb || failed.load()) return;
            const int32_t r0 = block_ptr[b], r1 = block_ptr[b + 1];
            Csr blk;
            blk.n = r1 - r0;
            blk.rp.resize((size_t)blk.n + 1);
            const int32_t p0 = a.rp[r0];
            for (int32_t i = r0; i <= r1; ++i) blk.rp[i - r0] = a.rp[i] - p0;
            blk.ci.resize((size_t)(a.rp[r1] - p0));
            blk.v.assign(a.v.begin() + p0, a.v.begin() + a.rp[r1]);
            for (int32_t q = p0; q < a.rp[r1]; ++q) blk.ci[q - p0] = a.ci[q] - r0;
            try {
                fac(blk, Ls[b], Us[b]);
            } catch (const Error &e) {
                if (!failed.exchange(true)) first_err = Error{e.code, e.msg + " (block " + std::to_string(b) + ")"};
                return;
            }
        }
    };
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int32_t nt = (int32_t)std::min<unsigned>(std::min<unsigned>(hw, 16u), (unsigned)std::max(1, nb));
    std::vector<std::thread> pool;
    for (int32_t t = 1; t < nt; ++t) pool.emplace_back(work);
    work();
    for (auto &th : pool) th.join();
    if (failed.load()) fail(first_err.code, first_err.msg);
    auto join = [&](std::vector<Csr> &parts, Csr &out) {
        out = Csr();
        out.n = a.n;
        out.rp.assign((size_t)a.n + 1, 0);
        size_t total = 0;
        for (auto &c : parts) total += c.ci.size();
        out.ci.reserve(total);
        out.v.reserve(total);
        for (int32_t b = 0; b < nb; ++b) {
            const int32_t r0 = block_ptr[b];
            const int64_t base = (int64_t)out.ci.size();
            for (int32_t q = 0; q < (int32_t)parts[b].ci.size(); ++q) out.ci.push_back(parts[b].ci[q] + r0);
            out.v.insert(out.v.end(), parts[b].v.begin(), parts[b].v.end());
            for (int32_t i = 0; i < parts[b].n; ++i) out.rp[r0 + i + 1] = (int32_t)(base + parts[b].rp[i + 1]);
            parts[b] = Csr();
        }
    };
    join(Ls, L);
    join(Us, U);
}

// Subdomain s owns {i : owner[i] == s}; `overlap` rings of graph neighbours in
// A extend it.  The block-diagonal matrix holds A_s = A[ext_s, ext_s] (the
// couplings to rows outside ext_s are dropped) with local, ascending order.
RasLayout ras_layout(const Csr &a, int32_t nsub, const int32_t *owner, int32_t overlap)
{
    const int32_t n = a.n;
    if (nsub <= 0 || !owner || overlap < 0) fail(HEC_ERR_INVALID_ARG, "bad RAS arguments");
    for (int32_t i = 0; i < n; ++i)
        if (owner[i] < 0 || owner[i] >= nsub) fail(HEC_ERR_INVALID_ARG, "owner out of range");
    RasLayout r;
    r.nsub = nsub;
    r.ext_ptr.assign((size_t)nsub + 1, 0);
    std::vector<std::vector<int32_t>> members(nsub);
    for (int32_t i = 0; i < n; ++i) members[owner[i]].push_back(i);
    std::vector<int32_t> mark(n, -1), local(n, -1);
    Csr &B = r.blockdiag;
    B.rp.push_back(0);
    for (int32_t s = 0; s < nsub; ++s) {
        std::vector<int32_t> ext = members[s];
        for (int32_t i : ext) mark[i] = s;
        std::vector<int32_t> frontier = ext;
        for (int32_t ring = 0; ring < overlap; ++ring) {
            std::vector<int32_t> nxt;
            for (int32_t i : frontier)
                for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
                    int32_t j = a.ci[p];
                    if (mark[j] != s) {
                        mark[j] = s;
                        nxt.push_back(j);
                    }
                }
            ext.insert(ext.end(), nxt.begin(), nxt.end());
            frontier.swap(nxt);
        }
        std::sort(ext.begin(), ext.end());
        const int32_t base = (int32_t)r.ext.size();
        for (size_t t = 0; t < ext.size(); ++t) local[ext[t]] = base + (int32_t)t;
        for (int32_t i : ext) {
            r.ext.push_back(i);
            r.owned.push_back(owner[i] == s ? 1 : 0);
            for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
                int32_t j = a.ci[p];
                if (mark[j] == s && local[j] >= base) {
                    B.ci.push_back(local[j]);
                    B.v.push_back(a.v[p]);
                }
            }
            B.rp.push_back((int32_t)B.ci.size());
        }
        for (int32_t i : ext) local[i] = -1;
        r.ext_ptr[s + 1] = (int32_t)r.ext.size();
    }
    B.n = (int32_t)r.ext.size();
    return r;
}

}  // namespace hec
