// bhq_lists.cpp -- host-side oct-tree and interaction-list builder (the
// input producer of the force path; not the accelerated part).
//
// Construction (Kodama & Ishiyama, Sec. 1 for the tree, Sec. 3.4 for the
// groups):
//   1. Every particle descends 21 levels from the root cube, taking the
//      upper half along an axis iff its coordinate is >= the cell centre;
//      the octant digits (x -> bit 0, y -> bit 1, z -> bit 2) form a 63-bit
//      key.  Particles are sorted by key (ties by input index).
//   2. Cells are cut from key ranges breadth-first: a cell with more than
//      nleaf particles, above depth 21, gets one child per non-empty
//      octant.  Particles inside a leaf are kept in input order.
//   3. Moments bottom-up: leaves from their particles; parents from their
//      children by the parallel-axis shift
//        Q = sum_c [Q_c + M_c (3 D D^T - |D|^2 1)],  T = sum_c [T_c + M_c |D|^2]
//      with D = com_c - com.
//   4. Groups: the largest cells with at most ncrit particles (or leaves).
//   5. Walk per group with an explicit stack, children in octant order:
//      a cell that contains the group is opened; otherwise it is accepted
//      iff side^2 < theta^2 d^2, d being the distance from its centre of
//      mass to the group cube (a one-particle cell becomes a j-particle);
//      a rejected leaf contributes its particles.
#include <algorithm>
#include <limits>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "bhq.h"

namespace {

constexpr int kMaxDepth = 21;

struct Cell {
    double center[3];
    double side;
    int64_t first, count;
    uint64_t key;       // octant digits of the path, left-aligned at depth 21
    int32_t depth;
    int32_t child0;     // first child id (children are consecutive), -1: leaf
    int32_t nchild;
    int32_t parent;
};

template <typename F>
void parallel_for(int64_t n, int nthreads, F f)
{
    if (n <= 0) return;
    int nt = nthreads;
    if (nt <= 0) nt = (int)std::thread::hardware_concurrency();
    if (nt < 1) nt = 1;
    if (nt > n) nt = (int)n;
    if (nt == 1) {
        for (int64_t k = 0; k < n; ++k) f(k);
        return;
    }
    std::atomic<int64_t> next(0);
    const int64_t grain = std::max<int64_t>(1, n / (int64_t)(nt * 64));
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t)
        pool.emplace_back([&]() {
            for (;;) {
                const int64_t a = next.fetch_add(grain);
                if (a >= n) break;
                const int64_t b = std::min(n, a + grain);
                for (int64_t k = a; k < b; ++k) f(k);
            }
        });
    for (auto &th : pool) th.join();
}

inline double min_image(double v, double box)
{
    return box > 0.0 ? v - box * std::nearbyint(v / box) : v;
}

}  // namespace

struct bhq_lists {
    int64_t n = 0;
    double box = 0.0;
    std::vector<int64_t> order;  // order[k] = input index of k-th particle
    std::vector<Cell> cells;
    std::vector<double> mass, com, q, tr;  // per cell: 1, 3, 6, 1
    std::vector<int32_t> groups;           // cell id per group
    std::vector<int64_t> jp_off, jp_idx, jc_off;
    std::vector<int32_t> jc_cell;
};

namespace {

// Does cell c contain cell g (c is g or an ancestor of g)?
inline bool contains(const Cell &c, const Cell &g)
{
    if (c.depth > g.depth) return false;
    const int sh = 3 * (kMaxDepth - c.depth);
    if (sh >= 64) return true;  // the root
    return (c.key >> sh) == (g.key >> sh);
}

inline double dist2_point_cube(const double *p, const double *c, double s,
                               double box)
{
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double v = std::fabs(min_image(p[k] - c[k], box)) - 0.5 * s;
        if (v > 0.0) d2 += v * v;
    }
    return d2;
}

inline double dist2_cube_cube(const double *c1, double s1, const double *c2,
                              double s2, double box)
{
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double v =
            std::fabs(min_image(c1[k] - c2[k], box)) - 0.5 * (s1 + s2);
        if (v > 0.0) d2 += v * v;
    }
    return d2;
}

// Squared distance from point p to the box [lo, hi] (minimum image),
// formed about the box centre.
inline double dist2_point_box(const double *p, const double *lo, const double *hi,
                              double box)
{
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double c = 0.5 * (lo[k] + hi[k]), h = 0.5 * (hi[k] - lo[k]);
        const double v = std::fabs(min_image(p[k] - c, box)) - h;
        if (v > 0.0) d2 += v * v;
    }
    return d2;
}

// With a cutoff rcut, an accepted cell whose centre of mass lies at least
// rcut (1 + 2^-16) from the bounding box of the group's particles is left
// out of the list: every pair it would form is beyond the cutoff and the
// split kernels skip it (the margin covers r^2 formed in FP32).  Returns
// the square of that distance, 0 without a cutoff.
inline double drop_dist2(double rcut)
{
    const double r = rcut * (1.0 + 0x1p-16);
    return rcut > 0.0 ? r * r : 0.0;
}

// Walk for one group; emits j-particles and j-cells through the callbacks.
// gbox: lo[3], hi[3] of the group's particles (read only with a cutoff).
template <typename EmitP, typename EmitC>
void walk_group(const bhq_lists &L, int32_t gid, const double *gbox, double theta2,
                double rcut, std::vector<int32_t> &stack, EmitP emit_p, EmitC emit_c)
{
    const double rdrop2 = drop_dist2(rcut);
    const Cell &g = L.cells[(size_t)gid];
    stack.clear();
    stack.push_back(0);
    while (!stack.empty()) {
        const int32_t id = stack.back();
        stack.pop_back();
        const Cell &c = L.cells[(size_t)id];
        if (!contains(c, g)) {
            if (rcut > 0.0 &&
                dist2_cube_cube(c.center, c.side, g.center, g.side, L.box) >
                    rcut * rcut)
                continue;
            const double d2 =
                dist2_point_cube(&L.com[3 * (size_t)id], g.center, g.side, L.box);
            if (c.side * c.side < theta2 * d2) {
                if (rdrop2 > 0.0 &&
                    dist2_point_box(&L.com[3 * (size_t)id], gbox, gbox + 3, L.box) >= rdrop2)
                    continue;
                if (c.count == 1)
                    emit_p(L.order[(size_t)c.first]);
                else
                    emit_c(id);
                continue;
            }
        }
        if (c.child0 < 0) {
            for (int64_t k = c.first; k < c.first + c.count; ++k)
                emit_p(L.order[(size_t)k]);
            continue;
        }
        // push children in reverse so they are visited in octant order
        for (int k = c.nchild - 1; k >= 0; --k) stack.push_back(c.child0 + k);
    }
}

}  // namespace

namespace {

int check_args(int64_t n, const double (*x)[3], const double *m, double theta,
               int ncrit, int nleaf, double box, double rcut)
{
    if (n < 1 || !x || !m || !(theta >= 0.0) || ncrit < 1 || nleaf < 1 ||
        nleaf > ncrit || !(box >= 0.0) || !(rcut >= 0.0) || n > 0x7fffffffLL)
        return BHQ_E_ARG;
    for (int64_t p = 0; p < n; ++p)
        if (!std::isfinite(x[p][0]) || !std::isfinite(x[p][1]) ||
            !std::isfinite(x[p][2]) || !std::isfinite(m[p]))
            return BHQ_E_NONFINITE;
    return BHQ_OK;
}

// Build the tree and lists of one particle set into *L (empty on entry).
int build_one(int64_t n, const double (*x)[3], const double *m, double theta,
              int ncrit, int nleaf, double box, double rcut, int nthreads,
              bhq_lists *L)
{
    try {
        L->n = n;
        L->box = box;

        // root cube
        double rc[3], rside;
        if (box > 0.0) {
            rc[0] = rc[1] = rc[2] = 0.5 * box;
            rside = box;
        } else {
            double lo[3] = {x[0][0], x[0][1], x[0][2]};
            double hi[3] = {lo[0], lo[1], lo[2]};
            for (int64_t p = 1; p < n; ++p)
                for (int k = 0; k < 3; ++k) {
                    lo[k] = std::min(lo[k], x[p][k]);
                    hi[k] = std::max(hi[k], x[p][k]);
                }
            double ext = 0.0;
            for (int k = 0; k < 3; ++k) {
                rc[k] = 0.5 * (lo[k] + hi[k]);
                ext = std::max(ext, hi[k] - lo[k]);
            }
            rside = ext > 0.0 ? ext * (1.0 + std::ldexp(1.0, -20)) : 1.0;
        }

        // 1. keys by descent, then sort
        std::vector<uint64_t> key((size_t)n);
        parallel_for(n, nthreads, [&](int64_t p) {
            double c[3] = {rc[0], rc[1], rc[2]};
            double s = rside;
            uint64_t k = 0;
            for (int lev = 0; lev < kMaxDepth; ++lev) {
                const double qd = s * 0.25;
                unsigned o = 0;
                for (int a = 0; a < 3; ++a) {
                    if (x[p][a] >= c[a]) {
                        o |= 1u << a;
                        c[a] = c[a] + qd;
                    } else {
                        c[a] = c[a] - qd;
                    }
                }
                k = (k << 3) | o;
                s = s * 0.5;
            }
            key[(size_t)p] = k;
        });
        L->order.resize((size_t)n);
        for (int64_t p = 0; p < n; ++p) L->order[(size_t)p] = p;
        std::sort(L->order.begin(), L->order.end(), [&](int64_t a, int64_t b) {
            const uint64_t ka = key[(size_t)a], kb = key[(size_t)b];
            return ka < kb || (ka == kb && a < b);
        });
        std::vector<uint64_t> skey((size_t)n);
        for (int64_t k = 0; k < n; ++k) skey[(size_t)k] = key[(size_t)L->order[(size_t)k]];
        std::vector<uint64_t>().swap(key);

        // 2. cells breadth-first from key ranges
        Cell root{};
        for (int k = 0; k < 3; ++k) root.center[k] = rc[k];
        root.side = rside;
        root.first = 0;
        root.count = n;
        root.key = 0;
        root.depth = 0;
        root.child0 = -1;
        root.nchild = 0;
        root.parent = -1;
        L->cells.push_back(root);
        for (size_t id = 0; id < L->cells.size(); ++id) {
            Cell c = L->cells[id];
            if (c.count <= nleaf || c.depth >= kMaxDepth) continue;
            const int sh = 3 * (kMaxDepth - 1 - c.depth);
            const int32_t child0 = (int32_t)L->cells.size();
            int32_t nch = 0;
            int64_t k = c.first;
            const int64_t end = c.first + c.count;
            while (k < end) {
                const unsigned o = (unsigned)((skey[(size_t)k] >> sh) & 7u);
                int64_t e = k;
                while (e < end && ((skey[(size_t)e] >> sh) & 7u) == o) ++e;
                Cell ch{};
                const double qd = c.side * 0.25;
                for (int a = 0; a < 3; ++a)
                    ch.center[a] = c.center[a] + (((o >> a) & 1u) ? qd : -qd);
                ch.side = c.side * 0.5;
                ch.first = k;
                ch.count = e - k;
                ch.key = c.key | ((uint64_t)o << sh);
                ch.depth = c.depth + 1;
                ch.child0 = -1;
                ch.nchild = 0;
                ch.parent = (int32_t)id;
                L->cells.push_back(ch);
                ++nch;
                k = e;
            }
            L->cells[id].child0 = child0;
            L->cells[id].nchild = nch;
        }
        const int64_t ncell = (int64_t)L->cells.size();
        if (ncell > 0x7fffffffLL) return BHQ_E_RANGE;
        // leaves keep input order among their particles
        for (const Cell &c : L->cells)
            if (c.child0 < 0)
                std::sort(L->order.begin() + c.first,
                          L->order.begin() + c.first + c.count);

        // 3. moments, children before parents (reverse breadth-first order)
        L->mass.assign((size_t)ncell, 0.0);
        L->com.assign((size_t)ncell * 3, 0.0);
        L->q.assign((size_t)ncell * 6, 0.0);
        L->tr.assign((size_t)ncell, 0.0);
        parallel_for(ncell, nthreads, [&](int64_t id) {
            const Cell &c = L->cells[(size_t)id];
            if (c.child0 >= 0) return;
            double M = 0.0, s[3] = {0.0, 0.0, 0.0};
            for (int64_t k = c.first; k < c.first + c.count; ++k) {
                const int64_t p = L->order[(size_t)k];
                M += m[p];
                for (int a = 0; a < 3; ++a) s[a] += m[p] * x[p][a];
            }
            double cm[3];
            for (int a = 0; a < 3; ++a) cm[a] = M > 0.0 ? s[a] / M : c.center[a];
            double q6[6] = {0, 0, 0, 0, 0, 0}, T = 0.0;
            for (int64_t k = c.first; k < c.first + c.count; ++k) {
                const int64_t p = L->order[(size_t)k];
                const double d0 = x[p][0] - cm[0], d1 = x[p][1] - cm[1],
                             d2 = x[p][2] - cm[2];
                const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                q6[0] += m[p] * (3.0 * d0 * d0 - r2);
                q6[1] += m[p] * 3.0 * d0 * d1;
                q6[2] += m[p] * 3.0 * d0 * d2;
                q6[3] += m[p] * (3.0 * d1 * d1 - r2);
                q6[4] += m[p] * 3.0 * d1 * d2;
                q6[5] += m[p] * (3.0 * d2 * d2 - r2);
                T += m[p] * r2;
            }
            L->mass[(size_t)id] = M;
            for (int a = 0; a < 3; ++a) L->com[3 * (size_t)id + a] = cm[a];
            for (int a = 0; a < 6; ++a) L->q[6 * (size_t)id + a] = q6[a];
            L->tr[(size_t)id] = T;
        });
        for (int64_t id = ncell - 1; id >= 0; --id) {
            const Cell &c = L->cells[(size_t)id];
            if (c.child0 < 0) continue;
            double M = 0.0, s[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < c.nchild; ++k) {
                const size_t ch = (size_t)(c.child0 + k);
                M += L->mass[ch];
                for (int a = 0; a < 3; ++a) s[a] += L->mass[ch] * L->com[3 * ch + a];
            }
            double cm[3];
            for (int a = 0; a < 3; ++a) cm[a] = M > 0.0 ? s[a] / M : c.center[a];
            double q6[6] = {0, 0, 0, 0, 0, 0}, T = 0.0;
            for (int k = 0; k < c.nchild; ++k) {
                const size_t ch = (size_t)(c.child0 + k);
                const double Mc = L->mass[ch];
                const double D[3] = {L->com[3 * ch] - cm[0], L->com[3 * ch + 1] - cm[1],
                                     L->com[3 * ch + 2] - cm[2]};
                const double D2 = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
                q6[0] += L->q[6 * ch + 0] + Mc * (3.0 * D[0] * D[0] - D2);
                q6[1] += L->q[6 * ch + 1] + Mc * 3.0 * D[0] * D[1];
                q6[2] += L->q[6 * ch + 2] + Mc * 3.0 * D[0] * D[2];
                q6[3] += L->q[6 * ch + 3] + Mc * (3.0 * D[1] * D[1] - D2);
                q6[4] += L->q[6 * ch + 4] + Mc * 3.0 * D[1] * D[2];
                q6[5] += L->q[6 * ch + 5] + Mc * (3.0 * D[2] * D[2] - D2);
                T += L->tr[ch] + Mc * D2;
            }
            L->mass[(size_t)id] = M;
            for (int a = 0; a < 3; ++a) L->com[3 * (size_t)id + a] = cm[a];
            for (int a = 0; a < 6; ++a) L->q[6 * (size_t)id + a] = q6[a];
            L->tr[(size_t)id] = T;
        }

        // 4. groups in depth-first order (so their particles are contiguous)
        {
            std::vector<int32_t> st{0};
            while (!st.empty()) {
                const int32_t id = st.back();
                st.pop_back();
                const Cell &c = L->cells[(size_t)id];
                if (c.count <= ncrit || c.child0 < 0) {
                    L->groups.push_back(id);
                    continue;
                }
                for (int k = c.nchild - 1; k >= 0; --k) st.push_back(c.child0 + k);
            }
        }
        const int64_t ng = (int64_t)L->groups.size();

        // bounding box of each group's particles (for the cutoff drop)
        std::vector<double> gbox;
        if (rcut > 0.0) {
            gbox.resize((size_t)ng * 6);
            for (int64_t gi = 0; gi < ng; ++gi) {
                const Cell &g = L->cells[(size_t)L->groups[(size_t)gi]];
                double *b = &gbox[(size_t)gi * 6];
                for (int k = 0; k < 3; ++k) {
                    b[k] = std::numeric_limits<double>::infinity();
                    b[3 + k] = -std::numeric_limits<double>::infinity();
                }
                for (int64_t q = g.first; q < g.first + g.count; ++q) {
                    const double *xp = x[L->order[(size_t)q]];
                    for (int k = 0; k < 3; ++k) {
                        b[k] = std::min(b[k], xp[k]);
                        b[3 + k] = std::max(b[3 + k], xp[k]);
                    }
                }
            }
        }
        auto gb = [&](int64_t gi) { return rcut > 0.0 ? &gbox[(size_t)gi * 6] : nullptr; };

        // 5. walk: count, prefix sums, fill
        const double theta2 = theta * theta;
        L->jp_off.assign((size_t)ng + 1, 0);
        L->jc_off.assign((size_t)ng + 1, 0);
        parallel_for(ng, nthreads, [&](int64_t gi) {
            thread_local std::vector<int32_t> stack;
            int64_t np = 0, nc = 0;
            walk_group(*L, L->groups[(size_t)gi], gb(gi), theta2, rcut, stack,
                       [&](int64_t) { ++np; }, [&](int32_t) { ++nc; });
            L->jp_off[(size_t)gi + 1] = np;
            L->jc_off[(size_t)gi + 1] = nc;
        });
        for (int64_t gi = 0; gi < ng; ++gi) {
            L->jp_off[(size_t)gi + 1] += L->jp_off[(size_t)gi];
            L->jc_off[(size_t)gi + 1] += L->jc_off[(size_t)gi];
        }
        L->jp_idx.resize((size_t)L->jp_off[(size_t)ng]);
        L->jc_cell.resize((size_t)L->jc_off[(size_t)ng]);
        parallel_for(ng, nthreads, [&](int64_t gi) {
            thread_local std::vector<int32_t> stack;
            int64_t *pp = L->jp_idx.data() + L->jp_off[(size_t)gi];
            int32_t *pc = L->jc_cell.data() + L->jc_off[(size_t)gi];
            walk_group(*L, L->groups[(size_t)gi], gb(gi), theta2, rcut, stack,
                       [&](int64_t p) { *pp++ = p; },
                       [&](int32_t c) { *pc++ = c; });
        });
    } catch (const std::bad_alloc &) {
        return BHQ_E_NOMEM;
    }
    return BHQ_OK;
}

}  // namespace

extern "C" {

int bhq_build_lists(int64_t n, const double (*x)[3], const double *m,
                    double theta, int ncrit, int nleaf, double box,
                    double rcut, int nthreads, bhq_lists **out)
{
    if (!out) return BHQ_E_ARG;
    *out = nullptr;
    int rc = check_args(n, x, m, theta, ncrit, nleaf, box, rcut);
    if (rc != BHQ_OK) return rc;
    bhq_lists *L = new (std::nothrow) bhq_lists();
    if (!L) return BHQ_E_NOMEM;
    rc = build_one(n, x, m, theta, ncrit, nleaf, box, rcut, nthreads, L);
    if (rc != BHQ_OK) {
        delete L;
        return rc;
    }
    *out = L;
    return BHQ_OK;
}

int bhq_build_lists_batch(int64_t nsys, const int64_t *sys_off,
                          const double (*x)[3], const double *m, double theta,
                          int ncrit, int nleaf, int nthreads, bhq_lists **out)
{
    if (!out) return BHQ_E_ARG;
    *out = nullptr;
    if (nsys < 1 || !sys_off || sys_off[0] != 0) return BHQ_E_ARG;
    for (int64_t s = 0; s < nsys; ++s)
        if (sys_off[s + 1] <= sys_off[s]) return BHQ_E_RANGE;
    const int64_t n = sys_off[nsys];
    int rc = check_args(n, x, m, theta, ncrit, nleaf, 0.0, 0.0);
    if (rc != BHQ_OK) return rc;
    std::vector<bhq_lists> part;
    try {
        part.resize((size_t)nsys);
    } catch (const std::bad_alloc &) {
        return BHQ_E_NOMEM;
    }
    // independent systems are built concurrently, one thread each
    std::vector<int> rcs((size_t)nsys, BHQ_OK);
    parallel_for(nsys, nthreads, [&](int64_t s) {
        const int64_t a = sys_off[s];
        rcs[(size_t)s] = build_one(sys_off[s + 1] - a, x + a, m + a, theta,
                                   ncrit, nleaf, 0.0, 0.0, 1, &part[(size_t)s]);
    });
    for (int r : rcs)
        if (r != BHQ_OK) return r;
    bhq_lists *L = new (std::nothrow) bhq_lists();
    if (!L) return BHQ_E_NOMEM;
    try {
        L->n = n;
        int64_t cell_base = 0, jp_base = 0, jc_base = 0;
        L->jp_off.push_back(0);
        L->jc_off.push_back(0);
        for (int64_t s = 0; s < nsys; ++s) {
            bhq_lists &P = part[(size_t)s];
            const int64_t a = sys_off[s];
            for (int64_t v : P.order) L->order.push_back(v + a);
            for (Cell c : P.cells) {
                c.first += a;
                if (c.child0 >= 0) c.child0 += (int32_t)cell_base;
                if (c.parent >= 0) c.parent += (int32_t)cell_base;
                L->cells.push_back(c);
            }
            L->mass.insert(L->mass.end(), P.mass.begin(), P.mass.end());
            L->com.insert(L->com.end(), P.com.begin(), P.com.end());
            L->q.insert(L->q.end(), P.q.begin(), P.q.end());
            L->tr.insert(L->tr.end(), P.tr.begin(), P.tr.end());
            for (int32_t g : P.groups) L->groups.push_back(g + (int32_t)cell_base);
            for (size_t g = 1; g < P.jp_off.size(); ++g) {
                L->jp_off.push_back(P.jp_off[g] + jp_base);
                L->jc_off.push_back(P.jc_off[g] + jc_base);
            }
            for (int64_t v : P.jp_idx) L->jp_idx.push_back(v + a);
            for (int32_t v : P.jc_cell) L->jc_cell.push_back(v + (int32_t)cell_base);
            cell_base += (int64_t)P.cells.size();
            jp_base += (int64_t)P.jp_idx.size();
            jc_base += (int64_t)P.jc_cell.size();
            if (cell_base > 0x7fffffffLL) {
                delete L;
                return BHQ_E_RANGE;
            }
            bhq_lists().jp_idx.swap(P.jp_idx);
        }
    } catch (const std::bad_alloc &) {
        delete L;
        return BHQ_E_NOMEM;
    }
    *out = L;
    return BHQ_OK;
}

int bhq_lists_sizes(const bhq_lists *L, int64_t sizes[4])
{
    if (!L || !sizes) return BHQ_E_ARG;
    const size_t ng = L->groups.size();
    sizes[0] = (int64_t)ng;
    sizes[1] = L->jp_off[ng];
    sizes[2] = L->jc_off[ng];
    sizes[3] = (int64_t)L->cells.size();
    return BHQ_OK;
}

int bhq_lists_export(const bhq_lists *L, int64_t *i_idx, int64_t *i_off,
                     double (*center)[3], double *side, int64_t *jp_off,
                     int64_t *jp_idx, int64_t *jc_off, int32_t *jc_cell)
{
    if (!L) return BHQ_E_ARG;
    const size_t ng = L->groups.size();
    if (i_idx) std::memcpy(i_idx, L->order.data(), L->order.size() * sizeof(int64_t));
    for (size_t g = 0; g < ng; ++g) {
        const Cell &c = L->cells[(size_t)L->groups[g]];
        if (i_off) i_off[g] = c.first;
        if (center)
            for (int a = 0; a < 3; ++a) center[g][a] = c.center[a];
        if (side) side[g] = c.side;
    }
    if (i_off) i_off[ng] = L->n;
    if (jp_off) std::memcpy(jp_off, L->jp_off.data(), (ng + 1) * sizeof(int64_t));
    if (jc_off) std::memcpy(jc_off, L->jc_off.data(), (ng + 1) * sizeof(int64_t));
    if (jp_idx) std::memcpy(jp_idx, L->jp_idx.data(), L->jp_idx.size() * sizeof(int64_t));
    if (jc_cell)
        std::memcpy(jc_cell, L->jc_cell.data(), L->jc_cell.size() * sizeof(int32_t));
    return BHQ_OK;
}

int bhq_lists_cells(const bhq_lists *L, double (*com)[3], double *mass,
                    double (*q)[6], double *trace)
{
    if (!L) return BHQ_E_ARG;
    const size_t nc = L->cells.size();
    if (com) std::memcpy(&com[0][0], L->com.data(), nc * 3 * sizeof(double));
    if (mass) std::memcpy(mass, L->mass.data(), nc * sizeof(double));
    if (q) std::memcpy(&q[0][0], L->q.data(), nc * 6 * sizeof(double));
    if (trace) std::memcpy(trace, L->tr.data(), nc * sizeof(double));
    return BHQ_OK;
}

int bhq_lists_free(bhq_lists *L)
{
    delete L;
    return BHQ_OK;
}

}  // extern "C"
