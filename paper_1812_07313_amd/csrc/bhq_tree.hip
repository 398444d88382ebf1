// bhq_tree.hip -- the oct-tree, its groups and the interaction lists built
// on the GPU from particles already in device memory.
//
// The construction is the host builder's (Kodama & Ishiyama, Sec. 1 for
// the tree, Sec. 3.4 for the groups and their shared lists), step by step,
// so that cells, moments, groups and lists come out identical:
//   1. root cube from the bounding box (or [0, box)^3); for a batch of
//      independent systems one root per system from that system's box;
//   2. a 63-bit key per particle by descending 21 levels (upper half along
//      an axis iff the coordinate is >= the cell centre), then a stable
//      radix sort by key (ties keep input order), segmented by system;
//   3. cells breadth-first, one level per pass: a cell with more than nleaf
//      particles above depth 21 gets one child per non-empty octant, found
//      by binary search in the sorted keys; children are numbered in the
//      order of their parents, then octants (the host's breadth-first ids);
//      particles inside a leaf return to input order; a batch's cells are
//      then renumbered system by system (each system's cells breadth first,
//      the host's concatenation of independently built systems);
//   4. moments: leaves from their particles, parents from their children
//      by the parallel-axis shift, deepest level first;
//   5. groups: the largest cells with at most ncrit particles (or leaves),
//      in depth-first order, which is the order of their first particle;
//   6. lists: eight lanes per group walk the tree depth first (children in
//      octant order, all children of an opened cell classified at once),
//      once to count and once to fill.  A cell that does not
//      contain the group is accepted iff side^2 < theta^2 d^2 (d: its
//      centre of mass to the group cube; minimum image in a periodic box,
//      where cells farther than rcut from the group are skipped, and
//      accepted cells whose centre of mass lies at least rcut (1 + 2^-16)
//      from the bounding box of the group's particles are left out: beyond
//      the cutoff for every particle of the group).
// Every floating-point decision (key digits, acceptance) and every moment
// is computed with the host builder's operations in the same order, with
// no contraction into fused multiply-adds, so the results agree bit for
// bit.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>

#include "bhq.h"
#include "bhq_internal.h"

#pragma clang fp contract(off)

namespace bhq {

namespace {

constexpr int kMaxDepth = 21;
constexpr int kFrames = kMaxDepth + 1;  // walk stack: root + one per depth
constexpr int kWalkBlock = 128;             // walk: 16 groups of 8 lanes per block
constexpr int kOct = 8;                     // lanes per group in the walk
constexpr int kXcds = 8;                    // XCDs of the chip
// walk grid: a multiple of kXcds blocks covering ng groups
inline unsigned walk_blocks(int64_t ng)
{
    const int64_t b = (ng + kWalkBlock / kOct - 1) / (kWalkBlock / kOct);
    return (unsigned)((b + kXcds - 1) / kXcds * kXcds);
}
constexpr int kBlock = 256;
constexpr int kBboxBlocks = 1024;

// What the walk reads of a cell: geometry and centre of mass (64 B), then
// the links (16 B; nchild in bits 0-7 and depth in bits 8-15 of .w).
struct alignas(64) WCell {
    double cx, cy, cz, side;
    double mx, my, mz;
    uint64_t key;
};
struct alignas(16) WLink {
    int32_t first, count, child0, nd;
};

struct Cells {
    double *cx, *cy, *cz, *side;
    int32_t *first, *count, *child0, *nchild, *parent, *depth, *sys;
    uint64_t *key;
};

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ---- 1. bounding box ------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_bbox_partial(const double *x, int64_t n,
                                                         double *part)
{
    __shared__ double s[6][kBlock];
    double lo[3], hi[3];
    const int64_t start = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t p0 = start < n ? start : 0;  // n >= 1
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = x[3 * p0 + a];
    for (int64_t p = start; p < n; p += stride)
        for (int a = 0; a < 3; ++a) {
            const double v = x[3 * p + a];
            lo[a] = v < lo[a] ? v : lo[a];
            hi[a] = v > hi[a] ? v : hi[a];
        }
    for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = lo[a];
        s[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int a = 0; a < 3; ++a) {
                const double l = s[a][threadIdx.x + h], u = s[3 + a][threadIdx.x + h];
                if (l < s[a][threadIdx.x]) s[a][threadIdx.x] = l;
                if (u > s[3 + a][threadIdx.x]) s[3 + a][threadIdx.x] = u;
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(kBlock) void k_bbox_final(double *part, int nb)
{
    __shared__ double s[6][kBlock];
    for (int a = 0; a < 6; ++a) s[a][threadIdx.x] = part[a];  // block 0
    for (int b = threadIdx.x; b < nb; b += kBlock)
        for (int a = 0; a < 3; ++a) {
            const double l = part[6 * b + a], u = part[6 * b + 3 + a];
            if (l < s[a][threadIdx.x]) s[a][threadIdx.x] = l;
            if (u > s[3 + a][threadIdx.x]) s[3 + a][threadIdx.x] = u;
        }
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int a = 0; a < 3; ++a) {
                const double l = s[a][threadIdx.x + h], u = s[3 + a][threadIdx.x + h];
                if (l < s[a][threadIdx.x]) s[a][threadIdx.x] = l;
                if (u > s[3 + a][threadIdx.x]) s[3 + a][threadIdx.x] = u;
            }
        __syncthreads();
    }
    __syncthreads();
    if (threadIdx.x < 6) part[threadIdx.x] = s[threadIdx.x][0];
}

// Non-finite positions or masses set flag[0]; a softening that is not
// finite and positive sets flag[1] (vector stores of 1).
__global__ __launch_bounds__(kBlock) void k_check_finite(const double *x, const double *m,
                                                         const double *eps2, int64_t n,
                                                         int *flag)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    if (!isfinite(x[3 * p]) || !isfinite(x[3 * p + 1]) || !isfinite(x[3 * p + 2]) ||
        !isfinite(m[p]))
        flag[0] = 1;
    if (eps2 && !(isfinite(eps2[p]) && eps2[p] >= kMinEps2)) flag[1] = 1;
}

// Bounding box of each system of a batch: one block per system.
__global__ __launch_bounds__(kBlock) void k_bbox_sys(const double *x, const int64_t *sys_off,
                                                     double *bb)
{
    __shared__ double sh[6][kBlock];
    const int64_t a = sys_off[blockIdx.x], e = sys_off[blockIdx.x + 1];
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) lo[k] = hi[k] = x[3 * a + k];
    for (int64_t p = a + threadIdx.x; p < e; p += kBlock)
        for (int k = 0; k < 3; ++k) {
            const double v = x[3 * p + k];
            lo[k] = v < lo[k] ? v : lo[k];
            hi[k] = v > hi[k] ? v : hi[k];
        }
    for (int k = 0; k < 3; ++k) {
        sh[k][threadIdx.x] = lo[k];
        sh[3 + k][threadIdx.x] = hi[k];
    }
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 3; ++k) {
                const double l = sh[k][threadIdx.x + h], u = sh[3 + k][threadIdx.x + h];
                if (l < sh[k][threadIdx.x]) sh[k][threadIdx.x] = l;
                if (u > sh[3 + k][threadIdx.x]) sh[3 + k][threadIdx.x] = u;
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) bb[6 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// ---- 2. keys ----------------------------------------------------------------

// roots[4 s .. 4 s + 3] = centre and side of system s's root cube.
__global__ __launch_bounds__(kBlock) void k_keys(const double *x, int64_t n,
                                                 const int64_t *sys_off, int nsys,
                                                 const double *roots, uint64_t *key,
                                                 int32_t *idx)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    int lo = 0, hi = nsys;  // system of p: sys_off[s] <= p < sys_off[s + 1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (sys_off[mid] <= p)
            lo = mid;
        else
            hi = mid;
    }
    const double *rt = roots + 4 * lo;
    const double xp[3] = {x[3 * p], x[3 * p + 1], x[3 * p + 2]};
    double c[3] = {rt[0], rt[1], rt[2]};
    double s = rt[3];
    uint64_t k = 0;
    for (int lev = 0; lev < kMaxDepth; ++lev) {
        const double qd = s * 0.25;
        unsigned o = 0;
        for (int a = 0; a < 3; ++a) {
            if (xp[a] >= c[a]) {
                o |= 1u << a;
                c[a] = c[a] + qd;
            } else {
                c[a] = c[a] - qd;
            }
        }
        k = (k << 3) | o;
        s = s * 0.5;
    }
    key[p] = k;
    idx[p] = (int32_t)p;
}

// ---- 3. cells ----------------------------------------------------------------

__device__ __forceinline__ int32_t lower_bound(const uint64_t *v, int32_t lo, int32_t hi,
                                               uint64_t x)
{
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (v[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Octant boundaries of cell c: b[o] .. b[o+1] holds octant o.
__device__ __forceinline__ void octant_bounds(const uint64_t *skey, const Cells &C,
                                              int32_t c, int sh, int32_t b[9])
{
    const int32_t f = C.first[c], e = f + C.count[c];
    const uint64_t k = C.key[c];
    b[0] = f;
    for (int o = 1; o < 8; ++o) b[o] = lower_bound(skey, b[o - 1], e, k | ((uint64_t)o << sh));
    b[8] = e;
}

// Level passes.  lv[l] is the first cell of level l (level l is cells
// [lv[l], lv[l+1])), in device memory, so that a rebuild can run its levels
// without the host reading their sizes.  A pass covers `bound` >= the
// level's width threads (a host-side upper bound when the width is not
// known there).

// nch[t] = number of children of cell lv[L] + t (0 beyond the level).
// After an overflow (*flag set) the level's cells may be incomplete: they
// are not read, and the level gets no children.
__global__ __launch_bounds__(kBlock) void k_level_count(Cells C, const uint64_t *skey,
                                                        const int32_t *lv, int L, int32_t bound,
                                                        int nleaf, const int *flag, int32_t *nch)
{
    const int32_t t = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (t >= bound) return;
    const int32_t c = lv[L] + t;
    int32_t n = 0;
    if (*flag == 0 && c < lv[L + 1] && C.count[c] > nleaf && C.depth[c] < kMaxDepth) {
        int32_t b[9];
        octant_bounds(skey, C, c, 3 * (kMaxDepth - 1 - C.depth[c]), b);
        for (int o = 0; o < 8; ++o) n += b[o + 1] > b[o];
    }
    nch[t] = n;
}

// Children of level L from the exclusive sums noff of nch; thread 0 sets
// lv[L + 2], the end of level L + 1.  Cells at or beyond `cap` are not
// written: the end is clamped to cap and *flag is set.
__global__ __launch_bounds__(kBlock) void k_level_write(Cells C, const uint64_t *skey, int32_t *lv,
                                                        int L, int32_t bound, const int32_t *nch,
                                                        const int32_t *noff, int32_t cap,
                                                        int *flag)
{
    const int32_t t = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    const int32_t lo = lv[L], hi = lv[L + 1];
    if (t == 0) {
        const int32_t w = hi - lo;
        const int64_t end = w > 0 ? (int64_t)hi + noff[w - 1] + nch[w - 1] : (int64_t)hi;
        lv[L + 2] = end > cap ? cap : (int32_t)end;
        if (end > cap) *flag = 1;
    }
    if (t >= bound) return;
    const int32_t c = lo + t;
    if (c >= hi) return;
    if (nch[t] == 0) return;
    const int32_t child0 = hi + noff[t];
    if ((int64_t)child0 + nch[t] > cap) return;
    const int d = C.depth[c];
    const int sh = 3 * (kMaxDepth - 1 - d);
    int32_t b[9];
    octant_bounds(skey, C, c, sh, b);
    const double qd = C.side[c] * 0.25;
    const double pc[3] = {C.cx[c], C.cy[c], C.cz[c]};
    int32_t j = 0;
    for (int o = 0; o < 8; ++o) {
        if (b[o + 1] <= b[o]) continue;
        const int32_t ch = child0 + j++;
        C.cx[ch] = pc[0] + (((o >> 0) & 1) ? qd : -qd);
        C.cy[ch] = pc[1] + (((o >> 1) & 1) ? qd : -qd);
        C.cz[ch] = pc[2] + (((o >> 2) & 1) ? qd : -qd);
        C.side[ch] = C.side[c] * 0.5;
        C.first[ch] = b[o];
        C.count[ch] = b[o + 1] - b[o];
        C.key[ch] = C.key[c] | ((uint64_t)o << sh);
        C.depth[ch] = d + 1;
        C.child0[ch] = -1;
        C.nchild[ch] = 0;
        C.parent[ch] = c;
        C.sys[ch] = C.sys[c];
    }
    C.child0[c] = child0;
    C.nchild[c] = j;
}

// Leaves put their particles back in input order (insertion sort; a leaf
// holds at most nleaf particles above depth 21, and at depth 21 its
// particles share one key and are already in input order).
__global__ __launch_bounds__(kBlock) void k_leaf_order(Cells C, int32_t ncell, int32_t *idx)
{
    const int32_t c = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (c >= ncell || C.child0[c] >= 0) return;
    const int32_t f = C.first[c], e = f + C.count[c];
    for (int32_t i = f + 1; i < e; ++i) {
        const int32_t v = idx[i];
        int32_t j = i - 1;
        while (j >= f && idx[j] > v) {
            idx[j + 1] = idx[j];
            --j;
        }
        idx[j + 1] = v;
    }
}

// ---- 4. moments ---------------------------------------------------------------

// Moments of a leaf from its particles, in input order (the host's sums, in
// the host's order): mass and centre of mass, then the traceless
// quadrupole and trace about the centre of mass.  P(k) gives particle k's
// (m, x, y, z).  NMAX > 0: n <= NMAX, and the loops are unrolled to NMAX
// (so that P may index registers); 0: plain loops.
template <int NMAX, typename Part>
__device__ __forceinline__ CellRec leaf_moments(int n, const double ctr[3], Part P)
{
    constexpr int kTrip = NMAX > 0 ? NMAX : 1;
    const int trip = NMAX > 0 ? NMAX : n;
    double M = 0.0, s[3] = {0.0, 0.0, 0.0};
#pragma unroll kTrip
    for (int k = 0; k < trip; ++k) {
        if (k >= n) break;
        const double4 q = P(k);
        M += q.x;
        s[0] += q.x * q.y;
        s[1] += q.x * q.z;
        s[2] += q.x * q.w;
    }
    double cm[3];
    for (int a = 0; a < 3; ++a) cm[a] = M > 0.0 ? s[a] / M : ctr[a];
    double q6[6] = {0, 0, 0, 0, 0, 0}, T = 0.0;
#pragma unroll kTrip
    for (int k = 0; k < trip; ++k) {
        if (k >= n) break;
        const double4 q = P(k);
        const double mp = q.x;
        const double d0 = q.y - cm[0], d1 = q.z - cm[1], d2 = q.w - cm[2];
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        q6[0] += mp * (3.0 * d0 * d0 - r2);
        q6[1] += mp * 3.0 * d0 * d1;
        q6[2] += mp * 3.0 * d0 * d2;
        q6[3] += mp * (3.0 * d1 * d1 - r2);
        q6[4] += mp * 3.0 * d1 * d2;
        q6[5] += mp * (3.0 * d2 * d2 - r2);
        T += mp * r2;
    }
    CellRec r;
    r.x = cm[0];
    r.y = cm[1];
    r.z = cm[2];
    r.m = M;
    r.q00 = q6[0];
    r.q01 = q6[1];
    r.q02 = q6[2];
    r.q11 = q6[3];
    r.q12 = q6[4];
    r.q22 = q6[5];
    r.t = T;
    r.pad = 0.0;
    return r;
}

// One thread per leaf.  A leaf of up to kLeafCache particles loads all of
// them into registers first (independent loads, all in flight at once)
// and sums from there; a larger one (a leaf at the depth limit) reads them
// from memory in each pass.
constexpr int kLeafCache = 8;

__global__ __launch_bounds__(kBlock) void k_moments_leaf(Cells C, int32_t ncell,
                                                         const int32_t *idx, const double *x,
                                                         const double *m, CellRec *pc)
{
    const int32_t c = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (c >= ncell || C.child0[c] >= 0) return;
    const int32_t f = C.first[c], n = C.count[c];
    const double ctr[3] = {C.cx[c], C.cy[c], C.cz[c]};
    auto mem = [&](int k) {
        const int64_t p = idx[f + k];
        return make_double4(m[p], x[3 * p], x[3 * p + 1], x[3 * p + 2]);
    };
    if (n <= kLeafCache) {
        double4 q[kLeafCache];
#pragma unroll
        for (int k = 0; k < kLeafCache; ++k)
            if (k < n) q[k] = mem(k);
        pc[c] = leaf_moments<kLeafCache>(n, ctr, [&](int k) { return q[k]; });
    } else {
        pc[c] = leaf_moments<0>(n, ctr, mem);
    }
}

__global__ __launch_bounds__(kBlock) void k_moments_level(Cells C, int32_t lo, int32_t hi,
                                                          CellRec *pc)
{
    const int32_t c = lo + (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (c >= hi || C.child0[c] < 0) return;
    const int32_t c0 = C.child0[c], nc = C.nchild[c];
    double M = 0.0, s[3] = {0.0, 0.0, 0.0};
    for (int32_t k = 0; k < nc; ++k) {
        const CellRec &h = pc[c0 + k];
        M += h.m;
        s[0] += h.m * h.x;
        s[1] += h.m * h.y;
        s[2] += h.m * h.z;
    }
    const double ctr[3] = {C.cx[c], C.cy[c], C.cz[c]};
    double cm[3];
    for (int a = 0; a < 3; ++a) cm[a] = M > 0.0 ? s[a] / M : ctr[a];
    double q6[6] = {0, 0, 0, 0, 0, 0}, T = 0.0;
    for (int32_t k = 0; k < nc; ++k) {
        const CellRec &h = pc[c0 + k];
        const double Mc = h.m;
        const double D[3] = {h.x - cm[0], h.y - cm[1], h.z - cm[2]};
        const double D2 = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
        q6[0] += h.q00 + Mc * (3.0 * D[0] * D[0] - D2);
        q6[1] += h.q01 + Mc * 3.0 * D[0] * D[1];
        q6[2] += h.q02 + Mc * 3.0 * D[0] * D[2];
        q6[3] += h.q11 + Mc * (3.0 * D[1] * D[1] - D2);
        q6[4] += h.q12 + Mc * 3.0 * D[1] * D[2];
        q6[5] += h.q22 + Mc * (3.0 * D[2] * D[2] - D2);
        T += h.t + Mc * D2;
    }
    CellRec r;
    r.x = cm[0];
    r.y = cm[1];
    r.z = cm[2];
    r.m = M;
    r.q00 = q6[0];
    r.q01 = q6[1];
    r.q02 = q6[2];
    r.q11 = q6[3];
    r.q12 = q6[4];
    r.q22 = q6[5];
    r.t = T;
    r.pad = 0.0;
    pc[c] = r;
}

// ---- 5. groups ----------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t *v, int64_t n, int32_t val)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < n) v[k] = val;
}

// A cell is a group iff it has at most ncrit particles or is a leaf, and
// its parent (if any) has more than ncrit.  gstart[first] = cell id.
__global__ __launch_bounds__(kBlock) void k_group_mark(Cells C, int32_t ncell, int ncrit,
                                                       int32_t *gstart)
{
    const int32_t c = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (c >= ncell) return;
    const bool cond = C.count[c] <= ncrit || C.child0[c] < 0;
    const bool top = C.parent[c] < 0 || C.count[C.parent[c]] > ncrit;
    if (cond && top) gstart[C.first[c]] = c;
}

struct NonNegative {
    __host__ __device__ bool operator()(const int32_t &v) const { return v >= 0; }
};

// ---- 6. walk -----------------------------------------------------------------

// |v - box rint(v / box)|, the distance to the nearest periodic image (|v|
// without a box).  For |v| < box / 4 the quotient rounds to below 1/2, rint
// gives 0 and the result is |v|: the division, a long instruction sequence
// in FP64, is taken only for the far cells.
__device__ __forceinline__ double abs_min_image(double v, double box)
{
    const double a = ::fabs(v);
    if (box > 0.0 && !(a < 0.25 * box)) return ::fabs(v - box * ::rint(v / box));
    return a;
}

__device__ __forceinline__ bool contains(uint64_t ckey, int cdepth, uint64_t gkey,
                                         int gdepth)
{
    if (cdepth > gdepth) return false;
    const int sh = 3 * (kMaxDepth - cdepth);
    if (sh >= 64) return true;
    return (ckey >> sh) == (gkey >> sh);
}

__global__ __launch_bounds__(kBlock) void k_walk_cells(Cells C, int32_t ncell,
                                                       const CellRec *pc, WCell *wc,
                                                       WLink *wl)
{
    const int32_t c = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (c >= ncell) return;
    WCell w;
    w.cx = C.cx[c];
    w.cy = C.cy[c];
    w.cz = C.cz[c];
    w.side = C.side[c];
    w.mx = pc[c].x;
    w.my = pc[c].y;
    w.mz = pc[c].z;
    w.key = C.key[c];
    wc[c] = w;
    WLink l;
    l.first = C.first[c];
    l.count = C.count[c];
    l.child0 = C.child0[c];
    l.nd = C.nchild[c] | (C.depth[c] << 8);
    wl[c] = l;
}

struct WalkArgs {
    const int32_t *groups;
    const int32_t *cell_sys;           // system of each cell
    const int32_t *sys_root;           // root cell of each system
    int64_t ng;
    const WCell *wc;
    const WLink *wl;
    double theta2, rcut, box;
    double rdrop2;                     // accepted cells this far (squared) from the
                                       // box of the group's particles are beyond the
                                       // cutoff for all of them and left out; 0: no
                                       // cutoff
    int64_t *jp_cnt, *jc_cnt;          // count pass
    const int64_t *jp_off, *jc_off;    // fill pass
    int32_t *jp_idx, *jc_idx;
    int *flag;                         // set if a stack would overflow
    int64_t cap_p, cap_c;              // slot sizes of the one-walk mode
    int frames;                        // frame stack depth: levels of the tree
    const double *gbox;                // [6 ng] lo, hi of each group's particles
                                       // (with a cutoff)
};

// A child of an opened cell, as the walk classifies it, in two ints:
//   skipped (beyond the cutoff)         {-1, 0}
//   j-cell id                           {id, 0}
//   particles first .. first + count-1  {first, count}, count >= 1 (an
//                                        accepted one-particle cell or an
//                                        opened leaf)
//   opened internal cell                {-2 - child0, nchild}
__device__ __forceinline__ int2 classify(const WalkArgs &W, int32_t id, const WCell &G,
                                         int gdepth, const double *gb)
{
    const WCell C = W.wc[id];
    const WLink L = W.wl[id];
    const int cdepth = L.nd >> 8;
    const double box = W.box;
    const double gc[3] = {G.cx, G.cy, G.cz};
    if (!contains(C.key, cdepth, G.key, gdepth)) {
        if (W.rcut > 0.0) {
            const double cc[3] = {C.cx, C.cy, C.cz};
            double d2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double v = abs_min_image(cc[k] - gc[k], box) -
                                 0.5 * (C.side + G.side);
                if (v > 0.0) d2 += v * v;
            }
            if (d2 > W.rcut * W.rcut) return make_int2(-1, 0);
        }
        const double cm[3] = {C.mx, C.my, C.mz};
        double d2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double v = abs_min_image(cm[k] - gc[k], box) - 0.5 * G.side;
            if (v > 0.0) d2 += v * v;
        }
        if (C.side * C.side < W.theta2 * d2) {
            // beyond the cutoff for every particle of the group
            if (W.rdrop2 > 0.0) {
                // distance to the box of the group's particles (centre
                // gb[0..2], half widths gb[3..5])
                double b2 = 0.0;
                for (int k = 0; k < 3; ++k) {
                    const double v = abs_min_image(cm[k] - gb[k], box) - gb[3 + k];
                    if (v > 0.0) b2 += v * v;
                }
                if (b2 >= W.rdrop2) return make_int2(-1, 0);
            }
            return L.count == 1 ? make_int2(L.first, 1) : make_int2(id, 0);
        }
    }
    if (L.child0 < 0) return L.count > 0 ? make_int2(L.first, L.count) : make_int2(-1, 0);
    return make_int2(-2 - L.child0, L.nd & 0xff);
}

// Data movement inside an octet (8 aligned lanes) by DPP, on the VALU:
// an inclusive prefix sum and a sum returned to every lane.  DPP works in
// rows of 16 lanes, which hold two octets; every read below stays inside
// the reading lane's octet (row_shr by d is used only by lanes k >= d).
template <int CTRL>
__device__ __forceinline__ int dpp(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}

__device__ __forceinline__ int octet_scan(int v, int k)
{
    int u = dpp<0x111>(v);  // row_shr:1
    v += k >= 1 ? u : 0;
    u = dpp<0x112>(v);      // row_shr:2
    v += k >= 2 ? u : 0;
    u = dpp<0x114>(v);      // row_shr:4
    v += k >= 4 ? u : 0;
    return v;
}

__device__ __forceinline__ int octet_sum(int v)
{
    v += dpp<0x141>(v);  // row_half_mirror: lane 7 - k of the octet
    v += dpp<0xB1>(v);   // quad_perm [1, 0, 3, 2]: lane k ^ 1
    v += dpp<0x4E>(v);   // quad_perm [2, 3, 0, 1]: lane k ^ 2
    return v;
}

// Octet walk: the 8 lanes of an octet walk one group.  Opening an internal
// cell loads and classifies all of its children at once, one per lane, and
// pushes them as a frame; a frame is emitted in octant order up to its next
// opened internal child, whose subtree is walked before the rest of the
// frame.  The lists therefore come out in the depth-first, octant order of
// the host builder's walk, while the chain of dependent loads per group is
// one per opened cell instead of one per visited cell.  The current frame
// lives in registers; each lane keeps its child's entry of every frame in
// LDS for the return from a subtree, and the frame's child count and cursor
// are stored once per octet, written by all 8 lanes with the same value.
// Control flow is uniform within an octet.  The fill pass writes only
// inside the group's own segments of the lists.
// Walk modes: count the entries; fill the lists at exact offsets; or fill
// fixed slots of cap_p / cap_c entries per group and count (one walk).
enum WalkMode { kWalkCount = 0, kWalkFill = 1, kWalkSlots = 2 };

template <int MODE>
__global__ __launch_bounds__(kWalkBlock) void k_walk(const WalkArgs W)
{
    // frame stack, W.frames deep (the tree's depth): a child entry per lane,
    // then nchild | cursor << 8 per octet (dynamic LDS: a shallow tree
    // leaves room for more resident waves)
    extern __shared__ int2 s_walk[];
    int2 (*s_ent)[kWalkBlock] = reinterpret_cast<int2 (*)[kWalkBlock]>(s_walk);
    int32_t (*s_hdr)[kWalkBlock / kOct] = reinterpret_cast<int32_t (*)[kWalkBlock / kOct]>(
        s_walk + (size_t)W.frames * kWalkBlock);
    const int t = threadIdx.x;
    const int k = t & (kOct - 1);
    const int o = t / kOct;
    // The hardware hands blocks to the XCDs round robin; XCD x walks the
    // contiguous range of groups [x per, (x + 1) per) of blocks, so that
    // neighbouring groups, whose walks read the same cells, share an L2.
    const unsigned per = gridDim.x / kXcds;
    const unsigned lb = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    const int64_t gi = (int64_t)lb * (kWalkBlock / kOct) + o;
    if (gi >= W.ng) return;  // whole octets leave; no block-wide synchronisation below
    const int32_t gid = W.groups[gi];
    const WCell G = W.wc[gid];
    const int gdepth = W.wl[gid].nd >> 8;
    // centre and half widths of the box (lo, hi) of the group's particles,
    // with the host builder's operations
    double gb[6] = {0, 0, 0, 0, 0, 0};
    if (W.rdrop2 > 0.0)
        for (int k = 0; k < 3; ++k) {
            const double lo = W.gbox[6 * gi + k], hi = W.gbox[6 * gi + 3 + k];
            gb[k] = 0.5 * (lo + hi);
            gb[3 + k] = 0.5 * (hi - lo);
        }
    int64_t np = 0, nc = 0;
    constexpr bool FILL = MODE != kWalkCount;
    int64_t pb = 0, cb = 0, pe = 0, ce = 0;  // where this group's entries go
    if (MODE == kWalkFill) {
        pb = W.jp_off[gi];
        cb = W.jc_off[gi];
        pe = W.jp_off[gi + 1];
        ce = W.jc_off[gi + 1];
    } else if (MODE == kWalkSlots) {
        pb = gi * W.cap_p;
        cb = gi * W.cap_c;
        pe = pb + W.cap_p;
        ce = cb + W.cap_c;
    }
    const int32_t root = W.sys_root[W.cell_sys[gid]];
    const WLink R = W.wl[root];
    int sp = 0, nch = 0, cur = 0;
    int2 e = make_int2(-1, 0);
    if (R.child0 < 0) {
        // a one-leaf tree: the root contains the group and is opened
        if (FILL)
            for (int32_t j = k; j < R.count && pb + j < pe; j += kOct)
                W.jp_idx[pb + j] = R.first + j;
        np = R.count;
    } else {
        nch = R.nd & 0xff;
        e = k < nch ? classify(W, R.child0 + k, G, gdepth, gb) : make_int2(-1, 0);
        s_ent[0][t] = e;
        sp = 1;
    }
    // Each round: emit and return from frames (cheap) until the octet must
    // open a child or is done, then open it (loads and classification).
    // Octets of a wave reach their next opening at different steps; taking
    // the openings in a round of their own lets the expensive part run for
    // all octets of the wave together.
    while (sp > 0) {
        int32_t c0 = 0;
        int n2 = -1;  // >= 0: open the cell whose children are c0 .. c0 + n2 - 1
        for (;;) {
            const bool mine = k >= cur && k < nch;
            // the first opened internal child at or after the cursor
            const uint64_t bal = __ballot(mine && e.x <= -2);
            const uint32_t om = (uint32_t)(bal >> (t & 63 & ~(kOct - 1))) & 0xffu;
            const int kstar = om ? __builtin_ctz(om) : nch;
            // emit the children before it
            const bool em = mine && k < kstar && e.x >= 0;
            const int vp = em ? e.y : 0;            // particles
            const int vc = em && e.y == 0 ? 1 : 0;  // cells
            if (FILL) {
                const int ip = octet_scan(vp, k), ic = octet_scan(vc, k);
                if (em) {
                    if (e.y == 0) {
                        const int64_t q = cb + nc + ic - 1;
                        if (q < ce) W.jc_idx[q] = e.x;
                    } else {
                        // the entries that fit in the group's segment (none
                        // past it: a slot overflow is detected from the counts)
                        const int64_t q = pb + np + ip - e.y;
                        const int32_t nw = (int32_t)(pe - q < (int64_t)e.y ? pe - q : e.y);
                        int32_t *dst = W.jp_idx + q;
                        for (int32_t j = 0; j < nw; ++j) dst[j] = e.x + j;
                    }
                }
            }
            np += octet_sum(vp);
            nc += octet_sum(vc);
            if (kstar < nch) {
                // descend into child kstar; this frame resumes after it
                c0 = -2 - __shfl(e.x, kstar, kOct);
                const int n = __shfl(e.y, kstar, kOct);
                cur = kstar + 1;
                if (sp < W.frames) {
                    s_hdr[sp - 1][o] = nch | cur << 8;
                    n2 = n;
                    break;
                }
                if (k == 0) *W.flag = 1;  // the subtree is left out; the build fails
                continue;
            }
            if (--sp == 0) break;
            e = s_ent[sp - 1][t];
            const int hdr = s_hdr[sp - 1][o];
            nch = hdr & 0xff;
            cur = hdr >> 8;
        }
        if (n2 < 0) break;
        e = k < n2 ? classify(W, c0 + k, G, gdepth, gb) : make_int2(-1, 0);
        s_ent[sp][t] = e;
        nch = n2;
        cur = 0;
        ++sp;
    }
    if (MODE != kWalkFill && k == 0) {
        W.jp_cnt[gi] = np;
        W.jc_cnt[gi] = nc;
    }
}

// Bounding box (lo[3], hi[3]) of each group's particles, for the cutoff
// drop; one thread per group over its particles in tree order.
__global__ __launch_bounds__(kBlock) void k_group_box(Cells C, const int32_t *groups,
                                                      int64_t ng, const int32_t *idx,
                                                      const double *x, double *gbox)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= ng) return;
    const int32_t c = groups[g];
    double b[6];
    for (int k = 0; k < 3; ++k) {
        b[k] = __builtin_inf();
        b[3 + k] = -__builtin_inf();
    }
    // chunks of 8 particles: their loads are independent and all in flight
    // at once (minimum and maximum do not depend on the order)
    constexpr int kChunk = 8;
    const int32_t f = C.first[c], e = f + C.count[c];
    for (int32_t q0 = f; q0 < e; q0 += kChunk) {
        double v[kChunk][3];
#pragma unroll
        for (int j = 0; j < kChunk; ++j)
            if (q0 + j < e) {
                const double *xp = x + 3 * (int64_t)idx[q0 + j];
                for (int k = 0; k < 3; ++k) v[j][k] = xp[k];
            }
#pragma unroll
        for (int j = 0; j < kChunk; ++j)
            if (q0 + j < e)
                for (int k = 0; k < 3; ++k) {
                    b[k] = v[j][k] < b[k] ? v[j][k] : b[k];
                    b[3 + k] = v[j][k] > b[3 + k] ? v[j][k] : b[3 + k];
                }
    }
    for (int k = 0; k < 6; ++k) gbox[6 * g + k] = b[k];
}

// Lists of one-walk builds: group g's entries [0, off[g+1] - off[g]) of
// its slot (cap entries from g cap) to out[off[g] ...]; one wave per group.
__global__ __launch_bounds__(kBlock) void k_compact(int64_t ng, const int64_t *off,
                                                    const int32_t *slot, int64_t cap,
                                                    int32_t *out)
{
    const int64_t g = (int64_t)blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
    if (g >= ng) return;
    const int lane = threadIdx.x & 63;
    const int64_t o = off[g], n = off[g + 1] - o;
    const int32_t *src = slot + g * cap;
    for (int64_t j = lane; j < n; j += 64) out[o + j] = src[j];
}

// stats[0], stats[1] = list totals (the scans' last entries), stats[4] =
// the walk's overflow flag; stats[2], stats[3] hold the longest lists.
__global__ void k_list_stats(int64_t ng, const int64_t *jp_off, const int64_t *jc_off,
                             const int *flag, int64_t *stats)
{
    stats[0] = jp_off[ng];
    stats[1] = jc_off[ng];
    stats[4] = *flag;
}

}  // namespace

hipError_t launch_compact_lists(int64_t ng, const int64_t *off, const int32_t *slot,
                                int64_t cap, int32_t *out, hipStream_t s)
{
    if (ng <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact, dim3(blocks(ng, kBlock / 64)), dim3(kBlock), 0, s, ng, off,
                       slot, cap, out);
    return hipGetLastError();
}

namespace {

// ---- outputs -----------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_particles_out(const int32_t *idx, int64_t n,
                                                          const double *x, const double *m,
                                                          const double *eps2, PartRec *pool,
                                                          double *xi, double *yi, double *zi,
                                                          double *e2i)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int64_t p = idx[k];
    if (eps2) e2i[k] = eps2[p];
    PartRec r;
    r.x = x[3 * p];
    r.y = x[3 * p + 1];
    r.z = x[3 * p + 2];
    r.m = m[p];
    pool[k] = r;
    xi[k] = r.x;
    yi[k] = r.y;
    zi[k] = r.z;
}

__global__ __launch_bounds__(kBlock) void k_groups_out(Cells C, const int32_t *groups,
                                                       int64_t ng, int64_t n, int64_t *i_off,
                                                       double *gcx, double *gcy, double *gcz)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g > ng) return;
    if (g == ng) {
        i_off[ng] = n;
        return;
    }
    const int32_t c = groups[g];
    i_off[g] = C.first[c];
    gcx[g] = C.cx[c];
    gcy[g] = C.cy[c];
    gcz[g] = C.cz[c];
}

__global__ __launch_bounds__(kBlock) void k_set_roots(Cells C, const double *roots,
                                                      const int64_t *sys_off, int nsys)
{
    const int sidx = blockIdx.x * kBlock + threadIdx.x;
    if (sidx >= nsys) return;
    C.cx[sidx] = roots[4 * sidx];
    C.cy[sidx] = roots[4 * sidx + 1];
    C.cz[sidx] = roots[4 * sidx + 2];
    C.side[sidx] = roots[4 * sidx + 3];
    C.first[sidx] = (int32_t)sys_off[sidx];
    C.count[sidx] = (int32_t)(sys_off[sidx + 1] - sys_off[sidx]);
    C.key[sidx] = 0;
    C.depth[sidx] = 0;
    C.child0[sidx] = -1;
    C.nchild[sidx] = 0;
    C.parent[sidx] = -1;
    C.sys[sidx] = sidx;
}

// Cells per (depth, system), for the renumbering of a batch.
__global__ __launch_bounds__(kBlock) void k_level_sys_count(Cells C, int32_t ncell, int nsys,
                                                            int32_t *cnt)
{
    const int32_t c = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (c >= ncell) return;
    atomicAdd(cnt + C.depth[c] * nsys + C.sys[c], 1);
}

// New id of cell c: base[l][s] + (c - first[l][s]) for its depth l and
// system s (device cells of one depth are ordered by system).
__global__ __launch_bounds__(kBlock) void k_perm(Cells C, int32_t ncell, int nsys,
                                                 const int32_t *base, const int32_t *first,
                                                 int32_t *perm)
{
    const int32_t c = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (c >= ncell) return;
    const int t = C.depth[c] * nsys + C.sys[c];
    perm[c] = base[t] + (c - first[t]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_permute(int32_t ncell, const int32_t *perm,
                                                    const T *in, T *out, bool ids)
{
    const int32_t c = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (c >= ncell) return;
    T v = in[c];
    if constexpr (sizeof(T) == 4) {
        if (ids && v >= 0) v = perm[v];
    }
    out[perm[c]] = v;
}

}  // namespace

// ---- host orchestration ---------------------------------------------------------

int build_tree_lists(const TreeParams &P, TreeOut &O, hipStream_t s, std::string *err)
{
    DevArray *B = O.buf;
    const int64_t n = P.n;
    int code = BHQ_OK;
    const char *what = "";
    auto hip = [&](hipError_t e, const char *w) -> bool {
        if (e == hipSuccess) return true;
        code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? BHQ_E_NOMEM
                                                                            : BHQ_E_HIP;
        what = w;
        return false;
    };
    auto fail = [&]() -> int {
        if (err) {
            *err = std::string("device list build: ") + what;
            if (code == BHQ_E_HIP || code == BHQ_E_NOMEM)
                *err += std::string(" (") + hipGetErrorString(hipGetLastError()) + ")";
        }
        return code;
    };
#define STEP(expr, w)              \
    do {                           \
        if (!hip((expr), (w))) return fail(); \
    } while (0)
#define LAUNCHED(w) STEP(hipGetLastError(), w)

    // input check, systems, root cubes
    const int nsys = (int)P.nsys;
    STEP(B[T_FLAG].reserve(64), "allocation");
    STEP(hipMemsetAsync(B[T_FLAG].p, 0, 64, s), "memset");
    hipLaunchKernelGGL(k_check_finite, dim3(blocks(n, kBlock)), dim3(kBlock), 0, s, P.x, P.m,
                       P.eps2, n, B[T_FLAG].as<int>());
    LAUNCHED("finite check");
    int hflag2[2] = {0, 0};
    STEP(hipMemcpyAsync(hflag2, B[T_FLAG].p, sizeof(hflag2), hipMemcpyDeviceToHost, s), "copy");
    STEP(hipStreamSynchronize(s), "sync");
    if (hflag2[0]) {
        code = BHQ_E_NONFINITE;
        what = "non-finite position or mass";
        return fail();
    }
    if (hflag2[1]) {
        code = BHQ_E_ARG;
        what = "eps2 must be finite and >= 2^-126";
        return fail();
    }
    STEP(B[T_SYSOFF].reserve((size_t)(nsys + 1) * 8), "allocation");
    STEP(B[T_SYSOFF32].reserve((size_t)(nsys + 1) * 4), "allocation");
    STEP(hipMemcpyAsync(B[T_SYSOFF].p, P.sys_off, (size_t)(nsys + 1) * 8,
                        hipMemcpyHostToDevice, s),
         "copy");
    std::vector<double> roots((size_t)nsys * 4);
    {
        std::vector<int32_t> so32((size_t)nsys + 1);
        for (int k = 0; k <= nsys; ++k) so32[(size_t)k] = (int32_t)P.sys_off[k];
        STEP(hipMemcpyAsync(B[T_SYSOFF32].p, so32.data(), (size_t)(nsys + 1) * 4,
                            hipMemcpyHostToDevice, s),
             "copy");
        std::vector<double> bb((size_t)nsys * 6);
        if (P.box > 0.0) {
            for (int k = 0; k < 3; ++k) roots[(size_t)k] = 0.5 * P.box;
            roots[3] = P.box;
        } else {
            if (nsys == 1) {
                const int nb = (int)std::min<int64_t>(kBboxBlocks, blocks(n, kBlock));
                STEP(B[T_BBOX].reserve((size_t)nb * 6 * sizeof(double)), "allocation");
                hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(kBlock), 0, s, P.x, n,
                                   B[T_BBOX].as<double>());
                LAUNCHED("bounding box");
                hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(kBlock), 0, s,
                                   B[T_BBOX].as<double>(), nb);
                LAUNCHED("bounding box");
            } else {
                STEP(B[T_BBOX].reserve((size_t)nsys * 6 * sizeof(double)), "allocation");
                hipLaunchKernelGGL(k_bbox_sys, dim3((unsigned)nsys), dim3(kBlock), 0, s, P.x,
                                   B[T_SYSOFF].as<int64_t>(), B[T_BBOX].as<double>());
                LAUNCHED("bounding boxes");
            }
            STEP(hipMemcpyAsync(bb.data(), B[T_BBOX].p, bb.size() * sizeof(double),
                                hipMemcpyDeviceToHost, s),
                 "copy");
            STEP(hipStreamSynchronize(s), "sync");
            for (int q = 0; q < nsys; ++q) {
                const double *b = &bb[(size_t)q * 6];
                double *rt = &roots[(size_t)q * 4];
                double ext = 0.0;
                for (int k = 0; k < 3; ++k) {
                    rt[k] = 0.5 * (b[k] + b[3 + k]);
                    ext = std::max(ext, b[3 + k] - b[k]);
                }
                rt[3] = ext > 0.0 ? ext * (1.0 + std::ldexp(1.0, -20)) : 1.0;
            }
        }
        STEP(B[T_ROOTS].reserve(roots.size() * sizeof(double)), "allocation");
        STEP(hipMemcpyAsync(B[T_ROOTS].p, roots.data(), roots.size() * sizeof(double),
                            hipMemcpyHostToDevice, s),
             "copy");
        STEP(hipStreamSynchronize(s), "sync");
    }

    // keys, sort
    STEP(B[T_KEY].reserve((size_t)n * 8), "allocation");
    STEP(B[T_KEY2].reserve((size_t)n * 8), "allocation");
    STEP(B[T_IDX0].reserve((size_t)n * 4), "allocation");
    STEP(O.order->reserve((size_t)n * 4), "allocation");
    hipLaunchKernelGGL(k_keys, dim3(blocks(n, kBlock)), dim3(kBlock), 0, s, P.x, n,
                       B[T_SYSOFF].as<int64_t>(), nsys, B[T_ROOTS].as<double>(),
                       B[T_KEY].as<uint64_t>(), B[T_IDX0].as<int32_t>());
    LAUNCHED("keys");
    // Stable sort of (key, input index) on key bits [lo_bit, 63).  Splitting
    // a cell at depth d reads the key digit at bits 3 (kMaxDepth - 1 - d),
    // so a tree of L levels needs the bits from 3 (kMaxDepth + 1 - L) up;
    // the order inside a leaf does not matter (leaves are put back in input
    // order).  A rebuild sorts the bits its previous depth needs; if the tree
    // turns out deeper, the keys are sorted again on all bits.
    auto sort_keys = [&](int lo_bit) -> bool {
        size_t tmp = 0;
        if (nsys == 1) {
            if (!hip(hipcub::DeviceRadixSort::SortPairs(
                         nullptr, tmp, B[T_KEY].as<uint64_t>(), B[T_KEY2].as<uint64_t>(),
                         B[T_IDX0].as<int32_t>(), O.order->as<int32_t>(), (int)n, lo_bit,
                         3 * kMaxDepth, s),
                     "sort size"))
                return false;
            if (!hip(B[T_SORT].reserve(std::max(tmp, B[T_SORT].cap)), "allocation")) return false;
            return hip(hipcub::DeviceRadixSort::SortPairs(
                           B[T_SORT].p, tmp, B[T_KEY].as<uint64_t>(), B[T_KEY2].as<uint64_t>(),
                           B[T_IDX0].as<int32_t>(), O.order->as<int32_t>(), (int)n, lo_bit,
                           3 * kMaxDepth, s),
                       "sort");
        }
        const int32_t *so = B[T_SYSOFF32].as<int32_t>();
        if (!hip(hipcub::DeviceSegmentedRadixSort::SortPairs(
                     nullptr, tmp, B[T_KEY].as<uint64_t>(), B[T_KEY2].as<uint64_t>(),
                     B[T_IDX0].as<int32_t>(), O.order->as<int32_t>(), (int)n, nsys, so, so + 1,
                     lo_bit, 3 * kMaxDepth, s),
                 "sort size"))
            return false;
        if (!hip(B[T_SORT].reserve(std::max(tmp, B[T_SORT].cap)), "allocation")) return false;
        return hip(hipcub::DeviceSegmentedRadixSort::SortPairs(
                       B[T_SORT].p, tmp, B[T_KEY].as<uint64_t>(), B[T_KEY2].as<uint64_t>(),
                       B[T_IDX0].as<int32_t>(), O.order->as<int32_t>(), (int)n, nsys, so,
                       so + 1, lo_bit, 3 * kMaxDepth, s),
                   "sort");
    };
    const bool spec = P.spec_levels > 0 && P.spec_cells > 0;
    const int sort_lo = spec ? 3 * std::max(0, kMaxDepth + 1 - P.spec_levels) : 0;
    if (!sort_keys(sort_lo)) return fail();
    const uint64_t *skey = B[T_KEY2].as<uint64_t>();
    int32_t *idx = O.order->as<int32_t>();

    // cells, level by level
    size_t cap = B[T_CX].p ? B[T_CX].cap / 8 : 0;
    const TreeBuf cbuf8[] = {T_CX, T_CY, T_CZ, T_SIDE, T_CKEY};
    const TreeBuf cbuf4[] = {T_FIRST, T_COUNT, T_CHILD0, T_NCHILD, T_PARENT, T_DEPTH, T_CSYS};
    auto cells = [&]() {
        Cells C;
        C.cx = B[T_CX].as<double>();
        C.cy = B[T_CY].as<double>();
        C.cz = B[T_CZ].as<double>();
        C.side = B[T_SIDE].as<double>();
        C.key = B[T_CKEY].as<uint64_t>();
        C.first = B[T_FIRST].as<int32_t>();
        C.count = B[T_COUNT].as<int32_t>();
        C.child0 = B[T_CHILD0].as<int32_t>();
        C.nchild = B[T_NCHILD].as<int32_t>();
        C.parent = B[T_PARENT].as<int32_t>();
        C.depth = B[T_DEPTH].as<int32_t>();
        C.sys = B[T_CSYS].as<int32_t>();
        return C;
    };
    auto ensure = [&](size_t need, size_t used) -> bool {
        if (need <= cap) return true;
        size_t nc = std::max(need, cap + cap / 2);
        for (TreeBuf b : cbuf8)
            if (!hip(B[b].grow(nc * 8, used * 8, s), "allocation")) return false;
        for (TreeBuf b : cbuf4)
            if (!hip(B[b].grow(nc * 4, used * 4, s), "allocation")) return false;
        cap = nc;
        return true;
    };
    if (!ensure((size_t)std::max<int64_t>(std::max<int64_t>(1024, n / 2), 2 * nsys), 0))
        return fail();
    hipLaunchKernelGGL(k_set_roots, dim3(blocks(nsys, kBlock)), dim3(kBlock), 0, s, cells(),
                       B[T_ROOTS].as<double>(), B[T_SYSOFF].as<int64_t>(), nsys);
    LAUNCHED("roots");
    std::vector<int32_t> level{0, nsys};  // level l is cells [level[l], level[l+1])
    STEP(B[T_NCH].reserve((size_t)std::max<int64_t>(n, 1) * 4 + 4), "allocation");
    STEP(B[T_NOFF].reserve((size_t)std::max<int64_t>(n, 1) * 4 + 4), "allocation");
    // level bounds on the device (kMaxDepth + 2 entries), then a flag
    STEP(B[T_LV].reserve((size_t)(kMaxDepth + 3) * 4), "allocation");
    int32_t *lv = B[T_LV].as<int32_t>();
    int *lvflag = reinterpret_cast<int *>(lv + kMaxDepth + 2);
    {
        const int32_t init[3] = {0, nsys, 0};
        STEP(hipMemcpyAsync(lv, init, 8, hipMemcpyHostToDevice, s), "copy");
        STEP(hipMemcpyAsync(lvflag, init + 2, 4, hipMemcpyHostToDevice, s), "copy");
    }
    auto scan = [&](int32_t bound) -> bool {
        size_t st = 0;
        if (!hip(hipcub::DeviceScan::ExclusiveSum(nullptr, st, B[T_NCH].as<int32_t>(),
                                                  B[T_NOFF].as<int32_t>(), bound, s),
                 "scan size"))
            return false;
        if (!hip(B[T_SORT].reserve(std::max(st, B[T_SORT].cap)), "allocation")) return false;
        return hip(hipcub::DeviceScan::ExclusiveSum(B[T_SORT].p, st, B[T_NCH].as<int32_t>(),
                                                    B[T_NOFF].as<int32_t>(), bound, s),
                   "scan");
    };
    auto level_pass = [&](int lev, int32_t bound) -> bool {
        hipLaunchKernelGGL(k_level_count, dim3(blocks(bound, kBlock)), dim3(kBlock), 0, s,
                           cells(), skey, (const int32_t *)lv, lev, bound, P.nleaf,
                           (const int *)lvflag, B[T_NCH].as<int32_t>());
        if (!hip(hipGetLastError(), "level count")) return false;
        if (!scan(bound)) return false;
        hipLaunchKernelGGL(k_level_write, dim3(blocks(bound, kBlock)), dim3(kBlock), 0, s,
                           cells(), skey, lv, lev, bound, B[T_NCH].as<int32_t>(),
                           B[T_NOFF].as<int32_t>(),
                           (int32_t)std::min<size_t>(cap, 0x7fffffff), lvflag);
        return hip(hipGetLastError(), "level write");
    };
    // A rebuild first runs as many levels as the previous build had with no
    // host synchronisation: widths bounded by 8 times the level above and by
    // n, cells by a capacity of 1.25 times the previous build's.  If the
    // cells overflow, the levels are built again below, one at a time; if
    // the tree goes deeper, the remaining levels are built that way.
    bool done = false;
    if (spec) {
        const size_t want = (size_t)P.spec_cells + (size_t)P.spec_cells / 4 + 1024;
        if (!ensure(std::min<size_t>(want, 0x7fffffff), (size_t)nsys)) return fail();
        const int nl = std::min(P.spec_levels, kMaxDepth);
        int64_t bound = nsys;
        for (int lev = 0; lev < nl; ++lev) {
            if (!level_pass(lev, (int32_t)bound)) return fail();
            bound = std::min<int64_t>(8 * bound, n);
        }
        std::vector<int32_t> hl((size_t)kMaxDepth + 3);
        STEP(hipMemcpyAsync(hl.data(), lv, hl.size() * 4, hipMemcpyDeviceToHost, s), "copy");
        STEP(hipStreamSynchronize(s), "sync");
        if (hl[(size_t)kMaxDepth + 2] == 0) {
            for (int lev = 0; lev < nl; ++lev) {
                const int32_t e = hl[(size_t)lev + 2];
                if (e == level.back()) {  // level lev + 1 is empty: the tree ends
                    done = true;
                    break;
                }
                level.push_back(e);
            }
        }
        if (!done) {
            // the cells overflowed, or the tree is deeper than the sorted
            // bits reach: sort on all bits and start again, level by level
            level.assign({0, nsys});
            if (sort_lo > 0 && !sort_keys(0)) return fail();
            const int32_t zero = 0;
            STEP(hipMemcpyAsync(lvflag, &zero, 4, hipMemcpyHostToDevice, s), "copy");
            STEP(hipStreamSynchronize(s), "sync");
        }
    }
    for (int lev = (int)level.size() - 2; !done && lev < kMaxDepth; ++lev) {
        const int32_t lo = level[(size_t)lev], hi = level[(size_t)lev + 1];
        const int32_t w = hi - lo;
        if (w <= 0) break;
        hipLaunchKernelGGL(k_level_count, dim3(blocks(w, kBlock)), dim3(kBlock), 0, s, cells(),
                           skey, (const int32_t *)lv, lev, w, P.nleaf, (const int *)lvflag,
                           B[T_NCH].as<int32_t>());
        LAUNCHED("level count");
        if (!scan(w)) return fail();
        int32_t tail[2];
        STEP(hipMemcpyAsync(&tail[0], B[T_NOFF].as<int32_t>() + (w - 1), 4,
                            hipMemcpyDeviceToHost, s),
             "copy");
        STEP(hipMemcpyAsync(&tail[1], B[T_NCH].as<int32_t>() + (w - 1), 4,
                            hipMemcpyDeviceToHost, s),
             "copy");
        STEP(hipStreamSynchronize(s), "sync");
        const int64_t total = (int64_t)tail[0] + tail[1];
        if (total == 0) break;
        if ((int64_t)hi + total > 0x7fffffffLL) {
            code = BHQ_E_RANGE;
            what = "more than 2^31 cells";
            return fail();
        }
        if (!ensure((size_t)(hi + total), (size_t)hi)) return fail();
        hipLaunchKernelGGL(k_level_write, dim3(blocks(w, kBlock)), dim3(kBlock), 0, s, cells(),
                           skey, lv, lev, w, B[T_NCH].as<int32_t>(), B[T_NOFF].as<int32_t>(),
                           (int32_t)std::min<size_t>(cap, 0x7fffffff), lvflag);
        LAUNCHED("level write");
        level.push_back((int32_t)(hi + total));
    }
    const int32_t ncell = level.back();
    hipLaunchKernelGGL(k_leaf_order, dim3(blocks(ncell, kBlock)), dim3(kBlock), 0, s, cells(),
                       ncell, idx);
    LAUNCHED("leaf order");

    // moments straight into the cell pool
    STEP(O.pool_c->reserve((size_t)ncell * sizeof(CellRec)), "allocation");
    CellRec *pc = O.pool_c->as<CellRec>();
    hipLaunchKernelGGL(k_moments_leaf, dim3(blocks(ncell, kBlock)), dim3(kBlock), 0, s,
                       cells(), ncell, idx, P.x, P.m, pc);
    LAUNCHED("leaf moments");
    for (int l = (int)level.size() - 2; l >= 0; --l) {
        const int32_t lo = level[(size_t)l], hi = level[(size_t)l + 1];
        hipLaunchKernelGGL(k_moments_level, dim3(blocks(hi - lo, kBlock)), dim3(kBlock), 0, s,
                           cells(), lo, hi, pc);
        LAUNCHED("cell moments");
    }

    // a batch: renumber the cells system by system (each system breadth
    // first), then the walk starts from each group's own root
    std::vector<int32_t> sys_root((size_t)nsys, 0);
    if (nsys > 1) {
        const int nl = (int)level.size() - 1;
        const size_t tab = (size_t)kFrames * nsys;
        STEP(B[T_LSC].reserve(tab * 4 * 3), "allocation");
        int32_t *cnt = B[T_LSC].as<int32_t>();
        STEP(hipMemsetAsync(cnt, 0, tab * 4, s), "memset");
        hipLaunchKernelGGL(k_level_sys_count, dim3(blocks(ncell, kBlock)), dim3(kBlock), 0, s,
                           cells(), ncell, nsys, cnt);
        LAUNCHED("level counts");
        std::vector<int32_t> hc(tab), base(tab, 0), first(tab, 0);
        STEP(hipMemcpyAsync(hc.data(), cnt, tab * 4, hipMemcpyDeviceToHost, s), "copy");
        STEP(hipStreamSynchronize(s), "sync");
        int64_t cb = 0;
        for (int q = 0; q < nsys; ++q) {
            sys_root[(size_t)q] = (int32_t)cb;
            for (int l = 0; l < nl; ++l) {
                base[(size_t)l * nsys + q] = (int32_t)cb;
                cb += hc[(size_t)l * nsys + q];
            }
        }
        for (int l = 0; l < nl; ++l) {
            int64_t f = level[(size_t)l];
            for (int q = 0; q < nsys; ++q) {
                first[(size_t)l * nsys + q] = (int32_t)f;
                f += hc[(size_t)l * nsys + q];
            }
        }
        STEP(hipMemcpyAsync(cnt + tab, base.data(), tab * 4, hipMemcpyHostToDevice, s), "copy");
        STEP(hipMemcpyAsync(cnt + 2 * tab, first.data(), tab * 4, hipMemcpyHostToDevice, s),
             "copy");
        STEP(B[T_PERM].reserve((size_t)ncell * 4), "allocation");
        int32_t *perm = B[T_PERM].as<int32_t>();
        hipLaunchKernelGGL(k_perm, dim3(blocks(ncell, kBlock)), dim3(kBlock), 0, s, cells(),
                           ncell, nsys, cnt + tab, cnt + 2 * tab, perm);
        LAUNCHED("renumbering");
        // permute each cell array into a scratch buffer and copy it back (the
        // arrays keep their allocations; everything is ordered on stream s)
        const unsigned g = blocks(ncell, kBlock);
        DevArray nb;
        if (!hip(nb.reserve((size_t)ncell * sizeof(CellRec)), "allocation")) return fail();
        auto apply = [&](DevArray &arr, size_t elem, int kind) -> bool {
            if (kind == 0)
                hipLaunchKernelGGL((k_permute<double>), dim3(g), dim3(kBlock), 0, s, ncell, perm,
                                   arr.as<double>(), nb.as<double>(), false);
            else if (kind == 1)
                hipLaunchKernelGGL((k_permute<uint64_t>), dim3(g), dim3(kBlock), 0, s, ncell,
                                   perm, arr.as<uint64_t>(), nb.as<uint64_t>(), false);
            else if (kind == 2 || kind == 3)
                hipLaunchKernelGGL((k_permute<int32_t>), dim3(g), dim3(kBlock), 0, s, ncell,
                                   perm, arr.as<int32_t>(), nb.as<int32_t>(), kind == 3);
            else
                hipLaunchKernelGGL((k_permute<CellRec>), dim3(g), dim3(kBlock), 0, s, ncell,
                                   perm, arr.as<CellRec>(), nb.as<CellRec>(), false);
            if (!hip(hipGetLastError(), "renumbering")) return false;
            return hip(hipMemcpyAsync(arr.p, nb.p, (size_t)ncell * elem,
                                      hipMemcpyDeviceToDevice, s),
                       "copy");
        };
        bool ok = true;
        for (TreeBuf b : {T_CX, T_CY, T_CZ, T_SIDE}) ok = ok && apply(B[b], 8, 0);
        ok = ok && apply(B[T_CKEY], 8, 1);
        for (TreeBuf b : {T_FIRST, T_COUNT, T_NCHILD, T_DEPTH, T_CSYS}) ok = ok && apply(B[b], 4, 2);
        for (TreeBuf b : {T_CHILD0, T_PARENT}) ok = ok && apply(B[b], 4, 3);
        ok = ok && apply(*O.pool_c, sizeof(CellRec), 4);
        (void)hipStreamSynchronize(s);
        nb.release();
        if (!ok) return fail();
    }
    STEP(B[T_SYSROOT].reserve((size_t)nsys * 4), "allocation");
    STEP(hipMemcpyAsync(B[T_SYSROOT].p, sys_root.data(), (size_t)nsys * 4,
                        hipMemcpyHostToDevice, s),
         "copy");

    // groups in depth-first order
    STEP(B[T_GSTART].reserve((size_t)n * 4), "allocation");
    STEP(B[T_GROUPS].reserve((size_t)n * 4), "allocation");
    STEP(B[T_NSEL].reserve(64), "allocation");
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks(n, kBlock)), dim3(kBlock), 0, s,
                       B[T_GSTART].as<int32_t>(), n, -1);
    LAUNCHED("fill");
    hipLaunchKernelGGL(k_group_mark, dim3(blocks(ncell, kBlock)), dim3(kBlock), 0, s, cells(),
                       ncell, P.ncrit, B[T_GSTART].as<int32_t>());
    LAUNCHED("groups");
    {
        size_t st = 0;
        STEP(hipcub::DeviceSelect::If(nullptr, st, B[T_GSTART].as<int32_t>(),
                                      B[T_GROUPS].as<int32_t>(), B[T_NSEL].as<int32_t>(),
                                      (int)n, NonNegative(), s),
             "select size");
        STEP(B[T_SORT].reserve(std::max(st, B[T_SORT].cap)), "allocation");
        STEP(hipcub::DeviceSelect::If(B[T_SORT].p, st, B[T_GSTART].as<int32_t>(),
                                      B[T_GROUPS].as<int32_t>(), B[T_NSEL].as<int32_t>(),
                                      (int)n, NonNegative(), s),
             "select");
    }
    int32_t ng32 = 0;
    STEP(hipMemcpyAsync(&ng32, B[T_NSEL].p, 4, hipMemcpyDeviceToHost, s), "copy");
    STEP(hipStreamSynchronize(s), "sync");
    const int64_t ng = ng32;
    const int32_t *groups = B[T_GROUPS].as<int32_t>();

    // walk: count, offsets, fill
    STEP(B[T_WC].reserve((size_t)ncell * sizeof(WCell)), "allocation");
    STEP(B[T_WL].reserve((size_t)ncell * sizeof(WLink)), "allocation");
    hipLaunchKernelGGL(k_walk_cells, dim3(blocks(ncell, kBlock)), dim3(kBlock), 0, s, cells(),
                       ncell, pc, B[T_WC].as<WCell>(), B[T_WL].as<WLink>());
    LAUNCHED("walk cells");
    STEP(B[T_JPCNT].reserve((size_t)(ng + 1) * 8), "allocation");
    STEP(B[T_JCCNT].reserve((size_t)(ng + 1) * 8), "allocation");
    STEP(O.jp_off->reserve((size_t)(ng + 1) * 8), "allocation");
    STEP(O.jc_off->reserve((size_t)(ng + 1) * 8), "allocation");
    STEP(hipMemsetAsync(B[T_JPCNT].as<int64_t>() + ng, 0, 8, s), "memset");
    STEP(hipMemsetAsync(B[T_JCCNT].as<int64_t>() + ng, 0, 8, s), "memset");
    WalkArgs W{};
    W.groups = groups;
    W.cell_sys = B[T_CSYS].as<int32_t>();
    W.sys_root = B[T_SYSROOT].as<int32_t>();
    W.ng = ng;
    W.wc = B[T_WC].as<WCell>();
    W.wl = B[T_WL].as<WLink>();
    W.theta2 = P.theta * P.theta;
    W.rcut = P.rcut;
    {
        const double r = P.rcut * (1.0 + 0x1p-16);
        W.rdrop2 = P.rcut > 0.0 ? r * r : 0.0;
    }
    W.box = P.box;
    W.jp_cnt = B[T_JPCNT].as<int64_t>();
    W.jc_cnt = B[T_JCCNT].as<int64_t>();
    W.flag = B[T_FLAG].as<int>();
    // one frame per level below the root: enough for the deepest opened cell
    W.frames = std::max(1, std::min(kFrames, (int)level.size() - 1));
    const size_t walk_lds = (size_t)W.frames * (kWalkBlock * sizeof(int2) + kWalkBlock / kOct * 4);
    W.gbox = nullptr;
    if (W.rdrop2 > 0.0) {
        STEP(B[T_GBOX].reserve((size_t)ng * 6 * 8), "allocation");
        hipLaunchKernelGGL(k_group_box, dim3(blocks(ng, kBlock)), dim3(kBlock), 0, s, cells(),
                           groups, ng, idx, P.x, B[T_GBOX].as<double>());
        LAUNCHED("group boxes");
        W.gbox = B[T_GBOX].as<double>();
    }
    // One walk into fixed slots when the caller gives capacities (from an
    // earlier build) and the slots fit the memory bound; else count first.
    const bool slots = P.cap_p > 0 && P.cap_c > 0 &&
                       (double)ng * (double)(P.cap_p + P.cap_c) * 4.0 <= (double)P.slot_bytes;
    if (slots) {
        STEP(B[T_JPSLOT].reserve((size_t)ng * (size_t)P.cap_p * 4), "allocation");
        STEP(B[T_JCSLOT].reserve((size_t)ng * (size_t)P.cap_c * 4), "allocation");
        W.cap_p = P.cap_p;
        W.cap_c = P.cap_c;
        W.jp_idx = B[T_JPSLOT].as<int32_t>();
        W.jc_idx = B[T_JCSLOT].as<int32_t>();
        hipLaunchKernelGGL(k_walk<kWalkSlots>, dim3(walk_blocks(ng)), dim3(kWalkBlock), walk_lds, s, W);
        LAUNCHED("walk (slots)");
    } else {
        hipLaunchKernelGGL(k_walk<kWalkCount>, dim3(walk_blocks(ng)), dim3(kWalkBlock), walk_lds, s, W);
        LAUNCHED("walk (count)");
    }
    for (int pass = 0; pass < 2; ++pass) {
        int64_t *cnt = pass ? B[T_JCCNT].as<int64_t>() : B[T_JPCNT].as<int64_t>();
        int64_t *off = pass ? O.jc_off->as<int64_t>() : O.jp_off->as<int64_t>();
        size_t st = 0;
        STEP(hipcub::DeviceScan::ExclusiveSum(nullptr, st, cnt, off, (int)(ng + 1), s),
             "scan size");
        STEP(B[T_SORT].reserve(std::max(st, B[T_SORT].cap)), "allocation");
        STEP(hipcub::DeviceScan::ExclusiveSum(B[T_SORT].p, st, cnt, off, (int)(ng + 1), s),
             "scan");
    }
    // list totals, longest lists and the walk's overflow flag: the host
    // needs only these five numbers (the offsets stay on the device)
    STEP(B[T_STATS].reserve(8 * sizeof(int64_t)), "allocation");
    int64_t *stats = B[T_STATS].as<int64_t>();
    for (int pass = 0; pass < 2; ++pass) {
        const int64_t *cnt = pass ? B[T_JCCNT].as<int64_t>() : B[T_JPCNT].as<int64_t>();
        size_t st = 0;
        STEP(hipcub::DeviceReduce::Max(nullptr, st, cnt, stats + 2 + pass, (int)ng, s),
             "reduce size");
        STEP(B[T_SORT].reserve(std::max(st, B[T_SORT].cap)), "allocation");
        STEP(hipcub::DeviceReduce::Max(B[T_SORT].p, st, cnt, stats + 2 + pass, (int)ng, s),
             "reduce");
    }
    hipLaunchKernelGGL(k_list_stats, dim3(1), dim3(1), 0, s, ng, O.jp_off->as<int64_t>(),
                       O.jc_off->as<int64_t>(), B[T_FLAG].as<int>(), stats);
    LAUNCHED("list totals");
    int64_t hstats[5] = {0, 0, 0, 0, 0};
    STEP(hipMemcpyAsync(hstats, stats, sizeof(hstats), hipMemcpyDeviceToHost, s), "copy");
    STEP(hipStreamSynchronize(s), "sync");
    if (hstats[4]) {
        code = BHQ_E_RANGE;
        what = "walk stack overflow";
        return fail();
    }
    const int64_t njp = hstats[0], njc = hstats[1];
    const int64_t max_p = hstats[2], max_c = hstats[3];
    O.one_walk = slots && max_p <= P.cap_p && max_c <= P.cap_c;
    O.slot_p = O.slot_c = 0;
    if (O.one_walk) {
        // every group's entries are in its slot: the slots become the lists
        // (the force kernel reads group g from g * slot size), and the old
        // list arrays the slots of the next rebuild
        std::swap(*O.jp_idx, B[T_JPSLOT]);
        std::swap(*O.jc_idx, B[T_JCSLOT]);
        O.slot_p = P.cap_p;
        O.slot_c = P.cap_c;
    } else {
        // The list arrays trade places with the slots on the next one-walk
        // rebuild, so they are given the size of its slots where those will
        // be used: then neither needs to grow again.
        int64_t want_p = njp, want_c = njc;
        const int64_t np2 = next_slot_cap(P.cap_p, max_p), nc2 = next_slot_cap(P.cap_c, max_c);
        if ((double)ng * (double)(np2 + nc2) * 4.0 <= (double)slot_memory_bound(njp, njc)) {
            want_p = std::max(want_p, ng * np2);
            want_c = std::max(want_c, ng * nc2);
        }
        STEP(O.jp_idx->reserve((size_t)std::max<int64_t>(want_p, 1) * 4), "allocation");
        STEP(O.jc_idx->reserve((size_t)std::max<int64_t>(want_c, 1) * 4), "allocation");
        W.jp_off = O.jp_off->as<int64_t>();
        W.jc_off = O.jc_off->as<int64_t>();
        W.jp_idx = O.jp_idx->as<int32_t>();
        W.jc_idx = O.jc_idx->as<int32_t>();
        hipLaunchKernelGGL(k_walk<kWalkFill>, dim3(walk_blocks(ng)), dim3(kWalkBlock), walk_lds, s, W);
        LAUNCHED("walk (fill)");
    }
    O.max_p = max_p;
    O.max_c = max_c;

    // particles and groups in the layout of the force context
    STEP(O.pool_p->reserve((size_t)n * sizeof(PartRec)), "allocation");
    STEP(O.xi->reserve((size_t)n * 8), "allocation");
    STEP(O.yi->reserve((size_t)n * 8), "allocation");
    STEP(O.zi->reserve((size_t)n * 8), "allocation");
    STEP(O.i_off->reserve((size_t)(ng + 1) * 8), "allocation");
    STEP(O.gcx->reserve((size_t)ng * 8), "allocation");
    STEP(O.gcy->reserve((size_t)ng * 8), "allocation");
    STEP(O.gcz->reserve((size_t)ng * 8), "allocation");
    if (P.eps2) STEP(O.e2i->reserve((size_t)n * 8), "allocation");
    hipLaunchKernelGGL(k_particles_out, dim3(blocks(n, kBlock)), dim3(kBlock), 0, s, idx, n,
                       P.x, P.m, P.eps2, O.pool_p->as<PartRec>(), O.xi->as<double>(),
                       O.yi->as<double>(), O.zi->as<double>(),
                       P.eps2 ? O.e2i->as<double>() : nullptr);
    LAUNCHED("particle pool");
    hipLaunchKernelGGL(k_groups_out, dim3(blocks(ng + 1, kBlock)), dim3(kBlock), 0, s, cells(),
                       groups, ng, n, O.i_off->as<int64_t>(), O.gcx->as<double>(),
                       O.gcy->as<double>(), O.gcz->as<double>());
    LAUNCHED("groups");
    STEP(hipStreamSynchronize(s), "sync");
    O.ng = ng;
    O.njp = njp;
    O.njc = njc;
    O.ncell = ncell;
    O.nlevels = (int)level.size() - 1;
#undef STEP
#undef LAUNCHED
    return BHQ_OK;
}

}  // namespace bhq
