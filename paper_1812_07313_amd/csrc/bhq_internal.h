// bhq_internal.h -- shared between the C-ABI layer (bhq_api.cpp) and the
// HIP kernels (bhq_kernels.hip).  Not part of the public ABI.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

namespace bhq {

// Group dispatch order, shared by the host planner and the device planner
// (constexpr functions compile for both sides, so the two give the same
// table).  Cost of a group in units of 1/100 of a particle term:
// ni (100 njp + 265 njc + 100): a cell term costs about 53/20 of a particle
// term, and the last term stands for loading and storing the i-particles.
constexpr uint64_t order_cost(int64_t ni, int64_t njp, int64_t njc)
{
    return (uint64_t)ni * (100u * (uint64_t)njp + 265u * (uint64_t)njc + 100u);
}

// XCD piece of group g: the piece holding the midpoint of the group's cost
// interval [before, before + cost) within the total, as
// floor((2 before + cost) / (2 total) * xcds) in FP64 (monotone in g);
// by group count when every group is empty.
constexpr int order_piece(uint64_t before, uint64_t cost, uint64_t total, int xcds, int64_t g,
                          int64_t ng)
{
    const int x = total > 0
                      ? (int)((double)(2 * before + cost) / (double)(2 * total) * (double)xcds)
                      : (int)(g * xcds / ng);
    return x < 0 ? 0 : (x > xcds - 1 ? xcds - 1 : x);
}

// One device array with reusable capacity (host-side handle).
struct DevArray {
    void *p = nullptr;
    size_t cap = 0;
    // At least `bytes` of capacity; old contents are not kept.  Growing an
    // existing block leaves 25 % headroom, so that sizes that drift upwards
    // from call to call (lists rebuilt every time step) do not free and
    // allocate again each time.
    hipError_t reserve(size_t bytes)
    {
        if (bytes <= cap && p) return hipSuccess;
        if (p) {
            (void)hipFree(p);
            p = nullptr;
            cap = 0;
            bytes += bytes / 4;
        }
        if (bytes == 0) bytes = 256;
        hipError_t e = hipMalloc(&p, bytes);
        if (e == hipSuccess) cap = bytes;
        return e;
    }
    // At least `bytes` of capacity, keeping the first `used` bytes (the
    // stream is synchronised before the old block is freed).
    hipError_t grow(size_t bytes, size_t used, hipStream_t s)
    {
        if (bytes <= cap && p) return hipSuccess;
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, bytes ? bytes : 256);
        if (e != hipSuccess) return e;
        if (p && used) e = hipMemcpyAsync(q, p, used, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            (void)hipFree(q);
            return e;
        }
        if (p) (void)hipFree(p);
        p = q;
        cap = bytes ? bytes : 256;
        return hipSuccess;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

// Pool records for index-mode lists (AoS, FP64).
struct alignas(32) PartRec {
    double x, y, z, m;
};
struct alignas(32) CellRec {
    double x, y, z, m;          // centre of mass, mass
    double q00, q01, q02, q11;  // quadrupole (List 1 order)
    double q12, q22, t, pad;    // ..., trace
};

// Device-side view of one force evaluation.  All arrays are SoA in device
// memory; i-particles and outputs are in group order.
struct ForceArgs {
    int64_t ng;                     // groups
    int64_t nslots;                 // entries of order (grid of one block
                                    // per slot)
    const int32_t *order;           // slot b holds group order[b], or -1
                                    // (empty slot)
    int xcds;                       // > 0: slot b belongs to XCD b % xcds
                                    // and the persistent kernel keeps one
                                    // counter per XCD in queue[0..xcds)
    const int64_t *i_off;           // [ng+1]
    const int64_t *jp_off;          // [ng+1]
    const int64_t *jc_off;          // [ng+1]
    const double *gcx, *gcy, *gcz;  // [ng] group reference points (FP64)
    const double *xi, *yi, *zi;     // [ni] i positions (FP64)
    const double *e2i;              // [ni] squared softening
    const double *jpx, *jpy, *jpz, *jpm;           // [njp] j-particles
    const double *jcx, *jcy, *jcz, *jcm;           // [njc] j-cell com, mass
    const double *q00, *q01, *q02, *q11, *q12, *q22;  // [njc] quadrupole
    const double *jct;              // [njc] trace (split kernel)
    double *ax, *ay, *az, *pot;     // [ni] results (FP64): element i at
                                    // ax[i * out_stride] (pot may be NULL)
    int64_t out_stride;             // 1: SoA arrays; 3: ax = a[.][0] of an
                                    // AoS a[ni][3] (ay, az the next ones)
    double box;                     // > 0: periodic minimum image
    double rs, rcut;                // split-kernel parameters
    unsigned int *queue;            // slot counters of the persistent kernel
                                    // (kQueueWords words, zeroed per launch)
    // Index-mode lists (all NULL for materialised lists): entry k of the
    // j-particle list is pool_p[jp_idx[k]], of the j-cell list
    // pool_c[jc_idx[k]].
    const PartRec *pool_p;
    const CellRec *pool_c;
    const int32_t *jp_idx;
    const int32_t *jc_idx;
    // > 0: index lists in per-group slots (rebuilt device lists): group g's
    // entries start at g * jp_slot (jc_slot) instead of jp_off[g]; their
    // counts are still jp_off[g + 1] - jp_off[g].
    int64_t jp_slot, jc_slot;
    // Cross-block j-split (LaunchCfg::jsplit = J > 1): the block for part
    // s of a group takes entries [n s / J, n (s + 1) / J) of each of its
    // lists and writes its sums for i-particle i to part[s * ni + i]
    // (x, y, z, -phi in the working precision: 16 B per entry in FP32,
    // 32 B in FP64); a reduction then adds the J parts of each particle in
    // the order s = 0, 1, ... and writes the results.
    void *part;
    int64_t ni;                     // i-particles (i_off[ng])
};

constexpr int kQueueWords = 64;  // capacity of ForceArgs::queue

// Launch shape.  block: threads per block (128 or 256), which is also the
// depth of one LDS tile; i_per_thread: i-particles per thread (1 or 2);
// persistent: one grid of blocks_per_cu * num_cu
// blocks pulling groups from ForceArgs::queue (blocks_per_cu <= 0: as many
// as fit), otherwise one block per group.
struct LaunchCfg {
    int block = 256;
    int i_per_thread = 2;  // i-particles owned by each thread: 1 or 2
    int persistent = 0;
    int blocks_per_cu = 0;
    int num_cu = 0;
    int jsplit = 1;        // parts of each group's lists (1, 2, 4 or 8)
    int waves_per_eu = 0;  // 0: compiler's choice; 6 or 8 (FP32, block 256)
};

constexpr int kMaxJsplit = 8;

// Static working memory for callers that cannot allocate (bhq_compute_noalloc):
// a file-scope device array in bhq_kernels.hip holding the persistent
// queue counters (the first kScratchQueueBytes) and the j-split parts (the
// next kScratchPartBytes).  Each device has its own copy.
constexpr size_t kScratchQueueBytes = 256;
constexpr size_t kScratchPartBytes = (size_t)16 << 20;
// Look up the array's device address on `device` (made current by the
// caller) once and keep it; returns the lookup's status.
hipError_t scratch_init(int device);
// The address found by scratch_init on `device`, or NULL.
void *scratch_ptr(int device);

// Pairs of the split kernels' lists inside the cutoff (FP64 decision),
// added to out[0] (particles), out[1] (cells); one block per group.
hipError_t launch_count_live(const ForceArgs &A, unsigned long long *out, hipStream_t s);
// One wave that records the shader clock over `ticks` of the constant-rate
// counter: out[0..3] = clock start, real start, clock end, real end.
hipError_t launch_clock_window(unsigned long long ticks, unsigned long long *out, hipStream_t s);

// Device-side uploads (bhq_upload.hip).  The check kernels OR these bits
// into *flag; launch_clear_flag zeroes it.
constexpr unsigned kBadNonFinite = 1, kBadNonPositive = 2, kBadOrder = 4, kBadRange = 8;

// Smallest accepted squared softening: the smallest normal FP32 number,
// 2^-126.  The softened kernels include each particle's self pair, where r^2
// = eps^2, and its reciprocal square root must be finite in FP32 (a smaller
// eps^2 flushes to zero there) and in the FP64 kernels' rsqrt, which handles
// only normal positive arguments.
constexpr double kMinEps2 = 0x1p-126;
hipError_t launch_clear_flag(unsigned *flag, hipStream_t s);
hipError_t launch_check_f64(const double *v, int64_t n, bool positive, unsigned *flag,
                            hipStream_t s);
hipError_t launch_check_offsets(const int64_t *off, int64_t ng, unsigned *flag, hipStream_t s);
hipError_t launch_check_idx(const int32_t *idx, int64_t n, int64_t pool, unsigned *flag,
                            hipStream_t s);
// column c of the AoS array v[n][w] (w <= 6) to out[c] (NULL: skipped)
hipError_t launch_unpack(const double *v, int64_t n, int w, double *const *out, hipStream_t s);
hipError_t launch_pack_particles(const double *x, const double *m, int64_t n, PartRec *out,
                                 hipStream_t s);
hipError_t launch_pack_cells(const double *x, const double *m, const double *q,
                             const double *t, int64_t n, CellRec *out, hipStream_t s);

// Launch the force kernel for (kernel, precision) on `stream`.  Returns
// the launch status.
hipError_t launch_force(int kernel, int precision, const ForceArgs &args,
                        const LaunchCfg &cfg, hipStream_t stream);

// Time-step helpers (bhq_integrate.hip).  order == NULL: identity.
hipError_t launch_scatter(const int32_t *order, int64_t n, const double *ax,
                          const double *ay, const double *az, const double *pot,
                          double *a_out, double *pot_out, hipStream_t s);
hipError_t launch_kick_drift(int64_t n, double *x, double *v, const double *a,
                             double dtk, double dtd, hipStream_t s);
hipError_t launch_wrap(int64_t n, double *x, double box, hipStream_t s);
hipError_t launch_fill_f64(double *v, int64_t n, double val, hipStream_t s);
// out row k = in row order[k] (rows of `words` 8-byte words); v[k] = k.
hipError_t launch_gather_rows(int64_t n, int words, const void *in, const int32_t *order,
                              void *out, hipStream_t s);
hipError_t launch_iota(int32_t *v, int64_t n, hipStream_t s);

// XCD dispatch order of ng groups whose offsets are in device memory,
// computed on the GPU; equal to the host planner's table.  Supported for
// window and tail up to 1024.  The table goes to `order`, its slot count
// to *nslots; returns a BHQ_* code (message in *what).  Synchronises s.
bool plan_order_device_supported(int window, int tail);
int plan_order_device(int64_t ng, const int64_t *i_off, const int64_t *jp_off,
                      const int64_t *jc_off, int window, int tail, int xcds, DevArray &order,
                      DevArray &scratch, int64_t *nslots, hipStream_t s, std::string *what);
int energy_partials();  // partial-sum slots (pairs) used by launch_energies
hipError_t launch_energies(int64_t n, const double *m, const double *v,
                           const double *pot, double eps, double *part,
                           double *out, hipStream_t s);

// Device construction of the tree, groups and index lists (bhq_tree.hip).
// Inputs: n particles, positions x[n][3] and masses m[n] in device memory.
struct TreeParams {
    const double *x;
    const double *m;
    const double *eps2;       // [n] per-particle softening squared, or NULL
    int64_t n;
    int64_t nsys;             // independent systems (1: one system)
    const int64_t *sys_off;   // host [nsys + 1]: system s is [sys_off[s], sys_off[s+1])
    double theta;
    int ncrit, nleaf;
    double box, rcut;
    // Per-group list capacities for a one-walk build (0: count, then fill).
    // With capacities the walk writes each group's entries into a slot of
    // that many entries and counts them; the lists are then compacted, or,
    // if a group overflowed its slot, filled by a second walk with the exact
    // offsets.
    int64_t cap_p = 0, cap_c = 0;
    int64_t slot_bytes = 0;  // upper bound on the slot memory of that mode
    // Depth (levels) and cell count of an earlier build of similar input:
    // the levels are then built without host synchronisation (0: unknown).
    int spec_levels = 0;
    int64_t spec_cells = 0;
};

// Slot sizing of one-walk rebuilds.  A group's slot holds 1.25 times the
// longest list of the previous build plus 32 entries; the current size is
// kept while that stays within [3/4, 1] of it, so that the slot memory
// keeps its size from step to step.
inline int64_t next_slot_cap(int64_t cur, int64_t longest)
{
    const int64_t want = longest + longest / 4 + 32;
    return (want <= cur && 4 * want >= 3 * cur) ? cur : want;
}

// Memory the slots of a rebuild may take (bytes): 4 times that of the
// previous build's lists plus 256 MiB.
inline int64_t slot_memory_bound(int64_t njp, int64_t njc)
{
    return 16 * (njp + njc) + ((int64_t)256 << 20);
}

// Builder working memory, kept between builds of one context.
enum TreeBuf {
    T_KEY, T_KEY2, T_IDX0, T_SORT, T_BBOX, T_FLAG,
    T_CX, T_CY, T_CZ, T_SIDE, T_FIRST, T_COUNT, T_CHILD0, T_NCHILD, T_PARENT,
    T_DEPTH, T_CKEY, T_NCH, T_NOFF, T_GSTART, T_GROUPS, T_NSEL, T_WC, T_WL,
    T_JPCNT, T_JCCNT, T_CSYS, T_SYSOFF, T_SYSOFF32, T_ROOTS, T_SYSROOT, T_LSC, T_PERM,
    T_JPSLOT, T_JCSLOT, T_GBOX, T_LV, T_STATS,
    T_COUNT_
};

// Where the results go: arrays of the force context, filled in the layout
// bhq_compute reads (i-particles, pools and lists in tree order).
struct TreeOut {
    DevArray *i_off, *jp_off, *jc_off;        // int64 [ng+1]
    DevArray *gcx, *gcy, *gcz;                // FP64 [ng] group centres
    DevArray *xi, *yi, *zi;                   // FP64 [n] i-particles
    DevArray *e2i;                            // FP64 [n] softening (when given)
    DevArray *pool_p;                         // PartRec [n], tree order
    DevArray *pool_c;                         // CellRec [ncell]
    DevArray *jp_idx, *jc_idx;                // int32 list entries
    DevArray *order;                          // int32 [n]: input index of
                                              // tree position k
    DevArray *buf;                            // [T_COUNT_] working memory
    // sizes, set on success (the offsets themselves stay on the device)
    int64_t ng = 0, njp = 0, njc = 0, ncell = 0;
    // longest particle and cell list of a group; whether one walk sufficed
    int64_t max_p = 0, max_c = 0;
    bool one_walk = false;
    // one walk: jp_idx / jc_idx hold the per-group slots of these sizes
    int64_t slot_p = 0, slot_c = 0;
    int nlevels = 0;  // levels of the tree (the root's included)
};

// Returns a BHQ_* code; on failure *err names the step.
int build_tree_lists(const TreeParams &P, TreeOut &O, hipStream_t stream,
                     std::string *err);

// Lists in per-group slots (slot entries per group, counts from off) to
// the compact layout out[off[g] ...].
hipError_t launch_compact_lists(int64_t ng, const int64_t *off, const int32_t *slot,
                                int64_t cap, int32_t *out, hipStream_t s);

}  // namespace bhq
