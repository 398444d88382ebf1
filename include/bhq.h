/*
 * bhq.h -- C ABI of libbhq: Barnes-Hut tree forces with monopole and
 * traceless-quadrupole cell terms, evaluated over per-group interaction
 * lists on an AMD Instinct MI355X (gfx950).
 *
 * The operation (Kodama & Ishiyama, arXiv:1812.07313):
 *   For every i-particle of group g, with d = r_j - r_i and
 *   rhat^2 = |d|^2 + eps_i^2 (G = 1):
 *     a_i   = sum_{j in P_g} m_j d / rhat^3
 *           + sum_{c in C_g} [ (phi_m + 5 phi_q) / rhat^2 d - Q_c d / rhat^5 ]
 *     phi_i = - sum_{j in P_g} m_j / rhat - sum_{c in C_g} (phi_m + phi_q)
 *   with phi_m = M_c / rhat and phi_q = d.Q_c.d / (2 rhat^5)
 *   (Sec. 3, eq. 1 for the potential, eqs. 4-7 for the acceleration;
 *   a is returned attractive and phi negative).  P_g (j-particles) and C_g
 *   (j-cells with mass, centre of mass and traceless quadrupole Q, eq. 2)
 *   are the group's interaction list; all i-particles of a group share it
 *   (the modified tree algorithm of Sec. 3.4).  The particle-particle part
 *   is summed before the cell part (List 4: assign, then add).
 *
 * Kernels: BHQ_QUAD (above), BHQ_MONO (cells as point masses, Q ignored:
 * the paper's "monopole" program), BHQ_SPLIT_QUAD / BHQ_SPLIT_MONO
 * (short-range Gaussian-split kernel Phi = -erfc(r / 2 r_s) / r with a
 * cutoff in a periodic box; not from the paper), BHQ_QUAD_SOFT (the
 * complete second-order expansion of the softened potential: eq. 1 plus the
 * trace term T_c eps^2 / (2 rhat^5) that eq. 1 leaves out, T_c = sum m
 * |x - com|^2, i.e. d.Q_c.d replaced by d.Q_c.d - T_c eps^2 in phi_q; the
 * traces come from set_jc's trace argument or the cell pool, and a NULL
 * trace in set_jc means T_c = 0, which makes it BHQ_QUAD).
 * Precisions: BHQ_FP32_OFS64 forms positions relative to the group centre
 * in FP64 and does all interaction arithmetic and accumulation in FP32;
 * BHQ_FP64 does everything in FP64.
 *
 * Conventions for every call:
 *   - Return value: BHQ_OK (0) or a negative BHQ_E_* code; nothing aborts
 *     or throws across the ABI.  bhq_last_error() describes the last
 *     failure on a context.
 *   - Host arrays passed to bhq_set_* are copied before the call returns
 *     (as the paper's set calls copy into their own structures, Sec. 3.4);
 *     the caller keeps ownership.  Device memory is owned by the context.
 *   - Positions are FP64, AoS: double (*x)[3] = x[k][0..2].
 *   - Quadrupoles are double (*q)[6] = (q00, q01, q02, q11, q12, q22), the
 *     order of the paper's j-cell structure (List 1); q22 is stored, not
 *     recomputed.
 *   - i-particles are given in group order: group g owns i-particles
 *     i_off[g] .. i_off[g+1]-1.
 *   - Lists are materialised: group g's j-particles are entries
 *     jp_off[g] .. jp_off[g+1]-1 of the j-particle arrays, its j-cells
 *     entries jc_off[g] .. jc_off[g+1]-1 of the j-cell arrays.
 *   - One context per host thread; calls on one context are not
 *     thread-safe.
 */
#ifndef BHQ_H
#define BHQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bhq_ctx bhq_ctx;
typedef struct bhq_lists bhq_lists;

/* return codes */
#define BHQ_OK 0
#define BHQ_E_ARG (-1)       /* invalid argument (null, negative, bad enum) */
#define BHQ_E_RANGE (-2)     /* offsets not monotone, or past the end        */
#define BHQ_E_NODEV (-3)     /* no usable GPU / device index out of range    */
#define BHQ_E_HIP (-4)       /* a HIP runtime call failed                    */
#define BHQ_E_NOMEM (-5)     /* host or device allocation failed             */
#define BHQ_E_STATE (-6)     /* call out of order (e.g. compute before set)  */
#define BHQ_E_NONFINITE (-7) /* NaN or infinity in an input                  */

/* kernels */
#define BHQ_MONO 0
#define BHQ_QUAD 1
#define BHQ_SPLIT_QUAD 2
#define BHQ_SPLIT_MONO 3
#define BHQ_QUAD_SOFT 4

/* precisions */
#define BHQ_FP32_OFS64 0
#define BHQ_FP64 1

/* Group dispatch orders (bhq_set_group_order, bhq_plan_order). */
#define BHQ_ORDER_COST 0   /* all groups, most expensive first            */
#define BHQ_ORDER_XCD 1    /* pieces of space per XCD, see below          */
#define BHQ_ORDER_WINDOW 256   /* default window of BHQ_ORDER_XCD          */
#define BHQ_ORDER_TAIL 1024    /* default tail of BHQ_ORDER_XCD            */
#define BHQ_XCDS 8 /* accelerator complex dies (own L2 each) of one gfx950 */

/* Create a context on HIP device `device` for the given kernel and
 * precision (the counterpart of opening the force library, g5_open in the
 * paper's driver, Sec. 3.4, List 4).  *out receives the context (NULL on
 * failure).
 * Errors: BHQ_E_ARG (null out, bad enum), BHQ_E_NODEV (no GPU, or device
 * out of range), BHQ_E_HIP, BHQ_E_NOMEM. */
int bhq_create(bhq_ctx **out, int device, int kernel, int precision);

/* Wait for outstanding work, free all device and host memory of the
 * context (g5_close, List 4).  NULL is accepted and ignored. */
int bhq_destroy(bhq_ctx *ctx);

/* Switch kernel and/or precision for later computes on the same data:
 * quadrupole cells (Sec. 3, eqs. 1, 4-7), monopole cells (the monopole
 * program of Secs. 4-5), the complete softened quadrupole, or the split
 * kinds (no counterpart in the paper); FP32 with FP64 offsets or FP64.
 * Errors: BHQ_E_ARG for an unknown kernel or precision. */
int bhq_set_kernel(bhq_ctx *ctx, int kernel, int precision);

/* One softening length for every i-particle: eps^2 = eps * eps (the
 * paper's set-eps-to-all call, List 4).  The softened kernels include each
 * particle's self pair (d = 0, r^2 = eps^2), which needs eps^2 >= 2^-126, a
 * normal FP32 number (eps >= about 1.1e-19; BHQ_E_ARG otherwise).
 * Overrides earlier per-particle values.  The split kernels do not use
 * eps. */
int bhq_set_eps(bhq_ctx *ctx, double eps);

/* Per-i-particle squared softening (the i-particle structure carries eps^2
 * per particle, List 2), in group order; ni must equal i_off[ng] of the
 * last bhq_set_groups.  Every value finite and >= 2^-126, as for bhq_set_eps
 * (BHQ_E_ARG / BHQ_E_NONFINITE otherwise). */
int bhq_set_eps2_i(bhq_ctx *ctx, int64_t ni, const double *eps2);

/* Short-range split parameters for the SPLIT kernels (no counterpart in
 * the paper; the short-range part of the TreePM force that Sec. 1 names
 * as the setting of tree codes in cosmology): r_s > 0, cutoff
 * rcut > 0; box > 0 selects a periodic cube of that side (minimum-image
 * separations), box == 0 an open boundary.  The FP32 split kernels take
 * erfc and the related radial functions from a table that covers
 * r / (2 r_s) <= 2.5 only, so bhq_compute returns BHQ_E_ARG for FP32 with
 * rcut > 5 r_s (FP64 has no such limit: it takes exp(-u^2) and
 * exp(u^2) erfc(u) from polynomial tables up to u = 4, forms erfc as their
 * product, and calls the library's exp and erfc beyond).  In a periodic box every
 * group cell plus 2 rcut must stay below half the box. */
int bhq_set_split(bhq_ctx *ctx, double rs, double rcut, double box);

/* Define the groups and the list sizes; must precede set_i / set_jp /
 * set_jc.  A group is the set of i-particles that share one interaction
 * list: the particles of a cell with at most n_crit of them (the modified
 * tree algorithm, Sec. 3.4, List 4).  ng >= 1 groups.
 *   i_off[ng+1]   i_off[0] == 0, non-decreasing; ni = i_off[ng]
 *   center[ng]    FP64 reference point of each group (its cell centre);
 *                 FP32 kernels form all positions relative to it
 *   jp_off[ng+1]  jp_off[0] == 0, non-decreasing; njp = jp_off[ng]
 *   jc_off[ng+1]  jc_off[0] == 0, non-decreasing; njc = jc_off[ng]
 * Errors: BHQ_E_ARG, BHQ_E_RANGE (offsets), BHQ_E_NONFINITE (centres),
 * BHQ_E_NOMEM. */
int bhq_set_groups(bhq_ctx *ctx, int64_t ng, const int64_t *i_off,
                   const double (*center)[3], const int64_t *jp_off,
                   const int64_t *jc_off);

/* i-particle positions, ni == i_off[ng], in group order (the coordinates
 * that g5c_calculate_force_on_xMC transmits, Sec. 3.4, List 3).  Errors:
 * BHQ_E_STATE before bhq_set_groups, BHQ_E_ARG for ni != i_off[ng],
 * BHQ_E_NONFINITE, BHQ_E_NOMEM. */
int bhq_set_i(bhq_ctx *ctx, int64_t ni, const double (*x)[3]);

/* j-particles: entries adr .. adr+n-1 of the materialised list arrays
 * (chunked filling allowed; adr + n <= njp): positions and masses, as
 * g5_set_xmjMC sets them (List 4).  Errors: BHQ_E_STATE before
 * bhq_set_groups, BHQ_E_RANGE past njp, BHQ_E_NONFINITE, BHQ_E_NOMEM. */
int bhq_set_jp(bhq_ctx *ctx, int64_t adr, int64_t n, const double (*x)[3],
               const double *m);

/* j-cells: entries adr .. adr+n-1 (adr + n <= njc), as g5c_set_xmjMC
 * sets them (Sec. 3.4, List 3): centre of mass x,
 * total mass m, quadrupole q (List 1 order), and the trace
 * T = sum m |x - com|^2 used by the SPLIT_QUAD kernel (may be NULL for the
 * other kernels; then T = 0). */
int bhq_set_jc(bhq_ctx *ctx, int64_t adr, int64_t n, const double (*x)[3],
               const double *m, const double (*q)[6], const double *trace);

/* Index-mode lists (alternative to bhq_set_jp / bhq_set_jc; the same
 * j-particles and j-cells as List 3's set calls, without a copy per list
 * entry): the j-data
 * live once in two pools and each list entry is an int32 index into them,
 * so neighbouring groups share the data (4 bytes per entry instead of a
 * copy).  After bhq_set_groups the lists are given either materialised or
 * as indices; mixing the two returns BHQ_E_STATE.
 *
 * Particle pool: n particles, x[n][3], m[n].  Cell pool: n cells, centre of
 * mass x, mass m, quadrupole q (List 1 order), trace (NULL: 0).  Setting a
 * pool invalidates the indices given against it (set them again). */
int bhq_set_pool_particles(bhq_ctx *ctx, int64_t n, const double (*x)[3],
                           const double *m);
int bhq_set_pool_cells(bhq_ctx *ctx, int64_t n, const double (*x)[3],
                       const double *m, const double (*q)[6],
                       const double *trace);

/* Index lists: entries adr .. adr+n-1 of the j-particle (resp. j-cell)
 * lists, each an index into the particle (resp. cell) pool.  The pool must
 * be set first; every index is checked on the host (0 <= idx < pool size,
 * else BHQ_E_RANGE), so the kernels never read outside the pools.  adr is a
 * position in the compact lists (group g's entries from jp_off[g]).  Lists
 * that a device rebuild left in per-group slots are first made compact;
 * that waits for all work on the device. */
int bhq_set_jp_idx(bhq_ctx *ctx, int64_t adr, int64_t n, const int32_t *idx);
int bhq_set_jc_idx(bhq_ctx *ctx, int64_t adr, int64_t n, const int32_t *idx);

/* ------------------------------------------------------------------------
 * Device-pointer twins of the set calls above: the same arguments, with
 * every array in device memory of the context's device (torch tensors or
 * hipMalloc'd arrays, each range inside one allocation; BHQ_E_ARG for host
 * memory, BHQ_E_RANGE for a range past the end of its allocation).  The
 * paper's set calls copy host data into the kernel's own structures
 * (Sec. 3.4, List 3); these copy device data the same way, without a host
 * round trip.  Each call waits for the context's last compute, checks the
 * caller's arrays on the device (the same checks as the host twin: finite
 * values, eps2 >= 2^-126, offsets from 0 and monotone, indices inside the pool),
 * and only then copies them into the context with kernels on `stream`
 * (NULL: the null stream).  It returns when the copy is complete: the
 * caller's memory is borrowed for the duration of the call, and may be
 * changed or freed once the call returns.  On a failed check the context
 * is left as it was.
 * ------------------------------------------------------------------------ */

/* bhq_set_groups with i_off, center, jp_off, jc_off in device memory.  The
 * group dispatch order is planned on the device (as for device-built
 * lists).  Also BHQ_E_RANGE for offsets that do not start at 0 or are not
 * monotone, BHQ_E_NONFINITE for centres. */
int bhq_set_groups_dev(bhq_ctx *ctx, int64_t ng, const int64_t *i_off,
                       const double (*center)[3], const int64_t *jp_off,
                       const int64_t *jc_off, void *stream);

/* bhq_set_i with x[ni][3] in device memory (group order). */
int bhq_set_i_dev(bhq_ctx *ctx, int64_t ni, const double (*x)[3], void *stream);

/* bhq_set_eps2_i with eps2[ni] in device memory (the per-particle eps^2 of
 * the i-particle structure, List 2). */
int bhq_set_eps2_i_dev(bhq_ctx *ctx, int64_t ni, const double *eps2, void *stream);

/* bhq_set_jp with x[n][3], m[n] in device memory: j-particle entries
 * adr .. adr+n-1 of the materialised lists (the paper's j-particle set
 * call, Sec. 3.4). */
int bhq_set_jp_dev(bhq_ctx *ctx, int64_t adr, int64_t n, const double (*x)[3],
                   const double *m, void *stream);

/* bhq_set_jc with x[n][3], m[n], q[n][6] (List 1 order), trace[n] (may be
 * NULL) in device memory: j-cell entries adr .. adr+n-1 (the paper's j-cell
 * set call, List 3). */
int bhq_set_jc_dev(bhq_ctx *ctx, int64_t adr, int64_t n, const double (*x)[3],
                   const double *m, const double (*q)[6], const double *trace,
                   void *stream);

/* bhq_set_pool_particles / bhq_set_pool_cells with device arrays. */
int bhq_set_pool_particles_dev(bhq_ctx *ctx, int64_t n, const double (*x)[3],
                               const double *m, void *stream);
int bhq_set_pool_cells_dev(bhq_ctx *ctx, int64_t n, const double (*x)[3],
                           const double *m, const double (*q)[6],
                           const double *trace, void *stream);

/* bhq_set_jp_idx / bhq_set_jc_idx with idx[n] in device memory; every index
 * is checked against its pool on the device (BHQ_E_RANGE). */
int bhq_set_jp_idx_dev(bhq_ctx *ctx, int64_t adr, int64_t n, const int32_t *idx,
                       void *stream);
int bhq_set_jc_idx_dev(bhq_ctx *ctx, int64_t adr, int64_t n, const int32_t *idx,
                       void *stream);

/* Launch the force evaluation on HIP stream `stream` (NULL: the null
 * stream): the forces and potentials of every group's list on its
 * i-particles, as g5_calculate_force_on_xMC and then
 * g5c_calculate_force_on_xMC compute them for one group (Sec. 3.4, Lists 3
 * and 4), for all groups in one launch.  Asynchronous.  Errors: BHQ_E_STATE if groups, i-particles or
 * softening are missing; BHQ_E_HIP on a launch failure. */
int bhq_compute(bhq_ctx *ctx, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the force
 * evaluation of bhq_compute with the context's inputs and launch shape,
 * allocating nothing.  Results go straight to the caller's device arrays
 * a[ni][3] and pot[ni] (FP64, group order; pot may be NULL), which must lie
 * in device memory of the context's device.  The persistent queue counters
 * and the j-split parts live in a static array of the library (256 B plus
 * 16 MiB per device, held until the process ends), so jsplit * ni * 16 B
 * (FP32) or 32 B (FP64) must fit 16 MiB: BHQ_E_RANGE otherwise.  Every call
 * on one device shares that array: calls that overlap in time on one
 * device (two streams, or two host threads) race and give wrong results.
 * No graph is recorded (use_graph is ignored).  Asynchronous on `stream`;
 * bhq_get_kernel_ms times it.  Errors as bhq_compute, plus BHQ_E_ARG / 
 * BHQ_E_RANGE for the output arrays. */
int bhq_compute_noalloc(bhq_ctx *ctx, double *a, double *pot, void *stream);

/* Wait for the last compute and copy out a[ni][3] and pot[ni] (FP64, group
 * order; the arrays ai and pi of List 3).  Either pointer may be NULL.
 * Errors: BHQ_E_STATE before a compute, BHQ_E_HIP. */
int bhq_get_result(bhq_ctx *ctx, double (*a)[3], double *pot);

/* Interaction counts of the current lists: n_pp = sum_g ni_g * njp_g,
 * n_pc = sum_g ni_g * njc_g (the interactions that the paper's throughput
 * counts, Sec. 5.2).  Errors: BHQ_E_ARG, BHQ_E_STATE before bhq_set_groups. */
int bhq_get_counts(const bhq_ctx *ctx, int64_t *n_pp, int64_t *n_pc);

/* Duration in milliseconds of the force kernel(s) of the last compute,
 * measured with HIP events on the compute stream (the force-calculation
 * time of Sec. 5).  Waits for it.  Errors: BHQ_E_STATE before a compute. */
int bhq_get_kernel_ms(bhq_ctx *ctx, double *ms);

/* Measurement support, no counterpart in the paper.
 * For the split kernels (BHQ_SPLIT_QUAD / BHQ_SPLIT_MONO): the number of
 * (i-particle, list entry) pairs of the context's lists that lie inside the
 * cutoff, i.e. that the kernels evaluate rather than mask: *pp for the
 * particle entries, *pc for the cell entries (the decision of the kernels:
 * FP64 offsets to the group centre, 0 < r^2 < rcut^2).  The list counts of
 * bhq_get_counts include the masked pairs too.  Synchronous (one counting
 * kernel).  Errors: BHQ_E_STATE (another kernel, or no lists), BHQ_E_ARG. */
int bhq_count_live(bhq_ctx *ctx, int64_t *pp, int64_t *pc);

/* The GPU's shader clock during other work (measurement support, no
 * counterpart in the paper):
 * bhq_clock_begin launches one wave on `stream` that reads the shader-clock
 * counter and the constant-rate counter, waits until wall_ms (in (0, 10000])
 * of the latter have passed, and reads both again; launch it on a stream of
 * its own just before the work to be observed.  bhq_clock_end waits for it
 * and returns the mean clock of the CU it ran on over that window, in MHz.
 * Errors: BHQ_E_ARG, BHQ_E_STATE (end without begin), BHQ_E_HIP. */
int bhq_clock_begin(bhq_ctx *ctx, double wall_ms, void *stream);
int bhq_clock_end(bhq_ctx *ctx, double *mhz);

/* Launch shape: the autotuner's knobs (ncrit, the other knob, shapes the
 * lists; the group size n_crit is the paper's tuning parameter, Sec. 3.4).
 *   block          threads per block, which is also the depth of one LDS
 *                  tile of list entries: 128 or 256 (0: 256)
 *   i_per_thread   i-particles owned by each thread, so that one LDS read of
 *                  a list entry feeds that many interactions (the paper packs
 *                  i-particles into SIMD registers for the same reuse,
 *                  Sec. 3.3): 1 or 2 (0: 2)
 *   blocks_per_cu  persistent grid size per compute unit, i.e. resident
 *                  blocks (waves) per CU (0: as many blocks as fit), ignored
 *                  when persistent == 0
 *   persistent     0: one block per launch slot of the group order
 *                  (bhq_set_group_order); 1: a machine-sized grid pulls
 *                  groups in that order from device counters
 *   use_graph      1: bhq_compute records its launches into a HIP graph once
 *                  and replays it while kernel, precision, shape and data
 *                  layout are unchanged (re-recorded otherwise)
 *   jsplit         1, 2, 4 or 8 (0: 1): each group's particle and cell lists
 *                  are cut into jsplit parts of nearly equal length, taken by
 *                  different blocks, whose partial sums a second kernel adds
 *                  in part order (for inputs with too few groups to fill the
 *                  GPU, the small-N regime of Sec. 5.2); the context keeps a
 *                  buffer of 32 jsplit ni bytes for the parts
 *   waves_per_eu   0: the compiler's register allocation; 6 or 8: kernel
 *                  instances whose registers are capped so that at least that
 *                  many waves fit on each SIMD (FP32 kernels at block 256;
 *                  FP64 kernels run the compiler's choice)
 * The persistent queue, graph replay and waves_per_eu do not change results
 * (bitwise).  block, i_per_thread and jsplit change how a group's lists are
 * split across threads and blocks and so the order of the FP32/FP64 sums
 * (results agree to rounding).  Errors: BHQ_E_ARG for values outside these
 * sets, or waves_per_eu != 0 with block 128. */
int bhq_set_tuning(bhq_ctx *ctx, int block, int i_per_thread, int blocks_per_cu,
                   int persistent, int use_graph, int jsplit, int waves_per_eu);

/* Current launch shape: out[0..6] = block, i_per_thread, blocks_per_cu,
 * persistent, use_graph, jsplit, waves_per_eu. */
int bhq_get_tuning(const bhq_ctx *ctx, int out[7]);

/* Order in which groups are handed to blocks (no counterpart in the paper,
 * whose driver evaluates one group per call, List 4).  Group g costs
 * c_g = ni_g (100 njp_g + 265 njc_g + 100), in 64-bit integers (a cell term
 * costs about 53/20 of a particle term; the last term stands for loading
 * and storing the i-particles).  Group g of the XCD order goes to piece
 * floor((2 B_g + c_g) / (2 T) xcds), with B_g the exact sum of the costs
 * before g and T their total, evaluated in FP64.
 *   BHQ_ORDER_COST  every group sorted by c_g, largest first (longest
 *                   processing time first: the last blocks are short).
 *   BHQ_ORDER_XCD   the groups, in the order the lists give them (the host
 *                   builder's depth-first order keeps neighbours in space
 *                   together), are cut into BHQ_XCDS contiguous pieces of
 *                   equal total cost.  The last `tail` groups of a piece
 *                   form one window, the groups before them windows of
 *                   `window` consecutive groups; each window is sorted by
 *                   c_g, largest first.  Slot b of the launch takes entry
 *                   b / BHQ_XCDS of piece b % BHQ_XCDS (shorter pieces are
 *                   padded with empty slots): gfx950 hands the blocks of a
 *                   grid to its XCDs round robin, so each piece runs on one
 *                   XCD, and the groups resident together there are
 *                   neighbours that share most list entries in that XCD's
 *                   L2.  The persistent kernel reads its XCD id and drains
 *                   that XCD's piece first, then the others'.  The sorted
 *                   tail keeps the last blocks of each XCD short.
 * The order never changes results (bitwise).  Default: BHQ_ORDER_XCD,
 * window BHQ_ORDER_WINDOW, tail BHQ_ORDER_TAIL.  Applies to the current
 * groups at once (when set) and to later bhq_set_groups calls.
 * Errors: BHQ_E_ARG (mode not 0 or 1, window outside [1, 2^24], tail
 * outside [0, 2^24]); BHQ_E_NOMEM / BHQ_E_HIP while uploading the table,
 * after which the groups must be set again. */
int bhq_set_group_order(bhq_ctx *ctx, int mode, int window, int tail);

/* Current group order: out[0..2] = mode, window, tail.  Errors:
 * BHQ_E_ARG for NULL. */
int bhq_get_group_order(const bhq_ctx *ctx, int out[3]);

/* (No counterpart in the paper.)
 * What the last bhq_build_lists_device(_batch) on ctx did: out[0] = 1 if
 * it walked the tree once (a rebuild: each group's entries went into a slot
 * of 1.25 times an earlier device build's longest list plus 32 entries, and
 * were compacted; the slot size is kept from build to build while that
 * formula gives between 3/4 of it and all of it), 0 if it counted first;
 * out[1], out[2] =
 * the longest particle and cell list of a group.  A rebuild whose groups
 * outgrow their slots, or whose slots would take more than 4 times the
 * previous lists' memory plus 256 MiB, counts first; the lists are the same
 * either way.  All zero before the first device build. */
int bhq_get_build_info(const bhq_ctx *ctx, int64_t out[3]);

/* (No counterpart in the paper: how one launch hands groups to blocks.)
 * The launch slot table in use (the order above applied to the current
 * groups): order[b] is the group of slot b or -1.  Lists built on the
 * device get their table computed on the device (for windows and tails up
 * to 1024), equal entry for entry to bhq_plan_order on their offsets.
 * order may be NULL to query *nslots; otherwise it holds cap entries
 * (host memory).  Errors: BHQ_E_ARG (null nslots), BHQ_E_STATE (no
 * groups), BHQ_E_RANGE (cap too small), BHQ_E_HIP. */
int bhq_get_order(bhq_ctx *ctx, int32_t *order, int64_t cap, int64_t *nslots);

/* The slot table of a dispatch order, computed on the host for offsets
 * i_off, jp_off, jc_off of ng >= 1 groups (as bhq_set_groups takes them),
 * with xcds in [1, 64] pieces: order[b] is the group of launch slot b, or
 * -1 for an empty slot.  BHQ_ORDER_COST gives ng slots; BHQ_ORDER_XCD
 * gives xcds * (the longest piece) slots, at most xcds * ng.  order may be
 * NULL to query *nslots; otherwise it holds cap entries.
 * Errors: BHQ_E_ARG (null pointer, ng, mode, window, tail or xcds out of
 * range), BHQ_E_RANGE (offsets not starting at 0 or not monotone, cap too
 * small), BHQ_E_NOMEM. */
int bhq_plan_order(int64_t ng, const int64_t *i_off, const int64_t *jp_off,
                   const int64_t *jc_off, int mode, int window, int tail,
                   int xcds, int32_t *order, int64_t cap, int64_t *nslots);

/* (No counterpart in the paper.)
 * Message for the last error on ctx (never NULL; "" when none).  With
 * ctx == NULL: the message of the last failed bhq_create on this thread. */
const char *bhq_last_error(const bhq_ctx *ctx);

/* ------------------------------------------------------------------------
 * Host-side tree and list construction (not the accelerated path; it
 * produces the inputs).  Oct-tree over the particles (Sec. 1), cell
 * moments M, centre of mass, Q (eq. 2) and trace, groups = the largest
 * tree cells holding at most ncrit particles (Sec. 3.4), and for each
 * group the list of j-cells accepted by l^2 < theta^2 d^2 (d: centre of
 * mass to the nearest point of the group's cell) and of j-particles from
 * the opened leaves.  The root is the cube on the bounding-box midpoint
 * with side = largest extent * (1 + 2^-20) (or [0, box)^3 when box > 0,
 * with minimum-image distances and cells farther than rcut pruned).
 * Particles go to the upper half of a cell along an axis iff their
 * coordinate is >= the cell centre; cells with more than nleaf particles
 * are split, down to depth 21.
 * ------------------------------------------------------------------------ */

/* Build the lists.  n >= 1 particles x[n][3], m[n] (FP64); theta >= 0;
 * ncrit >= 1; nleaf in [1, ncrit]; box >= 0; rcut >= 0 (0: no pruning).
 * nthreads <= 0 uses all hardware threads.  *out owns the result. */
int bhq_build_lists(int64_t n, const double (*x)[3], const double *m,
                    double theta, int ncrit, int nleaf, double box,
                    double rcut, int nthreads, bhq_lists **out);

/* Build lists for nsys independent systems in one object (for one batched
 * launch; no counterpart in the paper, which evaluates one system): system s is particles sys_off[s] .. sys_off[s+1]-1 of x and m
 * (sys_off[0] == 0, strictly increasing), open boundaries, one theta and
 * ncrit for all.  Each system gets its own tree; groups, i-particles and
 * list entries of system s follow those of system s-1, and every index in
 * the exported lists refers to the concatenated arrays.  Per-system
 * softening is given afterwards with bhq_set_eps2_i. */
int bhq_build_lists_batch(int64_t nsys, const int64_t *sys_off,
                          const double (*x)[3], const double *m, double theta,
                          int ncrit, int nleaf, int nthreads, bhq_lists **out);

/* sizes[0..3] = ng, njp, njc, number of tree cells. */
int bhq_lists_sizes(const bhq_lists *L, int64_t sizes[4]);

/* Copy the lists out (any pointer may be NULL):
 *   i_idx[n]          original index of the k-th i-particle (group order)
 *   i_off[ng+1], center[ng][3] (group cell centre), side[ng]
 *   jp_off[ng+1], jp_idx[njp]   (original particle indices)
 *   jc_off[ng+1], jc_cell[njc]  (tree cell ids)                          */
int bhq_lists_export(const bhq_lists *L, int64_t *i_idx, int64_t *i_off,
                     double (*center)[3], double *side, int64_t *jp_off,
                     int64_t *jp_idx, int64_t *jc_off, int32_t *jc_cell);

/* Copy out cell moments for cells 0..ncell-1 (any pointer may be NULL):
 * com[][3], mass[], q[][6], trace[]. */
int bhq_lists_cells(const bhq_lists *L, double (*com)[3], double *mass,
                    double (*q)[6], double *trace);

/* Upload the lists into a context: groups, i-particles (x gathered into
 * group order), the materialised j-particles and j-cells with their
 * moments.  x, m are the arrays the lists were built from. */
int bhq_set_lists(bhq_ctx *ctx, const bhq_lists *L, const double (*x)[3],
                  const double *m);

/* The same upload as index lists: the particle pool holds x, m in tree
 * order (entry k is input particle i_idx[k], the order bhq_lists_export
 * gives), the cell pool the tree cells; list entries are pool indices. */
int bhq_set_lists_indexed(bhq_ctx *ctx, const bhq_lists *L,
                          const double (*x)[3], const double *m);

/* Free lists (NULL accepted). */
int bhq_lists_free(bhq_lists *L);

/* ------------------------------------------------------------------------
 * Device-side tree and list construction: the same tree, groups and lists
 * as bhq_build_lists (same cells in the same breadth-first numbering, same
 * moments bit for bit, same groups, same list entries in the same order),
 * built on the GPU from particles already in device memory and left in
 * the context as index lists, ready for bhq_compute.
 * ------------------------------------------------------------------------ */

/* Build on ctx's device: n in [1, 2^31) particles, x[n][3] and m[n] FP64 in
 * device memory of that device (each range must lie inside one
 * allocation); theta >= 0, ncrit >= 1, nleaf in [1, ncrit], box >= 0,
 * rcut >= 0 as for bhq_build_lists.  Runs on `stream` (NULL: the default
 * stream) and returns when the lists are complete; the context then holds
 * the groups, i-particles, pools and lists (tree order) as
 * bhq_set_lists_indexed would leave them, and keeps its softening if it
 * was set with bhq_set_eps.  x and m are not kept.
 * Errors: BHQ_E_ARG (arguments, pointers that are not device memory),
 * BHQ_E_RANGE (a range outside its allocation, more than 2^31 cells),
 * BHQ_E_NONFINITE (a non-finite position or mass), BHQ_E_NOMEM, BHQ_E_HIP.
 * After a failure the context holds no lists. */
int bhq_build_lists_device(bhq_ctx *ctx, int64_t n, const double *x,
                           const double *m, double theta, int ncrit,
                           int nleaf, double box, double rcut, void *stream);

/* The same for nsys independent systems in one context, as
 * bhq_build_lists_batch builds them: system s is particles sys_off[s] ..
 * sys_off[s+1]-1 (host array, sys_off[0] == 0, strictly increasing, at
 * most 2^20 systems and 2^31 - 1 particles), open boundaries, one root per
 * system from its own bounding box; cells are numbered system by system.
 * eps2 (device, may be NULL) gives each particle's squared softening in
 * input order: the context then holds it in group order, as bhq_set_eps2_i
 * would (values must be finite and >= 2^-126: BHQ_E_ARG otherwise).
 * Errors as bhq_build_lists_device, BHQ_E_RANGE for bad offsets. */
int bhq_build_lists_device_batch(bhq_ctx *ctx, int64_t nsys,
                                 const int64_t *sys_off, const double *x,
                                 const double *m, const double *eps2,
                                 double theta, int ncrit, int nleaf,
                                 void *stream);

/* Sizes of the index lists a context holds: out[0..3] = groups, j-particle
 * entries, j-cell entries, cells in the cell pool.  BHQ_E_STATE without
 * index lists. */
int bhq_get_lists_sizes(const bhq_ctx *ctx, int64_t out[4]);

/* Copy a context's index lists to the host, in bhq_lists_export's layout:
 * i_idx[n] (input index of the k-th i-particle; only for lists from
 * bhq_set_lists_indexed or bhq_build_lists_device), i_off, jp_off, jc_off
 * [ng + 1], jp_idx[njp] (input particle indices for those lists, pool
 * indices otherwise), jc_idx[njc] (cell pool indices = cell ids).  Any
 * pointer may be NULL.  Errors: BHQ_E_STATE, BHQ_E_HIP, BHQ_E_NOMEM. */
int bhq_get_lists(bhq_ctx *ctx, int64_t *i_idx, int64_t *i_off,
                  int64_t *jp_off, int64_t *jp_idx, int64_t *jc_off,
                  int32_t *jc_idx);

/* Copy the cell pool to the host, as bhq_lists_cells gives it (any pointer
 * may be NULL).  Errors: BHQ_E_STATE (no cell pool), BHQ_E_HIP. */
int bhq_get_cells(bhq_ctx *ctx, double (*com)[3], double *mass,
                  double (*q)[6], double *trace);

/* ------------------------------------------------------------------------
 * Around the force evaluation in a time step (leapfrog, as the paper's
 * cold-collapse runs integrate, Sec. 5.2).  Arrays are FP64 in device
 * memory of ctx's device, particles in input order, x and v as [n][3].
 * ------------------------------------------------------------------------ */

/* Copy the last compute's accelerations a[ni][3] and potentials pot[ni]
 * (pot may be NULL) to device arrays in the particles' input order (for
 * lists from bhq_set_lists_indexed or bhq_build_lists_device; in group order
 * otherwise).  Runs on `stream` after the compute (it waits for it).
 * Errors: BHQ_E_STATE (no compute yet), BHQ_E_ARG / BHQ_E_RANGE (pointers),
 * BHQ_E_HIP. */
int bhq_get_result_device(bhq_ctx *ctx, double *a, double *pot, void *stream);

/* Put the caller's particle arrays into the tree order of the current lists
 * (built by bhq_build_lists_device(_batch) or set by bhq_set_lists_indexed):
 * each of the nf <= 16 arrays fields[f] (device memory, n rows of
 * row_bytes[f] bytes, a multiple of 8 from 8 to 64) is permuted in place so
 * that row k holds the particle at tree position k.  n must be the
 * particle count of the lists.  From then on the lists refer to the arrays
 * in that order: bhq_get_result_device writes row k for tree position k,
 * and bhq_get_lists reports the identity as i_idx.  For callers that keep
 * their particles in tree order between rebuilds (time stepping), so that
 * the next build reads them nearly in order.  Runs on `stream` after the
 * last bhq_compute, and returns when done.  Errors: BHQ_E_STATE (no lists
 * with a tree order), BHQ_E_ARG (n, nf, a field or its row size),
 * BHQ_E_RANGE (an array that is not device memory of that size),
 * BHQ_E_NOMEM / BHQ_E_HIP. */
int bhq_sort_to_tree_order(bhq_ctx *ctx, int64_t n, int nf, void *const *fields,
                           const int *row_bytes, void *stream);

/* Leapfrog step pieces on n particles: v += dt_kick * a, then, unless
 * dt_drift == 0, x += dt_drift * v (x may be NULL then).  A kick-drift-kick
 * step is kick_drift(dt/2, dt), forces, kick_drift(dt/2, 0); consecutive
 * steps merge the two half kicks into kick_drift(dt, dt).  Asynchronous on
 * `stream`.  Errors: BHQ_E_ARG, BHQ_E_RANGE, BHQ_E_NONFINITE, BHQ_E_HIP. */
int bhq_kick_drift(bhq_ctx *ctx, int64_t n, double *x, double *v,
                   const double *a, double dt_kick, double dt_drift,
                   void *stream);

/* Periodic images: every coordinate x <- x - box floor(x / box), then
 * x - box once more if rounding left it equal to box, so that x is in
 * [0, box) (as the periodic tree builders need).  Asynchronous on
 * `stream`.  Errors: BHQ_E_ARG (box <= 0), BHQ_E_RANGE, BHQ_E_HIP. */
int bhq_wrap_periodic(bhq_ctx *ctx, int64_t n, double *x, double box,
                      void *stream);

/* Energies of n particles: out[0] = K = 1/2 sum m |v|^2 and, when pot is
 * given (the potentials of the softened kernels, which include each
 * particle's self pair -m/eps), out[1] = W = 1/2 sum m (pot + m / eps);
 * out[1] = 0 without pot.  eps >= 0 (0: nothing removed).  Deterministic
 * (fixed-order reduction); waits for the result.
 * Errors: BHQ_E_ARG, BHQ_E_RANGE, BHQ_E_HIP. */
int bhq_energies(bhq_ctx *ctx, int64_t n, const double *m, const double *v,
                 const double *pot, double eps, double out[2], void *stream);

/* ------------------------------------------------------------------------
 * Particle-mesh long-range force: with the short-range split kernels
 * (pair potential -erfc(r / 2 r_s) / r) it makes a TreePM force (the
 * TreePM context of Sec. 1).  The long-range pair potential is
 * -erf(r / 2 r_s) / r, in the periodic box of side L with the mean density
 * removed (G = 1).  Method: triangular-shaped-cloud (TSC) assignment to an
 * n^3 mesh (mesh points at multiples of L / n), FFT, multiplication by
 * -4 pi exp(-k^2 r_s^2) / k^2 divided by the squared TSC window
 * prod sinc(k_a L / 2n)^6, gradient -i k (zero on the Nyquist planes),
 * inverse FFTs, TSC interpolation.  FP64 throughout; hipFFT for the FFTs.
 * The potential includes each particle's own smoothed long-range term
 * (about -m / (r_s sqrt(pi))).
 * ------------------------------------------------------------------------ */
typedef struct bhq_pm bhq_pm;

/* n: even mesh size in [4, 1024]; box > 0; rs > 0 (the split scale of
 * bhq_set_split).  Allocates the real, complex and interleaved meshes and
 * the FFT plans on `device`.  Errors: BHQ_E_ARG, BHQ_E_NODEV, BHQ_E_NOMEM, BHQ_E_HIP;
 * bhq_pm_last_error(NULL) describes a failed create. */
int bhq_pm_create(bhq_pm **out, int device, int nmesh, double box, double rs);

/* Waits for outstanding work and frees everything (NULL accepted). */
int bhq_pm_destroy(bhq_pm *pm);

/* Long-range acceleration and potential of n particles, x[n][3] (in
 * [0, box) or any periodic image) and m[n] in device memory: writes, or
 * with accumulate = 1 adds to, a[n][3] and pot[n] (pot may be NULL), in
 * the order of x.  The mass assignment gathers particles sorted by their
 * nearest mesh point in a fixed order, so results are bitwise reproducible.
 * Asynchronous on `stream`.  Errors: BHQ_E_ARG,
 * BHQ_E_RANGE (pointers), BHQ_E_HIP. */
int bhq_pm_compute(bhq_pm *pm, int64_t n, const double *x, const double *m,
                   double *a, double *pot, int accumulate, void *stream);

/* Duration of the last bhq_pm_compute in milliseconds (HIP events on its
 * stream); waits for it.  Errors: BHQ_E_STATE before any compute. */
int bhq_pm_get_ms(bhq_pm *pm, double *ms);

/* Message of the last error on pm (never NULL; with pm == NULL: the last
 * failed bhq_pm_create on this thread). */
const char *bhq_pm_last_error(const bhq_pm *pm);

#ifdef __cplusplus
}
#endif

#endif /* BHQ_H */
