// bhq_internal.h -- shared between the C-ABI layer (bhq_api.cpp) and the
// HIP kernels (bhq_kernels.hip).  Not part of the public ABI.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime_api.h>

namespace bhq {

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
    double *ax, *ay, *az, *pot;     // [ni] results (FP64)
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
};

// Launch the force kernel for (kernel, precision) on `stream`.  Returns
// the launch status.
hipError_t launch_force(int kernel, int precision, const ForceArgs &args,
                        const LaunchCfg &cfg, hipStream_t stream);

}  // namespace bhq
