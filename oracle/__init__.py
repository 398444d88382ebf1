"""FP64 CPU oracle for Barnes-Hut tree forces with monopole and traceless
quadrupole cell terms (Kodama & Ishiyama, arXiv:1812.07313, Sec. 1, Sec. 3
eqs. 1-7, Sec. 3.4, Sec. 4 eq. 8).

TEST INFRASTRUCTURE ONLY: this package is the checker.  Only the test suite,
the smoke check and the CPU-baseline leg of the benchmark may import it.  It
shares no code with the GPU library and is never called by it.
"""
from .oracle import (  # noqa: F401
    MONO, QUAD, SPLIT_QUAD, SPLIT_MONO, QUAD_SOFT, MASK_ABS, MASK_F64_OFS,
    split_keep, mask_flips, count_keep,
    build, lib, Tree, build_tree, eval_lists, direct, moments, pp_plummer,
    pc_quad, pc_quad_soft, pc_mono, pc_split, pp_split, split_derivs, num_threads,
    set_threads,
    materialise, relative_errors, leapfrog,
)
