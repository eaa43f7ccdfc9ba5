"""CPU FP64 oracle for the SamBaTen batch update.

SamBaTen: Sampling-based Batch Incremental Tensor Decomposition (Gujral,
Pasricha, Papalexakis).  The oracle is a plain, slow, deliberately simple
NumPy/SciPy implementation of what one update computes (Sec. 3, Algorithm 1)
plus the CP-ALS it relies on (Sec. 2.1) and the relative error of Sec. 4.2.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke entry
point and the CPU-baseline leg of the benchmark may import it.  The HIP
library never calls it and shares no code with it: where both sides need the
same random numbers, each implements Philox4x32-10 (Salmon et al., SC'11) and
the logarithm on its own from the published definitions.

Modules
-------
rng       Philox4x32-10, 53-bit uniforms, the basic-operation logarithm.
cp        unfoldings, Khatri-Rao, MTTKRP, normal-equation solve, CP-ALS, fit.
sambaten  measure of importance, weighted sampling, summaries, matching,
          row solve, zero-fill, averaging: the batch update itself.
nmode     the same update for a tensor of any order N >= 3 whose last mode
          grows (Sec. 2 notes that the method carries over).
"""


