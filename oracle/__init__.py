"""CPU FP64 oracle for the quasi-2D Ewald sums of arXiv:2403.01521.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may.  It shares no code, header, table or constant
generator with the GPU library: the only thing both sides consume is the
seeded input generator module (``workloads``), which holds none of the
method's arithmetic.

Contents (each function cites the passage of the paper it follows):

* ``soe``        -- a sum-of-exponentials fit of the Gaussian by a Talbot-contour
                    quadrature of its inverse-Laplace representation (Sec. 3,
                    the representation preceding the SOE approximations of xi).
* ``ewald2d``    -- O1, the exact Ewald2D sum: erfc real space, the spectral
                    Fourier modes with xi^+ + xi^- (Lemma 2.4), the k = 0 term
                    and the self term (Sec. 2.2).
* ``soewald2d``  -- O2, the SOE-approximated Ewald2D written as plain direct
                    pair sums (Sec. 3.2 pair kernels, App. E force kernels),
                    for all k in a cutoff or for a given random batch of modes
                    weighted as in the importance-sampling estimator (Sec. 4.1).
* ``recursion``  -- O3, the O(N) z-sorted recursion of Sec. 3.2 (and its
                    mirror twin for the j > i half) in plain C, FP64.
* ``rbsampler``  -- Philox4x32-10 and the Metropolis mode sampler (App. G),
                    and the normaliser H (Sec. 4.1).
* ``lattice``    -- brute-force direct lattice sums (Sec. 2.1, Thm 2.1),
                    used to pin O1 on tiny inputs.
* ``slabs``      -- the particle-slab term of charged walls (Sec. 2.4, Thm 2.7
                    and eq. spectial) and a BAOAB step of the Langevin
                    dynamics of Sec. 4.3.

Every function here is plain and slow on purpose.  Parity status of each
function (what pins it) is listed in the header of its module.
"""

from . import soe, ewald2d, soewald2d, rbsampler, lattice, slabs  # noqa: F401
