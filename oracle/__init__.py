"""CPU oracle for stochastic simulated quantum annealing (SSQA).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import this package.  The HIP
library never calls it and it never calls the HIP library; the two share no
code.  The only shared module is ``synth`` (seeded random graphs), which holds
none of the method's arithmetic.

The oracle is a plain, slow, step-by-step restatement of the paper in exact
integer arithmetic (numpy int64; the per-cycle product J.sigma is a float64
matrix product, which is exact because every partial sum is an integer far
below 2**53):

* ``philox``  Philox4x32-10 (Salmon et al., SC'11) and the noise-stream layout.
* ``gi``      GI QUBO (Eq. 8), QUBO form (Eq. 7), the QUBO-to-Ising mapping of
              Section 4.2, the integer scale S and the closed-form ground energy.
* ``ssqa``    J_perp and I_0 schedules (Section 4.2, Table 2; Section 4.4 for
              SSA), the SSQA update (Eq. 6a-c), SSA (Eq. 2a-c), the problem
              Hamiltonian (Eq. 1 / Eq. 5) and the QMC Hamiltonian (Eq. 4).
* ``metrics`` success probability over trials and time-to-solution (Eq. 10),
              equivalent cycles (Eq. 9).
* ``sa``      the traditional simulated-annealing baseline of Section 4.4 and
              Table 4 (serial single-spin Metropolis).

Parity status: every function here is pinned by a ``-m "not gpu"`` test to
something other than itself (published test vectors, brute force, closed forms,
special cases, values printed in the paper); see the test files.
"""

from . import gi, metrics, philox, sa, ssqa  # noqa: F401
