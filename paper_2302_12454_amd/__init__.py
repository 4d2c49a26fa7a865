"""MI355X-native stochastic simulated quantum annealing (SSQA).

The sweep (Eq. 6a-c of the paper) runs in hand-written gfx950 HIP kernels in
libssqa.so behind the C ABI of include/ssqa.h; ``api`` is its Python binding.
Importing the package does not load the library; the first call does, and fails
loudly if it has not been built.
"""

from .api import (  # noqa: F401
    SSQA_NO_TARGET,
    AnnealResult,
    AnnealState,
    Batch,
    Problem,
    SAResult,
    Server,
    SSQAError,
    ssqa_anneal,
    ssqa_anneal_noalloc,
    ssqa_batch_create,
    ssqa_create_problem,
    ssqa_energy,
    ssqa_gi_to_ising,
    ssqa_jperp_schedule,
    ssqa_philox4x32_10,
    ssqa_qmc_energy,
    ssqa_sa_accept_threshold,
    ssqa_sa_anneal,
    ssqa_sa_schedule,
    ssqa_server_create,
    ssqa_ssa_i0_schedule,
    ssqa_tune_anneal,
    ssqa_tune_batch,
    ssqa_tune_clear,
    ssqa_tune_entries,
    ssqa_tune_load,
    ssqa_tune_lookup,
    ssqa_tune_save,
    ssqa_tune_set,
)
