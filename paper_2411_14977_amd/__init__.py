"""MI355X (gfx950) spectral-element pressure-Poisson solver with p-multigrid.

Thin Python binding over the C ABI of ``libsem.so`` (declared in ``include/sem.h``): argument
marshalling only.  Every step of the solve runs in the library's HIP kernels; PyTorch provides
device memory and the stream.  Importing this package does not load the library; the first call
that needs it does, and raises ``RuntimeError`` if it has not been built
(``python -m paper_2411_14977_amd.build``).  There is no CPU fallback.
"""
from .binding import (  # noqa: F401
    SEM_F32, SEM_F32_GBF16, SEM_F64, SEM_OUTER_FPCG, SEM_OUTER_PDC, SEM_SMOOTH_CHEBYSHEV,
    SEM_SMOOTH_JACOBI, SemError, SolveInfo, Solver, lib, lib_path, sem_apply_laplacian,
    sem_apply_level, sem_assemble_rhs, sem_coarse_solve, sem_destroy, sem_get_level,
    sem_get_sizes, sem_gll, sem_mesh_desc_default, sem_mesh_setup, sem_node_coords,
    sem_num_levels, sem_pmg_vcycle, sem_poisson_solve, sem_prolong_add, sem_restrict,
    sem_set_smoother_bounds, sem_smooth, fine_x_nodes, sem_time_operator,
    sem_operator_bytes, sem_mlp_blob_size, sem_learned_features, sem_mlp_train, sem_mlp_forward,
    sem_mlp_gradients, sem_learned_load, sem_learned_enable, sem_learned_stage, blob_pack,
    blob_unpack,
)
