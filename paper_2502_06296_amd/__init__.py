"""MI355X channel pressure-Poisson and wall-normal Helmholtz solvers
(arXiv 2502.06296), as hand-written HIP kernels behind a C ABI.

    from paper_2502_06296_amd import poisson_plan, poisson_solve, pcr_prepare, pcr_apply

The library libpf_channel.so is built in-tree by ``paper_2502_06296_amd.build``;
importing this package does not load it, the first call does (and fails
loudly if it is missing).
"""
from .solver import (  # noqa: F401
    BCS, PRECISIONS, Graph, PcrPlan, PoissonPlan, grid_faces, helmholtz3d_plan, helmholtz3d_solve,
    helmholtz3d_update, pcr_apply, pcr_apply_batched,
    pcr_prepare, pcr_prepare_rows, pcr_set_stream, pcr_timing, pcr_timing_read, pcr_update_coef, pf_copy_kernel,
    pf_graph_begin, pf_graph_end, poisson_plan, poisson_project, poisson_set_status, poisson_set_stream,
    read_status,
    poisson_solve, poisson_solve_batched, poisson_solve_noalloc, poisson_timing, poisson_timing_read, run_batched, zop_rows)
