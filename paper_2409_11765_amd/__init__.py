"""MI355X (gfx950) IPOP-CMA-ES generation path.

Python side of the C ABI in include/cmaes_mi355x.h (see ``binding``).  The
package loads its in-tree HIP library on import and fails loudly if it is
missing; nothing here computes a CMA-ES step on the host.
"""

from .binding import (CMAES, CMAESBatch, CmaesError, CmaesOptions, KERNELS, OBJECTIVES, PHASES, PRECISIONS, STOP_BITS,  # noqa: F401
                      cmaes_ask, cmaes_create, cmaes_default_options, cmaes_destroy, cmaes_enable_timing,
                      cmaes_generation, cmaes_generation_with_z, cmaes_get_options, cmaes_ipop_run,
                      cmaes_kernel_times, cmaes_enable_kernel_timing, cmaes_last_error, cmaes_phase_times, cmaes_restart_ipop, cmaes_set_objective,
                      cmaes_set_options, cmaes_set_state, cmaes_state, cmaes_tell, library, LIB_PATH,
                      cmaes_batch_best, cmaes_batch_count, cmaes_batch_create, cmaes_batch_destroy,
                      cmaes_batch_generation, cmaes_batch_set_objective, cmaes_batch_set_options,
                      cmaes_batch_state, SITES, cmaes_autotune, cmaes_device_arch, cmaes_syrk_plan, cmaes_gemm_config_count,
                      cmaes_gemm_config_info, cmaes_get_gemm_config, cmaes_set_gemm_config,
                      cmaes_enable_graphs, cmaes_batch_enable_graphs, cmaes_set_eigen_correction, KReplicated, cmaes_krep_create,
                      cmaes_krep_destroy, cmaes_krep_generation, cmaes_krep_run, cmaes_krep_set_objective,
                      cmaes_krep_set_options, cmaes_krep_status)
