"""MI355X-native all-pairs Stokesian-dynamics mobility product (HIP, gfx950).

The compute path lives in the HIP shared library libsd.so built from
``csrc/`` (``python -m paper_1205_6333_amd.build``); the functions exported
here only marshal arguments to its C ABI (include/sd.h).  Importing the
package does not load the library; the first call does, and fails loudly if
the library is missing.  Seeded synthetic inputs are in ``workloads``.
"""
from .binding import (SD_AB2, SD_EULER, SD_FP32_KAHAN, SD_FP32_PLAIN, SD_FP64, SD_OSEEN,  # noqa
                      SD_OVERLAP_NONE, SD_OVERLAP_RPY, SD_RPY, Batch, SdError, lib,
                      mobility_adjoint, mobility_apply, mobility_apply_batched,
                      mobility_apply_noalloc, params,
                      sd_autotune, sd_autotune_clear, sd_get_kernel_config, sd_profile_enable,
                      sd_profile_read,
                      sd_profile_reset, sd_profile_times, sd_release, sd_run, sd_run_adjoint,
                      sd_run_batched,
                      sd_set_kernel_config, sd_step, sd_version)
from .binding import (lub, lubrication_forces, sd_mean_vector, sd_pack,  # noqa: E402,F401
                      sd_premise_counts, sd_run_lub)
from . import autograd  # noqa: E402,F401
from .binding import (SD_ACC_DS, SD_ACC_FP32, SD_ACC_FP64, SD_ACC_KAHAN, SD_POS_DS,  # noqa: E402,F401
                      SD_POS_FP32, SD_POS_FP64, cluster_frames, sd_cluster_run)
from .binding import (SD_MB_LINEAR, SD_MB_NAIVE, SD_MB_SMALLTILING, SD_MB_STRIDED,  # noqa: E402,F401
                      SD_MB_TILING, SD_MB_UNORDERED, sd_membench)
from .binding import sd_set_graph_mode  # noqa: E402,F401
