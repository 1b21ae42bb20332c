"""MI355X micromagnetic Monte Carlo (MMC) with variable magnetization length.

The compute path is the HIP library libmmc.so (C-ABI in include/mmc.h); this
package holds its sources (csrc/), the build script and a thin ctypes binding.
"""
from .mmc import (Batch, Chain, MMCError, MMC_DEMAG_FP32, MMC_DEMAG_OFF, MMC_DEMAG_SPLIT_BF16,  # noqa: F401
                  MMC_DEMAG_SPLIT_FP16, MMC_ERR_ARG, MMC_ERR_DEVICE, MMC_ERR_DOMAIN, MMC_ERR_OOM, MMC_ERR_STATE,
                  MMC_ERR_UNSUPPORTED, MMC_LEN_EXACT, MMC_LEN_PAPER, MMC_MF_BRILLOUIN_HALF, MMC_MF_LANGEVIN, MMC_SCHED_AUTO,
                  MMC_SCHED_GROUPS, MMC_SCHED_PERSISTENT, MUB, lib)
