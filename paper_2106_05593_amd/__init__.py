"""MI355X micromagnetic Monte Carlo (MMC) with variable magnetization length.

The compute path is the HIP library libmmc.so (C-ABI in include/mmc.h); this
package holds its sources (csrc/), the build script and a thin ctypes binding.
"""
from .mmc import (Batch, Chain, MMCError, MMC_DEMAG_FP32, MMC_DEMAG_OFF, MMC_LEN_EXACT, MMC_LEN_PAPER,  # noqa: F401
                  MMC_MF_BRILLOUIN_HALF, MMC_MF_LANGEVIN, MUB, lib)
