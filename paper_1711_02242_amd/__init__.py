"""MI355X-native phaseless AFQMC hot path (arXiv:1711.02242) behind a C ABI.

The compute path is the HIP library ``libafqmc.so`` (built by
``paper_1711_02242_amd.build``); ``System`` and ``Walkers`` only marshal
arguments to it.  There is no CPU fallback: without the library or a GPU the
calls raise.
"""

from ._lib import AfqmcError, EXPORTS, KERNEL_GROUPS, LIB_PATH, PRECISIONS, load  # noqa: F401
from .afqmc import Batch, System, Walkers, mfma_peak, modified_cholesky  # noqa: F401
