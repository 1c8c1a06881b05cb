"""MI355X (gfx950) implementation of Optimised Annealed SMC / OAIS
(Syed, Bouchard-Cote, Chern, Doucet, arXiv 2408.12057).

The compute runs in hand-written HIP kernels behind the C ABI of
``include/oasmc.h`` (``liboasmc.so``, built in-tree by ``build.py``).  This
package only marshals arguments: torch supplies device memory and the stream.
Importing the package does not load the library; the first call does, and it
raises if the library is missing.
"""
from .api import (  # noqa: F401
    Problem, asmc, adapt_schedule, dar_times, rejuvenate, zja, pt, autotune, shape, run, resample, resample_noalloc, philox, logreg_eval, target_eval, profile,
    library_path,
    OasmcError, logZ_backward, LogZ, BatchItem, run_batch,
)
