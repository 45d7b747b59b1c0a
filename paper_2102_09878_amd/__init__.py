"""MI355X-native spaQR least-squares hot path (arXiv 2102.09878).

The compute lives in libspaqr.so (HIP kernels for gfx950 behind the C-ABI of
include/spaqr.h); ``spaqr`` is its thin Python binding and ``autograd`` the
torch.autograd.Function of the least-squares solution.
"""
from .spaqr import (BatchSolver, Solver, SpaqrError, load, spaqr_adjoint, spaqr_batch_analyze, spaqr_batch_cgls,
                    spaqr_batch_info, spaqr_analyze, spaqr_apply, spaqr_apply_op,  # noqa: F401
                    spaqr_cgls, spaqr_destroy, spaqr_factor_stats, spaqr_factorize,
                    spaqr_factorize_forced, spaqr_get_op, spaqr_get_ordering, spaqr_get_ranks,
                    spaqr_set_values, spaqr_time_kernel)
from .autograd import LstsqFunction, lstsq  # noqa: F401,E402
