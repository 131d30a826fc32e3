"""MI355X (gfx950) evaluation of the muSR chi^2 and Poisson-likelihood costs.

The HIP library ``libmu.so`` (built from csrc/ by ``build.py``) implements the
C ABI of include/mu.h; this package binds it with ctypes and adds a
``torch.autograd.Function`` whose backward pass is the library's adjoint
gradient kernel.  There is no CPU fallback: without the built library or a
GPU every entry point raises.
"""

from ._abi import MuError, lib  # noqa: F401
from .api import (  # noqa: F401
    Context,
    Data,
    Theory,
    autotune,
    chi2_batch,
    chi2_eval,
    chi2_grad,
    fit_batch,
    histo_check,
    model_eval,
    theory_check,
)
from .autograd import Chi2  # noqa: F401
from .seeder import Seeder, gen_histos  # noqa: F401
