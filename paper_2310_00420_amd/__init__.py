"""MI355X (gfx950) implementation of the hot path of covariance-free EM (CoFEM) for clustered
multi-task compressive sensing (Lin & Ba, arXiv 2310.00420).

The computation lives in the HIP library ``libcmtcs.so`` (C ABI: ``include/cmtcs.h``); this
package only loads it and marshals arguments.  Importing :mod:`.api` fails loudly when the
library has not been built.
"""

from .api import Cmtcs, fit, MATH, CGSolve, PosteriorMean  # noqa: F401
from ._lib import CmtcsError, load  # noqa: F401

__all__ = ["Cmtcs", "fit", "MATH", "CGSolve", "PosteriorMean", "CmtcsError", "load"]
