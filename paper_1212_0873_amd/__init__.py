"""MI355X-native synchronous parallel coordinate descent (PCDM1) for the LASSO.

The method runs in the HIP library ``libpcdm.so`` (C ABI in include/pcdm.h);
this package only binds it.  Importing the package does not load the
library; the first call that needs it does, and raises ImportError if it has
not been built.
"""

from ._lib import (EXPORTS, LIB_PATH, PCDM_BF16, PCDM_F32, PCDM_F64, PCDMError,  # noqa: F401
                   load)
from .api import Batch, Problem, current_stream, sample, sample_draw  # noqa: F401
