"""FP64 CPU oracle (test infrastructure only; see pd_oracle's header).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The HIP product path never does.
"""
from .pd_oracle import *  # noqa: F401,F403
from .pd_oracle import __all__ as _l1_all
from .pd_tv_oracle import *  # noqa: F401,F403
from .pd_tv_oracle import __all__ as _tv_all

__all__ = list(_l1_all) + list(_tv_all)
