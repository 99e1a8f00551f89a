"""MI355X-native hybrid FE/FD time-domain Maxwell solver (forward, adjoint, gradient).

The compute path is the HIP library libddfem.so behind the C-ABI of include/dd.h;
this package only marshals arguments (torch supplies device memory and streams).
"""

from ._lib import DDError, load as load_library  # noqa: F401
from .solver import Problem  # noqa: F401
from .cga import CGA, CGAParams  # noqa: F401
