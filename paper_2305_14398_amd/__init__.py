"""MI355X-native unitary-matrix quantum-circuit simulation (hot path of arXiv 2305.14398).

The compute path lives in the HIP library ``libqsim.so`` (built from ``csrc/``)
behind a C ABI declared in ``include/qsim.h``; ``binding`` is its thin ctypes
binding and ``workloads`` the seeded circuit generators.  Importing this
package does not load the library; ``binding.lib()`` does, and raises if the
library has not been built.
"""
from . import workloads  # noqa: F401
