"""FP64 CPU oracle of the REDO propagator path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The GPU library never does, and this package imports nothing from
the GPU library: the two share no arithmetic, only the seeded inputs of
``paper_1707_02162_amd.workloads``.

Parity status of every function is stated in its module docstring.
"""
from .redo_oracle import *  # noqa: F401,F403
from .optim_oracle import bfgs_inverse_matrix, lbfgs_direction  # noqa: F401
