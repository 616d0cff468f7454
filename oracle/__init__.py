"""Plain CPU FP64 oracle of the space-time slab operators and solver.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check in
__graft_entry__.py and the cpu_baseline leg of bench.py may import, call,
link or run anything under oracle/.  The product path (the HIP library and
its binding) never touches it and shares no code with it.
"""
from .core import Problem, Space, Slab, build, dof_count  # noqa: F401
from . import tables  # noqa: F401
