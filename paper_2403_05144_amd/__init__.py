"""MI355X-native partitioned P-ERK time integration of adaptively refined DGSEM discretisations.

Hot path in HIP (libperk.so, C ABI in include/perk.h); this package is the thin Python side:
`_lib` marshals arguments to the C ABI, `solver.PerkSolver` owns torch device buffers and
streams, `partition_rule` holds the level -> member maps of Sec. 6.4.1.
"""
from .solver import PerkSolver, PerkError  # noqa: F401
from .batch import PerkBatch  # noqa: F401
