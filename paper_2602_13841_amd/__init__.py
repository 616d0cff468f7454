"""MI355X-native space-time multigrid Newton-Krylov slab solver.

The compute path is the HIP library libstmg.so (csrc/, C ABI in
include/stmg.h); `stmg` is its thin Python binding and `inputs` the seeded
synthetic input generator.
"""
