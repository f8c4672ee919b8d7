"""libqieo: QIEO (quantum-inspired evolutionary optimization) of the 0/1
knapsack on one AMD Instinct MI355X.  The compute path is HIP for gfx950
behind the C ABI in include/qieo.h; ``paper_2609_30862_amd.qieo`` is its
ctypes binding.  Importing this package loads nothing; import the binding
module to load libqieo.so."""

__all__ = ["qieo"]
