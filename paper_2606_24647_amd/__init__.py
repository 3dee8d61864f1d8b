"""gq: columnar query operators (filter, hash join, hash group-by, hash
partition) for AMD Instinct MI355X (gfx950), behind the C-ABI in include/gq.h.

Importing the package loads nothing; ``paper_2606_24647_amd.gq`` binds the HIP
library and fails loudly when it is missing.
"""
__version__ = "0.1.0"
