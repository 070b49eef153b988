"""CPU oracle for the upsampling step -- test infrastructure only.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this package; the product path never does.
"""
from . import upsample_oracle  # noqa: F401
