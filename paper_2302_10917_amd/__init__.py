"""MI355X-native macro-element HDG local-problem engine.

The product path is the HIP library libmhdg.so (csrc/, C ABI in
include/mhdg.h) driven through the ctypes binding in mhdg.py.
"""
from . import inputs  # noqa: F401
