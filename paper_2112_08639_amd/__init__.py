"""libdk: MI355X-native density-kernel hot path (arXiv 2112.08639).

The compute is the HIP library ``libdk.so`` built from ``csrc/`` (C ABI in
``include/dk.h``); ``_lib`` is its ctypes binding with the same function names
and ``pipeline`` sequences the calls for a density evaluation.
"""

from ._lib import DkError, FermiInfo, load  # noqa: F401
