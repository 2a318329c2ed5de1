"""PolyMinHash CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct CPU implementations of what the GPU signing
path computes (arXiv 2511.16576, Sec. 1 and Sec. 3.2, Alg. 1), written from
the paper.  Only the test suite, the package's smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code
with the GPU library, and the GPU library never imports it.

Parity status per function is listed in the docstrings of ``oracle.core``,
``oracle.mlp``, ``oracle.rings``, ``oracle.centre`` and ``oracle.ranked``.
"""
from .core import *  # noqa: F401,F403
from .ranked import *  # noqa: F401,F403
