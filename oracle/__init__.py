"""FP64 CPU oracle for the LeaFi hot path.

TEST INFRASTRUCTURE ONLY: the slow, obviously correct reference that the GPU
library is checked against.  Only `tests/`, `__graft_entry__.smoke()` and the
benchmark's CPU-baseline leg may import it; the library never does.  It shares
no code with the GPU path.  Functions whose result has no pin of its own are
marked "parity unpinned" in their docstring (none at present: the trained
filter weights are not an oracle output).
"""
from .core import *  # noqa: F401,F403
from .core import build_bruteforce, num_threads, set_num_threads  # noqa: F401
