"""CPU oracle of the collective multigrid method (arXiv 2302.13680).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product path.  It
shares no code with the GPU library.
"""
from .oracle import Oracle, build_oracle, oracle_lib_path  # noqa: F401
