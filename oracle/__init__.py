"""CPU reference (oracle) for Dense Inverse Search.  Test infrastructure only:
imported by the tests, the package smoke check and the benchmark's CPU leg,
never by the GPU product path."""
from .dis_oracle import *  # noqa: F401,F403
from . import dis_oracle, search_checks  # noqa: F401
