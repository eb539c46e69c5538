"""MI355X (gfx950) Robin-Schwarz subdomain solves for the gravity equation.

The compute path is the HIP library libsos.so (csrc/); `sos` is its ctypes
binding. Build with `python -m paper_2112_03851_amd.build`.
"""
from . import sos  # noqa: F401
from .sos import Problem, SosError  # noqa: F401
