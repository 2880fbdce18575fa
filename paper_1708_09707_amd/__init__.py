"""MI355X (gfx950) H-matrix library: Morton ordering, block cluster tree
traversal, batched ACA and batched H-matrix-vector product in HIP, behind the
C ABI of include/hmx.h.  See hmx.py for the Python binding."""
from . import hmx  # noqa: F401
from .hmx import HMatrix  # noqa: F401
