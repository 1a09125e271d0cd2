"""MI355X-native (gfx950) implementation of the NeDF composition hot path:
volume-rendering depth marcher, NeDF depth+ID with fallback and refinement,
deferred shading, shadows and NeDF training, behind the C ABI in
include/nedf.h.  ``api`` is the torch-facing binding."""
from . import _abi  # noqa: F401
