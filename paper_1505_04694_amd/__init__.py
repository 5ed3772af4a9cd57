"""MI355X-native hot path of thread-parallel anisotropic mesh adaptation
(after Rokos, Gorman, Jensen, Kelly, arXiv:1505.04694).

The adaptation runs in libpmesh.so (HIP, gfx950) behind the C ABI in
include/pm.h; ``pmesh`` is its Python binding and ``inputs`` builds the
seeded synthetic meshes and metric fields.
"""
from . import inputs  # noqa: F401
