"""AES-GCM for one AMD Instinct MI355X (gfx950): a fused AES-CTR + GHASH
tree-reduction hot path behind a C ABI (``include/gcm_mi355.h``).

``gcm`` is the ctypes binding; ``workloads`` holds the seeded synthetic
input generators (no cryptographic arithmetic); ``build`` compiles the HIP
library in-tree.
"""
from . import workloads  # noqa: F401

__all__ = ["gcm", "workloads", "build"]
