"""MI355X-native MPMC hard-disk sampler (HIP kernels behind a C ABI)."""
from . import mpmc  # noqa: F401
