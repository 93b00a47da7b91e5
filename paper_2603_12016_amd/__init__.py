"""MI355X-native per-ROI GLCM texture (HIP kernels behind the C ABI of include/nyx.h)."""
from . import nyx  # noqa: F401
from .nyx import *  # noqa: F401,F403
