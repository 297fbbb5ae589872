"""MI355X-native per-pixel beam tracer for non-rotating black holes (arXiv 2010.08735).

The GPU library (libbh.so, HIP for gfx950, C ABI in include/bh.h) is loaded lazily by
``paper_2010_08735_amd.bh.lib()``; ``scenes`` holds the seeded synthetic inputs."""
from . import scenes  # noqa: F401

__all__ = ["scenes", "bh"]
