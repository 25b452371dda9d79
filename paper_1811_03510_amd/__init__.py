"""MI355X-native direct ray tracing of Catmull-Clark patch scenes.

``ccs`` is the binding of the HIP library (include/ccs.h); ``scenes`` holds the
seeded synthetic workloads.
"""
from . import scenes  # noqa: F401
