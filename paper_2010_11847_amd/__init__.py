"""MI355X-native particle-mesh (PM) N-body library.

The compute path is the HIP library libpm.so (C ABI in include/pm.h); this
package only marshals arguments to it.  ``PMContext`` owns a device workspace
(a torch uint8 tensor) and a library context; its methods carry the names of
the C entry points.
"""
from .inputs import Workload, Cosmology  # noqa: F401


def __getattr__(name):
    if name in ("PMContext", "make_config"):
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
